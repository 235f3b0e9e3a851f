// Accessors of a problem's device tables, shared by the batched driver.
#pragma once

#include <string>

#include "kernels.h"

struct c0ip_problem;

template <typename T>
const c0ip::LevelCoef<T>& c0ip_internal_coef(c0ip_problem* p, int level);
template <typename T>
const c0ip::LevelEig<T>& c0ip_internal_eig(c0ip_problem* p, int level);
template <typename T>
const T* c0ip_internal_ptab(c0ip_problem* p, int level);
const double* c0ip_internal_coarse(c0ip_problem* p);
template <typename T>
int c0ip_internal_variant(c0ip_problem* p, int level);
// Parameters of the single-workgroup tail V-cycle (levels 0..LT) for this
// problem's options; returns LT, or -1 when the tail is not used.
template <typename T>
int c0ip_internal_tail(c0ip_problem* p, c0ip::TailParams<T>* P);
void c0ip_internal_set_error(const std::string& msg);
