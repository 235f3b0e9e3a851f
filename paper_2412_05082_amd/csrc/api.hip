// C ABI of libc0ip: level hierarchy, V-cycle (Algorithm 1) and flexible
// GMRES (Sec. 5.1-5.2) driving the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/c0ip.h"
#include "internal.h"
#include "kernels.h"
#include "exact.h"
#include "krylov_cg.h"
#include "mvs3d.h"
#include "pre2d.h"
#include "setup.h"

namespace {

thread_local std::string g_err;

c0ip_status fail(c0ip_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

struct HipFail {
  hipError_t e;
  const char* what;
};

#define HIP_TRY(expr)                                                \
  do {                                                               \
    hipError_t e_ = (expr);                                          \
    if (e_ != hipSuccess) throw HipFail{e_, #expr};                  \
  } while (0)

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    if (count <= n && p) return;
    release();
    HIP_TRY(hipMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T)));
    n = count;
  }
  void upload(const std::vector<T>& v) {
    alloc(v.size());
    HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  ~DevBuf() { release(); }
};

template <typename T>
std::vector<T> cast_vec(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

// Device data and work space of one precision on one level.
template <typename T>
struct LevelWork {
  DevBuf<T> tab, Q, lam, ptab;  // coefficient table, eigenbases, prolongation table
  DevBuf<T> tabref;             // the table scaled to h = 1 (default penalty only)
  DevBuf<T> x, b, r, scratch;   // V-cycle vectors and transfer scratch
  DevBuf<T> t;                  // 2D: second iterate buffer (smoothing steps are out of place)
  DevBuf<T> Aex;                // exact local solver: one dense patch inverse per boundary type
  c0ip::LevelCoef<T> coef;
  c0ip::LevelEig<T> eig;
  int avs_variant = 0;  // tile variant of the fused smoother (set by c0ip_autotune)
  bool ready = false;
};

struct Level {
  int N = 0, n1 = 0;
  int64_t ntot = 0;
  c0ip::Level1D lv;
  c0ip::RowClasses rc;
  std::vector<double> tab, Q, lam;  // host copies (float64)
  std::vector<double> Aex;          // exact local inverses [4 * 4][NN * NN] (local_solver 1)
  LevelWork<double> w64;
  LevelWork<float> w32;
};

}  // namespace

struct c0ip_problem {
  int dim = 2, k = 2, N = 2, L = 0;
  double gamma = 0;
  c0ip_mg_opts mg{};
  hipStream_t stream = nullptr;
  int device = 0;  // device current at creation
  std::vector<std::unique_ptr<Level>> lv;
  std::vector<double> ptab;  // prolongation table (float64 host copy)
  DevBuf<double> A0inv;
  // Krylov work space
  DevBuf<double> V, w, u, partial, hdev, ydev, r64;  // hdev: dots, then coefficients
  DevBuf<double> Z64;
  DevBuf<float> Z32;
  // flexible CG work space
  DevBuf<double> cg_p, cg_q, cg_z64, cg_sc, cg_partial;
  DevBuf<float> cg_z32;
  double* hpin = nullptr;  // pinned host staging for the per-step reductions
  // The V-cycle of the Krylov solves as a captured graph, per precision
  // ([0] float64, [1] float32; used when C0IP_VCYCLE_GRAPH=1): input u
  // (float64), or for float32 the finest level's b (u == NULL) or u cast
  // into it by the graph's first launch; output zfix.  Captured on first use
  // and again when the buffers or a tile variant changed.
  struct VGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* in = nullptr;
    const void* out = nullptr;
    void release() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
    }
  } vgraph[2];
  DevBuf<double> zfix64;
  DevBuf<float> zfix32;
  hipStream_t cap_stream = nullptr;  // capture only (the handle's stream may be the null stream)
  void invalidate_graphs() {
    vgraph[0].release();
    vgraph[1].release();
  }
  template <typename T>
  void vcycle_graph(const double* u, T* z);
  ~c0ip_problem() {
    invalidate_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (hpin) (void)hipHostFree(hpin);
  }

  int64_t ntot(int l) const { return lv[l]->ntot; }
  template <typename T>
  LevelWork<T>& work(int l);
  template <typename T>
  void prepare(int l);
  template <typename T>
  void smooth(int l, const T* b, T* x, int steps, bool x_is_zero);
  template <typename T>
  void smooth_from(int l, const T* b, T* from, T* x, int steps);
  template <typename T>
  void smooth_mvs(int l, const T* b, T* x, T* r, int steps, bool x_is_zero);
  // the 2D additive step fused with its residual (separable local solver, owner computes)
  bool fused2d() const { return dim == 2 && mg.scatter_mode == 0 && mg.smoother == 0 && mg.local_solver == 0; }
  // x_out = x_in + omega * sum_v R_v^T (local inverse) R_v r (owner computes; x_in may be null or x_out)
  template <typename T>
  void patch_step(int l, const T* r, const T* x_in, T* x_out, T om);
  template <typename T>
  void mg_level(int l, const T* b, T* x);
  template <typename T>
  void mg_level2d(int l, const T* b, T* x);
  // top level of the single-workgroup tail V-cycle in precision T (-1: none)
  int tailLT[2] = {-2, -2};
  template <typename T>
  int tail_level();
  template <typename T>
  void fill_tail(c0ip::TailParams<T>& P);
  template <typename T>
  void run_tail(const T* b, T* x);
  void check(hipError_t e, const char* what) {
    if (e != hipSuccess) throw HipFail{e, what};
  }
};

template <>
LevelWork<double>& c0ip_problem::work<double>(int l) {
  return lv[l]->w64;
}
template <>
LevelWork<float>& c0ip_problem::work<float>(int l) {
  return lv[l]->w32;
}

// Upload a level's tables in precision T and size its work vectors.
template <typename T>
void c0ip_problem::prepare(int l) {
  LevelWork<T>& w = work<T>(l);
  if (w.ready) return;
  Level& L_ = *lv[l];
  w.tab.upload(cast_vec<T>(L_.tab));
  w.Q.upload(cast_vec<T>(L_.Q));
  w.lam.upload(cast_vec<T>(L_.lam));
  w.ptab.upload(cast_vec<T>(ptab));
  w.coef.tab = w.tab.p;
  w.coef.nclass = L_.rc.nclass;
  w.coef.left = L_.rc.left;
  w.coef.right0 = L_.rc.right0;
  w.coef.periodic = L_.rc.periodic;
  if (gamma == (double)(k * (k + 1))) {
    // M = h M^, L = L^ / h, B = B^ / h^3 on a uniform mesh
    const double h = L_.lv.h, sc[3] = {1.0 / h, h, h * h * h};
    std::vector<double> r(L_.tab);
    const size_t per = r.size() / 3;
    for (size_t i = 0; i < r.size(); ++i) r[i] *= sc[i / per];
    w.tabref.upload(cast_vec<T>(r));
    w.coef.ref = w.tabref.p;
    w.coef.hinv = (T)(1.0 / h);
  }
  w.eig.Q = w.Q.p;
  w.eig.lam = w.lam.p;
  if (!L_.Aex.empty()) w.Aex.upload(cast_vec<T>(L_.Aex));
  w.x.alloc(L_.ntot);
  w.b.alloc(L_.ntot);
  w.r.alloc(L_.ntot);
  if (dim == 2) w.t.alloc(L_.ntot);
  if (l > 0) {
    const int64_t nf = L_.n1, nc = lv[l - 1]->n1;
    const int64_t s = dim == 2 ? nf * nc : 2 * nf * nf * nc;
    w.scratch.alloc(s);
  }
  w.ready = true;
}

// steps of the additive smoother on level l (x_is_zero: start from 0);
// result in x.  2D steps from a non-zero iterate are fused (residual kept in
// LDS) and run out of place, alternating between x and the level's r.
template <typename T>
void c0ip_problem::smooth(int l, const T* b, T* x, int steps, bool x_is_zero) {
  LevelWork<T>& w = work<T>(l);
  const int Nl = lv[l]->N;
  const T om = (T)mg.omega;
  if (steps <= 0) {
    if (x_is_zero) check(c0ip::launch_fill_t<T>(lv[l]->ntot, T(0), x, stream), "fill");
    return;
  }
  if (mg.smoother == 1) {
    smooth_mvs<T>(l, b, x, w.r.p, steps, x_is_zero);
    return;
  }
  if (mg.scatter_mode == 1) {  // atomic scatter: in place, residual through the level's r
    for (int s = 0; s < steps; ++s) {
      if (s == 0 && x_is_zero) {
        check(c0ip::launch_fill_t<T>(lv[l]->ntot, T(0), x, stream), "fill");
        check(c0ip::launch_patch2d_atomic<T>(k, Nl, w.eig, b, x, om, stream), "atomic smoother");
      } else {
        check(c0ip::launch_apply2d<T, T>(k, Nl, w.coef, x, b, w.r.p, stream), "residual");
        check(c0ip::launch_patch2d_atomic<T>(k, Nl, w.eig, w.r.p, x, om, stream), "atomic smoother");
      }
    }
    return;
  }
  int s0 = 0;
  if (x_is_zero) {
    patch_step<T>(l, b, nullptr, x, om);
    s0 = 1;
  }
  smooth_from(l, b, x, x, steps - s0);
}

// `steps` smoothing steps starting from the iterate in `from`, result in x
// (from may be x or the level's r buffer).
template <typename T>
void c0ip_problem::smooth_from(int l, const T* b, T* from, T* x, int steps) {
  LevelWork<T>& w = work<T>(l);
  const int Nl = lv[l]->N;
  const T om = (T)mg.omega;
  if (mg.scatter_mode == 1 || mg.smoother == 1) {
    if (from != x) check(hipMemcpyAsync(x, from, sizeof(T) * lv[l]->ntot, hipMemcpyDeviceToDevice, stream), "copy");
    smooth<T>(l, b, x, steps, false);
    return;
  }
  if (fused2d()) {
    T* cur = from;
    T* oth = (from == x) ? w.r.p : x;
    for (int s = 0; s < steps; ++s) {
      check(c0ip::launch_avs2d<T>(k, Nl, w.coef, w.eig, cur, b, oth, om, stream, 1, 0, nullptr, w.avs_variant),
            "fused smoother");
      std::swap(cur, oth);
    }
    if (cur != x)
      check(hipMemcpyAsync(x, cur, sizeof(T) * lv[l]->ntot, hipMemcpyDeviceToDevice, stream), "copy");
    return;
  }
  if (from != x) check(hipMemcpyAsync(x, from, sizeof(T) * lv[l]->ntot, hipMemcpyDeviceToDevice, stream), "copy");
  for (int s = 0; s < steps; ++s) {
    check(c0ip::launch_apply<T, T>(dim, k, Nl, w.coef, x, b, w.r.p, stream), "residual");
    patch_step<T>(l, w.r.p, x, x, om);
  }
}

template <typename T>
void c0ip_problem::patch_step(int l, const T* r, const T* x_in, T* x_out, T om) {
  LevelWork<T>& w = work<T>(l);
  if (mg.local_solver == 1)
    check(c0ip::launch_patch2d_exact<T>(k, lv[l]->N, w.Aex.p, r, x_in, x_out, om, stream), "exact local solves");
  else
    check(c0ip::launch_patch_smooth<T>(dim, k, lv[l]->N, w.eig, r, x_in, x_out, om, stream), "smoother");
}

// `steps` steps of the coloured multiplicative smoother on level l, in
// place on x: per colour c = 0..2^(d+1)-1, r = b - A x (r = b for the first colour
// of a step from x = 0), then x += omega * (local solves of colour c).  On
// 2D levels under 1.5 * 2^20 DoFs one launch per colour forms r on the colour's
// patch rows only; elsewhere r is a full residual pass (work vector r)
// before each colour.
template <typename T>
void c0ip_problem::smooth_mvs(int l, const T* b, T* x, T* r, int steps, bool x_is_zero) {
  LevelWork<T>& w = work<T>(l);
  const int Nl = lv[l]->N;
  const T om = (T)mg.omega;
  const int ncol = 1 << (dim + 1);
  // mvs_residual 0 (automatic): on 2D levels under 1.5 * 2^20 DoFs one launch per colour forms the residual
  // on the colour's patch rows (it halves the launches, which bound these levels); on finer levels a full
  // residual pass with the tiled operator precedes the colour's solves, where the operator's efficiency
  // wins. Measured per float64 step, in-launch against residual pass, in us: Q2 512^2 (1.05 M DoFs) 184
  // against 226, Q4 256^2 (1.05 M) 246 against 262, Q5 256^2 (1.64 M) 398 against 383, Q3 512^2 (2.36 M)
  // 357 against 315, Q7 256^2 (3.21 M) 1282 against 925.
  constexpr int64_t kMvsInLaunchBelow = int64_t(3) << 19;
  for (int s = 0; s < steps; ++s)
    for (int c = 0; c < ncol; ++c) {
      const bool zero = s == 0 && c == 0 && x_is_zero;
      if (zero) check(c0ip::launch_fill_t<T>(lv[l]->ntot, T(0), x, stream), "fill");
      const bool fused =
          dim == 2 && (mg.mvs_residual == 1 || (mg.mvs_residual == 0 && lv[l]->ntot < kMvsInLaunchBelow));
      const T* rc = zero ? b : (fused ? nullptr : r);
      if (!zero && !fused) check(c0ip::launch_apply<T, T>(dim, k, Nl, w.coef, x, b, r, stream), "residual");
      if (dim == 2 && mg.local_solver == 1)
        check(c0ip::launch_mvs2d_colour_exact<T>(k, Nl, c, w.coef, w.Aex.p, b, rc, x, om, stream),
              "multiplicative colour");
      else if (dim == 2)
        check(c0ip::launch_mvs2d_colour<T>(k, Nl, c, w.coef, w.eig, b, rc, x, om, stream),
              "multiplicative smoother colour");
      else
        check(c0ip::launch_mvs3d_colour<T>(k, Nl, c, w.eig, rc, x, om, stream), "multiplicative smoother colour");
    }
}

// The tail runs levels 0..LT in one launch: LT is the highest level (at
// most the finest, at most tail_levels - 1) whose vectors and tables fit in
// the LDS of one workgroup; below level 1 there is nothing to gain.
template <typename T>
int c0ip_problem::tail_level() {
  int& t = tailLT[sizeof(T) == 4 ? 1 : 0];
  if (t != -2) return t;
  t = -1;
  if (dim != 2 || k > 4 || mg.tail_levels == 0 || !fused2d()) return t;
  const int lim = c0ip::tail_lds_limit();
  int cap = std::min(L, c0ip::kTailMaxLevels - 1);
  if (mg.tail_levels > 0) cap = std::min(cap, mg.tail_levels - 1);
  int nclass[c0ip::kTailMaxLevels] = {};
  for (int l = 0; l <= cap; ++l) {
    nclass[l] = lv[l]->rc.nclass;
    if (c0ip::tail_bytes(k, l, nclass, (int)sizeof(T)) > lim) break;
    if (l >= 1) t = l;
  }
  if (t >= 1 && c0ip::configure_vtail<T>(k, c0ip::tail_bytes(k, t, nclass, (int)sizeof(T))) != hipSuccess) {
    (void)hipGetLastError();
    t = -1;
  }
  return t;
}

template <typename T>
void c0ip_problem::fill_tail(c0ip::TailParams<T>& P) {
  const int LT = tail_level<T>();
  P.LT = LT;
  for (int l = 0; l <= LT; ++l) {
    prepare<T>(l);
    const LevelWork<T>& w = work<T>(l);
    P.nclass[l] = w.coef.nclass;
    P.left[l] = w.coef.left;
    P.right0[l] = w.coef.right0;
    P.periodic[l] = w.coef.periodic;
    P.tab[l] = w.coef.tab;
    P.Q[l] = w.eig.Q;
    P.lam[l] = w.eig.lam;
  }
  P.ptab = work<T>(LT).ptab.p;
  P.Ainv = A0inv.p;
  P.omega = (T)mg.omega;
  P.pre = mg.pre_steps;
  P.post = mg.post_steps;
  P.coarse_mode = mg.coarse_mode;
}

template <typename T>
void c0ip_problem::run_tail(const T* b, T* x) {
  c0ip::TailParams<T> P;
  fill_tail<T>(P);
  c0ip::TailIO<T> io;
  for (int l = 0; l <= P.LT; ++l) io.nA[l] = 1;
  io.b[P.LT] = b;
  io.x[P.LT] = x;
  check(c0ip::launch_vtail<T>(k, P, io, 1, stream), "tail V-cycle");
}

// One 2D level of Algorithm 1 with out-of-place smoothing steps.  The
// iterate alternates between x and the level's t buffer; the pre-smoothing
// result lands in A, chosen so that the post-smoothing steps end in x.  The
// first post-smoothing step starts from A + P e inside the fused smoother
// (no separate prolongation pass).
template <typename T>
void c0ip_problem::mg_level2d(int l, const T* b, T* x) {
  LevelWork<T>& w = work<T>(l);
  LevelWork<T>& wc = work<T>(l - 1);
  const int Nl = lv[l]->N, pre = mg.pre_steps, post = mg.post_steps;
  const T om = (T)mg.omega;
  T* A = (post % 2 == 1) ? w.t.p : x;
  T* B = (A == x) ? w.t.p : x;
  const bool fused_pre = pre == 1 && Nl <= c0ip::kPre2dMaxN && k <= 3;
  if (fused_pre) {
    // x1 = S(0, b) and r = b - A x1 in one launch
    check(c0ip::launch_pre2d<T>(k, Nl, w.coef, w.eig, b, A, w.r.p, om, stream), "pre-smoother + residual");
  } else {
    if (pre == 0) {
      check(c0ip::launch_fill_t<T>(lv[l]->ntot, T(0), A, stream), "fill");
    } else {
      T* cur = (pre % 2 == 1) ? A : B;
      check(c0ip::launch_patch2d<T>(k, Nl, w.eig, b, nullptr, cur, om, stream), "smoother");
      for (int s = 1; s < pre; ++s) {
        T* nxt = (cur == A) ? B : A;
        check(c0ip::launch_avs2d<T>(k, Nl, w.coef, w.eig, cur, b, nxt, om, stream, 1, 0, nullptr, w.avs_variant),
              "fused smoother");
        cur = nxt;
      }
    }
    check(c0ip::launch_apply2d<T, T>(k, Nl, w.coef, A, b, w.r.p, stream), "residual");
  }
  check(c0ip::launch_restrict2d<T>(k, lv[l - 1]->N, w.ptab.p, w.r.p, wc.b.p, stream), "restrict");
  mg_level<T>(l - 1, wc.b.p, wc.x.p);
  if (post == 0) {
    check(c0ip::launch_prolong2d<T>(k, lv[l - 1]->N, w.ptab.p, wc.x.p, A, x, stream), "prolong");
    return;
  }
  check(c0ip::launch_avs2d<T>(k, Nl, w.coef, w.eig, A, b, B, om, stream, 1, 0, nullptr, w.avs_variant, wc.x.p,
                              w.ptab.p),
        "prolongation + fused smoother");
  T* cur = B;
  for (int s = 1; s < post; ++s) {
    T* nxt = (cur == A) ? B : A;
    check(c0ip::launch_avs2d<T>(k, Nl, w.coef, w.eig, cur, b, nxt, om, stream, 1, 0, nullptr, w.avs_variant),
          "fused smoother");
    cur = nxt;
  }
}

// x = MG_l(0, b) (Algorithm 1, returning right after the coarse solve).
template <typename T>
void c0ip_problem::mg_level(int l, const T* b, T* x) {
  if (l >= 1 && l == tail_level<T>()) {
    run_tail<T>(b, x);
    return;
  }
  if (l == 0) {
    if (mg.coarse_mode == 0) {
      check(c0ip::launch_coarse<T>(dim, k, A0inv.p, b, x, stream), "coarse solve");
    } else {
      patch_step<T>(0, b, nullptr, x, T(1));
    }
    return;
  }
  LevelWork<T>& w = work<T>(l);
  LevelWork<T>& wc = work<T>(l - 1);
  if (fused2d()) {
    mg_level2d<T>(l, b, x);
    return;
  }
  smooth<T>(l, b, x, mg.pre_steps, true);
  check(c0ip::launch_apply<T, T>(dim, k, lv[l]->N, w.coef, x, b, w.r.p, stream), "residual");
  check(c0ip::launch_restrict<T>(dim, k, lv[l - 1]->N, w.ptab.p, w.r.p, wc.b.p, w.scratch.p, stream), "restrict");
  mg_level<T>(l - 1, wc.b.p, wc.x.p);
  {
    check(c0ip::launch_prolong_add<T>(dim, k, lv[l - 1]->N, w.ptab.p, wc.x.p, x, w.scratch.p, stream), "prolong");
    smooth<T>(l, b, x, mg.post_steps, false);
  }
}

// z = MG_L(0, u) in precision T, launched eagerly or as one replay of a
// captured graph.  u is float64; in the float32 form u == NULL means that the
// input is already in the finest level's float32 b (else it is cast there
// first).  Every
// launch of the V-cycle goes to the handle's stream and allocates nothing
// once the levels are prepared, so the captured sequence is the eager one.
template <typename T>
void c0ip_problem::vcycle_graph(const double* u, T* z) {
  // Eager launches by default: with the host polling the Arnoldi reduction
  // it runs ahead of the device and the launches queue back to back, while a
  // graph replay leaves the device idle for ~8 us at its end (measured).
  // C0IP_VCYCLE_GRAPH=1 selects the captured graph.
  static const bool graph = [] {
    const char* e = std::getenv("C0IP_VCYCLE_GRAPH");
    return e && e[0] == '1';
  }();
  if (!graph) {
    for (int l = 0; l <= L; ++l) prepare<T>(l);
    if constexpr (sizeof(T) == 4) {
      LevelWork<float>& wf = work<float>(L);
      if (u) check(c0ip::launch_cast<double, float>(ntot(L), u, wf.b.p, stream), "cast");
      mg_level<float>(L, wf.b.p, (float*)z);
    } else {
      mg_level<double>(L, u, (double*)z);
    }
    return;
  }
  VGraph& g = vgraph[sizeof(T) == 4 ? 1 : 0];
  if (!g.exec || g.in != u || g.out != z) {
    g.release();
    for (int l = 0; l <= L; ++l) prepare<T>(l);
    (void)tail_level<T>();  // sets the tail kernel's LDS attribute outside the capture
    if (!cap_stream) check(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking), "capture stream");
    // record on the capture stream; the graph is launched on the handle's stream
    const hipStream_t user = stream;
    stream = cap_stream;
    check(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      if constexpr (sizeof(T) == 4) {
        LevelWork<float>& wf = work<float>(L);
        if (u) check(c0ip::launch_cast<double, float>(ntot(L), u, wf.b.p, stream), "cast");
        mg_level<float>(L, wf.b.p, (float*)z);
      } else {
        mg_level<double>(L, u, (double*)z);
      }
    } catch (...) {
      hipGraph_t dead = nullptr;
      (void)hipStreamEndCapture(stream, &dead);
      if (dead) (void)hipGraphDestroy(dead);
      stream = user;
      throw;
    }
    const hipError_t ec = hipStreamEndCapture(stream, &g.graph);
    stream = user;
    check(ec, "end capture");
    check(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0), "graph instantiate");
    g.in = u;
    g.out = z;
  }
  check(hipGraphLaunch(g.exec, stream), "graph launch");
}

namespace {

bool is_pow2(int n) { return n >= 2 && (n & (n - 1)) == 0; }

c0ip_status hip_fail(const HipFail& h) {
  return fail(C0IP_EHIP, std::string(h.what) + ": " + hipGetErrorString(h.e));
}

c0ip_status check_mesh(const c0ip_mesh_desc* m) {
  if (!m) return fail(C0IP_EINVAL, "mesh descriptor is NULL");
  if (m->dim != 2 && m->dim != 3) return fail(C0IP_EINVAL, "dim must be 2 or 3");
  if (m->degree < 2 || m->degree > 7) return fail(C0IP_EINVAL, "degree must be in [2,7]");
  if (!is_pow2(m->n_cells)) return fail(C0IP_EINVAL, "n_cells must be a power of two >= 2");
  if (m->n_cells > (1 << 16)) return fail(C0IP_EINVAL, "n_cells too large");
  {
    const int64_t n1 = (int64_t)m->degree * m->n_cells + 1;
    const int64_t nv = m->dim == 2 ? n1 * n1 : n1 * n1 * n1;
    if (nv >= (int64_t(1) << 31))
      return fail(C0IP_EINVAL, "mesh too large: " + std::to_string(nv) + " DoFs per vector (at most 2^31 - 1)");
  }
  return C0IP_OK;
}

int resolve_level(const c0ip_problem* p, int level) { return level < 0 ? p->L : level; }

}  // namespace

template <typename T>
const c0ip::LevelCoef<T>& c0ip_internal_coef(c0ip_problem* p, int level) {
  p->prepare<T>(level);
  return p->work<T>(level).coef;
}
template <typename T>
const c0ip::LevelEig<T>& c0ip_internal_eig(c0ip_problem* p, int level) {
  p->prepare<T>(level);
  return p->work<T>(level).eig;
}
template <typename T>
const T* c0ip_internal_ptab(c0ip_problem* p, int level) {
  p->prepare<T>(level);
  return p->work<T>(level).ptab.p;
}
const double* c0ip_internal_coarse(c0ip_problem* p) { return p->A0inv.p; }
void c0ip_internal_set_error(const std::string& msg) { g_err = msg; }
template const c0ip::LevelCoef<double>& c0ip_internal_coef<double>(c0ip_problem*, int);
template const c0ip::LevelCoef<float>& c0ip_internal_coef<float>(c0ip_problem*, int);
template const c0ip::LevelEig<double>& c0ip_internal_eig<double>(c0ip_problem*, int);
template const c0ip::LevelEig<float>& c0ip_internal_eig<float>(c0ip_problem*, int);
template <typename T>
int c0ip_internal_variant(c0ip_problem* p, int level) {
  return p->work<T>(level).avs_variant;
}
template <typename T>
int c0ip_internal_tail(c0ip_problem* p, c0ip::TailParams<T>* P) {
  const int LT = p->tail_level<T>();
  if (LT >= 1) p->fill_tail<T>(*P);
  return LT;
}
template int c0ip_internal_tail<double>(c0ip_problem*, c0ip::TailParams<double>*);
template int c0ip_internal_tail<float>(c0ip_problem*, c0ip::TailParams<float>*);
template int c0ip_internal_variant<double>(c0ip_problem*, int);
template int c0ip_internal_variant<float>(c0ip_problem*, int);
template const double* c0ip_internal_ptab<double>(c0ip_problem*, int);
template const float* c0ip_internal_ptab<float>(c0ip_problem*, int);

// Work space of c0ip_smoother_step_noalloc: a fixed device array, one copy
// per GPU (each GPU holds it until the process ends).  Host code never uses
// its name as an address: c0ip_create looks up the device address once per
// device (with that device current) and keeps it in g_scratch_addr.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};
hipError_t g_scratch_status[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Once per device, with that device current: the device address of scratch.
void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_done[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_status[device] = e;
  g_scratch_addr[device] = e == hipSuccess ? ptr : nullptr;
  if (e != hipSuccess) (void)hipGetLastError();
  g_scratch_done[device] = true;
}

void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_addr[device];
}

std::string scratch_error(int device) {
  if (device < 0 || device >= kMaxDevices) return "device index out of range";
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[device]) return "not set up";
  return hipGetErrorString(g_scratch_status[device]);
}

// Do the n elements of esz bytes at a and at b share any byte?
bool overlaps(const void* a, const void* b, int64_t n, size_t esz) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b, len = (uintptr_t)n * esz;
  return pa < pb + len && pb < pa + len;
}

// One out-of-place smoother step x_out = S(x_in, b) on level l (S(0, b) when
// x_in is null); r: residual work space of ntot(l) elements, used in 3D and
// by the atomic scatter.
template <typename T>
void smoother_step_on(c0ip_problem* p, int l, const T* b, const T* x_in, T* x_out, T* r) {
  LevelWork<T>& w = p->work<T>(l);
  const int Nl = p->lv[l]->N;
  const T om = (T)p->mg.omega;
  if (p->mg.smoother == 1) {
    if (x_in)
      p->check(hipMemcpyAsync(x_out, x_in, sizeof(T) * p->lv[l]->ntot, hipMemcpyDeviceToDevice, p->stream), "copy");
    p->smooth_mvs<T>(l, b, x_out, r, 1, x_in == nullptr);
    return;
  }
  if (p->mg.scatter_mode == 1) {
    if (x_in) {
      p->check(c0ip::launch_apply2d<T, T>(p->k, Nl, w.coef, x_in, b, r, p->stream), "residual");
      p->check(hipMemcpyAsync(x_out, x_in, sizeof(T) * p->lv[l]->ntot, hipMemcpyDeviceToDevice, p->stream), "copy");
    } else {
      p->check(c0ip::launch_fill_t<T>(p->lv[l]->ntot, T(0), x_out, p->stream), "fill");
    }
    p->check(c0ip::launch_patch2d_atomic<T>(p->k, Nl, w.eig, x_in ? r : b, x_out, om, p->stream), "atomic smoother");
  } else if (!x_in) {
    p->patch_step<T>(l, b, nullptr, x_out, om);
  } else if (p->fused2d()) {
    p->check(c0ip::launch_avs2d<T>(p->k, Nl, w.coef, w.eig, x_in, b, x_out, om, p->stream, 1, 0, nullptr,
                                   w.avs_variant),
             "fused smoother");
  } else {
    p->check(c0ip::launch_apply<T, T>(p->dim, p->k, Nl, w.coef, x_in, b, r, p->stream), "residual");
    p->patch_step<T>(l, r, x_in, x_out, om);
  }
}

}  // namespace

extern "C" {

const char* c0ip_last_error(void) { return g_err.c_str(); }

c0ip_status c0ip_create(const c0ip_mesh_desc* mesh, const c0ip_mg_opts* opts, void* hip_stream,
                        c0ip_problem** out) {
  g_err.clear();
  if (!out) return fail(C0IP_EINVAL, "out is NULL");
  *out = nullptr;
  c0ip_status st = check_mesh(mesh);
  if (st != C0IP_OK) return st;
  c0ip_mg_opts mg;
  if (opts) {
    mg = *opts;
  } else {
    mg.omega = mesh->dim == 2 ? 0.25 : 0.1;
    mg.pre_steps = mg.post_steps = 1;
    mg.vcycle_dtype = C0IP_F32;
    mg.coarse_mode = 0;
    mg.scatter_mode = 0;
    mg.tail_levels = -1;
    mg.smoother = 0;
    mg.local_solver = 0;
    mg.mvs_residual = 0;
  }
  if (!(mg.omega > 0) || !std::isfinite(mg.omega)) return fail(C0IP_EINVAL, "omega must be > 0");
  if (mg.mvs_residual < 0 || mg.mvs_residual > 2) return fail(C0IP_EINVAL, "mvs_residual must be 0, 1 or 2");
  if (mg.smoother != 0 && mg.smoother != 1) return fail(C0IP_EINVAL, "smoother must be 0 or 1");
  if (mg.smoother == 1 && mg.scatter_mode != 0)
    return fail(C0IP_EINVAL, "the multiplicative smoother takes scatter_mode 0");
  if (mg.local_solver != 0 && mg.local_solver != 1) return fail(C0IP_EINVAL, "local_solver must be 0 or 1");
  if (mg.local_solver == 1 && (mesh->dim != 2 || mg.scatter_mode != 0))
    return fail(C0IP_EUNSUPPORTED, "the exact local solver is built for 2D meshes with scatter_mode 0");
  if (mg.pre_steps < 0 || mg.post_steps < 0 || mg.pre_steps > 16 || mg.post_steps > 16)
    return fail(C0IP_EINVAL, "smoothing steps must be in [0,16]");
  if (mg.vcycle_dtype != C0IP_F64 && mg.vcycle_dtype != C0IP_F32) return fail(C0IP_EINVAL, "bad vcycle_dtype");
  if (mg.coarse_mode != 0 && mg.coarse_mode != 1) return fail(C0IP_EINVAL, "coarse_mode must be 0 or 1");
  if (mg.scatter_mode != 0 && mg.scatter_mode != 1) return fail(C0IP_EINVAL, "scatter_mode must be 0 or 1");
  if (mg.scatter_mode == 1 && mesh->dim != 2)
    return fail(C0IP_EUNSUPPORTED, "the atomic-scatter smoother is built for 2D meshes only");
  if (mg.tail_levels < -1) return fail(C0IP_EINVAL, "tail_levels must be >= -1");
  std::unique_ptr<c0ip_problem> p(new c0ip_problem());
  p->dim = mesh->dim;
  p->k = mesh->degree;
  p->N = mesh->n_cells;
  p->gamma = mesh->gamma > 0 ? mesh->gamma : (double)(p->k * (p->k + 1));
  p->mg = mg;
  p->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&p->device) != hipSuccess) {
    (void)hipGetLastError();
    return fail(C0IP_EHIP, "hipGetDevice failed");
  }
  scratch_setup(p->device);
  int L = 0;
  while ((2 << L) < p->N) ++L;
  p->L = L;
  try {
    p->ptab = c0ip::prolongation_table(p->k);
    for (int l = 0; l <= L; ++l) {
      std::unique_ptr<Level> lv(new Level());
      lv->N = 2 << l;
      lv->n1 = p->k * lv->N + 1;
      lv->ntot = (int64_t)lv->n1 * lv->n1 * (p->dim == 3 ? lv->n1 : 1);
      lv->lv = c0ip::build_level_1d(p->k, lv->N, p->gamma);
      lv->rc = c0ip::row_classes(lv->lv);
      lv->tab = c0ip::coefficient_table(lv->lv, lv->rc);
      // every row must equal its class representative
      {
        const int kk = p->k, W = 4 * kk + 1;
        const c0ip::Band* mats[3] = {&lv->lv.M, &lv->lv.L, &lv->lv.B};
        for (int m = 0; m < 3; ++m) {
          double mx = 0;
          for (double v : mats[m]->a) mx = std::max(mx, std::fabs(v));
          for (int i = 0; i < lv->n1; ++i) {
            int cls;
            if (!lv->rc.periodic || i < lv->rc.left) cls = i;
            else if (i >= lv->rc.right0) cls = lv->rc.left + (lv->n1 - 1 - i);
            else cls = 2 * lv->rc.left + i % kk;
            for (int o = -2 * kk; o <= 2 * kk; ++o) {
              int j = i + o;
              double a = (j >= 0 && j < lv->n1) ? mats[m]->get(i, j) : 0.0;
              double t = lv->tab[((size_t)m * lv->rc.nclass + cls) * W + (o + 2 * kk)];
              if (std::fabs(a - t) > 1e-12 * mx) return fail(C0IP_EINVAL, "1D band is not periodic");
            }
          }
        }
      }
      c0ip::PatchEigen pe;
      std::string err;
      if (!c0ip::build_patch_eigen(lv->lv, pe, err)) return fail(C0IP_EINVAL, err);
      const int n = pe.n;
      lv->Q.assign((size_t)4 * n * n, 0.0);
      lv->lam.assign((size_t)4 * n, 1.0);
      for (int t = 0; t < 4; ++t)
        if (pe.present[t]) {
          std::copy(pe.Q[t].begin(), pe.Q[t].end(), lv->Q.begin() + (size_t)t * n * n);
          std::copy(pe.lam[t].begin(), pe.lam[t].end(), lv->lam.begin() + (size_t)t * n);
        }
      if (p->mg.local_solver == 1) {
        // one dense inverse of the exact local matrix per boundary type (tx, ty) present on the level
        const int NN = n * n, Nl = lv->N;
        int rep[4] = {-1, -1, -1, -1};
        for (int v = 1; v <= Nl - 1; ++v)
          if (rep[c0ip::patch_variant(v, Nl)] < 0) rep[c0ip::patch_variant(v, Nl)] = v;
        lv->Aex.assign((size_t)16 * NN * NN, 0.0);
        for (int ty = 0; ty < 4; ++ty)
          for (int tx = 0; tx < 4; ++tx) {
            if (rep[tx] < 0 || rep[ty] < 0) continue;
            const int vert[2] = {rep[tx], rep[ty]};
            std::vector<double> inv;
            if (!c0ip::patch_exact_inverse(lv->lv, 2, vert, inv, err)) return fail(C0IP_EINVAL, err);
            std::copy(inv.begin(), inv.end(), lv->Aex.begin() + (size_t)(ty * 4 + tx) * NN * NN);
          }
      }
      p->lv.push_back(std::move(lv));
    }
    std::vector<double> Ainv;
    std::string err;
    if (!c0ip::coarse_inverse(p->lv[0]->lv, p->dim, Ainv, err)) return fail(C0IP_EINVAL, err);
    p->A0inv.upload(Ainv);
    for (int l = 0; l <= L; ++l) p->prepare<double>(l);
    if (p->mg.vcycle_dtype == C0IP_F32)
      for (int l = 0; l <= L; ++l) p->prepare<float>(l);
  } catch (const HipFail& h) {
    return hip_fail(h);
  } catch (const std::bad_alloc&) {
    return fail(C0IP_ENOMEM, "host allocation failed");
  }
  *out = p.release();
  return C0IP_OK;
}

c0ip_status c0ip_destroy(c0ip_problem* p) {
  g_err.clear();
  delete p;
  return C0IP_OK;
}

c0ip_status c0ip_num_levels(const c0ip_problem* p, int* n_levels) {
  if (!p || !n_levels) return fail(C0IP_EINVAL, "NULL argument");
  *n_levels = p->L + 1;
  return C0IP_OK;
}

c0ip_status c0ip_num_dofs(const c0ip_problem* p, int level, int64_t* n_total) {
  if (!p || !n_total) return fail(C0IP_EINVAL, "NULL argument");
  if (level < -1 || level > p->L) return fail(C0IP_EINVAL, "level out of range");
  *n_total = p->ntot(resolve_level(p, level));
  return C0IP_OK;
}

c0ip_status c0ip_apply_A(c0ip_problem* p, int level, c0ip_dtype dtype, const void* x, void* y) {
  g_err.clear();
  if (!p || !x || !y) return fail(C0IP_EINVAL, "NULL argument");
  if (level < -1 || level > p->L) return fail(C0IP_EINVAL, "level out of range");
  const int l = resolve_level(p, level);
  if (overlaps(x, y, p->ntot(l), dtype == C0IP_F32 ? sizeof(float) : sizeof(double)))
    return fail(C0IP_EINVAL, "x and y must not overlap");
  try {
    if (dtype == C0IP_F64) {
      p->check(c0ip::launch_apply<double, double>(p->dim, p->k, p->lv[l]->N, p->work<double>(l).coef,
                                                  (const double*)x, nullptr, (double*)y, p->stream),
               "apply_A");
    } else if (dtype == C0IP_F32) {
      p->prepare<float>(l);
      p->check(c0ip::launch_apply<float, float>(p->dim, p->k, p->lv[l]->N, p->work<float>(l).coef,
                                                (const float*)x, nullptr, (float*)y, p->stream),
               "apply_A");
    } else {
      return fail(C0IP_EINVAL, "bad dtype");
    }
  } catch (const HipFail& h) {
    return hip_fail(h);
  }
  return C0IP_OK;
}

c0ip_status c0ip_apply_smoother(c0ip_problem* p, int level, c0ip_dtype dtype, const void* b, void* x,
                                int x_is_zero) {
  g_err.clear();
  if (!p || !b || !x) return fail(C0IP_EINVAL, "NULL argument");
  if (level < -1 || level > p->L) return fail(C0IP_EINVAL, "level out of range");
  const int l = resolve_level(p, level);
  if (overlaps(b, x, p->ntot(l), dtype == C0IP_F32 ? sizeof(float) : sizeof(double)))
    return fail(C0IP_EINVAL, "b and x must not overlap");
  try {
    if (dtype == C0IP_F64) {
      p->smooth<double>(l, (const double*)b, (double*)x, 1, x_is_zero != 0);
    } else if (dtype == C0IP_F32) {
      p->prepare<float>(l);
      p->smooth<float>(l, (const float*)b, (float*)x, 1, x_is_zero != 0);
    } else {
      return fail(C0IP_EINVAL, "bad dtype");
    }
  } catch (const HipFail& h) {
    return hip_fail(h);
  }
  return C0IP_OK;
}

c0ip_status c0ip_smoother_step(c0ip_problem* p, int level, c0ip_dtype dtype, const void* b, const void* x_in,
                               void* x_out) {
  g_err.clear();
  if (!p || !b || !x_out) return fail(C0IP_EINVAL, "NULL argument");
  if (level < -1 || level > p->L) return fail(C0IP_EINVAL, "level out of range");
  if (dtype != C0IP_F64 && dtype != C0IP_F32) return fail(C0IP_EINVAL, "bad dtype");
  const int l = resolve_level(p, level);
  const size_t esz = dtype == C0IP_F64 ? sizeof(double) : sizeof(float);
  if (overlaps(x_out, b, p->ntot(l), esz) || (x_in && overlaps(x_out, x_in, p->ntot(l), esz)))
    return fail(C0IP_EINVAL, "x_out must not overlap b or x_in");
  try {
    if (dtype == C0IP_F64) {
      p->prepare<double>(l);
      smoother_step_on<double>(p, l, (const double*)b, (const double*)x_in, (double*)x_out, p->work<double>(l).r.p);
    } else {
      p->prepare<float>(l);
      smoother_step_on<float>(p, l, (const float*)b, (const float*)x_in, (float*)x_out, p->work<float>(l).r.p);
    }
  } catch (const HipFail& h) {
    return hip_fail(h);
  }
  return C0IP_OK;
}

c0ip_status c0ip_smoother_step_noalloc(c0ip_problem* p, int level, c0ip_dtype dtype, const void* b,
                                       const void* x_in, void* x_out) {
  g_err.clear();
  if (!p || !b || !x_out) return fail(C0IP_EINVAL, "NULL argument");
  if (level < -1 || level > p->L) return fail(C0IP_EINVAL, "level out of range");
  if (dtype != C0IP_F64 && dtype != C0IP_F32) return fail(C0IP_EINVAL, "bad dtype");
  const int l = resolve_level(p, level);
  const size_t esz = dtype == C0IP_F64 ? sizeof(double) : sizeof(float);
  if (overlaps(x_out, b, p->ntot(l), esz) || (x_in && overlaps(x_out, x_in, p->ntot(l), esz)))
    return fail(C0IP_EINVAL, "x_out must not overlap b or x_in");
  // the tables of this precision must exist already: setting them up allocates
  const bool ready = dtype == C0IP_F64 ? p->work<double>(l).ready : p->work<float>(l).ready;
  if (!ready)
    return fail(C0IP_EINVAL, "float32 tables are set up at creation only with vcycle_dtype = C0IP_F32 "
                             "(or by an earlier float32 call of another entry point)");
  // the residual goes through the work space in 3D, with the atomic scatter
  // and with the multiplicative smoother (after its first colour, also from 0)
  const bool needs_r = p->mg.smoother == 1 || (x_in && !p->fused2d());
  void* r = nullptr;
  if (needs_r) {
    if ((size_t)p->ntot(l) * esz > kNoAllocScratchBytes)
      return fail(C0IP_EINVAL, "level has " + std::to_string(p->ntot(l)) + " DoFs: the residual needs " +
                                   std::to_string((size_t)p->ntot(l) * esz) + " bytes, the fixed work space of " +
                                   "c0ip_smoother_step_noalloc holds " + std::to_string(kNoAllocScratchBytes));
    r = scratch_address(p->device);
    if (!r) return fail(C0IP_EHIP, "the fixed work space has no device address on this GPU: " + scratch_error(p->device));
  }
  try {
    if (dtype == C0IP_F64)
      smoother_step_on<double>(p, l, (const double*)b, (const double*)x_in, (double*)x_out, (double*)r);
    else
      smoother_step_on<float>(p, l, (const float*)b, (const float*)x_in, (float*)x_out, (float*)r);
  } catch (const HipFail& h) {
    return hip_fail(h);
  }
  return C0IP_OK;
}

c0ip_status c0ip_autotune(c0ip_problem* p, int reps) {
  g_err.clear();
  if (!p) return fail(C0IP_EINVAL, "NULL argument");
  if (reps < 1) reps = 3;
  if (p->dim != 2) return C0IP_OK;  // 3D kernels have one tile shape
  try {
    hipEvent_t e0, e1;
    p->check(hipEventCreate(&e0), "event");
    p->check(hipEventCreate(&e1), "event");
    auto tune = [&](auto tag) {
      using T = decltype(tag);
      for (int l = 1; l <= p->L; ++l) {
        LevelWork<T>& w = p->work<T>(l);
        if (!w.ready) continue;
        const int64_t n = p->lv[l]->ntot;
        const int Nl = p->lv[l]->N;
        p->check(c0ip::launch_fill_t<T>(n, T(0), w.x.p, p->stream), "fill");
        p->check(c0ip::launch_fill_t<T>(n, T(0), w.b.p, p->stream), "fill");
        float best = 1e30f;
        int bestv = 0;
        for (int v = 0; v < c0ip::avs2d_variants(p->k); ++v) {
          p->check(c0ip::launch_avs2d<T>(p->k, Nl, w.coef, w.eig, w.x.p, w.b.p, w.r.p, T(0.25), p->stream, 1, 0,
                                         nullptr, v),
                   "autotune");
          p->check(hipEventRecord(e0, p->stream), "event");
          for (int r = 0; r < reps; ++r)
            p->check(c0ip::launch_avs2d<T>(p->k, Nl, w.coef, w.eig, w.x.p, w.b.p, w.r.p, T(0.25), p->stream, 1, 0,
                                           nullptr, v),
                     "autotune");
          p->check(hipEventRecord(e1, p->stream), "event");
          p->check(hipEventSynchronize(e1), "sync");
          float ms = 0;
          p->check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
          if (ms < best) {
            best = ms;
            bestv = v;
          }
        }
        w.avs_variant = bestv;
        p->invalidate_graphs();
      }
    };
    tune(double{});
    tune(float{});
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  } catch (const HipFail& h) {
    return hip_fail(h);
  }
  return C0IP_OK;
}

c0ip_status c0ip_set_variant(c0ip_problem* p, int level, c0ip_dtype dtype, int variant) {
  if (!p) return fail(C0IP_EINVAL, "NULL argument");
  if (level < -1 || level > p->L) return fail(C0IP_EINVAL, "level out of range");
  if (variant < 0 || variant >= c0ip::avs2d_variants(p->k)) return fail(C0IP_EINVAL, "no such variant");
  const int l = resolve_level(p, level);
  if (dtype == C0IP_F32) p->lv[l]->w32.avs_variant = variant;
  else p->lv[l]->w64.avs_variant = variant;
  p->invalidate_graphs();
  return C0IP_OK;
}

c0ip_status c0ip_tuned_variant(const c0ip_problem* p, int level, c0ip_dtype dtype, int* variant) {
  if (!p || !variant) return fail(C0IP_EINVAL, "NULL argument");
  if (level < -1 || level > p->L) return fail(C0IP_EINVAL, "level out of range");
  const int l = resolve_level(p, level);
  *variant = dtype == C0IP_F32 ? p->lv[l]->w32.avs_variant : p->lv[l]->w64.avs_variant;
  return C0IP_OK;
}

c0ip_status c0ip_vcycle(c0ip_problem* p, c0ip_dtype dtype, const void* b, void* x) {
  g_err.clear();
  if (!p || !b || !x) return fail(C0IP_EINVAL, "NULL argument");
  if (overlaps(b, x, p->ntot(p->L), dtype == C0IP_F32 ? sizeof(float) : sizeof(double)))
    return fail(C0IP_EINVAL, "b and x must not overlap");
  try {
    if (dtype == C0IP_F64) {
      p->mg_level<double>(p->L, (const double*)b, (double*)x);
    } else if (dtype == C0IP_F32) {
      for (int l = 0; l <= p->L; ++l) p->prepare<float>(l);
      p->mg_level<float>(p->L, (const float*)b, (float*)x);
    } else {
      return fail(C0IP_EINVAL, "bad dtype");
    }
  } catch (const HipFail& h) {
    return hip_fail(h);
  }
  return C0IP_OK;
}

// The Krylov solves time their V-cycles with an event pair on every
// kTimeEvery-th iteration and scale the sum to all iterations.
constexpr int kTimeEvery = 8;

// Givens QR of the (j+2) x (j+1) Hessenberg H (row-major, leading dim m)
// applied to g0 e_1; returns |g_{j+1}| and leaves R, g for back substitution.
static double hessenberg_lsq(const std::vector<double>& H, int m, int j, double g0, std::vector<double>& R,
                             std::vector<double>& g) {
  const int nr = j + 2, nc = j + 1;
  R.assign((size_t)nr * nc, 0.0);
  for (int r = 0; r < nr; ++r)
    for (int c = 0; c < nc; ++c) R[(size_t)r * nc + c] = H[(size_t)r * m + c];
  g.assign(nr, 0.0);
  g[0] = g0;
  for (int c = 0; c < nc; ++c) {
    const double a = R[(size_t)c * nc + c], b = R[(size_t)(c + 1) * nc + c];
    const double den = std::hypot(a, b);
    const double cs = den > 0 ? a / den : 1.0, sn = den > 0 ? b / den : 0.0;
    for (int cc = c; cc < nc; ++cc) {
      const double x = R[(size_t)c * nc + cc], y = R[(size_t)(c + 1) * nc + cc];
      R[(size_t)c * nc + cc] = cs * x + sn * y;
      R[(size_t)(c + 1) * nc + cc] = -sn * x + cs * y;
    }
    const double x = g[c], y = g[c + 1];
    g[c] = cs * x + sn * y;
    g[c + 1] = -sn * x + cs * y;
  }
  return std::fabs(g[nr - 1]);
}

c0ip_status c0ip_solve(c0ip_problem* p, const c0ip_krylov_opts* opts, const double* b, double* x,
                       c0ip_solve_info* info) {
  g_err.clear();
  if (!p || !opts || !b || !x) return fail(C0IP_EINVAL, "NULL argument");
  if (!(opts->rtol > 0) || opts->max_iters < 1 || opts->restart < 1 || opts->restart > 64)
    return fail(C0IP_EINVAL, "bad Krylov options (rtol > 0, max_iters >= 1, restart in [1,64])");
  if (overlaps(b, x, p->ntot(p->L), sizeof(double))) return fail(C0IP_EINVAL, "b and x must not overlap");
  const int m = opts->restart, Lf = p->L;
  const int64_t n = p->ntot(Lf);
  const bool f32 = p->mg.vcycle_dtype == C0IP_F32;
  hipStream_t s = p->stream;
  c0ip_solve_info inf{};
  auto t0 = std::chrono::steady_clock::now();
  double t_vc = 0;
  int n_timed = 0;
  c0ip_status result = C0IP_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr, ef = nullptr;
  int its = 0;
  double last_est = 0, bnorm_out = 0;
  try {
    const int nblk = std::max(c0ip::multidot_blocks(n), c0ip::arnoldi_blocks(n));
    const int nblk_a = c0ip::arnoldi_blocks(n);
    p->V.alloc((size_t)m * n);
    p->w.alloc(n);
    p->r64.alloc(n);
    p->u.alloc(n);
    p->partial.alloc((size_t)(2 * m + 3) * nblk);
    p->hdev.alloc(4 * m + 8);  // [0, 2m+3): dots; [2m+3, 4m+8): coefficients (one copy to the host)
    double* coefd = p->hdev.p + 2 * m + 3;
    p->ydev.alloc(m);
    if (!p->hpin)
      p->check(hipHostMalloc((void**)&p->hpin, sizeof(double) * (4 * 64 + 16), hipHostMallocCoherent), "pinned alloc");
    if (f32) {
      p->Z32.alloc((size_t)m * n);
      p->zfix32.alloc(n);
      for (int l = 0; l <= Lf; ++l) p->prepare<float>(l);
    } else {
      p->Z64.alloc((size_t)m * n);
      p->zfix64.alloc(n);
    }
    p->check(hipEventCreate(&e0), "event");
    p->check(hipEventCreate(&e1), "event");
    p->check(hipEventCreateWithFlags(&ef, hipEventDisableTiming), "event");
    double* hh = p->hpin;  // [0, 2m+3): dots; [2m+3, 4m+8): coefficients
    double* hh_dev = nullptr;  // the same memory as the kernels address it
    p->check(hipHostGetDevicePointer((void**)&hh_dev, hh, 0), "host pointer");
    auto norm2 = [&](const double* v) {
      p->check(c0ip::launch_multidot(n, 1, v, n, v, p->partial.p, nblk, s), "multidot");
      p->check(c0ip::launch_reduce_partials(1, nblk, p->partial.p, p->hdev.p, 0, s), "reduce");
      p->check(hipMemcpyAsync(hh, p->hdev.p, sizeof(double), hipMemcpyDeviceToHost, s), "D2H");
      p->check(hipStreamSynchronize(s), "sync");
      return hh[0];
    };
    const auto& cf64 = p->work<double>(Lf).coef;
    // ||b|| over the free DoFs (boundary entries of b are ignored): r = b - A 0
    p->check(c0ip::launch_fill(n, 0.0, p->w.p, s), "fill");
    p->check(c0ip::launch_apply<double, double>(p->dim, p->k, p->N, cf64, p->w.p, b, p->r64.p, s), "mask b");
    const double bnorm = std::sqrt(norm2(p->r64.p));
    if (!std::isfinite(bnorm)) throw c0ip_status(C0IP_ENAN);
    bnorm_out = bnorm;
    if (opts->x0_is_zero) {
      p->check(c0ip::launch_fill(n, 0.0, x, s), "fill");
    } else {
      p->check(c0ip::launch_apply<double, double>(p->dim, p->k, p->N, cf64, x, b, p->r64.p, s), "residual");
    }
    double beta = std::sqrt(norm2(p->r64.p));
    std::vector<double> hist{beta};
    last_est = beta;
    bool converged = bnorm == 0.0 || beta <= opts->rtol * bnorm;
    std::vector<double> H((size_t)(m + 1) * m), R, g, y(m);
    while (!converged && its < opts->max_iters) {
      if (!(beta > 0) || !std::isfinite(beta)) throw c0ip_status(C0IP_ENAN);
      // lagged vector u = r / beta (re-normalised exactly at step 0)
      p->check(c0ip::launch_multidot(n, 1, p->r64.p, n, p->r64.p, p->partial.p, nblk, s), "multidot");
      p->check(c0ip::launch_reduce_partials(1, nblk, p->partial.p, p->hdev.p, 0, s), "reduce");
      p->check(c0ip::launch_normalize(n, p->r64.p, p->hdev.p, p->u.p, s), "normalize");
      std::fill(H.begin(), H.end(), 0.0);
      double g0 = beta;
      int jdone = 0;
      bool stop = false;
      for (int j = 0; j < m && !stop; ++j) {
        // V-cycle time sampled on every kTimeEvery-th iteration (an event
        // pair in the stream idles the GPU for a few microseconds)
        const bool timed = its % kTimeEvery == 0;
        if (timed) p->check(hipEventRecord(e0, s), "event");
        const double* Zp;
        bool zf32 = f32;
        // z = M u into Z_j; in 2D the operator's launch A z writes that copy
        if (f32) {
          float* Zj = p->Z32.p + (size_t)j * n;
          float* u32 = p->work<float>(Lf).b.p;  // the previous update wrote (float) u there
          if (j == 0) p->check(c0ip::launch_cast<double, float>(n, p->u.p, u32, s), "cast");
          p->vcycle_graph<float>(nullptr, p->zfix32.p);
          if (timed) p->check(hipEventRecord(e1, s), "event");
          if (p->dim == 2) {
            p->check(c0ip::launch_apply2d<float, double>(p->k, p->N, cf64, p->zfix32.p, nullptr, p->w.p, s, 1, 0,
                                                         nullptr, Zj),
                     "A z");
          } else {
            p->check(hipMemcpyAsync(Zj, p->zfix32.p, sizeof(float) * n, hipMemcpyDeviceToDevice, s), "copy z");
            p->check(c0ip::launch_apply<float, double>(p->dim, p->k, p->N, cf64, Zj, nullptr, p->w.p, s), "A z");
          }
          Zp = nullptr;
        } else {
          double* Zj = p->Z64.p + (size_t)j * n;
          p->vcycle_graph<double>(p->u.p, p->zfix64.p);
          if (timed) p->check(hipEventRecord(e1, s), "event");
          if (p->dim == 2) {
            p->check(c0ip::launch_apply2d<double, double>(p->k, p->N, cf64, p->zfix64.p, nullptr, p->w.p, s, 1, 0,
                                                          nullptr, Zj),
                     "A z");
          } else {
            p->check(hipMemcpyAsync(Zj, p->zfix64.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "copy z");
            p->check(c0ip::launch_apply<double, double>(p->dim, p->k, p->N, cf64, Zj, nullptr, p->w.p, s), "A z");
          }
          Zp = Zj;
        }
        (void)Zp;
        (void)zf32;
        // one reduction: V^T u, V^T w, u.u, u.w, w.w; coefficients on the device
        p->check(c0ip::launch_arnoldi_dots(n, j, p->V.p, n, p->u.p, p->w.p, p->partial.p, nblk_a, s), "dots");
        // sums and coefficients, also written straight into the pinned host
        // buffer; the event marks the end of that launch
        p->check(c0ip::launch_arnoldi_reduce_coef(j, nblk_a, p->partial.p, p->hdev.p, coefd, hh_dev, 2 * m + 3, s),
                 "reduce");
        p->check(hipEventRecord(ef, s), "event");
        // V_j = (u - V s)/alpha ; u <- w - V c - V_j h_v   (overlaps the host work below)
        p->check(c0ip::launch_arnoldi_update(n, j, p->V.p, n, p->u.p, p->w.p, coefd, p->V.p + (size_t)j * n, s,
                                             f32 ? p->work<float>(Lf).b.p : nullptr),
                 "update");
        // the host reads the sums once the reduction has completed (the
        // update runs meanwhile); stores of a kernel to pinned memory are
        // ordered for the host only by the launch's completion
        p->check(hipEventSynchronize(ef), "sync");
        if (timed) {
          float ms = 0;
          p->check(hipEventSynchronize(e1), "sync");
          p->check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
          t_vc += ms * 1e-3;
          ++n_timed;
        }
        const double* d = hh;
        const double* cf = hh + 2 * m + 3;
        const double alpha = cf[2 * j + 2], hv = cf[2 * j + 3];
        if (!std::isfinite(alpha) || !std::isfinite(hv) || !std::isfinite(d[2 * j + 2]))
          throw c0ip_status(C0IP_ENAN);
        if (j == 0) {
          g0 = beta * alpha;  // r = beta u = beta alpha V_0
        } else {
          for (int i = 0; i < j; ++i) H[(size_t)i * m + (j - 1)] += d[i];
          H[(size_t)j * m + (j - 1)] = alpha;
        }
        double cc = 0;
        for (int i = 0; i < j; ++i) {
          H[(size_t)i * m + j] = d[j + i];
          cc += d[j + i] * d[j + i];
        }
        H[(size_t)j * m + j] = hv;
        const double ww = d[2 * j + 2];
        double est2 = ww - cc - hv * hv;
        if (!(est2 > 1e-10 * ww)) est2 = norm2(p->u.p);  // heavy cancellation: exact norm
        H[(size_t)(j + 1) * m + j] = std::sqrt(std::max(est2, 0.0));
        const double res = hessenberg_lsq(H, m, j, g0, R, g);
        ++its;
        jdone = j + 1;
        hist.push_back(res);
        last_est = res;
        if (res <= opts->rtol * bnorm || H[(size_t)(j + 1) * m + j] == 0.0 || its >= opts->max_iters) stop = true;
      }
      // y = R^{-1} g, x += Z y
      hessenberg_lsq(H, m, jdone - 1, g0, R, g);
      const int nc = jdone;
      for (int i = jdone - 1; i >= 0; --i) {
        double t = g[i];
        for (int l2 = i + 1; l2 < jdone; ++l2) t -= R[(size_t)i * nc + l2] * y[l2];
        y[i] = t / R[(size_t)i * nc + i];
      }
      p->check(hipMemcpyAsync(p->ydev.p, y.data(), jdone * sizeof(double), hipMemcpyHostToDevice, s), "H2D");
      if (f32)
        p->check(c0ip::launch_update_solution<float>(n, jdone, p->Z32.p, n, p->ydev.p, x, s), "update");
      else
        p->check(c0ip::launch_update_solution<double>(n, jdone, p->Z64.p, n, p->ydev.p, x, s), "update");
      p->check(c0ip::launch_apply<double, double>(p->dim, p->k, p->N, cf64, x, b, p->r64.p, s), "residual");
      beta = std::sqrt(norm2(p->r64.p));
      converged = hist.back() <= opts->rtol * bnorm;
    }
    p->check(hipStreamSynchronize(s), "sync");
    inf.iterations = its;
    inf.converged = converged ? 1 : 0;
    inf.rel_res_est = bnorm > 0 ? hist.back() / bnorm : 0.0;
    inf.rel_res_true = bnorm > 0 ? beta / bnorm : 0.0;
    inf.frac_iters = (its > 0 && inf.rel_res_est > 0) ? 8.0 * its / (-std::log10(inf.rel_res_est)) : 0.0;
    if (!std::isfinite(beta)) result = fail(C0IP_ENAN, "non-finite residual");
    else if (!converged) result = fail(C0IP_NOT_CONVERGED, "max_iters reached");
  } catch (const HipFail& h) {
    result = hip_fail(h);
  } catch (c0ip_status st) {
    (void)hipStreamSynchronize(s);
    result = fail(st, "non-finite value in the Krylov iteration (iteration " + std::to_string(its + 1) + ")");
    inf.iterations = its;
    inf.rel_res_est = bnorm_out > 0 ? last_est / bnorm_out : 0.0;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (ef) (void)hipEventDestroy(ef);
  auto t1 = std::chrono::steady_clock::now();
  inf.seconds_total = std::chrono::duration<double>(t1 - t0).count();
  inf.seconds_vcycle = n_timed > 0 ? t_vc * its / n_timed : 0.0;
  inf.seconds_arnoldi = std::max(0.0, inf.seconds_total - t_vc);
  if (info) *info = inf;
  return result;
}

c0ip_status c0ip_solve_fcg(c0ip_problem* p, const c0ip_krylov_opts* opts, const double* b, double* x,
                           c0ip_solve_info* info) {
  g_err.clear();
  if (!p || !opts || !b || !x) return fail(C0IP_EINVAL, "NULL argument");
  if (!(opts->rtol > 0) || opts->max_iters < 1) return fail(C0IP_EINVAL, "bad Krylov options (rtol > 0, max_iters >= 1)");
  if (overlaps(b, x, p->ntot(p->L), sizeof(double))) return fail(C0IP_EINVAL, "b and x must not overlap");
  const int Lf = p->L;
  const int64_t n = p->ntot(Lf);
  const bool f32 = p->mg.vcycle_dtype == C0IP_F32;
  hipStream_t s = p->stream;
  c0ip_solve_info inf{};
  auto t0 = std::chrono::steady_clock::now();
  double t_vc = 0;
  int n_timed = 0;
  c0ip_status result = C0IP_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  try {
    namespace cg = c0ip::cg;
    const int nblk = cg::blocks(n);
    p->r64.alloc(n);
    p->w.alloc(n);
    p->cg_p.alloc(n);
    p->cg_q.alloc(n);
    p->cg_sc.alloc(cg::kSlots);
    p->cg_partial.alloc((size_t)2 * nblk);
    if (f32) {
      p->cg_z32.alloc(n);
      for (int l = 0; l <= Lf; ++l) p->prepare<float>(l);
    } else {
      p->cg_z64.alloc(n);
    }
    if (!p->hpin)
      p->check(hipHostMalloc((void**)&p->hpin, sizeof(double) * (4 * 64 + 16), hipHostMallocCoherent), "pinned alloc");
    p->check(hipEventCreate(&e0), "event");
    p->check(hipEventCreate(&e1), "event");
    double* hh = p->hpin;
    double* sc = p->cg_sc.p;
    double* r = p->r64.p;
    const auto& cf64 = p->work<double>(Lf).coef;
    auto rnorm2 = [&](const double* v) {
      p->check(cg::launch_dot<double>(n, v, v, p->cg_partial.p, nblk, s), "dot");
      p->check(cg::launch_reduce(1, nblk, p->cg_partial.p, sc, cg::kRR, 0, s), "reduce");
      p->check(hipMemcpyAsync(hh, sc + cg::kRR, sizeof(double), hipMemcpyDeviceToHost, s), "D2H");
      p->check(hipStreamSynchronize(s), "sync");
      return hh[0];
    };
    // ||b|| over the free DoFs (boundary entries of b are ignored): r = b - A 0
    p->check(c0ip::launch_fill(n, 0.0, p->w.p, s), "fill");
    p->check(c0ip::launch_apply<double, double>(p->dim, p->k, p->N, cf64, p->w.p, b, r, s), "mask b");
    const double bnorm = std::sqrt(rnorm2(r));
    if (!std::isfinite(bnorm)) throw c0ip_status(C0IP_ENAN);
    if (opts->x0_is_zero)
      p->check(c0ip::launch_fill(n, 0.0, x, s), "fill");
    else
      p->check(c0ip::launch_apply<double, double>(p->dim, p->k, p->N, cf64, x, b, r, s), "residual");
    double rr = opts->x0_is_zero ? bnorm * bnorm : rnorm2(r);
    const double r0 = std::sqrt(rr);
    int its = 0;
    bool converged = bnorm == 0.0 || std::sqrt(rr) <= opts->rtol * bnorm;
    while (!converged && its < opts->max_iters) {
      if (!std::isfinite(rr)) throw c0ip_status(C0IP_ENAN);
      const int first = its == 0;
      const bool timed = its % kTimeEvery == 0;  // sampled V-cycle timing, as in c0ip_solve
      if (timed) p->check(hipEventRecord(e0, s), "event");
      if (f32) {
        // (float) r: cast once, then written by each x, r update
        if (first) p->check(c0ip::launch_cast<double, float>(n, r, p->work<float>(Lf).b.p, s), "cast");
        p->vcycle_graph<float>(nullptr, p->cg_z32.p);
      }
      else p->vcycle_graph<double>(r, p->cg_z64.p);
      if (timed) p->check(hipEventRecord(e1, s), "event");
      // beta = (z . q_old) / (p_old . q_old); p = z - beta p_old
      if (!first) {
        if (f32) p->check(cg::launch_dot<float>(n, p->cg_z32.p, p->cg_q.p, p->cg_partial.p, nblk, s), "dot");
        else p->check(cg::launch_dot<double>(n, p->cg_z64.p, p->cg_q.p, p->cg_partial.p, nblk, s), "dot");
        p->check(cg::launch_reduce(1, nblk, p->cg_partial.p, sc, cg::kZQ, 1, s), "reduce");
      }
      if (f32) p->check(cg::launch_update_p<float>(n, p->cg_z32.p, sc, p->cg_p.p, first, s), "update p");
      else p->check(cg::launch_update_p<double>(n, p->cg_z64.p, sc, p->cg_p.p, first, s), "update p");
      // q = A p; alpha = (r . p) / (p . q); x += alpha p; r -= alpha q
      p->check(c0ip::launch_apply<double, double>(p->dim, p->k, p->N, cf64, p->cg_p.p, nullptr, p->cg_q.p, s), "A p");
      p->check(cg::launch_dot2(n, p->cg_p.p, p->cg_q.p, r, p->cg_partial.p, nblk, s), "dots");
      p->check(cg::launch_reduce(2, nblk, p->cg_partial.p, sc, cg::kPQ, 2, s), "reduce");
      p->check(cg::launch_update_xr(n, sc, p->cg_p.p, p->cg_q.p, x, r, p->cg_partial.p, nblk, s,
                                    f32 ? p->work<float>(Lf).b.p : nullptr),
               "update x, r");
      p->check(cg::launch_reduce(1, nblk, p->cg_partial.p, sc, cg::kRR, 0, s), "reduce");
      p->check(hipMemcpyAsync(hh, sc, cg::kSlots * sizeof(double), hipMemcpyDeviceToHost, s), "D2H");
      p->check(hipStreamSynchronize(s), "sync");
      if (timed) {
        float ms = 0;
        p->check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        t_vc += ms * 1e-3;
        ++n_timed;
      }
      ++its;
      rr = hh[cg::kRR];
      if (!std::isfinite(rr) || !std::isfinite(hh[cg::kALPHA])) throw c0ip_status(C0IP_ENAN);
      converged = std::sqrt(rr) <= opts->rtol * bnorm;
    }
    // true residual of the returned x
    p->check(c0ip::launch_apply<double, double>(p->dim, p->k, p->N, cf64, x, b, p->cg_q.p, s), "residual");
    const double rt = std::sqrt(rnorm2(p->cg_q.p));
    inf.iterations = its;
    inf.converged = converged ? 1 : 0;
    inf.rel_res_est = bnorm > 0 ? std::sqrt(rr) / bnorm : 0.0;
    inf.rel_res_true = bnorm > 0 ? rt / bnorm : 0.0;
    const double red = r0 > 0 ? std::sqrt(rr) / r0 : 0.0;
    inf.frac_iters = (its > 0 && red > 0 && red < 1) ? 8.0 * its / (-std::log10(red)) : 0.0;
    if (!std::isfinite(rt)) result = fail(C0IP_ENAN, "non-finite residual");
    else if (!converged) result = fail(C0IP_NOT_CONVERGED, "max_iters reached");
  } catch (const HipFail& h) {
    result = hip_fail(h);
  } catch (c0ip_status st) {
    (void)hipStreamSynchronize(s);
    result = fail(st, "non-finite value in the Krylov iteration");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  auto t1 = std::chrono::steady_clock::now();
  inf.seconds_total = std::chrono::duration<double>(t1 - t0).count();
  inf.seconds_vcycle = n_timed > 0 ? t_vc * inf.iterations / n_timed : 0.0;
  inf.seconds_arnoldi = std::max(0.0, inf.seconds_total - t_vc);
  if (info) *info = inf;
  return result;
}

c0ip_status c0ip_host_matrices_1d(int degree, int n_cells, double gamma, double* M, double* L, double* B) {
  g_err.clear();
  if (degree < 2 || degree > 7 || n_cells < 1 || !M || !L || !B) return fail(C0IP_EINVAL, "bad argument");
  const double gam = gamma > 0 ? gamma : (double)(degree * (degree + 1));
  c0ip::Level1D lv = c0ip::build_level_1d(degree, n_cells, gam);
  const int n1 = lv.n1;
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      M[(size_t)i * n1 + j] = lv.M.get(i, j);
      L[(size_t)i * n1 + j] = lv.L.get(i, j);
      B[(size_t)i * n1 + j] = lv.B.get(i, j);
    }
  return C0IP_OK;
}

c0ip_status c0ip_host_patch_inverse_exact(int dim, int degree, int n_cells, double gamma, const int* vertex,
                                          double* Ainv) {
  g_err.clear();
  if ((dim != 2 && dim != 3) || degree < 2 || degree > 7 || !is_pow2(n_cells) || !vertex || !Ainv)
    return fail(C0IP_EINVAL, "bad argument");
  for (int d = 0; d < dim; ++d)
    if (vertex[d] < 1 || vertex[d] > n_cells - 1) return fail(C0IP_EINVAL, "vertex out of range");
  const double gam = gamma > 0 ? gamma : (double)(degree * (degree + 1));
  c0ip::Level1D lv = c0ip::build_level_1d(degree, n_cells, gam);
  std::vector<double> inv;
  std::string err;
  if (!c0ip::patch_exact_inverse(lv, dim, vertex, inv, err)) return fail(C0IP_EINVAL, err);
  std::copy(inv.begin(), inv.end(), Ainv);
  return C0IP_OK;
}

c0ip_status c0ip_host_patch_inverse(int dim, int degree, int n_cells, double gamma, const int* vertex,
                                    double* Ainv) {
  g_err.clear();
  if ((dim != 2 && dim != 3) || degree < 2 || degree > 7 || !is_pow2(n_cells) || !vertex || !Ainv)
    return fail(C0IP_EINVAL, "bad argument");
  for (int d = 0; d < dim; ++d)
    if (vertex[d] < 1 || vertex[d] > n_cells - 1) return fail(C0IP_EINVAL, "vertex out of range");
  const double gam = gamma > 0 ? gamma : (double)(degree * (degree + 1));
  c0ip::Level1D lv = c0ip::build_level_1d(degree, n_cells, gam);
  c0ip::PatchEigen pe;
  std::string err;
  if (!c0ip::build_patch_eigen(lv, pe, err)) return fail(C0IP_EINVAL, err);
  const int n = pe.n;
  int np = 1;
  for (int d = 0; d < dim; ++d) np *= n;
  const std::vector<double>* Q[3];
  const std::vector<double>* lam[3];
  for (int d = 0; d < dim; ++d) {
    int t = c0ip::patch_variant(vertex[d], n_cells);
    Q[d] = &pe.Q[t];
    lam[d] = &pe.lam[t];
  }
  // Ainv = (Q_z (x) Q_y (x) Q_x) D^{-1} (...)^T, entry (r, c)
  for (int r = 0; r < np; ++r)
    for (int c = 0; c < np; ++c) {
      int ri[3] = {r % n, (r / n) % n, r / (n * n)}, ci[3] = {c % n, (c / n) % n, c / (n * n)};
      double s = 0;
      for (int e = 0; e < np; ++e) {
        int ei[3] = {e % n, (e / n) % n, e / (n * n)};
        double qr = 1, qc = 1, lsum = 0;
        for (int d = 0; d < dim; ++d) {
          qr *= (*Q[d])[ri[d] * n + ei[d]];
          qc *= (*Q[d])[ci[d] * n + ei[d]];
          lsum += (*lam[d])[ei[d]];
        }
        s += qr * qc / lsum;
      }
      Ainv[(size_t)r * np + c] = s;
    }
  return C0IP_OK;
}

}  // extern "C"
