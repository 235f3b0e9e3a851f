// Batched solves: many independent systems (problems x right-hand sides,
// uneven sizes and degrees) advance one flexible-GMRES step per round, and
// every round is one replay of a captured HIP graph.  The Krylov state of
// every system lives on the device: the round's last kernel runs the Givens
// step, advances the system or stops it, so rounds follow one another with
// no host work in between; the host only reads each round's state (copied
// out by the graph) a few rounds later and queues the solution update and
// restart of the systems that stopped.
//
// Systems are grouped by (k, gamma); within a group they are ordered by
// decreasing number of levels L_s, so at level l the systems still present
// (L_s >= l) form a prefix 0..A_l-1 and every mesh there has N_l = 2^(l+1)
// cells: each V-cycle step of a group is ONE launch over all its systems
// (system = blockIdx.z, vectors n_l apart in per-level slot buffers).  A
// system enters the V-cycle at its own finest level on the way down and
// leaves there on the way up (Algorithm 1 for each system).  Converged
// systems are masked off on the device, so the graph never changes.
// The Krylov kernels take per-system state records (sizes differ).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "../../include/c0ip.h"
#include "internal.h"
#include "kernels.h"

namespace c0ip {
namespace {

constexpr int kThreads = 256;
constexpr int kPer = 8;                 // entries per lane in the dot kernel
constexpr int kChunk = kThreads * kPer;  // entries per dot block
constexpr int kVec = 4;
constexpr int kEl = 4;                  // entries per lane in the copy and update kernels
constexpr int kElBlock = kThreads * kEl;
constexpr int kMaxM = 64;
constexpr int kRing = 3;      // round graphs (and state snapshots) in rotation
constexpr int kInFlight = 2;  // rounds queued ahead of the host's reading of the state

// Where a system stands between rounds.  The host writes the state once per
// solve; after that only the device changes it: the Givens kernel advances j
// or stops the system, the restart kernel re-activates it.
// kExact: the residual met at a restart is exactly zero (converged, x final).
enum : int { kRun = 0, kRestart = 1, kConverged = 2, kMaxIts = 3, kFailed = 4, kExact = 5 };

struct KrySys {
  double* V;         // m basis vectors, n apart
  double* u;         // current (unnormalised) Krylov vector
  const double* w;   // A z of the round
  void* Z;           // m preconditioned vectors (V-cycle precision), n apart
  void* vin;         // the V-cycle's right-hand-side slot
  const void* vout;  // the V-cycle's solution slot
  int* mask;         // this system's entry in its group's activity mask
  double* H;         // (m + 1) x m Hessenberg matrix, row-major
  double* y;         // m coefficients of the update x += Z y
  int64_t n;
  int64_t poff;  // offset of its partial sums
  int nblk;      // its blocks in the dots kernel
  int d0, u0;    // its first block in the dots grid and in the copy / update grid
  // changed on the device
  int j, its, status, active, epoch;
  double bnorm, beta, g0, last;
};

struct KryParams {  // options of the running solve (read by the Givens kernel)
  double rtol;
  int max_iters;
};

__device__ __forceinline__ double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// NT: non-temporal loads of the bases (when together they exceed the
// last-level cache).
// Grids of the Krylov kernels hold exactly each system's blocks, back to back:
// map[block] = its system, and the system's first block (d0 / u0) gives the
// block's place in it.
template <bool NT>
__global__ __launch_bounds__(kThreads) void bdots_kernel(const KrySys* __restrict__ sys, const int* __restrict__ map,
                                                         double* __restrict__ partial) {
  const KrySys d = sys[map[blockIdx.x]];
  if (!d.active) return;
  const int lb = blockIdx.x - d.d0;
  __shared__ double red[kThreads / 64][2 * kVec];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, j = d.j;
  const int64_t base = (int64_t)lb * kChunk + threadIdx.x;
  double* P = partial + d.poff;
  double ur[kPer], wr[kPer], e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int64_t i = base + (int64_t)e * kThreads;
    ur[e] = i < d.n ? d.u[i] : 0.0;
    wr[e] = i < d.n ? d.w[i] : 0.0;
    e0 += ur[e] * ur[e];
    e1 += ur[e] * wr[e];
    e2 += wr[e] * wr[e];
  }
  {
    const double x0 = wsum(e0), x1 = wsum(e1), x2 = wsum(e2);
    if (lane == 0) {
      red[wid][0] = x0;
      red[wid][1] = x1;
      red[wid][2] = x2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      double s = 0;
      for (int q = 0; q < kThreads / 64; ++q) s += red[q][threadIdx.x];
      P[(int64_t)(2 * j + threadIdx.x) * d.nblk + lb] = s;
    }
    __syncthreads();
  }
  for (int i0 = 0; i0 < j; i0 += kVec) {
    double au[kVec], aw[kVec];
#pragma unroll
    for (int q = 0; q < kVec; ++q) {
      au[q] = aw[q] = 0;
      if (i0 + q < j) {
        const double* vq = d.V + (int64_t)(i0 + q) * d.n;
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
          const int64_t i = base + (int64_t)e * kThreads;
          double v = 0.0;
          if (i < d.n) v = NT ? __builtin_nontemporal_load(vq + i) : vq[i];
          au[q] += v * ur[e];
          aw[q] += v * wr[e];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kVec; ++q) {
      const double x = wsum(au[q]), y = wsum(aw[q]);
      if (lane == 0) {
        red[wid][q] = x;
        red[wid][kVec + q] = y;
      }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kVec) {
      const int t = threadIdx.x, q = t % kVec;
      if (i0 + q < j) {
        double s = 0;
        for (int r = 0; r < kThreads / 64; ++r) s += red[r][t];
        P[(int64_t)(t < kVec ? i0 + q : j + i0 + q) * d.nblk + lb] = s;
      }
    }
    __syncthreads();
  }
}

// hout[s][row] = sum over the system's blocks; rows 0..2j+2
__global__ __launch_bounds__(kThreads) void breduce_kernel(const KrySys* __restrict__ sys, int m,
                                                           const double* __restrict__ partial,
                                                           double* __restrict__ hout) {
  const KrySys d = sys[blockIdx.y];
  const int row = blockIdx.x;
  if (!d.active || row >= 2 * d.j + 3) return;
  __shared__ double red[kThreads / 64];
  const double* P = partial + d.poff + (int64_t)row * d.nblk;
  double s = 0;
  for (int b = threadIdx.x; b < d.nblk; b += kThreads) s += P[b];
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int q = 0; q < kThreads / 64; ++q) t += red[q];
    hout[(int64_t)blockIdx.y * (2 * m + 3) + row] = t;
  }
}

// Update coefficients per system (same formulas as the single-system solve).
__global__ void bcoef_kernel(const KrySys* __restrict__ sys, int nsys, int m, const double* __restrict__ hout,
                             double* __restrict__ coef) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  const KrySys d = sys[s];
  if (!d.active) return;
  const int j = d.j;
  const double* h = hout + (int64_t)s * (2 * m + 3);
  double* c = coef + (int64_t)s * (2 * m + 5);
  double ss = 0, sc = 0;
  for (int i = 0; i < j; ++i) {
    ss += h[i] * h[i];
    sc += h[i] * h[j + i];
  }
  const double uu = h[2 * j], uw = h[2 * j + 1];
  const double a2 = uu - ss;
  const double alpha = a2 > 0 ? sqrt(a2) : 0.0;
  const double inv = alpha > 0 ? 1.0 / alpha : 0.0;
  const double hv = (uw - sc) * inv;
  for (int i = 0; i < j; ++i) {
    c[i] = h[i] * inv;
    c[j + i] = h[j + i] - h[i] * hv * inv;
  }
  c[2 * j] = inv;
  c[2 * j + 1] = hv * inv;
  c[2 * j + 2] = alpha;
  c[2 * j + 3] = hv;
  c[2 * j + 4] = uu > 0 ? ss / uu : 0.0;
}

__global__ __launch_bounds__(kThreads) void bupdate_kernel(const KrySys* __restrict__ sys, const int* __restrict__ map,
                                                           int m, const double* __restrict__ coef) {
  const int si = map[blockIdx.x];
  const KrySys d = sys[si];
  if (!d.active) return;
  const int j = d.j;
  const double* c = coef + (int64_t)si * (2 * m + 5);
  __shared__ double se[kMaxM], sf[kMaxM];
  for (int t = threadIdx.x; t < kMaxM; t += kThreads) {
    se[t] = t < j ? c[t] : 0.0;
    sf[t] = t < j ? c[j + t] : 0.0;
  }
  __syncthreads();
  const double inv = c[2 * j], dd = c[2 * j + 1];
  double* vout = d.V + (int64_t)j * d.n;
  const int64_t base = (int64_t)(blockIdx.x - d.u0) * kElBlock + threadIdx.x;
  double sv[kEl], sw[kEl];
#pragma unroll
  for (int e = 0; e < kEl; ++e) sv[e] = sw[e] = 0.0;
  for (int q = 0; q < j; ++q) {  // kEl independent loads per basis vector
    const double* vq = d.V + (int64_t)q * d.n;
    double v[kEl];
#pragma unroll
    for (int e = 0; e < kEl; ++e) {
      const int64_t i = base + (int64_t)e * kThreads;
      v[e] = i < d.n ? vq[i] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < kEl; ++e) {
      sv[e] += se[q] * v[e];
      sw[e] += sf[q] * v[e];
    }
  }
#pragma unroll
  for (int e = 0; e < kEl; ++e) {
    const int64_t i = base + (int64_t)e * kThreads;
    if (i < d.n) {
      const double ui = d.u[i], wi = d.w[i];
      vout[i] = ui * inv - sv[e];
      d.u[i] = wi - sw[e] - dd * ui;
    }
  }
}

// One Givens step per system (one workgroup each).  The round's reductions
// complete column j-1 of H (delayed re-orthogonalisation) and give column j,
// with h_{j+1,j} from Pythagoras (the explicit norm of the new u under heavy
// cancellation).  The QR factorisation of H by Givens rotations, applied to
// g0 e_1, gives the residual estimate |g_{j+1}|.  A system that converges,
// fills its basis or reaches max_iters leaves y = R^{-1} g for x += Z y and
// goes idle; otherwise it moves on to j + 1.  The arithmetic and its order
// are those of the single-system solve.
__global__ __launch_bounds__(kThreads) void bgivens_kernel(KrySys* __restrict__ sys, int m,
                                                           const double* __restrict__ hout,
                                                           const double* __restrict__ coef,
                                                           const KryParams* __restrict__ prm) {
  KrySys* ds = sys + blockIdx.x;
  const KrySys d = *ds;
  if (!d.active) return;
  __shared__ double R[(kMaxM + 1) * kMaxM];
  __shared__ double g[kMaxM + 1];
  __shared__ double rot[2];
  __shared__ double red[kThreads / 64];
  __shared__ double est_s;
  const int t = threadIdx.x, j = d.j, nc = j + 1, nr = j + 2;
  const double* h = hout + (int64_t)blockIdx.x * (2 * m + 3);
  const double* cf = coef + (int64_t)blockIdx.x * (2 * m + 5);
  const double alpha = cf[2 * j + 2], hv = cf[2 * j + 3], ww = h[2 * j + 2];
  if (!isfinite(alpha) || !isfinite(hv) || !isfinite(ww)) {
    if (t == 0) {
      ds->status = kFailed;
      ds->active = 0;
      *d.mask = 0;
    }
    return;
  }
  // columns 0..j of H with this round's entries, rows 0..j+1, into LDS
  for (int e = t; e < nr * nc; e += kThreads) {
    const int r = e / nc, c = e - r * nc;
    double v;
    if (c < j - 1)
      v = d.H[(int64_t)r * m + c];
    else if (c == j - 1)
      v = r < j ? d.H[(int64_t)r * m + c] + h[r] : (r == j ? alpha : 0.0);
    else
      v = r < j ? h[j + r] : (r == j ? hv : 0.0);
    R[e] = v;
  }
  if (t == 0) {
    double c2 = 0;
    for (int i = 0; i < j; ++i) c2 += h[j + i] * h[j + i];
    est_s = ww - c2 - hv * hv;
  }
  __syncthreads();
  double est2 = est_s;
  if (!(est2 > 1e-10 * ww)) {  // heavy cancellation: exact norm
    double sum = 0;
    for (int64_t i = t; i < d.n; i += kThreads) sum += d.u[i] * d.u[i];
    sum = wsum(sum);
    if ((t & 63) == 0) red[t >> 6] = sum;
    __syncthreads();
    est2 = 0;
    for (int q = 0; q < kThreads / 64; ++q) est2 += red[q];
  }
  const double hn = sqrt(fmax(est2, 0.0));
  const double g0 = j == 0 ? d.beta * alpha : d.g0;  // r = beta u = beta alpha V_0
  if (t == 0) {
    R[(j + 1) * nc + j] = hn;
    g[0] = g0;
    for (int r = 1; r < nr; ++r) g[r] = 0.0;
  }
  __syncthreads();
  // the completed column j-1 and the new column j back to H
  for (int r = t; r < nr; r += kThreads) {
    if (j > 0) d.H[(int64_t)r * m + j - 1] = R[r * nc + j - 1];
    d.H[(int64_t)r * m + j] = R[r * nc + j];
  }
  __syncthreads();
  for (int c = 0; c < nc; ++c) {
    if (t == 0) {
      const double a = R[c * nc + c], b = R[(c + 1) * nc + c];
      const double den = hypot(a, b);
      const double cs = den > 0 ? a / den : 1.0, sn = den > 0 ? b / den : 0.0;
      rot[0] = cs;
      rot[1] = sn;
      const double x = g[c], y = g[c + 1];
      g[c] = cs * x + sn * y;
      g[c + 1] = -sn * x + cs * y;
    }
    __syncthreads();
    const double cs = rot[0], sn = rot[1];
    for (int cc = c + t; cc < nc; cc += kThreads) {
      const double x = R[c * nc + cc], y = R[(c + 1) * nc + cc];
      R[c * nc + cc] = cs * x + sn * y;
      R[(c + 1) * nc + cc] = -sn * x + cs * y;
    }
    __syncthreads();
  }
  if (t == 0) {
    const double res = fabs(g[nr - 1]);
    const int its = d.its + 1;
    const bool conv = res <= prm->rtol * d.bnorm || hn == 0.0;
    ds->its = its;
    ds->last = res;
    ds->g0 = g0;
    if (conv || j + 1 == m || its >= prm->max_iters) {
      for (int i = nc - 1; i >= 0; --i) {  // y = R^{-1} g, into LDS row g
        double v = g[i];
        for (int l2 = i + 1; l2 < nc; ++l2) v -= R[i * nc + l2] * g[l2];
        g[i] = v / R[i * nc + i];
      }
      for (int i = 0; i < nc; ++i) d.y[i] = g[i];
      ds->status = conv ? kConverged : (its >= prm->max_iters ? kMaxIts : kRestart);
      ds->active = 0;
      *d.mask = 0;
    } else {
      ds->j = j + 1;
    }
  }
}

// A system that stopped, after x += Z y and r = b - A x: beta = ||r||; one
// that only filled its basis (and has u = r / beta) starts its next cycle.
__global__ __launch_bounds__(kThreads) void brestart_kernel(KrySys* __restrict__ ds, int m,
                                                            const double* __restrict__ nrm2) {
  const KrySys d = *ds;
  const double beta = sqrt(nrm2[0]);
  const bool again = d.status == kRestart && isfinite(beta) && beta > 0;
  if (again)
    for (int e = threadIdx.x; e < (m + 1) * m; e += kThreads) d.H[e] = 0.0;
  if (threadIdx.x == 0) {
    ds->beta = beta;
    ds->epoch = d.epoch + 1;
    if (again) {
      ds->j = 0;
      ds->status = kRun;
      ds->active = 1;
      *d.mask = 1;
    } else if (d.status == kRestart) {
      ds->status = isfinite(beta) ? kExact : kFailed;
    }
  }
}

template <typename Tv>
__global__ __launch_bounds__(kThreads) void bcopy_in_kernel(const KrySys* __restrict__ sys,
                                                            const int* __restrict__ map) {
  const KrySys d = sys[map[blockIdx.x]];
  if (!d.active) return;
  Tv* dst = (Tv*)d.vin;
  const int64_t base = (int64_t)(blockIdx.x - d.u0) * kElBlock + threadIdx.x;
#pragma unroll
  for (int e = 0; e < kEl; ++e) {
    const int64_t i = base + (int64_t)e * kThreads;
    if (i < d.n) dst[i] = (Tv)d.u[i];
  }
}

template <typename Tz>
__global__ __launch_bounds__(kThreads) void bcopy_out_kernel(const KrySys* __restrict__ sys,
                                                             const int* __restrict__ map) {
  const KrySys d = sys[map[blockIdx.x]];
  if (!d.active) return;
  const Tz* src = (const Tz*)d.vout;
  Tz* dst = (Tz*)d.Z + (int64_t)d.j * d.n;
  const int64_t base = (int64_t)(blockIdx.x - d.u0) * kElBlock + threadIdx.x;
#pragma unroll
  for (int e = 0; e < kEl; ++e) {
    const int64_t i = base + (int64_t)e * kThreads;
    if (i < d.n) dst[i] = src[i];
  }
}


}  // namespace
}  // namespace c0ip

using namespace c0ip;

namespace {

thread_local std::string b_err;
c0ip_status bfail(c0ip_status s, const std::string& m) {
  b_err = m;
  c0ip_internal_set_error(m);
  return s;
}

struct HErr {
  hipError_t e;
  const char* what;
};
inline void hchk(hipError_t e, const char* w) {
  if (e != hipSuccess) throw HErr{e, w};
}

template <typename T>
struct Buf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t c) {
    if (p && c <= n) return;
    if (p) (void)hipFree(p);
    p = nullptr;
    hchk(hipMalloc((void**)&p, std::max<size_t>(c, 1) * sizeof(T)), "hipMalloc");
    n = c;
  }
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

struct Sys {  // one (problem, right-hand side)
  int problem = 0, rhs = 0, group = 0, slot = 0, L = 0, N = 0;
  int64_t n = 0;
  const double* b = nullptr;
  double* x = nullptr;
  Buf<double> V, u, r;
  Buf<double> Z64;
  Buf<float> Z32;
  Buf<double> H, y;  // Hessenberg matrix and update coefficients (device)
  double bnorm = 0;
};

struct Group {
  int k = 0;
  double gamma = 0;
  int Lmax = 0;
  std::vector<int> members;  // system indices, slot order (descending L)
  std::vector<int> A;        // A[l] = systems with L_s >= l (a prefix of the slots)
  c0ip_problem* proto = nullptr;  // tables for levels 0..Lmax
  std::vector<std::unique_ptr<Buf<float>>> x32, b32, r32, t32;
  std::vector<std::unique_ptr<Buf<double>>> x64, b64, r64, t64;
  std::vector<std::unique_ptr<Buf<double>>> W;  // A z of systems whose finest level is l
  Buf<int> mask;
  hipStream_t stream = nullptr;  // its branch of a round (groups after the first)
  hipEvent_t join_ev = nullptr;
};

}  // namespace

struct c0ip_batch {
  int dim = 2;
  c0ip_mg_opts mg{};
  hipStream_t user = nullptr, s = nullptr;
  std::vector<Sys> sys;
  std::vector<Group> groups;
  std::vector<int> nrhs;
  std::vector<c0ip_mesh_desc> meshes;
  int m = 0;
  Buf<KrySys> dsys;
  Buf<KryParams> dprm;
  Buf<int> umap, dmap;  // block -> system maps of the copy / update and the dots grids
  int64_t umap_n = 0, dmap_n = 0;
  Buf<double> partial, hout, coef, scal;
  KrySys* hsys = nullptr;  // pinned: the solve's initial state, then the final one
  KrySys* hsnap = nullptr;  // pinned: kRing snapshots of the state, one per round in flight
  KryParams* hprm = nullptr;
  double* hscal = nullptr;
  hipGraph_t graph[kRing] = {};
  hipGraphExec_t exec[kRing] = {};
  hipEvent_t ev[kRing] = {};
  hipEvent_t fork_ev = nullptr;
  int graph_m = -1;
  ~c0ip_batch() {
    for (int i = 0; i < kRing; ++i) {
      if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
      if (graph[i]) (void)hipGraphDestroy(graph[i]);
      if (ev[i]) (void)hipEventDestroy(ev[i]);
    }
    for (auto& g : groups) {
      c0ip_destroy(g.proto);
      if (g.join_ev) (void)hipEventDestroy(g.join_ev);
      if (g.stream) (void)hipStreamDestroy(g.stream);
    }
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (hsys) (void)hipHostFree(hsys);
    if (hsnap) (void)hipHostFree(hsnap);
    if (hprm) (void)hipHostFree(hprm);
    if (hscal) (void)hipHostFree(hscal);
    if (s) (void)hipStreamDestroy(s);
  }

  template <typename T>
  void vcycle(Group& g, hipStream_t gs);
  void az(Group& g, hipStream_t st, bool f32);
  void record_round(int slot);
};

template <typename T>
static Buf<T>& lvbuf(Group& g, int which, int l);
template <>
Buf<float>& lvbuf<float>(Group& g, int which, int l) {
  return which == 0 ? *g.x32[l] : (which == 1 ? *g.b32[l] : (which == 2 ? *g.r32[l] : *g.t32[l]));
}
template <>
Buf<double>& lvbuf<double>(Group& g, int which, int l) {
  return which == 0 ? *g.x64[l] : (which == 1 ? *g.b64[l] : (which == 2 ? *g.r64[l] : *g.t64[l]));
}

// Algorithm 1 for every system of the group at once (see the file comment).
template <typename T>
void c0ip_batch::vcycle(Group& g, hipStream_t gs) {
  const int k = g.k, pre = mg.pre_steps, post = mg.post_steps;
  const T om = (T)mg.omega;
  auto n1 = [&](int l) { return (int64_t)(k * (2 << l) + 1) * (k * (2 << l) + 1); };
  const int* mask = g.mask.p;
  // levels 0..LT run as one single-workgroup launch per system (LT < 1: none)
  TailParams<T> tp;
  const int LT = c0ip_internal_tail<T>(g.proto, &tp);
  const int lo = LT >= 1 ? LT : 0;
  for (int l = g.Lmax; l > lo; --l) {
    const int nA = g.A[l];
    if (nA == 0) continue;
    const int Nl = 2 << l;
    const int64_t nl = n1(l);
    T *x = lvbuf<T>(g, 0, l).p, *b = lvbuf<T>(g, 1, l).p, *r = lvbuf<T>(g, 2, l).p;
    const auto& coef = c0ip_internal_coef<T>(g.proto, l);
    const auto& eig = c0ip_internal_eig<T>(g.proto, l);
    // the iterate alternates between x and t; the pre-smoothing result lands
    // in A, chosen so that the post-smoothing steps end in x
    T* A = (post % 2 == 1) ? lvbuf<T>(g, 3, l).p : x;
    T* B = (A == x) ? lvbuf<T>(g, 3, l).p : x;
    if (pre == 0) {
      hchk(launch_fill_t<T>(nA * nl, T(0), A, gs), "fill");
    } else {
      T* cur = (pre % 2 == 1) ? A : B;
      hchk(launch_patch2d<T>(k, Nl, eig, b, nullptr, cur, om, gs, nA, nl, mask), "patch");
      for (int st = 1; st < pre; ++st) {
        T* nxt = (cur == A) ? B : A;
        hchk(launch_avs2d<T>(k, Nl, coef, eig, cur, b, nxt, om, gs, nA, nl, mask, c0ip_internal_variant<T>(g.proto, l)),
             "fused smoother");
        cur = nxt;
      }
    }
    hchk(launch_apply2d<T, T>(k, Nl, coef, A, b, r, gs, nA, nl, mask), "residual");
    hchk(launch_restrict2d<T>(k, Nl / 2, c0ip_internal_ptab<T>(g.proto, l), r, lvbuf<T>(g, 1, l - 1).p, gs, nA, nl,
                              n1(l - 1), mask),
         "restrict");
  }
  if (LT >= 1) {
    TailIO<T> io;
    for (int l = 0; l <= LT; ++l) {
      io.b[l] = lvbuf<T>(g, 1, l).p;
      io.x[l] = lvbuf<T>(g, 0, l).p;
      io.stride[l] = n1(l);
      io.nA[l] = g.A[l];
    }
    io.active = mask;
    hchk(launch_vtail<T>(k, tp, io, g.A[0], gs), "tail V-cycle");
  } else {
    const int nA = g.A[0];
    if (mg.coarse_mode == 0)
      hchk(launch_coarse<T>(2, k, c0ip_internal_coarse(g.proto), lvbuf<T>(g, 1, 0).p, lvbuf<T>(g, 0, 0).p, gs, nA,
                            n1(0), mask),
           "coarse");
    else
      hchk(launch_patch2d<T>(k, 2, c0ip_internal_eig<T>(g.proto, 0), lvbuf<T>(g, 1, 0).p, nullptr,
                             lvbuf<T>(g, 0, 0).p, T(1), gs, nA, n1(0), mask),
           "coarse smooth");
  }
  for (int l = lo + 1; l <= g.Lmax; ++l) {
    const int nA = g.A[l];
    if (nA == 0) continue;
    const int Nl = 2 << l;
    const int64_t nl = n1(l);
    T *x = lvbuf<T>(g, 0, l).p, *b = lvbuf<T>(g, 1, l).p;
    const auto& coef = c0ip_internal_coef<T>(g.proto, l);
    const auto& eig = c0ip_internal_eig<T>(g.proto, l);
    const T* ptab = c0ip_internal_ptab<T>(g.proto, l);
    T* A = (post % 2 == 1) ? lvbuf<T>(g, 3, l).p : x;
    T* B = (A == x) ? lvbuf<T>(g, 3, l).p : x;
    if (post == 0) {
      hchk(launch_prolong2d<T>(k, Nl / 2, ptab, lvbuf<T>(g, 0, l - 1).p, A, x, gs, nA, n1(l - 1), nl, mask), "prolong");
      continue;
    }
    // first post-smoothing step from A + P e (fused), then alternate; ends in x
    hchk(launch_avs2d<T>(k, Nl, coef, eig, A, b, B, om, gs, nA, nl, mask, c0ip_internal_variant<T>(g.proto, l),
                         lvbuf<T>(g, 0, l - 1).p, ptab, n1(l - 1)),
         "prolongation + fused smoother");
    T* cur = B;
    for (int st = 1; st < post; ++st) {
      T* nxt = (cur == A) ? B : A;
      hchk(launch_avs2d<T>(k, Nl, coef, eig, cur, b, nxt, om, gs, nA, nl, mask, c0ip_internal_variant<T>(g.proto, l)),
           "fused smoother");
      cur = nxt;
    }
  }
}

// A z for every system of the group, at each system's finest level, into W.
void c0ip_batch::az(Group& g, hipStream_t st, bool f32) {
  for (int l = 0; l <= g.Lmax; ++l) {  // level 0 too: meshes of 2 x 2 cells
    const int first = (l + 1 <= g.Lmax) ? g.A[l + 1] : 0, cnt = g.A[l] - first;
    if (cnt <= 0) continue;
    const int Nl = 2 << l;
    const int64_t nl = (int64_t)(g.k * Nl + 1) * (g.k * Nl + 1);
    const auto& c64 = c0ip_internal_coef<double>(g.proto, l);
    if (f32)
      hchk(launch_apply2d<float, double>(g.k, Nl, c64, g.x32[l]->p + first * nl, nullptr, g.W[l]->p, st, cnt, nl,
                                         g.mask.p + first),
           "A z");
    else
      hchk(launch_apply2d<double, double>(g.k, Nl, c64, g.x64[l]->p + first * nl, nullptr, g.W[l]->p, st, cnt, nl,
                                          g.mask.p + first),
           "A z");
  }
}

// One round for every active system: V-cycle inputs, V-cycles, z -> Z_j,
// A z, one reduction, coefficients, the basis update, the Givens step, and a
// copy of every system's state to the host (snapshot slot `slot`).
void c0ip_batch::record_round(int slot) {
  const int ns = (int)sys.size();
  const bool f32 = mg.vcycle_dtype == C0IP_F32;
  const int gu = (int)umap_n, gd = (int)dmap_n;
  if (f32)
    bcopy_in_kernel<float><<<gu, kThreads, 0, s>>>(dsys.p, umap.p);
  else
    bcopy_in_kernel<double><<<gu, kThreads, 0, s>>>(dsys.p, umap.p);
  hchk(hipGetLastError(), "copy in");
  // the groups' V-cycles and A z are independent: group 0 on the round's
  // stream, every other group on a stream of its own, forked and joined by
  // events (parallel branches of the captured graph)
  hchk(hipEventRecord(fork_ev, s), "fork");
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Group& g = groups[gi];
    const hipStream_t st = gi == 0 ? s : g.stream;
    if (gi > 0) hchk(hipStreamWaitEvent(st, fork_ev, 0), "fork");
    if (f32)
      vcycle<float>(g, st);
    else
      vcycle<double>(g, st);
    az(g, st, f32);
    if (gi > 0) {
      hchk(hipEventRecord(g.join_ev, st), "join");
      hchk(hipStreamWaitEvent(s, g.join_ev, 0), "join");
    }
  }
  if (f32)
    bcopy_out_kernel<float><<<gu, kThreads, 0, s>>>(dsys.p, umap.p);
  else
    bcopy_out_kernel<double><<<gu, kThreads, 0, s>>>(dsys.p, umap.p);
  hchk(hipGetLastError(), "copy out");
  double vbytes = 0;
  for (auto& q : sys) vbytes += (double)q.n * m * sizeof(double);
  if (vbytes > 256.0 * (1 << 20))
    bdots_kernel<true><<<gd, kThreads, 0, s>>>(dsys.p, dmap.p, partial.p);
  else
    bdots_kernel<false><<<gd, kThreads, 0, s>>>(dsys.p, dmap.p, partial.p);
  hchk(hipGetLastError(), "dots");
  breduce_kernel<<<dim3(2 * m + 3, ns), kThreads, 0, s>>>(dsys.p, m, partial.p, hout.p);
  hchk(hipGetLastError(), "reduce");
  bcoef_kernel<<<(ns + 63) / 64, 64, 0, s>>>(dsys.p, ns, m, hout.p, coef.p);
  hchk(hipGetLastError(), "coef");
  bupdate_kernel<<<gu, kThreads, 0, s>>>(dsys.p, umap.p, m, coef.p);
  hchk(hipGetLastError(), "update");
  bgivens_kernel<<<ns, kThreads, 0, s>>>(dsys.p, m, hout.p, coef.p, dprm.p);
  hchk(hipGetLastError(), "givens");
  hchk(hipMemcpyAsync(hsnap + (size_t)slot * ns, dsys.p, sizeof(KrySys) * ns, hipMemcpyDeviceToHost, s), "D2H");
}

extern "C" {

c0ip_status c0ip_batch_create(const c0ip_mesh_desc* meshes, const int* n_rhs, int n_problems,
                              const c0ip_mg_opts* opts, void* hip_stream, c0ip_batch** out) {
  b_err.clear();
  if (!out || !meshes || !n_rhs || n_problems < 1) return bfail(C0IP_EINVAL, "bad batch arguments");
  *out = nullptr;
  c0ip_mg_opts mg;
  if (opts) {
    mg = *opts;
  } else {
    mg.omega = 0.25;
    mg.pre_steps = mg.post_steps = 1;
    mg.vcycle_dtype = C0IP_F32;
    mg.coarse_mode = 0;
    mg.scatter_mode = 0;
    mg.tail_levels = -1;
    mg.smoother = 0;
    mg.local_solver = 0;
    mg.mvs_residual = 0;
  }
  if (mg.mvs_residual != 0) return bfail(C0IP_EUNSUPPORTED, "batched solves take mvs_residual 0");
  if (mg.scatter_mode != 0)
    return bfail(C0IP_EUNSUPPORTED, "batched solves use the owner-computes smoother (scatter_mode 0)");
  if (mg.smoother != 0)
    return bfail(C0IP_EUNSUPPORTED, "batched solves use the additive smoother (smoother 0)");
  if (mg.local_solver != 0)
    return bfail(C0IP_EUNSUPPORTED, "batched solves use the separable local solver (local_solver 0)");
  for (int i = 0; i < n_problems; ++i) {  // every mesh, before any device call
    const c0ip_mesh_desc& md = meshes[i];
    if (md.dim != 2) return bfail(C0IP_EUNSUPPORTED, "batches are built for 2D meshes");
    if (n_rhs[i] < 1 || n_rhs[i] > 4096) return bfail(C0IP_EINVAL, "n_rhs must be in [1, 4096]");
    if (md.degree < 2 || md.degree > 7 || md.n_cells < 2 || (md.n_cells & (md.n_cells - 1)) ||
        md.n_cells > (1 << 16) ||
        ((int64_t)md.degree * md.n_cells + 1) * ((int64_t)md.degree * md.n_cells + 1) >= (int64_t(1) << 31))
      return bfail(C0IP_EINVAL, "bad mesh in batch (degree 2..7, n_cells a power of two, < 2^31 DoFs)");
  }
  std::unique_ptr<c0ip_batch> bt(new c0ip_batch());
  bt->mg = mg;
  bt->user = (hipStream_t)hip_stream;
  try {
    hchk(hipStreamCreateWithFlags(&bt->s, hipStreamNonBlocking), "stream");
    // systems
    for (int i = 0; i < n_problems; ++i) {
      const c0ip_mesh_desc& md = meshes[i];
      bt->meshes.push_back(md);
      bt->nrhs.push_back(n_rhs[i]);
      const double gam = md.gamma > 0 ? md.gamma : (double)(md.degree * (md.degree + 1));
      int gi = -1;
      for (size_t q = 0; q < bt->groups.size(); ++q)
        if (bt->groups[q].k == md.degree && bt->groups[q].gamma == gam) gi = (int)q;
      if (gi < 0) {
        bt->groups.emplace_back();
        bt->groups.back().k = md.degree;
        bt->groups.back().gamma = gam;
        gi = (int)bt->groups.size() - 1;
      }
      int L = 0;
      while ((2 << L) < md.n_cells) ++L;
      for (int r = 0; r < n_rhs[i]; ++r) {
        Sys q;
        q.problem = i;
        q.rhs = r;
        q.group = gi;
        q.L = L;
        q.N = md.n_cells;
        q.n = (int64_t)(md.degree * md.n_cells + 1) * (md.degree * md.n_cells + 1);
        bt->sys.push_back(std::move(q));
        bt->groups[gi].members.push_back((int)bt->sys.size() - 1);
      }
    }
    // groups: slot order, level prefix counts, tables, level slot buffers
    for (auto& g : bt->groups) {
      std::stable_sort(g.members.begin(), g.members.end(),
                       [&](int a, int b) { return bt->sys[a].L > bt->sys[b].L; });
      g.Lmax = bt->sys[g.members.front()].L;
      g.A.assign(g.Lmax + 2, 0);
      for (size_t si = 0; si < g.members.size(); ++si) {
        Sys& q = bt->sys[g.members[si]];
        q.slot = (int)si;
        for (int l = 0; l <= q.L; ++l) g.A[l]++;
      }
      c0ip_mesh_desc md{2, 2 << g.Lmax, g.k, g.gamma};
      c0ip_mg_opts mo = mg;
      c0ip_status st = c0ip_create(&md, &mo, (void*)bt->s, &g.proto);
      if (st != C0IP_OK) return st;
      st = c0ip_autotune(g.proto, 3);
      if (st != C0IP_OK) return st;
      const bool f32 = mg.vcycle_dtype == C0IP_F32;
      {  // choose (and allow the LDS of) the tail before any graph capture
        TailParams<float> t32;
        TailParams<double> t64;
        if (f32)
          (void)c0ip_internal_tail<float>(g.proto, &t32);
        else
          (void)c0ip_internal_tail<double>(g.proto, &t64);
      }
      for (int l = 0; l <= g.Lmax; ++l) {
        const int64_t nl = (int64_t)(g.k * (2 << l) + 1) * (g.k * (2 << l) + 1);
        const size_t cnt = (size_t)g.A[l] * nl;
        if (f32) {
          g.x32.emplace_back(new Buf<float>());
          g.b32.emplace_back(new Buf<float>());
          g.r32.emplace_back(new Buf<float>());
          g.t32.emplace_back(new Buf<float>());
          g.t32.back()->alloc(cnt);
          g.x32.back()->alloc(cnt);
          g.b32.back()->alloc(cnt);
          g.r32.back()->alloc(cnt);
        } else {
          g.x64.emplace_back(new Buf<double>());
          g.b64.emplace_back(new Buf<double>());
          g.r64.emplace_back(new Buf<double>());
          g.t64.emplace_back(new Buf<double>());
          g.t64.back()->alloc(cnt);
          g.x64.back()->alloc(cnt);
          g.b64.back()->alloc(cnt);
          g.r64.back()->alloc(cnt);
        }
        const int fin = g.A[l] - (l + 1 <= g.Lmax ? g.A[l + 1] : 0);
        g.W.emplace_back(new Buf<double>());
        g.W.back()->alloc((size_t)std::max(fin, 0) * nl);
      }
      g.mask.alloc(g.members.size());
      hchk(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking), "stream");
      hchk(hipEventCreateWithFlags(&g.join_ev, hipEventDisableTiming), "event");
    }
    hchk(hipEventCreateWithFlags(&bt->fork_ev, hipEventDisableTiming), "event");
  } catch (const HErr& h) {
    return bfail(C0IP_EHIP, std::string(h.what) + ": " + hipGetErrorString(h.e));
  } catch (const std::bad_alloc&) {
    return bfail(C0IP_ENOMEM, "host allocation failed");
  }
  *out = bt.release();
  return C0IP_OK;
}

c0ip_status c0ip_batch_destroy(c0ip_batch* bt) {
  delete bt;
  return C0IP_OK;
}

c0ip_status c0ip_batch_num_systems(const c0ip_batch* bt, int* n) {
  if (!bt || !n) return bfail(C0IP_EINVAL, "NULL argument");
  *n = (int)bt->sys.size();
  return C0IP_OK;
}

c0ip_status c0ip_batch_solve(c0ip_batch* bt, const c0ip_krylov_opts* opts, const double* const* b,
                             double* const* x, c0ip_solve_info* infos) {
  b_err.clear();
  if (!bt || !opts || !b || !x) return bfail(C0IP_EINVAL, "NULL argument");
  if (!(opts->rtol > 0) || opts->max_iters < 1 || opts->restart < 1 || opts->restart > kMaxM)
    return bfail(C0IP_EINVAL, "bad Krylov options (rtol > 0, max_iters >= 1, restart in [1,64])");
  const int m = opts->restart, ns = (int)bt->sys.size();
  const bool f32 = bt->mg.vcycle_dtype == C0IP_F32;
  hipStream_t s = bt->s;
  auto t0 = std::chrono::steady_clock::now();
  c0ip_status result = C0IP_OK;
  hipEvent_t ev = nullptr;
  try {
    for (int i = 0; i < (int)bt->meshes.size(); ++i)
      if (!b[i] || !x[i]) return bfail(C0IP_EINVAL, "NULL vector in batch");
    // order after the caller's pending work
    hchk(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
    hchk(hipEventRecord(ev, bt->user), "event");
    hchk(hipStreamWaitEvent(s, ev, 0), "wait");
    // work space
    bt->m = m;
    int64_t poff = 0;
    for (auto& q : bt->sys) {
      q.b = b[q.problem] + (size_t)q.rhs * q.n;
      q.x = x[q.problem] + (size_t)q.rhs * q.n;
      q.V.alloc((size_t)m * q.n);
      q.u.alloc(q.n);
      q.r.alloc(q.n);
      if (f32) q.Z32.alloc((size_t)m * q.n);
      else q.Z64.alloc((size_t)m * q.n);
      q.H.alloc((size_t)(m + 1) * m);
      q.y.alloc(m);
      poff += (int64_t)(2 * m + 3) * ((q.n + kChunk - 1) / kChunk);
    }
    int64_t nmax = 0;
    for (auto& q : bt->sys) nmax = std::max(nmax, q.n);
    bt->partial.alloc(std::max<int64_t>(poff, multidot_blocks(nmax)));
    bt->hout.alloc((size_t)ns * (2 * m + 3));
    bt->coef.alloc((size_t)ns * (2 * m + 5));
    bt->scal.alloc((size_t)2 * ns);
    bt->dsys.alloc(ns);
    bt->dprm.alloc(1);
    if (!bt->hsys) {
      hchk(hipHostMalloc((void**)&bt->hsys, sizeof(KrySys) * ns), "pinned");
      hchk(hipHostMalloc((void**)&bt->hsnap, sizeof(KrySys) * ns * kRing), "pinned");
      hchk(hipHostMalloc((void**)&bt->hprm, sizeof(KryParams)), "pinned");
      hchk(hipHostMalloc((void**)&bt->hscal, sizeof(double) * 2 * ns), "pinned");
      for (int i = 0; i < kRing; ++i) hchk(hipEventCreateWithFlags(&bt->ev[i], hipEventDisableTiming), "event");
    }
    // ||r||^2 of a system's r into scal[slot] (device), no host round trip
    auto norm2_dev = [&](const Sys& q, int slot) {
      const int nb = multidot_blocks(q.n);
      hchk(launch_multidot(q.n, 1, q.r.p, q.n, q.r.p, bt->partial.p, nb, s), "norm");
      hchk(launch_reduce_partials(1, nb, bt->partial.p, bt->scal.p + slot, 0, s), "norm");
    };
    auto residual = [&](Sys& q, const double* xx) {
      Group& g = bt->groups[q.group];
      hchk(launch_apply2d<double, double>(g.k, q.N, c0ip_internal_coef<double>(g.proto, q.L), xx, q.b, q.r.p, s),
           "residual");
    };
    // initial state: ||b|| over the free DoFs (r = b - A 0) and beta = ||b - A x0||, one host sync for all
    for (int i = 0; i < ns; ++i) {
      Sys& q = bt->sys[i];
      hchk(launch_fill(q.n, 0.0, q.u.p, s), "fill");
      residual(q, q.u.p);
      norm2_dev(q, 2 * i);
      if (opts->x0_is_zero) hchk(launch_fill(q.n, 0.0, q.x, s), "fill");
      else residual(q, q.x);
      norm2_dev(q, 2 * i + 1);
      hchk(launch_fill((size_t)(m + 1) * m, 0.0, q.H.p, s), "fill");
    }
    hchk(hipMemcpyAsync(bt->hscal, bt->scal.p, sizeof(double) * 2 * ns, hipMemcpyDeviceToHost, s), "D2H");
    hchk(hipStreamSynchronize(s), "sync");
    int running = 0;
    std::vector<int> host_epoch(ns, 0), done(ns, 0);
    for (int i = 0; i < ns; ++i) {
      Sys& q = bt->sys[i];
      Group& g = bt->groups[q.group];
      const int first = (q.L + 1 <= g.Lmax) ? g.A[q.L + 1] : 0;
      q.bnorm = std::sqrt(bt->hscal[2 * i]);
      const double beta = std::sqrt(bt->hscal[2 * i + 1]);
      KrySys& d = bt->hsys[i];
      d = KrySys{};
      d.V = q.V.p;
      d.u = q.u.p;
      d.w = g.W[q.L]->p + (int64_t)(q.slot - first) * q.n;
      d.Z = f32 ? (void*)q.Z32.p : (void*)q.Z64.p;
      d.vin = f32 ? (void*)(g.b32[q.L]->p + (int64_t)q.slot * q.n) : (void*)(g.b64[q.L]->p + (int64_t)q.slot * q.n);
      d.vout = f32 ? (const void*)(g.x32[q.L]->p + (int64_t)q.slot * q.n)
                   : (const void*)(g.x64[q.L]->p + (int64_t)q.slot * q.n);
      d.mask = g.mask.p + q.slot;
      d.H = q.H.p;
      d.y = q.y.p;
      d.n = q.n;
      d.nblk = (int)((q.n + kChunk - 1) / kChunk);
      d.bnorm = q.bnorm;
      d.beta = d.g0 = d.last = beta;
      const bool failed = !std::isfinite(q.bnorm) || !std::isfinite(beta);
      const bool conv = !failed && (q.bnorm == 0.0 || beta <= opts->rtol * q.bnorm);
      d.status = failed ? kFailed : (conv ? kConverged : kRun);
      d.active = d.status == kRun ? 1 : 0;
      if (d.active) {
        hchk(launch_normalize(q.n, q.r.p, bt->scal.p + 2 * i + 1, q.u.p, s), "normalize");
        ++running;
      } else {
        done[i] = 1;
      }
    }
    {
      // partial-sum offsets and the block -> system maps of the Krylov grids
      int64_t off = 0;
      std::vector<int> um, dm;
      for (int i = 0; i < ns; ++i) {
        KrySys& d = bt->hsys[i];
        d.poff = off;
        off += (int64_t)(2 * m + 3) * d.nblk;
        d.d0 = (int)dm.size();
        dm.insert(dm.end(), d.nblk, i);
        d.u0 = (int)um.size();
        um.insert(um.end(), (size_t)((d.n + kElBlock - 1) / kElBlock), i);
      }
      bt->umap.alloc(um.size());
      bt->dmap.alloc(dm.size());
      hchk(hipMemcpy(bt->umap.p, um.data(), sizeof(int) * um.size(), hipMemcpyHostToDevice), "H2D");
      hchk(hipMemcpy(bt->dmap.p, dm.data(), sizeof(int) * dm.size(), hipMemcpyHostToDevice), "H2D");
      if ((int64_t)um.size() != bt->umap_n || (int64_t)dm.size() != bt->dmap_n) bt->graph_m = -1;  // grid sizes
      bt->umap_n = (int64_t)um.size();
      bt->dmap_n = (int64_t)dm.size();
    }
    for (auto& g : bt->groups) {  // group masks from the initial state
      std::vector<int> msk(g.members.size());
      for (size_t si = 0; si < g.members.size(); ++si) msk[si] = bt->hsys[g.members[si]].active;
      hchk(hipMemcpy(g.mask.p, msk.data(), sizeof(int) * msk.size(), hipMemcpyHostToDevice), "H2D");
    }
    bt->hprm->rtol = opts->rtol;
    bt->hprm->max_iters = opts->max_iters;
    hchk(hipMemcpyAsync(bt->dprm.p, bt->hprm, sizeof(KryParams), hipMemcpyHostToDevice, s), "H2D");
    hchk(hipMemcpyAsync(bt->dsys.p, bt->hsys, sizeof(KrySys) * ns, hipMemcpyHostToDevice, s), "H2D");
    // capture the round graphs (reused while m is unchanged); they differ in their snapshot slot
    if (bt->graph_m != m) {
      for (int i = 0; i < kRing; ++i) {
        if (bt->exec[i]) (void)hipGraphExecDestroy(bt->exec[i]);
        if (bt->graph[i]) (void)hipGraphDestroy(bt->graph[i]);
        bt->exec[i] = nullptr;
        bt->graph[i] = nullptr;
      }
      bt->graph_m = -1;
      for (int i = 0; i < kRing; ++i) {
        hchk(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "capture");
        try {
          bt->record_round(i);
        } catch (...) {
          hipGraph_t tmp = nullptr;
          (void)hipStreamEndCapture(s, &tmp);
          if (tmp) (void)hipGraphDestroy(tmp);
          throw;
        }
        hchk(hipStreamEndCapture(s, &bt->graph[i]), "capture");
        hchk(hipGraphInstantiate(&bt->exec[i], bt->graph[i], nullptr, nullptr, 0), "instantiate");
      }
      bt->graph_m = m;
    }
    // Rounds run back to back with no host work between them: the device
    // advances and stops systems, and the host reads each round's state
    // snapshot kInFlight rounds later.  A stopped system's x += Z y,
    // residual and restart (or final beta) are queued behind the rounds in
    // flight; it sits idle (masked) until they run.  Every active system
    // spends at least one of its max_iters iterations per kInFlight + 1
    // rounds, which bounds the number of rounds.
    const int64_t max_rounds = (int64_t)(kInFlight + 2) * opts->max_iters + 16;
    int64_t t = 0;
    while (running > 0) {
      if (t >= max_rounds) throw HErr{hipErrorUnknown, "batched solve did not finish (internal error)"};
      const int slot = (int)(t % kRing);
      hchk(hipGraphLaunch(bt->exec[slot], s), "graph launch");
      hchk(hipEventRecord(bt->ev[slot], s), "event");
      ++t;
      if (t < kInFlight) continue;
      const int ps = (int)((t - kInFlight) % kRing);
      hchk(hipEventSynchronize(bt->ev[ps]), "sync");
      const KrySys* snap = bt->hsnap + (size_t)ps * ns;
      for (int i = 0; i < ns; ++i) {
        const KrySys& d = snap[i];
        if (done[i] || d.status == kRun || d.epoch != host_epoch[i]) continue;
        Sys& q = bt->sys[i];
        if (d.status == kFailed || d.status == kExact) {
          done[i] = 1;
          --running;
          continue;
        }
        const int jd = d.j + 1;
        if (f32)
          hchk(launch_update_solution<float>(q.n, jd, q.Z32.p, q.n, q.y.p, q.x, s), "update x");
        else
          hchk(launch_update_solution<double>(q.n, jd, q.Z64.p, q.n, q.y.p, q.x, s), "update x");
        residual(q, q.x);
        norm2_dev(q, 2 * i + 1);
        if (d.status == kRestart) hchk(launch_normalize(q.n, q.r.p, bt->scal.p + 2 * i + 1, q.u.p, s), "normalize");
        brestart_kernel<<<1, kThreads, 0, s>>>(bt->dsys.p + i, m, bt->scal.p + 2 * i + 1);
        hchk(hipGetLastError(), "restart");
        host_epoch[i]++;
        if (d.status != kRestart) {
          done[i] = 1;
          --running;
        }
      }
    }
    hchk(hipMemcpyAsync(bt->hsys, bt->dsys.p, sizeof(KrySys) * ns, hipMemcpyDeviceToHost, s), "D2H");
    hchk(hipStreamSynchronize(s), "sync");
    auto t1 = std::chrono::steady_clock::now();
    const double secs = std::chrono::duration<double>(t1 - t0).count();
    bool all = true, anynan = false;
    for (int i = 0; i < ns; ++i) {
      const KrySys& d = bt->hsys[i];
      const double bn = bt->sys[i].bnorm;
      const bool conv = d.status == kConverged || d.status == kExact;
      all = all && conv;
      anynan = anynan || d.status == kFailed || !std::isfinite(d.beta);
      if (infos) {
        c0ip_solve_info& inf = infos[i];
        inf = c0ip_solve_info{};
        inf.iterations = d.its;
        inf.converged = conv ? 1 : 0;
        inf.rel_res_est = bn > 0 ? d.last / bn : 0.0;
        inf.rel_res_true = bn > 0 ? d.beta / bn : 0.0;
        inf.frac_iters = (d.its > 0 && inf.rel_res_est > 0) ? 8.0 * d.its / (-std::log10(inf.rel_res_est)) : 0.0;
        inf.seconds_total = secs;
      }
    }
    if (anynan) result = bfail(C0IP_ENAN, "non-finite value in a batched system");
    else if (!all) result = bfail(C0IP_NOT_CONVERGED, "some systems reached max_iters");
  } catch (const HErr& h) {
    (void)hipStreamSynchronize(s);
    result = bfail(C0IP_EHIP, std::string(h.what) + ": " + hipGetErrorString(h.e));
  }
  if (ev) (void)hipEventDestroy(ev);
  return result;
}

}  // extern "C"
