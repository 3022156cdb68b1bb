// Solve phase: preconditioned CG with one smoothed-aggregation V-cycle per
// iteration, all on the GPU.  Every kernel here streams CSR data (HBM-bound):
//   - a group of G lanes per row (G = 1..64, G = 64 is a wavefront per row),
//     chosen per matrix from its row length; consecutive rows of a block are
//     consecutive in memory, so column/value streams are coalesced;
//   - rows are dealt to workgroups in contiguous chunks, and workgroups are
//     renumbered so that each XCD (workgroups are dispatched round-robin over
//     the 8 XCDs) works on one contiguous range, which keeps neighbour
//     gathers in that XCD's L2;
//   - dot products are fused into the producing kernel and reduced
//     deterministically (fixed tree + last-workgroup fold, no float atomics);
//   - CG scalars stay on the device; the host only reads a done flag every
//     few iterations.
// Method: PCG from x0 = 0 with recursive-residual stopping, true-residual
// verification and restart; damped-Jacobi/L1 V(nu_pre, nu_post) cycle with
// R = P^T and an exact coarsest solve (the oracle states the same algorithm
// step by step).  The FP32 cycle keeps CG vectors, dot products and updates
// in FP64 and runs the cycle on FP32 copies (bf16-stored P and R optional);
// the flexible (Polak-Ribiere) beta keeps CG consistent with that inexact
// preconditioner.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "amg_internal.hpp"

namespace amg {
namespace {

// ------------------------------------------------------------ geometry

// Workgroup index remapped so that XCD k (round-robin dispatch) owns the
// contiguous logical range [k*G/8, (k+1)*G/8).
__device__ inline int logical_block() {
  const int g = gridDim.x;
  if ((g & 7) == 0) return (blockIdx.x & 7) * (g >> 3) + (blockIdx.x >> 3);
  return blockIdx.x;
}

// Contiguous chunk range [c0, c1) of this workgroup; a chunk is kBlock/G rows.
template <int G>
__device__ inline void chunk_range(int n, int& c0, int& c1) {
  constexpr int rpp = kBlock / G;
  const int64_t chunks = ((int64_t)n + rpp - 1) / rpp;
  const int lb = logical_block();
  c0 = (int)(chunks * lb / gridDim.x);
  c1 = (int)(chunks * (lb + 1) / gridDim.x);
}

inline int stream_grid(int64_t n, int G) {
  const int64_t rpp = kBlock / G;
  int64_t chunks = (n + rpp - 1) / rpp;
  int64_t g = std::min<int64_t>(chunks, kMaxGrid);
  if (g >= 64) g = g / 8 * 8;
  return (int)std::max<int64_t>(g, 1);
}

template <class T>
__device__ inline T ld(const T* p) {
  return *p;
}

// Sum over the row of A: sum_j a_ij * f(j), lanes of a group stride the row.
#define ROW_SUM(G, rp, row, lane, body)                                          \
  do {                                                                           \
    for (int k_ = (rp)[row] + (lane); k_ < (rp)[(row) + 1]; k_ += (G)) { body; } \
  } while (0)

// --------------------------------------------------------- V-cycle kernels

// Pre-smoothing from zero fused with the residual:
//   x_i = sw_i b_i ;  r_i = b_i - sum_j a_ij (sw_j b_j).
template <int G, class VT, class BT, class T>
__global__ void __launch_bounds__(kBlock) k_pre(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                const VT* __restrict__ v, const T* __restrict__ sw,
                                                const BT* __restrict__ b, T* __restrict__ x, T* __restrict__ r,
                                                const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  int c0, c1;
  chunk_range<G>(n, c0, c1);
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  for (int c = c0; c < c1; ++c) {
    const int row = c * (kBlock / G) + grp;
    T s = 0;
    if (row < n) {
      ROW_SUM(G, rp, row, lane, {
        const int j = ci[k_];
        s += (T)v[k_] * (sw[j] * (T)b[j]);
      });
    }
    s = group_sum<G>(s);
    if (row < n && group_leader<G>()) {
      const T bi = (T)b[row];
      x[row] = sw[row] * bi;
      r[row] = bi - s;
    }
  }
}

// One further Jacobi sweep in residual form, fused with the new residual:
//   x'_i = x_i + sw_i r_i ;  r'_i = b_i - sum_j a_ij (x_j + sw_j r_j).
template <int G, class VT, class BT, class T>
__global__ void __launch_bounds__(kBlock) k_sweep(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const VT* __restrict__ v, const T* __restrict__ sw,
                                                  const BT* __restrict__ b, const T* __restrict__ x,
                                                  const T* __restrict__ r, T* __restrict__ x2, T* __restrict__ r2,
                                                  const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  int c0, c1;
  chunk_range<G>(n, c0, c1);
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  for (int c = c0; c < c1; ++c) {
    const int row = c * (kBlock / G) + grp;
    T s = 0;
    if (row < n) {
      ROW_SUM(G, rp, row, lane, {
        const int j = ci[k_];
        s += (T)v[k_] * (x[j] + sw[j] * r[j]);
      });
    }
    s = group_sum<G>(s);
    if (row < n && group_leader<G>()) {
      x2[row] = x[row] + sw[row] * r[row];
      r2[row] = (T)b[row] - s;
    }
  }
}

// Post-smoothing sweep out_i = x_i + sw_i (b_i - sum_j a_ij x_j).  RED = 1
// also reduces <b, out>; RED = 2 also <out, q> (level 0 of CG: b = r,
// out = z).
template <int G, class VT, class BT, class XT, class OT, int RED>
__global__ void __launch_bounds__(kBlock) k_post(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const VT* __restrict__ v, const XT* __restrict__ sw,
                                                 const BT* __restrict__ b, const XT* __restrict__ x,
                                                 OT* __restrict__ out, const double* __restrict__ q,
                                                 Ctl* __restrict__ ctl, double* __restrict__ partials, int first) {
  if (ctl && ctl->done) return;
  int c0, c1;
  chunk_range<G>(n, c0, c1);
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  double d0 = 0.0, d1 = 0.0;
  for (int c = c0; c < c1; ++c) {
    const int row = c * (kBlock / G) + grp;
    XT s = 0;
    if (row < n) {
      ROW_SUM(G, rp, row, lane, { s += (XT)v[k_] * x[ci[k_]]; });
    }
    s = group_sum<G>(s);
    if (row < n && group_leader<G>()) {
      const XT bi = (XT)b[row];
      const XT o = x[row] + sw[row] * (bi - s);
      out[row] = (OT)o;
      if constexpr (RED >= 1) d0 += (double)b[row] * (double)(OT)o;
      if constexpr (RED >= 2) d1 += (double)(OT)o * q[row];
    }
  }
  if constexpr (RED >= 1) {
    double vals[2] = {d0, d1};
    if (grid_sum<2>(vals, partials, &ctl->ticket[2]) && threadIdx.x == 0) {
      const double rzn = vals[0];
      if (first) {
        ctl->rz = rzn;
        ctl->beta = 0.0;
      } else if (ctl->flexible) {
        // Polak-Ribiere: beta = <z, r - r_old>/<z_old, r_old> = -<z, q>/<p, q>
        ctl->beta = -vals[1] / ctl->pq;
        ctl->rz = rzn;
      } else {
        ctl->beta = rzn / ctl->rz;
        ctl->rz = rzn;
      }
      ctl->rzn = rzn;
      ctl->zq = vals[1];
      if (!(rzn > 0.0)) {
        ctl->state = -1;
        ctl->done = 1;
      }
    }
  }
}

// b_c = R r (restriction), R stored as CSR with n_c rows.
template <int G, class RT, class XT, class YT>
__global__ void __launch_bounds__(kBlock) k_restrict(int nc, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const RT* __restrict__ v, const XT* __restrict__ x,
                                                     YT* __restrict__ y, const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  int c0, c1;
  chunk_range<G>(nc, c0, c1);
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  using CT = decltype(ValCvt<RT>::f(RT()));
  for (int c = c0; c < c1; ++c) {
    const int row = c * (kBlock / G) + grp;
    CT s = 0;
    if (row < nc) {
      ROW_SUM(G, rp, row, lane, { s += ValCvt<RT>::f(v[k_]) * (CT)x[ci[k_]]; });
    }
    s = group_sum<G>(s);
    if (row < nc && group_leader<G>()) y[row] = (YT)s;
  }
}

// x += P x_c (prolongation and coarse-grid correction).
template <int G, class PT, class T>
__global__ void __launch_bounds__(kBlock) k_prolong(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                    const PT* __restrict__ v, const T* __restrict__ xc,
                                                    T* __restrict__ x, const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  int c0, c1;
  chunk_range<G>(n, c0, c1);
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  for (int c = c0; c < c1; ++c) {
    const int row = c * (kBlock / G) + grp;
    T s = 0;
    if (row < n) {
      ROW_SUM(G, rp, row, lane, { s += (T)ValCvt<PT>::f(v[k_]) * xc[ci[k_]]; });
    }
    s = group_sum<G>(s);
    if (row < n && group_leader<G>()) x[row] = x[row] + s;
  }
}

// Coarsest solve x = A_L^-1 b with the explicit (symmetric) inverse:
// thread i reads column i = row i, coalesced across threads.
template <class T, class BT, class OT>
__global__ void __launch_bounds__(kBlock) k_coarse(int n, int m, const T* __restrict__ inv, const BT* __restrict__ b,
                                                   OT* __restrict__ x, const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  __shared__ T sb[kBlock];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  T s = 0;
  for (int j0 = 0; j0 < n; j0 += kBlock) {
    const int jj = j0 + threadIdx.x;
    sb[threadIdx.x] = jj < n ? (T)b[jj] : (T)0;
    __syncthreads();
    const int jn = min(kBlock, n - j0);
    if (i < n)
      for (int t = 0; t < jn; ++t) s += inv[(int64_t)(j0 + t) * m + i] * sb[t];
    __syncthreads();
  }
  if (i < n) x[i] = (OT)s;
}

// <r, z> and <z, q> after a single-level (direct) preconditioner.
__global__ void __launch_bounds__(kBlock) k_dots_rz(int n, const double* __restrict__ r, const double* __restrict__ z,
                                                    const double* __restrict__ q, Ctl* __restrict__ ctl,
                                                    double* __restrict__ partials, int first) {
  if (ctl->done) return;
  double d0 = 0.0, d1 = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    d0 += r[i] * z[i];
    d1 += z[i] * q[i];
  }
  double vals[2] = {d0, d1};
  if (grid_sum<2>(vals, partials, &ctl->ticket[2]) && threadIdx.x == 0) {
    const double rzn = vals[0];
    if (first) {
      ctl->rz = rzn;
      ctl->beta = 0.0;
    } else if (ctl->flexible) {
      ctl->beta = -vals[1] / ctl->pq;
      ctl->rz = rzn;
    } else {
      ctl->beta = rzn / ctl->rz;
      ctl->rz = rzn;
    }
    ctl->rzn = rzn;
    ctl->zq = vals[1];
    if (!(rzn > 0.0)) {
      ctl->state = -1;
      ctl->done = 1;
    }
  }
}

// ------------------------------------------------------------ CG kernels

// r = b, x = 0, <b, b>; the last workgroup initialises the control block.
__global__ void __launch_bounds__(kBlock) k_cg_init(int n, const double* __restrict__ b, double* __restrict__ r,
                                                    double* __restrict__ x, Ctl* __restrict__ ctl,
                                                    double* __restrict__ partials, double tol, int maxiter,
                                                    int flexible) {
  double bb = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double bi = b[i];
    r[i] = bi;
    x[i] = 0.0;
    bb += bi * bi;
  }
  double vals[1] = {bb};
  if (grid_sum<1>(vals, partials, &ctl->ticket[0]) && threadIdx.x == 0) {
    const double t = vals[0];
    ctl->bb = t;
    ctl->thresh = (tol * tol) * t;
    ctl->iters = 0;
    ctl->maxiter = maxiter;
    ctl->flexible = flexible;
    ctl->state = 0;
    ctl->done = 0;
    ctl->trr = 0.0;
    if (t == 0.0) {
      ctl->state = 3;  // zero right-hand side: x = 0
      ctl->done = 1;
    } else if (!(t == t)) {
      ctl->state = -1;
      ctl->done = 1;
    } else if (maxiter <= 0) {
      ctl->state = 2;
      ctl->done = 1;
    }
  }
}

// q = A p fused with <p, q>; the last workgroup forms alpha.
template <int G>
__global__ void __launch_bounds__(kBlock) k_spmv_dot(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const double* __restrict__ v, const double* __restrict__ p,
                                                     double* __restrict__ q, Ctl* __restrict__ ctl,
                                                     double* __restrict__ partials) {
  if (ctl->done) return;
  int c0, c1;
  chunk_range<G>(n, c0, c1);
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  double d = 0.0;
  for (int c = c0; c < c1; ++c) {
    const int row = c * (kBlock / G) + grp;
    double s = 0.0;
    if (row < n) {
      ROW_SUM(G, rp, row, lane, { s += v[k_] * p[ci[k_]]; });
    }
    s = group_sum<G>(s);
    if (row < n && group_leader<G>()) {
      q[row] = s;
      d += p[row] * s;
    }
  }
  double vals[1] = {d};
  if (grid_sum<1>(vals, partials, &ctl->ticket[0]) && threadIdx.x == 0) {
    const double pq = vals[0];
    ctl->pq = pq;
    if (!(pq > 0.0)) {
      ctl->state = -1;
      ctl->done = 1;
    } else {
      ctl->alpha = ctl->rz / pq;
    }
  }
}

// x += alpha p ; r -= alpha q ; <r, r>; the last workgroup tests convergence.
__global__ void __launch_bounds__(kBlock) k_cg_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                      const double* __restrict__ p, const double* __restrict__ q,
                                                      Ctl* __restrict__ ctl, double* __restrict__ partials) {
  if (ctl->done) return;
  const double alpha = ctl->alpha;
  double rr = 0.0;
  int c0, c1;
  chunk_range<1>(n, c0, c1);
  const int i0 = c0 * kBlock, i1 = min(n, c1 * kBlock);
  for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
    x[i] = x[i] + alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    rr += ri * ri;
  }
  double vals[1] = {rr};
  if (grid_sum<1>(vals, partials, &ctl->ticket[1]) && threadIdx.x == 0) {
    const double t = vals[0];
    ctl->rr = t;
    ctl->iters += 1;
    if (t <= ctl->thresh) {
      ctl->state = 1;
      ctl->done = 1;
    } else if (!(t == t)) {
      ctl->state = -1;
      ctl->done = 1;
    } else if (ctl->iters >= ctl->maxiter) {
      ctl->state = 2;
      ctl->done = 1;
    }
  }
}

// p = z + beta p  (p = z on the first iteration of a (re)start).
__global__ void __launch_bounds__(kBlock) k_xpay(int n, const double* __restrict__ z, double* __restrict__ p,
                                                 const Ctl* __restrict__ ctl, int first) {
  if (ctl->done) return;
  const double beta = ctl->beta;
  int c0, c1;
  chunk_range<1>(n, c0, c1);
  const int i0 = c0 * kBlock, i1 = min(n, c1 * kBlock);
  if (first)
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) p[i] = z[i];
  else
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) p[i] = z[i] + beta * p[i];
}

// r = b - A x and ||r||^2 (true residual, FP64).
template <int G>
__global__ void __launch_bounds__(kBlock) k_true_resid(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ v, const double* __restrict__ b,
                                                       const double* __restrict__ x, double* __restrict__ r,
                                                       Ctl* __restrict__ ctl, double* __restrict__ partials) {
  int c0, c1;
  chunk_range<G>(n, c0, c1);
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  double d = 0.0;
  for (int c = c0; c < c1; ++c) {
    const int row = c * (kBlock / G) + grp;
    double s = 0.0;
    if (row < n) {
      ROW_SUM(G, rp, row, lane, { s += v[k_] * x[ci[k_]]; });
    }
    s = group_sum<G>(s);
    if (row < n && group_leader<G>()) {
      const double ri = b[row] - s;
      r[row] = ri;
      d += ri * ri;
    }
  }
  double vals[1] = {d};
  if (grid_sum<1>(vals, partials, &ctl->ticket[3]) && threadIdx.x == 0) ctl->trr = vals[0];
}

__global__ void k_ctl_restart(Ctl* ctl) {
  ctl->done = 0;
  ctl->state = 0;
}

// grad_val[k] = -(lambda[row k] * x[col k]).
template <int G>
__global__ void __launch_bounds__(kBlock) k_pattern_grad(int n, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, const double* __restrict__ lam,
                                                         const double* __restrict__ x, double* __restrict__ g) {
  int c0, c1;
  chunk_range<G>(n, c0, c1);
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  for (int c = c0; c < c1; ++c) {
    const int row = c * (kBlock / G) + grp;
    if (row < n) {
      const double li = lam[row];
      for (int k = rp[row] + lane; k < rp[row + 1]; k += G) g[k] = -(li * x[ci[k]]);
    }
  }
}

// --------------------------------------------------------- dispatch

#define AMG_DISPATCH_G(g, ...)                      \
  switch (g) {                                      \
    case 1: { constexpr int G = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int G = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int G = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int G = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int G = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int G = 32; __VA_ARGS__; } break; \
    default: { constexpr int G = 64; __VA_ARGS__; } break; \
  }

struct CycleArgs {
  const double* r0;   // level-0 right-hand side (CG residual), FP64
  double* z0;         // level-0 result, FP64
  const double* q;    // CG q (flexible reduction), may be null
  Ctl* ctl;           // null: no early exit, no reductions
  double* partials;
  int red;            // 0 none, 1 <r,z>, 2 <r,z> and <z,q>
  int first;
};

template <class T>
struct Bufs;

template <>
struct Bufs<double> {
  static double* x(Level& L) { return L.x64.p; }
  static double* b(Level& L) { return L.b64.p; }
  static double* r(Level& L) { return L.r64.p; }
  static const double* v(Level& L) { return L.v.p; }
  static const double* sw(Level& L) { return L.sw.p; }
  static double* xs(Level& L) { return L.xs64.p; }
  static double* rs(Level& L) { return L.rs64.p; }
  static const double* inv(Coarse& C) { return C.inv.p; }
};
template <>
struct Bufs<float> {
  static float* x(Level& L) { return L.x32.p; }
  static float* b(Level& L) { return L.b32.p; }
  static float* r(Level& L) { return L.r32.p; }
  static const float* v(Level& L) { return L.v32.p; }
  static const float* sw(Level& L) { return L.sw32.p; }
  static float* xs(Level& L) { return L.xs32.p; }
  static float* rs(Level& L) { return L.rs32.p; }
  static const float* inv(Coarse& C) { return C.inv32.p; }
};

template <class T, class BT>
void launch_pre(Level& L, const BT* b, T* x, T* r, const Ctl* ctl, hipStream_t s) {
  AMG_DISPATCH_G(L.gA, hipLaunchKernelGGL((k_pre<G, T, BT, T>), dim3(stream_grid(L.n, G)), dim3(kBlock), 0, s, L.n,
                                          L.rp.p, L.ci.p, Bufs<T>::v(L), Bufs<T>::sw(L), b, x, r, ctl));
}

template <class T, class BT>
void launch_sweep(Level& L, const BT* b, const T* x, const T* r, T* x2, T* r2, const Ctl* ctl, hipStream_t s) {
  AMG_DISPATCH_G(L.gA, hipLaunchKernelGGL((k_sweep<G, T, BT, T>), dim3(stream_grid(L.n, G)), dim3(kBlock), 0, s,
                                          L.n, L.rp.p, L.ci.p, Bufs<T>::v(L), Bufs<T>::sw(L), b, x, r, x2, r2, ctl));
}

template <class T, class BT, class OT, int RED>
void launch_post(Level& L, const BT* b, const T* x, OT* out, const CycleArgs& a, hipStream_t s) {
  AMG_DISPATCH_G(L.gA, hipLaunchKernelGGL((k_post<G, T, BT, T, OT, RED>), dim3(stream_grid(L.n, G)), dim3(kBlock), 0,
                                          s, L.n, L.rp.p, L.ci.p, Bufs<T>::v(L), Bufs<T>::sw(L), b, x, out, a.q,
                                          a.ctl, a.partials, a.first));
}

template <class T, class XT>
void launch_restrict(Hierarchy& H, Level& L, const XT* r, T* bc, const Ctl* ctl, hipStream_t s) {
  const int nc = L.nagg;
  if constexpr (std::is_same<T, double>::value) {
    AMG_DISPATCH_G(L.gR, hipLaunchKernelGGL((k_restrict<G, double, XT, T>), dim3(stream_grid(nc, G)), dim3(kBlock),
                                            0, s, nc, L.rrp.p, L.rci.p, L.rv.p, r, bc, ctl));
  } else if (H.bf16()) {
    AMG_DISPATCH_G(L.gR, hipLaunchKernelGGL((k_restrict<G, uint16_t, XT, T>), dim3(stream_grid(nc, G)),
                                            dim3(kBlock), 0, s, nc, L.rrp.p, L.rci.p, L.rbf.p, r, bc, ctl));
  } else {
    AMG_DISPATCH_G(L.gR, hipLaunchKernelGGL((k_restrict<G, float, XT, T>), dim3(stream_grid(nc, G)), dim3(kBlock),
                                            0, s, nc, L.rrp.p, L.rci.p, L.rv32.p, r, bc, ctl));
  }
}

template <class T>
void launch_prolong(Hierarchy& H, Level& L, const T* xc, T* x, const Ctl* ctl, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    AMG_DISPATCH_G(L.gP, hipLaunchKernelGGL((k_prolong<G, double, T>), dim3(stream_grid(L.n, G)), dim3(kBlock), 0, s,
                                            L.n, L.prp.p, L.pci.p, L.pv.p, xc, x, ctl));
  } else if (H.bf16()) {
    AMG_DISPATCH_G(L.gP, hipLaunchKernelGGL((k_prolong<G, uint16_t, T>), dim3(stream_grid(L.n, G)), dim3(kBlock), 0,
                                            s, L.n, L.prp.p, L.pci.p, L.pbf.p, xc, x, ctl));
  } else {
    AMG_DISPATCH_G(L.gP, hipLaunchKernelGGL((k_prolong<G, float, T>), dim3(stream_grid(L.n, G)), dim3(kBlock), 0, s,
                                            L.n, L.prp.p, L.pci.p, L.pv32.p, xc, x, ctl));
  }
}

// One V-cycle on level-0 rhs a.r0 -> a.z0 (FP64 at the boundary, T inside).
// Extra smoothing sweeps (nu > 1) ping-pong through the level's spare buffers.
template <class T>
void vcycle_impl(Hierarchy& H, const CycleArgs& a, hipStream_t s) {
  const int nl = (int)H.lv.size();
  Coarse& C = H.co;
  const Ctl* ectl = a.ctl;
  if (nl == 1) {
    hipLaunchKernelGGL((k_coarse<double, double, double>), dim3((C.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       C.n, C.m, C.inv.p, a.r0, a.z0, ectl);
    if (a.red)
      hipLaunchKernelGGL(k_dots_rz, dim3(stream_grid(C.n, 1)), dim3(kBlock), 0, s, C.n, a.r0, a.z0,
                         a.q ? a.q : a.z0, a.ctl, a.partials, a.first);
    return;
  }
  T* cx[AMG_MAX_LEVELS];
  T* cr[AMG_MAX_LEVELS];
  T* sx[AMG_MAX_LEVELS];
  T* sr[AMG_MAX_LEVELS];
  const int npre = H.prm.nu_pre, npost = H.prm.nu_post;
  for (int l = 0; l < nl - 1; ++l) {
    Level& L = H.lv[l];
    cx[l] = Bufs<T>::x(L);
    cr[l] = Bufs<T>::r(L);
    sx[l] = Bufs<T>::xs(L);
    sr[l] = Bufs<T>::rs(L);
    if (l == 0) launch_pre<T, double>(L, a.r0, cx[l], cr[l], ectl, s);
    else launch_pre<T, T>(L, Bufs<T>::b(L), cx[l], cr[l], ectl, s);
    for (int k = 1; k < npre; ++k) {
      if (l == 0) launch_sweep<T, double>(L, a.r0, cx[l], cr[l], sx[l], sr[l], ectl, s);
      else launch_sweep<T, T>(L, Bufs<T>::b(L), cx[l], cr[l], sx[l], sr[l], ectl, s);
      std::swap(cx[l], sx[l]);
      std::swap(cr[l], sr[l]);
    }
    launch_restrict<T, T>(H, L, cr[l], Bufs<T>::b(H.lv[l + 1]), ectl, s);
  }
  T* res;
  {
    Level& Lc = H.lv[nl - 1];
    hipLaunchKernelGGL((k_coarse<T, T, T>), dim3((C.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, C.n, C.m,
                       Bufs<T>::inv(C), Bufs<T>::b(Lc), Bufs<T>::x(Lc), ectl);
    res = Bufs<T>::x(Lc);
  }
  for (int l = nl - 2; l >= 0; --l) {
    Level& L = H.lv[l];
    launch_prolong<T>(H, L, res, cx[l], ectl, s);
    // free T buffers of this level after restriction: cr[l] and, with nu_pre > 1, sx[l]
    T* cur = cx[l];
    T* spare[2] = {cr[l], sx[l]};
    for (int k = 0; k < npost; ++k) {
      const bool last = (k == npost - 1);
      if (l == 0 && last) {
        if (a.red == 2) launch_post<T, double, double, 2>(L, a.r0, cur, a.z0, a, s);
        else if (a.red == 1) launch_post<T, double, double, 1>(L, a.r0, cur, a.z0, a, s);
        else launch_post<T, double, double, 0>(L, a.r0, cur, a.z0, a, s);
      } else {
        T* dst = spare[k & 1];
        if (l == 0) launch_post<T, double, T, 0>(L, a.r0, cur, dst, a, s);
        else launch_post<T, T, T, 0>(L, Bufs<T>::b(L), cur, dst, a, s);
        spare[k & 1] = cur;
        cur = dst;
      }
    }
    res = cur;
  }
  AMG_HIP(hipGetLastError());
}

void vcycle(Hierarchy& H, const CycleArgs& a, hipStream_t s) {
  if (H.fp32()) vcycle_impl<float>(H, a, s);
  else vcycle_impl<double>(H, a, s);
}

void read_ctl(Hierarchy& H, hipStream_t s) {
  AMG_HIP(hipMemcpyAsync(H.h_ctl, H.ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
}

}  // namespace

// ================================================================ public

void choose_shapes(Hierarchy& H) {
  auto pick = [](int64_t nnz, int64_t rows) {
    if (rows <= 0) return 1;
    double avg = (double)nnz / (double)rows;
    int g = pow2_ceil((int)std::ceil(avg));
    return std::min(64, std::max(1, g));
  };
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level& L = H.lv[l];
    L.gA = pick(L.nnz, L.n);
    if (l + 1 < H.lv.size()) {
      L.gP = pick(L.pnnz, L.n);
      L.gR = pick(L.pnnz, L.nagg);
    }
  }
}

void alloc_solve_workspace(Hierarchy& H) {
  const int n = H.n;
  H.r.alloc(n);
  H.z.alloc(n);
  H.p.alloc(n);
  H.q.alloc(n);
  H.partials.alloc((int64_t)kMaxGrid * 4);
  if (!H.ctl.p) {
    H.ctl.alloc(1);
    AMG_HIP(hipMemset(H.ctl.p, 0, sizeof(Ctl)));
  }
  if (!H.h_ctl) AMG_HIP(hipHostMalloc((void**)&H.h_ctl, sizeof(Ctl), hipHostMallocDefault));
  // spare vectors for extra smoothing sweeps
  if (H.prm.nu_pre > 1 || H.prm.nu_post > 1) {
    for (Level& L : H.lv) {
      if (H.fp32()) { L.xs32.alloc(L.n); L.rs32.alloc(L.n); }
      else { L.xs64.alloc(L.n); L.rs64.alloc(L.n); }
    }
  }
}

void apply_vcycle(Hierarchy& H, const double* d_r, double* d_z, hipStream_t s) {
  CycleArgs a{d_r, d_z, nullptr, nullptr, nullptr, 0, 0};
  vcycle(H, a, s);
  AMG_HIP(hipGetLastError());
}

void pattern_grad(Hierarchy& H, const double* d_lam, const double* d_x, double* d_g, hipStream_t s) {
  Level& L = H.lv[0];
  AMG_DISPATCH_G(L.gA, hipLaunchKernelGGL((k_pattern_grad<G>), dim3(stream_grid(L.n, G)), dim3(kBlock), 0, s, L.n,
                                          L.rp.p, L.ci.p, d_lam, d_x, d_g));
  AMG_HIP(hipGetLastError());
}

amg_status pcg_solve(Hierarchy& H, const SolveOpts& o, const double* d_b, double* d_x, double tol, int nrhs,
                     amg_info* info, hipStream_t s) {
  if (nrhs != 1) throw Error(AMG_ERR_INVALID_ARG, "this entry point takes one right-hand side");
  auto t0 = std::chrono::steady_clock::now();
  Level& L0 = H.lv[0];
  const int n = H.n;
  const int flexible = o.flexible < 0 ? (H.fp32() ? 1 : 0) : o.flexible;
  Ctl* ctl = H.ctl.p;
  double* part = H.partials.p;
  const int gcg = stream_grid(n, 1);
  hipLaunchKernelGGL(k_cg_init, dim3(gcg), dim3(kBlock), 0, s, n, d_b, H.r.p, d_x, ctl, part, tol, o.maxiter,
                     flexible);
  AMG_HIP(hipGetLastError());
  const int chunk = o.check_every > 0 ? o.check_every : 4;
  int restarts = 0;
  amg_status st = AMG_OK;
  for (;;) {
    // (re)start: z = M^-1 r, rz = <r, z>, p = z
    CycleArgs a0{H.r.p, H.z.p, H.q.p, ctl, part, 1, 1};
    vcycle(H, a0, s);
    hipLaunchKernelGGL(k_xpay, dim3(gcg), dim3(kBlock), 0, s, n, H.z.p, H.p.p, ctl, 1);
    for (;;) {
      for (int it = 0; it < chunk; ++it) {
        AMG_DISPATCH_G(L0.gA, hipLaunchKernelGGL((k_spmv_dot<G>), dim3(stream_grid(n, G)), dim3(kBlock), 0, s, n,
                                                 L0.rp.p, L0.ci.p, L0.v.p, H.p.p, H.q.p, ctl, part));
        hipLaunchKernelGGL(k_cg_update, dim3(gcg), dim3(kBlock), 0, s, n, d_x, H.r.p, H.p.p, H.q.p, ctl, part);
        CycleArgs a{H.r.p, H.z.p, H.q.p, ctl, part, flexible ? 2 : 1, 0};
        vcycle(H, a, s);
        hipLaunchKernelGGL(k_xpay, dim3(gcg), dim3(kBlock), 0, s, n, H.z.p, H.p.p, ctl, 0);
      }
      AMG_HIP(hipGetLastError());
      read_ctl(H, s);
      if (H.h_ctl->done) break;
    }
    const int state = H.h_ctl->state;
    if (state == 3) {  // b = 0
      break;
    }
    if (state < 0) {
      st = AMG_ERR_BREAKDOWN;
      break;
    }
    // true residual r = b - A x
    AMG_DISPATCH_G(L0.gA, hipLaunchKernelGGL((k_true_resid<G>), dim3(stream_grid(n, G)), dim3(kBlock), 0, s, n,
                                             L0.rp.p, L0.ci.p, L0.v.p, d_b, d_x, H.r.p, ctl, part));
    read_ctl(H, s);
    const Ctl& c = *H.h_ctl;
    if (c.trr <= c.thresh) {
      st = AMG_OK;
      break;
    }
    if (state == 1 && restarts < 5 && c.iters < c.maxiter) {
      ++restarts;
      hipLaunchKernelGGL(k_ctl_restart, dim3(1), dim3(1), 0, s, ctl);
      continue;
    }
    st = AMG_NOT_CONVERGED;
    break;
  }
  const Ctl& c = *H.h_ctl;
  if (info) {
    info->iters = c.iters;
    info->status = st;
    info->restarts = restarts;
    info->rel_resid = c.state == 3 ? 0.0 : (c.bb > 0 ? std::sqrt(c.trr / c.bb) : 0.0);
    if (st == AMG_ERR_BREAKDOWN) info->rel_resid = NAN;
    info->cache_event = H.cache_event;
    info->setup_ms = H.setup_ms;
    info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

}  // namespace amg
