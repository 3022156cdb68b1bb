// Solve phase: preconditioned CG with one smoothed-aggregation V-cycle per
// iteration, all on the GPU.  Every sweep over a CSR matrix is HBM-bound and
// uses one of two kernel templates around a small operator (per-entry
// product, per-row epilogue):
//   - k_stream (rows of moderate length): a workgroup stages the row
//     pointers of a block of rows in LDS, loads all of the block's nonzeros
//     at once (up to kStreamCap/kBlock independent loads per thread, coalesced
//     column/value streams), stores the products in LDS and sums each row
//     there; with one lane per row the sum is the sequential fold in stored
//     order;
//   - k_vec (fallback for rows too long to stage): a group of G lanes per
//     row (G = 64 is a wavefront per row).
// Workgroups are renumbered so that each XCD (round-robin dispatch over the
// 8 XCDs) owns one contiguous range of rows, which keeps neighbour gathers
// in that XCD's L2.  Dot products are fused into the producing sweep as one
// partial per workgroup (plain stores); a single-workgroup finalize kernel
// folds the partials in a fixed order and forms the CG scalars on the
// device, so there are no float atomics and no device-wide fences.
// Method: PCG from x0 = 0 with recursive-residual stopping, true-residual
// verification and restart; damped-Jacobi/L1 V(nu_pre, nu_post) cycle with
// R = P^T and an exact coarsest solve.  The FP32 cycle keeps CG vectors, dot
// products and updates in FP64 and runs the cycle on FP32 copies (bf16-stored
// P and R optional); the flexible (Polak-Ribiere) beta keeps CG consistent
// with that inexact preconditioner.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>

#include "amg_internal.hpp"

namespace amg {
namespace {

// ------------------------------------------------------------ geometry

// Workgroup index remapped so that XCD k (round-robin dispatch) owns the
// contiguous logical range [k*G/8, (k+1)*G/8) when G is a multiple of 8.
__device__ inline int logical_block() {
  const int g = gridDim.x;
  if ((g & 7) == 0) return (blockIdx.x & 7) * (g >> 3) + (blockIdx.x >> 3);
  return blockIdx.x;
}

// Grid of `blocks` workgroups rounded up to a multiple of 8 (surplus
// workgroups find no rows and exit), so the XCD remap applies.
inline int round8(int64_t g) {
  if (g >= 64) g = (g + 7) / 8 * 8;
  return (int)std::max<int64_t>(g, 1);
}

// ----------------------------------------------------------- operators
// An operator supplies
//   PT prod(k, j)                 product for stored entry k (column j)
//   Row row_in(row)               the row's own operands (loaded by the sweep
//                                 kernels before the row sum is formed, so that
//                                 their latency overlaps the matrix stream)
//   void epi(row, s, in, d[])     consumes the row sum s; d[] collects dot partials
//   static constexpr int NRED     number of dot products reduced

// Direction update fused with the product: p' = z + beta p (p' = z on the
// first iteration of a (re)start) and q' = A p', <p', q'>.  q' is formed as
// A z + beta q (the same vector in exact arithmetic, since q = A p), so the
// sweep gathers z only; p and q are read at the row itself (q is updated in
// place by the row's own thread).  p' goes to the second direction buffer.
// beta is read from the device control block.
struct OpSpmvXpayDev {
  using PT = double;
  static constexpr int NRED = 1;
  const double* v;
  const double* z;
  const double* p;
  double* pn;
  double* q;
  const Ctl* ctl;
  int first;
  struct Row {
    double pr, qo, beta;
  };
  __device__ PT prod_v(double a, int j) const { return a * z[j]; }
  __device__ PT prod(int k, int j) const { return prod_v(v[k], j); }
  __device__ Row row_in(int row) const {
    if (first) return {z[row], 0.0, 0.0};
    const double beta = ctl->beta;
    return {z[row] + beta * p[row], q[row], beta};
  }
  __device__ void epi(int row, PT s, const Row& a, double* d) const {
    pn[row] = a.pr;
    const double qn = first ? s : s + a.beta * a.qo;
    q[row] = qn;
    d[0] += a.pr * qn;
  }
};

// r = b - A x, ||r||^2
struct OpTrueResid {
  using PT = double;
  static constexpr int NRED = 1;
  const double* v;
  const double* x;
  const double* b;
  double* r;
  struct Row {
    double b;
  };
  __device__ PT prod_v(PT a, int j) const { return a * x[j]; }
  __device__ PT prod(int k, int j) const { return prod_v(v[k], j); }
  __device__ Row row_in(int row) const { return {b[row]}; }
  __device__ void epi(int row, PT s, const Row& a, double* d) const {
    const double ri = a.b - s;
    r[row] = ri;
    d[0] += ri * ri;
  }
};

// BiCGSTAB product with its reductions: out = A in, <w, out> and, with
// NRED = 2, <out, out> (v = A y with <r^, v>; t = A z with <s, t>, <t, t>).
template <int N>
struct OpSpmvDots {
  using PT = double;
  static constexpr int NRED = N;
  const double* v;
  const double* in;
  double* out;
  const double* w;
  struct Row {
    double w;
  };
  __device__ PT prod_v(double a, int j) const { return a * in[j]; }
  __device__ PT prod(int k, int j) const { return prod_v(v[k], j); }
  __device__ Row row_in(int row) const { return {w[row]}; }
  __device__ void epi(int row, PT s, const Row& a, double* d) const {
    out[row] = s;
    d[0] += a.w * s;
    if constexpr (N == 2) d[1] += s * s;
  }
};

// Pre-smoothing from zero fused with the residual:
//   x_i = sw_i b_i ;  r_i = b_i - sum_j a_ij (sw_j b_j).
template <class T, class BT>
struct OpPre {
  using PT = T;
  static constexpr int NRED = 0;
  const T* v;
  const T* sw;
  const BT* b;
  T* x;
  T* r;
  struct Row {
    T b, w;
  };
  __device__ PT prod_v(PT a, int j) const { return a * (sw[j] * (T)b[j]); }
  __device__ PT prod(int k, int j) const { return prod_v(v[k], j); }
  __device__ Row row_in(int row) const { return {(T)b[row], sw[row]}; }
  __device__ void epi(int row, PT s, const Row& a, double*) const {
    x[row] = a.w * a.b;
    r[row] = a.b - s;
  }
};

// Residual of the pre-smoothed iterate when x = sw o b was already written
// by the producer of b:  r_i = b_i - sum_j a_ij x_j.
template <class T, class BT>
struct OpResid {
  using PT = T;
  static constexpr int NRED = 0;
  const T* v;
  const BT* b;
  const T* x;
  T* r;
  struct Row {
    T b;
  };
  __device__ PT prod_v(PT a, int j) const { return a * x[j]; }
  __device__ PT prod(int k, int j) const { return prod_v(v[k], j); }
  __device__ Row row_in(int row) const { return {(T)b[row]}; }
  __device__ void epi(int row, PT s, const Row& a, double*) const { r[row] = a.b - s; }
};

// Further Jacobi sweep in residual form, fused with the new residual:
//   x'_i = x_i + sw_i r_i ;  r'_i = b_i - sum_j a_ij (x_j + sw_j r_j).
template <class T, class BT>
struct OpSweep {
  using PT = T;
  static constexpr int NRED = 0;
  const T* v;
  const T* sw;
  const BT* b;
  const T* x;
  const T* r;
  T* x2;
  T* r2;
  struct Row {
    T x, w, r, b;
  };
  __device__ PT prod_v(PT a, int j) const { return a * (x[j] + sw[j] * r[j]); }
  __device__ PT prod(int k, int j) const { return prod_v(v[k], j); }
  __device__ Row row_in(int row) const { return {x[row], sw[row], r[row], (T)b[row]}; }
  __device__ void epi(int row, PT s, const Row& a, double*) const {
    x2[row] = a.x + a.w * a.r;
    r2[row] = a.b - s;
  }
};

// Post-smoothing out_i = x_i + sw_i (b_i - sum_j a_ij x_j); RED >= 1 also
// <b, out>, RED == 2 also <out, q> (level 0 of CG: b = r, out = z).
template <class T, class BT, class OT, int RED>
struct OpPost {
  using PT = T;
  static constexpr int NRED = RED;
  const T* v;
  const T* sw;
  const BT* b;
  const T* x;
  OT* out;
  const double* q;
  struct Row {
    BT b;
    T x, w;
    double q;
  };
  __device__ PT prod_v(PT a, int j) const { return a * x[j]; }
  __device__ PT prod(int k, int j) const { return prod_v(v[k], j); }
  __device__ Row row_in(int row) const {
    Row a{b[row], x[row], sw[row], 0.0};
    if constexpr (RED >= 2) a.q = q[row];
    return a;
  }
  __device__ void epi(int row, PT s, const Row& a, double* d) const {
    const T o = a.x + a.w * ((T)a.b - s);
    const OT oo = (OT)o;
    out[row] = oo;
    if constexpr (RED >= 1) d[0] += (double)a.b * (double)oo;
    if constexpr (RED >= 2) d[1] += (double)oo * a.q;
  }
};

// y = R x (restriction); R values of type RT (double, float or bf16 bits).
// Also writes the coarse level's pre-smoothed iterate xc = swc o y.
template <class RT, class T>
struct OpRestrict {
  using PT = T;
  static constexpr int NRED = 0;
  const RT* v;
  const T* x;
  T* y;
  const T* swc;
  T* xc;
  struct Row {
    T w;
  };
  __device__ PT prod_v(RT a, int j) const { return (T)ValCvt<RT>::f(a) * x[j]; }
  __device__ PT prod(int k, int j) const { return prod_v(v[k], j); }
  __device__ Row row_in(int row) const { return {xc ? swc[row] : (T)0}; }
  __device__ void epi(int row, PT s, const Row& a, double*) const {
    y[row] = s;
    if (xc) xc[row] = a.w * s;
  }
};

// x += P xc (prolongation and coarse-grid correction).
template <class RT, class T>
struct OpProlong {
  using PT = T;
  static constexpr int NRED = 0;
  const RT* v;
  const T* xc;
  T* x;
  struct Row {
    T x;
  };
  __device__ PT prod_v(RT a, int j) const { return (T)ValCvt<RT>::f(a) * xc[j]; }
  __device__ PT prod(int k, int j) const { return prod_v(v[k], j); }
  __device__ Row row_in(int row) const { return {x[row]}; }
  __device__ void epi(int row, PT s, const Row& a, double*) const { x[row] = a.x + s; }
};

template <int NRED>
__device__ inline void publish_partials(double (&d)[NRED > 0 ? NRED : 1], double* partials) {
  if constexpr (NRED > 0) {
    block_sum<NRED>(d);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int m = 0; m < NRED; ++m) partials[m * gridDim.x + blockIdx.x] = d[m];
    }
  }
}

// ------------------------------------------------------------ CSR sweeps

// U: staged entries per thread (the block's staging buffer holds kBlock*U
// entries; the shape sizes it to the matrix's largest row block, so that few
// of the unconditional loads are clamped duplicates).
template <int G3, int U, bool NT, class Op>
__global__ void __launch_bounds__(kBlock) k_stream(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                   Op op, const Ctl* __restrict__ ctl,
                                                   double* __restrict__ partials) {
  if ((ctl && ctl->done) || n <= 0) return;
  constexpr int RB = kBlock / G3;
  using PT = typename Op::PT;
  __shared__ int s_rp[RB + 1];
  __shared__ PT s_p[kBlock * U];
  const int r0 = logical_block() * RB;
  for (int t = threadIdx.x; t <= RB; t += kBlock) s_rp[t] = rp[min(r0 + t, n)];
  const int lr = threadIdx.x / G3, lane = threadIdx.x & (G3 - 1);
  const int row = r0 + lr;
  const typename Op::Row in = op.row_in(min(row, n - 1));
  __syncthreads();
  const int k0 = s_rp[0];
  const int nk = s_rp[RB] - k0;
  if (nk > 0) {
    // Loads are unconditional (indices clamped to the block's last entry) so
    // that all of them are in flight at once; only the LDS stores are masked.
    int col[U];
#pragma unroll
    for (int u = 0; u < U; ++u) col[u] = stream_load<NT>(ci + k0 + min((int)threadIdx.x + u * kBlock, nk - 1));
    PT pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      pv[u] = op.prod_v(stream_load<NT>(op.v + k0 + min((int)threadIdx.x + u * kBlock, nk - 1)), col[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = threadIdx.x + u * kBlock;
      if (j < nk) s_p[j] = pv[u];
    }
  }
  __syncthreads();
  PT s = 0;
  if (row < n) {
    const int e = s_rp[lr + 1] - k0;
    for (int k = s_rp[lr] - k0 + lane; k < e; k += G3) s += s_p[k];
  }
  s = group_sum<G3>(s);
  double d[Op::NRED > 0 ? Op::NRED : 1] = {};
  if (row < n && group_leader<G3>()) op.epi(row, s, in, d);
  publish_partials<Op::NRED>(d, partials);
}

template <int G, class Op>
__global__ void __launch_bounds__(kBlock) k_vec(int n, const int* __restrict__ rp, const int* __restrict__ ci, Op op,
                                                const Ctl* __restrict__ ctl, double* __restrict__ partials) {
  if ((ctl && ctl->done) || n <= 0) return;
  using PT = typename Op::PT;
  constexpr int RB = kBlock / G;
  const int lr = threadIdx.x / G, lane = threadIdx.x & (G - 1);
  double d[Op::NRED > 0 ? Op::NRED : 1] = {};
  constexpr int U = 4;
  for (int r0 = logical_block() * RB; r0 < n; r0 += gridDim.x * RB) {
    const int row = r0 + lr;
    const typename Op::Row in = op.row_in(min(row, n - 1));
    PT s = 0;
    if (row < n) {
      const int kb = rp[row], ke = rp[row + 1];
      // U entries per lane in flight (clamped indices, unconditional loads);
      // each lane still adds its entries k, k+G, k+2G, ... in that order
      for (int k = kb + lane; k < ke; k += U * G) {
        int cc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cc[u] = ci[min(k + u * G, ke - 1)];
        PT pv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) pv[u] = op.prod(min(k + u * G, ke - 1), cc[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) s = k + u * G < ke ? s + pv[u] : s;
      }
    }
    s = group_sum<G>(s);
    if (row < n && group_leader<G>()) op.epi(row, s, in, d);
  }
  publish_partials<Op::NRED>(d, partials);
}

// Sliced sweep: thread per row, the wave's 64 rows form one slice whose
// entries are stored column-major, so entry j of all 64 rows is one
// coalesced load.  The slice width is uniform across the wave; padding
// entries (column -1) are masked out of the sum.  Each row sums its entries
// in stored order (the same fold as a one-lane CSR sweep).
template <bool NT, class Op>
__global__ void __launch_bounds__(kBlock) k_sell(int n, const int* __restrict__ soff, const int* __restrict__ sci,
                                                 Op op, const Ctl* __restrict__ ctl, double* __restrict__ partials) {
  if ((ctl && ctl->done) || n <= 0) return;
  using PT = typename Op::PT;
  const int row = logical_block() * kBlock + threadIdx.x;
  const int rc = min(row, n - 1);
  const typename Op::Row in = op.row_in(rc);
  // the wave's 64 rows are one slice: its offsets are scalar loads, which
  // leave the vector loads of the row operands in flight
  const int sl = __builtin_amdgcn_readfirstlane(rc >> 6), lane = rc & 63;
  const int off = soff[sl];
  const int w = (soff[sl + 1] - off) >> 6;
  int col[kSellMaxW];
  typename std::remove_const<typename std::remove_pointer<decltype(op.v)>::type>::type val[kSellMaxW];
#pragma unroll
  for (int j = 0; j < kSellMaxW; ++j) {
    const int p = off + min(j, w - 1) * 64 + lane;
    col[j] = stream_load<NT>(sci + p);
    val[j] = stream_load<NT>(op.v + p);
  }
  PT pv[kSellMaxW];
#pragma unroll
  for (int j = 0; j < kSellMaxW; ++j) pv[j] = op.prod_v(val[j], col[j] < 0 ? rc : col[j]);
  PT s = 0;
#pragma unroll
  for (int j = 0; j < kSellMaxW; ++j) s = j < w && col[j] >= 0 ? s + pv[j] : s;
  double d[Op::NRED > 0 ? Op::NRED : 1] = {};
  if (row < n) op.epi(row, s, in, d);
  publish_partials<Op::NRED>(d, partials);
}

// Sliced sweep, offset form: slot j of the wave's slice holds offset
// slots[j].x for every row whose mask bit is set; the slot records are
// wave-uniform (scalar loads), so the only per-entry stream is the values.
// Each row adds its present entries in ascending offset (= column) order.
template <bool NT, class Op>
__global__ void __launch_bounds__(kBlock) k_sello(int n, const int* __restrict__ soff, const int4* __restrict__ slots,
                                                  Op op, const Ctl* __restrict__ ctl, double* __restrict__ partials) {
  if ((ctl && ctl->done) || n <= 0) return;
  using PT = typename Op::PT;
  const int row = logical_block() * kBlock + threadIdx.x;
  const int rc = min(row, n - 1);
  const typename Op::Row in = op.row_in(rc);
  const int sl = __builtin_amdgcn_readfirstlane(rc >> 6), lane = rc & 63;
  const int off = soff[sl];
  const int w = (soff[sl + 1] - off) >> 6;
  const int sb = off >> 6;
  typename std::remove_const<typename std::remove_pointer<decltype(op.v)>::type>::type val[kSellMaxW];
#pragma unroll
  for (int j = 0; j < kSellMaxW; ++j) val[j] = stream_load<NT>(op.v + off + min(j, w - 1) * 64 + lane);
  // the slice's kSellMaxW records as one block (the array is padded so the
  // last slice's block stays in bounds)
  int4 rec[kSellMaxW];
#pragma unroll
  for (int j = 0; j < kSellMaxW; ++j) rec[j] = slots[sb + j];
  int col[kSellMaxW];
  bool has[kSellMaxW];
#pragma unroll
  for (int j = 0; j < kSellMaxW; ++j) {
    const unsigned bits = lane < 32 ? (unsigned)rec[j].z : (unsigned)rec[j].w;
    has[j] = j < w && ((bits >> (lane & 31)) & 1u);
    col[j] = has[j] ? rc + rec[j].x : rc;
  }
  PT pv[kSellMaxW];
#pragma unroll
  for (int j = 0; j < kSellMaxW; ++j) pv[j] = op.prod_v(val[j], col[j]);
  PT s = 0;
#pragma unroll
  for (int j = 0; j < kSellMaxW; ++j) s = has[j] ? s + pv[j] : s;
  double d[Op::NRED > 0 ? Op::NRED : 1] = {};
  if (row < n) op.epi(row, s, in, d);
  publish_partials<Op::NRED>(d, partials);
}

#define AMG_DISPATCH_G(g, ...)                             \
  switch (g) {                                             \
    case 1: { constexpr int G = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int G = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int G = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int G = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int G = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int G = 32; __VA_ARGS__; } break; \
    default: { constexpr int G = 64; __VA_ARGS__; } break; \
  }

template <bool NT, class Op>
void sweep_form(const Shape& sh, int n, const int* rp, const int* ci, const Op& op, const Ctl* ctl,
                double* partials, hipStream_t s) {
  if (sh.stream == 3) {
    hipLaunchKernelGGL((k_sello<NT, Op>), dim3(sh.grid), dim3(kBlock), 0, s, n, rp, reinterpret_cast<const int4*>(ci),
                       op, ctl, partials);
  } else if (sh.stream == 2) {
    hipLaunchKernelGGL((k_sell<NT, Op>), dim3(sh.grid), dim3(kBlock), 0, s, n, rp, ci, op, ctl, partials);
  } else if (sh.stream) {
    switch (sh.u) {
      case 4:
        AMG_DISPATCH_G(sh.g, hipLaunchKernelGGL((k_stream<G, 4, NT, Op>), dim3(sh.grid), dim3(kBlock), 0, s, n, rp,
                                                ci, op, ctl, partials));
        break;
      case 8:
        AMG_DISPATCH_G(sh.g, hipLaunchKernelGGL((k_stream<G, 8, NT, Op>), dim3(sh.grid), dim3(kBlock), 0, s, n, rp,
                                                ci, op, ctl, partials));
        break;
      default:
        AMG_DISPATCH_G(sh.g, hipLaunchKernelGGL((k_stream<G, 12, NT, Op>), dim3(sh.grid), dim3(kBlock), 0, s, n,
                                                rp, ci, op, ctl, partials));
        break;
    }
  } else {
    AMG_DISPATCH_G(sh.g, hipLaunchKernelGGL((k_vec<G, Op>), dim3(sh.grid), dim3(kBlock), 0, s, n, rp, ci, op, ctl,
                                            partials));
  }
}

// One sweep over a CSR matrix with operator `op`; returns the grid size
// (= number of partials written per reduced value).
template <class Op>
int sweep(const Shape& sh, int n, const int* rp, const int* ci, const Op& op, const Ctl* ctl, double* partials,
          hipStream_t s) {
  if (sh.nt) sweep_form<true>(sh, n, rp, ci, op, ctl, partials, s);
  else sweep_form<false>(sh, n, rp, ci, op, ctl, partials, s);
  return sh.grid;
}

// ------------------------------------------------------- dense coarse solve

// x = A_L^-1 b with the explicit (symmetric) inverse: thread i reads
// column i = row i, coalesced across threads.
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

// ------------------------------------------------------- BLAS1 (FP64)

inline int vec_grid(int n) { return round8(((int64_t)n + kBlock * kVecPer - 1) / (kBlock * kVecPer)); }

// Element range of this workgroup: kBlock*kVecPer consecutive entries.
__device__ inline int vec_base() { return logical_block() * (kBlock * kVecPer); }

// r = b, x = 0, partial <b, b>.
__global__ void __launch_bounds__(kBlock) k_cg_init(int n, const double* __restrict__ b, double* __restrict__ r,
                                                    double* __restrict__ x, double* __restrict__ partials) {
  const int base = vec_base();
  double bv[kVecPer];
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    bv[u] = i < n ? b[i] : 0.0;
  }
  double d[1] = {0.0};
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    if (i < n) {
      r[i] = bv[u];
      x[i] = 0.0;
      d[0] += bv[u] * bv[u];
    }
  }
  publish_partials<1>(d, partials);
}

// x += alpha p ; r -= alpha q ; partial <r, r>; also the level-0
// pre-smoothed iterate x0 = sw o r of the next V-cycle (cycle precision T).
template <class T>
__global__ void __launch_bounds__(kBlock) k_cg_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                      const double* __restrict__ p, const double* __restrict__ q,
                                                      const T* __restrict__ sw, T* __restrict__ x0,
                                                      const Ctl* __restrict__ ctl, double* __restrict__ partials) {
  if (ctl->done) return;
  const double alpha = ctl->alpha;
  const int base = vec_base();
  double xv[kVecPer], rv[kVecPer], pv[kVecPer], qv[kVecPer];
  T wv[kVecPer];
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    const bool ok = i < n;
    xv[u] = ok ? x[i] : 0.0;
    rv[u] = ok ? r[i] : 0.0;
    pv[u] = ok ? p[i] : 0.0;
    qv[u] = ok ? q[i] : 0.0;
    wv[u] = ok ? sw[i] : (T)0;
  }
  double d[1] = {0.0};
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    if (i < n) {
      x[i] = xv[u] + alpha * pv[u];
      const double ri = rv[u] - alpha * qv[u];
      r[i] = ri;
      x0[i] = wv[u] * (T)ri;
      d[0] += ri * ri;
    }
  }
  publish_partials<1>(d, partials);
}

// z = r (the identity preconditioner of plain CG).
__global__ void __launch_bounds__(kBlock) k_copy_z(int n, const double* __restrict__ r, double* __restrict__ z,
                                                   const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  const int base = vec_base();
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    if (i < n) z[i] = r[i];
  }
}

// x0 = sw o r (first V-cycle of a solve or restart).
template <class T>
__global__ void __launch_bounds__(kBlock) k_sw_mul(int n, const T* __restrict__ sw, const double* __restrict__ r,
                                                   T* __restrict__ x0, const Ctl* __restrict__ ctl) {
  if (ctl && ctl->done) return;
  const int base = vec_base();
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    if (i < n) x0[i] = sw[i] * (T)r[i];
  }
}

// <r, z> and <z, q> partials after a single-level (direct) preconditioner.
__global__ void __launch_bounds__(kBlock) k_dots_rz(int n, const double* __restrict__ r, const double* __restrict__ z,
                                                    const double* __restrict__ q, const Ctl* __restrict__ ctl,
                                                    double* __restrict__ partials) {
  if (ctl->done) return;
  const int base = vec_base();
  double d[2] = {0.0, 0.0};
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    if (i < n) {
      d[0] += r[i] * z[i];
      d[1] += z[i] * q[i];
    }
  }
  publish_partials<2>(d, partials);
}

// grad_val[k] = -(lambda[row k] * x[col k]): a group of 8 lanes per row.
__global__ void __launch_bounds__(kBlock) k_pattern_grad(int n, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, const double* __restrict__ lam,
                                                         const double* __restrict__ x, double* __restrict__ g) {
  constexpr int G = 8;
  const int row = blockIdx.x * (kBlock / G) + threadIdx.x / G;
  const int lane = threadIdx.x & (G - 1);
  if (row >= n) return;
  const double li = lam[row];
  for (int k = rp[row] + lane; k < rp[row + 1]; k += G) g[k] = -(li * x[ci[k]]);
}

// ------------------------------------------------------- BiCGSTAB vectors

// r = b, r^ = b, x = 0, partial <b, b>.
__global__ void __launch_bounds__(kBlock) k_bi_init(int n, const double* __restrict__ b, double* __restrict__ r,
                                                    double* __restrict__ rh, double* __restrict__ x,
                                                    double* __restrict__ partials) {
  const int base = vec_base();
  double d[1] = {0.0};
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    if (i < n) {
      const double bi = b[i];
      r[i] = bi;
      rh[i] = bi;
      x[i] = 0.0;
      d[0] += bi * bi;
    }
  }
  publish_partials<1>(d, partials);
}

// p = r on the first iteration of a (re)start, else p = r + beta (p - omega v);
// with x0, also the next V-cycle's level-0 pre-smoothed iterate x0 = sw o p
// (cycle precision T), so that its first sweep only forms the residual.
template <class T>
__global__ void __launch_bounds__(kBlock) k_bi_dir(int n, const double* __restrict__ r,
                                                   const double* __restrict__ v, double* __restrict__ p,
                                                   const T* __restrict__ sw, T* __restrict__ x0,
                                                   const Ctl* __restrict__ ctl, int first) {
  if (ctl->done) return;
  const double beta = ctl->beta, omega = ctl->omega;
  const int base = vec_base();
  double rv[kVecPer], vv[kVecPer], pv[kVecPer];
  T wv[kVecPer];
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = min(base + (int)threadIdx.x + u * kBlock, n - 1);
    rv[u] = r[i];
    vv[u] = v[i];
    pv[u] = p[i];
    wv[u] = x0 ? sw[i] : (T)0;
  }
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    if (i < n) {
      const double pi = first ? rv[u] : rv[u] + beta * (pv[u] - omega * vv[u]);
      p[i] = pi;
      if (x0) x0[i] = wv[u] * (T)pi;
    }
  }
}

// x += alpha y ; s = r - alpha v ; partial <s, s>; with x0 also x0 = sw o s.
template <class T>
__global__ void __launch_bounds__(kBlock) k_bi_half(int n, double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ r, const double* __restrict__ v,
                                                    double* __restrict__ sv, const T* __restrict__ sw,
                                                    T* __restrict__ x0, const Ctl* __restrict__ ctl,
                                                    double* __restrict__ partials) {
  if (ctl->done) return;
  const double alpha = ctl->alpha;
  const int base = vec_base();
  double xv[kVecPer], yv[kVecPer], rv[kVecPer], vv[kVecPer];
  T wv[kVecPer];
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = min(base + (int)threadIdx.x + u * kBlock, n - 1);
    xv[u] = x[i];
    yv[u] = y[i];
    rv[u] = r[i];
    vv[u] = v[i];
    wv[u] = x0 ? sw[i] : (T)0;
  }
  double d[1] = {0.0};
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    if (i < n) {
      x[i] = xv[u] + alpha * yv[u];
      const double si = rv[u] - alpha * vv[u];
      sv[i] = si;
      if (x0) x0[i] = wv[u] * (T)si;
      d[0] += si * si;
    }
  }
  publish_partials<1>(d, partials);
}

// x += omega z ; r = s - omega t ; partials <r, r>, <r^, r>.
__global__ void __launch_bounds__(kBlock) k_bi_full(int n, double* __restrict__ x, const double* __restrict__ z,
                                                    const double* __restrict__ sv, const double* __restrict__ t,
                                                    const double* __restrict__ rh, double* __restrict__ r,
                                                    const Ctl* __restrict__ ctl, double* __restrict__ partials) {
  if (ctl->done) return;
  const double omega = ctl->omega;
  const int base = vec_base();
  double xv[kVecPer], zv[kVecPer], sl[kVecPer], tv[kVecPer], hv[kVecPer];
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = min(base + (int)threadIdx.x + u * kBlock, n - 1);
    xv[u] = x[i];
    zv[u] = z[i];
    sl[u] = sv[i];
    tv[u] = t[i];
    hv[u] = rh[i];
  }
  double d[2] = {0.0, 0.0};
#pragma unroll
  for (int u = 0; u < kVecPer; ++u) {
    const int i = base + threadIdx.x + u * kBlock;
    if (i < n) {
      x[i] = xv[u] + omega * zv[u];
      const double ri = sl[u] - omega * tv[u];
      r[i] = ri;
      d[0] += ri * ri;
      d[1] += hv[u] * ri;
    }
  }
  publish_partials<2>(d, partials);
}

// ------------------------------------------------------- finalize kernels

// Fixed-order fold of gridDim-sized partial arrays by one workgroup; the
// totals are valid in thread 0.
template <int NV>
__device__ inline void fold_partials(const double* __restrict__ partials, int np, double (&tot)[NV]) {
  __shared__ double red[NV][kFinBlock / 64];
  constexpr int UF = 8;
  double acc[NV];
#pragma unroll
  for (int m = 0; m < NV; ++m) {
    double s = 0.0;
    for (int b0 = 0; b0 < np; b0 += kFinBlock * UF) {
      double t[UF];
#pragma unroll
      for (int u = 0; u < UF; ++u) {
        const int b = b0 + threadIdx.x + u * kFinBlock;
        t[u] = b < np ? partials[m * np + b] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UF; ++u) s += t[u];
    }
    acc[m] = wave_sum(s);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int m = 0; m < NV; ++m) red[m][w] = acc[m];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      double s = red[m][0];
      for (int k = 1; k < kFinBlock / 64; ++k) s += red[m][k];
      tot[m] = s;
    }
  }
}

__global__ void __launch_bounds__(kFinBlock) k_fin_init(Ctl* ctl, const double* __restrict__ partials, int np,
                                                        double tol, int maxiter, int flexible) {
  double t[1];
  fold_partials<1>(partials, np, t);
  if (threadIdx.x != 0) return;
  const double bb = t[0];
  ctl->bb = bb;
  ctl->thresh = (tol * tol) * bb;
  ctl->iters = 0;
  ctl->maxiter = maxiter;
  ctl->flexible = flexible;
  ctl->state = 0;
  ctl->done = 0;
  ctl->trr = 0.0;
  ctl->rr = bb;
  if (bb == 0.0) {
    ctl->state = 3;  // zero right-hand side: x = 0
    ctl->done = 1;
  } else if (!(bb == bb)) {
    ctl->state = -1;
    ctl->done = 1;
  } else if (maxiter <= 0) {
    ctl->state = 2;
    ctl->done = 1;
  }
}

__global__ void __launch_bounds__(kFinBlock) k_fin_alpha(Ctl* ctl, const double* __restrict__ partials, int np) {
  if (ctl->done) return;
  double t[1];
  fold_partials<1>(partials, np, t);
  if (threadIdx.x != 0) return;
  const double pq = t[0];
  ctl->pq = pq;
  if (!(pq > 0.0)) {
    ctl->state = -1;
    ctl->done = 1;
  } else {
    ctl->alpha = ctl->rz / pq;
  }
}

__global__ void __launch_bounds__(kFinBlock) k_fin_update(Ctl* ctl, const double* __restrict__ partials, int np) {
  if (ctl->done) return;
  double t[1];
  fold_partials<1>(partials, np, t);
  if (threadIdx.x != 0) return;
  const double rr = t[0];
  ctl->rr = rr;
  ctl->iters += 1;
  if (rr <= ctl->thresh) {
    ctl->state = 1;
    ctl->done = 1;
  } else if (!(rr == rr)) {
    ctl->state = -1;
    ctl->done = 1;
  } else if (ctl->iters >= ctl->maxiter) {
    ctl->state = 2;
    ctl->done = 1;
  }
}

// beta: standard <r,z>/<r_old,z_old>; flexible (Polak-Ribiere)
// <z, r - r_old>/<z_old, r_old> = -<z, q>/<p, q>.
template <int NV>
__global__ void __launch_bounds__(kFinBlock) k_fin_beta(Ctl* ctl, const double* __restrict__ partials, int np,
                                                        int first) {
  if (ctl->done) return;
  double t[NV];
  fold_partials<NV>(partials, np, t);
  if (threadIdx.x != 0) return;
  const double rzn = t[0];
  const double zq = NV > 1 ? t[NV - 1] : 0.0;
  if (first) {
    ctl->beta = 0.0;
  } else if (ctl->flexible) {
    ctl->beta = -zq / ctl->pq;
  } else {
    ctl->beta = rzn / ctl->rz;
  }
  ctl->rz = rzn;
  ctl->rzn = rzn;
  ctl->zq = zq;
  if (!(rzn > 0.0)) {
    ctl->state = -1;
    ctl->done = 1;
  }
}

__global__ void __launch_bounds__(kFinBlock) k_fin_trr(Ctl* ctl, const double* __restrict__ partials, int np) {
  double t[1];
  fold_partials<1>(partials, np, t);
  if (threadIdx.x == 0) ctl->trr = t[0];
}

// BiCGSTAB scalars.  rho = <r^, r> (= ||b||^2 at the start, r^ = r = b).
__global__ void __launch_bounds__(kFinBlock) k_bfin_init(Ctl* ctl, const double* __restrict__ partials, int np,
                                                         double tol, int maxiter) {
  double t[1];
  fold_partials<1>(partials, np, t);
  if (threadIdx.x != 0) return;
  const double bb = t[0];
  ctl->bb = bb;
  ctl->thresh = (tol * tol) * bb;
  ctl->iters = 0;
  ctl->maxiter = maxiter;
  ctl->flexible = 0;
  ctl->state = 0;
  ctl->done = 0;
  ctl->trr = 0.0;
  ctl->rr = bb;
  ctl->rho = bb;
  ctl->alpha = 1.0;
  ctl->omega = 1.0;
  ctl->beta = 0.0;
  if (bb == 0.0) {
    ctl->state = 3;
    ctl->done = 1;
  } else if (!(bb == bb)) {
    ctl->state = -1;
    ctl->done = 1;
  } else if (maxiter <= 0) {
    ctl->state = 2;
    ctl->done = 1;
  }
}

// alpha = rho / <r^, v>
__global__ void __launch_bounds__(kFinBlock) k_bfin_alpha(Ctl* ctl, const double* __restrict__ partials, int np) {
  if (ctl->done) return;
  double t[1];
  fold_partials<1>(partials, np, t);
  if (threadIdx.x != 0) return;
  const double rv = t[0];
  if (!(rv != 0.0) || !(rv == rv)) {
    ctl->state = -1;
    ctl->done = 1;
  } else {
    ctl->alpha = ctl->rho / rv;
  }
}

// ||s||^2: the iteration is counted here; a small s ends the solve with
// x = x + alpha y (already written).
__global__ void __launch_bounds__(kFinBlock) k_bfin_half(Ctl* ctl, const double* __restrict__ partials, int np) {
  if (ctl->done) return;
  double t[1];
  fold_partials<1>(partials, np, t);
  if (threadIdx.x != 0) return;
  const double ss = t[0];
  ctl->rr = ss;
  ctl->iters += 1;
  if (ss <= ctl->thresh) {
    ctl->state = 1;
    ctl->done = 1;
  } else if (!(ss == ss)) {
    ctl->state = -1;
    ctl->done = 1;
  }
}

// omega = <t, s> / <t, t>
__global__ void __launch_bounds__(kFinBlock) k_bfin_omega(Ctl* ctl, const double* __restrict__ partials, int np) {
  if (ctl->done) return;
  double t[2];
  fold_partials<2>(partials, np, t);
  if (threadIdx.x != 0) return;
  const double ts = t[0], tt = t[1];
  const double om = ts / tt;
  if (!(tt > 0.0) || !(om != 0.0) || !(om == om)) {
    ctl->state = -1;
    ctl->done = 1;
  } else {
    ctl->omega = om;
  }
}

// ||r||^2 and the next rho = <r^, r>, beta = (rho / rho_old) (alpha / omega).
__global__ void __launch_bounds__(kFinBlock) k_bfin_full(Ctl* ctl, const double* __restrict__ partials, int np) {
  if (ctl->done) return;
  double t[2];
  fold_partials<2>(partials, np, t);
  if (threadIdx.x != 0) return;
  const double rr = t[0], rho = t[1];
  ctl->rr = rr;
  if (rr <= ctl->thresh) {
    ctl->state = 1;
    ctl->done = 1;
  } else if (!(rr == rr)) {
    ctl->state = -1;
    ctl->done = 1;
  } else if (ctl->iters >= ctl->maxiter) {
    ctl->state = 2;
    ctl->done = 1;
  } else if (!(rho != 0.0) || !(rho == rho)) {
    ctl->state = -1;
    ctl->done = 1;
  } else {
    ctl->beta = (rho / ctl->rho) * (ctl->alpha / ctl->omega);
    ctl->rho = rho;
  }
}

// Restart from the true residual r = b - A x (||r||^2 in trr): r^ = r is
// copied separately; rho = ||r||^2.
__global__ void k_bi_restart(Ctl* ctl) {
  ctl->done = 0;
  ctl->state = 0;
  ctl->rho = ctl->trr;
}

__global__ void k_ctl_restart(Ctl* ctl) {
  ctl->done = 0;
  ctl->state = 0;
}

void launch_fin_beta(Ctl* ctl, double* partials, int np, int first, int nv, hipStream_t s) {
  if (nv == 2) hipLaunchKernelGGL(k_fin_beta<2>, dim3(1), dim3(kFinBlock), 0, s, ctl, partials, np, first);
  else hipLaunchKernelGGL(k_fin_beta<1>, dim3(1), dim3(kFinBlock), 0, s, ctl, partials, np, first);
}

// ------------------------------------------------------------ V-cycle

// Copies the done flag (0 when there is none) into the instrument record.
__global__ void k_snap_done(const Ctl* ctl, int* dst) {
  if (threadIdx.x == 0) dst[0] = ctl ? ctl->done : 0;
}

// Records an event pair around a launch when (kernel, level) is instrumented,
// and, before the pair, the solve's done flag: a launch that starts with the
// flag set returns at once and is left out of the statistics.
struct InstScope {
  Hierarchy& H;
  hipStream_t s;
  bool on;
  InstScope(Hierarchy& h, int kid, int level, hipStream_t st, const Ctl* ctl) : H(h), s(st) {
    on = H.inst.kernel == kid && (H.inst.level == level || H.inst.level < 0) &&
         2 * (H.inst.used + 1) <= (int)H.inst.ev.size();
    if (on) {
      hipLaunchKernelGGL(k_snap_done, dim3(1), dim3(64), 0, s, ctl, H.inst.was_done.p + H.inst.used);
      AMG_HIP(hipEventRecord(H.inst.ev[2 * H.inst.used], s));
    }
  }
  ~InstScope() {
    if (on) {
      (void)hipEventRecord(H.inst.ev[2 * H.inst.used + 1], s);
      ++H.inst.used;
    }
  }
};

struct CycleArgs {
  const double* r0;   // level-0 right-hand side (CG residual), FP64
  double* z0;         // level-0 result, FP64
  const double* q;    // CG q (flexible reduction), may be null
  Ctl* ctl;           // null: no early exit, no reductions
  double* partials;
  int red;            // 0 none, 1 <r,z>, 2 <r,z> and <z,q>
  int first;
  int x0_ready;       // level-0 x = sw o r0 already written
};

template <class T>
struct Bufs;

template <>
struct Bufs<double> {
  static double* x(Level& L) { return L.x64.p; }
  static double* b(Level& L) { return L.b64.p; }
  static double* r(Level& L) { return L.r64.p; }
  static double* xs(Level& L) { return L.xs64.p; }
  static double* rs(Level& L) { return L.rs64.p; }
  static const double* v(Level& L) { return L.av(); }
  static const double* sw(Level& L) { return L.sw.p; }
  static const double* inv(Coarse& C) { return C.inv.p; }
};
template <>
struct Bufs<float> {
  static float* x(Level& L) { return L.x32.p; }
  static float* b(Level& L) { return L.b32.p; }
  static float* r(Level& L) { return L.r32.p; }
  static float* xs(Level& L) { return L.xs32.p; }
  static float* rs(Level& L) { return L.rs32.p; }
  static const float* v(Level& L) { return L.av32(); }
  static const float* sw(Level& L) { return L.sw32.p; }
  static const float* inv(Coarse& C) { return C.inv32.p; }
};

template <class T>
void launch_restrict(Hierarchy& H, Level& L, const T* r, T* bc, const T* swc, T* xc, const Ctl* ctl, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    sweep(L.shR, L.nagg, L.rrp.p, L.rci.p, OpRestrict<double, T>{L.rv.p, r, bc, swc, xc}, ctl, nullptr, s);
  } else if (H.bf16()) {
    sweep(L.shR, L.nagg, L.rrp.p, L.rci.p, OpRestrict<uint16_t, T>{L.rbf.p, r, bc, swc, xc}, ctl, nullptr, s);
  } else {
    sweep(L.shR, L.nagg, L.rrp.p, L.rci.p, OpRestrict<float, T>{L.rv32.p, r, bc, swc, xc}, ctl, nullptr, s);
  }
}

template <class T>
void launch_prolong(Hierarchy& H, Level& L, const T* xc, T* x, const Ctl* ctl, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    sweep(L.shP, L.n, L.prp.p, L.pci.p, OpProlong<double, T>{L.pv.p, xc, x}, ctl, nullptr, s);
  } else if (H.bf16()) {
    sweep(L.shP, L.n, L.prp.p, L.pci.p, OpProlong<uint16_t, T>{L.pbf.p, xc, x}, ctl, nullptr, s);
  } else {
    sweep(L.shP, L.n, L.prp.p, L.pci.p, OpProlong<float, T>{L.pv32.p, xc, x}, ctl, nullptr, s);
  }
}

// One V-cycle on level-0 rhs a.r0 -> a.z0 (FP64 at the boundary, T inside).
// With a.red, the level-0 post-smoother emits the <r,z> (and <z,q>) partials
// and the finalize kernel forms beta.  Extra smoothing sweeps (nu > 1)
// ping-pong through the level's spare buffers.
template <class T>
void vcycle_impl(Hierarchy& H, const CycleArgs& a, hipStream_t s) {
  const int nl = (int)H.lv.size();
  Coarse& C = H.co;
  Ctl* ctl = a.ctl;
  if (!H.prm.precondition) {
    // plain CG: z = r
    const int n = H.n;
    hipLaunchKernelGGL(k_copy_z, dim3(vec_grid(n)), dim3(kBlock), 0, s, n, a.r0, a.z0, ctl);
    if (a.red) {
      const int g = vec_grid(n);
      hipLaunchKernelGGL(k_dots_rz, dim3(g), dim3(kBlock), 0, s, n, a.r0, a.z0, a.q ? a.q : a.z0, ctl, a.partials);
      launch_fin_beta(ctl, a.partials, g, a.first, 2, s);
    }
    return;
  }
  if (nl == 1) {
    {
      InstScope is(H, KID_COARSE, 0, s, a.ctl);
      hipLaunchKernelGGL((k_coarse<double, double, double>), dim3((C.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                         C.n, C.m, C.inv.p, a.r0, a.z0, ctl);
    }
    if (a.red) {
      const int g = vec_grid(C.n);
      hipLaunchKernelGGL(k_dots_rz, dim3(g), dim3(kBlock), 0, s, C.n, a.r0, a.z0, a.q ? a.q : a.z0, ctl, a.partials);
      launch_fin_beta(ctl, a.partials, g, a.first, 2, s);
    }
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
    {
      // pre-smoothing from zero: x = sw o b was written by the producer of b
      // (CG update on level 0, restriction below), so only r = b - A x remains
      InstScope is(H, KID_PRE, l, s, a.ctl);
      if (l == 0 && !a.x0_ready)
        sweep(L.shA, L.n, L.arp(), L.aci(), OpPre<T, double>{Bufs<T>::v(L), Bufs<T>::sw(L), a.r0, cx[l], cr[l]}, ctl,
              nullptr, s);
      else if (l == 0)
        sweep(L.shA, L.n, L.arp(), L.aci(), OpResid<T, double>{Bufs<T>::v(L), a.r0, cx[l], cr[l]}, ctl, nullptr, s);
      else
        sweep(L.shA, L.n, L.arp(), L.aci(), OpResid<T, T>{Bufs<T>::v(L), Bufs<T>::b(L), cx[l], cr[l]}, ctl, nullptr,
              s);
    }
    for (int k = 1; k < npre; ++k) {
      if (l == 0)
        sweep(L.shA, L.n, L.arp(), L.aci(),
              OpSweep<T, double>{Bufs<T>::v(L), Bufs<T>::sw(L), a.r0, cx[l], cr[l], sx[l], sr[l]}, ctl, nullptr, s);
      else
        sweep(L.shA, L.n, L.arp(), L.aci(),
              OpSweep<T, T>{Bufs<T>::v(L), Bufs<T>::sw(L), Bufs<T>::b(L), cx[l], cr[l], sx[l], sr[l]}, ctl, nullptr,
              s);
      std::swap(cx[l], sx[l]);
      std::swap(cr[l], sr[l]);
    }
    {
      InstScope is(H, KID_RESTRICT, l, s, a.ctl);
      Level& Ln = H.lv[l + 1];
      const bool coarsest = (l + 1 == nl - 1);
      launch_restrict<T>(H, L, cr[l], Bufs<T>::b(Ln), coarsest ? nullptr : Bufs<T>::sw(Ln),
                         coarsest ? nullptr : Bufs<T>::x(Ln), ctl, s);
    }
  }
  T* res;
  {
    Level& Lc = H.lv[nl - 1];
    InstScope is(H, KID_COARSE, nl - 1, s, a.ctl);
    hipLaunchKernelGGL((k_coarse<T, T, T>), dim3((C.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, C.n, C.m,
                       Bufs<T>::inv(C), Bufs<T>::b(Lc), Bufs<T>::x(Lc), ctl);
    res = Bufs<T>::x(Lc);
  }
  for (int l = nl - 2; l >= 0; --l) {
    Level& L = H.lv[l];
    {
      InstScope is(H, KID_PROLONG, l, s, a.ctl);
      launch_prolong<T>(H, L, res, cx[l], ctl, s);
    }
    // free T buffers of this level after restriction: cr[l] and sx[l]
    T* cur = cx[l];
    T* spare[2] = {cr[l], sx[l]};
    for (int k = 0; k < npost; ++k) {
      const bool last = (k == npost - 1);
      const T* vv = Bufs<T>::v(L);
      const T* sw = Bufs<T>::sw(L);
      if (l == 0 && last) {
        int np = 0;
        {
          InstScope is(H, KID_POST, l, s, a.ctl);
          if (a.red == 2)
            np = sweep(L.shA, L.n, L.arp(), L.aci(), OpPost<T, double, double, 2>{vv, sw, a.r0, cur, a.z0, a.q}, ctl,
                       a.partials, s);
          else if (a.red == 1)
            np = sweep(L.shA, L.n, L.arp(), L.aci(), OpPost<T, double, double, 1>{vv, sw, a.r0, cur, a.z0, a.q}, ctl,
                       a.partials, s);
          else
            sweep(L.shA, L.n, L.arp(), L.aci(), OpPost<T, double, double, 0>{vv, sw, a.r0, cur, a.z0, nullptr}, ctl,
                  nullptr, s);
        }
        if (a.red) launch_fin_beta(ctl, a.partials, np, a.first, a.red, s);
      } else {
        T* dst = spare[k & 1];
        InstScope is(H, KID_POST, l, s, a.ctl);
        if (l == 0)
          sweep(L.shA, L.n, L.arp(), L.aci(), OpPost<T, double, T, 0>{vv, sw, a.r0, cur, dst, nullptr}, ctl, nullptr,
                s);
        else
          sweep(L.shA, L.n, L.arp(), L.aci(), OpPost<T, T, T, 0>{vv, sw, Bufs<T>::b(L), cur, dst, nullptr}, ctl,
                nullptr, s);
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

// Launch shape of a sweep over a CSR matrix with `n` rows (host row
// pointers): the most rows per workgroup whose nonzeros fit the staging
// buffer, with enough lanes per row for the in-LDS sums of long rows.
// Staged entries per thread of a CSR-stream launch whose largest row block
// holds mx entries.
int stream_u(int mx) {
  for (int u : {4, 8}) if (mx <= u * kBlock) return u;
  return 12;
}

Shape make_shape(const std::vector<int>& rp, int n) {
  Shape sh;
  const double avg = n > 0 ? (double)(rp[n] - rp[0]) / n : 1.0;
  for (int rb = kBlock; rb >= kBlock / 64; rb >>= 1) {
    const int lanes = kBlock / rb;
    if (lanes < avg / 16.0 && rb > kBlock / 64) continue;
    int mx = 0;
    for (int r0 = 0; r0 < n; r0 += rb) mx = std::max(mx, rp[std::min(r0 + rb, n)] - rp[r0]);
    if (mx <= kStreamCap) {
      sh.stream = 1;
      sh.g = lanes;
      sh.u = stream_u(mx);
      sh.rows_per_block = rb;
      sh.max_block_nnz = mx;
      sh.grid = round8(((int64_t)n + rb - 1) / rb);
      return sh;
    }
  }
  sh.stream = 0;
  sh.g = 64;
  sh.rows_per_block = kBlock / 64;
  sh.grid = round8(std::min<int64_t>(((int64_t)n + sh.rows_per_block - 1) / sh.rows_per_block, kMaxGrid));
  return sh;
}

std::vector<int> host_copy(const DBuf<int>& d, int64_t count) {
  std::vector<int> h((size_t)count);
  if (count) AMG_HIP(hipMemcpy(h.data(), d.p, sizeof(int) * count, hipMemcpyDeviceToHost));
  return h;
}

}  // namespace

// ================================================================ public

namespace {

// ------------------------------------------------------------- autotuner
//
// Candidate launch shapes of one matrix: every stream shape whose row blocks
// fit the staging buffer (1..64 lanes per row in the in-LDS sums) and the
// direct lanes-per-row form with 1..64 lanes.  Each is timed with HIP events on
// the operator that runs on that matrix in the cycle; the fastest wins.
// Choices are cached in memory and, when AMG_TUNE_CACHE names a file, in a
// text file of "key stream lanes rows_per_block" lines, so that later runs
// (and therefore their rounding) repeat the same choice.

std::vector<Shape> candidate_shapes(const std::vector<int>& rp, int n) {
  std::vector<Shape> out;
  for (int rb = kBlock; rb >= kBlock / 64; rb >>= 1) {
    int mx = 0;
    for (int r0 = 0; r0 < n; r0 += rb) mx = std::max(mx, rp[std::min(r0 + rb, n)] - rp[r0]);
    if (mx > kStreamCap) continue;
    Shape sh;
    sh.stream = 1;
    sh.g = kBlock / rb;
    sh.u = stream_u(mx);
    sh.rows_per_block = rb;
    sh.max_block_nnz = mx;
    sh.grid = round8(((int64_t)n + rb - 1) / rb);
    out.push_back(sh);
  }
  for (int g = 1; g <= 64; g <<= 1) {
    Shape sh;
    sh.stream = 0;
    sh.g = g;
    sh.rows_per_block = kBlock / g;
    sh.grid = round8(std::min<int64_t>(((int64_t)n + sh.rows_per_block - 1) / sh.rows_per_block, kMaxGrid));
    out.push_back(sh);
  }
  return out;
}

std::mutex g_tune_mu;
std::map<std::string, Shape> g_tune;
bool g_tune_loaded = false;

void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("AMG_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string key;
  Shape sh;
  while (f >> key >> sh.stream >> sh.g >> sh.rows_per_block) g_tune[key] = sh;
}

void tune_store(const std::string& key, const Shape& sh) {
  g_tune[key] = sh;
  const char* path = std::getenv("AMG_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  if (f) f << key << ' ' << sh.stream << ' ' << sh.g << ' ' << sh.rows_per_block << '\n';
}

template <class Op>
double time_shape(const Shape& sh, int n, const int* rp, const int* ci, const Op& op, hipStream_t s,
                  hipEvent_t e0, hipEvent_t e1) {
  for (int w = 0; w < 2; ++w) sweep(sh, n, rp, ci, op, nullptr, nullptr, s);
  AMG_HIP(hipEventRecord(e0, s));
  constexpr int reps = 5;
  for (int w = 0; w < reps; ++w) sweep(sh, n, rp, ci, op, nullptr, nullptr, s);
  AMG_HIP(hipEventRecord(e1, s));
  AMG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
  return ms / reps;
}

// Shape for one matrix: the tuned one when enabled, else the row-length rule.
template <class MakeOp>
Shape pick_shape(Hierarchy& H, const char* kind, int level, const DBuf<int>& rpd, const DBuf<int>& cid, int n,
                 int ncols, MakeOp make_op, hipStream_t s) {
  const std::vector<int> rp = host_copy(rpd, n + 1);
  Shape rule = make_shape(rp, n);
  if (!H.prm.autotune || n == 0) return rule;
  int maxrow = 0;
  for (int i = 0; i < n; ++i) maxrow = std::max(maxrow, rp[i + 1] - rp[i]);
  char key[256];
  std::snprintf(key, sizeof key, "%s:n%d:nnz%d:max%d:c%d:p%d:t%d:w%d", kind, n, rp[n], maxrow, ncols,
                H.prm.vcycle_prec, H.fp32() && H.prm.transfer_bf16, H.S);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load();
  auto it = g_tune.find(key);
  if (it != g_tune.end()) {
    Shape sh = it->second;
    // recompute the grid for this matrix
    for (const Shape& c : candidate_shapes(rp, n))
      if (c.stream == sh.stream && c.g == sh.g) return c;
  }
  // representative operands: unit vectors of the cycle precision
  const int64_t len = std::max<int64_t>(n, ncols) + 1;
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
  Shape best = rule;
  double tbest = 1e300;
  {
    auto op = make_op(len);
    for (const Shape& c : candidate_shapes(rp, n)) {
      const double t = time_shape(c, n, rpd.p, cid.p, op.op, s, e0, e1);
      if (t < tbest) {
        tbest = t;
        best = c;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)level;
  tune_store(key, best);
  return best;
}

// Owns the scratch vectors of a timing operator.
template <class Op, class T>
struct TuneOp {
  DBuf<T> a, b, c;
  Op op;
};

}  // namespace

bool tune_lookup(const std::string& key, Shape* out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load();
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

void tune_record(const std::string& key, const Shape& sh) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load();
  tune_store(key, sh);
}

void choose_shapes(Hierarchy& H, hipStream_t s) {
  const bool f32 = H.fp32();
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level& L = H.lv[l];
    const int nc = l + 1 < H.lv.size() ? L.nagg : 0;
    if (L.sell) {
      L.shA = Shape{};
      L.shA.stream = L.sell_form == 2 ? 3 : 2;
      L.shA.grid = round8(((int64_t)L.n + kBlock - 1) / kBlock);
    } else if (f32) {
      L.shA = pick_shape(H, "A", (int)l, L.rp, L.ci, L.n, nc, [&](int64_t len) {
        auto t = std::make_unique<TuneOp<OpResid<float, float>, float>>();
        t->a.alloc(len); t->b.alloc(len); t->c.alloc(len);
        AMG_HIP(hipMemsetAsync(t->a.p, 0, t->a.bytes(), s));
        AMG_HIP(hipMemsetAsync(t->b.p, 0, t->b.bytes(), s));
        t->op = OpResid<float, float>{L.v32.p, t->a.p, t->b.p, t->c.p};
        return std::move(*t);
      }, s);
    } else {
      L.shA = pick_shape(H, "A", (int)l, L.rp, L.ci, L.n, nc, [&](int64_t len) {
        TuneOp<OpResid<double, double>, double> t;
        t.a.alloc(len); t.b.alloc(len); t.c.alloc(len);
        AMG_HIP(hipMemsetAsync(t.a.p, 0, t.a.bytes(), s));
        AMG_HIP(hipMemsetAsync(t.b.p, 0, t.b.bytes(), s));
        t.op = OpResid<double, double>{L.v.p, t.a.p, t.b.p, t.c.p};
        return t;
      }, s);
    }
    // nontemporal entry streams for operators larger than the last-level cache
    const double abytes = L.sell ? (double)L.sell_len * (L.sell_form == 2 ? 8.0 : 12.0) : 12.0 * (double)L.nnz;
    L.shA.nt = abytes > kLlcBytes ? 1 : 0;
    if (l + 1 == H.lv.size()) continue;
    if (f32 && H.bf16()) {
      L.shP = pick_shape(H, "P", (int)l, L.prp, L.pci, L.n, nc, [&](int64_t len) {
        TuneOp<OpProlong<uint16_t, float>, float> t;
        t.a.alloc(len); t.b.alloc(len);
        AMG_HIP(hipMemsetAsync(t.a.p, 0, t.a.bytes(), s));
        AMG_HIP(hipMemsetAsync(t.b.p, 0, t.b.bytes(), s));
        t.op = OpProlong<uint16_t, float>{L.pbf.p, t.a.p, t.b.p};
        return t;
      }, s);
      L.shR = pick_shape(H, "R", (int)l, L.rrp, L.rci, L.nagg, L.n, [&](int64_t len) {
        TuneOp<OpRestrict<uint16_t, float>, float> t;
        t.a.alloc(len); t.b.alloc(len);
        AMG_HIP(hipMemsetAsync(t.a.p, 0, t.a.bytes(), s));
        t.op = OpRestrict<uint16_t, float>{L.rbf.p, t.a.p, t.b.p, nullptr, nullptr};
        return t;
      }, s);
    } else if (f32) {
      L.shP = pick_shape(H, "P", (int)l, L.prp, L.pci, L.n, nc, [&](int64_t len) {
        TuneOp<OpProlong<float, float>, float> t;
        t.a.alloc(len); t.b.alloc(len);
        AMG_HIP(hipMemsetAsync(t.a.p, 0, t.a.bytes(), s));
        AMG_HIP(hipMemsetAsync(t.b.p, 0, t.b.bytes(), s));
        t.op = OpProlong<float, float>{L.pv32.p, t.a.p, t.b.p};
        return t;
      }, s);
      L.shR = pick_shape(H, "R", (int)l, L.rrp, L.rci, L.nagg, L.n, [&](int64_t len) {
        TuneOp<OpRestrict<float, float>, float> t;
        t.a.alloc(len); t.b.alloc(len);
        AMG_HIP(hipMemsetAsync(t.a.p, 0, t.a.bytes(), s));
        t.op = OpRestrict<float, float>{L.rv32.p, t.a.p, t.b.p, nullptr, nullptr};
        return t;
      }, s);
    } else {
      L.shP = pick_shape(H, "P", (int)l, L.prp, L.pci, L.n, nc, [&](int64_t len) {
        TuneOp<OpProlong<double, double>, double> t;
        t.a.alloc(len); t.b.alloc(len);
        AMG_HIP(hipMemsetAsync(t.a.p, 0, t.a.bytes(), s));
        AMG_HIP(hipMemsetAsync(t.b.p, 0, t.b.bytes(), s));
        t.op = OpProlong<double, double>{L.pv.p, t.a.p, t.b.p};
        return t;
      }, s);
      L.shR = pick_shape(H, "R", (int)l, L.rrp, L.rci, L.nagg, L.n, [&](int64_t len) {
        TuneOp<OpRestrict<double, double>, double> t;
        t.a.alloc(len); t.b.alloc(len);
        AMG_HIP(hipMemsetAsync(t.a.p, 0, t.a.bytes(), s));
        t.op = OpRestrict<double, double>{L.rv.p, t.a.p, t.b.p, nullptr, nullptr};
        return t;
      }, s);
    }
    // the restriction gathers the fine vector, which a cached stream would
    // evict; the prolongation gathers only the (small) coarse vector, and
    // nontemporal loads measured slower there (192^3: 93.8 vs 89.7 us)
    const double pwb = f32 ? (H.bf16() ? 2.0 : 4.0) : 8.0;
    L.shR.nt = (pwb + 4.0) * (double)L.pnnz > kLlcBytes ? 1 : 0;
    L.shP.nt = 0;
  }
  AMG_HIP(hipStreamSynchronize(s));
}

int64_t solve_partials_count(const Hierarchy& H) {
  int64_t np = std::max<int64_t>(vec_grid(H.n), H.lv[0].shA.grid);
  np = std::max<int64_t>(np, vec_grid(H.co.n));
  return np * 4 + 64;
}

SolveWork solve_work(Hierarchy& H) {
  return SolveWork{H.r.p, H.z.p, H.p.p, H.z2.p, H.q.p, H.partials.p, H.ctl.p, H.h_ctl, true};
}

void alloc_solve_workspace(Hierarchy& H) {
  const int n = H.n;
  H.r.alloc(n);
  H.z.alloc(n);
  H.p.alloc(n);
  H.z2.alloc(n);
  H.q.alloc(n);
  H.partials.alloc(solve_partials_count(H));
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

// Algorithmic bytes of one launch: each matrix array streamed once, each
// distinct vector operand read once (neighbour gathers counted once), each
// output written once.
double kernel_bytes(const Hierarchy& H, int kid, int level, int flexible) {
  const int nl = (int)H.lv.size();
  if (level < 0 || level >= nl) return 0.0;
  const Level& L = H.lv[level];
  const double v = H.fp32() ? 4.0 : 8.0;                        // cycle vector/value bytes
  const double pw = H.fp32() ? (H.bf16() ? 2.0 : 4.0) : 8.0;   // transfer value bytes
  const double n = L.n, nnz = (double)L.nnz;
  auto M = [](double nz, double rows, double w) { return nz * (w + 4.0) + 4.0 * (rows + 1.0); };
  // operator matrix: the sliced copy when present (its padded values, and
  // columns or slot records, and slice offsets), else the CSR arrays
  auto MA = [&](double w) {
    if (!L.sell) return M(nnz, n, w);
    const double slices = 4.0 * ((L.n + 63) / 64 + 1.0);
    if (L.sell_form == 2) return (double)L.sell_len * w + 16.0 * (double)(L.sell_len / 64) + slices;
    return (double)L.sell_len * (w + 4.0) + slices;
  };
  const double bw = level == 0 ? 8.0 : v;                       // rhs of the level
  const bool has_next = level + 1 < nl;
  const bool next_coarsest = level + 2 == nl;
  switch (kid) {
    // direction update fused with the product: gathers z, reads old p and q,
    // writes new p and q
    case KID_SPMV_DOT: return MA(8.0) + 40.0 * n;
    // residual of the pre-smoothed iterate: reads b, gathers x, writes r
    case KID_PRE: return MA(v) + (bw + 2.0 * v) * n;
    case KID_POST: {
      const double ow = level == 0 ? 8.0 : v;
      return MA(v) + (bw + 2.0 * v + ow) * n + (level == 0 && flexible ? 8.0 * n : 0.0);
    }
    case KID_RESTRICT: {
      if (!has_next) return 0.0;
      const double nc = (double)L.nagg;
      return M((double)L.pnnz, nc, pw) + v * n + v * nc + (next_coarsest ? 0.0 : 2.0 * v * nc);
    }
    case KID_PROLONG:
      if (!has_next) return 0.0;
      return M((double)L.pnnz, n, pw) + v * (double)L.nagg + 2.0 * v * n;
    // x, r, p, q read; x, r written; sw read and x0 = sw o r written in cycle precision
    case KID_CG_UPDATE: return 48.0 * n + 2.0 * v * n;
    case KID_XPAY: return 0.0;  // fused into KID_SPMV_DOT
    case KID_COARSE: {
      const double nc = H.co.n;
      return nc * nc * (nl == 1 ? 8.0 : v) + 2.0 * nc * (nl == 1 ? 8.0 : v);
    }
  }
  return 0.0;
}

// Bytes of one PCG iteration (SpMV+dot, update, V-cycle, direction update).
double iteration_bytes(const Hierarchy& H, int flexible) {
  const int nl = (int)H.lv.size();
  if (!H.prm.precondition)  // plain CG: z = r (16n), <r,z>, <z,q> partials (24n)
    return kernel_bytes(H, KID_SPMV_DOT, 0, flexible) + kernel_bytes(H, KID_CG_UPDATE, 0, flexible) + 40.0 * H.n;
  double b = kernel_bytes(H, KID_SPMV_DOT, 0, flexible) + kernel_bytes(H, KID_CG_UPDATE, 0, flexible) +
             kernel_bytes(H, KID_XPAY, 0, flexible) + kernel_bytes(H, KID_COARSE, nl - 1, flexible);
  for (int l = 0; l < nl - 1; ++l) {
    const double n = H.lv[l].n;
    const double v = H.fp32() ? 4.0 : 8.0;
    b += kernel_bytes(H, KID_PRE, l, flexible) + kernel_bytes(H, KID_RESTRICT, l, flexible) +
         kernel_bytes(H, KID_PROLONG, l, flexible) + H.prm.nu_post * kernel_bytes(H, KID_POST, l, flexible);
    b += (H.prm.nu_pre - 1) * (kernel_bytes(H, KID_PRE, l, flexible) + 2.0 * v * n);
  }
  return b;
}

void set_instrument(Hierarchy& H, int kid, int level) {
  if (H.inst.ev.empty()) {
    H.inst.ev.resize(2 * 8192);
    for (auto& e : H.inst.ev) AMG_HIP(hipEventCreate(&e));
    H.inst.was_done.alloc(8192);
  }
  H.inst.kernel = kid;
  H.inst.level = level;
  H.inst.used = 0;
}

void read_instrument(Hierarchy& H, int* launches, double* total_ms, double* min_ms, double* max_ms) {
  double tot = 0.0, mn = 1e300, mx = 0.0;
  std::vector<int> done(H.inst.used);
  if (H.inst.used) {
    AMG_HIP(hipEventSynchronize(H.inst.ev[2 * H.inst.used - 1]));
    AMG_HIP(hipMemcpy(done.data(), H.inst.was_done.p, sizeof(int) * H.inst.used, hipMemcpyDeviceToHost));
  }
  int working = 0;
  for (int i = 0; i < H.inst.used; ++i) {
    if (done[i]) continue;
    float ms = 0.f;
    AMG_HIP(hipEventElapsedTime(&ms, H.inst.ev[2 * i], H.inst.ev[2 * i + 1]));
    tot += ms;
    mn = std::min(mn, (double)ms);
    mx = std::max(mx, (double)ms);
    ++working;
  }
  *launches = working;
  *total_ms = tot;
  *min_ms = working ? mn : 0.0;
  *max_ms = mx;
}

void apply_vcycle(Hierarchy& H, const double* d_r, double* d_z, hipStream_t s) {
  CycleArgs a{d_r, d_z, nullptr, nullptr, nullptr, 0, 0, 0};
  vcycle(H, a, s);
  AMG_HIP(hipGetLastError());
}

void pattern_grad(Hierarchy& H, const double* d_lam, const double* d_x, double* d_g, hipStream_t s) {
  Level& L = H.lv[0];
  const int grid = (int)(((int64_t)L.n + kBlock / 8 - 1) / (kBlock / 8));
  hipLaunchKernelGGL(k_pattern_grad, dim3(grid), dim3(kBlock), 0, s, L.n, L.rp.p, L.ci.p, d_lam, d_x, d_g);
  AMG_HIP(hipGetLastError());
}

template <class T>
void launch_cg_update(Hierarchy& H, const SolveWork& w, int n, double* d_x, const double* p, hipStream_t s) {
  Level& L0 = H.lv[0];
  hipLaunchKernelGGL((k_cg_update<T>), dim3(vec_grid(n)), dim3(kBlock), 0, s, n, d_x, w.r, p, w.q,
                     Bufs<T>::sw(L0), Bufs<T>::x(L0), w.ctl, w.partials);
}

template <class T>
void launch_sw_mul(Hierarchy& H, const SolveWork& w, int n, hipStream_t s) {
  Level& L0 = H.lv[0];
  hipLaunchKernelGGL((k_sw_mul<T>), dim3(vec_grid(n)), dim3(kBlock), 0, s, n, Bufs<T>::sw(L0), w.r,
                     Bufs<T>::x(L0), w.ctl);
}

void read_ctl(const SolveWork& w, hipStream_t s) {
  AMG_HIP(hipMemcpyAsync(w.h_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
}

// Captures the launches made by `body` on stream s into an executable graph;
// a failure ends the capture before the error propagates.
template <class F>
void capture_graph_impl(hipStream_t s, hipGraphExec_t& ex, F&& body) {
  hipGraph_t g = nullptr;
  AMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  AMG_HIP(hipStreamEndCapture(s, &g));
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    ex = nullptr;
    throw Error(AMG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
}

void capture_graph(hipStream_t s, hipGraphExec_t& ex, const std::function<void()>& body) {
  capture_graph_impl(s, ex, body);
}

// Library stream and join events for graph solves.
void graph_stream(Hierarchy& H) {
  if (!H.gr.gs) {
    AMG_HIP(hipStreamCreateWithFlags(&H.gr.gs, hipStreamNonBlocking));
    AMG_HIP(hipEventCreateWithFlags(&H.gr.ev_in, hipEventDisableTiming));
    AMG_HIP(hipEventCreateWithFlags(&H.gr.ev_out, hipEventDisableTiming));
  }
}

amg_status pcg_solve(Hierarchy& H, const SolveOpts& o, const SolveWork& w, const double* d_b, double* d_x,
                     double tol, amg_info* info, hipStream_t caller) {
  // hierarchies that fit one compute unit: the whole solve in one launch
  if (o.fused_small && H.inst.kernel < 0 && small_solve_ok(H))
    return pcg_solve_small(H, o, w, d_b, d_x, tol, info, caller);
  auto t0 = std::chrono::steady_clock::now();
  Level& L0 = H.lv[0];
  const int n = H.n;
  const bool multi = H.lv.size() > 1;
  // automatic: flexible whenever the preconditioner is not a fixed symmetric
  // operator (FP32 cycle, or unequal pre/post sweep counts)
  const int flexible = o.flexible < 0 ? ((H.fp32() || H.prm.nu_pre != H.prm.nu_post) ? 1 : 0) : o.flexible;
  const bool graphs = w.graphs && o.use_graphs && H.inst.kernel < 0;
  hipStream_t s = caller;
  if (graphs) {
    graph_stream(H);
    AMG_HIP(hipEventRecord(H.gr.ev_in, caller));
    AMG_HIP(hipStreamWaitEvent(H.gr.gs, H.gr.ev_in, 0));
    s = H.gr.gs;
    if (H.gr.key_x != d_x || H.gr.key_flex != flexible || H.gr.key_w != 1) {
      H.gr.reset();
      H.gr.key_x = d_x;
      H.gr.key_flex = flexible;
      H.gr.key_w = 1;
    }
  }
  Ctl* ctl = w.ctl;
  double* part = w.partials;
  const int gv = vec_grid(n);
  hipLaunchKernelGGL(k_cg_init, dim3(gv), dim3(kBlock), 0, s, n, d_b, w.r, d_x, part);
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kFinBlock), 0, s, ctl, part, gv, tol, o.maxiter, flexible);
  AMG_HIP(hipGetLastError());
  // search directions alternate between two buffers (the fused direction
  // update writes the new p while neighbours still gather the old one)
  double* pb[2] = {w.p, w.z2};
  int cur = 0;
  // one PCG iteration: p = z + beta p and q = A p; alpha; x, r update; z = M^-1 r, beta
  auto iteration = [&](int first, int c, hipStream_t st) {
    int np;
    {
      InstScope is(H, KID_SPMV_DOT, 0, st, ctl);
      np = sweep(L0.shA, n, L0.arp(), L0.aci(), OpSpmvXpayDev{L0.av(), w.z, pb[c], pb[c ^ 1], w.q, ctl, first},
                 ctl, part, st);
    }
    hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(kFinBlock), 0, st, ctl, part, np);
    {
      InstScope is(H, KID_CG_UPDATE, 0, st, ctl);
      if (H.fp32()) launch_cg_update<float>(H, w, n, d_x, pb[c ^ 1], st);
      else launch_cg_update<double>(H, w, n, d_x, pb[c ^ 1], st);
    }
    hipLaunchKernelGGL(k_fin_update, dim3(1), dim3(kFinBlock), 0, st, ctl, part, gv);
    CycleArgs a{w.r, w.z, w.q, ctl, part, flexible ? 2 : 1, 0, multi ? 1 : 0};
    vcycle(H, a, st);
  };
  // two iterations captured once per direction-buffer parity and replayed
  auto pair = [&](int c) {
    hipGraphExec_t& ex = H.gr.exec[c];
    if (!ex) capture_graph(s, ex, [&] {
        iteration(0, c, s);
        iteration(0, c ^ 1, s);
      });
    AMG_HIP(hipGraphLaunch(ex, s));
  };
  int restarts = 0;
  amg_status st = AMG_OK;
  for (;;) {
    // (re)start: z = M^-1 r, rz = <r, z>; the first direction is p = z
    if (multi) {
      if (H.fp32()) launch_sw_mul<float>(H, w, n, s);
      else launch_sw_mul<double>(H, w, n, s);
    }
    CycleArgs a0{w.r, w.z, w.q, ctl, part, 1, 1, multi ? 1 : 0};
    vcycle(H, a0, s);
    int first = 1;
    // Iterations are queued in chunks; between chunks the host reads the
    // control block and sizes the next chunk from the observed decay of
    // ||r||^2 so that few iterations are queued past convergence (those
    // return at once on the done flag).
    int chunk = o.check_every > 0 ? o.check_every : 4;
    int it_prev = -1;
    double rr_prev = 0.0;
    for (;;) {
      int left = chunk;
      if (first) {
        iteration(1, cur, s);
        cur ^= 1;
        first = 0;
        --left;
      }
      if (graphs)
        for (; left >= 2; left -= 2) pair(cur);
      for (; left > 0; --left) {
        iteration(0, cur, s);
        cur ^= 1;
      }
      AMG_HIP(hipGetLastError());
      read_ctl(w, s);
      if (w.h_ctl->done) break;
      if (o.check_every <= 0) {
        const Ctl& c = *w.h_ctl;
        if (it_prev < 0) {  // decay measured from ||r_0||^2 = ||b||^2
          it_prev = 0;
          rr_prev = c.bb;
        }
        int next = 4;
        if (c.thresh <= 0.0) {
          next = 32;
        } else if (c.iters > it_prev && rr_prev > 0.0 && c.rr > 0.0) {
          const double rate = std::log(c.rr / rr_prev) / (double)(c.iters - it_prev);
          if (rate < -1e-3) next = (int)std::min(64.0, std::ceil(std::log(c.thresh / c.rr) / rate));
        }
        it_prev = c.iters;
        rr_prev = c.rr;
        next = std::min(next, std::max(1, c.maxiter - c.iters));
        chunk = std::max(1, std::min(next, 32));
      }
    }
    const int state = w.h_ctl->state;
    if (state == 3) break;  // b = 0
    if (state < 0) {
      st = AMG_ERR_BREAKDOWN;
      break;
    }
    // true residual r = b - A x
    const int np = sweep(L0.shA, n, L0.arp(), L0.aci(), OpTrueResid{L0.av(), d_x, d_b, w.r}, nullptr, part, s);
    hipLaunchKernelGGL(k_fin_trr, dim3(1), dim3(kFinBlock), 0, s, ctl, part, np);
    read_ctl(w, s);
    const Ctl& c = *w.h_ctl;
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
  if (graphs) {
    AMG_HIP(hipEventRecord(H.gr.ev_out, s));
    AMG_HIP(hipStreamWaitEvent(caller, H.gr.ev_out, 0));
  }
  const Ctl& c = *w.h_ctl;
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

// Right-preconditioned BiCGSTAB (van der Vorst, 1992), the paper's default
// Krylov method (Section 2.1), from x0 = 0 with shadow residual r^ = b.
// One iteration, every scalar formed on the device:
//   p = r + beta (p - omega v)        k_bi_dir   (p = r after a (re)start)
//   y = M^-1 p                        V-cycle
//   v = A y, <r^, v>                  sweep      -> alpha = rho / <r^, v>
//   x += alpha y, s = r - alpha v     k_bi_half  -> ||s|| test, iteration count
//   z = M^-1 s                        V-cycle
//   t = A z, <s, t>, <t, t>           sweep      -> omega
//   x += omega z, r = s - omega t     k_bi_full  -> ||r|| test, rho, beta
// Stopping, verification and restarts follow pcg_solve.
amg_status bicgstab_solve(Hierarchy& H, const SolveOpts& o, const double* d_b, double* d_x, double tol,
                          amg_info* info, hipStream_t caller) {
  auto t0 = std::chrono::steady_clock::now();
  Level& L0 = H.lv[0];
  const int n = H.n;
  const bool graphs = o.use_graphs && H.inst.kernel < 0;
  if (!H.rh.p) {
    H.rh.alloc(n);
    H.bv.alloc(n);
    H.by.alloc(n);
    H.bs.alloc(n);
    H.bt2.alloc(n);
    AMG_HIP(hipMemsetAsync(H.bv.p, 0, H.bv.bytes(), caller));
  }
  hipStream_t s = caller;
  if (graphs) {
    graph_stream(H);
    AMG_HIP(hipEventRecord(H.gr.ev_in, caller));
    AMG_HIP(hipStreamWaitEvent(H.gr.gs, H.gr.ev_in, 0));
    s = H.gr.gs;
    if (H.gr.key_bx != d_x && H.gr.bexec) {
      (void)hipGraphExecDestroy(H.gr.bexec);
      H.gr.bexec = nullptr;
    }
    H.gr.key_bx = d_x;
  }
  Ctl* ctl = H.ctl.p;
  double* part = H.partials.p;
  double* r = H.r.p;
  double* p = H.p.p;
  double* z = H.z.p;
  double* rh = H.rh.p;
  double* v = H.bv.p;
  double* y = H.by.p;
  double* sv = H.bs.p;
  double* t = H.bt2.p;
  // no preconditioner: y = p and z = s are the same vectors (no copies)
  const bool prec = H.prm.precondition != 0;
  if (!prec) {
    y = p;
    z = sv;
  }
  const int gv = vec_grid(n);
  hipLaunchKernelGGL(k_bi_init, dim3(gv), dim3(kBlock), 0, s, n, d_b, r, rh, d_x, part);
  hipLaunchKernelGGL(k_bfin_init, dim3(1), dim3(kFinBlock), 0, s, ctl, part, gv, tol, o.maxiter);
  AMG_HIP(hipGetLastError());
  // with a multilevel cycle the vector kernels also write the level-0
  // pre-smoothed iterate of the V-cycle that follows them
  const bool x0w = prec && H.lv.size() > 1;
  auto launch_dir = [&](int first, hipStream_t st) {
    Level& L0c = H.lv[0];
    if (H.fp32())
      hipLaunchKernelGGL(k_bi_dir<float>, dim3(gv), dim3(kBlock), 0, st, n, r, v, p, Bufs<float>::sw(L0c),
                         x0w ? Bufs<float>::x(L0c) : nullptr, ctl, first);
    else
      hipLaunchKernelGGL(k_bi_dir<double>, dim3(gv), dim3(kBlock), 0, st, n, r, v, p, Bufs<double>::sw(L0c),
                         x0w ? Bufs<double>::x(L0c) : nullptr, ctl, first);
  };
  auto launch_half = [&](hipStream_t st) {
    Level& L0c = H.lv[0];
    if (H.fp32())
      hipLaunchKernelGGL(k_bi_half<float>, dim3(gv), dim3(kBlock), 0, st, n, d_x, y, r, v, sv, Bufs<float>::sw(L0c),
                         x0w ? Bufs<float>::x(L0c) : nullptr, ctl, part);
    else
      hipLaunchKernelGGL(k_bi_half<double>, dim3(gv), dim3(kBlock), 0, st, n, d_x, y, r, v, sv,
                         Bufs<double>::sw(L0c), x0w ? Bufs<double>::x(L0c) : nullptr, ctl, part);
  };
  auto iteration = [&](int first, hipStream_t st) {
    launch_dir(first, st);
    if (prec) vcycle(H, CycleArgs{p, y, nullptr, ctl, part, 0, 0, x0w ? 1 : 0}, st);
    int np;
    {
      InstScope is(H, KID_SPMV_DOT, 0, st, ctl);
      np = sweep(L0.shA, n, L0.arp(), L0.aci(), OpSpmvDots<1>{L0.av(), y, v, rh}, ctl, part, st);
    }
    hipLaunchKernelGGL(k_bfin_alpha, dim3(1), dim3(kFinBlock), 0, st, ctl, part, np);
    launch_half(st);
    hipLaunchKernelGGL(k_bfin_half, dim3(1), dim3(kFinBlock), 0, st, ctl, part, gv);
    if (prec) vcycle(H, CycleArgs{sv, z, nullptr, ctl, part, 0, 0, x0w ? 1 : 0}, st);
    {
      InstScope is(H, KID_SPMV_DOT, 0, st, ctl);
      np = sweep(L0.shA, n, L0.arp(), L0.aci(), OpSpmvDots<2>{L0.av(), z, t, sv}, ctl, part, st);
    }
    hipLaunchKernelGGL(k_bfin_omega, dim3(1), dim3(kFinBlock), 0, st, ctl, part, np);
    hipLaunchKernelGGL(k_bi_full, dim3(gv), dim3(kBlock), 0, st, n, d_x, z, sv, t, rh, r, ctl, part);
    hipLaunchKernelGGL(k_bfin_full, dim3(1), dim3(kFinBlock), 0, st, ctl, part, gv);
  };
  int restarts = 0;
  amg_status st = AMG_OK;
  for (;;) {
    int first = 1;
    int chunk = o.check_every > 0 ? o.check_every : 2;
    int it_prev = -1;
    double rr_prev = 0.0;
    for (;;) {
      int left = chunk;
      if (first) {
        iteration(1, s);
        first = 0;
        --left;
      }
      if (graphs && left > 0) {
        if (!H.gr.bexec) capture_graph(s, H.gr.bexec, [&] { iteration(0, s); });
        for (; left > 0; --left) AMG_HIP(hipGraphLaunch(H.gr.bexec, s));
      }
      for (; left > 0; --left) iteration(0, s);
      AMG_HIP(hipGetLastError());
      read_ctl(H, s);
      if (H.h_ctl->done) break;
      if (o.check_every <= 0) {
        // chunk sized from the observed decay of the residual norm, as in PCG
        const Ctl& c = *H.h_ctl;
        if (it_prev < 0) {
          it_prev = 0;
          rr_prev = c.bb;
        }
        int next = 2;
        if (c.thresh <= 0.0) {
          next = 16;
        } else if (c.iters > it_prev && rr_prev > 0.0 && c.rr > 0.0) {
          const double rate = std::log(c.rr / rr_prev) / (double)(c.iters - it_prev);
          if (rate < -1e-3) next = (int)std::min(32.0, std::ceil(std::log(c.thresh / c.rr) / rate));
        }
        it_prev = c.iters;
        rr_prev = c.rr;
        next = std::min(next, std::max(1, c.maxiter - c.iters));
        chunk = std::max(1, std::min(next, 16));
      }
    }
    const int state = H.h_ctl->state;
    if (state == 3) break;  // b = 0
    if (state < 0) {
      st = AMG_ERR_BREAKDOWN;
      break;
    }
    const int np = sweep(L0.shA, n, L0.arp(), L0.aci(), OpTrueResid{L0.av(), d_x, d_b, r}, nullptr, part, s);
    hipLaunchKernelGGL(k_fin_trr, dim3(1), dim3(kFinBlock), 0, s, ctl, part, np);
    read_ctl(H, s);
    const Ctl& c = *H.h_ctl;
    if (c.trr <= c.thresh) {
      st = AMG_OK;
      break;
    }
    if (state == 1 && restarts < 5 && c.iters < c.maxiter) {
      ++restarts;
      hipLaunchKernelGGL(k_bi_restart, dim3(1), dim3(1), 0, s, ctl);
      hipLaunchKernelGGL(k_copy_z, dim3(gv), dim3(kBlock), 0, s, n, r, rh, (const Ctl*)nullptr);
      continue;
    }
    st = AMG_NOT_CONVERGED;
    break;
  }
  if (graphs) {
    AMG_HIP(hipEventRecord(H.gr.ev_out, s));
    AMG_HIP(hipStreamWaitEvent(caller, H.gr.ev_out, 0));
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
