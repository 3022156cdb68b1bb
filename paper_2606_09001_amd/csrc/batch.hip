// Batched solves: W columns in one launch per step, vectors stored row-major
// [n][W].  Two forms share every kernel:
//   - many right-hand sides of one matrix (SYS = false): matrix values,
//     smoother weights and the coarse inverse are shared by all columns;
//   - many systems with one sparsity pattern (SYS = true, W = S): value
//     arrays are interleaved [entry][S], so column c reads its own values.
// Each column is an independent PCG (its own alpha, beta, convergence and
// restarts; converged columns are frozen), not block CG.
//
// Wide sweep kernel: a group of LW = 2^ceil(log2 W) lanes per row, lane =
// column; every lane of the group reads the row's column indices (one
// broadcast transaction), the gathers x[j][0..W) are contiguous, so each
// nonzero costs one coalesced W-wide access.  Column-wise dot products are
// reduced per workgroup in a fixed order and folded by a finalize kernel with
// one workgroup per column.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <map>
#include <type_traits>

#include "amg_internal.hpp"

namespace amg {
namespace {

constexpr int kWGrid = 2048;  // workgroups of the wide sweeps (partials per column)
constexpr int kWFin = 256;    // threads per finalize workgroup (one workgroup per column)

__device__ inline int logical_block_w() {
  const int g = gridDim.x;
  if ((g & 7) == 0) return (blockIdx.x & 7) * (g >> 3) + (blockIdx.x >> 3);
  return blockIdx.x;
}

inline int wide_grid(int64_t n, int LW) {
  const int64_t rb = kBlock / LW;
  int64_t g = std::min<int64_t>((n + rb - 1) / rb, kWGrid);
  if (g >= 64) g = g / 8 * 8;
  return (int)std::max<int64_t>(g, 1);
}

// V consecutive columns of a row-major [rows][W] array as one vector access:
// a lane of a wide sweep owns V adjacent columns (16-byte accesses for FP64
// vectors when V = 2).  The element index is a multiple of V and the arrays
// are aligned to V elements.
template <class T, int V>
struct LaneVec {
  using type = T __attribute__((ext_vector_type(V)));
};
template <class T>
struct LaneVec<T, 1> {
  using type = T;
};

template <int V, bool NT = false, class T>
__device__ inline void ldv(const T* p, int64_t e, T (&o)[V]) {
  using LT = typename LaneVec<T, V>::type;
  const LT x = stream_load<NT>(reinterpret_cast<const LT*>(p + e));
  if constexpr (V == 1) {
    o[0] = x;
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = x[v];
  }
}

template <int V, class T>
__device__ inline void stv(T* p, int64_t e, const T (&in)[V]) {
  using LT = typename LaneVec<T, V>::type;
  LT x;
  if constexpr (V == 1) {
    x = in[0];
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = in[v];
  }
  *reinterpret_cast<LT*>(p + e) = x;
}

// Values of stored entry k for columns c0 .. c0+V-1.  The per-system value
// arrays ([entry][S]) are streamed once per sweep and are many times larger
// than the last-level cache: nontemporal loads.
template <bool SYS, int V, class VT>
__device__ inline void vals_at(const VT* v, int64_t k, int c0, int W, VT (&o)[V]) {
  if constexpr (SYS) {
    ldv<V, true>(v, k * W + c0, o);
  } else {
    const VT a = v[k];
#pragma unroll
    for (int u = 0; u < V; ++u) o[u] = a;
  }
}
// Per-row quantity (smoother weight) for columns c0 .. c0+V-1.
template <bool SYS, int V, class T>
__device__ inline void rows_at(const T* p, int i, int c0, int W, T (&o)[V]) {
  if constexpr (SYS) {
    ldv<V, true>(p, (int64_t)i * W + c0, o);
  } else {
    const T a = p[i];
#pragma unroll
    for (int u = 0; u < V; ++u) o[u] = a;
  }
}
// Per-row quantity for one column (elementwise kernels).
template <bool SYS, class T>
__device__ inline T row_at(const T* v, int i, int c, int W) {
  if constexpr (SYS) return stream_load<true>(v + (int64_t)i * W + c);
  else return v[i];
}

// ----------------------------------------------------------- operators
//
// A wide sweep forms, per row and column, s = sum_k mul(a_k, gv[col_k]) over
// the row's entries in stored order.  Each operator supplies
//   GT, VT, PT          gathered-vector, matrix-value and sum types
//   v, gv               the values and the gathered vector ([operand rows][W])
//   kSquare             gv is indexed like the rows, so a window of it
//                       around a block's rows can be staged in LDS
//   cols<V>(c0)         per-column scalars of columns c0 .. c0+V-1
//   row_in<V>, epi<V>   the row's own operands and its outputs; kOwn: row_in
//                       takes the row's own entries of gv (xo), which the
//                       sweep reads from the staged window when it has one;
//                       kLateRow: the staged sweep loads them after the row's
//                       gathers instead of before
// and the sweep's per-column reductions in d[m * V + v].

struct NoCols {};

// r = b - A x  (x = sw o b written by the producer of b)
template <bool SYS, class T, class BT>
struct WResid {
  using PT = T;
  using VT = T;
  using GT = T;
  static constexpr bool kSys = SYS, kSquare = true, kOwn = false, kLateRow = false;
  static constexpr int NRED = 0;
  const T* v;
  const BT* b;
  const T* gv;
  T* r;
  int W;
  template <int V>
  __device__ NoCols cols(int) const { return {}; }
  __device__ static PT mul(VT a, GT g) { return a * g; }
  template <int V>
  struct Row {
    T b[V];
  };
  template <int V>
  __device__ Row<V> row_in(int row, int c0, NoCols, const GT (&)[V]) const {
    BT bb[V];
    ldv<V>(b, (int64_t)row * W + c0, bb);
    Row<V> a;
#pragma unroll
    for (int u = 0; u < V; ++u) a.b[u] = (T)bb[u];
    return a;
  }
  template <int V>
  __device__ void epi(int row, int c0, const PT (&s)[V], const Row<V>& a, NoCols, double*) const {
    T o[V];
#pragma unroll
    for (int u = 0; u < V; ++u) o[u] = a.b[u] - s[u];
    stv<V>(r, (int64_t)row * W + c0, o);
  }
};

// y = R x ; xc = swc o y
template <bool SYS, class RT, class T>
struct WRestrict {
  using PT = T;
  using VT = RT;
  using GT = T;
  static constexpr bool kSys = SYS, kSquare = false, kOwn = false, kLateRow = false;
  static constexpr int NRED = 0;
  const RT* v;
  const T* gv;
  T* y;
  const T* swc;
  T* xc;
  int W;
  template <int V>
  __device__ NoCols cols(int) const { return {}; }
  __device__ static PT mul(VT a, GT g) { return (T)ValCvt<RT>::f(a) * g; }
  template <int V>
  struct Row {
    T w[V];
  };
  template <int V>
  __device__ Row<V> row_in(int row, int c0, NoCols, const GT (&)[V]) const {
    Row<V> a;
    if (xc) {
      rows_at<SYS, V>(swc, row, c0, W, a.w);
    } else {
#pragma unroll
      for (int u = 0; u < V; ++u) a.w[u] = (T)0;
    }
    return a;
  }
  template <int V>
  __device__ void epi(int row, int c0, const PT (&s)[V], const Row<V>& a, NoCols, double*) const {
    const int64_t e = (int64_t)row * W + c0;
    stv<V>(y, e, s);
    if (xc) {
      T o[V];
#pragma unroll
      for (int u = 0; u < V; ++u) o[u] = a.w[u] * s[u];
      stv<V>(xc, e, o);
    }
  }
};

// x += P xc
template <bool SYS, class RT, class T>
struct WProlong {
  using PT = T;
  using VT = RT;
  using GT = T;
  static constexpr bool kSys = SYS, kSquare = false, kOwn = false, kLateRow = false;
  static constexpr int NRED = 0;
  const RT* v;
  const T* gv;
  T* x;
  int W;
  template <int V>
  __device__ NoCols cols(int) const { return {}; }
  __device__ static PT mul(VT a, GT g) { return (T)ValCvt<RT>::f(a) * g; }
  template <int V>
  struct Row {
    T x[V];
  };
  template <int V>
  __device__ Row<V> row_in(int row, int c0, NoCols, const GT (&)[V]) const {
    Row<V> a;
    ldv<V>(x, (int64_t)row * W + c0, a.x);
    return a;
  }
  template <int V>
  __device__ void epi(int row, int c0, const PT (&s)[V], const Row<V>& a, NoCols, double*) const {
    T o[V];
#pragma unroll
    for (int u = 0; u < V; ++u) o[u] = a.x[u] + s[u];
    stv<V>(x, (int64_t)row * W + c0, o);
  }
};

// out = x + sw o (b - A x); RED >= 1: <b, out>, RED == 2: <out, q> per column
template <bool SYS, class T, class BT, class OT, int RED>
struct WPost {
  using PT = T;
  using VT = T;
  using GT = T;
  static constexpr bool kSys = SYS, kSquare = true, kOwn = true, kLateRow = true;
  static constexpr int NRED = RED;
  const T* v;
  const T* sw;
  const BT* b;
  const T* gv;
  OT* out;
  const double* q;
  int W;
  template <int V>
  __device__ NoCols cols(int) const { return {}; }
  __device__ static PT mul(VT a, GT g) { return a * g; }
  template <int V>
  struct Row {
    BT b[V];
    T x[V], w[V];
    double q[V];
  };
  template <int V>
  __device__ Row<V> row_in(int row, int c0, NoCols, const GT (&xo)[V]) const {
    const int64_t e = (int64_t)row * W + c0;
    Row<V> a;
    ldv<V>(b, e, a.b);
#pragma unroll
    for (int u = 0; u < V; ++u) a.x[u] = xo[u];
    rows_at<SYS, V>(sw, row, c0, W, a.w);
    if constexpr (RED >= 2) ldv<V>(q, e, a.q);
    return a;
  }
  template <int V>
  __device__ void epi(int row, int c0, const PT (&s)[V], const Row<V>& a, NoCols, double* d) const {
    OT oo[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const T o = a.x[u] + a.w[u] * ((T)a.b[u] - s[u]);
      oo[u] = (OT)o;
      if constexpr (RED >= 1) d[u] += (double)a.b[u] * (double)oo[u];
      if constexpr (RED >= 2) d[V + u] += (double)oo[u] * a.q[u];
    }
    stv<V>(out, (int64_t)row * W + c0, oo);
  }
};

// p' = z + beta_c p and q' = A z + beta_c q (= A p'); p' = z and q' = A z for columns starting a
// (re)start; <p', q'>
template <bool SYS>
struct WSpmvXpay {
  using PT = double;
  using VT = double;
  using GT = double;
  static constexpr bool kSys = SYS, kSquare = true, kOwn = true, kLateRow = false;
  static constexpr int NRED = 1;
  const double* v;
  const double* gv;  // z
  const double* p;
  double* pn;
  double* q;
  const WCtl* ctl;
  int W;
  // q' = A p' is formed as A z + beta q (the same vector in exact
  // arithmetic, since q = A p), so the sweep gathers z only; p and q are read
  // at the row itself.  Both row operands are always loaded (no divergent
  // branch around a load); a column that (re)starts takes p' = z, q' = A z.
  template <int V>
  struct Cols {
    double beta[V];
    int first[V];
  };
  template <int V>
  __device__ Cols<V> cols(int c0) const {
    Cols<V> k;
#pragma unroll
    for (int u = 0; u < V; ++u) {
      k.beta[u] = ctl[c0 + u].beta;
      k.first[u] = ctl[c0 + u].first;
    }
    return k;
  }
  __device__ static PT mul(VT a, GT g) { return a * g; }
  template <int V>
  struct Row {
    double pr[V], qo[V];
  };
  template <int V>
  __device__ Row<V> row_in(int row, int c0, const Cols<V>& k, const GT (&zz)[V]) const {
    const int64_t e = (int64_t)row * W + c0;
    double pp[V];
    Row<V> a;
    ldv<V>(p, e, pp);
    ldv<V>(q, e, a.qo);
#pragma unroll
    for (int u = 0; u < V; ++u) a.pr[u] = k.first[u] ? zz[u] : zz[u] + k.beta[u] * pp[u];
    return a;
  }
  template <int V>
  __device__ void epi(int row, int c0, const PT (&s)[V], const Row<V>& a, const Cols<V>& k, double* d) const {
    const int64_t e = (int64_t)row * W + c0;
    double qn[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
      qn[u] = k.first[u] ? s[u] : s[u] + k.beta[u] * a.qo[u];
      d[u] += a.pr[u] * qn[u];
    }
    stv<V>(pn, e, a.pr);
    stv<V>(q, e, qn);
  }
};

// r = b - A x, ||r||^2 per column
template <bool SYS>
struct WTrueResid {
  using PT = double;
  using VT = double;
  using GT = double;
  static constexpr bool kSys = SYS, kSquare = true, kOwn = false, kLateRow = false;
  static constexpr int NRED = 1;
  const double* v;
  const double* gv;  // x
  const double* b;
  double* r;
  int W;
  template <int V>
  __device__ NoCols cols(int) const { return {}; }
  __device__ static PT mul(VT a, GT g) { return a * g; }
  template <int V>
  struct Row {
    double b[V];
  };
  template <int V>
  __device__ Row<V> row_in(int row, int c0, NoCols, const GT (&)[V]) const {
    Row<V> a;
    ldv<V>(b, (int64_t)row * W + c0, a.b);
    return a;
  }
  template <int V>
  __device__ void epi(int row, int c0, const PT (&s)[V], const Row<V>& a, NoCols, double* d) const {
    double o[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
      o[u] = a.b[u] - s[u];
      d[u] += o[u] * o[u];
    }
    stv<V>(r, (int64_t)row * W + c0, o);
  }
};

// Column-wise partial sums of one workgroup, folded over its rows in a
// fixed order: partials[(m*W + c)*gridDim + block].  d holds the lane's sums
// for its V columns, d[m*V + v]; lane l of a row group owns columns l*V + v.
// `red` is LDS scratch of NRED * kBlock * V doubles that no thread reads or
// writes any more.
template <int LW, int V, int NRED>
__device__ inline void publish_w(const double* d, int W, double* partials, double* red) {
  if constexpr (NRED > 0) {
    constexpr int RB = kBlock / LW, LV = LW * V;
#pragma unroll
    for (int m = 0; m < NRED; ++m)
#pragma unroll
      for (int u = 0; u < V; ++u) red[m * kBlock * V + threadIdx.x * V + u] = d[m * V + u];
    __syncthreads();
    if ((int)threadIdx.x < LV && (int)threadIdx.x < W) {
      const int c = threadIdx.x;
#pragma unroll
      for (int m = 0; m < NRED; ++m) {
        double s = 0.0;
        for (int r = 0; r < RB; ++r) s += red[m * kBlock * V + r * LV + c];
        partials[((int64_t)m * W + c) * gridDim.x + blockIdx.x] = s;
      }
    }
  }
}
template <int LW, int V, int NRED>
__device__ inline void publish_w(const double* d, int W, double* partials) {
  if constexpr (NRED > 0) {
    __shared__ double red[NRED * kBlock * V];
    publish_w<LW, V, NRED>(d, W, partials, red);
  }
}

// Row-group schedule of a wide sweep.  Workgroups are dispatched round-robin
// over the 8 XCDs; each XCD owns one contiguous eighth of the row groups,
// split into `spx` streams.  The workgroups of a stream (a team) take its
// groups in turn, so a stream advances as one front: the rows a front
// gathers from (its neighbours at short index distance) stay in that XCD's
// L2 while the front passes.  spx = G/8 gives every workgroup a contiguous
// range of its own.  spx = -1 is one front for the whole device:
// consecutive chunks of G/8 row groups go to the XCDs in turn, so the 8 XCDs
// sweep 8 neighbouring chunks at a time (for a 3D grid with chunks of about a
// plane, a row's neighbours in the adjacent planes are being swept by the
// neighbouring XCDs at the same time and are still in the last-level cache).
struct WideSched {
  int64_t first, end;
  int step;
};

__device__ inline WideSched wide_sched(int64_t groups, int spx) {
  const int G = gridDim.x;
  if (spx < 0 && (G & 7) == 0) {
    const int gx = G >> 3;
    return {(int64_t)(blockIdx.x & 7) * gx + (blockIdx.x >> 3), groups, G};
  }
  if ((G & 7) == 0 && spx > 0 && ((G >> 3) % spx) == 0) {
    const int gx = G >> 3;
    const int team = gx / spx;
    const int xcd = blockIdx.x & 7, w = blockIdx.x >> 3;
    const int stream = xcd * spx + w / team, member = w % team;
    const int64_t ns = 8ll * spx;
    const int64_t s0 = groups * stream / ns, s1 = groups * (stream + 1) / ns;
    return {s0 + member, s1, team};
  }
  const int lb = logical_block_w();
  return {groups * lb / G, groups * (lb + 1) / G, 1};
}

template <int LW, int V, class Op>
__global__ void __launch_bounds__(kBlock) k_wide(int n, int W, int spx, const int* __restrict__ rp,
                                                 const int* __restrict__ ci, Op op,
                                                 const BatchHead* __restrict__ head, double* __restrict__ partials) {
  if ((head && head->ndone >= head->W) || n <= 0) return;
  using PT = typename Op::PT;
  using VT = typename Op::VT;
  using GT = typename Op::GT;
  constexpr int RB = kBlock / LW;
  constexpr int U = 8;
  constexpr int NR = Op::NRED > 0 ? Op::NRED : 1;
  const int lr = threadIdx.x / LW, c0 = (threadIdx.x & (LW - 1)) * V;
  const bool live = c0 < W;
  const int cc0 = min(c0, W - V);  // lanes past the last column load a valid one and store nothing
  const int64_t groups = ((int64_t)n + RB - 1) / RB;
  const WideSched sc = wide_sched(groups, spx);
  double d[NR * V] = {};
  const auto cs = op.template cols<V>(cc0);
  // row pointers of the next row group are loaded one iteration ahead; the
  // entries of a row are loaded only where they exist (no loads past the
  // row's end), column indices first so that the U gathers go out together
  int k0 = 0, k1 = 0;
  if (sc.first < sc.end) {
    const int r = (int)min<int64_t>(sc.first * RB + lr, n - 1);
    k0 = rp[r];
    k1 = rp[r + 1];
  }
  for (int64_t g = sc.first; g < sc.end; g += sc.step) {
    const int row = (int)(g * RB + lr);
    const int rn = min(row + sc.step * RB, n - 1);
    const int kn0 = rp[rn], kn1 = rp[rn + 1];
    GT xo[V];
    if constexpr (Op::kOwn) ldv<V>(op.gv, (int64_t)min(row, n - 1) * W + cc0, xo);
    const auto in = op.template row_in<V>(min(row, n - 1), cc0, cs, xo);
    PT s[V] = {};
    if (row < n && live) {
      for (int kb = k0; kb < k1; kb += U) {
        int cols[U];
#pragma unroll
        for (int e = 0; e < U; ++e)
          if (kb + e < k1) cols[e] = ci[kb + e];
        PT pr[U][V];
#pragma unroll
        for (int e = 0; e < U; ++e) {
          if (kb + e < k1) {
            VT a[V];
            GT x[V];
            vals_at<Op::kSys, V>(op.v, kb + e, c0, W, a);
            ldv<V>(op.gv, (int64_t)cols[e] * W + c0, x);
#pragma unroll
            for (int u = 0; u < V; ++u) pr[e][u] = Op::mul(a[u], x[u]);
          }
        }
#pragma unroll
        for (int e = 0; e < U; ++e)
          if (kb + e < k1)
#pragma unroll
            for (int u = 0; u < V; ++u) s[u] += pr[e][u];
      }
      op.template epi<V>(row, c0, s, in, cs, d);
    }
    k0 = kn0;
    k1 = kn1;
  }
  publish_w<LW, V, Op::NRED>(d, W, partials);
}

// Instrumented launches (amg_instrument) of the batched solve: the done
// state of the batch (every column finished) is copied into the record
// before the event pair, so launches that return at once are left out.
__global__ void k_wsnap_done(const BatchHead* head, int* dst) {
  if (threadIdx.x == 0) dst[0] = head->ndone >= head->W ? 1 : 0;
}

struct WInstScope {
  Hierarchy& H;
  hipStream_t s;
  bool on;
  WInstScope(Hierarchy& h, int kid, int level, hipStream_t st) : H(h), s(st) {
    on = H.inst.kernel == kid && (H.inst.level == level || H.inst.level < 0) &&
         2 * (H.inst.used + 1) <= (int)H.inst.ev.size();
    if (on) {
      hipLaunchKernelGGL(k_wsnap_done, dim3(1), dim3(64), 0, s, H.bt.head.p, H.inst.was_done.p + H.inst.used);
      AMG_HIP(hipEventRecord(H.inst.ev[2 * H.inst.used], s));
    }
  }
  // closes the timed range (at most once)
  void end() {
    if (on) {
      (void)hipEventRecord(H.inst.ev[2 * H.inst.used + 1], s);
      ++H.inst.used;
      on = false;
    }
  }
  ~WInstScope() { end(); }
};

// ------------------------------------------------- elementwise (FP64 CG)

// r = b, x = 0, <b, b> per column
template <int LW>
__global__ void __launch_bounds__(kBlock) k_winit(int n, int W, const double* __restrict__ b, double* __restrict__ r,
                                                  double* __restrict__ x, double* __restrict__ partials) {
  constexpr int RB = kBlock / LW;
  const int lr = threadIdx.x / LW, c = threadIdx.x & (LW - 1);
  const int64_t groups = ((int64_t)n + RB - 1) / RB;
  const int lb = logical_block_w();
  const int g0 = (int)(groups * lb / gridDim.x), g1 = (int)(groups * (lb + 1) / gridDim.x);
  double d[1] = {0.0};
  for (int g = g0; g < g1; ++g) {
    const int row = g * RB + lr;
    if (row < n && c < W) {
      const int64_t e = (int64_t)row * W + c;
      const double bi = b[e];
      r[e] = bi;
      x[e] = 0.0;
      d[0] += bi * bi;
    }
  }
  publish_w<LW, 1, 1>(d, W, partials);
}

// Active columns: x += alpha p, r -= alpha q, x0 = sw o r, <r, r>.
template <int LW, bool SYS, class T>
__global__ void __launch_bounds__(kBlock) k_wupdate(int n, int W, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ p, const double* __restrict__ q,
                                                    const T* __restrict__ sw, T* __restrict__ x0,
                                                    const WCtl* __restrict__ ctl, const BatchHead* __restrict__ head,
                                                    double* __restrict__ partials) {
  if (head->ndone >= head->W) return;
  constexpr int RB = kBlock / LW;
  const int lr = threadIdx.x / LW, c = threadIdx.x & (LW - 1);
  const int64_t groups = ((int64_t)n + RB - 1) / RB;
  const int lb = logical_block_w();
  const int g0 = (int)(groups * lb / gridDim.x), g1 = (int)(groups * (lb + 1) / gridDim.x);
  const bool act = c < W && !ctl[c < W ? c : 0].done;
  const double alpha = c < W ? ctl[c].alpha : 0.0;
  double d[1] = {0.0};
  for (int g = g0; g < g1; ++g) {
    const int row = g * RB + lr;
    if (row < n && act) {
      const int64_t e = (int64_t)row * W + c;
      x[e] = x[e] + alpha * p[e];
      const double ri = r[e] - alpha * q[e];
      r[e] = ri;
      x0[e] = row_at<SYS>(sw, row, c, W) * (T)ri;
      d[0] += ri * ri;
    }
  }
  publish_w<LW, 1, 1>(d, W, partials);
}

// x0 = sw o r (start of a solve or restart)
template <int LW, bool SYS, class T>
__global__ void __launch_bounds__(kBlock) k_wswmul(int n, int W, const T* __restrict__ sw,
                                                   const double* __restrict__ r, T* __restrict__ x0) {
  constexpr int RB = kBlock / LW;
  const int lr = threadIdx.x / LW, c = threadIdx.x & (LW - 1);
  const int64_t groups = ((int64_t)n + RB - 1) / RB;
  const int lb = logical_block_w();
  const int g0 = (int)(groups * lb / gridDim.x), g1 = (int)(groups * (lb + 1) / gridDim.x);
  for (int g = g0; g < g1; ++g) {
    const int row = g * RB + lr;
    if (row < n && c < W) {
      const int64_t e = (int64_t)row * W + c;
      x0[e] = row_at<SYS>(sw, row, c, W) * (T)r[e];
    }
  }
}

// Dense coarsest solve per column: x[i][c] = sum_j inv_c[j][i] b[j][c].
template <bool SYS, class T>
__global__ void __launch_bounds__(kBlock) k_wcoarse(int n, int m, int W, const T* __restrict__ inv,
                                                    const T* __restrict__ b, T* __restrict__ x,
                                                    const BatchHead* __restrict__ head) {
  if (head && head->ndone >= head->W) return;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * W) return;
  const int i = (int)(t / W), c = (int)(t % W);
  const T* iv = inv + (SYS ? (int64_t)c * m * m : 0);
  T s = 0;
  for (int j = 0; j < n; ++j) s += iv[(int64_t)j * m + i] * b[(int64_t)j * W + c];
  x[t] = s;
}

// ----------------------------------------------------- finalize (per column)

template <int NV>
__device__ inline void wfold(const double* __restrict__ partials, int W, int np, int c, double (&tot)[NV]) {
  __shared__ double red[NV][kWFin / 64];
  double acc[NV];
#pragma unroll
  for (int m = 0; m < NV; ++m) {
    const double* src = partials + ((int64_t)m * W + c) * np;
    double s = 0.0;
    for (int b0 = 0; b0 < np; b0 += kWFin * 8) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = b0 + threadIdx.x + u * kWFin;
        t[u] = b < np ? src[b] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) s += t[u];
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
      for (int k = 1; k < kWFin / 64; ++k) s += red[m][k];
      tot[m] = s;
    }
  }
}

__device__ inline void finish_column(WCtl& cc, BatchHead* head, int state) {
  cc.state = state;
  cc.done = 1;
  atomicAdd(&head->ndone, 1);
}

__global__ void k_whead_reset(BatchHead* head, int W, int maxiter, int flexible) {
  head->ndone = 0;
  head->W = W;
  head->maxiter = maxiter;
  head->flexible = flexible;
}

__global__ void __launch_bounds__(kWFin) k_wfin_init(WCtl* ctl, BatchHead* head, const double* __restrict__ partials,
                                                     int W, int np, double tol) {
  const int c = blockIdx.x;
  double t[1];
  wfold<1>(partials, W, np, c, t);
  if (threadIdx.x != 0) return;
  WCtl& cc = ctl[c];
  const double bb = t[0];
  cc.bb = bb;
  cc.thresh = (tol * tol) * bb;
  cc.iters = 0;
  cc.state = 0;
  cc.done = 0;
  cc.first = 1;
  cc.restarts = 0;
  cc.trr = 0.0;
  cc.rr = bb;
  cc.beta = 0.0;
  if (bb == 0.0) finish_column(cc, head, 3);
  else if (!(bb == bb)) finish_column(cc, head, -1);
  else if (head->maxiter <= 0) finish_column(cc, head, 2);
}

__global__ void __launch_bounds__(kWFin) k_wfin_alpha(WCtl* ctl, BatchHead* head, const double* __restrict__ partials,
                                                      int W, int np) {
  if (head->ndone >= head->W) return;
  const int c = blockIdx.x;
  if (ctl[c].done) return;
  double t[1];
  wfold<1>(partials, W, np, c, t);
  if (threadIdx.x != 0) return;
  WCtl& cc = ctl[c];
  const double pq = t[0];
  cc.pq = pq;
  cc.first = 0;
  if (!(pq > 0.0)) finish_column(cc, head, -1);
  else cc.alpha = cc.rz / pq;
}

__global__ void __launch_bounds__(kWFin) k_wfin_update(WCtl* ctl, BatchHead* head,
                                                       const double* __restrict__ partials, int W, int np) {
  if (head->ndone >= head->W) return;
  const int c = blockIdx.x;
  if (ctl[c].done) return;
  double t[1];
  wfold<1>(partials, W, np, c, t);
  if (threadIdx.x != 0) return;
  WCtl& cc = ctl[c];
  const double rr = t[0];
  cc.rr = rr;
  cc.iters += 1;
  if (rr <= cc.thresh) finish_column(cc, head, 1);
  else if (!(rr == rr)) finish_column(cc, head, -1);
  else if (cc.iters >= head->maxiter) finish_column(cc, head, 2);
}

template <int NV>
__global__ void __launch_bounds__(kWFin) k_wfin_beta(WCtl* ctl, BatchHead* head, const double* __restrict__ partials,
                                                     int W, int np) {
  if (head->ndone >= head->W) return;
  const int c = blockIdx.x;
  if (ctl[c].done) return;
  double t[NV];
  wfold<NV>(partials, W, np, c, t);
  if (threadIdx.x != 0) return;
  WCtl& cc = ctl[c];
  const double rzn = t[0];
  const double zq = NV > 1 ? t[NV - 1] : 0.0;
  if (cc.first) cc.beta = 0.0;
  else if (head->flexible) cc.beta = -zq / cc.pq;
  else cc.beta = rzn / cc.rz;
  cc.rz = rzn;
  cc.zq = zq;
  if (!(rzn > 0.0)) finish_column(cc, head, -1);
}

__global__ void __launch_bounds__(kWFin) k_wfin_trr(WCtl* ctl, const double* __restrict__ partials, int W, int np) {
  const int c = blockIdx.x;
  double t[1];
  wfold<1>(partials, W, np, c, t);
  if (threadIdx.x == 0) ctl[c].trr = t[0];
}

// Columns flagged in mask restart from their true residual.
__global__ void k_wrestart(WCtl* ctl, BatchHead* head, const int* __restrict__ mask, int W) {
  int nre = 0;
  for (int c = 0; c < W; ++c)
    if (mask[c]) {
      ctl[c].done = 0;
      ctl[c].state = 0;
      ctl[c].first = 1;
      ctl[c].restarts += 1;
      ++nre;
    }
  head->ndone -= nre;
}

// Pattern gradients: systems -> per system; right-hand sides -> summed over
// columns in ascending order (the gradient of a loss over all columns with
// respect to the shared values).
template <bool SYS>
__global__ void __launch_bounds__(kBlock) k_wpattern_grad(int n, int W, const int* __restrict__ rp,
                                                          const int* __restrict__ ci, const double* __restrict__ lam,
                                                          const double* __restrict__ x, double* __restrict__ g) {
  const int row = blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  for (int k = rp[row]; k < rp[row + 1]; ++k) {
    const int j = ci[k];
    if constexpr (SYS) {
      for (int c = lane; c < W; c += 64)
        g[(int64_t)k * W + c] = -(lam[(int64_t)row * W + c] * x[(int64_t)j * W + c]);
    } else {
      if (lane == 0) {
        double s = 0.0;
        for (int c = 0; c < W; ++c) s += -(lam[(int64_t)row * W + c] * x[(int64_t)j * W + c]);
        g[k] = s;
      }
    }
  }
}

// --------------------------------------------------------------- dispatch

#define AMG_DISPATCH_LW(lw, ...)                            \
  switch (lw) {                                             \
    case 1: { constexpr int LW = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int LW = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int LW = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int LW = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int LW = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int LW = 32; __VA_ARGS__; } break; \
    default: { constexpr int LW = 64; __VA_ARGS__; } break; \
  }

// Staged wide sweep: per block of `br` rows, the workgroup loads the row
// pointers, the column indices and (shared-value form) the values with
// coalesced loads into LDS; each group of LW lanes then reads its row's
// entries from LDS and gathers x[j][c0 .. c0+V) for its columns.  For a
// square operator the block also stages the window of the gathered vector
// around its rows (rows r0 - 1 .. r0 + br, when it fits kWinBytes): entries
// whose column falls in it (the diagonal and its neighbours) are read from
// LDS, the others from global memory.  Blocks are scheduled like the row
// groups of k_wide (streams per XCD); the grid is the number of workgroups
// that are resident at once.
constexpr int kWCap = 1024;       // staged entries per block
constexpr int kWCapSq = 512;      // staged entries per block of a square operator (with its window)
constexpr int kWinBytes = 17408;  // staged window of the gathered vector

// Rows per block for which the window of a W-column FP64 vector fits.
inline int window_rows(int W) { return std::max(1, kWinBytes / (8 * std::max(W, 1)) - 2); }

template <int LW, int V, class Op>
__global__ void __launch_bounds__(kBlock) k_wide_st(int n, int W, int spx, int br, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, Op op,
                                                    const BatchHead* __restrict__ head,
                                                    double* __restrict__ partials) {
  if ((head && head->ndone >= head->W) || n <= 0) return;
  using PT = typename Op::PT;
  using VT = typename Op::VT;
  using GT = typename Op::GT;
  constexpr bool SYS = Op::kSys;
  constexpr int RB = kBlock / LW;
  constexpr int CAP = Op::kSquare ? kWCapSq : kWCap;
  constexpr int U = CAP / kBlock;
  constexpr int NR = Op::NRED > 0 ? Op::NRED : 1;
  constexpr int WE = Op::kSquare ? kWinBytes / (int)sizeof(GT) : 1;
  __shared__ int s_rp[kBlock + 1];
  __shared__ int s_ci[CAP];
  __shared__ VT s_v[SYS ? 1 : CAP];
  __shared__ __align__(16) GT s_g[WE];
  const int lr = threadIdx.x / LW, c0 = (threadIdx.x & (LW - 1)) * V;
  const bool live = c0 < W;
  const int cc0 = min(c0, W - V);
  const auto cs = op.template cols<V>(cc0);
  const int64_t blocks = ((int64_t)n + br - 1) / br;
  const WideSched sc = wide_sched(blocks, spx);
  const bool win = Op::kSquare && (int64_t)(br + 2) * W <= WE;
  double d[NR * V] = {};
  for (int64_t blk = sc.first; blk < sc.end; blk += sc.step) {
    const int r0 = (int)(blk * br);
    __syncthreads();  // the previous block's entries and window have been read
    for (int t = threadIdx.x; t <= br; t += kBlock) s_rp[t] = rp[min(r0 + t, n)];
    if (win) {
      // window row wr holds gathered row r0 - 1 + wr (clamped into the
      // operand: rows outside it are never referenced)
      const int nv = (br + 2) * W / V;
      for (int t = threadIdx.x; t < nv; t += kBlock) {
        const int wr = t * V / W, cw = t * V - wr * W;
        const int rr = min(max(r0 - 1 + wr, 0), n - 1);
        GT x[V];
        ldv<V>(op.gv, (int64_t)rr * W + cw, x);
        stv<V>(s_g, (int64_t)wr * W + cw, x);
      }
    }
    __syncthreads();
    const int k0 = s_rp[0], nk = s_rp[br] - k0;
    if (nk > 0) {
      int cv[U];
      VT vv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int jj = k0 + min((int)threadIdx.x + u * kBlock, nk - 1);
        cv[u] = ci[jj];
        if constexpr (!SYS) vv[u] = op.v[jj];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = threadIdx.x + u * kBlock;
        if (j < nk) {
          s_ci[j] = cv[u];
          if constexpr (!SYS) s_v[j] = vv[u];
        }
      }
    }
    __syncthreads();
    for (int q = lr; q < br; q += RB) {
      const int row = r0 + q;
      // the row's own operands: before the gathers (their loads overlap), or
      // for operators with many of them after (kLateRow: not live in
      // registers across the gather loop, one more workgroup per CU)
      const int rowc = min(row, n - 1);
      auto row_operands = [&]() {
        GT xo[V];
        if constexpr (Op::kOwn) {
          if (win) ldv<V>(s_g, (int64_t)(rowc - r0 + 1) * W + cc0, xo);
          else ldv<V>(op.gv, (int64_t)rowc * W + cc0, xo);
        }
        return op.template row_in<V>(rowc, cc0, cs, xo);
      };
      decltype(row_operands()) in_early{};
      if constexpr (!Op::kLateRow) in_early = row_operands();
      PT acc[V] = {};
      if (row < n && live) {
        const int a = s_rp[q] - k0, e = s_rp[q + 1] - k0;
        for (int kb = a; kb < e; kb += 8) {
          PT pr[8][V];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int k = kb + u;
            if (k < e) {
              VT val[V];
              GT x[V];
              if constexpr (SYS) {
                ldv<V, true>(op.v, (int64_t)(k0 + k) * W + c0, val);
              } else {
                const VT a1 = s_v[k];
#pragma unroll
                for (int w = 0; w < V; ++w) val[w] = a1;
              }
              const int col = s_ci[k];
              const int wr = col - r0 + 1;
              if (win && wr >= 0 && wr < br + 2) ldv<V>(s_g, (int64_t)wr * W + c0, x);
              else ldv<V>(op.gv, (int64_t)col * W + c0, x);
#pragma unroll
              for (int w = 0; w < V; ++w) pr[u][w] = Op::mul(val[w], x[w]);
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (kb + u < e)
#pragma unroll
              for (int w = 0; w < V; ++w) acc[w] += pr[u][w];
        }
        if constexpr (Op::kLateRow) op.template epi<V>(row, c0, acc, row_operands(), cs, d);
        else op.template epi<V>(row, c0, acc, in_early, cs, d);
      }
    }
  }
  if constexpr (Op::NRED > 0) {
    // the reduction reuses the window's LDS (every operator with a
    // reduction is square, and its window holds at least NRED*kBlock*V doubles)
    static_assert(Op::kSquare && (int64_t)WE * sizeof(GT) >= (int64_t)Op::NRED * kBlock * V * 8,
                  "window too small for the reduction");
    __syncthreads();
    publish_w<LW, V, Op::NRED>(d, W, partials, reinterpret_cast<double*>(s_g));
  }
}

// Workgroups of `kernel` resident at once on the device (a multiple of 8).
int resident_grid(const void* kernel) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  static int ncu = 0;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(kernel);
  if (it != cache.end()) return it->second;
  if (!ncu) {
    int dev = 0;
    AMG_HIP(hipGetDevice(&dev));
    AMG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  }
  int per_cu = 0;
  AMG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0));
  int g = std::max(1, per_cu) * std::max(1, ncu);
  g = std::max(8, std::min(g, kWGrid) / 8 * 8);
  cache[kernel] = g;
  return g;
}

// Columns per lane of a wide sweep: as many as make a 16-byte access of the
// gathered vector (two FP64 or four FP32 columns) and divide the width, at
// most vmax (1 for vectors not aligned to 16 bytes); and the lanes per row.
inline int wide_v(int W, int elem_bytes, int vmax) {
  int v = std::min(vmax, 16 / elem_bytes);
  while (v > 1 && W % v != 0) v >>= 1;
  return std::max(v, 1);
}
inline int wide_lanes(int W, int V) { return pow2_ceil((W + V - 1) / V); }

// br > 0: staged kernel with br rows per block; 0: direct kernel.
template <int V, class Op>
int wsweep_v(int spx, int br, int n, int W, const int* rp, const int* ci, const Op& op, const BatchHead* head,
             double* partials, hipStream_t s) {
  const int LWv = wide_lanes(W, V);
  int grid = 0;
  if (br > 0) {
    AMG_DISPATCH_LW(LWv, {
      const void* kp = reinterpret_cast<const void*>(&k_wide_st<LW, V, Op>);
      grid = std::min<int64_t>(resident_grid(kp), std::max<int64_t>(8, ((int64_t)n + br - 1) / br / 8 * 8));
      hipLaunchKernelGGL((k_wide_st<LW, V, Op>), dim3(grid), dim3(kBlock), 0, s, n, W, spx, br, rp, ci, op, head,
                         partials);
    });
  } else {
    grid = wide_grid(n, LWv);
    AMG_DISPATCH_LW(LWv, hipLaunchKernelGGL((k_wide<LW, V, Op>), dim3(grid), dim3(kBlock), 0, s, n, W, spx, rp, ci,
                                            op, head, partials));
  }
  return grid;
}

// A wide sweep with the columns per lane wide_v gives (every vector of the
// operator aligned to 16 bytes unless vmax = 1).
template <class Op>
int wsweep(int vmax, int spx, int br, int n, int W, const int* rp, const int* ci, const Op& op,
           const BatchHead* head, double* partials, hipStream_t s) {
  constexpr int eb = (int)sizeof(typename Op::GT);
  const int v = wide_v(W, eb, vmax);
  if constexpr (eb == 4) {
    if (v == 4) return wsweep_v<4>(spx, br, n, W, rp, ci, op, head, partials, s);
  }
  if (v >= 2) return wsweep_v<2>(spx, br, n, W, rp, ci, op, head, partials, s);
  return wsweep_v<1>(spx, br, n, W, rp, ci, op, head, partials, s);
}

std::vector<int> host_rows(const DBuf<int>& rp, int n) {
  std::vector<int> h(n + 1);
  AMG_HIP(hipMemcpy(h.data(), rp.p, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
  return h;
}

// Rows per staged block for a matrix: the largest power of two from the
// lane group's rows per step up to min(256, max_rows) whose blocks all fit
// `cap` staged entries; 0 when even the smallest does not (direct kernel).
int wide_block_rows(const std::vector<int>& rp, int n, int LWv, int max_rows, int cap) {
  const int rb = kBlock / LWv;
  int best = 0;
  for (int br = rb; br <= kBlock && (br == rb || br <= max_rows); br <<= 1) {
    int mx = 0;
    for (int r0 = 0; r0 < n; r0 += br) mx = std::max(mx, rp[std::min(r0 + br, n)] - rp[r0]);
    if (mx > cap) break;
    best = br;
  }
  return best;
}

template <class T>
struct WB;
template <>
struct WB<double> {
  static double* x(BatchLevel& B) { return B.x64.p; }
  static double* b(BatchLevel& B) { return B.b64.p; }
  static double* r(BatchLevel& B) { return B.r64.p; }
  static const double* v(Level& L) { return L.v.p; }
  static const double* sw(Level& L) { return L.sw.p; }
  static const double* inv(Coarse& C) { return C.inv.p; }
};
template <>
struct WB<float> {
  static float* x(BatchLevel& B) { return B.x32.p; }
  static float* b(BatchLevel& B) { return B.b32.p; }
  static float* r(BatchLevel& B) { return B.r32.p; }
  static const float* v(Level& L) { return L.v32.p; }
  static const float* sw(Level& L) { return L.sw32.p; }
  static const float* inv(Coarse& C) { return C.inv32.p; }
};

template <bool SYS, class T>
void w_restrict(Hierarchy& H, Level& L, int Vc, int spx, int br, int W, const T* r, T* bc, const T* swc, T* xc,
                hipStream_t s) {
  const BatchHead* hd = H.bt.head.p;
  if constexpr (std::is_same<T, double>::value) {
    wsweep(Vc, spx, br, L.nagg, W, L.rrp.p, L.rci.p, WRestrict<SYS, double, T>{L.rv.p, r, bc, swc, xc, W}, hd, nullptr, s);
  } else if (H.bf16()) {
    wsweep(Vc, spx, br, L.nagg, W, L.rrp.p, L.rci.p, WRestrict<SYS, uint16_t, T>{L.rbf.p, r, bc, swc, xc, W}, hd, nullptr,
           s);
  } else {
    wsweep(Vc, spx, br, L.nagg, W, L.rrp.p, L.rci.p, WRestrict<SYS, float, T>{L.rv32.p, r, bc, swc, xc, W}, hd, nullptr, s);
  }
}

template <bool SYS, class T>
void w_prolong(Hierarchy& H, Level& L, int Vc, int spx, int br, int W, const T* xc, T* x, hipStream_t s) {
  const BatchHead* hd = H.bt.head.p;
  if constexpr (std::is_same<T, double>::value) {
    wsweep(Vc, spx, br, L.n, W, L.prp.p, L.pci.p, WProlong<SYS, double, T>{L.pv.p, xc, x, W}, hd, nullptr, s);
  } else if (H.bf16()) {
    wsweep(Vc, spx, br, L.n, W, L.prp.p, L.pci.p, WProlong<SYS, uint16_t, T>{L.pbf.p, xc, x, W}, hd, nullptr, s);
  } else {
    wsweep(Vc, spx, br, L.n, W, L.prp.p, L.pci.p, WProlong<SYS, float, T>{L.pv32.p, xc, x, W}, hd, nullptr, s);
  }
}

// One batched V(1,1) cycle: level-0 rhs r0 [n][W] (FP64) -> z0 (FP64), with
// the level-0 pre-smoothed iterate already written; red = 1 or 2 emits the
// per-column <r,z> (and <z,q>) partials and the beta finalize.
template <bool SYS, class T>
void wvcycle(Hierarchy& H, int W, const double* r0, double* z0, const double* q, int red, hipStream_t s) {
  Batch& B = H.bt;
  const int Vc = 4;  // columns per lane: the widest the operands allow
  const int nl = (int)H.lv.size();
  const BatchHead* hd = B.head.p;
  double* part = B.partials.p;
  Coarse& C = H.co;
  for (int l = 0; l < nl - 1; ++l) {
    Level& L = H.lv[l];
    BatchLevel& BL = B.lv[l];
    {
      WInstScope is(H, KID_PRE, l, s);
      if (l == 0)
        wsweep(Vc, BL.spxA, BL.brA, L.n, W, L.rp.p, L.ci.p,
               WResid<SYS, T, double>{WB<T>::v(L), r0, WB<T>::x(BL), WB<T>::r(BL), W}, hd, nullptr, s);
      else
        wsweep(Vc, BL.spxA, BL.brA, L.n, W, L.rp.p, L.ci.p,
               WResid<SYS, T, T>{WB<T>::v(L), WB<T>::b(BL), WB<T>::x(BL), WB<T>::r(BL), W}, hd, nullptr, s);
    }
    Level& Ln = H.lv[l + 1];
    BatchLevel& BN = B.lv[l + 1];
    const bool coarsest = (l + 1 == nl - 1);
    WInstScope is(H, KID_RESTRICT, l, s);
    w_restrict<SYS, T>(H, L, Vc, BL.spxR, BL.brR, W, WB<T>::r(BL), WB<T>::b(BN), coarsest ? nullptr : WB<T>::sw(Ln),
                       coarsest ? nullptr : WB<T>::x(BN), s);
  }
  {
    WInstScope is(H, KID_COARSE, nl - 1, s);
    BatchLevel& BC = B.lv[nl - 1];
    const int64_t nt = (int64_t)C.n * W;
    hipLaunchKernelGGL((k_wcoarse<SYS, T>), dim3((int)((nt + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, C.n, C.m,
                       W, WB<T>::inv(C), WB<T>::b(BC), WB<T>::x(BC), hd);
  }
  T* res = WB<T>::x(B.lv[nl - 1]);
  for (int l = nl - 2; l >= 0; --l) {
    Level& L = H.lv[l];
    BatchLevel& BL = B.lv[l];
    {
      WInstScope is(H, KID_PROLONG, l, s);
      w_prolong<SYS, T>(H, L, Vc, BL.spxP, BL.brP, W, res, WB<T>::x(BL), s);
    }
    const T* vv = WB<T>::v(L);
    const T* sw = WB<T>::sw(L);
    WInstScope is(H, KID_POST, l, s);
    if (l == 0) {
      int np = 0;
      if (red == 2)
        np = wsweep(Vc, BL.spxA, BL.brA, L.n, W, L.rp.p, L.ci.p, WPost<SYS, T, double, double, 2>{vv, sw, r0, WB<T>::x(BL), z0, q, W},
                    hd, part, s);
      else if (red == 1)
        np = wsweep(Vc, BL.spxA, BL.brA, L.n, W, L.rp.p, L.ci.p, WPost<SYS, T, double, double, 1>{vv, sw, r0, WB<T>::x(BL), z0, q, W},
                    hd, part, s);
      else
        wsweep(Vc, BL.spxA, BL.brA, L.n, W, L.rp.p, L.ci.p, WPost<SYS, T, double, double, 0>{vv, sw, r0, WB<T>::x(BL), z0, q, W}, hd,
               nullptr, s);
      is.end();
      if (red == 2)
        hipLaunchKernelGGL(k_wfin_beta<2>, dim3(W), dim3(kWFin), 0, s, B.ctl.p, B.head.p, part, W, np);
      else if (red == 1)
        hipLaunchKernelGGL(k_wfin_beta<1>, dim3(W), dim3(kWFin), 0, s, B.ctl.p, B.head.p, part, W, np);
    } else {
      wsweep(Vc, BL.spxA, BL.brA, L.n, W, L.rp.p, L.ci.p,
             WPost<SYS, T, T, T, 0>{vv, sw, WB<T>::b(BL), WB<T>::x(BL), WB<T>::r(BL), nullptr, W}, hd, nullptr, s);
      res = WB<T>::r(BL);
    }
  }
  AMG_HIP(hipGetLastError());
}

void ensure_batch(Hierarchy& H, int W) {
  Batch& B = H.bt;
  if (B.W == W && B.ctl.p) return;
  const int64_t n = H.n;
  B.r.alloc(n * W);
  B.z.alloc(n * W);
  B.p.alloc(n * W);
  B.p2.alloc(n * W);
  B.q.alloc(n * W);
  B.partials.alloc((int64_t)2 * W * kWGrid + 64);
  B.ctl.alloc(W);
  B.head.alloc(1);
  B.mask.alloc(W);
  if (B.h_ctl) AMG_HIP(hipHostFree(B.h_ctl));
  if (!B.h_head) AMG_HIP(hipHostMalloc((void**)&B.h_head, sizeof(BatchHead), hipHostMallocDefault));
  if (B.h_mask) AMG_HIP(hipHostFree(B.h_mask));
  AMG_HIP(hipHostMalloc((void**)&B.h_ctl, sizeof(WCtl) * W, hipHostMallocDefault));
  AMG_HIP(hipHostMalloc((void**)&B.h_mask, sizeof(int) * W, hipHostMallocDefault));
  AMG_HIP(hipMemset(B.ctl.p, 0, sizeof(WCtl) * W));
  B.lv.clear();
  B.lv.resize(H.lv.size());
  B.tuned_W = 0;
  for (size_t l = 0; l < H.lv.size(); ++l) {
    const int64_t nl = (int64_t)H.lv[l].n * W;
    if (H.fp32()) {
      B.lv[l].x32.alloc(nl);
      B.lv[l].b32.alloc(nl);
      B.lv[l].r32.alloc(nl);
    } else {
      B.lv[l].x64.alloc(nl);
      B.lv[l].b64.alloc(nl);
      B.lv[l].r64.alloc(nl);
    }
  }
  B.W = W;
}

void read_batch(Hierarchy& H, int W, hipStream_t s) {
  AMG_HIP(hipMemcpyAsync(H.bt.h_head, H.bt.head.p, sizeof(BatchHead), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipMemcpyAsync(H.bt.h_ctl, H.bt.ctl.p, sizeof(WCtl) * W, hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------ stream-count tuner
//
// The number of row streams per XCD of each wide sweep (A, P and R of every
// level) is a locality choice: it does not change which operations a row
// performs.  Without autotuning every workgroup takes a contiguous range;
// with it, each candidate is timed with HIP events on the level's own
// operands and the fastest is kept and recorded in the tuning cache.

template <class Op>
double time_wide(int Vc, int spx, int br, int n, int W, const int* rp, const int* ci, const Op& op, hipStream_t s,
                 hipEvent_t e0, hipEvent_t e1) {
  wsweep(Vc, spx, br, n, W, rp, ci, op, nullptr, nullptr, s);
  AMG_HIP(hipEventRecord(e0, s));
  constexpr int reps = 3;
  for (int r = 0; r < reps; ++r) wsweep(Vc, spx, br, n, W, rp, ci, op, nullptr, nullptr, s);
  AMG_HIP(hipEventRecord(e1, s));
  AMG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
  return ms / reps;
}

// Candidate stream counts: divisors of the per-XCD workgroup count (the
// launch's grid depends on the kernel's residency, so the candidates are
// taken for the smallest resident grid that divides into 8 XCDs evenly).
std::vector<int> spx_candidates() {
  std::vector<int> out{0, -1};
  for (int spx : {64, 32, 16, 8, 4, 2, 1}) out.push_back(spx);
  return out;
}

// Picks the kernel form (staged with `br` rows per block, or direct) and the
// stream count of one wide sweep; returns the stream count and sets br.
template <class Op>
int pick_spx(Hierarchy& H, const char* kind, int W, int& br, int n, int nnz, const int* rp, const int* ci,
             const Op& op, hipStream_t s) {
  char key[160];
  std::snprintf(key, sizeof key, "wide%s:n%d:nnz%d:W%d:S%d:p%d:t%d:br%d", kind, n, nnz, W, H.S, H.prm.vcycle_prec,
                H.fp32() && H.prm.transfer_bf16, br);
  Shape sh;
  if (tune_lookup(key, &sh)) {
    br = sh.g ? br : 0;
    return sh.stream;
  }
  const int Vc = 4;
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
  int best = 0, best_br = 0;
  double tbest = 1e300;
  for (int form : {br, 0}) {  // staged (when the blocks fit), then direct
    for (int spx : spx_candidates()) {
      const double t = time_wide(Vc, spx, form, n, W, rp, ci, op, s, e0, e1);
      if (t < tbest) {
        tbest = t;
        best = spx;
        best_br = form;
      }
    }
    if (br == 0) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  sh = Shape{};
  sh.stream = best;
  sh.g = best_br ? 1 : 0;
  tune_record(key, sh);
  br = best_br;
  return best;
}

template <bool SYS, class T>
void tune_wide(Hierarchy& H, int W, hipStream_t s) {
  Batch& B = H.bt;
  if (B.tuned_W == W) return;
  B.tuned_W = W;
  const int LWv = wide_lanes(W, wide_v(W, 8, 2));
  for (size_t l = 0; l < H.lv.size(); ++l) {
    BatchLevel& BL = B.lv[l];
    Level& L = H.lv[l];
    BL.spxA = BL.spxP = BL.spxR = 0;
    BL.brA = BL.brP = BL.brR = 0;
    if (l + 1 == H.lv.size()) continue;
    // A's blocks are sized so that the window of its gathered vector fits
    BL.brA = wide_block_rows(host_rows(L.rp, L.n), L.n, LWv, window_rows(W), kWCapSq);
    BL.brP = wide_block_rows(host_rows(L.prp, L.n), L.n, LWv, kBlock, kWCap);
    BL.brR = wide_block_rows(host_rows(L.rrp, L.nagg), L.nagg, LWv, kBlock, kWCap);
    // per-system values cannot be staged: the direct form is the default there
    if (SYS && !H.prm.autotune) BL.brA = BL.brP = BL.brR = 0;
  }
  if (!H.prm.autotune) return;
  const int nl = (int)H.lv.size();
  for (int l = 0; l < nl; ++l) {
    BatchLevel& BL = B.lv[l];
    T* x = WB<T>::x(BL);
    T* b = WB<T>::b(BL);
    T* r = WB<T>::r(BL);
    const int64_t len = (int64_t)H.lv[l].n * W;
    AMG_HIP(hipMemsetAsync(x, 0, sizeof(T) * len, s));
    AMG_HIP(hipMemsetAsync(b, 0, sizeof(T) * len, s));
  }
  for (int l = 0; l + 1 < nl; ++l) {
    Level& L = H.lv[l];
    BatchLevel& BL = B.lv[l];
    BatchLevel& BN = B.lv[l + 1];
    BL.spxA = pick_spx(H, "A", W, BL.brA, L.n, (int)L.nnz, L.rp.p, L.ci.p,
                       WResid<SYS, T, T>{WB<T>::v(L), WB<T>::b(BL), WB<T>::x(BL), WB<T>::r(BL), W}, s);
    if constexpr (std::is_same<T, double>::value) {
      BL.spxP = pick_spx(H, "P", W, BL.brP, L.n, (int)L.pnnz, L.prp.p, L.pci.p,
                         WProlong<SYS, double, T>{L.pv.p, WB<T>::x(BN), WB<T>::r(BL), W}, s);
      BL.spxR = pick_spx(H, "R", W, BL.brR, L.nagg, (int)L.pnnz, L.rrp.p, L.rci.p,
                         WRestrict<SYS, double, T>{L.rv.p, WB<T>::x(BL), WB<T>::b(BN), nullptr, nullptr, W}, s);
    } else if (H.bf16()) {
      BL.spxP = pick_spx(H, "P", W, BL.brP, L.n, (int)L.pnnz, L.prp.p, L.pci.p,
                         WProlong<SYS, uint16_t, T>{L.pbf.p, WB<T>::x(BN), WB<T>::r(BL), W}, s);
      BL.spxR = pick_spx(H, "R", W, BL.brR, L.nagg, (int)L.pnnz, L.rrp.p, L.rci.p,
                         WRestrict<SYS, uint16_t, T>{L.rbf.p, WB<T>::x(BL), WB<T>::b(BN), nullptr, nullptr, W}, s);
    } else {
      BL.spxP = pick_spx(H, "P", W, BL.brP, L.n, (int)L.pnnz, L.prp.p, L.pci.p,
                         WProlong<SYS, float, T>{L.pv32.p, WB<T>::x(BN), WB<T>::r(BL), W}, s);
      BL.spxR = pick_spx(H, "R", W, BL.brR, L.nagg, (int)L.pnnz, L.rrp.p, L.rci.p,
                         WRestrict<SYS, float, T>{L.rv32.p, WB<T>::x(BL), WB<T>::b(BN), nullptr, nullptr, W}, s);
    }
  }
  AMG_HIP(hipStreamSynchronize(s));
}

template <bool SYS, class T>
amg_status solve_wide_impl(Hierarchy& H, const SolveOpts& o, const double* d_b, double* d_x, double tol, int W,
                           amg_info* info, hipStream_t caller) {
  auto t0 = std::chrono::steady_clock::now();
  ensure_batch(H, W);
  tune_wide<SYS, T>(H, W, caller);
  Batch& B = H.bt;
  Level& L0 = H.lv[0];
  const int n = H.n;
  const int LWv = pow2_ceil(W);
  const bool multi = H.lv.size() > 1;
  const int flexible = o.flexible < 0 ? ((H.fp32() || H.prm.nu_pre != H.prm.nu_post) ? 1 : 0) : o.flexible;
  if (!multi) throw Error(AMG_ERR_INVALID_ARG, "batched solves need at least two levels");
  const bool graphs = o.use_graphs != 0 && H.inst.kernel < 0;
  hipStream_t s = caller;
  if (graphs) {
    graph_stream(H);
    AMG_HIP(hipEventRecord(H.gr.ev_in, caller));
    AMG_HIP(hipStreamWaitEvent(H.gr.gs, H.gr.ev_in, 0));
    s = H.gr.gs;
    if (H.gr.key_x != d_x || H.gr.key_flex != flexible || H.gr.key_w != W) {
      H.gr.reset();
      H.gr.key_x = d_x;
      H.gr.key_flex = flexible;
      H.gr.key_w = W;
    }
  }
  double* part = B.partials.p;
  const int gw = wide_grid(n, LWv);
  hipLaunchKernelGGL(k_whead_reset, dim3(1), dim3(1), 0, s, B.head.p, W, o.maxiter, flexible);
  AMG_DISPATCH_LW(LWv, hipLaunchKernelGGL((k_winit<LW>), dim3(gw), dim3(kBlock), 0, s, n, W, d_b, B.r.p, d_x, part));
  hipLaunchKernelGGL(k_wfin_init, dim3(W), dim3(kWFin), 0, s, B.ctl.p, B.head.p, part, W, gw, tol);
  AMG_HIP(hipGetLastError());
  double* pb[2] = {B.p.p, B.p2.p};
  int cur = 0;
  int restarts = 0;
  amg_status st = AMG_OK;
  T* x0 = WB<T>::x(B.lv[0]);
  // one batched iteration (columns flagged `first` take p = z on device)
  auto iteration = [&](int c, hipStream_t stq) {
    int np;
    {
      WInstScope is(H, KID_SPMV_DOT, 0, stq);
      np = wsweep(4, B.lv[0].spxA, B.lv[0].brA, n, W, L0.rp.p, L0.ci.p,
                  WSpmvXpay<SYS>{L0.v.p, B.z.p, pb[c], pb[c ^ 1], B.q.p, B.ctl.p, W}, B.head.p, part, stq);
    }
    hipLaunchKernelGGL(k_wfin_alpha, dim3(W), dim3(kWFin), 0, stq, B.ctl.p, B.head.p, part, W, np);
    {
      WInstScope is(H, KID_CG_UPDATE, 0, stq);
      AMG_DISPATCH_LW(LWv, hipLaunchKernelGGL((k_wupdate<LW, SYS, T>), dim3(gw), dim3(kBlock), 0, stq, n, W, d_x,
                                              B.r.p, pb[c ^ 1], B.q.p, WB<T>::sw(L0), x0, B.ctl.p, B.head.p, part));
    }
    hipLaunchKernelGGL(k_wfin_update, dim3(W), dim3(kWFin), 0, stq, B.ctl.p, B.head.p, part, W, gw);
    wvcycle<SYS, T>(H, W, B.r.p, B.z.p, B.q.p, flexible ? 2 : 1, stq);
  };
  auto pair = [&](int c) {
    hipGraphExec_t& ex = H.gr.exec[c];
    if (!ex) capture_graph(s, ex, [&] {
        iteration(c, s);
        iteration(c ^ 1, s);
      });
    AMG_HIP(hipGraphLaunch(ex, s));
  };
  for (;;) {
    AMG_DISPATCH_LW(LWv, hipLaunchKernelGGL((k_wswmul<LW, SYS, T>), dim3(gw), dim3(kBlock), 0, s, n, W,
                                            WB<T>::sw(L0), B.r.p, x0));
    wvcycle<SYS, T>(H, W, B.r.p, B.z.p, B.q.p, 1, s);
    int chunk = o.check_every > 0 ? o.check_every : 4;
    int it_prev = -1;
    std::vector<double> rr_prev(W, 0.0);
    for (;;) {
      int left = chunk;
      if (graphs)
        for (; left >= 2; left -= 2) pair(cur);
      for (; left > 0; --left) {
        iteration(cur, s);
        cur ^= 1;
      }
      AMG_HIP(hipGetLastError());
      read_batch(H, W, s);
      if (B.h_head->ndone >= W) break;
      if (o.check_every <= 0) {
        // size the next chunk from the slowest active column's decay
        int next = 1;
        int maxit = 0;
        for (int c = 0; c < W; ++c) {
          const WCtl& cc = B.h_ctl[c];
          maxit = std::max(maxit, cc.iters);
          if (cc.done) continue;
          const double prev = it_prev < 0 ? cc.bb : rr_prev[c];
          const int i0 = it_prev < 0 ? 0 : it_prev;
          int nc = 4;
          if (cc.thresh <= 0.0) nc = 32;
          else if (cc.iters > i0 && prev > 0.0 && cc.rr > 0.0) {
            const double rate = std::log(cc.rr / prev) / (double)(cc.iters - i0);
            if (rate < -1e-3) nc = (int)std::min(64.0, std::ceil(std::log(cc.thresh / cc.rr) / rate));
          }
          next = std::max(next, nc);
        }
        for (int c = 0; c < W; ++c) rr_prev[c] = B.h_ctl[c].rr;
        it_prev = maxit;
        next = std::min(next, std::max(1, o.maxiter - maxit));
        chunk = std::max(1, std::min(next, 32));
      }
    }
    // true residuals of every column
    // the caller's x and b take two columns per lane only when 16-byte aligned
    const bool al = (((uintptr_t)d_x | (uintptr_t)d_b) & 15) == 0;
    const int np = wsweep(al ? 4 : 1, B.lv[0].spxA, B.lv[0].brA, n, W, L0.rp.p, L0.ci.p,
                          WTrueResid<SYS>{L0.v.p, d_x, d_b, B.r.p, W}, nullptr, part, s);
    hipLaunchKernelGGL(k_wfin_trr, dim3(W), dim3(kWFin), 0, s, B.ctl.p, part, W, np);
    read_batch(H, W, s);
    int nre = 0;
    for (int c = 0; c < W; ++c) {
      const WCtl& cc = B.h_ctl[c];
      const bool again = cc.state == 1 && cc.trr > cc.thresh && cc.restarts < 5 && cc.iters < o.maxiter;
      B.h_mask[c] = again ? 1 : 0;
      nre += again;
    }
    if (nre == 0) break;
    ++restarts;
    AMG_HIP(hipMemcpyAsync(B.mask.p, B.h_mask, sizeof(int) * W, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_wrestart, dim3(1), dim3(1), 0, s, B.ctl.p, B.head.p, B.mask.p, W);
  }
  if (graphs) {
    AMG_HIP(hipEventRecord(H.gr.ev_out, s));
    AMG_HIP(hipStreamWaitEvent(caller, H.gr.ev_out, 0));
  }
  // per-column outcome
  B.col_iters.assign(W, 0);
  B.col_status.assign(W, AMG_OK);
  B.col_relres.assign(W, 0.0);
  int maxit = 0;
  double maxrr = 0.0;
  for (int c = 0; c < W; ++c) {
    const WCtl& cc = B.h_ctl[c];
    int cs;
    if (cc.state < 0) cs = AMG_ERR_BREAKDOWN;
    else if (cc.state == 3 || cc.trr <= cc.thresh) cs = AMG_OK;
    else cs = AMG_NOT_CONVERGED;
    const double rr = cc.state == 3 ? 0.0 : (cc.bb > 0 ? std::sqrt(cc.trr / cc.bb) : 0.0);
    B.col_iters[c] = cc.iters;
    B.col_status[c] = cs;
    B.col_relres[c] = cs == AMG_ERR_BREAKDOWN ? NAN : rr;
    maxit = std::max(maxit, cc.iters);
    if (cs != AMG_ERR_BREAKDOWN) maxrr = std::max(maxrr, rr);
    if (cs == AMG_ERR_BREAKDOWN) st = AMG_ERR_BREAKDOWN;
    else if (cs == AMG_NOT_CONVERGED && st == AMG_OK) st = AMG_NOT_CONVERGED;
  }
  if (info) {
    info->iters = maxit;
    info->status = st;
    info->restarts = restarts;
    info->rel_resid = st == AMG_ERR_BREAKDOWN ? NAN : maxrr;
    info->cache_event = H.cache_event;
    info->setup_ms = H.setup_ms;
    info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

}  // namespace

// Algorithmic bytes of one launch of a batched sweep with W columns (every
// matrix array streamed once, every vector operand read once, every output
// written once).  The wide kernels sweep CSR; with S = W systems sharing the
// pattern the values, smoother weights and coarse inverses are per column
// ([entry][S]), with W right-hand sides of one matrix they are read once.
// Vectors are W columns wide.
double wide_kernel_bytes(const Hierarchy& H, int kid, int level, int flexible, int W) {
  const int nl = (int)H.lv.size();
  if (level < 0 || level >= nl || W < 1) return 0.0;
  const Level& L = H.lv[level];
  const double sys = H.S > 1 ? (double)W : 1.0;             // value streams per entry
  const double w = W;
  const double v = H.fp32() ? 4.0 : 8.0;                     // cycle values and vectors
  const double pw = H.fp32() ? (H.bf16() ? 2.0 : 4.0) : 8.0; // transfer values
  const double n = L.n, nc = L.nagg;
  auto M = [&](double nz, double rows, double vb) { return 4.0 * nz + 4.0 * (rows + 1.0) + vb * nz * sys; };
  const double bw = level == 0 ? 8.0 : v;
  const bool has_next = level + 1 < nl;
  const bool next_coarsest = level + 2 == nl;
  switch (kid) {
    // z gathered, p and q read at the row, p' = z + beta p and q' = A z + beta q written
    case KID_SPMV_DOT: return M((double)L.nnz, n, 8.0) + 40.0 * n * w;
    case KID_PRE: return M((double)L.nnz, n, v) + (bw + 2.0 * v) * n * w;
    case KID_POST: {
      const double ow = level == 0 ? 8.0 : v;
      return M((double)L.nnz, n, v) + (bw + v + ow) * n * w + v * n * sys + (level == 0 && flexible ? 8.0 * n * w : 0.0);
    }
    case KID_RESTRICT:
      if (!has_next) return 0.0;
      return M((double)L.pnnz, nc, pw) + v * n * w + v * nc * w + (next_coarsest ? 0.0 : v * nc * sys + v * nc * w);
    case KID_PROLONG:
      if (!has_next) return 0.0;
      return M((double)L.pnnz, n, pw) + v * nc * w + 2.0 * v * n * w;
    // x, r read and written, p and q read; sw read and x0 = sw o r written
    case KID_CG_UPDATE: return 48.0 * n * w + v * n * sys + v * n * w;
    case KID_XPAY: return 0.0;
    case KID_COARSE: {
      const double m = H.co.n;
      return m * m * v * sys + 2.0 * m * v * w;
    }
  }
  return 0.0;
}

// Bytes of one batched PCG iteration with every one of the W columns active.
double wide_iteration_bytes(const Hierarchy& H, int flexible, int W) {
  const int nl = (int)H.lv.size();
  double b = wide_kernel_bytes(H, KID_SPMV_DOT, 0, flexible, W) + wide_kernel_bytes(H, KID_CG_UPDATE, 0, flexible, W) +
             wide_kernel_bytes(H, KID_COARSE, nl - 1, flexible, W);
  for (int l = 0; l < nl - 1; ++l)
    b += wide_kernel_bytes(H, KID_PRE, l, flexible, W) + wide_kernel_bytes(H, KID_RESTRICT, l, flexible, W) +
         wide_kernel_bytes(H, KID_PROLONG, l, flexible, W) + wide_kernel_bytes(H, KID_POST, l, flexible, W);
  return b;
}

amg_status pcg_solve_wide(Hierarchy& H, const SolveOpts& o, const double* d_b, double* d_x, double tol, int W,
                          amg_info* info, hipStream_t s) {
  if (W < 1 || W > kMaxWidth) throw Error(AMG_ERR_INVALID_ARG, "batch width out of range");
  if (H.prm.nu_pre != 1 || H.prm.nu_post != 1) throw Error(AMG_ERR_INVALID_ARG, "batched solves use V(1,1)");
  const bool sys = H.S > 1;
  if (sys && W != H.S) throw Error(AMG_ERR_INVALID_ARG, "one column per system");
  if (sys) {
    if (H.fp32()) return solve_wide_impl<true, float>(H, o, d_b, d_x, tol, W, info, s);
    return solve_wide_impl<true, double>(H, o, d_b, d_x, tol, W, info, s);
  }
  if (H.fp32()) return solve_wide_impl<false, float>(H, o, d_b, d_x, tol, W, info, s);
  return solve_wide_impl<false, double>(H, o, d_b, d_x, tol, W, info, s);
}

void pattern_grad_wide(Hierarchy& H, const double* d_lam, const double* d_x, double* d_g, int W, hipStream_t s) {
  Level& L = H.lv[0];
  const int grid = (L.n + kBlock / 64 - 1) / (kBlock / 64);
  if (H.S > 1)
    hipLaunchKernelGGL(k_wpattern_grad<true>, dim3(grid), dim3(kBlock), 0, s, L.n, W, L.rp.p, L.ci.p, d_lam, d_x,
                       d_g);
  else
    hipLaunchKernelGGL(k_wpattern_grad<false>, dim3(grid), dim3(kBlock), 0, s, L.n, W, L.rp.p, L.ci.p, d_lam, d_x,
                       d_g);
  AMG_HIP(hipGetLastError());
}

}  // namespace amg
