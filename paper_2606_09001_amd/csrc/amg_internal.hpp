// Internal data structures and device primitives of the gfx950 AMG-PCG library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "amg355.h"

namespace amg {

// ------------------------------------------------------------------ errors

struct Error : std::runtime_error {
  amg_status status;
  Error(amg_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define AMG_HIP(call)                                                                                   \
  do {                                                                                                  \
    hipError_t e_ = (call);                                                                             \
    if (e_ != hipSuccess)                                                                               \
      throw ::amg::Error(e_ == hipErrorOutOfMemory ? AMG_ERR_OOM : AMG_ERR_HIP,                         \
                         std::string(#call) + ": " + hipGetErrorString(e_));                           \
  } while (0)

// --------------------------------------------------------------- memory

// Device buffer owned by a hierarchy.
template <class T>
struct DBuf {
  T* p = nullptr;
  int64_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(int64_t count) {
    if (count == n && p) return;
    release();
    if (count > 0) AMG_HIP(hipMalloc(&p, sizeof(T) * (size_t)count));
    n = count;
  }
  size_t bytes() const { return sizeof(T) * (size_t)n; }
};

// ------------------------------------------------------------- hierarchy

// Launch shape of a CSR sweep over one matrix.  stream: a workgroup stages
// rows_per_block rows (row pointers and products in LDS) and sums each row
// with `g` lanes; vec (fallback for very long rows): `g` lanes per row read
// the row directly.
struct Shape {
  int stream = 1;  // 1: CSR-stream, 0: lanes-per-row, 2: sliced (thread per row), 3: sliced, slot offsets
  int g = 1;
  int u = 8;       // CSR-stream: staged entries per thread (buffer of kBlock*u entries)
  int nt = 0;      // 1: the operator's entry stream is read with nontemporal loads
  int rows_per_block = 256;
  int grid = 1;
  int max_block_nnz = 0;
};

struct Level {
  int n = 0;
  int64_t nnz = 0;
  DBuf<int> rp, ci;           // A_l pattern
  DBuf<double> v;             // A_l values
  DBuf<float> v32;            // FP32 copy (FP32 cycle)
  // Sliced copy of A_l for levels of short rows (single system): slices of
  // 64 consecutive rows, entries stored column-major within a slice (entry j
  // of the slice's row r at soff[s] + 64 j + r), each row padded with
  // column -1 / value 0 to the slice's longest row.  sperm maps a sliced
  // position to its CSR position (-1: padding) for value refresh.
  //
  // Offset form (when every slice's rows use at most kSellMaxW distinct
  // column offsets col - row, as stencil operators do): slot j of a slice
  // holds the entries with offset slots[j].x of all its rows, in ascending
  // offset order; slots[j].z/.w are the 64-bit mask of the rows that have
  // that entry.  Values as above (0 where masked); no column array.
  bool sell = false;
  int sell_form = 0;          // 1: explicit columns, 2: slot offsets
  int64_t sell_len = 0;
  DBuf<int> soff, sci, sperm;
  DBuf<int4> sslot;
  DBuf<double> sv;
  DBuf<float> sv32;
  // arrays the operator sweeps over A_l read (sliced when present)
  const int* arp() const { return sell ? soff.p : rp.p; }
  const int* aci() const {
    return sell ? (sell_form == 2 ? reinterpret_cast<const int*>(sslot.p) : sci.p) : ci.p;
  }
  const double* av() const { return sell ? sv.p : v.p; }
  const float* av32() const { return sell ? sv32.p : v32.p; }
  DBuf<int> diagpos;          // position of a_ii in row i
  DBuf<double> dinv;          // 1 / a_ii
  DBuf<double> sw;            // smoother weight per row (omega/a_ii or 1/sum|a_ij|)
  DBuf<float> sw32;           // FP32 copy
  // strength graph
  DBuf<int> grp, gci;
  int64_t gnnz = 0;
  // aggregation (absent on the coarsest level)
  DBuf<int> agg;
  int nagg = 0;
  int mis_rounds = 0;
  double rho = 0.0, omegaP = 0.0;            // system 0
  std::vector<double> rhoS, omegaPS;         // per system
  // prolongator / restriction
  int64_t pnnz = 0;
  DBuf<int> prp, pci, rrp, rci, rperm;
  DBuf<double> pv, rv;
  DBuf<float> pv32, rv32;     // FP32 transfer copies (when not bf16)
  DBuf<uint16_t> pbf, rbf;    // bf16 transfer copies
  // Product maps of the numeric Galerkin products (the patterns are fixed, so
  // they are built once): for every output entry, the (x position, y
  // position) pairs of its terms in ascending inner index.  AP = A P uses
  // apm/apmo (per AP entry); A_{l+1} = R (AP) uses cm/cmo (per coarse entry).
  // Absent when they would exceed the memory budget (search kernels then).
  DBuf<int64_t> apmo, cmo;
  DBuf<int2> apm, cm;
  bool pmaps = false;
  // Map of the prolongator fill: P entry e sums A entries pak[pao[e] ..
  // pao[e+1]) (stored order) of row prow[e].
  DBuf<int> pao, pak, prow;
  // A*P intermediate (kept for value refresh)
  int64_t apnnz = 0;
  DBuf<int> aprp, apci;
  DBuf<double> apv;
  // cycle work vectors (FP64 and FP32)
  DBuf<double> x64, b64, r64, xs64, rs64;
  DBuf<float> x32, b32, r32, xs32, rs32;
  // kernel shapes (see choose_shapes)
  Shape shA, shP, shR;
};

struct Coarse {
  int n = 0;        // unknowns of the coarsest level
  int m = 0;        // padded to a multiple of 16
  DBuf<double> L;   // m*m factor, row-major: Cholesky (lower) or packed LU (nonsymmetric)
  DBuf<double> inv; // m*m inverse of the coarsest matrix, transposed ((j, i) holds (A^-1)_ij)
  DBuf<int> piv;    // nonsymmetric: LU row exchanges
  DBuf<float> inv32;
  DBuf<double> work;
};

// Device control block of one PCG or BiCGSTAB solve (single right-hand side).
struct Ctl {
  double bb, thresh;      // ||b||^2, tol^2 ||b||^2
  double rz, pq, rr;      // <r,z>, <p,Ap>, <r,r>
  double rzn, zq;         // new <r,z>, <z,q> (flexible)
  double alpha, beta;
  double rho, omega;      // BiCGSTAB: <r^, r>, <t, s>/<t, t>
  double trr;             // true residual ||b - A x||^2
  int iters, maxiter;
  int done;               // nonzero: kernels of the current solve return at once
  int state;              // 0 running, 1 converged (recursive), 2 iteration limit, -1 breakdown
  int flexible;
  int restarts;           // true-residual restarts (single-workgroup solve)
};

// Kernels that can be timed inside real solves (event pairs around every
// launch of one kernel at one level).
enum KernelId {
  KID_SPMV_DOT = 0, KID_PRE = 1, KID_POST = 2, KID_RESTRICT = 3, KID_PROLONG = 4,
  KID_CG_UPDATE = 5, KID_XPAY = 6, KID_COARSE = 7, KID_COUNT = 8
};

struct Instr {
  int kernel = -1, level = -1;
  std::vector<hipEvent_t> ev;  // begin/end pairs
  DBuf<int> was_done;          // per timed launch: the solve's done flag just before it
  int used = 0;
};

// Batched solves: W columns (right-hand sides of one matrix, or systems
// sharing a pattern), each an independent CG with its own scalars.
struct WCtl {
  double bb, thresh, rz, pq, rr, alpha, beta, trr, zq;
  int iters, state, done, first, restarts, pad_;
};
struct BatchHead {
  int ndone;     // columns finished (converged, iteration limit or breakdown)
  int W;
  int maxiter;
  int flexible;
};
struct BatchLevel {
  DBuf<double> x64, b64, r64;
  DBuf<float> x32, b32, r32;
  // row streams per XCD of the wide sweeps over A, P and R of this level
  // (0: one contiguous row range per workgroup)
  int spxA = 0, spxP = 0, spxR = 0;
  // rows per LDS-staged block of the wide sweeps over A, P and R (0: direct)
  int brA = 0, brP = 0, brR = 0;
};
struct Batch {
  int W = 0;
  int tuned_W = 0;  // width the stream counts were chosen for
  DBuf<double> r, z, p, p2, q, partials;
  DBuf<WCtl> ctl;
  DBuf<BatchHead> head;
  DBuf<int> mask;
  WCtl* h_ctl = nullptr;
  BatchHead* h_head = nullptr;
  int* h_mask = nullptr;
  std::vector<BatchLevel> lv;
  std::vector<int> col_iters, col_status;
  std::vector<double> col_relres;
};

// Captured PCG iterations.  Graph solves run on a library stream joined to
// the caller's stream by events (the caller's stream may be the legacy
// default stream, which cannot be captured).
struct Graphs {
  hipStream_t gs = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};   // pair of iterations, by direction-buffer parity
  hipGraphExec_t bexec = nullptr;                 // one BiCGSTAB iteration
  const void* key_x = nullptr;
  const void* key_bx = nullptr;
  int key_flex = -1;
  int key_w = 0;
  void reset();
  ~Graphs();
};

struct Hierarchy {
  amg_params prm{};
  Instr inst;
  Batch bt;
  Graphs gr;
  int S = 1;   // systems sharing the pattern (values interleaved [nnz][S])
  int n = 0;
  int64_t nnz = 0;
  std::vector<Level> lv;
  Coarse co;
  // solve workspace (level 0, FP64); BiCGSTAB adds r^, v, y, s, t
  DBuf<double> r, z, p, z2, q;
  DBuf<double> rh, bv, by, bs, bt2;
  // nonsymmetric adjoint: A^T (pattern, entry map, values) and its hierarchy,
  // built on first use and refreshed when A's values have changed since
  std::unique_ptr<Hierarchy> adj;
  DBuf<int> trp, tci, tperm;
  DBuf<double> tval;
  uint64_t val_version = 0, adj_version = 0;
  DBuf<double> partials;
  DBuf<Ctl> ctl;
  Ctl* h_ctl = nullptr;  // pinned host mirror
  DBuf<int> flags;       // device error flags / counters
  int* h_flags = nullptr;
  // cache bookkeeping
  uint64_t key = 0;
  int refs = 0;
  bool in_cache = false;
  // status of a value refresh that failed part-way (the levels then hold a
  // mix of old and new values): solves refuse with it until a refresh succeeds
  amg_status broken = AMG_OK;
  // single-workgroup solve (small.hip): lanes per R_0 row as a power-of-two
  // exponent, -1 when the hierarchy is not small enough
  int small_lgR = -1;
  bool small_checked = false;
  int cache_event = AMG_CACHE_COLD;
  double setup_ms = 0.0;
  bool fp32() const { return prm.vcycle_prec == AMG_PREC_FP32; }
  bool bf16() const { return fp32() && prm.transfer_bf16; }
  ~Hierarchy();
};

// Krylov workspace of one single-column PCG solve: the level-0 vectors, the
// per-workgroup partial sums, the device control block and a host copy of
// the control block.  Taken from the hierarchy's own buffers (solve_work) or
// from the static array of the allocation-free solve.
struct SolveWork {
  double *r, *z, *p, *z2, *q, *partials;
  Ctl* ctl;
  Ctl* h_ctl;
  bool graphs;  // hipGraph replay allowed (capture and instantiation allocate)
};

// Solve-time options carried by each handle.
struct SolveOpts {
  int maxiter;
  int flexible;     // -1 auto
  int check_every;  // 0 auto
  int use_graphs;   // replay captured iterations
  int fused_small;  // run small hierarchies' solves in one workgroup
};

}  // namespace amg

// A caller's reference on a (possibly shared) hierarchy, with its own
// solve-time options.
struct amg_handle_s {
  amg::Hierarchy* H;
  amg::SolveOpts opts;
};

namespace amg {

// setup.hip
void build_hierarchy(Hierarchy& H, const int* d_rp, const int* d_ci, const double* d_val, hipStream_t s);
void refresh_hierarchy(Hierarchy& H, const double* d_val, hipStream_t s);
void validate_csr(int n, int64_t nnz, const int* d_rp, const int* d_ci, int* d_flags, int* h_flags, hipStream_t s);
uint64_t pattern_hash(int n, int64_t nnz, const int* d_rp, const int* d_ci, int* d_flags, int* h_flags,
                      hipStream_t s);
bool pattern_equal(const Hierarchy& H, const int* d_rp, const int* d_ci, int* d_flags, int* h_flags, hipStream_t s);
bool values_equal(const Hierarchy& H, const double* d_val, int* d_flags, int* h_flags, hipStream_t s);
// float32 -> bfloat16 bits (f32_to_bf16) of n elements.
void convert_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s);
// A^T of the level-0 matrix: pattern (trp, tci) and entry map tperm (entry t
// of A^T is entry tperm[t] of A), then tval = A's values in that order.
void transpose_pattern(Hierarchy& H, hipStream_t s);
void transpose_values(Hierarchy& H, hipStream_t s);
// Sorted CSR pattern of A^T (n x n, nnz entries) and the entry map perm.
void transpose_csr_pattern(int n, int64_t nnz, const int* rp, const int* ci, DBuf<int>& trp, DBuf<int>& tci,
                           DBuf<int>& perm, hipStream_t s);
// probe.hip: matrix-free assembly by graph-colored probing
int color_columns(int n, int64_t nnz, const int* rp, const int* ci, int* color, int* d_flags, int* h_flags,
                  hipStream_t s);
void probe_vectors(int n, const int* color, int ncolors, double* V, int* d_flags, int* h_flags, hipStream_t s);
void probe_assemble(int n, const int* rp, const int* ci, const int* color, int ncolors, const double* Y, double* val,
                    int* d_flags, int* h_flags, hipStream_t s);
void probe_scatter(int n, const int* rp, const int* ci, const int* color, int ncolors, const double* dval,
                   double* dY, int* d_flags, int* h_flags, hipStream_t s);
// coarse.hip
void coarse_setup(Hierarchy& H, hipStream_t s);
// solve.hip
void alloc_solve_workspace(Hierarchy& H);
// Partial-sum slots a solve on H needs (the largest reducing grid, times the
// reductions per sweep, plus slack).
int64_t solve_partials_count(const Hierarchy& H);
SolveWork solve_work(Hierarchy& H);
// Persistent tuning cache (in memory and, when AMG_TUNE_CACHE names a file,
// in a text file): lookup and record of a launch choice under a key.
bool tune_lookup(const std::string& key, Shape* out);
void tune_record(const std::string& key, const Shape& sh);

amg_status pcg_solve(Hierarchy& H, const SolveOpts& o, const SolveWork& w, const double* d_b, double* d_x,
                     double tol, amg_info* info, hipStream_t s);
amg_status bicgstab_solve(Hierarchy& H, const SolveOpts& o, const double* d_b, double* d_x, double tol,
                          amg_info* info, hipStream_t s);
void apply_vcycle(Hierarchy& H, const double* d_r, double* d_z, hipStream_t s);
void pattern_grad(Hierarchy& H, const double* d_lam, const double* d_x, double* d_g, hipStream_t s);
void graph_stream(Hierarchy& H);
void capture_graph(hipStream_t s, hipGraphExec_t& ex, const std::function<void()>& body);
// small.hip
bool small_solve_ok(Hierarchy& H);
amg_status pcg_solve_small(Hierarchy& H, const SolveOpts& o, const SolveWork& w, const double* d_b, double* d_x,
                           double tol, amg_info* info, hipStream_t s);
// batch.hip
amg_status pcg_solve_wide(Hierarchy& H, const SolveOpts& o, const double* d_b, double* d_x, double tol, int W,
                          amg_info* info, hipStream_t s);
double wide_kernel_bytes(const Hierarchy& H, int kid, int level, int flexible, int W);
double wide_iteration_bytes(const Hierarchy& H, int flexible, int W);
void pattern_grad_wide(Hierarchy& H, const double* d_lam, const double* d_x, double* d_g, int W, hipStream_t s);
void choose_shapes(Hierarchy& H, hipStream_t s);
double kernel_bytes(const Hierarchy& H, int kid, int level, int flexible);
double iteration_bytes(const Hierarchy& H, int flexible);
void set_instrument(Hierarchy& H, int kid, int level);
void read_instrument(Hierarchy& H, int* launches, double* total_ms, double* min_ms, double* max_ms);

// ------------------------------------------------------- device helpers

constexpr int kBlock = 256;        // threads per block of the streaming kernels
constexpr int kMaxGrid = 2048;     // blocks of grid-stride kernels
constexpr int kStreamCap = 3072;   // most nonzeros a stream workgroup stages in LDS
// Last-level (Infinity) cache of the device: an operator whose entry stream
// is larger than this is read with nontemporal loads (it cannot stay cached
// between its sweeps, and caching it would only evict the gathered vectors).
constexpr double kLlcBytes = 256.0 * 1024 * 1024;
constexpr int kVecPer = 4;         // vector elements per thread in BLAS1 kernels
constexpr int kFinBlock = 1024;    // threads of the single-workgroup finalize kernels
constexpr int kMaxWidth = 64;       // columns of a batched solve (right-hand sides or systems)
constexpr int kSellMaxW = 8;        // longest row stored in the sliced form

__host__ __device__ inline int pow2_ceil(int x) {
  int g = 1;
  while (g < x) g <<= 1;
  return g;
}

// MurmurHash3 32-bit finalizer (public domain reference hash by A. Appleby).
__host__ __device__ inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Priority of node i in the independent-set selection (distinct per node).
__host__ __device__ inline uint64_t mis_key(int i) {
  return ((uint64_t)fmix32((uint32_t)i) << 32) | (uint64_t)(uint32_t)i;
}

// float -> bfloat16 bits, round to nearest even; NaN becomes a quiet NaN.
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

template <class T>
struct ValCvt;
template <>
struct ValCvt<double> { __device__ static double f(double v) { return v; } };
template <>
struct ValCvt<float> { __device__ static float f(float v) { return v; } };
template <>
struct ValCvt<uint16_t> { __device__ static float f(uint16_t v) { return bf16_to_f32(v); } };

#ifdef __HIPCC__
// Load of an operator's entry stream, nontemporal when NT.
template <bool NT, class T>
__device__ inline T stream_load(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// Row-shift DPP move of a double within rows of 16 lanes (lanes shifted in
// from outside the row read 0).
template <int SHIFT>
__device__ inline double dpp_row_shr(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x110 + SHIFT, 0xF, 0xF, true);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x110 + SHIFT, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int SHIFT>
__device__ inline float dpp_row_shr(float v) {
  int r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + SHIFT, 0xF, 0xF, true);
  return __int_as_float(r);
}

// Sum over aligned groups of G lanes; the total lands in the group's LAST
// lane (lane % G == G-1).  G <= 16 uses row-shift DPP, wider groups a
// butterfly through ds_bpermute (every lane then holds the total).
template <int G, class T>
__device__ inline T group_sum(T v) {
  if constexpr (G >= 2) v += dpp_row_shr<1>(v);
  if constexpr (G >= 4) v += dpp_row_shr<2>(v);
  if constexpr (G >= 8) v += dpp_row_shr<4>(v);
  if constexpr (G >= 16) v += dpp_row_shr<8>(v);
  if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}
template <int G>
__device__ inline bool group_leader() {
  return (threadIdx.x & (G - 1)) == (G - 1);
}

// Full-wavefront butterfly sum (every lane gets the total, fixed order).
template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum of NV values; result valid in thread 0.  Uses 8*NV*4 bytes of LDS.
template <int NV>
__device__ inline void block_sum(double (&v)[NV]) {
  __shared__ double red[NV][kBlock / 64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int m = 0; m < NV; ++m) v[m] = wave_sum(v[m]);
  if (l == 0) {
#pragma unroll
    for (int m = 0; m < NV; ++m) red[m][w] = v[m];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      double s = red[m][0];
      for (int k = 1; k < kBlock / 64; ++k) s += red[m][k];
      v[m] = s;
    }
  }
  __syncthreads();
}

#endif  // __HIPCC__

}  // namespace amg
