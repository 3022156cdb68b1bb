// Hierarchy construction on the GPU (smoothed aggregation), bit-exact by
// construction: every floating-point value is a fixed sequential fold in a
// canonical order (no atomics on floats, no FMA contraction; built with
// -ffp-contract=off), and the aggregation is the unique greedy distance-2
// independent set in decreasing key order, computed by parallel rounds.
//
// Setup reuse on a fixed pattern (Section 2.1, "C++/CUDA backend"): the
// refresh path keeps aggregates and every pattern and recomputes values only.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>

#include "amg_internal.hpp"

namespace amg {
namespace {

enum : int { F_BAD = 1, F_ZERO_DIAG = 2, F_NONSYM = 4, F_NOAGG = 8, F_MISMATCH = 16 };
enum : int8_t { S_UND = 0, S_ROOT = 1, S_EXCL = 2 };

inline int grid_for(int64_t items, int per_block = kBlock) {
  int64_t g = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, (int64_t)1 << 30));
}

void sync_flags(int* d_flags, int* h_flags, int count, hipStream_t s) {
  AMG_HIP(hipMemcpyAsync(h_flags, d_flags, sizeof(int) * count, hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
}

void zero_flags(int* d_flags, int count, hipStream_t s) {
  AMG_HIP(hipMemsetAsync(d_flags, 0, sizeof(int) * count, s));
}

// ------------------------------------------------------------ validation

__global__ void k_validate(int n, int64_t nnz, const int* __restrict__ rp, const int* __restrict__ ci,
                           int* flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int s = rp[i], e = rp[i + 1];
  bool bad = (i == 0 && s != 0) || (i == n - 1 && (int64_t)e != nnz) || s < 0 || e < s || (int64_t)e > nnz;
  if (bad) { atomicOr(flags, F_BAD); return; }
  bool diag = false;
  int prev = -1;
  for (int k = s; k < e; ++k) {
    int j = ci[k];
    if (j < 0 || j >= n || j <= prev) { atomicOr(flags, F_BAD); return; }
    diag |= (j == i);
    prev = j;
  }
  if (!diag) atomicOr(flags, F_ZERO_DIAG);
}

// ------------------------------------------------------------ hashing

__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void k_hash(int n, int64_t nnz, const int* __restrict__ rp, const int* __restrict__ ci,
                       unsigned long long* out) {
  uint64_t h = 0;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz; k += stride)
    h ^= splitmix64(((uint64_t)k << 32) ^ (uint32_t)ci[k]);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += stride)
    h ^= splitmix64(0x5bd1e995ull ^ ((uint64_t)(i + 1) << 33) ^ (uint32_t)rp[i]);
  for (int o = 32; o >= 1; o >>= 1) h ^= (uint64_t)__shfl_xor((unsigned long long)h, o, 64);
  if ((threadIdx.x & 63) == 0 && h) atomicXor(out, (unsigned long long)h);
}

template <class T>
__global__ void k_diff(int64_t count, const T* __restrict__ a, const T* __restrict__ b, int* flags) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool d = false;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count; k += stride) d |= (a[k] != b[k]);
  if (d) atomicOr(flags, F_MISMATCH);
}

__global__ void k_diff_bits(int64_t count, const double* __restrict__ a, const double* __restrict__ b,
                            int* flags) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool d = false;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count; k += stride)
    d |= (__double_as_longlong(a[k]) != __double_as_longlong(b[k]));
  if (d) atomicOr(flags, F_MISMATCH);
}

// ------------------------------------------------------- level numerics

// Diagonal position, 1/a_ii and the smoother weight of every row.
// Value arrays of several systems sharing the pattern are interleaved with
// stride vs (entry k of system s at [k*vs + s]); callers pass the pointers
// offset by s.
__global__ void k_diag(int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                       int vs, int* __restrict__ diagpos, double* __restrict__ dinv, double* __restrict__ sw,
                       float* __restrict__ sw32, double omega, int l1, int* flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int s = rp[i], e = rp[i + 1], pos = -1;
  double asum = 0.0;
  for (int k = s; k < e; ++k) {
    if (ci[k] == i) pos = k;
    asum += fabs(v[(int64_t)k * vs]);
  }
  const int64_t io = (int64_t)i * vs;
  if (pos < 0) {
    atomicOr(flags, F_ZERO_DIAG);
    diagpos[i] = s;
    dinv[io] = 0.0;
    sw[io] = 0.0;
    if (sw32) sw32[io] = 0.0f;
    return;
  }
  const double a = v[(int64_t)pos * vs];
  if (a == 0.0) atomicOr(flags, F_ZERO_DIAG);
  diagpos[i] = pos;
  double d = 1.0 / a;
  dinv[io] = d;
  double w = l1 ? 1.0 / asum : omega * d;
  sw[io] = w;
  if (sw32) sw32[io] = (float)w;
}

// Gershgorin bound max_i (sum_j |a_ij|) / |a_ii|; positive doubles order like
// their bit patterns, so an integer max is exact and order-free.
__global__ void k_rho(int n, const int* __restrict__ rp, const double* __restrict__ v, int vs,
                      const int* __restrict__ diagpos, unsigned long long* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long bits = 0;  // +0.0: below every ratio
  if (i < n) {
    double s = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) s += fabs(v[(int64_t)k * vs]);
    const double r = s / fabs(v[(int64_t)diagpos[i] * vs]);
    bits = (unsigned long long)__double_as_longlong(r);
  }
  // wavefront maximum first: one atomic per wave instead of one per row
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(bits, o, 64);
    bits = other > bits ? other : bits;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, bits);
}

// ------------------------------------------------------- strength graph

__global__ void k_sym_check(int n, const int* __restrict__ rp, const int* __restrict__ ci, int* flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    int j = ci[k];
    if (j == i) continue;
    int lo = rp[j], hi = rp[j + 1] - 1;
    bool found = false;
    while (lo <= hi) {
      int mid = (lo + hi) >> 1;
      int c = ci[mid];
      if (c == i) { found = true; break; }
      if (c < i) lo = mid + 1; else hi = mid - 1;
    }
    if (!found) { atomicOr(flags, F_NONSYM); return; }
  }
}

// Structurally symmetric pattern, theta = 0: the graph is A's pattern minus
// the diagonal (exactly one diagonal per row).
__global__ void k_graph_offdiag(int n, const int* __restrict__ rp, const int* __restrict__ ci, int* __restrict__ grp,
                                int* __restrict__ gci) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  grp[i] = rp[i] - i;
  if (i == n) return;
  int o = rp[i] - i;
  for (int k = rp[i]; k < rp[i + 1]; ++k)
    if (ci[k] != i) gci[o++] = ci[k];
}

__device__ inline bool strong(double aij, double aii, double ajj, double theta) {
  return theta <= 0.0 || fabs(aij) >= theta * sqrt(fabs(aii * ajj));
}

__global__ void k_edge_count(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                             const double* __restrict__ v, const int* __restrict__ diagpos, double theta,
                             int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    int j = ci[k];
    if (j != i && strong(v[k], v[diagpos[i]], v[diagpos[j]], theta)) c += 2;
  }
  cnt[i] = c;
}

__global__ void k_edge_emit(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                            const double* __restrict__ v, const int* __restrict__ diagpos, double theta,
                            const int* __restrict__ off, unsigned long long* __restrict__ keys) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = off[i];
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    int j = ci[k];
    if (j != i && strong(v[k], v[diagpos[i]], v[diagpos[j]], theta)) {
      keys[o++] = ((unsigned long long)(uint32_t)i << 32) | (uint32_t)j;
      keys[o++] = ((unsigned long long)(uint32_t)j << 32) | (uint32_t)i;
    }
  }
}

__global__ void k_edge_rows(int64_t m, const unsigned long long* __restrict__ keys, int* __restrict__ cnt,
                            int* __restrict__ gci) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m) return;
  unsigned long long k = keys[t];
  atomicAdd(cnt + (int)(k >> 32), 1);
  gci[t] = (int)(k & 0xffffffffu);
}

// ---------------------------------------------------- aggregation rounds

// m1[i] = 1 + max key among undecided nodes in {i} U N(i) (0 if none).
__global__ void k_mis_m1(int n, const int* __restrict__ grp, const int* __restrict__ gci,
                         const int8_t* __restrict__ state, unsigned long long* __restrict__ m1) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long best = state[i] == S_UND ? mis_key(i) + 1 : 0;
  for (int k = grp[i]; k < grp[i + 1]; ++k) {
    int j = gci[k];
    if (state[j] == S_UND) best = max(best, (unsigned long long)mis_key(j) + 1);
  }
  m1[i] = best;
}

// An undecided node whose key is the largest among undecided nodes within
// distance 2 becomes a root.
__global__ void k_mis_m2(int n, const int* __restrict__ grp, const int* __restrict__ gci,
                         const unsigned long long* __restrict__ m1, int8_t* __restrict__ state) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || state[i] != S_UND) return;
  unsigned long long best = m1[i];
  for (int k = grp[i]; k < grp[i + 1]; ++k) best = max(best, m1[gci[k]]);
  if (best == mis_key(i) + 1) state[i] = S_ROOT;
}

__global__ void k_mis_e1(int n, const int* __restrict__ grp, const int* __restrict__ gci,
                         const int8_t* __restrict__ state, int8_t* __restrict__ e1) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool r = state[i] == S_ROOT;
  for (int k = grp[i]; k < grp[i + 1] && !r; ++k) r = state[gci[k]] == S_ROOT;
  e1[i] = r;
}

// Undecided nodes within distance 2 of a root are excluded; the remaining
// undecided nodes are counted.
__global__ void k_mis_e2(int n, const int* __restrict__ grp, const int* __restrict__ gci,
                         const int8_t* __restrict__ e1, int8_t* __restrict__ state, int* __restrict__ undecided) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int und = 0;
  if (i < n && state[i] == S_UND) {
    bool r = e1[i];
    for (int k = grp[i]; k < grp[i + 1] && !r; ++k) r = e1[gci[k]];
    if (r) state[i] = S_EXCL; else und = 1;
  }
  const unsigned long long m = __ballot(und);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(undecided, (int)__popcll(m));
}

__global__ void k_is_root(int n, const int8_t* __restrict__ state, int* __restrict__ isroot) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) isroot[i] = state[i] == S_ROOT;
  if (i == n) isroot[n] = 0;
}

// Roots take their rank among roots (ascending index); their graph
// neighbours join them (unique: roots are at least 3 apart).
__global__ void k_agg_phase12(int n, const int* __restrict__ grp, const int* __restrict__ gci,
                              const int8_t* __restrict__ state, const int* __restrict__ rank,
                              int* __restrict__ agg2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int a = -1;
  if (state[i] == S_ROOT) {
    a = rank[i];
  } else {
    for (int k = grp[i]; k < grp[i + 1]; ++k) {
      int j = gci[k];
      if (state[j] == S_ROOT) { a = rank[j]; break; }
    }
  }
  agg2[i] = a;
}

// The remaining nodes join the smallest aggregate among their neighbours
// assigned in the previous step (reads only that step's state).
__global__ void k_agg_phase3(int n, const int* __restrict__ grp, const int* __restrict__ gci,
                             const int* __restrict__ agg2, int* __restrict__ agg, int* flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int a = agg2[i];
  if (a < 0) {
    for (int k = grp[i]; k < grp[i + 1]; ++k) {
      int b = agg2[gci[k]];
      if (b >= 0 && (a < 0 || b < a)) a = b;
    }
    if (a < 0) atomicOr(flags, F_NOAGG);
  }
  agg[i] = a;
}

// ------------------------------------------------------- prolongator

// Number of distinct aggregates touched by row i.
__global__ void k_p_count(int n, const int* __restrict__ rp, const int* __restrict__ ci, const int* __restrict__ agg,
                          int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == n) { cnt[n] = 0; return; }
  int prev = -1, c = 0;
  for (;;) {
    int nxt = INT_MAX;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      int a = agg[ci[k]];
      if (a > prev && a < nxt) nxt = a;
    }
    if (nxt == INT_MAX) break;
    ++c;
    prev = nxt;
  }
  cnt[i] = c;
}

// P = (I - omegaP D^-1 A) T: for each touched aggregate J (ascending),
// s_J = sum of a_ij over j in row i with agg(j) = J in stored order from
// +0.0, w = omegaP / a_ii, P_iJ = [J == agg(i)] - w*s_J (unfused).
__global__ void k_p_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                         int vs, const int* __restrict__ diagpos, const int* __restrict__ agg, double omegaP,
                         const int* __restrict__ prp, int* __restrict__ pci, double* __restrict__ pv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double w = omegaP / v[(int64_t)diagpos[i] * vs];
  int ai = agg[i];
  int pos = prp[i], prev = -1;
  for (;;) {
    int nxt = INT_MAX;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      int a = agg[ci[k]];
      if (a > prev && a < nxt) nxt = a;
    }
    if (nxt == INT_MAX) break;
    double sJ = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (agg[ci[k]] == nxt) sJ += v[(int64_t)k * vs];
    double delta = (nxt == ai) ? 1.0 : 0.0;
    double ws = w * sJ;
    if (pci) pci[pos] = nxt;
    pv[(int64_t)pos * vs] = delta - ws;
    ++pos;
    prev = nxt;
  }
}

// Map of the prolongator fill (thread per row): for each P entry of row i,
// the A entries of row i whose column lies in that entry's aggregate, in
// stored order, and the entry's row.
__global__ void k_pmap_build(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                             const int* __restrict__ agg, const int* __restrict__ prp, const int* __restrict__ pci,
                             int* __restrict__ pao, int* __restrict__ pak, int* __restrict__ prow) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int t = rp[i];
  for (int e = prp[i]; e < prp[i + 1]; ++e) {
    pao[e] = t;
    prow[e] = i;
    const int J = pci[e];
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (agg[ci[k]] == J) pak[t++] = k;
  }
  // entries whose column has no aggregate belong to no P entry
  for (; t < rp[i + 1]; ++t) pak[t] = -1;
  if (i == n - 1) pao[prp[n]] = rp[n];
}

// Prolongator values through the map (thread per entry): the same
// expression and fold as k_p_fill.
__global__ void k_p_refill(int64_t pnnz, const int* __restrict__ pao, const int* __restrict__ pak,
                           const int* __restrict__ prow, const int* __restrict__ pci, const double* __restrict__ v,
                           int vs, const int* __restrict__ diagpos, const int* __restrict__ agg, double omegaP,
                           double* __restrict__ pv) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= pnnz) return;
  const int i = prow[e];
  const double w = omegaP / v[(int64_t)diagpos[i] * vs];
  double sJ = 0.0;
  for (int t = pao[e]; t < pao[e + 1]; ++t)
    if (pak[t] >= 0) sJ += v[(int64_t)pak[t] * vs];
  const double delta = (pci[e] == agg[i]) ? 1.0 : 0.0;
  const double ws = w * sJ;
  pv[e * vs] = delta - ws;
}

__global__ void k_row_ids(int n, const int* __restrict__ rp, int* __restrict__ rowid) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) rowid[k] = i;
}

__global__ void k_iota(int64_t m, int* __restrict__ a) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < m) a[t] = (int)t;
}

__global__ void k_col_count(int64_t m, const int* __restrict__ ci, int* __restrict__ cnt) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < m) atomicAdd(cnt + ci[t], 1);
}

// R = P^T: entry t of R is entry perm[t] of P (stable sort by column keeps
// source rows ascending inside each row of R).
__global__ void k_r_fill(int64_t m, const int* __restrict__ perm, const int* __restrict__ rowid,
                         const double* __restrict__ pv, int vs, int* __restrict__ rci, double* __restrict__ rv) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m) return;
  int k = perm[t];
  if (rci) rci[t] = rowid[k];
  rv[t * vs] = pv[(int64_t)k * vs];
}

// Columns of a transposed pattern: entry t holds the source row of entry perm[t].
__global__ void k_t_cols(int64_t m, const int* __restrict__ perm, const int* __restrict__ rowid,
                         int* __restrict__ tci) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < m) tci[t] = rowid[perm[t]];
}

// ------------------------------------------------- canonical products

// Position of column J in the sorted column list [lo, hi), or -1.
__device__ inline int find_col(const int* __restrict__ ci, int lo, int hi, int J) {
  --hi;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    int c = ci[mid];
    if (c == J) return mid;
    if (c < J) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// Smallest column > prev in the sorted list [lo, hi), or INT_MAX.
__device__ inline int next_col(const int* __restrict__ ci, int lo, int hi, int prev) {
  int a = lo, b = hi;
  while (a < b) {
    int mid = (a + b) >> 1;
    if (ci[mid] <= prev) a = mid + 1; else b = mid;
  }
  return a < hi ? ci[a] : INT_MAX;
}

// Row i of C = X Y: distinct columns over the rows of Y selected by row i of X.
__global__ void k_spgemm_count(int nrows, const int* __restrict__ xrp, const int* __restrict__ xci,
                               const int* __restrict__ yrp, const int* __restrict__ yci, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > nrows) return;
  if (i == nrows) { cnt[nrows] = 0; return; }
  int prev = -1, c = 0;
  for (;;) {
    int nxt = INT_MAX;
    for (int a = xrp[i]; a < xrp[i + 1]; ++a) {
      int k = xci[a];
      nxt = min(nxt, next_col(yci, yrp[k], yrp[k + 1], prev));
    }
    if (nxt == INT_MAX) break;
    ++c;
    prev = nxt;
  }
  cnt[i] = c;
}

// Row i of C = X Y with one wavefront per row (rows with many candidates,
// such as R (A P)): every candidate column (the rows of Y selected by row i
// of X, split across the lanes) is inserted into an LDS hash set (open
// addressing, linear probing, compare-and-swap), so each distinct column is
// kept once however many candidates repeat it.  COLS = 0 counts them
// (cnt[i]; block nrows writes cnt[nrows] = 0); COLS = 1 compacts them and
// sorts them ascending (a bitonic network across the lanes, or in LDS beyond
// 64 columns).  A row with more than kSymTab / 2 distinct columns stops
// inserting and takes the sequential merge of k_spgemm_count in lane 0.
// The result is the pattern that merge gives (distinct columns, ascending).
constexpr int kSymTab = 2048;

template <int COLS>
__global__ void __launch_bounds__(64) k_spgemm_sym_w(int nrows, const int* __restrict__ xrp,
                                                     const int* __restrict__ xci, const int* __restrict__ yrp,
                                                     const int* __restrict__ yci, const int* __restrict__ crp,
                                                     int* __restrict__ out) {
  __shared__ int tab[kSymTab];
  __shared__ int s_cnt, s_over;
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= nrows) {
    if (!COLS && i == nrows && lane == 0) out[nrows] = 0;
    return;
  }
  const int a0 = xrp[i], a1 = xrp[i + 1];
  for (int t = lane; t < kSymTab; t += 64) tab[t] = -1;
  if (lane == 0) {
    s_cnt = 0;
    s_over = 0;
  }
  __syncthreads();
  // inserts stop once kSymTab / 2 distinct columns are in; a lane already
  // probing adds at most one more, so the table never fills and every probe
  // sequence ends
  for (int a = a0 + lane; a < a1; a += 64) {
    const int k = xci[a];
    for (int q = yrp[k]; q < yrp[k + 1]; ++q) {
      if (__hip_atomic_load(&s_over, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
      const int c = yci[q];
      unsigned h = ((unsigned)c * 2654435761u) & (kSymTab - 1);
      for (;;) {
        const int old = atomicCAS(&tab[h], -1, c);
        if (old == -1) {
          if (atomicAdd(&s_cnt, 1) + 1 > kSymTab / 2) atomicOr(&s_over, 1);
          break;
        }
        if (old == c) break;
        h = (h + 1) & (kSymTab - 1);
      }
    }
  }
  __syncthreads();
  if (s_over) {
    // sequential k-way merge (lane 0)
    if (lane != 0) return;
    int prev = -1, c = 0, pos = COLS ? crp[i] : 0;
    for (;;) {
      int nxt = INT_MAX;
      for (int a = a0; a < a1; ++a) {
        const int k = xci[a];
        nxt = min(nxt, next_col(yci, yrp[k], yrp[k + 1], prev));
      }
      if (nxt == INT_MAX) break;
      if (COLS) out[pos++] = nxt;
      ++c;
      prev = nxt;
    }
    if (!COLS) out[i] = c;
    return;
  }
  const int distinct = s_cnt;
  if (!COLS) {
    if (lane == 0) out[i] = distinct;
    return;
  }
  // compact the occupied slots to the front, in place: chunk t0's writes go
  // below t0 + 64, to slots already read (each chunk is read before it writes)
  int w = 0;
  for (int t0 = 0; t0 < kSymTab; t0 += 64) {
    const int c = tab[t0 + lane];
    const bool occ = c >= 0;
    const unsigned long long m = __ballot(occ);
    const int slot = w + __popcll(m & ((1ull << lane) - 1ull));
    __syncthreads();
    if (occ) tab[slot] = c;
    __syncthreads();
    w += __popcll(m);
  }
  const int pos = crp[i];
  if (distinct <= 64) {
    // bitonic sort across the lanes (INT_MAX padding sorts last)
    int v = lane < distinct ? tab[lane] : INT_MAX;
    for (int kk = 2; kk <= 64; kk <<= 1) {
      for (int j = kk >> 1; j > 0; j >>= 1) {
        const int o = __shfl_xor(v, j, 64);
        const bool lower = (lane & j) == 0;
        const bool up = (lane & kk) == 0;
        v = (lower == up) ? min(v, o) : max(v, o);
      }
    }
    if (lane < distinct) out[pos + lane] = v;
    return;
  }
  int S = 1;
  while (S < distinct) S <<= 1;
  for (int t = distinct + lane; t < S; t += 64) tab[t] = INT_MAX;
  __syncthreads();
  for (int kk = 2; kk <= S; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < S; t += 64) {
        const int u = t ^ j;
        if (u > t) {
          const int x = tab[t], y = tab[u];
          const bool up = (t & kk) == 0;
          if ((x > y) == up) {
            tab[t] = y;
            tab[u] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = lane; t < distinct; t += 64) out[pos + t] = tab[t];
}

// Values of C = X Y in canonical order: for every output column J
// (ascending), acc = +0.0 and for every k of row i of X in ascending order
// with y_kJ stored, acc += x_ik * y_kJ (product rounded, then sum rounded).
// This is the per-entry order of the row-by-row scatter "for k ascending, for
// J ascending: acc[J] += x_ik y_kJ".
__global__ void k_spgemm_fill(int nrows, const int* __restrict__ xrp, const int* __restrict__ xci,
                              const double* __restrict__ xv, const int* __restrict__ yrp, const int* __restrict__ yci,
                              const double* __restrict__ yv, const int* __restrict__ crp, int* __restrict__ cci,
                              double* __restrict__ cv, int vs) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  int pos = crp[i], prev = -1;
  for (;;) {
    int nxt = INT_MAX;
    for (int a = xrp[i]; a < xrp[i + 1]; ++a) {
      int k = xci[a];
      nxt = min(nxt, next_col(yci, yrp[k], yrp[k + 1], prev));
    }
    if (nxt == INT_MAX) break;
    double acc = 0.0;
    for (int a = xrp[i]; a < xrp[i + 1]; ++a) {
      int k = xci[a];
      int q = find_col(yci, yrp[k], yrp[k + 1], nxt);
      if (q >= 0) {
        double prod = xv[(int64_t)a * vs] * yv[(int64_t)q * vs];
        acc = acc + prod;
      }
    }
    if (cci) cci[pos] = nxt;
    cv[(int64_t)pos * vs] = acc;
    ++pos;
    prev = nxt;
  }
}

// Numeric C = X Y on a known pattern, one thread per stored entry (row i,
// column J): the same fold over k of row i of X in ascending order as
// k_spgemm_fill, so the values are identical; parallel over all entries.
__global__ void k_spgemm_fill_entries(int nrows, int64_t cnnz, const int* __restrict__ crp,
                                      const int* __restrict__ cci, const int* __restrict__ xrp,
                                      const int* __restrict__ xci, const double* __restrict__ xv,
                                      const int* __restrict__ yrp, const int* __restrict__ yci,
                                      const double* __restrict__ yv, double* __restrict__ cv, int vs) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= cnnz) return;
  // row of entry e: last i with crp[i] <= e
  int lo = 0, hi = nrows;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)crp[mid] <= e) lo = mid; else hi = mid;
  }
  const int i = lo;
  const int J = cci[e];
  double acc = 0.0;
  for (int a = xrp[i]; a < xrp[i + 1]; ++a) {
    const int k = xci[a];
    const int q = find_col(yci, yrp[k], yrp[k + 1], J);
    if (q >= 0) {
      double prod = xv[(int64_t)a * vs] * yv[(int64_t)q * vs];
      acc = acc + prod;
    }
  }
  cv[e * vs] = acc;
}

// Product map of C = X Y on C's fixed pattern: number of terms per entry.
__global__ void k_pm_count(int nrows, int64_t cnnz, const int* __restrict__ crp, const int* __restrict__ cci,
                           const int* __restrict__ xrp, const int* __restrict__ xci, const int* __restrict__ yrp,
                           const int* __restrict__ yci, int64_t* __restrict__ cnt) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e > cnnz) return;
  if (e == cnnz) {
    cnt[cnnz] = 0;
    return;
  }
  int lo = 0, hi = nrows;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)crp[mid] <= e) lo = mid; else hi = mid;
  }
  const int J = cci[e];
  int64_t c = 0;
  for (int a = xrp[lo]; a < xrp[lo + 1]; ++a) c += find_col(yci, yrp[xci[a]], yrp[xci[a] + 1], J) >= 0;
  cnt[e] = c;
}

// Product map, pass 2: the (x position, y position) pairs of each entry in
// ascending inner index (the order of the fold that forms the entry).
__global__ void k_pm_fill(int nrows, int64_t cnnz, const int* __restrict__ crp, const int* __restrict__ cci,
                          const int* __restrict__ xrp, const int* __restrict__ xci, const int* __restrict__ yrp,
                          const int* __restrict__ yci, const int64_t* __restrict__ off, int2* __restrict__ pairs) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= cnnz) return;
  int lo = 0, hi = nrows;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)crp[mid] <= e) lo = mid; else hi = mid;
  }
  const int J = cci[e];
  int64_t p = off[e];
  for (int a = xrp[lo]; a < xrp[lo + 1]; ++a) {
    const int q = find_col(yci, yrp[xci[a]], yrp[xci[a] + 1], J);
    if (q >= 0) pairs[p++] = make_int2(a, q);
  }
}

// Numeric product through the map: the same fold (ascending inner index, each
// product rounded before the add) as k_spgemm_fill_entries, with all loads
// independent of each other.
__global__ void k_pm_apply(int64_t cnnz, const int64_t* __restrict__ off, const int2* __restrict__ pairs,
                           const double* __restrict__ xv, const double* __restrict__ yv, double* __restrict__ cv,
                           int vs) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= cnnz) return;
  double acc = 0.0;
  const int64_t p0 = off[e], p1 = off[e + 1];
  // 4 terms in flight: unconditional loads at clamped positions, the adds
  // masked and in order
  constexpr int U = 4;
  for (int64_t p = p0; p < p1; p += U) {
    int2 t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = pairs[min(p + u, p1 - 1)];
    double prod[U];
#pragma unroll
    for (int u = 0; u < U; ++u) prod[u] = xv[(int64_t)t[u].x * vs] * yv[(int64_t)t[u].y * vs];
#pragma unroll
    for (int u = 0; u < U; ++u) acc = p + u < p1 ? acc + prod[u] : acc;
  }
  cv[e * vs] = acc;
}

// ------------------------------------------------------ precision copies

__global__ void k_to_f32(int64_t m, const double* __restrict__ a, float* __restrict__ b) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < m) b[t] = (float)a[t];
}

__global__ void k_to_bf16(int64_t m, const double* __restrict__ a, uint16_t* __restrict__ b) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < m) b[t] = f32_to_bf16((float)a[t]);
}

__global__ void k_f32_to_bf16(int64_t m, const float* __restrict__ a, uint16_t* __restrict__ b) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m; t += stride) b[t] = f32_to_bf16(a[t]);
}

// ------------------------------------------------------ sliced copy of A

// Entries per slice of 64 rows: 64 times the slice's longest row.
__global__ void k_sell_width(int n, int ns, const int* __restrict__ rp, int* __restrict__ cnt) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl > ns) return;
  if (sl == ns) {
    cnt[ns] = 0;
    return;
  }
  int w = 0;
  const int r1 = min(n, sl * 64 + 64);
  for (int i = sl * 64; i < r1; ++i) w = max(w, rp[i + 1] - rp[i]);
  cnt[sl] = 64 * w;
}

// Thread per (padded) row: its entries in stored order, then padding.
__global__ void k_sell_fill(int n, int ns, const int* __restrict__ rp, const int* __restrict__ ci,
                            const int* __restrict__ soff, int* __restrict__ sci, int* __restrict__ sperm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns * 64) return;
  const int sl = i >> 6, lane = i & 63;
  const int w = (soff[sl + 1] - soff[sl]) >> 6;
  const int k0 = i < n ? rp[i] : 0, len = i < n ? rp[i + 1] - k0 : 0;
  for (int j = 0; j < w; ++j) {
    const int64_t p = soff[sl] + (int64_t)j * 64 + lane;
    sci[p] = j < len ? ci[k0 + j] : -1;
    sperm[p] = j < len ? k0 + j : -1;
  }
}

// Offset form, pass 1: per slice, the sorted union of its rows' column
// offsets (col - row); 64 x its size (kSellMaxW + 1 when it overflows).
__global__ void k_sello_count(int n, int ns, const int* __restrict__ rp, const int* __restrict__ ci,
                              int* __restrict__ cnt, int* __restrict__ uoff) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl > ns) return;
  if (sl == ns) {
    cnt[ns] = 0;
    return;
  }
  int u[kSellMaxW];
  int m = 0;
  bool over = false;
  const int r1 = min(n, sl * 64 + 64);
  for (int i = sl * 64; i < r1 && !over; ++i) {
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int d = ci[k] - i;
      int pos = 0;
      while (pos < m && u[pos] < d) ++pos;
      if (pos < m && u[pos] == d) continue;
      if (m == kSellMaxW) {
        over = true;
        break;
      }
      for (int t = m; t > pos; --t) u[t] = u[t - 1];
      u[pos] = d;
      ++m;
    }
  }
  cnt[sl] = 64 * (over ? kSellMaxW + 1 : m);
  for (int j = 0; j < kSellMaxW; ++j) uoff[(int64_t)sl * kSellMaxW + j] = j < m ? u[j] : 0;
}

// Offset form, pass 2: slot records (offset, row mask) and the position map.
__global__ void k_sello_fill(int n, int ns, const int* __restrict__ rp, const int* __restrict__ ci,
                             const int* __restrict__ soff, const int* __restrict__ uoff, int4* __restrict__ slots,
                             int* __restrict__ sperm) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= ns) return;
  const int base = soff[sl], w = (soff[sl + 1] - base) >> 6;
  const int* u = uoff + (int64_t)sl * kSellMaxW;
  for (int p = base; p < base + 64 * w; ++p) sperm[p] = -1;
  unsigned long long mask[kSellMaxW] = {};
  const int r1 = min(n, sl * 64 + 64);
  for (int i = sl * 64; i < r1; ++i) {
    const int lane = i - sl * 64;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int d = ci[k] - i;
      int j = 0;
      while (j < w && u[j] != d) ++j;
      sperm[base + j * 64 + lane] = k;
      mask[j] |= 1ull << lane;
    }
  }
  for (int j = 0; j < w; ++j)
    slots[(base >> 6) + j] = make_int4(u[j], 0, (int)(unsigned)(mask[j] & 0xffffffffull), (int)(unsigned)(mask[j] >> 32));
}

__global__ void k_sell_vals(int64_t m, const int* __restrict__ sperm, const double* __restrict__ v,
                            double* __restrict__ sv, float* __restrict__ sv32) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= m) return;
  const int k = sperm[p];
  const double a = k >= 0 ? v[k] : 0.0;
  sv[p] = a;
  if (sv32) sv32[p] = (float)a;
}

// ---------------------------------------------------------- host helpers

template <class F>
void cub_call(F&& f, hipStream_t s) {
  size_t tmp = 0;
  AMG_HIP(f(nullptr, tmp));
  DBuf<unsigned char> buf;
  buf.alloc((int64_t)std::max<size_t>(tmp, 1));
  AMG_HIP(f(buf.p, tmp));
  AMG_HIP(hipStreamSynchronize(s));  // the temporary buffer is freed on return
}

// Exclusive scan of cnt[0..m) into out[0..m) (int).
void exclusive_scan(const int* cnt, int* out, int64_t m, hipStream_t s) {
  cub_call([&](void* t, size_t& b) { return hipcub::DeviceScan::ExclusiveSum(t, b, cnt, out, (int)m, s); }, s);
}

int64_t read_i64(const int64_t* d, hipStream_t s) {
  int64_t h = 0;
  AMG_HIP(hipMemcpyAsync(&h, d, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  return h;
}

// Builds the product map of C = X Y on C's pattern; false (and nothing kept)
// when its pairs would exceed `budget`.
bool build_product_map(int nrows, int64_t cnnz, const int* crp, const int* cci, const int* xrp, const int* xci,
                       const int* yrp, const int* yci, int64_t budget, DBuf<int64_t>& off, DBuf<int2>& pairs,
                       hipStream_t s) {
  DBuf<int64_t> cnt;
  cnt.alloc(cnnz + 1);
  hipLaunchKernelGGL(k_pm_count, dim3((unsigned)((cnnz + kBlock) / kBlock)), dim3(kBlock), 0, s, nrows, cnnz, crp, cci,
                     xrp, xci, yrp, yci, cnt.p);
  off.alloc(cnnz + 1);
  cub_call([&](void* t, size_t& b) {
    return hipcub::DeviceScan::ExclusiveSum(t, b, cnt.p, off.p, (int)(cnnz + 1), s);
  }, s);
  const int64_t total = read_i64(off.p + cnnz, s);
  if (total > budget) {
    off.release();
    return false;
  }
  pairs.alloc(std::max<int64_t>(total, 1));
  hipLaunchKernelGGL(k_pm_fill, dim3((unsigned)((cnnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, nrows, cnnz, crp,
                     cci, xrp, xci, yrp, yci, off.p, pairs.p);
  AMG_HIP(hipStreamSynchronize(s));  // cnt is freed on return
  return true;
}

int read_int(const int* d, hipStream_t s) {
  int h = 0;
  AMG_HIP(hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  return h;
}

void level_numerics(Hierarchy& H, Level& L, hipStream_t s) {
  const int S = H.S;
  L.diagpos.alloc(L.n);
  L.dinv.alloc((int64_t)L.n * S);
  L.sw.alloc((int64_t)L.n * S);
  if (H.fp32()) L.sw32.alloc((int64_t)L.n * S);
  zero_flags(H.flags.p, 1, s);
  for (int sy = 0; sy < S; ++sy)
    hipLaunchKernelGGL(k_diag, dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, L.rp.p, L.ci.p, L.v.p + sy, S,
                       L.diagpos.p, L.dinv.p + sy, L.sw.p + sy, H.fp32() ? L.sw32.p + sy : nullptr, H.prm.omega,
                       (int)(H.prm.smoother == AMG_SMOOTHER_L1), H.flags.p);
  AMG_HIP(hipGetLastError());
  sync_flags(H.flags.p, H.h_flags, 1, s);
  if (H.h_flags[0] & F_ZERO_DIAG) throw Error(AMG_ERR_ZERO_DIAG, "zero diagonal");
}

void strength_graph(Hierarchy& H, Level& L, hipStream_t s) {
  L.grp.alloc(L.n + 1);
  bool fast = H.prm.theta <= 0.0;
  if (fast) {
    zero_flags(H.flags.p, 1, s);
    hipLaunchKernelGGL(k_sym_check, dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, L.rp.p, L.ci.p, H.flags.p);
    sync_flags(H.flags.p, H.h_flags, 1, s);
    fast = !(H.h_flags[0] & F_NONSYM);
  }
  if (fast) {
    L.gnnz = L.nnz - L.n;
    L.gci.alloc(std::max<int64_t>(L.gnnz, 1));
    hipLaunchKernelGGL(k_graph_offdiag, dim3(grid_for(L.n + 1)), dim3(kBlock), 0, s, L.n, L.rp.p, L.ci.p, L.grp.p,
                       L.gci.p);
    AMG_HIP(hipGetLastError());
    return;
  }
  // general path: emit (i,j) and (j,i) for every strong entry, sort, unique
  DBuf<int> cnt, off;
  cnt.alloc(L.n + 1);
  off.alloc(L.n + 1);
  AMG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * (L.n + 1), s));
  hipLaunchKernelGGL(k_edge_count, dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, L.rp.p, L.ci.p, L.v.p,
                     L.diagpos.p, H.prm.theta, cnt.p);
  exclusive_scan(cnt.p, off.p, L.n + 1, s);
  int m = read_int(off.p + L.n, s);
  DBuf<unsigned long long> keys, sorted, uniq;
  DBuf<int> nuniq;
  nuniq.alloc(1);
  int64_t mm = std::max(m, 1);
  keys.alloc(mm);
  sorted.alloc(mm);
  uniq.alloc(mm);
  hipLaunchKernelGGL(k_edge_emit, dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, L.rp.p, L.ci.p, L.v.p, L.diagpos.p,
                     H.prm.theta, off.p, keys.p);
  cub_call([&](void* t, size_t& b) {
    return hipcub::DeviceRadixSort::SortKeys(t, b, keys.p, sorted.p, m, 0, 64, s);
  }, s);
  cub_call([&](void* t, size_t& b) {
    return hipcub::DeviceSelect::Unique(t, b, sorted.p, uniq.p, nuniq.p, m, s);
  }, s);
  int u = read_int(nuniq.p, s);
  L.gnnz = u;
  L.gci.alloc(std::max(u, 1));
  AMG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * (L.n + 1), s));
  if (u > 0)
    hipLaunchKernelGGL(k_edge_rows, dim3(grid_for(u)), dim3(kBlock), 0, s, (int64_t)u, uniq.p, cnt.p, L.gci.p);
  exclusive_scan(cnt.p, L.grp.p, L.n + 1, s);
  AMG_HIP(hipGetLastError());
}

// Returns the number of aggregates.
int aggregate(Hierarchy& H, Level& L, hipStream_t s) {
  const int n = L.n;
  DBuf<int8_t> state, e1;
  DBuf<unsigned long long> m1;
  state.alloc(n);
  e1.alloc(n);
  m1.alloc(n);
  AMG_HIP(hipMemsetAsync(state.p, 0, n, s));
  int rounds = 0;
  const dim3 g(grid_for(n)), b(kBlock);
  for (;;) {
    ++rounds;
    if (rounds > n + 1) throw Error(AMG_ERR_HIP, "independent-set rounds did not terminate");
    hipLaunchKernelGGL(k_mis_m1, g, b, 0, s, n, L.grp.p, L.gci.p, state.p, m1.p);
    hipLaunchKernelGGL(k_mis_m2, g, b, 0, s, n, L.grp.p, L.gci.p, m1.p, state.p);
    hipLaunchKernelGGL(k_mis_e1, g, b, 0, s, n, L.grp.p, L.gci.p, state.p, e1.p);
    zero_flags(H.flags.p + 1, 1, s);
    hipLaunchKernelGGL(k_mis_e2, g, b, 0, s, n, L.grp.p, L.gci.p, e1.p, state.p, H.flags.p + 1);
    AMG_HIP(hipGetLastError());
    sync_flags(H.flags.p + 1, H.h_flags + 1, 1, s);
    if (H.h_flags[1] == 0) break;
  }
  L.mis_rounds = rounds;
  DBuf<int> isroot, rank, agg2;
  isroot.alloc(n + 1);
  rank.alloc(n + 1);
  agg2.alloc(n);
  hipLaunchKernelGGL(k_is_root, dim3(grid_for(n + 1)), b, 0, s, n, state.p, isroot.p);
  exclusive_scan(isroot.p, rank.p, n + 1, s);
  int nagg = read_int(rank.p + n, s);
  hipLaunchKernelGGL(k_agg_phase12, g, b, 0, s, n, L.grp.p, L.gci.p, state.p, rank.p, agg2.p);
  L.agg.alloc(n);
  zero_flags(H.flags.p, 1, s);
  hipLaunchKernelGGL(k_agg_phase3, g, b, 0, s, n, L.grp.p, L.gci.p, agg2.p, L.agg.p, H.flags.p);
  AMG_HIP(hipGetLastError());
  sync_flags(H.flags.p, H.h_flags, 1, s);
  if (H.h_flags[0] & F_NOAGG) throw Error(AMG_ERR_HIP, "aggregation left a node unassigned");
  return nagg;
}

double gershgorin(Hierarchy& H, Level& L, int sy, hipStream_t s) {
  DBuf<unsigned long long> r;
  r.alloc(1);
  AMG_HIP(hipMemsetAsync(r.p, 0, sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_rho, dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, L.rp.p, L.v.p + sy, H.S, L.diagpos.p, r.p);
  AMG_HIP(hipGetLastError());
  unsigned long long bits = 0;
  AMG_HIP(hipMemcpyAsync(&bits, r.p, sizeof(bits), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  double rho;
  std::memcpy(&rho, &bits, sizeof(rho));
  return rho;
}

// Builds P, R and the Galerkin operator of level l+1 (symbolic when
// `symbolic`, else reusing the stored patterns).
void transfer_and_galerkin(Hierarchy& H, size_t l, bool symbolic, hipStream_t s) {
  Level& L = H.lv[l];
  const int n = L.n;
  const int S = H.S;
  const dim3 b(kBlock);
  L.rhoS.resize(S);
  L.omegaPS.resize(S);
  for (int sy = 0; sy < S; ++sy) {
    L.rhoS[sy] = gershgorin(H, L, sy, s);
    L.omegaPS[sy] = (4.0 / 3.0) / L.rhoS[sy];
  }
  L.rho = L.rhoS[0];
  L.omegaP = L.omegaPS[0];
  // P
  if (symbolic) {
    DBuf<int> cnt;
    cnt.alloc(n + 1);
    hipLaunchKernelGGL(k_p_count, dim3(grid_for(n + 1)), b, 0, s, n, L.rp.p, L.ci.p, L.agg.p, cnt.p);
    L.prp.alloc(n + 1);
    exclusive_scan(cnt.p, L.prp.p, n + 1, s);
    L.pnnz = read_int(L.prp.p + n, s);
    L.pci.alloc(L.pnnz);
    L.pv.alloc(L.pnnz * S);
  }
  if (symbolic) {
    hipLaunchKernelGGL(k_p_fill, dim3(grid_for(n)), b, 0, s, n, L.rp.p, L.ci.p, L.v.p, S, L.diagpos.p, L.agg.p,
                       L.omegaPS[0], L.prp.p, L.pci.p, L.pv.p);
    L.pao.alloc(L.pnnz + 1);
    L.pak.alloc(L.nnz);
    L.prow.alloc(L.pnnz);
    hipLaunchKernelGGL(k_pmap_build, dim3(grid_for(n)), b, 0, s, n, L.rp.p, L.ci.p, L.agg.p, L.prp.p, L.pci.p,
                       L.pao.p, L.pak.p, L.prow.p);
  }
  for (int sy = symbolic ? 1 : 0; sy < S; ++sy)
    hipLaunchKernelGGL(k_p_refill, dim3(grid_for(L.pnnz)), b, 0, s, L.pnnz, L.pao.p, L.pak.p, L.prow.p, L.pci.p,
                       L.v.p + sy, S, L.diagpos.p, L.agg.p, L.omegaPS[sy], L.pv.p + sy);
  AMG_HIP(hipGetLastError());
  // R = P^T
  const int nc = L.nagg;
  if (symbolic) {
    DBuf<int> rowid, iota, keys_out, cnt;
    rowid.alloc(L.pnnz);
    iota.alloc(L.pnnz);
    keys_out.alloc(L.pnnz);
    L.rperm.alloc(L.pnnz);
    hipLaunchKernelGGL(k_row_ids, dim3(grid_for(n)), b, 0, s, n, L.prp.p, rowid.p);
    hipLaunchKernelGGL(k_iota, dim3(grid_for(L.pnnz)), b, 0, s, L.pnnz, iota.p);
    int end_bit = 1;
    while ((1ll << end_bit) < (long long)nc) ++end_bit;
    cub_call([&](void* t, size_t& bb) {
      return hipcub::DeviceRadixSort::SortPairs(t, bb, L.pci.p, keys_out.p, iota.p, L.rperm.p, (int)L.pnnz, 0,
                                                end_bit, s);
    }, s);
    cnt.alloc(nc + 1);
    AMG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * (nc + 1), s));
    hipLaunchKernelGGL(k_col_count, dim3(grid_for(L.pnnz)), b, 0, s, L.pnnz, L.pci.p, cnt.p);
    L.rrp.alloc(nc + 1);
    exclusive_scan(cnt.p, L.rrp.p, nc + 1, s);
    L.rci.alloc(L.pnnz);
    L.rv.alloc(L.pnnz * S);
    for (int sy = 0; sy < S; ++sy)
      hipLaunchKernelGGL(k_r_fill, dim3(grid_for(L.pnnz)), b, 0, s, L.pnnz, L.rperm.p, rowid.p, L.pv.p + sy, S,
                         sy == 0 ? L.rci.p : (int*)nullptr, L.rv.p + sy);
    AMG_HIP(hipStreamSynchronize(s));
  } else {
    for (int sy = 0; sy < S; ++sy)
      hipLaunchKernelGGL(k_r_fill, dim3(grid_for(L.pnnz)), b, 0, s, L.pnnz, L.rperm.p, (const int*)nullptr,
                         L.pv.p + sy, S, (int*)nullptr, L.rv.p + sy);
  }
  AMG_HIP(hipGetLastError());
  // product maps for the refreshes (8 bytes per term; the budget keeps each
  // map within 128 bytes per fine-level nonzero: about 1.6 GB in all for
  // the 128^3 Poisson hierarchy)
  const int64_t budget = std::max<int64_t>(16 * (int64_t)H.lv[0].nnz, 1 << 20);
  // AP = A P.  Where rows meet many candidate columns (mean row length of A
  // times that of P at least 64, the coarser levels) the pattern comes from
  // the wavefront hash kernels and the values from the product map; short
  // rows take the thread-per-row merge, which forms the values in the same
  // pass.  Both give the same sorted pattern and the same canonical values.
  const bool wide_ap = symbolic && (double)L.nnz * (double)L.pnnz >= 64.0 * (double)n * (double)n;
  bool apmap = false;
  if (symbolic) {
    DBuf<int> cnt;
    cnt.alloc(n + 1);
    if (wide_ap)
      hipLaunchKernelGGL(k_spgemm_sym_w<0>, dim3(n + 1), dim3(64), 0, s, n, L.rp.p, L.ci.p, L.prp.p, L.pci.p,
                         (const int*)nullptr, cnt.p);
    else
      hipLaunchKernelGGL(k_spgemm_count, dim3(grid_for(n + 1)), b, 0, s, n, L.rp.p, L.ci.p, L.prp.p, L.pci.p, cnt.p);
    L.aprp.alloc(n + 1);
    exclusive_scan(cnt.p, L.aprp.p, n + 1, s);
    L.apnnz = read_int(L.aprp.p + n, s);
    L.apci.alloc(L.apnnz);
    L.apv.alloc(L.apnnz * S);
    if (wide_ap) {
      hipLaunchKernelGGL(k_spgemm_sym_w<1>, dim3(n), dim3(64), 0, s, n, L.rp.p, L.ci.p, L.prp.p, L.pci.p,
                         L.aprp.p, L.apci.p);
      AMG_HIP(hipGetLastError());
      apmap = build_product_map(n, L.apnnz, L.aprp.p, L.apci.p, L.rp.p, L.ci.p, L.prp.p, L.pci.p, budget, L.apmo,
                                L.apm, s);
      if (!apmap) {
        L.apmo.release();
        L.apm.release();
      }
    }
  }
  for (int sy = 0; sy < S; ++sy) {
    if (symbolic && sy == 0 && !wide_ap)
      hipLaunchKernelGGL(k_spgemm_fill, dim3(grid_for(n)), b, 0, s, n, L.rp.p, L.ci.p, L.v.p, L.prp.p, L.pci.p,
                         L.pv.p, L.aprp.p, L.apci.p, L.apv.p, S);
    else if (symbolic ? apmap : L.pmaps)
      hipLaunchKernelGGL(k_pm_apply, dim3(grid_for(L.apnnz)), b, 0, s, L.apnnz, L.apmo.p, L.apm.p, L.v.p + sy,
                         L.pv.p + sy, L.apv.p + sy, S);
    else
      hipLaunchKernelGGL(k_spgemm_fill_entries, dim3(grid_for(L.apnnz)), b, 0, s, n, L.apnnz, L.aprp.p, L.apci.p,
                         L.rp.p, L.ci.p, L.v.p + sy, L.prp.p, L.pci.p, L.pv.p + sy, L.apv.p + sy, S);
  }
  AMG_HIP(hipGetLastError());
  // A_{l+1} = R (A P)
  if (symbolic) {
    H.lv.emplace_back();
  }
  Level& C = H.lv[l + 1];
  Level& Lr = H.lv[l];  // re-fetch: emplace_back may reallocate
  if (symbolic) {
    C.n = nc;
    DBuf<int> cnt;
    cnt.alloc(nc + 1);
    hipLaunchKernelGGL(k_spgemm_sym_w<0>, dim3(nc + 1), dim3(64), 0, s, nc, Lr.rrp.p, Lr.rci.p, Lr.aprp.p,
                       Lr.apci.p, (const int*)nullptr, cnt.p);
    C.rp.alloc(nc + 1);
    exclusive_scan(cnt.p, C.rp.p, nc + 1, s);
    C.nnz = read_int(C.rp.p + nc, s);
    C.ci.alloc(C.nnz);
    C.v.alloc(C.nnz * S);
  }
  if (symbolic) {
    // column pattern of the coarse operator (wavefront per row), values below
    hipLaunchKernelGGL(k_spgemm_sym_w<1>, dim3(nc), dim3(64), 0, s, nc, Lr.rrp.p, Lr.rci.p, Lr.aprp.p, Lr.apci.p,
                       C.rp.p, C.ci.p);
    // (the wide levels built the map of AP above)
    Lr.pmaps = (wide_ap ? apmap
                        : build_product_map(n, Lr.apnnz, Lr.aprp.p, Lr.apci.p, Lr.rp.p, Lr.ci.p, Lr.prp.p, Lr.pci.p,
                                            budget, Lr.apmo, Lr.apm, s)) &&
               build_product_map(nc, C.nnz, C.rp.p, C.ci.p, Lr.rrp.p, Lr.rci.p, Lr.aprp.p, Lr.apci.p, budget,
                                 Lr.cmo, Lr.cm, s);
    if (!Lr.pmaps) {
      Lr.apmo.release();
      Lr.apm.release();
      Lr.cmo.release();
      Lr.cm.release();
    }
  }
  for (int sy = 0; sy < S; ++sy) {
    if (Lr.pmaps)
      hipLaunchKernelGGL(k_pm_apply, dim3(grid_for(C.nnz)), b, 0, s, C.nnz, Lr.cmo.p, Lr.cm.p, Lr.rv.p + sy,
                         Lr.apv.p + sy, C.v.p + sy, S);
    else
      hipLaunchKernelGGL(k_spgemm_fill_entries, dim3(grid_for(C.nnz)), b, 0, s, nc, C.nnz, C.rp.p, C.ci.p, Lr.rrp.p,
                         Lr.rci.p, Lr.rv.p + sy, Lr.aprp.p, Lr.apci.p, Lr.apv.p + sy, C.v.p + sy, S);
  }
  AMG_HIP(hipGetLastError());
}

void precision_copies(Hierarchy& H, hipStream_t s) {
  if (!H.fp32()) return;
  const dim3 b(kBlock);
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level& L = H.lv[l];
    const int64_t S = H.S;
    L.v32.alloc(L.nnz * S);
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(L.nnz * S)), b, 0, s, L.nnz * S, L.v.p, L.v32.p);
    if (l + 1 == H.lv.size()) break;
    if (H.bf16()) {
      L.pbf.alloc(L.pnnz * S);
      L.rbf.alloc(L.pnnz * S);
      hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(L.pnnz * S)), b, 0, s, L.pnnz * S, L.pv.p, L.pbf.p);
      hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(L.pnnz * S)), b, 0, s, L.pnnz * S, L.rv.p, L.rbf.p);
    } else {
      L.pv32.alloc(L.pnnz * S);
      L.rv32.alloc(L.pnnz * S);
      hipLaunchKernelGGL(k_to_f32, dim3(grid_for(L.pnnz * S)), b, 0, s, L.pnnz * S, L.pv.p, L.pv32.p);
      hipLaunchKernelGGL(k_to_f32, dim3(grid_for(L.pnnz * S)), b, 0, s, L.pnnz * S, L.rv.p, L.rv32.p);
    }
  }
  AMG_HIP(hipGetLastError());
}

// Sliced copies of the levels whose rows are short (longest row at most
// kSellMaxW, padding at most 1/8 of the nonzeros; one system only).  The
// pattern part is built once; values are gathered again on every refresh.
void sliced_copies(Hierarchy& H, bool build, hipStream_t s) {
  if (H.S != 1) return;
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level& L = H.lv[l];
    if (build) {
      L.sell = false;
      L.sell_form = 0;
      const int ns = (L.n + 63) / 64;
      DBuf<int> cnt;
      cnt.alloc(ns + 1);
      {
        // offset form first: every slice's offsets fit kSellMaxW slots
        DBuf<int> uoff;
        uoff.alloc((int64_t)ns * kSellMaxW);
        hipLaunchKernelGGL(k_sello_count, dim3((ns + kBlock) / kBlock), dim3(kBlock), 0, s, L.n, ns, L.rp.p, L.ci.p,
                           cnt.p, uoff.p);
        std::vector<int> h(ns + 1);
        AMG_HIP(hipMemcpyAsync(h.data(), cnt.p, sizeof(int) * (ns + 1), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        int64_t tot = 0;
        int wmax = 0;
        for (int i = 0; i < ns; ++i) {
          tot += h[i];
          wmax = std::max(wmax, h[i] / 64);
        }
        if (wmax <= kSellMaxW && tot * 8 <= L.nnz * 9 && tot < (int64_t)INT32_MAX) {
          L.soff.alloc(ns + 1);
          exclusive_scan(cnt.p, L.soff.p, ns + 1, s);
          L.sslot.alloc(tot / 64 + kSellMaxW);  // padded: a slice loads kSellMaxW records at once
          AMG_HIP(hipMemsetAsync(L.sslot.p, 0, L.sslot.bytes(), s));
          L.sperm.alloc(tot);
          hipLaunchKernelGGL(k_sello_fill, dim3((ns + kBlock - 1) / kBlock), dim3(kBlock), 0, s, L.n, ns, L.rp.p,
                             L.ci.p, L.soff.p, uoff.p, L.sslot.p, L.sperm.p);
          L.sv.alloc(tot);
          if (H.fp32()) L.sv32.alloc(tot);
          L.sell_len = tot;
          L.sell = true;
          L.sell_form = 2;
          AMG_HIP(hipStreamSynchronize(s));  // uoff is freed on leaving this scope
        }
      }
    }
    if (build && !L.sell) {
      const int ns = (L.n + 63) / 64;
      DBuf<int> cnt;
      cnt.alloc(ns + 1);
      hipLaunchKernelGGL(k_sell_width, dim3((ns + kBlock) / kBlock), dim3(kBlock), 0, s, L.n, ns, L.rp.p, cnt.p);
      std::vector<int> h(ns + 1);
      AMG_HIP(hipMemcpyAsync(h.data(), cnt.p, sizeof(int) * (ns + 1), hipMemcpyDeviceToHost, s));
      AMG_HIP(hipStreamSynchronize(s));
      int64_t tot = 0;
      int wmax = 0;
      for (int i = 0; i < ns; ++i) {
        tot += h[i];
        wmax = std::max(wmax, h[i] / 64);
      }
      if (wmax > kSellMaxW || tot * 8 > L.nnz * 9 || tot >= (int64_t)INT32_MAX) continue;
      L.soff.alloc(ns + 1);
      exclusive_scan(cnt.p, L.soff.p, ns + 1, s);
      L.sci.alloc(tot);
      L.sperm.alloc(tot);
      hipLaunchKernelGGL(k_sell_fill, dim3((ns * 64 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, L.n, ns, L.rp.p,
                         L.ci.p, L.soff.p, L.sci.p, L.sperm.p);
      L.sv.alloc(tot);
      if (H.fp32()) L.sv32.alloc(tot);
      L.sell_len = tot;
      L.sell = true;
      L.sell_form = 1;
    }
    if (!L.sell) continue;
    hipLaunchKernelGGL(k_sell_vals, dim3(grid_for(L.sell_len)), dim3(kBlock), 0, s, L.sell_len, L.sperm.p, L.v.p,
                       L.sv.p, H.fp32() ? L.sv32.p : nullptr);
  }
  AMG_HIP(hipGetLastError());
}

void alloc_cycle_vectors(Hierarchy& H) {
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level& L = H.lv[l];
    if (H.fp32()) {
      L.x32.alloc(L.n);
      L.b32.alloc(L.n);
      L.r32.alloc(L.n);
    } else {
      L.x64.alloc(L.n);
      L.b64.alloc(L.n);
      L.r64.alloc(L.n);
    }
  }
}

}  // namespace

// ================================================================ public

void validate_csr(int n, int64_t nnz, const int* d_rp, const int* d_ci, int* d_flags, int* h_flags, hipStream_t s) {
  zero_flags(d_flags, 1, s);
  hipLaunchKernelGGL(k_validate, dim3(grid_for(n)), dim3(kBlock), 0, s, n, nnz, d_rp, d_ci, d_flags);
  AMG_HIP(hipGetLastError());
  sync_flags(d_flags, h_flags, 1, s);
  if (h_flags[0] & F_BAD) throw Error(AMG_ERR_INVALID_ARG, "malformed CSR");
  if (h_flags[0] & F_ZERO_DIAG) throw Error(AMG_ERR_ZERO_DIAG, "row without a stored diagonal");
}

uint64_t pattern_hash(int n, int64_t nnz, const int* d_rp, const int* d_ci, int* d_flags, int* h_flags,
                      hipStream_t s) {
  AMG_HIP(hipMemsetAsync(d_flags, 0, 8, s));
  hipLaunchKernelGGL(k_hash, dim3(1024), dim3(kBlock), 0, s, n, nnz, d_rp, d_ci, (unsigned long long*)d_flags);
  AMG_HIP(hipGetLastError());
  sync_flags(d_flags, h_flags, 2, s);
  uint64_t h;
  std::memcpy(&h, h_flags, 8);
  return h;
}

bool pattern_equal(const Hierarchy& H, const int* d_rp, const int* d_ci, int* d_flags, int* h_flags, hipStream_t s) {
  const Level& L = H.lv[0];
  zero_flags(d_flags, 1, s);
  hipLaunchKernelGGL(k_diff<int>, dim3(1024), dim3(kBlock), 0, s, (int64_t)L.n + 1, d_rp, L.rp.p, d_flags);
  hipLaunchKernelGGL(k_diff<int>, dim3(1024), dim3(kBlock), 0, s, L.nnz, d_ci, L.ci.p, d_flags);
  AMG_HIP(hipGetLastError());
  sync_flags(d_flags, h_flags, 1, s);
  return !(h_flags[0] & F_MISMATCH);
}

bool values_equal(const Hierarchy& H, const double* d_val, int* d_flags, int* h_flags, hipStream_t s) {
  const Level& L = H.lv[0];
  zero_flags(d_flags, 1, s);
  hipLaunchKernelGGL(k_diff_bits, dim3(1024), dim3(kBlock), 0, s, L.nnz * H.S, d_val, L.v.p, d_flags);
  AMG_HIP(hipGetLastError());
  sync_flags(d_flags, h_flags, 1, s);
  return !(h_flags[0] & F_MISMATCH);
}

void build_hierarchy(Hierarchy& H, const int* d_rp, const int* d_ci, const double* d_val, hipStream_t s) {
  H.lv.clear();
  H.lv.emplace_back();
  {
    Level& L0 = H.lv[0];
    L0.n = H.n;
    L0.nnz = H.nnz;
    L0.rp.alloc(H.n + 1);
    L0.ci.alloc(H.nnz);
    L0.v.alloc(H.nnz * H.S);
    AMG_HIP(hipMemcpyAsync(L0.rp.p, d_rp, L0.rp.bytes(), hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(L0.ci.p, d_ci, L0.ci.bytes(), hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(L0.v.p, d_val, L0.v.bytes(), hipMemcpyDeviceToDevice, s));
  }
  for (size_t l = 0;; ++l) {
    Level& L = H.lv[l];
    level_numerics(H, L, s);
    bool last = L.n <= H.prm.max_coarse || (int)(l + 1) >= H.prm.max_levels || !H.prm.precondition;
    if (!last) {
      strength_graph(H, L, s);
      L.nagg = aggregate(H, L, s);
      if (10LL * L.nagg > 9LL * L.n) last = true;
    }
    if (last) {
      L.agg.release();
      L.nagg = 0;
      break;
    }
    transfer_and_galerkin(H, l, true, s);
  }
  if (H.prm.precondition) coarse_setup(H, s);
  precision_copies(H, s);
  sliced_copies(H, true, s);
  alloc_cycle_vectors(H);
  choose_shapes(H, s);
  alloc_solve_workspace(H);
  H.small_checked = false;
  small_solve_ok(H);
  AMG_HIP(hipStreamSynchronize(s));
}

// Pattern of A^T by a stable radix sort of the entries by column: entry t of
// A^T is entry perm[t] of A, and within a row of A^T the source rows ascend
// (the stable sort keeps A's row order), so the result is a sorted CSR
// pattern (with every diagonal stored when A has them).
void transpose_csr_pattern(int n, int64_t nnz, const int* rp, const int* ci, DBuf<int>& trp, DBuf<int>& tci,
                           DBuf<int>& perm, hipStream_t s) {
  const dim3 b(kBlock);
  DBuf<int> rowid, iota, keys_out, cnt;
  rowid.alloc(std::max<int64_t>(nnz, 1));
  iota.alloc(std::max<int64_t>(nnz, 1));
  keys_out.alloc(std::max<int64_t>(nnz, 1));
  perm.alloc(std::max<int64_t>(nnz, 1));
  hipLaunchKernelGGL(k_row_ids, dim3(grid_for(n)), b, 0, s, n, rp, rowid.p);
  hipLaunchKernelGGL(k_iota, dim3(grid_for(nnz)), b, 0, s, nnz, iota.p);
  int end_bit = 1;
  while ((1ll << end_bit) < (long long)n) ++end_bit;
  cub_call([&](void* t, size_t& bb) {
    return hipcub::DeviceRadixSort::SortPairs(t, bb, ci, keys_out.p, iota.p, perm.p, (int)nnz, 0, end_bit, s);
  }, s);
  cnt.alloc(n + 1);
  AMG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * (n + 1), s));
  hipLaunchKernelGGL(k_col_count, dim3(grid_for(nnz)), b, 0, s, nnz, ci, cnt.p);
  trp.alloc(n + 1);
  exclusive_scan(cnt.p, trp.p, n + 1, s);
  tci.alloc(std::max<int64_t>(nnz, 1));
  hipLaunchKernelGGL(k_t_cols, dim3(grid_for(nnz)), b, 0, s, nnz, perm.p, rowid.p, tci.p);
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipStreamSynchronize(s));
}

void convert_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s) {
  const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 16384);
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid), dim3(kBlock), 0, s, n, in, out);
  AMG_HIP(hipGetLastError());
}

// A^T of the level-0 matrix (pattern, entry map, values) for the adjoint of
// a nonsymmetric A.
void transpose_pattern(Hierarchy& H, hipStream_t s) {
  const Level& L = H.lv[0];
  transpose_csr_pattern(L.n, L.nnz, L.rp.p, L.ci.p, H.trp, H.tci, H.tperm, s);
  H.tval.alloc(L.nnz);
  transpose_values(H, s);
  AMG_HIP(hipStreamSynchronize(s));
}

// Values of A^T in its entry order from A's current values.
void transpose_values(Hierarchy& H, hipStream_t s) {
  const Level& L = H.lv[0];
  hipLaunchKernelGGL(k_r_fill, dim3(grid_for(L.nnz)), dim3(kBlock), 0, s, L.nnz, H.tperm.p, (const int*)nullptr,
                     L.v.p, 1, (int*)nullptr, H.tval.p);
  AMG_HIP(hipGetLastError());
}

void refresh_hierarchy(Hierarchy& H, const double* d_val, hipStream_t s) {
  if (H.prm.theta > 0.0) {
    // With a strength threshold the strength graph, hence the aggregates and
    // every coarse pattern, depend on the values: the hierarchy is set up
    // again from the stored pattern, so it never depends on the values it was
    // first built with.
    DBuf<int> rp, ci;
    rp.alloc(H.n + 1);
    ci.alloc(H.nnz);
    AMG_HIP(hipMemcpyAsync(rp.p, H.lv[0].rp.p, rp.bytes(), hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(ci.p, H.lv[0].ci.p, ci.bytes(), hipMemcpyDeviceToDevice, s));
    H.bt.W = 0;  // batched workspaces follow the (possibly different) levels
    build_hierarchy(H, rp.p, ci.p, d_val, s);
    return;
  }
  Level& L0 = H.lv[0];
  AMG_HIP(hipMemcpyAsync(L0.v.p, d_val, L0.v.bytes(), hipMemcpyDeviceToDevice, s));
  for (size_t l = 0; l < H.lv.size(); ++l) {
    level_numerics(H, H.lv[l], s);
    if (l + 1 == H.lv.size()) break;
    transfer_and_galerkin(H, l, false, s);
  }
  if (H.prm.precondition) coarse_setup(H, s);
  precision_copies(H, s);
  sliced_copies(H, false, s);
  AMG_HIP(hipStreamSynchronize(s));
}

}  // namespace amg
