// Matrix-free assembly by graph-colored probing (Section 2.1, "Matrix-free
// operator support"; Curtis, Powell and Reid 1974).  Given the sparsity
// pattern of an operator x -> A x, the columns are partitioned into colors
// so that no two columns of a color share a row; applying the operator to
// the 0/1 probe vector of each color then yields every stored entry, one
// operator application per color:  a_ij = (A v_color(j))_i.
//
// Coloring: the greedy coloring in decreasing node-key order (each column
// takes the smallest color not used by an already colored column sharing a
// row), computed by Jones-Plassmann rounds with the same fixed keys as the
// aggregation.  In a round, every uncolored column whose key is the largest
// among the uncolored columns it shares a row with takes the smallest color
// absent from its (already colored) conflicting columns.  Two such columns
// never conflict, and a column is colored exactly when all conflicting
// columns of larger key are, so the result equals the sequential greedy
// coloring column for column.
#include <algorithm>

#include "amg_internal.hpp"

namespace amg {
namespace {

inline int grid_of(int64_t items) { return (int)std::max<int64_t>(1, (items + kBlock - 1) / kBlock); }

// m1[i] = 1 + largest key among the uncolored columns of row i (0: none).
__global__ void k_color_rowmax(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                               const int* __restrict__ color, unsigned long long* __restrict__ m1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long best = 0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = ci[k];
    if (color[j] < 0) best = max(best, (unsigned long long)mis_key(j) + 1);
  }
  m1[i] = best;
}

// Uncolored column j (rows from the transposed pattern) that holds the
// largest key over all rows it appears in takes the smallest color that no
// column sharing one of those rows has; flags[0] |= 1 while columns remain,
// flags[1] = max(color) + 1.
__global__ void k_color_pick(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                             const int* __restrict__ trp, const int* __restrict__ tci,
                             const unsigned long long* __restrict__ m1, int* __restrict__ color, int* flags) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || color[j] >= 0) return;
  unsigned long long best = 0;
  for (int a = trp[j]; a < trp[j + 1]; ++a) best = max(best, m1[tci[a]]);
  if (best != (unsigned long long)mis_key(j) + 1) {
    atomicOr(flags, 1);
    return;
  }
  int c = -1;
  for (int base = 0; c < 0; base += 64) {
    unsigned long long used = 0;
    for (int a = trp[j]; a < trp[j + 1]; ++a) {
      const int i = tci[a];
      for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int cc = color[ci[k]] - base;
        if (cc >= 0 && cc < 64) used |= 1ull << cc;
      }
    }
    if (~used) c = base + __builtin_ctzll(~used);
  }
  color[j] = c;
  atomicMax(flags + 1, c + 1);
}

__global__ void k_fill_i32(int64_t m, int v, int* __restrict__ a) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < m) a[t] = v;
}

// flags[0] |= 2 for a color outside [0, ncolors).
__global__ void k_check_colors(int n, const int* __restrict__ color, int ncolors, int* flags) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n && (color[j] < 0 || color[j] >= ncolors)) atomicOr(flags, 2);
}

// V[c][j] = 1 if column j has color c, else 0 ([ncolors][n]).
__global__ void k_probe_vectors(int n, int ncolors, const int* __restrict__ color, double* __restrict__ V) {
  const int64_t m = (int64_t)ncolors * n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t / n), j = (int)(t - (int64_t)c * n);
    V[t] = color[j] == c ? 1.0 : 0.0;
  }
}

// val[k] = Y[color(col k)][row k] (thread per row).
__global__ void k_probe_assemble(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                 const int* __restrict__ color, const double* __restrict__ Y,
                                 double* __restrict__ val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) val[k] = Y[(int64_t)color[ci[k]] * n + i];
}

__global__ void k_zero_f64(int64_t m, double* __restrict__ a) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
    a[t] = 0.0;
}

// Adjoint of the assembly: dY[color(col k)][row k] = dval[k] (dY zeroed first;
// each (color, row) slot receives at most one entry).
__global__ void k_probe_scatter(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                const int* __restrict__ color, const double* __restrict__ dval,
                                double* __restrict__ dY) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) dY[(int64_t)color[ci[k]] * n + i] = dval[k];
}

void read_flags(int* d_flags, int* h_flags, int count, hipStream_t s) {
  AMG_HIP(hipMemcpyAsync(h_flags, d_flags, sizeof(int) * count, hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
}

void check_colors(int n, const int* color, int ncolors, int* d_flags, int* h_flags, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int64_t)1, 0, d_flags);
  hipLaunchKernelGGL(k_check_colors, dim3(grid_of(n)), dim3(kBlock), 0, s, n, color, ncolors, d_flags);
  AMG_HIP(hipGetLastError());
  read_flags(d_flags, h_flags, 1, s);
  if (h_flags[0] & 2) throw Error(AMG_ERR_INVALID_ARG, "color outside [0, ncolors)");
}

}  // namespace

int color_columns(int n, int64_t nnz, const int* rp, const int* ci, int* color, int* d_flags, int* h_flags,
                  hipStream_t s) {
  DBuf<int> trp, tci, perm;
  transpose_csr_pattern(n, nnz, rp, ci, trp, tci, perm, s);
  DBuf<unsigned long long> m1;
  m1.alloc(n);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(n)), dim3(kBlock), 0, s, (int64_t)n, -1, color);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int64_t)2, 0, d_flags);
  for (int round = 0;; ++round) {
    if (round > n + 1) throw Error(AMG_ERR_HIP, "coloring rounds did not terminate");
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int64_t)1, 0, d_flags);
    hipLaunchKernelGGL(k_color_rowmax, dim3(grid_of(n)), dim3(kBlock), 0, s, n, rp, ci, color, m1.p);
    hipLaunchKernelGGL(k_color_pick, dim3(grid_of(n)), dim3(kBlock), 0, s, n, rp, ci, trp.p, tci.p, m1.p, color,
                       d_flags);
    AMG_HIP(hipGetLastError());
    read_flags(d_flags, h_flags, 2, s);
    if (!(h_flags[0] & 1)) break;
  }
  return h_flags[1];
}

void probe_vectors(int n, const int* color, int ncolors, double* V, int* d_flags, int* h_flags, hipStream_t s) {
  check_colors(n, color, ncolors, d_flags, h_flags, s);
  const int64_t m = (int64_t)ncolors * n;
  hipLaunchKernelGGL(k_probe_vectors, dim3((int)std::min<int64_t>(grid_of(m), 65536)), dim3(kBlock), 0, s, n,
                     ncolors, color, V);
  AMG_HIP(hipGetLastError());
}

void probe_assemble(int n, const int* rp, const int* ci, const int* color, int ncolors, const double* Y, double* val,
                    int* d_flags, int* h_flags, hipStream_t s) {
  check_colors(n, color, ncolors, d_flags, h_flags, s);
  hipLaunchKernelGGL(k_probe_assemble, dim3(grid_of(n)), dim3(kBlock), 0, s, n, rp, ci, color, Y, val);
  AMG_HIP(hipGetLastError());
}

void probe_scatter(int n, const int* rp, const int* ci, const int* color, int ncolors, const double* dval,
                   double* dY, int* d_flags, int* h_flags, hipStream_t s) {
  check_colors(n, color, ncolors, d_flags, h_flags, s);
  const int64_t m = (int64_t)ncolors * n;
  hipLaunchKernelGGL(k_zero_f64, dim3((int)std::min<int64_t>(grid_of(m), 65536)), dim3(kBlock), 0, s, m, dY);
  hipLaunchKernelGGL(k_probe_scatter, dim3(grid_of(n)), dim3(kBlock), 0, s, n, rp, ci, color, dval, dY);
  AMG_HIP(hipGetLastError());
}

}  // namespace amg
