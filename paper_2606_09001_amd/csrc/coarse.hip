// Coarsest-level direct solve: dense FP64 Cholesky factorization of the
// coarsest Galerkin matrix (right-looking, 16-column panels; the rank-16
// trailing updates and the inverse product run on the FP64 matrix cores,
// v_mfma_f64_16x16x4f64), followed by the explicit inverse so that the
// per-cycle coarse solve is one dense matrix-vector product.  A nonsymmetric
// hierarchy factors the coarsest matrix by LU with partial pivoting instead
// (Gaussian elimination with row interchanges, one column per step, every
// entry updated by one rounded product and one rounded difference per step,
// in the same order as the sequential definition) and stores the transposed
// inverse, which the coarse-solve kernel reads the same way.
#include <algorithm>

#include "amg_internal.hpp"

namespace amg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kCoBlock = 256;  // one workgroup, four wavefronts

// Dense m x m (row-major) copy of the CSR matrix; padding rows/cols get the identity.
__global__ void k_densify(int n, int m, double* __restrict__ W) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t mm = (int64_t)m * m;
  for (int64_t e = t; e < mm; e += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(e / m), j = (int)(e % m);
    W[e] = (i == j && i >= n) ? 1.0 : 0.0;
  }
}

__global__ void k_scatter(int n, int m, const int* __restrict__ rp, const int* __restrict__ ci,
                          const double* __restrict__ v, int vs, double* __restrict__ W) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) W[(int64_t)i * m + ci[k]] = v[(int64_t)k * vs];
}

// C_tile(I,J) += A_tile * B_tile^T over 16 columns [k0, k0+16) of row
// blocks I and J of X (row-major, leading dimension m), with A = sgn * X.
// Operand layout of v_mfma_f64_16x16x4f64 (wave64): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; its four accumulator registers hold
// D[4*e + l/16][l%16], e = 0..3 (one row group per register).
__device__ inline void mfma_tile_update(double* __restrict__ W, int m, int I, int J, const double* __restrict__ X,
                                        int ldx, int k0, double sgn) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, q = l >> 4;
  d4 acc;
#pragma unroll
  for (int e = 0; e < 4; ++e) acc[e] = W[(int64_t)(I * 16 + 4 * e + q) * m + J * 16 + r];
#pragma unroll
  for (int kk = 0; kk < 16; kk += 4) {
    double a = sgn * X[(int64_t)(I * 16 + r) * ldx + k0 + kk + q];
    double b = X[(int64_t)(J * 16 + r) * ldx + k0 + kk + q];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) W[(int64_t)(I * 16 + 4 * e + q) * m + J * 16 + r] = acc[e];
}

// In-place Cholesky W = L L^T (lower triangle), one workgroup.  Panel of 16
// columns: column-by-column right-looking factorization restricted to the
// panel, then a rank-16 update of the trailing lower triangle on MFMA.
__global__ void __launch_bounds__(kCoBlock) k_cholesky(int m, double* __restrict__ W, int* flags) {
  const int tid = threadIdx.x;
  const int wave = tid >> 6, nwaves = kCoBlock / 64;
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int kb = 0; kb < m; kb += 16) {
    for (int k = kb; k < kb + 16; ++k) {
      if (tid == 0) {
        double d = W[(int64_t)k * m + k];
        if (!(d > 0.0)) { s_bad = 1; d = 1.0; }
        W[(int64_t)k * m + k] = sqrt(d);
      }
      __syncthreads();
      const double lkk = W[(int64_t)k * m + k];
      for (int i = k + 1 + tid; i < m; i += kCoBlock) W[(int64_t)i * m + k] /= lkk;
      __syncthreads();
      // update the remaining panel columns j in (k, kb+16), rows i >= j
      const int ncols = kb + 16 - (k + 1);
      if (ncols > 0) {
        const int64_t rows = m - (k + 1);
        for (int64_t t = tid; t < rows * ncols; t += kCoBlock) {
          int i = k + 1 + (int)(t / ncols);
          int j = k + 1 + (int)(t % ncols);
          if (i >= j) W[(int64_t)i * m + j] -= W[(int64_t)i * m + k] * W[(int64_t)j * m + k];
        }
      }
      __syncthreads();
    }
    // trailing update of tiles (I, J), kb/16 < J <= I
    const int T0 = kb / 16 + 1, T = m / 16;
    const int nt = T - T0;
    const int ntiles = nt * (nt + 1) / 2;
    for (int t = wave; t < ntiles; t += nwaves) {
      // t -> (I, J) with J <= I
      int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while ((a + 1) * (a + 2) / 2 <= t) ++a;
      while (a * (a + 1) / 2 > t) --a;
      int I = T0 + a, J = T0 + (t - a * (a + 1) / 2);
      mfma_tile_update(W, m, I, J, W, m, kb, -1.0);
    }
    __syncthreads();
  }
  // zero the strict upper triangle
  for (int64_t e = tid; e < (int64_t)m * m; e += kCoBlock) {
    int i = (int)(e / m), j = (int)(e % m);
    if (j > i) W[e] = 0.0;
  }
  if (tid == 0 && s_bad) atomicOr(flags, 1);
}

// Column solves of the triangular inverses: one wavefront per column, the
// column in LDS, each row's dot product spread over the wavefront (lane-
// strided partial sums, then a fixed butterfly).
constexpr int kTriWaves = 2;

// Makes the LDS writes of a wavefront visible to its other lanes.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Linv = L^-1 by forward substitution: Linv[i][j] = -(sum_{j<=k<i} L[i][k]
// Linv[k][j]) / L[i][i], Linv[j][j] = 1 / L[j][j].
__global__ void __launch_bounds__(64 * kTriWaves) k_tri_inverse(int m, const double* __restrict__ L,
                                                                double* __restrict__ Linv) {
  __shared__ double s_col[kTriWaves][AMG_MAX_DENSE_COARSE];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int j = blockIdx.x * kTriWaves + w;
  if (j >= m) return;  // the whole wavefront
  double* col = s_col[w];
  for (int i = l; i < m; i += 64) col[i] = 0.0;
  wave_lds_sync();
  if (l == 0) col[j] = 1.0 / L[(int64_t)j * m + j];
  wave_lds_sync();
  for (int i = j + 1; i < m; ++i) {
    const double* Li = L + (int64_t)i * m;
    double s = 0.0;
    for (int k = j + l; k < i; k += 64) s += Li[k] * col[k];
    s = wave_sum(s);
    if (l == 0) col[i] = -s / Li[i];
    wave_lds_sync();
  }
  for (int i = l; i < m; i += 64) Linv[(int64_t)i * m + j] = col[i];
}

// Transpose (m x m): Y = X^T.
__global__ void k_transpose(int m, const double* __restrict__ X, double* __restrict__ Y) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  int i = (int)(e / m), j = (int)(e % m);
  Y[(int64_t)j * m + i] = X[e];
}

// inv = Linv^T Linv = X X^T with X = Linv^T (row-major): tile (I, J) sums
// over all 16-column panels of X.  One wavefront per tile.
__global__ void k_gram(int m, const double* __restrict__ X, double* __restrict__ G) {
  const int T = m / 16;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wave >= T * T) return;
  const int I = wave / T, J = wave % T;
  const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < m; k0 += 16) {
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      double a = X[(int64_t)(I * 16 + r) * m + k0 + kk + q];
      double b = X[(int64_t)(J * 16 + r) * m + k0 + kk + q];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) G[(int64_t)(I * 16 + 4 * e + q) * m + J * 16 + r] = acc[e];
}

constexpr int kLuBlock = 1024;  // one workgroup, sixteen wavefronts

// In-place LU with partial pivoting of the m x m row-major W.  Step k: the
// pivot is the first row i >= k of largest |w_ik| (lowest index on ties), the
// two rows are exchanged over the full width, the multipliers w_ik / w_kk go
// below the diagonal and every w_ij (i, j > k) becomes w_ij - w_ik * w_kj.
// A zero (or NaN) pivot column sets flags bit 0.  Padding rows/columns are
// the identity and are never chosen for a column of the matrix.
__global__ void __launch_bounds__(kLuBlock) k_lu(int m, double* __restrict__ W, int* __restrict__ piv,
                                                 int* flags) {
  const int tid = threadIdx.x;
  constexpr int NW = kLuBlock / 64;
  __shared__ double s_best[NW];
  __shared__ int s_row[NW];
  __shared__ int s_p;
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    // pivot search: thread-local first maximum, then (value, lowest row)
    double best = -1.0;
    int br = m;
    bool nan = false;
    for (int i = k + tid; i < m; i += kLuBlock) {
      const double a = fabs(W[(int64_t)i * m + k]);
      nan |= !(a == a);
      if (a > best) { best = a; br = i; }
    }
    if (nan) s_bad = 1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int orow = __shfl_xor(br, o, 64);
      if (ob > best || (ob == best && orow < br)) { best = ob; br = orow; }
    }
    if ((tid & 63) == 0) { s_best[tid >> 6] = best; s_row[tid >> 6] = br; }
    __syncthreads();
    if (tid == 0) {
      double b = s_best[0];
      int r = s_row[0];
      for (int w = 1; w < NW; ++w)
        if (s_best[w] > b || (s_best[w] == b && s_row[w] < r)) { b = s_best[w]; r = s_row[w]; }
      if (!(b > 0.0)) { s_bad = 1; r = k; }
      s_p = r;
      piv[k] = r;
    }
    __syncthreads();
    const int p = s_p;
    if (p != k)
      for (int j = tid; j < m; j += kLuBlock) {
        const double t = W[(int64_t)k * m + j];
        W[(int64_t)k * m + j] = W[(int64_t)p * m + j];
        W[(int64_t)p * m + j] = t;
      }
    __syncthreads();
    const double ukk = W[(int64_t)k * m + k];
    const bool ok = ukk != 0.0;
    for (int i = k + 1 + tid; i < m; i += kLuBlock) W[(int64_t)i * m + k] = ok ? W[(int64_t)i * m + k] / ukk : 0.0;
    __syncthreads();
    const int r = m - (k + 1);
    for (int64_t e = tid; e < (int64_t)r * r; e += kLuBlock) {
      const int i = k + 1 + (int)(e / r), j = k + 1 + (int)(e % r);
      const double prod = W[(int64_t)i * m + k] * W[(int64_t)k * m + j];
      W[(int64_t)i * m + j] = W[(int64_t)i * m + j] - prod;
    }
    __syncthreads();
  }
  if (tid == 0 && s_bad) atomicOr(flags, 1);
}

// Row j of invT = column j of A^-1: y = P e_j (the recorded exchanges in
// order move the single 1 of e_j), unit-lower forward substitution
// y_i -= sum_{q<i} l_iq y_q, then upper back substitution
// y_i = (y_i - sum_{q>i} u_iq y_q) / u_ii.  One wavefront per column (as
// k_tri_inverse).
__global__ void __launch_bounds__(64 * kTriWaves) k_lu_inverse_t(int m, const double* __restrict__ LU,
                                                                 const int* __restrict__ piv,
                                                                 double* __restrict__ invT) {
  __shared__ double s_y[kTriWaves][AMG_MAX_DENSE_COARSE];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int j = blockIdx.x * kTriWaves + w;
  if (j >= m) return;  // the whole wavefront
  double* y = s_y[w];
  int pos = j;
  for (int k = 0; k < m; ++k) {
    const int p = piv[k];
    if (pos == k) pos = p;
    else if (pos == p) pos = k;
  }
  for (int i = l; i < m; i += 64) y[i] = i == pos ? 1.0 : 0.0;
  wave_lds_sync();
  for (int i = pos + 1; i < m; ++i) {  // entries before pos stay zero
    const double* Ri = LU + (int64_t)i * m;
    double s = 0.0;
    for (int q = pos + l; q < i; q += 64) s += Ri[q] * y[q];
    s = wave_sum(s);
    if (l == 0) y[i] = y[i] - s;
    wave_lds_sync();
  }
  for (int i = m - 1; i >= 0; --i) {
    const double* Ri = LU + (int64_t)i * m;
    double s = 0.0;
    for (int q = i + 1 + l; q < m; q += 64) s += Ri[q] * y[q];
    s = wave_sum(s);
    if (l == 0) y[i] = (y[i] - s) / Ri[i];
    wave_lds_sync();
  }
  for (int i = l; i < m; i += 64) invT[(int64_t)j * m + i] = y[i];
}

__global__ void k_inv_to_f32(int64_t mm, const double* __restrict__ a, float* __restrict__ b) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < mm) b[t] = (float)a[t];
}

}  // namespace

void coarse_setup(Hierarchy& H, hipStream_t s) {
  Level& L = H.lv.back();
  Coarse& C = H.co;
  if (L.n > AMG_MAX_DENSE_COARSE) throw Error(AMG_ERR_COARSE_TOO_LARGE, "coarsest level too large");
  C.n = L.n;
  C.m = (L.n + 15) / 16 * 16;
  const int m = C.m;
  const int S = H.S;
  const int64_t mm = (int64_t)m * m;
  C.L.alloc(mm * S);
  C.inv.alloc(mm * S);
  C.work.alloc(mm);
  const bool lu = !H.prm.symmetric;
  if (lu) C.piv.alloc((int64_t)m * S);
  const int grid = (int)std::min<int64_t>((mm + kBlock - 1) / kBlock, 4096);
  const int T = m / 16;
  AMG_HIP(hipMemsetAsync(H.flags.p, 0, sizeof(int), s));
  // one dense factorization (and inverse) per system sharing the pattern
  for (int sy = 0; sy < S; ++sy) {
    double* Ls = C.L.p + sy * mm;
    double* Is = C.inv.p + sy * mm;
    hipLaunchKernelGGL(k_densify, dim3(grid), dim3(kBlock), 0, s, C.n, m, Ls);
    hipLaunchKernelGGL(k_scatter, dim3((C.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, C.n, m, L.rp.p, L.ci.p,
                       L.v.p + sy, S, Ls);
    if (lu) {
      int* ps = C.piv.p + (int64_t)sy * m;
      hipLaunchKernelGGL(k_lu, dim3(1), dim3(kLuBlock), 0, s, m, Ls, ps, H.flags.p);
      hipLaunchKernelGGL(k_lu_inverse_t, dim3((m + kTriWaves - 1) / kTriWaves), dim3(64 * kTriWaves), 0, s, m, Ls,
                         ps, Is);
      continue;
    }
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(kCoBlock), 0, s, m, Ls, H.flags.p);
    hipLaunchKernelGGL(k_tri_inverse, dim3((m + kTriWaves - 1) / kTriWaves), dim3(64 * kTriWaves), 0, s, m, Ls,
                       Is);
    hipLaunchKernelGGL(k_transpose, dim3((int)((mm + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, m, Is, C.work.p);
    hipLaunchKernelGGL(k_gram, dim3((T * T * 64 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, m, C.work.p, Is);
  }
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipMemcpyAsync(H.h_flags, H.flags.p, sizeof(int), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  if (H.h_flags[0])
    throw Error(AMG_ERR_BREAKDOWN, lu ? "coarsest matrix is singular" : "coarsest matrix is not positive definite");
  if (H.fp32()) {
    C.inv32.alloc(mm * S);
    hipLaunchKernelGGL(k_inv_to_f32, dim3((int)((mm * S + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, mm * S,
                       C.inv.p, C.inv32.p);
  }
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipStreamSynchronize(s));
}

}  // namespace amg
