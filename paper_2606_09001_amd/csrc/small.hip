// Whole-solve PCG in one workgroup, for hierarchies small enough to live in
// one compute unit: two levels (the fine level and a dense coarsest level),
// at most 1024 fine rows.  The per-kernel path launches about twenty kernels
// per iteration, so a 1024-unknown solve is bound by launch and
// synchronisation latency, not by bytes.  Here one workgroup of 1024 threads
// (thread i owns fine row i) runs every iteration, restart and the final
// true-residual check in a single launch:
//   - the CG vectors and the cycle vectors live in LDS, so every gather of
//     a sweep is an LDS read;
//   - each thread keeps its rows of A_0 in registers for the whole solve
//     (A_0 is applied three times per iteration);
//   - P_0 and R_0 are staged in LDS once per solve; R_0 is applied with a
//     group of lanes per coarse row;
//   - the explicit coarse inverse is read from global memory (L2) by
//     wavefront column blocks: a wave takes a block of columns, so each
//     column's loads have a wave-uniform base and are coalesced over rows,
//     and the block sums are added per row in wave order;
//   - dot products are fixed-order block reductions (wave butterfly, then the
//     16 wave sums in order), so a solve is bitwise reproducible.
// The method is the one of pcg_solve: PCG from x0 = 0, damped-Jacobi (or L1)
// V(1,1) cycle with R = P^T and the exact coarse solve, recursive-residual
// stopping, true-residual verification with at most 5 restarts, flexible
// beta = -<z, q>/<p, q> when requested.  Rows are summed in stored order and
// q = A p is formed directly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "amg_internal.hpp"

namespace amg {
namespace {

constexpr int kST = 512;         // threads of the workgroup
constexpr int kSR = 2;           // fine rows per thread (rows t and t + kST)
constexpr int kSN = kST * kSR;   // largest fine level
constexpr int kSRow = 8;         // entries per row of A_0
constexpr int kSCoarse = 256;    // largest padded coarsest level
constexpr int kSPCap = 3200;     // entries of P_0 (and of R_0 = P_0^T) staged in LDS
constexpr int kSWaves = kST / 64;
constexpr int kSPairs = kSCoarse / 128;  // row-pair chunks per lane in the inverse product
constexpr int kSCols = 4;        // inverse columns per step (loads in flight: kSCols x rows per lane)

struct SmallArgs {
  int n, nc, m, lgR, maxiter, flexible;
  double tol;
  const int* arp;
  const int* aci;
  const double* av;
  const double* sw;
  const int* prp;
  const int* pci;
  const double* pv;
  const int* rrp;
  const int* rci;
  const double* rv;
  const double* inv;
  const double* b;
  double* x;
  Ctl* ctl;
};

// Keeps the compiler from moving memory operations across this point: the
// matrix loads of a phase are loop-invariant, and hoisting all of them out
// of the iteration loop would keep every phase's operands live in registers
// at once.
__device__ inline void phase_fence() { asm volatile("" ::: "memory"); }

// Returns v through an empty asm statement: the compiler cannot treat values
// derived from it as loop-invariant, so the loads they address stay in their
// phase instead of being hoisted out of the iteration loop.
__device__ inline int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// DPP move of a double within rows of 16 lanes (pattern `ctrl`).
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the wavefront, every lane gets the same bits: partner sums within
// quads (lane ^ 1, lane ^ 2), then the mirrored half row and row (lane i with
// 7 - i and 15 - i of its group), then across rows (lane ^ 16, lane ^ 32).
// Each step adds two equal-rank partial sums, so all lanes agree.
__device__ inline double wave_sum_fast(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Sum of v over the workgroup in a fixed order; every thread gets the total.
// `red` must not be reused before the next barrier.
__device__ inline double wg_sum(double v, double* red) {
  v = wave_sum_fast(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int k = 1; k < kST / 64; ++k) s += red[k];
  return s;
}

__global__ void __launch_bounds__(kST) k_pcg_small(SmallArgs a) {
  __shared__ double s_r[kSN], s_z[kSN], s_p[kSN], s_q[kSN], s_xc[kSN], s_rc[kSN];
  __shared__ double s_b1[kSCoarse], s_x1[kSCoarse];
  __shared__ double s_gp[kSWaves][kSCoarse];
  __shared__ double s_red[4][kST / 64];
  __shared__ int s_prp[kSN + 1], s_rrp[kSCoarse + 1];
  __shared__ int s_pci[kSPCap], s_rci[kSPCap];
  __shared__ double s_pv[kSPCap], s_rv[kSPCap];
  const int t = threadIdx.x;
  // P_0 and R_0 into LDS (their entry counts are at most kSPCap)
  const int pnz = a.prp[a.n];
  for (int i = t; i <= a.n; i += kST) s_prp[i] = a.prp[i];
  for (int i = t; i <= a.nc; i += kST) s_rrp[i] = a.rrp[i];
  for (int k = t; k < pnz; k += kST) {
    s_pci[k] = a.pci[k];
    s_pv[k] = a.pv[k];
    s_rci[k] = a.rci[k];
    s_rv[k] = a.rv[k];
  }
  // this thread's rows t + q kST: their rows of A_0 in registers (indices
  // clamped into the row; entries past the row's length are masked out of
  // every sum), their smoother weights, right-hand side and iterate
  int row[kSR], na[kSR], acol[kSR][kSRow];
  bool own[kSR];
  double aval[kSR][kSRow], swi[kSR], bi[kSR], xi[kSR];
#pragma unroll
  for (int q = 0; q < kSR; ++q) {
    own[q] = t + q * kST < a.n;
    row[q] = own[q] ? t + q * kST : a.n - 1;
    const int ka = a.arp[row[q]];
    na[q] = own[q] ? a.arp[row[q] + 1] - ka : 0;
#pragma unroll
    for (int j = 0; j < kSRow; ++j) {
      const int k = ka + min(j, max(na[q] - 1, 0));
      acol[q][j] = a.aci[k];
      aval[q][j] = a.av[k];
    }
    swi[q] = a.sw[row[q]];
    bi[q] = own[q] ? a.b[row[q]] : 0.0;
    xi[q] = 0.0;
  }
  __syncthreads();
  // row q of A_0 applied to an LDS vector, summed in stored order
  auto arow = [&](int q, const double* v) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kSRow; ++j) {
      const double pr = aval[q][j] * v[acol[q][j]];
      s = j < na[q] ? s + pr : s;
    }
    return s;
  };
  const int gR = 1 << a.lgR;
  const int rrow = t >> a.lgR, rl = t & (gR - 1);
  // coarse product: wave wv takes columns [c0w, c1w), lane ln the row pairs
  // (2 ln + 128 r, +1) for r < rpl, one 16-byte load per pair (a compute
  // unit reads L2 at twice the rate with 16-byte as with 8-byte lane
  // accesses); the wave index, column range and chunk count are
  // wave-uniform, so the column loads have scalar base addresses and the
  // loop has no divergent branches.  The padded order m is a multiple of 16.
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6), ln = t & 63;
  const int Lw = (a.nc + kSWaves - 1) / kSWaves;
  const int c0w = min(wv * Lw, a.nc), c1w = min(c0w + Lw, a.nc);
  const int rpl = (a.nc + 127) >> 7;

  // z = M^-1 r (s_r -> s_z); returns <r, z>, and <z, q> in zq when flexible
  auto vcycle = [&](double& zq) -> double {
#pragma unroll
    for (int q = 0; q < kSR; ++q)                  // pre-smoothing from zero
      if (own[q]) s_xc[row[q]] = swi[q] * s_r[row[q]];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSR; ++q)                  // its residual
      if (own[q]) s_rc[row[q]] = s_r[row[q]] - arow(q, s_xc);
    __syncthreads();
    {                                              // b_1 = R r_c, gR lanes per coarse row
      double s = 0.0;
      if (rrow < a.nc) {
        const int k1 = s_rrp[rrow + 1];
        int k = s_rrp[rrow] + rl;
        for (; k + 3 * gR < k1; k += 4 * gR) {     // four entries per step, summed in order
          const double p0 = s_rv[k] * s_rc[s_rci[k]];
          const double p1 = s_rv[k + gR] * s_rc[s_rci[k + gR]];
          const double p2 = s_rv[k + 2 * gR] * s_rc[s_rci[k + 2 * gR]];
          const double p3 = s_rv[k + 3 * gR] * s_rc[s_rci[k + 3 * gR]];
          s = s + p0;
          s = s + p1;
          s = s + p2;
          s = s + p3;
        }
        for (; k < k1; k += gR) s = s + s_rv[k] * s_rc[s_rci[k]];
      }
      for (int o = 1; o < gR; o <<= 1) s += __shfl_xor(s, o, 64);
      if (rrow < a.nc && rl == 0) s_b1[rrow] = s;
    }
    __syncthreads();
    {                                              // x_1 = A_c^-1 b_1
      phase_fence();
      double acc[kSPairs][2];
#pragma unroll
      for (int r = 0; r < kSPairs; ++r) acc[r][0] = acc[r][1] = 0.0;
      const int jend = opaque(c1w);
      for (int j0 = c0w; j0 < jend; j0 += kSCols) {
        // columns past the block's end and pairs past the padded order load
        // a valid pair (clamped) and are left out of the sums
        double2 v[kSCols][kSPairs];
#pragma unroll
        for (int u = 0; u < kSCols; ++u) {
          const double* col = a.inv + (int64_t)min(j0 + u, jend - 1) * a.m;
#pragma unroll
          for (int r = 0; r < kSPairs; ++r)
            if (r < rpl) v[u][r] = *reinterpret_cast<const double2*>(col + min(2 * ln + 128 * r, a.m - 2));
        }
#pragma unroll
        for (int u = 0; u < kSCols; ++u) {
          const double bj = s_b1[min(j0 + u, jend - 1)];
#pragma unroll
          for (int r = 0; r < kSPairs; ++r) {
            if (r < rpl) {
              const double p0 = v[u][r].x * bj, p1 = v[u][r].y * bj;
              acc[r][0] = j0 + u < jend ? acc[r][0] + p0 : acc[r][0];
              acc[r][1] = j0 + u < jend ? acc[r][1] + p1 : acc[r][1];
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < kSPairs; ++r)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (2 * ln + 128 * r + h < a.nc) s_gp[wv][2 * ln + 128 * r + h] = acc[r][h];
      __syncthreads();
      if (t < a.nc) {                              // the column blocks' sums in wave order
        double s = 0.0;
        for (int q = 0; q < kSWaves; ++q)
          if (q * Lw < a.nc) s += s_gp[q][t];
        s_x1[t] = s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSR; ++q) {                // x_c += P x_1
      if (!own[q]) continue;
      const int k1 = s_prp[row[q] + 1];
      double s = 0.0;
      for (int k = s_prp[row[q]]; k < k1; ++k) s = s + s_pv[k] * s_x1[s_pci[k]];
      s_xc[row[q]] = s_xc[row[q]] + s;
    }
    __syncthreads();
    double rz = 0.0, zqp = 0.0;                    // post-smoothing
#pragma unroll
    for (int q = 0; q < kSR; ++q) {
      if (!own[q]) continue;
      const int i = row[q];
      const double z = s_xc[i] + swi[q] * (s_r[i] - arow(q, s_xc));
      s_z[i] = z;
      rz += s_r[i] * z;
      zqp += z * s_q[i];
    }
    const double rzt = wg_sum(rz, s_red[0]);
    zq = a.flexible ? wg_sum(zqp, s_red[1]) : 0.0;
    return rzt;
  };

  // r = b, x = 0, ||b||^2
  double bbp = 0.0;
#pragma unroll
  for (int q = 0; q < kSR; ++q) {
    if (own[q]) s_r[row[q]] = bi[q];
    s_q[t + q * kST] = 0.0;
    bbp += bi[q] * bi[q];
  }
  const double bb = wg_sum(bbp, s_red[2]);
  const double thresh = (a.tol * a.tol) * bb;
  int iters = 0, restarts = 0, state = 0;
  double rz = 0.0, pq = 0.0, rr = bb, trr = bb;
  if (bb == 0.0) {
    state = 3;
    trr = 0.0;
  } else if (!(bb == bb)) {
    state = -1;
  } else {
    for (;;) {
      // (re)start: z = M^-1 r, p = z
      double zq;
      rz = vcycle(zq);
      if (!(rz > 0.0)) {
        state = -1;
        break;
      }
#pragma unroll
      for (int q = 0; q < kSR; ++q)
        if (own[q]) s_p[row[q]] = s_z[row[q]];
      state = 2;
      while (iters < a.maxiter) {
        __syncthreads();                           // p complete
        double qi[kSR], pqp = 0.0;
#pragma unroll
        for (int q = 0; q < kSR; ++q) {
          qi[q] = own[q] ? arow(q, s_p) : 0.0;
          if (own[q]) {
            s_q[row[q]] = qi[q];
            pqp += s_p[row[q]] * qi[q];
          }
        }
        pq = wg_sum(pqp, s_red[3]);
        if (!(pq > 0.0)) {
          state = -1;
          break;
        }
        const double alpha = rz / pq;
        double rrp = 0.0;
#pragma unroll
        for (int q = 0; q < kSR; ++q) {
          if (!own[q]) continue;
          const int i = row[q];
          xi[q] = xi[q] + alpha * s_p[i];
          const double ri = s_r[i] - alpha * qi[q];
          s_r[i] = ri;
          rrp += ri * ri;
        }
        ++iters;
        rr = wg_sum(rrp, s_red[2]);
        if (rr <= thresh) {
          state = 1;
          break;
        }
        if (!(rr == rr)) {
          state = -1;
          break;
        }
        const double rzn = vcycle(zq);
        if (!(rzn > 0.0)) {
          state = -1;
          break;
        }
        const double beta = a.flexible ? -zq / pq : rzn / rz;
        rz = rzn;
#pragma unroll
        for (int q = 0; q < kSR; ++q)
          if (own[q]) s_p[row[q]] = s_z[row[q]] + beta * s_p[row[q]];
      }
      if (state < 0) break;
      // true residual r = b - A x
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kSR; ++q)
        if (own[q]) s_xc[row[q]] = xi[q];
      __syncthreads();
      double tp = 0.0;
#pragma unroll
      for (int q = 0; q < kSR; ++q) {
        if (!own[q]) continue;
        const double ti = bi[q] - arow(q, s_xc);
        s_r[row[q]] = ti;
        tp += ti * ti;
      }
      trr = wg_sum(tp, s_red[3]);
      if (trr <= thresh) break;
      if (state == 1 && restarts < 5 && iters < a.maxiter) {
        ++restarts;
        __syncthreads();
        continue;
      }
      break;
    }
  }
#pragma unroll
  for (int q = 0; q < kSR; ++q)
    if (own[q]) a.x[row[q]] = state == 3 ? 0.0 : xi[q];
  if (t == 0) {
    Ctl& c = *a.ctl;
    c.bb = bb;
    c.thresh = thresh;
    c.rz = rz;
    c.pq = pq;
    c.rr = rr;
    c.trr = trr;
    c.iters = iters;
    c.maxiter = a.maxiter;
    c.state = state;
    c.done = 1;
    c.flexible = a.flexible;
    c.restarts = restarts;
  }
}

}  // namespace

// Whether H's solves can run as one workgroup: two levels, at most 1024 fine
// rows with at most 8 entries per row of A_0, at most kSPCap entries of P_0,
// a dense coarsest level of at most 256 (padded) rows; FP64 V(1,1) cycle of
// one system, PCG.  Decided once per hierarchy (host copies of the row
// pointers).  R_0 is applied with the most lanes per coarse row (a power of
// two up to 64) that keeps every coarse row's group within the workgroup.
bool small_solve_ok(Hierarchy& H) {
  if (H.small_checked) return H.small_lgR >= 0;
  H.small_checked = true;
  H.small_lgR = -1;
  if (H.lv.size() != 2 || H.S != 1 || H.fp32() || !H.prm.precondition || H.prm.nu_pre != 1 ||
      H.prm.nu_post != 1 || H.prm.solver != AMG_SOLVER_PCG || !H.prm.symmetric)
    return false;
  const Level& L = H.lv[0];
  if (L.n > kSN || L.n < 1 || H.co.m > kSCoarse || H.co.n != L.nagg || L.nagg < 1 || L.pnnz > kSPCap) return false;
  std::vector<int> h(L.n + 1);
  AMG_HIP(hipMemcpy(h.data(), L.rp.p, sizeof(int) * (L.n + 1), hipMemcpyDeviceToHost));
  for (int r = 0; r < L.n; ++r)
    if (h[r + 1] - h[r] > kSRow) return false;
  int lg = 0;
  while (lg < 6 && (int64_t)L.nagg * (2 << lg) <= kST) ++lg;
  H.small_lgR = lg;
  return true;
}

amg_status pcg_solve_small(Hierarchy& H, const SolveOpts& o, const SolveWork& w, const double* d_b, double* d_x,
                           double tol, amg_info* info, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  const Level& L = H.lv[0];
  SmallArgs a{};
  a.n = L.n;
  a.nc = H.co.n;
  a.m = H.co.m;
  a.lgR = H.small_lgR;
  a.maxiter = o.maxiter;
  a.flexible = o.flexible < 0 ? 0 : o.flexible;
  a.tol = tol;
  a.arp = L.rp.p;
  a.aci = L.ci.p;
  a.av = L.v.p;
  a.sw = L.sw.p;
  a.prp = L.prp.p;
  a.pci = L.pci.p;
  a.pv = L.pv.p;
  a.rrp = L.rrp.p;
  a.rci = L.rci.p;
  a.rv = L.rv.p;
  a.inv = H.co.inv.p;
  a.b = d_b;
  a.x = d_x;
  a.ctl = w.ctl;
  hipLaunchKernelGGL(k_pcg_small, dim3(1), dim3(kST), 0, s, a);
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipMemcpyAsync(w.h_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  const Ctl& c = *w.h_ctl;
  amg_status st;
  if (c.state == 3 || c.trr <= c.thresh) st = AMG_OK;
  else if (c.state < 0) st = AMG_ERR_BREAKDOWN;
  else st = AMG_NOT_CONVERGED;
  if (info) {
    info->iters = c.iters;
    info->status = st;
    info->restarts = c.restarts;
    info->rel_resid = c.state == 3 ? 0.0 : (c.bb > 0 ? std::sqrt(c.trr / c.bb) : 0.0);
    if (st == AMG_ERR_BREAKDOWN) info->rel_resid = NAN;
    info->cache_event = H.cache_event;
    info->setup_ms = H.setup_ms;
    info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

}  // namespace amg
