// C ABI entry points (include/amg355.h) and the setup cache.
//
// Cache (Section 2.1, "C++/CUDA backend"): hierarchies are kept in an LRU
// list keyed by a 64-bit hash of the full sparsity pattern together with n,
// nnz and the setup parameters; a hash hit is confirmed by comparing the
// whole pattern on the device.  A confirmed hit with different values
// refreshes the hierarchy in place (aggregates and patterns kept).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>

#include "amg_internal.hpp"

namespace amg {

void Graphs::reset() {
  for (auto& e : exec)
    if (e) {
      (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
  if (bexec) {
    (void)hipGraphExecDestroy(bexec);
    bexec = nullptr;
  }
  key_x = nullptr;
  key_bx = nullptr;
  key_flex = -1;
  key_w = 0;
}

Graphs::~Graphs() {
  reset();
  if (ev_in) (void)hipEventDestroy(ev_in);
  if (ev_out) (void)hipEventDestroy(ev_out);
  if (gs) (void)hipStreamDestroy(gs);
}

Hierarchy::~Hierarchy() {
  if (h_ctl) (void)hipHostFree(h_ctl);
  if (h_flags) (void)hipHostFree(h_flags);
  for (hipEvent_t e : inst.ev) (void)hipEventDestroy(e);
  if (bt.h_ctl) (void)hipHostFree(bt.h_ctl);
  if (bt.h_head) (void)hipHostFree(bt.h_head);
  if (bt.h_mask) (void)hipHostFree(bt.h_mask);
}

namespace {

std::mutex g_mu;
std::list<Hierarchy*> g_lru;  // front = most recently used
int g_capacity = 8;

void release(Hierarchy* H) {
  if (--H->refs <= 0) delete H;
}

void uncache(Hierarchy* H) {
  for (auto it = g_lru.begin(); it != g_lru.end(); ++it)
    if (*it == H) {
      g_lru.erase(it);
      H->in_cache = false;
      release(H);
      return;
    }
}

void evict_to(int cap) {
  while ((int)g_lru.size() > cap) {
    Hierarchy* H = g_lru.back();
    g_lru.pop_back();
    H->in_cache = false;
    release(H);
  }
}

uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h;
}

uint64_t params_hash(const amg_params& p) {
  uint64_t h = 0x12345678abcdefull;
  uint64_t t;
  h = mix(h, (uint64_t)p.vcycle_prec);
  h = mix(h, (uint64_t)p.transfer_bf16);
  std::memcpy(&t, &p.theta, 8);
  h = mix(h, t);
  h = mix(h, (uint64_t)p.max_coarse);
  h = mix(h, (uint64_t)p.max_levels);
  h = mix(h, (uint64_t)p.smoother);
  std::memcpy(&t, &p.omega, 8);
  h = mix(h, t);
  h = mix(h, (uint64_t)p.nu_pre);
  h = mix(h, (uint64_t)p.nu_post);
  h = mix(h, (uint64_t)p.autotune);
  h = mix(h, (uint64_t)p.precondition);
  h = mix(h, (uint64_t)p.symmetric);
  h = mix(h, (uint64_t)p.solver);
  return h;
}

bool same_setup_params(const amg_params& a, const amg_params& b) {
  return a.vcycle_prec == b.vcycle_prec && a.transfer_bf16 == b.transfer_bf16 && a.theta == b.theta &&
         a.max_coarse == b.max_coarse && a.max_levels == b.max_levels && a.smoother == b.smoother &&
         a.omega == b.omega && a.nu_pre == b.nu_pre && a.nu_post == b.nu_post && a.autotune == b.autotune &&
         a.precondition == b.precondition && a.symmetric == b.symmetric && a.solver == b.solver;
}

amg_status check_params(const amg_params& p) {
  if (p.vcycle_prec != AMG_PREC_FP64 && p.vcycle_prec != AMG_PREC_FP32) return AMG_ERR_INVALID_ARG;
  if (p.smoother != AMG_SMOOTHER_JACOBI && p.smoother != AMG_SMOOTHER_L1) return AMG_ERR_INVALID_ARG;
  if (p.max_levels < 1 || p.max_levels > AMG_MAX_LEVELS || p.max_coarse < 1) return AMG_ERR_INVALID_ARG;
  if (p.nu_pre < 1 || p.nu_post < 1 || p.nu_pre > 8 || p.nu_post > 8) return AMG_ERR_INVALID_ARG;
  if (!(p.omega > 0.0) || !(p.theta >= 0.0) || p.maxiter < 0) return AMG_ERR_INVALID_ARG;
  if (p.symmetric != 0 && p.symmetric != 1) return AMG_ERR_INVALID_ARG;
  if (p.precondition != 0 && p.precondition != 1) return AMG_ERR_INVALID_ARG;
  if (p.solver != AMG_SOLVER_PCG && p.solver != AMG_SOLVER_BICGSTAB) return AMG_ERR_INVALID_ARG;
  if (p.fused_small != 0 && p.fused_small != 1) return AMG_ERR_INVALID_ARG;
  // CG needs A = A^T; a nonsymmetric A is solved by BiCGSTAB
  if (!p.symmetric && p.solver != AMG_SOLVER_BICGSTAB) return AMG_ERR_INVALID_ARG;
  return AMG_OK;
}

// Scratch flags for calls made before a hierarchy exists.
struct GlobalFlags {
  int* d = nullptr;
  int* h = nullptr;
  int dev = -1;
} g_flags;

void ensure_global_flags() {
  int dev = 0;
  AMG_HIP(hipGetDevice(&dev));
  if (g_flags.d && g_flags.dev == dev) return;
  AMG_HIP(hipMalloc(&g_flags.d, 64));
  AMG_HIP(hipHostMalloc((void**)&g_flags.h, 64, hipHostMallocDefault));
  g_flags.dev = dev;
}

template <class F>
amg_status guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return e.status;
  } catch (const std::bad_alloc&) {
    return AMG_ERR_OOM;
  } catch (...) {
    return AMG_ERR_HIP;
  }
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Column c of a row-major [n][W] block to a contiguous vector and back.
__global__ void k_col_get(int n, int W, int c, const double* __restrict__ B, double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = B[(int64_t)i * W + c];
}

__global__ void k_col_put(int n, int W, int c, const double* __restrict__ v, double* __restrict__ B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) B[(int64_t)i * W + c] = v[i];
}

// BiCGSTAB for W right-hand sides of one matrix ([n][W] blocks): the columns
// are solved one after another, each by the single-column solve (the
// paper's batch support maps the solver over the right-hand sides
// sequentially, Section 2.2); per-column outcomes go to `rec` for
// amg_solve_columns, info holds the maximum iteration count and residual and
// the worst status.
amg_status bicgstab_columns(Hierarchy& H, const SolveOpts& o, const double* d_b, double* d_x, double tol, int W,
                            amg_info* info, hipStream_t s, Batch& rec) {
  auto t0 = std::chrono::steady_clock::now();
  const int n = H.n;
  DBuf<double> bc, xc;
  bc.alloc(n);
  xc.alloc(n);
  const int g = (n + 255) / 256;
  rec.col_iters.assign(W, 0);
  rec.col_status.assign(W, AMG_OK);
  rec.col_relres.assign(W, 0.0);
  int maxit = 0, restarts = 0;
  double maxrr = 0.0;
  amg_status st = AMG_OK;
  for (int c = 0; c < W; ++c) {
    hipLaunchKernelGGL(k_col_get, dim3(g), dim3(256), 0, s, n, W, c, d_b, bc.p);
    AMG_HIP(hipGetLastError());
    amg_info ci{};
    const amg_status cs = bicgstab_solve(H, o, bc.p, xc.p, tol, &ci, s);
    hipLaunchKernelGGL(k_col_put, dim3(g), dim3(256), 0, s, n, W, c, xc.p, d_x);
    AMG_HIP(hipGetLastError());
    rec.col_iters[c] = ci.iters;
    rec.col_status[c] = cs;
    rec.col_relres[c] = ci.rel_resid;
    maxit = std::max(maxit, ci.iters);
    restarts += ci.restarts;
    if (cs != AMG_ERR_BREAKDOWN) maxrr = std::max(maxrr, ci.rel_resid);
    if (cs == AMG_ERR_BREAKDOWN) st = AMG_ERR_BREAKDOWN;
    else if (cs == AMG_NOT_CONVERGED && st == AMG_OK) st = AMG_NOT_CONVERGED;
  }
  AMG_HIP(hipStreamSynchronize(s));
  if (info) {
    info->iters = maxit;
    info->status = st;
    info->restarts = restarts;
    info->rel_resid = st == AMG_ERR_BREAKDOWN ? NAN : maxrr;
    info->cache_event = H.cache_event;
    info->setup_ms = H.setup_ms;
    info->solve_ms = ms_since(t0);
  }
  return st;
}

// Hierarchy of A^T for the adjoint of a nonsymmetric A (Eq. (1)): formed on
// first use with A's parameters, kept with A's hierarchy (not in the cache)
// and refreshed from A's values when they have changed since.
Hierarchy& adjoint_hierarchy(Hierarchy& H, hipStream_t s) {
  if (!H.adj) {
    auto t0 = std::chrono::steady_clock::now();
    transpose_pattern(H, s);
    transpose_values(H, s);
    std::unique_ptr<Hierarchy> A(new Hierarchy);
    A->prm = H.prm;
    A->S = 1;
    A->n = H.n;
    A->nnz = H.nnz;
    A->lv.reserve(AMG_MAX_LEVELS + 1);
    A->flags.alloc(16);
    AMG_HIP(hipHostMalloc((void**)&A->h_flags, 64, hipHostMallocDefault));
    build_hierarchy(*A, H.trp.p, H.tci.p, H.tval.p, s);
    A->cache_event = AMG_CACHE_COLD;
    A->setup_ms = ms_since(t0);
    H.adj = std::move(A);
    H.adj_version = H.val_version;
  } else if (H.adj_version != H.val_version) {
    auto t0 = std::chrono::steady_clock::now();
    transpose_values(H, s);
    H.adj->gr.reset();
    refresh_hierarchy(*H.adj, H.tval.p, s);
    H.adj->cache_event = AMG_CACHE_REFRESH;
    H.adj->setup_ms = ms_since(t0);
    H.adj_version = H.val_version;
  }
  return *H.adj;
}

}  // namespace
}  // namespace amg

using namespace amg;

extern "C" {

void amg_params_default(amg_params* p) {
  if (!p) return;
  p->vcycle_prec = AMG_PREC_FP64;
  p->transfer_bf16 = 1;
  p->theta = 0.0;
  p->max_coarse = 256;
  p->max_levels = 20;
  p->smoother = AMG_SMOOTHER_JACOBI;
  p->omega = 2.0 / 3.0;
  p->nu_pre = 1;
  p->nu_post = 1;
  p->maxiter = 1000;
  p->flexible = -1;
  p->symmetric = 1;
  p->check_every = 0;
  p->use_graphs = 1;
  p->autotune = 0;
  p->precondition = 1;
  p->solver = AMG_SOLVER_PCG;
  p->fused_small = 1;
}

amg_status amg_setup(const amg_params* params, int32_t n, int64_t nnz, const int32_t* d_row_ptr,
                     const int32_t* d_col, const double* d_val, int32_t n_systems, hipStream_t stream,
                     amg_handle* out) {
  return guarded([&]() -> amg_status {
    if (!out || !d_row_ptr || !d_col || !d_val || n <= 0 || nnz < n || nnz >= (int64_t)INT32_MAX)
      return AMG_ERR_INVALID_ARG;
    if (n_systems < 1 || n_systems > kMaxWidth) return AMG_ERR_INVALID_ARG;
    amg_params prm;
    if (params) prm = *params;
    else amg_params_default(&prm);
    amg_status ps = check_params(prm);
    if (ps != AMG_OK) return ps;
    // several systems share one pattern-only aggregation (theta = 0) and the
    // one-sweep cycle of the batched kernels
    if (n_systems > 1 && (prm.theta != 0.0 || prm.nu_pre != 1 || prm.nu_post != 1)) return AMG_ERR_INVALID_ARG;
    if (n_systems > 1 && prm.solver != AMG_SOLVER_PCG) return AMG_ERR_INVALID_ARG;
    auto t0 = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lock(g_mu);
    ensure_global_flags();
    validate_csr(n, nnz, d_row_ptr, d_col, g_flags.d, g_flags.h, stream);
    const uint64_t key = mix(mix(mix(mix(pattern_hash(n, nnz, d_row_ptr, d_col, g_flags.d, g_flags.h, stream),
                                         (uint64_t)n), (uint64_t)nnz), params_hash(prm)), (uint64_t)n_systems);
    for (auto it = g_lru.begin(); it != g_lru.end(); ++it) {
      Hierarchy* H = *it;
      if (H->key != key || H->n != n || H->nnz != nnz || H->S != n_systems || !same_setup_params(H->prm, prm))
        continue;
      if (!pattern_equal(*H, d_row_ptr, d_col, g_flags.d, g_flags.h, stream)) continue;
      g_lru.splice(g_lru.begin(), g_lru, it);
      if (values_equal(*H, d_val, g_flags.d, g_flags.h, stream)) {
        H->cache_event = AMG_CACHE_HIT;
        H->setup_ms = ms_since(t0);
      } else if (H->refs > 1) {
        // Other callers' handles still hold this hierarchy for its values:
        // it stays as it is for them, and a hierarchy of the new values is
        // built below and takes its place in the cache (copy on write).
        uncache(H);
        break;
      } else {
        // only the cache holds it: the values are refreshed in place
        H->gr.reset();
        try {
          refresh_hierarchy(*H, d_val, stream);
        } catch (...) {
          // part-way refreshed: never handed out again
          (void)hipStreamSynchronize(stream);
          uncache(H);
          throw;
        }
        ++H->val_version;
        H->cache_event = AMG_CACHE_REFRESH;
        H->setup_ms = ms_since(t0);
      }
      ++H->refs;
      *out = new amg_handle_s{H, SolveOpts{prm.maxiter, prm.flexible, prm.check_every, prm.use_graphs, prm.fused_small}};
      return AMG_OK;
    }
    Hierarchy* H = new Hierarchy;
    H->prm = prm;
    H->S = n_systems;
    H->n = n;
    H->nnz = nnz;
    H->lv.reserve(AMG_MAX_LEVELS + 1);
    try {
      H->flags.alloc(16);
      AMG_HIP(hipHostMalloc((void**)&H->h_flags, 64, hipHostMallocDefault));
      build_hierarchy(*H, d_row_ptr, d_col, d_val, stream);
    } catch (...) {
      (void)hipStreamSynchronize(stream);
      delete H;
      throw;
    }
    H->key = key;
    H->cache_event = AMG_CACHE_COLD;
    H->setup_ms = ms_since(t0);
    H->refs = 1;  // the caller
    if (g_capacity > 0) {
      H->refs += 1;  // the cache
      H->in_cache = true;
      g_lru.push_front(H);
      evict_to(g_capacity);
    }
    *out = new amg_handle_s{H, SolveOpts{prm.maxiter, prm.flexible, prm.check_every, prm.use_graphs, prm.fused_small}};
    return AMG_OK;
  });
}

amg_status amg_update_values(amg_handle h, const double* d_val, hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (!h || !d_val) return AMG_ERR_INVALID_ARG;
    auto t0 = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lock(g_mu);
    Hierarchy* H = h->H;
    if (H->refs - (H->in_cache ? 1 : 0) > 1) {
      // Another caller's handle shares this hierarchy: this handle gets a
      // hierarchy of its own for the new values (copy on write, not cached);
      // the shared one keeps its values.
      std::unique_ptr<Hierarchy> N(new Hierarchy);
      N->prm = H->prm;
      N->S = H->S;
      N->n = H->n;
      N->nnz = H->nnz;
      N->lv.reserve(AMG_MAX_LEVELS + 1);
      N->flags.alloc(16);
      AMG_HIP(hipHostMalloc((void**)&N->h_flags, 64, hipHostMallocDefault));
      try {
        build_hierarchy(*N, H->lv[0].rp.p, H->lv[0].ci.p, d_val, stream);
      } catch (...) {
        (void)hipStreamSynchronize(stream);
        throw;
      }
      N->cache_event = AMG_CACHE_COLD;
      N->setup_ms = ms_since(t0);
      N->refs = 1;
      release(H);
      h->H = N.release();
      return AMG_OK;
    }
    H->gr.reset();
    try {
      refresh_hierarchy(*H, d_val, stream);
    } catch (const Error& e) {
      // part-way refreshed: out of the cache, and refused by solves until a
      // later refresh succeeds
      (void)hipStreamSynchronize(stream);
      H->broken = e.status;
      if (H->in_cache) uncache(H);
      throw;
    } catch (...) {
      (void)hipStreamSynchronize(stream);
      H->broken = AMG_ERR_HIP;
      if (H->in_cache) uncache(H);
      throw;
    }
    H->broken = AMG_OK;
    ++H->val_version;
    H->cache_event = AMG_CACHE_REFRESH;
    H->setup_ms = ms_since(t0);
    return AMG_OK;
  });
}

amg_status amg_solve(amg_handle h, const double* d_b, double* d_x, double tol, int32_t nrhs, amg_info* info,
                     hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (!h || !d_b || !d_x || nrhs < 1 || nrhs > kMaxWidth || !(tol >= 0.0)) return AMG_ERR_INVALID_ARG;
    Hierarchy& H = *h->H;
    if (H.broken != AMG_OK) return H.broken;
    if (H.S > 1 && nrhs != H.S) return AMG_ERR_INVALID_ARG;
    if (H.prm.solver == AMG_SOLVER_BICGSTAB) {
      if (nrhs == 1) return bicgstab_solve(H, h->opts, d_b, d_x, tol, info, stream);
      return bicgstab_columns(H, h->opts, d_b, d_x, tol, nrhs, info, stream, H.bt);
    }
    if (nrhs > 1 || H.S > 1) return pcg_solve_wide(H, h->opts, d_b, d_x, tol, nrhs, info, stream);
    return pcg_solve(H, h->opts, solve_work(H), d_b, d_x, tol, info, stream);
  });
}

amg_status amg_solve_adjoint(amg_handle h, const double* d_g, double* d_lambda, double tol, int32_t nrhs,
                             amg_info* info, hipStream_t stream) {
  // Symmetric A: A^T lambda = g is solved with A's own hierarchy and the
  // forward solver settings (Eq. (1)).
  if (!h || h->H->prm.symmetric) return amg_solve(h, d_g, d_lambda, tol, nrhs, info, stream);
  return guarded([&]() -> amg_status {
    if (!d_g || !d_lambda || nrhs < 1 || nrhs > kMaxWidth || !(tol >= 0.0)) return AMG_ERR_INVALID_ARG;
    Hierarchy& H = *h->H;
    if (H.broken != AMG_OK) return H.broken;
    Hierarchy* T;
    {
      // the lock covers building or refreshing A^T's hierarchy (shared state
      // of the cached hierarchy); the solve itself runs outside it, like
      // amg_solve
      std::lock_guard<std::mutex> lock(g_mu);
      T = &adjoint_hierarchy(H, stream);
    }
    amg_status st = nrhs == 1 ? bicgstab_solve(*T, h->opts, d_g, d_lambda, tol, info, stream)
                              : bicgstab_columns(*T, h->opts, d_g, d_lambda, tol, nrhs, info, stream, H.bt);
    if (info) {
      info->cache_event = H.cache_event;
      info->setup_ms = H.setup_ms;
    }
    return st;
  });
}

amg_status amg_pattern_grad(amg_handle h, const double* d_lambda, const double* d_x, double* d_grad_val,
                            hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (!h || !d_lambda || !d_x || !d_grad_val) return AMG_ERR_INVALID_ARG;
    if (h->H->S > 1) pattern_grad_wide(*h->H, d_lambda, d_x, d_grad_val, h->H->S, stream);
    else pattern_grad(*h->H, d_lambda, d_x, d_grad_val, stream);
    return AMG_OK;
  });
}

amg_status amg_pattern_grad_batched(amg_handle h, const double* d_lambda, const double* d_x, int32_t ncols,
                                    double* d_grad_val, hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (!h || !d_lambda || !d_x || !d_grad_val || ncols < 1 || ncols > kMaxWidth) return AMG_ERR_INVALID_ARG;
    Hierarchy& H = *h->H;
    if (H.S > 1 && ncols != H.S) return AMG_ERR_INVALID_ARG;
    if (ncols == 1 && H.S == 1) pattern_grad(H, d_lambda, d_x, d_grad_val, stream);
    else pattern_grad_wide(H, d_lambda, d_x, d_grad_val, ncols, stream);
    return AMG_OK;
  });
}

amg_status amg_solve_columns(amg_handle h, int32_t ncols, int* iters, double* rel_resid, int* status) {
  if (!h) return AMG_ERR_INVALID_ARG;
  const Batch& B = h->H->bt;
  if (ncols != (int)B.col_iters.size() || ncols < 1) return AMG_ERR_INVALID_ARG;
  for (int c = 0; c < ncols; ++c) {
    if (iters) iters[c] = B.col_iters[c];
    if (rel_resid) rel_resid[c] = B.col_relres[c];
    if (status) status[c] = B.col_status[c];
  }
  return AMG_OK;
}

amg_status amg_apply_vcycle(amg_handle h, const double* d_r, double* d_z, hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (!h || !d_r || !d_z) return AMG_ERR_INVALID_ARG;
    if (h->H->broken != AMG_OK) return h->H->broken;
    apply_vcycle(*h->H, d_r, d_z, stream);
    return AMG_OK;
  });
}

amg_status amg_color_columns(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                             int32_t* d_color, int32_t* ncolors, hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (!d_row_ptr || !d_col || !d_color || !ncolors || n <= 0 || nnz < n || nnz >= (int64_t)INT32_MAX)
      return AMG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    ensure_global_flags();
    validate_csr(n, nnz, d_row_ptr, d_col, g_flags.d, g_flags.h, stream);
    *ncolors = color_columns(n, nnz, d_row_ptr, d_col, d_color, g_flags.d, g_flags.h, stream);
    return AMG_OK;
  });
}

amg_status amg_probe_vectors(int32_t n, const int32_t* d_color, int32_t ncolors, double* d_V, hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (!d_color || !d_V || n <= 0 || ncolors <= 0) return AMG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    ensure_global_flags();
    probe_vectors(n, d_color, ncolors, d_V, g_flags.d, g_flags.h, stream);
    return AMG_OK;
  });
}

amg_status amg_probe_assemble(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                              const int32_t* d_color, int32_t ncolors, const double* d_Y, double* d_val,
                              hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (!d_row_ptr || !d_col || !d_color || !d_Y || !d_val || n <= 0 || nnz < n || nnz >= (int64_t)INT32_MAX ||
        ncolors <= 0)
      return AMG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    ensure_global_flags();
    validate_csr(n, nnz, d_row_ptr, d_col, g_flags.d, g_flags.h, stream);
    probe_assemble(n, d_row_ptr, d_col, d_color, ncolors, d_Y, d_val, g_flags.d, g_flags.h, stream);
    return AMG_OK;
  });
}

amg_status amg_probe_scatter(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                             const int32_t* d_color, int32_t ncolors, const double* d_dval, double* d_dY,
                             hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (!d_row_ptr || !d_col || !d_color || !d_dval || !d_dY || n <= 0 || nnz < n || nnz >= (int64_t)INT32_MAX ||
        ncolors <= 0)
      return AMG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    ensure_global_flags();
    validate_csr(n, nnz, d_row_ptr, d_col, g_flags.d, g_flags.h, stream);
    probe_scatter(n, d_row_ptr, d_col, d_color, ncolors, d_dval, d_dY, g_flags.d, g_flags.h, stream);
    return AMG_OK;
  });
}

amg_status amg_hierarchy_stats(amg_handle h, amg_hier_stats* out) {
  if (!h || !out) return AMG_ERR_INVALID_ARG;
  const Hierarchy& H = *h->H;
  std::memset(out, 0, sizeof(*out));
  out->num_levels = (int)H.lv.size();
  double tot = 0.0;
  for (size_t l = 0; l < H.lv.size() && l < AMG_MAX_LEVELS; ++l) {
    const Level& L = H.lv[l];
    out->n[l] = L.n;
    out->nnz[l] = L.nnz;
    out->nnz_p[l] = (l + 1 < H.lv.size()) ? L.pnnz : 0;
    out->nnz_g[l] = (l + 1 < H.lv.size()) ? L.gnnz : 0;
    out->rho[l] = L.rho;
    out->omega_p[l] = L.omegaP;
    out->mis_rounds[l] = L.mis_rounds;
    out->group_a[l] = L.shA.g;
    out->group_p[l] = L.shP.g;
    out->group_r[l] = L.shR.g;
    out->form_a[l] = L.shA.stream;
    out->sliced_len[l] = L.sell ? L.sell_len : 0;
    tot += (double)L.nnz;
  }
  out->operator_complexity = tot / (double)H.lv[0].nnz;
  out->single_workgroup = H.small_checked && H.small_lgR >= 0 ? 1 : 0;
  return AMG_OK;
}

static amg_status field_ptr(const Hierarchy& H, int level, int field, const void** p, int64_t* count, int* eb) {
  if (level < 0 || level >= (int)H.lv.size()) return AMG_ERR_INVALID_ARG;
  const Level& L = H.lv[level];
  const bool coarsest = level + 1 == (int)H.lv.size();
  const int64_t S = H.S;  // value fields hold S interleaved systems
  *p = nullptr;
  *count = 0;
  *eb = 0;
  switch (field) {
    case AMG_FIELD_AGG: if (coarsest) return AMG_ERR_INVALID_ARG; *p = L.agg.p; *count = L.n; *eb = 4; break;
    case AMG_FIELD_A_ROWPTR: *p = L.rp.p; *count = L.n + 1; *eb = 4; break;
    case AMG_FIELD_A_COL: *p = L.ci.p; *count = L.nnz; *eb = 4; break;
    case AMG_FIELD_A_VAL: *p = L.v.p; *count = L.nnz * S; *eb = 8; break;
    case AMG_FIELD_A_VAL32: if (!H.fp32()) return AMG_ERR_INVALID_ARG; *p = L.v32.p; *count = L.nnz * S; *eb = 4; break;
    case AMG_FIELD_DINV: *p = L.dinv.p; *count = L.n * S; *eb = 8; break;
    case AMG_FIELD_DINV32: if (!H.fp32()) return AMG_ERR_INVALID_ARG; *p = L.sw32.p; *count = L.n * S; *eb = 4; break;
    case AMG_FIELD_P_ROWPTR: if (coarsest) return AMG_ERR_INVALID_ARG; *p = L.prp.p; *count = L.n + 1; *eb = 4; break;
    case AMG_FIELD_P_COL: if (coarsest) return AMG_ERR_INVALID_ARG; *p = L.pci.p; *count = L.pnnz; *eb = 4; break;
    case AMG_FIELD_P_VAL: if (coarsest) return AMG_ERR_INVALID_ARG; *p = L.pv.p; *count = L.pnnz * S; *eb = 8; break;
    case AMG_FIELD_P_BF16: if (coarsest || !H.bf16()) return AMG_ERR_INVALID_ARG; *p = L.pbf.p; *count = L.pnnz * S; *eb = 2; break;
    case AMG_FIELD_R_ROWPTR: if (coarsest) return AMG_ERR_INVALID_ARG; *p = L.rrp.p; *count = L.nagg + 1; *eb = 4; break;
    case AMG_FIELD_R_COL: if (coarsest) return AMG_ERR_INVALID_ARG; *p = L.rci.p; *count = L.pnnz; *eb = 4; break;
    case AMG_FIELD_R_VAL: if (coarsest) return AMG_ERR_INVALID_ARG; *p = L.rv.p; *count = L.pnnz * S; *eb = 8; break;
    case AMG_FIELD_R_BF16: if (coarsest || !H.bf16()) return AMG_ERR_INVALID_ARG; *p = L.rbf.p; *count = L.pnnz * S; *eb = 2; break;
    case AMG_FIELD_G_ROWPTR: if (coarsest) return AMG_ERR_INVALID_ARG; *p = L.grp.p; *count = L.n + 1; *eb = 4; break;
    case AMG_FIELD_G_COL: if (coarsest) return AMG_ERR_INVALID_ARG; *p = L.gci.p; *count = L.gnnz; *eb = 4; break;
    case AMG_FIELD_COARSE_FACTOR: if (!coarsest) return AMG_ERR_INVALID_ARG; *p = H.co.L.p; *count = (int64_t)H.co.m * H.co.m * S; *eb = 8; break;
    case AMG_FIELD_COARSE_INV: if (!coarsest) return AMG_ERR_INVALID_ARG; *p = H.co.inv.p; *count = (int64_t)H.co.m * H.co.m * S; *eb = 8; break;
    case AMG_FIELD_SW: *p = L.sw.p; *count = L.n * S; *eb = 8; break;
    case AMG_FIELD_COARSE_INV32: if (!coarsest || !H.fp32()) return AMG_ERR_INVALID_ARG; *p = H.co.inv32.p; *count = (int64_t)H.co.m * H.co.m * S; *eb = 4; break;
    case AMG_FIELD_COARSE_PIVOTS: if (!coarsest || H.prm.symmetric) return AMG_ERR_INVALID_ARG; *p = H.co.piv.p; *count = (int64_t)H.co.m * S; *eb = 4; break;
    default: return AMG_ERR_INVALID_ARG;
  }
  return AMG_OK;
}

amg_status amg_field_info(amg_handle h, int level, int field, int64_t* count, int* elem_bytes) {
  if (!h || !count || !elem_bytes) return AMG_ERR_INVALID_ARG;
  const void* p;
  return field_ptr(*h->H, level, field, &p, count, elem_bytes);
}

amg_status amg_export_field(amg_handle h, int level, int field, void* d_dst, size_t dst_bytes, hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (!h || !d_dst) return AMG_ERR_INVALID_ARG;
    const void* p;
    int64_t count;
    int eb;
    amg_status st = field_ptr(*h->H, level, field, &p, &count, &eb);
    if (st != AMG_OK) return st;
    size_t bytes = (size_t)count * (size_t)eb;
    if (dst_bytes < bytes) return AMG_ERR_INVALID_ARG;
    if (bytes) AMG_HIP(hipMemcpyAsync(d_dst, p, bytes, hipMemcpyDeviceToDevice, stream));
    AMG_HIP(hipStreamSynchronize(stream));
    return AMG_OK;
  });
}

amg_status amg_destroy(amg_handle h) {
  if (!h) return AMG_ERR_INVALID_ARG;
  return guarded([&]() -> amg_status {
    std::lock_guard<std::mutex> lock(g_mu);
    (void)hipDeviceSynchronize();
    release(h->H);
    delete h;
    return AMG_OK;
  });
}

amg_status amg_finalize(void) {
  return guarded([&]() -> amg_status {
    std::lock_guard<std::mutex> lock(g_mu);
    (void)hipDeviceSynchronize();
    evict_to(0);
    return AMG_OK;
  });
}

int amg_cache_size(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  return (int)g_lru.size();
}

amg_status amg_set_cache_capacity(int capacity) {
  if (capacity < 0) return AMG_ERR_INVALID_ARG;
  return guarded([&]() -> amg_status {
    std::lock_guard<std::mutex> lock(g_mu);
    g_capacity = capacity;
    evict_to(capacity);
    return AMG_OK;
  });
}

amg_status amg_instrument(amg_handle h, int kernel, int level) {
  return guarded([&]() -> amg_status {
    if (!h || kernel < -1 || kernel >= KID_COUNT) return AMG_ERR_INVALID_ARG;
    set_instrument(*h->H, kernel, level);
    return AMG_OK;
  });
}

amg_status amg_instrument_read(amg_handle h, int* launches, double* total_ms, double* min_ms, double* max_ms) {
  return guarded([&]() -> amg_status {
    if (!h || !launches || !total_ms || !min_ms || !max_ms) return AMG_ERR_INVALID_ARG;
    read_instrument(*h->H, launches, total_ms, min_ms, max_ms);
    return AMG_OK;
  });
}

amg_status amg_kernel_bytes(amg_handle h, int kernel, int level, int flexible, double* bytes) {
  if (!h || !bytes) return AMG_ERR_INVALID_ARG;
  const Hierarchy& H = *h->H;
  if (kernel == -1) {
    *bytes = iteration_bytes(H, flexible);
    return AMG_OK;
  }
  if (kernel < 0 || kernel >= KID_COUNT || level < 0 || level >= (int)H.lv.size()) return AMG_ERR_INVALID_ARG;
  *bytes = kernel_bytes(H, kernel, level, flexible);
  return AMG_OK;
}

amg_status amg_kernel_bytes_batched(amg_handle h, int kernel, int level, int flexible, int32_t width,
                                    double* bytes) {
  if (!h || !bytes || width < 1 || width > kMaxWidth) return AMG_ERR_INVALID_ARG;
  const Hierarchy& H = *h->H;
  if (H.S > 1 && width != H.S) return AMG_ERR_INVALID_ARG;
  if (kernel == -1) {
    *bytes = wide_iteration_bytes(H, flexible, width);
    return AMG_OK;
  }
  if (kernel < 0 || kernel >= KID_COUNT || level < 0 || level >= (int)H.lv.size()) return AMG_ERR_INVALID_ARG;
  *bytes = wide_kernel_bytes(H, kernel, level, flexible, width);
  return AMG_OK;
}

amg_status amg_convert_bf16(const float* d_in, uint16_t* d_out, int64_t n, hipStream_t stream) {
  return guarded([&]() -> amg_status {
    if (n < 0 || (n > 0 && (!d_in || !d_out))) return AMG_ERR_INVALID_ARG;
    if (n > 0) convert_bf16(d_in, d_out, n, stream);
    return AMG_OK;
  });
}

const char* amg_status_string(amg_status s) {
  switch (s) {
    case AMG_OK: return "AMG_OK";
    case AMG_NOT_CONVERGED: return "AMG_NOT_CONVERGED";
    case AMG_ERR_INVALID_ARG: return "AMG_ERR_INVALID_ARG";
    case AMG_ERR_ZERO_DIAG: return "AMG_ERR_ZERO_DIAG";
    case AMG_ERR_PATTERN_MISMATCH: return "AMG_ERR_PATTERN_MISMATCH";
    case AMG_ERR_BREAKDOWN: return "AMG_ERR_BREAKDOWN";
    case AMG_ERR_OOM: return "AMG_ERR_OOM";
    case AMG_ERR_HIP: return "AMG_ERR_HIP";
    case AMG_ERR_COARSE_TOO_LARGE: return "AMG_ERR_COARSE_TOO_LARGE";
    case AMG_ERR_SCRATCH_LIMIT: return "AMG_ERR_SCRATCH_LIMIT";
  }
  return "AMG_UNKNOWN_STATUS";
}

}  // extern "C"
