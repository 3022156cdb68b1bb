// Allocation-free PCG solve (amg_solve_noalloc): the single-column PCG of
// amg_solve, with its Krylov workspace taken from one static device array
// per GPU instead of the handle's buffers, for callers that cannot allocate
// device memory.
//
// The array `scratch` below is a device symbol: in host code its name is a
// host-side stand-in, never a device address.  Its device address is looked
// up once per device with hipGetSymbolAddress (the device current at the
// first call on it) and only that address reaches kernels.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "amg_internal.hpp"

namespace amg {
namespace {

// Layout: [control block, 256 B][partial sums][r][z][p][p'][q]
constexpr size_t kCtlBytes = 256;
constexpr size_t kScratchBytes = AMG_NOALLOC_SCRATCH_BYTES;
static_assert(sizeof(Ctl) <= kCtlBytes, "control block exceeds its scratch slot");
static_assert(kScratchBytes == kCtlBytes + 8 * (size_t)AMG_NOALLOC_MAX_PARTIALS + 5 * 8 * (size_t)AMG_NOALLOC_MAX_N,
              "scratch layout");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first
// call on the device, with that device current).
unsigned char* scratch_address() {
  int dev = 0;
  AMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(AMG_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(AMG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  return static_cast<unsigned char*>(g_ptr[dev]);
}

// Clears the control block (every field a solve reads before writing it
// starts at zero, as in a freshly allocated block).
__global__ void k_clear_words(unsigned int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace
}  // namespace amg

using namespace amg;

extern "C" amg_status amg_solve_noalloc(amg_handle h, const double* d_b, double* d_x, double tol, amg_info* info,
                                        hipStream_t stream) {
  try {
    if (!h || !d_b || !d_x || !(tol >= 0.0)) return AMG_ERR_INVALID_ARG;
    Hierarchy& H = *h->H;
    if (H.broken != AMG_OK) return H.broken;
    if (H.prm.solver != AMG_SOLVER_PCG || H.S != 1) return AMG_ERR_INVALID_ARG;
    if ((int64_t)H.n > AMG_NOALLOC_MAX_N || solve_partials_count(H) > AMG_NOALLOC_MAX_PARTIALS)
      return AMG_ERR_SCRATCH_LIMIT;
    unsigned char* base = scratch_address();
    const size_t nmax = AMG_NOALLOC_MAX_N;
    SolveWork w;
    w.ctl = reinterpret_cast<Ctl*>(base);
    w.partials = reinterpret_cast<double*>(base + kCtlBytes);
    double* v = w.partials + AMG_NOALLOC_MAX_PARTIALS;
    w.r = v;
    w.z = v + nmax;
    w.p = v + 2 * nmax;
    w.z2 = v + 3 * nmax;
    w.q = v + 4 * nmax;
    Ctl host_ctl{};
    w.h_ctl = &host_ctl;
    w.graphs = false;
    hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, stream, reinterpret_cast<unsigned int*>(w.ctl),
                       (int)(kCtlBytes / 4));
    AMG_HIP(hipGetLastError());
    return pcg_solve(H, h->opts, w, d_b, d_x, tol, info, stream);
  } catch (const Error& e) {
    return e.status;
  } catch (...) {
    return AMG_ERR_HIP;
  }
}
