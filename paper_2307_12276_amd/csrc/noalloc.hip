// The Gershgorin interval end from the caller's unscaled fields, with no
// allocation and no op: the entry point for callers that cannot allocate
// (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc).  Same reduction as adl_spectral_bound(ADL_BOUND_GERSHGORIN) on
// an FP64 op of these fields (Gershgorin's row discs, Sec. 2): its block
// partials and arrival ticket live in a file-scope device array instead of
// the op's workspace, and the result goes to device memory, so the call
// neither synchronises nor allocates.
#include "bounds.h"
#include "op.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

namespace adl {
namespace {

// scratch: block partials of the reduction (one double per block, at most
// kScratchBlocks blocks, the most stats_blocks gives) and then the control
// block whose ticket the blocks count on.  Every call on a device shares
// that device's copy; calls that overlap on one device race.
constexpr int kScratchBlocks = 1024;
constexpr size_t kScratchCtlOffset = kScratchBlocks * sizeof(double);
constexpr size_t kScratchBytes = kScratchCtlOffset + 256;
static_assert(sizeof(Ctl) <= 256, "control block fits the scratch tail");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch (looked up once per device,
// with the device current); nullptr with *err set on failure.
void* scratch_on_current_device(hipError_t* err) {
  int dev = -1;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// the reduction's ticket (and the rest of the control block) must start at
// zero: cleared by a kernel (not a memset node, so that a captured graph
// replays it like any other launch)
__global__ void noalloc_ctl_reset_kernel(Ctl* ctl) {
  if (threadIdx.x == 0) {
    Ctl c{};
    *ctl = c;
  }
}

template <bool ADVF>
__global__ __launch_bounds__(kBlock) void noalloc_gershgorin_kernel(FieldView F, FieldScale sc, double* partials,
                                                                    Ctl* ctl, double* alpha_out) {
  gershgorin_blocks<double, ADVF, true>(F, partials, ctl, (int)gridDim.x, (int)blockIdx.x, alpha_out, sc);
}

}  // namespace
}  // namespace adl

using namespace adl;

extern "C" int adl_gershgorin_bound_noalloc(int nx, int ny, double hx, double hy, int bc, const double* Dxx,
                                            const double* Dxy, const double* Dyy, const double* ax,
                                            const double* ay, double ax_c, double ay_c, double* alpha_out,
                                            void* stream) {
  if (nx < 3 || ny < 3) return set_error(ADL_EINVAL, "nx, ny must be >= 3 (got %d, %d)", nx, ny);
  if ((long)nx * ny > (1L << 31)) return set_error(ADL_EINVAL, "grid too large (at most 2^31 points)");
  if (!(hx > 0.0) || !(hy > 0.0) || !std::isfinite(hx) || !std::isfinite(hy))
    return set_error(ADL_EINVAL, "hx, hy must be finite and > 0");
  if (bc != ADL_BC_PERIODIC && bc != ADL_BC_DIRICHLET) return set_error(ADL_EINVAL, "bad bc %d", bc);
  if (!Dxx || !Dxy || !Dyy) return set_error(ADL_EINVAL, "null tensor field");
  if ((ax == nullptr) != (ay == nullptr)) return set_error(ADL_EINVAL, "ax and ay must both be given or both NULL");
  if (!std::isfinite(ax_c) || !std::isfinite(ay_c)) return set_error(ADL_EINVAL, "advection constants not finite");
  if (!alpha_out) return set_error(ADL_EINVAL, "null alpha_out");
  const long n = (long)nx * ny;
  const int nb = stats_blocks(n);
  if (nb > kScratchBlocks) return set_error(ADL_EINVAL, "reduction needs %d blocks, scratch holds %d", nb, kScratchBlocks);
  hipError_t e = hipSuccess;
  unsigned char* base = static_cast<unsigned char*>(scratch_on_current_device(&e));
  if (!base) return set_error(ADL_EHIP, "scratch lookup failed: %s", hipGetErrorString(e));
  double* partials = reinterpret_cast<double*>(base);
  Ctl* ctl = reinterpret_cast<Ctl*>(base + kScratchCtlOffset);
  // the fields as an op would store them: Dxx / hx^2 etc., constants divided
  // as in adl_op_create
  FieldView f{};
  f.kxx = Dxx;
  f.kxy = Dxy;
  f.kyy = Dyy;
  f.ax = ax;
  f.ay = ay;
  f.axc = ax_c / (2.0 * hx);
  f.ayc = ay_c / (2.0 * hy);
  f.nx = nx;
  f.ny = ny;
  f.bc = bc;
  f.f32 = 0;
  const FieldScale sc{1.0 / (hx * hx), 1.0 / (4.0 * hx * hy), 1.0 / (hy * hy), 1.0 / (2.0 * hx), 1.0 / (2.0 * hy)};
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(noalloc_ctl_reset_kernel, dim3(1), dim3(64), 0, st, ctl);
  if (ax)
    hipLaunchKernelGGL(noalloc_gershgorin_kernel<true>, dim3(nb), dim3(kBlock), 0, st, f, sc, partials, ctl, alpha_out);
  else
    hipLaunchKernelGGL(noalloc_gershgorin_kernel<false>, dim3(nb), dim3(kBlock), 0, st, f, sc, partials, ctl,
                       alpha_out);
  e = hipGetLastError();
  if (e != hipSuccess) return set_error(ADL_EHIP, "Gershgorin launch failed: %s", hipGetErrorString(e));
  return ADL_OK;
}
