// Loss of the trajectory-optimisation workloads: the mean squared distance
// of the final positions to a target curve and its gradient, with the
// per-rod partial sums as the only scratch.  Also holds the entry point that
// takes that scratch from a static device array instead of a handle.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rods.h"
#include "rod_launch.h"

namespace rods {

// per-rod part of the MSE loss and dL/dx
template <typename T>
__global__ void k_loss(const int32_t* voff, int R, const T* x, const T* tgt, double* part,
                       T* dldx) {
  int r = blockIdx.x;
  int v0 = voff[r], N = voff[r + 1] - v0;
  __shared__ double red[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    V3<T> d = get3(x, 3 * (v0 + j)) - get3(tgt, 3 * (v0 + j));
    s += (double)dot(d, d);
    if (dldx) put3(dldx, 3 * (v0 + j), (T(2) / (T(R) * T(N))) * d);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[r] = red[0] / ((double)R * N);
}

// fixed-order sum of the per-rod loss parts (one thread)
template <typename T>
__global__ void k_loss_sum(const double* part, int R, T* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int r = 0; r < R; ++r) s += part[r];
  out[0] = (T)s;
}

// Every rod writes its own part (nothing accumulates across calls), so the
// parts need no clearing before a call.
template <typename T>
hipError_t launch_loss(const int32_t* voff, int R, const T* x, const T* tgt, double* part,
                       T* loss, T* dldx, hipStream_t st) {
  hipLaunchKernelGGL(k_loss<T>, dim3(R), dim3(256), 0, st, voff, R, x, tgt, part, dldx);
  if (loss) hipLaunchKernelGGL(k_loss_sum<T>, dim3(1), dim3(64), 0, st, part, R, loss);
  return hipGetLastError();
}

template hipError_t launch_loss<float>(const int32_t*, int, const float*, const float*, double*,
                                       float*, float*, hipStream_t);
template hipError_t launch_loss<double>(const int32_t*, int, const double*, const double*,
                                        double*, double*, double*, hipStream_t);

}  // namespace rods

// ---------------------------------------------------------------------------
// The loss without a handle.  Its per-rod parts live in `scratch`, a static
// device array: each GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` only names the symbol; its device
// address, one per device, comes from hipGetSymbolAddress with that device
// current, and only that address is ever handed to a kernel.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[ROD_LOSS_STATIC_MAX_RODS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};
}  // namespace

namespace rods {
// Looks up (once per device) the device address of `scratch` on the current
// device.  Called by rods_create and by the entry point's first call on a
// device.
int loss_scratch_setup(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ROD_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return ROD_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return ROD_EHIP;
    }
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  if (out) *out = g_scratch_dev[dev];
  return ROD_OK;
}
}  // namespace rods

extern "C" int rods_loss_mse_static(const int32_t* vert_offsets, int32_t n_rods,
                                    int32_t precision, const void* x, const void* target,
                                    void* loss, void* dL_dx, rods_stream_t stream) {
  if (!vert_offsets || !x || !target) return ROD_EINVAL;
  if (n_rods < 1 || n_rods > ROD_LOSS_STATIC_MAX_RODS) return ROD_EINVAL;
  if (precision != 4 && precision != 8) return ROD_EDTYPE;
  double* part = nullptr;
  int e = rods::loss_scratch_setup(&part);
  if (e) return e;
  hipStream_t st = (hipStream_t)stream;
  hipError_t he;
  if (precision == 4)
    he = rods::launch_loss<float>(vert_offsets, n_rods, (const float*)x, (const float*)target,
                                  part, (float*)loss, (float*)dL_dx, st);
  else
    he = rods::launch_loss<double>(vert_offsets, n_rods, (const double*)x,
                                   (const double*)target, part, (double*)loss, (double*)dL_dx,
                                   st);
  return he == hipSuccess ? ROD_OK : ROD_EHIP;
}
