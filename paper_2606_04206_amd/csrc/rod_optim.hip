// Elementwise kernels of the optimisation driver (App. B, Trajectory
// Optimization Setup and System Identification): one Adam update (Kingma and
// Ba, Algorithm 1) and the log/exp maps of parameters optimised in log
// space.  Bandwidth-bound, one thread per parameter.
#include <cmath>

#include "rod_launch.h"

namespace rods {

// p -= lr m_hat / (sqrt(v_hat) + eps) with m = b1 m + (1 - b1) g,
// v = b2 v + (1 - b2) g^2, m_hat = m / bc1, v_hat = v / bc2 (bc = 1 - b^t).
// scale (nullable) multiplies the gradient first: a parameter optimised as
// log q sees dL/dlog q = q dL/dq.
template <typename T>
__global__ void k_adam(T* p, const T* g, const T* scale, T* m, T* v, int64_t n, T lr, T b1, T b2,
                       T eps, T bc1, T bc2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T gi = scale ? scale[i] * g[i] : g[i];
  T mi = b1 * m[i] + (T(1) - b1) * gi;
  T vi = b2 * v[i] + (T(1) - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  T mh = mi / bc1, vh = vi / bc2;
  p[i] = p[i] - lr * mh / (sqrt(vh) + eps);
}

template <typename T>
__global__ void k_log(const T* a, T* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = log(a[i]);
}

template <typename T>
__global__ void k_exp(const T* a, T* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = exp(a[i]);
}

static inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

template <typename T>
hipError_t launch_adam(T* p, const T* g, const T* scale, T* m, T* v, int64_t n, double lr,
                       double b1, double b2, double eps, int t, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const double bc1 = 1.0 - std::pow(b1, t), bc2 = 1.0 - std::pow(b2, t);
  hipLaunchKernelGGL(k_adam<T>, grid_for(n), dim3(256), 0, st, p, g, scale, m, v, n, (T)lr,
                     (T)b1, (T)b2, (T)eps, (T)bc1, (T)bc2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_log(const T* a, T* out, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_log<T>, grid_for(n), dim3(256), 0, st, a, out, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_exp(const T* a, T* out, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_exp<T>, grid_for(n), dim3(256), 0, st, a, out, n);
  return hipGetLastError();
}

#define RODS_OPTIM_INST(T)                                                                       \
  template hipError_t launch_adam<T>(T*, const T*, const T*, T*, T*, int64_t, double, double,   \
                                     double, double, int, hipStream_t);                          \
  template hipError_t launch_log<T>(const T*, T*, int64_t, hipStream_t);                         \
  template hipError_t launch_exp<T>(const T*, T*, int64_t, hipStream_t);

RODS_OPTIM_INST(float)
RODS_OPTIM_INST(double)

}  // namespace rods
