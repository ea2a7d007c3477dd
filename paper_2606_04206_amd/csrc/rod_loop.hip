// Reference frames of closed rods (App. A.1, Loop Topology): the frames are
// parallel-transported around the loop, the holonomy angle psi_H left at the
// closing joint is measured against the first frame, and edge j's frame is
// turned about its tangent by -psi_H j / N, so that every joint carries the
// same share of it.
#include <hip/hip_runtime.h>

#include <vector>

#include "rods.h"
#include "rod_device.h"

namespace rods {

// minimal rotation taking unit ta to unit tb, applied to v (Rodrigues'
// formula with sin = |ta x tb|, cos = ta.tb), as in the time-stepping kernels
template <typename T>
__device__ __forceinline__ V3<T> loop_transport(V3<T> v, V3<T> ta, V3<T> tb) {
  V3<T> bb = cross(ta, tb);
  T c = dot(ta, tb);
  return c * v + cross(bb, v) + fdiv(dot(bb, v), T(1) + c) * bb;
}

// unit tangent of edge j of the closed rod starting at vertex v0 (edge N-1
// closes the loop onto vertex 0)
template <typename T>
__device__ __forceinline__ V3<T> loop_tangent(const T* x, int v0, int N, int j) {
  int k = j + 1 == N ? 0 : j + 1;
  V3<T> e = get3(x, 3 * (v0 + k)) - get3(x, 3 * (v0 + j));
  return (T(1) / sqrt(dot(e, e))) * e;
}

// One thread per closed rod: the transport around the loop is a chain of
// dependent rotations, and the rule runs once per rollout.  The transported
// frames are written to d1 in the first walk and turned in place in the
// second.
template <typename T>
__global__ void k_loop_frames(const int32_t* voff, int R, const T* x, T* d1, T* psi) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int v0 = voff[r], N = voff[r + 1] - v0;
  V3<T> t0 = loop_tangent(x, v0, N, 0);
  // first frame: the open-rod rule (z, or x for a first edge along z)
  V3<T> az = mk(T(0), T(0), T(1));
  V3<T> c = cross(t0, az);
  V3<T> av = sqrt(dot(c, c)) < T(1e-6) ? mk(T(1), T(0), T(0)) : az;
  V3<T> d0 = av - dot(av, t0) * t0;
  d0 = (T(1) / sqrt(dot(d0, d0))) * d0;
  put3(d1, 3 * v0, d0);
  V3<T> d = d0, t = t0;
  for (int j = 1; j < N; ++j) {
    V3<T> tn = loop_tangent(x, v0, N, j);
    d = loop_transport(d, t, tn);
    put3(d1, 3 * (v0 + j), d);
    t = tn;
  }
  V3<T> back = loop_transport(d, t, t0);
  T ps = atan2(dot(cross(d0, back), t0), dot(d0, back));
  if (psi) psi[r] = ps;
  for (int j = 1; j < N; ++j) {
    T phi = -ps * T(j) / T(N);
    T s = sin(phi), co = cos(phi);
    V3<T> tj = loop_tangent(x, v0, N, j);
    V3<T> dh = get3(d1, 3 * (v0 + j));
    put3(d1, 3 * (v0 + j), co * dh + s * cross(tj, dh));
  }
}

template <typename T>
hipError_t launch_loop_frames(const int32_t* voff, int R, const T* x, T* d1, T* psi,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_loop_frames<T>, dim3((R + 63) / 64), dim3(64), 0, st, voff, R, x, d1,
                     psi);
  return hipGetLastError();
}

}  // namespace rods

extern "C" int rods_loop_frames(const int32_t* vert_offsets, int32_t n_rods, int32_t precision,
                                const void* x, void* d1, void* psi, rods_stream_t stream) {
  if (!vert_offsets || !x || !d1 || n_rods < 0) return ROD_EINVAL;
  if (precision != 4 && precision != 8) return ROD_EDTYPE;
  if (n_rods == 0) return ROD_OK;
  hipStream_t st = (hipStream_t)stream;
  // the offsets are validated on the host: a loop needs three vertices
  std::vector<int32_t> off(n_rods + 1);
  if (hipMemcpyAsync(off.data(), vert_offsets, sizeof(int32_t) * (n_rods + 1),
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return ROD_EHIP;
  if (off[0] < 0) return ROD_EINVAL;
  for (int r = 0; r < n_rods; ++r)
    if (off[r + 1] - off[r] < 3) return ROD_EINVAL;
  hipError_t he;
  if (precision == 4)
    he = rods::launch_loop_frames<float>(vert_offsets, n_rods, (const float*)x, (float*)d1,
                                         (float*)psi, st);
  else
    he = rods::launch_loop_frames<double>(vert_offsets, n_rods, (const double*)x, (double*)d1,
                                          (double*)psi, st);
  return he == hipSuccess ? ROD_OK : ROD_EHIP;
}
