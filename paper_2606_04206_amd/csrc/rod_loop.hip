// Reference frames of closed rods (App. A.1, Loop Topology): the frames are
// parallel-transported around the loop, the holonomy angle psi_H left at the
// closing joint is measured against the first frame, and edge j's frame is
// turned about its tangent by -psi_H j / N, so that every joint carries the
// same share of it.  Also the adjoint of that rule, and the material
// curvature of closed rods (App. A.1, Bending, with the closing edge).
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

// adjoint of loop_transport: returns v's adjoint, adds ta's and tb's
template <typename T>
__device__ __forceinline__ V3<T> loop_transport_vjp(V3<T> v, V3<T> ta, V3<T> tb, V3<T> yb,
                                                    V3<T>& tab, V3<T>& tbb) {
  V3<T> bb = cross(ta, tb);
  T c = dot(ta, tb);
  T opc = T(1) + c, bv = dot(bb, v), by = dot(bb, yb);
  V3<T> vb = c * yb - cross(bb, yb) + (by / opc) * bb;
  T cb = dot(v, yb) - bv * by / (opc * opc);
  V3<T> b_b = cross(v, yb) + (T(1) / opc) * (bv * yb + by * v);
  tab += cross(tb, b_b) + cb * tb;
  tbb += cross(b_b, ta) + cb * ta;
  return vb;
}

// reference axis of the first frame: z, or x for a first edge along z
template <typename T>
__device__ __forceinline__ V3<T> loop_axis(V3<T> t0) {
  V3<T> az = mk(T(0), T(0), T(1));
  V3<T> c = cross(t0, az);
  return sqrt(dot(c, c)) < T(1e-6) ? mk(T(1), T(0), T(0)) : az;
}

// unit tangent of edge j of the closed rod starting at vertex v0 (edge N-1
// closes the loop onto vertex 0)
template <typename T>
__device__ __forceinline__ V3<T> loop_tangent(const T* x, int v0, int N, int j) {
  int k = j + 1 == N ? 0 : j + 1;
  V3<T> e = get3(x, 3 * (v0 + k)) - get3(x, 3 * (v0 + j));
  return (T(1) / sqrt(dot(e, e))) * e;
}

// unit quaternion (w, v): a rotation; products compose right to left
template <typename T>
struct LoopQuat {
  T w;
  V3<T> v;
};

// a * b: the rotation b, then a (renormalised, which only removes rounding
// drift: a product of unit quaternions is a unit quaternion)
template <typename T>
__device__ __forceinline__ LoopQuat<T> quat_mul(const LoopQuat<T>& a, const LoopQuat<T>& b) {
  LoopQuat<T> q{a.w * b.w - dot(a.v, b.v), a.w * b.v + b.w * a.v + cross(a.v, b.v)};
  const T s = T(1) / sqrt(q.w * q.w + dot(q.v, q.v));
  return {s * q.w, s * q.v};
}

// the minimal rotation taking unit ta to unit tb: (1 + ta.tb, ta x tb),
// normalised (its norm is sqrt(2 (1 + ta.tb)))
template <typename T>
__device__ __forceinline__ LoopQuat<T> quat_min_rotation(V3<T> ta, V3<T> tb) {
  const T c = T(1) + dot(ta, tb);
  const T s = T(1) / sqrt(T(2) * c);
  return {s * c, s * cross(ta, tb)};
}

template <typename T>
__device__ __forceinline__ V3<T> quat_apply(const LoopQuat<T>& q, V3<T> p) {
  const V3<T> u = cross(q.v, p);
  return p + (T(2) * q.w) * u + T(2) * cross(q.v, u);
}

template <typename T>
__device__ __forceinline__ LoopQuat<T> quat_shfl_up(const LoopQuat<T>& q, int off) {
  return {__shfl_up(q.w, off, 64),
          mk(__shfl_up(q.v.x, off, 64), __shfl_up(q.v.y, off, 64), __shfl_up(q.v.z, off, 64))};
}

template <typename T>
__device__ __forceinline__ LoopQuat<T> quat_shfl(const LoopQuat<T>& q, int src) {
  return {__shfl(q.w, src, 64),
          mk(__shfl(q.v.x, src, 64), __shfl(q.v.y, src, 64), __shfl(q.v.z, src, 64))};
}

// One wave per closed rod.  The frame of edge j is the first frame turned
// by the product of the minimal rotations of joints 1..j; each lane takes a
// contiguous run of joints, forms its run's product, and a prefix product
// over the wave's lanes (six shuffle rounds) gives every lane the rotation
// before its run.  The holonomy angle follows from the whole product and
// the closing joint's rotation; each lane then writes its edges' frames
// turned by -psi_H j / N.
template <typename T>
__global__ __launch_bounds__(64) void k_loop_frames(const int32_t* voff, const T* x, T* d1,
                                                     T* psi) {
  const int r = blockIdx.x, lane = threadIdx.x;
  const int v0 = voff[r], N = voff[r + 1] - v0;
  const int K = (N - 1 + 63) / 64;                    // joints per lane
  const int j0 = 1 + lane * K, j1 = min(N, 1 + (lane + 1) * K);
  const LoopQuat<T> one{T(1), zero3<T>()};
  // this lane's run of joints j0 .. j1-1 (joint j turns edge j-1 onto edge j)
  LoopQuat<T> run = one;
  for (int j = j0; j < j1; ++j)
    run = quat_mul(quat_min_rotation(loop_tangent(x, v0, N, j - 1), loop_tangent(x, v0, N, j)),
                   run);
  // inclusive prefix product over the lanes, later runs on the left
  LoopQuat<T> inc = run;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const LoopQuat<T> lo = quat_shfl_up(inc, off);
    if (lane >= off) inc = quat_mul(inc, lo);
  }
  LoopQuat<T> before = quat_shfl_up(inc, 1);
  if (lane == 0) before = one;
  const LoopQuat<T> all = quat_shfl(inc, 63);
  const V3<T> t0 = loop_tangent(x, v0, N, 0);
  const V3<T> av = loop_axis(t0);
  V3<T> d0 = av - dot(av, t0) * t0;
  d0 = (T(1) / sqrt(dot(d0, d0))) * d0;
  const V3<T> tl = loop_tangent(x, v0, N, N - 1);
  const V3<T> back = quat_apply(quat_min_rotation(tl, t0), quat_apply(all, d0));
  const T ps = atan2(dot(cross(d0, back), t0), dot(d0, back));
  if (lane == 0) {
    put3(d1, 3 * v0, d0);
    if (psi) psi[r] = ps;
  }
  LoopQuat<T> cur = before;
  for (int j = j0; j < j1; ++j) {
    const V3<T> tj = loop_tangent(x, v0, N, j);
    cur = quat_mul(quat_min_rotation(loop_tangent(x, v0, N, j - 1), tj), cur);
    const V3<T> dh = quat_apply(cur, d0);
    const T phi = -ps * T(j) / T(N);
    const T sn = sin(phi), co = cos(phi);
    put3(d1, 3 * (v0 + j), co * dh + sn * cross(tj, dh));
  }
}

// Adjoint of the rule, one thread per closed rod.  xb's rows hold the
// transported frames until each row's adjoint is final: the reverse walk
// over the joints (last first) reads the frames of rows j and j-1 at joint
// j, then edge j's adjoint is complete and rows j and j+1 take their share
// of it; the closing edge's share of row 0 waits in registers until row 0's
// frame has been read for the last time.
template <typename T>
__global__ void k_loop_frames_vjp(const int32_t* voff, int R, const T* x, const T* d1b,
                                  const T* psib, T* xb) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int v0 = voff[r], N = voff[r + 1] - v0;
  V3<T> t0 = loop_tangent(x, v0, N, 0);
  V3<T> av = loop_axis(t0);
  V3<T> d0 = av - dot(av, t0) * t0;
  d0 = (T(1) / sqrt(dot(d0, d0))) * d0;
  put3(xb, 3 * v0, d0);
  V3<T> d = d0, t = t0;
  for (int j = 1; j < N; ++j) {
    V3<T> tn = loop_tangent(x, v0, N, j);
    d = loop_transport(d, t, tn);
    put3(xb, 3 * (v0 + j), d);
    t = tn;
  }
  V3<T> back = loop_transport(d, t, t0);
  T sv = dot(cross(d0, back), t0), cv = dot(d0, back);
  T ps = atan2(sv, cv);
  // psi_H's adjoint: its own plus that of every edge's rotation angle
  T psb = psib ? psib[r] : T(0);
  for (int j = 1; j < N; ++j) {
    T phi = -ps * T(j) / T(N);
    T s = sin(phi), co = cos(phi);
    V3<T> tj = loop_tangent(x, v0, N, j);
    V3<T> dh = get3(xb, 3 * (v0 + j));
    V3<T> g = get3(d1b, 3 * (v0 + j));
    T phib = dot(g, co * cross(tj, dh) - s * dh);
    psb -= phib * T(j) / T(N);
  }
  // psi_H = atan2(t0.(d0 x back), d0.back)
  T den = sv * sv + cv * cv;
  T sb = psb * cv / den, cb = -psb * sv / den;
  V3<T> g0 = sb * cross(back, t0) + cb * back;
  V3<T> backb = sb * cross(t0, d0) + cb * d0;
  V3<T> t0b = sb * cross(d0, back);
  // the closing transport, then the joints from the last to the first
  V3<T> tnb = zero3<T>();
  V3<T> carry = loop_transport_vjp(d, t, t0, backb, tnb, t0b);
  V3<T> eclose = zero3<T>();
  for (int j = N - 1; j >= 1; --j) {
    int k = j + 1 == N ? 0 : j + 1;
    V3<T> e = get3(x, 3 * (v0 + k)) - get3(x, 3 * (v0 + j));
    T ell = sqrt(dot(e, e));
    V3<T> tj = (T(1) / ell) * e;
    T phi = -ps * T(j) / T(N);
    T s = sin(phi), co = cos(phi);
    V3<T> dh = get3(xb, 3 * (v0 + j));
    V3<T> g = get3(d1b, 3 * (v0 + j));
    V3<T> gh = carry + co * g + s * cross(g, tj);
    V3<T> tjb = tnb + s * cross(dh, g);
    V3<T> tpb = zero3<T>();
    carry = loop_transport_vjp(get3(xb, 3 * (v0 + j - 1)), loop_tangent(x, v0, N, j - 1), tj,
                               gh, tpb, tjb);
    V3<T> eb = (T(1) / ell) * (tjb - dot(tj, tjb) * tj);
    if (j == N - 1)
      eclose = eb;
    else
      put3(xb, 3 * (v0 + j + 1), get3(xb, 3 * (v0 + j + 1)) + eb);
    put3(xb, 3 * (v0 + j), -eb);
    tnb = tpb;
  }
  // edge 0: no rotation (phi = 0), the first frame's construction
  V3<T> gh = carry + get3(d1b, 3 * v0) + g0;
  T nd0;
  {
    V3<T> dd = av - dot(av, t0) * t0;
    nd0 = sqrt(dot(dd, dd));
  }
  V3<T> db = (T(1) / nd0) * (gh - dot(d0, gh) * d0);
  t0b += tnb - dot(av, t0) * db - dot(db, t0) * av;
  V3<T> e0 = get3(x, 3 * (v0 + 1)) - get3(x, 3 * v0);
  T ell0 = sqrt(dot(e0, e0));
  V3<T> eb0 = (T(1) / ell0) * (t0b - dot(t0, t0b) * t0);
  put3(xb, 3 * (v0 + 1), get3(xb, 3 * (v0 + 1)) + eb0);
  put3(xb, 3 * v0, eclose - eb0);
}

// Material curvature at every vertex of closed rods: vertex i joins edge
// i-1 (the closing edge for i = 0) and edge i.  One workgroup per rod, its
// lanes striding over the vertices, so the loads of a wave are contiguous.
template <typename T>
__global__ void k_loop_curvature(const int32_t* voff, const T* x, const T* d1, T* kappa) {
  const int r = blockIdx.x;
  const int v0 = voff[r], N = voff[r + 1] - v0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int ip = i == 0 ? N - 1 : i - 1;
    const V3<T> tp = loop_tangent(x, v0, N, ip), t = loop_tangent(x, v0, N, i);
    const V3<T> kb = (T(2) / (T(1) + dot(tp, t))) * cross(tp, t);
    const V3<T> dp = get3(d1, 3 * (v0 + ip)), d = get3(d1, 3 * (v0 + i));
    const V3<T> a1 = T(0.5) * (cross(tp, dp) + cross(t, d));
    const V3<T> a2 = T(0.5) * (dp + d);
    kappa[2 * (v0 + i)] = dot(kb, a1);
    kappa[2 * (v0 + i) + 1] = dot(kb, a2);
  }
}

// Adjoints that vertex v's curvature (kappa b . a1, kappa b . a2), with
// cotangent g, passes to its incoming edge v-1 (tangent, frame) and to its
// outgoing edge v.
template <typename T>
struct LoopCurvAdj {
  V3<T> tp_b, dp_b, t_b, d_b;
};

template <typename T>
__device__ __forceinline__ LoopCurvAdj<T> loop_curvature_vjp_at(const T* x, const T* d1,
                                                               const T* kb_b, int v0, int N,
                                                               int v) {
  const int vp = v == 0 ? N - 1 : v - 1;
  const V3<T> tp = loop_tangent(x, v0, N, vp), t = loop_tangent(x, v0, N, v);
  const V3<T> dp = get3(d1, 3 * (v0 + vp)), d = get3(d1, 3 * (v0 + v));
  const T g1 = kb_b[2 * (v0 + v)], g2 = kb_b[2 * (v0 + v) + 1];
  const T chi = T(1) + dot(tp, t);
  const V3<T> kb = (T(2) / chi) * cross(tp, t);
  const V3<T> a1 = T(0.5) * (cross(tp, dp) + cross(t, d));
  const V3<T> a2 = T(0.5) * (dp + d);
  const V3<T> kbb = g1 * a1 + g2 * a2;   // adjoint of kappa b
  const V3<T> w = (T(0.5) * g1) * kb;     // adjoint of tp x dp and of t x d
  const V3<T> cb = (T(2) / chi) * kbb;    // adjoint of tp x t
  const T chib = -dot(kb, kbb) / chi;     // adjoint of 1 + tp.t
  LoopCurvAdj<T> r;
  r.tp_b = cross(dp, w) + cross(t, cb) + chib * t;
  r.dp_b = (T(0.5) * g2) * kb + cross(w, tp);
  r.t_b = cross(d, w) + cross(cb, tp) + chib * tp;
  r.d_b = (T(0.5) * g2) * kb + cross(w, t);
  return r;
}

// Adjoint of k_loop_curvature, one workgroup per rod.  The thread of
// vertex i evaluates the adjoints of vertices i-1, i and i+1, which give
// the tangent adjoints of edges i-1 and i (hence row i of dL/dx) and the
// frame adjoint of edge i, so every output row has one writer.
template <typename T>
__global__ void k_loop_curvature_vjp(const int32_t* voff, const T* x, const T* d1,
                                     const T* kb_b, T* xb, T* d1b) {
  const int r = blockIdx.x;
  const int v0 = voff[r], N = voff[r + 1] - v0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int im = i == 0 ? N - 1 : i - 1, ip = i + 1 == N ? 0 : i + 1;
    const LoopCurvAdj<T> am = loop_curvature_vjp_at(x, d1, kb_b, v0, N, im);
    const LoopCurvAdj<T> a0 = loop_curvature_vjp_at(x, d1, kb_b, v0, N, i);
    const LoopCurvAdj<T> ap = loop_curvature_vjp_at(x, d1, kb_b, v0, N, ip);
    const V3<T> xm = get3(x, 3 * (v0 + im)), xi = get3(x, 3 * (v0 + i));
    const V3<T> xp = get3(x, 3 * (v0 + ip));
    // edge i (x_i -> x_{i+1}) and edge i-1 (x_{i-1} -> x_i)
    const V3<T> ei = xp - xi, em = xi - xm;
    const T li = sqrt(dot(ei, ei)), lm = sqrt(dot(em, em));
    const V3<T> ti = (T(1) / li) * ei, tm = (T(1) / lm) * em;
    const V3<T> gi = a0.t_b + ap.tp_b, gm = am.t_b + a0.tp_b;
    const V3<T> ebi = (T(1) / li) * (gi - dot(ti, gi) * ti);
    const V3<T> ebm = (T(1) / lm) * (gm - dot(tm, gm) * tm);
    put3(xb, 3 * (v0 + i), ebm - ebi);
    if (d1b) put3(d1b, 3 * (v0 + i), a0.d_b + ap.dp_b);
  }
}

template <typename T>
hipError_t launch_loop_frames(const int32_t* voff, int R, const T* x, T* d1, T* psi,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_loop_frames<T>, dim3(R), dim3(64), 0, st, voff, x, d1, psi);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_loop_frames_vjp(const int32_t* voff, int R, const T* x, const T* d1b,
                                  const T* psib, T* xb, hipStream_t st) {
  hipLaunchKernelGGL(k_loop_frames_vjp<T>, dim3((R + 63) / 64), dim3(64), 0, st, voff, R, x,
                     d1b, psib, xb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_loop_curvature(const int32_t* voff, int R, const T* x, const T* d1, T* kappa,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_loop_curvature<T>, dim3(R), dim3(128), 0, st, voff, x, d1, kappa);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_loop_curvature_vjp(const int32_t* voff, int R, const T* x, const T* d1,
                                     const T* kb_b, T* xb, T* d1b, hipStream_t st) {
  hipLaunchKernelGGL(k_loop_curvature_vjp<T>, dim3(R), dim3(128), 0, st, voff, x, d1, kb_b, xb,
                     d1b);
  return hipGetLastError();
}

// copies the offsets to the host and checks them: a loop needs three vertices
static int check_loop_offsets(const int32_t* voff, int R, hipStream_t st) {
  std::vector<int32_t> off(R + 1);
  if (hipMemcpyAsync(off.data(), voff, sizeof(int32_t) * (R + 1), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return ROD_EHIP;
  if (off[0] < 0) return ROD_EINVAL;
  for (int r = 0; r < R; ++r)
    if (off[r + 1] - off[r] < 3) return ROD_EINVAL;
  return ROD_OK;
}

}  // namespace rods

extern "C" int rods_loop_frames(const int32_t* vert_offsets, int32_t n_rods, int32_t precision,
                                const void* x, void* d1, void* psi, rods_stream_t stream) {
  if (!vert_offsets || !x || !d1 || n_rods < 0) return ROD_EINVAL;
  if (precision != 4 && precision != 8) return ROD_EDTYPE;
  if (n_rods == 0) return ROD_OK;
  hipStream_t st = (hipStream_t)stream;
  int e = rods::check_loop_offsets(vert_offsets, n_rods, st);
  if (e) return e;
  hipError_t he;
  if (precision == 4)
    he = rods::launch_loop_frames<float>(vert_offsets, n_rods, (const float*)x, (float*)d1,
                                         (float*)psi, st);
  else
    he = rods::launch_loop_frames<double>(vert_offsets, n_rods, (const double*)x, (double*)d1,
                                          (double*)psi, st);
  return he == hipSuccess ? ROD_OK : ROD_EHIP;
}

extern "C" int rods_loop_frames_vjp(const int32_t* vert_offsets, int32_t n_rods,
                                    int32_t precision, const void* x, const void* dL_dd1,
                                    const void* dL_dpsi, void* dL_dx, rods_stream_t stream) {
  if (!vert_offsets || !x || !dL_dd1 || !dL_dx || n_rods < 0) return ROD_EINVAL;
  if (precision != 4 && precision != 8) return ROD_EDTYPE;
  if (n_rods == 0) return ROD_OK;
  hipStream_t st = (hipStream_t)stream;
  int e = rods::check_loop_offsets(vert_offsets, n_rods, st);
  if (e) return e;
  hipError_t he;
  if (precision == 4)
    he = rods::launch_loop_frames_vjp<float>(vert_offsets, n_rods, (const float*)x,
                                             (const float*)dL_dd1, (const float*)dL_dpsi,
                                             (float*)dL_dx, st);
  else
    he = rods::launch_loop_frames_vjp<double>(vert_offsets, n_rods, (const double*)x,
                                              (const double*)dL_dd1, (const double*)dL_dpsi,
                                              (double*)dL_dx, st);
  return he == hipSuccess ? ROD_OK : ROD_EHIP;
}

extern "C" int rods_loop_curvature(const int32_t* vert_offsets, int32_t n_rods, int32_t precision,
                                   const void* x, const void* d1, void* kappa,
                                   rods_stream_t stream) {
  if (!vert_offsets || !x || !d1 || !kappa || n_rods < 0) return ROD_EINVAL;
  if (precision != 4 && precision != 8) return ROD_EDTYPE;
  if (n_rods == 0) return ROD_OK;
  hipStream_t st = (hipStream_t)stream;
  int e = rods::check_loop_offsets(vert_offsets, n_rods, st);
  if (e) return e;
  hipError_t he;
  if (precision == 4)
    he = rods::launch_loop_curvature<float>(vert_offsets, n_rods, (const float*)x,
                                            (const float*)d1, (float*)kappa, st);
  else
    he = rods::launch_loop_curvature<double>(vert_offsets, n_rods, (const double*)x,
                                             (const double*)d1, (double*)kappa, st);
  return he == hipSuccess ? ROD_OK : ROD_EHIP;
}

extern "C" int rods_loop_curvature_vjp(const int32_t* vert_offsets, int32_t n_rods,
                                       int32_t precision, const void* x, const void* d1,
                                       const void* dL_dkappa, void* dL_dx, void* dL_dd1,
                                       rods_stream_t stream) {
  if (!vert_offsets || !x || !d1 || !dL_dkappa || !dL_dx || n_rods < 0) return ROD_EINVAL;
  if (precision != 4 && precision != 8) return ROD_EDTYPE;
  if (n_rods == 0) return ROD_OK;
  hipStream_t st = (hipStream_t)stream;
  int e = rods::check_loop_offsets(vert_offsets, n_rods, st);
  if (e) return e;
  hipError_t he;
  if (precision == 4)
    he = rods::launch_loop_curvature_vjp<float>(vert_offsets, n_rods, (const float*)x,
                                                (const float*)d1, (const float*)dL_dkappa,
                                                (float*)dL_dx, (float*)dL_dd1, st);
  else
    he = rods::launch_loop_curvature_vjp<double>(vert_offsets, n_rods, (const double*)x,
                                                 (const double*)d1, (const double*)dL_dkappa,
                                                 (double*)dL_dx, (double*)dL_dd1, st);
  return he == hipSuccess ? ROD_OK : ROD_EHIP;
}
