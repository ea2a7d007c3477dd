// HIP kernels of the batched discrete-rod step and its adjoint (gfx950).
//
// One workgroup of W waves owns one rod for a whole launch (a segment of
// steps): the rod's state lives in VGPRs, team lane l holding the C
// consecutive vertices l*C .. l*C+C-1 and the edges that start at them.
// With C even, every even ("red") edge lies inside one lane and every odd
// ("black") edge but the lane's last lies inside one lane too, so an
// iteration of the inextensibility projection needs exactly one neighbour
// exchange pair (positions to the left, corrections to the right).
//
// The file is compiled four times: RODS_TU = 1 instantiates the kernels of
// rods with the twist degree of freedom, RODS_TU = 2 those of rods with
// self-contact, RODS_TU = 3 those of rods with both, the default everything
// else.
//
// Physics (DLO-Lab, Section 3.1 and Appendix A.1): bending forces of the
// discrete elastic rod with frames held fixed, stretching forces for
// extensible rods, symplectic Euler, soft SDF rigid contact (Section 3.2),
// N_C red-black inextensibility iterations, position-based velocity update,
// parallel transport of the reference frames and the plastic rest-curvature
// return map.  The adjoint kernel re-runs each substep from its stored start
// state (projection iterates kept in LDS) and applies the hand-written
// vector-Jacobian product of every sub-step in reverse.
#include "rod_device.h"
#include "rod_launch.h"
#include "rod_selfcontact.h"

#ifndef RODS_TU
#define RODS_TU 0
#endif

namespace rods {

constexpr int FLAG_INEXT = 1, FLAG_PLASTIC = 2, FLAG_SELF = 4;
// values per vertex slot of a stored state: x(3) v(3) kappa_bar(2) d1(3),
// and with the twist degree of freedom theta and its rate
template <bool TW>
constexpr int nfield() { return TW ? 13 : 11; }

template <typename T>
__device__ __forceinline__ V3<T> transport(V3<T> v, V3<T> ta, V3<T> tb) {
  V3<T> bb = cross(ta, tb);
  T c = dot(ta, tb);
  return c * v + cross(bb, v) + fdiv(dot(bb, v), T(1) + c) * bb;
}

// Adjoint of transport: y = R(ta->tb) v.  Returns v_b; adds to ta_b, tb_b.
template <typename T>
__device__ __forceinline__ V3<T> transport_vjp(V3<T> v, V3<T> ta, V3<T> tb, V3<T> yb,
                                               V3<T>& ta_b, V3<T>& tb_b) {
  V3<T> bb = cross(ta, tb);
  T c = dot(ta, tb);
  T bv = dot(bb, v), by = dot(bb, yb);
  T iopc = frcp(T(1) + c);
  V3<T> vb = c * yb - cross(bb, yb) + (by * iopc) * bb;
  T cb = dot(v, yb) - bv * by * iopc * iopc;
  V3<T> bbb = cross(v, yb) + iopc * (bv * yb + by * v);
  ta_b += cross(tb, bbb) + cb * tb;
  tb_b += cross(bbb, ta) + cb * ta;
  return vb;
}

// Bending stencil of an interior vertex (App. A.1, Bending), frames fixed:
// g0 = dU_b/de^{i-1}, g1 = dU_b/de^i.
template <typename T>
struct BendIn {
  V3<T> t0, t1, d1a, d1b, d2a, d2b;
  T il0, il1;      // inverse lengths of edges i-1 and i
  T kr0, kr1;
  T coef, ilbar;   // b / l_bar and 1 / l_bar (both 0 away from interior vertices)
};

template <typename T>
__device__ __forceinline__ void bend_grad(const BendIn<T>& q, V3<T>& g0, V3<T>& g1) {
  T ichi = frcp(T(1) + dot(q.t0, q.t1));
  V3<T> kbv = (T(2) * ichi) * cross(q.t0, q.t1);
  V3<T> a1 = T(0.5) * (q.d2a + q.d2b);
  V3<T> a2 = T(0.5) * (q.d1a + q.d1b);
  T k1 = dot(kbv, a1), k2 = dot(kbv, a2);
  T c1 = q.coef * (k1 - q.kr0), c2 = q.coef * (k2 - q.kr1);
  T s = c1 * k1 + c2 * k2;
  V3<T> A = (T(2) * ichi) * (c1 * a1 + c2 * a2);
  V3<T> tt = ichi * (q.t0 + q.t1);
  g0 = q.il0 * (cross(q.t1, A) - s * tt);
  g1 = q.il1 * (-(s * tt) - cross(q.t0, A));
}

template <typename T>
struct BendBar {
  V3<T> t0, t1, d1a, d1b, d2a, d2b;
  T l0, l1, kr0, kr1, b;
};

// Adjoint of bend_grad given g0_b, g1_b.
template <typename T>
__device__ __forceinline__ void bend_vjp(const BendIn<T>& q, V3<T> g0b, V3<T> g1b,
                                         BendBar<T>& o) {
  T chi = T(1) + dot(q.t0, q.t1);
  T ichi = frcp(chi);
  V3<T> nn = cross(q.t0, q.t1);
  V3<T> kbv = (T(2) * ichi) * nn;
  V3<T> a1 = T(0.5) * (q.d2a + q.d2b);
  V3<T> a2 = T(0.5) * (q.d1a + q.d1b);
  T k1 = dot(kbv, a1), k2 = dot(kbv, a2);
  const T coef = q.coef;
  T dk1 = k1 - q.kr0, dk2 = k2 - q.kr1;
  T c1 = coef * dk1, c2 = coef * dk2;
  T s = c1 * k1 + c2 * k2;
  V3<T> A = (T(2) * ichi) * (c1 * a1 + c2 * a2);
  V3<T> tt = ichi * (q.t0 + q.t1);
  const T il0 = q.il0, il1 = q.il1;
  V3<T> g0 = il0 * (cross(q.t1, A) - s * tt);
  V3<T> g1 = il1 * (-(s * tt) - cross(q.t0, A));
  // g = G / l
  V3<T> G0b = il0 * g0b, G1b = il1 * g1b;
  o.l0 = -dot(g0, g0b) * il0;
  o.l1 = -dot(g1, g1b) * il1;
  V3<T> Gsb = G0b + G1b;
  T sb = -dot(tt, Gsb);
  V3<T> ttb = (-s) * Gsb;
  V3<T> t0b = ichi * ttb - cross(A, G1b);
  V3<T> t1b = ichi * ttb + cross(A, G0b);
  V3<T> Ab = cross(G0b, q.t1) - cross(G1b, q.t0);
  T chib = -dot(tt, ttb) * ichi - dot(A, Ab) * ichi;
  T c1b = T(2) * ichi * dot(a1, Ab) + k1 * sb;
  T c2b = T(2) * ichi * dot(a2, Ab) + k2 * sb;
  V3<T> a1b = (T(2) * ichi * c1) * Ab;
  V3<T> a2b = (T(2) * ichi * c2) * Ab;
  T k1b = c1 * sb + coef * c1b;
  T k2b = c2 * sb + coef * c2b;
  o.kr0 = -coef * c1b;
  o.kr1 = -coef * c2b;
  o.b = (c1b * dk1 + c2b * dk2) * q.ilbar;
  V3<T> kbvb = k1b * a1 + k2b * a2;
  a1b += k1b * kbv;
  a2b += k2b * kbv;
  // kbv = 2 nn / chi, chi = 1 + t0.t1
  chib -= dot(kbv, kbvb) * ichi;
  V3<T> nb = (T(2) * ichi) * kbvb;
  t0b += cross(q.t1, nb) + chib * q.t1;
  t1b += cross(nb, q.t0) + chib * q.t0;
  o.t0 = t0b;
  o.t1 = t1b;
  o.d2a = T(0.5) * a1b;
  o.d2b = T(0.5) * a1b;
  o.d1a = T(0.5) * a2b;
  o.d1b = T(0.5) * a2b;
}

// Material curvature (kb.a1, kb.a2) at an interior vertex (App. A.1).
template <typename T>
__device__ __forceinline__ void curvature(V3<T> t0, V3<T> t1, V3<T> d1a, V3<T> d1b, T& k1, T& k2) {
  T ichi = frcp(T(1) + dot(t0, t1));
  V3<T> kbv = (T(2) * ichi) * cross(t0, t1);
  V3<T> a1 = T(0.5) * (cross(t0, d1a) + cross(t1, d1b));
  V3<T> a2 = T(0.5) * (d1a + d1b);
  k1 = dot(kbv, a1);
  k2 = dot(kbv, a2);
}

// Adjoint of curvature w.r.t. t0, t1, d1a, d1b (d2 = t x d1 inside).
template <typename T>
__device__ __forceinline__ void curvature_vjp(V3<T> t0, V3<T> t1, V3<T> d1a, V3<T> d1b, T k1b,
                                              T k2b, V3<T>& t0b, V3<T>& t1b, V3<T>& d1ab,
                                              V3<T>& d1bb) {
  T chi = T(1) + dot(t0, t1);
  T ichi = frcp(chi);
  V3<T> kbv = (T(2) * ichi) * cross(t0, t1);
  V3<T> d2a = cross(t0, d1a), d2b = cross(t1, d1b);
  V3<T> a1 = T(0.5) * (d2a + d2b);
  V3<T> a2 = T(0.5) * (d1a + d1b);
  V3<T> kbvb = k1b * a1 + k2b * a2;
  V3<T> a1b = k1b * kbv, a2b = k2b * kbv;
  T chib = -dot(kbv, kbvb) * ichi;
  V3<T> nb = (T(2) * ichi) * kbvb;
  t0b = cross(t1, nb) + chib * t1;
  t1b = cross(nb, t0) + chib * t0;
  V3<T> d2ab = T(0.5) * a1b;   // same for d2b
  d1ab = T(0.5) * a2b + cross(d2ab, t0);
  d1bb = T(0.5) * a2b + cross(d2ab, t1);
  t0b += cross(d1a, d2ab);
  t1b += cross(d1b, d2ab);
}

// ---------------------------------------------------------------------------
// Twist degree of freedom (App. A.1, DLO Representation and Twisting).  The
// material director m1 is the reference d1 turned by theta about t; the
// twisting strain at an interior vertex is theta^i - theta^{i-1} + m_ref_i
// (rest twist zero) with m_ref_i the signed angle, about t^i, from the
// spatial parallel transport of d1^{i-1} to d1^i.  Theta is a dynamic
// degree of freedom driven by -dU/dtheta; the twist energy acts on the
// vertices through the holonomy gradient dm_ref_i/de = (kb)_i / (2 |e|) of
// each adjacent edge.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ V3<T> material_m1(V3<T> t, V3<T> d1, T th) {
  T s = sin(th), c = cos(th);
  return c * d1 + s * cross(t, d1);
}

// Adjoint of material_m1: returns d1_b, adds to t_b and th_b.
template <typename T>
__device__ __forceinline__ V3<T> material_m1_vjp(V3<T> t, V3<T> d1, T th, V3<T> m1b, V3<T>& tb,
                                                 T& thb) {
  T s = sin(th), c = cos(th);
  thb += dot(m1b, c * cross(t, d1) - s * d1);
  tb += s * cross(d1, m1b);
  return c * m1b + s * cross(m1b, t);
}

// Twist stencil of an interior vertex: edges i-1 (a) and i (b) with their
// material (m1) and reference (d1) directors and angles; coef = b / l_bar,
// tcoef = beta / l_bar (both 0 away from interior vertices).
template <typename T>
struct TwIn {
  V3<T> t0, t1, m1a, m1b, d1a, d1b;
  T il0, il1, tha, thb;
  T kr0, kr1, coef, ilbar, tcoef;
};

// Adds the twist energy's edge gradients to g0 = dU/de^{i-1}, g1 = dU/de^i
// and returns the torques -dU/dtheta (bending through the material frames,
// and twisting) on edges i-1 (Ta) and i (Tb).
template <typename T>
__device__ __forceinline__ void twist_grad(const TwIn<T>& q, V3<T>& g0, V3<T>& g1, T& Ta,
                                           T& Tb) {
  T ichi = frcp(T(1) + dot(q.t0, q.t1));
  V3<T> kbv = (T(2) * ichi) * cross(q.t0, q.t1);
  V3<T> m2a = cross(q.t0, q.m1a), m2b = cross(q.t1, q.m1b);
  V3<T> a1 = T(0.5) * (m2a + m2b), a2 = T(0.5) * (q.m1a + q.m1b);
  T c1 = q.coef * (dot(kbv, a1) - q.kr0), c2 = q.coef * (dot(kbv, a2) - q.kr1);
  V3<T> u = transport(q.d1a, q.t0, q.t1);
  T g = q.tcoef * (q.thb - q.tha + atan2(dot(cross(u, q.d1b), q.t1), dot(u, q.d1b)));
  Ta = T(0.5) * (c1 * dot(kbv, q.m1a) - c2 * dot(kbv, m2a)) + g;
  Tb = T(0.5) * (c1 * dot(kbv, q.m1b) - c2 * dot(kbv, m2b)) - g;
  T hg = T(0.5) * g;
  g0 += (hg * q.il0) * kbv;
  g1 += (hg * q.il1) * kbv;
}

template <typename T>
struct TwBar {
  V3<T> t0, t1, m1a, m1b, m2a, m2b, d1a, d1b;
  T l0, l1, tha, thb, kr0, kr1, b;
};

// Adjoint of twist_grad given the adjoints of its g0, g1 contributions and
// of the two torques.  m2 = t x m1 is left to the caller (m2a, m2b).
template <typename T>
__device__ __forceinline__ void twist_vjp(const TwIn<T>& q, V3<T> g0b, V3<T> g1b, T Tab, T Tbb,
                                          TwBar<T>& o) {
  T ichi = frcp(T(1) + dot(q.t0, q.t1));
  V3<T> kbv = (T(2) * ichi) * cross(q.t0, q.t1);
  V3<T> m2a = cross(q.t0, q.m1a), m2b = cross(q.t1, q.m1b);
  V3<T> a1 = T(0.5) * (m2a + m2b), a2 = T(0.5) * (q.m1a + q.m1b);
  T dk1 = dot(kbv, a1) - q.kr0, dk2 = dot(kbv, a2) - q.kr1;
  T c1 = q.coef * dk1, c2 = q.coef * dk2;
  V3<T> u = transport(q.d1a, q.t0, q.t1);
  T sn = dot(cross(u, q.d1b), q.t1), cs = dot(u, q.d1b);
  T g = q.tcoef * (q.thb - q.tha + atan2(sn, cs));
  // g0 += (g/2) il0 kbv, g1 += (g/2) il1 kbv
  T k0 = dot(kbv, g0b), k1 = dot(kbv, g1b);
  T gb = T(0.5) * (q.il0 * k0 + q.il1 * k1) + Tab - Tbb;
  V3<T> kbvb = (T(0.5) * g * q.il0) * g0b + (T(0.5) * g * q.il1) * g1b;
  o.l0 = -T(0.5) * g * q.il0 * q.il0 * k0;
  o.l1 = -T(0.5) * g * q.il1 * q.il1 * k1;
  // bending torques
  V3<T> P1 = T(0.5) * (Tab * q.m1a + Tbb * q.m1b);
  V3<T> P2 = T(0.5) * (Tab * m2a + Tbb * m2b);
  T c1b = dot(kbv, P1), c2b = -dot(kbv, P2);
  kbvb += c1 * P1 - c2 * P2;
  T ca = T(0.5) * Tab, cb = T(0.5) * Tbb;
  V3<T> a1b = (q.coef * c1b) * kbv, a2b = (q.coef * c2b) * kbv;
  o.m1a = (ca * c1) * kbv + T(0.5) * a2b;
  o.m1b = (cb * c1) * kbv + T(0.5) * a2b;
  o.m2a = (-(ca * c2)) * kbv + T(0.5) * a1b;
  o.m2b = (-(cb * c2)) * kbv + T(0.5) * a1b;
  kbvb += (q.coef * c1b) * a1 + (q.coef * c2b) * a2;
  o.kr0 = -q.coef * c1b;
  o.kr1 = -q.coef * c2b;
  o.b = (c1b * dk1 + c2b * dk2) * q.ilbar;
  // twisting strain and reference twist (sn = cs = 0 where tcoef = 0)
  T taub = q.tcoef * gb;
  o.thb = taub;
  o.tha = -taub;
  T r2 = sn * sn + cs * cs;
  T mb = r2 > T(0) ? taub * frcp(r2) : T(0);
  T snb = cs * mb, csb = -(sn * mb);
  V3<T> ub = snb * cross(q.d1b, q.t1) + csb * q.d1b;
  o.d1b = snb * cross(q.t1, u) + csb * u;
  V3<T> t0b = zero3<T>();
  V3<T> t1b = snb * cross(u, q.d1b);
  o.d1a = transport_vjp(q.d1a, q.t0, q.t1, ub, t0b, t1b);
  // kbv = 2 (t0 x t1) / (1 + t0.t1)
  T chib = -dot(kbv, kbvb) * ichi;
  V3<T> nb = (T(2) * ichi) * kbvb;
  o.t0 = t0b + cross(q.t1, nb) + chib * q.t1;
  o.t1 = t1b + cross(nb, q.t0) + chib * q.t0;
}

// One inextensibility projection of edge (pj, pk) (App. A.1).  With
// lambda = (|D| - r) / W along t = D/|D|, pj moves by lambda wj t and pk by
// -lambda wk t; written here as s = 1 - r/|D|, pj += s aj D, pk -= s ak D
// with the per-edge ratios aj = wj/W, ak = wk/W (both zero for an edge that
// is not projected).  D is the edge vector it saw; returns 1/|D|.
template <typename T>
__device__ __forceinline__ T project_edge(V3<T>& pj, V3<T>& pk, T aj, T ak, T r, V3<T>& D) {
  D = pk - pj;
  T il = frsq(fmax(dot(D, D), T(1e-30)));
  T s = T(1) - r * il;
  pj += (s * aj) * D;
  pk -= (s * ak) * D;
  return il;
}

// Adjoint of project_edge from what it saw (D, 1/|D|): the Jacobian of
// s(D) D is (1 - r/|D|) I + r D D^T / |D|^3.  Given the adjoints Aj, Ak of
// the moved endpoints returns D_b, with pj_b = Aj - D_b and pk_b = Ak + D_b.
template <typename T>
__device__ __forceinline__ V3<T> project_edge_vjp(V3<T> D, T il, T aj, T ak, T r, V3<T> Aj,
                                                  V3<T> Ak) {
  V3<T> q = aj * Aj - ak * Ak;
  T ril = r * il;
  T c2 = ril * il * il * dot(D, q);   // left to right: finite when r = 0
  return (T(1) - ril) * q + c2 * D;
}

// ---------------------------------------------------------------------------
// rigid contact (Section 3.2): soft SDF impulses on free vertices
// ---------------------------------------------------------------------------
template <typename T>
struct Prim {
  int type;
  V3<T> a, b;
  T r;
};

template <typename T>
__device__ __forceinline__ Prim<T> load_prim(const RodArgs<T>& a, int k) {
  Prim<T> p;
  p.type = a.prim_type[k];
  p.a = get3(a.prim_a, 3 * k);
  p.b = get3(a.prim_b, 3 * k);
  p.r = a.prim_r[k];
  return p;
}

// signed distance, unit normal, and whether the capsule parameter is interior
template <typename T>
__device__ __forceinline__ T sdf_normal(const Prim<T>& p, V3<T> x, V3<T>& n, bool& interior,
                                        T& nq) {
  interior = false;
  if (p.type == 0) {
    n = p.b;
    nq = T(0);
    return dot(x - p.a, p.b);
  }
  V3<T> q;
  if (p.type == 1) {
    q = x - p.a;
  } else {
    V3<T> ab = p.b - p.a;
    T s = fdiv(dot(x - p.a, ab), dot(ab, ab));
    interior = (s > T(0)) && (s < T(1));
    s = s < T(0) ? T(0) : (s > T(1) ? T(1) : s);
    q = x - (p.a + s * ab);
  }
  nq = fsqrt(dot(q, q));
  n = frcp(nq) * q;
  return nq - p.r;
}

template <typename T>
__device__ __forceinline__ T exp_t(T a) { return exp(a); }

// One primitive's response on v; returns true when active.
template <typename T>
__device__ __forceinline__ bool contact_one(const Prim<T>& p, V3<T> x, T rad, T mu, T e, T eps_s,
                                            T f_thresh, V3<T>& v) {
  V3<T> n;
  bool interior;
  T nq;
  T sdf = sdf_normal(p, x, n, interior, nq);
  T d = rad - sdf;
  T f = d >= T(0) ? T(1) : exp_t(fdiv(d, eps_s));
  T vn = dot(v, n);
  if (!(f > f_thresh && vn < T(0))) return false;
  T dvn = -(T(1) + e) * vn;
  V3<T> vt = v - vn * n;
  T vtn = fsqrt(dot(vt, vt));
  T s = T(0);
  if (vtn > T(0)) {
    T sr = T(1) - fdiv(mu * dvn, vtn);
    s = sr > T(0) ? sr : T(0);
  }
  V3<T> vres = (-e * vn) * n + s * vt;
  v = (T(1) - f) * v + f * vres;
  return true;
}

// Adjoint of contact_one at input velocity vin (re-evaluated); vb is the
// adjoint of the output velocity, updated in place to that of the input;
// adds to xb.
template <typename T>
__device__ __forceinline__ void contact_one_vjp(const Prim<T>& p, V3<T> x, T rad, T mu, T e,
                                                T eps_s, T f_thresh, V3<T> vin, V3<T>& vb,
                                                V3<T>& xb) {
  V3<T> n;
  bool interior;
  T nq;
  T sdf = sdf_normal(p, x, n, interior, nq);
  T d = rad - sdf;
  T f = d >= T(0) ? T(1) : exp_t(fdiv(d, eps_s));
  T vn = dot(vin, n);
  if (!(f > f_thresh && vn < T(0))) return;
  T dvn = -(T(1) + e) * vn;
  V3<T> vt = vin - vn * n;
  T vtn = fsqrt(dot(vt, vt));
  T s = T(0);
  bool slide = false;
  if (vtn > T(0)) {
    T sr = T(1) - fdiv(mu * dvn, vtn);
    slide = sr > T(0);
    s = slide ? sr : T(0);
  }
  V3<T> vres = (-e * vn) * n + s * vt;
  V3<T> vob = vb;
  V3<T> vib = (T(1) - f) * vob;
  V3<T> vresb = f * vob;
  T fb = dot(vres - vin, vob);
  T vnb = -e * dot(n, vresb);
  V3<T> nb = (-e * vn) * vresb;
  T sb = dot(vt, vresb);
  V3<T> vtb = s * vresb;
  if (slide) {
    T dvnb = fdiv(-mu * sb, vtn);
    T vtnb = fdiv(mu * dvn * sb, vtn * vtn);
    vnb += -(T(1) + e) * dvnb;
    vtb += fdiv(vtnb, vtn) * vt;
  }
  vib += vtb;
  vnb -= dot(n, vtb);
  nb -= vn * vtb;
  vib += vnb * n;
  nb += vnb * vin;
  T db = d < T(0) ? fdiv(fb * f, eps_s) : T(0);
  T sdfb = -db;
  if (p.type == 0) {
    xb += sdfb * p.b;
  } else {
    V3<T> perp = frcp(nq) * (nb - dot(n, nb) * n);
    V3<T> g = sdfb * n + perp;
    if (p.type == 2 && interior) {
      V3<T> ab = p.b - p.a;
      V3<T> u = frcp(fsqrt(dot(ab, ab))) * ab;
      g -= dot(perp, u) * u;
    }
    xb += g;
  }
  vb = vib;
}

// Contact with a moving sphere (centre p.a, radius p.r; Section 3.2, Rigid
// Body): the response of contact_one acts on the velocity relative to the
// body's contact point c + R n, which moves at vb = Vb + Om x (R n).  Every
// vertex sees the body's substep-start state.  Returns true when active,
// with the unit normal in n.
template <typename T>
__device__ __forceinline__ bool contact_moving(const Prim<T>& p, V3<T> x, T rad, T mu, T e,
                                               T eps_s, T f_thresh, V3<T> Vb, V3<T> Om,
                                               V3<T>& v, V3<T>& n) {
  const V3<T> q = x - p.a;
  const T nq = fsqrt(dot(q, q));
  n = frcp(nq) * q;
  const T d = rad - (nq - p.r);
  const T f = d >= T(0) ? T(1) : exp_t(fdiv(d, eps_s));
  const V3<T> vb = Vb + cross(Om, p.r * n);
  const V3<T> vrel = v - vb;
  const T vn = dot(vrel, n);
  if (!(f > f_thresh && vn < T(0))) return false;
  const T dvn = -(T(1) + e) * vn;
  const V3<T> vt = vrel - vn * n;
  const T vtn = fsqrt(dot(vt, vt));
  T s = T(0);
  if (vtn > T(0)) {
    T sr = T(1) - fdiv(mu * dvn, vtn);
    s = sr > T(0) ? sr : T(0);
  }
  const V3<T> vres = (-e * vn) * n + s * vt;
  v = vb + ((T(1) - f) * vrel + f * vres);
  return true;
}

// Adjoint of contact_moving at input velocity vin, together with the
// reaction it feeds: the vertex's momentum change dp = m (v_out - vin) is
// summed into P and (R n) x dp into L, whose adjoints Pb, Lb are given.
// vb: adjoint of the output velocity, replaced by that of the input; xb +=
// the position adjoint; acc[0..8] += the adjoints of the body's centre,
// velocity and angular velocity.
template <typename T>
__device__ __forceinline__ void contact_moving_vjp(const Prim<T>& p, V3<T> x, T rad, T mu, T e,
                                                   T eps_s, T f_thresh, V3<T> Vb, V3<T> Om,
                                                   T m, V3<T> vin, V3<T> Pb, V3<T> Lb,
                                                   V3<T>& vb_adj, V3<T>& xb, T (&acc)[9]) {
  const V3<T> q = x - p.a;
  const T nq = fsqrt(dot(q, q));
  const V3<T> n = frcp(nq) * q;
  const T d = rad - (nq - p.r);
  const T f = d >= T(0) ? T(1) : exp_t(fdiv(d, eps_s));
  const V3<T> vbody = Vb + cross(Om, p.r * n);
  const V3<T> vrel = vin - vbody;
  const T vn = dot(vrel, n);
  if (!(f > f_thresh && vn < T(0))) return;
  const T dvn = -(T(1) + e) * vn;
  const V3<T> vt = vrel - vn * n;
  const T vtn = fsqrt(dot(vt, vt));
  T s = T(0);
  bool slide = false;
  if (vtn > T(0)) {
    T sr = T(1) - fdiv(mu * dvn, vtn);
    slide = sr > T(0);
    s = slide ? sr : T(0);
  }
  const V3<T> vres = (-e * vn) * n + s * vt;
  const V3<T> vout = vbody + ((T(1) - f) * vrel + f * vres);
  const V3<T> dp = m * (vout - vin);
  // reaction: P += dp, L += (R n) x dp
  const V3<T> dpb = Pb + p.r * cross(Lb, n);
  V3<T> nb = p.r * cross(dp, Lb);
  const V3<T> vob = vb_adj + m * dpb;
  // v_out = vb + (1 - f) v_rel + f v_res(v_rel, n)
  V3<T> vrb = (T(1) - f) * vob;
  const V3<T> vresb = f * vob;
  const T fb = dot(vres - vrel, vob);
  T vnb = -e * dot(n, vresb);
  nb += (-e * vn) * vresb;
  const T sb = dot(vt, vresb);
  V3<T> vtb = s * vresb;
  if (slide) {
    T dvnb = fdiv(-mu * sb, vtn);
    T vtnb = fdiv(mu * dvn * sb, vtn * vtn);
    vnb += -(T(1) + e) * dvnb;
    vtb += fdiv(vtnb, vtn) * vt;
  }
  vrb += vtb;
  vnb -= dot(n, vtb);
  nb -= vn * vtb;
  vrb += vnb * n;
  nb += vnb * vrel;
  // v_rel = vin - vb, vb = Vb + Om x (R n)
  const V3<T> vbb = vob - vrb;
  nb += p.r * cross(vbb, Om);
  const V3<T> omb = p.r * cross(n, vbb);
  // depth and normal through q = x - c
  const T db = d < T(0) ? fdiv(fb * f, eps_s) : T(0);
  const V3<T> g = (-db) * n + frcp(nq) * (nb - dot(n, nb) * n);
  xb += g;
  acc[0] -= g.x; acc[1] -= g.y; acc[2] -= g.z;
  acc[3] += vbb.x; acc[4] += vbb.y; acc[5] += vbb.z;
  acc[6] += omb.x; acc[7] += omb.y; acc[8] += omb.z;
  vb_adj = vrb - m * dpb;
}

// ---------------------------------------------------------------------------
// Per-lane rod state
// ---------------------------------------------------------------------------
template <typename T, int C>
struct Rec {   // what the adjoint needs from one substep's forward run
  V3<T> t[C], d1[C];
  T il[C], kr0[C], kr1[C];   // il: inverse edge lengths
  V3<T> tp, d1p;
  T ilp;
  V3<T> x[C], v1[C];
  V3<T> t1[C], d1n[C];
  T il1[C];
  V3<T> t1p, d1np;
  T kel0[C], kel1[C], inrm[C], phi[C];   // inrm = 1 / |kappa_el| on yield
  bool yld[C];
  V3<T> x1[C], v3[C];   // positions after projection, velocities before self-friction
  // twist: angles at the substep start and after the update, the previous
  // lane's last edge (angle, material d1 at the start)
  T th[C], th1[C], thp;
  V3<T> m1p;
};

// BD: the rod may have moving rigid bodies (instantiated for those rods only)
template <typename T, int C, int W, bool SC, bool TW = false, bool BD = false>
struct Rod {
  static constexpr int TL = 64 * W;   // lanes per team
  static constexpr int NV = TL * C;   // vertex capacity of the team
  static constexpr int NFIELD = nfield<TW>();
  int rod, N, v0, tl, flags, p0, p1;
  // self-contact: LDS staging, counts, hash and list offsets; the rod's
  // block of global pair scratch; the adjoint's contact-pass inputs (global)
  T *sc_pos, *sc_aux, *sc_adj, *sc_w, *sc_r;
  float* sc_vc;   // the adjoint's recorded per-vertex counts
  int *sc_cnt, *sc_fcnt, *sc_hcnt, *sc_hstart, *sc_items, *sc_lo, *sc_hi, *sc_slo, *sc_shi,
      *sc_tmp;
  int *g_hdr, *g_trilo, *g_hpos, *g_suphi, *g_cidx;
  SPair *g_pairs, *g_sup;
  // the substep's pair arrays: g_pairs, g_hpos, g_d0, g_d0b and g_rec point
  // either into the rod's global block (gb_*) or, when the substep's pairs
  // fit, into the LDS left over past the fixed layout (the hash, dead after
  // a build, and the rest of the workgroup's allocation); g_rec2 (the
  // adjoint's friction position adjoints) stays global
  int* gb_hpos;
  SPair* gb_pairs;
  T *gb_d0, *gb_d0b, *gb_rec, *g_rec2;
  unsigned char* sc_cache;
  int sc_cache_bytes;
  // the superset of candidates (pairs within the margin plus a skin at the
  // positions xb of its last build) and its size
  V3<T> sc_xb[C];
  bool sc_built;
  int sc_S;
  T *g_d0, *g_d0b, *g_rec;
  int sc_rv, sc_M, sc_P;
  T sc_cell0, sc_lmax;
  int sc_flags;
  // work counters of the self-contact sweeps: active pair-passes and pairs
  // in friction, summed into a.sc_stats at the end of the launch
  unsigned st_act, st_fric;
  T* ctape;
  T b, sig, rc, mu, e, K;
  T w[C], rest[C], lbar[C], ks[C], rad[C];
  T aj[C], ak[C];   // projection ratios w_j/W, w_k/W of the edge starting at vertex c
  // multi-wave teams: the previous lane's last edge (rest length, ratios,
  // edge vector at the predicted positions), which both of its lanes project
  T restp, ajp, akp;
  V3<T> E0p;
  T coef[C], ilbar[C];   // b / l_bar and 1 / l_bar at interior vertices, else 0
  // the forward (no recording) carries a substep's end geometry into the
  // next substep: the same values edges() and prev_edge() would recompute
  // from the same positions and frames
  bool geo_ok, prev_ok;
  V3<T> tc[C], tpc, d1pc;
  T lc[C], ilc[C], ilpc;
  int gs[C];
  V3<T> x[C], v[C], d1[C];
  T kr0[C], kr1[C];
  // twist: angle and rate per edge, inverse inertia (0: held), beta / l_bar
  T th[C], om[C], jt[C], tcoef[C];
  // moving rigid bodies of the rod (dyn: at least one): their state and, in
  // the adjoint, its adjoint, NB_VALS values per primitive slot k - p0 in LDS
  bool dyn;
  T *bs, *lbs;

  // every lane of the team calls these (they end with a team barrier)
  __device__ void body_setup(const RodArgs<T>& a, unsigned char* smem) {
    dyn = false;
    bs = lbs = nullptr;
    if (!BD || !a.bw) return;
    for (int k = p0; k < p1; ++k) dyn |= a.bw[k] > T(0);
    bs = reinterpret_cast<T*>(smem + a.body_lds);
    lbs = bs + NB_MAX * NB_VALS;
  }
  __device__ void load_bodies(T* dst, const T* src) const {
    for (int i = tl; i < (p1 - p0) * NB_VALS; i += TL) dst[i] = src[(int64_t)p0 * NB_VALS + i];
    __syncthreads();
  }
  // the adjoint's body tape, one substep ahead: each lane holds up to BPF
  // values of the rod's block in registers until install_bodies
  static constexpr int BPF = (NB_MAX * NB_VALS + TL - 1) / TL;
  __device__ void fetch_bodies(const T* src, T (&pf)[BPF]) const {
#pragma unroll
    for (int q = 0; q < BPF; ++q) {
      const int i = tl + q * TL;
      pf[q] = i < (p1 - p0) * NB_VALS ? src[(int64_t)p0 * NB_VALS + i] : T(0);
    }
  }
  __device__ void install_bodies(const T (&pf)[BPF]) const {
#pragma unroll
    for (int q = 0; q < BPF; ++q) {
      const int i = tl + q * TL;
      if (i < (p1 - p0) * NB_VALS) bs[i] = pf[q];
    }
    __syncthreads();
  }
  __device__ void store_bodies(T* dst, const T* src) const {
    for (int i = tl; i < (p1 - p0) * NB_VALS; i += TL) dst[(int64_t)p0 * NB_VALS + i] = src[i];
  }

  __device__ __forceinline__ int gi(int c) const { return tl * C + c; }
  __device__ __forceinline__ bool vvalid(int c) const { return gi(c) < N; }
  __device__ __forceinline__ bool evalid(int c) const { return gi(c) < N - 1; }
  __device__ __forceinline__ bool ivalid(int c) const { return gi(c) >= 1 && gi(c) <= N - 2; }

  __device__ void load_static(const RodArgs<T>& a, Team<T, W>& X) {
    rod = a.rods[blockIdx.x];
    v0 = a.voff[rod];
    N = a.voff[rod + 1] - v0;
    tl = threadIdx.x;
    flags = a.flags[rod];
    b = a.b[rod];
    sig = a.sigma[rod];
    rc = a.rc[rod];
    mu = a.mu[rod];
    e = a.restit[rod];
    K = a.K[rod];
    p0 = a.prim_off ? a.prim_off[rod] : 0;
    p1 = a.prim_off ? a.prim_off[rod + 1] : 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      int g = gi(c);
      bool vv = g < N;
      w[c] = vv ? a.w[v0 + g] : T(0);
      gs[c] = vv ? a.gslot[v0 + g] : -1;
      rad[c] = vv ? a.radius[v0 + g] : T(0);
      rest[c] = (g < N - 1) ? a.rest[v0 + g] : T(0);
    }
    T rp[1] = {rest[C - 1]};
    X.prev(rp);
    T rn[2] = {rad[0], w[0]};
    X.next(rn);
    const T wn = rn[1];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      T wk = c < C - 1 ? w[c + 1] : wn;
      T Wsum = w[c] + wk;
      bool pe = evalid(c) && Wsum > T(0);
      aj[c] = pe ? w[c] / Wsum : T(0);
      ak[c] = pe ? wk / Wsum : T(0);
      lbar[c] = ivalid(c) ? T(0.5) * ((c ? rest[c - 1] : rp[0]) + rest[c]) : T(0);
      ilbar[c] = ivalid(c) ? T(1) / lbar[c] : T(0);
      coef[c] = b * ilbar[c];
      T rb = T(0.5) * (rad[c] + (c < C - 1 ? rad[c + 1] : rn[0]));
      ks[c] = evalid(c) ? K * T(3.14159265358979323846) * rb * rb : T(0);
      if constexpr (TW) {
        // an edge with both vertices kinematic holds its twist
        jt[c] = pe ? a.jt[v0 + gi(c)] : T(0);
        T r2 = rad[c] * rad[c];
        tcoef[c] = ivalid(c) ? a.Gt[rod] * T(3.14159265358979323846) * r2 * r2 / T(2) * ilbar[c]
                             : T(0);
      }
    }
    if constexpr (W > 1) {
      T q[3] = {rest[C - 1], aj[C - 1], ak[C - 1]};
      X.prev(q);
      restp = q[0];
      ajp = q[1];
      akp = q[2];
    }
  }

  __device__ void load_state(const T* X, const T* Vv, const T* KB, const T* D1) {
    geo_ok = prev_ok = false;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      int g = gi(c), r = v0 + g;
      bool vv = g < N;
      x[c] = vv ? get3(X, 3 * r) : zero3<T>();
      v[c] = vv ? get3(Vv, 3 * r) : zero3<T>();
      kr0[c] = ivalid(c) ? KB[2 * r] : T(0);
      kr1[c] = ivalid(c) ? KB[2 * r + 1] : T(0);
      d1[c] = evalid(c) ? get3(D1, 3 * r) : zero3<T>();
    }
  }
  __device__ void load_twist(const T* TH, const T* OM) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      int r = v0 + gi(c);
      th[c] = evalid(c) ? TH[r] : T(0);
      om[c] = evalid(c) ? OM[r] : T(0);
    }
  }
  __device__ void store_twist(T* TH, T* OM) const {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      int g = gi(c), r = v0 + g;
      if (g < N) {
        TH[r] = th[c];   // zero on the last vertex row
        OM[r] = om[c];
      }
    }
  }

  __device__ void store_state(T* X, T* Vv, T* KB, T* D1) const {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      int g = gi(c), r = v0 + g;
      if (g < N) {
        put3(X, 3 * r, x[c]);
        put3(Vv, 3 * r, v[c]);
        KB[2 * r] = kr0[c];
        KB[2 * r + 1] = kr1[c];
        put3(D1, 3 * r, d1[c]);   // zero on the last vertex row
      }
    }
  }

  // tape layout of one rod block: value (field*C + c) of team lane l at
  // [(field*C + c) * TL + l] -- every access is a 64-lane contiguous run
  __device__ void store_tape(T* base) const {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      T vals[13] = {x[c].x, x[c].y, x[c].z, v[c].x, v[c].y, v[c].z,
                    kr0[c], kr1[c], d1[c].x, d1[c].y, d1[c].z, TW ? th[c] : T(0),
                    TW ? om[c] : T(0)};
#pragma unroll
      for (int f = 0; f < NFIELD; ++f) base[(f * C + c) * TL + tl] = vals[f];
    }
  }
  // the adjoint reads a stored state one substep ahead into registers
  // (prefetch), then installs it when that substep comes up
  __device__ void fetch_tape(const T* base, T (&buf)[NFIELD * C]) const {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int f = 0; f < NFIELD; ++f) buf[f * C + c] = base[(f * C + c) * TL + tl];
  }
  __device__ void install_tape(const T (&buf)[NFIELD * C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      x[c] = mk(buf[0 * C + c], buf[1 * C + c], buf[2 * C + c]);
      v[c] = mk(buf[3 * C + c], buf[4 * C + c], buf[5 * C + c]);
      kr0[c] = buf[6 * C + c];
      kr1[c] = buf[7 * C + c];
      d1[c] = mk(buf[8 * C + c], buf[9 * C + c], buf[10 * C + c]);
      if constexpr (TW) {
        th[c] = buf[11 * C + c];
        om[c] = buf[12 * C + c];
      }
    }
  }

  // grasp velocities of this lane's grasped vertices for action `act`
  __device__ void load_actions(const RodArgs<T>& a, int act, V3<T> (&ug)[C]) const {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      ug[c] = zero3<T>();
      if (gs[c] >= 0) ug[c] = get3(a.u, (int64_t)act * a.act_stride + (int64_t)(rod * a.G + gs[c]) * 3);
    }
  }

  // edge vectors at positions p: tangents, lengths and inverse lengths
  // (invalid edges: t = 0, l = 1/l = 1)
  __device__ void edges(Team<T, W>& X, const V3<T> (&p)[C], V3<T> (&t)[C], T (&l)[C],
                        T (&il)[C]) const {
    T pn[3] = {p[0].x, p[0].y, p[0].z};
    X.next(pn);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      V3<T> q = (c < C - 1) ? p[c + 1] : mk(pn[0], pn[1], pn[2]);
      V3<T> D = q - p[c];
      // explicit fused forms: every call site rounds identically, so the
      // forward's carried geometry equals a recomputation bit for bit
      T dd = fma(D.z, D.z, fma(D.y, D.y, D.x * D.x));
      T ii = frsq(dd);
      bool ok = evalid(c);
      l[c] = ok ? dd * ii : T(1);
      il[c] = ok ? ii : T(1);
      t[c] = ok ? ii * D : zero3<T>();
    }
  }

  // adjoint of edges(): adds the position adjoints to pb
  __device__ void edges_vjp(Team<T, W>& X, const V3<T> (&t)[C], const T (&il)[C],
                            const V3<T> (&tb)[C], const T (&lb)[C], V3<T> (&pb)[C]) const {
    V3<T> eb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      eb[c] = evalid(c) ? il[c] * (tb[c] - dot(t[c], tb[c]) * t[c]) + lb[c] * t[c]
                        : zero3<T>();
      pb[c] -= eb[c];
      if (c < C - 1) pb[c + 1] += eb[c];
    }
    T s[3] = {eb[C - 1].x, eb[C - 1].y, eb[C - 1].z};
    X.prev(s);
    pb[0] += mk(s[0], s[1], s[2]);
  }

  // projection tape: edge c of iteration it keeps (D, 1/|D|) as one
  // PROJ_TAPE-value record per lane, lanes contiguous
  __device__ __forceinline__ void tape_put(T* tape, int it, int c, V3<T> D, T il) const {
    Q4<T> q = {D.x, D.y, D.z, il};
    reinterpret_cast<Q4<T>*>(tape)[(it * C + c) * TL + tl] = q;
  }

  // N_C iterations of red (even edges) then black (odd edges) projections
  // of p = p0 + dl: the edge vectors of p0 are formed once, an iteration
  // adds the corrections' difference (more precise than differencing p)
  template <bool REC>
  __device__ void project(const RodArgs<T>& a, Team<T, W>& X, const V3<T> (&p0)[C],
                          V3<T> (&dl)[C], T* lds_tape) {
    const bool inext = (flags & FLAG_INEXT) != 0;
    V3<T> E0[C];
    {
      T pn[3] = {p0[0].x, p0[0].y, p0[0].z};
      X.next(pn);
#pragma unroll
      for (int c = 0; c < C; ++c)   // edges that are not projected get a unit dummy
        E0[c] = evalid(c) ? (c < C - 1 ? p0[c + 1] : mk(pn[0], pn[1], pn[2])) - p0[c]
                          : mk(T(1), T(0), T(0));
    }
    if constexpr (W > 1) {
      T ep[3] = {E0[C - 1].x, E0[C - 1].y, E0[C - 1].z};
      X.prev(ep);
      E0p = mk(ep[0], ep[1], ep[2]);
    }
    for (int it = 0; it < a.n_iters; ++it) {
      if (inext) project_iter<REC>(X, E0, dl, lds_tape, it);
      if constexpr (SC) {
        if (flags & FLAG_SELF) sc_pass<REC>(X, p0, dl, it, it == 0);
      }
    }
  }

  // one projection of edge c: D = E0 + (dl_k - dl_j); returns 1/|D|
  __device__ __forceinline__ T proj_edge(int c, const V3<T>& E0, V3<T>& dj, V3<T>& dk,
                                         V3<T>& D) const {
    D = E0 + (dk - dj);
    T il = frsq(dot(D, D));
    T s = T(1) - rest[c] * il;
    dj += (s * aj[c]) * D;
    dk -= (s * ak[c]) * D;
    return il;
  }

  template <bool REC>
  __device__ void project_iter(Team<T, W>& X, const V3<T> (&E0)[C], V3<T> (&dl)[C],
                               T* lds_tape, int it) {
    V3<T> D;
#pragma unroll
    for (int c = 0; c < C; c += 2) {   // red: even edges, inside the lane
      T il = proj_edge(c, E0[c], dl[c], dl[c + 1], D);
      if constexpr (REC) tape_put(lds_tape, it, c, D, il);
    }
#pragma unroll
    for (int c = 1; c < C - 1; c += 2) {   // black edges inside the lane
      T il = proj_edge(c, E0[c], dl[c], dl[c + 1], D);
      if constexpr (REC) tape_put(lds_tape, it, c, D, il);
    }
    // the lane's last (black) edge reaches into the next lane.  One wave:
    // project it here and send the next lane its endpoint's move.  Several
    // waves (a barrier per exchange): both lanes of the edge project it from
    // the same operands, after one exchange in both directions.
    if constexpr (W == 1) {
      T dn[3] = {dl[0].x, dl[0].y, dl[0].z};
      X.next(dn);
      D = E0[C - 1] + (mk(dn[0], dn[1], dn[2]) - dl[C - 1]);
      T il = frsq(dot(D, D));
      T sc = T(1) - rest[C - 1] * il;
      dl[C - 1] += (sc * aj[C - 1]) * D;
      if constexpr (REC) tape_put(lds_tape, it, C - 1, D, il);
      const T mk_ = -(sc * ak[C - 1]);
      T mv[3] = {mk_ * D.x, mk_ * D.y, mk_ * D.z};
      X.prev(mv);
      dl[0] += mk(mv[0], mv[1], mv[2]);
    } else {
      T up[3] = {dl[C - 1].x, dl[C - 1].y, dl[C - 1].z};
      T dn[3] = {dl[0].x, dl[0].y, dl[0].z};
      X.swap(up, dn);
      D = E0[C - 1] + (mk(dn[0], dn[1], dn[2]) - dl[C - 1]);
      const T il = frsq(dot(D, D));
      const T sc = T(1) - rest[C - 1] * il;
      const V3<T> Dp = E0p + (dl[0] - mk(up[0], up[1], up[2]));
      const T ilp = frsq(dot(Dp, Dp));
      const T scp = T(1) - restp * ilp;
      const T mk_ = -(scp * akp);
      const V3<T> mv = mk(mul_nc(mk_, Dp.x), mul_nc(mk_, Dp.y), mul_nc(mk_, Dp.z));
      dl[C - 1] += (sc * aj[C - 1]) * D;
      if constexpr (REC) tape_put(lds_tape, it, C - 1, D, il);
      if (tl > 0) dl[0] += mv;
    }
  }

  __device__ __forceinline__ void tape_load(const T* tape, int it, Q4<T> (&q)[C]) const {
#pragma unroll
    for (int c = 0; c < C; ++c) q[c] = reinterpret_cast<const Q4<T>*>(tape)[(it * C + c) * TL + tl];
  }

  // reverse sweep over the iterations.  Each iteration's tape records are
  // read one iteration ahead into alternating buffers (loop unrolled by
  // two, loads unconditional with a clamped index) so the LDS latency
  // overlaps the arithmetic.
  __device__ __forceinline__ void iter_vjp(Team<T, W>& X, V3<T> (&pb)[C], int it,
                                           const Q4<T> (&rec)[C]) {
    if constexpr (SC) {
      if (flags & FLAG_SELF) sc_pass_vjp(X, pb, it, it == 0);
    }
    if (flags & FLAG_INEXT) project_iter_vjp(X, pb, rec);
  }
  __device__ void project_vjp(const RodArgs<T>& a, Team<T, W>& X, V3<T> (&pb)[C],
                              const T* lds_tape) {
    int it = a.n_iters - 1;
    if (it < 0) return;
    Q4<T> A[C], B[C];
    tape_load(lds_tape, it, A);
    while (true) {
      tape_load(lds_tape, it > 0 ? it - 1 : 0, B);
      iter_vjp(X, pb, it, A);
      if (--it < 0) break;
      tape_load(lds_tape, it > 0 ? it - 1 : 0, A);
      iter_vjp(X, pb, it, B);
      if (--it < 0) break;
    }
  }

  __device__ void project_iter_vjp(Team<T, W>& X, V3<T> (&pb)[C], const Q4<T> (&rec)[C]) const {
    // the cross-lane black edge: its far endpoint's adjoint comes from the
    // next lane, the edge adjoint goes back to it (several waves: both
    // lanes evaluate it, after one exchange in both directions)
    const Q4<T>& q = rec[C - 1];
    if constexpr (W == 1) {
      T an[3] = {pb[0].x, pb[0].y, pb[0].z};
      X.next(an);
      V3<T> Db = project_edge_vjp(mk(q.x, q.y, q.z), q.w, aj[C - 1], ak[C - 1], rest[C - 1],
                                  pb[C - 1], mk(an[0], an[1], an[2]));
      pb[C - 1] -= Db;
      T s[3] = {Db.x, Db.y, Db.z};
      X.prev(s);
      pb[0] += mk(s[0], s[1], s[2]);
    } else {
      T up[7] = {pb[C - 1].x, pb[C - 1].y, pb[C - 1].z, q.x, q.y, q.z, q.w};
      T an[3] = {pb[0].x, pb[0].y, pb[0].z};
      X.swap(up, an);
      const V3<T> Db = project_edge_vjp(mk(q.x, q.y, q.z), q.w, aj[C - 1], ak[C - 1],
                                        rest[C - 1], pb[C - 1], mk(an[0], an[1], an[2]));
      const V3<T> Dbp = project_edge_vjp(mk(up[3], up[4], up[5]), up[6], ajp, akp, restp,
                                         mk(up[0], up[1], up[2]), pb[0]);
      pb[C - 1] -= Db;
      if (tl > 0) pb[0] += Dbp;
    }
#pragma unroll
    for (int c = 1; c < C - 1; c += 2) {   // black edges inside the lane
      V3<T> db = project_edge_vjp(mk(rec[c].x, rec[c].y, rec[c].z), rec[c].w, aj[c], ak[c],
                                  rest[c], pb[c], pb[c + 1]);
      pb[c] -= db;
      pb[c + 1] += db;
    }
#pragma unroll
    for (int c = 0; c < C; c += 2) {   // red
      V3<T> db = project_edge_vjp(mk(rec[c].x, rec[c].y, rec[c].z), rec[c].w, aj[c], ak[c],
                                  rest[c], pb[c], pb[c + 1]);
      pb[c] -= db;
      pb[c + 1] += db;
    }
  }

  // ------------------------------------------------------------ self-contact
  // The candidate pairs of a substep live in the rod's block of global pair
  // scratch (sized for every admissible pair: none is ever dropped), in one
  // compact list sorted by the lower edge.  Every sweep over the pairs deals
  // them round-robin to the team's lanes, so each pair is evaluated once and
  // the work is even across lanes; a pair's result goes to its records (one
  // half for each of its two edges), and each lane then gathers the records
  // of the pairs that touch its own edges in a fixed order (lower-edge pairs
  // in list order, then upper-edge pairs in upper-edge order), so every sum
  // is deterministic.
  //
  // LDS: staging (positions, velocities, adjoints), statics, per-vertex
  // counts of active pairs (this pass, first pass, adjoint's recorded
  // counts), the hash, per-edge list offsets, and the scan buffer.
  static constexpr int SC_TMP = 64;           // ints: scan and reduction slots
  // hash: groups of 27 buckets and the padded table (more groups where the
  // LDS has room: FP32 teams of 512 vertices and more)
  static constexpr int SC_G = sc_groups((int)sizeof(T), NV);
  static constexpr int SC_HT = sc_table((int)sizeof(T), NV, TL);
  // fixed part of the layout (the hash follows it, then the pair cache
  // reuses the hash's space and whatever more the launch allocates)
  static constexpr size_t sc_fixed_bytes() {
    return (sizeof(T) * (size_t)(11 * NV) + sizeof(float) * (size_t)NV +
            sizeof(int) * (size_t)(2 * NV + 4 * (NV + 4) + SC_TMP) + 15) / 16 * 16;
  }
  static constexpr size_t sc_bytes() {
    return sc_fixed_bytes() + sizeof(int) * (size_t)(SC_HT + (SC_HT + 4) + NV) + 64;
  }
  // rv: values of a pair's record (SC_RV_FWD in the forward kernels,
  // SC_RV_ADJ in the adjoint)
  __device__ void sc_layout(unsigned char* base, const RodArgs<T>& a, int rv, size_t xchg_off) {
    T* f = reinterpret_cast<T*>(base);
    sc_pos = f; f += 3 * NV;
    sc_aux = f; f += 3 * NV;
    sc_adj = f; f += 3 * NV;
    sc_w = f; f += NV;
    sc_r = f; f += NV;
    sc_vc = reinterpret_cast<float*>(f);
    int* q = reinterpret_cast<int*>(sc_vc + NV);
    sc_cnt = q; q += NV;
    sc_fcnt = q; q += NV;
    sc_lo = q; q += NV + 4;
    sc_hi = q; q += NV + 4;
    sc_slo = q; q += NV + 4;
    sc_shi = q; q += NV + 4;
    sc_tmp = q;
    sc_cache = base + sc_fixed_bytes();
    q = reinterpret_cast<int*>(sc_cache);
    sc_hcnt = q; q += SC_HT;
    sc_hstart = q; q += SC_HT + 4;
    sc_items = q;
    sc_cache_bytes = a.sc_lds - (int)(sc_cache - base) - (int)xchg_off;
    sc_rv = rv;
    sc_M = N - 2 - a.k_ex;
    const PairBlock pb = sc_block(N, a.k_ex, (int)sizeof(T), rv);
    unsigned char* g = a.pblk + a.pblk_off[rod];
    g_hdr = reinterpret_cast<int*>(g);
    g_trilo = reinterpret_cast<int*>(g + pb.trilo);
    g_sup = reinterpret_cast<SPair*>(g + pb.sup);
    g_suphi = reinterpret_cast<int*>(g + pb.suphi);
    g_cidx = reinterpret_cast<int*>(g + pb.cidx);
    g_pairs = gb_pairs = reinterpret_cast<SPair*>(g + pb.pairs);
    g_hpos = gb_hpos = reinterpret_cast<int*>(g + pb.hpos);
    g_d0 = gb_d0 = reinterpret_cast<T*>(g + pb.d0);
    g_d0b = gb_d0b = reinterpret_cast<T*>(g + pb.d0b);
    g_rec = gb_rec = reinterpret_cast<T*>(g + pb.rec);
    g_rec2 = reinterpret_cast<T*>(g + pb.rec2);
    sc_P = sc_S = 0;
    sc_built = false;
    st_act = st_fric = 0;
  }
  __device__ void sc_stats_out(const RodArgs<T>& a) const {
    if (!a.sc_stats) return;
    if (st_act) atomicAdd(a.sc_stats + 8 * rod + 3, (unsigned long long)st_act);
    if (st_fric) atomicAdd(a.sc_stats + 8 * rod + 4, (unsigned long long)st_fric);
  }
  __device__ void sc_stage(T* dst, const V3<T> (&vals)[C]) const {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      int g = gi(c);
      V3<T> q = vvalid(c) ? vals[c] : zero3<T>();
      dst[3 * g] = q.x;
      dst[3 * g + 1] = q.y;
      dst[3 * g + 2] = q.z;
    }
  }
  __device__ __forceinline__ V3<T> sc_at(const T* a, int v) const {
    return mk(a[3 * v], a[3 * v + 1], a[3 * v + 2]);
  }
  // static data into LDS; the hash cell is 2 r_max + delta_c + l where l is
  // the longest edge at the substep's predicted positions: a partner's
  // midpoint is within half of both edge lengths plus 2 r_max + delta_c of
  // the edge's own, so it lies in the 27 cells around the edge's cell
  __device__ void sc_setup(const RodArgs<T>& a) {
    sc_flags = 0;
    T m_r = T(0), m_l = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      int g = gi(c);
      sc_w[g] = w[c];
      sc_r[g] = rad[c];
      m_r = rad[c] > m_r ? rad[c] : m_r;
      m_l = rest[c] > m_l ? rest[c] : m_l;
    }
    // team maxima: wave maxima by lane shuffles, then the W wave values
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const T r2 = __shfl_xor(m_r, off, 64), l2 = __shfl_xor(m_l, off, 64);
      m_r = r2 > m_r ? r2 : m_r;
      m_l = l2 > m_l ? l2 : m_l;
    }
    T* red = reinterpret_cast<T*>(sc_tmp);
    if ((tl & 63) == 0) {
      red[2 * (tl >> 6)] = m_r;
      red[2 * (tl >> 6) + 1] = m_l;
    }
    __syncthreads();
    T rmax = T(0), lmax = T(0);
    for (int q = 0; q < W; ++q) {
      rmax = red[2 * q] > rmax ? red[2 * q] : rmax;
      lmax = red[2 * q + 1] > lmax ? red[2 * q + 1] : lmax;
    }
    sc_lmax = T(2) * lmax;
    sc_cell0 = T(2) * rmax + a.self_margin;
    __syncthreads();
  }

  // exclusive prefix sums over the team of two per-lane counts (lane order);
  // returns the totals.  Wave scan by lane shuffles, then the wave totals
  // through LDS.
  __device__ void sc_scan2(int a0, int a1, int& e0, int& e1, int& t0, int& t1) {
    const int lane = tl & 63, wave = tl >> 6;
    int i0 = a0, i1 = a1;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      int u0 = __shfl_up(i0, off, 64), u1 = __shfl_up(i1, off, 64);
      if (lane >= off) {
        i0 += u0;
        i1 += u1;
      }
    }
    if (lane == 63) {
      sc_tmp[2 * wave] = i0;
      sc_tmp[2 * wave + 1] = i1;
    }
    __syncthreads();
    int b0 = 0, b1 = 0;
    t0 = t1 = 0;
    for (int q = 0; q < W; ++q) {
      const int s0 = sc_tmp[2 * q], s1 = sc_tmp[2 * q + 1];
      if (q < wave) {
        b0 += s0;
        b1 += s1;
      }
      t0 += s0;
      t1 += s1;
    }
    e0 = b0 + i0 - a0;
    e1 = b1 + i1 - a1;
    __syncthreads();
  }

  // the exact candidate test of App. A.1's pairs (segment distance below
  // r_a + r_b + delta_c), lower edge first whichever edge asks
  __device__ __forceinline__ bool sc_near(int e, int j, T margin) const {
    const int lo = e < j ? e : j, hi = e < j ? j : e;
    V3<T> P1 = sc_at(sc_pos, lo), Q1 = sc_at(sc_pos, lo + 1);
    V3<T> P2 = sc_at(sc_pos, hi), Q2 = sc_at(sc_pos, hi + 1);
    Closest<T> cp = closest_params(P1, Q1, P2, Q2);
    V3<T> ca = (T(1) - cp.s) * P1 + cp.s * Q1;
    V3<T> cb = (T(1) - cp.u) * P2 + cp.u * Q2;
    V3<T> df = ca - cb;
    T ra = (T(1) - cp.s) * sc_r[lo] + cp.s * sc_r[lo + 1];
    T rb = (T(1) - cp.u) * sc_r[hi] + cp.u * sc_r[hi + 1];
    return fsqrt(dot(df, df)) < ra + rb + margin;
  }

  // Candidate pairs at the predicted positions p (App. A.1's pairs: segment
  // distance below r_a + r_b + delta_c, j - i > K_ex), by a neighbour list
  // with a skin: a superset of the pairs within delta_c + skin is built at
  // positions xb and kept while no vertex has moved by half the skin from
  // xb (a segment distance changes by at most the largest move of its two
  // segments' endpoints, so no pair outside the superset can be a
  // candidate); every substep tests each superset pair exactly.  The
  // superset is sorted by (lower, upper) edge, so the candidate list is the
  // same whenever the superset was built.
  // skin: half of 2 r_max + delta_c (a larger skin rebuilds less often and
  // filters a larger superset every substep; half measured fastest of a
  // quarter, a half and one on the 256 x 1024 helices)
  __device__ T sc_skin() const { return T(0.5) * sc_cell0; }
  __device__ void sc_broadphase(const RodArgs<T>& a, const V3<T> (&p)[C]) {
    sc_stage(sc_pos, p);
    T d2 = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (vvalid(c)) {
        const V3<T> d = p[c] - sc_xb[c];
        d2 = fmax(d2, dot(d, d));
      }
    }
    if (!sc_built) d2 = T(1e30);
    // team maximum of the moves (bits of a non-negative float, rounded up)
    int* mx = sc_tmp + 32;
    if (tl == 0) *mx = 0;
    __syncthreads();
    atomicMax(mx, __float_as_int((float)d2));
    __syncthreads();
    const T dmax = fsqrt((T)__int_as_float(*mx + 1));
    __syncthreads();
    const T skin = sc_skin();
    // slack of 1e-3 of the skin covers the rounding of the distance tests
    if (!(T(2) * dmax + T(1e-3) * skin < skin)) sc_build(a, p, skin);
    sc_filter(a);
  }

  // the superset at positions p: hash of edge midpoints (counting sort into
  // buckets, each sorted by edge), a search of the 27 cells around each
  // own edge for partners within delta_c + skin, their per-edge lists
  // sorted, the compact superset and its per-edge upper incidence
  __device__ void sc_build(const RodArgs<T>& a, const V3<T> (&p)[C], T skin) {
    sc_built = true;
    if (tl == 0 && a.sc_stats) atomicAdd(a.sc_stats + 8 * rod + 2, 1ull);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      sc_xb[c] = p[c];
      sc_cnt[gi(c)] = 0;   // counts of the pairs each edge is the upper edge of
      sc_slo[gi(c)] = 0;   // and the lower edge of
    }
    for (int i = tl; i < SC_HT; i += TL) sc_hcnt[i] = 0;
    int* lsq = sc_tmp;   // longest squared edge (bits of a non-negative real)
    int* ncand = sc_tmp + 48;   // pairs that pass the midpoint test
    if (tl == 0) {
      *lsq = 0;
      *ncand = 0;
    }
    __syncthreads();
    T l2 = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (evalid(c)) {
        V3<T> D = sc_at(sc_pos, gi(c) + 1) - sc_at(sc_pos, gi(c));
        l2 = fmax(l2, dot(D, D));
      }
    }
    atomicMax(lsq, __float_as_int((float)l2));
    __syncthreads();
    // the FP32 image of the longest edge, rounded up to the next float, is
    // an upper bound in either precision
    l2 = (T)__int_as_float(*lsq + 1);
    __syncthreads();   // sc_tmp is reused below
    if (l2 > sc_lmax * sc_lmax) sc_flags |= 4;
    const T cell0 = sc_cell0 + skin;
    // one part in 10^4 of slack keeps the 27-cell argument safe from rounding
    const T ig = frcp((cell0 + fsqrt(l2)) * T(1.0001));
    // edge midpoints (staged in sc_aux for the search) and their buckets
    int key[C], slot[C];
    V3<T> mid[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      key[c] = 0;
      slot[c] = 0;
      mid[c] = zero3<T>();
      if (evalid(c)) {
        const int e = gi(c);
        mid[c] = T(0.5) * (sc_at(sc_pos, e) + sc_at(sc_pos, e + 1));
        key[c] = sc_key<SC_G>(sc_cell(mid[c].x * ig), sc_cell(mid[c].y * ig),
                              sc_cell(mid[c].z * ig));
        slot[c] = atomicAdd(&sc_hcnt[key[c]], 1);
      }
    }
    __syncthreads();
    {
      constexpr int PER = SC_HT / TL;
      const int base = tl * PER;
      int sum = 0;
#pragma unroll
      for (int k = 0; k < PER; ++k) sum += sc_hcnt[base + k];
      int ex, dummy, tot, tot1;
      sc_scan2(sum, 0, ex, dummy, tot, tot1);
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        sc_hstart[base + k] = ex;
        ex += sc_hcnt[base + k];
      }
      if (tl == TL - 1) sc_hstart[SC_HT] = ex;
      __syncthreads();
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (evalid(c)) sc_items[sc_hstart[key[c]] + slot[c]] = gi(c);
      __syncthreads();
      // the fill order above is that of the atomics: sort every bucket
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int s0 = sc_hstart[base + k], s1 = sc_hstart[base + k + 1];
        for (int i = s0 + 1; i < s1; ++i) {
          const int v = sc_items[i];
          int j = i - 1;
          while (j >= s0 && sc_items[j] > v) {
            sc_items[j + 1] = sc_items[j];
            --j;
          }
          sc_items[j + 1] = v;
        }
        // the midpoints in the same order (sc_aux), so a search reads an
        // item's edge and midpoint independently
        for (int i = s0; i < s1; ++i) {
          const int j = sc_items[i];
          const V3<T> mj = T(0.5) * (sc_at(sc_pos, j) + sc_at(sc_pos, j + 1));
          sc_aux[3 * i] = mj.x;
          sc_aux[3 * i + 1] = mj.y;
          sc_aux[3 * i + 2] = mj.z;
        }
      }
      __syncthreads();
    }
    const T margin = a.self_margin + skin;
    // A partner's midpoint is within h_e + h_max + 2 r_max + margin of the
    // edge's own (segment distance >= midpoint distance minus both
    // half-lengths); the slack keeps every pair the exact test accepts.
    // Each edge looks for partners above it only (j - e > K_ex), so every
    // pair is met once, by its lower edge.  The search only lists the pairs
    // that pass the midpoint test (LDS past the hash, then the rod's cidx
    // block, which is free until the filter); the exact tests then run
    // round-robin over that list, so no lane waits on another's.
    const T h_max = T(0.5) * fsqrt(l2);
    const int64_t M = sc_M;
    int* cand = sc_items + NV;
    const int capc = sc_cache_bytes / (int)sizeof(int) - (2 * SC_HT + 4 + NV) > 0
                         ? sc_cache_bytes / (int)sizeof(int) - (2 * SC_HT + 4 + NV)
                         : 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int e = gi(c);
      const int jmin = e + a.k_ex + 1;
      // every lane runs the loops (no early exit) so the wave's slot
      // allocations see all its lanes; lanes without work find nothing
      const bool act = evalid(c) && jmin < N - 1;
      const V3<T> m = mid[c];
      const V3<T> PQ = act ? sc_at(sc_pos, e + 1) - sc_at(sc_pos, e) : zero3<T>();
      const T reach = (T(0.5) * fsqrt(dot(PQ, PQ)) + h_max + cell0) * T(1.0001) + T(1e-6);
      const T reach2 = act ? reach * reach : T(-1);
      // the 27 cells around the edge's cell: block coordinates, residues and
      // hash terms per axis, so a cell's bucket takes a few operations
      int rx[3], ry[3], rz[3];
      unsigned hx[3], hy[3], hz[3];
      {
        const int cc[3] = {sc_cell(m.x * ig), sc_cell(m.y * ig), sc_cell(m.z * ig)};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int bx = floor_div3(cc[0] + k - 1), by = floor_div3(cc[1] + k - 1),
                    bz = floor_div3(cc[2] + k - 1);
          rx[k] = cc[0] + k - 1 - 3 * bx;
          ry[k] = 3 * (cc[1] + k - 1 - 3 * by);
          rz[k] = 9 * (cc[2] + k - 1 - 3 * bz);
          hx[k] = (unsigned)bx * SC_H1;
          hy[k] = (unsigned)by * SC_H2;
          hz[k] = (unsigned)bz * SC_H3;
        }
      }
      // two items per round: their loads are independent (edge and midpoint
      // of a bucket slot), the second clamped into the bucket
#pragma unroll 1
      for (int d = 0; d < 27; ++d) {
        const int ix = d % 3, iy = (d / 3) % 3, iz = d / 9;
        const int kk = (int)((hx[ix] ^ hy[iy] ^ hz[iz]) & (unsigned)(SC_G - 1)) * 27 + rx[ix] +
                       ry[iy] + rz[iz];
        const int q1 = act ? sc_hstart[kk + 1] : 0;
        for (int q = act ? sc_hstart[kk] : 0; q < q1; q += 2) {
          const int qb = q + 1 < q1 ? q + 1 : q;
          const int ja = sc_items[q], jb = sc_items[qb];
          const V3<T> ma = sc_at(sc_aux, q) - m, mb = sc_at(sc_aux, qb) - m;
          const bool pa = ja >= jmin && dot(ma, ma) < reach2;
          const bool pb = q + 1 < q1 && jb >= jmin && dot(mb, mb) < reach2;
          const int sa = wave_alloc(ncand, pa), sb = wave_alloc(ncand, pb);
          if (pa) {
            if (sa < capc) cand[sa] = (e << 16) | ja; else g_cidx[sa] = (e << 16) | ja;
          }
          if (pb) {
            if (sb < capc) cand[sb] = (e << 16) | jb; else g_cidx[sb] = (e << 16) | jb;
          }
        }
      }
    }
    __syncthreads();
    {
      const int nc = *ncand;
      for (int k = tl; k < nc; k += TL) {
        const int v = k < capc ? cand[k] : g_cidx[k];
        const int e = v >> 16, j = v & 0xffff;
        if (!sc_near(e, j, margin)) continue;
        const int slot = atomicAdd(&sc_slo[e], 1);
        if (slot < M - e) g_trilo[sc_off_lo(e, M) + slot] = j; else sc_flags |= 2;
        atomicAdd(&sc_cnt[j], 1);
      }
    }
    __syncthreads();
    // each lane's lower lists: in increasing order (their fill order is that
    // of the atomics); counts of both kinds
    int nlo[C], nhi[C], slo = 0, shi = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int e = gi(c);
      nlo[c] = evalid(c) ? sc_slo[e] : 0;
      nhi[c] = sc_cnt[e];
      sc_cnt[e] = 0;   // fill counters of the upper-edge lists
      slo += nlo[c];
      shi += nhi[c];
      int* lo_out = g_trilo + sc_off_lo(e, M);
      for (int i = 1; i < nlo[c]; ++i) {
        const int v = lo_out[i];
        int j = i - 1;
        while (j >= 0 && lo_out[j] > v) {
          lo_out[j + 1] = lo_out[j];
          --j;
        }
        lo_out[j + 1] = v;
      }
    }
    int elo, ehi, tlo, thi;
    sc_scan2(slo, shi, elo, ehi, tlo, thi);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      sc_slo[gi(c)] = elo;
      sc_shi[gi(c)] = ehi;
      elo += nlo[c];
      ehi += nhi[c];
    }
    if (tl == 0) {
      sc_slo[NV] = tlo;
      sc_shi[NV] = thi;
    }
    if (tlo != thi) sc_flags |= 2;   // every pair has one lower and one upper edge
    sc_S = tlo;
    __syncthreads();
    // compact superset; each pair also takes a place in its upper edge's list
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (!evalid(c)) continue;
      const int e = gi(c);
      const int* lo_in = g_trilo + sc_off_lo(e, M);
      const int b0 = sc_slo[e];
      for (int q = 0; q < nlo[c]; ++q) {
        const int j = lo_in[q];
        g_sup[b0 + q] = SPair{(short)e, (short)j};
        const int at = atomicAdd(&sc_cnt[j], 1);
        if (at < sc_shi[j + 1] - sc_shi[j]) g_suphi[sc_shi[j] + at] = b0 + q;
        else sc_flags |= 2;
      }
    }
    __syncthreads();
    // the fill order of the upper-edge lists is that of the atomics: sort
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (!evalid(c)) continue;
      const int e = gi(c);
      if (sc_cnt[e] != nhi[c]) sc_flags |= 2;
      int* L = g_suphi + sc_shi[e];
      for (int i = 1; i < nhi[c]; ++i) {
        const int v = L[i];
        int j = i - 1;
        while (j >= 0 && L[j] > v) {
          L[j + 1] = L[j];
          --j;
        }
        L[j + 1] = v;
      }
    }
    __syncthreads();
  }

  // this substep's candidates: every superset pair tested exactly at the
  // staged positions, each lane a contiguous run of the superset, so the
  // compact list keeps the superset's order; then per edge the offsets of
  // its lower-edge run and its upper-edge list (indices, in order)
  __device__ void sc_filter(const RodArgs<T>& a) {
    const int run = (sc_S + TL - 1) / TL;
    const int s0 = tl * run < sc_S ? tl * run : sc_S;
    const int s1 = s0 + run < sc_S ? s0 + run : sc_S;
    int n = 0;
    for (int s = s0; s < s1; ++s) {
      const SPair pr = g_sup[s];
      const bool ok = sc_near(pr.lo, pr.hi, a.self_margin);
      g_cidx[s] = ok ? 1 : -1;
      n += ok ? 1 : 0;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      sc_lo[gi(c)] = 0;   // per-edge counts, then offsets
      sc_hi[gi(c)] = 0;
    }
    int base, dummy, tot, tot1;
    sc_scan2(n, 0, base, dummy, tot, tot1);
    // the substep's pair arrays go to LDS when they fit (the forward
    // kernels need no depth adjoints)
    const bool adj = sc_rv == SC_RV_ADJ;
    const int per = (int)(sizeof(SPair) + sizeof(int) + ((adj ? 2 : 1) + sc_rv) * sizeof(T));
    if (tot <= (sc_cache_bytes - (int)sizeof(T)) / per) {
      unsigned char* c = sc_cache;
      g_pairs = reinterpret_cast<SPair*>(c); c += sizeof(SPair) * tot;
      g_hpos = reinterpret_cast<int*>(c); c += sizeof(int) * tot;
      c = sc_cache + (c - sc_cache + sizeof(T) - 1) / sizeof(T) * sizeof(T);
      g_d0 = reinterpret_cast<T*>(c); c += sizeof(T) * tot;
      if (adj) {
        g_d0b = reinterpret_cast<T*>(c);
        c += sizeof(T) * tot;
      }
      g_rec = reinterpret_cast<T*>(c);
    } else {
      g_pairs = gb_pairs;
      g_hpos = gb_hpos;
      g_d0 = gb_d0;
      g_d0b = gb_d0b;
      g_rec = gb_rec;
    }
    for (int s = s0; s < s1; ++s) {
      if (g_cidx[s] < 0) continue;
      const SPair pr = g_sup[s];
      g_pairs[base] = pr;
      gb_pairs[base] = pr;   // kept in global memory for rods_sc_pairs
      g_cidx[s] = base++;
      atomicAdd(&sc_lo[pr.lo], 1);
      atomicAdd(&sc_hi[pr.hi], 1);
    }
    sc_P = tot;
    if (tl == 0) {
      g_hdr[0] = tot;
      if (a.sc_stats) {
        atomicAdd(a.sc_stats + 8 * rod, (unsigned long long)tot);
        atomicAdd(a.sc_stats + 8 * rod + 1, (unsigned long long)sc_S);
      }
    }
    __syncthreads();
    int nlo[C], nhi[C], slo = 0, shi = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      nlo[c] = sc_lo[gi(c)];
      nhi[c] = sc_hi[gi(c)];
      slo += nlo[c];
      shi += nhi[c];
    }
    int elo, ehi, tlo, thi;
    sc_scan2(slo, shi, elo, ehi, tlo, thi);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      sc_lo[gi(c)] = elo;
      sc_hi[gi(c)] = ehi;
      elo += nlo[c];
      ehi += nhi[c];
    }
    if (tl == 0) {
      sc_lo[NV] = tlo;
      sc_hi[NV] = thi;
    }
    // upper-edge lists: the superset's, filtered (the order carries over)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (!evalid(c)) continue;
      const int e = gi(c);
      int o = sc_hi[e];
      const int q1 = sc_shi[e + 1];
      for (int q = sc_shi[e]; q < q1; ++q) {
        const int k = g_cidx[g_suphi[q]];
        if (k >= 0) g_hpos[k] = o++;
      }
      if (o != sc_hi[e] + nhi[c]) sc_flags |= 2;
    }
    __syncthreads();
  }

  __device__ __forceinline__ PairGeo<T> sc_pair(const T* P, int lo, int hi) const {
    return pair_geo(sc_at(P, lo), sc_at(P, lo + 1), sc_at(P, hi), sc_at(P, hi + 1), sc_w[lo],
                    sc_w[lo + 1], sc_w[hi], sc_w[hi + 1], sc_r[lo], sc_r[lo + 1], sc_r[hi],
                    sc_r[hi + 1]);
  }
  // per-pair divisor of the Jacobi passes: the largest number of counted
  // pairs touching one of the pair's four vertices (at least 1)
  template <typename Q>
  __device__ __forceinline__ T sc_divisor(const Q* cnt, int lo, int hi) const {
    const Q a0 = cnt[lo] > cnt[lo + 1] ? cnt[lo] : cnt[lo + 1];
    const Q a1 = cnt[hi] > cnt[hi + 1] ? cnt[hi] : cnt[hi + 1];
    const T m = (T)(a0 > a1 ? a0 : a1);
    return m > T(1) ? m : T(1);
  }
  // Per-pair records: the lower edge's half (sc_rv / 2 values) at the
  // pair's place k in the list, the upper edge's half at its place in
  // upper-edge order (g_hpos[k]) after all lower halves; rec2 likewise.
  // Each own edge then sums its lower-edge run and its upper-edge run of
  // records, both contiguous, in a fixed order.
  __device__ __forceinline__ T* sc_rlo(T* base, int k) const {
    return base + (int64_t)k * (sc_rv / 2);
  }
  __device__ __forceinline__ T* sc_rhi(T* base, int k) const {
    return base + ((int64_t)sc_P + g_hpos[k]) * (sc_rv / 2);
  }
  // forward records (k n or dv_t, the edge's parameter s or u, reciprocal
  // divisor): the corrections of own edge e's two vertices, summed
  __device__ __forceinline__ void sc_gather_fwd(int e, V3<T>& dA, V3<T>& dB) const {
    dA = dB = zero3<T>();
    const T wa = sc_w[e], wb = sc_w[e + 1];
    const int RL = sc_rv / 2;   // 5 in the forward kernels, 6 in the adjoint's replay
    const int k1 = sc_lo[e + 1];
    for (int k = sc_lo[e]; k < k1; ++k) {
      const T* r = g_rec + (int64_t)k * RL;
      const V3<T> kn = mk(r[0], r[1], r[2]);
      const T s = r[3], im = r[4];
      dA += (wa * (T(1) - s) * im) * kn;
      dB += (wb * s * im) * kn;
    }
    const T* rh = g_rec + (int64_t)sc_P * RL;
    const int q1 = sc_hi[e + 1];
    for (int q = sc_hi[e]; q < q1; ++q) {
      const T* r = rh + (int64_t)q * RL;
      const V3<T> kn = mk(r[0], r[1], r[2]);
      const T u = r[3], im = r[4];
      dA -= (wa * (T(1) - u) * im) * kn;
      dB -= (wb * u * im) * kn;
    }
  }
  // adjoint records (the two vertex adjoints of the edge; the adjoint
  // kernel's halves are 6 values) from rec or rec2: the sums for own edge
  // e's two vertices
  __device__ __forceinline__ void sc_gather_adj(int e, const T* base, V3<T>& gA,
                                                V3<T>& gB) const {
    gA = gB = zero3<T>();
    const int k1 = sc_lo[e + 1];
    for (int k = sc_lo[e]; k < k1; ++k) {
      const T* r = base + (int64_t)k * 6;
      gA += get3(r, 0);
      gB += get3(r, 3);
    }
    const T* rh = base + (int64_t)sc_P * 6;
    const int q1 = sc_hi[e + 1];
    for (int q = sc_hi[e]; q < q1; ++q) {
      const T* r = rh + (int64_t)q * 6;
      gA += get3(r, 0);
      gB += get3(r, 3);
    }
  }

  // one Jacobi pass of the self-contact projection: a sweep over the pairs
  // evaluates each once (activity, depth, direction) and counts the active
  // pairs per vertex; a second sweep adds each pair's reciprocal divisor;
  // each lane then sums the corrections of the pairs touching its edges.
  // The first pass keeps the depths d0 and the counts for friction.
  template <bool REC>
  __device__ void sc_pass(Team<T, W>& X, const V3<T> (&p0)[C], V3<T> (&dl)[C], int it,
                          bool first) {
    V3<T> p[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      p[c] = p0[c] + dl[c];
      sc_cnt[gi(c)] = 0;
    }
    sc_stage(sc_pos, p);
    __syncthreads();
    // sweep 1: k n (n the unit direction, k = d / W), s, u
    for (int k = tl; k < sc_P; k += TL) {
      const SPair pr = g_pairs[k];
      PairGeo<T> g = sc_pair(sc_pos, pr.lo, pr.hi);
      if (first) g_d0[k] = g.act ? g.d : T(0);
      const T kk = g.act ? fdiv(g.d, g.W) : T(0);
      const V3<T> kn = kk * g.n;
      T* rl = sc_rlo(g_rec, k);
      T* rh = sc_rhi(g_rec, k);
      put3(rl, 0, kn);
      rl[3] = g.cp.s;
      put3(rh, 0, kn);
      rh[3] = g.cp.u;
      if (g.act) {
        ++st_act;
        atomicAdd(&sc_cnt[pr.lo], 1);
        atomicAdd(&sc_cnt[pr.lo + 1], 1);
        atomicAdd(&sc_cnt[pr.hi], 1);
        atomicAdd(&sc_cnt[pr.hi + 1], 1);
      }
    }
    __syncthreads();
    // sweep 2: the pair's divisor, from the completed counts
    for (int k = tl; k < sc_P; k += TL) {
      const SPair pr = g_pairs[k];
      const T im = frcp(sc_divisor(sc_cnt, pr.lo, pr.hi));
      sc_rlo(g_rec, k)[4] = im;
      sc_rhi(g_rec, k)[4] = im;
    }
    if (first) {
#pragma unroll
      for (int c = 0; c < C; ++c) sc_fcnt[gi(c)] = sc_cnt[gi(c)];
    }
    if constexpr (REC) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        Q4<T> q = {p[c].x, p[c].y, p[c].z, (T)sc_cnt[gi(c)]};
        reinterpret_cast<Q4<T>*>(ctape)[(it * C + c) * TL + tl] = q;
      }
    }
    __syncthreads();
    V3<T> dA[C], dB[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      dA[c] = dB[c] = zero3<T>();
      if (evalid(c)) sc_gather_fwd(gi(c), dA[c], dB[c]);
    }
    __syncthreads();
    T s3[3] = {dB[C - 1].x, dB[C - 1].y, dB[C - 1].z};
    X.prev(s3);
#pragma unroll
    for (int c = 0; c < C; ++c) dl[c] += dA[c] + (c ? dB[c - 1] : mk(s3[0], s3[1], s3[2]));
  }

  // self-friction on velocities v at final positions x1, for the pairs with
  // a positive first-pass depth; divisors from the first pass's counts
  __device__ void sc_friction(const RodArgs<T>& a, Team<T, W>& X, const V3<T> (&x1)[C],
                              V3<T> (&v)[C]) {
    sc_stage(sc_pos, x1);
    sc_stage(sc_aux, v);
    __syncthreads();
    for (int k = tl; k < sc_P; k += TL) {
      const T d0 = g_d0[k];
      const SPair pr = g_pairs[k];
      const int lo = pr.lo, hi = pr.hi;
      V3<T> dvt = zero3<T>();
      T s = T(0), u = T(0), iW = T(0);
      if (d0 > T(0)) {
        FricGeo<T> f = pair_friction(sc_at(sc_pos, lo), sc_at(sc_pos, lo + 1), sc_at(sc_pos, hi),
                                     sc_at(sc_pos, hi + 1), sc_at(sc_aux, lo),
                                     sc_at(sc_aux, lo + 1), sc_at(sc_aux, hi),
                                     sc_at(sc_aux, hi + 1), sc_w[lo], sc_w[lo + 1], sc_w[hi],
                                     sc_w[hi + 1], sc_r[lo], sc_r[lo + 1], sc_r[hi],
                                     sc_r[hi + 1], d0, mu, a.h);
        if (f.ok) {
          ++st_fric;
          dvt = f.dvt;
          s = f.g.cp.s;
          u = f.g.cp.u;
          iW = frcp(f.g.W * sc_divisor(sc_fcnt, lo, hi));
        }
      }
      T* rl = sc_rlo(g_rec, k);
      T* rh = sc_rhi(g_rec, k);
      put3(rl, 0, dvt);
      rl[3] = s;
      rl[4] = iW;
      put3(rh, 0, dvt);
      rh[3] = u;
      rh[4] = iW;
    }
    __syncthreads();
    V3<T> dA[C], dB[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      dA[c] = dB[c] = zero3<T>();
      if (evalid(c)) sc_gather_fwd(gi(c), dA[c], dB[c]);
    }
    __syncthreads();
    T s3[3] = {dB[C - 1].x, dB[C - 1].y, dB[C - 1].z};
    X.prev(s3);
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] += dA[c] + (c ? dB[c - 1] : mk(s3[0], s3[1], s3[2]));
  }

  // adjoint of sc_friction: lv (adjoint of friction's output velocity) ->
  // adjoint of its input velocity; adds position adjoints to xb; leaves the
  // adjoint of each pair's first-pass depth in g_d0b.  The velocity
  // adjoints of a pair go to its record, the position adjoints to rec2.
  __device__ void sc_friction_vjp(const RodArgs<T>& a, Team<T, W>& X, const Rec<T, C>& r,
                                  V3<T> (&lv)[C], V3<T> (&xb)[C]) {
    sc_stage(sc_pos, r.x1);
    sc_stage(sc_aux, r.v3);
    sc_stage(sc_adj, lv);
    __syncthreads();
    for (int k = tl; k < sc_P; k += TL) {
      const T d0 = g_d0[k];
      const SPair pr = g_pairs[k];
      const int lo = pr.lo, hi = pr.hi;
      T d0b = T(0);
      V3<T> b0 = zero3<T>(), b1 = zero3<T>(), b2 = zero3<T>(), b3 = zero3<T>();
      V3<T> q0 = zero3<T>(), q1 = zero3<T>(), q2 = zero3<T>(), q3 = zero3<T>();
      if (d0 > T(0)) {
        V3<T> P1 = sc_at(sc_pos, lo), Q1 = sc_at(sc_pos, lo + 1);
        V3<T> P2 = sc_at(sc_pos, hi), Q2 = sc_at(sc_pos, hi + 1);
        V3<T> vi = sc_at(sc_aux, lo), vi1 = sc_at(sc_aux, lo + 1);
        V3<T> vj = sc_at(sc_aux, hi), vj1 = sc_at(sc_aux, hi + 1);
        FricGeo<T> f = pair_friction(P1, Q1, P2, Q2, vi, vi1, vj, vj1, sc_w[lo], sc_w[lo + 1],
                                     sc_w[hi], sc_w[hi + 1], sc_r[lo], sc_r[lo + 1], sc_r[hi],
                                     sc_r[hi + 1], d0, mu, a.h);
        if (f.ok) {
          const T im = frcp(sc_divisor(sc_fcnt, lo, hi));
          d0b = pair_friction_vjp(P1, Q1, P2, Q2, vi, vi1, vj, vj1, f, sc_w[lo], sc_w[lo + 1],
                                  sc_w[hi], sc_w[hi + 1], mu, a.h, im * sc_at(sc_adj, lo),
                                  im * sc_at(sc_adj, lo + 1), im * sc_at(sc_adj, hi),
                                  im * sc_at(sc_adj, hi + 1), b0, b1, b2, b3, q0, q1, q2, q3);
        }
      }
      g_d0b[k] = d0b;
      T* ol = sc_rlo(g_rec, k);
      T* oh = sc_rhi(g_rec, k);
      put3(ol, 0, b0); put3(ol, 3, b1); put3(oh, 0, b2); put3(oh, 3, b3);
      ol = sc_rlo(g_rec2, k);
      oh = sc_rhi(g_rec2, k);
      put3(ol, 0, q0); put3(ol, 3, q1); put3(oh, 0, q2); put3(oh, 3, q3);
    }
    __syncthreads();
    V3<T> vA[C], vB[C], xA[C], xB[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      vA[c] = vB[c] = xA[c] = xB[c] = zero3<T>();
      if (!evalid(c)) continue;
      sc_gather_adj(gi(c), g_rec, vA[c], vB[c]);
      sc_gather_adj(gi(c), g_rec2, xA[c], xB[c]);
    }
    __syncthreads();
    T s6[6] = {vB[C - 1].x, vB[C - 1].y, vB[C - 1].z, xB[C - 1].x, xB[C - 1].y, xB[C - 1].z};
    X.prev(s6);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      lv[c] += vA[c] + (c ? vB[c - 1] : mk(s6[0], s6[1], s6[2]));
      xb[c] += xA[c] + (c ? xB[c - 1] : mk(s6[3], s6[4], s6[5]));
    }
  }

  // adjoint of the contact pass of iteration it (inputs and counts read
  // back from ctape); at it == 0 also the adjoint of the first-pass depths
  // left in g_d0b
  __device__ void sc_pass_vjp(Team<T, W>& X, V3<T> (&pb)[C], int it, bool with_depth) {
    V3<T> pin[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      Q4<T> q = reinterpret_cast<const Q4<T>*>(ctape)[(it * C + c) * TL + tl];
      pin[c] = mk(q.x, q.y, q.z);
      sc_vc[gi(c)] = (float)q.w;
    }
    sc_stage(sc_pos, pin);
    sc_stage(sc_adj, pb);
    __syncthreads();
    for (int k = tl; k < sc_P; k += TL) {
      const SPair pr = g_pairs[k];
      const int lo = pr.lo, hi = pr.hi;
      PairGeo<T> g = sc_pair(sc_pos, lo, hi);
      V3<T> b0 = zero3<T>(), b1 = zero3<T>(), b2 = zero3<T>(), b3 = zero3<T>();
      if (g.act) {
        V3<T> P1 = sc_at(sc_pos, lo), Q1 = sc_at(sc_pos, lo + 1);
        V3<T> P2 = sc_at(sc_pos, hi), Q2 = sc_at(sc_pos, hi + 1);
        const T im = frcp(sc_divisor(sc_vc, lo, hi));
        pair_proj_vjp(P1, Q1, P2, Q2, g, sc_w[lo], sc_w[lo + 1], sc_w[hi], sc_w[hi + 1],
                      sc_r[lo], sc_r[lo + 1], sc_r[hi], sc_r[hi + 1], im * sc_at(sc_adj, lo),
                      im * sc_at(sc_adj, lo + 1), im * sc_at(sc_adj, hi),
                      im * sc_at(sc_adj, hi + 1), b0, b1, b2, b3);
        if (with_depth) {
          const T d0b = g_d0b[k];
          if (d0b != T(0))
            pair_depth_vjp(P1, Q1, P2, Q2, g, sc_r[lo], sc_r[lo + 1], sc_r[hi], sc_r[hi + 1],
                           d0b, b0, b1, b2, b3);
        }
      }
      T* ol = sc_rlo(g_rec, k);
      T* oh = sc_rhi(g_rec, k);
      put3(ol, 0, b0); put3(ol, 3, b1); put3(oh, 0, b2); put3(oh, 3, b3);
    }
    __syncthreads();
    V3<T> cA[C], cB[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      cA[c] = cB[c] = zero3<T>();
      if (evalid(c)) sc_gather_adj(gi(c), g_rec, cA[c], cB[c]);
    }
    __syncthreads();
    T s3[3] = {cB[C - 1].x, cB[C - 1].y, cB[C - 1].z};
    X.prev(s3);
#pragma unroll
    for (int c = 0; c < C; ++c) pb[c] += cA[c] + (c ? cB[c - 1] : mk(s3[0], s3[1], s3[2]));
  }

  // gather the previous lane's last edge: tangent, inverse length, d1
  __device__ void prev_edge(Team<T, W>& X, const V3<T> (&t)[C], const T (&il)[C],
                            const V3<T> (&dd)[C], V3<T>& tp, T& ilp, V3<T>& dp) const {
    T pv[7] = {t[C - 1].x, t[C - 1].y, t[C - 1].z, il[C - 1], dd[C - 1].x, dd[C - 1].y,
               dd[C - 1].z};
    X.prev(pv);
    tp = mk(pv[0], pv[1], pv[2]);
    ilp = pv[3];
    dp = mk(pv[4], pv[5], pv[6]);
  }

  // twist: the previous lane's last edge with its material and reference
  // d1 and its angle
  __device__ void prev_edge_tw(Team<T, W>& X, const V3<T> (&t)[C], const T (&il)[C],
                               const V3<T> (&m1)[C], const V3<T> (&dd)[C], const T (&ang)[C],
                               V3<T>& tp, T& ilp, V3<T>& m1p, V3<T>& dp, T& angp) const {
    T pv[11] = {t[C - 1].x,  t[C - 1].y,  t[C - 1].z,  il[C - 1], m1[C - 1].x, m1[C - 1].y,
                m1[C - 1].z, dd[C - 1].x, dd[C - 1].y, dd[C - 1].z, ang[C - 1]};
    X.prev(pv);
    tp = mk(pv[0], pv[1], pv[2]);
    ilp = pv[3];
    m1p = mk(pv[4], pv[5], pv[6]);
    dp = mk(pv[7], pv[8], pv[9]);
    angp = pv[10];
  }

  // kr0/kr1: the rest curvature at the substep start (the adjoint passes the
  // recorded values: the replayed substep has already updated the registers)
  __device__ __forceinline__ BendIn<T> bend_in(int c, const V3<T> (&t)[C], const T (&il)[C],
                                               const V3<T> (&dd1)[C], V3<T> tp, T ilp,
                                               V3<T> d1p, const T (&k0)[C],
                                               const T (&k1)[C]) const {
    BendIn<T> q;
    q.t0 = c ? t[c - 1] : tp;
    q.t1 = t[c];
    q.il0 = c ? il[c - 1] : ilp;
    q.il1 = il[c];
    q.d1a = c ? dd1[c - 1] : d1p;
    q.d1b = dd1[c];
    q.d2a = cross(q.t0, q.d1a);
    q.d2b = cross(q.t1, q.d1b);
    q.kr0 = k0[c];
    q.kr1 = k1[c];
    q.coef = coef[c];
    q.ilbar = ilbar[c];
    return q;
  }

  // ---------------------------------------------------------------- substep
  template <bool REC>
  __device__ void substep(const RodArgs<T>& a, Team<T, W>& X, const V3<T> (&ug)[C],
                          Rec<T, C>* rc_, T* lds_tape) {
    const T h = a.h;
    const T ih = T(1) / h;
    const V3<T> g = mk(a.gx, a.gy, a.gz);
    // discrete decisions of this substep, for the optional branch log
    uint32_t bits[C];
#pragma unroll
    for (int c = 0; c < C; ++c) bits[c] = 0u;
    // S2 forces at x with frames fixed
    V3<T> t[C];
    T l[C], il[C];
    V3<T> tp, d1p;
    T ilp;
    if (!REC && geo_ok) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        t[c] = tc[c];
        l[c] = lc[c];
        il[c] = ilc[c];
      }
    } else {
      edges(X, x, t, l, il);
    }
    // twist: material directors m1 (bending sees them in place of d1)
    V3<T> m1[C], m1p;
    T thp = T(0), Tq[C], tq_prev = T(0);
    if constexpr (TW) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        m1[c] = material_m1(t[c], d1[c], th[c]);
        Tq[c] = T(0);
      }
      prev_edge_tw(X, t, il, m1, d1, th, tp, ilp, m1p, d1p, thp);
    } else if (!REC && prev_ok) {
      tp = tpc;
      ilp = ilpc;
      d1p = d1pc;
    } else {
      prev_edge(X, t, il, d1, tp, ilp, d1p);
    }
    V3<T> F[C];
#pragma unroll
    for (int c = 0; c < C; ++c) F[c] = zero3<T>();
    V3<T> to_prev = zero3<T>(), to_next = zero3<T>();
    // every vertex runs the stencil: away from interior vertices coef = 0
    // makes both gradients exactly zero (all inputs are finite there)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      BendIn<T> q = TW ? bend_in(c, t, il, m1, tp, ilp, m1p, kr0, kr1)
                       : bend_in(c, t, il, d1, tp, ilp, d1p, kr0, kr1);
      V3<T> g0, g1;
      bend_grad(q, g0, g1);
      if constexpr (TW) {
        TwIn<T> tq{q.t0,  q.t1,  q.d1a, q.d1b, c ? d1[c - 1] : d1p, d1[c], q.il0,
                   q.il1, c ? th[c - 1] : thp, th[c], q.kr0, q.kr1, q.coef, q.ilbar,
                   tcoef[c]};
        T Ta, Tb;
        twist_grad(tq, g0, g1, Ta, Tb);
        Tq[c] += Tb;
        if (c > 0) Tq[c - 1] += Ta; else tq_prev += Ta;
      }
      F[c] += g1 - g0;
      if (c > 0) F[c - 1] += g0; else to_prev += g0;
      if (c < C - 1) F[c + 1] -= g1; else to_next -= g1;
    }
    if (!(flags & FLAG_INEXT)) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (evalid(c)) {
          V3<T> q = (ks[c] * (fdiv(l[c], rest[c]) - T(1))) * t[c];
          F[c] += q;
          if (c < C - 1) F[c + 1] -= q; else to_next -= q;
        }
      }
    }
    if constexpr (TW) {
      T s[4] = {to_prev.x, to_prev.y, to_prev.z, tq_prev};
      X.next(s);
      F[C - 1] += mk(s[0], s[1], s[2]);
      Tq[C - 1] += s[3];
      T s2[3] = {to_next.x, to_next.y, to_next.z};
      X.prev(s2);
      F[0] += mk(s2[0], s2[1], s2[2]);
    } else {
      T s[3] = {to_prev.x, to_prev.y, to_prev.z};
      X.next(s);
      F[C - 1] += mk(s[0], s[1], s[2]);
      T s2[3] = {to_next.x, to_next.y, to_next.z};
      X.prev(s2);
      F[0] += mk(s2[0], s2[1], s2[2]);
    }
    if constexpr (REC) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        rc_->t[c] = t[c];
        rc_->il[c] = il[c];
        rc_->d1[c] = d1[c];
        rc_->kr0[c] = kr0[c];
        rc_->kr1[c] = kr1[c];
        rc_->x[c] = x[c];
      }
      rc_->tp = tp;
      rc_->ilp = ilp;
      rc_->d1p = d1p;
      if constexpr (TW) {
#pragma unroll
        for (int c = 0; c < C; ++c) rc_->th[c] = th[c];
        rc_->thp = thp;
        rc_->m1p = m1p;
      }
    }
    // S3 velocity update and kinematic vertices
#pragma unroll
    for (int c = 0; c < C; ++c) {
      V3<T> vn;
      if (gs[c] >= 0) vn = ug[c];
      else if (w[c] > T(0)) vn = v[c] + h * (g + w[c] * F[c]);
      else vn = zero3<T>();
      v[c] = vn;
      if constexpr (REC) rc_->v1[c] = vn;
    }
    if constexpr (TW) {
#pragma unroll
      for (int c = 0; c < C; ++c) om[c] = jt[c] > T(0) ? om[c] + (h * jt[c]) * Tq[c] : T(0);
    }
    // S4 rigid contact, primitives in order.  A moving body takes the
    // opposite of the summed momentum change and its moment, then its
    // centre moves (symplectic Euler); its block in LDS is rewritten once
    // every lane has read it (the team sum orders that).  The adjoint's
    // replay (REC) leaves the bodies at their substep-start state, which
    // is all its VJP reads.
    if (p1 > p0) {
      for (int k = p0; k < p1; ++k) {
        Prim<T> pr = load_prim(a, k);
        if (!(BD && dyn && a.bw[k] > T(0))) {
#pragma unroll
          for (int c = 0; c < C; ++c)
            if (w[c] > T(0) &&
                contact_one(pr, x[c], rad[c], mu, e, a.eps_s, a.f_thresh, v[c]) && k - p0 < 15)
              bits[c] |= 2u << (k - p0);
        } else {
          T* bk = bs + (k - p0) * NB_VALS;
          pr.a = V3<T>{bk[0], bk[1], bk[2]};
          const V3<T> Vb{bk[3], bk[4], bk[5]}, Om{bk[6], bk[7], bk[8]};
          T acc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
          for (int c = 0; c < C; ++c) {
            if (w[c] > T(0)) {
              const V3<T> vin = v[c];
              V3<T> n;
              const bool hit =
                  contact_moving(pr, x[c], rad[c], mu, e, a.eps_s, a.f_thresh, Vb, Om, v[c], n);
              if (hit && k - p0 < 15) bits[c] |= 2u << (k - p0);
              if (hit && !REC) {
                const V3<T> dp = (T(1) / w[c]) * (v[c] - vin);
                const V3<T> lm = cross(pr.r * n, dp);
                acc[0] += dp.x; acc[1] += dp.y; acc[2] += dp.z;
                acc[3] += lm.x; acc[4] += lm.y; acc[5] += lm.z;
              }
            }
          }
          if constexpr (REC) continue;
          X.sum(acc);
          if (tl == 0) {
            const T bwk = a.bw[k], bik = a.bii[k];
            const V3<T> V1 = Vb - bwk * V3<T>{acc[0], acc[1], acc[2]};
            const V3<T> Om1 = Om - bik * V3<T>{acc[3], acc[4], acc[5]};
            const V3<T> c1 = pr.a + h * V1;
            bk[0] = c1.x; bk[1] = c1.y; bk[2] = c1.z;
            bk[3] = V1.x; bk[4] = V1.y; bk[5] = V1.z;
            bk[6] = Om1.x; bk[7] = Om1.y; bk[8] = Om1.z;
          }
          __syncthreads();
        }
      }
    }
    // S5 predict.  The projections below act on p = p0 + dl with the
    // predicted positions p0 fixed and the corrections accumulated in dl,
    // so S8's (p - p0) / h is dl / h, free of the cancellation that FP32
    // positions would otherwise turn into velocity noise of ulp(x) / h.
    V3<T> p0[C], dl[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      p0[c] = x[c] + h * v[c];
      dl[c] = zero3<T>();
    }
    if constexpr (TW) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        th[c] += h * om[c];
        if constexpr (REC) rc_->th1[c] = th[c];
      }
    }
    // S6 self-contact candidates at the predicted positions
    const bool self_on = SC && (flags & FLAG_SELF);
    if constexpr (SC) {
      if (self_on) sc_broadphase(a, p0);
    }
    // S7 projections
    if ((flags & FLAG_INEXT) || self_on) project<REC>(a, X, p0, dl, lds_tape);
    if constexpr (SC) {
      if (self_on && a.n_iters > 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int n1 = sc_fcnt[gi(c)];
          bits[c] |= (uint32_t)(n1 < 255 ? n1 : 255) << 16;
        }
      }
    }
    // S8 velocity update from the corrections
#pragma unroll
    for (int c = 0; c < C; ++c) {
      v[c] += ih * dl[c];
      x[c] = p0[c] + dl[c];
    }
    // S9 self-friction (its depths come from the first contact pass)
    if constexpr (SC) {
      if (self_on && a.n_iters > 0) {
        if constexpr (REC) {
#pragma unroll
          for (int c = 0; c < C; ++c) {
            rc_->x1[c] = x[c];
            rc_->v3[c] = v[c];
          }
        }
        sc_friction(a, X, x, v);
      }
    }
    // S10 frames by parallel transport in time
    V3<T> t1[C];
    T l1[C], il1[C];
    edges(X, x, t1, l1, il1);
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (evalid(c)) d1[c] = transport(d1[c], t[c], t1[c]);
    if constexpr (REC) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        rc_->t1[c] = t1[c];
        rc_->il1[c] = il1[c];
        rc_->d1n[c] = d1[c];
        rc_->yld[c] = false;
      }
    } else {
      // the next substep starts from these positions and frames
#pragma unroll
      for (int c = 0; c < C; ++c) {
        tc[c] = t1[c];
        lc[c] = l1[c];
        ilc[c] = il1[c];
      }
      geo_ok = true;
      prev_ok = false;
    }
    // S11 plasticity.  Every vertex runs the return map: away from interior
    // vertices the curvature and kappa_bar are zero and so is the threshold,
    // so the (strict) yield test fails there.
    if (flags & FLAG_PLASTIC) {
      // material directors at the new positions and angles (d1 itself
      // without twist)
      V3<T> mn[C];
#pragma unroll
      for (int c = 0; c < C; ++c) mn[c] = TW ? material_m1(t1[c], d1[c], th[c]) : d1[c];
      V3<T> t1p, d1np;
      T il1p;
      prev_edge(X, t1, il1, mn, t1p, il1p, d1np);
      if constexpr (REC) {
        rc_->t1p = t1p;
        rc_->d1np = d1np;
      } else if constexpr (!TW) {
        tpc = t1p;
        ilpc = il1p;
        d1pc = d1np;
        prev_ok = true;
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        T k1, k2;
        curvature(c ? t1[c - 1] : t1p, t1[c], c ? mn[c - 1] : d1np, mn[c], k1, k2);
        T e0 = k1 - kr0[c], e1 = k2 - kr1[c];
        T ss = e0 * e0 + e1 * e1;
        T in = frsq(ss);
        T thr = sig * lbar[c];
        bool y = ss > T(0) && ss * in > thr;   // |kappa_el| = ss / sqrt(ss)
        T phi = y ? rc * (T(1) - thr * in) : T(0);
        if constexpr (REC) {
          rc_->kel0[c] = e0;
          rc_->kel1[c] = e1;
          rc_->inrm[c] = y ? in : T(1);
          rc_->phi[c] = phi;
          rc_->yld[c] = y;
        }
        kr0[c] += phi * e0;
        kr1[c] += phi * e1;
        if (y) bits[c] |= 1u;
      }
    }
    if (!REC && a.branch) {
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (vvalid(c)) a.branch[v0 + gi(c)] = bits[c];
    }
  }

  // ------------------------------------------------------------ substep VJP
  // lx, lv, lk0, lk1, ld1: adjoints of the substep's output state on entry,
  // of its input state on exit.
  __device__ void substep_vjp(const RodArgs<T>& a, Team<T, W>& X, const Rec<T, C>& r,
                              const T* lds_tape, V3<T> (&lx)[C], V3<T> (&lv)[C], T (&lk0)[C],
                              T (&lk1)[C], V3<T> (&ld1)[C], double (&accb)[C],
                              double (&accs)[C], V3<T> (&uacc)[C], T (&lth)[C], T (&lom)[C]) {
    const T h = a.h;
    const T ih = T(1) / h;
    // S11 plasticity: kr' = kr + phi kel on yield
    V3<T> t1b[C], d1nb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      t1b[c] = zero3<T>();
      d1nb[c] = ld1[c];
    }
    if (flags & FLAG_PLASTIC) {
      V3<T> tpb = zero3<T>(), dpb = zero3<T>();
      // twist: curvature of the material directors; their adjoints collect
      // in mnb and go to d1n, t1 and theta afterwards
      V3<T> mn[C], mnb[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        mn[c] = TW ? material_m1(r.t1[c], r.d1n[c], r.th1[c]) : r.d1n[c];
        mnb[c] = zero3<T>();
      }
      V3<T> (&dnb)[C] = TW ? mnb : d1nb;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (r.yld[c]) {   // never set away from interior vertices
          T o0 = lk0[c], o1 = lk1[c];
          T phi = r.phi[c], in = r.inrm[c], thr = sig * lbar[c];
          T phib = r.kel0[c] * o0 + r.kel1[c] * o1;
          T nrmb = rc * thr * in * in * phib;
          T thrb = -rc * in * phib;
          accs[c] += (double)(lbar[c] * thrb);
          T e0 = phi * o0 + (nrmb * in) * r.kel0[c];
          T e1 = phi * o1 + (nrmb * in) * r.kel1[c];
          lk0[c] -= e0;
          lk1[c] -= e1;
          V3<T> t0b, tcb, dab, dcb;
          curvature_vjp(c ? r.t1[c - 1] : r.t1p, r.t1[c], c ? mn[c - 1] : r.d1np, mn[c], e0, e1,
                        t0b, tcb, dab, dcb);
          if (c > 0) {
            t1b[c - 1] += t0b;
            dnb[c - 1] += dab;
          } else {
            tpb += t0b;
            dpb += dab;
          }
          t1b[c] += tcb;
          dnb[c] += dcb;
        }
      }
      T s[6] = {tpb.x, tpb.y, tpb.z, dpb.x, dpb.y, dpb.z};
      X.next(s);
      t1b[C - 1] += mk(s[0], s[1], s[2]);
      dnb[C - 1] += mk(s[3], s[4], s[5]);
      if constexpr (TW) {
#pragma unroll
        for (int c = 0; c < C; ++c)
          if (evalid(c)) d1nb[c] += material_m1_vjp(r.t1[c], r.d1n[c], r.th1[c], mnb[c], t1b[c], lth[c]);
      }
    }
    // S10 transport
    V3<T> tb[C], d1b[C];
    T lb[C], l1b[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      tb[c] = zero3<T>();
      lb[c] = T(0);
      l1b[c] = T(0);
      d1b[c] = zero3<T>();
      if (evalid(c)) d1b[c] = transport_vjp(r.d1[c], r.t[c], r.t1[c], d1nb[c], tb[c], t1b[c]);
    }
    V3<T> pb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) pb[c] = lx[c];
    edges_vjp(X, r.t1, r.il1, t1b, l1b, pb);
    // S9 self-friction
    if constexpr (SC) {
      if ((flags & FLAG_SELF) && a.n_iters > 0) sc_friction_vjp(a, X, r, lv, pb);
    }
    // S8: v' = v2 + (p - p0)/h, x' = p
    V3<T> v2b[C], p0b[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      pb[c] += ih * lv[c];
      v2b[c] = lv[c];
      p0b[c] = -(ih * lv[c]);
    }
    // S7
    if ((flags & FLAG_INEXT) || (SC && (flags & FLAG_SELF))) project_vjp(a, X, pb, lds_tape);
    // S5 p0 = x + h v2 (twist: theta' = theta + h omega')
    V3<T> xb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      p0b[c] += pb[c];
      xb[c] = p0b[c];
      v2b[c] += h * p0b[c];
      if constexpr (TW) lom[c] += h * lth[c];
    }
    // S4 rigid contact, primitives in reverse.
    if (BD && p1 > p0 && dyn) {
      // With moving bodies every lane walks the primitives in the same
      // (reverse) order, so that each body's adjoint can be summed over the
      // team: the input velocity of primitive k is re-evaluated from the
      // substep's post-S3 velocity; bs holds the substep-start body states.
      for (int k = p1 - 1; k >= p0; --k) {
        Prim<T> pk = load_prim(a, k);
        const bool mk = a.bw[k] > T(0);
        V3<T> Vk = zero3<T>(), Omk = zero3<T>(), Pb = zero3<T>(), Lb = zero3<T>();
        T lnew[9];
        T acc[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) acc[i] = T(0);
        if (mk) {
          const T* bk = bs + (k - p0) * NB_VALS;
          const T* lk = lbs + (k - p0) * NB_VALS;
          pk.a = V3<T>{bk[0], bk[1], bk[2]};
          Vk = V3<T>{bk[3], bk[4], bk[5]};
          Omk = V3<T>{bk[6], bk[7], bk[8]};
          // c1 = c0 + h V1, V1 = V0 - W P, Om1 = Om0 - I^-1 L
          const V3<T> cb{lk[0], lk[1], lk[2]};
          const V3<T> V1b = V3<T>{lk[3], lk[4], lk[5]} + h * cb;
          const V3<T> Om1b{lk[6], lk[7], lk[8]};
          Pb = (-a.bw[k]) * V1b;
          Lb = (-a.bii[k]) * Om1b;
          lnew[0] = cb.x; lnew[1] = cb.y; lnew[2] = cb.z;
          lnew[3] = V1b.x; lnew[4] = V1b.y; lnew[5] = V1b.z;
          lnew[6] = Om1b.x; lnew[7] = Om1b.y; lnew[8] = Om1b.z;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
          if (w[c] > T(0)) {
            V3<T> vk = r.v1[c];
            for (int j = p0; j < k; ++j) {
              Prim<T> pj = load_prim(a, j);
              if (a.bw[j] > T(0)) {
                const T* bj = bs + (j - p0) * NB_VALS;
                pj.a = V3<T>{bj[0], bj[1], bj[2]};
                V3<T> nn;
                contact_moving(pj, r.x[c], rad[c], mu, e, a.eps_s, a.f_thresh,
                               V3<T>{bj[3], bj[4], bj[5]}, V3<T>{bj[6], bj[7], bj[8]}, vk, nn);
              } else {
                contact_one(pj, r.x[c], rad[c], mu, e, a.eps_s, a.f_thresh, vk);
              }
            }
            if (mk)
              contact_moving_vjp(pk, r.x[c], rad[c], mu, e, a.eps_s, a.f_thresh, Vk, Omk,
                                 T(1) / w[c], vk, Pb, Lb, v2b[c], xb[c], acc);
            else
              contact_one_vjp(pk, r.x[c], rad[c], mu, e, a.eps_s, a.f_thresh, vk, v2b[c], xb[c]);
          }
        }
        if (mk) {
          X.sum(acc);
          if (tl == 0) {
            T* lk = lbs + (k - p0) * NB_VALS;
#pragma unroll
            for (int i = 0; i < 9; ++i) lk[i] = lnew[i] + acc[i];
          }
          __syncthreads();
        }
      }
    } else if (p1 > p0) {
      // One forward sweep re-runs the primitives in order and keeps the
      // input velocity of each active one (up to three; inactive primitives
      // leave v unchanged and have a zero VJP); more than three active
      // contacts fall back to re-evaluating each primitive's input from the
      // start.
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (w[c] > T(0)) {
          V3<T> vin = r.v1[c], vs0 = vin, vs1 = vin, vs2 = vin;
          int k0 = -1, k1 = -1, k2 = -1, na = 0;
          for (int j = p0; j < p1; ++j) {
            V3<T> vb4 = vin;
            if (contact_one(load_prim(a, j), r.x[c], rad[c], mu, e, a.eps_s, a.f_thresh, vin)) {
              if (na == 0) { vs0 = vb4; k0 = j; }
              else if (na == 1) { vs1 = vb4; k1 = j; }
              else if (na == 2) { vs2 = vb4; k2 = j; }
              ++na;
            }
          }
          if (na <= 3) {
            if (k2 >= 0)
              contact_one_vjp(load_prim(a, k2), r.x[c], rad[c], mu, e, a.eps_s, a.f_thresh, vs2,
                              v2b[c], xb[c]);
            if (k1 >= 0)
              contact_one_vjp(load_prim(a, k1), r.x[c], rad[c], mu, e, a.eps_s, a.f_thresh, vs1,
                              v2b[c], xb[c]);
            if (k0 >= 0)
              contact_one_vjp(load_prim(a, k0), r.x[c], rad[c], mu, e, a.eps_s, a.f_thresh, vs0,
                              v2b[c], xb[c]);
          } else {
            for (int k = p1 - 1; k >= p0; --k) {
              V3<T> vk = r.v1[c];
              for (int j = p0; j < k; ++j)
                contact_one(load_prim(a, j), r.x[c], rad[c], mu, e, a.eps_s, a.f_thresh, vk);
              contact_one_vjp(load_prim(a, k), r.x[c], rad[c], mu, e, a.eps_s, a.f_thresh, vk,
                              v2b[c], xb[c]);
            }
          }
        }
      }
    }
    // S3
    V3<T> Fb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (gs[c] >= 0) {
        uacc[c] += v2b[c];
        lv[c] = zero3<T>();
        Fb[c] = zero3<T>();
      } else if (w[c] > T(0)) {
        lv[c] = v2b[c];
        Fb[c] = (h * w[c]) * v2b[c];
      } else {
        lv[c] = zero3<T>();
        Fb[c] = zero3<T>();
      }
    }
    if constexpr (TW) {
      s2_vjp_twist(a, X, r, Fb, tb, lb, d1b, xb, lx, lk0, lk1, ld1, accb, lth, lom);
      return;
    }
    // S2 forces
    T fp[3] = {Fb[C - 1].x, Fb[C - 1].y, Fb[C - 1].z};
    X.prev(fp);
    T fn[3] = {Fb[0].x, Fb[0].y, Fb[0].z};
    X.next(fn);
    V3<T> Fp = mk(fp[0], fp[1], fp[2]), Fn = mk(fn[0], fn[1], fn[2]);
    V3<T> d2b[C];
#pragma unroll
    for (int c = 0; c < C; ++c) d2b[c] = zero3<T>();
    V3<T> tpb = zero3<T>(), d1pb = zero3<T>(), d2pb = zero3<T>();
    T lpb = T(0);
    // every vertex runs the stencil's VJP: away from interior vertices
    // coef = 1/l_bar = 0 makes every output exactly zero
#pragma unroll
    for (int c = 0; c < C; ++c) {
      BendIn<T> q = bend_in(c, r.t, r.il, r.d1, r.tp, r.ilp, r.d1p, r.kr0, r.kr1);
      V3<T> Fm = c ? Fb[c - 1] : Fp;
      V3<T> Fq = (c < C - 1) ? Fb[c + 1] : Fn;
      BendBar<T> o;
      bend_vjp(q, Fm - Fb[c], Fb[c] - Fq, o);
      lk0[c] += o.kr0;
      lk1[c] += o.kr1;
      accb[c] += (double)o.b;
      if (c > 0) {
        tb[c - 1] += o.t0;
        lb[c - 1] += o.l0;
        d1b[c - 1] += o.d1a;
        d2b[c - 1] += o.d2a;
      } else {
        tpb += o.t0;
        lpb += o.l0;
        d1pb += o.d1a;
        d2pb += o.d2a;
      }
      tb[c] += o.t1;
      lb[c] += o.l1;
      d1b[c] += o.d1b;
      d2b[c] += o.d2b;
    }
    if (!(flags & FLAG_INEXT)) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (evalid(c)) {
          V3<T> Fq = (c < C - 1) ? Fb[c + 1] : Fn;
          V3<T> qb = Fb[c] - Fq;
          T fs = ks[c] * (fdiv(frcp(r.il[c]), rest[c]) - T(1));
          tb[c] += fs * qb;
          lb[c] += fdiv(ks[c] * dot(qb, r.t[c]), rest[c]);
        }
      }
    }
    {
      T s[10] = {tpb.x, tpb.y, tpb.z, lpb, d1pb.x, d1pb.y, d1pb.z, d2pb.x, d2pb.y, d2pb.z};
      X.next(s);
      tb[C - 1] += mk(s[0], s[1], s[2]);
      lb[C - 1] += s[3];
      d1b[C - 1] += mk(s[4], s[5], s[6]);
      d2b[C - 1] += mk(s[7], s[8], s[9]);
    }
    // d2 = t x d1
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (evalid(c)) {
        tb[c] += cross(r.d1[c], d2b[c]);
        d1b[c] += cross(d2b[c], r.t[c]);
      } else {
        d1b[c] = zero3<T>();
      }
    }
    edges_vjp(X, r.t, r.il, tb, lb, xb);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      lx[c] = vvalid(c) ? xb[c] : zero3<T>();
      ld1[c] = d1b[c];
    }
  }

  // Twist rates (S3) and forces and torques (S2) of the adjoint for rods
  // with the twist degree of freedom: the bending stencil on the material
  // directors, the twist stencil, then m2 = t x m1 and m1 = R(theta) d1.
  __device__ void s2_vjp_twist(const RodArgs<T>& a, Team<T, W>& X, const Rec<T, C>& r,
                               const V3<T> (&Fb)[C], V3<T> (&tb)[C], T (&lb)[C],
                               V3<T> (&d1b)[C], V3<T> (&xb)[C], V3<T> (&lx)[C], T (&lk0)[C],
                               T (&lk1)[C], V3<T> (&ld1)[C], double (&accb)[C], T (&lth)[C],
                               T (&lom)[C]) {
    const T h = a.h;
    T Tqb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const bool fr = jt[c] > T(0);
      Tqb[c] = fr ? (h * jt[c]) * lom[c] : T(0);
      lom[c] = fr ? lom[c] : T(0);
    }
    T fp[4] = {Fb[C - 1].x, Fb[C - 1].y, Fb[C - 1].z, Tqb[C - 1]};
    X.prev(fp);
    T fn[3] = {Fb[0].x, Fb[0].y, Fb[0].z};
    X.next(fn);
    const V3<T> Fp = mk(fp[0], fp[1], fp[2]), Fn = mk(fn[0], fn[1], fn[2]);
    const T Tqp = fp[3];
    V3<T> m1[C], m1b[C], d2b[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      m1[c] = material_m1(r.t[c], r.d1[c], r.th[c]);
      m1b[c] = zero3<T>();
      d2b[c] = zero3<T>();
    }
    V3<T> tpb = zero3<T>(), m1pb = zero3<T>(), d2pb = zero3<T>(), rdpb = zero3<T>();
    T lpb = T(0), thpb = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      BendIn<T> q = bend_in(c, r.t, r.il, m1, r.tp, r.ilp, r.m1p, r.kr0, r.kr1);
      V3<T> Fm = c ? Fb[c - 1] : Fp;
      V3<T> Fq = (c < C - 1) ? Fb[c + 1] : Fn;
      V3<T> g0b = Fm - Fb[c], g1b = Fb[c] - Fq;
      BendBar<T> o;
      bend_vjp(q, g0b, g1b, o);
      TwIn<T> tq{q.t0,  q.t1,  q.d1a, q.d1b, c ? r.d1[c - 1] : r.d1p, r.d1[c], q.il0,
                 q.il1, c ? r.th[c - 1] : r.thp, r.th[c], q.kr0, q.kr1, q.coef, q.ilbar,
                 tcoef[c]};
      TwBar<T> ow;
      twist_vjp(tq, g0b, g1b, c ? Tqb[c - 1] : Tqp, Tqb[c], ow);
      lk0[c] += o.kr0 + ow.kr0;
      lk1[c] += o.kr1 + ow.kr1;
      accb[c] += (double)o.b + (double)ow.b;
      if (c > 0) {
        tb[c - 1] += o.t0 + ow.t0;
        lb[c - 1] += o.l0 + ow.l0;
        m1b[c - 1] += o.d1a + ow.m1a;
        d2b[c - 1] += o.d2a + ow.m2a;
        d1b[c - 1] += ow.d1a;
        lth[c - 1] += ow.tha;
      } else {
        tpb += o.t0 + ow.t0;
        lpb += o.l0 + ow.l0;
        m1pb += o.d1a + ow.m1a;
        d2pb += o.d2a + ow.m2a;
        rdpb += ow.d1a;
        thpb += ow.tha;
      }
      tb[c] += o.t1 + ow.t1;
      lb[c] += o.l1 + ow.l1;
      m1b[c] += o.d1b + ow.m1b;
      d2b[c] += o.d2b + ow.m2b;
      d1b[c] += ow.d1b;
      lth[c] += ow.thb;
    }
    if (!(flags & FLAG_INEXT)) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (evalid(c)) {
          V3<T> Fq = (c < C - 1) ? Fb[c + 1] : Fn;
          V3<T> qb = Fb[c] - Fq;
          T fs = ks[c] * (fdiv(frcp(r.il[c]), rest[c]) - T(1));
          tb[c] += fs * qb;
          lb[c] += fdiv(ks[c] * dot(qb, r.t[c]), rest[c]);
        }
      }
    }
    {
      T s[10] = {tpb.x, tpb.y, tpb.z, lpb, m1pb.x, m1pb.y, m1pb.z, d2pb.x, d2pb.y, d2pb.z};
      X.next(s);
      tb[C - 1] += mk(s[0], s[1], s[2]);
      lb[C - 1] += s[3];
      m1b[C - 1] += mk(s[4], s[5], s[6]);
      d2b[C - 1] += mk(s[7], s[8], s[9]);
      T s2[4] = {rdpb.x, rdpb.y, rdpb.z, thpb};
      X.next(s2);
      d1b[C - 1] += mk(s2[0], s2[1], s2[2]);
      lth[C - 1] += s2[3];
    }
    // m2 = t x m1, m1 = cos(theta) d1 + sin(theta) t x d1
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (evalid(c)) {
        tb[c] += cross(m1[c], d2b[c]);
        m1b[c] += cross(d2b[c], r.t[c]);
        d1b[c] += material_m1_vjp(r.t[c], r.d1[c], r.th[c], m1b[c], tb[c], lth[c]);
      } else {
        d1b[c] = zero3<T>();
        lth[c] = T(0);
        lom[c] = T(0);
      }
    }
    edges_vjp(X, r.t, r.il, tb, lb, xb);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      lx[c] = vvalid(c) ? xb[c] : zero3<T>();
      ld1[c] = d1b[c];
    }
  }
};

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <typename T, int W>
__device__ __forceinline__ size_t xchg_bytes() { return W > 1 ? 2 * W * XK * sizeof(T) : 0; }

// Forward: n_steps steps of every rod of the work list, the rod resident in
// registers the whole time.  TAPE: store every substep-start state.  SC:
// self-contact (position staging and the pair-record cache in LDS, the
// neighbour lists and pair lists in the rod's global pair block).
template <typename T, int C, int W, bool TAPE, bool SC, bool TW, bool BD>
__global__ __launch_bounds__(64 * W) void k_forward(RodArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  Team<T, W> X;
  X.init(reinterpret_cast<T*>(smem));
  Rod<T, C, W, SC, TW, BD> R;
  R.load_static(a, X);
  if constexpr (SC) {
    R.sc_layout(smem + xchg_bytes<T, W>(), a, SC_RV_FWD, xchg_bytes<T, W>());
    R.ctape = nullptr;
    R.sc_setup(a);
  }
  R.body_setup(a, smem);
  R.load_state(a.x, a.v, a.kb, a.d1);
  if constexpr (TW) R.load_twist(a.th, a.om);
  if (BD && R.dyn) R.load_bodies(R.bs, a.body);
  T* tape_rod = TAPE ? a.tape + a.tape_off[R.rod] : nullptr;
  for (int s = 0; s < a.n_steps; ++s) {
    V3<T> ug[C];
    R.load_actions(a, (a.step_off + s) / a.spa, ug);
    for (int k = 0; k < a.n_sub; ++k) {
      if constexpr (TAPE) {
        R.store_tape(tape_rod + (int64_t)(s * a.n_sub + k) * a.tape_stride);
        if (BD && R.dyn) R.store_bodies(a.btape + (int64_t)(s * a.n_sub + k) * a.bstride, R.bs);
      }
      R.template substep<false>(a, X, ug, nullptr, nullptr);
    }
  }
  R.store_state(a.x, a.v, a.kb, a.d1);
  if (a.ck_x) R.store_state(a.ck_x, a.ck_v, a.ck_kb, a.ck_d1);
  if (BD && R.dyn) {
    R.store_bodies(a.body, R.bs);
    if (a.ck_body) R.store_bodies(a.ck_body, R.bs);
  }
  if constexpr (TW) {
    R.store_twist(a.th, a.om);
    if (a.ck_x) R.store_twist(a.ck_th, a.ck_om);
  }
  bool bad = false;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    T s = dot(R.x[c], R.x[c]) + dot(R.v[c], R.v[c]);
    bad |= !(s == s) || s > T(1e30);
  }
  int fl = bad ? 1 : 0;
  if constexpr (SC) {
    fl |= R.sc_flags;
    R.sc_stats_out(a);
  }
  if (fl) atomicOr(a.status + R.rod, fl);
}

// Adjoint over the launch's steps, last to first, from the substep tape.
// GT: the projection iterates of a substep go to a rod-private block of
// global scratch (L2-resident) instead of LDS -- for teams whose iterates do
// not fit in LDS, and always with self-contact, whose buffers fill the LDS.
template <typename T, int C, int W, bool SC, bool GT, bool TW, bool BD>
__global__ __launch_bounds__(64 * W) void k_adjoint(RodArgs<T> a) {
  static_assert(GT || !SC, "self-contact keeps the iterates in global scratch");
  extern __shared__ __align__(16) unsigned char smem[];
  Team<T, W> X;
  X.init(reinterpret_cast<T*>(smem));
  Rod<T, C, W, SC, TW, BD> R;
  R.load_static(a, X);
  T* lds_tape;
  if constexpr (GT) {
    lds_tape = a.sc_tape + a.sc_off[R.rod];
  } else {
    lds_tape = reinterpret_cast<T*>(smem + xchg_bytes<T, W>());
  }
  if constexpr (SC) {
    // LDS holds the self-contact buffers; the contact-pass inputs follow the
    // projection iterates in the rod's scratch block (written and read
    // within a substep)
    R.sc_layout(smem + xchg_bytes<T, W>(), a, SC_RV_ADJ, xchg_bytes<T, W>());
    R.ctape = lds_tape + (size_t)a.n_iters * C * PROJ_TAPE * 64 * W;
    R.sc_setup(a);
  }
  R.body_setup(a, smem);
  if (BD && R.dyn) R.load_bodies(R.lbs, a.lbody);
  V3<T> lx[C], lv[C], ld1[C], uacc[C];
  T lk0[C], lk1[C], lth[C], lom[C];
  double accb[C], accs[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    int g = R.gi(c), row = R.v0 + g;
    bool vv = g < R.N;
    lx[c] = vv ? get3(a.lx, 3 * row) : zero3<T>();
    lv[c] = vv ? get3(a.lv, 3 * row) : zero3<T>();
    lk0[c] = R.ivalid(c) ? a.lkb[2 * row] : T(0);
    lk1[c] = R.ivalid(c) ? a.lkb[2 * row + 1] : T(0);
    ld1[c] = R.evalid(c) ? get3(a.ld1, 3 * row) : zero3<T>();
    lth[c] = (TW && R.evalid(c)) ? a.lth[row] : T(0);
    lom[c] = (TW && R.evalid(c)) ? a.lom[row] : T(0);
    accb[c] = 0.0;
    accs[c] = 0.0;
    uacc[c] = zero3<T>();
  }
  const T* tape_rod = a.tape + a.tape_off[R.rod];
  Rec<T, C> rec;
  T pf[Rod<T, C, W, SC, TW, BD>::NFIELD * C];
  R.fetch_tape(tape_rod + (int64_t)(a.n_steps * a.n_sub - 1) * a.tape_stride, pf);
  T bpf[Rod<T, C, W, SC, TW, BD>::BPF];
  if (BD && R.dyn) R.fetch_bodies(a.btape + (int64_t)(a.n_steps * a.n_sub - 1) * a.bstride, bpf);
  for (int s = a.n_steps - 1; s >= 0; --s) {
    const int act = (a.step_off + s) / a.spa;
    V3<T> ug[C];
    R.load_actions(a, act, ug);
    for (int k = a.n_sub - 1; k >= 0; --k) {
      R.install_tape(pf);
      const int nxt = s * a.n_sub + k - 1;   // the substep processed next
      if (nxt >= 0) R.fetch_tape(tape_rod + (int64_t)nxt * a.tape_stride, pf);
      // the substep-start body states (the replay leaves them unchanged)
      if (BD && R.dyn) {
        R.install_bodies(bpf);
        if (nxt >= 0) R.fetch_bodies(a.btape + (int64_t)nxt * a.bstride, bpf);
      }
      R.template substep<true>(a, X, ug, &rec, lds_tape);
      R.substep_vjp(a, X, rec, lds_tape, lx, lv, lk0, lk1, ld1, accb, accs, uacc, lth, lom);
    }
    // grasp-velocity gradient of this step's action
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (R.gs[c] >= 0) {
        T* o = a.dL_du + (int64_t)act * a.act_stride + (int64_t)(R.rod * a.G + R.gs[c]) * 3;
        o[0] += uacc[c].x;
        o[1] += uacc[c].y;
        o[2] += uacc[c].z;
        uacc[c] = zero3<T>();
      }
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    int g = R.gi(c), row = R.v0 + g;
    if (g < R.N) {
      put3(a.lx, 3 * row, lx[c]);
      put3(a.lv, 3 * row, lv[c]);
      a.lkb[2 * row] = lk0[c];
      a.lkb[2 * row + 1] = lk1[c];
      put3(a.ld1, 3 * row, ld1[c]);
      if constexpr (TW) {
        a.lth[row] = lth[c];
        a.lom[row] = lom[c];
      }
      a.acc_b[row] += accb[c];
      a.acc_s[row] += accs[c];
    }
  }
  if (BD && R.dyn) R.store_bodies(a.lbody, R.lbs);
  if constexpr (SC) R.sc_stats_out(a);
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

// Initial-frame rule, one thread per rod walking its edges.
template <typename T>
__global__ void k_init_frames(const int32_t* voff, int R, const T* x, T* d1) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int v0 = voff[r], N = voff[r + 1] - v0;
  V3<T> e = get3(x, 3 * (v0 + 1)) - get3(x, 3 * v0);
  V3<T> t = (T(1) / sqrt(dot(e, e))) * e;
  V3<T> az = mk(T(0), T(0), T(1));
  V3<T> c = cross(t, az);
  V3<T> av = sqrt(dot(c, c)) < T(1e-6) ? mk(T(1), T(0), T(0)) : az;
  V3<T> d = av - dot(av, t) * t;
  d = (T(1) / sqrt(dot(d, d))) * d;
  put3(d1, 3 * v0, d);
  for (int j = 1; j < N - 1; ++j) {
    V3<T> en = get3(x, 3 * (v0 + j + 1)) - get3(x, 3 * (v0 + j));
    V3<T> tn = (T(1) / sqrt(dot(en, en))) * en;
    d = transport(d, t, tn);
    put3(d1, 3 * (v0 + j), d);
    t = tn;
  }
  put3(d1, 3 * (v0 + N - 1), zero3<T>());
}

// Adjoint of the initial-frame rule: the frame adjoint d1b [V][3] (edge
// rows) maps onto the positions through the first frame's construction and
// the parallel transport along the rod; adds the result to xb.  One thread
// per rod: the frames are rebuilt forward into tmp, then the transports
// are reversed from the last edge to the first (the choice of the first
// frame's reference axis is piecewise constant).
template <typename T>
__global__ void k_init_frames_vjp(const int32_t* voff, int R, const T* x, const T* d1b, T* tmp,
                                  T* xb) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int v0 = voff[r], N = voff[r + 1] - v0;
  if (N < 2) return;
  auto edge = [&](int j, T& l) {
    V3<T> e = get3(x, 3 * (v0 + j + 1)) - get3(x, 3 * (v0 + j));
    l = sqrt(dot(e, e));
    return (T(1) / l) * e;
  };
  T l0;
  V3<T> t = edge(0, l0);
  const V3<T> t0 = t;
  V3<T> az = mk(T(0), T(0), T(1));
  V3<T> cz = cross(t, az);
  V3<T> av = sqrt(dot(cz, cz)) < T(1e-6) ? mk(T(1), T(0), T(0)) : az;
  V3<T> dd = av - dot(av, t) * t;
  const T nd = sqrt(dot(dd, dd));
  V3<T> d = (T(1) / nd) * dd;
  put3(tmp, 3 * v0, d);
  for (int j = 1; j < N - 1; ++j) {
    T lj;
    V3<T> tn = edge(j, lj);
    d = transport(d, t, tn);
    put3(tmp, 3 * (v0 + j), d);
    t = tn;
  }
  // reverse: edge j's tangent adjoint is complete once the transports into
  // and out of it are reversed
  V3<T> carry = zero3<T>(), pend = zero3<T>();
  for (int j = N - 2; j >= 1; --j) {
    T la, lb;
    const V3<T> ta = edge(j - 1, la), tb = edge(j, lb);
    V3<T> ta_b = zero3<T>(), tb_b = zero3<T>();
    carry = transport_vjp(get3(tmp, 3 * (v0 + j - 1)), ta, tb, get3(d1b, 3 * (v0 + j)) + carry,
                          ta_b, tb_b);
    const V3<T> tj = pend + tb_b;
    const V3<T> eb = (T(1) / lb) * (tj - dot(tb, tj) * tb);
    put3(xb, 3 * (v0 + j + 1), get3(xb, 3 * (v0 + j + 1)) + eb);
    put3(xb, 3 * (v0 + j), get3(xb, 3 * (v0 + j)) - eb);
    pend = ta_b;
  }
  // first frame: d1 = dd / |dd|, dd = a - (a.t) t
  const V3<T> g = get3(d1b, 3 * v0) + carry;
  const V3<T> u = (T(1) / nd) * dd;
  const V3<T> ddb = (T(1) / nd) * (g - dot(u, g) * u);
  const V3<T> t0b = pend - dot(av, t0) * ddb - dot(ddb, t0) * av;
  const V3<T> eb = (T(1) / l0) * (t0b - dot(t0, t0b) * t0);
  put3(xb, 3 * (v0 + 1), get3(xb, 3 * (v0 + 1)) + eb);
  put3(xb, 3 * v0, get3(xb, 3 * v0) - eb);
}

// Material curvature of a shape at every interior vertex.
template <typename T>
__global__ void k_curvature(const int32_t* voff, const int32_t* rod_of, int V, const T* x,
                            const T* d1, T* kappa) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  int r = rod_of[i];
  int v0 = voff[r], N = voff[r + 1] - v0, j = i - v0;
  T k1 = T(0), k2 = T(0);
  if (j >= 1 && j <= N - 2) {
    V3<T> e0 = get3(x, 3 * i) - get3(x, 3 * (i - 1));
    V3<T> e1 = get3(x, 3 * (i + 1)) - get3(x, 3 * i);
    V3<T> t0 = (T(1) / sqrt(dot(e0, e0))) * e0, t1 = (T(1) / sqrt(dot(e1, e1))) * e1;
    curvature(t0, t1, get3(d1, 3 * (i - 1)), get3(d1, 3 * i), k1, k2);
  }
  kappa[2 * i] = k1;
  kappa[2 * i + 1] = k2;
}

// per-rod fixed-order sum of per-vertex parameter partials
template <typename T>
__global__ void k_reduce_params(const int32_t* voff, int R, const double* acc_b,
                                const double* acc_s, T* db, T* ds) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double sb = 0.0, ss = 0.0;
  for (int i = voff[r]; i < voff[r + 1]; ++i) {
    sb += acc_b[i];
    ss += acc_s[i];
  }
  if (db) db[r] = (T)sb;
  if (ds) ds[r] = (T)ss;
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = val;
}

#if RODS_TU == 0
__global__ void k_selftest_exchange(int* out) {
  int l = threadIdx.x;
  int nx = dpp_from_next_i(l + 1) - 1;
  int pv = dpp_from_prev_i(l + 1) - 1;
  out[l] = nx;
  out[64 + l] = pv;
}
#endif

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

template <typename T, int C, int W, bool SC>
static size_t lds_bytes(int which, bool gt, int n_iters) {
  size_t xb = W > 1 ? 2 * W * XK * sizeof(T) : 0;
  if constexpr (SC) return xb + Rod<T, C, W, SC, false>::sc_bytes();
  if (which == 2 && !gt) return xb + (size_t)n_iters * C * PROJ_TAPE * 64 * W * sizeof(T);
  return xb;
}

template <typename T, int C, int W, bool SC, bool TW = false, bool BD = false>
static hipError_t launch_shape(int which, bool gt, const RodArgs<T>& a, int n_blocks,
                               hipStream_t st) {
  size_t lds = lds_bytes<T, C, W, SC>(which, gt, a.n_iters);
  RodArgs<T> b = a;
  if constexpr (SC) {
    // the pair cache takes whatever more the host offers (one workgroup
    // per CU either way), less the moving bodies' blocks
    size_t offer = (size_t)a.sc_lds;
    if constexpr (BD) {
      const size_t bl = body_lds_bytes<T>() + 16;
      offer = offer > bl ? offer - bl : 0;
    }
    if (offer > lds) lds = offer;
    b.sc_lds = (int32_t)lds;
  }
  if constexpr (BD) {
    // moving bodies: state and adjoint blocks after everything else
    b.body_lds = (int32_t)((lds + 15) / 16 * 16);
    lds = (size_t)b.body_lds + body_lds_bytes<T>();
  }
  auto go = [&](auto f) {
    if (lds > 65536) hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(f, dim3(n_blocks), dim3(64 * W), lds, st, b);
  };
  if (which == 0) {
    go(k_forward<T, C, W, false, SC, TW, BD>);
  } else if (which == 1) {
    go(k_forward<T, C, W, true, SC, TW, BD>);
  } else if constexpr (SC) {
    go(k_adjoint<T, C, W, true, true, TW, BD>);
  } else {
    if (gt) go(k_adjoint<T, C, W, false, true, TW, BD>);
    else go(k_adjoint<T, C, W, false, false, TW, BD>);
  }
  return hipGetLastError();
}

#if RODS_TU == 1
// Rods with the twist degree of freedom: two vertices per lane, without
// self-contact, with and without moving rigid bodies (this translation unit
// instantiates only these kernels).
template <typename T>
hipError_t launch_rods_twist(int which, int C, int W, bool GT, const RodArgs<T>& a,
                             int n_blocks, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (C != 2) return hipErrorInvalidValue;
  if (W == 1) return launch_shape<T, 2, 1, false, true>(which, GT, a, n_blocks, st);
  if (W == 2) return launch_shape<T, 2, 2, false, true>(which, GT, a, n_blocks, st);
  if (W == 4) return launch_shape<T, 2, 4, false, true>(which, GT, a, n_blocks, st);
  if (W == 8) return launch_shape<T, 2, 8, false, true>(which, GT, a, n_blocks, st);
  return hipErrorInvalidValue;
}
// ... and those with moving rigid bodies too (a.bw set)
template <typename T>
hipError_t launch_rods_twist_bodies(int which, int C, int W, bool GT, const RodArgs<T>& a,
                                    int n_blocks, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (C != 2 || !a.bw) return hipErrorInvalidValue;
  if (W == 1) return launch_shape<T, 2, 1, false, true, true>(which, GT, a, n_blocks, st);
  if (W == 2) return launch_shape<T, 2, 2, false, true, true>(which, GT, a, n_blocks, st);
  if (W == 4) return launch_shape<T, 2, 4, false, true, true>(which, GT, a, n_blocks, st);
  if (W == 8) return launch_shape<T, 2, 8, false, true, true>(which, GT, a, n_blocks, st);
  return hipErrorInvalidValue;
}
template hipError_t launch_rods_twist_bodies<float>(int, int, int, bool, const RodArgs<float>&,
                                                    int, hipStream_t);
template hipError_t launch_rods_twist_bodies<double>(int, int, int, bool,
                                                     const RodArgs<double>&, int, hipStream_t);
template hipError_t launch_rods_twist<float>(int, int, int, bool, const RodArgs<float>&, int,
                                             hipStream_t);
template hipError_t launch_rods_twist<double>(int, int, int, bool, const RodArgs<double>&, int,
                                              hipStream_t);
#elif RODS_TU == 2
// Rods with self-contact: FP32 teams of two vertices per lane and 1-8 waves
// or four vertices per lane and 4 waves, FP64 teams of two vertices per lane;
// with moving rigid bodies two vertices per lane (this translation unit
// instantiates only these kernels).
template <typename T>
hipError_t launch_rods_sc(int which, int C, int W, const RodArgs<T>& a, int n_blocks,
                          hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (C == 2 && W == 1) return launch_shape<T, 2, 1, true>(which, true, a, n_blocks, st);
  if (C == 2 && W == 2) return launch_shape<T, 2, 2, true>(which, true, a, n_blocks, st);
  if (C == 2 && W == 4) return launch_shape<T, 2, 4, true>(which, true, a, n_blocks, st);
  if (C == 2 && W == 8) return launch_shape<T, 2, 8, true>(which, true, a, n_blocks, st);
  if constexpr (sizeof(T) == 4) {
    if (C == 4 && W == 4) return launch_shape<T, 4, 4, true>(which, true, a, n_blocks, st);
  }
  return hipErrorInvalidValue;
}
// ... and those with moving rigid bodies too (two vertices per lane)
template <typename T>
hipError_t launch_rods_sc_bodies(int which, int C, int W, const RodArgs<T>& a, int n_blocks,
                                 hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (C != 2 || !a.bw) return hipErrorInvalidValue;
  if (W == 1) return launch_shape<T, 2, 1, true, false, true>(which, true, a, n_blocks, st);
  if (W == 2) return launch_shape<T, 2, 2, true, false, true>(which, true, a, n_blocks, st);
  if (W == 4) return launch_shape<T, 2, 4, true, false, true>(which, true, a, n_blocks, st);
  if (W == 8) return launch_shape<T, 2, 8, true, false, true>(which, true, a, n_blocks, st);
  return hipErrorInvalidValue;
}
template hipError_t launch_rods_sc_bodies<float>(int, int, int, const RodArgs<float>&, int,
                                                 hipStream_t);
template hipError_t launch_rods_sc_bodies<double>(int, int, int, const RodArgs<double>&, int,
                                                  hipStream_t);
template <typename T>
size_t sc_lds_bytes(int C, int W) {
  size_t xb = W > 1 ? 2 * W * XK * sizeof(T) : 0;
  if (C == 2 && W == 1) return xb + Rod<T, 2, 1, true>::sc_bytes();
  if (C == 2 && W == 2) return xb + Rod<T, 2, 2, true>::sc_bytes();
  if (C == 2 && W == 4) return xb + Rod<T, 2, 4, true>::sc_bytes();
  if (C == 2 && W == 8) return xb + Rod<T, 2, 8, true>::sc_bytes();
  if (sizeof(T) == 4 && C == 4 && W == 4) return xb + Rod<T, 4, 4, true>::sc_bytes();
  return (size_t)1 << 30;   // no self-contact kernel for this shape
}
template hipError_t launch_rods_sc<float>(int, int, int, const RodArgs<float>&, int, hipStream_t);
template hipError_t launch_rods_sc<double>(int, int, int, const RodArgs<double>&, int,
                                           hipStream_t);
template size_t sc_lds_bytes<float>(int, int);
template size_t sc_lds_bytes<double>(int, int);
#elif RODS_TU == 3
// Rods with the twist degree of freedom and self-contact: two vertices per
// lane, 1-8 waves (this translation unit instantiates only these kernels).
template <typename T>
hipError_t launch_rods_sc_twist(int which, int C, int W, const RodArgs<T>& a, int n_blocks,
                                hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (C != 2) return hipErrorInvalidValue;
  if (W == 1) return launch_shape<T, 2, 1, true, true>(which, true, a, n_blocks, st);
  if (W == 2) return launch_shape<T, 2, 2, true, true>(which, true, a, n_blocks, st);
  if (W == 4) return launch_shape<T, 2, 4, true, true>(which, true, a, n_blocks, st);
  if (W == 8) return launch_shape<T, 2, 8, true, true>(which, true, a, n_blocks, st);
  return hipErrorInvalidValue;
}
template hipError_t launch_rods_sc_twist<float>(int, int, int, const RodArgs<float>&, int,
                                                hipStream_t);
template hipError_t launch_rods_sc_twist<double>(int, int, int, const RodArgs<double>&, int,
                                                 hipStream_t);
#else
template <typename T>
hipError_t launch_rods(int which, int C, int W, bool SC, bool GT, const RodArgs<T>& a,
                       int n_blocks, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (SC) return launch_rods_sc<T>(which, C, W, a, n_blocks, st);
#define RODS_SHAPE(CC, WW) \
  if (C == CC && W == WW) return launch_shape<T, CC, WW, false>(which, GT, a, n_blocks, st);
  RODS_SHAPE(2, 1)
  RODS_SHAPE(2, 2)
  RODS_SHAPE(2, 3)
  RODS_SHAPE(2, 4)
  RODS_SHAPE(2, 8)
  if constexpr (sizeof(T) == 4) {
    RODS_SHAPE(4, 1)
    RODS_SHAPE(4, 2)
    RODS_SHAPE(4, 4)
  }
#undef RODS_SHAPE
  return hipErrorInvalidValue;
}

// Rods with moving rigid bodies: two vertices per lane, no self-contact or
// twist.
template <typename T>
hipError_t launch_rods_bodies(int which, int C, int W, bool GT, const RodArgs<T>& a,
                              int n_blocks, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (C != 2 || !a.bw) return hipErrorInvalidValue;
  if (W == 1) return launch_shape<T, 2, 1, false, false, true>(which, GT, a, n_blocks, st);
  if (W == 2) return launch_shape<T, 2, 2, false, false, true>(which, GT, a, n_blocks, st);
  if (W == 4) return launch_shape<T, 2, 4, false, false, true>(which, GT, a, n_blocks, st);
  if (W == 8) return launch_shape<T, 2, 8, false, false, true>(which, GT, a, n_blocks, st);
  return hipErrorInvalidValue;
}

template <typename T>
size_t kernel_lds_bytes(int which, int C, int W, bool SC, bool GT, int n_iters) {
  size_t xb = W > 1 ? 2 * W * XK * sizeof(T) : 0;
  if (SC) return sc_lds_bytes<T>(C, W);
  if (which == 2 && !GT) return xb + (size_t)n_iters * C * PROJ_TAPE * 64 * W * sizeof(T);
  return xb;
}

template <typename T>
hipError_t launch_init_frames(const int32_t* voff, int R, const T* x, T* d1, hipStream_t st) {
  hipLaunchKernelGGL(k_init_frames<T>, dim3((R + 63) / 64), dim3(64), 0, st, voff, R, x, d1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init_frames_vjp(const int32_t* voff, int R, const T* x, const T* d1b, T* tmp,
                                  T* xb, hipStream_t st) {
  hipLaunchKernelGGL(k_init_frames_vjp<T>, dim3((R + 63) / 64), dim3(64), 0, st, voff, R, x, d1b,
                     tmp, xb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_curvature(const int32_t* voff, const int32_t* rod_of, int V, const T* x,
                            const T* d1, T* kappa, hipStream_t st) {
  hipLaunchKernelGGL(k_curvature<T>, dim3((V + 255) / 256), dim3(256), 0, st, voff, rod_of, V, x,
                     d1, kappa);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce_params(const int32_t* voff, int R, const double* ab, const double* as,
                                T* db, T* ds, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_params<T>, dim3((R + 63) / 64), dim3(64), 0, st, voff, R, ab, as,
                     db, ds);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* p, int64_t n, T val, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, val);
  return hipGetLastError();
}

hipError_t launch_selftest_exchange(int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_selftest_exchange, dim3(1), dim3(64), 0, st, out);
  return hipGetLastError();
}

#define RODS_INST(T)                                                                          \
  template hipError_t launch_rods<T>(int, int, int, bool, bool, const RodArgs<T>&, int,       \
                                     hipStream_t);                                            \
  template hipError_t launch_rods_bodies<T>(int, int, int, bool, const RodArgs<T>&, int,      \
                                            hipStream_t);                                     \
  template size_t kernel_lds_bytes<T>(int, int, int, bool, bool, int);                         \
  template hipError_t launch_init_frames<T>(const int32_t*, int, const T*, T*, hipStream_t);  \
  template hipError_t launch_init_frames_vjp<T>(const int32_t*, int, const T*, const T*, T*, T*, \
                                                hipStream_t);                                 \
  template hipError_t launch_curvature<T>(const int32_t*, const int32_t*, int, const T*,      \
                                          const T*, T*, hipStream_t);                         \
  template hipError_t launch_reduce_params<T>(const int32_t*, int, const double*,             \
                                              const double*, T*, T*, hipStream_t);            \
  template hipError_t launch_fill<T>(T*, int64_t, T, hipStream_t);                             \

RODS_INST(float)
RODS_INST(double)
template hipError_t launch_fill<int32_t>(int32_t*, int64_t, int32_t, hipStream_t);
#endif

}  // namespace rods
