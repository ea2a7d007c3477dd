// Self-contact and self-friction of one rod (DLO-Lab App. A.1,
// "Self-collision and Friction") for the rod kernels: closest points of two
// segments (clamped segment-segment method, Ericson 5.1.9, with a parallel
// fallback), the per-pair position correction and velocity friction, and
// their vector-Jacobian products.  Pairs are always evaluated with the
// lower-indexed edge first, so the candidate test gives the same answer
// whichever of the two edges searches for the other.
//
// Also the layout of a rod's block of pair scratch in global memory, shared
// by the host (which sizes it) and the kernels.
#pragma once
#include "rod_device.h"

namespace rods {

// hash buckets of the broadphase grid: G groups of 27 keys, the table
// padded to a multiple of the team size (sc_groups, sc_table)
__host__ __device__ constexpr int sc_groups(int tsize, int nv) { return tsize == 4 && nv >= 512 ? 256 : 64; }
__host__ __device__ constexpr int sc_table(int tsize, int nv, int tl) {
  return (27 * sc_groups(tsize, nv) + tl - 1) / tl * tl;
}

// one candidate pair, lower edge first (edge indices of a self-contact
// rod, at most 1023, fit 16 bits)
struct alignas(4) SPair {
  short lo, hi;
};

// values per pair of the per-pair records, in two halves: the lower edge's
// half at the pair's place in the list, the upper edge's half at the pair's
// place in upper-edge order, so each edge gathers both kinds from contiguous
// runs.  Forward kernels 2 x 5 (k n, the edge's closest-point parameter s
// or u, the reciprocal divisor); the adjoint 2 x 6 (the adjoints of the
// edge's two vertices)
constexpr int SC_RV_FWD = 10, SC_RV_ADJ = 12;
static_assert(SC_RV_ADJ / 2 == 6 && SC_RV_ADJ / 2 >= SC_RV_FWD / 2,
              "the adjoint's record halves hold six values and a forward half");

// Largest number of admissible pairs (j - i > k_ex) among the n - 1 edges of
// a rod of n vertices: the pair scratch has room for all of them, so no
// candidate is ever dropped.  Edge e has at most cap_lo(e) = max(0, M - e)
// partners above it and cap_hi(e) = max(0, e - k_ex) below it, M = n-2-k_ex.
__host__ __device__ inline int64_t sc_pair_cap(int n, int k_ex) {
  const int64_t M = (int64_t)n - 2 - k_ex;
  return M > 0 ? M * (M + 1) / 2 : 0;
}
__host__ __device__ inline int64_t sc_off_lo(int64_t e, int64_t M) {
  if (M <= 0) return 0;
  return e <= M ? e * M - e * (e - 1) / 2 : M * (M + 1) / 2;
}
__host__ __device__ inline int64_t sc_off_hi(int64_t e, int64_t k_ex) {
  return e <= k_ex + 1 ? 0 : (e - 1 - k_ex) * (e - k_ex) / 2;
}

// byte offsets inside a rod's pair block (each section 256-byte aligned):
// the count of the current substep's pairs; for the superset of a neighbour
// list, the partners found by each edge above it (trilo, triangular per-edge
// slots), the compact superset (sup, sorted by lower and then upper edge),
// per edge the sorted superset indices of the pairs it is the upper edge of
// (suphi), and each superset pair's place in the substep's list or -1
// (cidx); the substep's compact pair list (sorted likewise), each pair's
// place in upper-edge order (hpos), the first-pass depths d0, their
// adjoints d0b, rv values of per-pair records, and (the adjoint's blocks,
// rv = SC_RV_ADJ) 12 more per pair for the position adjoints of friction
struct PairBlock {
  int64_t trilo, sup, suphi, cidx, pairs, hpos, d0, d0b, rec, rec2, bytes;
};
__host__ __device__ inline int64_t sc_align(int64_t b) { return (b + 255) / 256 * 256; }
__host__ __device__ inline PairBlock sc_block(int n, int k_ex, int tsize, int rv) {
  const int64_t P = sc_pair_cap(n, k_ex);
  PairBlock b;
  int64_t o = 256;
  b.trilo = o; o = sc_align(o + 4 * P);
  b.sup = o;   o = sc_align(o + 4 * P);
  b.suphi = o; o = sc_align(o + 4 * P);
  b.cidx = o;  o = sc_align(o + 4 * P);
  b.pairs = o; o = sc_align(o + 4 * P);
  b.hpos = o;  o = sc_align(o + 4 * P);
  b.d0 = o;    o = sc_align(o + (int64_t)tsize * P);
  b.d0b = o;   o = sc_align(o + (int64_t)tsize * P);
  b.rec = o;   o = sc_align(o + (int64_t)tsize * rv * P);
  b.rec2 = o;  o = sc_align(o + (rv == SC_RV_ADJ ? (int64_t)tsize * 12 * P : 0));
  b.bytes = o;
  return b;
}

template <typename T>
struct Closest {
  T s, u;
  bool gen, s_cl, lo, hi, s_alt_cl;
};

template <typename T>
__device__ __forceinline__ T clamp01(T x) { return x < T(0) ? T(0) : (x > T(1) ? T(1) : x); }

template <typename T>
__device__ __forceinline__ Closest<T> closest_params(V3<T> P1, V3<T> Q1, V3<T> P2, V3<T> Q2) {
  V3<T> d1 = Q1 - P1, d2 = Q2 - P2, r = P1 - P2;
  T a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r), c = dot(d1, r), b = dot(d1, d2);
  T denom = a * e - b * b;
  Closest<T> o;
  o.gen = denom > T(1e-12) * (a * e);
  T s_raw = o.gen ? fdiv(b * f - c * e, denom) : T(0);
  T s0 = clamp01(s_raw);
  o.s_cl = !o.gen || s_raw <= T(0) || s_raw >= T(1);
  T u_raw = fdiv(b * s0 + f, e);
  o.lo = u_raw < T(0);
  o.hi = u_raw > T(1);
  o.u = o.lo ? T(0) : (o.hi ? T(1) : u_raw);
  T s_alt_raw = o.lo ? fdiv(-c, a) : fdiv(b - c, a);
  o.s_alt_cl = s_alt_raw <= T(0) || s_alt_raw >= T(1);
  o.s = (o.lo || o.hi) ? clamp01(s_alt_raw) : s0;
  return o;
}

// Adjoint of closest_params on the recorded branch; adds to the endpoint adjoints.
template <typename T>
__device__ __forceinline__ void closest_params_vjp(V3<T> P1, V3<T> Q1, V3<T> P2, V3<T> Q2,
                                                   const Closest<T>& br, T s_b, T u_b,
                                                   V3<T>& P1b, V3<T>& Q1b, V3<T>& P2b,
                                                   V3<T>& Q2b) {
  V3<T> d1 = Q1 - P1, d2 = Q2 - P2, r = P1 - P2;
  T a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r), c = dot(d1, r), b = dot(d1, d2);
  T denom = a * e - b * b;
  T a_b = 0, b_b = 0, c_b = 0, e_b = 0, f_b = 0;
  bool uc = br.lo || br.hi;
  T s_alt_b = (uc && !br.s_alt_cl) ? s_b : T(0);
  T num = br.lo ? -c : b - c;
  const T ia = frcp(a);
  c_b += -s_alt_b * ia;
  if (br.hi) b_b += s_alt_b * ia;
  a_b += -s_alt_b * num * ia * ia;
  T dn = br.gen ? denom : T(1);
  const T idn = frcp(dn);
  T s_raw = br.gen ? (b * f - c * e) * idn : T(0);
  T s0 = clamp01(s_raw);
  T u_raw_b = uc ? T(0) : u_b;
  const T ie = frcp(e);
  b_b += u_raw_b * s0 * ie;
  f_b += u_raw_b * ie;
  e_b += -u_raw_b * (b * s0 + f) * ie * ie;
  T s0_b = u_raw_b * b * ie + (uc ? T(0) : s_b);
  T sr_b = br.s_cl ? T(0) : s0_b;
  b_b += sr_b * f * idn;
  f_b += sr_b * b * idn;
  c_b += -sr_b * e * idn;
  e_b += -sr_b * c * idn;
  T dn_b = -sr_b * s_raw * idn;
  a_b += dn_b * e;
  e_b += dn_b * a;
  b_b += T(-2) * dn_b * b;
  V3<T> d1_b = (T(2) * a_b) * d1 + c_b * r + b_b * d2;
  V3<T> d2_b = (T(2) * e_b) * d2 + f_b * r + b_b * d1;
  V3<T> r_b = f_b * d2 + c_b * d1;
  P1b += r_b - d1_b;
  Q1b += d1_b;
  P2b -= d2_b + r_b;
  Q2b += d2_b;
}

// Geometry of one pair (edge i = P1-Q1 before edge j = P2-Q2).
template <typename T>
struct PairGeo {
  Closest<T> cp;
  V3<T> diff, n;
  T dist, d, W, ra, rb;
  bool act;
};

template <typename T>
__device__ __forceinline__ PairGeo<T> pair_geo(V3<T> P1, V3<T> Q1, V3<T> P2, V3<T> Q2, T wi,
                                               T wi1, T wj, T wj1, T ri, T ri1, T rj, T rj1) {
  PairGeo<T> g;
  g.cp = closest_params(P1, Q1, P2, Q2);
  T s = g.cp.s, u = g.cp.u;
  V3<T> ca = (T(1) - s) * P1 + s * Q1;
  V3<T> cb = (T(1) - u) * P2 + u * Q2;
  g.ra = (T(1) - s) * ri + s * ri1;
  g.rb = (T(1) - u) * rj + u * rj1;
  g.W = wi * (T(1) - s) * (T(1) - s) + wi1 * s * s + wj * (T(1) - u) * (T(1) - u) + wj1 * u * u;
  g.diff = ca - cb;
  g.dist = fsqrt(dot(g.diff, g.diff));
  g.d = g.ra + g.rb - g.dist;
  g.act = g.d > T(0) && g.dist > T(1e-12) && g.W > T(0);
  g.n = frcp(g.act ? g.dist : T(1)) * g.diff;
  return g;
}

// Adjoint of the four corrections of an active pair given the adjoints gi,
// gi1, gj, gj1 of the pass outputs of its four vertices; returns the
// contributions to the adjoints of the pass inputs.
template <typename T>
__device__ __forceinline__ void pair_proj_vjp(V3<T> P1, V3<T> Q1, V3<T> P2, V3<T> Q2,
                                              const PairGeo<T>& g, T wi, T wi1, T wj, T wj1,
                                              T ri, T ri1, T rj, T rj1, V3<T> gi, V3<T> gi1,
                                              V3<T> gj, V3<T> gj1, V3<T>& P1b, V3<T>& Q1b,
                                              V3<T>& P2b, V3<T>& Q2b) {
  T s = g.cp.s, u = g.cp.u;
  V3<T> n = g.n;
  T kk = fdiv(g.d, g.W);
  T ni = dot(gi, n), ni1 = dot(gi1, n), nj = dot(gj, n), nj1 = dot(gj1, n);
  T kk_b = wi * (T(1) - s) * ni + wi1 * s * ni1 - wj * (T(1) - u) * nj - wj1 * u * nj1;
  V3<T> n_b = (kk * wi * (T(1) - s)) * gi + (kk * wi1 * s) * gi1 - (kk * wj * (T(1) - u)) * gj -
              (kk * wj1 * u) * gj1;
  T s_b = kk * (-wi * ni + wi1 * ni1);
  T u_b = kk * (wj * nj - wj1 * nj1);
  const T iW = frcp(g.W);
  T d_b = kk_b * iW;
  T W_b = -kk_b * g.d * iW * iW;
  s_b += W_b * (T(-2) * wi * (T(1) - s) + T(2) * wi1 * s);
  u_b += W_b * (T(-2) * wj * (T(1) - u) + T(2) * wj1 * u);
  V3<T> diff_b = frcp(g.dist) * (n_b - dot(n, n_b) * n) - d_b * n;
  s_b += d_b * (ri1 - ri);
  u_b += d_b * (rj1 - rj);
  s_b += dot(diff_b, Q1 - P1);
  u_b -= dot(diff_b, Q2 - P2);
  P1b += (T(1) - s) * diff_b;
  Q1b += s * diff_b;
  P2b -= (T(1) - u) * diff_b;
  Q2b -= u * diff_b;
  closest_params_vjp(P1, Q1, P2, Q2, g.cp, s_b, u_b, P1b, Q1b, P2b, Q2b);
}

// Adjoint of the first-pass depth d of an active pair w.r.t. its inputs.
template <typename T>
__device__ __forceinline__ void pair_depth_vjp(V3<T> P1, V3<T> Q1, V3<T> P2, V3<T> Q2,
                                               const PairGeo<T>& g, T ri, T ri1, T rj, T rj1,
                                               T d_b, V3<T>& P1b, V3<T>& Q1b, V3<T>& P2b,
                                               V3<T>& Q2b) {
  T s = g.cp.s, u = g.cp.u;
  T s_b = d_b * (ri1 - ri);
  T u_b = d_b * (rj1 - rj);
  V3<T> diff_b = (-d_b) * g.n;
  s_b += dot(diff_b, Q1 - P1);
  u_b -= dot(diff_b, Q2 - P2);
  P1b += (T(1) - s) * diff_b;
  Q1b += s * diff_b;
  P2b -= (T(1) - u) * diff_b;
  Q2b -= u * diff_b;
  closest_params_vjp(P1, Q1, P2, Q2, g.cp, s_b, u_b, P1b, Q1b, P2b, Q2b);
}

// Friction of one pair at final positions; velocities vi.. of the four
// vertices; writes the velocity changes of the four vertices.
template <typename T>
struct FricGeo {
  PairGeo<T> g;
  V3<T> vrel, vt, dvt;
  T vn, vtn, ratio, scale;
  bool ok, slide;
};

template <typename T>
__device__ __forceinline__ FricGeo<T> pair_friction(V3<T> P1, V3<T> Q1, V3<T> P2, V3<T> Q2,
                                                    V3<T> vi, V3<T> vi1, V3<T> vj, V3<T> vj1,
                                                    T wi, T wi1, T wj, T wj1, T ri, T ri1, T rj,
                                                    T rj1, T d0, T mu, T h) {
  FricGeo<T> f;
  f.g = pair_geo(P1, Q1, P2, Q2, wi, wi1, wj, wj1, ri, ri1, rj, rj1);
  T s = f.g.cp.s, u = f.g.cp.u;
  f.ok = f.g.dist > T(1e-12) && f.g.W > T(0);
  f.g.n = frcp(f.ok ? f.g.dist : T(1)) * f.g.diff;
  f.vrel = (T(1) - s) * vi + s * vi1 - (T(1) - u) * vj - u * vj1;
  f.vn = dot(f.vrel, f.g.n);
  f.vt = f.vrel - f.vn * f.g.n;
  T vtn = fsqrt(dot(f.vt, f.vt));
  f.ok = f.ok && vtn > T(0);
  f.vtn = f.ok ? vtn : T(1);
  f.ratio = fdiv(mu * d0, h * f.vtn);
  f.slide = f.ratio < T(1);
  f.scale = f.ok ? (f.slide ? f.ratio : T(1)) : T(0);
  f.dvt = (-f.scale) * f.vt;
  return f;
}

// Adjoint of a pair's friction given the adjoints of the four velocity
// outputs (gi..): adds to the adjoints of the four input velocities, of the
// four positions, and returns the adjoint of d0.
template <typename T>
__device__ __forceinline__ T pair_friction_vjp(V3<T> P1, V3<T> Q1, V3<T> P2, V3<T> Q2, V3<T> vi,
                                               V3<T> vi1, V3<T> vj, V3<T> vj1,
                                               const FricGeo<T>& f, T wi, T wi1, T wj, T wj1,
                                               T mu, T h, V3<T> gi, V3<T> gi1, V3<T> gj,
                                               V3<T> gj1, V3<T>& vib, V3<T>& vi1b, V3<T>& vjb,
                                               V3<T>& vj1b, V3<T>& P1b, V3<T>& Q1b, V3<T>& P2b,
                                               V3<T>& Q2b) {
  if (!f.ok) return T(0);
  T s = f.g.cp.s, u = f.g.cp.u;
  T W = f.g.W;
  V3<T> n = f.g.n;
  T ci = wi * (T(1) - s), ci1 = wi1 * s, cj = -wj * (T(1) - u), cj1 = -wj1 * u;
  V3<T> G = ci * gi + ci1 * gi1 + cj * gj + cj1 * gj1;
  const T iW = frcp(W);
  V3<T> dvt_b = iW * G;
  T W_b = -dot(G, f.dvt) * iW * iW;
  T s_b = (-wi * dot(gi, f.dvt) + wi1 * dot(gi1, f.dvt)) * iW;
  T u_b = (wj * dot(gj, f.dvt) - wj1 * dot(gj1, f.dvt)) * iW;
  T scale_b = -dot(dvt_b, f.vt);
  V3<T> vt_b = (-f.scale) * dvt_b;
  T d0_b = T(0);
  if (f.slide) {
    const T iv = frcp(f.vtn);
    d0_b = fdiv(scale_b * mu, h) * iv;
    T vtn_b = -scale_b * f.ratio * iv;
    vt_b += (vtn_b * iv) * f.vt;
  }
  V3<T> vrel_b = vt_b - dot(n, vt_b) * n;
  V3<T> n_b = -(f.vn * vt_b + dot(vt_b, n) * f.vrel);
  s_b += dot(vrel_b, vi1 - vi);
  u_b -= dot(vrel_b, vj1 - vj);
  vib += (T(1) - s) * vrel_b;
  vi1b += s * vrel_b;
  vjb -= (T(1) - u) * vrel_b;
  vj1b -= u * vrel_b;
  s_b += W_b * (T(-2) * wi * (T(1) - s) + T(2) * wi1 * s);
  u_b += W_b * (T(-2) * wj * (T(1) - u) + T(2) * wj1 * u);
  V3<T> diff_b = frcp(f.g.dist) * (n_b - dot(n, n_b) * n);
  s_b += dot(diff_b, Q1 - P1);
  u_b -= dot(diff_b, Q2 - P2);
  P1b += (T(1) - s) * diff_b;
  Q1b += s * diff_b;
  P2b -= (T(1) - u) * diff_b;
  Q2b -= u * diff_b;
  closest_params_vjp(P1, Q1, P2, Q2, f.g.cp, s_b, u_b, P1b, Q1b, P2b, Q2b);
  return d0_b;
}

// Bucket of grid cell (ix, iy, iz): cells are grouped in blocks of 3x3x3;
// the cell's place in its block picks one of 27 residues and a
// multiplicative hash of the block one of G groups (a power of two).  Two
// cells of any 3x3x3 neighbourhood differ by at most 2 along every axis, so
// their residues (and keys) differ: a search over the 27 cells around a
// cell visits every bucket at most once and finds every edge at most once.
// Blocks that share a group share buckets, so more groups mean fewer
// unrelated edges in a search.  Coordinates are clamped to +-2^20 cells
// beforehand.
__device__ __forceinline__ int floor_div3(int i) { return i >= 0 ? i / 3 : -((2 - i) / 3); }
constexpr unsigned SC_H1 = 73856093u, SC_H2 = 19349663u, SC_H3 = 83492791u;
template <int G>
__device__ __forceinline__ int sc_key(int ix, int iy, int iz) {
  const int bx = floor_div3(ix), by = floor_div3(iy), bz = floor_div3(iz);
  const int res = (ix - 3 * bx) + 3 * (iy - 3 * by) + 9 * (iz - 3 * bz);
  const unsigned g = ((unsigned)bx * SC_H1 ^ (unsigned)by * SC_H2 ^ (unsigned)bz * SC_H3) &
                     (unsigned)(G - 1);
  return (int)g * 27 + res;
}
template <typename T>
__device__ __forceinline__ int sc_cell(T c) {
  const T lim = T(1 << 20);
  return (int)floor(fmin(fmax(c, -lim), lim));
}

}  // namespace rods
