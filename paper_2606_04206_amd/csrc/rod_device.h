// Device-side helpers: 3-vectors, lane exchange inside a rod's team of
// lanes, and the kernel argument block.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rods {

template <typename T>
struct V3 {
  T x, y, z;
};

template <typename T>
__device__ __forceinline__ V3<T> mk(T a, T b, T c) { return V3<T>{a, b, c}; }
template <typename T>
__device__ __forceinline__ V3<T> zero3() { return V3<T>{T(0), T(0), T(0)}; }
template <typename T>
__device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a) { return {-a.x, -a.y, -a.z}; }
template <typename T>
__device__ __forceinline__ V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename T>
__device__ __forceinline__ V3<T>& operator+=(V3<T>& a, V3<T> b) { a.x += b.x; a.y += b.y; a.z += b.z; return a; }
template <typename T>
__device__ __forceinline__ V3<T>& operator-=(V3<T>& a, V3<T> b) { a.x -= b.x; a.y -= b.y; a.z -= b.z; return a; }
template <typename T>
__device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Reciprocal, quotient and square root.  FP32 uses the hardware
// instructions (v_rcp_f32, v_sqrt_f32: about 1 ulp) instead of the correctly
// rounded multi-instruction sequences; FP64 keeps IEEE division and sqrt.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) { return 1.0 / sqrt(x); }
template <typename T>
__device__ __forceinline__ T fdiv(T a, T b) { return a * frcp(b); }

// four values stored as one vector access (LDS or global)
template <typename T>
struct alignas(4 * sizeof(T)) Q4 {
  T x, y, z, w;
};
constexpr int PROJ_TAPE = 4;   // values per edge and iteration in the projection tape

// ---------------------------------------------------------------------------
// Lane exchange.  A rod is owned by a team of 64*W lanes (W waves of one
// workgroup); team lane l holds vertices l*C .. l*C+C-1.  Inside a wave the
// neighbour exchange is a DPP wavefront shift (a VALU move, no LDS); at a
// wave boundary the value goes through a small ping-pong LDS buffer with one
// barrier per exchange group.  Every exchange must be reached by all lanes
// of the workgroup (uniform control flow).
// ---------------------------------------------------------------------------

__device__ __forceinline__ int dpp_from_next_i(int v) {
  // wave_shl:1 -- lane i receives lane i+1; lane 63 receives 0 (bound_ctrl)
  return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ int dpp_from_prev_i(int v) {
  // wave_shr:1 -- lane i receives lane i-1; lane 0 receives 0 (bound_ctrl)
  return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ float dpp_from_next(float v) {
  return __int_as_float(dpp_from_next_i(__float_as_int(v)));
}
__device__ __forceinline__ float dpp_from_prev(float v) {
  return __int_as_float(dpp_from_prev_i(__float_as_int(v)));
}
__device__ __forceinline__ double dpp_from_next(double v) {
  long long b = __double_as_longlong(v);
  int lo = dpp_from_next_i((int)(b & 0xffffffffLL));
  int hi = dpp_from_next_i((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double dpp_from_prev(double v) {
  long long b = __double_as_longlong(v);
  int lo = dpp_from_prev_i((int)(b & 0xffffffffLL));
  int hi = dpp_from_prev_i((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave, the same value in every lane: within
// each row of 16 lanes a DPP shift-and-add chain (row_shr 1, 2, 4, 8; lanes
// shifted in from outside the row read 0) leaves the row's sum in its last
// lane, and the four row sums, read out with readlane, are added in row
// order.  No LDS, no cross-lane permute through the LDS crossbar.
__device__ __forceinline__ float dpp_row_shr(float v, int n) {
  int i = __float_as_int(v);
  switch (n) {
    case 1: i = __builtin_amdgcn_mov_dpp(i, 0x111, 0xf, 0xf, true); break;
    case 2: i = __builtin_amdgcn_mov_dpp(i, 0x112, 0xf, 0xf, true); break;
    case 4: i = __builtin_amdgcn_mov_dpp(i, 0x114, 0xf, 0xf, true); break;
    default: i = __builtin_amdgcn_mov_dpp(i, 0x118, 0xf, 0xf, true); break;
  }
  return __int_as_float(i);
}
__device__ __forceinline__ double dpp_row_shr(double v, int n) {
  long long b = __double_as_longlong(v);
  float lo = dpp_row_shr(__int_as_float((int)(b & 0xffffffffLL)), n);
  float hi = dpp_row_shr(__int_as_float((int)(b >> 32)), n);
  return __longlong_as_double(((long long)__float_as_int(hi) << 32) |
                              (unsigned int)__float_as_int(lo));
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp_row_shr(v, 1);
  v += dpp_row_shr(v, 2);
  v += dpp_row_shr(v, 4);
  v += dpp_row_shr(v, 8);
  return (read_lane(v, 15) + read_lane(v, 31)) + (read_lane(v, 47) + read_lane(v, 63));
}

// a product the compiler may not fuse into a following add (kept where a
// value must round exactly as it does when computed in another lane)
template <typename T>
__device__ __forceinline__ T mul_nc(T a, T b) {
#pragma clang fp contract(off)
  return a * b;
}

// slots for the active lanes of a wave whose pred holds: consecutive
// entries of the LDS counter *ctr in lane order, one atomic per wave (the
// leader's); -1 where pred is false
__device__ __forceinline__ int wave_alloc(int* ctr, bool pred) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return -1;
  const int rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  const int leader = __ffsll((unsigned long long)m) - 1;
  int base = 0;
  if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(ctr, __popcll(m));
  base = __shfl(base, leader, 64);
  return pred ? base + rank : -1;
}

constexpr int XK = 12;   // largest exchange group (values)
// moving rigid bodies: at most NB_MAX primitives on a rod with moving bodies;
// per primitive 9 values (centre, velocity, angular velocity)
constexpr int NB_MAX = 16;
constexpr int NB_VALS = 9;
template <typename T>
constexpr size_t body_lds_bytes() { return 2 * (size_t)NB_MAX * NB_VALS * sizeof(T); }

template <typename T, int W>
struct Team {
  T* buf;    // LDS: 2 (ping-pong) x W x XK values, only used when W > 1
  int pp;
  int wave, lane;

  __device__ void init(T* lds) {
    buf = lds;
    pp = 0;
    wave = threadIdx.x >> 6;
    lane = threadIdx.x & 63;
  }
  // v[k] <- value of team lane + 1 (0 past the team's end)
  template <int K>
  __device__ __forceinline__ void next(T (&v)[K]) {
    T r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = dpp_from_next(v[k]);
    if constexpr (W > 1) {
      T* b = buf + pp * (W * XK);
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) b[wave * XK + k] = v[k];
      }
      __syncthreads();
      if (lane == 63 && wave + 1 < W) {
#pragma unroll
        for (int k = 0; k < K; ++k) r[k] = b[(wave + 1) * XK + k];
      }
      pp ^= 1;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = r[k];
  }
  // v[k] <- value of team lane - 1 (0 before the team's start)
  template <int K>
  __device__ __forceinline__ void prev(T (&v)[K]) {
    T r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = dpp_from_prev(v[k]);
    if constexpr (W > 1) {
      T* b = buf + pp * (W * XK);
      if (lane == 63) {
#pragma unroll
        for (int k = 0; k < K; ++k) b[wave * XK + k] = v[k];
      }
      __syncthreads();
      if (lane == 0 && wave > 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) r[k] = b[(wave - 1) * XK + k];
      }
      pp ^= 1;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = r[k];
  }
  // both directions with one barrier: a[k] <- a[k] of team lane - 1 (0
  // before the team's start), b[k] <- b[k] of team lane + 1 (0 past its end)
  template <int KA, int KB>
  __device__ __forceinline__ void swap(T (&a)[KA], T (&b)[KB]) {
    static_assert(KA + KB <= XK, "exchange group too large");
    T ra[KA], rb[KB];
#pragma unroll
    for (int k = 0; k < KA; ++k) ra[k] = dpp_from_prev(a[k]);
#pragma unroll
    for (int k = 0; k < KB; ++k) rb[k] = dpp_from_next(b[k]);
    if constexpr (W > 1) {
      T* buf2 = buf + pp * (W * XK);
      if (lane == 63) {
#pragma unroll
        for (int k = 0; k < KA; ++k) buf2[wave * XK + k] = a[k];
      }
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < KB; ++k) buf2[wave * XK + KA + k] = b[k];
      }
      __syncthreads();
      if (lane == 0 && wave > 0) {
#pragma unroll
        for (int k = 0; k < KA; ++k) ra[k] = buf2[(wave - 1) * XK + k];
      }
      if (lane == 63 && wave + 1 < W) {
#pragma unroll
        for (int k = 0; k < KB; ++k) rb[k] = buf2[(wave + 1) * XK + KA + k];
      }
      pp ^= 1;
    }
#pragma unroll
    for (int k = 0; k < KA; ++k) a[k] = ra[k];
#pragma unroll
    for (int k = 0; k < KB; ++k) b[k] = rb[k];
  }
  // v[k] <- sum of v[k] over the team, in every lane (K <= XK): wave_sum in
  // each wave, then the W wave sums through LDS in wave order, so every
  // lane holds the same sum.
  template <int K>
  __device__ __forceinline__ void sum(T (&v)[K]) {
    static_assert(K <= XK, "exchange group too large");
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if constexpr (W > 1) {
      T* b = buf + pp * (W * XK);
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) b[wave * XK + k] = v[k];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < K; ++k) {
        T s = b[k];
        for (int q = 1; q < W; ++q) s += b[q * XK + k];
        v[k] = s;
      }
      pp ^= 1;
    }
  }
};

template <typename T>
__device__ __forceinline__ void put3(T* a, int o, V3<T> v) { a[o] = v.x; a[o + 1] = v.y; a[o + 2] = v.z; }
template <typename T>
__device__ __forceinline__ V3<T> get3(const T* a, int o) { return V3<T>{a[o], a[o + 1], a[o + 2]}; }

// ---------------------------------------------------------------------------
// Kernel arguments (one block passed by value)
// ---------------------------------------------------------------------------
template <typename T>
struct RodArgs {
  // topology and work list
  const int32_t* voff;      // [R+1]
  const int32_t* rods;      // rods of this launch, blockIdx.x -> rod
  const int64_t* tape_off;  // [R] offset of the rod's block inside one tape slice
  // per-rod parameters
  const T* b;
  const T* sigma;
  const T* rc;
  const T* mu;
  const T* restit;
  const T* K;
  const int32_t* flags;
  // per-vertex statics (CSR rows)
  const T* w;               // inverse mass, 0 for pinned and grasped vertices
  const T* rest;            // rest length of edge row j
  const T* radius;
  const int32_t* gslot;     // grasp slot of the vertex or -1
  // rigid primitives
  const int32_t* prim_off;  // [R+1]
  const int32_t* prim_type;
  const T* prim_a;          // [P][3]
  const T* prim_b;          // [P][3]
  const T* prim_r;          // [P]
  // state (read at start, written at end)
  T* x;
  T* v;
  T* kb;
  T* d1;
  // optional copy of the final state (checkpoint)
  T* ck_x;
  T* ck_v;
  T* ck_kb;
  T* ck_d1;
  // substep tape: substep-start states of the launch's steps
  T* tape;
  int64_t tape_stride;      // values per tape slice (one substep, all rods)
  // actions
  const T* u;               // action a of rod r, slot g at u[a*act_stride + (r*G+g)*3]
  int64_t act_stride;
  int32_t G;
  int32_t spa;              // steps per action
  int32_t step_off;         // global index of the launch's first step
  // adjoint state and outputs
  T* lx;
  T* lv;
  T* lkb;
  T* ld1;
  T* dL_du;
  double* acc_b;            // [V] per-vertex dL/db partials
  double* acc_s;            // [V] per-vertex dL/dsigma partials
  T* sc_tape;               // self-contact rods: projection iterates of one substep
  const int64_t* sc_off;    // [R] offset of the rod's block in sc_tape
  unsigned char* pblk;      // self-contact rods: pair scratch (bytes)
  const int64_t* pblk_off;  // [R] byte offset of the rod's pair block
  unsigned long long* sc_stats;  // self-contact work counters, [R][8] (nullable): pair-
                            // substeps, superset tests, superset builds, active
                            // pair-passes, pairs in friction
  int32_t sc_lds;           // self-contact launches: dynamic LDS bytes (the host's
                            // offer; the launch sets the amount it allocates)
  uint32_t* branch;         // [V] (nullable) discrete decisions of each vertex's last
                            // forward substep: bit0 yield, bit 1 + k rigid contact
                            // with primitive k of the rod (k < 15), bits 16-23 the
                            // active self-contact pairs at the vertex in the first
                            // projection pass (at most 255)
  int32_t* status;          // [R] bit0 non-finite, bit1 pair bookkeeping fault, bit2 stretched edge
  // twist degree of freedom (rods with the twist flag; edge rows)
  const T* Gt;              // [R] twisting modulus
  const T* jt;              // [V] inverse polar moment of inertia of edge row j
  T* th;                    // [V] twist angle (state)
  T* om;                    // [V] twist rate (state)
  T* ck_th;
  T* ck_om;
  T* lth;                   // adjoints of theta and its rate
  T* lom;
  // moving rigid bodies (sphere primitives with inverse mass > 0); bw null:
  // every primitive is static
  const T* bw;              // [P] inverse mass, 0 for static primitives
  const T* bii;             // [P] inverse moment of inertia (isotropic)
  T* body;                  // [P][9] centre, velocity, angular velocity (state)
  T* ck_body;               // optional copy of the final body state (checkpoint)
  T* btape;                 // substep-start body states, [substep][P][9]
  T* lbody;                 // [P][9] adjoint of the body state
  int64_t bstride;          // values per body-tape slice (P * 9)
  int32_t body_lds;         // byte offset of the team's body block in dynamic LDS
  // scalars
  T h;
  T gx, gy, gz;
  T eps_s, f_thresh, self_margin;
  int32_t n_sub, n_iters, n_steps, k_ex;
};

}  // namespace rods
