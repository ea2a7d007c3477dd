// C ABI of the batched rod simulator: validation, device allocation (all of
// it in rods_create), size bins and work lists, and the drivers of the
// rollout (segment checkpoints) and of the checkpointed backward pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <tuple>
#include <type_traits>
#include <vector>

#include "rods.h"
#include "rod_launch.h"
#include "rod_selfcontact.h"

using rods::RodArgs;

namespace {

// values per vertex of a checkpointed state: x 3, v 3, kappa_bar 2, d1 3,
// theta, theta_dot (the last two only used by twisting rods)
constexpr int NF = 13;
// values per vertex slot of the backward tape
static int tape_fields(bool tw) { return tw ? 13 : 11; }

struct Bin {
  int C, W;       // vertices per lane, waves per rod
  int n, off;     // rods bin_rods[off .. off+n)
  bool sc;        // rods with self-contact
  bool gt;        // the adjoint keeps projection iterates in global scratch
  bool tw;        // rods with the twist degree of freedom
  bool bd;        // rods with moving rigid bodies
};

// self-contact kernels exist for these shapes (FP64: C = 2 only, which
// shapes_for already requires)
static bool sc_shape_ok(int C, int W) {
  return (C == 2 && (W == 1 || W == 2 || W == 4 || W == 8)) || (C == 4 && W == 4);
}

// three-wave teams exist for two vertices per lane on rods without
// self-contact, twist or moving bodies (257-384 vertices then fill three
// quarters of a four-wave team's SIMDs)
static bool w3_ok(int C, bool sc, bool tw) { return C == 2 && !sc && !tw; }

// legal launch shapes for a rod of n vertices, smallest team first
static std::vector<std::pair<int, int>> shapes_for(int n, int prec, bool sc = false,
                                                   bool tw = false) {
  std::vector<std::pair<int, int>> out;
  const int Cs[2] = {2, 4};
  const int Ws[5] = {1, 2, 3, 4, 8};
  for (int C : Cs) {
    if ((prec == 8 || tw) && C != 2) continue;
    for (int W : Ws) {
      if (sc && !sc_shape_ok(C, W)) continue;
      if (W == 3 && !w3_ok(C, sc, tw)) continue;
      if (64 * W * C >= n) {
        out.push_back({C, W});
        break;
      }
    }
  }
  return out;
}

struct HandleBase {
  virtual ~HandleBase() {}
};

#define HIPCHK(expr)                        \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return (int)ROD_EHIP; \
  } while (0)

template <typename T>
struct Impl : HandleBase {
  int R = 0, V = 0, G = 0, P = 0, prec = 4;
  RodsDesc d{};
  std::vector<int32_t> voff_h;
  int n_ck = 0, n_act_max = 0;
  int device = 0;

  std::vector<void*> allocs;
  int32_t *voff = nullptr, *rod_of = nullptr, *gslot = nullptr, *flags = nullptr,
          *prim_off = nullptr, *prim_type = nullptr, *status = nullptr, *bin_rods = nullptr;
  T *b = nullptr, *sigma = nullptr, *rc = nullptr, *mu = nullptr, *restit = nullptr, *K = nullptr;
  T *w = nullptr, *rest = nullptr, *radius = nullptr, *prim_a = nullptr, *prim_b = nullptr,
    *prim_r = nullptr;
  T *x = nullptr, *v = nullptr, *kb = nullptr, *d1 = nullptr;
  T *sx = nullptr, *sv = nullptr, *skb = nullptr, *sd1 = nullptr;
  // twist degree of freedom: modulus per rod, inverse edge inertia, angle
  // and rate (state, scratch copy, adjoints)
  T *Gt = nullptr, *jt = nullptr, *th = nullptr, *om = nullptr, *sth = nullptr, *som = nullptr,
    *lth = nullptr, *lom = nullptr;
  T* ck = nullptr;          // [n_ck][V*NF]
  // moving rigid bodies (has_bodies): inverse mass and inertia per
  // primitive, state [P][9] with a scratch copy for replays, checkpoints
  // [n_ck][P][9], the substep tape (two buffers, as the vertex tape), the
  // adjoint, its seed, and the optimiser's start state
  bool has_bodies = false;
  T *bwv = nullptr, *biiv = nullptr, *body = nullptr, *sbody = nullptr, *ck_body = nullptr,
    *btape = nullptr, *btape2 = nullptr, *lbody = nullptr, *bseed = nullptr, *body_opt0 = nullptr;
  std::vector<T> body_init_h;   // centres of the primitives, at rest
  T* ckb(int k) const { return ck_body + (size_t)k * P * rods::NB_VALS; }
  T* btape_for(T* vtape) const { return vtape == tape2 ? btape2 : btape; }
  T* acts = nullptr;        // recorded actions [n_act_max][R][G][3]
  T* du_scratch = nullptr;  // dL/du when the caller does not want it
  // optimisation driver: Adam moments of the grasp velocities and of log b,
  // log b itself, dL/db, the final positions, dL/dx_T and the loss
  T *opt_mU = nullptr, *opt_vU = nullptr, *opt_mb = nullptr, *opt_vb = nullptr,
    *opt_logb = nullptr, *opt_db = nullptr, *opt_xT = nullptr, *opt_g = nullptr,
    *opt_loss = nullptr;
  T* tape = nullptr;
  int64_t tape_stride = 0, tape_cap = 0;
  int64_t* tape_off = nullptr;
  T* sc_tape = nullptr;          // self-contact projection iterates (one substep per rod)
  int64_t* sc_off = nullptr;
  int64_t sc_cap = 0;
  // self-contact pair scratch: one block per rod for the forward kernels and
  // one for the adjoint (the pipelined backward runs both at once), each with
  // room for every admissible pair of the rod
  unsigned char *pblk_f = nullptr, *pblk_a = nullptr;
  int64_t *pblk_off_f = nullptr, *pblk_off_a = nullptr;
  std::vector<int64_t> pblk_off_h;
  // self-contact work counters [2][R][8] (forward kernels, adjoint)
  unsigned long long* sc_stats = nullptr;
  size_t lds_max = 65536;
  T *lx = nullptr, *lv = nullptr, *lkb = nullptr, *ld1 = nullptr;
  double *acc_b = nullptr, *acc_s = nullptr, *loss_part = nullptr;
  std::vector<Bin> bins;
  std::vector<int32_t> bin_rods_h;
  bool recorded = false;
  // number of the current recording (1, 2, ... for each recorded rollout;
  // 0 when there is none): lets a caller check that a backward reads the
  // rollout it means
  int64_t rec_gen = 0, rec_count = 0;
  int n_rec = 0;
  int plain = 0;
  bool concurrent_bins = true;
  // graph of one step (all size bins) over the handle's own buffers
  hipStream_t cap_stream = nullptr;
  // backward pipelining: the tape of segment s-1 is replayed on side_stream
  // into the other half of a double-buffered tape while the adjoint of
  // segment s runs on the caller's stream (tape2 == nullptr: no room, the
  // segments run one after the other)
  T* tape2 = nullptr;
  // the recorded rollout writes the tape of its last segment itself, so the
  // backward starts with that segment's adjoint (valid until the backward
  // reuses the buffer)
  bool last_tape_ok = false;
  T* tape_for(int seg) const { return (plain || !tape2) ? tape : ((seg & 1) ? tape2 : tape); }
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_tape[2] = {nullptr, nullptr}, ev_adj[2] = {nullptr, nullptr};
  // size bins after the first run on streams of their own (default
  // priority), forked from and joined back to the caller's stream, so that
  // one bin's last, partly filled round of workgroups overlaps the others
  std::vector<hipStream_t> bin_streams;
  std::vector<hipEvent_t> bin_done;
  hipEvent_t ev_fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  T* u_step = nullptr;
  // kernel timing: event pairs around every launch batch, per kernel kind
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_used;   // (kind, index of the first event of a pair)
  size_t ev_next = 0;

  ~Impl() override {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (side_stream) (void)hipStreamDestroy(side_stream);
    for (hipStream_t s : bin_streams) (void)hipStreamDestroy(s);
    for (hipEvent_t e : bin_done) (void)hipEventDestroy(e);
    for (hipEvent_t e : {ev_start, ev_tape[0], ev_tape[1], ev_adj[0], ev_adj[1], ev_fork})
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
  }

  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }

  // One step through a captured HIP graph: the action is copied into the
  // handle's own buffer (outside the graph), then the graph of the step's
  // kernel launches is replayed.
  int step_graph(const T* u, hipStream_t st) {
    recorded = false;
    if (G > 0) HIPCHK(hipMemcpyAsync(u_step, u, sizeof(T) * (size_t)R * G * 3,
                                     hipMemcpyDeviceToDevice, st));
    if (!graph_exec) {
      RodArgs<T> a = args(cap_stream);
      a.u = u_step;
      a.act_stride = 0;
      a.spa = 1;
      a.step_off = 0;
      a.n_steps = 1;
      HIPCHK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
      int e = launch_all_(0, a, cap_stream);
      hipGraph_t g = nullptr;
      hipError_t ce = hipStreamEndCapture(cap_stream, &g);
      if (e) {
        if (g) (void)hipGraphDestroy(g);
        return e;
      }
      HIPCHK(ce);
      graph = g;
      HIPCHK(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(graph_exec, st));
    return ROD_OK;
  }

  int set_profiling(int on) {
    profiling = on != 0;
    if (profiling && ev_pool.empty()) {
      ev_pool.resize(4096);
      for (auto& e : ev_pool) HIPCHK(hipEventCreate(&e));
    }
    ev_used.clear();
    ev_next = 0;
    return ROD_OK;
  }

  // out[3*k + 0] = total ms, out[3*k + 1] = launch batches, out[3*k + 2] = max ms,
  // for k = 0 forward, 1 forward writing the tape, 2 adjoint
  int profile(double* out, hipStream_t st) {
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < 9; ++i) out[i] = 0.0;
    for (auto& u : ev_used) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev_pool[u.second], ev_pool[u.second + 1]));
      out[3 * u.first] += ms;
      out[3 * u.first + 1] += 1.0;
      out[3 * u.first + 2] = std::max(out[3 * u.first + 2], (double)ms);
    }
    ev_used.clear();
    ev_next = 0;
    return ROD_OK;
  }

  template <typename U>
  int alloc(U*& p, size_t n) {
    void* q = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&q, n * sizeof(U)) != hipSuccess) return ROD_ENOMEM;
    allocs.push_back(q);
    p = static_cast<U*>(q);
    return ROD_OK;
  }
  template <typename U>
  int upload(U*& p, const std::vector<U>& h) {
    int rc_ = alloc(p, h.size());
    if (rc_) return rc_;
    if (!h.empty()) HIPCHK(hipMemcpy(p, h.data(), h.size() * sizeof(U), hipMemcpyHostToDevice));
    return ROD_OK;
  }

  T* ck_x(int k) const { return ck + (size_t)k * V * NF; }
  T* ck_v(int k) const { return ck_x(k) + (size_t)V * 3; }
  T* ck_kb(int k) const { return ck_x(k) + (size_t)V * 6; }
  T* ck_d1(int k) const { return ck_x(k) + (size_t)V * 8; }
  T* ck_th(int k) const { return ck_x(k) + (size_t)V * 11; }
  T* ck_om(int k) const { return ck_x(k) + (size_t)V * 12; }

  int create(const RodsDesc* dd) {
    d = *dd;
    R = d.n_rods;
    G = d.n_grasp;
    prec = d.precision;
    HIPCHK(hipGetDevice(&device));
    voff_h.assign(d.vert_offsets, d.vert_offsets + R + 1);
    V = voff_h[R];
    P = d.prim_offsets ? d.prim_offsets[R] : 0;
    // ---- per-vertex statics
    std::vector<T> w_h(V), rest_h(V), rad_h(V);
    std::vector<int32_t> gslot_h(V, -1), rod_of_h(V);
    for (int r = 0; r < R; ++r) {
      for (int i = voff_h[r]; i < voff_h[r + 1]; ++i) {
        rod_of_h[i] = r;
        w_h[i] = (T)d.inv_mass[i];
        rad_h[i] = (T)d.radius[i];
        rest_h[i] = (i < voff_h[r + 1] - 1) ? (T)d.rest_len[i] : T(0);
      }
      for (int g = 0; g < G; ++g) {
        int li = d.grasp_idx[r * G + g];
        if (li >= 0) {
          gslot_h[voff_h[r] + li] = g;
          w_h[voff_h[r] + li] = T(0);   // grasped vertices are kinematic
        }
      }
    }
    // ---- per-rod parameters
    std::vector<T> b_h(R), s_h(R), rc_h(R), mu_h(R), e_h(R), K_h(R), G_h(R);
    std::vector<int32_t> fl_h(R);
    for (int r = 0; r < R; ++r) {
      const double* p = d.rod_params + (size_t)r * ROD_NPARAM;
      fl_h[r] = (int32_t)p[ROD_P_FLAGS];
      K_h[r] = (T)p[ROD_P_K];
      b_h[r] = (T)p[ROD_P_B];
      s_h[r] = (T)p[ROD_P_SIGMA];
      rc_h[r] = (T)p[ROD_P_RC];
      mu_h[r] = (T)p[ROD_P_MU];
      e_h[r] = (T)p[ROD_P_REST];
      G_h[r] = (T)p[ROD_P_G];
    }
    // ---- inverse twist inertia per edge row (twisting rods only)
    std::vector<T> jt_h(V, T(0));
    for (int r = 0; r < R; ++r)
      if (fl_h[r] & ROD_FLAG_TWIST)
        for (int i = voff_h[r]; i < voff_h[r + 1] - 1; ++i) jt_h[i] = (T)d.twist_inv_inertia[i];
    // ---- primitives
    std::vector<int32_t> pt_h(P), po_h(R + 1, 0);
    std::vector<T> pa_h(3 * (size_t)P), pb_h(3 * (size_t)P), pr_h(P);
    if (d.prim_offsets) po_h.assign(d.prim_offsets, d.prim_offsets + R + 1);
    for (int k = 0; k < P; ++k) {
      pt_h[k] = d.prims[k].type;
      for (int c = 0; c < 3; ++c) {
        pa_h[3 * k + c] = (T)d.prims[k].a[c];
        pb_h[3 * k + c] = (T)d.prims[k].b[c];
      }
      pr_h[k] = (T)d.prims[k].radius;
    }
    std::vector<T> bw_h(P, T(0)), bii_h(P, T(0));
    body_init_h.assign((size_t)P * rods::NB_VALS, T(0));
    for (int k = 0; k < P; ++k) {
      for (int c = 0; c < 3; ++c) body_init_h[(size_t)k * rods::NB_VALS + c] = pa_h[3 * k + c];
      if (d.prim_inv_mass && d.prim_inv_mass[k] > 0) {
        has_bodies = true;
        bw_h[k] = (T)d.prim_inv_mass[k];
        bii_h[k] = (T)d.prim_inv_inertia[k];
      }
    }
    // ---- size bins: smallest legal team per rod, largest rods first
    {
      int attr = 0;
      if (hipDeviceGetAttribute(&attr, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
              hipSuccess && attr > 0)
        lds_max = (size_t)attr;
    }
    std::vector<std::vector<int>> members;
    std::vector<std::tuple<int, int, bool, bool, bool>> keys;
    for (int r = 0; r < R; ++r) {
      const bool sc = (fl_h[r] & ROD_FLAG_SELF) != 0;
      const bool tw = (fl_h[r] & ROD_FLAG_TWIST) != 0;
      bool bd = false;
      for (int k = po_h[r]; k < po_h[r + 1]; ++k) bd |= bw_h[k] > T(0);
      auto sh = shapes_for(voff_h[r + 1] - voff_h[r], prec, sc, tw || bd);
      if (sh.empty()) return ROD_EINVAL;
      auto key = std::make_tuple(sh.front().first, sh.front().second, sc, tw, bd);
      size_t k = 0;
      while (k < keys.size() && keys[k] != key) ++k;
      if (k == keys.size()) {
        keys.push_back(key);
        members.emplace_back();
      }
      members[k].push_back(r);
    }
    for (size_t k = 0; k < keys.size(); ++k) {
      auto& m = members[k];
      std::stable_sort(m.begin(), m.end(), [&](int a, int b2) {
        return (voff_h[a + 1] - voff_h[a]) > (voff_h[b2 + 1] - voff_h[b2]);
      });
      Bin bn{std::get<0>(keys[k]), std::get<1>(keys[k]), (int)m.size(), (int)bin_rods_h.size(),
             std::get<2>(keys[k]), false, std::get<3>(keys[k]), std::get<4>(keys[k])};
      bn.gt = global_tape(bn.C, bn.W, bn.sc);
      if (rods::kernel_lds_bytes<T>(2, bn.C, bn.W, bn.sc, bn.gt, d.n_iters) + body_lds() > lds_max)
        return ROD_EINVAL;
      bins.push_back(bn);
      for (int r : m) bin_rods_h.push_back(r);
    }
    std::vector<int64_t> toff_h, soff_h;
    layout_offsets(toff_h, soff_h);
    tape_cap = 2 * tape_stride;   // autotuned teams are at most twice the smallest legal one
    // scratch for the projection iterates: room for every rod at twice its
    // smallest team, whatever shapes the autotuner picks
    sc_cap = 0;
    for (const Bin& bn : bins)
      sc_cap += (int64_t)bn.n * 2 * scratch_per_rod(bn.C, bn.W);
    // pair scratch of the rods with self-contact (byte offsets per rod)
    std::vector<int64_t> pof_h(R, 0), poa_h(R, 0);
    int64_t pbytes_f = 0, pbytes_a = 0;
    for (int r = 0; r < R; ++r) {
      if (!(fl_h[r] & ROD_FLAG_SELF)) continue;
      const int n = voff_h[r + 1] - voff_h[r];
      pof_h[r] = pbytes_f;
      poa_h[r] = pbytes_a;
      pbytes_f += rods::sc_block(n, d.k_exclude, (int)sizeof(T), rods::SC_RV_FWD).bytes;
      pbytes_a += rods::sc_block(n, d.k_exclude, (int)sizeof(T), rods::SC_RV_ADJ).bytes;
    }
    pblk_off_h = pof_h;
    n_ck = std::max(1, (d.max_steps + d.ckpt_every - 1) / d.ckpt_every);
    n_act_max = std::max(1, (d.max_steps + d.steps_per_action - 1) / d.steps_per_action);

    int e;
    if ((e = upload(voff, voff_h)) || (e = upload(rod_of, rod_of_h)) || (e = upload(gslot, gslot_h)) ||
        (e = upload(flags, fl_h)) || (e = upload(prim_off, po_h)) || (e = upload(prim_type, pt_h)) ||
        (e = upload(b, b_h)) || (e = upload(sigma, s_h)) || (e = upload(rc, rc_h)) ||
        (e = upload(mu, mu_h)) || (e = upload(restit, e_h)) || (e = upload(K, K_h)) ||
        (e = upload(w, w_h)) || (e = upload(rest, rest_h)) || (e = upload(radius, rad_h)) ||
        (e = upload(Gt, G_h)) || (e = upload(jt, jt_h)) ||
        (e = upload(prim_a, pa_h)) || (e = upload(prim_b, pb_h)) || (e = upload(prim_r, pr_h)) ||
        (e = upload(bin_rods, bin_rods_h)) || (e = upload(tape_off, toff_h)) ||
        (e = upload(sc_off, soff_h)) || (e = alloc(sc_tape, (size_t)sc_cap)) ||
        (e = upload(pblk_off_f, pof_h)) || (e = upload(pblk_off_a, poa_h)) ||
        (e = alloc(pblk_f, (size_t)pbytes_f)) || (e = alloc(pblk_a, (size_t)pbytes_a)) ||
        (e = alloc(sc_stats, (size_t)16 * R)))
      return e;
    HIPCHK(hipMemset(sc_stats, 0, sizeof(unsigned long long) * 16 * R));
    for (int r = 0; r < R; ++r)   // pair counts read 0 until a step has run
      if (fl_h[r] & ROD_FLAG_SELF) HIPCHK(hipMemset(pblk_f + pof_h[r], 0, sizeof(int32_t)));
    if ((e = alloc(x, 3 * (size_t)V)) || (e = alloc(v, 3 * (size_t)V)) ||
        (e = alloc(kb, 2 * (size_t)V)) || (e = alloc(d1, 3 * (size_t)V)) ||
        (e = alloc(sx, 3 * (size_t)V)) || (e = alloc(sv, 3 * (size_t)V)) ||
        (e = alloc(skb, 2 * (size_t)V)) || (e = alloc(sd1, 3 * (size_t)V)) ||
        (e = alloc(lx, 3 * (size_t)V)) || (e = alloc(lv, 3 * (size_t)V)) ||
        (e = alloc(lkb, 2 * (size_t)V)) || (e = alloc(ld1, 3 * (size_t)V)) ||
        (e = alloc(th, (size_t)V)) || (e = alloc(om, (size_t)V)) ||
        (e = alloc(sth, (size_t)V)) || (e = alloc(som, (size_t)V)) ||
        (e = alloc(lth, (size_t)V)) || (e = alloc(lom, (size_t)V)) ||
        (e = alloc(acc_b, (size_t)V)) || (e = alloc(acc_s, (size_t)V)) ||
        (e = alloc(loss_part, (size_t)R)) || (e = alloc(status, (size_t)R)) ||
        (e = alloc(ck, (size_t)n_ck * V * NF)) ||
        (e = alloc(acts, (size_t)n_act_max * R * G * 3)) ||
        (e = alloc(du_scratch, (size_t)n_act_max * R * G * 3)) ||
        (e = alloc(opt_mU, (size_t)n_act_max * R * G * 3)) ||
        (e = alloc(opt_vU, (size_t)n_act_max * R * G * 3)) ||
        (e = alloc(opt_mb, (size_t)R)) || (e = alloc(opt_vb, (size_t)R)) ||
        (e = alloc(opt_logb, (size_t)R)) || (e = alloc(opt_db, (size_t)R)) ||
        (e = alloc(opt_xT, 3 * (size_t)V)) || (e = alloc(opt_g, 3 * (size_t)V)) ||
        (e = alloc(opt_loss, 1)) ||
        (e = alloc(u_step, (size_t)R * G * 3)) ||
        (e = alloc(tape, (size_t)std::min(d.ckpt_every, std::max(1, d.max_steps)) * d.n_sub * (size_t)tape_cap)))
      return e;
    if (has_bodies) {
      const size_t nb = (size_t)P * rods::NB_VALS;
      const size_t nbt = (size_t)std::min(d.ckpt_every, std::max(1, d.max_steps)) * d.n_sub * nb;
      if ((e = upload(bwv, bw_h)) || (e = upload(biiv, bii_h)) || (e = upload(body, body_init_h)) ||
          (e = alloc(sbody, nb)) || (e = alloc(ck_body, (size_t)n_ck * nb)) ||
          (e = alloc(btape, nbt)) || (e = alloc(btape2, nbt)) || (e = alloc(lbody, nb)) ||
          (e = alloc(bseed, nb)) || (e = alloc(body_opt0, nb)))
        return e;
      HIPCHK(hipMemset(bseed, 0, sizeof(T) * nb));
      HIPCHK(hipMemset(lbody, 0, sizeof(T) * nb));
    }
    HIPCHK(hipMemset(x, 0, 3 * sizeof(T) * V));
    HIPCHK(hipMemset(v, 0, 3 * sizeof(T) * V));
    HIPCHK(hipMemset(kb, 0, 2 * sizeof(T) * V));
    HIPCHK(hipMemset(d1, 0, 3 * sizeof(T) * V));
    HIPCHK(hipMemset(th, 0, sizeof(T) * V));
    HIPCHK(hipMemset(om, 0, sizeof(T) * V));
    HIPCHK(hipMemset(ck, 0, sizeof(T) * (size_t)n_ck * V * NF));
    HIPCHK(hipMemset(status, 0, sizeof(int32_t) * R));
    HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&side_stream, hipStreamNonBlocking));
    for (hipEvent_t* ev : {&ev_start, &ev_tape[0], &ev_tape[1], &ev_adj[0], &ev_adj[1], &ev_fork})
      HIPCHK(hipEventCreateWithFlags(ev, hipEventDisableTiming));
    for (size_t i = 1; i < bins.size(); ++i) {
      bin_streams.push_back(nullptr);
      HIPCHK(hipStreamCreateWithFlags(&bin_streams.back(), hipStreamNonBlocking));
      bin_done.push_back(nullptr);
      HIPCHK(hipEventCreateWithFlags(&bin_done.back(), hipEventDisableTiming));
    }
    {
      // second tape buffer, if the device has room for it
      const size_t bytes = sizeof(T) * (size_t)std::min(d.ckpt_every, std::max(1, d.max_steps)) *
                           d.n_sub * (size_t)tape_cap;
      void* p2 = nullptr;
      if (hipMalloc(&p2, bytes) == hipSuccess) {
        allocs.push_back(p2);
        tape2 = static_cast<T*>(p2);
      } else {
        (void)hipGetLastError();
      }
    }
    HIPCHK(hipDeviceSynchronize());
    return ROD_OK;
  }

  int64_t sc_stride_ = 0;
  size_t body_lds() const { return has_bodies ? rods::body_lds_bytes<T>() + 16 : 0; }
  // values of global scratch per rod for the adjoint's projection iterates
  // (and, with self-contact, the contact-pass inputs)
  int64_t scratch_per_rod(int C, int W) const {
    return (int64_t)(rods::PROJ_TAPE + 4) * d.n_iters * C * 64 * W;
  }
  // iterates go to global scratch with self-contact, or when they do not fit
  // in LDS next to the lane-exchange buffers
  bool global_tape(int C, int W, bool sc) const {
    return sc || rods::kernel_lds_bytes<T>(2, C, W, false, false, d.n_iters) + body_lds() > lds_max;
  }
  // per-rod offsets of the backward tape block and of the self-contact
  // iterate block for the current launch shapes
  void layout_offsets(std::vector<int64_t>& toff_h, std::vector<int64_t>& soff_h) {
    toff_h.assign(R, 0);
    soff_h.assign(R, 0);
    int64_t off = 0, soff = 0;
    for (const Bin& bn : bins)
      for (int i = 0; i < bn.n; ++i) {
        int r = bin_rods_h[bn.off + i];
        toff_h[r] = off;
        off += (int64_t)tape_fields(bn.tw) * bn.C * 64 * bn.W;
        if (bn.gt) {
          soff_h[r] = soff;
          soff += scratch_per_rod(bn.C, bn.W);
        }
      }
    tape_stride = off;
    sc_stride_ = soff;
  }

  RodArgs<T> args(hipStream_t) const {
    RodArgs<T> a{};
    a.voff = voff;
    a.tape_off = tape_off;
    a.b = b; a.sigma = sigma; a.rc = rc; a.mu = mu; a.restit = restit; a.K = K;
    a.flags = flags;
    a.w = w; a.rest = rest; a.radius = radius; a.gslot = gslot;
    a.prim_off = prim_off; a.prim_type = prim_type; a.prim_a = prim_a; a.prim_b = prim_b;
    a.prim_r = prim_r;
    a.x = x; a.v = v; a.kb = kb; a.d1 = d1;
    a.tape_stride = tape_stride;
    a.act_stride = (int64_t)R * G * 3;
    a.G = G;
    a.spa = d.steps_per_action;
    a.lx = lx; a.lv = lv; a.lkb = lkb; a.ld1 = ld1;
    a.acc_b = acc_b; a.acc_s = acc_s;
    a.sc_tape = sc_tape; a.sc_off = sc_off;
    a.pblk = pblk_f; a.pblk_off = pblk_off_f;
    a.sc_lds = (int32_t)lds_max;
    a.status = status;
    a.Gt = Gt; a.jt = jt; a.th = th; a.om = om; a.lth = lth; a.lom = lom;
    if (has_bodies) {
      a.bw = bwv; a.bii = biiv; a.body = body; a.lbody = lbody; a.btape = btape;
      a.bstride = (int64_t)P * rods::NB_VALS;
    }
    a.h = (T)(d.dt / d.n_sub);
    a.gx = (T)d.gravity[0]; a.gy = (T)d.gravity[1]; a.gz = (T)d.gravity[2];
    a.eps_s = (T)d.eps_s; a.f_thresh = (T)d.f_thresh; a.self_margin = (T)d.self_margin;
    a.n_sub = d.n_sub; a.n_iters = d.n_iters; a.k_ex = d.k_exclude;
    return a;
  }

  // launch `which` for every bin (batched) or per rod (plain) over n_steps
  int launch_all(int which, RodArgs<T> a, hipStream_t st) {
    const bool timed = profiling && ev_next + 2 <= ev_pool.size();
    if (timed) HIPCHK(hipEventRecord(ev_pool[ev_next], st));
    int e = launch_all_(which, a, st);
    if (timed) {
      HIPCHK(hipEventRecord(ev_pool[ev_next + 1], st));
      ev_used.push_back({which, (int)ev_next});
      ev_next += 2;
    }
    return e;
  }

  static hipError_t launch_bin(int which, const Bin& bn, int C, int W, bool gt,
                               const RodArgs<T>& a, int n, hipStream_t st) {
    if (bn.tw && bn.sc) return rods::launch_rods_sc_twist<T>(which, C, W, a, n, st);
    if (bn.tw && bn.bd) return rods::launch_rods_twist_bodies<T>(which, C, W, gt, a, n, st);
    if (bn.sc && bn.bd) return rods::launch_rods_sc_bodies<T>(which, C, W, a, n, st);
    if (bn.tw) return rods::launch_rods_twist<T>(which, C, W, gt, a, n, st);
    if (bn.bd) return rods::launch_rods_bodies<T>(which, C, W, gt, a, n, st);
    return rods::launch_rods<T>(which, C, W, bn.sc, gt, a, n, st);
  }

  int launch_all_(int which, RodArgs<T> a, hipStream_t st) {
    a.sc_stats = sc_stats;
    if (which == 2) {   // the adjoint's own pair scratch and counters
      a.pblk = pblk_a;
      a.pblk_off = pblk_off_a;
      a.sc_stats = sc_stats + 8 * (size_t)R;
    }
    if (!plain) {
      // The bins touch disjoint rods.  They run concurrently except on the
      // backward's replay stream, whose work already overlaps the adjoint
      // and which must not queue behind it on shared bin streams.  Under
      // graph capture the bin streams join the capture through the fork
      // event and leave it through their completion events, so the graph
      // holds the same fork and join.
      const bool fork = concurrent_bins && bins.size() > 1 && st != side_stream;
      if (fork) HIPCHK(hipEventRecord(ev_fork, st));
      for (size_t i = 0; i < bins.size(); ++i) {
        const Bin& bn = bins[i];
        a.rods = bin_rods + bn.off;
        hipStream_t s = st;
        if (fork && i > 0) {
          s = bin_streams[i - 1];
          HIPCHK(hipStreamWaitEvent(s, ev_fork, 0));
        }
        HIPCHK(launch_bin(which, bn, bn.C, bn.W, bn.gt, a, bn.n, s));
        if (fork && i > 0) HIPCHK(hipEventRecord(bin_done[i - 1], s));
      }
      if (fork)
        for (size_t i = 1; i < bins.size(); ++i) HIPCHK(hipStreamWaitEvent(st, bin_done[i - 1], 0));
      return ROD_OK;
    }
    // plain path: one rod per launch, one step per launch
    const int n_steps = a.n_steps;
    const int step_off = a.step_off;
    T* tape0 = a.tape;
    T* btape0 = a.btape;
    for (const Bin& bn : bins) {
      for (int i = 0; i < bn.n; ++i) {
        RodArgs<T> b1 = a;
        b1.rods = bin_rods + bn.off + i;
        b1.n_steps = 1;
        for (int s0 = 0; s0 < n_steps; ++s0) {
          int s = (which == 2) ? (n_steps - 1 - s0) : s0;
          b1.step_off = step_off + s;
          if (tape0) b1.tape = tape0 + (int64_t)s * d.n_sub * tape_stride;
          if (btape0) b1.btape = btape0 + (int64_t)s * d.n_sub * a.bstride;
          b1.ck_x = (s == n_steps - 1) ? a.ck_x : nullptr;
          b1.ck_body = (s == n_steps - 1) ? a.ck_body : nullptr;
          HIPCHK(launch_bin(which, bn, bn.C, bn.W, bn.gt, b1, 1, st));
        }
      }
    }
    return ROD_OK;
  }

  int set_state(const T* x_, const T* v_, const T* kb_, const T* d1_, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(x, x_, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(v, v_, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    if (kb_) HIPCHK(hipMemcpyAsync(kb, kb_, sizeof(T) * 2 * V, hipMemcpyDeviceToDevice, st));
    else HIPCHK(rods::launch_fill<T>(kb, 2 * (int64_t)V, T(0), st));
    if (d1_) HIPCHK(hipMemcpyAsync(d1, d1_, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    else HIPCHK(rods::launch_init_frames<T>(voff, R, x, d1, st));
    HIPCHK(rods::launch_fill<T>(th, V, T(0), st));
    HIPCHK(rods::launch_fill<T>(om, V, T(0), st));
    HIPCHK(rods::launch_fill<int32_t>(status, R, 0, st));
    recorded = false;
    return ROD_OK;
  }

  int set_twist(const T* th_, const T* om_, hipStream_t st) {
    if (th_) HIPCHK(hipMemcpyAsync(th, th_, sizeof(T) * V, hipMemcpyDeviceToDevice, st));
    else HIPCHK(rods::launch_fill<T>(th, V, T(0), st));
    if (om_) HIPCHK(hipMemcpyAsync(om, om_, sizeof(T) * V, hipMemcpyDeviceToDevice, st));
    else HIPCHK(rods::launch_fill<T>(om, V, T(0), st));
    recorded = false;
    return ROD_OK;
  }

  int set_bodies(const T* b_, hipStream_t st) {
    if (!has_bodies) return ROD_OK;
    const size_t nb = (size_t)P * rods::NB_VALS;
    if (b_) HIPCHK(hipMemcpyAsync(body, b_, sizeof(T) * nb, hipMemcpyDeviceToDevice, st));
    else HIPCHK(hipMemcpyAsync(body, body_init_h.data(), sizeof(T) * nb, hipMemcpyHostToDevice, st));
    recorded = false;
    return ROD_OK;
  }

  int rollout(int n_steps, const T* u, T* x_final, int record, hipStream_t st) {
    if (n_steps < 0) return ROD_EINVAL;
    if (record && n_steps > d.max_steps) return ROD_ESTATE;
    recorded = false;
    if (n_steps == 0) {
      if (x_final) HIPCHK(hipMemcpyAsync(x_final, x, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
      return ROD_OK;
    }
    const int spa = d.steps_per_action;
    const int n_act = (n_steps + spa - 1) / spa;
    RodArgs<T> a = args(st);
    if (record) {
      if (G > 0)
        HIPCHK(hipMemcpyAsync(acts, u, sizeof(T) * (size_t)n_act * R * G * 3,
                              hipMemcpyDeviceToDevice, st));
      a.u = acts;
      const int Kc = d.ckpt_every;
      const int nseg = (n_steps + Kc - 1) / Kc;
      HIPCHK(hipMemcpyAsync(ck_x(0), x, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(ck_v(0), v, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(ck_kb(0), kb, sizeof(T) * 2 * V, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(ck_d1(0), d1, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(ck_th(0), th, sizeof(T) * V, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(ck_om(0), om, sizeof(T) * V, hipMemcpyDeviceToDevice, st));
      if (has_bodies)
        HIPCHK(hipMemcpyAsync(ckb(0), body, sizeof(T) * P * rods::NB_VALS, hipMemcpyDeviceToDevice, st));
      for (int seg = 0; seg < nseg; ++seg) {
        a.step_off = seg * Kc;
        a.n_steps = std::min(Kc, n_steps - seg * Kc);
        int which = 0;
        if (seg + 1 < nseg) {
          a.ck_x = ck_x(seg + 1); a.ck_v = ck_v(seg + 1); a.ck_kb = ck_kb(seg + 1);
          a.ck_d1 = ck_d1(seg + 1); a.ck_th = ck_th(seg + 1); a.ck_om = ck_om(seg + 1);
          a.ck_body = has_bodies ? ckb(seg + 1) : nullptr;
        } else {
          a.ck_x = a.ck_v = a.ck_kb = a.ck_d1 = nullptr;
          a.ck_body = nullptr;
          which = 1;   // the last segment also writes its substep tape
          a.tape = tape_for(seg);
          a.btape = btape_for(a.tape);
        }
        int e = launch_all(which, a, st);
        if (e) return e;
      }
      recorded = true;
      last_tape_ok = true;
      n_rec = n_steps;
      rec_gen = ++rec_count;
    } else {
      a.u = u;
      a.step_off = 0;
      a.n_steps = n_steps;
      int e = launch_all(0, a, st);
      if (e) return e;
    }
    if (x_final) HIPCHK(hipMemcpyAsync(x_final, x, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    return ROD_OK;
  }

  int step(const T* u, hipStream_t st, uint32_t* branch = nullptr) {
    RodArgs<T> a = args(st);
    a.u = u;
    a.branch = branch;
    a.act_stride = 0;
    a.spa = 1;
    a.step_off = 0;
    a.n_steps = 1;
    recorded = false;
    return launch_all(0, a, st);
  }

  int backward(const T* gxT, const T* gvT, T* du, T* db_, T* ds_, T* gx0, T* gv0,
               hipStream_t st) {
    if (!recorded) return ROD_ESTATE;
    const int n = n_rec, Kc = d.ckpt_every, nseg = (n + Kc - 1) / Kc;
    const int spa = d.steps_per_action;
    const int n_act = (n + spa - 1) / spa;
    T* dU = du ? du : du_scratch;
    HIPCHK(hipMemcpyAsync(lx, gxT, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    if (gvT) HIPCHK(hipMemcpyAsync(lv, gvT, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    else HIPCHK(rods::launch_fill<T>(lv, 3 * (int64_t)V, T(0), st));
    HIPCHK(rods::launch_fill<T>(lkb, 2 * (int64_t)V, T(0), st));
    HIPCHK(rods::launch_fill<T>(ld1, 3 * (int64_t)V, T(0), st));
    HIPCHK(rods::launch_fill<T>(lth, V, T(0), st));
    HIPCHK(rods::launch_fill<T>(lom, V, T(0), st));
    HIPCHK(rods::launch_fill<T>(dU, (int64_t)n_act * R * G * 3, T(0), st));
    HIPCHK(rods::launch_fill<double>(acc_b, V, 0.0, st));
    HIPCHK(rods::launch_fill<double>(acc_s, V, 0.0, st));
    if (has_bodies)
      HIPCHK(hipMemcpyAsync(lbody, bseed, sizeof(T) * P * rods::NB_VALS, hipMemcpyDeviceToDevice, st));
    // replay segment seg from its checkpoint on stream rs, writing its
    // substep-start states into buf
    auto replay = [&](int seg, T* buf, hipStream_t rs) -> int {
      const int s0 = seg * Kc, ns = std::min(Kc, n - s0);
      HIPCHK(hipMemcpyAsync(sx, ck_x(seg), sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, rs));
      HIPCHK(hipMemcpyAsync(sv, ck_v(seg), sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, rs));
      HIPCHK(hipMemcpyAsync(skb, ck_kb(seg), sizeof(T) * 2 * V, hipMemcpyDeviceToDevice, rs));
      HIPCHK(hipMemcpyAsync(sd1, ck_d1(seg), sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, rs));
      HIPCHK(hipMemcpyAsync(sth, ck_th(seg), sizeof(T) * V, hipMemcpyDeviceToDevice, rs));
      HIPCHK(hipMemcpyAsync(som, ck_om(seg), sizeof(T) * V, hipMemcpyDeviceToDevice, rs));
      if (has_bodies)
        HIPCHK(hipMemcpyAsync(sbody, ckb(seg), sizeof(T) * P * rods::NB_VALS,
                              hipMemcpyDeviceToDevice, rs));
      RodArgs<T> a = args(rs);
      a.x = sx; a.v = sv; a.kb = skb; a.d1 = sd1; a.th = sth; a.om = som;
      a.body = sbody;
      a.u = acts;
      a.step_off = s0;
      a.n_steps = ns;
      a.tape = buf;
      a.btape = btape_for(buf);
      return launch_all(1, a, rs);
    };
    auto adjoint = [&](int seg, T* buf) -> int {
      const int s0 = seg * Kc, ns = std::min(Kc, n - s0);
      RodArgs<T> a = args(st);
      a.x = sx; a.v = sv; a.kb = skb; a.d1 = sd1; a.th = sth; a.om = som;
      a.u = acts;
      a.step_off = s0;
      a.n_steps = ns;
      a.body = sbody;
      a.tape = buf;
      a.btape = btape_for(buf);
      a.dL_du = dU;
      return launch_all(2, a, st);
    };
    int e;
    const bool have_last = last_tape_ok;   // written by the recorded rollout
    last_tape_ok = false;                  // the buffers are reused below
    if (plain || !tape2) {
      for (int seg = nseg - 1; seg >= 0; --seg) {
        if (!(have_last && seg == nseg - 1) && (e = replay(seg, tape, st))) return e;
        if ((e = adjoint(seg, tape))) return e;
      }
    } else {
      T* buf[2] = {tape, tape2};
      HIPCHK(hipEventRecord(ev_start, st));
      HIPCHK(hipStreamWaitEvent(side_stream, ev_start, 0));
      if (have_last) {
        HIPCHK(hipEventRecord(ev_tape[(nseg - 1) & 1], st));
      } else {
        if ((e = replay(nseg - 1, buf[(nseg - 1) & 1], side_stream))) return e;
        HIPCHK(hipEventRecord(ev_tape[(nseg - 1) & 1], side_stream));
      }
      for (int seg = nseg - 1; seg >= 0; --seg) {
        if (seg >= 1) {
          // buffer (seg-1)&1 was last read by the adjoint of segment seg+1
          if (seg + 1 <= nseg - 1) HIPCHK(hipStreamWaitEvent(side_stream, ev_adj[(seg + 1) & 1], 0));
          if ((e = replay(seg - 1, buf[(seg - 1) & 1], side_stream))) return e;
          HIPCHK(hipEventRecord(ev_tape[(seg - 1) & 1], side_stream));
        }
        HIPCHK(hipStreamWaitEvent(st, ev_tape[seg & 1], 0));
        if ((e = adjoint(seg, buf[seg & 1]))) return e;
        HIPCHK(hipEventRecord(ev_adj[seg & 1], st));
      }
    }
    if (db_ || ds_) HIPCHK(rods::launch_reduce_params<T>(voff, R, acc_b, acc_s, db_, ds_, st));
    if (gx0) HIPCHK(hipMemcpyAsync(gx0, lx, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    if (gv0) HIPCHK(hipMemcpyAsync(gv0, lv, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    return ROD_OK;
  }

  // Adam with a cosine schedule and early stopping over rollout + loss +
  // adjoint (App. B); the iteration order is: set b = exp(log b), evaluate
  // the loss and gradients, record the loss, stop on `patience` stalls,
  // otherwise take the Adam step of iteration k (step count k + 1).
  int optimize(const RodsAdam* o, int n_steps, const T* x0, const T* v0, const T* kb0,
               const T* target, T* U, double* losses, int* n_done, hipStream_t st) {
    if (!o || o->iters < 1 || o->patience < 1 || !(o->what & 3) || n_steps < 1 ||
        n_steps > d.max_steps || !x0 || !v0 || !target || !U || !losses || !n_done)
      return ROD_EINVAL;
    const bool act = (o->what & 1) != 0, stiff = (o->what & 2) != 0;
    const int spa = d.steps_per_action;
    const int64_t nU = (int64_t)((n_steps + spa - 1) / spa) * R * G * 3;
    auto cosine = [&](int k, double lr0, double lr_min) {
      if (o->iters <= 1) return lr0;
      return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + std::cos(M_PI * k / (o->iters - 1)));
    };
    HIPCHK(rods::launch_fill<T>(opt_mU, nU, T(0), st));
    HIPCHK(rods::launch_fill<T>(opt_vU, nU, T(0), st));
    HIPCHK(rods::launch_fill<T>(opt_mb, R, T(0), st));
    HIPCHK(rods::launch_fill<T>(opt_vb, R, T(0), st));
    if (stiff) HIPCHK(rods::launch_log<T>(b, opt_logb, R, st));
    if (has_bodies)
      HIPCHK(hipMemcpyAsync(body_opt0, body, sizeof(T) * P * rods::NB_VALS, hipMemcpyDeviceToDevice, st));
    double best = HUGE_VAL;
    int stall = 0, done = 0;
    for (int k = 0; k < o->iters; ++k) {
      if (stiff) HIPCHK(rods::launch_exp<T>(opt_logb, b, R, st));
      int e = set_state(x0, v0, kb0, nullptr, st);
      if (!e && has_bodies) e = set_bodies(body_opt0, st);
      if (!e) e = rollout(n_steps, U, opt_xT, 1, st);
      if (e) return e;
      HIPCHK(rods::launch_loss<T>(voff, R, opt_xT, target, loss_part, opt_loss, opt_g, st));
      e = backward(opt_g, nullptr, du_scratch, stiff ? opt_db : nullptr, nullptr, nullptr, nullptr,
                   st);
      if (e) return e;
      T hl;
      HIPCHK(hipMemcpyAsync(&hl, opt_loss, sizeof(T), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      losses[k] = (double)hl;
      done = k + 1;
      if ((double)hl < best) {
        best = (double)hl;
        stall = 0;
      } else if (++stall >= o->patience) {
        break;
      }
      if (act)
        HIPCHK(rods::launch_adam<T>(U, du_scratch, nullptr, opt_mU, opt_vU, nU,
                                    cosine(k, o->lr0, o->lr_min), o->beta1, o->beta2, o->eps,
                                    k + 1, st));
      if (stiff)
        HIPCHK(rods::launch_adam<T>(opt_logb, opt_db, b, opt_mb, opt_vb, R,
                                    cosine(k, o->lr0_b, o->lr_min_b), o->beta1, o->beta2,
                                    o->eps, k + 1, st));
    }
    if (stiff) HIPCHK(rods::launch_exp<T>(opt_logb, b, R, st));
    *n_done = done;
    recorded = false;
    return ROD_OK;
  }

  // the forward block's candidate pairs of rod r, sorted
  int sc_pairs(int r, int32_t* out, int cap, int32_t* n_out, hipStream_t st) {
    if (r < 0 || r >= R || (!out && cap > 0) || !n_out || cap < 0) return ROD_EINVAL;
    std::vector<int32_t> fl(1);
    HIPCHK(hipMemcpyAsync(fl.data(), flags + r, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (!(fl[0] & ROD_FLAG_SELF)) return ROD_EINVAL;
    const int n = voff_h[r + 1] - voff_h[r];
    const rods::PairBlock pb = rods::sc_block(n, d.k_exclude, (int)sizeof(T), rods::SC_RV_FWD);
    const unsigned char* base = pblk_f + pblk_off_h[r];
    int32_t np = 0;
    HIPCHK(hipMemcpyAsync(&np, base, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (np < 0 || np > rods::sc_pair_cap(n, d.k_exclude)) return ROD_ESTATE;
    std::vector<rods::SPair> pr((size_t)np);
    if (np > 0)
      HIPCHK(hipMemcpyAsync(pr.data(), base + pb.pairs, sizeof(rods::SPair) * np,
                            hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::sort(pr.begin(), pr.end(), [](const rods::SPair& a, const rods::SPair& b) {
      return a.lo != b.lo ? a.lo < b.lo : a.hi < b.hi;
    });
    for (int k = 0; k < np && k < cap; ++k) {
      out[2 * k] = pr[k].lo;
      out[2 * k + 1] = pr[k].hi;
    }
    *n_out = np;
    return ROD_OK;
  }

  // sums over the rods of the self-contact work counters, forward kernels
  // then adjoint: out (host) [2][5]; reset zeroes them afterwards
  int sc_stats_read(int64_t* out, int reset, hipStream_t st) {
    if (!out) return ROD_EINVAL;
    std::vector<unsigned long long> h((size_t)16 * R);
    HIPCHK(hipMemcpyAsync(h.data(), sc_stats, sizeof(unsigned long long) * h.size(),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < 2; ++k)
      for (int i = 0; i < 5; ++i) {
        unsigned long long s = 0;
        for (int r = 0; r < R; ++r) s += h[(size_t)8 * (k * R + r) + i];
        out[5 * k + i] = (int64_t)s;
      }
    if (reset) HIPCHK(rods::launch_fill<int32_t>((int32_t*)sc_stats, 32 * (int64_t)R, 0, st));
    return ROD_OK;
  }

  int bin_nmax(const Bin& bn) const {
    int nmax = 0;
    for (int i = 0; i < bn.n; ++i) {
      int r = bin_rods_h[bn.off + i];
      nmax = std::max(nmax, voff_h[r + 1] - voff_h[r]);
    }
    return nmax;
  }
  // a launch shape the bin may use: a kernel exists for it, the team holds
  // the bin's largest rod and is at most twice its smallest legal team (the
  // tape and scratch are sized for that), and its LDS fits
  bool shape_legal(const Bin& bn, int C, int W) const {
    if (!(C == 2 || C == 4) || !(W == 1 || W == 2 || W == 3 || W == 4 || W == 8)) return false;
    if (W == 3 && !w3_ok(C, bn.sc, bn.tw || bn.bd)) return false;
    const int nmax = bin_nmax(bn);
    auto sh = shapes_for(nmax, prec, bn.sc, bn.tw || bn.bd);
    if (sh.empty()) return false;
    const int team0 = 64 * sh.front().first * sh.front().second;
    return 64 * W * C >= nmax && 64 * W * C <= 2 * team0 &&
           !((prec == 8 || bn.tw || bn.bd) && C != 2) && !(C == 4 && W == 8) &&
           (!bn.sc || sc_shape_ok(C, W)) &&
           rods::kernel_lds_bytes<T>(2, C, W, bn.sc, global_tape(C, W, bn.sc), d.n_iters) +
                   body_lds() <= lds_max;
  }
  // pins bin b to shape (C, W); the tape layout follows
  int set_shape(int b, int C, int W) {
    if (b < 0 || b >= (int)bins.size() || !shape_legal(bins[b], C, W)) return ROD_EINVAL;
    const Bin old = bins[b];
    bins[b].C = C;
    bins[b].W = W;
    bins[b].gt = global_tape(C, W, bins[b].sc);
    std::vector<int64_t> toff_h, soff_h;
    layout_offsets(toff_h, soff_h);
    if (tape_stride > tape_cap || sc_stride_ > sc_cap) {
      bins[b] = old;
      layout_offsets(toff_h, soff_h);
      return ROD_EINVAL;
    }
    drop_graph();
    HIPCHK(hipMemcpy(tape_off, toff_h.data(), sizeof(int64_t) * R, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(sc_off, soff_h.data(), sizeof(int64_t) * R, hipMemcpyHostToDevice));
    recorded = false;
    return ROD_OK;
  }

  int autotune(int n_steps, hipStream_t st) {
    // save state
    HIPCHK(hipMemcpyAsync(sx, x, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(sv, v, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(skb, kb, sizeof(T) * 2 * V, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(sd1, d1, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(sth, th, sizeof(T) * V, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(som, om, sizeof(T) * V, hipMemcpyDeviceToDevice, st));
    if (has_bodies)
      HIPCHK(hipMemcpyAsync(sbody, body, sizeof(T) * P * rods::NB_VALS, hipMemcpyDeviceToDevice, st));
    std::vector<T> zeros((size_t)std::max(1, R * G * 3), T(0));
    T* u0 = du_scratch;
    HIPCHK(hipMemcpyAsync(u0, zeros.data(), sizeof(T) * zeros.size(), hipMemcpyHostToDevice, st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // Coordinate descent over the bins: each candidate shape of a bin is
    // timed on a forward run of the whole batch, every bin launched as a
    // real step launches them (concurrently), with the bins before it at
    // their chosen shapes and those after it at their current ones, so a
    // shape that frees SIMDs for the other bins can win.
    const int plain0 = plain;
    plain = 0;
    int err = ROD_OK;
    for (Bin& bn : bins) {
      std::vector<std::pair<int, int>> cand;
      const int Cs[2] = {2, 4};
      const int Ws[5] = {1, 2, 3, 4, 8};
      for (int C : Cs)
        for (int W : Ws)
          if (shape_legal(bn, C, W)) cand.push_back({C, W});
      float best = 1e30f;
      std::pair<int, int> bestk{bn.C, bn.W};
      for (auto cw : cand) {
        bn.C = cw.first;
        bn.W = cw.second;
        bn.gt = global_tape(bn.C, bn.W, bn.sc);
        RodArgs<T> a = args(st);
        a.x = sx; a.v = sv; a.kb = skb; a.d1 = sd1;   // time on the scratch copy
        a.th = sth; a.om = som;
        a.body = sbody;
        a.u = u0; a.act_stride = 0; a.spa = 1; a.step_off = 0; a.n_steps = n_steps;
        float ms = 0;
        if ((err = launch_all_(0, a, st)) ||                                  // warm
            (err = hipEventRecord(e0, st) == hipSuccess ? ROD_OK : ROD_EHIP) ||
            (err = launch_all_(0, a, st)) ||
            (err = hipEventRecord(e1, st) == hipSuccess ? ROD_OK : ROD_EHIP) ||
            (err = hipEventSynchronize(e1) == hipSuccess ? ROD_OK : ROD_EHIP) ||
            (err = hipEventElapsedTime(&ms, e0, e1) == hipSuccess ? ROD_OK : ROD_EHIP))
          break;
        if (ms < best) { best = ms; bestk = cw; }
      }
      bn.C = bestk.first;
      bn.W = bestk.second;
      bn.gt = global_tape(bn.C, bn.W, bn.sc);
      if (err) break;
    }
    plain = plain0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err) return err;
    // the tape layouts depend on the shapes
    std::vector<int64_t> toff_h, soff_h;
    layout_offsets(toff_h, soff_h);
    if (tape_stride > tape_cap || sc_stride_ > sc_cap) return ROD_EINVAL;   // cannot grow after create
    drop_graph();
    HIPCHK(hipMemcpy(tape_off, toff_h.data(), sizeof(int64_t) * R, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(sc_off, soff_h.data(), sizeof(int64_t) * R, hipMemcpyHostToDevice));
    HIPCHK(hipStreamSynchronize(st));
    recorded = false;
    return ROD_OK;
  }
};

struct Holder {
  int prec;
  HandleBase* impl;
};

template <typename F>
int dispatch(RodsHandle* h, F&& f) {
  if (!h) return ROD_EINVAL;
  Holder* H = reinterpret_cast<Holder*>(h);
  if (H->prec == 4) return f(static_cast<Impl<float>*>(H->impl));
  return f(static_cast<Impl<double>*>(H->impl));
}

static int validate(const RodsDesc* d) {
  if (!d || d->n_rods < 1 || d->n_grasp < 0 || !d->vert_offsets || !d->rod_params ||
      !d->radius || !d->inv_mass || !d->rest_len)
    return ROD_EINVAL;
  if (d->precision != 4 && d->precision != 8) return ROD_EDTYPE;
  if (d->n_grasp > 0 && !d->grasp_idx) return ROD_EINVAL;
  if (d->vert_offsets[0] != 0) return ROD_EINVAL;
  for (int r = 0; r < d->n_rods; ++r) {
    int n = d->vert_offsets[r + 1] - d->vert_offsets[r];
    if (n < 2 || shapes_for(n, d->precision).empty()) return ROD_EINVAL;
    for (int g = 0; g < d->n_grasp; ++g) {
      int li = d->grasp_idx[r * d->n_grasp + g];
      if (li < -1 || li >= n) return ROD_EINVAL;
    }
    const double* p = d->rod_params + (size_t)r * ROD_NPARAM;
    int fl = (int)p[ROD_P_FLAGS];
    if (fl < 0 || fl > 15) return ROD_EINVAL;
    if (fl & ROD_FLAG_TWIST) {
      // twisting rods: two vertices per lane
      if (!d->twist_inv_inertia || !(p[ROD_P_G] >= 0) ||
          shapes_for(n, d->precision, (fl & ROD_FLAG_SELF) != 0, true).empty())
        return ROD_EINVAL;
      for (int i = d->vert_offsets[r]; i < d->vert_offsets[r + 1] - 1; ++i)
        if (!(d->twist_inv_inertia[i] >= 0)) return ROD_EINVAL;
    }
  }
  if (d->prim_offsets) {
    if (d->prim_offsets[0] != 0) return ROD_EINVAL;
    for (int r = 0; r < d->n_rods; ++r)
      if (d->prim_offsets[r + 1] < d->prim_offsets[r]) return ROD_EINVAL;
    int P = d->prim_offsets[d->n_rods];
    if (P > 0 && !d->prims) return ROD_EINVAL;
    for (int k = 0; k < P; ++k)
      if (d->prims[k].type < 0 || d->prims[k].type > 2) return ROD_EINVAL;
    if (d->prim_inv_mass) {
      // moving bodies: spheres, on rods of at most NB_MAX primitives, not on
      // rods with both self-contact and twist
      for (int r = 0; r < d->n_rods; ++r) {
        bool moving = false;
        for (int k = d->prim_offsets[r]; k < d->prim_offsets[r + 1]; ++k) {
          const double wk = d->prim_inv_mass[k];
          if (!(wk >= 0)) return ROD_EINVAL;
          if (wk > 0) {
            if (d->prims[k].type != ROD_PRIM_SPHERE || !d->prim_inv_inertia ||
                !(d->prim_inv_inertia[k] >= 0))
              return ROD_EINVAL;
            moving = true;
          }
        }
        const int fl = (int)d->rod_params[(size_t)r * ROD_NPARAM + ROD_P_FLAGS];
        if (moving && (d->prim_offsets[r + 1] - d->prim_offsets[r] > rods::NB_MAX ||
                       (fl & (ROD_FLAG_SELF | ROD_FLAG_TWIST)) ==
                           (ROD_FLAG_SELF | ROD_FLAG_TWIST)))
          return ROD_EINVAL;
      }
    }
  }
  if (!(d->dt > 0) || d->n_sub < 1 || d->n_iters < 0 || d->n_iters > 32 ||
      d->steps_per_action < 1 || d->ckpt_every < 1 || d->max_steps < 0 || !(d->eps_s > 0))
    return ROD_EINVAL;
  return ROD_OK;
}

}  // namespace

extern "C" {

struct RodsHandle {
  Holder h;
};

int rods_create(const RodsDesc* desc, RodsHandle** out) {
  if (!out) return ROD_EINVAL;
  *out = nullptr;
  int e = validate(desc);
  if (e) return e;
  // the handle-free loss's static scratch: locate it on this device now
  if ((e = rods::loss_scratch_setup(nullptr))) return e;
  RodsHandle* H = new (std::nothrow) RodsHandle;
  if (!H) return ROD_ENOMEM;
  H->h.prec = desc->precision;
  if (desc->precision == 4) {
    auto* I = new (std::nothrow) Impl<float>();
    H->h.impl = I;
    e = I ? I->create(desc) : ROD_ENOMEM;
  } else {
    auto* I = new (std::nothrow) Impl<double>();
    H->h.impl = I;
    e = I ? I->create(desc) : ROD_ENOMEM;
  }
  if (e) {
    delete H->h.impl;
    delete H;
    return e;
  }
  *out = H;
  return ROD_OK;
}

void rods_destroy(RodsHandle* h) {
  if (!h) return;
  delete h->h.impl;
  delete h;
}

const char* rods_strerror(int code) {
  switch (code) {
    case ROD_OK: return "ok";
    case ROD_EINVAL: return "invalid argument";
    case ROD_ENOMEM: return "device allocation failed";
    case ROD_EHIP: return "HIP runtime error";
    case ROD_ESTATE: return "call out of order (no recorded rollout, or n_steps > max_steps)";
    case ROD_EDTYPE: return "unsupported precision";
    default: return "unknown error";
  }
}

int rods_set_state(RodsHandle* h, const void* x, const void* v, const void* kappa_bar,
                   const void* d1, rods_stream_t stream) {
  if (!h || !x || !v) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    return I->set_state((const T*)x, (const T*)v, (const T*)kappa_bar, (const T*)d1,
                        (hipStream_t)stream);
  });
}

int rods_get_state(RodsHandle* h, void* x, void* v, void* kappa_bar, void* d1,
                   rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    hipStream_t st = (hipStream_t)stream;
    size_t V = I->V;
    if (x) HIPCHK(hipMemcpyAsync(x, I->x, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    if (v) HIPCHK(hipMemcpyAsync(v, I->v, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    if (kappa_bar) HIPCHK(hipMemcpyAsync(kappa_bar, I->kb, sizeof(T) * 2 * V, hipMemcpyDeviceToDevice, st));
    if (d1) HIPCHK(hipMemcpyAsync(d1, I->d1, sizeof(T) * 3 * V, hipMemcpyDeviceToDevice, st));
    return (int)ROD_OK;
  });
}

int rods_set_twist(RodsHandle* h, const void* theta, const void* theta_dot, rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    return I->set_twist((const T*)theta, (const T*)theta_dot, (hipStream_t)stream);
  });
}

int rods_get_twist(RodsHandle* h, void* theta, void* theta_dot, rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    hipStream_t st = (hipStream_t)stream;
    size_t V = I->V;
    if (theta) HIPCHK(hipMemcpyAsync(theta, I->th, sizeof(T) * V, hipMemcpyDeviceToDevice, st));
    if (theta_dot) HIPCHK(hipMemcpyAsync(theta_dot, I->om, sizeof(T) * V, hipMemcpyDeviceToDevice, st));
    return (int)ROD_OK;
  });
}

int rods_set_bodies(RodsHandle* h, const void* body, rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    return I->set_bodies((const T*)body, (hipStream_t)stream);
  });
}

int rods_get_bodies(RodsHandle* h, void* body, rods_stream_t stream) {
  if (!h || !body) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    hipStream_t st = (hipStream_t)stream;
    const size_t nb = (size_t)I->P * rods::NB_VALS;
    if (nb == 0) return (int)ROD_OK;
    if (I->has_bodies) HIPCHK(hipMemcpyAsync(body, I->body, sizeof(T) * nb, hipMemcpyDeviceToDevice, st));
    else HIPCHK(hipMemcpyAsync(body, I->body_init_h.data(), sizeof(T) * nb, hipMemcpyHostToDevice, st));
    return (int)ROD_OK;
  });
}

int rods_set_body_adjoint(RodsHandle* h, const void* dL_dbodyT, rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    hipStream_t st = (hipStream_t)stream;
    if (!I->has_bodies) return (int)ROD_OK;
    const int64_t nb = (int64_t)I->P * rods::NB_VALS;
    if (dL_dbodyT) HIPCHK(hipMemcpyAsync(I->bseed, dL_dbodyT, sizeof(T) * nb, hipMemcpyDeviceToDevice, st));
    else HIPCHK(rods::launch_fill<T>(I->bseed, nb, T(0), st));
    return (int)ROD_OK;
  });
}

int rods_get_body_adjoint(RodsHandle* h, void* dL_dbody0, rods_stream_t stream) {
  if (!h || !dL_dbody0) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    hipStream_t st = (hipStream_t)stream;
    const int64_t nb = (int64_t)I->P * rods::NB_VALS;
    if (nb == 0) return (int)ROD_OK;
    if (I->has_bodies) HIPCHK(hipMemcpyAsync(dL_dbody0, I->lbody, sizeof(T) * nb, hipMemcpyDeviceToDevice, st));
    else HIPCHK(rods::launch_fill<T>((T*)dL_dbody0, nb, T(0), st));
    return (int)ROD_OK;
  });
}

int rods_optimize(RodsHandle* h, const RodsAdam* opt, int32_t n_steps, const void* x0,
                  const void* v0, const void* kappa_bar0, const void* target, void* grasp_vel,
                  double* losses, int32_t* n_done, rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    int nd = 0;
    int e = I->optimize(opt, n_steps, (const T*)x0, (const T*)v0, (const T*)kappa_bar0,
                        (const T*)target, (T*)grasp_vel, losses, &nd, (hipStream_t)stream);
    if (n_done) *n_done = nd;
    return e;
  });
}

int rods_get_params(RodsHandle* h, void* b, void* sigma_y, rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    hipStream_t st = (hipStream_t)stream;
    if (b) HIPCHK(hipMemcpyAsync(b, I->b, sizeof(T) * I->R, hipMemcpyDeviceToDevice, st));
    if (sigma_y) HIPCHK(hipMemcpyAsync(sigma_y, I->sigma, sizeof(T) * I->R, hipMemcpyDeviceToDevice, st));
    return (int)ROD_OK;
  });
}

int rods_set_params(RodsHandle* h, const void* b, const void* sigma_y, rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    hipStream_t st = (hipStream_t)stream;
    if (b) HIPCHK(hipMemcpyAsync(I->b, b, sizeof(T) * I->R, hipMemcpyDeviceToDevice, st));
    if (sigma_y) HIPCHK(hipMemcpyAsync(I->sigma, sigma_y, sizeof(T) * I->R, hipMemcpyDeviceToDevice, st));
    I->recorded = false;
    return (int)ROD_OK;
  });
}

int rods_curvature(RodsHandle* h, const void* x, const void* d1, void* kappa,
                   rods_stream_t stream) {
  if (!h || !x || !kappa) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    hipStream_t st = (hipStream_t)stream;
    const T* dd = (const T*)d1;
    if (!dd) {
      HIPCHK(rods::launch_init_frames<T>(I->voff, I->R, (const T*)x, I->sd1, st));
      dd = I->sd1;
    }
    HIPCHK(rods::launch_curvature<T>(I->voff, I->rod_of, I->V, (const T*)x, dd, (T*)kappa, st));
    return (int)ROD_OK;
  });
}

int rods_step(RodsHandle* h, const void* grasp_vel, rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    if (I->G > 0 && !grasp_vel) return (int)ROD_EINVAL;
    return I->step((const T*)grasp_vel, (hipStream_t)stream);
  });
}

int rods_step_branches(RodsHandle* h, const void* grasp_vel, uint32_t* branch,
                       rods_stream_t stream) {
  if (!h || !branch) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    if (I->G > 0 && !grasp_vel) return (int)ROD_EINVAL;
    return I->step((const T*)grasp_vel, (hipStream_t)stream, branch);
  });
}

int rods_step_graph(RodsHandle* h, const void* grasp_vel, rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    if (I->G > 0 && !grasp_vel) return (int)ROD_EINVAL;
    return I->step_graph((const T*)grasp_vel, (hipStream_t)stream);
  });
}

int rods_rollout(RodsHandle* h, int32_t n_steps, const void* grasp_vel, void* x_final,
                 int32_t record, rods_stream_t stream) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    if (I->G > 0 && n_steps > 0 && !grasp_vel) return (int)ROD_EINVAL;
    return I->rollout(n_steps, (const T*)grasp_vel, (T*)x_final, record, (hipStream_t)stream);
  });
}

int rods_backward(RodsHandle* h, const void* dL_dxT, const void* dL_dvT, void* dL_du,
                  void* dL_db, void* dL_dsigma, void* dL_dx0, void* dL_dv0,
                  rods_stream_t stream) {
  if (!h || !dL_dxT) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    return I->backward((const T*)dL_dxT, (const T*)dL_dvT, (T*)dL_du, (T*)dL_db, (T*)dL_dsigma,
                       (T*)dL_dx0, (T*)dL_dv0, (hipStream_t)stream);
  });
}

int rods_loss_mse(RodsHandle* h, const void* x, const void* target, void* loss, void* dL_dx,
                  rods_stream_t stream) {
  if (!h || !x || !target) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    using T = std::remove_pointer_t<decltype(I->x)>;
    HIPCHK(rods::launch_loss<T>(I->voff, I->R, (const T*)x, (const T*)target, I->loss_part,
                                (T*)loss, (T*)dL_dx, (hipStream_t)stream));
    return (int)ROD_OK;
  });
}

int rods_status(RodsHandle* h, int32_t* flags, rods_stream_t stream) {
  if (!h || !flags) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamSynchronize(st) != hipSuccess) return (int)ROD_EHIP;
    if (hipMemcpy(flags, I->status, sizeof(int32_t) * I->R, hipMemcpyDeviceToHost) != hipSuccess)
      return (int)ROD_EHIP;
    return (int)ROD_OK;
  });
}

int rods_sc_pairs(RodsHandle* h, int32_t rod, int32_t* pairs, int32_t cap, int32_t* n_pairs,
                  rods_stream_t stream) {
  return dispatch(h, [&](auto* I) {
    return I->sc_pairs(rod, pairs, cap, n_pairs, (hipStream_t)stream);
  });
}

int rods_sc_stats(RodsHandle* h, int64_t* out, int32_t reset, rods_stream_t stream) {
  return dispatch(h, [&](auto* I) { return I->sc_stats_read(out, reset, (hipStream_t)stream); });
}

int rods_bins(RodsHandle* h, int32_t* out, int32_t max_bins) {
  if (!h || !out) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    int n = 0;
    for (const Bin& bn : I->bins) {
      if (n < max_bins) {
        out[3 * n] = bn.C;
        out[3 * n + 1] = bn.W;
        out[3 * n + 2] = bn.n;
      }
      ++n;
    }
    return n;
  });
}

int rods_autotune(RodsHandle* h, int32_t n_steps, rods_stream_t stream) {
  if (!h || n_steps < 1) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) { return I->autotune(n_steps, (hipStream_t)stream); });
}

int rods_set_launch_shape(RodsHandle* h, int32_t bin, int32_t vertices_per_lane, int32_t waves) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) { return I->set_shape(bin, vertices_per_lane, waves); });
}

int rods_set_plain(RodsHandle* h, int32_t plain) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) {
    I->plain = plain ? 1 : 0;
    I->drop_graph();
    // the tape buffers the backward reads depend on the path: a recording
    // made on the other path is not valid any more
    I->recorded = false;
    I->last_tape_ok = false;
    return (int)ROD_OK;
  });
}

int rods_frames_vjp(RodsHandle* h, const void* x0, void* dL_dx0, rods_stream_t stream) {
  if (!h || !x0 || !dL_dx0) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) -> int {
    using T = std::remove_pointer_t<decltype(I->x)>;
    HIPCHK(rods::launch_init_frames_vjp<T>(I->voff, I->R, (const T*)x0, I->ld1, I->sd1,
                                           (T*)dL_dx0, (hipStream_t)stream));
    return ROD_OK;
  });
}

int64_t rods_recording(RodsHandle* h) {
  if (!h) return ROD_EINVAL;
  Holder* H = reinterpret_cast<Holder*>(h);
  if (H->prec == 4) {
    auto* I = static_cast<Impl<float>*>(H->impl);
    return I->recorded ? I->rec_gen : 0;
  }
  auto* I = static_cast<Impl<double>*>(H->impl);
  return I->recorded ? I->rec_gen : 0;
}

int rods_set_profiling(RodsHandle* h, int32_t on) {
  if (!h) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) { return I->set_profiling(on); });
}

int rods_profile(RodsHandle* h, double* out, rods_stream_t stream) {
  if (!h || !out) return ROD_EINVAL;
  return dispatch(h, [&](auto* I) { return I->profile(out, (hipStream_t)stream); });
}

int rods_selftest_exchange(void* out, rods_stream_t stream) {
  if (!out) return ROD_EINVAL;
  if (rods::launch_selftest_exchange((int*)out, (hipStream_t)stream) != hipSuccess) return ROD_EHIP;
  return ROD_OK;
}

}  // extern "C"
