// Run loop: allocation of a simulation, the K-day forward with state
// snapshots every `ckpt` days, and the reverse pass that replays each
// segment from its snapshot before walking it backwards (the loop over days
// is unrolled by hand instead of being kept whole in memory, which is what
// automatic differentiation of the unrolled loop would do, Appendix B).
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "batched.h"
#include "day_kernels.h"
#include "loc.h"
#include "sim_internal.h"

namespace gabm {

static int blocks_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20));
}
static int blocks_capped(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 8192)); }

hipEvent_t Sim::next_event() {
  if (ev_used == ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ev_pool.push_back(e);
  }
  return ev_pool[ev_used++];
}

// brackets one launch with a pair of events when kernel timing is on
struct KTime {
  Sim& s;
  hipStream_t st;
  int cls;
  int a = -1;
  KTime(Sim& s_, hipStream_t st_, int cls_) : s(s_), st(st_), cls(cls_) {
    if (!s.time_kernels || s.use_graph) return;
    // time_kernels = k: every k-th launch of each class is bracketed
    if (s.kt_seq[cls]++ % s.time_kernels != 0) return;
    hipEvent_t e = s.next_event();
    if (!e) return;
    a = (int)s.ev_used - 1;
    hipEventRecord(e, st);
  }
  ~KTime() {
    if (a < 0) return;
    hipEvent_t e = s.next_event();
    if (!e) return;
    hipEventRecord(e, st);
    s.ev_k[cls].emplace_back(a, (int)s.ev_used - 1);
  }
};

gabm_status sim_kernel_times(Sim& s, gabm_kernel_times* out, int reset) {
  for (int c = 0; c < GABM_KT_N; ++c) {
    double tot = 0.0;
    for (auto& pr : s.ev_k[c]) {
      float ms = 0.f;
      GABM_HIP(hipEventSynchronize(s.ev_pool[pr.second]));
      GABM_HIP(hipEventElapsedTime(&ms, s.ev_pool[pr.first], s.ev_pool[pr.second]));
      tot += ms;
    }
    out->ms[c] = tot;
    out->launches[c] = (int64_t)s.ev_k[c].size();
  }
  if (reset) {
    for (auto& v : s.ev_k) v.clear();
    for (auto& n : s.kt_seq) n = 0;
    s.ev_used = 0;
  }
  return GABM_OK;
}

void Sim::release() {
  for (hipEvent_t e : ev_pool) hipEventDestroy(e);
  ev_pool.clear();
  for (auto& kv : fwd_graphs) hipGraphExecDestroy(kv.second);
  for (auto& kv : bwd_graphs) hipGraphExecDestroy(kv.second);
  fwd_graphs.clear();
  bwd_graphs.clear();
  void* ps[] = {rec[0], rec[1], maskI[0], maskI[1], maskI[2], maskE[0], maskE[1], maskE[2], A_er, Sv, x0, xi_ring,
                inf[0], inf[1], A_st, fl_st, S_st, ck_rec, ck_soft, cnt, cnt0, drm, Dbar, Dbar_eff, ring, Sbar, g[0], g[1],
                infbar_er, gR, gS, gi0, gz[0], gz[1], gz[2], Abuf, piece, anyI[0], anyI[1], anyI[2], wq, loc_P, gdw};
  for (void* p : ps) hipFree(p);
}

int sim_n_out(const Sim& s) { return s.per_pop ? s.n_reps * s.G->n_pops : s.B; }

// bytes of every device buffer of a simulation (the same arithmetic as the allocation)
struct Layout {
  size_t rec, mask, aer, soft_vec, soft_ring, st_A, st_fl, st_S, ck_rec, ck_soft, cnt, cnt0, drm, ring, sbar, g,
      ier, gR, gS, gi0, locp;
  size_t total() const {
    return 2 * rec + 6 * mask + aer + 4 * soft_vec + soft_ring + st_A + st_fl + st_S + ck_rec + ck_soft + cnt + cnt0 +
           3 * drm + ring + sbar + 2 * g + ier + gR + gS + gi0 + locp;
  }
};

static Layout layout(const Graph& G, int B, int64_t NVs, int n_out, int n_sets, int K, int W, int ckpt, int n_seg,
                     int mode, size_t rsz, bool has_aux, int64_t mask_words) {
  Layout L{};
  const size_t NB = (size_t)G.N * B;
  const size_t NV = (size_t)NVs;
  const bool soft = mode == GABM_SOFT;
  L.rec = NB * 4;
  L.mask = soft ? 0 : (size_t)mask_words * 8;
  L.aer = has_aux ? NB * 8 : 0;
  L.soft_vec = soft ? NB * rsz : 0;
  L.soft_ring = soft ? (size_t)W * NB * rsz : 0;
  const bool diff = mode != GABM_PLAIN;
  L.st_A = diff ? (size_t)ckpt * NV * rsz : 0;
  L.st_fl = (diff && !soft) ? (size_t)ckpt * NV : 0;
  L.st_S = (diff && soft) ? (size_t)ckpt * NB * rsz : 0;
  const size_t nck = (diff && n_seg > 1) ? (size_t)n_seg : 0;
  L.ck_rec = soft ? 0 : nck * NB * 4;
  L.ck_soft = soft ? nck * (size_t)(W + 2) * NB * rsz : 0;
  L.cnt = (size_t)n_out * K * kSlots * kCnt * 8;
  L.cnt0 = (size_t)n_out * kSlots * kCnt * 8;
  L.drm = (size_t)n_out * K * 8;
  L.ring = diff ? (size_t)W * NV * rsz : 0;
  L.sbar = diff ? NV * rsz : 0;
  L.g = diff ? NV * rsz : 0;
  L.ier = (diff && has_aux) ? NB * 8 : 0;
  L.locp = (size_t)2 * G.n_loc * 8;
  L.gR = (size_t)n_sets * K * kSlots * 8;
  L.gS = (size_t)n_sets * G.n_age * kSlots * 8;
  L.gi0 = (size_t)n_sets * kSlots * 8;
  return L;
}

// buffers of the persistent path (B = 1) and of the batched path (B > 1)
static size_t extra_bytes(const Sim& s) {
  const Graph& G = *s.G;
  size_t b = 3 * s.gz_bytes;
  if (s.fast_fwd_ok || s.fast_bwd_ok) b += (size_t)G.n_slices * G.N * 8 + (size_t)G.slice_chunk.back() * 16;
  if (s.B > 1) b += 3 * (size_t)s.any_words * 8 + (size_t)(3 * s.K + 1) * 4;
  if (s.has_dwell && s.mode == GABM_HARD_ST) b += (size_t)16 * kSlots * 8;
  return b;
}

static int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

static void sim_shape(Sim& s, const Graph& G, const gabm_params* p, const gabm_run_desc* run) {
  s.G = const_cast<Graph*>(&G);
  s.n_sets = p->n_sets;
  s.n_reps = std::max(1, run->n_reps);
  s.per_pop = p->per_pop_params ? 1 : 0;
  s.B = s.per_pop ? s.n_reps : s.n_sets * s.n_reps;
  s.K = p->K;
  s.tau_E = p->tau_E;
  s.tau_I = p->tau_I;
  s.W = p->tau_E + p->tau_I;
  s.n_age = G.n_age;
  s.mode = p->mode;
  s.ckpt = (run->ckpt_every <= 0 || run->ckpt_every >= p->K) ? p->K : run->ckpt_every;
  s.n_seg = (s.K + s.ckpt - 1) / s.ckpt;
  s.precision = run->precision;
  s.use_graph = run->use_hip_graph;
  s.time_kernels = run->time_kernels;
  s.schedule = run->schedule;
  {
    int dev = 0, ncu = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 0;
    s.n_cu = ncu;
  }
  s.has_iota = p->iota != nullptr;
  s.has_dwell = p->dwell_E != nullptr;
  const bool fast_shape = s.schedule == 0 && !s.has_iota && s.n_cu > 0 && s.B == 1 && G.n_slices > 0 &&
                          run->precision == GABM_F32 && s.mode != GABM_SOFT;
  s.fast_fwd_ok = fast_shape;
  s.fast_bwd_ok = fast_shape && s.mode == GABM_HARD_ST;
  s.rsz = run->precision == GABM_F64 ? 8 : 4;
  s.NB = (int64_t)G.N * s.B;
  s.NV = s.NB;
  if (s.B == 1) {
    s.bw = 0;
    s.mask_words = G.N / 64 + 2;
  } else {
    s.bw = (s.B + 31) / 32;
    s.mask_words = ((int64_t)G.N * s.bw + 1) / 2 + 2;
    s.LB = s.B > 32 ? 64 : next_pow2(s.B);
    s.spl = s.B <= 64 ? 1 : (s.B <= 128 ? 2 : 4);
    s.any_words = (int64_t)G.N / 64 + 2;
    s.b_any_lds = s.any_words <= kBAnyLdsWords;
    s.b_wide = s.schedule == 0 && s.LB == 64 && G.n_chunks > 0;
    if (s.b_wide) s.NV = (int64_t)G.N * 64 * s.spl;
  }
  s.gz_bytes = 0;
  if (s.fast_bwd_ok) s.gz_bytes = (size_t)s.mask_words * 8;
  if (s.B > 1 && s.mode != GABM_PLAIN) s.gz_bytes = (size_t)s.any_words * 8;
}

gabm_status sim_workspace(const Graph& G, const gabm_params* p, const gabm_run_desc* run, size_t* bytes) {
  Sim s;
  sim_shape(s, G, p, run);
  Layout L = layout(G, s.B, s.NV, sim_n_out(s), s.n_sets, s.K, s.W, s.ckpt, s.n_seg, s.mode, s.rsz, G.has_aux(),
                    s.mask_words);
  *bytes = L.total() + extra_bytes(s);
  return GABM_OK;
}

// launch sizes of the batched kernels: enough resident blocks to fill every
// compute unit (the day kernels take receiver tiles from a counter)
template <class K>
static int resident_grid(K kernel, size_t lds, int n_cu) {
  int nb = 0;
  if (lds > 65536) hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBBlock, lds) != hipSuccess || nb < 1) nb = 1;
  return nb * std::max(1, n_cu);
}

template <int SPL>
static void batched_grids(Sim& s) {
  const size_t lf = bfwd_lds(s.B, s.any_words, s.b_any_lds);
  const size_t lb = bbwd_lds(s.B, s.n_age, s.any_words, s.b_any_lds);
  s.bgrid_i = resident_grid(k_binit<SPL>, 0, s.n_cu);
  if (s.b_any_lds) {
    s.bgrid_f = s.b_wide ? resident_grid(k_bfwd64<SPL, true>, lf, s.n_cu) : resident_grid(k_bfwd<SPL, true>, lf, s.n_cu);
    s.bgrid_b = s.b_wide ? resident_grid(k_bbwd64<SPL, true>, lb, s.n_cu) : resident_grid(k_bbwd<SPL, true>, lb, s.n_cu);
  } else {
    s.bgrid_f = s.b_wide ? resident_grid(k_bfwd64<SPL, false>, lf, s.n_cu) : resident_grid(k_bfwd<SPL, false>, lf, s.n_cu);
    s.bgrid_b = s.b_wide ? resident_grid(k_bbwd64<SPL, false>, lb, s.n_cu) : resident_grid(k_bbwd<SPL, false>, lb, s.n_cu);
  }
}

static gabm_status batched_setup(Sim& s) {
  if (s.spl == 1) batched_grids<1>(s);
  else if (s.spl == 2) batched_grids<2>(s);
  else batched_grids<4>(s);
  GABM_HIP(hipGetLastError());
  return GABM_OK;
}

gabm_status sim_create(const Graph& G, const gabm_params* p, const gabm_run_desc* run, Sim& s) {
  sim_shape(s, G, p, run);
  Layout L = layout(G, s.B, s.NV, sim_n_out(s), s.n_sets, s.K, s.W, s.ckpt, s.n_seg, s.mode, s.rsz, G.has_aux(),
                    s.mask_words);
  auto al = [&](void** ptr, size_t n) -> gabm_status {
    if (n == 0) {
      *ptr = nullptr;
      return GABM_OK;
    }
    hipError_t e = hipMalloc(ptr, n);
    if (e != hipSuccess) {
      set_error(std::string("hipMalloc of simulation workspace failed: ") + hipGetErrorString(e));
      return GABM_ENOMEM;
    }
    return GABM_OK;
  };
#define AL(ptr, n)                                       \
  do {                                                   \
    gabm_status st_ = al((void**)&(ptr), (n));           \
    if (st_ != GABM_OK) { s.release(); return st_; }     \
  } while (0)
  AL(s.rec[0], L.rec);
  AL(s.rec[1], L.rec);
  for (int k = 0; k < 3; ++k) {
    AL(s.maskI[k], L.mask);
    AL(s.maskE[k], L.mask);
  }
  AL(s.A_er, L.aer);
  AL(s.Sv, L.soft_vec);
  AL(s.x0, L.soft_vec);
  AL(s.inf[0], L.soft_vec);
  AL(s.inf[1], L.soft_vec);
  AL(s.xi_ring, L.soft_ring);
  AL(s.A_st, L.st_A);
  AL(s.fl_st, L.st_fl);
  AL(s.S_st, L.st_S);
  AL(s.ck_rec, L.ck_rec);
  AL(s.ck_soft, L.ck_soft);
  AL(s.cnt, L.cnt);
  AL(s.cnt0, L.cnt0);
  AL(s.drm, L.drm);
  AL(s.Dbar, L.drm);
  AL(s.Dbar_eff, L.drm);
  AL(s.ring, L.ring);
  AL(s.Sbar, L.sbar);
  AL(s.g[0], L.g);
  AL(s.g[1], L.g);
  AL(s.infbar_er, L.ier);
  AL(s.loc_P, L.locp);
  if (s.has_dwell && s.mode == GABM_HARD_ST) AL(s.gdw, (size_t)16 * kSlots * 8);
  AL(s.gR, L.gR);
  AL(s.gS, L.gS);
  AL(s.gi0, L.gi0);
  for (int k = 0; k < 3; ++k) AL(s.gz[k], s.gz_bytes);
  if (s.fast_fwd_ok || s.fast_bwd_ok) {
    AL(s.Abuf, (size_t)G.n_slices * G.N * 8);
    AL(s.piece, (size_t)G.slice_chunk.back() * 2 * 8);
  }
  if (s.B > 1) {
    for (int k = 0; k < 3; ++k) AL(s.anyI[k], (size_t)s.any_words * 8);
    AL(s.wq, (size_t)(3 * s.K + 1) * 4);
    gabm_status rc = batched_setup(s);
    if (rc != GABM_OK) {
      s.release();
      return rc;
    }
  }
#undef AL
  return GABM_OK;
}

// ---------------------------------------------------------------- launch helpers

static void fill0(void* p, size_t bytes, hipStream_t st) {
  if (!p || bytes == 0) return;
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_capped((int64_t)(bytes / 8))), dim3(kBlock), 0, st,
                     (unsigned long long*)p, (int64_t)(bytes / 8), 0ull);
  if (bytes % 8) hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(kBlock), 0, st, (float*)((char*)p + bytes - 4), (int64_t)1);
}
static void copy_bytes(void* d, const void* s, size_t bytes, hipStream_t st) {
  if (bytes % 4 == 0)
    hipLaunchKernelGGL(k_copy_u32, dim3(blocks_capped((int64_t)(bytes / 4))), dim3(kBlock), 0, st, (uint32_t*)d,
                       (const uint32_t*)s, (int64_t)(bytes / 4));
}

static Rng make_rng(const gabm_rng* r) {
  Rng g;
  g.k0 = (uint32_t)r->seed;
  g.k1 = (uint32_t)(r->seed >> 32);
  return g;
}

template <typename RT>
static RT* store_ptr(void* base, const Sim& s, int slot) {
  return base ? (RT*)base + (int64_t)slot * s.NV : nullptr;
}

// B = 1 path ------------------------------------------------------------------

// arguments of the split kernels: the sender-sliced stream and its outputs
static GatherArgs gather_args(const Sim& s, const DGraph& dg, const unsigned long long* mask, const float* g,
                              double TI) {
  const Graph& G = *s.G;
  GatherArgs ga;
  ga.G = dg;
  ga.colp = G.fcolp;
  ga.wp = G.fwp;
  ga.chunk_hdr = G.fchunk_hdr;
  for (int p = 0; p <= kMaxSlices; ++p) ga.slice_chunk[p] = G.slice_chunk[std::min(p, G.n_slices)];
  ga.n_slices = G.n_slices;
  ga.mask = mask;
  ga.g = g;
  ga.out = s.Abuf;
  ga.piece = s.piece;
  ga.TI = TI;
  return ga;
}

// the agent-location layer's two passes for one day, adding into `acc`; with
// `fold` set only the pressures are formed here and `fold` receives what the
// split agent kernel needs to add the per-agent sums itself
template <class V>
static void loc_pass(Sim& s, const V& val, double* acc, hipStream_t st, LocFuse* fold = nullptr) {
  const Graph& G = *s.G;
  LocView L;
  L.N = G.N; L.n_loc = G.n_loc; L.V = G.n_visits;
  L.lv_agent = G.lv_agent; L.lv_loc = G.lv_loc; L.lv_w = G.lv_w;
  L.av_ptr = G.av_ptr; L.av_loc = G.av_loc; L.av_w = G.av_w;
  KTime kt(s, st, GABM_KT_LOC);
  // the pass's buffer was cleared by the previous pass (or by b1_init); this
  // pass clears the other one.  The sequence of passes of a run is fixed, so
  // a captured run replays the same buffer order.
  double* P = s.loc_P + (size_t)s.loc_par * G.n_loc;
  double* Pn = s.loc_P + (size_t)(1 - s.loc_par) * G.n_loc;
  hipLaunchKernelGGL(k_loc_pressure<V>, dim3(blocks_capped(G.n_visits)), dim3(kBlock), 0, st, L, val, P);
  if (fold) {
    fold->P = P;
    fold->P_next = Pn;
    fold->av_ptr = G.av_ptr;
    fold->av_loc = G.av_loc;
    fold->av_w = G.av_w;
    fold->n_loc = G.n_loc;
  } else {
    hipLaunchKernelGGL(k_loc_gather<V>, dim3(blocks_capped(std::max<int64_t>(G.N, G.n_loc))), dim3(kBlock), 0, st, L,
                       val, (const double*)P, acc, Pn);
  }
  s.loc_par = 1 - s.loc_par;
}

template <typename RT>
static void b1_init(Sim& s, const DParams& P, Rng rng, uint32_t stream, hipStream_t st) {
  const Graph& G = *s.G;
  const bool soft = s.mode == GABM_SOFT;
  // the daily-layer accumulator is cleared by each day's consumer; start clean
  fill0(s.A_er, s.A_er ? (size_t)s.NB * 8 : 0, st);
  // both pressure buffers of the location layer
  fill0(s.loc_P, s.loc_P ? (size_t)2 * G.n_loc * 8 : 0, st);
  s.loc_par = 0;
  // neighbour sums of the split path: rows without contacts are never written
  fill0(s.Abuf, s.Abuf ? (size_t)G.n_slices * G.N * 8 : 0, st);
  if (!soft)
    for (int k = 0; k < 3; ++k) {
      fill0(s.maskI[k], s.mask_words * 8, st);
      fill0(s.maskE[k], s.mask_words * 8, st);
    }
  else {
    fill0(s.xi_ring, (size_t)s.W * s.NB * sizeof(RT), st);
  }
  InitArgs<RT> a;
  a.G = G.view(); a.P = P; a.rng = rng; a.stream = stream; a.rec = s.rec[0]; a.maskI = s.maskI[0];
  a.x0 = (RT*)s.x0; a.Sv = (RT*)s.Sv; a.inf = (RT*)s.inf[0]; a.cnt0 = s.cnt0;
  s.cur = 0;
  if (soft) hipLaunchKernelGGL((k_init<RT, true>), dim3(blocks_for(G.N)), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_init<RT, false>), dim3(blocks_for(G.N)), dim3(kBlock), 0, st, a);
}

// one forward day; `slot` < 0 = do not store, `count` = accumulate aggregates
template <typename RT>
static void b1_day_fwd(Sim& s, const DParams& P, Rng rng, uint32_t stream, int t, int slot, bool count, hipStream_t st) {
  const Graph& G = *s.G;
  const bool soft = s.mode == GABM_SOFT;
  const bool withE = P.TE != 0.0;
  const bool has_er = G.has_er();
  const DGraph dg = G.view();
  if (has_er) {
    ErArgs e;
    e.G = dg; e.rng = rng; e.stream = stream; e.t = t; e.TE = P.TE; e.TI = P.TI; e.acc = s.A_er;
    if (P.iota && !soft) {  // hard senders' weights come from their exposure days
      e.rec = s.rec[s.cur];
      e.iota = P.iota;
      e.tau_E = P.tau_E;
      e.W = P.tau_E + P.tau_I;
    }
    const int nb = blocks_capped(dg.er_total);
    KTime ke(s, st, GABM_KT_ER);
    if (soft) hipLaunchKernelGGL(k_er_vec<RT>, dim3(nb), dim3(kBlock), 0, st, e, (const RT*)s.inf[s.cur]);
    else hipLaunchKernelGGL(k_er_fwd_hard, dim3(nb), dim3(kBlock), 0, st, e, (const uint32_t*)s.maskI[t % 3],
                            withE ? (const uint32_t*)s.maskE[t % 3] : nullptr);
  }
  const bool fast = std::is_same<RT, float>::value && s.fast_fwd_ok && !withE;
  LocFuse lf;
  if (G.n_visits > 0) {
    if (soft) {
      LocVecVal<RT> v;
      v.v = (const RT*)s.inf[s.cur];
      loc_pass(s, v, s.A_er, st);
    } else {
      LocHardVal v;
      v.mI = (const uint32_t*)s.maskI[t % 3];
      v.mE = withE ? (const uint32_t*)s.maskE[t % 3] : nullptr;
      v.TI = P.TI;
      v.TE = P.TE;
      if (P.iota) {
        v.rec = s.rec[s.cur];
        v.iota = P.iota;
        v.t = t;
        v.tau_E = P.tau_E;
        v.W = P.tau_E + P.tau_I;
      }
      loc_pass(s, v, s.A_er, st, fast ? &lf : nullptr);  // the split agent kernel adds the sums
    }
  }
  FwdArgs<RT> a;
  a.G = dg; a.P = P; a.rng = rng; a.stream = stream; a.t = t;
  a.rec_in = s.rec[s.cur]; a.rec_out = s.rec[1 - s.cur];
  a.mI_cur = (const uint32_t*)s.maskI[t % 3];
  a.mE_cur = withE ? (const uint32_t*)s.maskE[t % 3] : nullptr;
  a.mI_next = s.maskI[(t + 1) % 3];
  a.mE_next = withE ? s.maskE[(t + 1) % 3] : nullptr;
  a.mI_clr = s.maskI[(t + 2) % 3];
  a.mE_clr = withE ? s.maskE[(t + 2) % 3] : nullptr;
  a.mask_words = s.mask_words;
  a.A_er = G.has_aux() ? s.A_er : nullptr;
  a.inf_cur = (const RT*)s.inf[s.cur];
  a.inf_next = (RT*)s.inf[1 - s.cur];
  a.Sv = (RT*)s.Sv; a.x0 = (const RT*)s.x0; a.ring = (RT*)s.xi_ring;
  const bool store = slot >= 0 && s.mode != GABM_PLAIN;
  a.A_st = store ? store_ptr<RT>(s.A_st, s, slot) : nullptr;
  a.fl_st = (store && !soft) ? s.fl_st + (int64_t)slot * s.NV : nullptr;
  a.S_st = (store && soft) ? store_ptr<RT>(s.S_st, s, slot) : nullptr;
  a.cnt = count ? s.cnt : nullptr;
  a.lam_out = nullptr;
  a.lf = lf;
  if (fast) {
    const GatherArgs ga = gather_args(s, dg, s.maskI[t % 3], nullptr, P.TI);
    {
      KTime kt(s, st, GABM_KT_GATHER_FWD);
      hipLaunchKernelGGL(k_gather_fast<false>, dim3(s.n_cu), dim3(kFastBlock), 0, st, ga);
    }
    KTime kt(s, st, GABM_KT_AGENT_FWD);
    const FwdArgs<float>& af = *(FwdArgs<float>*)&a;
    const dim3 grid(blocks_for(G.N)), blk(kBlock);
    const SliceSums ss = slice_sums(ga);
    const int variant = (G.n_pops > 1 ? 4 : 0) | (P.dwell_E ? 2 : 0) | (lf.P ? 1 : 0);
    switch (variant) {
      case 0: hipLaunchKernelGGL((k_agent_fwd<false, false, false>), grid, blk, 0, st, af, ss); break;
      case 1: hipLaunchKernelGGL((k_agent_fwd<false, false, true>), grid, blk, 0, st, af, ss); break;
      case 2: hipLaunchKernelGGL((k_agent_fwd<false, true, false>), grid, blk, 0, st, af, ss); break;
      case 3: hipLaunchKernelGGL((k_agent_fwd<false, true, true>), grid, blk, 0, st, af, ss); break;
      case 4: hipLaunchKernelGGL((k_agent_fwd<true, false, false>), grid, blk, 0, st, af, ss); break;
      case 5: hipLaunchKernelGGL((k_agent_fwd<true, false, true>), grid, blk, 0, st, af, ss); break;
      case 6: hipLaunchKernelGGL((k_agent_fwd<true, true, false>), grid, blk, 0, st, af, ss); break;
      default: hipLaunchKernelGGL((k_agent_fwd<true, true, true>), grid, blk, 0, st, af, ss); break;
    }
  } else {
    KTime kt(s, st, GABM_KT_DAY_FWD);
    if (soft) hipLaunchKernelGGL((k_day_fwd<RT, true>), dim3(G.n_tiles), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_day_fwd<RT, false>), dim3(G.n_tiles), dim3(kBlock), 0, st, a);
  }
  s.cur = 1 - s.cur;
}

template <typename RT>
static void b1_snapshot(Sim& s, int seg, bool restore, hipStream_t st) {
  if (s.mode == GABM_SOFT) {
    RT* base = (RT*)s.ck_soft + (int64_t)seg * (s.W + 2) * s.NB;
    const size_t nb = s.NB * sizeof(RT);
    if (restore) {
      copy_bytes(s.Sv, base, nb, st);
      copy_bytes(s.inf[s.cur], base + s.NB, nb, st);
      copy_bytes(s.xi_ring, base + 2 * s.NB, nb * s.W, st);
    } else {
      copy_bytes(base, s.Sv, nb, st);
      copy_bytes(base + s.NB, s.inf[s.cur], nb, st);
      copy_bytes(base + 2 * s.NB, s.xi_ring, nb * s.W, st);
    }
  } else {
    uint32_t* base = s.ck_rec + (int64_t)seg * s.NB;
    if (restore) {
      copy_bytes(s.rec[s.cur], base, s.NB * 4, st);
    } else {
      copy_bytes(base, s.rec[s.cur], s.NB * 4, st);
    }
  }
}

template <typename RT>
static void b1_restore(Sim& s, int seg, int s0, hipStream_t st) {
  b1_snapshot<RT>(s, seg, true, st);
  if (s.mode != GABM_SOFT) {
    for (int k = 0; k < 3; ++k) {
      fill0(s.maskI[k], s.mask_words * 8, st);
      fill0(s.maskE[k], s.mask_words * 8, st);
    }
    hipLaunchKernelGGL(k_mask_from_rec, dim3(blocks_for(s.G->N)), dim3(kBlock), 0, st, s.rec[s.cur], s.G->N,
                       s.maskI[s0 % 3], s.maskE[s0 % 3], 1);
  }
}

template <typename RT>
static void b1_fin_fwd(Sim& s, const DParams& P, const double* target, int stride, const gabm_fwd_out* out,
                       hipStream_t st) {
  FinArgs f;
  f.K = s.K; f.n_sets = s.n_sets; f.soft = s.mode == GABM_SOFT; f.target_stride = stride; f.m = P.m;
  f.cnt = s.cnt; f.cnt0 = s.cnt0; f.counts = out ? out->counts : nullptr; f.drm = out ? out->drm : nullptr;
  f.deaths = out ? out->deaths : nullptr; f.loss = out ? out->loss : nullptr; f.drm_int = s.drm; f.Dbar = s.Dbar;
  f.target = target;
  hipLaunchKernelGGL(k_fin_fwd, dim3(sim_n_out(s)), dim3(kBlock), 0, st, f);
}

template <typename RT>
static void b1_day_bwd(Sim& s, const DParams& P, Rng rng, uint32_t stream, int t, int slot, hipStream_t st) {
  const Graph& G = *s.G;
  const bool soft = s.mode == GABM_SOFT;
  const bool has_er = G.has_er();
  const DGraph dg = G.view();
  const bool gather = t < s.K;
  if (gather && has_er) {
    ErArgs e;
    e.G = dg; e.rng = rng; e.stream = stream; e.t = t; e.TE = P.TE; e.TI = P.TI; e.acc = s.infbar_er;
    KTime ke(s, st, GABM_KT_ER);
    hipLaunchKernelGGL(k_er_vec<RT>, dim3(blocks_capped(dg.er_total)), dim3(kBlock), 0, st, e, (const RT*)s.g[t & 1]);
  }
  const bool fastb = std::is_same<RT, float>::value && s.fast_bwd_ok;
  LocFuse lf;
  if (gather && G.n_visits > 0) {
    LocVecVal<RT> v;
    v.v = (const RT*)s.g[t & 1];
    loc_pass(s, v, s.infbar_er, st, fastb ? &lf : nullptr);  // the split agent kernel adds the sums
  }
  BwdArgs<RT> a;
  a.G = dg; a.P = P; a.rng = rng; a.stream = stream; a.t = t; a.do_gather = gather ? 1 : 0;
  a.g_cur = (const RT*)s.g[t & 1];
  a.g_prev = (RT*)s.g[(t + 1) & 1];
  a.infbar_er = (gather && G.has_aux()) ? s.infbar_er : nullptr;
  a.ring = (RT*)s.ring; a.Sbar = (RT*)s.Sbar;
  a.A_st = t >= 1 ? store_ptr<RT>(s.A_st, s, slot) : nullptr;
  a.fl_st = (t >= 1 && !soft) ? s.fl_st + (int64_t)slot * s.NV : nullptr;
  a.S_st = (t >= 1 && soft) ? store_ptr<RT>(s.S_st, s, slot) : nullptr;
  a.Dbar = s.Dbar_eff; a.gR = s.gR; a.gS = s.gS; a.gi0 = s.gi0;
  a.gdw = s.gdw;
  a.lf = lf;
  if (fastb) {
    FastMasks fm;
    fm.cur = s.gz[t % 3];
    fm.next = s.gz[(t + 2) % 3];
    fm.clr = s.gz[(t + 1) % 3];
    fm.words = s.mask_words;
    const GatherArgs ga = gather_args(s, dg, s.gz[t % 3], (const float*)s.g[t & 1], 1.0);
    if (gather) {
      KTime kt(s, st, GABM_KT_GATHER_BWD);
      hipLaunchKernelGGL(k_gather_fast<true>, dim3(s.n_cu), dim3(kFastBlock), 0, st, ga);
    }
    KTime kt(s, st, GABM_KT_AGENT_BWD);
    const BwdArgs<float>& ab = *(BwdArgs<float>*)&a;
    const dim3 grid(blocks_for(G.N)), blk(kBlock);
    const SliceSums ss = slice_sums(ga);
    const int variant = (G.n_pops > 1 ? 4 : 0) | (P.dwell_E ? 2 : 0) | (lf.P ? 1 : 0);
    switch (variant) {
      case 0: hipLaunchKernelGGL((k_agent_bwd<false, false, false>), grid, blk, 0, st, ab, fm, ss); break;
      case 1: hipLaunchKernelGGL((k_agent_bwd<false, false, true>), grid, blk, 0, st, ab, fm, ss); break;
      case 2: hipLaunchKernelGGL((k_agent_bwd<false, true, false>), grid, blk, 0, st, ab, fm, ss); break;
      case 3: hipLaunchKernelGGL((k_agent_bwd<false, true, true>), grid, blk, 0, st, ab, fm, ss); break;
      case 4: hipLaunchKernelGGL((k_agent_bwd<true, false, false>), grid, blk, 0, st, ab, fm, ss); break;
      case 5: hipLaunchKernelGGL((k_agent_bwd<true, false, true>), grid, blk, 0, st, ab, fm, ss); break;
      case 6: hipLaunchKernelGGL((k_agent_bwd<true, true, false>), grid, blk, 0, st, ab, fm, ss); break;
      default: hipLaunchKernelGGL((k_agent_bwd<true, true, true>), grid, blk, 0, st, ab, fm, ss); break;
    }
  } else {
    KTime kt(s, st, GABM_KT_DAY_BWD);
    if (soft) hipLaunchKernelGGL((k_day_bwd<RT, true, false>), dim3(G.n_tiles), dim3(kBlock), 0, st, a);
    else if (P.dwell_E) hipLaunchKernelGGL((k_day_bwd<RT, false, true>), dim3(G.n_tiles), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_day_bwd<RT, false, false>), dim3(G.n_tiles), dim3(kBlock), 0, st, a);
  }
}

static void fin_bwd(Sim& s, const gabm_grads* out, hipStream_t st) {
  FinBwdArgs f;
  f.K = s.K; f.n_age = s.n_age; f.n_out = sim_n_out(s); f.n_sets = s.n_sets;
  f.gR = s.gR; f.gS = s.gS; f.gi0 = s.gi0; f.Dbar = s.Dbar_eff; f.drm_int = s.drm;
  f.dR = out->dR; f.dS = out->dS; f.dm = out->dm; f.di0 = out->di0;
  f.gdw = s.gdw; f.ddw_E = out->ddwell_E; f.ddw_I = out->ddwell_I; f.tau_E = s.tau_E; f.tau_I = s.tau_I;
  hipLaunchKernelGGL(k_fin_bwd, dim3(s.n_sets), dim3(kBlock), 0, st, f);
}

// batched path (B > 1) ----------------------------------------------------------

static BSims bsims(const Sim& s, uint32_t stream) {
  BSims S;
  S.B = s.B;
  S.n_sets = s.n_sets;
  S.indep = s.indep;
  S.stream0 = stream;
  S.bw = s.bw;
  S.LB = s.LB;
  return S;
}

static void bt_init(Sim& s, const DParams& P, Rng rng, uint32_t stream, hipStream_t st) {
  for (int k = 0; k < 3; ++k) fill0(s.anyI[k], (size_t)s.any_words * 8, st);
  BInitArgs a;
  a.G = s.G->view(); a.P = P; a.rng = rng; a.S = bsims(s, stream);
  a.rec = s.rec[0];
  a.mI = (uint32_t*)s.maskI[0];
  a.mE = P.TE != 0.0 ? (uint32_t*)s.maskE[0] : nullptr;
  a.any = s.anyI[0];
  a.cnt0 = s.cnt0;
  s.cur = 0;
  if (s.spl == 1) hipLaunchKernelGGL(k_binit<1>, dim3(s.bgrid_i), dim3(kBBlock), 0, st, a);
  else if (s.spl == 2) hipLaunchKernelGGL(k_binit<2>, dim3(s.bgrid_i), dim3(kBBlock), 0, st, a);
  else hipLaunchKernelGGL(k_binit<4>, dim3(s.bgrid_i), dim3(kBBlock), 0, st, a);
}

template <int SPL>
static void bt_launch_fwd(Sim& s, const BFwdArgs& a, hipStream_t st) {
  const size_t lds = bfwd_lds(s.B, s.any_words, s.b_any_lds);
  if (s.b_wide) {
    if (s.b_any_lds) hipLaunchKernelGGL((k_bfwd64<SPL, true>), dim3(s.bgrid_f), dim3(kBBlock), lds, st, a);
    else hipLaunchKernelGGL((k_bfwd64<SPL, false>), dim3(s.bgrid_f), dim3(kBBlock), lds, st, a);
  } else if (s.b_any_lds) {
    hipLaunchKernelGGL((k_bfwd<SPL, true>), dim3(s.bgrid_f), dim3(kBBlock), lds, st, a);
  } else {
    hipLaunchKernelGGL((k_bfwd<SPL, false>), dim3(s.bgrid_f), dim3(kBBlock), lds, st, a);
  }
}

template <int SPL>
static void bt_launch_bwd(Sim& s, const BBwdArgs& a, hipStream_t st) {
  const size_t lds = bbwd_lds(s.B, s.n_age, s.any_words, s.b_any_lds);
  if (s.b_wide) {
    if (s.b_any_lds) hipLaunchKernelGGL((k_bbwd64<SPL, true>), dim3(s.bgrid_b), dim3(kBBlock), lds, st, a);
    else hipLaunchKernelGGL((k_bbwd64<SPL, false>), dim3(s.bgrid_b), dim3(kBBlock), lds, st, a);
  } else if (s.b_any_lds) {
    hipLaunchKernelGGL((k_bbwd<SPL, true>), dim3(s.bgrid_b), dim3(kBBlock), lds, st, a);
  } else {
    hipLaunchKernelGGL((k_bbwd<SPL, false>), dim3(s.bgrid_b), dim3(kBBlock), lds, st, a);
  }
}

// one forward day of all simulations; `replay` = recomputation inside the reverse pass
static void bt_day_fwd(Sim& s, const DParams& P, Rng rng, uint32_t stream, int t, int slot, bool count, bool replay,
                       hipStream_t st) {
  const bool withE = P.TE != 0.0;
  BFwdArgs a;
  a.G = s.G->view(); a.P = P; a.rng = rng; a.S = bsims(s, stream); a.t = t;
  a.rec_in = s.rec[s.cur];
  a.rec_out = s.rec[1 - s.cur];
  a.mI = (const uint32_t*)s.maskI[t & 1];
  a.mE = withE ? (const uint32_t*)s.maskE[t & 1] : nullptr;
  a.mI_next = (uint32_t*)s.maskI[(t + 1) & 1];
  a.mE_next = withE ? (uint32_t*)s.maskE[(t + 1) & 1] : nullptr;
  a.any_cur = s.anyI[t % 3];
  a.any_next = s.anyI[(t + 1) % 3];
  a.any_clr = s.anyI[(t + 2) % 3];
  a.any_words = s.any_words;
  const bool store = slot >= 0 && s.mode != GABM_PLAIN;
  a.A_st = store ? (float*)s.A_st + (int64_t)slot * s.NV : nullptr;
  a.fl_st = store ? s.fl_st + (int64_t)slot * s.NV : nullptr;
  a.cnt = count ? s.cnt : nullptr;
  a.work = s.wq + (replay ? s.K + t : t);
  KTime kt(s, st, GABM_KT_DAY_FWD);
  if (s.spl == 1) bt_launch_fwd<1>(s, a, st);
  else if (s.spl == 2) bt_launch_fwd<2>(s, a, st);
  else bt_launch_fwd<4>(s, a, st);
  s.cur = 1 - s.cur;
}

static void bt_restore(Sim& s, const DParams& P, int seg, int s0, hipStream_t st) {
  copy_bytes(s.rec[s.cur], s.ck_rec + (int64_t)seg * s.NB, s.NB * 4, st);
  for (int k = 0; k < 3; ++k) fill0(s.anyI[k], (size_t)s.any_words * 8, st);
  BMaskArgs a;
  a.G = s.G->view(); a.S = bsims(s, 0);
  a.rec = s.rec[s.cur];
  a.mI = (uint32_t*)s.maskI[s0 & 1];
  a.mE = P.TE != 0.0 ? (uint32_t*)s.maskE[s0 & 1] : nullptr;
  a.any = s.anyI[s0 % 3];
  if (s.spl == 1) hipLaunchKernelGGL(k_bmask<1>, dim3(s.bgrid_i), dim3(kBBlock), 0, st, a);
  else if (s.spl == 2) hipLaunchKernelGGL(k_bmask<2>, dim3(s.bgrid_i), dim3(kBBlock), 0, st, a);
  else hipLaunchKernelGGL(k_bmask<4>, dim3(s.bgrid_i), dim3(kBBlock), 0, st, a);
}

// reverse step t of all simulations: gather of g^t (t < K), adjoint of day t-1
static void bt_day_bwd(Sim& s, const DParams& P, Rng rng, uint32_t stream, int t, int slot, hipStream_t st) {
  BBwdArgs a;
  a.G = s.G->view(); a.P = P; a.rng = rng; a.S = bsims(s, stream); a.t = t;
  a.do_gather = t < s.K ? 1 : 0;
  a.g_cur = (const float*)s.g[t & 1];
  a.g_prev = (float*)s.g[(t + 1) & 1];
  a.ring = (float*)s.ring;
  a.Sbar = (float*)s.Sbar;
  a.A_st = t >= 1 ? (const float*)s.A_st + (int64_t)slot * s.NV : nullptr;
  a.fl_st = t >= 1 ? s.fl_st + (int64_t)slot * s.NV : nullptr;
  a.Dbar = s.Dbar_eff;
  a.gz_cur = s.gz[t % 3];
  a.gz_next = s.gz[(t + 2) % 3];
  a.gz_clr = s.gz[(t + 1) % 3];
  a.any_words = s.any_words;
  a.gR = s.gR; a.gS = s.gS; a.gi0 = s.gi0;
  a.work = s.wq + 2 * s.K + t;
  KTime kt(s, st, GABM_KT_DAY_BWD);
  if (s.spl == 1) bt_launch_bwd<1>(s, a, st);
  else if (s.spl == 2) bt_launch_bwd<2>(s, a, st);
  else bt_launch_bwd<4>(s, a, st);
}

static void bwd_reset(Sim& s, const double* lw, const double* db, hipStream_t st) {
  const int64_t n = (int64_t)sim_n_out(s) * s.K;
  hipLaunchKernelGGL(k_dbar_eff, dim3(blocks_capped(n)), dim3(kBlock), 0, st, sim_n_out(s), s.K, s.Dbar, lw, db,
                     s.Dbar_eff);
  fill0(s.ring, (size_t)s.W * s.NV * s.rsz, st);
  fill0(s.Sbar, s.NV * s.rsz, st);
  fill0(s.infbar_er, s.infbar_er ? (size_t)s.NB * 8 : 0, st);
  // every run-level pass sequence starts from clear pressure buffers at parity
  // 0, whatever earlier (possibly replayed) sequences left in the host state
  fill0(s.loc_P, s.loc_P ? (size_t)2 * s.G->n_loc * 8 : 0, st);
  s.loc_par = 0;
  for (int k = 0; k < 3; ++k) fill0(s.gz[k], s.gz_bytes, st);
  if (s.wq) fill0(s.wq + s.K, (size_t)(2 * s.K + 1) * 4, st);  // counters of replayed days and reverse steps
  fill0(s.gR, (size_t)s.n_sets * s.K * kSlots * 8, st);
  fill0(s.gS, (size_t)s.n_sets * s.n_age * kSlots * 8, st);
  fill0(s.gi0, (size_t)s.n_sets * kSlots * 8, st);
  fill0(s.gdw, s.gdw ? (size_t)16 * kSlots * 8 : 0, st);
}

// ---------------------------------------------------------------- day loops of a run

template <typename RT>
static void run_forward(Sim& s, const DParams& P, Rng rng, uint32_t stream, const double* target, int stride,
                        const gabm_fwd_out* out, hipStream_t st) {
  const int last_s0 = (s.n_seg - 1) * s.ckpt;
  fill0(s.cnt, (size_t)sim_n_out(s) * s.K * kSlots * kCnt * 8, st);
  fill0(s.cnt0, (size_t)sim_n_out(s) * kSlots * kCnt * 8, st);
  if (s.B == 1) {
    b1_init<RT>(s, P, rng, stream, st);
    for (int t = 0; t < s.K; ++t) {
      if (s.n_seg > 1 && s.mode != GABM_PLAIN && t % s.ckpt == 0 && t < last_s0) b1_snapshot<RT>(s, t / s.ckpt, false, st);
      b1_day_fwd<RT>(s, P, rng, stream, t, t >= last_s0 ? t - last_s0 : -1, true, st);
    }
  } else {
    fill0(s.wq, (size_t)s.K * 4, st);
    bt_init(s, P, rng, stream, st);
    for (int t = 0; t < s.K; ++t) {
      if (s.n_seg > 1 && s.mode != GABM_PLAIN && t % s.ckpt == 0 && t < last_s0) b1_snapshot<RT>(s, t / s.ckpt, false, st);
      bt_day_fwd(s, P, rng, stream, t, t >= last_s0 ? t - last_s0 : -1, true, false, st);
    }
  }
  b1_fin_fwd<RT>(s, P, target, stride, out, st);
}

template <typename RT>
static void run_backward(Sim& s, const DParams& P, Rng rng, uint32_t stream, const double* lw, const double* db,
                         const gabm_grads* out, hipStream_t st) {
  bwd_reset(s, lw, db, st);
  const bool bt = s.B != 1;
  for (int seg = s.n_seg - 1; seg >= 0; --seg) {
    const int s0 = seg * s.ckpt, s1 = std::min(s.K, s0 + s.ckpt);
    if (seg != s.n_seg - 1) {
      if (bt) bt_restore(s, P, seg, s0, st);
      else b1_restore<RT>(s, seg, s0, st);
      for (int d = s0; d < s1; ++d) {
        if (bt) bt_day_fwd(s, P, rng, stream, d, d - s0, false, true, st);
        else b1_day_fwd<RT>(s, P, rng, stream, d, d - s0, false, st);
      }
    }
    for (int t = s1; t > s0; --t) {
      if (bt) bt_day_bwd(s, P, rng, stream, t, t - 1 - s0, st);
      else b1_day_bwd<RT>(s, P, rng, stream, t, t - 1 - s0, st);
    }
  }
  if (bt) bt_day_bwd(s, P, rng, stream, 0, 0, st);
  else b1_day_bwd<RT>(s, P, rng, stream, 0, 0, st);
  fin_bwd(s, out, st);
}

// captured or direct execution of a run function
template <class F>
static gabm_status execute(Sim& s, bool fwd, const void* k1, const void* k2, const void* k3, const void* k4,
                           const void* k5, const void* k6, const void* k7, const void* k8, const void* k9,
                           hipStream_t st, F f) {
  if (!s.use_graph) {
    f(st);
    GABM_HIP(hipGetLastError());
    return GABM_OK;
  }
  auto& cache = fwd ? s.fwd_graphs : s.bwd_graphs;
  auto key = std::make_tuple(k1, k2, k3, k4, k5, k6, k7, k8, k9);
  auto it = cache.find(key);
  if (it == cache.end()) {
    hipStream_t cs = st;
    bool own = false;
    if (cs == nullptr) {
      GABM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      own = true;
    }
    GABM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    f(cs);
    hipGraph_t graph;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess) {
      if (own) hipStreamDestroy(cs);
      set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      return GABM_EHIP;
    }
    hipGraphExec_t ex;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (own) hipStreamDestroy(cs);
    if (e != hipSuccess) {
      set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      return GABM_EHIP;
    }
    it = cache.emplace(key, ex).first;
  }
  GABM_HIP(hipGraphLaunch(it->second, st));
  return GABM_OK;
}

gabm_status sim_forward(Sim& s, const DParams& P, const gabm_rng* r, const double* target, int stride,
                        const gabm_fwd_out* out, hipStream_t st) {
  const Rng rng = make_rng(r);
  const uint32_t stream = r->replicate;
  s.indep = r->independent_sets ? 1 : 0;
  gabm_status rc;
  if (s.precision == GABM_F64)
    rc = execute(s, true, P.R, P.S, target, out ? out->counts : nullptr, out ? out->loss : nullptr,
                 (const void*)(uintptr_t)(r->seed ^ ((uint64_t)r->replicate << 40) ^ ((uint64_t)stride << 56) ^
                                          ((uint64_t)(r->independent_sets ? 1 : 0) << 63)), P.iota, P.dwell_E, P.dwell_I, st,
                 [&](hipStream_t cs) { run_forward<double>(s, P, rng, stream, target, stride, out, cs); });
  else
    rc = execute(s, true, P.R, P.S, target, out ? out->counts : nullptr, out ? out->loss : nullptr,
                 (const void*)(uintptr_t)(r->seed ^ ((uint64_t)r->replicate << 40) ^ ((uint64_t)stride << 56) ^
                                          ((uint64_t)(r->independent_sets ? 1 : 0) << 63)), P.iota, P.dwell_E, P.dwell_I, st,
                 [&](hipStream_t cs) { run_forward<float>(s, P, rng, stream, target, stride, out, cs); });
  if (rc == GABM_OK) {
    s.fwd_done = true;
    s.next_day = 0;
    s.next_bwd = s.K;
  }
  return rc;
}

gabm_status sim_backward(Sim& s, const DParams& P, const gabm_rng* r, const double* lw, const double* db,
                         const gabm_grads* out, hipStream_t st) {
  GABM_CHECK(s.fwd_done, GABM_ESTATE, "gabm_sim_backward before a completed forward run");
  GABM_CHECK(s.mode != GABM_PLAIN, GABM_ESTATE, "gabm_sim_backward on a PLAIN (forward-only) simulation");
  const Rng rng = make_rng(r);
  const uint32_t stream = r->replicate;
  s.indep = r->independent_sets ? 1 : 0;
  // a backward replays segments and so consumes the forward state
  s.fwd_done = false;
  if (s.precision == GABM_F64)
    return execute(s, false, P.R, lw, db, out->dR, out->di0,
                   (const void*)(uintptr_t)(r->seed ^ ((uint64_t)r->replicate << 40) ^
                                          ((uint64_t)(r->independent_sets ? 1 : 0) << 63)), P.iota, P.dwell_E, P.dwell_I, st,
                   [&](hipStream_t cs) { run_backward<double>(s, P, rng, stream, lw, db, out, cs); });
  return execute(s, false, P.R, lw, db, out->dR, out->di0,
                 (const void*)(uintptr_t)(r->seed ^ ((uint64_t)r->replicate << 40) ^
                                          ((uint64_t)(r->independent_sets ? 1 : 0) << 63)), P.iota, P.dwell_E, P.dwell_I, st,
                 [&](hipStream_t cs) { run_backward<float>(s, P, rng, stream, lw, db, out, cs); });
}

// ---------------------------------------------------------------- day-level entry points (B = 1 and batched)

template <typename RT>
static gabm_status day_fwd_t(Sim& s, const DParams& P, const gabm_rng* r, int day, const double* target, int stride,
                             const gabm_fwd_out* out, hipStream_t st) {
  const Rng rng = make_rng(r);
  const uint32_t stream = r->replicate;
  s.indep = r->independent_sets ? 1 : 0;
  if (day == 0) {
    fill0(s.cnt, (size_t)sim_n_out(s) * s.K * kSlots * kCnt * 8, st);
    fill0(s.cnt0, (size_t)sim_n_out(s) * kSlots * kCnt * 8, st);
    if (s.B == 1) {
      b1_init<RT>(s, P, rng, stream, st);
    } else {
      fill0(s.wq, (size_t)s.K * 4, st);
      bt_init(s, P, rng, stream, st);
    }
  }
  const int slot = s.ckpt == s.K ? day : -1;
  if (s.B == 1) b1_day_fwd<RT>(s, P, rng, stream, day, slot, true, st);
  else bt_day_fwd(s, P, rng, stream, day, slot, true, false, st);
  if (day == s.K - 1) b1_fin_fwd<RT>(s, P, target, stride, out, st);
  GABM_HIP(hipGetLastError());
  return GABM_OK;
}

gabm_status sim_day_fwd(Sim& s, const DParams& P, const gabm_rng* r, int day, const double* target, int stride,
                        const gabm_fwd_out* out, hipStream_t st) {
  GABM_CHECK(day >= 0 && day < s.K, GABM_ERANGE, "day outside [0, K)");
  GABM_CHECK(day == 0 || (day == s.next_day && !s.fwd_done), GABM_ESTATE, "gabm_day_fwd called out of order");
  gabm_status rc = s.precision == GABM_F64 ? day_fwd_t<double>(s, P, r, day, target, stride, out, st)
                                           : day_fwd_t<float>(s, P, r, day, target, stride, out, st);
  if (rc != GABM_OK) return rc;
  s.fwd_done = false;
  s.next_day = day + 1;
  if (day == s.K - 1) {
    s.fwd_done = true;
    s.next_bwd = s.K;
  }
  return GABM_OK;
}

template <typename RT>
static gabm_status day_bwd_t(Sim& s, const DParams& P, const gabm_rng* r, int day, const gabm_grads* out,
                             hipStream_t st) {
  const Rng rng = make_rng(r);
  const uint32_t stream = r->replicate;
  s.indep = r->independent_sets ? 1 : 0;
  if (day == s.K) bwd_reset(s, nullptr, nullptr, st);
  if (s.B == 1) b1_day_bwd<RT>(s, P, rng, stream, day, day >= 1 ? day - 1 : 0, st);
  else bt_day_bwd(s, P, rng, stream, day, day >= 1 ? day - 1 : 0, st);
  if (day == 0) fin_bwd(s, out, st);
  GABM_HIP(hipGetLastError());
  return GABM_OK;
}

gabm_status sim_day_bwd(Sim& s, const DParams& P, const gabm_rng* r, int day, const gabm_grads* out, hipStream_t st) {
  GABM_CHECK(s.mode != GABM_PLAIN, GABM_ESTATE, "reverse day on a PLAIN (forward-only) simulation");
  GABM_CHECK(s.ckpt == s.K, GABM_ESTATE, "gabm_day_bwd needs a simulation that keeps every day (ckpt_every = 0)");
  GABM_CHECK(s.fwd_done && day == s.next_bwd, GABM_ESTATE, "gabm_day_bwd called out of order or before a closed forward run");
  gabm_status rc = s.precision == GABM_F64 ? day_bwd_t<double>(s, P, r, day, out, st) : day_bwd_t<float>(s, P, r, day, out, st);
  if (rc != GABM_OK) return rc;
  s.next_bwd = day - 1;
  if (day == 0) s.fwd_done = false;
  return GABM_OK;
}

}  // namespace gabm
