// Simulation object: state, per-day stores, checkpoints and adjoint buffers.
#pragma once

#include <map>
#include <tuple>

#include "gabm_internal.h"

namespace gabm {

struct Sim {
  Graph* G = nullptr;
  // layout
  int32_t n_sets = 1, n_reps = 1, B = 1, K = 0, tau_E = 0, tau_I = 0, W = 0, n_age = 0, mode = 0, per_pop = 0;
  int32_t ckpt = 0;      // segment length (== K when everything is stored)
  int32_t n_seg = 1;
  int32_t precision = GABM_F32;
  int32_t use_graph = 0;
  bool has_iota = false;  // created with an infectiousness profile (tile kernels only)
  size_t rsz = 4;        // bytes of one stored real
  int64_t NB = 0;        // N * B
  int64_t NV = 0;        // entries of one per-simulation vector: N * B, or N * 64 * SPL lane-interleaved (B > 32)
  int64_t mask_words = 0;  // 64-bit words per mask buffer
  int32_t bw = 1;        // 32-bit mask words per agent (batched), 0 for B = 1 bit-packed layout

  // hard state
  uint32_t* rec[2] = {nullptr, nullptr};
  int cur = 0;  // rec[cur] holds the current day's records
  unsigned long long* maskI[3] = {nullptr, nullptr, nullptr};
  unsigned long long* maskE[3] = {nullptr, nullptr, nullptr};
  double* A_er = nullptr;
  // soft state (real = float or double)
  void* Sv = nullptr;
  void* x0 = nullptr;
  void* xi_ring = nullptr;  // [W][NB]
  void* inf[2] = {nullptr, nullptr};
  // per-day store for the reverse pass, [ckpt days][NB]
  void* A_st = nullptr;
  uint8_t* fl_st = nullptr;
  void* S_st = nullptr;
  int32_t store_base = 0;  // day held in slot 0
  // checkpoints, [n_seg][...]
  uint32_t* ck_rec = nullptr;
  void* ck_soft = nullptr;  // [n_seg][(W+2)*NB]: Sv, inf, ring
  // aggregates
  double* cnt = nullptr;   // [B][K][kSlots][kCnt]
  double* cnt0 = nullptr;  // [B][kSlots][kCnt]
  double* drm = nullptr;   // [B][K]
  double* Dbar = nullptr;  // [n_out][K] loss adjoint 2 (D - y) / K of the last forward
  double* Dbar_eff = nullptr;  // [n_out][K] deaths adjoint used by the reverse pass
  // reverse pass
  void* ring = nullptr;  // [W][NB]
  void* Sbar = nullptr;  // [NB]
  void* g[2] = {nullptr, nullptr};
  double* infbar_er = nullptr;  // [NB]
  double* loc_P = nullptr;      // [2][n_locations] location pressures; passes alternate buffers
  int loc_par = 0;              // buffer of the next pass (zero on entry)
  double* gR = nullptr;   // [n_sets][K][kSlots]
  double* gS = nullptr;   // [n_sets][n_age][kSlots]
  double* gi0 = nullptr;  // [n_sets][kSlots]
  double* gdw = nullptr;  // [16][kSlots] dwell log-weight gradients (runs created with dwell tables)
  bool has_dwell = false;

  // kernel timing: event pairs around each fused day kernel
  int32_t time_kernels = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_k[GABM_KT_N];  // per kernel class: indices into ev_pool
  int64_t kt_seq[GABM_KT_N] = {};                     // launches per class since the last reset
  size_t ev_used = 0;
  hipEvent_t next_event();

  // persistent kernels (float state, one simulation, fewer than 2^24 agents):
  // eligibility and the non-zero masks of the rate adjoint
  int n_cu = 0;
  int schedule = 0;  // 0 auto, 1 tile kernels only
  bool fast_fwd_ok = false, fast_bwd_ok = false;
  unsigned long long* gz[3] = {nullptr, nullptr, nullptr};
  size_t gz_bytes = 0;
  double* Abuf = nullptr;  // [N] neighbour sums handed from the gather to the agent pass
  double* piece = nullptr; // [2 * n_chunks] sums of rows crossing chunk boundaries

  // batched runs (B > 1): lane mapping, 'any simulation' masks of the forward
  // days (the reverse pass uses gz), per-launch tile counters, launch sizes
  int32_t LB = 64, spl = 1, indep = 0;
  int64_t any_words = 0;
  bool b_any_lds = true;
  bool b_wide = false;  // B > 32 with the packed contact form: one wave per tile, 64-contact windows
  unsigned long long* anyI[3] = {nullptr, nullptr, nullptr};
  unsigned int* wq = nullptr;  // [3K+1]: forward days, replayed days, reverse steps
  int bgrid_i = 0, bgrid_f = 0, bgrid_b = 0;

  int next_day = 0;     // forward progress for gabm_day_fwd
  int next_bwd = -1;    // reverse progress for gabm_day_bwd
  bool fwd_done = false;

  // captured graphs, keyed by the call's pointers
  std::map<std::tuple<const void*, const void*, const void*, const void*, const void*, const void*, const void*,
                      const void*, const void*>,
           hipGraphExec_t>
      fwd_graphs, bwd_graphs;

  void release();
};

}  // namespace gabm

struct gabm_sim_s {
  gabm::Sim s;
};
