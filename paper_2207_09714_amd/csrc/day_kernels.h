// Kernel argument blocks of the per-day kernels and their launch helpers.
//
// Aggregates are kept per "output": one per simulation b when parameter sets
// are batched (b = replicate * n_sets + set), one per (replicate, population)
// with per-population parameters.  In both layouts the parameter set of
// output o is o % n_sets.
#pragma once

#include "gabm_device.h"

namespace gabm {

template <typename RT>
struct InitArgs {
  DGraph G;
  DParams P;
  Rng rng;
  uint32_t stream;
  uint32_t* rec;
  unsigned long long* maskI;
  RT* x0;
  RT* Sv;
  RT* inf;
  double* cnt0;  // [n_out][kSlots][kCnt]
};

struct ErArgs {
  DGraph G;
  Rng rng;
  uint32_t stream;
  int t;
  double TE, TI;
  double* acc;  // [N]
  // hard forward with an infectiousness profile: the day's records and the
  // profile (null otherwise)
  const uint32_t* rec = nullptr;
  const float* iota = nullptr;
  int tau_E = 0, W = 0;
};

// The agent-location layer's per-agent sum folded into the split agent
// kernels: the day's pressures, the buffer to clear for the next pass, and the
// agent-sorted visits (P null: not folded).
struct LocFuse {
  const double* P = nullptr;
  double* P_next = nullptr;
  const int64_t* av_ptr = nullptr;
  const int32_t* av_loc = nullptr;
  const float* av_w = nullptr;
  int32_t n_loc = 0;
};

template <typename RT>
struct FwdArgs {
  DGraph G;
  DParams P;
  Rng rng;
  uint32_t stream;
  int t;
  const uint32_t* rec_in;
  uint32_t* rec_out;
  const uint32_t* mI_cur;  // 32-bit view of the current day's masks
  const uint32_t* mE_cur;  // NULL when T_E = 0
  unsigned long long* mI_next;
  unsigned long long* mE_next;
  unsigned long long* mI_clr;
  unsigned long long* mE_clr;
  int64_t mask_words;
  double* A_er;  // daily random layer sums (consumed and cleared), or NULL
  // relaxed state
  const RT* inf_cur;
  RT* inf_next;
  RT* Sv;
  const RT* x0;
  RT* ring;  // exposure history [W][N]
  // store for the reverse pass (already offset to day t), or NULL
  RT* A_st;
  uint8_t* fl_st;
  RT* S_st;
  double* cnt;  // [n_out][K][kSlots][kCnt] or NULL (no counting)
  double* lam_out;
  LocFuse lf;  // split agent kernel only
};

template <typename RT>
struct BwdArgs {
  DGraph G;
  DParams P;
  Rng rng;
  uint32_t stream;
  int t;
  int do_gather;
  const RT* g_cur;   // g^t
  RT* g_prev;        // g^{t-1}
  double* infbar_er; // or NULL
  RT* ring;          // [W][N] inf_bar history
  RT* Sbar;          // [N]
  const RT* A_st;    // day t-1 (offset), unused when t = 0
  const uint8_t* fl_st;
  const RT* S_st;
  const double* Dbar;  // [n_out][K]
  double* gR;          // [n_sets][K][kSlots]
  double* gS;          // [n_sets][n_age][kSlots]
  double* gi0;         // [n_sets][kSlots]
  double* gdw = nullptr;  // [16][kSlots] straight-through gradient of the dwell log weights (E 0-7, I 8-15), or null
  LocFuse lf;             // split agent kernel only
};

// non-zero masks of the rate adjoint g for the persistent reverse kernel
struct FastMasks {
  const unsigned long long* cur;  // g^t
  unsigned long long* next;       // g^{t-1}, written
  unsigned long long* clr;        // cleared for step t-2
  int64_t words;
};

struct FinArgs {
  int K, n_sets, soft, target_stride;
  const float* m;
  const double* cnt;
  const double* cnt0;
  double *counts, *drm, *deaths, *loss;
  double *drm_int, *Dbar;
  const double* target;
};

struct FinBwdArgs {
  int K, n_age, n_out, n_sets;
  const double *gR, *gS, *gi0, *Dbar, *drm_int;
  double *dR, *dS, *dm, *di0;
  const double* gdw = nullptr;  // dwell log-weight gradients: slots, then the outputs
  double *ddw_E = nullptr, *ddw_I = nullptr;
  int tau_E = 0, tau_I = 0;
};

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v);
__global__ void k_fill_f64(double* p, int64_t n);
__global__ void k_fill_f32(float* p, int64_t n);
__global__ void k_copy_u32(uint32_t* d, const uint32_t* s, int64_t n);
__global__ void k_copy_f64(double* d, const double* s, int64_t n);
__global__ void k_copy_f32(float* d, const float* s, int64_t n);
template <typename RT, bool SOFT>
__global__ void k_init(InitArgs<RT> a);
__global__ void k_mask_from_rec(const uint32_t* rec, int N, unsigned long long* mI, unsigned long long* mE, int withE);
__global__ void k_er_fwd_hard(ErArgs a, const uint32_t* mI, const uint32_t* mE);
template <typename RT>
__global__ void k_er_vec(ErArgs a, const RT* v);
__global__ void k_er_pairs_out(ErArgs a, int pop, int32_t* A, int32_t* B, int64_t cap);
template <typename RT, bool SOFT>
__global__ void k_day_fwd(FwdArgs<RT> a);
template <typename RT, bool SOFT, bool DWELL>  // DWELL: stochastic dwell tables (hard modes)
__global__ void k_day_bwd(BwdArgs<RT> a);
// persistent neighbour sum over the fast tiles with an LDS-resident mask
struct GatherArgs {
  DGraph G;
  // sender-sliced contact stream: packed senders, weights, chunk headers
  const uint32_t* colp;
  const float* wp;
  const unsigned long long* chunk_hdr;
  int64_t slice_chunk[kMaxSlices + 1];  // first chunk of each slice; [n_slices] = chunk count
  int32_t n_slices;
  const unsigned long long* mask;  // one bit per agent
  const float* g;                  // reverse: rate adjoints (read where the bit is set)
  double* out;                     // [n_slices][N] per-slice row sums (or a piece marker)
  double* piece;                   // [chunks][2]: first piece, last piece
  double TI;
};

// the neighbour sums as the agent pass reads them
struct SliceSums {
  const double* out;          // [n_slices][N]
  const double* piece;        // [chunks][2]: first piece, last piece
  int64_t N;
  int32_t n_slices;
};

inline SliceSums slice_sums(const GatherArgs& a) {
  SliceSums s;
  s.out = a.out;
  s.piece = a.piece;
  s.N = a.G.N;
  s.n_slices = a.n_slices;
  return s;
}

template <bool BWD>
__global__ void k_gather_fast(GatherArgs a);
// POPS: several populations (per-agent population, parameter set and output)
// DWELL: the parameters may carry stochastic dwell tables; LOC: the
// agent-location layer's per-agent sum is folded in (a.lf)
template <bool POPS, bool DWELL, bool LOC>
__global__ void k_agent_fwd(FwdArgs<float> a, SliceSums ga);
template <bool POPS, bool DWELL, bool LOC>
__global__ void k_agent_bwd(BwdArgs<float> a, FastMasks fm, SliceSums ga);
__global__ void k_fin_fwd(FinArgs a);
__global__ void k_dbar_eff(int n_out, int K, const double* Dbar, const double* w, const double* db, double* out);
__global__ void k_fin_bwd(FinBwdArgs a);

}  // namespace gabm
