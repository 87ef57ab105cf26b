// Batched simulations: B = n_sets * n_reps > 1 runs sharing one contact graph
// (several parameter sets and replicates of Section 3.2's calibration, one
// launch per day for all of them).
//
// State is batch-minor: value of simulation b of agent i at i * B + b (the
// wide kernels for B > 32 keep their per-simulation float vectors -- stored
// day, window ring, S adjoint, rate adjoint -- lane-interleaved instead, see
// batched.hip).  A
// receiver row is processed by a group of LB lanes (LB = 64 for B > 32, else
// the next power of two >= B); lane l of the group carries simulations
// l, l + 64, ... (SPL = ceil(B / 64) of them), so the contact stream of a
// row is read once for all simulations and every per-simulation load of a
// contact (infectious-mask word, rate adjoint) is a contiguous group access.
// Simulation b uses parameter set b % n_sets and Philox stream
// stream0 + b / n_sets (sets of one replicate share random numbers) or
// stream0 + b (independent streams).
#pragma once

#include "gabm_device.h"

namespace gabm {

constexpr int kBBlock = 512;          // threads per block of the batched day kernels
constexpr int kBUnroll = 8;           // contacts of a row whose loads are in flight together
constexpr int kBMaxB = 256;           // simulations per batched run (4 per lane)
constexpr int kBAnyLdsWords = 8192;   // 'any simulation' bits held in LDS up to 2^19 agents

struct BSims {
  int32_t B;        // simulations
  int32_t n_sets;   // parameter sets (set of simulation b = b % n_sets)
  int32_t indep;    // 1: a Philox stream per simulation; 0: per replicate
  uint32_t stream0;
  int32_t bw;       // 32-bit mask words per agent
  int32_t LB;       // lanes per receiver group
};

struct BInitArgs {
  DGraph G;
  DParams P;
  Rng rng;
  BSims S;
  uint32_t* rec;                // [N*B]
  uint32_t* mI;                 // [N*bw] day-0 infectious bits
  uint32_t* mE;                 // [N*bw] day-0 exposed bits (all clear), or NULL
  unsigned long long* any;      // [any_words] agents infectious in some simulation
  double* cnt0;                 // [B][kSlots][kCnt]
};

struct BMaskArgs {
  DGraph G;
  BSims S;
  const uint32_t* rec;
  uint32_t* mI;
  uint32_t* mE;                 // or NULL
  unsigned long long* any;
};

struct BFwdArgs {
  DGraph G;
  DParams P;
  Rng rng;
  BSims S;
  int32_t t;
  const uint32_t* rec_in;
  uint32_t* rec_out;
  const uint32_t* mI;           // day t bits, [N*bw]
  const uint32_t* mE;           // or NULL (T_E = 0)
  uint32_t* mI_next;            // day t+1 bits, fully rewritten
  uint32_t* mE_next;
  const unsigned long long* any_cur;  // day t: infectious (or exposed, T_E > 0) in some simulation
  unsigned long long* any_next;       // day t+1, OR-ed
  unsigned long long* any_clr;        // day t+2, cleared
  int64_t any_words;
  float* A_st;                  // [N*B] or NULL
  uint8_t* fl_st;               // [N*B] or NULL: bit 0 susceptible, bit 1 draw
  double* cnt;                  // [B][K][kSlots][kCnt] or NULL
  unsigned int* work;           // tile counter of this launch (starts at 0)
};

struct BBwdArgs {
  DGraph G;
  DParams P;
  Rng rng;
  BSims S;
  int32_t t;
  int32_t do_gather;
  const float* g_cur;           // [N*B] g^t
  float* g_prev;                // [N*B] g^{t-1}
  float* ring;                  // [W][N*B]
  float* Sbar;                  // [N*B]
  const float* A_st;            // day t-1
  const uint8_t* fl_st;
  const double* Dbar;           // [B][K]
  const unsigned long long* gz_cur;  // agents with g^t != 0 in some simulation
  unsigned long long* gz_next;
  unsigned long long* gz_clr;
  int64_t any_words;
  double* gR;                   // [n_sets][K][kSlots]
  double* gS;                   // [n_sets][n_age][kSlots]
  double* gi0;                  // [n_sets][kSlots]
  unsigned int* work;
};

template <int SPL>
__global__ void k_binit(BInitArgs a);
template <int SPL>
__global__ void k_bmask(BMaskArgs a);
template <int SPL, bool ANY_LDS>
__global__ void k_bfwd(BFwdArgs a);
template <int SPL, bool ANY_LDS>
__global__ void k_bfwd64(BFwdArgs a);
template <int SPL, bool ANY_LDS>
__global__ void k_bbwd(BBwdArgs a);
template <int SPL, bool ANY_LDS>
__global__ void k_bbwd64(BBwdArgs a);

// dynamic LDS bytes of the day kernels
inline size_t bfwd_lds(int B, int64_t any_words, bool any_lds) {
  return (any_lds ? (size_t)any_words * 8 : 0) + (size_t)B * 6 * 4;
}
inline size_t bbwd_lds(int B, int n_age, int64_t any_words, bool any_lds) {
  return (any_lds ? (size_t)any_words * 8 : 0) + (size_t)B * (n_age + 1) * 8;
}

}  // namespace gabm
