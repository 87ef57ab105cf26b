// Batched day kernels: B simulations sharing one contact graph, one launch
// per day for all of them (layout and lane mapping: batched.h).
//
// Forward day (Section 3.1, Eq. 1-3, Progress, Aggregate): for receiver i and
// simulation b, A_ib = T_I * sum of w_ji over senders j infectious in b
// (+ T_E * the same over exposed senders), formed in double precision in
// contact order; then the draw, progress, the records and bit masks of day
// t+1 and the daily counts -- all in the lanes that formed the sums.
// Reverse step t (Appendix B; the adjoint of the same sum is a gather over the
// same receiver-sorted CSR because every contact is listed both ways):
// inf_bar^t_ib = sum of w_ij g^t_jb, recorded in the window ring, then the
// agent adjoint of day t-1 (or of the initial draw at t = 0) and the
// parameter-gradient partials.
//
// Work distribution: receiver tiles (at most kBTileCap contacts and
// kBTileRows receivers, a longer row alone) are taken from a per-launch
// counter by one lane group at a time.  Senders inactive in every simulation
// (not infectious in the forward, zero adjoint in the reverse) are skipped by
// a one-bit-per-agent mask held in LDS; the per-simulation loads of active
// senders are raw buffer loads whose offset is pushed out of range for
// skipped contacts, so the hardware returns 0 without a memory request.
#include "agent.h"
#include "batched.h"

namespace gabm {

namespace {

constexpr int kRsrcWord3 = 0x00020000;   // fourth word of a raw buffer descriptor (gfx9 family)
constexpr uint32_t kOut = 0x80000000u;   // an offset past every buffer: reads as 0

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, p ? (int)bytes : 0, kRsrcWord3);
}
__device__ __forceinline__ uint32_t rload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

// the simulations of one lane
template <int SPL>
struct Slots {
  int b[SPL];
  bool ok[SPL];
  int set[SPL];
  uint32_t strm[SPL];
  uint32_t widx[SPL];
  uint32_t bsh[SPL];
};

template <int SPL>
__device__ __forceinline__ Slots<SPL> lane_slots(const BSims& S, int gl) {
  Slots<SPL> o;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int b = gl + S.LB * s;
    o.ok[s] = b < S.B;
    const int bb = o.ok[s] ? b : 0;
    o.b[s] = bb;
    o.set[s] = bb % S.n_sets;
    o.strm[s] = S.stream0 + (uint32_t)(S.indep ? bb : bb / S.n_sets);
    o.widx[s] = (uint32_t)bb >> 5;
    o.bsh[s] = (uint32_t)bb & 31u;
  }
  return o;
}

// Lane-interleaved layout of the per-simulation vectors of the wide kernels
// (B > 32): entry of simulation lane + 64 s of agent r at (r * 64 + lane) * SPL + s,
// so a lane moves all its simulations with one vector access.
template <int SPL>
__device__ __forceinline__ int64_t il_index(int64_t r, int lane, int s) {
  return (r * 64 + lane) * SPL + s;
}
template <int SPL>
__device__ __forceinline__ void il_load(const float* p, float (&o)[SPL]) {
  if constexpr (SPL == 1) {
    o[0] = *p;
  } else if constexpr (SPL == 2) {
    const float2 v = *(const float2*)p;
    o[0] = v.x; o[1] = v.y;
  } else {
    const float4 v = *(const float4*)p;
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
}
template <int SPL>
__device__ __forceinline__ void il_store(float* p, const float (&v)[SPL]) {
  if constexpr (SPL == 1) {
    *p = v[0];
  } else if constexpr (SPL == 2) {
    *(float2*)p = make_float2(v[0], v[1]);
  } else {
    *(float4*)p = make_float4(v[0], v[1], v[2], v[3]);
  }
}
template <int SPL>
__device__ __forceinline__ void il_load_bytes(const uint8_t* p, uint32_t (&o)[SPL]) {
  if constexpr (SPL == 1) {
    o[0] = *p;
  } else if constexpr (SPL == 2) {
    const uint32_t v = *(const uint16_t*)p;
    o[0] = v & 0xFFu; o[1] = v >> 8;
  } else {
    const uint32_t v = *(const uint32_t*)p;
    o[0] = v & 0xFFu; o[1] = (v >> 8) & 0xFFu; o[2] = (v >> 16) & 0xFFu; o[3] = v >> 24;
  }
}
// SPL floats of a lane from a raw buffer (zeros for an offset out of range).
// The wide loads are read back through bit casts to plain words: indexing
// their vector result directly made the compiler narrow the load to its first
// word.
struct Words2 { uint32_t x[2]; };
struct Words4 { uint32_t x[4]; };
template <int SPL>
__device__ __forceinline__ void il_rload(__amdgpu_buffer_rsrc_t r, uint32_t off, float (&o)[SPL]) {
  if constexpr (SPL == 1) {
    o[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  } else if constexpr (SPL == 2) {
    const Words2 v = __builtin_bit_cast(Words2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    o[0] = __builtin_bit_cast(float, v.x[0]); o[1] = __builtin_bit_cast(float, v.x[1]);
  } else {
    const Words4 v = __builtin_bit_cast(Words4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = __builtin_bit_cast(float, v.x[j]);
  }
}

// this group's bits of a wave ballot (bit k = lane k of the group)
__device__ __forceinline__ unsigned long long group_bits(unsigned long long bal, int gq, int LB) {
  return LB == 64 ? bal : (bal >> (gq * LB)) & ((1ull << LB) - 1ull);
}

// the group leader writes agent r's mask words from the ballots of its lanes
template <int SPL>
__device__ __forceinline__ void put_bits(uint32_t* m, int64_t r, const BSims& S, int gl, int gq,
                                         const unsigned long long (&bal)[SPL]) {
  if (m == nullptr || gl != 0) return;
  uint32_t* row = m + r * S.bw;
  if (S.LB == 64) {
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      if (2 * s < S.bw) row[2 * s] = (uint32_t)bal[s];
      if (2 * s + 1 < S.bw) row[2 * s + 1] = (uint32_t)(bal[s] >> 32);
    }
  } else {
    row[0] = (uint32_t)group_bits(bal[0], gq, S.LB);
  }
}

template <int SPL>
__device__ __forceinline__ bool group_any(const unsigned long long (&bal)[SPL], int gq, int LB) {
  unsigned long long x = 0ull;
#pragma unroll
  for (int s = 0; s < SPL; ++s) x |= group_bits(bal[s], gq, LB);
  return x != 0ull;
}

template <bool LDS>
__device__ __forceinline__ bool any_bit(const unsigned long long* s_any, const unsigned long long* g_any, uint32_t c) {
  const unsigned long long w = LDS ? s_any[c >> 6] : g_any[c >> 6];
  return ((w >> (c & 63u)) & 1ull) != 0ull;
}

// next tile of this lane group (broadcast from the group leader)
__device__ __forceinline__ int next_tile(unsigned int* work, int gl, int gq, int LB) {
  int tile = 0;
  if (gl == 0) tile = (int)atomicAdd(work, 1u);
  return __shfl(tile, gq * LB);
}

// The forward day of receiver r in every simulation of the calling lane
// group, from its neighbour sums: draw, progress, stored values, the day-t+1
// mask words and 'any' bit, per-lane counts.
template <int SPL, bool IL>
__device__ __forceinline__ void fwd_agent(const BFwdArgs& a, const Slots<SPL>& sl, int gl, int gq, int r,
                                          const double (&aI)[SPL], const double (&aE)[SPL], bool withE,
                                          unsigned int (&cnt)[SPL][6]) {
  const DGraph& G = a.G;
  const DParams& P = a.P;
  const BSims& S = a.S;
  const int p = pop_of_agent(G, r);
  const uint32_t loc = (uint32_t)(r - G.pop_off[p]);
  const int age = G.age[r];
  unsigned long long bI[SPL], bE[SPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    uint32_t newst = ST_S;
    if (sl.ok[s]) {
      const int64_t idx = (int64_t)r * S.B + sl.b[s];
      const double A = P.TI * aI[s] + (withE ? P.TE * aE[s] : 0.0);
      const HardDay hd = hard_agent_day<false>(P, a.rng, sl.strm[s], a.t, sl.set[s], p, loc, age, A, a.rec_in[idx], nullptr);
      a.rec_out[idx] = hd.rec;
      const int64_t sidx = IL ? il_index<SPL>(r, gl, s) : idx;
      if (a.A_st) a.A_st[sidx] = (float)A;
      if (a.fl_st) a.fl_st[sidx] = (uint8_t)((hd.was_s ? 1u : 0u) | (hd.h ? 2u : 0u));
      newst = hd.newst;
      cnt[s][newst] += 1u;
      if (hd.removed) cnt[s][5] += 1u;
    }
    bI[s] = __ballot(sl.ok[s] && newst == ST_I);
    bE[s] = __ballot(sl.ok[s] && newst == ST_E);
  }
  put_bits<SPL>(a.mI_next, r, S, gl, gq, bI);
  if (withE) put_bits<SPL>(a.mE_next, r, S, gl, gq, bE);
  const bool act = group_any<SPL>(bI, gq, S.LB) || (withE && group_any<SPL>(bE, gq, S.LB));
  if (gl == 0 && act) atomicOr(&a.any_next[r >> 6], 1ull << (r & 63));
}

// per-lane counts of a block into the day's FP64 aggregates
template <int SPL>
__device__ __forceinline__ void fwd_counts(const BFwdArgs& a, const Slots<SPL>& sl, unsigned int* s_cnt,
                                           const unsigned int (&cnt)[SPL][6]) {
#pragma unroll
  for (int s = 0; s < SPL; ++s)
    if (sl.ok[s])
#pragma unroll
      for (int c = 0; c < 6; ++c)
        if (cnt[s][c]) atomicAdd(&s_cnt[sl.b[s] * 6 + c], cnt[s][c]);
  __syncthreads();
  const int slot = blockIdx.x & (kSlots - 1);
  for (int x = threadIdx.x; x < a.S.B * 6; x += kBBlock) {
    const unsigned int v = s_cnt[x];
    if (v) atomicAdd(&a.cnt[(((int64_t)(x / 6) * a.P.K + a.t) * kSlots + slot) * kCnt + x % 6], (double)v);
  }
}

}  // namespace

// ----------------------------------------------------------------- initial infections
// One lane group per agent: the INIT draw of every simulation (Bernoulli(i0)
// of its set, entering I with a full timer), the day-0 masks and counts.
template <int SPL>
__global__ void __launch_bounds__(kBBlock) k_binit(BInitArgs a) {
  __shared__ double s_c[kBMaxB * 2];
  const int tid = threadIdx.x;
  const DGraph& G = a.G;
  const DParams& P = a.P;
  const BSims& S = a.S;
  for (int x = tid; x < S.B * 2; x += kBBlock) s_c[x] = 0.0;
  __syncthreads();
  const int LB = S.LB, lane = tid & 63, gl = lane & (LB - 1), gq = lane / LB;
  const Slots<SPL> sl = lane_slots<SPL>(S, gl);
  double cS[SPL], cI[SPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) cS[s] = cI[s] = 0.0;
  const int64_t per_block = kBBlock / LB;
  const int64_t ng = (int64_t)gridDim.x * per_block;
  for (int64_t i = blockIdx.x * per_block + tid / LB; i < G.N; i += ng) {
    const int p = pop_of_agent(G, (int)i);
    const uint32_t loc = (uint32_t)(i - G.pop_off[p]);
    unsigned long long bI[SPL], bE[SPL];
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      bool inf = false;
      if (sl.ok[s]) {
        const double u = unit_u(rng_block(a.rng, loc, kDayInit, TAG_INIT, (uint32_t)p, sl.strm[s]).x);
        inf = u < (double)P.i0[sl.set[s]];
        a.rec[i * S.B + sl.b[s]] = inf ? make_rec(ST_I, (uint32_t)P.tau_I, -1) : make_rec(ST_S, 0, -1);
        if (inf) cI[s] += 1.0; else cS[s] += 1.0;
      }
      bI[s] = __ballot(sl.ok[s] && inf);
      bE[s] = 0ull;
    }
    put_bits<SPL>(a.mI, i, S, gl, gq, bI);
    put_bits<SPL>(a.mE, i, S, gl, gq, bE);
    if (gl == 0 && group_any<SPL>(bI, gq, LB)) atomicOr(&a.any[i >> 6], 1ull << (i & 63));
  }
#pragma unroll
  for (int s = 0; s < SPL; ++s)
    if (sl.ok[s]) {
      if (cS[s] != 0.0) atomicAdd(&s_c[sl.b[s] * 2], cS[s]);
      if (cI[s] != 0.0) atomicAdd(&s_c[sl.b[s] * 2 + 1], cI[s]);
    }
  __syncthreads();
  const int slot = blockIdx.x & (kSlots - 1);
  for (int x = tid; x < S.B * 2; x += kBBlock) {
    const double v = s_c[x];
    if (v != 0.0) atomicAdd(&a.cnt0[((int64_t)(x >> 1) * kSlots + slot) * kCnt + ((x & 1) ? ST_I : ST_S)], v);
  }
}

// masks of the current day rebuilt from the records (checkpoint restore)
template <int SPL>
__global__ void __launch_bounds__(kBBlock) k_bmask(BMaskArgs a) {
  const int tid = threadIdx.x;
  const BSims& S = a.S;
  const int LB = S.LB, lane = tid & 63, gl = lane & (LB - 1), gq = lane / LB;
  const Slots<SPL> sl = lane_slots<SPL>(S, gl);
  const int64_t per_block = kBBlock / LB;
  const int64_t ng = (int64_t)gridDim.x * per_block;
  for (int64_t i = blockIdx.x * per_block + tid / LB; i < a.G.N; i += ng) {
    unsigned long long bI[SPL], bE[SPL];
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      const uint32_t st = sl.ok[s] ? rec_stage(a.rec[i * S.B + sl.b[s]]) : ST_S;
      bI[s] = __ballot(sl.ok[s] && st == ST_I);
      bE[s] = __ballot(sl.ok[s] && st == ST_E);
    }
    put_bits<SPL>(a.mI, i, S, gl, gq, bI);
    put_bits<SPL>(a.mE, i, S, gl, gq, bE);
    const bool act = group_any<SPL>(bI, gq, LB) || (a.mE != nullptr && group_any<SPL>(bE, gq, LB));
    if (gl == 0 && act) atomicOr(&a.any[i >> 6], 1ull << (i & 63));
  }
}

// ----------------------------------------------------------------- forward day
template <int SPL, bool ANY_LDS>
__global__ void __launch_bounds__(kBBlock) k_bfwd(BFwdArgs a) {
  extern __shared__ unsigned long long lds[];
  unsigned long long* s_any = lds;
  unsigned int* s_cnt = (unsigned int*)(lds + (ANY_LDS ? a.any_words : 0));
  const int tid = threadIdx.x;
  const DGraph& G = a.G;
  const DParams& P = a.P;
  const BSims& S = a.S;
  for (int x = tid; x < S.B * 6; x += kBBlock) s_cnt[x] = 0u;
  if (ANY_LDS)
    lds_fill<kBBlock, kBAnyLdsWords>(s_any, a.any_cur, (int)a.any_words);
  // the 'any' words of day t+2 (read last on day t-1, OR-ed next on day t+1)
  for (int64_t x = blockIdx.x * (int64_t)kBBlock + tid; x < a.any_words; x += (int64_t)gridDim.x * kBBlock)
    a.any_clr[x] = 0ull;
  __syncthreads();
  const int LB = S.LB, lane = tid & 63, gl = lane & (LB - 1), gq = lane / LB;
  const Slots<SPL> sl = lane_slots<SPL>(S, gl);
  const bool withE = a.mE != nullptr;
  const int64_t mbytes = (int64_t)G.N * S.bw * 4;
  const __amdgpu_buffer_rsrc_t rI = rsrc(a.mI, mbytes);
  const __amdgpu_buffer_rsrc_t rE = rsrc(a.mE, mbytes);
  unsigned int cnt[SPL][6];
#pragma unroll
  for (int s = 0; s < SPL; ++s)
#pragma unroll
    for (int c = 0; c < 6; ++c) cnt[s][c] = 0u;

  for (;;) {
    const int tile = next_tile(a.work, gl, gq, LB);
    if (tile >= G.n_btiles) break;
    const TileInfo ti = G.btiles[tile];
    int64_t e = ti.e0;
    int64_t e_next = G.row_ptr[ti.r0 + 1];
    for (int r = ti.r0; r < ti.r1; ++r) {
      const int64_t e1 = e_next;
      if (r + 1 < ti.r1) e_next = G.row_ptr[r + 2];
      double aI[SPL], aE[SPL];
#pragma unroll
      for (int s = 0; s < SPL; ++s) aI[s] = aE[s] = 0.0;
      for (; e < e1; e += kBUnroll) {
        uint32_t c[kBUnroll];
        float w[kBUnroll];
#pragma unroll
        for (int k = 0; k < kBUnroll; ++k) {
          const int64_t pos = e + k < e1 ? e + k : e1 - 1;
          c[k] = (uint32_t)G.col[pos];
          w[k] = G.w[pos];
        }
        uint32_t vi[kBUnroll][SPL], ve[kBUnroll][SPL];
#pragma unroll
        for (int k = 0; k < kBUnroll; ++k) {
          const bool need = (e + k < e1) && any_bit<ANY_LDS>(s_any, a.any_cur, c[k]);
#pragma unroll
          for (int s = 0; s < SPL; ++s) {
            const uint32_t off = need ? (c[k] * (uint32_t)S.bw + sl.widx[s]) * 4u : kOut;
            vi[k][s] = rload(rI, off);
            ve[k][s] = withE ? rload(rE, off) : 0u;
          }
        }
#pragma unroll
        for (int k = 0; k < kBUnroll; ++k)
#pragma unroll
          for (int s = 0; s < SPL; ++s) {
            if ((vi[k][s] >> sl.bsh[s]) & 1u) aI[s] += (double)w[k];
            if ((ve[k][s] >> sl.bsh[s]) & 1u) aE[s] += (double)w[k];
          }
      }
      e = e1;
      fwd_agent<SPL, false>(a, sl, gl, gq, r, aI, aE, withE, cnt);
    }
  }
  if (a.cnt != nullptr) fwd_counts<SPL>(a, sl, s_cnt, cnt);
}

// ----------------------------------------------------------------- forward day, B > 32 (one wave per tile)
// Lanes are simulations (b = lane + 64 s).  A tile's contacts are read 64 at
// a time, one per lane: the packed sender with its row-start count, the
// weight, and every mask word of the sender (zero, without a memory request,
// when the sender is infectious in no simulation).  A window therefore costs
// a few vector memory instructions instead of several per contact; the wave
// then walks the window's active contacts and row starts (two ballots) and
// reads each contact's values from the lane that loaded them.
template <int SPL, bool ANY_LDS>
__global__ void __launch_bounds__(kBBlock, 4) k_bfwd64(BFwdArgs a) {
  extern __shared__ unsigned long long lds[];
  unsigned long long* s_any = lds;
  unsigned int* s_cnt = (unsigned int*)(lds + (ANY_LDS ? a.any_words : 0));
  const int tid = threadIdx.x;
  const DGraph& G = a.G;
  const BSims& S = a.S;
  for (int x = tid; x < S.B * 6; x += kBBlock) s_cnt[x] = 0u;
  if (ANY_LDS)
    lds_fill<kBBlock, kBAnyLdsWords>(s_any, a.any_cur, (int)a.any_words);
  for (int64_t x = blockIdx.x * (int64_t)kBBlock + tid; x < a.any_words; x += (int64_t)gridDim.x * kBBlock)
    a.any_clr[x] = 0ull;
  __syncthreads();
  constexpr int MW = 2 * SPL;  // mask words a lane may need (bw <= MW)
  const int lane = tid & 63;
  const Slots<SPL> sl = lane_slots<SPL>(S, lane);
  const bool withE = a.mE != nullptr;
  const int64_t mbytes = (int64_t)G.N * S.bw * 4;
  const __amdgpu_buffer_rsrc_t rI = rsrc(a.mI, mbytes);
  const __amdgpu_buffer_rsrc_t rE = rsrc(a.mE, mbytes);
  unsigned int cnt[SPL][6];
#pragma unroll
  for (int s = 0; s < SPL; ++s)
#pragma unroll
    for (int c = 0; c < 6; ++c) cnt[s][c] = 0u;
  double aI[SPL], aE[SPL];

  for (;;) {
    const int tile = next_tile(a.work, lane, 0, 64);
    if (tile >= G.n_btiles) break;
    const TileInfo ti = G.btiles[tile];
    int open = ti.r0 - 1;  // receiver of the running sums (none yet)
#pragma unroll
    for (int s = 0; s < SPL; ++s) aI[s] = aE[s] = 0.0;
    // windows of 64 contacts, then one closing window without contacts whose
    // single row-start event closes the open receiver and the empty ones after it
    for (int64_t wb = ti.e0;; wb += 64) {
      const bool fin = wb >= ti.e1;
      const int nwin = fin ? 0 : (int)(ti.e1 - wb < 64 ? ti.e1 - wb : 64);
      const bool okc = lane < nwin;
      const int64_t pos = okc ? wb + lane : (fin ? ti.e0 : wb);
      const uint32_t pk = okc ? G.colp[pos] : 0u;
      const float wl = okc ? G.wp[pos] : 0.f;
      const uint32_t c = pk & 0xFFFFFFu;
      int adv = (int)(pk >> 24);
      if (lane == 0) {
        if (fin) adv = ti.r1 - open;
        else if (wb == ti.e0) adv -= ti.pad0;  // rows of earlier tiles starting here
      }
      const bool need = okc && any_bit<ANY_LDS>(s_any, a.any_cur, c);
      uint32_t mi[MW], me[MW];
#pragma unroll
      for (int q = 0; q < MW; ++q) {
        const uint32_t off = (need && q < S.bw) ? (c * (uint32_t)S.bw + (uint32_t)q) * 4u : kOut;
        mi[q] = rload(rI, off);
        me[q] = withE ? rload(rE, off) : 0u;
      }
      const unsigned long long rs = __ballot(adv > 0);
      const unsigned long long nd = __ballot(need);
      unsigned long long todo = rs | nd;
      while (todo) {
        const int k = __builtin_ctzll(todo);
        todo &= todo - 1ull;
        if ((rs >> k) & 1ull) {
          for (int na = __builtin_amdgcn_readlane(adv, k); na > 0; --na) {
            if (open >= ti.r0) fwd_agent<SPL, true>(a, sl, lane, 0, open, aI, aE, withE, cnt);
#pragma unroll
            for (int s = 0; s < SPL; ++s) aI[s] = aE[s] = 0.0;
            ++open;
          }
        }
        if ((nd >> k) & 1ull) {
          const double wk = (double)__builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wl), k));
#pragma unroll
          for (int s = 0; s < SPL; ++s) {
            // words 2s, 2s+1 of the sender are the bits of simulations lane + 64 s,
            // i.e. a lane mask: the add runs under it
            const uint64_t mI = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)mi[2 * s + 1], k) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int)mi[2 * s], k);
            if (__builtin_amdgcn_inverse_ballot_w64(mI)) aI[s] += wk;
            if (withE) {
              const uint64_t mE = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)me[2 * s + 1], k) << 32) |
                                  (uint32_t)__builtin_amdgcn_readlane((int)me[2 * s], k);
              if (__builtin_amdgcn_inverse_ballot_w64(mE)) aE[s] += wk;
            }
          }
        }
      }
      if (fin) break;
    }
  }
  if (a.cnt != nullptr) fwd_counts<SPL>(a, sl, s_cnt, cnt);
}

// ----------------------------------------------------------------- reverse step
template <int SPL, bool ANY_LDS>
__global__ void __launch_bounds__(kBBlock) k_bbwd(BBwdArgs a) {
  extern __shared__ unsigned long long lds[];
  const int tid = threadIdx.x;
  const DGraph& G = a.G;
  const DParams& P = a.P;
  const BSims& S = a.S;
  unsigned long long* s_any = lds;
  double* s_gS = (double*)(lds + (ANY_LDS ? a.any_words : 0));  // [B][n_age] sum of lam_bar * A / Z
  double* s_gi0 = s_gS + (int64_t)S.B * P.n_age;                 // [B]
  for (int x = tid; x < S.B * (P.n_age + 1); x += kBBlock) s_gS[x] = 0.0;
  if (ANY_LDS && a.do_gather)
    lds_fill<kBBlock, kBAnyLdsWords>(s_any, a.gz_cur, (int)a.any_words);
  for (int64_t x = blockIdx.x * (int64_t)kBBlock + tid; x < a.any_words; x += (int64_t)gridDim.x * kBBlock)
    a.gz_clr[x] = 0ull;
  __syncthreads();
  const int LB = S.LB, lane = tid & 63, gl = lane & (LB - 1), gq = lane / LB;
  const Slots<SPL> sl = lane_slots<SPL>(S, gl);
  const int t = a.t;
  const int W = P.tau_E + P.tau_I;
  const int64_t NB = (int64_t)G.N * S.B;
  const __amdgpu_buffer_rsrc_t rg = rsrc(a.g_cur, NB * 4);

  for (;;) {
    const int tile = next_tile(a.work, gl, gq, LB);
    if (tile >= G.n_btiles) break;
    const TileInfo ti = G.btiles[tile];
    int64_t e = ti.e0;
    int64_t e_next = G.row_ptr[ti.r0 + 1];
    for (int r = ti.r0; r < ti.r1; ++r) {
      const int64_t e1 = e_next;
      if (r + 1 < ti.r1) e_next = G.row_ptr[r + 2];
      double acc[SPL];
#pragma unroll
      for (int s = 0; s < SPL; ++s) acc[s] = 0.0;
      if (a.do_gather) {
        for (; e < e1; e += kBUnroll) {
          uint32_t c[kBUnroll];
          float w[kBUnroll];
#pragma unroll
          for (int k = 0; k < kBUnroll; ++k) {
            const int64_t pos = e + k < e1 ? e + k : e1 - 1;
            c[k] = (uint32_t)G.col[pos];
            w[k] = G.w[pos];
          }
          uint32_t v[kBUnroll][SPL];
#pragma unroll
          for (int k = 0; k < kBUnroll; ++k) {
            const bool need = (e + k < e1) && any_bit<ANY_LDS>(s_any, a.gz_cur, c[k]);
#pragma unroll
            for (int s = 0; s < SPL; ++s)
              v[k][s] = rload(rg, need ? (c[k] * (uint32_t)S.B + (uint32_t)sl.b[s]) * 4u : kOut);
          }
#pragma unroll
          for (int k = 0; k < kBUnroll; ++k)
#pragma unroll
            for (int s = 0; s < SPL; ++s) acc[s] += (double)w[k] * (double)__builtin_bit_cast(float, v[k][s]);
        }
      }
      e = e1;
      const int p = pop_of_agent(G, r);
      const uint32_t loc = (uint32_t)(r - G.pop_off[p]);
      const int age = G.age[r];
      unsigned long long bz[SPL];
#pragma unroll
      for (int s = 0; s < SPL; ++s) {
        float gnew = 0.f;
        if (sl.ok[s]) {
          const int b = sl.b[s], set = sl.set[s];
          const int64_t idx = (int64_t)r * S.B + b;
          if (a.do_gather) a.ring[(int64_t)(t % W) * NB + idx] = (float)acc[s];
          const double Sbar1 = (double)a.Sbar[idx];
          const double m = (double)P.m[set];
          if (t >= 1) {
            const int d = t - 1;
            double sE = 0.0, sI = 0.0;
            for (int k = 1; k <= W; ++k) {
              const double v = (double)a.ring[(int64_t)((d + k) % W) * NB + idx];
              if (k <= P.tau_E) sE += v; else sI += v;
            }
            const double drm_bar = (d + W < P.K) ? m * a.Dbar[(int64_t)b * P.K + d + W] : 0.0;
            const uint32_t fl = a.fl_st[idx];
            const double Aday = (double)a.A_st[idx];
            const AdjOut ad = agent_adjoint<true>(P, a.rng, sl.strm[s], d, set, p, loc, age, Aday, (double)(fl & 1u),
                                            (double)((fl >> 1) & 1u), false, sE, sI, Sbar1, drm_bar);
            a.Sbar[idx] = (float)ad.Sbar;
            a.g_prev[idx] = (float)ad.g;
            gnew = (float)ad.g;
            if (ad.lam_bar != 0.0) atomicAdd(&s_gS[b * P.n_age + age], ad.lam_bar * Aday / (double)P.Z[p]);
          } else {
            double sI = 0.0;
            for (int k = 0; k < P.tau_I; ++k) sI += (double)a.ring[(int64_t)(k % W) * NB + idx];
            const double x0_bar = P.TI * sI + ((P.tau_I - 1 < P.K) ? m * a.Dbar[(int64_t)b * P.K + P.tau_I - 1] : 0.0) - Sbar1;
            const double u = unit_u(rng_block(a.rng, loc, kDayInit, TAG_INIT, (uint32_t)p, sl.strm[s]).x);
            double y0, dy0;
            relaxed_init((double)P.i0[set], u, P.tau, y0, dy0);
            const double v = x0_bar * dy0;
            if (v != 0.0) atomicAdd(&s_gi0[b], v);
          }
        }
        bz[s] = __ballot(sl.ok[s] && gnew != 0.f);
      }
      if (gl == 0 && group_any<SPL>(bz, gq, LB)) atomicOr(&a.gz_next[r >> 6], 1ull << (r & 63));
    }
  }
  __syncthreads();
  const int slot = blockIdx.x & (kSlots - 1);
  if (t >= 1) {
    const int d = t - 1;
    for (int x = tid; x < S.B * P.n_age; x += kBBlock) {
      const double v = s_gS[x];
      if (v != 0.0) {
        const int set = (x / P.n_age) % S.n_sets, g = x % P.n_age;
        atomicAdd(&a.gS[((int64_t)set * P.n_age + g) * kSlots + slot], v * (double)P.R[set * P.K + d]);
      }
    }
    for (int b = tid; b < S.B; b += kBBlock) {
      const int set = b % S.n_sets;
      double acc = 0.0;
      for (int g = 0; g < P.n_age; ++g) acc += s_gS[b * P.n_age + g] * (double)P.S[set * P.n_age + g];
      if (acc != 0.0) atomicAdd(&a.gR[((int64_t)set * P.K + d) * kSlots + slot], acc);
    }
  } else {
    for (int b = tid; b < S.B; b += kBBlock) {
      const double v = s_gi0[b];
      if (v != 0.0) atomicAdd(&a.gi0[(int64_t)(b % S.n_sets) * kSlots + slot], v);
    }
  }
}

// ----------------------------------------------------------------- reverse step, B > 32 (one wave per tile)
// Lanes are simulations; the per-simulation vectors use the lane-interleaved
// layout, so the rate adjoints of one contact's sender are a single
// SPL-float load per lane.  Contacts are read 64 at a time, one per lane
// (packed sender with row starts, weight); the wave walks the window's row
// segments, gathering up to kBGather active senders of a segment at once.
constexpr int kBGather = 8;

template <int SPL>
__device__ __forceinline__ void bwd_agent64(const BBwdArgs& a, const Slots<SPL>& sl, int lane, int r,
                                            const double (&acc)[SPL], int64_t NV, double* s_gS, double* s_gi0) {
  const DGraph& G = a.G;
  const DParams& P = a.P;
  const int t = a.t;
  const int W = P.tau_E + P.tau_I;
  const int p = pop_of_agent(G, r);
  const uint32_t loc = (uint32_t)(r - G.pop_off[p]);
  const int age = G.age[r];
  const int64_t il = il_index<SPL>(r, lane, 0);
  if (a.do_gather) {
    float v[SPL];
#pragma unroll
    for (int s = 0; s < SPL; ++s) v[s] = (float)acc[s];
    il_store<SPL>(a.ring + (int64_t)(t % W) * NV + il, v);
  }
  float sb[SPL];
  il_load<SPL>(a.Sbar + il, sb);
  bool gnz = false;
  if (t >= 1) {
    const int d = t - 1;
    double sE[SPL], sI[SPL];
#pragma unroll
    for (int s = 0; s < SPL; ++s) sE[s] = sI[s] = 0.0;
    for (int k = 1; k <= W; ++k) {
      float v[SPL];
      il_load<SPL>(a.ring + (int64_t)((d + k) % W) * NV + il, v);
#pragma unroll
      for (int s = 0; s < SPL; ++s) {
        if (k <= P.tau_E) sE[s] += (double)v[s]; else sI[s] += (double)v[s];
      }
    }
    float Ad[SPL];
    uint32_t fl[SPL];
    il_load<SPL>(a.A_st + il, Ad);
    il_load_bytes<SPL>(a.fl_st + il, fl);
    float sb_new[SPL], g_new[SPL];
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      sb_new[s] = sb[s];
      g_new[s] = 0.f;
      if (sl.ok[s]) {
        const int b = sl.b[s], set = sl.set[s];
        const double drm_bar = (d + W < P.K) ? (double)P.m[set] * a.Dbar[(int64_t)b * P.K + d + W] : 0.0;
        const double Aday = (double)Ad[s];
        const AdjOut ad = agent_adjoint<true>(P, a.rng, sl.strm[s], d, set, p, loc, age, Aday, (double)(fl[s] & 1u),
                                        (double)((fl[s] >> 1) & 1u), false, sE[s], sI[s], (double)sb[s], drm_bar);
        sb_new[s] = (float)ad.Sbar;
        g_new[s] = (float)ad.g;
        if (g_new[s] != 0.f) gnz = true;
        if (ad.lam_bar != 0.0) atomicAdd(&s_gS[b * P.n_age + age], ad.lam_bar * Aday / (double)P.Z[p]);
      }
    }
    il_store<SPL>(a.Sbar + il, sb_new);
    il_store<SPL>(a.g_prev + il, g_new);
  } else {
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      if (!sl.ok[s]) continue;
      const int b = sl.b[s], set = sl.set[s];
      double sI = 0.0;
      for (int k = 0; k < P.tau_I; ++k) {
        float v[SPL];
        il_load<SPL>(a.ring + (int64_t)(k % W) * NV + il, v);
        sI += (double)v[s];
      }
      const double m = (double)P.m[set];
      const double x0_bar =
          P.TI * sI + ((P.tau_I - 1 < P.K) ? m * a.Dbar[(int64_t)b * P.K + P.tau_I - 1] : 0.0) - (double)sb[s];
      const double u = unit_u(rng_block(a.rng, loc, kDayInit, TAG_INIT, (uint32_t)p, sl.strm[s]).x);
      double y0, dy0;
      relaxed_init((double)P.i0[set], u, P.tau, y0, dy0);
      const double v = x0_bar * dy0;
      if (v != 0.0) atomicAdd(&s_gi0[b], v);
    }
  }
  if (__ballot(gnz) != 0ull && lane == 0) atomicOr(&a.gz_next[r >> 6], 1ull << (r & 63));
}

template <int SPL, bool ANY_LDS>
__global__ void __launch_bounds__(kBBlock, 4) k_bbwd64(BBwdArgs a) {
  extern __shared__ unsigned long long lds[];
  const int tid = threadIdx.x;
  const DGraph& G = a.G;
  const DParams& P = a.P;
  const BSims& S = a.S;
  unsigned long long* s_any = lds;
  double* s_gS = (double*)(lds + (ANY_LDS ? a.any_words : 0));  // [B][n_age] sum of lam_bar * A / Z
  double* s_gi0 = s_gS + (int64_t)S.B * P.n_age;                 // [B]
  for (int x = tid; x < S.B * (P.n_age + 1); x += kBBlock) s_gS[x] = 0.0;
  if (ANY_LDS && a.do_gather)
    lds_fill<kBBlock, kBAnyLdsWords>(s_any, a.gz_cur, (int)a.any_words);
  for (int64_t x = blockIdx.x * (int64_t)kBBlock + tid; x < a.any_words; x += (int64_t)gridDim.x * kBBlock)
    a.gz_clr[x] = 0ull;
  __syncthreads();
  const int lane = tid & 63;
  const Slots<SPL> sl = lane_slots<SPL>(S, lane);
  const int64_t NV = (int64_t)G.N * 64 * SPL;
  const __amdgpu_buffer_rsrc_t rg = rsrc(a.g_cur, NV * 4);
  double acc[SPL];

  for (;;) {
    const int tile = next_tile(a.work, lane, 0, 64);
    if (tile >= G.n_btiles) break;
    const TileInfo ti = G.btiles[tile];
    int open = ti.r0 - 1;
#pragma unroll
    for (int s = 0; s < SPL; ++s) acc[s] = 0.0;
    for (int64_t wb = ti.e0;; wb += 64) {
      const bool fin = wb >= ti.e1;
      const int nwin = fin ? 0 : (int)(ti.e1 - wb < 64 ? ti.e1 - wb : 64);
      const bool okc = lane < nwin;
      const int64_t pos = okc ? wb + lane : ti.e0;
      const uint32_t pk = okc ? G.colp[pos] : 0u;
      const float wl = okc ? G.wp[pos] : 0.f;
      const uint32_t c = pk & 0xFFFFFFu;
      int adv = (int)(pk >> 24);
      if (lane == 0) {
        if (fin) adv = ti.r1 - open;
        else if (wb == ti.e0) adv -= ti.pad0;
      }
      const bool need = a.do_gather && okc && any_bit<ANY_LDS>(s_any, a.gz_cur, c);
      const unsigned long long rs = __ballot(adv > 0);
      const unsigned long long nd = __ballot(need);
      // row segments of the window: [k0, next row start)
      int k0 = 0;
      for (;;) {
        if ((rs >> k0) & 1ull) {
          for (int na = __builtin_amdgcn_readlane(adv, k0); na > 0; --na) {
            if (open >= ti.r0) bwd_agent64<SPL>(a, sl, lane, open, acc, NV, s_gS, s_gi0);
#pragma unroll
            for (int s = 0; s < SPL; ++s) acc[s] = 0.0;
            ++open;
          }
        }
        const unsigned long long after = k0 < 63 ? (rs >> (k0 + 1)) << (k0 + 1) : 0ull;
        const int k1 = after ? __builtin_ctzll(after) : 64;
        unsigned long long act = nd & (k1 < 64 ? ((1ull << k1) - 1ull) : ~0ull) & ~((1ull << k0) - 1ull);
        while (act) {
          uint32_t off[kBGather];
          float wk[kBGather];
#pragma unroll
          for (int u = 0; u < kBGather; ++u) {
            off[u] = kOut;
            wk[u] = 0.f;
            if (act) {
              const int k = __builtin_ctzll(act);
              act &= act - 1ull;
              const uint32_t ck = (uint32_t)__builtin_amdgcn_readlane((int)c, k);
              off[u] = (uint32_t)il_index<SPL>(ck, lane, 0) * 4u;
              wk[u] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wl), k));
            }
          }
          float gv[kBGather][SPL];
#pragma unroll
          for (int u = 0; u < kBGather; ++u) il_rload<SPL>(rg, off[u], gv[u]);
#pragma unroll
          for (int u = 0; u < kBGather; ++u)
#pragma unroll
            for (int s = 0; s < SPL; ++s) acc[s] += (double)wk[u] * (double)gv[u][s];
        }
        if (k1 >= 64) break;
        k0 = k1;
      }
      if (fin) break;
    }
  }
  __syncthreads();
  const int slot = blockIdx.x & (kSlots - 1);
  if (a.t >= 1) {
    const int d = a.t - 1;
    for (int x = tid; x < S.B * P.n_age; x += kBBlock) {
      const double v = s_gS[x];
      if (v != 0.0) {
        const int set = (x / P.n_age) % S.n_sets, g = x % P.n_age;
        atomicAdd(&a.gS[((int64_t)set * P.n_age + g) * kSlots + slot], v * (double)P.R[set * P.K + d]);
      }
    }
    for (int b = tid; b < S.B; b += kBBlock) {
      const int set = b % S.n_sets;
      double sum = 0.0;
      for (int g = 0; g < P.n_age; ++g) sum += s_gS[b * P.n_age + g] * (double)P.S[set * P.n_age + g];
      if (sum != 0.0) atomicAdd(&a.gR[((int64_t)set * P.K + d) * kSlots + slot], sum);
    }
  } else {
    for (int b = tid; b < S.B; b += kBBlock) {
      const double v = s_gi0[b];
      if (v != 0.0) atomicAdd(&a.gi0[(int64_t)(b % S.n_sets) * kSlots + slot], v);
    }
  }
}

template __global__ void k_binit<1>(BInitArgs);
template __global__ void k_binit<2>(BInitArgs);
template __global__ void k_binit<4>(BInitArgs);
template __global__ void k_bmask<1>(BMaskArgs);
template __global__ void k_bmask<2>(BMaskArgs);
template __global__ void k_bmask<4>(BMaskArgs);
template __global__ void k_bfwd<1, true>(BFwdArgs);
template __global__ void k_bfwd<2, true>(BFwdArgs);
template __global__ void k_bfwd<4, true>(BFwdArgs);
template __global__ void k_bfwd<1, false>(BFwdArgs);
template __global__ void k_bfwd<2, false>(BFwdArgs);
template __global__ void k_bfwd<4, false>(BFwdArgs);
template __global__ void k_bfwd64<1, true>(BFwdArgs);
template __global__ void k_bfwd64<2, true>(BFwdArgs);
template __global__ void k_bfwd64<4, true>(BFwdArgs);
template __global__ void k_bfwd64<1, false>(BFwdArgs);
template __global__ void k_bfwd64<2, false>(BFwdArgs);
template __global__ void k_bfwd64<4, false>(BFwdArgs);
template __global__ void k_bbwd64<1, true>(BBwdArgs);
template __global__ void k_bbwd64<2, true>(BBwdArgs);
template __global__ void k_bbwd64<4, true>(BBwdArgs);
template __global__ void k_bbwd64<1, false>(BBwdArgs);
template __global__ void k_bbwd64<2, false>(BBwdArgs);
template __global__ void k_bbwd64<4, false>(BBwdArgs);
template __global__ void k_bbwd<1, true>(BBwdArgs);
template __global__ void k_bbwd<2, true>(BBwdArgs);
template __global__ void k_bbwd<4, true>(BBwdArgs);
template __global__ void k_bbwd<1, false>(BBwdArgs);
template __global__ void k_bbwd<2, false>(BBwdArgs);
template __global__ void k_bbwd<4, false>(BBwdArgs);

}  // namespace gabm
