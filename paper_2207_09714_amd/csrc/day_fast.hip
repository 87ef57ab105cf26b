// Split day kernels (float state, one simulation -- one parameter set, or one
// per packed population -- fewer than 2^24 agents): a persistent neighbour-sum
// kernel and an element-wise agent kernel.
//
// Neighbour sum.  One 1024-thread block per compute unit; the gathered side
// is a one-bit-per-agent mask held in LDS -- the infectious mask in the
// forward, the mask of non-zero rate adjoints g in the reverse pass -- so a
// gather costs an LDS read, and the reverse pass reads g from memory only for
// senders whose bit is set.  The contact list is split by sender into slices
// of 2^20 agents, whose mask fits the LDS; each slice is its own
// receiver-sorted stream and yields its own partial row sums, added in slice
// order by the agent pass.  The chunks of all slices are cut into one
// contiguous range per block; a block reloads the mask when its range enters
// the next slice, and ranges are numbered so that the blocks of one XCD
// share a contiguous part of the stream (and of the g vector in its L2).
// Each wave streams its own chunks of the block's range (see below), with
// loads software-pipelined across chunks.  Sums are double-precision sums of
// the same float terms in a fixed order.
//
// Agent pass.  One thread per agent finishes the day with the per-agent
// functions of agent.h (Section 3.1, Eq. 1-3 and Progress; the
// straight-through adjoint), so the serial per-agent arithmetic runs at full
// occupancy instead of inside the streaming loop.
#include "agent.h"
#include "day_kernels.h"
#include "loc.h"

namespace gabm {

// mask bit of a sender of the slice held in LDS: the slice's senders lie in
// [p << kSliceShift, (p + 1) << kSliceShift), so the low kSliceShift bits are
// the slice-local index; 32-bit words, one bit-field extract
__device__ __forceinline__ uint32_t lds_bit(const unsigned long long* m, uint32_t sender) {
  const uint32_t c = sender & ((1u << kSliceShift) - 1u);
  return __builtin_amdgcn_ubfe(((const uint32_t*)m)[c >> 5], c & 31u, 1u);
}

// ---------------------------------------------------------------- wave-parallel neighbour sum
//
// The destination-sorted contact list is cut into chunks of kChunk = 256
// contacts; a wave owns a chunk, lane l its contacts 4l .. 4l+3 (16-byte
// loads).  The packed sender carries, in its top byte, the number of rows
// (receivers) that start at that contact, so an integer prefix sum over the
// wave gives every contact's receiver and no row offsets are read.  Values
// stay in registers: each lane sums its contacts with a restart at each row
// start, a segmented scan over the wave carries partial sums between lanes,
// and the lane holding a row's last contact writes the row sum.  A row that
// crosses a chunk boundary leaves one piece per chunk (first_piece: the part
// of the row that began before the chunk; last_piece: the part of the
// chunk's last row that continues after it), added in chunk order by the
// agent pass; its sum slot holds a marker with the index of the chunk where
// it ends.  Waves are independent: no block barrier after the mask load.

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// neighbour-sum slot of a row that crosses a chunk boundary: a quiet NaN with
// a tag no arithmetic produces over 44 payload bits that hold the row's last
// chunk and the number of chunks back to its first
constexpr long long kPiecedTag = 0x7FFDA00000000000LL;
constexpr long long kPiecedMask = (long long)0xFFFFF00000000000ULL;
static_assert(kPieceChunkBits + kPieceBackBits == 44, "piece marker payload");
constexpr int kXcds = 8;  // workgroups are dispatched round-robin over the XCDs
// row-end stores of the forward / reverse gathers: compacted per lane, and the
// two pieces of a chunk in one 16-byte store
constexpr bool kCompactFwd = false, kCompactBwd = true;
constexpr bool kPairFwd = false, kPairBwd = true;
// software pipeline of the persistent gather (kGatherAhead <= kStages - 2)
constexpr int kStages = 3;
constexpr int kGatherAhead = 1;
static_assert(kGatherAhead >= 1 && kGatherAhead <= kStages - 2, "pipeline depth");
// fourth word of a raw buffer descriptor on gfx9-family chips (gfx950)
constexpr int kBufferWord3 = 0x00020000;
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct WStage {
  u32x4 p;   // packed senders of this lane's 4 contacts
  f32x4 w;
  uint32_t hdr;  // rows starting before the chunk | next-chunk row start << 31
  uint32_t back; // chunks back to the start of the row continuing into the chunk
  f32x4 g;   // reverse: adjoints of the senders whose mask bit is set, else 0
};

__device__ __forceinline__ void wstage_load(const GatherArgs& a, WStage& s, int64_t k) {
  const int lane = threadIdx.x & 63;
  const int64_t base = k * kChunk + lane * 4;
  s.p = __builtin_nontemporal_load((const u32x4*)(a.colp + base));
  s.w = __builtin_nontemporal_load((const f32x4*)(a.wp + base));
  const unsigned long long h = a.chunk_hdr[k];
  s.hdr = (uint32_t)h;
  s.back = (uint32_t)(h >> 32);
  s.g = f32x4{0.f, 0.f, 0.f, 0.f};
}

// Reverse: g of the senders whose mask bit is set.  The load is a raw buffer
// load whose offset is moved past the end of the buffer for a clear bit; the
// hardware returns 0 for such a lane without a memory request, so there is no
// branch around the load (a branch would make the compiler wait for it at
// once).
template <bool BWD>
__device__ __forceinline__ void wstage_gather(const unsigned long long* mask, __amdgpu_buffer_rsrc_t gbuf,
                                              WStage& s) {
  if (!BWD) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t c = s.p[j] & 0xFFFFFFu;
    // one common out-of-range offset for clear bits: the address unit then
    // sees a single line for all of them
    const uint32_t off = lds_bit(mask, c) ? c * 4u : 0x80000000u;
    s.g[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(gbuf, off, 0, 0));
  }
}

// DPP move of a lane value with 0 for lanes without a source (or outside the
// row mask).  With every row enabled, bound_ctrl makes a lane without a
// source read 0, so the destination needs no zeroing first.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_or0(int v) {
  if (ROWS == 0xF) return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_or0(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// one step of the segmented scan: the lane's window (count c, open sum x)
// combined with the window before it
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_scan_step(int& c, double& x) {
  const int c2 = dpp_or0<CTRL, ROWS>(c);
  const double x2 = dpp_or0<CTRL, ROWS>(x);
  if (c == 0) x += x2;
  c += c2;
}

template <bool BWD>
__device__ __forceinline__ void wave_chunk(const GatherArgs& a, const unsigned long long* mask, double* out,
                                           const WStage& s, int64_t k) {
  const int lane = threadIdx.x & 63;
  uint32_t adv[4];
  double v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    adv[j] = s.p[j] >> 24;
    if (BWD) {
      v[j] = (double)s.w[j] * (double)s.g[j];
    } else {  // the weight where the sender's bit is set, else +0
      const uint32_t keep = 0u - lds_bit(mask, s.p[j] & 0xFFFFFFu);
      v[j] = (double)__uint_as_float(__float_as_uint(s.w[j]) & keep);
    }
  }
  // this lane's open segment and row-start count
  int cnt = 0;
  double x = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (adv[j]) x = 0.0;
    x += v[j];
    cnt += (int)adv[j];
  }
  // wave scans: inclusive prefix of the counts and segmented inclusive scan
  // of x; a window of lanes holds a row start exactly when its count is
  // non-zero, so the segment flag needs no scan of its own.  DPP moves
  // (row shifts within 16 lanes, then the broadcasts of lanes 15 and 31)
  // keep the scan off the LDS crossbar.
  int ci = cnt;
  double xi = x;
  seg_scan_step<0x111, 0xF>(ci, xi);  // row_shr:1
  seg_scan_step<0x112, 0xF>(ci, xi);  // row_shr:2
  seg_scan_step<0x114, 0xF>(ci, xi);  // row_shr:4
  seg_scan_step<0x118, 0xF>(ci, xi);  // row_shr:8
  seg_scan_step<0x142, 0xA>(ci, xi);  // row_bcast:15 into rows 1 and 3
  seg_scan_step<0x143, 0xC>(ci, xi);  // row_bcast:31 into rows 2 and 3
  int cex = ci - cnt;
  double sx = dpp_or0<0x138, 0xF>(xi);  // wave_shr:1, the previous lane's scan
  int sf = cex > 0;
  if (lane == 0) sx = 0.0;
  // does a row start at the contact after this lane's last one?
  const uint32_t a_next = (uint32_t)dpp_or0<0x130, 0xF>((int)adv[0]);  // wave_shl:1
  const uint32_t after = lane == kWave - 1 ? (s.hdr >> 31) : a_next;
  const int64_t rowbase = (int64_t)(s.hdr & 0x7FFFFFFFu);
  // Row ends.  A row that began in an earlier chunk gets the piece marker
  // and its sum goes to the chunk's first piece.
  constexpr bool COMPACT = BWD ? kCompactBwd : kCompactFwd;
  constexpr bool PAIR = BWD ? kPairBwd : kPairFwd;
  const double marker = __longlong_as_double(kPiecedTag | ((long long)s.back << kPieceChunkBits) | k);
  bool has_first = false;
  double first = 0.0;
  // COMPACT: the rows ending in this lane's contacts go to slots 0..3 first,
  // so the wave issues one store per slot some lane uses (usually one)
  double val[4];
  uint32_t rw[4];
  int n_end = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (adv[j]) {
      sx = 0.0;
      sf = 1;
    }
    sx += v[j];
    cex += (int)adv[j];
    const uint32_t anext = j < 3 ? adv[j + 1] : after;
    if (anext) {  // the row of contact j ends here
      if (!sf) {
        has_first = true;
        first = sx;
      }
      const double x = sf ? sx : marker;
      const uint32_t r = (uint32_t)(rowbase + cex - 1);
      if (COMPACT) {
#pragma unroll
        for (int q = 0; q <= j; ++q)
          if (n_end == q) {
            val[q] = x;
            rw[q] = r;
          }
        ++n_end;
      } else {
        if (!sf && !PAIR) a.piece[2 * k] = sx;
        out[r] = x;
      }
    }
  }
  if (COMPACT) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (n_end > q) out[rw[q]] = val[q];
    if (!PAIR && has_first) a.piece[2 * k] = first;
  }
  if (PAIR) {
    // one 16-byte store from the last lane: the first piece (the continuing
    // row's part, or the whole chunk when no row starts in it) and the last
    // piece (the part of the chunk's last row that continues)
    const unsigned long long fm = __ballot(has_first);  // at most one lane
    double fp_row = 0.0;
    if (fm) {  // wave-uniform
      const int src = __builtin_ctzll(fm);
      const long long b = __double_as_longlong(first);
      const int lo = __builtin_amdgcn_readlane((int)b, src), hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
      fp_row = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    if (lane == kWave - 1) {
      double fp = fp_row, lp = 0.0;
      if (after == 0) {  // the chunk's last row continues
        if (sf) lp = sx;
        else fp = sx;
      }
      typedef double f64x2 __attribute__((ext_vector_type(2)));
      *(f64x2*)(a.piece + 2 * k) = f64x2{fp, lp};
    }
  } else if (lane == kWave - 1 && after == 0) {  // the chunk's last row continues
    if (sf) a.piece[2 * k + 1] = sx;
    else a.piece[2 * k] = sx;
  }
}

// The chunks [start, end) of one slice with stride `stride` (one wave's
// share of a block's range): kStages register stages rotate by unrolling;
// chunk c is reduced in step c, its contacts were requested kStages - 1 steps
// earlier and (reverse) its adjoints kGatherAhead steps earlier.
template <bool BWD>
__device__ __forceinline__ void gather_range(const GatherArgs& a, const unsigned long long* mask,
                                             __amdgpu_buffer_rsrc_t gbuf, double* out, int64_t start, int64_t end,
                                             int stride) {
  if (start >= end) return;
  const int64_t mine = (end - 1 - start) / stride + 1;
  auto chunk = [&](int64_t q) { return start + (q < mine ? q : mine - 1) * stride; };
  WStage st[kStages];
#pragma unroll
  for (int j = 0; j < kStages - 1; ++j) wstage_load(a, st[j], chunk(j));
#pragma unroll
  for (int j = 0; j < kGatherAhead; ++j) wstage_gather<BWD>(mask, gbuf, st[j]);
  for (int64_t q = 0; q < mine; q += kStages) {
#pragma unroll
    for (int j = 0; j < kStages; ++j) {
      if (q + j >= mine) break;
      wstage_load(a, st[(j + kStages - 1) % kStages], chunk(q + j + kStages - 1));
      wstage_gather<BWD>(mask, gbuf, st[(j + kGatherAhead) % kStages]);
      wave_chunk<BWD>(a, mask, out, st[j], chunk(q + j));
    }
  }
}

// Persistent edge-parallel neighbour sum: out / first_piece / last_piece as
// described above; forward values are the weights of infectious senders,
// reverse values w * g for senders with a non-zero adjoint.
template <bool BWD>
__global__ void __launch_bounds__(kFastBlock) k_gather_fast(GatherArgs a) {
  __shared__ unsigned long long mask[kFastMaskWords];
  const int tid = threadIdx.x;
  const DGraph& G = a.G;
  const int nblk = gridDim.x, b = blockIdx.x;
  const int j = (nblk % kXcds == 0) ? (b % kXcds) * (nblk / kXcds) + b / kXcds : b;
  const int64_t C = a.slice_chunk[a.n_slices];
  int64_t c0 = C * j / nblk;
  const int64_t c1 = C * (j + 1) / nblk;
  // raw buffer over g (N floats): offsets at or past N * 4 read as 0
  const __amdgpu_buffer_rsrc_t gbuf =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.g, (short)0, BWD ? G.N * 4 : 0, kBufferWord3);
  int p = 0;
  while (p + 1 < a.n_slices && a.slice_chunk[p + 1] <= c0) ++p;
  bool first = true;
  while (c0 < c1) {  // block-uniform: every wave takes each barrier
    const int64_t e = min(c1, a.slice_chunk[p + 1]);
    const uint32_t sbase = (uint32_t)p << kSliceShift;
    const int words = (int)min((int64_t)kFastMaskWords, ((int64_t)G.N - sbase + 63) >> 6);
    if (!first) __syncthreads();  // every wave is done with the previous slice's mask
    lds_fill<kFastBlock, kFastMaskWords>(mask, a.mask + (sbase >> 6), words);
    __syncthreads();
    first = false;
    gather_range<BWD>(a, mask, gbuf, a.out + (int64_t)p * G.N, c0 + (tid >> 6), e, kFastBlock / kWave);
    c0 = e;
    ++p;
  }
}

// neighbour sum of receiver i in slice p from the gather outputs: the row's
// own slot, unless the gather marked the row as crossing chunks (then the
// pieces, in chunk order, from the chunk where the row starts to the chunk
// where it ends, both read from the marker).  Rows without contacts keep the
// zero written at run start.
__device__ __forceinline__ double gathered_slice(const SliceSums& ga, int p, int i) {
  const double v = ga.out[(int64_t)p * ga.N + i];
  const long long bits = __double_as_longlong(v);
  if ((bits & kPiecedMask) != kPiecedTag) return v;
  const int64_t kB = bits & ((1LL << kPieceChunkBits) - 1);
  const int64_t kA = kB - ((bits >> kPieceChunkBits) & ((1LL << kPieceBackBits) - 1));
  double s = ga.piece[2 * kA + 1];
  for (int64_t k = kA + 1; k <= kB; ++k) s += ga.piece[2 * k];
  return s;
}

// neighbour sum of receiver i: the slices' sums in slice order
__device__ __forceinline__ double gathered(const SliceSums& ga, int i) {
  double s = gathered_slice(ga, 0, i);
  for (int p = 1; p < ga.n_slices; ++p) s += gathered_slice(ga, p, i);
  return s;
}

// ------------------------------------------------------------------ agent passes

// Forward: A = neighbour sum (+ daily random layer), draw, progress, masks of
// day t+1, counts.  Packed populations: each agent uses its population's
// normaliser and parameter set and counts into its output; a block whose
// agents share one output reduces its counts first.
template <bool POPS, bool DWELL, bool LOC>
__global__ void __launch_bounds__(kBlock) k_agent_fwd(FwdArgs<float> a, SliceSums ga) {
  __shared__ unsigned scnt[kCnt];
  const int tid = threadIdx.x;
  if (tid < kCnt) scnt[tid] = 0u;
  const DGraph& G = a.G;
  const DParams& P = a.P;
  const int t = a.t;
  // clear the masks of day t+2 (read last on day t-1, written next on day t+1)
  for (int64_t x = blockIdx.x * (int64_t)kBlock + tid; x < a.mask_words; x += (int64_t)gridDim.x * kBlock)
    a.mI_clr[x] = 0ull;
  if (LOC)  // the location pressures of the next pass start at zero
    for (int64_t l = blockIdx.x * (int64_t)kBlock + tid; l < a.lf.n_loc; l += (int64_t)gridDim.x * kBlock)
      a.lf.P_next[l] = 0.0;
  __syncthreads();
  const int i = blockIdx.x * kBlock + tid;
  const bool on = i < G.N;
  const int o_blk = POPS ? range_output(G, P, blockIdx.x * kBlock, min(G.N, (blockIdx.x + 1) * kBlock) - 1) : 0;
  const int slot = blockIdx.x & (kSlots - 1);
  auto cnt_at = [&](int o) { return a.cnt + (((int64_t)o * P.K + t) * kSlots + slot) * kCnt; };
  uint32_t newst = 0u;
  bool removed = false;
  int o = 0;
  if (on) {
    const int p = POPS ? pop_of_agent(G, i) : 0, set = POPS ? set_of(P, p) : 0;
    const uint32_t loc = (uint32_t)(POPS ? i - G.pop_off[p] : i);
    o = POPS && P.per_pop ? p : 0;
    double A = gathered(ga, i) * P.TI;
    if (a.A_er) {
      A += a.A_er[i];
      a.A_er[i] = 0.0;
    }
    if (LOC) A += loc_agent_sum(a.lf, i, P.TI * (double)mask_bit(a.mI_cur, i));
    if (a.A_st) a.A_st[i] = (float)A;
    const HardDay hd = hard_agent_day<DWELL>(P, a.rng, a.stream, t, set, p, loc, G.age[i], A, a.rec_in[i], nullptr);
    if (a.fl_st) a.fl_st[i] = (uint8_t)((hd.was_s ? 1u : 0u) | (hd.h ? 2u : 0u));
    newst = hd.newst;
    removed = hd.removed;
    a.rec_out[i] = hd.rec;
  }
  const int lane = tid & 63;
  const unsigned long long bI = __ballot(on && newst == ST_I);
  if (lane == 0) or_ballot(a.mI_next, blockIdx.x * kBlock + (tid & ~63), bI);
  if (a.cnt) {
    if (o_blk >= 0) {
      const unsigned long long c0 = __ballot(on && newst == ST_S), c1 = __ballot(on && newst == ST_E),
                               c3 = __ballot(on && newst == ST_R), c4 = __ballot(on && newst == ST_M),
                               c5 = __ballot(on && removed);
      if (lane == 0) {
        atomicAdd(&scnt[ST_S], (unsigned)__popcll(c0));
        atomicAdd(&scnt[ST_E], (unsigned)__popcll(c1));
        atomicAdd(&scnt[ST_I], (unsigned)__popcll(bI));
        atomicAdd(&scnt[ST_R], (unsigned)__popcll(c3));
        atomicAdd(&scnt[ST_M], (unsigned)__popcll(c4));
        atomicAdd(&scnt[5], (unsigned)__popcll(c5));
      }
      __syncthreads();
      if (tid < 6 && scnt[tid]) atomicAdd(&cnt_at(o_blk)[tid], (double)scnt[tid]);
    } else if (on) {  // a block across a population boundary
      double* c = cnt_at(o);
      atomicAdd(&c[newst], 1.0);
      if (removed) atomicAdd(&c[5], 1.0);
    }
  }
}

// Reverse step t: record inf_bar^t (+ daily random layer) in the window ring,
// then the adjoint of day t-1 (t >= 1) or of the initial infections (t = 0);
// g^{t-1} and its non-zero mask for the next step's gather.  Parameter-gradient
// partials are reduced per block when its agents share one parameter set.
template <bool POPS, bool DWELL, bool LOC>
__global__ void __launch_bounds__(kBlock) k_agent_bwd(BwdArgs<float> a, FastMasks fm, SliceSums ga) {
  __shared__ double sg[2 + 16];
  __shared__ double sdw[DWELL ? 16 : 1];  // dwell log-weight gradients (E 0-7, I 8-15)
  const int tid = threadIdx.x;
  if (tid < 18) sg[tid] = 0.0;
  if (DWELL && tid < 16) sdw[tid] = 0.0;
  const DGraph& G = a.G;
  const DParams& P = a.P;
  const int t = a.t;
  const int W = P.tau_E + P.tau_I;
  for (int64_t x = blockIdx.x * (int64_t)kBlock + tid; x < fm.words; x += (int64_t)gridDim.x * kBlock)
    fm.clr[x] = 0ull;
  if (LOC)  // the location pressures of the next pass start at zero
    for (int64_t l = blockIdx.x * (int64_t)kBlock + tid; l < a.lf.n_loc; l += (int64_t)gridDim.x * kBlock)
      a.lf.P_next[l] = 0.0;
  __syncthreads();
  const int i = blockIdx.x * kBlock + tid;
  const bool on = i < G.N;
  // the set (= output) of the block when uniform, else -1
  const int s_blk = POPS ? range_output(G, P, blockIdx.x * kBlock, min(G.N, (blockIdx.x + 1) * kBlock) - 1) : 0;
  const int slot = blockIdx.x & (kSlots - 1);
  double g_new = 0.0;
  if (on) {
    const int p = POPS ? pop_of_agent(G, i) : 0, set = POPS ? set_of(P, p) : 0;
    const uint32_t loc = (uint32_t)(POPS ? i - G.pop_off[p] : i);
    const int o = POPS && P.per_pop ? p : 0;
    const double m = P.m[set];
    double infbar = 0.0;
    if (a.do_gather) {
      infbar = gathered(ga, i);
      if (a.infbar_er) {
        infbar += a.infbar_er[i];
        a.infbar_er[i] = 0.0;
      }
      if (LOC) infbar += loc_agent_sum(a.lf, i, (double)a.g_cur[i]);
      a.ring[(int64_t)(t % W) * G.N + i] = (float)infbar;
    }
    const int age = G.age[i];
    const double Sbar1 = (double)a.Sbar[i];
    if (t >= 1) {
      const int d = t - 1;
      // E for dE days after exposure on day d, then I until day d + dL
      int dE = P.tau_E, dL = W;
      if (DWELL && P.dwell_E) {
        dE = dwell_E(P, a.rng, loc, (uint32_t)d, (uint32_t)p, a.stream);
        dL = dE + dwell_I(P, a.rng, loc, (uint32_t)d, (uint32_t)p, a.stream);
      }
      double sE = 0.0, sI = 0.0;
      for (int k = 1; k <= dL; ++k) {
        const double v = (double)a.ring[(int64_t)((d + k) % W) * G.N + i];
        if (k <= dE) sE += v; else sI += v;
      }
      const double drm_bar = (d + dL < P.K) ? m * a.Dbar[(int64_t)o * P.K + d + dL] : 0.0;
      const uint32_t fl = a.fl_st[i];
      const double Aday = (double)a.A_st[i];
      const AdjOut ad = agent_adjoint<true>(P, a.rng, a.stream, d, set, p, loc, age, Aday, (double)(fl & 1u),
                                            (double)((fl >> 1) & 1u), false, sE, sI, Sbar1, drm_bar);
      if (DWELL && a.gdw && (fl & 3u) == 3u) {  // an exposure on day d: its drawn lengths' gradient
        double cE[8], cI[8], pre[17], gE[8], gI[8];
        const int aS = dwell_relaxed(P.dwell_E, P.tau_E, a.rng, loc, (uint32_t)d, TAG_DWELL_E, (uint32_t)p, a.stream,
                                     P.tau, cE);
        const int bS = dwell_relaxed(P.dwell_I, P.tau_I, a.rng, loc, (uint32_t)d, TAG_DWELL_I, (uint32_t)p, a.stream,
                                     P.tau, cI);
        pre[0] = 0.0;
        for (int k = 1; k <= W; ++k) pre[k] = pre[k - 1] + (double)a.ring[(int64_t)((d + k) % W) * G.N + i];
        auto DR = [&](int x) { return d + x < P.K ? m * a.Dbar[(int64_t)o * P.K + d + x] : 0.0; };
        dwell_sensitivities(P, pre, aS, bS, DR, gE, gI);
        st_categorical(cE, gE, P.tau_E, P.tau, sdw);
        st_categorical(cI, gI, P.tau_I, P.tau, sdw + 8);
      }
      a.Sbar[i] = (float)ad.Sbar;
      a.g_prev[i] = (float)ad.g;
      g_new = (double)(float)ad.g;
      if (ad.lam_bar != 0.0) {
        const double base = ad.lam_bar * Aday / (double)P.Z[p];
        const double vR = base * (double)P.S[set * P.n_age + age], vS = base * (double)P.R[set * P.K + d];
        if (s_blk >= 0) {
          atomicAdd(&sg[0], vR);
          atomicAdd(&sg[2 + age], vS);
        } else {
          atomicAdd(&a.gR[((int64_t)set * P.K + d) * kSlots + slot], vR);
          atomicAdd(&a.gS[((int64_t)set * P.n_age + age) * kSlots + slot], vS);
        }
      }
    } else {
      double sI = 0.0;
      const int dI0 = DWELL ? dwell_I(P, a.rng, loc, kDayInit, (uint32_t)p, a.stream) : P.tau_I;
      for (int k = 0; k < dI0; ++k) sI += (double)a.ring[(int64_t)(k % W) * G.N + i];
      const double x0_bar = P.TI * sI + ((dI0 - 1 < P.K) ? m * a.Dbar[(int64_t)o * P.K + dI0 - 1] : 0.0) - Sbar1;
      const double u = unit_u(rng_block(a.rng, loc, kDayInit, TAG_INIT, (uint32_t)p, a.stream).x);
      double y0, dy0;
      relaxed_init((double)P.i0[set], u, P.tau, y0, dy0);
      const double v = x0_bar * dy0;
      if (v != 0.0) {
        if (s_blk >= 0) atomicAdd(&sg[1], v);
        else atomicAdd(&a.gi0[(int64_t)set * kSlots + slot], v);
      }
      if (DWELL && a.gdw && u < (double)P.i0[set]) {  // a hard initial infection: its I length's gradient
        double cI[8], gI[8];
        dwell_relaxed(P.dwell_I, P.tau_I, a.rng, loc, kDayInit, TAG_DWELL_I, (uint32_t)p, a.stream, P.tau, cI);
        double run = 0.0;
        for (int b = 1; b <= P.tau_I; ++b) {
          run += (double)a.ring[(int64_t)((b - 1) % W) * G.N + i];
          gI[b - 1] = P.TI * run + (b - 1 < P.K ? m * a.Dbar[(int64_t)o * P.K + b - 1] : 0.0);
        }
        st_categorical(cI, gI, P.tau_I, P.tau, sdw + 8);
      }
    }
  }
  const unsigned long long bz = __ballot(on && g_new != 0.0);
  if ((tid & 63) == 0) or_ballot(fm.next, blockIdx.x * kBlock + (tid & ~63), bz);
  __syncthreads();
  if (s_blk >= 0) {
    if (t >= 1) {
      if (tid == 0 && sg[0] != 0.0) atomicAdd(&a.gR[((int64_t)s_blk * P.K + (t - 1)) * kSlots + slot], sg[0]);
      if (tid < P.n_age && sg[2 + tid] != 0.0)
        atomicAdd(&a.gS[((int64_t)s_blk * P.n_age + tid) * kSlots + slot], sg[2 + tid]);
    } else if (tid == 0 && sg[1] != 0.0) {
      atomicAdd(&a.gi0[(int64_t)s_blk * kSlots + slot], sg[1]);
    }
  }
  if (DWELL && a.gdw && tid < 16 && sdw[tid] != 0.0) atomicAdd(&a.gdw[tid * kSlots + slot], sdw[tid]);
}

template __global__ void k_agent_fwd<false, false, false>(FwdArgs<float>, SliceSums);
template __global__ void k_agent_fwd<false, false, true>(FwdArgs<float>, SliceSums);
template __global__ void k_agent_fwd<false, true, false>(FwdArgs<float>, SliceSums);
template __global__ void k_agent_fwd<false, true, true>(FwdArgs<float>, SliceSums);
template __global__ void k_agent_fwd<true, false, false>(FwdArgs<float>, SliceSums);
template __global__ void k_agent_fwd<true, false, true>(FwdArgs<float>, SliceSums);
template __global__ void k_agent_fwd<true, true, false>(FwdArgs<float>, SliceSums);
template __global__ void k_agent_fwd<true, true, true>(FwdArgs<float>, SliceSums);
template __global__ void k_agent_bwd<false, false, false>(BwdArgs<float>, FastMasks, SliceSums);
template __global__ void k_agent_bwd<false, false, true>(BwdArgs<float>, FastMasks, SliceSums);
template __global__ void k_agent_bwd<false, true, false>(BwdArgs<float>, FastMasks, SliceSums);
template __global__ void k_agent_bwd<false, true, true>(BwdArgs<float>, FastMasks, SliceSums);
template __global__ void k_agent_bwd<true, false, false>(BwdArgs<float>, FastMasks, SliceSums);
template __global__ void k_agent_bwd<true, false, true>(BwdArgs<float>, FastMasks, SliceSums);
template __global__ void k_agent_bwd<true, true, false>(BwdArgs<float>, FastMasks, SliceSums);
template __global__ void k_agent_bwd<true, true, true>(BwdArgs<float>, FastMasks, SliceSums);
template __global__ void k_gather_fast<false>(GatherArgs);
template __global__ void k_gather_fast<true>(GatherArgs);

}  // namespace gabm
