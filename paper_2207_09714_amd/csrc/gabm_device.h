// Device-side building blocks of the gabm library (gfx950, wave64).
//
// Counter-based generator, relaxed Bernoulli sample, packed agent records,
// the kernel-argument views of the graph and parameters, and wave/block
// reductions.  Everything here is for the GPU path only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gabm {

constexpr int kBlock = 256;      // threads per block of every tile kernel
constexpr int kWave = 64;
constexpr int kTileCap = 2048;   // contacts staged in LDS per tile
constexpr int kTileRows = 256;   // receivers per tile (one thread each in the epilogue)
constexpr int kSlots = 64;       // spread of global FP64 accumulators (contention)
constexpr int kCnt = 8;          // per-day aggregates: S,E,I,R,M snapshot counts, removals, spare x2
constexpr uint32_t kDayInit = 0xFFFFFFFFu;
// persistent kernels: one 1024-thread block per compute unit holding a
// one-bit-per-agent mask in LDS
constexpr int kFastBlock = 1024;
constexpr int kFastMaskWords = 16384;  // 64-bit words of LDS mask: 2^20 agents (one sender slice)
// The split B = 1 kernels read a sender-sliced copy of the contact list:
// slice p holds the contacts whose sender lies in [p * 2^20, (p + 1) * 2^20),
// so one slice's mask fits the LDS mask above.
constexpr int kSliceShift = 20;
constexpr int kMaxSlices = 16;         // senders below 2^24
// a row crossing chunks is marked with its end chunk (kPieceChunkBits bits)
// and the number of chunks back to its start (kPieceBackBits bits)
constexpr int kPieceChunkBits = 27;
constexpr int kPieceBackBits = 17;
// receiver tiles of the batched kernels (one lane group per tile)
constexpr int kBTileCap = 512;
constexpr int kBTileRows = 64;
// wave chunks of the edge-parallel neighbour sum: 64 lanes x 4 contacts
constexpr int kChunk = 256;
constexpr int kChunkShift = 8;

enum : uint32_t { ST_S = 0, ST_E = 1, ST_I = 2, ST_R = 3, ST_M = 4 };
enum : uint32_t { TAG_INIT = 0, TAG_INFECT = 1, TAG_MORT = 2, TAG_ER = 3 };
// dwell-time draws: uniform k of a draw is word k mod 4 of the block with tag
// (base + k / 4); E lengths use tags 4-5, I lengths 6-7
enum : uint32_t { TAG_DWELL_E = 4, TAG_DWELL_I = 6 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with a Weyl-sequence key schedule.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t a = c.x, b = c.z;
    const uint32_t hi0 = __umulhi(0xD2511F53u, a), lo0 = 0xD2511F53u * a;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, b), lo1 = 0xCD9E8D57u * b;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

struct Rng {
  uint32_t k0, k1;  // key = seed
};

__device__ __forceinline__ uint4 rng_block(Rng g, uint32_t idx, uint32_t day, uint32_t tag, uint32_t pop,
                                           uint32_t stream) {
  return philox10(make_uint4(idx, day, tag | (pop << 8), stream), g.k0, g.k1);
}

// uniform on (0,1) from the top 23 bits: (2k+1)/2^24, exact in float and double
__device__ __forceinline__ double unit_u(uint32_t x) { return (double)(2u * (x >> 9) + 1u) * 0x1p-24; }

// ---------------------------------------------------------------------------
// Relaxed Bernoulli (binary concrete): y = sigmoid((logit q + log((1-u)/u))/tau).
__device__ __forceinline__ double sigm(double z) {
  if (z >= 0.0) return 1.0 / (1.0 + exp(-z));
  const double e = exp(z);
  return e / (1.0 + e);
}
__device__ __forceinline__ double log_sigm(double z) { return z >= 0.0 ? -log1p(exp(-z)) : z - log1p(exp(z)); }

// y and dy/dlambda for q = 1 - exp(-lambda); both 0 at lambda = 0
__device__ __forceinline__ void relaxed_sample(double lam, double q, double u, double tau, double& y, double& dydl) {
  if (!(q > 0.0)) {
    y = 0.0;
    dydl = 0.0;
    return;
  }
  const double z = (log(q) + lam + (log1p(-u) - log(u))) / tau;  // log(1-q) = -lambda
  y = sigm(z);
  dydl = exp(log_sigm(z) - log(q)) * sigm(-z) / tau;
}

// The same in single precision, for runs that store float state: the
// derivative feeds only the reverse pass (gradients), never a hard decision.
// With l = log((1-u)/u) (1-u is exact for these u), z tau = log(q) + lambda + l
// = log(expm1(lambda)) + l, so log q = z tau - lambda - l needs no logarithm of
// its own, and sigma(z), sigma(-z), log sigma(z) share e = exp(-|z|).
__device__ __forceinline__ void relaxed_sample_f(float lam, float u, float tau, float& y, float& dydl) {
  if (!(lam > 0.f)) {
    y = 0.f;
    dydl = 0.f;
    return;
  }
  const float it = 1.f / tau;
  const float l = logf((1.f - u) / u);
  const float zt = (lam < 20.f ? logf(expm1f(lam)) : lam) + l;  // log(e^lambda - 1) = lambda to float precision above 20
  const float z = zt * it;
  const float e = expf(-fabsf(z));
  const float r = 1.f / (1.f + e);
  const bool pos = z >= 0.f;
  y = pos ? r : e * r;
  const float s_neg = pos ? e * r : r;                  // sigma(-z)
  const float log_s = (pos ? 0.f : z) - log1pf(e);       // log sigma(z)
  dydl = expf(log_s - (zt - lam - l)) * s_neg * it;     // sigma(z) sigma(-z) / (tau q)
}

// y0 and dy0/di0 of the relaxed initial infection
__device__ __forceinline__ void relaxed_init(double i0, double u, double tau, double& y0, double& dy0) {
  const double z = (log(i0) - log1p(-i0) + (log1p(-u) - log(u))) / tau;
  y0 = sigm(z);
  dy0 = y0 * sigm(-z) / (tau * i0 * (1.0 - i0));
}

// ---------------------------------------------------------------------------
// Packed hard record: stage | timer << 8 | (int16) exposure day << 16.
__device__ __forceinline__ uint32_t rec_stage(uint32_t r) { return r & 0xFFu; }
__device__ __forceinline__ uint32_t rec_timer(uint32_t r) { return (r >> 8) & 0xFFu; }
__device__ __forceinline__ uint32_t make_rec(uint32_t st, uint32_t tm, int eday) {
  return st | (tm << 8) | ((uint32_t)(uint16_t)(int16_t)eday << 16);
}

// ---------------------------------------------------------------------------
// Kernel-argument views.

// One receiver tile: rows [r0, r1), contacts [e0, e1); 32 bytes, read with
// two independent 16-byte loads.  In the batched tile table, pad0 counts the
// (empty) rows of earlier tiles that also start at contact e0.
struct alignas(16) TileInfo {
  int64_t e0, e1;
  int32_t r0, r1, pad0, pad1;
};

struct DGraph {
  const int64_t* row_ptr;  // [N+1]
  const int32_t* col;      // [E] sender of each contact, rows = receivers
  const float* w;          // [E]
  const int32_t* tile_row; // [n_tiles+1]
  const TileInfo* tiles;   // [n_tiles]
  const TileInfo* btiles;  // [n_btiles] tiles of the batched kernels
  int32_t n_btiles;
  // edge-parallel form: sender | (rows starting at this contact) << 24, padded
  // with zero contacts to a multiple of kChunk; first row of each chunk
  const uint32_t* colp;    // [n_chunks * kChunk]
  const float* wp;         // [n_chunks * kChunk]
  // per chunk: rows that start before it | (a row starts right after it) << 31
  const uint32_t* chunk_row;  // [n_chunks]
  int64_t n_chunks;
  const uint8_t* age;      // [N]
  const uint16_t* pop_of;  // [N]
  const int32_t* pop_off;  // [n_pops+1]
  const int64_t* er_off;   // [n_pops+1] prefix of daily random pairs per population
  int32_t N, n_pops, n_tiles;
  int64_t er_total;        // pairs per day, all populations
  double er_mean;
  float er_w;
};

struct DParams {
  const float* R;   // [n_sets*K]
  const float* S;   // [n_sets*n_age]
  const float* m;   // [n_sets]
  const float* i0;  // [n_sets]
  const float* Z;   // [n_pops]
  double TE, TI, tau;
  int32_t K, tau_E, tau_I, n_age, mode, per_pop, n_sets;
  const float* iota;  // [tau_E + tau_I] infectiousness over days since exposure, or null (flat)
  // stochastic dwell times: log weights of the lengths 1..tau_E (E) and
  // 1..tau_I (I), or null for the fixed tau_E / tau_I
  const float* dwell_E;
  const float* dwell_I;
};

// Weight of the k-th day after exposure (k = 1 .. tau_E + tau_I): the
// profile value, 1 when flat.
__device__ __forceinline__ double iota_at(const DParams& P, int k) {
  if (!P.iota) return 1.0;
  const int W = P.tau_E + P.tau_I;
  return (double)P.iota[(k < 1 ? 1 : (k > W ? W : k)) - 1];
}
// Days since exposure on day t of an agent with packed record r (exposure day
// in the high half); an initial infection (exposure day -1 in the record)
// counts as exposed on day -tau_E - 1.
__device__ __forceinline__ int days_since_exposure(uint32_t r, int t, int tau_E) {
  const int e = (int)(int16_t)(r >> 16);
  return e < 0 ? t + tau_E + 1 : t - e;
}

// lambda = R * S[a] * A / Z evaluated left to right in double precision
__device__ __forceinline__ double rate(double R, double S, double A, double Z) { return R * S * A / Z; }

// ---------------------------------------------------------------------------
// Reductions.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// sum over a block of NT threads; every thread receives the result.
// `scratch` holds at least NT/kWave values.
template <int NT, typename T>
__device__ __forceinline__ T block_sum_n(T v, T* scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wv] = v;
  __syncthreads();
  T s = scratch[0];
#pragma unroll
  for (int k = 1; k < NT / kWave; ++k) s += scratch[k];
  return s;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
  return block_sum_n<kBlock>(v, scratch);
}

__device__ __forceinline__ int pop_of_agent(const DGraph& G, int i) { return G.n_pops == 1 ? 0 : (int)G.pop_of[i]; }
// parameter set of population p: its own with per-population parameters, else set 0
__device__ __forceinline__ int set_of(const DParams& P, int pop) { return P.per_pop ? pop : 0; }
// output (aggregate) index shared by agents [i0, i1], or -1 when they belong to
// populations with different outputs
__device__ __forceinline__ int range_output(const DGraph& G, const DParams& P, int i0, int i1) {
  if (!P.per_pop) return 0;
  const int p0 = pop_of_agent(G, i0);
  return p0 == pop_of_agent(G, i1) ? p0 : -1;
}

// one bit per agent, 64-bit words; OR the ballot of 64 consecutive agents
// starting at `base` into the mask
__device__ __forceinline__ void or_ballot(unsigned long long* mask, int base, unsigned long long bits) {
  if (bits == 0ull) return;
  const int wd = base >> 6, sh = base & 63;
  atomicOr(&mask[wd], bits << sh);
  if (sh) {
    const unsigned long long hi = bits >> (64 - sh);
    if (hi) atomicOr(&mask[wd + 1], hi);
  }
}

__device__ __forceinline__ uint32_t mask_bit(const uint32_t* mask32, int c) { return (mask32[c >> 5] >> (c & 31)) & 1u; }

// Copies n <= MAXW 64-bit words from global memory (16-byte aligned) into
// LDS with a block of NT threads.  Each thread issues all its loads (16 bytes
// each) before its first LDS write, so the copy costs about one memory round
// trip rather than one per word a thread moves.
template <int NT, int MAXW>
__device__ __forceinline__ void lds_fill(unsigned long long* lds, const unsigned long long* src, int n) {
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  constexpr int R = (MAXW / 2 + NT - 1) / NT;
  const int np = n >> 1;  // whole 16-byte pairs
  const int tid = threadIdx.x;
  u64x2 v[R];
  if (np > 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = *(const u64x2*)(src + 2 * min(tid + r * NT, np - 1));
  }
  const bool tail = (n & 1) && tid == 0;
  const unsigned long long last = tail ? src[n - 1] : 0ull;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int x = tid + r * NT;
    if (x < np) {
      lds[2 * x] = v[r].x;
      lds[2 * x + 1] = v[r].y;
    }
  }
  if (tail) lds[n - 1] = last;
}

}  // namespace gabm
