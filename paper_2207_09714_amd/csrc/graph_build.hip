// Contact-graph build: directed COO -> CSR with rows = receivers, each row
// sorted by (sender, weight); tile schedule for the transmission kernels;
// per-agent population table; symmetry check.
//
// The model treats interaction networks as (sparse) adjacency matrices and
// aggregates contacts with a permutation-invariant sum (Section 3.1 and
// Appendix A); the adjoint of that sum is a gather over the transpose, which
// for a symmetric contact graph is the same CSR.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "gabm_internal.h"

namespace gabm {

enum : uint32_t { BAD_ID = 1, BAD_SELF = 2, BAD_POP = 4, BAD_W = 8, BAD_AGE = 16, BAD_SYM = 32 };

__device__ __forceinline__ int pop_search(const int32_t* off, int n_pops, int i) {
  int lo = 0, hi = n_pops;  // off[lo] <= i < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void k_validate(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                           const float* __restrict__ w, int64_t E, int32_t N, const int32_t* pop_off, int n_pops,
                           uint32_t* flag) {
  uint32_t bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = src[e], d = dst[e];
    if (s < 0 || s >= N || d < 0 || d >= N) { bad |= BAD_ID; continue; }
    if (s == d) bad |= BAD_SELF;
    if (n_pops > 1 && pop_search(pop_off, n_pops, s) != pop_search(pop_off, n_pops, d)) bad |= BAD_POP;
    if (w) {
      const float x = w[e];
      if (!(x >= 0.f) || !isfinite(x)) bad |= BAD_W;
    }
  }
  if (bad) atomicOr(flag, bad);
}

__global__ void k_validate_age(const uint8_t* age, int32_t N, int n_age, uint32_t* flag) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
    if (age[i] >= n_age) atomicOr(flag, (uint32_t)BAD_AGE);
}

// histogram of receivers (both directions when symmetrising)
__global__ void k_degree(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, int64_t E, int sym,
                         unsigned long long* deg) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    atomicAdd(&deg[dst[e]], 1ull);
    if (sym) atomicAdd(&deg[src[e]], 1ull);
  }
}

// ---- exclusive scan of N+1 counts (three passes; block = 256 x 8 items)
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long v, unsigned long long* sh,
                                                              unsigned long long* total) {
  // inclusive wave scan
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  unsigned long long x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    unsigned long long y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  unsigned long long pre = 0, tot = 0;
  for (int k = 0; k < kBlock / kWave; ++k) {
    if (k < wv) pre += sh[k];
    tot += sh[k];
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

__global__ void k_scan_tiles(const unsigned long long* in, int64_t n, unsigned long long* out,
                             unsigned long long* tile_sums) {
  __shared__ unsigned long long sh[kBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  unsigned long long v[kScanItems], s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0ull;
    s += v[k];
  }
  unsigned long long tot;
  unsigned long long pre = block_excl_scan(s, sh, &tot);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = pre;
    pre += v[k];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ void k_scan_sums(unsigned long long* sums, int64_t n) {
  __shared__ unsigned long long sh[kBlock / kWave];
  unsigned long long carry = 0;
  for (int64_t b = 0; b < n; b += kBlock) {
    const int64_t i = b + threadIdx.x;
    const unsigned long long v = i < n ? sums[i] : 0ull;
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan(v, sh, &tot);
    if (i < n) sums[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
}

__global__ void k_scan_add(unsigned long long* out, int64_t n, const unsigned long long* sums, int64_t* row_ptr,
                           unsigned long long* cursor) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  const unsigned long long add = sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) {
      const unsigned long long v = out[base + k] + add;
      row_ptr[base + k] = (int64_t)v;
      cursor[base + k] = v;
    }
}

// scatter contacts into their receiver rows (order inside a row is fixed by
// the sort that follows)
__global__ void k_scatter(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                          const float* __restrict__ w, int64_t E, int sym, unsigned long long* cursor,
                          int32_t* col, float* wout) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = src[e], d = dst[e];
    const float x = w ? w[e] : 1.0f;
    unsigned long long p = atomicAdd(&cursor[d], 1ull);
    col[p] = s;
    wout[p] = x;
    if (sym) {
      p = atomicAdd(&cursor[s], 1ull);
      col[p] = d;
      wout[p] = x;
    }
  }
}

__device__ __forceinline__ unsigned long long edge_key(int32_t c, float w) {
  return ((unsigned long long)(uint32_t)c << 32) | (unsigned long long)__float_as_uint(w);
}

// rows of up to 32 contacts: one thread, insertion sort in place
__global__ void k_sort_short(const int64_t* row_ptr, int32_t N, int32_t* col, float* w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t a = row_ptr[i], b = row_ptr[i + 1];
  if (b - a < 2 || b - a > 32) return;
  for (int64_t x = a + 1; x < b; ++x) {
    const int32_t c = col[x];
    const float f = w[x];
    const unsigned long long k = edge_key(c, f);
    int64_t y = x - 1;
    while (y >= a && edge_key(col[y], w[y]) > k) {
      col[y + 1] = col[y];
      w[y + 1] = w[y];
      --y;
    }
    col[y + 1] = c;
    w[y + 1] = f;
  }
}

constexpr int kSortLds = 8192;

// rows longer than 32: one block per row, bitonic sort of the packed keys in
// LDS (rows up to kSortLds) or in a global scratch area (longer rows)
__global__ void __launch_bounds__(kBlock) k_sort_long(const int64_t* row_ptr, const int32_t* rows, int n_rows,
                                                      int32_t* col, float* w, unsigned long long* gscratch,
                                                      int64_t gscratch_len) {
  __shared__ unsigned long long sk[kSortLds];
  const int i = rows[blockIdx.x];
  const int64_t a = row_ptr[i], b = row_ptr[i + 1];
  const int64_t n = b - a;
  int64_t P = 1;
  while (P < n) P <<= 1;
  unsigned long long* keys = (P <= kSortLds) ? sk : gscratch;
  if (P > kSortLds && P > gscratch_len) return;  // host guarantees capacity
  for (int64_t x = threadIdx.x; x < P; x += kBlock) keys[x] = x < n ? edge_key(col[a + x], w[a + x]) : ~0ull;
  __syncthreads();
  for (int64_t k = 2; k <= P; k <<= 1) {
    for (int64_t j = k >> 1; j > 0; j >>= 1) {
      for (int64_t x = threadIdx.x; x < P; x += kBlock) {
        const int64_t y = x ^ j;
        if (y > x) {
          const unsigned long long kx = keys[x], ky = keys[y];
          const bool up = (x & k) == 0;
          if ((kx > ky) == up) {
            keys[x] = ky;
            keys[y] = kx;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int64_t x = threadIdx.x; x < n; x += kBlock) {
    const unsigned long long kk = keys[x];
    col[a + x] = (int32_t)(kk >> 32);
    w[a + x] = __uint_as_float((uint32_t)kk);
  }
}

__device__ __forceinline__ int64_t lower_key(const int32_t* col, const float* w, int64_t a, int64_t b,
                                             unsigned long long k) {
  while (a < b) {
    const int64_t mid = (a + b) >> 1;
    if (edge_key(col[mid], w[mid]) < k) a = mid + 1; else b = mid;
  }
  return a;
}

// symmetric iff for every stored (i <- j, w) the multiplicity of (j, w) in
// row i equals the multiplicity of (i, w) in row j
__global__ void k_check_sym(const int64_t* row_ptr, const int32_t* col, const float* w, int32_t N, uint32_t* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t a = row_ptr[i], b = row_ptr[i + 1];
  int64_t x = a;
  while (x < b) {
    const int32_t j = col[x];
    const float f = w[x];
    int64_t y = x + 1;
    while (y < b && col[y] == j && w[y] == f) ++y;
    const int64_t mult = y - x;
    const int64_t ja = row_ptr[j], jb = row_ptr[j + 1];
    const unsigned long long k = edge_key(i, f);
    const int64_t lo = lower_key(col, w, ja, jb, k);
    const int64_t hi = lower_key(col, w, ja, jb, k + 1);
    if (hi - lo != mult) {
      atomicOr(flag, (uint32_t)BAD_SYM);
      return;
    }
    x = y;
  }
}

// rows starting at each contact position (empty rows included; rows starting
// at the end of the contact list are not counted)
__global__ void k_row_starts(const int64_t* row_ptr, int32_t N, int64_t E, unsigned int* adv) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = row_ptr[r];
    if (p < E) atomicAdd(&adv[p], 1u);
  }
}

// packed sender | min(row starts, 255) << 24, zero padding up to n_pad; flag
// when a count does not fit in 8 bits
__global__ void k_pack_cols(const int32_t* col, const float* w, const unsigned int* adv, int64_t E, int64_t n_pad,
                            uint32_t* colp, float* wp, uint32_t* flag) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_pad; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < E) {
      const unsigned int a = adv[e];
      if (a > 255u) atomicOr(flag, 1u);
      colp[e] = (uint32_t)col[e] | (min(a, 255u) << 24);
      wp[e] = w[e];
    } else {
      colp[e] = 0u;
      wp[e] = 0.f;
    }
  }
}

// ---- sender-sliced stream of the split B = 1 kernels
//
// Slice p of receiver row r is the part of the row (sorted by sender) whose
// senders lie in [p << kSliceShift, (p + 1) << kSliceShift).  A row that is
// empty in a slice is still counted by the row-start byte of the slice's next
// contact; to keep that count below 256, an empty row whose index is a
// multiple of 128 gets one zero-weight contact (sender = the slice's first
// agent), which adds an exact 0 to its sum.

__device__ __forceinline__ int64_t lower_col(const int32_t* col, int64_t a, int64_t b, int32_t c) {
  while (a < b) {
    const int64_t mid = (a + b) >> 1;
    if (col[mid] < c) a = mid + 1; else b = mid;
  }
  return a;
}

constexpr int kSlicePadEvery = 128;

// contacts of row r in slice p, [P][N+1] with a zero at index N of each slice
__global__ void k_slice_count(const int64_t* row_ptr, const int32_t* col, int32_t N, int P, unsigned long long* cnt) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r <= N; r += (int64_t)gridDim.x * blockDim.x) {
    if (r == N) {
      for (int p = 0; p < P; ++p) cnt[(int64_t)p * (N + 1) + N] = 0ull;
      continue;
    }
    const int64_t e1 = row_ptr[r + 1];
    int64_t lo = row_ptr[r];
    for (int p = 0; p < P; ++p) {
      const int64_t hi = p == P - 1 ? e1 : lower_col(col, lo, e1, (p + 1) << kSliceShift);
      unsigned long long c = (unsigned long long)(hi - lo);
      if (c == 0 && (r % kSlicePadEvery) == 0) c = 1;
      cnt[(int64_t)p * (N + 1) + r] = c;
      lo = hi;
    }
  }
}

// copy each row's slices into the streams; count row starts per position.
// spos: exclusive scan of the counts over [P][N+1] (slice p's own offsets are
// spos[p][r] - spos[p][0]); cb: first chunk of each slice
__global__ void k_slice_fill(const int64_t* row_ptr, const int32_t* col, const float* w, int32_t N, int P,
                             const int64_t* spos, const int64_t* cb, uint32_t* fcolp, float* fwp, unsigned int* adv) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e1 = row_ptr[r + 1];
    int64_t lo = row_ptr[r];
    for (int p = 0; p < P; ++p) {
      const int64_t hi = p == P - 1 ? e1 : lower_col(col, lo, e1, (p + 1) << kSliceShift);
      const int64_t* sp = spos + (int64_t)p * (N + 1);
      const int64_t pos = sp[r] - sp[0], Ep = sp[N] - sp[0];
      const int64_t dst = cb[p] * kChunk + pos;
      if (hi > lo) {
        for (int64_t e = lo; e < hi; ++e) {
          fcolp[dst + (e - lo)] = (uint32_t)col[e];
          fwp[dst + (e - lo)] = w[e];
        }
      } else if ((r % kSlicePadEvery) == 0) {
        fcolp[dst] = (uint32_t)p << kSliceShift;
        fwp[dst] = 0.f;
      }
      if (pos < Ep) atomicAdd(&adv[dst], 1u);
      lo = hi;
    }
  }
}

// row-start byte of every position; zero-weight padding after each slice's
// contacts up to its chunk boundary; flag if a count does not fit in 8 bits
__global__ void k_slice_pack(const int64_t* spos, const int64_t* cb, int32_t N, int P, int64_t n_pad,
                             const unsigned int* adv, uint32_t* fcolp, float* fwp, uint32_t* flag) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_pad; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e >> kChunkShift;
    int p = 0;
    while (p + 1 < P && cb[p + 1] <= k) ++p;
    const int64_t* sp = spos + (int64_t)p * (N + 1);
    const int64_t local = e - cb[p] * kChunk, Ep = sp[N] - sp[0];
    if (local < Ep) {
      const unsigned int a = adv[e];
      if (a > 255u) atomicOr(flag, 1u);
      fcolp[e] |= min(a, 255u) << 24;
    } else {
      fcolp[e] = (uint32_t)p << kSliceShift;
      fwp[e] = 0.f;
    }
  }
}

// chunk header: rows of its slice that start before it | (a row starts at
// the contact after it) << 31 (always set for a slice's last chunk), and in
// the high word how many chunks back the row continuing into it started
__global__ void k_slice_chunk_row(const int64_t* spos, const int64_t* cb, int32_t N, int P, int64_t n_ch,
                                  unsigned long long* hdr) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_ch; k += (int64_t)gridDim.x * blockDim.x) {
    int p = 0;
    while (p + 1 < P && cb[p + 1] <= k) ++p;
    const int64_t* sp = spos + (int64_t)p * (N + 1);
    const int64_t kl = k - cb[p], nk = cb[p + 1] - cb[p];
    // rows r in [0, N] whose start (sp[r] - sp[0]) lies before position x of the slice
    auto before = [&](int64_t x) {
      int64_t a = 0, b = (int64_t)N + 1;
      while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (sp[mid] - sp[0] < x) a = mid + 1; else b = mid;
      }
      return a;
    };
    const int64_t rows = before(kl * kChunk);
    bool starts = true;
    if (kl + 1 < nk) {
      const int64_t rn = before((kl + 1) * kChunk);
      starts = rn < N && sp[rn] - sp[0] == (kl + 1) * kChunk;
    }
    // the last row starting before the chunk continues into it unless a row
    // starts at the chunk's first contact
    int64_t back = 0;
    if (rows > 0) {
      const int64_t x = sp[rows - 1] - sp[0];
      if (rows > N || sp[rows] - sp[0] != kl * kChunk) back = kl - (x >> kChunkShift);
    }
    hdr[k] = ((unsigned long long)back << 32) | (uint32_t)rows | (starts ? 0x80000000u : 0u);
  }
}

__global__ void k_pop_of(const int32_t* pop_off, int n_pops, int32_t N, uint16_t* pop_of) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
    pop_of[i] = (uint16_t)pop_search(pop_off, n_pops, i);
}

__global__ void k_weight_sum(const float* w, int64_t E, double* out) {
  __shared__ double sh[kBlock / kWave];
  double s = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x)
    s += (double)w[e];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) atomicAdd(out, s);
}

void Graph::release() {
  hipFree(row_ptr); hipFree(col); hipFree(w); hipFree(tile_row); hipFree(tiles); hipFree(btiles); hipFree(colp); hipFree(wp); hipFree(chunk_row); hipFree(age); hipFree(pop_of); hipFree(pop_off);
  hipFree(er_off);
  row_ptr = nullptr; col = nullptr; w = nullptr; tile_row = nullptr; tiles = nullptr; btiles = nullptr; colp = nullptr; wp = nullptr; chunk_row = nullptr;
  n_chunks = 0;
  hipFree(fcolp); hipFree(fwp); hipFree(fchunk_hdr);
  fcolp = nullptr; fwp = nullptr; fchunk_hdr = nullptr;
  n_slices = 0;
  slice_chunk.clear();
  age = nullptr; pop_of = nullptr;
  pop_off = nullptr; er_off = nullptr;
  hipFree(lv_agent); hipFree(lv_loc); hipFree(lv_w); hipFree(av_ptr); hipFree(av_loc); hipFree(av_w);
  hipFree(loc_scratch);
  loc_scratch = nullptr;
  lv_agent = nullptr; lv_loc = nullptr; lv_w = nullptr; av_ptr = nullptr; av_loc = nullptr; av_w = nullptr;
  n_loc = 0; n_visits = 0;
}

static int grid_for(int64_t n, int per = kBlock) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

// Greedy tiles of consecutive receivers: at most `rows` rows and `cap`
// staged contacts; a row longer than `cap` forms a tile alone.
static void make_tiles(const std::vector<int64_t>& rp, std::vector<int32_t>& tiles, int32_t& n_long, int32_t& maxdeg,
                       int64_t cap = kTileCap, int32_t rows = kTileRows) {
  const int32_t N = (int32_t)rp.size() - 1;
  tiles.clear();
  tiles.push_back(0);
  n_long = 0;
  maxdeg = 0;
  int32_t r = 0;
  while (r < N) {
    const int64_t d = rp[r + 1] - rp[r];
    maxdeg = std::max<int32_t>(maxdeg, (int32_t)d);
    if (d > cap) {
      ++n_long;
      ++r;
      tiles.push_back(r);
      continue;
    }
    int32_t r1 = r + 1;
    while (r1 < N && r1 - r < rows && rp[r1 + 1] - rp[r] <= cap) {
      maxdeg = std::max<int32_t>(maxdeg, (int32_t)(rp[r1 + 1] - rp[r1]));
      ++r1;
    }
    r = r1;
    tiles.push_back(r);
  }
}

// Sender-sliced stream of the split B = 1 kernels (from the sorted CSR).
static gabm_status build_sliced_stream(Graph& G, hipStream_t st) {
  const int32_t N = G.N;
  const int P = (int)(((int64_t)N + (1 << kSliceShift) - 1) >> kSliceShift);
  const int64_t n1 = (int64_t)P * (N + 1);
  const int64_t n_tiles = (n1 + kScanTile - 1) / kScanTile;
  unsigned long long *cnt = nullptr, *scan = nullptr, *sums = nullptr;
  int64_t *spos = nullptr, *cb = nullptr;
  unsigned int* adv = nullptr;
  uint32_t* flag = nullptr;
  auto cleanup = [&]() {
    hipFree(cnt); hipFree(scan); hipFree(sums); hipFree(spos); hipFree(cb); hipFree(adv); hipFree(flag);
  };
  auto fail = [&](hipError_t e, const char* what) {
    cleanup();
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return GABM_EHIP;
  };
  hipError_t e;
  if ((e = dalloc(&cnt, n1)) != hipSuccess || (e = dalloc(&scan, n1)) != hipSuccess ||
      (e = dalloc(&sums, n_tiles)) != hipSuccess || (e = dalloc(&spos, n1)) != hipSuccess ||
      (e = dalloc(&cb, P + 1)) != hipSuccess || (e = dalloc(&flag, 1)) != hipSuccess)
    return fail(e, "sliced stream: allocation");
  hipLaunchKernelGGL(k_slice_count, dim3(grid_for((int64_t)N + 1)), dim3(kBlock), 0, st, G.row_ptr, G.col, N, P, cnt);
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)n_tiles), dim3(kBlock), 0, st, cnt, n1, scan, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, st, sums, n_tiles);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)n_tiles), dim3(kBlock), 0, st, scan, n1, sums, spos, cnt);
  std::vector<int64_t> s0(P), sN(P);
  for (int p = 0; p < P; ++p) {
    const int64_t* sp = spos + (int64_t)p * (N + 1);
    if ((e = hipMemcpyAsync(&s0[p], sp, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(&sN[p], sp + N, 8, hipMemcpyDeviceToHost, st)) != hipSuccess)
      return fail(e, "sliced stream: totals");
  }
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail(e, "sliced stream: counts");
  std::vector<int64_t> chunk0(P + 1, 0);
  for (int p = 0; p < P; ++p) chunk0[p + 1] = chunk0[p] + (sN[p] - s0[p] + kChunk - 1) / kChunk;
  const int64_t nch = chunk0[P], npad = nch * kChunk;
  if (nch >= (int64_t(1) << kPieceChunkBits)) {  // chunk index does not fit the piece marker
    cleanup();
    return GABM_OK;
  }
  if ((e = dalloc(&adv, npad)) != hipSuccess || (e = dalloc(&G.fcolp, npad)) != hipSuccess ||
      (e = dalloc(&G.fwp, npad)) != hipSuccess || (e = dalloc(&G.fchunk_hdr, nch)) != hipSuccess)
    return fail(e, "sliced stream: allocation");
  if ((e = hipMemsetAsync(adv, 0, sizeof(unsigned int) * npad, st)) != hipSuccess ||
      (e = hipMemsetAsync(flag, 0, sizeof(uint32_t), st)) != hipSuccess ||
      (e = hipMemcpyAsync(cb, chunk0.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice, st)) != hipSuccess)
    return fail(e, "sliced stream: set-up");
  hipLaunchKernelGGL(k_slice_fill, dim3(grid_for(N)), dim3(kBlock), 0, st, G.row_ptr, G.col, G.w, N, P, spos, cb,
                     G.fcolp, G.fwp, adv);
  hipLaunchKernelGGL(k_slice_pack, dim3(grid_for(npad)), dim3(kBlock), 0, st, spos, cb, N, P, npad, adv, G.fcolp,
                     G.fwp, flag);
  hipLaunchKernelGGL(k_slice_chunk_row, dim3(grid_for(nch)), dim3(kBlock), 0, st, spos, cb, N, P, nch, G.fchunk_hdr);
  uint32_t of = 0;
  if ((e = hipMemcpyAsync(&of, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess || (e = hipGetLastError()) != hipSuccess)
    return fail(e, "sliced stream: build");
  cleanup();
  if (of) {  // cannot happen with the padding rule; keep the tile kernels only
    hipFree(G.fcolp);
    hipFree(G.fwp);
    hipFree(G.fchunk_hdr);
    G.fcolp = nullptr;
    G.fwp = nullptr;
    G.fchunk_hdr = nullptr;
    return GABM_OK;
  }
  G.n_slices = P;
  G.slice_chunk = chunk0;
  return GABM_OK;
}

// Agent-location layer: validates the visits on the host and stores them
// twice, grouped by location (the pressure pass reads runs of one location)
// and by agent (the per-agent pass).  Both groupings are counting sorts,
// stable in input order.
static gabm_status build_locations(const gabm_graph_desc* d, hipStream_t st, Graph& G) {
  const int64_t V = d->n_visits;
  const int32_t L = d->n_locations, N = d->n_agents;
  if (V == 0) return GABM_OK;
  std::vector<int32_t> va(V), vl(V);
  std::vector<float> vw(V);
  GABM_HIP(hipMemcpyAsync(va.data(), d->visit_agent, sizeof(int32_t) * V, hipMemcpyDeviceToHost, st));
  GABM_HIP(hipMemcpyAsync(vl.data(), d->visit_loc, sizeof(int32_t) * V, hipMemcpyDeviceToHost, st));
  GABM_HIP(hipMemcpyAsync(vw.data(), d->visit_w, sizeof(float) * V, hipMemcpyDeviceToHost, st));
  GABM_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> lpop(L, -1);
  std::vector<int64_t> lcnt(L + 1, 0), acnt((size_t)N + 1, 0);
  for (int64_t v = 0; v < V; ++v) {
    const int32_t a = va[v], l = vl[v];
    GABM_CHECK(a >= 0 && a < N, GABM_ERANGE, "visit with agent id outside [0, n_agents)");
    GABM_CHECK(l >= 0 && l < L, GABM_ERANGE, "visit with location id outside [0, n_locations)");
    GABM_CHECK(std::isfinite(vw[v]) && vw[v] >= 0.f, GABM_EINVAL, "visit weight negative or not finite");
    const int32_t p = (int32_t)(std::upper_bound(G.pop_off_h.begin(), G.pop_off_h.end(), a) - G.pop_off_h.begin()) - 1;
    GABM_CHECK(lpop[l] < 0 || lpop[l] == p, GABM_ERANGE, "location visited from different populations");
    lpop[l] = p;
    ++lcnt[l + 1];
    ++acnt[(size_t)a + 1];
  }
  for (int32_t l = 0; l < L; ++l) lcnt[l + 1] += lcnt[l];
  for (int32_t i = 0; i < N; ++i) acnt[(size_t)i + 1] += acnt[i];
  std::vector<int32_t> lv_a(V), lv_l(V), av_l(V);
  std::vector<float> lv_wh(V), av_wh(V);
  {
    std::vector<int64_t> cur(lcnt.begin(), lcnt.end() - 1);
    for (int64_t v = 0; v < V; ++v) {
      const int64_t k = cur[vl[v]]++;
      lv_a[k] = va[v];
      lv_l[k] = vl[v];
      lv_wh[k] = vw[v];
    }
  }
  {
    std::vector<int64_t> cur(acnt.begin(), acnt.end() - 1);
    for (int64_t v = 0; v < V; ++v) {
      const int64_t k = cur[va[v]]++;
      av_l[k] = vl[v];
      av_wh[k] = vw[v];
    }
  }
  // one visit per (agent, location): a second would make the agent meet itself
  for (int32_t i = 0; i < N; ++i) {
    const int64_t b = acnt[i], e = acnt[(size_t)i + 1];
    if (e - b < 2) continue;
    std::vector<int32_t> ls(av_l.begin() + b, av_l.begin() + e);
    std::sort(ls.begin(), ls.end());
    GABM_CHECK(std::adjacent_find(ls.begin(), ls.end()) == ls.end(), GABM_EINVAL,
               "an agent visits the same location twice");
  }
  G.n_loc = L;
  G.n_visits = V;
  GABM_HIP(dalloc(&G.lv_agent, V));
  GABM_HIP(dalloc(&G.lv_loc, V));
  GABM_HIP(dalloc(&G.lv_w, V));
  GABM_HIP(dalloc(&G.av_ptr, (size_t)N + 1));
  GABM_HIP(dalloc(&G.av_loc, V));
  GABM_HIP(dalloc(&G.av_w, V));
  GABM_HIP(dalloc(&G.loc_scratch, (size_t)2 * L));
  GABM_HIP(hipMemcpyAsync(G.lv_agent, lv_a.data(), sizeof(int32_t) * V, hipMemcpyHostToDevice, st));
  GABM_HIP(hipMemcpyAsync(G.lv_loc, lv_l.data(), sizeof(int32_t) * V, hipMemcpyHostToDevice, st));
  GABM_HIP(hipMemcpyAsync(G.lv_w, lv_wh.data(), sizeof(float) * V, hipMemcpyHostToDevice, st));
  GABM_HIP(hipMemcpyAsync(G.av_ptr, acnt.data(), sizeof(int64_t) * ((size_t)N + 1), hipMemcpyHostToDevice, st));
  GABM_HIP(hipMemcpyAsync(G.av_loc, av_l.data(), sizeof(int32_t) * V, hipMemcpyHostToDevice, st));
  GABM_HIP(hipMemcpyAsync(G.av_w, av_wh.data(), sizeof(float) * V, hipMemcpyHostToDevice, st));
  // the host vectors die on return: wait for the copies
  GABM_HIP(hipStreamSynchronize(st));
  return GABM_OK;
}

gabm_status build_graph(const gabm_graph_desc* d, hipStream_t st, Graph& G) {
  const int32_t N = d->n_agents;
  const int sym = (d->flags & GABM_SYMMETRIZE) ? 1 : 0;
  const int64_t Ein = d->n_edges;
  const int64_t E = sym ? 2 * Ein : Ein;
  G.N = N;
  G.n_pops = d->n_pops;
  G.n_age = d->n_age;
  G.E = E;
  G.pop_off_h.assign(d->pop_offsets, d->pop_offsets + d->n_pops + 1);
  G.er_mean = d->er_mean_deg;
  G.er_w = d->er_weight;
  G.er_off_h.assign(d->n_pops + 1, 0);
  for (int p = 0; p < d->n_pops; ++p) {
    const int64_t np = G.pop_off_h[p + 1] - G.pop_off_h[p];
    const int64_t M = (np >= 2 && d->er_mean_deg > 0.f) ? llround((double)np * (double)d->er_mean_deg / 2.0) : 0;
    G.er_off_h[p + 1] = G.er_off_h[p] + M;
  }

  GABM_HIP(dalloc(&G.pop_off, d->n_pops + 1));
  GABM_HIP(dalloc(&G.er_off, d->n_pops + 1));
  GABM_HIP(dalloc(&G.age, N));
  GABM_HIP(dalloc(&G.pop_of, N));
  GABM_HIP(dalloc(&G.row_ptr, (size_t)N + 1));
  GABM_HIP(dalloc(&G.col, E));
  GABM_HIP(dalloc(&G.w, E));
  GABM_HIP(hipMemcpyAsync(G.pop_off, G.pop_off_h.data(), sizeof(int32_t) * (d->n_pops + 1), hipMemcpyHostToDevice, st));
  GABM_HIP(hipMemcpyAsync(G.er_off, G.er_off_h.data(), sizeof(int64_t) * (d->n_pops + 1), hipMemcpyHostToDevice, st));
  GABM_HIP(hipMemcpyAsync(G.age, d->age, N, hipMemcpyDeviceToDevice, st));

  uint32_t* flag = nullptr;
  unsigned long long *deg = nullptr, *scan = nullptr, *sums = nullptr, *cursor = nullptr;
  double* wsum = nullptr;
  GABM_HIP(dalloc(&flag, 1));
  GABM_HIP(hipMemsetAsync(flag, 0, sizeof(uint32_t), st));
  const int64_t n1 = (int64_t)N + 1;
  const int64_t n_scan_tiles = (n1 + kScanTile - 1) / kScanTile;
  GABM_HIP(dalloc(&deg, n1));
  GABM_HIP(dalloc(&scan, n1));
  GABM_HIP(dalloc(&sums, n_scan_tiles));
  GABM_HIP(dalloc(&cursor, n1));
  GABM_HIP(dalloc(&wsum, 1));

  auto cleanup = [&]() {
    hipFree(flag); hipFree(deg); hipFree(scan); hipFree(sums); hipFree(cursor); hipFree(wsum);
  };

  if (Ein > 0)
    hipLaunchKernelGGL(k_validate, dim3(grid_for(Ein)), dim3(kBlock), 0, st, d->src, d->dst, d->w, Ein, N, G.pop_off,
                       d->n_pops, flag);
  hipLaunchKernelGGL(k_validate_age, dim3(grid_for(N)), dim3(kBlock), 0, st, G.age, N, d->n_age, flag);
  uint32_t hflag = 0;
  GABM_HIP(hipMemcpyAsync(&hflag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  GABM_HIP(hipStreamSynchronize(st));
  if (hflag) {
    cleanup();
    if (hflag & BAD_ID) { set_error("contact with agent id outside [0, n_agents)"); return GABM_ERANGE; }
    if (hflag & BAD_SELF) { set_error("self-contact (src == dst)"); return GABM_ERANGE; }
    if (hflag & BAD_POP) { set_error("contact between different populations"); return GABM_ERANGE; }
    if (hflag & BAD_AGE) { set_error("age group >= n_age"); return GABM_ERANGE; }
    set_error("contact weight negative or not finite");
    return GABM_EINVAL;
  }
  {
    const gabm_status rc = build_locations(d, st, G);
    if (rc != GABM_OK) {
      cleanup();
      return rc;
    }
  }

  GABM_HIP(hipMemsetAsync(deg, 0, sizeof(unsigned long long) * n1, st));
  if (Ein > 0)
    hipLaunchKernelGGL(k_degree, dim3(grid_for(Ein)), dim3(kBlock), 0, st, d->src, d->dst, Ein, sym, deg);
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)n_scan_tiles), dim3(kBlock), 0, st, deg, n1, scan, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, st, sums, n_scan_tiles);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)n_scan_tiles), dim3(kBlock), 0, st, scan, n1, sums, G.row_ptr, cursor);
  if (Ein > 0)
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(Ein)), dim3(kBlock), 0, st, d->src, d->dst, d->w, Ein, sym, cursor,
                       G.col, G.w);

  std::vector<int64_t> rp(n1);
  GABM_HIP(hipMemcpyAsync(rp.data(), G.row_ptr, sizeof(int64_t) * n1, hipMemcpyDeviceToHost, st));
  GABM_HIP(hipStreamSynchronize(st));
  if (rp[N] != E) {
    cleanup();
    set_error("internal: row_ptr total does not match the contact count");
    return GABM_EHIP;
  }

  // sort rows
  hipLaunchKernelGGL(k_sort_short, dim3(grid_for(N)), dim3(kBlock), 0, st, G.row_ptr, N, G.col, G.w);
  std::vector<int32_t> lrows, hrows;
  int64_t hmax = 0;
  for (int32_t i = 0; i < N; ++i) {
    const int64_t dd = rp[i + 1] - rp[i];
    if (dd > 32 && dd <= kSortLds) lrows.push_back(i);
    else if (dd > kSortLds) { hrows.push_back(i); hmax = std::max(hmax, dd); }
  }
  int32_t* drows = nullptr;
  unsigned long long* gscr = nullptr;
  int64_t P = 1;
  while (P < hmax) P <<= 1;
  if (!lrows.empty() || !hrows.empty()) {
    GABM_HIP(dalloc(&drows, lrows.size() + hrows.size()));
    GABM_HIP(hipMemcpyAsync(drows, lrows.data(), sizeof(int32_t) * lrows.size(), hipMemcpyHostToDevice, st));
    GABM_HIP(hipMemcpyAsync(drows + lrows.size(), hrows.data(), sizeof(int32_t) * hrows.size(), hipMemcpyHostToDevice, st));
    if (!hrows.empty()) GABM_HIP(dalloc(&gscr, P));
    if (!lrows.empty())
      hipLaunchKernelGGL(k_sort_long, dim3((unsigned)lrows.size()), dim3(kBlock), 0, st, G.row_ptr, drows,
                         (int)lrows.size(), G.col, G.w, gscr, (int64_t)0);
    // rows longer than the LDS sort share one scratch area: one at a time
    for (size_t k = 0; k < hrows.size(); ++k)
      hipLaunchKernelGGL(k_sort_long, dim3(1), dim3(kBlock), 0, st, G.row_ptr, drows + lrows.size() + k, 1, G.col,
                         G.w, gscr, P);
  }

  if (d->flags & GABM_CHECK_SYMMETRIC)
    hipLaunchKernelGGL(k_check_sym, dim3(grid_for(N)), dim3(kBlock), 0, st, G.row_ptr, G.col, G.w, N, flag);
  hipLaunchKernelGGL(k_pop_of, dim3(grid_for(N)), dim3(kBlock), 0, st, G.pop_off, d->n_pops, N, G.pop_of);
  GABM_HIP(hipMemsetAsync(wsum, 0, sizeof(double), st));
  if (E > 0) hipLaunchKernelGGL(k_weight_sum, dim3(grid_for(E, kBlock * 16)), dim3(kBlock), 0, st, G.w, E, wsum);

  std::vector<int32_t> tiles;
  make_tiles(rp, tiles, G.n_long, G.max_degree);
  G.n_tiles = (int32_t)tiles.size() - 1;
  GABM_HIP(dalloc(&G.tile_row, tiles.size()));
  GABM_HIP(hipMemcpyAsync(G.tile_row, tiles.data(), sizeof(int32_t) * tiles.size(), hipMemcpyHostToDevice, st));
  std::vector<TileInfo> tinfo(G.n_tiles);
  for (int32_t k = 0; k < G.n_tiles; ++k) {
    tinfo[k].r0 = tiles[k];
    tinfo[k].r1 = tiles[k + 1];
    tinfo[k].e0 = rp[tiles[k]];
    tinfo[k].e1 = rp[tiles[k + 1]];
    tinfo[k].pad0 = tinfo[k].pad1 = 0;
  }
  GABM_HIP(dalloc(&G.tiles, tinfo.size()));
  GABM_HIP(hipMemcpyAsync(G.tiles, tinfo.data(), sizeof(TileInfo) * tinfo.size(), hipMemcpyHostToDevice, st));
  {
    std::vector<int32_t> ft;
    int32_t nl = 0, md = 0;
    make_tiles(rp, ft, nl, md, kBTileCap, kBTileRows);
    G.n_btiles = (int32_t)ft.size() - 1;
    std::vector<TileInfo> fi(G.n_btiles);
    for (int32_t k = 0; k < G.n_btiles; ++k) {
      fi[k].r0 = ft[k];
      fi[k].r1 = ft[k + 1];
      fi[k].e0 = rp[ft[k]];
      fi[k].e1 = rp[ft[k + 1]];
      // rows of earlier tiles that start (empty) at this tile's first contact
      const int64_t first = std::lower_bound(rp.begin(), rp.begin() + ft[k], fi[k].e0) - rp.begin();
      fi[k].pad0 = (int32_t)(ft[k] - first);
      fi[k].pad1 = 0;
    }
    GABM_HIP(dalloc(&G.btiles, fi.size()));
    GABM_HIP(hipMemcpyAsync(G.btiles, fi.data(), sizeof(TileInfo) * fi.size(), hipMemcpyHostToDevice, st));
    GABM_HIP(hipStreamSynchronize(st));
  }
  // edge-parallel form for the persistent kernels (senders below 2^24)
  if (E > 0 && N < (1 << 24)) {
    const int64_t nch = (E + kChunk - 1) / kChunk;
    const int64_t npad = nch * kChunk;
    unsigned int* adv = nullptr;
    uint32_t* oflag = nullptr;
    GABM_HIP(dalloc(&adv, E));
    GABM_HIP(dalloc(&oflag, 1));
    GABM_HIP(hipMemsetAsync(adv, 0, sizeof(unsigned int) * E, st));
    GABM_HIP(hipMemsetAsync(oflag, 0, sizeof(uint32_t), st));
    GABM_HIP(dalloc(&G.colp, npad));
    GABM_HIP(dalloc(&G.wp, npad));
    hipLaunchKernelGGL(k_row_starts, dim3(grid_for(N)), dim3(kBlock), 0, st, G.row_ptr, N, E, adv);
    hipLaunchKernelGGL(k_pack_cols, dim3(grid_for(npad)), dim3(kBlock), 0, st, G.col, G.w, adv, E, npad, G.colp,
                       G.wp, oflag);
    // per chunk: rows starting before it, and in bit 31 whether a row starts
    // at the contact after it (always set for the last chunk, whose padding
    // ends the list)
    std::vector<uint32_t> crow(nch);
    {
      int64_t r = 0;  // rows r with rp[r] < k * kChunk
      for (int64_t k = 0; k < nch; ++k) {
        const int64_t e0 = k * kChunk;
        while (r <= N && rp[r] < e0) ++r;
        crow[k] = (uint32_t)r;
      }
      for (int64_t k = 0; k < nch; ++k) {  // crow[k + 1] is still unflagged here
        bool starts = true;
        if (k + 1 < nch) {
          const int64_t rn = crow[k + 1];  // first row starting at or after the next chunk
          starts = rn < N && rp[rn] == (k + 1) * kChunk;
        }
        if (starts) crow[k] |= 0x80000000u;
      }
    }
    GABM_HIP(dalloc(&G.chunk_row, nch));
    GABM_HIP(hipMemcpyAsync(G.chunk_row, crow.data(), sizeof(uint32_t) * nch, hipMemcpyHostToDevice, st));
    uint32_t of = 0;
    GABM_HIP(hipMemcpyAsync(&of, oflag, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GABM_HIP(hipStreamSynchronize(st));
    hipFree(adv);
    hipFree(oflag);
    if (of) {  // more than 255 consecutive empty rows somewhere: keep the tile kernels only
      hipFree(G.colp);
      hipFree(G.wp);
      hipFree(G.chunk_row);
      G.colp = nullptr;
      G.wp = nullptr;
      G.chunk_row = nullptr;
    } else {
      G.n_chunks = nch;
    }
  }
  if (E > 0 && N < (1 << 24)) {
    const gabm_status rc = build_sliced_stream(G, st);
    if (rc != GABM_OK) {
      hipFree(drows);
      hipFree(gscr);
      cleanup();
      return rc;
    }
  }
  GABM_HIP(hipMemcpyAsync(&hflag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  GABM_HIP(hipMemcpyAsync(&G.weight_sum, wsum, sizeof(double), hipMemcpyDeviceToHost, st));
  GABM_HIP(hipStreamSynchronize(st));
  GABM_HIP(hipGetLastError());
  hipFree(drows);
  hipFree(gscr);
  cleanup();
  if (hflag & BAD_SYM) {
    set_error("contact list is not symmetric");
    return GABM_ENOTSYM;
  }
  return GABM_OK;
}

}  // namespace gabm
