// Receiver-tile pass shared by the forward and reverse day kernels.
//
// A tile is a run of consecutive receivers whose contacts (at most kTileCap)
// are staged in LDS, then reduced per receiver by a group of lanes (the
// group width is the largest power of two such that all receivers of the
// tile get one); a single receiver with more than kTileCap contacts is
// reduced by the whole block.  Sums are formed in double precision.
//
// Memory-level parallelism: each thread owns kPer = kTileCap / kBlock
// contacts of the tile and issues all their sender/weight loads before any
// dependent gather, then all gathers, so one tile costs two memory round
// trips instead of one per contact batch.  The contact stream is read once
// per day, so it is loaded non-temporally and leaves the caches to the
// gathered per-agent vectors.
//
// Afterwards every thread of the block calls the epilogue with its receiver
// (thread t -> receiver r0 + t), so wave-wide ballots in the epilogue see
// consecutive agents.
#pragma once

#include "gabm_device.h"

namespace gabm {

constexpr int kPer = kTileCap / kBlock;

struct TileShared {
  double val[kTileCap];
  double row[kTileRows];
  int rofs[kTileRows + 1];
  double red[kBlock / kWave];
};

struct TileBounds {
  int r0, r1;
  int64_t e0, e1;
};

__device__ __forceinline__ TileBounds tile_bounds(const DGraph& G, int tile) {
  const TileInfo ti = G.tiles[tile];
  TileBounds b;
  b.r0 = ti.r0;
  b.r1 = ti.r1;
  b.e0 = ti.e0;
  b.e1 = ti.e1;
  return b;
}

// EdgeVal: double (int sender, float weight)
template <class EdgeVal, class Epilogue>
__device__ __forceinline__ void tile_pass(const DGraph& G, const TileBounds& tb, TileShared& sh, EdgeVal ev,
                                          Epilogue epi) {
  const int tid = threadIdx.x;
  const int r0 = tb.r0, nr = tb.r1 - tb.r0;
  const int64_t e0 = tb.e0, e1 = tb.e1;
  if (e1 - e0 > kTileCap) {  // one long receiver row, reduced by the block
    double acc = 0.0;
    for (int64_t base = e0; base < e1; base += kTileCap) {
      int c[kPer];
      float w[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int64_t e = base + tid + k * kBlock;
        const bool ok = e < e1;
        c[k] = ok ? __builtin_nontemporal_load(&G.col[e]) : -1;
        w[k] = ok ? __builtin_nontemporal_load(&G.w[e]) : 0.f;
      }
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        if (c[k] >= 0) acc += ev(c[k], w[k]);
    }
    acc = block_sum(acc, sh.red);
    epi(r0, acc, tid == 0);
    return;
  }
  for (int t = tid; t <= nr; t += kBlock) sh.rofs[t] = (int)(G.row_ptr[r0 + t] - e0);
  {
    int c[kPer];
    float w[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t e = e0 + tid + k * kBlock;
      const bool ok = e < e1;
      c[k] = ok ? __builtin_nontemporal_load(&G.col[e]) : -1;
      w[k] = ok ? __builtin_nontemporal_load(&G.w[e]) : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (c[k] >= 0) sh.val[tid + k * kBlock] = ev(c[k], w[k]);
  }
  __syncthreads();
  int tpr = kWave;
  while (tpr > 1 && tpr * nr > kBlock) tpr >>= 1;
  const int g = tid / tpr, k = tid & (tpr - 1);
  double acc = 0.0;
  if (g < nr) {
    const int s = sh.rofs[g], en = min(sh.rofs[g + 1], kTileCap);
    for (int j = s + k; j < en; j += tpr) acc += sh.val[j];
  }
  for (int off = tpr >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (g < nr && k == 0) sh.row[g] = acc;
  __syncthreads();
  const bool active = tid < nr;
  epi(r0 + tid, active ? sh.row[tid] : 0.0, active);
}

}  // namespace gabm
