// Receiver-tile pass shared by the forward and reverse day kernels.
//
// A tile is a run of consecutive receivers whose contacts (at most kTileCap)
// are staged in LDS with fully coalesced loads of the CSR, then reduced per
// receiver by a group of lanes (the group width is the largest power of two
// such that all receivers of the tile get one); a single receiver with more
// than kTileCap contacts is reduced by the whole block.  Sums are formed in
// double precision.  Afterwards every thread of the block calls the epilogue
// with its receiver (thread t -> receiver r0 + t), so wave-wide ballots in
// the epilogue see consecutive agents.
#pragma once

#include "gabm_device.h"

namespace gabm {

struct TileShared {
  double val[kTileCap];
  double row[kTileRows];
  double red[kBlock / kWave];
};

template <class EdgeVal, class Epilogue>
__device__ __forceinline__ void tile_pass(const DGraph& G, int tile, TileShared& sh, EdgeVal ev, Epilogue epi) {
  const int tid = threadIdx.x;
  const int r0 = G.tile_row[tile], r1 = G.tile_row[tile + 1];
  const int64_t e0 = G.row_ptr[r0], e1 = G.row_ptr[r1];
  const int nr = r1 - r0;
  if (e1 - e0 > kTileCap) {  // one long receiver row
    double acc = 0.0;
    for (int64_t e = e0 + tid; e < e1; e += kBlock) acc += ev(e);
    acc = block_sum(acc, sh.red);
    epi(r0, acc, tid == 0);
    return;
  }
  for (int64_t e = e0 + tid; e < e1; e += kBlock) sh.val[e - e0] = ev(e);
  __syncthreads();
  int tpr = kWave;
  while (tpr > 1 && tpr * nr > kBlock) tpr >>= 1;
  const int g = tid / tpr, k = tid & (tpr - 1);
  double acc = 0.0;
  if (g < nr) {
    const int64_t s = G.row_ptr[r0 + g] - e0, len = G.row_ptr[r0 + g + 1] - G.row_ptr[r0 + g];
    for (int64_t j = k; j < len; j += tpr) acc += sh.val[s + j];
  }
  for (int off = tpr >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (g < nr && k == 0) sh.row[g] = acc;
  __syncthreads();
  const bool active = tid < nr;
  epi(r0 + tid, active ? sh.row[tid] : 0.0, active);
}

}  // namespace gabm
