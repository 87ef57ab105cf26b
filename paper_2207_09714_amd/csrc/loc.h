// Agent-location layer (the GradABM-JUNE form of Section 6): agents meet at
// locations instead of along stored pairwise contacts.  For one day and one
// per-agent value x (the infectiousness of the forward step, the rate
// adjoint g of the reverse step):
//   pressure   P_l = sum over visits v at l of w_v * x_{a_v}
//   agent sum  acc_i += sum over visits v of i of w_v * (P_{l_v} - w_v * x_i)
// which is the neighbour sum over the clique graph w_ij = sum_l w_il * w_jl
// without self-contact.  That graph is symmetric, so the reverse step is the
// same two passes applied to g.  Storage and traffic are O(visits), where the
// expanded graph needs the sum of squared location sizes.
#pragma once

#include "day_kernels.h"
#include "gabm_device.h"

namespace gabm {

struct LocView {
  int32_t N = 0, n_loc = 0;
  int64_t V = 0;
  const int32_t* lv_agent = nullptr;  // location-sorted visits
  const int32_t* lv_loc = nullptr;
  const float* lv_w = nullptr;
  const int64_t* av_ptr = nullptr;    // agent-sorted visits
  const int32_t* av_loc = nullptr;
  const float* av_w = nullptr;
};

// hard state: T_I for an infectious agent, T_E for an exposed one (when the
// masks of exposed agents are kept), times the profile weight of its days
// since exposure when a profile is given
struct LocHardVal {
  const uint32_t* mI = nullptr;
  const uint32_t* mE = nullptr;
  double TI = 0.0, TE = 0.0;
  const uint32_t* rec = nullptr;
  const float* iota = nullptr;
  int t = 0, tau_E = 0, W = 0;
  __device__ __forceinline__ double at(int c) const {
    double v = TI * (double)mask_bit(mI, c);
    if (mE) v += TE * (double)mask_bit(mE, c);
    if (iota && v != 0.0) {
      const int k = days_since_exposure(rec[c], t, tau_E);
      v *= (double)iota[(k < 1 ? 1 : (k > W ? W : k)) - 1];
    }
    return v;
  }
};

// a dense per-agent vector (relaxed infectiousness, or the rate adjoint)
template <typename RT>
struct LocVecVal {
  const RT* v = nullptr;
  __device__ __forceinline__ double at(int c) const { return (double)v[c]; }
};

// P must be zero on entry (the previous pass's k_loc_gather clears it).  Each wave takes 64 consecutive location-sorted
// visits; a segmented scan over the wave (runs of one location are
// contiguous) leaves each run's total in its last lane, which adds it to P_l:
// one atomic per location and wave.
template <class V>
__global__ void __launch_bounds__(kBlock) k_loc_pressure(LocView L, V val, double* P) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < L.V; base += stride) {
    const int64_t v = base + threadIdx.x;
    int l = -1;
    double x = 0.0;
    if (v < L.V) {
      l = L.lv_loc[v];
      const double a = val.at(L.lv_agent[v]);
      if (a != 0.0) x = (double)L.lv_w[v] * a;
    }
    for (int d = 1; d < kWave; d <<= 1) {
      const double y = __shfl_up(x, d, kWave);
      const int ly = __shfl_up(l, d, kWave);
      if (lane >= d && ly == l) x += y;
    }
    const int ln = __shfl_down(l, 1, kWave);
    const bool last = lane == kWave - 1 || ln != l;
    if (l >= 0 && last && x != 0.0) atomicAdd(&P[l], x);
  }
}

// acc_i += sum over i's visits of w_v * (P_l - w_v * x_i); one thread per
// agent (an agent has a handful of visits).  The visitor's own share is
// formed with the same product as in the pressure pass and subtracted
// before the multiplication, without contraction, so an agent never meets
// itself.  The pressures alternate between two buffers: this pass also
// clears `P_next`, the one the next pass accumulates into, which saves a
// separate clearing launch per pass.
template <class V>
__global__ void __launch_bounds__(kBlock) k_loc_gather(LocView L, V val, const double* P, double* acc,
                                                       double* P_next) {
#pragma clang fp contract(off)
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x; l < L.n_loc; l += stride) P_next[l] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < L.N; i += stride) {
    const int64_t b = L.av_ptr[i], e = L.av_ptr[i + 1];
    if (b == e) continue;
    const double xi = val.at((int)i);
    double s = 0.0;
    for (int64_t k = b; k < e; ++k) {
      const double w = (double)L.av_w[k];
      const double own = xi != 0.0 ? w * xi : 0.0;
      s += w * (P[L.av_loc[k]] - own);
    }
    if (s != 0.0) acc[i] += s;
  }
}

// The per-agent sum of k_loc_gather for one agent, inside another kernel
// (same arithmetic, no contraction).
__device__ __forceinline__ double loc_agent_sum(const LocFuse& L, int64_t i, double xi) {
#pragma clang fp contract(off)
  const int64_t b = L.av_ptr[i], e = L.av_ptr[i + 1];
  double s = 0.0;
  for (int64_t k = b; k < e; ++k) {
    const double w = (double)L.av_w[k];
    const double own = xi != 0.0 ? w * xi : 0.0;
    s += w * (L.P[L.av_loc[k]] - own);
  }
  return s;
}

}  // namespace gabm
