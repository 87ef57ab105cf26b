// Fused per-day kernels of one simulation (B = 1): the forward day
// (Transmit + Bernoulli draw + Progress + aggregates) and the reverse day
// (gather of the rate adjoint over the CSR + agent adjoint of the previous
// day), plus initial infections, the daily random layer and the reductions
// that close a run.
//
// Model: Section 3.1 (Eq. 1-3, Transmit / Progress / Aggregate), assumptions
// A1-A6 of Appendix A (one-day steps; no transmission on the day of exposure;
// no reinfection; contacts accumulate within a day, not across days) and the
// Gumbel-softmax relaxation of Appendix B.
#include <type_traits>

#include "agent.h"
#include "day_kernels.h"
#include "tile.h"

namespace gabm {

// ----------------------------------------------------------------- helpers

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f64(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0;
}
__global__ void k_fill_f32(float* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.f;
}
__global__ void k_copy_u32(uint32_t* d, const uint32_t* s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) d[i] = s[i];
}
__global__ void k_copy_f64(double* d, const double* s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) d[i] = s[i];
}
__global__ void k_copy_f32(float* d, const float* s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) d[i] = s[i];
}

// ----------------------------------------------------------------- initial infections (t = 0)
// Each agent is infected with probability i0 (Bernoulli on its INIT uniform),
// entering I with a full timer; the relaxed value y0 is the soft state.
template <typename RT, bool SOFT>
__global__ void __launch_bounds__(kBlock) k_init(InitArgs<RT> a) {
  __shared__ double red[kBlock / kWave];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < a.G.N;
  bool inf_now = false;
  double cs = 0.0, ci = 0.0;
  int p = 0;
  if (active) {
    p = pop_of_agent(a.G, i);
    const int set = set_of(a.P, p);
    const uint32_t loc = (uint32_t)(i - a.G.pop_off[p]);
    const double u = unit_u(rng_block(a.rng, loc, kDayInit, TAG_INIT, (uint32_t)p, a.stream).x);
    const double i0 = a.P.i0[set];
    if (SOFT) {
      double y0, dy0;
      relaxed_init(i0, u, a.P.tau, y0, dy0);
      a.x0[i] = (RT)y0;
      a.Sv[i] = (RT)(1.0 - y0);
      a.inf[i] = (RT)(a.P.TI * iota_at(a.P, a.P.tau_E + 1) * y0);  // day 0: tau_E + 1 days since exposure
      cs = 1.0 - y0;
      ci = y0;
    } else {
      inf_now = u < i0;
      a.rec[i] = inf_now ? make_rec(ST_I, (uint32_t)dwell_I(a.P, a.rng, loc, kDayInit, (uint32_t)p, a.stream), -1)
                         : make_rec(ST_S, 0, -1);
      cs = inf_now ? 0.0 : 1.0;
      ci = inf_now ? 1.0 : 0.0;
    }
  }
  if (!SOFT) {
    const unsigned long long b = __ballot(active && inf_now);
    if ((threadIdx.x & 63) == 0) or_ballot(a.maskI, blockIdx.x * kBlock + (threadIdx.x & ~63), b);
  }
  const int first = blockIdx.x * kBlock;
  const int last = min(a.G.N, first + kBlock) - 1;
  const bool uni = !a.P.per_pop || pop_of_agent(a.G, first) == pop_of_agent(a.G, last);
  const int slot = blockIdx.x & (kSlots - 1);
  if (uni) {
    const int o = a.P.per_pop ? pop_of_agent(a.G, first) : 0;
    cs = block_sum(cs, red);
    ci = block_sum(ci, red);
    if (threadIdx.x == 0) {
      double* c = a.cnt0 + ((int64_t)o * kSlots + slot) * kCnt;
      atomicAdd(&c[ST_S], cs);
      atomicAdd(&c[ST_I], ci);
    }
  } else if (active) {
    double* c = a.cnt0 + ((int64_t)p * kSlots + slot) * kCnt;
    atomicAdd(&c[ST_S], cs);
    atomicAdd(&c[ST_I], ci);
  }
}

// rebuild the infectious bit masks of the current day from the records
__global__ void k_mask_from_rec(const uint32_t* rec, int N, unsigned long long* mI, unsigned long long* mE, int withE) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < N;
  const uint32_t st = active ? rec_stage(rec[i]) : 0u;
  const unsigned long long bI = __ballot(active && st == ST_I);
  const unsigned long long bE = __ballot(active && st == ST_E);
  if ((threadIdx.x & 63) == 0) {
    const int base = blockIdx.x * kBlock + (threadIdx.x & ~63);
    or_ballot(mI, base, bI);
    if (withE) or_ballot(mE, base, bE);
  }
}

// ----------------------------------------------------------------- daily random layer
// Pair k of population p on day t: endpoints from Philox words 0 and 1,
// i = floor(x0 * N_p / 2^32), j' = floor(x1 * (N_p - 1) / 2^32), j = j' + (j' >= i).
__device__ __forceinline__ void er_pair(const DGraph& G, Rng rng, uint32_t stream, int t, int64_t k, int& gi, int& gj) {
  int lo = 0, hi = G.n_pops;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (G.er_off[mid] <= k) lo = mid; else hi = mid;
  }
  const int p = lo;
  const uint32_t kk = (uint32_t)(k - G.er_off[p]);
  const int off = G.pop_off[p];
  const uint32_t np = (uint32_t)(G.pop_off[p + 1] - off);
  const uint4 x = rng_block(rng, kk, (uint32_t)t, TAG_ER, (uint32_t)p, stream);
  const uint32_t i = __umulhi(x.x, np);
  const uint32_t jp = __umulhi(x.y, np - 1u);
  gi = off + (int)i;
  gj = off + (int)(jp + (jp >= i ? 1u : 0u));
}

// profile weight of an infectious endpoint from its record
__device__ __forceinline__ double er_iota(const ErArgs& a, int i) {
  const int k = days_since_exposure(a.rec[i], a.t, a.tau_E);
  return (double)a.iota[(k < 1 ? 1 : (k > a.W ? a.W : k)) - 1];
}

__global__ void k_er_fwd_hard(ErArgs a, const uint32_t* mI, const uint32_t* mE) {
  const double w = a.G.er_w;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < a.G.er_total; k += (int64_t)gridDim.x * blockDim.x) {
    int i, j;
    er_pair(a.G, a.rng, a.stream, a.t, k, i, j);
    double vi = a.TI * (double)mask_bit(mI, i), vj = a.TI * (double)mask_bit(mI, j);
    if (mE) {
      vi += a.TE * (double)mask_bit(mE, i);
      vj += a.TE * (double)mask_bit(mE, j);
    }
    if (a.iota) {
      if (vi != 0.0) vi *= er_iota(a, i);
      if (vj != 0.0) vj *= er_iota(a, j);
    }
    if (vj != 0.0) atomicAdd(&a.acc[i], w * vj);
    if (vi != 0.0) atomicAdd(&a.acc[j], w * vi);
  }
}

// real-valued per-agent vector (soft infectiousness forward, adjoint backward)
template <typename RT>
__global__ void k_er_vec(ErArgs a, const RT* v) {
  const double w = a.G.er_w;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < a.G.er_total; k += (int64_t)gridDim.x * blockDim.x) {
    int i, j;
    er_pair(a.G, a.rng, a.stream, a.t, k, i, j);
    const double vi = (double)v[i], vj = (double)v[j];
    if (vj != 0.0) atomicAdd(&a.acc[i], w * vj);
    if (vi != 0.0) atomicAdd(&a.acc[j], w * vi);
  }
}

__global__ void k_er_pairs_out(ErArgs a, int pop, int32_t* A, int32_t* Bo, int64_t cap) {
  const int64_t base = a.G.er_off[pop], n = a.G.er_off[pop + 1] - base;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n && k < cap; k += (int64_t)gridDim.x * blockDim.x) {
    int i, j;
    er_pair(a.G, a.rng, a.stream, a.t, base + k, i, j);
    A[k] = i;
    Bo[k] = j;
  }
}

// ----------------------------------------------------------------- forward day
// Output (aggregate) index of a receiver tile when all its agents belong to
// one output, else -1 (only tiles that straddle two populations).
__device__ __forceinline__ int tile_output(const DGraph& G, const DParams& P, int tile) {
  if (!P.per_pop) return 0;
  const int r0 = G.tile_row[tile], rl = G.tile_row[tile + 1] - 1;
  const int p0 = pop_of_agent(G, r0);
  return p0 == pop_of_agent(G, rl) ? p0 : -1;
}

template <typename RT, bool SOFT>
__global__ void __launch_bounds__(kBlock) k_day_fwd(FwdArgs<RT> a) {
  __shared__ TileShared sh;
  __shared__ unsigned int scnt[kCnt];
  const int tid = threadIdx.x;
  if (tid < kCnt) scnt[tid] = 0u;
  if (!SOFT) {
    // clear the masks of day t+2 (read last on day t-1, written next on day t+1)
    const int64_t chunk = (a.mask_words + gridDim.x - 1) / gridDim.x;
    const int64_t w0 = blockIdx.x * chunk;
    for (int64_t x = w0 + tid; x < w0 + chunk && x < a.mask_words; x += kBlock) {
      a.mI_clr[x] = 0ull;
      if (a.mE_clr) a.mE_clr[x] = 0ull;
    }
  }
  const DGraph& G = a.G;
  const DParams& P = a.P;
  const int t = a.t;
  const int o_tile = tile_output(G, P, blockIdx.x);
  const int slot = blockIdx.x & (kSlots - 1);
  auto cnt_at = [&](int o) { return a.cnt + (((int64_t)o * P.K + t) * kSlots + slot) * kCnt; };

  // per-agent inputs of the epilogue, loaded before the contact stream
  const TileBounds tb = tile_bounds(G, blockIdx.x);
  const bool longrow = tb.e1 - tb.e0 > kTileCap;
  const int my_i = longrow ? tb.r0 : tb.r0 + tid;
  const bool my_on = longrow ? tid == 0 : tid < tb.r1 - tb.r0;
  uint32_t pre_rec = 0u;
  int pre_age = 0;
  double pre_aer = 0.0;
  if (my_on) {
    if (!SOFT) pre_rec = a.rec_in[my_i];
    pre_age = G.age[my_i];
    if (a.A_er) pre_aer = a.A_er[my_i];
  }

  auto ev = [&](int c, float wf) -> double {
    const double w = (double)wf;
    if (SOFT) return w * (double)a.inf_cur[c];
    double v = P.TI * (double)mask_bit(a.mI_cur, c);
    if (a.mE_cur) v += P.TE * (double)mask_bit(a.mE_cur, c);
    if (P.iota && v != 0.0) v *= iota_at(P, days_since_exposure(a.rec_in[c], t, P.tau_E));
    return w * v;
  };

  auto epi = [&](int i, double A, bool active) {
    uint32_t newst = 0;
    bool removed = false;
    double cS = 0, cE = 0, cI = 0, cRM = 0, cD = 0;
    int p = 0;
    if (active) {
      if (a.A_er) {
        A += pre_aer;
        a.A_er[i] = 0.0;
      }
      p = pop_of_agent(G, i);
      const int set = set_of(P, p);
      const uint32_t loc = (uint32_t)(i - G.pop_off[p]);
      if (a.A_st) a.A_st[i] = (RT)A;
      if (SOFT) {
        const double Rt = P.R[set * P.K + t], Sa = P.S[set * P.n_age + pre_age], Zp = P.Z[p];
        const double lam = rate(Rt, Sa, A, Zp);
        const double q = -expm1(-lam);
        const double u = unit_u(rng_block(a.rng, loc, (uint32_t)t, TAG_INFECT, (uint32_t)p, a.stream).x);
        if (a.lam_out) a.lam_out[i] = lam;
        double y, dydl;
        relaxed_sample(lam, q, u, P.tau, y, dydl);
        const double S0 = (double)a.Sv[i];
        const double xi = S0 * y;
        const double S1 = S0 - xi;
        if (a.S_st) a.S_st[i] = (RT)S0;
        a.Sv[i] = (RT)S1;
        const int W = P.tau_E + P.tau_I;
        RT* slotp = a.ring + (int64_t)(t % W) * G.N;
        const double old = (double)slotp[i];  // exposure of day t-W
        slotp[i] = (RT)xi;
        // exposure windows of day t+1 (wE, wI), and the same weighted by the
        // infectiousness profile (pE, pI)
        double wE = 0.0, wI = 0.0, pE = 0.0, pI = 0.0;
        for (int k = 1; k <= W; ++k) {
          const int u_ = t + 1 - k;
          if (u_ < 0) break;
          const double xv = (double)a.ring[(int64_t)(u_ % W) * G.N + i];
          if (k <= P.tau_E) {
            wE += xv;
            pE += iota_at(P, k) * xv;
          } else {
            wI += xv;
            pI += iota_at(P, k) * xv;
          }
        }
        const double x0 = (double)a.x0[i];
        if (t + 1 < P.tau_I) {
          wI += x0;
          pI += iota_at(P, t + 1 + P.tau_E + 1) * x0;
        }
        a.inf_next[i] = (RT)(P.TE * pE + P.TI * pI);
        cS = S1; cE = wE; cI = wI; cRM = 1.0 - S1 - wE - wI;
        cD = old + (t == P.tau_I - 1 ? x0 : 0.0);
      } else {
        const HardDay hd = hard_agent_day(P, a.rng, a.stream, t, set, p, loc, pre_age, A, pre_rec, a.lam_out ? &a.lam_out[i] : nullptr);
        if (a.fl_st) a.fl_st[i] = (uint8_t)((hd.was_s ? 1u : 0u) | (hd.h ? 2u : 0u));
        newst = hd.newst;
        removed = hd.removed;
        a.rec_out[i] = hd.rec;
      }
    }
    if (!SOFT) {
      const int lane = tid & 63;
      const unsigned long long bI = __ballot(active && newst == ST_I);
      const unsigned long long bE = __ballot(active && newst == ST_E);
      if (lane == 0) {
        or_ballot(a.mI_next, i, bI);
        if (a.mE_next) or_ballot(a.mE_next, i, bE);
      }
      if (a.cnt) {
        if (o_tile >= 0) {
          const unsigned long long c0 = __ballot(active && newst == ST_S), c3 = __ballot(active && newst == ST_R),
                                   c4 = __ballot(active && newst == ST_M), c5 = __ballot(active && removed);
          if (lane == 0) {
            atomicAdd(&scnt[ST_S], (unsigned)__popcll(c0));
            atomicAdd(&scnt[ST_E], (unsigned)__popcll(bE));
            atomicAdd(&scnt[ST_I], (unsigned)__popcll(bI));
            atomicAdd(&scnt[ST_R], (unsigned)__popcll(c3));
            atomicAdd(&scnt[ST_M], (unsigned)__popcll(c4));
            atomicAdd(&scnt[5], (unsigned)__popcll(c5));
          }
          __syncthreads();
          if (tid < 6 && scnt[tid]) atomicAdd(&cnt_at(o_tile)[tid], (double)scnt[tid]);
        } else if (active) {
          double* c = cnt_at(p);
          atomicAdd(&c[newst], 1.0);
          if (removed) atomicAdd(&c[5], 1.0);
        }
      }
    } else if (a.cnt) {
      if (o_tile >= 0) {
        cS = block_sum(cS, sh.red);
        cE = block_sum(cE, sh.red);
        cI = block_sum(cI, sh.red);
        cRM = block_sum(cRM, sh.red);
        cD = block_sum(cD, sh.red);
        if (tid == 0) {
          double* c = cnt_at(o_tile);
          atomicAdd(&c[ST_S], cS);
          atomicAdd(&c[ST_E], cE);
          atomicAdd(&c[ST_I], cI);
          atomicAdd(&c[ST_R], cRM);  // split into R and M by m when the run closes
          atomicAdd(&c[5], cD);
        }
      } else if (active) {
        double* c = cnt_at(p);
        atomicAdd(&c[ST_S], cS);
        atomicAdd(&c[ST_E], cE);
        atomicAdd(&c[ST_I], cI);
        atomicAdd(&c[ST_R], cRM);
        atomicAdd(&c[5], cD);
      }
    }
  };
  tile_pass(G, tb, sh, ev, epi);
}

// ----------------------------------------------------------------- reverse day
// Step t: inf_bar^t = sum over contacts of w * g^t (the adjoint of the
// neighbour sum is a gather over the same, symmetric CSR), then the agent
// adjoint of day t-1 (straight-through or exact relaxed derivative), and on
// t = 0 the adjoint of the initial infections.
template <typename RT, bool SOFT, bool DWELL>
__global__ void __launch_bounds__(kBlock) k_day_bwd(BwdArgs<RT> a) {
  __shared__ TileShared sh;
  __shared__ double sg[2 + 16];  // dR, di0, dS[n_age]
  __shared__ double sdw[16];     // dwell log-weight gradients (E 0-7, I 8-15)
  const int tid = threadIdx.x;
  if (tid < 18) sg[tid] = 0.0;
  if (tid < 16) sdw[tid] = 0.0;
  const DGraph& G = a.G;
  const DParams& P = a.P;
  const int t = a.t;
  const int W = P.tau_E + P.tau_I;
  const int o_tile = tile_output(G, P, blockIdx.x);  // == set of the tile when uniform
  const int slot = blockIdx.x & (kSlots - 1);

  // per-agent inputs of the epilogue, loaded before the contact stream
  const TileBounds tb = tile_bounds(G, blockIdx.x);
  const bool longrow = tb.e1 - tb.e0 > kTileCap;
  const int my_i = longrow ? tb.r0 : tb.r0 + tid;
  const bool my_on = longrow ? tid == 0 : tid < tb.r1 - tb.r0;
  int pre_age = 0;
  double pre_A = 0.0, pre_Sbar = 0.0, pre_ier = 0.0;
  uint32_t pre_fl = 0u;
  if (my_on) {
    pre_age = G.age[my_i];
    pre_Sbar = (double)a.Sbar[my_i];
    if (t >= 1) {
      pre_A = (double)a.A_st[my_i];
      if (!SOFT) pre_fl = a.fl_st[my_i];
    }
    if (a.do_gather && a.infbar_er) pre_ier = a.infbar_er[my_i];
  }

  auto ev = [&](int c, float wf) -> double {
    if (!a.do_gather) return 0.0;
    return (double)wf * (double)a.g_cur[c];
  };

  auto epi = [&](int i, double infbar, bool active) {
    if (active) {
      if (a.do_gather) {
        if (a.infbar_er) {
          infbar += pre_ier;
          a.infbar_er[i] = 0.0;
        }
        a.ring[(int64_t)(t % W) * G.N + i] = (RT)infbar;
      }
      const int p = pop_of_agent(G, i), set = set_of(P, p);
      const int o = P.per_pop ? p : 0;
      const uint32_t loc = (uint32_t)(i - G.pop_off[p]);
      const double m = P.m[set];
      if (t >= 1) {
        const int d = t - 1;
        // inf_bar over the days after exposure on day d (E for dE days, then
        // I until day d + dL), weighted by the profile
        int dE = P.tau_E, dL = W;
        if (DWELL && P.dwell_E) {
          dE = dwell_E(P, a.rng, loc, (uint32_t)d, (uint32_t)p, a.stream);
          dL = dE + dwell_I(P, a.rng, loc, (uint32_t)d, (uint32_t)p, a.stream);
        }
        double sE = 0.0, sI = 0.0;
        for (int k = 1; k <= dL; ++k) {
          const double v = iota_at(P, k) * (double)a.ring[(int64_t)((d + k) % W) * G.N + i];
          if (k <= dE) sE += v; else sI += v;
        }
        const double drm_bar = (d + dL < P.K) ? m * a.Dbar[(int64_t)o * P.K + d + dL] : 0.0;
        const double A = pre_A;
        double Sv, h;
        if (SOFT) {
          Sv = (double)a.S_st[i];
          h = 0.0;
        } else {
          Sv = (double)(pre_fl & 1u);
          h = (double)((pre_fl >> 1) & 1u);
        }
        const AdjOut ad = agent_adjoint<std::is_same<RT, float>::value>(P, a.rng, a.stream, d, set, p, loc, pre_age, A, Sv, h, SOFT, sE, sI, pre_Sbar,
                                        drm_bar);
        if (DWELL && !SOFT && a.gdw && Sv != 0.0 && h != 0.0) {  // an exposure on day d: its drawn lengths' gradient
          double cE[8], cI[8], pre[17], gE[8], gI[8];
          const int aS = dwell_relaxed(P.dwell_E, P.tau_E, a.rng, loc, (uint32_t)d, TAG_DWELL_E, (uint32_t)p, a.stream,
                                       P.tau, cE);
          const int bS = dwell_relaxed(P.dwell_I, P.tau_I, a.rng, loc, (uint32_t)d, TAG_DWELL_I, (uint32_t)p, a.stream,
                                       P.tau, cI);
          pre[0] = 0.0;
          for (int k = 1; k <= W; ++k)
            pre[k] = pre[k - 1] + iota_at(P, k) * (double)a.ring[(int64_t)((d + k) % W) * G.N + i];
          auto DR = [&](int x) { return d + x < P.K ? m * a.Dbar[(int64_t)o * P.K + d + x] : 0.0; };
          dwell_sensitivities(P, pre, aS, bS, DR, gE, gI);
          st_categorical(cE, gE, P.tau_E, P.tau, sdw);
          st_categorical(cI, gI, P.tau_I, P.tau, sdw + 8);
        }
        a.Sbar[i] = (RT)ad.Sbar;
        const double lam_bar = ad.lam_bar;
        a.g_prev[i] = (RT)ad.g;
        const double Rt = P.R[set * P.K + d], Sa = P.S[set * P.n_age + pre_age], Zp = P.Z[p];
        if (lam_bar != 0.0) {
          const double base = lam_bar * A / Zp;
          if (o_tile >= 0) {
            atomicAdd(&sg[0], base * Sa);
            atomicAdd(&sg[2 + pre_age], base * Rt);
          } else {
            atomicAdd(&a.gR[((int64_t)set * P.K + d) * kSlots + slot], base * Sa);
            atomicAdd(&a.gS[((int64_t)set * P.n_age + pre_age) * kSlots + slot], base * Rt);
          }
        }
      } else {
        // initial infections: x0_bar = T_I sum_{t<tau_I} inf_bar^t + m Dbar^{tau_I-1} - Sbar^0
        double sI = 0.0;  // day k is tau_E + 1 + k days after the initial infection's exposure
        const int dI0 = DWELL ? dwell_I(P, a.rng, loc, kDayInit, (uint32_t)p, a.stream) : P.tau_I;
        for (int k = 0; k < dI0; ++k) sI += iota_at(P, P.tau_E + 1 + k) * (double)a.ring[(int64_t)(k % W) * G.N + i];
        const double x0_bar =
            P.TI * sI + ((dI0 - 1 < P.K) ? m * a.Dbar[(int64_t)o * P.K + dI0 - 1] : 0.0) - pre_Sbar;
        const double u = unit_u(rng_block(a.rng, loc, kDayInit, TAG_INIT, (uint32_t)p, a.stream).x);
        double y0, dy0;
        relaxed_init((double)P.i0[set], u, P.tau, y0, dy0);
        const double v = x0_bar * dy0;
        if (v != 0.0) {
          if (o_tile >= 0) atomicAdd(&sg[1], v);
          else atomicAdd(&a.gi0[(int64_t)set * kSlots + slot], v);
        }
        if (DWELL && !SOFT && a.gdw && u < (double)P.i0[set]) {  // a hard initial infection: its I length's gradient
          double cI[8], gI[8];
          dwell_relaxed(P.dwell_I, P.tau_I, a.rng, loc, kDayInit, TAG_DWELL_I, (uint32_t)p, a.stream, P.tau, cI);
          double run = 0.0;
          for (int b = 1; b <= P.tau_I; ++b) {
            run += iota_at(P, P.tau_E + b) * (double)a.ring[(int64_t)((b - 1) % W) * G.N + i];
            gI[b - 1] = P.TI * run + (b - 1 < P.K ? m * a.Dbar[(int64_t)o * P.K + b - 1] : 0.0);
          }
          st_categorical(cI, gI, P.tau_I, P.tau, sdw + 8);
        }
      }
    }
    __syncthreads();
    if (o_tile >= 0) {
      const int set = o_tile;
      if (t >= 1) {
        if (tid == 0 && sg[0] != 0.0) atomicAdd(&a.gR[((int64_t)set * P.K + (t - 1)) * kSlots + slot], sg[0]);
        if (tid < P.n_age && sg[2 + tid] != 0.0)
          atomicAdd(&a.gS[((int64_t)set * P.n_age + tid) * kSlots + slot], sg[2 + tid]);
      } else if (tid == 0 && sg[1] != 0.0) {
        atomicAdd(&a.gi0[(int64_t)set * kSlots + slot], sg[1]);
      }
    }
    if (DWELL && a.gdw && tid < 16 && sdw[tid] != 0.0) atomicAdd(&a.gdw[tid * kSlots + slot], sdw[tid]);
  };
  tile_pass(G, tb, sh, ev, epi);
}

// ----------------------------------------------------------------- closing reductions
// One block per simulation: sum the spread accumulators of every day in a
// fixed order, form deaths, loss and the deaths adjoint 2 (D - y) / K.
__global__ void k_fin_fwd(FinArgs a) {
  const int o = blockIdx.x;
  __shared__ double red[kBlock / kWave];
  const double m = (double)a.m[o % a.n_sets];
  double lsum = 0.0;
  for (int t = threadIdx.x; t <= a.K; t += blockDim.x) {
    const double* src = t == 0 ? a.cnt0 + (int64_t)o * kSlots * kCnt : a.cnt + ((int64_t)o * a.K + (t - 1)) * kSlots * kCnt;
    double c[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < kSlots; ++s)
      for (int k = 0; k < 6; ++k) c[k] += src[s * kCnt + k];
    double* out = a.counts + ((int64_t)o * (a.K + 1) + t) * 5;
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2];
    if (a.soft) {
      out[3] = (1.0 - m) * c[3];
      out[4] = m * c[3];
    } else {
      out[3] = c[3];
      out[4] = c[4];
    }
    if (t >= 1) {
      const double drm = c[5];
      const double D = m * drm;
      const double y = a.target ? a.target[(int64_t)o * a.target_stride + (t - 1)] : D;
      a.drm_int[(int64_t)o * a.K + t - 1] = drm;
      if (a.drm) a.drm[(int64_t)o * a.K + t - 1] = drm;
      if (a.deaths) a.deaths[(int64_t)o * a.K + t - 1] = D;
      a.Dbar[(int64_t)o * a.K + t - 1] = 2.0 * (D - y) / a.K;
      lsum += (D - y) * (D - y);
    }
  }
  lsum = block_sum(lsum, red);
  if (threadIdx.x == 0 && a.loss) a.loss[o] = lsum / a.K;
}

// deaths adjoint of the reverse pass: weight * 2 (D - y) / K + upstream dL/dD
__global__ void k_dbar_eff(int n_out, int K, const double* Dbar, const double* w, const double* db, double* out) {
  const int64_t n = (int64_t)n_out * K;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(x / K);
    out[x] = (w ? w[o] : 1.0) * Dbar[x] + (db ? db[x] : 0.0);
  }
}

// One block per parameter set: sum slots into the outputs; dm from aggregates.
__global__ void k_fin_bwd(FinBwdArgs a) {
  const int set = blockIdx.x;
  __shared__ double red[kBlock / kWave];
  for (int t = threadIdx.x; t < a.K; t += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < kSlots; ++k) s += a.gR[((int64_t)set * a.K + t) * kSlots + k];
    a.dR[(int64_t)set * a.K + t] = s;
  }
  for (int g = threadIdx.x; g < a.n_age; g += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < kSlots; ++k) s += a.gS[((int64_t)set * a.n_age + g) * kSlots + k];
    a.dS[(int64_t)set * a.n_age + g] = s;
  }
  double dm = 0.0;
  for (int o = set; o < a.n_out; o += a.n_sets)
    for (int t = threadIdx.x; t < a.K; t += blockDim.x)
      dm += a.Dbar[(int64_t)o * a.K + t] * a.drm_int[(int64_t)o * a.K + t];
  dm = block_sum(dm, red);
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < kSlots; ++k) s += a.gi0[(int64_t)set * kSlots + k];
    a.di0[set] = s;
    a.dm[set] = dm;
  }
  if (set == 0 && a.gdw && (int)threadIdx.x < 16) {
    const int j = threadIdx.x;
    double s = 0.0;
    for (int k = 0; k < kSlots; ++k) s += a.gdw[j * kSlots + k];
    if (j < 8 && j < a.tau_E && a.ddw_E) a.ddw_E[j] = s;
    if (j >= 8 && j - 8 < a.tau_I && a.ddw_I) a.ddw_I[j - 8] = s;
  }
}

// ----------------------------------------------------------------- explicit instantiations
template __global__ void k_init<float, false>(InitArgs<float>);
template __global__ void k_init<float, true>(InitArgs<float>);
template __global__ void k_init<double, false>(InitArgs<double>);
template __global__ void k_init<double, true>(InitArgs<double>);
template __global__ void k_day_fwd<float, false>(FwdArgs<float>);
template __global__ void k_day_fwd<float, true>(FwdArgs<float>);
template __global__ void k_day_fwd<double, false>(FwdArgs<double>);
template __global__ void k_day_fwd<double, true>(FwdArgs<double>);
template __global__ void k_day_bwd<float, false, false>(BwdArgs<float>);
template __global__ void k_day_bwd<float, true, false>(BwdArgs<float>);
template __global__ void k_day_bwd<double, false, false>(BwdArgs<double>);
template __global__ void k_day_bwd<double, true, false>(BwdArgs<double>);
template __global__ void k_day_bwd<float, false, true>(BwdArgs<float>);
template __global__ void k_day_bwd<double, false, true>(BwdArgs<double>);
template __global__ void k_er_vec<float>(ErArgs, const float*);
template __global__ void k_er_vec<double>(ErArgs, const double*);

}  // namespace gabm
