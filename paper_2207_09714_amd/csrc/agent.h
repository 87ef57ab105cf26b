// Per-agent work of one day, shared by every kernel family.
//
// Forward (hard state): the Bernoulli draw of Eq. 3 on the aggregate rate
// and Progress (Section 3.1): E and I timers count down, E -> I after tau_E
// days, I -> R or M after tau_I days (M with probability m), and a
// susceptible agent whose draw succeeds becomes E (it cannot transmit on the
// day of exposure, assumption A2).
//
// Reverse (straight-through / relaxed adjoint of one day, for one agent):
//   xi_bar = m Dbar^{d+W} + T_I sum_{I window} inf_bar + T_E sum_{E window} inf_bar - Sbar^{d+1}
//   Sbar^d = Sbar^{d+1} + h^d xi_bar
//   lambda_bar = S^d xi_bar dy/dlambda,   g^d = R S_a / Z lambda_bar
// with the window sums over the W = tau_E + tau_I following days.
#pragma once

#include "gabm_device.h"

namespace gabm {

// Gumbel-max draw of a length in 1..n from log weights lw: the index that
// maximises lw[k] - log(-log u_k) is distributed as softmax(lw) (first
// maximum on a tie).  u_k is word k mod 4 of the block with tag tag0 + k / 4.
__device__ __forceinline__ int dwell_draw(const float* lw, int n, Rng rng, uint32_t loc, uint32_t day, uint32_t tag0,
                                          uint32_t p, uint32_t stream) {
  int best = 0;
  double bv = -INFINITY;
  uint4 x = make_uint4(0u, 0u, 0u, 0u);
  for (int k = 0; k < n; ++k) {
    if ((k & 3) == 0) x = rng_block(rng, loc, day, tag0 + (uint32_t)(k >> 2), p, stream);
    const uint32_t w = (k & 3) == 0 ? x.x : ((k & 3) == 1 ? x.y : ((k & 3) == 2 ? x.z : x.w));
    const double v = (double)lw[k] - log(-log(unit_u(w)));
    if (v > bv) {
      bv = v;
      best = k;
    }
  }
  return best + 1;
}

// E and I lengths of an exposure of agent `loc` (population p) on `day`
// (kDayInit for an initial infection's I length): drawn when the parameters
// carry dwell tables, tau_E / tau_I otherwise
__device__ __forceinline__ int dwell_E(const DParams& P, Rng rng, uint32_t loc, uint32_t day, uint32_t p,
                                       uint32_t stream) {
  return P.dwell_E ? dwell_draw(P.dwell_E, P.tau_E, rng, loc, day, TAG_DWELL_E, p, stream) : P.tau_E;
}
__device__ __forceinline__ int dwell_I(const DParams& P, Rng rng, uint32_t loc, uint32_t day, uint32_t p,
                                       uint32_t stream) {
  return P.dwell_I ? dwell_draw(P.dwell_I, P.tau_I, rng, loc, day, TAG_DWELL_I, p, stream) : P.tau_I;
}
// The relaxed one-hot ch = softmax((lw + G) / tau) of the same draw (the
// straight-through Gumbel-softmax of Jang, Gu & Poole 2017); returns the
// drawn length.
__device__ __forceinline__ int dwell_relaxed(const float* lw, int n, Rng rng, uint32_t loc, uint32_t day, uint32_t tag0,
                                             uint32_t p, uint32_t stream, double tau, double* ch) {
  int best = 0;
  double bv = -INFINITY, mx = -INFINITY;
  uint4 x = make_uint4(0u, 0u, 0u, 0u);
  for (int k = 0; k < n; ++k) {
    if ((k & 3) == 0) x = rng_block(rng, loc, day, tag0 + (uint32_t)(k >> 2), p, stream);
    const uint32_t w = (k & 3) == 0 ? x.x : ((k & 3) == 1 ? x.y : ((k & 3) == 2 ? x.z : x.w));
    const double v = (double)lw[k] - log(-log(unit_u(w)));
    if (v > bv) {
      bv = v;
      best = k;
    }
    ch[k] = v / tau;
    mx = fmax(mx, ch[k]);
  }
  double sum = 0.0;
  for (int k = 0; k < n; ++k) {
    ch[k] = exp(ch[k] - mx);
    sum += ch[k];
  }
  for (int k = 0; k < n; ++k) ch[k] /= sum;
  return best + 1;
}

// Straight-through gradient of the log weights of one draw: with g_j the
// loss's sensitivity to the one-hot's component j, adds
// c_j (g_j - <c, g>) / tau to acc[j] (the relaxed one-hot's Jacobian).
__device__ __forceinline__ void st_categorical(const double* c, const double* g, int n, double tau, double* acc) {
  double m = 0.0;
  for (int j = 0; j < n; ++j) m += c[j] * g[j];
  for (int j = 0; j < n; ++j) {
    const double v = c[j] * (g[j] - m) / tau;
    if (v != 0.0) atomicAdd(&acc[j], v);
  }
}

// Sensitivities of the loss to the E and I one-hots of an exposure on day d
// with drawn lengths aS, bS: pre[k] = sum of the rate-adjoint ring over the
// k days after d (k = 0..W), DR(x) = m Dbar of day d + x (0 past the run).
// An E length a puts E on days 1..a, I on a+1..a+bS and the removal on a+bS;
// an I length b puts I on aS+1..aS+b and the removal on aS+b.
template <class DRF>
__device__ __forceinline__ void dwell_sensitivities(const DParams& P, const double* pre, int aS, int bS, DRF DR,
                                                    double* gE, double* gI) {
  for (int a = 1; a <= P.tau_E; ++a)
    gE[a - 1] = P.TE * pre[a] + P.TI * (pre[a + bS] - pre[a]) + DR(a + bS);
  for (int b = 1; b <= P.tau_I; ++b) gI[b - 1] = P.TI * (pre[aS + b] - pre[aS]) + DR(aS + b);
}

// exposure day held in a packed record (-1: none, or an initial infection)
__device__ __forceinline__ int rec_eday(uint32_t r) { return (int)(int16_t)(r >> 16); }

struct HardDay {
  uint32_t rec;     // next record
  uint32_t newst;   // next stage
  bool removed;     // I -> R or M today
  bool h;           // the day's hard draw
  bool was_s;       // susceptible at the start of the day
};

// DWELL = false compiles the fixed tau_E / tau_I only (callers that never
// take dwell tables)
template <bool DWELL = true>
__device__ __forceinline__ HardDay hard_agent_day(const DParams& P, Rng rng, uint32_t stream, int t, int set, int p,
                                                  uint32_t loc, int age, double A, uint32_t r, double* lam_out) {
  const double Rt = P.R[set * P.K + t], Sa = P.S[set * P.n_age + age], Zp = P.Z[p];
  const double lam = rate(Rt, Sa, A, Zp);
  if (lam_out) *lam_out = lam;
  HardDay o;
  o.h = false;
  if (lam > 0.0) {  // q = 0 rejects every uniform in (0, 1): no draw needed
    const double q = -expm1(-lam);
    const double u = unit_u(rng_block(rng, loc, (uint32_t)t, TAG_INFECT, (uint32_t)p, stream).x);
    o.h = u < q;
  }
  const uint32_t st = rec_stage(r);
  uint32_t tm = rec_timer(r);
  o.was_s = st == ST_S;
  o.removed = false;
  o.newst = st;
  o.rec = r;
  if (st == ST_E || st == ST_I) {
    tm -= 1;
    if (tm == 0) {
      if (st == ST_E) {
        o.newst = ST_I;
        tm = DWELL ? (uint32_t)dwell_I(P, rng, loc, (uint32_t)rec_eday(r), (uint32_t)p, stream) : (uint32_t)P.tau_I;
      } else {
        const double um = unit_u(rng_block(rng, loc, (uint32_t)t, TAG_MORT, (uint32_t)p, stream).x);
        o.newst = um < (double)P.m[set] ? ST_M : ST_R;
        o.removed = true;
      }
    }
    o.rec = (r & 0xFFFF0000u) | (tm << 8) | o.newst;
  } else if (st == ST_S && o.h) {
    o.newst = ST_E;
    o.rec = make_rec(ST_E, DWELL ? (uint32_t)dwell_E(P, rng, loc, (uint32_t)t, (uint32_t)p, stream) : (uint32_t)P.tau_E,
                     t);
  }
  return o;
}

struct AdjOut {
  double Sbar;      // Sbar^d
  double g;         // g^d
  double lam_bar;
};

// One agent's adjoint of day d.  sE/sI: sums of inf_bar over the E and I
// windows after day d; Sv, h: susceptible indicator and draw of day d (hard
// values, or the relaxed ones in SOFT mode with `soft` set).  dy/dlambda is
// evaluated only when it can matter (S^d != 0 and A > 0), in single precision
// when LOWP is set (float-state runs; gradients only).
template <bool LOWP = false>
__device__ __forceinline__ AdjOut agent_adjoint(const DParams& P, Rng rng, uint32_t stream, int d, int set, int p,
                                                uint32_t loc, int age, double A, double Sv, double h, bool soft,
                                                double sE, double sI, double Sbar1, double drm_bar) {
  const double xi_bar = drm_bar + P.TI * sI + P.TE * sE - Sbar1;
  const float* Rp = P.R + set * P.K + d;
  const float* Sp = P.S + set * P.n_age + age;
  double dydl = 0.0;
  AdjOut o;
  if (LOWP) {  // rate, derivative and g in single precision (gradients only)
    const float rs_z = *Rp * *Sp / P.Z[p];
    if (soft || (Sv != 0.0 && A > 0.0)) {
      const double u = unit_u(rng_block(rng, loc, (uint32_t)d, TAG_INFECT, (uint32_t)p, stream).x);
      float yf, df;
      relaxed_sample_f(rs_z * (float)A, (float)u, (float)P.tau, yf, df);
      dydl = (double)df;
      if (soft) h = (double)yf;
    }
    o.Sbar = Sbar1 + h * xi_bar;
    o.lam_bar = Sv * xi_bar * dydl;
    o.g = (double)(rs_z * (float)o.lam_bar);
    return o;
  }
  const double Rt = *Rp, Sa = *Sp, Zp = P.Z[p];
  if (soft || (Sv != 0.0 && A > 0.0)) {
    const double lam = rate(Rt, Sa, A, Zp);
    const double u = unit_u(rng_block(rng, loc, (uint32_t)d, TAG_INFECT, (uint32_t)p, stream).x);
    const double q = -expm1(-lam);
    double y;
    relaxed_sample(lam, q, u, P.tau, y, dydl);
    if (soft) h = y;
  }
  o.Sbar = Sbar1 + h * xi_bar;
  o.lam_bar = Sv * xi_bar * dydl;
  o.g = Rt * Sa / Zp * o.lam_bar;
  return o;
}

}  // namespace gabm
