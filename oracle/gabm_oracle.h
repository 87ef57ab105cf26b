/*
 * FP64 reference ("oracle") for the differentiable agent-based epidemic
 * model of Chopra, Rodriguez et al., "Differentiable Agent-based
 * Epidemiology" (GradABM).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library;
 * it is not part of the product path.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code
 * with the GPU library: it has its own counter-based generator, its own
 * random-graph layer and its own arithmetic, all written from the paper
 * (Section 3.1, Eq. 1-3; Appendix A assumptions A1-A6; Appendix B) and from
 * the published Philox definition (Salmon, Moraes, Dror, Shaw, SC'11).
 *
 * It is a plain single-threaded loop over edges (in the order given) and
 * agents, in double precision.  Gradients are forward-mode tangents along
 * caller-given directions, so they are independent of the GPU's reverse
 * adjoint.
 *
 * Parity pins: see the test-suite.  Every function here is pinned except the
 * exact form of the per-contact rate, which the paper defers to an external
 * reference (Section 3.1, after Eq. 3): "parity unpinned" against the paper
 * for the constant Z; pinned internally by closed forms.  Partly unpinned:
 * the straight-through tangent along the I log weights of an exposure's
 * drawn lengths ("parity unpinned" on its own) shares its bilinear
 * window-tangent code with the relaxed mode, which finite differences pin;
 * the E weights of an exposure and the initial infections' I weights have
 * closed-form pins.
 */
#ifndef GABM_ORACLE_H
#define GABM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_S = 0, ORA_E = 1, ORA_I = 2, ORA_R = 3, ORA_M = 4 };
enum { ORA_TAG_INIT = 0, ORA_TAG_INFECT = 1, ORA_TAG_MORT = 2, ORA_TAG_ER = 3 };
/* dwell-time draws: uniform k of a draw is word k mod 4 of the block with tag
 * (base + k / 4), so an E draw uses tags 4-5 and an I draw tags 6-7 */
enum { ORA_TAG_DWELL_E = 4, ORA_TAG_DWELL_I = 6 };
enum { ORA_PLAIN = 0, ORA_HARD_ST = 1, ORA_SOFT = 2 };

typedef struct {
  int32_t n_agents;
  int32_t n_pops;
  const int32_t *pop_offsets; /* [n_pops+1], agents of population p are [off[p], off[p+1]) */
  int32_t pop_id_base;        /* population id used in the random counters for p = 0 */
  const uint8_t *age;         /* [n_agents], < n_age */
  int64_t n_edges;
  const int32_t *src, *dst;   /* directed contacts, both directions listed */
  const float *w;             /* [n_edges] contact weight */
  double er_mean_deg;         /* daily Erdos-Renyi layer, 0 = none */
  float er_weight;
  int32_t K, n_age, tau_E, tau_I, mode;
  const float *R;             /* [K]  reproduction number per day */
  const float *S;             /* [n_age] age susceptibility */
  const float *T;             /* [5]  stage transmissibility S,E,I,R,M (only E, I may be non-zero) */
  float m, i0, tau_g;
  const float *Z;             /* [n_pops] rate normaliser */
  uint64_t seed;
  uint32_t stream;
  const double *target;       /* [K] daily deaths to fit, or NULL (loss 0) */
  int32_t ndir;               /* tangent directions (0 = none) */
  const double *dR;           /* [ndir*K] */
  const double *dS;           /* [ndir*n_age] */
  const double *dm;           /* [ndir] */
  const double *di0;          /* [ndir] */
  const float *iota;          /* [tau_E + tau_I] infectiousness profile over days since exposure, or NULL
                                 (flat): an agent exposed on day u contributes T[stage] * iota[t - u - 1]
                                 on day t; an initial infection counts as exposed on day -tau_E - 1 */
  /* agent-location layer (the GradABM-JUNE form, Section 6): agent a_v visits location l_v
   * with weight w_v; a location's pressure is P_l = sum of w_v * v_{a_v} over
   * its visits, and each visit adds w_v * (P_l - w_v * v_{a_v}) to its agent
   * (every other visitor, not the agent itself).  Each (agent, location) pair
   * at most once.  n_visits = 0: none. */
  int32_t n_locations;
  int64_t n_visits;
  const int32_t *visit_agent, *visit_loc;
  const float *visit_w;
  double *loc_p;              /* [n_locations] scratch, or NULL when n_visits = 0 */
  /* stochastic dwell times (stage transition times drawn from discrete
   * distributions, Section 3.1; more complex progression, Section 6): log
   * weights of the lengths 1..tau_E of E and 1..tau_I of I (tau_E, tau_I <= 8
   * are then the longest lengths), or NULL for the fixed tau_E / tau_I.  Each
   * exposure of agent i on day u has its lengths drawn by Gumbel-max with the
   * uniforms of (i, u); an initial infection's I length uses day 2^32 - 1.
   * With an infectiousness profile (of tau_E + tau_I days) the days since
   * exposure keep their meaning: an exposure k days back weighs iota[k-1],
   * an initial infection t + tau_E + 1 days back. */
  const float *dwell_E, *dwell_I;
  /* tangent directions of the dwell log weights, [ndir*tau_E] and
   * [ndir*tau_I], or NULL (zero).  The drawn lengths get the straight-through
   * Gumbel-softmax rule (Jang, Gu & Poole 2017): the forward keeps the drawn
   * one-hot c, the tangent is that of the relaxed one-hot
   * softmax((lw + G) / tau_g) with the same Gumbel noise G, and the window
   * weights are bilinear in (c_E, c_I).  In SOFT mode the relaxed one-hots
   * replace the drawn lengths in the forward as well (a mixture of windows). */
  const double *ddwE, *ddwI;
} ora_cfg;

typedef struct {
  double *counts;   /* [(K+1)*5] stage counts of snapshots 0..K */
  double *drm;      /* [K] removals (I -> R or M) on each day */
  double *deaths;   /* [K] m * drm */
  double *loss;     /* [1] */
  double *A;        /* [K*n_agents] weighted infectious contact sum, or NULL */
  double *lam;      /* [K*n_agents] aggregate rate, or NULL */
  double *y;        /* [K*n_agents] relaxed sample, or NULL (not in PLAIN) */
  uint8_t *h;       /* [K*n_agents] hard infection draw, or NULL */
  uint8_t *stage;   /* [(K+1)*n_agents] stage of each snapshot, or NULL */
  double *dL;       /* [ndir] */
  double *dD;       /* [ndir*K] */
  int64_t *mismatch; /* [1] hard mode: stage machine vs exposure-window form disagreements */
} ora_out;

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* the Gumbel-max draw of a length in 1..n from log weights lw[n] */
int32_t ora_dwell_draw(const float *lw, int32_t n, uint64_t seed, uint32_t idx, uint32_t day, uint32_t tag0,
                       uint32_t pop, uint32_t stream);
double ora_uniform(uint64_t seed, uint32_t idx, uint32_t day, uint32_t tag, uint32_t pop, uint32_t stream);
int64_t ora_er_pairs(int32_t n_pop, double mean_deg, uint64_t seed, uint32_t day, uint32_t pop,
                     uint32_t stream, int32_t *a, int32_t *b, int64_t cap);
/* returns 0 on success, a negative code on invalid input */
int ora_run(const ora_cfg *cfg, ora_out *out);

#ifdef __cplusplus
}
#endif
#endif
