/*
 * FP64 oracle for the GradABM per-day transmission step.
 * TEST INFRASTRUCTURE ONLY -- see gabm_oracle.h.
 *
 * Model (Section 3.1):
 *   agent state X_j^t = {age a_j, stage d_j^t in {S,E,I,R,M}, last exposure e_j^t};
 *   Update (Eq. 1-2): Transmit for S agents, Progress for E and I agents;
 *   Transmit (Eq. 3): q = 1 - exp(-lambda_A), lambda_A the sum over contacts of a
 *   per-contact rate linear in R^t, the susceptibility S_a of the receiver and the
 *   transmissibility T_s of the sender's stage; infection ~ Bernoulli(q),
 *   relaxed with a Gumbel-softmax (binary concrete) sample for gradients;
 *   Progress: fixed transition times E->I after tau_E days, I->{R,M} after
 *   tau_I days, M with probability m;
 *   Aggregate: deaths = m * #{R,M}; loss = mean squared error of daily deaths.
 * Assumptions A1-A6 (Appendix A): one-day steps, no transmission on the day of
 * exposure, no reinfection, contacts accumulate within a day, not across days.
 *
 * Readings where the paper is silent (listed with the design notes):
 *   lambda_i = R^t * S[a_i] * A_i / Z_p  with  A_i = sum_{j->i} w_ji * T[d_j],
 *     evaluated as ((R*S)*A)/Z;
 *   initial infections: Bernoulli(i0) per agent, entering I with a full timer;
 *   the hard decision is u < q; the relaxed sample is
 *     y = sigmoid((logit q + log((1-u)/u)) / tau_g)  (same uniform u);
 *   the straight-through gradient uses dy/dlambda of that sample;
 *   the differentiable carrier through the fixed timers is the exposure
 *   history xi (multilinear form), xi_i^t = S_i^t h_i^t, S^{t+1} = S^t - xi^t;
 *   daily deaths D^t = m * (removals on day t).
 */
#include "gabm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------- Philox4x32-10 (Salmon et al., SC'11) ---------------- */

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u; /* Weyl key schedule */
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(uint64_t seed, uint32_t idx, uint32_t day, uint32_t tag, uint32_t pop, uint32_t stream,
                 uint32_t out[4]) {
  uint32_t ctr[4] = {idx, day, tag | (pop << 8), stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  ora_philox4x32_10(ctr, key, out);
}

/* uniform on (0,1): (2k+1) / 2^24 with k the top 23 bits of word 0 */
static double to_unit(uint32_t x) { return (double)(2u * (x >> 9) + 1u) * (1.0 / 16777216.0); }

double ora_uniform(uint64_t seed, uint32_t idx, uint32_t day, uint32_t tag, uint32_t pop, uint32_t stream) {
  uint32_t o[4];
  draw(seed, idx, day, tag, pop, stream, o);
  return to_unit(o[0]);
}

/* Gumbel-max (Gumbel 1954; the sampling view of Jang, Gu & Poole 2017): the
 * index maximising lw[k] + G_k with G_k = -log(-log u_k) is distributed as
 * softmax(lw); the first maximum wins a tie. */
int32_t ora_dwell_draw(const float *lw, int32_t n, uint64_t seed, uint32_t idx, uint32_t day, uint32_t tag0,
                       uint32_t pop, uint32_t stream) {
  uint32_t o[4];
  int32_t best = 0;
  double bv = -INFINITY;
  for (int32_t k = 0; k < n; ++k) {
    if (k % 4 == 0) draw(seed, idx, day, tag0 + (uint32_t)(k / 4), pop, stream, o);
    double v = (double)lw[k] - log(-log(to_unit(o[k % 4])));
    if (v > bv) {
      bv = v;
      best = k;
    }
  }
  return best + 1;
}

/* The relaxed one-hot of the same draw: ch = softmax((lw + G) / tau). */
static void dwell_relaxed(const float *lw, int32_t n, double tau, uint64_t seed, uint32_t idx, uint32_t day,
                          uint32_t tag0, uint32_t pop, uint32_t stream, double *ch) {
  uint32_t o[4];
  double mx = -INFINITY, sum = 0.0;
  for (int32_t k = 0; k < n; ++k) {
    if (k % 4 == 0) draw(seed, idx, day, tag0 + (uint32_t)(k / 4), pop, stream, o);
    ch[k] = ((double)lw[k] - log(-log(to_unit(o[k % 4])))) / tau;
    if (ch[k] > mx) mx = ch[k];
  }
  for (int32_t k = 0; k < n; ++k) {
    ch[k] = exp(ch[k] - mx);
    sum += ch[k];
  }
  for (int32_t k = 0; k < n; ++k) ch[k] /= sum;
}

/* Weights of an exposure k days back of being E, being I, and leaving I on
 * that day, for length weights cE over 1..tE and cI over 1..tI (one-hots of
 * drawn lengths, relaxed one-hots, or their tangents): E while k <= a; I
 * while a < k <= a + b; leaving on k = a + b. */
static void win_w(const double *cE, int32_t tE, const double *cI, int32_t tI, int32_t k, double *wE, double *wI,
                  double *wR) {
  double e = 0.0, i = 0.0, r = 0.0;
  for (int32_t a = 1; a <= tE; ++a) {
    double ca = cE[a - 1];
    if (ca == 0.0) continue;
    if (k <= a) {
      e += ca;
      continue;
    }
    int32_t m = k - a; /* the k-th day is day m of I */
    if (m > tI) continue;
    double tail = 0.0;
    for (int32_t b = m; b <= tI; ++b) tail += cI[b - 1];
    i += ca * tail;
    r += ca * cI[m - 1];
  }
  *wE = e;
  *wI = i;
  *wR = r;
}

/* dc = c * (dlw - <c, dlw>) / tau, the tangent of a relaxed one-hot */
static void relaxed_tangent(const double *c, const double *dlw, int32_t n, double tau, double *dc) {
  double m = 0.0;
  for (int32_t k = 0; k < n; ++k) m += c[k] * dlw[k];
  for (int32_t k = 0; k < n; ++k) dc[k] = c[k] * (dlw[k] - m) / tau;
}

/* Daily random-contact layer: G(n, M) with M = round(n*mean/2) undirected
 * pairs, endpoints from words 0 and 1 by exact 32x32->64 multiplication. */
int64_t ora_er_pairs(int32_t n_pop, double mean_deg, uint64_t seed, uint32_t day, uint32_t pop,
                     uint32_t stream, int32_t *a, int32_t *b, int64_t cap) {
  if (n_pop < 2 || mean_deg <= 0.0) return 0;
  int64_t M = llround((double)n_pop * mean_deg / 2.0);
  for (int64_t k = 0; k < M; ++k) {
    uint32_t o[4];
    draw(seed, (uint32_t)k, day, ORA_TAG_ER, pop, stream, o);
    uint32_t i = (uint32_t)(((uint64_t)o[0] * (uint64_t)(uint32_t)n_pop) >> 32);
    uint32_t jp = (uint32_t)(((uint64_t)o[1] * (uint64_t)(uint32_t)(n_pop - 1)) >> 32);
    uint32_t j = jp + (jp >= i ? 1u : 0u);
    if (k < cap) {
      a[k] = (int32_t)i;
      b[k] = (int32_t)j;
    }
  }
  return M;
}

/* ---------------- relaxed Bernoulli (binary concrete) ---------------- */

static double sigmoid(double z) {
  if (z >= 0) return 1.0 / (1.0 + exp(-z));
  double e = exp(z);
  return e / (1.0 + e);
}
static double log_sigmoid(double z) { return z >= 0 ? -log1p(exp(-z)) : z - log1p(exp(z)); }
/* logistic noise log((1-u)/u): the difference of two Gumbel(0,1) variates */
static double logistic_noise(double u) { return log1p(-u) - log(u); }

/* y = sigmoid((logit q + noise)/tau) and dy/dlambda, with q = 1 - exp(-lambda),
 * so dq/dlambda = 1 - q and dy/dlambda = y (1-y) / (tau q).  lambda = 0 gives
 * y = 0 and derivative 0 (the limit for tau < 1). */
static void relaxed(double lam, double q, double u, double tau, double *y, double *dydl) {
  if (!(q > 0.0)) {
    *y = 0.0;
    *dydl = 0.0;
    return;
  }
  double logit_q = log(q) + lam; /* log q - log(1-q), with log(1-q) = -lambda */
  double z = (logit_q + logistic_noise(u)) / tau;
  *y = sigmoid(z);
  *dydl = exp(log_sigmoid(z) - log(q)) * sigmoid(-z) / tau;
}

/* ---------------- simulation ---------------- */

typedef struct {
  int32_t n, W, ndir;
  double *xi;   /* [W*n] exposure history ring: xi^{t-1}..xi^{t-W} at slot u mod W */
  double *dxi;  /* [ndir*W*n] */
  double *Sv;   /* [n] susceptible indicator (relaxed in SOFT) */
  double *dSv;  /* [ndir*n] */
  double *x0;   /* [n] initial infection (hard or relaxed) */
  double *dx0;  /* [ndir*n] */
  double *inf;  /* [n] */
  double *dinf; /* [ndir*n] */
  double *A;    /* [n] */
  double *dA;   /* [ndir*n] */
  uint8_t *stage, *timer;
  uint8_t *dE, *dI;  /* [W*n] dwell lengths of an exposure on day u, at slot u mod W */
  uint8_t *dI0;      /* [n] I length of an initial infection */
  double *cE, *cI;   /* [W*n*8] relaxed one-hots of each slot's draws (with relaxed dwell or dwell tangents) */
  double *cI0;       /* [n*8] the same for the initial infections' I length */
  int32_t *eday;     /* [n] exposure day of the hard state */
  int32_t *pop_of, *local;
  int32_t *er_a, *er_b;
} ws_t;

static void ws_free(ws_t *w) {
  free(w->xi); free(w->dxi); free(w->Sv); free(w->dSv); free(w->x0); free(w->dx0);
  free(w->inf); free(w->dinf); free(w->A); free(w->dA); free(w->stage); free(w->timer);
  free(w->dE); free(w->dI); free(w->dI0); free(w->eday); free(w->cE); free(w->cI); free(w->cI0);
  free(w->pop_of); free(w->local); free(w->er_a); free(w->er_b);
}

/* Tangent of the window weights of ring slot sl (k days back) along
 * direction d of the dwell log weights: bilinear in (c_E, c_I), with c the
 * relaxed one-hots (rel_fwd) or the one-hots of the drawn lengths. */
static void dwell_dw(const ws_t *ws, const ora_cfg *c, int rel_fwd, size_t sl, int32_t d, int32_t k, double tau,
                     double *dwE, double *dwI, double *dwR) {
  const int32_t tE = c->tau_E, tI = c->tau_I;
  double cE[8], cI[8], dcE[8], dcI[8], zE[8] = {0}, zI[8] = {0};
  for (int32_t a = 0; a < tE; ++a) cE[a] = rel_fwd ? ws->cE[sl * 8 + a] : (a + 1 == ws->dE[sl] ? 1.0 : 0.0);
  for (int32_t b = 0; b < tI; ++b) cI[b] = rel_fwd ? ws->cI[sl * 8 + b] : (b + 1 == ws->dI[sl] ? 1.0 : 0.0);
  relaxed_tangent(ws->cE + sl * 8, c->ddwE ? c->ddwE + (size_t)d * tE : zE, tE, tau, dcE);
  relaxed_tangent(ws->cI + sl * 8, c->ddwI ? c->ddwI + (size_t)d * tI : zI, tI, tau, dcI);
  double e1, i1, r1, e2, i2, r2;
  win_w(dcE, tE, cI, tI, k, &e1, &i1, &r1);
  win_w(cE, tE, dcI, tI, k, &e2, &i2, &r2);
  *dwE = e1;
  *dwI = i1 + i2;
  *dwR = r1 + r2;
}

/* the same for an initial infection on day t (only an I length): I weight and leaving weight */
static void init_dw(const ws_t *ws, const ora_cfg *c, int32_t j, int32_t d, int32_t t, double tau, double *dwI,
                    double *dwR) {
  const int32_t tI = c->tau_I;
  double dcI[8], zI[8] = {0};
  relaxed_tangent(ws->cI0 + (size_t)j * 8, c->ddwI ? c->ddwI + (size_t)d * tI : zI, tI, tau, dcI);
  double s = 0.0;
  for (int32_t b = t + 1; b <= tI; ++b) s += dcI[b - 1];
  *dwI = s;
  *dwR = (t + 1 <= tI && t >= 0) ? dcI[t] : 0.0;
}

/* accumulate A_i = sum over contacts j->i of w * v_j (static layers in the
 * given order, then the day's random pairs in both directions) */
static void contact_sum(const ora_cfg *c, const ws_t *ws, int32_t t, const double *v, double *A) {
  int32_t n = c->n_agents;
  for (int32_t i = 0; i < n; ++i) A[i] = 0.0;
  for (int64_t e = 0; e < c->n_edges; ++e) A[c->dst[e]] += (double)c->w[e] * v[c->src[e]];
  if (c->n_visits > 0) {
    /* the two-hop sum over locations, without the visitor itself */
    double *P = c->loc_p;
    for (int32_t l = 0; l < c->n_locations; ++l) P[l] = 0.0;
    for (int64_t k = 0; k < c->n_visits; ++k) P[c->visit_loc[k]] += (double)c->visit_w[k] * v[c->visit_agent[k]];
    for (int64_t k = 0; k < c->n_visits; ++k) {
      const double wv = (double)c->visit_w[k];
      const int32_t a = c->visit_agent[k];
      A[a] += wv * (P[c->visit_loc[k]] - wv * v[a]);
    }
  }
  if (c->er_mean_deg > 0.0) {
    double wer = (double)c->er_weight;
    for (int32_t p = 0; p < c->n_pops; ++p) {
      int32_t off = c->pop_offsets[p], np = c->pop_offsets[p + 1] - off;
      int64_t M = ora_er_pairs(np, c->er_mean_deg, c->seed, (uint32_t)t, (uint32_t)(c->pop_id_base + p),
                               c->stream, ws->er_a, ws->er_b, (int64_t)(np * c->er_mean_deg) + 16);
      for (int64_t k = 0; k < M; ++k) {
        int32_t i = off + ws->er_a[k], j = off + ws->er_b[k];
        A[i] += wer * v[j];
        A[j] += wer * v[i];
      }
    }
  }
}

int ora_run(const ora_cfg *c, ora_out *o) {
  const int32_t n = c->n_agents, K = c->K, tE = c->tau_E, tI = c->tau_I, W = c->tau_E + c->tau_I;
  const int32_t nd = c->ndir;
  const int mode = c->mode;
  const int relaxed_needed = mode != ORA_PLAIN;
  if (n <= 0 || K <= 0 || tE < 1 || tI < 1 || c->n_pops < 1) return -1;
  if (c->T[ORA_S] != 0.f || c->T[ORA_R] != 0.f || c->T[ORA_M] != 0.f) return -2;
  if (relaxed_needed && !(c->tau_g > 0.f && c->tau_g < 1.f)) return -3;
  if (relaxed_needed && !(c->i0 > 0.f && c->i0 < 1.f)) return -4;
  if (mode == ORA_PLAIN && nd > 0) return -5;
  if (c->pop_offsets[0] != 0 || c->pop_offsets[c->n_pops] != n) return -6;
  const int dwell = c->dwell_E != NULL || c->dwell_I != NULL;
  if (dwell && (!c->dwell_E || !c->dwell_I || tE > 8 || tI > 8)) return -8;
  /* dwell tangents; relaxed windows in the forward (SOFT); either needs the relaxed one-hots */
  const int ddw = dwell && nd > 0 && (c->ddwE || c->ddwI);
  const int rel_fwd = dwell && mode == ORA_SOFT;
  const int rel = ddw || rel_fwd;
  if ((c->ddwE || c->ddwI) && (!dwell || mode == ORA_PLAIN)) return -9;

  const double TE = c->T[ORA_E], TI = c->T[ORA_I];
  const double m = c->m, i0 = c->i0, tau = c->tau_g;
  /* weight of the k-th day after exposure (k = 1..W): the profile value, 1 when flat */
#define IOTA(k) (c->iota ? (double)c->iota[(k) - 1] : 1.0)
  /* E, I and leaving weights of ring slot sl, k days back: the relaxed
   * mixture in SOFT mode with dwell tables, else the drawn (or fixed) lengths */
#define SLOT_W(sl, k, eW, iW, rW)                                                           \
  do {                                                                                      \
    if (rel_fwd) {                                                                          \
      win_w(ws.cE + (sl) * 8, tE, ws.cI + (sl) * 8, tI, (k), &(eW), &(iW), &(rW));          \
    } else {                                                                                \
      int32_t a_ = ws.dE[sl], b_ = ws.dI[sl];                                               \
      eW = (k) <= a_ ? 1.0 : 0.0;                                                           \
      iW = ((k) > a_ && (k) <= a_ + b_) ? 1.0 : 0.0;                                        \
      rW = (k) == a_ + b_ ? 1.0 : 0.0;                                                      \
    }                                                                                       \
  } while (0)
  /* an initial infection on day tt: I weight and leaving weight */
#define INIT_W(j, tt, iW, rW)                                                               \
  do {                                                                                      \
    if (rel_fwd) {                                                                          \
      double s_ = 0.0;                                                                      \
      for (int32_t b_ = (tt) + 1; b_ <= tI; ++b_) s_ += ws.cI0[(size_t)(j) * 8 + b_ - 1];   \
      iW = s_;                                                                              \
      rW = ((tt) + 1 <= tI) ? ws.cI0[(size_t)(j) * 8 + (tt)] : 0.0;                         \
    } else {                                                                                \
      iW = (tt) < ws.dI0[j] ? 1.0 : 0.0;                                                    \
      rW = (tt) == ws.dI0[j] - 1 ? 1.0 : 0.0;                                               \
    }                                                                                       \
  } while (0)

  ws_t ws;
  memset(&ws, 0, sizeof ws);
  ws.n = n; ws.W = W; ws.ndir = nd;
  ws.xi = calloc((size_t)W * n, sizeof(double));
  ws.Sv = calloc(n, sizeof(double));
  ws.x0 = calloc(n, sizeof(double));
  ws.inf = calloc(n, sizeof(double));
  ws.A = calloc(n, sizeof(double));
  ws.stage = calloc(n, 1);
  ws.timer = calloc(n, 1);
  ws.dE = calloc((size_t)W * n, 1);
  ws.dI = calloc((size_t)W * n, 1);
  ws.dI0 = calloc(n, 1);
  ws.eday = calloc(n, sizeof(int32_t));
  if (rel) {
    ws.cE = calloc((size_t)W * n * 8, sizeof(double));
    ws.cI = calloc((size_t)W * n * 8, sizeof(double));
    ws.cI0 = calloc((size_t)n * 8, sizeof(double));
    if (!ws.cE || !ws.cI || !ws.cI0) {
      ws_free(&ws);
      return -7;
    }
  }
  ws.pop_of = calloc(n, sizeof(int32_t));
  ws.local = calloc(n, sizeof(int32_t));
  int64_t er_cap = 16;
  for (int32_t p = 0; p < c->n_pops; ++p) {
    int32_t np = c->pop_offsets[p + 1] - c->pop_offsets[p];
    int64_t cp = (int64_t)(np * c->er_mean_deg) + 16;
    if (cp > er_cap) er_cap = cp;
  }
  ws.er_a = calloc(er_cap, sizeof(int32_t));
  ws.er_b = calloc(er_cap, sizeof(int32_t));
  if (nd > 0) {
    ws.dxi = calloc((size_t)nd * W * n, sizeof(double));
    ws.dSv = calloc((size_t)nd * n, sizeof(double));
    ws.dx0 = calloc((size_t)nd * n, sizeof(double));
    ws.dinf = calloc((size_t)nd * n, sizeof(double));
    ws.dA = calloc((size_t)nd * n, sizeof(double));
  }
  if (!ws.xi || !ws.Sv || !ws.x0 || !ws.inf || !ws.A || !ws.stage || !ws.timer || !ws.pop_of || !ws.local ||
      !ws.dE || !ws.dI || !ws.dI0 || !ws.eday ||
      !ws.er_a || !ws.er_b || (nd > 0 && (!ws.dxi || !ws.dSv || !ws.dx0 || !ws.dinf || !ws.dA))) {
    ws_free(&ws);
    return -7;
  }
  for (int32_t p = 0; p < c->n_pops; ++p)
    for (int32_t i = c->pop_offsets[p]; i < c->pop_offsets[p + 1]; ++i) {
      ws.pop_of[i] = p;
      ws.local[i] = i - c->pop_offsets[p];
    }

  double x0sum = 0.0, *dx0sum = nd ? calloc(nd, sizeof(double)) : NULL;
  double *drm_dir = nd ? calloc(nd, sizeof(double)) : NULL;
  int64_t mismatch = 0;

  /* ---- initial infections (t = 0) ---- */
  for (int32_t i = 0; i < n; ++i) {
    uint32_t pid = (uint32_t)(c->pop_id_base + ws.pop_of[i]);
    double u = ora_uniform(c->seed, (uint32_t)ws.local[i], 0xFFFFFFFFu, ORA_TAG_INIT, pid, c->stream);
    int hard = u < i0;
    ws.dI0[i] = (uint8_t)(dwell ? ora_dwell_draw(c->dwell_I, tI, c->seed, (uint32_t)ws.local[i], 0xFFFFFFFFu,
                                                 ORA_TAG_DWELL_I, pid, c->stream)
                                : tI);
    if (rel)
      dwell_relaxed(c->dwell_I, tI, tau, c->seed, (uint32_t)ws.local[i], 0xFFFFFFFFu, ORA_TAG_DWELL_I, pid, c->stream,
                    ws.cI0 + (size_t)i * 8);
    ws.stage[i] = hard ? ORA_I : ORA_S;
    ws.timer[i] = hard ? ws.dI0[i] : 0;
    double y0 = 0.0, dy0 = 0.0;
    if (relaxed_needed) {
      double z = (log(i0) - log1p(-i0) + logistic_noise(u)) / tau;
      y0 = sigmoid(z);
      dy0 = y0 * sigmoid(-z) / (tau * i0 * (1.0 - i0));
    }
    ws.x0[i] = (mode == ORA_SOFT) ? y0 : (double)hard;
    ws.Sv[i] = 1.0 - ws.x0[i];
    x0sum += ws.x0[i];
    for (int32_t d = 0; d < nd; ++d) {
      double v = dy0 * c->di0[d];
      ws.dx0[(size_t)d * n + i] = v;
      ws.dSv[(size_t)d * n + i] = -v;
      dx0sum[d] += v;
    }
  }

  double loss = 0.0;
  if (nd) for (int32_t d = 0; d < nd; ++d) o->dL[d] = 0.0;

#define SNAPSHOT(tt)                                                                        \
  do {                                                                                      \
    double *cc = o->counts + (size_t)(tt) * 5;                                              \
    for (int s_ = 0; s_ < 5; ++s_) cc[s_] = 0.0;                                            \
    if (mode == ORA_SOFT) {                                                                 \
      double sS = 0, sE = 0, sI = 0;                                                        \
      for (int32_t i_ = 0; i_ < n; ++i_) {                                                  \
        sS += ws.Sv[i_];                                                                    \
        for (int32_t k_ = 1; k_ <= W; ++k_) {                                               \
          int32_t u_ = (tt) - k_;                                                           \
          if (u_ < 0) break;                                                                \
          size_t sl_ = (size_t)(u_ % W) * n + i_;                                           \
          double eW_, iW_, rW_;                                                             \
          SLOT_W(sl_, k_, eW_, iW_, rW_);                                                   \
          if (eW_ == 0.0 && iW_ == 0.0) continue;                                           \
          double xv = ws.xi[sl_];                                                           \
          sE += eW_ * xv;                                                                   \
          sI += iW_ * xv;                                                                   \
        }                                                                                   \
        double i0W_, r0W_;                                                                  \
        INIT_W(i_, (tt), i0W_, r0W_);                                                       \
        (void)r0W_;                                                                         \
        if (i0W_ != 0.0) sI += i0W_ * ws.x0[i_];                                            \
      }                                                                                     \
      double rm = (double)n - sS - sE - sI;                                                 \
      cc[ORA_S] = sS; cc[ORA_E] = sE; cc[ORA_I] = sI;                                       \
      cc[ORA_R] = (1.0 - m) * rm; cc[ORA_M] = m * rm;                                       \
    } else {                                                                                \
      for (int32_t i_ = 0; i_ < n; ++i_) cc[ws.stage[i_]] += 1.0;                           \
    }                                                                                       \
    if (o->stage) memcpy(o->stage + (size_t)(tt) * n, ws.stage, (size_t)n);                 \
  } while (0)

  SNAPSHOT(0);

  for (int32_t t = 0; t < K; ++t) {
    /* ---- infectiousness of each agent at the start of day t ---- */
    for (int32_t j = 0; j < n; ++j) {
      /* wE, wI: exposures still in the E / I window; pE, pI: the same weighted by the profile */
      double wE = 0.0, wI = 0.0, pE = 0.0, pI = 0.0;
      for (int32_t k = 1; k <= W; ++k) {
        int32_t u = t - k;
        if (u < 0) break;
        size_t sl = (size_t)(u % W) * n + j;
        double eW, iW, rW;
        SLOT_W(sl, k, eW, iW, rW);
        if (eW == 0.0 && iW == 0.0) continue; /* that exposure has left I */
        double xv = ws.xi[sl];
        wE += eW * xv;
        pE += IOTA(k) * (eW * xv);
        wI += iW * xv;
        pI += IOTA(k) * (iW * xv);
      }
      double i0W, r0W;
      INIT_W(j, t, i0W, r0W);
      if (i0W != 0.0) { wI += i0W * ws.x0[j]; pI += IOTA(t + tE + 1) * (i0W * ws.x0[j]); }
      double win = TE * wE + TI * wI;
      double pwin = TE * pE + TI * pI;
      if (mode == ORA_SOFT) {
        ws.inf[j] = pwin;
      } else {
        double st = (double)c->T[ws.stage[j]];
        /* hard: one exposure at most is in the window, so pwin = T[stage] * iota(k) */
        ws.inf[j] = c->iota ? pwin : st;
        if (st != win) ++mismatch;
      }
      for (int32_t d = 0; d < nd; ++d) {
        double dE = 0.0, dI = 0.0;
        const double *dx = ws.dxi + (size_t)d * W * n;
        for (int32_t k = 1; k <= W; ++k) {
          int32_t u = t - k;
          if (u < 0) break;
          size_t sl = (size_t)(u % W) * n + j;
          double eW, iW, rW;
          SLOT_W(sl, k, eW, iW, rW);
          if (eW != 0.0 || iW != 0.0) {
            double xv = IOTA(k) * dx[sl];
            dE += eW * xv;
            dI += iW * xv;
          }
          if (ddw && ws.xi[sl] != 0.0) { /* the windows' own tangent along the dwell log weights */
            double a, b, r;
            dwell_dw(&ws, c, rel_fwd, sl, d, k, tau, &a, &b, &r);
            dE += IOTA(k) * (a * ws.xi[sl]);
            dI += IOTA(k) * (b * ws.xi[sl]);
          }
        }
        if (i0W != 0.0) dI += IOTA(t + tE + 1) * (i0W * ws.dx0[(size_t)d * n + j]);
        if (ddw && ws.x0[j] != 0.0) {
          double a, r;
          init_dw(&ws, c, j, d, t, tau, &a, &r);
          if (a != 0.0) dI += IOTA(t + tE + 1) * (a * ws.x0[j]); /* zero once t >= tau_I */
        }
        ws.dinf[(size_t)d * n + j] = TE * dE + TI * dI;
      }
    }

    /* ---- Transmit: contact sums (Eq. 3 argument) ---- */
    contact_sum(c, &ws, t, ws.inf, ws.A);
    for (int32_t d = 0; d < nd; ++d) contact_sum(c, &ws, t, ws.dinf + (size_t)d * n, ws.dA + (size_t)d * n);

    /* removals on day t in the exposure-window form: exposures of day t-W and
     * the initial infections on day tau_I - 1 */
    double drm_w = 0.0;
    if (dwell) {
      /* the exposures of day u leave I on day u + dE + dI; initial infections on day dI0 - 1 */
      for (int32_t d = 0; d < nd; ++d) drm_dir[d] = 0.0;
      for (int32_t i = 0; i < n; ++i) {
        for (int32_t k = 1; k <= W && t - k >= 0; ++k) {
          size_t sl = (size_t)((t - k) % W) * n + i;
          double eW, iW, rW;
          SLOT_W(sl, k, eW, iW, rW);
          if (rW != 0.0) {
            drm_w += rW * ws.xi[sl];
            for (int32_t d = 0; d < nd; ++d) drm_dir[d] += rW * ws.dxi[(size_t)d * W * n + sl];
          }
          if (ddw && ws.xi[sl] != 0.0)
            for (int32_t d = 0; d < nd; ++d) {
              double a, b, r;
              dwell_dw(&ws, c, rel_fwd, sl, d, k, tau, &a, &b, &r);
              drm_dir[d] += r * ws.xi[sl];
            }
        }
        double i0W, r0W;
        INIT_W(i, t, i0W, r0W);
        if (r0W != 0.0) {
          drm_w += r0W * ws.x0[i];
          for (int32_t d = 0; d < nd; ++d) drm_dir[d] += r0W * ws.dx0[(size_t)d * n + i];
        }
        if (ddw && ws.x0[i] != 0.0)
          for (int32_t d = 0; d < nd; ++d) {
            double a, r;
            init_dw(&ws, c, i, d, t, tau, &a, &r);
            drm_dir[d] += r * ws.x0[i];
          }
      }
    } else {
      int32_t u = t - W;
      if (u >= 0)
        for (int32_t i = 0; i < n; ++i) drm_w += ws.xi[(size_t)(u % W) * n + i];
      if (t == tI - 1) drm_w += x0sum;
      for (int32_t d = 0; d < nd; ++d) {
        double s = 0.0;
        if (u >= 0)
          for (int32_t i = 0; i < n; ++i) s += ws.dxi[((size_t)d * W + (u % W)) * n + i];
        if (t == tI - 1) s += dx0sum[d];
        drm_dir[d] = s;
      }
    }

    const double Rt = c->R[t];
    int32_t drm_hard = 0;
    for (int32_t i = 0; i < n; ++i) {
      int32_t p = ws.pop_of[i];
      uint32_t pid = (uint32_t)(c->pop_id_base + p);
      double Sa = c->S[c->age[i]], Zp = c->Z[p];
      double A = ws.A[i];
      double lam = Rt * Sa * A / Zp;
      double q = -expm1(-lam);
      double u = ora_uniform(c->seed, (uint32_t)ws.local[i], (uint32_t)t, ORA_TAG_INFECT, pid, c->stream);
      int hard = u < q;
      double y = 0.0, dydl = 0.0;
      if (relaxed_needed) relaxed(lam, q, u, tau, &y, &dydl);
      double hv = (mode == ORA_SOFT) ? y : (double)hard;
      double Sv = ws.Sv[i];
      double xi = Sv * hv;
      size_t slot = (size_t)(t % W) * n + i;
      if (o->A) o->A[(size_t)t * n + i] = A;
      if (o->lam) o->lam[(size_t)t * n + i] = lam;
      if (o->y) o->y[(size_t)t * n + i] = y;
      if (o->h) o->h[(size_t)t * n + i] = (uint8_t)hard;
      for (int32_t d = 0; d < nd; ++d) {
        double dlam = c->dR[(size_t)d * K + t] * Sa * A / Zp + Rt * c->dS[(size_t)d * c->n_age + c->age[i]] * A / Zp +
                      Rt * Sa * ws.dA[(size_t)d * n + i] / Zp;
        double dh = dydl * dlam;
        double dS_ = ws.dSv[(size_t)d * n + i];
        double dxi = dS_ * hv + Sv * dh;
        ws.dSv[(size_t)d * n + i] = dS_ - dxi;
        ws.dxi[((size_t)d * W) * n + slot] = dxi;
      }
      ws.Sv[i] = Sv - xi;
      ws.xi[slot] = xi; /* overwrites xi^{t-W}, already used above */
      /* the lengths an exposure of agent i on day t takes; they only weigh
       * exposure mass or its tangents, so without either any value serves */
      const int draw_now = dwell && (xi != 0.0 || nd > 0);
      ws.dE[slot] = (uint8_t)(draw_now ? ora_dwell_draw(c->dwell_E, tE, c->seed, (uint32_t)ws.local[i], (uint32_t)t,
                                                       ORA_TAG_DWELL_E, pid, c->stream)
                                       : tE);
      ws.dI[slot] = (uint8_t)(draw_now ? ora_dwell_draw(c->dwell_I, tI, c->seed, (uint32_t)ws.local[i], (uint32_t)t,
                                                       ORA_TAG_DWELL_I, pid, c->stream)
                                       : tI);
      if (rel && draw_now) {
        dwell_relaxed(c->dwell_E, tE, tau, c->seed, (uint32_t)ws.local[i], (uint32_t)t, ORA_TAG_DWELL_E, pid,
                      c->stream, ws.cE + slot * 8);
        dwell_relaxed(c->dwell_I, tI, tau, c->seed, (uint32_t)ws.local[i], (uint32_t)t, ORA_TAG_DWELL_I, pid,
                      c->stream, ws.cI + slot * 8);
      }

      /* ---- Progress (hard stage machine) ---- */
      if (mode != ORA_SOFT) {
        uint8_t st = ws.stage[i];
        if (st == ORA_E || st == ORA_I) {
          ws.timer[i] -= 1;
          if (ws.timer[i] == 0) {
            if (st == ORA_E) {
              ws.stage[i] = ORA_I;
              ws.timer[i] = ws.dI[(size_t)(ws.eday[i] % W) * n + i];
            } else {
              double um = ora_uniform(c->seed, (uint32_t)ws.local[i], (uint32_t)t, ORA_TAG_MORT, pid, c->stream);
              ws.stage[i] = um < m ? ORA_M : ORA_R;
              ++drm_hard;
            }
          }
        } else if (st == ORA_S && hard) {
          ws.stage[i] = ORA_E;
          ws.timer[i] = ws.dE[slot];
          ws.eday[i] = t;
        }
      }
    }
    if (mode != ORA_SOFT && (double)drm_hard != drm_w) ++mismatch;

    /* ---- Aggregate: daily deaths and loss ---- */
    double D = m * drm_w;
    o->drm[t] = drm_w;
    o->deaths[t] = D;
    double r = c->target ? D - c->target[t] : 0.0;
    loss += r * r;
    for (int32_t d = 0; d < nd; ++d) {
      double dD = c->dm[d] * drm_w + m * drm_dir[d];
      o->dD[(size_t)d * K + t] = dD;
      o->dL[d] += 2.0 * r * dD / (double)K;
    }
    SNAPSHOT(t + 1);
  }
#undef SNAPSHOT
#undef SLOT_W
#undef INIT_W
#undef IOTA
  *o->loss = loss / (double)K;
  if (o->mismatch) *o->mismatch = mismatch;
  free(dx0sum);
  free(drm_dir);
  ws_free(&ws);
  return 0;
}
