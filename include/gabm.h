/*
 * gabm -- GPU library for the per-day transmission step of a differentiable
 * agent-based epidemic model (Chopra, Rodriguez et al., "Differentiable
 * Agent-based Epidemiology", GradABM), for AMD Instinct MI355X (gfx950).
 *
 * Model (Section 3.1 of the paper):
 *   Each agent j has an age group a_j, a disease stage d_j^t in {S,E,I,R,M}
 *   and a last-exposure day e_j^t.  Each day (assumption A1, Appendix A):
 *   Transmit (Eq. 2-3) for susceptible agents: the aggregate rate
 *     lambda_i^t = R^t * S[a_i] * A_i^t / Z_p,  A_i^t = sum_{j->i} w_ji * T[d_j^t]
 *   (the per-contact rate is linear in each factor; the sum is the
 *   permutation-invariant aggregation), the infection probability
 *   q = 1 - exp(-lambda) (Eq. 3), and a Bernoulli(q) draw, relaxed for
 *   gradients by a straight-through Gumbel-softmax (binary concrete) sample;
 *   Progress for exposed and infected agents: E -> I after tau_E days,
 *   I -> R or M after tau_I days, M with probability m;
 *   Aggregate: deaths = m * #{R, M}; daily deaths D^t = m * (removals on day t).
 *   The contact graph must be symmetric: every directed contact j->i with
 *   weight w has its reverse i->j with the same weight.
 *
 * Randomness: Philox4x32-10 (Salmon et al., SC'11) with key = (lo32(seed),
 * hi32(seed)) and counter (local agent index or pair index, day (0xFFFFFFFF
 * for the initial draw), tag | population << 8, stream); word 0 gives the
 * uniform (2*(x>>9)+1) * 2^-24.  Tags: 0 initial infection, 1 infection,
 * 2 mortality, 3 daily random contact layer.
 *
 * Conventions for every entry point:
 *   - return GABM_OK (0) or an error code; gabm_last_error() gives a
 *     thread-local message for the last failing call on this thread;
 *   - "device" pointers are HIP device memory the caller owns; "host"
 *     pointers are ordinary memory read before the call returns;
 *   - arguments are validated on the host before any launch; invalid input
 *     launches nothing;
 *   - `stream` is a hipStream_t (NULL = the default stream); work is queued
 *     asynchronously on it unless the entry point says it synchronises;
 *   - a handle must not be used from several host threads at once.
 */
#ifndef GABM_H
#define GABM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GABM_OK = 0,
  GABM_EINVAL = 1,       /* invalid argument */
  GABM_ENOMEM = 2,       /* device allocation failed */
  GABM_EHIP = 3,         /* a HIP runtime call failed */
  GABM_ENOTSYM = 4,      /* contact list is not symmetric */
  GABM_ERANGE = 5,       /* an index or size is out of range */
  GABM_EUNSUPPORTED = 6, /* valid but not supported by this library */
  GABM_ESTATE = 7        /* call order violated (e.g. backward before forward) */
} gabm_status;

enum { GABM_STAGE_S = 0, GABM_STAGE_E = 1, GABM_STAGE_I = 2, GABM_STAGE_R = 3, GABM_STAGE_M = 4 };
enum { GABM_TAG_INIT = 0, GABM_TAG_INFECT = 1, GABM_TAG_MORT = 2, GABM_TAG_ER = 3 };

/* Simulation modes.  PLAIN: hard forward only.  HARD_ST: hard forward,
 * straight-through gradients.  SOFT: relaxed forward (the sample y replaces
 * the hard draw everywhere), exact gradients of the relaxed model. */
enum { GABM_PLAIN = 0, GABM_HARD_ST = 1, GABM_SOFT = 2 };

/* Storage precision of per-agent real state and adjoints. */
enum { GABM_F32 = 0, GABM_F64 = 1 };

/* Graph build flags. */
enum { GABM_SYMMETRIZE = 1u, GABM_CHECK_SYMMETRIC = 2u };

/* Packed per-agent record of the hard state: bits 0-7 stage, 8-15 timer
 * (days left in E or I), 16-31 last exposure day as int16 (-1 = never, or
 * infected at t = 0). */
typedef uint32_t gabm_rec;

const char *gabm_last_error(void);
const char *gabm_version(void);

/* ------------------------------------------------------------------ graph */

typedef struct gabm_graph_s *gabm_graph;

typedef struct {
  int32_t n_agents;            /* N >= 1 */
  int32_t n_pops;              /* populations packed block-diagonally, >= 1 */
  const int32_t *pop_offsets;  /* host [n_pops+1]: 0 = off[0] < off[1] < ... < off[n_pops] = N */
  const uint8_t *age;          /* device [N], each < n_age */
  int32_t n_age;               /* 1..16 */
  int64_t n_edges;             /* directed contacts in src/dst/w, may be 0 */
  const int32_t *src;          /* device [n_edges] sender j */
  const int32_t *dst;          /* device [n_edges] receiver i */
  const float *w;              /* device [n_edges] weight >= 0, or NULL for all 1 */
  uint32_t flags;              /* GABM_SYMMETRIZE: input lists each undirected contact once, the
                                  reverse is added; GABM_CHECK_SYMMETRIC: verify the (possibly
                                  symmetrised) list, fail with GABM_ENOTSYM otherwise */
  float er_mean_deg;           /* daily Erdos-Renyi layer per population: round(N_p*mean/2)
                                  undirected pairs drawn each day; 0 = none */
  float er_weight;             /* weight of the daily layer's contacts */
  /* Agent-location layer (the GradABM-JUNE form, Section 6): visit v puts
   * agent visit_agent[v] at location visit_loc[v] with weight visit_w[v].
   * Location l's pressure is P_l = sum of w_v * x_{a_v} over its visits (x =
   * the visitor's infectiousness: T[stage] times the profile, or the relaxed
   * value); each visit adds w_v * (P_l - w_v * x_{a_v}) to its agent's
   * neighbour sum, so the agent meets every other visitor of l with weight
   * w_v * w_u and never itself.  This equals a static layer with
   * w_ij = sum over shared locations of w_il * w_jl, stored in O(visits)
   * instead of O(sum of squared location sizes).  Every visitor of a location
   * must belong to one population (GABM_ERANGE otherwise); an agent visits a
   * location at most once (GABM_EINVAL).  n_visits = 0: no such layer. */
  int32_t n_locations;         /* >= 0; location ids in [0, n_locations) */
  int32_t reserved1;
  int64_t n_visits;            /* >= 0 */
  const int32_t *visit_agent;  /* device [n_visits] */
  const int32_t *visit_loc;    /* device [n_visits] */
  const float *visit_w;        /* device [n_visits], finite and >= 0 */
} gabm_graph_desc;

/* Builds the destination-sorted CSR (rows = receivers, each row sorted by
 * sender then weight), the tile schedule of the transmission kernels and the
 * per-agent population table.  Copies everything it needs; the caller's
 * arrays may be freed afterwards.  Rejects self-contacts, contacts across
 * populations and out-of-range ids (GABM_ERANGE), negative or non-finite
 * weights (GABM_EINVAL), asymmetric lists under GABM_CHECK_SYMMETRIC
 * (GABM_ENOTSYM).  SYNCHRONISES with `stream` (the only such call besides
 * gabm_graph_info / gabm_graph_destroy).  The library owns the handle's
 * device memory until gabm_graph_destroy. */
gabm_status gabm_graph_build(const gabm_graph_desc *desc, void *stream, gabm_graph *out);

typedef struct {
  int32_t n_agents, n_pops, n_age;
  int64_t n_edges;       /* directed contacts stored (static layers) */
  int32_t max_degree;
  int32_t n_tiles;       /* transmission-kernel tiles */
  int32_t n_long_rows;   /* rows processed by a whole block */
  double weight_sum;     /* sum of stored weights */
  int64_t er_pairs_per_day; /* undirected daily pairs over all populations */
  int32_t n_sender_slices;  /* slices of 2^20 senders in the contact stream of the
                               single-simulation split kernels; 0 = not built
                               (no contacts, or 2^24 agents or more) */
  int32_t reserved0;
  int64_t n_stream_chunks;  /* 256-contact chunks of that stream */
  int32_t n_locations;      /* agent-location layer: locations and visits (0 = none) */
  int32_t reserved1;
  int64_t n_visits;
} gabm_graph_stats;

gabm_status gabm_graph_info(gabm_graph g, gabm_graph_stats *stats);

/* Device pointers to the CSR: row_ptr [N+1] (int64), col [E] senders,
 * w [E].  Owned by the handle. */
gabm_status gabm_graph_csr(gabm_graph g, const int64_t **row_ptr, const int32_t **col, const float **w);

gabm_status gabm_graph_destroy(gabm_graph g);

/* ------------------------------------------------------------- parameters */

/* Parameters of n_sets simulations that share the graph.  All arrays are
 * device float32 and are only read.  With per_pop_params, parameter set p
 * applies to population p (n_sets = n_pops). */
typedef struct {
  int32_t n_sets;
  int32_t K;           /* days */
  int32_t tau_E;       /* days exposed, >= 1 */
  int32_t tau_I;       /* days infectious, >= 1; tau_E + tau_I <= 64 */
  int32_t mode;        /* GABM_PLAIN / GABM_HARD_ST / GABM_SOFT */
  int32_t per_pop_params;
  const float *R;      /* device [n_sets*K] reproduction number per day */
  const float *S;      /* device [n_sets*n_age] susceptibility per age group */
  const float *m;      /* device [n_sets] mortality fraction */
  const float *i0;     /* device [n_sets] initially infected fraction */
  const float *Z;      /* device [n_pops] rate normaliser > 0 */
  float T[5];          /* host: transmissibility of stages S,E,I,R,M; only E, I may be non-zero */
  float tau_g;         /* Gumbel-softmax temperature in (0,1); used by HARD_ST and SOFT */
  const float *iota;   /* device [tau_E + tau_I] infectiousness profile over days since exposure
                          (Section 3.1: the per-contact rate depends on the source's time since
                          exposure), finite and >= 0, or NULL for a flat profile: an agent exposed
                          on day u contributes T[stage] * iota[t - u - 1] on day t; an initial
                          infection counts as exposed on day -tau_E - 1.  B = 1 only (batched runs:
                          GABM_EUNSUPPORTED); a simulation keeps the choice (profile or not) it was
                          created with. */
  const float *dwell_E; /* stochastic dwell times (Section 3.1: transition times drawn from discrete
                          distributions; Section 6: stochastic progression): device [tau_E] and
                          [tau_I] log weights of the E lengths 1..tau_E and the I lengths 1..tau_I
                          (-inf: never), or both NULL for fixed tau_E / tau_I.  Each exposure of an
                          agent on day u draws both lengths by Gumbel-max, argmax_k lw[k] -
                          log(-log u_k), with Philox uniforms of (agent, u) (an initial infection's
                          I length: day 2^32 - 1); tau_E, tau_I <= 8 (GABM_EINVAL otherwise).  With
                          a profile, days since exposure keep their meaning (iota has tau_E + tau_I
                          values).  Hard modes only, B = 1 (GABM_EUNSUPPORTED otherwise).  NaN
                          weights are undefined. */
  const float *dwell_I;
} gabm_params;

typedef struct {
  uint64_t seed;
  uint32_t replicate;  /* stream offset for single-step calls */
  uint32_t independent_sets; /* 0: sets of one replicate share random numbers (common random
                                numbers); 1: every simulation has its own stream */
} gabm_rng;

/* ------------------------------------------------------- single steps (a2-a9) */

/* Infectiousness formats for gabm_transmit_fwd. */
enum { GABM_INF_REC = 0,   /* gabm_rec[N]: T[stage] */
       GABM_INF_F32 = 1,   /* float[N] */
       GABM_INF_F64 = 2,   /* double[N] */
       GABM_INF_BIT1 = 3 }; /* uint64_t[ceil(N/64)]: bit (c & 63) of word c >> 6 set when agent c is
                               infectious; value T[I] for a set bit, 0 otherwise (one bit cannot tell
                               exposed agents apart, so T[E] is not applied) */

/* Transmit (Eq. 3 argument): A_i = sum over the static contacts j->i of
 * w * inf_j, plus the day's random layer (when the graph has one), and
 * lambda_i = R^day * S[a_i] * A_i / Z_p for parameter set `set`.  Sums are
 * formed in double precision.  A, lambda: device double[N] (lambda may be
 * NULL).  With an agent-location layer its two-hop sums are added too; their
 * pressures use scratch memory owned by the graph, so such calls on one graph
 * must not overlap (nor overlap gabm_transmit_bwd on it). */
gabm_status gabm_transmit_fwd(gabm_graph g, const void *inf, int32_t inf_fmt, const gabm_params *p, int32_t set,
                              const gabm_rng *rng, int32_t day, double *A, double *lambda, void *stream);

/* Bernoulli draw of every agent from its rate (Eq. 3): q = 1 - exp(-lambda),
 * u the day's infection uniform, hard h = [u < q], relaxed
 * y = sigmoid((logit q + log((1-u)/u)) / tau_g) and dy/dlambda.  lambda is
 * device double[N]; outputs device h uint8[N], y and dydl double[N] (y and
 * dydl may be NULL). */
gabm_status gabm_sample_infect(gabm_graph g, const double *lambda, const gabm_params *p, const gabm_rng *rng,
                               int32_t day, uint8_t *h, double *y, double *dydl, void *stream);

/* Progress (hard): E and I timers count down; E -> I, I -> R or M (mortality
 * uniform < m of set `set`); susceptible agents with h = 1 become E.  Writes
 * rec_out and adds, to counts (device double[6]), the stage counts of the new
 * snapshot S,E,I,R,M and the day's removals. */
gabm_status gabm_progress_stages(gabm_graph g, const gabm_rec *rec_in, const uint8_t *h, const gabm_params *p,
                                 int32_t set, const gabm_rng *rng, int32_t day, gabm_rec *rec_out, double *counts,
                                 void *stream);

/* Backward of the neighbour sum (adjoint of gabm_transmit_fwd with respect
 * to inf): infbar_j = sum_{i in N(j)} w_ij * g_i, a gather over the same CSR
 * (valid because the contact graph is symmetric), plus the day's random
 * layer and the agent-location layer (symmetric as well; same scratch rule
 * as gabm_transmit_fwd).  g, infbar: device double[N]. */
gabm_status gabm_transmit_bwd(gabm_graph g, const double *gvec, const gabm_rng *rng, int32_t day, double *infbar,
                              void *stream);

/* Parameter gradients of one day from the rate adjoint lambda_bar:
 * dR[0] += sum_i lambda_bar_i S[a_i] A_i / Z_p,
 * dS[a] += sum_{i: a_i = a} lambda_bar_i R^day A_i / Z_p.  Inputs device
 * double[N]; dR device double[1], dS device double[n_age] (accumulated). */
gabm_status gabm_param_grad_reduce(gabm_graph g, const double *lambda_bar, const double *A, const gabm_params *p,
                                   int32_t set, int32_t day, double *dR, double *dS, void *stream);

/* The day's random contact pairs (a_k, b_k) of population `pop` in agent ids
 * (global), k < round(N_p*mean/2).  Device int32 outputs of capacity `cap`;
 * *count (host) receives the number of pairs.  Synchronises. */
gabm_status gabm_er_daily(gabm_graph g, int32_t pop, const gabm_rng *rng, int32_t day, int32_t *a, int32_t *b,
                          int64_t cap, int64_t *count, void *stream);

/* ------------------------------------------------------------- whole runs */

typedef struct gabm_sim_s *gabm_sim;

typedef struct {
  int32_t n_reps;      /* replicates per parameter set; B = n_sets * n_reps simulations
                          (B = n_reps with per-population parameters) */
  int32_t ckpt_every;  /* keep per-day values for the backward only inside segments of this
                          many days, recomputing each segment from a state snapshot; 0 = keep all */
  int32_t precision;   /* GABM_F32 or GABM_F64 storage */
  int32_t use_hip_graph; /* capture each forward segment / backward day loop in a hipGraph */
  int32_t schedule;    /* 0: choose per simulation (B = 1: persistent LDS-mask kernels when
                          eligible: float state, hard or straight-through mode, T_E = 0, fewer
                          than 2^24 agents (one LDS mask per slice of 2^20 senders), one
                          parameter set or one per packed population; B > 32: one wave per
                          tile with 64-contact windows);
                          1: receiver-tile kernels (B = 1) / lane-group kernels (B > 1) only;
                          any other value: GABM_EINVAL.
                          gabm_autotune picks between them by measurement. */
  int32_t time_kernels; /* k > 0: record HIP events around every k-th launch of each class of day
                           kernel (eager launches only; see gabm_sim_kernel_times); 0: off */
} gabm_run_desc;

/* Creates a simulation object on a built graph for the given parameter
 * layout (n_sets, K, tau_E, tau_I, mode, per_pop_params of `p`; pointers in
 * `p` are not kept).  Allocates its device workspace (gabm_sim_workspace_size
 * bytes) with hipMalloc.  A graph with an agent-location layer takes B = 1
 * (GABM_EUNSUPPORTED for batched runs); the layer adds two launches per day
 * in each direction (location pressures, then the per-agent sums). */
gabm_status gabm_sim_create(gabm_graph g, const gabm_params *p, const gabm_run_desc *run, gabm_sim *out);
gabm_status gabm_sim_workspace_size(gabm_graph g, const gabm_params *p, const gabm_run_desc *run, size_t *bytes);

typedef struct {
  double *counts;  /* device [B*(K+1)*5] stage counts per snapshot (S,E,I,R,M) */
  double *drm;     /* device [B*K] removals per day */
  double *deaths;  /* device [B*K] m * removals */
  double *loss;    /* device [B] mean over days of (deaths - target)^2 */
} gabm_fwd_out;

/* Runs K days forward for all B simulations.  target: device double [B*K]
 * (or [K], broadcast, when target_stride = 0), or NULL for loss = 0.  Keeps
 * what the backward needs (per checkpoint settings).  Asynchronous. */
gabm_status gabm_sim_forward(gabm_sim s, const gabm_params *p, const gabm_rng *rng, const double *target,
                             int32_t target_stride, const gabm_fwd_out *out, void *stream);

typedef struct {
  double *dR;   /* device [n_sets*K] dL/dR^t */
  double *dS;   /* device [n_sets*n_age] */
  double *dm;   /* device [n_sets] */
  double *di0;  /* device [n_sets] */
  double *ddwell_E; /* device [tau_E] straight-through gradient with respect to the dwell log weights
                       of the E lengths (Gumbel-softmax rule: the drawn one-hot forward, the tangent of
                       softmax((lw + G) / tau_g) with the same noise G, Section 3.1), summed over every
                       exposure; simulations created with dwell tables in HARD_ST mode; NULL: skip */
  double *ddwell_I; /* device [tau_I] the same for the I lengths (exposures and initial infections) */
} gabm_grads;

/* Reverse pass of the last gabm_sim_forward (same p and rng): gradients of
 * sum_o loss_weight[o] * loss_o + sum_{o,t} deaths_bar[o*K+t] * deaths_o^t with
 * respect to R, S, m and i0 -- straight-through (HARD_ST) or exact (SOFT) --
 * recomputing checkpoint segments from their snapshots.  loss_weight: device
 * double [n_out] or NULL (all 1); deaths_bar: device double [n_out*K] or
 * NULL (0).  n_out = B outputs (n_reps * n_pops with per-population
 * parameters).  Overwrites the outputs.  A backward consumes the forward run:
 * call gabm_sim_forward again before the next backward.  Asynchronous. */
gabm_status gabm_sim_backward(gabm_sim s, const gabm_params *p, const gabm_rng *rng, const double *loss_weight,
                              const double *deaths_bar, const gabm_grads *out, void *stream);

/* One fused forward day (Transmit + draw + Progress + aggregates) and one
 * fused reverse day: the building blocks gabm_sim_forward and
 * gabm_sim_backward launch, exposed for custom drivers.
 * gabm_day_fwd: `day` must be the next day of the run (0 starts a new run
 * with the initial draw); per-day values for the reverse pass are kept only
 * when the simulation keeps every day (ckpt_every = 0); `target` and `out`
 * are used when `day` = K-1, which closes the run as gabm_sim_forward does.
 * gabm_day_bwd: reverse step `day` = K, K-1, ..., 0 in that order after a
 * closed forward run of a simulation that keeps every day; step d gathers
 * the rate adjoint of day d (d < K) and applies the agent adjoint of day d-1
 * (d > 0) or of the initial infections (d = 0); `out` is written at d = 0;
 * the objective is the sum of the run's losses.
 * Out-of-order calls fail with GABM_ESTATE. */
gabm_status gabm_day_fwd(gabm_sim s, const gabm_params *p, const gabm_rng *rng, int32_t day, const double *target,
                         int32_t target_stride, const gabm_fwd_out *out, void *stream);
gabm_status gabm_day_bwd(gabm_sim s, const gabm_params *p, const gabm_rng *rng, int32_t day, const gabm_grads *out,
                         void *stream);

/* Device pointers to the simulation's current hard records (gabm_rec[B*N],
 * agent-major: record of simulation b of agent i at i*B + b), for tests. */
gabm_status gabm_sim_records(gabm_sim s, const gabm_rec **rec);

/* Durations of the day kernels launched since the last reset, per kernel
 * class, from a pair of HIP events recorded around the sampled launches (every
 * time_kernels-th launch of each class, counted from the last reset) on their
 * launch stream, when the simulation was created with time_kernels > 0 and
 * use_hip_graph = 0.  ms and launches cover the timed launches only, so
 * ms / launches is the mean duration of a launch.  Synchronises with the
 * recorded events.  reset != 0 clears the record.  Classes:
 *   GABM_KT_GATHER_FWD  persistent neighbour sum of the forward day
 *   GABM_KT_AGENT_FWD   per-agent forward day (draw, progress, masks, counts)
 *   GABM_KT_DAY_FWD     fused tiled forward day (when the split path is not used)
 *   GABM_KT_GATHER_BWD  persistent neighbour sum of the reverse step
 *   GABM_KT_AGENT_BWD   per-agent reverse step (window ring, adjoint, grads)
 *   GABM_KT_DAY_BWD     fused tiled reverse step
 *   GABM_KT_ER          daily random layer (forward or reverse)
 *   GABM_KT_LOC         agent-location layer (pressures and per-agent sums) */
enum {
  GABM_KT_GATHER_FWD = 0,
  GABM_KT_AGENT_FWD = 1,
  GABM_KT_DAY_FWD = 2,
  GABM_KT_GATHER_BWD = 3,
  GABM_KT_AGENT_BWD = 4,
  GABM_KT_DAY_BWD = 5,
  GABM_KT_ER = 6,
  GABM_KT_LOC = 7,
  GABM_KT_N = 8
};
typedef struct {
  double ms[GABM_KT_N];        /* total duration per class */
  int64_t launches[GABM_KT_N]; /* launches per class */
} gabm_kernel_times;

gabm_status gabm_sim_kernel_times(gabm_sim s, gabm_kernel_times *out, int32_t reset);

/* Autotuner for the kernel schedule (gabm_run_desc.schedule): for every
 * schedule of the library (GABM_N_SCHEDULES), creates a temporary simulation
 * of the run (p, run) with that schedule, times `days` forward days of it on
 * `stream` (HIP events, after a warm-up day), and returns in *best a copy of
 * *run with the fastest schedule.  ms_per_day (host, GABM_N_SCHEDULES
 * entries, may be NULL) receives the measured times.  Allocates and frees
 * the temporary workspaces (hipMalloc); synchronises with `stream`.  days
 * must be in [1, K].  The parameters in p are only read. */
#define GABM_N_SCHEDULES 2
gabm_status gabm_autotune(gabm_graph g, const gabm_params *p, const gabm_run_desc *run, const gabm_rng *rng,
                          int32_t days, gabm_run_desc *best, double *ms_per_day, void *stream);

gabm_status gabm_sim_destroy(gabm_sim s);

#ifdef __cplusplus
}
#endif
#endif
