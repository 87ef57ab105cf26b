// C ABI of the gabm library: argument validation, error reporting, graph and
// simulation handles, and the single-step entry points (each one step of the
// day, unfused, in double precision, for tests and custom pipelines).
#include <cmath>
#include <cstdio>
#include <string>

#include "agent.h"
#include "batched.h"
#include "day_kernels.h"
#include "loc.h"
#include "sim_internal.h"
#include "tile.h"

namespace gabm {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

gabm_status build_graph(const gabm_graph_desc* d, hipStream_t st, Graph& G);
gabm_status sim_workspace(const Graph& G, const gabm_params* p, const gabm_run_desc* run, size_t* bytes);
gabm_status sim_create(const Graph& G, const gabm_params* p, const gabm_run_desc* run, Sim& s);
gabm_status sim_forward(Sim& s, const DParams& P, const gabm_rng* r, const double* target, int stride,
                        const gabm_fwd_out* out, hipStream_t st);
gabm_status sim_backward(Sim& s, const DParams& P, const gabm_rng* r, const double* loss_weight,
                         const double* deaths_bar, const gabm_grads* out, hipStream_t st);
gabm_status sim_day_fwd(Sim& s, const DParams& P, const gabm_rng* r, int day, const double* target, int stride,
                        const gabm_fwd_out* out, hipStream_t st);
gabm_status sim_day_bwd(Sim& s, const DParams& P, const gabm_rng* r, int day, const gabm_grads* out, hipStream_t st);
int sim_n_out(const Sim& s);
gabm_status sim_kernel_times(Sim& s, gabm_kernel_times* out, int reset);

gabm_status check_params(const Graph& G, const gabm_params* p, DParams* out) {
  GABM_CHECK(p != nullptr, GABM_EINVAL, "params is NULL");
  GABM_CHECK(p->n_sets >= 1, GABM_EINVAL, "n_sets must be >= 1");
  GABM_CHECK(p->K >= 1 && p->K <= 32767, GABM_EINVAL, "K must be in [1, 32767]");
  GABM_CHECK(p->tau_E >= 1 && p->tau_I >= 1 && p->tau_E + p->tau_I <= 64 && p->tau_E < 256 && p->tau_I < 256,
             GABM_EINVAL, "tau_E, tau_I must be >= 1 with tau_E + tau_I <= 64");
  GABM_CHECK(p->mode == GABM_PLAIN || p->mode == GABM_HARD_ST || p->mode == GABM_SOFT, GABM_EINVAL, "unknown mode");
  GABM_CHECK(p->R && p->S && p->m && p->i0 && p->Z, GABM_EINVAL, "a parameter pointer is NULL");
  GABM_CHECK(!p->per_pop_params || p->n_sets == G.n_pops, GABM_EINVAL,
             "per-population parameters need n_sets == n_pops");
  GABM_CHECK(p->T[0] == 0.f && p->T[3] == 0.f && p->T[4] == 0.f, GABM_EUNSUPPORTED,
             "only exposed and infected agents may transmit (T[S] = T[R] = T[M] = 0)");
  GABM_CHECK(std::isfinite(p->T[1]) && std::isfinite(p->T[2]) && p->T[1] >= 0.f && p->T[2] >= 0.f, GABM_EINVAL,
             "transmissibility must be finite and >= 0");
  if (p->mode != GABM_PLAIN)
    GABM_CHECK(p->tau_g > 0.f && p->tau_g < 1.f, GABM_EINVAL, "tau_g must be in (0, 1) for differentiable modes");
  DParams& P = *out;
  P.R = p->R; P.S = p->S; P.m = p->m; P.i0 = p->i0; P.Z = p->Z;
  P.TE = p->T[1]; P.TI = p->T[2]; P.tau = p->tau_g;
  P.K = p->K; P.tau_E = p->tau_E; P.tau_I = p->tau_I; P.n_age = G.n_age; P.mode = p->mode;
  P.per_pop = p->per_pop_params ? 1 : 0; P.n_sets = p->n_sets;
  P.iota = p->iota;
  GABM_CHECK((p->dwell_E == nullptr) == (p->dwell_I == nullptr), GABM_EINVAL,
             "dwell_E and dwell_I are given together or not at all");
  if (p->dwell_E) {
    GABM_CHECK(p->tau_E <= 8 && p->tau_I <= 8, GABM_EINVAL, "dwell tables cover at most 8 days each");
    GABM_CHECK(p->mode != GABM_SOFT, GABM_EUNSUPPORTED, "dwell tables run in the hard modes (PLAIN, HARD_ST)");
  }
  P.dwell_E = p->dwell_E;
  P.dwell_I = p->dwell_I;
  return GABM_OK;
}

// ---------------------------------------------------------------- single-step kernels

struct StepInf {
  const void* v;
  int fmt;
  double TE, TI;
  // records only: the infectiousness profile (null = flat) and the day
  const float* iota = nullptr;
  int day = 0, tau_E = 0, W = 0;
  __device__ __forceinline__ double at(int c) const {
    if (fmt == GABM_INF_F32) return (double)((const float*)v)[c];
    if (fmt == GABM_INF_F64) return ((const double*)v)[c];
    if (fmt == GABM_INF_BIT1) return ((((const unsigned long long*)v)[c >> 6] >> (c & 63)) & 1ull) ? TI : 0.0;
    const uint32_t r = ((const uint32_t*)v)[c];
    const uint32_t st = rec_stage(r);
    const double T = st == ST_I ? TI : (st == ST_E ? TE : 0.0);
    if (!iota || T == 0.0) return T;
    const int k = days_since_exposure(r, day, tau_E);
    return T * (double)iota[(k < 1 ? 1 : (k > W ? W : k)) - 1];
  }
};

// the agent-location layer's two passes for one step, adding into `out`
// (pressures in the graph's scratch)
static void step_locations(const Graph& G, const StepInf& si, double* out, hipStream_t st);

__global__ void __launch_bounds__(kBlock) k_step_gather(DGraph G, StepInf inf, double* out) {
  __shared__ TileShared sh;
  auto ev = [&](int c, float w) -> double { return (double)w * inf.at(c); };
  auto epi = [&](int i, double A, bool active) {
    if (active) out[i] = A;
  };
  tile_pass(G, tile_bounds(G, blockIdx.x), sh, ev, epi);
}

__device__ __forceinline__ void er_pair_step(const DGraph& G, Rng rng, uint32_t stream, int t, int64_t k, int& gi,
                                             int& gj) {
  int lo = 0, hi = G.n_pops;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (G.er_off[mid] <= k) lo = mid; else hi = mid;
  }
  const uint32_t kk = (uint32_t)(k - G.er_off[lo]);
  const int off = G.pop_off[lo];
  const uint32_t np = (uint32_t)(G.pop_off[lo + 1] - off);
  const uint4 x = rng_block(rng, kk, (uint32_t)t, TAG_ER, (uint32_t)lo, stream);
  const uint32_t i = __umulhi(x.x, np);
  const uint32_t jp = __umulhi(x.y, np - 1u);
  gi = off + (int)i;
  gj = off + (int)(jp + (jp >= i ? 1u : 0u));
}

__global__ void k_step_er(DGraph G, Rng rng, uint32_t stream, int t, StepInf inf, double* acc) {
  const double w = G.er_w;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < G.er_total; k += (int64_t)gridDim.x * blockDim.x) {
    int i, j;
    er_pair_step(G, rng, stream, t, k, i, j);
    const double vi = inf.at(i), vj = inf.at(j);
    if (vj != 0.0) atomicAdd(&acc[i], w * vj);
    if (vi != 0.0) atomicAdd(&acc[j], w * vi);
  }
}

__global__ void k_step_rate(DGraph G, DParams P, int set, int t, const double* A, double* lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.N) return;
  const int p = pop_of_agent(G, i);
  const int s = P.per_pop ? p : set;
  lam[i] = rate(P.R[s * P.K + t], P.S[s * P.n_age + G.age[i]], A[i], P.Z[p]);
}

__global__ void k_step_sample(DGraph G, DParams P, Rng rng, uint32_t stream, int t, const double* lam, uint8_t* h,
                              double* y, double* dydl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.N) return;
  const int p = pop_of_agent(G, i);
  const uint32_t loc = (uint32_t)(i - G.pop_off[p]);
  const double l = lam[i];
  const double q = -expm1(-l);
  const double u = unit_u(rng_block(rng, loc, (uint32_t)t, TAG_INFECT, (uint32_t)p, stream).x);
  h[i] = u < q ? 1 : 0;
  if (y || dydl) {
    double yy, dd;
    relaxed_sample(l, q, u, P.tau, yy, dd);
    if (y) y[i] = yy;
    if (dydl) dydl[i] = dd;
  }
}

__global__ void k_step_progress(DGraph G, DParams P, int set, Rng rng, uint32_t stream, int t, const uint32_t* rin,
                                const uint8_t* h, uint32_t* rout, double* counts) {
  __shared__ double red[kBlock / kWave];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double c[6] = {0, 0, 0, 0, 0, 0};
  if (i < G.N) {
    const int p = pop_of_agent(G, i);
    const int s = P.per_pop ? p : set;
    const uint32_t loc = (uint32_t)(i - G.pop_off[p]);
    const uint32_t r = rin[i];
    const uint32_t st = rec_stage(r);
    uint32_t tm = rec_timer(r), ns = st, nr = r;
    if (st == ST_E || st == ST_I) {
      tm -= 1;
      if (tm == 0) {
        if (st == ST_E) {
          ns = ST_I;
          tm = (uint32_t)dwell_I(P, rng, loc, (uint32_t)rec_eday(r), (uint32_t)p, stream);
        } else {
          const double um = unit_u(rng_block(rng, loc, (uint32_t)t, TAG_MORT, (uint32_t)p, stream).x);
          ns = um < (double)P.m[s] ? ST_M : ST_R;
          c[5] = 1.0;
        }
      }
      nr = (r & 0xFFFF0000u) | (tm << 8) | ns;
    } else if (st == ST_S && h[i]) {
      ns = ST_E;
      nr = make_rec(ST_E, (uint32_t)dwell_E(P, rng, loc, (uint32_t)t, (uint32_t)p, stream), t);
    }
    rout[i] = nr;
    c[ns] = 1.0;
  }
  for (int k = 0; k < 6; ++k) {
    const double v = block_sum(c[k], red);
    if (threadIdx.x == 0 && v != 0.0) atomicAdd(&counts[k], v);
  }
}

__global__ void k_step_param(DGraph G, DParams P, int set, int t, const double* lam_bar, const double* A, double* dR,
                             double* dS) {
  __shared__ double red[kBlock / kWave];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double r = 0.0;
  double sa[16];
  for (int a = 0; a < 16; ++a) sa[a] = 0.0;
  if (i < G.N) {
    const int p = pop_of_agent(G, i);
    const int s = P.per_pop ? p : set;
    const double Rt = P.R[s * P.K + t], Sa = P.S[s * P.n_age + G.age[i]], Zp = P.Z[p];
    const double base = lam_bar[i] * A[i] / Zp;
    r = base * Sa;
    sa[G.age[i]] = base * Rt;
  }
  const double v = block_sum(r, red);
  if (threadIdx.x == 0 && v != 0.0) atomicAdd(dR, v);
  for (int a = 0; a < P.n_age; ++a) {
    const double x = block_sum(sa[a], red);
    if (threadIdx.x == 0 && x != 0.0) atomicAdd(&dS[a], x);
  }
}

static int nblk(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 1 << 20)); }

static Rng rng_of(const gabm_rng* r) {
  Rng g;
  g.k0 = (uint32_t)r->seed;
  g.k1 = (uint32_t)(r->seed >> 32);
  return g;
}

}  // namespace gabm

using namespace gabm;

#define TRY(expr)                      \
  do {                                 \
    try {                              \
      return (expr);                   \
    } catch (const std::exception& e) { \
      set_error(e.what());             \
      return GABM_ENOMEM;              \
    }                                  \
  } while (0)

extern "C" {

const char* gabm_last_error(void) { return g_err.c_str(); }
const char* gabm_version(void) { return "gabm 0.1 (gfx950)"; }

gabm_status gabm_graph_build(const gabm_graph_desc* d, void* stream, gabm_graph* out) {
  GABM_CHECK(d && out, GABM_EINVAL, "desc or out is NULL");
  *out = nullptr;
  GABM_CHECK(d->n_agents >= 1, GABM_EINVAL, "n_agents must be >= 1");
  GABM_CHECK(d->n_pops >= 1 && d->n_pops <= 65535, GABM_EINVAL, "n_pops must be in [1, 65535]");
  GABM_CHECK(d->pop_offsets != nullptr, GABM_EINVAL, "pop_offsets is NULL");
  GABM_CHECK(d->pop_offsets[0] == 0 && d->pop_offsets[d->n_pops] == d->n_agents, GABM_EINVAL,
             "pop_offsets must start at 0 and end at n_agents");
  for (int p = 0; p < d->n_pops; ++p)
    GABM_CHECK(d->pop_offsets[p + 1] > d->pop_offsets[p], GABM_EINVAL, "pop_offsets must be strictly increasing");
  GABM_CHECK(d->age != nullptr, GABM_EINVAL, "age is NULL");
  GABM_CHECK(d->n_age >= 1 && d->n_age <= 16, GABM_EINVAL, "n_age must be in [1, 16]");
  GABM_CHECK(d->n_edges >= 0, GABM_EINVAL, "n_edges must be >= 0");
  GABM_CHECK(d->n_edges == 0 || (d->src && d->dst), GABM_EINVAL, "src or dst is NULL");
  GABM_CHECK(std::isfinite(d->er_mean_deg) && d->er_mean_deg >= 0.f && std::isfinite(d->er_weight) &&
                 d->er_weight >= 0.f,
             GABM_EINVAL, "daily layer mean degree and weight must be finite and >= 0");
  GABM_CHECK(d->n_locations >= 0 && d->n_visits >= 0, GABM_EINVAL, "n_locations and n_visits must be >= 0");
  GABM_CHECK(d->n_visits == 0 || (d->visit_agent && d->visit_loc && d->visit_w), GABM_EINVAL,
             "visit_agent, visit_loc or visit_w is NULL");
  GABM_CHECK(d->n_visits < ((int64_t)1 << 31), GABM_ERANGE, "too many visits");
  const int64_t E = (d->flags & GABM_SYMMETRIZE) ? 2 * d->n_edges : d->n_edges;
  GABM_CHECK(E < ((int64_t)1 << 40), GABM_ERANGE, "too many contacts");
  gabm_graph h = new (std::nothrow) gabm_graph_s();
  GABM_CHECK(h != nullptr, GABM_ENOMEM, "host allocation failed");
  gabm_status rc = build_graph(d, (hipStream_t)stream, h->g);
  if (rc != GABM_OK) {
    h->g.release();
    delete h;
    return rc;
  }
  *out = h;
  return GABM_OK;
}

gabm_status gabm_graph_info(gabm_graph g, gabm_graph_stats* s) {
  GABM_CHECK(g && s, GABM_EINVAL, "graph or stats is NULL");
  const Graph& G = g->g;
  s->n_agents = G.N; s->n_pops = G.n_pops; s->n_age = G.n_age; s->n_edges = G.E; s->max_degree = G.max_degree;
  s->n_tiles = G.n_tiles; s->n_long_rows = G.n_long; s->weight_sum = G.weight_sum;
  s->er_pairs_per_day = G.er_off_h.back();
  s->n_sender_slices = G.n_slices;
  s->reserved0 = 0;
  s->n_stream_chunks = G.slice_chunk.empty() ? 0 : G.slice_chunk.back();
  s->n_locations = G.n_loc;
  s->reserved1 = 0;
  s->n_visits = G.n_visits;
  return GABM_OK;
}

gabm_status gabm_graph_csr(gabm_graph g, const int64_t** row_ptr, const int32_t** col, const float** w) {
  GABM_CHECK(g, GABM_EINVAL, "graph is NULL");
  if (row_ptr) *row_ptr = g->g.row_ptr;
  if (col) *col = g->g.col;
  if (w) *w = g->g.w;
  return GABM_OK;
}

gabm_status gabm_graph_destroy(gabm_graph g) {
  if (!g) return GABM_OK;
  g->g.release();
  delete g;
  return GABM_OK;
}

gabm_status gabm_transmit_fwd(gabm_graph g, const void* inf, int32_t fmt, const gabm_params* p, int32_t set,
                              const gabm_rng* rng, int32_t day, double* A, double* lambda, void* stream) {
  GABM_CHECK(g && inf && A && rng, GABM_EINVAL, "graph, inf, A or rng is NULL");
  GABM_CHECK(fmt == GABM_INF_REC || fmt == GABM_INF_F32 || fmt == GABM_INF_F64 || fmt == GABM_INF_BIT1, GABM_EINVAL,
             "unknown inf format");
  const Graph& G = g->g;
  DParams P;
  gabm_status rc = check_params(G, p, &P);
  if (rc != GABM_OK) return rc;
  GABM_CHECK(day >= 0 && day < p->K, GABM_ERANGE, "day outside [0, K)");
  GABM_CHECK(set >= 0 && set < p->n_sets, GABM_ERANGE, "set outside [0, n_sets)");
  hipStream_t st = (hipStream_t)stream;
  StepInf si{inf, fmt, P.TE, P.TI};
  si.iota = P.iota;
  si.day = day;
  si.tau_E = P.tau_E;
  si.W = P.tau_E + P.tau_I;
  const DGraph dg = G.view();
  hipLaunchKernelGGL(k_step_gather, dim3(G.n_tiles), dim3(kBlock), 0, st, dg, si, A);
  if (dg.er_total > 0)
    hipLaunchKernelGGL(k_step_er, dim3(nblk(dg.er_total)), dim3(kBlock), 0, st, dg, rng_of(rng), rng->replicate, day,
                       si, A);
  step_locations(G, si, A, st);
  if (lambda) hipLaunchKernelGGL(k_step_rate, dim3(nblk(G.N)), dim3(kBlock), 0, st, dg, P, set, day, A, lambda);
  GABM_HIP(hipGetLastError());
  return GABM_OK;
}

gabm_status gabm_sample_infect(gabm_graph g, const double* lambda, const gabm_params* p, const gabm_rng* rng,
                               int32_t day, uint8_t* h, double* y, double* dydl, void* stream) {
  GABM_CHECK(g && lambda && h && rng, GABM_EINVAL, "graph, lambda, h or rng is NULL");
  const Graph& G = g->g;
  DParams P;
  gabm_status rc = check_params(G, p, &P);
  if (rc != GABM_OK) return rc;
  GABM_CHECK(day >= 0 && day < p->K, GABM_ERANGE, "day outside [0, K)");
  GABM_CHECK((!y && !dydl) || (p->tau_g > 0.f && p->tau_g < 1.f), GABM_EINVAL, "relaxed sample needs tau_g in (0,1)");
  hipLaunchKernelGGL(k_step_sample, dim3(nblk(G.N)), dim3(kBlock), 0, (hipStream_t)stream, G.view(), P, rng_of(rng),
                     rng->replicate, day, lambda, h, y, dydl);
  GABM_HIP(hipGetLastError());
  return GABM_OK;
}

gabm_status gabm_progress_stages(gabm_graph g, const gabm_rec* rec_in, const uint8_t* h, const gabm_params* p,
                                 int32_t set, const gabm_rng* rng, int32_t day, gabm_rec* rec_out, double* counts,
                                 void* stream) {
  GABM_CHECK(g && rec_in && h && rec_out && counts && rng, GABM_EINVAL, "a pointer argument is NULL");
  GABM_CHECK(rec_in != rec_out, GABM_EINVAL, "rec_in and rec_out must differ");
  const Graph& G = g->g;
  DParams P;
  gabm_status rc = check_params(G, p, &P);
  if (rc != GABM_OK) return rc;
  GABM_CHECK(day >= 0 && day < p->K, GABM_ERANGE, "day outside [0, K)");
  GABM_CHECK(set >= 0 && set < p->n_sets, GABM_ERANGE, "set outside [0, n_sets)");
  hipLaunchKernelGGL(k_step_progress, dim3(nblk(G.N)), dim3(kBlock), 0, (hipStream_t)stream, G.view(), P, set,
                     rng_of(rng), rng->replicate, day, rec_in, h, rec_out, counts);
  GABM_HIP(hipGetLastError());
  return GABM_OK;
}

gabm_status gabm_transmit_bwd(gabm_graph g, const double* gvec, const gabm_rng* rng, int32_t day, double* infbar,
                              void* stream) {
  GABM_CHECK(g && gvec && infbar && rng, GABM_EINVAL, "graph, g, infbar or rng is NULL");
  GABM_CHECK(day >= 0, GABM_ERANGE, "day must be >= 0");
  const Graph& G = g->g;
  hipStream_t st = (hipStream_t)stream;
  StepInf si{gvec, GABM_INF_F64, 0.0, 0.0};
  const DGraph dg = G.view();
  hipLaunchKernelGGL(k_step_gather, dim3(G.n_tiles), dim3(kBlock), 0, st, dg, si, infbar);
  if (dg.er_total > 0)
    hipLaunchKernelGGL(k_step_er, dim3(nblk(dg.er_total)), dim3(kBlock), 0, st, dg, rng_of(rng), rng->replicate, day,
                       si, infbar);
  step_locations(G, si, infbar, st);
  GABM_HIP(hipGetLastError());
  return GABM_OK;
}

namespace gabm {
static void step_locations(const Graph& G, const StepInf& si, double* out, hipStream_t st) {
  if (G.n_visits == 0) return;
  LocView L;
  L.N = G.N; L.n_loc = G.n_loc; L.V = G.n_visits;
  L.lv_agent = G.lv_agent; L.lv_loc = G.lv_loc; L.lv_w = G.lv_w;
  L.av_ptr = G.av_ptr; L.av_loc = G.av_loc; L.av_w = G.av_w;
  hipLaunchKernelGGL(k_fill_f64, dim3(nblk(G.n_loc)), dim3(kBlock), 0, st, G.loc_scratch, (int64_t)G.n_loc);
  hipLaunchKernelGGL(k_loc_pressure<StepInf>, dim3(nblk(G.n_visits)), dim3(kBlock), 0, st, L, si, G.loc_scratch);
  hipLaunchKernelGGL(k_loc_gather<StepInf>, dim3(nblk(std::max<int64_t>(G.N, G.n_loc))), dim3(kBlock), 0, st, L, si,
                     (const double*)G.loc_scratch, out, G.loc_scratch + G.n_loc);
}
}  // namespace gabm

gabm_status gabm_param_grad_reduce(gabm_graph g, const double* lambda_bar, const double* A, const gabm_params* p,
                                   int32_t set, int32_t day, double* dR, double* dS, void* stream) {
  GABM_CHECK(g && lambda_bar && A && dR && dS, GABM_EINVAL, "a pointer argument is NULL");
  const Graph& G = g->g;
  DParams P;
  gabm_status rc = check_params(G, p, &P);
  if (rc != GABM_OK) return rc;
  GABM_CHECK(day >= 0 && day < p->K, GABM_ERANGE, "day outside [0, K)");
  GABM_CHECK(set >= 0 && set < p->n_sets, GABM_ERANGE, "set outside [0, n_sets)");
  GABM_CHECK(!p->per_pop_params, GABM_EUNSUPPORTED, "single-step parameter reduction takes one parameter set");
  hipLaunchKernelGGL(k_step_param, dim3(nblk(G.N)), dim3(kBlock), 0, (hipStream_t)stream, G.view(), P, set, day,
                     lambda_bar, A, dR, dS);
  GABM_HIP(hipGetLastError());
  return GABM_OK;
}

gabm_status gabm_er_daily(gabm_graph g, int32_t pop, const gabm_rng* rng, int32_t day, int32_t* a, int32_t* b,
                          int64_t cap, int64_t* count, void* stream) {
  GABM_CHECK(g && rng && count, GABM_EINVAL, "graph, rng or count is NULL");
  const Graph& G = g->g;
  GABM_CHECK(pop >= 0 && pop < G.n_pops, GABM_ERANGE, "pop outside [0, n_pops)");
  GABM_CHECK(day >= 0, GABM_ERANGE, "day must be >= 0");
  const int64_t n = G.er_off_h[pop + 1] - G.er_off_h[pop];
  *count = n;
  if (n > 0 && cap > 0) {
    GABM_CHECK(a && b, GABM_EINVAL, "a or b is NULL");
    ErArgs e;
    e.G = G.view(); e.rng = rng_of(rng); e.stream = rng->replicate; e.t = day; e.TE = 0; e.TI = 0; e.acc = nullptr;
    hipLaunchKernelGGL(k_er_pairs_out, dim3(nblk(std::min(n, cap))), dim3(kBlock), 0, (hipStream_t)stream, e, pop, a,
                       b, cap);
    GABM_HIP(hipGetLastError());
  }
  GABM_HIP(hipStreamSynchronize((hipStream_t)stream));
  return GABM_OK;
}

static gabm_status check_run(const Graph& G, const gabm_params* p, const gabm_run_desc* run) {
  GABM_CHECK(run != nullptr, GABM_EINVAL, "run desc is NULL");
  GABM_CHECK(run->n_reps >= 1, GABM_EINVAL, "n_reps must be >= 1");
  GABM_CHECK(run->ckpt_every >= 0, GABM_EINVAL, "ckpt_every must be >= 0");
  GABM_CHECK(run->precision == GABM_F32 || run->precision == GABM_F64, GABM_EINVAL, "unknown precision");
  GABM_CHECK(run->time_kernels >= 0, GABM_EINVAL, "time_kernels must be >= 0");
  GABM_CHECK(run->schedule == 0 || run->schedule == 1, GABM_EINVAL, "schedule must be 0 or 1");
  const int64_t B = p->per_pop_params ? run->n_reps : (int64_t)p->n_sets * run->n_reps;
  if (B > 1) {
    GABM_CHECK(p->iota == nullptr, GABM_EUNSUPPORTED, "batched runs take no infectiousness profile");
    GABM_CHECK(G.n_visits == 0, GABM_EUNSUPPORTED, "batched runs take no agent-location layer");
    GABM_CHECK(p->dwell_E == nullptr, GABM_EUNSUPPORTED, "batched runs take no dwell tables");
    GABM_CHECK(B <= kBMaxB, GABM_EUNSUPPORTED, "a batched run takes at most 256 simulations");
    GABM_CHECK(!p->per_pop_params, GABM_EUNSUPPORTED,
               "batched runs take one parameter set per simulation (per-population parameters need B = 1)");
    GABM_CHECK(p->mode != GABM_SOFT, GABM_EUNSUPPORTED, "batched runs use hard states (PLAIN or HARD_ST)");
    GABM_CHECK(run->precision == GABM_F32, GABM_EUNSUPPORTED, "batched runs store float state");
    GABM_CHECK(G.er_off_h.empty() || G.er_off_h.back() == 0, GABM_EUNSUPPORTED,
               "batched runs take static contact layers only (no daily random layer)");
    // per-simulation vectors may be padded to 64 lanes x (1, 2 or 4) simulations per agent
    const int64_t padded = B > 32 ? 64 * (B <= 64 ? 1 : (B <= 128 ? 2 : 4)) : B;
    GABM_CHECK((int64_t)G.N * padded <= ((int64_t)1 << 29), GABM_EUNSUPPORTED,
               "a batched run needs N * B <= 2^29 (B rounded up to 64, 128 or 256 above 32)");
  }
  return GABM_OK;
}

gabm_status gabm_sim_workspace_size(gabm_graph g, const gabm_params* p, const gabm_run_desc* run, size_t* bytes) {
  GABM_CHECK(g && bytes, GABM_EINVAL, "graph or bytes is NULL");
  DParams P;
  gabm_status rc = check_params(g->g, p, &P);
  if (rc != GABM_OK) return rc;
  rc = check_run(g->g, p, run);
  if (rc != GABM_OK) return rc;
  return sim_workspace(g->g, p, run, bytes);
}

gabm_status gabm_sim_create(gabm_graph g, const gabm_params* p, const gabm_run_desc* run, gabm_sim* out) {
  GABM_CHECK(g && out, GABM_EINVAL, "graph or out is NULL");
  *out = nullptr;
  DParams P;
  gabm_status rc = check_params(g->g, p, &P);
  if (rc != GABM_OK) return rc;
  rc = check_run(g->g, p, run);
  if (rc != GABM_OK) return rc;
  gabm_sim s = new (std::nothrow) gabm_sim_s();
  GABM_CHECK(s != nullptr, GABM_ENOMEM, "host allocation failed");
  rc = sim_create(g->g, p, run, s->s);
  if (rc != GABM_OK) {
    delete s;
    return rc;
  }
  *out = s;
  return GABM_OK;
}

static gabm_status sim_params(gabm_sim s, const gabm_params* p, DParams* P) {
  GABM_CHECK(s, GABM_EINVAL, "simulation is NULL");
  gabm_status rc = check_params(*s->s.G, p, P);
  if (rc != GABM_OK) return rc;
  const Sim& S = s->s;
  GABM_CHECK(p->n_sets == S.n_sets && p->K == S.K && p->tau_E == S.tau_E && p->tau_I == S.tau_I &&
                 p->mode == S.mode && (p->per_pop_params ? 1 : 0) == S.per_pop && (p->iota != nullptr) == S.has_iota &&
                     (p->dwell_E != nullptr) == S.has_dwell,
             GABM_EINVAL, "params layout differs from the one the simulation was created with");
  return GABM_OK;
}

gabm_status gabm_sim_forward(gabm_sim s, const gabm_params* p, const gabm_rng* rng, const double* target,
                             int32_t target_stride, const gabm_fwd_out* out, void* stream) {
  DParams P;
  gabm_status rc = sim_params(s, p, &P);
  if (rc != GABM_OK) return rc;
  GABM_CHECK(rng != nullptr, GABM_EINVAL, "rng is NULL");
  GABM_CHECK(out && out->counts, GABM_EINVAL, "out.counts is required");
  GABM_CHECK(target_stride == 0 || target_stride >= s->s.K, GABM_EINVAL, "target_stride must be 0 or >= K");
  return sim_forward(s->s, P, rng, target, target_stride, out, (hipStream_t)stream);
}

gabm_status gabm_sim_backward(gabm_sim s, const gabm_params* p, const gabm_rng* rng, const double* loss_weight,
                              const double* deaths_bar, const gabm_grads* out, void* stream) {
  DParams P;
  gabm_status rc = sim_params(s, p, &P);
  if (rc != GABM_OK) return rc;
  GABM_CHECK(rng != nullptr, GABM_EINVAL, "rng is NULL");
  GABM_CHECK(out && out->dR && out->dS && out->dm && out->di0, GABM_EINVAL, "gradient outputs are required");
  return sim_backward(s->s, P, rng, loss_weight, deaths_bar, out, (hipStream_t)stream);
}

gabm_status gabm_day_fwd(gabm_sim s, const gabm_params* p, const gabm_rng* rng, int32_t day, const double* target,
                         int32_t target_stride, const gabm_fwd_out* out, void* stream) {
  DParams P;
  gabm_status rc = sim_params(s, p, &P);
  if (rc != GABM_OK) return rc;
  GABM_CHECK(rng != nullptr, GABM_EINVAL, "rng is NULL");
  GABM_CHECK(day != s->s.K - 1 || (out && out->counts), GABM_EINVAL, "out.counts is required on the last day");
  return sim_day_fwd(s->s, P, rng, day, target, target_stride, out, (hipStream_t)stream);
}

gabm_status gabm_day_bwd(gabm_sim s, const gabm_params* p, const gabm_rng* rng, int32_t day, const gabm_grads* out,
                         void* stream) {
  DParams P;
  gabm_status rc = sim_params(s, p, &P);
  if (rc != GABM_OK) return rc;
  GABM_CHECK(rng != nullptr, GABM_EINVAL, "rng is NULL");
  GABM_CHECK(day != 0 || (out && out->dR && out->dS && out->dm && out->di0), GABM_EINVAL,
             "gradient outputs are required on day 0");
  return sim_day_bwd(s->s, P, rng, day, out, (hipStream_t)stream);
}

gabm_status gabm_sim_records(gabm_sim s, const gabm_rec** rec) {
  GABM_CHECK(s && rec, GABM_EINVAL, "simulation or rec is NULL");
  *rec = s->s.rec[s->s.cur];
  return GABM_OK;
}

gabm_status gabm_sim_kernel_times(gabm_sim s, gabm_kernel_times* out, int32_t reset) {
  GABM_CHECK(s && out, GABM_EINVAL, "simulation or out is NULL");
  return sim_kernel_times(s->s, out, reset);
}

gabm_status gabm_autotune(gabm_graph g, const gabm_params* p, const gabm_run_desc* run, const gabm_rng* rng,
                          int32_t days, gabm_run_desc* best, double* ms_per_day, void* stream) {
  GABM_CHECK(g && best && rng, GABM_EINVAL, "graph, best or rng is NULL");
  DParams P;
  gabm_status rc = check_params(g->g, p, &P);
  if (rc != GABM_OK) return rc;
  rc = check_run(g->g, p, run);
  if (rc != GABM_OK) return rc;
  GABM_CHECK(days >= 1 && days <= p->K, GABM_ERANGE, "days outside [1, K]");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GABM_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    set_error("hipEventCreate failed");
    return GABM_EHIP;
  }
  int best_sched = 0;
  float best_ms = 0.f;
  for (int sched = 0; sched < GABM_N_SCHEDULES && rc == GABM_OK; ++sched) {
    gabm_run_desc r = *run;
    r.schedule = sched;
    r.use_hip_graph = 0;
    r.time_kernels = 0;
    Sim* s = new (std::nothrow) Sim();
    if (!s) {
      set_error("host allocation failed");
      rc = GABM_ENOMEM;
      break;
    }
    rc = sim_create(g->g, p, &r, *s);
    if (rc == GABM_OK) rc = sim_day_fwd(*s, P, rng, 0, nullptr, 0, nullptr, st);  // warm-up
    float ms = 0.f;
    if (rc == GABM_OK && hipEventRecord(e0, st) != hipSuccess) rc = GABM_EHIP;
    for (int d = 0; d < days && rc == GABM_OK; ++d) rc = sim_day_fwd(*s, P, rng, d, nullptr, 0, nullptr, st);
    if (rc == GABM_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) {
      set_error("timing events failed");
      rc = GABM_EHIP;
    }
    s->release();
    delete s;
    if (rc != GABM_OK) break;
    if (ms_per_day) ms_per_day[sched] = ms / days;
    if (sched == 0 || ms < best_ms) {
      best_ms = ms;
      best_sched = sched;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != GABM_OK) return rc;
  *best = *run;
  best->schedule = best_sched;
  return GABM_OK;
}

gabm_status gabm_sim_destroy(gabm_sim s) {
  if (!s) return GABM_OK;
  s->s.release();
  delete s;
  return GABM_OK;
}

}  // extern "C"
