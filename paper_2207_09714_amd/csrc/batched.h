// Batched simulations (B = n_sets * n_reps > 1 sharing one graph): one wave
// per receiver, one lane per simulation.
#pragma once

#include "sim_internal.h"

namespace gabm {

template <typename RT>
void batched_init(Sim& s, const DParams& P, Rng rng, hipStream_t st);
template <typename RT>
void batched_day_fwd(Sim& s, const DParams& P, Rng rng, int t, int slot, bool count, hipStream_t st);
void batched_fin_fwd(Sim& s, const DParams& P, const double* target, int stride, const gabm_fwd_out* out, hipStream_t st);
template <typename RT>
void batched_day_bwd(Sim& s, const DParams& P, Rng rng, int t, int slot, hipStream_t st);
template <typename RT>
void batched_forward(Sim& s, const DParams& P, Rng rng, const double* target, int stride, const gabm_fwd_out* out,
                     hipStream_t st);
template <typename RT>
void batched_backward(Sim& s, const DParams& P, Rng rng, const gabm_grads* out, hipStream_t st);

}  // namespace gabm
