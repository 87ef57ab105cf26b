// Batched simulations sharing one contact graph (placeholder: the entry
// points reject B > 1 until the lane-per-simulation kernels land).
#include "batched.h"

namespace gabm {

template <typename RT>
void batched_init(Sim&, const DParams&, Rng, hipStream_t) {}
template <typename RT>
void batched_day_fwd(Sim&, const DParams&, Rng, int, int, bool, hipStream_t) {}
void batched_fin_fwd(Sim&, const DParams&, const double*, int, const gabm_fwd_out*, hipStream_t) {}
template <typename RT>
void batched_day_bwd(Sim&, const DParams&, Rng, int, int, hipStream_t) {}
template <typename RT>
void batched_forward(Sim&, const DParams&, Rng, const double*, int, const gabm_fwd_out*, hipStream_t) {}
template <typename RT>
void batched_backward(Sim&, const DParams&, Rng, const gabm_grads*, hipStream_t) {}

template void batched_init<float>(Sim&, const DParams&, Rng, hipStream_t);
template void batched_init<double>(Sim&, const DParams&, Rng, hipStream_t);
template void batched_day_fwd<float>(Sim&, const DParams&, Rng, int, int, bool, hipStream_t);
template void batched_day_fwd<double>(Sim&, const DParams&, Rng, int, int, bool, hipStream_t);
template void batched_day_bwd<float>(Sim&, const DParams&, Rng, int, int, hipStream_t);
template void batched_day_bwd<double>(Sim&, const DParams&, Rng, int, int, hipStream_t);
template void batched_forward<float>(Sim&, const DParams&, Rng, const double*, int, const gabm_fwd_out*, hipStream_t);
template void batched_forward<double>(Sim&, const DParams&, Rng, const double*, int, const gabm_fwd_out*, hipStream_t);
template void batched_backward<float>(Sim&, const DParams&, Rng, const gabm_grads*, hipStream_t);
template void batched_backward<double>(Sim&, const DParams&, Rng, const gabm_grads*, hipStream_t);

}  // namespace gabm
