"""ctypes view of libgabm.so (include/gabm.h).  Argument marshalling only.

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgabm.so")

OK, EINVAL, ENOMEM, EHIP, ENOTSYM, ERANGE, EUNSUPPORTED, ESTATE = range(8)
STATUS_NAMES = {0: "GABM_OK", 1: "GABM_EINVAL", 2: "GABM_ENOMEM", 3: "GABM_EHIP", 4: "GABM_ENOTSYM",
                5: "GABM_ERANGE", 6: "GABM_EUNSUPPORTED", 7: "GABM_ESTATE"}
PLAIN, HARD_ST, SOFT = 0, 1, 2
F32, F64 = 0, 1
SYMMETRIZE, CHECK_SYMMETRIC = 1, 2
INF_REC, INF_F32, INF_F64, INF_BIT1 = 0, 1, 2, 3
TAG_INIT, TAG_INFECT, TAG_MORT, TAG_ER = 0, 1, 2, 3

EXPORTS = (
    "gabm_last_error", "gabm_version", "gabm_graph_build", "gabm_graph_info", "gabm_graph_csr", "gabm_graph_destroy",
    "gabm_transmit_fwd", "gabm_sample_infect", "gabm_progress_stages", "gabm_transmit_bwd",
    "gabm_param_grad_reduce", "gabm_er_daily", "gabm_sim_create", "gabm_sim_workspace_size", "gabm_sim_forward",
    "gabm_sim_backward", "gabm_day_fwd", "gabm_day_bwd", "gabm_sim_records", "gabm_sim_kernel_times",
    "gabm_sim_destroy", "gabm_autotune",
)
N_SCHEDULES = 2


class GabmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class GraphDesc(C.Structure):
    _fields_ = [("n_agents", C.c_int32), ("n_pops", C.c_int32), ("pop_offsets", C.c_void_p), ("age", C.c_void_p),
                ("n_age", C.c_int32), ("n_edges", C.c_int64), ("src", C.c_void_p), ("dst", C.c_void_p),
                ("w", C.c_void_p), ("flags", C.c_uint32), ("er_mean_deg", C.c_float), ("er_weight", C.c_float),
                ("n_locations", C.c_int32), ("reserved1", C.c_int32), ("n_visits", C.c_int64),
                ("visit_agent", C.c_void_p), ("visit_loc", C.c_void_p), ("visit_w", C.c_void_p)]


class GraphStats(C.Structure):
    _fields_ = [("n_agents", C.c_int32), ("n_pops", C.c_int32), ("n_age", C.c_int32), ("n_edges", C.c_int64),
                ("max_degree", C.c_int32), ("n_tiles", C.c_int32), ("n_long_rows", C.c_int32),
                ("weight_sum", C.c_double), ("er_pairs_per_day", C.c_int64), ("n_sender_slices", C.c_int32),
                ("reserved0", C.c_int32), ("n_stream_chunks", C.c_int64), ("n_locations", C.c_int32),
                ("reserved1", C.c_int32), ("n_visits", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("n_sets", C.c_int32), ("K", C.c_int32), ("tau_E", C.c_int32), ("tau_I", C.c_int32),
                ("mode", C.c_int32), ("per_pop_params", C.c_int32), ("R", C.c_void_p), ("S", C.c_void_p),
                ("m", C.c_void_p), ("i0", C.c_void_p), ("Z", C.c_void_p), ("T", C.c_float * 5),
                ("tau_g", C.c_float), ("iota", C.c_void_p), ("dwell_E", C.c_void_p), ("dwell_I", C.c_void_p)]


class Rng(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("replicate", C.c_uint32), ("independent_sets", C.c_uint32)]


class RunDesc(C.Structure):
    _fields_ = [("n_reps", C.c_int32), ("ckpt_every", C.c_int32), ("precision", C.c_int32),
                ("use_hip_graph", C.c_int32), ("schedule", C.c_int32), ("time_kernels", C.c_int32)]


KT_CLASSES = ("gather_fwd", "agent_fwd", "day_fwd", "gather_bwd", "agent_bwd", "day_bwd", "er", "loc")


class KernelTimes(C.Structure):
    _fields_ = [("ms", C.c_double * len(KT_CLASSES)), ("launches", C.c_int64 * len(KT_CLASSES))]


class FwdOut(C.Structure):
    _fields_ = [("counts", C.c_void_p), ("drm", C.c_void_p), ("deaths", C.c_void_p), ("loss", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("dR", C.c_void_p), ("dS", C.c_void_p), ("dm", C.c_void_p), ("di0", C.c_void_p),
                ("ddwell_E", C.c_void_p), ("ddwell_I", C.c_void_p)]


_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libgabm.so is not built ({LIB_PATH}); run __graft_entry__.build() or "
                          f"python paper_2207_09714_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "gabm_last_error": ([], C.c_char_p),
        "gabm_version": ([], C.c_char_p),
        "gabm_graph_build": ([C.POINTER(GraphDesc), vp, C.POINTER(vp)], C.c_int),
        "gabm_graph_info": ([vp, C.POINTER(GraphStats)], C.c_int),
        "gabm_graph_csr": ([vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)], C.c_int),
        "gabm_graph_destroy": ([vp], C.c_int),
        "gabm_transmit_fwd": ([vp, vp, i32, C.POINTER(Params), i32, C.POINTER(Rng), i32, vp, vp, vp], C.c_int),
        "gabm_sample_infect": ([vp, vp, C.POINTER(Params), C.POINTER(Rng), i32, vp, vp, vp, vp], C.c_int),
        "gabm_progress_stages": ([vp, vp, vp, C.POINTER(Params), i32, C.POINTER(Rng), i32, vp, vp, vp], C.c_int),
        "gabm_transmit_bwd": ([vp, vp, C.POINTER(Rng), i32, vp, vp], C.c_int),
        "gabm_param_grad_reduce": ([vp, vp, vp, C.POINTER(Params), i32, i32, vp, vp, vp], C.c_int),
        "gabm_er_daily": ([vp, i32, C.POINTER(Rng), i32, vp, vp, i64, C.POINTER(C.c_int64), vp], C.c_int),
        "gabm_sim_create": ([vp, C.POINTER(Params), C.POINTER(RunDesc), C.POINTER(vp)], C.c_int),
        "gabm_sim_workspace_size": ([vp, C.POINTER(Params), C.POINTER(RunDesc), C.POINTER(C.c_size_t)], C.c_int),
        "gabm_sim_forward": ([vp, C.POINTER(Params), C.POINTER(Rng), vp, i32, C.POINTER(FwdOut), vp], C.c_int),
        "gabm_sim_backward": ([vp, C.POINTER(Params), C.POINTER(Rng), vp, vp, C.POINTER(Grads), vp], C.c_int),
        "gabm_day_fwd": ([vp, C.POINTER(Params), C.POINTER(Rng), i32, vp, i32, C.POINTER(FwdOut), vp], C.c_int),
        "gabm_day_bwd": ([vp, C.POINTER(Params), C.POINTER(Rng), i32, C.POINTER(Grads), vp], C.c_int),
        "gabm_sim_records": ([vp, C.POINTER(vp)], C.c_int),
        "gabm_sim_kernel_times": ([vp, C.POINTER(KernelTimes), i32], C.c_int),
        "gabm_sim_destroy": ([vp], C.c_int),
        "gabm_autotune": ([vp, C.POINTER(Params), C.POINTER(RunDesc), C.POINTER(Rng), i32, C.POINTER(RunDesc),
                           C.POINTER(C.c_double), vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != OK:
        raise GabmError(rc, lib().gabm_last_error().decode(errors="replace"))
