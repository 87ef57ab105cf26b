"""Python binding of libgabm (one function per C entry point, same names
without the ``gabm_`` prefix) plus the autograd wrapper.

Only argument marshalling happens here: every step of the simulation runs in
the library's HIP kernels.  PyTorch provides device memory and streams.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from ._lib import GabmError, check, lib  # noqa: F401

PLAIN, HARD_ST, SOFT = L.PLAIN, L.HARD_ST, L.SOFT
F32, F64 = L.F32, L.F64


def _dev():
    if not torch.cuda.is_available():
        raise RuntimeError("gabm needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch.device("cuda", torch.cuda.current_device())


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _on_dev(x, dtype, dev):
    if isinstance(x, torch.Tensor):
        return x.to(device=dev, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=dev)


def version() -> str:
    return lib().gabm_version().decode()


# ---------------------------------------------------------------- graph

class Graph:
    """Contact graph handle (gabm_graph_build).  Inputs may be numpy arrays or
    tensors; they are copied to the device and then into the library."""

    def __init__(self, *, n_agents, src, dst, w=None, age, n_age=8, pop_offsets=None, er_mean_deg=0.0,
                 er_weight=0.0, symmetrize=False, check_symmetric=True, visits=None, n_locations=None,
                 stream=None):
        """visits: optional agent-location layer (agent[V], location[V],
        weight[V]); n_locations defaults to the largest location id + 1."""
        dev = _dev()
        self.n_agents = int(n_agents)
        offs = np.asarray([0, self.n_agents] if pop_offsets is None else pop_offsets, np.int32)
        self._offs = np.ascontiguousarray(offs)
        age_d = _on_dev(age, torch.uint8, dev)
        src_d = _on_dev(src, torch.int32, dev)
        dst_d = _on_dev(dst, torch.int32, dev)
        w_d = None if w is None else _on_dev(w, torch.float32, dev)
        d = L.GraphDesc()
        d.n_agents, d.n_pops, d.pop_offsets = self.n_agents, len(offs) - 1, self._offs.ctypes.data
        d.age, d.n_age, d.n_edges = age_d.data_ptr(), int(n_age), int(src_d.numel())
        d.src, d.dst = src_d.data_ptr(), dst_d.data_ptr()
        d.w = None if w_d is None else w_d.data_ptr()
        d.flags = (L.SYMMETRIZE if symmetrize else 0) | (L.CHECK_SYMMETRIC if check_symmetric else 0)
        d.er_mean_deg, d.er_weight = float(er_mean_deg), float(er_weight)
        if visits is not None:
            va_d = _on_dev(visits[0], torch.int32, dev)
            vl_d = _on_dev(visits[1], torch.int32, dev)
            vw_d = _on_dev(visits[2], torch.float32, dev)
            if not (va_d.numel() == vl_d.numel() == vw_d.numel()):
                raise ValueError("visit arrays differ in length")
            if n_locations is None:
                n_locations = int(vl_d.max().item()) + 1 if vl_d.numel() else 0
            d.n_locations, d.n_visits = int(n_locations), int(va_d.numel())
            d.visit_agent, d.visit_loc, d.visit_w = va_d.data_ptr(), vl_d.data_ptr(), vw_d.data_ptr()
        h = C.c_void_p()
        torch.cuda.synchronize()
        check(lib().gabm_graph_build(C.byref(d), C.c_void_p(_stream(stream)), C.byref(h)))
        self.handle = h
        self.n_pops = len(offs) - 1
        self.n_age = int(n_age)
        self.pop_offsets = offs

    def info(self) -> dict:
        s = L.GraphStats()
        check(lib().gabm_graph_info(self.handle, C.byref(s)))
        return {k: getattr(s, k) for k, _ in L.GraphStats._fields_}

    def csr(self):
        """Copies of the CSR (row_ptr int64 [N+1], col int32 [E], w float32 [E]) as device tensors."""
        rp, col, w = C.c_void_p(), C.c_void_p(), C.c_void_p()
        check(lib().gabm_graph_csr(self.handle, C.byref(rp), C.byref(col), C.byref(w)))
        E = self.info()["n_edges"]
        return (_copy_from(rp.value, self.n_agents + 1, torch.int64), _copy_from(col.value, E, torch.int32),
                _copy_from(w.value, E, torch.float32))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().gabm_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def _copy_from(ptr, n, dtype):
    """Device-to-device copy of n elements at a raw device pointer into a new tensor."""
    global _hip
    out = torch.empty(int(n), dtype=dtype, device=_dev())
    if n == 0 or not ptr:
        return out
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    torch.cuda.synchronize()
    rc = _hip.hipMemcpy(C.c_void_p(out.data_ptr()), C.c_void_p(ptr), out.numel() * out.element_size(), 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out


def graph_build(**kw) -> Graph:
    return Graph(**kw)


# ---------------------------------------------------------------- parameters

class ParamBlock:
    """gabm_params with the device tensors it points to kept alive."""

    def __init__(self, *, R, S, m, i0, Z, K, n_sets, tau_E=3, tau_I=5, mode=HARD_ST, per_pop_params=False,
                 T=(0, 0, 1, 0, 0), tau_g=0.5, iota=None, dwell=None):
        dev = _dev()
        self.R = _on_dev(R, torch.float32, dev).reshape(n_sets, K)
        self.S = _on_dev(S, torch.float32, dev).reshape(n_sets, -1)
        self.m = _on_dev(m, torch.float32, dev).reshape(n_sets)
        self.i0 = _on_dev(i0, torch.float32, dev).reshape(n_sets)
        self.Z = _on_dev(np.atleast_1d(np.asarray(Z, np.float32)) if not isinstance(Z, torch.Tensor) else Z,
                         torch.float32, dev).reshape(-1)
        p = L.Params()
        p.n_sets, p.K, p.tau_E, p.tau_I, p.mode = int(n_sets), int(K), int(tau_E), int(tau_I), int(mode)
        p.per_pop_params = 1 if per_pop_params else 0
        p.R, p.S, p.m, p.i0, p.Z = (self.R.data_ptr(), self.S.data_ptr(), self.m.data_ptr(), self.i0.data_ptr(),
                                    self.Z.data_ptr())
        for k in range(5):
            p.T[k] = float(np.float32(T[k]))
        p.tau_g = float(np.float32(tau_g))
        # infectiousness profile over the tau_E + tau_I days after exposure (None = flat)
        self.iota = None if iota is None else _on_dev(iota, torch.float32, dev).reshape(-1)
        if self.iota is not None and self.iota.numel() != tau_E + tau_I:
            raise ValueError("iota needs tau_E + tau_I values")
        p.iota = None if self.iota is None else self.iota.data_ptr()
        # stochastic dwell times: (log weights of E lengths 1..tau_E, of I lengths 1..tau_I)
        self.dwell = None
        if dwell is not None:
            dE = _on_dev(dwell[0], torch.float32, dev).reshape(-1)
            dI = _on_dev(dwell[1], torch.float32, dev).reshape(-1)
            if dE.numel() != tau_E or dI.numel() != tau_I:
                raise ValueError("dwell tables need tau_E and tau_I values")
            self.dwell = (dE, dI)
            p.dwell_E, p.dwell_I = dE.data_ptr(), dI.data_ptr()
        self.c = p


def make_rng(seed: int, replicate: int = 0, independent_sets: bool = False):
    r = L.Rng()
    r.seed, r.replicate, r.independent_sets = int(seed), int(replicate), 1 if independent_sets else 0
    return r


# ---------------------------------------------------------------- single steps

def transmit_fwd(graph: Graph, inf: torch.Tensor, fmt: int, params: ParamBlock, set_index: int, rng, day: int,
                 A: torch.Tensor, lam: torch.Tensor | None = None, stream=None):
    check(lib().gabm_transmit_fwd(graph.handle, _ptr(inf), int(fmt), C.byref(params.c), int(set_index),
                                  C.byref(rng), int(day), _ptr(A), _ptr(lam), C.c_void_p(_stream(stream))))


def sample_infect(graph: Graph, lam, params: ParamBlock, rng, day: int, h, y=None, dydl=None, stream=None):
    check(lib().gabm_sample_infect(graph.handle, _ptr(lam), C.byref(params.c), C.byref(rng), int(day), _ptr(h),
                                   _ptr(y), _ptr(dydl), C.c_void_p(_stream(stream))))


def progress_stages(graph: Graph, rec_in, h, params: ParamBlock, set_index: int, rng, day: int, rec_out, counts,
                    stream=None):
    check(lib().gabm_progress_stages(graph.handle, _ptr(rec_in), _ptr(h), C.byref(params.c), int(set_index),
                                     C.byref(rng), int(day), _ptr(rec_out), _ptr(counts),
                                     C.c_void_p(_stream(stream))))


def transmit_bwd(graph: Graph, g, rng, day: int, infbar, stream=None):
    check(lib().gabm_transmit_bwd(graph.handle, _ptr(g), C.byref(rng), int(day), _ptr(infbar),
                                  C.c_void_p(_stream(stream))))


def param_grad_reduce(graph: Graph, lam_bar, A, params: ParamBlock, set_index: int, day: int, dR, dS, stream=None):
    check(lib().gabm_param_grad_reduce(graph.handle, _ptr(lam_bar), _ptr(A), C.byref(params.c), int(set_index),
                                       int(day), _ptr(dR), _ptr(dS), C.c_void_p(_stream(stream))))


def er_daily(graph: Graph, pop: int, rng, day: int, stream=None):
    cnt = C.c_int64()
    check(lib().gabm_er_daily(graph.handle, int(pop), C.byref(rng), int(day), None, None, 0, C.byref(cnt),
                              C.c_void_p(_stream(stream))))
    n = cnt.value
    a = torch.empty(max(n, 1), dtype=torch.int32, device=_dev())
    b = torch.empty(max(n, 1), dtype=torch.int32, device=_dev())
    check(lib().gabm_er_daily(graph.handle, int(pop), C.byref(rng), int(day), _ptr(a), _ptr(b), n, C.byref(cnt),
                              C.c_void_p(_stream(stream))))
    return a[:n], b[:n]


# ---------------------------------------------------------------- whole runs

def autotune(graph: "Graph", *, R, S, m, i0, Z, K, n_sets=1, n_reps=1, tau_E=3, tau_I=5, mode=HARD_ST,
             per_pop_params=False, ckpt_every=0, precision=F32, T=(0, 0, 1, 0, 0), tau_g=0.5, seed=0, days=8,
             stream=None):
    """gabm_autotune: time `days` forward days under every kernel schedule and
    return (fastest schedule, milliseconds per day of each schedule)."""
    pb = ParamBlock(R=R, S=S, m=m, i0=i0, Z=Z, K=K, n_sets=n_sets, tau_E=tau_E, tau_I=tau_I, mode=mode,
                    per_pop_params=per_pop_params, T=T, tau_g=tau_g)
    run = L.RunDesc()
    run.n_reps, run.ckpt_every, run.precision, run.use_hip_graph, run.schedule, run.time_kernels = (
        int(n_reps), int(ckpt_every), int(precision), 0, 0, 0)
    best = L.RunDesc()
    ms = (C.c_double * L.N_SCHEDULES)()
    rng = make_rng(seed)
    check(lib().gabm_autotune(graph.handle, C.byref(pb.c), C.byref(run), C.byref(rng), int(days), C.byref(best), ms,
                              C.c_void_p(_stream(stream))))
    return int(best.schedule), [float(x) for x in ms]


class Simulator:
    """gabm_sim: K-day runs of n_sets x n_reps simulations on one graph."""

    def __init__(self, graph: Graph, *, n_sets=1, K, Z, tau_E=3, tau_I=5, mode=HARD_ST, n_reps=1,
                 per_pop_params=False, ckpt_every=0, precision=F32, use_hip_graph=False, T=(0, 0, 1, 0, 0),
                 tau_g=0.5, time_kernels=False, schedule=0, iota=None, dwell=None):
        self.graph = graph
        self.n_sets, self.K, self.n_reps = int(n_sets), int(K), int(n_reps)
        self.per_pop = bool(per_pop_params)
        self.layout = dict(K=K, n_sets=n_sets, tau_E=tau_E, tau_I=tau_I, mode=mode, per_pop_params=per_pop_params,
                           T=T, tau_g=tau_g, iota=iota, dwell=dwell)
        self.Z = Z
        self.n_out = self.n_reps * (graph.n_pops if self.per_pop else self.n_sets)
        zeros = torch.zeros(self.n_sets * max(K, graph.n_age), device=_dev())
        pb = self.params(zeros[: n_sets * K], zeros[: n_sets * graph.n_age], zeros[:n_sets] + 0.5,
                         zeros[:n_sets] + 0.5)
        run = L.RunDesc()
        run.n_reps, run.ckpt_every, run.precision, run.use_hip_graph, run.schedule, run.time_kernels = (
            int(n_reps), int(ckpt_every), int(precision), 1 if use_hip_graph else 0, int(schedule),
            int(time_kernels))
        self._run = run
        h = C.c_void_p()
        check(lib().gabm_sim_create(graph.handle, C.byref(pb.c), C.byref(run), C.byref(h)))
        self.handle = h
        dev = _dev()
        self.counts = torch.zeros(self.n_out, K + 1, 5, dtype=torch.float64, device=dev)
        self.drm = torch.zeros(self.n_out, K, dtype=torch.float64, device=dev)
        self.deaths = torch.zeros(self.n_out, K, dtype=torch.float64, device=dev)
        self.loss = torch.zeros(self.n_out, dtype=torch.float64, device=dev)
        self.dR = torch.zeros(self.n_sets, K, dtype=torch.float64, device=dev)
        self.dS = torch.zeros(self.n_sets, graph.n_age, dtype=torch.float64, device=dev)
        self.dm = torch.zeros(self.n_sets, dtype=torch.float64, device=dev)
        self.di0 = torch.zeros(self.n_sets, dtype=torch.float64, device=dev)
        # straight-through gradients of the dwell log weights (HARD_ST runs with dwell tables)
        self.ddwell = None
        if dwell is not None and mode == HARD_ST:
            self.ddwell = (torch.zeros(tau_E, dtype=torch.float64, device=dev),
                           torch.zeros(tau_I, dtype=torch.float64, device=dev))

    def workspace_size(self) -> int:
        pb = self.params(torch.zeros(self.n_sets, self.K), torch.zeros(self.n_sets, self.graph.n_age),
                         torch.zeros(self.n_sets), torch.zeros(self.n_sets))
        n = C.c_size_t()
        check(lib().gabm_sim_workspace_size(self.graph.handle, C.byref(pb.c), C.byref(self._run), C.byref(n)))
        return int(n.value)

    def params(self, R, S, m, i0) -> ParamBlock:
        return ParamBlock(R=R, S=S, m=m, i0=i0, Z=self.Z, **self.layout)

    def _out(self):
        o = L.FwdOut()
        o.counts, o.drm, o.deaths, o.loss = (self.counts.data_ptr(), self.drm.data_ptr(), self.deaths.data_ptr(),
                                             self.loss.data_ptr())
        return o

    def _grads(self):
        g = L.Grads()
        g.dR, g.dS, g.dm, g.di0 = self.dR.data_ptr(), self.dS.data_ptr(), self.dm.data_ptr(), self.di0.data_ptr()
        if self.ddwell is not None:
            g.ddwell_E, g.ddwell_I = self.ddwell[0].data_ptr(), self.ddwell[1].data_ptr()
        return g

    @staticmethod
    def _target(target, K):
        if target is None:
            return None, 0
        t = target.to(dtype=torch.float64).contiguous() if isinstance(target, torch.Tensor) else \
            torch.as_tensor(np.asarray(target, np.float64), device=_dev())
        t = t.to(_dev())
        return t, (0 if t.dim() == 1 else K)

    def forward(self, params: ParamBlock, seed=0, replicate=0, target=None, stream=None, independent_sets=False):
        rng = make_rng(seed, replicate, independent_sets)
        tgt, stride = self._target(target, self.K)
        self._keep = (params, tgt)
        out = self._out()
        check(lib().gabm_sim_forward(self.handle, C.byref(params.c), C.byref(rng), _ptr(tgt), stride,
                                     C.byref(out), C.c_void_p(_stream(stream))))
        return dict(counts=self.counts, drm=self.drm, deaths=self.deaths, loss=self.loss)

    def backward(self, params: ParamBlock, seed=0, replicate=0, loss_weight=None, deaths_bar=None, stream=None,
                 independent_sets=False):
        rng = make_rng(seed, replicate, independent_sets)
        lw = None if loss_weight is None else loss_weight.to(torch.float64).contiguous()
        db = None if deaths_bar is None else deaths_bar.to(torch.float64).contiguous()
        self._keep_b = (params, lw, db)
        g = self._grads()
        check(lib().gabm_sim_backward(self.handle, C.byref(params.c), C.byref(rng), _ptr(lw), _ptr(db),
                                      C.byref(g), C.c_void_p(_stream(stream))))
        out = dict(dR=self.dR, dS=self.dS, dm=self.dm, di0=self.di0)
        if self.ddwell is not None:
            out["ddwell_E"], out["ddwell_I"] = self.ddwell
        return out

    def day_fwd(self, params: ParamBlock, day, seed=0, replicate=0, target=None, stream=None, independent_sets=False):
        rng = make_rng(seed, replicate, independent_sets)
        tgt, stride = self._target(target, self.K)
        self._keep = (params, tgt)
        out = self._out()
        check(lib().gabm_day_fwd(self.handle, C.byref(params.c), C.byref(rng), int(day), _ptr(tgt), stride,
                                 C.byref(out), C.c_void_p(_stream(stream))))

    def day_bwd(self, params: ParamBlock, day, seed=0, replicate=0, stream=None, independent_sets=False):
        rng = make_rng(seed, replicate, independent_sets)
        g = self._grads()
        check(lib().gabm_day_bwd(self.handle, C.byref(params.c), C.byref(rng), int(day), C.byref(g),
                                 C.c_void_p(_stream(stream))))

    def kernel_times(self, reset=True) -> dict:
        kt = L.KernelTimes()
        check(lib().gabm_sim_kernel_times(self.handle, C.byref(kt), 1 if reset else 0))
        return {name: {"ms": kt.ms[c], "launches": int(kt.launches[c])} for c, name in enumerate(L.KT_CLASSES)}

    def records(self) -> torch.Tensor:
        p = C.c_void_p()
        check(lib().gabm_sim_records(self.handle, C.byref(p)))
        return _copy_from(p.value, self.graph.n_agents * (self.n_reps if self.per_pop else self.n_sets * self.n_reps),
                          torch.int32)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().gabm_sim_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GabmSim(torch.autograd.Function):
    """loss [n_out], deaths [n_out, K] = GabmSim.apply(R, S, m, i0, sim, seed, target).

    R [n_sets, K], S [n_sets, n_age], m [n_sets], i0 [n_sets] (float32 cuda).
    The backward is the library's hand-written adjoint (straight-through in
    HARD_ST mode, exact in SOFT mode) with checkpoint recomputation."""

    @staticmethod
    def forward(ctx, R, S, m, i0, sim: Simulator, seed: int, target):
        pb = sim.params(R.detach(), S.detach(), m.detach(), i0.detach())
        out = sim.forward(pb, seed=seed, target=target)
        ctx.sim, ctx.seed, ctx.pb = sim, seed, pb
        ctx.dtypes = (R.dtype, S.dtype, m.dtype, i0.dtype)
        return out["loss"].clone(), out["deaths"].clone()

    @staticmethod
    def backward(ctx, gloss, gdeaths):
        sim = ctx.sim
        g = sim.backward(ctx.pb, seed=ctx.seed, loss_weight=gloss, deaths_bar=gdeaths)
        dt = ctx.dtypes
        return (g["dR"].to(dt[0]).clone(), g["dS"].to(dt[1]).clone(), g["dm"].to(dt[2]).clone(),
                g["di0"].to(dt[3]).clone(), None, None, None)
