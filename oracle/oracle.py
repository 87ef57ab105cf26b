"""Python access to the FP64 C oracle (ctypes).

TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library or its binding.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "gabm_oracle.c")

PLAIN, HARD_ST, SOFT = 0, 1, 2
STAGES = ("S", "E", "I", "R", "M")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, single thread)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Cfg(C.Structure):
    _fields_ = [
        ("n_agents", C.c_int32), ("n_pops", C.c_int32), ("pop_offsets", C.c_void_p), ("pop_id_base", C.c_int32),
        ("age", C.c_void_p), ("n_edges", C.c_int64), ("src", C.c_void_p), ("dst", C.c_void_p), ("w", C.c_void_p),
        ("er_mean_deg", C.c_double), ("er_weight", C.c_float),
        ("K", C.c_int32), ("n_age", C.c_int32), ("tau_E", C.c_int32), ("tau_I", C.c_int32), ("mode", C.c_int32),
        ("R", C.c_void_p), ("S", C.c_void_p), ("T", C.c_void_p),
        ("m", C.c_float), ("i0", C.c_float), ("tau_g", C.c_float), ("Z", C.c_void_p),
        ("seed", C.c_uint64), ("stream", C.c_uint32), ("target", C.c_void_p),
        ("ndir", C.c_int32), ("dR", C.c_void_p), ("dS", C.c_void_p), ("dm", C.c_void_p), ("di0", C.c_void_p),
        ("iota", C.c_void_p),
        ("n_locations", C.c_int32), ("n_visits", C.c_int64), ("visit_agent", C.c_void_p), ("visit_loc", C.c_void_p),
        ("visit_w", C.c_void_p), ("loc_p", C.c_void_p), ("dwell_E", C.c_void_p), ("dwell_I", C.c_void_p),
        ("ddwE", C.c_void_p), ("ddwI", C.c_void_p),
    ]


class _Out(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("counts", "drm", "deaths", "loss", "A", "lam", "y", "h", "stage", "dL", "dD", "mismatch")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.ora_run.argtypes = [C.POINTER(_Cfg), C.POINTER(_Out)]
        _lib.ora_run.restype = C.c_int
        _lib.ora_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.ora_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        _lib.ora_uniform.restype = C.c_double
        _lib.ora_er_pairs.argtypes = [C.c_int32, C.c_double, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                      C.c_void_p, C.c_void_p, C.c_int64]
        _lib.ora_er_pairs.restype = C.c_int64
        _lib.ora_dwell_draw.argtypes = [C.c_void_p, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint32, C.c_uint32]
        _lib.ora_dwell_draw.restype = C.c_int32
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().ora_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def uniform(seed: int, idx: int, day: int, tag: int, pop: int = 0, stream: int = 0) -> float:
    return lib().ora_uniform(seed, idx, day, tag, pop, stream)


TAG_DWELL_E, TAG_DWELL_I = 4, 6


def dwell_draw(log_weights, seed: int, idx: int, day: int, tag: int, pop: int = 0, stream: int = 0) -> int:
    """The Gumbel-max draw of a length in 1..len(log_weights) for agent idx and
    day (tag TAG_DWELL_E or TAG_DWELL_I)."""
    lw = np.ascontiguousarray(log_weights, np.float32)
    return int(lib().ora_dwell_draw(_p(lw), len(lw), seed, idx & 0xFFFFFFFF, day & 0xFFFFFFFF, tag, pop, stream))


def er_pairs(n_pop: int, mean_deg: float, seed: int, day: int, pop: int = 0, stream: int = 0):
    cap = int(n_pop * mean_deg) + 16
    a = np.zeros(cap, np.int32)
    b = np.zeros(cap, np.int32)
    M = lib().ora_er_pairs(n_pop, mean_deg, seed, day, pop, stream, _p(a), _p(b), cap)
    return a[:M].copy(), b[:M].copy()


def standard_directions(K: int, n_age: int):
    """The 11 gradient directions: R (every day together), S[0..n_age-1], m, i0."""
    nd = 1 + n_age + 2
    dR = np.zeros((nd, K))
    dS = np.zeros((nd, n_age))
    dm = np.zeros(nd)
    di0 = np.zeros(nd)
    dR[0, :] = 1.0
    for a in range(n_age):
        dS[1 + a, a] = 1.0
    dm[1 + n_age] = 1.0
    di0[2 + n_age] = 1.0
    return dR, dS, dm, di0


def dwell_directions(K: int, n_age: int, tau_E: int, tau_I: int):
    """standard_directions followed by one unit direction per dwell log
    weight (E lengths 1..tau_E, then I lengths 1..tau_I), as six arrays."""
    dR, dS, dm, di0 = standard_directions(K, n_age)
    n0 = dR.shape[0]
    nd = n0 + tau_E + tau_I
    pad = lambda x: np.concatenate([x, np.zeros((nd - n0,) + x.shape[1:])])  # noqa: E731
    ddE = np.zeros((nd, tau_E))
    ddI = np.zeros((nd, tau_I))
    for a in range(tau_E):
        ddE[n0 + a, a] = 1.0
    for b in range(tau_I):
        ddI[n0 + tau_E + b, b] = 1.0
    return pad(dR), pad(dS), pad(dm), pad(di0), ddE, ddI


def run(*, age, pop_offsets, src, dst, w, K, R, S, m, i0, Z, T=(0, 0, 1, 0, 0), tau_E=3, tau_I=5,
        mode=PLAIN, tau_g=0.5, seed=0, stream=0, pop_id_base=0, er_mean_deg=0.0, er_weight=0.0,
        target=None, directions=None, want_agents=False, want_stage=False, iota=None, visits=None, dwell=None):
    """Run one simulation.  Parameters are float32 values (widened exactly).

    ``iota`` = infectiousness profile over days since exposure ([tau_E +
    tau_I], float32; None = flat): an agent exposed on day u contributes
    T[stage] * iota[t - u - 1] on day t.

    ``visits`` = (agent[V], location[V], weight[V]) of the agent-location
    layer, or None: a location's pressure is the weighted sum over its
    visitors, and each visit adds weight * (pressure - own share) to its agent.

    ``dwell`` = (log-weights of the E lengths 1..tau_E, of the I lengths
    1..tau_I) for stochastic dwell times drawn per exposure by Gumbel-max, or
    None for the fixed tau_E / tau_I.

    ``directions`` = (dR[nd,K], dS[nd,n_age], dm[nd], di0[nd]) or None, with
    optionally two more, (ddw_E[nd,tau_E], ddw_I[nd,tau_I]), the directions of
    the dwell log weights (straight-through Gumbel-softmax tangents).
    Returns a dict with counts [K+1,5], drm [K], deaths [K], loss, and when
    requested per-agent arrays [K,N] (A, lam, y, h), stage [K+1,N], dL [nd],
    dD [nd,K], mismatch.
    """
    age = np.ascontiguousarray(age, np.uint8)
    n = int(age.shape[0])
    offs = np.ascontiguousarray(pop_offsets, np.int32)
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    w = np.ascontiguousarray(w, np.float32)
    Rv = np.ascontiguousarray(np.broadcast_to(np.asarray(R, np.float32), (K,)), np.float32)
    Sv = np.ascontiguousarray(S, np.float32).reshape(-1)
    Tv = np.ascontiguousarray(T, np.float32)
    Zv = np.ascontiguousarray(np.atleast_1d(np.asarray(Z, np.float32)), np.float32)
    tg = None if target is None else np.ascontiguousarray(target, np.float64)
    cfg = _Cfg()
    cfg.n_agents, cfg.n_pops, cfg.pop_offsets, cfg.pop_id_base = n, len(offs) - 1, _p(offs), pop_id_base
    cfg.age, cfg.n_edges, cfg.src, cfg.dst, cfg.w = _p(age), len(src), _p(src), _p(dst), _p(w)
    cfg.er_mean_deg, cfg.er_weight = float(er_mean_deg), float(er_weight)
    cfg.K, cfg.n_age, cfg.tau_E, cfg.tau_I, cfg.mode = K, len(Sv), tau_E, tau_I, mode
    cfg.R, cfg.S, cfg.T = _p(Rv), _p(Sv), _p(Tv)
    cfg.m, cfg.i0, cfg.tau_g, cfg.Z = float(np.float32(m)), float(np.float32(i0)), float(np.float32(tau_g)), _p(Zv)
    cfg.seed, cfg.stream, cfg.target = int(seed), int(stream), _p(tg)
    keep = [age, offs, src, dst, w, Rv, Sv, Tv, Zv, tg]
    if iota is not None:
        iv = np.ascontiguousarray(iota, np.float32).reshape(-1)
        if iv.shape[0] != tau_E + tau_I:
            raise ValueError("iota needs tau_E + tau_I values")
        cfg.iota = _p(iv)
        keep.append(iv)
    if visits is not None:
        va = np.ascontiguousarray(visits[0], np.int32)
        vl = np.ascontiguousarray(visits[1], np.int32)
        vw = np.ascontiguousarray(visits[2], np.float32)
        nl = int(vl.max()) + 1 if len(vl) else 0
        lp = np.zeros(max(nl, 1))
        cfg.n_locations, cfg.n_visits = nl, len(va)
        cfg.visit_agent, cfg.visit_loc, cfg.visit_w, cfg.loc_p = _p(va), _p(vl), _p(vw), _p(lp)
        keep += [va, vl, vw, lp]
    if dwell is not None:
        dE = np.ascontiguousarray(dwell[0], np.float32).reshape(-1)
        dI = np.ascontiguousarray(dwell[1], np.float32).reshape(-1)
        if dE.shape[0] != tau_E or dI.shape[0] != tau_I:
            raise ValueError("dwell tables need tau_E and tau_I values")
        cfg.dwell_E, cfg.dwell_I = _p(dE), _p(dI)
        keep += [dE, dI]
    nd = 0
    if directions is not None:
        dR, dS, dm, di0 = (np.ascontiguousarray(x, np.float64) for x in directions[:4])
        nd = dR.shape[0]
        cfg.ndir, cfg.dR, cfg.dS, cfg.dm, cfg.di0 = nd, _p(dR), _p(dS), _p(dm), _p(di0)
        keep += [dR, dS, dm, di0]
        if len(directions) > 4:  # tangents of the dwell log weights
            ddE, ddI = (np.ascontiguousarray(x, np.float64) for x in directions[4:6])
            cfg.ddwE, cfg.ddwI = _p(ddE), _p(ddI)
            keep += [ddE, ddI]
    res = {
        "counts": np.zeros((K + 1, 5)), "drm": np.zeros(K), "deaths": np.zeros(K), "loss": np.zeros(1),
        "mismatch": np.zeros(1, np.int64),
    }
    if want_agents:
        res.update(A=np.zeros((K, n)), lam=np.zeros((K, n)), y=np.zeros((K, n)), h=np.zeros((K, n), np.uint8))
    if want_stage:
        res["stage"] = np.zeros((K + 1, n), np.uint8)
    if nd:
        res.update(dL=np.zeros(nd), dD=np.zeros((nd, K)))
    out = _Out()
    for k in _Out._fields_:
        setattr(out, k[0], _p(res.get(k[0])))
    rc = lib().ora_run(C.byref(cfg), C.byref(out))
    if rc != 0:
        raise ValueError(f"oracle rejected the configuration (code {rc})")
    del keep
    res["loss"] = float(res["loss"][0])
    res["mismatch"] = int(res["mismatch"][0])
    return res


def run_workload(wl, *, mode=None, set_index=0, stream=0, seed=None, R=None, target=None, directions=None,
                 want_agents=False, want_stage=False, pop_index=None, iota=None, visits=None, dwell=None):
    """Run a ``synth`` workload on the oracle (one simulation).  For packed
    populations pass ``pop_index`` to simulate that population alone with its
    own parameter set (populations do not share contacts)."""
    if pop_index is not None:
        offs = wl.pop.pop_offsets
        lo, hi = int(offs[pop_index]), int(offs[pop_index + 1])
        sel = (wl.dst >= lo) & (wl.dst < hi)
        return run(age=wl.pop.age[lo:hi], pop_offsets=np.array([0, hi - lo], np.int32),
                   src=wl.src[sel] - lo, dst=wl.dst[sel] - lo, w=wl.w[sel], K=wl.K,
                   R=wl.R[pop_index] if R is None else R, S=wl.S[pop_index], m=wl.m[pop_index],
                   i0=wl.i0[pop_index], Z=wl.Z[pop_index:pop_index + 1], T=wl.T, tau_E=wl.tau_E,
                   tau_I=wl.tau_I, mode=wl.mode if mode is None else mode, tau_g=wl.tau_g,
                   seed=wl.seed if seed is None else seed, stream=stream, pop_id_base=pop_index,
                   er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight, target=target,
                   directions=directions, want_agents=want_agents, want_stage=want_stage, iota=iota, dwell=dwell)
    return run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K,
               R=wl.R[set_index] if R is None else R, S=wl.S[set_index], m=wl.m[set_index], i0=wl.i0[set_index],
               Z=wl.Z, T=wl.T, tau_E=wl.tau_E, tau_I=wl.tau_I, mode=wl.mode if mode is None else mode,
               tau_g=wl.tau_g, seed=wl.seed if seed is None else seed, stream=stream,
               er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight, target=target, directions=directions,
               want_agents=want_agents, want_stage=want_stage, iota=iota, visits=visits, dwell=dwell)
