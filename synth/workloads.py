"""The five synthetic workloads (populations, contact layers, parameters).

Each workload fixes the shapes and value distributions of a simulation run:
population size, age mix, contact layers and their weights, the daily
random (Erdos-Renyi) layer, the horizon, the disease timers and the
parameter values.  The paper's own populations come from US census and
mobility data (Section 4, Appendix E), which are not available; these
synthetic graphs stand in for them.

Names:

* ``c1``  plain forward, N=10,000: households (w=1.0) + daily ER layer
  (mean degree 10, w=0.5); 30 days.
* ``c2``  differentiable, N=100,000: c1's layers + workplaces (60 %
  coverage, w=0.8); 60 days; Gumbel temperature 0.5, straight-through.
* ``c3``  differentiable at scale, N=1,000,000: households, workplaces and a
  Chung-Lu community layer (gamma 2.5, mean degree 15); one weight per
  undirected edge, uniform on (0,1]; 90 days; checkpoint every 10 days.
* ``c4a`` batched: one shared 250,000-agent graph built like c3; 64
  parameter sets x 2 replicates; 45 days.
* ``c4b`` packed: 24 populations of log-uniform size in [20k, 500k], each
  built like c3 and with its own parameter set; 45 days.
* ``c5``  largest: N=8,000,000; Chung-Lu gamma 2.2, mean degree 20, cap
  5,000; 120 days; checkpoint every 15 days.

The normaliser Z of each population (the expected weighted degree times
the infectious period) is an input of the model; it is computed here once
from the realised static layer and the ER layer's expected contribution and
rounded to float32.
"""

from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

from .graphs import (
    Population,
    chung_lu,
    households,
    quantized_unit_weights,
    to_symmetric_coo,
    workplaces,
)

CONFIG_NAMES = ("c1", "c2", "c3", "c4a", "c4b", "c5")

GRAPH_SEED = 0x5EED
N_AGE = 8

# Modes, shared vocabulary with the library and the oracle.
MODE_PLAIN = 0
MODE_HARD_ST = 1
MODE_SOFT = 2


@dataclass
class Workload:
    name: str
    pop: Population
    src: np.ndarray
    dst: np.ndarray
    w: np.ndarray
    er_mean_deg: float
    er_weight: float
    K: int
    tau_E: int
    tau_I: int
    T: np.ndarray  # float32 [5] stage transmissibility S,E,I,R,M
    R: np.ndarray  # float32 [n_sets, K]
    S: np.ndarray  # float32 [n_sets, N_AGE]
    m: np.ndarray  # float32 [n_sets]
    i0: np.ndarray  # float32 [n_sets]
    Z: np.ndarray  # float32 [n_pops]
    tau_g: float
    mode: int
    seed: int
    n_reps: int = 1
    per_pop_params: bool = False
    ckpt_every: int = 0  # 0 = keep every day
    target: np.ndarray | None = None  # float64 [K] daily deaths
    notes: dict = field(default_factory=dict)

    @property
    def n_agents(self) -> int:
        return self.pop.n_agents

    @property
    def n_edges(self) -> int:
        return int(len(self.src))

    @property
    def n_sets(self) -> int:
        return int(self.R.shape[0])


def normaliser(pop: Population, dst: np.ndarray, w: np.ndarray, er_mean_deg: float, er_weight: float, tau_I: int) -> np.ndarray:
    """Z_p = tau_I * (realised static weighted degree + ER expectation),
    per population, rounded to float32."""
    offs = pop.pop_offsets
    wsum = np.zeros(pop.n_pops, np.float64)
    if len(dst):
        # every weight is a multiple of 2^-24, so these float64 sums are exact
        # whatever order they are formed in
        if pop.n_pops == 1:
            wsum[0] = np.sum(w, dtype=np.float64)
        else:
            p_of_edge = np.searchsorted(offs, dst, side="right") - 1
            wsum = np.bincount(p_of_edge, weights=w.astype(np.float64), minlength=pop.n_pops)
    sizes = np.diff(offs).astype(np.float64)
    kbar = wsum / sizes + float(er_mean_deg) * float(np.float32(er_weight))
    return (tau_I * kbar).astype(np.float32)


def _c3_like_layers(n: int, rng: np.random.Generator, gamma: float, mean_deg: float, cap: float | None):
    ha, hb = households(n, rng)
    wa, wb = workplaces(n, rng, 0.6, 5, 50)
    ca, cb = chung_lu(n, rng, gamma, mean_deg, cap)
    return [
        (ha, hb, quantized_unit_weights(rng, len(ha))),
        (wa, wb, quantized_unit_weights(rng, len(wa))),
        (ca, cb, quantized_unit_weights(rng, len(ca))),
    ]


def _ages(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.integers(0, N_AGE, size=n).astype(np.uint8)


def _susceptibility(rng: np.random.Generator, lo: float, hi: float, n_sets: int) -> np.ndarray:
    return rng.uniform(lo, hi, size=(n_sets, N_AGE)).astype(np.float32)


def _cache_dir() -> str | None:
    d = os.environ.get("GABM_SYNTH_CACHE")
    return d if d else None


def make_workload(name: str, n_agents: int | None = None, K: int | None = None, mode: int | None = None,
                  n_sets: int | None = None, n_reps: int | None = None, n_pops: int | None = None) -> Workload:
    """Build one workload.  ``n_agents``/``K``/``n_sets``/``n_reps``/``n_pops``
    shrink it for tests; the defaults give the full configuration."""
    if name not in CONFIG_NAMES:
        raise ValueError(f"unknown workload {name!r}")
    key = (name, n_agents, K, mode, n_sets, n_reps, n_pops)
    cdir = _cache_dir()
    if cdir:
        fn = os.path.join(cdir, "wl_" + "_".join(str(k) for k in key) + ".npz")
        if os.path.exists(fn):
            return _load(fn)
    wl = _build(name, n_agents, K, mode, n_sets, n_reps, n_pops)
    if cdir:
        os.makedirs(cdir, exist_ok=True)
        _save(fn, wl)
    return wl


def _build(name, n_agents, K, mode, n_sets, n_reps, n_pops) -> Workload:
    g = np.random.default_rng(GRAPH_SEED)
    pr = np.random.default_rng(GRAPH_SEED + 1)  # parameter draws
    T = np.array([0, 0, 1, 0, 0], np.float32)
    tau_E, tau_I = 3, 5
    notes: dict = {}

    if name in ("c1", "c2"):
        n = n_agents or (10_000 if name == "c1" else 100_000)
        ha, hb = households(n, g)
        layers = [(ha, hb, 1.0)]
        if name == "c2":
            wa, wb = workplaces(n, g, 0.6, 5, 50)
            layers.append((wa, wb, 0.8))
        src, dst, w = to_symmetric_coo(layers)
        pop = Population(n, _ages(n, g), np.array([0, n], np.int32))
        er_mean, er_w = 10.0, 0.5
        KK = K or (30 if name == "c1" else 60)
        S = _susceptibility(pr, 0.5, 1.0, 1)
        R = np.full((1, KK), 2.5, np.float32)
        md = MODE_PLAIN if name == "c1" else MODE_HARD_ST
        wl = Workload(name, pop, src, dst, w, er_mean, er_w, KK, tau_E, tau_I, T, R, S,
                      np.array([0.01], np.float32), np.array([0.01], np.float32),
                      normaliser(pop, dst, w, er_mean, er_w, tau_I), 0.5,
                      md if mode is None else mode, 0, ckpt_every=0 if name == "c1" else 10, notes=notes)
        return wl

    if name in ("c3", "c5"):
        n = n_agents or (1_000_000 if name == "c3" else 8_000_000)
        if name == "c3":
            gamma, mean, cap = 2.5, 15.0, float(np.sqrt(n * 15.0))
        else:
            gamma, mean, cap = 2.2, 20.0, 5000.0
        src, dst, w = to_symmetric_coo(_c3_like_layers(n, g, gamma, mean, cap))
        pop = Population(n, _ages(n, g), np.array([0, n], np.int32))
        KK = K or (90 if name == "c3" else 120)
        S = _susceptibility(pr, 0.5, 1.0, 1)
        R = np.full((1, KK), 2.5, np.float32)
        notes.update(gamma=gamma, mean_deg=mean, cap=cap)
        return Workload(name, pop, src, dst, w, 0.0, 0.0, KK, tau_E, tau_I, T, R, S,
                        np.array([0.01], np.float32), np.array([0.01], np.float32),
                        normaliser(pop, dst, w, 0.0, 0.0, tau_I), 0.5,
                        MODE_HARD_ST if mode is None else mode, 0,
                        ckpt_every=10 if name == "c3" else 15, notes=notes)

    if name == "c4a":
        n = n_agents or 250_000
        src, dst, w = to_symmetric_coo(_c3_like_layers(n, g, 2.5, 15.0, float(np.sqrt(n * 15.0))))
        pop = Population(n, _ages(n, g), np.array([0, n], np.int32))
        KK = K or 45
        ns = n_sets or 64
        R = np.repeat(pr.uniform(1.5, 4.0, size=(ns, 1)).astype(np.float32), KK, axis=1)
        S = _susceptibility(pr, 0.3, 1.0, ns)
        return Workload(name, pop, src, dst, w, 0.0, 0.0, KK, tau_E, tau_I, T, R, S,
                        np.full(ns, 0.01, np.float32), np.full(ns, 0.01, np.float32),
                        normaliser(pop, dst, w, 0.0, 0.0, tau_I), 0.5,
                        MODE_HARD_ST if mode is None else mode, 0, n_reps=n_reps or 2,
                        ckpt_every=0, notes=notes)

    # c4b: packed populations, one parameter set per population
    npops = n_pops or 24
    if n_agents is None:
        sizes = np.exp(pr.uniform(np.log(2e4), np.log(5e5), size=npops)).astype(np.int64)
    else:
        # same 1:25 size spread as the full workload, largest = n_agents
        sizes = np.maximum(8, np.exp(pr.uniform(np.log(n_agents / 25), np.log(n_agents), size=npops))).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    layers_all = []
    for p in range(npops):
        np_ = int(sizes[p])
        for a, b, w in _c3_like_layers(np_, g, 2.5, 15.0, float(np.sqrt(np_ * 15.0))):
            layers_all.append((a + offs[p], b + offs[p], w))
    src, dst, w = to_symmetric_coo(layers_all)
    n = int(offs[-1])
    pop = Population(n, _ages(n, g), offs)
    KK = K or 45
    R = np.repeat(pr.uniform(1.5, 4.0, size=(npops, 1)).astype(np.float32), KK, axis=1)
    S = _susceptibility(pr, 0.3, 1.0, npops)
    return Workload(name, pop, src, dst, w, 0.0, 0.0, KK, tau_E, tau_I, T, R, S,
                    np.full(npops, 0.01, np.float32), np.full(npops, 0.01, np.float32),
                    normaliser(pop, dst, w, 0.0, 0.0, tau_I), 0.5,
                    MODE_HARD_ST if mode is None else mode, 0, per_pop_params=True,
                    ckpt_every=0, notes=notes)


_ARRAYS = ("src", "dst", "w", "T", "R", "S", "m", "i0", "Z")


def _save(fn: str, wl: Workload) -> None:
    d = {k: getattr(wl, k) for k in _ARRAYS}
    d["age"] = wl.pop.age
    d["pop_offsets"] = wl.pop.pop_offsets
    d["scalars"] = np.array([wl.er_mean_deg, wl.er_weight, wl.K, wl.tau_E, wl.tau_I, wl.tau_g,
                             wl.mode, wl.seed, wl.n_reps, int(wl.per_pop_params), wl.ckpt_every], np.float64)
    d["name"] = np.array(wl.name)
    tmp = fn + ".tmp.npz"
    np.savez(tmp, **d)
    os.replace(tmp, fn)


def _load(fn: str) -> Workload:
    z = np.load(fn, allow_pickle=False)
    sc = z["scalars"]
    pop = Population(int(z["age"].shape[0]), z["age"], z["pop_offsets"])
    return Workload(str(z["name"]), pop, z["src"], z["dst"], z["w"], float(sc[0]), float(sc[1]), int(sc[2]),
                    int(sc[3]), int(sc[4]), z["T"], z["R"], z["S"], z["m"], z["i0"], z["Z"], float(sc[5]),
                    int(sc[6]), int(sc[7]), n_reps=int(sc[8]), per_pop_params=bool(sc[9]), ckpt_every=int(sc[10]))
