"""GPU parity of the agent-location layer (the GradABM-JUNE form of Section 6:
agents meet at locations; a location's pressure is the weighted sum of its
visitors' infectiousness, and each visit adds its weight times the pressure
less the visitor's own share).  Whole runs against the FP64 oracle --
trajectories bit-exact (visit weights k/64 and contact weights multiples of
2^-24 keep every sum exact), gradients against its forward-mode tangents --
on both kernel schedules, with the static layers and the daily random layer
alongside, with presymptomatic transmission and the infectiousness profile,
on packed populations, and on a graph of locations alone against the same
run on the expanded contact graph; plus the argument checks."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from synth import location_degree, location_visits, make_workload  # noqa: E402

PROFILE = np.array([0.25, 0.5, 0.75, 1.5, 1.75, 1.25, 0.75, 0.25], np.float32)
T_PRE = (0.0, 0.5, 1.0, 0.0, 0.0)


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def G():
    from paper_2207_09714_amd import gabm

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return gabm


@pytest.fixture(scope="module")
def O():
    from oracle import oracle

    return oracle


def with_visits(wl, seed=7, kmax=32):
    """The workload's visits and its normaliser raised by the layer's mean
    weighted degree (times the infectious period)."""
    va, vl, vw, nl = location_visits(wl.pop, np.random.default_rng(seed), kmax=kmax)
    deg = location_degree(wl.n_agents, (va, vl, vw))
    offs = wl.pop.pop_offsets
    Z = np.array([wl.Z[p] + wl.tau_I * deg[offs[p]:offs[p + 1]].mean() for p in range(wl.pop.n_pops)], np.float32)
    return (va, vl, vw), nl, Z


def graph_of(G, wl, visits, nl, **kw):
    return G.Graph(n_agents=wl.n_agents, src=wl.src, dst=wl.dst, w=wl.w, age=wl.pop.age, n_age=8,
                   pop_offsets=wl.pop.pop_offsets, er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight,
                   visits=visits, n_locations=nl, **kw)


def assert_grads(got, want, tol=1e-4):
    scale = np.maximum(np.abs(want), 1e-3 * np.max(np.abs(want)))
    err = np.abs(got - want) / scale
    assert np.all(err <= tol), f"max scaled error {err.max():.3g}\n got {got}\nwant {want}"


def grads_vec(gr, per_pop=False):
    if per_pop:
        return gr
    return np.concatenate([[gr["dR"][0].sum().item()], gr["dS"][0].cpu().numpy(), gr["dm"].cpu().numpy(),
                           gr["di0"].cpu().numpy()])


CASES = [
    # mode, precision, schedule, T, profile
    (1, 0, 0, None, False),
    (1, 0, 1, None, False),
    (1, 1, 0, None, False),
    (2, 1, 0, None, False),
    (0, 0, 0, None, False),
    (1, 0, 0, T_PRE, True),
    (2, 1, 0, T_PRE, True),
]
IDS = ["hard_st-f32-split", "hard_st-f32-tiles", "hard_st-f64", "soft-f64", "plain-f32", "hard_st-profile",
       "soft-profile"]


@pytest.mark.parametrize("mode,precision,schedule,T,profile", CASES, ids=IDS)
def test_location_runs_match_oracle(G, O, mode, precision, schedule, T, profile):
    wl = make_workload("c2", n_agents=6000, K=24)
    visits, nl, Z = with_visits(wl)
    T = wl.T if T is None else np.asarray(T, np.float32)
    iota = PROFILE if profile else None
    tgt = np.linspace(0.0, 0.6, wl.K)
    _say(f"location run N={wl.n_agents} V={len(visits[0])} L={nl} mode={mode} precision={precision} "
         f"schedule={schedule} profile={profile}")
    g = graph_of(G, wl, visits, nl)
    info = g.info()
    assert info["n_locations"] == nl and info["n_visits"] == len(visits[0])
    sim = G.Simulator(g, K=wl.K, Z=Z, mode=mode, precision=precision, ckpt_every=5, T=T, tau_g=wl.tau_g,
                      iota=iota, schedule=schedule)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    out = sim.forward(pb, seed=wl.seed, target=torch.tensor(tgt, device="cuda"))
    dirs = O.standard_directions(wl.K, 8) if mode != 0 else None
    omode = {0: O.PLAIN, 1: O.HARD_ST, 2: O.SOFT}[mode]
    ref = O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K, R=wl.R[0],
                S=wl.S[0], m=wl.m[0], i0=wl.i0[0], Z=Z, T=T, mode=omode, tau_g=wl.tau_g, seed=wl.seed,
                er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight, target=tgt, directions=dirs, iota=iota,
                visits=visits)
    counts = out["counts"][0].cpu().numpy()
    if mode == 2:
        assert np.allclose(counts, ref["counts"], rtol=1e-10, atol=1e-9)
    else:
        assert np.array_equal(counts, ref["counts"])
        assert ref["mismatch"] == 0
    assert float(out["loss"][0]) == pytest.approx(ref["loss"], rel=1e-10)
    if mode != 0:
        gr = sim.backward(pb, seed=wl.seed)
        assert_grads(grads_vec(gr), ref["dL"])


def test_location_layer_changes_the_epidemic(G):
    """The same run with and without the layer differs (it is not ignored)."""
    wl = make_workload("c2", n_agents=6000, K=24)
    visits, nl, Z = with_visits(wl)
    res = {}
    for name, v in (("without", None), ("with", visits)):
        g = graph_of(G, wl, v, nl if v is not None else None)
        sim = G.Simulator(g, K=wl.K, Z=Z, mode=G.HARD_ST, tau_g=wl.tau_g)
        out = sim.forward(sim.params(wl.R, wl.S, wl.m, wl.i0), seed=wl.seed)
        res[name] = out["counts"][0].cpu().numpy().copy()
    assert not np.array_equal(res["without"], res["with"])
    assert res["with"][-1][0] < res["without"][-1][0]  # more contacts: fewer left susceptible


def _expanded(visits):
    """The clique graph the visits stand for, both directions listed."""
    va, vl, vw = visits
    pair = {}
    by_loc = {}
    for a, l, w in zip(va.tolist(), vl.tolist(), vw.tolist()):
        by_loc.setdefault(l, []).append((a, w))
    for members in by_loc.values():
        for a, wa in members:
            for b, wb in members:
                if a != b:
                    pair[(a, b)] = pair.get((a, b), 0.0) + wa * wb
    keys = list(pair)
    src = np.array([b for a, b in keys], np.int32)
    dst = np.array([a for a, b in keys], np.int32)
    w = np.array([pair[k] for k in keys], np.float64)
    assert np.array_equal(w.astype(np.float32).astype(np.float64), w)  # exact in float32
    return src, dst, w.astype(np.float32)


@pytest.mark.parametrize("mode", [1, 2], ids=["hard_st", "soft"])
def test_locations_alone_equal_the_expanded_graph(G, O, mode):
    """A graph of locations only (no stored contacts: the tile kernels) against
    the same run on the expanded clique graph (GPU) and on the oracle."""
    wl = make_workload("c1", n_agents=3000, K=20)
    va, vl, vw, nl = location_visits(wl.pop, np.random.default_rng(11), school=(20, 60), work=(5, 30),
                                     leisure=(5, 40), kmax=32)
    visits = (va, vl, vw)
    deg = location_degree(wl.n_agents, visits)
    Z = np.array([wl.tau_I * deg.mean()], np.float32)
    src, dst, w = _expanded(visits)
    _say(f"locations alone N={wl.n_agents} V={len(va)} L={nl} expanded E={len(src)} mode={mode}")
    age = wl.pop.age
    ga = G.Graph(n_agents=wl.n_agents, src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32), age=age,
                 visits=visits, n_locations=nl)
    gb = G.Graph(n_agents=wl.n_agents, src=src, dst=dst, w=w, age=age)
    tgt = torch.tensor(np.linspace(0.0, 0.5, wl.K), device="cuda")
    outs, grads = [], []
    for g in (ga, gb):
        sim = G.Simulator(g, K=wl.K, Z=Z, mode=mode, precision=1, ckpt_every=4, tau_g=wl.tau_g)
        pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
        outs.append(sim.forward(pb, seed=wl.seed, target=tgt))
        grads.append(grads_vec(sim.backward(pb, seed=wl.seed)))
    ca, cb = (o["counts"][0].cpu().numpy() for o in outs)
    omode = O.HARD_ST if mode == 1 else O.SOFT
    ref = O.run(age=age, pop_offsets=[0, wl.n_agents], src=[], dst=[], w=[], K=wl.K, R=wl.R[0], S=wl.S[0],
                m=wl.m[0], i0=wl.i0[0], Z=Z, T=wl.T, mode=omode, tau_g=wl.tau_g, seed=wl.seed,
                target=tgt.cpu().numpy(), directions=O.standard_directions(wl.K, 8), visits=visits)
    if mode == 1:
        assert np.array_equal(ca, cb) and np.array_equal(ca, ref["counts"])
    else:
        assert np.allclose(ca, cb, rtol=1e-10, atol=1e-9) and np.allclose(ca, ref["counts"], rtol=1e-10, atol=1e-9)
    assert ca[-1][0] < wl.n_agents * 0.95  # the layer spreads infection
    assert_grads(grads[0], ref["dL"])
    assert_grads(grads[1], ref["dL"])


def test_location_layer_on_packed_populations(G, O):
    """Packed populations, each with its own venues and parameter set: each
    population's trajectory equals the oracle's run of it alone."""
    wl = make_workload("c4b", n_agents=4000, K=16, n_pops=3)
    visits, nl, Z = with_visits(wl, seed=5)
    P = wl.pop.n_pops
    _say(f"packed populations with locations N={wl.n_agents} pops={P} V={len(visits[0])}")
    g = graph_of(G, wl, visits, nl)
    sim = G.Simulator(g, n_sets=P, K=wl.K, Z=Z, mode=G.HARD_ST, per_pop_params=True, tau_g=wl.tau_g)
    out = sim.forward(sim.params(wl.R, wl.S, wl.m, wl.i0), seed=wl.seed)
    counts = out["counts"].cpu().numpy()
    offs = wl.pop.pop_offsets
    va, vl, vw = visits
    for p in range(P):
        lo, hi = int(offs[p]), int(offs[p + 1])
        sel = (wl.dst >= lo) & (wl.dst < hi)
        vs = (va >= lo) & (va < hi)
        # the population's own locations, renumbered from 0
        _, vloc = np.unique(vl[vs], return_inverse=True)
        ref = O.run(age=wl.pop.age[lo:hi], pop_offsets=[0, hi - lo], src=wl.src[sel] - lo, dst=wl.dst[sel] - lo,
                    w=wl.w[sel], K=wl.K, R=wl.R[p], S=wl.S[p], m=wl.m[p], i0=wl.i0[p], Z=Z[p:p + 1], T=wl.T,
                    mode=O.HARD_ST, tau_g=wl.tau_g, seed=wl.seed, pop_id_base=p,
                    visits=(va[vs] - lo, vloc.astype(np.int32), vw[vs]))
        assert np.array_equal(counts[p], ref["counts"]), p


def test_location_argument_checks(G):
    from paper_2207_09714_amd import _lib as L

    wl = make_workload("c1", n_agents=2000, K=8)
    n = wl.n_agents
    good = (np.array([0, 1, 2, 3], np.int32), np.array([0, 0, 1, 1], np.int32), np.full(4, 0.5, np.float32))

    def build(visits, nl=None, offs=None):
        return G.Graph(n_agents=n, src=wl.src, dst=wl.dst, w=wl.w, age=wl.pop.age, visits=visits, n_locations=nl,
                       pop_offsets=offs)

    def code_of(visits, nl=None, offs=None):
        with pytest.raises(L.GabmError) as e:
            build(visits, nl, offs)
        return e.value.code

    assert build(good).info()["n_visits"] == 4
    assert code_of((good[0], good[1], good[2]), nl=1) == L.ERANGE  # location id >= n_locations
    assert code_of((np.array([0, n], np.int32), good[1][:2], good[2][:2])) == L.ERANGE  # agent id out of range
    assert code_of((good[0], good[1], np.array([0.5, -0.5, 0.5, 0.5], np.float32))) == L.EINVAL
    assert code_of((good[0], good[1], np.array([0.5, np.nan, 0.5, 0.5], np.float32))) == L.EINVAL
    assert code_of((np.array([0, 0], np.int32), np.array([1, 1], np.int32), np.full(2, 0.5, np.float32))) == L.EINVAL
    # one location visited from two populations (agents 10 and 1500 with offsets [0, 1000, n])
    two = np.array([0, 1000, n], np.int32)
    cross = (np.array([10, 1500], np.int32), np.array([0, 0], np.int32), np.full(2, 0.5, np.float32))
    sel = ((wl.dst < 1000) == (wl.src < 1000))  # the contacts that stay inside a population
    with pytest.raises(L.GabmError) as e:
        G.Graph(n_agents=n, src=wl.src[sel], dst=wl.dst[sel], w=wl.w[sel], age=wl.pop.age, visits=cross,
                pop_offsets=two)
    assert e.value.code == L.ERANGE
    # batched runs do not take the layer
    g = build(good)
    with pytest.raises(L.GabmError) as e:
        G.Simulator(g, n_sets=2, K=wl.K, Z=wl.Z, mode=G.HARD_ST)
    assert e.value.code == L.EUNSUPPORTED


def test_single_step_sums_with_locations(G, O):
    """gabm_transmit_fwd from day-0 records on a graph with contacts, the
    daily random layer and venues equals the oracle's day-0 sums bit for bit;
    gabm_transmit_bwd of a vector equals the forward sum of the same vector
    (every layer is symmetric), exactly for dyadic values."""
    wl = make_workload("c2", n_agents=6000, K=4)
    visits, nl, Z = with_visits(wl)
    g = graph_of(G, wl, visits, nl)
    ref = O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K, R=wl.R[0],
                S=wl.S[0], m=wl.m[0], i0=wl.i0[0], Z=Z, T=wl.T, mode=O.PLAIN, seed=wl.seed,
                er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight, want_agents=True, want_stage=True,
                visits=visits)
    st0 = ref["stage"][0].astype(np.uint32)
    rec = np.where(st0 == 2, 2 | (5 << 8) | (0xFFFF << 16), 0 | (0xFFFF << 16)).astype(np.uint32)
    pb = G.ParamBlock(R=wl.R, S=wl.S, m=wl.m, i0=wl.i0, Z=Z, K=wl.K, n_sets=1, mode=G.PLAIN, T=wl.T)
    rng = G.make_rng(wl.seed)
    A = torch.zeros(wl.n_agents, dtype=torch.float64, device="cuda")
    G.transmit_fwd(g, torch.tensor(rec.view(np.int32), device="cuda"), 0, pb, 0, rng, 0, A)
    torch.cuda.synchronize()
    assert np.array_equal(A.cpu().numpy(), ref["A"][0])
    gv = torch.tensor(np.random.default_rng(3).integers(-512, 513, wl.n_agents) / 1024.0, device="cuda")
    fwd = torch.zeros_like(gv)
    bwd = torch.zeros_like(gv)
    G.transmit_fwd(g, gv, 2, pb, 0, rng, 1, fwd)
    G.transmit_bwd(g, gv, rng, 1, bwd)
    torch.cuda.synchronize()
    assert torch.equal(fwd, bwd) and float(fwd.abs().max()) > 0


def test_location_layer_hip_graph_replays_and_timing(G):
    """Captured day loops (the pressure buffer is cleared by a fill kernel in
    the graph) replay to the eager result three times, with eager work in
    between; eager kernel timing counts one location pass per forward day,
    per replayed day and per reverse gather."""
    wl = make_workload("c2", n_agents=6000, K=20)
    visits, nl, Z = with_visits(wl)
    _say(f"location layer under hipGraph N={wl.n_agents} V={len(visits[0])}")
    g = graph_of(G, wl, visits, nl)
    t = torch.tensor(np.linspace(0.0, 0.5, wl.K), device="cuda")
    res = {}
    for hip_graph in (False, True):
        sim = G.Simulator(g, K=wl.K, Z=Z, mode=G.HARD_ST, ckpt_every=6, use_hip_graph=hip_graph, tau_g=wl.tau_g,
                          time_kernels=not hip_graph)
        pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
        runs = []
        for rep in range(3 if hip_graph else 1):
            out = sim.forward(pb, seed=wl.seed, target=t)
            gr = sim.backward(pb, seed=wl.seed)
            runs.append((out["counts"].cpu().numpy().copy(), grads_vec(gr)))
            x = torch.randn(1000, device="cuda").sum()
            torch.cuda.synchronize()
            del x
        if not hip_graph:
            kt = sim.kernel_times(reset=True)
            n_seg = (wl.K + 5) // 6
            assert kt["loc"]["launches"] == wl.K + (n_seg - 1) * 6 + wl.K, kt
            assert kt["loc"]["ms"] > 0
        res[hip_graph] = runs
    c0, g0 = res[False][0]
    for c, gv in res[True]:
        assert np.array_equal(c, c0)
        assert np.allclose(gv, g0, rtol=1e-9)


def test_location_layer_day_level_entry_points_after_replays(G):
    """The per-day entry points on a location graph, run after captured runs
    have been replayed on the same simulation (the pressure buffers must start
    clear whatever the replays left), equal the whole run."""
    wl = make_workload("c2", n_agents=6000, K=15)
    visits, nl, Z = with_visits(wl)
    _say(f"location layer, day-level entry points after replays N={wl.n_agents}")
    g = graph_of(G, wl, visits, nl)
    t = torch.tensor(np.linspace(0.0, 0.5, wl.K), device="cuda")
    eager = G.Simulator(g, K=wl.K, Z=Z, mode=G.HARD_ST, ckpt_every=0, tau_g=wl.tau_g)
    pe = eager.params(wl.R, wl.S, wl.m, wl.i0)
    out = eager.forward(pe, seed=wl.seed, target=t)
    want_c = out["counts"].cpu().numpy().copy()
    want_g = grads_vec(eager.backward(pe, seed=wl.seed))
    sim = G.Simulator(g, K=wl.K, Z=Z, mode=G.HARD_ST, ckpt_every=0, tau_g=wl.tau_g, use_hip_graph=True)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    for _ in range(2):
        sim.forward(pb, seed=wl.seed, target=t)
        sim.backward(pb, seed=wl.seed)
    sim.forward(pb, seed=wl.seed, target=t)  # replayed forward, then the reverse day by day
    for d in range(wl.K, -1, -1):
        sim.day_bwd(pb, d, seed=wl.seed)
    assert np.allclose(grads_vec({"dR": sim.dR, "dS": sim.dS, "dm": sim.dm, "di0": sim.di0}), want_g, rtol=1e-9)
    for d in range(wl.K):
        sim.day_fwd(pb, d, seed=wl.seed, target=t)
    assert np.array_equal(sim.counts.cpu().numpy(), want_c)


@pytest.mark.timeout(300)
def test_full_size_c3_with_venues(G, O):
    """The 1M-agent, 90-day workload plus the JUNE-like venues of the
    benchmark's location leg (1.1M visits), in its launch configuration
    (split kernels, float32 state, straight-through mode, checkpoint every 10
    days): daily counts and removals equal the oracle's."""
    wl = make_workload("c3")
    va, vl, vw, nl = location_visits(wl.pop, np.random.default_rng(0x10C))
    deg = location_degree(wl.n_agents, (va, vl, vw))
    Z = (wl.Z + np.float32(wl.tau_I * deg.mean())).astype(np.float32)
    _say(f"full c3 with venues N={wl.n_agents} E={wl.n_edges} V={len(va)} L={nl} K={wl.K}")
    g = G.Graph(n_agents=wl.n_agents, src=wl.src, dst=wl.dst, w=wl.w, age=wl.pop.age, visits=(va, vl, vw),
                n_locations=nl)
    sim = G.Simulator(g, K=wl.K, Z=Z, mode=G.HARD_ST, ckpt_every=10, tau_g=wl.tau_g)
    out = sim.forward(sim.params(wl.R, wl.S, wl.m, wl.i0), seed=wl.seed)
    counts = out["counts"][0].cpu().numpy()
    drm = out["drm"][0].cpu().numpy()
    del sim, g
    ref = O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K, R=wl.R[0],
                S=wl.S[0], m=wl.m[0], i0=wl.i0[0], Z=Z, T=wl.T, mode=O.PLAIN, seed=wl.seed, visits=(va, vl, vw))
    assert np.array_equal(counts, ref["counts"])
    assert np.array_equal(drm, ref["drm"])


def test_location_layer_edge_cases(G, O):
    """Venues with a single visitor (they add nothing), zero-weight visits,
    agents without visits, unused location ids above the largest one visited,
    and visits listed in random order: trajectories equal the oracle's, and
    the per-agent accumulators start clean on a second run."""
    wl = make_workload("c1", n_agents=3000, K=16)
    rng = np.random.default_rng(5)
    n = wl.n_agents
    members = rng.permutation(n)[: n // 2]  # half the agents visit nothing
    va = np.concatenate([members, members[:200]]).astype(np.int32)
    vl = np.concatenate([rng.integers(0, 60, len(members)), 60 + np.arange(200)]).astype(np.int32)  # 200 singletons
    vw = (rng.integers(0, 33, len(va)) / 64.0).astype(np.float32)  # some weights 0
    order = rng.permutation(len(va))
    visits = (va[order], vl[order], vw[order])
    deg = location_degree(n, visits)
    Z = (wl.Z + np.float32(wl.tau_I * deg.mean())).astype(np.float32)
    _say(f"location edge cases N={n} V={len(va)}")
    g = G.Graph(n_agents=n, src=wl.src, dst=wl.dst, w=wl.w, age=wl.pop.age, er_mean_deg=wl.er_mean_deg,
                er_weight=wl.er_weight, visits=visits, n_locations=400)
    assert g.info()["n_locations"] == 400
    sim = G.Simulator(g, K=wl.K, Z=Z, mode=G.HARD_ST, ckpt_every=4, tau_g=wl.tau_g)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    ref = O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K, R=wl.R[0],
                S=wl.S[0], m=wl.m[0], i0=wl.i0[0], Z=Z, T=wl.T, mode=O.HARD_ST, tau_g=wl.tau_g, seed=wl.seed,
                er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight, visits=visits)
    for rep in range(2):
        out = sim.forward(pb, seed=wl.seed)
        assert np.array_equal(out["counts"][0].cpu().numpy(), ref["counts"]), rep
        sim.backward(pb, seed=wl.seed)
