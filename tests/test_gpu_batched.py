"""GPU parity of batched runs (B = n_sets x n_reps simulations on one graph).

Simulation b uses parameter set b % n_sets and the Philox stream
replicate + b // n_sets (sets of one replicate share random numbers) or
replicate + b (independent streams).  Each simulation is checked against its
own oracle run: daily counts and final stages bit for bit, the loss to
1e-12, and the per-set gradients (summed over replicates) to the same bar as
the single-simulation tests.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from synth import make_workload  # noqa: E402


def _say(msg):
    print(f"[gpu-batched] {msg}", flush=True)


@pytest.fixture(scope="module")
def G():
    from paper_2207_09714_amd import gabm

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return gabm


@pytest.fixture(scope="module")
def O():
    from oracle import oracle

    return oracle


def graph_of(G, wl):
    return G.Graph(n_agents=wl.n_agents, src=wl.src, dst=wl.dst, w=wl.w, age=wl.pop.age, n_age=8,
                   pop_offsets=wl.pop.pop_offsets, er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight)


def run_batched(G, wl, *, mode=1, ckpt=0, target=None, backward=False, T=None, indep=False, hip_graph=False,
                graph=None, replicate=0):
    g = graph if graph is not None else graph_of(G, wl)
    sim = G.Simulator(g, n_sets=wl.n_sets, n_reps=wl.n_reps, K=wl.K, Z=wl.Z, mode=mode, ckpt_every=ckpt,
                      T=wl.T if T is None else T, tau_g=wl.tau_g, use_hip_graph=hip_graph)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    tg = None if target is None else torch.tensor(target, device="cuda")
    out = sim.forward(pb, seed=wl.seed, target=tg, independent_sets=indep, replicate=replicate)
    res = {k: v.cpu().numpy().copy() for k, v in out.items()}
    if backward:
        gr = sim.backward(pb, seed=wl.seed, independent_sets=indep, replicate=replicate)
        res.update({k: v.cpu().numpy().copy() for k, v in gr.items()})
    res["records"] = sim.records().cpu().numpy().reshape(wl.n_agents, -1)
    res["_sim"], res["_pb"], res["_tg"] = sim, pb, tg
    return res


def oracle_sim(O, wl, b, *, mode, indep=False, target=None, directions=None, T=None, replicate=0):
    set_index, rep = b % wl.n_sets, b // wl.n_sets
    stream = replicate + (b if indep else rep)
    kw = {}
    if T is not None:
        kw["T"] = T
    return O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K,
                 R=wl.R[set_index], S=wl.S[set_index], m=wl.m[set_index], i0=wl.i0[set_index], Z=wl.Z,
                 tau_E=wl.tau_E, tau_I=wl.tau_I, mode=mode, tau_g=wl.tau_g, seed=wl.seed, stream=stream,
                 target=target, directions=directions, want_stage=True, **kw)


def assert_grads(got, want, tol=1e-4):
    scale = np.maximum(np.abs(want), 1e-3 * np.max(np.abs(want)))
    err = np.abs(got - want) / scale
    assert np.all(err <= tol), f"max scaled error {err.max():.3g} at {np.argmax(err)}\n got {got}\nwant {want}"


def check_forward(O, wl, r, *, mode, indep=False, sims=None, T=None, replicate=0):
    B = wl.n_sets * wl.n_reps
    for b in (range(B) if sims is None else sims):
        ref = oracle_sim(O, wl, b, mode=mode, indep=indep, T=T, replicate=replicate)
        assert np.array_equal(r["counts"][b], ref["counts"]), f"counts of simulation {b}"
        assert np.array_equal(r["drm"][b], ref["drm"]), f"removals of simulation {b}"
        final = ref["stage"].reshape(wl.K + 1, wl.n_agents)[wl.K]
        assert np.array_equal(r["records"][:, b] & 0xFF, final), f"final stages of simulation {b}"


# lane layouts: B = 6 (groups of 8 lanes), 40 (one 64-lane group, lanes idle),
# 70 (two simulations per lane) and 130 (four per lane)
@pytest.mark.parametrize("n_sets,n_reps,n_agents,K", [(3, 2, 3000, 20), (20, 2, 1500, 14), (35, 2, 1200, 12),
                                                     (65, 2, 600, 10)])
def test_batched_forward_bit_exact(G, O, n_sets, n_reps, n_agents, K):
    wl = make_workload("c4a", n_agents=n_agents, K=K, n_sets=n_sets, n_reps=n_reps)
    _say(f"forward B={n_sets * n_reps} N={wl.n_agents} E={wl.n_edges} K={K}")
    r = run_batched(G, wl, mode=1)
    B = n_sets * n_reps
    check_forward(O, wl, r, mode=O.HARD_ST, sims=sorted({0, 1, n_sets - 1, n_sets, B // 2, B - 1}))


def test_batched_plain_and_independent_streams(G, O):
    wl = make_workload("c4a", n_agents=2000, K=16, n_sets=5, n_reps=3)
    _say("plain forward, independent streams, replicate offset 7")
    r = run_batched(G, wl, mode=0, indep=True, replicate=7)
    check_forward(O, wl, r, mode=O.PLAIN, indep=True, replicate=7)
    # with common random numbers the two replicates of one set differ, sets of one replicate share draws
    r2 = run_batched(G, wl, mode=0, indep=False)
    check_forward(O, wl, r2, mode=O.PLAIN, sims=[0, 4, 5, 14])


def test_batched_presymptomatic_transmission(G, O):
    wl = make_workload("c4a", n_agents=2500, K=15, n_sets=4, n_reps=2)
    T = np.array([0, 0.5, 1, 0, 0], np.float32)
    _say("forward with T_E = 0.5")
    r = run_batched(G, wl, mode=1, T=T)
    check_forward(O, wl, r, mode=O.HARD_ST, T=T)


def test_batched_gradients_match_oracle_tangents(G, O):
    wl = make_workload("c4a", n_agents=3000, K=20, n_sets=3, n_reps=2)
    tgt = np.linspace(0.0, 0.5, wl.K)
    _say("batched straight-through gradients, checkpoint every 6 days")
    r = run_batched(G, wl, mode=1, ckpt=6, target=tgt, backward=True)
    dirs = O.standard_directions(wl.K, 8)
    want = {s: np.zeros(11) for s in range(wl.n_sets)}
    for b in range(wl.n_sets * wl.n_reps):
        ref = oracle_sim(O, wl, b, mode=O.HARD_ST, target=tgt, directions=dirs)
        assert np.array_equal(r["counts"][b], ref["counts"])
        assert abs(r["loss"][b] - ref["loss"]) <= 1e-12 * max(1.0, abs(ref["loss"]))
        want[b % wl.n_sets] += ref["dL"]
    for s in range(wl.n_sets):
        got = np.concatenate([[r["dR"][s].sum()], r["dS"][s], [r["dm"][s]], [r["di0"][s]]])
        assert_grads(got, want[s])


def test_batched_two_lanes_per_simulation_gradients(G, O):
    wl = make_workload("c4a", n_agents=1000, K=12, n_sets=36, n_reps=2)
    tgt = np.linspace(0.0, 0.2, wl.K)
    _say("batched gradients, B=72 (two simulations per lane)")
    r = run_batched(G, wl, mode=1, ckpt=4, target=tgt, backward=True)
    dirs = O.standard_directions(wl.K, 8)
    for s in (0, 17, 35):
        want = np.zeros(11)
        for rep in range(wl.n_reps):
            b = rep * wl.n_sets + s
            want += oracle_sim(O, wl, b, mode=O.HARD_ST, target=tgt, directions=dirs)["dL"]
        got = np.concatenate([[r["dR"][s].sum()], r["dS"][s], [r["dm"][s]], [r["di0"][s]]])
        assert_grads(got, want)


@pytest.mark.parametrize("n_sets,n_reps", [(8, 2), (20, 2)])
def test_batched_checkpoint_and_hip_graph_invariance(G, n_sets, n_reps):
    wl = make_workload("c4a", n_agents=4000, K=18, n_sets=n_sets, n_reps=n_reps)
    tgt = np.linspace(0.0, 0.8, wl.K)
    _say("batched checkpoint interval and hipGraph capture")
    g = graph_of(G, wl)
    a = run_batched(G, wl, mode=1, ckpt=0, target=tgt, backward=True, graph=g)
    b = run_batched(G, wl, mode=1, ckpt=5, target=tgt, backward=True, graph=g, hip_graph=True)
    assert np.array_equal(a["counts"], b["counts"])
    for k in ("dR", "dS", "dm", "di0"):
        assert np.allclose(a[k], b[k], rtol=1e-10, atol=1e-14), k
    # a second replay of the captured run
    sim, pb = b["_sim"], b["_pb"]
    sim.forward(pb, seed=wl.seed, target=b["_tg"])
    gr = sim.backward(pb, seed=wl.seed)
    assert np.array_equal(sim.counts.cpu().numpy(), a["counts"])
    assert np.allclose(gr["dR"].cpu().numpy(), a["dR"], rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("n_sets,n_reps", [(4, 2), (17, 4)])
def test_batched_day_level_entry_points(G, n_sets, n_reps):
    wl = make_workload("c4a", n_agents=2000, K=10, n_sets=n_sets, n_reps=n_reps)
    tgt = torch.tensor(np.linspace(0.0, 0.3, wl.K), device="cuda")
    _say("batched day-level entry points")
    g = graph_of(G, wl)
    ref = run_batched(G, wl, mode=1, ckpt=0, target=tgt.cpu().numpy(), backward=True, graph=g)
    sim = G.Simulator(g, n_sets=wl.n_sets, n_reps=wl.n_reps, K=wl.K, Z=wl.Z, mode=1, ckpt_every=0, T=wl.T,
                      tau_g=wl.tau_g)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    for d in range(wl.K):
        sim.day_fwd(pb, d, seed=wl.seed, target=tgt)
    assert np.array_equal(sim.counts.cpu().numpy(), ref["counts"])
    for d in range(wl.K, -1, -1):
        sim.day_bwd(pb, d, seed=wl.seed)
    assert np.allclose(sim.dR.cpu().numpy(), ref["dR"], rtol=1e-10, atol=1e-14)
    assert np.allclose(sim.dS.cpu().numpy(), ref["dS"], rtol=1e-10, atol=1e-14)


def test_batched_large_population_reads_masks_from_memory(G, O):
    # more than 2^19 agents: the 'any simulation' bits no longer fit in LDS
    wl = make_workload("c4a", n_agents=560_000, K=5, n_sets=2, n_reps=1)
    _say(f"batched forward N={wl.n_agents} E={wl.n_edges}")
    r = run_batched(G, wl, mode=1)
    check_forward(O, wl, r, mode=O.HARD_ST)


def test_batched_unsupported_shapes_fail_cleanly(G):
    wl = make_workload("c2", n_agents=2000, K=8)
    g = graph_of(G, wl)  # has a daily random layer
    with pytest.raises(G.L.GabmError, match="daily random layer"):
        G.Simulator(g, n_sets=1, n_reps=2, K=wl.K, Z=wl.Z, mode=1)
    wl2 = make_workload("c4a", n_agents=1000, K=8, n_sets=2, n_reps=1)
    g2 = graph_of(G, wl2)
    with pytest.raises(G.L.GabmError, match="hard states"):
        G.Simulator(g2, n_sets=2, K=wl2.K, Z=wl2.Z, mode=2)
    with pytest.raises(G.L.GabmError, match="at most 256"):
        G.Simulator(g2, n_sets=2, n_reps=129, K=wl2.K, Z=wl2.Z, mode=1)


def test_batched_wide_and_group_kernels_agree(G):
    # schedule 0 uses the wave-per-tile kernels for B > 32, schedule 1 the lane-group kernels
    wl = make_workload("c4a", n_agents=2500, K=14, n_sets=36, n_reps=2)
    tgt = torch.tensor(np.linspace(0.0, 0.4, wl.K), device="cuda")
    _say("wide vs lane-group batched kernels, B=72")
    g = graph_of(G, wl)
    out = []
    for schedule in (0, 1):
        sim = G.Simulator(g, n_sets=wl.n_sets, n_reps=wl.n_reps, K=wl.K, Z=wl.Z, mode=1, ckpt_every=5, T=wl.T,
                          tau_g=wl.tau_g, schedule=schedule)
        pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
        f = sim.forward(pb, seed=wl.seed, target=tgt)
        r = {k: v.cpu().numpy().copy() for k, v in f.items()}
        r.update({k: v.cpu().numpy().copy() for k, v in sim.backward(pb, seed=wl.seed).items()})
        out.append(r)
    a, b = out
    assert np.array_equal(a["counts"], b["counts"])
    assert np.array_equal(a["loss"], b["loss"])
    for k in ("dR", "dS", "dm", "di0"):
        assert np.allclose(a[k], b[k], rtol=1e-10, atol=1e-14), k


@pytest.mark.parametrize("n_sets,n_reps,name", [(1, 1, "c2"), (20, 2, "c4a")])
def test_autotune_picks_a_schedule_that_matches(G, n_sets, n_reps, name):
    if name == "c2":
        wl = make_workload("c2", n_agents=20000, K=12)
    else:
        wl = make_workload("c4a", n_agents=5000, K=12, n_sets=n_sets, n_reps=n_reps)
    _say(f"autotune {name} B={n_sets * n_reps}")
    g = graph_of(G, wl)
    best, ms = G.autotune(g, R=wl.R, S=wl.S, m=wl.m, i0=wl.i0, Z=wl.Z, K=wl.K, n_sets=n_sets, n_reps=n_reps, mode=1,
                          T=wl.T, tau_g=wl.tau_g, seed=wl.seed, days=4)
    assert best in (0, 1) and len(ms) == 2 and all(x > 0 for x in ms)
    assert ms[best] == min(ms)
    res = []
    for schedule in (0, best):
        sim = G.Simulator(g, n_sets=n_sets, n_reps=n_reps, K=wl.K, Z=wl.Z, mode=1, T=wl.T, tau_g=wl.tau_g,
                          schedule=schedule)
        pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
        res.append(sim.forward(pb, seed=wl.seed)["counts"].cpu().numpy().copy())
    assert np.array_equal(res[0], res[1])


@pytest.mark.timeout(420)
def test_full_size_c4a_sampled(G, O):
    """The full batched workload (250k agents, 9.5M contacts per day, 45 days,
    64 parameter sets x 2 replicates) in the benchmark's launch configuration
    (the autotuner's schedule, every day kept, an all-zero deaths target).
    Four simulations -- both replicates, both ends of the lane layout -- equal
    their own oracle runs bit for bit (daily counts, removals, final stages).
    Per set, dL/dm equals its closed form (2/K) sum_reps sum_t (D - y) drm, and
    sum_t R^t dL/dR^t = sum_a S_a dL/dS_a (rates depend on R and S only
    through their products)."""
    wl = make_workload("c4a")
    B = wl.n_sets * wl.n_reps
    _say(f"full c4a N={wl.n_agents} E={wl.n_edges} K={wl.K} B={B}")
    g = graph_of(G, wl)
    sched, _ = G.autotune(g, R=wl.R, S=wl.S, m=wl.m, i0=wl.i0, Z=wl.Z, K=wl.K, n_sets=wl.n_sets, n_reps=wl.n_reps,
                          mode=G.HARD_ST, ckpt_every=wl.ckpt_every, tau_g=wl.tau_g, seed=wl.seed, days=4)
    sim = G.Simulator(g, n_sets=wl.n_sets, n_reps=wl.n_reps, K=wl.K, Z=wl.Z, mode=G.HARD_ST,
                      ckpt_every=wl.ckpt_every, tau_g=wl.tau_g, schedule=sched)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    tgt = np.zeros(wl.K)
    out = sim.forward(pb, seed=wl.seed, target=torch.tensor(tgt, device="cuda"))
    r = {k: v.cpu().numpy().copy() for k, v in out.items()}
    r.update({k: v.cpu().numpy().copy() for k, v in sim.backward(pb, seed=wl.seed).items()})
    r["records"] = sim.records().cpu().numpy().reshape(wl.n_agents, -1)
    check_forward(O, wl, r, mode=O.PLAIN, sims=[0, wl.n_sets - 1, wl.n_sets, B - 1])
    for s in range(wl.n_sets):
        m = float(np.float32(wl.m[s]))
        dm = sum(2.0 / wl.K * np.sum((m * r["drm"][s + q * wl.n_sets] - tgt) * r["drm"][s + q * wl.n_sets])
                 for q in range(wl.n_reps))
        assert r["dm"][s] == pytest.approx(dm, rel=1e-12), s
        R = wl.R[s].astype(np.float64)
        S = wl.S[s].astype(np.float64)
        lhs, rhs = np.sum(R * r["dR"][s]), np.sum(S * r["dS"][s])
        mag = np.sum(np.abs(R * r["dR"][s])) + np.sum(np.abs(S * r["dS"][s]))
        assert abs(lhs - rhs) <= 1e-5 * mag, (s, lhs, rhs, mag)
