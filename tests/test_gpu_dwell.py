"""GPU parity of stochastic dwell times (Section 3.1: stage transition times
drawn from discrete distributions; Section 6: stochastic progression): each
exposure of an agent on day u takes an E length and an I length drawn by
Gumbel-max with the Philox uniforms of (agent, u).  Whole runs against the
FP64 oracle -- trajectories and final per-agent stages bit-exact, gradients
against its forward-mode tangents -- on both kernel schedules, with
presymptomatic transmission, on packed populations and under hipGraph
capture; one-hot tables equal the fixed-time model bit for bit; argument
checks."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from synth import make_workload  # noqa: E402

# log weights of the E lengths 1..3 and the I lengths 1..5
DWELL = (np.log(np.array([0.2, 0.5, 0.3], np.float32)), np.log(np.array([0.1, 0.2, 0.3, 0.25, 0.15], np.float32)))
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


def graph_of(G, wl):
    return G.Graph(n_agents=wl.n_agents, src=wl.src, dst=wl.dst, w=wl.w, age=wl.pop.age, n_age=8,
                   pop_offsets=wl.pop.pop_offsets, er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight)


def assert_grads(got, want, tol=1e-4):
    scale = np.maximum(np.abs(want), 1e-3 * np.max(np.abs(want)))
    err = np.abs(got - want) / scale
    assert np.all(err <= tol), f"max scaled error {err.max():.3g}\n got {got}\nwant {want}"


def grads_vec(gr, row=0):
    return np.concatenate([[gr["dR"][row].sum().item()], gr["dS"][row].cpu().numpy(), [gr["dm"][row].item()],
                           [gr["di0"][row].item()]])


CASES = [(1, 0, 0, None), (1, 0, 1, None), (1, 1, 0, None), (0, 0, 0, None), (1, 0, 0, T_PRE)]
IDS = ["hard_st-f32-split", "hard_st-f32-tiles", "hard_st-f64", "plain-f32", "hard_st-presymptomatic"]


@pytest.mark.parametrize("mode,precision,schedule,T", CASES, ids=IDS)
def test_dwell_runs_match_oracle(G, O, mode, precision, schedule, T):
    wl = make_workload("c2", n_agents=6000, K=30)
    T = wl.T if T is None else np.asarray(T, np.float32)
    tgt = np.linspace(0.0, 0.6, wl.K)
    _say(f"dwell run N={wl.n_agents} K={wl.K} mode={mode} precision={precision} schedule={schedule} T={list(T)}")
    g = graph_of(G, wl)
    sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=mode, precision=precision, ckpt_every=7, T=T, tau_g=wl.tau_g,
                      schedule=schedule, dwell=DWELL)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    out = sim.forward(pb, seed=wl.seed, target=torch.tensor(tgt, device="cuda"))
    rec = sim.records().cpu().numpy().view(np.uint32)
    dirs = O.standard_directions(wl.K, 8) if mode != 0 else None
    omode = O.HARD_ST if mode == 1 else O.PLAIN
    ref = O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K, R=wl.R[0],
                S=wl.S[0], m=wl.m[0], i0=wl.i0[0], Z=wl.Z, T=T, mode=omode, tau_g=wl.tau_g, seed=wl.seed,
                er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight, target=tgt, directions=dirs, dwell=DWELL,
                want_stage=True)
    assert np.array_equal(out["counts"][0].cpu().numpy(), ref["counts"])
    assert ref["mismatch"] == 0
    assert np.array_equal((rec & 0xFF).astype(np.uint8), ref["stage"][-1])  # every agent's final stage
    assert float(out["loss"][0]) == pytest.approx(ref["loss"], rel=1e-10)
    if mode != 0:
        gr = sim.backward(pb, seed=wl.seed)
        assert_grads(grads_vec(gr), ref["dL"])


def test_one_hot_dwell_tables_equal_the_fixed_model(G):
    """All weight on tau_E and tau_I: the same trajectory as the run without
    tables, bit for bit, and the same gradients up to the order of their
    atomic reductions; the stochastic tables change the run."""
    wl = make_workload("c2", n_agents=6000, K=24)
    g = graph_of(G, wl)
    ninf = np.float32(-np.inf)
    onehot = (np.array([ninf, ninf, 0.0], np.float32), np.array([ninf] * 4 + [0.0], np.float32))
    tgt = torch.tensor(np.linspace(0.0, 0.5, wl.K), device="cuda")
    res = {}
    for name, dw in (("fixed", None), ("onehot", onehot), ("dwell", DWELL)):
        sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=G.HARD_ST, ckpt_every=6, tau_g=wl.tau_g, dwell=dw)
        pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
        out = sim.forward(pb, seed=wl.seed, target=tgt)
        res[name] = (out["counts"][0].cpu().numpy().copy(), grads_vec(sim.backward(pb, seed=wl.seed)))
    assert np.array_equal(res["fixed"][0], res["onehot"][0])
    assert np.allclose(res["fixed"][1], res["onehot"][1], rtol=1e-12, atol=0)
    assert not np.array_equal(res["fixed"][0], res["dwell"][0])


def test_dwell_on_packed_populations(G, O):
    """Packed populations, each with its own parameter set: each population's
    trajectory and gradients equal the oracle's run of it alone."""
    wl = make_workload("c4b", n_agents=5000, K=20, n_pops=3)
    P = wl.pop.n_pops
    tgt = np.linspace(0.0, 0.5, wl.K)
    _say(f"dwell packed populations N={wl.n_agents} pops={P}")
    g = graph_of(G, wl)
    sim = G.Simulator(g, n_sets=P, K=wl.K, Z=wl.Z, mode=G.HARD_ST, per_pop_params=True, ckpt_every=5,
                      tau_g=wl.tau_g, dwell=DWELL)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    out = sim.forward(pb, seed=wl.seed, target=torch.tensor(tgt, device="cuda"))
    gr = sim.backward(pb, seed=wl.seed)
    dirs = O.standard_directions(wl.K, 8)
    for p in range(P):
        ref = O.run_workload(wl, pop_index=p, mode=O.HARD_ST, target=tgt, directions=dirs, dwell=DWELL)
        assert np.array_equal(out["counts"][p].cpu().numpy(), ref["counts"]), p
        assert_grads(grads_vec(gr, p), ref["dL"])


def test_dwell_hip_graph_replays(G):
    wl = make_workload("c2", n_agents=6000, K=20)
    g = graph_of(G, wl)
    tgt = torch.tensor(np.linspace(0.0, 0.5, wl.K), device="cuda")
    runs = {}
    for hip_graph in (False, True):
        sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=G.HARD_ST, ckpt_every=6, tau_g=wl.tau_g, dwell=DWELL,
                          use_hip_graph=hip_graph)
        pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
        runs[hip_graph] = []
        for rep in range(3 if hip_graph else 1):
            out = sim.forward(pb, seed=wl.seed, target=tgt)
            runs[hip_graph].append((out["counts"].cpu().numpy().copy(), grads_vec(sim.backward(pb, seed=wl.seed))))
            x = torch.randn(1000, device="cuda").sum()
            torch.cuda.synchronize()
            del x
    c0, g0 = runs[False][0]
    for c, gv in runs[True]:
        assert np.array_equal(c, c0)
        assert np.allclose(gv, g0, rtol=1e-9)


def test_dwell_argument_checks(G):
    from paper_2207_09714_amd import _lib as L

    wl = make_workload("c2", n_agents=3000, K=8)
    g = graph_of(G, wl)

    def code(**kw):
        with pytest.raises(L.GabmError) as e:
            G.Simulator(g, K=wl.K, Z=wl.Z, tau_g=wl.tau_g, **kw)
        return e.value.code

    assert code(mode=G.SOFT, dwell=DWELL) == L.EUNSUPPORTED
    assert code(mode=G.HARD_ST, tau_E=9, dwell=(np.zeros(9, np.float32), DWELL[1])) == L.EINVAL
    with pytest.raises(ValueError):
        G.Simulator(g, K=wl.K, Z=wl.Z, mode=G.HARD_ST, dwell=(DWELL[0], DWELL[1][:4]))
    wb = make_workload("c3", n_agents=3000, K=8)
    gb = G.Graph(n_agents=wb.n_agents, src=wb.src, dst=wb.dst, w=wb.w, age=wb.pop.age)
    with pytest.raises(L.GabmError) as e:
        G.Simulator(gb, n_sets=2, K=wb.K, Z=wb.Z, mode=G.HARD_ST, tau_g=wb.tau_g, dwell=DWELL)
    assert e.value.code == L.EUNSUPPORTED


@pytest.mark.timeout(300)
def test_full_size_c3_with_dwell(G, O):
    """The 1M-agent, 90-day workload with drawn dwell times in the benchmark's
    launch configuration (split kernels, float32 state, straight-through mode,
    checkpoint every 10 days): daily counts, removals and every agent's final
    stage equal the oracle's."""
    wl = make_workload("c3")
    _say(f"full c3 with dwell tables N={wl.n_agents} E={wl.n_edges} K={wl.K}")
    g = G.Graph(n_agents=wl.n_agents, src=wl.src, dst=wl.dst, w=wl.w, age=wl.pop.age)
    sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=G.HARD_ST, ckpt_every=10, tau_g=wl.tau_g, dwell=DWELL)
    out = sim.forward(sim.params(wl.R, wl.S, wl.m, wl.i0), seed=wl.seed)
    counts = out["counts"][0].cpu().numpy()
    drm = out["drm"][0].cpu().numpy()
    last = (sim.records().cpu().numpy().view(np.uint32) & 0xFF).astype(np.uint8)
    del sim, g
    ref = O.run_workload(wl, mode=O.PLAIN, want_stage=True, dwell=DWELL)
    assert ref["mismatch"] == 0
    assert np.array_equal(counts, ref["counts"])
    assert np.array_equal(drm, ref["drm"])
    assert np.array_equal(last, ref["stage"][-1])


@pytest.mark.parametrize("precision,schedule", [(0, 0), (0, 1), (1, 0)], ids=["f32-split", "f32-tiles", "f64"])
def test_dwell_weight_gradients_match_oracle(G, O, precision, schedule):
    """Straight-through Gumbel-softmax gradients with respect to the dwell log
    weights (every exposure's E and I one-hots and every initial infection's I
    one-hot, through the relaxed one-hot of the same noise) against the
    oracle's forward-mode tangents along each log weight."""
    wl = make_workload("c2", n_agents=6000, K=30)
    tgt = np.linspace(0.0, 0.6, wl.K)
    _say(f"dwell weight gradients N={wl.n_agents} K={wl.K} precision={precision} schedule={schedule}")
    g = graph_of(G, wl)
    sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=G.HARD_ST, precision=precision, ckpt_every=7, tau_g=wl.tau_g,
                      schedule=schedule, dwell=DWELL)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    sim.forward(pb, seed=wl.seed, target=torch.tensor(tgt, device="cuda"))
    gr = sim.backward(pb, seed=wl.seed)
    dirs = O.dwell_directions(wl.K, 8, 3, 5)
    ref = O.run_workload(wl, mode=O.HARD_ST, target=tgt, directions=dirs, dwell=DWELL)
    want = ref["dL"][11:]
    got = np.concatenate([gr["ddwell_E"].cpu().numpy(), gr["ddwell_I"].cpu().numpy()])
    assert np.max(np.abs(want)) > 0
    assert_grads(got, want)
    assert_grads(grads_vec(gr), ref["dL"][:11])  # the other gradients are unchanged by the extra outputs


def test_dwell_weight_gradients_on_packed_populations(G, O):
    """One table for all populations: its gradient is the sum of each
    population's oracle tangents."""
    wl = make_workload("c4b", n_agents=5000, K=20, n_pops=3)
    P = wl.pop.n_pops
    tgt = np.linspace(0.0, 0.5, wl.K)
    g = graph_of(G, wl)
    sim = G.Simulator(g, n_sets=P, K=wl.K, Z=wl.Z, mode=G.HARD_ST, per_pop_params=True, ckpt_every=5,
                      tau_g=wl.tau_g, dwell=DWELL)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    sim.forward(pb, seed=wl.seed, target=torch.tensor(tgt, device="cuda"))
    gr = sim.backward(pb, seed=wl.seed)
    dirs = O.dwell_directions(wl.K, 8, 3, 5)
    want = sum(O.run_workload(wl, pop_index=p, mode=O.HARD_ST, target=tgt, directions=dirs, dwell=DWELL)["dL"][11:]
               for p in range(P))
    got = np.concatenate([gr["ddwell_E"].cpu().numpy(), gr["ddwell_I"].cpu().numpy()])
    assert_grads(got, want)


PROFILE = np.array([0.25, 0.5, 0.75, 1.5, 1.75, 1.25, 0.75, 0.25], np.float32)


def test_dwell_with_profile_matches_oracle(G, O):
    """Drawn dwell times with an infectiousness profile over days since
    exposure and presymptomatic transmission (receiver-tile kernels): counts
    bit-exact, gradients with respect to R, S, m, i0 and the dwell log weights
    against the oracle's tangents."""
    wl = make_workload("c2", n_agents=6000, K=30)
    tgt = np.linspace(0.0, 0.6, wl.K)
    _say(f"dwell with profile N={wl.n_agents} K={wl.K}")
    g = graph_of(G, wl)
    sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=G.HARD_ST, ckpt_every=7, T=T_PRE, tau_g=wl.tau_g, dwell=DWELL,
                      iota=PROFILE)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    out = sim.forward(pb, seed=wl.seed, target=torch.tensor(tgt, device="cuda"))
    gr = sim.backward(pb, seed=wl.seed)
    ref = O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K, R=wl.R[0],
                S=wl.S[0], m=wl.m[0], i0=wl.i0[0], Z=wl.Z, T=np.asarray(T_PRE, np.float32), mode=O.HARD_ST,
                tau_g=wl.tau_g, seed=wl.seed, er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight, target=tgt,
                directions=O.dwell_directions(wl.K, 8, 3, 5), dwell=DWELL, iota=PROFILE)
    assert np.array_equal(out["counts"][0].cpu().numpy(), ref["counts"])
    assert ref["mismatch"] == 0
    assert_grads(grads_vec(gr), ref["dL"][:11])
    got = np.concatenate([gr["ddwell_E"].cpu().numpy(), gr["ddwell_I"].cpu().numpy()])
    assert_grads(got, ref["dL"][11:])
