"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bars: bit-exact for integer results (CSR, random pairs, hard decisions,
stage trajectories, daily counts); rates within 1e-5 relative (in practice
exact: both sides sum exactly representable terms in double); gradients per
component within 1e-4 * max(|g*|, 1e-3 ||g*||_inf).
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


from synth import make_workload  # noqa: E402


def graph_of(G, wl, **kw):
    return G.Graph(n_agents=wl.n_agents, src=wl.src, dst=wl.dst, w=wl.w, age=wl.pop.age, n_age=8,
                   pop_offsets=wl.pop.pop_offsets, er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight, **kw)


def run_gpu(G, wl, *, mode=None, precision=0, ckpt=0, target=None, hip_graph=False, backward=False, T=None,
            R=None, graph=None, reps=1, schedule=0):
    mode = wl.mode if mode is None else mode
    g = graph if graph is not None else graph_of(G, wl)
    per_pop = wl.per_pop_params
    sim = G.Simulator(g, n_sets=wl.n_sets, K=wl.K, Z=wl.Z, mode=mode, ckpt_every=ckpt, precision=precision,
                      use_hip_graph=hip_graph, T=wl.T if T is None else T, tau_g=wl.tau_g, per_pop_params=per_pop,
                      n_reps=reps, schedule=schedule)
    pb = sim.params(wl.R if R is None else R, wl.S, wl.m, wl.i0)
    out = sim.forward(pb, seed=wl.seed, target=None if target is None else torch.tensor(target, device="cuda"))
    res = {k: v.cpu().numpy().copy() for k, v in out.items()}
    if backward:
        gr = sim.backward(pb, seed=wl.seed)
        res.update({k: v.cpu().numpy().copy() for k, v in gr.items()})
    res["records"] = sim.records().cpu().numpy()
    res["_sim"] = sim
    return res


def grad_vector(r):
    return np.concatenate([[r["dR"][0].sum()], r["dS"][0], [r["dm"][0]], [r["di0"][0]]])


def assert_grads(got, want, tol=1e-4):
    scale = np.maximum(np.abs(want), 1e-3 * np.max(np.abs(want)))
    err = np.abs(got - want) / scale
    assert np.all(err <= tol), f"max scaled error {err.max():.3g} at {np.argmax(err)}\n got {got}\nwant {want}"


# ---------------------------------------------------------------- graph build

def test_csr_matches_coo(G):
    wl = make_workload("c3", n_agents=20000, K=5)
    _say(f"csr c3 N={wl.n_agents} E={wl.n_edges}")
    g = graph_of(G, wl)
    rp, col, w = (x.cpu().numpy() for x in g.csr())
    info = g.info()
    assert info["n_edges"] == wl.n_edges and rp[0] == 0 and rp[-1] == wl.n_edges and np.all(np.diff(rp) >= 0)
    dst = np.repeat(np.arange(wl.n_agents), np.diff(rp))
    got = np.lexsort((w.view(np.uint32), col, dst))
    want = np.lexsort((wl.w.view(np.uint32), wl.src, wl.dst))
    assert np.array_equal(dst[got], wl.dst[want]) and np.array_equal(col[got], wl.src[want])
    assert np.array_equal(w[got], wl.w[want])
    # rows sorted by (sender, weight): the lexsort above is the identity
    assert np.array_equal(got, np.arange(len(got)))
    assert info["max_degree"] == np.diff(rp).max()
    assert abs(info["weight_sum"] - wl.w.astype(np.float64).sum()) < 1e-6 * wl.w.sum()


def test_symmetrize_and_errors(G):
    from paper_2207_09714_amd import _lib as L

    _say("graph build flags and errors")
    rng = np.random.default_rng(5)
    n = 3000
    a = rng.integers(0, n, 20000)
    b = rng.integers(0, n, 20000)
    keep = a != b
    a, b = a[keep], b[keep]
    w = (rng.integers(1, 1 << 24, len(a)) * 2.0**-24).astype(np.float32)
    age = rng.integers(0, 8, n).astype(np.uint8)
    g1 = G.Graph(n_agents=n, src=a, dst=b, w=w, age=age, symmetrize=True)
    g2 = G.Graph(n_agents=n, src=np.concatenate([a, b]), dst=np.concatenate([b, a]), w=np.concatenate([w, w]), age=age)
    for x, y in zip(g1.csr(), g2.csr()):
        assert torch.equal(x, y)
    with pytest.raises(L.GabmError) as e:
        G.Graph(n_agents=n, src=a, dst=b, w=w, age=age)  # one direction only
    assert e.value.code == L.ENOTSYM
    with pytest.raises(L.GabmError) as e:
        G.Graph(n_agents=n, src=[0, 1, 1], dst=[1, 0, 1], age=age, check_symmetric=False)
    assert e.value.code == L.ERANGE
    with pytest.raises(L.GabmError) as e:
        G.Graph(n_agents=n, src=[0, n], dst=[n, 0], age=age)
    assert e.value.code == L.ERANGE
    with pytest.raises(L.GabmError) as e:
        G.Graph(n_agents=n, src=[0, 1], dst=[1, 0], w=[-1.0, -1.0], age=age)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.GabmError) as e:
        G.Graph(n_agents=n, src=[0, 2000], dst=[2000, 0], age=age, pop_offsets=[0, 1000, n])
    assert e.value.code == L.ERANGE
    bad_age = age.copy()
    bad_age[7] = 9
    with pytest.raises(L.GabmError) as e:
        G.Graph(n_agents=n, src=[0, 1], dst=[1, 0], age=bad_age)
    assert e.value.code == L.ERANGE
    # run descriptions are checked on the host before any allocation
    for kw in (dict(schedule=2), dict(schedule=-1), dict(ckpt_every=-1), dict(n_reps=0)):
        with pytest.raises(L.GabmError) as e:
            G.Simulator(g1, K=4, Z=[1.0], mode=G.HARD_ST, **kw)
        assert e.value.code == L.EINVAL, kw


def test_daily_random_pairs_bit_exact(G, O):
    wl = make_workload("c4b", n_agents=3000, K=4, n_pops=3)
    _say("daily random pairs")
    g = G.Graph(n_agents=wl.n_agents, src=wl.src, dst=wl.dst, w=wl.w, age=wl.pop.age,
                pop_offsets=wl.pop.pop_offsets, er_mean_deg=7.5, er_weight=0.5)
    offs = wl.pop.pop_offsets
    for day in (0, 3, 17):
        for p in range(3):
            a, b = G.er_daily(g, p, G.make_rng(1234, 2), day)
            ea, eb = O.er_pairs(int(offs[p + 1] - offs[p]), 7.5, 1234, day, p, 2)
            assert np.array_equal(a.cpu().numpy(), ea + offs[p]) and np.array_equal(b.cpu().numpy(), eb + offs[p])


# ---------------------------------------------------------------- single steps

def test_single_steps_match_oracle(G, O):
    wl = make_workload("c1", K=12)
    _say(f"single steps c1 N={wl.n_agents}")
    ref = O.run_workload(wl, mode=O.HARD_ST, want_agents=True, want_stage=True)
    g = graph_of(G, wl)
    pb = G.ParamBlock(R=wl.R, S=wl.S, m=wl.m, i0=wl.i0, Z=wl.Z, K=wl.K, n_sets=1, mode=G.HARD_ST, tau_g=wl.tau_g)
    rng = G.make_rng(wl.seed)
    N = wl.n_agents
    A = torch.zeros(N, dtype=torch.float64, device="cuda")
    lam = torch.zeros_like(A)
    h = torch.zeros(N, dtype=torch.uint8, device="cuda")
    y = torch.zeros_like(A)
    dydl = torch.zeros_like(A)
    for t in (0, 4, 9):
        rec = torch.tensor(ref["stage"][t].astype(np.int32), device="cuda")  # timers irrelevant to the rate
        G.transmit_fwd(g, rec, 0, pb, 0, rng, t, A, lam)
        G.sample_infect(g, lam, pb, rng, t, h, y, dydl)
        torch.cuda.synchronize()
        assert np.array_equal(A.cpu().numpy(), ref["A"][t])
        lg, lr = lam.cpu().numpy(), ref["lam"][t]
        assert np.all(np.abs(lg - lr) <= 1e-15 * np.abs(lr))
        assert np.array_equal(h.cpu().numpy(), ref["h"][t])
        assert np.allclose(y.cpu().numpy(), ref["y"][t], rtol=1e-12, atol=1e-300)
        # float32 and float64 infectiousness vectors give the same sums
        inf = torch.tensor((ref["stage"][t] == 2).astype(np.float32), device="cuda")
        A2 = torch.zeros_like(A)
        G.transmit_fwd(g, inf, 1, pb, 0, rng, t, A2)
        G.transmit_fwd(g, inf.double(), 2, pb, 0, rng, t, A)
        assert torch.equal(A, A2) and np.array_equal(A.cpu().numpy(), ref["A"][t])
        # one bit per agent (the workload has T[E] = 0)
        by = np.packbits(ref["stage"][t] == 2, bitorder="little")
        words = np.zeros(((N + 63) // 64) * 8, np.uint8)
        words[: len(by)] = by
        bits = torch.tensor(words.view(np.int64), device="cuda")
        A2.zero_()
        G.transmit_fwd(g, bits, 3, pb, 0, rng, t, A2)
        assert torch.equal(A, A2)

    # adjoint of the neighbour sum: a gather over the transpose (dense check)
    gv = torch.tensor(np.random.default_rng(1).standard_normal(N), device="cuda")
    ib = torch.zeros_like(gv)
    G.transmit_bwd(g, gv, rng, 3, ib)
    a_er, b_er = O.er_pairs(N, wl.er_mean_deg, wl.seed, 3)
    want = np.zeros(N)
    gn = gv.cpu().numpy()
    np.add.at(want, wl.src, wl.w.astype(np.float64) * gn[wl.dst])
    np.add.at(want, a_er, 0.5 * gn[b_er])
    np.add.at(want, b_er, 0.5 * gn[a_er])
    torch.cuda.synchronize()
    assert np.allclose(ib.cpu().numpy(), want, rtol=1e-12, atol=1e-12)

    # parameter reduction of one day
    lb = torch.tensor(np.random.default_rng(2).standard_normal(N), device="cuda")
    At = torch.tensor(ref["A"][5], device="cuda")
    dR = torch.zeros(1, dtype=torch.float64, device="cuda")
    dS = torch.zeros(8, dtype=torch.float64, device="cuda")
    G.param_grad_reduce(g, lb, At, pb, 0, 5, dR, dS)
    lbn = lb.cpu().numpy()
    Sa = wl.S[0].astype(np.float64)[wl.pop.age]
    Z = float(wl.Z[0])
    assert np.isclose(dR.item(), np.sum(lbn * Sa * ref["A"][5] / Z), rtol=1e-12)
    wantS = np.bincount(wl.pop.age, lbn * float(wl.R[0, 5]) * ref["A"][5] / Z, minlength=8)
    assert np.allclose(dS.cpu().numpy(), wantS, rtol=1e-12, atol=1e-14)

    # progress from the oracle's records of day t: next stages equal
    rec = run_gpu(G, wl, mode=G.HARD_ST)["records"]
    assert np.array_equal(rec & 0xFF, ref["stage"][-1])


# ---------------------------------------------------------------- whole forward runs

CASES = [
    ("c1", dict(), dict(mode=0, precision=1)),
    ("c1", dict(), dict(mode=0, precision=0)),
    ("c2", dict(n_agents=8000, K=30), dict(mode=1, ckpt=7)),
    ("c3", dict(n_agents=30000, K=40), dict(mode=1, ckpt=10)),
    ("c3", dict(n_agents=30000, K=40), dict(mode=1, T=(0, 0.4, 1, 0, 0))),
    ("c4b", dict(n_agents=6000, K=25, n_pops=5), dict(mode=1)),
]


@pytest.mark.parametrize("name,wkw,rkw", CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(CASES)])
def test_forward_trajectory_bit_exact(G, O, name, wkw, rkw):
    wl = make_workload(name, **wkw)
    _say(f"forward {name} {wkw} {rkw}")
    T = rkw.get("T")
    r = run_gpu(G, wl, **rkw)
    if wl.per_pop_params:
        for p in range(wl.pop.n_pops):
            ref = O.run_workload(wl, pop_index=p, mode=rkw["mode"], want_stage=True)
            assert np.array_equal(r["counts"][p], ref["counts"]), p
            assert np.array_equal(r["drm"][p], ref["drm"])
            lo, hi = wl.pop.pop_offsets[p], wl.pop.pop_offsets[p + 1]
            assert np.array_equal(r["records"][lo:hi] & 0xFF, ref["stage"][-1])
        return
    kw = {} if T is None else {}
    ref = O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K, R=wl.R[0],
                S=wl.S[0], m=wl.m[0], i0=wl.i0[0], Z=wl.Z, T=wl.T if T is None else T, mode=rkw["mode"],
                tau_g=wl.tau_g, er_mean_deg=wl.er_mean_deg, er_weight=wl.er_weight, want_stage=True, **kw)
    assert np.array_equal(r["counts"][0], ref["counts"])
    assert np.array_equal(r["drm"][0], ref["drm"])
    assert np.array_equal(r["deaths"][0], ref["deaths"])
    st = r["records"] & 0xFF
    assert np.array_equal(st, ref["stage"][-1])


def test_packed_populations_gradients(G, O):
    """Packed populations, each with its own parameter set, on the split
    kernels (blocks of agents that straddle two populations count and reduce
    per agent): each population's trajectory and gradients equal the oracle's
    run of that population alone, and the tile kernels agree."""
    wl = make_workload("c4b", n_agents=5000, K=16, n_pops=4)
    _say(f"packed populations N={wl.n_agents} pops={wl.pop.n_pops} offsets={list(wl.pop.pop_offsets)}")
    assert any(int(o) % 256 for o in wl.pop.pop_offsets[1:-1])
    tgt = np.linspace(0.0, 0.5, wl.K)
    fast = run_gpu(G, wl, mode=1, ckpt=5, target=tgt, backward=True, schedule=0)
    tile = run_gpu(G, wl, mode=1, ckpt=5, target=tgt, backward=True, schedule=1)
    assert np.array_equal(fast["counts"], tile["counts"]) and np.array_equal(fast["records"], tile["records"])
    for k in ("dR", "dS", "dm", "di0"):
        assert np.allclose(fast[k], tile[k], rtol=1e-6, atol=1e-9 * np.abs(tile[k]).max()), k
    dirs = O.standard_directions(wl.K, 8)
    for p in range(wl.pop.n_pops):
        ref = O.run_workload(wl, pop_index=p, mode=O.HARD_ST, target=tgt, directions=dirs)
        assert np.array_equal(fast["counts"][p], ref["counts"]), p
        got = np.concatenate([[fast["dR"][p].sum()], fast["dS"][p], [fast["dm"][p]], [fast["di0"][p]]])
        assert_grads(got, ref["dL"])


@pytest.mark.parametrize("name,wkw", [("c3", dict(n_agents=40000, K=30)), ("c2", dict(n_agents=6000, K=20))])
def test_persistent_and_tile_kernels_agree(G, O, name, wkw):
    """The persistent LDS-mask kernels and the receiver-tile kernels give the
    same trajectory (bit-exact) and the same gradients."""
    wl = make_workload(name, **wkw)
    tgt = np.linspace(0.0, 1.0, wl.K)
    _say(f"persistent vs tile {name} {wkw}")
    fast = run_gpu(G, wl, mode=1, ckpt=6, target=tgt, backward=True, schedule=0)
    tile = run_gpu(G, wl, mode=1, ckpt=6, target=tgt, backward=True, schedule=1)
    assert np.array_equal(fast["counts"], tile["counts"]) and np.array_equal(fast["records"], tile["records"])
    for k in ("dR", "dS", "dm", "di0"):
        assert np.allclose(fast[k], tile[k], rtol=1e-6, atol=1e-9 * np.abs(tile[k]).max()), k
    ref = O.run_workload(wl, mode=O.HARD_ST, target=tgt, directions=O.standard_directions(wl.K, 8))
    assert np.array_equal(fast["counts"][0], ref["counts"])
    assert_grads(grad_vector(fast), ref["dL"])


def test_sender_slices_match_oracle_and_tile_kernels(G, O):
    """Above 2^20 agents the split kernels read the contact list cut into
    sender slices of 2^20 agents (one LDS mask each) and add the slices'
    partial sums per receiver: 1.3M agents give two slices.  Trajectory equal
    to the oracle's; trajectory and gradients equal to the tile kernels',
    which read the whole CSR in one pass."""
    wl = make_workload("c3", n_agents=1_300_000, K=16)
    _say(f"sender slices c3 N={wl.n_agents} E={wl.n_edges} K={wl.K}")
    g = graph_of(G, wl)
    info = g.info()
    assert info["n_sender_slices"] == 2
    assert info["n_stream_chunks"] >= (wl.n_edges + 255) // 256
    tgt = np.linspace(0.0, 2.0, wl.K)
    fast = run_gpu(G, wl, mode=1, ckpt=5, target=tgt, backward=True, graph=g, schedule=0)
    tile = run_gpu(G, wl, mode=1, ckpt=5, target=tgt, backward=True, graph=g, schedule=1)
    assert np.array_equal(fast["counts"], tile["counts"]) and np.array_equal(fast["records"], tile["records"])
    for k in ("dR", "dS", "dm", "di0"):
        assert np.allclose(fast[k], tile[k], rtol=1e-6, atol=1e-9 * np.abs(tile[k]).max()), k
    ref = O.run_workload(wl, mode=O.PLAIN, target=tgt)
    assert np.array_equal(fast["counts"][0], ref["counts"])
    assert np.array_equal(fast["drm"][0], ref["drm"])
    assert fast["loss"][0] == pytest.approx(ref["loss"], rel=1e-12)


def test_packed_populations_across_sender_slices(G, O):
    """1.6M agents in 4 packed populations: two sender slices, one population
    across the slice border, and runs of hundreds of thousands of rows that are
    empty within a slice (kept below 256 per row-start byte by zero-weight
    contacts).  Each population's trajectory equals the oracle's; the split
    and tile kernels agree on trajectories and gradients."""
    wl = make_workload("c4b", n_agents=800_000, K=8, n_pops=4)
    offs = [int(o) for o in wl.pop.pop_offsets]
    _say(f"packed populations across slices N={wl.n_agents} offsets={offs}")
    assert any(a < (1 << 20) < b for a, b in zip(offs[:-1], offs[1:]))
    g = graph_of(G, wl)
    assert g.info()["n_sender_slices"] == 2
    tgt = np.linspace(0.0, 1.0, wl.K)
    fast = run_gpu(G, wl, mode=1, ckpt=3, target=tgt, backward=True, graph=g, schedule=0)
    tile = run_gpu(G, wl, mode=1, ckpt=3, target=tgt, backward=True, graph=g, schedule=1)
    assert np.array_equal(fast["counts"], tile["counts"]) and np.array_equal(fast["records"], tile["records"])
    for k in ("dR", "dS", "dm", "di0"):
        assert np.allclose(fast[k], tile[k], rtol=1e-6, atol=1e-9 * np.abs(tile[k]).max()), k
    for p in range(wl.pop.n_pops):
        ref = O.run_workload(wl, pop_index=p, mode=O.PLAIN, target=tgt)
        assert np.array_equal(fast["counts"][p], ref["counts"]), p
        assert fast["loss"][p] == pytest.approx(ref["loss"], rel=1e-12), p


@pytest.mark.parametrize("n", [(1 << 20), (1 << 20) + 1])
def test_sender_slice_boundaries(G, O, n):
    """Households only (sparse rows, many of them empty within a slice) on
    exactly 2^20 agents (one slice) and 2^20 + 1 (a second slice holding one
    agent's contacts): trajectories equal the oracle's, gradients equal the
    tile kernels'."""
    from synth.graphs import households, quantized_unit_weights, to_symmetric_coo

    rng = np.random.default_rng(n)
    ha, hb = households(n, rng)
    src, dst, w = to_symmetric_coo([(ha, hb, quantized_unit_weights(rng, len(ha)))])
    age = (np.arange(n) % 8).astype(np.uint8)
    K = 8
    Z = np.float32(5.0 * float(np.sum(w, dtype=np.float64)) / n)
    S = np.linspace(0.5, 1, 8).astype(np.float32)
    g = G.Graph(n_agents=n, src=src, dst=dst, w=w, age=age)
    assert g.info()["n_sender_slices"] == (1 if n == (1 << 20) else 2)
    tgt = torch.tensor(np.linspace(0.0, 50.0, K), device="cuda")
    res = {}
    for sched in (0, 1):
        sim = G.Simulator(g, K=K, Z=[Z], mode=G.HARD_ST, ckpt_every=3, schedule=sched)
        pb = sim.params(np.full(K, 4.0, np.float32), S, [0.05], [0.05])
        out = sim.forward(pb, seed=5, target=tgt)
        r = {k: v.cpu().numpy().copy() for k, v in out.items()}
        r.update({k: v.cpu().numpy().copy() for k, v in sim.backward(pb, seed=5).items()})
        res[sched] = r
    ref = O.run(age=age, pop_offsets=[0, n], src=src, dst=dst, w=w, K=K, R=4.0, S=S, m=0.05, i0=0.05, Z=Z,
                mode=O.PLAIN, seed=5, target=tgt.cpu().numpy())
    assert np.array_equal(res[0]["counts"][0], ref["counts"])
    assert np.array_equal(res[1]["counts"][0], ref["counts"])
    for k in ("dR", "dS", "dm", "di0"):
        assert np.allclose(res[0][k], res[1][k], rtol=1e-6, atol=1e-9 * np.abs(res[1][k]).max()), k


def test_long_rows_and_edge_cases(G, O):
    _say("long rows / edge cases")
    # a hub with 6000 contacts (longer than one tile) plus a household layer
    n = 9000
    hub = np.zeros(6000, np.int64)
    leaves = np.arange(1, 6001)
    from synth.graphs import households, to_symmetric_coo
    ha, hb = households(n, np.random.default_rng(0))
    src, dst, w = to_symmetric_coo([(hub, leaves, 0.25), (ha, hb, 1.0)])
    age = (np.arange(n) % 8).astype(np.uint8)
    Z = np.float32(20.0)
    S = np.linspace(0.5, 1, 8).astype(np.float32)
    g = G.Graph(n_agents=n, src=src, dst=dst, w=w, age=age)
    assert g.info()["n_long_rows"] >= 1
    K = 15
    ref = O.run(age=age, pop_offsets=[0, n], src=src, dst=dst, w=w, K=K, R=3.0, S=S, m=0.05, i0=0.05, Z=Z,
                mode=O.HARD_ST, seed=3)
    for sched in (0, 1):
        sim = G.Simulator(g, K=K, Z=Z, mode=G.HARD_ST, schedule=sched)
        pb = sim.params(np.full(K, 3.0, np.float32), S, [0.05], [0.05])
        out = sim.forward(pb, seed=3)
        assert np.array_equal(out["counts"][0].cpu().numpy(), ref["counts"]), sched
    # a single agent with no contacts; and everyone infected
    g1 = G.Graph(n_agents=1, src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32), age=[3])
    s1 = G.Simulator(g1, K=3, Z=[1.0], mode=G.PLAIN)
    o1 = s1.forward(s1.params(np.ones(3, np.float32), S, [0.5], [0.999999]), seed=1)
    r1 = O.run(age=[3], pop_offsets=[0, 1], src=[], dst=[], w=[], K=3, R=1.0, S=S, m=0.5, i0=0.999999, Z=1.0, seed=1)
    assert np.array_equal(o1["counts"][0].cpu().numpy(), r1["counts"])


def test_full_size_c3_forward_bit_exact(G, O):
    """The 1M-agent, 90-day workload in the launch configuration the benchmark
    times (float32 state, straight-through mode, checkpoint every 10 days,
    day loop captured in a hipGraph): daily counts and final stages equal the
    oracle's."""
    wl = make_workload("c3")
    _say(f"full c3 N={wl.n_agents} E={wl.n_edges} K={wl.K}")
    r = run_gpu(G, wl, mode=1, ckpt=10, hip_graph=True)
    ref = O.run_workload(wl, mode=O.PLAIN, want_stage=False)
    assert np.array_equal(r["counts"][0], ref["counts"])
    assert np.array_equal(r["drm"][0], ref["drm"])


def _golden():
    import importlib.util
    import os

    fn = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_targets.py")
    spec = importlib.util.spec_from_file_location("gabm_golden", fn)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.timeout(420)
def test_full_size_c5(G):
    """The largest workload (8M agents, about 344M directed contacts per day,
    120 days, checkpoint every 15 days) in the launch configuration of a
    benchmark run: float32 state, straight-through gradients, day loops
    captured in hipGraphs.  The oracle needs minutes for this run, so its
    result is read from the record tests/golden/make_targets.py --run wrote:

    * daily stage counts and removals equal the oracle's, and so does the
      FP64 loss;
    * the mortality gradient equals its closed form (2/K) sum_t (D^t - y^t)
      drm^t (m reaches the loss only through D = m drm in this mode);
    * the R and S gradients satisfy sum_t R^t dL/dR^t = sum_a S_a dL/dS_a,
      since every rate depends on them only through the products R^t S_a."""
    gold = _golden()
    ref = gold.read_run("c5")
    wl = make_workload("c5")
    _say(f"full c5 N={wl.n_agents} E={wl.n_edges} K={wl.K}")
    tgt = gold.read_target("c5")[: wl.K]
    r = run_gpu(G, wl, mode=1, ckpt=15, target=tgt, backward=True, hip_graph=True)
    assert np.array_equal(r["counts"][0], ref["counts"])
    assert np.array_equal(r["drm"][0], ref["drm"])
    assert r["loss"][0] == pytest.approx(ref["loss"], rel=1e-12)
    m = float(np.float32(wl.m[0]))
    D = m * ref["drm"]
    dm = 2.0 / wl.K * np.sum((D - tgt) * ref["drm"])
    assert r["dm"][0] == pytest.approx(dm, rel=1e-12)
    R = wl.R[0].astype(np.float64)
    S = wl.S[0].astype(np.float64)
    lhs, rhs = np.sum(R * r["dR"][0]), np.sum(S * r["dS"][0])
    mag = np.sum(np.abs(R * r["dR"][0])) + np.sum(np.abs(S * r["dS"][0]))
    assert np.all(np.isfinite(r["dR"][0])) and np.all(np.isfinite(r["dS"][0])) and np.isfinite(r["di0"][0])
    assert abs(lhs - rhs) <= 1e-5 * mag, (lhs, rhs, mag)


@pytest.mark.timeout(420)
def test_full_size_c4b_sampled(G, O):
    """The full packed workload (24 populations, 2.48M agents, 94M contacts
    per day, 45 days, a parameter set per population, every day kept) in the
    benchmark's launch configuration.  The smallest, a middle and the largest
    population equal the oracle's run of that population alone (daily counts,
    removals, loss); every population's dL/dm equals its closed form and its
    R and S gradients satisfy the homogeneity identity."""
    wl = make_workload("c4b")
    sizes = np.diff(wl.pop.pop_offsets)
    _say(f"full c4b N={wl.n_agents} E={wl.n_edges} K={wl.K} pops={wl.pop.n_pops}")
    tgt = np.linspace(0.0, 20.0, wl.K)
    r = run_gpu(G, wl, mode=1, ckpt=wl.ckpt_every, target=tgt, backward=True)
    order = np.argsort(sizes)
    for p in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        ref = O.run_workload(wl, pop_index=p, mode=O.PLAIN, target=tgt)
        assert np.array_equal(r["counts"][p], ref["counts"]), p
        assert np.array_equal(r["drm"][p], ref["drm"]), p
        assert r["loss"][p] == pytest.approx(ref["loss"], rel=1e-12), p
    for p in range(wl.pop.n_pops):
        m = float(np.float32(wl.m[p]))
        dm = 2.0 / wl.K * np.sum((m * r["drm"][p] - tgt) * r["drm"][p])
        assert r["dm"][p] == pytest.approx(dm, rel=1e-12), p
        R = wl.R[p].astype(np.float64)
        S = wl.S[p].astype(np.float64)
        lhs, rhs = np.sum(R * r["dR"][p]), np.sum(S * r["dS"][p])
        mag = np.sum(np.abs(R * r["dR"][p])) + np.sum(np.abs(S * r["dS"][p]))
        assert abs(lhs - rhs) <= 1e-5 * mag, (p, lhs, rhs, mag)


@pytest.mark.timeout(300)
def test_full_size_c2(G, O):
    """The full 100k-agent workload with its daily random layer (60 days,
    checkpoint every 10 days, the stored target), eager and with each run
    captured in a hipGraph: trajectory equal to the oracle's, gradients equal
    to the oracle's forward-mode tangents."""
    gold = _golden()
    wl = make_workload("c2")
    tgt = gold.read_target("c2")[: wl.K]
    ref = O.run_workload(wl, mode=O.HARD_ST, target=tgt, directions=O.standard_directions(wl.K, 8))
    for hip_graph in (False, True):
        _say(f"full c2 N={wl.n_agents} E={wl.n_edges} K={wl.K} hip_graph={hip_graph}")
        r = run_gpu(G, wl, mode=1, ckpt=10, target=tgt, backward=True, hip_graph=hip_graph)
        assert np.array_equal(r["counts"][0], ref["counts"]), hip_graph
        assert np.array_equal(r["drm"][0], ref["drm"]), hip_graph
        assert r["loss"][0] == pytest.approx(ref["loss"], rel=1e-12)
        assert_grads(grad_vector(r), ref["dL"])


# ---------------------------------------------------------------- gradients

@pytest.fixture(scope="module")
def grad_case():
    wl = make_workload("c2", n_agents=5000, K=24)
    tgt = np.linspace(0.0, 0.6, wl.K)
    return wl, tgt


def test_relaxed_gradients_match_central_differences(G):
    """In the relaxed mode (every sample a binary-concrete value, so the loss
    is smooth in the parameters) with double-precision state, the adjoint
    gradients of the deaths loss with respect to R on one day, the
    susceptibility of one age group, the mortality rate and the initial
    infected fraction equal central differences of the library's own loss at
    the same Philox seed (households, workplaces and the daily random layer)."""
    wl = make_workload("c2", n_agents=3000, K=20)
    _say(f"relaxed gradients vs central differences N={wl.n_agents} K={wl.K}")
    g = graph_of(G, wl)
    t = torch.tensor(np.linspace(0.0, 0.3, wl.K), device="cuda")
    sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=G.SOFT, precision=G.F64, ckpt_every=5, tau_g=wl.tau_g)
    base = dict(R=wl.R.astype(np.float32).copy(), S=wl.S.astype(np.float32).copy(),
                m=wl.m.astype(np.float32).copy(), i0=wl.i0.astype(np.float32).copy())

    def loss(p):
        out = sim.forward(sim.params(p["R"], p["S"], p["m"], p["i0"]), seed=wl.seed, target=t)
        return float(out["loss"][0].item())

    pb = sim.params(base["R"], base["S"], base["m"], base["i0"])
    sim.forward(pb, seed=wl.seed, target=t)
    gr = {k: v.cpu().numpy().copy() for k, v in sim.backward(pb, seed=wl.seed).items()}
    # R on day 3: infections that day can still die before the horizon
    cases = [("R", (0, 3), gr["dR"][0, 3]), ("S", (0, 3), gr["dS"][0, 3]), ("m", (0,), gr["dm"][0]),
             ("i0", (0,), gr["di0"][0])]
    got, fd = [], []
    for name, idx, adj in cases:
        x = float(base[name][idx])
        vals = []
        for sign in (1.0, -1.0):
            p = {k: v.copy() for k, v in base.items()}
            p[name][idx] = np.float32(x * (1.0 + sign * 2.0**-9))
            vals.append((loss(p), float(p[name][idx])))
        (lp, xp), (lm, xm) = vals
        got.append(adj)
        fd.append((lp - lm) / (xp - xm))
    got, fd = np.array(got), np.array(fd)
    _say(f"adjoint {got} central differences {fd}")
    assert np.all(fd != 0.0), fd
    scale = np.maximum(np.abs(fd), 1e-3 * np.max(np.abs(fd)))
    assert np.all(np.abs(got - fd) <= 1e-4 * scale), (got, fd)


@pytest.mark.parametrize("precision", [0, 1])
def test_straight_through_gradients(G, O, grad_case, precision):
    wl, tgt = grad_case
    _say(f"hard-ST gradients precision={precision}")
    r = run_gpu(G, wl, mode=1, precision=precision, ckpt=5, target=tgt, backward=True)
    ref = O.run_workload(wl, mode=O.HARD_ST, target=tgt, directions=O.standard_directions(wl.K, 8))
    assert np.array_equal(r["counts"][0], ref["counts"])
    assert abs(r["loss"][0] - ref["loss"]) <= 1e-12 * max(1.0, abs(ref["loss"]))
    assert_grads(grad_vector(r), ref["dL"])


@pytest.mark.parametrize("precision,tol", [(1, 1e-8), (0, 1e-4)])
def test_soft_gradients(G, O, grad_case, precision, tol):
    wl, tgt = grad_case
    _say(f"soft gradients precision={precision}")
    r = run_gpu(G, wl, mode=2, precision=precision, ckpt=6, target=tgt, backward=True)
    ref = O.run_workload(wl, mode=O.SOFT, target=tgt, directions=O.standard_directions(wl.K, 8))
    # relaxed counts are sums over agents of values stored in the run's precision
    atol = (1e-9 if precision == 1 else 2e-6) * wl.n_agents
    assert np.allclose(r["counts"][0], ref["counts"], rtol=10 * tol, atol=atol)
    assert abs(r["loss"][0] - ref["loss"]) <= 10 * tol * abs(ref["loss"]) + 1e-12
    assert_grads(grad_vector(r), ref["dL"], tol)


def test_per_day_reproduction_number_gradient(G, O):
    wl = make_workload("c2", n_agents=3000, K=14)
    tgt = np.linspace(0.0, 0.3, wl.K)
    _say("per-day R gradient")
    r = run_gpu(G, wl, mode=1, target=tgt, backward=True)
    K = wl.K
    dirs = (np.eye(K), np.zeros((K, 8)), np.zeros(K), np.zeros(K))
    ref = O.run_workload(wl, mode=O.HARD_ST, target=tgt, directions=dirs)
    assert_grads(r["dR"][0], ref["dL"])


def test_checkpoint_interval_does_not_change_gradients(G, grad_case):
    wl, tgt = grad_case
    _say("checkpoint invariance")
    base = grad_vector(run_gpu(G, wl, mode=1, ckpt=0, target=tgt, backward=True))
    for k in (1, 5, 7, 23):
        got = grad_vector(run_gpu(G, wl, mode=1, ckpt=k, target=tgt, backward=True))
        assert np.allclose(got, base, rtol=1e-9, atol=1e-12 * np.abs(base).max()), k


def test_hip_graph_replays_match_eager(G, grad_case):
    wl, tgt = grad_case
    _say("hipGraph replays")
    eager = run_gpu(G, wl, mode=1, ckpt=5, target=tgt, backward=True)
    g = graph_of(G, wl)
    sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=1, ckpt_every=5, use_hip_graph=True, tau_g=wl.tau_g)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    t = torch.tensor(tgt, device="cuda")
    for rep in range(3):
        out = sim.forward(pb, seed=wl.seed, target=t)
        assert np.array_equal(out["counts"].cpu().numpy(), eager["counts"]), rep
        gr = sim.backward(pb, seed=wl.seed)
        gv = np.concatenate([[gr["dR"][0].sum().item()], gr["dS"][0].cpu().numpy(), gr["dm"].cpu().numpy(),
                             gr["di0"].cpu().numpy()])
        assert np.allclose(gv, grad_vector(eager), rtol=1e-9), rep
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        del x


def test_kernel_timing_counts_every_launch(G, grad_case):
    wl, tgt = grad_case
    hip_graph = False
    _say("kernel timing of eager launches")
    g = graph_of(G, wl)
    sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=1, ckpt_every=6, use_hip_graph=hip_graph, time_kernels=True,
                      tau_g=wl.tau_g)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    t = torch.tensor(tgt, device="cuda")
    ref = None
    for rep in range(2):
        sim.kernel_times(reset=True)
        out = sim.forward(pb, seed=wl.seed, target=t)
        sim.backward(pb, seed=wl.seed)
        kt = sim.kernel_times(reset=True)
        fwd = sum(v["launches"] for k, v in kt.items() if k in ("gather_fwd", "day_fwd"))
        bwd = sum(v["launches"] for k, v in kt.items() if k in ("agent_bwd", "day_bwd"))
        # K forward days, the replay of all segments but the last, K + 1 reverse steps
        n_seg = (wl.K + 5) // 6
        assert fwd == wl.K + (n_seg - 1) * 6, kt
        assert bwd == wl.K + 1, kt
        assert all(v["ms"] > 0 for v in kt.values() if v["launches"]), kt
        counts = out["counts"].cpu().numpy().copy()
        if ref is None:
            ref = counts
        assert np.array_equal(counts, ref)


def test_autograd_function_and_deaths_adjoint(G, O, grad_case):
    wl, tgt = grad_case
    _say("autograd function")
    g = graph_of(G, wl)
    sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=1, ckpt_every=6, tau_g=wl.tau_g)
    R = torch.tensor(wl.R, device="cuda", requires_grad=True)
    S = torch.tensor(wl.S, device="cuda", requires_grad=True)
    m = torch.tensor(wl.m, device="cuda", requires_grad=True)
    i0 = torch.tensor(wl.i0, device="cuda", requires_grad=True)
    c = torch.linspace(-1, 2, wl.K, device="cuda", dtype=torch.float64)
    loss, deaths = G.GabmSim.apply(R, S, m, i0, sim, wl.seed, torch.tensor(tgt, device="cuda"))
    obj = 3.0 * loss.sum() + (c * deaths[0]).sum()
    obj.backward()
    ref = O.run_workload(wl, mode=O.HARD_ST, target=tgt, directions=O.standard_directions(wl.K, 8))
    want = 3.0 * ref["dL"] + ref["dD"] @ c.cpu().numpy()
    got = np.concatenate([[R.grad.sum().item()], S.grad[0].cpu().numpy(), m.grad.cpu().numpy(),
                          i0.grad.cpu().numpy()])
    assert_grads(got, want)


def test_day_level_entry_points_match_run(G, grad_case):
    wl, tgt = grad_case
    _say("day-level entry points")
    run = run_gpu(G, wl, mode=1, ckpt=0, target=tgt, backward=True)
    g = graph_of(G, wl)
    sim = G.Simulator(g, K=wl.K, Z=wl.Z, mode=1, ckpt_every=0, tau_g=wl.tau_g)
    pb = sim.params(wl.R, wl.S, wl.m, wl.i0)
    t = torch.tensor(tgt, device="cuda")
    for d in range(wl.K):
        sim.day_fwd(pb, d, seed=wl.seed, target=t)
    assert np.array_equal(sim.counts.cpu().numpy(), run["counts"])
    for d in range(wl.K, -1, -1):
        sim.day_bwd(pb, d, seed=wl.seed)
    got = np.concatenate([[sim.dR[0].sum().item()], sim.dS[0].cpu().numpy(), sim.dm.cpu().numpy(),
                          sim.di0.cpu().numpy()])
    assert np.allclose(got, grad_vector(run), rtol=1e-9)
    from paper_2207_09714_amd import _lib as L
    with pytest.raises(L.GabmError) as e:
        sim.day_bwd(pb, 3, seed=wl.seed)
    assert e.value.code == L.ESTATE
