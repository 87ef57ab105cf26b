"""Pins of the FP64 oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: each check uses a published
value (Philox known answers), an exact probability computed without random
numbers (brute-force enumeration), a closed form, a large-N limit
(final-size relation, fixed-delay mean field, SEIRM ODE of Appendix D),
finite differences of the oracle's own loss (which pin its tangents), or an
invariant implied by assumptions A1-A6 (Appendix A).
"""

import os

import numpy as np
import pytest
from scipy import stats

from oracle import enumerate as EN
from oracle import meanfield as MF
from oracle import oracle as O
from synth import make_workload
from synth.graphs import complete_pairs, to_symmetric_coo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert list(O.philox(v[0:4], v[4:6])) == v[6:10]


def test_uniform_grid_and_moments():
    us = np.array([O.uniform(7, i, 3, O_TAG_INFECT, 0, 0) for i in range(20000)])
    k = us * 2**24
    assert np.all(k == np.round(k)) and np.all(np.round(k).astype(np.int64) % 2 == 1)
    assert us.min() > 0 and us.max() < 1
    # word 0 of the counter (idx, day, tag|pop<<8, stream) gives the uniform
    o = O.philox([5, 3, O_TAG_INFECT, 0], [7, 0])
    assert O.uniform(7, 5, 3, O_TAG_INFECT, 0, 0) == (2 * (int(o[0]) >> 9) + 1) / 2**24
    assert abs(us.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(us))
    assert stats.kstest(us, "uniform").pvalue > 1e-3


O_TAG_INIT, O_TAG_INFECT, O_TAG_MORT, O_TAG_ER = 0, 1, 2, 3


def test_decision_frequency_matches_q():
    # P(u < q) = q for the grid uniform, to within the grid spacing
    us = np.array([O.uniform(11, i, 0, O_TAG_INFECT) for i in range(200000)])
    for q in (0.013, 0.25, 0.5, 0.9):
        f = np.mean(us < q)
        assert abs(f - q) < 5 * np.sqrt(q * (1 - q) / len(us))


# ---------------------------------------------------------------- ER layer
def test_er_pairs_counts_and_uniformity():
    n = 1000
    a, b = O.er_pairs(n, 10.0, 123, 4)
    assert len(a) == round(n * 10 / 2)
    assert np.all(a != b) and a.min() >= 0 and b.min() >= 0 and max(a.max(), b.max()) < n
    deg = np.bincount(np.concatenate([a, b]), minlength=n)
    assert abs(deg.mean() - 10.0) < 1e-12
    # endpoint i uniform on [0,n); j uniform on the other n-1 agents
    assert stats.chisquare(np.bincount(a, minlength=n)).pvalue > 1e-4
    a2, _ = O.er_pairs(n, 10.0, 123, 5)
    assert not np.array_equal(a, a2)  # resampled each day


# ---------------------------------------------------------------- invariants
@pytest.fixture(scope="module")
def c1_run():
    wl = make_workload("c1")
    return wl, O.run_workload(wl, want_stage=True, want_agents=True)


def test_counts_conserved_and_monotone(c1_run):
    wl, r = c1_run
    c = r["counts"]
    assert np.all(c.sum(axis=1) == wl.n_agents)
    ever = wl.n_agents - c[:, 0]
    assert np.all(np.diff(ever) >= 0)
    assert np.all(np.diff(c[:, 3] + c[:, 4]) >= 0)
    assert r["mismatch"] == 0  # stage machine == exposure-window form, every agent and day


def test_stage_durations_and_no_reinfection(c1_run):
    wl, r = c1_run
    st = r["stage"]  # [K+1, N]
    K = wl.K
    for i in range(0, wl.n_agents, 7):
        s = st[:, i]
        # no agent leaves R or M, and no agent returns to S
        rm = np.nonzero(s >= 3)[0]
        if len(rm):
            assert np.all(s[rm[0]:] == s[rm[0]])
        ns = np.nonzero(s != 0)[0]
        if len(ns):
            assert np.all(s[ns[0]:] != 0)
        e_days = np.nonzero(s == 1)[0]
        i_days = np.nonzero(s == 2)[0]
        if len(e_days) and e_days[0] > 0 and e_days[0] + 3 + 5 <= K:
            assert len(e_days) == 3 and len(i_days) == 5
            assert np.all(np.diff(e_days) == 1) and i_days[0] == e_days[-1] + 1


def test_infections_only_for_susceptibles(c1_run):
    wl, r = c1_run
    st = r["stage"]
    h = r["h"]
    new_e = (st[1:] == 1) & (st[:-1] == 0)
    assert np.array_equal(new_e, (h == 1) & (st[:-1] == 0))


def test_r_zero_and_no_infectious_mean_nothing_happens():
    wl = make_workload("c1", K=15)
    r = O.run_workload(wl, R=np.zeros(wl.K, np.float32), want_agents=True)
    assert np.all(r["lam"] == 0.0)
    assert np.all(r["counts"][1:, 1] == 0)  # no exposures ever
    r2 = O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K, R=2.5,
               S=wl.S[0], m=0.01, i0=0.0, Z=wl.Z, er_mean_deg=10, er_weight=0.5, want_agents=True)
    assert np.all(r2["A"] == 0.0) and np.all(r2["counts"][:, 0] == wl.n_agents)


# ---------------------------------------------------------------- closed forms for the rate
def _forced_initial(n, want_infected, seed_range=range(5000), i0=0.5):
    """Find a seed whose initial Bernoulli(i0) draws infect exactly the given set."""
    for s in seed_range:
        u = np.array([O.uniform(s, i, 0xFFFFFFFF, O_TAG_INIT) for i in range(n)])
        if np.array_equal(u < np.float32(i0), np.asarray(want_infected, bool)):
            return s
    raise RuntimeError("no seed found")


def test_star_rate_closed_form():
    # centre 0 with 4 leaves; leaves 1..3 infectious, leaf 4 not
    n = 5
    pairs = (np.array([0, 0, 0, 0]), np.array([1, 2, 3, 4]))
    wts = np.array([0.25, 0.5, 0.75, 1.0], np.float32)
    src, dst, w = to_symmetric_coo([(pairs[0], pairs[1], wts)])
    seed = _forced_initial(n, [0, 1, 1, 1, 0])
    age = np.array([3, 0, 1, 2, 5], np.uint8)
    S = np.linspace(0.3, 1.0, 8).astype(np.float32)
    R, Z, TI = np.float32(2.0), np.float32(7.5), np.float32(0.75)
    r = O.run(age=age, pop_offsets=[0, n], src=src, dst=dst, w=w, K=1, R=R, S=S, m=0.1, i0=0.5, Z=Z,
              T=[0, 0, TI, 0, 0], seed=seed, want_agents=True)
    lam = r["lam"][0]
    # centre: sum of infectious leaf weights, receiver's susceptibility
    expect_c = float(R) * float(S[3]) * (0.25 + 0.5 + 0.75) * float(TI) / float(Z)
    assert lam[0] == pytest.approx(expect_c, rel=1e-15)
    # leaves see only the centre, which is susceptible: zero rate
    assert np.all(lam[1:] == 0.0)
    # linear in R, exactly zero at R = 0
    r2 = O.run(age=age, pop_offsets=[0, n], src=src, dst=dst, w=w, K=1, R=2 * R, S=S, m=0.1, i0=0.5, Z=Z,
               T=[0, 0, TI, 0, 0], seed=seed, want_agents=True)
    assert r2["lam"][0][0] == pytest.approx(2 * expect_c, rel=1e-15)


def test_edge_order_does_not_matter():
    wl = make_workload("c3", n_agents=3000, K=12)
    perm = np.random.default_rng(3).permutation(wl.n_edges)
    r1 = O.run_workload(wl, want_agents=True)
    r2 = O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src[perm], dst=wl.dst[perm], w=wl.w[perm],
               K=wl.K, R=wl.R[0], S=wl.S[0], m=wl.m[0], i0=wl.i0[0], Z=wl.Z, want_agents=True)
    # weights lie on the 2^-24 grid, so the double sums are exact in any order
    assert np.array_equal(r1["A"], r2["A"]) and np.array_equal(r1["counts"], r2["counts"])


# ---------------------------------------------------------------- brute force
TINY = {
    "pair": (2, [(0, 1, 1.0)]),
    "path4": (4, [(0, 1, 1.0), (1, 2, 0.5), (2, 3, 1.0)]),
    "star5": (5, [(0, 1, 1.0), (0, 2, 1.0), (0, 3, 0.5), (0, 4, 0.25)]),
    "tri_pendant": (4, [(0, 1, 1.0), (1, 2, 1.0), (0, 2, 0.75), (2, 3, 1.0)]),
    "k4": (4, [(a, b, 1.0) for a in range(4) for b in range(a + 1, 4)]),
}


@pytest.mark.parametrize("name", sorted(TINY))
def test_monte_carlo_matches_exact_distribution(name):
    n, und = TINY[name]
    a = np.array([e[0] for e in und])
    b = np.array([e[1] for e in und])
    wts = np.array([e[2] for e in und], np.float32)
    src, dst, w = to_symmetric_coo([(a, b, wts)])
    age = (np.arange(n) * 3 % 8).astype(np.uint8)
    S = np.linspace(0.4, 1.0, 8).astype(np.float32)
    R, Z, m, i0 = np.float32(3.0), np.float32(2.0), np.float32(0.3), np.float32(0.3)
    T = np.array([0, 0.5, 1, 0, 0], np.float32)  # presymptomatic transmission too
    tE, tI, K = 1, 2, 9
    edges = [(int(s), int(d), float(x)) for s, d, x in zip(src, dst, w)]
    final, exp_drm, _ = EN.exact_distribution(n, edges, age, [float(R)] * K, [float(x) for x in S],
                                              [float(x) for x in T], float(m), float(i0), float(Z), tE, tI, K)
    reps = 12000
    obs = {}
    drm = np.zeros((reps, K))
    for s in range(reps):
        r = O.run(age=age, pop_offsets=[0, n], src=src, dst=dst, w=w, K=K, R=R, S=S, m=m, i0=i0, Z=Z, T=T,
                  tau_E=tE, tau_I=tI, seed=99, stream=s, want_stage=True)
        key = tuple(int(x) for x in r["stage"][-1])
        obs[key] = obs.get(key, 0) + 1
        drm[s] = r["drm"]
    assert sum(final.values()) == pytest.approx(1.0, abs=1e-12)
    assert set(obs) <= set(final)
    keys = sorted(final, key=lambda k: -final[k])
    exp_counts = np.array([final[k] * reps for k in keys])
    obs_counts = np.array([obs.get(k, 0) for k in keys], float)
    big = exp_counts >= 5
    e_b = np.append(exp_counts[big], exp_counts[~big].sum())
    o_b = np.append(obs_counts[big], obs_counts[~big].sum())
    if e_b[-1] < 5:
        e_b[-2] += e_b[-1]; o_b[-2] += o_b[-1]
        e_b, o_b = e_b[:-1], o_b[:-1]
    assert stats.chisquare(o_b, e_b).pvalue > 1e-3
    se = drm.std(axis=0, ddof=1) / np.sqrt(reps) + 1e-12
    assert np.all(np.abs(drm.mean(axis=0) - np.array(exp_drm)) <= 5 * se + 1e-9)


# ---------------------------------------------------------------- large-N limits
def _complete_runs(N, K, R, S, seeds, T=(0, 0, 1, 0, 0), m=0.01, i0=0.02):
    a, b = complete_pairs(N)
    src, dst, w = to_symmetric_coo([(a, b, 1.0)])
    age = (np.arange(N) % 8).astype(np.uint8)
    Z = np.float32(5 * (N - 1))
    out = []
    for s in seeds:
        out.append(O.run(age=age, pop_offsets=[0, N], src=src, dst=dst, w=w, K=K, R=R, S=S, m=m, i0=i0, Z=Z,
                         T=T, seed=s, want_stage=True))
    return age, out


@pytest.fixture(scope="module")
def complete_graph_runs():
    N, K = 1200, 110
    S = np.array([0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 0.55, 0.95], np.float32)
    age, runs = _complete_runs(N, K, np.float32(2.5), S, range(12))
    return N, K, S, age, runs


def test_final_size_relation(complete_graph_runs):
    N, K, S, age, runs = complete_graph_runs
    sizes = np.bincount(age, minlength=8)
    fin = []
    x0 = []
    for r in runs:
        st = r["stage"]
        assert r["counts"][-1, 1] + r["counts"][-1, 2] == 0  # epidemic over
        fin.append(np.bincount(age[st[-1] == 0], minlength=8))
        x0.append(np.bincount(age[st[0] == 2], minlength=8))
    fin = np.mean(fin, axis=0)
    x0 = np.mean(x0, axis=0)
    pred = MF.final_size(2.5, S, sizes - x0, x0.sum(), N)
    # per age group, the escaping fraction follows exp(-R S_a (N - S_inf)/(N-1))
    assert np.all(np.abs(fin - pred) <= 0.04 * sizes)
    assert abs(fin.sum() - pred.sum()) <= 0.02 * N


def test_mean_field_curve(complete_graph_runs):
    N, K, S, age, runs = complete_graph_runs
    sizes = np.bincount(age, minlength=8)
    x0 = np.mean([np.bincount(age[r["stage"][0] == 2], minlength=8) for r in runs], axis=0)
    S_mf, drm_mf = MF.mean_field(2.5, S, sizes, x0, N, K, 3, 5, 0.01)
    S_mc = np.mean([r["counts"][:, 0] for r in runs], axis=0)
    assert np.max(np.abs(S_mc - S_mf)) <= 0.04 * N
    c_mc = np.cumsum(np.mean([r["drm"] for r in runs], axis=0))
    assert np.max(np.abs(c_mc - np.cumsum(drm_mf))) <= 0.04 * N


def test_presymptomatic_transmission_scales_final_size():
    # T_E > 0 adds T_E tau_E / tau_I to the reproduction number
    N, K = 800, 120
    S = np.ones(8, np.float32)
    age, runs = _complete_runs(N, K, np.float32(1.2), S, range(8), T=(0, 0.5, 1.0, 0, 0))
    fin = np.mean([r["counts"][-1, 0] for r in runs])
    x0 = np.mean([r["counts"][0, 2] for r in runs])
    pred = MF.final_size(1.2, [1.0], [N - x0], x0, N, T_I=1.0, T_E=0.5)[0]
    pred_wrong = MF.final_size(1.2, [1.0], [N - x0], x0, N, T_I=1.0, T_E=0.0)[0]
    assert abs(fin - pred) <= 0.03 * N
    assert abs(fin - pred_wrong) > 0.1 * N


def test_seirm_ode_limit():
    # homogeneous susceptibility: same final size as the SEIRM ODE with R0 = R
    N, K = 1200, 110
    S = np.ones(8, np.float32)
    age, runs = _complete_runs(N, K, np.float32(2.0), S, range(8))
    x0 = np.mean([r["counts"][0, 2] for r in runs])
    ode = MF.seirm_ode(2.0, N, x0, 3, 5, 0.01, 400)
    fin_abm = np.mean([r["counts"][-1, 0] for r in runs])
    assert abs(ode[-1, 0] - fin_abm) <= 0.02 * N
    # deaths: m times everyone ever removed, both models
    dead_abm = np.mean([r["counts"][-1, 4] for r in runs])
    assert abs(dead_abm - ode[-1, 4]) <= 5 * np.sqrt(0.01 * (N - fin_abm) / len(runs)) + 1.0
    # the fixed-delay and exponential-delay epidemics differ in shape but
    # not in order of magnitude of the timing
    peak_abm = np.argmax(np.mean([r["counts"][:, 2] for r in runs], axis=0))
    peak_ode = np.argmax(ode[:, 2])
    assert abs(int(peak_abm) - int(peak_ode)) <= 15


# ---------------------------------------------------------------- gradients
def _soft_setup():
    wl = make_workload("c2", n_agents=1500, K=22)
    tgt = np.linspace(0.0, 0.3, wl.K)
    return wl, tgt


def _loss(wl, tgt, R, S, m, i0, mode, iota=None, dwell=None):
    return O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K, R=R, S=S,
                 m=m, i0=i0, Z=wl.Z, mode=mode, tau_g=wl.tau_g, er_mean_deg=wl.er_mean_deg,
                 er_weight=wl.er_weight, target=tgt, iota=iota, dwell=dwell)["loss"]


# an infectiousness profile over the 8 days after exposure (rising, then
# falling), values exact in float32
PROFILE = np.array([0.25, 0.5, 0.75, 1.5, 1.75, 1.25, 0.75, 0.25], np.float32)
# stochastic dwell times: log weights of the E lengths 1..3 and the I lengths 1..5
DWELL = (np.log(np.array([0.2, 0.5, 0.3], np.float32)), np.log(np.array([0.1, 0.2, 0.3, 0.25, 0.15], np.float32)))


@pytest.mark.parametrize("iota,dwell", [(None, None), (PROFILE, None), (None, DWELL)], ids=["flat", "profile", "dwell"])
def test_soft_tangents_match_finite_differences(iota, dwell):
    wl, tgt = _soft_setup()
    R0, S0, m0, i00 = np.float32(2.5), wl.S[0].copy(), np.float32(0.01), np.float32(0.01)
    dirs = O.standard_directions(wl.K, 8)
    r = O.run_workload(wl, mode=O.SOFT, R=np.full(wl.K, R0, np.float32), target=tgt, directions=dirs, iota=iota,
                       dwell=dwell)
    g = r["dL"]
    assert r["loss"] == pytest.approx(_loss(wl, tgt, R0, S0, m0, i00, O.SOFT, iota, dwell), rel=0, abs=0)

    def fd(k, h):
        def at(delta):
            R, S, m, i0 = R0, S0.copy(), m0, i00
            if k == 0:
                R = np.float32(R0 + delta)
            elif k <= 8:
                S[k - 1] = np.float32(S0[k - 1] + delta)
            elif k == 9:
                m = np.float32(m0 + delta)
            else:
                i0 = np.float32(i00 + delta)
            return _loss(wl, tgt, R, S, m, i0, O.SOFT, iota, dwell)
        d1 = (at(h) - at(-h)) / (2 * h)
        d2 = (at(h / 2) - at(-h / 2)) / h
        return (4 * d2 - d1) / 3  # Richardson

    # perturbations exactly representable in float32 around each value
    steps = [2.0**-8] + [2.0**-12] * 8 + [2.0**-15, 2.0**-15]
    gmax = np.max(np.abs(g))
    for k in range(11):
        f = fd(k, steps[k])
        assert abs(f - g[k]) <= 1e-6 * max(abs(g[k]), 1e-3 * gmax), (k, f, g[k])


def test_hard_mortality_gradient_closed_form():
    wl = make_workload("c2", n_agents=3000, K=25)
    tgt = np.linspace(0, 1, wl.K)
    r = O.run_workload(wl, mode=O.HARD_ST, target=tgt, directions=O.standard_directions(wl.K, 8))
    D = r["deaths"]
    expect = 2.0 / wl.K * np.sum((D - tgt) * r["drm"])
    assert r["dL"][9] == pytest.approx(expect, rel=1e-13)
    # PLAIN and HARD_ST follow the same trajectory
    r0 = O.run_workload(wl, mode=O.PLAIN, target=tgt)
    assert np.array_equal(r0["counts"], r["counts"]) and r0["loss"] == r["loss"]


def test_two_agent_straight_through_gradient_by_hand():
    # agent 0 starts infectious, agent 1 susceptible; tau_E = tau_I = 1, K = 3
    seed = _forced_initial(2, [1, 0])
    src, dst, w = to_symmetric_coo([(np.array([0]), np.array([1]), np.array([0.75], np.float32))])
    age = np.array([2, 5], np.uint8)
    S = np.linspace(0.3, 1.0, 8).astype(np.float32)
    R, Z, m, tau = 1.5, 0.5, 0.25, 0.5
    tgt = np.array([0.1, 0.0, 0.2])
    r = O.run(age=age, pop_offsets=[0, 2], src=src, dst=dst, w=w, K=3, R=R, S=S, m=m, i0=0.5, Z=Z, tau_E=1,
              tau_I=1, mode=O.HARD_ST, tau_g=tau, seed=seed, target=tgt, directions=O.standard_directions(3, 8),
              want_agents=True)
    lam = R * float(S[5]) * 0.75 / Z
    q = -np.expm1(-lam)
    u = O.uniform(seed, 1, 0, O_TAG_INFECT)
    h = float(u < q)
    z = (np.log(q / (1 - q)) + np.log((1 - u) / u)) / tau
    y = 1 / (1 + np.exp(-z))
    dydl = y * (1 - y) / (tau * q)
    # deaths: day 0 removes agent 0 (initial), day 2 removes agent 1 if exposed on day 0
    D = np.array([m * 1.0, 0.0, m * h])
    assert np.allclose(r["deaths"], D, rtol=0, atol=1e-15)
    res = D - tgt
    dL_dR = 2 / 3 * res[2] * m * dydl * float(S[5]) * 0.75 / Z
    dL_dS5 = 2 / 3 * res[2] * m * dydl * R * 0.75 / Z
    dL_dm = 2 / 3 * (res[0] * 1.0 + res[2] * h)
    assert r["dL"][0] == pytest.approx(dL_dR, rel=1e-12)
    assert r["dL"][1 + 5] == pytest.approx(dL_dS5, rel=1e-12)
    assert r["dL"][9] == pytest.approx(dL_dm, rel=1e-12)
    for a in (0, 1, 2, 3, 4, 6, 7):
        assert r["dL"][1 + a] == 0.0


def test_profile_of_ones_is_the_flat_model():
    """A profile of ones reproduces the model without a profile exactly:
    trajectories, rates and tangents, hard and relaxed."""
    wl = make_workload("c2", n_agents=2000, K=20)
    tgt = np.linspace(0.0, 0.3, wl.K)
    dirs = O.standard_directions(wl.K, 8)
    for mode in (O.HARD_ST, O.SOFT):
        a = O.run_workload(wl, mode=mode, target=tgt, directions=dirs, want_agents=True)
        b = O.run_workload(wl, mode=mode, target=tgt, directions=dirs, want_agents=True,
                           iota=np.ones(wl.tau_E + wl.tau_I, np.float32))
        for k in ("counts", "A", "lam", "dL"):
            assert np.array_equal(a[k], b[k]), (mode, k)


def test_profile_indexing_closed_form():
    """Three agents on a path 0 - 1 - 2, agent 0 initially infected, presymptomatic
    transmissibility T[E] = 0.5: with R huge on day 0 and zero afterwards,
    agent 1 is exposed on day 0 and nobody else ever is.  Then agent 2's
    contact sum on day t is T[stage] * iota[t - 1] (exposed on day 0, days
    since exposure t), and agent 1's is T[I] * iota[t + tau_E] (an initial
    infection counts as exposed on day -tau_E - 1)."""
    tE, tI, K = 3, 5, 12
    W = tE + tI
    T = (0.0, 0.5, 1.0, 0.0, 0.0)
    R = np.zeros(K, np.float32)
    R[0] = 1e6
    kw = dict(age=np.zeros(3, np.uint8), pop_offsets=[0, 3], src=[0, 1, 1, 2], dst=[1, 0, 2, 1],
              w=np.ones(4, np.float32), K=K, R=R, S=[1.0], m=0.0, i0=0.5, Z=[1.0], T=T, tau_E=tE, tau_I=tI,
              mode=O.PLAIN, iota=PROFILE, want_agents=True, want_stage=True)
    for seed in range(500):  # a seed whose initial draws infect agent 0 only
        r = O.run(seed=seed, **kw)
        if list(r["stage"][0]) == [O.STAGES.index("I"), 0, 0]:
            break
    else:
        pytest.fail("no seed infects agent 0 alone")
    assert r["h"][0][1] == 1 and r["h"][1:, 1].sum() == 0 and r["h"][:, 2].sum() == 0
    for t in range(K):
        a1 = T[2] * PROFILE[t + tE] if t < tI else 0.0
        k = t  # agent 1's days since exposure
        a2 = (T[1] if k <= tE else T[2]) * PROFILE[k - 1] if 1 <= k <= W else 0.0
        assert r["A"][t][1] == np.float64(a1), t
        assert r["A"][t][2] == np.float64(a2), t


def _random_visits(n, n_loc, rng, max_visits=3):
    """Each agent visits 1..max_visits distinct locations, weights k/64."""
    ag, lo, wt = [], [], []
    for a in range(n):
        for l in rng.choice(n_loc, rng.integers(1, max_visits + 1), replace=False):
            ag.append(a)
            lo.append(int(l))
            wt.append(rng.integers(1, 65) / 64.0)
    return np.array(ag, np.int32), np.array(lo, np.int32), np.array(wt, np.float32)


def _expanded(n, visits):
    """The contact graph the location layer stands for: w_ij = sum over shared
    locations of w_il * w_jl, for i != j, both directions listed."""
    ag, lo, wt = visits
    by_loc = {}
    for a, l, w in zip(ag, lo, wt):
        by_loc.setdefault(int(l), []).append((int(a), float(w)))
    pair = {}
    for members in by_loc.values():
        for a, wa in members:
            for b, wb in members:
                if a != b:
                    pair[(a, b)] = pair.get((a, b), 0.0) + wa * wb
    src = np.array([b for (a, b) in pair], np.int32)
    dst = np.array([a for (a, b) in pair], np.int32)
    w = np.array([pair[k] for k in pair], np.float32)
    assert np.array_equal(w.astype(np.float64), np.array([pair[k] for k in pair]))  # exact in float32
    return src, dst, w


@pytest.mark.parametrize("mode", [O.PLAIN, O.HARD_ST, O.SOFT], ids=["plain", "hard_st", "soft"])
def test_location_layer_equals_its_contact_graph(mode):
    """The two-hop sum over locations equals the neighbour sum over the
    expanded graph (w_ij = sum of w_il w_jl over shared locations, i != j):
    with visit weights k/64 every hard sum is exact, so trajectories, contact
    sums and loss agree bit for bit; tangents and relaxed values to rounding."""
    rng = np.random.default_rng(11)
    n, K = 400, 16
    visits = _random_visits(n, 40, rng)
    src, dst, w = _expanded(n, visits)
    age = (np.arange(n) % 8).astype(np.uint8)
    S = np.linspace(0.5, 1.0, 8).astype(np.float32)
    tgt = np.linspace(0.0, 0.5, K)
    dirs = O.standard_directions(K, 8) if mode != O.PLAIN else None
    kw = dict(age=age, pop_offsets=[0, n], K=K, R=1.5, S=S, m=0.05, i0=0.05, Z=[40.0], mode=mode, seed=3,
              target=tgt, directions=dirs, want_agents=True)
    a = O.run(src=[], dst=[], w=[], visits=visits, **kw)
    b = O.run(src=src, dst=dst, w=w, **kw)
    if mode == O.SOFT:
        assert np.allclose(a["A"], b["A"], rtol=1e-13, atol=1e-15)
        assert a["loss"] == pytest.approx(b["loss"], rel=1e-12)
        assert np.allclose(a["dL"], b["dL"], rtol=1e-10, atol=1e-14)
    else:
        assert np.array_equal(a["counts"], b["counts"]) and np.array_equal(a["A"], b["A"])
        assert a["loss"] == b["loss"]
        if dirs is not None:  # tangents are real-valued: equal up to the order of their sums
            assert np.allclose(a["dL"], b["dL"], rtol=1e-11, atol=1e-14 * np.abs(b["dL"]).max())
    assert a["counts"][-1][0] < n  # the layer spreads infection


def test_location_layer_excludes_the_visitor():
    """Agent 0 alone at location 0 and with agent 1 at location 1 (weights
    1/2 and 3/4 for agent 0, 1/4 for agent 1), agent 1 infected at the start:
    agent 0's sum is (3/4)(1/4) T_I on every infectious day, agent 1's is 0."""
    visits = (np.array([0, 0, 1], np.int32), np.array([0, 1, 1], np.int32), np.array([0.5, 0.75, 0.25], np.float32))
    kw = dict(age=np.zeros(2, np.uint8), pop_offsets=[0, 2], src=[], dst=[], w=[], K=4, R=0.0, S=[1.0], m=0.0,
              i0=0.5, Z=[1.0], mode=O.PLAIN, visits=visits, want_agents=True, want_stage=True)
    for seed in range(500):
        r = O.run(seed=seed, **kw)
        if list(r["stage"][0]) == [0, O.STAGES.index("I")]:
            break
    else:
        pytest.fail("no seed infects agent 1 alone")
    for t in range(4):
        assert r["A"][t][0] == 0.75 * 0.25 and r["A"][t][1] == 0.0


# ---------------------------------------------------------------- stochastic dwell times


def test_dwell_draw_frequencies():
    """The Gumbel-max draw over (agent, day) counters follows softmax of the
    log weights (chi-square over 40,000 draws), for E and I tables, including
    a length of weight zero that is never drawn."""
    lwE = np.log(np.array([0.2, 0.5, 0.3], np.float32))
    lwI = np.array([np.log(0.1), np.log(0.2), -np.inf, np.log(0.45), np.log(0.25)], np.float32)
    for lw, tag in ((lwE, O.TAG_DWELL_E), (lwI, O.TAG_DWELL_I)):
        p = np.exp(lw.astype(np.float64))
        p /= p.sum()
        draws = np.array([O.dwell_draw(lw, 11, i, d, tag) for i in range(2000) for d in range(20)])
        counts = np.bincount(draws - 1, minlength=len(lw))
        if not np.all(p > 0):
            assert np.all(counts[p == 0] == 0)
        keep = p > 0
        chi2 = np.sum((counts[keep] - p[keep] * len(draws)) ** 2 / (p[keep] * len(draws)))
        assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4, (counts, p)
    # E and I draws of one exposure are not the same stream
    e = [O.dwell_draw(np.zeros(8, np.float32), 5, i, 3, O.TAG_DWELL_E) for i in range(200)]
    i_ = [O.dwell_draw(np.zeros(8, np.float32), 5, i, 3, O.TAG_DWELL_I) for i in range(200)]
    assert e != i_


@pytest.mark.parametrize("mode", [O.PLAIN, O.HARD_ST, O.SOFT], ids=["plain", "hard_st", "soft"])
def test_one_hot_dwell_tables_are_the_fixed_model(mode):
    """Tables that put all weight on tau_E and tau_I reproduce the model with
    fixed dwell times bit for bit: trajectories, sums, loss and tangents."""
    wl = make_workload("c2", n_agents=3000, K=20)
    tgt = np.linspace(0.0, 0.5, wl.K)
    ninf = np.float32(-np.inf)
    onehot = (np.array([ninf, ninf, 0.0], np.float32), np.array([ninf] * 4 + [0.0], np.float32))
    dirs = O.standard_directions(wl.K, 8) if mode != O.PLAIN else None
    a = O.run_workload(wl, mode=mode, target=tgt, directions=dirs, want_agents=True, want_stage=True)
    b = O.run_workload(wl, mode=mode, target=tgt, directions=dirs, want_agents=True, want_stage=True, dwell=onehot)
    for k in ("counts", "A", "stage", "drm"):
        assert np.array_equal(a[k], b[k]), k
    assert a["loss"] == b["loss"]
    if dirs is not None:
        assert np.array_equal(a["dL"], b["dL"])


ST_E, ST_I = 1, 2  # stage codes of the exposed and infectious stages


def _runs_of(stage_row, value):
    """(start, length) of each maximal run of `value` in a stage trajectory."""
    out, start = [], None
    for t, s in enumerate(stage_row):
        if s == value and start is None:
            start = t
        elif s != value and start is not None:
            out.append((start, t - start))
            start = None
    if start is not None:
        out.append((start, None))  # still running at the end
    return out


def test_dwell_stage_durations_follow_the_draws():
    """In a hard run every exposure's E and I spells last exactly the lengths
    drawn for (agent, exposure day), initial infections' I spells the length
    drawn for day 2^32 - 1, and the exposure-window form agrees with the stage
    machine (no mismatch); the E lengths observed over the run follow the
    table (chi-square)."""
    wl = make_workload("c2", n_agents=4000, K=40)
    r = O.run_workload(wl, mode=O.PLAIN, want_stage=True, dwell=DWELL)
    assert r["mismatch"] == 0
    st = r["stage"]  # [K+1, N]
    seen_E = []
    n_checked = 0
    for i in range(wl.n_agents):
        row = st[:, i]
        if row[0] == ST_I:
            d0 = O.dwell_draw(DWELL[1], wl.seed, i, 0xFFFFFFFF, O.TAG_DWELL_I)
            runs = _runs_of(row, ST_I)
            assert runs[0][0] == 0
            if runs[0][1] is not None:
                assert runs[0][1] == d0, (i, runs, d0)
            continue
        for start, length in _runs_of(row, ST_E):
            u = start - 1  # exposed during day u, E from snapshot u + 1
            dE = O.dwell_draw(DWELL[0], wl.seed, i, u, O.TAG_DWELL_E)
            dI = O.dwell_draw(DWELL[1], wl.seed, i, u, O.TAG_DWELL_I)
            if length is None:
                continue
            assert length == dE, (i, u, length, dE)
            seen_E.append(length)
            irun = [x for x in _runs_of(row, ST_I) if x[0] == start + length]
            assert irun, (i, u)
            if irun[0][1] is not None:
                assert irun[0][1] == dI, (i, u, irun, dI)
                n_checked += 1
    assert n_checked > 200
    p = np.exp(DWELL[0].astype(np.float64))
    p /= p.sum()
    counts = np.bincount(np.array(seen_E) - 1, minlength=3)
    chi2 = np.sum((counts - p * len(seen_E)) ** 2 / (p * len(seen_E)))
    assert stats.chi2.sf(chi2, 2) > 1e-4, counts


def test_dwell_tables_are_checked():
    wl = make_workload("c1", n_agents=500, K=5)
    with pytest.raises(ValueError):  # lengths of at most 8 days
        O.run(age=wl.pop.age, pop_offsets=wl.pop.pop_offsets, src=wl.src, dst=wl.dst, w=wl.w, K=wl.K, R=2.5,
              S=wl.S[0], m=0.01, i0=0.01, Z=wl.Z, tau_E=9, tau_I=5,
              dwell=(np.zeros(9, np.float32), np.zeros(5, np.float32)))


@pytest.mark.parametrize("iota", [None, PROFILE], ids=["flat", "profile"])
def test_soft_dwell_weight_tangents_match_finite_differences(iota):
    """Relaxed mode with dwell tables: the relaxed one-hots of the Gumbel-max
    draws weight a mixture of windows, so the loss is smooth in the log weights
    and the tangents along each of them equal central differences (also with
    an infectiousness profile over days since exposure)."""
    wl, tgt = _soft_setup()
    K = wl.K
    dirs = O.dwell_directions(K, 8, 3, 5)
    r = O.run_workload(wl, mode=O.SOFT, target=tgt, directions=dirs, dwell=DWELL, iota=iota)
    g = r["dL"][11:]
    assert np.all(np.isfinite(g)) and np.max(np.abs(g)) > 0

    def loss_at(which, k, delta):
        lw = [DWELL[0].copy(), DWELL[1].copy()]
        lw[which][k] = np.float32(lw[which][k] + delta)
        return O.run_workload(wl, mode=O.SOFT, target=tgt, dwell=tuple(lw), iota=iota)["loss"]

    h = 2.0**-8
    gmax = np.max(np.abs(g))
    for idx in range(8):
        which, k = (0, idx) if idx < 3 else (1, idx - 3)
        d1 = (loss_at(which, k, h) - loss_at(which, k, -h)) / (2 * h)
        d2 = (loss_at(which, k, h / 2) - loss_at(which, k, -h / 2)) / h
        fd = (4 * d2 - d1) / 3
        assert abs(fd - g[idx]) <= 1e-6 * max(abs(g[idx]), 1e-3 * gmax), (idx, fd, g[idx])


def _relaxed_one_hot(lw, seed, idx, day, tag0, tau):
    """Gumbel noise of the (idx, day) counter, re-derived from Philox words:
    the drawn length and softmax((lw + G) / tau)."""
    G = []
    for k in range(len(lw)):
        o = O.philox([idx, day, tag0 + k // 4, 0], [seed & 0xFFFFFFFF, seed >> 32])
        u = (2 * (int(o[k % 4]) >> 9) + 1) / 2.0**24
        G.append(-np.log(-np.log(u)))
    v = lw.astype(np.float64) + np.array(G)
    e = np.exp((v - v.max()) / tau)
    return int(np.argmax(v)) + 1, e / e.sum()


def test_straight_through_dwell_gradient_of_an_initial_infection():
    """One agent, initially infected, no contacts: its removal falls on day
    b - 1 for the drawn I length b, and the straight-through gradient of the
    loss with respect to the I log weight j is
    (2/K) sum_t (D_t - y_t) m dc_{t+1}, with dc_k = c_k (delta_kj - c_j) / tau
    the tangent of the relaxed one-hot c of the same Gumbel noise."""
    K, m, tau = 10, float(np.float32(0.3)), 0.5  # parameters are float32 values
    tgt = np.linspace(0.0, 0.2, K)
    seed = next(s for s in range(100) if O.uniform(s, 0, 0xFFFFFFFF, 0) < 0.5)
    dirs = O.dwell_directions(K, 1, 3, 5)
    r = O.run(age=np.zeros(1, np.uint8), pop_offsets=[0, 1], src=[], dst=[], w=[], K=K, R=2.0, S=[1.0], m=m,
              i0=0.5, Z=[1.0], mode=O.HARD_ST, tau_g=tau, seed=seed, target=tgt, directions=dirs, dwell=DWELL)
    b, c = _relaxed_one_hot(DWELL[1], seed, 0, 0xFFFFFFFF, O.TAG_DWELL_I, tau)
    assert r["drm"][b - 1] == 1.0 and r["drm"].sum() == 1.0
    resid = r["deaths"] - tgt
    for j in range(5):
        dc = c * ((np.arange(5) == j) - c[j]) / tau
        want = 2.0 / K * sum(resid[t] * m * dc[t] for t in range(min(K, 5)))
        assert r["dL"][4 + 3 + j] == pytest.approx(want, rel=1e-12, abs=1e-15), j  # after R, S, m, i0, 3 E
    assert np.all(r["dL"][4:7] == 0.0)  # no exposures: the E weights do not matter


def test_straight_through_dwell_gradient_of_an_exposure():
    """Two agents in contact: agent 0 initially infected, agent 1 exposed on
    day u.  Along the E log weights nothing but agent 1's removal moves
    (agent 0 has no E length and is no longer susceptible), and agent 1's
    removal falls on day u + a + b for its drawn lengths, so the gradient with
    respect to E log weight j is (2/K) sum_k (D_{u+k} - y_{u+k}) m dc_{k-b},
    dc the relaxed one-hot's tangent of agent 1's E draw."""
    K, m, tau = 20, float(np.float32(0.3)), 0.5
    tgt = np.linspace(0.0, 0.2, K)
    kw = dict(age=np.zeros(2, np.uint8), pop_offsets=[0, 2], src=[0, 1], dst=[1, 0], w=[1.0, 1.0], K=K, R=3.0,
              S=[1.0], m=m, i0=0.5, Z=[1.0], mode=O.HARD_ST, tau_g=tau, target=tgt, dwell=DWELL)
    for seed in range(400):
        if not (O.uniform(seed, 0, 0xFFFFFFFF, 0) < 0.5 <= O.uniform(seed, 1, 0xFFFFFFFF, 0)):
            continue
        r = O.run(seed=seed, want_agents=True, want_stage=True, **kw)
        exposed = [t for t in range(K) if r["h"][t, 1] and r["stage"][t, 1] == 0]
        if exposed and exposed[0] + 3 + 5 < K:
            break
    else:
        pytest.skip("no seed with an early exposure")
    u = exposed[0]
    a, cE = _relaxed_one_hot(DWELL[0], seed, 1, u, O.TAG_DWELL_E, tau)
    b, _ = _relaxed_one_hot(DWELL[1], seed, 1, u, O.TAG_DWELL_I, tau)
    # E from snapshot u + 1, removed during day u + a + b
    assert r["stage"][u + a + b + 1, 1] in (3, 4) and r["stage"][u + a + b, 1] == ST_I
    dirs = O.dwell_directions(K, 1, 3, 5)
    rd = O.run(seed=seed, directions=dirs, **kw)
    resid = rd["deaths"] - tgt
    wants = []
    for j in range(3):
        dc = cE * ((np.arange(3) == j) - cE[j]) / tau
        want = sum(2.0 / K * resid[u + k] * m * dc[k - b - 1] for k in range(b + 1, b + 4) if u + k < K)
        assert rd["dL"][4 + j] == pytest.approx(want, rel=1e-12, abs=1e-15), (j, rd["dL"][4 + j], want)
        wants.append(want)
    assert max(abs(w) for w in wants) > 1e-6
