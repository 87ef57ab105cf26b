"""Exact outcome distribution of the stochastic simulator on tiny graphs.

TEST INFRASTRUCTURE ONLY.  This is a second, independent statement of the
model's semantics (Section 3.1: Transmit for susceptible agents with
probability q = 1 - exp(-lambda_A) (Eq. 3), Progress with fixed transition
times and mortality fraction m; Appendix A assumptions A1-A6), written as
a Markov chain over joint agent states and propagated exactly, with no
random numbers.  The oracle's Monte Carlo frequencies must agree with it.
"""

from __future__ import annotations

import itertools
import math
from collections import defaultdict

S, E, I, R, M = range(5)


def exact_distribution(n, edges, age, R_t, Sa, T, m, i0, Z, tau_E, tau_I, K):
    """Propagate the joint distribution of (stage, timer) per agent.

    edges: list of (src, dst, w) directed contacts.  Returns
    (final distribution {stage tuple: prob}, expected removals per day [K],
    expected stage counts per snapshot [K+1][5]).
    """
    dist = defaultdict(float)
    for init in itertools.product((0, 1), repeat=n):
        p = 1.0
        st = []
        for x in init:
            p *= i0 if x else (1.0 - i0)
            st.append((I, tau_I) if x else (S, 0))
        if p > 0:
            dist[tuple(st)] += p
    exp_drm = [0.0] * K
    exp_counts = [[0.0] * 5 for _ in range(K + 1)]

    def add_counts(t, d):
        for state, p in d.items():
            for s, _ in state:
                exp_counts[t][s] += p

    add_counts(0, dist)
    for t in range(K):
        new = defaultdict(float)
        for state, p in dist.items():
            A = [0.0] * n
            for src, dst, w in edges:
                A[dst] += w * T[state[src][0]]
            options = []
            for i, (s, tm) in enumerate(state):
                if s == S:
                    lam = R_t[t] * Sa[age[i]] * A[i] / Z
                    q = 1.0 - math.exp(-lam)
                    options.append([((E, tau_E), q, 0), ((S, 0), 1.0 - q, 0)])
                elif s in (E, I):
                    tm2 = tm - 1
                    if tm2 > 0:
                        options.append([((s, tm2), 1.0, 0)])
                    elif s == E:
                        options.append([((I, tau_I), 1.0, 0)])
                    else:
                        options.append([((M, 0), m, 1), ((R, 0), 1.0 - m, 1)])
                else:
                    options.append([((s, 0), 1.0, 0)])
            for combo in itertools.product(*options):
                pc = p
                removed = 0
                for _, pr, rm in combo:
                    pc *= pr
                    removed += rm
                if pc == 0.0:
                    continue
                new[tuple(c[0] for c in combo)] += pc
                exp_drm[t] += pc * removed
        dist = new
        add_counts(t + 1, dist)
    final = defaultdict(float)
    for state, p in dist.items():
        final[tuple(s for s, _ in state)] += p
    return dict(final), exp_drm, exp_counts
