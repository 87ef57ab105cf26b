"""Large-population limits of the simulator on a complete contact graph.

TEST INFRASTRUCTURE ONLY.  On a complete graph with unit weights and
normaliser Z = tau_I (N-1), every susceptible agent of age group a sees the
same rate R S_a I^t / (tau_I (N-1)), so as N grows the stochastic simulation
approaches deterministic limits that can be written down without the
simulator:

* the final-size relation (holds for any infectious-period distribution):
  s_a = exp(-R S_a (N - S_inf) / (N - 1)) for the escaping fraction of
  group a, with S_inf = sum_a S_a0 s_a;
* the discrete mean-field recurrence with the fixed delays tau_E, tau_I;
* the SEIRM ordinary differential equations of the paper's appendix
  (Appendix D): dS = -beta S I / N, dE = beta S I / N - alpha E,
  dI = alpha E - (gamma + mu) I, dR = gamma I, dM = mu I, with
  beta = R / tau_I, alpha = 1 / tau_E, gamma + mu = 1 / tau_I, mu = m / tau_I,
  so that R0 = beta / (gamma + mu) = R.
"""

from __future__ import annotations

import numpy as np


def final_size(R, Sa, group_sizes, initial_infected, N, T_I=1.0, T_E=0.0, tau_E=3, tau_I=5, iters=10_000):
    """Expected final number of never-infected agents per group (fixed point).

    With transmissibility T_E while exposed and T_I while infectious, an
    infected agent contributes (T_E tau_E + T_I tau_I) / tau_I times R of
    total hazard, spread over N - 1 others."""
    Sa = np.asarray(Sa, float)
    S0 = np.asarray(group_sizes, float)  # susceptible at t=0 per group
    reff = R * (T_E * tau_E + T_I * tau_I) / tau_I
    s = np.ones_like(Sa)
    for _ in range(iters):
        S_inf = float((S0 * s).sum())
        s_new = np.exp(-reff * Sa * (N - S_inf) / (N - 1))
        if np.max(np.abs(s_new - s)) < 1e-15:
            s = s_new
            break
        s = s_new
    return S0 * s


def mean_field(R, Sa_of_group, group_sizes, x0_per_group, N, K, tau_E, tau_I, m):
    """Discrete-time mean-field recurrence with fixed delays.

    Returns (expected susceptible per snapshot [K+1], expected removals per
    day [K]).  x0_per_group is the expected number initially infected."""
    Sa = np.asarray(Sa_of_group, float)
    Sg = np.asarray(group_sizes, float) - np.asarray(x0_per_group, float)
    x0 = float(np.sum(x0_per_group))
    new = np.zeros(K)
    S_hist = [Sg.sum()]
    drm = np.zeros(K)
    for t in range(K):
        I = sum(new[u] for u in range(max(0, t - tau_E - tau_I), t - tau_E) if u >= 0)
        if t < tau_I:
            I += x0
        lam = R * Sa * I / (tau_I * (N - 1))
        inf = Sg * (1.0 - np.exp(-lam))
        new[t] = inf.sum()
        Sg = Sg - inf
        S_hist.append(Sg.sum())
        u = t - tau_E - tau_I
        drm[t] = (new[u] if u >= 0 else 0.0) + (x0 if t == tau_I - 1 else 0.0)
    return np.array(S_hist), drm


def seirm_ode(R, N, I0, tau_E, tau_I, m, K, steps_per_day=200):
    """Integrate the SEIRM ODE with classical RK4; returns S, E, I, R, M at
    integer days 0..K (arrays of length K+1)."""
    beta, alpha, g_plus_mu = R / tau_I, 1.0 / tau_E, 1.0 / tau_I
    mu = m / tau_I
    gamma = g_plus_mu - mu

    def f(y):
        s, e, i, r, mm = y
        inf = beta * s * i / N
        return np.array([-inf, inf - alpha * e, alpha * e - (gamma + mu) * i, gamma * i, mu * i])

    y = np.array([N - I0, 0.0, I0, 0.0, 0.0])
    out = [y.copy()]
    h = 1.0 / steps_per_day
    for _ in range(K):
        for _ in range(steps_per_day):
            k1 = f(y)
            k2 = f(y + 0.5 * h * k1)
            k3 = f(y + 0.5 * h * k2)
            k4 = f(y + h * k3)
            y = y + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        out.append(y.copy())
    return np.array(out)
