"""C-GradABM: gradient-based calibration of the simulator's parameters.

Section 3.2 describes calibration as an outer loop around the simulator: each
step runs the K-day simulation with the current parameters, measures the loss
between simulated and observed daily deaths, and moves the parameters
against the gradient of that loss.  The C- variant of Section 4 updates the
simulation parameters themselves (no calibration network), with the plain
gradient-descent rule theta <- theta - alpha * dL/dtheta.  Parameters may vary
in time (Section 4, experimental setup): here the reproduction number is
piecewise constant over blocks of `period` days (period 1: one value per day;
7: one per week), and the per-age susceptibility, the mortality rate and the
initial infected fraction are constant over the run.

Every gradient comes from the library's adjoint through `GabmSim`
(straight-through in HARD_ST mode, exact in SOFT mode); the per-block
gradient of R is the sum of its days' gradients.  Two update rules:
* "gd": the paper's rule on the parameters themselves, then a projection
  into the valid ranges (R > 0; S, m, i0 in (0, 1));
* "adam": Adam on the logarithms of the parameters (relative steps, so
  parameters of different scales share one learning rate), then the same
  projection.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from . import gabm

# valid ranges enforced after every update
R_RANGE = (1e-3, 50.0)
S_RANGE = (1e-3, 1.0)
M_RANGE = (1e-4, 1.0 - 1e-4)
I0_RANGE = (1e-5, 1.0 - 1e-5)
_RANGES = {"R": R_RANGE, "S": S_RANGE, "m": M_RANGE, "i0": I0_RANGE}


@dataclass
class CalibrationResult:
    R: torch.Tensor          # [n_sets, K] per-day reproduction number
    R_blocks: torch.Tensor   # [n_sets, n_blocks] its block values
    S: torch.Tensor          # [n_sets, n_age]
    m: torch.Tensor          # [n_sets]
    i0: torch.Tensor         # [n_sets]
    loss: list = field(default_factory=list)  # summed loss before each update, then after the last


def block_index(K: int, period: int, device=None) -> torch.Tensor:
    """Block of every day: day t belongs to block t // period."""
    if period < 1:
        raise ValueError("period must be >= 1")
    return torch.arange(K, device=device) // period


def to_blocks(R: torch.Tensor, period: int) -> torch.Tensor:
    """Block values of a per-day R [n_sets, K]: the mean of each block's days."""
    K = R.shape[-1]
    idx = block_index(K, period, R.device)
    nb = int(idx[-1].item()) + 1
    tot = torch.zeros(R.shape[0], nb, dtype=R.dtype, device=R.device).index_add_(1, idx, R)
    cnt = torch.bincount(idx, minlength=nb).to(R.dtype)
    return tot / cnt


def _project(name: str, x: torch.Tensor) -> None:
    lo, hi = _RANGES[name]
    x.clamp_(lo, hi)


def calibrate(sim: gabm.Simulator, target, R, S, m, i0, *, steps: int = 50, lr: float = 0.05, period: int = 7,
              optimizer: str = "adam", seed: int = 0, fit=("R", "S", "m", "i0")) -> CalibrationResult:
    """Fit the parameters listed in `fit` to the daily-deaths `target` ([K] or
    [n_out, K]) with `steps` updates; the others stay at their given values.

    R is given per day ([n_sets, K]); it is reduced to block means over
    `period` days, and the fitted R is piecewise constant on those blocks.
    S [n_sets, n_age], m [n_sets], i0 [n_sets].  The simulator's mode decides
    the gradient (straight-through or exact); the seed fixes the Philox
    stream, so every step simulates the same random numbers."""
    if optimizer not in ("gd", "adam"):
        raise ValueError("optimizer must be 'gd' or 'adam'")
    bad = set(fit) - set(_RANGES)
    if bad:
        raise ValueError(f"unknown parameters to fit: {sorted(bad)}")
    dev = gabm._dev()
    f32 = dict(dtype=torch.float32, device=dev)
    K = sim.K
    idx = block_index(K, period, dev)
    vals = {"R": to_blocks(torch.as_tensor(R, **f32).reshape(sim.n_sets, K), period),
            "S": torch.as_tensor(S, **f32).reshape(sim.n_sets, -1).clone(),
            "m": torch.as_tensor(m, **f32).reshape(sim.n_sets).clone(),
            "i0": torch.as_tensor(i0, **f32).reshape(sim.n_sets).clone()}
    for k, v in vals.items():
        _project(k, v)
    tgt = torch.as_tensor(target, dtype=torch.float64, device=dev)

    # the optimised variables: the parameters themselves ("gd") or their logarithms ("adam")
    if optimizer == "adam":
        var = {k: vals[k].log().requires_grad_(k in fit) for k in vals}
        opt = torch.optim.Adam([var[k] for k in fit], lr=lr)
    else:
        var = {k: vals[k].requires_grad_(k in fit) for k in vals}
        opt = None

    def params():
        p = {k: (v.exp() if optimizer == "adam" else v) for k, v in var.items()}
        return p["R"][:, idx], p["S"], p["m"], p["i0"]

    losses = []
    for _ in range(steps):
        Rt, St, mt, it = params()
        loss, _ = gabm.GabmSim.apply(Rt, St, mt, it, sim, seed, tgt)
        total = loss.sum()
        losses.append(float(total.item()))
        for k in fit:
            var[k].grad = None
        total.backward()
        with torch.no_grad():
            if opt is not None:
                opt.step()
                for k in fit:  # the projection, in log space
                    lo, hi = _RANGES[k]
                    var[k].clamp_(math.log(lo), math.log(hi))
            else:
                for k in fit:
                    var[k] -= lr * var[k].grad
                    _project(k, var[k])
    with torch.no_grad():
        Rt, St, mt, it = params()
        out = sim.forward(sim.params(Rt, St, mt, it), seed=seed, target=tgt)
        losses.append(float(out["loss"].sum().item()))
        Rb = var["R"].exp() if optimizer == "adam" else var["R"]
        return CalibrationResult(R=Rt.detach().clone(), R_blocks=Rb.detach().clone(), S=St.detach().clone(),
                                 m=mt.detach().clone(), i0=it.detach().clone(), loss=losses)
