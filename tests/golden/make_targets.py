"""Writes the oracle outputs that the tests and the benchmark read from files.

* ``targets_<name>.txt``: the daily-deaths target of a differentiable
  workload, i.e. the oracle's daily deaths at R = 3.0 with simulation seed 1
  (the runs being calibrated use R = 2.5, seed 0).
* ``oracle_run_<name>.txt`` (with ``--run``): the oracle's run of the
  workload itself (its own R, seed 0) against that target: the daily stage
  counts, the daily removals ``drm`` and the loss.  A full-size run of the
  largest workload takes the oracle minutes, so the GPU test compares with
  this record instead of running the oracle.

Only the oracle is called.
Usage: python tests/golden/make_targets.py [--run] [names...]
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from synth import make_workload  # noqa: E402


def target_for(name: str) -> np.ndarray:
    wl = make_workload(name)
    r = O.run_workload(wl, mode=O.PLAIN, seed=1, R=np.full(wl.K, 3.0, np.float32))
    return r["deaths"]


def read_target(name: str) -> np.ndarray:
    fn = os.path.join(HERE, f"targets_{name}.txt")
    return np.array([float(l) for l in open(fn) if l.strip() and not l.startswith("#")])


def write_targets(name: str) -> None:
    d = target_for(name)
    fn = os.path.join(HERE, f"targets_{name}.txt")
    with open(fn, "w") as f:
        f.write(f"# daily deaths of workload {name}: oracle, R = 3.0, seed 1 (tests/golden/make_targets.py)\n")
        for x in d:
            f.write(f"{float(x)!r}\n")
    print(fn, len(d), float(d.sum()))


def write_run(name: str) -> None:
    wl = make_workload(name)
    tgt = read_target(name)[: wl.K]
    r = O.run_workload(wl, mode=O.PLAIN, target=tgt)
    fn = os.path.join(HERE, f"oracle_run_{name}.txt")
    with open(fn, "w") as f:
        f.write(f"# workload {name}: oracle run, own parameters, seed {wl.seed}, against targets_{name}.txt "
                f"(tests/golden/make_targets.py --run)\n")
        f.write(f"# n_agents {wl.n_agents} n_edges {wl.n_edges} K {wl.K}\n")
        f.write(f"loss {float(r['loss'])!r}\n")
        f.write("# day S E I R M drm (counts at the start of the day; drm of the day, none on day K)\n")
        for t in range(wl.K + 1):
            c = " ".join(str(int(x)) for x in r["counts"][t])
            d = str(int(r["drm"][t])) if t < wl.K else "-"
            f.write(f"{t} {c} {d}\n")
    print(fn, float(r["loss"]))


def read_run(name: str) -> dict:
    """Counts [K+1, 5], drm [K] and loss of a stored oracle run."""
    loss, rows = None, []
    for line in open(os.path.join(HERE, f"oracle_run_{name}.txt")):
        if line.startswith("#") or not line.strip():
            continue
        p = line.split()
        if p[0] == "loss":
            loss = float(p[1])
        else:
            rows.append(p)
    counts = np.array([[float(x) for x in p[1:6]] for p in rows])
    drm = np.array([float(p[6]) for p in rows[:-1]])
    return {"counts": counts, "drm": drm, "loss": loss}


def main(argv):
    run = "--run" in argv
    names = [a for a in argv if not a.startswith("--")] or ["c2", "c3"]
    for name in names:
        if run:
            write_run(name)
        else:
            write_targets(name)


if __name__ == "__main__":
    main(sys.argv[1:])
