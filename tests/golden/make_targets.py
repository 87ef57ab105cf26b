"""Writes the daily-deaths targets of the differentiable workloads.

The target trajectory of a workload is the oracle's daily deaths at R = 3.0
with simulation seed 1 (the runs being calibrated use R = 2.5, seed 0).  Only
the oracle is called.  Usage: python tests/golden/make_targets.py [names...]
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


def main(names):
    for name in names:
        d = target_for(name)
        fn = os.path.join(HERE, f"targets_{name}.txt")
        with open(fn, "w") as f:
            f.write(f"# daily deaths of workload {name}: oracle, R = 3.0, seed 1 (tests/golden/make_targets.py)\n")
            for x in d:
                f.write(f"{float(x)!r}\n")
        print(fn, len(d), float(d.sum()))


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2", "c3"])
