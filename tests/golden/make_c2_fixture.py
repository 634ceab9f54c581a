"""Writes tests/golden/c2_512x256_oracle.json with the oracle's own results
for the benchmark workload (512 x 256 grid, P = 32, K = 4; seeded initial
state from paper_1510_02237_amd.workloads): the relative l2 error of every
iterate's final slice against the serial fine run (eq. errorDef), the basis
dimensions after each subspace update (Algorithm 2), and 64 seeded samples
of the final iterate q^K_P.  Calls only the oracle and the input generator.

    python tests/golden/make_c2_fixture.py     (about 5 minutes on one core)
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.operators import Params  # noqa: E402
from paper_1510_02237_amd import workloads as W  # noqa: E402


def main():
    prob, K, u0 = W.config("c2_512x256")
    prm = Params(**prob)
    ref = oracle.serial_fine(u0, prm)
    out = oracle.kse_parareal(u0, prm, K=K, history=True)
    qK = out["q"][-1]
    errs = [oracle.rel_l2(it[-1], ref) for it in out["iters"]]
    rng = np.random.default_rng(2024)
    idx = rng.choice(qK.size, size=64, replace=False)
    flat = qK.ravel()
    res = dict(
        source="oracle.kse_parareal (Algorithm 2) and oracle.serial_fine on "
               "workloads.config('c2_512x256')",
        K=K, P=prob["P"], ranks=[int(r) for r in out["ranks"]],
        eps_vs_serial_fine=errs,
        final_norm2=float(np.linalg.norm(flat)),
        final_max=float(np.abs(flat).max()),
        sample_index=[int(i) for i in idx],
        sample_value=[float(flat[i]) for i in idx])
    with open(os.path.join(HERE, "c2_512x256_oracle.json"), "w") as f:
        json.dump(res, f, indent=1)
    print("errors", errs, "ranks", out["ranks"])


if __name__ == "__main__":
    main()
