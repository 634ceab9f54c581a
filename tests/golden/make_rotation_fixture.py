"""Writes tests/golden/rotation_40x40_oracle.json with the oracle's own
results for the solid-body-rotation runs of Section 3.2 on 40 x 40 cells
(workloads.rotation_problem: c_s = 30, fine CFL 0.2, T = 2, one coarse step
per slice, windows of P slices): for every cell (coarse CFL, P, K) of
Tables 1 and 2 the relative l2 error of the windowed KSE-Parareal result at
T = 2 against the serial fine run (eq. errorDef), plus 64 seeded samples of
the final state of the cell (4, 6, 2) -- the rot_40x40 workload -- and of
the serial fine run.  Calls only the oracle and the input generator.

    python tests/golden/make_rotation_fixture.py    (about 5 minutes on 8 cores)
"""

import json
import os
import sys

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.operators import Params  # noqa: E402
from paper_1510_02237_amd import workloads as W  # noqa: E402

N = 40
CENTRE = (0.5, 0.65)
SAMPLE_CELL = (4.0, 6, 2)


def _u0():
    return W.ic_cosine_bell(N, N, centre=CENTRE)


def _cell(args):
    cc, P, K = args
    prm = Params(**W.rotation_problem(N, P, cc))
    return args, oracle.kse_parareal(_u0(), prm, K=K)["q"][prm.P]


def _serial(_):
    prm = Params(**W.rotation_problem(N, 6, 4.0))
    return oracle.serial_fine(_u0(), prm)


def main():
    from multiprocessing import Pool
    cells = sorted(W.PAPER_TABLE_CELLS, key=lambda c: -c[2])  # long first
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        ref_async = pool.map_async(_serial, [0])
        results = dict(pool.map(_cell, cells))
        ref = ref_async.get()[0]
    rng = np.random.default_rng(2025)
    idx = rng.choice(ref.size, size=64, replace=False)
    fin = results[SAMPLE_CELL].ravel()
    res = dict(
        source="oracle.kse_parareal (Algorithm 2, windows) and "
               "oracle.serial_fine on workloads.rotation_problem(40, P, cfl_c) "
               "from workloads.ic_cosine_bell(40, 40, centre=(0.5, 0.65))",
        cells=[dict(cfl_c=cc, P=P, K=K,
                    eps=oracle.rel_l2(results[(cc, P, K)], ref))
               for (cc, P, K) in W.PAPER_TABLE_CELLS],
        serial_norm2=float(np.linalg.norm(ref)),
        sample_cell=dict(cfl_c=SAMPLE_CELL[0], P=SAMPLE_CELL[1],
                         K=SAMPLE_CELL[2]),
        sample_index=[int(i) for i in idx],
        serial_sample=[float(ref.ravel()[i]) for i in idx],
        final_sample=[float(fin[i]) for i in idx],
        final_max=float(np.abs(fin).max()))
    with open(os.path.join(HERE, "rotation_40x40_oracle.json"), "w") as f:
        json.dump(res, f, indent=1)
    for c in res["cells"]:
        print(c)


if __name__ == "__main__":
    main()
