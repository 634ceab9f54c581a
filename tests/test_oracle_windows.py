"""Pins of the oracle's windowed KSE-Parareal: the parallel steps of
Section 2.1 run one after the other, each from the previous window's final
state and from an empty subspace (the initialization of Algorithm 2).

What fixes the expected values, independently of the windowed driver:
  * with K = P iterations every window reproduces the serial fine run over
    its slices (Section 2.1), so the windows together reproduce F applied
    windows * P times, computed here with a plain loop over fine_F;
  * with K = 0 every window is the coarse prediction, so the windows
    together give G applied windows * P times;
  * two windows equal two separate one-window solves of half the length,
    the second started from the first one's result;
  * the subspace restarts in every window: each window's ranks follow the
    sum_j (P - j) sequence of a fresh run.
"""

import numpy as np
import pytest

import oracle
from oracle.operators import Params
from paper_1510_02237_amd import workloads as W


def windowed(nx=16, nz=8, P=4, windows=3, U=0.1):
    """One coarse step per slice: T = windows * P * dt_g."""
    prob = W.problem(nx, nz, P, U=U, windows=windows)
    prob["T"] = windows * P * prob["dt_g"]
    return Params(**prob)


def u0_for(prm, seed=5):
    return W.ic_bumps(prm.nx, prm.nz, seed, nbumps=2, noise=1e-3, width=0.12)


def test_slice_is_one_coarse_step():
    prm = windowed()
    assert prm.n_g == 1 and prm.n_f == 10
    assert prm.slice_length == pytest.approx(prm.dt_g)
    for name in ("c1w_64x32", "c2w_512x256"):
        prob, K, u0 = W.config(name)
        p = Params(**prob)
        assert p.n_g == 1 and p.windows * p.P * p.dt_g == pytest.approx(p.T)


def test_K_equals_P_gives_serial_fine_over_all_windows():
    prm = windowed(P=4, windows=3)
    u0 = u0_for(prm)
    out = oracle.kse_parareal(u0, prm, K=prm.P)
    q = u0.copy()
    for w in range(prm.windows):
        for _ in range(prm.P):
            q = oracle.fine_F(q, prm)
        assert np.array_equal(out["window_ends"][w], q), w
    assert np.array_equal(oracle.serial_fine(u0, prm), q)


def test_K_zero_is_the_chained_coarse_run():
    prm = windowed(P=4, windows=3)
    u0 = u0_for(prm)
    out = oracle.kse_parareal(u0, prm, K=0)
    q = u0.copy()
    for w in range(prm.windows):
        for _ in range(prm.P):
            q = oracle.coarse_G(q, prm)
        assert np.array_equal(out["window_ends"][w], q), w


@pytest.mark.parametrize("krylov", [True, False])
def test_two_windows_are_two_chained_solves(krylov):
    prm2 = windowed(P=4, windows=2)
    half = Params(**{**prm2.__dict__, "windows": 1, "T": prm2.T / 2})
    u0 = u0_for(prm2)
    K = 2
    both = oracle.kse_parareal(u0, prm2, K=K, krylov=krylov)
    first = oracle.kse_parareal(u0, half, K=K, krylov=krylov)
    second = oracle.kse_parareal(first["q"][half.P], half, K=K, krylov=krylov)
    assert np.array_equal(both["window_ends"][0], first["q"][half.P])
    assert np.array_equal(both["q"][prm2.P], second["q"][half.P])


def test_subspace_restarts_in_every_window():
    prm = windowed(24, 16, P=6, windows=3)
    out = oracle.kse_parareal(u0_for(prm), prm, K=3)
    want = list(np.cumsum([prm.P - j for j in range(3)]))
    assert out["window_ranks"] == [want] * prm.windows


def test_windowed_kse_beats_coarse_only():
    """c1w (the paper's decomposition of the 64x32 run): each iteration
    brings the windowed solution closer to the serial fine run."""
    prob, K, u0 = W.config("c1w_64x32")
    prm = Params(**prob)
    ref = oracle.serial_fine(u0, prm)
    eps = [oracle.rel_l2(oracle.kse_parareal(u0, prm, K=k)["q"][prm.P], ref)
           for k in range(K + 1)]
    assert eps[-1] < 0.5 * eps[0]
    assert all(b < a for a, b in zip(eps, eps[1:]))
