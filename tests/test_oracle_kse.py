"""Pins of the oracle's KSE-Parareal (Section 2.2, Algorithm 2) and of its
subspace update (eq. subspaceUpdate, eq. Genhance, eq. modifiedCoarse).

What fixes the expected values here, independently of the oracle's code:
  * Parareal reproduces the serial fine run on slices 0..k after k
    iterations, and everywhere after N_c iterations (Section 2.1);
  * every old iterate q^k_i lies in S^k, so K(q^k_i) = F(q^k_i) exactly in
    exact arithmetic -- this checks the F(S) bookkeeping of eq. Genhance;
  * dim S^k grows by at most N_c per iteration and, for generic data, by
    exactly the number of not-yet-converged slices (Section 2.3);
  * the method converges once dim S^k stops growing (Section 2.2);
  * an independent dense brute force on an 8x8 grid: F and G assembled as
    matrices, the projector taken from an SVD instead of a pivoted QR and
    F(P x) computed as M_F P x instead of through F(S);
  * LAPACK orthogonality, idempotence and linearity checks;
  * invariances: homogeneity and periodic shifts.
"""

import numpy as np
import pytest

import oracle
from oracle.operators import Params
from paper_1510_02237_amd import workloads as W


def small(nx=16, nz=8, P=4, U=0.1, T=1.0):
    return Params(**W.problem(nx, nz, P, U=U, T=T))


def u0_for(prm, seed=11, noise=1e-3):
    return W.ic_bumps(prm.nx, prm.nz, seed, nbumps=2, noise=noise, width=0.12)


def test_rel_l2_definition():
    a = np.array([[3.0, 4.0]])
    assert oracle.rel_l2(a, a) == 0.0
    assert oracle.rel_l2(np.zeros_like(a), a) == 1.0
    assert abs(oracle.rel_l2(a + np.array([[0.0, 5.0]]), a) - 1.0) < 1e-15


def test_subspace_update_invariants():
    prm = small(24, 16, P=6)
    u0 = u0_for(prm)
    out = oracle.kse_parareal(u0, prm, K=2)
    S, FS = out["S"], out["FS"]
    r = S.shape[1]
    assert np.abs(S.T @ S - np.eye(r)).max() <= 1e-12
    rng = np.random.default_rng(0)
    x = rng.normal(size=S.shape[0])
    Px = S @ (S.T @ x)
    assert np.linalg.norm(S @ (S.T @ Px) - Px) <= 1e-12 * np.linalg.norm(x)
    # P a = a for every raw column a = q^j_i that went into the basis.
    hist = oracle.kse_parareal(u0, prm, K=2, history=True)["iters"]
    for k in range(2):
        for i in range(prm.P):
            a = hist[k][i].ravel()
            assert np.linalg.norm(S @ (S.T @ a) - a) <= 1e-12 * np.linalg.norm(a)
    # Linearity (eq. Genhance): the stored F(S) is F applied to each s_j.
    for j in (0, r // 2, r - 1):
        fj = oracle.fine_F(S[:, j].reshape(u0.shape), prm).ravel()
        assert np.linalg.norm(fj - FS[:, j]) <= 1e-11 * np.linalg.norm(fj)


def test_K_equals_P_reproduces_serial_fine_bitwise():
    prm = small(16, 8, P=4)
    u0 = u0_for(prm)
    out = oracle.kse_parareal(u0, prm, K=prm.P, history=True)
    seq = [u0]
    for i in range(prm.P):
        seq.append(oracle.fine_F(seq[-1], prm))
    assert np.array_equal(out["q"][prm.P], seq[prm.P])
    # After k iterations slices 0..k are exact; slice k+1 is not (yet).
    for k, it in enumerate(out["iters"]):
        for i in range(min(k, prm.P) + 1):
            assert np.array_equal(it[i], seq[i]), (k, i)
        if k + 1 <= prm.P and k < prm.P:
            assert not np.array_equal(it[k + 1], seq[k + 1])


def test_K_of_old_iterate_equals_fine_result():
    """q^k_i is in S^k, so (I - P)q^k_i = 0 and K(q^k_i) = F(q^k_i)."""
    prm = small(24, 16, P=6)
    u0 = u0_for(prm)
    K = 2
    out = oracle.kse_parareal(u0, prm, K=K, history=True)
    q_prev = out["iters"][K - 1]
    for i in range(prm.P):
        kq = oracle.kse_apply(q_prev[i], out["S"], out["FS"], prm)
        ref = out["qt"][i + 1]
        assert np.linalg.norm(kq - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("P", [4, 8])
def test_rank_sequence(P):
    """dim S^k = sum_{j<=k} (P - j): q^k_0 = q_0 repeats every iteration and
    the j slices that have converged repeat their previous values."""
    prm = small(32, 16, P=P) if P == 8 else small(16, 8, P=P)
    out = oracle.kse_parareal(u0_for(prm), prm, K=min(P, 5))
    want = list(np.cumsum([P - j for j in range(len(out["ranks"]))]))
    assert out["ranks"] == want
    # The rank decision has a wide margin: kept columns sit far above the
    # tolerance, dropped ones at rounding level.
    for r, dg in zip(out["ranks"], out["diagR"]):
        assert dg[r - 1] / dg[0] > 1e-6
        if r < dg.size:
            assert dg[r] / dg[0] < 1e-13


def test_converges_once_dimension_stops_growing():
    """Section 2.2: once dim S^k no longer increases the iteration has
    converged to the serial fine solution (8x8 grid, 32 slices)."""
    prm = Params(**W.problem(8, 8, 32, U=0.1, T=8.0))
    rng = np.random.default_rng(7)
    u0 = rng.normal(size=(3, 8, 8))
    out = oracle.kse_parareal(u0, prm, K=7, history=True)
    ref = oracle.serial_fine(u0, prm)
    ranks = out["ranks"]
    k = next(k for k in range(1, len(ranks)) if ranks[k] == ranks[k - 1])
    assert oracle.rel_l2(out["iters"][k - 1][-1], ref) > 1e-3
    assert oracle.rel_l2(out["iters"][k][-1], ref) < 1e-8


# ------------------------------------------------------- dense brute force

def dense_operator(fn, shape):
    d = int(np.prod(shape))
    M = np.empty((d, d))
    for j in range(d):
        e = np.zeros(d)
        e[j] = 1.0
        M[:, j] = fn(e.reshape(shape)).ravel()
    return M


def dense_kse(u0, MF, MG, P, K, krylov=True, tol=1e-10):
    """Algorithm 2 with dense matrices; the projector comes from an SVD of
    the raw columns and F(P x) is M_F P x."""
    x0 = u0.ravel()
    q = [x0]
    for i in range(P):
        q.append(MG @ q[i])
    cols = []
    d = x0.size
    for _ in range(K):
        qt = [None] + [MF @ q[i] for i in range(P)]
        Pk = np.zeros((d, d))
        if krylov:
            cols += q[:P]
            Uu, s, _ = np.linalg.svd(np.stack(cols, axis=1), full_matrices=False)
            r = int(np.count_nonzero(s > tol * s[0]))
            Pk = Uu[:, :r] @ Uu[:, :r].T

        def Kop(x):
            px = Pk @ x
            return MG @ (x - px) + MF @ px

        new = [x0]
        for i in range(P):
            new.append(qt[i + 1] + Kop(new[i]) - Kop(q[i]))
        q = new
    return q


@pytest.mark.parametrize("krylov", [True, False])
def test_dense_brute_force_8x8(krylov):
    prm = Params(**W.problem(8, 8, 4, U=0.2))
    shape = (3, 8, 8)
    rng = np.random.default_rng(5)
    u0 = rng.normal(size=shape)
    MF = dense_operator(lambda q: oracle.fine_F(q, prm), shape)
    MG = dense_operator(lambda q: oracle.coarse_G(q, prm), shape)
    K = 3
    want = dense_kse(u0, MF, MG, prm.P, K, krylov=krylov)
    out = oracle.kse_parareal(u0, prm, K=K, krylov=krylov)
    for i in range(prm.P + 1):
        assert oracle.rel_l2(out["q"][i], want[i].reshape(shape)) <= 1e-12


def test_original_parareal_unstable_kse_stable_on_acoustics():
    """Section 3.1's observation in miniature: with the same F and G, the
    original Parareal's iterates are far from the fine run where KSE's are
    already close (U = 0.2 on a 16x8 grid, 8 slices)."""
    prm = Params(**W.problem(16, 8, 8, U=0.2))
    u0 = u0_for(prm)
    ref = oracle.serial_fine(u0, prm)
    e_kse = oracle.rel_l2(oracle.kse_parareal(u0, prm, K=3)["q"][-1], ref)
    e_par = oracle.rel_l2(oracle.parareal(u0, prm, K=3)["q"][-1], ref)
    assert e_kse < e_par


# ------------------------------------------------------------ invariances

def test_homogeneity():
    prm = small(16, 8, P=4)
    u0 = u0_for(prm)
    a = oracle.kse_parareal(u0, prm, K=2)["q"][-1]
    b = oracle.kse_parareal(2.0 * u0, prm, K=2)["q"][-1]
    assert np.abs(b - 2.0 * a).max() <= 1e-14 * np.abs(a).max()


def test_periodic_shift_equivariance():
    prm = small(16, 8, P=4)
    u0 = u0_for(prm)
    sh = lambda q: np.roll(np.roll(q, 3, axis=2), -2, axis=1)
    a = oracle.kse_parareal(u0, prm, K=2)["q"][-1]
    b = oracle.kse_parareal(sh(u0), prm, K=2)["q"][-1]
    assert oracle.rel_l2(b, sh(a)) <= 1e-12


def test_c1_error_decreases_per_iteration():
    """Section 3.2.4: each iteration lowers the error against the serial
    fine run (the paper reports about half an order of magnitude)."""
    prob, K, u0 = W.config("c1_64x32")
    prm = Params(**prob)
    ref = oracle.serial_fine(u0, prm)
    out = oracle.kse_parareal(u0, prm, K=K, history=True)
    errs = [oracle.rel_l2(it[-1], ref) for it in out["iters"]]
    assert all(errs[k + 1] < 0.8 * errs[k] for k in range(K))
    assert out["ranks"] == [8, 15, 21]


# ----------------------------------------------- stopping criterion r^k

def test_residual_is_the_iterate_difference():
    """r^k of Section 2.1 against differences of the stored iterates."""
    prm = small(16, 8, P=4)
    u0 = u0_for(prm)
    out = oracle.kse_parareal(u0, prm, K=3, history=True)
    it = out["iters"]
    for k, r in enumerate(out["residuals"]):
        num = max(np.linalg.norm(it[k + 1][i] - it[k][i]) for i in range(1, prm.P + 1))
        den = max(np.linalg.norm(it[k + 1][i]) for i in range(1, prm.P + 1))
        assert r == pytest.approx(num / den, rel=1e-14)


def test_residual_vanishes_once_every_slice_is_exact():
    """After P iterations all slices are the serial fine run (Section 2.1);
    one more iteration changes nothing, so r^P = 0 exactly."""
    prm = small(16, 8, P=4)
    out = oracle.kse_parareal(u0_for(prm), prm, K=prm.P + 1)
    assert out["residuals"][prm.P] == 0.0
    assert out["residuals"][prm.P - 1] > 0.0


def test_stopping_criterion_stops_at_first_small_residual():
    prm = small(24, 16, P=6)
    u0 = u0_for(prm)
    full = oracle.kse_parareal(u0, prm, K=6)
    tol = 0.5 * (full["residuals"][1] + full["residuals"][2])
    assert full["residuals"][2] < tol < full["residuals"][1]
    stop = oracle.kse_parareal(u0, prm, K=6, stop_tol=tol)
    assert stop["iterations"] == 3
    part = oracle.kse_parareal(u0, prm, K=3)
    assert all(np.array_equal(a, b) for a, b in zip(stop["q"], part["q"]))
