"""Krylov-subspace-enhanced Parareal in the oracle (Section 2.2, Algorithm 2).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Notation follows the paper: q^k_i is the iterate at t_i in iteration k,
qt^k_{i+1} = F(q^k_i) the fine result, S^k the span of every q^j_i seen so
far (j <= k, i < N_c), F(S^k) the fine images, P^k the Euclidean orthogonal
projector onto S^k.

The subspace update is done as the paper does it: a full QR decomposition
with column pivoting of all raw columns, every iteration (eq.
subspaceUpdate; the paper calls LAPACK DGEQP3, which is exactly what
``scipy.linalg.qr(pivoting=True)`` runs).  Because the problem is linear,
F of an orthonormal basis vector is the same combination of the stored fine
results (eq. Genhance): with A Pi = Q R, S = Q[:, :r] = A Pi[:, :r] R_r^{-1},
so F(S) = F(A) Pi[:, :r] R_r^{-1}.  The rank r counts |R_jj| > rank_tol *
|R_11|.

Readings taken where the paper is silent (also listed with the design notes):
  * the correction is evaluated as qt + (K(new) - K(old)), algebraically the
    same as Algorithm 2's K(new) + qt - K(old); it keeps slices that have
    converged bitwise equal to the serial fine run;
  * the iteration count is fixed (no stopping test, Section 2.1);
  * windows (the parallel steps of Section 2.1) run one after the other,
    each starting from the previous window's final state q^K_P and, as
    Algorithm 2's initialization says, from an empty subspace.
"""

import numpy as np
import scipy.linalg

from .operators import Params
from .propagators import fine_F, coarse_G


def rel_l2(q_par, q_seq):
    """epsilon of eq. errorDef: ||q_par - q_seq||_2 / ||q_seq||_2 over all
    three fields."""
    a = np.asarray(q_par, dtype=np.float64).ravel()
    b = np.asarray(q_seq, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def subspace_update(A, FA, rank_tol):
    """Orthonormal basis S of span(A) and F(S) (eq. subspaceUpdate,
    eq. Genhance).

    A, FA: (d, m) raw columns q^j_i and their fine images.
    Returns (S (d, r), FS (d, r), |diag R| (m,)).
    """
    A = np.asarray(A, dtype=np.float64)
    FA = np.asarray(FA, dtype=np.float64)
    if A.shape[1] == 0:
        return A[:, :0].copy(), FA[:, :0].copy(), np.zeros(0)
    Q, R, piv = scipy.linalg.qr(A, mode="economic", pivoting=True)
    diag = np.abs(np.diag(R))
    r = int(np.count_nonzero(diag > rank_tol * diag[0])) if diag[0] > 0 else 0
    S = Q[:, :r]
    # F(S) = F(A[:, piv[:r]]) R_r^{-1}, i.e. solve X R_r = FA[:, piv[:r]].
    FS = scipy.linalg.solve_triangular(R[:r, :r], FA[:, piv[:r]].T,
                                       trans="T", lower=False).T
    return S, FS, diag


def kse_apply(x, S, FS, prm: Params):
    """K(x) = G((I - P) x) + F(P x) with P = S S^T and F(P x) = F(S) S^T x
    (eq. modifiedCoarse, eq. Genhance).  An empty basis gives G(x)."""
    shape = np.shape(x)
    v = np.asarray(x, dtype=np.float64).ravel()
    if S.shape[1] == 0:
        return coarse_G(v.reshape(shape), prm)
    alpha = S.T @ v
    perp = v - S @ alpha
    return coarse_G(perp.reshape(shape), prm) + (FS @ alpha).reshape(shape)


def _vec(states):
    return np.stack([np.asarray(s, dtype=np.float64).ravel() for s in states],
                    axis=1)


def residual(new, old):
    """The error estimate of Section 2.1, r^k = max_i ||q^{k+1}_i - q^k_i||
    (Euclidean norm over all fields, i = 1..N_c), divided by
    max_i ||q^{k+1}_i|| so that it does not depend on the scale of u0."""
    num = max(np.linalg.norm(np.ravel(a) - np.ravel(b))
              for a, b in zip(new[1:], old[1:]))
    den = max(np.linalg.norm(np.ravel(a)) for a in new[1:])
    return float(num / den) if den > 0 else 0.0


def kse_parareal(u0, prm: Params, K, krylov=True, history=False,
                 stop_tol=0.0):
    """Algorithm 2 (or Algorithm 1 with ``krylov=False``, i.e. S = empty)
    over the ``prm.windows`` parallel steps of Section 2.1.

    With ``stop_tol`` > 0 a window stops after the first iteration k whose
    error estimate ``residual`` is <= stop_tol (Section 2.1's stopping
    criterion), K being the maximum; ``residuals`` and ``iterations`` of the
    last window are returned.

    Returns the last window's dict (see ``_one_window``) with, in addition,
      window_ends   the final state q^K_P of every window
      window_ranks  ``ranks`` of every window (krylov only)
    With one window this is exactly ``_one_window``'s result plus those two
    entries.
    """
    u = np.asarray(u0, dtype=np.float64)
    ends, wranks = [], []
    out = None
    for _ in range(prm.windows):
        out = _one_window(u, prm, K, krylov=krylov, history=history,
                          stop_tol=stop_tol)
        u = out["q"][prm.P]
        ends.append(u)
        if krylov:
            wranks.append(out["ranks"])
    out["window_ends"] = ends
    if krylov:
        out["window_ranks"] = wranks
    return out


def _one_window(u0, prm: Params, K, krylov=True, history=False,
                stop_tol=0.0):
    """One parallel step of Algorithm 2 (Algorithm 1 with ``krylov=False``)
    on the P slices that start at u0.

    Returns a dict:
      q       list of P+1 states q^K_0..q^K_P (q[P] is the window's end)
      ranks   dim S^k after each iteration's update (krylov only)
      diagR   |R_jj| of each iteration's pivoted QR (krylov only)
      S, FS   the last basis and its fine images (krylov only)
      qt      the last iteration's fine results, qt[i+1] = F(q^{K-1}_i)
      iters   with history=True: q^k for k = 0..K
      residuals  r^k of every iteration done (see ``residual``)
      iterations the number of iterations done
    """
    u0 = np.asarray(u0, dtype=np.float64)
    P = prm.P
    shape = u0.shape
    d = u0.size
    # Initialization: coarse prediction over all slices.
    q = [u0.copy()]
    for i in range(P):
        q.append(coarse_G(q[i], prm))
    A_cols, FA_cols = [], []
    S = np.zeros((d, 0))
    FS = np.zeros((d, 0))
    ranks, diags, iters = [], [], [list(q)] if history else None
    qt = None
    residuals = []
    for k in range(K):
        # Parallel predictor step.
        qt = [None] + [fine_F(q[i], prm) for i in range(P)]
        if krylov:
            # Update S^{k-1} -> S^k and F(S^k) with the pairs (q^k_i, qt^k_{i+1}).
            A_cols += [q[i] for i in range(P)]
            FA_cols += [qt[i + 1] for i in range(P)]
            S, FS, diag = subspace_update(_vec(A_cols), _vec(FA_cols),
                                          prm.rank_tol)
            ranks.append(S.shape[1])
            diags.append(diag)
        # Sequential correction step.
        new = [u0.copy()]
        for i in range(P):
            k_new = kse_apply(new[i], S, FS, prm)
            k_old = kse_apply(q[i], S, FS, prm)
            new.append(qt[i + 1] + (k_new - k_old))
        residuals.append(residual(new, q))
        q = new
        if history:
            iters.append(list(q))
        if stop_tol > 0 and residuals[-1] <= stop_tol:
            break
    out = {"q": q, "qt": qt, "residuals": residuals,
           "iterations": len(residuals)}
    if krylov:
        out.update(ranks=ranks, diagR=diags, S=S, FS=FS)
    if history:
        out["iters"] = iters
    return out


def parareal(u0, prm: Params, K, history=False):
    """Algorithm 1: the original Parareal (the S = empty case of Algorithm 2)."""
    return kse_parareal(u0, prm, K, krylov=False, history=history)
