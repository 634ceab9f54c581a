"""Pins of the oracle's Section 3.1 propagators (scheme "rk3"): F is RK-3
with the sixth-order centred advective flux, G is RK-3 with the first-order
upwind flux, both with second-order centred acoustic fluxes and no damping,
advection with velocity (U, V).

What fixes the expected values, independently of the oracle's flux form:
  * the sixth-order centred derivative converges at order 6 against the
    exact derivative of a smooth periodic function;
  * on one Fourier mode both right-hand sides equal the symbol matrix built
    from the point-stencil weights, and n RK-3 steps equal R(dt A)^n with
    R(Z) = I + Z + Z^2/2 + Z^3/6;
  * the paper's finding (Section 3.1): on the acoustic-advection example
    the original Parareal grows without bound while KSE-Parareal stays on
    the fine solution.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import operators as ops
from oracle import propagators as prop
from oracle.operators import Params
from paper_1510_02237_amd import workloads as W
from test_oracle_operators import apply_complex
from test_oracle_propagators import rk3_poly


def _prm(**kw):
    base = dict(nx=32, nz=16, c_s=1.0, U=0.7, V=-0.4, dt_f=1e-3, dt_g=6e-3,
                P=1, T=6e-3, nu_f=0.0, nu_c=0.0, n_sound=1, scheme="rk3")
    base.update(kw)
    return Params(**base)


def test_rk3_scheme_rejects_rotation():
    with pytest.raises(ValueError):
        _prm(gamma=1.0)


def test_centred6_is_sixth_order():
    errs, hs = [], []
    for n in (32, 64, 128):
        x = (np.arange(n) + 0.5) / n
        f = np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x)
        exact = 2 * np.pi * np.cos(2 * np.pi * x) - 1.8 * np.pi * np.sin(6 * np.pi * x)
        q = np.tile(f, (4, 1))
        d = ops.flux_div(ops.flux_centred6(q, 1), 1.0 / n, 1)[0]
        errs.append(np.abs(d - exact).max())
        hs.append(1.0 / n)
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(2)]
    assert min(orders) > 5.7


def rk3_symbol(prm, kx, kz, coarse):
    """Symbol matrix of the Section 3.1 right-hand side from the stencil
    weights: centred-6 derivative (-1, 9, -45, 0, 45, -9, 1)/60 on i-3..i+3,
    first-order upwind (1 - e^{-i theta}) for a positive velocity (mirrored
    for a negative one), centred-2 acoustics i sin(theta)."""
    tx, tz = 2 * np.pi * kx / prm.nx, 2 * np.pi * kz / prm.nz
    e = lambda m, t: np.exp(1j * m * t)

    def c6(t, h):
        return (-e(-3, t) + 9 * e(-2, t) - 45 * e(-1, t) + 45 * e(1, t)
                - 9 * e(2, t) + e(3, t)) / (60 * h)

    def up1(t, h, vel):
        return (1 - e(-1, t)) / h if vel >= 0 else (e(1, t) - 1) / h

    if coarse:
        adv = prm.U * up1(tx, prm.dx, prm.U) + prm.V * up1(tz, prm.dz, prm.V)
    else:
        adv = prm.U * c6(tx, prm.dx) + prm.V * c6(tz, prm.dz)
    dx2 = 1j * np.sin(tx) / prm.dx
    dz2 = 1j * np.sin(tz) / prm.dz
    c = prm.c_s
    return np.array([[-adv, 0, -c * dx2],
                     [0, -adv, -c * dz2],
                     [-c * dx2, -c * dz2, -adv]])


@pytest.mark.parametrize("coarse", [False, True])
@pytest.mark.parametrize("U,V", [(0.7, -0.4), (-1.0, 1.0), (0.0, 0.5)])
@pytest.mark.parametrize("kx,kz", [(1, 0), (3, -2), (16, 8), (5, 7)])
def test_rhs_symbol(coarse, U, V, kx, kz):
    prm = _prm(U=U, V=V)
    v = np.array([0.3 - 0.2j, 1.0, -0.5j])
    got = apply_complex(lambda q: ops.rhs_rk3_pair(q, prm, coarse), prm,
                        kx, kz, v)
    want = rk3_symbol(prm, kx, kz, coarse) @ v
    # scale of the operator (a mode can make the symbol vanish, e.g. the
    # centred ones at theta = pi)
    scale = (abs(prm.U) + prm.c_s) / prm.dx + (abs(prm.V) + prm.c_s) / prm.dz
    assert np.abs(got - want).max() <= 1e-13 * scale * np.abs(v).max()


@pytest.mark.parametrize("kx,kz", [(1, 1), (4, -3), (16, 8)])
def test_F_and_G_single_mode_closed_form(kx, kz):
    prm = _prm()
    v = np.array([1.0, 0.2 + 0.4j, -0.3])
    got = apply_complex(lambda q: prop.fine_F(q, prm, 5), prm, kx, kz, v)
    R = rk3_poly(prm.dt_f * rk3_symbol(prm, kx, kz, False))
    want = np.linalg.matrix_power(R, 5) @ v
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    got = apply_complex(lambda q: prop.coarse_G(q, prm, 3), prm, kx, kz, v)
    R = rk3_poly(prm.dt_g * rk3_symbol(prm, kx, kz, True))
    want = np.linalg.matrix_power(R, 3) @ v
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_demo_workload_parameters():
    prob, K, u0 = W.config("demo_40x40")
    prm = Params(**prob)
    assert prm.scheme == "rk3" and (prm.U, prm.V, prm.c_s) == (1.0, 1.0, 1.0)
    assert prm.n_g == 1 and prm.n_f == 6 and prm.windows * prm.P == 72
    assert prm.T == pytest.approx(1.0)
    assert prm.dt_g * prm.U / prm.dx == pytest.approx(40 / 72)
    assert u0[0].max() <= 1.0 and u0[0].min() == 0.0 and not u0[1:].any()


@pytest.mark.parametrize("c_s", [1.0, 0.0])
def test_original_parareal_unstable_kse_stable(c_s):
    """Section 3.1: over the first windows of the example, max|q| of the
    original Parareal grows by orders of magnitude, KSE-Parareal stays with
    the fine solution (c_s = 0 is the pure-advection case of the paper's
    first figure, with u advected and w = p = 0)."""
    prob, K, u0 = W.config("demo_40x40")
    prob = dict(prob, c_s=c_s, windows=7)
    prob["T"] = 7 * prob["P"] * prob["dt_g"]
    prm = Params(**prob)
    par = oracle.kse_parareal(u0, prm, K=K, krylov=False)
    kse = oracle.kse_parareal(u0, prm, K=K)
    q = u0.copy()
    for w in range(prm.windows):
        for _ in range(prm.P):
            q = oracle.fine_F(q, prm)
        fmax = np.abs(q).max()
        # KSE follows the fine run's max|q| (the paper's figure: the lines
        # essentially coincide) ...
        assert abs(np.abs(kse["window_ends"][w]).max() - fmax) <= 0.05 * fmax, w
    assert oracle.rel_l2(kse["q"][prm.P], q) < 0.2
    # ... while the original Parareal grows without bound.
    amax = [np.abs(e).max() for e in par["window_ends"]]
    assert amax[-1] > 100 * fmax
    assert amax[-1] > 5 * amax[-2] > 25 * amax[-3]
