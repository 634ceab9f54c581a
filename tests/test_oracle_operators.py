"""Pins of the oracle's spatial operators against calculus and Fourier
symbols (Section 3: flux-form finite differences; eq. acousticAd;
eq. dampingCoeff).

None of these tests reuses the oracle's own formulas: convergence orders are
measured against exact derivatives of smooth periodic functions, and the
single-mode tests compare with the Fourier symbol of the equivalent
point stencil, derived independently of the flux form the oracle uses.
"""

import math

import numpy as np
import pytest

from oracle import operators as ops
from oracle.operators import Params

pytestmark = pytest.mark.filterwarnings("ignore")


def _grid(nx, nz):
    x = (np.arange(nx) + 0.5) / nx
    z = (np.arange(nz) + 0.5) / nz
    return np.meshgrid(x, z)


def _order(errs, hs):
    return [math.log(errs[i] / errs[i + 1]) / math.log(hs[i] / hs[i + 1])
            for i in range(len(errs) - 1)]


# ------------------------------------------------------------------ orders

@pytest.mark.parametrize("U", [0.7, -0.7])
def test_upwind5_is_fifth_order(U):
    """The 6-point upwind-biased stencil of order 5 is unique, so measuring
    order 5 pins its coefficients (and the upwind side for either sign)."""
    errs, hs = [], []
    for n in (32, 64, 128):
        X, _ = _grid(n, 4)
        q = np.sin(2 * np.pi * X) + 0.3 * np.cos(6 * np.pi * X)
        exact = 2 * np.pi * np.cos(2 * np.pi * X) - 1.8 * np.pi * np.sin(6 * np.pi * X)
        tend = ops.flux_div(ops.flux_upwind5(q, U, 1), 1.0 / n, 1)  # = U q_x
        errs.append(np.abs(tend / U - exact).max())
        hs.append(1.0 / n)
    assert min(_order(errs, hs)) > 4.8


@pytest.mark.parametrize("flux,order", [("centred4", 4), ("centred2", 2)])
@pytest.mark.parametrize("axis", [0, 1])
def test_centred_orders(flux, order, axis):
    errs, hs = [], []
    for n in (16, 32, 64, 128):
        X, Z = _grid(n, n)
        C = X if axis == 1 else Z
        q = np.sin(2 * np.pi * C) + 0.5 * np.sin(4 * np.pi * C + 1.0)
        exact = 2 * np.pi * np.cos(2 * np.pi * C) + 2 * np.pi * np.cos(4 * np.pi * C + 1.0)
        f = getattr(ops, "flux_" + flux)(q, axis)
        errs.append(np.abs(ops.flux_div(f, 1.0 / n, axis) - exact).max())
        hs.append(1.0 / n)
    assert min(_order(errs, hs)) > order - 0.2
    assert max(_order(errs, hs)) < order + 0.5


def test_upwind1_first_order():
    errs, hs = [], []
    for n in (32, 64, 128, 256):
        X, _ = _grid(n, 4)
        q = np.sin(2 * np.pi * X)
        exact = 2 * np.pi * np.cos(2 * np.pi * X)
        errs.append(np.abs(ops.flux_div(ops.flux_upwind1(q, 1.0, 1), 1.0 / n, 1)
                           - exact).max())
        hs.append(1.0 / n)
    o = _order(errs, hs)
    assert 0.9 < min(o) and max(o) < 1.1


def test_grad_div_second_order():
    """(div u)_x and (div u)_z against the exact second derivatives."""
    errs, hs = [], []
    for n in (32, 64, 128):
        X, Z = _grid(n, n // 2)
        a, b = 2 * np.pi, 4 * np.pi
        u = np.sin(a * X) * np.cos(b * Z)
        w = np.cos(a * X + 0.3) * np.sin(b * Z)
        # div = a cos(aX)cos(bZ) + b cos(aX+.3)cos(bZ)
        dxdiv = -a * a * np.sin(a * X) * np.cos(b * Z) - a * b * np.sin(a * X + 0.3) * np.cos(b * Z)
        dzdiv = -a * b * np.cos(a * X) * np.sin(b * Z) - b * b * np.cos(a * X + 0.3) * np.sin(b * Z)
        gx, gz = ops.grad_div(u, w, 1.0 / n, 2.0 / n)
        errs.append(max(np.abs(gx - dxdiv).max(), np.abs(gz - dzdiv).max()))
        hs.append(1.0 / n)
    o = _order(errs, hs)
    assert min(o) > 1.8


# ---------------------------------------------------------- Fourier symbols

def _symbols(tx, tz, dx, dz, U):
    """Point-stencil symbols, written from the stencil weights:
    upwind-5 derivative (-2,15,-60,20,30,-3)/60 on i-3..i+2 for U >= 0
    (mirrored for U < 0), centred-4 (1,-8,0,8,-1)/12, compact grad-div."""
    e = lambda m, t: np.exp(1j * m * t)
    if U >= 0:
        a5 = (-2 * e(-3, tx) + 15 * e(-2, tx) - 60 * e(-1, tx) + 20
              + 30 * e(1, tx) - 3 * e(2, tx)) / (60 * dx)
        a1 = (1 - e(-1, tx)) / dx
    else:
        a5 = (3 * e(-2, tx) - 30 * e(-1, tx) - 20 + 60 * e(1, tx)
              - 15 * e(2, tx) + 2 * e(3, tx)) / (60 * dx)
        a1 = (e(1, tx) - 1) / dx
    dx4 = 1j * (8 * np.sin(tx) - np.sin(2 * tx)) / (6 * dx)
    dz4 = 1j * (8 * np.sin(tz) - np.sin(2 * tz)) / (6 * dz)
    dx2 = 1j * np.sin(tx) / dx
    dz2 = 1j * np.sin(tz) / dz
    gxx = -4 * np.sin(tx / 2) ** 2 / dx ** 2
    gzz = -4 * np.sin(tz / 2) ** 2 / dz ** 2
    gxz = -np.sin(tx) * np.sin(tz) / (dx * dz)
    return dict(a5=a5, a1=a1, dx4=dx4, dz4=dz4, dx2=dx2, dz2=dz2,
                gxx=gxx, gzz=gzz, gxz=gxz)


def fine_symbol(prm, kx, kz):
    tx, tz = 2 * np.pi * kx / prm.nx, 2 * np.pi * kz / prm.nz
    s = _symbols(tx, tz, prm.dx, prm.dz, prm.U)
    ax = prm.nu_f * prm.dx ** 2 / prm.dt_f
    az = prm.nu_f * prm.dz ** 2 / prm.dt_f
    c, U = prm.c_s, prm.U
    return np.array([
        [-U * s["a5"] + ax * s["gxx"], ax * s["gxz"], -c * s["dx4"]],
        [az * s["gxz"], -U * s["a5"] + az * s["gzz"], -c * s["dz4"]],
        [-c * s["dx4"], -c * s["dz4"], -U * s["a5"]]])


def mode(prm, kx, kz, v):
    """Real part of v e^{i(theta_x i + theta_z j)} as a (3, nz, nx) state,
    and the complex phase field."""
    jj, ii = np.meshgrid(np.arange(prm.nz), np.arange(prm.nx), indexing="ij")
    ph = np.exp(1j * (2 * np.pi * kx * ii / prm.nx + 2 * np.pi * kz * jj / prm.nz))
    return ph


def apply_complex(fn, prm, kx, kz, v):
    """Apply a real linear operator to v e^{i theta.x} via its real and
    imaginary parts; return the complex 3-vector it multiplies the phase by."""
    ph = mode(prm, kx, kz, v)
    q = np.stack([vi * ph for vi in v])
    out = fn(q.real) + 1j * fn(q.imag)
    coef = out / ph[None]
    # The result must be a pure mode: the same coefficient at every point.
    assert np.abs(coef - coef[:, :1, :1]).max() < 1e-9 * (1 + np.abs(coef).max())
    return coef[:, 0, 0]


@pytest.mark.parametrize("U", [0.1, -0.25, 0.0])
@pytest.mark.parametrize("kx,kz", [(1, 0), (0, 1), (3, 2), (5, -3), (16, 8), (31, 15)])
def test_fine_rhs_symbol(U, kx, kz):
    prm = Params(nx=64, nz=32, c_s=1.3, U=U, dt_f=1e-3, dt_g=1e-2, P=1)
    rng = np.random.default_rng(kx * 100 + kz)
    v = rng.normal(size=3) + 1j * rng.normal(size=3)
    got = apply_complex(lambda q: ops.rhs_fine(q, prm), prm, kx, kz, v)
    want = fine_symbol(prm, kx, kz) @ v
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


def test_acoustic_operator_is_energy_neutral():
    """With U = 0 and no damping the semi-discrete acoustic operator is
    skew-symmetric, so <q, f(q)> = 0: the total energy of eq. acousticAd
    (Section 3.2.3) is conserved by the spatial discretisation."""
    prm = Params(nx=24, nz=16, c_s=1.0, U=0.0, dt_f=1e-3, dt_g=1e-2, P=1,
                 nu_f=0.0)
    rng = np.random.default_rng(0)
    for _ in range(3):
        q = rng.normal(size=(3, 16, 24))
        f = ops.rhs_fine(q, prm)
        assert abs(np.sum(q * f)) < 1e-10 * np.sum(q * q) * 24 * 6


def test_upwind_and_damping_dissipate():
    """Upwinding and divergence damping only remove energy."""
    prm = Params(nx=24, nz=16, c_s=0.0, U=0.3, dt_f=1e-3, dt_g=1e-2, P=1)
    rng = np.random.default_rng(1)
    for _ in range(3):
        q = rng.normal(size=(3, 16, 24))
        assert np.sum(q * ops.rhs_fine(q, prm)) < 0.0


def test_coarse_slow_tendency_symbol():
    prm = Params(nx=32, nz=16, c_s=1.0, U=0.2, dt_f=1e-3, dt_g=1e-2, P=1)
    for kx, kz in [(1, 0), (4, 3), (16, 8)]:
        v = np.array([1.0, -0.5 + 0.2j, 0.3j])
        got = apply_complex(lambda q: ops.coarse_slow_tendency(q, prm), prm, kx, kz, v)
        s = _symbols(2 * np.pi * kx / 32, 2 * np.pi * kz / 16, prm.dx, prm.dz, prm.U)
        assert np.allclose(got, -prm.U * s["a1"] * v, rtol=1e-12, atol=1e-12)
