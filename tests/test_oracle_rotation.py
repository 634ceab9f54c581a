"""Pins of the oracle's split scheme with a velocity that varies in space:
advection by (U + gamma (z - 1/2), V - gamma (x - 1/2)), the solid-body
rotation of eq. adVel when U = V = 0, and the option of second-order
acoustic fluxes in F (Section 3 computes the acoustic fluxes of both
propagators to second order).

What fixes the expected values, independently of the oracle's code:
  * constant velocity (gamma = 0, U and V of either sign): one Fourier mode
    evolves by the amplification matrices written here from the stencil
    weights (upwind-5 along both axes, mirrored for a negative component;
    second- or fourth-order centred acoustics);
  * the rotation field is invariant under a quarter turn of the square
    about its centre, and so is the discretisation on an n x n grid: F and
    G commute with the quarter turn of the grid that carries (u, w) as a
    vector and p as a scalar.  A wrong sign of the z-velocity, an upwind
    side taken from the wrong component, or a velocity table transposed
    between rows and columns breaks the symmetry;
  * with c_s = 0 and no damping every field is a passive scalar carried by
    the rotation (eq. acousticAd): after a quarter revolution the cosine
    bell sits at the exactly rotated position, clockwise for gamma > 0;
  * flux form: the domain sum of every field is conserved by F and G for
    any velocity of this family.
"""

import math

import numpy as np
import pytest

from oracle import propagators as prop
from oracle import operators as ops
from oracle.operators import Params
from paper_1510_02237_amd import workloads as W
from test_oracle_operators import apply_complex


def _prm(**kw):
    base = dict(nx=32, nz=16, c_s=1.0, U=0.1, V=-0.07, dt_f=0.2 / 32,
                dt_g=2.0 / 32, P=1, T=2.0 / 32)
    base.update(kw)
    return Params(**base)


def _e(m, t):
    return np.exp(1j * m * t)


def _up5(t, h, vel):
    """Upwind-5 derivative symbol from its point weights
    (-2, 15, -60, 20, 30, -3)/60 on i-3..i+2, mirrored for vel < 0."""
    if vel >= 0:
        return (-2 * _e(-3, t) + 15 * _e(-2, t) - 60 * _e(-1, t) + 20
                + 30 * _e(1, t) - 3 * _e(2, t)) / (60 * h)
    return (3 * _e(-2, t) - 30 * _e(-1, t) - 20 + 60 * _e(1, t)
            - 15 * _e(2, t) + 2 * _e(3, t)) / (60 * h)


def _up1(t, h, vel):
    return (1 - _e(-1, t)) / h if vel >= 0 else (_e(1, t) - 1) / h


def _centred(t, h, order):
    if order == 2:
        return 1j * np.sin(t) / h
    return 1j * (8 * np.sin(t) - np.sin(2 * t)) / (6 * h)


def _damping(tx, tz, dx, dz):
    gxx = -4 * np.sin(tx / 2) ** 2 / dx ** 2
    gzz = -4 * np.sin(tz / 2) ** 2 / dz ** 2
    gxz = -np.sin(tx) * np.sin(tz) / (dx * dz)
    return gxx, gzz, gxz


def fine_symbol_uv(prm, kx, kz):
    tx, tz = 2 * np.pi * kx / prm.nx, 2 * np.pi * kz / prm.nz
    adv = -prm.U * _up5(tx, prm.dx, prm.U) - prm.V * _up5(tz, prm.dz, prm.V)
    dx_, dz_ = (_centred(tx, prm.dx, prm.fine_acoustic_order),
                _centred(tz, prm.dz, prm.fine_acoustic_order))
    gxx, gzz, gxz = _damping(tx, tz, prm.dx, prm.dz)
    ax = prm.nu_f * prm.dx ** 2 / prm.dt_f
    az = prm.nu_f * prm.dz ** 2 / prm.dt_f
    c = prm.c_s
    return np.array([
        [adv + ax * gxx, ax * gxz, -c * dx_],
        [az * gxz, adv + az * gzz, -c * dz_],
        [-c * dx_, -c * dz_, adv]])


def coarse_symbol_uv(prm, kx, kz):
    """One partially split step: slow tendency -U a1(x) - V a1(z) frozen,
    N_sound forward-backward substeps with second-order acoustics."""
    tx, tz = 2 * np.pi * kx / prm.nx, 2 * np.pi * kz / prm.nz
    Rs = -prm.U * _up1(tx, prm.dx, prm.U) - prm.V * _up1(tz, prm.dz, prm.V)
    dx2, dz2 = _centred(tx, prm.dx, 2), _centred(tz, prm.dz, 2)
    gxx, gzz, gxz = _damping(tx, tz, prm.dx, prm.dz)
    dtau = prm.dt_g / prm.n_sound
    ax = prm.nu_c * prm.dx ** 2 / dtau
    az = prm.nu_c * prm.dz ** 2 / dtau
    c = prm.c_s
    E = np.eye(3)
    Y = np.eye(3, dtype=complex)
    for _ in range(prm.n_sound):
        u, w, p = Y
        un = u + dtau * (Rs * E[0] - c * dx2 * p + ax * (gxx * u + gxz * w))
        wn = w + dtau * (Rs * E[1] - c * dz2 * p + az * (gzz * w + gxz * u))
        pn = p + dtau * (Rs * E[2] - c * (dx2 * un + dz2 * wn))
        Y = np.array([un, wn, pn])
    return Y


def rk3_poly(Z):
    I = np.eye(3)
    return I + Z + Z @ Z / 2 + Z @ Z @ Z / 6


def test_parameters():
    Params(nx=8, nz=8, c_s=1.0, U=0.1, V=0.1, dt_f=1e-3, dt_g=1e-2, P=1)
    with pytest.raises(ValueError):
        Params(nx=8, nz=8, c_s=1.0, U=0.1, gamma=1.0, dt_f=1e-3, dt_g=1e-2,
               P=1, scheme="rk3")
    with pytest.raises(ValueError):
        Params(nx=8, nz=8, c_s=1.0, U=0.1, dt_f=1e-3, dt_g=1e-2, P=1,
               fine_acoustic_order=6)


def test_velocity_of_eq_adVel():
    prm = _prm(nx=40, nz=40, U=0.0, V=0.0, gamma=math.pi)
    ux, vz = ops.velocity_x(prm)[:, 0], ops.velocity_z(prm)[0]
    z = (np.arange(40) + 0.5) / 40
    assert np.allclose(ux, math.pi * (z - 0.5), rtol=0, atol=1e-15)
    assert np.allclose(vz, -math.pi * (z - 0.5), rtol=0, atol=1e-15)
    # largest speed along an axis about 1.5 (Section 3.2)
    assert 1.5 < np.abs(ux).max() < math.pi / 2


@pytest.mark.parametrize("order", [4, 2])
@pytest.mark.parametrize("U,V", [(0.1, -0.07), (-0.2, 0.15), (0.0, 0.2)])
@pytest.mark.parametrize("kx,kz", [(1, 1), (3, -2), (7, 5), (16, 8)])
def test_fine_single_mode_closed_form(order, U, V, kx, kz):
    prm = _prm(U=U, V=V, fine_acoustic_order=order)
    v = np.array([0.3 + 0.1j, -0.7, 1.0 - 0.4j])
    got = apply_complex(lambda q: prop.fine_F(q, prm, 5), prm, kx, kz, v)
    want = np.linalg.matrix_power(
        rk3_poly(prm.dt_f * fine_symbol_uv(prm, kx, kz)), 5) @ v
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("U,V", [(0.1, -0.07), (-0.05, 0.1)])
@pytest.mark.parametrize("kx,kz", [(1, 0), (0, 1), (2, 3), (9, -4), (16, 8)])
def test_coarse_single_mode_closed_form(U, V, kx, kz):
    prm = _prm(U=U, V=V)
    v = np.array([1.0, 0.2 - 0.5j, -0.3j])
    got = apply_complex(lambda q: prop.coarse_G(q, prm, 2), prm, kx, kz, v)
    want = np.linalg.matrix_power(coarse_symbol_uv(prm, kx, kz), 2) @ v
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def quarter_turn(q):
    """The state rotated a quarter turn clockwise about the centre of the
    n x n grid: value at cell (i', j') taken from cell (i, j) = (n-1-j', i'),
    with the velocity vector (u, w) turned to (w, -u)."""
    u, w, p = q
    return np.stack([np.rot90(w), -np.rot90(u), np.rot90(p)])


def test_quarter_turn_is_a_rotation_of_the_grid():
    """The map moves the cell centre (x, z) to (z, 1 - x), the clockwise
    quarter turn about (1/2, 1/2)."""
    n = 8
    X, Z = np.meshgrid((np.arange(n) + 0.5) / n, (np.arange(n) + 0.5) / n)
    q = np.stack([X, Z, X])
    r = quarter_turn(q)
    # rotated p at (x', z') equals the old x of its pre-image (1 - z', x')
    assert np.allclose(r[2], 1.0 - Z)


@pytest.mark.parametrize("order", [2, 4])
def test_F_and_G_commute_with_the_quarter_turn(order):
    prm = _prm(nx=24, nz=24, U=0.0, V=0.0, gamma=math.pi, c_s=3.0,
               dt_f=0.2 / (24 * 3.0), dt_g=2.0 / (24 * 3.0),
               fine_acoustic_order=order)
    rng = np.random.default_rng(11)
    q = rng.normal(size=(3, 24, 24))
    f1 = prop.fine_F(quarter_turn(q), prm, 3)
    f2 = quarter_turn(prop.fine_F(q, prm, 3))
    assert np.abs(f1 - f2).max() <= 1e-13 * np.abs(f2).max()
    g1 = prop.coarse_G(quarter_turn(q), prm, 2)
    g2 = quarter_turn(prop.coarse_G(q, prm, 2))
    assert np.abs(g1 - g2).max() <= 1e-13 * np.abs(g2).max()


def test_quarter_turn_symmetry_needs_the_rotation_field():
    """The symmetry is a property of the rotation: a constant velocity
    along x breaks it (the check above is not vacuous)."""
    prm = _prm(nx=24, nz=24, U=0.5, V=0.0, gamma=0.0, c_s=3.0,
               dt_f=0.2 / (24 * 3.0), dt_g=2.0 / (24 * 3.0))
    rng = np.random.default_rng(11)
    q = rng.normal(size=(3, 24, 24))
    f1 = prop.fine_F(quarter_turn(q), prm, 3)
    f2 = quarter_turn(prop.fine_F(q, prm, 3))
    assert np.abs(f1 - f2).max() > 1e-3 * np.abs(f2).max()


def _bell(n, centre):
    return W.ic_cosine_bell(n, n, centre=centre)[0]


def test_quarter_revolution_carries_the_bell_clockwise():
    """c_s = 0, no damping: u is carried by the rotation.  After t = 1/2
    (a quarter of the revolution period 2) the bell starting at (0.5, 0.65)
    lies at (0.65, 0.5); the counter-clockwise position (0.35, 0.5) is far
    off.  The error bound is the discretisation error of upwind-5 on a bell
    ten cells wide."""
    n = 80
    prm = Params(nx=n, nz=n, c_s=0.0, U=0.0, V=0.0, gamma=math.pi,
                 dt_f=1.0 / 500, dt_g=1.0 / 500, P=1, T=0.5, nu_f=0.0,
                 nu_c=0.0, n_sound=1)
    q0 = np.zeros((3, n, n))
    q0[0] = _bell(n, (0.5, 0.65))
    q = prop.fine_F(q0, prm, 250)
    cw, ccw = _bell(n, (0.65, 0.5)), _bell(n, (0.35, 0.5))
    err = np.linalg.norm(q[0] - cw) / np.linalg.norm(cw)
    assert err < 0.05
    assert np.linalg.norm(q[0] - ccw) / np.linalg.norm(ccw) > 1.0
    assert np.abs(q[1:]).max() == 0.0
    # the coarse propagator (first-order upwind, forward Euler at Courant
    # number 0.25 per direction) carries it the same way, smeared
    qg = prop.coarse_G(q0, prm, 250)
    assert (np.linalg.norm(qg[0] - cw) < 0.5 * np.linalg.norm(qg[0] - ccw))


@pytest.mark.parametrize("gamma,U,V", [(math.pi, 0.0, 0.0), (2.0, 0.3, -0.2)])
def test_flux_form_conserves_every_field(gamma, U, V):
    prm = _prm(nx=20, nz=12, U=U, V=V, gamma=gamma, c_s=2.0,
               dt_f=0.2 / (20 * 2.0), dt_g=2.0 / (20 * 2.0))
    rng = np.random.default_rng(4)
    q = rng.normal(size=(3, 12, 20))
    s0 = q.sum(axis=(1, 2))
    for out in (prop.fine_F(q, prm, 4), prop.coarse_G(q, prm, 2)):
        assert np.abs(out.sum(axis=(1, 2)) - s0).max() < 1e-11


def test_rotation_workloads_are_the_paper_runs():
    prob, K, u0 = W.config("rot_40x40")
    prm = Params(**prob)
    # fine CFL 0.2 and coarse CFL 4 (Table 2) with c_s = 30
    assert prm.c_s * prm.dt_f / prm.dx == pytest.approx(0.2)
    assert prm.c_s * prm.dt_g / prm.dx == pytest.approx(4.0)
    assert prm.n_g == 1 and prm.P == 6 and prm.windows == 100
    assert prm.windows * prm.P * prm.dt_g == pytest.approx(2.0)
    assert prm.fine_acoustic_order == 2 and prm.gamma == math.pi
    for cc, P, K in W.PAPER_TABLE_CELLS:
        p = Params(**W.rotation_problem(40, P, cc))
        assert p.n_g == 1 and p.n_f == round(cc / 0.2)


@pytest.mark.parametrize("cfl_c", [2.0, 4.0])
def test_rotation_propagators_do_not_grow(cfl_c):
    """The propagators of the paper's runs on the rotation field itself (not
    diagonalised by Fourier modes): 600 coarse steps and 200 fine steps from
    a random state grow its norm by less than 1 %.  A spectral radius of
    1.01 would grow it by a factor of about 400 over the coarse steps."""
    prm = Params(**W.rotation_problem(40, 6, cfl_c))
    rng = np.random.default_rng(0)
    q0 = rng.normal(size=(3, 40, 40))
    q = q0.copy()
    for _ in range(600):
        q = prop.coarse_step(q, prm)
    assert np.linalg.norm(q) < 1.01 * np.linalg.norm(q0)
    q = prop.fine_F(q0, prm, 200)
    assert np.linalg.norm(q) < 1.01 * np.linalg.norm(q0)


def test_frozen_coefficients_are_pessimistic_at_coarse_cfl_4():
    """Frozen at the corner velocity (both components 1.53), the coarse
    symbol of the coarse-CFL-4 run exceeds 1 on long waves, although the
    propagator on the rotation field does not grow (above): the Fourier
    scan is exact only for a constant velocity."""
    prm = Params(**W.rotation_problem(40, 6, 4.0))
    ux = ops.velocity_x(prm)[:, 0]
    p = Params(**{**prm.__dict__, "gamma": 0.0, "U": ux.max(),
                  "V": ux.max()})
    rho = max(np.abs(np.linalg.eigvals(coarse_symbol_uv(p, kx, kz))).max()
              for kx in range(6) for kz in range(6))
    assert rho > 1.04


def test_less_diffusive_G_grows_on_the_rotation_too():
    """The less diffusive G of Section 3.2 (third-order slow tendency,
    nu_c = 0.005, N_sound = 8, coarse CFL 2) on the rotating flow of the
    paper's energy runs: unlike the frozen-coefficient estimate of the main
    runs, its growth is real -- a factor above 100 in 200 steps."""
    prob = W.rotation_problem(40, 6, 2.0)
    prob.update(nu_f=0.0, nu_c=0.005, n_sound=8)
    prm = Params(**prob, coarse_order=3)
    rng = np.random.default_rng(0)
    q0 = rng.normal(size=(3, 40, 40))
    q = q0.copy()
    for _ in range(200):
        q = prop.coarse_step(q, prm)
    assert np.linalg.norm(q) > 100.0 * np.linalg.norm(q0)
