"""Pins of the oracle's propagators F and G (Section 3.2).

F (three-stage RK3): on one Fourier mode the discrete solution after n steps
must be R(Z)^n v with Z = dt * A(theta) the symbol matrix of the fine
operator and R(Z) = I + Z + Z^2/2 + Z^3/6 -- the stability polynomial shared
by every three-stage third-order Runge-Kutta method on a linear problem.
G (partially split forward Euler with forward-backward acoustic substeps):
on one mode the step is the product of the substep matrices with the slow
tendency frozen at the start of the step.  Plus: third-order temporal
convergence of F against the matrix exponential, constant states are fixed
points, and the propagators are stable at the workload parameters.
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import propagators as prop
from oracle.operators import Params
from test_oracle_operators import _symbols, apply_complex, fine_symbol


def _prm(**kw):
    base = dict(nx=32, nz=16, c_s=1.0, U=0.1, dt_f=0.2 / 32, dt_g=2.0 / 32,
                P=8, T=1.0)
    base.update(kw)
    return Params(**base)


def rk3_poly(Z):
    I = np.eye(3)
    return I + Z + Z @ Z / 2 + Z @ Z @ Z / 6


@pytest.mark.parametrize("U", [0.1, -0.2])
@pytest.mark.parametrize("kx,kz", [(1, 1), (3, -2), (7, 5), (16, 8)])
def test_fine_F_single_mode_closed_form(U, kx, kz):
    prm = _prm(U=U)
    v = np.array([0.3 + 0.1j, -0.7, 1.0 - 0.4j])
    nsteps = 7
    got = apply_complex(lambda q: prop.fine_F(q, prm, nsteps), prm, kx, kz, v)
    R = rk3_poly(prm.dt_f * fine_symbol(prm, kx, kz))
    want = np.linalg.matrix_power(R, nsteps) @ v
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def coarse_step_symbol(prm, kx, kz):
    """3x3 amplification of one coarse step on mode (kx, kz)."""
    s = _symbols(2 * np.pi * kx / prm.nx, 2 * np.pi * kz / prm.nz,
                 prm.dx, prm.dz, prm.U)
    dtau = prm.dt_g / prm.n_sound
    ax = prm.nu_c * prm.dx ** 2 / dtau
    az = prm.nu_c * prm.dz ** 2 / dtau
    c = prm.c_s
    Rs = -prm.U * s["a1"]          # frozen slow tendency = Rs * q^n
    Y = np.eye(3, dtype=complex)   # maps q^n -> current substep state
    for _ in range(prm.n_sound):
        u, w, p = Y
        un = u + dtau * (Rs * np.eye(3)[0] - c * s["dx2"] * p
                         + ax * (s["gxx"] * u + s["gxz"] * w))
        wn = w + dtau * (Rs * np.eye(3)[1] - c * s["dz2"] * p
                         + az * (s["gzz"] * w + s["gxz"] * u))
        pn = p + dtau * (Rs * np.eye(3)[2] - c * (s["dx2"] * un + s["dz2"] * wn))
        Y = np.array([un, wn, pn])
    return Y


@pytest.mark.parametrize("U,ns", [(0.1, 4), (0.2, 6), (-0.3, 10)])
@pytest.mark.parametrize("kx,kz", [(1, 0), (2, 3), (9, -4), (16, 8)])
def test_coarse_G_single_mode_closed_form(U, ns, kx, kz):
    prm = _prm(U=U, n_sound=ns)
    v = np.array([1.0, 0.2 - 0.5j, -0.3j])
    got = apply_complex(lambda q: prop.coarse_G(q, prm, 3), prm, kx, kz, v)
    want = np.linalg.matrix_power(coarse_step_symbol(prm, kx, kz), 3) @ v
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_fine_third_order_in_time():
    """With nu_f = 0 (damping scales with 1/dt) the RK3 error against the
    exact semi-discrete solution exp(t A) v falls by 2^3 per halving of dt:
    the temporal-error check of Section 3.2.4 on one mode."""
    kx, kz = 2, 1
    v = np.array([0.0, 0.0, 1.0 + 0j])
    errs = []
    for m in (1, 2, 4):
        prm = _prm(nu_f=0.0, dt_f=0.02 / m)
        got = apply_complex(lambda q: prop.fine_F(q, prm, 20 * m), prm, kx, kz, v)
        exact = scipy.linalg.expm(0.4 * fine_symbol(prm, kx, kz)) @ v
        errs.append(np.abs(got - exact).max())
    assert 7.0 < errs[0] / errs[1] < 9.0 and 7.0 < errs[1] / errs[2] < 9.0


def test_constant_state_is_fixed_point():
    prm = _prm()
    q = np.ones((3, prm.nz, prm.nx)) * np.array([0.5, -1.0, 2.0])[:, None, None]
    assert np.array_equal(prop.coarse_G(q, prm), q)
    assert np.abs(prop.fine_F(q, prm) - q).max() < 1e-14


@pytest.mark.parametrize("U,ns", [(0.1, 4), (0.15, 4), (0.2, 6), (0.3, 10)])
def test_workload_propagators_are_stable(U, ns):
    """Spectral radius <= 1 over every mode of a 2:1-cell grid at fine CFL
    0.2 and coarse CFL 2 (the workload parameters)."""
    prm = _prm(U=U, n_sound=ns)
    worst_f = worst_g = 0.0
    for kx in range(prm.nx):
        for kz in range(prm.nz):
            Rf = rk3_poly(prm.dt_f * fine_symbol(prm, kx, kz))
            worst_f = max(worst_f, np.abs(np.linalg.eigvals(Rf)).max())
            Rg = coarse_step_symbol(prm, kx, kz)
            worst_g = max(worst_g, np.abs(np.linalg.eigvals(Rg)).max())
    assert worst_f <= 1 + 1e-12 and worst_g <= 1 + 1e-12


def test_coarse_unstable_beyond_rule():
    """N_sound = 4 is not enough at U = 0.3: the reason the workloads raise
    N_sound with U."""
    prm = _prm(U=0.3, n_sound=4)
    worst = max(np.abs(np.linalg.eigvals(coarse_step_symbol(prm, kx, kz))).max()
                for kx in range(prm.nx) for kz in range(prm.nz))
    assert worst > 1.05


def test_serial_fine_is_F_composed():
    prm = _prm(P=3, T=0.375)
    rng = np.random.default_rng(3)
    q0 = rng.normal(size=(3, prm.nz, prm.nx))
    a = prop.serial_fine(q0, prm)
    b = prop.fine_F(prop.fine_F(prop.fine_F(q0, prm), prm), prm)
    assert np.array_equal(a, b)
    assert np.array_equal(prop.fine_F(q0, prm, 3 * prm.n_f), a)


# ------------------------------------- the less diffusive G of Section 3.2

def _a3(tx, dx, U):
    """Third-order upwind derivative from its point weights (1, -6, 3, 2)/6
    at i-2..i+1 for U >= 0, mirrored for U < 0."""
    e = lambda m: np.exp(1j * m * tx)
    if U >= 0:
        return (e(-2) - 6 * e(-1) + 3 + 2 * e(1)) / (6 * dx)
    return (-2 * e(-1) - 3 + 6 * e(1) - e(2)) / (6 * dx)


def test_upwind3_is_third_order():
    from oracle import operators as ops
    errs = []
    for n in (32, 64, 128):
        x = (np.arange(n) + 0.5) / n
        f = np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x)
        exact = 2 * np.pi * np.cos(2 * np.pi * x) - 1.8 * np.pi * np.sin(6 * np.pi * x)
        for vel in (0.7, -0.7):
            q = np.tile(f, (4, 1))
            d = ops.flux_div(ops.flux_upwind3(q, vel, 1), 1.0 / n, 1)[0] / vel
            errs.append((n, vel, np.abs(d - exact).max()))
    for vel in (0.7, -0.7):
        e = [x[2] for x in errs if x[1] == vel]
        o = [np.log2(e[i] / e[i + 1]) for i in range(2)]
        assert min(o) > 2.9, (vel, o)


@pytest.mark.parametrize("U", [0.1, -0.2])
@pytest.mark.parametrize("kx,kz", [(1, 0), (2, 3), (9, -4), (16, 8)])
def test_less_diffusive_G_single_mode(U, kx, kz):
    """One coarse step with the third-order slow tendency is the product of
    the substep matrices with R frozen, as for the first-order G."""
    prm = _prm(U=U, n_sound=8, nu_c=0.005, coarse_order=3)
    v = np.array([1.0, 0.2 - 0.5j, -0.3j])
    got = apply_complex(lambda q: prop.coarse_G(q, prm, 2), prm, kx, kz, v)
    s = _symbols(2 * np.pi * kx / prm.nx, 2 * np.pi * kz / prm.nz,
                 prm.dx, prm.dz, prm.U)
    s["a1"] = _a3(2 * np.pi * kx / prm.nx, prm.dx, prm.U)
    Y = _coarse_step_from(prm, s)
    want = np.linalg.matrix_power(Y, 2) @ v
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def _coarse_step_from(prm, s):
    dtau = prm.dt_g / prm.n_sound
    ax = prm.nu_c * prm.dx ** 2 / dtau
    az = prm.nu_c * prm.dz ** 2 / dtau
    c = prm.c_s
    Rs = -prm.U * s["a1"]
    Y = np.eye(3, dtype=complex)
    for _ in range(prm.n_sound):
        u, w, p = Y
        un = u + dtau * (Rs * np.eye(3)[0] - c * s["dx2"] * p
                         + ax * (s["gxx"] * u + s["gxz"] * w))
        wn = w + dtau * (Rs * np.eye(3)[1] - c * s["dz2"] * p
                         + az * (s["gzz"] * w + s["gxz"] * u))
        pn = p + dtau * (Rs * np.eye(3)[2] - c * (s["dx2"] * un + s["dz2"] * wn))
        Y = np.array([un, wn, pn])
    return Y


def _worst_less_diffusive(nu_c):
    """Largest spectral radius of one coarse step with the third-order slow
    tendency, N_sound = 8, on the 64 x 32 grid at coarse CFL 2, U = 0.1."""
    prm = _prm(nx=64, nz=32, U=0.1, dt_f=0.2 / 64, dt_g=2.0 / 64, n_sound=8,
               nu_f=0.0, nu_c=nu_c, coarse_order=3)
    worst = 0.0
    for kx in range(prm.nx):
        for kz in range(prm.nz):
            s = _symbols(2 * np.pi * kx / prm.nx, 2 * np.pi * kz / prm.nz,
                         prm.dx, prm.dz, prm.U)
            s["a1"] = _a3(2 * np.pi * kx / prm.nx, prm.dx, prm.U)
            worst = max(worst, np.abs(np.linalg.eigvals(_coarse_step_from(prm, s))).max())
    return worst


def test_less_diffusive_G_is_unstable_under_these_readings():
    """Section 3.2's less diffusive G (third-order slow tendency, nu_c =
    0.005, N_sound = 8) grows under the readings taken here (frozen slow
    tendency over forward-backward substeps): forward Euler on a
    third-order upwind tendency amplifies low wavenumbers, whose upwind
    damping is only fourth order in the wavenumber.  More divergence
    damping does not remove it."""
    assert _worst_less_diffusive(0.005) > 1.1
    assert _worst_less_diffusive(0.1) > 1.005
