"""The oracle's propagators against a full spectral propagator on arbitrary
states (not single modes).

On the periodic grid with a constant velocity every discrete Fourier mode
is invariant, so F and G act on the 3-vector of Fourier coefficients of
each mode by their amplification matrices.  Transforming a random state
with the FFT, multiplying every coefficient vector by R(theta)^n and
transforming back is an independent implementation of the propagators in
a different basis: it shares nothing with the oracle's stencil code but
the amplification matrices, which the tests write from the stencil weights.
A mistake confined to some modes (an aliasing or wrap error, a wrong
stencil offset that a single low mode does not excite) shows up here.
"""

import numpy as np
import pytest

from oracle import propagators as prop
from oracle.operators import Params
from test_oracle_operators import fine_symbol
from test_oracle_propagators import coarse_step_symbol, rk3_poly
from test_oracle_rotation import coarse_symbol_uv, fine_symbol_uv
from test_oracle_rk3_scheme import rk3_symbol


def spectral(q, prm, step_matrix, nsteps):
    """IFFT(M(theta)^n FFT(q)) with M(theta) = step_matrix(prm, kx, kz)."""
    nz, nx = prm.nz, prm.nx
    qh = np.fft.fft2(q, axes=(1, 2))  # qh[f, kz, kx]
    out = np.empty_like(qh)
    for kz in range(nz):
        for kx in range(nx):
            M = np.linalg.matrix_power(step_matrix(prm, kx, kz), nsteps)
            out[:, kz, kx] = M @ qh[:, kz, kx]
    back = np.fft.ifft2(out, axes=(1, 2))
    assert np.abs(back.imag).max() <= 1e-12 * np.abs(back.real).max()
    return back.real


def _state(prm, seed):
    return np.random.default_rng(seed).normal(size=(3, prm.nz, prm.nx))


def _close(a, b, tol=1e-12):
    return np.abs(a - b).max() <= tol * np.abs(b).max()


@pytest.mark.parametrize("nx,nz,U", [(32, 16, 0.1), (24, 24, -0.25),
                                     (20, 12, 0.3)])
def test_split_scheme_x_advection(nx, nz, U):
    prm = Params(nx=nx, nz=nz, c_s=1.0, U=U, dt_f=0.2 / nx, dt_g=2.0 / nx,
                 P=1, T=2.0 / nx, n_sound=10)
    q = _state(prm, nx + nz)
    f_step = lambda p, kx, kz: rk3_poly(p.dt_f * fine_symbol(p, kx, kz))
    assert _close(prop.fine_F(q, prm, 6), spectral(q, prm, f_step, 6))
    assert _close(prop.coarse_G(q, prm, 2),
                  spectral(q, prm, coarse_step_symbol, 2))


@pytest.mark.parametrize("order", [4, 2])
@pytest.mark.parametrize("U,V", [(0.1, -0.07), (-0.2, 0.15)])
def test_split_scheme_with_z_velocity(order, U, V):
    prm = Params(nx=24, nz=16, c_s=1.5, U=U, V=V, dt_f=0.2 / 36,
                 dt_g=2.0 / 36, P=1, T=2.0 / 36, fine_acoustic_order=order)
    q = _state(prm, 3)
    f_step = lambda p, kx, kz: rk3_poly(p.dt_f * fine_symbol_uv(p, kx, kz))
    assert _close(prop.fine_F(q, prm, 5), spectral(q, prm, f_step, 5))
    assert _close(prop.coarse_G(q, prm, 2),
                  spectral(q, prm, coarse_symbol_uv, 2))


def test_section_3_1_pair():
    prm = Params(nx=20, nz=20, c_s=1.0, U=1.0, V=1.0, dt_f=1.0 / 432,
                 dt_g=1.0 / 72, P=1, T=1.0 / 72, nu_f=0.0, nu_c=0.0,
                 n_sound=1, scheme="rk3")
    q = _state(prm, 9)
    f_step = lambda p, kx, kz: rk3_poly(p.dt_f * rk3_symbol(p, kx, kz, False))
    g_step = lambda p, kx, kz: rk3_poly(p.dt_g * rk3_symbol(p, kx, kz, True))
    assert _close(prop.fine_F(q, prm, 6), spectral(q, prm, f_step, 6))
    assert _close(prop.coarse_G(q, prm, 1), spectral(q, prm, g_step, 1))
