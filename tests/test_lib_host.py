"""Host-side checks of the HIP library that need no GPU: it loads, exports
every entry point its header declares, and its host logic (argument
validation, the von Neumann stability scan, footprints) is right.

The stability scan is pinned against the amplification matrices the oracle
tests build from the stencil weights (test_oracle_propagators), with numpy's
eigenvalue routine: an independent formulation of the same symbols.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1510_02237_amd import binding, workloads as W
from oracle.operators import Params
from test_oracle_operators import fine_symbol
from test_oracle_propagators import coarse_step_symbol, rk3_poly

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libpararealhip.h")


@pytest.fixture(scope="module")
def lib():
    return binding.load()


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(pr_[a-z_0-9]+)\s*\(", txt)
    return sorted(set(names))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    # and the binding knows all of them
    assert set(names) <= set(binding._SIGS)


def test_opts_default(lib):
    o = binding.default_opts()
    assert o.nu_f == 0.005 and o.nu_c == 0.1 and o.n_sound == 4
    assert o.rank_tol == 1e-10 and o.form == binding.PR_FORM_BATCHED
    assert o.skip_converged == 1 and o.tile_nt == 0 and o.tile_zc == 0
    assert o.windows == 1


def test_strerror(lib):
    assert lib.pr_strerror(0) == b"ok"
    assert lib.pr_strerror(-4) == b"unstable propagator"
    assert lib.pr_strerror(-99) == b"unknown error"


def _scan(prm):
    rf = rg = 0.0
    for kx in range(prm.nx):
        for kz in range(prm.nz):
            Rf = rk3_poly(prm.dt_f * fine_symbol(prm, kx, kz))
            rf = max(rf, np.abs(np.linalg.eigvals(Rf)).max())
            rg = max(rg, np.abs(np.linalg.eigvals(
                coarse_step_symbol(prm, kx, kz))).max())
    return rf, rg


@pytest.mark.parametrize("nx,nz,U,ns", [(32, 16, 0.1, 4), (16, 16, -0.2, 6),
                                        (24, 12, 0.3, 4), (24, 12, 0.3, 10)])
def test_stability_scan_matches_symbols(lib, nx, nz, U, ns):
    prob = W.problem(nx, nz, 4, U=U, n_sound=ns)
    prm = Params(**prob)
    want_f, want_g = _scan(prm)
    got_f, got_g = binding.check_stability(nx, nz, prob["c_s"], U,
                                           prob["dt_f"], prob["dt_g"],
                                           n_sound=ns)
    assert abs(got_f - want_f) < 1e-12
    assert abs(got_g - want_g) < 1e-12


def test_stability_of_workload_rule(lib):
    """The N_sound rule of the workloads keeps G stable up to U = 0.3 on
    the 2:1 grids; N_sound = 4 is not enough at U = 0.3."""
    for U in (0.0, 0.1, 0.15, 0.2, 0.25, 0.3):
        prob = W.problem(64, 32, 8, U=U)
        rf, rg = binding.check_stability(64, 32, 1.0, U, prob["dt_f"],
                                         prob["dt_g"], n_sound=prob["n_sound"])
        assert rf <= 1 + 1e-12 and rg <= 1 + 1e-12, U
    prob = W.problem(64, 32, 8, U=0.3, n_sound=4)
    _, rg = binding.check_stability(64, 32, 1.0, 0.3, prob["dt_f"],
                                    prob["dt_g"], n_sound=4)
    assert rg > 1.05


@pytest.mark.parametrize("U,V,c_s", [(1.0, 1.0, 1.0), (-0.7, 0.4, 0.0),
                                     (0.3, -1.2, 2.0)])
def test_stability_scan_rk3_scheme(lib, U, V, c_s):
    """Section 3.1 pair: the scan's spectral radii against numpy eigenvalues
    of R(dt A) with A written from the stencil weights (the symbols the
    oracle's tests pin)."""
    from test_oracle_rk3_scheme import rk3_symbol
    nx = nz = 16
    dt_g = 0.6 / nx / (abs(U) + abs(V) + c_s)
    dt_f = dt_g / 6
    prm = Params(nx=nx, nz=nz, c_s=c_s, U=U, V=V, dt_f=dt_f, dt_g=dt_g, P=1,
                 T=dt_g, nu_f=0.0, nu_c=0.0, n_sound=1, scheme="rk3")
    want_f = want_g = 0.0
    for kx in range(nx):
        for kz in range(nz):
            want_f = max(want_f, np.abs(np.linalg.eigvals(
                rk3_poly(dt_f * rk3_symbol(prm, kx, kz, False)))).max())
            want_g = max(want_g, np.abs(np.linalg.eigvals(
                rk3_poly(dt_g * rk3_symbol(prm, kx, kz, True)))).max())
    got_f, got_g = binding.check_stability(nx, nz, c_s, U, dt_f, dt_g,
                                           scheme="rk3", V=V, n_sound=1)
    assert abs(got_f - want_f) < 1e-12 and abs(got_g - want_g) < 1e-12


def test_demo_pair_is_stable(lib):
    prob, K, u0 = W.config("demo_40x40")
    rf, rg = binding.check_stability(40, 40, prob["c_s"], prob["U"],
                                     prob["dt_f"], prob["dt_g"], scheme="rk3",
                                     V=prob["V"], n_sound=1)
    assert rf <= 1 + 1e-12 and rg <= 1 + 1e-12


@pytest.mark.parametrize("U,V,order", [(0.1, -0.07, 4), (-0.2, 0.15, 2),
                                       (0.0, 0.2, 4)])
def test_stability_scan_split_with_z_velocity(lib, U, V, order):
    """Split pair with a constant (U, V) and either acoustic order: the
    scan against numpy eigenvalues of the amplification matrices written
    from the stencil weights."""
    from test_oracle_rotation import fine_symbol_uv, coarse_symbol_uv
    prm = Params(nx=16, nz=12, c_s=1.0, U=U, V=V, dt_f=0.2 / 16,
                 dt_g=2.0 / 16, P=1, T=2.0 / 16, fine_acoustic_order=order)
    want_f = want_g = 0.0
    for kx in range(prm.nx):
        for kz in range(prm.nz):
            want_f = max(want_f, np.abs(np.linalg.eigvals(
                rk3_poly(prm.dt_f * fine_symbol_uv(prm, kx, kz)))).max())
            want_g = max(want_g, np.abs(np.linalg.eigvals(
                coarse_symbol_uv(prm, kx, kz))).max())
    got_f, got_g = binding.check_stability(16, 12, 1.0, U, prm.dt_f, prm.dt_g,
                                           V=V, fine_acoustic_order=order)
    assert abs(got_f - want_f) < 1e-12 and abs(got_g - want_g) < 1e-12


def test_stability_scan_rotation_is_frozen_at_extreme_velocities(lib):
    """With gamma != 0 the scan reports the largest radii of the symbols
    frozen at the four extreme (x-velocity of a row, z-velocity of a
    column) pairs."""
    from oracle import operators as ops
    from test_oracle_rotation import fine_symbol_uv, coarse_symbol_uv
    base = dict(nx=16, nz=16, c_s=3.0, U=0.1, V=-0.2, dt_f=0.2 / 48,
                dt_g=2.0 / 48, P=1, T=2.0 / 48, fine_acoustic_order=2)
    rot = Params(**base, gamma=2.0)
    ux, vz = ops.velocity_x(rot)[:, 0], ops.velocity_z(rot)[0]
    want_f = want_g = 0.0
    for u in (ux.min(), ux.max()):
        for v in (vz.min(), vz.max()):
            p = Params(**{**base, "U": u, "V": v})
            for kx in range(16):
                for kz in range(16):
                    want_f = max(want_f, np.abs(np.linalg.eigvals(
                        rk3_poly(p.dt_f * fine_symbol_uv(p, kx, kz)))).max())
                    want_g = max(want_g, np.abs(np.linalg.eigvals(
                        coarse_symbol_uv(p, kx, kz))).max())
    got_f, got_g = binding.check_stability(16, 16, 3.0, 0.1, rot.dt_f,
                                           rot.dt_g, V=-0.2, gamma=2.0,
                                           fine_acoustic_order=2)
    assert abs(got_f - want_f) < 1e-12 and abs(got_g - want_g) < 1e-12


def test_rotation_frozen_estimate_exceeds_one_at_coarse_cfl_4(lib):
    """The frozen-coefficient estimate of the paper's coarse-CFL-4 run
    exceeds 1, but the propagator does not grow on the rotating flow (the
    oracle's pins), which is why pr_create does not enforce it when gamma
    is set (the GPU tests create this context)."""
    prob = W.rotation_problem(40, 6, 4.0)
    _, rg = binding.check_stability(
        40, 40, prob["c_s"], 0.0, prob["dt_f"], prob["dt_g"],
        gamma=prob["gamma"], fine_acoustic_order=2, n_sound=4,
        windows=prob["windows"])
    assert rg > 1.04


@pytest.mark.parametrize("U", [0.1, -0.2])
def test_stability_scan_third_order_coarse(lib, U):
    """The less diffusive G of Section 3.2 (third-order slow tendency,
    nu_c = 0.005, N_sound = 8): the scan against numpy eigenvalues of the
    substep product written from the stencil weights; it exceeds 1."""
    from test_oracle_operators import _symbols
    from test_oracle_propagators import _a3, _coarse_step_from
    prm = Params(nx=16, nz=12, c_s=1.0, U=U, dt_f=0.2 / 16, dt_g=2.0 / 16,
                 P=1, T=2.0 / 16, n_sound=8, nu_f=0.0, nu_c=0.005,
                 coarse_order=3)
    want = 0.0
    for kx in range(prm.nx):
        for kz in range(prm.nz):
            s = _symbols(2 * np.pi * kx / prm.nx, 2 * np.pi * kz / prm.nz,
                         prm.dx, prm.dz, prm.U)
            s["a1"] = _a3(2 * np.pi * kx / prm.nx, prm.dx, prm.U)
            want = max(want, np.abs(np.linalg.eigvals(
                _coarse_step_from(prm, s))).max())
    _, got = binding.check_stability(16, 12, 1.0, U, prm.dt_f, prm.dt_g,
                                     n_sound=8, nu_f=0.0, nu_c=0.005,
                                     coarse_order=3)
    assert abs(got - want) < 1e-12 and got > 1.0


def _create(lib, nx, nz, c_s, U, dt_f, dt_g, P, T=1.0, **opts):
    h = ctypes.c_void_p()
    o = binding.default_opts(**opts)
    rc = lib.pr_create_ex(ctypes.byref(binding.grid(nx, nz, T)), c_s, U, dt_f,
                          dt_g, P, ctypes.byref(o), None, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("kw,why", [
    (dict(nx=7), "nx and nz must be >= 8"),
    (dict(nz=4), "nx and nz must be >= 8"),
    (dict(P=0), "P must be"),
    (dict(dt_f=0.3 / 64), "dt_f"),
    (dict(dt_g=0.0), "time steps"),
    (dict(n_sound=0), "n_sound"),
    (dict(tile_nt=100), "tile_nt"),
    (dict(tile_nt=512), "tile_nt"),
    (dict(tile_zc=10), "tile_zc"),
    (dict(windows=0), "windows"),
    (dict(windows=3), "(T/(windows*P))/dt_f"),
    (dict(scheme=7), "scheme"),
    (dict(scheme=1, gamma=1.0), "gamma must be 0"),
    (dict(gamma=float("nan")), "V and gamma must be finite"),
    (dict(fine_acoustic_order=3), "fine_acoustic_order"),
    (dict(coarse_order=2), "coarse_order must be 1 or 3"),
    (dict(scheme=1, coarse_order=3), "coarse_order must be 1 with"),
    (dict(stop_tol=-1.0), "stop_tol"),
])
def test_create_rejects_bad_arguments(lib, kw, why):
    args = dict(nx=64, nz=32, c_s=1.0, U=0.1, dt_f=0.2 / 64, dt_g=2.0 / 64,
                P=8)
    opts = {k: kw.pop(k) for k in list(kw) if k in ("n_sound", "tile_nt",
                                                   "tile_zc", "windows",
                                                   "scheme", "V", "stop_tol",
                                                   "gamma",
                                                   "fine_acoustic_order",
                                                   "coarse_order")}
    args.update(kw)
    rc, h = _create(lib, **args, **opts)
    assert rc == binding.PR_EINVAL and not h.value
    assert why in lib.pr_last_error(None).decode()


def test_create_rejects_unstable_coarse(lib):
    prob = W.problem(64, 32, 8, U=0.3, n_sound=4)
    rc, h = _create(lib, 64, 32, 1.0, 0.3, prob["dt_f"], prob["dt_g"], 8,
                    n_sound=4)
    assert rc == binding.PR_EUNSTABLE and not h.value
    # the less diffusive G with a constant velocity
    prob = W.problem(64, 32, 8, U=0.1)
    rc, h = _create(lib, 64, 32, 1.0, 0.1, prob["dt_f"], prob["dt_g"], 8,
                    n_sound=8, coarse_order=3)
    assert rc == binding.PR_EUNSTABLE and not h.value


def test_footprint():
    b = binding.footprint(512, 256, 32, 4)
    d = 3 * 512 * 256
    # basis S and D(S) of P*K vectors dominate
    assert 2 * 32 * 4 * d * 8 < b < 2.2 * (2 * 32 * 4 + 8 * 32) * d * 8
    assert binding.footprint(64, 32, 8, 0) > 0
