"""The propagator pair of the instability example (Section 3.1, scheme
PR_SCHEME_RK3) on the GPU against the oracle: F (RK-3, sixth-order centred
advective flux) and G (RK-3, first-order upwind) per slice, the windowed
KSE-Parareal and original Parareal solves, and the paper's finding that
the original Parareal is unstable on this example while KSE-Parareal is
not."""

import ctypes

import numpy as np
import pytest

import oracle
from oracle.operators import Params
from paper_1510_02237_amd import binding, workloads as W
from gpu_cases import rel_l2, say

pytestmark = pytest.mark.gpu


def rk3_problem(nx, nz, U, V, c_s=1.0, P=2, n_g=3, ratio=4, dt_g=0.004):
    return dict(nx=nx, nz=nz, c_s=c_s, U=U, V=V, dt_f=dt_g / ratio, dt_g=dt_g,
                P=P, T=P * n_g * dt_g, nu_f=0.0, nu_c=0.0, n_sound=1,
                rank_tol=1e-10, windows=1, scheme="rk3")


@pytest.mark.parametrize("nx,nz", [(40, 40), (37, 19), (64, 32)])
@pytest.mark.parametrize("U,V", [(1.0, 1.0), (-0.7, 0.4)])
def test_rk3_propagators_match_oracle(nx, nz, U, V):
    prob = rk3_problem(nx, nz, U, V)
    prm = Params(**prob)
    say(f"rk3 propagators {nx}x{nz} U={U} V={V}")
    rng = np.random.default_rng(nx + nz)
    Q = rng.normal(size=(3, 3, nz, nx))
    ctx = binding.Context.from_problem(prob)
    FQ = ctx.fine_sweep(Q)
    for s in range(3):
        assert rel_l2(FQ[s], oracle.fine_F(Q[s], prm)) <= 1e-12, s
        assert rel_l2(ctx.coarse_step(Q[s]), oracle.coarse_G(Q[s], prm)) <= 1e-12, s


@pytest.fixture(scope="module")
def demo3():
    prob, K, u0 = W.config("demo_40x40")
    prob = dict(prob, windows=3)
    prob["T"] = 3 * prob["P"] * prob["dt_g"]
    return prob, K, u0


@pytest.mark.parametrize("parareal", [False, True])
def test_demo_solve_matches_oracle(demo3, parareal):
    prob, K, u0 = demo3
    prm = Params(**prob)
    say(f"demo solve parareal={parareal}")
    ctx = binding.Context.from_problem(prob)
    got = ctx.solve(u0, K, parareal=parareal)
    want = oracle.kse_parareal(u0, prm, K=K, krylov=not parareal)
    assert rel_l2(got, want["q"][prm.P]) <= 1e-10
    if not parareal:
        assert ctx.stats()["rank"] == want["window_ranks"][-1]


def test_demo_K_equals_P_is_serial_fine(demo3):
    prob, K, u0 = demo3
    ctx = binding.Context.from_problem(prob)
    say("demo K = P")
    assert np.array_equal(ctx.solve(u0, prob["P"]), ctx.serial_fine(u0))


@pytest.mark.parametrize("c_s", [1.0, 0.0])
def test_demo_original_parareal_unstable_kse_stable(c_s):
    """Section 3.1 on the GPU: after 7 windows the original Parareal's
    max|q| is orders of magnitude above the fine run's, KSE-Parareal stays
    with the fine run, and both agree with the oracle's runs."""
    prob, K, u0 = W.config("demo_40x40")
    prob = dict(prob, c_s=c_s, windows=7)
    prob["T"] = 7 * prob["P"] * prob["dt_g"]
    say(f"demo instability c_s={c_s}")
    ctx = binding.Context.from_problem(prob)
    ref = ctx.serial_fine(u0)
    par = ctx.solve(u0, K, parareal=True)
    kse = ctx.solve(u0, K)
    fmax = np.abs(ref).max()
    assert np.abs(par).max() > 100 * fmax
    assert abs(np.abs(kse).max() - fmax) <= 0.05 * fmax
    assert rel_l2(kse, ref) < 0.2
    prm = Params(**prob)
    want = oracle.kse_parareal(u0, prm, K=K, krylov=False)["q"][prm.P]
    assert rel_l2(par, want) <= 1e-8
    assert rel_l2(ref, oracle.serial_fine(u0, prm)) <= 1e-11


def test_server_rejects_rk3_scheme():
    lib = binding.load()
    h = ctypes.c_void_p()
    assert lib.pr_server_create(0, 0, 2, ctypes.byref(h)) == 0
    try:
        prob = rk3_problem(40, 40, 1.0, 1.0)
        o = binding.default_opts(scheme="rk3", V=1.0, nu_f=0.0, nu_c=0.0,
                                 n_sound=1)
        t = ctypes.c_uint64()
        u0 = np.zeros((3, 40, 40))
        rc = lib.pr_submit_ex(h, ctypes.byref(binding.grid(40, 40, prob["T"])),
                              prob["c_s"], prob["U"], prob["dt_f"],
                              prob["dt_g"], prob["P"], 2, ctypes.byref(o),
                              u0.ctypes.data, ctypes.byref(t))
        assert rc == binding.PR_EINVAL
        assert b"split scheme" in lib.pr_server_last_error(h)
    finally:
        lib.pr_server_destroy(h)
