"""Windowed KSE-Parareal on the GPU (the parallel steps of Section 2.1,
each starting from the previous window's final state with an empty
subspace) against the oracle's windowed run, and its exact special cases."""

import ctypes

import numpy as np
import pytest

import oracle
from oracle.operators import Params
from paper_1510_02237_amd import binding, workloads as W
from gpu_cases import rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1w():
    prob, K, u0 = W.config("c1w_64x32")
    return prob, K, u0


@pytest.mark.parametrize("parareal", [False, True])
def test_windowed_solve_matches_oracle(c1w, parareal):
    prob, K, u0 = c1w
    prm = Params(**prob)
    say(f"windowed solve {prob['windows']} x {prob['P']} parareal={parareal}")
    ctx = binding.Context.from_problem(prob)
    got = ctx.solve(u0, K, parareal=parareal)
    want = oracle.kse_parareal(u0, prm, K=K, krylov=not parareal)
    assert rel_l2(got, want["q"][prm.P]) <= 1e-10
    if not parareal:
        assert ctx.stats()["rank"] == want["window_ranks"][-1]
    # the slices output holds the last window
    _, sl = ctx.solve(u0, K, slices=True, parareal=parareal)
    for i in (0, prm.P // 2, prm.P):
        assert rel_l2(sl[i], want["q"][i]) <= 1e-10, i


def test_windowed_exact_cases(c1w):
    torch = pytest.importorskip("torch")
    prob, K, u0 = c1w
    P, M = prob["P"], prob["windows"]
    ctx = binding.Context.from_problem(prob)
    u0d = torch.from_numpy(u0).cuda()
    say("windowed K = P and K = 0")
    ref = ctx.serial_fine(u0d).cpu().numpy()
    assert np.array_equal(ctx.solve(u0d, P).cpu().numpy(), ref)
    prm = Params(**prob)
    q = u0.copy()
    for _ in range(M * P):
        q = oracle.coarse_G(q, prm)
    assert rel_l2(ctx.solve(u0d, 0).cpu().numpy(), q) <= 1e-10
    st = ctx.stats()
    assert st["iterations"] == 0
    # one window equals the same problem on [0, T/M]
    one = dict(prob, windows=1, T=prob["T"] / M)
    a = binding.Context.from_problem(one).solve(u0d, K).cpu().numpy()
    two = dict(prob, windows=1, T=prob["T"] / M)
    b = binding.Context.from_problem(two).solve(
        torch.from_numpy(a).cuda(), K).cpu().numpy()
    both = binding.Context.from_problem(dict(prob, windows=2,
                                             T=2 * prob["T"] / M))
    assert np.array_equal(both.solve(u0d, K).cpu().numpy(), b)


def test_server_rejects_windows():
    lib = binding.load()
    h = ctypes.c_void_p()
    assert lib.pr_server_create(0, 0, 2, ctypes.byref(h)) == 0
    try:
        prob, K, u0 = W.config("c1w_64x32")
        o = binding.default_opts(windows=2, n_sound=prob["n_sound"])
        t = ctypes.c_uint64()
        u0 = np.ascontiguousarray(u0)
        rc = lib.pr_submit_ex(h, ctypes.byref(binding.grid(prob["nx"], prob["nz"],
                                                           prob["T"])),
                              prob["c_s"], prob["U"], prob["dt_f"], prob["dt_g"],
                              prob["P"], K, ctypes.byref(o), u0.ctypes.data,
                              ctypes.byref(t))
        assert rc == binding.PR_EINVAL
        assert b"one window" in lib.pr_server_last_error(h)
    finally:
        lib.pr_server_destroy(h)
