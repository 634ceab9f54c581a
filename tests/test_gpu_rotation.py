"""The split scheme with a velocity that varies in space on the GPU against
the oracle: the solid-body rotation of eq. adVel (Section 3.2), constant
velocities with a z-component, and second-order fine acoustics.  F runs in
the stage form with per-row and per-column advective weights; the coarse
kernel evaluates G's frozen slow tendency from the same kind of weights in
the first launch of each coarse step, and with more than one substep launch
stores it for the others.

Sizes: the paper's 40 x 40 and 80 x 80 grids (the stage kernel's 16 x 16
tiles end in a ragged tail on 40 x 40), plus a non-square grid with a
constant (U, V); N_sound 4 (one substep launch), 6 and 8 (two).  The whole
T = 2 runs of Tables 1 and 2 are checked against the oracle's own runs of
the same cells stored in tests/golden (written by make_rotation_fixture.py).
"""

import ctypes
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.operators import Params
from paper_1510_02237_amd import binding, workloads as W
from gpu_cases import rel_l2, say

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "rotation_40x40_oracle.json")


def short(prob, windows):
    """The same run cut to its first ``windows`` windows."""
    prob = dict(prob, windows=windows)
    prob["T"] = windows * prob["P"] * prob["dt_g"]
    return prob


def uv_problem(nx, nz, U, V, order, n_sound, P=2):
    prob = W.problem(nx, nz, P, U=U, n_sound=n_sound)
    prob.update(V=V, fine_acoustic_order=order)
    prob["T"] = P * prob["dt_g"]
    return prob


def _cases():
    rot40 = short(W.rotation_problem(40, 6, 4.0), 1)
    rot80 = short(W.rotation_problem(80, 6, 2.0), 1)
    # the less diffusive G of the energy runs (Section 3.2): third-order
    # slow tendency, nu_c = 0.005, N_sound = 8 (two substep launches), no
    # fine damping
    rot40_o3 = short(W.rotation_problem(40, 6, 2.0), 1)
    rot40_o3.update(coarse_order=3, nu_c=0.005, nu_f=0.0, n_sound=8)
    return [("rot40_cc4", rot40), ("rot80_cc2", rot80),
            ("rot40_ns6", dict(rot40, n_sound=6)), ("rot40_o3", rot40_o3),
            ("uv_48x24_o4", uv_problem(48, 24, 0.1, -0.07, 4, 4)),
            ("uv_40x24_o2_ns6", uv_problem(40, 24, -0.2, 0.15, 2, 6))]


@pytest.mark.parametrize("name,prob", _cases(), ids=[c[0] for c in _cases()])
def test_propagators_match_oracle(name, prob):
    prm = Params(**prob)
    say(f"rotation propagators {name}")
    rng = np.random.default_rng(len(name))
    Q = rng.normal(size=(3, 3, prob["nz"], prob["nx"]))
    Q[0] = W.ic_cosine_bell(prob["nx"], prob["nz"], centre=(0.5, 0.65))
    ctx = binding.Context.from_problem(prob)
    FQ = ctx.fine_sweep(Q)
    for s in range(3):
        assert rel_l2(FQ[s], oracle.fine_F(Q[s], prm)) <= 1e-12, s
        assert rel_l2(ctx.coarse_step(Q[s]), oracle.coarse_G(Q[s], prm)) <= 1e-12, s


def test_batched_coarse_matches_single():
    """The subspace update applies G to a block of states at once (the
    batched slow tendency and substep launches); the K(q) image of a basis
    vector must equal the single-state G plus its fine part."""
    torch = pytest.importorskip("torch")
    prob = short(W.rotation_problem(40, 6, 4.0), 1)
    say("rotation batched coarse")
    ctx = binding.Context.from_problem(prob)
    rng = np.random.default_rng(3)
    Q = rng.normal(size=(6, 3, 40, 40))
    FQ = ctx.fine_sweep(Q)
    r = ctx.krylov_update(Q, FQ)
    assert r == 6
    # Q lies in the basis, so K(Q[s]) = F(Q[s]) (eq. modifiedCoarse)
    for s in (0, 5):
        got = ctx.coarse_step(Q[s], use_krylov=True)
        assert rel_l2(got, FQ[s]) <= 1e-10, s


def test_less_diffusive_G_windowed_solve_matches_oracle():
    """Two windows of the energy-run configuration with the third-order
    coarse slow tendency (Section 3.2) on the GPU against the oracle."""
    prob = short(W.rotation_problem(40, 6, 2.0), 2)
    prob.update(coarse_order=3, nu_c=0.005, nu_f=0.0, n_sound=8)
    prm = Params(**prob)
    u0 = W.ic_cosine_bell(40, 40, centre=(0.5, 0.65))
    say("rotation less diffusive G solve")
    ctx = binding.Context.from_problem(prob)
    got = ctx.solve(u0, 2)
    want = oracle.kse_parareal(u0, prm, K=2)
    assert rel_l2(got, want["q"][prm.P]) <= 1e-10
    assert ctx.stats()["rank"] == want["window_ranks"][-1]


@pytest.fixture(scope="module")
def rot3():
    prob, K, u0 = W.config("rot_40x40")
    return short(prob, 3), K, u0


@pytest.mark.parametrize("K,parareal", [(1, False), (2, False), (3, False),
                                        (2, True)])
def test_windowed_solve_matches_oracle(rot3, K, parareal):
    prob, _, u0 = rot3
    prm = Params(**prob)
    say(f"rotation solve K={K} parareal={parareal}")
    ctx = binding.Context.from_problem(prob)
    got = ctx.solve(u0, K, parareal=parareal)
    want = oracle.kse_parareal(u0, prm, K=K, krylov=not parareal)
    assert rel_l2(got, want["q"][prm.P]) <= 1e-10
    if not parareal:
        assert ctx.stats()["rank"] == want["window_ranks"][-1]


def test_windowed_solve_exact_and_homogeneous(rot3):
    torch = pytest.importorskip("torch")
    prob, K, u0 = rot3
    say("rotation K = P and homogeneity")
    ctx = binding.Context.from_problem(prob)
    u0d = torch.from_numpy(u0).cuda()
    assert torch.equal(ctx.solve(u0d, prob["P"]), ctx.serial_fine(u0d))
    a = ctx.solve(u0d, K)
    assert torch.equal(ctx.solve(2.0 * u0d, K), 2.0 * a)


def test_paper_table_cells_match_oracle_runs():
    """Every cell (coarse CFL, P, K) of Tables 1 and 2 run to T = 2 (75 to
    300 windows): the error against the serial fine run equals the oracle's
    to 1e-9, the serial fine run and the final state of the cell (4, 6, 2)
    match the oracle's at 64 sampled points."""
    torch = pytest.importorskip("torch")
    fx = json.load(open(FIXTURE))
    u0 = W.ic_cosine_bell(40, 40, centre=(0.5, 0.65))
    u0d = torch.from_numpy(u0).cuda()
    ref = None
    idx = np.array(fx["sample_index"])
    for cell in fx["cells"]:
        cc, P, K = cell["cfl_c"], cell["P"], cell["K"]
        say(f"table cell cfl_c={cc} P={P} K={K}")
        ctx = binding.Context.from_problem(W.rotation_problem(40, P, cc))
        if ref is None:
            ref = ctx.serial_fine(u0d).cpu().numpy()
            assert np.abs(ref.ravel()[idx] - fx["serial_sample"]).max() <= \
                1e-10 * np.abs(ref).max()
            assert abs(np.linalg.norm(ref) - fx["serial_norm2"]) <= \
                1e-10 * fx["serial_norm2"]
        got = ctx.solve(u0d, K).cpu().numpy()
        assert abs(rel_l2(got, ref) - cell["eps"]) <= 1e-9, cell
        if (cc, P, K) == tuple(fx["sample_cell"][k] for k in ("cfl_c", "P", "K")):
            assert np.abs(got.ravel()[idx] - fx["final_sample"]).max() <= \
                1e-10 * fx["final_max"]


def test_create_accepts_coarse_cfl_4_rotation():
    """The frozen-coefficient estimate of this run exceeds 1 (host tests),
    yet pr_create accepts it: with gamma != 0 the estimate is not enforced."""
    prob = W.rotation_problem(40, 6, 4.0)
    ctx = binding.Context.from_problem(prob)
    assert ctx.opts.gamma == math.pi


def test_server_rejects_rotation():
    lib = binding.load()
    srv = ctypes.c_void_p()
    assert lib.pr_server_create(0, 1 << 30, 2, ctypes.byref(srv)) == 0
    try:
        prob = W.problem(64, 32, 8)
        u0 = np.zeros((3, 32, 64))
        t = ctypes.c_uint64()
        for kw in (dict(gamma=1.0), dict(V=0.1), dict(fine_acoustic_order=2),
                   dict(coarse_order=3)):
            o = binding.default_opts(**kw)
            rc = lib.pr_submit_ex(
                srv, ctypes.byref(binding.grid(64, 32)), 1.0, 0.1,
                prob["dt_f"], prob["dt_g"], 8, 2, ctypes.byref(o),
                u0.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t))
            assert rc == binding.PR_EINVAL, kw
    finally:
        lib.pr_server_destroy(srv)
