"""GPU parity of the fine and coarse propagators (Section 3.2) against the
oracle: relative l2 error <= 1e-12 per fine sweep and per coarse step, on
grids that span several workgroup tiles with ragged edges in x and z, both
signs of U, every launch form and every tile shape (bitwise equal among the
fused forms and shapes).  The fused step marches odd chunks upwards; the
chunk heights below give several chunks per slice with a ragged last chunk
that is odd for some of them, so both directions and the ragged upward
chunk are compared with the oracle and with each other."""

import numpy as np
import pytest

import oracle
from oracle.operators import Params
from paper_1510_02237_amd import binding
from gpu_cases import small_problem, rand_states, smooth_state, rel_l2, say

pytestmark = pytest.mark.gpu

TOL_SWEEP = 1e-12

GRIDS = [(8, 8), (16, 8), (64, 32), (100, 40), (300, 20), (37, 19)]


@pytest.mark.parametrize("nx,nz", GRIDS)
@pytest.mark.parametrize("U", [0.1, -0.25, 0.0])
def test_fine_sweep_matches_oracle(nx, nz, U):
    prob = small_problem(nx, nz, 3, U=U)
    say(f"fine sweep {nx}x{nz} U={U}")
    Q = rand_states(prob, 3, seed=nx * 7 + nz)
    ctx = binding.Context.from_problem(prob)
    FQ = ctx.fine_sweep(Q)
    prm = Params(**prob)
    for s in range(3):
        want = oracle.fine_F(Q[s], prm)
        assert rel_l2(FQ[s], want) <= TOL_SWEEP, (s, rel_l2(FQ[s], want))


@pytest.mark.parametrize("nx,nz,U", [(100, 40, 0.1), (37, 19, -0.2),
                                     (300, 20, 0.05)])
def test_fine_forms_and_tiles_agree(nx, nz, U):
    """Batched and plain forms and every tile shape give bitwise the same
    result (the per-point arithmetic does not depend on the tiling); the
    unfused stagewise form agrees to rounding."""
    prob = small_problem(nx, nz, 4, U=U)
    Q = rand_states(prob, 4, seed=3)
    say(f"forms {nx}x{nz}")
    ref = binding.Context.from_problem(prob, tile_nt=256,
                                       tile_zc=64).fine_sweep(Q)
    for nt in (128, 192, 256):
        for zc in (8, 12, 28, 32, 60, 124):
            say(f"  tile {nt}x{zc}")
            got = binding.Context.from_problem(prob, tile_nt=nt,
                                               tile_zc=zc).fine_sweep(Q)
            assert np.array_equal(got, ref), (nt, zc)
    plain = binding.Context.from_problem(prob, form="plain").fine_sweep(Q)
    assert np.array_equal(plain, ref)
    stw = binding.Context.from_problem(prob, form="stagewise").fine_sweep(Q)
    assert rel_l2(stw, ref) <= TOL_SWEEP


@pytest.mark.parametrize("nx,nz", [(128, 24), (256, 13), (512, 12)])
@pytest.mark.parametrize("U", [0.1, -0.25])
def test_fine_full_row_tiles(nx, nz, U):
    """One workgroup per periodic row (tile_nt = nx, no x-halo): parity with
    the oracle, and bitwise agreement with the halo tiles and with every
    chunk height, including a ragged last chunk."""
    prob = small_problem(nx, nz, 3, U=U)
    Q = rand_states(prob, 3, seed=nx + nz)
    say(f"full-row {nx}x{nz} U={U}")
    ref = binding.Context.from_problem(prob, tile_nt=192,
                                       tile_zc=8).fine_sweep(Q)
    prm = Params(**prob)
    for s in range(3):
        assert rel_l2(ref[s], oracle.fine_F(Q[s], prm)) <= TOL_SWEEP, s
    for zc in (4, 8, 12, 20, 32):
        say(f"  tile {nx}x{zc}")
        got = binding.Context.from_problem(prob, tile_nt=nx,
                                           tile_zc=zc).fine_sweep(Q)
        assert np.array_equal(got, ref), zc


def test_fine_sweep_device_tensors():
    torch = pytest.importorskip("torch")
    prob = small_problem(64, 32, 2, U=0.1)
    Q = rand_states(prob, 2, seed=9)
    say("fine sweep torch")
    ctx = binding.Context.from_problem(prob)
    host = ctx.fine_sweep(Q)
    dev = ctx.fine_sweep(torch.from_numpy(Q).cuda())
    assert np.array_equal(dev.cpu().numpy(), host)


@pytest.mark.parametrize("nx,nz", [(8, 8), (64, 32), (50, 70), (130, 33)])
@pytest.mark.parametrize("U,ns", [(0.1, 4), (-0.2, 6), (0.3, 10), (0.0, 5)])
def test_coarse_step_matches_oracle(nx, nz, U, ns):
    prob = small_problem(nx, nz, 2, U=U, n_g=2, n_sound=ns)
    say(f"coarse {nx}x{nz} U={U} ns={ns}")
    q = rand_states(prob, 1, seed=ns)[0]
    ctx = binding.Context.from_problem(prob)
    got = ctx.coarse_step(q)
    want = oracle.coarse_G(q, Params(**prob))
    assert rel_l2(got, want) <= TOL_SWEEP


def test_serial_fine_matches_oracle():
    prob = small_problem(64, 32, 4, U=0.1)
    u0 = smooth_state(prob, 5)
    say("serial fine")
    ctx = binding.Context.from_problem(prob)
    prm = Params(**prob)
    for ns in (1, 3, 4):
        want = oracle.serial_fine(u0, prm, nslices=ns)
        assert rel_l2(ctx.serial_fine(u0, ns), want) <= TOL_SWEEP


def test_stats_report_the_fine_tile():
    """pr_stats names the fused-step tile of the solve: the one set in the
    options, else the autotuner's choice; none in the stage form."""
    prob = small_problem(100, 40, 4, U=0.1)
    u0 = smooth_state(prob, 1)
    say("stats tile")
    ctx = binding.Context.from_problem(prob, tile_nt=192, tile_zc=28)
    ctx.solve(u0, 2)
    st = ctx.stats()
    assert (st["tile_nt"], st["tile_zc"]) == (192, 28)
    ctx = binding.Context.from_problem(prob)
    ctx.solve(u0, 2)
    st = ctx.stats()
    assert st["tile_nt"] in (128, 192, 256), st
    assert st["tile_zc"] > 0 and st["tile_zc"] % 4 == 0, st
    stw = binding.Context.from_problem(prob, form="stagewise")
    stw.solve(u0, 2)
    assert (stw.stats()["tile_nt"], stw.stats()["tile_zc"]) == (0, 0)
