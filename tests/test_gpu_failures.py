"""Failure paths forced from the host: every kernel still runs to its end
and the library turns the condition into an error code.

  * A non-finite initial state makes the iterate non-finite; the check
    after the solve returns PR_EDIVERGED, for a context and for a served
    request, and leaves both usable.
  * A basis reservation the device cannot hold (hipMalloc fails) returns
    PR_ENOMEM and leaves the context usable.
"""

import numpy as np
import pytest

from paper_1510_02237_amd import binding, workloads as W
from gpu_cases import small_problem, smooth_state, say
from test_gpu_server import Server

pytestmark = pytest.mark.gpu


def _nan_state(prob):
    u = smooth_state(prob, 3)
    u[2, prob["nz"] // 2, prob["nx"] // 3] = np.nan
    return u


def test_non_finite_state_reports_diverged():
    prob = small_problem(64, 32, 4)
    say("diverged solve")
    ctx = binding.Context.from_problem(prob)
    with pytest.raises(binding.PRError) as e:
        ctx.solve(_nan_state(prob), 2)
    assert e.value.code == binding.PR_EDIVERGED
    u0 = smooth_state(prob, 3)
    a = ctx.solve(u0, 2)
    b = binding.Context.from_problem(prob).solve(u0, 2)
    assert np.array_equal(a, b)


def test_served_non_finite_request_reports_diverged():
    prob = small_problem(64, 32, 4)
    say("diverged served request")
    srv = Server(max_inflight=2)
    try:
        rc, bad = srv.submit(prob, 2, _nan_state(prob))
        assert rc == 0
        u0 = smooth_state(prob, 3)
        rc, good = srv.submit(prob, 2, u0)
        assert rc == 0
        assert srv.wait(bad, u0.shape)[0] == binding.PR_EDIVERGED
        rc, out, _ = srv.wait(good, u0.shape)
        assert rc == 0
        assert np.array_equal(out, binding.Context.from_problem(prob).solve(u0, 2))
    finally:
        srv.close()


def test_unsatisfiable_reservation_is_enomem():
    prob, K, u0 = W.config("c2_512x256")
    say("unsatisfiable basis reservation")
    ctx = binding.Context.from_problem(prob)
    # 65536 vectors of 3 * 512 * 256 doubles: about 206 TB
    with pytest.raises(binding.PRError) as e:
        ctx.reserve_basis(65536)
    assert e.value.code == binding.PR_ENOMEM
    # the context is unchanged: a solve still gives the fresh context's result
    a = ctx.solve(u0, 1)
    b = binding.Context.from_problem(prob).solve(u0, 1)
    assert np.array_equal(a, b)
