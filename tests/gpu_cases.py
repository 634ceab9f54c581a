"""Shared problem builders for the GPU parity tests (no arithmetic of the
method here: only parameter choices and seeded inputs)."""

import sys

import numpy as np

from paper_1510_02237_amd import workloads as W


def small_problem(nx, nz, P, U=0.1, n_g=1, n_sound=None):
    """Workload parameters (fine CFL 0.2, coarse step 10 fine steps) with
    the window length set so each slice holds n_g coarse and 10 n_g fine
    steps."""
    prob = W.problem(nx, nz, P, U=U, n_sound=n_sound)
    prob["T"] = P * n_g * prob["dt_g"]
    return prob


def rand_states(prob, n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, 3, prob["nz"], prob["nx"]))


def smooth_state(prob, seed, nbumps=2, noise=1e-3):
    return W.ic_bumps(prob["nx"], prob["nz"], seed, nbumps=nbumps, noise=noise,
                      width=0.1)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def say(*a):
    print(*a, file=sys.stderr, flush=True)
