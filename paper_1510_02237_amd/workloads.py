"""Seeded synthetic workloads: problem parameters and initial conditions.

This module holds no arithmetic of the method.  It only draws inputs (grid,
physical and time-step parameters, initial states, request streams) so that
the HIP library and the test oracle receive the same arrays.  It imports
nothing but numpy.

State layout: float64 array (3, nz, nx), fields (u, w, p), x fastest.

Parameter readings of the constant-velocity workloads (advection by a
constant U along x; the paper's own rotating-flow runs are built by
``rotation_problem``):
  * fine step  dt_f = 0.2 * min(dx, dz) / c_s   (fine CFL 0.2, Section 3.2)
  * coarse step dt_g = 10 * dt_f                 (coarse CFL 2.0, Table 1)
  * nu_f = 0.005, nu_c = 0.1 (Section 3.2)
  * N_sound: the smallest of 4, 6, 8, 10 for which the split-explicit coarse
    propagator is stable at the given U (4 up to U = 0.15, 6 up to 0.2,
    8 up to 0.25, 10 up to 0.3); the paper raises N_sound the same way to
    keep G stable (Section 3.2.3)
  * one window: P slices of length T/P, T = 1
"""

import math

import numpy as np

NU_F = 0.005
NU_C = 0.1
RANK_TOL = 1e-10


def n_sound_for(U):
    """Minimum stable number of acoustic substeps for |U| <= 0.3."""
    a = abs(U)
    for limit, ns in ((0.15, 4), (0.2, 6), (0.25, 8), (0.3, 10)):
        if a <= limit + 1e-12:
            return ns
    raise ValueError(f"no stable N_sound tabulated for U={U}")


def problem(nx, nz, P, U=0.1, c_s=1.0, T=1.0, cfl_f=0.2, coarse_ratio=10,
            n_sound=None, windows=1):
    """Plain dict of problem parameters shared by the library and the oracle.
    ``windows`` parallel steps of P slices cover [0, T]."""
    dt_f = cfl_f * min(1.0 / nx, 1.0 / nz) / c_s
    return dict(nx=int(nx), nz=int(nz), c_s=float(c_s), U=float(U),
                dt_f=dt_f, dt_g=coarse_ratio * dt_f, P=int(P), T=float(T),
                nu_f=NU_F, nu_c=NU_C,
                n_sound=int(n_sound if n_sound is not None else n_sound_for(U)),
                rank_tol=RANK_TOL, windows=int(windows))


def one_coarse_step_windows(prob):
    """The window count that makes every slice one coarse step (the paper's
    runs: N_c = N_p coarse intervals per parallel step, Section 2.1):
    T / (P * dt_g)."""
    m = prob["T"] / (prob["P"] * prob["dt_g"])
    M = int(round(m))
    if M < 1 or abs(M - m) > 1e-9 * m:
        raise ValueError("T / (P dt_g) is not an integer")
    return M


def rotation_problem(n, P, cfl_c, T=2.0):
    """The solid-body-rotation runs of Section 3.2 on n x n cells: velocity
    pi (z - 1/2, -(x - 1/2)) (eq. adVel, one revolution in T = 2), c_s = 30,
    fine CFL 0.2, coarse CFL ``cfl_c`` (2 or 4 in Tables 1-2), N_sound = 4,
    nu_f = 0.005, nu_c = 0.1, second-order acoustic fluxes in both
    propagators, and the paper's decomposition: every slice is one coarse
    step, windows of P slices cover [0, T]."""
    ratio = int(round(cfl_c / 0.2))
    prob = problem(n, n, P, U=0.0, c_s=30.0, T=T, cfl_f=0.2,
                   coarse_ratio=ratio, n_sound=4)
    prob.update(gamma=math.pi, fine_acoustic_order=2)
    prob["windows"] = one_coarse_step_windows(prob)
    return prob


def _cell_centres(nx, nz):
    x = (np.arange(nx) + 0.5) / nx
    z = (np.arange(nz) + 0.5) / nz
    return np.meshgrid(x, z)  # (nz, nx) each


def gaussian_bump(nx, nz, centre, width=0.05, amp=1.0):
    """amp * exp(-(dx^2 + dz^2) / (2 width^2)) with periodic minimum-image
    distances to ``centre`` on the unit square."""
    X, Z = _cell_centres(nx, nz)
    ddx = X - centre[0]
    ddz = Z - centre[1]
    ddx -= np.round(ddx)
    ddz -= np.round(ddz)
    return amp * np.exp(-(ddx * ddx + ddz * ddz) / (2.0 * width * width))


def ic_bumps(nx, nz, seed, nbumps=1, noise=0.0, width=0.05, amp=1.0):
    """Pressure = sum of ``nbumps`` Gaussian bumps at uniformly drawn centres;
    u, w = N(0, noise^2) i.i.d. per point (zero when noise == 0)."""
    rng = np.random.default_rng(seed)
    q = np.zeros((3, nz, nx))
    for _ in range(nbumps):
        c = rng.random(2)
        q[2] += gaussian_bump(nx, nz, c, width, amp)
    if noise > 0.0:
        q[0] += rng.normal(0.0, noise, (nz, nx))
        q[1] += rng.normal(0.0, noise, (nz, nx))
    return q


def ic_fourier(nx, nz, seed, nmodes=32, kmax=64):
    """Pressure = sum of ``nmodes`` random-phase Fourier modes
    cos(2 pi (kx x + kz z) + phi) / sqrt(nmodes) with integer
    1 <= max(|kx|, |kz|) <= kmax; u = w = 0."""
    rng = np.random.default_rng(seed)
    X, Z = _cell_centres(nx, nz)
    q = np.zeros((3, nz, nx))
    m = 0
    while m < nmodes:
        kx, kz = rng.integers(-kmax, kmax + 1, size=2)
        if max(abs(kx), abs(kz)) == 0:
            continue
        phi = rng.random() * 2.0 * math.pi
        q[2] += np.cos(2.0 * math.pi * (kx * X + kz * Z) + phi)
        m += 1
    q[2] /= math.sqrt(nmodes)
    return q


def ic_cosine_bell(nx, nz, centre=(0.5, 0.5)):
    """The initial value of the instability example (Section 3.1): u =
    (cos(pi r) + 1)/2 with r = min(1, 4 sqrt(((x-x0)/0.5)^2 +
    ((z-z0)/0.5)^2)), w = p = 0."""
    X, Z = _cell_centres(nx, nz)
    r = np.minimum(1.0, 4.0 * np.sqrt(((X - centre[0]) / 0.5) ** 2
                                      + ((Z - centre[1]) / 0.5) ** 2))
    q = np.zeros((3, nz, nx))
    q[0] = 0.5 * (np.cos(np.pi * r) + 1.0)
    return q


# The five workloads: small oracle-scale run, single plain solve, batched
# fused solve, serving stream, large single instance.
CONFIGS = {
    "c1_64x32": dict(nx=64, nz=32, P=8, K=3, U=0.1, seed=1,
                     ic=dict(kind="bumps", nbumps=1)),
    "c2_512x256": dict(nx=512, nz=256, P=32, K=4, U=0.1, seed=2,
                       ic=dict(kind="bumps", nbumps=4, noise=1e-3)),
    "c3_1024x512": dict(nx=1024, nz=512, P=64, K=5, U=0.1, seed=3,
                        ic=dict(kind="bumps", nbumps=4, noise=1e-3)),
    "c5_4096x1024": dict(nx=4096, nz=1024, P=128, K=4, U=0.2, seed=5,
                         ic=dict(kind="fourier", nmodes=32, kmax=64)),
    # The paper's own time decomposition (Section 2.1): every slice is one
    # coarse step, [0, T] is covered by T / (P dt_g) windows of P slices.
    "c1w_64x32": dict(nx=64, nz=32, P=8, K=3, U=0.1, seed=1,
                      ic=dict(kind="bumps", nbumps=1), windows="one_step"),
    "c2w_512x256": dict(nx=512, nz=256, P=32, K=4, U=0.1, seed=2,
                        ic=dict(kind="bumps", nbumps=4, noise=1e-3),
                        windows="one_step"),
    # The instability example of Section 3.1 on the acoustic-advection
    # system: 40 x 40 cells, U = (1, 1), c_s = 1, RK-3 for both propagators
    # (scheme "rk3"), 6 slices per window, 5 iterations.  Delta t = 1/72
    # (Courant number U Delta t / dx = 0.556 per direction) and delta t =
    # Delta t / 6 (0.093) make T = 1 exactly 12 windows of 6 coarse steps;
    # Delta t = 1/66 (0.606) would make the coarse propagator itself
    # unstable at c_s = 1.
    "demo_40x40": dict(nx=40, nz=40, P=6, K=5, U=1.0, V=1.0, c_s=1.0,
                       ic=dict(kind="cosine_bell"), scheme="rk3",
                       dt_g=1.0 / 72.0, coarse_ratio=6, windows=12),
    # The paper's own runs (Section 3.2, Figures vorticity to energy, Table
    # 2): solid-body rotation at coarse CFL 4 with N_p = 6 slices per
    # window, 100 windows over T = 2, the cosine bell in u at (0.5, 0.65).
    "rot_40x40": dict(nx=40, nz=40, P=6, K=2, rotation=dict(cfl_c=4.0),
                      ic=dict(kind="cosine_bell", centre=(0.5, 0.65))),
    "rot_80x80": dict(nx=80, nz=80, P=6, K=2, rotation=dict(cfl_c=4.0),
                      ic=dict(kind="cosine_bell", centre=(0.5, 0.65))),
}

# The cells of Tables 1 and 2 of Section 3.2 on 40 x 40 cells: (coarse CFL,
# slices per window, iterations per window).
PAPER_TABLE_CELLS = tuple(
    (cc, P, K) for cc in (2.0, 4.0)
    for P, kmax in ((4, 2), (6, 3), (8, 4)) for K in range(1, kmax + 1))


def config(name):
    """(problem dict, K, initial state) of a named workload."""
    c = CONFIGS[name]
    if "rotation" in c:
        prob = rotation_problem(c["nx"], c["P"], **c["rotation"])
        return prob, c["K"], ic_cosine_bell(c["nx"], c["nz"],
                                            centre=c["ic"]["centre"])
    prob = problem(c["nx"], c["nz"], c["P"], U=c["U"], c_s=c.get("c_s", 1.0),
                   n_sound=1 if c.get("scheme") == "rk3" else None)
    if c.get("windows") == "one_step":
        prob["windows"] = one_coarse_step_windows(prob)
    elif "windows" in c:
        prob["windows"] = c["windows"]
    if c.get("scheme") == "rk3":
        # Section 3.1: no damping, no acoustic substeps
        prob.update(scheme="rk3", V=c["V"], nu_f=0.0, nu_c=0.0, n_sound=1,
                    dt_g=c["dt_g"], dt_f=c["dt_g"] / c["coarse_ratio"])
        prob["T"] = prob["windows"] * prob["P"] * prob["dt_g"]
    ic = dict(c["ic"])
    kind = ic.pop("kind")
    if kind == "bumps":
        u0 = ic_bumps(c["nx"], c["nz"], c["seed"], **ic)
    elif kind == "cosine_bell":
        u0 = ic_cosine_bell(c["nx"], c["nz"], **ic)
    else:
        u0 = ic_fourier(c["nx"], c["nz"], c["seed"], **ic)
    return prob, c["K"], u0


SERVE_GRIDS = ((128, 64), (256, 128), (512, 256), (1024, 512))
# Arrival rate of the served stream (requests per second): 0.8 times the
# closed-loop throughput of the same seeded mix, 8.0 solves/s on one MI355X
# with 64 requests submitted at once (bench.py --serve-calibrate --serve 64),
# measured once and frozen here.
SERVE_RATE = 6.4
SERVE_SLICES = (8, 16, 32, 64)


def serving_stream(n_requests, rate_per_s, seed=4, grids=SERVE_GRIDS,
                   slices=SERVE_SLICES, K=4):
    """Seeded Poisson stream of KSE-Parareal requests.

    Each request: grid uniform over ``grids``, U ~ U[0, 0.3], P uniform over
    ``slices``, K fixed, 1-4 Gaussian pressure bumps.  Arrival times are the
    cumulative sums of Exp(rate) gaps.  Returns a list of dicts with keys
    t_arrival, prob, K, u0 (u0 is generated lazily by ``request_state``).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        nx, nz = grids[rng.integers(len(grids))]
        P = int(slices[rng.integers(len(slices))])
        U = float(rng.uniform(0.0, 0.3))
        nb = int(rng.integers(1, 5))
        reqs.append(dict(id=r, t_arrival=t, prob=problem(nx, nz, P, U=U), K=K,
                         ic_seed=int(rng.integers(1 << 31)), nbumps=nb))
    return reqs


def request_state(req):
    p = req["prob"]
    return ic_bumps(p["nx"], p["nz"], req["ic_seed"], nbumps=req["nbumps"])
