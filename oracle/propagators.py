"""Fine and coarse propagators of the oracle (Section 3.2).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

F: non-split three-stage Runge-Kutta (the Wicker-Skamarock RK3 of the NWP
   literature the paper cites: stages at 1/3, 1/2 and 1 of the step, each
   restarting from q^n) with the fine right-hand side ``rhs_fine``.
G: partially split forward Euler: the advective (slow) tendency is computed
   once per coarse step and held fixed while N_sound forward-backward
   acoustic substeps advance the state.

With scheme "rk3" (the instability example of Section 3.1) both F and G
are RK3 with the right-hand sides of ``rhs_rk3_pair``: sixth-order centred
advective fluxes in F, first-order upwind in G.

Both map a state over one slice, i.e. n_f fine or n_g coarse steps, as
F_{delta t}(q, t_{i+1}, t_i) and G_{Delta t}(q, t_{i+1}, t_i) of Section
2.1.  The system is autonomous, so neither depends on t_i.
"""

import numpy as np

from .operators import (Params, rhs_fine, rhs_rk3_pair, coarse_slow_tendency,
                        acoustic_substep)


def _fine_rhs(prm: Params):
    if prm.scheme == "rk3":
        return lambda q, p: rhs_rk3_pair(q, p, coarse=False)
    return rhs_fine


def rk3_step(q, dt, prm: Params, rhs=None):
    """One RK3 step of the fine right-hand side (or ``rhs``):
    q* = q + dt/3 f(q), q** = q + dt/2 f(q*), q^{n+1} = q + dt f(q**)."""
    f = _fine_rhs(prm) if rhs is None else rhs
    q1 = q + (dt / 3.0) * f(q, prm)
    q2 = q + (dt / 2.0) * f(q1, prm)
    return q + dt * f(q2, prm)


def fine_F(q, prm: Params, nsteps=None):
    """F over one slice: ``nsteps`` (default n_f) RK3 steps of dt_f."""
    n = prm.n_f if nsteps is None else nsteps
    q = np.array(q, dtype=np.float64, copy=True)
    for _ in range(n):
        q = rk3_step(q, prm.dt_f, prm)
    return q


def coarse_step(q, prm: Params):
    """One coarse step of length dt_g: partially split forward Euler, or
    for scheme "rk3" one RK3 step of the first-order upwind right-hand
    side."""
    if prm.scheme == "rk3":
        return rk3_step(q, prm.dt_g, prm,
                        rhs=lambda x, p: rhs_rk3_pair(x, p, coarse=True))
    R = coarse_slow_tendency(q, prm)
    dtau = prm.dt_g / prm.n_sound
    for _ in range(prm.n_sound):
        q = acoustic_substep(q, R, dtau, prm)
    return q


def coarse_G(q, prm: Params, nsteps=None):
    """G over one slice: ``nsteps`` (default n_g) coarse steps."""
    n = prm.n_g if nsteps is None else nsteps
    q = np.array(q, dtype=np.float64, copy=True)
    for _ in range(n):
        q = coarse_step(q, prm)
    return q


def serial_fine(u0, prm: Params, nslices=None):
    """Reference run of F sequentially over ``nslices`` slices (default all
    windows * P of them), i.e. q_seq of eq. errorDef at t = T."""
    q = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(prm.windows * prm.P if nslices is None else nslices):
        q = fine_F(q, prm)
    return q
