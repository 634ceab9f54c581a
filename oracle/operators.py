"""Flux-form finite-difference operators of the oracle (Section 3).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper writes the semi-discrete system in conservation form on equal
rectangular cells: the tendency of a cell value is minus the x-difference of
interface fluxes over dx minus the z-difference of interface fluxes over dz
(Section 3, the flux-difference formula below eq. acousticAd).  Every
operator here is written that way: an interface flux is computed on the
x- (or z-) faces, then differenced.  The flux stencils are those of the
Wicker-Skamarock family the paper cites for orders one to six.

The acoustic-advection system (eq. acousticAd) with the paper's divergence
damping (the modified momentum equations of Section 3.2, coefficients of
eq. dampingCoeff) reads, for an advection velocity (U_x, U_z),

    u_t = -U_x u_x - U_z u_z - c_s p_x         + alpha_1 (div u)_x
    w_t = -U_x w_x - U_z w_z - c_s p_z         + alpha_2 (div u)_z
    p_t = -U_x p_x - U_z p_z - c_s (u_x + w_z)

The velocity is (U + gamma (z - Lz/2), V - gamma (x - Lx/2)): a constant
part plus the solid-body rotation of eq. adVel (gamma = pi there, U = V = 0).
Its x-component depends on z only and its z-component on x only, so it is
divergence-free, the advective form equals the flux form, and the velocity
on an x-face (a z-face) is the exact value of the row (the column): no
interpolation to the faces is needed.

Array convention: a field is an (nz, nx) array, x along axis 1.
``_at(q, m, axis)`` returns the field shifted so that entry i holds q_{i+m}
(periodic).
"""

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Params:
    """One KSE-Parareal problem on the periodic unit square.

    nx, nz      cells along x and z (dx = Lx/nx, dz = Lz/nz)
    c_s         sound speed
    U, V        constant part of the advection velocity along x and z
    gamma       rotation rate of the solid-body part of the velocity (eq.
                adVel: gamma = pi, one revolution in T = 2); split scheme only
    dt_f, dt_g  fine step (delta t) and coarse step (Delta t)
    P           number of time slices N_c of one window (parallel step)
    T           end time
    windows     number of parallel steps M_p (Section 2.1): [0, T] is
                covered by ``windows`` windows of P slices each, a slice
                being T / (windows * P) long
    scheme      "split": the propagators of Section 3.2 (F: RK-3, fifth-order
                upwind advection, fourth-order centred acoustics, damping;
                G: partially split forward Euler).  "rk3": those of the
                instability example of Section 3.1 (F: RK-3 with the
                sixth-order centred advective flux; G: RK-3 with the
                first-order upwind flux; both with second-order centred
                acoustic fluxes and no damping)
    coarse_order  order of the upwind advective flux of the split G: 1 (the
                main runs of Section 3.2) or 3 (its less diffusive G)
    fine_acoustic_order  order of the centred acoustic fluxes of the split
                F: 4, or 2 (Section 3 computes the acoustic fluxes of both
                propagators to second order)
    nu_f, nu_c  divergence-damping factors of F and G (eq. dampingCoeff)
    n_sound     acoustic substeps per coarse step (N_sound, Section 3.2)
    rank_tol    relative tolerance on |R_jj|/|R_11| for the rank of the
                pivoted QR in the subspace update (the paper names DGEQP3
                but no tolerance)
    """

    nx: int
    nz: int
    c_s: float
    U: float
    dt_f: float
    dt_g: float
    P: int
    T: float = 1.0
    nu_f: float = 0.005
    nu_c: float = 0.1
    n_sound: int = 4
    rank_tol: float = 1e-10
    Lx: float = 1.0
    Lz: float = 1.0
    windows: int = 1
    scheme: str = "split"
    V: float = 0.0
    coarse_order: int = 1
    gamma: float = 0.0
    fine_acoustic_order: int = 4

    def __post_init__(self):
        if self.scheme not in ("split", "rk3"):
            raise ValueError(f"unknown scheme {self.scheme!r}")
        if self.scheme == "rk3" and self.gamma != 0.0:
            raise ValueError("the Section 3.1 pair advects with a constant "
                             "velocity (gamma = 0)")
        if self.coarse_order not in (1, 3):
            raise ValueError("coarse_order must be 1 or 3")
        if self.fine_acoustic_order not in (2, 4):
            raise ValueError("fine_acoustic_order must be 2 or 4")

    @property
    def dx(self):
        return self.Lx / self.nx

    @property
    def dz(self):
        return self.Lz / self.nz

    @property
    def d(self):
        return 3 * self.nx * self.nz

    @property
    def slice_length(self):
        """Length of one time slice, T / (windows * P)."""
        return self.T / (self.windows * self.P)

    @property
    def n_f(self):
        """Fine steps per slice, N_f = slice length / dt_f (Section 2.1)."""
        return _integer_ratio(self.slice_length, self.dt_f)

    @property
    def n_g(self):
        """Coarse steps per slice, slice length / dt_g."""
        return _integer_ratio(self.slice_length, self.dt_g)


def _integer_ratio(a, b):
    n = int(round(a / b))
    if n < 1 or abs(n * b - a) > 1e-9 * abs(a):
        raise ValueError(f"{a} is not an integer multiple of {b}")
    return n


def velocity_x(prm: Params):
    """x-component of the advection velocity on the x-faces of each row,
    shape (nz, 1): U + gamma (z_j - Lz/2) at the row's height z_j."""
    z = (np.arange(prm.nz) + 0.5) * prm.dz
    return (prm.U + prm.gamma * (z - 0.5 * prm.Lz))[:, None]


def velocity_z(prm: Params):
    """z-component of the advection velocity on the z-faces of each column,
    shape (1, nx): V - gamma (x_i - Lx/2) at the column's position x_i."""
    x = (np.arange(prm.nx) + 0.5) * prm.dx
    return (prm.V - prm.gamma * (x - 0.5 * prm.Lx))[None, :]


def _at(q, m, axis):
    """q_{i+m} along ``axis`` with periodic wrap."""
    return np.roll(q, -m, axis=axis)


# ---------------------------------------------------------------------------
# Interface fluxes.  Each returns the flux on the face i+1/2 (stored at i).
# ---------------------------------------------------------------------------

def flux_upwind5(q, vel, axis):
    """Fifth-order upwind advective flux of the Wicker-Skamarock family:
    the sixth-order centred flux minus |vel| times a fifth-difference
    dissipation term.  Valid for either sign of ``vel``."""
    c6 = (37.0 * (_at(q, 1, axis) + q)
          - 8.0 * (_at(q, 2, axis) + _at(q, -1, axis))
          + (_at(q, 3, axis) + _at(q, -2, axis)))
    dis = ((_at(q, 3, axis) - _at(q, -2, axis))
           - 5.0 * (_at(q, 2, axis) - _at(q, -1, axis))
           + 10.0 * (_at(q, 1, axis) - q))
    return vel / 60.0 * c6 - abs(vel) / 60.0 * dis


def flux_centred6(q, axis):
    """Sixth-order centred interface value of the Wicker-Skamarock family,
    (37(q_i + q_{i+1}) - 8(q_{i-1} + q_{i+2}) + (q_{i-2} + q_{i+3}))/60."""
    return (37.0 * (q + _at(q, 1, axis))
            - 8.0 * (_at(q, -1, axis) + _at(q, 2, axis))
            + (_at(q, -2, axis) + _at(q, 3, axis))) / 60.0


def flux_upwind3(q, vel, axis):
    """Third-order upwind advective flux of the Wicker-Skamarock family:
    the fourth-order centred flux plus |vel| times a third-difference
    dissipation term."""
    c4 = 7.0 * (q + _at(q, 1, axis)) - (_at(q, -1, axis) + _at(q, 2, axis))
    dis = ((_at(q, 2, axis) - _at(q, -1, axis))
           - 3.0 * (_at(q, 1, axis) - q))
    return vel / 12.0 * c4 + abs(vel) / 12.0 * dis


def flux_upwind1(q, vel, axis):
    """First-order upwind advective flux: centred average minus |vel|/2
    times the jump."""
    return (vel * 0.5 * (q + _at(q, 1, axis))
            - abs(vel) * 0.5 * (_at(q, 1, axis) - q))


def flux_centred4(q, axis):
    """Fourth-order centred interface value (7(q_i+q_{i+1}) - (q_{i-1}+q_{i+2}))/12."""
    return (7.0 * (q + _at(q, 1, axis))
            - (_at(q, -1, axis) + _at(q, 2, axis))) / 12.0


def flux_centred2(q, axis):
    """Second-order centred interface value (q_i + q_{i+1})/2."""
    return 0.5 * (q + _at(q, 1, axis))


def flux_div(flux, h, axis):
    """(F_{i+1/2} - F_{i-1/2}) / h."""
    return (flux - _at(flux, -1, axis)) / h


# ---------------------------------------------------------------------------
# Divergence damping: alpha_1 (div u)_x and alpha_2 (div u)_z.
# div u is evaluated on the faces where it is differenced: on an x-face the
# normal derivative u_x is the two-point jump and the tangential w_z is the
# centred z-difference of the face-averaged w; likewise on a z-face.  The
# face values are then differenced like any flux.
# ---------------------------------------------------------------------------

def grad_div(u, w, dx, dz):
    """Return ((div u)_x, (div u)_z) at cell centres."""
    X, Z = 1, 0
    w_face = 0.5 * (w + _at(w, 1, X))                     # w on x-faces
    div_xface = (_at(u, 1, X) - u) / dx + \
        (_at(w_face, 1, Z) - _at(w_face, -1, Z)) / (2.0 * dz)
    u_face = 0.5 * (u + _at(u, 1, Z))                     # u on z-faces
    div_zface = (_at(w, 1, Z) - w) / dz + \
        (_at(u_face, 1, X) - _at(u_face, -1, X)) / (2.0 * dx)
    return flux_div(div_xface, dx, X), flux_div(div_zface, dz, Z)


# ---------------------------------------------------------------------------
# Right-hand sides.
# ---------------------------------------------------------------------------

def advection(f, prm: Params, flux):
    """Flux-form advective tendency (U_x f)_x + (U_z f)_z of one field with
    the upwind interface flux ``flux`` in both directions.  The z-term is
    left out when the velocity has no z-component (V = gamma = 0)."""
    X, Z = 1, 0
    a = flux_div(flux(f, velocity_x(prm), X), prm.dx, X)
    if prm.V != 0.0 or prm.gamma != 0.0:
        a = a + flux_div(flux(f, velocity_z(prm), Z), prm.dz, Z)
    return a


def rhs_fine(q, prm: Params):
    """f(q) of the fine propagator F (Section 3.2 and eq. acousticAd):
    fifth-order upwind advection, fourth-order (or, with
    fine_acoustic_order 2, second-order) centred acoustic fluxes and
    divergence damping with alpha = nu_f * h^2 / dt_f (eq. dampingCoeff,
    tau = delta t)."""
    X, Z = 1, 0
    u, w, p = q
    dx, dz, c = prm.dx, prm.dz, prm.c_s
    ac = flux_centred4 if prm.fine_acoustic_order == 4 else flux_centred2
    ax = prm.nu_f * dx * dx / prm.dt_f
    az = prm.nu_f * dz * dz / prm.dt_f
    gdx, gdz = grad_div(u, w, dx, dz)
    fu = (-advection(u, prm, flux_upwind5)
          - c * flux_div(ac(p, X), dx, X) + ax * gdx)
    fw = (-advection(w, prm, flux_upwind5)
          - c * flux_div(ac(p, Z), dz, Z) + az * gdz)
    fp = (-advection(p, prm, flux_upwind5)
          - c * (flux_div(ac(u, X), dx, X) + flux_div(ac(w, Z), dz, Z)))
    return np.stack([fu, fw, fp])


def rhs_rk3_pair(q, prm: Params, coarse):
    """f(q) of the Section 3.1 propagators (scheme "rk3"): advection with
    velocity (U, V) by the sixth-order centred flux (F) or the first-order
    upwind flux (G) in both directions, acoustic fluxes second-order
    centred, no damping."""
    X, Z = 1, 0
    u, w, p = q
    dx, dz, c, U, V = prm.dx, prm.dz, prm.c_s, prm.U, prm.V
    if coarse:
        adv = lambda f: (flux_div(flux_upwind1(f, U, X), dx, X)
                         + flux_div(flux_upwind1(f, V, Z), dz, Z))
    else:
        adv = lambda f: (flux_div(U * flux_centred6(f, X), dx, X)
                         + flux_div(V * flux_centred6(f, Z), dz, Z))
    fu = -adv(u) - c * flux_div(flux_centred2(p, X), dx, X)
    fw = -adv(w) - c * flux_div(flux_centred2(p, Z), dz, Z)
    fp = -adv(p) - c * (flux_div(flux_centred2(u, X), dx, X)
                        + flux_div(flux_centred2(w, Z), dz, Z))
    return np.stack([fu, fw, fp])


def coarse_slow_tendency(q, prm: Params):
    """Slow (advective) tendency of the partially split coarse scheme:
    first-order upwind advection (third-order with ``coarse_order`` 3, the
    less diffusive G of Section 3.2), evaluated once per coarse step and
    held fixed over its acoustic substeps (Section 3.2)."""
    flux = flux_upwind3 if prm.coarse_order == 3 else flux_upwind1
    return np.stack([-advection(f, prm, flux) for f in q])


def acoustic_substep(q, R, dtau, prm: Params):
    """One forward-backward acoustic substep of length dtau = Delta t/N_sound
    (Section 3.2): momentum forward with the old pressure and divergence
    damping (alpha = nu_c h^2 / dtau), then pressure backward with the new
    velocities.  ``R`` is the frozen slow tendency."""
    X, Z = 1, 0
    u, w, p = q
    dx, dz, c = prm.dx, prm.dz, prm.c_s
    ax = prm.nu_c * dx * dx / dtau
    az = prm.nu_c * dz * dz / dtau
    gdx, gdz = grad_div(u, w, dx, dz)
    un = u + dtau * (R[0] - c * flux_div(flux_centred2(p, X), dx, X)
                     + ax * gdx)
    wn = w + dtau * (R[1] - c * flux_div(flux_centred2(p, Z), dz, Z)
                     + az * gdz)
    pn = p + dtau * (R[2] - c * (flux_div(flux_centred2(un, X), dx, X)
                                 + flux_div(flux_centred2(wn, Z), dz, Z)))
    return np.stack([un, wn, pn])
