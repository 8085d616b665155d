"""Units, time step and Yee dispersion constants (oracle, FP64).

Normalised units used throughout the oracle: c = 1 and the laser angular
frequency omega = 1, so lengths are in c/omega, times in 1/omega, fields in
m c omega / |e| (a field of amplitude a0 is the paper's a0 = |e|E0/(m c omega),
Sec. II.A, Fig. 3 caption), densities in the critical density n_c (so a
species of density n has omega_p^2 = n q^2/m) and momenta u = gamma*beta.
Maxwell's equations (1)-(2) become dB/dt = -curl E, dE/dt = curl B - J.

Configurations are written in "lambda units" (lambda = 1, c = 1); one lambda
is 2*pi internal length units and one lambda/c is 2*pi internal time units.
"""
import math

TWO_PI = 2.0 * math.pi
LAMBDA = TWO_PI          # one wavelength in internal length units
PERIOD = TWO_PI          # one laser period in internal time units

DISP_PAPER2 = 0          # second-order forms, Eqs. (12)-(14)
DISP_EXACT = 1           # exact Yee forms, Eqs. (10)-(11)
DISP_VACUUM = 2          # v_phi = v_g = c, B0 = E0 (continuum)
DISP_PLASMA = 3          # exact Yee forms with an analytic current J1, Sec. IV


def default_dt(dx_min, dim):
    """Time step rule stated after Eq. (14): c dt / dx = 0.95 / sqrt(D)."""
    return 0.95 / math.sqrt(dim) * dx_min


def dispersion(mode, dx, dt, wp2=0.0, zeta=1.0):
    """Phase velocity, group velocity and B0/E0 of a Yee-advanced wave.

    ``dx`` is the cell size along the propagation axis and ``dt`` the time
    step, both internal units; omega = 1.  Returns (v_phi, v_g, b_over_e, k).

    * PAPER2: Eqs. (12), (13), (14), the second-order forms the paper uses
      for E1 and B1.
    * EXACT:  Eq. (10) solved for k, v_g = d omega / d k from the same
      relation, B0/E0 from Eq. (11).
    * VACUUM: the continuum limit (Sec. II.A, last paragraph: the naive
      choice that is only consistent without a grid).
    * PLASMA: Sec. IV, the Yee scheme with the analytic current J1 of a
      linear plasma response evaluated at the half step: the dispersion
      relation sin^2(w dt/2) - (wp2/w^2)(w dt/2) sin(w dt/2) zeta =
      (c dt/dx)^2 sin^2(k dx/2) solved for k, v_g = d omega/d k from the same
      relation (zeta held fixed), and B0/E0 = cos(w dt/2) sqrt(1 - (wp2/w^2)
      zeta (w dt/2)/sin(w dt/2)).  wp2 is omega_p^2 of the density J1 uses,
      zeta the factor of the plasma's discrete response.  wp2 = 0 gives EXACT.
    """
    omega = 1.0
    if mode == DISP_PAPER2:
        c2 = (dt / dx) ** 2
        v_phi = 1.0 - (1.0 / 24.0) * (1.0 - c2) * (omega * dx) ** 2
        v_g = 1.0 - (1.0 / 8.0) * (1.0 - c2) * (omega * dx) ** 2
        b_over_e = 1.0 - (omega * dt) ** 2 / 8.0
    elif mode == DISP_EXACT:
        courant = dt / dx
        # sin^2(omega dt/2) = courant^2 sin^2(k dx/2)
        k = (2.0 / dx) * math.asin(math.sin(omega * dt / 2.0) / courant)
        v_phi = omega / k
        # differentiate both sides of Eq. (10):
        # sin(w dt/2) cos(w dt/2) dt dw = C^2 sin(k dx/2) cos(k dx/2) dx dk
        num = courant ** 2 * math.sin(k * dx / 2.0) * math.cos(k * dx / 2.0) * dx
        den = math.sin(omega * dt / 2.0) * math.cos(omega * dt / 2.0) * dt
        v_g = num / den
        b_over_e = math.cos(omega * dt / 2.0)
    elif mode == DISP_PLASMA:
        courant = dt / dx
        h = omega * dt / 2.0
        s, c = math.sin(h), math.cos(h)
        lhs = s * s - (wp2 / omega ** 2) * h * s * zeta
        if not (lhs > 0.0) or math.sqrt(lhs) / courant > 1.0:
            raise ValueError("no propagating Yee mode for this plasma density")
        k = (2.0 / dx) * math.asin(math.sqrt(lhs) / courant)
        v_phi = omega / k
        # lhs(w) = sin^2(w dt/2) - wp2 zeta (dt/2) sin(w dt/2) / w
        dlhs = s * c * dt - wp2 * zeta * (dt / 2.0) * ((dt / 2.0) * c / omega - s / omega ** 2)
        drhs = courant ** 2 * math.sin(k * dx / 2.0) * math.cos(k * dx / 2.0) * dx
        v_g = drhs / dlhs
        b_over_e = c * math.sqrt(1.0 - (wp2 / omega ** 2) * zeta * h / s)
    elif mode == DISP_VACUUM:
        v_phi, v_g, b_over_e = 1.0, 1.0, 1.0
    else:
        raise ValueError("unknown dispersion mode %r" % (mode,))
    return v_phi, v_g, b_over_e, omega / v_phi
