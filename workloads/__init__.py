"""Seeded synthetic workloads shared by the tests, the smoke check and the bench.

This module only produces inputs: box sizes, boundary types, wing placement,
flow parameters (Re, J, f) and seeded random arrays.  It holds none of the
method's arithmetic: the mapping from (Re, J, f) to lattice parameters, marker
generation and kinematics are done separately by the solver library and by the
oracle.  Both sides receive the same dicts and arrays from here.

Workloads follow the paper's setups (clap & fling of two elliptic foils of
aspect ratio 5, Sec. 3.3; sweep Re x J x f) lifted to 3D D3Q19 boxes.
"""
from __future__ import annotations

import math

import numpy as np

# Boundary codes, per face (-x, +x, -y, +y, -z, +z).
PERIODIC, WALL, VELOCITY, PRESSURE, ZH_VELOCITY, ZH_PRESSURE = 0, 1, 2, 3, 4, 5
# alpha(t) shapes.
ALPHA_CONST, ALPHA_SIN, ALPHA_ABS_SIN = 0, 1, 2

RE_SET = (75.0, 100.0, 150.0)
J_SET = (0.001, 0.01, 2.0)
F_SET = (0.05, 0.25)
KAPPA = 0.2          # lattice tip speed per unit "Hz": U_tip = KAPPA * f
PHI_OPEN = 2.0 * math.pi / 3.0   # maximum opening angle, 120 degrees (Sec. 3.3, Eq. 24)


def velocity_noise(shape_zyx, seed, amp=1e-4, dtype=np.float64):
    """Uniform noise in [-amp, amp] per velocity component, PCG64(seed).

    Returns an array of shape (3, nz, ny, nx), component order (x, y, z).
    """
    nz, ny, nx = shape_zyx
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-amp, amp, size=(3, nz, ny, nx)).astype(dtype)


def box(nx, ny, nz, bc, tau, u_in=(0.0, 0.0, 0.0), rho_out=1.0,
        body_force=(0.0, 0.0, 0.0), u_ref=1.0, area_ref=1.0):
    """A plain box description (lattice units)."""
    return dict(nx=int(nx), ny=int(ny), nz=int(nz), bc=list(bc), tau=float(tau),
                u_in=[float(v) for v in u_in], rho_out=float(rho_out),
                body_force=[float(v) for v in body_force],
                u_ref=float(u_ref), area_ref=float(area_ref))


def wing(chord, thickness, hinge, pivot_frac, theta0, sense, alpha_shape,
         alpha_mean=0.0, alpha_amp=0.0, period_steps=1.0, phase=0.0,
         trans_amp=0.0, trans_angle=0.0, ds=1.0):
    """One rigid elliptic foil extruded over the full periodic span."""
    return dict(chord=float(chord), thickness=float(thickness), ds=float(ds),
                hinge=[float(hinge[0]), float(hinge[1])],
                pivot_frac=float(pivot_frac), theta0=float(theta0),
                sense=float(sense), alpha_shape=int(alpha_shape),
                alpha_mean=float(alpha_mean), alpha_amp=float(alpha_amp),
                period_steps=None if period_steps is None else float(period_steps),
                phase=float(phase),
                trans_amp=float(trans_amp), trans_angle=float(trans_angle))


def plate_case(nx=64, ny=32, nz=32, chord=10.0, aspect=5.0, u_inf=0.02, re=100.0,
               aoa_deg=30.0, centre=(20.0, 15.5)):
    """Fixed elliptic plate at an angle of attack in a channel.

    Inlet at -x with uniform u_inf, equilibrium outlet at +x (rho = 1),
    half-way bounce-back walls in y, periodic span in z.  Re = u_inf*c/nu, so
    the relaxation time is passed as (re, u_inf, chord) and the solver maps it.
    Returns (box_params, wings, physics) where physics holds the raw numbers;
    `tau` is left out of the box and follows from physics on each side.
    """
    phys = dict(kind="plate", re=re, u_inf=u_inf, chord=chord)
    bx = dict(nx=nx, ny=ny, nz=nz,
              bc=[VELOCITY, PRESSURE, WALL, WALL, PERIODIC, PERIODIC],
              u_in=[u_inf, 0.0, 0.0], rho_out=1.0, body_force=[0.0, 0.0, 0.0],
              u_ref=u_inf, area_ref=chord * nz)
    # chord angle -aoa: leading edge upstream and above the trailing edge
    wg = [wing(chord, chord / aspect, centre, 0.5, -math.radians(aoa_deg), -1.0,
               ALPHA_CONST)]
    return bx, wg, phys


def cylinder_case(nx=64, ny=48, nz=8, d=8.0, re=10.0, u_inf=0.04, centre=None):
    """Stationary circular cylinder in a channel (Sec. 3.1): Zou-He velocity
    inlet and pressure outlet, bounce-back walls in y, periodic span; the
    cylinder is an elliptic foil with equal axes.  Re = u_inf d / nu.  The
    defaults keep tau near 0.6: with BGK the Zou-He velocity inlet grows
    unstable as tau approaches 1/2 (it diverges within ~120 steps at 0.512)."""
    phys = dict(kind="plate", re=re, u_inf=u_inf, chord=d)
    bx = dict(nx=nx, ny=ny, nz=nz, bc=[ZH_VELOCITY, ZH_PRESSURE, WALL, WALL, PERIODIC, PERIODIC],
              u_in=[u_inf, 0.0, 0.0], rho_out=1.0, body_force=[0.0, 0.0, 0.0],
              u_ref=u_inf, area_ref=d * nz)
    if centre is None:
        centre = (nx / 4.0, ny / 2.0 - 0.3)   # slightly off the mid-plane: shedding starts sooner
    wg = [wing(d, d, centre, 0.5, 0.0, 1.0, ALPHA_CONST)]
    return bx, wg, phys


def figure_eight_case(nx=64, ny=64, nz=8, chord=15.0, aspect=7.5, a0_over_c=2.5,
                      beta=math.pi / 3.0, re=75.0, u_tip=0.05):
    """Hovering elliptic wing on the figure-eight stroke of Sec. 3.2: the
    centre sweeps along a stroke plane inclined at beta with amplitude A0/2
    (Eq. 20) while the wing pitches about its centre with
    alpha = pi/4 - pi/4 sin(2 pi t / T) (Eq. 21).  Closed box (walls in x
    and y), periodic span.  Re = U_tip c / nu with U_tip = pi f A0 (Eq. 22);
    the lattice tip speed u_tip fixes f, so each side maps (re, u_tip,
    chord, A0) to tau and the period itself.
    """
    a0 = a0_over_c * chord
    phys = dict(kind="figure_eight", re=re, u_tip=u_tip, chord=chord, a0=a0)
    bx = dict(nx=nx, ny=ny, nz=nz, bc=[WALL, WALL, WALL, WALL, PERIODIC, PERIODIC],
              u_in=[0.0, 0.0, 0.0], rho_out=1.0, body_force=[0.0, 0.0, 0.0],
              u_ref=u_tip, area_ref=chord * nz)
    centre = (nx / 2.0 - 0.5, ny / 2.0 - 0.5)
    wg = [wing(chord, chord / aspect, centre, 0.5, beta, 1.0, ALPHA_SIN,
               alpha_mean=math.pi / 4.0, alpha_amp=-math.pi / 4.0, period_steps=None,
               trans_amp=0.5 * a0, trans_angle=beta)]
    return bx, wg, phys


def clap_gap(chord, aspect=5.0):
    """Distance between the two chord lines at the hinges.

    The paper takes c/2, chosen so that the lattice nodes around the markers
    of one foil do not interact with the other (Sec. 3.3).  With the 4-point
    kernel that needs the facing surfaces (chord lines less one thickness)
    at least 4 cells apart; for short chords c/2 is too small, so the gap is
    max(c/2, thickness + 5).  At chord 20 and above this is c/2.
    """
    return max(0.5 * chord, chord / aspect + 5.0)


def clap_fling_case(nx=256, ny=192, nz=192, chord=20.0, aspect=5.0,
                    re=100.0, j=0.01, f=0.25):
    """Two foils hinged at their trailing edges, clap & fling.

    alpha(t) = (pi/3)|sin(2 pi t / T)|; the upper foil turns with sense -1 and
    the lower with +1 so both leading edges open outward.  Hinges at
    x = 3 nx / 8 and y = ny/2 - 1/2 +- gap/2 (mirror plane between cell
    rows), gap = clap_gap(chord).  Flow parameters are returned raw in
    `physics`; the solver maps them.
    """
    phys = dict(kind="clap_fling", re=re, j=j, f=f, chord=chord, kappa=KAPPA)
    xh = 3.0 * nx / 8.0
    ymid = ny / 2.0 - 0.5
    half = 0.5 * clap_gap(chord, aspect)
    bx = dict(nx=nx, ny=ny, nz=nz,
              bc=[VELOCITY, PRESSURE, WALL, WALL, PERIODIC, PERIODIC],
              u_in=None, rho_out=1.0, body_force=[0.0, 0.0, 0.0],
              u_ref=None, area_ref=chord * nz)
    wg = []
    for sense, yh in ((-1.0, ymid + half), (1.0, ymid - half)):
        # period_steps is left None: it follows from (f, chord) through the
        # lattice mapping, which each solver side computes itself
        wg.append(wing(chord, chord / aspect, (xh, yh), 1.0, 0.0, sense,
                       ALPHA_ABS_SIN, alpha_mean=0.0, alpha_amp=math.pi / 3.0,
                       period_steps=None, phase=0.0))
    return bx, wg, phys


def taylor_green_velocity(n, u0):
    """3D Taylor-Green initial velocity on an n^3 periodic box, k = 2 pi / n.

    u = u0 sin(kx) cos(ky) cos(kz), v = -u0 cos(kx) sin(ky) cos(kz), w = 0.
    Returns (3, n, n, n) (z, y, x order in the last three axes).
    """
    k = 2.0 * math.pi / n
    x = np.arange(n, dtype=np.float64)
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    u = np.empty((3, n, n, n))
    u[0] = u0 * np.sin(k * xx) * np.cos(k * yy) * np.cos(k * zz)
    u[1] = -u0 * np.cos(k * xx) * np.sin(k * yy) * np.cos(k * zz)
    u[2] = 0.0
    return u


def taylor_green_density(n, u0):
    """Density of the 3D Taylor-Green initial pressure field on an n^3 box:
    p - p0 = (u0^2 / 16) (cos 2kx + cos 2ky)(cos 2kz + 2) with rho0 = 1 and
    rho = 1 + 3 (p - p0) (lattice sound speed squared 1/3).  (z, y, x) order."""
    k = 2.0 * math.pi / n
    x = np.arange(n, dtype=np.float64)
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    p = (u0 * u0 / 16.0) * (np.cos(2 * k * xx) + np.cos(2 * k * yy)) * (np.cos(2 * k * zz) + 2.0)
    return 1.0 + 3.0 * p


def taylor_green_case(n=256, re=100.0, u0=0.05):
    """Fully periodic n^3 box for the Taylor-Green vortex at Re = u0 / (k nu),
    k = 2 pi / n.  Returns (box, rho0, u0 field, nu)."""
    k = 2.0 * math.pi / n
    nu = u0 / (k * re)
    bx = box(n, n, n, [PERIODIC] * 6, 3.0 * nu + 0.5)
    return bx, taylor_green_density(n, u0), taylor_green_velocity(n, u0), nu


SERVE_DOMAINS = ((64, 64, 64), (96, 80, 80), (128, 96, 96), (160, 128, 128))


def serve_requests(n=64, seed=0, arrival_seed=1, rate=None, steps=1000):
    """Seeded sweep requests: (Re, J, f) uniform over the 18 combinations and a
    domain uniform over SERVE_DOMAINS with chord = ny / 8.  Arrival times are
    Poisson with the given rate (requests per second); rate None = all at t=0.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    combos = [(r, jj, ff) for r in RE_SET for jj in J_SET for ff in F_SET]
    reqs = []
    arr = np.random.Generator(np.random.PCG64(arrival_seed))
    t = 0.0
    for i in range(n):
        re, jj, ff = combos[int(rng.integers(len(combos)))]
        nx, ny, nz = SERVE_DOMAINS[int(rng.integers(len(SERVE_DOMAINS)))]
        if rate is not None:
            t += float(arr.exponential(1.0 / rate))
        reqs.append(dict(id=i, re=re, j=jj, f=ff, nx=nx, ny=ny, nz=nz,
                         chord=ny / 8.0, steps=int(steps), arrival=t))
    return reqs
