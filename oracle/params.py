"""Physical parameters to lattice units (oracle; test-only).

Eq. 3: tau = 3 nu dt / dx^2 + 1/2, with dx = dt = 1.
Clap & fling (Sec. 3.3-3.4): the tip speed is U_tip = 2 Phi f c with the
maximum opening angle Phi = 120 degrees, J = U_inf / U_tip (Eq. 24) and
Re = U_tip c / nu (Eq. 22 with the clap & fling tip speed).  The paper quotes
f in Hz with no time unit for the lattice; the reading taken here is a
lattice tip speed U_tip = kappa f (kappa = 0.2 by default), so the period is
T = 2 Phi c / U_tip steps.  At fixed Re and J the continuum problem does not
depend on f; in the lattice f then sets the Mach number and tau, as in the
paper, where frequency is varied at fixed Re by changing the viscosity.
"""
from __future__ import annotations

import math

PHI_OPEN = 2.0 * math.pi / 3.0


def tau_from_nu(nu):
    """Eq. 3 in lattice units."""
    return 3.0 * nu + 0.5


def clap_fling(re, j, f, chord, kappa=0.2):
    u_tip = kappa * f
    nu = u_tip * chord / re
    return dict(u_tip=u_tip, nu=nu, tau=tau_from_nu(nu), u_inf=j * u_tip,
                period_steps=2.0 * PHI_OPEN * chord / u_tip)


def plate(re, u_inf, chord):
    """Fixed plate: Re = U_inf c / nu."""
    nu = u_inf * chord / re
    return dict(nu=nu, tau=tau_from_nu(nu))


def figure_eight(re, u_tip, chord, a0):
    """Figure-eight hovering (Sec. 3.2): Re = U_tip c / nu with the maximum
    centre speed U_tip = pi f A0 (Eq. 22), so the period is T = 1/f =
    pi A0 / U_tip steps."""
    nu = u_tip * chord / re
    return dict(nu=nu, tau=tau_from_nu(nu), period_steps=math.pi * a0 / u_tip)


def complete_case(bx, wings, phys):
    """Fill tau, inlet velocity, reference velocity and wing periods from the
    raw physics of a workload description.  Returns new (box, wings)."""
    bx = dict(bx)
    wings = [dict(w) for w in wings]
    if phys["kind"] == "plate":
        p = plate(phys["re"], phys["u_inf"], phys["chord"])
        bx["tau"] = p["tau"]
        for w in wings:
            if w.get("period_steps") is None:
                w["period_steps"] = 1.0
    elif phys["kind"] == "clap_fling":
        p = clap_fling(phys["re"], phys["j"], phys["f"], phys["chord"], phys.get("kappa", 0.2))
        bx["tau"] = p["tau"]
        bx["u_in"] = [p["u_inf"], 0.0, 0.0]
        bx["u_ref"] = p["u_tip"]
        for w in wings:
            w["period_steps"] = p["period_steps"]
    elif phys["kind"] == "figure_eight":
        p = figure_eight(phys["re"], phys["u_tip"], phys["chord"], phys["a0"])
        bx["tau"] = p["tau"]
        bx["u_ref"] = phys["u_tip"]
        for w in wings:
            w["period_steps"] = p["period_steps"]
    else:
        raise ValueError(phys["kind"])
    return bx, wings
