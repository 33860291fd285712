"""Physical <-> lattice-unit conversion of the flow parameters.

Section 2.1 fixes dx = dt = 1 and a reference density of 1 in lattice units
and relates the shear relaxation rate to the kinematic viscosity,
nu_LU = (1/omega - 1/2)/3.  Section 3.1 defines Re = U h0 / nu,
Fr = U / sqrt(g h0) and We = rho U^2 h0 / sigma, and Table 1 lists dx, dt,
omega, U_LU and h0 for runs E1 and E4.
"""
from __future__ import annotations

import math


def nu_lattice(nu_phys: float, dx: float, dt: float) -> float:
    """Kinematic viscosity in lattice units: nu dt / dx^2."""
    return nu_phys * dt / (dx * dx)


def omega_from_nu(nu_lu: float) -> float:
    """Shear relaxation rate giving lattice viscosity nu_lu."""
    return 1.0 / (3.0 * nu_lu + 0.5)


def nu_from_omega(omega: float) -> float:
    return (1.0 / omega - 0.5) / 3.0


def reynolds(U_lu: float, h0_lu: float, nu_lu: float) -> float:
    return U_lu * h0_lu / nu_lu


def gravity_from_froude(U_lu: float, h0_lu: float, Fr: float) -> float:
    """Gravitational acceleration (lattice units) that gives Froude number Fr."""
    return (U_lu / Fr) ** 2 / h0_lu


def froude(U_phys: float, g_phys: float, h0_phys: float) -> float:
    return U_phys / math.sqrt(g_phys * h0_phys)


def sigma_from_weber(U_lu: float, h0_lu: float, We: float, rho: float = 1.0) -> float:
    return rho * U_lu * U_lu * h0_lu / We


def weber(rho_phys: float, U_phys: float, h0_phys: float, sigma_phys: float) -> float:
    return rho_phys * U_phys * U_phys * h0_phys / sigma_phys


def physical_velocity(U_lu: float, dx: float, dt: float) -> float:
    return U_lu * dx / dt
