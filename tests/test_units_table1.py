"""Unit conversion against the values printed in Table 1 (Section 3.1).

Inputs: dx, dt, U_LU, h0/d50 from Table 1 and d50_LU = 11.6, nu = 1e-6 m^2/s,
sigma = 7.2e-2 kg/s^2 from Section 3.1 (fixture tests/golden/table1.json).
Printed outputs reproduced: omega (three decimals) and Re (two significant
figures) for both runs, Fr of E4 (three significant figures) and We of E1
(within 1 %).  E1's printed Fr is not reproduced by its other entries
(1.246 vs 1.31) and E4's We only to 2.5 %, so those two are not asserted.
"""
import json
import math
import os

from paper_2301_10674_amd import units

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))


def derived(run):
    r = GOLD["runs"][run]
    nu_lu = units.nu_lattice(GOLD["nu_water"], r["dx"], r["dt"])
    h0_lu = r["h0_over_d50"] * GOLD["d50_lu"]
    U = units.physical_velocity(r["U_lu"], r["dx"], r["dt"])
    h0 = h0_lu * r["dx"]
    return dict(
        omega=units.omega_from_nu(nu_lu),
        Re=units.reynolds(r["U_lu"], h0_lu, nu_lu),
        Fr=units.froude(U, GOLD["g"], h0),
        We=units.weber(GOLD["rho_water"], U, h0, GOLD["sigma_water"]),
    )


def sig(x, n):
    return round(x, -int(math.floor(math.log10(abs(x)))) + (n - 1))


def test_omega_and_reynolds():
    for run in ("E1", "E4"):
        d = derived(run)
        r = GOLD["runs"][run]
        assert round(d["omega"], 3) == r["omega"]
        assert sig(d["Re"], 2) == r["Re"]


def test_froude_e4_and_weber_e1():
    assert sig(derived("E4")["Fr"], 3) == GOLD["runs"]["E4"]["Fr"]
    assert abs(derived("E1")["We"] / GOLD["runs"]["E1"]["We"] - 1) < 0.01


def test_omega_viscosity_roundtrip():
    for om in (0.7, 1.0, 1.9, 1.997):
        assert abs(units.omega_from_nu(units.nu_from_omega(om)) - om) < 1e-14
