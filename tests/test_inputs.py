"""The seeded problem builders state the paper's test problems (no arithmetic
of the method): geometry and parameters as the paper gives them."""
import math

import numpy as np

import lbm_inputs as li


def test_heater_annulus_is_sec_4_4():
    c = li.heater_annulus(Da=1e-4)
    assert (c["nr"], c["nz"]) == (200, 200)
    L, H = c["L"], c["nz"] - 1
    assert L == 199 and c["r0"] == L           # R* = 2: r_i = L
    assert H / L == 1.0                        # A = 1
    heated = [k for k in range(c["nz"]) if c["flux_zlo"] <= k <= c["flux_zhi"]]
    assert heated[0] == 60 and heated[-1] == 139 and len(heated) == 80   # 0.3 H .. 0.7 H
    assert math.isclose(c["flux_rmin"] * L, 10.0)                       # q' L / k = dT = 10
    assert (c["T_rmax"], c["T_ref"], c["T_init"], c["delta_T"]) == (1.0, 1.0, 1.0, 10.0)
    assert (c["Ra"], c["Pr"], c["phi"], c["F_phi"]) == (1e7, 0.7, 0.9, 0.0)
    assert (c["therm_rmin"], c["therm_rmax"], c["therm_z"]) == ("flux", "fixed", "adiabatic")


def test_developing_pipe_is_sec_4_1():
    c = li.developing_pipe(Da=1e-2)
    assert c["nr"] == 41 and c["r0"] == 0.5 and c["L"] == 40.5   # r_i = 40.5: 81 cells across
    assert c["nz"] == 649                                          # H = A r_i = 648
    nu = (c["tau_nu"] - 0.5) / 3.0
    assert math.isclose(c["u_in"] * c["L"] / nu, 100.0)            # Re = 100 with L = r_i
    assert math.isclose(c["Ma"] * math.sqrt(1.0 / 3.0), c["u_in"])  # residual scaled by u_in
    assert (c["side_rmin"], c["side_z"], c["therm_z"]) == ("axis", "flow", "fixed")
    s = li.plug_start(c)
    assert s.shape == (3, c["nz"], c["nr"]) and np.all(s[0] == c["u_in"]) and np.all(s[1] == 0)


def test_porous_annulus_is_sec_4_3():
    for ra_star in (200.0, 500.0, 2000.0):
        c = li.porous_annulus_43(ra_star)
        assert (c["nr"], c["nz"]) == (300, 300)
        assert math.isclose(c["Ra"] * c["Da"], ra_star)            # Ra* = Ra Da
        assert math.isclose((c["r0"] + c["L"]) / c["r0"], 5.338)   # R*
        assert (c["phi"], c["Da"], c["Pr"]) == (0.3698, 1.66e-6, 1.0)
        assert c["F_phi"] < 0                                       # Ergun, Eq. (8)


def test_table2_annulus_is_sec_4_2():
    c = li.table2(1e4)
    assert (c["nr"], c["nz"]) == (100, 200)
    assert (c["phi"], c["Da"], c["Pr"]) == (1.0, 1e8, 0.7)
    assert math.isclose((c["r0"] + c["L"]) / c["r0"], 2.0)
    assert c["T_ref"] == 0.5 * (c["T_rmin"] + c["T_rmax"])
