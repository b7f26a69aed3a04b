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


def test_porosity_field_recipe():
    """Seeded, reproducible; mean 0.6 and standard deviation 0.15 before the
    clip to [0.3, 0.95]; spatially correlated over about sigma = 8 cells."""
    a = li.porosity_grf(512, 512, seed=1409)
    b = li.porosity_grf(512, 512, seed=1409)
    c = li.porosity_grf(512, 512, seed=1410)
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c)
    assert a.min() >= 0.3 and a.max() <= 0.95
    assert abs(a.mean() - 0.6) < 0.01 and abs(a.std() - 0.15) < 0.01
    d = a - a.mean()
    corr = lambda s: float((d[:, s:] * d[:, :-s]).mean() / d.var())  # noqa: E731
    assert corr(1) > 0.95 and corr(8) > 0.5 and corr(64) < 0.1


def test_sweep_distribution():
    """1024 annuli: grid sides uniform on {32, ..., 512}; Ra, Da and R*
    log-uniform on their ranges; phi uniform on [0.3, 0.95]; Pr from
    {0.71, 1, 7}; Ergun Forchheimer coefficient; reproducible from the seed."""
    cfgs = li.sweep(n_inst=1024, seed=1409)
    assert cfgs == li.sweep(n_inst=1024, seed=1409)
    nr = np.array([c["nr"] for c in cfgs])
    nz = np.array([c["nz"] for c in cfgs])
    sizes = set(range(32, 513, 32))
    assert set(nr) == sizes and set(nz) == sizes
    ra = np.log10([c["Ra"] for c in cfgs])
    da = np.log10([c["Da"] for c in cfgs])
    rs = np.log([(c["r0"] + c["L"]) / c["r0"] for c in cfgs])
    phi = np.array([c["phi"] for c in cfgs])
    assert 3.0 <= ra.min() and ra.max() <= 6.0 and abs(ra.mean() - 4.5) < 0.1
    assert -6.0 <= da.min() and da.max() <= -2.0 and abs(da.mean() + 4.0) < 0.15
    assert np.log(1.2) - 1e-12 <= rs.min() and rs.max() <= np.log(10.0) + 1e-12
    assert abs(rs.mean() - 0.5 * (np.log(1.2) + np.log(10.0))) < 0.05
    assert 0.3 <= phi.min() and phi.max() <= 0.95 and abs(phi.mean() - 0.625) < 0.02
    assert {c["Pr"] for c in cfgs} == {0.71, 1.0, 7.0}
    assert all(c["F_phi"] < 0 for c in cfgs)
    assert all(c["L"] == c["nr"] - 1 for c in cfgs)
