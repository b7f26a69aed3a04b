"""Pins of the oracle's isoflux wall, heater Nusselt number and stream function
(Sec. 4.4, Eqs. 43-44, Table 3) against closed forms and conservation.

- Radial conduction from an isoflux inner wall to a fixed-temperature outer
  wall has the closed form T = T_o + (q'/k) r_i ln(r_o / r); the heater
  Nusselt number is then (R* - 1) / ln R* and the outer-wall one r_i / L.  The
  wall rule imposes the flux across the half-way face r_i + 1/2, so the
  oracle's error is first order, (r_i + 1/2) / r_i - 1: it must be at most
  that and halve when the grid is refined.
- With a partial heater and no flow, the heat leaving through the outer wall
  must match the heat put in, up to a first-order wall error that halves with
  the grid.
- The stream function integrates r u_z dr by the trapezoid rule, which is
  exact when r u_z is linear in r.
"""
import math

import numpy as np
import pytest

import lbm_inputs as li


def _conduction(oracle_mod, scale):
    nr = 20 * scale + 1
    L = nr - 1.0
    ri = 2.0 * L  # R* = 1.5
    q = 0.1 / scale
    cfg = dict(nr=nr, nz=4, r0=ri, L=L, side_rmin="wall", side_rmax="wall", side_z="periodic",
               therm_rmin="flux", therm_rmax="fixed", therm_z="adiabatic", T_rmax=1.0,
               T_ref=1.0, T_init=1.0, delta_T=q * L, flux_rmin=q, Ra=0.0, tau_nu=0.8, Pr=1.0,
               phi=1.0, Da=1e8)
    r = ri + np.arange(nr)
    exact = 1.0 + q * ri * np.log((ri + L) / r)
    init = np.zeros((3, 4, nr))
    init[2] = exact
    o = oracle_mod.Oracle(cfg, init=init)
    alpha = 0.2 * o.derived()["tau_T"]
    o.step(int(10 * 0.405 * L * L / alpha))  # ten decay times of the slowest mode
    T = o.macros()["T"]
    nu_i, nu_o = o.nusselt()
    o.close()
    return dict(err=np.abs(T - exact[None, :]).max() / (exact[0] - 1.0), ri=ri, L=L, nu_i=nu_i,
                nu_o=nu_o, spread=np.ptp(T, axis=0).max())


def test_isoflux_conduction_closed_form(oracle_mod):
    a, b = _conduction(oracle_mod, 1), _conduction(oracle_mod, 2)
    for c in (a, b):
        first_order = 0.5 / c["ri"]
        assert c["err"] <= 1.05 * first_order, c
        assert c["spread"] <= 1e-12  # uniform along z
        nu_exact = c["L"] / (c["ri"] * math.log(1.5))  # (R* - 1) / ln R*
        assert abs(c["nu_i"] - nu_exact) <= 1.05 * first_order * nu_exact, c
        assert abs(c["nu_o"] - c["ri"] / c["L"]) <= 1.05 * first_order * c["ri"] / c["L"], c
    assert 0.45 <= b["err"] / a["err"] <= 0.55


def test_heater_window_wall_rule(oracle_mod):
    """Heated wall nodes sit q'/k above their fluid neighbour, the rest of the
    inner wall copies it, and the window is {k : z_lo <= k <= z_hi}."""
    cfg = li.heater_annulus(Da=1e-2, nr=24, nz=32, Ra=1e5)  # window 9.3 <= z <= 21.7
    o = oracle_mod.Oracle(cfg)
    o.step(300)
    T = o.macros()["T"]
    o.close()
    q = cfg["flux_rmin"]
    heated = np.array([cfg["flux_zlo"] <= k <= cfg["flux_zhi"] for k in range(32)])
    assert heated.sum() == 12 and heated[10] and not heated[9] and heated[21] and not heated[22]
    d = T[:, 0] - T[:, 1]
    np.testing.assert_allclose(d[1:-1][heated[1:-1]], q, rtol=0, atol=1e-12)
    np.testing.assert_allclose(d[1:-1][~heated[1:-1]], 0.0, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(T[:, -1], cfg["T_rmax"])  # outer wall held


def test_zero_flux_is_adiabatic(oracle_mod):
    a = li.heater_annulus(Da=1e-3, nr=20, nz=16, Ra=1e5)
    a.update(therm_rmin="flux", flux_rmin=0.0, therm_rmax="fixed", T_rmax=0.0, delta_T=1.0)
    b = dict(a, therm_rmin="adiabatic")
    init = np.zeros((3, 16, 20))
    init[2] = np.random.default_rng(5).uniform(0, 1, (16, 20))
    out = []
    for c in (a, b):
        o = oracle_mod.Oracle(c, init=init)
        o.step(50)
        out.append(o.macros())
        o.close()
    for k in ("uz", "ur", "p", "T"):
        np.testing.assert_array_equal(out[0][k], out[1][k])


def _balance(oracle_mod, n):
    cfg = li.heater_annulus(Da=1e8, nr=n, nz=n, Ra=0.0, phi=1.0, Pr=1.0)
    cfg["tau_nu"] = 0.8
    o = oracle_mod.Oracle(cfg)
    L = n - 1.0
    o.step(int(6 * 0.405 * L * L / (0.2 * o.derived()["tau_T"])))
    nu_o = o.nusselt()[1]
    o.close()
    heated = sum(cfg["flux_zlo"] <= k <= cfg["flux_zhi"] for k in range(n))
    # Heat in over the half-way face: 2 pi (r_i + 1/2) q' per heated node; out:
    # Eq. (42) on the outer wall, nu_o = r_o int(-dT/dr) dz / (H dT), dT = q' L / k.
    expect = (cfg["r0"] + 0.5) * heated / (L * L)
    return nu_o / expect - 1.0


def test_heater_energy_balance_converges(oracle_mod):
    e21, e41 = _balance(oracle_mod, 21), _balance(oracle_mod, 41)
    assert 0.0 < e21 <= 0.06 and 0.0 < e41 <= 0.03
    assert 0.4 <= e41 / e21 <= 0.6


def test_stream_function_linear_integrand_exact(oracle_mod):
    rng = np.random.default_rng(7)
    nz, nr, r0 = 5, 37, 12.5
    r = r0 + np.arange(nr)
    a, b = rng.normal(size=(nz, 1)), rng.normal(size=(nz, 1))
    uz = a + b / r[None, :]
    psi, mx = oracle_mod.stream_function(uz, r0)
    exact = a * (r * r - r0 * r0)[None, :] / 2.0 + b * (r - r0)[None, :]
    np.testing.assert_allclose(psi, exact, rtol=1e-12, atol=1e-12)
    assert mx == pytest.approx(np.abs(exact).max(), rel=1e-12)
    assert np.all(psi[:, 0] == 0.0)


def test_stream_function_from_the_axis_exact(oracle_mod):
    """In a pipe psi vanishes on the axis r = 0, half a row below row 0: plug
    flow u_z = a has psi = a r^2 / 2, which the trapezoid rule (r u_z linear)
    gives exactly, row 0 included."""
    rng = np.random.default_rng(8)
    nz, nr = 4, 29
    r = 0.5 + np.arange(nr)
    a = rng.normal(size=(nz, 1))
    psi, mx = oracle_mod.stream_function(np.broadcast_to(a, (nz, nr)), 0.5, axis=True)
    exact = a * (r * r)[None, :] / 2.0
    np.testing.assert_allclose(psi, exact, rtol=1e-13, atol=1e-15)
    assert mx == pytest.approx(np.abs(exact).max(), rel=1e-13)


def test_stream_function_closes_on_outer_wall(oracle_mod):
    """Steady convection carries no net mass through a horizontal section, so
    psi returns to about zero on the outer wall (trapezoid and wall errors)."""
    cfg = li.heater_annulus(Da=1e-2, nr=21, nz=21, Ra=1e4)
    o = oracle_mod.Oracle(cfg)
    o.step(int(3 * 400 / (o.derived()["nu"] / 0.7)))
    uz = o.macros()["uz"]
    o.close()
    psi, mx = oracle_mod.stream_function(uz, cfg["r0"])
    assert mx > 0.1
    assert np.abs(psi[:, -1]).max() <= 0.05 * mx
    # heated fluid rises along the inner wall, so the upward flux inside radius r
    # (psi) is positive at mid-height and mid-gap
    assert psi[10, 10] > 0
