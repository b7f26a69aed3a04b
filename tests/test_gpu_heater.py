"""GPU: isoflux heater walls, the heater Nusselt number (Eqs. 43-44) and the
stream function against the FP64 oracle, and the Sec. 4.4 problem (Table 3)."""
import numpy as np
import pytest

import lbm_inputs as li
from tests.parity import U_FLOOR, assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1409_5929_amd import lbm

    lbm._load()  # raises if the HIP library is missing: no CPU fallback
    return lbm


def _cases():
    a = li.heater_annulus(Da=1e-2, nr=48, nz=40, Ra=1e5)           # window 11.7..27.3
    b = li.heater_annulus(Da=1e-4, nr=67, nz=33, Ra=1e6, Rstar=4.0)  # ragged rows and strips
    c = li.heater_annulus(Da=1e-2, nr=30, nz=30, Ra=1e5)
    c.update(flux_zlo=-5.0, flux_zhi=100.0)                          # heater reaches the corners
    d = li.heater_annulus(Da=1e-3, nr=40, nz=36, Ra=1e5)
    d.update(therm_rmin="fixed", T_rmin=1.0, therm_rmax="flux", flux_rmax=-0.05,
             flux_zlo=3.0, flux_zhi=20.0)                            # cooling flux on the outer wall
    return [("heater 48x40", a), ("heater 67x33 R*=4", b), ("heater to corners", c),
            ("outer flux wall", d)]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
@pytest.mark.parametrize("n", [0, 1, 7, 200])
def test_heater_fields_nusselt_psi_parity(L, oracle_mod, case, n):
    name, cfg = case
    lat = L.Lattice(cfg, check_interval=0)
    lat.step(n)
    g = lat.fields()
    psi, mx = lat.stream_function()
    lat.close()
    o = oracle_mod.Oracle(cfg)
    o.step(n)
    m = o.macros()
    o.close()
    assert_parity(g, m, label=f"{name} n={n}", u_floor=U_FLOOR)
    psi_o, mx_o = oracle_mod.stream_function(m["uz"], cfg["r0"])
    # psi carries the FP32 velocity error times r: compare against max |psi|
    # with the velocity floor's share as a lower bound
    scale = max(mx_o, U_FLOOR * cfg["r0"] * cfg["nr"])
    assert np.abs(psi - psi_o).max() <= 1e-5 * scale, name
    assert abs(mx - mx_o) <= 1e-5 * scale
    # psi of the GPU fields, recomputed on the host in FP64, equals the device result
    psi_h, _ = oracle_mod.stream_function(g["uz"].astype(np.float64), cfg["r0"])
    np.testing.assert_allclose(psi, psi_h, rtol=1e-6, atol=1e-6 * max(mx, 1e-30))


def test_heater_nusselt_reduction(L, oracle_mod):
    """The heater mean of Eqs. (43)-(44) from the device check reduction."""
    for name, cfg in _cases():
        n = 100
        lat = L.Lattice(cfg, check_interval=50)
        lat.step(n + 1)
        r = lat.residual()
        lat.close()
        o = oracle_mod.Oracle(cfg)
        o.step(n)
        nui, nuo = o.nusselt()
        o.close()
        # Eq. (42) on a fixed wall: each one-sided difference (coefficient
        # magnitudes summing to 4 / 2) carries the FP32 rounding of T, so the
        # H-point integral times r_w / (H dT) is good to 4 2^-24 max|T| r_w / dT.
        tmax = max(abs(cfg["T_rmin"]), abs(cfg["T_rmax"]), abs(cfg["T_init"])) + abs(cfg["delta_T"])
        floor = 4 * 2.0 ** -24 * tmax * (cfg["r0"] + cfg["nr"] - 1) / abs(cfg["delta_T"])
        assert abs(r["nu_i"][0] - nui) <= 1e-5 * abs(nui) + floor, (name, r["nu_i"][0], nui)
        assert abs(r["nu_o"][0] - nuo) <= 1e-5 * abs(nuo) + floor, (name, r["nu_o"][0], nuo)


def test_flux_wall_validation(L):
    bad = li.heater_annulus(Da=1e-2, nr=20, nz=20)
    bad["therm_z"] = "flux"
    with pytest.raises(L.LbmError):
        L.Lattice(bad)
    bad = li.heater_annulus(Da=1e-2, nr=20, nz=20)
    bad["flux_rmin"] = float("nan")
    with pytest.raises(L.LbmError):
        L.Lattice(bad)


@pytest.mark.parametrize("Da, nu_paper, psi_paper", [(1e-4, 9.21, 5.69), (1e-2, 17.09, 16.38)])
def test_table3_heater(L, Da, nu_paper, psi_paper):
    """Sec. 4.4 / Table 3 at Ra = 1e7, Pr = 0.7, phi = 0.9 on the paper's
    200 x 200 grid, run to a residual of 1e-10: the heater Nusselt number
    within 2 % and max |psi| / (alpha L) within 3 % of the paper's values, and
    the heat leaving through the outer wall within 2 % of what the heater puts
    in.  (Da = 1e-6 takes 17 million steps; the package's study module runs it.)"""
    cfg = li.heater_annulus(Da=Da)
    lat = L.Lattice(cfg, check_interval=2000, tol=1e-10, max_steps=12_000_000)
    while lat.info()["status"] == "running":
        lat.step(1_000_000)
    r = lat.residual()
    info = lat.info()
    _, psi_max = lat.stream_function(field=False)
    lat.close()
    from paper_1409_5929_amd.studies import alpha_e

    Lg = cfg["L"]
    psi = psi_max / (alpha_e(cfg) * Lg)
    heated = sum(cfg["flux_zlo"] <= k <= cfg["flux_zhi"] for k in range(cfg["nz"]))
    balance = (cfg["r0"] + 0.5) * heated / (Lg * (cfg["nz"] - 1))
    print(f"Da={Da:g}: Nu={r['nu_i'][0]:.4f} (paper {nu_paper}) |psi|max/(alpha L)={psi:.3f} "
          f"(paper {psi_paper}) Nu_o={r['nu_o'][0]:.4f} (balance {balance:.4f}) t={info['t']}",
          flush=True)
    assert info["status"] == "converged"
    assert abs(r["nu_i"][0] - nu_paper) <= 0.02 * nu_paper
    assert abs(psi - psi_paper) <= 0.03 * psi_paper
    assert abs(r["nu_o"][0] - balance) <= 0.02 * balance


def test_stream_function_into_device_memory(L):
    """lbm_axi_stream_function with a device destination (written on the
    handle's stream) equals the host-destination result."""
    import ctypes

    import torch

    cfg = li.heater_annulus(Da=1e-2, nr=48, nz=40, Ra=1e5)
    lat = L.Lattice(cfg, check_interval=0)
    lat.step(300)
    psi_h, mx_h = lat.stream_function()
    dev = torch.empty((cfg["nz"], cfg["nr"]), dtype=torch.float32, device="cuda")
    mx = ctypes.c_double()
    rc = lat._lib.lbm_axi_stream_function(lat._h, 0, dev.data_ptr(), ctypes.byref(mx), 1)
    assert rc == 0
    lat.sync()
    np.testing.assert_array_equal(dev.cpu().numpy(), psi_h)
    assert mx.value == mx_h
    lat.close()
