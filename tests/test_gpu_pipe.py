"""GPU: inlet/outlet columns (Sec. 4.1), the axis with axial boundaries, and
the pipe Nusselt number (Eqs. 40-41) against the FP64 oracle; steady states
against the oracle's committed run and against Table 1."""
import numpy as np
import pytest

import lbm_inputs as li
from tests.parity import U_FLOOR, assert_parity, tol_fp32
from tests.test_oracle_pipe import read_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1409_5929_amd import lbm

    lbm._load()  # raises if the HIP library is missing: no CPU fallback
    return lbm


def _cylinder():
    """Closed vertical cylinder heated from below (axis, wall, axial walls)."""
    return dict(nr=24, nz=30, r0=0.5, L=23.5, side_rmin="axis", side_rmax="wall", side_z="wall",
                therm_rmin="adiabatic", therm_rmax="adiabatic", therm_z="fixed", T_zmin=1.0,
                T_zmax=0.0, T_ref=0.5, T_init=0.5, delta_T=1.0, phi=0.8, Da=1e-2, F_phi=li.ERGUN,
                Ra=1e5, Pr=0.7, Ma=0.1)


def _cases():
    a = li.developing_pipe(Da=1e8, nr=21, A=2.0, u_in=0.02)
    b = li.developing_pipe(Da=1e-2, nr=19, A=3.0, u_in=0.01, F_phi=li.ERGUN, phi=0.7, T_in=0.3)
    bphi = li.porosity_grf(b["nz"], b["nr"], seed=21, sigma=3.0)
    c = li.developing_pipe(Da=1e-3, nr=13, A=4.0, u_in=0.01)
    c.update(therm_rmax="flux", flux_rmax=0.02, therm_z="fixed")  # uniform heat flux wall
    return [("clear pipe 21x42", a, None), ("porous pipe, field, Ergun", b, bphi),
            ("flux-heated pipe", c, None), ("closed cylinder", _cylinder(), None)]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
@pytest.mark.parametrize("n", [0, 1, 2, 7, 200])
def test_pipe_fields_parity(L, oracle_mod, case, n):
    name, cfg, phi = case
    init = li.plug_start(cfg) if cfg.get("side_z") == "flow" else None
    lat = L.Lattice(cfg, phi=phi, init=init, check_interval=0)
    lat.step(n)
    g = lat.fields()
    # a closed cylinder carries no net axial flux: only the area mean is defined
    weights = [True] if cfg["side_z"] != "flow" else [False, True]
    gpu_nu = [lat.pipe_nusselt(area=a) for a in weights]
    gpu_psi, gpu_mx = lat.stream_function()
    lat.close()
    o = oracle_mod.Oracle(cfg, phi_field=phi, init=init)
    o.step(n)
    m = o.macros()
    orc_nu = [o.pipe_nusselt(area=a) for a in weights]
    o.close()
    assert_parity(g, m, tol=tol_fp32(n), label=f"{name} n={n}", u_floor=U_FLOOR)
    # stream function from the axis
    psi_o, mx_o = oracle_mod.stream_function(m["uz"], cfg["r0"], axis=True)
    scale = max(mx_o, U_FLOOR * cfg["nr"] ** 2)
    assert np.abs(gpu_psi - psi_o).max() <= 1e-5 * scale, name
    assert abs(gpu_mx - mx_o) <= 1e-5 * scale
    for (nu_g, tb_g), (nu_o, tb_o) in zip(gpu_nu, orc_nu):
        # T_b is a weighted mean of T: the FP32 rounding of T and u bounds its error
        assert np.abs(tb_g - tb_o).max() <= 1e-5 * max(1.0, np.abs(tb_o).max())
        ok = np.isfinite(nu_o) & (np.abs(m["T"][:, -1] - tb_o) > 1e-3)
        np.testing.assert_allclose(nu_g[ok], nu_o[ok], rtol=1e-3, atol=1e-4)


def test_pipe_nusselt_refuses_an_annulus(L):
    lat = L.Lattice(li.annulus(nr=16, nz=16), check_interval=0)
    with pytest.raises(L.LbmError):
        lat.pipe_nusselt()
    lat.close()


def test_quarter_and_half_resolution_pipes_match_oracle_golden(L):
    """The committed oracle runs (clear pipe and Da = 1e-2 at r_i = 10.5 and
    20.5, Re = 25, each to a residual of 1e-10): the GPU, run for the same
    number of steps from the same start, gives the same local Nu along the pipe."""
    from tests.golden.make_pipe_golden import config

    g = read_golden()
    keys = sorted(g)
    cfgs = [config(da, nr) for nr, da in keys]
    lat = L.Lattice(cfgs, init=[li.plug_start(c) for c in cfgs], check_interval=0)
    done = 0
    for i in sorted(range(len(keys)), key=lambda i: g[keys[i]]["steps"]):
        # instances advance together: read each one when it reaches its step count
        n = g[keys[i]]["steps"] - done
        if n > 0:
            lat.step(n)
            done += n
        nu, _ = lat.pipe_nusselt(i)
        ref = g[keys[i]]["nu"]
        sl = slice(2, ref.size - 2)
        err = np.abs(nu[sl] - ref[sl]).max() / np.abs(ref[sl]).max()
        print(f"nr={keys[i][0]} Da={keys[i][1]:g}: steps {done}, max rel diff of Nu {err:.2e}", flush=True)
        assert err <= 2e-3
    lat.close()


def test_table1_fully_developed_nusselt(L):
    """Sec. 4.1 / Table 1 at the paper's grid spacing (r_i = 40.5), Re = 100 and
    Pr = 0.7 in a pipe long enough to develop (A = 32): Nu at z = 0.9 H within
    3 % of the paper's values for every Darcy number."""
    from paper_1409_5929_amd.studies import TABLE1, table1

    for o in table1(A=32.0, log=lambda s: print(s, flush=True)):
        paper = TABLE1[o["Da"]][0]
        assert abs(o["nu"] - paper) <= 0.03 * paper, o
