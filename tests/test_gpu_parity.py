"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Every test builds its inputs with the seeded generators of ``lbm_inputs``,
runs the same number of steps in both implementations and compares the
macroscopic fields node by node (u = (u_z, u_r) as one vector, p, T:
relative L2 <= 1e-5 for FP32; node classes bit-exact).
"""
import numpy as np
import pytest

import lbm_inputs as li
from tests.parity import TOL_FP32, U_FLOOR, assert_parity, rel_errors, window

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1409_5929_amd import lbm

    lbm._load()  # raises if the HIP library is missing: no CPU fallback
    return lbm


def gpu_fields(L, cfg, n, phi=None, init=None, **kw):
    lat = L.Lattice(cfg, phi=phi, init=init, **kw)
    lat.step(n)
    out = lat.fields()
    lat.close()
    return out


def orc_fields(oracle_mod, cfg, n, phi=None, init=None):
    o = oracle_mod.Oracle(cfg, phi_field=phi, init=init)
    o.step(n)
    return o.macros()


@pytest.mark.parametrize("F_phi", [li.ERGUN, 0.0])
def test_pipe_config1(L, oracle_mod, F_phi):
    cfg = li.pipe(nr=64, nz=8, F_phi=F_phi)
    n = 500
    assert_parity(gpu_fields(L, cfg, n), orc_fields(oracle_mod, cfg, n), label=f"pipe F={F_phi}")


def test_annulus_config2(L, oracle_mod):
    cfg = li.annulus(nr=256, nz=256, Ra=1e5, Da=1e-4)
    n = 200
    assert_parity(gpu_fields(L, cfg, n), orc_fields(oracle_mod, cfg, n), label="annulus 256^2")


def test_variable_porosity_512(L, oracle_mod):
    cfg, _ = li.variable_porosity_annulus(n=512, Ra=1e6, Da=1e-3)
    phi = li.porosity_grf(512, 512, seed=1409)
    n = 100
    assert_parity(gpu_fields(L, cfg, n, phi=phi), orc_fields(oracle_mod, cfg, n, phi=phi),
                  label="variable porosity 512^2")


def _cases():
    rng = np.random.default_rng(11)
    out = []
    out.append(("tiny 3x3", li.annulus(nr=3, nz=3, Ra=1e4, Da=1e-2), None, None))
    out.append(("ragged 65x17", li.annulus(nr=65, nz=17, Ra=1e5, Da=1e-3, Rstar=3.0), None, None))
    out.append(("ragged 130x33 field", li.annulus(nr=130, nz=33, Ra=1e5, Da=1e-3),
                li.porosity_grf(33, 130, seed=3, sigma=3.0), None))
    c = li.annulus(nr=40, nz=24, Ra=1e5, Da=1e-2, F_phi=0.3)
    c.update(src_printed=1, therm_z="fixed", T_zmin=0.2, T_zmax=0.8)
    out.append(("printed source, fixed z", c, None, None))
    c = dict(nr=70, nz=10, r0=400.0, L=10.0, side_rmin="periodic", side_rmax="periodic",
             side_z="periodic", phi=0.6, Da=1e-2, F_phi=-1.0, tau_nu=1.0, Pr=1.0, accel_z=1e-5,
             T_rmin=1.0, T_rmax=0.0, T_ref=0.5)
    init = np.stack([rng.normal(0, 0.01, (10, 70)), rng.normal(0, 0.01, (10, 70)),
                     rng.uniform(0, 1, (10, 70))])
    out.append(("periodic r and z, start fields", c, None, init))
    c = li.annulus(nr=33, nz=20, Ra=1e5, Da=1e-2, Rstar=10.0, phi=0.9)
    init = np.stack([rng.normal(0, 0.01, (20, 33)), rng.normal(0, 0.01, (20, 33)),
                     rng.uniform(0, 1, (20, 33))])
    out.append(("small r (R*=10), start fields", c, None, init))
    out.append(("pipe ragged 97x5", li.pipe(nr=97, nz=5), None, None))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
@pytest.mark.parametrize("n", [0, 1, 2, 7])
def test_edge_cases_each_parity(L, oracle_mod, case, n):
    name, cfg, phi, init = case
    assert_parity(gpu_fields(L, cfg, n, phi=phi, init=init),
                  orc_fields(oracle_mod, cfg, n, phi=phi, init=init), label=f"{name} n={n}",
                  u_floor=U_FLOOR)


def test_residual_and_nusselt_reductions(L, oracle_mod):
    """FP64 residual and Eq. (42) Nusselt numbers at a check step."""
    cfg = li.annulus(nr=64, nz=48, Ra=1e5, Da=1e-2)
    n = 100
    lat = L.Lattice(cfg, check_interval=50)
    lat.step(n + 1)  # the check at level n runs inside the step from n to n + 1
    r = lat.residual()
    info = lat.info()
    lat.close()
    o = oracle_mod.Oracle(cfg)
    o.step(n - 50)
    o.snapshot()
    o.step(50)
    ro = o.residual()
    nui, nuo = o.nusselt()
    assert info["t_check"] == n
    assert abs(r["res"][0] - ro["res"]) <= 1e-3 * ro["res"]
    assert abs(r["nu_i"][0] - nui) <= 1e-5 * abs(nui)
    assert abs(r["nu_o"][0] - nuo) <= 1e-5 * abs(nuo) + 1e-9


def test_batched_instances_match_single_runs(L, oracle_mod):
    cfgs = [li.annulus(nr=96, nz=40, Ra=1e5, Da=1e-3),
            li.annulus(nr=33, nz=130, Ra=1e4, Da=1e-5, Rstar=5.0, Pr=7.0),
            li.annulus(nr=64, nz=64, Ra=1e6, Da=1e-2, phi=0.4, Rstar=1.3)]
    n = 30
    lat = L.Lattice(cfgs, check_interval=10)
    lat.step(n)
    batched = [lat.fields(i) for i in range(3)]
    lat.close()
    for i, c in enumerate(cfgs):
        single = gpu_fields(L, c, n, check_interval=10)
        for k in ("uz", "ur", "p", "T", "mask", "drho"):
            np.testing.assert_array_equal(batched[i][k], single[k])
    assert_parity(batched[1], orc_fields(oracle_mod, cfgs[1], n), label="batched instance 1")


def test_run_states(L):
    """Converged instances stop; a NaN start is reported as diverged."""
    cond = li.annulus(nr=17, nz=6, Rstar=2.0, phi=1.0, Da=1e8, Ra=0.0, Pr=0.5, F_phi=0.0)
    cond["tau_nu"] = 0.8
    nan_init = np.zeros((3, 8, 9), np.float32)
    nan_init[2, 4, 4] = np.nan
    bad = li.annulus(nr=9, nz=8, Ra=1e4, Da=1e-2)
    lat = L.Lattice([cond, bad], init=[None, nan_init], check_interval=100, tol=1e-7,
                    max_steps=10**6)
    for _ in range(100):
        lat.step(5000)
        if lat.info(0)["status"] != "running":
            break
    st = lat.residual()
    assert lat.info(0)["status"] == "converged" and st["res"][0] <= 1e-7
    t_stop = lat.info(0)["t"]
    lat.step(1000)
    assert lat.info(0)["t"] == t_stop
    assert lat.info(1)["status"] == "diverged"
    lat.close()


def test_stalled_at_max_steps(L):
    cfg = li.annulus(nr=20, nz=20, Ra=1e5, Da=1e-2)
    lat = L.Lattice(cfg, check_interval=100, tol=1e-12, max_steps=300)
    lat.step(1000)
    assert lat.info()["status"] == "stalled"
    assert lat.info()["t"] == 301  # the check at step 300 runs in the step from 300 to 301
    lat.close()


def test_device_fields_equal_host_fields(L):
    import torch

    cfg = li.annulus(nr=50, nz=30, Ra=1e5, Da=1e-3)
    lat = L.Lattice(cfg)
    lat.step(9)
    host = lat.fields()
    dev = lat.fields_device()
    torch.cuda.synchronize()
    for k in ("uz", "ur", "p", "T"):
        np.testing.assert_array_equal(dev[k].cpu().numpy(), host[k])
    lat.set_timing(True)
    lat.step(10)
    ms, launches = lat.kernel_time()
    assert launches == 10 and ms > 0
    lat.close()


@pytest.mark.parametrize("own_stream", [False, True])
def test_device_fields_from_a_handle_on_another_stream(L, own_stream):
    """A handle on a stream other than torch's current one (a torch side
    stream, or the library's own when given the null stream): the device
    fields are read on torch's stream with no synchronisation by the caller."""
    import torch

    cfg = li.annulus(nr=300, nz=200, Ra=1e5, Da=1e-3)
    side = torch.cuda.Stream()
    lat = L.Lattice(cfg, stream=0 if own_stream else side.cuda_stream)
    lat.step(41)
    dev = lat.fields_device()
    got = {k: dev[k].cpu().numpy() for k in ("uz", "ur", "p", "T")}
    host = lat.fields()
    lat.close()
    for k in ("uz", "ur", "p", "T"):
        np.testing.assert_array_equal(got[k], host[k])


@pytest.mark.parametrize("Ra, nu_paper", [(1e3, 1.710), (1e4, 3.211), (1e5, 5.768)])
def test_table2_mean_nusselt(L, Ra, nu_paper):
    """Sec. 4.2 / Table 2: annulus without porous medium, 100 x 200 grid,
    steady mean Nusselt number on the inner wall within 2 % of the paper."""
    cfg = li.table2(Ra)
    lat = L.Lattice(cfg, check_interval=1000, tol=1e-8, max_steps=800_000)
    while lat.info()["status"] == "running":
        lat.step(50_000)
    r = lat.residual()
    info = lat.info()
    lat.close()
    print(f"Ra={Ra:g}: Nu_i={r['nu_i'][0]:.4f} Nu_o={r['nu_o'][0]:.4f} paper {nu_paper} "
          f"status={info['status']} t={info['t']} res={r['res'][0]:.2e}", flush=True)
    assert info["status"] == "converged"
    assert abs(r["nu_i"][0] - nu_paper) <= 0.02 * nu_paper
    assert abs(r["nu_i"][0] - r["nu_o"][0]) <= 0.02 * nu_paper


def _window(cfg, phi, j0, k0, w):
    """Sub-problem of a larger one: a w x w window whose sides are the real
    walls where it touches them and walls (contaminating only a margin)
    elsewhere."""
    c = dict(cfg)
    nr = cfg["nr"]
    c.update(nr=w, nz=w, r0=cfg["r0"] + j0)
    if j0 > 0:
        c.update(side_rmin="wall", therm_rmin="adiabatic")
    if j0 + w < nr:
        c.update(side_rmax="wall", therm_rmax="adiabatic")
    return c, phi[k0:k0 + w, j0:j0 + w]


def test_full_size_sampled_windows(L, oracle_mod):
    """8192^2 throughput problem in the benchmark's launch configuration: after
    n steps every node farther than n + 2 from a window's artificial sides
    depends only on the window, so the oracle run on the window gives it
    exactly.  Node classes are checked over the whole grid."""
    size, n, w = 8192, 4, 28
    cfg, _ = li.variable_porosity_annulus(n=size)
    phi = li.porosity_grf(size, size, seed=1409)
    lat = L.Lattice(cfg, phi=phi, check_interval=100)
    lat.step(n)
    g = lat.fields()
    lat.close()
    m = g["mask"]
    assert (m[1:-1, 1:-1] == 0).all()
    assert (m[1:-1, 0] == 1).all() and (m[1:-1, -1] == 2).all()
    assert (m[0, 1:-1] == 4).all() and (m[-1, 1:-1] == 8).all()
    assert m[0, 0] == 5 and m[0, -1] == 6 and m[-1, 0] == 9 and m[-1, -1] == 10
    margin = n + 2
    spots = [(0, 0), (0, size // 2), (size - w, size - w), (size // 3, 0),
             (size // 2, size // 2), (size - w, 1234), (4000, size - w)]
    worst = 0.0
    for j0, k0 in spots:
        c, ph = _window(cfg, phi, j0, k0, w)
        c["side_z"] = "wall"
        o = orc_fields(oracle_mod, c, n, phi=ph)
        jl = 0 if j0 == 0 else margin
        jh = w if j0 + w == size else w - margin
        kl = 0 if k0 == 0 else margin
        kh = w if k0 + w == size else w - margin
        sub = window(g, slice(k0 + kl, k0 + kh), slice(j0 + jl, j0 + jh))
        ref = window(o, slice(kl, kh), slice(jl, jh))
        np.testing.assert_array_equal(sub["mask"], ref["mask"])
        e = rel_errors(sub, ref)
        worst = max(worst, *e.values())
        assert max(e.values()) <= TOL_FP32, (j0, k0, e)
    print(f"8192^2 windows: worst rel L2 {worst:.2e}", flush=True)


@pytest.mark.parametrize("ra_star", [200.0, 2000.0])
def test_porous_annulus_sec43_parity(L, oracle_mod, ra_star):
    """Sec. 4.3 parameters (R* = 5.338, phi = 0.3698, Da = 1.66e-6, Ergun F_phi,
    Ra* = Ra Da) on a ragged 75 x 70 grid: fields after 300 steps."""
    cfg = li.porous_annulus_43(ra_star, nr=75, nz=70)
    assert_parity(gpu_fields(L, cfg, 300), orc_fields(oracle_mod, cfg, 300),
                  label=f"sec. 4.3 Ra*={ra_star:g}", u_floor=U_FLOOR)
