"""Shifted 16-bit population storage (FP16, BF16; all arithmetic in FP32)
against the FP64 oracle, and the in-place storage conversion.

Tolerances follow from the storage formats.  A stored slot is a deviation
from the quiescent state, rounded stochastically (unbiased) with unit
roundoff u16 = 2^-11 (FP16) or 2^-8 (BF16) relative to that deviation; the
resting temperature population stays in FP32.  The macroscopic fields are
sums of 5-9 such slots and the errors of successive steps are independent and
damped by the collision, so the field error stays within a few u16: the
bound used is 6 u16 (FP16 2.9e-3, BF16 2.3e-2) in relative L2.
"""
import os

import numpy as np
import pytest

import lbm_inputs as li
from tests.parity import RHO_FLOOR_16, rel_errors, tol_fp32, window

pytestmark = pytest.mark.gpu

U16 = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_nu_oracle.txt")


@pytest.fixture(scope="module")
def L():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1409_5929_amd import lbm

    lbm._load()
    return lbm


def golden_nu():
    """Steady Nu_i, Nu_o of the Table 2 annulus from the FP64 oracle."""
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        ra, _, _, nui, nuo = line.split()
        out[float(ra)] = (float(nui), float(nuo))
    return out


# The throughput problem's precision study: the same recipe (variable
# porosity, Ra = 1e6, Da = 1e-3) at 512^2, 2000 steps from the cold start,
# in FP32 and in shifted FP16 / BF16 storage, each against the FP64 oracle:
# per field and for the inner-wall Nusselt number (Eq. 42) at step 2000.
STUDY_N, STUDY_STEPS = 512, 2000


@pytest.fixture(scope="module")
def study_oracle(oracle_mod):
    cfg, _ = li.variable_porosity_annulus(n=STUDY_N, Ra=1e6, Da=1e-3)
    phi = li.porosity_grf(STUDY_N, STUDY_N, seed=1409)
    o = oracle_mod.Oracle(cfg, phi_field=phi)
    o.step(STUDY_STEPS)
    m = o.macros()
    nu_i, nu_o = o.nusselt()
    o.close()
    return cfg, phi, m, nu_i, nu_o


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_precision_study_512_2000_steps(L, study_oracle, storage):
    """Fields after 2000 steps: FP32 within 1e-5 sqrt(n / 100) = 4.5e-5 relative
    L2 of the oracle (the rounding of FP32 storage accumulates over the
    transient; 1e-5 holds at 100 steps, test_variable_porosity_512), the 16-bit
    storages within 6 u16 (temperature error against the temperature
    difference); Nu_i at step 2000 within 1e-5 (FP32), 1e-3 (FP16) and 6 u16
    (BF16) of the oracle's."""
    cfg, phi, m, nu_i, nu_o = study_oracle
    lat = L.Lattice(cfg, phi=phi, storage=storage, check_interval=STUDY_STEPS // 2)
    lat.step(STUDY_STEPS)
    g = lat.fields()
    lat.step(1)  # the check at level 2000 runs in the step from 2000 to 2001
    r = lat.residual()
    t_check = lat.info()["t_check"]
    lat.close()
    assert t_check == STUDY_STEPS
    np.testing.assert_array_equal(g["mask"], m["mask"])
    if storage == "fp32":
        e = rel_errors(g, m)
    else:
        e = rel_errors(g, m, t_floor=cfg["delta_T"], rho_floor=RHO_FLOOR_16)
    e_nu = abs(r["nu_i"][0] - nu_i) / abs(nu_i)
    tol = tol_fp32(STUDY_STEPS) if storage == "fp32" else 6 * U16[storage]
    tol_nu = {"fp32": 1e-5, "fp16": 1e-3, "bf16": 6 * U16["bf16"]}[storage]
    print(f"{storage} {STUDY_N}^2 n={STUDY_STEPS}: rel L2 u {e['u']:.2e} rho-rho_bar {e['rho']:.2e} "
          f"T-T_bar {e['T']:.2e} p {e['p']:.2e}; Nu_i {r['nu_i'][0]:.6f} vs {nu_i:.6f} "
          f"(rel {e_nu:.2e}); Nu_o {r['nu_o'][0]:.6f} vs {nu_o:.6f} (tol {tol:.1e}, Nu {tol_nu:.1e})",
          flush=True)
    for k, v in e.items():
        assert v <= tol, (storage, k, v)
    assert e_nu <= tol_nu, (storage, e_nu)


@pytest.mark.parametrize("Ra,steps", [(1e3, 150_000), (1e4, 250_000)])
def test_fp16_steady_nusselt_within_1e3(L, Ra, steps):
    """Table 2 annulus in FP16 storage: the wall Nusselt numbers, averaged
    over the last 8 checks (10^4 steps apart) to average out the rounding
    noise, lie within 1e-3 of the oracle's steady values."""
    ref = golden_nu()[Ra]
    lat = L.Lattice(li.table2(Ra), storage="fp16", check_interval=10_000)
    lat.step(steps - 8 * 10_000 + 1)
    nus = []
    for _ in range(8):
        r = lat.residual()
        nus.append((r["nu_i"][0], r["nu_o"][0]))
        lat.step(10_000)
    lat.close()
    nui, nuo = np.mean(nus, axis=0)
    print(f"Ra={Ra:g} FP16: Nu_i {nui:.6f} (oracle {ref[0]:.6f}), Nu_o {nuo:.6f} (oracle {ref[1]:.6f})",
          flush=True)
    assert abs(nui - ref[0]) <= 1e-3 * ref[0]
    assert abs(nuo - ref[1]) <= 1e-3 * ref[1]


def test_handoff_fp16_then_fp32_reaches_fp32_steady_state(L):
    """Precision handoff: FP16 storage until its residual stops falling, then
    conversion to FP32 in place and on to res <= 1e-9.  The result is the
    FP32 steady state: Nu within 1e-4 of the oracle's steady values."""
    Ra = 1e4
    ref = golden_nu()[Ra]
    lat = L.Lattice(li.table2(Ra), storage="fp16", check_interval=1000, tol=1e-9, max_steps=2_000_000)
    best, flat = np.inf, 0
    while flat < 5 and lat.info()["t"] < 400_000:
        lat.step(1000)
        res = lat.residual()["res"][0]
        if res < 0.7 * best:
            best, flat = res, 0
        else:
            flat += 1
    t16 = lat.info()["t"]
    lat.set_storage("fp32")
    while lat.info()["status"] == "running":
        lat.step(20_000)
    r = lat.residual()
    info = lat.info()
    lat.close()
    print(f"handoff at t={t16} (res {best:.2e}), FP32 converged at t={info['t']}: "
          f"Nu_i {r['nu_i'][0]:.6f} Nu_o {r['nu_o'][0]:.6f}", flush=True)
    assert info["status"] == "converged"
    assert t16 > 0.5 * info["t"]  # most of the iterations ran in 16-bit storage
    assert abs(r["nu_i"][0] - ref[0]) <= 1e-4 * ref[0]
    assert abs(r["nu_o"][0] - ref[1]) <= 1e-4 * ref[1]


@pytest.mark.parametrize("to", ["fp16", "bf16"])
def test_set_storage_keeps_the_state(L, to):
    """FP32 -> 16-bit -> FP32 changes every field by at most the 16-bit
    rounding (to nearest: u16 / 2 per slot, relative to the deviations)."""
    cfgs = [li.annulus(nr=96, nz=72, Ra=1e5, Da=1e-3),
            li.annulus(nr=65, nz=130, Ra=1e4, Da=1e-5, Rstar=5.0, Pr=7.0)]
    lat = L.Lattice(cfgs, check_interval=50)
    lat.step(300)
    before = [lat.fields(i) for i in range(2)]
    lat.set_storage(to)
    mid = [lat.fields(i) for i in range(2)]
    lat.set_storage("fp32")
    after = [lat.fields(i) for i in range(2)]
    t = lat.info()["t"]
    lat.step(10)  # still steps after two conversions
    lat.close()
    assert t == 300
    for i in range(2):
        np.testing.assert_array_equal(before[i]["mask"], after[i]["mask"])
        for state in (mid[i], after[i]):
            e = rel_errors(state, before[i])
            assert max(e.values()) <= 3 * U16[to], (i, e)


@pytest.mark.parametrize("extra", [0, 1])
def test_converged_instance_resumes_in_its_own_layout(L, extra):
    """A storage conversion restarts a converged instance from the state at
    which it stopped.  Instance 0 converges at an odd level (a check step plus
    one), is dropped from the launch, and the handle runs on to a level of the
    other parity (extra = 0: an aligning step of its own is needed) or of the
    same parity (extra = 1).  After the FP32 -> FP32 conversion (exact) it
    takes further steps; its fields then equal, bit for bit, those of an
    uninterrupted run of as many steps as it has taken, and so do those of
    instance 1, which never stopped."""
    cfg = li.annulus(nr=48, nz=40, Ra=1e4, Da=1e-3)
    lat = L.Lattice([dict(cfg, tol=2e-3), dict(cfg, tol=0.0)], check_interval=10)
    while lat.info(0)["status"] == "running" and lat.info(1)["t"] < 100_000:
        lat.step(10)
    t_stop = lat.info(0)["t"]
    assert t_stop % 2 == 1 and lat.info(1)["t"] % 2 == 0
    assert lat.compact() == 1
    lat.step(extra)
    lat.set_storage("fp32")
    info0 = lat.info(0)
    assert info0["status"] == "running"
    assert info0["t"] == t_stop + (1 - extra), (info0, t_stop)
    lat.step(57)
    own0 = lat.info(0)["t"]
    own1 = lat.info(1)["t"]
    got = [lat.fields(0), lat.fields(1)]
    lat.close()
    print(f"stopped at {t_stop}, restarted at {info0['t']}, own steps {own0} / handle {own1}",
          flush=True)
    assert own0 > info0["t"]
    for f, n in zip(got, (own0, own1)):
        ref = L.Lattice(cfg, check_interval=0)
        ref.step(n)
        r = ref.fields()
        ref.close()
        for k in ("uz", "ur", "p", "T", "mask", "drho"):
            np.testing.assert_array_equal(f[k], r[k], err_msg=f"{k} after {n} steps")


def test_fp32_to_fp32_conversion_is_exact(L):
    cfg = li.annulus(nr=70, nz=40, Ra=1e5, Da=1e-3)
    lat = L.Lattice(cfg, check_interval=0)
    lat.step(51)
    a = lat.fields()
    lat.set_storage("fp32")
    b = lat.fields()
    lat.step(7)
    c = lat.fields()
    lat.close()
    ref = L.Lattice(cfg, check_interval=0)
    ref.step(58)
    d = ref.fields()
    ref.close()
    for k in ("uz", "ur", "p", "T", "mask", "drho"):
        np.testing.assert_array_equal(a[k], b[k])
        np.testing.assert_array_equal(c[k], d[k])


def test_fp16_beyond_4gib_uses_flat_addressing(L, oracle_mod):
    """A 13000^2 annulus in FP16 storage: 4.7 GB of populations, beyond the
    4 GiB reach of 32-bit buffer offsets, so the step kernels take the flat
    (64-bit address) path.  Windows of the field after 4 steps against the
    oracle on the same windows (every node farther than n + 2 from a window's
    artificial sides depends only on the window), at the FP16 bound."""
    from tests.test_gpu_parity import _window

    size, n, w = 13000, 4, 28
    cfg, _ = li.variable_porosity_annulus(n=size)
    phi = li.porosity_grf(size, size, seed=1409)
    lat = L.Lattice(cfg, phi=phi, storage="fp16", check_interval=0)
    assert lat.info()["device_bytes"] > 14 * size * size * 2 > 4 * 2 ** 30
    lat.step(n)
    g = lat.fields()
    lat.close()
    margin = n + 2
    tol = 6 * U16["fp16"]
    for j0, k0 in [(0, 0), (size - w, size // 2), (size // 2, size - w)]:
        c, ph = _window(cfg, phi, j0, k0, w)
        c["side_z"] = "wall"
        o = oracle_mod.Oracle(c, phi_field=ph)
        o.step(n)
        m = o.macros()
        o.close()
        jl = 0 if j0 == 0 else margin
        jh = w if j0 + w == size else w - margin
        kl = 0 if k0 == 0 else margin
        kh = w if k0 + w == size else w - margin
        sub = window(g, slice(k0 + kl, k0 + kh), slice(j0 + jl, j0 + jh))
        ref = window(m, slice(kl, kh), slice(jl, jh))
        np.testing.assert_array_equal(sub["mask"], ref["mask"])
        e = rel_errors(sub, ref, u_floor=1e-3 * li.U_SCALE, t_floor=cfg["delta_T"],
                      rho_floor=RHO_FLOOR_16)
        print(f"13000^2 FP16 window {(j0, k0)}: {e}", flush=True)
        assert max(e.values()) <= tol, (j0, k0, e)



def test_fp16_between_2_and_4_gib_uses_unsigned_buffer_offsets(L, oracle_mod):
    """A 10000^2 annulus in FP16 storage: 2.8 GB of populations, below 4 GiB,
    so the step kernels use buffer addressing, but the byte offsets of the
    last three planes (g_2, g_3, g_4) and the array size pass 2^31 and must
    be taken as unsigned 32-bit values.  Windows after 4 steps against the
    oracle, at the FP16 bound."""
    from tests.test_gpu_parity import _window

    size, n, w = 10000, 4, 28
    cfg, _ = li.variable_porosity_annulus(n=size)
    phi = li.porosity_grf(size, size, seed=1409)
    lat = L.Lattice(cfg, phi=phi, storage="fp16", check_interval=0)
    stride = (size + 63) // 64 * 64
    pop = 14 * stride * size * 2
    assert 2 ** 31 < 11 * stride * size * 2 and pop < 4 * 2 ** 30
    lat.step(n)
    g = lat.fields()
    lat.close()
    margin = n + 2
    tol = 6 * U16["fp16"]
    for j0, k0 in [(0, 0), (size - w, size // 2), (size // 2, size - w), (3333, 6666)]:
        c, ph = _window(cfg, phi, j0, k0, w)
        c["side_z"] = "wall"
        o = oracle_mod.Oracle(c, phi_field=ph)
        o.step(n)
        m = o.macros()
        o.close()
        jl = 0 if j0 == 0 else margin
        jh = w if j0 + w == size else w - margin
        kl = 0 if k0 == 0 else margin
        kh = w if k0 + w == size else w - margin
        sub = window(g, slice(k0 + kl, k0 + kh), slice(j0 + jl, j0 + jh))
        ref = window(m, slice(kl, kh), slice(jl, jh))
        np.testing.assert_array_equal(sub["mask"], ref["mask"])
        e = rel_errors(sub, ref, u_floor=1e-3 * li.U_SCALE, t_floor=cfg["delta_T"],
                      rho_floor=RHO_FLOOR_16)
        print(f"10000^2 FP16 window {(j0, k0)}: {e}", flush=True)
        assert max(e.values()) <= tol, (j0, k0, e)


def test_fp32_beyond_2g_elements(L, oracle_mod):
    """The same 13000^2 annulus in FP32: 14 planes of 169M nodes are 2.37G
    elements (9.5 GB), so element offsets pass 2^31 and the FP32 steps,
    whose odd step has its own load pipeline, must index in 64 bits.
    Windows after 5 steps (both parities and a second even step) against the
    oracle at the FP32 bound."""
    from tests.parity import TOL_FP32
    from tests.test_gpu_parity import _window

    size, n, w = 13000, 5, 30
    cfg, _ = li.variable_porosity_annulus(n=size)
    phi = li.porosity_grf(size, size, seed=1409)
    lat = L.Lattice(cfg, phi=phi, storage="fp32", check_interval=0)
    assert lat.info()["device_bytes"] > 14 * size * size * 4 > 8 * 2 ** 30
    lat.step(n)
    g = lat.fields()
    lat.close()
    margin = n + 2
    for j0, k0 in [(0, 0), (size - w, size // 2), (size // 2, size - w), (size - w, size - w)]:
        c, ph = _window(cfg, phi, j0, k0, w)
        c["side_z"] = "wall"
        o = oracle_mod.Oracle(c, phi_field=ph)
        o.step(n)
        m = o.macros()
        o.close()
        jl = 0 if j0 == 0 else margin
        jh = w if j0 + w == size else w - margin
        kl = 0 if k0 == 0 else margin
        kh = w if k0 + w == size else w - margin
        sub = window(g, slice(k0 + kl, k0 + kh), slice(j0 + jl, j0 + jh))
        ref = window(m, slice(kl, kh), slice(jl, jh))
        np.testing.assert_array_equal(sub["mask"], ref["mask"])
        e = rel_errors(sub, ref)
        print(f"13000^2 FP32 window {(j0, k0)}: {e}", flush=True)
        assert max(e.values()) <= TOL_FP32, (j0, k0, e)

def _boundary_cases():
    heater = li.heater_annulus(Da=1e-2, nr=48, nz=40, Ra=1e5)
    pipe = li.developing_pipe(Da=1e-2, nr=21, A=2.0, u_in=0.02)
    cyl = dict(nr=24, nz=30, r0=0.5, L=23.5, side_rmin="axis", side_rmax="wall", side_z="wall",
               therm_rmin="adiabatic", therm_rmax="adiabatic", therm_z="fixed", T_zmin=1.0,
               T_zmax=0.0, T_ref=0.5, T_init=0.5, delta_T=1.0, phi=0.8, Da=1e-2, F_phi=li.ERGUN,
               Ra=1e5, Pr=0.7, Ma=0.1)
    return [("heater", heater, None), ("pipe inlet/outlet", pipe, li.plug_start(pipe)),
            ("closed cylinder", cyl, None)]


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
@pytest.mark.parametrize("case", _boundary_cases(), ids=lambda c: c[0])
def test_storage_error_with_flux_inlet_outlet_and_axis_walls(L, oracle_mod, storage, case):
    """The isoflux heater, inlet/outlet columns and an axis with axial walls in
    16-bit storage, 500 steps: the same 6 u16 bound (velocity error measured
    against 1 % of Ma c_s where the flow is slower, temperature error against
    the temperature difference, density error against 10 % of Ma)."""
    from tests.parity import U_FLOOR

    name, cfg, init = case
    n = 500
    lat = L.Lattice(cfg, init=init, storage=storage, check_interval=0)
    lat.step(n)
    g = lat.fields()
    lat.close()
    o = oracle_mod.Oracle(cfg, init=init)
    o.step(n)
    m = o.macros()
    np.testing.assert_array_equal(g["mask"], m["mask"])
    e = rel_errors(g, m, U_FLOOR, t_floor=abs(cfg["delta_T"]), rho_floor=RHO_FLOOR_16)
    tol = 6 * U16[storage]
    print(f"{storage} {name}: rel L2 u {e['u']:.2e} rho-rho_bar {e['rho']:.2e} T-T_bar {e['T']:.2e} "
          f"p {e['p']:.2e} (tol {tol:.1e})", flush=True)
    for k, v in e.items():
        assert v <= tol, (storage, name, k, v)


def test_fp16_handoff_heater_steady_nusselt(L):
    """Table 3 heater (Da = 1e-2, 200 x 200): 1.5 million steps in FP16
    storage (of about 2.5 million to a residual of 1e-10), then handed over to
    FP32 in place and run to 1e-10.  At the handoff the FP16 run's heater
    Nusselt number is within 2e-3 of an FP32 run's at the same step; at the
    end the two agree within 1e-3 and lie within 2 % of the paper's 17.09."""
    cfg = li.heater_annulus(Da=1e-2)
    switch = 1_500_000

    def run(storage):
        lat = L.Lattice(cfg, storage=storage, check_interval=2000, tol=1e-10, max_steps=8_000_000)
        lat.step(switch + 1)  # the check at level `switch` runs in the step after it
        nu_mid = lat.residual()["nu_i"][0]
        if storage != "fp32":
            lat.set_storage("fp32")
        while lat.info()["status"] == "running":
            lat.step(100_000)
        out = (nu_mid, lat.residual()["nu_i"][0], lat.info())
        lat.close()
        return out

    m32, nu32, i32 = run("fp32")
    m16, nu16, i16 = run("fp16")
    print(f"heater Da=1e-2 at {switch} steps: FP32 Nu {m32:.5f}, FP16 Nu {m16:.5f}; final: FP32 "
          f"{nu32:.5f} ({i32['t']} steps), FP16 then FP32 {nu16:.5f} ({i16['t']} steps)", flush=True)
    assert i32["status"] == "converged" and i16["status"] == "converged"
    assert abs(m16 - m32) <= 2e-3 * m32
    assert abs(nu16 - nu32) <= 1e-3 * nu32
    assert abs(nu16 - 17.09) <= 0.02 * 17.09


def _window(cfg, phi, j0, k0, w):
    """w x w sub-problem: real walls where the window touches them, walls
    elsewhere (which contaminate only a margin)."""
    c = dict(cfg)
    c.update(nr=w, nz=w, r0=cfg["r0"] + j0, side_z="wall")
    if j0 > 0:
        c.update(side_rmin="wall", therm_rmin="adiabatic")
    if j0 + w < cfg["nr"]:
        c.update(side_rmax="wall", therm_rmax="adiabatic")
    return c, phi[k0:k0 + w, j0:j0 + w]


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_full_size_16bit_sampled_windows(L, oracle_mod, storage):
    """8192^2 throughput problem in 16-bit storage, in the benchmark's launch
    configuration: after n steps a node farther than n + 2 from a window's
    artificial sides depends only on the window, so the oracle run on the
    window gives it up to the storage rounding; the bound is the 512^2 one,
    6 u16 in relative L2 (velocity measured against a floor near rest).  Where
    the oracle's temperature is identically zero (cold outer wall, before the
    heat arrives) T is checked absolutely, against 6 u16 dT."""
    from tests.parity import U_FLOOR

    size, n, w = 8192, 32, 100
    cfg, _ = li.variable_porosity_annulus(n=size)
    phi = li.porosity_grf(size, size, seed=1409)
    lat = L.Lattice(cfg, phi=phi, storage=storage, check_interval=100)
    lat.step(n)
    g = lat.fields()
    lat.close()
    tol = 6 * U16[storage]
    margin = n + 2
    worst = 0.0
    for j0, k0 in [(0, 0), (0, size // 2), (0, size - w), (size - w, size - w), (size - w, 1234)]:
        c, ph = _window(cfg, phi, j0, k0, w)
        o = oracle_mod.Oracle(c, phi_field=ph)
        o.step(n)
        m = o.macros()
        o.close()
        jl = 0 if j0 == 0 else margin
        jh = w if j0 + w == size else w - margin
        kl = 0 if k0 == 0 else margin
        kh = w if k0 + w == size else w - margin
        sub = window(g, slice(k0 + kl, k0 + kh), slice(j0 + jl, j0 + jh))
        ref = window(m, slice(kl, kh), slice(jl, jh))
        np.testing.assert_array_equal(sub["mask"], ref["mask"])
        e = rel_errors(sub, ref, u_floor=U_FLOOR, t_floor=cfg["delta_T"], rho_floor=RHO_FLOOR_16)
        if not np.any(ref["T"]):
            e["T"] = float(np.abs(sub["T"]).max() / cfg["delta_T"])
        print(f"{storage} 8192^2 window ({j0}, {k0}) n={n}: u {e['u']:.2e} p {e['p']:.2e} "
              f"T {e['T']:.2e} (tol {tol:.1e})", flush=True)
        worst = max(worst, *e.values())
        for k, v in e.items():
            assert v <= tol, (storage, j0, k0, k, v)
    print(f"{storage} 8192^2 windows: worst {worst:.2e}", flush=True)
