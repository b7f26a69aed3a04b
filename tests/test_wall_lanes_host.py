"""The radial wall lanes of the step kernel, checked on the host (no GPU).

A host build of the kernel's node code (tests/wall_lanes_host.hip, FP32
storage) runs each fluid row as a wave of the step kernel does: every node of
the row loads before any node of the row stores.  With wall lanes, the lane of
a no-slip wall column loads its owner's populations and runs its wall node
through the fluid collision: the non-equilibrium extrapolation of Sec. 4 fed
into the shared back-transform and stores, its populations that stream into
no fluid node written into the wall column's own slots.  Without wall lanes
the owner computes the wall node after its own update.  For each problem and
both parities:
* the two variants give bit-identical fields (the same FP32 operations);
* both match the FP64 oracle within the FP32 bound;
* no store reaches the padding columns of any row (sentinel values).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import lbm_inputs as li
import oracle
from tests.parity import RHO_FLOOR, RHO_FLOOR_16, U_FLOOR, rel_errors, tol_fp32

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "wall_lanes_host.hip")
LIB = os.path.join(HERE, "libwall_lanes_host.so")
DEPS = [SRC] + [os.path.join(ROOT, "paper_1409_5929_amd", "csrc", f) for f in ("lbm_axi_dev.h", "lbm_axi_desc.h")]


def build_host_lib(force: bool = False) -> str:
    """Compile the host build of the node code (hipcc, host code only used)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(f) for f in DEPS):
        hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-shared", "-fPIC",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp", SRC])
        os.replace(LIB + ".tmp", LIB)
    return LIB


@pytest.fixture(scope="module")
def host():
    lib = ctypes.CDLL(build_host_lib())
    fp = ctypes.POINTER(ctypes.c_float)
    lib.host_wall_lane_steps.argtypes = [ctypes.c_void_p, fp, fp, ctypes.c_int, ctypes.c_int, fp, fp, fp, fp]
    lib.host_wall_lane_steps.restype = ctypes.c_int
    from paper_1409_5929_amd import lbm

    def run(cfg, n, init, wlmode, phi=None):
        p = lbm.make_params(cfg, check_interval=0)
        out = {k: np.zeros((cfg["nz"], cfg["nr"]), np.float32) for k in ("uz", "ur", "drho", "T")}
        ini = np.ascontiguousarray(init, np.float32)
        ph = None if phi is None else np.ascontiguousarray(phi, np.float32)
        rc = lib.host_wall_lane_steps(ctypes.byref(p), ph.ctypes.data_as(fp) if ph is not None else None,
                                      ini.ctypes.data_as(fp), n, wlmode,
                                      *[out[k].ctypes.data_as(fp) for k in ("uz", "ur", "drho", "T")])
        assert rc == 0, f"host steps returned {rc} (-2: a store reached a row's padding)"
        return out

    return run


def _init(cfg, seed):
    if cfg.get("side_z") == "flow":
        return li.plug_start(cfg)
    rng = np.random.default_rng(seed)
    a = np.zeros((3, cfg["nz"], cfg["nr"]))
    a[0] = rng.uniform(-0.01, 0.01, a[0].shape) + cfg.get("u_in", 0.0)
    a[1] = rng.uniform(-0.01, 0.01, a[1].shape)
    a[2] = cfg.get("T_init", 0.0) + rng.uniform(0.0, 0.2, a[2].shape) * cfg.get("delta_T", 1.0)
    return a


def _cases():
    cyl = dict(r0=0.5, side_rmin="axis", therm_rmin="adiabatic", therm_z="fixed", T_zmin=1.0, T_zmax=0.0,
               T_rmax=0.0, delta_T=1.0, T_ref=0.5, L=20.0, phi=0.7, Da=1e-2, F_phi=-1.0, Ra=1e4, Pr=0.7,
               nr=21, nz=30)
    sw = li.sweep(n_inst=8, seed=1409, sizes=np.arange(32, 161, 32))
    return [
        ("annulus 66 wide (r_max lane in its owner's wave)", li.annulus(nr=66, nz=21, Ra=1e5, Da=1e-3), True),
        ("annulus 65 wide (owner keeps the r_max wall)", li.annulus(nr=65, nz=19, Ra=1e5, Da=1e-3), False),
        ("three columns", li.annulus(nr=3, nz=11, Ra=1e4, Da=1e-2), False),
        ("periodic ends", dict(li.annulus(nr=30, nz=16, Ra=1e4, Da=1e-2), side_z="periodic", accel_z=1e-4), False),
        ("isoflux heater", li.heater_annulus(Da=1e-2, nr=40, nz=40), False),
        ("pipe: axis, outer wall, inlet and outlet", li.developing_pipe(Da=1e-2, nr=45, A=2.0, u_in=0.01), False),
        ("closed cylinder: axis, outer wall, z walls", cyl, False),
        ("sweep instance", sw[3], False),
    ]


@pytest.mark.parametrize("n", [7, 8])
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0].split(" (")[0].split(":")[0])
def test_wall_lanes_match_the_owner_pass_and_the_oracle(host, case, n):
    name, cfg, field = case
    phi = li.porosity_grf(cfg["nz"], cfg["nr"], seed=5) if field else None
    init = _init(cfg, 1409 + n)
    with_lanes = host(cfg, n, init, 1, phi)
    owners = host(cfg, n, init, 0, phi)
    for k in ("uz", "ur", "drho", "T"):
        np.testing.assert_array_equal(with_lanes[k], owners[k], err_msg=f"{name}, {n} steps: {k}")
    o = oracle.Oracle(cfg, phi_field=phi, init=init)
    o.step(n)
    m = o.macros()
    o.close()
    fluid = m["mask"] == 0
    ref = {k: np.where(fluid, m[k], 0.0) for k in ("uz", "ur", "T")}
    ref["rho"] = np.where(fluid, m["rho"], 1.0)
    ref["p"] = m["p"]
    got = {k: np.where(fluid, with_lanes[k], 0.0) for k in ("uz", "ur", "T")}
    got["rho"] = np.where(fluid, 1.0 + with_lanes["drho"].astype(np.float64), 1.0)
    got["p"] = m["p"]  # the host build returns no pressure; it is compared on the GPU
    rho_floor = RHO_FLOOR_16 if cfg.get("side_z") == "flow" and n > 8 else RHO_FLOOR
    e = rel_errors(got, ref, u_floor=U_FLOOR, rho_floor=rho_floor)
    print(f"{name}, {n} steps: " + " ".join(f"{k} {v:.1e}" for k, v in e.items()), flush=True)
    assert max(e.values()) <= tol_fp32(n), (name, n, e)
