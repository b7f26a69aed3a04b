"""Launch shapes of the step kernel do not change results.

Each node's update is the same arithmetic whichever thread performs it, so the
strip length kz (nodes per thread along z), the cap on resident blocks per
compute unit and the default shapes, which differ between the two parities of
the AA step, must all give bit-identical fields, residuals and Nusselt
numbers. Checked against the default shape on grids whose sizes are multiples
of neither the 64-lane block width nor the strip height, with every side
condition in one handle (fixed-temperature walls with a porosity field,
periodic ends, an isoflux heater, an axis with inlet and outlet), from random
start fields, with the shape changed after an odd number of steps and check
steps on both sides of the change."""
import numpy as np
import pytest

import lbm_inputs as li

pytestmark = pytest.mark.gpu

KEYS = ("uz", "ur", "p", "T", "mask", "drho")


@pytest.fixture(scope="module")
def L():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1409_5929_amd import lbm

    lbm._load()
    return lbm


def _problems():
    rng = np.random.default_rng(1409)
    walls = li.annulus(nr=131, nz=77, Ra=1e5, Da=1e-3)
    periodic = dict(li.annulus(nr=65, nz=33, Ra=1e4, Da=1e-2, Rstar=5.0), side_z="periodic")
    heater = li.heater_annulus(Da=1e-2, nr=70, nz=45)
    pipe = li.developing_pipe(Da=1e-2, nr=45, A=2.0, u_in=0.01)
    cfgs = [walls, periodic, heater, pipe]
    inits = []
    for c in cfgs:
        a = np.zeros((3, c["nz"], c["nr"]))
        a[0] = rng.uniform(-0.01, 0.01, a[0].shape) + c.get("u_in", 0.0)
        a[1] = rng.uniform(-0.01, 0.01, a[1].shape)
        a[2] = c["T_init"] + rng.uniform(0.0, 0.2, a[2].shape) * c["delta_T"]
        inits.append(a)
    phis = [li.porosity_grf(77, 131, seed=7), None, None, None]
    return cfgs, phis, inits


def _run(L, storage, shape):
    cfgs, phis, inits = _problems()
    lat = L.Lattice(cfgs, phi=phis, init=inits, storage=storage, check_interval=5)
    lat.step(7)
    if shape is not None:
        lat.set_tiles(*shape)
    lat.step(16)
    out = dict(fields=[lat.fields(i) for i in range(len(cfgs))], res=lat.residual(),
               t=lat.info()["t"])
    lat.close()
    return out


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
def test_launch_shape_does_not_change_results(L, storage):
    ref = _run(L, storage, None)
    assert ref["t"] == 23
    for f in ref["fields"]:
        assert all(np.isfinite(f[k]).all() for k in ("uz", "ur", "p", "T"))
    for shape in [(1, 0), (2, 0), (3, 0), (5, 3), (8, 0), (16, 2), (64, 0)]:
        got = _run(L, storage, shape)
        for i, (a, b) in enumerate(zip(ref["fields"], got["fields"])):
            for k in KEYS:
                np.testing.assert_array_equal(a[k], b[k], err_msg=f"{storage} {shape} instance {i}: {k}")
        for k in ("res", "nu_i", "nu_o", "status"):
            np.testing.assert_array_equal(ref["res"][k], got["res"][k], err_msg=f"{storage} {shape}: {k}")


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("case", ["annulus field", "pipe axis periodic", "closed cylinder"])
def test_pattern_probe_leaves_the_state_unchanged(L, storage, case):
    """The streaming-ceiling probe makes the step's loads and stores and puts
    every value back where node_load read it; afterwards the run continues
    bit for bit as if the probe had not run, at either parity.  This also shows
    that the probe's slot map (node_slots) is node_load's, slot for slot.  The
    lane-width probe (an in-place stream at 2 to 16 bytes per lane) is run in
    the same way."""
    if case == "annulus field":
        cfg = li.annulus(nr=150, nz=70, Ra=1e5, Da=1e-3)
        phi = li.porosity_grf(70, 150, seed=2, sigma=3.0)
    elif case == "pipe axis periodic":
        cfg, phi = li.pipe(nr=70, nz=12), None
    else:
        cfg = li.pipe(nr=33, nz=40)
        cfg.update(side_z="wall", therm_z="fixed", T_zmin=1.0, T_zmax=0.0)
        phi = None
    got = []
    for probe in (False, True):
        lat = L.Lattice(cfg, phi=phi, storage=storage, check_interval=0)
        lat.step(7)
        if probe:
            r = lat.pattern_bandwidth(reps=3)
            assert r["even_gbs"] > 0 and r["odd_gbs"] > 0 and r["stream_gbs"] > 0
        lat.step(4)
        if probe:
            lat.pattern_bandwidth(reps=2)
            w = lat.lane_bandwidth(reps=2)  # lane-width probe: also an identity
            assert all(np.isfinite(v) and v > 0 for v in w.values()), w
        lat.step(3)
        got.append(lat.fields())
        lat.close()
    for k in KEYS:
        np.testing.assert_array_equal(got[0][k], got[1][k], err_msg=k)
