"""The stream function entry point that allocates nothing
(lbm_axi_stream_function_static), called through the C ABI, against the
allocating lbm_axi_stream_function: two calls in a row, the second on a
smaller instance (the shared static scratch still holds the first call's
values), bit for bit; an instance beyond the scratch's limits is refused."""
import ctypes

import numpy as np
import pytest

import lbm_inputs as li

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1409_5929_amd import lbm as m

    m._load()
    return m


def _static(lib, lat, psi, mx):
    p = ctypes.c_void_p(psi.data_ptr()) if psi is not None else None
    m = ctypes.c_void_p(mx.data_ptr()) if mx is not None else None
    return lib.lbm_axi_stream_function_static(lat._h, 0, p, m)


def test_static_stream_function_equals_the_allocating_one(lbm):
    import torch

    lib = lbm._load()
    cases = [("heater 300x220", li.heater_annulus(Da=1e-4, nr=300, nz=220), 301),
             ("pipe 41x30 (axis)", li.pipe(nr=41, nz=30), 200)]
    for name, cfg, n in cases:
        lat = lbm.Lattice(cfg, check_interval=0)
        lat.step(n)
        psi_ref, mx_ref = lat.stream_function()  # allocating entry point, host outputs
        nz, nr = lat.shapes[0]
        psi = torch.full((nz, nr), float("nan"), dtype=torch.float32, device="cuda")
        mx = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        assert _static(lib, lat, psi, mx) == 0, lib.lbm_axi_last_error()
        lat.sync()
        got, got_mx = psi.cpu().numpy(), mx.item()
        # max only, no field
        mx2 = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        assert _static(lib, lat, None, mx2) == 0
        lat.sync()
        lat.close()
        print(f"{name}: max |psi| {got_mx:.6e} (allocating {mx_ref:.6e})", flush=True)
        np.testing.assert_array_equal(got, psi_ref, err_msg=name)
        assert got_mx == mx_ref and mx2.item() == mx_ref, name


def test_static_stream_function_refuses_more_columns_than_its_scratch(lbm):
    import torch

    lib = lbm._load()
    cfg = li.pipe(nr=3, nz=70_000)
    lat = lbm.Lattice(cfg, check_interval=0)
    mx = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert _static(lib, lat, None, mx) == -1  # LBM_AXI_EINVAL
    assert "scratch" in lib.lbm_axi_last_error().decode()
    lat.close()


def test_binding_method_checks_the_tensors_and_makes_the_same_call(lbm):
    """Lattice.stream_function_static: caller device tensors of the right size
    give the allocating entry point's values; a tensor too small for the
    instance is refused before the library writes through it."""
    import torch

    lat = lbm.Lattice(li.pipe(nr=41, nz=30), check_interval=0)
    lat.step(200)
    psi_ref, mx_ref = lat.stream_function()
    nz, nr = lat.shapes[0]
    psi = torch.full((nz, nr), float("nan"), dtype=torch.float32, device="cuda")
    mx = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    lat.stream_function_static(0, psi, mx)
    lat.sync()
    got, got_mx = psi.cpu().numpy(), mx.item()
    with pytest.raises(ValueError):
        lat.stream_function_static(0, torch.zeros((nz, nr - 1), dtype=torch.float32, device="cuda"), None)
    lat.close()
    np.testing.assert_array_equal(got, psi_ref)
    assert got_mx == mx_ref
