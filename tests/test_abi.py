"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every entry point the header declares, its parameter struct has the layout of
the header, and invalid problems are refused before any device call."""
import ctypes
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "lbm_axi.h")


def _lib():
    from paper_1409_5929_amd import lbm

    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("liblbm_axi.so not built (run __graft_entry__.build())")
    return lbm._load(), lbm


def test_library_exports_every_declared_symbol():
    lib, _ = _lib()
    text = open(HEADER).read()
    names = sorted(set(re.findall(r"\b(lbm_axi_[a-z_]+)\s*\(", text)))
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), f"{n} declared in the header but not exported"


def test_params_layout_matches_header(tmp_path):
    """ctypes offsets of lbm_axi_params equal what a C compiler computes from the header."""
    _, lbm = _lib()
    fields = [f for f, _ in lbm.Params._fields_]
    cname = {"lambda_": "lambda"}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm_axi.h"', "int main(void){",
           'printf("%zu\\n", sizeof(lbm_axi_params));']
    for f in fields:
        src.append(f'printf("%zu\\n", offsetof(lbm_axi_params, {cname.get(f, f)}));')
    src.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), "-o", str(exe), str(c)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == ctypes.sizeof(lbm.Params)
    for f, off in zip(fields, vals[1:]):
        assert getattr(lbm.Params, f).offset == off, f


def test_default_params_are_the_papers_rates():
    _, lbm = _lib()
    p = lbm.make_params({"nr": 8, "nz": 8})
    assert (p.s_e, p.s_eps, p.s_q, p.s_j) == (1.1, 1.1, 1.2, 1.0)
    assert (p.J, p.lambda_, p.sigma, p.Ma) == (1.0, 1.0, 1.0, 0.1)


@pytest.mark.parametrize("bad, code", [
    (dict(nr=2), -1),                              # grid too small
    (dict(sigma=2.0), -4),                         # heat-capacity ratio other than 1
    (dict(side_rmin="axis", r0=1.0), -1),          # axis needs cell-centred rows
    (dict(side_rmax="axis"), -1),                  # axis only at r_min
    (dict(side_rmin="periodic"), -1),              # one-sided radial periodicity
    (dict(phi=1.5), -1),                           # porosity out of range
    (dict(tau_nu=0.0, Ra=0.0), -1),                # no way to set tau_nu
    (dict(side_rmin="flow"), -1),                  # inlet/outlet only along z
    (dict(side_z="flow", nz=2), -1),               # inlet and outlet need three columns
    (dict(therm_z="flux"), -1),                    # flux walls are radial only
    (dict(side_z="flow", u_in=float("nan")), -1),
    (dict(storage=7), -1),
])
def test_invalid_problems_are_refused_without_a_device(bad, code):
    lib, lbm = _lib()
    cfg = dict(nr=16, nz=16, r0=10.0, L=15.0, tau_nu=0.8, phi=0.5, Da=1e-2)
    storage = bad.pop("storage", 0)
    cfg.update(bad)
    p = lbm.make_params(cfg, storage=storage)
    h = ctypes.c_void_p()
    rc = lib.lbm_axi_create(ctypes.byref(p), 1, None, None, None, ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert lib.lbm_axi_last_error().decode()


def test_null_handles_are_refused():
    lib, _ = _lib()
    assert lib.lbm_axi_step(None, 1) == -1
    assert lib.lbm_axi_sync(None) == -1
    assert lib.lbm_axi_set_storage(None, 1, 0) == -1
    assert lib.lbm_axi_set_tiles(None, 4, 0) == -1
    assert lib.lbm_axi_set_wall_lanes(None, 1, None) == -1
    assert lib.lbm_axi_lane_bandwidth(None, 1, None) == -1
    assert lib.lbm_axi_set_graph(None, 32) == -1
    assert lib.lbm_axi_compact(None, None) == -1
    assert lib.lbm_axi_autotune(None, 1, None, None, None) == -1
    assert lib.lbm_axi_stream_function(None, 0, None, None, 0) == -1
    assert lib.lbm_axi_pipe_nusselt(None, 0, 0, None, None) == -1
    assert lib.lbm_axi_density_deviation(None, 0, None, 0) == -1
    assert lib.lbm_axi_pattern_bandwidth(None, 1, None) == -1
    assert lib.lbm_axi_stream_function_static(None, 0, None, None) == -1
    assert lib.lbm_axi_derived(None, None) == -1
    lib.lbm_axi_destroy(None)  # allowed


def test_network_library_exports_and_counts_parameters():
    from oracle import no_oracle as N
    from paper_1409_5929_amd import no

    if not os.path.exists(no.LIB_PATH):
        pytest.skip("liblbm_no.so not built (run __graft_entry__.build())")
    lib = no._load()
    text = open(os.path.join(ROOT, "include", "lbm_no.h")).read()
    names = sorted(set(re.findall(r"\b(lbm_no_[a-z_]+)\s*\(", text)))
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), f"{n} declared in lbm_no.h but not exported"
    for w in [(8, 16, 24, 32), (48, 96, 192, 384), (1, 1, 1, 1)]:
        assert no.param_count(w) == N.param_count(w)
    bad = (ctypes.c_int32 * 4)(0, 1, 1, 1)
    n = ctypes.c_int64()
    assert lib.lbm_no_param_count(bad, ctypes.byref(n)) == -1
    # create checks its arguments before any device call: the limits of lbm_no.h
    par = (ctypes.c_float * 1)()
    for widths, hh, ww, mb in [((8, 16, 24, 33), 64, 64, 1), ((0, 16, 24, 32), 64, 64, 1),
                               ((8, 16, 24, 1026), 64, 64, 1), ((8, 16, 24, 32), 60, 64, 1),
                               ((8, 16, 24, 32), 64, 2056, 1), ((8, 16, 24, 32), 64, 64, 0),
                               ((8, 16, 24, 32), 2048, 2048, 9)]:
        handle = ctypes.c_void_p(1)
        rc = lib.lbm_no_create((ctypes.c_int32 * 4)(*widths), hh, ww, mb, par, None, ctypes.byref(handle))
        assert rc == -1 and handle.value is None, (widths, hh, ww, mb, rc)
    assert lib.lbm_no_forward(None, None, 1, None) == -1
    assert lib.lbm_no_adam(None, 1e-3, 0.9, 0.999, 1e-8) == -1
    lib.lbm_no_destroy(None)


def test_binding_has_every_entry_point_by_name():
    """Every lbm_axi_<name> of the header is Lattice.<name> (create is the
    constructor; default_params fills problem dictionaries; last_error is read
    by the error path)."""
    from paper_1409_5929_amd.lbm import Lattice

    text = open(HEADER).read()
    names = sorted(set(re.findall(r"\blbm_axi_([a-z_]+)\s*\(", text)))
    special = {"create", "default_params", "last_error"}
    missing = [n for n in names if n not in special and not callable(getattr(Lattice, n, None))]
    assert not missing, missing


def test_network_binding_has_every_entry_point_by_name():
    from paper_1409_5929_amd import no

    text = open(os.path.join(ROOT, "include", "lbm_no.h")).read()
    names = sorted(set(re.findall(r"\blbm_no_([a-z_]+)\s*\(", text)))
    special = {"create", "param_count", "last_error"}
    missing = [n for n in names if n not in special and not callable(getattr(no.WarmStartNet, n, None))]
    assert not missing, missing
    assert callable(no.param_count)
