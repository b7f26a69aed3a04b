"""Argument checks of the Python bindings that guard memory the libraries
read or write through raw pointers, exercised on the host (no device call is
reached): the network's parameter vector (the library copies
lbm_no_param_count floats from it) and the caller tensors of the stream
function entry point that allocates nothing (nz nr floats and one double are
written through them)."""
import numpy as np
import pytest
import torch

from paper_1409_5929_amd import lbm, no


def test_network_set_params_refuses_a_vector_of_the_wrong_length():
    if not __import__("os").path.exists(no.LIB_PATH):
        pytest.skip("liblbm_no.so not built (run __graft_entry__.build())")
    net = object.__new__(no.WarmStartNet)  # no device handle: the check comes first
    net.widths, net._h, net._lib = (8, 16, 24, 32), None, None
    n = no.param_count(net.widths)
    for bad in (n - 1, n + 1, 0):
        with pytest.raises(no.NoError, match="wrong length"):
            net.set_params(np.zeros(bad, np.float32))


def test_static_stream_function_refuses_tensors_it_cannot_write():
    lat = object.__new__(lbm.Lattice)  # no device handle: the checks come first
    lat.shapes = [(4, 5)]
    ok_max = torch.zeros(1, dtype=torch.float64)
    shape = "contiguous torch.float32 tensor of 20 elements"
    bad = [
        (torch.zeros(19, dtype=torch.float32), None, shape),                     # too small
        (torch.zeros((4, 5), dtype=torch.float64), None, shape),                 # wrong type
        (torch.zeros((5, 8), dtype=torch.float32)[:, :4], None, shape),          # strided view
        (None, torch.zeros(2, dtype=torch.float64), "torch.float64 tensor of 1 elements"),
        (None, torch.zeros(1, dtype=torch.float32), "torch.float64 tensor of 1 elements"),
        (torch.zeros((4, 5), dtype=torch.float32), None, "psi: expected device memory"),
        (None, ok_max, "psi_absmax: expected device memory"),
    ]
    for psi, mx, msg in bad:
        with pytest.raises(ValueError, match=msg):
            lat.stream_function_static(0, psi, mx)
