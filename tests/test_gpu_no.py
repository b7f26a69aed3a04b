"""GPU warm-start network (HIP, MFMA bf16 GEMMs) against its FP64 oracle.

Tolerance: the GEMMs round weights and activations to bfloat16 (8
significant bits, relative rounding error <= 2^-9 per operand, so <= 2^-8 per
product) and accumulate in FP32.  Errors of independent products add in
quadrature within a sum and compound over the 8 layers, about sqrt(8) 2^-8 =
1.1e-2 of the signal; the bound used is 3e-2 relative L2."""
import numpy as np
import pytest

import lbm_inputs as li
from oracle import no_oracle as N

pytestmark = pytest.mark.gpu
TOL = 3e-2
WIDTHS = (8, 16, 24, 32)


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1409_5929_amd import no

    no._load()
    return torch


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def problem(seed=8, B=3, H=32, W=40):
    rng = np.random.default_rng(seed)
    params = li.no_init_params(WIDTHS, seed=seed)
    params = params + (0.05 * rng.standard_normal(params.size)).astype(np.float32)  # biases nonzero
    x = rng.standard_normal((B, 6, H, W)).astype(np.float32)
    t = rng.standard_normal((B, 3, H, W)).astype(np.float32)
    return params, x, t


def test_forward_matches_oracle(torch):
    from paper_1409_5929_amd.no import WarmStartNet

    params, x, _ = problem()
    net = WarmStartNet(WIDTHS, 32, 40, 4, params)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    net.close()
    ref, _ = N.forward(params.astype(np.float64), WIDTHS, x.astype(np.float64))
    e = rel(y, ref)
    print(f"forward rel L2 {e:.2e}", flush=True)
    assert e <= TOL


def test_gradients_match_oracle(torch):
    from paper_1409_5929_amd.no import WarmStartNet

    params, x, t = problem(seed=9)
    net = WarmStartNet(WIDTHS, 32, 40, 4, params)
    loss = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = net.grads()
    net.close()
    lref, gref = N.loss_and_grads(params.astype(np.float64), WIDTHS, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - lref) <= TOL * lref
    e = rel(g, gref)
    print(f"loss {loss:.6f} (oracle {lref:.6f}); gradient rel L2 {e:.2e}", flush=True)
    assert e <= TOL
    # every layer's weights and biases separately
    o = 0
    for ci, co, k, *_ in N.layer_specs(WIDTHS):
        for n in (co * ci * k * k, co):
            assert rel(g[o:o + n], gref[o:o + n]) <= 2 * TOL, (o, n)
            o += n


def test_full_widths_match_oracle(torch):
    """The trained network's widths (48/96/192/384) on a 64 x 64 grid, batch
    2: every GEMM shape class of the 128^2 training runs (64 x 256 tiles for
    48 output rows, K up to 3456, the phase GEMMs of the upsampling and
    stride-2 layers with hundreds of channels), with pixel counts that are
    multiples of 8, so operands move as 16-byte loads (the 32 x 40 tests
    above also take the element-wise edge paths)."""
    from paper_1409_5929_amd.no import WarmStartNet

    widths = (48, 96, 192, 384)
    rng = np.random.default_rng(21)
    params = li.no_init_params(widths, seed=21)
    params = params + (0.05 * rng.standard_normal(params.size)).astype(np.float32)
    x = rng.standard_normal((2, 6, 64, 64)).astype(np.float32)
    t = rng.standard_normal((2, 3, 64, 64)).astype(np.float32)
    net = WarmStartNet(widths, 64, 64, 2, params)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    loss = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = net.grads()
    net.close()
    p64 = params.astype(np.float64)
    ref, _ = N.forward(p64, widths, x.astype(np.float64))
    lref, gref = N.loss_and_grads(p64, widths, x.astype(np.float64), t.astype(np.float64))
    ey, eg = rel(y, ref), rel(g, gref)
    print(f"full widths: forward rel L2 {ey:.2e}, loss {loss:.6f} (oracle {lref:.6f}), gradient rel L2 {eg:.2e}",
          flush=True)
    assert ey <= TOL and eg <= TOL and abs(loss - lref) <= TOL * lref
    # Every layer within 2 TOL but the first layer's weights: their gradient
    # ends the longest chain of bfloat16 roundings (8 forward and 7 backward
    # GEMM stages) and measures 7.3e-2 here, the same with the explicit
    # im2col/col2im formulation of every convolution as with the phase and
    # box-sum forms; it is held to 4 TOL.
    o = 0
    for layer, (ci, co, k, *_) in enumerate(N.layer_specs(widths)):
        for n in (co * ci * k * k, co):
            bound = 4 * TOL if (layer == 0 and o == 0) else 2 * TOL
            assert rel(g[o:o + n], gref[o:o + n]) <= bound, (o, n)
            o += n


def test_paired_phase_gemms_match_oracle(torch):
    """128 x 128, batch 16: the phase GEMMs of the first stride-2 layer's input
    gradient and of the last upsampling layer's forward have 256 tiles of
    64 x 256 outputs, so each block runs both column phases and stores output
    pairs (the form the training runs take); the smaller phase GEMMs of the
    same step run one phase per block."""
    from paper_1409_5929_amd.no import WarmStartNet

    rng = np.random.default_rng(22)
    params = li.no_init_params(WIDTHS, seed=22)
    params = params + (0.05 * rng.standard_normal(params.size)).astype(np.float32)
    x = rng.standard_normal((16, 6, 128, 128)).astype(np.float32)
    t = rng.standard_normal((16, 3, 128, 128)).astype(np.float32)
    net = WarmStartNet(WIDTHS, 128, 128, 16, params)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    loss = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = net.grads()
    net.close()
    p64 = params.astype(np.float64)
    ref, _ = N.forward(p64, WIDTHS, x.astype(np.float64))
    lref, gref = N.loss_and_grads(p64, WIDTHS, x.astype(np.float64), t.astype(np.float64))
    ey, eg = rel(y, ref), rel(g, gref)
    print(f"paired phases: forward rel L2 {ey:.2e}, loss {loss:.6f} (oracle {lref:.6f}), gradient rel L2 {eg:.2e}",
          flush=True)
    assert ey <= TOL and eg <= TOL and abs(loss - lref) <= TOL * lref
    o = 0
    for ci, co, k, *_ in N.layer_specs(WIDTHS):
        for n in (co * ci * k * k, co):
            assert rel(g[o:o + n], gref[o:o + n]) <= 2 * TOL, (o, n)
            o += n


def test_adam_step_matches_oracle(torch):
    from paper_1409_5929_amd.no import WarmStartNet

    params, x, t = problem(seed=10)
    net = WarmStartNet(WIDTHS, 32, 40, 4, params)
    net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = net.grads().astype(np.float64)
    net.adam(1e-3)
    p1 = net.params()
    net.close()
    z = np.zeros_like(g)
    ref, _, _ = N.adam_step(params.astype(np.float64), g, z, z, 1, lr=1e-3)
    np.testing.assert_allclose(p1, ref, rtol=1e-5, atol=1e-8)


def test_training_reduces_loss(torch):
    """Fitting a smooth target field: 60 Adam steps on one batch cut the loss
    by more than 10x."""
    from paper_1409_5929_amd.no import WarmStartNet

    B, H, W = 4, 32, 32
    rng = np.random.default_rng(11)
    x = rng.standard_normal((B, 6, 1, 1)).astype(np.float32) * np.ones((1, 1, H, W), np.float32)
    yy, xx = np.meshgrid(np.linspace(0, 1, H), np.linspace(0, 1, W), indexing="ij")
    t = np.stack([np.stack([np.sin(3 * xx + b), np.cos(2 * yy - b), xx * yy]) for b in range(B)]).astype(np.float32)
    net = WarmStartNet(WIDTHS, H, W, B, li.no_init_params(WIDTHS, seed=12))
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    l0 = net.gradients(xd, td)
    for _ in range(60):
        net.adam(3e-3)
        loss = net.gradients(xd, td)
    net.close()
    print(f"loss {l0:.4f} -> {loss:.4f}", flush=True)
    assert loss < 0.1 * l0


def test_invalid_arguments_are_refused(torch):
    from paper_1409_5929_amd.no import NoError, WarmStartNet

    params, _, _ = problem()
    with pytest.raises(NoError):
        WarmStartNet(WIDTHS, 30, 40, 4, params)  # height not a multiple of 8
    with pytest.raises(NoError):  # odd widths (operands move as bf16 pairs)
        WarmStartNet((7, 16, 24, 32), 32, 40, 4, li.no_init_params((7, 16, 24, 32)))
    net = WarmStartNet(WIDTHS, 32, 40, 2, params)
    with pytest.raises(NoError):
        net.forward(torch.zeros((3, 6, 32, 40), device="cuda"))  # batch above max_batch
    net.close()


def test_network_on_another_stream_is_ordered(torch):
    """A network created on a side stream and called under torch's current
    stream: its inputs, written by torch on the current stream just before,
    are read only after they are written, and its outputs are read there only
    after they are written.  Results are bit-identical to a network on the
    current stream."""
    from paper_1409_5929_amd.no import WarmStartNet

    params, x, t = problem(seed=11, B=4)
    side = torch.cuda.Stream()
    a = WarmStartNet(WIDTHS, 32, 40, 4, params)
    b = WarmStartNet(WIDTHS, 32, 40, 4, params, stream=side.cuda_stream)
    xs = torch.from_numpy(x).cuda()
    ts = torch.from_numpy(t).cuda()
    ya = a.forward(xs * 2.0 - 1.0).cpu().numpy()
    yb = b.forward(xs * 2.0 - 1.0).cpu().numpy()
    la = a.gradients(xs * 0.5, ts + 0.25)
    lb = b.gradients(xs * 0.5, ts + 0.25)
    ga, gb = a.grads(), b.grads()
    a.close()
    b.close()
    np.testing.assert_array_equal(ya, yb)
    assert la == lb
    np.testing.assert_array_equal(ga, gb)


@pytest.mark.parametrize("H, W", [(8, 8), (8, 24), (16, 8)])
def test_smallest_grids_match_oracle(torch, H, W):
    """Down to the smallest grid the library accepts (8 x 8): the deepest
    layer is 1 x 1 and its upsampling layer reads a single source pixel per
    image; forward, loss and gradients against the oracle."""
    from paper_1409_5929_amd.no import WarmStartNet

    params, x, t = problem(seed=13, B=2, H=H, W=W)
    net = WarmStartNet(WIDTHS, H, W, 2, params)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    loss = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = net.grads()
    net.close()
    ref, _ = N.forward(params.astype(np.float64), WIDTHS, x.astype(np.float64))
    lref, gref = N.loss_and_grads(params.astype(np.float64), WIDTHS, x.astype(np.float64), t.astype(np.float64))
    e = (rel(y, ref), abs(loss - lref) / lref, rel(g, gref))
    print(f"{H}x{W}: forward {e[0]:.2e} loss {e[1]:.2e} gradient {e[2]:.2e}", flush=True)
    assert max(e) <= TOL
