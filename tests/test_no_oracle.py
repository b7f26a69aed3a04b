"""Pins of the warm-start network oracle (CPU, FP64) against library routines
and the mathematics: convolution = scipy's 2-D cross-correlation summed over
input channels, gradients = central finite differences, upsampling and its
adjoint satisfy <up x, y> = <x, up^T y>, one Adam step from rest equals its
closed form."""
import numpy as np
import pytest
from scipy.signal import correlate2d

import lbm_inputs as li
from oracle import no_oracle as N


@pytest.mark.parametrize("k,stride", [(3, 1), (3, 2), (1, 1)])
def test_conv_is_channel_summed_cross_correlation(k, stride):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 10, 12))
    W = rng.standard_normal((4, 3, k, k))
    b = rng.standard_normal(4)
    y = N.conv(x, W, b, stride)
    p = (k - 1) // 2
    for bi in range(2):
        for o in range(4):
            ref = sum(correlate2d(np.pad(x[bi, c], p), W[o, c], mode="valid") for c in range(3))
            ref = ref[::stride, ::stride] + b[o]
            np.testing.assert_allclose(y[bi, o], ref, rtol=1e-12, atol=1e-12)


def test_upsample_adjoint():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 3, 5, 7))
    g = rng.standard_normal((2, 3, 10, 14))
    assert abs(np.sum(N.upsample2(x) * g) - np.sum(x * N.upsample2_adjoint(g))) < 1e-10


def test_gradients_match_finite_differences():
    widths = (3, 4, 5, 6)
    params = li.no_init_params(widths, seed=11).astype(np.float64)
    params += 0.05 * np.random.default_rng(5).standard_normal(params.size)  # nonzero biases too
    rng = np.random.default_rng(6)
    x = rng.standard_normal((2, 6, 16, 16))
    t = rng.standard_normal((2, 3, 16, 16))
    loss, g = N.loss_and_grads(params, widths, x, t)
    assert g.size == N.param_count(widths) == params.size
    idx = rng.choice(params.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(params)
        e[i] = h
        fd = (N.loss_and_grads(params + e, widths, x, t)[0] - N.loss_and_grads(params - e, widths, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(7)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    z = np.zeros(50)
    p1, m, v = N.adam_step(p, g, z, z, 1, lr=1e-3, eps=1e-8)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_feature_planes():
    cfg = li.annulus(nr=128, nz=128, Rstar=2.0, Ra=1e6, Da=1e-2, phi=0.95, Pr=1.0)
    f = li.no_features(cfg)
    assert f.shape == (6, 128, 128)
    np.testing.assert_allclose(f[:5, 0, 0], [1.0, 1.0, 1.0, 0.0, np.log(2) / np.log(10)], rtol=1e-6)
    np.testing.assert_allclose(f[5, 0, [0, -1]], [0.5, 1.0], rtol=1e-6)


def test_conduction_profile_closed_form():
    """T = T_o + (T_i - T_o) ln(r_o / r) / ln R*: wall values, and r dT/dr
    constant (zero divergence of the radial conduction flux)."""
    cfg = li.annulus(nr=65, nz=8, Rstar=3.0)
    T = li.conduction_T(cfg)[0]
    r = cfg["r0"] + np.arange(65)
    assert abs(T[0] - cfg["T_rmin"]) < 1e-12 and abs(T[-1] - cfg["T_rmax"]) < 1e-12
    flux = r * np.gradient(T, r)
    np.testing.assert_allclose(flux[2:-2], flux[2], rtol=1e-3)


def test_targets_and_fields_are_inverse():
    cfg = li.annulus(nr=32, nz=24, Rstar=2.0)
    rng = np.random.default_rng(2)
    f = {k: rng.standard_normal((24, 32)).astype(np.float32) for k in ("uz", "ur", "T")}
    back = li.no_fields(li.no_targets(f, cfg), cfg)
    for i, k in enumerate(("uz", "ur", "T")):
        np.testing.assert_allclose(back[i], f[k], rtol=1e-5, atol=1e-6)


def test_committed_weights_load_in_bfloat16():
    from paper_1409_5929_amd import warmstart as ws

    p = ws.load_weights(ws.WEIGHTS)
    assert p.size == N.param_count(ws.WIDTHS)
    assert np.isfinite(p).all()
    assert (p.view(np.uint32) & 0xFFFF == 0).all()  # bfloat16 values
