"""The forms in which the network library runs three of its convolutions,
checked as exact rewritings of the convolution (FP64, against torch's
convolution and its autograd on the CPU; no GPU, no library code):

* upsampling layers (3 x 3, padding 1, over a 2x nearest-neighbour
  upsampled source): the forward as four phase convolutions with 2 x 2
  effective taps over the source grid, reading two runs of a tap-major 3 x 3
  im2col of the source (k_gemm PH, forward_up);
* their weight and input gradients from the 2 x 2 box sums D[t][o][s] of dz
  on the source grid (k_dmap);
* stride-2 layers (3 x 3, padding 1): the input gradient as four phase
  GEMMs over a stack of dz shifted by (ey, ex) in {0, 1}^2 (k_emap,
  input_grad_s2), with the tap tables of prep_phase.
The index maps written here are the ones the kernels use (row runs, gaps,
taps per phase); a wrong run, gap, tap or phase offset fails these checks.
"""
import numpy as np
import torch

F = torch.nn.functional


def _up(x):
    return x.repeat_interleave(2, 2).repeat_interleave(2, 3)


def test_upsampling_forward_as_phase_convolutions():
    g = torch.Generator().manual_seed(1)
    B, cin, cout, Hs, Ws = 2, 5, 3, 4, 6
    src = torch.randn(B, cin, Hs, Ws, dtype=torch.float64, generator=g)
    W = torch.randn(cout, cin, 3, 3, dtype=torch.float64, generator=g)
    z = F.conv2d(_up(src), W, padding=1).numpy()
    s, Wn = src.numpy(), W.numpy()
    # tap-major 3 x 3 im2col of the source: row (3 (dy + 1) + dx + 1) cin + c
    col = np.zeros((9 * cin, B, Hs, Ws))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            t = 3 * (dy + 1) + dx + 1
            for y in range(Hs):
                for x in range(Ws):
                    if 0 <= y + dy < Hs and 0 <= x + dx < Ws:
                        col[t * cin:(t + 1) * cin, :, y, x] = s[:, :, y + dy, x + dx].T
    col = col.reshape(9 * cin, -1)
    out = np.zeros_like(z)
    for q in range(4):
        a, b = q >> 1, q & 1
        # effective taps: output row 2y + a reads source row y + floor((a + ky - 1) / 2)
        Weff = np.zeros((cout, 2, 2, cin))
        for u in range(2):
            for v in range(2):
                for ky in range(3):
                    for kx in range(3):
                        if ((a + ky + 1) >> 1) - 1 == a - 1 + u and ((b + kx + 1) >> 1) - 1 == b - 1 + v:
                            Weff[:, u, v, :] += Wn[:, :, ky, kx]
        Weff = Weff.reshape(cout, 4 * cin)
        base, run, gap = (3 * a + b) * cin, 2 * cin, cin
        rows = [base + k + (gap if k >= run else 0) for k in range(4 * cin)]
        out.transpose(1, 0, 2, 3)[:, :, a::2, b::2] = (Weff @ col[rows]).reshape(cout, B, Hs, Ws)
    np.testing.assert_allclose(out, z, rtol=0, atol=1e-12)


def test_upsampling_gradients_from_box_sums():
    g = torch.Generator().manual_seed(2)
    B, cin, cout, Hs, Ws = 2, 5, 3, 4, 6
    src = torch.randn(B, cin, Hs, Ws, dtype=torch.float64, generator=g, requires_grad=True)
    W = torch.randn(cout, cin, 3, 3, dtype=torch.float64, generator=g, requires_grad=True)
    z = F.conv2d(_up(src), W, padding=1)
    dz = torch.randn(z.shape, dtype=torch.float64, generator=g)
    (z * dz).sum().backward()
    dz = dz.numpy()
    Ho, Wo = 2 * Hs, 2 * Ws
    # D[t][o][b][sy][sx]: tap (ky, kx) takes output rows 2sy + 1 - ky, 2sy + 2 - ky
    # (block rows 2 - ky, 3 - ky of the 4 x 4 block from 2sy - 1), likewise columns
    D = np.zeros((9, cout, B, Hs, Ws))
    for sy in range(Hs):
        for sx in range(Ws):
            v = np.zeros((cout, B, 4, 4))
            for i in range(4):
                for j in range(4):
                    Y, X = 2 * sy - 1 + i, 2 * sx - 1 + j
                    if 0 <= Y < Ho and 0 <= X < Wo:
                        v[:, :, i, j] = dz[:, :, Y, X].T
            for ky in range(3):
                for kx in range(3):
                    D[3 * ky + kx, :, :, sy, sx] = v[:, :, 2 - ky:4 - ky, 2 - kx:4 - kx].sum(axis=(2, 3))
    s = src.detach().numpy()
    Wn = W.detach().numpy().reshape(cout, cin, 9)
    dsrc = np.einsum("oct,tobyx->bcyx", Wn, D)
    np.testing.assert_allclose(dsrc, src.grad.numpy(), rtol=0, atol=1e-12)
    # weight gradient as rows (t cout + o), columns c, then the tap-major
    # permutation of k_sum_splits: (t cout + o) cin + c -> (o cin + c) 9 + t
    C = np.einsum("tobyx,bcyx->toc", D, s).reshape(-1)
    i = np.arange(C.size)
    tap, r = i // (cout * cin), i % (cout * cin)
    dW = np.empty_like(C)
    dW[r * 9 + tap] = C
    np.testing.assert_allclose(dW.reshape(cout, cin, 3, 3), W.grad.numpy(), rtol=0, atol=1e-12)


def test_stride2_input_gradient_as_phase_gemms():
    g = torch.Generator().manual_seed(3)
    B, cin, cout, Hi, Wi = 2, 5, 3, 8, 10
    x = torch.randn(B, cin, Hi, Wi, dtype=torch.float64, generator=g, requires_grad=True)
    W = torch.randn(cout, cin, 3, 3, dtype=torch.float64, generator=g)
    z = F.conv2d(x, W, stride=2, padding=1)
    Ho, Wo = z.shape[2:]
    dz = torch.randn(z.shape, dtype=torch.float64, generator=g)
    (z * dz).sum().backward()
    dzn, Wn = dz.numpy(), W.numpy()
    # E[(2 ey + ex) cout + o][s] = dz[o][y + ey][x + ex]
    E = np.zeros((4 * cout, B, Ho, Wo))
    for ey in range(2):
        for ex in range(2):
            for y in range(Ho):
                for xx in range(Wo):
                    if y + ey < Ho and xx + ex < Wo:
                        E[(2 * ey + ex) * cout:(2 * ey + ex + 1) * cout, :, y, xx] = dzn[:, :, y + ey, xx + ex].T
    E = E.reshape(4 * cout, -1)
    dx = np.zeros((cin, B, Hi, Wi))
    for q in range(4):
        a, b = q >> 1, q & 1
        nx = 1 + b
        Wd = np.zeros((cin, (1 + a) * nx * cout))
        for kk in range(Wd.shape[1]):
            e, o = divmod(kk, cout)
            ey, ex = divmod(e, nx)
            ky = 1 if a == 0 else (2 if ey == 0 else 0)
            kx = 1 if b == 0 else (2 if ex == 0 else 0)
            Wd[:, kk] = Wn[o, :, ky, kx]
        run, gap = (1 + b) * cout, (1 - b) * cout
        rows = [k + (gap if k >= run else 0) for k in range(Wd.shape[1])]
        dx[:, :, a::2, b::2] = (Wd @ E[rows]).reshape(cin, B, Ho, Wo)
    np.testing.assert_allclose(dx.transpose(1, 0, 2, 3), x.grad.numpy(), rtol=0, atol=1e-12)
