"""The learned warm start: the committed network (trained by
paper_1409_5929_amd.warmstart on steady fields of the solver itself) against
its FP64 oracle, and what its prediction gains over a cold start on held-out
problems of the sweep distribution (128^2, run to res <= 1e-8)."""
import numpy as np
import pytest

import lbm_inputs as li
from oracle import no_oracle as N

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1409_5929_amd import warmstart

    return warmstart


def test_trained_network_matches_oracle(ws):
    """bf16 GEMMs against FP64 on the trained weights, measured on the start
    fields the solver receives.  The trained output is a small correction
    (to the conduction profile) computed from much larger hidden activations,
    so the bf16 rounding error (3e-2 of the activations, as in the network
    tests) is stated against the fields: T in relative L2, the velocity in
    units of the characteristic velocity U = Ma c_s (rms)."""
    import torch

    from paper_1409_5929_amd.no import WarmStartNet

    params = ws.load_weights(ws.WEIGHTS)
    cfg = ws.held_out(41)[40]
    x = li.no_features(cfg)[None]
    net = WarmStartNet(ws.WIDTHS, ws.GRID, ws.GRID, 1, params)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    net.close()
    ref, _ = N.forward(params.astype(np.float64), ws.WIDTHS, x.astype(np.float64))
    fg, fr = li.no_fields(y[0], cfg), li.no_fields(ref[0].astype(np.float32), cfg)
    eT = np.linalg.norm(fg[2] - fr[2]) / np.linalg.norm(fr[2])
    eu = np.sqrt(np.mean((fg[0] - fr[0]) ** 2 + (fg[1] - fr[1]) ** 2)) / li.U_SCALE
    eo = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"trained network vs oracle: output rel L2 {eo:.2e}; start T rel L2 {eT:.2e}, "
          f"u rms / U {eu:.2e}", flush=True)
    assert eT <= 3e-2 and eu <= 3e-2


def test_learned_start_beats_the_conduction_start(ws):
    """64 held-out problems from the cold start, the network's start and the
    non-learned conduction-profile start, each to the warm-start stopping rule
    (res <= 1e-8 and extrapolated remaining change <= 1e-4).  Over the
    problems that converge from all three: the learned start takes fewer
    steps in total than the conduction start (and than the cold start), and
    every problem's Nu_i lies within 1e-3 of the cold start's, from both."""
    from paper_1409_5929_amd.no import WarmStartNet

    cfgs = ws.held_out(64)
    net = WarmStartNet(ws.WIDTHS, ws.GRID, ws.GRID, 32, ws.load_weights(ws.WEIGHTS))
    pred = ws.predict(net, cfgs)
    net.close()
    assert np.isfinite(pred).all()
    cold = ws.solve(cfgs, max_steps=600_000, fields=False)
    warm = ws.solve(cfgs, init=list(pred), max_steps=600_000, fields=False)
    cond = ws.solve(cfgs, init=[ws.conduction_start(c) for c in cfgs], max_steps=600_000, fields=False)
    ok = (cold["status"] == 1) & (warm["status"] == 1) & (cond["status"] == 1)
    wc, dc, wd = ws.compare(cold, warm, ok), ws.compare(cold, cond, ok), ws.compare(cond, warm, ok)
    print(f"converged cold/warm/conduction {int((cold['status'] == 1).sum())}/"
          f"{int((warm['status'] == 1).sum())}/{int((cond['status'] == 1).sum())} of {len(cfgs)}; "
          f"warm vs cold {wc}; conduction vs cold {dc}; warm vs conduction {wd}", flush=True)
    assert ok.sum() >= 32
    assert wd["steps_ratio_total"] < 1.0
    assert wc["steps_ratio_total"] < 1.0
    assert wc["nu_rel_diff_max"] <= 1e-3 and dc["nu_rel_diff_max"] <= 1e-3
