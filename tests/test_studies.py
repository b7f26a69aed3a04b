"""Host-side pieces of the paper's validation runs (no GPU)."""
import pytest

import lbm_inputs as li
from paper_1409_5929_amd import studies


@pytest.mark.parametrize("cfg", [li.heater_annulus(Da=1e-4, nr=40, nz=40),
                                 li.heater_annulus(Da=1e-2, nr=200, nz=200),
                                 li.table2(1e4)])
def test_psi_scale_is_the_oracles_thermal_diffusivity(oracle_mod, cfg):
    """Table 3's |psi|max is reported in units of alpha_e L with
    alpha_e = c_sT^2 tau_T, which the study takes from the library
    (lbm_axi_derived); it must equal the oracle's, and so must the library's
    other derived constants (Eqs. 9, 31, 39)."""
    from paper_1409_5929_amd import lbm

    o = oracle_mod.Oracle(dict(cfg, nr=8, nz=8) if cfg["nr"] > 8 else cfg)
    ref = o.derived()
    o.close()
    assert studies.alpha_e(cfg) == pytest.approx(0.2 * ref["tau_T"], rel=1e-14)
    got = lbm.derived(cfg)
    for k in ("tau_nu", "tau_T", "nu_e", "nu", "K_ref", "gbeta"):
        assert got[k] == pytest.approx(ref[k], rel=1e-14, abs=1e-300), k


def test_cli_refuses_unknown_cases():
    with pytest.raises(SystemExit):
        studies.main(["table9"])
