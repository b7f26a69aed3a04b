"""Host-side pieces of the paper's validation runs (no GPU)."""
import pytest

import lbm_inputs as li
from paper_1409_5929_amd import studies


@pytest.mark.parametrize("cfg", [li.heater_annulus(Da=1e-4, nr=40, nz=40),
                                 li.heater_annulus(Da=1e-2, nr=200, nz=200),
                                 li.table2(1e4)])
def test_psi_scale_is_the_oracles_thermal_diffusivity(oracle_mod, cfg):
    """Table 3's |psi|max is reported in units of alpha_e L with
    alpha_e = c_sT^2 tau_T; the study's Eq. (39) must give the oracle's tau_T."""
    o = oracle_mod.Oracle(dict(cfg, nr=8, nz=8) if cfg["nr"] > 8 else cfg)
    tau_T = o.derived()["tau_T"]
    o.close()
    assert studies.alpha_e(cfg) == pytest.approx(0.2 * tau_T, rel=1e-14)


def test_cli_refuses_unknown_cases():
    with pytest.raises(SystemExit):
        studies.main(["table9"])
