"""The product path has no CPU fallback: without its HIP libraries every entry
raises, and the package never loads the FP64 oracle."""
import os
import subprocess
import sys

import pytest

import lbm_inputs as li

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_missing_library_raises(monkeypatch, tmp_path):
    from paper_1409_5929_amd import lbm, no

    monkeypatch.setattr(lbm, "LIB_PATH", str(tmp_path / "liblbm_axi.so"))
    monkeypatch.setattr(lbm, "_lib", None)
    with pytest.raises(RuntimeError, match="is missing"):
        lbm.Lattice(li.annulus(nr=16, nz=16))
    monkeypatch.setattr(no, "LIB_PATH", str(tmp_path / "liblbm_no.so"))
    monkeypatch.setattr(no, "_lib", None)
    with pytest.raises(no.NoError, match="is missing"):
        no._load()


def test_package_does_not_load_the_oracle():
    code = ("import sys, paper_1409_5929_amd, paper_1409_5929_amd.lbm, paper_1409_5929_amd.no, "
            "paper_1409_5929_amd.studies, paper_1409_5929_amd.warmstart\n"
            "bad = sorted(m for m in sys.modules if m == 'oracle' or m.startswith('oracle.'))\n"
            "assert not bad, bad\n")
    subprocess.run([sys.executable, "-c", code], cwd=ROOT, check=True, timeout=120)
    pkg = os.path.join(ROOT, "paper_1409_5929_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "lbm_oracle" not in text and "no_oracle" not in text, f
