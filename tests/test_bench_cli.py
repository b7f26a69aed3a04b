"""bench.py's command line on the host: more than one GPU is refused with a
message, before anything touches a device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], capture_output=True,
                       text=True, timeout=120, cwd=ROOT, env=env)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr


def _undefined_globals(path):
    """Names that a function of the file reads as globals but that neither the
    module (imports, definitions, assignments) nor the builtins define."""
    import builtins
    import symtable

    src = open(path).read()
    top = symtable.symtable(src, path, "exec")
    defined = set(dir(builtins)) | {"__file__", "__name__", "__doc__", "__spec__", "__path__"}
    defined |= {s.get_name() for s in top.get_symbols()
                                    if s.is_assigned() or s.is_imported()}
    missing = []

    def walk(t):
        for s in t.get_symbols():
            if t.get_type() == "function" and s.is_referenced() and s.is_global() and not s.is_declared_global():
                if s.get_name() not in defined:
                    missing.append(f"{t.get_name()}: {s.get_name()}")
        for c in t.get_children():
            walk(c)

    walk(top)
    return missing


@pytest.mark.parametrize("rel", ["bench.py", "__graft_entry__.py", "paper_1409_5929_amd/lbm.py",
                                 "paper_1409_5929_amd/no.py", "paper_1409_5929_amd/warmstart.py",
                                 "paper_1409_5929_amd/studies.py", "lbm_inputs/__init__.py"])
def test_no_function_reads_an_undefined_global(rel):
    """A function that calls a name nothing defines fails only when that line
    runs, which for bench.py is on the GPU after minutes of work."""
    assert _undefined_globals(os.path.join(ROOT, rel)) == []
