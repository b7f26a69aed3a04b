"""bench.py on the host: more than one GPU is refused with a message, before
anything touches a device; every function's globals are defined; the counter
traffic on the bench line is tied to the kernel source it was measured on."""
import json
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


def test_traffic_is_reported_only_for_the_kernel_source_it_was_taken_on(tmp_path, monkeypatch):
    """The counter traffic on the bench line belongs to the kernel source it
    was measured on: the same bytes while the hash of the kernel sources
    matches the file's, none once a source differs."""
    sys.path.insert(0, ROOT)
    import bench

    srcs = []
    for i, p in enumerate(bench.KERNEL_SOURCES):
        q = tmp_path / f"src{i}"
        q.write_bytes(open(p, "rb").read())
        srcs.append(str(q))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", srcs)
    record = {"source_sha": bench.kernel_source_sha(), "note": "test",
              "fp32": {"bytes_per_launch": 123}, "fp16": {"bytes_per_launch": 45}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(record))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("fp32") == 123 and bench.measured_traffic("fp16") == 45
    assert bench.measured_traffic("bf16") is None
    with open(srcs[-1], "ab") as g:
        g.write(b"\n// changed\n")
    assert bench.measured_traffic("fp32") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("fp32") is None
