"""Register resources of the step kernels, read from the built library's own
code objects (the AMDGPU metadata notes of each gfx950 code object; no GPU):
* no FP32 step kernel uses scratch (no register spills);
* every 16-bit step kernel fits four waves per SIMD (at most 128 VGPRs, the
  occupancy the 16-bit kernels ask for);
* the buffer-addressed 16-bit plain step kernels, which run every population
  array below 4 GiB (the single-grid runs and the batched sweep), use no
  scratch, with and without wall lanes.
Template arguments are read from the mangled kernel names:
k_step<storage, ODD, MODE (0 step, 1 step with macroscopic output, 2 fields),
BUF (buffer addressing), WL (wall lanes)>.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1409_5929_amd", "liblbm_axi.so")
LLVM = os.environ.get("ROCM_LLVM_BIN", "/opt/rocm/llvm/bin")
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
STEP = re.compile(r"k_stepI(6__half|14__hip_bfloat16|f)Lb([01])ELi([012])ELb([01])ELb([01])E")
TYPES = {"f": "fp32", "6__half": "fp16", "14__hip_bfloat16": "bf16"}


def _parse_notes(text):
    """Kernel name -> its metadata fields (the fields that follow .name)."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.match(r"\s+-?\s*\.(\w+):\s+(\S+)", line)
        if not m:
            continue
        key, val = m.groups()
        if key == "name" and val.startswith("_Z"):
            cur = out.setdefault(val, {})
        elif cur is not None and key in ("private_segment_fixed_size", "vgpr_count", "vgpr_spill_count"):
            cur.setdefault(key, int(val))
    return out


@pytest.fixture(scope="module")
def step_kernels(tmp_path_factory):
    if not os.path.exists(LIB):
        pytest.skip("liblbm_axi.so not built (run __graft_entry__.build())")
    tools = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
    if not all(os.path.exists(t) for t in tools):
        pytest.skip("ROCm LLVM tools not found")
    d = tmp_path_factory.mktemp("codeobj")
    fat = d / "fatbin"
    subprocess.check_call([tools[0], f"--dump-section=.hip_fatbin={fat}", LIB, str(d / "lib.so")])
    data = fat.read_bytes()
    # one offload bundle per translation unit (FP32 and 16-bit kernels)
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)]
    assert starts and starts[0] == 0
    kernels = {}
    for n, s in enumerate(starts):
        part, co = d / f"bundle{n}", d / f"co{n}"
        part.write_bytes(data[s:])
        subprocess.check_call([tools[1], "--type=o", f"--targets={TARGET}", f"--input={part}",
                               f"--output={co}", "--unbundle"])
        kernels.update(_parse_notes(subprocess.check_output([tools[2], "--notes", str(co)], text=True)))
    steps = {}
    for name, meta in kernels.items():
        m = STEP.search(name)
        if m:
            t, odd, mode, buf, wl = m.groups()
            steps[(TYPES[t], int(odd), int(mode), int(buf), int(wl))] = meta
    return steps


def test_every_plain_step_variant_is_in_the_library(step_kernels):
    for odd in (0, 1):
        for wl in (0, 1):
            assert ("fp32", odd, 0, 0, wl) in step_kernels
            for t in ("fp16", "bf16"):
                assert (t, odd, 0, 1, wl) in step_kernels
                assert (t, odd, 0, 0, wl) in step_kernels


def test_fp32_step_kernels_do_not_spill(step_kernels):
    fp32 = {k: v for k, v in step_kernels.items() if k[0] == "fp32"}
    assert fp32
    for k, v in fp32.items():
        assert v["private_segment_fixed_size"] == 0 and v.get("vgpr_spill_count", 0) == 0, (k, v)


def test_16_bit_step_kernels_fit_four_waves_per_simd(step_kernels):
    s16 = {k: v for k, v in step_kernels.items() if k[0] != "fp32"}
    assert s16
    for k, v in s16.items():
        assert v["vgpr_count"] <= 128, (k, v)


def test_buffer_addressed_16_bit_plain_steps_do_not_spill(step_kernels):
    for k, v in step_kernels.items():
        if k[0] != "fp32" and k[2] == 0 and k[3] == 1:
            assert v["private_segment_fixed_size"] == 0 and v.get("vgpr_spill_count", 0) == 0, (k, v)
