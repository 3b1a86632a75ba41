"""Device-code guards, checked on the gfx950 assembly that hipcc emits for
every HIP source (no GPU needed):

* no indexed register moves (``s_set_gpr_idx_on`` / ``v_movrel*``): a register
  array indexed by a run-time value compiles to them, and the compiler may
  execute such a write speculatively, for an index that the source guards out,
  onto registers past the array;
* no private (scratch) segment: every kernel keeps its per-lane state in
  registers;
* no packed-FP32 instructions (the library is built without them).
"""

import os
import re
import subprocess

import pytest

from paper_2506_04976_amd import build as petbuild

HIP_SOURCES = [s for s in petbuild.SOURCES if s.endswith(".hip")]


@pytest.fixture(scope="module")
def assembly(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = {}
    d = tmp_path_factory.mktemp("asm")
    for src in HIP_SOURCES:
        s_file = str(d / (src + ".s"))
        flags = [f for f in petbuild.FLAGS if f not in ("-fPIC", "-shared")]
        cmd = [hipcc] + flags + ["-S", "--cuda-device-only", "-o", s_file, os.path.join(petbuild.CSRC, src)]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-2000:]
        with open(s_file) as f:
            out[src] = f.read()
    return out


def _kernels(text):
    """(name, body) of each kernel in an assembly listing."""
    names = re.findall(r"^(_Z\S+):", text, flags=re.M)
    parts = re.split(r"^_Z\S+:.*$", text, flags=re.M)[1:]
    return list(zip(names, parts))


@pytest.mark.parametrize("src", HIP_SOURCES)
def test_no_indexed_register_moves(assembly, src):
    bad = [name for name, body in _kernels(assembly[src]) if re.search(r"s_set_gpr_idx_on|v_movrel", body)]
    assert not bad, f"{src}: run-time register indexing in {bad}"


@pytest.mark.parametrize("src", HIP_SOURCES)
def test_no_scratch_and_no_packed_fp32(assembly, src):
    text = assembly[src]
    sizes = [int(v) for v in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", text)]
    assert sizes and max(sizes) == 0, f"{src}: scratch in use"
    assert not re.search(r"v_pk_(add|mul|fma)_f32", text), f"{src}: packed FP32 instruction"
