"""CPU regression guard on the generated gfx950 code: no scalar memory load may use an
immediate offset that is not a multiple of 4. The scalar unit drops the low address bits
of its operands, so a misaligned base/offset split reads the wrong dword (a descriptor
field read this way once returned the op header as a matrix index and the load left its
buffer)."""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2301_05451_amd", "csrc")
SMEM = re.compile(r"\b(s_load_\w+|s_buffer_load\w*)\s+s\[?[\d:]+\]?,\s*s\[[\d:]+\],\s*(0x[0-9a-f]+|\d+)\s*$")


def _sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


@pytest.mark.parametrize("src", _sources())
def test_no_misaligned_scalar_loads(src):
    from paper_2301_05451_amd import build as b

    with tempfile.TemporaryDirectory() as d:
        cmd = [b.hipcc(), *b.FLAGS, "-S", "--cuda-device-only", os.path.join(CSRC, src), "-o",
               os.path.join(d, "out.s")]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        bad, kern = [], None
        for line in open(os.path.join(d, "out.s")):
            m = re.match(r"^(_Z\S+):", line)
            if m:
                kern = m.group(1)
            m = SMEM.search(line)
            if m and int(m.group(2), 0) % 4:
                bad.append((kern, line.strip()))
        assert not bad, bad[:5]


# Register-resident tiles: the fused stage kernels keep every amplitude in registers; a
# private (scratch) segment means an array was demoted to memory, a several-fold slowdown.
NO_SCRATCH = [
    ("sv_kernels.hip", r"_ZN2tq15sv_stage_kernelI[fd]Li[1-4]E"),
    ("sv_kernels.hip", r"_ZN2tq21sv_batch_stage_kernelI[fd]Li[1-4]E"),
    ("sv_adjoint.hip", r"_ZN2tq16adj_stage_kernelIfLi[1-4]E"),
    ("sv_adjoint.hip", r"_ZN2tq16adj_stage_kernelIdLi[1-3]E"),
]


@pytest.mark.parametrize("src,pattern", NO_SCRATCH)
def test_stage_kernels_use_no_scratch(src, pattern):
    from paper_2301_05451_amd import build as b

    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "out.s")
        r = subprocess.run([b.hipcc(), *b.FLAGS, "-S", "--cuda-device-only", os.path.join(CSRC, src), "-o", out],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        text = open(out).read()
        seen = 0
        for blk in text.split(".agpr_count")[1:]:
            name = re.search(r"\.name:\s+(\S+)", blk)
            if not name or not re.match(pattern, name.group(1)):
                continue
            seen += 1
            priv = int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", blk).group(1))
            assert priv == 0, (name.group(1), priv)
        assert seen > 0
