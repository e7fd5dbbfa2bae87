"""CPU regression guard on the generated gfx950 code: no scalar memory load may use an
immediate offset that is not a multiple of 4. The scalar unit drops the low address bits
of its operands, so a misaligned base/offset split reads the wrong dword (a descriptor
field read this way once returned the op header as a matrix index and the load left its
buffer)."""
import concurrent.futures as cf
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


@pytest.fixture(scope="module")
def device_asm():
    """gfx950 assembly of every source, compiled once (in parallel) for all checks here."""
    from paper_2301_05451_amd import build as b

    with tempfile.TemporaryDirectory() as d:
        def one(src):
            out = os.path.join(d, src + ".s")
            r = subprocess.run([b.hipcc(), *b.FLAGS, "-S", "--cuda-device-only", os.path.join(CSRC, src), "-o", out],
                               capture_output=True, text=True)
            return src, (open(out).read() if r.returncode == 0 else None), r.stderr[-2000:]

        srcs = _sources()
        with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
            yield {src: (text, err) for src, text, err in ex.map(one, srcs)}


def _asm(device_asm, src):
    text, err = device_asm[src]
    assert text is not None, err
    return text


@pytest.mark.parametrize("src", _sources())
def test_no_misaligned_scalar_loads(src, device_asm):
    bad, kern = [], None
    for line in _asm(device_asm, src).splitlines():
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
    ("sv_kernels.hip", r"_ZN2tq19sv_stage_kernel_t12I[fd]Li[1-4]E"),
    ("sv_kernels.hip", r"_ZN2tq(15sv_stage_kernel|19sv_stage_kernel_t12|21sv_batch_stage_kernel)IfLi5E"),
    ("sv_kernels.hip", r"_ZN2tq21sv_batch_stage_kernelI[fd]Li[1-4]E"),
    ("sv_adjoint.hip", r"_ZN2tq16adj_stage_kernelIfLi[1-4]E"),
    ("sv_adjoint.hip", r"_ZN2tq16adj_stage_kernelIdLi[1-3]E"),
]


@pytest.mark.parametrize("src,pattern", NO_SCRATCH)
def test_stage_kernels_use_no_scratch(src, pattern, device_asm):
    seen = 0
    for blk in _asm(device_asm, src).split(".agpr_count")[1:]:
        name = re.search(r"\.name:\s+(\S+)", blk)
        if not name or not re.match(pattern, name.group(1)):
            continue
        seen += 1
        priv = int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", blk).group(1))
        assert priv == 0, (name.group(1), priv)
    assert seen > 0
