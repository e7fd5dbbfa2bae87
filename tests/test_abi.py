"""CPU checks of the C ABI: the library loads and exports every symbol the header declares;
the host record layouts match the header."""
import ctypes as ct
import os
import re

import numpy as np

from paper_2301_05451_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(tq_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2301_05451_amd import lib

    names = _declared()
    assert {"tq_sv_apply", "tq_expval", "tq_sv_backward", "tq_ctx_create"} <= names
    missing = [n for n in sorted(names) if not hasattr(lib.raw(), n)]
    assert not missing, missing


def test_record_layouts_match_header():
    from paper_2301_05451_amd import lib

    assert W.GATE_DTYPE.itemsize == 48 and W.GATE_DTYPE.fields["pscale"][1] == 24
    assert W.ZTERM_DTYPE.itemsize == 24
    assert ct.sizeof(lib.Batch) == 48
    assert ct.sizeof(lib.SvOpts) == 16


def test_version_and_empty_error():
    from paper_2301_05451_amd import lib

    assert lib.raw().tq_version() >= 100
    assert isinstance(lib.last_error(), str)


def test_ctx_create_fails_cleanly_without_gpu():
    import torch

    from paper_2301_05451_amd import lib

    if torch.cuda.is_available():
        return
    h = ct.c_void_p()
    st = lib.raw().tq_ctx_create(0, ct.byref(h))
    assert st != 0 and not h.value
    assert lib.last_error()


def test_batch_spec_packing():
    from paper_2301_05451_amd import lib

    rng = np.random.default_rng(0)
    cs = [W.random_circuit(n, 5, rng) for n in (3, 5, 4)]
    spec = lib.BatchSpec.from_circuits(cs)
    assert list(spec.state_off) == [0, 8, 40]
    assert spec.total_amps == 56
    assert list(spec.gate_off) == [0, 5, 10]
