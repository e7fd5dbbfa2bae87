"""Benchmark of the state-vector hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): a 24-qubit state-vector
circuit of 20 brickwork layers (RX, RY, RZ on every qubit with angles U[0, 2pi), then CZ on
alternating neighbour pairs), 1670 gates, complex64 (2^24 amplitudes, 128 MiB), observable
sum_i Z_i, batch 1. One step = |0..0> preparation + every gate (fused LDS-tile sweeps) +
the expectation value, all in libtq kernels, inputs resident in HBM.

Prints one JSON line. ``value`` is gates*amps/s = 1670 * 2^24 / seconds per step.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2301_05451_amd  # noqa: E402,F401  (pins the system HIP runtime before torch loads)

METRIC = "gates·amps/s (HBM % peak), TN GFLOP/s (MFMA %), grad circuits/s at ≤1e-5 err"
HBM_PEAK_GBS = 8000.0
# Non-packed FP32 VALU: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
ALU_PEAK_PUBLISHED_TFLOPS = 157.3


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(c, seconds_hint=True):
    """The oracle (complex128 numpy) on a bounded sample: the first brickwork layer (84 of
    the 1670 gates) on the full 24-qubit register, scaled to gates*amps/s."""
    from oracle import sv as osv

    sample = c.gates[:84]
    t0 = time.perf_counter()
    osv.run(c.n, sample, c.params)
    dt = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS")
    return {"value": len(sample) * (1 << c.n) / dt, "unit": "gate*amps/s",
            "cores": int(threads) if threads and threads.isdigit() else os.cpu_count(),
            "kind": "oracle",
            "sample": f"first brickwork layer ({len(sample)} gates) of the 24-qubit circuit, complex128, "
                      f"{dt:.1f} s on {cpu_model()} (numpy tensordot per gate)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--plain-steps", type=int, default=1, help="steps of the one-sweep-per-gate path")
    ap.add_argument("--tile-bits", type=int, default=0)
    ap.add_argument("--reg-bits", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2301_05451_amd import lib
    from paper_2301_05451_amd import workloads as W

    c = W.brickwork()
    n, G = c.n, c.gates.shape[0]
    spec = lib.BatchSpec.uniform(n, c.gates, 1, c.n_params)
    params = torch.tensor(c.params, dtype=torch.float32, device="cuda")
    psi = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    opts = dict(tile_bits=args.tile_bits, reg_bits=args.reg_bits)
    info = lib.plan_info(n, c.gates, mode=0, **opts)

    def step():
        lib.init_states(psi, spec, 0)
        lib.sv_apply(psi, params, spec, mode=0, **opts)
        return lib.expval(psi, spec, c.terms, 1)

    for _ in range(args.warmup):
        f = step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_start.record()
    for k in range(args.steps):
        lib.init_states(psi, spec, 0)
        ev[k][0].record()
        lib.sv_apply(psi, params, spec, mode=0, **opts)
        ev[k][1].record()
        f = lib.expval(psi, spec, c.terms, 1)
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    apply_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    value = G * (1 << n) / (wall / args.steps)

    # dominant kernel: the fused stage sweep. One launch moves 2 x 2^n x 8 bytes and does
    # flops_per_amp(stage) x 2^n flops; averaged over the circuit's stages.
    stages = info["sweeps"]
    stage_ms = apply_ms / stages  # includes the one small gate-build launch per call
    bytes_per_stage = 2 * (1 << n) * 8
    flops_per_stage = info["flops_per_amp"] * (1 << n) / stages
    gbs = bytes_per_stage / (stage_ms * 1e-3) / 1e9
    tflops = flops_per_stage / (stage_ms * 1e-3) / 1e12
    t_hbm = bytes_per_stage / (HBM_PEAK_GBS * 1e9)
    t_alu = flops_per_stage / (ALU_PEAK_TFLOPS * 1e12)
    if t_alu >= t_hbm:
        roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": round(ALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                "frac": round(tflops / ALU_PEAK_TFLOPS, 4), "traffic": None,
                "peak_published_fp32_vector": ALU_PEAK_PUBLISHED_TFLOPS,
                "hbm_achieved_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
    roof.update({"kernel": "sv_stage_kernel<float,%d>" % info["reg_bits"], "launches_per_step": stages,
                 "avg_launch_us": round(stage_ms * 1e3, 2)})

    # the plain path (one HBM sweep per gate) on the same circuit, for comparison
    plain = None
    if args.plain_steps > 0:
        pinfo = lib.plan_info(n, c.gates, mode=1)
        lib.init_states(psi, spec, 0)
        lib.sv_apply(psi, params, spec, mode=1)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.plain_steps):
            lib.init_states(psi, spec, 0)
            lib.sv_apply(psi, params, spec, mode=1)
            fp = lib.expval(psi, spec, c.terms, 1)
        b.record()
        torch.cuda.synchronize()
        pms = a.elapsed_time(b) / args.plain_steps
        plain = {"gate*amps/s": G * (1 << n) / (pms * 1e-3), "ms_per_step": round(pms, 3),
                 "sweeps": pinfo["sweeps"],
                 "avg_sweep_GBs": round(pinfo["sweeps"] * bytes_per_stage / (pms * 1e-3) / 1e9, 1),
                 "expval_agrees": bool(abs(float(fp[0, 0]) - float(f[0, 0])) < 1e-4)}

    out = {
        "metric": METRIC, "value": value, "unit": "gate*amps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "24-qubit brickwork state-vector circuit: 20 layers of RX,RY,RZ on all qubits "
                               "+ CZ on alternating neighbour pairs (1670 gates), complex64, sum_i Z_i, batch 1",
                   "qubits": n, "gates": G, "fused_sweeps": stages, "tile_bits": info["tile_bits"],
                   "reg_bits": info["reg_bits"]},
        "roofline": roof,
        "expval_sum_z": float(f[0, 0]),
        "plain": plain,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(c)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
