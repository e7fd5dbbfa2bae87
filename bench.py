"""Benchmark of the state-vector hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): a 24-qubit state-vector
circuit of 20 brickwork layers (RX, RY, RZ on every qubit with angles U[0, 2pi), then CZ on
alternating neighbour pairs), 1670 gates, complex64 (2^24 amplitudes, 128 MiB), observable
sum_i Z_i, batch 1. One step = |0..0> preparation + every gate (fused LDS-tile sweeps; the
first one forms |0..0> itself, tq_sv_run) + the expectation value, all in libtq kernels,
inputs resident in HBM.

Prints one JSON line. ``value`` is gates*amps/s = 1670 * 2^24 / seconds per step.
"""
import argparse
import json
import math
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


def cpu_threads():
    """Threads the oracle's numpy can use: the BLAS pools' sizes (threadpoolctl), else 1."""
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        return max([int(p.get("num_threads", 1)) for p in info] + [1])
    except Exception:
        return 1


def cpu_baseline(c, seconds_hint=True):
    """The oracle (complex128 numpy) on a bounded sample: the first three brickwork layers
    (251 of the 1670 gates, about 10-15 s) on the full 24-qubit register, scaled to
    gates*amps/s."""
    from oracle import sv as osv

    sample = c.gates[:251]
    t0 = time.perf_counter()
    osv.run(c.n, sample, c.params)
    dt = time.perf_counter() - t0
    return {"value": len(sample) * (1 << c.n) / dt, "unit": "gate*amps/s",
            "cores": cpu_threads(), "kind": "oracle",
            "sample": f"first three brickwork layers ({len(sample)} gates) of the 24-qubit circuit, complex128, "
                      f"{dt:.1f} s on {cpu_model()} (numpy tensordot per gate; elementwise work runs on one "
                      f"core, the tensordot products on the BLAS threads)"}


def cpu_plan():
    """The oracle timed on every workload (the CPU-baseline plan), bounded samples stated per
    entry; wall times with time.perf_counter. Long: minutes (the whole 24-qubit circuit)."""
    import numpy as np

    from oracle import sv as osv
    from oracle import tn as otn
    from paper_2301_05451_amd import workloads as W

    def log(m):
        print("cpu-plan: " + m, file=sys.stderr, flush=True)

    out = {"cpu": cpu_model(), "os_cpu_count": os.cpu_count(), "blas_threads": cpu_threads(),
           "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}
    c1 = W.hea_ring()
    t0 = time.perf_counter()
    osv.circuit_f(c1)
    out["hea10_s_per_circuit"] = time.perf_counter() - t0
    c2 = W.brickwork()
    t0 = time.perf_counter()
    psi = osv.initial_state(c2.n).reshape((2,) * c2.n)
    for k in range(0, len(c2.gates), 84):  # the whole circuit, in chunks (progress lines)
        psi = osv.run(c2.n, c2.gates[k:k + 84], c2.params, init=psi.reshape(-1)).reshape((2,) * c2.n)
        log(f"brickwork24 {min(k + 84, len(c2.gates))}/{len(c2.gates)} gates, {time.perf_counter() - t0:.0f} s")
    dt = time.perf_counter() - t0
    out["brickwork24_full_s"] = dt
    out["brickwork24_gate_amps_per_s"] = len(c2.gates) * (1 << c2.n) / dt
    del psi
    gates, x, theta, y = W.qnn_batch()
    n = 16
    t0 = time.perf_counter()
    for b in range(32):
        osv.circuit_f(W.Circuit(n, gates, np.concatenate([x[b], theta]), 1, W.zterms([([0], 1.0, 0)])))
    fwd = (time.perf_counter() - t0) / 32
    cb = W.Circuit(n, gates, np.concatenate([x[0], theta]), 1, W.zterms([([0], 1.0, 0)]))
    t0 = time.perf_counter()
    for p in range(0, 272, 17):  # 16 of the 272 parameters, two shifted circuits each
        for sft in (np.pi / 2, -np.pi / 2):
            pp = cb.params.copy()
            pp[p] += sft
            osv.circuit_f(cb, pp)
    ps = (time.perf_counter() - t0) / 16
    out["qnn16"] = {"forward_s_per_sample": fwd, "forward_512_s_extrapolated": fwd * 512,
                    "param_shift_s_per_parameter": ps, "param_shift_s_per_sample_extrapolated": ps * 272,
                    "sample": "forward of 32 of the 512 samples; parameter shift of 16 of 272 parameters of one sample"}
    log("qnn16 done")
    circs = W.uneven_batch()
    per_n = {}
    for nq in range(8, 21):
        sel = [cc for cc in circs if cc.n == nq][:2]
        t0 = time.perf_counter()
        for cc in sel:
            osv.circuit_f(cc)
        per_n[nq] = (time.perf_counter() - t0) / max(1, len(sel))
        log(f"uneven n={nq}: {per_n[nq]:.2f} s per circuit")
    hist = {nq: sum(1 for cc in circs if cc.n == nq) for nq in range(8, 21)}
    out["uneven1024"] = {"s_per_circuit_by_n": per_n,
                         "forward_s_extrapolated": sum(per_n[k] * hist[k] for k in per_n),
                         "sample": "2 circuits per qubit count, forward only; total extrapolated to the batch's n histogram"}
    prob3 = W.qaoa_maxcut(p=3)
    cones = sorted((len(otn.qaoa_cone(prob3, e)[3]), e) for e in prob3.edges)
    small = [e for sz, e in cones if sz <= 24]
    t0 = time.perf_counter()
    for e in small:
        otn.qaoa_edge_zz_sv(prob3, e)
    cone_sv = (time.perf_counter() - t0) / max(1, len(small))
    t0 = time.perf_counter()
    for _, e in cones[:4]:
        otn.qaoa_edge_zz_tn(prob3, e)
    tn4 = (time.perf_counter() - t0) / 4
    out["qaoa50"] = {"p3_cone_sv_s_per_network": cone_sv, "p3_cone_sv_networks": len(small),
                     "p3_einsum_tn_s_per_network": tn4,
                     "sample": "QAOA p=3 (cones of 19-30 qubits): cone state vector for the cones of at most 24 "
                               "qubits, the oracle's einsum network for the 4 smallest cones. At p=4 every cone "
                               "has 30 or more qubits (a 16 GiB complex128 state) and the einsum order does not "
                               "finish within minutes, so p=4 is not timed on the CPU."}
    log("qaoa done")
    return out


def measured_traffic():
    """HBM bytes per stage-kernel launch from the committed rocprofv3 counter summary, if
    the kernel sources still hash to what was profiled (else None: the counters are stale)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "sv_stage_brickwork24_c64_hbm_counters.txt")
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(("traffic_", "source_")))
    srcs = ["paper_2301_05451_amd/csrc/sv_kernels.hip", "paper_2301_05451_amd/csrc/sv_device.h",
            "paper_2301_05451_amd/csrc/schedule.hip", "paper_2301_05451_amd/csrc/tq_internal.h"]
    h = hashlib.sha256()
    for f in srcs:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if vals.get("source_sha256", "").strip() != h.hexdigest():
        return None
    return int(vals["traffic_bytes_per_launch"])


def _timed(fn, steps, warmup):
    """Mean milliseconds of fn() over `steps` calls after `warmup` calls (HIP events on the
    current stream, which every libtq call here is launched on)."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


PEAKS = {}


def measure_peaks(reps=5):
    """Attainable peaks of this device from libtq's fixed probe kernels (tq_peak_probe): best of
    `reps` timings with HIP events on the launch stream, of one launch (the 8 GiB buffers and the
    compute probes, milliseconds each) or of 20 back-to-back launches (the state-sized buffers,
    tens of microseconds each, as the state kernels run). The 8 GiB stream
    copy and read are far beyond the L2 and the 256 MiB last-level cache, so they measure HBM.
    The 256 MiB copy and the 128 MiB read have the footprint of a 2^24-amplitude complex64
    state: data of that size stays partly in the last-level cache between passes, which is
    what the state kernels see."""
    import torch

    from paper_2301_05451_amd import lib

    def best(kind, buf, iters=1, launches=1):
        w = lib.peak_probe(kind, buf, iters)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(launches):
                w = lib.peak_probe(kind, buf, iters)
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b) / launches)
        return w / (min(ms) * 1e-3), min(ms)

    big = torch.zeros(8 << 30, dtype=torch.uint8, device="cuda")
    hbm_copy, hbm_copy_ms = best(lib.PEAK_COPY, big)
    hbm_read, hbm_read_ms = best(lib.PEAK_READ, big)
    del big
    torch.cuda.empty_cache()
    st = torch.zeros(1 << 28, dtype=torch.uint8, device="cuda")
    st_copy, st_copy_ms = best(lib.PEAK_COPY, st, launches=20)
    st_read, st_read_ms = best(lib.PEAK_READ, st[: 1 << 27], launches=20)
    del st
    out = torch.zeros(2048 * 256 * 8, dtype=torch.uint8, device="cuda")
    fma, fma_ms = best(lib.PEAK_FP32_FMA, out, 32768)
    m32, m32_ms = best(lib.PEAK_FP32_MFMA, out, 4096)
    m64, m64_ms = best(lib.PEAK_FP64_MFMA, out, 2048)
    del out
    torch.cuda.synchronize()
    PEAKS.update({"hbm_copy_GBs": hbm_copy / 1e9, "hbm_read_GBs": hbm_read / 1e9, "state_copy_GBs": st_copy / 1e9,
                  "state_read_GBs": st_read / 1e9, "fp32_fma_TFLOPs": fma / 1e12, "fp32_mfma_TFLOPs": m32 / 1e12,
                  "fp64_mfma_TFLOPs": m64 / 1e12})

    def bw(v, ms):
        return {"GBs": round(v / 1e9, 1), "frac_of_datasheet": round(v / 1e9 / HBM_PEAK_GBS, 4), "ms": round(ms, 3)}

    def fl(v, ms, sheet):
        return {"TFLOPs": round(v / 1e12, 2), "datasheet": round(sheet, 1),
                "frac_of_datasheet": round(v / 1e12 / sheet, 4), "ms": round(ms, 3)}

    return {
        "method": "libtq probe kernels (tq_peak_probe), best of %d timings (HIP events) of one launch, or of "
                  "20 back-to-back launches for the state-sized buffers" % reps,
        "hbm_copy_8GiB": bw(hbm_copy, hbm_copy_ms),
        "hbm_read_8GiB": bw(hbm_read, hbm_read_ms),
        "copy_256MiB_state_footprint": bw(st_copy, st_copy_ms),
        "read_128MiB_state": bw(st_read, st_read_ms),
        "fp32_fma_nonpacked": fl(fma, fma_ms, ALU_PEAK_TFLOPS),
        "fp32_mfma_16x16x4": fl(m32, m32_ms, 157.3),
        "fp64_mfma_16x16x4": fl(m64, m64_ms, 78.6),
    }


def _mfrac(achieved, key):
    """achieved / the measured attainable peak `key` (same unit), or None when not measured."""
    v = PEAKS.get(key)
    return round(achieved / v, 4) if v else None


def bench_qnn(steps):
    """16-qubit, 8-layer QNN over 512 samples (angle-encoded inputs, shared weights), MSE loss
    on <Z0>: one training step = compiled-batch forward + loss gradient + adjoint backward,
    replayed as HIP graphs. Compared with the GPU parameter-shift rule and with a loop of
    single-circuit calls, on the same device."""
    import numpy as np
    import torch

    from paper_2301_05451_amd import lib, sv
    from paper_2301_05451_amd import workloads as W

    n, B = 16, 512
    gates, x, theta, y = W.qnn_batch(n=n, layers=8, batch=B, seed=1003)
    P = n + theta.shape[0]
    pb = np.concatenate([x, np.broadcast_to(theta, (B, theta.shape[0]))], 1)
    spec = lib.BatchSpec.uniform(n, gates, B, P)
    terms = W.zterms([([0], 1.0, 0)])
    params = torch.tensor(pb.reshape(-1), dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")[:, None]
    svb = lib.SVBatch(spec, terms, 1, graph=True)
    states = svb.new_states()
    out = torch.empty(B, 1, device="cuda")
    w = torch.empty(B, 1, device="cuda")
    grad = torch.zeros_like(params)
    # shapes (tile and register bits) of both passes chosen by the autotuner, on the device
    tuned_f = svb.autotune(params, states, which=0, reps=3)
    svb.forward(params, states, out)
    tuned_b = svb.autotune(params, states, which=1, reps=3)

    def step():
        svb.forward(params, states, out)
        torch.sub(out, yt, out=w).mul_(2.0 / B)  # dL/df of the mean squared error
        svb.backward(params, states, w, grad)

    ms = _timed(step, steps, 3)
    fwd_ms = _timed(lambda: svb.forward(params, states, out), steps, 2)
    fpa = lib.plan_info(n, gates)["flops_per_amp"]
    fwd_flops = fpa * (1 << n) * B
    # GPU parameter shift on 4 samples (2P shifted circuits each), same weights
    sel = slice(0, 4)
    ps_ms = _timed(lambda: sv.param_shift_grad_gpu(params.reshape(B, P)[sel], gates, n, terms, 1, w[sel]), 2, 1)
    g_ps = sv.param_shift_grad_gpu(params.reshape(B, P)[sel], gates, n, terms, 1, w[sel])
    err = (grad.reshape(B, P)[sel] - g_ps).abs().max().item()
    # loop of single-circuit calls (16 samples, one circuit per call)
    one = lib.BatchSpec.uniform(n, gates, 1, P)
    psi1 = torch.empty(1 << n, dtype=torch.complex64, device="cuda")

    def loop16():
        for b in range(16):
            pr = params[b * P:(b + 1) * P]
            lib.init_states(psi1, one, 0)
            lib.sv_apply(psi1, pr, one)
            lib.expval(psi1, one, terms, 1)
            lib.sv_backward(psi1, pr, one, terms, 1, w[b:b + 1])

    loop_ms = _timed(loop16, 2, 1) / 16
    gate_amps = gates.shape[0] * (1 << n) * B
    return {"workload": "16-qubit 8-layer QNN (RY encoding, RY/RZ layers, CNOT chain; 392 gates, 272 params), "
                        "batch 512, complex64, MSE on <Z0>",
            "grad_circuits_per_s": B / (ms * 1e-3), "ms_per_step": round(ms, 3),
            "forward_gate_amps_per_s": gate_amps / (ms * 1e-3),
            "param_shift_gpu_circuits_per_s": 4 / (ps_ms * 1e-3),
            "adjoint_speedup_vs_param_shift": round((ps_ms / 4) / (ms / B), 1),
            "max_abs_grad_diff_vs_param_shift": err,
            "single_call_loop_circuits_per_s": 1 / (loop_ms * 1e-3),
            "batched_speedup_vs_single_calls": round(loop_ms / (ms / B), 1),
            "levels": svb.info["levels"], "graph_replays": svb.info["graph_replays"],
            "autotuned_forward": [int(tuned_f[0]), int(tuned_f[1])],
            "autotuned_backward": [int(tuned_b[0]), int(tuned_b[1])],
            "forward_ms": round(fwd_ms, 4),
            "roofline_forward": {"bound": "alu", "kernel": "sv_batch_stage_kernel (all levels of one forward)",
                                 "achieved": round(fwd_flops / (fwd_ms * 1e-3) / 1e12, 3), "peak": round(ALU_PEAK_TFLOPS, 1),
                                 "unit": "TFLOP/s", "frac": round(fwd_flops / (fwd_ms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS, 4),
                                 "frac_measured": _mfrac(fwd_flops / (fwd_ms * 1e-3) / 1e12, "fp32_fma_TFLOPs"),
                                 "algorithmic_flops": fwd_flops, "flops_per_amp": fpa}}


def bench_uneven(steps):
    """1024 random circuits, n uniform in 8..20, 2n layers of U3 on every qubit + floor(n/2)
    random CNOT pairs, <Z0> and its full gradient: compiled batch (autotuned, graph-replayed)
    vs a loop of single-circuit calls."""
    import numpy as np
    import torch

    from paper_2301_05451_amd import lib
    from paper_2301_05451_amd import workloads as W

    circs = W.uneven_batch()
    spec = lib.BatchSpec.from_circuits(circs)
    terms = W.zterms([([0], 1.0, 0)])
    params = torch.tensor(np.concatenate([c.params for c in circs]), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    svb = lib.SVBatch(spec, terms, 1, graph=True)
    compile_s = time.perf_counter() - t0
    states = svb.new_states()
    tf = svb.autotune(params, states, which=0, reps=1)
    svb.forward(params, states)
    tb = svb.autotune(params, states, which=1, reps=1)
    out = torch.empty(len(circs), 1, device="cuda")
    w = torch.ones(len(circs), 1, device="cuda")
    grad = torch.zeros_like(params)
    fwd_ms = _timed(lambda: svb.forward(params, states, out), steps, 3)

    def step():
        svb.forward(params, states, out)
        svb.backward(params, states, w, grad)

    ms = _timed(step, steps, 3)
    gate_amps = int(sum(c.gates.shape[0] << c.n for c in circs))
    fwd_flops = float(sum(lib.plan_info(c.n, c.gates)["flops_per_amp"] * (1 << c.n) for c in circs))
    # single-circuit calls, one circuit per call
    specs1 = [lib.BatchSpec.from_circuits([c]) for c in circs]
    offs = spec.param_off

    def loop():
        for i, c in enumerate(circs):
            one = specs1[i]
            pr = params[int(offs[i]):int(offs[i]) + c.n_params]
            psi1 = lib.zero_states(one, torch.complex64)
            lib.sv_apply(psi1, pr, one)
            lib.expval(psi1, one, terms, 1)
            lib.sv_backward(psi1, pr, one, terms, 1, w[i:i + 1])

    loop_ms = _timed(loop, 1, 1)
    return {"workload": "1024 random circuits, n uniform in 8..20 (seeded), 2n layers of U3 on all qubits + "
                        "floor(n/2) random CNOT pairs, complex64, <Z0> + full gradient",
            "grad_circuits_per_s": len(circs) / (ms * 1e-3), "ms_per_step": round(ms, 3),
            "forward_ms": round(fwd_ms, 3), "forward_gate_amps_per_s": gate_amps / (fwd_ms * 1e-3),
            "gate_amps": gate_amps, "compile_s": round(compile_s, 2),
            "autotuned_forward": list(tf[:2]), "autotuned_backward": list(tb[:2]),
            "single_call_loop_grad_circuits_per_s": len(circs) / (loop_ms * 1e-3),
            "batched_speedup_vs_single_calls": round(loop_ms / ms, 1),
            "levels": svb.info["levels"], "items": svb.info["items"],
            "roofline_forward": {"bound": "alu", "kernel": "sv_batch_stage_kernel (all levels of one forward)",
                                 "achieved": round(fwd_flops / (fwd_ms * 1e-3) / 1e12, 3), "peak": round(ALU_PEAK_TFLOPS, 1),
                                 "unit": "TFLOP/s", "frac": round(fwd_flops / (fwd_ms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS, 4),
                                 "frac_measured": _mfrac(fwd_flops / (fwd_ms * 1e-3) / 1e12, "fp32_fma_TFLOPs"),
                                 "algorithmic_flops": fwd_flops}}


def _workers():
    return max(1, min(16, os.cpu_count() or 1))


def bench_tn(steps, configs=("p3", "p4", "p4_sliced20"), batch_only=False):
    """QAOA MaxCut on a seeded random 3-regular graph of 50 nodes (75 edges): one light-cone
    network per edge for <Z_i Z_j>, value + gradient of (gamma, beta), all 75 networks in
    one batched call. Trees: the fewest-FLOP tree of the path search's pool (min-fill,
    min-degree, greedy, recursive bisection). p = 3, p = 4, and p = 4 sliced so that no
    intermediate exceeds 2^20 elements. Plus one dense pairwise step on the FP32-MFMA
    complex GEMM path."""
    import numpy as np
    import torch

    from paper_2301_05451_amd import lib, tn
    from paper_2301_05451_amd import workloads as W

    res = {}
    for name, p, target in (("p3", 3, None), ("p4", 4, None), ("p4_sliced20", 4, 20)):
        if name not in configs:
            continue
        prob = W.qaoa_maxcut(p=p)
        t0 = time.perf_counter()
        planned = tn.plan_qaoa(prob, target_rank=target, workers=_workers())
        progs = [tn.TNProgram(net, tree) for net, tree in planned]
        plan_s = time.perf_counter() - t0
        print(f"bench: TN {name} planned in {plan_s:.1f} s", file=sys.stderr, flush=True)
        pars = [torch.tensor(pg.net.params, dtype=torch.float32, device="cuda") for pg in progs]

        def run_single():
            for pg, pt in zip(progs, pars):
                pg.value(pt)
                pg.grad(pt)

        batch = tn.TNBatch(progs)

        def run_batch():
            batch.value_and_grads(pars)

        ms1 = _timed(run_single, 1, 1) if not batch_only else float("nan")
        ms = _timed(run_batch, max(2, steps // 2), 1)
        vb = torch.stack([v[0] for v in batch.values(pars)]).cpu().numpy()
        vs = np.array([pg.value(pt).cpu().numpy()[0] for pg, pt in zip(progs, pars)])
        flops = sum(pg.plan.info["flops"] for pg in progs)  # contraction only, 8 real flops per complex MAC
        gemm = sum(pg.plan.info["gemm_flops"] for pg in progs)
        byts = 0.0  # algorithmic bytes of the forward steps: read both operands, write the result
        for pg in progs:
            S = 2 ** len(pg.tree.sliced)
            for a, b, o in tn.tree_steps(pg.net, pg.tree):
                byts += (2.0 ** len(a) + 2.0 ** len(b) + 2.0 ** len(o)) * 8 * S
        res[name] = {"networks": len(progs), "plan_s": round(plan_s, 2),
                     "ms_value_and_grad_all": round(ms, 3),
                     "grad_networks_per_s": len(progs) / (ms * 1e-3),
                     "single_calls_ms": round(ms1, 3) if not batch_only else None,
                     "batched_speedup_vs_single_calls": round(ms1 / ms, 2) if not batch_only else None,
                     "batched_equals_single": bool(np.array_equal(vb, vs)),
                     "maxcut_value": float(np.sum((1.0 - vb.real) / 2.0)),
                     "contraction_flops_per_pass": flops,
                     "gemm_flop_share": gemm / max(flops, 1),
                     # value + gradient = about 3 forward passes of algorithmic work (the
                     # reverse pass recomputes the forward: not counted)
                     "tn_gflops": 3 * flops / (ms * 1e-3) / 1e9,
                     "step_bytes_per_pass": byts,
                     "hbm_GBs_of_step_bytes": 3 * byts / (ms * 1e-3) / 1e9,
                     "max_width": max(pg.tree.max_rank for pg in progs),
                     "sliced_networks": sum(1 for pg in progs if pg.tree.sliced),
                     "slices_total": sum(2 ** len(pg.tree.sliced) for pg in progs)}
    if batch_only:
        return res
    # dense step: C[b,m,n] = sum_k A[b,m,k] B[b,k,n], b = 1 bit, M = N = 2^12, K = 2^10
    b, m, k, nn = [0], list(range(1, 13)), list(range(13, 23)), list(range(23, 35))
    plan = lib.TnPlan([b + m + k, b + k + nn], [(0, 1)], out_inds=b + m + nn)
    g = torch.Generator(device="cuda").manual_seed(5)
    leaves = torch.randn(plan.leaf_elems, dtype=torch.complex64, device="cuda", generator=g)
    work = torch.empty(max(plan.workspace_bytes(False), 16), dtype=torch.uint8, device="cuda")
    ms = _timed(lambda: lib.tn_contract(plan, leaves, work), steps, 2)
    fl = 8 * 2 * (1 << 12) * (1 << 12) * (1 << 10)
    # sampled entries against a float64 sum over k
    C = lib.tn_contract(plan, leaves, work)
    A = leaves[:plan.leaf_offsets[1]].reshape(2, 1 << 12, 1 << 10)
    Bm = leaves[plan.leaf_offsets[1]:].reshape(2, 1 << 10, 1 << 12)
    rs = np.random.default_rng(9)
    errs = []
    for _ in range(16):
        bb, mm, nn_ = int(rs.integers(2)), int(rs.integers(1 << 12)), int(rs.integers(1 << 12))
        a = A[bb, mm].cpu().numpy().astype(np.complex128)
        bcol = Bm[bb, :, nn_].cpu().numpy().astype(np.complex128)
        want = np.dot(a, bcol)
        got = complex(C.reshape(2, 1 << 12, 1 << 12)[bb, mm, nn_].item())
        errs.append(abs(got - want) / np.sqrt(np.sum(np.abs(a) ** 2) * np.sum(np.abs(bcol) ** 2)))
    res["dense_step"] = {"shape": "batch 2, M = N = 4096, K = 1024 complex", "gemm_steps": plan.info["gemm_steps"],
                         "ms": round(ms, 3), "tflops": fl / (ms * 1e-3) / 1e12,
                         "mfma_frac_fp32": fl / (ms * 1e-3) / 157.3e12,
                         "mfma_frac_fp32_measured": _mfrac(fl / (ms * 1e-3) / 1e12, "fp32_mfma_TFLOPs"),
                         "sampled_rel_err": float(max(errs))}
    # the same step in complex128 on FP64 MFMA (peak 78.6 TFLOP/s)
    plan2 = lib.TnPlan([b + m + k, b + k + nn], [(0, 1)], out_inds=b + m + nn, c128=True)
    leaves2 = leaves.to(torch.complex128)
    work2 = torch.empty(max(plan2.workspace_bytes(False), 16), dtype=torch.uint8, device="cuda")
    ms2 = _timed(lambda: lib.tn_contract(plan2, leaves2, work2), steps, 2)
    C2 = lib.tn_contract(plan2, leaves2, work2).reshape(2, 1 << 12, 1 << 12)
    A2 = leaves2[:plan2.leaf_offsets[1]].reshape(2, 1 << 12, 1 << 10)
    B2 = leaves2[plan2.leaf_offsets[1]:].reshape(2, 1 << 10, 1 << 12)
    errs2 = []
    for _ in range(16):
        bb, mm, nn_ = int(rs.integers(2)), int(rs.integers(1 << 12)), int(rs.integers(1 << 12))
        a = A2[bb, mm].cpu().numpy()
        bcol = B2[bb, :, nn_].cpu().numpy()
        errs2.append(abs(complex(C2[bb, mm, nn_].item()) - np.dot(a, bcol)) /
                     np.sqrt(np.sum(np.abs(a) ** 2) * np.sum(np.abs(bcol) ** 2)))
    res["dense_step_c128"] = {"shape": "batch 2, M = N = 4096, K = 1024 complex128", "gemm_steps": plan2.info["gemm_steps"],
                              "ms": round(ms2, 3), "tflops": fl / (ms2 * 1e-3) / 1e12,
                              "mfma_frac_fp64": fl / (ms2 * 1e-3) / 78.6e12,
                              "mfma_frac_fp64_measured": _mfrac(fl / (ms2 * 1e-3) / 1e12, "fp64_mfma_TFLOPs"),
                              "sampled_rel_err": float(max(errs2))}
    return res


def bench_mqr():
    """Multiple-qubit rotation (the paper's Sec. 6.1 benchmark): 500 training iterations of a
    4-layer hardware-efficient network minimising sum_i <Z_i> from |0..0>, each iteration a
    compiled forward + adjoint backward + on-device gradient-descent update (lr 0.1)."""
    import torch

    from paper_2301_05451_amd import mqr

    out = {"workload": "MQR: 4 layers of RY, RZ on all qubits + CNOT chain, cost sum_i <Z_i>, "
                       "500 gradient-descent iterations (lr 0.1), complex64", "runs": []}
    for n in (4, 8, 12, 16, 20):
        tr = mqr.MQRTrainer(mqr.mqr_circuit(n, layers=4), lr=0.1)
        tr.run(3)  # warm-up: compiles the graphs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = tr.run(500)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        h = hist.cpu().numpy()
        out["runs"].append({"qubits": n, "params": int(tr.params.numel()), "s_per_500_iters": round(dt, 4),
                            "iters_per_s": round(500 / dt, 1), "cost_first": float(h[0]),
                            "cost_last": float(h[-1])})
    return out


def bench_costmodel():
    """Learned ranking of contraction trees and slicings (QAOA p = 4): the cost-model MLP is
    trained on the GPU from measured times (value + gradient) of the candidates (path-search
    trees x slicings to width, width - 2, width - 4) of 10 light-cone networks on each of
    three other seeded 50-node graphs, then picks one candidate for each of 25 networks of the
    workload graph (held out); its picks are timed against the fewest-FLOP picks and against
    the fastest measured candidate (the most any ranking could gain)."""
    from paper_2301_05451_amd import costmodel
    from paper_2301_05451_amd import workloads as W

    t0 = time.perf_counter()
    train = []
    for seed in (2001, 2002, 2003):
        g = costmodel.qaoa_graph(seed)
        train += costmodel.plan_candidates(g, g.edges[::7][:10], workers=_workers())
    prob = W.qaoa_maxcut(p=4)
    test = costmodel.plan_candidates(prob, prob.edges[::3], workers=_workers())
    plan_s = time.perf_counter() - t0
    print(f"bench: ranking candidates planned in {plan_s:.1f} s", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    r = costmodel.ranking_experiment(train, test, reps=5,
                                     log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    r.update({"workload": "QAOA p=4: 10 networks on each of 3 training graphs, 25 held-out networks of the "
                          "workload graph; candidates = 6 path-search trees x 3 slicings",
              "plan_s": round(plan_s, 1), "measure_and_fit_s": round(time.perf_counter() - t1, 1)})
    for k in ("ms_flop_ranked", "ms_mlp_ranked", "ms_fastest_measured"):
        r[k] = round(r[k], 2)
    r["learned_gain"] = round(r["learned_gain"], 3)
    r["max_possible_gain"] = round(r["max_possible_gain"], 3)
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-plan", action="store_true",
                    help="also time the oracle on every workload (minutes; adds cpu_plan to the JSON line)")
    ap.add_argument("--extras", default="qnn16_batch512,uneven1024,tn_qaoa50,mqr,tree_ranking",
                    help="comma-separated measurements besides the headline")
    ap.add_argument("--plain-steps", type=int, default=1, help="steps of the one-sweep-per-gate path")
    ap.add_argument("--tn-configs", default="p3,p4,p4_sliced20",
                    help="QAOA network sets of the tn_qaoa50 measurement (for profiling one of them)")
    ap.add_argument("--tn-batch-only", action="store_true",
                    help="tn_qaoa50: time the batched calls only (no single-call loop, no dense step)")
    ap.add_argument("--tile-bits", type=int, default=0)
    ap.add_argument("--reg-bits", type=int, default=0)
    ap.add_argument("--coal-bits", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the QNN batch, uneven batch and tensor-network measurements")
    ap.add_argument("--no-peaks", action="store_true", help="skip the attainable-peak probes")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="calibration only: 10 device-to-device copies of this many bytes (the known "
                         "traffic that scales the HBM byte counters), then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2301_05451_amd import lib
    from paper_2301_05451_amd import workloads as W

    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 10}), flush=True)
        return

    peaks = None if args.no_peaks else measure_peaks()

    c = W.brickwork()
    n, G = c.n, c.gates.shape[0]
    spec = lib.BatchSpec.uniform(n, c.gates, 1, c.n_params)
    params = torch.tensor(c.params, dtype=torch.float32, device="cuda")
    psi = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    opts = dict(tile_bits=args.tile_bits, reg_bits=args.reg_bits, coal_bits=args.coal_bits)
    info = lib.plan_info(n, c.gates, mode=0, **opts)

    def step():
        lib.sv_run(psi, params, spec, basis=0, mode=0, **opts)
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
        ev[k][0].record()
        lib.sv_run(psi, params, spec, basis=0, mode=0, **opts)
        ev[k][1].record()
        f = lib.expval(psi, spec, c.terms, 1)
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    apply_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    value = G * (1 << n) / (wall / args.steps)

    # dominant kernel: the fused stage sweep. One launch reads and writes the 2^n x 8-byte
    # state (the first only writes it) and does flops_per_amp(stage) x 2^n flops; averaged
    # over the circuit's stages.
    stages = info["sweeps"]
    stage_ms = apply_ms / stages  # includes the one small gate-build launch per call
    # every stage reads and writes the state, except the first, which forms |0..0> and only writes
    bytes_per_stage = (2 * stages - 1) * (1 << n) * 8 / stages
    flops_per_stage = info["flops_per_amp"] * (1 << n) / stages
    gbs = bytes_per_stage / (stage_ms * 1e-3) / 1e9
    tflops = flops_per_stage / (stage_ms * 1e-3) / 1e12
    t_hbm = bytes_per_stage / (HBM_PEAK_GBS * 1e9)
    t_alu = flops_per_stage / (ALU_PEAK_TFLOPS * 1e12)
    if t_alu >= t_hbm:
        roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": round(ALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                "frac": round(tflops / ALU_PEAK_TFLOPS, 4), "frac_measured": _mfrac(tflops, "fp32_fma_TFLOPs"),
                "traffic": measured_traffic(),
                "algorithmic_bytes": bytes_per_stage, "algorithmic_flops": flops_per_stage,
                "peak_published_fp32_vector": ALU_PEAK_PUBLISHED_TFLOPS,
                "hbm_achieved_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                "hbm_frac_measured": _mfrac(gbs, "state_copy_GBs")}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "frac_measured": _mfrac(gbs, "state_copy_GBs"),
                "traffic": measured_traffic(),
                "algorithmic_bytes": bytes_per_stage}
    kname = "sv_stage_kernel_t12<float,%d>" if info["tile_bits"] == 12 else "sv_stage_kernel<float,%d>"
    roof.update({"kernel": kname % info["reg_bits"], "launches_per_step": stages,
                 "avg_launch_us": round(stage_ms * 1e3, 2)})

    # the expectation value alone (partial-sum + final launches): a streaming read of the state
    ev_ms = _timed(lambda: lib.expval(psi, spec, c.terms, 1), args.steps, 2)
    ev_bytes = (1 << n) * 8
    expval_roof = {"bound": "hbm", "kernel": "expval_partial_kernel + expval_final_kernel", "terms": int(c.terms.shape[0]),
                   "achieved": round(ev_bytes / (ev_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(ev_bytes / (ev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "frac_measured": _mfrac(ev_bytes / (ev_ms * 1e-3) / 1e9, "state_read_GBs"), "us": round(ev_ms * 1e3, 2),
                   "algorithmic_bytes": ev_bytes}

    # the plain path (one HBM sweep per gate) on the same circuit, for comparison
    plain = None
    if args.plain_steps > 0:
        pinfo = lib.plan_info(n, c.gates, mode=1)
        lib.sv_run(psi, params, spec, basis=0, mode=1)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.plain_steps):
            lib.sv_run(psi, params, spec, basis=0, mode=1)
            fp = lib.expval(psi, spec, c.terms, 1)
        b.record()
        torch.cuda.synchronize()
        pms = a.elapsed_time(b) / args.plain_steps
        sweep_bytes = 2 * (1 << n) * 8  # one gate: the state read and written
        plain = {"gate*amps/s": G * (1 << n) / (pms * 1e-3), "ms_per_step": round(pms, 3),
                 "sweeps": pinfo["sweeps"],
                 "avg_sweep_GBs": round(pinfo["sweeps"] * sweep_bytes / (pms * 1e-3) / 1e9, 1),
                 "avg_sweep_frac_measured": _mfrac(pinfo["sweeps"] * sweep_bytes / (pms * 1e-3) / 1e9, "state_copy_GBs"),
                 "expval_agrees": bool(abs(float(fp[0, 0]) - float(f[0, 0])) < 1e-4)}

    out = {
        "metric": METRIC, "value": value, "unit": "gate*amps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "24-qubit brickwork state-vector circuit: 20 layers of RX,RY,RZ on all qubits "
                               "+ CZ on alternating neighbour pairs (1670 gates), complex64, sum_i Z_i, batch 1",
                   "qubits": n, "gates": G, "fused_sweeps": stages, "tile_bits": info["tile_bits"],
                   "reg_bits": info["reg_bits"], "coal_bits": args.coal_bits or None,
                   "flops_per_amp": info["flops_per_amp"], "phases": info["phases"],
                   "exchanges": info["exchanges"]},
        "roofline": roof,
        "roofline_expval": expval_roof,
        "measured_peaks": peaks,
        "expval_sum_z": float(f[0, 0]),
        "plain": plain,
    }
    if not args.no_extras:
        wanted = set(x.strip() for x in args.extras.split(",") if x.strip())
        for key, fn in (("qnn16_batch512", lambda: bench_qnn(max(5, args.steps // 2))),
                        ("uneven1024", lambda: bench_uneven(max(3, args.steps // 4))),
                        ("tn_qaoa50", lambda: bench_tn(max(4, args.steps // 2), args.tn_configs.split(","),
                                                       args.tn_batch_only)),
                        ("mqr", bench_mqr),
                        ("tree_ranking", bench_costmodel)):
            if key not in wanted:
                continue
            t0 = time.perf_counter()
            out[key] = fn()
            print(f"bench: {key} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(c)
    if args.cpu_plan:
        out["cpu_plan"] = cpu_plan()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
