"""PyTorch interface of the state-vector path (the quantum-to-classical interface of the
paper's Sec. 4.3): ``torch.autograd.Function``s whose forward runs tq_sv_init +
tq_sv_apply + tq_expval (or a compiled batch's tq_svb_forward) and whose backward runs the
adjoint sweep tq_sv_backward (tq_svb_backward).

All arithmetic runs in libtq kernels; torch provides device memory, streams and the
autograd graph around the circuit.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import lib
from . import workloads as W


class SVExpval(torch.autograd.Function):
    """out[i, o] = <psi_i| O_o |psi_i>, psi_i = U_i(params_i) |0..0>.

    ``params`` is a flat tensor laid out as the batch's param_off says (float32 for
    complex64, float64 for complex128). Gradients flow to ``params`` only.
    """

    @staticmethod
    def forward(ctx, params, spec, terms, n_obs, cdtype, fwd_opts, bwd_opts):
        params = params.contiguous()
        psi = torch.empty(spec.total_amps, dtype=cdtype, device=params.device)
        lib.init_states(psi, spec, 0)
        lib.sv_apply(psi, params, spec, **fwd_opts)
        out = lib.expval(psi, spec, terms, n_obs)
        ctx.save_for_backward(params, psi)
        ctx.spec, ctx.terms, ctx.n_obs, ctx.bwd_opts = spec, terms, n_obs, bwd_opts
        return out

    @staticmethod
    def backward(ctx, grad_out):
        params, psi = ctx.saved_tensors
        g = lib.sv_backward(psi, params, ctx.spec, ctx.terms, ctx.n_obs, grad_out.contiguous().to(params.dtype),
                            **ctx.bwd_opts)
        return g, None, None, None, None, None, None


def expval(params, spec, terms, n_obs=1, dtype=torch.complex64, fwd_opts=None, bwd_opts=None):
    """Differentiable expectation values of a batch of circuits."""
    return SVExpval.apply(params, spec, terms, n_obs, dtype, fwd_opts or {}, bwd_opts or {})


class BatchExpval(torch.autograd.Function):
    """Differentiable expectation values of a compiled batch (lib.SVBatch): forward is
    tq_svb_forward, backward tq_svb_backward. The final states stay in ``states`` (no
    copy), so the backward pass must run before that buffer is reused by another forward."""

    @staticmethod
    def forward(ctx, params, svb, states):
        params = params.contiguous()
        out = svb.forward(params, states)
        ctx.save_for_backward(params)
        ctx.svb, ctx.states = svb, states
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (params,) = ctx.saved_tensors
        g = ctx.svb.backward(params, ctx.states, grad_out.contiguous().to(params.dtype))
        return g, None, None


def batch_expval(params, svb, states=None):
    """``svb`` = lib.SVBatch. ``states`` (optional) is reused as the state buffer, which
    lets graph replays see the same pointers every step."""
    if states is None:
        states = svb.new_states(params.device)
    return BatchExpval.apply(params, svb, states)


def shifted_param_sets(params, spec):
    """Parameter-shift rule of the paper's Sec. 4.2 with s = pi/2, k = 1/2, valid when
    every parameter of the batch's (single) gate list appears in exactly one gate slot with
    pscale 1 (as in the QNN workloads): returns [2P, P] shifted copies of one circuit's
    parameter vector (+s rows then -s rows)."""
    P = params.numel()
    eye = torch.eye(P, dtype=params.dtype, device=params.device) * (math.pi / 2)
    return torch.cat([params[None, :] + eye, params[None, :] - eye], 0)


def param_shift_grad_gpu(params_b, gates, n, terms, n_obs, weights, dtype=torch.complex64, chunk=None):
    """GPU parameter-shift baseline: for each circuit b (row of params_b [B, P]) evaluate
    its 2P shifted circuits in batched launches and combine
    d(sum_o w_o <O_o>)/d p = 1/2 [f(p + pi/2) - f(p - pi/2)] (single-occurrence parameters)."""
    B, P = params_b.shape
    grads = torch.empty_like(params_b)
    chunk = chunk or max(1, 4096 // max(1, 2 * P))
    for b0 in range(0, B, chunk):
        rows = []
        for b in range(b0, min(B, b0 + chunk)):
            rows.append(shifted_param_sets(params_b[b], None))
        stack = torch.cat(rows, 0).contiguous()
        spec = lib.BatchSpec.uniform(n, gates, stack.shape[0], P)
        psi = torch.empty(spec.total_amps, dtype=dtype, device=params_b.device)
        lib.init_states(psi, spec, 0)
        lib.sv_apply(psi, stack.reshape(-1), spec)
        f = lib.expval(psi, spec, terms, n_obs).to(torch.float64)  # [rows*2P, n_obs]
        f = f.reshape(-1, 2 * P, n_obs)
        w = weights[b0:b0 + f.shape[0]].to(torch.float64)  # [nb, n_obs]
        fw = (f * w[:, None, :]).sum(-1)  # [nb, 2P]
        grads[b0:b0 + f.shape[0]] = (0.5 * (fw[:, :P] - fw[:, P:])).to(params_b.dtype)
    return grads


def single_occurrence(gates, n_params):
    """True if every parameter index appears in exactly one angle slot with pscale 1."""
    seen = np.zeros(n_params, dtype=int)
    for g in gates:
        for j in range(W.N_ANGLES[int(g["op"])]):
            p = int(g["pidx"][j])
            if p >= 0:
                if float(g["pscale"][j]) != 1.0:
                    return False
                seen[p] += 1
    return bool(np.all(seen == 1))
