"""Gradient of the dissociated population with respect to the incident pulse.

Y(knots, omega) = mean_i [norm of molecule i beyond r_diss + its absorbed
norm] at the end of a coupled run driven by E_inc(t) = A(t) cos(omega t),
A piecewise linear through the knots.  The backward pass runs the
hand-written adjoint of the coupled step (adjoint_step in libmsqd) in
reverse, with checkpoint-and-recompute: the forward run stores the full
state every K steps; the backward pass restores each checkpoint in turn,
recomputes its K steps keeping the wavepackets and gathered fields of every
step in device memory, and sweeps back through them.  The forward run keeps
the history of its last segment in that same buffer, so the reverse sweep
starts without a recompute.  The last stage, the chain rule from
dY/dE_inc(t_n) to the pulse parameters, is a small contraction with the
pulse's Jacobian.
"""

from __future__ import annotations

import numpy as np
import torch

from . import msqd


class CoupledYield(torch.autograd.Function):
    @staticmethod
    def forward(ctx, knots, omega, cfg, prec="fp32", ckpt_every=None, mol_every=1):
        from workloads.pulses import source_values
        K = int(ckpt_every or cfg.ckpt_every)
        n_steps = cfg.n_steps
        kn = knots.detach().cpu().numpy().astype(np.float64)
        w = float(omega.detach().cpu())
        src = source_values(cfg, 0, n_steps, knots=kn, omega=w)
        # no monitor: the objective does not involve the transmitted flux
        sysm = msqd.Coupled(cfg, prec=prec, mol_every=mol_every, n_freq=0)
        hist = _history_buffers(sysm, K, n_steps)
        ckpts = []
        slot_of = []
        for s0 in range(0, n_steps, K):
            s1 = min(s0 + K, n_steps)
            if s1 < n_steps:
                ckpts.append(sysm.snapshot())
                sysm.step(src[s0:s1])
            else:
                # the last segment straight into the history buffer; the live
                # wavepackets then take its final state
                ckpts.append(None)
                slot_of, cur = _segment_history(sysm, src, s0, s1, *hist)
                sysm.mol.psi.copy_(hist[0][cur])
        # the objective: the mean over molecules of the library's FP64 sum of
        # the per-molecule dissociated populations (dipole_readout)
        Y = sysm.ensemble_sums()[-1].detach().clone() / sysm.mol.desc.n_mol
        ctx.sysm, ctx.ckpts, ctx.src, ctx.K = sysm, ckpts, src, K
        ctx.hist, ctx.last_slots = hist, slot_of
        ctx.cfg, ctx.kn, ctx.w = cfg, kn, w
        return Y

    @staticmethod
    def backward(ctx, gY):
        g = source_gradient(ctx.sysm, ctx.ckpts, ctx.src, ctx.K, hist=ctx.hist, last_slots=ctx.last_slots)
        ctx.hist = None
        from workloads.pulses import source_jacobian
        jac = source_jacobian(ctx.cfg, 0, len(ctx.src), knots=ctx.kn, omega=ctx.w)
        dp = jac @ g.cpu().numpy()
        scale = float(gY)
        dk = torch.as_tensor(dp[:-1] * scale, dtype=torch.float64)
        dw = torch.as_tensor(dp[-1] * scale, dtype=torch.float64)
        return dk, dw, None, None, None, None


def _device_empty(shape, dtype, dev):
    """torch.empty on the device; when the caching allocator cannot place a
    buffer this large among the blocks it holds, release them and try once
    more."""
    try:
        return torch.empty(shape, dtype=dtype, device=dev)
    except torch.cuda.OutOfMemoryError:
        torch.cuda.empty_cache()
        return torch.empty(shape, dtype=dtype, device=dev)


def _history_buffers(sysm, K, n_steps):
    """One history buffer of K + 1 wavepacket slots and K gathered fields,
    reused by every segment (57 GB for the differentiation workload in FP32,
    115 GB in FP64)."""
    dev = sysm.mol.psi.device
    n_mol = sysm.mol.desc.n_mol
    psi_all = _device_empty((min(K, n_steps) + 1,) + tuple(sysm.mol.psi.shape), sysm.mol.psi.dtype, dev)
    e_all = torch.empty((min(K, n_steps), max(n_mol, 1)), dtype=torch.float64, device=dev)
    return psi_all, e_all


def _segment_history(sysm, src, s0, s1, psi_all, e_all):
    """Advance sysm over steps s0..s1-1 from its current state, keeping the
    segment's wavepackets and the fields gathered at its molecular steps
    (e_all[t - s0]; sysm.E_mol is not updated): slot 0 is the state at s0, and
    each step that moves the molecules reads its slot and writes the next one
    (coupled_step's out-of-place form), so no step copies a state.  Returns
    the slot holding the state before each step, and the slot of the final
    state.  The live wavepackets are left as they were."""
    n_mol = sysm.mol.desc.n_mol
    M = sysm.mol_every
    psi_all[0].copy_(sysm.mol.psi)
    cur = 0
    slot_of = []
    for t in range(s0, s1):
        slot_of.append(cur)
        if t % M == 0 and n_mol > 0:
            # the gathered field straight into its history slot (the reverse
            # sweep reads it at these steps only)
            sysm.step_out_of_place(src[t], psi_all[cur], psi_all[t - s0 + 1], E_out=e_all[t - s0])
            cur = t - s0 + 1
        else:
            sysm.step(src[t:t + 1])
    return slot_of, cur


def source_gradient(sysm, ckpts, src, K, hist=None, last_slots=None):
    """dY/dsrc[n] for every step, from the final state held by sysm, by
    reverse sweeps over checkpointed segments (device float64 [n_steps]).
    ckpts[seg] is the state at the start of segment seg; hist, when given, is
    the history buffer, and last_slots the slots of the last segment already
    in it (its checkpoint may then be None)."""
    n_steps = len(src)
    dev = sysm.mol.psi.device
    adj, buffers = sysm.adjoint_buffers()
    msqd.adjoint_init_yield(sysm.desc, sysm.state, adj)
    g = torch.zeros(n_steps, dtype=torch.float64, device=dev)
    n_mol = sysm.mol.desc.n_mol
    M = sysm.mol_every
    psi_all, e_all = hist if hist is not None else _history_buffers(sysm, K, n_steps)
    last = len(ckpts) - 1
    for seg in reversed(range(len(ckpts))):
        s0 = seg * K
        s1 = min(s0 + K, n_steps)
        if seg == last and last_slots:
            slot_of = last_slots
        else:
            sysm.restore(ckpts[seg])
            slot_of, _ = _segment_history(sysm, src, s0, s1, psi_all, e_all)
        for t in reversed(range(s0, s1)):
            i = slot_of[t - s0]
            # at a molecular step the state after it sits in slot t - s0 + 1;
            # it is not read again (the FP64 adjoint step uses it as scratch)
            nxt = psi_all[t - s0 + 1] if (t % M == 0 and n_mol > 0) else None
            msqd.adjoint_step(sysm.desc, sysm.state, psi_all[i], e_all[t - s0], adj, t, g[t:t + 1],
                              psi_np1=nxt)
    del psi_all, e_all
    buffers.clear()
    return g


def yield_and_gradient(cfg, knots, omega, prec="fp32", ckpt_every=None, mol_every=1):
    """(Y, dY/dknots, dY/domega) for a run of cfg, with the molecules
    stepped every mol_every field steps."""
    k = torch.as_tensor(np.asarray(knots, np.float64)).requires_grad_(True)
    w = torch.as_tensor(float(omega), dtype=torch.float64).requires_grad_(True)
    Y = CoupledYield.apply(k, w, cfg, prec, ckpt_every, mol_every)
    Y.backward()
    return float(Y.detach()), k.grad.numpy().copy(), float(w.grad)
