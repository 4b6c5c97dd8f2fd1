"""Gradient of the dissociated population with respect to the incident pulse.

Y(knots, omega) = mean_i [norm of molecule i beyond r_diss + its absorbed
norm] at the end of a coupled run driven by E_inc(t) = A(t) cos(omega t),
A piecewise linear through the knots.  The backward pass runs the
hand-written adjoint of the coupled step (adjoint_step in libmsqd) in
reverse, with checkpoint-and-recompute: the forward run stores the full
state every K steps; the backward pass restores each checkpoint in turn,
recomputes its K steps keeping the wavepackets and gathered fields of every
step in device memory, and sweeps back through them.  The last stage, the
chain rule from dY/dE_inc(t_n) to the pulse parameters, is a small
contraction with the pulse's Jacobian.
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
        sysm = msqd.Coupled(cfg, prec=prec, mol_every=mol_every)
        ckpts = []
        for s0 in range(0, n_steps, K):
            ckpts.append(sysm.snapshot())
            sysm.step(src[s0:min(s0 + K, n_steps)])
        # the objective: the mean over molecules of the library's FP64 sum of
        # the per-molecule dissociated populations (dipole_readout)
        Y = sysm.ensemble_sums()[-1].detach().clone() / sysm.mol.desc.n_mol
        ctx.sysm, ctx.ckpts, ctx.src, ctx.K = sysm, ckpts, src, K
        ctx.cfg, ctx.kn, ctx.w = cfg, kn, w
        return Y

    @staticmethod
    def backward(ctx, gY):
        g = source_gradient(ctx.sysm, ctx.ckpts, ctx.src, ctx.K)
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


def source_gradient(sysm, ckpts, src, K):
    """dY/dsrc[n] for every step, from the final state held by sysm, by
    reverse sweeps over checkpointed segments (device float64 [n_steps])."""
    n_steps = len(src)
    dev = sysm.mol.psi.device
    adj, buffers = sysm.adjoint_buffers()
    msqd.adjoint_init_yield(sysm.desc, sysm.state, adj)
    g = torch.zeros(n_steps, dtype=torch.float64, device=dev)
    n_mol = sysm.mol.desc.n_mol
    M = sysm.mol_every
    # one history buffer of K + 1 wavepacket slots, reused by every segment
    # (57 GB for the differentiation workload in FP32, 115 GB in FP64)
    psi_all = _device_empty((min(K, n_steps) + 1,) + tuple(sysm.mol.psi.shape), sysm.mol.psi.dtype, dev)
    e_all = torch.empty((min(K, n_steps), max(n_mol, 1)), dtype=torch.float64, device=dev)
    for seg in reversed(range(len(ckpts))):
        s0 = seg * K
        s1 = min(s0 + K, n_steps)
        sysm.restore(ckpts[seg])
        # the segment's wavepackets: slot 0 is the checkpoint, and each step
        # that moves the molecules reads its slot and writes the next one
        # (coupled_step's out-of-place form), so no step copies a state
        psi_hist = psi_all[:s1 - s0 + 1]
        e_hist = e_all[:s1 - s0]
        psi_hist[0].copy_(sysm.mol.psi)
        cur = 0
        slot_of = []                      # slot holding the state before step t
        for t in range(s0, s1):
            slot_of.append(cur)
            if t % M == 0 and n_mol > 0:
                sysm.step_out_of_place(src[t], psi_hist[cur], psi_hist[t - s0 + 1])
                cur = t - s0 + 1
            else:
                sysm.step(src[t:t + 1])
            e_hist[t - s0].copy_(sysm.E_mol)
        for t in reversed(range(s0, s1)):
            i = slot_of[t - s0]
            # at a molecular step the state after it sits in slot t - s0 + 1;
            # it is not read again (the FP64 adjoint step uses it as scratch)
            nxt = psi_hist[t - s0 + 1] if (t % M == 0 and n_mol > 0) else None
            msqd.adjoint_step(sysm.desc, sysm.state, psi_hist[i], e_hist[t - s0], adj, t, g[t:t + 1],
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
