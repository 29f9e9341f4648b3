"""Gradient of a detected energy with respect to the opacity fields.

``detected_energy(ctx, I0, kappa_a, kappa_s, eta, nsteps, face, ...)`` runs
``nsteps`` fused steps of the HIP library and returns, as a 0-d float64
tensor, the energy that streams out through ``face`` summed over the states
entering the steps (``diag[1 + face]`` of ``lbrt_step``).  It is a
``torch.autograd.Function``: ``backward`` runs the reverse sweep with
``lbrt_adjoint_step`` and returns the gradients with respect to kappa_a,
kappa_s and eta.  Compose other dependences in torch (e.g. local thermal
equilibrium ``eta = kappa_a * B`` chains the eta gradient into kappa_a).

Checkpointing: the forward pass keeps the state every ``checkpoint_every``
steps; the backward pass recomputes each segment's states from its
checkpoint (``checkpoint_every`` states live at a time) and sweeps it in
reverse.  Every step and adjoint step runs in the library's kernels; this
module only sequences calls and holds buffers.
"""
from __future__ import annotations

import torch

from . import LBRT_DIAG_LEN, LBRT_FP64, lbrt_adjoint_step, lbrt_step


def _forward(lb, I0, kappa_a, kappa_s, eta, nsteps, face, K, vel, inflow):
    """Runs the steps; returns (L as a 0-d float64 tensor, checkpoints)."""
    cur = I0.detach().clone()
    nxt = torch.empty_like(cur)
    diag = torch.zeros(LBRT_DIAG_LEN, dtype=torch.float64, device=I0.device)
    L = torch.zeros((), dtype=torch.float64, device=I0.device)
    ckpts = []
    done = 0
    while done < nsteps:
        k = min(K, nsteps - done)
        ckpts.append(cur.clone())
        lbrt_step(lb, cur, nxt, kappa_a, kappa_s, eta, vel=vel, inflow=inflow, nsteps=k,
                  diag=diag)
        L = L + diag[1 + face]
        if k % 2 == 1:
            cur, nxt = nxt, cur
        done += k
    return L, ckpts


def _reverse(lb, ckpts, kappa_a, kappa_s, eta, nsteps, face, K, vel, inflow):
    """The reverse sweep; returns (g_kappa_a, g_kappa_s, g_eta) in float64 for
    FP64 storage and float32 otherwise."""
    gdt = torch.float64 if lb.desc.c.storage == LBRT_FP64 else torch.float32
    nc = lb.desc.ncell
    dev = ckpts[0].device
    g = [torch.zeros(nc, dtype=gdt, device=dev) for _ in range(3)]
    lam = torch.zeros_like(ckpts[0])
    lam_out = torch.empty_like(lam)
    for s in range(len(ckpts) - 1, -1, -1):
        k = min(K, nsteps - s * K)
        # recompute the segment's states from its checkpoint
        states = [ckpts[s]]
        for _ in range(k - 1):
            nxt = torch.empty_like(states[-1])
            lbrt_step(lb, states[-1], nxt, kappa_a, kappa_s, eta, vel=vel, inflow=inflow,
                      nsteps=1)
            states.append(nxt)
        for j in range(k - 1, -1, -1):
            lbrt_adjoint_step(lb, states[j], lam, lam_out, face, g[0], g[1], g[2], kappa_a,
                              kappa_s, eta, vel=vel, inflow=inflow)
            lam, lam_out = lam_out, lam
        del states
    return g[0], g[1], g[2]


class _DetectedEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, kappa_a, kappa_s, eta, lb, I0, nsteps, face, checkpoint_every, vel,
                inflow):
        K = max(1, int(checkpoint_every))
        L, ckpts = _forward(lb, I0, kappa_a, kappa_s, eta, nsteps, face, K, vel, inflow)
        fctx.lb, fctx.nsteps, fctx.face, fctx.K = lb, nsteps, face, K
        fctx.vel, fctx.inflow, fctx.ckpts = vel, inflow, ckpts
        fctx.save_for_backward(kappa_a, kappa_s, eta)
        return L

    @staticmethod
    def backward(fctx, gL):
        kappa_a, kappa_s, eta = fctx.saved_tensors
        g = _reverse(fctx.lb, fctx.ckpts, kappa_a, kappa_s, eta, fctx.nsteps, fctx.face,
                     fctx.K, fctx.vel, fctx.inflow)
        fctx.ckpts = None
        scale = gL.to(torch.float64)
        out = [(x.to(torch.float64) * scale).to(kappa_a.dtype) for x in g]
        return out[0], out[1], out[2], None, None, None, None, None, None, None


def detected_energy(lb, I0, kappa_a, kappa_s, eta, nsteps: int, face: int = 1,
                    checkpoint_every: int = 8, vel=None, inflow=None):
    """Energy through ``face`` over ``nsteps`` steps from state ``I0``
    (differentiable in kappa_a, kappa_s, eta; float32 fields of ncell)."""
    return _DetectedEnergy.apply(kappa_a, kappa_s, eta, lb, I0, int(nsteps), int(face),
                                 int(checkpoint_every), vel, inflow)


def detected_energy_gradient(lb, I0, kappa_a, kappa_s, eta, nsteps: int, face: int = 1,
                             checkpoint_every: int = 8, vel=None, inflow=None):
    """(L, g_kappa_a, g_kappa_s, g_eta) without autograd; the gradients keep the
    library's precision (float64 for FP64 storage)."""
    K = max(1, int(checkpoint_every))
    with torch.no_grad():
        L, ckpts = _forward(lb, I0, kappa_a, kappa_s, eta, int(nsteps), int(face), K, vel,
                            inflow)
        g = _reverse(lb, ckpts, kappa_a, kappa_s, eta, int(nsteps), int(face), K, vel, inflow)
    return (L,) + g
