"""Training driver of the learned right preconditioner.

Training pairs (r, x) satisfy J x = r with J the solver's own Jacobian:

* Krylov pairs: ``jfnk_newton_step`` records, for every FGMRES iteration of the
  physics-preconditioned solve, the preconditioned direction z_j and its image
  J z_j (the solver's Jv kernel).
* Noise pairs: x is seeded Gaussian noise with the per-field RMS of the recorded
  directions and r = J x through ``jfnk_jv``.  Fitting these is the
  least-squares (Frobenius) problem of a local approximate inverse, which covers
  the rough directions a Krylov basis contains.

Training runs Adam steps of ``jfnk_net_train_step`` on mini-batches alternating
between the two kinds, with a cosine learning-rate decay.  All arithmetic runs in
the HIP library (the noise is drawn by torch's seeded device generator as an
input); this module only orders the calls and picks the mini-batches.
"""
from __future__ import annotations

import numpy as np

from . import inputs as I

# Per-layer dilations of the 3 x 3 kernels: 1, 2, 4, 8 give every output a dense
# 31 x 31 receptive field with the parameters and flops of four plain layers.
DILATIONS = (1, 2, 4, 8)


def collect_pairs(ctx, u0, steps, cap, eta=1e-3, pc="physics", inner="f32", krylov=True, **kw):
    """Advance ``steps`` implicit steps from u0 (FP64 device tensor), recording
    pairs (r, du) with J du = r: the preconditioned Krylov directions z_j and
    their images J z_j of every FGMRES iteration (krylov=True), or the Newton
    systems (-R, du).  Returns float32 (count, n) device tensors and the final
    state."""
    import torch
    n = ctx.n
    R = torch.empty((cap, n), dtype=torch.float32, device=u0.device)
    DU = torch.empty_like(R)
    count = [0]
    u = u0.clone()
    nxt = torch.empty_like(u)
    for _ in range(steps):
        nxt.copy_(u)
        ctx.newton_step(u, nxt, rtol=1e-8, inner=inner, pc=pc, forcing="fixed", eta=eta,
                        record=(R, DU, count), record_krylov=krylov, **kw)
        u.copy_(nxt)
        if count[0] >= cap:
            break
    return R[: count[0]], DU[: count[0]], u


class NoisePairs:
    """(J x, x) pairs for a frozen state u: x seeded Gaussian with field RMS sigma."""

    def __init__(self, ctx, u, sigma, seed=0):
        import torch
        self.ctx = ctx
        self.u32 = u.float().contiguous()
        self.sigma = torch.as_tensor(np.asarray(sigma, dtype=np.float32), device=u.device)
        self.gen = torch.Generator(device=u.device)
        self.gen.manual_seed(seed)
        p = ctx.prob
        self.shape = (p.nf, p.nz * p.ny * p.nx)

    def batch(self, B):
        import torch
        X = torch.randn((B,) + self.shape, generator=self.gen, device=self.u32.device, dtype=torch.float32)
        X = (X * self.sigma[None, :, None]).reshape(B, -1).contiguous()
        R = torch.empty_like(X)
        for b in range(B):
            self.ctx.jv(self.u32, X[b], R[b], mode="stable")
        return R, X


def field_rms(DU, nf):
    """Per-field RMS of recorded directions (scales of the noise pairs)."""
    return DU.reshape(DU.shape[0], nf, -1).pow(2).mean(dim=(0, 2)).sqrt().cpu().numpy()


def train_mixed(ctx, R, DU, u, iters=2000, lr=2e-3, batch=8, seed=0, theta0=None, noise_every=2,
                dilations=DILATIONS, loss="solution"):
    """The recipe used by the benchmark and tests: noise pairs at the state u on
    every step but one in ``noise_every``, recorded Krylov pairs on the others;
    ``loss`` selects the training norm (see ``Context.net_set_loss``)."""
    import torch
    nf = ctx.prob.nf
    ctx.net_init(dilations)
    ctx.net_set_loss(loss)
    theta = I.net_init_params(nf, seed=seed, dim=ctx.prob.dim) if theta0 is None else np.asarray(theta0)
    ctx.net_set_params(theta.astype(np.float32))
    noise = NoisePairs(ctx, u, field_rms(DU, nf), seed=seed + 1)
    rng = np.random.Generator(np.random.PCG64(seed + 17))
    losses = []
    for it in range(iters):
        step_lr = lr * 0.5 * (1 + np.cos(np.pi * it / iters)) + 1e-5
        if R.shape[0] == 0 or it % noise_every != 1:
            Rb, Xb = noise.batch(batch)
        else:
            idx = torch.as_tensor(rng.choice(R.shape[0], size=min(batch, R.shape[0]), replace=False),
                                  device=R.device)
            Rb, Xb = R.index_select(0, idx).contiguous(), DU.index_select(0, idx).contiguous()
        losses.append(ctx.net_train_step(Rb, Xb, step_lr))
    return ctx.net_get_params(), losses


def train(ctx, R, DU, iters, lr=2e-3, batch=4, seed=0, theta0=None, lr_decay=True, dilations=DILATIONS):
    """Adam on mini-batches of recorded pairs only; returns (theta, per-step losses)."""
    import torch
    nf = ctx.prob.nf
    ctx.net_init(dilations)
    theta = I.net_init_params(nf, seed=seed, dim=ctx.prob.dim) if theta0 is None else np.asarray(theta0)
    ctx.net_set_params(theta.astype(np.float32))
    rng = np.random.Generator(np.random.PCG64(seed + 17))
    npairs = R.shape[0]
    losses = []
    for it in range(iters):
        idx = torch.as_tensor(rng.choice(npairs, size=min(batch, npairs), replace=False), device=R.device)
        Rb = R.index_select(0, idx).contiguous()
        Db = DU.index_select(0, idx).contiguous()
        step_lr = lr * (0.5 * (1 + np.cos(np.pi * it / iters)) if lr_decay else 1.0)
        losses.append(ctx.net_train_step(Rb, Db, max(step_lr, 1e-6)))
    return ctx.net_get_params(), losses


def held_out_loss(ctx, R, DU):
    loss, _ = ctx.net_loss_grad(R.contiguous(), DU.contiguous(), want_grad=False)
    return loss
