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


# --------------------------------------------------------------------------- #
# 3D network trained on crops of solver pairs from 3D and 2D runs
# --------------------------------------------------------------------------- #
def embed_2d(V2, nx, nz, ny):
    """2D vectors (count, 4 nz nx) of fields (u, w, p, theta) -> y-invariant 3D
    vectors (count, 5 nz ny nx) of fields (u, v = 0, w, p, theta).  A 2D pair
    (J2 x = r) embeds as a 3D pair of the same spacing and time step: the 3D
    operator acts on a y-invariant field with v = 0 as the 2D one does on its
    x-z slice."""
    import torch
    c = V2.shape[0]
    a = V2.reshape(c, 4, nz, 1, nx)
    out = torch.zeros((c, 5, nz, ny, nx), dtype=V2.dtype, device=V2.device)
    out[:, 0] = a[:, 0]
    out[:, 2:] = a[:, 1:]
    return out.reshape(c, -1)


def crops(V, grid, crop, idx, starts):
    """Crops of size crop = (cx, cy, cz) of the vectors V[idx] on grid =
    (nf, nz, ny, nx), one start (x0, y0, z0) per vector; returns (len(idx), n_crop)."""
    import torch
    nf, nz, ny, nx = grid
    cx, cy, cz = crop
    out = []
    for i, (x0, y0, z0) in zip(idx, starts):
        g = V[int(i)].view(nf, nz, ny, nx)
        out.append(g[:, z0:z0 + cz, y0:y0 + cy, x0:x0 + cx].reshape(-1))
    return torch.stack(out).contiguous()


def random_starts(rng, grid, crop, k, centers=None):
    """Crop starts: uniform over the grid, or around the given centres (x, y, z)
    with a jitter of a quarter crop, clamped to the grid."""
    nf, nz, ny, nx = grid
    cx, cy, cz = crop
    out = []
    for q in range(k):
        if centers is None:
            out.append((int(rng.integers(0, nx - cx + 1)), int(rng.integers(0, ny - cy + 1)),
                        int(rng.integers(0, nz - cz + 1))))
            continue
        c = centers[q]
        st = []
        for ci, cn, n in zip(c, (cx, cy, cz), (nx, ny, nz)):
            j = cn // 4
            s0 = ci - cn // 2 + int(rng.integers(-j, j + 1))
            st.append(int(min(max(s0, 0), n - cn)))
        out.append(tuple(st))
    return out


def support_centers(V, grid):
    """Grid point (x, y, z) of the largest summed field magnitude of each vector:
    Krylov directions started from a localised residual vanish far from it, and a
    crop must hold some of the direction to carry a relative loss."""
    nf, nz, ny, nx = grid
    a = V.view(V.shape[0], nf, nz * ny * nx).abs().sum(dim=1)
    idx = a.argmax(dim=1).cpu().numpy()
    return [(int(i % nx), int((i // nx) % ny), int(i // (nx * ny))) for i in idx]


def train_3d_crops(ctx, sources, iters=600, lr=2e-3, batch=4, seed=0, noise=None, theta0=None):
    """Adam on crops of 3D pairs.  sources: list of (R, DU, grid, crop) with R, DU
    float32 device tensors (count, n) on grid = (nf, nz, ny, nx) and crop =
    (cx, cy, cz); noise: optional (NoisePairs on the context's grid, crop) whose
    full-grid pairs are cropped.  Steps cycle through the sources (and the noise
    pairs); returns (theta, losses)."""
    nf = ctx.prob.nf
    ctx.net_init()
    theta = I.net_init_params(nf, seed=seed, dim=3) if theta0 is None else np.asarray(theta0)
    ctx.net_set_params(theta.astype(np.float32))
    rng = np.random.Generator(np.random.PCG64(seed + 23))
    kinds = list(range(len(sources))) + (["noise"] if noise is not None else [])
    centers = [support_centers(DU, grid) for (R, DU, grid, crop) in sources]
    p = ctx.prob
    full = (p.nf, p.nz, p.ny, p.nx)
    losses = []
    for it in range(iters):
        step_lr = lr * 0.5 * (1 + np.cos(np.pi * it / iters)) + 1e-5
        kind = kinds[it % len(kinds)]
        if kind == "noise":
            gen, crop = noise
            Rn, Xn = gen.batch(1)
            st = random_starts(rng, full, crop, batch)
            Rb = crops(Rn, full, crop, [0] * batch, st)
            Xb = crops(Xn, full, crop, [0] * batch, st)
        else:
            R, DU, grid, crop = sources[kind]
            idx = rng.choice(R.shape[0], size=min(batch, R.shape[0]), replace=False)
            st = random_starts(rng, grid, crop, len(idx), [centers[kind][i] for i in idx])
            Rb, Xb = crops(R, grid, crop, idx, st), crops(DU, grid, crop, idx, st)
        losses.append(ctx.net_train_step(Rb, Xb, step_lr, crop=crop))
    return ctx.net_get_params(), losses
