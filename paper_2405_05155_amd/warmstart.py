"""Relaxation drivers: plain relaxation to a residue threshold, training-set
generation from its trajectory, training of the warm-start network with the
library's kernels, and warm-started relaxation.

Host-side control only (loops, residue checks, accept/revert, batching):
every arithmetic step runs in libsph.so.  The learned step can only shorten
a run: it is applied every `every` iterations, the residue is re-evaluated,
and the move is reverted if the residue rose; the plain relaxation always
finishes the job and judges the residue.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import sph as S
from .inputs import Workload


@dataclass
class RelaxRun:
    iterations: int
    seconds: float
    residue: float
    history: list = field(default_factory=list)
    accepted: int = 0
    attempted: int = 0


def setup(w: Workload, kernel=S.LAGUERRE_GAUSS):
    f = w.fields
    dom = S.Domain(dim=3, h=w.h, kappa=2.0, lo=w.lo, hi=w.hi, periodic=(0, 0, 0), kernel=S.LAGUERRE_GAUSS)
    prm = S.relax_params(f["center"], f["radius"], p0=f["p0"], rho=f["rho"], kernel=kernel)
    return dom, prm


def relax_plain(ctx: S.Context, w: Workload, tol=1e-4, check_every=10, max_iter=20000, snapshot_every=0,
                snapshot_until=0, pos=None):
    """Relax until the residue (checked every `check_every` iterations) is
    below tol.  Returns (RelaxRun, final positions, snapshots dict k -> pos)."""
    dom, prm = setup(w)
    pos = torch.as_tensor(w.pos, device="cuda").clone() if pos is None else pos
    vol = torch.as_tensor(w.vol, device="cuda")
    u = torch.zeros_like(pos)
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    snaps = {}
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    while it < max_iter:
        if snapshot_every and it % snapshot_every == 0 and it <= snapshot_until:
            snaps[it] = pos.clone()
        step = check_every
        if snapshot_every:
            step = min(step, snapshot_every - it % snapshot_every)
        ctx.relax_step(dom, prm, pos, u, vol, step, res)
        it += step
        if it % check_every == 0:
            r = float(res.item())
            hist.append((it, r))
            if r < tol:
                break
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    return RelaxRun(it, secs, hist[-1][1] if hist else float("nan"), hist), pos, snaps


def relax_warm(ctx: S.Context, w: Workload, params, tol=1e-4, check_every=10, every=20, max_iter=20000,
               stop_mlp_below=0.0, max_rejects=1, reset_u=True):
    """Plain relaxation with the learned move tried every `every` iterations
    (kept only if it lowers the residue; the carried displacement is reset
    after an accepted move).  After `max_rejects` consecutive rejections the
    learned move is no longer tried (a try costs about a dozen iterations:
    features, inference and two residue evaluations)."""
    dom, prm = setup(w)
    pos = torch.as_tensor(w.pos, device="cuda").clone()
    vol = torch.as_tensor(w.vol, device="cuda")
    u = torch.zeros_like(pos)
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    acc = att = rej = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    r_now = None
    while it < max_iter:
        if it % every == 0 and rej < max_rejects and (r_now is None or r_now > stop_mlp_below):
            r0, _ = ctx.relax_residue(dom, prm, pos, vol, want_g=False)
            saved = pos.clone()
            ctx.mlp_apply(dom, prm, pos, params)
            r1, _ = ctx.relax_residue(dom, prm, pos, vol, want_g=False)
            att += 1
            if float(r1.item()) < float(r0.item()):
                acc += 1
                rej = 0
                if reset_u:
                    u.zero_()
            else:
                rej += 1
                pos.copy_(saved)
        ctx.relax_step(dom, prm, pos, u, vol, check_every, res)
        it += check_every
        r_now = float(res.item())
        hist.append((it, r_now))
        if r_now < tol:
            break
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    return RelaxRun(it, secs, hist[-1][1] if hist else float("nan"), hist, acc, att), pos


def training_set(ctx: S.Context, w: Workload, snaps: dict, final_pos, horizon=None, ks=None):
    """Features of the snapshots ks (default: all) and targets
    (r_{k+horizon} - r_k)/h, or (r_final - r_k)/h when horizon is None."""
    dom, prm = setup(w)
    feats, targs = [], []
    for k in (sorted(snaps) if ks is None else ks):
        p = snaps[k]
        nxt = final_pos if horizon is None else snaps[k + horizon]
        feats.append(ctx.mlp_features(dom, prm, p))
        targs.append(ctx.mlp_targets(p, nxt, w.h))
    return torch.cat(feats), torch.cat(targs)


def train(ctx: S.Context, feat, target, epochs=50, batch=65536, lr=1e-3, weight_decay=0.01, seed=0, init=None,
          log_every=0):
    """AdamW on shuffled mini-batches (the last partial batch of an epoch is
    dropped).  Returns (params, per-epoch mean loss)."""
    n = feat.shape[0]
    g = torch.Generator(device="cuda").manual_seed(seed)
    params = torch.as_tensor(init, device="cuda").clone()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    adam = S.adamw_params(lr=lr, weight_decay=weight_decay)
    step = 0
    losses = []
    nb = n // batch
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device="cuda")
        if nb == 0:
            losses.append(float("nan"))
            continue
        # the nb steps of the epoch in one call; batches gathered by row index inside the kernel
        ls = ctx.mlp_train_epoch(adam, step + 1, params, m, v, perm, feat, target, batch)
        step += nb
        losses.append(float(ls.double().sum().item()) / nb)
        if log_every and (ep + 1) % log_every == 0:
            print(f"epoch {ep + 1} loss {losses[-1]:.4e}", flush=True)
    return params, losses
