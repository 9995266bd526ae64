"""Shared test helpers: device set-up, the oracle side of each workload and
the scaled tolerance.  Imported by tests only."""
from __future__ import annotations

import functools

import numpy as np

import oracle as O
from paper_2405_05155_amd import inputs as I


def scaled_check(gpu, ref, scale, rtol, name):
    """|gpu - ref| <= rtol * max(|ref|, scale) elementwise, where scale is the
    absolute-sum scale sum_j |term_ij| of each output (the error bound of a
    compensated sum of FP32 terms is proportional to it)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.broadcast_to(np.asarray(scale, dtype=np.float64), ref.shape)
    err = np.abs(gpu - ref)
    bound = rtol * np.maximum(np.abs(ref), scale)
    bad = err > bound
    worst = float(np.max(err / np.maximum(bound, 1e-300))) if err.size else 0.0
    assert not bad.any(), f"{name}: {int(bad.sum())}/{bad.size} beyond tolerance, worst err/bound {worst:.3g}"
    return worst


def normwise(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(gpu - ref) / max(np.linalg.norm(ref), 1e-300))


def oracle_box(w):
    return O.make_box(w.dim, lo=w.lo, hi=w.hi, periodic=w.periodic)


def csr_rows_equal(rp_a, col_a, rp_b, col_b, rows=None):
    """Compare CSR a (full, indexed by particle) with CSR b (indexed by
    position in `rows`, or full).  Returns the first differing row or None."""
    rp_a, col_a = np.asarray(rp_a), np.asarray(col_a)
    rp_b, col_b = np.asarray(rp_b), np.asarray(col_b)
    it = range(len(rp_b) - 1)
    for k in it:
        i = rows[k] if rows is not None else k
        a = col_a[rp_a[i]:rp_a[i + 1]]
        b = col_b[rp_b[k]:rp_b[k + 1]]
        if a.shape != b.shape or not np.array_equal(a, b):
            return i
    return None


def two_ring_B(box, pos, h, rc, rows):
    """Oracle B on rows and on all their neighbours (for RHS checks on a
    sample of rows).  Returns (rp_rows, col_rows, B_full) with B_full zero
    outside the ring."""
    rc2 = rc * rc
    rp, col = O.neighbors_grid(box, pos, rc, rc2, rows=rows)
    ring = np.unique(np.concatenate([np.asarray(rows, dtype=np.int64), col.astype(np.int64)]))
    rp2, col2 = O.neighbors_grid(box, pos, rc, rc2, rows=ring)
    n = pos.shape[1]
    dim = box.dim
    return rp, col, ring, rp2, col2


def sample_rows(n, k, seed):
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([[0, n - 1], rng.choice(n, size=min(k, n), replace=False)]))
    return rows.astype(np.int64)


@functools.lru_cache(maxsize=None)
def oracle_relaxed_sphere(nside, kernel=O.LAGUERRE_GAUSS, tol=1e-4, max_iter=400):
    """The oracle's relaxation (kernel LG or Wendland) of the seed-2 sphere
    fill at dx = 1/nside until R < tol or max_iter iterations (a fresh
    neighbour search every iteration).  Returns (workload, box, FP32
    positions, residue of the returned positions); cached: callers must not
    modify the arrays."""
    w = I.sphere_fill(dx=1.0 / nside, seed=2)
    box = O.make_box(3, periodic=(0, 0, 0))
    f = w.fields
    prm = O.relax_params(w.h, f["center"], f["radius"], kernel=kernel)
    pos = w.pos.astype(np.float64)
    u = np.zeros_like(pos)
    rc = 2.0 * w.h
    r = float("nan")
    for _ in range(max_iter):
        rp, col = O.neighbors_grid(box, pos, rc, rc * rc)
        new, u, r, _ = O.relax_step(box, pos, u, prm, rp, col, w.vol)
        if r < tol:
            break
        pos = new
    else:
        rp, col = O.neighbors_grid(box, pos, rc, rc * rc)
        _, _, r, _ = O.relax_step(box, pos, np.zeros_like(pos), prm, rp, col, w.vol)
    return w, box, pos.astype(np.float32), r


def oracle_lg_relaxed_sphere(nside, tol=1e-4, max_iter=400):
    """The oracle's LG relaxation of the seed-2 sphere fill at dx = 1/nside
    until R < tol: (workload, box, FP32 positions)."""
    w, box, pos, _ = oracle_relaxed_sphere(nside, O.LAGUERRE_GAUSS, tol, max_iter)
    return w, box, pos


@functools.lru_cache(maxsize=None)
def oracle_relaxed_circle(ndiv, kernel=O.LAGUERRE_GAUSS, tol=1e-4, max_iter=None, seed=2):
    """The oracle's relaxation of the circle of the error analysis (D = 2,
    dp = D / ndiv, seeded fill jittered by +-0.4 dp) with `kernel` until
    R < tol or max_iter iterations (400 for Wendland, which stalls near
    6e-4; 3000 for LG), a fresh neighbour search every iteration.  Returns
    (workload, box, FP32 positions, residue of the returned positions,
    iterations); cached: callers must not modify the arrays."""
    if max_iter is None:
        max_iter = 400 if kernel == O.WENDLAND else 3000
    w = I.circle_fill(dx=2.0 / ndiv, seed=seed)
    box = O.make_box(2, lo=w.lo + (0.0,), hi=w.hi + (0.0,), periodic=(0, 0, 0))
    f = w.fields
    prm = O.relax_params(w.h, f["center"], f["radius"], kernel=kernel)
    pos = w.pos.astype(np.float64)
    u = np.zeros_like(pos)
    rc = 2.0 * w.h
    r = float("nan")
    it = 0
    for it in range(1, max_iter + 1):
        rp, col = O.neighbors_grid(box, pos, rc, rc * rc)
        new, u, r, _ = O.relax_step(box, pos, u, prm, rp, col, w.vol)
        if r < tol:
            break
        pos = new
    else:
        rp, col = O.neighbors_grid(box, pos, rc, rc * rc)
        _, _, r, _ = O.relax_step(box, pos, np.zeros_like(pos), prm, rp, col, w.vol)
    return w, box, pos.astype(np.float32), r, it
