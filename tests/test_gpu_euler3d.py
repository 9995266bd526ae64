"""GPU parity of the 3-D Eulerian Heun stages (Eq. 19 with Eq. 28, the
limited linearised solver of Eqs. 26-27; two-stage Heun steps) against the
FP64 oracle, in the stage kernels and launch configuration that the 200^3
Taylor-Green workload runs (fixed-stride rows, lanes per particle from the
row length, packed 64-byte per-particle records), and the equal-accuracy
check of the truncated kernel in 3-D.

Bars: one step per element, |inc_gpu - inc_ref| <= 1e-5 (|inc_ref| +
1.5 dt S) + 4 eps |state| (the increment of one step is a few hundred ulps
of the stored FP32 state); runs of many steps normwise (relative L2 <=
1e-3).  S is the absolute-sum scale of a particle's rates, for the
momentum rows the largest of its components' scales: the pair terms pass
through B_i + B_j, whose FP32 entries carry errors of order eps |B| also
where the exact entry vanishes (the off-diagonal entries on a lattice), so
each component's error follows the scale of all of them (m_z starts at zero
on the Taylor-Green field and its own scale is the smallest).
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle as O
from paper_2405_05155_amd import inputs as I
from tests.gpu_helpers import normwise, oracle_box, sample_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS32 = float(np.finfo(np.float32).eps)


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_05155_amd import sph
    sph.lib()
    return sph


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _params(S, w, dt):
    f = w.fields
    return (S.euler_params(c=f["c"], rho0=f["rho0_eos"], rho_ref=f["rho_ref"], eta=f["eta"], mu=f["mu"], dt=dt),
            O.euler_params(c=f["c"], rho0=f["rho0_eos"], eta=f["eta"], mu=f["mu"], dt=dt))


def _check_increment(new_g, old, new_o, scale, dt):
    """scale: S per element ([n]) or per component ([d][n], reduced to the
    largest component of each particle)."""
    scale = np.asarray(scale, dtype=np.float64)
    if scale.ndim == 2:
        scale = scale.max(axis=0)
    inc_g, inc_o = new_g - old, new_o - old
    bound = 1e-5 * (np.abs(inc_o) + 1.5 * dt * scale) + 4 * EPS32 * np.abs(new_o)
    ratio = np.abs(inc_g - inc_o) / bound
    k = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    assert not (ratio > 1).any(), (f"{int((ratio > 1).sum())} of {ratio.size} beyond the bar, worst "
                                   f"{float(ratio[k]):.3g} at {k}: gpu {new_g[k]!r} oracle {new_o[k]!r} "
                                   f"old {old[k]!r} bound {bound[k]:.3g}")


@pytest.mark.parametrize("nu", [0.0, 0.01])
@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_euler_heun_3d_steps(S, kappa, nu):
    """32^3 Taylor-Green jittered by +-0.05 dx (non-uniform B): one Heun step
    per element, then 50 steps normwise, against the oracle's Heun steps."""
    w = I.taylor_green_3d(nside=32, nu=nu, jitter=0.05, seed=11)
    dt = w.meta["dt"]
    box = oracle_box(w)
    rc = kappa * w.h
    rp, col = O.neighbors_grid(box, w.pos, rc, rc * rc)
    Bo, nd = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol)
    assert nd == 0
    pg, po = _params(S, w, dt)
    drho0 = w.fields["drho"].astype(np.float64)
    mom0 = w.fields["mom"].astype(np.float64)
    rho0 = 1.0 + drho0

    ctx = S.Context(3)
    ctx.build_cells(S.Domain(dim=3, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=w.periodic), dev(w.pos))
    ctx.correction_B(dev(w.vol))
    d, m = dev(w.fields["drho"]), dev(w.fields["mom"])
    ctx.euler_step(pg, d, m, 1)
    r1, m1 = O.euler_heun(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho0, mom0, 1)
    _, _, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho0, mom0)
    _check_increment(host(d).astype(np.float64), drho0, r1 - 1.0, s_dr, dt)
    _check_increment(host(m).astype(np.float64), mom0, m1, s_dm, dt)

    ctx.euler_step(pg, d, m, 49)
    r50, m50 = O.euler_heun(box, w.pos, w.h, rp, col, w.vol, Bo, po, r1, m1, 49)
    ctx.close()
    assert normwise(host(m), m50) < 1e-3
    assert normwise(host(d), r50 - 1.0) < 1e-3


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_euler_heun_3d_step_full_size_sampled(S, kappa):
    """One Heun step of the 200^3 Taylor-Green workload (8M particles) in the
    launch configuration its timed run uses, on 24 sampled particles: the
    oracle evaluates the first stage on the samples and their neighbours,
    then the second stage on the samples, with B on the two rings of
    neighbours around them."""
    w = I.taylor_green_3d(nside=200)
    box = oracle_box(w)
    rc = kappa * w.h
    dt = w.meta["dt"]
    rows = sample_rows(w.n, 24, seed=13)
    rp_s, col_s = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=rows)
    ring1 = np.unique(np.concatenate([rows, col_s.astype(np.int64)]))
    rp_1, col_1 = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=ring1)
    ring2 = np.unique(np.concatenate([ring1, col_1.astype(np.int64)]))
    rp_2, col_2 = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=ring2)
    B_2, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp_2, col_2, w.vol, rows=ring2)
    B_full = np.zeros((w.n, 3, 3))
    B_full[ring2] = B_2
    pg, po = _params(S, w, dt)
    drho0 = w.fields["drho"].astype(np.float64)
    mom0 = w.fields["mom"].astype(np.float64)
    rho0 = 1.0 + drho0
    d1, m1, _, _ = O.euler_rhs(box, w.pos, w.h, rp_1, col_1, w.vol, B_full, po, rho0, mom0, rows=ring1)
    rho_s, mom_s = rho0.copy(), mom0.copy()
    rho_s[ring1] += dt * d1
    mom_s[:, ring1] += dt * m1
    d2, m2, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp_s, col_s, w.vol, B_full, po, rho_s, mom_s, rows=rows)
    rho_n = 0.5 * (rho0[rows] + rho_s[rows] + dt * d2)
    mom_n = 0.5 * (mom0[:, rows] + mom_s[:, rows] + dt * m2)

    ctx = S.Context(3)
    ctx.build_cells(S.Domain(dim=3, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=w.periodic), dev(w.pos))
    ctx.correction_B(dev(w.vol))
    d, m = dev(w.fields["drho"]), dev(w.fields["mom"])
    ctx.euler_step(pg, d, m, 1)
    assert ctx.euler_path() == S.PATH_WINDOWS  # the stage kernels of the timed run
    dg, mg = host(d)[rows].astype(np.float64), host(m)[:, rows].astype(np.float64)
    ctx.close()
    _check_increment(dg, drho0[rows], rho_n - 1.0, s_dr, dt)
    _check_increment(mg, mom0[:, rows], mom_n, s_dm, dt)


def _ke_rate(rho, mom, dr, dm, vol):
    """-(dK/dt)/K for K = sum_i V_i |m_i|^2 / (2 rho_i) from the rates."""
    V = vol.astype(np.float64)
    m2 = (mom ** 2).sum(0)
    K = np.sum(V * m2 / (2 * rho))
    dK = np.sum(V * ((mom * dm).sum(0) / rho - m2 * dr / (2 * rho ** 2)))
    return -dK / K


def test_truncated_kernel_equal_accuracy_taylor_green_3d(S):
    """The 3-D Taylor-Green field is an eigenfunction of the Laplacian
    (lap u = -12 pi^2 u), so its kinetic energy starts to decay at exactly
    24 pi^2 nu.  The decay rate of the GPU rates at t = 0 on 48^3 is within
    25% of it at both cut-offs (the rest is the limiter's dissipation, which
    falls with resolution), and the truncated kernel's error is at most
    1.10x the standard kernel's."""
    w = I.taylor_green_3d(nside=48)
    f = w.fields
    exact = 24 * math.pi ** 2 * f["nu"]
    rho = 1.0 + f["drho"].astype(np.float64)
    mom = f["mom"].astype(np.float64)
    pg, _ = _params(S, w, 0.0)
    err = {}
    for kappa in (1.6, 2.0):
        ctx = S.Context(3)
        ctx.build_cells(S.Domain(dim=3, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=w.periodic), dev(w.pos))
        ctx.correction_B(dev(w.vol))
        dr, dm = ctx.euler_rhs(pg, dev(f["drho"]), dev(f["mom"]))
        rate = _ke_rate(rho, mom, host(dr).astype(np.float64), host(dm).astype(np.float64), w.vol)
        ctx.close()
        err[kappa] = abs(rate / exact - 1.0)
    assert err[1.6] < 0.25 and err[2.0] < 0.25, err
    assert err[1.6] <= 1.10 * err[2.0], err


def _run_paths(S, w, kappa, dt, steps):
    """Rates, then `steps` Heun steps, of the bound configuration; returns
    (rates, state after the steps, path of the last call)."""
    pg, _ = _params(S, w, dt)
    ctx = S.Context(3)
    ctx.build_cells(S.Domain(dim=3, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=w.periodic), dev(w.pos))
    ctx.correction_B(dev(w.vol))
    d, m = dev(w.fields["drho"]), dev(w.fields["mom"])
    dr, dm = ctx.euler_rhs(pg, d, m)
    path_rhs = ctx.euler_path()
    ctx.euler_step(pg, d, m, steps)
    path = ctx.euler_path()
    out = [host(dr).copy(), host(dm).copy(), host(d).copy(), host(m).copy()]
    ctx.close()
    assert path_rhs == path
    return out, path


@pytest.mark.parametrize("kappa,threads", [(1.6, "256"), (1.6, "512"), (2.0, "256"), (2.0, "512")])
def test_euler_3d_windows_bit_identical(S, kappa, threads, monkeypatch):
    """The stage kernels that read the neighbour records from LDS windows
    against the kernels that gather them: the same rates and the same state
    after 5 Heun steps, bit for bit (same pairs in the same order, same
    sums), for workgroups of 256 and 512 threads (blocks of 64 and 128
    slots), on a jittered 30^3 Taylor-Green field (27,000 particles: the
    last block is ragged, the rows uneven)."""
    w = I.taylor_green_3d(nside=30, nu=0.01, jitter=0.05, seed=21)
    monkeypatch.setenv("SPH_EULER_WINDOW_THREADS", threads)
    monkeypatch.setenv("SPH_EULER_WINDOW", "0")
    ref, p0 = _run_paths(S, w, kappa, w.meta["dt"], 5)
    monkeypatch.delenv("SPH_EULER_WINDOW")
    got, p1 = _run_paths(S, w, kappa, w.meta["dt"], 5)
    assert p0 == S.PATH_RECORDS and p1 == S.PATH_WINDOWS, (p0, p1)
    for a, b, name in zip(got, ref, ("drho_dt", "dmom_dt", "drho", "mom")):
        assert np.array_equal(a, b), (name, int(np.sum(a != b)))


def test_euler_3d_window_fallbacks(S, monkeypatch):
    """Configurations the windows do not serve run the gathering kernels:
    one or two lanes per particle (short rows), CSR rows, and blocks whose
    window would exceed 1024 records (h = 2 dx: rows of ~270 entries,
    windows of ~1,300 records for 64 slots)."""
    w = I.taylor_green_3d(nside=24, nu=0.01, jitter=0.05, seed=3)
    for lanes in ("1", "2"):
        monkeypatch.setenv("SPH_EULER_LANES", lanes)
        _, p = _run_paths(S, w, 1.6, w.meta["dt"], 1)
        assert p == S.PATH_RECORDS, lanes
    monkeypatch.delenv("SPH_EULER_LANES")
    wide = dataclasses.replace(w, h=2.0 / 24)
    monkeypatch.setenv("SPH_EULER_WINDOW_THREADS", "256")
    _, p = _run_paths(S, wide, 2.0, w.meta["dt"], 1)
    assert p == S.PATH_RECORDS
    monkeypatch.delenv("SPH_EULER_WINDOW_THREADS")
    monkeypatch.setenv("SPH_PAIR_ROWS", "csr")
    _, p = _run_paths(S, w, 1.6, w.meta["dt"], 1)
    assert p == S.PATH_RECORDS


def test_euler_3d_windows_rebuilt_with_the_configuration(S):
    """One context bound to a new configuration (another cut-off, then
    another field size) rebuilds its windows: each call's rates equal a
    fresh context's bit for bit."""
    cases = [(I.taylor_green_3d(nside=24, nu=0.01, jitter=0.05, seed=5), 1.6),
             (I.taylor_green_3d(nside=24, nu=0.01, jitter=0.05, seed=5), 2.0),
             (I.taylor_green_3d(nside=28, nu=0.01, jitter=0.05, seed=6), 1.6)]
    shared = S.Context(3)
    for w, kappa in cases:
        pg, _ = _params(S, w, w.meta["dt"])
        got = []
        for ctx in (shared, S.Context(3)):
            ctx.build_cells(S.Domain(dim=3, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=w.periodic), dev(w.pos))
            ctx.correction_B(dev(w.vol))
            dr, dm = ctx.euler_rhs(pg, dev(w.fields["drho"]), dev(w.fields["mom"]))
            assert ctx.euler_path() == S.PATH_WINDOWS
            got.append((host(dr).copy(), host(dm).copy()))
            if ctx is not shared:
                ctx.close()
        assert np.array_equal(got[0][0], got[1][0]) and np.array_equal(got[0][1], got[1][1]), (w.n, kappa)
    shared.close()
