"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
identical seeded inputs.

Neighbour sets must match bit for bit.  FP32 fields must satisfy, per
element, |gpu - ref| <= 1e-5 max(|ref|, S) with S the absolute-sum scale
sum_j |term_ij| of that output (the error bound of a compensated sum of
FP32 terms scales with it, not with the possibly cancelled result); runs
of many steps are compared normwise (relative L2 <= 1e-3).
"""
import numpy as np
import pytest

import oracle as O
from paper_2405_05155_amd import inputs as I
from tests.gpu_helpers import (csr_rows_equal, normwise, oracle_box, oracle_lg_relaxed_sphere, sample_rows,
                               scaled_check)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-5


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


def gpu_ctx(S, w, kappa, kernel=0):
    ctx = S.Context(w.dim)
    dom = S.Domain(dim=w.dim, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=w.periodic, kernel=kernel)
    ctx.build_cells(dom, dev(w.pos))
    return ctx


# ------------------------------------------------------------------ neighbours

@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_neighbours_single_step_bit_exact(S, seed, kappa):
    w = I.single_step_2d(seed=seed)
    ctx = gpu_ctx(S, w, kappa)
    rp, col = ctx.neighbors()
    rc = kappa * w.h
    rp_o, col_o = O.neighbors_grid(oracle_box(w), w.pos, rc, rc * rc)
    assert np.array_equal(host(rp), rp_o)
    assert np.array_equal(host(col), col_o)


def test_neighbours_exact_ties(S):
    t = I.adversarial_ties_2d(kappa=2.0)
    ctx = gpu_ctx(S, t, 2.0)
    rp, col = ctx.neighbors()
    rc = 2.0 * t.h
    rp_o, col_o = O.neighbors_brute(oracle_box(t), t.pos, rc * rc)
    assert np.array_equal(host(rp), rp_o) and np.array_equal(host(col), col_o)


@pytest.mark.parametrize("dim,n,periodic", [(3, 1000, True), (3, 1001, False), (2, 777, False), (2, 1, True)])
def test_neighbours_random_ragged(S, dim, n, periodic):
    w = I.random_points(n, dim, seed=n, periodic=periodic)
    for kappa in (2.0, 1.6):
        if periodic and 3 * kappa * w.h * 1.001 > 1.0:
            continue
        ctx = gpu_ctx(S, w, kappa)
        rp, col = ctx.neighbors()
        rc = kappa * w.h
        rp_o, col_o = O.neighbors_brute(oracle_box(w), w.pos, rc * rc)
        assert np.array_equal(host(rp), rp_o) and np.array_equal(host(col), col_o)


def test_neighbours_empty_configuration(S):
    ctx = S.Context(2)
    ctx.build_cells(S.Domain(dim=2, h=0.05, kappa=2.0), torch.empty((2, 0), device="cuda"))
    rp, col = ctx.neighbors()
    assert host(rp).tolist() == [0] and col.numel() == 0


def test_invalid_arguments_raise(S):
    ctx = S.Context(2)
    with pytest.raises(S.SphError):
        ctx.build_cells(S.Domain(dim=2, h=0.3, kappa=2.0), dev(np.zeros((2, 4))))  # box < 3 kappa h
    # nothing bound: the C layer refuses before enqueueing anything
    assert S.lib().sph_kernel_sum(ctx._h, None, None) == S.SPH_ERR_STATE
    assert b"no configuration bound" in S.lib().sph_last_error(ctx._h)
    with pytest.raises(S.SphError):
        ctx.build_cells(S.Domain(dim=3, h=0.01, kappa=2.0), dev(np.zeros((2, 4))))  # dim mismatch


# ------------------------------------------------------------------ kernel sum, B, gradient

def _c0_oracle(w, kappa):
    box = oracle_box(w)
    rc = kappa * w.h
    rp, col = O.neighbors_grid(box, w.pos, rc, rc * rc)
    B, nd = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol)
    return box, rp, col, B, nd


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_kernel_sum_and_table1(S, kappa):
    w = I.single_step_2d(seed=0)
    ctx = gpu_ctx(S, w, kappa)
    out = host(ctx.kernel_sum(dev(w.vol)))
    box, rp, col, _, _ = _c0_oracle(w, kappa)
    ref = O.kernel_sum(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol)
    scaled_check(out, ref, ref, RTOL, "kernel sum")
    # Table 1 lattice row on the GPU: L2(f=1) = 0.010 (SW), 0.006 (TW)
    lat = I.periodic_square_case(32, 2, 1.3, 0.0, None, "lattice")
    ctx = gpu_ctx(S, lat, kappa)
    s = host(ctx.kernel_sum(dev(lat.vol))).astype(np.float64)
    err = np.sqrt(np.mean((s - 1.0) ** 2))
    assert round(err, 3) == {2.0: 0.010, 1.6: 0.006}[kappa]


@pytest.mark.parametrize("seed", [0, 3])
@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_correction_matrix(S, seed, kappa):
    w = I.single_step_2d(seed=seed)
    ctx = gpu_ctx(S, w, kappa)
    B, B64, nd = ctx.correction_B(dev(w.vol), want_fp64=True)
    box, rp, col, Bo, ndo = _c0_oracle(w, kappa)
    assert nd == ndo == 0
    scale = np.abs(Bo).reshape(w.n, -1).max(axis=1)[:, None, None]
    scaled_check(host(B), Bo, scale, RTOL, "B fp32")
    scaled_check(host(B64), Bo, scale, RTOL, "B fp64")
    assert np.array_equal(host(B), np.transpose(host(B), (0, 2, 1)))


def _grad_scale(w, box, rp, col, Bo, f, h):
    """||B_i||_max * sum_j |f_j - f_i| |dW/dr| V_j (per row, all components)."""
    pos = w.pos.astype(np.float64)
    n = w.n
    rows = np.repeat(np.arange(n), np.diff(rp))
    d = pos[:, rows] - pos[:, col]
    for a in range(w.dim):  # minimum image on the workload's periodic axes
        if w.periodic[a]:
            L = w.hi[a] - w.lo[a]
            d[a] -= L * np.round(d[a] / L)
    r = np.sqrt((d ** 2).sum(0))
    t = np.abs(f[col] - f[rows]) * np.abs(O.kernel_dWdr(O.WENDLAND, w.dim, h, r)) * w.vol[col]
    s = np.bincount(rows, weights=t, minlength=n)
    return s * np.abs(Bo).reshape(n, -1).max(axis=1) * w.dim


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_corrected_gradient(S, kappa):
    w = I.single_step_2d(seed=1)
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    box, rp, col, Bo, _ = _c0_oracle(w, kappa)
    rho = 1.0 + w.fields["drho"].astype(np.float64)
    fields = {"rho": w.fields["drho"], "ux": w.fields["mom"][0] / rho, "uy": w.fields["mom"][1] / rho,
              "p": (100.0 * rho)}
    for name, f in fields.items():
        f32 = np.asarray(f, dtype=np.float32)
        g = host(ctx.gradient(dev(f32)))
        ref = O.gradient(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol, Bo, f32)
        scale = _grad_scale(w, box, rp, col, Bo, f32.astype(np.float64), w.h)
        scaled_check(g, ref, scale[None, :], RTOL, f"gradient {name}")


@pytest.mark.parametrize("corrected", [False, True])
@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_gradient_error_analysis_lattice(S, kappa, corrected):
    """The error analysis of Sec. 2.3.3 on the lattice (Fig. 2, upper panel):
    the GPU's gradient of f = exp(-x^2/0.1) at dp = D/10, D/20, D/40, with
    the correction or with B = I, per element against the oracle, and its
    L2 error of df/dx (Eq. 10) within 1e-4 of the oracle's."""
    for nside in (10, 20, 40):
        w = I.gradient_lattice_2d(nside)
        ctx = gpu_ctx(S, w, kappa)
        box, rp, col, Bo, _ = _c0_oracle(w, kappa)
        if corrected:
            ctx.correction_B(dev(w.vol))
        else:
            Bo = np.tile(np.eye(2), (w.n, 1, 1))
            ctx.set_correction(dev(w.vol), dev(Bo.astype(np.float32)))
        f = w.fields["f"]
        g = host(ctx.gradient(dev(f)))
        ref = O.gradient(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol, Bo, f)
        scale = _grad_scale(w, box, rp, col, Bo, f.astype(np.float64), w.h)
        scaled_check(g, ref, scale[None, :], RTOL, f"gradient {nside}")
        ex = w.fields["dfdx"]
        e_gpu = np.linalg.norm(g[0] - ex) / np.linalg.norm(ex)
        e_ref = np.linalg.norm(ref[0] - ex) / np.linalg.norm(ex)
        assert abs(e_gpu - e_ref) < 1e-4 * e_ref


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_gradient_on_lg_relaxed_sphere(S, kappa):
    """The gradient of the error analysis's test function on an LG-relaxed
    sphere (the oracle's relaxation of the dx = 1/32 fill), with the
    correction and with B = I, per element against the oracle."""
    w, box, pos = oracle_lg_relaxed_sphere(32)
    f, _ = I.sphere_gradient_fields(pos, w.fields["center"], w.fields["radius"])
    f = f.astype(np.float32)
    rc = kappa * w.h
    rp, col = O.neighbors_grid(box, pos, rc, rc * rc)
    Bc, _ = O.correction_B(box, pos, O.WENDLAND, w.h, rp, col, w.vol)
    ctx = S.Context(3)
    ctx.build_cells(S.Domain(dim=3, h=w.h, kappa=kappa, periodic=(0, 0, 0)), dev(pos))
    w2 = I.Workload(name="relaxed", dim=3, pos=pos, vol=w.vol, h=w.h, lo=w.lo, hi=w.hi, periodic=w.periodic)
    for corrected in (False, True):
        if corrected:
            ctx.correction_B(dev(w.vol))
            B = Bc
        else:
            B = np.tile(np.eye(3), (w.n, 1, 1))
            ctx.set_correction(dev(w.vol), dev(B.astype(np.float32)))
        g = host(ctx.gradient(dev(f)))
        ref = O.gradient(box, pos, O.WENDLAND, w.h, rp, col, w.vol, B, f)
        scale = _grad_scale(w2, box, rp, col, B, f.astype(np.float64), w.h)
        scaled_check(g, ref, scale[None, :], RTOL, f"gradient corrected={corrected}")


# ------------------------------------------------------------------ Eulerian RHS

def _euler_prm(S, w, dt=0.0):
    f = w.fields
    return (S.euler_params(c=f["c"], rho0=f["rho0_eos"], rho_ref=f["rho_ref"], eta=f["eta"], mu=f["mu"], dt=dt),
            O.euler_params(c=f["c"], rho0=f["rho0_eos"], eta=f["eta"], mu=f["mu"], dt=dt))


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("kappa", [2.0, 1.6])
@pytest.mark.parametrize("mu", [0.0, 0.01])
def test_euler_rhs_single_step(S, seed, kappa, mu):
    w = I.single_step_2d(seed=seed)
    w.fields["mu"] = mu
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    pg, po = _euler_prm(S, w)
    dr, dm = ctx.euler_rhs(pg, dev(w.fields["drho"]), dev(w.fields["mom"]))
    box, rp, col, Bo, _ = _c0_oracle(w, kappa)
    rho = w.fields["rho_ref"] + w.fields["drho"].astype(np.float64)
    r_dr, r_dm, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho, w.fields["mom"])
    scaled_check(host(dr), r_dr, s_dr, RTOL, "drho/dt")
    scaled_check(host(dm), r_dm, s_dm, RTOL, "dmom/dt")


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_euler_heun_steps_taylor_green(S, kappa):
    w = I.taylor_green_2d(nside=64, nu=0.01)
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    dt = w.meta["dt"]
    pg, po = _euler_prm(S, w, dt)
    box, rp, col, Bo, _ = _c0_oracle(w, kappa)
    drho0 = w.fields["drho"].astype(np.float64)
    mom0 = w.fields["mom"].astype(np.float64)
    rho0 = 1.0 + drho0
    # one step: the increment matches to 1e-5 of itself plus the FP32
    # resolution of the stored state (the increment of one step is only
    # ~1e3 ulps of the state)
    d = dev(w.fields["drho"])
    m = dev(w.fields["mom"])
    ctx.euler_step(pg, d, m, 1)
    r1, m1 = O.euler_heun(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho0, mom0, 1)
    eps = np.finfo(np.float32).eps
    _, _, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho0, mom0)
    inc_g, inc_o = host(d) - drho0, (r1 - 1.0) - drho0
    assert np.all(np.abs(inc_g - inc_o) <= 1e-5 * (np.abs(inc_o) + 1.5 * dt * s_dr) + 4 * eps * np.abs(r1 - 1.0))
    inc_g, inc_o = host(m) - mom0, m1 - mom0
    assert np.all(np.abs(inc_g - inc_o) <= 1e-5 * (np.abs(inc_o) + 1.5 * dt * s_dm) + 4 * eps * np.abs(m1))
    # many steps: normwise 1e-3 on the state
    ctx.euler_step(pg, d, m, 99)
    r100, m100 = O.euler_heun(box, w.pos, w.h, rp, col, w.vol, Bo, po, r1, m1, 99)
    assert normwise(host(m), m100) < 1e-3
    assert normwise(host(d), r100 - 1.0) < 1e-3


@pytest.mark.parametrize("rows", ["batch2", "batch4", "batch8", "ell", "csr"])
@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_euler_rhs_row_layouts(S, rows, kappa, monkeypatch):
    """Each row layout of the per-particle kernel against the oracle: short
    rows batched per lane (2, 4 or 8 lanes per particle; 2 lanes only where
    six entries per lane cover the row), the pipelined loop over fixed-stride
    rows and over the CSR rows."""
    env = {"batch2": {"SPH_EULER_BATCH_LANES": "2"}, "batch4": {"SPH_EULER_BATCH_LANES": "4"},
           "batch8": {"SPH_EULER_BATCH_LANES": "8"},
           "ell": {"SPH_EULER_BATCH_LANES": "0"},
           "csr": {"SPH_EULER_BATCH_LANES": "0", "SPH_PAIR_ROWS": "csr"}}[rows]
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    w = I.single_step_2d(seed=1)
    w.fields["mu"] = 0.01
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    pg, po = _euler_prm(S, w)
    dr, dm = ctx.euler_rhs(pg, dev(w.fields["drho"]), dev(w.fields["mom"]))
    box, rp, col, Bo, _ = _c0_oracle(w, kappa)
    rho = w.fields["rho_ref"] + w.fields["drho"].astype(np.float64)
    r_dr, r_dm, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho, w.fields["mom"])
    scaled_check(host(dr), r_dr, s_dr, RTOL, "drho/dt")
    scaled_check(host(dm), r_dm, s_dm, RTOL, "dmom/dt")


@pytest.mark.parametrize("lanes", ["auto", "2"])
@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_euler_batched_rows_ragged(S, kappa, lanes, monkeypatch):
    """Batched short rows on a 64^2 lattice with 157 particles removed: 3,939
    slots (a ragged last workgroup) and rows of 8-12 (1.6h) or 14-20 (2h)
    entries, padded; lanes per particle as chosen for this size (four) or
    two (the large-launch choice for rows of up to 12).  Rates and one Heun
    step (the stage kernels write the state) against the oracle."""
    if lanes != "auto":
        monkeypatch.setenv("SPH_EULER_BATCH_LANES", lanes)
    w = I.taylor_green_2d(nside=64, nu=0.01)
    keep = np.sort(np.random.default_rng(9).choice(w.n, w.n - 157, replace=False))
    w.pos = np.ascontiguousarray(w.pos[:, keep])
    w.vol = np.ascontiguousarray(w.vol[keep])
    w.fields["drho"] = np.ascontiguousarray(w.fields["drho"][keep])
    w.fields["mom"] = np.ascontiguousarray(w.fields["mom"][:, keep])
    assert w.n == 3939
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    dt = w.meta["dt"]
    pg, po = _euler_prm(S, w, dt)
    box, rp, col, Bo, _ = _c0_oracle(w, kappa)
    assert np.diff(rp).max() <= (12 if kappa == 1.6 else 20)  # short rows: the batched kernel
    drho0 = w.fields["drho"].astype(np.float64)
    mom0 = w.fields["mom"].astype(np.float64)
    rho0 = w.fields["rho_ref"] + drho0
    dr, dm = ctx.euler_rhs(pg, dev(w.fields["drho"]), dev(w.fields["mom"]))
    r_dr, r_dm, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho0, mom0)
    scaled_check(host(dr), r_dr, s_dr, RTOL, "drho/dt")
    scaled_check(host(dm), r_dm, s_dm, RTOL, "dmom/dt")
    d = dev(w.fields["drho"])
    m = dev(w.fields["mom"])
    ctx.euler_step(pg, d, m, 1)
    r1, m1 = O.euler_heun(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho0, mom0, 1)
    eps = np.finfo(np.float32).eps
    inc_g, inc_o = host(d) - drho0, (r1 - w.fields["rho_ref"]) - drho0
    assert np.all(np.abs(inc_g - inc_o) <= 1e-5 * (np.abs(inc_o) + 1.5 * dt * s_dr)
                  + 4 * eps * np.abs(r1 - w.fields["rho_ref"]))
    inc_g, inc_o = host(m) - mom0, m1 - mom0
    assert np.all(np.abs(inc_g - inc_o) <= 1e-5 * (np.abs(inc_o) + 1.5 * dt * s_dm) + 4 * eps * np.abs(m1))


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_double_shear_layer(S, kappa):
    """Double shear layer (inviscid, Sec. 4.2) at the paper's 128^2: rates
    against the oracle element by element; 50 Heun steps to the per-step
    bar; the full run to t = 1.2 (2,166 steps) through integral quantities.
    Without viscosity the limiter damps only approaching pairs, and the run
    amplifies rounding-level differences: two FP64 oracle runs whose initial
    momenta differ by 1e-7 (relative) end ~10% apart in the momentum field
    but within ~1e-3 in kinetic energy.  So at t = 1.2: total mass and
    momentum conserved (the pair fluxes are antisymmetric) and the kinetic
    energy within 5e-3 of the oracle's."""
    w = I.double_shear_layer(nside=128)
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    dt = w.meta["dt"]
    pg, po = _euler_prm(S, w, dt)
    box, rp, col, Bo, _ = _c0_oracle(w, kappa)
    V = w.vol.astype(np.float64)
    drho0 = w.fields["drho"].astype(np.float64)
    mom0 = w.fields["mom"].astype(np.float64)
    rho0 = w.fields["rho_ref"] + drho0
    dr, dm = ctx.euler_rhs(pg, dev(w.fields["drho"]), dev(w.fields["mom"]))
    r_dr, r_dm, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho0, mom0)
    scaled_check(host(dr), r_dr, s_dr, RTOL, "drho/dt")
    scaled_check(host(dm), r_dm, s_dm, RTOL, "dmom/dt")
    d = dev(w.fields["drho"])
    m = dev(w.fields["mom"])
    ctx.euler_step(pg, d, m, 50)
    r50, m50 = O.euler_heun(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho0, mom0, 50)
    assert normwise(host(m), m50) < 1e-5
    assert normwise(host(d), r50 - w.fields["rho_ref"]) < 1e-3  # drho itself is ~1e-3: 1e-6 of rho
    steps = int(round(1.2 / dt))
    ctx.euler_step(pg, d, m, steps - 50)
    r1, m1 = O.euler_heun(box, w.pos, w.h, rp, col, w.vol, Bo, po, r50, m50, steps - 50)
    rg = w.fields["rho_ref"] + host(d).astype(np.float64)
    mg = host(m).astype(np.float64)
    scale_m = np.sum(np.abs(mom0).sum(0) * V)
    mass_drift = abs(np.sum(rg * V) - np.sum(rho0 * V)) / np.sum(rho0 * V)
    mom_drift = np.abs(mg @ V - mom0 @ V).max() / scale_m
    ke = lambda r, mm: 0.5 * np.sum((mm ** 2).sum(0) / r * V)
    ke_diff = abs(ke(rg, mg) - ke(r1, m1)) / ke(r1, m1)
    print(f"kappa {kappa}: mass drift {mass_drift:.3g}, momentum drift {mom_drift:.3g}, "
          f"KE/KE0 {ke(rg, mg) / ke(rho0, mom0):.4f} (oracle {ke(r1, m1) / ke(rho0, mom0):.4f}), KE diff {ke_diff:.3g}")
    assert mass_drift < 1e-6 and mom_drift < 1e-6
    assert ke_diff < 5e-3


def _mixed_box_3d(nside=24, seed=5):
    """Jittered 3-D lattice, periodic in x and z, open in y (free surfaces)."""
    w = I.taylor_green_3d(nside=nside)
    rng = np.random.default_rng(seed)
    dx = w.meta["dx"]
    q = w.meta["quantum"]
    pos = w.pos.astype(np.float64) + rng.uniform(-0.2 * dx, 0.2 * dx, size=w.pos.shape)
    w.pos = I.wrap_periodic(pos, 0.0, 1.0, q).astype(np.float32)
    w.periodic = (1, 0, 1)
    return w


@pytest.mark.parametrize("geo", ["records", "split"])
@pytest.mark.parametrize("rows", ["ell", "csr"])
@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_euler_rhs_3d_geometry_records(S, rows, kappa, geo, monkeypatch):
    """3-D rates on a jittered box with an open axis: through the packed
    per-particle records (geometry and state in one 64-byte record, packed
    from the cached correction at each call) and through the separate
    geometry arrays of the generic kernel (SPH_EULER_GEO=split), against the
    oracle, again after the correction is recomputed for new volumes."""
    if rows == "csr":
        monkeypatch.setenv("SPH_PAIR_ROWS", "csr")
    if geo == "split":
        monkeypatch.setenv("SPH_EULER_GEO", "split")
    w = _mixed_box_3d()
    ctx = gpu_ctx(S, w, kappa)
    pg, po = _euler_prm(S, w)
    box = oracle_box(w)
    rc = kappa * w.h
    rp, col = O.neighbors_grid(box, w.pos, rc, rc * rc)
    rho = w.fields["rho_ref"] + w.fields["drho"].astype(np.float64)
    rng = np.random.default_rng(11)
    vols = [w.vol, (w.vol * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, w.n))).astype(np.float32)]
    for vol in vols:
        ctx.correction_B(dev(vol))
        dr, dm = ctx.euler_rhs(pg, dev(w.fields["drho"]), dev(w.fields["mom"]))
        Bo, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp, col, vol)
        r_dr, r_dm, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp, col, vol, Bo, po, rho, w.fields["mom"])
        scaled_check(host(dr), r_dr, s_dr, RTOL, "drho/dt")
        scaled_check(host(dm), r_dm, s_dm, RTOL, "dmom/dt")


@pytest.mark.parametrize("lanes", ["1", "2", "4", "8"])
@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_euler_3d_lanes_and_chunks(S, kappa, lanes, monkeypatch):
    """The 3-D stage on every lanes-per-particle mapping (1, 2, 4, 8 lanes;
    the chunk of pairs per lane follows the row length) against the oracle:
    rates on the jittered open box and one Heun step of a jittered periodic
    Taylor-Green cube."""
    monkeypatch.setenv("SPH_EULER_LANES", lanes)
    w = _mixed_box_3d()
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    pg, po = _euler_prm(S, w)
    box, rp, col, Bo, _ = _c0_oracle(w, kappa)
    rho = w.fields["rho_ref"] + w.fields["drho"].astype(np.float64)
    dr, dm = ctx.euler_rhs(pg, dev(w.fields["drho"]), dev(w.fields["mom"]))
    r_dr, r_dm, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho, w.fields["mom"])
    scaled_check(host(dr), r_dr, s_dr, RTOL, "drho/dt")
    scaled_check(host(dm), r_dm, s_dm, RTOL, "dmom/dt")
    ctx.close()
    w = I.taylor_green_3d(nside=24, jitter=0.1, seed=4)
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    dt = w.meta["dt"]
    pg, po = _euler_prm(S, w, dt)
    box, rp, col, Bo, _ = _c0_oracle(w, kappa)
    drho0 = w.fields["drho"].astype(np.float64)
    mom0 = w.fields["mom"].astype(np.float64)
    d, m = dev(w.fields["drho"]), dev(w.fields["mom"])
    ctx.euler_step(pg, d, m, 1)
    r1, m1 = O.euler_heun(box, w.pos, w.h, rp, col, w.vol, Bo, po, 1.0 + drho0, mom0, 1)
    _, _, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, 1.0 + drho0, mom0)
    eps = np.finfo(np.float32).eps
    inc_g, inc_o = host(d) - drho0, (r1 - 1.0) - drho0
    assert np.all(np.abs(inc_g - inc_o) <= 1e-5 * (np.abs(inc_o) + 1.5 * dt * s_dr) + 4 * eps * np.abs(r1 - 1.0))
    inc_g, inc_o = host(m) - mom0, m1 - mom0
    assert np.all(np.abs(inc_g - inc_o) <= 1e-5 * (np.abs(inc_o) + 1.5 * dt * s_dm) + 4 * eps * np.abs(m1))


@pytest.mark.parametrize("case", ["mixed3d", "tiny2d"])
@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_euler_rhs_box_geometries(S, case, kappa):
    """Box edge cases against the oracle: a 3-D box with an open axis
    (neighbourhoods clipped at the free surfaces; windows of uneven length)
    and a small periodic 2-D box (16^2 particles, six cells per axis at
    2h)."""
    w = _mixed_box_3d() if case == "mixed3d" else I.taylor_green_2d(nside=16)
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    pg, po = _euler_prm(S, w)
    dr, dm = ctx.euler_rhs(pg, dev(w.fields["drho"]), dev(w.fields["mom"]))
    box, rp, col, Bo, _ = _c0_oracle(w, kappa)
    rho = w.fields["rho_ref"] + w.fields["drho"].astype(np.float64)
    r_dr, r_dm, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, rho, w.fields["mom"])
    scaled_check(host(dr), r_dr, s_dr, RTOL, "drho/dt")
    scaled_check(host(dm), r_dm, s_dm, RTOL, "dmom/dt")


def test_euler_rhs_full_size_taylor_green_sampled(S):
    """512^2 Taylor-Green (the timed workload): neighbour rows, B and the RHS
    on a sample of particles, against the oracle computed on those rows."""
    w = I.taylor_green_2d(nside=512)
    box = oracle_box(w)
    rows = sample_rows(w.n, 48, seed=7)
    for kappa in (2.0, 1.6):
        rc = kappa * w.h
        ctx = gpu_ctx(S, w, kappa)
        rp, col = ctx.neighbors()
        rp_g, col_g = host(rp), host(col)
        rp_o, col_o = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=rows)
        assert csr_rows_equal(rp_g, col_g, rp_o, col_o, rows) is None
        B, _, nd = ctx.correction_B(dev(w.vol))
        assert nd == 0
        ring = np.unique(np.concatenate([rows, col_o.astype(np.int64)]))
        rp_r, col_r = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=ring)
        B_r, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp_r, col_r, w.vol, rows=ring)
        Bg = host(B)
        scale = np.abs(B_r).reshape(len(ring), -1).max(axis=1)[:, None, None]
        scaled_check(Bg[ring], B_r, scale, RTOL, "B sampled")
        B_full = np.zeros((w.n, 2, 2))
        B_full[ring] = B_r
        pg, po = _euler_prm(S, w)
        dr, dm = ctx.euler_rhs(pg, dev(w.fields["drho"]), dev(w.fields["mom"]))
        rho = 1.0 + w.fields["drho"].astype(np.float64)
        r_dr, r_dm, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp_o, col_o, w.vol, B_full, po, rho,
                                             w.fields["mom"], rows=rows)
        scaled_check(host(dr)[rows], r_dr, s_dr, RTOL, "drho/dt sampled")
        scaled_check(host(dm)[:, rows], r_dm, s_dm, RTOL, "dmom/dt sampled")


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_euler_heun_step_full_size_sampled(S, kappa):
    """One Heun step of the 512^2 Taylor-Green workload through the stage
    kernels the bench times, on 24 sampled particles: the oracle evaluates
    the first stage on the samples and their neighbours, then the second
    stage on the samples (U* = U + dt R(U), U' = (U + U* + dt R(U*)) / 2),
    with B on the two rings of neighbours around them."""
    w = I.taylor_green_2d(nside=512)
    box = oracle_box(w)
    rc = kappa * w.h
    dt = w.meta["dt"]
    rows = sample_rows(w.n, 24, seed=9)
    rp_s, col_s = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=rows)
    ring1 = np.unique(np.concatenate([rows, col_s.astype(np.int64)]))
    rp_1, col_1 = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=ring1)
    ring2 = np.unique(np.concatenate([ring1, col_1.astype(np.int64)]))
    rp_2, col_2 = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=ring2)
    B_2, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp_2, col_2, w.vol, rows=ring2)
    B_full = np.zeros((w.n, 2, 2))
    B_full[ring2] = B_2
    pg, po = _euler_prm(S, w, dt)
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
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    d, m = dev(w.fields["drho"]), dev(w.fields["mom"])
    ctx.euler_step(pg, d, m, 1)
    eps = np.finfo(np.float32).eps
    inc_g, inc_o = host(d)[rows] - drho0[rows], (rho_n - 1.0) - drho0[rows]
    assert np.all(np.abs(inc_g - inc_o) <= 1e-5 * (np.abs(inc_o) + 1.5 * dt * s_dr) + 4 * eps * np.abs(rho_n - 1.0))
    inc_g, inc_o = host(m)[:, rows] - mom0[:, rows], mom_n - mom0[:, rows]
    assert np.all(np.abs(inc_g - inc_o) <= 1e-5 * (np.abs(inc_o) + 1.5 * dt * s_dm) + 4 * eps * np.abs(mom_n))


@pytest.mark.parametrize("nside", [80, 104, 200])
def test_euler_rhs_3d_taylor_green_sampled(S, nside):
    """3-D Taylor-Green at 80^3 and 104^3 (the two sizes take different
    lanes-per-particle mappings: 2 and 1) and at the 200^3 of the bench's
    3-D line (8M particles, its launch configuration)."""
    w = I.taylor_green_3d(nside=nside)
    box = oracle_box(w)
    rows = sample_rows(w.n, 24, seed=3)
    for kappa in (2.0, 1.6):
        rc = kappa * w.h
        ctx = gpu_ctx(S, w, kappa)
        rp, col = ctx.neighbors()
        rp_o, col_o = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=rows)
        assert csr_rows_equal(host(rp), host(col), rp_o, col_o, rows) is None
        ctx.correction_B(dev(w.vol))
        ring = np.unique(np.concatenate([rows, col_o.astype(np.int64)]))
        rp_r, col_r = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=ring)
        B_r, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp_r, col_r, w.vol, rows=ring)
        B_full = np.zeros((w.n, 3, 3))
        B_full[ring] = B_r
        pg, po = _euler_prm(S, w)
        dr, dm = ctx.euler_rhs(pg, dev(w.fields["drho"]), dev(w.fields["mom"]))
        rho = 1.0 + w.fields["drho"].astype(np.float64)
        r_dr, r_dm, s_dr, s_dm = O.euler_rhs(box, w.pos, w.h, rp_o, col_o, w.vol, B_full, po, rho,
                                             w.fields["mom"], rows=rows)
        scaled_check(host(dr)[rows], r_dr, s_dr, RTOL, "3d drho/dt")
        scaled_check(host(dm)[:, rows], r_dm, s_dm, RTOL, "3d dmom/dt")


# ------------------------------------------------------------------ total Lagrangian

def _plate(nx=24):
    return I.cantilever_plate(nx=nx, length=0.2, thick=0.02 * 3, width=0.04)


def _tl_setup(S, w, kappa, model):
    ctx = gpu_ctx(S, w, kappa)
    _, _, nd = ctx.correction_B(dev(w.vol))
    box = oracle_box(w)
    rc = kappa * w.h
    rp, col = O.neighbors_grid(box, w.pos, rc, rc * rc)
    Bo, ndo = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol)
    assert nd == ndo
    f = w.fields
    pg = S.tlsph_params(f["rho0"], f["E"], f["nu"], dt=w.meta["dt"], model=model)
    po = O.tlsph_params(f["rho0"], f["E"], f["nu"], dt=w.meta["dt"], model=model)
    return ctx, box, rp, col, Bo, pg, po


@pytest.mark.parametrize("kappa", [2.0, 1.6])
@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("rows", ["ell", "csr", "ell1", "ell4"])
def test_tlsph_rhs(S, kappa, model, rows, monkeypatch):
    """rows: fixed-stride or CSR rows; ell1 / ell4 force 1 or 4 lanes per particle."""
    if rows == "csr":
        monkeypatch.setenv("SPH_PAIR_ROWS", "csr")
    if rows in ("ell1", "ell4"):
        monkeypatch.setenv("SPH_TLSPH_LANES", rows[-1])
    w = _plate()
    ctx, box, rp, col, Bo, pg, po = _tl_setup(S, w, kappa, model)
    rng = np.random.default_rng(2)
    F = (np.eye(3)[None] + 0.01 * rng.normal(size=(w.n, 3, 3))).astype(np.float32)
    vel = w.fields["vel"]
    fixed = w.fields["fixed"]
    dF, acc = ctx.tlsph_rhs(pg, dev(vel), dev(F), dev(fixed, torch.int32))
    r_dF, r_acc, s_acc = O.tlsph_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, vel, F, fixed)
    scaled_check(host(acc), r_acc, s_acc, RTOL, "acc")
    scaled_check(host(dF), r_dF, _df_scale(w, rp, col, Bo, vel)[:, None, None], RTOL, "dF/dt")


def _df_scale(w, rp, col, Bo, vel):
    """dF/dt scale per row: ||B_i|| sum_j V_j |v_j - v_i| |dW/dr|."""
    pos = w.pos.astype(np.float64)
    rows = np.repeat(np.arange(w.n), np.diff(rp))
    d = pos[:, rows] - pos[:, col]
    r = np.sqrt((d ** 2).sum(0))
    t = np.abs(vel[:, col] - vel[:, rows]).max(0) * np.abs(O.kernel_dWdr(O.WENDLAND, 3, w.h, r)) * w.vol[col]
    return np.bincount(rows, weights=t, minlength=w.n) * np.abs(Bo).reshape(w.n, -1).max(1) * 3


@pytest.mark.parametrize("kappa", [2.0, 1.6])
@pytest.mark.parametrize("model", [0, 1])
def test_tlsph_windows_match_gathers(S, kappa, model, monkeypatch):
    """Both total-Lagrangian loops with the neighbour records read from LDS
    windows against the kernels that gather them: the same pairs in the
    same order, plus zero-separation padding pairs (which can move a
    compensated sum by an ulp), so deformation rates and accelerations agree
    to a few FP32 ulps of their absolute-sum scales.  The path taken is the
    one asked for."""
    w = _plate()
    rng = np.random.default_rng(4)
    F = (np.eye(3)[None] + 0.01 * rng.normal(size=(w.n, 3, 3))).astype(np.float32)
    out = {}
    for win in ("0", "1"):
        monkeypatch.setenv("SPH_TLSPH_WINDOW", win)
        ctx, box, rp, col, Bo, pg, po = _tl_setup(S, w, kappa, model)
        dF, acc = ctx.tlsph_rhs(pg, dev(w.fields["vel"]), dev(F), dev(w.fields["fixed"], torch.int32))
        out[win] = (host(dF).copy(), host(acc).copy(), ctx.tlsph_path())
        ctx.close()
    assert out["0"][2] == S.PATH_GENERIC and out["1"][2] == S.PATH_WINDOWS
    _, r_acc, s_acc = O.tlsph_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, w.fields["vel"], F, w.fields["fixed"])
    eps = float(np.finfo(np.float32).eps)
    s_df = _df_scale(w, rp, col, Bo, w.fields["vel"])[:, None, None]
    assert np.all(np.abs(out["1"][0] - out["0"][0]) <= 8 * eps * s_df)
    assert np.all(np.abs(out["1"][1] - out["0"][1]) <= 8 * eps * s_acc)


@pytest.mark.parametrize("kappa", [2.0, 1.6])
@pytest.mark.parametrize("rows", ["ell", "csr"])
def test_tlsph_steps(S, kappa, rows, monkeypatch):
    if rows == "csr":
        monkeypatch.setenv("SPH_PAIR_ROWS", "csr")
    w = _plate()
    ctx, box, rp, col, Bo, pg, po = _tl_setup(S, w, kappa, 0)
    F0 = np.tile(np.eye(3, dtype=np.float32), (w.n, 1, 1))
    vel0 = w.fields["vel"]
    fixed = w.fields["fixed"]
    _, acc0, _ = O.tlsph_rhs(box, w.pos, w.h, rp, col, w.vol, Bo, po, vel0, F0, fixed)
    nsteps = 100
    pos_o, vel_o, F_o, acc_o = O.tlsph_step(box, w.pos, w.h, rp, col, w.vol, Bo, po, fixed, w.pos, vel0, F0,
                                            acc0, nsteps)
    pos = dev(w.pos)
    vel = dev(vel0)
    F = dev(F0)
    _, acc = ctx.tlsph_rhs(pg, vel, F, dev(fixed, torch.int32))
    ctx.tlsph_step(pg, dev(fixed, torch.int32), pos, vel, F, acc, nsteps)
    assert normwise(host(vel), vel_o) < 1e-3
    assert normwise(host(F) - np.eye(3), F_o - np.eye(3)) < 1e-3
    assert normwise(host(pos) - w.pos, pos_o - w.pos) < 1e-3
    assert np.all(host(vel)[:, fixed.astype(bool)] == 0.0)


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_tlsph_full_size_plate_sampled(S, kappa):
    """The 1,604,932-particle plate of the bench (dx = 0.2/430, neo-Hookean)
    in the launch configuration the bench times: deformation rate and
    acceleration of 32 sampled particles against the oracle, with every
    particle's F perturbed (the sampled rows' neighbours' stresses enter)."""
    w = I.cantilever_plate(nx=430)
    assert w.n == 1604932
    box = oracle_box(w)
    rc = kappa * w.h
    rows = sample_rows(w.n, 32, seed=11)
    ctx = gpu_ctx(S, w, kappa)
    ctx.correction_B(dev(w.vol))
    rp_o, col_o = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=rows)
    ring = np.unique(np.concatenate([rows, col_o.astype(np.int64)]))
    rp_r, col_r = O.neighbors_grid(box, w.pos, rc, rc * rc, rows=ring)
    B_r, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp_r, col_r, w.vol, rows=ring)
    B_full = np.zeros((w.n, 3, 3))
    B_full[ring] = B_r
    f = w.fields
    pg = S.tlsph_params(f["rho0"], f["E"], f["nu"], dt=w.meta["dt"], model=0)
    po = O.tlsph_params(f["rho0"], f["E"], f["nu"], dt=w.meta["dt"], model=0)
    rng = np.random.default_rng(5)
    F = (np.eye(3, dtype=np.float32)[None] + 0.01 * rng.standard_normal((w.n, 3, 3)).astype(np.float32))
    vel, fixed = f["vel"], f["fixed"]
    dF, acc = ctx.tlsph_rhs(pg, dev(vel), dev(F), dev(fixed, torch.int32))
    r_dF, r_acc, s_acc = O.tlsph_rhs(box, w.pos, w.h, rp_o, col_o, w.vol, B_full, po, vel, F, fixed, rows=rows)
    scaled_check(host(acc)[:, rows], r_acc, s_acc, RTOL, "acc sampled")
    pos = w.pos.astype(np.float64)
    owner = np.repeat(rows, np.diff(rp_o))
    d = pos[:, owner] - pos[:, col_o]
    r = np.sqrt((d ** 2).sum(0))
    t = np.abs(vel[:, col_o] - vel[:, owner]).max(0) * np.abs(O.kernel_dWdr(O.WENDLAND, 3, w.h, r)) * w.vol[col_o]
    sc = np.bincount(np.repeat(np.arange(len(rows)), np.diff(rp_o)), weights=t, minlength=len(rows))
    sc = sc * np.abs(B_full[rows]).reshape(len(rows), -1).max(1) * 3
    scaled_check(host(dF)[rows], r_dF, sc[:, None, None], RTOL, "dF/dt sampled")


def test_truncated_kernel_equal_accuracy_taylor_green():
    """At equal time step and step count, the 1.6h run's velocity error
    against the decaying Taylor-Green solution is within 10% of the 2h
    run's (128^2 lattice, 200 Heun steps, nu = 0.01)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_05155_amd import sph as S
    w = I.taylor_green_2d(nside=128)
    f = w.fields
    x = w.pos.astype(np.float64)
    steps = 200
    t = steps * w.meta["dt"]
    ue = np.exp(-8.0 * np.pi ** 2 * f["nu"] * t) * np.stack(
        [np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1]), -np.cos(2 * np.pi * x[0]) * np.sin(2 * np.pi * x[1])])
    err = {}
    for kappa in (2.0, 1.6):
        ctx = S.Context(2)
        ctx.build_cells(S.Domain(dim=2, h=w.h, kappa=kappa), dev(w.pos))
        ctx.correction_B(dev(w.vol))
        prm = S.euler_params(c=f["c"], rho0=f["rho0_eos"], rho_ref=f["rho_ref"], eta=f["eta"], mu=f["mu"],
                             dt=w.meta["dt"])
        d, m = dev(f["drho"]), dev(f["mom"])
        ctx.euler_step(prm, d, m, steps)
        u = host(m).astype(np.float64) / (1.0 + host(d).astype(np.float64))
        err[kappa] = np.linalg.norm(u - ue) / np.linalg.norm(ue)
    assert err[1.6] <= 1.10 * err[2.0], err
