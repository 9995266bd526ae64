"""Edge cases through the C ABI: an empty configuration at every call, and
particles without neighbours or with a single neighbour (the correction
matrix of Eq. (9) degenerates and is replaced by the identity, counted; the
fluxes reduce to one pair), against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2405_05155_amd import inputs as I
from tests.gpu_helpers import oracle_box, scaled_check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("dim", [2, 3])
def test_empty_configuration_every_call(S, dim):
    ctx = S.Context(dim)
    ctx.build_cells(S.Domain(dim=dim, h=0.05, kappa=2.0), torch.empty((dim, 0), device="cuda"))
    vol = torch.empty(0, device="cuda")
    vec = torch.empty((dim, 0), device="cuda")
    assert ctx.kernel_sum(vol).numel() == 0
    B, _, nd = ctx.correction_B(vol)
    assert B.numel() == 0 and nd == 0
    assert ctx.gradient(vol).numel() == 0
    prm = S.euler_params(c=10.0, rho0=1.0, rho_ref=1.0, eta=15.0, mu=0.01, dt=1e-4)
    dr, dm = ctx.euler_rhs(prm, vol, vec)
    assert dr.numel() == 0 and dm.numel() == 0
    ctx.euler_step(prm, vol, vec, 3)
    if dim == 2:
        hp = S.hllc_params(1.4, 1.0, 1e-4)
        dr, dm, de = ctx.hllc_rhs(hp, vol, vec, vol)
        assert dr.numel() == 0 and dm.numel() == 0 and de.numel() == 0
        ctx.hllc_step(hp, vol, vec, vol, 3)
    if dim == 3:
        tp = S.tlsph_params(1000.0, 2e6, 0.3975, dt=1e-6, model=0)
        F = torch.empty((0, 3, 3), device="cuda")
        fixed = torch.empty(0, dtype=torch.int32, device="cuda")
        dF, acc = ctx.tlsph_rhs(tp, vec, F, fixed)
        assert dF.numel() == 0 and acc.numel() == 0
        ctx.tlsph_step(tp, fixed, vec.clone(), vec.clone(), F, acc, 2)
        lg = S.Domain(dim=3, h=0.01, kappa=2.0, periodic=(0, 0, 0), kernel=S.LAGUERRE_GAUSS)
        rp = S.relax_params((0.5, 0.5, 0.5), 0.3)
        res, g = ctx.relax_residue(lg, rp, vec, vol)
        assert host(res)[0] == 0.0 and g.numel() == 0
        ctx.relax_step(lg, rp, vec.clone(), vec.clone(), vol, 2)
        feat = ctx.mlp_features(lg, rp, vec)
        assert feat.shape[0] == 0
        params = dev(np.zeros(S.MLP_NPARAMS, dtype=np.float32))
        assert ctx.mlp_forward(params, feat).shape == (0, 3)
        ctx.mlp_apply(lg, rp, vec.clone(), params)
    torch.cuda.synchronize()


def _sparse_case_2d():
    """Three isolated particles, one lone pair, and a 6x6 lattice patch, in
    the open unit square (quantised coordinates)."""
    q = I.quantum_for(1.0)
    dx = 1.0 / 64
    h = 1.3 * dx
    pts = [(0.1, 0.1), (0.9, 0.1), (0.5, 0.9),            # isolated
           (0.3, 0.5), (0.3 + 1.5 * dx, 0.5)]               # a lone pair
    for a in range(6):
        for b in range(6):
            pts.append((0.6 + a * dx, 0.4 + b * dx))
    pos = I.quantise(np.array(pts).T, q).astype(np.float32)
    vol = np.full(pos.shape[1], dx * dx, dtype=np.float32)
    rng = np.random.default_rng(4)
    drho = (0.01 * rng.standard_normal(pos.shape[1])).astype(np.float32)
    mom = (0.1 * rng.standard_normal((2, pos.shape[1]))).astype(np.float32)
    return pos, vol, h, drho, mom


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_isolated_particles_and_lone_pair(S, kappa):
    pos, vol, h, drho, mom = _sparse_case_2d()
    n = pos.shape[1]
    ctx = S.Context(2)
    dom = S.Domain(dim=2, h=h, kappa=kappa, periodic=(0, 0))
    ctx.build_cells(dom, dev(pos))
    rp, col = ctx.neighbors()
    box = O.make_box(2, periodic=(0, 0))
    rc = kappa * h
    rp_o, col_o = O.neighbors_brute(box, pos, rc * rc)
    assert np.array_equal(host(rp), rp_o) and np.array_equal(host(col), col_o)
    assert rp_o[1] == 0 and rp_o[3] == 0        # isolated rows are empty
    assert rp_o[4] - rp_o[3] == 1               # the pair sees only its partner
    ks = host(ctx.kernel_sum(dev(vol)))
    ks_o = O.kernel_sum(box, pos, O.WENDLAND, h, rp_o, col_o, vol)
    scaled_check(ks, ks_o, ks_o, 1e-5, "kernel sum")
    B, _, nd = ctx.correction_B(dev(vol))
    B_o, nd_o = O.correction_B(box, pos, O.WENDLAND, h, rp_o, col_o, vol)
    assert nd == nd_o and nd >= 5                # isolated and paired rows degenerate
    Bg = host(B)
    for i in range(3):
        assert np.array_equal(Bg[i], np.eye(2, dtype=np.float32))
    scale = np.abs(B_o).reshape(n, -1).max(axis=1)[:, None, None]
    scaled_check(Bg, B_o, scale, 1e-5, "B")
    prm = S.euler_params(c=10.0, rho0=0.0, rho_ref=1.0, eta=15.0, mu=0.01)
    po = O.euler_params(c=10.0, rho0=0.0, eta=15.0, mu=0.01, dt=0.0)
    dr, dm = ctx.euler_rhs(prm, dev(drho), dev(mom))
    rho = 1.0 + drho.astype(np.float64)
    r_dr, r_dm, s_dr, s_dm = O.euler_rhs(box, pos, h, rp_o, col_o, vol, B_o, po, rho, mom)
    scaled_check(host(dr), r_dr, s_dr, 1e-5, "drho/dt")
    scaled_check(host(dm), r_dm, s_dm, 1e-5, "dmom/dt")
    assert np.all(host(dr)[:3] == 0.0) and np.all(host(dm)[:, :3] == 0.0)
    # the compressible rows on the same particles
    rng = np.random.default_rng(8)
    rho_c = rng.uniform(0.5, 2.0, n)
    v = rng.normal(size=(2, n))
    p_c = rng.uniform(0.5, 2.0, n)
    E = p_c / 0.4 + 0.5 * rho_c * (v ** 2).sum(0)
    rho_c, mom_c, E = rho_c.astype(np.float32), (rho_c * v).astype(np.float32), E.astype(np.float32)
    dr, dm, de = ctx.hllc_rhs(S.hllc_params(1.4, 1.0), dev(rho_c), dev(mom_c), dev(E))
    r_dr, r_dm, r_de, s_dr, s_dm, s_de = O.hllc_rhs(box, pos, h, rp_o, col_o, vol, B_o, O.hllc_params(1.4, 1.0),
                                                    rho_c, mom_c, E)
    scaled_check(host(dr), r_dr, s_dr, 1e-5, "hllc drho/dt")
    scaled_check(host(dm), r_dm, s_dm, 1e-5, "hllc dmom/dt")
    scaled_check(host(de), r_de, s_de, 1e-5, "hllc dE/dt")
    assert np.all(host(dr)[:3] == 0.0) and np.all(host(de)[:3] == 0.0)
