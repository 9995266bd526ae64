"""Compressible rows (limited HLLC, energy equation, ideal gas; 2-D) through
the C ABI against the FP64 oracle: rates per element on jittered particles
with random states (shocks, supersonic pairs, crossed wave-speed estimates),
in every row layout; Heun steps on an advected density wave; argument
checks."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2405_05155_amd import inputs as I
from gpu_helpers import normwise, oracle_box, scaled_check

pytestmark = pytest.mark.gpu
RTOL = 1e-5
GAMMA = 1.4


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


def _ctx(S, w, kappa):
    ctx = S.Context(2)
    ctx.build_cells(S.Domain(dim=2, h=w.h, kappa=kappa, lo=w.lo, hi=w.hi, periodic=w.periodic), dev(w.pos))
    ctx.correction_B(dev(w.vol))
    return ctx


def _oracle_geometry(w, kappa):
    box = oracle_box(w)
    rc = kappa * w.h
    rp, col = O.neighbors_grid(box, w.pos, rc, rc * rc)
    B, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol)
    return box, rp, col, B


def _random_states(n, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, n)
    v = rng.normal(size=(2, n)) * 1.5
    p = rng.uniform(0.3, 3.0, n)
    E = p / (GAMMA - 1.0) + 0.5 * rho * (v ** 2).sum(0)
    return rho.astype(np.float32), (rho * v).astype(np.float32), E.astype(np.float32)


@pytest.mark.parametrize("rows", ["auto", "batch2", "batch4", "batch8", "ell", "csr"])
@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_hllc_rhs_matches_oracle(S, kappa, rows, monkeypatch):
    env = {"auto": {}, "batch2": {"SPH_EULER_BATCH_LANES": "2"}, "batch4": {"SPH_EULER_BATCH_LANES": "4"},
           "batch8": {"SPH_EULER_BATCH_LANES": "8"}, "ell": {"SPH_EULER_BATCH_LANES": "0"},
           "csr": {"SPH_EULER_BATCH_LANES": "0", "SPH_PAIR_ROWS": "csr"}}[rows]
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    w = I.periodic_square_case(64, 2, 1.3, 0.05, 3, "jittered")
    rho, mom, E = _random_states(w.n, 7)
    ctx = _ctx(S, w, kappa)
    prm = S.hllc_params(GAMMA, 1.0)
    dr, dm, de = ctx.hllc_rhs(prm, dev(rho), dev(mom), dev(E))
    box, rp, col, B = _oracle_geometry(w, kappa)
    r_dr, r_dm, r_de, s_dr, s_dm, s_de = O.hllc_rhs(box, w.pos, w.h, rp, col, w.vol, B, O.hllc_params(GAMMA, 1.0),
                                                    rho, mom, E)
    scaled_check(host(dr), r_dr, s_dr, RTOL, "drho/dt")
    scaled_check(host(dm), r_dm, s_dm, RTOL, "dmom/dt")
    scaled_check(host(de), r_de, s_de, RTOL, "dE/dt")


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_hllc_steps_density_wave(S, kappa):
    """50 Heun steps of the advected density wave (64^2): each step's
    increment to the per-step bar, then the state normwise."""
    w = I.density_wave_2d(nside=64)
    f = w.fields
    dt = w.meta["dt"]
    ctx = _ctx(S, w, kappa)
    prm = S.hllc_params(GAMMA, 1.0, dt)
    box, rp, col, B = _oracle_geometry(w, kappa)
    po = O.hllc_params(GAMMA, 1.0, dt)
    rho0, mom0, E0 = (f[k].astype(np.float64) for k in ("rho", "mom", "E"))
    r, m, e = dev(f["rho"]), dev(f["mom"]), dev(f["E"])
    ctx.hllc_step(prm, r, m, e, 1)
    r1, m1, e1 = O.hllc_heun(box, w.pos, w.h, rp, col, w.vol, B, po, rho0, mom0, E0, 1)
    _, _, _, s_dr, s_dm, s_de = O.hllc_rhs(box, w.pos, w.h, rp, col, w.vol, B, po, rho0, mom0, E0)
    eps = np.finfo(np.float32).eps
    for g, o0, o1, s in ((host(r), rho0, r1, s_dr), (host(m), mom0, m1, s_dm), (host(e), E0, e1, s_de)):
        inc_g, inc_o = g - o0, o1 - o0
        assert np.all(np.abs(inc_g - inc_o) <= 1e-5 * (np.abs(inc_o) + 1.5 * dt * s) + 4 * eps * np.abs(o1))
    ctx.hllc_step(prm, r, m, e, 49)
    r50, m50, e50 = O.hllc_heun(box, w.pos, w.h, rp, col, w.vol, B, po, r1, m1, e1, 49)
    assert normwise(host(r), r50) < 1e-5
    assert normwise(host(m), m50) < 1e-5
    assert normwise(host(e), e50) < 1e-5


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_hllc_sod_shock_tube(S, kappa):
    """Sod's shock tube (strip 256 x 16): rates of the discontinuous initial
    state per element, then the run to t = 0.1 (78 Heun steps) against the
    oracle's run, normwise."""
    w = I.sod_strip_2d(256)
    f = w.fields
    dt = w.meta["dt"]
    ctx = _ctx(S, w, kappa)
    prm = S.hllc_params(GAMMA, 1.0, dt)
    box, rp, col, B = _oracle_geometry(w, kappa)
    po = O.hllc_params(GAMMA, 1.0, dt)
    dr, dm, de = ctx.hllc_rhs(prm, dev(f["rho"]), dev(f["mom"]), dev(f["E"]))
    r_dr, r_dm, r_de, s_dr, s_dm, s_de = O.hllc_rhs(box, w.pos, w.h, rp, col, w.vol, B, po, f["rho"], f["mom"],
                                                    f["E"])
    scaled_check(host(dr), r_dr, s_dr, RTOL, "drho/dt")
    scaled_check(host(dm), r_dm, s_dm, RTOL, "dmom/dt")
    scaled_check(host(de), r_de, s_de, RTOL, "dE/dt")
    steps = int(round(0.1 / dt))
    r, m, e = dev(f["rho"]), dev(f["mom"]), dev(f["E"])
    ctx.hllc_step(prm, r, m, e, steps)
    ro, mo, eo = O.hllc_heun(box, w.pos, w.h, rp, col, w.vol, B, po, f["rho"], f["mom"], f["E"], steps)
    assert normwise(host(r), ro) < 1e-3
    assert normwise(host(m), mo) < 1e-3
    assert normwise(host(e), eo) < 1e-3


def test_hllc_arguments(S):
    w = I.density_wave_2d(nside=16)
    ctx = _ctx(S, w, 1.6)
    f = w.fields
    r, m, e = dev(f["rho"]), dev(f["mom"]), dev(f["E"])
    with pytest.raises(S.SphError, match="gamma"):
        ctx.hllc_rhs(S.hllc_params(1.0, 1.0), r, m, e)
    with pytest.raises(S.SphError, match="dt"):
        ctx.hllc_step(S.hllc_params(GAMMA, 1.0, 0.0), r, m, e, 1)
    ctx3 = S.Context(3)
    w3 = I.taylor_green_3d(nside=12)
    ctx3.build_cells(S.Domain(dim=3, h=w3.h, kappa=1.6), dev(w3.pos))
    ctx3.correction_B(dev(w3.vol))
    z = dev(np.zeros(w3.n, np.float32))
    with pytest.raises(S.SphError, match="2-D"):
        ctx3.hllc_rhs(S.hllc_params(GAMMA, 1.0), z, dev(np.zeros((3, w3.n), np.float32)), z)
