"""Pins of the oracle's compressible rows (limited HLLC, energy equation,
ideal gas) against things other than itself: special states of the Riemann
problem whose answer is known without the solver (equal states, supersonic
pairs, a symmetric collision, mirror symmetry), invariants of the discrete
equations (zero rates for a uniform state on a lattice, conservation of
mass, momentum and energy), the exact solution of an advected density wave
and the exact solution of Sod's shock tube (paper_2405_05155_amd/exact.py,
the textbook exact Riemann solver, which shares nothing with the oracle).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2405_05155_amd import inputs as I
from paper_2405_05155_amd.exact import sod_density as _exact_sod_density

GAMMA = 1.4


def _energy(rho, v, p):
    return p / (GAMMA - 1.0) + 0.5 * rho * float(np.dot(v, v))


def _unit(rng, dim):
    n = rng.normal(size=dim)
    return n / np.linalg.norm(n)


@pytest.mark.parametrize("dim", [2, 3])
def test_equal_states_give_the_state_back(dim):
    """With l = r there is no wave: the interface carries the state itself
    (whatever the direction, the tangential velocity and the limiter)."""
    rng = np.random.default_rng(1)
    prm = O.hllc_params(GAMMA, 1.0)
    for _ in range(20):
        nrm = _unit(rng, dim)
        rho, p = rng.uniform(0.2, 3.0), rng.uniform(0.1, 5.0)
        v = rng.normal(size=dim) * 0.5
        rI, vI, pI, EI = O.hllc_interface(nrm, prm, rho, v, p, rho, v, p)
        assert rI == pytest.approx(rho, rel=1e-13) and pI == pytest.approx(p, rel=1e-13)
        assert np.allclose(vI, v, rtol=0, atol=1e-13)
        assert EI == pytest.approx(_energy(rho, v, p), rel=1e-13)


def test_supersonic_pairs_take_the_upwind_state():
    """All waves moving right (u - c > 0 on the left) leave the left state at
    the interface; all moving left, the right state."""
    prm = O.hllc_params(GAMMA, 1.0)
    nrm = np.array([1.0, 0.0])
    vl, vr = np.array([3.0, 0.2]), np.array([2.5, -0.1])
    rI, vI, pI, EI = O.hllc_interface(nrm, prm, 1.0, vl, 1.0, 0.5, vr, 0.4)
    assert (rI, pI) == (1.0, 1.0) and np.array_equal(vI, vl) and EI == pytest.approx(_energy(1.0, vl, 1.0))
    rI, vI, pI, EI = O.hllc_interface(nrm, prm, 1.0, -vl, 1.0, 0.5, -vr, 0.4)
    assert (rI, pI) == (0.5, 0.4) and np.array_equal(vI, -vr) and EI == pytest.approx(_energy(0.5, -vr, 0.4))


def test_symmetric_collision_gives_the_impedance_pressure():
    """Two equal states colliding head on at speed U (c/2 <= U < c: subsonic,
    limiter fully on since (u_l - u_r)/c = 2U/c >= 1): the interface is at
    rest, the pressure is p + rho c U (the acoustic impedance relation, from
    either side of the fan: p* = p_l + rho_l c_l (u_l - u*)), the tangential
    velocity is kept, and the left star density is rho (S_l - u_l)/(S_l - u*)
    = rho c/(c - U) with S_l = U - c."""
    prm = O.hllc_params(GAMMA, 1.0)
    rho, p = 1.0, 1.0
    c = np.sqrt(GAMMA * p / rho)
    U = 0.75 * c
    nrm = np.array([0.0, 1.0])
    vl, vr = np.array([0.3, U]), np.array([0.3, -U])
    rI, vI, pI, EI = O.hllc_interface(nrm, prm, rho, vl, p, rho, vr, p)
    assert vI[1] == pytest.approx(0.0, abs=1e-14)
    assert vI[0] == pytest.approx(0.3, rel=1e-14)
    assert pI == pytest.approx(p + rho * c * U, rel=1e-13)
    # left star state (u* = 0): rho (S_l - u_l)/(S_l - 0) with S_l = U - c
    assert rI == pytest.approx(rho * (-c) / (U - c), rel=1e-13)


def test_diverging_pairs_are_dissipation_free():
    """Separating states (u_l < u_r) switch the limiter off: the middle
    pressure is the plain mean of the two pressures."""
    prm = O.hllc_params(GAMMA, 1.0)
    rng = np.random.default_rng(3)
    for _ in range(20):
        nrm = _unit(rng, 2)
        rl, rr = rng.uniform(0.5, 2.0, 2)
        pl, pr = rng.uniform(0.5, 2.0, 2)
        t = np.array([-nrm[1], nrm[0]]) * rng.normal()
        vl, vr = -0.2 * nrm + t, 0.3 * nrm + t
        _, _, pI, _ = O.hllc_interface(nrm, prm, rl, vl, pl, rr, vr, pr)
        assert pI == pytest.approx(0.5 * (pl + pr), rel=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_mirror_symmetry(dim):
    """Swapping the two states and reversing the direction gives the same
    interface state (the pair terms of Eq. (19) are then antisymmetric)."""
    rng = np.random.default_rng(4)
    prm = O.hllc_params(GAMMA, 1.0)
    for _ in range(50):
        nrm = _unit(rng, dim)
        rl, rr = rng.uniform(0.3, 3.0, 2)
        pl, pr = rng.uniform(0.2, 4.0, 2)
        vl, vr = rng.normal(size=dim), rng.normal(size=dim)
        a = O.hllc_interface(nrm, prm, rl, vl, pl, rr, vr, pr)
        b = O.hllc_interface(-nrm, prm, rr, vr, pr, rl, vl, pl)
        if abs(np.dot(a[1], nrm)) < 1e-12:  # a contact exactly at rest picks a side
            continue
        assert a[0] == pytest.approx(b[0], rel=1e-12) and a[2] == pytest.approx(b[2], rel=1e-12)
        assert np.allclose(a[1], b[1], rtol=1e-12, atol=1e-12) and a[3] == pytest.approx(b[3], rel=1e-12)


def _setup(w, kappa):
    box = O.make_box(2, lo=w.lo, hi=w.hi, periodic=w.periodic)
    rc = kappa * w.h
    rp, col = O.neighbors_grid(box, w.pos, rc, rc * rc)
    B, _ = O.correction_B(box, w.pos, O.WENDLAND, w.h, rp, col, w.vol)
    return box, rp, col, B


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_uniform_state_on_a_lattice_has_zero_rates(kappa):
    """A uniform moving gas on a lattice: the corrected gradients of the
    constant flux cancel by symmetry, so every rate vanishes."""
    w = I.periodic_square_case(32, 2, 1.3, 0.0, None, "lattice")
    box, rp, col, B = _setup(w, kappa)
    rho = np.full(w.n, 1.3)
    v = np.array([0.7, -0.4])
    mom = np.outer(v, rho)
    E = np.full(w.n, _energy(1.3, v, 2.0))
    dr, dm, de, sr, sm, se = O.hllc_rhs(box, w.pos, w.h, rp, col, w.vol, B, O.hllc_params(GAMMA, 1.0), rho, mom, E)
    assert np.abs(dr).max() < 1e-12 * sr.max()
    assert np.abs(dm).max() < 1e-12 * sm.max()
    assert np.abs(de).max() < 1e-12 * se.max()


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_rates_conserve_mass_momentum_and_energy(kappa):
    """Jittered particles, random states (including shocks and supersonic
    pairs): the volume-weighted totals of all rates vanish."""
    w = I.periodic_square_case(32, 2, 1.3, 0.2, 5, "jittered")
    box, rp, col, B = _setup(w, kappa)
    rng = np.random.default_rng(6)
    rho = rng.uniform(0.5, 2.0, w.n)
    v = rng.normal(size=(2, w.n)) * 1.5
    p = rng.uniform(0.3, 3.0, w.n)
    E = p / (GAMMA - 1.0) + 0.5 * rho * (v ** 2).sum(0)
    dr, dm, de, sr, sm, se = O.hllc_rhs(box, w.pos, w.h, rp, col, w.vol, B, O.hllc_params(GAMMA, 1.0),
                                        rho, rho * v, E)
    V = w.vol.astype(np.float64)
    assert abs(np.sum(V * dr)) < 1e-12 * np.sum(V * sr)
    for a in range(2):
        assert abs(np.sum(V * dm[a])) < 1e-12 * np.sum(V * sm[a])
    assert abs(np.sum(V * de)) < 1e-12 * np.sum(V * se)


def _wave_error(nside, kappa):
    w = I.density_wave_2d(nside=nside, amplitude=0.1, U=1.0, p0=1.0)
    box, rp, col, B = _setup(w, kappa)
    f = w.fields
    dt = w.meta["dt"]
    steps = int(round(0.25 / dt))
    t = steps * dt
    rho, mom, E = O.hllc_heun(box, w.pos, w.h, rp, col, w.vol, B, O.hllc_params(GAMMA, 1.0, dt),
                              f["rho"], f["mom"], f["E"], steps)
    x = w.pos[0].astype(np.float64)
    exact = 1.0 + 0.1 * np.sin(2 * np.pi * (x - t))
    unmoved = 1.0 + 0.1 * np.sin(2 * np.pi * x)
    v = mom / rho
    p = (GAMMA - 1.0) * (E - 0.5 * rho * (v ** 2).sum(0))
    V = w.vol.astype(np.float64)
    drift = (abs(np.sum(V * rho) - np.sum(V * f["rho"].astype(np.float64))),
             abs(np.sum(V * E) - np.sum(V * f["E"].astype(np.float64))))
    return (np.linalg.norm(rho - exact) / np.linalg.norm(unmoved - exact), np.abs(p - 1.0).max(),
            max(np.abs(v[0] - 1.0).max(), np.abs(v[1]).max()), drift)


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_density_wave_is_advected(kappa):
    """rho = 1 + 0.1 sin(2 pi x) carried at U = 1 with uniform pressure (a
    contact wave, exact solution the shifted profile): after a quarter
    period the error against the shifted profile is a small fraction of the
    distance between the shifted and unshifted profiles (1 for a wave that
    stands still, about 1.4 for one moving the wrong way), it falls with
    resolution, pressure and velocity stay uniform, mass and energy are
    conserved."""
    e48, p48, v48, d48 = _wave_error(48, kappa)
    e96, p96, v96, d96 = _wave_error(96, kappa)
    assert e48 < 0.1 and e96 < 0.6 * e48
    assert max(p48, p96) < 1e-3 and max(v48, v96) < 1e-3
    assert max(d48 + d96) < 1e-11


def _sod_error(nx, kappa):
    w = I.sod_strip_2d(nx)
    box, rp, col, B = _setup(w, kappa)
    f = w.fields
    dt = w.meta["dt"]
    steps = int(round(0.1 / dt))
    t = steps * dt
    rho, mom, E = O.hllc_heun(box, w.pos, w.h, rp, col, w.vol, B, O.hllc_params(GAMMA, 1.0, dt),
                              f["rho"], f["mom"], f["E"], steps)
    x = w.pos[0].astype(np.float64)
    sel = x >= 0.5
    exact = np.array([_exact_sod_density((xx - 0.75) / t) for xx in x[sel]])
    V = w.vol.astype(np.float64)
    drift = (abs(np.sum(V * rho) - np.sum(V * f["rho"].astype(np.float64))),
             abs(np.sum(V * E) - np.sum(V * f["E"].astype(np.float64))))
    return float(np.mean(np.abs(rho[sel] - exact))), drift


@pytest.mark.parametrize("kappa", [2.0, 1.6])
def test_sod_shock_tube(kappa):
    """Sod's shock tube in a periodic strip: at t = 0.1 the densities on
    [1/2, 1) (the Riemann problem at x = 3/4: rarefaction, contact, shock)
    follow the exact solution with a mean error below 1.5e-2 at dx = 1/256
    that falls at 1/512, with mass and energy conserved.  The exact sampler
    reproduces the textbook star densities 0.42632 and 0.26557."""
    assert abs(_exact_sod_density(0.5) - 0.42632) < 1e-4
    assert abs(_exact_sod_density(1.5) - 0.26557) < 1e-4
    e256, d256 = _sod_error(256, kappa)
    e512, d512 = _sod_error(512, kappa)
    assert e256 < 1.5e-2 and e512 < 0.75 * e256
    assert max(d256 + d512) < 1e-11
