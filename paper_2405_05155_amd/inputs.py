"""Seeded synthetic workloads shared by the HIP path's callers and the oracle.

This module holds only input generators: lattices, seeded jitter, the
quantisation of coordinates, and the initial fields of the workloads.  It
contains none of the SPH method's arithmetic (no kernels, sums, solvers or
integrators), so both the HIP library's tests and the oracle can draw their
inputs from it without sharing any of the method.

Quantisation.  Every coordinate is rounded to a multiple of q = 2**(e - 23)
with 2**e >= max|coordinate|.  Differences of two such numbers are exact in
FP32, so the GPU (FP32 positions) and the oracle (FP64) see identical pair
vectors r_ij and identical squared distances in FP64, which makes neighbour
sets comparable bit for bit.

All arrays returned are numpy: positions float32 SoA [dim][n].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def quantum_for(max_abs: float) -> float:
    e = math.ceil(math.log2(max_abs)) if max_abs > 0 else 0
    return 2.0 ** (e - 23)


def quantise(x: np.ndarray, q: float) -> np.ndarray:
    return (np.round(np.asarray(x, dtype=np.float64) / q) * q)


def wrap_periodic(x: np.ndarray, lo: float, hi: float, q: float) -> np.ndarray:
    """Map into [lo, hi) after quantisation (box length a multiple of q)."""
    L = hi - lo
    x = lo + np.mod(x - lo, L)
    x = quantise(x, q)
    x[x >= hi] -= L
    x[x < lo] += L
    return x


@dataclass
class Workload:
    name: str
    dim: int
    pos: np.ndarray                  # float32 [dim][n]
    vol: np.ndarray                  # float32 [n]
    h: float
    lo: tuple
    hi: tuple
    periodic: tuple
    fields: dict = field(default_factory=dict)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])


def lattice(nside, dim, L=1.0, lo=0.0):
    """Cell-centred lattice (i + 1/2) dx, row-major with axis 0 fastest."""
    dx = L / nside
    axes = [lo + (np.arange(nside) + 0.5) * dx for _ in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    # axis 0 fastest: transpose so that flattening runs x first
    pts = np.stack([g.transpose(tuple(range(dim))[::-1]).reshape(-1) for g in grids])
    return pts, dx


def periodic_square_case(nside: int, dim: int, h_over_dx: float, jitter: float, seed: int | None,
                         name: str) -> Workload:
    pos, dx = lattice(nside, dim)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        pos = pos + rng.uniform(-jitter * dx, jitter * dx, size=pos.shape)
    q = quantum_for(1.0)
    pos = wrap_periodic(pos, 0.0, 1.0, q)
    vol = np.full(pos.shape[1], dx ** dim)
    return Workload(name=name, dim=dim, pos=pos.astype(np.float32), vol=vol.astype(np.float32),
                    h=h_over_dx * dx, lo=(0.0,) * dim, hi=(1.0,) * dim, periodic=(1,) * dim,
                    meta={"dx": dx, "quantum": q, "seed": seed})


# ------------------------------------------------------------------ C0

def single_step_2d(seed: int = 0, nside: int = 64, c: float = 10.0) -> Workload:
    """2-D single-step evaluation: nside^2 particles on the periodic unit
    square, h = 1.3 dx, uniform jitter +-0.05 dx; rho = 1 + 0.01 sin sin,
    Taylor-Green velocity, p = rho c^2 (EOS reference density 0)."""
    w = periodic_square_case(nside, 2, 1.3, 0.05, seed, f"single_step_2d_seed{seed}")
    x = w.pos.astype(np.float64)
    s2x, s2y = np.sin(2 * np.pi * x[0]), np.sin(2 * np.pi * x[1])
    c2x, c2y = np.cos(2 * np.pi * x[0]), np.cos(2 * np.pi * x[1])
    drho = 0.01 * s2x * s2y                       # density = 1 + drho
    u = np.stack([s2x * c2y, -c2x * s2y])
    rho = 1.0 + drho
    mom = rho * u
    w.fields = {"rho_ref": 1.0, "drho": drho.astype(np.float32), "mom": mom.astype(np.float32),
                "c": c, "rho0_eos": 0.0, "eta": 15.0, "mu": 0.0}
    return w


def adversarial_ties_2d(kappa: float = 2.0, nside: int = 64, seed: int = 0):
    """Particles placed exactly on, one quantum inside and one quantum
    outside the cut-off radius.  h is chosen so that kappa*h is an exact
    multiple of the quantum (so r = kappa h is representable exactly)."""
    q = quantum_for(1.0)
    dx = 1.0 / nside
    m = int(round(kappa * 1.3 * dx / q))
    h = m * q / kappa
    rng = np.random.default_rng(seed)
    base = []
    for t in range(16):
        cx, cy = 0.1 + 0.05 * t, 0.2 + 0.04 * (t % 4)
        base.append((cx, cy))
    pts = []
    for t, (cx, cy) in enumerate(base):
        cx, cy = quantise(cx, q), quantise(cy, q)
        pts.append((cx, cy))
        off = [(m, 0), (0, m + 1), (-(m - 1), 0)][t % 3]
        pts.append((cx + off[0] * q, cy + off[1] * q))
    # a Pythagorean exact tie: 3-4-5 scaled (only when m divisible by 5)
    k5 = m // 5
    if k5 > 0:
        cx, cy = quantise(0.6, q), quantise(0.7, q)
        pts.append((cx, cy))
        pts.append((cx + 3 * k5 * q, cy + 4 * k5 * q))
    extra = rng.uniform(0.0, 1.0, size=(64, 2))
    pts = np.array(pts + [tuple(e) for e in extra]).T
    pts = wrap_periodic(pts, 0.0, 1.0, q)
    vol = np.full(pts.shape[1], dx * dx)
    return Workload(name=f"ties_k{kappa}", dim=2, pos=pts.astype(np.float32), vol=vol.astype(np.float32),
                    h=h, lo=(0.0, 0.0), hi=(1.0, 1.0), periodic=(1, 1),
                    meta={"dx": dx, "quantum": q, "m": m, "rc_exact": m * q})


def gradient_lattice_2d(nside: int) -> Workload:
    """The error analysis of Sec. 2.3.3 on the lattice distribution: dp = D /
    nside with D = 2, h = 1.3 dp, f = exp(-x^2 / 0.1).  The lattice fills the
    periodic square [-1, 1)^2 around the paper's circle of diameter 2 (every
    particle an interior one, as for Table 1's lattice row; f is periodic to
    exp(-10) there)."""
    pos, dp = lattice(nside, 2, L=2.0, lo=-1.0)
    q = quantum_for(1.0)
    pos = wrap_periodic(pos, -1.0, 1.0, q)
    vol = np.full(pos.shape[1], dp * dp)
    x = pos[0].astype(np.float32).astype(np.float64)
    f = np.exp(-x ** 2 / 0.1)
    w = Workload(name=f"gradient_lattice_{nside}", dim=2, pos=pos.astype(np.float32), vol=vol.astype(np.float32),
                 h=1.3 * dp, lo=(-1.0, -1.0), hi=(1.0, 1.0), periodic=(1, 1), meta={"dx": dp, "quantum": q})
    w.fields = {"f": f.astype(np.float32), "dfdx": (-20.0 * x * f)}
    return w


def sphere_gradient_fields(pos, center, radius):
    """The error analysis's test function on a filled sphere, scaled to its
    radius: f = exp(-((x - c_x) / R)^2 / 0.1) (the paper's exp(-x^2/0.1) on a
    circle of radius 1) and df/dx, at FP32 positions pos [3][n]."""
    x = (np.asarray(pos, dtype=np.float32).astype(np.float64)[0] - center[0]) / radius
    f = np.exp(-x ** 2 / 0.1)
    return f, -2.0 * x / (0.1 * radius) * f


# ------------------------------------------------------------------ C1 / C4b

def taylor_green_2d(nside: int = 512, c: float = 10.0, nu: float = 0.01) -> Workload:
    """2-D Taylor-Green vortex on the periodic unit square, exact lattice,
    h = 1.3 dx; u = (sin 2pi x cos 2pi y, -cos 2pi x sin 2pi y),
    p = (cos 4pi x + cos 4pi y)/4, rho = 1 + p/c^2."""
    w = periodic_square_case(nside, 2, 1.3, 0.0, None, f"taylor_green_2d_{nside}")
    x = w.pos.astype(np.float64)
    u = np.stack([np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1]),
                  -np.cos(2 * np.pi * x[0]) * np.sin(2 * np.pi * x[1])])
    p = 0.25 * (np.cos(4 * np.pi * x[0]) + np.cos(4 * np.pi * x[1]))
    drho = p / c ** 2
    mom = (1.0 + drho) * u
    w.fields = {"rho_ref": 1.0, "drho": drho.astype(np.float32), "mom": mom.astype(np.float32),
                "c": c, "rho0_eos": 1.0, "eta": 15.0, "mu": 1.0 * nu, "nu": nu}
    dx = w.meta["dx"]
    w.meta["dt"] = min(0.6 * w.h / (c + 1.0), 0.125 * w.h ** 2 / nu) if nu > 0 else 0.6 * w.h / (c + 1.0)
    return w


def double_shear_layer(nside: int = 128, c: float = 10.0, width: float = 1.0 / 30.0,
                       delta: float = 0.05) -> Workload:
    """Doubly periodic shear layer in the unit square, inviscid (Sec. 4.2):
    exact lattice, h = 1.3 dx,
    u_x = tanh((y - 1/4)/width) for y <= 1/2, tanh((3/4 - y)/width) above,
    u_y = delta sin(2 pi x); uniform density rho = 1 (uniform pressure)."""
    w = periodic_square_case(nside, 2, 1.3, 0.0, None, f"double_shear_layer_{nside}")
    x = w.pos.astype(np.float64)
    ux = np.where(x[1] <= 0.5, np.tanh((x[1] - 0.25) / width), np.tanh((0.75 - x[1]) / width))
    uy = delta * np.sin(2 * np.pi * x[0])
    drho = np.zeros(w.n)
    mom = np.stack([ux, uy])
    w.fields = {"rho_ref": 1.0, "drho": drho.astype(np.float32), "mom": mom.astype(np.float32),
                "c": c, "rho0_eos": 1.0, "eta": 15.0, "mu": 0.0, "nu": 0.0}
    w.meta["dt"] = 0.6 * w.h / (c + 1.0)
    return w


def density_wave_2d(nside: int = 512, amplitude: float = 0.1, U: float = 1.0, p0: float = 1.0,
                    gamma: float = 1.4) -> Workload:
    """Compressible ideal gas on the periodic unit square, exact lattice,
    h = 1.3 dx: a density wave rho = 1 + amplitude sin(2 pi x) carried by the
    uniform velocity (U, 0) at uniform pressure p0 (exact solution: the
    profile shifted by U t); E = p0/(gamma - 1) + rho U^2/2 per unit volume."""
    w = periodic_square_case(nside, 2, 1.3, 0.0, None, f"density_wave_2d_{nside}")
    x = w.pos.astype(np.float64)
    rho = 1.0 + amplitude * np.sin(2 * np.pi * x[0])
    mom = np.stack([rho * U, np.zeros(w.n)])
    E = p0 / (gamma - 1.0) + 0.5 * rho * U * U
    w.fields = {"rho": rho.astype(np.float32), "mom": mom.astype(np.float32), "E": E.astype(np.float32),
                "gamma": gamma, "eta": 1.0, "U": U, "p0": p0, "amplitude": amplitude}
    c_max = math.sqrt(gamma * p0 / (1.0 - amplitude))
    w.meta["dt"] = 0.6 * w.h / (abs(U) + c_max)
    return w


def sod_strip_2d(nx: int = 256, ny: int = 16, gamma: float = 1.4) -> Workload:
    """Sod's shock tube in a periodic strip [0, 1) x [0, ny/nx) of lattice
    particles, h = 1.3 dx: rho = 1, p = 1 for 1/4 <= x < 3/4, rho = 0.125,
    p = 0.1 elsewhere, at rest (two mirror-image Riemann problems at x = 1/4
    and 3/4 whose waves do not meet before t = 0.2).  Powers of two for nx
    and ny keep dx and the strip height exact."""
    dx = 1.0 / nx
    xs = (np.arange(nx) + 0.5) * dx
    ys = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    pos = np.stack([X.T.reshape(-1), Y.T.reshape(-1)])
    q = quantum_for(1.0)
    hi_y = ny * dx
    pos = np.stack([wrap_periodic(pos[0], 0.0, 1.0, q), wrap_periodic(pos[1], 0.0, hi_y, q)])
    x = pos[0]
    inside = (x >= 0.25) & (x < 0.75)
    rho = np.where(inside, 1.0, 0.125)
    p = np.where(inside, 1.0, 0.1)
    E = p / (gamma - 1.0)
    w = Workload(name=f"sod_strip_{nx}x{ny}", dim=2, pos=pos.astype(np.float32),
                 vol=np.full(pos.shape[1], dx * dx, dtype=np.float32), h=1.3 * dx, lo=(0.0, 0.0),
                 hi=(1.0, hi_y), periodic=(1, 1), meta={"dx": dx, "quantum": q})
    w.fields = {"rho": rho.astype(np.float32), "mom": np.zeros((2, w.n), np.float32), "E": E.astype(np.float32),
                "gamma": gamma, "eta": 1.0}
    c_max = math.sqrt(gamma)
    w.meta["dt"] = 0.3 * w.h / c_max
    return w


def taylor_green_3d(nside: int = 200, c: float = 10.0, nu: float = 0.01, jitter: float = 0.0,
                    seed: int | None = None) -> Workload:
    """3-D Taylor-Green field in the periodic unit cube, h = 1.3 dx, on the
    exact lattice (or jittered by seeded uniform +-jitter dx per component);
    u = sin cos cos, v = -cos sin cos, w = 0,
    p = (cos 4pi x + cos 4pi y)(cos 4pi z + 2)/16, rho = 1 + p/c^2."""
    w = periodic_square_case(nside, 3, 1.3, jitter, seed, f"taylor_green_3d_{nside}")
    x = w.pos.astype(np.float64)
    sx, sy, sz = (np.sin(2 * np.pi * x[a]) for a in range(3))
    cx, cy, cz = (np.cos(2 * np.pi * x[a]) for a in range(3))
    u = np.stack([sx * cy * cz, -cx * sy * cz, np.zeros_like(sx)])
    p = (np.cos(4 * np.pi * x[0]) + np.cos(4 * np.pi * x[1])) * (np.cos(4 * np.pi * x[2]) + 2.0) / 16.0
    drho = p / c ** 2
    mom = (1.0 + drho) * u
    w.fields = {"rho_ref": 1.0, "drho": drho.astype(np.float32), "mom": mom.astype(np.float32),
                "c": c, "rho0_eos": 1.0, "eta": 15.0, "mu": 1.0 * nu, "nu": nu}
    w.meta["dt"] = min(0.6 * w.h / (c + 1.0), 0.125 * w.h ** 2 / nu) if nu > 0 else 0.6 * w.h / (c + 1.0)
    return w


# ------------------------------------------------------------------ C2

def cantilever_plate(nx: int = 430, length: float = 0.2, thick: float = 0.02, width: float = 0.04,
                     clamp_layers: int = 4, E: float = 2.0e6, nu: float = 0.3975, rho0: float = 1000.0,
                     vf: float = 0.05) -> Workload:
    """3-D cantilever plate, x = length, y = thickness (bending), z = width,
    clamped by `clamp_layers` layers of fixed particles at x < 0.  Initial
    velocity v_y = vf c0 f(x)/f(L) with f the first clamped-free beam mode
    (beta L = 1.875104), c0 = sqrt(K/rho0), K = E/(3(1-2 nu))."""
    dx = length / nx
    ny = int(round(thick / dx))
    nz = int(round(width / dx))
    xs = (np.arange(-clamp_layers, nx) + 0.5) * dx
    ys = (np.arange(ny) + 0.5) * dx
    zs = (np.arange(nz) + 0.5) * dx
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    pos = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)])
    q = quantum_for(max(length, width, thick, clamp_layers * dx))
    pos = quantise(pos, q)
    n = pos.shape[1]
    fixed = (pos[0] < 0.0).astype(np.int32)
    K = E / (3.0 * (1.0 - 2.0 * nu))
    c0 = math.sqrt(K / rho0)
    bl = 1.875104
    beta = bl / length
    kk = (math.cosh(bl) + math.cos(bl)) / (math.sinh(bl) + math.sin(bl))

    def mode(x):
        return (np.cosh(beta * x) - np.cos(beta * x)) - kk * (np.sinh(beta * x) - np.sin(beta * x))

    xp = np.clip(pos[0], 0.0, None)
    vel = np.zeros((3, n))
    vel[1] = vf * c0 * mode(xp) / mode(length)
    vel[:, fixed.astype(bool)] = 0.0
    h = 1.15 * dx
    dt = 0.6 * h / (c0 + np.abs(vel).max())
    vol = np.full(n, dx ** 3)
    lo = (-(clamp_layers + 1) * dx, 0.0, 0.0)
    hi = (length + dx, thick + dx, width + dx)
    return Workload(name=f"cantilever_plate_{nx}", dim=3, pos=pos.astype(np.float32),
                    vol=vol.astype(np.float32), h=h, lo=lo, hi=hi, periodic=(0, 0, 0),
                    fields={"vel": vel.astype(np.float32), "fixed": fixed, "E": E, "nu": nu, "rho0": rho0},
                    meta={"dx": dx, "quantum": q, "dt": dt, "c0": c0, "shape": (nz, ny, nx + clamp_layers)})


# ------------------------------------------------------------------ C3

def sphere_fill(dx: float = 1.0 / 260, radius: float = 0.3, center=(0.5, 0.5, 0.5),
                jitter: float = 0.4, seed: int = 1) -> Workload:
    """Cell-centred lattice points of the unit cube with |r - c| < R,
    perturbed by seeded uniform +-jitter*dx per component and quantised."""
    nside = int(round(1.0 / dx))
    axis = (np.arange(nside) + 0.5) * dx
    keep = []
    c = np.asarray(center)
    # build slab by slab to bound memory
    Y, X = np.meshgrid(axis, axis, indexing="ij")
    for kz, z in enumerate(axis):
        r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (z - c[2]) ** 2
        m = r2 < radius ** 2
        if m.any():
            keep.append(np.stack([X[m], Y[m], np.full(m.sum(), z)]))
    pos = np.concatenate(keep, axis=1)
    rng = np.random.default_rng(seed)
    pos = pos + rng.uniform(-jitter * dx, jitter * dx, size=pos.shape)
    q = quantum_for(1.0)
    pos = quantise(pos, q)
    n = pos.shape[1]
    vol = np.full(n, dx ** 3)
    h = 1.3 * dx
    return Workload(name=f"sphere_relax_{nside}_seed{seed}", dim=3, pos=pos.astype(np.float32),
                    vol=vol.astype(np.float32), h=h, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                    periodic=(0, 0, 0), fields={"center": tuple(center), "radius": radius, "p0": 1.0, "rho": 1.0},
                    meta={"dx": dx, "quantum": q, "seed": seed})


def circle_fill(dx: float = 0.2, radius: float = 1.0, jitter: float = 0.4, seed: int = 2) -> Workload:
    """2-D counterpart of sphere_fill for the error analysis's circle
    (diameter D = 2 R, centre at the origin): cell-centred lattice points
    (i + 1/2) dx of the square [-R, R]^2 with |r| < R, perturbed by seeded
    uniform +-jitter*dx per component and quantised; box [-1.5 R, 1.5 R]^2,
    open; h = 1.3 dx, V = dx^2."""
    nside = int(round(2.0 * radius / dx))
    axis = -radius + (np.arange(nside) + 0.5) * dx
    Y, X = np.meshgrid(axis, axis, indexing="ij")
    m = X ** 2 + Y ** 2 < radius ** 2
    pos = np.stack([X[m], Y[m]])
    rng = np.random.default_rng(seed)
    pos = pos + rng.uniform(-jitter * dx, jitter * dx, size=pos.shape)
    q = quantum_for(2.0 * radius)
    pos = quantise(pos, q)
    n = pos.shape[1]
    vol = np.full(n, dx ** 2)
    b = 1.5 * radius
    return Workload(name=f"circle_relax_{nside}_seed{seed}", dim=2, pos=pos.astype(np.float32),
                    vol=vol.astype(np.float32), h=1.3 * dx, lo=(-b, -b), hi=(b, b), periodic=(0, 0),
                    fields={"center": (0.0, 0.0, 0.0), "radius": radius, "p0": 1.0, "rho": 1.0},
                    meta={"dx": dx, "quantum": q, "seed": seed})


def circle_gradient_fields(pos):
    """The error analysis's function on the circle of diameter 2 about the
    origin: f = exp(-x^2/0.1) and its exact df/dx = -20 x f, at FP32
    positions [2][n] (FP64 values)."""
    x = np.asarray(pos, dtype=np.float64)[0]
    f = np.exp(-x * x / 0.1)
    return f, -20.0 * x * f


def random_points(n: int, dim: int, seed: int, periodic: bool = True, h_over_dx: float = 1.3) -> Workload:
    """Uniform random points in the unit box (for neighbour-search tests)."""
    rng = np.random.default_rng(seed)
    q = quantum_for(1.0)
    pos = rng.uniform(0.0, 1.0, size=(dim, n))
    pos = wrap_periodic(pos, 0.0, 1.0, q) if periodic else np.clip(quantise(pos, q), 0.0, 1.0 - q)
    dx = n ** (-1.0 / dim)
    vol = np.full(n, dx ** dim)
    return Workload(name=f"random_{dim}d_{n}_seed{seed}", dim=dim, pos=pos.astype(np.float32),
                    vol=vol.astype(np.float32), h=h_over_dx * dx, lo=(0.0,) * dim, hi=(1.0,) * dim,
                    periodic=(int(periodic),) * dim, meta={"dx": dx, "quantum": q, "seed": seed})
