"""FP64 CPU oracle for the truncated-Wendland SPH hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2405_05155_amd``) and imports nothing from it.

The arithmetic lives in ``sph_oracle.c`` (plain C, FP64, ascending-j sums);
this module only marshals numpy arrays into it.  The MLP part of the oracle is
plain numpy in ``oracle/mlp.py``.  All inputs are promoted to float64 here;
FP32 inputs promote exactly.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsph_oracle.so")

WENDLAND = 0
LAGUERRE_GAUSS = 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Box(C.Structure):
    _fields_ = [("dim", C.c_int), ("periodic", C.c_int * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class EulerParams(C.Structure):
    _fields_ = [("c", C.c_double), ("rho0", C.c_double), ("eta", C.c_double),
                ("mu", C.c_double), ("dt", C.c_double)]


class HllcParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("eta", C.c_double), ("dt", C.c_double)]


class TlsphParams(C.Structure):
    _fields_ = [("rho0", C.c_double), ("E", C.c_double), ("nu", C.c_double),
                ("dt", C.c_double), ("model", C.c_int)]


class RelaxParams(C.Structure):
    _fields_ = [("p0", C.c_double), ("rho", C.c_double), ("h", C.c_double),
                ("center", C.c_double * 3), ("radius", C.c_double),
                ("kappa", C.c_double), ("mu", C.c_double), ("max_move", C.c_double), ("kernel", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB_PATH if os.path.exists(_LIB_PATH) else build()
        L = C.CDLL(path)
        d, i64, i32, vp = C.c_double, C.c_int64, C.c_int, C.c_void_p
        L.or_num_threads.restype = C.c_int
        L.or_kernel_W.restype = d
        L.or_kernel_W.argtypes = [i32, i32, d, d]
        L.or_kernel_dWdr.restype = d
        L.or_kernel_dWdr.argtypes = [i32, i32, d, d]
        L.or_kernel_eval.argtypes = [i32, i32, d, i64, vp, vp, vp]
        L.or_neighbors_brute.restype = i64
        L.or_neighbors_brute.argtypes = [vp, i64, vp, d, i64, vp, vp, vp, i64]
        L.or_neighbors_grid.restype = i64
        L.or_neighbors_grid.argtypes = [vp, i64, vp, d, d, i64, vp, vp, vp, i64]
        L.or_kernel_sum.argtypes = [vp, i64, vp, i32, d, i64, vp, vp, vp, vp, vp]
        L.or_correction_B.restype = i64
        L.or_correction_B.argtypes = [vp, i64, vp, i32, d, i64, vp, vp, vp, vp, vp]
        L.or_gradient.argtypes = [vp, i64, vp, i32, d, i64, vp, vp, vp, vp, vp, vp, vp]
        L.or_euler_rhs.argtypes = [vp, i64, vp, d, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.or_euler_heun.argtypes = [vp, i64, vp, d, vp, vp, vp, vp, vp, vp, vp, i64]
        L.or_hllc_interface.argtypes = [i32, vp, d, d, d, vp, d, d, vp, d, vp, vp, vp, vp]
        L.or_hllc_rhs.argtypes = [vp, i64, vp, d, i64] + [vp] * 15
        L.or_hllc_heun.argtypes = [vp, i64, vp, d, vp, vp, vp, vp, vp, vp, vp, vp, i64]
        L.or_tlsph_stress.argtypes = [i32, vp, vp, vp]
        L.or_tlsph_rhs.argtypes = [vp, i64, vp, d, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.or_tlsph_step.argtypes = [vp, i64, vp, d, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i64]
        L.or_relax_tail.restype = d
        L.or_relax_tail.argtypes = [vp, d]
        L.or_relax_tail2.restype = d
        L.or_relax_tail2.argtypes = [vp, d]
        L.or_relax_g.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.or_relax_step.restype = d
        L.or_relax_step.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers

def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_box(dim, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), periodic=(1, 1, 1)) -> Box:
    b = Box()
    b.dim = int(dim)
    for a in range(3):
        b.periodic[a] = int(periodic[a]) if a < dim else 0
        b.lo[a] = float(lo[a]) if a < len(lo) else 0.0
        b.hi[a] = float(hi[a]) if a < len(hi) else 1.0
    return b


def _rows(rows, n):
    if rows is None:
        return None, n
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    return r, int(r.shape[0])


def num_threads() -> int:
    return int(lib().or_num_threads())


# ---------------------------------------------------------------- kernels

def kernel_W(kernel, dim, h, r):
    r = _f64(np.atleast_1d(r))
    W = np.empty_like(r)
    lib().or_kernel_eval(kernel, dim, h, r.size, _p(r), _p(W), None)
    return W


def kernel_dWdr(kernel, dim, h, r):
    r = _f64(np.atleast_1d(r))
    D = np.empty_like(r)
    lib().or_kernel_eval(kernel, dim, h, r.size, _p(r), None, _p(D))
    return D


# ---------------------------------------------------------------- neighbours

def neighbors_brute(box, pos, rc2, rows=None):
    """CSR (row_ptr int64, col int32) of {j != i : |r_ij|^2 <= rc2}, brute force."""
    pos = _f64(pos)
    n = pos.shape[1]
    r, m = _rows(rows, n)
    rp = np.zeros(m + 1, dtype=np.int64)
    nnz = lib().or_neighbors_brute(C.byref(box), n, _p(pos), rc2, m, _p(r), _p(rp), None, 0)
    col = np.empty(max(nnz, 1), dtype=np.int32)
    lib().or_neighbors_brute(C.byref(box), n, _p(pos), rc2, m, _p(r), _p(rp), _p(col), nnz)
    return rp, col[:nnz]


def neighbors_grid(box, pos, rc, rc2, rows=None):
    """Same set as neighbors_brute, found through a uniform cell grid."""
    pos = _f64(pos)
    n = pos.shape[1]
    r, m = _rows(rows, n)
    rp = np.zeros(m + 1, dtype=np.int64)
    nnz = lib().or_neighbors_grid(C.byref(box), n, _p(pos), rc, rc2, m, _p(r), _p(rp), None, 0)
    col = np.empty(max(nnz, 1), dtype=np.int32)
    lib().or_neighbors_grid(C.byref(box), n, _p(pos), rc, rc2, m, _p(r), _p(rp), _p(col), nnz)
    return rp, col[:nnz]


# ---------------------------------------------------------------- pair sums

def kernel_sum(box, pos, kernel, h, row_ptr, col, vol, rows=None):
    pos, vol = _f64(pos), _f64(vol)
    n = pos.shape[1]
    r, m = _rows(rows, n)
    out = np.empty(m)
    lib().or_kernel_sum(C.byref(box), n, _p(pos), kernel, h, m, _p(r), _p(row_ptr), _p(col), _p(vol), _p(out))
    return out


def correction_B(box, pos, kernel, h, row_ptr, col, vol, rows=None):
    """Returns (B [m][d][d], number of degenerate rows)."""
    pos, vol = _f64(pos), _f64(vol)
    n, d = pos.shape[1], box.dim
    r, m = _rows(rows, n)
    B = np.empty((m, d, d))
    ndeg = lib().or_correction_B(C.byref(box), n, _p(pos), kernel, h, m, _p(r), _p(row_ptr), _p(col),
                                 _p(vol), _p(B))
    return B, int(ndeg)


def gradient(box, pos, kernel, h, row_ptr, col, vol, B, f, rows=None):
    """B is full [n][d][d] (rows i used); returns grad [d][m]."""
    pos, vol, B, f = _f64(pos), _f64(vol), _f64(B), _f64(f)
    n, d = pos.shape[1], box.dim
    r, m = _rows(rows, n)
    out = np.empty((d, m))
    lib().or_gradient(C.byref(box), n, _p(pos), kernel, h, m, _p(r), _p(row_ptr), _p(col), _p(vol), _p(B),
                      _p(f), _p(out))
    return out


def euler_params(c, rho0, eta=15.0, mu=0.0, dt=0.0) -> EulerParams:
    p = EulerParams()
    p.c, p.rho0, p.eta, p.mu, p.dt = c, rho0, eta, mu, dt
    return p


def euler_rhs(box, pos, h, row_ptr, col, vol, B, prm, rho, mom, rows=None):
    """Returns (drho [m], dmom [d][m], scale_rho [m], scale_mom [d][m]).

    rho is the density (not a deviation); mom = rho v, [d][n]; B full [n][d][d].
    """
    pos, vol, B, rho, mom = _f64(pos), _f64(vol), _f64(B), _f64(rho), _f64(mom)
    n, d = pos.shape[1], box.dim
    r, m = _rows(rows, n)
    dr, dm = np.empty(m), np.empty((d, m))
    sr, sm = np.empty(m), np.empty((d, m))
    lib().or_euler_rhs(C.byref(box), n, _p(pos), h, m, _p(r), _p(row_ptr), _p(col), _p(vol), _p(B),
                       C.byref(prm), _p(rho), _p(mom), _p(dr), _p(dm), _p(sr), _p(sm))
    return dr, dm, sr, sm


def euler_heun(box, pos, h, row_ptr, col, vol, B, prm, rho, mom, nsteps):
    pos, vol, B = _f64(pos), _f64(vol), _f64(B)
    rho, mom = _f64(rho).copy(), _f64(mom).copy()
    lib().or_euler_heun(C.byref(box), pos.shape[1], _p(pos), h, _p(row_ptr), _p(col), _p(vol), _p(B),
                        C.byref(prm), _p(rho), _p(mom), int(nsteps))
    return rho, mom


def hllc_params(gamma=1.4, eta=1.0, dt=0.0) -> HllcParams:
    p = HllcParams()
    p.gamma, p.eta, p.dt = gamma, eta, dt
    return p


def hllc_interface(nrm, prm, rho_l, v_l, p_l, rho_r, v_r, p_r):
    """Interface state (rho, v [d], p, E) of one pair's limited HLLC problem
    along the unit vector nrm (left state l, right state r)."""
    nrm, v_l, v_r = _f64(nrm), _f64(v_l), _f64(v_r)
    dim = nrm.shape[0]
    rI, pI, EI = C.c_double(), C.c_double(), C.c_double()
    vI = np.zeros(dim)
    lib().or_hllc_interface(dim, _p(nrm), prm.gamma, prm.eta, float(rho_l), _p(v_l), float(p_l),
                            float(rho_r), _p(v_r), float(p_r), C.byref(rI), _p(vI), C.byref(pI), C.byref(EI))
    return rI.value, vI, pI.value, EI.value


def hllc_rhs(box, pos, h, row_ptr, col, vol, B, prm, rho, mom, E, rows=None):
    """Compressible rates: returns (drho [m], dmom [d][m], dE [m], scale_rho,
    scale_mom, scale_E); rho the density, mom = rho v [d][n], E the total
    energy per unit volume, B full [n][d][d]."""
    pos, vol, B, rho, mom, E = _f64(pos), _f64(vol), _f64(B), _f64(rho), _f64(mom), _f64(E)
    n, d = pos.shape[1], box.dim
    r, m = _rows(rows, n)
    dr, dm, de = np.empty(m), np.empty((d, m)), np.empty(m)
    sr, sm, se = np.empty(m), np.empty((d, m)), np.empty(m)
    lib().or_hllc_rhs(C.byref(box), n, _p(pos), h, m, _p(r), _p(row_ptr), _p(col), _p(vol), _p(B),
                      C.byref(prm), _p(rho), _p(mom), _p(E), _p(dr), _p(dm), _p(de), _p(sr), _p(sm), _p(se))
    return dr, dm, de, sr, sm, se


def hllc_heun(box, pos, h, row_ptr, col, vol, B, prm, rho, mom, E, nsteps):
    pos, vol, B = _f64(pos), _f64(vol), _f64(B)
    rho, mom, E = _f64(rho).copy(), _f64(mom).copy(), _f64(E).copy()
    lib().or_hllc_heun(C.byref(box), pos.shape[1], _p(pos), h, _p(row_ptr), _p(col), _p(vol), _p(B),
                       C.byref(prm), _p(rho), _p(mom), _p(E), int(nsteps))
    return rho, mom, E


def tlsph_params(rho0, E, nu, dt=0.0, model=0) -> TlsphParams:
    p = TlsphParams()
    p.rho0, p.E, p.nu, p.dt, p.model = rho0, E, nu, dt, model
    return p


def tlsph_stress(dim, prm, F):
    F = _f64(F)
    P = np.empty_like(F)
    lib().or_tlsph_stress(dim, C.byref(prm), _p(F), _p(P))
    return P


def tlsph_rhs(box, pos0, h, row_ptr, col, vol0, B0, prm, vel, F, fixed=None, rows=None):
    """Returns (dFdt [m][d][d], acc [d][m], scale_acc [d][m]); F, B0 full [n][d][d]."""
    pos0, vol0, B0, vel, F = _f64(pos0), _f64(vol0), _f64(B0), _f64(vel), _f64(F)
    fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, dtype=np.int32))
    n, d = pos0.shape[1], box.dim
    r, m = _rows(rows, n)
    dF, acc, sa = np.empty((m, d, d)), np.empty((d, m)), np.empty((d, m))
    lib().or_tlsph_rhs(C.byref(box), n, _p(pos0), h, m, _p(r), _p(row_ptr), _p(col), _p(vol0), _p(B0),
                       C.byref(prm), _p(vel), _p(F), _p(fx), _p(dF), _p(acc), _p(sa))
    return dF, acc, sa


def tlsph_step(box, pos0, h, row_ptr, col, vol0, B0, prm, fixed, pos, vel, F, acc, nsteps):
    pos0, vol0, B0 = _f64(pos0), _f64(vol0), _f64(B0)
    pos, vel, F, acc = _f64(pos).copy(), _f64(vel).copy(), _f64(F).copy(), _f64(acc).copy()
    fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, dtype=np.int32))
    lib().or_tlsph_step(C.byref(box), pos0.shape[1], _p(pos0), h, _p(row_ptr), _p(col), _p(vol0), _p(B0),
                        C.byref(prm), _p(fx), _p(pos), _p(vel), _p(F), _p(acc), int(nsteps))
    return pos, vel, F, acc


def relax_params(h, center, radius, p0=1.0, rho=1.0, kappa=0.1, mu=0.9, max_move=0.1,
                 kernel=LAGUERRE_GAUSS) -> RelaxParams:
    """kernel: LAGUERRE_GAUSS (Eq. 8) or WENDLAND (Eq. 6, support 2h)."""
    p = RelaxParams()
    p.p0, p.rho, p.h, p.radius = p0, rho, h, radius
    p.kappa, p.mu, p.max_move, p.kernel = kappa, mu, max_move, kernel
    for a in range(3):
        p.center[a] = center[a]
    return p


def relax_tail(prm, rho_c, dim=3):
    """Exterior kernel-gradient integral T(rho_c): sphere (dim 3) or circle (dim 2)."""
    f = lib().or_relax_tail2 if dim == 2 else lib().or_relax_tail
    return f(C.byref(prm), float(rho_c))


def relax_g(box, pos, prm, row_ptr, col, vol, rows=None):
    """Returns (g [dim][m], scale [dim][m])."""
    pos, vol = _f64(pos), _f64(vol)
    n = pos.shape[1]
    r, m = _rows(rows, n)
    g, s = np.empty((box.dim, m)), np.empty((box.dim, m))
    lib().or_relax_g(C.byref(box), n, _p(pos), C.byref(prm), m, _p(r), _p(row_ptr), _p(col), _p(vol), _p(g), _p(s))
    return g, s


def relax_step(box, pos, u, prm, row_ptr, col, vol):
    """One iteration; returns (new positions, new carried displacement,
    residue of the input positions, g of the input positions)."""
    pos, u, vol = _f64(pos).copy(), _f64(u).copy(), _f64(vol)
    g = np.empty_like(pos)
    res = lib().or_relax_step(C.byref(box), pos.shape[1], _p(pos), _p(u), C.byref(prm), _p(row_ptr), _p(col),
                              _p(vol), _p(g))
    return pos, u, res, g


def relax_run(box, pos, prm, vol, iters, u=None):
    """iters iterations with a fresh neighbour search each; returns
    (positions, u, residues per iteration)."""
    pos = _f64(pos).copy()
    u = np.zeros_like(pos) if u is None else _f64(u).copy()
    rc = 2.0 * prm.h
    res = []
    for _ in range(iters):
        rp, col = neighbors_grid(box, pos, rc, rc * rc)
        pos, u, r, _ = relax_step(box, pos, u, prm, rp, col, vol)
        res.append(r)
    return pos, u, np.array(res)
