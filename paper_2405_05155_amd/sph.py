"""Thin ctypes binding of libsph.so (the C ABI in include/sph.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libsph.so.  Tensors must be CUDA (HIP) tensors of the stated
dtype, contiguous, on the context's device; they are passed by data_ptr()
and the calls are enqueued on the stream given at context creation
(torch's current stream by default).  If libsph.so is missing the first call
raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsph.so")

SPH_OK, SPH_ERR_ARG, SPH_ERR_CAPACITY, SPH_ERR_HIP, SPH_ERR_STATE = 0, -1, -2, -3, -5
WENDLAND, LAGUERRE_GAUSS = 0, 1
PATH_NONE, PATH_GENERIC, PATH_RECORDS, PATH_WINDOWS = 0, 1, 2, 3


class SphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class sph_domain(C.Structure):
    _fields_ = [("dim", C.c_int), ("periodic", C.c_int * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("h", C.c_double), ("kappa", C.c_double), ("kernel", C.c_int)]


class sph_euler_params(C.Structure):
    _fields_ = [("c", C.c_double), ("rho0", C.c_double), ("rho_ref", C.c_double), ("eta", C.c_double),
                ("mu", C.c_double), ("dt", C.c_double)]


class sph_hllc_params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("eta", C.c_double), ("dt", C.c_double)]


class sph_tlsph_params(C.Structure):
    _fields_ = [("rho0", C.c_double), ("E", C.c_double), ("nu", C.c_double), ("dt", C.c_double),
                ("model", C.c_int)]


class sph_relax_params(C.Structure):
    _fields_ = [("p0", C.c_double), ("rho", C.c_double), ("center", C.c_double * 3), ("radius", C.c_double),
                ("kappa", C.c_double), ("damping", C.c_double), ("max_move", C.c_double), ("kernel", C.c_int32)]


_lib = None

# (name, restype, argtypes)
_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_SIGS = [
    ("sph_ctx_create", C.c_int, [C.POINTER(C.c_void_p), C.c_int, _vp]),
    ("sph_ctx_destroy", None, [_vp]),
    ("sph_last_error", C.c_char_p, [_vp]),
    ("sph_set_stream", C.c_int, [_vp, _vp]),
    ("sph_euler_path", C.c_int, [_vp]),
    ("sph_tlsph_path", C.c_int, [_vp]),
    ("sph_build_cells", C.c_int, [_vp, C.POINTER(sph_domain), _i32, _vp]),
    ("sph_neighbors", C.c_int, [_vp, _vp, _vp, _i64, C.POINTER(C.c_int64)]),
    ("sph_kernel_sum", C.c_int, [_vp, _vp, _vp]),
    ("sph_correction_B", C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(C.c_int32)]),
    ("sph_set_correction", C.c_int, [_vp, _vp, _vp]),
    ("sph_gradient", C.c_int, [_vp, _vp, _vp]),
    ("sph_euler_rhs", C.c_int, [_vp, C.POINTER(sph_euler_params), _vp, _vp, _vp, _vp]),
    ("sph_euler_step", C.c_int, [_vp, C.POINTER(sph_euler_params), _vp, _vp, _i32]),
    ("sph_hllc_rhs", C.c_int, [_vp, C.POINTER(sph_hllc_params), _vp, _vp, _vp, _vp, _vp, _vp]),
    ("sph_hllc_step", C.c_int, [_vp, C.POINTER(sph_hllc_params), _vp, _vp, _vp, _i32]),
    ("sph_tlsph_rhs", C.c_int, [_vp, C.POINTER(sph_tlsph_params), _vp, _vp, _vp, _vp, _vp]),
    ("sph_tlsph_step", C.c_int, [_vp, C.POINTER(sph_tlsph_params), _vp, _vp, _vp, _vp, _vp, _i32]),
]
_SIGS += [
    ("sph_relax_step", C.c_int, [_vp, C.POINTER(sph_domain), C.POINTER(sph_relax_params), _i32, _vp, _vp, _vp,
                                 _vp, _i32]),
    ("sph_relax_residue", C.c_int, [_vp, C.POINTER(sph_domain), C.POINTER(sph_relax_params), _i32, _vp, _vp, _vp,
                                    _vp]),
]
_SIGS += [
    ("sph_mlp_features", C.c_int, [_vp, C.POINTER(sph_domain), C.POINTER(sph_relax_params), _i32, _vp, _vp]),
    ("sph_mlp_forward", C.c_int, [_vp, _vp, _i32, _vp, _vp]),
    ("sph_mlp_train_step", C.c_int, [_vp, _vp, _i64, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    ("sph_mlp_targets", C.c_int, [_vp, _i32, C.c_double, _vp, _vp, _vp]),
    ("sph_mlp_train_step_noalloc", C.c_int, [_vp, _vp, _i64, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    ("sph_mlp_train_epoch", C.c_int, [_vp, _vp, _i64, _vp, _vp, _vp, _i32, _i32, _i64, _vp, _vp, _vp, _vp]),
    ("sph_mlp_apply", C.c_int, [_vp, C.POINTER(sph_domain), C.POINTER(sph_relax_params), _i32, _vp, _vp]),
]
_OPTIONAL_SIGS = []

MLP_NPARAMS = 29827
MLP_FEAT_STRIDE = 128


class sph_adamw_params(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("weight_decay", C.c_double)]


def adamw_params(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.01) -> sph_adamw_params:
    p = sph_adamw_params()
    p.lr, p.beta1, p.beta2, p.eps, p.weight_decay = lr, beta1, beta2, eps, weight_decay
    return p


def lib():
    """Load libsph.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_2405_05155_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS + _OPTIONAL_SIGS:
            if not hasattr(L, name):
                continue
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(t, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


@dataclass
class Domain:
    dim: int
    h: float
    kappa: float
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    periodic: tuple = (1, 1, 1)
    kernel: int = WENDLAND

    def to_c(self) -> sph_domain:
        d = sph_domain()
        d.dim, d.h, d.kappa, d.kernel = int(self.dim), float(self.h), float(self.kappa), int(self.kernel)
        for a in range(3):
            d.periodic[a] = int(self.periodic[a]) if a < self.dim and a < len(self.periodic) else 0
            d.lo[a] = float(self.lo[a]) if a < len(self.lo) else 0.0
            d.hi[a] = float(self.hi[a]) if a < len(self.hi) else 1.0
        return d


def euler_params(c, rho0, rho_ref, eta=15.0, mu=0.0, dt=0.0) -> sph_euler_params:
    p = sph_euler_params()
    p.c, p.rho0, p.rho_ref, p.eta, p.mu, p.dt = c, rho0, rho_ref, eta, mu, dt
    return p


def hllc_params(gamma=1.4, eta=1.0, dt=0.0) -> sph_hllc_params:
    p = sph_hllc_params()
    p.gamma, p.eta, p.dt = gamma, eta, dt
    return p


def tlsph_params(rho0, E, nu, dt=0.0, model=0) -> sph_tlsph_params:
    p = sph_tlsph_params()
    p.rho0, p.E, p.nu, p.dt, p.model = rho0, E, nu, dt, model
    return p


def relax_params(center, radius, p0=1.0, rho=1.0, kappa=0.1, damping=0.9, max_move=0.1,
                 kernel=LAGUERRE_GAUSS) -> sph_relax_params:
    """kernel: LAGUERRE_GAUSS (Eq. 8) or WENDLAND (Eq. 6, support 2h)."""
    p = sph_relax_params()
    p.p0, p.rho, p.radius, p.kappa, p.damping, p.max_move = p0, rho, radius, kappa, damping, max_move
    p.kernel = kernel
    for a in range(3):
        p.center[a] = center[a]
    return p


class Context:
    """One sph_ctx: a bound particle configuration on one device and stream."""

    def __init__(self, dim: int, stream=None):
        L = lib()
        self.dim = dim
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = C.c_void_p()
        rc = L.sph_ctx_create(C.byref(h), dim, C.c_void_p(stream.cuda_stream))
        if rc != SPH_OK:
            raise SphError(rc, "sph_ctx_create failed")
        self._h = h
        self.n = 0
        self.nnz = 0

    @property
    def stream(self):
        """The torch stream the context enqueues its kernels on."""
        return self._stream

    def close(self):
        if getattr(self, "_h", None):
            lib().sph_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != SPH_OK:
            msg = lib().sph_last_error(self._h)
            raise SphError(rc, msg.decode() if msg else "")

    def _dev(self):
        return torch.device("cuda", torch.cuda.current_device())

    def euler_path(self) -> int:
        """Pair-loop variant of the last Eulerian call (PATH_NONE, PATH_GENERIC, PATH_RECORDS, PATH_WINDOWS)."""
        return int(lib().sph_euler_path(self._h))

    def tlsph_path(self) -> int:
        """Variant of the stress-divergence loop in the last total-Lagrangian call (PATH_GENERIC, PATH_WINDOWS)."""
        return int(lib().sph_tlsph_path(self._h))

    # ------------------------------------------------------------ neighbours
    def build_cells(self, domain: Domain, pos: torch.Tensor):
        n = pos.shape[-1] if pos.numel() else 0
        self._check(lib().sph_build_cells(self._h, C.byref(domain.to_c()), n,
                                          _ptr(pos, torch.float32, self.dim * n, "pos")))
        self.n = n
        self.domain = domain
        cnt = C.c_int64(0)  # the pair count (no export: row_ptr NULL only reports it)
        lib().sph_neighbors(self._h, None, None, 0, C.byref(cnt))
        self.nnz = int(cnt.value)
        return self

    def neighbors(self):
        cnt = C.c_int64(0)
        rc = lib().sph_neighbors(self._h, None, None, 0, C.byref(cnt))
        if rc not in (SPH_OK, SPH_ERR_ARG, SPH_ERR_CAPACITY):
            self._check(rc)
        nnz = int(cnt.value)
        row_ptr = torch.empty(self.n + 1, dtype=torch.int64, device=self._dev())
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=self._dev())
        self._check(lib().sph_neighbors(self._h, _ptr(row_ptr), _ptr(col), nnz, C.byref(cnt)))
        self.nnz = nnz
        return row_ptr, col[:nnz]

    # ------------------------------------------------------------ sums
    def kernel_sum(self, vol):
        out = torch.empty(self.n, dtype=torch.float32, device=self._dev())
        self._check(lib().sph_kernel_sum(self._h, _ptr(vol, torch.float32, self.n, "vol"), _ptr(out)))
        return out

    def correction_B(self, vol, want_fp64=False, count=True):
        d = self.dim
        B = torch.empty((self.n, d, d), dtype=torch.float32, device=self._dev())
        B64 = torch.empty((self.n, d, d), dtype=torch.float64, device=self._dev()) if want_fp64 else None
        nd = C.c_int32(0)
        self._check(lib().sph_correction_B(self._h, _ptr(vol, torch.float32, self.n, "vol"), _ptr(B), _ptr(B64),
                                           C.byref(nd) if count else None))
        return B, B64, (int(nd.value) if count else None)

    def set_correction(self, vol, B):
        self._check(lib().sph_set_correction(self._h, _ptr(vol, torch.float32, self.n, "vol"),
                                             _ptr(B, torch.float32, self.n * self.dim * self.dim, "B")))

    def gradient(self, f):
        g = torch.empty((self.dim, self.n), dtype=torch.float32, device=self._dev())
        self._check(lib().sph_gradient(self._h, _ptr(f, torch.float32, self.n, "f"), _ptr(g)))
        return g

    # ------------------------------------------------------------ Eulerian
    def euler_rhs(self, prm, drho, mom):
        dr = torch.empty(self.n, dtype=torch.float32, device=self._dev())
        dm = torch.empty((self.dim, self.n), dtype=torch.float32, device=self._dev())
        self._check(lib().sph_euler_rhs(self._h, C.byref(prm), _ptr(drho, torch.float32, self.n, "drho"),
                                        _ptr(mom, torch.float32, self.dim * self.n, "mom"), _ptr(dr), _ptr(dm)))
        return dr, dm

    def euler_step(self, prm, drho, mom, nsteps):
        self._check(lib().sph_euler_step(self._h, C.byref(prm), _ptr(drho, torch.float32, self.n, "drho"),
                                         _ptr(mom, torch.float32, self.dim * self.n, "mom"), int(nsteps)))

    def hllc_rhs(self, prm, rho, mom, E):
        dr = torch.empty(self.n, dtype=torch.float32, device=self._dev())
        dm = torch.empty((self.dim, self.n), dtype=torch.float32, device=self._dev())
        de = torch.empty(self.n, dtype=torch.float32, device=self._dev())
        self._check(lib().sph_hllc_rhs(self._h, C.byref(prm), _ptr(rho, torch.float32, self.n, "rho"),
                                       _ptr(mom, torch.float32, self.dim * self.n, "mom"),
                                       _ptr(E, torch.float32, self.n, "E"), _ptr(dr), _ptr(dm), _ptr(de)))
        return dr, dm, de

    def hllc_step(self, prm, rho, mom, E, nsteps):
        self._check(lib().sph_hllc_step(self._h, C.byref(prm), _ptr(rho, torch.float32, self.n, "rho"),
                                        _ptr(mom, torch.float32, self.dim * self.n, "mom"),
                                        _ptr(E, torch.float32, self.n, "E"), int(nsteps)))

    # ------------------------------------------------------------ total Lagrangian
    def tlsph_rhs(self, prm, vel, F, fixed=None):
        dF = torch.empty((self.n, 3, 3), dtype=torch.float32, device=self._dev())
        acc = torch.empty((3, self.n), dtype=torch.float32, device=self._dev())
        self._check(lib().sph_tlsph_rhs(self._h, C.byref(prm), _ptr(vel, torch.float32, 3 * self.n, "vel"),
                                        _ptr(F, torch.float32, 9 * self.n, "F"),
                                        _ptr(fixed, torch.int32, self.n, "fixed"), _ptr(dF), _ptr(acc)))
        return dF, acc

    def tlsph_step(self, prm, fixed, pos, vel, F, acc, nsteps):
        self._check(lib().sph_tlsph_step(self._h, C.byref(prm), _ptr(fixed, torch.int32, self.n, "fixed"),
                                         _ptr(pos, torch.float32, 3 * self.n, "pos"),
                                         _ptr(vel, torch.float32, 3 * self.n, "vel"),
                                         _ptr(F, torch.float32, 9 * self.n, "F"),
                                         _ptr(acc, torch.float32, 3 * self.n, "acc"), int(nsteps)))


    # ------------------------------------------------------------ relaxation
    def relax_step(self, domain: Domain, prm, pos, u, vol, niter, residue=None):
        """niter iterations in place (pos, u: [dim][n]); residue: optional
        device float64 tensor [1]."""
        d = self.dim
        n = pos.shape[-1] if pos.numel() else 0
        self._check(lib().sph_relax_step(self._h, C.byref(domain.to_c()), C.byref(prm), n,
                                         _ptr(pos, torch.float32, d * n, "pos"), _ptr(u, torch.float32, d * n, "u"),
                                         _ptr(vol, torch.float32, n, "vol"), _ptr(residue, torch.float64, 1, "residue"),
                                         int(niter)))

    def relax_residue(self, domain: Domain, prm, pos, vol, want_g=True):
        d = self.dim
        n = pos.shape[-1] if pos.numel() else 0
        res = torch.zeros(1, dtype=torch.float64, device=self._dev())
        g = torch.empty((d, n), dtype=torch.float32, device=self._dev()) if want_g else None
        self._check(lib().sph_relax_residue(self._h, C.byref(domain.to_c()), C.byref(prm), n,
                                            _ptr(pos, torch.float32, d * n, "pos"), _ptr(vol, torch.float32, n, "vol"),
                                            _ptr(g), _ptr(res)))
        return res, g


    # ------------------------------------------------------------ learned warm start
    def mlp_features(self, domain: Domain, prm, pos):
        """BF16 feature rows (int16 bit patterns) [n][MLP_FEAT_STRIDE]."""
        n = pos.shape[-1] if pos.numel() else 0
        feat = torch.empty((n, MLP_FEAT_STRIDE), dtype=torch.int16, device=self._dev())
        self._check(lib().sph_mlp_features(self._h, C.byref(domain.to_c()), C.byref(prm), n,
                                           _ptr(pos, torch.float32, 3 * n, "pos"), _ptr(feat)))
        return feat

    def mlp_forward(self, params, feat):
        n = feat.shape[0]
        out = torch.empty((n, 3), dtype=torch.float32, device=self._dev())
        self._check(lib().sph_mlp_forward(self._h, _ptr(params, torch.float32, MLP_NPARAMS, "params"), n,
                                          _ptr(feat, torch.int16, n * MLP_FEAT_STRIDE, "feat"), _ptr(out)))
        return out

    def mlp_train_step(self, adam, step, params, m, v, feat, target, want_loss=True, want_grad=False):
        B = feat.shape[0]
        loss = torch.zeros(1, dtype=torch.float32, device=self._dev()) if want_loss else None
        grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=self._dev()) if want_grad else None
        self._check(lib().sph_mlp_train_step(self._h, C.byref(adam), int(step),
                                             _ptr(params, torch.float32, MLP_NPARAMS, "params"),
                                             _ptr(m, torch.float32, MLP_NPARAMS, "m"),
                                             _ptr(v, torch.float32, MLP_NPARAMS, "v"), B,
                                             _ptr(feat, torch.int16, B * MLP_FEAT_STRIDE, "feat"),
                                             _ptr(target, torch.float32, B * 3, "target"), _ptr(loss), _ptr(grad)))
        return loss, grad

    def mlp_targets(self, pos_from, pos_to, h):
        """(pos_to - pos_from) / h as [n][3] (positions [3][n])."""
        n = pos_from.shape[-1] if pos_from.numel() else 0
        out = torch.empty((n, 3), dtype=torch.float32, device=self._dev())
        self._check(lib().sph_mlp_targets(self._h, n, float(h), _ptr(pos_from, torch.float32, 3 * n, "from"),
                                          _ptr(pos_to, torch.float32, 3 * n, "to"), _ptr(out)))
        return out

    def mlp_train_step_noalloc(self, adam, step, params, m, v, feat, target, loss=None, grad=None):
        """sph_mlp_train_step_noalloc: the caller passes every buffer (loss:
        device FP32 [1], grad: device FP32 [MLP_NPARAMS], both optional);
        neither this method nor the library allocates."""
        B = feat.shape[0]
        self._check(lib().sph_mlp_train_step_noalloc(self._h, C.byref(adam), int(step),
                                                     _ptr(params, torch.float32, MLP_NPARAMS, "params"),
                                                     _ptr(m, torch.float32, MLP_NPARAMS, "m"),
                                                     _ptr(v, torch.float32, MLP_NPARAMS, "v"), B,
                                                     _ptr(feat, torch.int16, B * MLP_FEAT_STRIDE, "feat"),
                                                     _ptr(target, torch.float32, B * 3, "target"),
                                                     _ptr(loss, torch.float32, 1, "loss"),
                                                     _ptr(grad, torch.float32, MLP_NPARAMS, "grad")))

    def mlp_train_epoch(self, adam, step0, params, m, v, rows, feat, target, batch, want_losses=True):
        """Steps step0 .. step0 + nbatch - 1 over the batches rows[b*batch:(b+1)*batch]
        (int64 row indices into feat/target, nbatch = len(rows) // batch)."""
        nbatch = rows.numel() // batch
        rows = rows[:nbatch * batch]
        nrows = feat.shape[0]
        losses = torch.zeros(nbatch, dtype=torch.float32, device=self._dev()) if want_losses else None
        self._check(lib().sph_mlp_train_epoch(self._h, C.byref(adam), int(step0),
                                              _ptr(params, torch.float32, MLP_NPARAMS, "params"),
                                              _ptr(m, torch.float32, MLP_NPARAMS, "m"),
                                              _ptr(v, torch.float32, MLP_NPARAMS, "v"), int(batch), int(nbatch),
                                              int(nrows), _ptr(rows, torch.int64, nbatch * batch, "rows"),
                                              _ptr(feat, torch.int16, nrows * MLP_FEAT_STRIDE, "feat"),
                                              _ptr(target, torch.float32, nrows * 3, "target"), _ptr(losses)))
        return losses

    def mlp_apply(self, domain: Domain, prm, pos, params):
        n = pos.shape[-1] if pos.numel() else 0
        self._check(lib().sph_mlp_apply(self._h, C.byref(domain.to_c()), C.byref(prm), n,
                                        _ptr(pos, torch.float32, 3 * n, "pos"),
                                        _ptr(params, torch.float32, MLP_NPARAMS, "params")))


# Module-level functions named as the C calls (same argument order, with the
# Context in place of the sph_ctx pointer).
def sph_euler_path(ctx: Context):
    return ctx.euler_path()


def sph_tlsph_path(ctx: Context):
    return ctx.tlsph_path()


def sph_build_cells(ctx: Context, domain: Domain, pos):
    return ctx.build_cells(domain, pos)


def sph_neighbors(ctx: Context):
    return ctx.neighbors()


def sph_kernel_sum(ctx: Context, vol):
    return ctx.kernel_sum(vol)


def sph_correction_B(ctx: Context, vol, want_fp64=False):
    return ctx.correction_B(vol, want_fp64)


def sph_set_correction(ctx: Context, vol, B):
    return ctx.set_correction(vol, B)


def sph_gradient(ctx: Context, f):
    return ctx.gradient(f)


def sph_euler_rhs(ctx: Context, prm, drho, mom):
    return ctx.euler_rhs(prm, drho, mom)


def sph_euler_step(ctx: Context, prm, drho, mom, nsteps):
    return ctx.euler_step(prm, drho, mom, nsteps)


def sph_hllc_rhs(ctx: Context, prm, rho, mom, E):
    return ctx.hllc_rhs(prm, rho, mom, E)


def sph_hllc_step(ctx: Context, prm, rho, mom, E, nsteps):
    return ctx.hllc_step(prm, rho, mom, E, nsteps)


def sph_tlsph_rhs(ctx: Context, prm, vel, F, fixed=None):
    return ctx.tlsph_rhs(prm, vel, F, fixed)


def sph_tlsph_step(ctx: Context, prm, fixed, pos, vel, F, acc, nsteps):
    return ctx.tlsph_step(prm, fixed, pos, vel, F, acc, nsteps)


def sph_relax_step(ctx: Context, domain, prm, pos, u, vol, niter, residue=None):
    return ctx.relax_step(domain, prm, pos, u, vol, niter, residue)


def sph_relax_residue(ctx: Context, domain, prm, pos, vol, want_g=True):
    return ctx.relax_residue(domain, prm, pos, vol, want_g)


def sph_mlp_features(ctx: Context, domain, prm, pos):
    return ctx.mlp_features(domain, prm, pos)


def sph_mlp_forward(ctx: Context, params, feat):
    return ctx.mlp_forward(params, feat)


def sph_mlp_train_step(ctx: Context, adam, step, params, m, v, feat, target, want_loss=True, want_grad=False):
    return ctx.mlp_train_step(adam, step, params, m, v, feat, target, want_loss, want_grad)


def sph_mlp_targets(ctx: Context, pos_from, pos_to, h):
    return ctx.mlp_targets(pos_from, pos_to, h)


def sph_mlp_train_step_noalloc(ctx: Context, adam, step, params, m, v, feat, target, loss=None, grad=None):
    return ctx.mlp_train_step_noalloc(adam, step, params, m, v, feat, target, loss, grad)


def sph_mlp_train_epoch(ctx: Context, adam, step0, params, m, v, rows, feat, target, batch, want_losses=True):
    return ctx.mlp_train_epoch(adam, step0, params, m, v, rows, feat, target, batch, want_losses)


def sph_mlp_apply(ctx: Context, domain, prm, pos, params):
    return ctx.mlp_apply(domain, prm, pos, params)
