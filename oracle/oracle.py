"""ctypes wrapper of the FP64 CPU oracle (``pft_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
module and this module never imports the GPU library.

Every array is a C-contiguous numpy ``complex128`` array of shape (nx, ny, nz)
(z fastest); propagator stores have shape (K+1, nx, ny, nz).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pft_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RQM4 = 0
SPLIT2 = 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over lines)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("ns", ctypes.c_int32), ("f", ctypes.c_double), ("chiN", ctypes.c_double),
                ("C", ctypes.c_double), ("scheme", ctypes.c_int32), ("naive_dft", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 3)]


@dataclass
class Params:
    """Diblock-melt model and discretisation (lengths in R_g)."""
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    ns: int
    f: float
    chiN: float
    C: float = 1.0
    scheme: int = RQM4
    naive_dft: bool = False
    bc: tuple = (0, 0, 0)    # per axis: 0 periodic, 1 reflecting (Neumann), 2 absorbing (Dirichlet)

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def M(self):
        return self.nx * self.ny * self.nz

    @property
    def volume(self):
        return self.lx * self.ly * self.lz

    def _c(self):
        if not (0.0 < self.f < 1.0):
            raise ValueError("f must lie in (0, 1)")
        if self.ns < 2:
            raise ValueError("ns must be >= 2")
        return _Params(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz, self.ns,
                       self.f, self.chiN, self.C, self.scheme, int(self.naive_dft),
                       (ctypes.c_int32 * 3)(*self.bc))


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER(_Params)
        vp, i32, f64, u64, i64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_uint64, ctypes.c_int64)
        sig = {
            "or_set_threads": (None, [ctypes.c_int]),
            "or_get_threads": (ctypes.c_int, []),
            "or_contour": (ctypes.c_int, [i32, f64, vp, vp, vp]),
            "or_trapezoid": (None, [ctypes.c_int, vp, vp, vp, vp]),
            "or_mode": (i32, [i32, i32]),
            "or_dft3_naive": (None, [vp, vp, i32, i32, i32, i32]),
            "or_fft3": (None, [vp, i32, i32, i32, i32]),
            "or_ksq_grid": (None, [P, vp]),
            "or_diffuse": (None, [P, f64, vp]),
            "or_step": (None, [P, i32, f64, vp, vp, vp, vp]),
            "or_block_fields": (None, [P, vp, vp, vp, vp]),
            "or_propagate": (ctypes.c_int, [P, vp, vp, vp, vp]),
            "or_densities": (None, [P, vp, vp, vp, vp, vp, vp]),
            "or_hamiltonian": (None, [P, vp, vp, f64, f64, vp, vp]),
            "or_forces": (None, [P, vp, vp, vp, vp, vp]),
            "or_philox4x64_10": (None, [vp, vp, vp]),
            "or_gaussian": (None, [u64, u64, u64, i32, i64, vp]),
            "or_em_update": (None, [P, vp, vp, vp, vp, f64, f64, f64, i32, u64, u64, u64]),
            "or_adjoint": (ctypes.c_int, [P, vp, vp, vp, vp, vp]),
            "or_edwards_propagate": (ctypes.c_int, [P, vp, vp]),
            "or_edwards_densities": (None, [P, vp, vp, vp]),
            "or_edwards_hamiltonian": (None, [P, f64, vp, f64, f64, vp, vp]),
            "or_edwards_force": (None, [P, f64, vp, vp, vp]),
            "or_edwards_em_update": (None, [P, f64, vp, vp, f64, f64, i32, u64, u64, u64]),
            "or_edwards_evaluate": (ctypes.c_int, [P, f64, vp, vp, vp, vp, vp]),
            "or_debye": (f64, [f64]),
            "or_sis_update": (None, [P, vp, vp, vp, vp, f64, f64, f64, i32, u64, u64, u64]),
            "or_edwards_sis_update": (None, [P, f64, vp, vp, f64, f64, i32, u64, u64, u64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _cfield(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def contour(ns: int, f: float):
    """Step lengths h[K], blocks blk[K] (0 = A, 1 = B) and the junction node J."""
    h = np.zeros(ns + 2)
    blk = np.zeros(ns + 2, dtype=np.int32)
    J = np.zeros(1, dtype=np.int32)
    K = lib().or_contour(ns, f, _ptr(h), _ptr(blk), _ptr(J))
    return h[:K].copy(), blk[:K].copy(), int(J[0])


def trapezoid(h: np.ndarray, blk: np.ndarray):
    K = len(h)
    h = np.ascontiguousarray(h, dtype=np.float64)
    blk = np.ascontiguousarray(blk, dtype=np.int32)
    ta, tb = np.zeros(K + 1), np.zeros(K + 1)
    lib().or_trapezoid(K, _ptr(h), _ptr(blk), _ptr(ta), _ptr(tb))
    return ta, tb


def mode(j: int, n: int) -> int:
    return int(lib().or_mode(j, n))


def fft3(a: np.ndarray, sign: int = -1) -> np.ndarray:
    out = np.array(a, dtype=np.complex128, order="C", copy=True)
    lib().or_fft3(_ptr(out), *out.shape, sign)
    return out


def dft3_naive(a: np.ndarray, sign: int = -1) -> np.ndarray:
    a = _cfield(a)
    out = np.empty_like(a)
    lib().or_dft3_naive(_ptr(a), _ptr(out), *a.shape, sign)
    return out


def ksq_grid(p: Params) -> np.ndarray:
    out = np.empty(p.shape)
    lib().or_ksq_grid(ctypes.byref(p._c()), _ptr(out))
    return out


def diffuse(p: Params, h: float, u: np.ndarray) -> np.ndarray:
    out = np.array(u, dtype=np.complex128, order="C", copy=True)
    lib().or_diffuse(ctypes.byref(p._c()), h, _ptr(out))
    return out


def step(p: Params, h: float, w: np.ndarray, q: np.ndarray, scheme=None) -> np.ndarray:
    """One contour step T_h(q; w) of the chosen scheme."""
    w, q = _cfield(w, p.shape), _cfield(q, p.shape)
    out = np.empty_like(q)
    work = np.empty((2,) + p.shape, dtype=np.complex128)
    lib().or_step(ctypes.byref(p._c()), p.scheme if scheme is None else scheme, h,
                  _ptr(w), _ptr(q), _ptr(out), _ptr(work))
    return out


def block_fields(p: Params, wp, wm):
    wp, wm = _cfield(wp, p.shape), _cfield(wm, p.shape)
    wA, wB = np.empty_like(wp), np.empty_like(wp)
    lib().or_block_fields(ctypes.byref(p._c()), _ptr(wp), _ptr(wm), _ptr(wA), _ptr(wB))
    return wA, wB


def propagate(p: Params, wp, wm, forward: bool = True, backward: bool = True):
    """Stored propagators q[K+1] and q-dagger[K+1] (each may be skipped)."""
    wp, wm = _cfield(wp, p.shape), _cfield(wm, p.shape)
    h, _, _ = contour(p.ns, p.f)
    K = len(h)
    qs = np.empty((K + 1,) + p.shape, dtype=np.complex128) if forward else None
    qds = np.empty((K + 1,) + p.shape, dtype=np.complex128) if backward else None
    lib().or_propagate(ctypes.byref(p._c()), _ptr(wp), _ptr(wm),
                       _ptr(qs) if forward else None, _ptr(qds) if backward else None)
    return qs, qds


def densities(p: Params, qs, qds):
    """(phi_A, phi_B, Q, Qnode) from stored propagators."""
    qs, qds = _cfield(qs), _cfield(qds)
    K = qs.shape[0] - 1
    phiA, phiB = np.empty(p.shape, np.complex128), np.empty(p.shape, np.complex128)
    Q = np.zeros(1, np.complex128)
    Qn = np.zeros(K + 1, np.complex128)
    lib().or_densities(ctypes.byref(p._c()), _ptr(qs), _ptr(qds), _ptr(phiA), _ptr(phiB),
                       _ptr(Q), _ptr(Qn))
    return phiA, phiB, complex(Q[0]), Qn


def hamiltonian(p: Params, wp, wm, Q: complex):
    """(H, h = H / (C V)) of Eq. (3)."""
    wp, wm = _cfield(wp, p.shape), _cfield(wm, p.shape)
    H = np.zeros(1, np.complex128)
    hi = np.zeros(1, np.complex128)
    lib().or_hamiltonian(ctypes.byref(p._c()), _ptr(wp), _ptr(wm),
                         Q.real, Q.imag, _ptr(H), _ptr(hi))
    return complex(H[0]), complex(hi[0])


def forces(p: Params, wm, phiA, phiB):
    wm, phiA, phiB = (_cfield(a, p.shape) for a in (wm, phiA, phiB))
    Fp, Fm = np.empty_like(wm), np.empty_like(wm)
    lib().or_forces(ctypes.byref(p._c()), _ptr(wm), _ptr(phiA), _ptr(phiB), _ptr(Fp), _ptr(Fm))
    return Fp, Fm


def philox4x64_10(counter, key) -> np.ndarray:
    ctr = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_ptr(ctr), _ptr(k), _ptr(out))
    return out


def gaussian(seed: int, replica: int, step_: int, field: int, M: int) -> np.ndarray:
    xi = np.zeros(M)
    lib().or_gaussian(seed, replica, step_, field, M, _ptr(xi))
    return xi


def em_update(p: Params, wp, wm, phiA, phiB, dt, lam_p=1.0, lam_m=1.0, noise=False,
              seed=0, replica=0, step_=0):
    """Return the updated (w_+, w_-) after one explicit Euler-Maruyama step."""
    wp = np.array(wp, dtype=np.complex128, order="C", copy=True)
    wm = np.array(wm, dtype=np.complex128, order="C", copy=True)
    phiA, phiB = _cfield(phiA, p.shape), _cfield(phiB, p.shape)
    lib().or_em_update(ctypes.byref(p._c()), _ptr(wp), _ptr(wm), _ptr(phiA), _ptr(phiB),
                       dt, lam_p, lam_m, int(bool(noise)), seed, replica, step_)
    return wp, wm


def evaluate(p: Params, wp, wm):
    """Full evaluation: dict with phiA, phiB, Q, Qnode, H, h, K."""
    qs, qds = propagate(p, wp, wm)
    phiA, phiB, Q, Qn = densities(p, qs, qds)
    H, hi = hamiltonian(p, wp, wm, Q)
    return {"phiA": phiA, "phiB": phiB, "Q": Q, "Qnode": Qn, "H": H, "h": hi,
            "K": qs.shape[0] - 1}


def adjoint(p: Params, wp, wm):
    """(dH/dw_+, dH/dw_-, dH/dL[3]) by reverse mode through the split steps.
    With walls the steps diffuse through the walled operator (cosine / sine
    modes, k = pi m / L along a walled axis), and dH/dL_a takes the axis
    Laplacian in that axis's own mode basis."""
    wp, wm = _cfield(wp, p.shape), _cfield(wm, p.shape)
    gp, gm = np.empty_like(wp), np.empty_like(wp)
    dL = np.zeros(3, np.complex128)
    lib().or_adjoint(ctypes.byref(p._c()), _ptr(wp), _ptr(wm), _ptr(gp), _ptr(gm), _ptr(dL))
    return gp, gm, dL


# ------------------------------------------------------------- Edwards model --

def edwards_propagate(p: Params, omega):
    """q[ns+1] in the field i*omega (one species, no junction)."""
    omega = _cfield(omega, p.shape)
    qs = np.empty((p.ns + 1,) + p.shape, dtype=np.complex128)
    lib().or_edwards_propagate(ctypes.byref(p._c()), _ptr(omega), _ptr(qs))
    return qs


def edwards_densities(p: Params, qs):
    """(phi, Q) with q-dagger = q."""
    qs = _cfield(qs)
    phi = np.empty(p.shape, np.complex128)
    Q = np.zeros(1, np.complex128)
    lib().or_edwards_densities(ctypes.byref(p._c()), _ptr(qs), _ptr(phi), _ptr(Q))
    return phi, complex(Q[0])


def edwards_hamiltonian(p: Params, B: float, omega, Q: complex):
    omega = _cfield(omega, p.shape)
    H = np.zeros(1, np.complex128)
    hi = np.zeros(1, np.complex128)
    lib().or_edwards_hamiltonian(ctypes.byref(p._c()), B, _ptr(omega), Q.real, Q.imag, _ptr(H), _ptr(hi))
    return complex(H[0]), complex(hi[0])


def edwards_force(p: Params, B: float, omega, phi):
    omega, phi = _cfield(omega, p.shape), _cfield(phi, p.shape)
    F = np.empty_like(omega)
    lib().or_edwards_force(ctypes.byref(p._c()), B, _ptr(omega), _ptr(phi), _ptr(F))
    return F


def edwards_em_update(p: Params, B: float, omega, phi, dt, lam=1.0, noise=False, seed=0, replica=0, step_=0):
    omega = np.array(omega, dtype=np.complex128, order="C", copy=True)
    phi = _cfield(phi, p.shape)
    lib().or_edwards_em_update(ctypes.byref(p._c()), B, _ptr(omega), _ptr(phi), dt, lam, int(bool(noise)),
                               seed, replica, step_)
    return omega


def edwards_evaluate(p: Params, B: float, omega):
    """dict with phi, Q, H, h, K."""
    omega = _cfield(omega, p.shape)
    phi = np.empty(p.shape, np.complex128)
    Q = np.zeros(1, np.complex128)
    H = np.zeros(1, np.complex128)
    hi = np.zeros(1, np.complex128)
    K = lib().or_edwards_evaluate(ctypes.byref(p._c()), B, _ptr(omega), _ptr(phi), _ptr(Q), _ptr(H), _ptr(hi))
    return {"phi": phi, "Q": complex(Q[0]), "H": complex(H[0]), "h": complex(hi[0]), "K": K}


# ------------------------------------------------------ semi-implicit step --

def debye(x: float) -> float:
    return lib().or_debye(float(x))


def _sis_walls_ok(p: Params):
    if any(b == 2 for b in p.bc):
        raise ValueError("the semi-implicit step has no diagonal linear response between absorbing walls")


def sis_update(p: Params, wp, wm, phiA, phiB, dt, lam_p=1.0, lam_m=1.0, noise=False, seed=0, replica=0, step_=0):
    """Return the updated (w_+, w_-) after one semi-implicit step (Eq. (10));
    periodic axes filter in the Fourier basis, reflecting ones in the cosine basis."""
    _sis_walls_ok(p)
    wp = np.array(wp, dtype=np.complex128, order="C", copy=True)
    wm = np.array(wm, dtype=np.complex128, order="C", copy=True)
    phiA, phiB = _cfield(phiA, p.shape), _cfield(phiB, p.shape)
    lib().or_sis_update(ctypes.byref(p._c()), _ptr(wp), _ptr(wm), _ptr(phiA), _ptr(phiB),
                        dt, lam_p, lam_m, int(bool(noise)), seed, replica, step_)
    return wp, wm


def edwards_sis_update(p: Params, B: float, omega, phi, dt, lam=1.0, noise=False, seed=0, replica=0, step_=0):
    _sis_walls_ok(p)
    omega = np.array(omega, dtype=np.complex128, order="C", copy=True)
    phi = _cfield(phi, p.shape)
    lib().or_edwards_sis_update(ctypes.byref(p._c()), B, _ptr(omega), _ptr(phi), dt, lam, int(bool(noise)),
                                seed, replica, step_)
    return omega
