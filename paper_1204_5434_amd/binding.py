"""Thin ctypes binding of the C ABI in ``include/pft.h`` (argument marshalling only).

Every step of the path runs in the HIP kernels of ``libpft.so``; this module
checks tensor dtype, device, shape and contiguity, then passes raw device
pointers and the current HIP stream.  There is no CPU fallback: if the library
is not built, or no GPU is present, calls fail loudly.

Tensors are torch ``complex128`` on the GPU with shape (nx, ny, nz); scalars
(Q, H) are complex128 tensors of shape (1,) on the GPU.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, replace

import torch  # loaded first so the library binds to torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpft.so")

PFT_OK, PFT_E_INVALID, PFT_E_UNSUPPORTED, PFT_E_NOMEM, PFT_E_DEVICE, PFT_E_NONFINITE, PFT_E_STATE = range(7)
PFT_C128, PFT_C64 = 0, 1
PFT_RQM4, PFT_SPLIT2 = 0, 1
PFT_DIBLOCK, PFT_EDWARDS = 0, 1
PFT_STORE_BOTH, PFT_STORE_Q, PFT_STORE_HOST = 0, 1, 2
PFT_PERIODIC, PFT_REFLECTING, PFT_ABSORBING = 0, 1, 2

SUPPORTED_AXES = (8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128, 192, 256)

EXPORTS = ("pft_create", "pft_destroy", "pft_last_error", "pft_status_string", "pft_contour_plan",
           "pft_num_steps", "pft_propagate", "pft_densities", "pft_hamiltonian", "pft_cl_step",
           "pft_node_q", "pft_get_slice", "pft_apply_step", "pft_diffuse", "pft_debug_kgrid",
           "pft_status_flags", "pft_noise_words", "pft_noise_normals", "pft_profile_begin",
           "pft_profile_end", "pft_copy_probe", "pft_adjoint", "pft_batch_create", "pft_batch_destroy",
           "pft_batch_last_error", "pft_batch_evaluate", "pft_batch_cl_steps", "pft_batch_sync",
           "pft_autotune", "pft_tune_save", "pft_tune_load", "pft_set_variant", "pft_set_concurrent_sweeps",
           "pft_set_fused_planes", "pft_fused_planes", "pft_evaluate_graph", "pft_set_box",
           "pft_cl_step_static")

# Kernel variants per axis length (variant 0 always exists), at most MAX_VARIANTS.
MAX_VARIANTS = 4
VARIANTS = {8: (0,), 12: (0,), 16: (0, 1, 2), 20: (0,), 24: (0, 1), 32: (0, 1, 2), 40: (0, 1), 48: (0, 1),
            64: (0, 1, 2, 3), 80: (0,), 96: (0, 1), 128: (0, 1, 2), 192: (0,), 256: (0, 1)}

KERNEL_KINDS = ("tables", "zpass", "ypass", "xpass", "density", "reduce", "yzpass")

# Square yz-plane sides with a fused yz pass, per precision (complex double, complex float).
FUSED_PLANES = {0: (8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96), 1: (8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128)}


class PftError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


class pft_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("ns", ctypes.c_int32), ("f", ctypes.c_double), ("chiN", ctypes.c_double),
                ("C", ctypes.c_double), ("precision", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("model", ctypes.c_int32), ("B", ctypes.c_double), ("storage", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 3)]


class pft_step(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("lambda_plus", ctypes.c_double),
                ("lambda_minus", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint64), ("step", ctypes.c_uint64), ("noise", ctypes.c_int32),
                ("update", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libpft.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_double)
        P = ctypes.POINTER
        sig = {
            "pft_create": (i32, [P(pft_params), vp, P(vp)]),
            "pft_destroy": (None, [vp]),
            "pft_last_error": (ctypes.c_char_p, [vp]),
            "pft_status_string": (ctypes.c_char_p, [i32]),
            "pft_contour_plan": (i32, [i32, f64, vp, vp, vp]),
            "pft_num_steps": (i32, [vp]),
            "pft_propagate": (i32, [vp, vp, vp]),
            "pft_densities": (i32, [vp, vp, vp, vp]),
            "pft_evaluate_graph": (i32, [vp, vp, vp, vp, vp, vp, i32]),
            "pft_hamiltonian": (i32, [vp, vp, vp, vp, vp]),
            "pft_set_box": (i32, [vp, f64, f64, f64]),
            "pft_cl_step": (i32, [vp, vp, vp, P(pft_step), vp, vp, vp, vp]),
            "pft_cl_step_static": (i32, [vp, vp, vp, P(pft_step), vp, vp, vp, vp]),
            "pft_node_q": (i32, [vp, vp]),
            "pft_get_slice": (i32, [vp, i32, i32, vp]),
            "pft_apply_step": (i32, [vp, i32, vp, vp]),
            "pft_diffuse": (i32, [vp, vp, f64]),
            "pft_debug_kgrid": (i32, [vp, vp]),
            "pft_status_flags": (i32, [vp, P(ctypes.c_uint32)]),
            "pft_noise_words": (i32, [u64, u64, u64, i32, i64, vp, vp]),
            "pft_noise_normals": (i32, [u64, u64, u64, i32, i64, vp, vp]),
            "pft_profile_begin": (i32, [vp]),
            "pft_profile_end": (i32, [vp, vp, vp, vp]),
            "pft_copy_probe": (i32, [vp, vp, i64, vp]),
            "pft_adjoint": (i32, [vp, vp, vp, i32, vp, vp, vp, vp]),
            "pft_batch_create": (i32, [P(pft_params), i32, vp, P(vp)]),
            "pft_batch_destroy": (None, [vp]),
            "pft_batch_last_error": (ctypes.c_char_p, [vp]),
            "pft_batch_evaluate": (i32, [vp, vp, vp, vp, vp, vp, vp]),
            "pft_batch_cl_steps": (i32, [vp, vp, vp, P(pft_step), i32, vp, i64]),
            "pft_batch_sync": (i32, [vp]),
            "pft_autotune": (i32, [i32, vp, i32, vp, vp, vp]),
            "pft_tune_save": (i32, [ctypes.c_char_p]),
            "pft_tune_load": (i32, [ctypes.c_char_p]),
            "pft_set_variant": (i32, [vp, i32, i32]),
            "pft_set_concurrent_sweeps": (i32, [vp, i32]),
            "pft_set_fused_planes": (i32, [vp, i32]),
            "pft_fused_planes": (i32, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _status_name(status: int) -> str:
    try:
        return load().pft_status_string(status).decode()
    except Exception:  # library not loadable: still report the number
        return f"status {status}"


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _field(t: torch.Tensor, shape, name: str) -> int:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def _opt(t, shape, name):
    return None if t is None else _field(t, shape, name)


def pft_contour_plan(ns: int, f: float):
    """Host-only contour plan: (h[K], blk[K], junction J)."""
    import numpy as np
    h = np.zeros(ns + 1)
    blk = np.zeros(ns + 1, dtype=np.int32)
    J = np.zeros(1, dtype=np.int32)
    K = load().pft_contour_plan(ns, f, h.ctypes.data, blk.ctypes.data, J.ctypes.data)
    if K < 0:
        raise PftError(PFT_E_INVALID, "invalid contour parameters")
    return h[:K].copy(), blk[:K].copy(), int(J[0])


@dataclass
class Params:
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
    precision: int = PFT_C128
    scheme: int = PFT_RQM4
    model: int = 0
    B: float = 0.0
    storage: int = 0
    bc: tuple = (0, 0, 0)

    def c(self) -> pft_params:
        return pft_params(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz, self.ns, self.f,
                          self.chiN, self.C, self.precision, self.scheme, self.model, self.B, self.storage,
                          (ctypes.c_int32 * 3)(*self.bc))


class Context:
    """Owns a ``pft_ctx``; methods are the C entry points with tensors."""

    def __init__(self, params: Params, stream: int | None = None):
        lib = load()
        self.params = params
        self.shape = (params.nx, params.ny, params.nz)
        handle = ctypes.c_void_p()
        st = lib.pft_create(ctypes.byref(params.c()), _stream() if stream is None else stream,
                            ctypes.byref(handle))
        if st != PFT_OK:
            raise PftError(st, "pft_create failed")
        self._h = handle
        self.K = lib.pft_num_steps(self._h)

    def close(self):
        if getattr(self, "_h", None):
            load().pft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != PFT_OK:
            raise PftError(st, load().pft_last_error(self._h).decode())

    # -- entry points -------------------------------------------------------
    def pft_propagate(self, w_plus, w_minus):
        self._check(load().pft_propagate(self._h, _field(w_plus, self.shape, "w_plus"),
                                         self._wm(w_minus)))

    def _wm(self, w_minus):
        # the Edwards model has one field (passed as w_plus); w_minus may be None
        if w_minus is None and self.params.model == PFT_EDWARDS:
            return None
        return _field(w_minus, self.shape, "w_minus")

    def pft_densities(self, phi_a, phi_b, Q=None):
        self._check(load().pft_densities(self._h, _field(phi_a, self.shape, "phi_a"),
                                         _field(phi_b, self.shape, "phi_b"), _opt(Q, (1,), "Q")))

    def pft_evaluate_graph(self, w_plus, w_minus, phi_a, phi_b, Q=None, nreps: int = 1):
        self._check(load().pft_evaluate_graph(self._h, _field(w_plus, self.shape, "w_plus"), self._wm(w_minus),
                                              _field(phi_a, self.shape, "phi_a"),
                                              _field(phi_b, self.shape, "phi_b"), _opt(Q, (1,), "Q"), int(nreps)))

    def pft_set_box(self, lx: float, ly: float, lz: float):
        self._check(load().pft_set_box(self._h, float(lx), float(ly), float(lz)))
        self.params = replace(self.params, lx=float(lx), ly=float(ly), lz=float(lz))

    def pft_hamiltonian(self, w_plus, w_minus, H, h_intensive=None):
        self._check(load().pft_hamiltonian(self._h, _field(w_plus, self.shape, "w_plus"),
                                           self._wm(w_minus),
                                           _field(H, (1,), "H"), _opt(h_intensive, (1,), "h")))

    def pft_cl_step(self, w_plus, w_minus, step: pft_step, phi_a=None, phi_b=None, Q=None, H=None):
        self._check(load().pft_cl_step(self._h, _field(w_plus, self.shape, "w_plus"),
                                       self._wm(w_minus), ctypes.byref(step),
                                       _opt(phi_a, self.shape, "phi_a"), _opt(phi_b, self.shape, "phi_b"),
                                       _opt(Q, (1,), "Q"), _opt(H, (1,), "H")))

    def pft_cl_step_static(self, w_plus, w_minus, step: pft_step, phi_a=None, phi_b=None, Q=None, H=None):
        """pft_cl_step with the semi-implicit step's work memory in the
        library's fixed device array (no allocation)."""
        self._check(load().pft_cl_step_static(self._h, _field(w_plus, self.shape, "w_plus"),
                                              self._wm(w_minus), ctypes.byref(step),
                                              _opt(phi_a, self.shape, "phi_a"), _opt(phi_b, self.shape, "phi_b"),
                                              _opt(Q, (1,), "Q"), _opt(H, (1,), "H")))

    def pft_node_q(self, qnode):
        self._check(load().pft_node_q(self._h, _field(qnode, (self.K + 1,), "qnode")))

    def pft_get_slice(self, which: int, node: int, out):
        self._check(load().pft_get_slice(self._h, which, node, _field(out, self.shape, "out")))

    def pft_apply_step(self, step_index: int, q_in, q_out):
        self._check(load().pft_apply_step(self._h, step_index, _field(q_in, self.shape, "q_in"),
                                          _field(q_out, self.shape, "q_out")))

    def pft_diffuse(self, u, h: float):
        self._check(load().pft_diffuse(self._h, _field(u, self.shape, "u"), float(h)))

    def pft_debug_kgrid(self):
        import numpy as np
        out = np.zeros(self.shape, dtype=np.int32)
        self._check(load().pft_debug_kgrid(self._h, out.ctypes.data))
        return out

    def pft_status_flags(self) -> int:
        flags = ctypes.c_uint32(0)
        st = load().pft_status_flags(self._h, ctypes.byref(flags))
        if st not in (PFT_OK, PFT_E_NONFINITE):
            self._check(st)
        return flags.value

    def pft_adjoint(self, w_plus, w_minus, dH_dwplus, dH_dwminus, dH_dL=None, H=None, ckpt_every: int = 0):
        self._check(load().pft_adjoint(self._h, _field(w_plus, self.shape, "w_plus"),
                                       _field(w_minus, self.shape, "w_minus"), int(ckpt_every),
                                       _field(dH_dwplus, self.shape, "dH_dwplus"),
                                       _field(dH_dwminus, self.shape, "dH_dwminus"),
                                       _opt(dH_dL, (3,), "dH_dL"), _opt(H, (1,), "H")))

    def pft_set_concurrent_sweeps(self, on: bool):
        self._check(load().pft_set_concurrent_sweeps(self._h, int(bool(on))))

    def pft_set_fused_planes(self, on):
        """0 / False: axis schedule; 1 / True: fused yz passes in both sweeps;
        2: in the conjugate sweep only."""
        self._check(load().pft_set_fused_planes(self._h, int(on)))

    def pft_fused_planes(self) -> int:
        return load().pft_fused_planes(self._h)

    def pft_set_variant(self, axis: int, variant: int):
        self._check(load().pft_set_variant(self._h, axis, variant))

    def pft_profile_begin(self):
        self._check(load().pft_profile_begin(self._h))

    def pft_profile_end(self):
        """{kind: (ms, launches, algorithmic bytes)} since pft_profile_begin."""
        import numpy as np
        n = len(KERNEL_KINDS)
        ms, cnt, by = np.zeros(n), np.zeros(n, np.int64), np.zeros(n)
        self._check(load().pft_profile_end(self._h, ms.ctypes.data, cnt.ctypes.data, by.ctypes.data))
        return {k: (float(ms[i]), int(cnt[i]), float(by[i])) for i, k in enumerate(KERNEL_KINDS)}

    # -- conveniences (allocate outputs, still all-GPU) ----------------------
    def evaluate(self, w_plus, w_minus=None):
        """propagate + densities + hamiltonian; returns dict of GPU tensors
        (Edwards model: w_plus is omega, w_minus None, phiA is phi)."""
        dev = w_plus.device
        phi_a = torch.empty(self.shape, dtype=torch.complex128, device=dev)
        phi_b = torch.empty_like(phi_a)
        Q = torch.empty(1, dtype=torch.complex128, device=dev)
        H = torch.empty(1, dtype=torch.complex128, device=dev)
        hint = torch.empty(1, dtype=torch.complex128, device=dev)
        self.pft_propagate(w_plus, w_minus)
        self.pft_densities(phi_a, phi_b, Q)
        self.pft_hamiltonian(w_plus, w_minus, H, hint)
        return {"phiA": phi_a, "phiB": phi_b, "Q": Q, "H": H, "h": hint}


def pft_noise_words(seed: int, replica: int, step: int, field: int, M: int, device="cuda"):
    out = torch.empty(4 * ((M + 3) // 4), dtype=torch.int64, device=device)
    st = load().pft_noise_words(seed, replica, step, field, M, out.data_ptr(), _stream())
    if st != PFT_OK:
        raise PftError(st, "pft_noise_words failed")
    return out


def pft_noise_normals(seed: int, replica: int, step: int, field: int, M: int, device="cuda"):
    out = torch.empty(M, dtype=torch.float64, device=device)
    st = load().pft_noise_normals(seed, replica, step, field, M, out.data_ptr(), _stream())
    if st != PFT_OK:
        raise PftError(st, "pft_noise_normals failed")
    return out


def pft_copy_probe(src: torch.Tensor, dst: torch.Tensor):
    """Plain device copy of src into dst through the library's copy kernel."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous CUDA tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst sizes differ")
    st = load().pft_copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, _stream())
    if st != PFT_OK:
        raise PftError(st, "pft_copy_probe failed")


class Batch:
    """Owns a ``pft_batch`` of independent replicas (each its own Params)."""

    def __init__(self, params_list, stream: int | None = None):
        lib = load()
        self.params = list(params_list)
        self.n = len(self.params)
        self.shapes = [(p.nx, p.ny, p.nz) for p in self.params]
        arr = (pft_params * self.n)(*[p.c() for p in self.params])
        handle = ctypes.c_void_p()
        st = lib.pft_batch_create(arr, self.n, _stream() if stream is None else stream, ctypes.byref(handle))
        if st != PFT_OK:
            raise PftError(st, "pft_batch_create failed")
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            load().pft_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != PFT_OK:
            raise PftError(st, load().pft_batch_last_error(self._h).decode())

    def _ptrs(self, tensors, name, optional=False):
        if tensors is None and optional:
            return None
        if len(tensors) != self.n:
            raise ValueError(f"{name}: expected {self.n} tensors")
        return (ctypes.c_void_p * self.n)(*[_field(t, s, name) for t, s in zip(tensors, self.shapes)])

    def pft_batch_evaluate(self, w_plus, w_minus, phi_a, phi_b, Q, H):
        self._check(load().pft_batch_evaluate(self._h, self._ptrs(w_plus, "w_plus"),
                                              self._ptrs(w_minus, "w_minus", optional=True),
                                              self._ptrs(phi_a, "phi_a"), self._ptrs(phi_b, "phi_b"),
                                              _field(Q, (self.n,), "Q"), _field(H, (self.n,), "H")))

    def pft_batch_cl_steps(self, w_plus, w_minus, step: pft_step, nsteps: int, log=None):
        rows = 0 if log is None else log.shape[0]
        if log is not None:
            _field(log, (rows, self.n, 2), "log")
        self._check(load().pft_batch_cl_steps(self._h, self._ptrs(w_plus, "w_plus"),
                                              self._ptrs(w_minus, "w_minus", optional=True),
                                              ctypes.byref(step), int(nsteps),
                                              None if log is None else log.data_ptr(), rows))

    def pft_batch_sync(self):
        self._check(load().pft_batch_sync(self._h))


def pft_autotune(precision: int, sizes):
    """Time every kernel variant for each axis length; returns
    ({N: (z variant, x variant, y variant)},
     {N: [[z ms per variant], [x ms per variant], [y ms per variant]]})."""
    import numpy as np
    nv = MAX_VARIANTS
    sz = np.ascontiguousarray(sizes, dtype=np.int32)
    ch = np.zeros(3 * len(sz), dtype=np.int32)
    tm = np.zeros(3 * nv * len(sz))
    st = load().pft_autotune(precision, sz.ctypes.data, len(sz), _stream(), ch.ctypes.data, tm.ctypes.data)
    if st != PFT_OK:
        raise PftError(st, "pft_autotune failed")
    return ({int(n): tuple(int(v) for v in ch[3 * i:3 * i + 3]) for i, n in enumerate(sz)},
            {int(n): tm[3 * nv * i:3 * nv * (i + 1)].reshape(3, nv).tolist() for i, n in enumerate(sz)})


def pft_tune_save(path: str):
    if load().pft_tune_save(path.encode()) != PFT_OK:
        raise PftError(PFT_E_INVALID, f"cannot write {path}")


def pft_tune_load(path: str):
    if load().pft_tune_load(path.encode()) != PFT_OK:
        raise PftError(PFT_E_INVALID, f"cannot read {path}")
