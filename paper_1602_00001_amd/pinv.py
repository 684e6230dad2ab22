"""Python binding of libpinv (C-ABI in include/pinv.h): argument marshalling only.

Every step of the solve runs in the HIP library; torch provides device memory
(tensors) and streams.  Importing this module loads ``_lib/libpinv.so`` and
fails loudly if it has not been built (``__graft_entry__.build()``).

Layouts: right-hand sides, solutions and adjoint vectors are torch float64
CUDA tensors of shape [nrhs, N] (row r = right-hand side r, contiguous), which
is the library's column-major N x nrhs layout with ld = N.  Nodal arrays
(permittivity, Dirichlet data, eps-gradient) are [n_y, n_x].
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PINV_LIBRARY: another build of the same library (the sanitized host build,
# _lib/libpinv_san.so); the default is the release build
LIB_PATH = os.environ.get("PINV_LIBRARY") or os.path.join(_HERE, "_lib", "libpinv.so")

OK, E_INVALID_ARG, E_NOT_SPD, E_OOM, E_HIP, E_UNSUPPORTED, E_STATE, E_IO = 0, -1, -2, -3, -4, -5, -6, -7
MODES = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3, "int8": 4, "fp64_sym": 5, "fix16_tile": 6}
SCALE_ROW = 0
NOALLOC_SCRATCH_BYTES = 64 << 20   # PINV_NOALLOC_SCRATCH_BYTES


class PinvError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("h", ctypes.c_double)]


class Grid3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("_pad", ctypes.c_int32),
                ("h", ctypes.c_double)]


class GridGeneral(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("n", ctypes.c_int32), ("h", ctypes.c_double),
                ("has_fp64", ctypes.c_int32), ("int8_slices", ctypes.c_int32), ("has_fp32", ctypes.c_int32),
                ("has_bf16", ctypes.c_int32), ("has_lift", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("nz", ctypes.c_int32), ("general", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("has_sym", ctypes.c_int32),
                ("has_tile16", ctypes.c_int32), ("fp64_symmetric", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("rho", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("ld", ctypes.c_int64), ("nrhs", ctypes.c_int32), ("_pad", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, vp, dp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
    P = ctypes.POINTER
    sig = {
        "pinv_build_inverse": ([P(Grid), dp, dp, vp, P(vp)], i32),
        "pinv_build_inverse_3d": ([P(Grid3), dp, dp, vp, P(vp)], i32),
        "pinv_build_inverse_general": ([P(GridGeneral), dp, dp, dp, vp, P(vp)], i32),
        "pinv_build_inverse_beta": ([P(Grid), dp, dp, vp, P(vp)], i32),
        "pinv_import_inverse": ([P(Grid), dp, i64, dp, dp, dp, vp, P(vp)], i32),
        "pinv_export_inverse": ([vp, dp, i64, dp, vp], i32),
        "pinv_quantize_inverse": ([vp, i32, i32, i32, vp], i32),
        "pinv_prepare_split": ([vp, i32, vp], i32),
        "pinv_export_quantized": ([vp, vp, vp, vp], i32),
        "pinv_export_tile16": ([vp, vp, vp, vp], i32),
        "pinv_apply_inverse": ([vp, i32, i32, dp, i64, i32, dp, i64, vp], i32),
        "pinv_apply_inverse_noalloc": ([vp, i32, dp, i64, i32, dp, i64, vp], i32),
        "pinv_apply_inverse_adjoint": ([vp, i32, i32, dp, i64, i32, dp, i64, vp], i32),
        "pinv_grad_eps": ([vp, dp, i64, dp, i64, i32, dp, vp], i32),
        "pinv_grad_eps_general": ([vp, dp, i64, dp, i64, i32, dp, dp, vp], i32),
        "pinv_grad_beta": ([vp, dp, i64, dp, i64, i32, dp, vp], i32),
        "pinv_apply_batched": ([P(Request), i32, i32, i32, vp], i32),
        "pinv_batched_release": ([], i32),
        "pinv_get_info": ([vp, P(Info)], i32),
        "pinv_destroy": ([vp], i32),
        "pinv_trace_enable": ([i32], i32),
        "pinv_trace_read": ([ctypes.c_char_p, P(ctypes.c_double), P(i64)], i32),
        "pinv_trace_read_each": ([ctypes.c_char_p, P(ctypes.c_double), i64, P(ctypes.c_double), P(i64)], i32),
        "pinv_int8_variants": ([], i32),
        "pinv_set_int8_variant": ([vp, i32, i32], i32),
        "pinv_autotune_int8": ([vp, i32, dp, i64, i32, i32, P(ctypes.c_double), i32, P(i32), vp], i32),
        "pinv_save": ([vp, ctypes.c_char_p, vp], i32),
        "pinv_load": ([ctypes.c_char_p, vp, P(vp)], i32),
        "pinv_status_string": ([i32], ctypes.c_char_p),
        "pinv_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()

EXPORTED = ("pinv_build_inverse", "pinv_build_inverse_3d", "pinv_build_inverse_general", "pinv_build_inverse_beta", "pinv_grad_eps_general", "pinv_grad_beta", "pinv_import_inverse", "pinv_export_inverse", "pinv_quantize_inverse",
            "pinv_prepare_split", "pinv_export_quantized", "pinv_export_tile16", "pinv_apply_inverse", "pinv_apply_inverse_noalloc", "pinv_apply_inverse_adjoint",
            "pinv_grad_eps", "pinv_apply_batched", "pinv_batched_release", "pinv_get_info", "pinv_destroy", "pinv_status_string",
            "pinv_version", "pinv_trace_enable", "pinv_trace_read", "pinv_trace_read_each", "pinv_int8_variants",
            "pinv_set_int8_variant", "pinv_autotune_int8", "pinv_save", "pinv_load")


def status_string(st):
    return lib.pinv_status_string(int(st)).decode()


def version():
    return lib.pinv_version().decode()


def int8_variants():
    return int(lib.pinv_int8_variants())


def trace_enable(on=True):
    """Record HIP events around every kernel the library launches."""
    _check(lib.pinv_trace_enable(int(bool(on))), "pinv_trace_enable")


def trace_read(kernel):
    """(total milliseconds, launches) of the recorded launches of one kernel family."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib.pinv_trace_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)), "pinv_trace_read")
    return ms.value, cnt.value


def trace_read_each(kernel, cap=4096):
    """(list of per-launch milliseconds, launches) of the recorded launches of
    one kernel family, in launch order (at most ``cap`` listed)."""
    buf = (ctypes.c_double * cap)()
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib.pinv_trace_read_each(kernel.encode(), buf, cap, ctypes.byref(ms), ctypes.byref(cnt)),
           "pinv_trace_read_each")
    return list(buf[:min(cnt.value, cap)]), cnt.value


def _check(st, what):
    if st != OK:
        raise PinvError(st, what)


def _host_nodal(a, nx, ny):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.shape != (ny, nx):
        raise ValueError(f"nodal array must have shape ({ny}, {nx}), got {a.shape}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _mode(mode):
    if isinstance(mode, str):
        return MODES[mode]
    return int(mode)


def _vectors(t, n, name):
    """[nrhs, N] float64 CUDA tensor with contiguous rows -> (ptr, ld, nrhs)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() == 1:
        t = t.view(1, -1)
    if t.dim() == 2 and t.shape[1] == n and t.shape[0] == 0:
        return ctypes.c_void_p(t.data_ptr()), n, 0     # empty block: torch reports zero strides
    if t.dim() != 2 or t.shape[1] != n or (n > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must have shape [nrhs, {n}] with contiguous rows")
    ld = t.stride(0) if t.shape[0] > 1 else n
    return ctypes.c_void_p(t.data_ptr()), ld, t.shape[0]


class PoissonInverse:
    """A precomputed dense inverse of the 5-point operator on one grid."""

    def __init__(self, handle, nx, ny, h, nz=0):
        self._h = handle
        self.nx, self.ny, self.nz, self.h = nx, ny, nz, h
        self.n = (nx - 2) * (ny - 2) * (nz - 2 if nz else 1)

    # -- construction ---------------------------------------------------------
    @classmethod
    def build(cls, nx, ny, h=None, eps=None, u_boundary=None, stream=None):
        """Steps 1-2 on the GPU: assemble K from nodal eps and invert it."""
        if h is None:
            h = 1.0 / (max(nx, ny) - 1)
        g = Grid(nx, ny, h)
        e = _host_nodal(eps, nx, ny)
        ub = _host_nodal(u_boundary, nx, ny)
        out = ctypes.c_void_p()
        _check(lib.pinv_build_inverse(ctypes.byref(g), _ptr(e), _ptr(ub), _stream(stream), ctypes.byref(out)),
               "pinv_build_inverse")
        return cls(out, nx, ny, h)

    @classmethod
    def build3d(cls, nx, ny, nz, h=None, eps=None, u_boundary=None, stream=None):
        """Steps 1-2 for the 3-D 7-point operator; nodal arrays are [nz, ny, nx]."""
        if h is None:
            h = 1.0 / (max(nx, ny, nz) - 1)
        g = Grid3(nx, ny, nz, 0, h)

        def nodal(a):
            if a is None:
                return None
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
            if a.shape != (nz, ny, nx):
                raise ValueError(f"nodal array must have shape ({nz}, {ny}, {nx}), got {a.shape}")
            return a

        e, ub = nodal(eps), nodal(u_boundary)
        out = ctypes.c_void_p()
        _check(lib.pinv_build_inverse_3d(ctypes.byref(g), _ptr(e), _ptr(ub), _stream(stream), ctypes.byref(out)),
               "pinv_build_inverse_3d")
        return cls(out, nx, ny, h, nz)

    @classmethod
    def build_general(cls, x, y, eps_x=None, eps_y=None, u_boundary=None, stream=None):
        """Steps 1-2 on a non-uniform tensor grid (node coordinates x, y) with
        permittivity per direction; the op's h is 1 (G holds K^{-1} diag(A))."""
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        y = np.ascontiguousarray(np.asarray(y, dtype=np.float64))
        nx, ny = x.size, y.size
        g = GridGeneral(nx, ny, x.ctypes.data_as(ctypes.c_void_p), y.ctypes.data_as(ctypes.c_void_p))
        ex, ey, ub = (_host_nodal(a, nx, ny) for a in (eps_x, eps_y, u_boundary))
        out = ctypes.c_void_p()
        _check(lib.pinv_build_inverse_general(ctypes.byref(g), _ptr(ex), _ptr(ey), _ptr(ub), _stream(stream),
                                              ctypes.byref(out)), "pinv_build_inverse_general")
        return cls(out, nx, ny, 1.0)

    @classmethod
    def build_beta(cls, nx, ny, beta, u_boundary=None, stream=None):
        """Steps 1-2 for Eq. 3 with arbitrary coefficients beta [4, ny, nx]
        (directions i-1, i+1, j-1, j+1): GPU LU inverse with partial pivoting;
        the op's h is 1 and apply gives u = A^{-1}(rho + b_B)."""
        b = np.ascontiguousarray(np.asarray(beta, dtype=np.float64))
        if b.shape != (4, ny, nx):
            raise ValueError(f"beta must have shape (4, {ny}, {nx}), got {b.shape}")
        ub = _host_nodal(u_boundary, nx, ny)
        out = ctypes.c_void_p()
        _check(lib.pinv_build_inverse_beta(ctypes.byref(Grid(nx, ny, 1.0)), _ptr(b), _ptr(ub), _stream(stream),
                                           ctypes.byref(out)), "pinv_build_inverse_beta")
        return cls(out, nx, ny, 1.0)

    @classmethod
    def from_inverse(cls, nx, ny, h, G, eps=None, u_boundary=None, w=None, stream=None):
        """Create from a host inverse G [N, N] (row-major float64)."""
        G = np.ascontiguousarray(np.asarray(G, dtype=np.float64))
        n = (nx - 2) * (ny - 2)
        if G.shape != (n, n):
            raise ValueError(f"G must be ({n}, {n})")
        g = Grid(nx, ny, h)
        e = _host_nodal(eps, nx, ny)
        ub = _host_nodal(u_boundary, nx, ny)
        wv = None if w is None else np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(n))
        out = ctypes.c_void_p()
        _check(lib.pinv_import_inverse(ctypes.byref(g), _ptr(G), n, _ptr(e), _ptr(ub), _ptr(wv), _stream(stream),
                                       ctypes.byref(out)), "pinv_import_inverse")
        return cls(out, nx, ny, h)

    @classmethod
    def load(cls, path, stream=None):
        """An op from a file written by save() (no rebuild)."""
        out = ctypes.c_void_p()
        _check(lib.pinv_load(os.fsencode(path), _stream(stream), ctypes.byref(out)), "pinv_load")
        h = cls(out, 3, 3, 1.0)
        i = h.info()
        h.nx, h.ny, h.nz, h.h, h.n = i["nx"], i["ny"], i["nz"], i["h"], i["n"]
        return h

    def save(self, path, stream=None):
        """Write the op's G and/or int8 slices, lift and grid to a file."""
        _check(lib.pinv_save(self._h, os.fsencode(path), _stream(stream)), "pinv_save")
        return self

    # -- representations ------------------------------------------------------
    def quantize(self, bits, keep_fp64=True, stream=None):
        _check(lib.pinv_quantize_inverse(self._h, int(bits), SCALE_ROW, int(bool(keep_fp64)), _stream(stream)),
               "pinv_quantize_inverse")
        return self

    def prepare_split(self, mode, stream=None):
        _check(lib.pinv_prepare_split(self._h, _mode(mode), _stream(stream)), "pinv_prepare_split")
        return self

    def export_inverse(self, stream=None):
        G = np.empty((self.n, self.n), dtype=np.float64)
        w = np.empty(self.n, dtype=np.float64)
        _check(lib.pinv_export_inverse(self._h, _ptr(G), self.n, _ptr(w), _stream(stream)), "pinv_export_inverse")
        return G, w

    def export_quantized(self, stream=None):
        S = self.info()["int8_slices"]
        if S == 0:
            raise PinvError(E_STATE, "export_quantized")
        Q = np.empty((S, self.n, self.n), dtype=np.int8)
        e = np.empty(self.n, dtype=np.int32)
        _check(lib.pinv_export_quantized(self._h, _ptr(Q), _ptr(e), _stream(stream)), "pinv_export_quantized")
        return Q, e

    def export_tile16(self, stream=None):
        """(q int16 [N, N], tile exponents int32 [T, T]) of the 16-bit copy with
        64 x 64 tile scales (after ``prepare_split("fix16_tile")``)."""
        T = -(-self.n // 64)
        q = np.empty((self.n, self.n), dtype=np.int16)
        e = np.empty((T, T), dtype=np.int32)
        _check(lib.pinv_export_tile16(self._h, _ptr(q), _ptr(e), _stream(stream)), "pinv_export_tile16")
        return q, e

    # -- the solve and its derivatives ----------------------------------------
    def apply(self, rho, mode="fp64", rho_bits=16, out=None, stream=None):
        """u = L^{-1} rho for rho [nrhs, N] (float64, CUDA)."""
        import torch
        p_rho, ld_rho, nrhs = _vectors(rho, self.n, "rho")
        if out is None:
            out = torch.empty((nrhs, self.n), dtype=torch.float64, device=rho.device)
        p_u, ld_u, nu = _vectors(out, self.n, "out")
        if nu != nrhs:
            raise ValueError("out must have as many rows as rho")
        _check(lib.pinv_apply_inverse(self._h, _mode(mode), int(rho_bits), p_rho, ld_rho, nrhs, p_u, ld_u,
                                      _stream(stream)), "pinv_apply_inverse")
        return out

    def apply_noalloc(self, rho, rho_bits=16, out=None, stream=None):
        """The INT8 apply through pinv_apply_inverse_noalloc (no device
        allocation inside the call; ``out`` must then be given by callers that
        cannot allocate either)."""
        import torch
        p_rho, ld_rho, nrhs = _vectors(rho, self.n, "rho")
        if out is None:
            out = torch.empty((nrhs, self.n), dtype=torch.float64, device=rho.device)
        p_u, ld_u, nu = _vectors(out, self.n, "out")
        if nu != nrhs:
            raise ValueError("out must have as many rows as rho")
        _check(lib.pinv_apply_inverse_noalloc(self._h, int(rho_bits), p_rho, ld_rho, nrhs, p_u, ld_u, _stream(stream)),
               "pinv_apply_inverse_noalloc")
        return out

    def apply_adjoint(self, g, mode="fp64", g_bits=16, out=None, stream=None):
        """lambda = dLoss/drho = -h^2 G^T g."""
        import torch
        p_g, ld_g, nrhs = _vectors(g, self.n, "g")
        if out is None:
            out = torch.empty((nrhs, self.n), dtype=torch.float64, device=g.device)
        p_l, ld_l, nl = _vectors(out, self.n, "out")
        if nl != nrhs:
            raise ValueError("out must have as many rows as g")
        _check(lib.pinv_apply_inverse_adjoint(self._h, _mode(mode), int(g_bits), p_g, ld_g, nrhs, p_l, ld_l,
                                              _stream(stream)), "pinv_apply_inverse_adjoint")
        return out

    def grad_eps(self, u, lam, out=None, stream=None):
        """Nodal dLoss/deps [n_y, n_x] ([n_z, n_y, n_x] for a 3-D op) from forward
        solutions and adjoint outputs."""
        import torch
        p_u, ld_u, nu = _vectors(u, self.n, "u")
        p_l, ld_l, nl = _vectors(lam, self.n, "lambda")
        if nu != nl:
            raise ValueError("u and lambda must have the same number of rows")
        shape = (self.nz, self.ny, self.nx) if self.nz else (self.ny, self.nx)
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=u.device)
        if out.dtype != torch.float64 or not out.is_contiguous() or tuple(out.shape) != shape:
            raise ValueError(f"out must be a contiguous float64 {list(shape)} tensor")
        _check(lib.pinv_grad_eps(self._h, p_u, ld_u, p_l, ld_l, nu, ctypes.c_void_p(out.data_ptr()),
                                 _stream(stream)), "pinv_grad_eps")
        return out

    def grad_eps_general(self, u, lam, split=True, stream=None):
        """Per-direction dLoss/deps_x, dLoss/deps_y ([n_y, n_x] each) for an op
        from :meth:`build_general`; with split=False one [n_y, n_x] array, the
        gradient with respect to a single field used for both directions."""
        import torch
        p_u, ld_u, nu = _vectors(u, self.n, "u")
        p_l, ld_l, nl = _vectors(lam, self.n, "lambda")
        if nu != nl:
            raise ValueError("u and lambda must have the same number of rows")
        gx = torch.empty((self.ny, self.nx), dtype=torch.float64, device=u.device)
        gy = torch.empty_like(gx) if split else None
        _check(lib.pinv_grad_eps_general(self._h, p_u, ld_u, p_l, ld_l, nu, ctypes.c_void_p(gx.data_ptr()),
                                         ctypes.c_void_p(gy.data_ptr()) if split else None, _stream(stream)),
               "pinv_grad_eps_general")
        return (gx, gy) if split else gx

    def grad_beta(self, u, lam, stream=None):
        """dLoss/dbeta [4, n_y, n_x] for an op from :meth:`build_beta`, from forward
        solutions u and adjoint outputs lam (= A^{-T} g)."""
        import torch
        p_u, ld_u, nu = _vectors(u, self.n, "u")
        p_l, ld_l, nl = _vectors(lam, self.n, "lambda")
        if nu != nl:
            raise ValueError("u and lambda must have the same number of rows")
        out = torch.empty((4, self.ny, self.nx), dtype=torch.float64, device=u.device)
        _check(lib.pinv_grad_beta(self._h, p_u, ld_u, p_l, ld_l, nu, ctypes.c_void_p(out.data_ptr()),
                                  _stream(stream)), "pinv_grad_beta")
        return out

    def set_int8_variant(self, rho_bits, variant):
        _check(lib.pinv_set_int8_variant(self._h, int(rho_bits), int(variant)), "pinv_set_int8_variant")

    def autotune_int8(self, rho_bits=16, rho=None, nrhs=None, reps=10, stream=None):
        """Time every int8 kernel variant on this op and keep the fastest.
        rho: representative right-hand sides ([nrhs, N] float64 CUDA tensor),
        or None for random digits of ``nrhs`` columns.
        Returns (best variant id, list of mean ms per launch).  With
        PINV_AUTOTUNE_CACHE naming a file, a stored choice is taken without
        timing (the list then holds its stored time and -1 elsewhere) and a new
        choice is appended there."""
        if rho is not None:
            p, ld, R = _vectors(rho, self.n, "rho")
        else:
            p, ld, R = None, 0, int(nrhs if nrhs is not None else 1024)
        nv = lib.pinv_int8_variants()
        ms = (ctypes.c_double * nv)()
        best = ctypes.c_int32(-1)
        _check(lib.pinv_autotune_int8(self._h, int(rho_bits), p, ld, R, int(reps), ms, nv, ctypes.byref(best),
                                      _stream(stream)), "pinv_autotune_int8")
        return best.value, list(ms)

    def info(self):
        i = Info()
        _check(lib.pinv_get_info(self._h, ctypes.byref(i)), "pinv_get_info")
        return {f: getattr(i, f) for f, _ in Info._fields_}

    def close(self):
        if self._h:
            lib.pinv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def batched_release():
    """Drop the cached plans of apply_batched (device and pinned memory)."""
    _check(lib.pinv_batched_release(), "pinv_batched_release")


def apply_batched(requests, mode="int8", rho_bits=16, stream=None):
    """requests: list of (PoissonInverse, rho [nrhs, N], u [nrhs, N]) with the
    same row stride for rho and u."""
    arr = (Request * len(requests))()
    for i, (op, rho, u) in enumerate(requests):
        p_r, ld_r, nr = _vectors(rho, op.n, "rho")
        p_u, ld_u, nu = _vectors(u, op.n, "u")
        if ld_r != ld_u or nr != nu:
            raise ValueError("rho and u of a request must share shape and stride")
        arr[i] = Request(op._h, p_r, p_u, ld_r, nr, 0)
    _check(lib.pinv_apply_batched(arr, len(requests), _mode(mode), int(rho_bits), _stream(stream)),
           "pinv_apply_batched")
