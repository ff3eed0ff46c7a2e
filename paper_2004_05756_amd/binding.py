"""ctypes binding of libtopo_rom.so (argument marshalling only).

Tensors are torch tensors on the GPU; their device pointers and the current HIP
stream are handed to the C ABI declared in include/topo_rom.h.  No arithmetic of the
method happens here.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libtopo_rom.so")

TOPO_OK, TOPO_EINVAL, TOPO_ENOMEM, TOPO_ENOCONV, TOPO_ENOTSPD, TOPO_EDEVICE, TOPO_EAGAIN = \
    0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1

# every symbol the public headers declare
EXPORTED = (
    "topo_ctx_create", "topo_ctx_destroy", "topo_last_error", "topo_strerror",
    "topo_ctx_workspace_bytes", "topo_element_stiffness", "topo_element_factor", "topo_apply",
    "topo_hdm_solve", "topo_hdm_solve_batch", "topo_hdm_gradient_batch",
    "topo_hdm_gradient", "topo_rom_build", "topo_rom_solve", "topo_rom_solve_noalloc",
    "topo_rom_solve_noalloc_max_bytes", "topo_rom_estimate",
    "topo_rom_gradient", "topo_pod_push", "topo_pod_basis", "topo_filter_forward",
    "topo_filter_adjoint", "topo_ctx_set_timing", "topo_ctx_kernel_time",
)
POD_MAX_WINDOW = 48


class TopoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_strerror(code)} ({code}): {msg}")
        self.code = code


class TopoMesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nel", C.c_int32 * 3), ("h", C.c_double * 3),
                ("E0", C.c_double), ("Emin", C.c_double), ("nu", C.c_double),
                ("penal", C.c_double), ("plane", C.c_int32)]


class TopoInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("refinements", C.c_int32), ("rel_resid", C.c_double),
                ("compliance_raw", C.c_double), ("compliance_corr", C.c_double),
                ("fp64_fallback", C.c_int32), ("status", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = C.c_void_p
_SIGS = {
    "topo_ctx_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_size_t]),
    "topo_ctx_destroy": (C.c_int, [_P]),
    "topo_last_error": (C.c_char_p, [_P]),
    "topo_strerror": (C.c_char_p, [C.c_int32]),
    "topo_ctx_workspace_bytes": (C.c_size_t, [_P]),
    "topo_ctx_set_timing": (C.c_int, [_P, C.c_int32]),
    "topo_ctx_kernel_time": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int64), C.c_int32]),
    "topo_element_stiffness": (C.c_int, [C.POINTER(TopoMesh), C.POINTER(C.c_double)]),
    "topo_element_factor": (C.c_int, [C.POINTER(TopoMesh), C.POINTER(C.c_double)]),
    "topo_apply": (C.c_int, [_P, C.POINTER(TopoMesh), _P, _P, _P, _P, C.c_int32, C.c_int32, _P]),
    "topo_hdm_solve": (C.c_int, [_P, C.POINTER(TopoMesh), _P, _P, _P, _P, C.c_double, C.c_int32,
                                 C.c_int32, C.POINTER(C.c_double), C.POINTER(TopoInfo), _P]),
    "topo_hdm_solve_batch": (C.c_int, [_P, C.POINTER(TopoMesh), _P, _P, _P, _P, C.c_int32, C.c_double,
                                       C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(TopoInfo), _P]),
    "topo_hdm_gradient": (C.c_int, [_P, C.POINTER(TopoMesh), _P, _P, _P, _P]),
    "topo_hdm_gradient_batch": (C.c_int, [_P, C.POINTER(TopoMesh), _P, _P, C.c_int32, _P, _P]),
    "topo_rom_build": (C.c_int, [_P, C.POINTER(TopoMesh), _P, C.c_int32, C.c_int32, C.c_int32, _P,
                                 _P, _P, C.c_int32, _P, _P, C.c_int32, _P]),
    "topo_rom_solve": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P, _P]),
    "topo_rom_solve_noalloc": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P, _P]),
    "topo_rom_solve_noalloc_max_bytes": (C.c_size_t, []),
    "topo_rom_estimate": (C.c_int, [_P, C.POINTER(TopoMesh), _P, C.c_int32, C.c_int32, C.c_int32,
                                    _P, _P, _P, C.c_int32, _P, _P, _P, _P, C.c_int32, _P, _P]),
    "topo_rom_gradient": (C.c_int, [_P, C.POINTER(TopoMesh), _P, C.c_int32, C.c_int32, C.c_int32,
                                    _P, _P, C.c_int32, _P, _P, _P]),
    "topo_filter_forward": (C.c_int, [_P, C.POINTER(TopoMesh), C.c_double, _P, C.c_int32, _P, _P,
                                      C.c_double, C.c_int32, C.c_int32, C.POINTER(C.c_int32), _P]),
    "topo_filter_adjoint": (C.c_int, [_P, C.POINTER(TopoMesh), C.c_double, _P, C.c_int32, _P, _P,
                                      C.c_double, C.c_int32, C.c_int32, C.POINTER(C.c_int32), _P]),
    "topo_pod_push": (C.c_int, [_P, C.c_int64, C.c_int32, _P, _P, C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32), _P, _P]),
    "topo_pod_basis": (C.c_int, [_P, C.c_int64, C.c_int32, _P, _P, C.c_int32, _P, C.c_int32,
                                 C.c_double, _P, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), _P, _P]),
}

_lib = None
_lock = threading.Lock()


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the shared library (no GPU needed) and declare every signature."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise RuntimeError(f"HIP library not built: {path} (run paper_2004_05756_amd.build)")
            lib = C.CDLL(path)
            for name, (res, args) in _SIGS.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
        return _lib


def _strerror(code):
    try:
        return load().topo_strerror(code).decode()
    except Exception:  # pragma: no cover - library missing
        return str(code)


def make_mesh(mesh) -> TopoMesh:
    """TopoMesh from any object with nel, h, E0, Emin, nu, penal (and optional plane)."""
    m = TopoMesh()
    nel = tuple(mesh.nel)
    m.dim = len(nel)
    for i in range(3):
        m.nel[i] = nel[i] if i < len(nel) else 1
        m.h[i] = float(mesh.h[i]) if i < len(nel) else 1.0
    m.E0, m.Emin, m.nu, m.penal = float(mesh.E0), float(mesh.Emin), float(mesh.nu), float(mesh.penal)
    m.plane = int(getattr(mesh, "plane", 0))
    return m


def element_stiffness(mesh):
    import numpy as np
    m = make_mesh(mesh)
    ne = m.dim * 2 ** m.dim
    out = (C.c_double * (ne * ne))()
    rc = load().topo_element_stiffness(C.byref(m), out)
    if rc != TOPO_OK:
        raise TopoError(rc, "element stiffness")
    return np.frombuffer(out, dtype=np.float64).reshape(ne, ne).copy()


def element_factor(mesh):
    """The 51-entry symmetry-blocked factor table of the element operator."""
    import numpy as np
    m = make_mesh(mesh)
    out = (C.c_double * 51)()
    rc = load().topo_element_factor(C.byref(m), out)
    if rc != TOPO_OK:
        raise TopoError(rc, "element factor")
    return np.frombuffer(out, dtype=np.float64).copy()


def _ptr(t, dtype=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def mesh_sizes(m: TopoMesh):
    """(elements, nodes, DOFs) of a TopoMesh."""
    ne, nn = 1, 1
    for i in range(m.dim):
        ne *= int(m.nel[i])
        nn *= int(m.nel[i]) + 1
    return ne, nn, m.dim * nn


def _numel(t, n, name):
    """Raise ValueError unless tensor t (if given) holds exactly n entries: a mis-shaped
    array would make the kernels read or write outside it."""
    if t is not None and int(t.numel()) != int(n):
        raise ValueError(f"{name} has {int(t.numel())} entries, expected {int(n)}")


def _rows(phi, n_dofs, k):
    if phi.dim() != 2 or int(phi.shape[0]) != n_dofs:
        raise ValueError(f"phi must be [N_u={n_dofs}][ldphi], got {tuple(phi.shape)}")
    if not 1 <= int(k) <= int(phi.shape[1]):
        raise ValueError(f"k={k} must lie in [1, ldphi={int(phi.shape[1])}]")


def _solve_shapes(B, k, k2, fhat, yhat, Jk, status):
    if k != k2:
        raise ValueError(f"Khat must be [B][k][k], got [{B}][{k}][{k2}]")
    _numel(fhat, k, "fhat")
    _numel(yhat, B * k, "yhat")
    _numel(Jk, B, "Jk")
    _numel(status, B, "status")


class Context:
    """One library context (device workspace + element tables) on one GPU."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self.lib = load()
        self.device = device
        h = C.c_void_p()
        rc = self.lib.topo_ctx_create(C.byref(h), device, int(budget_bytes))
        if rc != TOPO_OK:
            raise TopoError(rc, "context creation")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.topo_ctx_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != TOPO_OK:
            raise TopoError(rc, f"{what}: {self.lib.topo_last_error(self.h).decode()}")

    def workspace_bytes(self):
        return self.lib.topo_ctx_workspace_bytes(self.h)

    def set_timing(self, every: int):
        """Sample one launch in `every` of each hot kernel with HIP events (0 = off)."""
        self._check(self.lib.topo_ctx_set_timing(self.h, int(every)), "set_timing")

    def kernel_time(self, name: str, reset: bool = False, launches: bool = False):
        """(sampled launches, summed device ms) of one hot kernel, and with launches=True
        also the launches issued while timing was on."""
        n = C.c_int64()
        ms = C.c_double()
        nl = C.c_int64()
        rc = self.lib.topo_ctx_kernel_time(self.h, name.encode(), C.byref(n), C.byref(ms), C.byref(nl),
                                           int(reset))
        self._check(rc, "kernel_time")
        if launches:
            return int(n.value), float(ms.value), int(nl.value)
        return int(n.value), float(ms.value)

    # -- full-order model -------------------------------------------------------------
    def apply(self, mesh, rho, mask, x, y=None, prec=FP64, stream=None):
        import torch
        dt = torch.float64 if prec == FP64 else torch.float32
        B = rho.shape[0] if rho.dim() == 2 else 1
        if y is None:
            y = torch.empty_like(x)
        m = make_mesh(mesh)
        ne, _, nu = mesh_sizes(m)
        _numel(rho, B * ne, "rho")
        _numel(mask, nu, "mask")
        _numel(x, B * nu, "x")
        _numel(y, B * nu, "y")
        rc = self.lib.topo_apply(self.h, C.byref(m), _ptr(rho, torch.float64, "rho"),
                                 _ptr(mask, torch.uint8, "mask"), _ptr(x, dt, "x"),
                                 _ptr(y, dt, "y"), B, prec, _stream(stream))
        self._check(rc, "apply")
        return y

    def hdm_solve(self, mesh, rho, mask, f, u=None, rtol=1e-10, maxit=200000, prec=FP64,
                  stream=None, check=True):
        import torch
        if u is None:
            u = torch.empty_like(f)
        m = make_mesh(mesh)
        ne, _, nu = mesh_sizes(m)
        _numel(rho, ne, "rho")
        _numel(mask, nu, "mask")
        _numel(f, nu, "f")
        _numel(u, nu, "u")
        info = TopoInfo()
        comp = C.c_double()
        rc = self.lib.topo_hdm_solve(self.h, C.byref(m), _ptr(rho, torch.float64, "rho"),
                                     _ptr(mask, torch.uint8, "mask"), _ptr(f, torch.float64, "f"),
                                     _ptr(u, torch.float64, "u"), float(rtol), int(maxit), prec,
                                     C.byref(comp), C.byref(info), _stream(stream))
        if check:
            self._check(rc, "hdm_solve")
        d = info.as_dict()
        d["status"] = rc
        return u, d

    def hdm_solve_batch(self, mesh, rho, mask, f, u=None, rtol=1e-10, maxit=200000, prec=FP64,
                        stream=None, check=True):
        """B fields rho [B][N_e] sharing mask and load f: u [B][N_u] and one info dict per
        field (topo_hdm_solve_batch; each field's result does not depend on the batch)."""
        import torch
        if rho.dim() == 1:
            rho = rho.unsqueeze(0)
        B = int(rho.shape[0])
        if u is None:
            u = torch.empty((B, f.numel()), dtype=torch.float64, device=f.device)
        m = make_mesh(mesh)
        ne, _, nu = mesh_sizes(m)
        _numel(rho, B * ne, "rho")
        _numel(mask, nu, "mask")
        _numel(f, nu, "f")
        _numel(u, B * nu, "u")
        infos = (TopoInfo * B)()
        comp = (C.c_double * B)()
        rc = self.lib.topo_hdm_solve_batch(self.h, C.byref(m), _ptr(rho, torch.float64, "rho"),
                                           _ptr(mask, torch.uint8, "mask"), _ptr(f, torch.float64, "f"),
                                           _ptr(u, torch.float64, "u"), B, float(rtol), int(maxit), prec,
                                           comp, infos, _stream(stream))
        if check:
            self._check(rc, "hdm_solve_batch")
        return u, [infos[b].as_dict() for b in range(B)]

    def hdm_gradient_batch(self, mesh, rho, u, dc=None, stream=None):
        """dc/drho [B][N_e] of B fields at their states u [B][N_u] (topo_hdm_gradient_batch)."""
        import torch
        if rho.dim() == 1:
            rho = rho.unsqueeze(0)
        B = int(rho.shape[0])
        if dc is None:
            dc = torch.empty_like(rho)
        m = make_mesh(mesh)
        ne, _, nu = mesh_sizes(m)
        _numel(rho, B * ne, "rho")
        _numel(u, B * nu, "u")
        _numel(dc, B * ne, "dc")
        rc = self.lib.topo_hdm_gradient_batch(self.h, C.byref(m), _ptr(rho, torch.float64, "rho"),
                                              _ptr(u, torch.float64, "u"), B, _ptr(dc, torch.float64, "dc"),
                                              _stream(stream))
        self._check(rc, "hdm_gradient_batch")
        return dc

    def hdm_gradient(self, mesh, rho, u, dc=None, stream=None):
        import torch
        if dc is None:
            dc = torch.empty_like(rho)
        m = make_mesh(mesh)
        ne, _, nu = mesh_sizes(m)
        _numel(rho, ne, "rho")
        _numel(u, nu, "u")
        _numel(dc, ne, "dc")
        rc = self.lib.topo_hdm_gradient(self.h, C.byref(m), _ptr(rho, torch.float64, "rho"),
                                        _ptr(u, torch.float64, "u"), _ptr(dc, torch.float64, "dc"),
                                        _stream(stream))
        self._check(rc, "hdm_gradient")
        return dc

    # -- reduced-order model ----------------------------------------------------------
    def rom_build(self, mesh, phi, k, mask, f, rho, prec=MIXED, with_fhat=True, Khat=None,
                  fhat=None, stream=None):
        import torch
        if rho.dim() == 1:
            rho = rho.unsqueeze(0)
        B = rho.shape[0]
        dev = rho.device
        if Khat is None:
            Khat = torch.empty((B, k, k), dtype=torch.float64, device=dev)
        if with_fhat and fhat is None:
            fhat = torch.empty(k, dtype=torch.float64, device=dev)
        m = make_mesh(mesh)
        ne, _, nu = mesh_sizes(m)
        _rows(phi, nu, k)
        _numel(rho, B * ne, "rho")
        _numel(mask, nu, "mask")
        _numel(f, nu, "f")
        _numel(Khat, B * k * k, "Khat")
        _numel(fhat if with_fhat else None, k, "fhat")
        fp32 = 1 if phi.dtype == torch.float32 else 0
        rc = self.lib.topo_rom_build(self.h, C.byref(m), _ptr(phi, None, "phi"), fp32, int(k),
                                     int(phi.shape[1]), _ptr(mask, torch.uint8, "mask"),
                                     _ptr(f, torch.float64, "f"), _ptr(rho, torch.float64, "rho"), B,
                                     _ptr(Khat, torch.float64, "Khat"),
                                     _ptr(fhat, torch.float64, "fhat") if with_fhat else None,
                                     prec, _stream(stream))
        self._check(rc, "rom_build")
        return Khat, fhat

    def rom_solve(self, Khat, fhat, status=None, yhat=None, Jk=None, stream=None):
        import torch
        B, k, k2 = Khat.shape
        if yhat is None:
            yhat = torch.empty((B, k), dtype=torch.float64, device=Khat.device)
        if Jk is None:
            Jk = torch.empty(B, dtype=torch.float64, device=Khat.device)
        _solve_shapes(B, k, k2, fhat, yhat, Jk, status)
        rc = self.lib.topo_rom_solve(self.h, k, B, _ptr(Khat, torch.float64, "Khat"),
                                     _ptr(fhat, torch.float64, "fhat"), _ptr(yhat, torch.float64, "yhat"),
                                     _ptr(Jk, torch.float64, "Jk"),
                                     _ptr(status, torch.int32, "status") if status is not None else None,
                                     _stream(stream))
        self._check(rc, "rom_solve")
        return yhat, Jk

    def rom_solve_noalloc(self, Khat, fhat, status, yhat, Jk, stream=None):
        """topo_rom_solve_noalloc: the reduced solve with its factors in the library's
        fixed device array (no device allocation); every output tensor is the caller's."""
        import torch
        B, k, k2 = Khat.shape
        _solve_shapes(B, k, k2, fhat, yhat, Jk, status)
        rc = self.lib.topo_rom_solve_noalloc(self.h, k, B, _ptr(Khat, torch.float64, "Khat"),
                                             _ptr(fhat, torch.float64, "fhat"),
                                             _ptr(yhat, torch.float64, "yhat"), _ptr(Jk, torch.float64, "Jk"),
                                             _ptr(status, torch.int32, "status"), _stream(stream))
        self._check(rc, "rom_solve_noalloc")
        return yhat, Jk

    def rom_estimate(self, mesh, phi, k, mask, f, rho, Khat, yhat, max_refine=1, stream=None,
                     Jk=None, resnorm=None, dJ=None):
        """u = Phi yhat, ||f - K u|| with optional reduced refinement of yhat; with a dJ
        tensor [B][N_e] also the ROM sensitivity at the returned yhat (topo_rom_estimate)."""
        import torch
        if rho.dim() == 1:
            rho = rho.unsqueeze(0)
        B = rho.shape[0]
        dev = rho.device
        if Jk is None:
            Jk = torch.empty(B, dtype=torch.float64, device=dev)
        if resnorm is None:
            resnorm = torch.empty(B, dtype=torch.float64, device=dev)
        m = make_mesh(mesh)
        ne, _, nu = mesh_sizes(m)
        _rows(phi, nu, k)
        _numel(rho, B * ne, "rho")
        _numel(mask, nu, "mask")
        _numel(f, nu, "f")
        _numel(Khat, B * k * k, "Khat")
        _numel(yhat, B * k, "yhat")
        _numel(Jk, B, "Jk")
        _numel(resnorm, B, "resnorm")
        _numel(dJ, B * ne, "dJ")
        fp32 = 1 if phi.dtype == torch.float32 else 0
        rc = self.lib.topo_rom_estimate(self.h, C.byref(m), _ptr(phi, None, "phi"), fp32, int(k),
                                        int(phi.shape[1]), _ptr(mask, torch.uint8, "mask"),
                                        _ptr(f, torch.float64, "f"), _ptr(rho, torch.float64, "rho"),
                                        B, _ptr(Khat, torch.float64, "Khat") if Khat is not None else None,
                                        _ptr(yhat, torch.float64, "yhat"), _ptr(Jk, torch.float64, "Jk"),
                                        _ptr(resnorm, torch.float64, "resnorm"), int(max_refine),
                                        _ptr(dJ, torch.float64, "dJ"), _stream(stream))
        self._check(rc, "rom_estimate")
        return yhat, Jk, resnorm

    def rom_gradient(self, mesh, phi, k, mask, rho, yhat, dJ=None, stream=None):
        """dJ_k/drho [B][N_e] at the ROM state Phi yhat (topo_rom_gradient)."""
        import torch
        if rho.dim() == 1:
            rho = rho.unsqueeze(0)
        if yhat.dim() == 1:
            yhat = yhat.unsqueeze(0)
        B = rho.shape[0]
        if dJ is None:
            dJ = torch.empty_like(rho, dtype=torch.float64)
        m = make_mesh(mesh)
        ne, _, nu = mesh_sizes(m)
        _rows(phi, nu, k)
        _numel(rho, B * ne, "rho")
        _numel(mask, nu, "mask")
        _numel(yhat, B * k, "yhat")
        _numel(dJ, B * ne, "dJ")
        fp32 = 1 if phi.dtype == torch.float32 else 0
        rc = self.lib.topo_rom_gradient(self.h, C.byref(m), _ptr(phi, None, "phi"), fp32, int(k),
                                        int(phi.shape[1]), _ptr(mask, torch.uint8, "mask"),
                                        _ptr(rho, torch.float64, "rho"), B,
                                        _ptr(yhat, torch.float64, "yhat"), _ptr(dJ, torch.float64, "dJ"),
                                        _stream(stream))
        self._check(rc, "rom_gradient")
        return dJ

    def _filter(self, fn, name, mesh, r, x, out, nodal, rtol, maxit, warm, stream):
        import torch
        if x.dim() == 1:
            x = x.unsqueeze(0)
        B = x.shape[0]
        if out is None:
            out = torch.empty_like(x, dtype=torch.float64)
        m = make_mesh(mesh)
        ne, nn, _ = mesh_sizes(m)
        _numel(x, B * ne, "input")
        _numel(out, B * ne, "output")
        _numel(nodal, B * nn, "nodal")
        its = C.c_int32(0)
        rc = fn(self.h, C.byref(m), float(r), _ptr(x, torch.float64, "input"), B,
                _ptr(out, torch.float64, "output"), _ptr(nodal, torch.float64, "nodal"), float(rtol),
                int(maxit), 1 if (warm and nodal is not None) else 0, C.byref(its), _stream(stream))
        self._check(rc, name)
        return out, its.value

    def filter_forward(self, mesh, r, psi, rho=None, phi=None, rtol=1e-12, maxit=20000, warm=False,
                       stream=None):
        """rho*(psi) through the Helmholtz filter [B][N_e]; returns (rho, iterations).  With
        warm=True, phi holds the initial guess (topo_filter_forward)."""
        return self._filter(self.lib.topo_filter_forward, "filter_forward", mesh, r, psi, rho, phi, rtol,
                            maxit, warm, stream)

    def filter_adjoint(self, mesh, r, v, g=None, mu=None, rtol=1e-12, maxit=20000, warm=False, stream=None):
        """(d rho*/d psi)^T v [B][N_e]; returns (g, iterations).  With warm=True, mu holds
        the initial guess (topo_filter_adjoint)."""
        return self._filter(self.lib.topo_filter_adjoint, "filter_adjoint", mesh, r, v, g, mu, rtol, maxit,
                            warm, stream)

    def pod_push(self, S, G, state, u, stream=None):
        """Push snapshot u into the window (S [L][n], G [L][L], state = [count, next]
        host ints, updated in place) (topo_pod_push)."""
        import torch
        L, n = S.shape
        _numel(G, L * L, "G")
        _numel(u, n, "u")
        cnt, nxt = C.c_int32(int(state[0])), C.c_int32(int(state[1]))
        rc = self.lib.topo_pod_push(self.h, int(n), int(L), _ptr(S, torch.float64, "S"),
                                    _ptr(G, torch.float64, "G"), C.byref(cnt), C.byref(nxt),
                                    _ptr(u, torch.float64, "u"), _stream(stream))
        self._check(rc, "pod_push")
        state[0], state[1] = cnt.value, nxt.value

    def pod_basis(self, S, G, count, u, nmax, phi, rtol=1e-7, sigma=None, stream=None):
        """Basis GramSchmidt([POD(window), u]) written into phi [n][ldphi] (f32 or f64);
        returns (columns written, POD columns kept) (topo_pod_basis)."""
        import torch
        L, n = S.shape
        _numel(G, L * L, "G")
        _numel(u, n, "u")
        if phi.dim() != 2 or int(phi.shape[0]) != n:
            raise ValueError(f"phi must be [n={n}][ldphi], got {tuple(phi.shape)}")
        _numel(sigma, int(count), "sigma")
        ncols, npod = C.c_int32(0), C.c_int32(0)
        fp32 = 1 if phi.dtype == torch.float32 else 0
        if phi.dtype not in (torch.float32, torch.float64):
            raise TypeError("phi must be float32 or float64")
        rc = self.lib.topo_pod_basis(self.h, int(n), int(L), _ptr(S, torch.float64, "S"),
                                     _ptr(G, torch.float64, "G"), int(count),
                                     _ptr(u, torch.float64, "u"), int(nmax), float(rtol),
                                     _ptr(phi, None, "phi"), fp32, int(phi.shape[1]),
                                     C.byref(ncols), C.byref(npod),
                                     _ptr(sigma, torch.float64, "sigma"), _stream(stream))
        self._check(rc, "pod_basis")
        return ncols.value, npod.value


class SnapshotWindow:
    """Device-resident window of the L most recent snapshots of length n and their Gram
    matrix, for Context.pod_push / pod_basis."""

    def __init__(self, ctx, n, L, device="cuda"):
        import torch
        self.ctx = ctx
        self.S = torch.zeros((L, n), dtype=torch.float64, device=device)
        self.G = torch.zeros((L, L), dtype=torch.float64, device=device)
        self.state = [0, 0]

    @property
    def count(self):
        return self.state[0]

    def push(self, u, stream=None):
        self.ctx.pod_push(self.S, self.G, self.state, u, stream)

    def basis(self, u, nmax, phi, rtol=1e-7, sigma=None, stream=None):
        return self.ctx.pod_basis(self.S, self.G, self.count, u, nmax, phi, rtol, sigma, stream)


_ctx = {}


def context(device: int = 0) -> Context:
    """Process-wide default context per device."""
    if device not in _ctx:
        _ctx[device] = Context(device)
    return _ctx[device]


def lib():
    return load()


# ----------------------------------------------------------------------------------
# Request server (include/topo_serve.h)
# ----------------------------------------------------------------------------------
REQ_HDM, REQ_ROM = 0, 1

SERVE_EXPORTED = (
    "topo_server_create", "topo_server_destroy", "topo_server_register_mesh",
    "topo_server_register_basis", "topo_server_submit", "topo_server_wait", "topo_server_poll",
    "topo_server_stats", "topo_server_last_error",
)


class TopoRequest(C.Structure):
    _fields_ = [("kind", C.c_int32), ("mesh_id", C.c_int32), ("basis_id", C.c_int32), ("k", C.c_int32),
                ("prec", C.c_int32), ("max_refine", C.c_int32), ("maxit", C.c_int32),
                ("rho_on_device", C.c_int32), ("rtol", C.c_double), ("rho", C.c_void_p)]


class TopoResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("kind", C.c_int32), ("iters", C.c_int32), ("batch", C.c_int32),
                ("worker", C.c_int32), ("pad", C.c_int32), ("J", C.c_double), ("resnorm", C.c_double),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class TopoServeStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("jobs", C.c_int64), ("rom_jobs", C.c_int64), ("hdm_jobs", C.c_int64),
                ("mean_rom_batch", C.c_double), ("mean_hdm_batch", C.c_double), ("budget_bytes", C.c_size_t),
                ("resident_bytes", C.c_size_t), ("held_bytes", C.c_size_t), ("max_held_bytes", C.c_size_t),
                ("p50_latency_s", C.c_double * 2), ("p99_latency_s", C.c_double * 2),
                ("workers", C.c_int32), ("pad", C.c_int32)]


_SERVE_SIGS = {
    "topo_server_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_size_t, C.c_int32, C.c_int32]),
    "topo_server_destroy": (C.c_int, [_P]),
    "topo_server_register_mesh": (C.c_int, [_P, C.POINTER(TopoMesh), _P, _P, C.POINTER(C.c_int32)]),
    "topo_server_register_basis": (C.c_int, [_P, C.c_int32, _P, C.c_int32, C.c_int32, C.c_int32,
                                             C.POINTER(C.c_int32)]),
    "topo_server_submit": (C.c_int, [_P, C.POINTER(TopoRequest), C.POINTER(C.c_uint64)]),
    "topo_server_wait": (C.c_int, [_P, C.c_uint64, C.POINTER(TopoResult)]),
    "topo_server_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(TopoResult)]),
    "topo_server_stats": (C.c_int, [_P, C.POINTER(TopoServeStats)]),
    "topo_server_last_error": (C.c_char_p, [_P]),
}


def _load_serve():
    lib = load()
    if not getattr(lib, "_serve_declared", False):
        for name, (res, args) in _SERVE_SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        lib._serve_declared = True
    return lib


class Server:
    """Continuous-batching request server (worker streams, HBM-budget admission,
    fused ROM batches).  Registration takes host (numpy) arrays."""

    def __init__(self, device=0, budget_bytes=16 << 30, max_batch=16, workers=4):
        import numpy as np  # noqa: F401
        self.lib = _load_serve()
        h = C.c_void_p()
        rc = self.lib.topo_server_create(C.byref(h), device, int(budget_bytes), int(max_batch), int(workers))
        if rc != TOPO_OK:
            raise TopoError(rc, "server creation")
        self.h = h
        self._meshes = {}
        self._held = {}  # device densities of pending requests, by ticket

    def _check(self, rc, what):
        if rc != TOPO_OK:
            raise TopoError(rc, f"{what}: {self.lib.topo_server_last_error(self.h).decode()}")

    def last_error(self):
        """Message of the last failed request or call ("" if none)."""
        return self.lib.topo_server_last_error(self.h).decode()

    def close(self):
        if getattr(self, "h", None):
            self.lib.topo_server_destroy(self.h)
            self.h = None
        getattr(self, "_held", {}).clear()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def register_mesh(self, mesh, mask, f):
        import numpy as np
        m = make_mesh(mesh)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        f = np.ascontiguousarray(f, dtype=np.float64)
        mid = C.c_int32()
        rc = self.lib.topo_server_register_mesh(self.h, C.byref(m), mask.ctypes.data, f.ctypes.data, C.byref(mid))
        self._check(rc, "register_mesh")
        self._meshes[mid.value] = mesh
        return mid.value

    def register_basis(self, mesh_id, phi, kmax=None):
        import numpy as np
        phi = np.ascontiguousarray(phi)
        fp32 = 1 if phi.dtype == np.float32 else 0
        if not fp32:
            phi = np.ascontiguousarray(phi, dtype=np.float64)
        kmax = int(kmax or phi.shape[1])
        bid = C.c_int32()
        rc = self.lib.topo_server_register_basis(self.h, int(mesh_id), phi.ctypes.data, fp32, kmax,
                                                 int(phi.shape[1]), C.byref(bid))
        self._check(rc, "register_basis")
        return bid.value

    def _submit(self, req, rho):
        import numpy as np
        t = C.c_uint64()
        mesh = self._meshes.get(int(req.mesh_id))
        on_dev = hasattr(rho, "is_cuda") and rho.is_cuda
        if mesh is not None:
            ne, _, _ = mesh_sizes(make_mesh(mesh))
            n = int(rho.numel()) if on_dev else int(np.asarray(rho).size)
            if n != ne:
                raise ValueError(f"rho has {n} entries, the mesh has {ne} elements")
        if on_dev:
            import torch
            req.rho = _ptr(rho, torch.float64, "rho")
            req.rho_on_device = 1
            # the worker reads rho later on its own stream: everything queued on the
            # caller's stream (the producer of rho) must have finished, and the tensor
            # must stay alive until the request completes (released by wait / poll)
            torch.cuda.current_stream(rho.device).synchronize()
            keep = rho
        else:
            keep = np.ascontiguousarray(rho, dtype=np.float64)
            req.rho = keep.ctypes.data
            req.rho_on_device = 0
        rc = self.lib.topo_server_submit(self.h, C.byref(req), C.byref(t))
        self._check(rc, "submit")
        if on_dev:
            self._held[t.value] = keep
        return t.value

    def submit_hdm(self, mesh_id, rho, rtol=1e-10, prec=MIXED, maxit=0):
        r = TopoRequest(kind=REQ_HDM, mesh_id=int(mesh_id), basis_id=-1, k=0, prec=int(prec), max_refine=0,
                        maxit=int(maxit), rtol=float(rtol))
        return self._submit(r, rho)

    def submit_rom(self, mesh_id, basis_id, k, rho, prec=MIXED, max_refine=1):
        r = TopoRequest(kind=REQ_ROM, mesh_id=int(mesh_id), basis_id=int(basis_id), k=int(k), prec=int(prec),
                        max_refine=int(max_refine), maxit=0, rtol=0.0)
        return self._submit(r, rho)

    def wait(self, ticket):
        res = TopoResult()
        self.lib.topo_server_wait(self.h, C.c_uint64(ticket), C.byref(res))
        self._held.pop(ticket, None)
        return res.as_dict()

    def poll(self, ticket):
        res = TopoResult()
        rc = self.lib.topo_server_poll(self.h, C.c_uint64(ticket), C.byref(res))
        if rc == TOPO_EAGAIN:
            return None
        self._held.pop(ticket, None)
        return res.as_dict()

    def stats(self):
        st = TopoServeStats()
        self._check(self.lib.topo_server_stats(self.h, C.byref(st)), "stats")
        d = {f: getattr(st, f) for f, _ in st._fields_ if f not in ("pad", "p50_latency_s", "p99_latency_s")}
        d["p50_latency_s"] = {"hdm": st.p50_latency_s[0], "rom": st.p50_latency_s[1]}
        d["p99_latency_s"] = {"hdm": st.p99_latency_s[0], "rom": st.p99_latency_s[1]}
        return d
