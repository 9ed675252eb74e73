"""MI355X-native preconditioned CG / pipelined CG for finite-volume Laplacian
systems in OpenFOAM LDU form (arXiv 1505.07630, Sections 2 and 4.1).

A thin binding over libfvpcg.so (include/fvpcg.h): every function below only
marshals torch tensors (device memory) and the current HIP stream into the
C ABI; all arithmetic runs in the library's HIP kernels.  There is no CPU
fallback: without the built library, or with tensors not on the GPU, calls
raise.

    mesh = Mesh(n_cells, owner, neighbour)          # int32 cuda tensors
    A = Matrix(mesh, diag, upper, lower=None)       # float64 cuda tensors
    x, stats = solve(A, b, tol=1e-8, method="pipecg", precond="jacobi")
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (BREAKDOWN, CG, DEVICE_ERROR, FP32_COPY, INVALID_ARG, INVALID_MESH, NOT_CONVERGED, OK,  # noqa: F401
                   OUT_OF_MEMORY, PIPECG, PIPECG_LITERAL, PRECOND_JACOBI, PRECOND_NONE, STATUS_NAMES, UNSUPPORTED,
                   ExtensionMissing, Stats)

METHODS = {"cg": CG, "pipecg": PIPECG, "pipecg_literal": PIPECG_LITERAL}
PRECONDS = {"none": PRECOND_NONE, "jacobi": PRECOND_JACOBI}


class FVPCGError(RuntimeError):
    def __init__(self, code, where, message):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({code}): {message}")


def lib():
    return _lib.load()


def _check(code, where):
    if code < 0:
        msg = lib().fvpcg_last_error()
        raise FVPCGError(code, where, msg.decode(errors="replace") if msg else "")
    return code


def _stream(stream=None):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, n, name):
    """Device pointer of a contiguous CUDA tensor of `n` elements of `dtype`."""
    import torch

    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements (got {t.numel()})")
    return ctypes.c_void_p(t.data_ptr())


def fvpcg_version() -> int:
    return lib().fvpcg_version()


def fvpcg_last_error() -> str:
    m = lib().fvpcg_last_error()
    return m.decode() if m else ""


version = fvpcg_version
last_error = fvpcg_last_error


# ---------------------------------------------------------------- C-ABI names

def fvpcg_mesh_create(n_cells, owner, neighbour, stream=None):
    import torch

    F = owner.numel()
    h = ctypes.c_void_p()
    _check(lib().fvpcg_mesh_create(int(n_cells), int(F), _ptr(owner, torch.int32, F, "owner"),
                                   _ptr(neighbour, torch.int32, F, "neighbour"), _stream(stream), ctypes.byref(h)),
           "fvpcg_mesh_create")
    return h


def fvpcg_mesh_destroy(h):
    return _check(lib().fvpcg_mesh_destroy(h), "fvpcg_mesh_destroy")


def fvpcg_mesh_info(h):
    n, f, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().fvpcg_mesh_info(h, ctypes.byref(n), ctypes.byref(f), ctypes.byref(w)), "fvpcg_mesh_info")
    return n.value, f.value, w.value


def fvpcg_matrix_create(mesh_h, n, F, diag, upper, lower=None, flags=0, stream=None):
    import torch

    h = ctypes.c_void_p()
    _check(lib().fvpcg_matrix_create(mesh_h, _ptr(diag, torch.float64, n, "diag"),
                                     _ptr(upper, torch.float64, F, "upper"), _ptr(lower, torch.float64, F, "lower"),
                                     int(flags), _stream(stream), ctypes.byref(h)), "fvpcg_matrix_create")
    return h


def fvpcg_matrix_update(h, n, F, diag, upper, lower=None, stream=None):
    import torch

    return _check(lib().fvpcg_matrix_update(h, _ptr(diag, torch.float64, n, "diag"),
                                            _ptr(upper, torch.float64, F, "upper"),
                                            _ptr(lower, torch.float64, F, "lower"), _stream(stream)),
                  "fvpcg_matrix_update")


def fvpcg_matrix_destroy(h):
    return _check(lib().fvpcg_matrix_destroy(h), "fvpcg_matrix_destroy")


# ---------------------------------------------------------------- handles

class Mesh:
    """Validated LDU addressing on the device (owner < neighbour, sorted)."""

    def __init__(self, n_cells, owner, neighbour, stream=None):
        self.n = int(n_cells)
        self.F = int(owner.numel())
        self.owner = owner
        self.neighbour = neighbour
        self._h = fvpcg_mesh_create(self.n, owner, neighbour, stream)
        _, _, self.ell_width = fvpcg_mesh_info(self._h)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            fvpcg_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    """LDU coefficients on a Mesh.  lower=None means symmetric (lower = upper)."""

    def __init__(self, mesh: Mesh, diag, upper, lower=None, fp32_copy=False, stream=None):
        self.mesh = mesh  # keeps the mesh alive
        self.sym = lower is None
        self.fp32 = bool(fp32_copy)
        self._h = fvpcg_matrix_create(mesh.handle, mesh.n, mesh.F, diag, upper, lower,
                                      FP32_COPY if fp32_copy else 0, stream)

    @property
    def n(self):
        return self.mesh.n

    @property
    def handle(self):
        return self._h

    def update(self, diag, upper, lower=None, stream=None):
        fvpcg_matrix_update(self._h, self.mesh.n, self.mesh.F, diag, upper, lower, stream)

    def close(self):
        if getattr(self, "_h", None):
            fvpcg_matrix_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fvpcg_spmv(A: Matrix, v, y=None, stream=None):
    import torch

    if y is None:
        y = torch.empty_like(v)
    _check(lib().fvpcg_spmv(A.handle, _ptr(v, torch.float64, A.n, "v"), _ptr(y, torch.float64, A.n, "y"),
                            _stream(stream)), "fvpcg_spmv")
    return y


spmv = fvpcg_spmv


def fvpcg_solve(A: Matrix, b, x=None, tol=1e-8, maxit=10000, method="pipecg", precond="jacobi", stream=None):
    """Solve A x = b; x (if given) holds x0 and is overwritten.  Returns
    (x, stats dict).  Raises FVPCGError on negative status codes."""
    import torch

    if x is None:
        x = torch.zeros_like(b)
    st = Stats()
    code = lib().fvpcg_solve(A.handle, _ptr(b, torch.float64, A.n, "b"), _ptr(x, torch.float64, A.n, "x"),
                             float(tol), int(maxit), METHODS[method], PRECONDS[precond], _stream(stream),
                             ctypes.byref(st))
    _check(code, "fvpcg_solve")
    return x, st.asdict()


solve = fvpcg_solve


def fvpcg_solve_noalloc(A: Matrix, b, x, tol=1e-8, maxit=10000, method="pipecg", precond="jacobi", stream=None):
    """fvpcg_solve without any device allocation (the library's fixed work
    space, at most NOALLOC_MAX_CELLS cells): x holds x0 and is overwritten.
    Returns (x, stats dict)."""
    import torch

    st = Stats()
    code = lib().fvpcg_solve_noalloc(A.handle, _ptr(b, torch.float64, A.n, "b"), _ptr(x, torch.float64, A.n, "x"),
                                     float(tol), int(maxit), METHODS[method], PRECONDS[precond], _stream(stream),
                                     ctypes.byref(st))
    _check(code, "fvpcg_solve_noalloc")
    return x, st.asdict()


solve_noalloc = fvpcg_solve_noalloc
NOALLOC_MAX_CELLS = 1048576


def fvpcg_solve_bicgstab(A: Matrix, b, x=None, tol=1e-8, maxit=10000, precond="jacobi", stream=None):
    """BiCGSTAB for A x = b (A may be non-symmetric); x (if given) holds x0
    and is overwritten.  Returns (x, stats dict).  Raises FVPCGError on
    negative status codes."""
    import torch

    if x is None:
        x = torch.zeros_like(b)
    st = Stats()
    code = lib().fvpcg_solve_bicgstab(A.handle, _ptr(b, torch.float64, A.n, "b"), _ptr(x, torch.float64, A.n, "x"),
                                      float(tol), int(maxit), PRECONDS[precond], _stream(stream), ctypes.byref(st))
    _check(code, "fvpcg_solve_bicgstab")
    return x, st.asdict()


solve_bicgstab = fvpcg_solve_bicgstab


def fvpcg_solve_bicgstab_multi(A: Matrix, b, x=None, tol=1e-8, maxit=10000, precond="jacobi", stream=None):
    """BiCGSTAB for nrhs = b.shape[0] (1..4) right-hand sides with the same
    matrix, solved together; b and x are (nrhs, n) float64 CUDA tensors (x,
    if given, holds x0 and is overwritten).  Returns (x, [stats per
    component]).  Raises FVPCGError if a component broke down."""
    import torch

    if b.dim() != 2:
        raise ValueError("b must have shape (nrhs, n)")
    nr = int(b.shape[0])
    if x is None:
        x = torch.zeros_like(b)
    st = (Stats * max(nr, 1))()
    code = lib().fvpcg_solve_bicgstab_multi(A.handle, nr, _ptr(b, torch.float64, nr * A.n, "b"),
                                            _ptr(x, torch.float64, nr * A.n, "x"), float(tol), int(maxit),
                                            PRECONDS[precond], _stream(stream), st)
    _check(code, "fvpcg_solve_bicgstab_multi")
    return x, [st[k].asdict() for k in range(nr)]


solve_bicgstab_multi = fvpcg_solve_bicgstab_multi


def fvpcg_solve_mixed(A: Matrix, b, x=None, outer_tol=1e-10, inner_tol=1e-5, max_outer=30, max_inner=20000,
                      stream=None):
    import torch

    if x is None:
        x = torch.zeros_like(b)
    st = Stats()
    code = lib().fvpcg_solve_mixed(A.handle, _ptr(b, torch.float64, A.n, "b"), _ptr(x, torch.float64, A.n, "x"),
                                   float(outer_tol), float(inner_tol), int(max_outer), int(max_inner),
                                   _stream(stream), ctypes.byref(st))
    _check(code, "fvpcg_solve_mixed")
    return x, st.asdict()


solve_mixed = fvpcg_solve_mixed


def fvpcg_solve_mixed_reliable(A: Matrix, b, x=None, tol=1e-10, update_every=10, maxit=100000, stream=None):
    """FP32 pipelined Jacobi-CG whose recurrences are re-anchored to the FP64
    residual every `update_every` iterations (reliable updates)."""
    import torch

    if x is None:
        x = torch.zeros_like(b)
    st = Stats()
    code = lib().fvpcg_solve_mixed_reliable(A.handle, _ptr(b, torch.float64, A.n, "b"),
                                            _ptr(x, torch.float64, A.n, "x"), float(tol), int(update_every),
                                            int(maxit), _stream(stream), ctypes.byref(st))
    _check(code, "fvpcg_solve_mixed_reliable")
    return x, st.asdict()


solve_mixed_reliable = fvpcg_solve_mixed_reliable


def fvpcg_solve_backward(A: Matrix, x, g, want=("b", "diag", "upper", "lower"), tol=1e-10, maxit=10000,
                         method="pipecg", precond="jacobi", stream=None):
    """Adjoint of a solve: returns (dict of gradients, stats)."""
    import torch

    n, F = A.mesh.n, A.mesh.F
    out = {}
    for k in want:
        if k in ("b", "diag"):
            out[k] = torch.empty(n, dtype=torch.float64, device=x.device)
        elif k == "upper" or (k == "lower" and not A.sym):
            out[k] = torch.empty(F, dtype=torch.float64, device=x.device)
    st = Stats()
    code = lib().fvpcg_solve_backward(A.handle, _ptr(x, torch.float64, n, "x"), _ptr(g, torch.float64, n, "g"),
                                      _ptr(out.get("b"), torch.float64, n, "grad_b"),
                                      _ptr(out.get("diag"), torch.float64, n, "grad_diag"),
                                      _ptr(out.get("upper"), torch.float64, F, "grad_upper"),
                                      _ptr(out.get("lower"), torch.float64, F, "grad_lower"), float(tol), int(maxit),
                                      METHODS[method], PRECONDS[precond], _stream(stream), ctypes.byref(st))
    _check(code, "fvpcg_solve_backward")
    return out, st.asdict()


solve_backward = fvpcg_solve_backward


# ---------------------------------------------------------------- batched

class Batch:
    """nsys independent LDU systems, concatenated; owner/neighbour are local
    to each system; cell_off/face_off are host int sequences (nsys+1)."""

    def __init__(self, cell_off, face_off, owner, neighbour, diag, upper, lower=None, stream=None):
        import numpy as np
        import torch

        self.cell_off = np.ascontiguousarray(np.asarray(cell_off), dtype=np.int32)
        self.face_off = np.ascontiguousarray(np.asarray(face_off), dtype=np.int32)
        self.nsys = int(self.cell_off.shape[0] - 1)
        self.n = int(self.cell_off[-1])
        self.F = int(self.face_off[-1])
        self.sym = lower is None
        h = ctypes.c_void_p()
        _check(lib().fvpcg_batch_create(
            self.nsys, self.cell_off.ctypes.data_as(ctypes.c_void_p), self.face_off.ctypes.data_as(ctypes.c_void_p),
            _ptr(owner, torch.int32, self.F, "owner"), _ptr(neighbour, torch.int32, self.F, "neighbour"),
            _ptr(diag, torch.float64, self.n, "diag"), _ptr(upper, torch.float64, self.F, "upper"),
            _ptr(lower, torch.float64, self.F, "lower"), 0, _stream(stream), ctypes.byref(h)), "fvpcg_batch_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().fvpcg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fvpcg_batch_create(cell_off, face_off, owner, neighbour, diag, upper, lower=None, stream=None) -> Batch:
    """The C-ABI name of `Batch(...)`: the handle is `.handle`, released by
    `fvpcg_batch_destroy` (or `.close()`)."""
    return Batch(cell_off, face_off, owner, neighbour, diag, upper, lower, stream)


def fvpcg_batch_destroy(B: Batch):
    B.close()
    return OK


def fvpcg_solve_batched(B: Batch, b, x=None, tol=1e-8, maxit=10000, method="pipecg", precond="jacobi",
                        stream=None):
    """Returns (x, list of per-system stats dicts, overall status code)."""
    import torch

    if x is None:
        x = torch.zeros_like(b)
    st = (Stats * B.nsys)()
    code = lib().fvpcg_solve_batched(B.handle, _ptr(b, torch.float64, B.n, "b"), _ptr(x, torch.float64, B.n, "x"),
                                     float(tol), int(maxit), METHODS[method], PRECONDS[precond], _stream(stream),
                                     ctypes.cast(st, ctypes.POINTER(Stats)))
    _check(code, "fvpcg_solve_batched")
    return x, [s.asdict() for s in st], code


solve_batched = fvpcg_solve_batched


def fvpcg_solve_batched_backward(B: Batch, x, g, tol=1e-10, maxit=10000, method="pipecg", precond="jacobi",
                                 stream=None):
    import torch

    out = {"b": torch.empty(B.n, dtype=torch.float64, device=x.device),
           "diag": torch.empty(B.n, dtype=torch.float64, device=x.device),
           "upper": torch.empty(B.F, dtype=torch.float64, device=x.device)}
    if not B.sym:
        out["lower"] = torch.empty(B.F, dtype=torch.float64, device=x.device)
    st = (Stats * B.nsys)()
    code = lib().fvpcg_solve_batched_backward(
        B.handle, _ptr(x, torch.float64, B.n, "x"), _ptr(g, torch.float64, B.n, "g"),
        _ptr(out["b"], torch.float64, B.n, "grad_b"), _ptr(out["diag"], torch.float64, B.n, "grad_diag"),
        _ptr(out["upper"], torch.float64, B.F, "grad_upper"), _ptr(out.get("lower"), torch.float64, B.F, "grad_lower"),
        float(tol), int(maxit), METHODS[method], PRECONDS[precond], _stream(stream),
        ctypes.cast(st, ctypes.POINTER(Stats)))
    _check(code, "fvpcg_solve_batched_backward")
    return out, [s.asdict() for s in st], code


solve_batched_backward = fvpcg_solve_batched_backward


# ---------------------------------------------------------------- transient diffusion

def fvpcg_assemble_transient(mesh: Mesh, k_face, w_face, vol, bdiag, bsrc, dt, T_old, diag=None, upper=None, b=None,
                             stream=None):
    """(diag, upper, b) of one implicit-Euler step of the heat equation."""
    import torch

    n, F = mesh.n, mesh.F
    diag = torch.empty_like(vol) if diag is None else diag
    upper = torch.empty_like(k_face) if upper is None else upper
    b = torch.empty_like(vol) if b is None else b
    _check(lib().fvpcg_assemble_transient(mesh.handle, _ptr(k_face, torch.float64, F, "k_face"),
                                          _ptr(w_face, torch.float64, F, "w_face"), _ptr(vol, torch.float64, n, "vol"),
                                          _ptr(bdiag, torch.float64, n, "bdiag"), _ptr(bsrc, torch.float64, n, "bsrc"),
                                          float(dt), _ptr(T_old, torch.float64, n, "T_old"),
                                          _ptr(diag, torch.float64, n, "diag"), _ptr(upper, torch.float64, F, "upper"),
                                          _ptr(b, torch.float64, n, "b"), _stream(stream)), "fvpcg_assemble_transient")
    return diag, upper, b


assemble_transient = fvpcg_assemble_transient


def fvpcg_transient_run(A: Matrix, k_face, w_face, vol, bdiag, bsrc, dt, nsteps, T, tol=1e-8, maxit=100000,
                        method="pipecg", stream=None):
    """Advance T (in place) by nsteps implicit-Euler steps; returns (T, stats)."""
    import torch

    n, F = A.n, A.mesh.F
    st = Stats()
    code = lib().fvpcg_transient_run(A.handle, _ptr(k_face, torch.float64, F, "k_face"),
                                     _ptr(w_face, torch.float64, F, "w_face"), _ptr(vol, torch.float64, n, "vol"),
                                     _ptr(bdiag, torch.float64, n, "bdiag"), _ptr(bsrc, torch.float64, n, "bsrc"),
                                     float(dt), int(nsteps), _ptr(T, torch.float64, n, "T"), float(tol), int(maxit),
                                     METHODS[method], _stream(stream), ctypes.byref(st))
    _check(code, "fvpcg_transient_run")
    return T, st.asdict()


transient_run = fvpcg_transient_run


# ---------------------------------------------------------------- icoFoam PISO

PSOLVERS = {"jacobi": _lib.PSOLVER_JACOBI, "amg": _lib.PSOLVER_AMG}


class Piso:
    """icoFoam's PISO step on a Mesh of cubes of side h (fvpcg_piso_*):
    face_dir/face_sgn int8[F], bwall/blid [n], bgrad [3][n] device tensors
    (copied); the Mesh must outlive it."""

    def __init__(self, mesh: Mesh, face_dir, face_sgn, bwall, blid, bgrad, h, nu, pressure_solver="jacobi",
                 stream=None):
        import torch

        n, F = mesh.n, mesh.F
        h_ = ctypes.c_void_p()
        _check(lib().fvpcg_piso_create(
            mesh.handle, _ptr(face_dir, torch.int8, F, "face_dir"), _ptr(face_sgn, torch.int8, F, "face_sgn"),
            _ptr(bwall, torch.float64, n, "bwall"), _ptr(blid, torch.float64, n, "blid"),
            _ptr(bgrad, torch.float64, 3 * n, "bgrad"), float(h), float(nu), PSOLVERS[pressure_solver],
            _stream(stream), ctypes.byref(h_)), "fvpcg_piso_create")
        self._h = h_
        self.mesh = mesh

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().fvpcg_piso_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fvpcg_piso_create(mesh, face_dir, face_sgn, bwall, blid, bgrad, h, nu, pressure_solver="jacobi", stream=None):
    return Piso(mesh, face_dir, face_sgn, bwall, blid, bgrad, h, nu, pressure_solver, stream)


def fvpcg_piso_destroy(ps: Piso):
    ps.close()
    return OK


def fvpcg_piso_run(ps: Piso, dt, nsteps, U, p, phi, n_corr=2, tol_u=1e-8, tol_p=1e-8, maxit=100000, stream=None):
    """nsteps PISO steps; U [3][n], p [n], phi [F] device tensors updated in
    place.  Returns (momentum stats, pressure stats)."""
    import torch

    n, F = ps.mesh.n, ps.mesh.F
    st = (Stats * 2)()
    code = lib().fvpcg_piso_run(ps.handle, float(dt), int(nsteps), int(n_corr), _ptr(U, torch.float64, 3 * n, "U"),
                                _ptr(p, torch.float64, n, "p"), _ptr(phi, torch.float64, F, "phi"), float(tol_u),
                                float(tol_p), int(maxit), _stream(stream), ctypes.cast(st, ctypes.POINTER(Stats)))
    _check(code, "fvpcg_piso_run")
    return st[0].asdict(), st[1].asdict()


piso_run = fvpcg_piso_run


# ---------------------------------------------------------------- AMG

class AMG:
    """Smoothed-aggregation AMG hierarchy of a (symmetric) Matrix; the Matrix
    must outlive it."""

    def __init__(self, A: Matrix, theta=0.02, max_levels=12, coarse_size=64, seed=1, stream=None):
        h = ctypes.c_void_p()
        _check(lib().fvpcg_amg_create(A.handle, float(theta), int(max_levels), int(coarse_size), int(seed),
                                      _stream(stream), ctypes.byref(h)), "fvpcg_amg_create")
        self._h = h
        self.A = A
        self.n = A.n

    @property
    def handle(self):
        return self._h

    @property
    def levels(self):
        lv = ctypes.c_int32()
        _check(lib().fvpcg_amg_info(self._h, -1, ctypes.byref(lv), None, None), "fvpcg_amg_info")
        return lv.value

    def refresh(self, stream=None):
        """The hierarchy for the matrix's current coefficients (after an
        update), aggregates and patterns kept."""
        _check(lib().fvpcg_amg_refresh(self._h, _stream(stream)), "fvpcg_amg_refresh")

    def level_info(self, level):
        lv, n, nnz = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().fvpcg_amg_info(self._h, int(level), ctypes.byref(lv), ctypes.byref(n), ctypes.byref(nnz)),
               "fvpcg_amg_info")
        return {"n": n.value, "nnz": nnz.value}

    def aggregates(self, level):
        import numpy as np

        out = np.empty(self.level_info(level)["n"], dtype=np.int32)
        _check(lib().fvpcg_amg_aggregates(self._h, int(level), out.ctypes.data_as(ctypes.c_void_p)),
               "fvpcg_amg_aggregates")
        return out

    def export(self, level, which="A"):
        """(indptr, indices, data, shape) of level `level`'s A (levels >= 1),
        P or R, copied to the host."""
        import numpy as np

        w = {"A": 0, "P": 1, "R": 2}[which]
        rows, cols, nnz = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        args = (self._h, int(level), w, ctypes.byref(rows), ctypes.byref(cols), ctypes.byref(nnz))
        _check(lib().fvpcg_amg_export(*args, None, None, None), "fvpcg_amg_export")
        ptr = np.empty(rows.value + 1, dtype=np.int32)
        col = np.empty(max(nnz.value, 1), dtype=np.int32)
        val = np.empty(max(nnz.value, 1))
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().fvpcg_amg_export(*args, vp(ptr), vp(col), vp(val)), "fvpcg_amg_export")
        return ptr, col[:nnz.value], val[:nnz.value], (rows.value, cols.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().fvpcg_amg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fvpcg_amg_create(A: Matrix, theta=0.02, max_levels=12, coarse_size=64, seed=1, stream=None) -> AMG:
    return AMG(A, theta, max_levels, coarse_size, seed, stream)


def fvpcg_amg_destroy(M: AMG):
    M.close()
    return OK


def fvpcg_amg_info(M: AMG, level=0):
    return dict(M.level_info(level), levels=M.levels)


def fvpcg_amg_aggregates(M: AMG, level=0):
    return M.aggregates(level)


def fvpcg_amg_export(M: AMG, level=1, which="A"):
    return M.export(level, which)


def fvpcg_amg_refresh(amg, stream=None):
    """The hierarchy for the matrix's current coefficients (AMG.refresh)."""
    amg.refresh(stream)


amg_refresh = fvpcg_amg_refresh


def fvpcg_amg_apply(M: AMG, r, z=None, stream=None):
    """z = M^-1 r (one V-cycle)."""
    import torch

    if z is None:
        z = torch.empty_like(r)
    _check(lib().fvpcg_amg_apply(M.handle, _ptr(r, torch.float64, M.n, "r"), _ptr(z, torch.float64, M.n, "z"),
                                 _stream(stream)), "fvpcg_amg_apply")
    return z


amg_apply = fvpcg_amg_apply


def fvpcg_solve_amg(M: AMG, b, x=None, tol=1e-8, maxit=1000, method="cg", stream=None):
    """CG preconditioned by one AMG cycle: method "cg" (standard form) or
    "pipecg" (pipelined, literal recurrences)."""
    import torch

    if x is None:
        x = torch.zeros_like(b)
    st = Stats()
    code = lib().fvpcg_solve_amg(M.handle, _ptr(b, torch.float64, M.n, "b"), _ptr(x, torch.float64, M.n, "x"),
                                 float(tol), int(maxit), METHODS[method], _stream(stream), ctypes.byref(st))
    _check(code, "fvpcg_solve_amg")
    return x, st.asdict()


solve_amg = fvpcg_solve_amg


def fvpcg_stream_calibrate(bytes_per_array=0, stream=None):
    c, t = ctypes.c_double(), ctypes.c_double()
    _check(lib().fvpcg_stream_calibrate(_stream(stream), int(bytes_per_array), ctypes.byref(c), ctypes.byref(t)),
           "fvpcg_stream_calibrate")
    return {"copy_gbs": c.value, "triad_gbs": t.value}


stream_calibrate = fvpcg_stream_calibrate


def fvpcg_stream_mix(n_read, n_write, bytes_per_array=0, stream=None):
    """Attainable GB/s of a kernel streaming n_read arrays in and n_write out."""
    g = ctypes.c_double()
    _check(lib().fvpcg_stream_mix(_stream(stream), int(bytes_per_array), int(n_read), int(n_write), ctypes.byref(g)),
           "fvpcg_stream_mix")
    return g.value


stream_mix = fvpcg_stream_mix

from .autograd import FVSolve, fv_solve  # noqa: E402,F401
