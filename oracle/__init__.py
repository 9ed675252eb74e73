"""ctypes shim over the plain-C CPU oracle -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is built from ``oracle/oracle.c`` with gcc
(``-O2 -ffp-contract=off``, no fast-math) and shares nothing with the HIP
library.  Every function takes NumPy arrays (the seeded inputs) and returns
NumPy results.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# the same sources with OpenMP: or_cg and or_pipecg over all host threads,
# bitwise the single-thread results (timing and full-size references only)
LIB_OMP_PATH = os.path.join(HERE, "liboracle_omp.so")

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, -3
PRECOND = {"none": 0, "jacobi": 1}


SOURCES = ("oracle.c", "amg.c", "transient.c", "bicgstab.c", "piso.c")


def build(force: bool = True) -> str:
    """Compile the oracle's C sources into liboracle.so (plain C99, gcc) and
    the OpenMP timing build liboracle_omp.so."""
    srcs = [os.path.join(HERE, f) for f in SOURCES]
    newest = max(os.path.getmtime(f) for f in srcs + [os.path.join(HERE, "oracle.h")])
    for path, extra in ((LIB_PATH, []), (LIB_OMP_PATH, ["-fopenmp"])):
        if not force and os.path.exists(path) and os.path.getmtime(path) >= newest:
            continue
        tmp = path + ".tmp"
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-Wextra", *extra, "-o", tmp, *srcs, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return LIB_PATH


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("r0_norm", ctypes.c_double), ("b_norm", ctypes.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_libs = {}


def lib(omp: bool = False):
    """The single-thread oracle, or (omp=True) its OpenMP timing build."""
    path = LIB_OMP_PATH if omp else LIB_PATH
    if path not in _libs:
        if not os.path.exists(path):
            build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32 = ctypes.c_int32
        d = ctypes.c_double
        L.or_spmv.argtypes = [i32, i32, P, P, P, P, P, P, P]
        L.or_spmv.restype = None
        L.or_dot.argtypes = [i32, P, P]
        L.or_dot.restype = d
        L.or_cg.argtypes = [i32, i32, P, P, P, P, P, P, P, d, i32, i32, P, P, P, P]
        L.or_cg.restype = i32
        L.or_pipecg.argtypes = [i32, i32, P, P, P, P, P, P, P, d, i32, i32, i32, P, P]
        L.or_pipecg.restype = i32
        L.or_refine.argtypes = [i32, i32, P, P, P, P, P, P, P, d, d, i32, i32, P]
        L.or_refine.restype = i32
        L.or_mixed_reliable.argtypes = [i32, i32, P, P, P, P, P, P, P, d, i32, i32, P]
        L.or_mixed_reliable.restype = i32
        L.or_amg_setup.argtypes = [i32, i32, P, P, P, P, P, d, i32, i32, ctypes.c_uint64]
        L.or_amg_aggregate.argtypes = [i32, P, P, P, d, P, ctypes.c_uint64, i32, P]
        L.or_amg_aggregate.restype = i32
        L.or_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.or_splitmix64.restype = ctypes.c_uint64
        L.or_amg_priority.argtypes = [ctypes.c_uint64, i32, i32]
        L.or_amg_priority.restype = ctypes.c_uint64
        L.or_amg_setup.restype = P
        L.or_amg_free.argtypes = [P]
        L.or_amg_free.restype = None
        L.or_amg_refresh.argtypes = [P, i32, i32, P, P, P, P, P]
        L.or_amg_refresh.restype = i32
        L.or_amg_levels.argtypes = [P]
        L.or_amg_levels.restype = i32
        L.or_amg_level_info.argtypes = [P, i32, P, P, P, P]
        L.or_amg_level_info.restype = None
        L.or_amg_aggregates.argtypes = [P, i32, P]
        L.or_amg_aggregates.restype = None
        L.or_amg_export.argtypes = [P, i32, i32, P, P, P, P, P]
        L.or_amg_export.restype = i32
        L.or_amg_vcycle.argtypes = [P, P, P]
        L.or_amg_vcycle.restype = None
        L.or_amg_pcg.argtypes = [P, P, P, d, i32, P]
        L.or_amg_pcg.restype = i32
        L.or_amg_pipecg.argtypes = [P, P, P, d, i32, P]
        L.or_amg_pipecg.restype = i32
        L.or_assemble_transient.argtypes = [i32, i32, P, P, P, P, P, P, P, d, P, P, P, P]
        L.or_assemble_transient.restype = None
        L.or_transient_run.argtypes = [i32, i32, P, P, P, P, P, P, P, d, i32, P, d, i32, P]
        L.or_transient_run.restype = i32
        L.or_bicgstab.argtypes = [i32, i32, P, P, P, P, P, P, P, d, i32, i32, P, P, P, P]
        L.or_bicgstab.restype = i32
        L.or_adjoint_grads.argtypes = [i32, i32, P, P, P, P, P, P, P]
        L.or_adjoint_grads.restype = None
        L.or_piso_momentum.argtypes = [i32, i32, P, P, P, P, P, d, d, d, P, P, P, P, P]
        L.or_piso_momentum.restype = None
        L.or_piso_gradp.argtypes = [i32, i32, P, P, P, P, P, d, P, P]
        L.or_piso_gradp.restype = None
        L.or_piso_div.argtypes = [i32, i32, P, P, P, P]
        L.or_piso_div.restype = None
        L.or_piso_pressure_system.argtypes = [i32, i32, P, P, P, P, d, P, P, P, P, P, P, P, P, P, P, P, P]
        L.or_piso_pressure_system.restype = None
        L.or_piso_run.argtypes = [i32, i32, P, P, P, P, P, P, P, d, d, d, i32, i32, P, P, P, d, d, i32, P, P]
        L.or_piso_run.restype = i32
        L.or_threads.argtypes = []
        L.or_threads.restype = i32
        L.or_set_threads.argtypes = [i32]
        L.or_set_threads.restype = None
        _libs[path] = L
    return _libs[path]


def threads(omp: bool = True) -> int:
    """Threads the (OpenMP) build runs or_cg / or_pipecg on."""
    return int(lib(omp).or_threads())


def set_threads(t: int) -> None:
    lib(True).or_set_threads(int(t))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _Sys:
    """Arrays of one LDU system, converted once."""

    def __init__(self, n, owner, nb, diag, upper, lower=None):
        self.n = int(n)
        self.owner = _i32(owner)
        self.nb = _i32(nb)
        self.F = int(self.owner.shape[0])
        self.diag = _f64(diag)
        self.upper = _f64(upper)
        self.lower = self.upper if lower is None else _f64(lower)

    def args(self):
        return (self.n, self.F, _p(self.owner), _p(self.nb), _p(self.diag), _p(self.upper), _p(self.lower))


def system(case):
    return _Sys(case.n, case.owner, case.neighbour, case.diag, case.upper, case.lower)


def _as_sys(A):
    return A if isinstance(A, _Sys) else system(A)


def spmv(A, v):
    A = _as_sys(A)
    v = _f64(v)
    y = np.empty(A.n)
    lib().or_spmv(*A.args(), _p(v), _p(y))
    return y


def dot(a, b):
    a = _f64(a)
    b = _f64(b)
    return lib().or_dot(a.shape[0], _p(a), _p(b))


def cg(A, b, x0=None, tol=1e-8, maxit=10000, precond="jacobi", history=False, omp=False):
    """Standard PCG.  Returns (x, stats dict[, history dict]).  omp: the
    OpenMP build (bitwise the same result)."""
    A = _as_sys(A)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    st = Stats()
    m = max(int(maxit), 0) + 1
    ah = np.zeros(m) if history else None
    bh = np.zeros(m) if history else None
    rh = np.zeros(m) if history else None
    lib(omp).or_cg(*A.args(), _p(b), _p(x), float(tol), int(maxit), PRECOND[precond], ctypes.byref(st),
                   _p(ah), _p(bh), _p(rh))
    s = st.asdict()
    if history:
        k = s["iters"]
        return x, s, {"alpha": ah[:k], "beta": bh[:k], "res": rh[: k + 1]}
    return x, s


def bicgstab(A, b, x0=None, tol=1e-8, maxit=10000, precond="jacobi", history=False):
    """Preconditioned BiCGSTAB.  Returns (x, stats dict[, history dict])."""
    A = _as_sys(A)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    st = Stats()
    m = max(int(maxit), 0) + 1
    ah = np.zeros(m) if history else None
    oh = np.zeros(m) if history else None
    rh = np.zeros(m) if history else None
    lib().or_bicgstab(*A.args(), _p(b), _p(x), float(tol), int(maxit), PRECOND[precond], ctypes.byref(st),
                      _p(ah), _p(oh), _p(rh))
    s = st.asdict()
    if history:
        k = s["iters"]
        return x, s, {"alpha": ah[:k], "omega": oh[:k], "res": rh[: k + 1]}
    return x, s


def pipecg(A, b, x0=None, tol=1e-8, maxit=10000, precond="jacobi", folded=True, history=False, omp=False):
    """Pipelined PCG (literal or Jacobi-folded).  Returns (x, stats[, res]).
    omp: the OpenMP build (bitwise the same result)."""
    A = _as_sys(A)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    st = Stats()
    rh = np.zeros(max(int(maxit), 0) + 1) if history else None
    lib(omp).or_pipecg(*A.args(), _p(b), _p(x), float(tol), int(maxit), PRECOND[precond], int(bool(folded)),
                       ctypes.byref(st), _p(rh))
    s = st.asdict()
    if history:
        return x, s, rh[: s["iters"] + 1]
    return x, s


def refine(A, b, x0=None, outer_tol=1e-10, inner_tol=1e-5, max_outer=50, max_inner=20000):
    A = _as_sys(A)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    st = Stats()
    lib().or_refine(*A.args(), _p(b), _p(x), float(outer_tol), float(inner_tol), int(max_outer), int(max_inner),
                    ctypes.byref(st))
    return x, st.asdict()


def mixed_reliable(A, b, x0=None, tol=1e-10, update_every=20, maxit=100000):
    A = _as_sys(A)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    st = Stats()
    lib().or_mixed_reliable(*A.args(), _p(b), _p(x), float(tol), int(update_every), int(maxit), ctypes.byref(st))
    return x, st.asdict()


def splitmix64(seed, k):
    """Element k of the SplitMix64 sequence started at `seed` (amg.c)."""
    return int(lib().or_splitmix64(int(seed), int(k)))


def amg_priority(seed, level, i):
    """Aggregation priority of unknown i on `level`: 31 random bits, then i."""
    return int(lib().or_amg_priority(int(seed), int(level), int(i)))


def aggregate(ptr, col, val, theta, key=None, seed=1, level=0):
    """Distance-2 MIS aggregation of one CSR level: (aggregate per row, count).
    key: optional explicit priorities (distinct uint64, larger first)."""
    ptr, col, val = _i32(ptr), _i32(col), _f64(val)
    n = ptr.size - 1
    out = np.empty(max(n, 1), dtype=np.int32)
    kk = None if key is None else np.ascontiguousarray(key, dtype=np.uint64)
    na = lib().or_amg_aggregate(n, _p(ptr), _p(col), _p(val), float(theta), None if kk is None else _p(kk),
                                int(seed), int(level), _p(out))
    return out[:n], na


class AMG:
    """Smoothed-aggregation AMG hierarchy built by the oracle (amg.c)."""

    def __init__(self, A, theta=0.02, max_levels=12, coarse_size=64, seed=1):
        A = _as_sys(A)
        self._sys = A
        self.n = A.n
        h = lib().or_amg_setup(*A.args(), float(theta), int(max_levels), int(coarse_size), int(seed))
        if not h:
            raise ValueError("AMG setup failed: coarsest level not positive definite")
        self._h = ctypes.c_void_p(h)

    def refresh(self, A):
        """New coefficients of the same mesh, the aggregates kept."""
        A = _as_sys(A)
        if A.n != self.n or lib().or_amg_refresh(self._h, *A.args()) != 0:
            raise ValueError("AMG refresh failed: another size, or coarsest level not positive definite")
        self._sys = A

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_amg_free(self._h)
            self._h = None

    @property
    def levels(self):
        return lib().or_amg_levels(self._h)

    def level_info(self, l):
        n, nnz, nc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        w = ctypes.c_double()
        lib().or_amg_level_info(self._h, int(l), ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(nc),
                                ctypes.byref(w))
        return {"n": n.value, "nnz": nnz.value, "n_coarse": nc.value, "omega": w.value}

    def aggregates(self, l):
        out = np.empty(self.level_info(l)["n"], dtype=np.int32)
        lib().or_amg_aggregates(self._h, int(l), _p(out))
        return out

    def export(self, l, which="A"):
        """(indptr, indices, data, shape) of level l's A or P."""
        w = 0 if which == "A" else 1
        rows, cols = ctypes.c_int32(), ctypes.c_int32()
        nnz = lib().or_amg_export(self._h, int(l), w, ctypes.byref(rows), ctypes.byref(cols), None, None, None)
        ptr = np.empty(rows.value + 1, dtype=np.int32)
        col = np.empty(nnz, dtype=np.int32)
        val = np.empty(nnz)
        lib().or_amg_export(self._h, int(l), w, ctypes.byref(rows), ctypes.byref(cols), _p(ptr), _p(col), _p(val))
        return ptr, col, val, (rows.value, cols.value)

    def vcycle(self, b):
        b = _f64(b)
        x = np.empty(self.n)
        lib().or_amg_vcycle(self._h, _p(b), _p(x))
        return x

    def pcg(self, b, x0=None, tol=1e-8, maxit=1000, pipelined=False):
        b = _f64(b)
        x = np.zeros(self.n) if x0 is None else _f64(x0).copy()
        st = Stats()
        fn = lib().or_amg_pipecg if pipelined else lib().or_amg_pcg
        fn(self._h, _p(b), _p(x), float(tol), int(maxit), ctypes.byref(st))
        return x, st.asdict()


def assemble_transient(t, T_old, dt=None):
    """(diag, upper, b) of one implicit-Euler step of a fvcases.Transient."""
    keep = [_i32(t.owner), _i32(t.neighbour), _f64(t.k_face), _f64(t.w_face), _f64(t.vol), _f64(t.bdiag),
            _f64(t.bsrc)]
    T_old = _f64(T_old)
    diag, upper, b = np.empty(t.n), np.empty(t.F), np.empty(t.n)
    lib().or_assemble_transient(t.n, t.F, *[_p(a) for a in keep], float(t.dt if dt is None else dt), _p(T_old),
                                _p(diag), _p(upper), _p(b))
    return diag, upper, b


def transient_run(t, nsteps, T0=None, tol=1e-10, maxit=100000, dt=None):
    """Field after nsteps implicit-Euler steps, and the total CG iterations."""
    keep = [_i32(t.owner), _i32(t.neighbour), _f64(t.k_face), _f64(t.w_face), _f64(t.vol), _f64(t.bdiag),
            _f64(t.bsrc)]
    T = (_f64(t.T0) if T0 is None else _f64(T0)).copy()
    its = ctypes.c_int32()
    status = lib().or_transient_run(t.n, t.F, *[_p(a) for a in keep], float(t.dt if dt is None else dt),
                                    int(nsteps), _p(T), float(tol), int(maxit), ctypes.byref(its))
    return T, {"status": status, "iters": its.value}


def adjoint_grads(A, x, lam):
    A = _as_sys(A)
    x = _f64(x)
    lam = _f64(lam)
    gd = np.empty(A.n)
    gu = np.empty(A.F)
    gl = np.empty(A.F)
    lib().or_adjoint_grads(A.n, A.F, _p(A.owner), _p(A.nb), _p(x), _p(lam), _p(gd), _p(gu), _p(gl))
    return gd, gu, gl


def dense(A):
    """Dense matrix of an LDU system (for tiny cases)."""
    A = _as_sys(A)
    M = np.diag(A.diag.copy())
    M[A.owner, A.nb] += A.upper
    M[A.nb, A.owner] += A.lower
    return M


# ---------------------------------------------------------------- PISO (icoFoam)

def _i8(a):
    return np.ascontiguousarray(a, dtype=np.int8)


def _piso_geom(pc):
    return (_i32(pc.owner), _i32(pc.neighbour), _i8(pc.face_dir), _i8(pc.face_sgn))


def piso_momentum(pc, phi, U_old, dt=None):
    """(diag, upper, lower, bH[3][n]) of the momentum matrix of a fvcases.Piso."""
    o, m, fd, fs = _piso_geom(pc)
    phi, U_old = _f64(phi), _f64(U_old)
    bw, bl = _f64(pc.bwall), _f64(pc.blid)
    diag, bH = np.empty(pc.n), np.empty((3, pc.n))
    upper, lower = np.empty(pc.F), np.empty(pc.F)
    lib().or_piso_momentum(pc.n, pc.F, _p(o), _p(m), _p(phi), _p(bw), _p(bl), float(pc.h), float(pc.nu),
                           float(pc.dt if dt is None else dt), _p(U_old), _p(diag), _p(upper), _p(lower), _p(bH))
    return diag, upper, lower, bH


def piso_gradp(pc, p):
    o, m, fd, fs = _piso_geom(pc)
    p, bg = _f64(p), _f64(pc.bgrad)
    g = np.empty((3, pc.n))
    lib().or_piso_gradp(pc.n, pc.F, _p(o), _p(m), _p(fd), _p(fs), _p(bg), float(pc.h), _p(p), _p(g))
    return g


def piso_div(pc, phi):
    o, m, _, _ = _piso_geom(pc)
    phi = _f64(phi)
    out = np.empty(pc.n)
    lib().or_piso_div(pc.n, pc.F, _p(o), _p(m), _p(phi), _p(out))
    return out


def piso_pressure_system(pc, diag, upper, lower, bH, U):
    """One corrector's pieces: dict of HbyA, rAU, phiHbyA, cf, pdiag, pupper, prhs."""
    o, m, fd, fs = _piso_geom(pc)
    ins = [_f64(a) for a in (diag, upper, lower, bH, U)]
    out = {"HbyA": np.empty((3, pc.n)), "rAU": np.empty(pc.n), "phiHbyA": np.empty(pc.F), "cf": np.empty(pc.F),
           "pdiag": np.empty(pc.n), "pupper": np.empty(pc.F), "prhs": np.empty(pc.n)}
    lib().or_piso_pressure_system(pc.n, pc.F, _p(o), _p(m), _p(fd), _p(fs), float(pc.h), *[_p(a) for a in ins],
                                  *[_p(out[k]) for k in ("HbyA", "rAU", "phiHbyA", "cf", "pdiag", "pupper", "prhs")])
    return out


def piso_run(pc, nsteps, n_corr=2, U=None, p=None, phi=None, tol_u=1e-10, tol_p=1e-10, maxit=100000, dt=None):
    """nsteps PISO steps from (U, p, phi) (default: the case's initial
    state).  Returns (U, p, phi, status, momentum iterations, pressure
    iterations)."""
    o, m, fd, fs = _piso_geom(pc)
    U = _f64(pc.U0 if U is None else U).copy()
    p = _f64(pc.p0 if p is None else p).copy()
    phi = _f64(pc.phi0 if phi is None else phi).copy()
    bw, bl, bg = _f64(pc.bwall), _f64(pc.blid), _f64(pc.bgrad)
    iu, ip = ctypes.c_int32(), ctypes.c_int32()
    status = lib().or_piso_run(pc.n, pc.F, _p(o), _p(m), _p(fd), _p(fs), _p(bw), _p(bl), _p(bg), float(pc.h),
                               float(pc.nu), float(pc.dt if dt is None else dt), int(nsteps), int(n_corr), _p(U),
                               _p(p), _p(phi), float(tol_u), float(tol_p), int(maxit), ctypes.byref(iu),
                               ctypes.byref(ip))
    return U, p, phi, status, iu.value, ip.value
