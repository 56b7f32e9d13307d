"""Python face of the CPU oracle (``libccmg_oracle.so``, plain C, FP64).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The solver package never imports this.

Every function works on numpy arrays laid out [nz][ny][nx] (x fastest) and
mirrors one step of the cell-centered multigrid method of Bartuschat & Ruede
(arXiv:1410.6609); the C source cites the section each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "ccmg_oracle.c"), os.path.join(_HERE, "levelops.inc")]
# CCMG_ORACLE_LIB names another build of the same sources (the sanitizer run)
LIB_PATH = os.environ.get("CCMG_ORACLE_LIB") or os.path.join(_HERE, "libccmg_oracle.so")
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]

OK, E_ARG, E_NONFINITE, E_NOCONV = 0, -1, -5, -6


def build(force: bool = True, out: Optional[str] = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (no FP contraction, OpenMP).  sanitize: with
    AddressSanitizer and UndefinedBehaviorSanitizer (UB aborts), into `out`."""
    out = out or LIB_PATH
    if not force and os.path.exists(out):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-Wall", "-Wno-unknown-pragmas", "-Wno-unused-function",
           *(SANITIZE_FLAGS if sanitize else []), "-o", tmp, _SRC[0], "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, out)
    return out


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_longlong)
        I, D = ctypes.c_int, ctypes.c_double
        sig = {
            "or_num_threads": ([], I),
            "or_set_num_threads": ([I], None),
            "or_diag_at": ([I, I, I, ip, I, I, I], I),
            "or_apply": ([I, I, I, D, I, ip, dp, dp], None),
            "or_residual": ([I, I, I, D, I, ip, dp, dp, dp], None),
            "or_norm2": ([ctypes.c_longlong, dp], D),
            "or_rbgs_sweep": ([I, I, I, D, I, ip, dp, dp], None),
            "or_restrict": ([I, I, I, dp, dp], None),
            "or_prolong_add": ([I, I, I, dp, D, dp], None),
            "or_cg": ([I, I, I, D, I, ip, dp, dp, D, I], I),
            "or_fold": ([I, I, I, D, ip, dp, dp, dp], None),
            "or_deposit": ([I, I, I, D, I, dp, dp, dp, D, dp, lp], None),
            "or_dq": ([I, I, I, D, I, dp, dp, D, dp, dp], None),
            "or_fold_field": ([I, I, I, D, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_void_p), dp, dp], None),
            "or_deposit_sub": ([I, I, I, D, I, dp, dp, dp, D, I, I, dp, dp], None),
            "or_dq_sub": ([I, I, I, D, I, dp, dp, D, I, I, dp, dp], None),
            "or_gradient": ([I, I, I, D, ip, dp, ctypes.POINTER(ctypes.c_void_p), dp, dp], None),
            "or_coulomb": ([I, I, I, D, ip, dp, ctypes.POINTER(ctypes.c_void_p), dp, I, dp, dp, dp, I, I, dp],
                           None),
            "or_vc_faces": ([I, I, I, ip, dp, dp, dp, dp], None),
            "or_vc_coarsen": ([I, I, I, dp, dp, dp, dp, dp, dp], None),
            "or_vc_apply": ([I, I, I, D, I, ip, dp, dp, dp, dp, dp], None),
            "or_vc_rbgs_sweep": ([I, I, I, D, I, ip, dp, dp, dp, dp, dp, I], None),
            "or_vc_fold": ([I, I, I, D, ip, dp, ctypes.POINTER(ctypes.c_void_p), dp, dp, dp, dp, dp], None),
            "or_vc_solve": ([I, I, I, D, ip, I, I, I, D, D, I, dp, dp, dp, D, I, dp, ip], I),
            "or_coulomb_adjoint": ([I, I, I, D, ip, dp, ctypes.POINTER(ctypes.c_void_p), dp, I, dp, dp, dp, I, I,
                                    dp, dp, dp], None),
            "or_solve": ([I, I, I, D, ip, I, I, I, D, D, I, dp, dp, D, I, dp, ip], I),
            "or_solve_ir": ([I, I, I, D, ip, I, I, I, D, D, I, I, dp, dp, D, I, dp, ip], I),
            "or_pb_apply": ([I, I, I, D, I, ip, D, dp, dp], None),
            "or_pb_rbgs_sweep": ([I, I, I, D, I, ip, D, dp, dp], None),
            "or_pb_cg": ([I, I, I, D, I, ip, D, dp, dp, D, I], I),
            "or_pb_solve": ([I, I, I, D, ip, I, I, I, D, D, I, D, dp, dp, D, I, dp, ip], I),
            "or_pb_nl_residual": ([I, I, I, D, ip, D, dp, dp, dp], None),
            "or_pb_nl_solve": ([I, I, I, D, ip, I, I, I, D, D, I, D, I, dp, dp, D, I, dp, ip], I),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _kinds(kinds: Sequence[int]):
    arr = (ctypes.c_int * 6)(*[int(k) for k in kinds])
    return arr


def _shape(a: np.ndarray) -> Tuple[int, int, int]:
    nz, ny, nx = a.shape
    return nx, ny, nz


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))


def diag_at(shape, kinds, i, j, k) -> int:
    nx, ny, nz = shape
    return lib().or_diag_at(nx, ny, nz, _kinds(kinds), i, j, k)


def apply(phi: np.ndarray, h: float, kinds, level: int = 0) -> np.ndarray:
    """A_l phi on a level of spacing 2^l h (operator scale 1/(2^l h^2))."""
    phi = _f64(phi)
    out = np.empty_like(phi)
    nx, ny, nz = _shape(phi)
    lib().or_apply(nx, ny, nz, h, level, _kinds(kinds), _dp(phi), _dp(out))
    return out


def residual(phi, b, h, kinds, level: int = 0) -> np.ndarray:
    phi, b = _f64(phi), _f64(b)
    r = np.empty_like(phi)
    nx, ny, nz = _shape(phi)
    lib().or_residual(nx, ny, nz, h, level, _kinds(kinds), _dp(phi), _dp(b), _dp(r))
    return r


def norm2(v) -> float:
    v = _f64(v)
    return lib().or_norm2(v.size, _dp(v))


def rbgs_sweep(phi, b, h, kinds, level: int = 0, sweeps: int = 1) -> np.ndarray:
    phi = _f64(phi).copy()
    b = _f64(b)
    nx, ny, nz = _shape(phi)
    for _ in range(sweeps):
        lib().or_rbgs_sweep(nx, ny, nz, h, level, _kinds(kinds), _dp(phi), _dp(b))
    return phi


def restrict(r) -> np.ndarray:
    r = _f64(r)
    nx, ny, nz = _shape(r)
    out = np.empty((nz // 2, ny // 2, nx // 2))
    lib().or_restrict(nx, ny, nz, _dp(r), _dp(out))
    return out


def prolong_add(phi_fine, e_coarse, omega: float) -> np.ndarray:
    phi = _f64(phi_fine).copy()
    e = _f64(e_coarse)
    nx, ny, nz = _shape(phi)
    lib().or_prolong_add(nx, ny, nz, _dp(e), omega, _dp(phi))
    return phi


def cg(b, h, kinds, level: int = 0, rtol: float = 1e-13, maxit: Optional[int] = None):
    b = _f64(b)
    x = np.zeros_like(b)
    nx, ny, nz = _shape(b)
    maxit = 2 * b.size if maxit is None else maxit
    it = lib().or_cg(nx, ny, nz, h, level, _kinds(kinds), _dp(b), _dp(x), rtol, maxit)
    return x, it


def fold(f, h, kinds, values) -> np.ndarray:
    f = _f64(f)
    b = np.empty_like(f)
    nx, ny, nz = _shape(f)
    vals = (ctypes.c_double * 6)(*[float(v) for v in values])
    lib().or_fold(nx, ny, nz, h, _kinds(kinds), vals, _dp(f), _dp(b))
    return b


def fold_field(f, h, kinds, values, faces) -> np.ndarray:
    """Fold with per-cell boundary values; faces[fc] is None (constant
    values[fc]) or an array of the face's shape: x faces (nz, ny), y faces
    (nz, nx), z faces (ny, nx)."""
    f = _f64(f)
    b = np.empty_like(f)
    nx, ny, nz = _shape(f)
    shapes = [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2
    keep = [None if a is None else _f64(a).reshape(shapes[i]) for i, a in enumerate(faces)]
    ptrs = (ctypes.c_void_p * 6)(*[None if a is None else a.ctypes.data for a in keep])
    vals = (ctypes.c_double * 6)(*[float(v) for v in values])
    lib().or_fold_field(nx, ny, nz, h, _kinds(kinds), vals, ptrs, _dp(f), _dp(b))
    return b


def _faces(shape, faces):
    nx, ny, nz = shape
    shapes = [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2
    faces = faces if faces is not None else [None] * 6
    keep = [None if a is None else _f64(a).reshape(shapes[i]) for i, a in enumerate(faces)]
    return keep, (ctypes.c_void_p * 6)(*[None if a is None else a.ctypes.data for a in keep])


def gradient(phi, h, kinds, values, faces=None) -> np.ndarray:
    """[3, nz, ny, nx]: D3Q19 gradient inside, D3Q7 with boundary ghosts on the boundary layer."""
    phi = _f64(phi)
    nx, ny, nz = _shape(phi)
    out = np.empty((3, nz, ny, nx))
    keep, ptrs = _faces((nx, ny, nz), faces)
    vals = (ctypes.c_double * 6)(*[float(v) for v in values])
    lib().or_gradient(nx, ny, nz, h, _kinds(kinds), vals, ptrs, _dp(phi), _dp(out))
    return out


def coulomb(phi, h, kinds, values, centers, radii, q, subsample: int = 1, mode: int = 0, faces=None) -> np.ndarray:
    """Electrostatic force per sphere, [n, 3]."""
    phi = _f64(phi)
    nx, ny, nz = _shape(phi)
    centers, radii, q = _f64(centers).reshape(-1, 3), _f64(radii), _f64(q)
    out = np.zeros((radii.shape[0], 3))
    keep, ptrs = _faces((nx, ny, nz), faces)
    vals = (ctypes.c_double * 6)(*[float(v) for v in values])
    lib().or_coulomb(nx, ny, nz, h, _kinds(kinds), vals, ptrs, _dp(phi), radii.shape[0], _dp(centers), _dp(radii),
                     _dp(q), subsample, mode, _dp(out))
    return out


def coulomb_adjoint(phi, h, kinds, values, centers, radii, q, gF, subsample: int = 1, mode: int = 0, faces=None):
    """(mu = dL/dphi field, direct dL/dq_s at fixed phi) for a loss with dL/dF = gF [n, 3]."""
    phi = _f64(phi)
    nx, ny, nz = _shape(phi)
    centers, radii, q = _f64(centers).reshape(-1, 3), _f64(radii), _f64(q)
    gF = _f64(gF).reshape(-1, 3)
    mu = np.empty_like(phi)
    direct = np.zeros(radii.shape[0])
    keep, ptrs = _faces((nx, ny, nz), faces)
    vals = (ctypes.c_double * 6)(*[float(v) for v in values])
    lib().or_coulomb_adjoint(nx, ny, nz, h, _kinds(kinds), vals, ptrs, _dp(phi), radii.shape[0], _dp(centers),
                             _dp(radii), _dp(q), subsample, mode, _dp(gF), _dp(mu), _dp(direct))
    return mu, direct


def deposit(shape, h, centers, radii, q, eps: float = 1.0):
    """Returns (f = rho/eps [nz][ny][nx], n_s per sphere)."""
    nx, ny, nz = shape
    centers, radii, q = _f64(centers).reshape(-1, 3), _f64(radii), _f64(q)
    n = radii.shape[0]
    f = np.empty((nz, ny, nx))
    counts = np.zeros(n, dtype=np.int64)
    lib().or_deposit(nx, ny, nz, h, n, _dp(centers), _dp(radii), _dp(q), eps, _dp(f),
                     counts.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
    return f, counts


def dq(lam, h, centers, radii, eps: float = 1.0) -> np.ndarray:
    lam = _f64(lam)
    nx, ny, nz = _shape(lam)
    centers, radii = _f64(centers).reshape(-1, 3), _f64(radii)
    out = np.zeros(radii.shape[0])
    lib().or_dq(nx, ny, nz, h, radii.shape[0], _dp(centers), _dp(radii), eps, _dp(lam), _dp(out))
    return out


def deposit_sub(shape, h, centers, radii, q, eps: float = 1.0, subsample: int = 2, mode: int = 0):
    """Sub-sampled deposition; returns (f = rho/eps, W_s = summed overlap ratios)."""
    nx, ny, nz = shape
    centers, radii, q = _f64(centers).reshape(-1, 3), _f64(radii), _f64(q)
    n = radii.shape[0]
    f = np.empty((nz, ny, nx))
    wsum = np.zeros(n)
    lib().or_deposit_sub(nx, ny, nz, h, n, _dp(centers), _dp(radii), _dp(q), eps, subsample, mode, _dp(f),
                         _dp(wsum))
    return f, wsum


def dq_sub(lam, h, centers, radii, eps: float = 1.0, subsample: int = 2, mode: int = 0) -> np.ndarray:
    lam = _f64(lam)
    nx, ny, nz = _shape(lam)
    centers, radii = _f64(centers).reshape(-1, 3), _f64(radii)
    out = np.zeros(radii.shape[0])
    lib().or_dq_sub(nx, ny, nz, h, radii.shape[0], _dp(centers), _dp(radii), eps, subsample, mode, _dp(lam),
                    _dp(out))
    return out


def default_cg_maxit(shape, levels) -> int:
    nx, ny, nz = shape
    d = 1 << (levels - 1)
    return 2 * (nx // d) * (ny // d) * (nz // d)


def solve(b, h, kinds, levels, nu1=2, nu2=2, omega=2.0, rtol=1e-10, max_cycles=100,
          phi0=None, cg_rtol=1e-13, cg_maxit=None):
    """FP64 multigrid on the folded RHS b. Returns (phi, history, status)."""
    b = _f64(b)
    phi = np.zeros_like(b) if phi0 is None else _f64(phi0).copy()
    nx, ny, nz = _shape(b)
    hist = np.zeros(max_cycles + 1)
    cyc = ctypes.c_int(0)
    cg_maxit = default_cg_maxit((nx, ny, nz), levels) if cg_maxit is None else cg_maxit
    st = lib().or_solve(nx, ny, nz, h, _kinds(kinds), levels, nu1, nu2, omega, cg_rtol, cg_maxit,
                        _dp(b), _dp(phi), rtol, max_cycles, _dp(hist), ctypes.byref(cyc))
    if st == E_ARG:
        raise ValueError("oracle: invalid hierarchy")
    return phi, hist[: cyc.value + 1].copy(), st


def solve_ir(b, h, kinds, levels, inner=2, nu1=2, nu2=2, omega=2.0, rtol=1e-10, max_outer=100,
             phi0=None, cg_rtol=1e-6, cg_maxit=None):
    """FP32-in-FP64 iterative refinement. Returns (phi, history, status).  cg_rtol is the
    coarsest CG's tolerance inside the FP32 cycles (the refinement's only CG): 1e-6 by
    default, as the GPU's, since an FP32 correction carries about seven digits."""
    b = _f64(b)
    phi = np.zeros_like(b) if phi0 is None else _f64(phi0).copy()
    nx, ny, nz = _shape(b)
    hist = np.zeros(max_outer + 1)
    cyc = ctypes.c_int(0)
    cg_maxit = default_cg_maxit((nx, ny, nz), levels) if cg_maxit is None else cg_maxit
    st = lib().or_solve_ir(nx, ny, nz, h, _kinds(kinds), levels, nu1, nu2, omega, cg_rtol, cg_maxit,
                           inner, _dp(b), _dp(phi), rtol, max_outer, _dp(hist), ctypes.byref(cyc))
    if st == E_ARG:
        raise ValueError("oracle: invalid hierarchy")
    return phi, hist[: cyc.value + 1].copy(), st


def solve_problem(f, h, kinds, values, levels, **kw):
    """Fold the boundary conditions into f and solve: the whole forward path."""
    return solve(fold(f, h, kinds, values), h, kinds, levels, **kw)


def adjoint(g, h, kinds, levels, **kw):
    """lambda = A^{-1} g (A symmetric; homogeneous boundary values)."""
    return solve(_f64(g), h, kinds, levels, **kw)


# ---- variable permittivity ----------------------------------------------------
def vc_faces(eps, kinds=(0,) * 6):
    """Normalised face coefficients (x [nz][ny][nx+1], y [nz][ny+1][nx], z [nz+1][ny][nx])
    from a cell permittivity [nz][ny][nx]: harmonic means; a boundary face takes the
    cell's value, a periodic one the harmonic mean across the wrap."""
    eps = _f64(eps)
    nx, ny, nz = _shape(eps)
    kx, ky, kz = np.empty((nz, ny, nx + 1)), np.empty((nz, ny + 1, nx)), np.empty((nz + 1, ny, nx))
    lib().or_vc_faces(nx, ny, nz, _kinds(kinds), _dp(eps), _dp(kx), _dp(ky), _dp(kz))
    return kx, ky, kz


def vc_coarsen(k):
    kx, ky, kz = (_f64(a) for a in k)
    nz, ny, nx1 = kx.shape
    nx = nx1 - 1
    c = (np.empty((nz // 2, ny // 2, nx // 2 + 1)), np.empty((nz // 2, ny // 2 + 1, nx // 2)),
         np.empty((nz // 2 + 1, ny // 2, nx // 2)))
    lib().or_vc_coarsen(nx, ny, nz, _dp(kx), _dp(ky), _dp(kz), _dp(c[0]), _dp(c[1]), _dp(c[2]))
    return c


def vc_apply(phi, h, kinds, k, level=0):
    phi = _f64(phi)
    nx, ny, nz = _shape(phi)
    kx, ky, kz = (_f64(a) for a in k)
    out = np.empty_like(phi)
    lib().or_vc_apply(nx, ny, nz, h, level, _kinds(kinds), _dp(kx), _dp(ky), _dp(kz), _dp(phi), _dp(out))
    return out


def vc_rbgs_sweep(phi, b, h, kinds, k, level=0, sweeps=1):
    phi = _f64(phi).copy()
    b = _f64(b)
    nx, ny, nz = _shape(phi)
    kx, ky, kz = (_f64(a) for a in k)
    lib().or_vc_rbgs_sweep(nx, ny, nz, h, level, _kinds(kinds), _dp(kx), _dp(ky), _dp(kz), _dp(phi), _dp(b), sweeps)
    return phi


def vc_fold(f, h, kinds, values, k, faces=None):
    f = _f64(f)
    nx, ny, nz = _shape(f)
    kx, ky, kz = (_f64(a) for a in k)
    keep, ptrs = _faces((nx, ny, nz), faces)
    vals = (ctypes.c_double * 6)(*[float(v) for v in values])
    b = np.empty_like(f)
    lib().or_vc_fold(nx, ny, nz, h, _kinds(kinds), vals, ptrs, _dp(kx), _dp(ky), _dp(kz), _dp(f), _dp(b))
    return b


def vc_solve(b, h, kinds, levels, eps, nu1=2, nu2=2, omega=2.0, rtol=1e-10, max_cycles=100, phi0=None,
             cg_rtol=1e-13, cg_maxit=None):
    """FP64 multigrid for -div(eps grad phi) on the folded RHS b. Returns (phi, history, status)."""
    b = _f64(b)
    eps = _f64(eps)
    phi = np.zeros_like(b) if phi0 is None else _f64(phi0).copy()
    nx, ny, nz = _shape(b)
    hist = np.zeros(max_cycles + 1)
    cyc = ctypes.c_int(0)
    cg_maxit = default_cg_maxit((nx, ny, nz), levels) if cg_maxit is None else cg_maxit
    st = lib().or_vc_solve(nx, ny, nz, h, _kinds(kinds), levels, nu1, nu2, omega, cg_rtol, cg_maxit, _dp(eps),
                           _dp(b), _dp(phi), rtol, max_cycles, _dp(hist), ctypes.byref(cyc))
    if st == E_ARG:
        raise ValueError("oracle: invalid hierarchy")
    return phi, hist[: cyc.value + 1].copy(), st


# ---- Poisson-Boltzmann (extension; the equation and iteration are the reading
# written in ccmg_oracle.c) ---------------------------------------------------

def pb_apply(phi, h, kinds, k2, level: int = 0) -> np.ndarray:
    """(A_l + k2 I) phi: the linearised Poisson-Boltzmann operator."""
    phi = _f64(phi)
    out = np.empty_like(phi)
    nx, ny, nz = _shape(phi)
    lib().or_pb_apply(nx, ny, nz, h, level, _kinds(kinds), float(k2), _dp(phi), _dp(out))
    return out


def pb_rbgs_sweep(phi, b, h, kinds, k2, level: int = 0, sweeps: int = 1) -> np.ndarray:
    phi = _f64(phi).copy()
    b = _f64(b)
    nx, ny, nz = _shape(phi)
    for _ in range(sweeps):
        lib().or_pb_rbgs_sweep(nx, ny, nz, h, level, _kinds(kinds), float(k2), _dp(phi), _dp(b))
    return phi


def pb_cg(b, h, kinds, k2, level: int = 0, rtol: float = 1e-13, maxit: Optional[int] = None):
    b = _f64(b)
    x = np.zeros_like(b)
    nx, ny, nz = _shape(b)
    maxit = 2 * b.size if maxit is None else maxit
    it = lib().or_pb_cg(nx, ny, nz, h, level, _kinds(kinds), float(k2), _dp(b), _dp(x), rtol, maxit)
    return x, it


def pb_solve(b, h, kinds, levels, k2, nu1=2, nu2=2, omega=2.0, rtol=1e-10, max_cycles=100,
             phi0=None, cg_rtol=1e-13, cg_maxit=None):
    """Linear (Debye-Hueckel) Poisson-Boltzmann multigrid on the folded RHS b.
    Returns (phi, history, status)."""
    b = _f64(b)
    phi = np.zeros_like(b) if phi0 is None else _f64(phi0).copy()
    nx, ny, nz = _shape(b)
    hist = np.zeros(max_cycles + 1)
    cyc = ctypes.c_int(0)
    cg_maxit = default_cg_maxit((nx, ny, nz), levels) if cg_maxit is None else cg_maxit
    st = lib().or_pb_solve(nx, ny, nz, h, _kinds(kinds), levels, nu1, nu2, omega, cg_rtol, cg_maxit,
                           float(k2), _dp(b), _dp(phi), rtol, max_cycles, _dp(hist), ctypes.byref(cyc))
    if st == E_ARG:
        raise ValueError("oracle: invalid hierarchy")
    return phi, hist[: cyc.value + 1].copy(), st


def pb_nl_residual(psi, b, h, kinds, k2) -> np.ndarray:
    """b - A psi - k2 sinh(psi) on the finest level."""
    psi, b = _f64(psi), _f64(b)
    r = np.empty_like(psi)
    nx, ny, nz = _shape(psi)
    lib().or_pb_nl_residual(nx, ny, nz, h, _kinds(kinds), float(k2), _dp(psi), _dp(b), _dp(r))
    return r


def pb_nl_solve(b, h, kinds, levels, k2, inner=2, nu1=2, nu2=2, omega=2.0, rtol=1e-10, max_outer=200,
                psi0=None, cg_rtol=1e-13, cg_maxit=None):
    """Nonlinear Poisson-Boltzmann -Lap(psi) + k2 sinh(psi) = f on the folded RHS b
    by the shifted chord iteration (inner linear V-cycles per step).  Returns
    (psi, history, status)."""
    b = _f64(b)
    psi = np.zeros_like(b) if psi0 is None else _f64(psi0).copy()
    nx, ny, nz = _shape(b)
    hist = np.zeros(max_outer + 1)
    cyc = ctypes.c_int(0)
    cg_maxit = default_cg_maxit((nx, ny, nz), levels) if cg_maxit is None else cg_maxit
    st = lib().or_pb_nl_solve(nx, ny, nz, h, _kinds(kinds), levels, nu1, nu2, omega, cg_rtol, cg_maxit,
                              float(k2), int(inner), _dp(b), _dp(psi), rtol, max_outer, _dp(hist),
                              ctypes.byref(cyc))
    if st == E_ARG:
        raise ValueError("oracle: invalid hierarchy")
    return psi, hist[: cyc.value + 1].copy(), st
