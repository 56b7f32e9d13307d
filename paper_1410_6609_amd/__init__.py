"""MI355X cell-centered multigrid solver for the electric-potential Poisson problem.

Thin Python binding of ``libccmg.so`` (C ABI in ``include/ccmg.h``).  Every
step of the method runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch supplies device memory (tensors, the workspace)
and the stream.  The method is the cell-centered multigrid of Bartuschat &
Ruede, "Parallel Multiphysics Simulations of Charged Particles in
Microfluidic Flows" (arXiv:1410.6609), Sec. 2.4, Sec. 3 and Sec. 5.3.

There is no CPU fallback: if the library is missing, importing a solver
raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import torch

__all__ = [
    "DIRICHLET", "NEUMANN", "PERIODIC", "FP64", "FP32_IR", "SPREAD", "VOLUME", "CcmgError", "Options", "Stats", "Solver",
    "PoissonFn", "RhsSolveFn", "lib", "load_library", "LIB_PATH", "exported_symbols",
]

DIRICHLET, NEUMANN, PERIODIC = 0, 1, 2
FP64, FP32_IR = 0, 1
SPREAD, VOLUME = 0, 1   # normalisations of the sub-sampled deposition
MAX_SUBSAMPLE = 8
OK, E_ARG, E_DIMS, E_SINGULAR, E_HIP, E_NONFINITE, E_NOCONV, E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
_ERR_NAMES = {E_ARG: "E_ARG", E_DIMS: "E_DIMS", E_SINGULAR: "E_SINGULAR", E_HIP: "E_HIP",
              E_NONFINITE: "E_NONFINITE", E_NOCONV: "E_NOCONV", E_STATE: "E_STATE"}
MAX_CYCLES = 1000

# CCMG_LIB names another build of the same sources (the host-sanitizer run)
LIB_PATH = os.environ.get("CCMG_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libccmg.so")


class CcmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Face(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("value", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("levels", ctypes.c_int),
                ("omega", ctypes.c_double), ("precision", ctypes.c_int),
                ("ir_inner_cycles", ctypes.c_int), ("cg_rtol", ctypes.c_double),
                ("cg_maxit", ctypes.c_int), ("fuse_sweeps", ctypes.c_int), ("bottom_cells", ctypes.c_int),
                ("variable_eps", ctypes.c_int), ("ir_cg_rtol", ctypes.c_double), ("kappa2", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("inner_cycles", ctypes.c_int),
                ("rel_res0", ctypes.c_double), ("rel_res", ctypes.c_double),
                ("seconds", ctypes.c_double)]


@dataclass
class Options:
    nu1: int = 2
    nu2: int = 2
    levels: int = 0
    omega: float = 2.0
    precision: int = FP64
    ir_inner_cycles: int = 4
    cg_rtol: float = 1e-13
    cg_maxit: int = 0
    fuse_sweeps: int = 2
    bottom_cells: int = 4096
    variable_eps: int = 0
    ir_cg_rtol: float = 1e-6
    kappa2: float = 0.0   # Poisson-Boltzmann: squared inverse Debye length (0: Poisson)

    def _c(self) -> _Options:
        return _Options(self.nu1, self.nu2, self.levels, self.omega, self.precision,
                        self.ir_inner_cycles, self.cg_rtol, self.cg_maxit, self.fuse_sweeps,
                        self.bottom_cells, self.variable_eps, self.ir_cg_rtol, self.kappa2)


@dataclass
class Stats:
    cycles: int
    inner_cycles: int
    rel_res0: float
    rel_res: float
    seconds: float
    status: int = 0


_lib = None

_VP = ctypes.c_void_p
_SIGS = {
    "ccmg_default_options": ([ctypes.POINTER(_Options)], None),
    "ccmg_create": ([ctypes.POINTER(_VP), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                     ctypes.POINTER(_Face), ctypes.POINTER(_Options), _VP], ctypes.c_int),
    "ccmg_workspace_bytes": ([_VP], ctypes.c_size_t),
    "ccmg_set_workspace": ([_VP, _VP, ctypes.c_size_t], ctypes.c_int),
    "ccmg_set_stream": ([_VP, _VP], ctypes.c_int),
    "ccmg_num_levels": ([_VP], ctypes.c_int),
    "ccmg_level_dims": ([_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "ccmg_deposit_charges": ([_VP, ctypes.c_int, _VP, _VP, _VP, ctypes.c_double, _VP, _VP], ctypes.c_int),
    "ccmg_deposit_charges_sub": ([_VP, ctypes.c_int, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                  _VP, _VP], ctypes.c_int),
    "ccmg_charge_gradient": ([_VP, ctypes.c_int, _VP, _VP, ctypes.c_double, ctypes.c_int, ctypes.c_int, _VP, _VP],
                             ctypes.c_int),
    "ccmg_set_face_values": ([_VP, ctypes.c_int, _VP], ctypes.c_int),
    "ccmg_gradient": ([_VP, _VP, _VP], ctypes.c_int),
    "ccmg_set_permittivity": ([_VP, _VP], ctypes.c_int),
    "ccmg_coulomb_adjoint": ([_VP, _VP, ctypes.c_int, _VP, _VP, _VP, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP],
                             ctypes.c_int),
    "ccmg_coulomb_force": ([_VP, _VP, ctypes.c_int, _VP, _VP, _VP, ctypes.c_int, ctypes.c_int, _VP], ctypes.c_int),
    "ccmg_force_charge_gradient": ([_VP, _VP, ctypes.c_int, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP, _VP, ctypes.c_double,
                                    ctypes.c_int, ctypes.POINTER(_Stats)], ctypes.c_int),
    "ccmg_vcycle": ([_VP, _VP, _VP, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "ccmg_vcycles": ([_VP, _VP, _VP, ctypes.c_int, _VP], ctypes.c_int),
    "ccmg_solve": ([_VP, _VP, _VP, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_Stats)], ctypes.c_int),
    "ccmg_solve_zero": ([_VP, _VP, _VP, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_Stats)], ctypes.c_int),
    "ccmg_solve_zero_static": ([_VP, _VP, _VP, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_Stats)], ctypes.c_int),
    "ccmg_solve_pb": ([_VP, _VP, _VP, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Stats)],
                      ctypes.c_int),
    "ccmg_adjoint_solve": ([_VP, _VP, _VP, ctypes.c_int, _VP, _VP, ctypes.c_double, _VP, _VP,
                            ctypes.c_double, ctypes.c_int, ctypes.POINTER(_Stats)], ctypes.c_int),
    "ccmg_residual": ([_VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "ccmg_smooth": ([_VP, _VP, _VP, ctypes.c_int], ctypes.c_int),
    "ccmg_history": ([_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_int], ctypes.c_int),
    "ccmg_profile_enable": ([_VP, ctypes.c_int], ctypes.c_int),
    "ccmg_profile_read": ([_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                           ctypes.c_int], ctypes.c_int),
    "ccmg_last_error": ([_VP], ctypes.c_char_p),
    "ccmg_destroy": ([_VP], None),
}


def exported_symbols() -> Sequence[str]:
    return tuple(_SIGS)


def load_library(path: str) -> ctypes.CDLL:
    """Load a build of the library at `path` with the C signatures set (for
    Solver(library=...): another build of the same sources, e.g. other tile
    macros).  Raises if the file is missing."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_1410_6609_amd/build.py`")
    L = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


def lib() -> ctypes.CDLL:
    """Load libccmg.so (built by paper_1410_6609_amd/build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        _lib = load_library(LIB_PATH)
    return _lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Solver:
    """One solver context: grid, faces, options, workspace (a torch tensor).

    shape = (nx, ny, nz); fields are tensors of shape (nz, ny, nx), float64, on
    the solver's device.  faces: 6 pairs (kind, value) for x-, x+, y-, y+, z-, z+.
    """

    def __init__(self, shape: Tuple[int, int, int], h: float, faces: Sequence[Tuple[int, float]],
                 options: Optional[Options] = None, device="cuda", workspace: bool = True,
                 library: Optional[ctypes.CDLL] = None):
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the solver runs on a GPU device only")
        self.shape = tuple(int(n) for n in shape)
        self.h = float(h)
        self.faces = [(int(k), float(v)) for k, v in faces]
        if len(self.faces) != 6:
            raise ValueError("six faces required")
        self.options = options or Options()
        L = lib() if library is None else library   # every call of this solver goes to L
        self._L = L
        arr = (_Face * 6)(*[_Face(k, v) for k, v in self.faces])
        opt = self.options._c()
        handle = ctypes.c_void_p()
        nx, ny, nz = self.shape
        with torch.cuda.device(self.device):
            rc = L.ccmg_create(ctypes.byref(handle), nx, ny, nz, self.h, arr, ctypes.byref(opt),
                               _stream_handle(self.device))
        if rc != OK:
            raise CcmgError(rc, L.ccmg_last_error(None).decode())
        self._h = handle
        nbytes = L.ccmg_workspace_bytes(handle)
        self.workspace = None
        if not workspace:   # only solve_static() can run: it uses the library's static scratch
            return
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self._check(L.ccmg_set_workspace(handle, ctypes.c_void_p(aligned), nbytes))

    # -- plumbing -------------------------------------------------------------
    def __del__(self):
        h, L = getattr(self, "_h", None), getattr(self, "_L", None)
        if h is not None and L is not None:
            L.ccmg_destroy(h)
            self._h = None

    def _check(self, rc: int, allow=()):
        if rc != OK and rc not in allow:
            raise CcmgError(rc, self._L.ccmg_last_error(self._h).decode())
        return rc

    def _bind_stream(self):
        self._L.ccmg_set_stream(self._h, _stream_handle(self.device))

    def _field(self, t: torch.Tensor, name: str) -> torch.Tensor:
        nx, ny, nz = self.shape
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a tensor")
        if t.device != self.device or t.dtype != torch.float64 or tuple(t.shape) != (nz, ny, nx):
            raise ValueError(f"{name} must be float64 of shape {(nz, ny, nx)} on {self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _spheres(self, centers, radii):
        centers = centers.to(self.device, torch.float64).contiguous().reshape(-1, 3)
        radii = radii.to(self.device, torch.float64).contiguous().reshape(-1)
        if centers.shape[0] != radii.shape[0]:
            raise ValueError("centers and radii disagree in length")
        return centers, radii

    @property
    def levels(self) -> int:
        return self._L.ccmg_num_levels(self._h)

    def level_dims(self, l: int) -> Tuple[int, int, int]:
        d = (ctypes.c_int * 3)()
        self._check(self._L.ccmg_level_dims(self._h, l, d))
        return tuple(d)

    def zeros(self) -> torch.Tensor:
        nx, ny, nz = self.shape
        return torch.zeros((nz, ny, nx), dtype=torch.float64, device=self.device)

    # -- the method -----------------------------------------------------------
    def deposit(self, centers, radii, q, eps: float = 1.0, out: Optional[torch.Tensor] = None,
                counts: bool = False, subsample: int = 1, mode: int = SPREAD):
        """f = rho / eps from charged spheres.  subsample = 1 and mode SPREAD is
        the naive volume mapping (counts: n_s per sphere, int32); otherwise the
        sub-sampled deposition (counts: the summed overlap ratios W_s, float64)."""
        centers, radii = self._spheres(centers, radii)
        q = q.to(self.device, torch.float64).contiguous().reshape(-1)
        n = radii.shape[0]
        if q.shape[0] != n:
            raise ValueError("q and radii disagree in length")
        f = self.zeros() if out is None else self._field(out, "out")
        self._bind_stream()
        if subsample == 1 and mode == SPREAD:
            cnt = torch.zeros(n, dtype=torch.int32, device=self.device) if counts else None
            self._check(self._L.ccmg_deposit_charges(self._h, n, _ptr(centers), _ptr(radii), _ptr(q), float(eps),
                                                   _ptr(f), _ptr(cnt)))
        else:
            cnt = torch.zeros(n, dtype=torch.float64, device=self.device) if counts else None
            self._check(self._L.ccmg_deposit_charges_sub(self._h, n, _ptr(centers), _ptr(radii), _ptr(q), float(eps),
                                                       int(subsample), int(mode), _ptr(f), _ptr(cnt)))
        return (f, cnt) if counts else f

    def charge_gradient(self, lam: torch.Tensor, centers, radii, eps: float = 1.0, subsample: int = 1,
                        mode: int = SPREAD) -> torch.Tensor:
        """dL/dq per sphere from the adjoint field lam = dL/df."""
        lam = self._field(lam, "lam")
        c, r = self._spheres(centers, radii)
        dq = torch.zeros(r.shape[0], dtype=torch.float64, device=self.device)
        self._bind_stream()
        self._check(self._L.ccmg_charge_gradient(self._h, r.shape[0], _ptr(c), _ptr(r), float(eps), int(subsample),
                                               int(mode), _ptr(lam), _ptr(dq)))
        return dq

    def gradient(self, phi: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """grad phi as a (3, nz, ny, nx) tensor (D3Q19 inside, D3Q7 with boundary ghosts)."""
        phi = self._field(phi, "phi")
        nx, ny, nz = self.shape
        g = torch.empty((3, nz, ny, nx), dtype=torch.float64, device=self.device) if out is None else out
        if (tuple(g.shape) != (3, nz, ny, nx) or g.dtype != torch.float64 or g.device != self.device
                or not g.is_contiguous()):
            raise ValueError("out must be a contiguous float64 tensor of shape (3, nz, ny, nx)")
        self._bind_stream()
        self._check(self._L.ccmg_gradient(self._h, _ptr(phi), _ptr(g)))
        return g

    def coulomb_force(self, phi: torch.Tensor, centers, radii, q, subsample: int = 1, mode: int = SPREAD,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Electrostatic force per sphere, (n, 3)."""
        phi = self._field(phi, "phi")
        c, r = self._spheres(centers, radii)
        q = q.to(self.device, torch.float64).contiguous().reshape(-1)
        n = r.shape[0]
        if q.shape[0] != n:
            raise ValueError("q and radii disagree in length")
        F = torch.zeros((n, 3), dtype=torch.float64, device=self.device) if out is None else out
        if tuple(F.shape) != (n, 3) or F.dtype != torch.float64 or F.device != self.device or not F.is_contiguous():
            raise ValueError(f"out must be a contiguous float64 tensor of shape ({n}, 3) on {self.device}")
        self._bind_stream()
        self._check(self._L.ccmg_coulomb_force(self._h, _ptr(phi), n, _ptr(c), _ptr(r), _ptr(q), int(subsample),
                                             int(mode), _ptr(F)))
        return F

    def coulomb_adjoint(self, phi: torch.Tensor, centers, radii, q, gF: torch.Tensor, subsample: int = 1,
                        mode: int = SPREAD):
        """(mu = dL/dphi, direct per-sphere term) for dL/dF = gF of shape (n, 3)."""
        phi = self._field(phi, "phi")
        c, r = self._spheres(centers, radii)
        q = q.to(self.device, torch.float64).contiguous().reshape(-1)
        gF = gF.to(self.device, torch.float64).contiguous().reshape(-1, 3)
        n = r.shape[0]
        if q.shape[0] != n or gF.shape[0] != n:
            raise ValueError("q, gF and radii disagree in length")
        mu = self.zeros()
        direct = torch.zeros(n, dtype=torch.float64, device=self.device)
        self._bind_stream()
        self._check(self._L.ccmg_coulomb_adjoint(self._h, _ptr(phi), n, _ptr(c), _ptr(r), _ptr(q), int(subsample),
                                               int(mode), _ptr(gF), _ptr(mu), _ptr(direct)))
        return mu, direct

    def force_charge_gradient(self, phi: torch.Tensor, centers, radii, q, gF: torch.Tensor, eps: float = 1.0,
                              force_subsample: int = 1, force_mode: int = SPREAD, deposit_subsample: int = 1,
                              deposit_mode: int = SPREAD, rtol: float = 1e-10, max_cycles: int = 100):
        """dL/dq for a loss on the forces computed from phi = A^-1 b(deposit(q))
        (ccmg_force_charge_gradient: force adjoint, adjoint solve and the
        deposition's charge gradient, all on the device)."""
        phi = self._field(phi, "phi")
        c, r = self._spheres(centers, radii)
        q = q.to(self.device, torch.float64).contiguous().reshape(-1)
        gF = gF.to(self.device, torch.float64).contiguous().reshape(-1, 3)
        n = r.shape[0]
        if q.shape[0] != n or gF.shape[0] != n:
            raise ValueError("q, gF and radii disagree in length")
        mu, lam = self.zeros(), self.zeros()
        dq = torch.zeros(n, dtype=torch.float64, device=self.device)
        st = _Stats()
        self._bind_stream()
        self._check(self._L.ccmg_force_charge_gradient(
            self._h, _ptr(phi), n, _ptr(c), _ptr(r), _ptr(q), float(eps), int(force_subsample), int(force_mode),
            int(deposit_subsample), int(deposit_mode), _ptr(gF), _ptr(mu), _ptr(lam), _ptr(dq), float(rtol),
            int(max_cycles), ctypes.byref(st)))
        return dq

    def set_permittivity(self, eps: Optional[torch.Tensor]) -> None:
        """Cell-wise permittivity (None: back to the constant operator); needs
        Options(variable_eps=1).  Afterwards solves take f = rho."""
        v = None
        if eps is not None:
            v = self._field(eps.to(self.device, torch.float64).contiguous(), "eps")
        self._bind_stream()
        self._check(self._L.ccmg_set_permittivity(self._h, _ptr(v)))
        self._eps_keep = v   # read by the enqueued kernels

    def set_face_values(self, face: int, values: Optional[torch.Tensor]) -> None:
        """Per-cell boundary values of one face (None: back to the constant):
        x faces (nz, ny), y faces (nz, nx), z faces (ny, nx)."""
        nx, ny, nz = self.shape
        shape = [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2
        v = None
        if values is not None:
            v = values.to(self.device, torch.float64).contiguous()
            if tuple(v.shape) != shape[face]:
                raise ValueError(f"face {face} values must have shape {shape[face]}")
        self._bind_stream()
        self._check(self._L.ccmg_set_face_values(self._h, int(face), _ptr(v)))
        self._face_keep = getattr(self, "_face_keep", {})
        self._face_keep[face] = v   # the copy is stream-ordered: keep the source until it ran

    def solve(self, f: torch.Tensor, phi: Optional[torch.Tensor] = None, rtol: float = 1e-10,
              max_cycles: int = 100, check: bool = True, zero_guess: bool = False):
        """Solve A phi = b(f) in place on phi.  phi holds the initial guess,
        unless zero_guess is set or phi is None: then the solve starts from
        phi = 0 (ccmg_solve_zero) and phi is output only.  Returns (phi, Stats)."""
        f = self._field(f, "f")
        if phi is None:
            nx, ny, nz = self.shape
            phi = torch.empty((nz, ny, nx), dtype=torch.float64, device=self.device)
            zero_guess = True
        else:
            phi = self._field(phi, "phi")
        st = _Stats()
        self._bind_stream()
        fn = self._L.ccmg_solve_zero if zero_guess else self._L.ccmg_solve
        rc = fn(self._h, _ptr(phi), _ptr(f), float(rtol), int(max_cycles), ctypes.byref(st))
        if check:
            self._check(rc)
        s = Stats(st.cycles, st.inner_cycles, st.rel_res0, st.rel_res, st.seconds, rc)
        return phi, s

    def solve_static(self, f: torch.Tensor, phi: torch.Tensor, rtol: float = 1e-10, max_cycles: int = 100,
                     check: bool = True):
        """The solve from phi = 0 on the library's static device scratch
        (ccmg_solve_zero_static): no device memory is allocated, here or in the
        library; phi (output) and f are the caller's.  Returns (phi, Stats)."""
        f = self._field(f, "f")
        phi = self._field(phi, "phi")
        st = _Stats()
        self._bind_stream()
        rc = self._L.ccmg_solve_zero_static(self._h, _ptr(phi), _ptr(f), float(rtol), int(max_cycles),
                                          ctypes.byref(st))
        if check:
            self._check(rc)
        return phi, Stats(st.cycles, st.inner_cycles, st.rel_res0, st.rel_res, st.seconds, rc)

    def solve_pb(self, f: torch.Tensor, psi: Optional[torch.Tensor] = None, rtol: float = 1e-10,
                 max_outer: int = 200, inner: int = 2, check: bool = True):
        """Nonlinear Poisson-Boltzmann -Lap(psi) + kappa2 sinh(psi) = f (ccmg_solve_pb;
        the solver's options set kappa2).  psi: initial guess (None: zero), updated
        in place.  Returns (psi, Stats)."""
        f = self._field(f, "f")
        psi = self.zeros() if psi is None else self._field(psi, "psi")
        st = _Stats()
        self._bind_stream()
        rc = self._L.ccmg_solve_pb(self._h, _ptr(psi), _ptr(f), float(rtol), int(max_outer), int(inner),
                                 ctypes.byref(st))
        if check:
            self._check(rc)
        return psi, Stats(st.cycles, st.inner_cycles, st.rel_res0, st.rel_res, st.seconds, rc)

    def vcycle(self, phi: torch.Tensor, f: torch.Tensor, norm: bool = True) -> Optional[float]:
        f = self._field(f, "f")
        phi = self._field(phi, "phi")
        out = ctypes.c_double(0.0)
        self._bind_stream()
        self._check(self._L.ccmg_vcycle(self._h, _ptr(phi), _ptr(f), ctypes.byref(out) if norm else None))
        return out.value if norm else None

    def vcycles(self, phi: torch.Tensor, f: torch.Tensor, ncycles: int,
                rel_out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """`ncycles` warm-started cycles on phi, enqueued without waiting;
        rel_out (a float64 device tensor of one element, or None) receives the
        relative residual after the last cycle."""
        phi = self._field(phi, "phi")
        f = self._field(f, "f")
        if rel_out is not None and (rel_out.device != self.device or rel_out.dtype != torch.float64
                                    or rel_out.numel() != 1):
            raise ValueError("rel_out must be one float64 element on the solver's device")
        self._bind_stream()
        self._check(self._L.ccmg_vcycles(self._h, _ptr(phi), _ptr(f), int(ncycles), _ptr(rel_out)))
        return phi

    def adjoint(self, g: torch.Tensor, centers=None, radii=None, eps: float = 1.0, rtol: float = 1e-10,
                max_cycles: int = 100, want_drho: bool = False, lam: Optional[torch.Tensor] = None,
                check: bool = True, subsample: int = 1, mode: int = SPREAD):
        """lambda = A^{-1} g; optional dL/dq per sphere (for the deposition with
        the same subsample and mode) and dL/drho.  Returns (lam, dq, drho, Stats)."""
        g = self._field(g, "g")
        lam = self.zeros() if lam is None else self._field(lam, "lam")
        naive = subsample == 1 and mode == SPREAD
        n = 0
        dq = None
        c = r = None
        if centers is not None:
            c, r = self._spheres(centers, radii)
            n = r.shape[0]
            dq = torch.zeros(n, dtype=torch.float64, device=self.device)
        drho = self.zeros() if want_drho else None
        st = _Stats()
        self._bind_stream()
        nn = n if naive else 0
        rc = self._L.ccmg_adjoint_solve(self._h, _ptr(g), _ptr(lam), nn, _ptr(c), _ptr(r), float(eps),
                                      _ptr(dq) if naive else None, _ptr(drho), float(rtol), int(max_cycles),
                                      ctypes.byref(st))
        if check:
            self._check(rc)
        if n > 0 and not naive and rc in (OK, E_NOCONV):
            self._check(self._L.ccmg_charge_gradient(self._h, n, _ptr(c), _ptr(r), float(eps), int(subsample),
                                                   int(mode), _ptr(lam), _ptr(dq)))
        return lam, dq, drho, Stats(st.cycles, st.inner_cycles, st.rel_res0, st.rel_res, st.seconds, rc)

    def residual(self, phi: torch.Tensor, f: torch.Tensor, want_field: bool = True):
        phi = self._field(phi, "phi")
        f = self._field(f, "f")
        r = self.zeros() if want_field else None
        out = ctypes.c_double(0.0)
        self._bind_stream()
        self._check(self._L.ccmg_residual(self._h, _ptr(phi), _ptr(f), _ptr(r), ctypes.byref(out)))
        return r, out.value

    def smooth(self, phi: torch.Tensor, f: torch.Tensor, sweeps: int = 1) -> torch.Tensor:
        phi = self._field(phi, "phi")
        f = self._field(f, "f")
        self._bind_stream()
        self._check(self._L.ccmg_smooth(self._h, _ptr(phi), _ptr(f), int(sweeps)))
        return phi

    def profile(self, on: bool = True) -> None:
        self._check(self._L.ccmg_profile_enable(self._h, int(on)))

    def profile_read(self, which: int, reset: bool = True) -> Tuple[float, int]:
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int(0)
        self._check(self._L.ccmg_profile_read(self._h, which, ctypes.byref(ms), ctypes.byref(n), int(reset)))
        return ms.value, n.value

    def history(self):
        buf = (ctypes.c_double * (MAX_CYCLES + 1))()
        n = self._L.ccmg_history(self._h, buf, MAX_CYCLES + 1)
        return list(buf[:n])


class PoissonFn(torch.autograd.Function):
    """phi = A^{-1} b(deposit(q)) for charged spheres; backward gives dL/dq by the
    adjoint multigrid solve of the same symmetric operator."""

    @staticmethod
    def forward(ctx, q, centers, radii, solver: Solver, eps: float = 1.0, rtol: float = 1e-10,
                max_cycles: int = 100, subsample: int = 1, mode: int = SPREAD):
        f = solver.deposit(centers, radii, q, eps, subsample=subsample, mode=mode)
        phi, st = solver.solve(f, rtol=rtol, max_cycles=max_cycles)
        ctx.solver, ctx.eps, ctx.rtol, ctx.max_cycles = solver, eps, rtol, max_cycles
        ctx.subsample, ctx.mode = subsample, mode
        ctx.save_for_backward(centers, radii)
        ctx.stats = st
        return phi

    @staticmethod
    def backward(ctx, grad_phi):
        centers, radii = ctx.saved_tensors
        g = grad_phi.contiguous().to(torch.float64)
        _, dq, _, _ = ctx.solver.adjoint(g, centers, radii, ctx.eps, ctx.rtol, ctx.max_cycles,
                                         subsample=ctx.subsample, mode=ctx.mode)
        return dq, None, None, None, None, None, None, None, None


class CoulombForceFn(torch.autograd.Function):
    """Forces on charged spheres: q -> deposition -> phi = A^-1 b -> F (n, 3);
    backward by the force adjoint, one adjoint solve and the deposition's
    charge gradient."""

    @staticmethod
    def forward(ctx, q, centers, radii, solver: Solver, eps: float = 1.0, rtol: float = 1e-10,
                max_cycles: int = 100, subsample: int = 1, mode: int = SPREAD):
        f = solver.deposit(centers, radii, q, eps, subsample=subsample, mode=mode)
        phi, _ = solver.solve(f, rtol=rtol, max_cycles=max_cycles)
        F = solver.coulomb_force(phi, centers, radii, q, subsample=subsample, mode=mode)
        ctx.solver, ctx.eps, ctx.rtol, ctx.max_cycles = solver, eps, rtol, max_cycles
        ctx.subsample, ctx.mode = subsample, mode
        ctx.save_for_backward(q, centers, radii, phi)
        return F

    @staticmethod
    def backward(ctx, grad_F):
        q, centers, radii, phi = ctx.saved_tensors
        dq = ctx.solver.force_charge_gradient(phi, centers, radii, q.detach(), grad_F, ctx.eps, ctx.subsample,
                                              ctx.mode, ctx.subsample, ctx.mode, ctx.rtol, ctx.max_cycles)
        return dq, None, None, None, None, None, None, None, None


class RhsSolveFn(torch.autograd.Function):
    """phi = A^{-1} b(f) for a right-hand side f = rho / eps; backward gives
    dL/df = lambda."""

    @staticmethod
    def forward(ctx, f, solver: Solver, rtol: float = 1e-10, max_cycles: int = 100):
        phi, _ = solver.solve(f.contiguous(), rtol=rtol, max_cycles=max_cycles)
        ctx.solver, ctx.rtol, ctx.max_cycles = solver, rtol, max_cycles
        return phi

    @staticmethod
    def backward(ctx, grad_phi):
        lam, _, _, _ = ctx.solver.adjoint(grad_phi.contiguous().to(torch.float64), rtol=ctx.rtol,
                                          max_cycles=ctx.max_cycles)
        return lam, None, None, None
