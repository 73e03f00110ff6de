"""ctypes binding of ``libqmg.so`` (the C ABI declared in ``include/qmg.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory (the grid workspace) and the HIP stream.  The
binding raises if the library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqmg.so")

QMG_OK, QMG_EINVAL, QMG_ENOMEM, QMG_EHIP, QMG_ESTATE, QMG_ENOTCONV, QMG_EINDEF, QMG_EBUSY = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "QMG_OK", -1: "QMG_EINVAL", -2: "QMG_ENOMEM", -3: "QMG_EHIP",
                -4: "QMG_ESTATE", -5: "QMG_ENOTCONV", -6: "QMG_EINDEF", -7: "QMG_EBUSY"}
QMG_HOST, QMG_DEVICE = 0, 1
GEOMETRIC, GALERKIN_DLINEAR, BOXMG = 0, 1, 2
PLAIN_FP64, HIER_FP64, HIER_FP32, HIER_FP16, HIER_BF16, HIER_BPA = 0, 1, 2, 3, 4, 5
OP_MATVEC, OP_RESIDUAL, OP_JACOBI, OP_RESTRICT, OP_PROLONG, OP_SMOOTH = 0, 1, 2, 3, 4, 5
SMOOTHERS = {"jacobi": 0, "block": 1}
CYCLES = {"mult": 0, "add": 1, "bpx": 2}
RESTRICTIONS = {"transpose": 0, "injection": 1, "aggregation": 2}
DAMPINGS = {"exp": 0, "const": 1}
COARSE_SOLVERS = {"direct": 0, "sweeps": 1}
ITERATES = {"store": 0, "fp64": 1, "fp32": 2}

TRANSFERS = {"geometric": GEOMETRIC, "galerkin": GALERKIN_DLINEAR, "boxmg": BOXMG}
STORES = {"plain64": PLAIN_FP64, "hier64": HIER_FP64, "hier32": HIER_FP32,
          "hier16": HIER_FP16, "bf16": HIER_BF16, "bpa": HIER_BPA}


REGION_BALL, REGION_LEVELSET_BAND, REGION_CELL_LIST = 0, 1, 2


class Region(C.Structure):
    _fields_ = [("kind", C.c_int), ("level", C.c_int), ("params", C.c_void_p), ("n_params", C.c_int)]


class GridDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("max_level", C.c_int), ("base_level", C.c_int),
                ("refine", C.c_void_p), ("n_regions", C.c_int), ("regions", C.c_void_p)]


class SolverOpts(C.Structure):
    _fields_ = [("transfer", C.c_int), ("store", C.c_int), ("mu_pre", C.c_int),
                ("mu_post", C.c_int), ("omega", C.c_double), ("coarsest_level", C.c_int),
                ("check_definite", C.c_int), ("inner_cycles", C.c_int), ("use_graphs", C.c_int),
                ("stagnation", C.c_double), ("smoother", C.c_int), ("bj_sweeps", C.c_int),
                ("cycle", C.c_int), ("damping", C.c_int), ("eps_mf", C.c_double), ("restriction", C.c_int),
                ("coarse_solver", C.c_int), ("eps_zero", C.c_double), ("iterate", C.c_int)]


class SolveReport(C.Structure):
    _fields_ = [("cycles", C.c_int), ("outer_iters", C.c_int), ("relres", C.c_double),
                ("coarsest_level_used", C.c_int), ("vertex_updates", C.c_int64),
                ("bytes_operators", C.c_size_t), ("zero_delta_fraction", C.c_double),
                ("seconds", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("active", C.c_int64), ("queued", C.c_int64), ("hbm_budget", C.c_size_t),
                ("hbm_in_use", C.c_size_t), ("hbm_peak", C.c_size_t), ("max_slots", C.c_int),
                ("deferred", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# every entry point of include/qmg.h with its ctypes signature
_SIGS = {
    "qmg_version": (C.c_char_p, []),
    "qmg_workspace_bytes": (C.c_int, [C.POINTER(GridDesc), C.POINTER(SolverOpts), C.POINTER(C.c_size_t)]),
    "qmg_default_opts": (C.c_int, [C.POINTER(SolverOpts)]),
    "qmg_region_flags": (C.c_int, [C.POINTER(GridDesc), C.c_void_p, C.c_int64]),
    "qmg_create_grid": (C.c_int, [C.POINTER(GridDesc), C.POINTER(SolverOpts), C.c_void_p, C.c_size_t,
                                  C.c_void_p, C.POINTER(C.c_void_p)]),
    "qmg_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int)]),
    "qmg_unknown_coords": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "qmg_leaf_cell_centres": (C.c_int, [C.c_void_p, C.c_void_p]),
    "qmg_set_coefficients": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int]),
    "qmg_build_operators": (C.c_int, [C.c_void_p, C.POINTER(SolveReport)]),
    "qmg_vcycle": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "qmg_solve": (C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_void_p, C.POINTER(SolveReport)]),
    "qmg_get_solution": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "qmg_residual": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "qmg_set_solution": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "qmg_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "qmg_profile_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "qmg_destroy_grid": (C.c_int, [C.c_void_p]),
    "qmg_last_error": (C.c_char_p, [C.c_void_p]),
    "qmg_get_operator": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "qmg_get_prolongation": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "qmg_refine_flags": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.POINTER(C.c_int64)]),
    "qmg_refine_flags_noalloc": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.POINTER(C.c_int64)]),
    "qmg_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "qmg_server_create": (C.c_int, [C.c_size_t, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "qmg_server_submit": (C.c_int, [C.c_void_p, C.POINTER(GridDesc), C.POINTER(SolverOpts), C.c_void_p,
                                    C.c_void_p, C.c_double, C.c_int, C.c_double, C.POINTER(C.c_uint64)]),
    "qmg_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int), C.c_void_p,
                                  C.POINTER(SolveReport), C.POINTER(C.c_double)]),
    "qmg_server_drain": (C.c_int, [C.c_void_p]),
    "qmg_server_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "qmg_server_last_error": (C.c_char_p, [C.c_void_p]),
    "qmg_server_destroy": (C.c_int, [C.c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class QmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_opts(transfer="boxmg", store="hier64", mu=(2, 2), omega=0.6, coarsest_level=1,
              check_definite=True, inner_cycles=1, graphs=True, stagnation=0.0, smoother="jacobi",
              bj_sweeps=1, cycle="mult", damping="exp", eps_mf=1e-8,
              restriction="transpose", coarse_solver="direct", eps_zero=0.0, iterate="store") -> SolverOpts:
    """qmg_solver_opts from names (the header documents every field):
    transfer "geometric" | "galerkin" | "boxmg"; store "plain64" | "hier64" |
    "hier32" | "hier16" | "bf16" | "bpa" (eps_mf: the bpa coding error);
    smoother "jacobi" | "block" (bj_sweeps Gauss-Seidel sweeps per patch);
    cycle "mult" | "add" | "bpx" with damping "exp" | "const"; restriction
    "transpose" | "injection" | "aggregation"; stagnation > 0 raises the
    coarsest level when a cycle reduces the residual by less than that
    factor; coarse_solver "direct" | "sweeps"; eps_zero the zero-delta
    threshold (0: default); iterate "store" | "fp64" | "fp32"."""
    o = SolverOpts()
    o.transfer = TRANSFERS[transfer] if isinstance(transfer, str) else int(transfer)
    o.store = STORES[store] if isinstance(store, str) else int(store)
    o.mu_pre, o.mu_post = int(mu[0]), int(mu[1])
    o.omega = float(omega)
    o.coarsest_level = int(coarsest_level)
    o.check_definite = 1 if check_definite else 0
    o.inner_cycles = int(inner_cycles)
    o.use_graphs = 1 if graphs else 0
    o.stagnation = float(stagnation)
    o.smoother = SMOOTHERS[smoother] if isinstance(smoother, str) else int(smoother)
    o.bj_sweeps = int(bj_sweeps)
    o.cycle = CYCLES[cycle] if isinstance(cycle, str) else int(cycle)
    o.damping = DAMPINGS[damping] if isinstance(damping, str) else int(damping)
    o.eps_mf = float(eps_mf)
    o.restriction = RESTRICTIONS[restriction] if isinstance(restriction, str) else int(restriction)
    o.coarse_solver = COARSE_SOLVERS[coarse_solver] if isinstance(coarse_solver, str) else int(coarse_solver)
    o.eps_zero = float(eps_zero)
    o.iterate = ITERATES[iterate] if isinstance(iterate, str) else int(iterate)
    return o


def pack_refine(dim: int, base: int, level: int, flags) -> np.ndarray:
    """Refinement flags of levels base..level-1 as the library's byte array
    (``flags[l]``: array of shape (3^l,)*dim over the cells of level l, NumPy
    axes (z,) y, x; missing levels mean no refinement)."""
    parts = []
    for l in range(base, level):
        shape = (3 ** l,) * dim
        a = np.asarray(flags.get(l, np.zeros(shape, bool)))
        if a.shape != shape:
            raise ValueError(f"refinement flags of level {l} must have shape {shape}")
        parts.append(np.ascontiguousarray(a != 0, dtype=np.uint8).ravel())
    return np.ascontiguousarray(np.concatenate(parts))


def make_desc(dim: int, level: int, base_level=None, refine=None, regions=None) -> GridDesc:
    """qmg_grid_desc: regular (base_level None), or an adaptive spacetree from
    refinement flags (``refine``: {level: bool array}) and/or regions
    (``regions``: list of (kind, level, params) with the header's parameter
    layouts).  The returned structure keeps its arrays alive."""
    desc = GridDesc(int(dim), int(level))
    if base_level is not None and int(base_level) not in (0, int(level)):
        desc.base_level = int(base_level)
        if refine is not None or not regions:
            desc._refine = pack_refine(int(dim), int(base_level), int(level), refine or {})
            desc.refine = desc._refine.ctypes.data_as(C.c_void_p)
        if regions:
            desc._params = [np.ascontiguousarray(p, dtype=np.float64) for _, _, p in regions]
            arr = (Region * len(regions))()
            for i, ((kind, lv, _), p) in enumerate(zip(regions, desc._params)):
                arr[i] = Region(int(kind), int(lv), p.ctypes.data_as(C.c_void_p), int(p.size))
            desc._regions = arr
            desc.n_regions = len(regions)
            desc.regions = C.cast(arr, C.c_void_p)
    elif regions:
        raise ValueError("regions need an adaptive grid (base_level)")
    return desc


def region_flags(dim: int, level: int, base_level: int, regions, refine=None) -> dict:
    """The library's refinement flags for ``regions`` (and ``refine``), as
    {level: bool array (3^l,)*dim in NumPy axes (z,) y, x} for levels
    base..level-1 (host evaluation; no device needed)."""
    lib = load()
    desc = make_desc(dim, level, base_level, refine, regions)
    total = sum(3 ** (l * dim) for l in range(base_level, level))
    out = np.zeros(total, dtype=np.uint8)
    rc = lib.qmg_region_flags(C.byref(desc), _ptr(out), int(total))
    if rc != QMG_OK:
        raise QmgError(rc, lib.qmg_last_error(None).decode())
    flags, k = {}, 0
    for l in range(base_level, level):
        m = 3 ** (l * dim)
        flags[l] = out[k:k + m].reshape((3 ** l,) * dim).astype(bool)
        k += m
    return flags


class Grid:
    """One grid of the unit square/cube (regular, or an adaptive spacetree when
    ``base_level`` and ``refine`` are given) with its operators and iterates.

    The workspace is a torch uint8 CUDA tensor owned by this object; work runs on
    ``stream`` (a torch.cuda.Stream, default: the current stream)."""

    def __init__(self, dim: int, level: int, opts: Optional[SolverOpts] = None, stream=None,
                 device: str = "cuda", base_level: Optional[int] = None, refine=None, regions=None):
        import torch
        self.lib = load()
        self.dim, self.level = int(dim), int(level)
        self.opts = opts if opts is not None else make_opts()
        self.desc = make_desc(self.dim, self.level, base_level, refine, regions)
        self.adaptive = base_level is not None and int(base_level) not in (0, self.level)
        nbytes = C.c_size_t(0)
        self._check(self.lib.qmg_workspace_bytes(C.byref(self.desc), C.byref(self.opts), C.byref(nbytes)), None)
        self.workspace_bytes = int(nbytes.value)
        self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        self._check(self.lib.qmg_create_grid(C.byref(self.desc), C.byref(self.opts),
                                             C.c_void_p(self._ws.data_ptr()), nbytes,
                                             C.c_void_p(self.stream.cuda_stream), C.byref(h)), None)
        self.h = h
        self.n = 3 ** self.level
        nu, nc, nl = C.c_int64(0), C.c_int64(0), C.c_int(0)
        self._check(self.lib.qmg_sizes(self.h, C.byref(nu), C.byref(nc), C.byref(nl)), self.h)
        self.n_unknowns, self.n_cells = int(nu.value), int(nc.value)

    def unknown_coords(self):
        """(coordinates (n_unknowns, dim), level of each unknown)."""
        xyz = np.zeros((self.n_unknowns, self.dim))
        lev = np.zeros(self.n_unknowns, dtype=np.int8)
        self._check(self.lib.qmg_unknown_coords(self.h, _ptr(xyz), _ptr(lev)), self.h)
        return xyz, lev

    def cell_centres(self):
        xyz = np.zeros((self.n_cells, self.dim))
        self._check(self.lib.qmg_leaf_cell_centres(self.h, _ptr(xyz)), self.h)
        return xyz

    # -- errors --------------------------------------------------------------
    def _check(self, rc, h, allow=()):
        if rc != QMG_OK and rc not in allow:
            msg = self.lib.qmg_last_error(h).decode() if h is not None else \
                self.lib.qmg_last_error(None).decode()
            raise QmgError(rc, msg)
        return rc

    # -- main path -----------------------------------------------------------
    def set_coefficients(self, eps, f, v=None):
        """eps per leaf cell, f per unknown: NumPy arrays (host) or contiguous
        float64 torch tensors on the grid's device (used in place).  ``v``
        (host only): velocities per cell, shape (d,) + cells, for the
        convection term."""
        if hasattr(eps, "data_ptr") and hasattr(f, "data_ptr"):
            import torch
            if v is not None:
                raise ValueError("velocities are taken from host memory")
            for t in (eps, f):
                if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                    raise ValueError("device inputs must be contiguous float64 tensors on the GPU")
            if eps.numel() != self.n_cells or f.numel() != self.n_unknowns:
                raise ValueError(f"eps must hold {self.n_cells} values and f {self.n_unknowns}")
            self._check(self.lib.qmg_set_coefficients(self.h, C.c_void_p(eps.data_ptr()), 1,
                                                      C.c_void_p(f.data_ptr()), QMG_DEVICE), self.h)
            return
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        f = np.ascontiguousarray(f, dtype=np.float64)
        if eps.size != self.n_cells or f.size != self.n_unknowns:
            raise ValueError(f"eps must hold {self.n_cells} values and f {self.n_unknowns}")
        ncomp = 1
        if v is not None:
            v = np.ascontiguousarray(v, dtype=np.float64)
            if v.size != self.dim * self.n_cells:
                raise ValueError(f"v must hold {self.dim} x {self.n_cells} values")
            eps = np.concatenate([eps.ravel(), v.ravel()])
            ncomp = 1 + self.dim
        self._check(self.lib.qmg_set_coefficients(self.h, _ptr(eps), ncomp, _ptr(f), QMG_HOST), self.h)

    def build(self) -> dict:
        rep = SolveReport()
        self._check(self.lib.qmg_build_operators(self.h, C.byref(rep)), self.h)
        return rep.as_dict()

    def vcycle(self, n: int = 1) -> np.ndarray:
        rr = np.zeros(max(n, 1))
        self._check(self.lib.qmg_vcycle(self.h, int(n), _ptr(rr)), self.h)
        return rr[:n]

    def solve(self, tol: float = 1e-8, max_cycles: int = 500):
        hist = np.zeros(max(max_cycles, 1))
        rep = SolveReport()
        rc = self._check(self.lib.qmg_solve(self.h, float(tol), int(max_cycles), _ptr(hist), C.byref(rep)),
                         self.h, allow=(QMG_ENOTCONV,))
        d = rep.as_dict()
        d["status"] = STATUS_NAMES[rc]
        return d, hist[: max(rep.outer_iters - 1, 0)]

    def solution(self) -> np.ndarray:
        u = np.zeros(self.n_unknowns)
        self._check(self.lib.qmg_get_solution(self.h, _ptr(u), QMG_HOST), self.h)
        return u

    def residual(self) -> np.ndarray:
        """b - A u per unknown (composite system when adaptive; FP64 iterates)."""
        r = np.zeros(self.n_unknowns)
        self._check(self.lib.qmg_residual(self.h, _ptr(r), QMG_HOST), self.h)
        return r

    def set_solution(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        self._check(self.lib.qmg_set_solution(self.h, _ptr(u), QMG_HOST), self.h)

    def profile(self, every=1):
        """Time every ``every``-th finest-level sweep with HIP events (0 or
        False: off; True: every sweep)."""
        every = (1 if every else 0) if isinstance(every, bool) else int(every)
        self._check(self.lib.qmg_profile_enable(self.h, every), self.h)

    def profile_read(self):
        n = C.c_int64(0)
        ms = C.c_double(0.0)
        self._check(self.lib.qmg_profile_read(self.h, C.byref(n), C.byref(ms)), self.h)
        return int(n.value), float(ms.value)

    # -- inspection ----------------------------------------------------------
    def _lat_shape(self, level):
        return (3 ** level + 1,) * self.dim

    def operator(self, level: int) -> np.ndarray:
        out = np.zeros((3 ** self.dim,) + self._lat_shape(level))
        self._check(self.lib.qmg_get_operator(self.h, int(level), _ptr(out)), self.h)
        return out

    def refine_flags(self, res_tol: float = 1e-2, fraction: float = 0.1, noalloc: bool = False) -> np.ndarray:
        """Cells of the finest level flagged by the refinement criterion, as a
        boolean array of shape (3^L,)*d (NumPy axes (z,) y, x).  ``noalloc``
        takes the entry point that allocates no device memory."""
        n = 3 ** self.level
        out = np.zeros((n,) * self.dim, dtype=np.uint8)
        cnt = C.c_int64(0)
        fn = self.lib.qmg_refine_flags_noalloc if noalloc else self.lib.qmg_refine_flags
        self._check(fn(self.h, float(res_tol), float(fraction), out.ctypes.data_as(C.c_void_p), C.byref(cnt)),
                    self.h)
        assert int(cnt.value) == int(out.sum())
        return out.astype(bool)

    def prolongation(self, level: int) -> np.ndarray:
        out = np.zeros((2 ** self.dim,) + self._lat_shape(level))
        self._check(self.lib.qmg_get_prolongation(self.h, int(level), _ptr(out)), self.h)
        return out

    def apply(self, op: int, level: int, x: Optional[np.ndarray], b: Optional[np.ndarray] = None) -> np.ndarray:
        """One step on ``level``; ``x=None`` with OP_JACOBI is the sweep from
        a zero iterate."""
        xp = None
        if x is not None:
            x = np.ascontiguousarray(x, dtype=np.float64)
            xp = _ptr(x)
        out_level = level - 1 if op == OP_RESTRICT else level
        out = np.zeros(self._lat_shape(out_level))
        bp = None
        if b is not None:
            b = np.ascontiguousarray(b, dtype=np.float64)
            bp = _ptr(b)
        self._check(self.lib.qmg_apply(self.h, int(op), int(level), xp, bp, _ptr(out)), self.h)
        return out

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.qmg_destroy_grid(self.h)
            self.h = C.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Persistent solve server on the current HIP device (see qmg_server_* in
    include/qmg.h).  Requests carry their own grid size, coefficients, options
    and tolerance; results come back through poll()."""

    def __init__(self, hbm_budget: int, max_slots: int = 8, stream=None):
        import torch
        torch.cuda.init()
        self.lib = load()
        h = C.c_void_p()
        st = C.c_void_p(stream.cuda_stream) if stream is not None else C.c_void_p()
        rc = self.lib.qmg_server_create(C.c_size_t(int(hbm_budget)), int(max_slots), st, C.byref(h))
        if rc != QMG_OK:
            raise QmgError(rc, self.lib.qmg_server_last_error(None).decode())
        self.h = h
        self._n = {}

    def _err(self, rc):
        raise QmgError(rc, self.lib.qmg_server_last_error(self.h).decode())

    def submit(self, dim: int, level: int, eps, f, opts: SolverOpts, tol: float = 1e-8,
               max_cycles: int = 1000, t_arrival: float = -1.0) -> int:
        """Queues one request; ``t_arrival`` seconds on the server clock (from
        its creation; negative: now) is when it arrives."""
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        f = np.ascontiguousarray(f, dtype=np.float64)
        n = 3 ** level
        if eps.size != n ** dim or f.size != (n - 1) ** dim:
            raise ValueError("eps must hold n^d values and f (n-1)^d values")
        desc = GridDesc(int(dim), int(level))
        t = C.c_uint64(0)
        rc = self.lib.qmg_server_submit(self.h, C.byref(desc), C.byref(opts), _ptr(eps), _ptr(f),
                                        float(tol), int(max_cycles), float(t_arrival), C.byref(t))
        if rc != QMG_OK:
            self._err(rc)
        self._n[t.value] = f.size
        return int(t.value)

    def poll(self, ticket: int):
        """(done, status name, solution or None, report dict, latency seconds)."""
        done = C.c_int(0)
        u = np.zeros(self._n[ticket])
        rep = SolveReport()
        lat = C.c_double(0.0)
        rc = self.lib.qmg_server_poll(self.h, C.c_uint64(ticket), C.byref(done), _ptr(u), C.byref(rep),
                                      C.byref(lat))
        if not done.value:
            if rc != QMG_OK:
                self._err(rc)
            return False, None, None, None, None
        del self._n[ticket]
        return True, STATUS_NAMES.get(rc, str(rc)), u, rep.as_dict(), float(lat.value)

    def drain(self):
        rc = self.lib.qmg_server_drain(self.h)
        if rc != QMG_OK:
            self._err(rc)

    def stats(self) -> dict:
        st = ServerStats()
        rc = self.lib.qmg_server_stats(self.h, C.byref(st))
        if rc != QMG_OK:
            self._err(rc)
        return st.as_dict()

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.qmg_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(dim: int, level: int, opts: SolverOpts) -> int:
    lib = load()
    nb = C.c_size_t(0)
    rc = lib.qmg_workspace_bytes(C.byref(GridDesc(int(dim), int(level))), C.byref(opts), C.byref(nb))
    if rc != QMG_OK:
        raise QmgError(rc, lib.qmg_last_error(None).decode())
    return int(nb.value)


def version() -> str:
    return load().qmg_version().decode()
