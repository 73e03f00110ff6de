"""Multigrid hierarchy, V-cycle and the outer loops (oracle).

* Algorithm 1 / Sect. 4.1: multiplicative V(mu_pre, mu_post) cycles with damped
  point Jacobi, u <- u + omega diag(A)^-1 (b - A u), out of place.
* Sect. 4.3: coarse operators A_{l-1} = P^T A_l P (Galerkin and BoxMG) or the
  rediscretisation (geometric); the coarsest level moves up when a Galerkin
  operator fails the diagonal check.
* Results section ("/e"): an exact coarsest-level solve; otherwise mu_pre+mu_post
  Jacobi sweeps on the coarsest level.
* Sect. 4.3 (dynamic coarsest level): between two cycles the coarsest level
  moves one level up when the residual stagnates or grows (``raise_coarsest``).
* Sect. "Spacetree block smoothers": block Jacobi BJ(m) runs m Gauss-Seidel
  sweeps on the (k-1)^d iota-vertices of every 3^d patch and Jacobi on the
  c- and gamma-vertices (``block_jacobi``).

Readings:

* Regular grids use the correction scheme: r = b - A u, b_{l-1} = P^T r,
  u_{l-1} = 0, recurse, u += P u_{l-1}.  For Galerkin operators this produces the
  same iterates as the paper's FAS/HTMG form (A_{l-1} I u cancels R A P I u), and
  for rediscretised coarse operators it equals classic FAS, which keeps the fine
  solution a fixed point.
* The coarsest level is solved exactly when it has at most ``direct_max``
  unknowns (COARSE_DIRECT_MAX by default; a dense LU factorisation up to that
  size, a sparse LU factorisation above it, both library routines), otherwise
  by mu_pre + mu_post Jacobi sweeps from zero.
* The relative residual is the unweighted 2-norm over interior unknowns relative
  to ||b||_2 (the paper reduces ||r||_2 by 1e8).
* Stagnation is read as ||r_k|| > theta ||r_{k-1}|| for a threshold theta
  (an option; the paper names none), checked after every cycle that has not
  reached the tolerance, ||r_0|| being the residual of the start value.  The
  level moves up to L - 1 at most (the base level on an adaptive grid); the new
  coarsest level is solved exactly with its own operator when it has at most
  COARSE_DIRECT_MAX unknowns, otherwise by mu_pre + mu_post sweeps, and the
  raise lasts for the rest of the hierarchy's life.
* Additive cycles (Alg. 2 and the additive multigrid appendix) in their
  unpipelined form: one cycle restricts the fine residual down the whole
  hierarchy (r_{l-1} = P_l^T r_l), takes one damped Jacobi step from zero on
  every level (an exact solve on the coarsest level when it is direct), and
  adds the prolongated sum of the corrections to the fine iterate.  The
  paper's traversal pipelines this across half a grid sweep; the iterates
  per cycle are the same.  Damping is constant (omega on every level) or
  exponential (omega^(L - l + 1) on level l).
* BPX cycles (Alg. 3) in the same unpipelined form: the paper's helper i
  carries the level's Jacobi update at the c-points, which the level does not
  apply; the finer level subtracts its prolongation at the other vertices.
  Per cycle this gives e_l = d_l + P_l (e_{l-1} - I_l d_l), I_l the injection
  to the c-points, so every vertex is updated by the coarsest level that
  holds it and the finer levels add only their hierarchical surplus
  d_l - P_l I_l d_l.
* Block Jacobi readings: a patch is the 3^d block of vertices of one cell of
  the next coarser level; its iota-vertices are those with no coordinate
  divisible by 3.  One BJ(m) step first runs m lexicographic (x fastest)
  Gauss-Seidel sweeps, undamped, over each patch's iota-vertices, with every
  other value held, and then the damped Jacobi update on the c- and
  gamma-vertices from the iterate that already holds the new iota values; the
  iota-vertices keep their Gauss-Seidel values.  Patches do not share
  iota-vertices and no iota-vertex is a stencil neighbour of another patch's,
  so their order does not matter.  The smoother serves every smoothing step
  of the cycle (the paper's traversal could not use it while coarsening; an
  explicit cycle has no such limit), the coarsest level's sweeps included.
* Mixed precision (not in the paper): an FP64 defect-correction loop
  x += V32(fp32(b - A x)) whose inner V-cycles run in FP32 on operators rebuilt
  from quantised hierarchical deltas (see ``store``); the coarsest solve of the
  inner cycle stays in FP64.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import (geometric_stencil, convection_stencil, stencil_to_csr, csr_to_stencil, coarsen_eps)
from .transfer import dlinear_P, boxmg_P, injection_R, aggregation_R
from .galerkin import rap, definiteness_violations
from .store import quantise, delta_zero, EPS_ZERO, fp16_exponent, bpa_value, bpa_encode, BPA_WIDTHS

COARSE_DIRECT_MAX = 1024
COARSE_DIRECT_LIMIT = 26 ** 3     # the largest exact coarsest solve offered (3D level 3)


def factor_coarse(A, direct_max=COARSE_DIRECT_MAX):
    """Factorisation of the coarsest operator for its exact solve, or None
    when the level is larger than ``direct_max`` (it is then smoothed)."""
    n = A.shape[0]
    if n > direct_max:
        return None
    if n <= COARSE_DIRECT_MAX:
        return sla.lu_factor(A.toarray().astype(np.float64))
    return spla.splu(sp.csc_matrix(A, dtype=np.float64))


def coarse_solve(fac, b):
    """x = A_c^-1 b with a factorisation from ``factor_coarse``."""
    b = np.asarray(b, dtype=np.float64)
    if isinstance(fac, tuple):
        return sla.lu_solve(fac, b)
    return fac.solve(b)


class IndefiniteError(RuntimeError):
    """Every Galerkin coarse operator failed the diagonal check."""


@dataclasses.dataclass
class Hierarchy:
    d: int
    L: int
    lc: int
    transfer: str
    A: Dict[int, sp.csr_matrix]
    P: Dict[int, sp.csr_matrix]
    eps: Dict[int, np.ndarray]
    omega: float = 0.6
    mu_pre: int = 2
    mu_post: int = 2
    coarse_lu: Optional[tuple] = None
    dtype: type = np.float64
    smoother: str = "jacobi"       # "jacobi" or "block" (block Jacobi)
    bj_sweeps: int = 1             # Gauss-Seidel sweeps per patch in block Jacobi
    R: Optional[Dict[int, sp.csr_matrix]] = None   # restriction per level; None: P^T
    direct_max: int = COARSE_DIRECT_MAX            # largest coarsest level solved exactly

    def diag(self, l):
        return self.A[l].diagonal()


def build_hierarchy(eps, d, L, transfer="boxmg", lc=1, omega=0.6, mu_pre=2, mu_post=2,
                    check_definite=True, perturb=None, smoother="jacobi", bj_sweeps=1, v=None,
                    restriction="transpose", direct_max=COARSE_DIRECT_MAX):
    """Operators of all levels from the finest coefficients (Sect. 4.3, 3.4).

    ``v`` (per-cell velocities, shape (d,)+(n,)*d) adds the convection term of
    eq. (1) to the finest operator; its coarse operators then come from the
    Galerkin product only.  ``restriction`` "injection" (R = I) or
    "aggregation" (unit weights on the 3^d fine vertices within 1 of 3V) takes
    that R (the Petrov-Galerkin variants of the convection results) in R A P
    and in the cycle.  ``perturb`` (tests only) is applied to every Galerkin product
    before it is used; the tests pass one-ulp random noise to measure how far
    FP64 rounding alone moves the results (the noise floor of a parity
    comparison)."""
    if transfer not in ("geometric", "galerkin", "boxmg"):
        raise ValueError(transfer)
    if restriction not in ("transpose", "injection", "aggregation"):
        raise ValueError(restriction)
    if v is not None and transfer == "geometric":
        raise ValueError("convection needs Galerkin coarse operators")
    if restriction != "transpose" and transfer == "geometric":
        raise ValueError("injection and aggregation are Petrov-Galerkin restrictions")
    eps_l = {L: np.asarray(eps, dtype=np.float64)}
    for l in range(L, 0, -1):
        eps_l[l - 1] = coarsen_eps(eps_l[l], d)
    S = geometric_stencil(eps_l[L], d, L)
    if v is not None:
        S = S + convection_stencil(v, d, L)
    A = {L: stencil_to_csr(S, d, L)}
    P = {}
    R = None if restriction == "transpose" else {}
    lc_used = lc
    for l in range(L, lc, -1):
        if transfer == "boxmg":
            Pl = boxmg_P(csr_to_stencil(A[l], d, l), d, l)
        else:
            Pl = dlinear_P(d, l)
        if transfer == "geometric":
            Ac = stencil_to_csr(geometric_stencil(eps_l[l - 1], d, l - 1), d, l - 1)
        else:
            Rl = None
            if restriction == "injection":
                Rl = injection_R(d, l)
            elif restriction == "aggregation":
                Rl = aggregation_R(d, l)
            Ac = rap(A[l], Pl, Rl)
            if R is not None:
                R[l] = Rl
            if perturb is not None:
                Ac = perturb(Ac)
            if check_definite and len(definiteness_violations(Ac)) > 0:
                lc_used = l
                break
        P[l] = Pl
        A[l - 1] = Ac
    if lc_used >= L:
        raise IndefiniteError("coarsest level would reach the finest level")
    if R is not None:
        R = {l: R[l] for l in P}
    H = Hierarchy(d, L, lc_used, transfer, A, P, eps_l, omega, mu_pre, mu_post,
                  smoother=smoother, bj_sweeps=bj_sweeps, R=R, direct_max=direct_max)
    H.coarse_lu = factor_coarse(A[lc_used], direct_max)
    return H


def jacobi(A, diag, u, b, omega):
    return u + omega * (b - A @ u) / diag


def residual(A, u, b):
    return b - A @ u


def iota_positions(d, l):
    """Unknown indices of the iota-vertices of level l grouped by their
    position in the patch: entry p (lexicographic, x fastest over {1,2}^d)
    lists that vertex of every patch, patches in unknown order."""
    n = 3 ** l
    m = n - 1
    out = []
    for p in range(2 ** d):
        loc = [1 + ((p >> a) & 1) for a in range(d)]        # offsets inside the patch, x first
        axes = [np.arange(loc[a], n, 3) for a in range(d)]  # coordinates 3c + loc
        grids = np.meshgrid(*axes[::-1], indexing="ij")     # numpy order (z,) y, x
        idx = np.zeros(grids[0].shape, dtype=np.int64)
        for a in range(d):                                  # unknown index: (i-1) + m (j-1) + m^2 (k-1)
            idx += (grids[d - 1 - a] - 1) * m ** a
        out.append(idx.ravel())
    return out


def block_jacobi(A, D, u, b, omega, sweeps, d, l):
    """One block Jacobi step (see module notes): Gauss-Seidel on the
    iota-vertices of every patch, then damped Jacobi on the others."""
    u = np.array(u, copy=True)
    pos = iota_positions(d, l)
    for _ in range(sweeps):
        for idx in pos:          # the same patch position of every patch at once
            u[idx] = u[idx] + (b[idx] - A[idx] @ u) / D[idx]
    iota = np.zeros(len(u), dtype=bool)
    for idx in pos:
        iota[idx] = True
    out = u + omega * (b - A @ u) / D
    out[iota] = u[iota]
    return out


def smooth(H, l, A, D, u, b):
    """One smoothing step of the hierarchy's smoother on level l."""
    om = H.dtype(H.omega)
    if H.smoother == "block":
        return block_jacobi(A, D, u, b, om, H.bj_sweeps, H.d, l).astype(H.dtype)
    return jacobi(A, D, u, b, om)


def vcycle(H, l, u, b):
    """One V(mu_pre, mu_post) cycle on level l (correction scheme)."""
    A = H.A[l]
    dt = H.dtype
    D = A.diagonal()
    if l == H.lc:
        if H.coarse_lu is not None:
            return coarse_solve(H.coarse_lu, b).astype(dt)
        for _ in range(H.mu_pre + H.mu_post):
            u = smooth(H, l, A, D, u, b)
        return u
    for _ in range(H.mu_pre):
        u = smooth(H, l, A, D, u, b)
    r = b - A @ u
    P = H.P[l]
    Rl = P.T if H.R is None else H.R[l]
    bc = (Rl @ r).astype(dt)
    ec = vcycle(H, l - 1, np.zeros(P.shape[1], dtype=dt), bc)
    u = u + P @ ec
    for _ in range(H.mu_post):
        u = smooth(H, l, A, D, u, b)
    return u


def additive_cycle(H, u, b, damping="exp"):
    """One additive multigrid cycle (see module notes): u + sum over levels
    of P (omega_l D_l^-1 R r); the coarsest level is solved exactly when the
    hierarchy holds its factorisation."""
    L, lc = H.L, H.lc
    dt = H.dtype
    r = {L: (b - H.A[L] @ u).astype(dt)}
    for l in range(L, lc, -1):
        r[l - 1] = (H.P[l].T @ r[l]).astype(dt)

    def om(l):
        return dt(H.omega ** (L - l + 1) if damping == "exp" else H.omega)

    if H.coarse_lu is not None:
        e = coarse_solve(H.coarse_lu, r[lc]).astype(dt)
    else:
        e = om(lc) * r[lc] / H.A[lc].diagonal()
    for l in range(lc + 1, L + 1):
        e = om(l) * r[l] / H.A[l].diagonal() + H.P[l] @ e
    return u + e


def cpoint_positions(d, l):
    """Unknown index on level l of every interior vertex of level l-1 (its
    c-point: lattice coordinates times 3), in level l-1 unknown order."""
    mc, mf = 3 ** (l - 1) - 1, 3 ** l - 1
    axes = [3 * np.arange(1, mc + 1) - 1] * d            # fine coordinate minus one
    grids = np.meshgrid(*axes, indexing="ij")            # numpy order (z,) y, x
    idx = np.zeros(grids[0].shape, dtype=np.int64)
    for a in range(d):
        idx += grids[d - 1 - a] * mf ** a
    return idx.ravel()


def bpx_cycle(H, u, b, damping="const"):
    """One BPX cycle (Alg. 3, additive multigrid appendix) in its unpipelined
    form (see module notes): as ``additive_cycle``, but level l contributes
    only the hierarchical surplus of its Jacobi correction,
    d_l - P_l (d_l at the c-points), so a vertex takes its correction from the
    coarsest level that holds it."""
    L, lc = H.L, H.lc
    dt = H.dtype
    r = {L: (b - H.A[L] @ u).astype(dt)}
    for l in range(L, lc, -1):
        r[l - 1] = (H.P[l].T @ r[l]).astype(dt)

    def om(l):
        return dt(H.omega ** (L - l + 1) if damping == "exp" else H.omega)

    if H.coarse_lu is not None:
        e = coarse_solve(H.coarse_lu, r[lc]).astype(dt)
    else:
        e = om(lc) * r[lc] / H.A[lc].diagonal()
    for l in range(lc + 1, L + 1):
        dl = om(l) * r[l] / H.A[l].diagonal()
        e = dl + H.P[l] @ (e - dl[cpoint_positions(H.d, l)])
    return u + e


def solve_additive(H, b, tol=1e-8, max_cycles=1000, damping="exp", cycles=None, bpx=False):
    """Additive (or, with ``bpx``, BPX) cycles from zero until the relative
    residual reaches tol (or exactly ``cycles``).  Returns (u, relres
    history)."""
    A = H.A[H.L]
    u = np.zeros(A.shape[0])
    hist = []
    n = cycles if cycles is not None else max_cycles
    step = bpx_cycle if bpx else additive_cycle
    for _ in range(n):
        u = step(H, u, b, damping)
        hist.append(relres(A, u, b))
        if cycles is None and hist[-1] <= tol:
            break
    return u, hist


def raise_coarsest(H, top=None):
    """Dynamic coarsest level (Sect. 4.3): move l_c one level up, to ``top``
    (default L - 1) at most; the new coarsest level is solved with its own
    operator.  Returns whether the level moved."""
    top = H.L - 1 if top is None else top
    if H.lc + 1 > top:
        return False
    H.lc += 1
    Ac = H.A[H.lc]
    H.coarse_lu = factor_coarse(Ac, H.direct_max)
    return True


def stagnated(rr, rr_prev, theta, tol):
    """The trigger of the dynamic coarsest level: not converged, and the
    residual fell by less than the factor theta (or grew) over the cycle."""
    return theta > 0 and rr > tol and rr > theta * rr_prev


def relres(A, u, b):
    return float(np.linalg.norm(b - A @ u) / np.linalg.norm(b))


def solve(H, b, tol=1e-8, max_cycles=100, u0=None, cycles=None, stagnation=0.0):
    """V-cycles from u0 (default 0) until ||b - A u|| / ||b|| <= tol, or exactly
    ``cycles`` cycles when given.  With ``stagnation`` > 0 the coarsest level
    moves up after a cycle that reduced the residual by less than that factor.
    Returns (u, history of relres per cycle)."""
    A = H.A[H.L]
    u = np.zeros(A.shape[0]) if u0 is None else np.array(u0, dtype=np.float64)
    hist: List[float] = []
    prev = relres(A, u, b)
    n = cycles if cycles is not None else max_cycles
    for k in range(n):
        u = vcycle(H, H.L, u, b)
        hist.append(relres(A, u, b))
        if cycles is None and hist[-1] <= tol:
            break
        # the check runs only between two cycles
        if k + 1 < n and stagnated(hist[-1], prev, stagnation, tol):
            raise_coarsest(H)
        prev = hist[-1]
    return u, hist


def direct_solve(A, b):
    return spla.spsolve(sp.csc_matrix(A), b)


def quantised_hierarchy(H, fmt, eps_mf=None):
    """Hierarchy rebuilt from quantised hierarchical deltas:
    A_geom(eps_l) + q(A_hat_l) and P_dlin + q(P_hat_l), quantised per vertex as
    in ``store``; the finest operator is the geometric one (its delta is zero
    by construction).  For the IEEE formats it is the FP32 inner hierarchy of
    the mixed loop (pinned entry by entry by each format's rounding bound,
    and exactly for constant eps, in the oracle tests).  For
    "bpa" (with ``eps_mf``) it is an FP64 hierarchy, the form in which the
    paper solves with its codec.  An exact coarsest-level solve keeps the
    factorisation of the full operator."""
    d = H.d
    bpa = fmt == "bpa"
    if bpa and not (eps_mf is not None and eps_mf > 0):
        raise ValueError("bpa needs eps_mf > 0")
    dt = np.float64 if bpa else np.float32
    A32, P32 = {}, {}
    for l, Al in H.A.items():
        G = geometric_stencil(H.eps[l], d, l)
        if l == H.L:
            A32[l] = stencil_to_csr(G, d, l).astype(dt)
            continue
        S = csr_to_stencil(Al, d, l)
        dlt = S - G
        if bpa:
            q = bpa_encode(dlt, eps_mf, axis=0)[0]
        else:
            q = quantise(dlt, fmt, axis=0)
            q[:, delta_zero(dlt, G)] = 0.0
        A32[l] = stencil_to_csr(G + q, d, l).astype(dt)
    for l, Pl in H.P.items():
        Pd = dlinear_P(d, l)
        dP = sp.csr_matrix(Pl - Pd)
        dP.sum_duplicates()
        rows = np.repeat(np.arange(dP.shape[0]), np.diff(dP.indptr))
        vals = dP.data.copy()
        if bpa:
            width = np.full(dP.shape[0], -1)
            out = np.zeros_like(vals)
            for w in BPA_WIDTHS:
                qv = bpa_value(vals, w)[0]
                err = np.zeros(dP.shape[0])
                np.maximum.at(err, rows, np.abs(qv - vals))
                ok = (err <= eps_mf) & (width < 0)
                out[ok[rows]] = qv[ok[rows]]
                width[ok] = w
            q = sp.csr_matrix((out, dP.indices, dP.indptr), shape=dP.shape)
            P32[l] = (Pd + q).astype(dt).tocsr()
            continue
        if fmt == "fp16":
            mx = np.zeros(dP.shape[0])
            np.maximum.at(mx, rows, np.abs(vals))
            e = fp16_exponent(mx)
            sc = np.ldexp(1.0, e[rows])
            vals = (vals / sc).astype(np.float32).astype(np.float16).astype(np.float64) * sc
        else:
            vals = quantise(vals, fmt)
        # zero rows whose delta is negligible against the d-linear weights
        mxd = np.zeros(dP.shape[0])
        np.maximum.at(mxd, rows, np.abs(dP.data))
        mxp = np.asarray(abs(Pd).max(axis=1).todense()).ravel()
        zero = mxd <= EPS_ZERO * mxp
        vals[zero[rows]] = 0.0
        q = sp.csr_matrix((vals, dP.indices, dP.indptr), shape=dP.shape)
        P32[l] = (Pd + q).astype(dt).tocsr()
    Hq = Hierarchy(d, H.L, H.lc, H.transfer, A32, P32, H.eps, H.omega, H.mu_pre, H.mu_post,
                   H.coarse_lu, dt, H.smoother, H.bj_sweeps, direct_max=H.direct_max)
    return Hq


def mixed_solve(H, Hq, b, tol=1e-8, max_outer=100, inner_cycles=1, stagnation=0.0):
    """FP64 defect correction around FP32 inner V-cycles (see module notes).
    With ``stagnation`` > 0 the inner hierarchy's coarsest level moves up after
    an outer iteration that reduced the residual by less than that factor.
    Returns (x, relres history)."""
    A = H.A[H.L]
    x = np.zeros(A.shape[0])
    nb = np.linalg.norm(b)
    hist = []
    for _ in range(max_outer):
        r = b - A @ x
        rr = float(np.linalg.norm(r) / nb)
        hist.append(rr)
        if rr <= tol:
            break
        if len(hist) > 1 and stagnated(rr, hist[-2], stagnation, tol):
            raise_coarsest(Hq)
        r32 = r.astype(np.float32)
        e = np.zeros_like(r32)
        for _ in range(inner_cycles):
            e = vcycle(Hq, Hq.L, e, r32)
        x = x + e.astype(np.float64)
    return x, hist
