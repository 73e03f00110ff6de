"""Hierarchical operator store (oracle, FP64 with emulated quantisation).

Sect. 5 ("Stencil compression"): hierarchical operators
A_hat = A - A_rediscretised and P_hat = P - P_dlinear (R_hat = P_hat^T) are
small for smooth coefficients; a vertex whose hierarchical operator is zero
drops its stencil, otherwise the entries are stored compressed.

The IEEE formats here replace the paper's byte-stream codec (a reading of
the paper): the deltas are rounded to nearest-even in FP64, FP32, BF16 or
FP16.  Rounding rules, fixed so that both the oracle and the GPU take the same
decisions:

* FP32: one rounding of the FP64 delta.
* BF16: round the FP64 delta to FP32, then FP32 to BF16 (nearest-even).
* FP16: per stencil (per vertex) a power-of-two scale 2^e with e the smallest
  integer such that max|delta| <= 2^(15+e); the scaled FP64 value delta/2^e is
  rounded to FP32 and then to FP16 (nearest-even).  The paper stores one exponent
  byte per entry (m * 2^e); one exponent per stencil is a reading of the paper.
* bpa (Sect. 5, the paper's own codec): every entry x of a vertex's delta is
  stored as m * 2^e, e in one signed byte and m a signed integer of bpa - 1
  bytes; per vertex bpa is the smallest of {0, 2, 3, ..., 8} for which every
  entry satisfies |m 2^e - x| <= eps_mf (bpa 0: the vertex stores nothing and
  its delta counts as zero).  Readings: m is two's complement, so
  |m| <= 2^(8(bpa-1)-1) - 1; e is the smallest integer for which the rounded
  (nearest-even) m = rint(x / 2^e) fits; an entry whose e would fall below
  -128 is stored as zero (its value is below 2^-72); the set {0, 2, ..., 8}
  has eight members, three bits per operator.
* A vertex's delta counts as zero when max|delta| <= EPS_ZERO * max|A_geom row|
  with EPS_ZERO = 2^-40 (about 9e-13).  Galerkin/BoxMG reproduce the
  rediscretisation only to rounding for constant coefficients, and that
  rounding compounds over the levels (several hundred ulp of the row scale after
  three Galerkin products); 2^-40 leaves a wide margin above it while staying far
  below any iterate precision.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.
"""
from __future__ import annotations

import numpy as np

EPS_ZERO = 2.0 ** -40


def hier_deltas(A_stencil, Ageom_stencil):
    """A_hat = A - A_geom per vertex and entry (stencil arrays)."""
    return np.asarray(A_stencil) - np.asarray(Ageom_stencil)


def delta_zero(delta, geom, axis=0):
    """True where a vertex's delta (entries along ``axis``) counts as zero."""
    mx = np.max(np.abs(delta), axis=axis)
    scale = np.max(np.abs(geom), axis=axis)
    return mx <= EPS_ZERO * scale


def _bf16_from_f32(x32):
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    r = ((u + bias) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def fp16_exponent(maxabs):
    """Smallest integer e with maxabs <= 2^(15+e) (0 for maxabs == 0)."""
    maxabs = np.asarray(maxabs, dtype=np.float64)
    m, E = np.frexp(maxabs)                 # maxabs = m * 2^E, m in [0.5, 1)
    e = np.where(m == 0.5, E - 16, E - 15)
    e = np.where(maxabs == 0.0, 0, e)
    return e.astype(np.int64)


def quantise(delta, fmt, axis=0):
    """Round hierarchical deltas to ``fmt`` in {"fp64","fp32","bf16","fp16"} and
    return the values the store reconstructs (as FP64).  For "fp16" the scale is
    chosen per vertex over the entries along ``axis``."""
    delta = np.asarray(delta, dtype=np.float64)
    if fmt == "fp64":
        return delta.copy()
    if fmt == "fp32":
        return delta.astype(np.float32).astype(np.float64)
    if fmt == "bf16":
        return _bf16_from_f32(delta.astype(np.float32)).astype(np.float64)
    if fmt == "fp16":
        e = fp16_exponent(np.max(np.abs(delta), axis=axis))
        scale = np.ldexp(1.0, np.expand_dims(e, axis))
        scaled = delta / scale                      # exact (power of two)
        q = scaled.astype(np.float32).astype(np.float16).astype(np.float64)
        return q * scale
    raise ValueError(fmt)


BPA_WIDTHS = (0, 2, 3, 4, 5, 6, 7, 8)


def bpa_value(x, bpa):
    """f_bpa(x) = m 2^e elementwise (see module notes); also returns e and m."""
    x = np.asarray(x, dtype=np.float64)
    if bpa == 0:
        z = np.zeros(x.shape, dtype=np.int64)
        return np.zeros_like(x), z, z
    bits = 8 * (bpa - 1) - 1                  # magnitude bits of m
    mmax = 2.0 ** bits - 1.0
    _, E = np.frexp(np.abs(x))                # |x| = f 2^E, f in [0.5, 1)
    e = E.astype(np.int64) - bits             # |x| / 2^e in [2^(bits-1), 2^bits)
    m = np.rint(np.ldexp(x, -e))
    over = np.abs(m) > mmax                   # rounding reached 2^bits
    e = np.where(over, e + 1, e)
    m = np.rint(np.ldexp(x, -e))
    zero = (x == 0.0) | (e < -128)
    e = np.where(zero, 0, e)
    m = np.where(zero, 0.0, m)
    if np.any(e > 127):
        raise ValueError("delta too large for a one-byte exponent")
    return np.ldexp(m, e), e, m.astype(np.int64)


def bpa_encode(delta, eps_mf, axis=0):
    """Per vertex (entries along ``axis``) the smallest bpa whose values are
    all within eps_mf of the delta; returns (decoded values, bpa per vertex)."""
    delta = np.moveaxis(np.asarray(delta, dtype=np.float64), axis, 0)
    out = np.zeros_like(delta)
    width = np.full(delta.shape[1:], -1, dtype=np.int64)
    for w in BPA_WIDTHS:
        q = bpa_value(delta, w)[0]
        ok = (np.max(np.abs(q - delta), axis=0) <= eps_mf) & (width < 0)
        out[:, ok] = q[:, ok]
        width[ok] = w
    return np.moveaxis(out, 0, axis), width


def P_to_parent_weights(P, d, level_f):
    """Per fine lattice vertex f the weights of its 2^d candidate parents
    V = floor(f/3) + kappa (kappa in {0,1}^d, x fastest), from a sparse P
    (fine x coarse interior unknowns).  Shape (2^d,) + (nf+1,)*d."""
    import itertools
    import scipy.sparse as sp
    from .fem import _unknown_numbering
    nf = 3 ** level_f
    nc = nf // 3
    numf = _unknown_numbering(d, level_f)
    numc = _unknown_numbering(d, level_f - 1)
    P = sp.csr_matrix(P)
    W = np.zeros((2 ** d,) + (nf + 1,) * d)
    grid = np.stack(np.meshgrid(*([np.arange(nf + 1)] * d), indexing="ij")[::-1], -1)  # [..., i] coord i
    grid = grid.reshape(-1, d)          # rows in C order of (z,y,x); columns x,y,z
    frow = numf.reshape(-1)
    for ki, kappa in enumerate([tuple(reversed(t)) for t in itertools.product((0, 1), repeat=d)]):
        Vc = grid // 3 + np.array(kappa)
        inside = np.all(Vc <= nc, axis=1)
        ccol = np.full(len(grid), -1)
        ccol[inside] = numc[tuple(Vc[inside][:, i] for i in reversed(range(d)))]
        ok = (frow >= 0) & (ccol >= 0)
        vals = np.zeros(len(grid))
        vals[ok] = np.asarray(P[frow[ok], ccol[ok]]).ravel()
        W[ki] = vals.reshape((nf + 1,) * d)
    return W
