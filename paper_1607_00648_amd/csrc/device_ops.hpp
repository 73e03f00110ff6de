// Device-side building blocks: rediscretised Q1 stencil rows from per-cell
// coefficients, decoding of the hierarchical delta store, d-linear weights.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "qmg_internal.hpp"

namespace qmg {

template <int D>
struct Dim {
  static constexpr int NS = (D == 2) ? 9 : 27;   // stencil entries
  static constexpr int NC = 1 << D;              // cells around a vertex / parents of a vertex
};

__host__ __device__ constexpr int off_x(int k) { return k % 3 - 1; }
__host__ __device__ constexpr int off_y(int k) { return (k / 3) % 3 - 1; }
__host__ __device__ constexpr int off_z(int k) { return k / 9 - 1; }

// Q1 element-matrix entry of two corners of one cell with unit scalar
// coefficient, as a function of how many coordinates differ (tensor product of
// the 1D stiffness [[1,-1],[-1,1]] and mass [[1/3,1/6],[1/6,1/3]]), without the
// h^(d-2) factor.
__host__ __device__ constexpr double kref(int d, int ndiff) {
  return d == 2 ? (ndiff == 0 ? 2.0 / 3.0 : ndiff == 1 ? -1.0 / 6.0 : -1.0 / 3.0)
                : (ndiff == 0 ? 1.0 / 3.0 : ndiff == 1 ? 0.0 : -1.0 / 12.0);
}

template <int D>
__host__ __device__ constexpr int ndiff_of(int k) {
  return (off_x(k) != 0) + (off_y(k) != 0) + (D == 3 ? (off_z(k) != 0) : 0);
}

// Cell s (s = sx + 2 sy + 4 sz) around vertex v is the cell with low corner
// v - s; it contains the neighbour v + o iff s_i + o_i is 0 or 1 on every axis.
template <int D>
__host__ __device__ constexpr bool cell_has(int s, int k) {
  return (s & 1) + off_x(k) >= 0 && (s & 1) + off_x(k) <= 1 &&
         ((s >> 1) & 1) + off_y(k) >= 0 && ((s >> 1) & 1) + off_y(k) <= 1 &&
         (D == 2 || (((s >> 2) & 1) + off_z(k) >= 0 && ((s >> 2) & 1) + off_z(k) <= 1));
}

__host__ __device__ inline int64_t slot_off(const Lat& L, int ox, int oy, int oz) {
  return (int64_t)ox + (int64_t)oy * L.pitch + (int64_t)oz * L.plane;
}

// Rediscretised stencil row of vertex v (interior) from the coefficients of its
// 2^d cells (eq. "03_solver:stencils": sum over cells of element-matrix rows).
// Entries pointing at boundary vertices are kept (they multiply u = 0).
template <int D, typename T>
__device__ inline void geom_row(const T* __restrict__ eps, int64_t v, const Lat& L,
                                T (&a)[Dim<D>::NS]) {
  T ce[Dim<D>::NC];
#pragma unroll
  for (int s = 0; s < Dim<D>::NC; ++s)
    ce[s] = eps[v - slot_off(L, s & 1, (s >> 1) & 1, (s >> 2) & 1)];
  const T hs = (D == 3) ? (T)L.h : (T)1;
#pragma unroll
  for (int k = 0; k < Dim<D>::NS; ++k) {
    if (kref(D, ndiff_of<D>(k)) == 0.0) {
      a[k] = (T)0;
      continue;
    }
    T e = (T)0;
#pragma unroll
    for (int s = 0; s < Dim<D>::NC; ++s)
      if (cell_has<D>(s, k)) e += ce[s];
    a[k] = hs * (T)kref(D, ndiff_of<D>(k)) * e;
  }
}

// One rediscretised entry a(v, o_k) with Dirichlet entries dropped (v and v+o
// must both be interior for a non-zero value).  Used by the build kernels.
template <int D>
__device__ inline double geom_entry(const double* __restrict__ eps, int64_t v, int i, int j, int kk,
                                    int k, const Lat& L) {
  const int ox = off_x(k), oy = off_y(k), oz = (D == 3) ? off_z(k) : 0;
  const int n = L.n;
  if (i + ox <= 0 || i + ox >= n || j + oy <= 0 || j + oy >= n) return 0.0;
  if (D == 3 && (kk + oz <= 0 || kk + oz >= n)) return 0.0;
  const double w = kref(D, ndiff_of<D>(k));
  if (w == 0.0) return 0.0;
  double e = 0.0;
  for (int s = 0; s < Dim<D>::NC; ++s)
    if (cell_has<D>(s, k)) e += eps[v - slot_off(L, s & 1, (s >> 1) & 1, (s >> 2) & 1)];
  return ((D == 3) ? L.h : 1.0) * w * e;
}

// Decoding of one stored delta value.
template <int FMT>
struct Dec;
template <>
struct Dec<F64> {
  using S = double;
  __device__ static double get(const void* p, int64_t i) { return ((const double*)p)[i]; }
};
template <>
struct Dec<F32> {
  using S = float;
  __device__ static float get(const void* p, int64_t i) { return ((const float*)p)[i]; }
};
template <>
struct Dec<F16> {
  using S = _Float16;
  __device__ static float get(const void* p, int64_t i) { return (float)((const _Float16*)p)[i]; }
};
template <>
struct Dec<BF16> {
  using S = uint16_t;
  __device__ static float get(const void* p, int64_t i) {
    return __uint_as_float(((uint32_t)((const uint16_t*)p)[i]) << 16);
  }
};

// bpa codec (Sect. 5): x ~ m 2^e with e in one signed byte and m a
// two's-complement integer of bpa - 1 bytes, e the smallest exponent for which
// the rounded (nearest-even) m fits; bpa 0, x = 0 and exponents below -128
// code zero.  Every step is exact, so host and device agree bit for bit.
__host__ __device__ inline double bpa_code(double x, int bpa, int& e_out, long long& m_out) {
  e_out = 0;
  m_out = 0;
  if (bpa == 0 || x == 0.0) return 0.0;
  const int bits = 8 * (bpa - 1) - 1;
  const double mmax = ldexp(1.0, bits) - 1.0;
  int E = 0;
  frexp(fabs(x), &E);
  int e = E - bits;
  double m = rint(ldexp(x, -e));
  if (fabs(m) > mmax) {
    ++e;
    m = rint(ldexp(x, -e));
  }
  if (e < -128) return 0.0;
  e_out = e > 127 ? 127 : e;
  m_out = (long long)m;
  return ldexp(m, e);
}
// Smallest bpa in {0, 2, ..., 8} that codes every entry within eps_mf.
__host__ __device__ inline int bpa_width(const double* x, int n, double eps_mf) {
  int e;
  long long m;
  for (int w = 0; w <= 8; w += (w == 0 ? 2 : 1)) {
    bool ok = true;
    for (int k = 0; k < n; ++k) ok = ok && fabs(bpa_code(x[k], w, e, m) - x[k]) <= eps_mf;
    if (ok) return w;
  }
  return 8;
}
// Entry k of lane `lane` in a BPA block (see Store).
__device__ inline double bpa_entry(const Store& st, int32_t cb, int nent, int k, int lane) {
  const int64_t ow = st.boff[cb];
  const int W = (int)(ow >> 56);
  const uint8_t* p = (const uint8_t*)st.payload + (ow & ((int64_t(1) << 56) - 1)) + lane;
  const int e = (int8_t)p[k * kSeg];
  uint64_t u = 0;
  for (int j = 0; j < W - 1; ++j) u |= (uint64_t)p[(int64_t)(nent * (1 + j) + k) * kSeg] << (8 * j);
  const int sh = 64 - 8 * (W - 1);
  const int64_t m = (int64_t)(u << sh) >> sh;
  return ldexp((double)m, e);
}

// Adds the stored delta of vertex v (nent entries) to a[] when its block is
// non-zero.  The payload is read unconditionally (block 0 stands in for a zero
// block; stores are allocated in full) and selected, so that the loads of
// several vertices can be in flight together.
template <int FMT, int NENT, typename T>
__device__ inline void add_delta(const Store& st, int64_t v, T (&a)[NENT]) {
  const int32_t cb = st.blk[v / kSeg];
  const int64_t cbl = cb >= 0 ? cb : 0;
  const int lane = (int)(v % kSeg);
  const int64_t base = cbl * NENT * kSeg + lane;
  if constexpr (FMT == BPA) {
    // variable-width blocks: nothing to read ahead for a zero block
    if (cb >= 0) {
#pragma unroll
      for (int k = 0; k < NENT; ++k) a[k] += (T)bpa_entry(st, cb, NENT, k, lane);
    }
  } else if constexpr (FMT == F16) {
    const int e = st.scale[cbl * kSeg + lane];
#pragma unroll
    for (int k = 0; k < NENT; ++k) {
      const T dv = (T)ldexpf(Dec<FMT>::get(st.payload, base + (int64_t)k * kSeg), e);
      a[k] = cb >= 0 ? a[k] + dv : a[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < NENT; ++k) {
      const T dv = (T)Dec<FMT>::get(st.payload, base + (int64_t)k * kSeg);
      a[k] = cb >= 0 ? a[k] + dv : a[k];
    }
  }
}

// Tile of this workgroup.  Workgroups are dispatched round-robin over the 8
// XCDs, each with its own L2; the dispatch index is remapped so that every XCD
// walks one contiguous range of tiles (x tiles fastest, then rows, then
// planes), and the halo rows a tile shares with the tile above or below are
// mostly reread from the same L2.  t is the tile's linear index.
struct Tile {
  int x, y, z;
  unsigned t;
};
__device__ inline Tile xcd_tile() {
  constexpr unsigned kXcd = 8;
  const unsigned nx = gridDim.x, ny = gridDim.y;
  const unsigned N = nx * ny * gridDim.z;
  const unsigned b = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const unsigned q = N / kXcd, r = N % kXcd, k = b % kXcd;
  Tile T;
  T.t = k * q + min(k, r) + b / kXcd;
  T.x = (int)(T.t % nx);
  T.y = (int)((T.t / nx) % ny);
  T.z = (int)(T.t / (nx * ny));
  return T;
}

// d-linear weight of the parent at floor(f/3) + kappa along one axis, r = f mod 3.
__host__ __device__ constexpr double dlin1(int r, int kappa) {
  return kappa == 0 ? (r == 0 ? 1.0 : r == 1 ? 2.0 / 3.0 : 1.0 / 3.0)
                    : (r == 0 ? 0.0 : r == 1 ? 1.0 / 3.0 : 2.0 / 3.0);
}

}  // namespace qmg
