// Per-vertex operations of one level shared by the per-level kernels and the
// fused single-workgroup coarse-level kernel: stencil rows (rediscretised on
// the fly, plus stored deltas, or plain FP64), prolongation weights, and the
// restriction / prolongation gathers.
#pragma once

#include "device_ops.hpp"

namespace qmg {

// Stencil row of interior vertex v as the smoother applies it.
template <int D, typename T, int SRC, int FMT>
__device__ inline void op_row(const T* __restrict__ eps, const Store& A, const Lat& L, int64_t v,
                              T (&a)[Dim<D>::NS]) {
  constexpr int NS = Dim<D>::NS;
  if (SRC == SRC_PLAIN) {
    const double* Ad = (const double*)A.dense;
#pragma unroll
    for (int k = 0; k < NS; ++k) a[k] = (T)Ad[(int64_t)k * L.nslot + v];
  } else {
    geom_row<D, T>(eps, v, L, a);
    if (SRC == SRC_HIER) add_delta<FMT, NS, T>(A, v, a);
  }
}

// sum_k a_k u(v + o_k)
template <int D, typename T, int SRC>
__device__ inline T row_dot(const T (&a)[Dim<D>::NS], const T* __restrict__ u, const Lat& L, int64_t v) {
  T au = (T)0;
#pragma unroll
  for (int k = 0; k < Dim<D>::NS; ++k) {
    if (D == 3 && SRC == SRC_GEOM && kref(3, ndiff_of<3>(k)) == 0.0) continue;
    au += a[k] * u[v + slot_off(L, off_x(k), off_y(k), D == 3 ? off_z(k) : 0)];
  }
  return au;
}

// Weight of the parent floor(f/3)+kappa at fine vertex f (slot vf; r = f mod 3).
template <int D, int SRC, int FMT>
__device__ inline double pweight(const Store& P, const Lat& Lf, int64_t vf, int rx, int ry, int rz,
                                 int kap) {
  const int kx = kap & 1, ky = (kap >> 1) & 1, kz = (kap >> 2) & 1;
  if (SRC == SRC_PLAIN) return ((const double*)P.dense)[(int64_t)kap * Lf.nslot + vf];
  double w = dlin1(rx, kx) * dlin1(ry, ky) * (D == 3 ? dlin1(rz, kz) : 1.0);
  if (SRC == SRC_HIER) {
    // the payload is read unconditionally (block 0 stands in for a zero
    // block, the store is allocated in full) and selected, so that the loads
    // of many weights can be in flight together
    const int32_t cb = P.blk[vf / kSeg];
    const int64_t cbl = cb >= 0 ? cb : 0;
    const int lane = (int)(vf % kSeg);
    if constexpr (FMT == BPA) {
      w = cb >= 0 ? w + bpa_entry(P, cb, Dim<D>::NC, kap, lane) : w;
    } else {
      const int64_t idx = (cbl * Dim<D>::NC + kap) * kSeg + lane;
      double dv = (double)Dec<FMT>::get(P.payload, idx);
      if (FMT == F16) dv = ldexp(dv, (int)P.scale[cbl * kSeg + lane]);
      w = cb >= 0 ? w + dv : w;
    }
  }
  return w;
}


// (P^T r)(V) for interior coarse vertex (I,J,K): gather over fine f = 3V + o,
// o in [-2,2]^d, with R = P^T.
template <int D, typename T, int SRC, int FMT>
__device__ inline T restrict_at(const Lat& Lf, const T* __restrict__ r, const Store& P, int I, int J, int K) {
  const int64_t vf0 = 3 * I + (int64_t)3 * J * Lf.pitch + (int64_t)3 * K * Lf.plane;
  T acc = (T)0;
  const int zlo = (D == 3) ? -2 : 0, zhi = (D == 3) ? 2 : 0;
#pragma unroll
  for (int oz = zlo; oz <= zhi; ++oz)
#pragma unroll
    for (int oy = -2; oy <= 2; ++oy)
#pragma unroll
      for (int ox = -2; ox <= 2; ++ox) {
        const int64_t vf = vf0 + slot_off(Lf, ox, oy, oz);
        const int kap = (ox < 0 ? 1 : 0) | (oy < 0 ? 2 : 0) | (oz < 0 ? 4 : 0);
        double w;
        if (SRC == SRC_GEOM) {
          w = (1.0 - abs(ox) / 3.0) * (1.0 - abs(oy) / 3.0) * (D == 3 ? (1.0 - abs(oz) / 3.0) : 1.0);
        } else {
          w = pweight<D, SRC, FMT>(P, Lf, vf, (ox + 3) % 3, (oy + 3) % 3, (oz + 3) % 3, kap);
        }
        acc += (T)w * r[vf];
      }
  return acc;
}

// (P e)(f) for interior fine vertex (i,j,k) at slot vf.
template <int D, typename T, int SRC, int FMT>
__device__ inline T prolong_at(const Lat& Lf, const Lat& Lc, const T* __restrict__ ec, const Store& P,
                               int i, int j, int kz, int64_t vf) {
  const int qx = i / 3, qy = j / 3, qz = kz / 3;
  const int rx = i - 3 * qx, ry = j - 3 * qy, rz = kz - 3 * qz;
  const int64_t vc = qx + (int64_t)qy * Lc.pitch + (int64_t)qz * Lc.plane;
  T acc = (T)0;
#pragma unroll
  for (int kap = 0; kap < Dim<D>::NC; ++kap) {
    const int kx = kap & 1, ky = (kap >> 1) & 1, kk = (kap >> 2) & 1;
    if ((kx && rx == 0) || (ky && ry == 0) || (kk && rz == 0)) continue;
    const double w = pweight<D, SRC, FMT>(P, Lf, vf, rx, ry, rz, kap);
    acc += (T)w * ec[vc + slot_off(Lc, kx, ky, kk)];
  }
  return acc;
}

}  // namespace qmg
