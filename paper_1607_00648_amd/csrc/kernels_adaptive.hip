// Kernels of the adaptive levels (finer than the complete base level).
//
// An adaptive level keeps the full lattice of its level but only the 64 x 4
// (x, y) tiles that hold vertices of existing cells are launched: blockIdx.x
// indexes a tile list.  Every slot carries its vertex class (Sect. 3): leaf
// (unrefined, an unknown), refined (a finer copy exists), hanging (fewer than
// 2^d cells of the level), or outside/boundary.  Smoothing and residuals act
// on leaf and refined vertices; hanging vertices hold the d-linear interpolant
// of the coarser level; refined coarse vertices receive the value of their
// finer copy and the FAS right-hand side.
#include "level_ops.hpp"
#include <hip/hip_ext.h>

namespace qmg {

namespace {

constexpr int TX = 64, TY = 4;

struct Slot {
  int i, j, k;
  int64_t v;
  bool valid;
};

template <int D>
__device__ inline Slot tile_slot(const Lat& L, const int32_t* __restrict__ tiles) {
  const int32_t* t = tiles + 3 * (int64_t)blockIdx.x;
  Slot s;
  s.i = t[0] * TX + threadIdx.x;
  s.j = t[1] * TY + threadIdx.y;
  s.k = (D == 3) ? t[2] : 0;
  s.valid = s.i <= L.n && s.j <= L.n;
  s.v = s.i + (int64_t)s.j * L.pitch + (int64_t)s.k * L.plane;
  return s;
}

__device__ inline bool active(int8_t t) { return t == VT_LEAF || t == VT_REFINED; }

__device__ inline double block_sum_256(double x) {
  __shared__ double red[4];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  const int t = threadIdx.x + threadIdx.y * TX;
  if ((t & 63) == 0) red[t >> 6] = x;
  __syncthreads();
  double s = 0.0;
  if (t == 0) s = ((red[0] + red[1]) + red[2]) + red[3];
  return s;
}

// mode 0: Jacobi sweep, 1: sweep from zero, 2: residual (0 off the active set)
template <int D, typename T, typename TO, int SRC, int FMT, int MODE>
__global__ __launch_bounds__(256) void k_ad_stencil(Lat L, const int32_t* __restrict__ tiles,
                                                    const int8_t* __restrict__ vt, const T* __restrict__ u,
                                                    const T* __restrict__ b, TO* __restrict__ out,
                                                    const T* __restrict__ eps, Store A, T omega,
                                                    double* __restrict__ partial) {
  constexpr int NS = Dim<D>::NS;
  const Slot s = tile_slot<D>(L, tiles);
  double sq = 0.0;
  if (s.valid) {
    const int8_t t = vt[s.v];
    if (active(t)) {
      T a[NS];
      op_row<D, T, SRC, FMT>(eps, A, L, s.v, a);
      if (MODE == 1) {
        out[s.v] = (TO)(omega * b[s.v] / a[NS / 2]);
      } else {
        const T res = b[s.v] - row_dot<D, T, SRC>(a, u, L, s.v);
        if (MODE == 0) {
          out[s.v] = (TO)(u[s.v] + omega * res / a[NS / 2]);
        } else {
          out[s.v] = (TO)res;
          if (t == VT_LEAF) sq = (double)res * (double)res;
        }
      }
    } else {
      // hanging / outside values travel with the iterate (zero from zero)
      out[s.v] = (MODE == 0) ? (TO)u[s.v] : (TO)0;
    }
  }
  if (partial != nullptr) {
    const double tot = block_sum_256(sq);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[blockIdx.x] = tot;
  }
}

// 3D adaptive levels: a workgroup of kBrickX x kBrickY threads (32 x 8; a
// wavefront covers two x-rows) owns one listed brick of as many slots and
// marches over its 16 interior planes.  Three planes of the
// iterate (brick plus a halo of one vertex) and two planes of cell
// coefficients ring through LDS, so each value comes from memory once per
// brick instead of once per neighbour.  Every thread updates the
// leaf or refined vertex at its position on each plane (same expressions and
// order as k_ad_stencil) and copies a hanging value (mode 0) or zeroes it
// (mode 2); other slots are not touched.  Workgroup w runs on XCD w % 8; the
// brick list (ordered z, y, x) is cut into eight contiguous ranges, one per
// XCD, so that neighbouring bricks share an L2.
constexpr int BX = kBrickX, BY = kBrickY, BZ = kBrickZ;
constexpr int BUW = BX + 2, BUH = BY + 2;  // iterate plane region: x0-1..x0+BX, y0-1..y0+BY
constexpr int BEW = BX + 1, BEH = BY + 1;  // cell plane region: x0-1..x0+BX-1, y0-1..y0+BY-1

template <typename T, typename TO, int SRC, int FMT, int MODE>
__global__ __launch_bounds__(BX * BY) void k_ad_march(Lat L, const int32_t* __restrict__ bricks, int nb,
                                                      const int8_t* __restrict__ vt, const T* __restrict__ u,
                                                      const T* __restrict__ b, TO* __restrict__ out,
                                                      const T* __restrict__ eps, Store A, T omega,
                                                      double* __restrict__ partial) {
  constexpr int NS = 27;
  constexpr int NT = BX * BY;
  static_assert(BUW * BUH <= 2 * NT && BEW * BEH <= 2 * NT, "two values per thread");
  __shared__ T up[3][BUW * BUH];
  __shared__ T ep[2][BEW * BEH];
  __shared__ double red[NT / 64];
  const int per = (nb + 7) / 8;
  const int bi = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (bi >= nb) return;  // the whole workgroup
  const int32_t* br = bricks + 3 * (int64_t)bi;
  const int n = L.n;
  const int x0 = br[0] * BX, y0 = br[1] * BY;
  const int k0 = 1 + br[2] * BZ, k1 = min(k0 + BZ, n);  // interior planes [k0, k1)
  const int tid = threadIdx.x;
  const int lx = tid % BX, ly = tid / BX;
  const int i = x0 + lx, j = y0 + ly;
  const bool inplane = i >= 1 && i < n && j >= 1 && j < n;
  auto fetch_u = [&](int k, T (&r)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + h * NT;
      const int x = x0 - 1 + e % BUW, y = y0 - 1 + e / BUW;
      r[h] = (e < BUW * BUH && x >= 0 && x <= n && y >= 0 && y <= n && k <= n)
                 ? u[x + (int64_t)y * L.pitch + (int64_t)k * L.plane] : (T)0;
    }
  };
  auto fetch_e = [&](int k, T (&r)[2]) {  // cells with low corner on plane k
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + h * NT;
      const int x = x0 - 1 + e % BEW, y = y0 - 1 + e / BEW;
      r[h] = (e < BEW * BEH && x >= 0 && x < n && y >= 0 && y < n && k < n)
                 ? eps[x + (int64_t)y * L.pitch + (int64_t)k * L.plane] : (T)0;
    }
  };
  auto put_u = [&](int k, const T (&r)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (tid + h * NT < BUW * BUH) up[k % 3][tid + h * NT] = r[h];
  };
  auto put_e = [&](int k, const T (&r)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (tid + h * NT < BEW * BEH) ep[k % 2][tid + h * NT] = r[h];
  };
  T ru[2] = {(T)0, (T)0}, re[2] = {(T)0, (T)0};
  fetch_u(k0 - 1, ru);
  put_u(k0 - 1, ru);
  fetch_u(k0, ru);
  put_u(k0, ru);
  fetch_u(k0 + 1, ru);
  if (SRC != SRC_PLAIN) {
    fetch_e(k0 - 1, re);
    put_e(k0 - 1, re);
    fetch_e(k0, re);
  }
  const int64_t vij = i + (int64_t)j * L.pitch;
  int8_t tnext = inplane ? vt[vij + (int64_t)k0 * L.plane] : (int8_t)VT_OUT;
  T bnext = (tnext == VT_LEAF || tnext == VT_REFINED) ? b[vij + (int64_t)k0 * L.plane] : (T)0;
  double sq = 0.0;
  for (int k = k0; k < k1; ++k) {
    const int8_t tv = tnext;
    const T bv = bnext;
    if (inplane && k + 1 < k1) {
      tnext = vt[vij + (int64_t)(k + 1) * L.plane];
      bnext = (tnext == VT_LEAF || tnext == VT_REFINED) ? b[vij + (int64_t)(k + 1) * L.plane] : (T)0;
    }
    put_u(k + 1, ru);
    if (k + 1 < k1) fetch_u(k + 2, ru);
    if (SRC != SRC_PLAIN) {
      put_e(k, re);
      if (k + 1 < k1) fetch_e(k + 1, re);
    }
    __syncthreads();
    const int64_t v = vij + (int64_t)k * L.plane;
    if (tv == VT_LEAF || tv == VT_REFINED) {
      T au = (T)0, dg = (T)0;
      if (SRC == SRC_GEOM) {
        // rediscretised entries formed and applied one at a time (no row
        // array held in registers); same operations in the same order
        T ce[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int sx = c & 1, sy = (c >> 1) & 1, sz = (c >> 2) & 1;
          ce[c] = ep[(k - sz) % 2][(ly + 1 - sy) * BEW + (lx + 1 - sx)];
        }
        const T hs = (T)L.h;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          if (kref(3, ndiff_of<3>(q)) == 0.0) continue;
          T e = (T)0;
#pragma unroll
          for (int c = 0; c < 8; ++c)
            if (cell_has<3>(c, q)) e += ce[c];
          const T aq = hs * (T)kref(3, ndiff_of<3>(q)) * e;
          if (q == NS / 2) dg = aq;
          au += aq * up[(k + off_z(q) + 3) % 3][(ly + 1 + off_y(q)) * BUW + (lx + 1 + off_x(q))];
        }
      } else {
        T a[NS];
        if (SRC == SRC_PLAIN) {
          const double* Ad = (const double*)A.dense;
#pragma unroll
          for (int q = 0; q < NS; ++q) a[q] = (T)Ad[(int64_t)q * L.nslot + v];
        } else {
          T ce[8];
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const int sx = c & 1, sy = (c >> 1) & 1, sz = (c >> 2) & 1;
            ce[c] = ep[(k - sz) % 2][(ly + 1 - sy) * BEW + (lx + 1 - sx)];
          }
          const T hs = (T)L.h;
#pragma unroll
          for (int q = 0; q < NS; ++q) {
            if (kref(3, ndiff_of<3>(q)) == 0.0) {
              a[q] = (T)0;
              continue;
            }
            T e = (T)0;
#pragma unroll
            for (int c = 0; c < 8; ++c)
              if (cell_has<3>(c, q)) e += ce[c];
            a[q] = hs * (T)kref(3, ndiff_of<3>(q)) * e;
          }
          add_delta<FMT, NS, T>(A, v, a);
        }
#pragma unroll
        for (int q = 0; q < NS; ++q)
          au += a[q] * up[(k + off_z(q) + 3) % 3][(ly + 1 + off_y(q)) * BUW + (lx + 1 + off_x(q))];
        dg = a[NS / 2];
      }
      const T uc = up[k % 3][(ly + 1) * BUW + lx + 1];
      if (MODE == 0) {
        out[v] = (TO)(uc + omega * (bv - au) / dg);
      } else {
        const T res = bv - au;
        out[v] = (TO)res;
        if (tv == VT_LEAF) sq += (double)res * (double)res;
      }
    } else if (tv == VT_HANGING) {
      out[v] = (MODE == 0) ? (TO)up[k % 3][(ly + 1) * BUW + lx + 1] : (TO)0;
    }
    __syncthreads();
  }
  if (partial != nullptr) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) sq += __shfl_xor(sq, m, 64);
    if ((tid & 63) == 0) red[tid >> 6] = sq;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < NT / 64; ++w) t += red[w];
      partial[bi] = t;
    }
  }
}

// (P (uc - sc))(f) at fine vertex (i,j,k), sc nullable; P d-linear (GEOM),
// stored deltas (HIER) or plain weights
template <int D, typename T, int PSRC, int PFMT>
__device__ inline T interp_at(const Lat& Lf, const Lat& Lc, const Store& P, int i, int j, int k, int64_t vf,
                              const T* __restrict__ uc, const T* __restrict__ sc) {
  const int qx = i / 3, qy = j / 3, qz = k / 3;
  const int rx = i - 3 * qx, ry = j - 3 * qy, rz = k - 3 * qz;
  const int64_t vc = qx + (int64_t)qy * Lc.pitch + (int64_t)qz * Lc.plane;
  T acc = (T)0;
#pragma unroll
  for (int kap = 0; kap < Dim<D>::NC; ++kap) {
    const int kx = kap & 1, ky = (kap >> 1) & 1, kk = (kap >> 2) & 1;
    if ((kx && rx == 0) || (ky && ry == 0) || (kk && rz == 0)) continue;
    const double w = pweight<D, PSRC, PFMT>(P, Lf, vf, rx, ry, rz, kap);
    const int64_t c = vc + slot_off(Lc, kx, ky, kk);
    acc += (T)w * (sc ? uc[c] - sc[c] : uc[c]);
  }
  return acc;
}

// hanging vertices of the fine level := interpolant P u_c of the coarse level
template <int D, typename T, int PSRC, int PFMT>
__global__ __launch_bounds__(256) void k_ad_hang(Lat Lf, Lat Lc, const int32_t* __restrict__ tiles,
                                                 const int8_t* __restrict__ vt, T* __restrict__ uf,
                                                 const T* __restrict__ uc, Store P) {
  const Slot s = tile_slot<D>(Lf, tiles);
  if (!s.valid || vt[s.v] != VT_HANGING) return;
  uf[s.v] = interp_at<D, T, PSRC, PFMT>(Lf, Lc, P, s.i, s.j, s.k, s.v, uc, (const T*)nullptr);
}

// The same over the list of the level's hanging vertices (a thin share of
// the tiles' slots: the band's boundary layer).
template <int D, typename T, int PSRC, int PFMT>
__global__ __launch_bounds__(256) void k_ad_hang_list(Lat Lf, Lat Lc, const int64_t* __restrict__ hang,
                                                      int64_t nh, T* __restrict__ uf, const T* __restrict__ uc,
                                                      Store P) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nh) return;
  const int64_t v = hang[q];
  int i, j, k = 0;
  int64_t r = v;
  if (D == 3) {
    k = (int)(v / Lf.plane);
    r = v - (int64_t)k * Lf.plane;
  }
  j = (int)(r / Lf.pitch);
  i = (int)(r - (int64_t)j * Lf.pitch);
  uf[v] = interp_at<D, T, PSRC, PFMT>(Lf, Lc, P, i, j, k, v, uc, (const T*)nullptr);
}

// refined coarse vertices := value of the finer copy (over coarse tiles)
template <int D, typename T>
__global__ __launch_bounds__(256) void k_ad_inject(Lat Lf, Lat Lc, const int32_t* __restrict__ tiles,
                                                   const int8_t* __restrict__ vtc, const T* __restrict__ uf,
                                                   T* __restrict__ uc) {
  const Slot s = tile_slot<D>(Lc, tiles);
  if (!s.valid || vtc[s.v] != VT_REFINED) return;
  uc[s.v] = uf[3 * s.i + (int64_t)3 * s.j * Lf.pitch + (int64_t)3 * s.k * Lf.plane];
}

// FAS right-hand side of refined coarse vertices: (P^T r)(V) + (A_c u_c)(V);
// r is zero off the fine active set
template <int D, typename T, int SRC, int FMT, int PSRC, int PFMT>
__global__ __launch_bounds__(256) void k_ad_fas_rhs(Lat Lf, Lat Lc, const int32_t* __restrict__ tiles,
                                                    const int8_t* __restrict__ vtc, const T* __restrict__ rf,
                                                    const T* __restrict__ uc, const T* __restrict__ epsc,
                                                    Store Ac, T* __restrict__ bc, Store P) {
  constexpr int NS = Dim<D>::NS;
  const Slot s = tile_slot<D>(Lc, tiles);
  if (!s.valid || vtc[s.v] != VT_REFINED) return;
  const T rr = restrict_at<D, T, PSRC, PFMT>(Lf, rf, P, s.i, s.j, s.k);
  T a[NS];
  op_row<D, T, SRC, FMT>(epsc, Ac, Lc, s.v, a);
  bc[s.v] = rr + row_dot<D, T, SRC>(a, uc, Lc, s.v);
}

// The same from the list of refined coarse vertices (interior indices), one
// wavefront per vertex: the lanes share the 5^d restriction terms and add
// them in a fixed shuffle tree; lane 0 adds the coarse row.
template <int D, typename T, int SRC, int FMT, int PSRC, int PFMT>
__global__ __launch_bounds__(256) void k_ad_fas_rhs_list(Lat Lf, Lat Lc, const int32_t* __restrict__ verts,
                                                         int64_t nverts, const T* __restrict__ rf,
                                                         const T* __restrict__ uc, const T* __restrict__ epsc,
                                                         Store Ac, T* __restrict__ bc, Store P) {
  constexpr int NS = Dim<D>::NS, NO = (D == 3) ? 125 : 25;
  const int lane = threadIdx.x & 63;
  const int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (idx >= nverts) return;  // uniform per wavefront
  const int m = Lc.n - 1;
  const int64_t vv = verts[idx];
  const int I = (int)(vv % m) + 1, J = (int)((vv / m) % m) + 1, K = (D == 3) ? (int)(vv / ((int64_t)m * m)) + 1 : 0;
  const int64_t vf0 = 3 * I + (int64_t)3 * J * Lf.pitch + (int64_t)3 * K * Lf.plane;
  T acc = (T)0;
  for (int o = lane; o < NO; o += 64) {
    const int ox = o % 5 - 2, oy = (o / 5) % 5 - 2, oz = (D == 3) ? o / 25 - 2 : 0;
    const int64_t vf = vf0 + slot_off(Lf, ox, oy, oz);
    const int kap = (ox < 0 ? 1 : 0) | (oy < 0 ? 2 : 0) | (oz < 0 ? 4 : 0);
    double w;
    if (PSRC == SRC_GEOM)
      w = (1.0 - abs(ox) / 3.0) * (1.0 - abs(oy) / 3.0) * (D == 3 ? (1.0 - abs(oz) / 3.0) : 1.0);
    else
      w = pweight<D, PSRC, PFMT>(P, Lf, vf, (ox + 3) % 3, (oy + 3) % 3, (oz + 3) % 3, kap);
    acc += (T)w * rf[vf];
  }
#pragma unroll
  for (int mm = 32; mm >= 1; mm >>= 1) acc += __shfl_xor(acc, mm, 64);
  if (lane == 0) {
    const int64_t v = I + (int64_t)J * Lc.pitch + (int64_t)K * Lc.plane;
    T a[NS];
    op_row<D, T, SRC, FMT>(epsc, Ac, Lc, v, a);
    bc[v] = acc + row_dot<D, T, SRC>(a, uc, Lc, v);
  }
}

// The FAS restriction by coarse cell: the fine vertices f with floor(f/3) = C
// (3^d of them, local 0..2 per axis) belong to cell C alone, and their
// parents are C's corners C + kappa, so (P^T r)(V) is the sum over the 2^d
// cells C = V - kappa of cell C's part for its corner kappa.  One group of
// threads per listed refined cell forms the 2^d parts (fine vertices in a
// fixed order); part[slot(C) * 2^d + kappa].
template <int D, typename T, int PSRC, int PFMT>
__global__ __launch_bounds__(256) void k_ad_restrict_cells(Lat Lf, Lat Lc, const int32_t* __restrict__ cells,
                                                           int64_t ncells, const T* __restrict__ rf,
                                                           T* __restrict__ part, Store P) {
  constexpr int NV = (D == 3) ? 27 : 9, NK = Dim<D>::NC, TPC = (D == 3) ? 32 : 16, CPB = 256 / TPC;
  __shared__ T prod[CPB][NV][NK];
  const int lc = threadIdx.x / TPC, q = threadIdx.x % TPC;
  const int64_t ci = (int64_t)blockIdx.x * CPB + lc;
  const bool on = ci < ncells;
  const int n = Lc.n;
  int Cx = 0, Cy = 0, Cz = 0;
  if (on) {
    const int64_t c = cells[ci];
    Cx = (int)(c % n);
    Cy = (int)((c / n) % n);
    Cz = (D == 3) ? (int)(c / ((int64_t)n * n)) : 0;
  }
  if (on && q < NV) {
    const int rx = q % 3, ry = (q / 3) % 3, rz = (D == 3) ? q / 9 : 0;
    const int64_t vf = (3 * Cx + rx) + (int64_t)(3 * Cy + ry) * Lf.pitch + (int64_t)(3 * Cz + rz) * Lf.plane;
    const T r = rf[vf];
#pragma unroll
    for (int kap = 0; kap < NK; ++kap) {
      const int kx = kap & 1, ky = (kap >> 1) & 1, kz = (kap >> 2) & 1;
      double w = 0.0;
      if (!((kx && rx == 0) || (ky && ry == 0) || (kz && rz == 0)))
        w = pweight<D, PSRC, PFMT>(P, Lf, vf, rx, ry, rz, kap);
      prod[lc][q][kap] = (T)w * r;
    }
  }
  __syncthreads();
  if (on && q < NK) {
    T acc = (T)0;
#pragma unroll
    for (int i = 0; i < NV; ++i) acc += prod[lc][i][q];
    const int64_t sc = Cx + (int64_t)Cy * Lc.pitch + (int64_t)Cz * Lc.plane;
    part[sc * NK + q] = acc;
  }
}

// FAS right-hand side of the listed refined coarse vertices from the cell
// parts: sum over the corners in order, then the coarse row.
template <int D, typename T, int SRC, int FMT>
__global__ __launch_bounds__(256) void k_ad_fas_rhs_cells(Lat Lc, const int32_t* __restrict__ verts, int64_t nverts,
                                                          const T* __restrict__ part, const T* __restrict__ uc,
                                                          const T* __restrict__ epsc, Store Ac, T* __restrict__ bc) {
  constexpr int NS = Dim<D>::NS, NK = Dim<D>::NC;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nverts) return;
  const int m = Lc.n - 1;
  const int64_t vv = verts[idx];
  const int I = (int)(vv % m) + 1, J = (int)((vv / m) % m) + 1, K = (D == 3) ? (int)(vv / ((int64_t)m * m)) + 1 : 0;
  T rr = (T)0;
#pragma unroll
  for (int kap = 0; kap < NK; ++kap) {
    const int64_t sc = (I - (kap & 1)) + (int64_t)(J - ((kap >> 1) & 1)) * Lc.pitch +
                       (D == 3 ? (int64_t)(K - ((kap >> 2) & 1)) * Lc.plane : 0);
    rr += part[sc * NK + kap];
  }
  const int64_t v = I + (int64_t)J * Lc.pitch + (int64_t)K * Lc.plane;
  T a[NS];
  op_row<D, T, SRC, FMT>(epsc, Ac, Lc, v, a);
  bc[v] = rr + row_dot<D, T, SRC>(a, uc, Lc, v);
}

// FAS correction: active fine vertices += P (u_c - saved_c)
template <int D, typename T, int PSRC, int PFMT>
__global__ __launch_bounds__(256) void k_ad_correct(Lat Lf, Lat Lc, const int32_t* __restrict__ tiles,
                                                    const int8_t* __restrict__ vt, T* __restrict__ uf,
                                                    const T* __restrict__ uc, const T* __restrict__ sc, Store P) {
  const Slot s = tile_slot<D>(Lf, tiles);
  if (!s.valid || !active(vt[s.v])) return;
  uf[s.v] += interp_at<D, T, PSRC, PFMT>(Lf, Lc, P, s.i, s.j, s.k, s.v, uc, sc);
}

// The same over the list of the level's leaf and refined vertices.
template <int D, typename T, int PSRC, int PFMT>
__global__ __launch_bounds__(256) void k_ad_correct_list(Lat Lf, Lat Lc, const int64_t* __restrict__ act,
                                                         int64_t na, T* __restrict__ uf, const T* __restrict__ uc,
                                                         const T* __restrict__ sc, Store P) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= na) return;
  const int64_t v = act[q];
  int i, j, k = 0;
  int64_t r = v;
  if (D == 3) {
    k = (int)(v / Lf.plane);
    r = v - (int64_t)k * Lf.plane;
  }
  j = (int)(r / Lf.pitch);
  i = (int)(r - (int64_t)j * Lf.pitch);
  uf[v] += interp_at<D, T, PSRC, PFMT>(Lf, Lc, P, i, j, k, v, uc, sc);
}

// Cell kernels over a whole level: thread (I, J) takes kCellPlanes planes of
// cells, with every load of a phase issued before any is used (a chain of
// dependent loads per plane leaves these launches bound by memory latency).
// A cell is read by a row only when one of its corners is a vertex of the
// level (leaf, refined or hanging): every row the kernels form, at such
// vertices, reads only such cells.  kCellPlanes is a multiple of 3, so that
// the thread's planes start on a parent plane.
constexpr int kCellPlanes = 15;

inline dim3 cell_walk_grid(const Lat& L) {
  return dim3((unsigned)(L.pitch / TX), (unsigned)((L.n + TY - 1) / TY),
              (unsigned)(L.d == 3 ? (L.n + kCellPlanes - 1) / kCellPlanes : 1));
}

// Bit q (q < K1 - K0): cell (I, J, K0 + q) is read by a row of the level;
// col: slot of (I, J) on plane 0, with I, J < n and K0 < K1 <= n.
template <int D>
__device__ inline uint32_t read_cell_planes(const Lat& L, const int8_t* __restrict__ vt, int64_t col, int K0,
                                            int K1) {
  uint32_t qm = 0;  // bit q: a corner (i..i+1, j..j+1) on plane K0 + q is a vertex
#pragma unroll
  for (int q = 0; q <= kCellPlanes; ++q) {
    if (q > K1 - K0 || (D == 2 && q > 0)) break;
    const int64_t v = col + (int64_t)(K0 + q) * L.plane;
    const bool any = (vt[v] != VT_OUT) | (vt[v + 1] != VT_OUT) | (vt[v + L.pitch] != VT_OUT) |
                     (vt[v + L.pitch + 1] != VT_OUT);
    qm |= (uint32_t)any << q;
  }
  const uint32_t planes = (D == 3) ? (qm | (qm >> 1)) : qm;
  return planes & ((1u << (K1 - K0)) - 1u);
}

// cell coefficients of cells that do not exist: the covering (parent) cell's;
// only cells a row of the level (vertex classes vtf) reads are written.
// ef32 (nullable): the single-precision copy of every such cell as well
// (the pass over the cells a row reads is then made once).
template <int D>
__global__ __launch_bounds__(256) void k_ad_virtual_eps(Lat Lf, Lat Lc, const int8_t* __restrict__ crefc,
                                                        const int8_t* __restrict__ vtf,
                                                        const double* __restrict__ ec, double* __restrict__ ef,
                                                        float* __restrict__ ef32) {
  constexpr int NP = kCellPlanes / 3;  // parent planes of a thread
  const int I = blockIdx.x * TX + threadIdx.x;
  const int J = blockIdx.y * TY + threadIdx.y;
  if (I >= Lf.n || J >= Lf.n) return;
  const int K0 = (D == 3) ? (int)blockIdx.z * kCellPlanes : 0;
  const int K1 = (D == 3) ? min(K0 + kCellPlanes, Lf.n) : 1;
  const int64_t col = I + (int64_t)J * Lf.pitch;
  const uint32_t m = read_cell_planes<D>(Lf, vtf, col, K0, K1);
  if (m == 0) return;
  const int64_t pcol = I / 3 + (int64_t)(J / 3) * Lc.pitch + (int64_t)(K0 / 3) * Lc.plane;
  double pe[NP];
  bool keep[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const bool need = ((m >> (3 * p)) & 7u) != 0;  // cell planes K0 + 3p .. K0 + 3p + 2
    const int64_t pc = pcol + (int64_t)p * Lc.plane;
    keep[p] = !need || crefc[pc] != 0;
    pe[p] = need ? ec[pc] : 0.0;
  }
  double own[kCellPlanes];  // existing cells' own values (for ef32)
#pragma unroll
  for (int q = 0; q < kCellPlanes; ++q)
    own[q] = (ef32 != nullptr && ((m >> q) & 1u) && keep[q / 3]) ? ef[col + (int64_t)(K0 + q) * Lf.plane] : 0.0;
#pragma unroll
  for (int q = 0; q < kCellPlanes; ++q) {
    if (!((m >> q) & 1u)) continue;
    const int64_t c = col + (int64_t)(K0 + q) * Lf.plane;
    if (!keep[q / 3]) {
      ef[c] = pe[q / 3];
      if (ef32 != nullptr) ef32[c] = (float)pe[q / 3];
    } else if (ef32 != nullptr) {
      ef32[c] = (float)own[q];
    }
  }
}

// single-precision cell coefficients of an adaptive level on the cells a row
// of the level reads
template <int D>
__global__ __launch_bounds__(256) void k_ad_convert_cells(Lat L, const int8_t* __restrict__ vt,
                                                          const double* __restrict__ in, float* __restrict__ out) {
  const int I = blockIdx.x * TX + threadIdx.x;
  const int J = blockIdx.y * TY + threadIdx.y;
  if (I >= L.n || J >= L.n) return;
  const int K0 = (D == 3) ? (int)blockIdx.z * kCellPlanes : 0;
  const int K1 = (D == 3) ? min(K0 + kCellPlanes, L.n) : 1;
  const int64_t col = I + (int64_t)J * L.pitch + (int64_t)K0 * L.plane;
  const uint32_t m = read_cell_planes<D>(L, vt, I + (int64_t)J * L.pitch, K0, K1);
  if (m == 0) return;
  double x[kCellPlanes];
#pragma unroll
  for (int q = 0; q < kCellPlanes; ++q) x[q] = ((m >> q) & 1u) ? in[col + (int64_t)q * L.plane] : 0.0;
#pragma unroll
  for (int q = 0; q < kCellPlanes; ++q)
    if ((m >> q) & 1u) out[col + (int64_t)q * L.plane] = (float)x[q];
}

// dst := src on every slot of the listed tiles
template <int D, typename T>
__global__ __launch_bounds__(256) void k_ad_copy(Lat L, const int32_t* __restrict__ tiles,
                                                 const T* __restrict__ src, T* __restrict__ dst) {
  const Slot s = tile_slot<D>(L, tiles);
  if (s.valid) dst[s.v] = src[s.v];
}

// zero on every slot of the listed tiles (vt given: on the slots of the
// level's vertices only); kZeroTiles tiles per workgroup (one 256-slot tile
// per workgroup leaves the fill bound by workgroup dispatch)
constexpr int kZeroTiles = 8;
template <int D, typename T>
__global__ __launch_bounds__(256) void k_ad_zero(Lat L, const int32_t* __restrict__ tiles, int ntiles,
                                                 T* __restrict__ p, int narr, const int8_t* __restrict__ vt) {
  const int q0 = (int)blockIdx.x * kZeroTiles, q1 = min(q0 + kZeroTiles, ntiles);
  for (int q = q0; q < q1; ++q) {
    const int32_t* t = tiles + 3 * (int64_t)q;
    const int i = t[0] * TX + threadIdx.x, j = t[1] * TY + threadIdx.y, k = (D == 3) ? t[2] : 0;
    if (i > L.n || j > L.n) continue;
    const int64_t v = i + (int64_t)j * L.pitch + (int64_t)k * L.plane;
    if (vt != nullptr && vt[v] == VT_OUT) continue;
    for (int a = 0; a < narr; ++a) p[(int64_t)a * L.nslot + v] = (T)0;
  }
}

// x64 += e32 on the leaves; residual of the mixed loop at the leaves in FP64
template <int D>
__global__ __launch_bounds__(256) void k_ad_axpy(Lat L, const int32_t* __restrict__ tiles,
                                                 const int8_t* __restrict__ vt, double* __restrict__ x,
                                                 const float* __restrict__ e) {
  const Slot s = tile_slot<D>(L, tiles);
  if (s.valid && vt[s.v] == VT_LEAF) x[s.v] += (double)e[s.v];
}

// The same over the level's leaf and refined vertices (refined ones skipped).
__global__ __launch_bounds__(256) void k_ad_axpy_list(const int64_t* __restrict__ act, int64_t na,
                                                      const int8_t* __restrict__ vt, double* __restrict__ x,
                                                      const float* __restrict__ e) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= na) return;
  const int64_t v = act[q];
  if (vt[v] == VT_LEAF) x[v] += (double)e[v];
}

// cell coefficients of a level: refined cells take the mean of their children
template <int D>
__global__ __launch_bounds__(256) void k_ad_coarsen_eps(Lat Lf, Lat Lc, const int8_t* __restrict__ cref,
                                                        const double* __restrict__ ef, double* __restrict__ ec) {
  const int I = blockIdx.x * TX + threadIdx.x;
  const int J = blockIdx.y * TY + threadIdx.y;
  const int K = (D == 3) ? (int)blockIdx.z : 0;
  if (I >= Lc.n || J >= Lc.n || (D == 3 && K >= Lc.n)) return;
  const int64_t vc = I + (int64_t)J * Lc.pitch + (int64_t)K * Lc.plane;
  if (!cref[vc]) return;
  double s = 0.0;
  const int zc = (D == 3) ? 3 : 1;
  for (int c = 0; c < zc; ++c)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a)
        s += ef[(3 * I + a) + (int64_t)(3 * J + b) * Lf.pitch + (int64_t)(3 * K + c) * Lf.plane];
  ec[vc] = s / (D == 3 ? 27.0 : 9.0);
}

// stencil rows of a level for the next Galerkin product: refined rows keep the
// Galerkin result, leaf rows take the rediscretised stencil, other rows zero
// (cleared: those of the level's vertices hold zero already, and rows outside
// the level are never read; neither is written)
template <int D>
__global__ __launch_bounds__(256) void k_ad_merge_rows(Lat L, const int8_t* __restrict__ vt,
                                                       const double* __restrict__ eps, double* __restrict__ A,
                                                       int cleared) {
  constexpr int NS = Dim<D>::NS;
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int kz = (D == 3) ? (int)blockIdx.z : 0;
  if (i > L.n || j > L.n) return;
  const int64_t v = i + (int64_t)j * L.pitch + (int64_t)kz * L.plane;
  const int8_t t = vt[v];
  if (t == VT_REFINED) return;
  if (t == VT_LEAF) {
    double a[NS];
    geom_row<D, double>(eps, v, L, a);
    for (int k = 0; k < NS; ++k) {
      const int ii = i + off_x(k), jj = j + off_y(k), kk = kz + (D == 3 ? off_z(k) : 0);
      const bool in = ii >= 1 && ii < L.n && jj >= 1 && jj < L.n && (D == 2 || (kk >= 1 && kk < L.n));
      A[(int64_t)k * L.nslot + v] = in ? a[k] : 0.0;
    }
  } else if (!cleared) {
    for (int k = 0; k < NS; ++k) A[(int64_t)k * L.nslot + v] = 0.0;
  }
}

// packed leaf values <-> lattice slots (slot lists in unknown order)
template <typename T>
__global__ void k_ad_scatter(const int64_t* __restrict__ slots, int64_t n, const double* __restrict__ in,
                             double scale, T* __restrict__ lat) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) lat[slots[t]] = (T)(scale * in[t]);
}
template <typename T>
__global__ void k_ad_gather(const int64_t* __restrict__ slots, int64_t n, const T* __restrict__ lat,
                            double* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) out[t] = (double)lat[slots[t]];
}

inline dim3 tiles_grid(int ntiles) { return dim3((unsigned)ntiles); }
inline unsigned list_blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
inline dim3 full_grid(const Lat& L) {
  return dim3((unsigned)(L.pitch / TX), (unsigned)((L.n + 1 + TY - 1) / TY), (unsigned)(L.d == 3 ? L.n + 1 : 1));
}

template <int D, typename T, typename TO, int SRC, int FMT>
void ad_stencil_mode(const AdTiles& t, int mode, const T* u, const T* b, TO* out, const T* eps,
                     const Store& A, T omega, double* partial, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (D == 3 && t.nb >= kMarchMinBricks && (mode == 0 || mode == 2)) {
    const dim3 gm((unsigned)(8 * ((t.nb + 7) / 8))), bm(BX * BY);
    if (mode == 0 && e0 != nullptr)
      hipExtLaunchKernelGGL((k_ad_march<T, TO, SRC, FMT, 0>), gm, bm, 0, s, e0, e1, 0, t.L, t.bricks, t.nb, t.vt,
                            u, b, out, eps, A, omega, partial);
    else if (mode == 0)
      hipLaunchKernelGGL((k_ad_march<T, TO, SRC, FMT, 0>), gm, bm, 0, s, t.L, t.bricks, t.nb, t.vt, u, b, out, eps,
                         A, omega, partial);
    else
      hipLaunchKernelGGL((k_ad_march<T, TO, SRC, FMT, 2>), gm, bm, 0, s, t.L, t.bricks, t.nb, t.vt, u, b, out, eps,
                         A, omega, partial);
    return;
  }
  const dim3 g = tiles_grid(t.n), bl(TX, TY, 1);
  if (e0 != nullptr && mode == 0) {  // per-dispatch timestamps of a timed sweep
    hipExtLaunchKernelGGL((k_ad_stencil<D, T, TO, SRC, FMT, 0>), g, bl, 0, s, e0, e1, 0, t.L, t.tiles, t.vt, u,
                          b, out, eps, A, omega, partial);
    return;
  }
  switch (mode) {
    case 0: hipLaunchKernelGGL((k_ad_stencil<D, T, TO, SRC, FMT, 0>), g, bl, 0, s, t.L, t.tiles, t.vt, u, b, out, eps, A, omega, partial); break;
    case 1: hipLaunchKernelGGL((k_ad_stencil<D, T, TO, SRC, FMT, 1>), g, bl, 0, s, t.L, t.tiles, t.vt, u, b, out, eps, A, omega, partial); break;
    default: hipLaunchKernelGGL((k_ad_stencil<D, T, TO, SRC, FMT, 2>), g, bl, 0, s, t.L, t.tiles, t.vt, u, b, out, eps, A, omega, partial); break;
  }
}

template <int D, typename T, typename TO>
void ad_stencil_src(const AdTiles& t, int mode, const T* u, const T* b, TO* out, const T* eps,
                    const Store& A, T omega, double* partial, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
#define QMG_ADS(SRCV, FMTV) ad_stencil_mode<D, T, TO, SRCV, FMTV>(t, mode, u, b, out, eps, A, omega, partial, s, e0, e1)
  if (A.src == SRC_GEOM) return QMG_ADS(SRC_GEOM, F64);
  if (A.src == SRC_PLAIN) return QMG_ADS(SRC_PLAIN, F64);
  switch (A.fmt) {
    case F64: return QMG_ADS(SRC_HIER, F64);
    case F32: return QMG_ADS(SRC_HIER, F32);
    case F16: return QMG_ADS(SRC_HIER, F16);
    default: return QMG_ADS(SRC_HIER, BF16);
  }
#undef QMG_ADS
}

template <int D, typename T, int PSRC>
void ad_fas_src(const AdTiles& tc, const Lat& Lf, const T* rf, const T* uc, const T* epsc, const Store& Ac,
                T* bc, const Store& P, hipStream_t s, const int32_t* verts, int64_t nverts,
                const int32_t* cells, int64_t ncells, T* part) {
  const dim3 g = tiles_grid(tc.n), bl(TX, TY, 1);
  const dim3 gl((unsigned)((nverts + 3) / 4)), bll(256);
  const bool by_cells = verts && cells && part;
  if (by_cells && ncells > 0) {
    constexpr int CPB = (D == 3) ? 8 : 16;
    hipLaunchKernelGGL((k_ad_restrict_cells<D, T, PSRC, F64>), dim3(list_blocks(ncells, CPB)), dim3(256), 0, s, Lf,
                       tc.L, cells, ncells, rf, part, P);
  }
  const dim3 gv(list_blocks(nverts, 256));
#define QMG_FAS(SRCV, FMTV)                                                                              \
  do {                                                                                                   \
    if (by_cells)                                                                                        \
      hipLaunchKernelGGL((k_ad_fas_rhs_cells<D, T, SRCV, FMTV>), gv, bll, 0, s, tc.L, verts, nverts, part, uc, \
                         epsc, Ac, bc);                                                                  \
    else if (verts)                                                                                      \
      hipLaunchKernelGGL((k_ad_fas_rhs_list<D, T, SRCV, FMTV, PSRC, F64>), gl, bll, 0, s, Lf, tc.L, verts, \
                         nverts, rf, uc, epsc, Ac, bc, P);                                               \
    else                                                                                                 \
      hipLaunchKernelGGL((k_ad_fas_rhs<D, T, SRCV, FMTV, PSRC, F64>), g, bl, 0, s, Lf, tc.L, tc.tiles, tc.vt, \
                         rf, uc, epsc, Ac, bc, P);                                                       \
  } while (0)
  if (Ac.src == SRC_GEOM) QMG_FAS(SRC_GEOM, F64);
  else if (Ac.src == SRC_PLAIN) QMG_FAS(SRC_PLAIN, F64);
  else if (Ac.fmt == F64) QMG_FAS(SRC_HIER, F64);
  else if (Ac.fmt == F32) QMG_FAS(SRC_HIER, F32);
  else if (Ac.fmt == F16) QMG_FAS(SRC_HIER, F16);
  else QMG_FAS(SRC_HIER, BF16);
#undef QMG_FAS
}

// prolongation stores of adaptive levels: d-linear, FP64 deltas or plain
inline void check_ad_P(const Store& P) {
  if (P.src == SRC_HIER && P.fmt != F64) throw HipError("adaptive levels keep their prolongation in FP64");
}

}  // namespace

template <typename T, typename TO>
int launch_ad_stencil(const AdTiles& t, int mode, const T* u, const T* b, TO* out, const T* eps,
                      const Store& A, T omega, double* partial, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (t.n <= 0) return 0;
  if (t.L.d == 2) ad_stencil_src<2, T, TO>(t, mode, u, b, out, eps, A, omega, partial, s, e0, e1);
  else ad_stencil_src<3, T, TO>(t, mode, u, b, out, eps, A, omega, partial, s, e0, e1);
  QMG_HIP(hipGetLastError());
  if (partial == nullptr) return 0;
  return (t.L.d == 3 && t.nb >= kMarchMinBricks && (mode == 0 || mode == 2)) ? t.nb : t.n;
}
template int launch_ad_stencil<double, double>(const AdTiles&, int, const double*, const double*, double*, const double*, const Store&, double, double*, hipStream_t, hipEvent_t, hipEvent_t);
template int launch_ad_stencil<float, float>(const AdTiles&, int, const float*, const float*, float*, const float*, const Store&, float, double*, hipStream_t, hipEvent_t, hipEvent_t);
template int launch_ad_stencil<double, float>(const AdTiles&, int, const double*, const double*, float*, const double*, const Store&, double, double*, hipStream_t, hipEvent_t, hipEvent_t);

template <typename T>
void launch_ad_hang(const AdTiles& tf, const Lat& Lc, T* uf, const T* uc, const Store& P, hipStream_t s) {
  if (tf.n <= 0) return;
  check_ad_P(P);
  if (tf.hang != nullptr) {
    if (tf.nh <= 0) return;
    const dim3 gl(list_blocks(tf.nh, 256));
#define QMG_HANGL(DV, PS) \
  hipLaunchKernelGGL((k_ad_hang_list<DV, T, PS, F64>), gl, dim3(256), 0, s, tf.L, Lc, tf.hang, tf.nh, uf, uc, P)
    if (tf.L.d == 2) {
      if (P.src == SRC_HIER) QMG_HANGL(2, SRC_HIER); else if (P.src == SRC_PLAIN) QMG_HANGL(2, SRC_PLAIN); else QMG_HANGL(2, SRC_GEOM);
    } else {
      if (P.src == SRC_HIER) QMG_HANGL(3, SRC_HIER); else if (P.src == SRC_PLAIN) QMG_HANGL(3, SRC_PLAIN); else QMG_HANGL(3, SRC_GEOM);
    }
#undef QMG_HANGL
    QMG_HIP(hipGetLastError());
    return;
  }
  const dim3 g = tiles_grid(tf.n), bl(TX, TY, 1);
#define QMG_HANG(DV, PS) hipLaunchKernelGGL((k_ad_hang<DV, T, PS, F64>), g, bl, 0, s, tf.L, Lc, tf.tiles, tf.vt, uf, uc, P)
  if (tf.L.d == 2) {
    if (P.src == SRC_HIER) QMG_HANG(2, SRC_HIER); else if (P.src == SRC_PLAIN) QMG_HANG(2, SRC_PLAIN); else QMG_HANG(2, SRC_GEOM);
  } else {
    if (P.src == SRC_HIER) QMG_HANG(3, SRC_HIER); else if (P.src == SRC_PLAIN) QMG_HANG(3, SRC_PLAIN); else QMG_HANG(3, SRC_GEOM);
  }
#undef QMG_HANG
  QMG_HIP(hipGetLastError());
}

template <typename T>
void launch_ad_inject(const AdTiles& tc, const Lat& Lf, const T* uf, T* uc, hipStream_t s) {
  if (tc.n <= 0) return;
  const dim3 g = tiles_grid(tc.n), bl(TX, TY, 1);
  if (tc.L.d == 2) hipLaunchKernelGGL((k_ad_inject<2, T>), g, bl, 0, s, Lf, tc.L, tc.tiles, tc.vt, uf, uc);
  else hipLaunchKernelGGL((k_ad_inject<3, T>), g, bl, 0, s, Lf, tc.L, tc.tiles, tc.vt, uf, uc);
  QMG_HIP(hipGetLastError());
}

template <typename T>
void launch_ad_fas_rhs(const AdTiles& tc, const Lat& Lf, const T* rf, const T* uc, const T* epsc,
                       const Store& Ac, T* bc, const Store& P, hipStream_t s, const int32_t* verts,
                       int64_t nverts, const int32_t* cells, int64_t ncells, T* part) {
  if (tc.n <= 0 || (verts && nverts <= 0)) return;
  check_ad_P(P);
  if (tc.L.d == 2) {
    if (P.src == SRC_HIER) ad_fas_src<2, T, SRC_HIER>(tc, Lf, rf, uc, epsc, Ac, bc, P, s, verts, nverts, cells, ncells, part);
    else if (P.src == SRC_PLAIN) ad_fas_src<2, T, SRC_PLAIN>(tc, Lf, rf, uc, epsc, Ac, bc, P, s, verts, nverts, cells, ncells, part);
    else ad_fas_src<2, T, SRC_GEOM>(tc, Lf, rf, uc, epsc, Ac, bc, P, s, verts, nverts, cells, ncells, part);
  } else {
    if (P.src == SRC_HIER) ad_fas_src<3, T, SRC_HIER>(tc, Lf, rf, uc, epsc, Ac, bc, P, s, verts, nverts, cells, ncells, part);
    else if (P.src == SRC_PLAIN) ad_fas_src<3, T, SRC_PLAIN>(tc, Lf, rf, uc, epsc, Ac, bc, P, s, verts, nverts, cells, ncells, part);
    else ad_fas_src<3, T, SRC_GEOM>(tc, Lf, rf, uc, epsc, Ac, bc, P, s, verts, nverts, cells, ncells, part);
  }
  QMG_HIP(hipGetLastError());
}

template <typename T>
void launch_ad_correct(const AdTiles& tf, const Lat& Lc, T* uf, const T* uc, const T* sc, const Store& P,
                       hipStream_t s) {
  if (tf.n <= 0) return;
  check_ad_P(P);
  if (tf.act != nullptr) {
    if (tf.na <= 0) return;
    const dim3 gl(list_blocks(tf.na, 256));
#define QMG_CORRL(DV, PS) \
  hipLaunchKernelGGL((k_ad_correct_list<DV, T, PS, F64>), gl, dim3(256), 0, s, tf.L, Lc, tf.act, tf.na, uf, uc, sc, P)
    if (tf.L.d == 2) {
      if (P.src == SRC_HIER) QMG_CORRL(2, SRC_HIER); else if (P.src == SRC_PLAIN) QMG_CORRL(2, SRC_PLAIN); else QMG_CORRL(2, SRC_GEOM);
    } else {
      if (P.src == SRC_HIER) QMG_CORRL(3, SRC_HIER); else if (P.src == SRC_PLAIN) QMG_CORRL(3, SRC_PLAIN); else QMG_CORRL(3, SRC_GEOM);
    }
#undef QMG_CORRL
    QMG_HIP(hipGetLastError());
    return;
  }
  const dim3 g = tiles_grid(tf.n), bl(TX, TY, 1);
#define QMG_CORR(DV, PS) hipLaunchKernelGGL((k_ad_correct<DV, T, PS, F64>), g, bl, 0, s, tf.L, Lc, tf.tiles, tf.vt, uf, uc, sc, P)
  if (tf.L.d == 2) {
    if (P.src == SRC_HIER) QMG_CORR(2, SRC_HIER); else if (P.src == SRC_PLAIN) QMG_CORR(2, SRC_PLAIN); else QMG_CORR(2, SRC_GEOM);
  } else {
    if (P.src == SRC_HIER) QMG_CORR(3, SRC_HIER); else if (P.src == SRC_PLAIN) QMG_CORR(3, SRC_PLAIN); else QMG_CORR(3, SRC_GEOM);
  }
#undef QMG_CORR
  QMG_HIP(hipGetLastError());
}

void launch_ad_virtual_eps(const Lat& Lf, const Lat& Lc, const int8_t* crefc, const int8_t* vtf, const double* ec,
                           double* ef, float* ef32, hipStream_t s) {
  const dim3 g = cell_walk_grid(Lf), bl(TX, TY, 1);
  if (Lf.d == 2) hipLaunchKernelGGL(k_ad_virtual_eps<2>, g, bl, 0, s, Lf, Lc, crefc, vtf, ec, ef, ef32);
  else hipLaunchKernelGGL(k_ad_virtual_eps<3>, g, bl, 0, s, Lf, Lc, crefc, vtf, ec, ef, ef32);
  QMG_HIP(hipGetLastError());
}

void launch_ad_convert_cells(const Lat& L, const int8_t* vt, const double* in, float* out, hipStream_t s) {
  const dim3 g = cell_walk_grid(L), bl(TX, TY, 1);
  if (L.d == 2) hipLaunchKernelGGL(k_ad_convert_cells<2>, g, bl, 0, s, L, vt, in, out);
  else hipLaunchKernelGGL(k_ad_convert_cells<3>, g, bl, 0, s, L, vt, in, out);
  QMG_HIP(hipGetLastError());
}

template <typename T>
void launch_ad_copy(const AdTiles& t, const T* src, T* dst, hipStream_t s) {
  if (t.n <= 0) return;
  const dim3 g = tiles_grid(t.n), bl(TX, TY, 1);
  if (t.L.d == 2) hipLaunchKernelGGL((k_ad_copy<2, T>), g, bl, 0, s, t.L, t.tiles, src, dst);
  else hipLaunchKernelGGL((k_ad_copy<3, T>), g, bl, 0, s, t.L, t.tiles, src, dst);
  QMG_HIP(hipGetLastError());
}

template <typename T>
void launch_ad_zero(const AdTiles& t, T* p, hipStream_t s, int narr, bool vertices_only) {
  if (t.n <= 0) return;
  const dim3 g((unsigned)((t.n + kZeroTiles - 1) / kZeroTiles)), bl(TX, TY, 1);
  const int8_t* vt = vertices_only ? t.vt : nullptr;
  if (t.L.d == 2) hipLaunchKernelGGL((k_ad_zero<2, T>), g, bl, 0, s, t.L, t.tiles, t.n, p, narr, vt);
  else hipLaunchKernelGGL((k_ad_zero<3, T>), g, bl, 0, s, t.L, t.tiles, t.n, p, narr, vt);
  QMG_HIP(hipGetLastError());
}

void launch_ad_axpy(const AdTiles& t, double* x, const float* e, hipStream_t s) {
  if (t.n <= 0) return;
  if (t.act != nullptr) {
    if (t.na > 0)
      hipLaunchKernelGGL(k_ad_axpy_list, dim3(list_blocks(t.na, 256)), dim3(256), 0, s, t.act, t.na, t.vt, x, e);
    QMG_HIP(hipGetLastError());
    return;
  }
  const dim3 g = tiles_grid(t.n), bl(TX, TY, 1);
  if (t.L.d == 2) hipLaunchKernelGGL(k_ad_axpy<2>, g, bl, 0, s, t.L, t.tiles, t.vt, x, e);
  else hipLaunchKernelGGL(k_ad_axpy<3>, g, bl, 0, s, t.L, t.tiles, t.vt, x, e);
  QMG_HIP(hipGetLastError());
}

void launch_ad_coarsen_eps(const Lat& Lf, const Lat& Lc, const int8_t* cref, const double* ef, double* ec,
                           hipStream_t s) {
  const dim3 g = full_grid(Lc), bl(TX, TY, 1);
  if (Lc.d == 2) hipLaunchKernelGGL(k_ad_coarsen_eps<2>, g, bl, 0, s, Lf, Lc, cref, ef, ec);
  else hipLaunchKernelGGL(k_ad_coarsen_eps<3>, g, bl, 0, s, Lf, Lc, cref, ef, ec);
  QMG_HIP(hipGetLastError());
}

void launch_ad_merge_rows(const Lat& L, const int8_t* vt, const double* eps, double* A, bool cleared,
                          hipStream_t s) {
  const dim3 g = full_grid(L), bl(TX, TY, 1);
  if (L.d == 2) hipLaunchKernelGGL(k_ad_merge_rows<2>, g, bl, 0, s, L, vt, eps, A, (int)cleared);
  else hipLaunchKernelGGL(k_ad_merge_rows<3>, g, bl, 0, s, L, vt, eps, A, (int)cleared);
  QMG_HIP(hipGetLastError());
}

template <typename T>
void launch_ad_scatter(const int64_t* slots, int64_t n, const double* in, double scale, T* lat, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_ad_scatter<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, slots, n, in, scale, lat);
  QMG_HIP(hipGetLastError());
}
template <typename T>
void launch_ad_gather(const int64_t* slots, int64_t n, const T* lat, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_ad_gather<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, slots, n, lat, out);
  QMG_HIP(hipGetLastError());
}

template void launch_ad_hang<double>(const AdTiles&, const Lat&, double*, const double*, const Store&, hipStream_t);
template void launch_ad_hang<float>(const AdTiles&, const Lat&, float*, const float*, const Store&, hipStream_t);
template void launch_ad_inject<double>(const AdTiles&, const Lat&, const double*, double*, hipStream_t);
template void launch_ad_inject<float>(const AdTiles&, const Lat&, const float*, float*, hipStream_t);
template void launch_ad_fas_rhs<double>(const AdTiles&, const Lat&, const double*, const double*, const double*, const Store&, double*, const Store&, hipStream_t, const int32_t*, int64_t, const int32_t*, int64_t, double*);
template void launch_ad_fas_rhs<float>(const AdTiles&, const Lat&, const float*, const float*, const float*, const Store&, float*, const Store&, hipStream_t, const int32_t*, int64_t, const int32_t*, int64_t, float*);
template void launch_ad_correct<double>(const AdTiles&, const Lat&, double*, const double*, const double*, const Store&, hipStream_t);
template void launch_ad_correct<float>(const AdTiles&, const Lat&, float*, const float*, const float*, const Store&, hipStream_t);
template void launch_ad_copy<double>(const AdTiles&, const double*, double*, hipStream_t);
template void launch_ad_copy<float>(const AdTiles&, const float*, float*, hipStream_t);
template void launch_ad_zero<double>(const AdTiles&, double*, hipStream_t, int, bool);
template void launch_ad_zero<float>(const AdTiles&, float*, hipStream_t, int, bool);
template void launch_ad_scatter<double>(const int64_t*, int64_t, const double*, double, double*, hipStream_t);
template void launch_ad_scatter<float>(const int64_t*, int64_t, const double*, double, float*, hipStream_t);
template void launch_ad_gather<double>(const int64_t*, int64_t, const double*, double*, hipStream_t);
template void launch_ad_gather<float>(const int64_t*, int64_t, const float*, double*, hipStream_t);

}  // namespace qmg
