// Operator construction kernels: coefficient coarsening, BoxMG prolongation
// (Sect. 4.4 and the BoxMG appendix), Galerkin R A P (Sect. 4.3) with the
// definiteness check, and the hierarchical delta store (Sect. 5).  All FP64.
#include <stdexcept>
#include "device_ops.hpp"

namespace qmg {

namespace {

constexpr int TX = 64, TY = 4;

inline dim3 tile_grid(const Lat& L) {
  return dim3((unsigned)(L.pitch / TX), (unsigned)((L.n + 1 + TY - 1) / TY),
              (unsigned)(L.d == 3 ? L.n + 1 : 1));
}
inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ inline bool interior(const Lat& L, int i, int j, int k) {
  return i >= 1 && i < L.n && j >= 1 && j < L.n && (L.d == 2 || (k >= 1 && k < L.n));
}

template <int D>
__global__ __launch_bounds__(256) void k_coarsen_eps(Lat Lf, Lat Lc, const double* __restrict__ ef,
                                                     double* __restrict__ ec) {
  const int I = blockIdx.x * TX + threadIdx.x;
  const int J = blockIdx.y * TY + threadIdx.y;
  const int K = (D == 3) ? (int)blockIdx.z : 0;
  if (I >= Lc.n || J >= Lc.n || (D == 3 && K >= Lc.n)) return;
  double s = 0.0;
  const int zc = (D == 3) ? 3 : 1;
  for (int c = 0; c < zc; ++c)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a)
        s += ef[(3 * I + a) + (int64_t)(3 * J + b) * Lf.pitch + (int64_t)(3 * K + c) * Lf.plane];
  ec[I + (int64_t)J * Lc.pitch + (int64_t)K * Lc.plane] = s / (D == 3 ? 27.0 : 9.0);
}

// Operator row of an interior vertex as the smoother applies it, with entries
// pointing at boundary vertices dropped.
template <int D, int SRC, int FMT>
__global__ __launch_bounds__(256) void k_materialise(Lat L, const double* __restrict__ eps, Store A,
                                                     double* __restrict__ out) {
  constexpr int NS = Dim<D>::NS;
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int kz = (D == 3) ? (int)blockIdx.z : 0;
  if (!interior(L, i, j, kz)) return;
  const int64_t v = i + (int64_t)j * L.pitch + (int64_t)kz * L.plane;
  double a[NS];
  if (SRC == SRC_PLAIN) {
    for (int k = 0; k < NS; ++k) a[k] = ((const double*)A.dense)[(int64_t)k * L.nslot + v];
  } else {
    geom_row<D, double>(eps, v, L, a);
    if (SRC == SRC_HIER) add_delta<FMT, NS, double>(A, v, a);
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const bool in = interior(L, i + off_x(k), j + off_y(k), kz + (D == 3 ? off_z(k) : 0));
    out[(int64_t)k * L.nslot + v] = in ? a[k] : 0.0;
  }
}

// d-linear weight of parent floor(f/3)+kappa with non-parents and boundary
// coarse vertices dropped.
template <int D>
__device__ inline double dlin_dropped(const Lat& Lc, int i, int j, int k, int kap) {
  const int kx = kap & 1, ky = (kap >> 1) & 1, kz = (kap >> 2) & 1;
  const int qx = i / 3, qy = j / 3, qz = k / 3;
  const int rx = i - 3 * qx, ry = j - 3 * qy, rz = k - 3 * qz;
  if ((kx && rx == 0) || (ky && ry == 0) || (D == 3 && kz && rz == 0)) return 0.0;
  if (!interior(Lc, qx + kx, qy + ky, D == 3 ? qz + kz : 0)) return 0.0;
  return dlin1(rx, kx) * dlin1(ry, ky) * (D == 3 ? dlin1(rz, kz) : 1.0);
}

template <int D, int SRC, int FMT>
__global__ __launch_bounds__(256) void k_materialise_P(Lat Lf, Lat Lc, Store P, double* __restrict__ out) {
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int kz = (D == 3) ? (int)blockIdx.z : 0;
  if (!interior(Lf, i, j, kz)) return;
  const int64_t v = i + (int64_t)j * Lf.pitch + (int64_t)kz * Lf.plane;
  double w[Dim<D>::NC];
  for (int c = 0; c < Dim<D>::NC; ++c) {
    if (SRC == SRC_PLAIN) w[c] = ((const double*)P.dense)[(int64_t)c * Lf.nslot + v];
    else w[c] = dlin_dropped<D>(Lc, i, j, kz, c);
  }
  if (SRC == SRC_HIER) add_delta<FMT, Dim<D>::NC, double>(P, v, w);
  for (int c = 0; c < Dim<D>::NC; ++c) out[(int64_t)c * Lf.nslot + v] = w[c];
}

// ---------------------------------------------------------------------------
// BoxMG.  One thread per (interior coarse vertex V, orthant sigma).  In the
// reference frame y in {0..3}^d the fine vertex is 3V + sigma*y and the stencil
// offset o' is the true offset sigma*o'.  Unknowns p(y), y in {0,1,2}^d; p = 0
// where a coordinate is 3.  Groups are solved in order: c-point (p = 1), lines
// (stencil collapsed onto the line's axis), faces in 3D (collapsed along the
// normal), interior (full stencils), each group depending only on earlier ones.
// ---------------------------------------------------------------------------
template <int D>
struct BoxFetch {
  const double* A;  // FP64 stencils (entry-major) or null: rediscretise from eps
  const double* eps;
  Lat L;
  const int8_t* vt = nullptr;  // optional: rows only at leaf and refined vertices
  bool hanging_rows = false;   // with vt: hanging rows rediscretised from eps
  __device__ double operator()(int64_t v, int i, int j, int k, int kk) const {
    if (vt) {
      const int8_t t = vt[v];
      if (hanging_rows && t == VT_HANGING) return geom_entry<D>(eps, v, i, j, k, kk, L);
      if (t != VT_LEAF && t != VT_REFINED) return 0.0;
    }
    if (A) return A[(int64_t)kk * L.nslot + v];
    return geom_entry<D>(eps, v, i, j, k, kk, L);
  }
};

// Row of fine vertex v as BoxFetch gives it, one entry at a time from a
// prepared state: the stored row, or the rediscretised row from the 2^d cell
// coefficients held in registers (boundary entries dropped), or nothing.
template <int D>
struct RowSrc {
  int mode = 0;  // 0: empty row, 1: stored row, 2: rediscretised row
  double ce[Dim<D>::NC];
  __device__ RowSrc(const BoxFetch<D>& F, int64_t v) {
    bool geo = F.A == nullptr;
    mode = 1;
    if (F.vt) {
      const int8_t t = F.vt[v];
      if (F.hanging_rows && t == VT_HANGING) geo = true;
      else if (t != VT_LEAF && t != VT_REFINED) mode = 0;
    }
    if (mode == 1 && geo) mode = 2;
#pragma unroll
    for (int s = 0; s < Dim<D>::NC; ++s)
      ce[s] = mode == 2 ? F.eps[v - slot_off(F.L, s & 1, (s >> 1) & 1, (s >> 2) & 1)] : 0.0;
  }
  // entry k of the row of v = (i, j, kz); the neighbour must be checked for
  // being interior by the caller when mode == 2
  __device__ double entry(const BoxFetch<D>& F, int64_t v, int k) const {
    if (mode == 1) return F.A[(int64_t)k * F.L.nslot + v];
    const int nd = (off_x(k) != 0) + (off_y(k) != 0) + (D == 3 ? (off_z(k) != 0) : 0);
    const double w = kref(D, nd);
    double e = 0.0;
#pragma unroll
    for (int s = 0; s < Dim<D>::NC; ++s) {
      const int sx = s & 1, sy = (s >> 1) & 1, sz = (s >> 2) & 1;
      const bool has = sx + off_x(k) >= 0 && sx + off_x(k) <= 1 && sy + off_y(k) >= 0 && sy + off_y(k) <= 1 &&
                       (D == 2 || (sz + off_z(k) >= 0 && sz + off_z(k) <= 1));
      e += has ? ce[s] : 0.0;
    }
    return ((D == 3) ? F.L.h : 1.0) * w * e;
  }
};

__host__ __device__ constexpr int pidx(int yx, int yy, int yz) { return yx + 3 * yy + 9 * yz; }

// The 27 reference-frame weights of one thread, kept in LDS (one column per
// thread of the 64-thread workgroup) to leave registers to the patch systems.
struct PCol {
  double* base;
  __device__ double& operator[](int i) const { return base[i * 64]; }
};

template <int D, int S>
__device__ inline void box_group(const BoxFetch<D>& F, int Vx, int Vy, int Vz, int sx, int sy, int sz,
                                 const PCol& p) {
  // unknowns: y with y_i in {1,2} for i in S, 0 otherwise
  constexpr int m = 1 << ((S & 1) + ((S >> 1) & 1) + ((S >> 2) & 1));
  double M[m][m];
  double rhs[m];
#pragma unroll
  for (int r = 0; r < m; ++r) {
    rhs[r] = 0.0;
#pragma unroll
    for (int c = 0; c < m; ++c) M[r][c] = 0.0;
  }
  // enumerate group members: bit b of r selects value 1 or 2 on the b-th axis of S
#pragma unroll
  for (int r = 0; r < m; ++r) {
    int y[3] = {0, 0, 0};
    {
      int bit = 0;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
        if (S & (1 << ax)) { y[ax] = 1 + ((r >> bit) & 1); ++bit; }
    }
    const int fx = 3 * Vx + sx * y[0], fy = 3 * Vy + sy * y[1], fz = 3 * Vz + sz * y[2];
    const int64_t v = fx + (int64_t)fy * F.L.pitch + (int64_t)fz * F.L.plane;
    const RowSrc<D> row(F, v);  // the member's row, fetched once
    // The row in the reference frame: the cell coefficients of a rediscretised
    // row mirrored (axis a flipped: cell bit a flipped), and per axis whether
    // the true neighbour one step back / ahead in the reference frame is an
    // interior vertex (entries towards Dirichlet vertices are dropped).  With
    // the frame fixed, every entry below is a fixed sum of these values, so
    // the unrolled code stays small; a stored row is read at the mirrored
    // entry.
    double cr[Dim<D>::NC];
#pragma unroll
    for (int c = 0; c < Dim<D>::NC; ++c) cr[c] = row.ce[c];
    if (sx < 0) {
#pragma unroll
      for (int c = 0; c < Dim<D>::NC; c += 2) { const double t = cr[c]; cr[c] = cr[c + 1]; cr[c + 1] = t; }
    }
    if (sy < 0) {
#pragma unroll
      for (int c = 0; c < Dim<D>::NC; ++c)
        if (!(c & 2)) { const double t = cr[c]; cr[c] = cr[c + 2]; cr[c + 2] = t; }
    }
    if (D == 3 && sz < 0) {
#pragma unroll
      for (int c = 0; c < Dim<D>::NC; ++c)
        if (!(c & 4)) { const double t = cr[c]; cr[c] = cr[c + 4]; cr[c + 4] = t; }
    }
    const int n = F.L.n;
    const bool okm[3] = {fx - sx >= 1 && fx - sx <= n - 1, fy - sy >= 1 && fy - sy <= n - 1,
                         D == 2 || (fz - sz >= 1 && fz - sz <= n - 1)};
    const bool okp[3] = {fx + sx >= 1 && fx + sx <= n - 1, fy + sy >= 1 && fy + sy <= n - 1,
                         D == 2 || (fz + sz >= 1 && fz + sz <= n - 1)};
    const double hs = (D == 3) ? F.L.h : 1.0;
#pragma unroll
    for (int k = 0; k < Dim<D>::NS; ++k) {
      const int o[3] = {off_x(k), off_y(k), D == 3 ? off_z(k) : 0};
      int w[3];
      bool far = false, ingroup = true;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        w[ax] = y[ax] + ((S & (1 << ax)) ? o[ax] : 0);
        if (w[ax] == 3) far = true;
        const bool nz = w[ax] != 0;
        if (nz != (((S >> ax) & 1) != 0)) ingroup = false;
      }
      if (far) continue;
      double a = 0.0;
      if (row.mode == 2) {
        const double kw = kref(D, ndiff_of<D>(k));
        if (kw != 0.0) {
          bool ok = true;
#pragma unroll
          for (int ax = 0; ax < 3; ++ax)
            if (o[ax] != 0) ok = ok && (o[ax] < 0 ? okm[ax] : okp[ax]);
          double e = 0.0;
#pragma unroll
          for (int c = 0; c < Dim<D>::NC; ++c)
            if (cell_has<D>(c, k)) e += cr[c];
          a = ok ? hs * kw * e : 0.0;
        }
      } else if (row.mode == 1) {
        const int ks = (sx * o[0] + 1) + 3 * (sy * o[1] + 1) + (D == 3 ? 9 * (sz * o[2] + 1) : 0);
        a = F.A[(int64_t)ks * F.L.nslot + v];
      }
      if (ingroup) {
        int col = 0, bit = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
          if (S & (1 << ax)) { col |= (w[ax] - 1) << bit; ++bit; }
        M[r][col] += a;
      } else {
        rhs[r] -= a * p[pidx(w[0], w[1], w[2])];
      }
    }
  }
  // Gaussian elimination (the systems are diagonally dominant M-matrices for
  // FEM stencils of positive coefficients; no pivoting)
#pragma unroll
  for (int c = 0; c < m; ++c) {
    const double inv = 1.0 / M[c][c];
#pragma unroll
    for (int r = c + 1; r < m; ++r) {
      const double f = M[r][c] * inv;
#pragma unroll
      for (int q = c; q < m; ++q) M[r][q] -= f * M[c][q];
      rhs[r] -= f * rhs[c];
    }
  }
  double sol[m];
#pragma unroll
  for (int c = m - 1; c >= 0; --c) {
    double t = rhs[c];
#pragma unroll
    for (int q = c + 1; q < m; ++q) t -= M[c][q] * sol[q];
    sol[c] = t / M[c][c];
  }
#pragma unroll
  for (int r = 0; r < m; ++r) {
    int y[3] = {0, 0, 0};
    int bit = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
      if (S & (1 << ax)) { y[ax] = 1 + ((r >> bit) & 1); ++bit; }
    p[pidx(y[0], y[1], y[2])] = sol[r];
  }
}

// refined flag of the coarse cell of orthant (sx, sy, sz) at coarse vertex V
__device__ inline bool orthant_refined(const int8_t* cref, const Lat& Lc, int Vx, int Vy, int Vz, int sx, int sy,
                                       int sz) {
  const int cx = Vx + (sx < 0 ? -1 : 0), cy = Vy + (sy < 0 ? -1 : 0), cz = Vz + (sz < 0 ? -1 : 0);
  return cref[cx + (int64_t)cy * Lc.pitch + (int64_t)cz * Lc.plane] != 0;
}

// Weights towards a coarse corner V on the Dirichlet boundary are dropped:
// zero on the interior fine vertices 3V + s y (y in 0..2 per axis) of the
// orthant s that points into a refined cell, with the entries towards the
// second parent along the shared axes (y_i = 0; weight zero).  Several
// threads may write the same zeros.
template <int D>
__device__ inline void zero_boundary_orthant(const Lat& Lf, double* __restrict__ Pw, int Vx, int Vy, int Vz,
                                             int sx, int sy, int sz, int yx_only = -1) {
  const int zmax = (D == 3) ? 3 : 1;
  const int yx0 = yx_only < 0 ? 0 : yx_only, yx1 = yx_only < 0 ? 3 : yx_only + 1;
  for (int yz = 0; yz < zmax; ++yz)
    for (int yy = 0; yy < 3; ++yy)
      for (int yx = yx0; yx < yx1; ++yx) {
        const int fx = 3 * Vx + sx * yx, fy = 3 * Vy + sy * yy, fz = 3 * Vz + sz * yz;
        if (!interior(Lf, fx, fy, fz)) continue;
        const int zmask = (yx == 0 ? 1 : 0) | (yy == 0 ? 2 : 0) | ((D == 3 && yz == 0) ? 4 : 0);
        const int kap = ((sx < 0 && yx > 0) ? 1 : 0) | ((sy < 0 && yy > 0) ? 2 : 0) |
                        ((D == 3 && sz < 0 && yz > 0) ? 4 : 0);
        const int64_t vf = fx + (int64_t)fy * Lf.pitch + (int64_t)fz * Lf.plane;
        for (int sub = 0; sub < (1 << D); ++sub)
          if ((sub & ~zmask) == 0) Pw[(int64_t)(kap | sub) * Lf.nslot + vf] = 0.0;
      }
}

// MINW wavefronts per SIMD at least.  With 2 (the rediscretised rows of a
// finest level) the 3D patch systems, which otherwise take the whole
// register file, spill some registers, which is cheaper than the lost
// latency hiding (level-6 BoxMG of the band workload 10.1 -> 8.7 ms); rows
// read from a stored operator keep one wavefront (level 5: 1.06 against
// 1.26 ms).
// cref (nullable): refined flags of the coarse cells; patches of cells that
// are not refined are skipped (adaptive levels)
// cells (nullable): list of the refined coarse cells; thread (cell, corner)
// solves the corner's orthant, which points into the cell
// Writes the reference region of orthant (sx, sy, sz) at coarse vertex V,
// value(yx, yy, yz) at fine vertex 3V + s y.  A point on an axis (y_i = 0) is
// shared by the orthants that differ only on such axes; it is written by the
// one of lowest rank (rank: bit i set when the orthant is negative on shared
// axis i) among those whose patch is computed: the + orthant on regular
// levels (cref null), the next refined one on adaptive levels.  The writer
// also writes the entries towards the second parent along the shared axes
// (at distance 3: weight zero), which no orthant computes; with them every
// entry of every fine vertex of a refined coarse cell is written once.
// dirty (nullable): the 64-slot blocks written are marked 1 there.
// yx_only (>= 0): only the points at that distance along x.
template <int D, class PV>
__device__ inline void write_orthant(const Lat& Lf, const Lat& Lc, double* __restrict__ Pw,
                                     const int8_t* __restrict__ cref, int Vx, int Vy, int Vz, int sx, int sy,
                                     int sz, PV&& value, int32_t* __restrict__ dirty = nullptr, int yx_only = -1) {
  const int zmax = (D == 3) ? 3 : 1;
  const int sneg = (sx < 0 ? 1 : 0) | (sy < 0 ? 2 : 0) | (sz < 0 ? 4 : 0);
  const int yx0 = yx_only < 0 ? 0 : yx_only, yx1 = yx_only < 0 ? 3 : yx_only + 1;
  for (int yz = 0; yz < zmax; ++yz)
    for (int yy = 0; yy < 3; ++yy)
      for (int yx = yx0; yx < yx1; ++yx) {
        const int zmask = (yx == 0 ? 1 : 0) | (yy == 0 ? 2 : 0) | ((D == 3 && yz == 0) ? 4 : 0);
        const int myrank = sneg & zmask;
        bool mine = true;
        if (cref == nullptr) {
          mine = myrank == 0;
        } else {
          for (int c = 0; c < myrank && mine; ++c) {
            if ((c & ~zmask) != 0) continue;  // candidates differ on shared axes only
            const int ox = (zmask & 1) ? ((c & 1) ? -1 : 1) : sx;
            const int oy = (zmask & 2) ? ((c & 2) ? -1 : 1) : sy;
            const int oz = (zmask & 4) ? ((c & 4) ? -1 : 1) : sz;
            if (orthant_refined(cref, Lc, Vx, Vy, Vz, ox, oy, oz)) mine = false;
          }
        }
        if (!mine) continue;
        const int fx = 3 * Vx + sx * yx, fy = 3 * Vy + sy * yy, fz = 3 * Vz + sz * yz;
        const int kap = ((sx < 0 && yx > 0) ? 1 : 0) | ((sy < 0 && yy > 0) ? 2 : 0) |
                        ((D == 3 && sz < 0 && yz > 0) ? 4 : 0);
        const int64_t vf = fx + (int64_t)fy * Lf.pitch + (int64_t)fz * Lf.plane;
        Pw[(int64_t)kap * Lf.nslot + vf] = value(yx, yy, yz);
        for (int sub = 1; sub < (1 << D); ++sub)
          if ((sub & ~zmask) == 0) Pw[(int64_t)(kap | sub) * Lf.nslot + vf] = 0.0;
        if (dirty != nullptr) dirty[vf / kSeg] = 1;
      }
}

// d-linear weight of a coarse vertex at distance y (0..2 fine steps) along one
// axis of its orthant
__device__ inline double dlin_ref(int y) { return y == 0 ? 1.0 : (y == 1 ? 2.0 / 3.0 : 1.0 / 3.0); }

// Constant-coefficient pass of the listed 3D cells with rediscretised rows.
// A cell whose 125 fine cells and the layer around them carry one eps (every
// row of its eight orthant systems reads only these) gets the d-linear
// weights of its orthants, which BoxMG reproduces there (up to rounding); the
// others are appended to dlist (count in *dcount) for the solve.  Kept apart
// from the solver kernel, whose register use leaves two wavefronts per SIMD:
// this pass is bound by memory and wants many more.
// Workgroup: kBoxCells cells, eight wavefronts.  The cells' eps are compared
// by all threads against each cell's centre value (a flag per cell in LDS);
// then wavefront w writes orthant w of every uniform cell, lane (cell, yx)
// the nine points at distance yx along x, so that the lanes of one store
// cover consecutive slots of a row when the listed cells are x-neighbours.
constexpr int kBoxCells = 21;  // 3 * 21 = 63 lanes of a wavefront
__global__ __launch_bounds__(512) void k_boxmg_uniform3(Lat Lf, Lat Lc, const double* __restrict__ eps,
                                                        double* __restrict__ Pw, const int8_t* __restrict__ cref,
                                                        const int32_t* __restrict__ cells, int64_t ncells,
                                                        int32_t* __restrict__ dlist, int32_t* __restrict__ dcount) {
  __shared__ int cc[3 * kBoxCells];
  __shared__ double cref_eps[kBoxCells];
  __shared__ int nonuni[kBoxCells];
  const int t = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * kBoxCells;
  const int ncw = (int)min<int64_t>(kBoxCells, ncells - c0);  // cells of this workgroup (>= 1)
  const int n = Lc.n;
  if (t < ncw) {
    const int64_t c = cells[c0 + t];
    const int x = (int)(c % n), y = (int)((c / n) % n), z = (int)(c / ((int64_t)n * n));
    cc[3 * t] = x;
    cc[3 * t + 1] = y;
    cc[3 * t + 2] = z;
    cref_eps[t] = eps[(3 * x + 1) + (int64_t)(3 * y + 1) * Lf.pitch + (int64_t)(3 * z + 1) * Lf.plane];
    nonuni[t] = 0;
  }
  __syncthreads();
  for (int k = t; k < ncw * 125; k += 512) {
    const int lc = k / 125, e = k - 125 * lc;
    const int x = 3 * cc[3 * lc] - 1 + e % 5, y = 3 * cc[3 * lc + 1] - 1 + (e / 5) % 5,
              z = 3 * cc[3 * lc + 2] - 1 + e / 25;
    if (x < 0 || y < 0 || z < 0 || x >= Lf.n || y >= Lf.n || z >= Lf.n) continue;
    if (!(eps[x + (int64_t)y * Lf.pitch + (int64_t)z * Lf.plane] == cref_eps[lc])) nonuni[lc] = 1;
  }
  __syncthreads();
  const int lane = t & 63, orth = t >> 6;
  if (orth == 0) {
    // the listed cells take consecutive places after one atomic increment
    const bool listed = lane < ncw && nonuni[lane] != 0;
    const uint64_t lead = __ballot(listed);
    int base = 0;
    if (lane == 0 && lead != 0) base = atomicAdd(dcount, (int)__popcll(lead));
    base = __shfl(base, 0, 64);
    if (listed) dlist[base + (int)__popcll(lead & ((1ull << lane) - 1ull))] = cells[c0 + lane];
  }
  const int lc = lane / 3, yx = lane - 3 * lc;
  if (lc >= ncw || nonuni[lc] != 0) return;
  const int Vx = cc[3 * lc] + (orth & 1), Vy = cc[3 * lc + 1] + ((orth >> 1) & 1),
            Vz = cc[3 * lc + 2] + ((orth >> 2) & 1);
  const int sx = (orth & 1) ? -1 : 1, sy = (orth & 2) ? -1 : 1, sz = (orth & 4) ? -1 : 1;
  if (!interior(Lc, Vx, Vy, Vz)) {
    zero_boundary_orthant<3>(Lf, Pw, Vx, Vy, Vz, sx, sy, sz, yx);
    return;
  }
  write_orthant<3>(Lf, Lc, Pw, cref, Vx, Vy, Vz, sx, sy, sz,
                   [](int ax, int ay, int az) { return dlin_ref(ax) * dlin_ref(ay) * dlin_ref(az); }, nullptr,
                   yx);
}

// pass (3D, listed cells): 0 solves every cell; 2 solves the *dcount cells
// of `cells` (the list k_boxmg_uniform3 leaves), in dense wavefronts instead
// of beside constant-coefficient cells that would wait for them.  dirty
// (nullable): marks the 64-slot blocks this launch writes.
template <int D, int MINW>
__global__ __launch_bounds__(64, MINW) void k_boxmg(Lat Lf, Lat Lc, BoxFetch<D> F, double* __restrict__ Pw,
                                              const int8_t* __restrict__ cref, const int32_t* __restrict__ cells,
                                              int64_t ncells, const int32_t* __restrict__ dcount, int pass,
                                              int32_t* __restrict__ dirty) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int m = Lc.n - 1;
  int orth, Vx, Vy, Vz;
  bool uniform = false;  // d-linear weights without the solve
  __shared__ double pl[27 * 64];
  if constexpr (D == 3) {
    // 3D: the 64 threads are the 8 corners of 8 coarse cells (the listed
    // ones, or every cell of a regular level), so that the corners sharing a
    // cell's member rows run together
    __shared__ int cc[8 * 3];
    const int n = Lc.n;
    const int lc = threadIdx.x >> 3;
    const int64_t ci = (int64_t)blockIdx.x * 8 + lc;
    const int64_t nc = pass == 2 ? (int64_t)*dcount : (cells ? ncells : (int64_t)n * n * n);
    bool active = ci < nc;
    if ((threadIdx.x & 7) == 0) {
      int x = -1000, y = -1000, z = -1000;
      if (active) {
        const int64_t c = cells ? (int64_t)cells[ci] : ci;
        x = (int)(c % n);
        y = (int)((c / n) % n);
        z = (int)(c / ((int64_t)n * n));
      }
      cc[3 * lc] = x;
      cc[3 * lc + 1] = y;
      cc[3 * lc + 2] = z;
    }
    __syncthreads();
    // Rediscretised rows: every row of the cell's eight orthant systems reads
    // only the cell's fine cells and the layer of fine cells around them.  A
    // constant coefficient there makes the rows those of constant eps, for
    // which BoxMG reproduces the d-linear weights (up to rounding); they are
    // then written without the solve.  The eight lanes of the cell split the
    // 125 cells (those inside the domain).
    if (F.A == nullptr && pass != 2) {
      const int x0 = 3 * cc[3 * lc] - 1, y0 = 3 * cc[3 * lc + 1] - 1, z0 = 3 * cc[3 * lc + 2] - 1;
      double lo = INFINITY, hi = -INFINITY;
      for (int e = (int)(threadIdx.x & 7); e < 125; e += 8) {
        const int x = x0 + e % 5, y = y0 + (e / 5) % 5, z = z0 + e / 25;
        if (x < 0 || y < 0 || z < 0 || x >= Lf.n || y >= Lf.n || z >= Lf.n) continue;
        const double v = F.eps[x + (int64_t)y * Lf.pitch + (int64_t)z * Lf.plane];
        lo = fmin(lo, v);
        hi = fmax(hi, v);
      }
#pragma unroll
      for (int o = 1; o < 8; o <<= 1) {
        lo = fmin(lo, __shfl_xor(lo, o, 64));
        hi = fmax(hi, __shfl_xor(hi, o, 64));
      }
      uniform = lo == hi;
    }
    if (!active) return;
    orth = (int)(threadIdx.x & 7);
    Vx = cc[3 * lc] + (orth & 1);
    Vy = cc[3 * lc + 1] + ((orth >> 1) & 1);
    Vz = cc[3 * lc + 2] + ((orth >> 2) & 1);
    if (!interior(Lc, Vx, Vy, Vz)) {
      if (cells) zero_boundary_orthant<D>(Lf, Pw, Vx, Vy, Vz, (orth & 1) ? -1 : 1, (orth & 2) ? -1 : 1,
                                          (orth & 4) ? -1 : 1);
      return;
    }
  } else if (cells) {
    if (t >= ncells * Dim<D>::NC) return;
    orth = (int)(t % Dim<D>::NC);
    const int64_t c = cells[t / Dim<D>::NC];
    const int n = Lc.n;
    Vx = (int)(c % n) + (orth & 1);
    Vy = (int)((c / n) % n) + ((orth >> 1) & 1);
    Vz = (D == 3) ? (int)(c / ((int64_t)n * n)) + ((orth >> 2) & 1) : 0;
    if (!interior(Lc, Vx, Vy, Vz)) {
      zero_boundary_orthant<D>(Lf, Pw, Vx, Vy, Vz, (orth & 1) ? -1 : 1, (orth & 2) ? -1 : 1,
                               (D == 3 && (orth & 4)) ? -1 : 1);
      return;
    }
  } else {
    const int64_t nV = (D == 3) ? (int64_t)m * m * m : (int64_t)m * m;
    if (t >= nV * Dim<D>::NC) return;
    orth = (int)(t % Dim<D>::NC);
    const int64_t Vi = t / Dim<D>::NC;
    Vx = (int)(Vi % m) + 1;
    Vy = (int)((Vi / m) % m) + 1;
    Vz = (D == 3) ? (int)(Vi / ((int64_t)m * m)) + 1 : 0;
  }
  const int sx = (orth & 1) ? -1 : 1, sy = (orth & 2) ? -1 : 1, sz = (D == 3 && (orth & 4)) ? -1 : 1;
  if (cref && !orthant_refined(cref, Lc, Vx, Vy, Vz, sx, sy, sz)) return;
  const PCol p{pl + threadIdx.x};
  if (uniform) {
    // d-linear weight of V at 3V + s y: the product over the axes of 1 - y_i / 3
#pragma unroll
    for (int q = 0; q < 27; ++q) {
      const int y0 = q % 3, y1 = (q / 3) % 3, y2 = q / 9;
      const double w0 = y0 == 0 ? 1.0 : (y0 == 1 ? 2.0 / 3.0 : 1.0 / 3.0);
      const double w1 = y1 == 0 ? 1.0 : (y1 == 1 ? 2.0 / 3.0 : 1.0 / 3.0);
      const double w2 = y2 == 0 ? 1.0 : (y2 == 1 ? 2.0 / 3.0 : 1.0 / 3.0);
      p[pidx(y0, y1, y2)] = w0 * w1 * w2;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 27; ++q) p[q] = 0.0;
    p[0] = 1.0;
    box_group<D, 1>(F, Vx, Vy, Vz, sx, sy, sz, p);
    box_group<D, 2>(F, Vx, Vy, Vz, sx, sy, sz, p);
    if constexpr (D == 3) {
      box_group<D, 4>(F, Vx, Vy, Vz, sx, sy, sz, p);
      box_group<D, 3>(F, Vx, Vy, Vz, sx, sy, sz, p);
      box_group<D, 5>(F, Vx, Vy, Vz, sx, sy, sz, p);
      box_group<D, 6>(F, Vx, Vy, Vz, sx, sy, sz, p);
      box_group<D, 7>(F, Vx, Vy, Vz, sx, sy, sz, p);
    } else {
      box_group<D, 3>(F, Vx, Vy, Vz, sx, sy, sz, p);
    }
  }
  write_orthant<D>(
      Lf, Lc, Pw, cref, Vx, Vy, Vz, sx, sy, sz, [&](int yx, int yy, int yz) { return p[pidx(yx, yy, yz)]; },
      dirty);
}

// ---------------------------------------------------------------------------
// Galerkin product (Sect. 4.3): A_c(V, W) = sum_i sum_j P(i,V) a(i,j) P(j,W)
// for interior coarse V and W in 3^d(V), i within 2 of 3V and |i - j| <= 1.
// ---------------------------------------------------------------------------
template <int D>
struct PFetch {
  const double* W;  // FP64 parent weights (2^d * nslot) or null for d-linear
  Lat Lf, Lc;
  // weight of coarse vertex (Vx,Vy,Vz) at fine (i,j,k); the caller guarantees
  // |f - 3V| <= 2 per axis
  __device__ double operator()(int i, int j, int k, int Vx, int Vy, int Vz) const {
    const int kx = Vx - i / 3, ky = Vy - j / 3, kz = (D == 3) ? Vz - k / 3 : 0;
    if (W) {
      const int64_t v = i + (int64_t)j * Lf.pitch + (int64_t)k * Lf.plane;
      return W[(int64_t)(kx | (ky << 1) | (kz << 2)) * Lf.nslot + v];
    }
    double w = (1.0 - abs(i - 3 * Vx) / 3.0) * (1.0 - abs(j - 3 * Vy) / 3.0);
    if (D == 3) w *= (1.0 - abs(k - 3 * Vz) / 3.0);
    return w;
  }
};

// Work shape of the Galerkin kernel: VPB coarse vertices V per workgroup
// (one in 3D, ten in 2D), 5^d fine vertices i within 2 of 3V each, and the
// fine region 3V + [-3, 3]^d that their stencils reach.
template <int D>
struct RapShape {
  static constexpr int NI = (D == 3) ? 125 : 25;
  static constexpr int VPB = (D == 3) ? 1 : 10;
  static constexpr int NT = (D == 3) ? 192 : 256;
  static constexpr int RW = 7;
  static constexpr int NR = (D == 3) ? 343 : 49;
  static constexpr int NP = (D == 3) ? 5 : 1;  // parts of one entry's sum (planes of j)
};

// A_c(V, W) = sum_j (sum_i P(i,V) a(i,j)) P(j,W), i within 2 of 3V, |i - j| <= 1,
// in three phases over LDS, each a gather in a fixed order:
//   1. one thread per i: P(i,V) and the row of i (from the store, or
//      rediscretised from eps with boundary entries dropped);
//   2. one task per fine j of the region: t(j) = sum_i P(i,V) a(i,j);
//   3. one thread per entry W - V in [-1,1]^d: sum over the j within 2 of 3W
//      of t(j) P(j,W).
// vtc (nullable): coarse vertex classes; rows of vertices that are not
// refined are left zero.  vlist (nullable): the nlist coarse vertices to form
// (interior indices); the others are not visited.
template <int D>
__global__ __launch_bounds__(RapShape<D>::NT) void k_rap(Lat Lf, Lat Lc, BoxFetch<D> A, PFetch<D> P,
                                                         double* __restrict__ Ac,
                                                         const int8_t* __restrict__ vtc,
                                                         const int32_t* __restrict__ vlist, int64_t nlist,
                                                         int rmode) {
  using S = RapShape<D>;
  constexpr int NS = Dim<D>::NS, NC = Dim<D>::NC;
  __shared__ double arow[S::VPB * S::NI * NS];
  __shared__ double piv[S::VPB * S::NI];
  __shared__ double tj[S::VPB * S::NR];
  __shared__ int vco[S::VPB * 4];  // per vertex: x, y, z, active
  __shared__ double tpart[S::VPB * Dim<D>::NS * S::NP];
  const int m = Lc.n - 1;
  const int64_t nV = vlist ? nlist : ((D == 3) ? (int64_t)m * m * m : (int64_t)m * m);
  const int t = threadIdx.x;
  if (t < S::VPB) {
    const int64_t idx = (int64_t)blockIdx.x * S::VPB + t;
    int vx = 1, vy = 1, vz = 0, on = 0;
    if (idx < nV) {
      const int64_t vv = vlist ? (int64_t)vlist[idx] : idx;
      vx = (int)(vv % m) + 1;
      vy = (int)((vv / m) % m) + 1;
      vz = (D == 3) ? (int)(vv / ((int64_t)m * m)) + 1 : 0;
      on = (vtc == nullptr || vtc[vx + (int64_t)vy * Lc.pitch + (int64_t)vz * Lc.plane] == VT_REFINED) ? 1 : 2;
    }
    vco[4 * t] = vx;
    vco[4 * t + 1] = vy;
    vco[4 * t + 2] = vz;
    vco[4 * t + 3] = on;  // 0: none, 1: form the row, 2: write a zero row
  }
  __syncthreads();
  // phase 1: weights and rows of the i of each vertex
  {
    const int vs = t / S::NI, q = t - (t / S::NI) * S::NI;
    if (vs < S::VPB) {
      double pi = 0.0;
      double* ar = arow + (vs * S::NI + q) * NS;
      if (vco[4 * vs + 3] == 1) {
        const int Vx = vco[4 * vs], Vy = vco[4 * vs + 1], Vz = vco[4 * vs + 2];
        const int ix = 3 * Vx + q % 5 - 2, iy = 3 * Vy + (q / 5) % 5 - 2, iz = (D == 3) ? 3 * Vz + q / 25 - 2 : 0;
        // Petrov-Galerkin R (rmode 1: injection, only i = 3V; 2: aggregation,
        // unit weights on the i within 1 of 3V) or R = P^T (rmode 0)
        if (rmode == 1) pi = q == S::NI / 2 ? 1.0 : 0.0;
        else if (rmode == 2)
          pi = (abs(ix - 3 * Vx) <= 1 && abs(iy - 3 * Vy) <= 1 && (D == 2 || abs(iz - 3 * Vz) <= 1)) ? 1.0 : 0.0;
        else pi = P(ix, iy, iz, Vx, Vy, Vz);
        const int64_t vi = ix + (int64_t)iy * Lf.pitch + (int64_t)iz * Lf.plane;
        const RowSrc<D> row(A, vi);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          double a = 0.0;
          if (row.mode == 1 || (row.mode == 2 && interior(Lf, ix + off_x(k), iy + off_y(k),
                                                            iz + (D == 3 ? off_z(k) : 0))))
            a = row.entry(A, vi, k);
          ar[k] = a;
        }
      } else {
#pragma unroll
        for (int k = 0; k < NS; ++k) ar[k] = 0.0;
      }
      piv[vs * S::NI + q] = pi;
    }
  }
  __syncthreads();
  // phase 2: t(j) = sum_i P(i,V) a(i,j) over the i = j - o_k inside the box
  for (int e = t; e < S::VPB * S::NR; e += S::NT) {
    const int vs = e / S::NR, jr = e - (e / S::NR) * S::NR;
    const int jx = jr % S::RW - 3, jy = (jr / S::RW) % S::RW - 3, jz = (D == 3) ? jr / (S::RW * S::RW) - 3 : 0;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int ox = jx - off_x(k), oy = jy - off_y(k), oz = (D == 3) ? jz - off_z(k) : 0;
      if (ox < -2 || ox > 2 || oy < -2 || oy > 2 || oz < -2 || oz > 2) continue;
      const int qi = (ox + 2) + 5 * (oy + 2) + (D == 3 ? 25 * (oz + 2) : 0);
      acc += piv[vs * S::NI + qi] * arow[(vs * S::NI + qi) * NS + k];
    }
    tj[e] = acc;
  }
  __syncthreads();
  // phase 3: A_c(V, W) = sum_j t(j) P(j, W), j within 2 of 3W inside the
  // region; in 3D each entry's sum is split over the (up to 5) planes of j,
  // whose partial sums are then added in order
  if (t < S::VPB * NS * S::NP) {
    const int vs = t / (NS * S::NP), w = (t / S::NP) % NS, part = t % S::NP;
    const int on = vco[4 * vs + 3];
    double acc = 0.0;
    if (on == 1) {
      const int Vx = vco[4 * vs], Vy = vco[4 * vs + 1], Vz = vco[4 * vs + 2];
      const int dx = off_x(w), dy = off_y(w), dz = (D == 3) ? off_z(w) : 0;
      // region offsets of j per axis: [3d - 2, 3d + 2] clipped to [-3, 3]
      const int xl = max(3 * dx - 2, -3), xh = min(3 * dx + 2, 3);
      const int yl = max(3 * dy - 2, -3), yh = min(3 * dy + 2, 3);
      const int zl = (D == 3) ? max(3 * dz - 2, -3) + part : 0;
      const int zh = (D == 3) ? min(min(3 * dz + 2, 3), zl) : 0;
      if (interior(Lc, Vx + dx, Vy + dy, Vz + dz)) {
        for (int jz = zl; jz <= zh; ++jz)
          for (int jy = yl; jy <= yh; ++jy)
#pragma unroll 5
            for (int jx = xl; jx <= xh; ++jx) {
              const int jr = (jx + 3) + S::RW * ((jy + 3) + (D == 3 ? S::RW * (jz + 3) : 0));
              // parent index of W at j: W - floor(j/3) per axis (j = 3V + offset)
              const int kx = dx - (jx + 3) / 3 + 1, ky = dy - (jy + 3) / 3 + 1;
              const int kz = (D == 3) ? dz - (jz + 3) / 3 + 1 : 0;
              double pj;
              if (P.W) {  // BoxMG weight of W at j, from the L2-resident weight arrays
                const int64_t vj = (3 * Vx + jx) + (int64_t)(3 * Vy + jy) * Lf.pitch +
                                   (D == 3 ? (int64_t)(3 * Vz + jz) * Lf.plane : 0);
                pj = P.W[(int64_t)(kx | (ky << 1) | (kz << 2)) * Lf.nslot + vj];
              } else {
                const int rx = (jx + 3) % 3, ry = (jy + 3) % 3, rz = (D == 3) ? (jz + 3) % 3 : 0;
                pj = dlin1(rx, kx) * dlin1(ry, ky) * (D == 3 ? dlin1(rz, kz) : 1.0);
              }
              acc += tj[vs * S::NR + jr] * pj;
            }
      }
    }
    tpart[t] = acc;
  }
  __syncthreads();
  if (t < S::VPB * NS) {
    const int vs = t / NS, w = t - (t / NS) * NS;
    if (vco[4 * vs + 3] != 0) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < S::NP; ++q) acc += tpart[t * S::NP + q];
      Ac[(int64_t)w * Lc.nslot + vco[4 * vs] + (int64_t)vco[4 * vs + 1] * Lc.pitch +
         (int64_t)vco[4 * vs + 2] * Lc.plane] = acc;
    }
  }
}

// Galerkin product from a rediscretised 3D fine operator (the finest level),
// cell by cell.  The fine operator is the sum over fine cells e of
// h eps_e K, with K the Q1 reference element matrix (kref by the number of
// coordinates in which two corners differ), restricted to the rows m(a) = 1
// of vertices that have one (leaf vertices of an adaptive level; every
// interior vertex of a regular one), so
//   A_c(V,W) = sum_e h eps_e sum_{a,b in e} P(a,V) m(a) K(a,b) P(b,W).
// This is P^T A P of the row form: every fine cell that touches a vertex of
// V's support (within 2 of 3V) lies among the 6^3 cells around 3V.
// One workgroup per coarse vertex V.  The prolongation weights of the 7^3
// fine vertices around 3V (all eight parents), the 6^3 cell coefficients and
// the row mask are staged in LDS with row-contiguous loads; then
//   t(j)     = sum_{a} pv(a) sum_{e containing a and j} h eps_e K(a,j),
//              pv(a) = P(a,V) m(a)                             (343 j)
//   A_c(V,W) = sum_j t(j) P(j,W)                               (27 W, each
//              split over the five planes of j and added in order).
// In t(j) the 3D Q1 element couples j with itself (all 8 cells), with its 12
// face-diagonal neighbours (the 2 cells they share) and its 8 body-diagonal
// neighbours (1 cell); its edge neighbours have K = 0.
// Every sum runs in a fixed order, so results are bitwise reproducible.
constexpr int kRfR = 7;                    // region width (vertices) per axis
constexpr int kRfNR = kRfR * kRfR * kRfR;  // 343 region vertices
constexpr int kRfP = kRfR + 2;             // pv with a zero border of one
constexpr int kRfNT = 384;
constexpr int kRfLoads = (8 * kRfNR + kRfNT - 1) / kRfNT;

__global__ __launch_bounds__(kRfNT) void k_rap_fine3(Lat Lf, Lat Lc, const double* __restrict__ eps,
                                                     const double* __restrict__ Pw,
                                                     const int8_t* __restrict__ vt_fine,
                                                     double* __restrict__ Ac, const int8_t* __restrict__ vtc,
                                                     const int32_t* __restrict__ vlist, int64_t nlist) {
  __shared__ double pw[8 * kRfNR];             // [parent kappa][region vertex], x fastest
  __shared__ double ec[216];                   // cells with low corner 3V + [-3, 2]^3
  __shared__ double pv[kRfP * kRfP * kRfP];    // P(a,V) m(a), zero beyond 2 of 3V
  __shared__ double tj[kRfNR];
  double* const tpart = pv;  // 27 * 5 partial sums, once pv is no longer read
  const int m = Lc.n - 1;
  const int t = threadIdx.x;
  // a 2D grid of workgroups (x fastest): one dimension of a launch is
  // limited to 2^32 work-items, which a regular level-5 list exceeds
  const int64_t idx = blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
  const int64_t nV = vlist ? nlist : (int64_t)m * m * m;
  if (idx >= nV) return;  // uniform over the workgroup
  const int64_t vv = vlist ? (int64_t)vlist[idx] : idx;
  const int Vx = (int)(vv % m) + 1, Vy = (int)((vv / m) % m) + 1, Vz = (int)(vv / ((int64_t)m * m)) + 1;
  const int64_t vc = Vx + (int64_t)Vy * Lc.pitch + (int64_t)Vz * Lc.plane;
  const bool form = vtc == nullptr || vtc[vc] == VT_REFINED;
  if (!form) {  // a listed vertex that is not refined keeps a zero row
    if (t < 27) Ac[(int64_t)t * Lc.nslot + vc] = 0.0;
    return;
  }
  // region origin: fine vertex 3V - 3 per axis (inside the lattice: V >= 1)
  const int64_t r0 = (3 * Vx - 3) + (int64_t)(3 * Vy - 3) * Lf.pitch + (int64_t)(3 * Vz - 3) * Lf.plane;
  // stage the weights of all eight parents of every region vertex
  {
    double w[kRfLoads];
#pragma unroll
    for (int r = 0; r < kRfLoads; ++r) {
      const int e = t + r * kRfNT;
      w[r] = 0.0;
      if (e < 8 * kRfNR) {
        const int kap = e / kRfNR, q = e - kap * kRfNR;
        const int qx = q % kRfR, qy = (q / kRfR) % kRfR, qz = q / (kRfR * kRfR);
        if (Pw) {
          w[r] = Pw[(int64_t)kap * Lf.nslot + r0 + qx + (int64_t)qy * Lf.pitch + (int64_t)qz * Lf.plane];
        } else {  // d-linear: parent floor(j/3) + kappa, j = 3V - 3 + q
          w[r] = dlin1(qx % 3, kap & 1) * dlin1(qy % 3, (kap >> 1) & 1) * dlin1(qz % 3, kap >> 2);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kRfLoads; ++r) {
      const int e = t + r * kRfNT;
      if (e < 8 * kRfNR) pw[e] = w[r];
    }
  }
  if (t < 216) {
    const int cx = t % 6, cy = (t / 6) % 6, cz = t / 36;
    ec[t] = eps[r0 + cx + (int64_t)cy * Lf.pitch + (int64_t)cz * Lf.plane];
  }
  for (int q = t; q < kRfP * kRfP * kRfP; q += kRfNT) pv[q] = 0.0;
  int8_t cls = VT_LEAF;
  if (vt_fine && t < kRfNR) {
    const int qx = t % kRfR, qy = (t / kRfR) % kRfR, qz = t / (kRfR * kRfR);
    cls = vt_fine[r0 + qx + (int64_t)qy * Lf.pitch + (int64_t)qz * Lf.plane];
  }
  __syncthreads();
  // pv(a) = P(a, V) m(a) for a = 3V + o, |o| <= 2 per axis: V is parent
  // kappa = -floor(o / 3) of a (1 for o < 0, else 0)
  if (t < kRfNR) {
    const int qx = t % kRfR, qy = (t / kRfR) % kRfR, qz = t / (kRfR * kRfR);
    const int ox = qx - 3, oy = qy - 3, oz = qz - 3;
    const bool has_row = cls == VT_LEAF || cls == VT_REFINED;
    if (ox >= -2 && ox <= 2 && oy >= -2 && oy <= 2 && oz >= -2 && oz <= 2 && has_row) {
      const int kap = (ox < 0 ? 1 : 0) | (oy < 0 ? 2 : 0) | (oz < 0 ? 4 : 0);
      pv[(qx + 1) + kRfP * ((qy + 1) + kRfP * (qz + 1))] = pw[kap * kRfNR + t];
    }
  }
  __syncthreads();
  if (t < kRfNR) {
    const int qx = t % kRfR, qy = (t / kRfR) % kRfR, qz = t / (kRfR * kRfR);
    const int jx = 3 * Vx - 3 + qx, jy = 3 * Vy - 3 + qy, jz = 3 * Vz - 3 + qz;
    double acc = 0.0;
    if (interior(Lf, jx, jy, jz)) {
      // coefficient of cell j - c (c in {0,1}^3), zero outside the staged cells
      double E[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int ex = qx - (c & 1), ey = qy - ((c >> 1) & 1), ez = qz - (c >> 2);
        E[c] = (ex >= 0 && ex <= 5 && ey >= 0 && ey <= 5 && ez >= 0 && ez <= 5) ? ec[ex + 6 * (ey + 6 * ez)]
                                                                                : 0.0;
      }
      const int j0 = (qx + 1) + kRfP * ((qy + 1) + kRfP * (qz + 1));
      double sE = 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c) sE += E[c];
      acc = kref(3, 0) * pv[j0] * sE;
      // neighbour j + delta, delta in {-1,0,1}^3: a cell j - c holds it when
      // c = 1 on the axes with delta = -1 and c = 0 where delta = +1
#pragma unroll
      for (int k = 0; k < 27; ++k) {
        const int dx = off_x(k), dy = off_y(k), dz = off_z(k);
        const int nd = (dx != 0) + (dy != 0) + (dz != 0);
        if (nd < 2) continue;  // the centre is done; edge neighbours have K = 0
        double es = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
          const bool holds = (dx == 0 || cx == (dx < 0 ? 1 : 0)) && (dy == 0 || cy == (dy < 0 ? 1 : 0)) &&
                             (dz == 0 || cz == (dz < 0 ? 1 : 0));
          if (holds) es += E[c];
        }
        acc += kref(3, nd) * pv[j0 + dx + kRfP * (dy + kRfP * dz)] * es;
      }
      acc *= Lf.h;
    }
    tj[t] = acc;
  }
  __syncthreads();
  // A_c(V, W), W = V + d: the j = 3V + o within 2 of 3W, split over planes
  if (t < 27 * 5) {
    const int w = t / 5, part = t % 5;
    const int dx = off_x(w), dy = off_y(w), dz = off_z(w);
    double acc = 0.0;
    if (interior(Lc, Vx + dx, Vy + dy, Vz + dz)) {
      const int xl = max(3 * dx - 2, -3), xh = min(3 * dx + 2, 3);
      const int yl = max(3 * dy - 2, -3), yh = min(3 * dy + 2, 3);
      const int zl = max(3 * dz - 2, -3) + part;
      const int zh = min(min(3 * dz + 2, 3), zl);
      for (int oz = zl; oz <= zh; ++oz)
        for (int oy = yl; oy <= yh; ++oy)
#pragma unroll 5
          for (int ox = xl; ox <= xh; ++ox) {
            const int q = (ox + 3) + kRfR * ((oy + 3) + kRfR * (oz + 3));
            // W's parent index at j: d - floor(o / 3) per axis
            const int kx = dx - (ox + 3) / 3 + 1, ky = dy - (oy + 3) / 3 + 1, kz = dz - (oz + 3) / 3 + 1;
            acc += tj[q] * pw[(kx | (ky << 1) | (kz << 2)) * kRfNR + q];
          }
    }
    tpart[t] = acc;
  }
  __syncthreads();
  if (t < 27) {
    double acc = 0.0;
#pragma unroll
    for (int p = 0; p < 5; ++p) acc += tpart[t * 5 + p];
    Ac[(int64_t)t * Lc.nslot + vc] = acc;
  }
}

// The same product coarse cell by coarse cell (adaptive levels, where only
// the refined coarse cells take part).  A coarse cell C holds 27 fine cells
// and 4^3 fine vertices b (local 0..3 per axis); its element matrix is
//   A_C(V,W) = sum_b T(b,V) P(b,W),
//   T(b,V)   = sum_{a in C} P(a,V) m(a) sum_{e in C containing a and b} h eps_e K(a,b),
// over the corners V, W of C, and the coarse row of V sums the element
// matrices of its eight cells.  A fine vertex b's parents inside C: along an
// axis, local 0 is coarse plane C (parent C, kappa 0; the second parent has
// weight zero), 1 and 2 lie between (kappa 0 and 1), 3 is plane C + 1 (parent
// C + 1 only, kappa 0).  One workgroup of 64 threads (one per b) per listed
// cell; 4 KB of fine data per cell instead of 22 KB per coarse vertex.
__global__ __launch_bounds__(64) void k_rap_cells3(Lat Lf, Lat Lc, const double* __restrict__ eps,
                                                   const double* __restrict__ Pw,
                                                   const int8_t* __restrict__ vt_fine,
                                                   const int32_t* __restrict__ cells, int64_t ncells,
                                                   double* __restrict__ AC) {
  __shared__ double P[64 * 8];  // [b][corner]
  __shared__ double T[64 * 8];
  __shared__ double E[27];
  __shared__ double msk[64];    // m(b): 1 where b has a row, else 0
  const int64_t ci = blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
  if (ci >= ncells) return;  // uniform over the workgroup
  const int n = Lc.n;
  const int64_t c = cells[ci];
  const int Cx = (int)(c % n), Cy = (int)((c / n) % n), Cz = (int)(c / ((int64_t)n * n));
  const int t = threadIdx.x;
  const int lx = t & 3, ly = (t >> 2) & 3, lz = t >> 4;
  const int bx = 3 * Cx + lx, by = 3 * Cy + ly, bz = 3 * Cz + lz;
  const int64_t vb = bx + (int64_t)by * Lf.pitch + (int64_t)bz * Lf.plane;
  const int8_t cls = vt_fine ? vt_fine[vb] : (int8_t)VT_LEAF;
  const bool has_row = cls == VT_LEAF || cls == VT_REFINED;
  // The weights towards C's corners at its 64 fine vertices come from BoxMG
  // edge, face and interior systems (whichever orthant writes them) whose
  // rows read only the 125 fine cells of C and the layer around it.  With one
  // coefficient there they are the d-linear weights; with every vertex
  // inside the domain and with a row the product is then the coarse element
  // matrix, written without loading the weights.
  {
    double lo = INFINITY, hi = -INFINITY;
    for (int e = t; e < 125; e += 64) {
      const int x = 3 * Cx - 1 + e % 5, y = 3 * Cy - 1 + (e / 5) % 5, z = 3 * Cz - 1 + e / 25;
      if (x < 0 || y < 0 || z < 0 || x >= Lf.n || y >= Lf.n || z >= Lf.n) continue;
      const double v = eps[x + (int64_t)y * Lf.pitch + (int64_t)z * Lf.plane];
      lo = fmin(lo, v);
      hi = fmax(hi, v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, o, 64));
      hi = fmax(hi, __shfl_xor(hi, o, 64));
    }
    if (__syncthreads_and(lo == hi && has_row && interior(Lf, bx, by, bz))) {
      const int V = t >> 3, Wc = t & 7;
      const int nd = (V ^ Wc) == 0 ? 0 : __popc((unsigned)(V ^ Wc));
      AC[ci * 64 + t] = kref(3, nd) * lo * (3.0 * Lf.h);
      return;
    }
  }
  bool dlin = true;  // every weight the d-linear one, bit for bit
#pragma unroll
  for (int cc = 0; cc < 8; ++cc) {
    const int kx = (cc & 1) - (lx == 3 ? 1 : 0), ky = ((cc >> 1) & 1) - (ly == 3 ? 1 : 0),
              kz = (cc >> 2) - (lz == 3 ? 1 : 0);
    double w = 0.0;
    // parents that exist, less the second parent of a vertex on a coarse
    // plane (local 0), whose weight is zero by construction
    const bool par = kx >= 0 && ky >= 0 && kz >= 0 && !(kx == 1 && lx == 0) && !(ky == 1 && ly == 0) &&
                     !(kz == 1 && lz == 0);
    if (par) {
      const int kap = kx | (ky << 1) | (kz << 2);
      const double wd = dlin1(bx % 3, kx) * dlin1(by % 3, ky) * dlin1(bz % 3, kz);
      w = Pw ? Pw[(int64_t)kap * Lf.nslot + vb] : wd;
      dlin = dlin && w == wd;
    }
    P[t * 8 + cc] = w;
  }
  msk[t] = has_row ? 1.0 : 0.0;
  if (t < 27) {
    const int ex = t % 3, ey = (t / 3) % 3, ez = t / 9;
    E[t] = eps[(3 * Cx + ex) + (int64_t)(3 * Cy + ey) * Lf.pitch + (int64_t)(3 * Cz + ez) * Lf.plane];
  }
  __syncthreads();
  // Every fine vertex of the cell inside the domain, with a row and the
  // d-linear weights, and one coefficient on the 27 fine cells: the product
  // is then the Galerkin product of nested d-linear spaces, the coarse
  // element matrix of that coefficient (side 3h), written without the sums.
  if (__syncthreads_and(has_row && dlin && interior(Lf, bx, by, bz) && (t >= 27 || E[t] == E[0]))) {
    const int V = t >> 3, Wc = t & 7;
    const int nd = (V ^ Wc) == 0 ? 0 : __popc((unsigned)(V ^ Wc));
    AC[ci * 64 + t] = kref(3, nd) * E[0] * (3.0 * Lf.h);
    return;
  }
  {
    double acc[8];
#pragma unroll
    for (int V = 0; V < 8; ++V) acc[V] = 0.0;
    if (interior(Lf, bx, by, bz)) {
      // cells b - c of C (local cell coordinates 0..2)
      double Ec[8];
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int ex = lx - (cc & 1), ey = ly - ((cc >> 1) & 1), ez = lz - (cc >> 2);
        Ec[cc] = (ex >= 0 && ex <= 2 && ey >= 0 && ey <= 2 && ez >= 0 && ez <= 2) ? E[ex + 3 * (ey + 3 * ez)] : 0.0;
      }
      double sE = 0.0;
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) sE += Ec[cc];
      const double mb = msk[t];
#pragma unroll
      for (int V = 0; V < 8; ++V) acc[V] = kref(3, 0) * (P[t * 8 + V] * mb) * sE;
      // neighbours b + delta inside the closed cell; the 3D Q1 element couples
      // face- and body-diagonal neighbours only (edge neighbours: K = 0)
#pragma unroll
      for (int k = 0; k < 27; ++k) {
        const int dx = off_x(k), dy = off_y(k), dz = off_z(k);
        const int nd = (dx != 0) + (dy != 0) + (dz != 0);
        if (nd < 2) continue;
        const int ax = lx + dx, ay = ly + dy, az = lz + dz;
        if (ax < 0 || ax > 3 || ay < 0 || ay > 3 || az < 0 || az > 3) continue;
        double es = 0.0;
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
          const int cx = cc & 1, cy = (cc >> 1) & 1, cz = cc >> 2;
          const bool holds = (dx == 0 || cx == (dx < 0 ? 1 : 0)) && (dy == 0 || cy == (dy < 0 ? 1 : 0)) &&
                             (dz == 0 || cz == (dz < 0 ? 1 : 0));
          if (holds) es += Ec[cc];
        }
        const int a = ax + 4 * (ay + 4 * az);
        const double kw = kref(3, nd) * es, ma = msk[a];
#pragma unroll
        for (int V = 0; V < 8; ++V) acc[V] += kw * (P[a * 8 + V] * ma);
      }
#pragma unroll
      for (int V = 0; V < 8; ++V) acc[V] *= Lf.h;
    }
#pragma unroll
    for (int V = 0; V < 8; ++V) T[t * 8 + V] = acc[V];
  }
  __syncthreads();
  {
    const int V = t >> 3, Wc = t & 7;
    double acc = 0.0;
    for (int b = 0; b < 64; ++b) acc += T[b * 8 + V] * P[b * 8 + Wc];
    AC[ci * 64 + t] = acc;
  }
}

// Coarse rows of the listed vertices from the element matrices of their eight
// refined cells (cidx: list index of each coarse cell, -1 when not listed);
// entry W - V sums the cells that hold both, in corner order.  Rows of
// listed vertices that are not refined, and entries towards boundary
// vertices, are zero.
__global__ __launch_bounds__(256) void k_rap_assemble3(Lat Lc, const double* __restrict__ AC,
                                                       const int32_t* __restrict__ cidx,
                                                       const int32_t* __restrict__ vlist, int64_t nlist,
                                                       const int8_t* __restrict__ vtc, double* __restrict__ Ac) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nlist) return;
  const int n = Lc.n, m = n - 1;
  const int64_t vv = vlist[i];
  const int Vx = (int)(vv % m) + 1, Vy = (int)((vv / m) % m) + 1, Vz = (int)(vv / ((int64_t)m * m)) + 1;
  const int64_t vc = Vx + (int64_t)Vy * Lc.pitch + (int64_t)Vz * Lc.plane;
  double acc[27];
#pragma unroll
  for (int w = 0; w < 27; ++w) acc[w] = 0.0;
  if (vtc == nullptr || vtc[vc] == VT_REFINED) {
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int cx = Vx - (cc & 1), cy = Vy - ((cc >> 1) & 1), cz = Vz - (cc >> 2);
      const int32_t idx = cidx[cx + (int64_t)n * (cy + (int64_t)n * cz)];
      if (idx < 0) continue;
      const double* row = AC + (int64_t)idx * 64 + cc * 8;
#pragma unroll
      for (int wl = 0; wl < 8; ++wl) {
        const int dx = (wl & 1) - (cc & 1), dy = ((wl >> 1) & 1) - ((cc >> 1) & 1), dz = (wl >> 2) - (cc >> 2);
        acc[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] += row[wl];
      }
    }
  }
#pragma unroll
  for (int w = 0; w < 27; ++w) {
    const bool in = interior(Lc, Vx + off_x(w), Vy + off_y(w), Vz + off_z(w));
    Ac[(int64_t)w * Lc.nslot + vc] = in ? acc[w] : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_cell_index(const int32_t* __restrict__ cells, int64_t ncells,
                                                    int32_t* __restrict__ cidx) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < ncells) cidx[cells[i]] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <int D>
__global__ __launch_bounds__(256) void k_check_rows(Lat Lc, const double* __restrict__ Ac,
                                                    int* __restrict__ bad) {
  constexpr int NS = Dim<D>::NS;
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int kz = (D == 3) ? (int)blockIdx.z : 0;
  if (!interior(Lc, i, j, kz)) return;
  const int64_t v = i + (int64_t)j * Lc.pitch + (int64_t)kz * Lc.plane;
  const double dg = Ac[(int64_t)(NS / 2) * Lc.nslot + v];
  double off = 0.0;
  for (int k = 0; k < NS; ++k)
    if (k != NS / 2) off += fabs(Ac[(int64_t)k * Lc.nslot + v]);
  if (dg == 0.0 && off == 0.0) return;  // no row (adaptive levels: not a refined vertex)
  if (dg <= 0.0 || dg < (1.0 - kDomSlack) * off) atomicAdd(bad, 1);
}

// ---------------------------------------------------------------------------
// Convection term of eq. (1): the Galerkin Q1 element matrix of (v . grad) u
// with v constant per cell, C(a,b) = h^(d-1) sum_i v_i g(a_i,b_i)
// prod_{j!=i} m(a_j,b_j), g = [[-1/2, 1/2], [-1/2, 1/2]], m the unit 1D mass;
// added to the rows of the interior vertices (entries towards boundary
// vertices dropped).  vel holds d arrays of cell slots.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr double conv_g(int a, int b) { return b ? 0.5 : -0.5; }
__host__ __device__ constexpr double conv_m(int a, int b) { return a == b ? 1.0 / 3.0 : 1.0 / 6.0; }

template <int D>
__global__ __launch_bounds__(256) void k_conv_add(Lat L, const double* __restrict__ vel, double* __restrict__ A) {
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int kz = (D == 3) ? (int)blockIdx.z : 0;
  if (!interior(L, i, j, kz)) return;
  const int64_t v = i + (int64_t)j * L.pitch + (int64_t)kz * L.plane;
  const double hd1 = D == 3 ? L.h * L.h : L.h;
  constexpr int NS = Dim<D>::NS;
  double row[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) row[k] = 0.0;
  for (int sc = 0; sc < (1 << D); ++sc) {  // the vertex is corner s of cell v - s
    const int s0 = sc & 1, s1 = (sc >> 1) & 1, s2 = (sc >> 2) & 1;
    const int64_t cell = v - s0 - (int64_t)s1 * L.pitch - (D == 3 ? (int64_t)s2 * L.plane : 0);
    double vc[3];
    for (int a = 0; a < D; ++a) vc[a] = vel[(int64_t)a * L.nslot + cell];
    for (int wc = 0; wc < (1 << D); ++wc) {
      const int w0 = wc & 1, w1 = (wc >> 1) & 1, w2 = (wc >> 2) & 1;
      double c;
      if (D == 2) {
        c = vc[0] * conv_g(s0, w0) * conv_m(s1, w1) + vc[1] * conv_m(s0, w0) * conv_g(s1, w1);
      } else {
        c = vc[0] * conv_g(s0, w0) * conv_m(s1, w1) * conv_m(s2, w2) +
            vc[1] * conv_m(s0, w0) * conv_g(s1, w1) * conv_m(s2, w2) +
            vc[2] * conv_m(s0, w0) * conv_m(s1, w1) * conv_g(s2, w2);
      }
      const int k = (w0 - s0 + 1) + 3 * (w1 - s1 + 1) + (D == 3 ? 9 * (w2 - s2 + 1) : 0);
      row[k] += hd1 * c;
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (!interior(L, i + off_x(k), j + off_y(k), kz + (D == 3 ? off_z(k) : 0))) continue;
    A[(int64_t)k * L.nslot + v] += row[k];
  }
}

// ---------------------------------------------------------------------------
// Delta store.  One wavefront = one 64-slot block.
// ---------------------------------------------------------------------------
template <int D, bool IS_P>
__device__ inline int load_delta(const Lat& L, const Lat& Lc, const double* __restrict__ full,
                                 const double* __restrict__ eps, const int8_t* __restrict__ vt, int i, int j,
                                 int kz, int64_t v, double (&dl)[27], double& refmax) {
  constexpr int NE = IS_P ? Dim<D>::NC : Dim<D>::NS;
  refmax = 0.0;
  // vt (adaptive levels): rows of slots outside the level are never read
  if (!interior(L, i, j, kz) || (vt != nullptr && vt[v] == VT_OUT)) {
    for (int k = 0; k < NE; ++k) dl[k] = 0.0;
    return NE;
  }
  if (IS_P) {
    for (int c = 0; c < NE; ++c) {
      const double r = dlin_dropped<D>(Lc, i, j, kz, c);
      dl[c] = full[(int64_t)c * L.nslot + v] - r;
      refmax = fmax(refmax, fabs(r));
    }
  } else {
    double g[Dim<D>::NS];
    geom_row<D, double>(eps, v, L, g);
    for (int k = 0; k < NE; ++k) {
      const bool in = interior(L, i + off_x(k), j + off_y(k), kz + (D == 3 ? off_z(k) : 0));
      const double r = in ? g[k] : 0.0;
      dl[k] = full[(int64_t)k * L.nslot + v] - r;
      refmax = fmax(refmax, fabs(r));
    }
  }
  return NE;
}

// Per 64-slot block (one wavefront): 1 when any vertex's delta is non-zero
// (max|delta| > eps_zero * max|reference|), else 0.  With eps_mf > 0 the
// block's width instead: the largest per-vertex bpa (0 for all-zero codes).
// marked: blk holds 1 for the blocks whose entries may differ from their
// reference and 0 for the others, which are known zero and not loaded.
template <int D, bool IS_P>
__global__ __launch_bounds__(256) void k_delta_flags(Lat L, Lat Lc, const double* __restrict__ full,
                                                     const double* __restrict__ eps,
                                                     int32_t* __restrict__ blk, double eps_mf,
                                                     const int32_t* __restrict__ tiles, double eps_zero,
                                                     const int8_t* __restrict__ vt, int marked) {
  const int32_t* tl = tiles ? tiles + 3 * (int64_t)blockIdx.x : nullptr;
  const int i = (tl ? tl[0] : (int)blockIdx.x) * TX + threadIdx.x;
  const int j = (tl ? tl[1] : (int)blockIdx.y) * TY + threadIdx.y;
  const int kz = (D == 3) ? (tl ? tl[2] : (int)blockIdx.z) : 0;
  const bool inlat = j <= L.n && (D == 2 || kz <= L.n);
  const int64_t v = i + (int64_t)j * L.pitch + (int64_t)kz * L.plane;
  double dl[27], refmax;
  int nz = 0;
  // a clean block keeps its zero (one wavefront is one block: every lane
  // reads the flag before lane 0 writes it)
  const bool clean = marked && inlat && blk[v / kSeg] == 0;
  if (inlat && !clean) {
    const int ne = load_delta<D, IS_P>(L, Lc, full, eps, vt, i, j, kz, v, dl, refmax);
    if (eps_mf > 0.0) {
      nz = bpa_width(dl, ne, eps_mf);
    } else {
      double mx = 0.0;
      for (int k = 0; k < ne; ++k) mx = fmax(mx, fabs(dl[k]));
      nz = mx > eps_zero * refmax;
    }
  }
  // maximum over the wavefront (flags: any)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nz = max(nz, __shfl_xor(nz, o, 64));
  if (inlat && threadIdx.x == 0) blk[v / kSeg] = nz;
}

// Inclusive sum over the 1024 threads of the workgroup; `ws` holds 16 partial
// sums in LDS.  Returns the thread's exclusive prefix.
__device__ inline int32_t block_excl_scan(int32_t f, int32_t* ws) {
  int32_t x = f;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) ws[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < 16; ++w) {
      const int32_t t = ws[w];
      ws[w] = s;
      s += t;
    }
  }
  __syncthreads();
  return ws[threadIdx.x >> 6] + x - f;
}

// Exclusive scan of the block flags (widths) into compact ids (-1 for zero
// blocks) and, with boff, of the widths into byte offsets, in three passes:
// each workgroup sums its chunk of kScanChunk blocks, one workgroup scans the
// chunk sums, and each workgroup rescans its chunk from its base.  Integer
// sums, so the result does not depend on the split.
constexpr int kScanPer = 8;
constexpr int kScanChunk = 1024 * kScanPer;

__global__ __launch_bounds__(1024) void k_scan_sum(const int32_t* __restrict__ blk, int64_t nblk,
                                                   int32_t* __restrict__ csum) {
  __shared__ int32_t wsum[16], wsw[16];
  const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
  int32_t f = 0, w = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    const int64_t idx = c0 + (int64_t)q * 1024 + threadIdx.x;
    const int32_t v = idx < nblk ? blk[idx] : 0;
    f += v > 0 ? 1 : 0;
    w += v;
  }
  const int32_t ef = block_excl_scan(f, wsum);
  const int32_t ew = block_excl_scan(w, wsw);
  if (threadIdx.x == 1023) {
    csum[2 * blockIdx.x] = ef + f;
    csum[2 * blockIdx.x + 1] = ew + w;
  }
}

__global__ __launch_bounds__(1024) void k_scan_chunks(int32_t* __restrict__ csum, int64_t nchunk,
                                                      int32_t* __restrict__ total) {
  __shared__ int32_t wsum[16], wsw[16];
  __shared__ int32_t base_s, basew_s;
  if (threadIdx.x == 0) base_s = basew_s = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nchunk; c0 += 1024) {
    const int64_t idx = c0 + threadIdx.x;
    const int32_t f = idx < nchunk ? csum[2 * idx] : 0;
    const int32_t w = idx < nchunk ? csum[2 * idx + 1] : 0;
    const int32_t ef = base_s + block_excl_scan(f, wsum);
    const int32_t ew = basew_s + block_excl_scan(w, wsw);
    if (idx < nchunk) {
      csum[2 * idx] = ef;
      csum[2 * idx + 1] = ew;
    }
    __syncthreads();
    if (threadIdx.x == 1023) {
      base_s = ef + f;
      basew_s = ew + w;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = base_s;
}

__global__ __launch_bounds__(1024) void k_scan_write(int32_t* __restrict__ blk, int64_t nblk,
                                                     const int32_t* __restrict__ csum,
                                                     int64_t* __restrict__ boff, int64_t unit) {
  __shared__ int32_t wsum[16], wsw[16];
  __shared__ int32_t base_s, basew_s;
  if (threadIdx.x == 0) {
    base_s = csum[2 * blockIdx.x];
    basew_s = csum[2 * blockIdx.x + 1];
  }
  __syncthreads();
  const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
  for (int q = 0; q < kScanPer; ++q) {
    const int64_t idx = c0 + (int64_t)q * 1024 + threadIdx.x;
    const int32_t w = (idx < nblk) ? blk[idx] : 0;
    const int32_t f = w > 0 ? 1 : 0;
    const int32_t excl = base_s + block_excl_scan(f, wsum);
    const int32_t exw = basew_s + block_excl_scan(w, wsw);
    if (idx < nblk) blk[idx] = f ? excl : -1;
    if (boff && f) boff[excl] = (int64_t)exw * unit | ((int64_t)w << 56);
    __syncthreads();
    if (threadIdx.x == 1023) {
      base_s = excl + f;
      basew_s = exw + w;
    }
    __syncthreads();
  }
}

__device__ inline uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <int D, bool IS_P, int FMT>
__global__ __launch_bounds__(256) void k_delta_write(Lat L, Lat Lc, const double* __restrict__ full,
                                                     const double* __restrict__ eps,
                                                     const int32_t* __restrict__ blk,
                                                     void* __restrict__ payload,
                                                     int8_t* __restrict__ scale,
                                                     const int64_t* __restrict__ boff, double eps_mf,
                                                     const int32_t* __restrict__ tiles,
                                                     const int8_t* __restrict__ vt) {
  constexpr int NE = IS_P ? Dim<D>::NC : Dim<D>::NS;
  const int32_t* tl = tiles ? tiles + 3 * (int64_t)blockIdx.x : nullptr;
  const int i = (tl ? tl[0] : (int)blockIdx.x) * TX + threadIdx.x;
  const int j = (tl ? tl[1] : (int)blockIdx.y) * TY + threadIdx.y;
  const int kz = (D == 3) ? (tl ? tl[2] : (int)blockIdx.z) : 0;
  if (j > L.n || (D == 3 && kz > L.n)) return;
  const int64_t v = i + (int64_t)j * L.pitch + (int64_t)kz * L.plane;
  const int32_t cb = blk[v / kSeg];
  if (cb < 0) return;
  double dl[27], refmax;
  load_delta<D, IS_P>(L, Lc, full, eps, vt, i, j, kz, v, dl, refmax);
  const int lane = (int)(v % kSeg);
  const int64_t base = (int64_t)cb * NE * kSeg + lane;
  if (FMT == BPA) {
    // every entry at the vertex's own width, stored in the block's width
    const int64_t ow = boff[cb];
    const int W = (int)(ow >> 56);
    uint8_t* p = (uint8_t*)payload + (ow & ((int64_t(1) << 56) - 1)) + lane;
    const int wv = bpa_width(dl, NE, eps_mf);
    for (int k = 0; k < NE; ++k) {
      int e;
      long long m;
      bpa_code(dl[k], wv, e, m);
      p[k * kSeg] = (uint8_t)(int8_t)e;
      for (int jb = 0; jb < W - 1; ++jb)
        p[(int64_t)(NE * (1 + jb) + k) * kSeg] = (uint8_t)(((unsigned long long)m >> (8 * jb)) & 0xFFu);
    }
  } else if (FMT == F16) {
    double mx = 0.0;
    for (int k = 0; k < NE; ++k) mx = fmax(mx, fabs(dl[k]));
    int E = 0;
    const double m = frexp(mx, &E);  // mx = m 2^E, m in [0.5, 1)
    int e = (mx == 0.0) ? 0 : (m == 0.5 ? E - 16 : E - 15);
    e = max(-128, min(127, e));
    scale[(int64_t)cb * kSeg + lane] = (int8_t)e;
    for (int k = 0; k < NE; ++k)
      ((_Float16*)payload)[base + (int64_t)k * kSeg] = (_Float16)(float)ldexp(dl[k], -e);
  } else {
    for (int k = 0; k < NE; ++k) {
      const int64_t q = base + (int64_t)k * kSeg;
      if (FMT == F64) ((double*)payload)[q] = dl[k];
      else if (FMT == F32) ((float*)payload)[q] = (float)dl[k];
      else ((uint16_t*)payload)[q] = bf16_rne((float)dl[k]);
    }
  }
}

}  // namespace

void launch_coarsen_eps(const Lat& Lf, const Lat& Lc, const double* epsf, double* epsc, hipStream_t s) {
  const dim3 g = tile_grid(Lc), bl(TX, TY, 1);
  if (Lf.d == 2) hipLaunchKernelGGL(k_coarsen_eps<2>, g, bl, 0, s, Lf, Lc, epsf, epsc);
  else hipLaunchKernelGGL(k_coarsen_eps<3>, g, bl, 0, s, Lf, Lc, epsf, epsc);
  QMG_HIP(hipGetLastError());
}

void launch_materialise(const Lat& L, const double* eps, const Store& A, double* out, hipStream_t s) {
  const dim3 g = tile_grid(L), bl(TX, TY, 1);
#define QMG_MAT(DV, SRCV, FMTV) hipLaunchKernelGGL((k_materialise<DV, SRCV, FMTV>), g, bl, 0, s, L, eps, A, out)
#define QMG_MAT_D(DV)                                   \
  do {                                                  \
    if (A.src == SRC_GEOM) QMG_MAT(DV, SRC_GEOM, F64);  \
    else if (A.src == SRC_PLAIN) QMG_MAT(DV, SRC_PLAIN, F64); \
    else if (A.fmt == F64) QMG_MAT(DV, SRC_HIER, F64);  \
    else if (A.fmt == F32) QMG_MAT(DV, SRC_HIER, F32);  \
    else if (A.fmt == F16) QMG_MAT(DV, SRC_HIER, F16);  \
    else if (A.fmt == BPA) QMG_MAT(DV, SRC_HIER, BPA);  \
    else QMG_MAT(DV, SRC_HIER, BF16);                   \
  } while (0)
  if (L.d == 2) QMG_MAT_D(2);
  else QMG_MAT_D(3);
#undef QMG_MAT_D
#undef QMG_MAT
  QMG_HIP(hipGetLastError());
}

void launch_materialise_P(const Lat& Lf, const Lat& Lc, const Store& P, double* out, hipStream_t s) {
  const dim3 g = tile_grid(Lf), bl(TX, TY, 1);
#define QMG_MP(DV, SRCV, FMTV) hipLaunchKernelGGL((k_materialise_P<DV, SRCV, FMTV>), g, bl, 0, s, Lf, Lc, P, out)
#define QMG_MP_D(DV)                                    \
  do {                                                  \
    if (P.src == SRC_GEOM) QMG_MP(DV, SRC_GEOM, F64);   \
    else if (P.src == SRC_PLAIN) QMG_MP(DV, SRC_PLAIN, F64); \
    else if (P.fmt == F64) QMG_MP(DV, SRC_HIER, F64);   \
    else if (P.fmt == F32) QMG_MP(DV, SRC_HIER, F32);   \
    else if (P.fmt == F16) QMG_MP(DV, SRC_HIER, F16);   \
    else if (P.fmt == BPA) QMG_MP(DV, SRC_HIER, BPA);   \
    else QMG_MP(DV, SRC_HIER, BF16);                    \
  } while (0)
  if (Lf.d == 2) QMG_MP_D(2);
  else QMG_MP_D(3);
#undef QMG_MP_D
#undef QMG_MP
  QMG_HIP(hipGetLastError());
}

bool launch_boxmg(const Lat& Lf, const Lat& Lc, const double* Afine, const double* epsf, double* Pw,
                  hipStream_t s, const int8_t* vt_fine, const int8_t* cref_coarse, const int32_t* cells,
                  int64_t n_cells, void* scratch, size_t scratch_bytes, int32_t* dirty) {
  const int m = Lc.n - 1;
  if (m <= 0) return false;
  const int64_t nv = (Lf.d == 3) ? (int64_t)m * m * m : (int64_t)m * m;
  const int64_t nt = (cells ? n_cells : nv) * (Lf.d == 3 ? 8 : 4);
  if (nt == 0) return false;
  bool marked = false;
  if (Lf.d == 2) {
    BoxFetch<2> F{Afine, epsf, Lf, vt_fine, vt_fine != nullptr};
    hipLaunchKernelGGL((k_boxmg<2, 1>), dim3(blocks_for(nt, 64)), dim3(64), 0, s, Lf, Lc, F, Pw, cref_coarse, cells,
                       n_cells, nullptr, 0, nullptr);
  } else {
    // 8 coarse cells (all their corners) per workgroup
    const int64_t nc = cells ? n_cells : (int64_t)Lc.n * Lc.n * Lc.n;
    const dim3 g(blocks_for(nc, 8));
    BoxFetch<3> F{Afine, epsf, Lf, vt_fine, vt_fine != nullptr};
    const bool split = Afine == nullptr && cells != nullptr && scratch != nullptr &&
                       scratch_bytes >= (size_t)(n_cells + 16) * sizeof(int32_t);
    if (split) {
      // count, then the list of the cells whose patches need the solve
      int32_t* dcount = (int32_t*)scratch;
      int32_t* dlist = dcount + 16;
      hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, dcount, (int64_t)1, 0);
      hipLaunchKernelGGL(k_boxmg_uniform3, dim3(blocks_for(n_cells, kBoxCells)), dim3(512), 0, s, Lf, Lc,
                         epsf, Pw, cref_coarse, cells, n_cells, dlist, dcount);
      hipLaunchKernelGGL((k_boxmg<3, 2>), g, dim3(64), 0, s, Lf, Lc, F, Pw, cref_coarse, (const int32_t*)dlist,
                         n_cells, (const int32_t*)dcount, 2, dirty);
      marked = dirty != nullptr;
    } else if (Afine == nullptr) {
      hipLaunchKernelGGL((k_boxmg<3, 2>), g, dim3(64), 0, s, Lf, Lc, F, Pw, cref_coarse, cells, n_cells, nullptr,
                         0, nullptr);
    } else {
      hipLaunchKernelGGL((k_boxmg<3, 1>), g, dim3(64), 0, s, Lf, Lc, F, Pw, cref_coarse, cells, n_cells, nullptr,
                         0, nullptr);
    }
  }
  QMG_HIP(hipGetLastError());
  return marked;
}

void launch_rap(const Lat& Lf, const Lat& Lc, const double* Afine, const double* epsf,
                const double* Pw, double* Ac, hipStream_t s, const int8_t* vt_fine, const int8_t* vt_coarse,
                const int32_t* verts, int64_t n_verts, int rmode) {
  const int m = Lc.n - 1;
  if (m <= 0) return;
  const int64_t nV = verts ? n_verts : (Lf.d == 3 ? (int64_t)m * m * m : (int64_t)m * m);
  if (nV == 0) return;
  if (Lf.d == 2) {
    using S = RapShape<2>;
    BoxFetch<2> A{Afine, epsf, Lf, vt_fine};
    PFetch<2> P{Pw, Lf, Lc};
    hipLaunchKernelGGL(k_rap<2>, dim3(blocks_for(nV, S::VPB)), dim3(S::NT), 0, s, Lf, Lc, A, P, Ac, vt_coarse,
                       verts, n_verts, rmode);
  } else if (Afine == nullptr && rmode == 0) {
    // rediscretised fine operator: the cell-by-cell product
    const int64_t gx = std::min<int64_t>(nV, 65536);
    hipLaunchKernelGGL(k_rap_fine3, dim3((unsigned)gx, (unsigned)((nV + gx - 1) / gx)), dim3(kRfNT), 0, s, Lf, Lc,
                       epsf, Pw, vt_fine, Ac, vt_coarse, verts, n_verts);
  } else {
    using S = RapShape<3>;
    BoxFetch<3> A{Afine, epsf, Lf, vt_fine};
    PFetch<3> P{Pw, Lf, Lc};
    hipLaunchKernelGGL(k_rap<3>, dim3(blocks_for(nV, S::VPB)), dim3(S::NT), 0, s, Lf, Lc, A, P, Ac, vt_coarse,
                       verts, n_verts, rmode);
  }
  QMG_HIP(hipGetLastError());
}

bool launch_rap_cells(const Lat& Lf, const Lat& Lc, const double* epsf, const double* Pw, double* Ac,
                      hipStream_t s, const int8_t* vt_fine, const int8_t* vt_coarse, const int32_t* verts,
                      int64_t n_verts, const int32_t* cells, int64_t n_cells, void* scratch, size_t scratch_bytes) {
  if (Lf.d != 3 || cells == nullptr || verts == nullptr) return false;
  const int64_t ncc = (int64_t)Lc.n * Lc.n * Lc.n;
  const size_t need = (size_t)n_cells * 64 * sizeof(double) + (size_t)ncc * sizeof(int32_t);
  if (need > scratch_bytes || ncc > INT32_MAX) return false;
  double* AC = (double*)scratch;
  int32_t* cidx = (int32_t*)(AC + n_cells * 64);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(ncc, 256)), dim3(256), 0, s, cidx, ncc, -1);
  if (n_cells > 0) {
    hipLaunchKernelGGL(k_cell_index, dim3(blocks_for(n_cells, 256)), dim3(256), 0, s, cells, n_cells, cidx);
    const int64_t gx = std::min<int64_t>(n_cells, 65536);
    hipLaunchKernelGGL(k_rap_cells3, dim3((unsigned)gx, (unsigned)((n_cells + gx - 1) / gx)), dim3(64), 0, s, Lf,
                       Lc, epsf, Pw, vt_fine, cells, n_cells, AC);
  }
  if (n_verts > 0)
    hipLaunchKernelGGL(k_rap_assemble3, dim3(blocks_for(n_verts, 256)), dim3(256), 0, s, Lc, AC, cidx, verts,
                       n_verts, vt_coarse, Ac);
  QMG_HIP(hipGetLastError());
  return true;
}

void launch_conv_add(const Lat& L, const double* vel, double* A, hipStream_t s) {
  const dim3 g = tile_grid(L), bl(TX, TY, 1);
  if (L.d == 2) hipLaunchKernelGGL(k_conv_add<2>, g, bl, 0, s, L, vel, A);
  else hipLaunchKernelGGL(k_conv_add<3>, g, bl, 0, s, L, vel, A);
  QMG_HIP(hipGetLastError());
}

void launch_check_rows(const Lat& Lc, const double* Ac, int* bad, hipStream_t s) {
  const dim3 g = tile_grid(Lc), bl(TX, TY, 1);
  if (Lc.d == 2) hipLaunchKernelGGL(k_check_rows<2>, g, bl, 0, s, Lc, Ac, bad);
  else hipLaunchKernelGGL(k_check_rows<3>, g, bl, 0, s, Lc, Ac, bad);
  QMG_HIP(hipGetLastError());
}

void launch_delta_flags(const Lat& L, const Lat& Lc, bool is_P, const double* full, const double* eps,
                        int32_t* blk, hipStream_t s, double eps_mf, const int32_t* tiles, int ntiles,
                        double eps_zero, const int8_t* vt, bool marked) {
  if (!(eps_zero > 0.0)) eps_zero = kEpsZero;
  const dim3 g = tiles ? dim3((unsigned)ntiles) : tile_grid(L), bl(TX, TY, 1);
  // blocks of unlisted tiles: zero (with marked blocks they are zero already)
  if (tiles && !marked) launch_zero<int32_t>(blk, L.nslot / kSeg, s);
  if (tiles && ntiles == 0) return;
  if (L.d == 2) {
    if (is_P) hipLaunchKernelGGL((k_delta_flags<2, true>), g, bl, 0, s, L, Lc, full, eps, blk, eps_mf, tiles, eps_zero, vt, (int)marked);
    else hipLaunchKernelGGL((k_delta_flags<2, false>), g, bl, 0, s, L, Lc, full, eps, blk, eps_mf, tiles, eps_zero, vt, (int)marked);
  } else {
    if (is_P) hipLaunchKernelGGL((k_delta_flags<3, true>), g, bl, 0, s, L, Lc, full, eps, blk, eps_mf, tiles, eps_zero, vt, (int)marked);
    else hipLaunchKernelGGL((k_delta_flags<3, false>), g, bl, 0, s, L, Lc, full, eps, blk, eps_mf, tiles, eps_zero, vt, (int)marked);
  }
  QMG_HIP(hipGetLastError());
}

int64_t scan_scratch_ints(int64_t nblk) { return 2 * ((nblk + kScanChunk - 1) / kScanChunk) + 2; }

void launch_scan_blocks(int32_t* blk, int64_t nblk, int32_t* total, hipStream_t s, int64_t* boff,
                        int64_t unit, int32_t* csum) {
  const int64_t nchunk = (nblk + kScanChunk - 1) / kScanChunk;
  if (nchunk > 0) hipLaunchKernelGGL(k_scan_sum, dim3((unsigned)nchunk), dim3(1024), 0, s, blk, nblk, csum);
  hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(1024), 0, s, csum, nchunk, total);
  if (nchunk > 0)
    hipLaunchKernelGGL(k_scan_write, dim3((unsigned)nchunk), dim3(1024), 0, s, blk, nblk, csum, boff, unit);
  QMG_HIP(hipGetLastError());
}

void launch_delta_write(const Lat& L, const Lat& Lc, bool is_P, int fmt, const double* full,
                        const double* eps, const int32_t* blk, void* payload, int8_t* scale,
                        hipStream_t s, const int64_t* boff, double eps_mf, const int32_t* tiles, int ntiles,
                        const int8_t* vt) {
  const dim3 g = tiles ? dim3((unsigned)ntiles) : tile_grid(L), bl(TX, TY, 1);
  if (fmt == BPA && (!boff || !(eps_mf > 0.0))) throw std::runtime_error("BPA store without offsets or eps_mf");
  if (tiles && ntiles == 0) return;
#define QMG_DW(DV, PV, FV) \
  hipLaunchKernelGGL((k_delta_write<DV, PV, FV>), g, bl, 0, s, L, Lc, full, eps, blk, payload, scale, boff, eps_mf, \
                     tiles, vt)
#define QMG_DW_F(DV, PV)                  \
  do {                                    \
    if (fmt == F64) QMG_DW(DV, PV, F64);  \
    else if (fmt == F32) QMG_DW(DV, PV, F32); \
    else if (fmt == F16) QMG_DW(DV, PV, F16); \
    else if (fmt == BPA) QMG_DW(DV, PV, BPA); \
    else QMG_DW(DV, PV, BF16);            \
  } while (0)
  if (L.d == 2) {
    if (is_P) QMG_DW_F(2, true);
    else QMG_DW_F(2, false);
  } else {
    if (is_P) QMG_DW_F(3, true);
    else QMG_DW_F(3, false);
  }
#undef QMG_DW_F
#undef QMG_DW
  QMG_HIP(hipGetLastError());
}

}  // namespace qmg
