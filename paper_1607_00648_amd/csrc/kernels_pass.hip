// Fused smoothing passes of one regular 2D level (Alg. 1 per level): an
// optional prolongation-add u += P e, one or two damped Jacobi sweeps and an
// optional residual r = b - A u (with norm partials), in one launch.
//
// A workgroup of 1024 threads owns a 64 x 8 (or 56 x 10) output tile, one
// region point per thread, so that every thread issues its loads at once (the
// passes are bound by memory latency, not bandwidth).  The iterate is staged in LDS on the
// tile plus a halo of K vertices, K = number of neighbour-dependent stages
// (sweeps, residual); stage s produces its values on the tile plus a halo of
// K - s, so the next stage finds every neighbour in LDS.  Each thread keeps the
// stencil rows of its region points in registers, decoded once per pass.  The
// values are computed with the same expressions, in the same order, as the
// single-step kernels; halo points are computed redundantly by neighbouring
// tiles.  Algorithmic traffic per vertex: eps, u, b read once, u written once,
// r written once when asked (plus e and P for the prolongation).
#include <hip/hip_ext.h>

#include "level_ops.hpp"

namespace qmg {

namespace {

constexpr int NT = 1024;
constexpr int KMAX = 3;
constexpr int NS2 = 9;
// Output tiles: 64 x 8, or 56 x 10 (region 62 x 16 = 992 points, still one
// per thread).  Two 1024-thread workgroups are resident per CU, 512 on the
// chip; a level takes the tile with fewer such rounds of workgroups (the
// 729^2-cell level: 1104 tiles of 64 x 8 need three rounds, the last one
// nearly empty; 1022 tiles of 56 x 10 need two).
constexpr int kResidentPasses = 512;
template <int PXT, int PYT>
struct PassTile {
  static constexpr int PX = PXT, PY = PYT;
  static constexpr int WMAX = PX + 2 * KMAX, HMAX = PY + 2 * KMAX;
  static constexpr int PTS = (WMAX * HMAX + NT - 1) / NT;
  static dim3 grid(const Lat& L) {
    return dim3((unsigned)((L.n + 1 + PX - 1) / PX), (unsigned)((L.n + 1 + PY - 1) / PY), 1);
  }
  static int count(const Lat& L) {
    const dim3 g = grid(L);
    return (int)(g.x * g.y);
  }
};
using TileA = PassTile<64, 8>;
using TileB = PassTile<56, 10>;
static_assert(TileA::PTS == 1 && TileB::PTS == 1, "one region point per thread");

bool use_tile_b(const Lat& L) {
  const int ra = (TileA::count(L) + kResidentPasses - 1) / kResidentPasses;
  const int rb = (TileB::count(L) + kResidentPasses - 1) / kResidentPasses;
  return rb < ra;
}

template <typename T, int FMT>
__device__ inline T prolong_any(const PassArgs<T>& p, int i, int j, int64_t vf) {
  switch (p.P.src) {
    case SRC_HIER: return prolong_at<2, T, SRC_HIER, FMT>(p.L, p.Lc, p.ec, p.P, i, j, 0, vf);
    case SRC_PLAIN: return prolong_at<2, T, SRC_PLAIN, F64>(p.L, p.Lc, p.ec, p.P, i, j, 0, vf);
    default: return prolong_at<2, T, SRC_GEOM, F64>(p.L, p.Lc, p.ec, p.P, i, j, 0, vf);
  }
}

template <typename T, int SRC, int FMT, class TL>
__global__ __launch_bounds__(NT) void k_pass2d(PassArgs<T> p) {
  constexpr int PX = TL::PX, PY = TL::PY, WMAX = TL::WMAX, HMAX = TL::HMAX, PTS = TL::PTS;
  __shared__ T buf[2][WMAX * HMAX];
  __shared__ double red[NT / 64];
  const int K = p.nsw + (p.res ? 1 : 0);
  const int W = PX + 2 * K, H = PY + 2 * K;
  const Tile tl = xcd_tile();
  const int x0 = tl.x * PX - K, y0 = tl.y * PY - K;
  const int n = p.L.n;
  const int tid = threadIdx.x;

  T a[PTS][NS2];
  T bb[PTS];
  int64_t vv[PTS];
  bool inter[PTS];
  int rxs[PTS], rys[PTS];  // region coordinates (divisions done once)
#pragma unroll
  for (int m = 0; m < PTS; ++m) {
    const int q = tid + NT * m;
    rys[m] = q / W;
    rxs[m] = q - rys[m] * W;
    const int i = x0 + rxs[m], j = y0 + rys[m];
    const bool valid = q < W * H;
    const bool inside = valid && i >= 0 && i <= n && j >= 0 && j <= n;
    inter[m] = inside && i >= 1 && i < n && j >= 1 && j < n;
    vv[m] = inside ? i + (int64_t)j * p.L.pitch : 0;
    T u0 = (T)0;
    if (inside && !p.zero_first) u0 = p.u[vv[m]];
    if (inter[m] && p.pro) u0 += prolong_any<T, FMT>(p, i, j, vv[m]);
    if (valid) buf[0][q] = u0;
    bb[m] = (T)0;
    if (inter[m]) {
      op_row<2, T, SRC, FMT>(p.eps, p.A, p.L, vv[m], a[m]);
      bb[m] = p.b[vv[m]];
    }
  }
  __syncthreads();

  int cur = 0;
  for (int s = 1; s <= p.nsw; ++s) {
#pragma unroll
    for (int m = 0; m < PTS; ++m) {
      const int q = tid + NT * m;
      const int rx = rxs[m], ry = rys[m];
      if (q >= W * H || rx < s || rx >= W - s || ry < s || ry >= H - s) continue;
      T nu = buf[cur][q];
      if (inter[m]) {
        if (s == 1 && p.zero_first) {
          nu = p.omega * bb[m] / a[m][NS2 / 2];
        } else {
          T au = (T)0;
#pragma unroll
          for (int k = 0; k < NS2; ++k) au += a[m][k] * buf[cur][q + off_x(k) + off_y(k) * W];
          nu = buf[cur][q] + p.omega * (bb[m] - au) / a[m][NS2 / 2];
        }
      }
      buf[cur ^ 1][q] = nu;
    }
    __syncthreads();
    cur ^= 1;
  }

  double sq = 0.0;
#pragma unroll
  for (int m = 0; m < PTS; ++m) {
    const int q = tid + NT * m;
    const int rx = rxs[m], ry = rys[m];
    if (q >= W * H || rx < K || rx >= W - K || ry < K || ry >= H - K || !inter[m]) continue;
    p.out[vv[m]] = buf[cur][q];
    if (p.res) {
      T au = (T)0;
#pragma unroll
      for (int k = 0; k < NS2; ++k) au += a[m][k] * buf[cur][q + off_x(k) + off_y(k) * W];
      const T res = bb[m] - au;
      p.r[vv[m]] = res;
      sq += (double)res * (double)res;
    }
  }
  if (p.partial != nullptr) {
#pragma unroll
    for (int mm = 32; mm >= 1; mm >>= 1) sq += __shfl_xor(sq, mm, 64);
    if ((tid & 63) == 0) red[tid >> 6] = sq;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) t += red[w];
      p.partial[tl.t] = t;
    }
  }
}

}  // namespace

template <typename T>
void launch_pass2d(const PassArgs<T>& p, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop) {
  if (p.L.d != 2) throw ApiError(QMG_EINVAL, "fused passes are 2D only");
  if (p.nsw < 0 || p.nsw > 2 || p.nsw + (p.res ? 1 : 0) > KMAX || p.nsw + (p.res ? 1 : 0) < 1)
    throw ApiError(QMG_EINVAL, "fused pass: 1 or 2 sweeps plus an optional residual");
  if (p.pro && p.zero_first) throw ApiError(QMG_EINVAL, "fused pass: prolongation into a zero iterate");
  const bool tb = use_tile_b(p.L);
  const dim3 g = tb ? TileB::grid(p.L) : TileA::grid(p.L), bl(NT, 1, 1);
#define QMG_PASS_T(SRCV, FMTV, TLV)                                                               \
  do {                                                                                            \
    if (ev_start != nullptr)                                                                      \
      hipExtLaunchKernelGGL((k_pass2d<T, SRCV, FMTV, TLV>), g, bl, 0, s, ev_start, ev_stop, 0, p); \
    else                                                                                          \
      hipLaunchKernelGGL((k_pass2d<T, SRCV, FMTV, TLV>), g, bl, 0, s, p);                         \
  } while (0)
#define QMG_PASS(SRCV, FMTV)                 \
  do {                                       \
    if (tb) QMG_PASS_T(SRCV, FMTV, TileB);   \
    else QMG_PASS_T(SRCV, FMTV, TileA);      \
  } while (0)
  if (p.A.src == SRC_GEOM) {
    switch (p.P.fmt) {  // the prolongation store shares the level format
      case F32: QMG_PASS(SRC_GEOM, F32); break;
      case F16: QMG_PASS(SRC_GEOM, F16); break;
      case BF16: QMG_PASS(SRC_GEOM, BF16); break;
      case BPA: QMG_PASS(SRC_GEOM, BPA); break;
      default: QMG_PASS(SRC_GEOM, F64); break;
    }
  } else if (p.A.src == SRC_PLAIN) {
    QMG_PASS(SRC_PLAIN, F64);
  } else {
    switch (p.A.fmt) {
      case F32: QMG_PASS(SRC_HIER, F32); break;
      case F16: QMG_PASS(SRC_HIER, F16); break;
      case BF16: QMG_PASS(SRC_HIER, BF16); break;
      case BPA: QMG_PASS(SRC_HIER, BPA); break;
      default: QMG_PASS(SRC_HIER, F64); break;
    }
  }
#undef QMG_PASS
#undef QMG_PASS_T
  QMG_HIP(hipGetLastError());
}

int pass2d_partials(const Lat& L) { return use_tile_b(L) ? TileB::count(L) : TileA::count(L); }

template void launch_pass2d<double>(const PassArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_pass2d<float>(const PassArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace qmg
