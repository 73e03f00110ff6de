// Coarse part of the V-cycle in one workgroup, with the levels held in LDS.
//
// The coarse levels of a tripartitioned hierarchy are tiny (2D: 676, 64 and 4
// unknowns on levels 3, 2, 1), so seven launches per level cost far more than
// the arithmetic, and a workgroup walking them in global memory is bound by L2
// latency.  This kernel loads, once per cycle, the stencil rows (rebuilt from
// the coefficients and the delta store) and the prolongation weights of levels
// lc..lf into LDS, keeps every iterate of those levels in LDS, and runs the
// whole V-cycle from level lf (which has just received its restricted
// right-hand side and starts from zero) down to the coarsest level and back up:
// every phase is a strided loop over a level's interior vertices followed by a
// workgroup barrier.  Only the final iterate of level lf goes back to global
// memory.  The operators do not change between cycles, so the rows and weights
// are decoded once per build into an image of the LDS contents in global
// memory; each launch copies that image in with 16-byte loads.
#include "level_ops.hpp"
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <mutex>

namespace qmg {

namespace {

template <int D>
constexpr int block_of() { return D == 2 ? 1024 : 256; }

// 32-bit index arithmetic (the fused levels have a few thousand vertices).
// Division by m is a multiply-high with mag = floor((2^32 - 1) / m) + 1, exact
// for m >= 2 and indices below 2^22 (error below 2^-10 of one unit).
__device__ inline int divm(int x, unsigned mag) { return (int)__umulhi((unsigned)x, mag); }
__device__ inline void vertex_of(int idx, int m, unsigned mag, int d, int& i, int& j, int& k) {
  const int q = divm(idx, mag);
  i = idx - q * m + 1;
  if (d == 3) {
    const int r = divm(q, mag);
    j = q - r * m + 1;
    k = r + 1;
  } else {
    j = q + 1;
    k = 0;
  }
}

// compact LDS index of vertex (i,j,k) of a level with w = n+1 vertices per axis
__device__ inline int cidx(int w, int i, int j, int k) { return i + w * (j + w * k); }

template <int D, typename T, int ASRC, int PSRC, int FMT>
struct Fused {
  static constexpr int NS = Dim<D>::NS, NC = Dim<D>::NC, BS = block_of<D>();
  const FusedArgs<T>& a;
  char* smem;
  const unsigned* mag;  // division magic of m(s) per level (kernel arguments)
  __device__ Fused(const FusedArgs<T>& args, char* s) : a(args), smem(s), mag(args.mag) {}

  __device__ int w(int s) const { return a.L[s].n + 1; }
  __device__ int m(int s) const { return a.L[s].n - 1; }
  __device__ int nint(int s) const { return D == 3 ? m(s) * m(s) * m(s) : m(s) * m(s); }
  __device__ T* vec(int s, int which) const {  // 0 u, 1 t, 2 b, 3 r
    return (T*)(smem + a.lds_vec[s]) + which * a.lds_nslot[s];
  }
  __device__ T* rows(int s) const { return (T*)(smem + a.lds_rows[s]); }
  __device__ T* pw(int s) const { return (T*)(smem + a.lds_pw[s]); }

  // Levels with at most 64 interior vertices are worked by wave 0 alone.
  __device__ bool small(int s) const { return nint(s) <= 64; }
  // Barrier after a phase: the whole workgroup, or, when the phase's writers
  // and the next phase's readers all lie in wave 0 (wave0), an ordering of
  // that wave's LDS accesses only.  The condition is uniform, so every wave
  // passes the same sequence of workgroup barriers.
  __device__ void sync(bool wave0) const {
    if (wave0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  }

  __device__ T row_dot_lds(const T* row, const T* u, int ws, int c) const {
    T acc = (T)0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int o = off_x(k) + ws * (off_y(k) + (D == 3 ? ws * off_z(k) : 0));
      acc += row[k] * u[c + o];
    }
    return acc;
  }

  // zero iterates, stencil rows and parent weights at the layout's offsets from
  // `smem` (LDS, or the global image)
  __device__ void build_static() const {
    for (int s = 0; s <= a.lf - a.lc; ++s) {
      const Lat& L = a.L[s];
      const int ws = w(s), ms = m(s);
      const int nsl = a.lds_nslot[s];
      for (int q = threadIdx.x; q < 4 * nsl; q += BS) vec(s, 0)[q] = (T)0;
      for (int idx = threadIdx.x; idx < nint(s); idx += BS) {
        int i, j, k;
        vertex_of(idx, ms, mag[s], D, i, j, k);
        const int64_t v = i + (int64_t)j * L.pitch + (int64_t)k * L.plane;
        T r[NS];
        op_row<D, T, ASRC, FMT>(a.eps[s], a.A[s], L, v, r);
        T* dst = rows(s) + (int64_t)idx * NS;
#pragma unroll
        for (int e = 0; e < NS; ++e) dst[e] = r[e];
        if (s >= 1 && PSRC != SRC_GEOM && a.pw_lds) {
          const int rx = i % 3, ry = j % 3, rz = k % 3;
          T* pd = pw(s) + (int64_t)cidx(ws, i, j, k) * NC;
#pragma unroll
          for (int c = 0; c < NC; ++c) pd[c] = (T)pweight<D, PSRC, FMT>(a.P[s], L, v, rx, ry, rz, c);
        }
      }
    }
  }

  __device__ void load() const {
    if (a.img != nullptr) {
      const uint4* src = (const uint4*)a.img;
      uint4* dst = (uint4*)smem;
      for (int q = threadIdx.x; q < a.lds_bytes / 16; q += BS) dst[q] = src[q];
    } else {
      build_static();
    }
    __syncthreads();
    // restricted right-hand side of the top level
    const int top = a.lf - a.lc;
    const Lat& L = a.L[top];
    for (int idx = threadIdx.x; idx < nint(top); idx += BS) {
      int i, j, k;
      vertex_of(idx, m(top), mag[top], D, i, j, k);
      vec(top, 2)[cidx(w(top), i, j, k)] = a.b[top][i + (int64_t)j * L.pitch + (int64_t)k * L.plane];
    }
    __syncthreads();
  }

  // one Jacobi sweep u -> out on level s (from zero: u not read)
  __device__ void sweep(int s, const T* u, T* out, bool from_zero) const {
    const int ws = w(s), ms = m(s);
    const T* bv = vec(s, 2);
    for (int idx = threadIdx.x; idx < nint(s); idx += BS) {
      int i, j, k;
      vertex_of(idx, ms, mag[s], D, i, j, k);
      const int c = cidx(ws, i, j, k);
      const T* row = rows(s) + (int64_t)idx * NS;
      const T dg = row[NS / 2];
      out[c] = from_zero ? a.omega * bv[c] / dg : u[c] + a.omega * (bv[c] - row_dot_lds(row, u, ws, c)) / dg;
    }
    sync(small(s));
  }

  // One block Jacobi step on level s (Sect. "Spacetree block smoothers"), as
  // the per-level kernels take it: bj_sweeps Gauss-Seidel sweeps over every
  // patch's iota-vertices in u (in place; patch = 3^d vertices of one coarser
  // cell, iota = no coordinate divisible by 3), then the damped Jacobi update
  // of the other vertices into out, iota-vertices copied.
  __device__ void bj_step(int s, T* u, T* out, bool from_zero) const {
    constexpr int NP = NC;  // 2^d iota-vertices per patch
    const int ws = w(s), ms = m(s);
    const T* bv = vec(s, 2);
    if (from_zero) {
      for (int idx = threadIdx.x; idx < nint(s); idx += BS) {
        int i, j, k;
        vertex_of(idx, ms, mag[s], D, i, j, k);
        u[cidx(ws, i, j, k)] = (T)0;
      }
      sync(small(s));
    }
    const int np = a.L[s].n / 3;
    const int npatch = D == 3 ? np * np * np : np * np;
    for (int t = threadIdx.x; t < npatch; t += BS) {
      const int px = t % np, py = (t / np) % np, pz = D == 3 ? t / (np * np) : 0;
      T C[NP][NP], sp[NP], uu[NP];
      int cp[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int lx = p & 1, ly = (p >> 1) & 1, lz = (p >> 2) & 1;
        const int i = 3 * px + 1 + lx, j = 3 * py + 1 + ly, k = D == 3 ? 3 * pz + 1 + lz : 0;
        const int c = cidx(ws, i, j, k);
        cp[p] = c;
        const T* row = rows(s) + (int64_t)((i - 1) + ms * ((j - 1) + ms * (D == 3 ? k - 1 : 0))) * NS;
#pragma unroll
        for (int q = 0; q < NP; ++q) C[p][q] = (T)0;
        T rest = bv[c];
#pragma unroll
        for (int e = 0; e < NS; ++e) {
          const int qx = lx + off_x(e), qy = ly + off_y(e), qz = D == 3 ? lz + off_z(e) : 0;
          if (qx >= 0 && qx <= 1 && qy >= 0 && qy <= 1 && qz >= 0 && qz <= 1)
            C[p][qx | (qy << 1) | (qz << 2)] = row[e];
          else
            rest -= row[e] * u[c + off_x(e) + ws * (off_y(e) + (D == 3 ? ws * off_z(e) : 0))];
        }
        sp[p] = rest;
        uu[p] = u[c];
      }
      for (int sw = 0; sw < a.bj_sweeps; ++sw) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          T r = sp[p];
#pragma unroll
          for (int q = 0; q < NP; ++q) r -= C[p][q] * uu[q];
          uu[p] += r / C[p][p];
        }
      }
#pragma unroll
      for (int p = 0; p < NP; ++p) u[cp[p]] = uu[p];
    }
    sync(small(s));
    for (int idx = threadIdx.x; idx < nint(s); idx += BS) {
      int i, j, k;
      vertex_of(idx, ms, mag[s], D, i, j, k);
      const int c = cidx(ws, i, j, k);
      const T* row = rows(s) + (int64_t)idx * NS;
      const bool iota = i % 3 != 0 && j % 3 != 0 && (D == 2 || k % 3 != 0);
      out[c] = iota ? u[c] : u[c] + a.omega * (bv[c] - row_dot_lds(row, u, ws, c)) / row[NS / 2];
    }
    sync(small(s));
  }

  // returns the buffer index (0 = u, 1 = t) holding the result
  __device__ int smooth(int s, int cur, int mu, bool zero_init) const {
    for (int q = 0; q < mu; ++q) {
      if (a.bj_sweeps > 0) bj_step(s, vec(s, cur), vec(s, 1 - cur), zero_init && q == 0);
      else sweep(s, vec(s, cur), vec(s, 1 - cur), zero_init && q == 0);
      cur = 1 - cur;
    }
    return cur;
  }

  __device__ T weight(int s, int fc, int i, int j, int k, int kap) const {
    const int rx = i % 3, ry = j % 3, rz = k % 3;
    if (PSRC == SRC_GEOM)
      return (T)(dlin1(rx, kap & 1) * dlin1(ry, (kap >> 1) & 1) * (D == 3 ? dlin1(rz, (kap >> 2) & 1) : 1.0));
    if (!a.pw_lds) {
      const Lat& L = a.L[s];
      return (T)pweight<D, PSRC, FMT>(a.P[s], L, i + (int64_t)j * L.pitch + (int64_t)k * L.plane, rx, ry, rz, kap);
    }
    return pw(s)[(int64_t)fc * NC + kap];
  }

  __device__ void run() const {
    const int top = a.lf - a.lc;
    int cur[kMaxFused];
    for (int s = top; s >= 1; --s) {
      cur[s] = smooth(s, 0, a.mu_pre, true);
      const int ws = w(s), ms = m(s);
      const T* u = vec(s, cur[s]);
      T* r = vec(s, 3);
      for (int idx = threadIdx.x; idx < nint(s); idx += BS) {
        int i, j, k;
        vertex_of(idx, ms, mag[s], D, i, j, k);
        const int c = cidx(ws, i, j, k);
        r[c] = vec(s, 2)[c] - row_dot_lds(rows(s) + (int64_t)idx * NS, u, ws, c);
      }
      sync(small(s));  // the restriction's threads are a subset
      const int wc = w(s - 1), mc = m(s - 1);
      T* bc = vec(s - 1, 2);
      for (int idx = threadIdx.x; idx < nint(s - 1); idx += BS) {
        int I, J, K;
        vertex_of(idx, mc, mag[s - 1], D, I, J, K);
        T acc = (T)0;
        const int zlo = (D == 3) ? -2 : 0, zhi = (D == 3) ? 2 : 0;
        for (int oz = zlo; oz <= zhi; ++oz)
          for (int oy = -2; oy <= 2; ++oy)
#pragma unroll
            for (int ox = -2; ox <= 2; ++ox) {
              const int fi = 3 * I + ox, fj = 3 * J + oy, fk = 3 * K + oz;
              const int fc = cidx(ws, fi, fj, fk);
              const int kap = (ox < 0 ? 1 : 0) | (oy < 0 ? 2 : 0) | (oz < 0 ? 4 : 0);
              acc += weight(s, fc, fi, fj, fk, kap) * r[fc];
            }
        bc[cidx(wc, I, J, K)] = acc;
      }
      sync(small(s - 1));
    }
    // coarsest level
    if (a.coarse_direct) {
      const int ws = w(0), ms = m(0);
      const T* b0 = vec(0, 2);
      T* u0 = vec(0, 0);
      for (int row = threadIdx.x; row < a.nc; row += BS) {
        double acc = 0.0;
        for (int c = 0; c < a.nc; ++c) {
          int i, j, k;
          vertex_of(c, ms, mag[0], D, i, j, k);
          acc += a.Ainv[(int64_t)row * a.nc + c] * (double)b0[cidx(ws, i, j, k)];
        }
        int i, j, k;
        vertex_of(row, ms, mag[0], D, i, j, k);
        u0[cidx(ws, i, j, k)] = (T)acc;
      }
      sync(small(0) && a.nc <= 64);
      cur[0] = 0;
    } else {
      cur[0] = smooth(0, 0, a.mu_pre + a.mu_post, true);
    }
    for (int s = 1; s <= top; ++s) {
      // first level above the wave-0 levels: their results to every wave
      if (small(s - 1) && !small(s)) __syncthreads();
      const int ws = w(s), ms = m(s), wc = w(s - 1);
      T* u = vec(s, cur[s]);
      const T* ec = vec(s - 1, cur[s - 1]);
      for (int idx = threadIdx.x; idx < nint(s); idx += BS) {
        int i, j, k;
        vertex_of(idx, ms, mag[s], D, i, j, k);
        const int fc = cidx(ws, i, j, k);
        const int qx = i / 3, qy = j / 3, qz = k / 3;
        T acc = (T)0;
#pragma unroll
        for (int kap = 0; kap < NC; ++kap) {
          const int kx = kap & 1, ky = (kap >> 1) & 1, kz = (kap >> 2) & 1;
          if ((kx && i % 3 == 0) || (ky && j % 3 == 0) || (kz && k % 3 == 0)) continue;
          acc += weight(s, fc, i, j, k, kap) * ec[cidx(wc, qx + kx, qy + ky, qz + kz)];
        }
        u[fc] += acc;
      }
      sync(small(s));
      cur[s] = smooth(s, cur[s], a.mu_post, false);
    }
    // result of level lf back to global memory
    const Lat& L = a.L[top];
    const T* res = vec(top, cur[top]);
    for (int idx = threadIdx.x; idx < nint(top); idx += BS) {
      int i, j, k;
      vertex_of(idx, m(top), mag[top], D, i, j, k);
      a.u[top][i + (int64_t)j * L.pitch + (int64_t)k * L.plane] = res[cidx(w(top), i, j, k)];
    }
  }
};

template <int D, typename T, int ASRC, int PSRC, int FMT>
__global__ __launch_bounds__(block_of<D>()) void k_fused_coarse(FusedArgs<T> a) {
  extern __shared__ char smem[];
  Fused<D, T, ASRC, PSRC, FMT> f(a, smem);
  f.load();
  f.run();
}

template <int D, typename T, int ASRC, int PSRC, int FMT>
__global__ __launch_bounds__(block_of<D>()) void k_fused_prepare(FusedArgs<T> a) {
  Fused<D, T, ASRC, PSRC, FMT> f(a, a.img);
  f.build_static();
}

// Opts one kernel instance in to the device's whole per-workgroup LDS, once
// per device.  Server workers launch from several host threads at once, and
// grids of different sizes share an instance, so the attribute is set to the
// device maximum (never lowered) under a lock, and a per-device bit records
// it.  The first call for an instance comes from the build (launch with
// prepare set), outside any stream capture.
// The tag makes every kernel instance its own template instance, so that
// each keeps its own per-device bits (the kernel pointers of one iterate type
// share a function type).
template <typename Tag, typename Kern>
void lds_optin_once(Kern kernel) {
  static std::mutex mu;
  static std::atomic<uint64_t> done{0};
  int dev = 0;
  QMG_HIP(hipGetDevice(&dev));
  const uint64_t bit = dev < 64 ? (uint64_t)1 << dev : 0;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return;
  std::lock_guard<std::mutex> lk(mu);
  if (bit && (done.load(std::memory_order_relaxed) & bit)) return;
  int optin = 0;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || optin <= 0) {
    (void)hipGetLastError();
    optin = 64 * 1024;
  }
  QMG_HIP(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, optin));
  done.fetch_or(bit, std::memory_order_release);
}

template <int D, typename T, int AS, int PS, int F>
struct FusedTag {};

template <int D, typename T, int AS, int PS, int F>
void launch_one(const FusedArgs<T>& a, hipStream_t s, bool prepare) {
  lds_optin_once<FusedTag<D, T, AS, PS, F>>(k_fused_coarse<D, T, AS, PS, F>);
  if (prepare) {
    hipLaunchKernelGGL((k_fused_prepare<D, T, AS, PS, F>), dim3(1), dim3(block_of<D>()), 0, s, a);
    return;
  }
  hipLaunchKernelGGL((k_fused_coarse<D, T, AS, PS, F>), dim3(1), dim3(block_of<D>()), a.lds_bytes, s, a);
}

template <int D, typename T>
void dispatch_fused(const FusedArgs<T>& a, int asrc, int psrc, int fmt, hipStream_t s, bool prep) {
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      throw HipError(std::string("error pending before the fused coarse launch: ") + hipGetErrorString(e));
  }
  if (asrc == SRC_PLAIN) {
    launch_one<D, T, SRC_PLAIN, SRC_PLAIN, F64>(a, s, prep);
  } else if (asrc == SRC_GEOM) {
    launch_one<D, T, SRC_GEOM, SRC_GEOM, F64>(a, s, prep);
  } else {
    const bool ph = psrc == SRC_HIER;
    switch (fmt) {
      case F64: if (ph) launch_one<D, T, SRC_HIER, SRC_HIER, F64>(a, s, prep); else launch_one<D, T, SRC_HIER, SRC_GEOM, F64>(a, s, prep); break;
      case F32: if (ph) launch_one<D, T, SRC_HIER, SRC_HIER, F32>(a, s, prep); else launch_one<D, T, SRC_HIER, SRC_GEOM, F32>(a, s, prep); break;
      case F16: if (ph) launch_one<D, T, SRC_HIER, SRC_HIER, F16>(a, s, prep); else launch_one<D, T, SRC_HIER, SRC_GEOM, F16>(a, s, prep); break;
      case BPA: if (ph) launch_one<D, T, SRC_HIER, SRC_HIER, BPA>(a, s, prep); else launch_one<D, T, SRC_HIER, SRC_GEOM, BPA>(a, s, prep); break;
      default: if (ph) launch_one<D, T, SRC_HIER, SRC_HIER, BF16>(a, s, prep); else launch_one<D, T, SRC_HIER, SRC_GEOM, BF16>(a, s, prep); break;
    }
  }
  QMG_HIP(hipGetLastError());
}

}  // namespace

template <typename T>
size_t fused_lds_layout(int d, FusedArgs<T>& a, bool p_stored, bool pw_lds) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 15) & ~size_t(15);
    const size_t p = off;
    off += bytes;
    return p;
  };
  const int NS = d == 2 ? 9 : 27, NC = 1 << d;
  // sizes in 64 bits: the candidate levels of a large grid exceed any LDS by
  // far, and their layout is only measured, never launched
  for (int s = 0; s <= a.lf - a.lc; ++s) {
    const int64_t w = a.L[s].n + 1, m = a.L[s].n - 1;
    const int64_t nsl = d == 3 ? w * w * w : w * w;
    const int64_t nin = d == 3 ? m * m * m : m * m;
    a.lds_nslot[s] = (int)std::min<int64_t>(nsl, INT32_MAX);
    a.mag[s] = 0xFFFFFFFFu / (unsigned)m + 1u;
    const size_t pv = take((size_t)4 * nsl * sizeof(T));
    const size_t pr = take((size_t)nin * NS * sizeof(T));
    const size_t pp = (s >= 1 && p_stored && pw_lds) ? take((size_t)nsl * NC * sizeof(T)) : 0;
    a.lds_vec[s] = (int)std::min<size_t>(pv, INT32_MAX);
    a.lds_rows[s] = (int)std::min<size_t>(pr, INT32_MAX);
    a.lds_pw[s] = (int)std::min<size_t>(pp, INT32_MAX);
  }
  a.pw_lds = pw_lds ? 1 : 0;
  const size_t total = (off + 15) & ~size_t(15);
  a.lds_bytes = (int)std::min<size_t>(total, INT32_MAX);
  return total;
}
template size_t fused_lds_layout<double>(int, FusedArgs<double>&, bool, bool);
template size_t fused_lds_layout<float>(int, FusedArgs<float>&, bool, bool);

template <typename T>
void launch_fused_coarse(int d, const FusedArgs<T>& a, int asrc, int psrc, int fmt, hipStream_t s) {
  if (a.lf - a.lc + 1 > kMaxFused) throw HipError("fused coarse cycle: too many levels");
  if (a.img != nullptr && a.lds_bytes > kFusedImgBytes) throw HipError("fused coarse cycle: image too large");
  if (d == 2) dispatch_fused<2, T>(a, asrc, psrc, fmt, s, false);
  else dispatch_fused<3, T>(a, asrc, psrc, fmt, s, false);
}
template void launch_fused_coarse<double>(int, const FusedArgs<double>&, int, int, int, hipStream_t);
template void launch_fused_coarse<float>(int, const FusedArgs<float>&, int, int, int, hipStream_t);

template <typename T>
void launch_fused_prepare(int d, const FusedArgs<T>& a, int asrc, int psrc, int fmt, hipStream_t s) {
  if (a.img == nullptr || a.lds_bytes > kFusedImgBytes) throw HipError("fused coarse cycle: no room for the image");
  if (d == 2) dispatch_fused<2, T>(a, asrc, psrc, fmt, s, true);
  else dispatch_fused<3, T>(a, asrc, psrc, fmt, s, true);
}
template void launch_fused_prepare<double>(int, const FusedArgs<double>&, int, int, int, hipStream_t);
template void launch_fused_prepare<float>(int, const FusedArgs<float>&, int, int, int, hipStream_t);

}  // namespace qmg
