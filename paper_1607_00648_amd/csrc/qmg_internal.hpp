// Internal definitions shared by the HIP kernels and the host driver of the
// quasi-matrix-free multigrid library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/qmg.h"

namespace qmg {

// ---------------------------------------------------------------------------
// Constants of the method and of the data layout
// ---------------------------------------------------------------------------
constexpr int kSeg = 64;                       // lattice slots per store block (one wavefront)
constexpr double kEpsZero = 9.094947017729282e-13;  // 2^-40: default zero-delta threshold (relative)
constexpr double kDomSlack = 1e-10;            // diagonal-dominance slack of the definiteness check
constexpr int kCoarseDirectMax = 1024;         // coarsest levels up to this size are solved exactly

enum Fmt { F64 = 0, F32 = 1, F16 = 2, BF16 = 3, BPA = 4 };
enum Src { SRC_GEOM = 0, SRC_PLAIN = 1, SRC_HIER = 2 };

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ApiError : std::runtime_error {
  int code;
  ApiError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define QMG_STR2_(x) #x
#define QMG_STR_(x) QMG_STR2_(x)
#define QMG_HIP(call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      throw ::qmg::HipError(std::string(#call) + " [" + ::qmg::src_name(__FILE__) +            \
                            ":" QMG_STR_(__LINE__) "]: " + hipGetErrorString(e_));             \
  } while (0)

inline const char* src_name(const char* path) {
  const char* b = path;
  for (const char* p = path; *p; ++p)
    if (*p == '/') b = p + 1;
  return b;
}

// ---------------------------------------------------------------------------
// Lattice of one regular level.  Vertex (i,j,k), 0 <= i,j,k <= n, lives at slot
// i + pitch*j + plane*k; pitch is a multiple of 64 so that every 64-slot block
// lies in one x-row.  Cell c (low corner (i,j,k), 0 <= i,j,k < n) uses the slot
// of its low corner, so cell arrays share the vertex layout.
// ---------------------------------------------------------------------------
struct Lat {
  int d;
  int n;          // cells per axis
  int pitch;      // slots per x-row
  int64_t plane;  // slots per z-plane (pitch * (n+1)); 0 in 2D
  int64_t nslot;  // total slots
  double h;       // 1/n
};

inline Lat make_lat(int d, int level) {
  Lat L{};
  L.d = d;
  L.n = 1;
  for (int i = 0; i < level; ++i) L.n *= 3;
  L.pitch = ((L.n + 1 + kSeg - 1) / kSeg) * kSeg;
  L.plane = (d == 3) ? (int64_t)L.pitch * (L.n + 1) : 0;
  L.nslot = (d == 3) ? L.plane * (L.n + 1) : (int64_t)L.pitch * (L.n + 1);
  L.h = 1.0 / L.n;
  return L;
}

// Operator store of one level (stencils: 3^d entries per vertex; prolongation:
// 2^d parent weights per fine vertex).
//   SRC_GEOM : nothing stored, the rediscretised stencil / d-linear weights
//   SRC_PLAIN: `dense` holds nent arrays of nslot doubles (entry-major)
//   SRC_HIER : rediscretised / d-linear part on the fly plus a delta; `blk[b]`
//              is the compact index of 64-slot block b or -1 for an all-zero
//              delta; `payload` holds [cblk][nent][64] values of format `fmt`;
//              `scale` holds [cblk][64] power-of-two exponents (FP16 only).
//              BPA (the paper's codec, Sect. 5): block c of width W bytes per
//              entry starts at byte boff[c] & (2^56 - 1) of `payload`, W =
//              boff[c] >> 56 in 2..8; it holds [nent][64] signed exponent
//              bytes, then for j = 0..W-2 byte j (little endian) of the
//              two's-complement mantissas, [nent][64] each.  The value is
//              m 2^e.
struct Store {
  int src = SRC_GEOM;
  int fmt = F64;
  int nent = 0;
  const void* dense = nullptr;
  const int32_t* blk = nullptr;
  const void* payload = nullptr;
  const int8_t* scale = nullptr;
  const int64_t* boff = nullptr;
};

// ---------------------------------------------------------------------------
// Kernel launchers (kernels_level.hip / kernels_build.hip)
// ---------------------------------------------------------------------------
// Smoothing / residual / matvec on one level.  mode: 0 = Jacobi sweep
// (out = u + omega D^-1 (b - A u)), 1 = Jacobi sweep from u = 0 (u not read),
// 2 = residual out = b - A u, 3 = matvec out = A u, 4 = the Jacobi half of a
// block Jacobi step (iota-vertices copied, the others as mode 0).  When `partial` is non-null
// (modes 2 and 3) each workgroup adds its sum of squares of `out` there.
// T is double or float; eps has the iterate type.
// With ev_start/ev_stop the launch carries per-dispatch start/end timestamps.
template <typename T>
void launch_stencil(const Lat& L, int mode, const T* u, const T* b, T* out, const T* eps,
                    const Store& A, T omega, double* partial, int* n_partial, hipStream_t s,
                    hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// Block Jacobi, Gauss-Seidel half: `sweeps` lexicographic sweeps over the
// iota-vertices of every patch of level L, in place in u.
template <typename T>
void launch_bj_iota(const Lat& L, T* u, const T* b, const T* eps, const Store& A, int sweeps, hipStream_t s);

// Finest-level FP64 residual for the mixed loop: r32 = fp32(b - A x), partial
// sums of squares of the FP64 residual.
void launch_residual_mixed(const Lat& L, const double* x, const double* b, float* r32,
                           const double* eps, double* partial, int* n_partial, hipStream_t s);

// Sum of `n` partials into out[0] in a fixed order (one workgroup).  With
// `hist`, the sum is also stored at hist[*counter] (when below cap) and the
// device counter advanced, so that replayed cycles keep a norm history.
// Input staging: dst = scale * src (grid-stride over `blocks` blocks of 256;
// src may be dst, or the caller's device array), per-block sums of squares of
// the scaled values into partial[0..blocks), and a count of non-finite (or,
// with positive, non-positive) entries of src added to *bad.
void launch_prep_input(const double* src, double* dst, int64_t n, double scale, bool positive, double* partial,
                       int blocks, int* bad, hipStream_t s);
void launch_sum_partials(const double* partial, int n, double* out, hipStream_t s,
                         double* hist = nullptr, int* counter = nullptr, int cap = 0);
// `chunk` cycles' partial sums at once (stride apart) into hist[0..chunk);
// out[0] gets the last and the history counter becomes ctr_end.
void launch_sum_partials_multi(const double* partial, int n, int stride, int chunk, double* out, double* hist,
                               int* counter, int ctr_end, hipStream_t s);

// Restriction bc = P^T r (gather per coarse vertex).  Lf: fine lattice.
template <typename T>
void launch_restrict(const Lat& Lf, const Lat& Lc, const T* r, T* bc, const Store& P, hipStream_t s);

// Prolongation uf = (add ? uf : 0) + P ec (gather per fine vertex).
template <typename T>
void launch_prolong(const Lat& Lf, const Lat& Lc, const T* ec, T* uf, const Store& P, hipStream_t s);

// x64 += e32 on the interior.
// ec[V] -= xf[3V] - yf[3V] (yf may be null) at every interior coarse vertex V:
// the BPX surplus of a level's Jacobi step
template <typename T>
void launch_cpoint_sub(const Lat& Lf, const Lat& Lc, const T* xf, const T* yf, T* ec, hipStream_t s);
// Refinement criterion on a regular level: per-slot differences (-1 where no
// candidate) with their bit-pattern minimum and maximum in mm[0..1]; the
// ten-bin histogram of the candidates; the flags of the cells (x fastest)
// with a corner in bin >= kstar.
void launch_refine_delta(const Lat& L, const double* u, const double* r, double res_tol, double* delta,
                         unsigned long long* mm, hipStream_t s);
void launch_refine_hist(const Lat& L, const double* delta, double lo, double width, int spread, int* cnt,
                        hipStream_t s);
void launch_refine_cells(const Lat& L, const double* delta, double lo, double width, int spread, int kstar,
                         uint8_t* flags, hipStream_t s);
void launch_axpy_mixed(const Lat& L, double* x, const float* e, hipStream_t s);

// Conversions between iterate types and between packed unknown vectors and
// lattice arrays.
template <typename Ti, typename To>
void launch_convert(const Lat& L, const Ti* in, To* out, hipStream_t s);
template <typename T>
void launch_scatter_unknowns(const Lat& L, const double* in, T* lat, hipStream_t s);
template <typename T>
void launch_gather_unknowns(const Lat& L, const T* lat, double* out, hipStream_t s);
template <typename T>
void launch_scatter_cells(const Lat& L, const double* in, T* lat, hipStream_t s);

// Coarsest solve u = Ainv b over the interior unknowns (Ainv FP64, nc x nc).
template <typename T>
void launch_coarse_solve(const Lat& L, const double* Ainv, int nc, const T* b, T* u, hipStream_t s);
// Ainv (n x n, n <= kCoarseDirectMax) := inverse of the coarsest operator
// assembled from its full stencil array, on the device; *status = 1 when it
// is singular.
void launch_coarse_inverse(const Lat& L, const double* Afull, int n, double* Ainv, int* status, hipStream_t s);

// ---- build ----
// eps of level l-1 = mean of the 3^d children (lattice cell layout).
void launch_coarsen_eps(const Lat& Lf, const Lat& Lc, const double* epsf, double* epsc,
                        hipStream_t s);
// Materialise the operator of a level as FP64 stencils (entry-major, nent*nslot).
void launch_materialise(const Lat& L, const double* eps, const Store& A, double* out,
                        hipStream_t s);
// Materialise prolongation weights as FP64 (2^d * nslot of the fine level; Lc
// is the coarse lattice).
void launch_materialise_P(const Lat& Lf, const Lat& Lc, const Store& P, double* out, hipStream_t s);
// BoxMG P (Sect. 4.4): writes 2^d*nslot FP64 parent weights of the fine level.
// Afine: FP64 stencils of the fine level (entry-major); when null, the fine
// operator is rediscretised from epsf on the fly.
// vt_fine / cref_coarse (adaptive levels, nullable): fine vertex classes (rows
// of leaf and refined vertices from Afine or eps, hanging rows rediscretised
// from eps, others zero) and the refined flags of the coarse cells (only
// refined cells are patches).  cells (nullable, with cref_coarse): the n_cells
// refined coarse cells (cell index, x fastest); only their corners are solved.
// scratch (nullable, 3D listed cells with rediscretised rows): device memory
// of at least (n_cells + 16) ints; the constant-coefficient cells are then
// written first and the others solved in a second launch over their list.
// dirty (nullable, one int per 64-slot block of the fine level, zero on
// entry): the solve marks the blocks it writes; the weights of the others
// equal their d-linear reference exactly.  Returns whether it did (the split
// ran with dirty given).
bool launch_boxmg(const Lat& Lf, const Lat& Lc, const double* Afine, const double* epsf,
                  double* Pw, hipStream_t s, const int8_t* vt_fine = nullptr,
                  const int8_t* cref_coarse = nullptr, const int32_t* cells = nullptr, int64_t n_cells = 0,
                  void* scratch = nullptr, size_t scratch_bytes = 0, int32_t* dirty = nullptr);
// Galerkin RAP (Sect. 4.3): coarse FP64 stencils from fine stencils (or eps on
// the fly when Afine is null) and FP64 parent weights (d-linear when Pw null).
// vt_fine (nullable): vertex classes of the fine level; rows of vertices that
// are neither leaf nor refined count as zero.
// vt_coarse (nullable): only rows of refined coarse vertices are formed.
// verts (nullable): those n_verts vertices as interior indices (x fastest);
// only they are visited (the other rows must have been zeroed).
void launch_rap(const Lat& Lf, const Lat& Lc, const double* Afine, const double* epsf,
                const double* Pw, double* Ac, hipStream_t s, const int8_t* vt_fine = nullptr,
                const int8_t* vt_coarse = nullptr, const int32_t* verts = nullptr, int64_t n_verts = 0,
                int rmode = 0);
// The Galerkin product of the finest 3D adaptive level coarse cell by coarse
// cell: element matrices of the listed refined cells in `scratch`, then the
// rows of the listed refined vertices.  Returns false (nothing launched) when
// scratch_bytes cannot hold 64 doubles per cell plus an int per coarse cell.
bool launch_rap_cells(const Lat& Lf, const Lat& Lc, const double* epsf, const double* Pw, double* Ac,
                      hipStream_t s, const int8_t* vt_fine, const int8_t* vt_coarse, const int32_t* verts,
                      int64_t n_verts, const int32_t* cells, int64_t n_cells, void* scratch, size_t scratch_bytes);
// Adds the convection term (v constant per cell, d arrays of cell slots in
// vel) to the full stencils A of level L.
void launch_conv_add(const Lat& L, const double* vel, double* A, hipStream_t s);
// Petrov-Galerkin restrictions at interior coarse V: rmode 1, injection
// bc[V] = rf[3V]; rmode 2, aggregation bc[V] = sum of rf over the 3^d fine
// vertices within 1 of 3V.  (rmode 0, R = P^T, is launch_restrict.)
template <typename T>
void launch_inject(const Lat& Lf, const Lat& Lc, const T* rf, T* bc, hipStream_t s, int rmode = 1);
// Definiteness check of coarse stencils; counts failing rows into *bad.
void launch_check_rows(const Lat& Lc, const double* Ac, int* bad, hipStream_t s);
// Hierarchical delta store: per-block zero flags, compaction and payload.  The
// reference is the rediscretised stencil from eps (stencils) or the d-linear
// weights (is_P; Lc is then the coarse lattice), both with Dirichlet entries
// dropped.  blk gets 0/1 per block, then compact ids from the scan.  With
// eps_mf > 0 (the BPA format) blk gets the block's width instead: the largest
// per-vertex bpa, 0 when every vertex codes to zero; the scan then also writes
// boff (byte offset and width per compact block; `unit` = nent * 64 bytes per
// width step).
// tiles (nullable): only the listed 64 x 4 tiles of an adaptive level are
// encoded; the blocks of the others are flagged zero.  vt (nullable): the
// level's vertex classes; slots outside the level (no row or weight of theirs
// is ever read) take a zero delta, so that their blocks are not stored.
// marked: blk arrives with 1 on every block whose entries may differ from
// their reference and 0 elsewhere (the BoxMG launch marks them); the others
// are not loaded.
void launch_delta_flags(const Lat& L, const Lat& Lc, bool is_P, const double* full,
                        const double* eps, int32_t* blk, hipStream_t s, double eps_mf = 0.0,
                        const int32_t* tiles = nullptr, int ntiles = 0, double eps_zero = 0.0,
                        const int8_t* vt = nullptr, bool marked = false);
// csum: device scratch of scan_scratch_ints(nblk) ints (chunk sums).
void launch_scan_blocks(int32_t* blk, int64_t nblk, int32_t* total, hipStream_t s, int64_t* boff,
                        int64_t unit, int32_t* csum);
int64_t scan_scratch_ints(int64_t nblk);
void launch_delta_write(const Lat& L, const Lat& Lc, bool is_P, int fmt, const double* full,
                        const double* eps, const int32_t* blk, void* payload, int8_t* scale,
                        hipStream_t s, const int64_t* boff = nullptr, double eps_mf = 0.0,
                        const int32_t* tiles = nullptr, int ntiles = 0, const int8_t* vt = nullptr);

// Coarse part of the V-cycle in one workgroup with levels lc..lf held in LDS
// (lf starting from zero after its right-hand side was restricted into b of
// index lf - lc).  Index s of every array is level lc + s.
constexpr int kMaxFused = 8;
template <typename T>
struct FusedArgs {
  int lc, lf, mu_pre, mu_post, coarse_direct, nc;
  int bj_sweeps;  // block Jacobi smoother: Gauss-Seidel sweeps per patch (0: Jacobi)
  T omega;
  const double* Ainv;
  Lat L[kMaxFused];
  Store A[kMaxFused], P[kMaxFused];
  const T* eps[kMaxFused];
  T* u[kMaxFused];
  T* b[kMaxFused];
  // LDS layout (byte offsets): 4 iterate arrays (u, t, b, r) over the compact
  // (n+1)^d lattice, stencil rows of the interior, parent weights (when pw_lds)
  int lds_vec[kMaxFused], lds_rows[kMaxFused], lds_pw[kMaxFused], lds_nslot[kMaxFused];
  int lds_bytes, pw_lds;
  unsigned mag[kMaxFused];  // floor((2^32 - 1) / (n - 1)) + 1 per level: exact division by n - 1
  // precomputed LDS image (zero iterates, stencil rows, parent weights) in
  // global memory, copied into LDS at the start of every launch (nullable:
  // then the rows and weights are decoded in the kernel)
  char* img;
};
// Bytes reserved per grid for that image (the largest LDS a workgroup may use).
constexpr int kFusedImgBytes = 160 * 1024;
// Fills the LDS layout of `a` (levels lc..lf already set) and returns its bytes.
template <typename T>
size_t fused_lds_layout(int d, FusedArgs<T>& a, bool p_stored, bool pw_lds);
template <typename T>
void launch_fused_coarse(int d, const FusedArgs<T>& a, int asrc, int psrc, int fmt, hipStream_t s);
// Writes the LDS image of `a` (layout filled) to a.img (once per operator build).
template <typename T>
void launch_fused_prepare(int d, const FusedArgs<T>& a, int asrc, int psrc, int fmt, hipStream_t s);

// Fill lattice array with zeros (kernel, not memset, so it can live in graphs).
template <typename T>
void launch_zero(T* p, int64_t n, hipStream_t s);

// ---- fused smoothing passes of regular 2D levels (kernels_pass.hip) ----
// One launch: optional prolongation-add u += P e (pro), nsw (1 or 2) damped
// Jacobi sweeps from u (the first from zero when zero_first) into out, and an
// optional residual r = b - A out (res) with per-tile norm partials (partial,
// nullable; pass2d_partials(L) entries).
template <typename T>
struct PassArgs {
  Lat L, Lc;
  const T* u = nullptr;
  T* out = nullptr;
  const T* b = nullptr;
  T* r = nullptr;
  const T* eps = nullptr;
  const T* ec = nullptr;
  Store A, P;
  T omega = (T)0;
  int pro = 0, nsw = 1, res = 0, zero_first = 0;
  double* partial = nullptr;
};
template <typename T>
void launch_pass2d(const PassArgs<T>& p, hipStream_t s, hipEvent_t ev_start = nullptr,
                   hipEvent_t ev_stop = nullptr);
int pass2d_partials(const Lat& L);

// ---- adaptive levels (kernels_adaptive.hip) ----
enum VertexClass : int8_t { VT_OUT = 0, VT_LEAF = 1, VT_REFINED = 2, VT_HANGING = 3 };
// Active 64 x 4 (x, y) tiles of one level (3 ints per tile: x tile, y tile,
// z plane) and the vertex class of every slot of the level.
// On 3D adaptive levels also the 32 x 8 x 16 bricks (x brick, y brick,
// chunk of 16 interior planes) that hold a leaf, refined or hanging vertex,
// for the plane-marching sweep.  Bricks 32 slots wide fit a thin refined band
// better than 64-wide ones: on a level-6 band 32 x 16 bricks cover 2.2 slots
// per active vertex against 2.8, and load 3.0 halo-inclusive slots against
// 4.0.  Eight rows (256-thread workgroups, more of them per CU, each waiting
// at its barriers for four wavefronts) sweep that band in 550 us against 567
// for sixteen rows and 656 for 64 x 4.
struct AdTiles {
  Lat L;
  const int32_t* tiles = nullptr;
  const int8_t* vt = nullptr;
  int n = 0;
  const int32_t* bricks = nullptr;
  int nb = 0;
  // levels above the base: the hanging vertices' slots (hang == nullptr:
  // no list, the hanging values are found on the tiles)
  const int64_t* hang = nullptr;
  int64_t nh = 0;
  // levels above the base: the leaf and refined vertices' slots
  const int64_t* act = nullptr;
  int64_t na = 0;
};
constexpr int kBrickX = 32, kBrickY = 8, kBrickZ = 16;
constexpr int kMarchMinBricks = 4096;  // fewer bricks march serially: the tiles are faster
// mode 0: Jacobi sweep of leaf and refined vertices, 1: the same from zero,
// 2: residual (zero at hanging vertices; partial: per-workgroup sums of
// squares over the leaves).  Hanging values travel with the iterate (mode 0
// copies them).  Levels with at least kMarchMinBricks bricks take the
// brick-marching kernel for modes 0 and 2 (slots outside the active set and
// its hanging vertices are then not written); others one workgroup per
// listed tile plane.  Returns the number of partials written (0 when
// partial is null).  e0/e1 (mode 0 only, nullable): per-dispatch timestamps.
template <typename T, typename TO>
int launch_ad_stencil(const AdTiles& t, int mode, const T* u, const T* b, TO* out, const T* eps,
                      const Store& A, T omega, double* partial, hipStream_t s, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr);
// P: the fine level's prolongation store (d-linear, FP64 deltas, or plain)
template <typename T>
void launch_ad_hang(const AdTiles& tf, const Lat& Lc, T* uf, const T* uc, const Store& P, hipStream_t s);
template <typename T>
void launch_ad_inject(const AdTiles& tc, const Lat& Lf, const T* uf, T* uc, hipStream_t s);
// verts (nullable): the refined vertices of the coarse level (interior
// indices); then one wavefront per listed vertex instead of one thread per
// slot of the coarse level's active tiles.  With the refined cells and a
// part buffer (2^d iterates per coarse slot) the restriction runs by cell.
template <typename T>
void launch_ad_fas_rhs(const AdTiles& tc, const Lat& Lf, const T* rf, const T* uc, const T* epsc,
                       const Store& Ac, T* bc, const Store& P, hipStream_t s, const int32_t* verts = nullptr,
                       int64_t nverts = 0, const int32_t* cells = nullptr, int64_t ncells = 0, T* part = nullptr);
template <typename T>
void launch_ad_correct(const AdTiles& tf, const Lat& Lc, T* uf, const T* uc, const T* sc, const Store& P,
                       hipStream_t s);
// coefficients of the level-l cells that do not exist := their parent cell's
// vtf: vertex classes of the fine level; cells with no corner among its
// vertices are not written (no row reads them).  ef32 (nullable): also the
// single-precision copy of every cell a row reads (as launch_ad_convert_cells).
void launch_ad_virtual_eps(const Lat& Lf, const Lat& Lc, const int8_t* crefc, const int8_t* vtf, const double* ec,
                           double* ef, float* ef32, hipStream_t s);
// out := (float) in on the cells next to a vertex of the level (vt)
void launch_ad_convert_cells(const Lat& L, const int8_t* vt, const double* in, float* out, hipStream_t s);
template <typename T>
void launch_ad_copy(const AdTiles& t, const T* src, T* dst, hipStream_t s);
template <typename T>
// narr lattice arrays back to back; vertices_only: the slots of the level's
// vertices (not outside) only
void launch_ad_zero(const AdTiles& t, T* p, hipStream_t s, int narr = 1, bool vertices_only = false);
void launch_ad_axpy(const AdTiles& t, double* x, const float* e, hipStream_t s);
void launch_ad_coarsen_eps(const Lat& Lf, const Lat& Lc, const int8_t* cref, const double* ef, double* ec,
                           hipStream_t s);
// cleared: A holds zero on the rows of the level's vertices but the refined
// ones (only leaf rows are written; rows of slots outside the level are never
// read)
void launch_ad_merge_rows(const Lat& L, const int8_t* vt, const double* eps, double* A, bool cleared,
                          hipStream_t s);
template <typename T>
void launch_ad_scatter(const int64_t* slots, int64_t n, const double* in, double scale, T* lat, hipStream_t s);
template <typename T>
void launch_ad_gather(const int64_t* slots, int64_t n, const T* lat, double* out, hipStream_t s);

// ---- solve loop as a state machine (api.cpp); used by the server ----
constexpr int kHistCap = 1024;  // cycles per batch between host synchronisations

// qmg_create_grid with an optional caller-owned pinned host buffer of kHistCap
// doubles for the residual history (the server reuses one per slot).
int create_grid(const qmg_grid_desc* desc, const qmg_solver_opts* opts, void* device_buf, size_t bytes,
                void* stream, double* pinned_hist, qmg_grid_t** out);

struct SolveState {
  double tol = 1e-8;
  int max_cycles = 0;
  int cycles = 0, outer = 0, batch = 2;
  double rr = 0.0, rr_prev = 0.0;
  std::vector<double> history;
  bool done = false;
  double t0 = 0.0;
};
// Residual of the current iterate (blocking); st.done if nothing to do.
void solve_begin(qmg_grid_t* g, SolveState& st, double tol, int max_cycles);
// Enqueues the next batch of cycles (non-blocking).
void solve_enqueue(qmg_grid_t* g, SolveState& st);
// True when the batch in flight has finished on the device.
bool solve_ready(qmg_grid_t* g);
// Reads the finished batch's norms and updates the state (sets st.done).
void solve_collect(qmg_grid_t* g, SolveState& st);
void solve_fill_report(qmg_grid_t* g, const SolveState& st, qmg_solve_report* rep);

}  // namespace qmg
