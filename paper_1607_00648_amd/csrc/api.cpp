// Host driver and C ABI of the quasi-matrix-free multigrid library: workspace
// layout, coefficient upload, operator construction (Sect. 4.3, 3.4, 4),
// V-cycles (Alg. 1, correction-scheme form on regular grids), the FP64
// defect-correction loop around FP32 cycles, and inspection entry points.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "qmg_internal.hpp"

using namespace qmg;

namespace {

thread_local std::string g_thread_err;


int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// bytes per stored entry (BPA: the widest block, one exponent byte and seven
// mantissa bytes)
size_t fmt_size(int fmt) { return (fmt == F64 || fmt == BPA) ? 8 : fmt == F32 ? 4 : 2; }

int store_fmt(int store) {
  switch (store) {
    case QMG_HIER_FP32: return F32;
    case QMG_HIER_FP16: return F16;
    case QMG_HIER_BF16: return BF16;
    case QMG_HIER_BPA: return BPA;
    default: return F64;
  }
}

struct LevelBuf {
  Lat L{};
  double* eps64 = nullptr;
  float* eps32 = nullptr;
  void* u = nullptr;  // iterate type
  void* t = nullptr;
  void* b = nullptr;
  void* r = nullptr;
  Store A, P;
  double* Adense = nullptr;
  double* Pdense = nullptr;
  int32_t* Ablk = nullptr;
  void* Apay = nullptr;
  int8_t* Ascale = nullptr;
  int32_t* Pblk = nullptr;
  void* Ppay = nullptr;
  int8_t* Pscale = nullptr;
  int64_t* Aoff = nullptr;  // BPA: offset and width per compact block
  int64_t* Poff = nullptr;
  int64_t Anz = -1, Pnz = -1;  // stored non-zero blocks (-1: no store)
  // adaptive spacetrees, levels base..L: vertex classes, refined-cell flags,
  // active tiles and the saved iterate of the FAS cycle
  int8_t* vt = nullptr;
  int8_t* cref = nullptr;
  int32_t* tiles = nullptr;
  int ntiles = 0;
  int32_t* bricks = nullptr;  // 3D: bricks for the plane-marching sweep
  int nbricks = 0;
  int64_t* hang = nullptr;  // slots of the hanging vertices (levels above the base)
  int64_t nhang = 0;
  int64_t* act = nullptr;  // slots of the leaf and refined vertices (levels above the base)
  int64_t nact = 0;
  void* rpart = nullptr;  // coarse levels of an adaptive pair: FAS restriction parts per cell slot
  int32_t* rv = nullptr;  // refined vertices and cells (levels base..L-1), for the build
  int64_t nrv = 0;
  int32_t* rc = nullptr;
  int64_t nrc = 0;
  void* sv = nullptr;
  double* x64 = nullptr;  // FP32 iterates: FP64 solution and right-hand side of the level
  double* b64 = nullptr;
  AdTiles ad() const {
    AdTiles t;
    t.L = L;
    t.tiles = tiles;
    t.vt = vt;
    t.n = ntiles;
    t.bricks = bricks;
    t.nb = nbricks;
    t.hang = hang;
    t.nh = nhang;
    t.act = act;
    t.na = nact;
    return t;
  }
};

// Host-side linearisation of one level of an adaptive spacetree.
struct HostLevel {
  std::vector<int8_t> vt;         // vertex class per lattice slot
  std::vector<int8_t> cref;       // refined flag per cell slot
  std::vector<int32_t> tiles;     // active tiles (x tile, y tile, z plane)
  std::vector<int32_t> bricks;    // 3D: bricks holding a leaf, refined or hanging vertex
  std::vector<int64_t> leaf;      // slots of the unknowns (x fastest)
  std::vector<int64_t> hang;      // slots of the hanging vertices (x fastest)
  std::vector<int64_t> act;       // slots of the leaf and refined vertices (x fastest)
  std::vector<int64_t> cells;     // slots of the leaf cells (x fastest)
  std::vector<int32_t> rverts;    // refined interior vertices (interior index, x fastest)
  std::vector<int32_t> rcells;    // refined cells (cell index, x fastest)
  int64_t n_active = 0;           // leaf + refined vertices
};

// Bump allocator over the workspace; with base == nullptr it only measures.
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(int64_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(count, 0) * sizeof(T);
    return p;
  }
};

}  // namespace

struct qmg_grid {
  qmg_grid_desc desc{};
  qmg_solver_opts opts{};
  int d = 2, Lmax = 2, lcq = 1, lc = 1;
  bool mixed = false, plain = false;
  int fmt = F64;
  std::vector<LevelBuf> lv;
  double* x64 = nullptr;    // mixed: FP64 solution on the finest level
  double* bfin = nullptr;   // mixed: FP64 right-hand side on the finest level
  double* stage = nullptr;  // packed IO staging (nslot of the finest level)
  double* vel = nullptr;    // convection: d arrays of finest cell slots (library-owned)
  void* rscr = nullptr;     // refinement criterion: extrema and bin counts (library-owned)
  double* norm_dst = nullptr;  // where the finest pass leaves its norm partials (null: partial)
  bool has_conv = false;
  double* partial = nullptr;
  int npart = 0;   // entries of `partial`
  int npart1 = 0;  // partials of one residual norm (stride of deferred ones)
  double* dscal = nullptr;
  int* dcount = nullptr;
  int32_t* dtotal = nullptr;
  int32_t* scan_tmp = nullptr;  // chunk sums of the block scans
  double* Ainv = nullptr;
  int64_t ainv_cap = 0;
  int nc = 0;
  bool coarse_direct = false;
  int lf = -1;  // top level of the fused single-workgroup coarse cycle (-1: none)
  bool lf_pw_lds = true;
  char* fimg = nullptr;      // LDS image of the fused coarse levels (kFusedImgBytes)
  bool fimg_ready = false;
  int64_t lds_max = 65536;  // LDS bytes one workgroup may use on this device
  double* tmpA[2] = {nullptr, nullptr};
  double* tmpP = nullptr;
  char* base = nullptr;
  size_t bytes = 0;
  bool owns = false;
  bool own_hnorm = true;  // pinned history buffer allocated by the grid
  hipStream_t stream = nullptr;
  bool have_coef = false, have_ops = false;
  // adaptive levels: every slot outside the active tiles holds zero in the
  // iterate, right-hand side and coefficient arrays (no kernel writes there
  // after the first set_coefficients cleared the whole lattices)
  bool lattices_clear = false;
  double bnorm = 0.0;
  int64_t n_unknowns = 0;
  size_t bytes_ops = 0;
  double zero_frac = 0.0;
  std::string err;
  // adaptive spacetree (base < L); a regular grid has base == L
  bool adaptive = false;
  int lb = 0;  // base level (complete level of the spacetree)
  std::vector<HostLevel> hl;
  int64_t* unk_slots = nullptr;   // device copies of the leaf / leaf-cell slot lists
  int64_t* cell_slots = nullptr;
  int64_t n_cells = 0;
  // device norm history of replayed cycles, its pinned host copy and the
  // event marking the end of the batch in flight
  double* dhist = nullptr;
  int* dctr = nullptr;
  double* hnorm = nullptr;
  hipEvent_t bev = nullptr;
  int inflight = 0;
  // one cycle (+ residual norm) captured as a HIP graph
  hipGraphExec_t gexec = nullptr;
  bool own_stream = false;
  // optional HIP-event timing of every finest-level smoothing launch
  int prof_every = 0;       // time every k-th finest-level sweep (0: off)
  int64_t prof_count = 0;   // finest-level sweeps since profiling was enabled
  std::vector<hipEvent_t> prof_ev;  // start/stop pairs
  size_t prof_used = 0;
  int64_t prof_launches = 0;
  double prof_ms = 0.0;
};

namespace {

void set_err(qmg_grid_t* g, const std::string& m) {
  if (g) g->err = m;
  g_thread_err = m;
}

template <class F>
int guard(qmg_grid_t* g, F&& f) {
  try {
    // The launch checks below read the thread's last HIP error; one left
    // behind by other code on this thread (the caller's own HIP calls) is not
    // this call's, so it is cleared first.
    (void)hipGetLastError();
    f();
    return QMG_OK;
  } catch (const ApiError& e) {
    set_err(g, e.what());
    return e.code;
  } catch (const HipError& e) {
    set_err(g, e.what());
    return QMG_EHIP;
  } catch (const std::bad_alloc&) {
    set_err(g, "host allocation failed");
    return QMG_ENOMEM;
  } catch (const std::exception& e) {
    set_err(g, e.what());
    return QMG_EINVAL;
  }
}

void validate_region(const qmg_region& r, int d, int L) {
  if (r.level < 0 || r.level > L) throw ApiError(QMG_EINVAL, "region level out of range (0..max_level)");
  if (r.n_params < 0 || (r.n_params > 0 && !r.params)) throw ApiError(QMG_EINVAL, "bad region parameters");
  for (int i = 0; i < r.n_params; ++i)
    if (!std::isfinite(r.params[i])) throw ApiError(QMG_EINVAL, "region parameters must be finite");
  if (r.kind == QMG_REGION_BALL) {
    if (r.n_params != d + 1 || !(r.params[d] > 0.0)) throw ApiError(QMG_EINVAL, "a ball takes centre and radius > 0");
  } else if (r.kind == QMG_REGION_LEVELSET_BAND) {
    if (r.n_params < 3) throw ApiError(QMG_EINVAL, "a level-set band takes tau, amplitude, M, k, phases");
    const double M = r.params[2];
    if (!(M >= 1.0 && M <= 65536.0 && M == std::floor(M)) || r.n_params != 3 + (int)M * (d + 1))
      throw ApiError(QMG_EINVAL, "a level-set band takes 3 + M (d + 1) values");
    if (!(r.params[0] >= 0.0)) throw ApiError(QMG_EINVAL, "band half-width tau must be >= 0");
  } else if (r.kind == QMG_REGION_CELL_LIST) {
    if (r.n_params % (d + 1) != 0) throw ApiError(QMG_EINVAL, "a cell list takes groups of 1 + d values");
    for (int q = 0; q < r.n_params; q += d + 1) {
      const double lv = r.params[q];
      if (!(lv >= 0.0 && lv <= L && lv == std::floor(lv))) throw ApiError(QMG_EINVAL, "cell list: bad level");
      const double n = std::pow(3.0, lv);
      for (int a = 1; a <= d; ++a)
        if (!(r.params[q + a] >= 0.0 && r.params[q + a] < n && r.params[q + a] == std::floor(r.params[q + a])))
          throw ApiError(QMG_EINVAL, "cell list: cell index out of range");
    }
  } else {
    throw ApiError(QMG_EINVAL, "unknown region kind");
  }
}

void validate(const qmg_grid_desc* desc, const qmg_solver_opts* o) {
  if (!desc || !o) throw ApiError(QMG_EINVAL, "null descriptor or options");
  if (desc->dim != 2 && desc->dim != 3) throw ApiError(QMG_EINVAL, "dim must be 2 or 3");
  if (desc->max_level < 2 || desc->max_level > (desc->dim == 2 ? 10 : 6))
    throw ApiError(QMG_EINVAL, "max_level out of range (2..10 in 2D, 2..6 in 3D)");
  if (o->transfer < QMG_GEOMETRIC || o->transfer > QMG_BOXMG) throw ApiError(QMG_EINVAL, "bad transfer");
  if (o->store < QMG_PLAIN_FP64 || o->store > QMG_HIER_BPA) throw ApiError(QMG_EINVAL, "bad store");
  if (o->store == QMG_HIER_BPA && !(o->eps_mf > 0.0 && o->eps_mf <= 1.0))
    throw ApiError(QMG_EINVAL, "the bpa store needs 0 < eps_mf <= 1");
  if (o->mu_pre < 1 || o->mu_post < 1) throw ApiError(QMG_EINVAL, "mu_pre and mu_post must be >= 1");
  if (!(o->omega > 0.0 && o->omega < 2.0)) throw ApiError(QMG_EINVAL, "omega must lie in (0, 2)");
  if (o->coarsest_level < 1 || o->coarsest_level > desc->max_level - 1)
    throw ApiError(QMG_EINVAL, "coarsest_level must satisfy 1 <= lc < max_level");
  if (o->inner_cycles < 1) throw ApiError(QMG_EINVAL, "inner_cycles must be >= 1");
  if (!(o->stagnation >= 0.0 && o->stagnation < 1e6))
    throw ApiError(QMG_EINVAL, "stagnation must be 0 (off) or a positive factor");
  if (o->smoother != QMG_SMOOTH_JACOBI && o->smoother != QMG_SMOOTH_BLOCK) throw ApiError(QMG_EINVAL, "bad smoother");
  if (o->smoother == QMG_SMOOTH_BLOCK && (o->bj_sweeps < 1 || o->bj_sweeps > 64))
    throw ApiError(QMG_EINVAL, "bj_sweeps must lie in 1..64");
  if (o->cycle != QMG_CYCLE_MULT && o->cycle != QMG_CYCLE_ADD && o->cycle != QMG_CYCLE_BPX)
    throw ApiError(QMG_EINVAL, "bad cycle");
  if (o->damping != QMG_DAMP_EXP && o->damping != QMG_DAMP_CONST) throw ApiError(QMG_EINVAL, "bad damping");
  if (o->restriction != QMG_R_TRANSPOSE && o->restriction != QMG_R_INJECTION &&
      o->restriction != QMG_R_AGGREGATION)
    throw ApiError(QMG_EINVAL, "bad restriction");
  if (o->restriction != QMG_R_TRANSPOSE && (o->transfer == QMG_GEOMETRIC || o->cycle != QMG_CYCLE_MULT))
    throw ApiError(QMG_EINVAL, "injection and aggregation are Petrov-Galerkin restrictions of multiplicative cycles");
  if (o->cycle != QMG_CYCLE_MULT && o->smoother != QMG_SMOOTH_JACOBI)
    throw ApiError(QMG_EINVAL, "additive and BPX cycles take one Jacobi step per level");
  if (o->coarse_solver != QMG_COARSE_DIRECT && o->coarse_solver != QMG_COARSE_SWEEPS)
    throw ApiError(QMG_EINVAL, "bad coarse_solver");
  if (!(o->eps_zero >= 0.0 && o->eps_zero <= 1e-2)) throw ApiError(QMG_EINVAL, "eps_zero must lie in [0, 1e-2]");
  if (o->iterate != QMG_IT_STORE && o->iterate != QMG_IT_FP64 && o->iterate != QMG_IT_FP32)
    throw ApiError(QMG_EINVAL, "bad iterate");
  {
    const bool reduced = o->store >= QMG_HIER_FP32 && o->store <= QMG_HIER_BF16;
    if (o->iterate == QMG_IT_FP64 && reduced)
      throw ApiError(QMG_EINVAL, "FP32, FP16 and BF16 deltas run with FP32 iterates");
    if (o->iterate == QMG_IT_FP32 && (o->store == QMG_PLAIN_FP64 || o->store == QMG_HIER_BPA))
      throw ApiError(QMG_EINVAL, "FP32 iterates run on the HIER_FP64, FP32, FP16 or BF16 stores");
    if (o->iterate == QMG_IT_FP32 && (o->cycle != QMG_CYCLE_MULT || o->smoother != QMG_SMOOTH_JACOBI ||
                                      o->restriction != QMG_R_TRANSPOSE) && !reduced)
      throw ApiError(QMG_EINVAL, "FP32 iterates with HIER_FP64 deltas run multiplicative Jacobi cycles");
  }
  const bool adaptive = desc->base_level != 0 && desc->base_level != desc->max_level;
  if (!adaptive && desc->n_regions != 0)
    throw ApiError(QMG_EINVAL, "refinement regions need an adaptive grid (1 <= base < max_level)");
  if (adaptive) {
    if (desc->base_level < 1 || desc->base_level > desc->max_level)
      throw ApiError(QMG_EINVAL, "base_level must satisfy 1 <= base <= max_level");
    if (desc->n_regions < 0 || (desc->n_regions > 0 && !desc->regions))
      throw ApiError(QMG_EINVAL, "bad region list");
    if (!desc->refine && desc->n_regions == 0)
      throw ApiError(QMG_EINVAL, "adaptive grid without refinement flags or regions");
    for (int r = 0; r < desc->n_regions; ++r) validate_region(desc->regions[r], desc->dim, desc->max_level);
    if (o->coarsest_level > desc->base_level)
      throw ApiError(QMG_EINVAL, "coarsest_level must not exceed base_level");
    if (o->smoother == QMG_SMOOTH_BLOCK) throw ApiError(QMG_EINVAL, "block Jacobi runs on regular grids");
    if (o->cycle != QMG_CYCLE_MULT) throw ApiError(QMG_EINVAL, "additive and BPX cycles run on regular grids");
    if (o->store == QMG_HIER_BPA) throw ApiError(QMG_EINVAL, "the bpa store runs on regular grids");
    if (o->restriction != QMG_R_TRANSPOSE)
      throw ApiError(QMG_EINVAL, "injection and aggregation run on regular grids");
  }
}

// Does cell c (indices x first) of level l meet a ball or level-set band
// region?  The arithmetic follows the stated definitions term by term: box
// [c/n, c/n + 1/n], sample points c/n + (o/2)/n, phi summed over m in order.
bool region_meets(const qmg_region& r, int d, int l, const int64_t* c) {
  const double n = std::pow(3.0, l);
  double lo[3];
  for (int a = 0; a < d; ++a) lo[a] = (double)c[a] / n;
  if (r.kind == QMG_REGION_BALL) {
    double s2 = 0.0;
    for (int a = 0; a < d; ++a) {
      const double hi = lo[a] + 1.0 / n;
      const double g = std::max(std::max(lo[a] - r.params[a], 0.0), std::max(r.params[a] - hi, 0.0));
      s2 += g * g;
    }
    return std::sqrt(s2) < r.params[d];
  }
  const double tau = r.params[0], amp = r.params[1];
  const int M = (int)r.params[2];
  const double* k = r.params + 3;
  const double* ph = r.params + 3 + (size_t)M * d;
  double mn = INFINITY, mx = -INFINITY, amin = INFINITY;
  const int ns = d == 3 ? 27 : 9;
  for (int s = 0; s < ns; ++s) {
    const int o[3] = {s % 3, (s / 3) % 3, s / 9};
    double x[3];
    for (int a = 0; a < d; ++a) x[a] = lo[a] + (o[a] * 0.5) / n;
    double acc = 0.0;
    for (int m = 0; m < M; ++m) {
      double t = 0.0;
      for (int a = 0; a < d; ++a) t += x[a] * k[(size_t)m * d + a];
      acc += std::cos(t + ph[m]);
    }
    const double phi = amp * acc;
    mn = std::min(mn, phi);
    mx = std::max(mx, phi);
    amin = std::min(amin, std::fabs(phi));
  }
  return amin < tau || (mn < 0.0 && mx > 0.0);
}

// Refinement flags of levels base..L-1 (one byte per cell, level after
// level): the caller's bytes OR-ed with every region.  Existence is tracked
// level by level so that only existing cells are evaluated; the cells of a
// level are split over host threads.
std::vector<uint8_t> refine_flags(const qmg_grid_desc* desc) {
  const int d = desc->dim, L = desc->max_level, base = desc->base_level;
  std::vector<int64_t> off(L + 1, 0);
  int64_t total = 0;
  for (int l = base; l < L; ++l) {
    off[l] = total;
    total += (int64_t)std::llround(std::pow(3.0, (double)l * d));
  }
  std::vector<uint8_t> out((size_t)total, 0);
  if (desc->refine) std::memcpy(out.data(), desc->refine, (size_t)total);
  for (int r = 0; r < desc->n_regions; ++r) {
    const qmg_region& R = desc->regions[r];
    if (R.kind != QMG_REGION_CELL_LIST) continue;
    for (int q = 0; q < R.n_params; q += d + 1) {
      const int lv = (int)R.params[q];
      if (lv < base || lv >= std::min(L, R.level)) continue;
      const int64_t n = (int64_t)std::llround(std::pow(3.0, lv));
      int64_t idx = 0;
      for (int a = d; a >= 1; --a) idx = idx * n + (int64_t)R.params[q + a];
      out[(size_t)(off[lv] + idx)] = 1;
    }
  }
  unsigned nth = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  std::vector<uint8_t> ref_prev;
  for (int l = base; l < L; ++l) {
    const int64_t n = (int64_t)std::llround(std::pow(3.0, l));
    const int64_t ncell = d == 3 ? n * n * n : n * n;
    const int64_t np = n / 3;
    uint8_t* fl = out.data() + off[l];
    std::vector<const qmg_region*> act;
    for (int r = 0; r < desc->n_regions; ++r)
      if (desc->regions[r].kind != QMG_REGION_CELL_LIST && desc->regions[r].level > l) act.push_back(&desc->regions[r]);
    auto exists = [&](int64_t c) -> bool {
      if (l == base) return true;
      const int64_t cx = c % n, cy = (c / n) % n, cz = d == 3 ? c / (n * n) : 0;
      return ref_prev[(size_t)(cx / 3 + np * (cy / 3 + (d == 3 ? np * (cz / 3) : 0)))] != 0;
    };
    if (!act.empty()) {
      auto work = [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
          if (fl[c] || !exists(c)) continue;
          const int64_t ci[3] = {c % n, (c / n) % n, d == 3 ? c / (n * n) : 0};
          for (const qmg_region* R : act)
            if (region_meets(*R, d, l, ci)) {
              fl[c] = 1;
              break;
            }
        }
      };
      if (ncell < 4096 || nth == 1) {
        work(0, ncell);
      } else {
        std::vector<std::thread> th;
        const int64_t chunk = (ncell + nth - 1) / nth;
        for (unsigned t = 0; t < nth; ++t) {
          const int64_t c0 = std::min<int64_t>(ncell, (int64_t)t * chunk), c1 = std::min<int64_t>(ncell, c0 + chunk);
          th.emplace_back(work, c0, c1);
        }
        for (std::thread& x : th) x.join();
      }
    }
    std::vector<uint8_t> ref((size_t)ncell);
    for (int64_t c = 0; c < ncell; ++c) ref[(size_t)c] = (uint8_t)(fl[c] && exists(c));
    ref_prev.swap(ref);
  }
  return out;
}

// Spacetree of levels base..L (Sect. 3): cells of level base all exist; a
// cell of a finer level exists when its parent is refined; a cell is refined
// when it exists, its flag is set and it is not on level L.  Vertex classes:
// hanging (fewer than 2^d existing cells), refined (all 2^d cells refined),
// leaf (the other non-hanging interior vertices), outside/boundary.
void linearise(qmg_grid_t* g) {
  const int d = g->d, L = g->Lmax, base = g->lb;
  g->hl.assign(L + 1, HostLevel{});
  std::vector<uint8_t> ref_prev;
  const uint8_t* fl = g->desc.refine;
  int64_t nprev = 0;
  for (int l = base; l <= L; ++l) {
    const Lat Lt = make_lat(d, l);
    const int64_t n = Lt.n;
    const int64_t ncell = d == 3 ? n * n * n : n * n;
    std::vector<uint8_t> exist((size_t)ncell), ref((size_t)ncell, 0);
    for (int64_t c = 0; c < ncell; ++c) {
      if (l == base) {
        exist[c] = 1;
      } else {
        const int64_t cx = c % n, cy = (c / n) % n, cz = d == 3 ? c / (n * n) : 0;
        const int64_t pc = cx / 3 + nprev * (cy / 3 + (d == 3 ? nprev * (cz / 3) : 0));
        exist[c] = ref_prev[pc];
      }
      if (l < L) ref[c] = exist[c] && fl[c] != 0;
    }
    if (l < L) fl += ncell;
    HostLevel& H = g->hl[l];
    H.vt.assign((size_t)Lt.nslot, VT_OUT);
    H.cref.assign((size_t)Lt.nslot, 0);
    auto cell = [&](int64_t i, int64_t j, int64_t k) -> int64_t { return i + n * (j + n * k); };
    for (int64_t k = 0; k < (d == 3 ? n : 1); ++k)
      for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
          const int64_t c = cell(i, j, k);
          const int64_t sl = i + j * Lt.pitch + k * Lt.plane;
          if (ref[c]) {
            H.cref[(size_t)sl] = 1;
            H.rcells.push_back((int32_t)c);
          }
          if (exist[c] && !ref[c]) H.cells.push_back(sl);
        }
    for (int64_t k = (d == 3 ? 1 : 0); k <= (d == 3 ? n - 1 : 0); ++k)
      for (int64_t j = 1; j <= n - 1; ++j)
        for (int64_t i = 1; i <= n - 1; ++i) {
          int cnt = 0, nref = 0;
          for (int s = 0; s < (1 << d); ++s) {
            const int64_t c = cell(i - (s & 1), j - ((s >> 1) & 1), d == 3 ? k - ((s >> 2) & 1) : 0);
            cnt += exist[c];
            nref += ref[c];
          }
          const int64_t sl = i + j * Lt.pitch + k * Lt.plane;
          int8_t t = VT_OUT;
          if (cnt == (1 << d)) t = (nref == (1 << d)) ? VT_REFINED : VT_LEAF;
          else if (cnt > 0) t = VT_HANGING;
          H.vt[(size_t)sl] = t;
          if (t == VT_LEAF) H.leaf.push_back(sl);
          if (t == VT_HANGING) H.hang.push_back(sl);
          if (t == VT_LEAF || t == VT_REFINED) H.act.push_back(sl);
          if (t == VT_REFINED)
            H.rverts.push_back((int32_t)((i - 1) + (n - 1) * ((j - 1) + (n - 1) * (d == 3 ? k - 1 : 0))));
          if (t == VT_LEAF || t == VT_REFINED) ++H.n_active;
        }
    // active tiles: every tile of the base level; on finer levels the tiles
    // holding a vertex that is not outside
    const int ntx = Lt.pitch / 64, nty = (int)((n + 1 + 3) / 4), ntz = d == 3 ? (int)n + 1 : 1;
    for (int tz = 0; tz < ntz; ++tz)
      for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx) {
          bool any = l == base;
          for (int jj = ty * 4; jj < std::min<int64_t>(ty * 4 + 4, n + 1) && !any; ++jj)
            for (int ii = tx * 64; ii < std::min<int64_t>(tx * 64 + 64, n + 1) && !any; ++ii)
              any = H.vt[(size_t)(ii + jj * Lt.pitch + tz * Lt.plane)] != VT_OUT;
          if (any) {
            H.tiles.push_back(tx);
            H.tiles.push_back(ty);
            H.tiles.push_back(tz);
          }
        }
    // bricks of kBrickX x kBrickY slots and kBrickZ interior planes (plane
    // 1 + kBrickZ bz on), listed z, y, x, that hold a vertex the sweep reads
    // or writes (leaf, refined or hanging)
    if (d == 3 && l > base) {
      const int nbx = Lt.pitch / kBrickX, nby = (int)((n + 1 + kBrickY - 1) / kBrickY);
      const int nbz = (int)((n - 1 + kBrickZ - 1) / kBrickZ);
      for (int bz = 0; bz < nbz; ++bz)
        for (int by = 0; by < nby; ++by)
          for (int bx = 0; bx < nbx; ++bx) {
            bool any = false;
            const int64_t k0 = 1 + (int64_t)bz * kBrickZ, k1 = std::min<int64_t>(k0 + kBrickZ, n);
            for (int64_t kk = k0; kk < k1 && !any; ++kk)
              for (int64_t jj = (int64_t)by * kBrickY; jj < std::min<int64_t>((int64_t)by * kBrickY + kBrickY, n + 1) && !any; ++jj)
                for (int64_t ii = (int64_t)bx * kBrickX; ii < std::min<int64_t>((int64_t)bx * kBrickX + kBrickX, n + 1); ++ii) {
                  const int8_t t = H.vt[(size_t)(ii + jj * Lt.pitch + kk * Lt.plane)];
                  if (t == VT_LEAF || t == VT_REFINED || t == VT_HANGING) {
                    any = true;
                    break;
                  }
                }
            if (any) {
              H.bricks.push_back(bx);
              H.bricks.push_back(by);
              H.bricks.push_back(bz);
            }
          }
    }
    ref_prev.swap(ref);
    nprev = n;
  }
}

int64_t n_interior(const Lat& L) {
  const int64_t m = L.n - 1;
  return L.d == 3 ? m * m * m : m * m;
}

// Eager cycles on regular grids defer the per-cycle reduction of the residual
// norm partials and run it once for several cycles.
constexpr int kDeferNorms = 32;
bool defers_norms(const qmg_grid_t* g) { return !g->adaptive; }

int npartials(const Lat& L) {
  return (L.pitch / 64) * ((L.n + 1 + 3) / 4) * (L.d == 3 ? L.n + 1 : 1);
}

// Format of the stored prolongation of fine level l: the store's, except on
// adaptive levels, where P also defines the hanging values of the composite
// system and stays FP64.
int p_fmt(const qmg_grid_t* g, int l) { return (g->adaptive && l > g->lb) ? (int)F64 : g->fmt; }

// Lays out every buffer of the grid in the arena (measure or assign).
void layout(qmg_grid_t* g, Arena& a) {
  const int d = g->d, L = g->Lmax, lcq = g->lcq;
  const int NS = ipow(3, d), NC = 1 << d;
  const size_t it = g->mixed ? sizeof(float) : sizeof(double);
  const bool galerkin = g->opts.transfer != QMG_GEOMETRIC;
  const bool boxmg = g->opts.transfer == QMG_BOXMG;
  g->lv.assign(L + 1, LevelBuf{});
  for (int l = 0; l <= L; ++l) g->lv[l].L = make_lat(d, l);
  int64_t n_unk = 0, n_cells = 0, ad_partials = 0;
  if (g->adaptive) {
    for (int l = g->lb; l <= L; ++l) {
      LevelBuf& B = g->lv[l];
      const HostLevel& H = g->hl[l];
      B.ntiles = (int)(H.tiles.size() / 3);
      B.nbricks = (int)(H.bricks.size() / 3);
      B.vt = a.take<int8_t>(B.L.nslot);
      if (l < L) B.cref = a.take<int8_t>(B.L.nslot);
      B.tiles = a.take<int32_t>((int64_t)H.tiles.size());
      B.bricks = a.take<int32_t>((int64_t)H.bricks.size());
      if (l > g->lb) {
        B.nhang = (int64_t)H.hang.size();
        B.hang = a.take<int64_t>(std::max<int64_t>(B.nhang, 1));
        B.nact = (int64_t)H.act.size();
        B.act = a.take<int64_t>(std::max<int64_t>(B.nact, 1));
      }
      if (l < L) B.sv = a.take<char>(B.L.nslot * (int64_t)it);
      if (l < L) {
        B.nrv = (int64_t)H.rverts.size();
        B.rv = a.take<int32_t>(std::max<int64_t>(B.nrv, 1));
        B.nrc = (int64_t)H.rcells.size();
        B.rc = a.take<int32_t>(std::max<int64_t>(B.nrc, 1));
        B.rpart = a.take<char>(B.L.nslot * (int64_t)(1 << d) * it);
      }
      if (g->mixed) {
        B.x64 = a.take<double>(B.L.nslot);
        B.b64 = a.take<double>(B.L.nslot);
      }
      n_unk += (int64_t)H.leaf.size();
      n_cells += (int64_t)H.cells.size();
      ad_partials += B.ntiles;
    }
    g->unk_slots = a.take<int64_t>(n_unk);
    g->cell_slots = a.take<int64_t>(n_cells);
  }
  for (int l = lcq; l <= L; ++l) {
    LevelBuf& B = g->lv[l];
    const int64_t ns = B.L.nslot;
    B.eps64 = a.take<double>(ns);
    if (g->mixed) B.eps32 = a.take<float>(ns);
    B.u = a.take<char>(ns * it);
    B.t = a.take<char>(ns * it);
    B.b = a.take<char>(ns * it);
    B.r = a.take<char>(ns * it);
    const bool hasA = (l < L) || g->plain;
    if (hasA) {
      if (g->plain) {
        B.Adense = a.take<double>(ns * NS);
      } else if (galerkin && l < L) {
        B.Ablk = a.take<int32_t>(ns / kSeg);
        B.Apay = a.take<char>(ns * NS * fmt_size(g->fmt));
        if (g->fmt == F16) B.Ascale = a.take<int8_t>(ns);
        if (g->fmt == BPA) B.Aoff = a.take<int64_t>(ns / kSeg);
      }
    }
    if (l > lcq) {
      const int pf = p_fmt(g, l);
      if (g->plain) {
        B.Pdense = a.take<double>(ns * NC);
      } else if (boxmg) {
        B.Pblk = a.take<int32_t>(ns / kSeg);
        B.Ppay = a.take<char>(ns * NC * fmt_size(pf));
        if (pf == F16) B.Pscale = a.take<int8_t>(ns);
        if (pf == BPA) B.Poff = a.take<int64_t>(ns / kSeg);
      }
    }
  }
  if (!g->plain) {
    const int64_t nsA = g->lv[L - 1].L.nslot;
    g->tmpA[0] = a.take<double>(nsA * NS);
    g->tmpA[1] = a.take<double>(nsA * NS);
    if (boxmg) g->tmpP = a.take<double>(g->lv[L].L.nslot * NC);
  }
  if (g->mixed && !g->adaptive) {
    g->x64 = a.take<double>(g->lv[L].L.nslot);
    g->bfin = a.take<double>(g->lv[L].L.nslot);
  }
  g->stage = a.take<double>(g->lv[L].L.nslot);
  g->npart = (int)std::max<int64_t>(npartials(g->lv[L].L), ad_partials);
  g->npart1 = g->npart;
  if (defers_norms(g)) g->npart = kDeferNorms * g->npart1;
  g->partial = a.take<double>(g->npart);
  g->dscal = a.take<double>(8);
  g->dcount = a.take<int>(8);
  g->dtotal = a.take<int32_t>(2 * (L + 1));
  g->scan_tmp = a.take<int32_t>(scan_scratch_ints(g->lv[L].L.nslot / kSeg));
  g->fimg = a.take<char>(kFusedImgBytes);
  g->dhist = a.take<double>(kHistCap);
  g->dctr = a.take<int>(64);
  int64_t cap = 0;
  for (int l = lcq; l < L; ++l) {
    const int64_t m = n_interior(g->lv[l].L);
    if (m <= kCoarseDirectMax) cap = std::max(cap, m * m);
  }
  g->ainv_cap = cap;
  g->Ainv = a.take<double>(cap);
  (void)galerkin;
}

void init_modes(qmg_grid_t* g, const qmg_grid_desc* desc, const qmg_solver_opts* o) {
  g->desc = *desc;
  g->opts = *o;
  g->d = desc->dim;
  g->Lmax = desc->max_level;
  g->lcq = o->coarsest_level;
  g->lc = g->lcq;
  g->plain = o->store == QMG_PLAIN_FP64;
  g->mixed = (o->store >= QMG_HIER_FP32 && o->store <= QMG_HIER_BF16) ||
             (o->iterate == QMG_IT_FP32 && o->store == QMG_HIER_FP64);
  g->fmt = store_fmt(o->store);
  g->adaptive = desc->base_level != 0 && desc->base_level != desc->max_level;
  g->lb = g->adaptive ? desc->base_level : desc->max_level;
  if (g->adaptive) {
    std::vector<uint8_t> flags;
    if (desc->n_regions > 0) {
      flags = refine_flags(desc);
      g->desc.refine = flags.data();
    }
    linearise(g);
  }
  // the caller's arrays are not kept
  g->desc.refine = nullptr;
  g->desc.regions = nullptr;
  g->desc.n_regions = 0;
}

// uploads the host linearisation (after the device layout is assigned)
void upload_linearisation(qmg_grid_t* g) {
  if (!g->adaptive) return;
  int64_t uo = 0, co = 0;
  for (int l = g->lb; l <= g->Lmax; ++l) {
    LevelBuf& B = g->lv[l];
    HostLevel& H = g->hl[l];
    QMG_HIP(hipMemcpy(B.vt, H.vt.data(), H.vt.size(), hipMemcpyHostToDevice));
    if (B.cref) QMG_HIP(hipMemcpy(B.cref, H.cref.data(), H.cref.size(), hipMemcpyHostToDevice));
    if (!H.tiles.empty())
      QMG_HIP(hipMemcpy(B.tiles, H.tiles.data(), H.tiles.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!H.bricks.empty())
      QMG_HIP(hipMemcpy(B.bricks, H.bricks.data(), H.bricks.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (B.nhang > 0) QMG_HIP(hipMemcpy(B.hang, H.hang.data(), B.nhang * sizeof(int64_t), hipMemcpyHostToDevice));
    if (B.nact > 0) QMG_HIP(hipMemcpy(B.act, H.act.data(), B.nact * sizeof(int64_t), hipMemcpyHostToDevice));
    if (B.nrv > 0) QMG_HIP(hipMemcpy(B.rv, H.rverts.data(), B.nrv * sizeof(int32_t), hipMemcpyHostToDevice));
    if (B.nrc > 0) QMG_HIP(hipMemcpy(B.rc, H.rcells.data(), B.nrc * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!H.leaf.empty())
      QMG_HIP(hipMemcpy(g->unk_slots + uo, H.leaf.data(), H.leaf.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    if (!H.cells.empty())
      QMG_HIP(hipMemcpy(g->cell_slots + co, H.cells.data(), H.cells.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    uo += (int64_t)H.leaf.size();
    co += (int64_t)H.cells.size();
    // the class arrays stay on the host for numbering; drop the bulky ones
    H.vt.clear();
    H.vt.shrink_to_fit();
    H.cref.clear();
    H.cref.shrink_to_fit();
    H.rverts.clear();
    H.rverts.shrink_to_fit();
    H.rcells.clear();
    H.rcells.shrink_to_fit();
  }
  g->n_unknowns = uo;
  g->n_cells = co;
}

hipStream_t S(qmg_grid_t* g) { return g->stream; }

template <typename T>
const T* eps_of(const LevelBuf& B);
template <>
const double* eps_of<double>(const LevelBuf& B) { return B.eps64; }
template <>
const float* eps_of<float>(const LevelBuf& B) { return B.eps32; }

// ---------------------------------------------------------------------------
// V-cycle (Alg. 1 read as the correction scheme on regular grids)
// ---------------------------------------------------------------------------
void prof_harvest(qmg_grid_t* g) {
  if (g->prof_used == 0) return;
  QMG_HIP(hipEventSynchronize(g->prof_ev[2 * g->prof_used - 1]));
  for (size_t i = 0; i < g->prof_used; ++i) {
    float ms = 0.f;
    QMG_HIP(hipEventElapsedTime(&ms, g->prof_ev[2 * i], g->prof_ev[2 * i + 1]));
    g->prof_ms += ms;
  }
  g->prof_launches += (int64_t)g->prof_used;
  g->prof_used = 0;
}

hipEvent_t* prof_pair(qmg_grid_t* g) {
  constexpr size_t kPool = 2048;
  if (g->prof_used == kPool) prof_harvest(g);
  if (2 * (g->prof_used + 1) > g->prof_ev.size()) {
    hipEvent_t a, b;
    QMG_HIP(hipEventCreate(&a));
    QMG_HIP(hipEventCreate(&b));
    g->prof_ev.push_back(a);
    g->prof_ev.push_back(b);
  }
  return &g->prof_ev[2 * g->prof_used++];
}

// Restriction of the residual of level F into the right-hand side of C: P^T,
// or injection / aggregation for the Petrov-Galerkin variants.
template <typename T>
void restrict_to(qmg_grid_t* g, LevelBuf& F, LevelBuf& C, const T* r, T* bc) {
  if (g->opts.restriction != QMG_R_TRANSPOSE) launch_inject<T>(F.L, C.L, r, bc, S(g), g->opts.restriction);
  else launch_restrict<T>(F.L, C.L, r, bc, F.P, S(g));
}

template <typename T>
void smooth(qmg_grid_t* g, LevelBuf& B, int sweeps, bool zero_init) {
  const T om = (T)g->opts.omega;
  const bool finest = g->prof_every > 0 && B.L.n == g->lv[g->Lmax].L.n;
  if (g->opts.smoother == QMG_SMOOTH_BLOCK) {
    // block Jacobi: Gauss-Seidel on the iota-vertices in place, then the
    // Jacobi half into the other buffer
    if (zero_init) launch_zero<T>((T*)B.u, B.L.nslot, S(g));
    for (int k = 0; k < sweeps; ++k) {
      launch_bj_iota<T>(B.L, (T*)B.u, (const T*)B.b, eps_of<T>(B), B.A, g->opts.bj_sweeps, S(g));
      launch_stencil<T>(B.L, 4, (const T*)B.u, (const T*)B.b, (T*)B.t, eps_of<T>(B), B.A, om, nullptr,
                        nullptr, S(g));
      std::swap(B.u, B.t);
    }
    return;
  }
  for (int k = 0; k < sweeps; ++k) {
    const int mode = (k == 0 && zero_init) ? 1 : 0;
    // timed: every k-th full Jacobi sweep of the finest level (not the sweep
    // from a zero iterate, which reads no iterate)
    const bool timed = finest && mode == 0 && (g->prof_count++ % g->prof_every) == 0;
    hipEvent_t* ev = timed ? prof_pair(g) : nullptr;
    launch_stencil<T>(B.L, mode, (const T*)B.u, (const T*)B.b, (T*)B.t, eps_of<T>(B), B.A, om,
                      nullptr, nullptr, S(g), ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
    std::swap(B.u, B.t);
  }
}

template <typename T>
FusedArgs<T> fused_args(qmg_grid_t* g, int lf) {
  FusedArgs<T> a{};
  a.lc = g->lc;
  a.lf = lf;
  a.mu_pre = g->opts.mu_pre;
  a.mu_post = g->opts.mu_post;
  a.bj_sweeps = g->opts.smoother == QMG_SMOOTH_BLOCK ? g->opts.bj_sweeps : 0;
  a.coarse_direct = g->coarse_direct ? 1 : 0;
  a.nc = g->nc;
  a.omega = (T)g->opts.omega;
  a.Ainv = g->Ainv;
  a.img = g->fimg_ready ? g->fimg : nullptr;
  for (int l = g->lc; l <= lf; ++l) {
    LevelBuf& B = g->lv[l];
    const int s = l - g->lc;
    a.L[s] = B.L;
    a.A[s] = B.A;
    a.P[s] = B.P;
    a.eps[s] = eps_of<T>(B);
    a.u[s] = (T*)B.u;
    a.b[s] = (T*)B.b;
  }
  return a;
}

bool p_stored(const qmg_grid_t* g) {
  return g->lc + 1 <= g->Lmax && g->lv[g->lc + 1].P.src != SRC_GEOM;
}

// Largest level whose coarse cycle fits in the LDS of one workgroup (-1: none);
// prolongation weights go to LDS when they fit as well.
template <typename T>
int choose_fused_top(qmg_grid_t* g, bool& pw_lds) {
  int best = -1;
  if (g->opts.restriction != QMG_R_TRANSPOSE) return best;  // the fused cycle restricts with P^T
  for (int lf = g->lc; lf < g->lb && lf - g->lc + 1 <= kMaxFused; ++lf) {
    bool fits = false;
    for (int pl = 1; pl >= 0 && !fits; --pl) {
      FusedArgs<T> a = fused_args<T>(g, lf);
      if (fused_lds_layout<T>(g->d, a, p_stored(g), pl == 1) <= (size_t)g->lds_max) {
        best = lf;
        pw_lds = pl == 1;
        fits = true;
      }
    }
    if (!fits) break;  // a larger top level needs more still
  }
  return best;
}

// Decodes the fused levels' rows and weights once into the LDS image.
template <typename T>
void prepare_fused(qmg_grid_t* g) {
  FusedArgs<T> a = fused_args<T>(g, g->lf);
  if (fused_lds_layout<T>(g->d, a, p_stored(g), g->lf_pw_lds) > (size_t)kFusedImgBytes) return;
  a.img = g->fimg;
  const int psrc = g->lf > g->lc ? g->lv[g->lc + 1].P.src : SRC_GEOM;
  launch_fused_prepare<T>(g->d, a, g->lv[g->lf].A.src, psrc, g->fmt, S(g));
  g->fimg_ready = true;
}

template <typename T>
void fused_coarse(qmg_grid_t* g) {
  FusedArgs<T> a = fused_args<T>(g, g->lf);
  fused_lds_layout<T>(g->d, a, p_stored(g), g->lf_pw_lds);
  const int psrc = g->lf > g->lc ? g->lv[g->lc + 1].P.src : SRC_GEOM;
  launch_fused_coarse<T>(g->d, a, g->lv[g->lf].A.src, psrc, g->fmt, S(g));
}

// Smoothing of a regular 2D level as fused passes of at most two sweeps each
// (kernels_pass.hip): the first pass may start with the prolongation-add from
// C or from a zero iterate, the last may end with the residual (into B.r, and
// norm partials when `partial` is given).
template <typename T>
void passes(qmg_grid_t* g, LevelBuf& B, const LevelBuf* C, int sweeps, bool zero_init, bool residual,
            double* partial) {
  const bool finest = g->prof_every > 0 && B.L.n == g->lv[g->Lmax].L.n && C == nullptr;
  int left = sweeps;
  bool first = true;
  while (left > 0) {
    const int k = std::min(left, 2);
    const bool last = left == k;
    PassArgs<T> p;
    p.L = B.L;
    if (C) p.Lc = C->L;
    p.u = (const T*)B.u;
    p.out = (T*)B.t;
    p.b = (const T*)B.b;
    p.r = (T*)B.r;
    p.eps = eps_of<T>(B);
    p.ec = C ? (const T*)C->u : nullptr;
    p.A = B.A;
    p.P = B.P;
    p.omega = (T)g->opts.omega;
    p.pro = (first && C) ? 1 : 0;
    p.nsw = k;
    p.res = (last && residual) ? 1 : 0;
    p.zero_first = (first && zero_init) ? 1 : 0;
    p.partial = last ? partial : nullptr;
    const bool timed = finest && first && (g->prof_count++ % g->prof_every) == 0;
    hipEvent_t* ev = timed ? prof_pair(g) : nullptr;
    launch_pass2d<T>(p, S(g), ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
    std::swap(B.u, B.t);
    left -= k;
    first = false;
  }
}

template <typename T>
void vcycle_ad(qmg_grid_t* g, int l);

// One V-cycle from level l.  With want_norm on the finest regular 2D level,
// the last post-smoothing pass also leaves the residual norm partials of the
// new iterate in g->partial (returns true).
template <typename T>
bool vcycle(qmg_grid_t* g, int l, bool zero_init, bool want_norm = false) {
  if (l > g->lb) {
    vcycle_ad<T>(g, l);
    return false;
  }
  LevelBuf& F = g->lv[l];
  const int mu = g->opts.mu_pre, nu = g->opts.mu_post;
  if (l == g->lf && l < g->Lmax && zero_init) {
    fused_coarse<T>(g);
    return false;
  }
  if (l == g->lc) {
    if (g->coarse_direct)
      launch_coarse_solve<T>(F.L, g->Ainv, g->nc, (const T*)F.b, (T*)F.u, S(g));
    else
      smooth<T>(g, F, mu + nu, zero_init);
    return false;
  }
  LevelBuf& Cb = g->lv[l - 1];
  if (g->d == 2 && g->opts.smoother == QMG_SMOOTH_JACOBI) {  // fused passes
    passes<T>(g, F, nullptr, mu, zero_init, true, nullptr);
    restrict_to<T>(g, F, Cb, (const T*)F.r, (T*)Cb.b);
    vcycle<T>(g, l - 1, true);
    const bool norm = want_norm && l == g->Lmax;
    passes<T>(g, F, &Cb, nu, false, norm, norm ? (g->norm_dst ? g->norm_dst : g->partial) : nullptr);
    return norm;
  }
  smooth<T>(g, F, mu, zero_init);
  launch_stencil<T>(F.L, 2, (const T*)F.u, (const T*)F.b, (T*)F.r, eps_of<T>(F), F.A, (T)0, nullptr,
                    nullptr, S(g));
  LevelBuf& C = g->lv[l - 1];
  restrict_to<T>(g, F, C, (const T*)F.r, (T*)C.b);
  vcycle<T>(g, l - 1, true);
  launch_prolong<T>(F.L, C.L, (const T*)C.u, (T*)F.u, F.P, S(g));
  smooth<T>(g, F, nu, false);
  return false;
}

// Smoothing sweeps of an adaptive level over its leaf and refined vertices.
template <typename T>
void smooth_ad(qmg_grid_t* g, LevelBuf& B, int sweeps) {
  const T om = (T)g->opts.omega;
  const AdTiles t = B.ad();
  const bool finest = g->prof_every > 0 && B.L.n == g->lv[g->Lmax].L.n;
  for (int k = 0; k < sweeps; ++k) {
    // timed: every k-th sweep of the finest adaptive level
    const bool timed = finest && (g->prof_count++ % g->prof_every) == 0;
    hipEvent_t* ev = timed ? prof_pair(g) : nullptr;
    launch_ad_stencil<T, T>(t, 0, (const T*)B.u, (const T*)B.b, (T*)B.t, eps_of<T>(B), B.A, om, nullptr, S(g),
                            ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
    std::swap(B.u, B.t);
  }
}

// FAS V-cycle step on an adaptive level (Sect. 3): hanging vertices take the
// interpolant of the coarser level, the leaf and refined vertices are
// smoothed, refined coarse vertices receive the finer values (injection) and
// the FAS right-hand side R r + A_c I u (R = P^T), the coarse level is
// cycled, and the change of the coarse iterate is prolongated (P: d-linear or
// BoxMG, which also gives the hanging values).  The complete base level
// continues with the correction-scheme cycle.
template <typename T>
void vcycle_ad(qmg_grid_t* g, int l) {
  LevelBuf& F = g->lv[l];
  LevelBuf& C = g->lv[l - 1];
  const AdTiles tf = F.ad(), tc = C.ad();
  launch_ad_hang<T>(tf, C.L, (T*)F.u, (const T*)C.u, F.P, S(g));
  smooth_ad<T>(g, F, g->opts.mu_pre);
  launch_ad_stencil<T, T>(tf, 2, (const T*)F.u, (const T*)F.b, (T*)F.r, eps_of<T>(F), F.A, (T)0, nullptr, S(g));
  launch_ad_inject<T>(tc, F.L, (const T*)F.u, (T*)C.u, S(g));
  launch_ad_copy<T>(tc, (const T*)C.u, (T*)C.sv, S(g));
  launch_ad_fas_rhs<T>(tc, F.L, (const T*)F.r, (const T*)C.u, eps_of<T>(C), C.A, (T*)C.b, F.P, S(g), C.rv,
                       C.nrv, C.rc, C.nrc, (T*)C.rpart);
  vcycle<T>(g, l - 1, false);
  launch_ad_correct<T>(tf, C.L, (T*)F.u, (const T*)C.u, (const T*)C.sv, F.P, S(g));
  launch_ad_hang<T>(tf, C.L, (T*)F.u, (const T*)C.u, F.P, S(g));
  smooth_ad<T>(g, F, g->opts.mu_post);
}

// Refined vertices take their finest copy (top down), then hanging vertices
// the interpolant of the level below (bottom up).
// (on the FP64 solution x64 of every level when the iterates are FP32, on the
// iterates themselves otherwise)
template <typename T>
void composite_state_of(qmg_grid_t* g, T* (*field)(LevelBuf&)) {
  for (int l = g->Lmax; l > g->lb; --l)
    launch_ad_inject<T>(g->lv[l - 1].ad(), g->lv[l].L, field(g->lv[l]), field(g->lv[l - 1]), S(g));
  for (int l = g->lb + 1; l <= g->Lmax; ++l)
    launch_ad_hang<T>(g->lv[l].ad(), g->lv[l - 1].L, field(g->lv[l]), field(g->lv[l - 1]), g->lv[l].P, S(g));
}
double* iterate64(LevelBuf& B) { return (double*)B.u; }
float* iterate32(LevelBuf& B) { return (float*)B.u; }
double* solution64(LevelBuf& B) { return B.x64; }

void composite_state(qmg_grid_t* g) {
  if (g->mixed) composite_state_of<double>(g, solution64);
  else composite_state_of<double>(g, iterate64);
}

int64_t updates_per_cycle(const qmg_grid_t* g) {
  int64_t s = 0;
  // additive and BPX cycles: one Jacobi step per level
  const int sw = g->opts.cycle != QMG_CYCLE_MULT ? 1 : g->opts.mu_pre + g->opts.mu_post;
  for (int l = g->lc + 1; l <= g->Lmax; ++l)
    s += (int64_t)sw * (l > g->lb ? g->hl[l].n_active : n_interior(g->lv[l].L));
  if (!g->coarse_direct) s += (int64_t)sw * n_interior(g->lv[g->lc].L);
  return s;
}

double read_scalar(qmg_grid_t* g) {
  double h = 0.0;
  QMG_HIP(hipMemcpyAsync(&h, g->dscal, sizeof(double), hipMemcpyDeviceToHost, S(g)));
  QMG_HIP(hipStreamSynchronize(S(g)));
  return h;
}

// ||b - A u||_2 on the finest level, FP64 (the FP32 residual of the mixed loop
// is written to the finest inner right-hand side on the way).
// On an adaptive spacetree: the composite residual over the leaves of every
// level, after the refined and hanging values are made consistent.
// Residual norm partials of the finest level into `dst` (default: partial),
// then (sum) their reduction, recorded in the history when `record`.  Returns
// the number of partials.
int enqueue_residual_norm(qmg_grid_t* g, bool record, bool partials_ready = false, double* dst = nullptr,
                          bool sum = true) {
  LevelBuf& F = g->lv[g->Lmax];
  int np = 0;
  double* part = dst ? dst : g->partial;
  if (partials_ready) {  // left by the cycle's last fused pass
    np = pass2d_partials(F.L);
  } else if (g->adaptive && g->mixed) {
    // FP64 composite residual of x64 at the leaves (rediscretised leaf rows
    // from eps64); its FP32 rounding becomes the inner right-hand side
    composite_state(g);
    Store geom;
    for (int l = g->lb; l <= g->Lmax; ++l) {
      LevelBuf& B = g->lv[l];
      np += launch_ad_stencil<double, float>(B.ad(), 2, B.x64, B.b64, (float*)B.b, B.eps64, geom, 0.0,
                                             g->partial + np, S(g));
    }
  } else if (g->adaptive) {
    composite_state(g);
    for (int l = g->lb; l <= g->Lmax; ++l) {
      LevelBuf& B = g->lv[l];
      np += launch_ad_stencil<double, double>(B.ad(), 2, (const double*)B.u, (const double*)B.b, (double*)B.r,
                                              B.eps64, B.A, 0.0, g->partial + np, S(g));
    }
  } else if (g->mixed) {
    launch_residual_mixed(F.L, g->x64, g->bfin, (float*)F.b, F.eps64, part, &np, S(g));
  } else {
    launch_stencil<double>(F.L, 2, (const double*)F.u, (const double*)F.b, (double*)F.r, F.eps64,
                           F.A, 0.0, part, &np, S(g));
  }
  if (!sum) return np;
  if (record)
    launch_sum_partials(part, np, g->dscal, S(g), g->dhist, g->dctr, kHistCap);
  else
    launch_sum_partials(part, np, g->dscal, S(g));
  return np;
}

double finest_residual_norm(qmg_grid_t* g) {
  enqueue_residual_norm(g, false);
  return std::sqrt(read_scalar(g));
}

// One "cycle" of the public API: a V-cycle (FP64) or an outer defect-correction
// iteration with inner FP32 V-cycles (the residual has been formed already).
// Returns true when the cycle left the finest residual norm partials.
// Additive cycle (Alg. 2, unpipelined): r_L = b - A u restricted down to every
// level, one damped Jacobi step from zero per level (exact on a direct
// coarsest level), corrections summed coarse to fine, u += e_L.  The finest
// level's own correction is the Jacobi sweep from u.  BPX (Alg. 3) sums
// e_l = d_l + P (e_{l-1} - d_l at the c-points) instead.
template <typename T>
void additive_cycle(qmg_grid_t* g, bool zero_init) {
  const int L = g->Lmax, lc = g->lc;
  LevelBuf& F = g->lv[L];
  const double w = g->opts.omega;
  auto om = [&](int l) { return (T)(g->opts.damping == QMG_DAMP_EXP ? std::pow(w, L - l + 1) : w); };
  if (zero_init) launch_zero<T>((T*)F.u, F.L.nslot, S(g));
  launch_stencil<T>(F.L, 2, (const T*)F.u, (const T*)F.b, (T*)F.r, eps_of<T>(F), F.A, (T)0, nullptr, nullptr,
                    S(g));
  for (int l = L; l > lc; --l)
    launch_restrict<T>(g->lv[l].L, g->lv[l - 1].L, (const T*)g->lv[l].r, (T*)g->lv[l - 1].r, g->lv[l].P, S(g));
  LevelBuf& C = g->lv[lc];
  if (g->coarse_direct)
    launch_coarse_solve<T>(C.L, g->Ainv, g->nc, (const T*)C.r, (T*)C.u, S(g));
  else
    launch_stencil<T>(C.L, 1, (const T*)C.u, (const T*)C.r, (T*)C.u, eps_of<T>(C), C.A, om(lc), nullptr, nullptr,
                      S(g));
  const bool bpx = g->opts.cycle == QMG_CYCLE_BPX;
  for (int l = lc + 1; l < L; ++l) {
    LevelBuf& B = g->lv[l];
    LevelBuf& C1 = g->lv[l - 1];
    launch_stencil<T>(B.L, 1, (const T*)B.u, (const T*)B.r, (T*)B.u, eps_of<T>(B), B.A, om(l), nullptr, nullptr,
                      S(g));
    // BPX: the coarser correction replaces this level's step at the c-points
    if (bpx) launch_cpoint_sub<T>(B.L, C1.L, (const T*)B.u, (const T*)nullptr, (T*)C1.u, S(g));
    launch_prolong<T>(B.L, C1.L, (const T*)C1.u, (T*)B.u, B.P, S(g));
  }
  launch_stencil<T>(F.L, 0, (const T*)F.u, (const T*)F.b, (T*)F.t, eps_of<T>(F), F.A, om(L), nullptr, nullptr,
                    S(g));
  // the finest step is t - u
  if (bpx) launch_cpoint_sub<T>(F.L, g->lv[L - 1].L, (const T*)F.t, (const T*)F.u, (T*)g->lv[L - 1].u, S(g));
  launch_prolong<T>(F.L, g->lv[L - 1].L, (const T*)g->lv[L - 1].u, (T*)F.t, F.P, S(g));
  std::swap(F.u, F.t);
}

bool one_cycle(qmg_grid_t* g) {
  if (g->opts.cycle != QMG_CYCLE_MULT) {
    if (!g->mixed) {
      additive_cycle<double>(g, false);
      return false;
    }
    for (int m = 0; m < g->opts.inner_cycles; ++m) additive_cycle<float>(g, m == 0);
    launch_axpy_mixed(g->lv[g->Lmax].L, g->x64, (const float*)g->lv[g->Lmax].u, S(g));
    return false;
  }
  if (!g->mixed) return vcycle<double>(g, g->Lmax, false, true);
  if (g->adaptive) {
    // inner FAS cycles on the correction, from zero on every level
    for (int l = g->lcq; l <= g->Lmax; ++l) {
      LevelBuf& B = g->lv[l];
      if (l >= g->lb) launch_ad_zero<float>(B.ad(), (float*)B.u, S(g));
      else launch_zero<float>((float*)B.u, B.L.nslot, S(g));
    }
    for (int m = 0; m < g->opts.inner_cycles; ++m) {
      if (m > 0) composite_state_of<float>(g, iterate32);
      vcycle<float>(g, g->Lmax, false);
    }
    for (int l = g->lb; l <= g->Lmax; ++l) launch_ad_axpy(g->lv[l].ad(), g->lv[l].x64, (const float*)g->lv[l].u, S(g));
    return false;
  }
  for (int m = 0; m < g->opts.inner_cycles; ++m) vcycle<float>(g, g->Lmax, m == 0);
  launch_axpy_mixed(g->lv[g->Lmax].L, g->x64, (const float*)g->lv[g->Lmax].u, S(g));
  return false;
}

// one cycle followed by the recorded residual norm
void cycle_and_norm(qmg_grid_t* g) {
  const bool ready = one_cycle(g);
  enqueue_residual_norm(g, true, ready);
}

void drop_graph(qmg_grid_t* g) {
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  g->gexec = nullptr;
}

// Replaying one captured cycle needs every level to end a cycle in the buffer
// it started from, i.e. an even number of sweeps per level.
bool graph_usable(const qmg_grid_t* g) {
  if (g->prof_every > 0 || !g->opts.use_graphs) return false;
  if (g->opts.cycle != QMG_CYCLE_MULT) return false;  // one buffer swap per cycle on the finest level
  const int mu = g->opts.mu_pre, nu = g->opts.mu_post;
  // single sweeps (3D, coarsest level, block Jacobi) and fused passes of two (2D)
  if (g->opts.smoother != QMG_SMOOTH_JACOBI) return (mu + nu) % 2 == 0;
  return (mu + nu) % 2 == 0 && ((mu + 1) / 2 + (nu + 1) / 2) % 2 == 0;
}

void ensure_graph(qmg_grid_t* g) {
  if (g->gexec) return;
  hipGraph_t graph = nullptr;
  QMG_HIP(hipStreamBeginCapture(S(g), hipStreamCaptureModeThreadLocal));
  try {
    cycle_and_norm(g);
  } catch (...) {
    hipGraph_t dummy = nullptr;
    (void)hipStreamEndCapture(S(g), &dummy);
    if (dummy) (void)hipGraphDestroy(dummy);
    throw;
  }
  QMG_HIP(hipStreamEndCapture(S(g), &graph));
  const hipError_t e = hipGraphInstantiate(&g->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    g->gexec = nullptr;
    throw HipError(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
}

// Enqueues B cycles, each followed by the finest residual norm recorded on the
// device, then the copy of the B squared norms to pinned host memory and an
// event; nothing waits.
void enqueue_batch(qmg_grid_t* g, int B) {
  if (B <= 0 || B > kHistCap) throw ApiError(QMG_EINVAL, "batch size out of range");
  launch_zero<int>(g->dctr, 1, S(g));
  if (graph_usable(g)) {
    ensure_graph(g);
    for (int c = 0; c < B; ++c) QMG_HIP(hipGraphLaunch(g->gexec, S(g)));
  } else if (defers_norms(g)) {
    // the residual norm partials of up to kDeferNorms cycles lie side by side
    // (left by the finest 2D pass or by the residual kernel); one launch
    // reduces them
    int done = 0;
    try {
      while (done < B) {
        const int chunk = std::min(B - done, kDeferNorms);
        int np = -1;
        for (int c = 0; c < chunk; ++c) {
          double* dst = g->partial + (int64_t)c * g->npart1;
          g->norm_dst = dst;
          const bool ready = one_cycle(g);
          const int npc = enqueue_residual_norm(g, true, ready, dst, false);
          if (npc > g->npart1 || (np >= 0 && npc != np))
            throw HipError("internal: residual norm partials do not fit their stride");
          np = npc;
        }
        launch_sum_partials_multi(g->partial, np, g->npart1, chunk, g->dscal, g->dhist + done, g->dctr,
                                  done + chunk, S(g));
        done += chunk;
      }
    } catch (...) {
      g->norm_dst = nullptr;
      throw;
    }
    g->norm_dst = nullptr;
  } else {
    for (int c = 0; c < B; ++c) cycle_and_norm(g);
  }
  QMG_HIP(hipMemcpyAsync(g->hnorm, g->dhist, (size_t)B * sizeof(double), hipMemcpyDeviceToHost, S(g)));
  QMG_HIP(hipEventRecord(g->bev, S(g)));
  g->inflight = B;
}

bool batch_ready(qmg_grid_t* g) {
  const hipError_t e = hipEventQuery(g->bev);
  if (e == hipSuccess) return true;
  if (e == hipErrorNotReady) return false;
  throw HipError(std::string("hipEventQuery: ") + hipGetErrorString(e));
}

// Waits for the batch in flight and returns its residual norms.
std::vector<double> collect_batch(qmg_grid_t* g) {
  QMG_HIP(hipEventSynchronize(g->bev));
  std::vector<double> out((size_t)g->inflight);
  for (int c = 0; c < g->inflight; ++c) out[c] = std::sqrt(g->hnorm[c]);
  g->inflight = 0;
  return out;
}

std::vector<double> run_batch(qmg_grid_t* g, int B) {
  enqueue_batch(g, B);
  return collect_batch(g);
}

// ---------------------------------------------------------------------------
// Build (Sect. 4.3 and 3.4; store of Sect. 5)
// ---------------------------------------------------------------------------
// marked: B's block flags of P already hold the BoxMG launch's marks (1 on
// the blocks its solve wrote, 0 elsewhere).
void encode(qmg_grid_t* g, LevelBuf& B, const Lat& Lc, bool is_P, const double* full, int slot, int fmt,
            bool marked = false) {
  int32_t* blk = is_P ? B.Pblk : B.Ablk;
  void* pay = is_P ? B.Ppay : B.Apay;
  int8_t* sc = is_P ? B.Pscale : B.Ascale;
  int64_t* off = is_P ? B.Poff : B.Aoff;
  const double eps_mf = fmt == BPA ? g->opts.eps_mf : 0.0;
  const int64_t unit = (int64_t)(is_P ? (1 << B.L.d) : ipow(3, B.L.d)) * kSeg;
  // adaptive levels above the base level: only their listed tiles hold
  // operators the cycles read, and there only the slots of the level's
  // vertices
  const bool tl = g->adaptive && B.tiles != nullptr && B.L.n > g->lv[g->lb].L.n;
  launch_delta_flags(B.L, Lc, is_P, full, B.eps64, blk, S(g), eps_mf, tl ? B.tiles : nullptr, tl ? B.ntiles : 0,
                     g->opts.eps_zero, tl ? B.vt : nullptr, marked && tl && is_P);
  launch_scan_blocks(blk, B.L.nslot / kSeg, g->dtotal + slot, S(g), off, unit, g->scan_tmp);
  launch_delta_write(B.L, Lc, is_P, fmt, full, B.eps64, blk, pay, sc, S(g), off, eps_mf, tl ? B.tiles : nullptr,
                     tl ? B.ntiles : 0, tl ? B.vt : nullptr);
}

// The coarsest solve (a10): a dense inverse of the level's FP64 operator,
// assembled and inverted on the device (Gauss-Jordan with partial pivoting,
// one workgroup), when the level has at most kCoarseDirectMax unknowns and
// the exact solve is selected; otherwise the cycle smooths the level.  A
// singular operator is reported by check_coarse after the next
// synchronisation.
void setup_coarse(qmg_grid_t* g, const double* Afull) {
  LevelBuf& C = g->lv[g->lc];
  const int64_t n = n_interior(C.L);
  g->nc = (int)std::min<int64_t>(n, 1 << 30);
  g->coarse_direct = g->opts.coarse_solver == QMG_COARSE_DIRECT && n <= kCoarseDirectMax && n * n <= g->ainv_cap;
  if (!g->coarse_direct) return;
  launch_coarse_inverse(C.L, Afull, (int)n, g->Ainv, g->dcount + 4, S(g));
}

void check_coarse(qmg_grid_t* g) {
  if (!g->coarse_direct) return;
  int st = 0;
  QMG_HIP(hipMemcpyAsync(&st, g->dcount + 4, sizeof(int), hipMemcpyDeviceToHost, S(g)));
  QMG_HIP(hipStreamSynchronize(S(g)));
  if (st != 0) throw ApiError(QMG_EINDEF, "singular coarsest operator");
}

void assign_stores(qmg_grid_t* g) {
  const bool galerkin = g->opts.transfer != QMG_GEOMETRIC;
  const bool boxmg = g->opts.transfer == QMG_BOXMG;
  const int d = g->d;
  for (int l = g->lcq; l <= g->Lmax; ++l) {
    LevelBuf& B = g->lv[l];
    B.A = Store{};
    B.P = Store{};
    B.A.nent = ipow(3, d);
    B.P.nent = 1 << d;
    if (g->plain) {
      B.A.src = SRC_PLAIN;
      B.A.dense = B.Adense;
      B.P.src = SRC_PLAIN;
      B.P.dense = B.Pdense;
      continue;
    }
    if (galerkin && l < g->Lmax && B.Ablk) {
      B.A.src = SRC_HIER;
      B.A.fmt = g->fmt;
      B.A.blk = B.Ablk;
      B.A.payload = B.Apay;
      B.A.scale = B.Ascale;
      B.A.boff = B.Aoff;
    }
    if (boxmg && B.Pblk) {
      B.P.src = SRC_HIER;
      B.P.fmt = p_fmt(g, l);
      B.P.blk = B.Pblk;
      B.P.payload = B.Ppay;
      B.P.scale = B.Pscale;
      B.P.boff = B.Poff;
    }
  }
}

void build(qmg_grid_t* g, qmg_solve_report* info) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!g->have_coef) throw ApiError(QMG_ESTATE, "set_coefficients must precede build_operators");
  drop_graph(g);
  const int L = g->Lmax, d = g->d, NS = ipow(3, d), NC = 1 << d;
  const bool galerkin = g->opts.transfer != QMG_GEOMETRIC;
  const bool boxmg = g->opts.transfer == QMG_BOXMG;
  hipStream_t s = S(g);
  // cell coefficients of coarser levels: means of the children (refined cells
  // of the adaptive levels, every cell from the base level down)
  for (int l = L; l > g->lcq; --l) {
    if (l > g->lb)
      launch_ad_coarsen_eps(g->lv[l].L, g->lv[l - 1].L, g->lv[l - 1].cref, g->lv[l].eps64, g->lv[l - 1].eps64, s);
    else
      launch_coarsen_eps(g->lv[l].L, g->lv[l - 1].L, g->lv[l].eps64, g->lv[l - 1].eps64, s);
  }
  // BoxMG on adaptive levels: cells that do not exist carry their covering
  // cell's coefficient, from which hanging rows are rediscretised (with
  // mixed precision the same pass writes the single-precision copy)
  const bool virt = g->adaptive && boxmg;
  if (virt)
    for (int l = g->lb + 1; l <= L; ++l)
      launch_ad_virtual_eps(g->lv[l].L, g->lv[l - 1].L, g->lv[l - 1].cref, g->lv[l].vt, g->lv[l - 1].eps64,
                            g->lv[l].eps64, g->mixed ? g->lv[l].eps32 : nullptr, s);
  // single-precision coefficients; above the base level only the cells next
  // to a vertex of the level, which are all a row reads
  if (g->mixed)
    for (int l = g->lcq; l <= L; ++l) {
      if (g->adaptive && l > g->lb) {
        if (!virt) launch_ad_convert_cells(g->lv[l].L, g->lv[l].vt, g->lv[l].eps64, g->lv[l].eps32, s);
      } else {
        launch_convert<double, float>(g->lv[l].L, g->lv[l].eps64, g->lv[l].eps32, s);
      }
    }
  g->lc = g->lcq;
  assign_stores(g);  // views used by materialise below (plain stores)
  auto fullA = [&](int l) -> double* {
    if (g->plain) return g->lv[l].Adense;
    return g->tmpA[l & 1];
  };
  Store geom;
  // rows of an adaptive level: refined vertices keep the Galerkin (or
  // rediscretised) row, leaves take the rediscretised one, others none
  // (cleared: the other rows of the level's vertices hold zero already)
  auto merge = [&](int l, double* full, bool cleared) {
    if (g->adaptive && l >= g->lb) launch_ad_merge_rows(g->lv[l].L, g->lv[l].vt, g->lv[l].eps64, full, cleared, s);
  };
  if (g->plain) {
    launch_materialise(g->lv[L].L, g->lv[L].eps64, geom, g->lv[L].Adense, s);
    if (g->has_conv) launch_conv_add(g->lv[L].L, g->vel, g->lv[L].Adense, s);
    merge(L, g->lv[L].Adense, false);
  }
  for (int l = g->lcq; l <= L; ++l) {
    g->lv[l].Anz = -1;
    g->lv[l].Pnz = -1;
  }
  std::vector<int> encodedA, encodedP;
  int lc_used = g->lcq;
  for (int l = L; l > g->lcq; --l) {
    LevelBuf& F = g->lv[l];
    LevelBuf& C = g->lv[l - 1];
    const double* Afine = (l == L) ? (g->plain ? F.Adense : nullptr) : fullA(l);
    const double* Pw = nullptr;
    bool p_marked = false;
    if (boxmg) {
      double* Pt = g->plain ? F.Pdense : g->tmpP;
      const bool ad = g->adaptive && l > g->lb;
      // adaptive levels: every weight of the level's vertices (all the
      // encoder and the kernels read) is written by the BoxMG kernel itself
      if (!ad) launch_zero<double>(Pt, F.L.nslot * NC, s);
      // the finest level's rediscretised rows: the work stencil buffer of
      // level L (unused until the Galerkin product) holds the list of cells
      // whose patches need the solve
      void* bscr = (l == L && !Afine && !g->plain) ? (void*)g->tmpA[L & 1] : nullptr;
      const size_t bscr_bytes = bscr ? (size_t)NS * g->lv[L - 1].L.nslot * sizeof(double) : 0;
      // the prolongation's block flags collect the blocks the solve writes
      int32_t* dirty = (bscr && F.Pblk) ? F.Pblk : nullptr;
      if (dirty) launch_zero<int32_t>(dirty, F.L.nslot / kSeg, s);
      p_marked = launch_boxmg(F.L, C.L, Afine, F.eps64, Pt, s, ad ? F.vt : nullptr, ad ? C.cref : nullptr,
                              ad ? C.rc : nullptr, ad ? C.nrc : 0, bscr, bscr_bytes, dirty);
      Pw = Pt;
    } else if (g->plain) {
      Store dl;
      launch_materialise_P(F.L, C.L, dl, F.Pdense, s);
      Pw = F.Pdense;
    }
    double* Ac = fullA(l - 1);
    if (!galerkin) {
      // rediscretised coarse operator: stored only in the plain store, and
      // needed in full on the coarsest level for the exact solve
      if (g->plain || l - 1 == g->lcq) {
        launch_materialise(C.L, C.eps64, geom, Ac, s);
        merge(l - 1, Ac, false);
      }
    } else {
      // adaptive levels above the base: rows of the level's vertices only
      // (no kernel and not the encoder reads others)
      if (g->adaptive && l - 1 > g->lb) launch_ad_zero<double>(C.ad(), Ac, s, NS, true);
      else launch_zero<double>(Ac, C.L.nslot * NS, s);
      // the finest adaptive level's rows exist only at leaf vertices
      const int8_t* mask = (g->adaptive && l == L && !Afine) ? F.vt : nullptr;
      const bool adc = g->adaptive && l - 1 >= g->lb;
      // the finest 3D adaptive level: coarse cell by coarse cell, with the
      // element matrices in the unused work stencil buffer of level L
      bool by_cells = false;
      if (g->d == 3 && adc && l == L && !Afine && g->opts.restriction == QMG_R_TRANSPOSE)
        by_cells = launch_rap_cells(F.L, C.L, F.eps64, Pw, Ac, s, mask, C.vt, C.rv, C.nrv, C.rc, C.nrc,
                                    g->tmpA[L & 1], (size_t)NS * g->lv[L - 1].L.nslot * sizeof(double));
      if (!by_cells)
        launch_rap(F.L, C.L, Afine, F.eps64, Pw, Ac, s, mask, adc ? C.vt : nullptr, adc ? C.rv : nullptr,
                   adc ? C.nrv : 0, g->opts.restriction);
      // the products write the listed refined rows only, over zero
      merge(l - 1, Ac, true);
      // the fallback of a failed check raises the coarsest level, which is
      // possible only below the base level of an adaptive spacetree
      if (g->opts.check_definite && l - 1 < g->lb) {
        launch_zero<int>(g->dcount, 1, s);
        launch_check_rows(C.L, Ac, g->dcount, s);
        int bad = 0;
        QMG_HIP(hipMemcpyAsync(&bad, g->dcount, sizeof(int), hipMemcpyDeviceToHost, s));
        QMG_HIP(hipStreamSynchronize(s));
        if (bad > 0) {
          lc_used = l;
          break;
        }
      }
    }
    if (!g->plain) {
      if (boxmg) {
        encode(g, F, C.L, true, Pw, 2 * l + 1, p_fmt(g, l), p_marked);
        encodedP.push_back(l);
      }
      if (galerkin) {
        encode(g, C, C.L, false, Ac, 2 * (l - 1), g->fmt);
        encodedA.push_back(l - 1);
      }
    }
    lc_used = l - 1;
  }
  if (lc_used >= L) throw ApiError(QMG_EINDEF, "every Galerkin coarse operator failed the definiteness check");
  g->lc = lc_used;
  // stored-operator bookkeeping
  std::vector<int32_t> tot(2 * (L + 1), 0);
  QMG_HIP(hipMemcpyAsync(tot.data(), g->dtotal, tot.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  QMG_HIP(hipStreamSynchronize(s));
  size_t bytes = 0;
  int64_t blocks = 0, zero_blocks = 0;
  // BPA blocks vary in width: the payload ends where the last block does
  auto bpa_bytes = [&](const int64_t* off, int64_t n, int nent) -> size_t {
    if (n <= 0) return 0;
    int64_t ow = 0;
    QMG_HIP(hipMemcpyAsync(&ow, off + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QMG_HIP(hipStreamSynchronize(s));
    return (size_t)(ow & ((int64_t(1) << 56) - 1)) + (size_t)nent * kSeg * (size_t)(ow >> 56) + (size_t)n * 8;
  };
  for (int l : encodedA) {
    g->lv[l].Anz = tot[2 * l];
    const int64_t nb = g->lv[l].L.nslot / kSeg;
    blocks += nb;
    zero_blocks += nb - tot[2 * l];
    bytes += (size_t)nb * 4;
    if (g->fmt == BPA) bytes += bpa_bytes(g->lv[l].Aoff, tot[2 * l], NS);
    else bytes += (size_t)tot[2 * l] * kSeg * (NS * fmt_size(g->fmt) + (g->fmt == F16 ? 1 : 0));
  }
  for (int l : encodedP) {
    g->lv[l].Pnz = tot[2 * l + 1];
    const int64_t nb = g->lv[l].L.nslot / kSeg;
    blocks += nb;
    zero_blocks += nb - tot[2 * l + 1];
    const int pf = p_fmt(g, l);
    bytes += (size_t)nb * 4;
    if (pf == BPA) bytes += bpa_bytes(g->lv[l].Poff, tot[2 * l + 1], NC);
    else bytes += (size_t)tot[2 * l + 1] * kSeg * (NC * fmt_size(pf) + (pf == F16 ? 1 : 0));
  }
  if (g->plain) {
    for (int l = g->lc; l <= L; ++l) bytes += (size_t)g->lv[l].L.nslot * NS * 8;
    for (int l = g->lc + 1; l <= L; ++l) bytes += (size_t)g->lv[l].L.nslot * NC * 8;
  }
  g->bytes_ops = bytes;
  g->zero_frac = blocks ? (double)zero_blocks / (double)blocks : 1.0;
  // levels coarser than lc are unused; the coarsest level's own stencil is
  // the FP64 Galerkin (or rediscretised) operator
  assign_stores(g);
  for (int l = g->lcq; l < g->lc; ++l) {
    g->lv[l].A = Store{};
    g->lv[l].P = Store{};
  }
  g->lv[g->lc].P = Store{};
  double* Alc = fullA(g->lc);
  if (!galerkin && !g->plain && g->lc == L) launch_materialise(g->lv[L].L, g->lv[L].eps64, geom, Alc, s);
  setup_coarse(g, Alc);
  {
    int dev = 0, optin = 0;
    QMG_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && optin > 0)
      g->lds_max = optin;
    else
      (void)hipGetLastError();
  }
  g->lf = g->mixed ? choose_fused_top<float>(g, g->lf_pw_lds) : choose_fused_top<double>(g, g->lf_pw_lds);
  g->fimg_ready = false;
  if (g->lf >= 0) {
    if (g->mixed) prepare_fused<float>(g);
    else prepare_fused<double>(g);
  }
  check_coarse(g);
  g->have_ops = true;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->coarsest_level_used = g->lc;
    info->bytes_operators = g->bytes_ops;
    info->zero_delta_fraction = g->zero_frac;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
}

// Dynamic coarsest level (Sect. 4.3): moves l_c one level up, to L - 1 at
// most (the base level on an adaptive grid).  The new coarsest level's stored
// operator is decoded to FP64 for its exact solve (or it is smoothed when too
// large); the levels below drop out of the cycle.  Returns whether it moved.
bool raise_coarsest(qmg_grid_t* g) {
  const int top = g->adaptive ? std::min(g->lb, g->Lmax - 1) : g->Lmax - 1;
  if (g->lc + 1 > top) return false;
  drop_graph(g);
  const int l = g->lc + 1;
  LevelBuf& B = g->lv[l];
  double* full = B.Adense;
  if (!g->plain) {
    full = g->tmpA[0];  // sized for level L - 1
    launch_materialise(B.L, B.eps64, B.A, full, S(g));
  }
  g->lv[g->lc].A = Store{};
  g->lv[g->lc].P = Store{};
  g->lc = l;
  B.P = Store{};
  setup_coarse(g, full);
  g->lf = g->mixed ? choose_fused_top<float>(g, g->lf_pw_lds) : choose_fused_top<double>(g, g->lf_pw_lds);
  g->fimg_ready = false;
  if (g->lf >= 0) {
    if (g->mixed) prepare_fused<float>(g);
    else prepare_fused<double>(g);
  }
  QMG_HIP(hipStreamSynchronize(S(g)));
  check_coarse(g);
  return true;
}

void need_ops(qmg_grid_t* g) {
  if (!g) throw ApiError(QMG_EINVAL, "null grid");
  if (!g->have_ops) throw ApiError(QMG_ESTATE, "build_operators must precede cycles");
}

void copy_in(qmg_grid_t* g, double* dst_dev, const double* src, int64_t n, int mem) {
  QMG_HIP(hipMemcpyAsync(dst_dev, src, n * sizeof(double),
                         mem == QMG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, S(g)));
}

// Device array the input checks read: the caller's own for device memory,
// else the staging buffer after a copy from the host.
const double* input_on_device(qmg_grid_t* g, const double* src, int64_t n, int mem) {
  if (mem == QMG_DEVICE) return src;
  copy_in(g, g->stage, src, n, mem);
  return g->stage;
}

// Lattice arrays in host inspection calls have (n+1)^d values without padding.
std::vector<double> unpitch(const Lat& L, const std::vector<double>& h, int nent) {
  const int64_t w = L.n + 1;
  const int64_t per = L.d == 3 ? w * w * w : w * w;
  std::vector<double> out((size_t)nent * per);
  for (int e = 0; e < nent; ++e)
    for (int64_t k = 0; k < (L.d == 3 ? w : 1); ++k)
      for (int64_t j = 0; j < w; ++j)
        for (int64_t i = 0; i < w; ++i)
          out[(size_t)e * per + i + w * (j + w * k)] = h[(size_t)e * L.nslot + i + j * L.pitch + k * L.plane];
  return out;
}

std::vector<double> pitch_in(const Lat& L, const double* a) {
  const int64_t w = L.n + 1;
  std::vector<double> out((size_t)L.nslot, 0.0);
  for (int64_t k = 0; k < (L.d == 3 ? w : 1); ++k)
    for (int64_t j = 0; j < w; ++j)
      for (int64_t i = 0; i < w; ++i) out[(size_t)(i + j * L.pitch + k * L.plane)] = a[i + w * (j + w * k)];
  return out;
}

template <typename T>
void upload_lattice(qmg_grid_t* g, const Lat& L, const double* host, T* dst) {
  std::vector<double> p = pitch_in(L, host);
  QMG_HIP(hipMemcpyAsync(g->stage, p.data(), p.size() * sizeof(double), hipMemcpyHostToDevice, S(g)));
  if (sizeof(T) == sizeof(double))
    QMG_HIP(hipMemcpyAsync(dst, g->stage, p.size() * sizeof(double), hipMemcpyDeviceToDevice, S(g)));
  else
    launch_convert<double, float>(L, g->stage, (float*)dst, S(g));
  QMG_HIP(hipStreamSynchronize(S(g)));
}

template <typename T>
void download_lattice(qmg_grid_t* g, const Lat& L, const T* src, double* host) {
  if (sizeof(T) == sizeof(double))
    QMG_HIP(hipMemcpyAsync(g->stage, src, L.nslot * sizeof(double), hipMemcpyDeviceToDevice, S(g)));
  else
    launch_convert<float, double>(L, (const float*)src, g->stage, S(g));
  std::vector<double> h((size_t)L.nslot);
  QMG_HIP(hipMemcpyAsync(h.data(), g->stage, h.size() * sizeof(double), hipMemcpyDeviceToHost, S(g)));
  QMG_HIP(hipStreamSynchronize(S(g)));
  std::vector<double> o = unpitch(L, h, 1);
  std::memcpy(host, o.data(), o.size() * sizeof(double));
}

template <typename T>
void apply_op(qmg_grid_t* g, int op, int level, const double* x, const double* b, double* out) {
  if (level < g->lc || level > g->Lmax) throw ApiError(QMG_EINVAL, "level outside the built hierarchy");
  LevelBuf& B = g->lv[level];
  const T om = (T)g->opts.omega;
  if (op == QMG_OP_RESTRICT || op == QMG_OP_PROLONG) {
    if (level <= g->lc) throw ApiError(QMG_EINVAL, "transfer needs level > coarsest level");
    LevelBuf& C = g->lv[level - 1];
    if (op == QMG_OP_RESTRICT) {
      upload_lattice<T>(g, B.L, x, (T*)B.r);
      launch_zero<T>((T*)C.b, C.L.nslot, S(g));
      restrict_to<T>(g, B, C, (const T*)B.r, (T*)C.b);
      download_lattice<T>(g, C.L, (const T*)C.b, out);
    } else {
      upload_lattice<T>(g, C.L, x, (T*)C.u);
      if (b) upload_lattice<T>(g, B.L, b, (T*)B.u);
      else launch_zero<T>((T*)B.u, B.L.nslot, S(g));
      launch_prolong<T>(B.L, C.L, (const T*)C.u, (T*)B.u, B.P, S(g));
      download_lattice<T>(g, B.L, (const T*)B.u, out);
    }
    return;
  }
  // a missing x (Jacobi only) is the sweep from a zero iterate
  if (x) upload_lattice<T>(g, B.L, x, (T*)B.u);
  else launch_zero<T>((T*)B.u, B.L.nslot, S(g));
  if (b) upload_lattice<T>(g, B.L, b, (T*)B.b);
  else launch_zero<T>((T*)B.b, B.L.nslot, S(g));
  launch_zero<T>((T*)B.t, B.L.nslot, S(g));
  if (op == QMG_OP_SMOOTH) {  // one step of the grid's smoother (result in B.u)
    smooth<T>(g, B, 1, false);
    download_lattice<T>(g, B.L, (const T*)B.u, out);
    return;
  }
  const int mode = op == QMG_OP_MATVEC ? 3 : op == QMG_OP_RESIDUAL ? 2 : x ? 0 : 1;
  launch_stencil<T>(B.L, mode, (const T*)B.u, (const T*)B.b, (T*)B.t, eps_of<T>(B), B.A, om, nullptr,
                    nullptr, S(g));
  download_lattice<T>(g, B.L, (const T*)B.t, out);
}

// position of a lattice slot (+ offset in units of h) on level l
void slot_xyz(const Lat& L, int64_t sl, double off, double* out) {
  const int64_t k = L.d == 3 ? sl / L.plane : 0, rem = sl - k * L.plane;
  out[0] = ((double)(rem % L.pitch) + off) * L.h;
  out[1] = ((double)(rem / L.pitch) + off) * L.h;
  if (L.d == 3) out[2] = ((double)k + off) * L.h;
}

}  // namespace

// ---------------------------------------------------------------------------
// Solve loop as a state machine (used blocking by qmg_solve and polled by the
// server).  Cycles run in batches between host synchronisations; the batch
// length follows the observed convergence factor so that the tolerance is
// reached in the last cycle of a batch (a batch is never cut short: cycles
// after the crossing are kept and counted).
// ---------------------------------------------------------------------------
namespace qmg {

void solve_begin(qmg_grid_t* g, SolveState& st, double tol, int max_cycles) {
  need_ops(g);
  if (max_cycles < 0 || !(tol >= 0.0)) throw ApiError(QMG_EINVAL, "bad tolerance or cycle limit");
  st = SolveState{};
  st.tol = tol;
  st.max_cycles = max_cycles;
  st.t0 = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  st.rr = (g->bnorm > 0) ? finest_residual_norm(g) / g->bnorm : 0.0;
  st.outer = 1;
  st.done = !(st.rr > tol) || max_cycles == 0;
}

void solve_enqueue(qmg_grid_t* g, SolveState& st) {
  // the stagnation check needs the residual of every cycle before the next
  const int B = g->opts.stagnation > 0.0 ? 1 : std::max(1, std::min({st.batch, st.max_cycles - st.cycles, kHistCap}));
  enqueue_batch(g, B);
}

bool solve_ready(qmg_grid_t* g) { return batch_ready(g); }

void solve_collect(qmg_grid_t* g, SolveState& st) {
  const int B = g->inflight;
  const std::vector<double> nr = collect_batch(g);
  for (int c = 0; c < B; ++c) st.history.push_back(nr[c] / g->bnorm);
  st.cycles += B;
  st.outer += B;
  st.rr_prev = st.rr;
  st.rr = nr[B - 1] / g->bnorm;
  const double rho = (st.rr > 0 && st.rr_prev > 0) ? std::pow(st.rr / st.rr_prev, 1.0 / B) : 0.0;
  if (rho > 0.0 && rho < 1.0 && st.rr > st.tol) {
    // half the predicted remainder: multigrid factors often improve over the
    // first cycles, so a full prediction would overshoot
    const double need = std::log(st.tol / st.rr) / std::log(rho);
    st.batch = std::max(1, std::min((int)std::floor(0.5 * need), 64));
  } else {
    st.batch = 1;
  }
  st.done = !(st.rr > st.tol) || st.cycles >= st.max_cycles || !std::isfinite(st.rr);
  if (!st.done && g->opts.stagnation > 0.0 && st.rr > g->opts.stagnation * st.rr_prev) raise_coarsest(g);
}

void solve_fill_report(qmg_grid_t* g, const SolveState& st, qmg_solve_report* rep) {
  if (!rep) return;
  std::memset(rep, 0, sizeof(*rep));
  const int inner = g->mixed ? g->opts.inner_cycles : 1;
  rep->cycles = st.cycles * inner;
  rep->outer_iters = st.outer;
  rep->relres = st.rr;
  rep->coarsest_level_used = g->lc;
  rep->vertex_updates = (int64_t)st.cycles * inner * updates_per_cycle(g);
  rep->bytes_operators = g->bytes_ops;
  rep->zero_delta_fraction = g->zero_frac;
  rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count() - st.t0;
}

}  // namespace qmg

namespace qmg {

int create_grid(const qmg_grid_desc* desc, const qmg_solver_opts* opts, void* device_buf, size_t bytes,
                void* stream, double* pinned_hist, qmg_grid_t** out) {
  return guard(nullptr, [&] {
    validate(desc, opts);
    if (!out) throw ApiError(QMG_EINVAL, "null output handle");
    *out = nullptr;
    qmg_grid_t* g = new qmg_grid_t();
    try {
      init_modes(g, desc, opts);
      g->stream = (hipStream_t)stream;
      if (g->stream == nullptr) {  // graph capture needs a stream other than the null stream
        QMG_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
        g->own_stream = true;
      }
      Arena probe;
      layout(g, probe);
      const size_t need = probe.off + 256;
      if (device_buf) {
        if (bytes < need)
          throw ApiError(QMG_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
        g->base = (char*)device_buf;
        g->bytes = bytes;
      } else {
        void* p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess) {
          (void)hipGetLastError();
          throw ApiError(QMG_ENOMEM, "device allocation of " + std::to_string(need) + " bytes failed");
        }
        g->base = (char*)p;
        g->bytes = need;
        g->owns = true;
      }
      Arena a;
      a.base = (char*)(((uintptr_t)g->base + 255) & ~(uintptr_t)255);
      layout(g, a);
      QMG_HIP(hipMemsetAsync(g->base, 0, need, g->stream));
      if (pinned_hist) {
        g->hnorm = pinned_hist;
        g->own_hnorm = false;
      } else {
        QMG_HIP(hipHostMalloc((void**)&g->hnorm, kHistCap * sizeof(double), hipHostMallocDefault));
      }
      QMG_HIP(hipEventCreateWithFlags(&g->bev, hipEventDisableTiming));
      QMG_HIP(hipStreamSynchronize(g->stream));
      g->n_unknowns = n_interior(g->lv[g->Lmax].L);
      upload_linearisation(g);
    } catch (...) {
      if (g->owns && g->base) (void)hipFree(g->base);
      if (g->vel) (void)hipFree(g->vel);
      if (g->rscr) (void)hipFree(g->rscr);
      if (g->hnorm && g->own_hnorm) (void)hipHostFree(g->hnorm);
      if (g->bev) (void)hipEventDestroy(g->bev);
      if (g->own_stream) (void)hipStreamDestroy(g->stream);
      delete g;
      throw;
    }
    *out = g;
  });
}

}  // namespace qmg

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* qmg_version(void) { return "qmg-mi355x 0.1 (gfx950)"; }

int qmg_default_opts(qmg_solver_opts* o) {
  if (!o) return QMG_EINVAL;
  o->transfer = QMG_BOXMG;
  o->store = QMG_HIER_FP64;
  o->mu_pre = 2;
  o->mu_post = 2;
  o->omega = 0.6;
  o->coarsest_level = 1;
  o->check_definite = 1;
  o->inner_cycles = 1;
  o->use_graphs = 1;
  o->stagnation = 0.0;
  o->smoother = QMG_SMOOTH_JACOBI;
  o->bj_sweeps = 1;
  o->cycle = QMG_CYCLE_MULT;
  o->damping = QMG_DAMP_EXP;
  o->eps_mf = 1e-8;
  o->restriction = QMG_R_TRANSPOSE;
  o->coarse_solver = QMG_COARSE_DIRECT;
  o->eps_zero = 0.0;
  o->iterate = QMG_IT_STORE;
  return QMG_OK;
}

int qmg_workspace_bytes(const qmg_grid_desc* desc, const qmg_solver_opts* opts, size_t* bytes) {
  return guard(nullptr, [&] {
    validate(desc, opts);
    if (!bytes) throw ApiError(QMG_EINVAL, "null bytes");
    qmg_grid_t g;
    init_modes(&g, desc, opts);
    Arena a;
    layout(&g, a);
    *bytes = a.off + 256;
  });
}

int qmg_region_flags(const qmg_grid_desc* desc, uint8_t* flags, int64_t n_flags) {
  return guard(nullptr, [&] {
    if (!desc || !flags) throw ApiError(QMG_EINVAL, "null argument");
    qmg_solver_opts o{};
    qmg_default_opts(&o);
    validate(desc, &o);
    if (desc->base_level == 0 || desc->base_level == desc->max_level)
      throw ApiError(QMG_EINVAL, "refinement flags belong to an adaptive grid");
    int64_t total = 0;
    for (int l = desc->base_level; l < desc->max_level; ++l)
      total += (int64_t)std::llround(std::pow(3.0, (double)l * desc->dim));
    if (n_flags != total) throw ApiError(QMG_EINVAL, "flags must hold " + std::to_string(total) + " bytes");
    const std::vector<uint8_t> f = refine_flags(desc);
    std::memcpy(flags, f.data(), (size_t)total);
  });
}

int qmg_create_grid(const qmg_grid_desc* desc, const qmg_solver_opts* opts, void* device_buf,
                    size_t bytes, void* stream, qmg_grid_t** out) {
  return qmg::create_grid(desc, opts, device_buf, bytes, stream, nullptr, out);
}

int qmg_sizes(const qmg_grid_t* g, int64_t* n_unknowns, int64_t* n_leaf_cells, int* n_levels) {
  if (!g) return QMG_EINVAL;
  const Lat& L = g->lv[g->Lmax].L;
  if (n_unknowns) *n_unknowns = g->n_unknowns;
  if (n_leaf_cells) *n_leaf_cells = g->adaptive ? g->n_cells : g->d == 3 ? (int64_t)L.n * L.n * L.n : (int64_t)L.n * L.n;
  if (n_levels) *n_levels = g->Lmax + 1;
  return QMG_OK;
}

int qmg_unknown_coords(const qmg_grid_t* g, double* xyz, int8_t* level) {
  if (!g || !xyz) return QMG_EINVAL;
  if (g->adaptive) {
    int64_t r = 0;
    for (int l = g->lb; l <= g->Lmax; ++l)
      for (int64_t sl : g->hl[l].leaf) {
        slot_xyz(g->lv[l].L, sl, 0.0, xyz + r * g->d);
        if (level) level[r] = (int8_t)l;
        ++r;
      }
    return QMG_OK;
  }
  const Lat& L = g->lv[g->Lmax].L;
  const int m = L.n - 1;
  for (int64_t r = 0; r < g->n_unknowns; ++r) {
    xyz[r * g->d + 0] = (double)(r % m + 1) * L.h;
    xyz[r * g->d + 1] = (double)((r / m) % m + 1) * L.h;
    if (g->d == 3) xyz[r * g->d + 2] = (double)(r / ((int64_t)m * m) + 1) * L.h;
    if (level) level[r] = (int8_t)g->Lmax;
  }
  return QMG_OK;
}

int qmg_leaf_cell_centres(const qmg_grid_t* g, double* xyz) {
  if (!g || !xyz) return QMG_EINVAL;
  if (g->adaptive) {
    int64_t r = 0;
    for (int l = g->lb; l <= g->Lmax; ++l)
      for (int64_t sl : g->hl[l].cells) slot_xyz(g->lv[l].L, sl, 0.5, xyz + (r++) * g->d);
    return QMG_OK;
  }
  const Lat& L = g->lv[g->Lmax].L;
  const int64_t n = L.n, nc = g->d == 3 ? n * n * n : n * n;
  for (int64_t c = 0; c < nc; ++c) {
    xyz[c * g->d + 0] = ((double)(c % n) + 0.5) * L.h;
    xyz[c * g->d + 1] = ((double)((c / n) % n) + 0.5) * L.h;
    if (g->d == 3) xyz[c * g->d + 2] = ((double)(c / (n * n)) + 0.5) * L.h;
  }
  return QMG_OK;
}

int qmg_set_coefficients(qmg_grid_t* g, const double* eps, int ncomp, const double* f, int mem) {
  return guard(g, [&] {
    if (!g || !eps || !f) throw ApiError(QMG_EINVAL, "null argument");
    if (ncomp != 1 && ncomp != 1 + g->d)
      throw ApiError(QMG_EINVAL, "ncomp must be 1 (eps) or 1 + d (eps and the velocity components)");
    if (ncomp > 1 && (g->adaptive || !g->plain || g->opts.transfer == QMG_GEOMETRIC))
      throw ApiError(QMG_EINVAL, "convection needs a regular grid, the plain store and Galerkin coarse operators");
    if (mem != QMG_HOST && mem != QMG_DEVICE) throw ApiError(QMG_EINVAL, "bad mem flag");
    g->have_coef = false;
    g->have_ops = false;
    drop_graph(g);
    LevelBuf& F = g->lv[g->Lmax];
    const Lat& L = F.L;
    const int64_t ncell = g->adaptive ? g->n_cells : L.d == 3 ? (int64_t)L.n * L.n * L.n : (int64_t)L.n * L.n;
    const int64_t nu = g->n_unknowns;
    hipStream_t s = S(g);
    auto blocks = [&](int64_t n, int share) {
      return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, g->npart / share));
    };
    launch_zero<int>(g->dcount, 3, s);
    // cell coefficients: staged, checked on the device, scattered per level
    launch_prep_input(input_on_device(g, eps, ncell, mem), g->stage, ncell, 1.0, true, g->partial,
                      blocks(ncell, 1), g->dcount, s);
    if (g->adaptive) {
      int64_t co = 0;
      for (int l = g->lb; l <= g->Lmax; ++l) {
        LevelBuf& B = g->lv[l];
        const int64_t cnt = (int64_t)g->hl[l].cells.size();
        // later calls overwrite the leaf cells; refined cells are coarsened
        // and missing ones given their covering value by the build
        if (!g->lattices_clear) launch_zero<double>(B.eps64, B.L.nslot, s);
        launch_ad_scatter<double>(g->cell_slots + co, cnt, g->stage + co, 1.0, B.eps64, s);
        co += cnt;
      }
    } else {
      launch_scatter_cells<double>(L, g->stage, F.eps64, s);
    }
    // velocities (components 1..d): staged, checked finite, scattered
    g->has_conv = ncomp > 1;
    if (g->has_conv) {
      if (!g->vel) QMG_HIP(hipMalloc(&g->vel, (size_t)g->d * L.nslot * sizeof(double)));
      launch_zero<double>(g->vel, (int64_t)g->d * L.nslot, s);
      for (int c = 0; c < g->d; ++c) {
        launch_prep_input(input_on_device(g, eps + (int64_t)(1 + c) * ncell, ncell, mem), g->stage, ncell, 1.0,
                          false, g->partial, blocks(ncell, 1), g->dcount + 2, s);
        launch_scatter_cells<double>(L, g->stage, g->vel + (int64_t)c * L.nslot, s);
      }
    }
    // right-hand side b = h_l^d f of every unknown (level l), and its norm
    const double* fin = input_on_device(g, f, nu, mem);
    const int nlev = g->Lmax - g->lb + 1;
    int np = 0;
    int64_t off = 0;
    for (int l = g->lb; l <= g->Lmax; ++l) {
      double hd = 1.0;
      for (int i = 0; i < g->d; ++i) hd *= g->lv[l].L.h;
      const int64_t cnt = g->adaptive ? (int64_t)g->hl[l].leaf.size() : nu;
      const int nb = blocks(cnt, nlev);
      if (cnt > 0) {
        launch_prep_input(fin + off, g->stage + off, cnt, hd, false, g->partial + np, nb, g->dcount + 1, s);
        np += nb;
      }
      off += cnt;
    }
    launch_sum_partials(g->partial, np, g->dscal, s);
    if (g->adaptive) {
      int64_t uo = 0;
      for (int l = g->lcq; l <= g->Lmax; ++l) {
        LevelBuf& B = g->lv[l];
        // adaptive levels after the first call: the active tiles only
        const bool tiles_only = g->lattices_clear && l >= g->lb;
        for (void* v : {B.u, B.t, B.b}) {
          if (tiles_only && g->mixed) launch_ad_zero<float>(B.ad(), (float*)v, s);
          else if (tiles_only) launch_ad_zero<double>(B.ad(), (double*)v, s);
          else if (g->mixed) launch_zero<float>((float*)v, B.L.nslot, s);
          else launch_zero<double>((double*)v, B.L.nslot, s);
        }
        if (l < g->lb) continue;
        double* bdst = g->mixed ? B.b64 : (double*)B.b;
        if (g->mixed) {
          if (tiles_only) {
            launch_ad_zero<double>(B.ad(), B.x64, s);
            launch_ad_zero<double>(B.ad(), B.b64, s);
          } else {
            launch_zero<double>(B.x64, B.L.nslot, s);
            launch_zero<double>(B.b64, B.L.nslot, s);
          }
        }
        const int64_t cnt = (int64_t)g->hl[l].leaf.size();
        launch_ad_scatter<double>(g->unk_slots + uo, cnt, g->stage + uo, 1.0, bdst, s);
        uo += cnt;
      }
    } else if (g->mixed) {
      launch_scatter_unknowns<double>(L, g->stage, g->bfin, s);
      launch_zero<double>(g->x64, L.nslot, s);
    } else {
      launch_scatter_unknowns<double>(L, g->stage, (double*)F.b, s);
      launch_zero<double>((double*)F.u, L.nslot, s);
    }
    int bad[3] = {0, 0, 0};
    double b2 = 0.0;
    QMG_HIP(hipMemcpyAsync(bad, g->dcount, sizeof(bad), hipMemcpyDeviceToHost, s));
    QMG_HIP(hipMemcpyAsync(&b2, g->dscal, sizeof(double), hipMemcpyDeviceToHost, s));
    QMG_HIP(hipStreamSynchronize(s));
    if (bad[0] > 0) throw ApiError(QMG_EINVAL, "eps must be positive and finite");
    if (bad[1] > 0) throw ApiError(QMG_EINVAL, "f must be finite");
    if (bad[2] > 0) throw ApiError(QMG_EINVAL, "the velocities must be finite");
    g->bnorm = std::sqrt(b2);
    g->have_coef = true;
    if (g->adaptive) g->lattices_clear = true;
  });
}

int qmg_build_operators(qmg_grid_t* g, qmg_solve_report* info) {
  return guard(g, [&] {
    if (!g) throw ApiError(QMG_EINVAL, "null grid");
    build(g, info);
  });
}

int qmg_vcycle(qmg_grid_t* g, int n, double* relres) {
  return guard(g, [&] {
    need_ops(g);
    if (n < 0) throw ApiError(QMG_EINVAL, "negative cycle count");
    if (g->mixed && n > 0) finest_residual_norm(g);  // forms the inner right-hand side
    int done = 0;
    while (done < n) {
      const int B = std::min(n - done, kHistCap);
      const std::vector<double> nr = run_batch(g, B);
      if (relres)
        for (int c = 0; c < B; ++c) relres[done + c] = nr[c] / g->bnorm;
      done += B;
    }
  });
}

int qmg_solve(qmg_grid_t* g, double rel_tol, int max_cycles, double* history, qmg_solve_report* rep) {
  int status = QMG_OK;
  const int rc = guard(g, [&] {
    SolveState st;
    solve_begin(g, st, rel_tol, max_cycles);
    while (!st.done) {
      solve_enqueue(g, st);
      solve_collect(g, st);
    }
    if (history)
      for (size_t c = 0; c < st.history.size(); ++c) history[c] = st.history[c];
    solve_fill_report(g, st, rep);
    if (!(st.rr <= rel_tol)) {
      status = QMG_ENOTCONV;
      set_err(g, "tolerance not reached: relres " + std::to_string(st.rr) + " after " +
                     std::to_string(st.cycles) + " cycles");
    }
  });
  return rc != QMG_OK ? rc : status;
}

int qmg_get_solution(const qmg_grid_t* cg, double* u, int mem) {
  qmg_grid_t* g = const_cast<qmg_grid_t*>(cg);
  return guard(g, [&] {
    if (!g || !u) throw ApiError(QMG_EINVAL, "null argument");
    LevelBuf& F = g->lv[g->Lmax];
    if (g->adaptive) {
      int64_t uo = 0;
      for (int l = g->lb; l <= g->Lmax; ++l) {
        const int64_t cnt = (int64_t)g->hl[l].leaf.size();
        const double* src = g->mixed ? g->lv[l].x64 : (const double*)g->lv[l].u;
        launch_ad_gather<double>(g->unk_slots + uo, cnt, src, g->stage + uo, S(g));
        uo += cnt;
      }
    } else {
      const double* src = g->mixed ? g->x64 : (const double*)F.u;
      launch_gather_unknowns<double>(F.L, src, g->stage, S(g));
    }
    QMG_HIP(hipMemcpyAsync(u, g->stage, g->n_unknowns * sizeof(double),
                           mem == QMG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, S(g)));
    QMG_HIP(hipStreamSynchronize(S(g)));
  });
}

int qmg_residual(qmg_grid_t* g, double* r, int mem) {
  return guard(g, [&] {
    if (!g || !r) throw ApiError(QMG_EINVAL, "null argument");
    if (!g->have_coef) throw ApiError(QMG_ESTATE, "no coefficients set");
    if (g->mixed) throw ApiError(QMG_EINVAL, "the residual vector is offered for FP64 iterates");
    if (g->adaptive && !g->have_ops) throw ApiError(QMG_ESTATE, "operators not built");
    enqueue_residual_norm(g, false);
    LevelBuf& F = g->lv[g->Lmax];
    if (g->adaptive) {
      int64_t uo = 0;
      for (int l = g->lb; l <= g->Lmax; ++l) {
        const int64_t cnt = (int64_t)g->hl[l].leaf.size();
        launch_ad_gather<double>(g->unk_slots + uo, cnt, (const double*)g->lv[l].r, g->stage + uo, S(g));
        uo += cnt;
      }
    } else {
      launch_gather_unknowns<double>(F.L, (const double*)F.r, g->stage, S(g));
    }
    QMG_HIP(hipMemcpyAsync(r, g->stage, g->n_unknowns * sizeof(double),
                           mem == QMG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, S(g)));
    QMG_HIP(hipStreamSynchronize(S(g)));
  });
}

int qmg_set_solution(qmg_grid_t* g, const double* u, int mem) {
  return guard(g, [&] {
    if (!g || !u) throw ApiError(QMG_EINVAL, "null argument");
    LevelBuf& F = g->lv[g->Lmax];
    copy_in(g, g->stage, u, g->n_unknowns, mem);
    if (g->adaptive) {
      int64_t uo = 0;
      for (int l = g->lb; l <= g->Lmax; ++l) {
        const int64_t cnt = (int64_t)g->hl[l].leaf.size();
        double* dst = g->mixed ? g->lv[l].x64 : (double*)g->lv[l].u;
        launch_ad_scatter<double>(g->unk_slots + uo, cnt, g->stage + uo, 1.0, dst, S(g));
        uo += cnt;
      }
      // refined and hanging values are functions of the leaves
      composite_state(g);
    } else {
      launch_scatter_unknowns<double>(F.L, g->stage, g->mixed ? g->x64 : (double*)F.u, S(g));
    }
    QMG_HIP(hipStreamSynchronize(S(g)));
  });
}

int qmg_profile_enable(qmg_grid_t* g, int on) {
  return guard(g, [&] {
    if (!g) throw ApiError(QMG_EINVAL, "null grid");
    if (on < 0) throw ApiError(QMG_EINVAL, "profile stride must be >= 0");
    prof_harvest(g);
    g->prof_every = on;
    g->prof_count = 0;
    drop_graph(g);
  });
}

int qmg_profile_read(qmg_grid_t* g, int64_t* launches, double* total_ms) {
  return guard(g, [&] {
    if (!g || !launches || !total_ms) throw ApiError(QMG_EINVAL, "null argument");
    prof_harvest(g);
    *launches = g->prof_launches;
    *total_ms = g->prof_ms;
    g->prof_launches = 0;
    g->prof_ms = 0.0;
  });
}

int qmg_destroy_grid(qmg_grid_t* g) {
  if (!g) return QMG_EINVAL;
  int rc = QMG_OK;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  else (void)hipDeviceSynchronize();
  drop_graph(g);
  for (hipEvent_t e : g->prof_ev) (void)hipEventDestroy(e);
  if (g->owns && g->base && hipFree(g->base) != hipSuccess) rc = QMG_EHIP;
  if (g->vel && hipFree(g->vel) != hipSuccess) rc = QMG_EHIP;
  if (g->rscr && hipFree(g->rscr) != hipSuccess) rc = QMG_EHIP;
  if (g->hnorm && g->own_hnorm) (void)hipHostFree(g->hnorm);
  if (g->bev) (void)hipEventDestroy(g->bev);
  if (g->own_stream) (void)hipStreamDestroy(g->stream);
  delete g;
  return rc;
}

const char* qmg_last_error(const qmg_grid_t* g) {
  if (g) return g->err.c_str();
  return g_thread_err.c_str();
}

int qmg_get_operator(const qmg_grid_t* cg, int level, double* stencils) {
  qmg_grid_t* g = const_cast<qmg_grid_t*>(cg);
  return guard(g, [&] {
    if (!g || !stencils) throw ApiError(QMG_EINVAL, "null argument");
    if (level < g->lcq || level > g->Lmax) throw ApiError(QMG_EINVAL, "level out of range");
    if (level < g->Lmax && !g->have_ops) throw ApiError(QMG_ESTATE, "operators not built");
    if (level < g->lc) throw ApiError(QMG_EINVAL, "level below the coarsest level used");
    LevelBuf& B = g->lv[level];
    const int NS = ipow(3, g->d);
    double* tmp = nullptr;
    QMG_HIP(hipMalloc(&tmp, (size_t)NS * B.L.nslot * sizeof(double)));
    std::vector<double> h((size_t)NS * B.L.nslot);
    try {
      launch_zero<double>(tmp, (int64_t)NS * B.L.nslot, S(g));
      if (level == g->lc && !g->plain && g->opts.transfer != QMG_GEOMETRIC && level < g->Lmax) {
        // the coarsest level keeps its full FP64 Galerkin operator for the solve
        QMG_HIP(hipMemcpyAsync(tmp, g->tmpA[level & 1], h.size() * sizeof(double), hipMemcpyDeviceToDevice, S(g)));
      } else {
        launch_materialise(B.L, B.eps64, B.A, tmp, S(g));
      }
      QMG_HIP(hipMemcpyAsync(h.data(), tmp, h.size() * sizeof(double), hipMemcpyDeviceToHost, S(g)));
      QMG_HIP(hipStreamSynchronize(S(g)));
    } catch (...) {
      (void)hipFree(tmp);
      throw;
    }
    QMG_HIP(hipFree(tmp));
    std::vector<double> o = unpitch(B.L, h, NS);
    std::memcpy(stencils, o.data(), o.size() * sizeof(double));
  });
}

}  // extern "C"

namespace {

// Refinement criterion on the finest level, with its extrema (two 8-byte
// words at `scr`) and ten bin counts (ints at scr + 64) in `scr`: device
// memory of kRefineScratch bytes, whatever the grid size.
constexpr size_t kRefineScratch = 64 + 10 * sizeof(int);

void refine_flags_with(qmg_grid_t* g, double res_tol, double fraction, uint8_t* cell_flags, int64_t* n_flagged,
                       void* scr) {
  LevelBuf& F = g->lv[g->Lmax];
  const Lat& L = F.L;
  hipStream_t s = S(g);
  const int64_t ncell = L.d == 3 ? (int64_t)L.n * L.n * L.n : (int64_t)L.n * L.n;
  // r = b - A u on the finest level
  launch_stencil<double>(L, 2, (const double*)F.u, (const double*)F.b, (double*)F.r, eps_of<double>(F), F.A,
                         0.0, nullptr, nullptr, s);
  unsigned long long* mm = (unsigned long long*)scr;
  int* cnt = (int*)((char*)scr + 64);
  const unsigned long long init[2] = {~0ull, 0ull};
  QMG_HIP(hipMemcpyAsync(mm, init, sizeof(init), hipMemcpyHostToDevice, s));
  double* delta = g->stage;  // nslot doubles
  launch_refine_delta(L, (const double*)F.u, (const double*)F.r, res_tol, delta, mm, s);
  unsigned long long ext[2];
  QMG_HIP(hipMemcpyAsync(ext, mm, sizeof(ext), hipMemcpyDeviceToHost, s));
  QMG_HIP(hipStreamSynchronize(s));
  int64_t flagged = 0;
  double lo = 0.0, hi = 0.0;
  std::memcpy(&lo, &ext[0], sizeof(double));
  std::memcpy(&hi, &ext[1], sizeof(double));
  if (ext[0] == ~0ull || hi == 0.0) {  // no candidate, or nothing varies
    std::memset(cell_flags, 0, (size_t)ncell);
  } else {
    const int spread = hi > lo ? 1 : 0;
    const double width = (hi - lo) / 10.0;
    launch_zero<int>(cnt, 10, s);
    launch_refine_hist(L, delta, lo, width, spread, cnt, s);
    int counts[10];
    QMG_HIP(hipMemcpyAsync(counts, cnt, sizeof(counts), hipMemcpyDeviceToHost, s));
    QMG_HIP(hipStreamSynchronize(s));
    int64_t ncand = 0;
    for (int b = 0; b < 10; ++b) ncand += counts[b];
    const double need = fraction * (double)ncand;
    int64_t cum = 0;
    int kstar = 9;
    for (int b = 9; b >= 0; --b) {
      cum += counts[b];
      kstar = b;
      if ((double)cum >= need) break;
    }
    uint8_t* dflags = (uint8_t*)F.t;  // nslot iterates: at least ncell bytes
    launch_refine_cells(L, delta, lo, width, spread, kstar, dflags, s);
    QMG_HIP(hipMemcpyAsync(cell_flags, dflags, (size_t)ncell, hipMemcpyDeviceToHost, s));
    QMG_HIP(hipStreamSynchronize(s));
    for (int64_t c = 0; c < ncell; ++c) flagged += cell_flags[c] ? 1 : 0;
  }
  if (n_flagged) *n_flagged = flagged;
}

void refine_flags_check(qmg_grid_t* g, double res_tol, double fraction, uint8_t* cell_flags) {
  if (!g || !cell_flags) throw ApiError(QMG_EINVAL, "null argument");
  if (g->adaptive) throw ApiError(QMG_EINVAL, "the refinement criterion runs on regular grids");
  if (g->mixed) throw ApiError(QMG_EINVAL, "the refinement criterion needs FP64 iterates");
  if (!(res_tol > 0.0) || !(fraction > 0.0 && fraction <= 1.0))
    throw ApiError(QMG_EINVAL, "need res_tol > 0 and 0 < fraction <= 1");
  need_ops(g);
}

// Scratch of the entry point that allocates nothing: one copy per device,
// held until the process ends.  Host code never passes `scratch` itself
// (its name is a host-side stand-in there); it looks up the device address
// once per device and uses that.
constexpr size_t kNoAllocScratch = 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];
static_assert(kRefineScratch <= kNoAllocScratch, "the refinement criterion fits the scratch at any grid size");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_on_current_device() {
  int dev = 0;
  QMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw ApiError(QMG_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      throw HipError(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int qmg_refine_flags_noalloc(qmg_grid_t* g, double res_tol, double fraction, uint8_t* cell_flags,
                             int64_t* n_flagged) {
  return guard(g, [&] {
    refine_flags_check(g, res_tol, fraction, cell_flags);
    int dev = 0, gdev = 0;
    QMG_HIP(hipGetDevice(&dev));
    QMG_HIP(hipPointerGetAttribute(&gdev, HIP_POINTER_ATTRIBUTE_DEVICE_ORDINAL, (hipDeviceptr_t)g->base));
    if (dev != gdev) throw ApiError(QMG_EINVAL, "the grid lives on another device than the current one");
    refine_flags_with(g, res_tol, fraction, cell_flags, n_flagged, scratch_on_current_device());
  });
}

int qmg_refine_flags(qmg_grid_t* g, double res_tol, double fraction, uint8_t* cell_flags, int64_t* n_flagged) {
  return guard(g, [&] {
    refine_flags_check(g, res_tol, fraction, cell_flags);
    if (!g->rscr) QMG_HIP(hipMalloc(&g->rscr, 256));
    refine_flags_with(g, res_tol, fraction, cell_flags, n_flagged, g->rscr);
  });
}

int qmg_get_prolongation(const qmg_grid_t* cg, int level, double* weights) {
  qmg_grid_t* g = const_cast<qmg_grid_t*>(cg);
  return guard(g, [&] {
    if (!g || !weights) throw ApiError(QMG_EINVAL, "null argument");
    if (!g->have_ops) throw ApiError(QMG_ESTATE, "operators not built");
    if (level <= g->lc || level > g->Lmax) throw ApiError(QMG_EINVAL, "level out of range");
    LevelBuf& B = g->lv[level];
    const int NC = 1 << g->d;
    double* tmp = nullptr;
    QMG_HIP(hipMalloc(&tmp, (size_t)NC * B.L.nslot * sizeof(double)));
    std::vector<double> h((size_t)NC * B.L.nslot);
    try {
      launch_zero<double>(tmp, (int64_t)NC * B.L.nslot, S(g));
      launch_materialise_P(B.L, g->lv[level - 1].L, B.P, tmp, S(g));
      QMG_HIP(hipMemcpyAsync(h.data(), tmp, h.size() * sizeof(double), hipMemcpyDeviceToHost, S(g)));
      QMG_HIP(hipStreamSynchronize(S(g)));
    } catch (...) {
      (void)hipFree(tmp);
      throw;
    }
    QMG_HIP(hipFree(tmp));
    std::vector<double> o = unpitch(B.L, h, NC);
    std::memcpy(weights, o.data(), o.size() * sizeof(double));
  });
}

int qmg_apply(qmg_grid_t* g, int op, int level, const double* x, const double* b, double* out) {
  return guard(g, [&] {
    if (!g || !out || (!x && op != QMG_OP_JACOBI)) throw ApiError(QMG_EINVAL, "null argument");
    if (op < QMG_OP_MATVEC || op > QMG_OP_SMOOTH) throw ApiError(QMG_EINVAL, "bad op");
    if (op == QMG_OP_SMOOTH && g->adaptive) throw ApiError(QMG_EINVAL, "smoothing step on regular grids only");
    if (!g->have_coef) throw ApiError(QMG_ESTATE, "coefficients not set");
    if (level < g->Lmax && !g->have_ops) throw ApiError(QMG_ESTATE, "operators not built");
    if ((op == QMG_OP_RESTRICT || op == QMG_OP_PROLONG) && !g->have_ops)
      throw ApiError(QMG_ESTATE, "operators not built");
    if (g->mixed) {
      if (!g->have_ops)  // eps32 of the finest level is set at build
        launch_convert<double, float>(g->lv[g->Lmax].L, g->lv[g->Lmax].eps64, g->lv[g->Lmax].eps32, S(g));
      apply_op<float>(g, op, level, x, b, out);
    } else {
      apply_op<double>(g, op, level, x, b, out);
    }
  });
}

}  // extern "C"
