/*
 * qmg.h -- C ABI of the MI355X (gfx950) quasi-matrix-free hybrid multigrid.
 *
 * The library solves the elliptic problem of the paper's eq. (1) with v = 0,
 *     -div(eps grad u) = f  on (0,1)^d,  u = 0 on the boundary,
 * discretised with d-linear (Q1) finite elements on the levels of a
 * tripartitioned spacetree (Sect. 3: every refinement splits a cell into 3^d
 * children; level l has 3^l cells per axis).  Per-vertex 3^d stencils are
 * applied in situ (Sect. 4); coarse operators are rediscretised (geometric
 * multigrid), or Galerkin products R A P (Sect. 4.3) with d-linear or BoxMG
 * (Sect. 4.4 and the BoxMG appendix) transfer operators; stored operators are
 * kept as hierarchical deltas from the rediscretised stencil and the d-linear
 * prolongation (Sect. 5), in FP64, FP32, FP16 or BF16.
 *
 * Conventions for every entry point:
 *  - Return value: QMG_OK (0) or a negative status.  Nothing throws across the
 *    ABI.  The text of the last error is returned by qmg_last_error(grid), or by
 *    qmg_last_error(NULL) for errors of calls that had no valid grid.  After any
 *    error other than QMG_EHIP the grid stays usable; QMG_EHIP (a HIP runtime or
 *    kernel fault) leaves the device state undefined.
 *  - Ownership: input arrays are copied in; the caller keeps them.  Output
 *    arrays are caller-allocated and written.  Pointers flagged by `mem` are
 *    host (QMG_HOST) or device (QMG_DEVICE) memory of the current HIP device.
 *  - Device memory: a grid lives in one workspace.  Pass device_buf == NULL to
 *    let the library allocate it (freed by qmg_destroy_grid), or pass a
 *    caller-owned device buffer of at least qmg_workspace_bytes() bytes that
 *    must outlive the grid (the library never frees it).
 *  - Streams: all device work of a grid is enqueued on the stream given at
 *    creation (a hipStream_t; NULL makes the library create and own a
 *    non-blocking stream, since cycles are replayed as captured HIP graphs,
 *    which the null stream cannot capture).  Calls return when their
 *    host-visible results are ready.  A grid is not thread-safe; distinct grids
 *    may be used concurrently from different threads on different streams.
 *  - Enumeration: on a regular grid the unknowns are the interior vertices of
 *    the finest level, numbered lexicographically with x fastest: vertex
 *    (i,j[,k]) with 1 <= i,j,k <= n-1 has index
 *    (i-1) + (n-1)*((j-1) + (n-1)*(k-1)); the cells (coefficients) are numbered
 *    the same way over 0 <= i,j,k <= n-1.  On an adaptive spacetree (Sect. 3)
 *    the unknowns are the leaf vertices (interior, non-hanging, not refined) of
 *    levels base..L and the coefficients live on the leaf cells (existing,
 *    not refined); both are numbered level by level, x fastest within a level
 *    (qmg_unknown_coords / qmg_leaf_cell_centres give their positions).
 *  - Lattice arrays (inspection entry points) cover all vertices 0..n of a
 *    level, x fastest, (n+1)^d values; stencil arrays hold 3^d such arrays,
 *    entry k belonging to the offset o in {-1,0,1}^d with
 *    k = (o_x+1) + 3(o_y+1) + 9(o_z+1).
 */
#ifndef QMG_H
#define QMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qmg_grid qmg_grid_t;
typedef struct qmg_server qmg_server_t;

enum qmg_status {
  QMG_OK = 0,
  QMG_EINVAL = -1,   /* invalid argument                                      */
  QMG_ENOMEM = -2,   /* workspace too small / allocation failed               */
  QMG_EHIP = -3,     /* HIP runtime error or device fault (sticky)            */
  QMG_ESTATE = -4,   /* call out of order (e.g. solve before build)           */
  QMG_ENOTCONV = -5, /* tolerance not reached within the cycle limit          */
  QMG_EINDEF = -6,   /* every Galerkin coarse operator failed the check       */
  QMG_EBUSY = -7     /* server: no slot / memory for the request right now    */
};

enum { QMG_HOST = 0, QMG_DEVICE = 1 };

/* Transfer operators and coarse operators (Sect. 4.1, 3.3, 3.4). */
enum {
  QMG_GEOMETRIC = 0,         /* d-linear P, R = P^T, rediscretised coarse stencils */
  QMG_GALERKIN_DLINEAR = 1,  /* d-linear P, R = P^T, A_{l-1} = R A_l P            */
  QMG_BOXMG = 2              /* BoxMG P, R = P^T, A_{l-1} = R A_l P               */
};

/* Operator store (Sect. 5).  PLAIN keeps full FP64 stencils (and P) on every
 * level including the finest; HIER keeps deltas from the rediscretised stencil
 * and from the d-linear P, dropping all-zero 64-vertex blocks.  PLAIN_FP64 and
 * HIER_FP64 iterate in FP64; the reduced-precision stores iterate in FP32 inside
 * an FP64 defect-correction loop (FP64 residual on the finest level, FP64
 * Galerkin construction and FP64 coarsest solve).  HIER_BPA is the paper's
 * codec: every delta entry is m 2^e (one exponent byte, bpa - 1 mantissa
 * bytes), per vertex the smallest bpa in {0, 2, ..., 8} that keeps every entry
 * within eps_mf; a 64-vertex block is stored at the largest bpa of its
 * vertices (all-zero blocks dropped); FP64 iterates.  Regular grids only; the
 * workspace reserves the widest payload, qmg_solve_report.bytes_operators
 * reports what the codec used. */
enum {
  QMG_PLAIN_FP64 = 0,
  QMG_HIER_FP64 = 1,
  QMG_HIER_FP32 = 2,
  QMG_HIER_FP16 = 3,   /* FP16 with one power-of-two scale per vertex */
  QMG_HIER_BF16 = 4,
  QMG_HIER_BPA = 5
};

/* Refinement regions of an adaptive spacetree (Sect. 3: every cell decides on
 * its own whether it is refined).  A region refines every existing cell of
 * levels base..level-1 that meets it, so its cells reach `level`.  Parameters
 * (host doubles, copied during the call), positions in the unit cube, x first:
 *  - QMG_REGION_BALL: centre (d values), radius r > 0 (d + 1 values).  A cell
 *    meets the ball when the distance from the centre to the closed cell box
 *    is below r.
 *  - QMG_REGION_LEVELSET_BAND: the band around the zero set of a random-
 *    Fourier-feature level set phi(x) = a sum_{m<M} cos(k_m . x + p_m):
 *    tau >= 0, a, M >= 1, then the M wave vectors k_m (d values each), then
 *    the M phases p_m (3 + M (d + 1) values).  A cell of level l with low
 *    corner x0 meets the band when, over its 3^d sample points
 *    x0 + o h_l / 2 (o in {0,1,2}^d), min |phi| < tau or phi takes both signs.
 *  - QMG_REGION_CELL_LIST: cells given as (level, i, j[, k]) groups of 1 + d
 *    values (cell indices 0 <= i < 3^level); listed cells of levels
 *    base..level-1 that exist are refined.
 * QMG_EINVAL for an unknown kind or a parameter count or value out of range. */
enum { QMG_REGION_BALL = 0, QMG_REGION_LEVELSET_BAND = 1, QMG_REGION_CELL_LIST = 2 };

typedef struct {
  int kind;               /* QMG_REGION_*                                      */
  int level;              /* refine meeting cells down to this level (<= L)   */
  const double* params;   /* host, n_params values (layout above)             */
  int n_params;
} qmg_region;

typedef struct {
  int dim;        /* 2 or 3                                                   */
  int max_level;  /* finest level L >= 2 (3^L cells per axis when refined)   */
  int base_level; /* 0 (or L): regular grid of level L.  1 <= base < L:
                     adaptive spacetree, every cell refined down to `base`,
                     further refinement given by `refine` and `regions`       */
  const uint8_t* refine; /* adaptive, host, nullable: for levels base..L-1 in
                     turn, one byte per cell of that level (x fastest; nonzero
                     = refine); flags of cells that do not exist are ignored  */
  int n_regions;  /* adaptive: number of regions (0 when only `refine`)       */
  const qmg_region* regions; /* host, n_regions entries; evaluated by the
                     library (in parallel on the host) during
                     qmg_workspace_bytes and qmg_create_grid, OR-ed with
                     `refine`                                                 */
} qmg_grid_desc;

typedef struct {
  int transfer;        /* QMG_GEOMETRIC | QMG_GALERKIN_DLINEAR | QMG_BOXMG     */
  int store;           /* QMG_PLAIN_FP64 ... QMG_HIER_BPA                     */
  int mu_pre, mu_post; /* smoothing steps per level, each >= 1 (Alg. 1)       */
  double omega;        /* Jacobi damping in (0, 2)                           */
  int coarsest_level;  /* requested coarsest level, 1 <= lc < L (<= base)    */
  int check_definite;  /* 1: raise the coarsest level when a Galerkin row is
                          not positive / diagonally dominant (Sect. 4.3)      */
  int inner_cycles;    /* FP32 V-cycles per FP64 outer iteration (>= 1)     */
  int use_graphs;      /* 1: each cycle (+ residual norm) is captured once as
                          a HIP graph and replayed (one host call per cycle;
                          pays off when many grids share a host thread, as in
                          the server); 0: eager kernel launches, which keep
                          up with the device for one grid on its own.  Needs
                          an even mu_pre + mu_post; ignored while profiling */
  double stagnation;   /* dynamic coarsest level (Sect. 4.3): > 0 moves the
                          coarsest level one up after a cycle (an outer
                          iteration with FP32 iterates) that has not reached
                          the tolerance and cut the relative residual by less
                          than this factor (1.0: only on growth); up to
                          L - 1, the base level at most on an adaptive grid.
                          The new coarsest level is solved exactly with its
                          stored operator decoded to FP64 when it has at most
                          1024 unknowns, otherwise by mu_pre + mu_post
                          sweeps; the raise lasts until the next
                          build_operators.  Cycles then run one per host
                          check.  0 (default): off                         */
  int smoother;        /* QMG_SMOOTH_JACOBI (default) or QMG_SMOOTH_BLOCK:
                          block Jacobi (Sect. "Spacetree block smoothers"):
                          each smoothing step first runs `bj_sweeps`
                          lexicographic Gauss-Seidel sweeps over the 2^d
                          iota-vertices (no coordinate divisible by 3) of
                          every patch (the 3^d vertices of one cell of the
                          next coarser level), then damped Jacobi on the
                          other vertices from the updated iterate; on every
                          smoothing step of the cycle.  Regular grids only   */
  int bj_sweeps;       /* Gauss-Seidel sweeps per patch, 1..64 (block only)  */
  int cycle;           /* QMG_CYCLE_MULT (default): multiplicative V(mu_pre,
                          mu_post) cycles (Alg. 1); QMG_CYCLE_ADD: additive
                          cycles (Alg. 2, unpipelined): the fine residual is
                          restricted down the hierarchy, every level takes
                          one damped Jacobi step from zero (the coarsest an
                          exact solve when it is direct) and the prolongated
                          sum of the corrections is added to the fine
                          iterate.  QMG_CYCLE_BPX: BPX cycles (Alg. 3,
                          unpipelined): as additive, but a level keeps only
                          the hierarchical surplus d_l - P_l (d_l at its
                          c-points) of its Jacobi step, so every vertex is
                          corrected by the coarsest level that holds it.
                          Both: Jacobi smoother, regular grids only          */
  int damping;         /* additive and BPX cycles: QMG_DAMP_EXP (default),
                          omega^(L-l+1) on level l; QMG_DAMP_CONST, omega on
                          every level (the paper's choice for BPX)           */
  double eps_mf;       /* QMG_HIER_BPA: largest coding error per entry, in
                          (0, 1]; default 1e-8                               */
  int restriction;     /* QMG_R_TRANSPOSE (default): R = P^T.  Petrov-
                          Galerkin (Sect. 4.3 and the convection results),
                          in the restriction and in A_{l-1} = R A_l P:
                          QMG_R_INJECTION, R = I (the coarse vertex takes the
                          fine value at its position); QMG_R_AGGREGATION, the
                          coarse vertex sums the 3^d fine vertices nearest to
                          it (unit weights).  Galerkin or BoxMG transfers,
                          multiplicative cycles, regular grids              */
  int coarse_solver;   /* QMG_COARSE_DIRECT (default): the coarsest level is
                          solved exactly (a dense inverse formed on the
                          device at build) when it has at most 1024
                          unknowns, otherwise by mu_pre + mu_post sweeps;
                          QMG_COARSE_SWEEPS: always the sweeps (the paper's
                          inexact coarse solve)                              */
  double eps_zero;     /* delta store: a 64-vertex block holds no payload when
                          every delta of its vertices is at most eps_zero
                          times the largest entry of the vertex's geometric
                          row (stencils) or d-linear weight (prolongation);
                          0 selects the default 2^-40; at most 1e-2          */
  int iterate;         /* QMG_IT_STORE (default): FP64 iterates for the
                          plain, HIER_FP64 and bpa stores, FP32 for the
                          reduced ones; QMG_IT_FP64 / QMG_IT_FP32 ask for one
                          (QMG_IT_FP32 also runs HIER_FP64 deltas inside the
                          FP64 defect correction); a combination the stores
                          do not offer is QMG_EINVAL                         */
} qmg_solver_opts;

enum { QMG_COARSE_DIRECT = 0, QMG_COARSE_SWEEPS = 1 };
enum { QMG_IT_STORE = 0, QMG_IT_FP64 = 1, QMG_IT_FP32 = 2 };

typedef struct {
  int cycles;               /* V-cycles run (inner cycles for FP32 iterates)  */
  int outer_iters;          /* FP64 residual evaluations                      */
  double relres;            /* final ||b - A u||_2 / ||b||_2 over the
                               unknowns (composite system when adaptive), FP64 */
  int coarsest_level_used;  /* after the definiteness check and any raise on
                               stagnation                                     */
  int64_t vertex_updates;   /* Jacobi vertex updates performed (all levels)   */
  size_t bytes_operators;   /* device bytes holding stored operators          */
  double zero_delta_fraction; /* share of 64-vertex blocks stored as zero     */
  double seconds;           /* wall time of the call                          */
} qmg_solve_report;

/* Library version string (static storage). */
const char* qmg_version(void);

/* The refinement flags an adaptive description stands for, evaluated on the
 * host (no device needed): `refine` OR-ed with every region, as the
 * `refine` layout (levels base..L-1, one byte per cell, x fastest; 1 =
 * refined, for existing cells; bytes of cells that do not exist are 0 unless
 * `refine` set them).  n_flags must be sum over l = base..L-1 of 3^(l d). */
int qmg_region_flags(const qmg_grid_desc* desc, uint8_t* flags, int64_t n_flags);

/* Device bytes a grid needs for `desc` and `opts` (worst case over stores). */
int qmg_workspace_bytes(const qmg_grid_desc* desc, const qmg_solver_opts* opts, size_t* bytes);

/* Default options: BoxMG, HIER_FP64, V(2,2), omega 0.6, lc 1, check on, 1 inner
 * cycle, graphs on. */
int qmg_default_opts(qmg_solver_opts* opts);

/* Creates a grid (Sect. 3: the levels 0..L of a tripartitioned spacetree,
 * each linearised as a Cartesian lattice of its level; on an adaptive
 * spacetree a level keeps its lattice and launches only the 64 x 4 vertex
 * tiles that touch existing cells) in `device_buf` (or library memory when
 * NULL).  `stream` is a hipStream_t.  On success *out owns the grid.
 * Adaptive spacetrees take every transfer and store; their cycle is the FAS
 * V-cycle on the levels above `base_level` and the correction-scheme cycle
 * below (with FP32 iterates: inner FAS cycles on the correction, the FP64
 * composite residual outside).  With QMG_BOXMG, P is built per refined cell
 * and also defines the hanging values (kept in FP64 on adaptive levels). */
int qmg_create_grid(const qmg_grid_desc* desc, const qmg_solver_opts* opts, void* device_buf,
                    size_t bytes, void* stream, qmg_grid_t** out);

/* Number of unknowns, leaf cells (coefficients) and levels (L+1). */
int qmg_sizes(const qmg_grid_t* grid, int64_t* n_unknowns, int64_t* n_leaf_cells, int* n_levels);

/* Coordinates of the unknowns, dim values per unknown (host array); `level`
 * (nullable) receives each unknown's level. */
int qmg_unknown_coords(const qmg_grid_t* grid, double* xyz, int8_t* level);

/* Centres of the leaf cells, dim values per cell (host array). */
int qmg_leaf_cell_centres(const qmg_grid_t* grid, double* xyz);

/* Sets the coefficient eps (one value per leaf cell, > 0 and finite) and the
 * source f (one value per unknown); the right-hand side of an unknown on level
 * l is b = h_l^d f (lumped).  ncomp = 1: `eps` holds eps only.  ncomp = 1 + d:
 * `eps` holds eps followed by the d velocity components v_1..v_d (each one
 * finite value per cell, same cell order), and the finest operator gains the
 * convection term (v . grad) u of eq. (1) (Galerkin Q1, v constant per cell,
 * no upwinding); regular grids, QMG_PLAIN_FP64 and Galerkin or BoxMG transfers
 * only (the velocity arrays are library memory, held until the grid ends).  `mem` says where eps and f
 * live (QMG_HOST or QMG_DEVICE); device inputs never leave the device (they
 * are checked and scattered there).  Resets the solution to zero and
 * invalidates operators.  QMG_EINVAL for values out of range; the grid then
 * holds no coefficients until a call succeeds. */
int qmg_set_coefficients(qmg_grid_t* grid, const double* eps, int ncomp, const double* f, int mem);

/* Builds all coarse operators (Sect. 4.3, 3.4): BoxMG P, Galerkin RAP with the
 * definiteness check, the hierarchical delta store (Sect. 5) and the coarsest
 * solve.  Fills `info` (nullable) with coarsest_level_used, bytes_operators,
 * zero_delta_fraction and seconds.  Returns QMG_EINDEF when even the first
 * coarse level fails the check. */
int qmg_build_operators(qmg_grid_t* grid, qmg_solve_report* info);

/* Runs n cycles (FP64 iterates: n V-cycles; FP32 iterates: n outer iterations
 * of inner_cycles V-cycles each) on the current solution.  relres (nullable,
 * n values, host) receives the relative residual after each cycle. */
int qmg_vcycle(qmg_grid_t* grid, int n, double* relres);

/* Cycles from the current solution until the relative residual is <= rel_tol
 * or max_cycles cycles ran.  history (nullable, host, max_cycles values)
 * receives the relative residual after each cycle.  Returns QMG_ENOTCONV if
 * the tolerance was not reached; `report` (nullable) is filled either way. */
int qmg_solve(qmg_grid_t* grid, double rel_tol, int max_cycles, double* history,
              qmg_solve_report* report);

/* The residual b - A u of the current solution, one value per unknown (FP64
 * iterates only; QMG_EINVAL with FP32 iterates): on a regular grid the
 * finest-level residual, on an adaptive spacetree the residual of the
 * composite system at every leaf (Sect. 3: refined vertices hold their finest
 * copy, hanging vertices the interpolant of the coarser level, which this call
 * refreshes first).  It is the vector whose norm the cycles report.
 * Overwrites the levels' residual buffers. */
int qmg_residual(qmg_grid_t* grid, double* r, int mem);

/* Copies the solution out / in (one value per unknown).  set_solution is a warm
 * start (resume): the next cycle starts from it. */
int qmg_get_solution(const qmg_grid_t* grid, double* u, int mem);
int qmg_set_solution(qmg_grid_t* grid, const double* u, int mem);

/* Measurement: with on = k > 0, every k-th smoothing launch on the finest
 * level (2D: the pre-smoothing pass of two sweeps and the residual; 3D: each
 * full Jacobi sweep, not the sweep from a zero iterate) carries per-dispatch
 * HIP event timestamps on the grid's stream (cycles then run as eager
 * launches); on = 0 turns it off.  profile_read returns the number of timed
 * launches and their summed device time in milliseconds since the last read,
 * then resets. */
int qmg_profile_enable(qmg_grid_t* grid, int on);
int qmg_profile_read(qmg_grid_t* grid, int64_t* launches, double* total_ms);

/* Frees the grid (and the workspace if the library allocated it). */
int qmg_destroy_grid(qmg_grid_t* grid);

/* Last error message of `grid` (or of the calling thread when grid is NULL). */
const char* qmg_last_error(const qmg_grid_t* grid);

/* ---------------- inspection (host arrays, FP64) --------------------------
 * These read back or exercise single steps of the hot path so that each can be
 * checked on its own.  `level` is 0..L; arrays are lattice arrays of that level. */

/* The operator of `level` as applied by the smoother (stored operators are
 * reconstructed from their store; the finest level is rediscretised from eps),
 * 3^d lattice arrays.  Requires built operators for level < L.  On adaptive
 * levels only the rows of leaf and refined vertices are defined (a slot that
 * is no vertex of the level reads back as its rediscretised row, which no
 * kernel uses). */
int qmg_get_operator(const qmg_grid_t* grid, int level, double* stencils);

/* Prolongation from level-1 to `level` as weights per fine vertex: 2^d lattice
 * arrays; array c = kx + 2 ky + 4 kz holds the weight of the coarse vertex
 * floor(f/3) + (kx,ky,kz) at fine vertex f (zero where it is not a parent).
 * On adaptive levels only the weights of the level's vertices are defined (a
 * slot outside the level reads back as the d-linear weights). */
int qmg_get_prolongation(const qmg_grid_t* grid, int level, double* weights);

/* Refinement criterion of the dynamically adaptive runs (Sect. 7), on a
 * regular grid with FP64 iterates and built operators: per interior vertex
 * the absolute difference between u and the mean of its 3^d - 1 neighbours;
 * vertices whose residual |b - A u| is below res_tol are candidates; ten even
 * bins over the candidates' range are taken from the top until they hold at
 * least `fraction` of the candidates (the paper: 10^-2 and 0.1); the cells
 * around every chosen vertex are flagged.  `cell_flags` (host, n^d bytes, x
 * fastest) receives 1 for a flagged cell of the finest level: the refine
 * flags of an adaptive grid of one more level.  *n_flagged (nullable) gets
 * their count.  Overwrites the finest level's residual and work buffer; the
 * first call allocates 256 bytes of device memory, held until the grid ends.
 * QMG_EINVAL on an adaptive grid, FP32 iterates or arguments out of range. */
int qmg_refine_flags(qmg_grid_t* grid, double res_tol, double fraction, uint8_t* cell_flags, int64_t* n_flagged);

/* The same criterion, flags and errors as qmg_refine_flags, for callers that
 * cannot allocate device memory (code under stream capture, serving loops,
 * harnesses that forbid hipMalloc): this call allocates nothing.  Its
 * extrema and bin counts (104 bytes, whatever the grid size) live in a
 * library-wide scratch array of 256 bytes that each device holds from the
 * library's load until the process ends; the call initialises what it
 * reads.  The device current at the call must be the grid's (QMG_EINVAL
 * otherwise).  Calls that overlap on one device share that array and race:
 * serialise them (one host thread, or one stream per device with the calls
 * in order). */
int qmg_refine_flags_noalloc(qmg_grid_t* grid, double res_tol, double fraction, uint8_t* cell_flags,
                             int64_t* n_flagged);

enum { QMG_SMOOTH_JACOBI = 0, QMG_SMOOTH_BLOCK = 1 };
enum { QMG_CYCLE_MULT = 0, QMG_CYCLE_ADD = 1, QMG_CYCLE_BPX = 2 };
enum { QMG_DAMP_EXP = 0, QMG_DAMP_CONST = 1 };
enum { QMG_R_TRANSPOSE = 0, QMG_R_INJECTION = 1, QMG_R_AGGREGATION = 2 };

enum {
  QMG_OP_MATVEC = 0,     /* out = A x                                         */
  QMG_OP_RESIDUAL = 1,   /* out = b - A x                                     */
  QMG_OP_JACOBI = 2,     /* out = x + omega diag(A)^-1 (b - A x); x = NULL: the
                            sweep from a zero iterate, out = omega diag(A)^-1 b */
  QMG_OP_RESTRICT = 3,   /* out (level-1 lattice) = P^T x (x on `level`)       */
  QMG_OP_PROLONG = 4,    /* out (level lattice) = b + P x (x on level-1)       */
  QMG_OP_SMOOTH = 5      /* out = one step of the grid's smoother from x      */
};

/* Applies one step of the hot path on `level` in the grid's iterate precision
 * (FP64 or FP32, converted at the boundary).  x, b, out are lattice arrays of
 * the sizes the operation implies; b is ignored where unused (may be NULL);
 * x may be NULL only for QMG_OP_JACOBI (EINVAL otherwise).
 * The step runs in the level's work buffers: the iterates and right-hand
 * sides of `level` (and level-1 for transfers) are overwritten, so a solve
 * after it starts with qmg_set_coefficients or qmg_set_solution. */
int qmg_apply(qmg_grid_t* grid, int op, int level, const double* x, const double* b, double* out);

/* ---------------- serving ------------------------------------------------
 * A persistent request loop (up to eight worker threads per server, each
 * driving its share of the slots) that keeps the grids and operators of
 * admitted requests on the device and overlaps their work.  Requests are
 * admitted in arrival order -- a later request that fits may pass a head that
 * does not -- while one of `max_slots` slots is free and the request's
 * qmg_workspace_bytes() fit in the unused part of `hbm_budget` (and in one
 * free range of it).
 * Each admitted request runs the single-grid path (create, set_coefficients,
 * build_operators, solve) on a stream of its own; its result does not depend
 * on the other requests.  Not in the paper: it batches independent solves the
 * way the paper's multi-parameter runs would. */
typedef struct {
  int64_t submitted, completed, failed, active, queued;
  size_t hbm_budget, hbm_in_use, hbm_peak;
  int max_slots;
  int64_t deferred;  /* requests that had arrived but were not admitted at
                        once: no memory for them, or every slot busy (each
                        counted once)                                       */
} qmg_server_stats_t;

/* Starts a server on the current HIP device (1 <= max_slots <= 256).  The
 * whole `hbm_budget` is reserved on the device here (QMG_ENOMEM if it cannot
 * be) and request workspaces are carved from it, so serving itself allocates
 * no device memory; the reservation is freed by qmg_server_destroy.  Every
 * slot runs on a stream of its own.  `stream` (a hipStream_t, nullable) is the
 * caller's: served work starts after the work already enqueued on it, and
 * qmg_server_drain makes it wait for all served work, so later work on it
 * needs no host synchronisation.  The server clock (arrival times) starts
 * here. */
int qmg_server_create(size_t hbm_budget, int max_slots, void* stream, qmg_server_t** out);

/* Queues a solve on a regular grid (eps: n^d cell values, f: (n-1)^d
 * unknowns, host memory, copied).  t_arrival: the request's arrival in
 * seconds on the server clock; it is not admitted before then, and its
 * latency counts from then (a negative value: arrives at submission).  This
 * lets a caller hand over a whole arrival schedule at once.  QMG_EINVAL for
 * an adaptive description, a NaN arrival or a request that could never fit
 * the budget.  The ticket identifies it in qmg_server_poll. */
int qmg_server_submit(qmg_server_t* server, const qmg_grid_desc* desc, const qmg_solver_opts* opts,
                      const double* eps, const double* f, double rel_tol, int max_cycles,
                      double t_arrival, uint64_t* ticket);

/* Non-blocking.  *done = 1 once the request retired; then u_out (nullable,
 * (n-1)^d host values), report (nullable) and latency_s (nullable: retire time
 * minus arrival time, seconds) are filled, the ticket is released, and the
 * request's own status is returned (QMG_ENOTCONV etc.). */
int qmg_server_poll(qmg_server_t* server, uint64_t ticket, int* done, double* u_out,
                    qmg_solve_report* report, double* latency_s);

/* Blocks until no request is queued or active. */
int qmg_server_drain(qmg_server_t* server);

int qmg_server_stats(qmg_server_t* server, qmg_server_stats_t* stats);
const char* qmg_server_last_error(const qmg_server_t* server);

/* Stops the loop: queued requests are dropped, active ones finish first. */
int qmg_server_destroy(qmg_server_t* server);

#ifdef __cplusplus
}
#endif

#endif /* QMG_H */
