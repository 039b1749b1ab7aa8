/*
 * fams.h -- C ABI of the MI355X F-AMS pressure solver.
 *
 * F-AMS (Tene, Al Kobaisi, Hajibeygi, "Algebraic multiscale method for flow in
 * heterogeneous porous media with embedded discrete fractures") solves the
 * fine-scale EDFM system A p = q of the paper's Eq. (A-dis-mf): rows ordered
 * [matrix cells | fracture cells].  Given coarse grids for both media (Sec. 3,
 * Fig. 2) it builds the prolongation P column by column from local basis
 * functions in wirebasket order (Sec. 3.1, App. A) for one of four coupling
 * strategies, the coarse operator A_c = R A P with R = P^T (Sec. 3, App. A),
 * and iterates the two-stage scheme of Table 1 (multiscale stage + ILU(0)
 * smoothing) either as a Richardson loop or as the preconditioner of GMRES
 * (Sec. 4.6).  From any iterate, a finite-volume stage yields a
 * mass-conservative fine-scale flux field (Sec. 3.2, Sec. 4.6).
 *
 * Memory and ownership
 *   - Every array argument marked "device" is caller-owned GPU memory (e.g. a
 *     torch tensor on the current device), read during the call only.
 *     fams_setup copies everything it keeps into handle-owned device memory.
 *   - Every array marked "host" is caller-owned host memory.
 *   - All device work of a call is issued on the stream given to fams_setup
 *     (NULL = the default stream); calls that return host scalars synchronise
 *     that stream before returning.
 *   - A handle is used by one host thread / stream at a time; distinct handles
 *     are independent.  Calls from several host threads of one process at
 *     once are not supported; concurrent work on one GPU comes from one
 *     process per concurrent stream of requests (as the serving loop does).
 *
 * Environment
 *   - FAMS_LDS_LIMIT=<bytes> lowers the LDS budget of the local block solves
 *     (read when a handle first sizes them); blocks whose band no longer fits
 *     move to the global-memory storage modes.  For tests and tuning.
 *
 * Errors: no exceptions cross the ABI.  Negative status = error (on a setup
 * error *out is NULL and nothing is leaked; on a solve error the handle stays
 * valid); positive status = the iteration stopped without meeting rtol, with
 * the info record filled in.
 */
#ifndef FAMS_H_
#define FAMS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fams_handle_s* fams_handle_t;

typedef enum {
  FAMS_OK = 0,
  FAMS_NOT_CONVERGED = 1,        /* max_iter reached; info filled in */
  FAMS_DIVERGED = 2,             /* ||r|| > 1e8 ||r0|| or not finite */
  FAMS_ERR_INVALID_ARG = -1,     /* NULL/size/option error, NaN in q */
  FAMS_ERR_BAD_GRID = -2,        /* inconsistent wb_type / primal / vertex */
  FAMS_ERR_SINGULAR_LOCAL = -3,  /* a local block has no higher-rank neighbour,
                                    or a non-positive pivot in its solve */
  FAMS_ERR_SINGULAR_COARSE = -4, /* zero pivot in the coarse LU */
  FAMS_ERR_ZERO_PIVOT_ILU = -5,  /* non-positive ILU(0) pivot */
  FAMS_ERR_OOM = -6,             /* device allocation failed */
  FAMS_ERR_DEVICE = -7,          /* a HIP runtime call failed */
  FAMS_ERR_CAPACITY = -8         /* an internal per-block limit was exceeded */
} fams_status_t;

/* Coupling strategy of the basis functions (Sec. 3, the four definitions;
 * App. A.1-A.4). */
typedef enum { FAMS_DECOUPLED = 0, FAMS_FRAC = 1, FAMS_ROCK = 2, FAMS_COUPLED = 3 } fams_variant_t;

/* FP64 = everything in double.  MIXED = basis construction, ILU(0) storage
 * and the whole preconditioner in float; residual, Krylov vectors, solution
 * update, coarse solve and flux in double (a flexible outer loop). */
typedef enum { FAMS_PREC_FP64 = 0, FAMS_PREC_MIXED = 1 } fams_precision_t;

/* Outer iteration: the Table 1 loop, or GMRES with Table 1 steps 5-7 as a
 * right preconditioner (flexible GMRES, Sec. 4.6). */
typedef enum { FAMS_RICHARDSON = 0, FAMS_GMRES = 1 } fams_outer_t;
/* Restriction operator R of the coarse stage (Sec. 3, 3.2): MSFE (R = P^T, the
   default and the paper's choice for its experiments; SPD coarse operator for
   SPD A), MSFV (row i has a 1 on every cell of primal block i; coarse-scale
   mass conservation) or MSMIX (MSFV rows for the coarse nodes that lie in a
   fracture, MSFE rows for the matrix ones). */
typedef enum { FAMS_RESTRICT_FE = 0, FAMS_RESTRICT_FV = 1, FAMS_RESTRICT_MIX = 2 } fams_restriction_t;

/* Fine system A (Eq. A-dis-mf).  Rows/columns: matrix cells 0..n_matrix-1 in
 * natural grid order, then fracture cells, then (optionally) the last n_wells
 * unknowns: one pressure per well (Sec. 3: each well is a single fine-scale
 * unknown mapped to the coarse scale by the identity).  A well's row and
 * column hold the Peaceman couplings of Sec. 2 (q^w = beta (p^w - p) in every
 * perforated matrix or fracture cell).  CSR with columns sorted within each
 * row and the diagonal stored.  A must be symmetric positive definite with
 * non-positive off-diagonals (TPFA + EDFM connectivity + well indices). */
typedef struct {
  int64_t n;                  /* total fine unknowns (< 2^31) */
  int64_t n_matrix;           /* matrix cells; rows >= n_matrix are fracture cells
                                 (or wells) */
  int64_t nnz;                /* stored entries (< 2^31) */
  const int64_t* row_ptr;     /* device [n+1] */
  const int32_t* col_idx;     /* device [nnz] */
  const double* val;          /* device [nnz] */
  int64_t n_wells;            /* wells: rows n - n_wells .. n - 1 (0 = none).  Each
                                 is a coarse node of its own (class 3, in the
                                 vertex list, a primal block of its own); its
                                 basis function is computed like every other one,
                                 with the well above every cell of both media in
                                 the wirebasket order, so the perforated cells
                                 take the well's value as Dirichlet data in all
                                 four strategies (the beta term of the skeleton
                                 equation, Sec. 3.1) and P^ww = I, P^wm = P^wf = 0
                                 (Eq. prolongation_single) */
} fams_csr_t;

/* Coarse grids of both media (Sec. 3, Fig. 2).  wb_type is the wirebasket
 * class of each cell (0 = interior, 1 = face, 2 = edge, 3 = vertex; fracture
 * cells are never 0, App. A); vertex[K] is the coarse node of primal block K,
 * the only cell of class 3 in it; primal[i] is the primal block of cell i
 * (used by the finite-volume restriction, Sec. 3.2). */
typedef struct {
  int64_t n_coarse;           /* coarse nodes, matrix and fracture */
  const int8_t* wb_type;      /* device [n] */
  const int32_t* primal;      /* device [n], values in [0, n_coarse) */
  const int64_t* vertex;      /* device [n_coarse] */
} fams_grid_t;

/* Optional device-memory hook (e.g. a framework's caching allocator).  NULL
 * in fams_setup = hipMallocAsync/hipFreeAsync on the handle's stream.  Every
 * device buffer of the handle comes from `alloc` (called with the handle's
 * stream) and goes back through `free`, the last ones in fams_destroy; alloc
 * returns NULL when it cannot serve the size (the call then fails with
 * FAMS_ERR_OOM, except while fams_solve picks its lock-step group width).  A
 * caching hook lets handles created one after another reuse memory instead of
 * allocating it afresh (on MI355X a 140 GB lock-step work space allocated
 * anew after an earlier handle released its memory cost ~4 s of host time on
 * its first solve; taken from a cache, nothing).  The hook must stay valid
 * until fams_destroy returns. */
typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, void* stream);
} fams_allocator_t;

typedef struct {
  int32_t variant;            /* fams_variant_t */
  int32_t precision;          /* fams_precision_t */
  double trunc_alpha;         /* drop |P_ij| < alpha, rescale row (Sec. 4.3); 0 = off */
  int64_t merge_cap;          /* Coupled-AMS: max cells of a merged block (Sec. 3.1) */
  int32_t smoother;           /* 1 = ILU(0) post-smoothing (Table 1 step 7), 0 = none,
                                 2 = ILU(0) followed by a second stage on the per-medium
                                 sub-systems (Sec. 3.2): one ILU(0) application of
                                 diag(A^mm, A^ff) to the updated residual */
  int32_t profile;            /* 1 = time every kernel launch of this handle with HIP
                                 events from setup on (see fams_get_kernel_stats) */
  int32_t restriction;        /* fams_restriction_t; MSFV and MSMIX make the coarse
                                 operator non-symmetric: its inverse then comes from LU
                                 with partial pivoting.  Other values: FAMS_ERR_INVALID_ARG */
  int32_t nonsymmetric;       /* 0: A is symmetric (banded LDL^T local solves, SPD
                                 coarse inverse).  1: A may be non-symmetric (a
                                 linearised compressible system inside a Newton loop,
                                 Eq. dis-mf and Table 1 steps 1-2): banded LU local
                                 solves without pivoting, the coarse inverse from LU
                                 with partial pivoting; the conservative flux
                                 reconstruction (defined for the incompressible
                                 system) is refused with FAMS_ERR_INVALID_ARG */
} fams_setup_opts_t;

typedef struct {
  int32_t outer;              /* fams_outer_t */
  int32_t restart;            /* GMRES restart length (e.g. 30) */
  double rtol;                /* stop when ||q - A p||_2 <= rtol ||q - A p0||_2 */
  int32_t max_iter;           /* preconditioner applications (Table 1 sweeps) */
  int32_t use_initial_guess;  /* 0: p0 = 0; 1: p holds p0 on entry */
} fams_solve_opts_t;

typedef struct {
  int32_t status;             /* fams_status_t of this right-hand side */
  int32_t iterations;
  double rel_residual;        /* true ||q - A p|| / ||q - A p0|| at exit */
  double ms;                  /* wall time of this right-hand side */
} fams_info_t;

typedef struct {
  int64_t n, n_matrix, nnz;
  int64_t n_coarse;
  int64_t nnz_P;              /* after truncation */
  int64_t n_blocks;           /* local blocks (components) solved */
  int64_t max_block;          /* largest local block (cells) */
  int64_t fp32_fallback_blocks; /* MIXED: blocks re-solved in FP64 */
  int64_t ilu_levels_lower, ilu_levels_upper;
  double ms_setup;
  int64_t device_bytes;       /* device memory held by the handle */
  double local_flops;         /* arithmetic of the banded local factorisations,
                                 all levels (with the substitutions of blocks
                                 too wide for the wavefront solver) */
  double local_subst_flops;   /* arithmetic of the local substitutions done by
                                 the wavefront solver, all levels */
  int64_t peak_device_bytes;  /* most device memory the handle has held at once
                                 (setup, solves and flux reconstructions so far) */
  int64_t long_waits;         /* dependency waits of the dataflow ILU(0) sweeps and
                                 LU solves that lasted over ~1 ms, all solves so far
                                 (waits that long mean the workgroups holding the
                                 dependencies were not running, e.g. another
                                 process's work on the device; a wait gives up at
                                 2 s with FAMS_ERR_DEVICE) */
  int64_t tiled_rows;         /* rows that the lock-step products with A visit in
                                 slabs of grid lines marched along z (the first
                                 n_matrix rows when they form a 3D grid in natural
                                 order, found at the first lock-step solve; 0
                                 before it or otherwise); an order for cache reuse
                                 only, the results do not depend on it */
} fams_setup_info_t;

/* ---- lifecycle -------------------------------------------------------- */

/* Upper bound of the device memory a handle for this system will hold
 * through its setup and its solves (host-only estimate from sizes; used for
 * admission): `restart` sizes the GMRES work space and `max_nrhs` the
 * lock-step work space of fams_solve with several right-hand sides (groups of
 * up to 32).  Both smoother settings are covered.  Not covered: the flux
 * reconstruction's work space (two dense n_coarse^2 FP64 matrices and the
 * primal blocks' banded factors).  Errors: FAMS_ERR_INVALID_ARG for
 * non-positive sizes, restart or max_nrhs. */
fams_status_t fams_footprint(int64_t n, int64_t nnz, int64_t n_coarse, int32_t precision,
                             int32_t restart, int32_t max_nrhs, size_t* bytes_upper_bound);

/* Setup (Table 1 step 4 and the coarse system of step 5, plus the ILU(0)
 * factors): ranks and local blocks, basis functions in wirebasket order
 * (App. A), optional truncation (Sec. 4.3), R = P^T, A_c = P^T A P (dense
 * FP64), its LU with partial pivoting and inverse, ILU(0) of A in natural
 * order.  Everything stays device resident in the handle.  Blocking. */
fams_status_t fams_setup(const fams_csr_t* A, const fams_grid_t* grid,
                         const fams_setup_opts_t* opts, const fams_allocator_t* allocator,
                         void* hip_stream, fams_handle_t* out);

/* New values of A on the setup's pattern (same n, nnz, row_ptr and col_idx;
   `val` is a device pointer to nnz doubles, copied).  Table 1, steps 2 and 4,
   and Sec. 3.1: the basis functions follow the fine-scale properties only
   when these change beyond a threshold.  The ILU(0) factors, A_c and its
   inverse are always rebuilt from the new A; P (and R) are recomputed when
   max |a_new - a_basis| / |a_basis| over the entries exceeds `threshold`
   (a_basis: the values P was last computed from; threshold < 0 always
   recomputes), and *basis_recomputed says which happened.  The flux stage's
   FV operator is rebuilt on its next use.  Errors as fams_setup; after an
   error the handle is to be destroyed. */
fams_status_t fams_update_values(fams_handle_t h, const double* val, double threshold,
                                 int32_t* basis_recomputed);

/* Solve A p = q for nrhs right-hand sides (device, column-major [n x nrhs];
 * pageable host memory is refused with FAMS_ERR_INVALID_ARG).  Several
 * right-hand sides reuse the setup in lock-step groups of up to 32 (as many
 * as the free device memory holds, with 10% left to the caller; with an
 * allocation hook, the widest group whose work space the hook grants, halving
 * while it returns NULL): every pass over A, P, R, the ILU(0)
 * factors and A_c^{-1} serves the whole group, while each right-hand side
 * keeps its own outer iteration and stopping test (Sec. 4.6 reuses one setup
 * for a sequence of solves).  info (host, [nrhs], may be NULL).  Returns the
 * worst status. */
fams_status_t fams_solve(fams_handle_t h, const double* q, double* p, int32_t nrhs,
                         const fams_solve_opts_t* opts, fams_info_t* info);

/* Conservative flux reconstruction after an FV stage (Sec. 3.2, Sec. 4.6):
 * flux (device [nnz], in A's CSR slots): off-diagonal slot (i,j) holds the
 * flux F_ij from i to j; the diagonal slot holds E_i, the boundary/source
 * exchange, so that sum_j F_ij + E_i = 0 for every cell.  p_fv (device [n],
 * may be NULL) receives the FV-stage pressure.  *max_rel_imbalance (host) =
 * max_i |sum_j F_ij + E_i| / max_i (sum_j |F_ij| + |E_i|). */
fams_status_t fams_reconstruct_flux(fams_handle_t h, const double* q, const double* p,
                                    double* flux, double* p_fv, double* max_rel_imbalance);

fams_status_t fams_get_setup_info(fams_handle_t h, fams_setup_info_t* info);
fams_status_t fams_destroy(fams_handle_t h);
const char* fams_status_string(fams_status_t s);

/* ---- inspection (tests, profiling) ------------------------------------ */

/* P (CSR n x n_coarse, after truncation) copied to host; pass NULL arrays to
 * query nnz first.  row_ptr [n+1], col [nnz], val [nnz] (host). */
fams_status_t fams_get_prolongation(fams_handle_t h, int64_t* nnz, int64_t* row_ptr,
                                    int32_t* col, double* val);
/* Dense A_c = P^T A P, column-major [n_coarse^2] (host). */
fams_status_t fams_get_coarse_matrix(fams_handle_t h, double* ac);
/* ILU(0) factors in A's CSR slots (L unit lower below the diagonal, U on and
 * above), FP64 [nnz] (host). */
fams_status_t fams_get_ilu(fams_handle_t h, double* lu_val);
/* One application of Table 1 steps 5-7 to a residual r: z = dp_{1/2} +
 * dp_{2/2} (device [n] each). */
fams_status_t fams_apply_stage(fams_handle_t h, const double* r, double* z);
/* fams_apply_stage without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and result as fams_apply_stage (the same
 * kernels in the same order); the stage's scratch vectors live in one static
 * device array of 128 MiB that every GPU the library runs on holds until the
 * process ends, shared by all calls on that GPU: calls that overlap on one GPU
 * race.  The scratch needs 32n + 8 n_c (2 + ceil(n_c / 64)) bytes (FP64) or
 * 20n + the same coarse part (precision form), each part rounded up to 256
 * bytes; a larger system is refused with FAMS_ERR_CAPACITY.  Kernel timing
 * (fams_set_profiling) is not recorded for this call.  Synchronises the
 * handle's stream. */
fams_status_t fams_apply_stage_noalloc(fams_handle_t h, const double* r, double* z);

/* The dense kernels of the coarse system on an n x n column-major FP64
 * matrix a (device), result in out (device, n x n), on the default stream:
 *   op 0: out = a a          (the FP64 MFMA product used by the inverses)
 *   op 1: out = a^{-1} by blocked Gauss-Jordan without pivoting (A_c, SPD);
 *         FAMS_ERR_SINGULAR_COARSE if a pivot is not positive
 *   op 2: out = a^{-1} by LU with partial pivoting and triangular solves
 *   op 3: out = a^{-1} column by column with the dataflow LU solve (the FV
 *         stage's solver: one wavefront per 64-row chunk, chunks handed over
 *         through flags with bounded waits)
 *   op 4: out = the packed LU factors of P a (unit L below the diagonal, U on
 *         and above it, rows interchanged as LAPACK getrf leaves them)
 * For tests of those kernels; blocking. */
fams_status_t fams_dense_op(int32_t op, int32_t n, const double* a, double* out);

/* Per-kernel timing with HIP events on the handle's stream: enable (1) or
 * disable (0); then read total milliseconds and launch counts per kernel
 * name (host strings valid until the handle is destroyed). */
fams_status_t fams_set_profiling(fams_handle_t h, int32_t on);
fams_status_t fams_get_kernel_stats(fams_handle_t h, int32_t max_entries, int32_t* n_entries,
                                    const char** names, double* total_ms, int64_t* launches);

/* ---- host helpers for coarse grids (not timed) ------------------------ */

/* Structured matrix grid nx*ny*nz with coarsening cx*cy*cz (Sec. 3,
 * Fig. 2): the coarse node of each primal block is its centre cell per axis
 * (start + floor(len/2)); a cell's class is the number of its coordinates
 * lying on a coarse-node plane.  Host arrays: wb_type [n], primal [n],
 * vertex [ceil(nx/cx)*ceil(ny/cy)*ceil(nz/cz)]; blocks numbered x fastest. */
fams_status_t fams_grid_structured(int32_t nx, int32_t ny, int32_t nz, int32_t cx, int32_t cy,
                                   int32_t cz, int8_t* wb_type, int32_t* primal, int64_t* vertex,
                                   int64_t* n_coarse);

/* Fracture coarse grid: the distance-based coarsening of Table 2 run on the
 * x-y projection of each network (projected columns and their adjacency),
 * extruded along z with coarse layers k mod r_z == r_z/2 (or a plate's middle
 * layer when it has none) (Sec. 4.3).  A fracture cell is a vertex when its
 * column is a vertex column and its layer a coarse layer, an edge when
 * exactly one holds, a face otherwise.  Edge blocks without a vertex
 * neighbour and face blocks without an edge/vertex neighbour get their
 * lowest cell promoted to vertex.  Primal block of a fracture cell = nearest
 * vertex by graph distance (ties: lower coarse id).  Inputs (host):
 * A's CSR (to read fracture-fracture connections), cell_col/cell_z [n_f],
 * col_plate [n_cols], column graph col_ptr [n_cols+1]/col_adj, plate_zlo/
 * plate_zhi [n_plates]; d_min <= 0 means infinity.  Outputs (host): wb_type
 * and primal [n_f] for the fracture cells, vertex [n_f] (capacity) with the
 * fine indices of the fracture coarse nodes in ascending order, their count
 * in *n_coarse_frac; fracture coarse ids start at n_coarse_matrix. */
fams_status_t fams_grid_fracture(int64_t n_matrix, int64_t n, const int64_t* row_ptr,
                                 const int32_t* col_idx, const int32_t* cell_col,
                                 const int32_t* cell_z, int64_t n_cols, const int32_t* col_plate,
                                 const int64_t* col_ptr, const int32_t* col_adj, int64_t n_plates,
                                 const int32_t* plate_zlo, const int32_t* plate_zhi, int32_t d_min,
                                 int32_t r_z, int64_t n_coarse_matrix, int8_t* wb_type,
                                 int32_t* primal, int64_t* vertex, int64_t* n_coarse_frac);

#ifdef __cplusplus
}
#endif
#endif /* FAMS_H_ */
