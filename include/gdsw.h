/*
 * gdsw.h -- C ABI of the MI355X monolithic multilevel GDSW library.
 *
 * The library builds and applies the monolithic multilevel overlapping
 * Schwarz preconditioner with GDSW coarse spaces for the saddle-point system
 * K [u; p] = [F; 0] of eq. (2.1) (Q2 velocity, P1-discontinuous pressure),
 * and solves that system with restarted flexible GMRES (section 3).
 *
 *   setup  : index/overlap maps (section 2.1), local blocks A_i = R_i K R_i^T
 *            and their pivoted LU, the GDSW basis Phi (interface partition of
 *            unity times translations / pressure constants, extended by
 *            Phi_I = -A_II^{-1} A_{I,Gamma} Phi_Gamma), the Galerkin operator
 *            A_0 = Phi^T K Phi, recursed over the levels of section 2.2, and a
 *            direct factorization of the coarsest operator;
 *   apply  : z = B r with B of eq. (2.2);
 *   solve  : x with ||b - K x|| / ||b|| <= tol by FGMRES(m) preconditioned by B.
 *
 * All compute runs in HIP kernels on the current device.  Device pointers are
 * plain hipMalloc'ed (or PyTorch-owned) memory; host pointers are ordinary
 * process memory.  Every call is ordered on the hipStream_t passed as `stream`
 * (NULL = the legacy default stream).
 *
 * Ownership: the library copies everything it keeps during gdsw_setup; the
 * caller may free every input after it returns.  A context owns its device
 * memory until gdsw_destroy, which waits for the context's work and hands
 * the blocks to a process-wide cache (per device, at most 64 GiB) that later
 * setups reuse; cached blocks are released when the process exits (scratch
 * needed only during setup goes back to that cache when gdsw_setup returns).
 * The host side of setup runs its parallel loops on worker threads the library
 * creates once per process (at most 16, GDSW_HOST_THREADS to change); they
 * stay until the process exits.  Calls on one context must not overlap.
 *
 * Errors: every int-returning call returns one of the GDSW_* codes below;
 * gdsw_last_error() gives a message for the calling thread's last failure.
 */
#ifndef GDSW_H
#define GDSW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GDSW_OK = 0,
  GDSW_NOTCONV = 1,     /* solve: max_it reached; x holds the last iterate          */
  GDSW_EINVAL = -1,     /* bad sizes, ids or inconsistent maps                      */
  GDSW_ESINGULAR = -2,  /* zero pivot in a local or coarse factorization (level and
                           part are named in gdsw_last_error())                    */
  GDSW_ENOMEM = -3,     /* device allocation failed                                  */
  GDSW_EHIP = -4        /* a HIP runtime call failed                                 */
};

enum { GDSW_COMBINE_RESTRICTED = 0, GDSW_COMBINE_ADDITIVE = 1 };
enum { GDSW_MAX_RHS = 32 };   /* right-hand sides per gdsw_apply_multi / gdsw_solve_multi call */
enum { GDSW_FP64 = 0, GDSW_MIXED = 1 };

/*
 * The problem (eq. (2.1) after Dirichlet elimination) and its decomposition.
 *
 * Free dofs are numbered velocity first (3*node + d, compacted), then
 * pressure (4*elem + m, compacted); K is the n x n CSR matrix over them.
 *   rowptr, col, val : DEVICE pointers, CSR with sorted column indices.
 *   node_dof  [n_nodes*3] HOST: free dof of (node, direction) or -1 (Dirichlet).
 *   elem_node [n_elem*27] HOST: Q2 nodes of each element in local lexicographic
 *             order (local node k sits at lattice offset (k%3, (k/3)%3, k/9)).
 *   elem_pdof [n_elem*4]  HOST: pressure dofs, mode 0 = constant, 1..3 = the
 *             linear modes in xi, eta, zeta; -1 = eliminated.
 *   elem_part [n_elem]    HOST: level-1 part (subdomain) of each element.
 *   levels    L >= 2: the number of levels of section 2.2 (levels 1..L-1 carry
 *             overlapping local solves, level L is solved directly).
 *   n_parts   [L-1] HOST: number of parts on levels 1..L-1.
 *   part_parent [L-2] HOST pointers: part_parent[l-1][i] is the level-(l+1)
 *             part that level-l part i belongs to.
 * A coarse level (l >= 2) with a single part becomes the coarsest level.
 */
typedef struct gdsw_problem {
  int64_t n;
  const int64_t* rowptr;
  const int32_t* col;
  const double* val;
  int32_t n_nodes;
  const int32_t* node_dof;
  int32_t n_elem;
  const int32_t* elem_node;
  const int32_t* elem_pdof;
  const int32_t* elem_part;
  int32_t levels;
  const int32_t* n_parts;
  const int32_t* const* part_parent;
} gdsw_problem;

/*
 * overlap   : layers of the level's node graph added around each part's
 *             closure (default 1; section 3 uses one layer on all levels).
 * combine   : GDSW_COMBINE_RESTRICTED (default: every dof keeps the local
 *             solution of its owning part) or GDSW_COMBINE_ADDITIVE (the
 *             R_i^T sum printed in eq. (2.2)).
 * precision : GDSW_FP64, or GDSW_MIXED (local factors, interior factors and
 *             Phi_I in FP32; K, Galerkin accumulation, Krylov vectors,
 *             Gram-Schmidt and the coarsest factorization in FP64).
 * restart   : FGMRES restart length m, 1..250 (default 30; GDSW_EINVAL outside).
 * max_it    : cap on total inner iterations (default 1000).
 * tol       : relative residual target (default 1e-8).
 * no_coarse : 1 = omit the coarsest correction (one-level Schwarz for L = 2).
 * panel     : LU panel width, 0 = built-in default.
 * profile   : 1 = time every launch of the local-solve kernels (all levels)
 *             with HIP events recorded by the dispatch itself on the stream it
 *             runs on (reported by gdsw_get_stats); eager applies only.
 * graph     : 1 = inside gdsw_solve, each apply runs as a captured hipGraph
 *             (one per Krylov column, captured on first use and replayed by
 *             later solves on the same context); the solve then runs on a
 *             stream of the context, ordered after and before `stream`.
 * tune      : bit 0 (1): at the end of setup, time the local solves of every
 *             level with 2, 4 and 8 wavefronts per matrix and keep the fastest
 *             (gdsw_stats.ls_waves; results bit-identical to any fixed choice);
 *             bit 1 (2): time the batched LU variants of every level (paired
 *             64-column steps with rank-128 trailing updates or single steps
 *             with rank-64 updates; size-classed or batch-wide register
 *             panels; FP64 only: half- or full-width register panels for
 *             panels of 769..2048 rows) and keep the fastest
 *             (gdsw_stats.lu_variant; the variants agree up to rounding).
 *             Choices are kept per batch shape for the process and, with the
 *             environment variable GDSW_TUNE_CACHE=<file>, in that file; a
 *             shape found there is not timed again.  0 = ls_waves, paired
 *             steps, half-width panels.
 * ls_waves  : wavefronts per matrix of the local solves on every level when
 *             tune = 0: 0 = default (8), or 2, 4, 8.  Every choice gives
 *             bit-identical results (only the scheduling differs).
 */
typedef struct gdsw_options {
  int32_t overlap;
  int32_t combine;
  int32_t precision;
  int32_t restart;
  int32_t max_it;
  double tol;
  int32_t no_coarse;
  int32_t panel;
  int32_t profile;
  int32_t graph;
  int32_t tune;
  int32_t ls_waves;
  int32_t lu_variant;   /* batched LU variant when tune bit 1 is clear: bit 0 = single 64-column steps
                           with rank-64 updates (else paired, rank 128), bit 1 = full-width FP64 panels,
                           bit 2 = each matrix's panel in the smallest register panel that holds it
                           (one launch per size class) */
  int32_t pressure_gamma; /* P1disc pressure in the coarse space (section 2.1): 0 = the constant mode of
                             every element is an interface dof and the linear modes are interior
                             (saddle-point extension); 1 = every pressure mode is an interface dof
                             (velocity-only extension; the coarse columns are the same) */
} gdsw_options;

typedef struct gdsw_solve_info {
  int32_t iterations;    /* total inner FGMRES iterations                     */
  int32_t restarts;      /* completed cycles                                  */
  int32_t converged;     /* 1 if the true relative residual reached tol      */
  double rel_residual;   /* true ||b - K x||_2 / ||b||_2 in FP64              */
  double ms_apply, ms_spmv, ms_orth, ms_total;   /* wall-clock per phase     */
  int32_t reorthogonalizations;  /* iterations whose Gram-Schmidt took a second pass */
} gdsw_solve_info;

/* Sizes and algorithmic work of a built hierarchy (for reporting). */
typedef struct gdsw_stats {
  int32_t levels;                 /* effective number of levels               */
  int64_t n[8];                   /* rows of the level-l operator, l = 1..L    */
  int32_t parts[8];               /* parts on level l (0 on the coarsest)      */
  int64_t sum_ni[8];              /* sum of local block sizes on level l       */
  int32_t max_ni[8];
  int64_t factor_bytes[8];        /* bytes of local LU factors on level l      */
  double factor_flops[8];         /* sum (2/3) n_i^3 on level l                */
  double interior_flops[8];       /* interior LU + extension solves on level l */
  int64_t nnz[8];                 /* nonzeros of the level-l operator          */
  /* ms_maps: host map building; ms_extract: other host preparation (lists, patterns, uploads);
   * ms_factor / ms_basis / ms_coarse: GPU time of the local LU, basis + Galerkin and coarsest
   * phases (they overlap); ms_total: wall clock of gdsw_setup; ms_galerkin: unused (0). */
  double ms_maps, ms_extract, ms_factor, ms_basis, ms_galerkin, ms_coarse, ms_total;
  /* profile = 1 only: event-timed level-1 local-solve launches since setup */
  int64_t local_solve_launches;
  double ms_local_solve;          /* summed kernel time                         */
  /* algorithmic bytes of one launch: sum_i (e_i s + 20 n_i), e_i = elements of the factor tiles
   * the substitution reads (diagonal 64 x 64 tiles and off-diagonal tiles with a nonzero; n_i^2
   * for blocks of more than 64 tiles per side) */
  double local_solve_bytes;
  int32_t ls_waves[8];            /* wavefronts per matrix used by the local solves of level l */
  /* setup timeline from GPU events, in ms after the setup's first event on the caller's stream:
   * [l][0] begin and [l][1] end of level l+1's local factorization (side stream) and of its
   * basis + Galerkin phase (caller's stream); tl_coarsest: the coarsest factorization. */
  double tl_factor[8][2];
  double tl_basis[8][2];
  double tl_coarsest[2];
  /* GPU time of the batched LU kernels of level l alone (events around them on the
   * factorization stream; other setup work runs concurrently on other streams) */
  double ms_lu[8];
  /* algorithmic bytes of one apply: sum over Schwarz levels and parts of
   * e_i s + 24 n_i (factor tiles read, pivoted index, gathered r, local solution, scattered z),
   * plus 2 |Phi_I| s (restriction and prolongation), plus 8 n_c^2 (coarsest inverse);
   * s = 8 (FP64) or 4 (FP32 factors) */
  double apply_bytes;
  int32_t lu_variant[8];          /* batched LU variant of level l (see tune) */
  /* profile = 1: event-timed local-solve launches of every level (level 1 also above) */
  int64_t local_solve_launches_level[8];
  double ms_local_solve_level[8];
  double local_solve_bytes_level[8]; /* algorithmic bytes of one launch of level l */
  /* algorithmic bytes of one gdsw_spmv: 8 per value, 4 per column index read (once for a
   * group of three rows with one column list), 24 per row (row pointer, x, y) */
  double spmv_bytes;
} gdsw_stats;

/* Index maps of one level, host copies owned by the context (valid until
 * gdsw_destroy).  Lists are concatenated with int64 offsets [count+1]. */
typedef struct gdsw_maps_view {
  int32_t n_dof;           /* rows of this level's operator                 */
  int32_t n_parts;
  const int64_t* dom_ptr;  /* overlapping dof sets D_i, sorted               */
  const int32_t* dom;
  const int64_t* int_ptr;  /* interior dof sets I_i, sorted                  */
  const int32_t* inter;
  int32_t n_gamma_nodes;   /* interface nodes, ascending                    */
  const int32_t* gamma_nodes;
  int32_t n_entities;      /* interface entities ordered by smallest node     */
  const int64_t* ent_ptr;
  const int32_t* ent_nodes;
  const int32_t* ent_kind; /* 0 vertex, 1 edge, 2 face                      */
  int32_t n_coarse;        /* columns of Phi = coarse dofs of the next level  */
  const int32_t* col_entity; /* entity of a velocity column, -1-part for a pressure column */
  const int32_t* col_dir;  /* 0..2 velocity direction, 3 pressure           */
  const int32_t* owner;    /* [n_dof] part that owns each dof (restricted combine) */
} gdsw_maps_view;

typedef struct gdsw_ctx gdsw_ctx;   /* opaque */

/* Fill `opt` with the defaults listed above. */
void gdsw_default_options(gdsw_options* opt);

/* Build the hierarchy (section 2.1 for each level, recursion of section 2.2).
 * prob: see gdsw_problem; K is read during the call and copied.
 * opt : NULL = defaults.
 * out : receives a new context on success (NULL on failure).
 * Returns GDSW_EINVAL for inconsistent input, GDSW_ESINGULAR if a local,
 * interior or coarse block has a zero pivot, GDSW_ENOMEM or GDSW_EHIP. */
int gdsw_setup(const gdsw_problem* prob, const gdsw_options* opt, void* stream, gdsw_ctx** out);

/* z = B r, B of eq. (2.2).  r, z: DEVICE FP64 vectors of length n (may not alias). */
int gdsw_apply(gdsw_ctx* ctx, const double* r, double* z, void* stream);

/* Solve K x = b by FGMRES(restart) preconditioned by B (section 3), x0 = 0.
 * b, x: DEVICE FP64 vectors of length n.  Orthogonalization: classical
 * Gram-Schmidt with a second pass in the iterations where the first removed
 * more than half of |w|^2 (the test of Daniel, Gragg, Kaufman and Stewart).
 * Synchronizes the stream once per
 * inner iteration (to read the Hessenberg column).  Returns GDSW_OK or
 * GDSW_NOTCONV (x then holds the last iterate); info may be NULL. */
int gdsw_solve(gdsw_ctx* ctx, const double* b, double* x, void* stream, gdsw_solve_info* info);

/* gdsw_solve without any allocation, for callers that cannot allocate device
 * memory (tight serving loops, code whose allocations are forbidden or
 * recorded).  Same arguments, result and return codes as gdsw_solve (x is
 * bit-identical to gdsw_solve's), but the FGMRES workspace
 * ((2 restart + 2) n doubles plus a few partial-sum blocks) lives in a static
 * device array of 128 MiB that the library holds on every device it runs on
 * until the process ends (about n <= 270,000 rows at restart 30).  Larger
 * problems return GDSW_EINVAL with the size in gdsw_last_error().  It calls
 * no hipMalloc / hipFree: the page-locked host buffer and the event it reads
 * the Hessenberg column through are created by gdsw_setup.  Applies run
 * eagerly (also on graph = 1 contexts) and are not profiled.  Every call on
 * one device shares that device's array: calls that overlap in time on one
 * device (different threads or streams) race and must not be issued; nothing
 * in the array has to start at zero (every value is written before it is
 * read).  Not capturable into a graph: it synchronizes the stream once per
 * iteration like gdsw_solve. */
int gdsw_solve_noalloc(gdsw_ctx* ctx, const double* b, double* x, void* stream, gdsw_solve_info* info);

/* Z[:, s] = B R[:, s] for s < k (eq. (2.2) applied to k vectors at once): the
 * local solves of every level read each factor once per chunk of up to 8
 * right-hand sides instead of once per vector -- for the regime of section 3
 * in which the preconditioned solver is invoked many times to low accuracy.
 * R, Z: DEVICE FP64, column-major, column s at R + s ldr (ldr, ldz >= n; R and
 * Z may not alias); 1 <= k <= GDSW_MAX_RHS.  Each column agrees with gdsw_apply
 * on it to rounding (the local solves' panel updates run on the matrix cores).
 * The context keeps workspaces for k vectors, allocated on
 * first use.  Returns GDSW_EINVAL for bad arguments. */
int gdsw_apply_multi(gdsw_ctx* ctx, int32_t k, const double* R, int64_t ldr, double* Z, int64_t ldz, void* stream);

/* k independent FGMRES solves K x_s = b_s (section 3) in lockstep: one
 * gdsw_apply_multi per inner iteration serves every system still iterating.
 * B, X: DEVICE FP64, column-major (ldb, ldx >= n; no aliasing); info: k entries
 * (may be NULL).  Each system runs gdsw_solve's iteration on b_s with the
 * multi-vector apply (same tolerance and restarts; iterates agree with
 * gdsw_solve's to rounding).  Returns GDSW_OK if every system converged, GDSW_NOTCONV otherwise
 * (each x_s then holds its last iterate; info[s].converged tells which).
 * Synchronizes the stream once per inner iteration for all systems. */
int gdsw_solve_multi(gdsw_ctx* ctx, int32_t k, const double* B, int64_t ldb, double* X, int64_t ldx, void* stream,
                     gdsw_solve_info* info);

/* ---- two-grid geometric multigrid with the GDSW solver as coarse solver ----
 * Section 3's second role: the linearized system of a refined mesh is solved
 * by geometric multigrid whose coarse problem (one uniform coarsening) is
 * solved by FGMRES preconditioned by the multilevel GDSW method, only to a
 * relative reduction of 1e-1.  One cycle z = M r (z starts at 0):
 *   nu_pre times  z <- z + omega S (r - K_f z)
 *   then          z <- z + P x_c, x_c = FGMRES(K_c, B, P^T (r - K_f z)) to the coarse context's tol
 *   nu_post times z <- z + omega S (r - K_f z)
 * fine   : a context on the fine problem; its operator is K_f, its apply is the
 *          smoother S (set it up with no_coarse = 1 and levels = 2 for a damped
 *          one-level restricted Schwarz smoother), its options (restart, tol,
 *          max_it) govern gdsw_mg_solve.
 * coarse : a context on the coarse problem (its tol is the coarse reduction).
 * P      : n_fine x n_coarse prolongation, PT = P^T (n_coarse x n_fine), both
 *          DEVICE CSR (int64 row pointers, int32 columns, FP64 values), copied.
 * Both contexts must outlive the multigrid object and must not be used for
 * anything else while one of its calls runs.  Returns GDSW_EINVAL when sizes
 * do not match the contexts. */
typedef struct gdsw_mg gdsw_mg;   /* opaque */
int gdsw_mg_create(gdsw_ctx* fine, gdsw_ctx* coarse, int64_t n_fine, int64_t n_coarse, const int64_t* p_rowptr,
                   const int32_t* p_col, const double* p_val, const int64_t* pt_rowptr, const int32_t* pt_col,
                   const double* pt_val, int32_t nu_pre, int32_t nu_post, double omega, void* stream,
                   gdsw_mg** out);
/* z = M r, one cycle.  r, z: DEVICE FP64 of length n_fine (no aliasing). */
int gdsw_mg_apply(gdsw_mg* mg, const double* r, double* z, void* stream);
/* FGMRES on K_f x = b (the fine context's restart, tol and max_it) with the
 * cycle as preconditioner; same return codes and info as gdsw_solve. */
int gdsw_mg_solve(gdsw_mg* mg, const double* b, double* x, void* stream, gdsw_solve_info* info);
/* Cycles run and coarse FGMRES iterations summed over them since creation. */
int gdsw_mg_counts(gdsw_mg* mg, int64_t* cycles, int64_t* coarse_iterations);
void gdsw_mg_destroy(gdsw_mg* mg);

/* y = K x with the level-1 operator (CSR SpMV).  x, y: DEVICE FP64, length n. */
int gdsw_spmv(gdsw_ctx* ctx, const double* x, double* y, void* stream);

/* Sum of the local solutions of one level in the library's scatter order:
 * w holds the local vectors of all parts back to back (part i's block has the
 * length of D_i, entries in D_i order); z[g] = 0.0 + sum over the parts whose
 * block holds g, ascending part id (restricted combine: only the owner).
 * w, z: DEVICE FP64.  level is 1-based and must carry local solves. */
int gdsw_scatter_local(gdsw_ctx* ctx, int32_t level, const double* w, double* z, void* stream);

/* Host views of the index maps of a level that carries local solves (1-based):
 * the overlapping dof sets D_i and interior sets I_i, the interface nodes and
 * their entities (vertices, edges, faces), the coarse columns of Phi and the
 * owner of every dof -- the sets section 2.1 defines for one level, on the
 * level mesh of the recursion of section 2.2 for levels >= 2.
 * The view points into the context (valid until gdsw_destroy; not to be freed).
 * Returns GDSW_EINVAL for a NULL argument or a level without local solves. */
int gdsw_export_maps(gdsw_ctx* ctx, int32_t level, gdsw_maps_view* out);

/* Sizes, algorithmic work and setup timings of the hierarchy. */
int gdsw_get_stats(gdsw_ctx* ctx, gdsw_stats* out);

/* Host-only dry run: validates the problem and builds the index maps of every
 * level (no device allocation, no kernel launch; K's device arrays are not
 * read).  For inspection and admission control.  Returns GDSW_EINVAL for
 * inconsistent input. */
typedef struct gdsw_plan gdsw_plan;   /* opaque */
int gdsw_plan_create(const gdsw_problem* prob, const gdsw_options* opt, gdsw_plan** out);
/* Number of levels carrying local solves, and whether a direct coarsest level follows. */
int gdsw_plan_levels(gdsw_plan* plan, int32_t* schwarz_levels, int32_t* has_coarsest);
/* Host views of the maps of level `level` (1-based), valid until gdsw_plan_destroy. */
int gdsw_plan_maps(gdsw_plan* plan, int32_t level, gdsw_maps_view* out);
void gdsw_plan_destroy(gdsw_plan* plan);

/* Estimated peak device bytes of the context of this problem (its setup scratch
 * included), for admission control; host-only integer work, no device
 * allocation. Returns 0 on error. */
size_t gdsw_footprint_bytes(const gdsw_problem* prob, const gdsw_options* opt);

/* Release every resource of the context (NULL is a no-op): waits for the
 * work of the context's calls (on the streams they were given and on its own
 * streams; other work on the device is not waited for), returns the device
 * blocks to the process-wide cache and frees the host memory. */
void gdsw_destroy(gdsw_ctx* ctx);

/* Message of the calling thread's last failure ("" if none). */
const char* gdsw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
