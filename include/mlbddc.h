/*
 * mlbddc.h -- C ABI of the MI355X multilevel BDDC library.
 *
 * The library solves K u = f for a finite-element stiffness matrix K by
 * preconditioned conjugate gradients on the reduced interface problem
 * S^ u^ = g^ (Sistek, Mandel, Sousedik, Burda, "Parallel implementation of
 * Multilevel BDDC", section 2), with the multilevel BDDC preconditioner of
 * Algorithms 1 (set-up) and 2 (apply).  All numerical work runs in HIP
 * kernels on one gfx950 device; host code only plans index structures.
 *
 * Conventions
 *  - Every entry point returns an mlbddc_status: 0 on success, a negative
 *    code on failure.  Nothing throws or aborts across the ABI.  After a
 *    failure, mlbddc_last_error() describes it.
 *  - "host" pointers are read during the call only; the library copies what
 *    it keeps.  "device" pointers are borrowed for the call, must hold the
 *    stated number of elements, and must not alias each other.
 *  - All device work is ordered on the stream given to mlbddc_create (0 =
 *    the null stream).  Calls return once the work is queued unless stated.
 *  - A handle is not thread-safe.
 *  - Vectors of free DOFs are numbered as follows: free nodes in increasing
 *    node order, node components innermost (DOF = free_node * ndof + c).
 *    Interface vectors are numbered by increasing free-DOF index.
 */
#ifndef MLBDDC_H
#define MLBDDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mlbddc_status;
typedef struct mlbddc_handle_s* mlbddc_t;

enum {
  MLBDDC_OK = 0,
  MLBDDC_E_ARG = -1,              /* invalid argument or inconsistent mesh / partition */
  MLBDDC_E_HIP = -2,              /* a HIP runtime call failed */
  MLBDDC_E_NOMEM = -3,            /* device or host allocation failed */
  MLBDDC_E_STATE = -4,            /* call out of order (e.g. apply before setup) */
  MLBDDC_E_NOT_SPD = -5,          /* non-positive pivot in a subdomain factorization */
  MLBDDC_E_SINGULAR_CONSTRAINTS = -6, /* constrained local problem singular */
  MLBDDC_E_NOT_CONVERGED = -7,    /* PCG reached max_iter; u holds the last iterate */
  MLBDDC_E_BREAKDOWN = -8,        /* PCG breakdown: p^T S p <= 0 or not finite */
  MLBDDC_E_NO_DEVICE = -9         /* no usable HIP device */
};

enum { MLBDDC_FP64 = 0, MLBDDC_MIXED = 1 };                  /* precision modes */
enum { MLBDDC_CORNERS = 1, MLBDDC_EDGES = 2, MLBDDC_FACES = 4, MLBDDC_ALL_PRIMAL = 8 };
enum { MLBDDC_W_STIFFNESS = 0, MLBDDC_W_MULTIPLICITY = 1 };  /* interface weights */
enum { MLBDDC_POISSON_Q1 = 0, MLBDDC_ELASTICITY_HEX8 = 1 };  /* element kinds */

typedef struct {
  int32_t precision;   /* MLBDDC_FP64: every factor in FP64.  MLBDDC_MIXED: the
                          preconditioner's local factors and solves in FP32; the
                          interface operator S^, PCG vectors and dots, weights and
                          the top coarse factor stay FP64. */
  double rtol;         /* PCG stop: ||r^|| / ||g^|| < rtol (default 1e-8) */
  int32_t max_iter;    /* default 1000 */
  int32_t weights;     /* MLBDDC_W_* */
  int32_t use_graph;   /* capture one PCG iteration as a HIP graph (1) or launch eagerly (0) */
  int32_t panel_tiles; /* tile columns per panel of the subdomain-matrix factorizations
                          (0 = from the tune table, else 4) */
  int32_t device;      /* HIP device ordinal */
  int32_t panel_tiles_precond; /* same for the constrained local problems (0 = tune table / 4) */
  const char* tune_table;      /* path of a tune table written by the autotuner, or NULL;
                                  lines "<K|M> <f64|f32> <ceil(log2(max tiles per side))> <panel> [<stage>]",
                                  "MV <f64|f32> 0 <tiles per workgroup>", "PANEL <f64|f32> 0 <stage>"
                                  (staged columns of the panel products; else the job's) and
                                  "SHAPE f32 0 <16|32|3>" (FP32 tile product form, as mfma_f32) */
  int32_t lookahead;   /* 0 (default): one stream.  1: each factorization updates the next panel's
                          columns first on the library stream and the rest of the trailing matrix on a
                          second stream, so the next panel's factorization can overlap that bulk update */
  int32_t side_stream; /* 1 (default): in mixed precision the level-1 local operator product G_i r_i runs
                          on a second stream beside the coarse levels of the apply.  0: one stream.
                          Both give bitwise the same results */
  int32_t stage_cols;  /* columns of a tile staged per step of the MFMA tile products of the
                          factorizations: 16, 32 or 64 (0 = from the tune table, else 32).  Every value
                          gives bitwise the same results */
  int32_t mv_group_tiles; /* stored tiles per workgroup of the large tile matrix-vector products (S^,
                          the level-1 local operators): 1 or 2 (0 = from the tune table per precision,
                          else 1).  Both give bitwise the same results */
  int32_t mfma_f32;    /* form of the FP32 tile products of the factorizations: 16 (FP32 MFMA 16x16x4),
                          32 (FP32 MFMA 32x32x2) or 3 (each FP32 operand split exactly into three
                          bfloat16 pieces, six of the nine piece products on the bf16 MFMA 16x16x32,
                          the dropped ones below 2^-23 |a||b|; takes at least 32 staged columns;
                          faster, but the preconditioner's error grows two to four times)
                          (0 = from the tune table, else 16).  The forms sum the products in
                          different orders: results agree to FP32 rounding */
} mlbddc_options;

typedef struct {
  int32_t dim;               /* 2 or 3 */
  int32_t ndof_per_node;     /* 1 (Poisson) or dim (elasticity) */
  int64_t n_nodes;
  int64_t n_elems;
  int32_t nodes_per_elem;    /* 4 (quadrilateral) or 8 (hexahedron) */
  const int32_t* elem_nodes; /* host [n_elems * nodes_per_elem] */
  const double* elem_matrix_ref; /* host [nd * nd], nd = nodes_per_elem * ndof_per_node;
                                    unit-modulus element matrix K_e^0, DOFs node-major */
  const double* elem_scale;  /* host [n_elems]: element modulus E_e (K_e = E_e K_e^0) */
  const uint8_t* dirichlet_nodes; /* host [n_nodes]: 1 = all components fixed to zero */
} mlbddc_mesh;

typedef struct {
  int32_t n_levels;             /* L >= 2: levels 1..L-1 are BDDC levels, level L the coarse problem */
  const int32_t* elem_to_sub;   /* host [n_elems]: level-1 subdomain of every element, 0..N1-1 */
  const int32_t* const* sub_to_parent; /* host [L-2] arrays: for l = 2..L-1, the level-l
                                          subdomain of every level-(l-1) subdomain */
  int32_t constraints;          /* MLBDDC_CORNERS | MLBDDC_EDGES | MLBDDC_FACES on every level, or
                                   MLBDDC_ALL_PRIMAL (every interface node primal, level 1) */
} mlbddc_partition;

typedef struct {
  int32_t iterations;  /* operator applications of PCG */
  int32_t converged;
  double rel_res;      /* final ||r^|| / ||g^|| (recursive residual) */
  double lambda_min;   /* Lanczos estimates of the spectrum of M S^ */
  double lambda_max;
  double t_plan;       /* seconds: host planning and preparation in the last setup (the device
                          already factorizes the parts prepared first meanwhile) */
  double t_setup_num;  /* seconds: device set-up still running when the host preparation ended
                          (setup), or the whole numeric set-up (update_coefficients);
                          t_plan + t_setup_num is the set-up wall time */
  double t_solve;      /* seconds: condensation + PCG + interior recovery */
} mlbddc_stats;

typedef struct {
  mlbddc_status status;
  int32_t level;       /* 1-based level of a factorization failure, else 0 */
  int32_t subdomain;   /* subdomain of a factorization failure, else -1 */
  int32_t column;      /* local column of a factorization failure, else -1 */
  char message[256];
} mlbddc_error;

/* Text of a status code.  Never fails. */
const char* mlbddc_status_string(mlbddc_status code);

/* Default options (FP64, rtol 1e-8, max_iter 1000, stiffness weights, no graph). */
void mlbddc_default_options(mlbddc_options* opt);

/* Device memory provider.  alloc(bytes, ctx) returns device memory of at
 * least `bytes` bytes on options->device, aligned to 256 bytes, or NULL when
 * it has none (the library then releases its cached blocks once and retries,
 * else fails with E_NOMEM); free(ptr, ctx) takes back a block that alloc
 * returned.  Both are called from the thread that calls setup, update and
 * destroy, only while that call runs.  A block is handed back only when no
 * queued library work uses it any more: before free, the library has
 * synchronized every stream it used the block on, so an allocator that
 * reuses blocks on the caller's stream needs no further ordering.  With a
 * caching allocator (e.g. a framework's), the library owns no device memory
 * of its own. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} mlbddc_allocator;

/* Create a handle on options->device, ordering all work on `stream`
 * (a hipStream_t passed as void*).  *h receives the handle.  `alloc`
 * (copied; may be NULL = hipMalloc / hipFree) provides every device block
 * the handle uses (the operators of every level, work vectors, index maps);
 * pinned host staging buffers are allocated by the library itself.
 * Errors: E_ARG (bad options, an allocator without alloc or free),
 * E_NO_DEVICE, E_HIP.  This follows the paper's statement of the problem
 * (section 2): one handle holds one decomposition of one mesh. */
mlbddc_status mlbddc_create(mlbddc_t* h, const mlbddc_options* opt, const mlbddc_allocator* alloc, void* stream);

/* Set-up (Algorithm 1): plan the levels from the mesh and partition on the
 * host (interface classification into faces, edges and vertices; corner
 * selection; constraint rows of C_i; weights E_i; pseudo-mesh of every next
 * level), then on the device assemble the subdomain matrices K_i, factorize
 * their interiors, form the local Schur complements, factorize the
 * constrained local problems of Eq. (1), form the coarse bases Psi_i and the
 * coarse matrices K_Ci, assemble the next level and recurse; factorize the
 * top coarse matrix.  Synchronizes the stream.
 * Errors: E_ARG (bad maps, empty subdomain, element in no subdomain),
 * E_NOT_SPD (level, subdomain and column in mlbddc_last_error),
 * E_SINGULAR_CONSTRAINTS, E_NOMEM, E_HIP. */
mlbddc_status mlbddc_setup(mlbddc_t h, const mlbddc_mesh* mesh, const mlbddc_partition* part);

/* Redo the numeric set-up with new element moduli (device [n_elems] FP64),
 * keeping the planned structure.  Synchronizes the stream.  Errors as setup. */
mlbddc_status mlbddc_update_coefficients(mlbddc_t h, const double* elem_scale_dev);

/* Sizes after setup: free DOFs, level-1 interface size, coarse size of
 * level `level` (1-based, 1..L-1), number of level-l subdomains. */
int64_t mlbddc_num_dofs(mlbddc_t h);
int64_t mlbddc_interface_size(mlbddc_t h);
int64_t mlbddc_coarse_size(mlbddc_t h, int32_t level);
int64_t mlbddc_num_subdomains(mlbddc_t h, int32_t level);

/* The level-1 interface after setup: out[k] = free-DOF index of interface
 * entry k (increasing), host [interface_size].  E_STATE before setup. */
mlbddc_status mlbddc_interface_dofs(mlbddc_t h, int64_t* out);

/* Local sizes of the level-`level` subdomains after setup: out[3*i + 0..2] =
 * {interior DOFs, interface DOFs, constraints} of subdomain i (host
 * [3 * num_subdomains(level)]).  Used to count algorithmic bytes and flops. */
mlbddc_status mlbddc_subdomain_sizes(mlbddc_t h, int32_t level, int64_t* out);

/* z^ = M_BDDC r^ (one application of Algorithm 2) on the level-1 interface.
 * r_dev, z_dev: device FP64 [interface_size].  Asynchronous.  E_STATE before setup. */
mlbddc_status mlbddc_apply(mlbddc_t h, const double* r_dev, double* z_dev);

/* y = S^ x, the interface Schur complement (section 2).  Device FP64
 * [interface_size].  Asynchronous.  E_STATE before setup. */
mlbddc_status mlbddc_apply_schur(mlbddc_t h, const double* x_dev, double* y_dev);

/* y = S^ x as mlbddc_apply_schur, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the work vectors (the gathered subdomain copies of x
 * and the products) live in a 64 MiB device array of the library, held on
 * every device it runs on until the process ends, and nothing is allocated.
 * E_ARG when 16 bytes per flat interface entry (the subdomain interface
 * sizes, each rounded up to 64) exceed 64 MiB, E_STATE before setup.  All
 * calls on one device share that array: calls that overlap on one device
 * (several streams or threads) race.  Result equal to mlbddc_apply_schur up
 * to rounding (another summation order).  Asynchronous. */
mlbddc_status mlbddc_apply_schur_noalloc(mlbddc_t h, const double* x_dev, double* y_dev);

/* Condensed right-hand side g^ = f_G - sum_i R_i^T K_GI K_II^{-1} f_I.
 * f_dev: device FP64 [num_dofs]; g_dev: device FP64 [interface_size]. */
mlbddc_status mlbddc_condense(mlbddc_t h, const double* f_dev, double* g_dev);

/* Solve K u = f: condense, run BDDC-preconditioned CG on the interface from
 * u^_0 = 0 (or the interface part of u0_dev when not NULL) until
 * ||r^||/||g^|| < rtol, recover the interiors.  f_dev, u_dev, u0_dev: device
 * FP64 [num_dofs].  Synchronizes the stream; fills *st when not NULL.
 * Errors: E_NOT_CONVERGED (u holds the last iterate), E_BREAKDOWN, E_STATE. */
mlbddc_status mlbddc_solve(mlbddc_t h, const double* f_dev, double* u_dev, const double* u0_dev,
                           mlbddc_stats* st);

/* out_e = E_e a_e^T K_e^0 b_e for free-DOF vectors a, b (device FP64
 * [num_dofs]; fixed DOFs count as zero); out_dev: device FP64 [n_elems].
 * With a = lambda (adjoint) and b = u this is the element sensitivity
 * -dJ/dtheta_e of J = f^T u for E_e = exp(theta_e). */
mlbddc_status mlbddc_element_energy(mlbddc_t h, const double* a_dev, const double* b_dev, double* out_dev);

/* Copy a level's coarse matrix K_C (dense, row-major, coarse_size^2 FP64)
 * to host memory; for tests. */
mlbddc_status mlbddc_get_coarse_matrix(mlbddc_t h, int32_t level, double* host_out);

/* Kernel-level profiling (for rooflines).  When enabled, HIP events are
 * recorded around every factorization launch of a set-up (on the stream the
 * launch runs on), and around the tile product kernel of the level-1
 * interface operator S^ and of the level-1 local operators G_i in every
 * apply_schur / apply call made outside stream capture (PCG iterations
 * replayed from a graph are not timed).  mlbddc_get_profile synchronizes
 * those events and returns, per kernel class, the accumulated device time,
 * the number of launches, the algorithmic flops of the tiles the
 * factorization launches processed (dense tile counts: a tile update with k
 * inner tile columns is 2*64^3*k flops, a diagonal tile 64^3/3 for the
 * factor plus 64^3/3 for its inverse) and the algorithmic bytes the product
 * launches streamed (the stored lower triangles, 8 or 4 bytes per entry of
 * sum_i n_i (n_i + 1) / 2).  Enabling resets the counters. */
enum {
  MLBDDC_PROF_UPDATE_FP64 = 0,  /* trailing / in-panel tile updates, FP64 MFMA */
  MLBDDC_PROF_UPDATE_FP32 = 1,  /* trailing / in-panel tile updates, FP32 MFMA */
  MLBDDC_PROF_PANEL = 2,        /* panel solves with inverted diagonal tiles */
  MLBDDC_PROF_DIAG = 3,         /* diagonal tile factor + inverse */
  MLBDDC_PROF_NEGATE = 4,       /* sign flips between elimination phases (none are launched: the second
                                   phase reads the first phase's trailing block with the opposite sign) */
  MLBDDC_PROF_SCHUR_MV = 5,     /* S^ tile products (k_mv_tiles, FP64) */
  MLBDDC_PROF_PRECOND_MV = 6,   /* level-1 G_i tile products (k_mv_tiles, FP32 or FP64) */
  MLBDDC_PROF_N = 8
};
typedef struct {
  double time_s[MLBDDC_PROF_N];
  double flops[MLBDDC_PROF_N];
  int64_t launches[MLBDDC_PROF_N];
  int64_t tiles[MLBDDC_PROF_N];   /* tile tasks processed */
  double job_time_s[2];           /* wall time of the factorization jobs: [0] subdomain
                                     matrices (all levels), [1] constrained local problems */
  int32_t panel[2];               /* panel widths of the largest K and M jobs of the last set-up */
  double bytes[MLBDDC_PROF_N];    /* algorithmic bytes of the product classes */
  int32_t stage[2];               /* staged columns of the largest K and M jobs of the last set-up */
} mlbddc_profile;
mlbddc_status mlbddc_set_profiling(mlbddc_t h, int32_t enable);
mlbddc_status mlbddc_get_profile(mlbddc_t h, mlbddc_profile* out);

/* Release all device and host memory of the handle. */
mlbddc_status mlbddc_destroy(mlbddc_t h);

/* Description of the last failure on this handle (or of the last failed
 * mlbddc_create when h is NULL). */
mlbddc_status mlbddc_last_error(mlbddc_t h, mlbddc_error* info);

/* ---------------------------------------------------------------------------
 * Host-only helpers (no device needed).
 * ------------------------------------------------------------------------- */

/* Unit-modulus element matrix K_e^0 of a structured element of side h:
 * kind MLBDDC_POISSON_Q1 (4 x 4, -Laplace, bilinear square) or
 * MLBDDC_ELASTICITY_HEX8 (24 x 24, trilinear cube, isotropic with Poisson
 * ratio nu, 2x2x2 Gauss rule).  out: host, row-major. */
mlbddc_status mlbddc_element_matrix(int32_t kind, double h, double nu, double* out);

/* Consistent nodal load of a constant source / body force on one element:
 * out[node * ndof + c] = force[c] * volume / nodes. */
mlbddc_status mlbddc_element_load(int32_t kind, double h, const double* force, double* out);

/* Load vector of the free DOFs: f = sum over the mesh's elements of the
 * element load `elem_load` (host [nodes_per_elem * ndof_per_node], node-major,
 * e.g. from mlbddc_element_load), with the DOFs of Dirichlet nodes dropped.
 * f: host [n_free_dofs], overwritten.  E_ARG when n_free_dofs does not match
 * the mesh or a node index is out of range. */
mlbddc_status mlbddc_assemble_load(const mlbddc_mesh* mesh, const double* elem_load, double* f, int64_t n_free_dofs);

/* Plan the decomposition on the host only and report its structure:
 * counts[level-1][0..5] = {subdomains, interface DOFs, coarse DOFs, corners,
 * edges, faces} for levels 1..L-1.  counts: host [(L-1) * 6]. */
mlbddc_status mlbddc_plan_counts(const mlbddc_mesh* mesh, const mlbddc_partition* part, int64_t* counts);

/* Level-1 plan details for tests: interface free-DOF list (host
 * [interface_size]) and, for subdomain `sub`, its local interface DOFs as
 * interface indices (host [n_gamma]) with their multiplicity weights.
 * Pass NULL for outputs not wanted; *n_gamma receives the count. */
mlbddc_status mlbddc_plan_interface(const mlbddc_mesh* mesh, const mlbddc_partition* part, int64_t* iface_dofs,
                                    int32_t sub, int64_t* n_gamma, int64_t* sub_iface);

#ifdef __cplusplus
}
#endif
#endif /* MLBDDC_H */
