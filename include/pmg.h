/*
 * pmg.h -- C-ABI of libpmg.so: iterative solution of the Laplace problem of
 * fully nonlinear potential flow (Sec. 2, eq. laplaceproblem) discretised by
 * the Galerkin spectral element method on extruded, curvilinear prism meshes
 * (Sec. 3.1, eq. laplaceproblemdiscrete), solved by a Krylov method
 * preconditioned by geometric p-multigrid V-cycles that coarsen the
 * polynomial order P -> floor(P/2) -> ... -> 1 on one fixed mesh (Sec. 5,
 * Alg. 1-3), on one AMD Instinct MI355X (gfx950).
 *
 * Conventions
 *  - Status: 0 ok; > 0 warning (outputs valid); < 0 error.  On error the
 *    outputs are untouched unless stated; pmg_last_error() gives the message.
 *  - Pointers marked "device" are device memory of the context's GPU (for
 *    example torch tensor data_ptr()); "host" pointers are CPU memory.  The
 *    caller owns every pointer it passes; the context owns what it allocates
 *    and frees it in pmg_destroy().
 *  - `stream` is a hipStream_t (NULL = default stream); all device work is
 *    enqueued on it in order.  Calls that return host data synchronise it.
 *  - Indices are 0-based int32.  Global node numbering of level l
 *    (order P_l): g = id2d * (L*P_l + 1) + z, z = layer*P_l + c, with the 2D
 *    numbering documented at pmg_gather_map().  Element e = t*L + layer, local
 *    node n = c*Np_tri + a (c vertical LGL node, a triangle node).
 *  - A context is not thread safe; distinct contexts are independent.
 *  - Results are deterministic: the same inputs on the same device give
 *    bitwise identical outputs (fixed reduction order, no atomics in sums).
 */
#ifndef PMG_H
#define PMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PMG_ABI_VERSION 7

enum pmg_status {
  PMG_OK = 0,
  PMG_NOT_CONVERGED = 1,   /* imax reached; phi holds the last iterate       */
  PMG_FALLBACK_USED = 2,   /* learned guess rejected; baseline guess used     */
  PMG_EINVAL = -1,         /* bad argument                                    */
  PMG_ENOMEM = -2,         /* device allocation failed                        */
  PMG_EDEVICE = -3,        /* HIP runtime error                               */
  PMG_EBREAKDOWN = -4,     /* p^T A p <= 0 or z^T r <= 0 (indefinite M or A)   */
  PMG_ENONFINITE = -5,     /* NaN/Inf in boundary data or iterate             */
  PMG_EMESH = -6,          /* non-positive Jacobian (inverted element)        */
  PMG_ESTATE = -7          /* call not valid in this state (e.g. host-only)    */
};

/* Arithmetic of the preconditioner (Sec. 1 mentions mixed precision as a way to
 * accelerate multigrid; the outer residual and Krylov recurrences are always
 * FP64).
 *   PMG_MIXED_FP32   V-cycle vectors, geometric factors and MFMA operands in FP32
 *   PMG_MIXED_BF16   FP32 vectors; geometric factors and MFMA operands in BF16,
 *                    FP32 accumulation
 *   PMG_MIXED_BF16G  FP32 vectors and FP32 MFMA arithmetic on geometric factors
 *                    stored in BF16 (half the bytes of FP32 G, FP32 operands)
 *   PMG_MIXED_BF16X3 as BF16G, but every product of the element operator's
 *                    contractions is a_hi b_hi + a_hi b_lo + a_lo b_hi of BF16
 *                    parts (x_hi = bf16(x), x_lo = bf16(x - x_hi)) on BF16 MFMA
 *                    with FP32 accumulation: about 16 significant bits at BF16
 *                    matrix-core rates (levels of in-plane order 6; the
 *                    other levels run as BF16G)
 *   PMG_MIXED_BF16X2 as BF16X3 with the reference matrices rounded to BF16
 *                    (a_lo = 0): the element operator is that of slightly
 *                    perturbed reference matrices, still symmetric, applied
 *                    with vectors kept to about 16 bits; two BF16 MFMAs per
 *                    product (levels of in-plane order 6; the other levels
 *                    run as BF16G)
 * Vectors of the float V-cycle (pmg_apply, pmg_smooth, ...) are float for all
 * five. */
enum pmg_precision { PMG_FP64 = 0, PMG_MIXED_FP32 = 1, PMG_MIXED_BF16 = 2, PMG_MIXED_BF16G = 3,
                     PMG_MIXED_BF16X3 = 4, PMG_MIXED_BF16X2 = 5 };

/* Outer iteration: Alg. 3 (PCG), flexible PCG (Polak-Ribiere beta), Alg. 2
 * (preconditioned defect correction), stand-alone V-cycles. */
enum pmg_krylov { PMG_PCG = 0, PMG_FPCG = 1, PMG_PDC = 2, PMG_MG = 3 };

/* Initial guess of pmg_solve: the caller's phi, zero, the extrapolation
 * 2 phi_{n-1} - phi_{n-2} of the two previous solutions plus the learned
 * correction (falls back to the extrapolation when its residual is not
 * smaller), or the extrapolation alone.  The ...3 forms use the third-order
 * extrapolation 3 phi_{n-1} - 3 phi_{n-2} + phi_{n-3} of three previous
 * solutions as the base (a network for LEARNED3 is trained on targets and
 * features relative to that base: pmg_features with p3). */
enum pmg_guess { PMG_GUESS_GIVEN = 0, PMG_GUESS_ZERO = 1, PMG_GUESS_LEARNED = 2, PMG_GUESS_EXTRAP = 3,
                 PMG_GUESS_EXTRAP3 = 4, PMG_GUESS_LEARNED3 = 5 };

/* Coarsest (P = 1) level of Alg. 1: exact solve through a dense inverse of the
 * free-node matrix, or a fixed-degree Jacobi-preconditioned Chebyshev
 * iteration on [lmin, lmax] (a linear, symmetric approximation). */
enum pmg_coarse { PMG_COARSE_EXACT = 0, PMG_COARSE_CHEBYSHEV = 1 };

/* Smoother of eq. sec_form on every non-coarsest level: damped Jacobi
 * (S^-1 = omega D^-1, nu sweeps), Chebyshev-accelerated Jacobi (a degree-nu
 * polynomial in D^-1 A, linear and symmetric, so Alg. 3 applies unchanged), or
 * the overlapping additive Schwarz preconditioner of Sec. 5.2 (eq. Mass,
 * eq. weights): S^-1 = W sum_k R_k^T (R_k A R_k^T)^-1 R_k with one subdomain
 * per prism (the prism's nodes plus the overlap of pmg_options.overlap in the
 * prisms that touch it, Dirichlet nodes left out) and W the inverse count of
 * subdomains holding each node; nu sweeps damped by omega.  Pre-
 * smoothing uses S^-1, post-smoothing its transpose sum_k R_k^T A_k^-1 R_k W,
 * so the V-cycle stays symmetric.  The local inverses are dense (FP64, with
 * FP32 and BF16 copies for the mixed V-cycles) and are rebuilt by every
 * pmg_set_surface. */
enum pmg_smoother { PMG_SMOOTH_JACOBI = 0, PMG_SMOOTH_CHEBYSHEV = 1, PMG_SMOOTH_SCHWARZ = 2 };

typedef struct pmg_ctx pmg_ctx;
typedef struct pmg_net pmg_net;

/* Triangle mesh of the xy-plane extruded over n_layers uniform sigma layers
 * between a flat bottom z = -depth and the free surface z = eta (Sec. 3.1,
 * Sec. 6.2).  Host memory, read only during pmg_create. */
typedef struct pmg_mesh {
  int32_t nv;
  const double* xy;          /* [nv][2] vertex coordinates                      */
  int32_t nt;
  const int32_t* tri;        /* [nt][3] counter-clockwise vertex ids            */
  const int32_t* edge_tag;   /* [nt][3] tag (0..31) of edge (tri[i], tri[i+1]); 0 interior */
  int32_t ncurved;
  const int32_t* curved_edge;/* [ncurved][2] vertex pairs on a circle (nullable) */
  const double* circle;      /* [ncurved][3] cx, cy, R (nullable)               */
  int32_t n_layers;          /* >= 1; nt * n_layers < 2^31 prisms and fewer than 2^32 nodes on
                                the finest level (PMG_EINVAL otherwise) */
  double depth;
} pmg_mesh;

typedef struct pmg_options {
  int32_t P;              /* finest triangle order, 1..8 (vertical order: PZ)   */
  int32_t nu1, nu2;       /* pre/post smoothing sweeps (Alg. 1) of the finest
                             level, and of every level unless nu1_coarse /
                             nu2_coarse say otherwise                          */
  double omega[8];        /* per level; <= 0: 4/(3*lambda) with lambda = 1.05 x
                             30-step power estimate of lambda_max(D^-1 A)
                             (Schwarz: of the spectral radius of S^-1 A, the
                             2-norm of the last step; the paper's form is 1)   */
  int32_t precision;      /* pmg_precision of the V-cycle                        */
  int32_t krylov;         /* pmg_krylov                                          */
  uint32_t dirichlet_tags;/* bit k set: lateral edges tagged k are Dirichlet      */
  int32_t top_neumann;    /* 1: no Dirichlet at the surface (pure Neumann tests) */
  int32_t coarse;         /* pmg_coarse                                          */
  int32_t cheb_degree;    /* Chebyshev steps of the coarse solve; <= 0: the degree
                             giving a 0.1 error reduction over [lmin, lmax]      */
  double cheb_lmin, cheb_lmax; /* interval of D^-1 A; <= 0: estimated (below)      */
  double cheb_ratio;      /* > 0: lmax from a power estimate, lmin = lmax/ratio;
                             <= 0: both from 120 Lanczos steps (0.9 x smallest,
                             1.05 x largest Ritz value)                          */
  int32_t exact_max;      /* largest free coarse size for the dense inverse      */
  uint64_t seed;          /* counter-based start vector of the power iterations  */
  int32_t host_only;      /* 1: numbering only, no device memory (queries only)  */
  int32_t kernel_variant; /* 0: MFMA element operator where available, 1: generic */
  int32_t smoother;       /* pmg_smoother                                         */
  double smooth_ratio;    /* Chebyshev smoother interval [lambda/ratio, lambda],
                             lambda = 4/(3 omega) of the level                   */
  int32_t coarsening;     /* pmg_coarsening: order sequence of the levels        */
  int32_t overlap;        /* Schwarz overlap: a node of a touching prism joins
                             subdomain k when it lies within `overlap` lattice
                             steps in the triangle and along the extrusion of the
                             entity the two prisms share (0: block Jacobi, 1: one
                             overlapping node in each direction, Sec. 5.2); -1:
                             the refined variant of Sec. 6.3, ceil((P_l+1)/2) in
                             the triangle and ceil((PZ_l+1)/2) vertically      */
  int32_t schwarz_store;  /* Schwarz local inverses kept: bit 0 FP64, bit 1 FP32,
                             bit 2 BF16 (0: all three).  A smoothing step in a
                             precision whose copy is not kept fails with EINVAL.
                             The set-up works in FP64 chunks of
                             schwarz_chunk entries                             */
  int64_t schwarz_chunk;  /* entries of an FP64 set-up chunk; <= 0: 2^29 (4 GiB) */
  int32_t geometry;       /* pmg_geometry of the MFMA element operators          */
  int32_t PZ;             /* finest vertical order, 1..8; <= 0: P.  The geometry
                             is the isoparametric map of triangle order P on
                             every level (the sigma map is affine along the
                             extrusion inside a layer, so PZ does not change it).
                             Level orders must be among those the library builds
                             (pmg_create fails with PMG_EINVAL otherwise): any
                             isotropic P; with PZ != P the EQUAL sequences of
                             (4,2), (5,3), (6,4), (2,4), (3,6), (4,8) and the
                             XY_FIRST sequences of (3,6), (2,4), (4,8)           */
  int32_t fused_sum;      /* 1: where the MFMA element operator can (layer
                             counts dividing 16, orders up to 16 (node, prism)
                             pairs per thread, column-factor geometry for
                             FP64/FP32), it sums each triangle column's layers
                             itself and writes one value per (triangle, node,
                             z); a node kernel then adds the triangles sharing
                             each vertex or edge node and applies the step's
                             epilogue (the direct-stiffness sum of Sec. 3.1).
                             0 (default, as fast on the benchmark meshes):
                             element results through the element layout and
                             the node-centric sum kernel.  Both use no atomics
                             and a fixed order (bitwise reproducible); they
                             differ by rounding                               */
  int32_t graphs;         /* 1: inside pmg_solve the preconditioner's V-cycle
                             (its kernels and arguments fixed while the context
                             is unchanged) is captured once as a HIP graph on
                             the caller's stream and replayed: the first
                             V-cycle after a change of the context (surface,
                             parameters, solver, reuse mode, stream) runs
                             eagerly, the next is captured.  Results are
                             bitwise those of the eager V-cycle.  Never on the
                             null stream.  0 (default): always eager; on the
                             benchmark meshes the GPU never waits for the
                             host's launches, so replay gains nothing there,
                             and each capture costs a V-cycle's launches    */
  int32_t dss;            /* direct-stiffness sum of the element-layout results
                             (Sec. 3.1): 0 (default) node-centric, one thread
                             per node gathering its triangles' values in
                             ascending order; 1 coloured: the triangles are
                             coloured so that no two of a colour share a node
                             (pmg_dss_colours), each colour's triangle columns
                             are added into an L-vector in one launch, and one
                             more pass applies the step's epilogue.  No
                             atomics and a fixed order either way (bitwise
                             reproducible); the two differ by rounding.
                             fused_sum, where it applies, takes precedence   */
  int32_t nu1_coarse, nu2_coarse; /* pre/post sweeps of the levels below the
                             finest (the coarsest level is solved, never
                             smoothed); < 0 (default): nu1, nu2, one pair for
                             every level as Alg. 1 passes it down the
                             recursion.  Fewer sweeps there are a tuning: the
                             V-cycle stays symmetric while each level's pre and
                             post counts agree                                  */
} pmg_options;

/* Geometric factors read by the MFMA element operators.  STORED: the six
 * factors of G = w det(J) J^-1 J^-T (the metric of the weak form, Sec. 3.1) at
 * every cubature point of every prism, streamed from memory.  COLUMN
 * (default): the prisms of a column are the sigma-transform of one triangle
 * (eq. jacobian: z = -h + s (eta + h), s affine in each layer), so G at
 * vertical point k of layer l is
 * zw_k (B0, B1, s B2, B3, s B4, s^2 B5 + B6) with seven factors B per
 * triangle cubature point shared by the column; the kernels read those and form
 * G in registers, in the precision of their arithmetic (FP64, FP32).  The BF16
 * and BF16G precisions keep their stored BF16 factors (BF16X3 and BF16X2 on
 * the levels without their split kernels too). */
enum pmg_geometry { PMG_GEOM_STORED = 0, PMG_GEOM_COLUMN = 1 };

/* Order sequence of the levels, from the finest (P, PZ); each coarsening step
 * takes an order p to max(1, floor(p/2)).  BOTH: both orders together (Sec. 5,
 * Table BTcoarse: 6 -> 3 -> 1).  XY_FIRST: the triangle order is coarsened
 * first with the vertical order kept, then the vertical order, (P,PZ) ->
 * (P/2,PZ) -> ... -> (1,PZ) -> (1,PZ/2) -> ... -> (1,1): in-plane
 * semi-coarsening for prisms whose in-plane node spacing is much finer than
 * the vertical one.  EQUAL: semi-coarsening of the direction of higher order,
 * each step to max(lower order, floor(higher/2)), until the two agree, then
 * both together (Sec. 6.2, Table BTcoarse3D: (5,3) -> (3,3) -> (1,1); with
 * PZ > P the vertical order goes first). */
enum pmg_coarsening { PMG_COARSEN_BOTH = 0, PMG_COARSEN_XY_FIRST = 1, PMG_COARSEN_EQUAL = 2 };

typedef struct pmg_level_info {
  int32_t order;          /* P_l: order on the triangle */
  int32_t np;             /* nodes per prism (P+1)(P+2)/2 (PZ+1) */
  int32_t nq;             /* cubature points per prism (P+1)^2 (PZ+1) */
  int32_t n_colours;
  int64_t n_dof;          /* all global nodes of the level */
  int64_t n_free;         /* nodes not on the Dirichlet boundary */
  int64_t n_elem;
  int64_t n_surface;      /* 2D nodes = surface nodes of the level */
  int32_t order_z;        /* PZ_l: order along the extrusion */
} pmg_level_info;

typedef struct pmg_stats {
  int32_t iters;          /* outer iterations performed */
  int32_t n_hist;         /* entries of res_hist (iters + 1, capped at 512) */
  double rel_res;         /* ||f - A phi||_2 / ||f||_2 over free nodes, FP64 (stop-test quantity) */
  double norm_f;          /* ||f||_2 of the lifted right-hand side */
  double res_hist[512];   /* ||r_m||_2, m = 0..iters; q_m = res_hist[m]/res_hist[m-1] (eq. convrate) */
  double t_solve_ms;      /* wall time of pmg_solve on the stream (hipEvents) */
  double t_guess_ms;      /* part spent building the initial guess */
  int32_t fallback;       /* 1 if a learned guess was rejected */
  int32_t n_vcycles;      /* preconditioner applications */
  int32_t n_fine_applies; /* FP64 fine-operator applications */
  int32_t n_graph_vcycles;/* V-cycles replayed from a captured graph (pmg_options.graphs) */
} pmg_stats;

/* Fill `opt` with defaults: P=6, nu1=nu2=2, auto omega, FP64, PCG, exact
 * coarse solve with exact_max=12000 (Chebyshev: Lanczos interval, automatic
 * degree). */
void pmg_options_default(pmg_options* opt);

/* Build the level hierarchy: numbering, gather maps, colouring, reference
 * matrices and transfers of every level (Sec. 5, Sec. 5.1), and device
 * buffers.  The geometry is set by pmg_set_surface() (flat eta = 0 after
 * create).  Errors: EINVAL (bad sizes/order), EMESH (degenerate triangle),
 * ENOMEM, EDEVICE; message from pmg_global_error(). */
int pmg_create(const pmg_mesh* mesh, const pmg_options* opt, pmg_ctx** out);
void pmg_destroy(pmg_ctx* ctx);
const char* pmg_last_error(const pmg_ctx* ctx);
const char* pmg_global_error(void);
int pmg_abi_version(void);

int pmg_n_levels(const pmg_ctx* ctx);
int pmg_level_info_get(const pmg_ctx* ctx, int level, pmg_level_info* info);

/* Gather map of level `level`, host [n_elem][np]: global node of local node
 * n of element e.  2D numbering: vertex v -> v; edge-interior node m = 1..P-1
 * counted from the lower vertex id -> nv + edge*(P-1) + m-1, edges being the
 * (min,max) vertex pairs sorted lexicographically; triangle-interior node of
 * rank k (local order: j outer, i inner) -> nv + ne*(P-1) + t*(P-1)(P-2)/2 + k.
 * Bit-exact contract. */
int pmg_gather_map(const pmg_ctx* ctx, int level, int32_t* map);
/* Greedy element colouring (host [n_elem]): ascending elements take the
 * smallest colour not used by a lower element sharing a node. */
int pmg_colours(const pmg_ctx* ctx, int level, int32_t* colour);
/* Triangle colouring of the coloured direct-stiffness sum (pmg_options.dss,
 * host [n_triangles]): ascending triangles take the smallest colour not used
 * by a lower triangle sharing a vertex (triangles sharing any 2D node share a
 * vertex).  Host-only contexts too. */
int pmg_dss_colours(const pmg_ctx* ctx, int level, int32_t* colour);
/* xy of the surface (= 2D) nodes of the finest level, host [n_surface][2]. */
int pmg_surface_xy(const pmg_ctx* ctx, double* xy);
/* 1 for Dirichlet nodes of a level, host [n_dof]. */
int pmg_dirichlet_mask(const pmg_ctx* ctx, int level, uint8_t* mask);

/* Set the free surface: eta at the finest-level surface nodes (device
 * [n_surface] FP64).  Nodes follow z = -depth + sigma*(eta + depth) (Sec. 3.1's
 * sigma coordinate with d = eta + h); recomputes the geometric factors of all
 * levels at their cubature points from the finest isoparametric map, the
 * Jacobi diagonals, omega (when automatic) and the coarse solver.
 * Errors: EMESH if any det J <= 0 (context keeps its previous surface). */
int pmg_set_surface(pmg_ctx* ctx, const double* eta, void* stream);
/* xyz of the global nodes of a level under the current surface, host [n_dof][3]. */
int pmg_node_xyz(pmg_ctx* ctx, int level, double* xyz);

/* y = A_l x (stiffness of level l, eq. laplaceproblemdiscrete with A = -L).
 * precision PMG_FP64: x, y double; PMG_MIXED_FP32 / PMG_MIXED_BF16: x, y float
 * with FP32 or BF16 geometric factors.  flags bit 0: mask (x and y taken as
 * zero on Dirichlet nodes, i.e. A_FF). Device [n_dof]. */
int pmg_apply(pmg_ctx* ctx, int level, int precision, int flags, const void* x, void* y, void* stream);
/* Diagonal of A_l (device double [n_dof]). */
int pmg_diagonal(pmg_ctx* ctx, int level, double* d, void* stream);
/* Damped Jacobi sweeps u <- u + omega D^-1 (f - A u) on free nodes (eq. sec_form). */
int pmg_smooth(pmg_ctx* ctx, int level, int precision, int sweeps, const void* f, void* u, void* stream);
/* Nested-space transfers between level l and l+1 (Sec. 5.1): prolongation
 * interpolates and averages over the elements sharing a node; restriction is
 * its transpose (eq. rest).  Both zero on Dirichlet nodes. */
int pmg_prolong(pmg_ctx* ctx, int level, int precision, const void* xc, void* yf, void* stream);
int pmg_restrict(pmg_ctx* ctx, int level, int precision, const void* xf, void* yc, void* stream);
/* Coarsest-level solve of Alg. 1 (exact or Chebyshev, per options). */
int pmg_coarse_solve(pmg_ctx* ctx, int precision, const void* f, void* u, void* stream);
/* One V-cycle of Alg. 1 from a zero guess: z = M^-1 r on the finest level. */
int pmg_vcycle(pmg_ctx* ctx, int precision, const void* r, void* z, void* stream);
/* Coarse solver in use: mode (pmg_coarse), Chebyshev degree and interval,
 * free unknowns of the coarsest level. */
int pmg_coarse_info(const pmg_ctx* ctx, int* mode, int* degree, double* lmin, double* lmax, int64_t* n_free);
/* Smoothing weights and coarse interval in use.  Values set here (> 0) are
 * kept by later pmg_set_surface calls instead of being re-estimated: the
 * t = 0 parameters are reused along a time history (Sec. 6, strategy I). */
int pmg_get_params(const pmg_ctx* ctx, double* omega /*[n_levels]*/, double* cheb_lmin, double* cheb_lmax);
int pmg_set_params(pmg_ctx* ctx, const double* omega /*[n_levels] or NULL*/, double cheb_lmin, double cheb_lmax);

/* Solve A phi = b (b = 0: no-flux walls, bottom and bodies) with phi = Dirichlet
 * data on the Dirichlet nodes (lifting f = -A phi_D), to
 * ||f - A phi||_2 <= rtol ||f||_2 + atol (stop test of Sec. 5), with the outer
 * iteration and precision of the options.
 *  phi_surf: device [n_surface] values at the surface nodes, or NULL;
 *  phi_bc:   device [n_dof] values read at every Dirichlet node, or NULL
 *            (required when lateral Dirichlet tags are set);
 *  phi:      device [n_dof]; in: guess (GUESS_GIVEN), out: solution.
 *  net:      learned model for GUESS_LEARNED(3) (else NULL); hist_phi: host
 *            array of device pointers to the previous solutions [n_dof],
 *            newest first: two for LEARNED/EXTRAP, three for LEARNED3/EXTRAP3,
 *            else NULL.
 *  stats:    host, may be NULL.
 * Returns OK, NOT_CONVERGED (phi = last iterate), FALLBACK_USED, or an error
 * (EBREAKDOWN, ENONFINITE, EINVAL, EDEVICE). */
int pmg_solve(pmg_ctx* ctx, const double* phi_surf, const double* phi_bc, double* phi, int guess_mode,
              const pmg_net* net, const double* const* hist_phi, double rtol, double atol, int32_t imax,
              pmg_stats* stats, void* stream);

/* Subdomains of the Schwarz smoother on a non-coarsest level (available in
 * host-only contexts too).  dt, dz: overlap in lattice steps in the triangle
 * and along the extrusion; n_sub: subdomains (one per prism); max_size:
 * largest subdomain; total: sum of the subdomain sizes; inv_entries: entries
 * of the kept local inverses in one precision (each stored as the 32 x 32
 * tiles of its upper block triangle, ceil(n/32) (ceil(n/32) + 1) / 2 tiles).
 * EINVAL when the smoother is not PMG_SMOOTH_SCHWARZ or the level is the
 * coarsest. */
typedef struct pmg_schwarz_info {
  int32_t dt, dz;
  int64_t n_sub;
  int32_t max_size;
  int64_t total;
  int64_t inv_entries;
} pmg_schwarz_info;
int pmg_schwarz_info_get(const pmg_ctx* ctx, int level, pmg_schwarz_info* info);
/* Free global nodes of every subdomain, ascending (host buffers: ptr
 * [n_sub+1], nodes [total]; subdomain k is nodes[ptr[k] .. ptr[k+1])).
 * Bit-exact contract. */
int pmg_schwarz_nodes(const pmg_ctx* ctx, int level, int32_t* ptr, int32_t* nodes);

/* Operator reuse across surfaces (Sec. 6, Fig. simstrats).
 * NONE: every pmg_set_surface rebuilds the operators of all levels from the
 *   new surface (NONLIN on every level: the paper's strategy III).
 * T0: the preconditioner of the surface current at this call is kept (the
 *   paper's strategy I: S^-1 and the coarse operators of t = 0).  Later
 *   pmg_set_surface calls update only the finest level's FP64 geometric
 *   factors, which the outer iteration (and the FP64 V-cycle's finest level)
 *   applies; coarse operators, diagonals, Schwarz inverses, the coarse solve
 *   and the finest level's FP32 / BF16 factors of the mixed V-cycle stay.
 * LIN: the coarse levels are rebuilt once on the flat surface eta = 0 (the
 *   linear formulation on every level but the finest: the paper's strategy
 *   II) and kept; the finest level, its smoother data included, follows every
 *   surface.
 * T0 and LIN fix the smoothing weights and the coarse Chebyshev interval and
 * degree at their current values (pmg_set_params changes them).  EINVAL for
 * an unknown mode. */
enum pmg_reuse { PMG_REUSE_NONE = 0, PMG_REUSE_T0 = 1, PMG_REUSE_LIN = 2 };
int pmg_set_reuse(pmg_ctx* ctx, int mode, void* stream);

/* Change the preconditioner precision and the outer iteration of later solves
 * (pmg_precision, pmg_krylov).  The hierarchy is kept. */
int pmg_set_solver(pmg_ctx* ctx, int precision, int krylov);

/* Kernels that pmg_time_kernel() can time in isolation. */
enum pmg_kernel { PMG_K_ELEMENT_OP = 0, PMG_K_ASSEMBLE = 1, PMG_K_GEOMETRY = 2, PMG_K_RESTRICT = 3,
                  PMG_K_PROLONG = 4, PMG_K_COPY = 5, PMG_K_SCHWARZ = 6, PMG_K_COLSUM_OP = 7,
                  PMG_K_COL_SUM_STORE = 8, PMG_K_COL_SUM_CHEB = 9 };
/* Average duration (ms) of `reps` back-to-back launches of one kernel of
 * level `level` on `stream`, bracketed by hipEvents on that stream (for
 * roofline measurement).  The element operator reads the level's work vector;
 * results are discarded.  PMG_K_ASSEMBLE is the direct-stiffness sum of the
 * element layout with the store epilogue, in the form pmg_options.dss selects
 * (node-centric, or every colour pass and the epilogue pass of the coloured
 * sum).  PMG_K_COPY is a plain device copy of the level's
 * FP64 vector (n_dof * 8 bytes read and written): the reference point that
 * scales hardware byte counters.  PMG_K_PROLONG is the prolongation from
 * level + 1 to `level` as the V-cycle runs it (node-wise where the level pair
 * keeps one order, else element-wise with its averaging sum).  PMG_K_SCHWARZ is the batched local solve of
 * the Schwarz smoother (inverse storage: FP64 for PMG_FP64, FP32 for
 * PMG_MIXED_FP32, BF16 for the BF16 precisions); EINVAL when the smoother is
 * not PMG_SMOOTH_SCHWARZ or the level is the coarsest.  PMG_K_COLSUM_OP: the
 * element operator writing column sums (pmg_options.fused_sum); PMG_K_COL_SUM_STORE
 * / PMG_K_COL_SUM_CHEB: the node kernel that sums them, with the epilogue
 * y = A x or a Chebyshev smoothing step (r -= A d; d = w d + c D^-1 r;
 * x += d); EINVAL where the level has no column-sum path. */
int pmg_time_kernel(pmg_ctx* ctx, int kernel, int level, int precision, int reps, double* ms_per_launch,
                    void* stream);

/* ---- free-surface time stepping (eq. FSeta, eq. FSphi; ERK4 as in Sec. 6.1,
 * Sec. 6.2) ------------------------------------------------------------------
 * State: eta and the surface potential phi~ at the finest-level surface nodes
 * (device [n_surface] FP64, the 2D node order of pmg_surface_xy).  Each
 * right-hand side sets the surface to the stage's eta (pmg_set_surface: an
 * inverted element gives EMESH), solves the Laplace problem with phi = phi~
 * at the surface (pmg_solve with the context's precision and outer
 * iteration), and evaluates
 *   eta_t  = -grad eta . grad phi~ + w~ (1 + |grad eta|^2)
 *   phi~_t = -g eta - 1/2 (|grad phi~|^2 - w~^2 (1 + |grad eta|^2)).
 * grad: x and y derivatives of the order-P interpolant on every triangle
 * (isoparametric map), averaged over the triangles sharing a node.  w~: the
 * derivative of phi along the column of the top prism at the surface node,
 * times 2L / (eta + depth) (d/dz at fixed x, y under the sigma map).
 * The first call fixes the smoothing weights and the coarse Chebyshev
 * interval and degree at their current values for all later surfaces (the
 * parameter part of the paper's strategy I); geometric factors, diagonals and
 * the coarse operator follow every surface. */

/* (fx, fy) = horizontal gradient of a surface field f (device [n_surface] each). */
int pmg_surface_grad(pmg_ctx* ctx, const double* f, double* fx, double* fy, void* stream);
/* w~ of a finest-level field phi (device [n_dof]) under the current surface:
 * w (device [n_surface]). */
int pmg_surface_w(pmg_ctx* ctx, const double* phi, double* w, void* stream);
/* deta = eta_t, dphis = phi~_t at (eta, phis), g the gravitational
 * acceleration.  phi (device [n_dof]) receives the Laplace solution; with
 * warm != 0 it is also the initial guess of the solve.  stats (nullable)
 * receives the solve's statistics.  Returns the solve's status (OK or
 * NOT_CONVERGED; the right-hand side is evaluated either way) or an error. */
int pmg_fnpf_rhs(pmg_ctx* ctx, const double* eta, const double* phis, double g, double* phi, int32_t warm,
                 double rtol, double atol, int32_t imax, double* deta, double* dphis, pmg_stats* stats,
                 void* stream);
typedef struct pmg_fnpf_stats {
  int32_t iters[4];       /* outer iterations of the four stage solves */
  double rel_res[4];      /* their final relative residuals */
  double t_step_ms;       /* wall time of the step on the stream (hipEvents) */
  double t_solve_ms;      /* part spent in the four pmg_solve calls */
  int32_t status;         /* worst stage status */
} pmg_fnpf_stats;
/* One classical fourth-order Runge-Kutta step of (eta, phis) over dt, in
 * place.  phi carries the Laplace solution from stage to stage.  Stage solves
 * start from a prediction linear in time over steps of dt/2: the first from
 * phi when warm != 0 (the last stage's solution of the previous step), else
 * from zero; the second (t + dt/2) from 2 phi(t) - phi(t - dt/2) when the
 * previous call was a step of the same dt (its third stage), else from
 * phi(t); the third from the second's solution; the fourth (t + dt) from
 * 2 phi(t + dt/2) - phi(t).  On return phi holds the last stage's solution.  On
 * an error eta and phis are left unchanged; NOT_CONVERGED stages are
 * reported in stats and the step completes.  The context's surface is the
 * last stage's afterwards. */
int pmg_fnpf_erk4(pmg_ctx* ctx, double* eta, double* phis, double dt, double g, double* phi, int32_t warm,
                  double rtol, double atol, int32_t imax, pmg_fnpf_stats* stats, void* stream);

/* ---- learned warm start (a small multilayer perceptron, FP32) -------------
 * The network maps per-node features of the network level (pmg_net_level: the
 * coarsest level, order (1,1)) to the correction of the extrapolated guess;
 * pmg_solve prolongates it to the finest level with the multigrid transfers.  Features of node g = (vertex v,
 * level z) with gf its finest-level twin and top the finest surface node of
 * column v: [z/L, x, y scaled to [-1,1], distance to the nearest circle,
 * p1[gf]-p2[gf], surf[v]-base[top], p1[top]-p2[top]]; target
 * pnow[gf] - base[gf], with base = 2 p1 - p2, or 3 p1 - 3 p2 + p3 when p3 is
 * given.  Layers: dense y = x W + b (W fan_in x fan_out
 * row-major), SiLU on hidden layers, linear scalar output; MSE loss; Adam
 * (0.9, 0.999, 1e-8) with bias correction.  Flat parameter order: W_0, b_0,
 * W_1, b_1, ...  pmg_net_forward / pmg_net_loss_grad act on raw inputs; the
 * solve and pmg_net_train use the normalisation (inputs (x - mean) * inv_std,
 * output times tscale) fitted by pmg_net_train. */
/* Index of the network level (its n_dof is the row count n1 of the features). */
int pmg_net_level(const pmg_ctx* ctx);
/* Features (device float [n1][7]) and, if T and pnow are given, targets
 * (device float [n1]) of the network level's nodes; surf device [n_surface], p1, p2,
 * p3 (nullable: second-order base), pnow device [n_dof] of the finest level. */
int pmg_features(pmg_ctx* ctx, const double* surf, const double* p1, const double* p2, const double* p3,
                 const double* pnow, float* X, float* T, void* stream);
/* Network with `depth` hidden layers of `width` units on the context's GPU;
 * weights uniform in +-1/sqrt(fan_in) from the counter generator of `seed`. */
int pmg_net_create(const pmg_ctx* ctx, int32_t width, int32_t depth, uint64_t seed, pmg_net** out);
void pmg_net_destroy(pmg_net* net);
int pmg_net_size(const pmg_net* net, int64_t* n_params, int32_t* d_in, int32_t* width, int32_t* depth);
/* host copies of the parameters and the normalisation (any pointer may be NULL) */
int pmg_net_get_params(const pmg_net* net, float* theta, float* mean, float* inv_std, double* tscale);
int pmg_net_set_params(pmg_net* net, const float* theta, const float* mean, const float* inv_std, double tscale);
/* raw network output y (device [rows]) of inputs X (device [rows][d_in]) */
int pmg_net_forward(pmg_net* net, const float* X, int64_t rows, float* y, void* stream);
/* pmg_net_forward for callers that cannot allocate device memory at the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same output, bit for bit, with the
 * hidden activations in a fixed 8 MiB array per GPU (rows in chunks of 4096,
 * two 4096 x 256 FP32 halves) instead of buffers the network allocates on
 * first use.  Calls no hipMalloc/hipFree.  Networks whose hidden width exceeds
 * 256 are rejected with PMG_EINVAL (message in pmg_global_error).  X (device
 * [rows][d_in]) and y (device [rows]) are the caller's; rows = 0 does nothing.
 * Every call on one GPU shares that GPU's array and keeps the previous call's
 * contents: calls that overlap on one GPU (other streams, other threads, other
 * networks) race and must be serialised by the caller. */
int pmg_net_forward_noalloc(pmg_net* net, const float* X, int64_t rows, float* y, void* stream);
/* raw MSE loss of a batch and its gradient (host [n_params], nullable); the
 * gradient also stays on the device for pmg_net_adam_step */
int pmg_net_loss_grad(pmg_net* net, const float* X, const float* T, int32_t rows, double* loss, float* grad,
                      void* stream);
int pmg_net_adam_step(pmg_net* net, double lr, void* stream);
/* fit the normalisation to (X, T) (device [rows][d_in], [rows]) and run `steps`
 * Adam steps on mini-batches drawn with the counter generator; final_loss =
 * mean normalised loss of the last 20 steps */
int pmg_net_train(pmg_net* net, const float* X, const float* T, int64_t rows, int32_t steps, int32_t batch,
                  double lr, uint64_t seed, double* final_loss, void* stream);
/* versioned binary file with an FNV-1a checksum; load requires equal shapes */
int pmg_net_save(const pmg_net* net, const char* path);
int pmg_net_load(pmg_net* net, const char* path);

#ifdef __cplusplus
}
#endif
#endif /* PMG_H */
