/*
 * sem.h -- C ABI of libsem, the MI355X (gfx950) spectral-element Helmholtz hot path.
 *
 * The operations follow Jansson et al., "Neko: a modern, portable, and
 * scalable framework for high-fidelity computational fluid dynamics"
 * (arXiv 2107.01243):
 *   - sem_ax_helm          the matrix-free element operator of Section 2, Eq. 9-10,
 *                          with the argument order of the ax_compute interface
 *                          (Section 3.1, Listing 1: w, u, coef, msh, Xh);
 *   - sem_gs_op            the gather-scatter QQ^T of Eq. 10 (Section 3.2,
 *                          Algorithm 1, its local gather + scatter);
 *   - sem_pcg_solve        the Jacobi-preconditioned CG of the velocity solve
 *                          (Section 4), in FP64 or as FP64 flexible CG around an
 *                          FP32 inner solve ("other precision formats", Section 10);
 *   - sem_ax_helm_adjoint  d(v^T A_L(h1) u)/d h1 per quadrature point, from the
 *                          linearity of Eq. 9 in the coefficient.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.  A "local" field holds n_p = nelv * lx^3 values, element-major, point
 *   (i,j,k) of element e at e*lx^3 + i + lx*(j + lx*k) (i fastest): the 4-D arrays
 *   of Listing 1.  nfields > 1 fields are stored back to back (field f starts at
 *   f * n_p).  Geometric factors are 6 planes of n_p values: G11, G22, G33, G12,
 *   G13, G23.
 * Memory.  Pointers documented "device" are caller-owned GPU allocations; "host"
 *   pointers are caller-owned CPU memory.  Handles and every internal buffer are
 *   owned by the library and released by the matching *_destroy call.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   sem_ax_helm, sem_gs_op, sem_mask and sem_ax_helm_adjoint only enqueue work
 *   and return.  sem_pcg_solve synchronises the stream to poll convergence.
 * Errors.  Every call returns a sem_status; nothing aborts or throws.  Invalid
 *   arguments are rejected before any launch.  sem_last_error() returns a
 *   thread-local description of the last failure.
 * Device.  Handles are bound to the HIP device current at creation; calls must
 *   be made with that device current.
 */
#ifndef SEM_H
#define SEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SEM_OK = 0,
    SEM_ERR_INVALID = -1,        /* bad argument (size, lx, NULL, aliasing, dtype)   */
    SEM_ERR_OOM = -2,            /* device or host allocation failed                  */
    SEM_ERR_HIP = -3,            /* a HIP runtime call failed (message has details)   */
    SEM_ERR_NOT_CONVERGED = -4,  /* solver hit max_iter; x and info are valid         */
    SEM_ERR_BREAKDOWN = -5,      /* non-positive or non-finite curvature in CG        */
    SEM_ERR_UNSUPPORTED = -6     /* valid request this library does not implement    */
} sem_status;

typedef enum { SEM_F64 = 0, SEM_F32 = 1 } sem_dtype;

/* Library limits: lx in [SEM_LX_MIN, SEM_LX_MAX]; nfields in {1, 3}. */
#define SEM_LX_MIN 2
#define SEM_LX_MAX 16

/* Stopping margin shared by every solver (sem_pcg_solve, sem_gmres_solve,
 * sem_proj_solve).  A solve asked for a relative tolerance rtol > 0 iterates until
 * both its recursive residual and its own FP64 evaluation of the true residual meet
 * |b - A x| <= SEM_RTOL_MARGIN * rtol * |b|.  Another FP64 evaluation of the same
 * residual (other summation order, FMA or not, geometric factors computed by other
 * code) differs by rounding of order eps * |A| |x|, which reaches ~15% of 1e-10 on
 * meshes of 1e8 points; the margin keeps such evaluations at or below rtol. */
#define SEM_RTOL_MARGIN 0.8

/* Size of the fixed device workspace of sem_pcg_solve_noalloc: at most
 * SEM_NOALLOC_MAX_POINTS = n_p * nfields local values per solve; the workspace holds
 * four vectors of that length, 2^17 reduction partials and 4 KiB of scalars. */
#define SEM_NOALLOC_MAX_POINTS (1 << 21)
#define SEM_NOALLOC_WORKSPACE_BYTES ((4LL * SEM_NOALLOC_MAX_POINTS + 131072 + 512) * 8)

typedef struct sem_space_s *sem_space; /* Xh: lx, GLL points/weights, D (Eq. 7-9)   */
typedef struct sem_mesh_s *sem_mesh;   /* msh: nelv, lx, global ids, Dirichlet mask  */
typedef struct sem_coef_s *sem_coef;   /* coef: G, B, h1, h2, Jacobi cache            */
typedef struct sem_gs_s *sem_gs;       /* gs: pair list + block lists for QQ^T        */
typedef struct sem_proj_s *sem_proj;   /* proj: previous-solution projection space    */

/* Flag for sem_coef_create*: also keep FP32 copies of G, B, D (needed by SEM_F32
 * calls and by the mixed-precision solve). */
#define SEM_COEF_F32 1u

/* ---------------------------------------------------------------- space (Xh)
 * GLL points xi (end points -1, +1, interior the roots of L'_N), weights
 * w_i = 2/(N(N+1) L_N(xi_i)^2) and the derivative matrix D[i*lx + l] = l_l'(xi_i)
 * of the degree-N Lagrange basis through them (Section 2, Eq. 7-9; Eq. 7 is
 * printed garbled in the paper and is read as that basis).
 * lx outside [SEM_LX_MIN, SEM_LX_MAX] -> SEM_ERR_INVALID. */
sem_status sem_space_create(int lx, sem_space *Xh);
/* Host copies: xi[lx], w[lx], D[lx*lx] (any may be NULL). */
sem_status sem_space_get(sem_space Xh, double *xi, double *w, double *D);
void sem_space_destroy(sem_space Xh);

/* ---------------------------------------------------------------- synthetic box mesh
 * Host helper producing the structured test meshes: nx*ny*nz hexahedra on
 * [0,1]^3, element e = ex + nx*(ey + ny*ez), node (i,j,k) at
 * ((ex + (xi_i+1)/2)/nx, (ey + (xi_j+1)/2)/ny, (ez + (xi_k+1)/2)/nz), then moved by
 * x += eps sin(2 pi y) sin(2 pi z), y += eps sin(2 pi z) sin(2 pi x),
 * z += eps sin(2 pi x) sin(2 pi y) (all evaluated at the undeformed point).
 * Global id = (ex*N+i) + Mx*((ey*N+j) + My*(ez*N+k)), M = n*N + 1 per direction.
 * dirichlet = 1 on the six walls (Eq. 5).  Outputs are host arrays of n_p
 * values (xyz: 3*n_p, x plane then y then z); any output may be NULL.
 * Note: the library takes its own GLL points from lx, so a mesh is tied to lx. */
sem_status sem_box_mesh(int nx, int ny, int nz, int lx, double eps,
                        int64_t *glb, uint8_t *dirichlet, double *xyz);

/* ---------------------------------------------------------------- mesh (msh)
 * glb_host: n_p = nelv*lx^3 global ids (any non-negative int64, "a unique global
 * number" per degree of freedom, Section 2).  dirichlet_host: n_p flags (nonzero =
 * homogeneous Dirichlet node, Eq. 5) or NULL for none.  Copies are taken.
 * The Dirichlet flags must agree on all copies of a global id (else INVALID). */
sem_status sem_mesh_create(int64_t nelv, int lx, const int64_t *glb_host,
                           const uint8_t *dirichlet_host, sem_mesh *msh);
sem_status sem_mesh_size(sem_mesh msh, int64_t *nelv, int *lx, int64_t *n_local,
                         int64_t *n_unique, int64_t *n_dirichlet_local);
void sem_mesh_destroy(sem_mesh msh);

/* ---------------------------------------------------------------- gather-scatter (gs)
 * Builds the QQ^T maps of Eq. 10 from the mesh's global ids (Section 3.2): local
 * indices are grouped by global id; ids with exactly two copies form the pair
 * list (the "injective" ids of Section 3.2), ids with more copies form variable
 * length blocks; ids with one copy are skipped.  Canonical order: pairs and
 * blocks by ascending global id, indices within a group ascending.  The sum
 * over a group is taken in that order, so sem_gs_op is bit-reproducible.
 * Indices are int32: n_p must be < 2^31. */
sem_status sem_gs_create(sem_mesh msh, sem_gs *gs);
sem_status sem_gs_sizes(sem_gs gs, int64_t *npairs, int64_t *nblocks, int64_t *nblock_entries);
/* Host copies of the maps: pairs[2*npairs] (a0,b0,a1,b1,...), blk_ptr[nblocks+1],
 * blk_idx[nblock_entries]; mult[n_p] (multiplicity of each local point, uint8,
 * may be NULL).  Any output may be NULL. */
sem_status sem_gs_export_maps(sem_gs gs, int32_t *pairs, int64_t *blk_ptr, int32_t *blk_idx,
                              uint8_t *mult);
void sem_gs_destroy(sem_gs gs);

/* u <- QQ^T u on nfields contiguous local fields (device, dtype dt), in place
 * (Eq. 10; Algorithm 1, local gather + scatter). */
sem_status sem_gs_op(void *u, int nfields, sem_gs gs, sem_dtype dt, void *stream);

/* u <- 0 on the mesh's Dirichlet points (Eq. 5), nfields contiguous fields. */
sem_status sem_mask(void *u, int nfields, sem_mesh msh, sem_dtype dt, void *stream);

/* ---------------------------------------------------------------- coefficients (coef)
 * Geometric factors of Eq. 9 from nodal coordinates xyz_dev (device FP64, 3*n_p:
 * x plane, y plane, z plane), isoparametric: metric = D applied to the
 * coordinates, J its determinant, G_ab = rho J grad r_a . grad r_b, B = rho J,
 * rho the tensor GLL weight.  Fails with SEM_ERR_INVALID if any J <= 0.
 * h1 = 1, h2 = 0 until sem_coef_set_helmholtz is called.  Enqueued on stream and
 * synchronised before return. */
sem_status sem_coef_create(sem_space Xh, sem_mesh msh, const double *xyz_dev, unsigned flags,
                           void *stream, sem_coef *coef);
/* Same, from given factors: G6_dev (device FP64, 6*n_p), B_dev (device FP64, n_p). */
sem_status sem_coef_create_from_G(sem_space Xh, sem_mesh msh, const double *G6_dev,
                                  const double *B_dev, unsigned flags, void *stream,
                                  sem_coef *coef);
/* Helmholtz coefficients A = h1 K + h2 B (Section 4: h1 = 1/Re, h2 = b0/dt).
 * h1_dev / h2_dev: device FP64 fields of n_p values (copied), or NULL to use the
 * scalar.  Invalidates the cached Jacobi diagonal. */
sem_status sem_coef_set_helmholtz(sem_coef coef, const double *h1_dev, double h1,
                                  const double *h2_dev, double h2, void *stream);
/* Device copies of the FP64 factors (G6_dev: 6*n_p, B_dev: n_p; either may be NULL). */
sem_status sem_coef_export(sem_coef coef, double *G6_dev, double *B_dev, void *stream);
void sem_coef_destroy(sem_coef coef);

/* ---------------------------------------------------------------- operators
 * w = A_L u on nfields (1 or 3) contiguous fields: per element
 * w = h1 D^T G D u + h2 B u (Eq. 9, unassembled; Eq. 10 is completed by
 * sem_gs_op).  u, w: device, dtype dt, nfields*n_p values, must not overlap.
 * dt = SEM_F32 needs a coef created with SEM_COEF_F32 (FP32 G, B, D, h1, h2). */
sem_status sem_ax_helm(void *w, const void *u, sem_coef coef, sem_mesh msh, sem_space Xh,
                       int nfields, sem_dtype dt, void *stream);

/* g_p = (D v)_p^T G_p (D u)_p at every local point = d(v^T A_L(h1) u)/d h1_p.
 * g, u, v: device, dtype dt, n_p values; g must not overlap u or v. */
sem_status sem_ax_helm_adjoint(void *g, const void *u, const void *v, sem_coef coef,
                               sem_mesh msh, sem_space Xh, sem_dtype dt, void *stream);

/* Jacobi inverse used by the solvers: dinv = 1 / QQ^T(diag A_L), 0 on Dirichlet
 * points (device FP64 output, n_p, caller-owned).  The preconditioner of the velocity
 * solves is Jacobi (Section 4); the paper does not define its blocks, and this is
 * point Jacobi: the exact diagonal of the assembled operator of Eq. 10, including the
 * G12/G13/G23 cross terms at element boundaries.  The result is also cached in coef
 * (recomputed after sem_coef_set_helmholtz).  Enqueued on stream. */
sem_status sem_jacobi_inverse(double *dinv, sem_coef coef, sem_mesh msh, sem_space Xh,
                              sem_gs gs, void *stream);

/* ---------------------------------------------------------------- solver */
typedef struct {
    double rtol;        /* stop when |r|/|b| <= SEM_RTOL_MARGIN * rtol (unique-node
                           2-norms) for the recursive residual and for the FP64 true
                           residual b - A x; <= 0: run exactly max_iter iterations   */
    int max_iter;       /* outer iteration cap (>= 1)                                 */
    int check_every;    /* host polls convergence every this many iterations (>= 1)   */
    int mixed;          /* 0: FP64 Jacobi-PCG.
                           1: Jacobi-PCG iterating in FP32 (FP32 operator, vectors and
                              preconditioner, FP64 dot accumulation) with FP64 reliable
                              updates: whenever the FP32 residual has dropped by `delta`,
                              x is accumulated in FP64, the true residual b - A x is
                              recomputed with the FP64 operator and replaces the FP32 one
                              (the search direction is kept); convergence is decided on
                              that FP64 residual.  max_iter caps the FP32 iterations.
                           2: FP64 flexible CG preconditioned by an FP32 Jacobi-PCG
                              inner solve (inner_rtol, inner_max_iter).
                           1 and 2 need a coef created with SEM_COEF_F32.               */
    double inner_rtol;  /* mixed: nominal relative tolerance of each inner solve; an
                           inner solve asks for no more than 0.1x the reduction still
                           needed to reach rtol (never tighter than inner_rtol, at most
                           0.5)                                                          */
    int inner_max_iter; /* mixed: iteration cap of each inner solve                    */
    int use_x0;         /* 1: x holds the initial guess on entry; 0: start from 0      */
    double delta;       /* mixed == 1: residual-replacement factor in (0, 1); 0 -> 0.5.
                           A segment shorter than 8 iterations squares it for the
                           next one (floor 1e-3), so fast-converging systems are not
                           replaced every iteration.                                */
    int variant;        /* mixed == 0 only.  0: two-reduction Jacobi-PCG (Hestenes-
                           Stiefel form); 1: single-reduction form (Chronopoulos-Gear):
                           both inner products of an iteration come from one pass, the
                           one reduction phase per iteration that Section 10 asks for
                           across GPUs; same iterates in exact arithmetic.          */
} sem_pcg_params;

typedef struct {
    int iters;          /* FP64: CG iterations; mixed 1: residual replacements;
                           mixed 2: outer flexible-CG iterations                        */
    int inner_iters;    /* mixed: total FP32 CG iterations                             */
    int converged;      /* 1 when the stopping test was met (sem_proj_solve: when
                           true_rel_res <= rtol)                                      */
    double rel_res;     /* recursive |r|/|b| at exit                                   */
    double true_rel_res;/* |b - A x|/|b| recomputed in FP64 at exit                    */
} sem_pcg_info;

/* Solve mask QQ^T A_L(h1,h2) x = b for nfields (1 or 3) independent fields.
 * b: device FP64, assembled and masked (b = mask QQ^T f), nfields*n_p values.
 * x: device FP64, in: guess (if use_x0), out: solution.  info: host array of
 * nfields entries (may be NULL).  Returns SEM_ERR_NOT_CONVERGED or
 * SEM_ERR_BREAKDOWN with x and info valid when a field fails. */
sem_status sem_pcg_solve(double *x, const double *b, int nfields, sem_coef coef, sem_mesh msh,
                         sem_space Xh, sem_gs gs, const sem_pcg_params *params,
                         sem_pcg_info *info, void *stream);

/* Allocation-free variant of sem_pcg_solve, for callers that cannot allocate device
 * memory (serving loops and harnesses that forbid hipMalloc, code that must not
 * change the device heap).  Same arguments, same iterates and results as
 * sem_pcg_solve with mixed = 0 and variant = 0 (the FP64 two-reduction Jacobi-PCG),
 * which is the only form it accepts.  Its scratch (CG vectors, Jacobi inverse,
 * reduction partials, scalars) lives in a fixed device workspace of
 * SEM_NOALLOC_WORKSPACE_BYTES (65 MiB) that every GPU the library runs on holds from
 * the first call until the process ends; the call allocates no device or pinned host
 * memory.  The Jacobi inverse is recomputed on every call (not cached in coef).
 * Errors (SEM_ERR_INVALID, before any launch): n_p * nfields above
 * SEM_NOALLOC_MAX_POINTS; a gs handle not yet resident on the device (any allocating
 * call that uses it -- sem_gs_op, sem_jacobi_inverse, sem_pcg_solve -- uploads it);
 * every error of sem_pcg_solve.  All calls on one GPU share the workspace, which keeps
 * the last call's contents: calls that overlap in time on one GPU (other host threads
 * or streams) race and must be serialised by the caller. */
sem_status sem_pcg_solve_noalloc(double *x, const double *b, int nfields, sem_coef coef, sem_mesh msh,
                                 sem_space Xh, sem_gs gs, const sem_pcg_params *params,
                                 sem_pcg_info *info, void *stream);

/* ---------------------------------------------------------------- GMRES
 * The paper's pressure equation is solved with GMRES (Section 4, Table 2).
 * Flexible GMRES(m) (Saad, Algorithm 9.6): right preconditioning with a
 * preconditioner that may change between steps, Arnoldi in the unique-node inner
 * product by classical Gram-Schmidt applied twice (for m <= 32 each vector's second
 * pass is made in the same passes over the data as the next vector's first), Givens
 * rotations, restart after m steps from the true residual b - A x.  Solves mask QQ^T A_L(h1, h2) x = b for one
 * field (x, b device FP64, b assembled and masked).  Converged when |b - A x| <= rtol |b|
 * for the true residual (checked at every restart and at exit; both the cycle's
 * least-squares estimate and that check use SEM_RTOL_MARGIN * rtol).  Device memory:
 * (2 m + 2) vectors of n_p values, kept by the coef handle between calls. */
typedef struct {
    double rtol;      /* > 0, relative to |b|                                          */
    int max_iter;     /* total Arnoldi steps (>= 1)                                    */
    int restart;      /* Krylov dimension m of one cycle, 1..200                       */
    int precond;      /* 0: point Jacobi (the exact assembled diagonal); 1: two-level
                         additive Schwarz (sem_schwarz_apply, overlap 0); 2: the same
                         with the one-point overlap (sem_schwarz_apply, overlap 1)     */
    int use_x0;       /* 1: x holds the initial guess on entry; 0: start from 0         */
    int coarse_iters; /* precond 1: CG steps of each coarse solve (0 -> 10)             */
} sem_gmres_params;
/* info: iters = Arnoldi steps, inner_iters = cycles (restarts + 1), rel_res and
 * true_rel_res = |b - A x| / |b| at exit.  SEM_ERR_NOT_CONVERGED with x valid when
 * max_iter is reached first. */
sem_status sem_gmres_solve(double *x, const double *b, sem_coef coef, sem_mesh msh, sem_space Xh,
                           sem_gs gs, const sem_gmres_params *params, sem_pcg_info *info, void *stream);

/* z = M0^{-1} r, the two-level additive overlapping Schwarz preconditioner of the
 * pressure solve (Section 4: M0^{-1} = R0^T A0^{-1} R0 + sum_k Rk^T Ak~^{-1} Rk, coarse grid
 * on linear elements solved by about ten CG iterations).  Local problem k: element k's
 * lx^3 points with homogeneous Dirichlet conditions one first-GLL-spacing beyond each
 * face (neighbouring problems overlap on the shared face points); Ak~ is the separable
 * box approximation h1 (Mt x Ms x Kr + Mt x Ks x Mr + Kt x Ms x Mr) + h2 Mt x Ms x Mr with,
 * per direction, the GLL stiffness and mass of the element length
 * L = 2 / sqrt(mean over the element of G_dd / B) and one linear segment of the first
 * spacing at each end, inverted by fast diagonalisation.  The local solutions are
 * summed over shared points (QQ^T) and divided by the multiplicity.  Coarse space:
 * trilinear functions of the element vertices (the corners' global ids), A0 = P^T A P
 * (Galerkin) on the free vertices, coarse_iters Jacobi-CG steps from zero (a fixed
 * count, so the preconditioner varies slightly between applications; GMRES is
 * flexible).  Needs scalar h1 and h2 (SEM_ERR_UNSUPPORTED otherwise).  r: device FP64,
 * assembled and masked; z: device FP64, not overlapping r.  The first call for a
 * (coef, gs) pair builds the data (host eigen-decompositions, eight operator
 * applications); changing h1 or h2 rebuilds it.  Device memory ~ (3 lx^2 + 3 lx + 8) per
 * element plus one byte per point, plus the coarse system.
 *
 * overlap = 1: the minimal overlap of one point (Section 4 names an overlapping
 * Schwarz method).  Every local problem also holds, beyond each face the element
 * shares with a neighbour (found from the global ids: the other element holding the
 * face's points, in any orientation), the layer of that neighbour's points one GLL
 * index inside it, with the neighbour's residual as right-hand side; along that
 * direction the extension node is joined to the face node by the first-spacing
 * segment and held by a Dirichlet condition one second GLL spacing beyond it.  Faces
 * without a neighbour keep the overlap-0 segment; the box's edge and corner points
 * get zero right-hand side.  Each local solution is kept on the element's own points
 * only (restricted additive Schwarz), then summed and averaged as above.  Extra
 * device memory ~ (3 (lx+2)^2 + 3 (lx+2)) doubles and 24 int32 per element, built on
 * the first overlap call; SEM_ERR_INVALID if a face is held by more than two elements
 * or two elements share a face's corners but not its points.  overlap: 0 or 1. */
sem_status sem_schwarz_apply(double *z, const double *r, sem_coef coef, sem_mesh msh, sem_space Xh,
                             sem_gs gs, int coarse_iters, int overlap, void *stream);

/* ---------------------------------------------------------------- projection space
 * Initial guesses from previous solutions (the paper keeps a space of 20 previous
 * pressure solutions, Section 4 and Table 2, following Nek5000).  The handle holds
 * up to max_vectors A-orthonormal vectors X_i, (X_i, A X_j) = delta_ij in the
 * unique-node inner product, and their images A X_i, for the operator of coef
 * (A = mask QQ^T A_L(h1, h2)) on one scalar field: 2 * max_vectors * n_p FP64
 * values of device memory plus four scratch vectors, owned by the handle.
 * The operator must not change while the space is in use: call sem_proj_reset
 * after changing h1 or h2.  The handle keeps pointers to coef, msh, Xh and gs,
 * which must outlive it.  Not thread-safe; calls are ordered on `stream`. */
sem_status sem_proj_create(sem_coef coef, sem_mesh msh, sem_space Xh, sem_gs gs, int max_vectors,
                           sem_proj *proj);
sem_status sem_proj_size(sem_proj proj, int *count, int *max_vectors, int *restarts);
sem_status sem_proj_reset(sem_proj proj);
/* x0 = sum_i (X_i, b) X_i, the best approximation of A^{-1} b from the space in the
 * A-norm (equivalently (X_i, b - A x0) = 0 for every i), and r = b - A x0 computed
 * from the stored images.  b assembled and masked; x0, r, b device FP64 (n_p values),
 * pairwise non-overlapping.  An empty space gives x0 = 0, r = b. */
sem_status sem_proj_project(sem_proj proj, double *x0, double *r, const double *b, void *stream);
/* Add the solution x of a system whose projection was x0: the new direction x - x0
 * is A-orthogonalised against the space (classical Gram-Schmidt, two passes, one
 * operator application) and appended unless it is dependent to rounding (*added = 0).
 * A full space restarts from x alone (counted in restarts). */
sem_status sem_proj_update(sem_proj proj, const double *x, const double *x0, int *added, void *stream);
/* Project, solve A dx = b - A x0 with sem_pcg_solve (params as there, rtol > 0,
 * relative to |b|: the correction solve stops once |b - A x| <= rtol |b|), set
 * x = x0 + dx, add x to the space.  info: iters / inner_iters of the correction
 * solve, rel_res and true_rel_res relative to |b|.  Returns what the correction
 * solve returned (SEM_ERR_NOT_CONVERGED with x valid). */
sem_status sem_proj_solve(double *x, const double *b, sem_proj proj, const sem_pcg_params *params,
                          sem_pcg_info *info, void *stream);
void sem_proj_destroy(sem_proj proj);

/* ---------------------------------------------------------------- measurement
 * STREAM triad a = b + s*c over n FP64 values (device, caller-owned, a must not
 * overlap b or c): the micro-benchmark the paper's performance model takes its
 * memory bandwidth beta from (Section 8).  Enqueued on stream. */
sem_status sem_stream_triad(double *a, const double *b, const double *c, double s, int64_t n,
                            void *stream);

/* ---------------------------------------------------------------- misc */
const char *sem_last_error(void);
const char *sem_version(void);
/* SEM_RTOL_MARGIN as built into the library. */
double sem_rtol_margin(void);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H */
