/*
 * hmx.h -- C ABI of libhmx, the MI355X (gfx950) H-matrix boundary-element operator library.
 *
 * Problem statement (Alouges & Aussal, "FEM and BEM simulations with the Gypsilab framework",
 * arXiv 1804.00995):
 *   - a triangulated surface and a quadrature rule per triangle give the points and weights
 *     (x_k, w_k) of the discretisation (Section 3: integrals are sums over the simplices' Gauss
 *     points with their weights; Section 4.2, a domain is a mesh plus a quadrature formula);
 *   - the BEM matrices are products around the dense kernel matrix G_kl = G(x_k, y_l)
 *     (Section 5, eq. (BEM)), with the Helmholtz kernel G(x, y) = e^{ik|x-y|} / (4 pi |x-y|)
 *     (Section 5.2, eq. (Helmholtz));
 *   - given a tolerance, the same matrices are returned compressed as H-matrices and used through
 *     the usual matrix product (Section 5.3); without it they are dense (Section 5.1).
 * The operator built here is the collocation form at the quadrature points with source weights,
 *   K = G W_y,  K_ml = G(x_m, x_l) w_l,  and K_ml = 0 when x_m = x_l,
 * applied to complex vectors.  The compression (cluster tree, admissibility, partially pivoted
 * ACA) is not described in the paper; libhmx uses a bounding-box bisection tree, the
 * admissibility min(diam) <= eta * dist, and ACA with the Frobenius-norm stopping rule at tol.
 * On top of these operators: the Galerkin P1 system of the acoustic example and the EFIE, MFIE
 * and CFIE on RWG elements of the electromagnetic one (Sections 5.4 and 5.5), with their GMRES
 * solves.
 *
 * Conventions for every entry point:
 *   - every function returns an hmx_status (0 = success); on failure nothing is returned through
 *     the out-arguments, no partial operator exists, and hmx_last_error() gives a message
 *     (thread-local, valid until the next call on the same thread);
 *   - "device" pointers are HIP device memory on the current device; "host" pointers are host
 *     memory; the library never takes ownership of caller memory and copies what it keeps;
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream);
 *   - complex vectors are interleaved (re, im): double pairs for HMX_FP64 operators, float pairs
 *     for HMX_FP32_MIXED operators; operator vectors have one entry per quadrature point, in the
 *     original triangle-major order m = n_q * t + q (the P1 and RWG spaces' vectors: one entry
 *     per vertex or per edge).
 */
#ifndef HMX_H
#define HMX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HMX_OK = 0,
  HMX_EINVAL = -1,       /* invalid argument (checked before any work is enqueued) */
  HMX_ENOMEM = -2,       /* device or host allocation failed */
  HMX_EDEVICE = -3,      /* a HIP runtime call or kernel failed */
  HMX_EUNSUPPORTED = -4, /* valid request outside what this library supports */
  HMX_EINTERNAL = -5     /* internal consistency check failed */
} hmx_status;

typedef enum {
  HMX_LAPLACE = 0,    /* G = 1 / (4 pi r) */
  HMX_HELMHOLTZ = 1,  /* G = e^{ikr} / (4 pi r) */
  /* Gradient kernels (Section 5.1: kernels such as grady[exp(ikr)/r]j, the j-th component of
   * the gradient in y): dG/dy_j = e^{ikr} (ikr - 1) (y_j - x_j) / (4 pi r^3), Laplace at k = 0;
   * 0 at r = 0.  Combined with the source normals they give the double-layer operator. */
  HMX_GRADY_X = 2,
  HMX_GRADY_Y = 3,
  HMX_GRADY_Z = 4,
  HMX_TEST_POLY2 = 99 /* test only: G = (1 + x.y)^2, exact separable rank 10 */
} hmx_kernel;

typedef enum {
  HMX_FP64 = 0,      /* everything in FP64, vectors c128 */
  HMX_FP32_MIXED = 1 /* blocks, factors and vectors in FP32 (c64); distance, phase k*r, ACA
                        pivots and norms in FP64 */
} hmx_precision;

typedef enum {
  HMX_RANK_ADAPTIVE = 0, /* plain adaptive ACA: each block's factors grow in slots taken from a
                            device pool as its rank grows */
  HMX_RANK_LEARNED = 1   /* the factor pool is reserved (and checked against the device
                            memory) from the rank MLP's predictions, and blocks are scheduled by
                            predicted work; blocks past their prediction continue adaptively */
} hmx_rank_model;

typedef struct {
  int32_t struct_size;   /* sizeof(hmx_params): ABI guard */
  double tol;            /* ACA tolerance; tol <= 0 builds the dense operator */
  int32_t leaf_size;     /* cluster-tree leaf size L (split while a node holds > L points) */
  double eta;            /* admissibility: far when min(diam) <= eta * dist */
  int32_t precision;     /* hmx_precision */
  int32_t rank_model;    /* hmx_rank_model */
  int32_t initial_rank;  /* adaptive mode: first rank capacity per far block (>= 1) */
  double force_pred_scale; /* learned mode: multiplies the predicted rank (tests force overflow) */
  int32_t force_rank_cap;  /* > 0: caps every far block's ACA rank (tests force dense fallback) */
  int64_t pool_limit_bytes; /* > 0: fail with HMX_ENOMEM when the operator would exceed this */
  /* ACA schedule (results may differ in rounding between schedules, not in method):
   * far blocks with m + n >= aca_big_mn run in aca_big_threads-thread workgroups, those with
   * m, n <= 64 one per wavefront, the others in aca_mid_threads-thread workgroups; blocks with m + n >= aca_gram_min_mn
   * take the cross terms from Gram matrices (one read of the factors per step); aca_serial = 1
   * runs the three classes one after the other instead of on three concurrent streams.
   * hmx_autotune picks these for a workload. */
  int32_t aca_big_mn;      /* >= 2 (default 4096) */
  int32_t aca_gram_min_mn; /* >= 0 (default 1024) */
  int32_t aca_serial;      /* 0 or 1 (default 0) */
  int32_t aca_mid_threads; /* workgroup size of the blocks between the wavefront and the
                              large-block classes: 256, 128 (default) or 64 */
  int32_t aca_arena;       /* 1 (default): each workgroup places its blocks' factors one after
                              the other in arenas taken from the slot pool, a block keeping
                              exactly rank (m + n) entries (no copies); 0: every block starts
                              in a pool slot of its own of initial_rank columns and doubles */
  /* Row share (the part of the operator one of row_shares devices would hold): with
   * row_shares = 2^s > 1, the operator keeps only the rows of cluster-tree node number
   * row_share (breadth-first order) at level s, against all columns; the product then writes
   * K x on those rows and 0 elsewhere, and the shares' products sum to the whole product.
   * Requires tol > 0 and a single mesh; HMX_EUNSUPPORTED when the tree has a leaf above level
   * s or a block would cross the share's boundary. */
  int32_t row_shares; /* power of two >= 1 (default 1) */
  int32_t row_share;  /* 0 <= row_share < row_shares (default 0) */
  int64_t force_pool_bytes; /* > 0: size of the first ACA slot pool (tests force further rounds) */
  int32_t max_far_mn; /* > 0 (default 12288): an admissible pair with more than max_far_mn
                         points (m + n) is split into its children's pairs instead of becoming
                         one far block (smaller ranks, less ACA work and better balance per
                         block); 0: no limit (the plain admissibility recursion) */
  int32_t aca_big_threads; /* workgroup size of the blocks with m + n >= aca_big_mn: 512 (one
                              workgroup per CU), 256 (two per CU in FP64, three in FP32) or 0
                              (default: 512 for FP64, 256 for FP32) */
  int32_t aca_small_mn; /* >= 0 (default 1024): blocks with m + n below it (other than the
                           wavefront blocks) run in 64-thread workgroups holding 256 ACA
                           coefficients, many per CU, with direct cross sums whatever
                           aca_gram_min_mn says; 0 puts them in the middle class */
  int32_t aca_wave; /* 1: blocks with m, n <= 64 run one per wavefront with their factors in
                       registers; 0 (default): they go to the small-block class, which was
                       measured faster on MI355X (FP64 by about 2 ms at 245 760 points) */
  /* Singular correction (Section 5.2, regularization of the kernels): with regularize = 1 every
   * close pair of the near field gets, on top of its kernel entry, the exact y-integral of the
   * 1/(4 pi r) part over the source triangle minus that part's Gauss value (nothing is subtracted
   * for r = 0, whose entry is 0).  The three rule points of a triangle carry the linear function
   * through their values, so the rule must have 3 non-collinear points.  A pair (x, point of
   * triangle T) is close when |x - centroid(T)| <= reg_radius * (longest edge of T); close pairs
   * that fall in far blocks keep the plain kernel.  Needs a mesh (hmx_build, hmx_build_batch;
   * HMX_EINVAL for hmx_build_points), the Laplace or Helmholtz kernel (else HMX_EINVAL) and
   * tol > 0 (HMX_EUNSUPPORTED for the dense operator).  The correction is assembled into the
   * near-field blocks: the product costs the same with or without it. */
  int32_t regularize; /* 0 (default) or 1 */
  double reg_radius;  /* > 0 (default 2) */
  /* Near field (Section 4: terms may be stored or computed on the fly): 0 (default) assembles
   * the near blocks once in the build and the product reads them; 1 stores nothing and the
   * product evaluates each near entry G(x_i, y_j) w_j again, from source tiles staged in LDS
   * (the same entries, so the same product up to rounding; no near-field memory, no assembly
   * time, about one kernel evaluation per near entry per product).  1 needs regularize = 0
   * (HMX_EUNSUPPORTED otherwise: the correction lives in stored blocks); ignored by dense
   * operators (tol <= 0), whose product is always computed on the fly.  With near_mode = 1,
   * hmx_matvec_multi applies the operator one vector at a time. */
  int32_t near_mode;
  /* > 0: initial capacity, in pairs, of the block recursion's frontier and list buffers (tests
   * force the path that enlarges them and runs the recursion again); 0: from the leaf count. */
  int64_t force_block_cap;
} hmx_params;

/* Fills `p` with the defaults: tol 1e-3, leaf 64, eta 1.5, FP64, adaptive ranks,
 * initial_rank 16, force_pred_scale 1, no rank cap, no pool limit, ACA schedule 4096 / 1024 /
 * concurrent / arenas, one row share, far blocks up to 12288 points, no singular correction
 * (reg_radius 2), stored near field. */
hmx_status hmx_params_default(hmx_params* p);

typedef struct hmx_op hmx_op; /* opaque, library-owned; free with hmx_destroy */

/* Quadrature points and weights of a triangle mesh (Section 3: points and weights over all
 * simplices; Section 4.2: mesh + quadrature formula).
 *   vtx  device, n_vtx x 3 doubles, row-major vertex coordinates;
 *   tri  device, n_tri x 3 int32, 0-based vertex indices;
 *   q_bary host, n_q x 3 barycentric coordinates; q_w host, n_q reference weights (sum 1);
 *   xyzw device output, 4 x M doubles (M = n_q * n_tri): X[M], Y[M], Z[M], W[M] with
 *        x_{n_q t + q} = sum_j q_bary[q][j] * vtx[tri[t][j]], W = area(t) * q_w[q].
 * Errors: HMX_EINVAL for null pointers, n_q < 1, a rule whose weights do not sum to 1 within
 * 1e-12 or whose barycentrics leave the triangle, a triangle index out of range, or a
 * non-finite vertex coordinate (the last two are detected on the device). Synchronous. */
hmx_status hmx_quad_points(const double* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                           const double* q_bary, const double* q_w, int32_t n_q, double* xyzw,
                           void* stream);

/* Builds the operator K = G W_y of a triangle mesh with a quadrature rule (arguments as in
 * hmx_quad_points) for kernel `kern` and wavenumber k >= 0 (Section 5.1 / 5.3: dense without a
 * tolerance, H-matrix with one).  With p->tol > 0 the H-matrix is built on the device: cluster
 * tree, block tree, near-field blocks, ACA on far blocks.  `p` may be NULL for the defaults.
 * Synchronous: returns when the operator is complete.  On success *out owns all of its device
 * memory. Errors: HMX_EINVAL (arguments as above, k < 0, leaf_size < 1, eta <= 0),
 * HMX_ENOMEM, HMX_EDEVICE, HMX_EUNSUPPORTED (more than 2^23 points in H-matrix mode). */
hmx_status hmx_build(const double* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                     const double* q_bary, const double* q_w, int32_t n_q, int32_t kern, double k,
                     const hmx_params* p, void* stream, hmx_op** out);

/* Same as hmx_build from given points: xyzw device, 4 x M doubles laid out as in
 * hmx_quad_points (X, Y, Z, W).  Vectors then follow the order of these points. */
hmx_status hmx_build_points(const double* xyzw, int64_t M, int32_t kern, double k,
                            const hmx_params* p, void* stream, hmx_op** out);

/* The potential of a source quadrature at other points (Section 5.1: the matrix
 * C_ij = int G(x_i, y) psi_j(y) dy for a collection of points x_i, with the y-integral by the
 * quadrature of eq. (BEM)): K_il = G(t_i, x_l) w_l for Mt targets t_i and Ms sources (x_l, w_l),
 * e.g. the field radiated onto points off the surface.
 *   txyz device, 3 x Mt doubles: the targets' X[Mt], Y[Mt], Z[Mt];
 *   xyzw device, 4 x Ms doubles: the sources as in hmx_build_points (from hmx_quad_points).
 * hmx_matvec then takes x with Ms entries (source order) and writes y with Mt entries (target
 * order).  With tol > 0 the targets and the sources get a cluster tree each (two roots of one
 * forest) and the block tree pairs target clusters with source clusters only; tol <= 0 gives the
 * dense operator.  A target that coincides with a source gets 0 from it.  Errors: as
 * hmx_build_points; HMX_EINVAL for Mt < 1 or Ms < 1 and for the singular correction (it needs a
 * mesh), HMX_EUNSUPPORTED for row shares and for more than 2^23 - 1 points in total in H-matrix
 * mode.  Synchronous. */
hmx_status hmx_build_rect(const double* txyz, int64_t Mt, const double* xyzw, int64_t Ms,
                          int32_t kern, double k, const hmx_params* p, void* stream,
                          hmx_op** out);

/* Galerkin P1 operator (eq. (BEM) with test and trial functions: A = Phi^T W_x K Phi, Phi[k, v]
 * the P1 hat function of vertex v at quadrature point k, W_x the point weights, K = G W_y the
 * operator) and its iterative solve, as in the paper's acoustic example (Section 5.4: the Galerkin
 * single-layer equation of the sound-soft sphere, with the kernel's correction).
 * hmx_p1_create: the P1 space of the mesh `op` was built on (hmx_build with the same vtx, tri
 * and rule; the caller keeps op alive while the space is used).  vtx, tri device arrays as in
 * hmx_build; q_bary, q_w host.  Errors: HMX_EINVAL for null pointers, a rule or mesh that
 * hmx_build rejects, or an operator whose point count is not n_q n_tri (or one built by
 * hmx_build_rect); HMX_EUNSUPPORTED for a row-share operator.  Synchronous. */
typedef struct hmx_p1 hmx_p1;
hmx_status hmx_p1_create(const hmx_op* op, const double* vtx, int64_t n_vtx, const int32_t* tri,
                         int64_t n_tri, const double* q_bary, const double* q_w, int32_t n_q,
                         void* stream, hmx_p1** out);
void hmx_p1_destroy(hmx_p1* p); /* NULL is accepted */
/* xp = Phi xv (xv: n_vtx entries, xp: n_q n_tri, original point order) and yv = Phi^T W zp;
 * device vectors of the operator's complex type (c128 or c64).  Asynchronous on `stream`. */
hmx_status hmx_p1_interp(const hmx_p1* p, const void* xv, void* xp, void* stream);
hmx_status hmx_p1_project(const hmx_p1* p, const void* zp, void* yv, void* stream);
/* yv = A xv = Phi^T W K Phi xv (n_vtx entries each; the space holds the scratch, so products on
 * one space must not overlap in time).  Asynchronous on `stream`; allocates nothing. */
hmx_status hmx_galerkin_matvec(const hmx_p1* p, const void* xv, void* yv, void* stream);
/* Solves A x = b by restarted GMRES(restart) from x = 0: classical Gram-Schmidt with one
 * reorthogonalisation, stopping when the residual estimate is at most tol ||b|| or after
 * max_iter products.  b, x device (n_vtx entries, the operator's complex type; x is
 * overwritten).  *iters receives the products spent and *relres ||b - A x|| / ||b|| of the
 * returned x (the true residual; the caller compares it with tol).  Inner products accumulate
 * in FP64.  Errors: HMX_EINVAL for null pointers, restart outside [1, 1000], max_iter < 0 or a
 * negative or non-finite tol.  Synchronous. */
hmx_status hmx_gmres(const hmx_p1* p, const void* b, void* x, int32_t restart, int32_t max_iter,
                     double tol, void* stream, int32_t* iters, double* relres);

/* Electromagnetic scattering (Section 5.5) on lowest-order Raviart-Thomas (RWG) elements
 * (Section 4): one unknown per edge of a closed, consistently oriented mesh, edges numbered in
 * increasing (a, b), a < b their vertex numbers.  On triangle t the edge opposite local vertex j
 * carries psi(y) = s l / (2 A) (y - p_j) (l its length, A the area, p_j the opposite vertex,
 * s = +1 on the triangle whose vertex order runs a -> b along the edge, -1 on the other), with
 * divergence s l / A; n = (v1 - v0) x (v2 - v0) / |.| is outward for an outward-oriented mesh.
 * The CFIE matrix, for beta in [0, 1], is
 *   A = -beta T + (1 - beta) (Id / 2 - NxK),
 *   T = i k sum_d Psi_d^T W K Psi_d - (i / k) D^T W K D       (EFIE; K the single layer),
 *   NxK_ij = int int (n x psi_i)(x) . (grad_y G(x, y) x psi_j(y)) dx dy   (MFIE double layer),
 *   Id the RWG mass matrix,
 * all integrals by the point quadrature; beta = 1 is the EFIE (as -T), beta = 0 the MFIE.
 * hmx_rwg_create: the space of the mesh the operators were built on (hmx_build with the same
 * vtx, tri and rule): `single` the Helmholtz single layer (kernel HMX_HELMHOLTZ, with or without
 * the correction) for beta > 0, grad_x/y/z the kernels HMX_GRADY_X/Y/Z for beta < 1 (all three
 * or none), one wavenumber k > 0 and one precision; the caller keeps them alive while the space
 * is used.  vtx, tri device arrays as in hmx_build; q_bary, q_w host.  Errors: HMX_EINVAL for
 * null pointers, missing or mismatched operators, a mesh that is not closed and consistently
 * oriented (every edge in exactly two triangles, run in opposite directions) or that hmx_build
 * rejects; HMX_EUNSUPPORTED for row-share operators.  Synchronous. */
typedef struct hmx_rwg hmx_rwg;
hmx_status hmx_rwg_create(const hmx_op* single, const hmx_op* grad_x, const hmx_op* grad_y,
                          const hmx_op* grad_z, const double* vtx, int64_t n_vtx,
                          const int32_t* tri, int64_t n_tri, const double* q_bary,
                          const double* q_w, int32_t n_q, void* stream, hmx_rwg** out);
void hmx_rwg_destroy(hmx_rwg* r); /* NULL is accepted */
/* Number of edges (unknowns), and the edges' vertex pairs (device int32, 2 per edge, a < b;
 * asynchronous on `stream`). */
hmx_status hmx_rwg_n_edges(const hmx_rwg* r, int64_t* n_edges);
hmx_status hmx_rwg_edges(const hmx_rwg* r, int32_t* edges, void* stream);
/* u = the field sum_e x_e psi_e at the quadrature points: 4 n_q n_tri entries, component-major
 * (J_x, J_y, J_z, div J), original point order; x has n_edges entries.  Device vectors of the
 * operators' complex type.  Asynchronous on `stream`. */
hmx_status hmx_rwg_interp(const hmx_rwg* r, const void* x, void* u, void* stream);
/* b_i = beta <psi_i, E_inc> - (1 - beta) <n x psi_i, H_inc>: the CFIE right-hand side from the
 * incident fields at the quadrature points (3 n_q n_tri entries each, component-major; e_inc
 * may be NULL when beta = 0, h_inc when beta = 1).  Asynchronous on `stream`. */
hmx_status hmx_rwg_rhs(const hmx_rwg* r, double beta, const void* e_inc, const void* h_inc,
                       void* b, void* stream);
/* y = A x (n_edges entries each): 4 single-layer products for beta > 0 and 6 gradient-kernel
 * products for beta < 1.  The space holds the scratch, so products on one space must not
 * overlap in time.  Errors: HMX_EINVAL for null pointers, beta outside [0, 1] or an operator the
 * beta needs that the space lacks.  Asynchronous on `stream`; allocates nothing. */
hmx_status hmx_cfie_matvec(const hmx_rwg* r, double beta, const void* x, void* y, void* stream);
/* Solves A x = b by restarted GMRES as hmx_gmres does (same stopping rule and reports).
 * Errors: as hmx_cfie_matvec and hmx_gmres.  Synchronous. */
hmx_status hmx_cfie_gmres(const hmx_rwg* r, double beta, const void* b, void* x, int32_t restart,
                          int32_t max_iter, double tol, void* stream, int32_t* iters,
                          double* relres);

/* One surface of a batch: vtx, tri device arrays as in hmx_build, and the surface's wavenumber. */
typedef struct {
  const double* vtx;
  int64_t n_vtx;
  const int32_t* tri;
  int64_t n_tri;
  double k;
} hmx_mesh;

/* Builds one operator for n_meshes independent surfaces that share the quadrature rule, the
 * kernel and the parameters (each surface keeps its own wavenumber).  The result is the
 * block-diagonal operator diag(K_0, ..., K_{n-1}) on the concatenated points: the points of mesh
 * i occupy [off_i, off_{i+1}) with off_0 = 0 and off_{i+1} = off_i + n_q * meshes[i].n_tri, and
 * the surfaces never interact (each gets its own cluster tree under a common forest, and blocks
 * pair clusters of one surface only).  All surfaces are built and applied together, so one set
 * of launches serves the whole batch.  Vectors for hmx_matvec are the per-mesh vectors
 * concatenated in mesh order; each slice is that mesh's product K_i x_i.  meshes host array.
 * Requires p->tol > 0 (the dense form is the single-mesh hmx_build).  Errors: as hmx_build for
 * each mesh, HMX_EINVAL for n_meshes < 1 or tol <= 0, HMX_EUNSUPPORTED for more than 2^23 - 1
 * points in total.  Synchronous.
 * There is no product over an array of separate operators: the batch is one operator, so that
 * hmx_matvec (and a graph of it) applies every mesh in one launch set, and hmx_mesh_offsets
 * gives each mesh's slice of x and y. */
hmx_status hmx_build_batch(const hmx_mesh* meshes, int32_t n_meshes, const double* q_bary,
                           const double* q_w, int32_t n_q, int32_t kern, const hmx_params* p,
                           void* stream, hmx_op** out);

/* Mesh offsets of an operator: *n_meshes receives the number of meshes (1 for operators built
 * by hmx_build / hmx_build_points / hmx_build_rect, whose offsets are {0, length of x}); off
 * (host, may be NULL) receives n_meshes + 1 offsets when cap >= n_meshes + 1, else HMX_EINVAL. */
hmx_status hmx_mesh_offsets(const hmx_op* op, int64_t* off, int32_t cap, int32_t* n_meshes);

/* y = K x (Section 5.3: the compressed matrix applied through the product).
 *   x, y device, M complex entries each (c128 for FP64 operators, c64 for FP32 ones), in the
 *   original point order (an hmx_build_rect operator: x has Ms entries, y Mt); x and y must not
 *   alias.
 * Asynchronous on `stream`; allocates nothing and performs no host synchronisation, so it can
 * be captured in a HIP graph.  The operator holds the product's scratch vectors: products on
 * the same operator must not overlap in time (different operators are independent).
 * Errors: HMX_EINVAL for null pointers. */
hmx_status hmx_matvec(const hmx_op* op, const void* x, void* y, void* stream);

/* y_r = K x_r for r < nr (Section 5.3, as hmx_matvec, for several vectors at once): an H-matrix
 * operator is applied to groups of four, then two, then one vector, each group in one product
 * that reads the operator's entries once; a dense operator takes one product per vector.  The
 * result of each vector is bit-identical to hmx_matvec's (same summation order).
 *   x, y: host arrays of nr device pointers, each vector as in hmx_matvec; no y[r] may equal
 *   any x[q] or another y[q] (HMX_EINVAL).
 *   work: device scratch of hmx_matvec_multi_work_bytes(op) bytes (0 for a dense operator, where
 *   work may be NULL), owned by the caller; products using the same work buffer or operator
 *   must not overlap in time.
 * Asynchronous on `stream`; allocates nothing.  Errors: HMX_EINVAL for null pointers, nr < 1,
 * aliased vectors or a missing work buffer. */
hmx_status hmx_matvec_multi_work_bytes(const hmx_op* op, size_t* bytes);
hmx_status hmx_matvec_multi(const hmx_op* op, int32_t nr, const void* const* x, void* const* y,
                            void* work, void* stream);

/* hmx_matvec_multi without a work buffer, for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc).  The scratch is a
 * static device array of HMX_STATIC_WORK_BYTES bytes inside the library, one on each device it
 * runs on, held until the process ends; its address is looked up once per device on the first
 * call there (that call synchronises nothing but may load the library's code object).  Results
 * are bit-identical to hmx_matvec_multi's.  Every call on one device shares that device's array:
 * calls that overlap in time on one device (any streams, any operators) race and give wrong
 * results; calls in order on one stream, or separated by synchronisation, are safe.  Nothing in
 * the array needs clearing between calls (every entry a product reads it has written first).
 * Asynchronous on `stream`; allocates nothing (no hipMalloc, no library allocation).
 * Errors: as hmx_matvec_multi; HMX_EINVAL when hmx_matvec_multi_work_bytes(op) exceeds
 * HMX_STATIC_WORK_BYTES; HMX_EDEVICE when the array's device address cannot be obtained. */
#define HMX_STATIC_WORK_BYTES ((size_t)64 << 20)
hmx_status hmx_matvec_multi_static(const hmx_op* op, int32_t nr, const void* const* x,
                                   void* const* y, void* stream);

/* Product replay: hmx_matvec(op, x, y) captured once into a HIP graph (fixed operator and
 * vector addresses) and replayed with one launch per call.  The graph holds kernels only.
 * hmx_graph_create captures on a private stream and instantiates (synchronous); hmx_graph_launch
 * enqueues `reps` replays on `stream` (asynchronous); the operator must outlive the graph and
 * replays follow the same no-overlap rule as hmx_matvec. */
typedef struct hmx_graph hmx_graph;
hmx_status hmx_graph_create(const hmx_op* op, const void* x, void* y, hmx_graph** out);
hmx_status hmx_graph_launch(hmx_graph* g, int32_t reps, void* stream);
void hmx_graph_destroy(hmx_graph* g); /* NULL is accepted */

/* Autotuner of the build schedule (max_far_mn, aca_big_mn, aca_gram_min_mn, aca_mid_threads,
 * aca_big_threads, aca_small_mn, aca_wave, aca_serial of hmx_params).  Times
 * hmx_build_points(xyzw, M, kern, k) under a grid of settings, each stage at the best of the
 * previous ones: far-block bounds {none, 32768, 16384, 12288, 8192}; class thresholds {2048, 4096,
 * 8192, none} x Gram thresholds {0, 1024, 4096, none} on concurrent streams; middle-class
 * workgroups {256, 128, 64}; large-block workgroups {512, 256}; small-block bounds {512, 2048,
 * none}; the other wavefront setting; serial classes; best of two builds each.  *out receives *p (defaults when
 * NULL) with the fastest settings, *best_ms (may be NULL) that build time in ms.
 * cache_path (host string, may be NULL): a JSON file of earlier choices keyed by device
 * architecture, precision, kernel, floor(log2 M), tolerance decade, leaf size, eta and the rank
 * model; a key found there is returned without timing, a new one is added to the file.  Synchronous; builds
 * and frees up to 63 operators (31 settings, two builds each, one warm-up).  Errors: as
 * hmx_build_points, HMX_EINVAL for tol <= 0 or an unwritable cache file. */
hmx_status hmx_autotune(const double* xyzw, int64_t M, int32_t kern, double k,
                        const hmx_params* p, const char* cache_path, void* stream,
                        hmx_params* out, double* best_ms);

/* The same search for a batch (hmx_build_batch of meshes, n_meshes, q_bary, q_w, n_q, kern,
 * with *p's method, precision and rank model): each setting is timed on the whole batch build.
 * Cache key as hmx_autotune's with "|batch<n_meshes>" after the kernel and M the total number
 * of points; a learned-layout search (p->rank_model = HMX_RANK_LEARNED, model set) is keyed
 * apart ("|learned") from an adaptive one.  Synchronous; builds and frees up to 63 batch
 * operators.  Errors: as hmx_build_batch, HMX_EINVAL for tol <= 0 or an unwritable cache. */
hmx_status hmx_autotune_batch(const hmx_mesh* meshes, int32_t n_meshes, const double* q_bary,
                              const double* q_w, int32_t n_q, int32_t kern, const hmx_params* p,
                              const char* cache_path, void* stream, hmx_params* out,
                              double* best_ms);

typedef struct {
  int64_t n_points, n_nodes, n_leaves, n_near, n_far;
  int64_t near_entries;   /* sum of m*n over near blocks */
  int64_t far_entries;    /* sum of r*(m+n) over low-rank far blocks */
  int64_t dense_far;      /* far blocks stored dense (ACA not converged at the rank cap) */
  int64_t dense_far_entries;
  int64_t max_rank, sum_rank;
  int64_t overflow_blocks; /* blocks moved to a larger slot, or continued in a later round */
  int64_t bytes;           /* device bytes held by the operator (slot pools trimmed to use) */
  int32_t precision, is_dense;
  double t_tree_ms, t_blocks_ms, t_near_ms, t_aca_ms, t_total_ms; /* build phases (events) */
  int64_t kernel_evals;    /* Green-kernel evaluations spent in the build (near entries only when
                            * they are stored: near_mode 0) */
  int64_t factor_bytes;    /* device bytes of the slots holding far-block factors (used part) */
  int64_t predicted_entries; /* learned layout: sum of r_alloc * (m + n) over far blocks */
  /* ACA by block class: [0] m + n >= aca_big_mn (aca_big_threads-thread workgroups), [1] the
   * other workgroup blocks (aca_mid_threads threads), [2] m, n <= 64 (one wavefront each), [3]
   * m + n < aca_small_mn (64-thread workgroups).  aca_ms: duration of the class's
   * first launch (events on the stream it ran on); aca_bytes: bytes the method must move for
   * the class, es (m + n) r (r + 1) / 2 per block of final rank r (step k reads the k previous
   * columns of U and V once and writes one column pair; es = bytes of one complex entry). */
  int64_t aca_blocks[4];
  double aca_ms[4];
  int64_t aca_bytes[4];
  int32_t aca_rounds; /* ACA launch rounds: 1 + continuation rounds (device pool exhausted) */
  int64_t row_begin, row_end; /* rows held, in cluster positions (all rows: 0, n_points) */
  int64_t n_rows, n_cols;     /* product shape: y has n_rows entries, x has n_cols (n_points
                                 both, except for hmx_build_rect operators: Mt and Ms) */
  int64_t pool_reserved_bytes; /* factor-slot pools reserved during the build (the generic
                                  estimate, or the learned layout's predictions, plus any
                                  continuation pools); after ACA each pool is trimmed to the
                                  slots it handed out (factor_bytes), the rest going back to the
                                  library's allocator for later buffers */
} hmx_info_t;

/* Sizes, counts and build timings of an operator. */
hmx_status hmx_info(const hmx_op* op, hmx_info_t* out);

/* Cluster tree export (host outputs, sized from hmx_info): perm[M] (cluster position -> point
 * index), and per node in breadth-first order begin, end, level, child0, child1 (-1 = leaf),
 * box (6 doubles: lo xyz, hi xyz).  Any output pointer may be NULL. */
hmx_status hmx_export_tree(const hmx_op* op, int32_t* perm, int64_t* begin, int64_t* end,
                           int32_t* level, int32_t* child0, int32_t* child1, double* box);

/* Block export (host outputs): near (n_near x 4) and far (n_far x 4) int64 rows
 * (t.begin, t.end, s.begin, s.end) in cluster positions, sorted lexicographically, and far ranks
 * (-1 for a far block stored dense).  Any output pointer may be NULL. */
hmx_status hmx_export_blocks(const hmx_op* op, int64_t* near_rc, int64_t* far_rc, int32_t* ranks);

/* Factors of far block b (host outputs, complex of the operator's precision): U (m x r) and
 * V (n x r) column-major with block ~ U V^T; for a dense far block U receives the m x n block
 * and V is untouched.  *rank receives r (or -1 for dense). */
hmx_status hmx_export_far(const hmx_op* op, int64_t b, void* U, void* V, int32_t* rank);

/* Test support (apply-only checks against another implementation's factors): replaces the
 * factors of the operator's low-rank far blocks.  ranks host, n_far entries in the order of
 * hmx_export_blocks: the new rank r_b of each low-rank block (0 <= r_b <= min(m, n)), and -1 for
 * each block stored dense (which keeps its entries).  U, V host, complex of the operator's
 * precision: for each low-rank block in turn, U_b (m x r_b) concatenated into U and V_b
 * (n x r_b) into V, column-major, with the block ~ U_b V_b^T.  The operator copies them into a
 * new factor pool (the old factors stay allocated until hmx_destroy).  Synchronous; not to be
 * called while a product on the operator is in flight or captured in a graph. */
hmx_status hmx_import_far(hmx_op* op, const int32_t* ranks, const void* U, const void* V);

/* ------------------------------------------------------------------ learned block ranks
 * The paper shows the local rank of each block of its H-matrix (Section 5.4, the spy plot of
 * the compressed acoustic operator) but does not predict it.  libhmx can lay out the factor
 * storage from ranks predicted by a small network: 4 -> 64 -> 64 -> 1 with ReLU, FP32, input the
 * standardized block features [log2 m, log2 n, ln(dist / max diam), k max diam / (2 pi)], output
 * ln(1 + rank).  Parameters are one float vector of HMX_MLP_NPARAMS entries:
 *   W1 (64 x 4, row-major) | b1 (64) | W2 (64 x 64, row-major) | b2 (64) | W3 (64) | b3 (1).
 * `norm` is 8 floats: the 4 feature means, then the 4 feature standard deviations (> 0). */
#define HMX_MLP_NPARAMS 4545

/* Raw (unstandardized) features of the operator's far blocks, in the order of
 * hmx_export_blocks: feat host, n_far x 4 floats. */
hmx_status hmx_far_features(const hmx_op* op, float* feat);

/* Predicted ln(1 + rank) of n blocks: theta, norm host; feat device (n x 4 raw features);
 * out device (n floats).  Synchronous. */
hmx_status hmx_mlp_predict(const float* theta, const float* norm, const float* feat, int64_t n,
                           float* out, void* stream);

/* Mean squared error (1/n) sum (o - y)^2 of the network on n samples and its gradient:
 * theta host; X device (n x 4 standardized features); y device (n targets); grad host
 * (HMX_MLP_NPARAMS); loss host.  n <= 2^24.  Synchronous. */
hmx_status hmx_mlp_loss_grad(const float* theta, const float* X, const float* y, int64_t n,
                             float* grad, float* loss, void* stream);

/* Trains the network with Adam (beta 0.9 / 0.999, eps 1e-8, bias-corrected) on minibatches of
 * `batch` consecutive samples, `epochs` passes in order (shuffle beforehand if wanted).
 * theta host, initial values in, trained values out; X, y device as in hmx_mlp_loss_grad;
 * loss_hist host (epochs floats, mean batch loss per epoch) or NULL.  Synchronous. */
hmx_status hmx_mlp_train(float* theta, const float* X, const float* y, int64_t n, int32_t epochs,
                         int32_t batch, float lr, float* loss_hist, void* stream);

/* Sets the process-wide model used by builds with rank_model = HMX_RANK_LEARNED.  Each far block
 * is predicted r_alloc = min(rank cap, ceil(alpha * max(exp(pred) - 1, 0)) + beta) columns (at
 * least 1).  The build reserves the factor pool as sum r_alloc (m + n) entries before ACA runs
 * (HMX_ENOMEM when that exceeds 90% of the free device memory) and runs the blocks of each class
 * in decreasing r_alloc^2 (m + n).  The pivots and factors are those of plain adaptive ACA.
 * theta, norm host (copied); theta NULL clears the model.  alpha > 0, beta >= 0. */
hmx_status hmx_set_rank_model(const float* theta, const float* norm, float alpha, float beta);

/* Frees the operator and all of its device memory; NULL is accepted. */
void hmx_destroy(hmx_op* op);

/* Message of the last failed call on this thread ("" when none). */
const char* hmx_last_error(void);

/* The library keeps freed device blocks for reuse by later builds (a caching allocator, so that
 * repeated builds do not map and unmap memory); this returns the cached blocks of the current
 * device to the HIP runtime.  Live operators are not affected. */
void hmx_release_cache(void);

#ifdef __cplusplus
}
#endif

#endif /* HMX_H */
