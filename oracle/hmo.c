/*
 * hmo.c -- plain CPU FP64 oracle for the H-matrix BEM hot path (test infrastructure only).
 *
 * Only the test suite, the package's smoke check and the bench's CPU-baseline leg load this
 * library.  It shares no source, header or table with the HIP library: it is written from the
 * paper's definitions, is deliberately simple (no blocking, no fusion, no reordering beyond what
 * the definitions state), uses libm sin/cos/sqrt and C99 complex arithmetic in double, and is
 * compiled with contraction off so that every sum is evaluated in the written order.
 *
 * Paper: Alouges & Aussal, "FEM and BEM simulations with the Gypsilab framework" (arXiv 1804.00995).
 *   O1 quadrature points/weights .......... Section 3 (points x_k, weights omega_k over all simplices)
 *   O2 dense product ...................... Section 5, eq. (BEM) and the Helmholtz kernel eq.
 *                                           (G_kl = G(x_k, y_l), G = e^{ikr}/(4 pi r)); source
 *                                           weights applied as W_y; pairs with r = 0 give 0.
 *   O3 cluster tree, O4 block tree ........ paper silent (Section 5.3 only says the matrix is
 *                                           compressed to a tolerance); bounding-box bisection and
 *                                           the standard min(diam) <= eta * dist admissibility.
 *   O5 partially pivoted ACA .............. paper silent; Bebendorf-style partial pivoting with
 *                                           the Frobenius-norm stopping rule at tolerance tol.
 *   O6 H-matrix times vector .............. Section 5.3 (the compressed matrix used like a
 *                                           matrix through the product operator).
 *   O7 singular correction ................ Section 5.2 (regularization of the kernels): the
 *                                           1/(4 pi r) part integrated in y analytically over
 *                                           close source triangles, minus its Gauss value.
 *   O9 Galerkin P1 operator ............... eq. (BEM): Phi^T W_x K Phi with the P1 basis at the
 *                                           quadrature points (oracle/__init__.py, numpy)
 *   O8 collocation at other points ........ Section 5.1 (C_ij = int G(x_i, y) psi_j(y) dy for a
 *                                           collection of points x_i), with the y-integral by
 *                                           the quadrature of eq. (BEM).
 * Pinned by the CPU tests: closed-form sphere eigenvalues, quadrature exactness, exact-rank and
 * SVD (Eckart-Young) bounds for ACA, brute-force coverage of the block partition.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex cplx;

#define HMO_LAPLACE 0
#define HMO_HELMHOLTZ 1
#define HMO_POLY2 99
#define HMO_GRADY_X 2 /* d/dy_j of the Helmholtz kernel, j = 0, 1, 2 (Laplace at k = 0) */
#define HMO_GRADY_Y 3
#define HMO_GRADY_Z 4

static const double PI = 3.14159265358979323846;

int hmo_max_threads(void) { return omp_get_max_threads(); }

static void set_threads(int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

/* ---------------------------------------------------------------- O1: quadrature points */
/* For triangle t with vertices a, b, c and reference rule (lambda_q, what_q):
 *   x_{nq*t+q} = lambda_q1 a + lambda_q2 b + lambda_q3 c,  w_{nq*t+q} = area(t) * what_q,
 *   area(t) = |(b - a) x (c - a)| / 2. */
int hmo_quad_points(const double *vtx, int64_t nv, const int32_t *tri, int64_t nt,
                    const double *bary, const double *what, int32_t nq,
                    double *X, double *Y, double *Z, double *W)
{
    for (int64_t t = 0; t < nt; ++t) {
        int32_t ia = tri[3 * t], ib = tri[3 * t + 1], ic = tri[3 * t + 2];
        if (ia < 0 || ib < 0 || ic < 0 || ia >= nv || ib >= nv || ic >= nv) return -1;
        const double *a = vtx + 3 * (int64_t)ia, *b = vtx + 3 * (int64_t)ib, *c = vtx + 3 * (int64_t)ic;
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double n0 = e1[1] * e2[2] - e1[2] * e2[1];
        double n1 = e1[2] * e2[0] - e1[0] * e2[2];
        double n2 = e1[0] * e2[1] - e1[1] * e2[0];
        double area = 0.5 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        for (int32_t q = 0; q < nq; ++q) {
            int64_t m = (int64_t)nq * t + q;
            const double *l = bary + 3 * q;
            X[m] = l[0] * a[0] + l[1] * b[0] + l[2] * c[0];
            Y[m] = l[0] * a[1] + l[1] * b[1] + l[2] * c[1];
            Z[m] = l[0] * a[2] + l[1] * b[2] + l[2] * c[2];
            W[m] = area * what[q];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ Green kernel */
/* G(x, y) = exp(i k |x - y|) / (4 pi |x - y|); Laplace is k = 0; 0 when |x - y| = 0.
 * GRADY_j: the j-th component of its gradient in y (Section 5.1, grady[exp(ikr)/r]j).
 * The test-only kernel POLY2 is (1 + x.y)^2, a separable function of exact rank 10. */
static cplx green(int kern, double k, const double *x, const double *y)
{
    if (kern == HMO_POLY2) {
        double d = 1.0 + (x[0] * y[0] + x[1] * y[1] + x[2] * y[2]);
        return d * d;
    }
    double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r == 0.0) return 0.0;
    if (kern >= HMO_GRADY_X && kern <= HMO_GRADY_Z) {
        /* d/dy_j of e^{ikr}/(4 pi r): (d/dr)(e^{ikr}/(4 pi r)) * dr/dy_j with
         * (d/dr) = e^{ikr} (ikr - 1) / (4 pi r^2) and dr/dy_j = (y_j - x_j) / r */
        int j = kern - HMO_GRADY_X;
        double kr = k * r;
        cplx e = cos(kr) + I * sin(kr);
        return e * (I * kr - 1.0) / (4.0 * PI * r * r) * ((y[j] - x[j]) / r);
    }
    double kr = (kern == HMO_LAPLACE) ? 0.0 : k * r;
    return (cos(kr) + I * sin(kr)) / (4.0 * PI * r);
}

/* Pairwise kernel values G(x_i, y_i) for i < n (x, y: n x 3 row-major). */
void hmo_green(int32_t kern, double k, const double *x, const double *y, int64_t n, cplx *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = green(kern, k, x + 3 * i, y + 3 * i);
}

/* ---------------------------------------------------------------- O2: dense product */
/* y_i = sum_l G(x_i, x_l) w_l x_l over l ascending, for the requested rows i.
 * Points are given as SoA arrays X, Y, Z and weights W (length M). */
void hmo_dense_rows(const double *X, const double *Y, const double *Z, const double *W, int64_t M,
                    int32_t kern, double k, const cplx *x, const int64_t *rows, int64_t nrows,
                    cplx *y, int32_t nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ii = 0; ii < nrows; ++ii) {
        int64_t i = rows ? rows[ii] : ii;
        double xi[3] = {X[i], Y[i], Z[i]};
        cplx acc = 0.0;
        for (int64_t l = 0; l < M; ++l) {
            double xl[3] = {X[l], Y[l], Z[l]};
            acc += green(kern, k, xi, xl) * W[l] * x[l];
        }
        y[ii] = acc;
    }
}

/* ---------------------------------------------------------------- O8: other target points */
/* Section 5.1 (integrals with one integration and a collection of points): the potential of the
 * source quadrature at targets that are not source points,
 *   y_i = sum_l G(t_i, x_l) w_l x_l  (l ascending),
 * for the requested target rows (all Mt when rows is NULL).  A target that coincides with a
 * source point gets 0 from it, as in the square operator. */
void hmo_rect_rows(const double *TX, const double *TY, const double *TZ, int64_t Mt,
                   const double *X, const double *Y, const double *Z, const double *W, int64_t Ms,
                   int32_t kern, double k, const cplx *x, const int64_t *rows, int64_t nrows,
                   cplx *y, int32_t nthreads)
{
    set_threads(nthreads);
    if (!rows) nrows = Mt;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ii = 0; ii < nrows; ++ii) {
        int64_t i = rows ? rows[ii] : ii;
        double ti[3] = {TX[i], TY[i], TZ[i]};
        cplx acc = 0.0;
        for (int64_t l = 0; l < Ms; ++l) {
            double xl[3] = {X[l], Y[l], Z[l]};
            acc += green(kern, k, ti, xl) * W[l] * x[l];
        }
        y[ii] = acc;
    }
}

/* ---------------------------------------------------------------- O7: singular correction */
/* Section 5.2 (regularization of the kernels).  The kernel behaves like 1/(4 pi |x - y|) as
 * y -> x; that part is integrated over the source triangle exactly in y while x stays a
 * quadrature point, and the Gauss-rule value of the same integral is subtracted, for close pairs
 * only (a sparse correction).
 *
 * Reading (the paper corrects Galerkin entries of a finite element space; this operator acts on
 * values at the quadrature points): a rule of three non-collinear points per triangle carries
 * exactly one linear function per triangle through the three values, so the trial function of
 * point q of triangle T is L_q, the linear function on T with L_q = 1 at its q-th point and 0 at
 * the other two.  The correction of the pair (target x, source point y_l = q-th point of T) is
 *   c(x, l) = ( int_T L_q(y) / |x - y| dy  -  g(x, y_l) w_l ) / (4 pi),
 * g(x, y) = 1 / |x - y|, and g = 0 when x = y (the operator sets its r = 0 entries to 0, so
 * nothing is subtracted there).  A pair is close when |x - c_T| <= alpha * d_T (c_T the
 * centroid, d_T the longest edge of T).
 *
 * The y-integrals over a flat triangle T = (v0, v1, v2) use the edge sums of Wilton, Rao,
 * Glisson, Schaubert, Al-Bundak and Butler (IEEE Trans. Antennas Propag. 32(3), 1984) and
 * Graglia (IEEE Trans. Antennas Propag. 41(10), 1993).  With n the unit normal of
 * (v1 - v0) x (v2 - v0), h = n.(x - v0), rho = x - h n the projection of x on the plane, and for
 * each edge (a, b) = (v_i, v_{i+1}) its unit direction s, in-plane outward normal m = s x n,
 * l+ = (b - rho).s, l- = (a - rho).s, P = (a - rho).m, R0^2 = P^2 + h^2, R+- = sqrt(R0^2 + l+-^2),
 * f = ln((R+ + l+) / (R- + l-)):
 *   I1      = int_T 1 / |x - y| dy        = sum_edges [ P f - |h| (atan(P l+ / (R0^2 + |h| R+))
 *                                                               - atan(P l- / (R0^2 + |h| R-))) ]
 *   Irho    = int_T (y - rho) / |x - y| dy = sum_edges m (R0^2 f + l+ R+ - l- R-) / 2.
 * An edge whose line passes through x (R0 = 0) contributes only m (l+ R+ - l- R-) / 2 (the other
 * terms vanish with P and R0).  R + l is evaluated as R0^2 / (R - l) when l < 0 (the same number,
 * without cancellation). */
static void sub3(const double *a, const double *b, double *c)
{
    c[0] = a[0] - b[0];
    c[1] = a[1] - b[1];
    c[2] = a[2] - b[2];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double r_plus_l(double R, double l, double R02) { return l >= 0.0 ? R + l : R02 / (R - l); }

/* out = {I1, Irho_x, Irho_y, Irho_z} for target x and triangle tv = (v0, v1, v2) (9 doubles). */
void hmo_tri_moments(const double *x, const double *tv, double *out)
{
    const double *v[3] = {tv, tv + 3, tv + 6};
    double e1[3], e2[3], N[3], n[3], rho[3];
    sub3(v[1], v[0], e1);
    sub3(v[2], v[0], e2);
    cross3(e1, e2, N);
    double A2 = sqrt(dot3(N, N));
    for (int d = 0; d < 3; ++d) n[d] = N[d] / A2;
    double xv[3];
    sub3(x, v[0], xv);
    double h = dot3(n, xv), ah = fabs(h);
    for (int d = 0; d < 3; ++d) rho[d] = x[d] - h * n[d];
    double I1 = 0.0, Ir[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; ++i) {
        const double *a = v[i], *b = v[(i + 1) % 3];
        double s[3], m[3], br[3], ar[3];
        sub3(b, a, s);
        double L = sqrt(dot3(s, s));
        for (int d = 0; d < 3; ++d) s[d] /= L;
        cross3(s, n, m);
        sub3(b, rho, br);
        sub3(a, rho, ar);
        double lp = dot3(br, s), lm = dot3(ar, s), P = dot3(ar, m);
        double R02 = P * P + h * h;
        double Rp = sqrt(R02 + lp * lp), Rm = sqrt(R02 + lm * lm);
        double c = 0.5 * (lp * Rp - lm * Rm);
        if (R02 > 1e-24 * L * L) {
            double f = log(r_plus_l(Rp, lp, R02) / r_plus_l(Rm, lm, R02));
            double beta = atan(P * lp / (R02 + ah * Rp)) - atan(P * lm / (R02 + ah * Rm));
            I1 += P * f - ah * beta;
            c += 0.5 * R02 * f;
        }
        for (int d = 0; d < 3; ++d) Ir[d] += c * m[d];
    }
    out[0] = I1;
    out[1] = Ir[0];
    out[2] = Ir[1];
    out[3] = Ir[2];
}

/* out[q] = int_T L_q(y) / |x - y| dy for q = 0, 1, 2, where L_q = sum_i lag[3 q + i] lambda_i
 * (lambda_i the barycentric coordinates of T).  Each lambda_i is affine, so with rho the
 * projection of x: int lambda_i / R = lambda_i(rho) I1 + grad(lambda_i) . Irho. */
void hmo_tri_lagrange(const double *x, const double *tv, const double *lag, double *out)
{
    const double *v[3] = {tv, tv + 3, tv + 6};
    double mom[4];
    hmo_tri_moments(x, tv, mom);
    double e1[3], e2[3], N[3], n[3], xv[3], rho[3];
    sub3(v[1], v[0], e1);
    sub3(v[2], v[0], e2);
    cross3(e1, e2, N);
    double A2 = sqrt(dot3(N, N));
    for (int d = 0; d < 3; ++d) n[d] = N[d] / A2;
    sub3(x, v[0], xv);
    double h = dot3(n, xv);
    for (int d = 0; d < 3; ++d) rho[d] = x[d] - h * n[d];
    double J[3];
    for (int i = 0; i < 3; ++i) {
        const double *b = v[(i + 1) % 3], *c = v[(i + 2) % 3];
        double br[3], cr[3], bc[3], cb[3], g[3];
        sub3(b, rho, br);
        sub3(c, rho, cr);
        cross3(br, cr, bc);
        double lam = dot3(bc, n) / A2; /* lambda_i(rho) */
        sub3(c, b, cb);
        cross3(n, cb, g);              /* A2 * grad(lambda_i) */
        J[i] = lam * mom[0] + (g[0] * mom[1] + g[1] * mom[2] + g[2] * mom[3]) / A2;
    }
    for (int q = 0; q < 3; ++q) out[q] = lag[3 * q] * J[0] + lag[3 * q + 1] * J[1] + lag[3 * q + 2] * J[2];
}

/* Mesh data of the correction: vertices, triangles, points per triangle (3), the Lagrange
 * matrix of the rule and the closeness factor alpha. */
typedef struct {
    const double *vtx;
    const int32_t *tri;
    int32_t nq;
    double lag[9];
    double alpha;
} reg_t;

static void tri_vertices(const reg_t *R, int64_t t, double *tv)
{
    for (int j = 0; j < 3; ++j)
        for (int d = 0; d < 3; ++d) tv[3 * j + d] = R->vtx[3 * (int64_t)R->tri[3 * t + j] + d];
}

/* Is triangle tv close to x: |x - c_T|^2 <= alpha^2 d_T^2. */
static int tri_close(const reg_t *R, const double *x, const double *tv)
{
    double c[3], e[3], d2 = 0.0;
    for (int d = 0; d < 3; ++d) c[d] = (tv[d] + tv[3 + d] + tv[6 + d]) / 3.0;
    for (int j = 0; j < 3; ++j) {
        sub3(tv + 3 * ((j + 1) % 3), tv + 3 * j, e);
        double l2 = dot3(e, e);
        if (l2 > d2) d2 = l2;
    }
    double xc[3];
    sub3(x, c, xc);
    return dot3(xc, xc) <= R->alpha * R->alpha * d2;
}

/* c(x, l) of the definition above for source point l (original index) at y with weight w, or 0
 * when the pair is not close. */
static double reg_corr(const reg_t *R, const double *x, int64_t l, const double *y, double w)
{
    int64_t t = l / R->nq;
    int q = (int)(l - t * R->nq);
    double tv[9];
    tri_vertices(R, t, tv);
    if (!tri_close(R, x, tv)) return 0.0;
    double J[3];
    hmo_tri_lagrange(x, tv, R->lag, J);
    double xy[3];
    sub3(x, y, xy);
    double r = sqrt(dot3(xy, xy));
    double gauss = r == 0.0 ? 0.0 : w / r;
    return (J[q] - gauss) / (4.0 * PI);
}

/* y_ii = sum over every close pair (i, l) of c(x_i, l) x_l for the requested rows i = rows[ii]
 * (all M rows when rows is NULL); points are the nq-point rule's, triangle-major: l = nq t + q. */
void hmo_reg_apply(const double *X, const double *Y, const double *Z, const double *W, int64_t M,
                   const double *vtx, const int32_t *tri, int64_t ntri, int32_t nq, const double *lag,
                   double alpha, const cplx *x, const int64_t *rows, int64_t nrows, cplx *y,
                   int32_t nthreads)
{
    set_threads(nthreads);
    reg_t R = {vtx, tri, nq, {0}, alpha};
    memcpy(R.lag, lag, sizeof(R.lag));
    if (!rows) nrows = M;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ii = 0; ii < nrows; ++ii) {
        int64_t i = rows ? rows[ii] : ii;
        double xi[3] = {X[i], Y[i], Z[i]};
        cplx acc = 0.0;
        for (int64_t t = 0; t < ntri; ++t) {
            double tv[9];
            tri_vertices(&R, t, tv);
            if (!tri_close(&R, xi, tv)) continue;
            for (int q = 0; q < nq; ++q) {
                int64_t l = nq * t + q;
                double yl[3] = {X[l], Y[l], Z[l]};
                acc += reg_corr(&R, xi, l, yl, W[l]) * x[l];
            }
        }
        y[ii] = acc;
    }
}

/* The point operator as a matrix: K[i * M + l] = G(x_i, x_l) w_l (row-major, M x M). */
void hmo_dense_matrix(const double *X, const double *Y, const double *Z, const double *W, int64_t M,
                      int32_t kern, double k, cplx *K)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        double xi[3] = {X[i], Y[i], Z[i]};
        for (int64_t l = 0; l < M; ++l) {
            double xl[3] = {X[l], Y[l], Z[l]};
            K[i * M + l] = green(kern, k, xi, xl) * W[l];
        }
    }
}

/* The correction of every close pair as a matrix: C[i * M + l] = c(x_i, l) (row-major, M x M,
 * zero for pairs that are not close). */
void hmo_reg_matrix(const double *X, const double *Y, const double *Z, const double *W, int64_t M,
                    const double *vtx, const int32_t *tri, int64_t ntri, int32_t nq,
                    const double *lag, double alpha, double *C, int32_t nthreads)
{
    set_threads(nthreads);
    reg_t R = {vtx, tri, nq, {0}, alpha};
    memcpy(R.lag, lag, sizeof(R.lag));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < M; ++i) {
        double xi[3] = {X[i], Y[i], Z[i]};
        for (int64_t l = 0; l < M; ++l) C[i * M + l] = 0.0;
        for (int64_t t = 0; t < ntri; ++t) {
            double tv[9];
            tri_vertices(&R, t, tv);
            if (!tri_close(&R, xi, tv)) continue;
            for (int q = 0; q < nq; ++q) {
                int64_t l = nq * t + q;
                double yl[3] = {X[l], Y[l], Z[l]};
                C[i * M + l] = reg_corr(&R, xi, l, yl, W[l]);
            }
        }
    }
}

/* ---------------------------------------------------------------- O3: cluster tree */
/* Nodes hold a range [begin, end) of the cluster ordering perm (perm[p] = original index of the
 * point at cluster position p), the tight axis-aligned box of their points, and two children or
 * none.  A node is split while it holds more than `leaf` points: along the longest box side
 * (ties resolved x < y < z) at the side's midpoint 0.5 * (lo + hi); points with coordinate < mid
 * go to the first child, the others to the second, each side keeping its relative order.  A
 * node whose box has zero extent, or whose split would leave a side empty, is a leaf. */
typedef struct {
    int64_t M, cap, n;
    int32_t leaf;
    const double *P[3];
    int32_t *perm, *tmp;
    int64_t *begin, *end;
    int32_t *child0, *child1, *level;
    double *box; /* 6 per node: lo x, lo y, lo z, hi x, hi y, hi z */
} tree_t;

static int32_t tree_node(tree_t *T, int64_t b, int64_t e, int32_t lev)
{
    int32_t id = (int32_t)T->n++;
    T->begin[id] = b;
    T->end[id] = e;
    T->level[id] = lev;
    T->child0[id] = T->child1[id] = -1;
    double *bx = T->box + 6 * (int64_t)id;
    for (int d = 0; d < 3; ++d) {
        bx[d] = INFINITY;
        bx[3 + d] = -INFINITY;
    }
    for (int64_t p = b; p < e; ++p)
        for (int d = 0; d < 3; ++d) {
            double c = T->P[d][T->perm[p]];
            if (c < bx[d]) bx[d] = c;
            if (c > bx[3 + d]) bx[3 + d] = c;
        }
    if (e - b <= T->leaf) return id;
    int axis = 0;
    double ext = bx[3] - bx[0];
    for (int d = 1; d < 3; ++d)
        if (bx[3 + d] - bx[d] > ext) {
            ext = bx[3 + d] - bx[d];
            axis = d;
        }
    if (!(ext > 0.0)) return id;
    double mid = 0.5 * (bx[axis] + bx[3 + axis]);
    int64_t nl = 0;
    for (int64_t p = b; p < e; ++p)
        if (T->P[axis][T->perm[p]] < mid) nl++;
    if (nl == 0 || nl == e - b) return id;
    int64_t il = b, ir = b + nl;
    for (int64_t p = b; p < e; ++p) {
        int32_t g = T->perm[p];
        if (T->P[axis][g] < mid) T->tmp[il++] = g;
        else T->tmp[ir++] = g;
    }
    memcpy(T->perm + b, T->tmp + b, sizeof(int32_t) * (size_t)(e - b));
    int32_t c0 = tree_node(T, b, b + nl, lev + 1);
    int32_t c1 = tree_node(T, b + nl, e, lev + 1);
    T->child0[id] = c0;
    T->child1[id] = c1;
    return id;
}

/* ---------------------------------------------------------------- O4: block tree */
/* diam(t) = length of the box diagonal; dist(t, s) = Euclidean distance between the boxes (0
 * when they overlap).  Starting from (root, root): the pair is far (admissible) when
 * min(diam_t^2, diam_s^2) <= eta^2 dist^2; otherwise it is near when both are leaves; otherwise
 * the non-leaf side(s) are split (2 or 4 child pairs).  Both lists are sorted by
 * (t.begin, t.end, s.begin, s.end). */
static double diam2(const double *bx)
{
    double ex = bx[3] - bx[0], ey = bx[4] - bx[1], ez = bx[5] - bx[2];
    return ex * ex + ey * ey + ez * ez;
}

static double dist2(const double *a, const double *b)
{
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        double g = 0.0;
        if (b[d] - a[3 + d] > g) g = b[d] - a[3 + d];
        if (a[d] - b[3 + d] > g) g = a[d] - b[3 + d];
        s = s + g * g;
    }
    return s;
}

typedef struct {
    int32_t *t, *s;
    int64_t n, cap;
} pairs_t;

static void pairs_push(pairs_t *L, int32_t t, int32_t s)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->t = realloc(L->t, sizeof(int32_t) * (size_t)L->cap);
        L->s = realloc(L->s, sizeof(int32_t) * (size_t)L->cap);
    }
    L->t[L->n] = t;
    L->s[L->n] = s;
    L->n++;
}

/* max_mn > 0 bounds the far blocks: an admissible pair whose two clusters hold more than max_mn
 * points together is not taken as one far block but recursed into like an inadmissible one
 * (a pair of leaves is far whatever its size).  max_mn = 0 is the plain definition above. */
static void block_rec(const tree_t *T, double eta2, int64_t max_mn, int32_t t, int32_t s,
                      pairs_t *nearL, pairs_t *farL)
{
    const double *bt = T->box + 6 * (int64_t)t, *bs = T->box + 6 * (int64_t)s;
    double dt = diam2(bt), ds = diam2(bs);
    double dmin = dt < ds ? dt : ds;
    int lt = T->child0[t] < 0, ls = T->child0[s] < 0;
    int64_t mn = (T->end[t] - T->begin[t]) + (T->end[s] - T->begin[s]);
    int small = max_mn <= 0 || mn <= max_mn || (lt && ls);
    if (small && dmin <= eta2 * dist2(bt, bs)) {
        pairs_push(farL, t, s);
        return;
    }
    if (lt && ls) {
        pairs_push(nearL, t, s);
    } else if (lt) {
        block_rec(T, eta2, max_mn, t, T->child0[s], nearL, farL);
        block_rec(T, eta2, max_mn, t, T->child1[s], nearL, farL);
    } else if (ls) {
        block_rec(T, eta2, max_mn, T->child0[t], s, nearL, farL);
        block_rec(T, eta2, max_mn, T->child1[t], s, nearL, farL);
    } else {
        block_rec(T, eta2, max_mn, T->child0[t], T->child0[s], nearL, farL);
        block_rec(T, eta2, max_mn, T->child0[t], T->child1[s], nearL, farL);
        block_rec(T, eta2, max_mn, T->child1[t], T->child0[s], nearL, farL);
        block_rec(T, eta2, max_mn, T->child1[t], T->child1[s], nearL, farL);
    }
}

static const tree_t *g_sort_tree;

static int cmp_pair(const void *pa, const void *pb)
{
    const int32_t *a = pa, *b = pb;
    const tree_t *T = g_sort_tree;
    int64_t ka[4] = {T->begin[a[0]], T->end[a[0]], T->begin[a[1]], T->end[a[1]]};
    int64_t kb[4] = {T->begin[b[0]], T->end[b[0]], T->begin[b[1]], T->end[b[1]]};
    for (int i = 0; i < 4; ++i)
        if (ka[i] != kb[i]) return ka[i] < kb[i] ? -1 : 1;
    return 0;
}

static void sort_pairs(const tree_t *T, pairs_t *L)
{
    int32_t *buf = malloc(sizeof(int32_t) * 2 * (size_t)(L->n ? L->n : 1));
    for (int64_t i = 0; i < L->n; ++i) {
        buf[2 * i] = L->t[i];
        buf[2 * i + 1] = L->s[i];
    }
    g_sort_tree = T;
    qsort(buf, (size_t)L->n, 2 * sizeof(int32_t), cmp_pair);
    for (int64_t i = 0; i < L->n; ++i) {
        L->t[i] = buf[2 * i];
        L->s[i] = buf[2 * i + 1];
    }
    free(buf);
}

/* ---------------------------------------------------------------- O5: ACA */
/* Partially pivoted adaptive cross approximation of an m x n matrix given entry by entry,
 * A ~ sum_k u_k v_k^T (u_k: m, v_k: n; U, V stored column-major with the k-th column holding
 * u_k, v_k).  Step k, with pivot row i_k:
 *   (1) residual row  R_j = a(i_k, j) - sum_{l<k} u_l[i_k] v_l[j];
 *   (2) pivot column  j_k = argmax over unused columns of |R_j|^2 (lowest index on ties);
 *       a residual row whose maximum is <= 1e-300 marks the row used, moves to the lowest unused
 *       row and does not count as a step;
 *   (3) v_k = R / R_{j_k};
 *   (4) u_k[i] = a(i, j_k) - sum_{l<k} v_l[j_k] u_l[i];
 *   (5) |S_k|_F^2 = |S_{k-1}|_F^2 + 2 Re sum_{l<k} (u_l^H u_k)(v_l^H v_k) + |u_k|^2 |v_k|^2;
 *   (6) stop (keeping term k) when |u_k| |v_k| <= tol |S_k|_F has held at ACA_STOP_STEPS
 *       consecutive steps (a zero residual row in between neither counts nor resets);
 *   (7) next pivot row: argmax over unused rows of |u_k[i]|^2 (lowest index on ties).
 * A single step meeting (6) is not enough: the pivot row can fall where the block is already
 * well approximated while other rows are not, so that |u_k| |v_k| is small by accident; on an
 * elongated ellipsoid this stops a 963 x 955 block at rank 8 with 10% error.  Requiring the
 * rule at two consecutive steps, each with its own pivot row, removes those stops.
 * The rank is capped at rcap = floor(m n / (m + n)); a block not converged at rcap is reported
 * as not converged (the caller stores it dense). */
#define ACA_STOP_STEPS 2

typedef cplx (*entry_fn)(const void *ctx, int64_t i, int64_t j);

typedef struct {
    int64_t m, n, rank, cap;
    int converged;
    cplx *U, *V; /* m x cap, n x cap column-major */
} aca_t;

static void aca_grow(aca_t *F, int64_t need)
{
    if (need <= F->cap) return;
    int64_t nc = F->cap ? F->cap : 8;
    while (nc < need) nc *= 2;
    F->U = realloc(F->U, sizeof(cplx) * (size_t)(F->m * nc));
    F->V = realloc(F->V, sizeof(cplx) * (size_t)(F->n * nc));
    F->cap = nc;
}

static void aca_run(entry_fn a, const void *ctx, int64_t m, int64_t n, double tol, int64_t rcap, aca_t *F)
{
    F->m = m;
    F->n = n;
    F->rank = 0;
    F->cap = 0;
    F->U = F->V = NULL;
    F->converged = 0;
    if (rcap <= 0) return;
    char *row_used = calloc((size_t)m, 1), *col_used = calloc((size_t)n, 1);
    cplx *R = malloc(sizeof(cplx) * (size_t)n);
    double norm2 = 0.0;
    int64_t ik = 0;
    int hits = 0; /* consecutive steps that met the stopping rule */
    while (1) {
        /* (1) residual row */
        for (int64_t j = 0; j < n; ++j) {
            cplx s = a(ctx, ik, j);
            for (int64_t l = 0; l < F->rank; ++l) s -= F->U[l * m + ik] * F->V[l * n + j];
            R[j] = s;
        }
        /* (2) pivot column */
        int64_t jk = -1;
        double best = -1.0;
        for (int64_t j = 0; j < n; ++j) {
            if (col_used[j]) continue;
            double v2 = creal(R[j]) * creal(R[j]) + cimag(R[j]) * cimag(R[j]);
            if (v2 > best) {
                best = v2;
                jk = j;
            }
        }
        if (jk < 0 || best <= 1e-300) {
            row_used[ik] = 1;
            int64_t nxt = -1;
            for (int64_t i = 0; i < m; ++i)
                if (!row_used[i]) {
                    nxt = i;
                    break;
                }
            if (nxt < 0) {
                F->converged = 1;
                break;
            }
            ik = nxt;
            continue;
        }
        if (F->rank == rcap) break; /* a further term is needed beyond the cap */
        aca_grow(F, F->rank + 1);
        int64_t k = F->rank;
        cplx *v = F->V + k * n, *u = F->U + k * m;
        /* (3) */
        cplx piv = R[jk];
        for (int64_t j = 0; j < n; ++j) v[j] = R[j] / piv;
        /* (4) residual column */
        for (int64_t i = 0; i < m; ++i) {
            cplx s = a(ctx, i, jk);
            for (int64_t l = 0; l < k; ++l) s -= F->V[l * n + jk] * F->U[l * m + i];
            u[i] = s;
        }
        row_used[ik] = 1;
        col_used[jk] = 1;
        /* (5) norm of the approximant */
        double nu2 = 0.0, nv2 = 0.0;
        for (int64_t i = 0; i < m; ++i) nu2 += creal(u[i]) * creal(u[i]) + cimag(u[i]) * cimag(u[i]);
        for (int64_t j = 0; j < n; ++j) nv2 += creal(v[j]) * creal(v[j]) + cimag(v[j]) * cimag(v[j]);
        double cross = 0.0;
        for (int64_t l = 0; l < k; ++l) {
            cplx du = 0.0, dv = 0.0;
            for (int64_t i = 0; i < m; ++i) du += conj(F->U[l * m + i]) * u[i];
            for (int64_t j = 0; j < n; ++j) dv += conj(F->V[l * n + j]) * v[j];
            cross += creal(du * dv);
        }
        norm2 = norm2 + 2.0 * cross + nu2 * nv2;
        F->rank = k + 1;
        /* (6) stopping rule */
        if (sqrt(nu2) * sqrt(nv2) <= tol * sqrt(norm2)) {
            if (++hits >= ACA_STOP_STEPS) {
                F->converged = 1;
                break;
            }
        } else {
            hits = 0;
        }
        /* (7) next pivot row */
        int64_t nxt = -1;
        best = -1.0;
        for (int64_t i = 0; i < m; ++i) {
            if (row_used[i]) continue;
            double v2 = creal(u[i]) * creal(u[i]) + cimag(u[i]) * cimag(u[i]);
            if (v2 > best) {
                best = v2;
                nxt = i;
            }
        }
        if (nxt < 0) {
            F->converged = 1;
            break;
        }
        ik = nxt;
    }
    free(row_used);
    free(col_used);
    free(R);
}

typedef struct {
    const cplx *A;
    int64_t n;
} dense_ctx;

static cplx dense_entry(const void *c, int64_t i, int64_t j)
{
    const dense_ctx *d = c;
    return d->A[i * d->n + j];
}

/* ACA of a dense row-major m x n matrix.  U (m x cap) and V (n x cap) column-major; returns the
 * rank in *rank and 1 when converged, 0 otherwise (-1 when cap is too small for the result). */
int hmo_aca_dense(const cplx *A, int64_t m, int64_t n, double tol, int64_t rcap,
                  cplx *U, cplx *V, int64_t cap, int64_t *rank)
{
    dense_ctx c = {A, n};
    aca_t F;
    aca_run(dense_entry, &c, m, n, tol, rcap, &F);
    *rank = F.rank;
    int ret = F.converged;
    if (F.rank > cap) ret = -1;
    else {
        memcpy(U, F.U, sizeof(cplx) * (size_t)(m * F.rank));
        memcpy(V, F.V, sizeof(cplx) * (size_t)(n * F.rank));
    }
    free(F.U);
    free(F.V);
    return ret;
}

/* ---------------------------------------------------------------- H-matrix build / product */
typedef struct {
    int64_t M;
    int32_t kern;
    double k, tol, eta;
    int32_t leaf;
    double *X, *Y, *Z, *W; /* original order */
    tree_t T;
    pairs_t nearL, farL;
    cplx **nearK;        /* per near block, m x n column-major */
    aca_t *farF;         /* per far block */
    cplx **farDense;     /* per far block: dense fallback (or NULL) */
    int has_reg;         /* near blocks carry the singular correction (O7) */
    reg_t reg;
} hmo_h;

typedef struct {
    const hmo_h *H;
    int64_t tb, sb;
} block_ctx;

static cplx block_entry(const void *c, int64_t i, int64_t j)
{
    const block_ctx *b = c;
    const hmo_h *H = b->H;
    int64_t gi = H->T.perm[b->tb + i], gj = H->T.perm[b->sb + j];
    double xi[3] = {H->X[gi], H->Y[gi], H->Z[gi]};
    double xj[3] = {H->X[gj], H->Y[gj], H->Z[gj]};
    return green(H->kern, H->k, xi, xj) * H->W[gj];
}

static cplx *dense_block(const hmo_h *H, int64_t tb, int64_t m, int64_t sb, int64_t n)
{
    block_ctx c = {H, tb, sb};
    cplx *K = malloc(sizeof(cplx) * (size_t)(m * n));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) K[j * m + i] = block_entry(&c, i, j);
    return K;
}

/* O7 inside the H-matrix: the close pairs of a near block get their correction (far blocks,
 * including those stored dense, keep the plain kernel). */
static void correct_block(const hmo_h *H, cplx *K, int64_t tb, int64_t m, int64_t sb, int64_t n)
{
    for (int64_t j = 0; j < n; ++j) {
        int64_t gj = H->T.perm[sb + j];
        double yj[3] = {H->X[gj], H->Y[gj], H->Z[gj]};
        for (int64_t i = 0; i < m; ++i) {
            int64_t gi = H->T.perm[tb + i];
            double xi[3] = {H->X[gi], H->Y[gi], H->Z[gi]};
            K[j * m + i] += reg_corr(&H->reg, xi, gj, yj, H->W[gj]);
        }
    }
}

/* vtx == NULL: no correction; otherwise the near blocks carry O7 for the mesh (vtx, tri) whose
 * nq-point rule produced the points, with Lagrange matrix lag and closeness factor alpha. */
void *hmo_hbuild(const double *X, const double *Y, const double *Z, const double *W, int64_t M,
                 int32_t kern, double k, int32_t leaf, double eta, double tol, int32_t nthreads,
                 int64_t max_mn, const double *vtx, const int32_t *tri, int32_t nq,
                 const double *lag, double alpha)
{
    set_threads(nthreads);
    hmo_h *H = calloc(1, sizeof(hmo_h));
    if (vtx) {
        H->has_reg = 1;
        H->reg.vtx = vtx;
        H->reg.tri = tri;
        H->reg.nq = nq;
        memcpy(H->reg.lag, lag, sizeof(H->reg.lag));
        H->reg.alpha = alpha;
    }
    H->M = M;
    H->kern = kern;
    H->k = k;
    H->tol = tol;
    H->eta = eta;
    H->leaf = leaf;
    H->X = malloc(sizeof(double) * (size_t)M);
    H->Y = malloc(sizeof(double) * (size_t)M);
    H->Z = malloc(sizeof(double) * (size_t)M);
    H->W = malloc(sizeof(double) * (size_t)M);
    memcpy(H->X, X, sizeof(double) * (size_t)M);
    memcpy(H->Y, Y, sizeof(double) * (size_t)M);
    memcpy(H->Z, Z, sizeof(double) * (size_t)M);
    memcpy(H->W, W, sizeof(double) * (size_t)M);
    tree_t *T = &H->T;
    T->M = M;
    T->cap = 2 * M + 1;
    T->leaf = leaf;
    T->P[0] = H->X;
    T->P[1] = H->Y;
    T->P[2] = H->Z;
    T->perm = malloc(sizeof(int32_t) * (size_t)M);
    T->tmp = malloc(sizeof(int32_t) * (size_t)M);
    for (int64_t i = 0; i < M; ++i) T->perm[i] = (int32_t)i;
    T->begin = malloc(sizeof(int64_t) * (size_t)T->cap);
    T->end = malloc(sizeof(int64_t) * (size_t)T->cap);
    T->child0 = malloc(sizeof(int32_t) * (size_t)T->cap);
    T->child1 = malloc(sizeof(int32_t) * (size_t)T->cap);
    T->level = malloc(sizeof(int32_t) * (size_t)T->cap);
    T->box = malloc(sizeof(double) * 6 * (size_t)T->cap);
    tree_node(T, 0, M, 0);
    block_rec(T, eta * eta, max_mn, 0, 0, &H->nearL, &H->farL);
    sort_pairs(T, &H->nearL);
    sort_pairs(T, &H->farL);
    int64_t nn = H->nearL.n, nf = H->farL.n;
    H->nearK = calloc((size_t)(nn ? nn : 1), sizeof(cplx *));
    H->farF = calloc((size_t)(nf ? nf : 1), sizeof(aca_t));
    H->farDense = calloc((size_t)(nf ? nf : 1), sizeof(cplx *));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nn; ++b) {
        int32_t t = H->nearL.t[b], s = H->nearL.s[b];
        H->nearK[b] = dense_block(H, T->begin[t], T->end[t] - T->begin[t], T->begin[s], T->end[s] - T->begin[s]);
        if (H->has_reg)
            correct_block(H, H->nearK[b], T->begin[t], T->end[t] - T->begin[t], T->begin[s],
                          T->end[s] - T->begin[s]);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nf; ++b) {
        int32_t t = H->farL.t[b], s = H->farL.s[b];
        int64_t m = T->end[t] - T->begin[t], n = T->end[s] - T->begin[s];
        block_ctx c = {H, T->begin[t], T->begin[s]};
        int64_t rcap = (m * n) / (m + n);
        aca_run(block_entry, &c, m, n, tol, rcap, &H->farF[b]);
        if (!H->farF[b].converged) H->farDense[b] = dense_block(H, T->begin[t], m, T->begin[s], n);
    }
    return H;
}

/* y = H x with x, y in the original point order.  Every entry of y sums the near blocks in list
 * order (columns ascending), then the far blocks in list order (terms ascending), with
 * t_l = sum_j V[l][j] x_j (columns ascending) per far block.  The rows are split over threads by
 * cluster-tree leaves: each thread owns whole leaves and applies every block that covers them
 * in that order, so the sums are the same for any thread count. */
void hmo_hmatvec(const void *hp, const cplx *x, cplx *y)
{
    const hmo_h *H = hp;
    const tree_t *T = &H->T;
    int64_t M = H->M, nn = H->nearL.n, nf = H->farL.n;
    cplx *xp = malloc(sizeof(cplx) * (size_t)M), *yp = calloc((size_t)M, sizeof(cplx));
    for (int64_t p = 0; p < M; ++p) xp[p] = x[T->perm[p]];
    /* the leaves in cluster order and the leaf of every position */
    int64_t nl = 0, nodes = T->n;
    for (int64_t i = 0; i < nodes; ++i) nl += T->child0[i] < 0;
    int64_t *lb = malloc(sizeof(int64_t) * (size_t)(nl + 1));
    int32_t *leaf_of = malloc(sizeof(int32_t) * (size_t)(M ? M : 1));
    for (int64_t i = 0; i < nodes; ++i)
        if (T->child0[i] < 0)
            for (int64_t p = T->begin[i]; p < T->end[i]; ++p) leaf_of[p] = -1 - (int32_t)i;
    /* number the leaves by position */
    for (int64_t p = 0, q = 0; p < M; ++p)
        if (p == 0 || leaf_of[p] != leaf_of[p - 1]) lb[q++] = p;
    lb[nl] = M;
    for (int64_t q = 0; q < nl; ++q)
        for (int64_t p = lb[q]; p < lb[q + 1]; ++p) leaf_of[p] = (int32_t)q;
    /* per leaf, the blocks covering it: near blocks, then far blocks, each in list order */
    int64_t *ptr = calloc((size_t)(nl + 1), sizeof(int64_t));
    for (int64_t b = 0; b < nn + nf; ++b) {
        int32_t t = b < nn ? H->nearL.t[b] : H->farL.t[b - nn];
        for (int64_t q = leaf_of[T->begin[t]]; q <= leaf_of[T->end[t] - 1]; ++q) ++ptr[q + 1];
    }
    for (int64_t q = 0; q < nl; ++q) ptr[q + 1] += ptr[q];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(nl + 1));
    memcpy(fill, ptr, sizeof(int64_t) * (size_t)(nl + 1));
    int64_t *lst = malloc(sizeof(int64_t) * (size_t)(ptr[nl] ? ptr[nl] : 1));
    for (int64_t b = 0; b < nn + nf; ++b) {
        int32_t t = b < nn ? H->nearL.t[b] : H->farL.t[b - nn];
        for (int64_t q = leaf_of[T->begin[t]]; q <= leaf_of[T->end[t] - 1]; ++q) lst[fill[q]++] = b;
    }
    /* t_b = V_b^T x_s of the low-rank far blocks */
    int64_t *toff = malloc(sizeof(int64_t) * (size_t)(nf + 1));
    toff[0] = 0;
    for (int64_t b = 0; b < nf; ++b) toff[b + 1] = toff[b] + (H->farDense[b] ? 0 : H->farF[b].rank);
    cplx *tv = malloc(sizeof(cplx) * (size_t)(toff[nf] ? toff[nf] : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < nf; ++b) {
        if (H->farDense[b]) continue;
        int32_t s = H->farL.s[b];
        int64_t sb = T->begin[s], n = T->end[s] - sb;
        const aca_t *F = &H->farF[b];
        for (int64_t l = 0; l < F->rank; ++l) {
            cplx tl = 0.0;
            for (int64_t j = 0; j < n; ++j) tl += F->V[l * n + j] * xp[sb + j];
            tv[toff[b] + l] = tl;
        }
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nl; ++q) {
        for (int64_t e = ptr[q]; e < ptr[q + 1]; ++e) {
            int64_t b = lst[e];
            int far = b >= nn;
            int32_t t = far ? H->farL.t[b - nn] : H->nearL.t[b];
            int32_t s = far ? H->farL.s[b - nn] : H->nearL.s[b];
            int64_t tb = T->begin[t], m = T->end[t] - tb, sb = T->begin[s], n = T->end[s] - sb;
            int64_t i0 = lb[q] - tb, i1 = lb[q + 1] - tb; /* this leaf's rows of the block */
            const cplx *K = far ? H->farDense[b - nn] : H->nearK[b];
            if (K) {
                for (int64_t j = 0; j < n; ++j)
                    for (int64_t i = i0; i < i1; ++i) yp[tb + i] += K[j * m + i] * xp[sb + j];
                continue;
            }
            const aca_t *F = &H->farF[b - nn];
            const cplx *tb_ = tv + toff[b - nn];
            for (int64_t l = 0; l < F->rank; ++l)
                for (int64_t i = i0; i < i1; ++i) yp[tb + i] += F->U[l * m + i] * tb_[l];
        }
    }
    for (int64_t p = 0; p < M; ++p) y[T->perm[p]] = yp[p];
    free(xp);
    free(yp);
    free(lb);
    free(leaf_of);
    free(ptr);
    free(fill);
    free(lst);
    free(toff);
    free(tv);
}

/* Sizes: [0] nodes, [1] near blocks, [2] far blocks, [3] sum m*n over near, [4] sum r*(m+n)
 * over converged far, [5] dense-fallback far blocks, [6] sum m*n over dense-fallback far,
 * [7] max rank, [8] sum of ranks. */
void hmo_hinfo(const void *hp, int64_t *out)
{
    const hmo_h *H = hp;
    const tree_t *T = &H->T;
    int64_t snear = 0, sfar = 0, nd = 0, sd = 0, rmax = 0, rsum = 0;
    for (int64_t b = 0; b < H->nearL.n; ++b) {
        int32_t t = H->nearL.t[b], s = H->nearL.s[b];
        snear += (T->end[t] - T->begin[t]) * (T->end[s] - T->begin[s]);
    }
    for (int64_t b = 0; b < H->farL.n; ++b) {
        int32_t t = H->farL.t[b], s = H->farL.s[b];
        int64_t m = T->end[t] - T->begin[t], n = T->end[s] - T->begin[s];
        if (H->farDense[b]) {
            nd++;
            sd += m * n;
        } else {
            sfar += H->farF[b].rank * (m + n);
            if (H->farF[b].rank > rmax) rmax = H->farF[b].rank;
            rsum += H->farF[b].rank;
        }
    }
    out[0] = T->n;
    out[1] = H->nearL.n;
    out[2] = H->farL.n;
    out[3] = snear;
    out[4] = sfar;
    out[5] = nd;
    out[6] = sd;
    out[7] = rmax;
    out[8] = rsum;
}

/* Tree export: perm (M), and per node begin, end, level, child0, child1, box (6). */
void hmo_htree(const void *hp, int32_t *perm, int64_t *begin, int64_t *end, int32_t *level,
               int32_t *child0, int32_t *child1, double *box)
{
    const hmo_h *H = hp;
    const tree_t *T = &H->T;
    memcpy(perm, T->perm, sizeof(int32_t) * (size_t)H->M);
    memcpy(begin, T->begin, sizeof(int64_t) * (size_t)T->n);
    memcpy(end, T->end, sizeof(int64_t) * (size_t)T->n);
    memcpy(level, T->level, sizeof(int32_t) * (size_t)T->n);
    memcpy(child0, T->child0, sizeof(int32_t) * (size_t)T->n);
    memcpy(child1, T->child1, sizeof(int32_t) * (size_t)T->n);
    memcpy(box, T->box, sizeof(double) * 6 * (size_t)T->n);
}

/* Block export as node ranges: near (nn x 4) and far (nf x 4) rows (t.begin, t.end, s.begin,
 * s.end); far ranks (-1 for a dense-fallback block). */
void hmo_hblocks(const void *hp, int64_t *nearR, int64_t *farR, int64_t *ranks)
{
    const hmo_h *H = hp;
    const tree_t *T = &H->T;
    for (int64_t b = 0; b < H->nearL.n; ++b) {
        int32_t t = H->nearL.t[b], s = H->nearL.s[b];
        nearR[4 * b] = T->begin[t];
        nearR[4 * b + 1] = T->end[t];
        nearR[4 * b + 2] = T->begin[s];
        nearR[4 * b + 3] = T->end[s];
    }
    for (int64_t b = 0; b < H->farL.n; ++b) {
        int32_t t = H->farL.t[b], s = H->farL.s[b];
        farR[4 * b] = T->begin[t];
        farR[4 * b + 1] = T->end[t];
        farR[4 * b + 2] = T->begin[s];
        farR[4 * b + 3] = T->end[s];
        ranks[b] = H->farDense[b] ? -1 : H->farF[b].rank;
    }
}

/* Factors of far block b: U (m x rank) and V (n x rank) column-major, A_b ~ U V^T. */
int64_t hmo_hfar_factors(const void *hp, int64_t b, cplx *U, cplx *V)
{
    const hmo_h *H = hp;
    const aca_t *F = &H->farF[b];
    if (H->farDense[b]) return -1;
    memcpy(U, F->U, sizeof(cplx) * (size_t)(F->m * F->rank));
    memcpy(V, F->V, sizeof(cplx) * (size_t)(F->n * F->rank));
    return F->rank;
}

void hmo_hfree(void *hp)
{
    hmo_h *H = hp;
    if (!H) return;
    for (int64_t b = 0; b < H->nearL.n; ++b) free(H->nearK[b]);
    for (int64_t b = 0; b < H->farL.n; ++b) {
        free(H->farF[b].U);
        free(H->farF[b].V);
        free(H->farDense[b]);
    }
    free(H->nearK);
    free(H->farF);
    free(H->farDense);
    free(H->nearL.t);
    free(H->nearL.s);
    free(H->farL.t);
    free(H->farL.s);
    tree_t *T = &H->T;
    free(T->perm);
    free(T->tmp);
    free(T->begin);
    free(T->end);
    free(T->child0);
    free(T->child1);
    free(T->level);
    free(T->box);
    free(H->X);
    free(H->Y);
    free(H->Z);
    free(H->W);
    free(H);
}
