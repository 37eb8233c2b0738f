/*
 * sem_oracle.c -- plain FP64 CPU oracle for the spectral-element Helmholtz
 * hot path (Jansson et al., "Neko", arXiv 2107.01243).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * path: GLL points, the derivative matrix, the box mesh, the geometric factors,
 * the gather-scatter groups and every solver step are computed here from their
 * definitions, independently.
 *
 * Style: plain loops, no blocking, no fusion, FP64 throughout, built with
 * -O2 -ffp-contract=off.  OpenMP only splits independent outer loops.
 *
 * Layout: local ("L") element-major, point (i,j,k) of element e at
 * e*lx^3 + i + lx*(j + lx*k), i fastest (the 4-D arrays w(:,:,:,:),
 * u(:,:,:,:) of the paper's ax_compute interface, Section 3.1, Listing 1).
 * Geometric factors are stored as six planes of n_p values in the order
 * G11, G22, G33, G12, G13, G23.
 *
 * Readings of the paper that this file adopts (the paper is silent or its
 * text is garbled at these points):
 *  - Eq. 7 (the GLL Lagrange basis) is printed garbled; l_i is read as the
 *    degree-N Lagrange interpolant through the N+1 GLL points, which are
 *    -1, +1 and the roots of L'_N.
 *  - G^e of Eq. 9 is not defined in the paper; it is read as the standard
 *    isoparametric factor G_ab = rho * J * (grad r_a . grad r_b), with rho the
 *    tensor GLL weight and J the Jacobian determinant, the metric computed by
 *    applying D to the nodal coordinates.
 *  - The Helmholtz operator is A = h1*K + h2*B (K the weak -Laplacian of
 *    Eq. 6 and 9, B the diagonal GLL mass), i.e. the SPD form of the
 *    velocity equation of Section 4 with h1 = 1/Re, h2 = b0/dt.
 *  - Direct stiffness summation QQ^T (Eq. 10) sums the copies of every
 *    global id in ascending local-index order and writes the sum back to all
 *    copies.
 *  - Global inner products of continuous local vectors weight each local
 *    entry by 1/multiplicity (the unique-node Euclidean product).
 *  - "Block Jacobi" (Section 4) is read as point Jacobi: the exact diagonal
 *    of the assembled operator.
 *  - Homogeneous Dirichlet conditions (Eq. 5) are imposed by zeroing the
 *    rows and columns of boundary nodes (mask).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* Legendre polynomial L_N and its derivative at x (three-term recurrence). */
static void legendre(int N, double x, double *LN, double *dLN)
{
    double p0 = 1.0, p1 = x;
    if (N == 0) { *LN = 1.0; *dLN = 0.0; return; }
    for (int n = 1; n < N; ++n) {
        double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *LN = p1;
    /* derivative from (x^2-1) L_N' = N (x L_N - L_{N-1}); valid off +-1 */
    if (fabs(fabs(x) - 1.0) > 0.0)
        *dLN = N * (x * p1 - p0) / (x * x - 1.0);
    else
        *dLN = (x > 0 ? 1.0 : ((N % 2) ? 1.0 : -1.0)) * 0.5 * N * (N + 1.0);
}

/*
 * GLL points and weights (Section 2, Eq. 7-8).  xi_0 = -1, xi_N = +1, the
 * interior points are the roots of L'_N found by Newton's method from the
 * Chebyshev-Gauss-Lobatto guesses; w_i = 2 / (N (N+1) L_N(xi_i)^2).
 * Returns 0 on success, -1 for lx outside [2, 32].
 */
/* Host threads of the parallel loops (timing at a stated core count); returns the
 * count in effect before the call.  No arithmetic depends on it except the order of
 * the partial sums of the inner products. */
EXPORT int orc_set_threads(int nthreads)
{
    const int before = omp_get_max_threads();
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return before;
}

EXPORT int orc_gll(int lx, double *xi, double *w)
{
    if (lx < 2 || lx > 32) return -1;
    const int N = lx - 1;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double L, dL;
            legendre(N, x, &L, &dL);
            /* L'' from Legendre's equation (1-x^2) L'' - 2x L' + N(N+1) L = 0 */
            double d2L = (2.0 * x * dL - N * (N + 1.0) * L) / (1.0 - x * x);
            double dx = dL / d2L;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        xi[i] = x;
    }
    /* the point set is symmetric about 0 */
    for (int i = 0; i < lx / 2; ++i) {
        double a = 0.5 * (xi[N - i] - xi[i]);
        xi[i] = -a;
        xi[N - i] = a;
    }
    if (lx % 2) xi[N / 2] = 0.0;
    for (int i = 0; i <= N; ++i) {
        double L, dL;
        legendre(N, xi[i], &L, &dL);
        w[i] = 2.0 / (N * (N + 1.0) * L * L);
    }
    return 0;
}

/*
 * Derivative matrix D[i*lx + l] = l_l'(xi_i): the derivative of the l-th
 * Lagrange basis function at point i ("D the local derivatives", Eq. 9).
 * Closed form for GLL points: L_N(xi_i) / (L_N(xi_l) (xi_i - xi_l)) off the
 * diagonal, -N(N+1)/4 at (0,0), +N(N+1)/4 at (N,N), zero elsewhere.
 */
EXPORT int orc_deriv_matrix(int lx, const double *xi, double *D)
{
    if (lx < 2 || lx > 32) return -1;
    const int N = lx - 1;
    double LN[32];
    for (int i = 0; i < lx; ++i) {
        double dL;
        legendre(N, xi[i], &LN[i], &dL);
    }
    for (int i = 0; i < lx; ++i)
        for (int l = 0; l < lx; ++l) {
            double v;
            if (i != l)
                v = LN[i] / (LN[l] * (xi[i] - xi[l]));
            else if (i == 0)
                v = -0.25 * N * (N + 1.0);
            else if (i == N)
                v = 0.25 * N * (N + 1.0);
            else
                v = 0.0;
            D[i * lx + l] = v;
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/*
 * Structured box mesh of nx*ny*nz hexahedra on [0,1]^3 (the synthetic
 * stand-in for the paper's hexahedral meshes, Section 2).  Element
 * e = ex + nx*(ey + ny*ez); node (i,j,k) sits at
 *   x = (ex + (xi_i+1)/2)/nx,  y likewise with (ey, xi_j, ny),  z with (ez, xi_k, nz),
 * then moved by the smooth map
 *   x' = x + eps sin(2 pi y) sin(2 pi z),
 *   y' = y + eps sin(2 pi z) sin(2 pi x),
 *   z' = z + eps sin(2 pi x) sin(2 pi y),
 * all three evaluated at the undeformed (x, y, z).
 * Global numbering (Section 2, "a unique global number"): the tensor grid
 * index (ex*N+i, ey*N+j, ez*N+k) flattened with x fastest.  A node is
 * Dirichlet when any grid index lies on the box boundary (Eq. 5).
 */
EXPORT void orc_box_mesh(int nx, int ny, int nz, int lx, double eps, const double *xi,
                         int64_t *glb, uint8_t *dirichlet,
                         double *x, double *y, double *z)
{
    const int N = lx - 1;
    const int64_t Mx = (int64_t)nx * N + 1, My = (int64_t)ny * N + 1, Mz = (int64_t)nz * N + 1;
    const int64_t nelv = (int64_t)nx * ny * nz;
    const int64_t npe = (int64_t)lx * lx * lx;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nelv; ++e) {
        const int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / ((int64_t)nx * ny);
        for (int k = 0; k < lx; ++k)
            for (int j = 0; j < lx; ++j)
                for (int i = 0; i < lx; ++i) {
                    const int64_t p = e * npe + i + lx * (j + (int64_t)lx * k);
                    const int64_t gx = ex * N + i, gy = ey * N + j, gz = ez * N + k;
                    if (glb) glb[p] = gx + Mx * (gy + My * gz);
                    if (dirichlet)
                        dirichlet[p] = (gx == 0 || gx == Mx - 1 || gy == 0 || gy == My - 1 ||
                                        gz == 0 || gz == Mz - 1) ? 1 : 0;
                    const double x0 = (ex + 0.5 * (xi[i] + 1.0)) / nx;
                    const double y0 = (ey + 0.5 * (xi[j] + 1.0)) / ny;
                    const double z0 = (ez + 0.5 * (xi[k] + 1.0)) / nz;
                    const double tp = 2.0 * M_PI;
                    x[p] = x0 + eps * sin(tp * y0) * sin(tp * z0);
                    y[p] = y0 + eps * sin(tp * z0) * sin(tp * x0);
                    z[p] = z0 + eps * sin(tp * x0) * sin(tp * y0);
                }
    }
}

/* ------------------------------------------------------------------ */
/*
 * Geometric factors of Eq. 9 (isoparametric reading, see file header).
 * For every point: the metric x_r = sum_l D[i][l] x_ljk, x_s = sum_l D[j][l] x_ilk,
 * x_t = sum_l D[k][l] x_ijl (same for y, z); J = det of the 3x3 metric;
 * grad r, grad s, grad t = rows of its inverse;
 * G_ab = rho J (grad a . grad b) with rho = w_i w_j w_k;  B = rho J.
 * Returns the number of points with J <= 0 (0 for a valid mesh).
 */
EXPORT int64_t orc_geometry(int64_t nelv, int lx, const double *D, const double *w,
                            const double *x, const double *y, const double *z,
                            double *G, double *B, double *Jout)
{
    const int64_t npe = (int64_t)lx * lx * lx;
    const int64_t n = nelv * npe;
    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t e = 0; e < nelv; ++e) {
        const double *X[3] = {x + e * npe, y + e * npe, z + e * npe};
        for (int k = 0; k < lx; ++k)
            for (int j = 0; j < lx; ++j)
                for (int i = 0; i < lx; ++i) {
                    /* m[c][d] = d x_c / d r_d */
                    double m[3][3];
                    for (int c = 0; c < 3; ++c) {
                        double dr = 0.0, ds = 0.0, dt = 0.0;
                        for (int l = 0; l < lx; ++l) {
                            dr += D[i * lx + l] * X[c][l + lx * (j + lx * k)];
                            ds += D[j * lx + l] * X[c][i + lx * (l + lx * k)];
                            dt += D[k * lx + l] * X[c][i + lx * (j + lx * l)];
                        }
                        m[c][0] = dr;
                        m[c][1] = ds;
                        m[c][2] = dt;
                    }
                    const double J = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
                                   - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
                                   + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
                    /* inverse: inv[d][c] = d r_d / d x_c = cofactor(c,d) / J */
                    double inv[3][3];
                    inv[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) / J;
                    inv[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / J;
                    inv[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / J;
                    inv[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) / J;
                    inv[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / J;
                    inv[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / J;
                    inv[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) / J;
                    inv[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) / J;
                    inv[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / J;
                    const double rho = w[i] * w[j] * w[k];
                    const int64_t p = e * npe + i + lx * (j + (int64_t)lx * k);
                    static const int A[6] = {0, 1, 2, 0, 0, 1};
                    static const int Bi[6] = {0, 1, 2, 1, 2, 2};
                    for (int f = 0; f < 6; ++f) {
                        double dot = 0.0;
                        for (int c = 0; c < 3; ++c) dot += inv[A[f]][c] * inv[Bi[f]][c];
                        G[f * n + p] = rho * J * dot;
                    }
                    B[p] = rho * J;
                    if (Jout) Jout[p] = J;
                    if (!(J > 0.0)) bad += 1;
                }
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/*
 * Unassembled Helmholtz operator w = A_L u, A^e = h1 D^T G^e D + h2 B^e
 * (Eq. 9-10 with the Helmholtz reading above).  Per element:
 *   ur_ijk = sum_l D[i][l] u_ljk,  us_ijk = sum_l D[j][l] u_ilk,  ut_ijk = sum_l D[k][l] u_ijl
 *   [wr ws wt] = h1 * G * [ur us ut]   (G symmetric 3x3 per point)
 *   w_ijk = sum_l D[l][i] wr_ljk + sum_l D[l][j] ws_ilk + sum_l D[l][k] wt_ijl + h2 B u.
 * h1 / h2: per-point arrays, or NULL to use the scalars h1s / h2s.  B may be
 * NULL when h2 is the scalar 0.
 */
EXPORT void orc_ax_helm(int64_t nelv, int lx, const double *D, const double *G,
                        const double *B, const double *h1, double h1s,
                        const double *h2, double h2s, const double *u, double *w)
{
    const int64_t npe = (int64_t)lx * lx * lx;
    const int64_t n = nelv * npe;
#pragma omp parallel
    {
        double *wr = malloc(sizeof(double) * npe);
        double *ws = malloc(sizeof(double) * npe);
        double *wt = malloc(sizeof(double) * npe);
#pragma omp for schedule(static)
        for (int64_t e = 0; e < nelv; ++e) {
            const double *ue = u + e * npe;
            for (int k = 0; k < lx; ++k)
                for (int j = 0; j < lx; ++j)
                    for (int i = 0; i < lx; ++i) {
                        double ur = 0.0, us = 0.0, ut = 0.0;
                        for (int l = 0; l < lx; ++l) {
                            ur += D[i * lx + l] * ue[l + lx * (j + lx * k)];
                            us += D[j * lx + l] * ue[i + lx * (l + lx * k)];
                            ut += D[k * lx + l] * ue[i + lx * (j + lx * l)];
                        }
                        const int q = i + lx * (j + lx * k);
                        const int64_t p = e * npe + q;
                        const double c = h1 ? h1[p] : h1s;
                        const double g11 = G[0 * n + p], g22 = G[1 * n + p], g33 = G[2 * n + p];
                        const double g12 = G[3 * n + p], g13 = G[4 * n + p], g23 = G[5 * n + p];
                        wr[q] = c * (g11 * ur + g12 * us + g13 * ut);
                        ws[q] = c * (g12 * ur + g22 * us + g23 * ut);
                        wt[q] = c * (g13 * ur + g23 * us + g33 * ut);
                    }
            for (int k = 0; k < lx; ++k)
                for (int j = 0; j < lx; ++j)
                    for (int i = 0; i < lx; ++i) {
                        double s = 0.0;
                        for (int l = 0; l < lx; ++l) {
                            s += D[l * lx + i] * wr[l + lx * (j + lx * k)];
                            s += D[l * lx + j] * ws[i + lx * (l + lx * k)];
                            s += D[l * lx + k] * wt[i + lx * (j + lx * l)];
                        }
                        const int64_t p = e * npe + i + lx * (j + (int64_t)lx * k);
                        const double c2 = h2 ? h2[p] : h2s;
                        if (c2 != 0.0) s += c2 * B[p] * ue[i + lx * (j + lx * k)];
                        w[p] = s;
                    }
        }
        free(wr);
        free(ws);
        free(wt);
    }
}

/*
 * Adjoint of A_L with respect to h1 (the h1-linearity of Eq. 9):
 *   g_p = [vr vs vt]_p  G_p  [ur us ut]_p^T,
 * so that d(v^T A_L(h1) u)/d h1_p = g_p and sum_p h1_p g_p = v^T A_L u for h2 = 0.
 */
EXPORT void orc_ax_adjoint(int64_t nelv, int lx, const double *D, const double *G,
                           const double *u, const double *v, double *g)
{
    const int64_t npe = (int64_t)lx * lx * lx;
    const int64_t n = nelv * npe;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nelv; ++e) {
        const double *ue = u + e * npe, *ve = v + e * npe;
        for (int k = 0; k < lx; ++k)
            for (int j = 0; j < lx; ++j)
                for (int i = 0; i < lx; ++i) {
                    double ur = 0, us = 0, ut = 0, vr = 0, vs = 0, vt = 0;
                    for (int l = 0; l < lx; ++l) {
                        ur += D[i * lx + l] * ue[l + lx * (j + lx * k)];
                        us += D[j * lx + l] * ue[i + lx * (l + lx * k)];
                        ut += D[k * lx + l] * ue[i + lx * (j + lx * l)];
                        vr += D[i * lx + l] * ve[l + lx * (j + lx * k)];
                        vs += D[j * lx + l] * ve[i + lx * (l + lx * k)];
                        vt += D[k * lx + l] * ve[i + lx * (j + lx * l)];
                    }
                    const int64_t p = e * npe + i + lx * (j + (int64_t)lx * k);
                    const double g11 = G[0 * n + p], g22 = G[1 * n + p], g33 = G[2 * n + p];
                    const double g12 = G[3 * n + p], g13 = G[4 * n + p], g23 = G[5 * n + p];
                    g[p] = vr * (g11 * ur + g12 * us + g13 * ut)
                         + vs * (g12 * ur + g22 * us + g23 * ut)
                         + vt * (g13 * ur + g23 * us + g33 * ut);
                }
    }
}

/* ------------------------------------------------------------------ */
/*
 * Gather-scatter QQ^T (Eq. 10; local gather+scatter of Algorithm 1).
 * The oracle keeps every global id with two or more local copies as a
 * group: the copies' local indices in ascending order, groups in ascending
 * global id.
 */
typedef struct {
    int64_t n;        /* local points */
    int64_t ngroups;  /* ids with multiplicity >= 2 */
    int64_t *off;     /* ngroups+1 */
    int64_t *idx;     /* off[ngroups] local indices */
    int64_t *gid;     /* ngroups global ids */
} orc_gs;

typedef struct { int64_t g, i; } gi_pair;

static int cmp_gi(const void *a, const void *b)
{
    const gi_pair *x = a, *y = b;
    if (x->g != y->g) return x->g < y->g ? -1 : 1;
    return (x->i > y->i) - (x->i < y->i);
}

EXPORT orc_gs *orc_gs_create(int64_t n, const int64_t *glb)
{
    gi_pair *s = malloc(sizeof(gi_pair) * (n > 0 ? n : 1));
    for (int64_t p = 0; p < n; ++p) { s[p].g = glb[p]; s[p].i = p; }
    qsort(s, n, sizeof(gi_pair), cmp_gi);
    orc_gs *gs = calloc(1, sizeof(orc_gs));
    gs->n = n;
    int64_t ng = 0, ne = 0;
    for (int64_t a = 0; a < n;) {
        int64_t b = a;
        while (b < n && s[b].g == s[a].g) ++b;
        if (b - a >= 2) { ng += 1; ne += b - a; }
        a = b;
    }
    gs->ngroups = ng;
    gs->off = malloc(sizeof(int64_t) * (ng + 1));
    gs->idx = malloc(sizeof(int64_t) * (ne > 0 ? ne : 1));
    gs->gid = malloc(sizeof(int64_t) * (ng > 0 ? ng : 1));
    ng = 0;
    ne = 0;
    gs->off[0] = 0;
    for (int64_t a = 0; a < n;) {
        int64_t b = a;
        while (b < n && s[b].g == s[a].g) ++b;
        if (b - a >= 2) {
            for (int64_t c = a; c < b; ++c) gs->idx[ne++] = s[c].i;
            gs->gid[ng] = s[a].g;
            gs->off[++ng] = ne;
        }
        a = b;
    }
    free(s);
    return gs;
}

EXPORT int64_t orc_gs_ngroups(const orc_gs *gs) { return gs->ngroups; }
EXPORT int64_t orc_gs_nentries(const orc_gs *gs) { return gs->off[gs->ngroups]; }

EXPORT void orc_gs_groups(const orc_gs *gs, int64_t *off, int64_t *idx, int64_t *gid)
{
    memcpy(off, gs->off, sizeof(int64_t) * (gs->ngroups + 1));
    memcpy(idx, gs->idx, sizeof(int64_t) * gs->off[gs->ngroups]);
    memcpy(gid, gs->gid, sizeof(int64_t) * gs->ngroups);
}

/* u <- QQ^T u: sum the copies sequentially in ascending local order, write back. */
EXPORT void orc_gs_op(const orc_gs *gs, double *u)
{
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < gs->ngroups; ++g) {
        double s = 0.0;
        for (int64_t c = gs->off[g]; c < gs->off[g + 1]; ++c) s += u[gs->idx[c]];
        for (int64_t c = gs->off[g]; c < gs->off[g + 1]; ++c) u[gs->idx[c]] = s;
    }
}

EXPORT void orc_gs_free(orc_gs *gs)
{
    if (!gs) return;
    free(gs->off);
    free(gs->idx);
    free(gs->gid);
    free(gs);
}

/* multiplicity of every local point: QQ^T applied to ones */
EXPORT void orc_multiplicity(const orc_gs *gs, double *mult)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < gs->n; ++p) mult[p] = 1.0;
    orc_gs_op(gs, mult);
}

/* ------------------------------------------------------------------ */
/*
 * Assembled, masked operator in local layout: w = mask QQ^T A_L u (Eq. 10 with
 * homogeneous Dirichlet rows zeroed).
 */
EXPORT void orc_apply(int64_t nelv, int lx, const double *D, const double *G,
                      const double *B, const double *h1, double h1s,
                      const double *h2, double h2s, const orc_gs *gs,
                      const uint8_t *dirichlet, const double *u, double *w)
{
    const int64_t n = nelv * (int64_t)lx * lx * lx;
    orc_ax_helm(nelv, lx, D, G, B, h1, h1s, h2, h2s, u, w);
    orc_gs_op(gs, w);
    if (dirichlet)
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < n; ++p)
            if (dirichlet[p]) w[p] = 0.0;
}

/*
 * Diagonal of the unassembled operator at every local point (point-Jacobi
 * reading of the velocity preconditioner, Section 4):
 *   d_ijk = sum_l D[l][i]^2 (h1 G11)_ljk + sum_l D[l][j]^2 (h1 G22)_ilk
 *         + sum_l D[l][k]^2 (h1 G33)_ijl
 *         + 2 D[i][i] D[j][j] (h1 G12)_ijk + 2 D[i][i] D[k][k] (h1 G13)_ijk
 *         + 2 D[j][j] D[k][k] (h1 G23)_ijk + h2 B_ijk
 * (the diagonal of sum_ab D_a^T diag(h1 G_ab) D_b; cross terms survive only at
 * points where the D diagonal entries are non-zero).
 */
EXPORT void orc_diag(int64_t nelv, int lx, const double *D, const double *G,
                     const double *B, const double *h1, double h1s,
                     const double *h2, double h2s, double *d)
{
    const int64_t npe = (int64_t)lx * lx * lx;
    const int64_t n = nelv * npe;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nelv; ++e) {
        const int64_t b0 = e * npe;
        for (int k = 0; k < lx; ++k)
            for (int j = 0; j < lx; ++j)
                for (int i = 0; i < lx; ++i) {
                    const int64_t p = b0 + i + lx * (j + (int64_t)lx * k);
                    double s = 0.0;
                    for (int l = 0; l < lx; ++l) {
                        const int64_t pr = b0 + l + lx * (j + (int64_t)lx * k);
                        const int64_t ps = b0 + i + lx * (l + (int64_t)lx * k);
                        const int64_t pt = b0 + i + lx * (j + (int64_t)lx * l);
                        const double cr = h1 ? h1[pr] : h1s;
                        const double cs = h1 ? h1[ps] : h1s;
                        const double ct = h1 ? h1[pt] : h1s;
                        s += D[l * lx + i] * D[l * lx + i] * cr * G[0 * n + pr];
                        s += D[l * lx + j] * D[l * lx + j] * cs * G[1 * n + ps];
                        s += D[l * lx + k] * D[l * lx + k] * ct * G[2 * n + pt];
                    }
                    const double c = h1 ? h1[p] : h1s;
                    const double di = D[i * lx + i], dj = D[j * lx + j], dk = D[k * lx + k];
                    s += 2.0 * di * dj * c * G[3 * n + p];
                    s += 2.0 * di * dk * c * G[4 * n + p];
                    s += 2.0 * dj * dk * c * G[5 * n + p];
                    const double c2 = h2 ? h2[p] : h2s;
                    if (c2 != 0.0) s += c2 * B[p];
                    d[p] = s;
                }
    }
}

/* Jacobi inverse: dinv = 1 / QQ^T(diag), zero on Dirichlet points. */
EXPORT void orc_jacobi_dinv(int64_t nelv, int lx, const double *D, const double *G,
                            const double *B, const double *h1, double h1s,
                            const double *h2, double h2s, const orc_gs *gs,
                            const uint8_t *dirichlet, double *dinv)
{
    const int64_t n = nelv * (int64_t)lx * lx * lx;
    orc_diag(nelv, lx, D, G, B, h1, h1s, h2, h2s, dinv);
    orc_gs_op(gs, dinv);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p)
        dinv[p] = (dirichlet && dirichlet[p]) ? 0.0 : 1.0 / dinv[p];
}

/* (a, b) = sum_L a_L b_L / mult_L */
static double wdot(int64_t n, const double *a, const double *b, const double *mult)
{
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (int64_t p = 0; p < n; ++p) s += a[p] * b[p] / mult[p];
    return s;
}

EXPORT double orc_wdot(int64_t n, const double *a, const double *b, const double *mult)
{
    return wdot(n, a, b, mult);
}

/*
 * Jacobi-preconditioned conjugate gradients on mask QQ^T A_L x = b (the
 * velocity solver of Section 4 with the point-Jacobi reading), textbook form:
 *   r = b - A x, z = dinv r, p = z;
 *   repeat: w = A p; alpha = (r,z)/(p,w); x += alpha p; r -= alpha w;
 *           stop if |r|/|b| <= rtol; z = dinv r; beta = (r,z)_new/(r,z)_old;
 *           p = z + beta p.
 * Norms and dots are the 1/mult-weighted products.  rtol <= 0 runs exactly
 * max_iter iterations.  x holds the initial guess on entry.  progress (may be NULL)
 * is called with the iteration count and |r|/|b| every `every` iterations.
 * Returns 0 converged (or fixed count done), 1 not converged, 2 breakdown.
 */
typedef void (*orc_progress_fn)(int iteration, double rel_res);

EXPORT int orc_pcg(int64_t nelv, int lx, const double *D, const double *G,
                   const double *B, const double *h1, double h1s,
                   const double *h2, double h2s, const orc_gs *gs,
                   const uint8_t *dirichlet, const double *dinv,
                   const double *b, double *x, double rtol, int max_iter,
                   int *iters_out, double *relres_out, orc_progress_fn progress, int every)
{
    const int64_t n = nelv * (int64_t)lx * lx * lx;
    double *mult = malloc(sizeof(double) * n);
    double *r = malloc(sizeof(double) * n);
    double *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n);
    double *w = malloc(sizeof(double) * n);
    orc_multiplicity(gs, mult);

    orc_apply(nelv, lx, D, G, B, h1, h1s, h2, h2s, gs, dirichlet, x, w);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) r[q] = b[q] - w[q];
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) z[q] = dinv[q] * r[q];
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) p[q] = z[q];
    const double bnorm = sqrt(wdot(n, b, b, mult));
    double rz = wdot(n, r, z, mult);
    double rel = sqrt(wdot(n, r, r, mult)) / (bnorm > 0 ? bnorm : 1.0);
    int it = 0, status = 1;
    if (bnorm == 0.0 || (rtol > 0 && rel <= rtol)) status = 0;
    while (status == 1 && it < max_iter) {
        orc_apply(nelv, lx, D, G, B, h1, h1s, h2, h2s, gs, dirichlet, p, w);
        const double pw = wdot(n, p, w, mult);
        if (!(pw > 0.0) || !isfinite(rz)) { status = 2; break; }
        const double alpha = rz / pw;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n; ++q) x[q] += alpha * p[q];
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n; ++q) r[q] -= alpha * w[q];
        it += 1;
        rel = sqrt(wdot(n, r, r, mult)) / bnorm;
        if (progress && every > 0 && it % every == 0) progress(it, rel);
        if (rtol > 0 && rel <= rtol) { status = 0; break; }
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n; ++q) z[q] = dinv[q] * r[q];
        const double rz_new = wdot(n, r, z, mult);
        if (rz_new == 0.0) { status = 0; break; }
        const double beta = rz_new / rz;
        rz = rz_new;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n; ++q) p[q] = z[q] + beta * p[q];
    }
    if (status == 1 && rtol <= 0 && it == max_iter) status = 0;
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = rel;
    free(mult);
    free(r);
    free(z);
    free(p);
    free(w);
    return status;
}
