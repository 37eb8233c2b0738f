// schwarz_kernels.hip -- local solves and coarse prolongation of the two-level
// additive Schwarz preconditioner of the pressure solve (Section 4 of arXiv
// 2107.01243), for gfx950.
//
// The local problem of an element is a separable box operator
//   A~ = h1 (Mt x Ms x Kr + Mt x Ks x Mr + Kt x Ms x Mr) + h2 Mt x Ms x Mr,
// solved by fast diagonalisation: with, per direction, the eigenvectors S (row-major
// [node][mode]) and eigenvalues of the 1-D generalised problem K S = M S Lambda,
//   z = (St x Ss x Sr) diag(1 / (h1 (lr_i + ls_j + lt_k) + h2)) (St x Ss x Sr)^T r.
// Two boxes: the element's own lx^3 points (k_fdm), and those points plus one layer
// of extension points beyond every face (k_fdm_ov, (lx + 2)^3 points: the minimal
// overlap of one point, the extension layer's right-hand side gathered from the face
// neighbour; only the element's own points are written back).
//
// Compiled once per lx (-DSEM_LX=<lx>), like the operator kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sem_kernels.h"
#include "sem_pencil.h"

#ifndef SEM_LX
#error "compile with -DSEM_LX=<lx>"
#endif

namespace sem {

// y = M x along one pencil of X points, M row-major (a copy of S or of its transpose in
// LDS), each y[m] summed over ascending l.
template <int X>
__device__ __forceinline__ void fdm_mul(const double *M, const double (&x)[X], double (&y)[X])
{
#pragma unroll
    for (int m = 0; m < X; ++m) {
        double s = M[m * X] * x[0];
#pragma unroll
        for (int l = 1; l < X; ++l) s = fma(M[m * X + l], x[l], s);
        y[m] = s;
    }
}

// Stage one element's S (3 X^2 values) and lambda (3 X) in LDS with coalesced loads:
// S is kept twice, transposed for the forward transforms and as is for the inverse
// ones, so that the two phases read distinct arrays and no matrix stays live in
// registers between them (both are read back as broadcasts).
template <int X, int NT>
__device__ __forceinline__ void fdm_stage(const double *Se, const double *le, double *Sf, double *Si, double *lam,
                                          int t)
{
    constexpr int X2 = X * X;
    for (int q = t; q < 3 * X2; q += NT) {
        const double v = Se[q];
        const int d = q / X2, l = (q % X2) / X, m = q % X;
        Si[q] = v;
        Sf[d * X2 + m * X + l] = v;
    }
    for (int q = t; q < 3 * X; q += NT) lam[q] = le[q];
}

// Coarse restriction of one element: pr[h] = the sum over the element's owned points
// of r times the trilinear function of corner q = t + h NT (for q < 8; corner
// c = a + 2 b + 4 c'), from each pencil's sums s0, s1 against the two linear functions
// along t (lane t holds pencil tl when own is set), then along s and along r through
// LDS, in a fixed order.  red: 2 lx^2 + 4 lx doubles.
template <int LX, int NT>
__device__ __forceinline__ void corner_sums(double s0, double s1, bool own, int tl, int t, const double *lin,
                                            double *red, double (&pr)[(8 + NT - 1) / NT])
{
    constexpr int L2 = LX * LX, NQ = (8 + NT - 1) / NT;
    if (own) {
        red[tl] = s0;
        red[L2 + tl] = s1;
    }
    bsync<NT>();
    for (int q = t; q < 4 * LX; q += NT) {
        const int i = q % LX, cb = q / LX;  // cb = (j side) + 2 (k side)
        const double *rk = red + (cb >> 1) * L2 + i;
        const double *lj = lin + (cb & 1) * LX;
        double s = 0.0;
        for (int j = 0; j < LX; ++j) s = fma(lj[j], rk[LX * j], s);
        red[2 * L2 + q] = s;
    }
    bsync<NT>();
#pragma unroll
    for (int h = 0; h < NQ; ++h) {
        const int q = t + h * NT;
        if (q >= 8) break;
        const double *li = lin + (q & 1) * LX;
        const double *u = red + 2 * L2 + (q >> 1) * LX;
        double s = 0.0;
        for (int i = 0; i < LX; ++i) s = fma(li[i], u[i], s);
        pr[h] = s;
    }
}

// The fast-diagonalisation solve on an X^3 box held as t-pencils (lane t = a + X b holds
// points (a, b, 0..X-1) in x): forward transform along t in registers, along r and
// along s through the box in LDS (row stride X + 1), the division by
// h1 (lr_a + ls_j + lt_b) + h2, and the inverse transforms along s and along r.  The
// result is left in cube for the caller's inverse transform along t.  Expects S and
// lambda staged and a barrier after the staging.
template <int X, int NT>
__device__ __forceinline__ void fdm_core(double (&x)[X], double (&y)[X], double *cube, const double *Sf,
                                         const double *Si, const double *lam, double h1, double h2, int a, int b)
{
    constexpr int X2 = X * X;
    fdm_mul<X>(Sf + 2 * X2, x, y);
#pragma unroll
    for (int k = 0; k < X; ++k) cube[lidx<X>(a, b, k)] = y[k];
    bsync<NT>();
    // r-pencil (j = a, k = b)
#pragma unroll
    for (int i = 0; i < X; ++i) x[i] = cube[lidx<X>(i, a, b)];
    fdm_mul<X>(Sf, x, y);
#pragma unroll
    for (int i = 0; i < X; ++i) cube[lidx<X>(i, a, b)] = y[i];
    bsync<NT>();
    // s-pencil (i = a, k = b)
#pragma unroll
    for (int j = 0; j < X; ++j) x[j] = cube[lidx<X>(a, j, b)];
    fdm_mul<X>(Sf + X2, x, y);
    {
        const double lra = lam[a], ltb = lam[2 * X + b];
#pragma unroll
        for (int j = 0; j < X; ++j) y[j] /= h1 * (lra + lam[X + j] + ltb) + h2;
    }
    fdm_mul<X>(Si + X2, y, x);
#pragma unroll
    for (int j = 0; j < X; ++j) cube[lidx<X>(a, j, b)] = x[j];
    bsync<NT>();
#pragma unroll
    for (int i = 0; i < X; ++i) y[i] = cube[lidx<X>(i, a, b)];
    fdm_mul<X>(Si, y, x);
#pragma unroll
    for (int i = 0; i < X; ++i) cube[lidx<X>(i, a, b)] = x[i];
    bsync<NT>();
}

// Element's own box: one element per workgroup of lx^2 lanes.  Lane t = a + lx b keeps
// its t-pencil (i = a, j = b) in registers, so the two t-direction transforms are
// register-only.
template <int LX>
__global__ __launch_bounds__(LX * LX) void k_fdm(FdmArgs A)
{
    constexpr int L2 = LX * LX, L3 = L2 * LX, NT = L2, NQ = (8 + NT - 1) / NT;
    __shared__ double cube[L2 * (LX + 1)];
    __shared__ double red[2 * L2 + 4 * LX];
    __shared__ __align__(16) double Sf[3 * L2];  // S^T per direction (forward)
    __shared__ __align__(16) double Si[3 * L2];  // S per direction (inverse)
    __shared__ double lam[3 * LX];
    const int64_t e = blockIdx.x;
    const int t = threadIdx.x, a = t % LX, b = t / LX;
    fdm_stage<LX, NT>(A.S + e * 3 * L2, A.lam + e * 3 * LX, Sf, Si, lam, t);
    const double *__restrict__ lin = A.lin;
    double x[LX], y[LX];
    const double *r = A.r + e * L3;
#pragma unroll
    for (int k = 0; k < LX; ++k) x[k] = r[k * L2 + t];
    double pr[NQ];
    if (A.part) {
        const uint8_t *ow = A.owner + e * L3;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < LX; ++k) {
            const double v = ow[k * L2 + t] ? x[k] : 0.0;
            s0 = fma(lin[k], v, s0);
            s1 = fma(lin[LX + k], v, s1);
        }
        corner_sums<LX, NT>(s0, s1, true, t, t, lin, red, pr);
    }
    bsync<NT>();  // S and lambda staged
    fdm_core<LX, NT>(x, y, cube, Sf, Si, lam, A.h1, A.h2, a, b);
#pragma unroll
    for (int k = 0; k < LX; ++k) y[k] = cube[lidx<LX>(a, b, k)];
    fdm_mul<LX>(Si + 2 * L2, y, x);
    double *z = A.z + e * L3;
#pragma unroll
    for (int k = 0; k < LX; ++k) z[k * L2 + t] = x[k];
    if (A.part) {
#pragma unroll
        for (int h = 0; h < NQ; ++h) {
            const int q = t + h * NT;
            if (q >= 8) break;
            A.part[e * 8 + q] = pr[h];
        }
    }
}

// Residual at the extension point of face f (face coordinates fa, fb) of the element
// whose face table fc (6 x {neighbour, base, sa, sb}) is staged in LDS; zero where the
// face has no neighbour.
template <int LX>
__device__ __forceinline__ double ext_value(const double *__restrict__ r, const int32_t *fc, int f, int fa, int fb)
{
    constexpr int64_t L3 = (int64_t)LX * LX * LX;
    const int32_t e2 = fc[4 * f];
    if (e2 < 0) return 0.0;
    return r[(int64_t)e2 * L3 + fc[4 * f + 1] + fa * fc[4 * f + 2] + fb * fc[4 * f + 3]];
}

// Element box extended by one point beyond each face: one element per workgroup of
// X^2 lanes, X = lx + 2.  Lane t = a + X b holds the extended t-pencil (a, b, 0..X-1);
// extended coordinate c is element coordinate c - 1.  Its right-hand side:
//  - own points (1 <= a, b, k <= lx): r of the element, read coalesced per t-slab;
//  - one coordinate outside (a face layer): r at the neighbour's point one GLL index
//    inside it (face table A.face), zero without a neighbour;
//  - two or three coordinates outside (box edges and corners): zero.
// The 1-D operators of a face without a neighbour hold a decoupled extension node, so
// with its zero right-hand side the solve there equals the element-only one.  Only the
// own points are transformed back along t and written.
template <int LX>
__global__ __launch_bounds__((LX + 2) * (LX + 2)) void k_fdm_ov(FdmArgs A)
{
    constexpr int X = LX + 2, X2 = X * X, L2 = LX * LX, L3 = L2 * LX, NT = X2, NQ = (8 + NT - 1) / NT;
    __shared__ double cube[X2 * (X + 1)];
    __shared__ double red[2 * L2 + 4 * LX];
    __shared__ __align__(16) double Sf[3 * X2];
    __shared__ __align__(16) double Si[3 * X2];
    __shared__ double lam[3 * X];
    __shared__ int32_t fc[24];
    const int64_t e = blockIdx.x;
    const int t = threadIdx.x, a = t % X, b = t / X;
    fdm_stage<X, NT>(A.S + e * 3 * X2, A.lam + e * 3 * X, Sf, Si, lam, t);
    for (int q = t; q < 24; q += NT) fc[q] = A.face[e * 24 + q];  // NT is 16 at lx = 2
    bsync<NT>();  // face table, S and lambda staged
    const double *__restrict__ r = A.r;
    const bool ia = a >= 1 && a <= LX, ib = b >= 1 && b <= LX, own = ia && ib;
    double x[X], y[X];
#pragma unroll
    for (int k = 0; k < X; ++k) x[k] = 0.0;
    if (own) {
        const double *re = r + e * L3 + (a - 1) + LX * (b - 1);
#pragma unroll
        for (int k = 0; k < LX; ++k) x[k + 1] = re[k * L2];
        x[0] = ext_value<LX>(r, fc, 4, a - 1, b - 1);      // face t = 0
        x[X - 1] = ext_value<LX>(r, fc, 5, a - 1, b - 1);  // face t = lx - 1
    } else if (ia != ib) {
        // an r face layer (a outside: face coordinates (j, k)) or an s face layer
        // (b outside: face coordinates (i, k))
        const int f = ib ? (a == X - 1 ? 1 : 0) : (b == X - 1 ? 3 : 2);
        const int fa = ib ? b - 1 : a - 1;
#pragma unroll
        for (int k = 0; k < LX; ++k) x[k + 1] = ext_value<LX>(r, fc, f, fa, k);
    }
    double pr[NQ];
    if (A.part) {
        double s0 = 0.0, s1 = 0.0;
        if (own) {
            const uint8_t *ow = A.owner + e * L3 + (a - 1) + LX * (b - 1);
            const double *__restrict__ lin = A.lin;
#pragma unroll
            for (int k = 0; k < LX; ++k) {
                const double v = ow[k * L2] ? x[k + 1] : 0.0;
                s0 = fma(lin[k], v, s0);
                s1 = fma(lin[LX + k], v, s1);
            }
        }
        corner_sums<LX, NT>(s0, s1, own, (a - 1) + LX * (b - 1), t, A.lin, red, pr);
    }
    fdm_core<X, NT>(x, y, cube, Sf, Si, lam, A.h1, A.h2, a, b);
    if (own) {
#pragma unroll
        for (int k = 0; k < X; ++k) y[k] = cube[lidx<X>(a, b, k)];
        double *z = A.z + e * L3 + (a - 1) + LX * (b - 1);
        const double *St = Si + 2 * X2;
#pragma unroll
        for (int m = 1; m <= LX; ++m) {
            double s = St[m * X] * y[0];
#pragma unroll
            for (int l = 1; l < X; ++l) s = fma(St[m * X + l], y[l], s);
            z[(m - 1) * L2] = s;
        }
    }
    if (A.part) {
#pragma unroll
        for (int h = 0; h < NQ; ++h) {
            const int q = t + h * NT;
            if (q >= 8) break;
            A.part[e * 8 + q] = pr[h];
        }
    }
}

// Coarse prolongation: the element's eight coarse values interpolated trilinearly
// (along r, then s on the two t faces, then t per point), added to the
// multiplicity-averaged local solution.  Lanes as in the t-pencil layout; whole
// elements per workgroup.
template <int LX>
struct ProlongShape {
    static constexpr int L2 = LX * LX;
    static constexpr int EPB = 256 / L2 > 0 ? 256 / L2 : 1;
    static constexpr int NT = EPB * L2;
};

template <int LX>
__global__ __launch_bounds__(ProlongShape<LX>::NT) void k_prolong(ProlongArgs A)
{
    constexpr int L2 = LX * LX, L3 = L2 * LX, EPB = ProlongShape<LX>::EPB;
    const int el = threadIdx.x / L2, t = threadIdx.x - el * L2;
    const int64_t e = (int64_t)blockIdx.x * EPB + el;
    if (e >= A.nelv) return;
    const int a = t % LX, b = t / LX;
    const double *__restrict__ lin = A.lin;
    double c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = A.e0[A.cvert[e * 8 + q]];
    const double ra0 = lin[a], ra1 = lin[LX + a], sb0 = lin[b], sb1 = lin[LX + b];
    double f[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
        const double y0 = fma(ra1, c[4 * kc + 1], ra0 * c[4 * kc]);
        const double y1 = fma(ra1, c[4 * kc + 3], ra0 * c[4 * kc + 2]);
        f[kc] = fma(sb1, y1, sb0 * y0);
    }
    double *z = A.z + e * L3;
    const uint8_t *mu = A.mult + e * L3;
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        const double v = fma(lin[LX + k], f[1], lin[k] * f[0]);
        z[k * L2 + t] = z[k * L2 + t] / (double)mu[k * L2 + t] + v;
    }
}

}  // namespace sem

#define SEM_PASTE2(a, b) a##b
#define SEM_PASTE(a, b) SEM_PASTE2(a, b)

extern "C" {

// A->face set: the extended box (S, lam of size lx + 2 per direction); else the
// element's own box.
hipError_t SEM_PASTE(sem_launch_fdm_lx, SEM_LX)(const sem::FdmArgs *A, hipStream_t st)
{
    if (A->nelv == 0) return hipSuccess;
    if (A->nelv > 0x7fffffff) return hipErrorInvalidValue;
    if (A->part && (!A->owner || !A->lin)) return hipErrorInvalidValue;
    if (A->face)
        hipLaunchKernelGGL((sem::k_fdm_ov<SEM_LX>), dim3((unsigned)A->nelv), dim3((SEM_LX + 2) * (SEM_LX + 2)), 0,
                           st, *A);
    else
        hipLaunchKernelGGL((sem::k_fdm<SEM_LX>), dim3((unsigned)A->nelv), dim3(SEM_LX * SEM_LX), 0, st, *A);
    return hipGetLastError();
}
hipError_t SEM_PASTE(sem_launch_prolong_lx, SEM_LX)(const sem::ProlongArgs *A, hipStream_t st)
{
    using Sh = sem::ProlongShape<SEM_LX>;
    if (A->nelv == 0) return hipSuccess;
    const int64_t g = (A->nelv + Sh::EPB - 1) / Sh::EPB;
    if (g > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sem::k_prolong<SEM_LX>), dim3((unsigned)g), dim3(Sh::NT), 0, st, *A);
    return hipGetLastError();
}

}  // extern "C"
