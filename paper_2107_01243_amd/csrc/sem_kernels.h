// sem_kernels.h -- argument blocks shared by the HIP kernels and the host driver
// of libsem (internal; not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sem {

// 1-D GLL derivative matrix d[i*LX + l] = l_l'(xi_i), passed by value so that it
// sits in the kernel-argument segment and is read with scalar loads.
template <int LX, typename T>
struct DMat {
    T d[LX * LX];
};

// Even-odd form of D used by the operator kernels.  GLL points are symmetric, so
// D is centro-antisymmetric: D[N-m][N-l] = -D[m][l] (N = LX-1).  With H = LX/2,
// e_l = u_l + u_{N-l}, o_l = u_l - u_{N-l} (l < H) and c = u_H (odd LX only):
//   (D u)_m     =  sum_l S[m][l] e_l + cm[m] c + sum_l A[m][l] o_l
//   (D u)_{N-m} = -sum_l S[m][l] e_l - cm[m] c + sum_l A[m][l] o_l      (m < H)
//   (D u)_H     =  sum_l rm[l] o_l                                      (odd LX)
// with S = (D[m][l] + D[m][N-l])/2, A = (D[m][l] - D[m][N-l])/2, cm[m] = D[m][H],
// rm[l] = D[H][l].  D^T has the same structure with S^T -> A and A^T -> S, so one
// set of constants serves both products (half the FMAs of the dense product, and
// half the wave-uniform constants).
template <int LX, typename T>
struct DEo {
    static constexpr int H = LX / 2;
    static constexpr int HM = (LX % 2) ? H : 1;
    T S[H * H];
    T A[H * H];
    T cm[HM];
    T rm[HM];
};

template <int LX>
struct WVec {
    double w[LX];
};

// w = A_L u
template <typename T>
struct AxArgs {
    T *w;
    const T *u;
    const T *G;   // 6 planes of n
    const T *B;   // n (read only when the mass term is active)
    const T *h1;  // n or nullptr (then h1s)
    const T *h2;  // n or nullptr (then h2s)
    T h1s, h2s;
    int64_t n;    // points per field
    int64_t nelv;
    const void *deo = nullptr;  // device copy of the even-odd D of this lx and precision
};

// Per-field scalars of one CG solve, resident in device memory.
struct CgScalars {
    double rz;      // (r, z) of the current iterate
    double alpha;
    double beta;    // used by the next matvec: p = z + beta p
    double rr;      // (r, r)
    double bb;      // (b, b)
    double rtol;
    int iter;       // iterations completed
    int max_iter;
    int stop;       // nonzero: this field's iterates are frozen
    int status;     // 0 running/converged, 1 not converged, 2 breakdown
    int primed;     // single-reduction CG: 0 until the first step length is set
};

// p = dinv r + beta p;  w = A_L p;  per-workgroup partial sums of p.w.
// Single-reduction form: u = dinv r;  w = A_L u;  partial sums of u.w.
template <typename T>
struct CgMatvecArgs {
    T *p;
    T *w;
    const T *r;
    const T *dinv;
    const T *G;
    const T *B;
    const T *h1;
    const T *h2;
    T h1s, h2s;
    int64_t n;
    int64_t nelv;
    const CgScalars *scal;  // one per field
    double *partial;        // [field][workgroup]
    const void *deo = nullptr;  // device copy of the even-odd D of this lx and precision
};

template <typename T>
struct AdjArgs {
    T *g;
    const T *u;
    const T *v;
    const T *G;
    int64_t n;
    int64_t nelv;
    const void *deo = nullptr;  // device copy of the even-odd D of this lx and precision
};

struct GeomArgs {
    const double *xyz;  // 3 planes of n
    double *G;          // 6 planes of n
    double *B;
    unsigned *nbad;     // count of points with J <= 0
    int64_t n;
};

struct DiagArgs {
    double *d;
    const double *G;
    const double *B;
    const double *h1;
    const double *h2;
    double h1s, h2s;
    int64_t n;
};

// Local solves of the two-level Schwarz preconditioner (fast diagonalisation):
// z_e = (S_t x S_s x S_r) diag(1 / (h1 (lr_i + ls_j + lt_k) + h2)) (S_t x S_s x S_r)^T r_e,
// with per element and direction the eigenvectors S (row-major [point][mode]) and
// eigenvalues of the 1-D generalised problem K S = M S Lambda, on the element's own
// box (X = lx points per direction) or, when face is set, on the box extended by one
// point beyond each face (X = lx + 2; the extension layers' right-hand side is the
// face neighbours' residual, see face; only the own points of z are written).  When
// part is set, the same pass also forms the coarse restriction of r: per element the
// eight sums over its owned points of r times the trilinear corner functions.
struct FdmArgs {
    double *z;             // [nelv][lx^3]
    const double *r;       // [nelv][lx^3]
    const double *S;       // [nelv][3][X][X]
    const double *lam;     // [nelv][3][X]
    const uint8_t *owner;  // [nelv][lx^3] one copy per global id (restriction weights)
    const double *lin;     // [2][lx]: (1 - xi_i) / 2, (1 + xi_i) / 2 at the GLL points
    double *part;          // [nelv][8] restriction sums (corner c = a + 2 b + 4 c'), or nullptr
    // [nelv][6][4] or nullptr: per face f = 2 d + side {e2, base, sa, sb}: the point of
    // neighbour e2 under face point (fa, fb) (fa, fb the two other local coordinates,
    // ascending direction order) is base + fa sa + fb sb in e2; e2 = -1: no neighbour
    const int32_t *face;
    double h1, h2;
    int64_t nelv;
};

// Coarse prolongation with the multiplicity average of the local solves:
// z = z / mult + sum over the eight corners c of e0[cvert[e][c]] phi_c, phi_c the
// trilinear corner function (a product of the linear functions in lin).
struct ProlongArgs {
    double *z;
    const uint8_t *mult;
    const double *lin;     // [2][lx]
    const double *e0;      // coarse vector
    const int32_t *cvert;  // [nelv][8]
    int64_t nelv;
};

}  // namespace sem
