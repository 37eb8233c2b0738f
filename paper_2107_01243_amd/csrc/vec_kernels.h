// vec_kernels.h -- argument blocks of the gather-scatter and Krylov-vector kernels
// (internal to libsem).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sem_kernels.h"

namespace sem {

// CG scalars folded into the gather-scatter launch from the partial sums of the
// kernels before it.  partial [field][nblk]: the matvec's (v, A v).
// mode 0 (two-reduction CG): alpha_f = rz_f / (p, A p)_f.
// mode 1 (single-reduction CG): with (r, u) and (r, r) from the update's partials
// partial2 [2][field][nblk2] (or, before the first step, from the scalars), gives
// beta, alpha, the iteration count and the stopping state.
struct AlphaJob {
    const double *partial;
    int64_t nblk;
    CgScalars *scal;
    int mode;
    const double *partial2;
    int64_t nblk2;
};

// Single-reduction CG update: p = dinv r + beta p; s = w + beta s; x += alpha p;
// r -= alpha s (not on Dirichlet points); partial sums of the new (r, dinv r), (r, r).
struct Cg1UpdateArgs {
    double *x;
    double *r;
    double *p;
    double *s;
    const double *w;
    const double *dinv;
    const uint8_t *owner;
    const CgScalars *scal;
    double *partial;  // [2][field][grid]: (r, dinv r), (r, r) of the updated r
    int64_t n;
    int nfields;
};

template <typename T>
struct GsArgs {
    T *u;
    const int32_t *pairs;    // 2 * npairs
    const int64_t *blk_ptr;  // nblocks + 1
    const int32_t *blk_idx;
    int64_t npairs, nblocks;
    int64_t n;               // points per field
    int nfields;
    const CgScalars *skip;   // optional: fields with skip[f].stop are left untouched
    const AlphaJob *alpha_job;  // optional (device pointer)
    // entry-parallel form (used when nent > 0; pairs/blocks then hold only groups
    // with more than 64 copies)
    // one word per entry: the local index, bit 31 set on the first entry of a group;
    // 0xffffffff pads a 64-entry segment (no group straddles a segment)
    const uint32_t *ent_word;
    int64_t nent;
    int max_group;
};

template <typename T>
struct CgInitArgs {
    const T *b;
    const T *w;       // QQ^T A_L x0, or nullptr when x0 = 0
    T *r;
    T *p;
    const T *dinv;
    const uint8_t *owner;
    double *partial;  // [3][field][grid]
    int64_t n;
    int nfields;
};

template <typename T>
struct CgUpdateArgs {
    T *x;
    T *r;
    const T *p;
    const T *w;
    const T *dinv;
    const uint8_t *owner;
    const CgScalars *scal;
    double *partial;  // [2][field][grid]
    int64_t n;
    int nfields;
};

struct CgFinishArgs {
    const double *partial;
    int64_t nblk;
    CgScalars *scal;
    double *hist;     // optional [field][hist_len] relative residual history
    int hist_len;
    int nfields;
};

// Per-field state of the reliable-update mixed solve (device resident).
struct RelState {
    double bb64;   // (b, b) of the FP64 system
    double rr64;   // (r, r) of the latest FP64 true residual
    double tol;    // FP64 relative residual target
    double delta;  // FP32 segment: reduce the residual by this factor, then replace it
    int done;      // 1: converged (or failed) -- no further segments
    int outer;     // residual replacements performed
    int last_iter; // iteration count at the latest replacement
};

// r32 = (float) r64, x32 = 0 (optionally p32 = 0), partials of (r32, dinv r32),
// (r32, r32) and (r64, r64) over owned points, for fields not done.
struct RelRestartArgs {
    const double *r64;
    float *r32;
    float *x32;
    float *p32;        // zeroed when non-null (first segment)
    const float *dinv32;
    const uint8_t *owner;
    const RelState *rel;
    double *partial;   // [3][field][grid]
    int64_t n;
    int nfields;
};

struct DotArgs {
    const double *a[4];
    const double *b[4];
    const uint8_t *owner;
    double *partial;  // [nd][field][grid]
    int64_t n;
    int nd;
    int nfields;
};

// Linear combinations of basis vectors (projection space, GMRES solution update):
// up to PB vectors per launch, coefficients by value.
constexpr int PB = 8;

// y = sum_i c_i V_i (mode 0), y += sum_i c_i V_i (mode 1), y = src + sum_i c_i V_i (mode 2)
struct CombArgs {
    double *y;
    const double *src;
    const double *V;
    int64_t ld;
    int l;
    int mode;
    double c[PB];
    int64_t n;
};

// ---------------------------------------------------------------- GMRES Arnoldi
// One pass over the data against up to ARN_MAXV basis vectors (unique-node product):
//   mode 0: partial dots (V_i, w), i < m, and (w, w);
//   mode 1: y = w - sum_i coef[i] V_i, partial dots (V_i, y) and (y, y);
//   mode 2: y = (w - sum_i coef[i] V_i) * scale[0].
// Partials are [m + 1][grid] (the squared norm last); coef and scale are device values
// (outputs of the previous reduction), so a whole Gram-Schmidt step needs no host sync.
constexpr int ARN_MAXV = 32;
struct ArnArgs {
    const double *V;       // basis vector i at V + i * ld
    int64_t ld;
    int m;                 // basis vectors in use, 1..ARN_MAXV
    const double *w;       // input
    double *y;             // output (modes 1, 2); may be w
    const uint8_t *owner;  // one copy per global id
    const double *coef;    // [m] (modes 1, 2)
    const double *scale;   // [1] (mode 2)
    double *partial;       // [m + 1][grid] (modes 0, 1)
    int64_t n;
};

// Delayed two-pass classical Gram-Schmidt step: the second pass for the previous
// basis vector u (orthogonalised once, one step ago) is made in the same passes as
// the first pass for the new vector w.  With Q = V_0..V_{j-1} (orthonormal):
//   dots:   a = Q^T u, (u, u), b = Q^T w, (u, w), (w, w)  -> partial rows
//           [a (j), (u,u), b (j), (u,w), (w,w)] of length 2 j + 3;
//   update: u <- (u - Q a) / rho                          (the final q_j)
//           w <- (w - Q c - delta u) / nu                  (the next u)
// with the coefficients in coef: [a (j), c (j), 1/rho, delta, 1/nu].
struct DcgsArgs {
    const double *V;       // basis vector i at V + i * ld
    int64_t ld;
    int j;                 // finished basis vectors, 0..ARN_MAXV - 1
    double *u;
    double *w;
    const uint8_t *owner;  // one copy per global id
    const double *coef;    // update pass
    double *partial;       // dots pass: [2 j + 3][grid]
    int64_t n;
};

// ---------------------------------------------------------------- two-level Schwarz
// out[e][c] = sum over element e's points p of phi[c][p] v[e][p] (owner[p] if owner).
struct CornerArgs {
    const double *v;
    const uint8_t *owner;  // nullptr: every point counts
    const double *phi;     // [8][lx^3] trilinear basis at the GLL points
    double *out;           // [nelv][8]
    int64_t nelv;
    int lx3;
};

// Fixed-count Jacobi-CG on the coarse system (Dirichlet vertices: identity rows), the
// matrix in ELL form (column-major [width][nv]; a row's entries in ascending column,
// padding value 0 with the row's own column).  The right-hand side is gathered from
// the per-element restriction sums: b[v] = sum over (e, c) at vertex v, ascending e
// (0 at Dirichlet vertices).
struct CoarseArgs {
    const int32_t *ci;
    const double *val;
    int width;
    const double *dinv;
    const double *part;    // [nelv * 8] restriction sums
    const int64_t *vptr;   // [nv + 1]
    const int32_t *vidx;   // e * 8 + c
    const uint8_t *vdir;   // [nv]
    double *x, *r, *z, *p0, *p1, *q;
    double *partial;       // [3][grid]: (r, z) in two slots, (p, q)
    int64_t nv;
};

}  // namespace sem
