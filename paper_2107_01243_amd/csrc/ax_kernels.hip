// ax_kernels.hip -- element-local kernels of the SEM Helmholtz operator for gfx950.
//
// Operator (Jansson et al., arXiv 2107.01243, Section 2, Eq. 9):
//   w_e = h1 D^T G_e D u_e + h2 B_e u_e  on every hexahedral element,
// with D the 1-D GLL derivative matrix applied along r, s and t, and G_e the six
// geometric factors (G11, G22, G33, G12, G13, G23) per point.
//
// Work decomposition ("pencil" layout).  One element is handled by lx*lx lanes.
// A lane with in-element index t = a + lx*b owns, at different stages,
//   t-pencil: the lx points (i = a, j = b, k = 0..lx-1)   (its home layout)
//   r-pencil: the lx points (i = 0..lx-1, j = a, k = b)
//   s-pencil: the lx points (i = a, j = 0..lx-1, k = b)
// In the home layout the lanes of an element read and write HBM at offsets
// t + lx^2 k: for each k one wave instruction covers lx^2 consecutive values, so
// every global access is fully coalesced.  Each 1-D derivative is a
// register-only product with D in its even-odd form (half the FMAs of the dense
// lx x lx product); its entries are wave-uniform (they travel in the
// kernel-argument segment and are read through scalar loads).  LDS is used only
// to transpose pencils; every LDS row has stride lx+1 so that the three pencil
// access patterns are free of bank conflicts.
//
// This file is compiled once per lx (-DSEM_LX=<lx>) so that the per-lx
// instantiations build in parallel; it exports plain host launchers.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "sem_kernels.h"
#include "sem_pencil.h"

#ifndef SEM_LX
#error "compile with -DSEM_LX=<lx>"
#endif
#define SEM_BOUNDS(NT) __launch_bounds__((NT))
#define SEM_BOUNDS2(NT, W) __launch_bounds__((NT)) __attribute__((amdgpu_waves_per_eu((W))))

namespace sem {

// ------------------------------------------------------------------ launch shape
// Elements per workgroup: fill whole wave64s where possible, keep the two LDS
// transpose buffers within 64 KB (up to 160 KB for a single large element), keep
// the register budget that the workgroup's size leaves each lane above what a lane
// needs, and aim at about 256 lanes per workgroup.
template <int LX, typename T>
struct Shape {
    static constexpr int NP = LX * LX;                       // lanes per element
    static constexpr int PAD = LX + 1;                       // LDS row stride
    static constexpr int ESZ = NP * PAD;                     // one LDS buffer, one element
    static constexpr int EBYTES = 2 * ESZ * (int)sizeof(T);  // LDS per element
    // 32-bit registers a lane needs, estimated: six geometric-factor rows and about
    // eight more pencil rows (u, its three derivatives, w, h1, h2 B, dinv), plus
    // scalars.  A SIMD gives 512 per lane to one wave, 512 / k to each of k waves, and
    // a workgroup of W waves puts ceil(W / 4) of them on one SIMD.
    static constexpr int REGS = 14 * LX * (int)sizeof(T) / 4 + 40;
    static constexpr int MAX_WAVES = 4 * (512 / REGS > 1 ? 512 / REGS : 1);
    static constexpr int pick()
    {
        int best = 1;
        double best_score = 1e9;
        for (int e = 1; e * NP <= 1024; ++e) {
            if (e > 1 && e * EBYTES > 64 * 1024) break;
            const int thr = e * NP;
            const int waves = (thr + 63) / 64;
            if (e > 1 && waves > MAX_WAVES) break;
            const double waste = double(waves * 64 - thr) / double(waves * 64);
            const double dist = (thr > 256 ? thr - 256 : 256 - thr) / 1024.0;
            const double score = waste + 0.25 * dist;
            if (score < best_score - 1e-12) { best_score = score; best = e; }
        }
        return best;
    }
#ifndef SEM_LEAN_LX
#define SEM_LEAN_LX 10
#endif
    // lx >= SEM_LEAN_LX: the register-lean kernels, one element per workgroup, with a
    // floor on the waves per SIMD the register allocation must leave room for (two
    // FP64 / four FP32 up to lx = 12, half that above)
    static constexpr bool LEAN = LX >= SEM_LEAN_LX;
    static constexpr int EPB = LEAN ? 1 : pick();
    static constexpr int NT = EPB * NP;
    static constexpr int MINW = !LEAN ? 1 : (sizeof(T) == 8 ? (LX <= 12 ? 2 : 1) : (LX <= 12 ? 4 : 2));
};

template <int LX, typename T>
struct Lds {
    T buf[2][Shape<LX, T>::EPB][Shape<LX, T>::ESZ];
};

// out = D in   (derivative along the pencil), even-odd form
template <int LX, typename T>
__device__ __forceinline__ void dmul(const DEo<LX, T> &D, const T (&in)[LX], T (&out)[LX])
{
    constexpr int H = LX / 2, N = LX - 1;
    T e[H > 0 ? H : 1], o[H > 0 ? H : 1];
#pragma unroll
    for (int l = 0; l < H; ++l) {
        e[l] = in[l] + in[N - l];
        o[l] = in[l] - in[N - l];
    }
#pragma unroll
    for (int m = 0; m < H; ++m) {
        T se = D.S[m * H] * e[0];
        T ao = D.A[m * H] * o[0];
#pragma unroll
        for (int l = 1; l < H; ++l) {
            se = fma(D.S[m * H + l], e[l], se);
            ao = fma(D.A[m * H + l], o[l], ao);
        }
        if constexpr (LX % 2 == 1) se = fma(D.cm[m], in[H], se);
        out[m] = ao + se;
        out[N - m] = ao - se;
    }
    if constexpr (LX % 2 == 1) {
        T c = T(0);
#pragma unroll
        for (int l = 0; l < H; ++l) c = fma(D.rm[l], o[l], c);
        out[H] = c;
    }
}

// out = D^T in   (transposed derivative along the pencil), even-odd form
template <int LX, typename T>
__device__ __forceinline__ void dtmul(const DEo<LX, T> &D, const T (&in)[LX], T (&out)[LX])
{
    constexpr int H = LX / 2, N = LX - 1;
    T e[H > 0 ? H : 1], o[H > 0 ? H : 1];
#pragma unroll
    for (int l = 0; l < H; ++l) {
        e[l] = in[l] + in[N - l];
        o[l] = in[l] - in[N - l];
    }
#pragma unroll
    for (int m = 0; m < H; ++m) {
        T se = D.A[m] * e[0];
        T ao = D.S[m] * o[0];
#pragma unroll
        for (int l = 1; l < H; ++l) {
            se = fma(D.A[l * H + m], e[l], se);
            ao = fma(D.S[l * H + m], o[l], ao);
        }
        if constexpr (LX % 2 == 1) se = fma(D.rm[m], in[H], se);
        out[m] = ao + se;
        out[N - m] = ao - se;
    }
    if constexpr (LX % 2 == 1) {
        T c = T(0);
#pragma unroll
        for (int l = 0; l < H; ++l) c = fma(D.cm[l], o[l], c);
        out[H] = c;
    }
}

// Where a kernel reads D from.  DArg: the kernel-argument copy (wave-uniform values
// the compiler keeps in scalar registers; right when they fit, as in FP32 and up to
// lx = 8 in FP64).  DMem: a copy in device memory read with scalar loads one row at a
// time where it is used; at lx = 12 in FP64 the 72 doubles of the even-odd D exceed the
// scalar register file, and holding them costs a spill to vector-register lanes plus
// two v_readlane per use (more VALU instructions than the FMAs themselves).
template <int LX, typename T>
struct DArg {
    const DEo<LX, T> &D;
    __device__ void mul(const T (&in)[LX], T (&out)[LX]) const { dmul<LX, T>(D, in, out); }
    __device__ void tmul(const T (&in)[LX], T (&out)[LX]) const { dtmul<LX, T>(D, in, out); }
};

// p + 0 with the 0 opaque to the optimiser: loads through the result are not merged
// with, or moved ahead of, loads through another such pointer; the address space of
// p is kept (an opaque pointer would turn global loads into flat ones).
template <typename T>
__device__ __forceinline__ const T *fresh(const T *p)
{
    int64_t z = 0;
    asm volatile("" : "+s"(z));
    return p + z;
}

template <int LX, typename T>
struct DMem {
    const DEo<LX, T> *Dg;
    __device__ void mul(const T (&in)[LX], T (&out)[LX]) const
    {
        constexpr int H = LX / 2, N = LX - 1;
        T e[H > 0 ? H : 1], o[H > 0 ? H : 1];
#pragma unroll
        for (int l = 0; l < H; ++l) {
            e[l] = in[l] + in[N - l];
            o[l] = in[l] - in[N - l];
        }
#pragma unroll
        for (int m = 0; m < H; ++m) {
            const DEo<LX, T> *R = fresh(Dg);  // this row's constants loaded here
            T se = R->S[m * H] * e[0];
            T ao = R->A[m * H] * o[0];
#pragma unroll
            for (int l = 1; l < H; ++l) {
                se = fma(R->S[m * H + l], e[l], se);
                ao = fma(R->A[m * H + l], o[l], ao);
            }
            if constexpr (LX % 2 == 1) se = fma(R->cm[m], in[H], se);
            out[m] = ao + se;
            out[N - m] = ao - se;
        }
        if constexpr (LX % 2 == 1) {
            const DEo<LX, T> *R = fresh(Dg);
            T c = T(0);
#pragma unroll
            for (int l = 0; l < H; ++l) c = fma(R->rm[l], o[l], c);
            out[H] = c;
        }
    }
    __device__ void tmul(const T (&in)[LX], T (&out)[LX]) const
    {
        constexpr int H = LX / 2, N = LX - 1;
        T e[H > 0 ? H : 1], o[H > 0 ? H : 1];
#pragma unroll
        for (int l = 0; l < H; ++l) {
            e[l] = in[l] + in[N - l];
            o[l] = in[l] - in[N - l];
        }
#pragma unroll
        for (int m = 0; m < H; ++m) {
            const DEo<LX, T> *R = fresh(Dg);
            T se = R->A[m] * e[0];
            T ao = R->S[m] * o[0];
#pragma unroll
            for (int l = 1; l < H; ++l) {
                se = fma(R->A[l * H + m], e[l], se);
                ao = fma(R->S[l * H + m], o[l], ao);
            }
            if constexpr (LX % 2 == 1) se = fma(R->rm[m], in[H], se);
            out[m] = ao + se;
            out[N - m] = ao - se;
        }
        if constexpr (LX % 2 == 1) {
            const DEo<LX, T> *R = fresh(Dg);
            T c = T(0);
#pragma unroll
            for (int l = 0; l < H; ++l) c = fma(R->cm[l], o[l], c);
            out[H] = c;
        }
    }
};

// Reference-space gradient of one field held as the lane's t-pencil `u`.
// Returns ur, us, ut as t-pencils.  Uses both LDS buffers; ends synchronised.
template <int LX, typename T>
__device__ __forceinline__ void grad(const DEo<LX, T> &D, const T (&u)[LX], T *s0, T *s1,
                                     int a, int b, T (&ur)[LX], T (&us)[LX], T (&ut)[LX])
{
    dmul<LX, T>(D, u, ut);
#pragma unroll
    for (int k = 0; k < LX; ++k) s0[lidx<LX>(a, b, k)] = u[k];
    esync<LX>();
    T v[LX], q[LX];
#pragma unroll
    for (int l = 0; l < LX; ++l) v[l] = s0[lidx<LX>(l, a, b)];   // r-pencil (j=a, k=b)
    dmul<LX, T>(D, v, q);
    T v2[LX], q2[LX];
#pragma unroll
    for (int l = 0; l < LX; ++l) v2[l] = s0[lidx<LX>(a, l, b)];  // s-pencil (i=a, k=b)
    dmul<LX, T>(D, v2, q2);
#pragma unroll
    for (int m = 0; m < LX; ++m) s1[lidx<LX>(m, a, b)] = q[m];
    esync<LX>();
#pragma unroll
    for (int m = 0; m < LX; ++m) s0[lidx<LX>(a, m, b)] = q2[m];
    esync<LX>();
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        ur[k] = s1[lidx<LX>(a, b, k)];
        us[k] = s0[lidx<LX>(a, b, k)];
    }
    esync<LX>();
}

// acc = D_r^T wr + D_s^T ws + D_t^T wt for t-pencils wr, ws, wt.  Ends synchronised.
template <int LX, typename T>
__device__ __forceinline__ void div(const DEo<LX, T> &D, const T (&wr)[LX], const T (&ws)[LX],
                                    const T (&wt)[LX], T *s0, T *s1, int a, int b, T (&acc)[LX])
{
    dtmul<LX, T>(D, wt, acc);
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        s0[lidx<LX>(a, b, k)] = wr[k];
        s1[lidx<LX>(a, b, k)] = ws[k];
    }
    esync<LX>();
    T v[LX], q[LX], v2[LX], q2[LX];
#pragma unroll
    for (int l = 0; l < LX; ++l) v[l] = s0[lidx<LX>(l, a, b)];
#pragma unroll
    for (int l = 0; l < LX; ++l) v2[l] = s1[lidx<LX>(a, l, b)];
    dtmul<LX, T>(D, v, q);
    dtmul<LX, T>(D, v2, q2);
    esync<LX>();
#pragma unroll
    for (int m = 0; m < LX; ++m) {
        s0[lidx<LX>(m, a, b)] = q[m];
        s1[lidx<LX>(a, m, b)] = q2[m];
    }
    esync<LX>();
#pragma unroll
    for (int k = 0; k < LX; ++k) acc[k] += s0[lidx<LX>(a, b, k)] + s1[lidx<LX>(a, b, k)];
    esync<LX>();
}

// A t-pencil in HBM: values p[k * lx^2], k = 0..lx-1 (p = element base + t).
template <int LX, typename T>
__device__ __forceinline__ void load_row(T (&r)[LX], const T *__restrict__ p, bool act)
{
    if (act) {
#pragma unroll
        for (int k = 0; k < LX; ++k) r[k] = p[k * LX * LX];
    } else {
#pragma unroll
        for (int k = 0; k < LX; ++k) r[k] = T(0);
    }
}

// Geometric-factor pencils are streamed once per application and the six planes
// (6 words per point) never fit the 256 MB last-level cache at production sizes, so
// they are read with non-temporal loads: this keeps the cache for the vectors
// (u, w, the Krylov vectors) that are reused between launches.
template <int LX, typename T>
__device__ __forceinline__ void load_g(T (&r)[LX], const T *__restrict__ p, bool act)
{
    if (!act) {
#pragma unroll
        for (int k = 0; k < LX; ++k) r[k] = T(0);
        return;
    }
#pragma unroll
    for (int k = 0; k < LX; ++k) r[k] = __builtin_nontemporal_load(p + k * LX * LX);
}

template <int LX, typename T>
__device__ __forceinline__ void store_row(T *__restrict__ p, const T (&r)[LX], bool act)
{
    if (act) {
#pragma unroll
        for (int k = 0; k < LX; ++k) p[k * LX * LX] = r[k];
    }
}

// Helmholtz coefficients of one pencil.  GEN = false is the Poisson-type case
// (h1 a scalar, no mass term): nothing per point is held, which keeps the
// register footprint low; GEN = true handles h1 / h2 fields and the mass term.
template <int LX, typename T, bool GEN>
struct RowCoef {
    T h1[GEN ? LX : 1];
    T h2b[GEN ? LX : 1];  // h2 * B
    bool mass = false;
};

template <int LX, typename T, bool GEN, typename Args>
__device__ __forceinline__ void load_coef(RowCoef<LX, T, GEN> &c, const Args &A, int64_t row, bool act)
{
    if constexpr (GEN) {
        if (A.h1) load_row<LX, T>(c.h1, A.h1 + row, act);
        else {
#pragma unroll
            for (int i = 0; i < LX; ++i) c.h1[i] = A.h1s;
        }
        c.mass = A.h2 != nullptr || A.h2s != T(0);
        if (c.mass) {
            load_row<LX, T>(c.h2b, A.B + row, act);
            if (A.h2) {
                T h2[LX];
                load_row<LX, T>(h2, A.h2 + row, act);
#pragma unroll
                for (int i = 0; i < LX; ++i) c.h2b[i] *= h2[i];
            } else {
#pragma unroll
                for (int i = 0; i < LX; ++i) c.h2b[i] *= A.h2s;
            }
        }
    }
}

// Apply h1 * G at every point of the pencil (in place: ur,us,ut -> wr,ws,wt).
template <int LX, typename T, bool GEN>
__device__ __forceinline__ void apply_G(const T (&g)[6][LX], const RowCoef<LX, T, GEN> &c, T h1s,
                                        T (&ur)[LX], T (&us)[LX], T (&ut)[LX])
{
#pragma unroll
    for (int i = 0; i < LX; ++i) {
        const T h = GEN ? c.h1[i] : h1s;
        const T r = ur[i], s = us[i], t = ut[i];
        ur[i] = h * (g[0][i] * r + g[3][i] * s + g[4][i] * t);
        us[i] = h * (g[3][i] * r + g[1][i] * s + g[5][i] * t);
        ut[i] = h * (g[4][i] * r + g[5][i] * s + g[2][i] * t);
    }
}

// w += h2 B u (general case only).
template <int LX, typename T, bool GEN>
__device__ __forceinline__ void add_mass(const RowCoef<LX, T, GEN> &c, const T (&u)[LX], T (&w)[LX])
{
    if constexpr (GEN) {
        if (c.mass) {
#pragma unroll
            for (int i = 0; i < LX; ++i) w[i] = fma(c.h2b[i], u[i], w[i]);
        }
    }
}

// ------------------------------------------------------------------ w = A_L u
// NF fields share one read of G (and B, h1, h2).
template <int LX, typename T, int NF, bool GEN>
__global__ SEM_BOUNDS2((Shape<LX, T>::NT), (Shape<LX, T>::MINW)) void k_ax_helm(AxArgs<T> A, DEo<LX, T> D)
{
    using S = Shape<LX, T>;
    __shared__ Lds<LX, T> lds;
    const int tid = threadIdx.x;
    const int slot = tid / S::NP;
    const int t = tid - slot * S::NP;
    const int a = t % LX, b = t / LX;
    const int64_t e = (int64_t)blockIdx.x * S::EPB + slot;
    const bool act = e < A.nelv;
    const int64_t row = e * (int64_t)(LX * LX * LX) + t;  // base of this lane's t-pencil
    T *s0 = lds.buf[0][slot], *s1 = lds.buf[1][slot];

    T g[6][LX];
#pragma unroll
    for (int f = 0; f < 6; ++f) load_g<LX, T>(g[f], A.G + f * A.n + row, act);
    RowCoef<LX, T, GEN> c;
    load_coef<LX, T, GEN>(c, A, row, act);
    // the next field's row is loaded while the current one is processed
    T un[LX];
    load_row<LX, T>(un, A.u + row, act);
#pragma unroll 1
    for (int f = 0; f < NF; ++f) {
        T u[LX];
#pragma unroll
        for (int k = 0; k < LX; ++k) u[k] = un[k];
        if (f + 1 < NF) load_row<LX, T>(un, A.u + (f + 1) * A.n + row, act);
        T ur[LX], us[LX], ut[LX];
        grad<LX, T>(D, u, s0, s1, a, b, ur, us, ut);
        apply_G<LX, T, GEN>(g, c, A.h1s, ur, us, ut);
        T w[LX];
        div<LX, T>(D, ur, us, ut, s0, s1, a, b, w);
        add_mass<LX, T, GEN>(c, u, w);
        store_row<LX, T>(A.w + f * A.n + row, w, act);
    }
}

// ------------------------------------------------------------------ fused CG matvec
// Two-reduction CG (CG1 = false): p = dinv r + beta p (stored), w = A_L p.
// Single-reduction CG (CG1 = true, Chronopoulos-Gear): u = dinv r (not stored),
// w = A_L u.  Either way the workgroup's partial sum of v . w (v = p or u) is written:
// v^T A v by the unassembled identity of Eq. 10.
template <int LX, typename T, int NF, bool GEN, bool CG1>
__global__ SEM_BOUNDS2((Shape<LX, T>::NT), (Shape<LX, T>::MINW)) void k_cg_matvec(CgMatvecArgs<T> A, DEo<LX, T> D)
{
    using S = Shape<LX, T>;
    static_assert(S::NT >= 64, "the partial-sum reduction needs a full first wave");
    __shared__ Lds<LX, T> lds;
    __shared__ double red[NF][S::NT];
    const int tid = threadIdx.x;
    const int slot = tid / S::NP;
    const int t = tid - slot * S::NP;
    const int a = t % LX, b = t / LX;
    const int64_t e = (int64_t)blockIdx.x * S::EPB + slot;
    const bool act = e < A.nelv;
    const int64_t row = e * (int64_t)(LX * LX * LX) + t;  // base of this lane's t-pencil
    T *s0 = lds.buf[0][slot], *s1 = lds.buf[1][slot];
    // a launch queued after every field has stopped (between host polls) reads
    // nothing: the same flags for every lane, so the exit is uniform
    bool live = false;
#pragma unroll
    for (int f = 0; f < NF; ++f) live = live || !A.scal[f].stop;
    if (!live) return;

    T g[6][LX];
#pragma unroll
    for (int f = 0; f < 6; ++f) load_g<LX, T>(g[f], A.G + f * A.n + row, act);
    RowCoef<LX, T, GEN> c;
    load_coef<LX, T, GEN>(c, A, row, act);
    T dinv[LX];
    // the CG vectors too are streamed with non-temporal hints: one iteration moves
    // several times the last-level cache, and keeping them out of it leaves room for
    // the gather-scatter's index lists and w, which the next kernel reads (measured:
    // 0.763 -> 0.687 s per FP64 solve at 32^3 x lx=8)
    load_g<LX, T>(dinv, A.dinv + row, act);

    double part[NF];
#pragma unroll 1
    for (int f = 0; f < NF; ++f) {
        part[f] = 0.0;
        const CgScalars *sc = A.scal + f;
        if (sc->stop) continue;  // uniform: every lane reads the same flag
        T r[LX], p[LX];
        load_g<LX, T>(r, A.r + f * A.n + row, act);
        if constexpr (CG1) {
#pragma unroll
            for (int i = 0; i < LX; ++i) p[i] = dinv[i] * r[i];
        } else {
            const T beta = (T)sc->beta;
            load_g<LX, T>(p, A.p + f * A.n + row, act);
#pragma unroll
            for (int i = 0; i < LX; ++i) p[i] = fma(beta, p[i], dinv[i] * r[i]);
            if (act) {
#pragma unroll
                for (int k = 0; k < LX; ++k) __builtin_nontemporal_store(p[k], A.p + f * A.n + row + k * LX * LX);
            }
        }
        T ur[LX], us[LX], ut[LX];
        grad<LX, T>(D, p, s0, s1, a, b, ur, us, ut);
        apply_G<LX, T, GEN>(g, c, A.h1s, ur, us, ut);
        T w[LX];
        div<LX, T>(D, ur, us, ut, s0, s1, a, b, w);
        add_mass<LX, T, GEN>(c, p, w);
        store_row<LX, T>(A.w + f * A.n + row, w, act);
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < LX; ++i) s += (double)p[i] * (double)w[i];
        part[f] = s;
    }
    // workgroup reduction in a fixed order (deterministic): the first wave (always
    // full, NT >= 64) sums strided slices, then a butterfly inside that wave.
#pragma unroll
    for (int q = 0; q < NF; ++q) red[q][tid] = part[q];
    __syncthreads();
    if (tid < 64) {
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            double v = 0.0;
            for (int k = tid; k < S::NT; k += 64) v += red[q][k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (tid == 0) A.partial[(int64_t)q * gridDim.x + blockIdx.x] = v;
        }
    }
}

// ------------------------------------------------------------------ register-lean variants
// At large lx a lane's six G pencils (6 lx words) held next to a field's pencils
// exhaust the register file (one wave per SIMD at lx = 12 in FP64), which leaves a
// compute unit one workgroup that alternates between loading and computing.  The
// lean kernels (lx >= SEM_LEAN_LX) hold nothing across the phases of a field: G,
// h1, B and dinv are read in chunks of ceil(lx/2) points where they are used, the r
// and s derivatives run one after the other, and one element is one workgroup.  The
// registers saved let two (FP64) or four (FP32) waves share a SIMD, so the loads of
// one workgroup overlap the arithmetic of others.  With three fields the chunks are
// read again for every field with ordinary (cached) loads: the first field brings
// them from HBM, the other two find them in the cache.

template <bool NTL, typename T>
__device__ __forceinline__ T ldx(const T *p)
{
    if constexpr (NTL) return __builtin_nontemporal_load(p);
    else return *p;
}

// Reference-space gradient, the r and s derivatives sequenced to keep one pencil pair
// live at a time.  Same LDS protocol as grad (both buffers, ends synchronised).
template <int LX, typename T, typename DS>
__device__ __forceinline__ void grad_lean(const DS &D, const T (&u)[LX], T *s0, T *s1, int a, int b,
                                          T (&ur)[LX], T (&us)[LX], T (&ut)[LX])
{
#pragma unroll
    for (int k = 0; k < LX; ++k) s0[lidx<LX>(a, b, k)] = u[k];
    D.mul(u, ut);
    esync<LX>();
    {
        T v[LX], q[LX];
#pragma unroll
        for (int l = 0; l < LX; ++l) v[l] = s0[lidx<LX>(l, a, b)];   // r-pencil (j=a, k=b)
        D.mul(v, q);
#pragma unroll
        for (int m = 0; m < LX; ++m) s1[lidx<LX>(m, a, b)] = q[m];
    }
    __builtin_amdgcn_sched_barrier(0);
    {
        T v[LX], q[LX];
#pragma unroll
        for (int l = 0; l < LX; ++l) v[l] = s0[lidx<LX>(a, l, b)];   // s-pencil (i=a, k=b)
        D.mul(v, q);
        esync<LX>();
#pragma unroll
        for (int m = 0; m < LX; ++m) s0[lidx<LX>(a, m, b)] = q[m];
    }
    esync<LX>();
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        ur[k] = s1[lidx<LX>(a, b, k)];
        us[k] = s0[lidx<LX>(a, b, k)];
    }
    esync<LX>();
}

// acc = D_r^T wr + D_s^T ws + D_t^T wt, sequenced as grad_lean.  Ends synchronised.
template <int LX, typename T, typename DS>
__device__ __forceinline__ void div_lean(const DS &D, const T (&wr)[LX], const T (&ws)[LX],
                                         const T (&wt)[LX], T *s0, T *s1, int a, int b, T (&acc)[LX])
{
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        s0[lidx<LX>(a, b, k)] = wr[k];
        s1[lidx<LX>(a, b, k)] = ws[k];
    }
    D.tmul(wt, acc);
    esync<LX>();
    T q[LX], q2[LX];
    {
        T v[LX];
#pragma unroll
        for (int l = 0; l < LX; ++l) v[l] = s0[lidx<LX>(l, a, b)];
        D.tmul(v, q);
    }
    __builtin_amdgcn_sched_barrier(0);
    {
        T v[LX];
#pragma unroll
        for (int l = 0; l < LX; ++l) v[l] = s1[lidx<LX>(a, l, b)];
        D.tmul(v, q2);
    }
    esync<LX>();
#pragma unroll
    for (int m = 0; m < LX; ++m) {
        s0[lidx<LX>(m, a, b)] = q[m];
        s1[lidx<LX>(a, m, b)] = q2[m];
    }
    esync<LX>();
#pragma unroll
    for (int k = 0; k < LX; ++k) acc[k] += s0[lidx<LX>(a, b, k)] + s1[lidx<LX>(a, b, k)];
    esync<LX>();
}

// Four-buffer forms (A, B, C, E: one element each).  The transposes of a field pass
// go through buffers that no lane can still be reading, which takes four workgroup
// barriers per pass instead of eight: grad writes u to A, the r and s derivatives to B
// and C; div writes w_r to A and w_s to E, their transposed derivatives to B and C.
// Every buffer written after a barrier was last read before that barrier, including
// across consecutive passes (the next pass writes B and C only after its first
// barrier, which every lane reaches after its reads of B and C).
template <int LX, typename T, typename DS>
__device__ __forceinline__ void grad4(const DS &D, const T (&u)[LX], T *A, T *B, T *C, int a, int b,
                                      T (&ur)[LX], T (&us)[LX], T (&ut)[LX])
{
#pragma unroll
    for (int k = 0; k < LX; ++k) A[lidx<LX>(a, b, k)] = u[k];
    D.mul(u, ut);
    esync<LX>();
    {
        T v[LX], q[LX];
#pragma unroll
        for (int l = 0; l < LX; ++l) v[l] = A[lidx<LX>(l, a, b)];   // r-pencil (j=a, k=b)
        D.mul(v, q);
#pragma unroll
        for (int m = 0; m < LX; ++m) B[lidx<LX>(m, a, b)] = q[m];
    }
    __builtin_amdgcn_sched_barrier(0);
    {
        T v[LX], q[LX];
#pragma unroll
        for (int l = 0; l < LX; ++l) v[l] = A[lidx<LX>(a, l, b)];   // s-pencil (i=a, k=b)
        D.mul(v, q);
#pragma unroll
        for (int m = 0; m < LX; ++m) C[lidx<LX>(a, m, b)] = q[m];
    }
    esync<LX>();
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        ur[k] = B[lidx<LX>(a, b, k)];
        us[k] = C[lidx<LX>(a, b, k)];
    }
}

template <int LX, typename T, typename DS>
__device__ __forceinline__ void div4(const DS &D, const T (&wr)[LX], const T (&ws)[LX], const T (&wt)[LX], T *A,
                                     T *B, T *C, T *E, int a, int b, T (&acc)[LX])
{
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        A[lidx<LX>(a, b, k)] = wr[k];
        E[lidx<LX>(a, b, k)] = ws[k];
    }
    D.tmul(wt, acc);
    esync<LX>();
    {
        T v[LX], q[LX];
#pragma unroll
        for (int l = 0; l < LX; ++l) v[l] = A[lidx<LX>(l, a, b)];
        D.tmul(v, q);
#pragma unroll
        for (int m = 0; m < LX; ++m) B[lidx<LX>(m, a, b)] = q[m];
    }
    __builtin_amdgcn_sched_barrier(0);
    {
        T v[LX], q[LX];
#pragma unroll
        for (int l = 0; l < LX; ++l) v[l] = E[lidx<LX>(a, l, b)];
        D.tmul(v, q);
#pragma unroll
        for (int m = 0; m < LX; ++m) C[lidx<LX>(a, m, b)] = q[m];
    }
    esync<LX>();
#pragma unroll
    for (int k = 0; k < LX; ++k) acc[k] += B[lidx<LX>(a, b, k)] + C[lidx<LX>(a, b, k)];
}



// Pencil loads and stores of the lean kernels.  eb is the element's base in one plane
// (wave-uniform: one element per workgroup, every workgroup holds an element), t the
// lane's column; the address is a uniform base plus a small per-lane offset, which
// keeps per-lane 64-bit addresses out of the registers.
template <int LX, typename T, bool NTL>
__device__ __forceinline__ void lpencil(T (&r)[LX], const T *__restrict__ eb, unsigned t)
{
#pragma unroll
    for (int k = 0; k < LX; ++k) r[k] = ldx<NTL>(eb + k * LX * LX + t);
}

template <int LX, typename T>
__device__ __forceinline__ void spencil(T *__restrict__ eb, unsigned t, const T (&r)[LX])
{
#pragma unroll
    for (int k = 0; k < LX; ++k) eb[k * LX * LX + t] = r[k];
}

// Coefficient forms of the lean kernels, fixed at compile time so that no pointer test
// or branch sits between the loads and the arithmetic that uses them.
enum LeanKind : int {
    KPOISSON = 0,  // h1 scalar, no mass term
    KHELM = 1,     // h1 scalar, h2 scalar != 0 (velocity Helmholtz)
    KH1F = 2,      // h1 field, h2 scalar != 0
    KGEN = 3       // anything else: h1 and h2 scalars or fields, tested at run time
};

template <typename T>
__device__ __forceinline__ const T *ebase(const T *p, int64_t off) { return p ? p + off : nullptr; }


// (ur, us, ut) <- h1 G (ur, us, ut) with G (and the h1 field) read in chunks of C
// points, Ge = G + element base (plane stride n).  NTL: non-temporal loads (G used by
// one field only).  The chunks are not requested before the gradient is done.
template <int LX, typename T, int KIND, bool NTL>
__device__ __forceinline__ void apply_G_lean(const T *__restrict__ Ge, const T *__restrict__ h1e, T h1s, int64_t n,
                                             unsigned t, T (&ur)[LX], T (&us)[LX], T (&ut)[LX])
{
    constexpr int C = sizeof(T) == 8 ? (LX + 2) / 3 : (LX + 1) / 2;
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k0 = 0; k0 < LX; k0 += C) {
        T g[6][C], h[C];
#pragma unroll
        for (int kk = 0; kk < C; ++kk) {
            if (k0 + kk < LX) {
                const unsigned o = (k0 + kk) * (LX * LX) + t;
#pragma unroll
                for (int f = 0; f < 6; ++f) g[f][kk] = ldx<NTL>(Ge + f * n + o);
                if constexpr (KIND == KH1F) h[kk] = h1e[o];
                else if constexpr (KIND == KGEN) h[kk] = h1e ? h1e[o] : h1s;
                else h[kk] = h1s;
            }
        }
#pragma unroll
        for (int kk = 0; kk < C; ++kk) {
            const int k = k0 + kk;
            if (k < LX) {
                const T r = ur[k], s = us[k], q = ut[k];
                ur[k] = h[kk] * (g[0][kk] * r + g[3][kk] * s + g[4][kk] * q);
                us[k] = h[kk] * (g[3][kk] * r + g[1][kk] * s + g[5][kk] * q);
                ut[k] = h[kk] * (g[4][kk] * r + g[5][kk] * s + g[2][kk] * q);
            }
        }
    }
}

// h2 B at the lane's points (zero for KPOISSON), B and the h2 field read here.
template <int LX, typename T, int KIND>
__device__ __forceinline__ T mass_coef(const T *__restrict__ Be, const T *__restrict__ h2e, T h2s, unsigned o)
{
    if constexpr (KIND == KGEN) return h2e ? h2e[o] * Be[o] : h2s * Be[o];
    else return h2s * Be[o];
}

// w += h2 B u for u held in registers.
template <int LX, typename T, int KIND>
__device__ __forceinline__ void add_mass_lean(const T *__restrict__ Be, const T *__restrict__ h2e, T h2s, unsigned t,
                                              const T (&u)[LX], T (&w)[LX])
{
    if constexpr (KIND != KPOISSON) {
        if (KIND != KGEN || h2e || h2s != T(0)) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < LX; ++k) w[k] = fma(mass_coef<LX, T, KIND>(Be, h2e, h2s, k * (LX * LX) + t), u[k], w[k]);
        }
    }
}

// w += h2 B u with u reloaded from ue (read moments before, so served by the cache).
template <int LX, typename T, int KIND>
__device__ __forceinline__ void add_mass_reload(const T *__restrict__ Be, const T *__restrict__ h2e, T h2s, unsigned t,
                                                const T *__restrict__ ue, T (&w)[LX])
{
    if constexpr (KIND != KPOISSON) {
        if (KIND != KGEN || h2e || h2s != T(0)) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < LX; ++k) {
                const unsigned o = k * (LX * LX) + t;
                w[k] = fma(mass_coef<LX, T, KIND>(Be, h2e, h2s, o), ue[o], w[k]);
            }
        }
    }
}

// (ur, us, ut) <- h1 G (ur, us, ut) from G pencils held in registers.
template <int LX, typename T, int KIND>
__device__ __forceinline__ void apply_G_regs(const T (&g)[6][LX], const T *__restrict__ h1e, T h1s, unsigned t,
                                             T (&ur)[LX], T (&us)[LX], T (&ut)[LX])
{
#pragma unroll
    for (int k = 0; k < LX; ++k) {
        T h;
        if constexpr (KIND == KH1F) h = h1e[k * (LX * LX) + t];
        else if constexpr (KIND == KGEN) h = h1e ? h1e[k * (LX * LX) + t] : h1s;
        else h = h1s;
        const T r = ur[k], s = us[k], q = ut[k];
        ur[k] = h * (g[0][k] * r + g[3][k] * s + g[4][k] * q);
        us[k] = h * (g[3][k] * r + g[1][k] * s + g[5][k] * q);
        ut[k] = h * (g[4][k] * r + g[5][k] * s + g[2][k] * q);
    }
}

// The gradient and divergence halves of a field pass on NB LDS buffers.
template <int LX, typename T, int NB, typename DS>
__device__ __forceinline__ void grad_nb(const DS &D, const T (&u)[LX], T (*buf)[Shape<LX, T>::ESZ], int a, int b,
                                        T (&ur)[LX], T (&us)[LX], T (&ut)[LX])
{
    if constexpr (NB == 4) grad4<LX, T>(D, u, buf[0], buf[1], buf[2], a, b, ur, us, ut);
    else grad_lean<LX, T>(D, u, buf[0], buf[1], a, b, ur, us, ut);
}

template <int LX, typename T, int NB, typename DS>
__device__ __forceinline__ void div_nb(const DS &D, const T (&wr)[LX], const T (&ws)[LX], const T (&wt)[LX],
                                       T (*buf)[Shape<LX, T>::ESZ], int a, int b, T (&w)[LX])
{
    if constexpr (NB == 4) div4<LX, T>(D, wr, ws, wt, buf[0], buf[1], buf[2], buf[3], a, b, w);
    else div_lean<LX, T>(D, wr, ws, wt, buf[0], buf[1], a, b, w);
}

// Launch configuration of the lean kernels, per precision, field count and kernel
// (CG: the fused CG matvec, which also keeps p for its dot product).
//  * HOLD: with three fields sharing one G, hold G's six pencils in registers (loaded
//    once, non-temporal) instead of reading them in chunks for every field; pays for the
//    FP32 operator up to lx = 12 (in FP64 the held pencils would cost the second wave
//    per SIMD; the FP32 CG matvec, which also holds p, is faster reading chunks at
//    three waves per SIMD: 4.6 -> 3.7 ms at 48^3 x lx = 12).
//  * NB: LDS element buffers, 4 (grad4 / div4: four barriers per field pass) or 2
//    (grad_lean / div_lean: eight); in FP64 four would halve the workgroups a compute
//    unit holds.
//  * MINW: waves per SIMD the register allocation is held to.
#ifndef SEM_AX_HOLD
#define SEM_AX_HOLD 1
#endif
#ifndef SEM_CG_HOLD
#define SEM_CG_HOLD 0
#endif
#ifndef SEM_AX_NB32
#define SEM_AX_NB32 4
#endif
#ifndef SEM_CG_NB32
#define SEM_CG_NB32 4
#endif
#ifndef SEM_CG_W32H
#define SEM_CG_W32H 3
#endif
template <int LX, typename T, int NF, bool CG>
struct LeanCfg {
    static constexpr bool F32 = sizeof(T) == 4;
    static constexpr bool HOLD = NF > 1 && F32 && LX <= 12 && (CG ? SEM_CG_HOLD : SEM_AX_HOLD);
    static constexpr int NB = F32 ? (CG ? SEM_CG_NB32 : SEM_AX_NB32) : 2;
    static constexpr int MINW = HOLD ? (CG ? SEM_CG_W32H : 3)
                                     : ((!CG && NF > 1 && !F32 && LX <= 12) ? 3 : Shape<LX, T>::MINW);
};

template <int LX, typename T, int NB>
struct LeanBufs {
    T buf[NB][Shape<LX, T>::ESZ];
};

// One element per workgroup; the grid holds exactly nelv workgroups.
template <int LX, typename T, int NF, int KIND, typename DS>
__device__ __forceinline__ void ax_lean_body(const DS &D, const AxArgs<T> &A)
{
    using S = Shape<LX, T>;
    using C = LeanCfg<LX, T, NF, false>;
    constexpr bool HOLD = C::HOLD;
    constexpr int NB = C::NB;
    static_assert(S::EPB == 1, "one element per workgroup");
    __shared__ LeanBufs<LX, T, NB> lds;
    const unsigned t = threadIdx.x;
    const int a = t % LX, b = t / LX;
    const int64_t e0 = (int64_t)blockIdx.x * (LX * LX * LX);
    const T *Ge = A.G + e0;
    const T *h1e = KIND >= KH1F ? ebase(A.h1, e0) : nullptr;
    T g[HOLD ? 6 : 1][LX];
    if constexpr (HOLD) {
#pragma unroll
        for (int q = 0; q < 6; ++q) lpencil<LX, T, true>(g[q], Ge + q * A.n, t);
    }
#pragma unroll 1
    for (int f = 0; f < NF; ++f) {
        const int64_t fe = f * A.n + e0;
        T w[LX];
        {
            T ur[LX], us[LX], ut[LX];
            {
                T u[LX];
                lpencil<LX, T, false>(u, A.u + fe, t);
                grad_nb<LX, T, NB>(D, u, lds.buf, a, b, ur, us, ut);
            }
            if constexpr (HOLD) apply_G_regs<LX, T, KIND>(g, h1e ? fresh(h1e) : h1e, A.h1s, t, ur, us, ut);
            else apply_G_lean<LX, T, KIND, NF == 1>(fresh(Ge), h1e ? fresh(h1e) : h1e, A.h1s, A.n, t, ur, us, ut);
            div_nb<LX, T, NB>(D, ur, us, ut, lds.buf, a, b, w);
        }
        add_mass_reload<LX, T, KIND>(A.B + e0, KIND == KGEN ? ebase(A.h2, e0) : nullptr, A.h2s, t, A.u + fe, w);
        spencil<LX, T>(A.w + fe, t, w);
    }
}

// DMem in FP64 (the even-odd D does not fit the scalar registers), DArg in FP32.
template <int LX, typename T, int NF, int KIND>
__global__ SEM_BOUNDS2((Shape<LX, T>::NT), (LeanCfg<LX, T, NF, false>::MINW)) void k_ax_helm_lean(
    AxArgs<T> A, DEo<LX, T> D, const DEo<LX, T> *__restrict__ Dg)
{
    if constexpr (sizeof(T) == 8) ax_lean_body<LX, T, NF, KIND>(DMem<LX, T>{Dg}, A);
    else ax_lean_body<LX, T, NF, KIND>(DArg<LX, T>{D}, A);
}

template <int LX, typename T, int NF, int KIND, bool CG1, typename DS>
__device__ __forceinline__ void cg_lean_body(const DS &D, const CgMatvecArgs<T> &A)
{
    using S = Shape<LX, T>;
    using C = LeanCfg<LX, T, NF, true>;
    constexpr bool HOLD = C::HOLD;
    static_assert(S::EPB == 1 && S::NT >= 64, "one element per workgroup of at least one wave");
    constexpr int NB = C::NB;
    __shared__ LeanBufs<LX, T, NB> lds;
    __shared__ double red[NF][S::NT];
    const unsigned t = threadIdx.x;
    const int a = t % LX, b = t / LX;
    const int64_t e0 = (int64_t)blockIdx.x * (LX * LX * LX);
    bool live = false;
#pragma unroll
    for (int f = 0; f < NF; ++f) live = live || !A.scal[f].stop;
    if (!live) return;
    const T *Ge = A.G + e0;
    const T *h1e = KIND >= KH1F ? ebase(A.h1, e0) : nullptr;
    T g[HOLD ? 6 : 1][LX];
    if constexpr (HOLD) {
#pragma unroll
        for (int q = 0; q < 6; ++q) lpencil<LX, T, true>(g[q], Ge + q * A.n, t);
    }
    double part[NF];
#pragma unroll 1
    for (int f = 0; f < NF; ++f) {
        part[f] = 0.0;
        const CgScalars *sc = A.scal + f;
        if (sc->stop) continue;  // uniform
        const int64_t fe = f * A.n + e0;
        T p[LX];
        {
            T r[LX], dv[LX];
            lpencil<LX, T, true>(r, A.r + fe, t);
            lpencil<LX, T, NF == 1>(dv, A.dinv + e0, t);
            if constexpr (CG1) {
#pragma unroll
                for (int i = 0; i < LX; ++i) p[i] = dv[i] * r[i];
            } else {
                const T beta = (T)sc->beta;
                lpencil<LX, T, true>(p, A.p + fe, t);
#pragma unroll
                for (int i = 0; i < LX; ++i) p[i] = fma(beta, p[i], dv[i] * r[i]);
#pragma unroll
                for (int k = 0; k < LX; ++k) __builtin_nontemporal_store(p[k], A.p + fe + k * LX * LX + t);
            }
        }
        T w[LX];
        {
            T ur[LX], us[LX], ut[LX];
            grad_nb<LX, T, NB>(D, p, lds.buf, a, b, ur, us, ut);
            if constexpr (HOLD) apply_G_regs<LX, T, KIND>(g, h1e ? fresh(h1e) : h1e, A.h1s, t, ur, us, ut);
            else apply_G_lean<LX, T, KIND, NF == 1>(fresh(Ge), h1e ? fresh(h1e) : h1e, A.h1s, A.n, t, ur, us, ut);
            div_nb<LX, T, NB>(D, ur, us, ut, lds.buf, a, b, w);
        }
        add_mass_lean<LX, T, KIND>(A.B + e0, KIND == KGEN ? ebase(A.h2, e0) : nullptr, A.h2s, t, p, w);
        spencil<LX, T>(A.w + fe, t, w);
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < LX; ++i) sum += (double)p[i] * (double)w[i];
        part[f] = sum;
    }
#pragma unroll
    for (int q = 0; q < NF; ++q) red[q][t] = part[q];
    __syncthreads();
    if (t < 64) {
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            double v = 0.0;
            for (unsigned k = t; k < S::NT; k += 64) v += red[q][k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (t == 0) A.partial[(int64_t)q * gridDim.x + blockIdx.x] = v;
        }
    }
}

template <int LX, typename T, int NF, int KIND, bool CG1>
__global__ SEM_BOUNDS2((Shape<LX, T>::NT), (LeanCfg<LX, T, NF, true>::MINW)) void k_cg_matvec_lean(
    CgMatvecArgs<T> A, DEo<LX, T> D, const DEo<LX, T> *__restrict__ Dg)
{
    if constexpr (sizeof(T) == 8) cg_lean_body<LX, T, NF, KIND, CG1>(DMem<LX, T>{Dg}, A);
    else cg_lean_body<LX, T, NF, KIND, CG1>(DArg<LX, T>{D}, A);
}

// g = (D v)^T G (D u) per point, lean form: G (D u) is formed first (G read in
// chunks), then the gradient of v is taken and contracted with it.
template <int LX, typename T, typename DS>
__device__ __forceinline__ void adj_lean_body(const DS &D, const AdjArgs<T> &A)
{
    using S = Shape<LX, T>;
    static_assert(S::EPB == 1, "one element per workgroup");
    __shared__ Lds<LX, T> lds;
    const unsigned t = threadIdx.x;
    const int a = t % LX, b = t / LX;
    const int64_t e0 = (int64_t)blockIdx.x * (LX * LX * LX);
    T *s0 = lds.buf[0][0], *s1 = lds.buf[1][0];
    T wr[LX], ws[LX], wt[LX];
    {
        T u[LX];
        lpencil<LX, T, false>(u, A.u + e0, t);
        grad_lean<LX, T>(D, u, s0, s1, a, b, wr, ws, wt);
    }
    apply_G_lean<LX, T, KPOISSON, true>(fresh(A.G + e0), (const T *)nullptr, T(1), A.n, t, wr, ws, wt);
    T vr[LX], vs[LX], vt[LX];
    {
        T v[LX];
        lpencil<LX, T, false>(v, A.v + e0, t);
        grad_lean<LX, T>(D, v, s0, s1, a, b, vr, vs, vt);
    }
    T out[LX];
#pragma unroll
    for (int i = 0; i < LX; ++i) out[i] = vr[i] * wr[i] + vs[i] * ws[i] + vt[i] * wt[i];
    spencil<LX, T>(A.g + e0, t, out);
}

template <int LX, typename T>
__global__ SEM_BOUNDS2((Shape<LX, T>::NT), (Shape<LX, T>::MINW)) void k_ax_adjoint_lean(
    AdjArgs<T> A, DEo<LX, T> D, const DEo<LX, T> *__restrict__ Dg)
{
    if constexpr (sizeof(T) == 8) adj_lean_body<LX, T>(DMem<LX, T>{Dg}, A);
    else adj_lean_body<LX, T>(DArg<LX, T>{D}, A);
}

// ------------------------------------------------------------------ h1-adjoint
// g = (D v)^T G (D u) per point.
template <int LX, typename T>
__global__ SEM_BOUNDS2((Shape<LX, T>::NT), (Shape<LX, T>::MINW)) void k_ax_adjoint(AdjArgs<T> A, DEo<LX, T> D)
{
    using S = Shape<LX, T>;
    __shared__ Lds<LX, T> lds;
    const int tid = threadIdx.x;
    const int slot = tid / S::NP;
    const int t = tid - slot * S::NP;
    const int a = t % LX, b = t / LX;
    const int64_t e = (int64_t)blockIdx.x * S::EPB + slot;
    const bool act = e < A.nelv;
    const int64_t row = e * (int64_t)(LX * LX * LX) + t;  // base of this lane's t-pencil
    T *s0 = lds.buf[0][slot], *s1 = lds.buf[1][slot];

    T u[LX], v[LX];
    load_row<LX, T>(u, A.u + row, act);
    load_row<LX, T>(v, A.v + row, act);
    T g[6][LX];
#pragma unroll
    for (int f = 0; f < 6; ++f) load_g<LX, T>(g[f], A.G + f * A.n + row, act);
    T ur[LX], us[LX], ut[LX], vr[LX], vs[LX], vt[LX];
    grad<LX, T>(D, u, s0, s1, a, b, ur, us, ut);
    grad<LX, T>(D, v, s0, s1, a, b, vr, vs, vt);
    T out[LX];
#pragma unroll
    for (int i = 0; i < LX; ++i) {
        const T r = ur[i], s = us[i], q = ut[i];
        out[i] = vr[i] * (g[0][i] * r + g[3][i] * s + g[4][i] * q)
               + vs[i] * (g[3][i] * r + g[1][i] * s + g[5][i] * q)
               + vt[i] * (g[4][i] * r + g[5][i] * s + g[2][i] * q);
    }
    store_row<LX, T>(A.g + row, out, act);
}

// ------------------------------------------------------------------ setup kernels
// Geometric factors from nodal coordinates (isoparametric metric, FP64).
// One thread per point; plain loops (setup only).
template <int LX>
__global__ __launch_bounds__(256) void k_geometry(GeomArgs A, DMat<LX, double> D, WVec<LX> W)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    constexpr int NPE = LX * LX * LX;
    const int64_t e = p / NPE;
    const int q = (int)(p - e * NPE);
    const int i = q % LX, j = (q / LX) % LX, k = q / (LX * LX);
    const int64_t b0 = e * NPE;
    double m[3][3];
    for (int c = 0; c < 3; ++c) {
        const double *X = A.xyz + c * A.n + b0;
        double dr = 0, ds = 0, dt = 0;
#pragma unroll
        for (int l = 0; l < LX; ++l) {
            dr = fma(D.d[i * LX + l], X[l + LX * (j + LX * k)], dr);
            ds = fma(D.d[j * LX + l], X[i + LX * (l + LX * k)], ds);
            dt = fma(D.d[k * LX + l], X[i + LX * (j + LX * l)], dt);
        }
        m[c][0] = dr;
        m[c][1] = ds;
        m[c][2] = dt;
    }
    // cofactors: C[c][d] = d(det)/d m[c][d];  inverse: dr_d/dx_c = C[c][d] / J
    double C[3][3];
    C[0][0] = m[1][1] * m[2][2] - m[1][2] * m[2][1];
    C[0][1] = m[1][2] * m[2][0] - m[1][0] * m[2][2];
    C[0][2] = m[1][0] * m[2][1] - m[1][1] * m[2][0];
    C[1][0] = m[0][2] * m[2][1] - m[0][1] * m[2][2];
    C[1][1] = m[0][0] * m[2][2] - m[0][2] * m[2][0];
    C[1][2] = m[0][1] * m[2][0] - m[0][0] * m[2][1];
    C[2][0] = m[0][1] * m[1][2] - m[0][2] * m[1][1];
    C[2][1] = m[0][2] * m[1][0] - m[0][0] * m[1][2];
    C[2][2] = m[0][0] * m[1][1] - m[0][1] * m[1][0];
    const double J = m[0][0] * C[0][0] + m[0][1] * C[0][1] + m[0][2] * C[0][2];
    const double rho = W.w[i] * W.w[j] * W.w[k];
    // G_ab = rho J sum_c (C[c][a]/J)(C[c][b]/J) = rho/J sum_c C[c][a] C[c][b]
    const double s = rho / J;
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int f = 0; f < 6; ++f) {
        const double d = C[0][ia[f]] * C[0][ib[f]] + C[1][ia[f]] * C[1][ib[f]] + C[2][ia[f]] * C[2][ib[f]];
        A.G[f * A.n + p] = s * d;
    }
    A.B[p] = rho * J;
    if (!(J > 0.0)) atomicAdd(A.nbad, 1u);
}

// Diagonal of the unassembled operator (point Jacobi), FP64, one thread per point.
template <int LX>
__global__ __launch_bounds__(256) void k_diag(DiagArgs A, DMat<LX, double> D)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    constexpr int NPE = LX * LX * LX;
    const int64_t e = p / NPE;
    const int q = (int)(p - e * NPE);
    const int i = q % LX, j = (q / LX) % LX, k = q / (LX * LX);
    const int64_t b0 = e * NPE;
    const double *G = A.G;
    const int64_t n = A.n;
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < LX; ++l) {
        const int64_t pr = b0 + l + LX * (j + LX * k);
        const int64_t ps = b0 + i + LX * (l + LX * k);
        const int64_t pt = b0 + i + LX * (j + LX * l);
        const double cr = A.h1 ? A.h1[pr] : A.h1s;
        const double cs = A.h1 ? A.h1[ps] : A.h1s;
        const double ct = A.h1 ? A.h1[pt] : A.h1s;
        const double dri = D.d[l * LX + i], dsj = D.d[l * LX + j], dtk = D.d[l * LX + k];
        s += dri * dri * cr * G[pr];
        s += dsj * dsj * cs * G[n + ps];
        s += dtk * dtk * ct * G[2 * n + pt];
    }
    const double c = A.h1 ? A.h1[p] : A.h1s;
    const double di = D.d[i * LX + i], dj = D.d[j * LX + j], dk = D.d[k * LX + k];
    s += 2.0 * di * dj * c * G[3 * n + p];
    s += 2.0 * di * dk * c * G[4 * n + p];
    s += 2.0 * dj * dk * c * G[5 * n + p];
    const double c2 = A.h2 ? A.h2[p] : A.h2s;
    if (c2 != 0.0) s += c2 * A.B[p];
    A.d[p] = s;
}

}  // namespace sem

// ------------------------------------------------------------------ host launchers
#define SEM_PASTE2(a, b) a##b
#define SEM_PASTE(a, b) SEM_PASTE2(a, b)

namespace {
template <int LX, typename T>
sem::DMat<LX, T> make_dmat(const double *D)
{
    sem::DMat<LX, T> m;
    for (int q = 0; q < LX * LX; ++q) m.d[q] = (T)D[q];
    return m;
}

template <int LX, typename T>
sem::DEo<LX, T> make_deo(const double *D)
{
    using E = sem::DEo<LX, T>;
    constexpr int H = E::H, N = LX - 1;
    E m{};
    for (int a = 0; a < H; ++a)
        for (int l = 0; l < H; ++l) {
            m.S[a * H + l] = (T)(0.5 * (D[a * LX + l] + D[a * LX + (N - l)]));
            m.A[a * H + l] = (T)(0.5 * (D[a * LX + l] - D[a * LX + (N - l)]));
        }
    if constexpr (LX % 2 == 1) {
        for (int a = 0; a < H; ++a) {
            m.cm[a] = (T)D[a * LX + H];
            m.rm[a] = (T)D[H * LX + a];
        }
    }
    return m;
}

// Coefficient form of a lean launch (see LeanKind).
template <typename T>
int lean_kind(const T *h1, const T *h2, T h2s)
{
    if (h2) return sem::KGEN;
    if (h2s == T(0)) return h1 ? sem::KGEN : sem::KPOISSON;
    return h1 ? sem::KH1F : sem::KHELM;
}

template <typename T>
hipError_t launch_ax(const sem::AxArgs<T> &A, const double *D, int nfields, hipStream_t st)
{
    using S = sem::Shape<SEM_LX, T>;
    const unsigned grid = (unsigned)((A.nelv + S::EPB - 1) / S::EPB);
    if (grid == 0) return hipSuccess;
    const auto Dm = make_deo<SEM_LX, T>(D);
    if constexpr (S::LEAN) {
        if (sizeof(T) == 8 && !A.deo) return hipErrorInvalidValue;
        const int kind = lean_kind(A.h1, A.h2, A.h2s);
#define SEM_LEAN_AX(NF_, K_)                                                                               \
    hipLaunchKernelGGL((sem::k_ax_helm_lean<SEM_LX, T, NF_, K_>), dim3(grid), dim3(S::NT), 0, st, A, Dm, \
                       (const sem::DEo<SEM_LX, T> *)A.deo)
        if (nfields == 3) {
            switch (kind) {
            case sem::KPOISSON: SEM_LEAN_AX(3, sem::KPOISSON); break;
            case sem::KHELM: SEM_LEAN_AX(3, sem::KHELM); break;
            case sem::KH1F: SEM_LEAN_AX(3, sem::KH1F); break;
            default: SEM_LEAN_AX(3, sem::KGEN); break;
            }
        } else {
            switch (kind) {
            case sem::KPOISSON: SEM_LEAN_AX(1, sem::KPOISSON); break;
            case sem::KHELM: SEM_LEAN_AX(1, sem::KHELM); break;
            case sem::KH1F: SEM_LEAN_AX(1, sem::KH1F); break;
            default: SEM_LEAN_AX(1, sem::KGEN); break;
            }
        }
#undef SEM_LEAN_AX
    } else {
        const bool gen = A.h1 || A.h2 || A.h2s != T(0);
        if (nfields == 3) {
            if (gen) hipLaunchKernelGGL((sem::k_ax_helm<SEM_LX, T, 3, true>), dim3(grid), dim3(S::NT), 0, st, A, Dm);
            else hipLaunchKernelGGL((sem::k_ax_helm<SEM_LX, T, 3, false>), dim3(grid), dim3(S::NT), 0, st, A, Dm);
        } else {
            if (gen) hipLaunchKernelGGL((sem::k_ax_helm<SEM_LX, T, 1, true>), dim3(grid), dim3(S::NT), 0, st, A, Dm);
            else hipLaunchKernelGGL((sem::k_ax_helm<SEM_LX, T, 1, false>), dim3(grid), dim3(S::NT), 0, st, A, Dm);
        }
    }
    return hipGetLastError();
}

template <typename T, bool CG1>
hipError_t launch_cg(const sem::CgMatvecArgs<T> &A, const double *D, int nfields, hipStream_t st)
{
    using S = sem::Shape<SEM_LX, T>;
    const unsigned grid = (unsigned)((A.nelv + S::EPB - 1) / S::EPB);
    if (grid == 0) return hipSuccess;
    const auto Dm = make_deo<SEM_LX, T>(D);
    if constexpr (S::LEAN) {
        if (sizeof(T) == 8 && !A.deo) return hipErrorInvalidValue;
        const int kind = lean_kind(A.h1, A.h2, A.h2s);
#define SEM_LEAN_CG(NF_, K_)                                                                               \
    hipLaunchKernelGGL((sem::k_cg_matvec_lean<SEM_LX, T, NF_, K_, CG1>), dim3(grid), dim3(S::NT), 0, st, A, Dm, \
                       (const sem::DEo<SEM_LX, T> *)A.deo)
        if (nfields == 3) {
            switch (kind) {
            case sem::KPOISSON: SEM_LEAN_CG(3, sem::KPOISSON); break;
            case sem::KHELM: SEM_LEAN_CG(3, sem::KHELM); break;
            case sem::KH1F: SEM_LEAN_CG(3, sem::KH1F); break;
            default: SEM_LEAN_CG(3, sem::KGEN); break;
            }
        } else {
            switch (kind) {
            case sem::KPOISSON: SEM_LEAN_CG(1, sem::KPOISSON); break;
            case sem::KHELM: SEM_LEAN_CG(1, sem::KHELM); break;
            case sem::KH1F: SEM_LEAN_CG(1, sem::KH1F); break;
            default: SEM_LEAN_CG(1, sem::KGEN); break;
            }
        }
#undef SEM_LEAN_CG
    } else {
        const bool gen = A.h1 || A.h2 || A.h2s != T(0);
        if (nfields == 3) {
            if (gen) hipLaunchKernelGGL((sem::k_cg_matvec<SEM_LX, T, 3, true, CG1>), dim3(grid), dim3(S::NT), 0, st, A, Dm);
            else hipLaunchKernelGGL((sem::k_cg_matvec<SEM_LX, T, 3, false, CG1>), dim3(grid), dim3(S::NT), 0, st, A, Dm);
        } else {
            if (gen) hipLaunchKernelGGL((sem::k_cg_matvec<SEM_LX, T, 1, true, CG1>), dim3(grid), dim3(S::NT), 0, st, A, Dm);
            else hipLaunchKernelGGL((sem::k_cg_matvec<SEM_LX, T, 1, false, CG1>), dim3(grid), dim3(S::NT), 0, st, A, Dm);
        }
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj(const sem::AdjArgs<T> &A, const double *D, hipStream_t st)
{
    using S = sem::Shape<SEM_LX, T>;
    const unsigned grid = (unsigned)((A.nelv + S::EPB - 1) / S::EPB);
    if (grid == 0) return hipSuccess;
    if constexpr (S::LEAN) {
        if (sizeof(T) == 8 && !A.deo) return hipErrorInvalidValue;
        hipLaunchKernelGGL((sem::k_ax_adjoint_lean<SEM_LX, T>), dim3(grid), dim3(S::NT), 0, st, A,
                           make_deo<SEM_LX, T>(D), (const sem::DEo<SEM_LX, T> *)A.deo);
    }
    else
        hipLaunchKernelGGL((sem::k_ax_adjoint<SEM_LX, T>), dim3(grid), dim3(S::NT), 0, st, A,
                           make_deo<SEM_LX, T>(D));
    return hipGetLastError();
}
}  // namespace

extern "C" {

hipError_t SEM_PASTE(sem_launch_ax_f64_lx, SEM_LX)(const sem::AxArgs<double> *A, const double *D,
                                                    int nfields, hipStream_t st)
{
    return launch_ax<double>(*A, D, nfields, st);
}
hipError_t SEM_PASTE(sem_launch_ax_f32_lx, SEM_LX)(const sem::AxArgs<float> *A, const double *D,
                                                    int nfields, hipStream_t st)
{
    return launch_ax<float>(*A, D, nfields, st);
}
hipError_t SEM_PASTE(sem_launch_cg_f64_lx, SEM_LX)(const sem::CgMatvecArgs<double> *A,
                                                    const double *D, int nfields, hipStream_t st)
{
    return launch_cg<double, false>(*A, D, nfields, st);
}
hipError_t SEM_PASTE(sem_launch_cg_f32_lx, SEM_LX)(const sem::CgMatvecArgs<float> *A,
                                                    const double *D, int nfields, hipStream_t st)
{
    return launch_cg<float, false>(*A, D, nfields, st);
}
hipError_t SEM_PASTE(sem_launch_cg1_f64_lx, SEM_LX)(const sem::CgMatvecArgs<double> *A,
                                                     const double *D, int nfields, hipStream_t st)
{
    return launch_cg<double, true>(*A, D, nfields, st);
}
hipError_t SEM_PASTE(sem_launch_adj_f64_lx, SEM_LX)(const sem::AdjArgs<double> *A, const double *D,
                                                     hipStream_t st)
{
    return launch_adj<double>(*A, D, st);
}
hipError_t SEM_PASTE(sem_launch_adj_f32_lx, SEM_LX)(const sem::AdjArgs<float> *A, const double *D,
                                                     hipStream_t st)
{
    return launch_adj<float>(*A, D, st);
}
hipError_t SEM_PASTE(sem_launch_geom_lx, SEM_LX)(const sem::GeomArgs *A, const double *D,
                                                  const double *w, hipStream_t st)
{
    if (A->n == 0) return hipSuccess;
    sem::WVec<SEM_LX> W;
    for (int i = 0; i < SEM_LX; ++i) W.w[i] = w[i];
    const unsigned grid = (unsigned)((A->n + 255) / 256);
    hipLaunchKernelGGL((sem::k_geometry<SEM_LX>), dim3(grid), dim3(256), 0, st, *A,
                       make_dmat<SEM_LX, double>(D), W);
    return hipGetLastError();
}
hipError_t SEM_PASTE(sem_launch_diag_lx, SEM_LX)(const sem::DiagArgs *A, const double *D,
                                                  hipStream_t st)
{
    if (A->n == 0) return hipSuccess;
    const unsigned grid = (unsigned)((A->n + 255) / 256);
    hipLaunchKernelGGL((sem::k_diag<SEM_LX>), dim3(grid), dim3(256), 0, st, *A,
                       make_dmat<SEM_LX, double>(D));
    return hipGetLastError();
}
// The even-odd D of this lx in FP64 and FP32 (the DEo layouts), for the device copy
// the lean FP64 kernels read (out64, out32: host buffers of the two struct sizes).
void SEM_PASTE(sem_deo_fill_lx, SEM_LX)(const double *D, void *out64, void *out32)
{
    const auto m64 = make_deo<SEM_LX, double>(D);
    const auto m32 = make_deo<SEM_LX, float>(D);
    memcpy(out64, &m64, sizeof(m64));
    memcpy(out32, &m32, sizeof(m32));
}
// number of per-workgroup partials the CG matvec writes per field
int64_t SEM_PASTE(sem_cg_nblocks_f64_lx, SEM_LX)(int64_t nelv)
{
    using S = sem::Shape<SEM_LX, double>;
    return (nelv + S::EPB - 1) / S::EPB;
}
int64_t SEM_PASTE(sem_cg_nblocks_f32_lx, SEM_LX)(int64_t nelv)
{
    using S = sem::Shape<SEM_LX, float>;
    return (nelv + S::EPB - 1) / S::EPB;
}
}
