// vec_kernels.hip -- gather-scatter, masking and Krylov-vector kernels of libsem (gfx950).
//
// Gather-scatter QQ^T (Jansson et al., arXiv 2107.01243, Eq. 10 and the local
// gather + scatter of Algorithm 1): ids with two copies are a pair list (the
// "injective" ids of Section 3.2), ids with more copies are CSR blocks.  One lane
// per pair / block sums the copies in ascending local order starting from +0 and
// writes the sum back, so the result is deterministic and bit-reproducible.
//
// CG / flexible-CG vector kernels: streaming, one point per lane per step with
// grid-stride loops, FP64 accumulation of every inner product, per-workgroup
// partial sums reduced afterwards in a fixed order by a single workgroup
// (deterministic; no floating-point atomics).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "sem_kernels.h"
#include "vec_kernels.h"

#ifndef SEM_GS_XCD
#define SEM_GS_XCD 1
#endif

namespace sem {

#ifndef SEM_VCH
#define SEM_VCH 2
#endif

constexpr int VT = 256;   // lanes per workgroup of the streaming kernels
// Streaming kernels: workgroup b handles the contiguous chunk [b*CHUNK, (b+1)*CHUNK)
// (VCH points per lane); the grid is as wide as the vector, and the number of
// per-workgroup partial sums stays n / CHUNK.
constexpr int VCH = SEM_VCH;
constexpr int64_t CHUNK = (int64_t)VT * VCH;
constexpr int RT = 1024;  // lanes of the single-workgroup reduction kernels

#ifndef SEM_UPD64
#define SEM_UPD64 2
#endif
#ifndef SEM_GS_EPL
#define SEM_GS_EPL 2
#endif
constexpr int GEPL = SEM_GS_EPL;  // 64-entry segments per wave of the entry-parallel gs
#ifndef SEM_UPD32
#define SEM_UPD32 8
#endif
// Points per lane of one CG-update workgroup, per precision: an FP32 chunk moves half
// the bytes of an FP64 one, so it takes more points to amortise the workgroup's
// reduction epilogue (and it halves the partials the finish kernel sums).
template <typename T> struct UpdChunk;
template <> struct UpdChunk<double> { static constexpr int UV = SEM_UPD64; };
template <> struct UpdChunk<float> { static constexpr int UV = SEM_UPD32; };

// Sum `nblk` partials in a fixed order inside one workgroup of NTH lanes: lane t
// accumulates entries t, t+NTH, ... into four interleaved accumulators (loads in
// flight), combines them, then a fixed binary tree in LDS.  Deterministic for a
// given (nblk, NTH).  Returns the sum to every lane.
template <int NTH>
__device__ double block_sum_fixed(const double *part, int64_t nblk, double *sh)
{
    const int tid = threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t q = tid;
    for (; q + 3 * NTH < nblk; q += 4 * NTH) {
        a0 += part[q];
        a1 += part[q + NTH];
        a2 += part[q + 2 * NTH];
        a3 += part[q + 3 * NTH];
    }
    for (; q < nblk; q += NTH) a0 += part[q];
    sh[tid] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    for (int w = NTH / 2; w > 0; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Single-reduction CG (Chronopoulos-Gear) scalars once r_k and w_k = A u_k are known
// (u_k = dinv r_k): gamma = (r_k, u_k), delta = (u_k, A u_k), rr = (r_k, r_k).  On the
// first call (primed == 0) beta = 0 and alpha = gamma / delta; afterwards
// beta = gamma / gamma_old and alpha = gamma / (delta - beta gamma / alpha_old), which
// reproduce the two-reduction CG recurrences in exact arithmetic.
__device__ inline void cg1_fold(CgScalars &s, double gamma, double delta, double rr)
{
    if (s.stop) return;
    const bool first = s.primed == 0;
    if (!first) s.iter += 1;
    s.rr = rr;
    const double rel = s.bb > 0.0 ? sqrt(rr / s.bb) : 0.0;
    if (!isfinite(gamma) || !isfinite(delta) || !isfinite(rr)) {
        s.stop = 1;
        s.status = 2;
        return;
    }
    if ((s.rtol > 0.0 && rel <= s.rtol) || gamma == 0.0) {
        s.stop = 1;
        s.rz = gamma;
        return;
    }
    if (s.iter >= s.max_iter) {
        s.stop = 1;
        s.status = (s.rtol > 0.0) ? 1 : 0;
        return;
    }
    const double beta = first ? 0.0 : gamma / s.rz;
    const double den = first ? delta : delta - beta * gamma / s.alpha;
    if (!(den > 0.0) || !isfinite(den)) {
        s.stop = 1;
        s.status = 2;
        s.alpha = 0.0;
        return;
    }
    s.beta = beta;
    s.alpha = gamma / den;
    s.rz = gamma;
    s.primed = 1;
}

// Fold of the CG scalars for every field by workgroup 0 of a gather-scatter launch
// (the matvec whose partials it reads ended before this launch began).
template <int NTH>
__device__ void fold_job(const AlphaJob &J, int nfields, double *sh)
{
    for (int f = 0; f < nfields; ++f) {
        if (J.mode == 0) {
            const double pw = block_sum_fixed<NTH>(J.partial + f * J.nblk, J.nblk, sh);
            if (threadIdx.x == 0) {
                CgScalars &sc = J.scal[f];
                if (!sc.stop) {
                    if (!(pw > 0.0) || !isfinite(pw) || !isfinite(sc.rz)) {
                        sc.stop = 1;
                        sc.status = 2;
                        sc.alpha = 0.0;
                    } else {
                        sc.alpha = sc.rz / pw;
                    }
                }
            }
        } else {
            const double d = block_sum_fixed<NTH>(J.partial + f * J.nblk, J.nblk, sh);
            CgScalars &sc = J.scal[f];
            double g = sc.rz, rr = sc.rr;  // before the first step: from the start kernels
            if (sc.primed) {               // uniform: every lane reads the same flag
                g = block_sum_fixed<NTH>(J.partial2 + (0 * nfields + f) * J.nblk2, J.nblk2, sh);
                rr = block_sum_fixed<NTH>(J.partial2 + (1 * nfields + f) * J.nblk2, J.nblk2, sh);
            }
            if (threadIdx.x == 0) cg1_fold(sc, g, d, rr);
            __syncthreads();  // the next field's reads follow lane 0's update
        }
    }
}

// ------------------------------------------------------------------ gather-scatter
template <typename T>
__global__ __launch_bounds__(VT) void k_gs(GsArgs<T> A)
{
    // Workgroups are dealt to the 8 XCDs round-robin by the hardware.  Map them so
    // that XCD x processes one contiguous slice of the group list (which is ordered
    // by element), so each XCD's L2 works on one contiguous range of elements.
#if SEM_GS_XCD
    const unsigned per = gridDim.x / 8;  // the launcher rounds the grid up to 8 * per
    const unsigned lb = (blockIdx.x % 8) * per + blockIdx.x / 8;
#else
    const unsigned lb = blockIdx.x;
#endif
    const int64_t tid = (int64_t)lb * VT + threadIdx.x;
    for (int f = 0; f < A.nfields; ++f) {
        if (A.skip && A.skip[f].stop) continue;
        T *u = A.u + f * A.n;
        if (tid < A.npairs) {
            const int32_t a = A.pairs[2 * tid], b = A.pairs[2 * tid + 1];
            const T s = (T(0) + u[a]) + u[b];
            u[a] = s;
            u[b] = s;
        } else if (tid < A.npairs + A.nblocks) {
            const int64_t g = tid - A.npairs;
            const int64_t lo = A.blk_ptr[g], hi = A.blk_ptr[g + 1];
            T s = T(0);
            for (int64_t c = lo; c < hi; ++c) s += u[A.blk_idx[c]];
            for (int64_t c = lo; c < hi; ++c) u[A.blk_idx[c]] = s;
        }
    }
    // Optional fold of the CG step length: alpha_f = rz_f / (p, A p)_f from the
    // matvec's partials (complete, since that kernel ended before this one began).
    if (A.alpha_job && blockIdx.x == 0) {
        __shared__ double sh[VT];
        fold_job<VT>(*A.alpha_job, A.nfields, sh);
    }
}

// Entry-parallel gather-scatter: a lane owns one shared entry in each of the
// wave's segments of 64 (ascending global id, groups never straddle a segment).  Every lane of a group reads the group's values
// from its neighbour lanes and sums them in ascending local order from +0, so all
// copies receive the identical, canonical sum; then each lane writes its own copy.
// The shuffle loop runs max_group times for the whole wave (all lanes active).
template <typename T>
__global__ __launch_bounds__(VT) void k_gs_entries(GsArgs<T> A)
{
#if SEM_GS_XCD
    const unsigned per = gridDim.x / 8;
    const unsigned lb = (blockIdx.x % 8) * per + blockIdx.x / 8;
#else
    const unsigned lb = blockIdx.x;
#endif
    if (A.skip) {
        // every field stopped: nothing to gather, and no step length left to set
        bool live = false;
        for (int f = 0; f < A.nfields; ++f) live = live || !A.skip[f].stop;
        if (!live) return;
    }
    // each wave owns GEPL consecutive 64-entry segments; lane l handles entry l of
    // each, so its GEPL index -> value loads are independent and in flight together
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = ((int64_t)lb * VT + (int64_t)wave * 64) * GEPL + lane;
    int32_t e[GEPL];
    int cnt[GEPL], lead[GEPL];
    // a group's extent from the start flags of the segment: its first lane is the
    // nearest flagged lane at or below this one, its end the next flagged lane (padding
    // counts as flagged, and every segment opens with a flagged lane)
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
#pragma unroll
    for (int k = 0; k < GEPL; ++k) {
        const int64_t t = base + 64 * k;
        const uint32_t wd = t < A.nent ? A.ent_word[t] : 0xffffffffu;
        const bool pad = wd == 0xffffffffu;
        e[k] = pad ? -1 : (int32_t)(wd & 0x7fffffffu);
        const uint64_t M = __ballot(pad || (wd >> 31) != 0);
        lead[k] = 63 - __clzll((long long)(M & upto));
        const uint64_t above = M & ~upto;
        cnt[k] = (above ? __ffsll((long long)above) - 1 : 64) - lead[k];
    }
    for (int f = 0; f < A.nfields; ++f) {
        if (A.skip && A.skip[f].stop) continue;
        T *u = A.u + f * A.n;
        T v[GEPL], s[GEPL];
#pragma unroll
        for (int k = 0; k < GEPL; ++k) {
            v[k] = (e[k] >= 0) ? u[e[k]] : T(0);
            s[k] = T(0);
        }
        for (int q = 0; q < A.max_group; ++q) {
#pragma unroll
            for (int k = 0; k < GEPL; ++k) {
                const int src = lead[k] + q;
                const T x = __shfl(v[k], src < 64 ? src : lane, 64);
                if (q < cnt[k]) s[k] += x;
            }
        }
#pragma unroll
        for (int k = 0; k < GEPL; ++k)
            if (e[k] >= 0) u[e[k]] = s[k];
    }
    if (A.alpha_job && blockIdx.x == 0) {
        __shared__ double sh[VT];
        fold_job<VT>(*A.alpha_job, A.nfields, sh);
    }
}

// ------------------------------------------------------------------ basis combinations
// Linear combination of up to PB basis vectors (coefficients by value).
__global__ __launch_bounds__(VT) void k_comb(CombArgs A)
{
    // the starting vector is chosen once per launch (uniform): none, y itself, or src.
    // (Selecting it per point with a nested conditional was compiled, for src, into a
    // load through a scalar register that was never assigned on that path.)
    const double *s0 = (A.mode == 1) ? A.y : A.src;
    const bool start = A.mode != 0;
    const int64_t t_end = min(A.n, (int64_t)(blockIdx.x + 1) * CHUNK);
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x; t < t_end; t += VT) {
        double s = 0.0;
        if (start) s = s0[t];
#pragma unroll
        for (int i = 0; i < PB; ++i)
            if (i < A.l) s = fma(A.c[i], A.V[i * A.ld + t], s);
        A.y[t] = s;
    }
}

// Arnoldi pass (see ArnArgs).  Each workgroup streams one contiguous chunk of
// points; every lane keeps the m basis values of its point in registers, so the
// combination and the dots of the combined vector need one read of each vector.
// The basis (tens of vectors, far beyond the last-level cache) is read with
// non-temporal hints, as in the Gram-Schmidt passes below.
template <int MV, int MODE>
__global__ __launch_bounds__(VT) void k_arn(ArnArgs A, int64_t chunk)
{
    const int m = A.m;
    double c[MV];
    double sc = 1.0;
    if constexpr (MODE != 0) {
#pragma unroll
        for (int i = 0; i < MV; ++i) c[i] = (i < m) ? A.coef[i] : 0.0;
        if constexpr (MODE == 2) sc = A.scale[0];
    }
    double acc[MV + 1];
#pragma unroll
    for (int i = 0; i <= MV; ++i) acc[i] = 0.0;
    const int64_t t0 = (int64_t)blockIdx.x * chunk;
    const int64_t t1 = min(A.n, t0 + chunk);
    for (int64_t t = t0 + threadIdx.x; t < t1; t += VT) {
        double v[MV];
#pragma unroll
        for (int i = 0; i < MV; ++i) v[i] = (i < m) ? __builtin_nontemporal_load(A.V + i * A.ld + t) : 0.0;
        double y = A.w[t];
        if constexpr (MODE != 0) {
#pragma unroll
            for (int i = 0; i < MV; ++i)
                if (i < m) y = fma(-c[i], v[i], y);
            if constexpr (MODE == 2) y *= sc;
            A.y[t] = y;
        }
        if constexpr (MODE != 2) {
            const double yo = A.owner[t] ? y : 0.0;
#pragma unroll
            for (int i = 0; i < MV; ++i)
                if (i < m) acc[i] = fma(v[i], yo, acc[i]);
            acc[MV] = fma(y, yo, acc[MV]);
        }
    }
    if constexpr (MODE != 2) {
        __shared__ double sh[VT / 64][MV + 1];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int i = 0; i <= MV; ++i) {
            if (i < m || i == MV) {
                double x = acc[i];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
                if (lane == 0) sh[wave][i] = x;
            }
        }
        __syncthreads();
        const int q = threadIdx.x;
        if (q <= m) {
            const int src = (q < m) ? q : MV;
            double x = 0.0;
#pragma unroll
            for (int w4 = 0; w4 < VT / 64; ++w4) x += sh[w4][src];
            A.partial[(int64_t)q * gridDim.x + blockIdx.x] = x;
        }
    }
}

// Sums of nq rows of per-workgroup partials, one wave per row, fixed order.  With
// pyth, the last row is a squared norm |y|^2 and the others the coefficients h of a
// second Gram-Schmidt pass: out[nq] = sqrt(|y|^2 - |h|^2) (the norm after that pass,
// by the Pythagorean identity) and out[nq + 1] = its reciprocal (0 if not positive).
__global__ __launch_bounds__(RT) void k_arn_finish(const double *partial, int64_t nblk, int nq, int pyth,
                                                   double *out)
{
    __shared__ double sh[ARN_MAXV + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = wave; q < nq; q += RT / 64) {
        double s = 0.0;
        for (int64_t b = lane; b < nblk; b += 64) s += partial[(int64_t)q * nblk + b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) {
            out[q] = s;
            sh[q] = s;
        }
    }
    if (pyth) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const int m = nq - 1;
            double hh = sh[m];
            for (int i = 0; i < m; ++i) hh = fma(-sh[i], sh[i], hh);
            hh = hh > 0.0 ? hh : 0.0;
            out[nq] = sqrt(hh);
            out[nq + 1] = hh > 0.0 ? 1.0 / sqrt(hh) : 0.0;
        }
    }
}

// Dots pass of the delayed Gram-Schmidt step (see DcgsArgs).
template <int MV>
__global__ __launch_bounds__(VT) void k_dcgs_dots(DcgsArgs A, int64_t chunk)
{
    constexpr int NR = 2 * MV + 3;
    const int j = A.j;
    double ua[MV], wb[MV], uu = 0.0, uw = 0.0, ww = 0.0;
#pragma unroll
    for (int i = 0; i < MV; ++i) ua[i] = wb[i] = 0.0;
    const int64_t t0 = (int64_t)blockIdx.x * chunk;
    const int64_t t1 = min(A.n, t0 + chunk);
    for (int64_t t = t0 + threadIdx.x; t < t1; t += VT) {
        double v[MV];
#pragma unroll
        for (int i = 0; i < MV; ++i) v[i] = (i < j) ? __builtin_nontemporal_load(A.V + i * A.ld + t) : 0.0;
        const double u = A.u[t], w = A.w[t];
        const bool own = A.owner[t] != 0;
        const double uo = own ? u : 0.0, wo = own ? w : 0.0;
#pragma unroll
        for (int i = 0; i < MV; ++i)
            if (i < j) {
                ua[i] = fma(v[i], uo, ua[i]);
                wb[i] = fma(v[i], wo, wb[i]);
            }
        uu = fma(u, uo, uu);
        uw = fma(u, wo, uw);
        ww = fma(w, wo, ww);
    }
    // rows: a_0..a_{j-1}, (u,u), b_0..b_{j-1}, (u,w), (w,w)
    __shared__ double sh[VT / 64][NR];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto put = [&](int q, double x) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) sh[wave][q] = x;
    };
#pragma unroll
    for (int i = 0; i < MV; ++i)
        if (i < j) {
            put(i, ua[i]);
            put(j + 1 + i, wb[i]);
        }
    put(j, uu);
    put(2 * j + 1, uw);
    put(2 * j + 2, ww);
    __syncthreads();
    const int q = threadIdx.x;
    if (q < 2 * j + 3) {
        double x = 0.0;
#pragma unroll
        for (int w4 = 0; w4 < VT / 64; ++w4) x += sh[w4][q];
        A.partial[(int64_t)q * gridDim.x + blockIdx.x] = x;
    }
}

// Update pass of the delayed Gram-Schmidt step (see DcgsArgs).
template <int MV>
__global__ __launch_bounds__(VT) void k_dcgs_update(DcgsArgs A, int64_t chunk)
{
    const int j = A.j;
    const double *cf = A.coef;
    double ca[MV], cc[MV];
#pragma unroll
    for (int i = 0; i < MV; ++i) {
        ca[i] = (i < j) ? cf[i] : 0.0;
        cc[i] = (i < j) ? cf[j + i] : 0.0;
    }
    const double irho = cf[2 * j], del = cf[2 * j + 1], inu = cf[2 * j + 2];
    const int64_t t0 = (int64_t)blockIdx.x * chunk;
    const int64_t t1 = min(A.n, t0 + chunk);
    for (int64_t t = t0 + threadIdx.x; t < t1; t += VT) {
        double v[MV];
#pragma unroll
        for (int i = 0; i < MV; ++i) v[i] = (i < j) ? __builtin_nontemporal_load(A.V + i * A.ld + t) : 0.0;
        const double u = A.u[t];
        double q = u, y = A.w[t];
#pragma unroll
        for (int i = 0; i < MV; ++i)
            if (i < j) {
                q = fma(-ca[i], v[i], q);
                y = fma(-cc[i], v[i], y);
            }
        y = fma(-del, u, y);
        A.u[t] = q * irho;
        A.w[t] = y * inu;
    }
}

// Reduction of the dots pass, one wave per row in a fixed order: out[0..2j+3) = the
// row sums; then at out + 2 j + 3 the update coefficients and the step's scalars:
//   rho^2 = (u,u) - |a|^2,  gamma = ((u,w) - a.b) / rho,  delta = gamma / rho,
//   nu^2 = (w,w) - |b|^2 - gamma^2  (Pythagorean identities),  c = b - delta a;
//   [a (j), c (j), 1/rho, delta, 1/nu, rho, gamma, nu]  (reciprocals 0 when not positive).
__global__ __launch_bounds__(RT) void k_dcgs_finish(const double *partial, int64_t nblk, int j, double *out)
{
    __shared__ double sh[2 * ARN_MAXV + 3];
    const int nq = 2 * j + 3;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = wave; q < nq; q += RT / 64) {
        double s = 0.0;
        for (int64_t b = lane; b < nblk; b += 64) s += partial[(int64_t)q * nblk + b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) {
            out[q] = s;
            sh[q] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double *a = sh, *b = sh + j + 1;
        double aa = sh[j], ab = sh[2 * j + 1], bb = sh[2 * j + 2];
        for (int i = 0; i < j; ++i) {
            aa = fma(-a[i], a[i], aa);
            ab = fma(-a[i], b[i], ab);
            bb = fma(-b[i], b[i], bb);
        }
        const double rho = aa > 0.0 ? sqrt(aa) : 0.0;
        const double gam = rho > 0.0 ? ab / rho : 0.0;
        const double del = rho > 0.0 ? gam / rho : 0.0;
        double nn = fma(-gam, gam, bb);
        nn = nn > 0.0 ? nn : 0.0;
        const double nu = sqrt(nn);
        double *cf = out + nq;
        for (int i = 0; i < j; ++i) {
            cf[i] = a[i];
            cf[j + i] = fma(-del, a[i], b[i]);
        }
        cf[2 * j] = rho > 0.0 ? 1.0 / rho : 0.0;
        cf[2 * j + 1] = del;
        cf[2 * j + 2] = nu > 0.0 ? 1.0 / nu : 0.0;
        cf[2 * j + 3] = rho;
        cf[2 * j + 4] = gam;
        cf[2 * j + 5] = nu;
    }
}

// y = a * b pointwise (point-Jacobi preconditioning of a Krylov vector).
__global__ __launch_bounds__(VT) void k_hadamard(double *y, const double *a, const double *b, int64_t n)
{
    const int64_t t_end = min(n, (int64_t)(blockIdx.x + 1) * CHUNK);
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x; t < t_end; t += VT) y[t] = a[t] * b[t];
}

// ------------------------------------------------------------------ two-level Schwarz
// Per element, the eight weighted sums against the trilinear corner functions (used at
// setup for the Galerkin products P_e^T A_e P_e from probe vectors; the restriction
// P^T r of an application is formed inside the local-solve kernel).
__global__ __launch_bounds__(VT) void k_corner(CornerArgs A)
{
    __shared__ double sh[8][VT / 64];
    const int64_t e = blockIdx.x;
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
    for (int p = threadIdx.x; p < A.lx3; p += VT) {
        const int64_t t = e * A.lx3 + p;
        const double x = (A.owner && !A.owner[t]) ? 0.0 : A.v[t];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = fma(A.phi[c * A.lx3 + p], x, acc[c]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        double x = acc[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) sh[c][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double x = 0.0;
#pragma unroll
        for (int q = 0; q < VT / 64; ++q) x += sh[threadIdx.x][q];
        A.out[e * 8 + threadIdx.x] = x;
    }
}

// Sum of the nblk per-workgroup partials in one fixed order, returned to every lane
// of the workgroup.  Each workgroup of a launch computes the same value, so a
// kernel can use a grid-wide reduction of the previous launch without a separate
// scalar kernel (the coarse system has only a few hundred partials).
__device__ __forceinline__ double all_sum(const double *part, int64_t nblk, double *sh)
{
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < nblk; q += VT) s += part[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double v = sh[0];
#pragma unroll
    for (int q = 1; q < VT / 64; ++q) v += sh[q];
    __syncthreads();
    return v;
}

__device__ __forceinline__ void block_partial(double v, double *out, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < VT / 64; ++q) s += sh[q];
        *out = s;
    }
}

// Coarse Jacobi-CG, start: b gathered from the restriction sums; x = 0, r = b,
// z = D r; partial of (r, z) into slot 0.
__global__ __launch_bounds__(VT) void k_ccg_start(CoarseArgs A)
{
    __shared__ double sh[VT / 64];
    const int64_t v = (int64_t)blockIdx.x * VT + threadIdx.x;
    double rz = 0.0;
    if (v < A.nv) {
        double b = 0.0;
        if (!A.vdir[v])
            for (int64_t q = A.vptr[v]; q < A.vptr[v + 1]; ++q) b += A.part[A.vidx[q]];
        const double zv = A.dinv[v] * b;
        A.x[v] = 0.0;
        A.r[v] = b;
        A.z[v] = zv;
        rz = b * zv;
    }
    block_partial(rz, A.partial + blockIdx.x, sh);
}

// Step it, first half: beta from the two latest (r, z) sums (it > 0), the new
// direction p = z + beta p_old formed for the own row and, on the fly, for every
// column the row touches; q = A p; partial of (p, q) into slot 2.  p alternates
// between p0 (even steps) and p1 (odd steps).  SPL lanes share a row (entries
// w = part, part + SPL, ...; summed across the lanes in a fixed order), so a row's
// gathers are split over SPL lanes; the grid is SPL times that of the other kernels
// (g, the row-per-lane grid, passed in).
#ifndef SEM_CCG_SPL
#define SEM_CCG_SPL 4
#endif
constexpr int SPL = SEM_CCG_SPL;
__global__ __launch_bounds__(VT) void k_ccg_spmv(CoarseArgs A, int it, int64_t g)
{
    __shared__ double sh[VT / 64];
    double beta = 0.0;
    if (it > 0) {
        const double rz = all_sum(A.partial + (it & 1) * g, g, sh);
        const double rz_old = all_sum(A.partial + ((it + 1) & 1) * g, g, sh);
        beta = (rz_old != 0.0) ? rz / rz_old : 0.0;
    }
    double *pn = (it & 1) ? A.p1 : A.p0;
    const double *po = (it & 1) ? A.p0 : A.p1;
    const int part = threadIdx.x % SPL;
    const int64_t v = ((int64_t)blockIdx.x * VT + threadIdx.x) / SPL;
    double pq = 0.0;
    if (v < A.nv) {
        double s = 0.0;
        for (int w = part; w < A.width; w += SPL) {
            const int64_t k = (int64_t)w * A.nv + v;
            const int32_t c = A.ci[k];
            const double pc = (it > 0) ? fma(beta, po[c], A.z[c]) : A.z[c];
            s = fma(A.val[k], pc, s);
        }
#pragma unroll
        for (int off = 1; off < SPL; off <<= 1) s += __shfl_xor(s, off, 64);
        if (part == 0) {
            const double pv = (it > 0) ? fma(beta, po[v], A.z[v]) : A.z[v];
            pn[v] = pv;
            A.q[v] = s;
            pq = pv * s;
        }
    }
    block_partial(pq, A.partial + 2 * g + blockIdx.x, sh);
}

// Step it, second half: alpha = (r, z) / (p, q); x += alpha p, r -= alpha q,
// z = D r; partial of the new (r, z) into the other slot.
__global__ __launch_bounds__(VT) void k_ccg_update(CoarseArgs A, int it)
{
    __shared__ double sh[VT / 64];
    const int64_t g = gridDim.x;
    const double rz = all_sum(A.partial + (it & 1) * g, g, sh);
    const double pq = all_sum(A.partial + 2 * g, SPL * g, sh);
    const double alpha = (pq > 0.0 && isfinite(pq)) ? rz / pq : 0.0;
    const double *pn = (it & 1) ? A.p1 : A.p0;
    const int64_t v = (int64_t)blockIdx.x * VT + threadIdx.x;
    double rzn = 0.0;
    if (v < A.nv) {
        A.x[v] = fma(alpha, pn[v], A.x[v]);
        const double rv = fma(-alpha, A.q[v], A.r[v]);
        A.r[v] = rv;
        const double zv = A.dinv[v] * rv;
        A.z[v] = zv;
        rzn = rv * zv;
    }
    block_partial(rzn, A.partial + ((it + 1) & 1) * g + blockIdx.x, sh);
}

// Per element, the sums over its points of G_dd / B for d = r, s, t (the local
// solves' element lengths), in a fixed order: out[e][d].
__global__ __launch_bounds__(VT) void k_elem_gb(const double *G, const double *B, double *out, int64_t n, int lx3)
{
    __shared__ double sh[3][VT / 64];
    const int64_t e = blockIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < lx3; p += VT) {
        const int64_t t = e * lx3 + p;
        const double b = B[t];
#pragma unroll
        for (int d = 0; d < 3; ++d) s[d] += G[d * n + t] / b;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double x = s[d];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) sh[d][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double x = 0.0;
#pragma unroll
        for (int q = 0; q < VT / 64; ++q) x += sh[threadIdx.x][q];
        out[e * 3 + threadIdx.x] = x;
    }
}

// Probe vector for the Galerkin coarse matrix: v[e][p] = phi[c][p] in every element.
__global__ __launch_bounds__(VT) void k_probe(double *v, const double *phi, int c, int64_t nelv, int lx3)
{
    const int64_t t = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (t >= nelv * lx3) return;
    v[t] = phi[c * lx3 + (int)(t % lx3)];
}

// STREAM triad a = b + s c (bandwidth micro-benchmark).
__global__ __launch_bounds__(VT) void k_triad(double *__restrict__ a, const double *__restrict__ b,
                                              const double *__restrict__ c, double s, int64_t n)
{
    const int64_t t_end = min(n, (int64_t)(blockIdx.x + 1) * CHUNK);
#pragma unroll
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x; t < t_end; t += VT) a[t] = fma(s, c[t], b[t]);
}

// u[idx] = 0 for every listed index, each field.
template <typename T>
__global__ __launch_bounds__(VT) void k_mask(T *u, const int32_t *idx, int64_t m, int64_t n, int nfields)
{
    const int64_t t = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (t >= m) return;
    for (int f = 0; f < nfields; ++f) u[f * n + idx[t]] = T(0);
}

template <typename T>
__global__ __launch_bounds__(VT) void k_fill(T *u, T v, int64_t m)
{
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min((int64_t)(m), (int64_t)(blockIdx.x + 1) * CHUNK); t < t_end; t += VT)
        u[t] = v;
}

// dst = (TD)(scale * src)
template <typename TD, typename TS>
__global__ __launch_bounds__(VT) void k_cast(TD *dst, const TS *src, double scale, int64_t m)
{
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min((int64_t)(m), (int64_t)(blockIdx.x + 1) * CHUNK); t < t_end; t += VT)
        dst[t] = (TD)(scale * (double)src[t]);
}

// ------------------------------------------------------------------ Jacobi inverse
// dinv = 1/d (d already summed over copies), 0 on Dirichlet points.
__global__ __launch_bounds__(VT) void k_invert(double *d, const uint8_t *dir, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * VT + threadIdx.x;
    if (t >= n) return;
    d[t] = (dir && dir[t]) ? 0.0 : 1.0 / d[t];
}

// ------------------------------------------------------------------ CG kernels
// Initial residual: r = b - w (w = QQ^T A_L x0), zero where dinv == 0 (Dirichlet);
// p = 0; partials of (r, dinv r), (r, r), (b, b) over owned points.
template <typename T>
__global__ __launch_bounds__(VT) void k_cg_init(CgInitArgs<T> A)
{
    __shared__ double sh[3][VT];
    const int f = blockIdx.y;
    const T *b = A.b + f * A.n;
    const T *w = A.w ? A.w + f * A.n : nullptr;
    T *r = A.r + f * A.n;
    T *p = A.p + f * A.n;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min((int64_t)(A.n), (int64_t)(blockIdx.x + 1) * CHUNK); t < t_end; t += VT) {
        const T di = A.dinv[t];
        const T bi = b[t];
        const T ri = (di != T(0)) ? (w ? bi - w[t] : bi) : T(0);
        r[t] = ri;
        p[t] = T(0);
        if (A.owner[t]) {
            rz += (double)ri * (double)(di * ri);
            rr += (double)ri * (double)ri;
            bb += (double)bi * (double)bi;
        }
    }
    sh[0][threadIdx.x] = rz;
    sh[1][threadIdx.x] = rr;
    sh[2][threadIdx.x] = bb;
    __syncthreads();
    for (int s = VT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) A.partial[((int64_t)q * A.nfields + f) * gridDim.x + blockIdx.x] = sh[q][0];
}

// Finish the initial reductions: rz, rr, bb; beta = 0; stop at once when b = 0
// or the initial guess already meets the tolerance.
__global__ __launch_bounds__(RT) void k_cg_start(CgFinishArgs A)
{
    __shared__ double sh[RT];
    for (int f = 0; f < A.nfields; ++f) {
        const double rz = block_sum_fixed<RT>(A.partial + (0 * A.nfields + f) * A.nblk, A.nblk, sh);
        const double rr = block_sum_fixed<RT>(A.partial + (1 * A.nfields + f) * A.nblk, A.nblk, sh);
        const double bb = block_sum_fixed<RT>(A.partial + (2 * A.nfields + f) * A.nblk, A.nblk, sh);
        if (threadIdx.x == 0) {
            CgScalars &s = A.scal[f];
            s.rz = rz;
            s.rr = rr;
            s.bb = bb;
            s.beta = 0.0;
            s.alpha = 0.0;
            s.iter = 0;
            s.status = 0;
            s.stop = 0;
            const double rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
            if (A.hist) A.hist[(int64_t)f * A.hist_len] = rel;
            if (!isfinite(bb) || !isfinite(rr) || !isfinite(rz)) { s.stop = 1; s.status = 2; }
            else if (bb == 0.0 || (s.rtol > 0.0 && rel <= s.rtol)) s.stop = 1;
            else if (s.max_iter <= 0) { s.stop = 1; s.status = 1; }
        }
    }
}

// x += alpha p; r -= alpha w (not on Dirichlet points); partials of (r, dinv r), (r, r).
// Workgroup b streams the contiguous chunk of UV * VT points starting at b * UV * VT
// (UV per precision: see upd_chunk); its two partials are reduced by wave
// butterflies and then the four waves in order (deterministic, one barrier).
template <typename T>
__global__ __launch_bounds__(VT) void k_cg_update(CgUpdateArgs<T> A)
{
    constexpr int UV = UpdChunk<T>::UV;
    __shared__ double sh[2][VT / 64];
    const int f = blockIdx.y;
    double rz = 0.0, rr = 0.0;
    T *x = A.x + f * A.n;
    T *r = A.r + f * A.n;
    const T *p = A.p + f * A.n;
    const T *w = A.w + f * A.n;
    if constexpr (sizeof(T) == 4) {
        // FP32: the field's stop flag and step length (written by the previous
        // kernels, so not in the scalar cache) are requested together with the
        // chunk's operands, not before them (indices past the end are clamped to the
        // last point, so every load is in bounds and unconditional; those lanes store
        // and accumulate nothing).  Measured: 79 -> 67 us at 16.8M points.  (In FP64
        // the same form was slower.)
        // With several fields, launches queued after a field has stopped (its segment
        // ended between host polls) are frequent and each would still read every operand
        // of that field: there the flag is tested first (it costs one scalar-load latency
        // per workgroup, negligible against a multi-field chunk).
        if (A.nfields > 1 && A.scal[f].stop) return;
        const int stop = A.scal[f].stop;
        const T alpha = (T)A.scal[f].alpha;
        const int64_t t0 = (int64_t)blockIdx.x * UV * VT + threadIdx.x;
        T di[UV], xv[UV], pv[UV], rv[UV], wv[UV];
        uint8_t own[UV];
#pragma unroll
        for (int u = 0; u < UV; ++u) {
            const int64_t t = min(t0 + (int64_t)u * VT, A.n - 1);
            di[u] = __builtin_nontemporal_load(A.dinv + t);
            xv[u] = __builtin_nontemporal_load(x + t);
            pv[u] = __builtin_nontemporal_load(p + t);
            rv[u] = __builtin_nontemporal_load(r + t);
            wv[u] = w[t];
            own[u] = A.owner[t];
        }
        // keep the loads here (not sunk below the stop test): an empty use of each value
#pragma unroll
        for (int u = 0; u < UV; ++u)
            asm volatile("" ::"v"(di[u]), "v"(xv[u]), "v"(pv[u]), "v"(rv[u]), "v"(wv[u]), "v"((int)own[u]));
        asm volatile("" ::"s"(alpha), "s"(stop));
        if (!stop) {
#pragma unroll
            for (int u = 0; u < UV; ++u) {
                const int64_t t = t0 + (int64_t)u * VT;
                if (t >= A.n) break;
                __builtin_nontemporal_store(fma(alpha, pv[u], xv[u]), x + t);
                T ri = rv[u];
                if (di[u] != T(0)) {
                    ri = fma(-alpha, wv[u], ri);
                    __builtin_nontemporal_store(ri, r + t);
                }
                if (own[u]) {
                    rz += (double)ri * (double)(di[u] * ri);
                    rr += (double)ri * (double)ri;
                }
            }
        }
    } else {
        const CgScalars &sc = A.scal[f];
        if (!sc.stop) {
            const T alpha = (T)sc.alpha;
            const int64_t t0 = (int64_t)blockIdx.x * UV * VT;
            const int64_t t_end = min(A.n, t0 + (int64_t)UV * VT);
#pragma unroll
            for (int64_t t = t0 + threadIdx.x; t < t_end; t += VT) {
                const T di = __builtin_nontemporal_load(A.dinv + t);
                // x, p, r and dinv are streamed with non-temporal hints (x is touched
                // only here; the others are next read a whole iteration later), so that
                // the last-level cache keeps w and the gather-scatter's index lists.
                __builtin_nontemporal_store(fma(alpha, __builtin_nontemporal_load(p + t), __builtin_nontemporal_load(x + t)), x + t);
                T ri = __builtin_nontemporal_load(r + t);
                if (di != T(0)) {
                    ri = fma(-alpha, w[t], ri);
                    __builtin_nontemporal_store(ri, r + t);
                }
                if (A.owner[t]) {
                    rz += (double)ri * (double)(di * ri);
                    rr += (double)ri * (double)ri;
                }
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        rz += __shfl_xor(rz, off, 64);
        rr += __shfl_xor(rr, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wave] = rz;
        sh[1][wave] = rr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int q = 0; q < VT / 64; ++q) {
            a += sh[0][q];
            b += sh[1][q];
        }
        A.partial[((int64_t)0 * A.nfields + f) * gridDim.x + blockIdx.x] = a;
        A.partial[((int64_t)1 * A.nfields + f) * gridDim.x + blockIdx.x] = b;
    }
}

// Single-reduction CG update (Chronopoulos-Gear): with u = dinv r recomputed on the
// fly, p = u + beta p, s = w + beta s (s = A p carried as a vector), x += alpha p,
// r -= alpha s on non-Dirichlet points, and the partial sums of the new (r, dinv r)
// and (r, r) over owned points (wave butterflies, then the waves in order).  They are
// reduced together with the next matvec's (u, A u): one reduction phase per iteration.
__global__ __launch_bounds__(VT) void k_cg1_update(Cg1UpdateArgs A)
{
    __shared__ double sh[2][VT / 64];
    const int f = blockIdx.y;
    const CgScalars &sc = A.scal[f];
    double rz = 0.0, rr = 0.0;
    if (!sc.stop) {
        const double alpha = sc.alpha, beta = sc.beta;
        double *x = A.x + f * A.n;
        double *r = A.r + f * A.n;
        double *p = A.p + f * A.n;
        double *s = A.s + f * A.n;
        const double *w = A.w + f * A.n;
        const int64_t t_end = min(A.n, (int64_t)(blockIdx.x + 1) * CHUNK);
#pragma unroll
        for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x; t < t_end; t += VT) {
            // every vector but w streamed non-temporally, as in the two-reduction update
            const double di = __builtin_nontemporal_load(A.dinv + t);
            double ri = __builtin_nontemporal_load(r + t);
            const double pn = fma(beta, __builtin_nontemporal_load(p + t), di * ri);
            const double sn = fma(beta, __builtin_nontemporal_load(s + t), w[t]);
            __builtin_nontemporal_store(pn, p + t);
            __builtin_nontemporal_store(sn, s + t);
            __builtin_nontemporal_store(fma(alpha, pn, __builtin_nontemporal_load(x + t)), x + t);
            if (di != 0.0) {
                ri = fma(-alpha, sn, ri);
                __builtin_nontemporal_store(ri, r + t);
            }
            if (A.owner[t]) {
                rz += ri * (di * ri);
                rr += ri * ri;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        rz += __shfl_xor(rz, off, 64);
        rr += __shfl_xor(rr, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wave] = rz;
        sh[1][wave] = rr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int q = 0; q < VT / 64; ++q) {
            a += sh[0][q];
            b += sh[1][q];
        }
        A.partial[((int64_t)0 * A.nfields + f) * gridDim.x + blockIdx.x] = a;
        A.partial[((int64_t)1 * A.nfields + f) * gridDim.x + blockIdx.x] = b;
    }
}

// End of one CG iteration: beta = rz_new / rz_old, convergence and iteration cap.
// Two sums of nblk partials in one pass, fixed order: lane t accumulates entries
// t, t + NTH, ... of both arrays (four interleaved accumulators each, eight loads in
// flight), a butterfly per wave, then the NTH / 64 wave sums in order.  Every lane
// gets both results.
template <int NTH>
__device__ void block_sum2_fixed(const double *pa, const double *pb, int64_t nblk, double *sh, double &ra,
                                 double &rb)
{
    const int tid = threadIdx.x;
    double a[4] = {0.0, 0.0, 0.0, 0.0}, b[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t q = tid;
    for (; q + 3 * NTH < nblk; q += 4 * NTH) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] += pa[q + u * NTH];
            b[u] += pb[q + u * NTH];
        }
    }
    for (; q < nblk; q += NTH) {
        a[0] += pa[q];
        b[0] += pb[q];
    }
    double x = (a[0] + a[1]) + (a[2] + a[3]), y = (b[0] + b[1]) + (b[2] + b[3]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off, 64);
        y += __shfl_xor(y, off, 64);
    }
    if ((tid & 63) == 0) {
        sh[2 * (tid >> 6)] = x;
        sh[2 * (tid >> 6) + 1] = y;
    }
    __syncthreads();
    ra = 0.0;
    rb = 0.0;
#pragma unroll
    for (int w = 0; w < NTH / 64; ++w) {
        ra += sh[2 * w];
        rb += sh[2 * w + 1];
    }
    __syncthreads();
}

__global__ __launch_bounds__(RT) void k_cg_finish(CgFinishArgs A)
{
    __shared__ double sh[2 * (RT / 64)];
    for (int f = 0; f < A.nfields; ++f) {
        double rz, rr;
        block_sum2_fixed<RT>(A.partial + (0 * A.nfields + f) * A.nblk, A.partial + (1 * A.nfields + f) * A.nblk,
                             A.nblk, sh, rz, rr);
        if (threadIdx.x == 0) {
            CgScalars &s = A.scal[f];
            if (!s.stop) {
                s.iter += 1;
                s.rr = rr;
                const double rel = sqrt(rr / s.bb);
                if (A.hist && s.iter < A.hist_len) A.hist[(int64_t)f * A.hist_len + s.iter] = rel;
                s.beta = rz / s.rz;
                s.rz = rz;
                if (s.rtol > 0.0 && rel <= s.rtol) s.stop = 1;
                else if (!isfinite(rr) || !isfinite(rz)) { s.stop = 1; s.status = 2; }
                else if (rz == 0.0) s.stop = 1;
                else if (s.iter >= s.max_iter) { s.stop = 1; s.status = (s.rtol > 0.0) ? 1 : 0; }
            }
        }
    }
}

// ------------------------------------------------------------------ reliable-update mixed CG
// Restart data for a new FP32 segment from the FP64 true residual r64.
__global__ __launch_bounds__(VT) void k_rel_restart(RelRestartArgs A)
{
    __shared__ double sh[3][VT];
    const int f = blockIdx.y;
    double rz = 0.0, rr = 0.0, r64 = 0.0;
    if (!A.rel[f].done) {
        const double *rs = A.r64 + f * A.n;
        float *r = A.r32 + f * A.n;
        float *x = A.x32 + f * A.n;
        float *p = A.p32 ? A.p32 + f * A.n : nullptr;
        for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min(A.n, (int64_t)(blockIdx.x + 1) * CHUNK);
             t < t_end; t += VT) {
            const double rd = rs[t];
            const float ri = (float)rd;
            r[t] = ri;
            x[t] = 0.0f;
            if (p) p[t] = 0.0f;
            if (A.owner[t]) {
                rz += (double)ri * (double)(A.dinv32[t] * ri);
                rr += (double)ri * (double)ri;
                r64 += rd * rd;
            }
        }
    }
    sh[0][threadIdx.x] = rz;
    sh[1][threadIdx.x] = rr;
    sh[2][threadIdx.x] = r64;
    __syncthreads();
    for (int s = VT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) A.partial[((int64_t)q * A.nfields + f) * gridDim.x + blockIdx.x] = sh[q][0];
}

// Start (first = 1) or resume an FP32 segment after a residual replacement.  The
// FP64 true residual decides convergence.  Resuming keeps the search direction p:
// beta is rescaled to the replaced residual, beta = (r_new, z_new) / (r_old, z_old).
// The segment stops once its residual has dropped by max(delta, half of the
// reduction still needed), at most 0.5.
__global__ __launch_bounds__(RT) void k_rel_resume(CgFinishArgs F, RelState *rel, int first)
{
    __shared__ double sh[RT];
    for (int f = 0; f < F.nfields; ++f) {
        const double rz = block_sum_fixed<RT>(F.partial + (0 * F.nfields + f) * F.nblk, F.nblk, sh);
        const double rr = block_sum_fixed<RT>(F.partial + (1 * F.nfields + f) * F.nblk, F.nblk, sh);
        const double r64 = block_sum_fixed<RT>(F.partial + (2 * F.nfields + f) * F.nblk, F.nblk, sh);
        if (threadIdx.x == 0) {
            RelState &R = rel[f];
            CgScalars &s = F.scal[f];
            if (R.done) continue;
            R.rr64 = r64;
            R.outer += first ? 0 : 1;
            // the segment that just ended failed (breakdown) or used up the iterations
            if (!first && s.status != 0) {
                R.done = 1;
                s.stop = 1;
                continue;
            }
            const double rel64 = R.bb64 > 0.0 ? sqrt(r64 / R.bb64) : 0.0;
            if (!isfinite(r64) || !isfinite(rz)) {
                R.done = 1;
                s.stop = 1;
                s.status = 2;
                continue;
            }
            if (R.bb64 == 0.0 || rel64 <= R.tol) {
                R.done = 1;
                s.stop = 1;
                s.status = 0;
                continue;
            }
            if (first) {
                s.beta = 0.0;
                s.iter = 0;
            } else {
                s.beta = (s.rz != 0.0) ? s.beta * (rz / s.rz) : 0.0;
                // a fast-converging system reaches delta within a few iterations:
                // ask for more reduction per segment so replacements stay rare
                if (s.iter - R.last_iter < 8) R.delta = fmax(R.delta * R.delta, 1e-3);
            }
            R.last_iter = s.iter;
            s.rz = rz;
            s.rr = rr;
            s.bb = rr;  // the segment's reference residual
            const double need = R.tol / rel64;
            s.rtol = fmin(0.5, fmax(R.delta, 0.5 * need));
            s.alpha = 0.0;
            s.status = 0;
            s.stop = 0;
            if (s.iter >= s.max_iter) {
                s.stop = 1;
                s.status = 1;
                R.done = 1;
            }
        }
    }
}

// Residual replacement for a CG in precision T: partials of (r, dinv r) and (r, r)
// for a freshly recomputed residual r, on fields flagged in `redo`.
template <typename T>
__global__ __launch_bounds__(VT) void k_cg_replace(const T *r_all, const T *dinv, const uint8_t *owner,
                                                   const int *redo, double *partial, int64_t n, int nfields)
{
    __shared__ double sh[2][VT];
    const int f = blockIdx.y;
    double rz = 0.0, rr = 0.0;
    if (redo[f]) {
        const T *r = r_all + f * n;
        for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min(n, (int64_t)(blockIdx.x + 1) * CHUNK);
             t < t_end; t += VT) {
            if (owner[t]) {
                const T ri = r[t];
                rz += (double)ri * (double)(dinv[t] * ri);
                rr += (double)ri * (double)ri;
            }
        }
    }
    sh[0][threadIdx.x] = rz;
    sh[1][threadIdx.x] = rr;
    __syncthreads();
    for (int s = VT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 2; ++q) partial[((int64_t)q * nfields + f) * gridDim.x + blockIdx.x] = sh[q][0];
}

// Resume the CG of the fields flagged in `redo` after their residual was replaced:
// beta rescaled to the replaced residual, recursive norms reset, iteration continues
// (unless the iteration cap is reached).
__global__ __launch_bounds__(RT) void k_cg_resume(CgFinishArgs F, const int *redo)
{
    __shared__ double sh[RT];
    for (int f = 0; f < F.nfields; ++f) {
        const double rz = block_sum_fixed<RT>(F.partial + (0 * F.nfields + f) * F.nblk, F.nblk, sh);
        const double rr = block_sum_fixed<RT>(F.partial + (1 * F.nfields + f) * F.nblk, F.nblk, sh);
        if (threadIdx.x == 0 && redo[f]) {
            CgScalars &s = F.scal[f];
            s.beta = (s.rz != 0.0) ? s.beta * (rz / s.rz) : 0.0;
            s.rz = rz;
            s.rr = rr;
            if (!isfinite(rz) || !isfinite(rr)) {
                s.stop = 1;
                s.status = 2;
            } else if (s.iter >= s.max_iter) {
                s.stop = 1;
                s.status = 1;
            } else {
                s.stop = 0;
                s.status = 0;
            }
        }
    }
}

// x64 += (double) x32 on fields not done before this segment (done_before[f] == 0).
__global__ __launch_bounds__(VT) void k_add_f32(double *x64, const float *x32, const int *skip, int64_t n)
{
    const int f = blockIdx.y;
    if (skip[f]) return;
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min(n, (int64_t)(blockIdx.x + 1) * CHUNK);
         t < t_end; t += VT)
        x64[f * n + t] += (double)x32[f * n + t];
}

// ------------------------------------------------------------------ generic dots
// partial[q][f][block] for q in 0..nd-1: sum over owned points of a_q * b_q (FP64).
__global__ __launch_bounds__(VT) void k_dots(DotArgs A)
{
    __shared__ double sh[4][VT];
    const int f = blockIdx.y;
    double acc[4] = {0, 0, 0, 0};
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min((int64_t)(A.n), (int64_t)(blockIdx.x + 1) * CHUNK); t < t_end; t += VT) {
        if (!A.owner[t]) continue;
        for (int q = 0; q < A.nd; ++q) acc[q] += A.a[q][f * A.n + t] * A.b[q][f * A.n + t];
    }
    for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = VT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < A.nd; ++q)
            A.partial[((int64_t)q * A.nfields + f) * gridDim.x + blockIdx.x] = sh[q][0];
}

// out[q*nfields + f] = sum of partials, fixed order.
__global__ __launch_bounds__(RT) void k_dots_finish(const double *partial, int64_t nblk, int nq,
                                                     double *out)
{
    __shared__ double sh[RT];
    for (int q = 0; q < nq; ++q) {
        const double s = block_sum_fixed<RT>(partial + q * nblk, nblk, sh);
        if (threadIdx.x == 0) out[q] = s;
    }
}

// r = b - w masked (dinv == 0 marks Dirichlet points); used for true residuals.
__global__ __launch_bounds__(VT) void k_residual(double *r, const double *b, const double *w,
                                                 const double *dinv, int64_t n, int nfields)
{
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min((int64_t)(n), (int64_t)(blockIdx.x + 1) * CHUNK); t < t_end; t += VT) {
        const double di = dinv[t];
        for (int f = 0; f < nfields; ++f)
            r[f * n + t] = (di != 0.0) ? b[f * n + t] - w[f * n + t] : 0.0;
    }
}

// ------------------------------------------------------------------ flexible CG (outer, FP64)
// p = z - beta_f p   (beta_f from coef[f]);  fields with coef[f] flagged done are left alone.
__global__ __launch_bounds__(VT) void k_fcg_dir(double *p, const double *z, const double *beta,
                                                const int *done, int64_t n, int nfields)
{
    const int f = blockIdx.y;
    if (done[f]) return;
    const double bf = beta[f];
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min((int64_t)(n), (int64_t)(blockIdx.x + 1) * CHUNK); t < t_end; t += VT)
        p[f * n + t] = z[f * n + t] - bf * p[f * n + t];
}

// x += alpha p; r -= alpha q (not on Dirichlet points).
__global__ __launch_bounds__(VT) void k_fcg_update(double *x, double *r, const double *p,
                                                   const double *q, const double *dinv,
                                                   const double *alpha, const int *done, int64_t n,
                                                   int nfields)
{
    const int f = blockIdx.y;
    if (done[f]) return;
    const double a = alpha[f];
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min((int64_t)(n), (int64_t)(blockIdx.x + 1) * CHUNK); t < t_end; t += VT) {
        x[f * n + t] = fma(a, p[f * n + t], x[f * n + t]);
        if (dinv[t] != 0.0) r[f * n + t] = fma(-a, q[f * n + t], r[f * n + t]);
    }
}

// r32 = (float)(r / |r|_f)  per field (fields flagged done get 0).
__global__ __launch_bounds__(VT) void k_fcg_scale_down(float *r32, const double *r,
                                                       const double *inv_norm, const int *done,
                                                       int64_t n, int nfields)
{
    const int f = blockIdx.y;
    const double s = done[f] ? 0.0 : inv_norm[f];
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min((int64_t)(n), (int64_t)(blockIdx.x + 1) * CHUNK); t < t_end; t += VT)
        r32[f * n + t] = (float)(s * r[f * n + t]);
}

// z = |r|_f * (double) y32
__global__ __launch_bounds__(VT) void k_fcg_scale_up(double *z, const float *y32, const double *norm,
                                                     int64_t n, int nfields)
{
    const int f = blockIdx.y;
    const double s = norm[f];
    for (int64_t t = (int64_t)blockIdx.x * CHUNK + threadIdx.x, t_end = min((int64_t)(n), (int64_t)(blockIdx.x + 1) * CHUNK); t < t_end; t += VT)
        z[f * n + t] = s * (double)y32[f * n + t];
}

}  // namespace sem

// ------------------------------------------------------------------ host launchers
using namespace sem;

static unsigned stream_grid(int64_t n)
{
    const int64_t g = (n + CHUNK - 1) / CHUNK;
    return (unsigned)(g < 1 ? 1 : g);
}

static unsigned gs_grid(int64_t work)
{
    int64_t g = (work + VT - 1) / VT;
    if (g < 1) g = 1;
    return (unsigned)(8 * ((g + 7) / 8));  // multiple of 8: see the XCD mapping in k_gs
}

extern "C" {

unsigned sem_vec_grid(int64_t n) { return stream_grid(n); }
// workgroups of the CG update in precision f32 ? FP32 : FP64
unsigned sem_update_grid(int64_t n, int f32)
{
    const int64_t c = (int64_t)VT * (f32 ? UpdChunk<float>::UV : UpdChunk<double>::UV);
    const int64_t g = (n + c - 1) / c;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // extern "C"

// Entry-parallel kernel for groups of up to 64 copies, then (rarely) the per-group
// kernel for larger groups.  The step-length fold runs in the first launch only.
template <typename T>
static hipError_t launch_gs_t(const GsArgs<T> *A, hipStream_t st)
{
    if (A->nent > 0) {
        hipLaunchKernelGGL(k_gs_entries<T>, dim3(gs_grid((A->nent + GEPL - 1) / GEPL)), dim3(VT), 0, st, *A);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || A->npairs + A->nblocks == 0) return e;
        GsArgs<T> B = *A;
        B.alpha_job = nullptr;
        hipLaunchKernelGGL(k_gs<T>, dim3(gs_grid(B.npairs + B.nblocks)), dim3(VT), 0, st, B);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_gs<T>, dim3(gs_grid(A->npairs + A->nblocks)), dim3(VT), 0, st, *A);
    return hipGetLastError();
}
// Workgroups of the Arnoldi passes: contiguous chunks of whole 256-point rows, at
// most 1024 workgroups (four per CU), so the partial rows stay short.
static int64_t arn_chunk(int64_t n)
{
    const int64_t rows = (n + VT - 1) / VT;
    const int64_t per = (rows + 1023) / 1024;
    return (per < 1 ? 1 : per) * VT;
}
static unsigned arn_grid(int64_t n)
{
    const int64_t c = arn_chunk(n);
    const int64_t g = (n + c - 1) / c;
    return (unsigned)(g < 1 ? 1 : g);
}
template <int MV>
static void launch_dcgs(const DcgsArgs &A, int pass, hipStream_t st)
{
    const unsigned g = arn_grid(A.n);
    const int64_t c = arn_chunk(A.n);
    if (pass == 0) hipLaunchKernelGGL((k_dcgs_dots<MV>), dim3(g), dim3(VT), 0, st, A, c);
    else hipLaunchKernelGGL((k_dcgs_update<MV>), dim3(g), dim3(VT), 0, st, A, c);
}
template <int MV>
static void launch_arn(const ArnArgs &A, int mode, hipStream_t st)
{
    const unsigned g = arn_grid(A.n);
    const int64_t c = arn_chunk(A.n);
    if (mode == 0) hipLaunchKernelGGL((k_arn<MV, 0>), dim3(g), dim3(VT), 0, st, A, c);
    else if (mode == 1) hipLaunchKernelGGL((k_arn<MV, 1>), dim3(g), dim3(VT), 0, st, A, c);
    else hipLaunchKernelGGL((k_arn<MV, 2>), dim3(g), dim3(VT), 0, st, A, c);
}
extern "C" {
hipError_t sem_launch_gs_f64(const GsArgs<double> *A, hipStream_t st) { return launch_gs_t<double>(A, st); }
hipError_t sem_launch_gs_f32(const GsArgs<float> *A, hipStream_t st) { return launch_gs_t<float>(A, st); }
hipError_t sem_launch_mask(void *u, int is_f32, const int32_t *idx, int64_t m, int64_t n, int nfields,
                           hipStream_t st)
{
    if (m == 0) return hipSuccess;
    const unsigned grid = (unsigned)((m + VT - 1) / VT);
    if (is_f32)
        hipLaunchKernelGGL(k_mask<float>, dim3(grid), dim3(VT), 0, st, (float *)u, idx, m, n, nfields);
    else
        hipLaunchKernelGGL(k_mask<double>, dim3(grid), dim3(VT), 0, st, (double *)u, idx, m, n, nfields);
    return hipGetLastError();
}
hipError_t sem_launch_fill_f64(double *u, double v, int64_t m, hipStream_t st)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<double>, dim3(stream_grid(m)), dim3(VT), 0, st, u, v, m);
    return hipGetLastError();
}
hipError_t sem_launch_fill_f32(float *u, float v, int64_t m, hipStream_t st)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<float>, dim3(stream_grid(m)), dim3(VT), 0, st, u, v, m);
    return hipGetLastError();
}
hipError_t sem_launch_cast_f32_f64(float *dst, const double *src, double scale, int64_t m, hipStream_t st)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL((k_cast<float, double>), dim3(stream_grid(m)), dim3(VT), 0, st, dst, src, scale, m);
    return hipGetLastError();
}
hipError_t sem_launch_triad(double *a, const double *b, const double *c, double s, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_triad, dim3(stream_grid(n)), dim3(VT), 0, st, a, b, c, s, n);
    return hipGetLastError();
}
hipError_t sem_launch_invert(double *d, const uint8_t *dir, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_invert, dim3((unsigned)((n + VT - 1) / VT)), dim3(VT), 0, st, d, dir, n);
    return hipGetLastError();
}
hipError_t sem_launch_cg_init_f64(const CgInitArgs<double> *A, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_init<double>, dim3(grid, A->nfields), dim3(VT), 0, st, *A);
    return hipGetLastError();
}
hipError_t sem_launch_cg_init_f32(const CgInitArgs<float> *A, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_init<float>, dim3(grid, A->nfields), dim3(VT), 0, st, *A);
    return hipGetLastError();
}
hipError_t sem_launch_cg_start(const CgFinishArgs *A, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(RT), 0, st, *A);
    return hipGetLastError();
}
hipError_t sem_launch_cg_update_f64(const CgUpdateArgs<double> *A, unsigned grid, hipStream_t st)
{
    if ((int64_t)grid * VT * UpdChunk<double>::UV < A->n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cg_update<double>, dim3(grid, A->nfields), dim3(VT), 0, st, *A);
    return hipGetLastError();
}
hipError_t sem_launch_cg_update_f32(const CgUpdateArgs<float> *A, unsigned grid, hipStream_t st)
{
    if ((int64_t)grid * VT * UpdChunk<float>::UV < A->n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cg_update<float>, dim3(grid, A->nfields), dim3(VT), 0, st, *A);
    return hipGetLastError();
}
hipError_t sem_launch_cg1_update(const Cg1UpdateArgs *A, hipStream_t st)
{
    if (A->n == 0) return hipSuccess;
    if (!A->owner || !A->partial) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cg1_update, dim3(stream_grid(A->n), A->nfields), dim3(VT), 0, st, *A);
    return hipGetLastError();
}
hipError_t sem_launch_cg_finish(const CgFinishArgs *A, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_finish, dim3(1), dim3(RT), 0, st, *A);
    return hipGetLastError();
}
hipError_t sem_launch_rel_restart(const RelRestartArgs *A, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_rel_restart, dim3(grid, A->nfields), dim3(VT), 0, st, *A);
    return hipGetLastError();
}
hipError_t sem_launch_rel_resume(const CgFinishArgs *F, RelState *rel, int first, hipStream_t st)
{
    hipLaunchKernelGGL(k_rel_resume, dim3(1), dim3(RT), 0, st, *F, rel, first);
    return hipGetLastError();
}
hipError_t sem_launch_add_f32(double *x64, const float *x32, const int *skip, int64_t n, int nfields,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_add_f32, dim3(stream_grid(n), nfields), dim3(VT), 0, st, x64, x32, skip, n);
    return hipGetLastError();
}
hipError_t sem_launch_cg_replace_f64(const double *r, const double *dinv, const uint8_t *owner, const int *redo,
                                     double *partial, int64_t n, int nfields, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_replace<double>, dim3(stream_grid(n), nfields), dim3(VT), 0, st, r, dinv, owner, redo,
                       partial, n, nfields);
    return hipGetLastError();
}
hipError_t sem_launch_cg_resume(const CgFinishArgs *F, const int *redo, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_resume, dim3(1), dim3(RT), 0, st, *F, redo);
    return hipGetLastError();
}
hipError_t sem_launch_comb(const CombArgs *A, hipStream_t st)
{
    if (A->l < 0 || A->l > PB || A->mode < 0 || A->mode > 2) return hipErrorInvalidValue;
    if (A->n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_comb, dim3(stream_grid(A->n)), dim3(VT), 0, st, *A);
    return hipGetLastError();
}
unsigned sem_arn_grid(int64_t n) { return arn_grid(n); }
hipError_t sem_launch_dcgs(const DcgsArgs *A, int pass, hipStream_t st)
{
    if (A->j < 0 || A->j >= ARN_MAXV || pass < 0 || pass > 1 || A->n < 1) return hipErrorInvalidValue;
    if (pass == 1 && !A->coef) return hipErrorInvalidValue;
    if (A->j <= 8) launch_dcgs<8>(*A, pass, st);
    else if (A->j <= 16) launch_dcgs<16>(*A, pass, st);
    else launch_dcgs<32>(*A, pass, st);
    return hipGetLastError();
}
hipError_t sem_launch_dcgs_finish(const double *partial, int64_t nblk, int j, double *out, hipStream_t st)
{
    if (j < 0 || j >= ARN_MAXV) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dcgs_finish, dim3(1), dim3(RT), 0, st, partial, nblk, j, out);
    return hipGetLastError();
}
hipError_t sem_launch_arn(const ArnArgs *A, int mode, hipStream_t st)
{
    if (A->m < 1 || A->m > ARN_MAXV || mode < 0 || mode > 2 || A->n < 1) return hipErrorInvalidValue;
    if (mode != 0 && !A->coef) return hipErrorInvalidValue;
    if (mode == 2 && !A->scale) return hipErrorInvalidValue;
    if (A->m <= 8) launch_arn<8>(*A, mode, st);
    else if (A->m <= 16) launch_arn<16>(*A, mode, st);
    else launch_arn<32>(*A, mode, st);
    return hipGetLastError();
}
hipError_t sem_launch_arn_finish(const double *partial, int64_t nblk, int nq, int pyth, double *out, hipStream_t st)
{
    if (nq < 1 || nq > ARN_MAXV + 1 || (pyth && nq < 2)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_arn_finish, dim3(1), dim3(RT), 0, st, partial, nblk, nq, pyth, out);
    return hipGetLastError();
}
hipError_t sem_launch_hadamard(double *y, const double *a, const double *b, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hadamard, dim3(stream_grid(n)), dim3(VT), 0, st, y, a, b, n);
    return hipGetLastError();
}
hipError_t sem_launch_corner(const CornerArgs *A, hipStream_t st)
{
    if (A->nelv == 0) return hipSuccess;
    if (A->nelv > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_corner, dim3((unsigned)A->nelv), dim3(VT), 0, st, *A);
    return hipGetLastError();
}
// iters fixed-count Jacobi-CG steps on the coarse system from x = 0, two launches per
// step and no host sync; partial must hold (2 + SPL) * ceil(nv / VT) values.
// lanes per row of the coarse SpMV (the coarse partial buffer is sized by it)
int sem_coarse_split() { return SPL; }

hipError_t sem_launch_coarse_cg(const CoarseArgs *A, int iters, hipStream_t st)
{
    if (A->nv == 0) return hipSuccess;
    if (A->width < 1 || A->nv > 0x7fffffffLL * VT) return hipErrorInvalidValue;
    const unsigned g = (unsigned)((A->nv + VT - 1) / VT);
    hipLaunchKernelGGL(k_ccg_start, dim3(g), dim3(VT), 0, st, *A);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_ccg_spmv, dim3(g * SPL), dim3(VT), 0, st, *A, it, (int64_t)g);
        hipLaunchKernelGGL(k_ccg_update, dim3(g), dim3(VT), 0, st, *A, it);
    }
    return hipGetLastError();
}
hipError_t sem_launch_elem_gb(const double *G, const double *B, double *out, int64_t nelv, int lx3,
                              hipStream_t st)
{
    if (nelv == 0) return hipSuccess;
    if (nelv > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_elem_gb, dim3((unsigned)nelv), dim3(VT), 0, st, G, B, out, nelv * lx3, lx3);
    return hipGetLastError();
}
hipError_t sem_launch_probe(double *v, const double *phi, int c, int64_t nelv, int lx3, hipStream_t st)
{
    const int64_t n = nelv * lx3;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe, dim3((unsigned)((n + VT - 1) / VT)), dim3(VT), 0, st, v, phi, c, nelv, lx3);
    return hipGetLastError();
}
hipError_t sem_launch_dots(const DotArgs *A, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_dots, dim3(grid, A->nfields), dim3(VT), 0, st, *A);
    return hipGetLastError();
}
hipError_t sem_launch_dots_finish(const double *partial, int64_t nblk, int nq, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_dots_finish, dim3(1), dim3(RT), 0, st, partial, nblk, nq, out);
    return hipGetLastError();
}
hipError_t sem_launch_residual(double *r, const double *b, const double *w, const double *dinv,
                               int64_t n, int nfields, hipStream_t st)
{
    hipLaunchKernelGGL(k_residual, dim3(stream_grid(n)), dim3(VT), 0, st, r, b, w, dinv, n, nfields);
    return hipGetLastError();
}
hipError_t sem_launch_fcg_dir(double *p, const double *z, const double *beta, const int *done,
                              int64_t n, int nfields, hipStream_t st)
{
    hipLaunchKernelGGL(k_fcg_dir, dim3(stream_grid(n), nfields), dim3(VT), 0, st, p, z, beta, done, n, nfields);
    return hipGetLastError();
}
hipError_t sem_launch_fcg_update(double *x, double *r, const double *p, const double *q,
                                 const double *dinv, const double *alpha, const int *done,
                                 int64_t n, int nfields, hipStream_t st)
{
    hipLaunchKernelGGL(k_fcg_update, dim3(stream_grid(n), nfields), dim3(VT), 0, st, x, r, p, q, dinv,
                       alpha, done, n, nfields);
    return hipGetLastError();
}
hipError_t sem_launch_fcg_scale_down(float *r32, const double *r, const double *inv_norm,
                                     const int *done, int64_t n, int nfields, hipStream_t st)
{
    hipLaunchKernelGGL(k_fcg_scale_down, dim3(stream_grid(n), nfields), dim3(VT), 0, st, r32, r,
                       inv_norm, done, n, nfields);
    return hipGetLastError();
}
hipError_t sem_launch_fcg_scale_up(double *z, const float *y32, const double *norm, int64_t n,
                                   int nfields, hipStream_t st)
{
    hipLaunchKernelGGL(k_fcg_scale_up, dim3(stream_grid(n), nfields), dim3(VT), 0, st, z, y32, norm,
                       n, nfields);
    return hipGetLastError();
}

}  // extern "C"
