// sem_internal.h -- declarations shared by the translation units of libsem's C ABI
// (sem_api.cpp: handles and operators; sem_cg.cpp: the CG solvers; sem_proj.cpp: the
// projection space; sem_gmres.cpp: GMRES and the two-level Schwarz preconditioner):
// the handle layouts, the per-lx launcher table, error and allocation helpers, and
// the device helpers the drivers share.  Internal: include/sem.h is the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sem.h"
#include "sem_host.h"
#include "sem_kernels.h"
#include "vec_kernels.h"

// kernel argument types (sem_kernels.h, vec_kernels.h)
using namespace sem;

#ifndef SEM_GS_ELEMENT_ORDER
#define SEM_GS_ELEMENT_ORDER 0
#endif
#ifndef SEM_GS_ENTRY
#define SEM_GS_ENTRY 1
#endif

// ------------------------------------------------------------------ launcher table
#define SEM_LX_LIST(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

#define SEM_DECL(L)                                                                                     \
    extern "C" hipError_t sem_launch_ax_f64_lx##L(const AxArgs<double> *, const double *, int, hipStream_t); \
    extern "C" hipError_t sem_launch_ax_f32_lx##L(const AxArgs<float> *, const double *, int, hipStream_t);  \
    extern "C" hipError_t sem_launch_cg_f64_lx##L(const CgMatvecArgs<double> *, const double *, int,        \
                                                  hipStream_t);                                             \
    extern "C" hipError_t sem_launch_cg_f32_lx##L(const CgMatvecArgs<float> *, const double *, int,         \
                                                  hipStream_t);                                             \
    extern "C" hipError_t sem_launch_cg1_f64_lx##L(const CgMatvecArgs<double> *, const double *, int,       \
                                                   hipStream_t);                                            \
    extern "C" hipError_t sem_launch_fdm_lx##L(const FdmArgs *, hipStream_t);                               \
    extern "C" hipError_t sem_launch_prolong_lx##L(const ProlongArgs *, hipStream_t);                       \
    extern "C" hipError_t sem_launch_adj_f64_lx##L(const AdjArgs<double> *, const double *, hipStream_t);   \
    extern "C" hipError_t sem_launch_adj_f32_lx##L(const AdjArgs<float> *, const double *, hipStream_t);    \
    extern "C" hipError_t sem_launch_geom_lx##L(const GeomArgs *, const double *, const double *,           \
                                                hipStream_t);                                               \
    extern "C" hipError_t sem_launch_diag_lx##L(const DiagArgs *, const double *, hipStream_t);             \
    extern "C" int64_t sem_cg_nblocks_f64_lx##L(int64_t);                                                   \
    extern "C" int64_t sem_cg_nblocks_f32_lx##L(int64_t);                                                   \
    extern "C" void sem_deo_fill_lx##L(const double *, void *, void *);
SEM_LX_LIST(SEM_DECL)

extern "C" {
unsigned sem_vec_grid(int64_t n);
unsigned sem_update_grid(int64_t n, int f32);
hipError_t sem_launch_gs_f64(const GsArgs<double> *, hipStream_t);
hipError_t sem_launch_gs_f32(const GsArgs<float> *, hipStream_t);
hipError_t sem_launch_mask(void *, int, const int32_t *, int64_t, int64_t, int, hipStream_t);
hipError_t sem_launch_fill_f64(double *, double, int64_t, hipStream_t);
hipError_t sem_launch_fill_f32(float *, float, int64_t, hipStream_t);
hipError_t sem_launch_cast_f32_f64(float *, const double *, double, int64_t, hipStream_t);
hipError_t sem_launch_invert(double *, const uint8_t *, int64_t, hipStream_t);
hipError_t sem_launch_triad(double *, const double *, const double *, double, int64_t, hipStream_t);
hipError_t sem_launch_cg_init_f64(const CgInitArgs<double> *, unsigned, hipStream_t);
hipError_t sem_launch_cg_init_f32(const CgInitArgs<float> *, unsigned, hipStream_t);
hipError_t sem_launch_cg_start(const CgFinishArgs *, hipStream_t);
hipError_t sem_launch_cg_update_f64(const CgUpdateArgs<double> *, unsigned, hipStream_t);
hipError_t sem_launch_cg_update_f32(const CgUpdateArgs<float> *, unsigned, hipStream_t);
hipError_t sem_launch_cg_finish(const CgFinishArgs *, hipStream_t);
hipError_t sem_launch_cg1_update(const Cg1UpdateArgs *, hipStream_t);
hipError_t sem_launch_dots(const DotArgs *, unsigned, hipStream_t);
hipError_t sem_launch_rel_restart(const RelRestartArgs *, unsigned, hipStream_t);
hipError_t sem_launch_cg_replace_f64(const double *, const double *, const uint8_t *, const int *, double *, int64_t,
                                     int, hipStream_t);
hipError_t sem_launch_cg_resume(const CgFinishArgs *, const int *, hipStream_t);
hipError_t sem_launch_rel_resume(const CgFinishArgs *, RelState *, int, hipStream_t);
hipError_t sem_launch_add_f32(double *, const float *, const int *, int64_t, int, hipStream_t);
hipError_t sem_launch_dots_finish(const double *, int64_t, int, double *, hipStream_t);
hipError_t sem_launch_comb(const CombArgs *, hipStream_t);
hipError_t sem_launch_hadamard(double *, const double *, const double *, int64_t, hipStream_t);
unsigned sem_arn_grid(int64_t n);
hipError_t sem_launch_dcgs(const DcgsArgs *, int, hipStream_t);
hipError_t sem_launch_dcgs_finish(const double *, int64_t, int, double *, hipStream_t);
hipError_t sem_launch_arn(const ArnArgs *, int, hipStream_t);
hipError_t sem_launch_arn_finish(const double *, int64_t, int, int, double *, hipStream_t);
hipError_t sem_launch_corner(const CornerArgs *, hipStream_t);
hipError_t sem_launch_coarse_cg(const CoarseArgs *, int, hipStream_t);
int sem_coarse_split();
hipError_t sem_launch_elem_gb(const double *, const double *, double *, int64_t, int, hipStream_t);
hipError_t sem_launch_probe(double *, const double *, int, int64_t, int, hipStream_t);
hipError_t sem_launch_residual(double *, const double *, const double *, const double *, int64_t, int,
                               hipStream_t);
hipError_t sem_launch_fcg_dir(double *, const double *, const double *, const int *, int64_t, int,
                              hipStream_t);
hipError_t sem_launch_fcg_update(double *, double *, const double *, const double *, const double *,
                                 const double *, const int *, int64_t, int, hipStream_t);
hipError_t sem_launch_fcg_scale_down(float *, const double *, const double *, const int *, int64_t, int,
                                     hipStream_t);
hipError_t sem_launch_fcg_scale_up(double *, const float *, const double *, int64_t, int, hipStream_t);
}

namespace __attribute__((visibility("hidden"))) semi {

struct LxFns {
    hipError_t (*ax64)(const AxArgs<double> *, const double *, int, hipStream_t);
    hipError_t (*ax32)(const AxArgs<float> *, const double *, int, hipStream_t);
    hipError_t (*cg64)(const CgMatvecArgs<double> *, const double *, int, hipStream_t);
    hipError_t (*cg32)(const CgMatvecArgs<float> *, const double *, int, hipStream_t);
    hipError_t (*cg1)(const CgMatvecArgs<double> *, const double *, int, hipStream_t);
    hipError_t (*fdm)(const FdmArgs *, hipStream_t);
    hipError_t (*prolong)(const ProlongArgs *, hipStream_t);
    hipError_t (*adj64)(const AdjArgs<double> *, const double *, hipStream_t);
    hipError_t (*adj32)(const AdjArgs<float> *, const double *, hipStream_t);
    hipError_t (*geom)(const GeomArgs *, const double *, const double *, hipStream_t);
    hipError_t (*diag)(const DiagArgs *, const double *, hipStream_t);
    int64_t (*nblk64)(int64_t);
    int64_t (*nblk32)(int64_t);
    void (*deo)(const double *, void *, void *);
};

// launchers of the kernels instantiated for one lx
const LxFns &fns(int lx);

// records a message for sem_last_error() and returns s
sem_status fail(sem_status s, const char *fmt, ...);

#define HIP_TRY(x)                                                                                     \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess)                                                                          \
            return fail(e_ == hipErrorOutOfMemory ? SEM_ERR_OOM : SEM_ERR_HIP, "%s failed: %s (%s:%d)", \
                        #x, hipGetErrorString(e_), __FILE__, __LINE__);                                \
    } while (0)

#define SEM_TRY(x)                          \
    do {                                    \
        sem_status s_ = (x);                \
        if (s_ != SEM_OK) return s_;        \
    } while (0)

inline hipStream_t S(void *s) { return (hipStream_t)s; }

template <typename P>
sem_status dalloc(P **p, size_t count)
{
    *p = nullptr;
    if (count == 0) return SEM_OK;
    hipError_t e = hipMalloc((void **)p, count * sizeof(P));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? SEM_ERR_OOM : SEM_ERR_HIP, "hipMalloc of %zu bytes failed: %s",
                    count * sizeof(P), hipGetErrorString(e));
    }
    return SEM_OK;
}

template <typename P>
void dfree(P *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

sem_status current_device(int *dev);
bool overlap(const void *a, size_t na, const void *b, size_t nb);

}  // namespace semi

// ------------------------------------------------------------------ handle types
struct sem_space_s {
    int lx;
    double xi[SEM_LX_MAX], w[SEM_LX_MAX], D[SEM_LX_MAX * SEM_LX_MAX];
};

struct sem_mesh_s {
    int64_t nelv = 0;
    int lx = 0;
    int64_t n = 0;
    std::vector<int64_t> glb;
    std::vector<uint8_t> dir;     // empty when no Dirichlet points
    std::vector<int32_t> dir_idx; // local indices of Dirichlet points
    int64_t n_unique = -1;        // filled by the gs builder
    // device copies (uploaded lazily)
    int device = -1;
    uint8_t *d_dir = nullptr;
    int32_t *d_dir_idx = nullptr;
};

struct sem_gs_s {
    sem_mesh msh = nullptr;
    semh::GsMaps m;
    int device = -1;
    int32_t *d_pairs = nullptr;
    int64_t *d_blk_ptr = nullptr;
    int32_t *d_blk_idx = nullptr;
    uint8_t *d_owner = nullptr;
    uint32_t *d_ent_word = nullptr;  // entry-parallel list, one packed word per entry
    bool entries = false;  // entry-parallel execution (groups > 64 copies via d_blk_*)
    int64_t npairs() const { return (int64_t)m.pairs.size() / 2; }
    int64_t nblocks() const { return (int64_t)m.blk_ptr.size() - 1; }
    // work of the per-group kernel as uploaded
    int64_t dev_npairs = 0, dev_nblocks = 0;
};

namespace __attribute__((visibility("hidden"))) semi {

// Scratch owned by a coef handle, grown on demand.
struct Work {
    int64_t cap_n = 0;   // points per field the buffers hold
    int cap_f = 0;       // fields
    bool mixed = false;
    double *r = nullptr, *p = nullptr, *w = nullptr;          // CG (FP64)
    double *z = nullptr, *q = nullptr;                         // flexible CG outer
    float *r32 = nullptr, *y32 = nullptr, *p32 = nullptr, *w32 = nullptr;  // inner FP32 CG
    float *ri32 = nullptr;
    double *partial = nullptr;
    int64_t partial_len = 0;
    int64_t nb = 0;                 // partial sums per row of W.partial
    CgScalars *scal = nullptr;      // device [fields]
    CgScalars *h_scal = nullptr;    // pinned mirror
    AlphaJob *job64 = nullptr;      // device, for the FP64 matvec grid
    AlphaJob *job32 = nullptr;      // device, for the FP32 matvec grid
    AlphaJob *job_cg1 = nullptr;    // device, single-reduction CG fold (FP64 matvec grid)
    double *s = nullptr;            // single-reduction CG: s = A p (FP64), allocated on first use
    double *dots = nullptr;         // device results of k_dots_finish
    double *h_dots = nullptr;       // pinned mirror
    double *fcg = nullptr;          // device: beta[3], alpha[3], norm[3], inv_norm[3]
    double *h_fcg = nullptr;        // pinned mirror
    int *done = nullptr;            // device [3]
    int *h_done = nullptr;          // pinned mirror
    // flexible GMRES: V (m + 1 vectors), Z (m vectors), a work vector; inner products
    double *gm = nullptr;
    int gm_m = 0;
    double *gm_part = nullptr, *gm_out = nullptr, *gm_hout = nullptr;
    RelState *rel = nullptr;        // device [3], reliable-update mixed solve
    RelState *h_rel = nullptr;      // pinned mirror
    void release()
    {
        dfree(r); dfree(p); dfree(w); dfree(z); dfree(q);
        dfree(r32); dfree(y32); dfree(p32); dfree(w32); dfree(ri32);
        dfree(partial); dfree(scal); dfree(job64); dfree(job32); dfree(dots); dfree(fcg); dfree(done); dfree(rel);
        dfree(job_cg1); dfree(s);
        dfree(gm); dfree(gm_part); dfree(gm_out);
        if (gm_hout) (void)hipHostFree(gm_hout);
        gm_hout = nullptr;
        gm_m = 0;
        if (h_rel) (void)hipHostFree(h_rel);
        h_rel = nullptr;
        if (h_scal) (void)hipHostFree(h_scal);
        if (h_dots) (void)hipHostFree(h_dots);
        if (h_fcg) (void)hipHostFree(h_fcg);
        if (h_done) (void)hipHostFree(h_done);
        h_scal = nullptr; h_dots = nullptr; h_fcg = nullptr; h_done = nullptr;
        cap_n = 0; cap_f = 0; mixed = false; partial_len = 0; nb = 0;
    }
};


// Two-level additive Schwarz preconditioner data, built on first use for a (coef, gs)
// pair and dropped when the Helmholtz coefficients change.
struct SchwarzData {
    bool valid = false;
    const void *gs = nullptr;
    double *S = nullptr, *lam = nullptr;  // [nelv][3][lx][lx], [nelv][3][lx]
    double *phi = nullptr;                // [8][lx^3] (setup probes)
    double *lin = nullptr;                // [2][lx] linear functions at the GLL points
    int32_t *cvert = nullptr;             // [nelv][8]
    int64_t nv = 0;
    int64_t *v_ptr = nullptr;
    int32_t *v_idx = nullptr;
    uint8_t *v_dir = nullptr;
    int width = 0;                        // ELL row width of the coarse matrix
    int32_t *ell_ci = nullptr;            // [width][nv]
    double *ell_val = nullptr, *dinv0 = nullptr;
    double *part = nullptr;               // [nelv * 8]
    double *cv = nullptr;                 // [6][nv]: x, r, z, p0, p1, q
    double *cpart = nullptr;              // [2 + sem_coarse_split()][ceil(nv / 256)]
    uint8_t *mult = nullptr;              // [n]
    // one-point overlap (built on first use): local operators on the element box
    // extended by one point beyond each face, and the face-neighbour table
    bool ov_valid = false;
    double *S_ov = nullptr, *lam_ov = nullptr;  // [nelv][3][lx+2][lx+2], [nelv][3][lx+2]
    int32_t *face = nullptr;                    // [nelv][6][4]
    void release()
    {
        dfree(S); dfree(lam); dfree(phi); dfree(lin); dfree(cvert); dfree(v_ptr); dfree(v_idx); dfree(v_dir);
        dfree(ell_ci); dfree(ell_val); dfree(dinv0); dfree(part); dfree(cv); dfree(cpart);
        dfree(mult);
        dfree(S_ov); dfree(lam_ov); dfree(face);
        ov_valid = false;
        width = 0;
        valid = false;
        gs = nullptr;
        nv = 0;
    }
};

}  // namespace semi

struct sem_coef_s {
    sem_space Xh = nullptr;
    sem_mesh msh = nullptr;
    int lx = 0;
    int64_t n = 0, nelv = 0;
    int device = -1;
    unsigned flags = 0;
    double *G = nullptr, *B = nullptr;
    float *G32 = nullptr, *B32 = nullptr;
    double h1s = 1.0, h2s = 0.0;
    double *h1 = nullptr, *h2 = nullptr;
    float *h1_32 = nullptr, *h2_32 = nullptr;
    double *dinv = nullptr;
    float *dinv32 = nullptr;
    void *deo64 = nullptr, *deo32 = nullptr;  // device copies of the even-odd D (FP64, FP32)
    bool dinv_valid = false;
    const void *dinv_gs = nullptr;
    semi::Work ws;
    semi::SchwarzData sz;
};

namespace __attribute__((visibility("hidden"))) semi {

sem_status check_device(int want);
sem_status mesh_upload(sem_mesh m);
sem_status gs_upload(sem_gs g);
sem_status check_coef(sem_coef c, sem_mesh msh, sem_space Xh);

template <typename T>
sem_status launch_gs(T *u, int nf, sem_gs g, const CgScalars *skip, const AlphaJob *job, hipStream_t st)
{
    GsArgs<T> A;
    A.u = u;
    A.pairs = g->d_pairs;
    A.blk_ptr = g->d_blk_ptr;
    A.blk_idx = g->d_blk_idx;
    A.npairs = g->dev_npairs;
    A.nblocks = g->dev_nblocks;
    A.n = g->m.n;
    A.nfields = nf;
    A.skip = skip;
    A.alpha_job = job;
    A.ent_word = g->d_ent_word;
    A.nent = g->entries ? (int64_t)g->m.ent_idx.size() : 0;
    A.max_group = g->m.max_group;
    if (A.npairs + A.nblocks + A.nent == 0 && job == nullptr) return SEM_OK;
    hipError_t e;
    if constexpr (sizeof(T) == 8) e = sem_launch_gs_f64(&A, st);
    else e = sem_launch_gs_f32(&A, st);
    HIP_TRY(e);
    return SEM_OK;
}

template <typename T>
sem_status launch_ax(sem_coef c, T *w, const T *u, int nf, hipStream_t st)
{
    AxArgs<T> A;
    A.w = w;
    A.u = u;
    A.n = c->n;
    A.nelv = c->nelv;
    hipError_t e;
    if constexpr (sizeof(T) == 8) {
        A.G = c->G; A.B = c->B; A.h1 = c->h1; A.h2 = c->h2; A.h1s = c->h1s; A.h2s = c->h2s;
        A.deo = c->deo64;
        e = fns(c->lx).ax64(&A, c->Xh->D, nf, st);
    } else {
        A.G = c->G32; A.B = c->B32; A.h1 = c->h1_32; A.h2 = c->h2_32;
        A.h1s = (float)c->h1s; A.h2s = (float)c->h2s;
        A.deo = c->deo32;
        e = fns(c->lx).ax32(&A, c->Xh->D, nf, st);
    }
    HIP_TRY(e);
    return SEM_OK;
}

// Jacobi inverse (point Jacobi: exact assembled diagonal), cached per (coef, gs).
sem_status ensure_dinv(sem_coef c, sem_gs g, hipStream_t st);
// The same inverse written to dinv (n_p values), no caching and no allocation.
sem_status compute_dinv(sem_coef c, sem_gs g, double *dinv, hipStream_t st);
// CG scratch of a coef handle for nf fields (and the FP32 vectors when mixed).
sem_status ensure_work(sem_coef c, int nf, bool mixed);
// Row stride of the CG reduction partials (the widest grid of the CG kernels); the
// partial buffer holds (4 nf + 3) rows.
int64_t cg_partial_stride(sem_coef c);
// FP64 two-reduction Jacobi-PCG (sem_pcg_solve with mixed = 0, variant = 0) on the
// scratch W (r, p, w, partial, scal, job64, dots, done and their host mirrors) and the
// Jacobi inverse dinv; P->rtol is the final target.
sem_status pcg_fp64(double *x, const double *b, int nf, sem_coef c, sem_gs g, const sem_pcg_params *P,
                    sem_pcg_info *info, Work &W, const double *dinv, hipStream_t st);
// Argument checks of sem_pcg_solve (SEM_OK for a valid call, including n_p = 0).
sem_status check_pcg_args(const double *x, const double *b, int nfields, sem_coef coef, sem_mesh msh, sem_space Xh,
                          sem_gs gs, const sem_pcg_params *params);
// Owner-weighted dots on the device: out[q*nf + f] = sum_owned a_q b_q (field f), on
// the partial rows and result slots of W (c->ws in the second form).
sem_status dots(sem_coef c, Work &W, sem_gs g, int nf, int nd, const double *const *a, const double *const *b,
                double *host_out, hipStream_t st);
sem_status dots(sem_coef c, sem_gs g, int nf, int nd, const double *const *a, const double *const *b,
                double *host_out, hipStream_t st);
// True FP64 residual |b - A x| / |b| per field (uses W.w and W.r as scratch; c->ws and
// c->dinv in the second form).
sem_status true_residual(sem_coef c, Work &W, const double *dinv, sem_gs g, int nf, const double *x,
                         const double *b, double *rel, hipStream_t st);
sem_status true_residual(sem_coef c, sem_gs g, int nf, const double *x, const double *b, double *rel,
                         hipStream_t st);

// Inner products and linear combinations over sets of vectors of n points (the
// projection space and the Krylov bases): up to PB vectors per pass.
struct VecCtx {
    int64_t n;
    const uint8_t *owner;  // unique-node inner product: one copy of each global id
    double *partial;       // device partial rows of the dot passes
    double *out;           // device results
    double *h_out;         // pinned mirror
};

// host_out[i] = (V_i, v) over unique nodes, i < l (V_i = V + i ld)
sem_status vdots(const VecCtx &X, const double *V, int64_t ld, int l, const double *v, double *host_out,
                 hipStream_t st);
// y = [src +] sum_i c_i V_i (mode 0: y = sum; 1: y += sum; 2: y = src + sum)
sem_status vcomb(const VecCtx &X, double *y, const double *src, const double *V, int64_t ld, int l,
                 const double *c, int mode, hipStream_t st);

}  // namespace semi
