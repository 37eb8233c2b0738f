// sem_api.cpp -- the C ABI of libsem: handles, validation, device residency and the
// Krylov drivers (Jansson et al., arXiv 2107.01243: Eq. 9-10 operator, Section 3.2
// gather-scatter, Section 4 Jacobi-preconditioned CG, Section 10 precision outlook).
//
// Device residency: the mesh and gather-scatter handles are built on the host and
// uploaded on first device use, so their host logic (maps, counts, validation)
// is usable on machines without a GPU.  Everything numeric runs in the HIP
// kernels of ax_kernels.hip and vec_kernels.hip; the drivers only sequence
// launches and poll a few device scalars.
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
    extern "C" int64_t sem_cg_nblocks_f32_lx##L(int64_t);
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

namespace {

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
};

const LxFns &fns(int lx)
{
#define SEM_ROW(L)                                                                                 \
    {sem_launch_ax_f64_lx##L, sem_launch_ax_f32_lx##L, sem_launch_cg_f64_lx##L, sem_launch_cg_f32_lx##L, \
     sem_launch_cg1_f64_lx##L, sem_launch_fdm_lx##L, sem_launch_prolong_lx##L,                     \
     sem_launch_adj_f64_lx##L, sem_launch_adj_f32_lx##L, sem_launch_geom_lx##L, sem_launch_diag_lx##L,  \
     sem_cg_nblocks_f64_lx##L, sem_cg_nblocks_f32_lx##L},
    static const LxFns table[] = {SEM_LX_LIST(SEM_ROW)};
    return table[lx - SEM_LX_MIN];
}

thread_local std::string g_err;

sem_status fail(sem_status s, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

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

sem_status current_device(int *dev)
{
    HIP_TRY(hipGetDevice(dev));
    return SEM_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

}  // namespace

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
    int32_t *d_ent_idx = nullptr;
    uint16_t *d_ent_meta = nullptr;
    bool entries = false;  // entry-parallel execution (groups > 64 copies via d_blk_*)
    int64_t npairs() const { return (int64_t)m.pairs.size() / 2; }
    int64_t nblocks() const { return (int64_t)m.blk_ptr.size() - 1; }
    // work of the per-group kernel as uploaded
    int64_t dev_npairs = 0, dev_nblocks = 0;
};

namespace {

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

}  // namespace

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
    double *cpart = nullptr;              // [3][ceil(nv / 256)]
    uint8_t *mult = nullptr;              // [n]
    void release()
    {
        dfree(S); dfree(lam); dfree(phi); dfree(lin); dfree(cvert); dfree(v_ptr); dfree(v_idx); dfree(v_dir);
        dfree(ell_ci); dfree(ell_val); dfree(dinv0); dfree(part); dfree(cv); dfree(cpart);
        dfree(mult);
        width = 0;
        valid = false;
        gs = nullptr;
        nv = 0;
    }
};

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
    bool dinv_valid = false;
    const void *dinv_gs = nullptr;
    Work ws;
    SchwarzData sz;
};

// ------------------------------------------------------------------ small helpers
namespace {

sem_status check_device(int want)
{
    int dev;
    SEM_TRY(current_device(&dev));
    if (dev != want) return fail(SEM_ERR_INVALID, "handle belongs to device %d but device %d is current", want, dev);
    return SEM_OK;
}

sem_status mesh_upload(sem_mesh m)
{
    if (m->device >= 0) return check_device(m->device);
    int dev;
    SEM_TRY(current_device(&dev));
    if (!m->dir.empty()) {
        SEM_TRY(dalloc(&m->d_dir, m->n));
        HIP_TRY(hipMemcpy(m->d_dir, m->dir.data(), m->n, hipMemcpyHostToDevice));
    }
    if (!m->dir_idx.empty()) {
        SEM_TRY(dalloc(&m->d_dir_idx, m->dir_idx.size()));
        HIP_TRY(hipMemcpy(m->d_dir_idx, m->dir_idx.data(), m->dir_idx.size() * 4, hipMemcpyHostToDevice));
    }
    m->device = dev;
    return SEM_OK;
}

sem_status gs_upload(sem_gs g)
{
    if (g->device >= 0) return check_device(g->device);
    int dev;
    SEM_TRY(current_device(&dev));
    const auto &m = g->m;
    // Device execution order.  Ascending global id (the canonical order) keeps lanes
    // that handle consecutive ids on shared memory segments (for faces normal to the
    // fastest grid direction, lane q's partner and lane q+1's point share a row);
    // ordering by element instead was measured slower.  Each group's own summation
    // order is the same either way.
#if SEM_GS_ENTRY
    // Entry-parallel execution: the per-group kernel keeps only groups > 64 copies.
    const std::vector<int32_t> pairs, &blk_idx = m.big_idx;
    const std::vector<int64_t> &blk_ptr = m.big_ptr;
    g->entries = true;
    SEM_TRY(dalloc(&g->d_ent_idx, m.ent_idx.size()));
    SEM_TRY(dalloc(&g->d_ent_meta, m.ent_meta.size()));
    if (!m.ent_idx.empty()) {
        HIP_TRY(hipMemcpy(g->d_ent_idx, m.ent_idx.data(), m.ent_idx.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(g->d_ent_meta, m.ent_meta.data(), m.ent_meta.size() * 2, hipMemcpyHostToDevice));
    }
#elif SEM_GS_ELEMENT_ORDER
    std::vector<int32_t> pairs, blk_idx;
    std::vector<int64_t> blk_ptr;
    semh::element_order(m, pairs, blk_ptr, blk_idx);
#else
    const std::vector<int32_t> &pairs = m.pairs, &blk_idx = m.blk_idx;
    const std::vector<int64_t> &blk_ptr = m.blk_ptr;
#endif
    g->dev_npairs = (int64_t)pairs.size() / 2;
    g->dev_nblocks = (int64_t)blk_ptr.size() - 1;
    SEM_TRY(dalloc(&g->d_pairs, pairs.size()));
    SEM_TRY(dalloc(&g->d_blk_ptr, blk_ptr.size()));
    SEM_TRY(dalloc(&g->d_blk_idx, blk_idx.size()));
    SEM_TRY(dalloc(&g->d_owner, m.owner.size()));
    if (!pairs.empty()) HIP_TRY(hipMemcpy(g->d_pairs, pairs.data(), pairs.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->d_blk_ptr, blk_ptr.data(), blk_ptr.size() * 8, hipMemcpyHostToDevice));
    if (!blk_idx.empty())
        HIP_TRY(hipMemcpy(g->d_blk_idx, blk_idx.data(), blk_idx.size() * 4, hipMemcpyHostToDevice));
    if (!m.owner.empty()) HIP_TRY(hipMemcpy(g->d_owner, m.owner.data(), m.owner.size(), hipMemcpyHostToDevice));
    g->device = dev;
    return SEM_OK;
}

sem_status check_coef(sem_coef c, sem_mesh msh, sem_space Xh)
{
    if (!c || !msh || !Xh) return fail(SEM_ERR_INVALID, "NULL handle");
    if (c->msh != msh) return fail(SEM_ERR_INVALID, "coef was created for a different mesh");
    if (c->Xh != Xh) return fail(SEM_ERR_INVALID, "coef was created for a different space");
    return check_device(c->device);
}

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
    A.ent_idx = g->d_ent_idx;
    A.ent_meta = g->d_ent_meta;
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
        e = fns(c->lx).ax64(&A, c->Xh->D, nf, st);
    } else {
        A.G = c->G32; A.B = c->B32; A.h1 = c->h1_32; A.h2 = c->h2_32;
        A.h1s = (float)c->h1s; A.h2s = (float)c->h2s;
        e = fns(c->lx).ax32(&A, c->Xh->D, nf, st);
    }
    HIP_TRY(e);
    return SEM_OK;
}

// Jacobi inverse (point Jacobi: exact assembled diagonal), cached per (coef, gs).
sem_status ensure_dinv(sem_coef c, sem_gs g, hipStream_t st)
{
    if (c->dinv_valid && c->dinv_gs == (const void *)g) return SEM_OK;
    if (!c->dinv) SEM_TRY(dalloc(&c->dinv, c->n));
    DiagArgs A;
    A.d = c->dinv;
    A.G = c->G;
    A.B = c->B;
    A.h1 = c->h1;
    A.h2 = c->h2;
    A.h1s = c->h1s;
    A.h2s = c->h2s;
    A.n = c->n;
    HIP_TRY(fns(c->lx).diag(&A, c->Xh->D, st));
    SEM_TRY(launch_gs<double>(c->dinv, 1, g, nullptr, nullptr, st));
    HIP_TRY(sem_launch_invert(c->dinv, c->msh->d_dir, c->n, st));
    if (c->flags & SEM_COEF_F32) {
        if (!c->dinv32) SEM_TRY(dalloc(&c->dinv32, c->n));
        HIP_TRY(sem_launch_cast_f32_f64(c->dinv32, c->dinv, 1.0, c->n, st));
    }
    c->dinv_valid = true;
    c->dinv_gs = g;
    return SEM_OK;
}

sem_status ensure_work(sem_coef c, int nf, bool mixed)
{
    Work &W = c->ws;
    if (W.cap_n == c->n && W.cap_f >= nf && (W.mixed || !mixed)) return SEM_OK;
    W.release();
    const int64_t n = c->n;
    const int64_t nn = n * nf;
    SEM_TRY(dalloc(&W.r, nn));
    SEM_TRY(dalloc(&W.p, nn));
    SEM_TRY(dalloc(&W.w, nn));
    if (mixed) {
        SEM_TRY(dalloc(&W.z, nn));
        SEM_TRY(dalloc(&W.q, nn));
        SEM_TRY(dalloc(&W.r32, nn));
        SEM_TRY(dalloc(&W.y32, nn));
        SEM_TRY(dalloc(&W.p32, nn));
        SEM_TRY(dalloc(&W.w32, nn));
        SEM_TRY(dalloc(&W.ri32, nn));
    }
    const int64_t nb = std::max<int64_t>({fns(c->lx).nblk64(c->nelv), fns(c->lx).nblk32(c->nelv),
                                          (int64_t)sem_vec_grid(n), (int64_t)sem_update_grid(n, 0),
                                          (int64_t)sem_update_grid(n, 1)});
    // 4 rows per field, plus the single-reduction update partials at offset 3 nb
    W.partial_len = (4 * (int64_t)nf + 3) * nb;
    W.nb = nb;
    SEM_TRY(dalloc(&W.partial, W.partial_len));
    SEM_TRY(dalloc(&W.scal, nf));
    SEM_TRY(dalloc(&W.job64, 1));
    SEM_TRY(dalloc(&W.job32, 1));
    SEM_TRY(dalloc(&W.job_cg1, 1));
    SEM_TRY(dalloc(&W.dots, 4 * nf));
    SEM_TRY(dalloc(&W.fcg, 4 * nf));
    SEM_TRY(dalloc(&W.done, nf));
    HIP_TRY(hipHostMalloc((void **)&W.h_scal, sizeof(CgScalars) * nf, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&W.h_dots, sizeof(double) * 4 * nf, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&W.h_fcg, sizeof(double) * 4 * nf, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&W.h_done, sizeof(int) * nf, hipHostMallocDefault));
    SEM_TRY(dalloc(&W.rel, nf));
    HIP_TRY(hipHostMalloc((void **)&W.h_rel, sizeof(RelState) * nf, hipHostMallocDefault));
    const AlphaJob j64{W.partial, fns(c->lx).nblk64(c->nelv), W.scal};
    const AlphaJob j32{W.partial, fns(c->lx).nblk32(c->nelv), W.scal};
    HIP_TRY(hipMemcpy(W.job64, &j64, sizeof(AlphaJob), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(W.job32, &j32, sizeof(AlphaJob), hipMemcpyHostToDevice));
    // single-reduction fold: matvec partials [f][nblk64] at the start of W.partial, the
    // update's [2][f][grid] after three rows of nb (clear of the matvec's up to 3 fields)
    const AlphaJob j1{W.partial, fns(c->lx).nblk64(c->nelv), W.scal, 1, W.partial + 3 * nb,
                      (int64_t)sem_vec_grid(n)};
    HIP_TRY(hipMemcpy(W.job_cg1, &j1, sizeof(AlphaJob), hipMemcpyHostToDevice));
    W.cap_n = n;
    W.cap_f = nf;
    W.mixed = mixed;
    return SEM_OK;
}

// Owner-weighted dots on the device: out[q*nf + f] = sum_owned a_q b_q (field f).
sem_status dots(sem_coef c, sem_gs g, int nf, int nd, const double *const *a, const double *const *b,
                double *host_out, hipStream_t st)
{
    Work &W = c->ws;
    DotArgs A;
    for (int q = 0; q < 4; ++q) {
        A.a[q] = q < nd ? a[q] : nullptr;
        A.b[q] = q < nd ? b[q] : nullptr;
    }
    A.owner = g->d_owner;
    A.partial = W.partial;
    A.n = c->n;
    A.nd = nd;
    A.nfields = nf;
    const unsigned grid = sem_vec_grid(c->n);
    HIP_TRY(sem_launch_dots(&A, grid, st));
    HIP_TRY(sem_launch_dots_finish(W.partial, grid, nd * nf, W.dots, st));
    HIP_TRY(hipMemcpyAsync(W.h_dots, W.dots, sizeof(double) * nd * nf, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(host_out, W.h_dots, sizeof(double) * nd * nf);
    return SEM_OK;
}

template <typename T>
sem_status cg_iterate(sem_coef c, sem_gs g, int nf, T *x, T *r, T *p, T *w, const T *dinv, int max_iter,
                      int check_every, double *hist, int hist_len, hipStream_t st);

// Jacobi-PCG in precision T on nf fields.  x is the iterate (zeroed unless use_x0),
// b the assembled, masked right-hand side.  Per-field results land in W.h_scal.
template <typename T>
sem_status cg_run(sem_coef c, sem_gs g, int nf, T *x, const T *b, bool use_x0, T *r, T *p, T *w,
                  const T *dinv, const double *rtol, int max_iter, int check_every, double *hist, int hist_len,
                  hipStream_t st)
{
    Work &W = c->ws;
    const int64_t n = c->n;
    if (use_x0) {
        SEM_TRY(launch_ax<T>(c, w, x, nf, st));
        SEM_TRY(launch_gs<T>(w, nf, g, nullptr, nullptr, st));
    } else {
        if constexpr (sizeof(T) == 8) HIP_TRY(sem_launch_fill_f64(x, 0.0, n * nf, st));
        else HIP_TRY(sem_launch_fill_f32(x, 0.0f, n * nf, st));
    }
    for (int f = 0; f < nf; ++f) {
        CgScalars s{};
        s.rtol = rtol[f];
        s.max_iter = max_iter;
        W.h_scal[f] = s;
    }
    HIP_TRY(hipMemcpyAsync(W.scal, W.h_scal, sizeof(CgScalars) * nf, hipMemcpyHostToDevice, st));
    const unsigned vg = sem_vec_grid(n);
    {
        CgInitArgs<T> A;
        A.b = b;
        A.w = use_x0 ? w : nullptr;
        A.r = r;
        A.p = p;
        A.dinv = dinv;
        A.owner = g->d_owner;
        A.partial = W.partial;
        A.n = n;
        A.nfields = nf;
        if constexpr (sizeof(T) == 8) HIP_TRY(sem_launch_cg_init_f64(&A, vg, st));
        else HIP_TRY(sem_launch_cg_init_f32(&A, vg, st));
        CgFinishArgs F{W.partial, (int64_t)vg, W.scal, hist, hist_len, nf};
        HIP_TRY(sem_launch_cg_start(&F, st));
    }
    return cg_iterate<T>(c, g, nf, x, r, p, w, dinv, max_iter, check_every, hist, hist_len, st);
}

// Iterate the CG state held in W.scal until every field has stopped.
template <typename T>
sem_status cg_iterate(sem_coef c, sem_gs g, int nf, T *x, T *r, T *p, T *w, const T *dinv, int max_iter,
                      int check_every, double *hist, int hist_len, hipStream_t st)
{
    Work &W = c->ws;
    const int64_t n = c->n;
    const bool f64 = sizeof(T) == 8;
    const unsigned ug = sem_update_grid(n, f64 ? 0 : 1);
    const AlphaJob *job = f64 ? W.job64 : W.job32;
    CgMatvecArgs<T> M;
    M.p = p;
    M.w = w;
    M.r = r;
    M.dinv = dinv;
    if constexpr (sizeof(T) == 8) {
        M.G = c->G; M.B = c->B; M.h1 = c->h1; M.h2 = c->h2; M.h1s = c->h1s; M.h2s = c->h2s;
    } else {
        M.G = c->G32; M.B = c->B32; M.h1 = c->h1_32; M.h2 = c->h2_32;
        M.h1s = (float)c->h1s; M.h2s = (float)c->h2s;
    }
    M.n = n;
    M.nelv = c->nelv;
    M.scal = W.scal;
    M.partial = W.partial;
    CgUpdateArgs<T> U{x, r, p, w, dinv, g->d_owner, W.scal, W.partial, n, nf};
    CgFinishArgs F{W.partial, (int64_t)ug, W.scal, hist, hist_len, nf};
    if (check_every < 1) check_every = 1;
    const int64_t max_batches = (int64_t)(max_iter + check_every - 1) / check_every + 2;
    // first poll right after initialisation (b = 0 or an exact initial guess)
    HIP_TRY(hipMemcpyAsync(W.h_scal, W.scal, sizeof(CgScalars) * nf, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t bt = 0; bt < max_batches; ++bt) {
        bool all = true;
        for (int f = 0; f < nf; ++f) all = all && W.h_scal[f].stop;
        if (all) break;
        int launched_max = 0;
        for (int f = 0; f < nf; ++f) launched_max = std::max(launched_max, W.h_scal[f].iter);
        const int todo = std::min(check_every, std::max(1, max_iter - launched_max));
        for (int it = 0; it < todo; ++it) {
            if constexpr (sizeof(T) == 8) HIP_TRY(fns(c->lx).cg64(&M, c->Xh->D, nf, st));
            else HIP_TRY(fns(c->lx).cg32(&M, c->Xh->D, nf, st));
            SEM_TRY(launch_gs<T>(w, nf, g, W.scal, job, st));
            if constexpr (sizeof(T) == 8) HIP_TRY(sem_launch_cg_update_f64(&U, ug, st));
            else HIP_TRY(sem_launch_cg_update_f32(&U, ug, st));
            HIP_TRY(sem_launch_cg_finish(&F, st));
        }
        HIP_TRY(hipMemcpyAsync(W.h_scal, W.scal, sizeof(CgScalars) * nf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return SEM_OK;
}

// True FP64 residual |b - A x| / |b| per field (uses W.w and W.r as scratch).
sem_status true_residual(sem_coef c, sem_gs g, int nf, const double *x, const double *b, double *rel,
                         hipStream_t st)
{
    Work &W = c->ws;
    SEM_TRY(launch_ax<double>(c, W.w, x, nf, st));
    SEM_TRY(launch_gs<double>(W.w, nf, g, nullptr, nullptr, st));
    HIP_TRY(sem_launch_residual(W.r, b, W.w, c->dinv, c->n, nf, st));
    const double *a[2] = {W.r, b};
    double out[6];
    SEM_TRY(dots(c, g, nf, 2, a, a, out, st));
    for (int f = 0; f < nf; ++f) {
        const double rr = out[0 * nf + f], bb = out[1 * nf + f];
        rel[f] = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    }
    return SEM_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char *sem_last_error(void) { return g_err.c_str(); }
const char *sem_version(void) { return "libsem 0.1 (gfx950)"; }

// ------------------------------------------------------------------ space
sem_status sem_space_create(int lx, sem_space *Xh)
{
    if (!Xh) return fail(SEM_ERR_INVALID, "Xh is NULL");
    *Xh = nullptr;
    if (lx < SEM_LX_MIN || lx > SEM_LX_MAX) return fail(SEM_ERR_INVALID, "lx=%d outside [%d, %d]", lx, SEM_LX_MIN, SEM_LX_MAX);
    sem_space s = new (std::nothrow) sem_space_s();
    if (!s) return fail(SEM_ERR_OOM, "out of host memory");
    s->lx = lx;
    semh::gll_space(lx, s->xi, s->w, s->D);
    *Xh = s;
    return SEM_OK;
}

sem_status sem_space_get(sem_space Xh, double *xi, double *w, double *D)
{
    if (!Xh) return fail(SEM_ERR_INVALID, "Xh is NULL");
    const int lx = Xh->lx;
    if (xi) std::memcpy(xi, Xh->xi, sizeof(double) * lx);
    if (w) std::memcpy(w, Xh->w, sizeof(double) * lx);
    if (D) std::memcpy(D, Xh->D, sizeof(double) * lx * lx);
    return SEM_OK;
}

void sem_space_destroy(sem_space Xh) { delete Xh; }

// ------------------------------------------------------------------ box mesh
sem_status sem_box_mesh(int nx, int ny, int nz, int lx, double eps, int64_t *glb, uint8_t *dirichlet,
                        double *xyz)
{
    if (nx < 1 || ny < 1 || nz < 1) return fail(SEM_ERR_INVALID, "element counts must be >= 1");
    if (lx < SEM_LX_MIN || lx > SEM_LX_MAX) return fail(SEM_ERR_INVALID, "lx=%d outside [%d, %d]", lx, SEM_LX_MIN, SEM_LX_MAX);
    if (!(std::fabs(eps) < 0.5)) return fail(SEM_ERR_INVALID, "deformation amplitude must be finite and < 0.5");
    double xi[SEM_LX_MAX], w[SEM_LX_MAX], D[SEM_LX_MAX * SEM_LX_MAX];
    semh::gll_space(lx, xi, w, D);
    semh::box_mesh(nx, ny, nz, lx, eps, xi, glb, dirichlet, xyz);
    return SEM_OK;
}

// ------------------------------------------------------------------ mesh
sem_status sem_mesh_create(int64_t nelv, int lx, const int64_t *glb_host, const uint8_t *dirichlet_host,
                           sem_mesh *msh)
{
    if (!msh) return fail(SEM_ERR_INVALID, "msh is NULL");
    *msh = nullptr;
    if (lx < SEM_LX_MIN || lx > SEM_LX_MAX) return fail(SEM_ERR_INVALID, "lx=%d outside [%d, %d]", lx, SEM_LX_MIN, SEM_LX_MAX);
    if (nelv < 0) return fail(SEM_ERR_INVALID, "nelv < 0");
    const int64_t n = nelv * (int64_t)lx * lx * lx;
    if (n > 0 && !glb_host) return fail(SEM_ERR_INVALID, "glb is NULL");
    if (n >= ((int64_t)1 << 31)) return fail(SEM_ERR_INVALID, "n_local = %lld exceeds 2^31-1", (long long)n);
    sem_mesh m = new (std::nothrow) sem_mesh_s();
    if (!m) return fail(SEM_ERR_OOM, "out of host memory");
    m->nelv = nelv;
    m->lx = lx;
    m->n = n;
    m->glb.assign(glb_host, glb_host + n);
    for (int64_t p = 0; p < n; ++p)
        if (m->glb[p] < 0) {
            delete m;
            return fail(SEM_ERR_INVALID, "negative global id at %lld", (long long)p);
        }
    if (dirichlet_host) {
        m->dir.resize(n);
        for (int64_t p = 0; p < n; ++p) {
            m->dir[p] = dirichlet_host[p] ? 1 : 0;
            if (m->dir[p]) m->dir_idx.push_back((int32_t)p);
        }
        if (m->dir_idx.empty()) m->dir.clear();
    }
    *msh = m;
    return SEM_OK;
}

sem_status sem_mesh_size(sem_mesh msh, int64_t *nelv, int *lx, int64_t *n_local, int64_t *n_unique,
                         int64_t *n_dirichlet_local)
{
    if (!msh) return fail(SEM_ERR_INVALID, "msh is NULL");
    if (nelv) *nelv = msh->nelv;
    if (lx) *lx = msh->lx;
    if (n_local) *n_local = msh->n;
    if (n_unique) {
        if (msh->n_unique < 0) {
            std::vector<int64_t> s(msh->glb);
            std::sort(s.begin(), s.end());
            msh->n_unique = (int64_t)(std::unique(s.begin(), s.end()) - s.begin());
        }
        *n_unique = msh->n_unique;
    }
    if (n_dirichlet_local) *n_dirichlet_local = (int64_t)msh->dir_idx.size();
    return SEM_OK;
}

void sem_mesh_destroy(sem_mesh msh)
{
    if (!msh) return;
    dfree(msh->d_dir);
    dfree(msh->d_dir_idx);
    delete msh;
}

// ------------------------------------------------------------------ gather-scatter
sem_status sem_gs_create(sem_mesh msh, sem_gs *gs)
{
    if (!gs) return fail(SEM_ERR_INVALID, "gs is NULL");
    *gs = nullptr;
    if (!msh) return fail(SEM_ERR_INVALID, "msh is NULL");
    sem_gs g = new (std::nothrow) sem_gs_s();
    if (!g) return fail(SEM_ERR_OOM, "out of host memory");
    std::string msg;
    if (!semh::build_gs_maps(msh->n, msh->glb.data(), msh->dir.empty() ? nullptr : msh->dir.data(), g->m, msg)) {
        delete g;
        return fail(SEM_ERR_INVALID, "%s", msg.c_str());
    }
    g->msh = msh;
    msh->n_unique = g->m.n_unique;
    *gs = g;
    return SEM_OK;
}

sem_status sem_gs_sizes(sem_gs gs, int64_t *npairs, int64_t *nblocks, int64_t *nblock_entries)
{
    if (!gs) return fail(SEM_ERR_INVALID, "gs is NULL");
    if (npairs) *npairs = gs->npairs();
    if (nblocks) *nblocks = gs->nblocks();
    if (nblock_entries) *nblock_entries = (int64_t)gs->m.blk_idx.size();
    return SEM_OK;
}

sem_status sem_gs_export_maps(sem_gs gs, int32_t *pairs, int64_t *blk_ptr, int32_t *blk_idx, uint8_t *mult)
{
    if (!gs) return fail(SEM_ERR_INVALID, "gs is NULL");
    const auto &m = gs->m;
    if (pairs && !m.pairs.empty()) std::memcpy(pairs, m.pairs.data(), m.pairs.size() * 4);
    if (blk_ptr) std::memcpy(blk_ptr, m.blk_ptr.data(), m.blk_ptr.size() * 8);
    if (blk_idx && !m.blk_idx.empty()) std::memcpy(blk_idx, m.blk_idx.data(), m.blk_idx.size() * 4);
    if (mult && !m.mult.empty()) std::memcpy(mult, m.mult.data(), m.mult.size());
    return SEM_OK;
}

void sem_gs_destroy(sem_gs gs)
{
    if (!gs) return;
    dfree(gs->d_pairs);
    dfree(gs->d_blk_ptr);
    dfree(gs->d_blk_idx);
    dfree(gs->d_owner);
    dfree(gs->d_ent_idx);
    dfree(gs->d_ent_meta);
    delete gs;
}

sem_status sem_gs_op(void *u, int nfields, sem_gs gs, sem_dtype dt, void *stream)
{
    if (!gs) return fail(SEM_ERR_INVALID, "gs is NULL");
    if (nfields != 1 && nfields != 3) return fail(SEM_ERR_INVALID, "nfields must be 1 or 3");
    if (dt != SEM_F64 && dt != SEM_F32) return fail(SEM_ERR_INVALID, "bad dtype");
    if (!u && gs->m.n > 0) return fail(SEM_ERR_INVALID, "u is NULL");
    SEM_TRY(gs_upload(gs));
    if (dt == SEM_F64) return launch_gs<double>((double *)u, nfields, gs, nullptr, nullptr, S(stream));
    return launch_gs<float>((float *)u, nfields, gs, nullptr, nullptr, S(stream));
}

sem_status sem_mask(void *u, int nfields, sem_mesh msh, sem_dtype dt, void *stream)
{
    if (!msh) return fail(SEM_ERR_INVALID, "msh is NULL");
    if (nfields != 1 && nfields != 3) return fail(SEM_ERR_INVALID, "nfields must be 1 or 3");
    if (dt != SEM_F64 && dt != SEM_F32) return fail(SEM_ERR_INVALID, "bad dtype");
    if (!u && msh->n > 0) return fail(SEM_ERR_INVALID, "u is NULL");
    SEM_TRY(mesh_upload(msh));
    HIP_TRY(sem_launch_mask(u, dt == SEM_F32, msh->d_dir_idx, (int64_t)msh->dir_idx.size(), msh->n, nfields,
                            S(stream)));
    return SEM_OK;
}

// ------------------------------------------------------------------ coef
static sem_status coef_alloc(sem_space Xh, sem_mesh msh, unsigned flags, sem_coef *out)
{
    if (!out) return fail(SEM_ERR_INVALID, "coef is NULL");
    *out = nullptr;
    if (!Xh || !msh) return fail(SEM_ERR_INVALID, "NULL handle");
    if (Xh->lx != msh->lx) return fail(SEM_ERR_INVALID, "space lx=%d but mesh lx=%d", Xh->lx, msh->lx);
    if (flags & ~SEM_COEF_F32) return fail(SEM_ERR_INVALID, "unknown flags 0x%x", flags);
    SEM_TRY(mesh_upload(msh));
    sem_coef c = new (std::nothrow) sem_coef_s();
    if (!c) return fail(SEM_ERR_OOM, "out of host memory");
    c->Xh = Xh;
    c->msh = msh;
    c->lx = Xh->lx;
    c->n = msh->n;
    c->nelv = msh->nelv;
    c->flags = flags;
    c->device = msh->device;
    sem_status s;
    if ((s = dalloc(&c->G, 6 * c->n)) != SEM_OK || (s = dalloc(&c->B, c->n)) != SEM_OK) {
        sem_coef_destroy(c);
        return s;
    }
    if (flags & SEM_COEF_F32) {
        if ((s = dalloc(&c->G32, 6 * c->n)) != SEM_OK || (s = dalloc(&c->B32, c->n)) != SEM_OK) {
            sem_coef_destroy(c);
            return s;
        }
    }
    *out = c;
    return SEM_OK;
}

static sem_status coef_finish(sem_coef c, hipStream_t st)
{
    if (c->flags & SEM_COEF_F32) {
        HIP_TRY(sem_launch_cast_f32_f64(c->G32, c->G, 1.0, 6 * c->n, st));
        HIP_TRY(sem_launch_cast_f32_f64(c->B32, c->B, 1.0, c->n, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    return SEM_OK;
}

sem_status sem_coef_create(sem_space Xh, sem_mesh msh, const double *xyz_dev, unsigned flags, void *stream,
                           sem_coef *coef)
{
    if (!xyz_dev && msh && msh->n > 0) return fail(SEM_ERR_INVALID, "xyz is NULL");
    SEM_TRY(coef_alloc(Xh, msh, flags, coef));
    sem_coef c = *coef;
    hipStream_t st = S(stream);
    unsigned *nbad = nullptr;
    sem_status s = dalloc(&nbad, 1);
    if (s != SEM_OK) { sem_coef_destroy(c); *coef = nullptr; return s; }
    unsigned hbad = 0;
    hipError_t e = hipMemcpyAsync(nbad, &hbad, sizeof(unsigned), hipMemcpyHostToDevice, st);
    GeomArgs A{xyz_dev, c->G, c->B, nbad, c->n};
    if (e == hipSuccess) e = fns(c->lx).geom(&A, Xh->D, Xh->w, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, nbad, sizeof(unsigned), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(nbad);
    if (e != hipSuccess) {
        sem_coef_destroy(c);
        *coef = nullptr;
        return fail(SEM_ERR_HIP, "geometry setup failed: %s", hipGetErrorString(e));
    }
    if (hbad) {
        sem_coef_destroy(c);
        *coef = nullptr;
        return fail(SEM_ERR_INVALID, "%u points have a non-positive Jacobian", hbad);
    }
    s = coef_finish(c, st);
    if (s != SEM_OK) { sem_coef_destroy(c); *coef = nullptr; }
    return s;
}

sem_status sem_coef_create_from_G(sem_space Xh, sem_mesh msh, const double *G6_dev, const double *B_dev,
                                  unsigned flags, void *stream, sem_coef *coef)
{
    if ((!G6_dev || !B_dev) && msh && msh->n > 0) return fail(SEM_ERR_INVALID, "G or B is NULL");
    SEM_TRY(coef_alloc(Xh, msh, flags, coef));
    sem_coef c = *coef;
    hipStream_t st = S(stream);
    hipError_t e = hipSuccess;
    if (c->n > 0) {
        e = hipMemcpyAsync(c->G, G6_dev, sizeof(double) * 6 * c->n, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(c->B, B_dev, sizeof(double) * c->n, hipMemcpyDeviceToDevice, st);
    }
    if (e != hipSuccess) {
        sem_coef_destroy(c);
        *coef = nullptr;
        return fail(SEM_ERR_HIP, "copy of G/B failed: %s", hipGetErrorString(e));
    }
    sem_status s = coef_finish(c, st);
    if (s != SEM_OK) { sem_coef_destroy(c); *coef = nullptr; }
    return s;
}

sem_status sem_coef_set_helmholtz(sem_coef c, const double *h1_dev, double h1, const double *h2_dev, double h2,
                                  void *stream)
{
    if (!c) return fail(SEM_ERR_INVALID, "coef is NULL");
    SEM_TRY(check_device(c->device));
    if (!h1_dev && !std::isfinite(h1)) return fail(SEM_ERR_INVALID, "h1 is not finite");
    if (!h2_dev && !std::isfinite(h2)) return fail(SEM_ERR_INVALID, "h2 is not finite");
    hipStream_t st = S(stream);
    const bool f32 = c->flags & SEM_COEF_F32;
    if (h1_dev) {
        if (!c->h1) SEM_TRY(dalloc(&c->h1, c->n));
        HIP_TRY(hipMemcpyAsync(c->h1, h1_dev, sizeof(double) * c->n, hipMemcpyDeviceToDevice, st));
        if (f32) {
            if (!c->h1_32) SEM_TRY(dalloc(&c->h1_32, c->n));
            HIP_TRY(sem_launch_cast_f32_f64(c->h1_32, c->h1, 1.0, c->n, st));
        }
    } else {
        dfree(c->h1);
        dfree(c->h1_32);
        c->h1s = h1;
    }
    if (h2_dev) {
        if (!c->h2) SEM_TRY(dalloc(&c->h2, c->n));
        HIP_TRY(hipMemcpyAsync(c->h2, h2_dev, sizeof(double) * c->n, hipMemcpyDeviceToDevice, st));
        if (f32) {
            if (!c->h2_32) SEM_TRY(dalloc(&c->h2_32, c->n));
            HIP_TRY(sem_launch_cast_f32_f64(c->h2_32, c->h2, 1.0, c->n, st));
        }
    } else {
        dfree(c->h2);
        dfree(c->h2_32);
        c->h2s = h2;
    }
    c->dinv_valid = false;
    c->sz.valid = false;
    return SEM_OK;
}

sem_status sem_coef_export(sem_coef c, double *G6_dev, double *B_dev, void *stream)
{
    if (!c) return fail(SEM_ERR_INVALID, "coef is NULL");
    SEM_TRY(check_device(c->device));
    if (G6_dev && c->n > 0)
        HIP_TRY(hipMemcpyAsync(G6_dev, c->G, sizeof(double) * 6 * c->n, hipMemcpyDeviceToDevice, S(stream)));
    if (B_dev) HIP_TRY(hipMemcpyAsync(B_dev, c->B, sizeof(double) * c->n, hipMemcpyDeviceToDevice, S(stream)));
    return SEM_OK;
}

void sem_coef_destroy(sem_coef c)
{
    if (!c) return;
    c->ws.release();
    c->sz.release();
    dfree(c->G); dfree(c->B); dfree(c->G32); dfree(c->B32);
    dfree(c->h1); dfree(c->h2); dfree(c->h1_32); dfree(c->h2_32);
    dfree(c->dinv); dfree(c->dinv32);
    delete c;
}

// ------------------------------------------------------------------ operators
sem_status sem_ax_helm(void *w, const void *u, sem_coef coef, sem_mesh msh, sem_space Xh, int nfields,
                       sem_dtype dt, void *stream)
{
    SEM_TRY(check_coef(coef, msh, Xh));
    if (nfields != 1 && nfields != 3) return fail(SEM_ERR_INVALID, "nfields must be 1 or 3");
    if (dt != SEM_F64 && dt != SEM_F32) return fail(SEM_ERR_INVALID, "bad dtype");
    if (dt == SEM_F32 && !(coef->flags & SEM_COEF_F32)) return fail(SEM_ERR_INVALID, "SEM_F32 needs a coef created with SEM_COEF_F32");
    const size_t bytes = (size_t)coef->n * nfields * (dt == SEM_F64 ? 8 : 4);
    if (bytes == 0) return SEM_OK;
    if (!w || !u) return fail(SEM_ERR_INVALID, "w or u is NULL");
    if (overlap(w, bytes, u, bytes)) return fail(SEM_ERR_INVALID, "w and u overlap");
    if (dt == SEM_F64) return launch_ax<double>(coef, (double *)w, (const double *)u, nfields, S(stream));
    return launch_ax<float>(coef, (float *)w, (const float *)u, nfields, S(stream));
}

sem_status sem_ax_helm_adjoint(void *g, const void *u, const void *v, sem_coef coef, sem_mesh msh,
                               sem_space Xh, sem_dtype dt, void *stream)
{
    SEM_TRY(check_coef(coef, msh, Xh));
    if (dt != SEM_F64 && dt != SEM_F32) return fail(SEM_ERR_INVALID, "bad dtype");
    if (dt == SEM_F32 && !(coef->flags & SEM_COEF_F32)) return fail(SEM_ERR_INVALID, "SEM_F32 needs a coef created with SEM_COEF_F32");
    const size_t bytes = (size_t)coef->n * (dt == SEM_F64 ? 8 : 4);
    if (bytes == 0) return SEM_OK;
    if (!g || !u || !v) return fail(SEM_ERR_INVALID, "g, u or v is NULL");
    if (overlap(g, bytes, u, bytes) || overlap(g, bytes, v, bytes)) return fail(SEM_ERR_INVALID, "g overlaps u or v");
    hipError_t e;
    if (dt == SEM_F64) {
        AdjArgs<double> A{(double *)g, (const double *)u, (const double *)v, coef->G, coef->n, coef->nelv};
        e = fns(coef->lx).adj64(&A, Xh->D, S(stream));
    } else {
        AdjArgs<float> A{(float *)g, (const float *)u, (const float *)v, coef->G32, coef->n, coef->nelv};
        e = fns(coef->lx).adj32(&A, Xh->D, S(stream));
    }
    HIP_TRY(e);
    return SEM_OK;
}

sem_status sem_jacobi_inverse(double *dinv, sem_coef coef, sem_mesh msh, sem_space Xh, sem_gs gs, void *stream)
{
    SEM_TRY(check_coef(coef, msh, Xh));
    if (!gs || gs->msh != msh) return fail(SEM_ERR_INVALID, "gs is NULL or built for another mesh");
    if (!dinv && coef->n > 0) return fail(SEM_ERR_INVALID, "dinv is NULL");
    SEM_TRY(gs_upload(gs));
    SEM_TRY(ensure_dinv(coef, gs, S(stream)));
    if (coef->n > 0)
        HIP_TRY(hipMemcpyAsync(dinv, coef->dinv, sizeof(double) * coef->n, hipMemcpyDeviceToDevice, S(stream)));
    return SEM_OK;
}

// ------------------------------------------------------------------ measurement
sem_status sem_stream_triad(double *a, const double *b, const double *c, double s, int64_t n, void *stream)
{
    if (n < 0) return fail(SEM_ERR_INVALID, "n < 0");
    if (n == 0) return SEM_OK;
    if (!a || !b || !c) return fail(SEM_ERR_INVALID, "NULL pointer");
    const size_t bytes = (size_t)n * 8;
    if (overlap(a, bytes, b, bytes) || overlap(a, bytes, c, bytes)) return fail(SEM_ERR_INVALID, "a overlaps b or c");
    HIP_TRY(sem_launch_triad(a, b, c, s, n, S(stream)));
    return SEM_OK;
}

// ------------------------------------------------------------------ solver
// Single-reduction Jacobi-PCG (Chronopoulos-Gear) in FP64.  Per iteration: update
// (p, s, x, r), matvec of r (u = dinv r, w = A_L u, partials of (r,u), (u,Au), (r,r)),
// gather-scatter of w whose first workgroup folds the scalars.  After the recursive
// residual meets rtol the true residual is checked; a field that misses it restarts
// the recurrences from its current iterate (beta = 0), keeping its iteration count.
static sem_status pcg_cg1(double *x, const double *b, int nf, sem_coef c, sem_gs g, const sem_pcg_params *P,
                          sem_pcg_info *info, hipStream_t st)
{
    Work &W = c->ws;
    const int64_t n = c->n, nn = n * nf;
    if (!W.s) SEM_TRY(dalloc(&W.s, (size_t)W.cap_n * W.cap_f));
    // initial residual and scalars exactly as for the two-reduction form
    if (P->use_x0) {
        SEM_TRY(launch_ax<double>(c, W.w, x, nf, st));
        SEM_TRY(launch_gs<double>(W.w, nf, g, nullptr, nullptr, st));
    } else {
        HIP_TRY(sem_launch_fill_f64(x, 0.0, nn, st));
    }
    for (int f = 0; f < nf; ++f) {
        CgScalars s{};
        s.rtol = P->rtol;
        s.max_iter = P->max_iter;
        W.h_scal[f] = s;
    }
    HIP_TRY(hipMemcpyAsync(W.scal, W.h_scal, sizeof(CgScalars) * nf, hipMemcpyHostToDevice, st));
    const unsigned vg = sem_vec_grid(n);
    {
        CgInitArgs<double> A{b, P->use_x0 ? W.w : nullptr, W.r, W.p, c->dinv, g->d_owner, W.partial, n, nf};
        HIP_TRY(sem_launch_cg_init_f64(&A, vg, st));
        CgFinishArgs F{W.partial, (int64_t)vg, W.scal, nullptr, 0, nf};
        HIP_TRY(sem_launch_cg_start(&F, st));
    }
    HIP_TRY(sem_launch_fill_f64(W.s, 0.0, nn, st));
    CgMatvecArgs<double> M{};
    M.r = W.r;
    M.w = W.w;
    M.dinv = c->dinv;
    M.G = c->G; M.B = c->B; M.h1 = c->h1; M.h2 = c->h2; M.h1s = c->h1s; M.h2s = c->h2s;
    M.n = n;
    M.nelv = c->nelv;
    M.scal = W.scal;
    M.partial = W.partial;
    // the update's partials go where the fold job reads them (see ensure_work)
    const Cg1UpdateArgs U{x, W.r, W.p, W.s, W.w, c->dinv, g->d_owner, W.scal, W.partial + 3 * W.nb, n, nf};
    auto prime = [&]() -> sem_status {  // matvec of the current r and the first fold
        HIP_TRY(fns(c->lx).cg1(&M, c->Xh->D, nf, st));
        return launch_gs<double>(W.w, nf, g, W.scal, W.job_cg1, st);
    };
    auto iterate = [&]() -> sem_status {
        const int check_every = std::max(1, P->check_every);
        const int64_t max_batches = (int64_t)(P->max_iter + check_every - 1) / check_every + 2;
        HIP_TRY(hipMemcpyAsync(W.h_scal, W.scal, sizeof(CgScalars) * nf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int64_t bt = 0; bt < max_batches; ++bt) {
            bool all = true;
            int done_max = 0;
            for (int f = 0; f < nf; ++f) {
                all = all && W.h_scal[f].stop;
                done_max = std::max(done_max, W.h_scal[f].iter);
            }
            if (all) break;
            const int todo = std::min(check_every, std::max(1, P->max_iter - done_max));
            for (int it = 0; it < todo; ++it) {
                HIP_TRY(sem_launch_cg1_update(&U, st));
                SEM_TRY(prime());
            }
            HIP_TRY(hipMemcpyAsync(W.h_scal, W.scal, sizeof(CgScalars) * nf, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        return SEM_OK;
    };
    SEM_TRY(prime());
    SEM_TRY(iterate());
    double tr[3];
    for (int round = 0;; ++round) {
        SEM_TRY(true_residual(c, g, nf, x, b, tr, st));  // leaves b - A x in W.r
        bool any = false;
        for (int f = 0; f < nf; ++f) {
            CgScalars &s = W.h_scal[f];
            const bool redo = s.status == 0 && P->rtol > 0 && s.bb > 0 && tr[f] > P->rtol && s.iter < P->max_iter;
            if (redo) {
                s.stop = 0;
                s.primed = 0;
            } else {
                s.stop = 1;
            }
            any = any || redo;
        }
        if (!any || round >= 16) break;
        // restart the fields that missed rtol from their current iterate: r is the
        // true residual (with its (r, dinv r) and (r, r)), p and s start from zero
        // (beta = 0 at the first fold)
        for (int f = 0; f < nf; ++f) W.h_done[f] = W.h_scal[f].stop ? 0 : 1;
        HIP_TRY(hipMemcpyAsync(W.scal, W.h_scal, sizeof(CgScalars) * nf, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(W.done, W.h_done, sizeof(int) * nf, hipMemcpyHostToDevice, st));
        HIP_TRY(sem_launch_cg_replace_f64(W.r, c->dinv, g->d_owner, W.done, W.partial, n, nf, st));
        CgFinishArgs F{W.partial, (int64_t)vg, W.scal, nullptr, 0, nf};
        HIP_TRY(sem_launch_cg_resume(&F, W.done, st));
        HIP_TRY(sem_launch_fill_f64(W.p, 0.0, nn, st));
        HIP_TRY(sem_launch_fill_f64(W.s, 0.0, nn, st));
        SEM_TRY(prime());
        SEM_TRY(iterate());
    }
    sem_status out = SEM_OK;
    for (int f = 0; f < nf; ++f) {
        const CgScalars &s = W.h_scal[f];
        const double rel = s.bb == 0.0 ? 0.0 : std::sqrt(s.rr / s.bb);
        const bool conv = s.status == 0 && std::isfinite(rel) && (P->rtol <= 0 || (rel <= P->rtol && tr[f] <= P->rtol));
        if (info) {
            info[f].iters = s.iter;
            info[f].inner_iters = 0;
            info[f].converged = conv ? 1 : 0;
            info[f].rel_res = rel;
            info[f].true_rel_res = tr[f];
        }
        if (s.status == 2) out = fail(SEM_ERR_BREAKDOWN, "CG breakdown in field %d at iteration %d", f, s.iter);
        else if (!conv && out == SEM_OK)
            out = fail(SEM_ERR_NOT_CONVERGED, "field %d: |r|/|b| = %.3e after %d iterations", f, rel, s.iter);
    }
    return out;
}

static sem_status pcg_fp64(double *x, const double *b, int nf, sem_coef c, sem_gs g, const sem_pcg_params *P,
                           sem_pcg_info *info, hipStream_t st)
{
    Work &W = c->ws;
    const double rtol[3] = {P->rtol, P->rtol, P->rtol};
    SEM_TRY(cg_run<double>(c, g, nf, x, b, P->use_x0 != 0, W.r, W.p, W.w, c->dinv, rtol, P->max_iter,
                           P->check_every, nullptr, 0, st));
    // A field counts as converged only when its true residual |b - A x| / |b| meets
    // rtol.  When the recursive residual has drifted below it, the true residual
    // (left in W.r by true_residual) replaces it and the iteration continues with
    // its search direction.
    double tr[3];
    for (int round = 0;; ++round) {
        SEM_TRY(true_residual(c, g, nf, x, b, tr, st));
        bool any = false;
        for (int f = 0; f < nf; ++f) {
            const CgScalars &s = W.h_scal[f];
            W.h_done[f] = (s.status == 0 && P->rtol > 0 && s.bb > 0 && tr[f] > P->rtol && s.iter < P->max_iter) ? 1 : 0;
            any = any || W.h_done[f];
        }
        if (!any || round >= 16) break;
        const unsigned vg = sem_vec_grid(c->n);
        HIP_TRY(hipMemcpyAsync(W.done, W.h_done, sizeof(int) * nf, hipMemcpyHostToDevice, st));
        HIP_TRY(sem_launch_cg_replace_f64(W.r, c->dinv, g->d_owner, W.done, W.partial, c->n, nf, st));
        CgFinishArgs F{W.partial, (int64_t)vg, W.scal, nullptr, 0, nf};
        HIP_TRY(sem_launch_cg_resume(&F, W.done, st));
        SEM_TRY(cg_iterate<double>(c, g, nf, x, W.r, W.p, W.w, c->dinv, P->max_iter, P->check_every, nullptr, 0, st));
    }
    CgScalars res[3];
    std::memcpy(res, W.h_scal, sizeof(CgScalars) * nf);
    sem_status out = SEM_OK;
    for (int f = 0; f < nf; ++f) {
        const CgScalars &s = res[f];
        const double rel = s.bb == 0.0 ? 0.0 : std::sqrt(s.rr / s.bb);
        const bool conv = s.status == 0 && std::isfinite(rel) && (P->rtol <= 0 || (rel <= P->rtol && tr[f] <= P->rtol));
        if (info) {
            info[f].iters = s.iter;
            info[f].inner_iters = 0;
            info[f].converged = conv ? 1 : 0;
            info[f].rel_res = rel;
            info[f].true_rel_res = tr[f];
        }
        if (s.status == 2) out = fail(SEM_ERR_BREAKDOWN, "CG breakdown in field %d at iteration %d", f, s.iter);
        else if (!conv && out == SEM_OK)
            out = fail(SEM_ERR_NOT_CONVERGED, "field %d: |r|/|b| = %.3e after %d iterations", f, rel, s.iter);
    }
    return out;
}

// Jacobi-PCG iterating in FP32 with FP64 reliable updates (residual replacement):
// the FP32 iteration runs in segments; a segment ends once its residual has dropped
// by delta (device side); then x += x32 in FP64, r = b - A64 x in FP64, the FP32
// residual is replaced by it and the iteration resumes with its search direction.
// Convergence is decided on the FP64 true residual.
static sem_status pcg_mixed_reliable(double *x, const double *b, int nf, sem_coef c, sem_gs g,
                                     const sem_pcg_params *P, sem_pcg_info *info, hipStream_t st)
{
    Work &W = c->ws;
    const int64_t n = c->n;
    const int64_t nn = n * nf;
    const unsigned vg = sem_vec_grid(n);
    // FP64 residual of the initial guess
    if (P->use_x0) {
        SEM_TRY(launch_ax<double>(c, W.w, x, nf, st));
        SEM_TRY(launch_gs<double>(W.w, nf, g, nullptr, nullptr, st));
        HIP_TRY(sem_launch_residual(W.r, b, W.w, c->dinv, n, nf, st));
    } else {
        HIP_TRY(sem_launch_fill_f64(x, 0.0, nn, st));
        HIP_TRY(hipMemcpyAsync(W.r, b, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
    }
    double bb[3];
    {
        const double *a[1] = {b};
        SEM_TRY(dots(c, g, nf, 1, a, a, bb, st));
    }
    const double delta = (P->delta > 0.0 && P->delta < 1.0) ? P->delta : 0.5;
    for (int f = 0; f < nf; ++f) {
        W.h_rel[f] = RelState{bb[f], 0.0, P->rtol, delta, 0, 0, 0};
        CgScalars s{};
        s.max_iter = P->max_iter;
        W.h_scal[f] = s;
    }
    HIP_TRY(hipMemcpyAsync(W.rel, W.h_rel, sizeof(RelState) * nf, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(W.scal, W.h_scal, sizeof(CgScalars) * nf, hipMemcpyHostToDevice, st));
    RelRestartArgs RA{W.r, W.r32, W.y32, W.p32, c->dinv32, g->d_owner, W.rel, W.partial, n, nf};
    CgFinishArgs RF{W.partial, (int64_t)vg, W.scal, nullptr, 0, nf};
    HIP_TRY(sem_launch_rel_restart(&RA, vg, st));
    HIP_TRY(sem_launch_rel_resume(&RF, W.rel, 1, st));
    RA.p32 = nullptr;  // later segments keep the search direction

    CgMatvecArgs<float> M;
    M.p = W.p32;
    M.w = W.w32;
    M.r = W.r32;
    M.dinv = c->dinv32;
    M.G = c->G32; M.B = c->B32; M.h1 = c->h1_32; M.h2 = c->h2_32;
    M.h1s = (float)c->h1s; M.h2s = (float)c->h2s;
    M.n = n;
    M.nelv = c->nelv;
    M.scal = W.scal;
    M.partial = W.partial;
    CgUpdateArgs<float> U{W.y32, W.r32, W.p32, W.w32, c->dinv32, g->d_owner, W.scal, W.partial, n, nf};
    const unsigned ug = sem_update_grid(n, 1);
    CgFinishArgs F{W.partial, (int64_t)ug, W.scal, nullptr, 0, nf};
    const int check_every = std::max(1, P->check_every);
    const int64_t max_polls = (int64_t)P->max_iter / check_every + 64 * 64;
    for (int64_t poll = 0; poll < max_polls; ++poll) {
        HIP_TRY(hipMemcpyAsync(W.h_scal, W.scal, sizeof(CgScalars) * nf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(W.h_rel, W.rel, sizeof(RelState) * nf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        bool all_stopped = true, all_done = true;
        for (int f = 0; f < nf; ++f) {
            all_stopped = all_stopped && W.h_scal[f].stop;
            all_done = all_done && W.h_rel[f].done;
        }
        if (all_done) break;
        if (all_stopped) {
            // end of a segment: accumulate x and replace the residual (fields not done)
            for (int f = 0; f < nf; ++f) W.h_done[f] = W.h_rel[f].done;
            HIP_TRY(hipMemcpyAsync(W.done, W.h_done, sizeof(int) * nf, hipMemcpyHostToDevice, st));
            HIP_TRY(sem_launch_add_f32(x, W.y32, W.done, n, nf, st));
            SEM_TRY(launch_ax<double>(c, W.w, x, nf, st));
            SEM_TRY(launch_gs<double>(W.w, nf, g, nullptr, nullptr, st));
            HIP_TRY(sem_launch_residual(W.r, b, W.w, c->dinv, n, nf, st));
            HIP_TRY(sem_launch_rel_restart(&RA, vg, st));
            HIP_TRY(sem_launch_rel_resume(&RF, W.rel, 0, st));
            continue;
        }
        for (int it = 0; it < check_every; ++it) {
            HIP_TRY(fns(c->lx).cg32(&M, c->Xh->D, nf, st));
            SEM_TRY(launch_gs<float>(W.w32, nf, g, W.scal, W.job32, st));
            HIP_TRY(sem_launch_cg_update_f32(&U, ug, st));
            HIP_TRY(sem_launch_cg_finish(&F, st));
        }
    }
    sem_status out = SEM_OK;
    for (int f = 0; f < nf; ++f) {
        const RelState &R = W.h_rel[f];
        const CgScalars &s = W.h_scal[f];
        const double rel = R.bb64 == 0.0 ? 0.0 : std::sqrt(R.rr64 / R.bb64);
        const bool conv = R.done && s.status == 0 && std::isfinite(rel) && rel <= P->rtol;
        if (info) {
            info[f].iters = R.outer;
            info[f].inner_iters = s.iter;
            info[f].converged = conv ? 1 : 0;
            info[f].rel_res = rel;
            info[f].true_rel_res = rel;  // the FP64 true residual of the returned x
        }
        if (s.status == 2) out = fail(SEM_ERR_BREAKDOWN, "CG breakdown in field %d", f);
        else if (!conv && out == SEM_OK)
            out = fail(SEM_ERR_NOT_CONVERGED, "field %d: |r|/|b| = %.3e after %d iterations", f, rel, s.iter);
    }
    return out;
}

// Flexible CG, FP64 outer iteration, preconditioned by an FP32 Jacobi-PCG solve.
static sem_status pcg_mixed(double *x, const double *b, int nf, sem_coef c, sem_gs g, const sem_pcg_params *P,
                            sem_pcg_info *info, hipStream_t st)
{
    Work &W = c->ws;
    const int64_t n = c->n;
    const int64_t nn = n * nf;
    // r = b - A x
    if (P->use_x0) {
        SEM_TRY(launch_ax<double>(c, W.w, x, nf, st));
        SEM_TRY(launch_gs<double>(W.w, nf, g, nullptr, nullptr, st));
        HIP_TRY(sem_launch_residual(W.r, b, W.w, c->dinv, n, nf, st));
    } else {
        HIP_TRY(sem_launch_fill_f64(x, 0.0, nn, st));
        HIP_TRY(hipMemcpyAsync(W.r, b, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(sem_launch_fill_f64(W.p, 0.0, nn, st));
    double bb[3], rr[3], pq_old[3] = {0, 0, 0};
    {
        const double *a[2] = {b, W.r};
        double out[6];
        SEM_TRY(dots(c, g, nf, 2, a, a, out, st));
        for (int f = 0; f < nf; ++f) { bb[f] = out[f]; rr[f] = out[nf + f]; }
    }
    int done[3] = {0, 0, 0}, status[3] = {0, 0, 0}, iters[3] = {0, 0, 0}, inner[3] = {0, 0, 0};
    for (int f = 0; f < nf; ++f) {
        if (!std::isfinite(bb[f]) || !std::isfinite(rr[f])) { done[f] = 1; status[f] = 2; }
        else if (bb[f] == 0.0 || (P->rtol > 0 && std::sqrt(rr[f] / bb[f]) <= P->rtol)) done[f] = 1;
    }
    double tr[3] = {0, 0, 0};
    int k = 0;
    for (int round = 0;; ++round) {
    for (; k < P->max_iter; ++k) {
        bool all = true;
        for (int f = 0; f < nf; ++f) all = all && done[f];
        if (all) break;
        // z = |r| * P32(r / |r|)
        for (int f = 0; f < nf; ++f) {
            const double nr = std::sqrt(rr[f]);
            W.h_fcg[2 * nf + f] = nr;
            W.h_fcg[3 * nf + f] = (done[f] || nr == 0.0) ? 0.0 : 1.0 / nr;
            W.h_done[f] = done[f];
        }
        HIP_TRY(hipMemcpyAsync(W.fcg, W.h_fcg, sizeof(double) * 4 * nf, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(W.done, W.h_done, sizeof(int) * nf, hipMemcpyHostToDevice, st));
        HIP_TRY(sem_launch_fcg_scale_down(W.r32, W.r, W.fcg + 3 * nf, W.done, n, nf, st));
        // Inner tolerance: the nominal inner_rtol, loosened on the last outer steps to
        // the reduction still needed (with a factor 0.1 of margin), at most 0.5.
        double tau[3];
        for (int f = 0; f < nf; ++f) {
            const double need = (rr[f] > 0.0) ? 0.1 * P->rtol * std::sqrt(bb[f] / rr[f]) : 0.5;
            tau[f] = std::min(0.5, std::max(P->inner_rtol, need));
        }
        SEM_TRY(cg_run<float>(c, g, nf, W.y32, W.r32, false, W.ri32, W.p32, W.w32, c->dinv32, tau,
                              P->inner_max_iter, std::max(1, P->check_every), nullptr, 0, st));
        for (int f = 0; f < nf; ++f) inner[f] += W.h_scal[f].iter;
        HIP_TRY(sem_launch_fcg_scale_up(W.z, W.y32, W.fcg + 2 * nf, n, nf, st));
        // p = z - beta p,  beta = (z, q_old) / (p_old, q_old)
        if (k == 0) {
            for (int f = 0; f < nf; ++f) W.h_fcg[f] = 0.0;
        } else {
            const double *a[1] = {W.z}, *bq[1] = {W.q};
            double zq[3];
            SEM_TRY(dots(c, g, nf, 1, a, bq, zq, st));
            for (int f = 0; f < nf; ++f) W.h_fcg[f] = pq_old[f] != 0.0 ? zq[f] / pq_old[f] : 0.0;
        }
        HIP_TRY(hipMemcpyAsync(W.fcg, W.h_fcg, sizeof(double) * nf, hipMemcpyHostToDevice, st));
        HIP_TRY(sem_launch_fcg_dir(W.p, W.z, W.fcg, W.done, n, nf, st));
        // q = A p
        SEM_TRY(launch_ax<double>(c, W.q, W.p, nf, st));
        SEM_TRY(launch_gs<double>(W.q, nf, g, nullptr, nullptr, st));
        double pq[3], pr[3];
        {
            const double *a[2] = {W.p, W.p}, *bq[2] = {W.q, W.r};
            double out[6];
            SEM_TRY(dots(c, g, nf, 2, a, bq, out, st));
            for (int f = 0; f < nf; ++f) { pq[f] = out[f]; pr[f] = out[nf + f]; }
        }
        for (int f = 0; f < nf; ++f) {
            if (done[f]) { W.h_fcg[nf + f] = 0.0; continue; }
            if (!(pq[f] > 0.0) || !std::isfinite(pq[f]) || !std::isfinite(pr[f])) {
                done[f] = 1;
                status[f] = 2;
                W.h_fcg[nf + f] = 0.0;
                continue;
            }
            W.h_fcg[nf + f] = pr[f] / pq[f];
            pq_old[f] = pq[f];
        }
        for (int f = 0; f < nf; ++f) W.h_done[f] = done[f];
        HIP_TRY(hipMemcpyAsync(W.fcg + nf, W.h_fcg + nf, sizeof(double) * nf, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(W.done, W.h_done, sizeof(int) * nf, hipMemcpyHostToDevice, st));
        HIP_TRY(sem_launch_fcg_update(x, W.r, W.p, W.q, c->dinv, W.fcg + nf, W.done, n, nf, st));
        {
            const double *a[1] = {W.r};
            double out[3];
            SEM_TRY(dots(c, g, nf, 1, a, a, out, st));
            for (int f = 0; f < nf; ++f) {
                if (done[f]) continue;
                rr[f] = out[f];
                iters[f] += 1;
                const double rel = std::sqrt(rr[f] / bb[f]);
                if (!std::isfinite(rel)) { done[f] = 1; status[f] = 2; }
                else if (P->rtol > 0 && rel <= P->rtol) done[f] = 1;
            }
        }
    }
    // verify on the true residual; fields whose recursive residual drifted below it
    // continue from the true residual (left in W.r by true_residual)
    SEM_TRY(true_residual(c, g, nf, x, b, tr, st));
    bool again = false;
    for (int f = 0; f < nf; ++f) {
        if (status[f] == 0 && bb[f] > 0.0 && tr[f] > P->rtol && k < P->max_iter) {
            done[f] = 0;
            rr[f] = tr[f] * tr[f] * bb[f];
            again = true;
        }
    }
    if (!again || round >= 16) break;
    }
    sem_status out = SEM_OK;
    for (int f = 0; f < nf; ++f) {
        const double rel = bb[f] == 0.0 ? 0.0 : std::sqrt(rr[f] / bb[f]);
        const bool conv = status[f] == 0 && std::isfinite(rel) && (P->rtol <= 0 || (rel <= P->rtol && tr[f] <= P->rtol));
        if (info) {
            info[f].iters = iters[f];
            info[f].inner_iters = inner[f];
            info[f].converged = conv ? 1 : 0;
            info[f].rel_res = rel;
            info[f].true_rel_res = tr[f];
        }
        if (status[f] == 2) out = fail(SEM_ERR_BREAKDOWN, "flexible CG breakdown in field %d", f);
        else if (!conv && out == SEM_OK)
            out = fail(SEM_ERR_NOT_CONVERGED, "field %d: |r|/|b| = %.3e after %d outer iterations", f, rel, iters[f]);
    }
    return out;
}

sem_status sem_pcg_solve(double *x, const double *b, int nfields, sem_coef coef, sem_mesh msh, sem_space Xh,
                         sem_gs gs, const sem_pcg_params *params, sem_pcg_info *info, void *stream)
{
    SEM_TRY(check_coef(coef, msh, Xh));
    if (!gs || gs->msh != msh) return fail(SEM_ERR_INVALID, "gs is NULL or built for another mesh");
    if (!params) return fail(SEM_ERR_INVALID, "params is NULL");
    if (nfields != 1 && nfields != 3) return fail(SEM_ERR_INVALID, "nfields must be 1 or 3");
    const sem_pcg_params &P = *params;
    if (P.max_iter < 1) return fail(SEM_ERR_INVALID, "max_iter must be >= 1");
    if (!std::isfinite(P.rtol)) return fail(SEM_ERR_INVALID, "rtol is not finite");
    if (P.mixed < 0 || P.mixed > 2) return fail(SEM_ERR_INVALID, "mixed must be 0, 1 or 2");
    if (P.mixed) {
        if (!(coef->flags & SEM_COEF_F32)) return fail(SEM_ERR_INVALID, "mixed solve needs a coef created with SEM_COEF_F32");
        if (P.rtol <= 0) return fail(SEM_ERR_INVALID, "mixed solve needs rtol > 0");
    }
    if (P.variant != 0 && P.variant != 1) return fail(SEM_ERR_INVALID, "variant must be 0 or 1");
    if (P.variant == 1 && P.mixed != 0) return fail(SEM_ERR_INVALID, "the single-reduction form is FP64 only (mixed = 0)");
    if (P.mixed == 1 && !(P.delta == 0.0 || (P.delta > 0.0 && P.delta < 1.0)))
        return fail(SEM_ERR_INVALID, "delta must be 0 (default) or in (0, 1)");
    if (P.mixed == 2) {
        if (!(P.inner_rtol > 0.0 && P.inner_rtol < 1.0)) return fail(SEM_ERR_INVALID, "inner_rtol must be in (0, 1)");
        if (P.inner_max_iter < 1) return fail(SEM_ERR_INVALID, "inner_max_iter must be >= 1");
    }
    const size_t bytes = (size_t)coef->n * nfields * 8;
    if (bytes == 0) return SEM_OK;
    if (!x || !b) return fail(SEM_ERR_INVALID, "x or b is NULL");
    if (overlap(x, bytes, b, bytes)) return fail(SEM_ERR_INVALID, "x and b overlap");
    hipStream_t st = S(stream);
    SEM_TRY(gs_upload(gs));
    SEM_TRY(ensure_dinv(coef, gs, st));
    SEM_TRY(ensure_work(coef, nfields, P.mixed != 0));
    if (P.mixed == 1) return pcg_mixed_reliable(x, b, nfields, coef, gs, &P, info, st);
    if (P.mixed == 2) return pcg_mixed(x, b, nfields, coef, gs, &P, info, st);
    if (P.variant == 1) return pcg_cg1(x, b, nfields, coef, gs, &P, info, st);
    return pcg_fp64(x, b, nfields, coef, gs, &P, info, st);
}

// ------------------------------------------------------------------ projection space
// Previous solutions of one scalar system, kept A-orthonormal with their images
// (Fischer's projection; the paper keeps 20 of them for its pressure solves).
struct sem_proj_s {
    sem_coef coef = nullptr;
    sem_mesh msh = nullptr;
    sem_space Xh = nullptr;
    sem_gs gs = nullptr;
    int m = 0;          // capacity
    int count = 0;      // basis vectors held
    int restarts = 0;
    int64_t n = 0;
    int device = -1;
    double *X = nullptr;   // [m][n] basis, (X_i, A X_j) = delta_ij
    double *AX = nullptr;  // [m][n] images A X_i
    double *x0 = nullptr, *r = nullptr, *d = nullptr, *w = nullptr;  // [n] scratch
    double *partial = nullptr;  // [PB][grid]
    double *out = nullptr;      // [m] device results of the inner products
    double *h_out = nullptr;    // pinned mirror
};

static void proj_free(sem_proj P)
{
    dfree(P->X); dfree(P->AX); dfree(P->x0); dfree(P->r); dfree(P->d); dfree(P->w);
    dfree(P->partial); dfree(P->out);
    if (P->h_out) (void)hipHostFree(P->h_out);
    P->h_out = nullptr;
}

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
static sem_status vdots(const VecCtx &X, const double *V, int64_t ld, int l, const double *v, double *host_out,
                        hipStream_t st)
{
    if (X.n == 0) {
        std::fill(host_out, host_out + l, 0.0);
        return SEM_OK;
    }
    // up to ARN_MAXV vectors per pass over the data; each pass's reduction also
    // yields (v, v) one slot past its rows, overwritten by the next pass
    const int64_t G = sem_arn_grid(X.n);
    for (int i0 = 0; i0 < l; i0 += ARN_MAXV) {
        const int cl = std::min(ARN_MAXV, l - i0);
        ArnArgs A{V + (int64_t)i0 * ld, ld, cl, v, nullptr, X.owner, nullptr, nullptr, X.partial, X.n};
        HIP_TRY(sem_launch_arn(&A, 0, st));
        HIP_TRY(sem_launch_arn_finish(X.partial, G, cl + 1, 0, X.out + i0, st));
    }
    HIP_TRY(hipMemcpyAsync(X.h_out, X.out, sizeof(double) * l, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(host_out, X.h_out, sizeof(double) * l);
    return SEM_OK;
}

// y = [src +] sum_i c_i V_i (mode 0: y = sum; 1: y += sum; 2: y = src + sum)
static sem_status vcomb(const VecCtx &X, double *y, const double *src, const double *V, int64_t ld, int l,
                        const double *c, int mode, hipStream_t st)
{
    int i0 = 0;
    do {
        CombArgs A{};
        A.y = y;
        A.src = src;
        A.V = V + (int64_t)i0 * ld;
        A.ld = ld;
        A.l = std::min(PB, l - i0);
        A.mode = (i0 == 0) ? mode : 1;
        for (int i = 0; i < A.l; ++i) A.c[i] = c[i0 + i];
        A.n = X.n;
        HIP_TRY(sem_launch_comb(&A, st));
        i0 += PB;
    } while (i0 < l);
    return SEM_OK;
}

static VecCtx proj_ctx(sem_proj P) { return VecCtx{P->n, P->gs->d_owner, P->partial, P->out, P->h_out}; }

static sem_status proj_dots(sem_proj P, const double *V, int l, const double *v, double *host_out, hipStream_t st)
{
    return vdots(proj_ctx(P), V, P->n, l, v, host_out, st);
}

static sem_status proj_comb(sem_proj P, double *y, const double *src, const double *V, int l, const double *c,
                            int mode, hipStream_t st)
{
    return vcomb(proj_ctx(P), y, src, V, P->n, l, c, mode, st);
}

// w = mask QQ^T A_L d
static sem_status proj_apply(sem_proj P, double *w, const double *d, hipStream_t st)
{
    SEM_TRY(launch_ax<double>(P->coef, w, d, 1, st));
    SEM_TRY(launch_gs<double>(w, 1, P->gs, nullptr, nullptr, st));
    HIP_TRY(sem_launch_mask(w, 0, P->msh->d_dir_idx, (int64_t)P->msh->dir_idx.size(), P->n, 1, st));
    return SEM_OK;
}

static sem_status proj_check(sem_proj P)
{
    if (!P) return fail(SEM_ERR_INVALID, "proj is NULL");
    return check_device(P->device);
}

static sem_status proj_project(sem_proj P, double *x0, double *r, const double *b, hipStream_t st)
{
    if (P->count == 0) {
        HIP_TRY(sem_launch_fill_f64(x0, 0.0, P->n, st));
        return proj_comb(P, r, b, nullptr, 0, nullptr, 2, st);
    }
    std::vector<double> a(P->count), na(P->count);
    SEM_TRY(proj_dots(P, P->X, P->count, b, a.data(), st));
    for (int i = 0; i < P->count; ++i) na[i] = -a[i];
    SEM_TRY(proj_comb(P, x0, nullptr, P->X, P->count, a.data(), 0, st));
    return proj_comb(P, r, b, P->AX, P->count, na.data(), 2, st);
}

static sem_status proj_update(sem_proj P, const double *x, const double *x0, int *added, hipStream_t st)
{
    *added = 0;
    const double minus1 = -1.0;
    if (P->count == P->m) {
        // full: restart the space from the latest solution alone
        P->count = 0;
        P->restarts += 1;
        SEM_TRY(proj_comb(P, P->d, x, nullptr, 0, nullptr, 2, st));
    } else {
        SEM_TRY(proj_comb(P, P->d, x, x0, 1, &minus1, 2, st));
    }
    SEM_TRY(proj_apply(P, P->w, P->d, st));
    double nrm0;
    SEM_TRY(proj_dots(P, P->d, 1, P->w, &nrm0, st));
    if (!(nrm0 > 0.0) || !std::isfinite(nrm0)) return SEM_OK;
    // classical Gram-Schmidt in the A inner product, twice
    std::vector<double> g(std::max(P->count, 1));
    for (int pass = 0; pass < 2 && P->count > 0; ++pass) {
        SEM_TRY(proj_dots(P, P->X, P->count, P->w, g.data(), st));
        for (double &v : g) v = -v;
        SEM_TRY(proj_comb(P, P->d, nullptr, P->X, P->count, g.data(), 1, st));
        SEM_TRY(proj_comb(P, P->w, nullptr, P->AX, P->count, g.data(), 1, st));
    }
    double nrm;
    SEM_TRY(proj_dots(P, P->d, 1, P->w, &nrm, st));
    // nothing new (the solution already lies in the space, to rounding)
    if (!(nrm > 1e-14 * nrm0) || !std::isfinite(nrm)) return SEM_OK;
    const double sc = 1.0 / std::sqrt(nrm);
    SEM_TRY(proj_comb(P, P->X + (int64_t)P->count * P->n, nullptr, P->d, 1, &sc, 0, st));
    SEM_TRY(proj_comb(P, P->AX + (int64_t)P->count * P->n, nullptr, P->w, 1, &sc, 0, st));
    P->count += 1;
    *added = 1;
    return SEM_OK;
}

sem_status sem_proj_create(sem_coef coef, sem_mesh msh, sem_space Xh, sem_gs gs, int max_vectors, sem_proj *proj)
{
    if (!proj) return fail(SEM_ERR_INVALID, "proj is NULL");
    *proj = nullptr;
    SEM_TRY(check_coef(coef, msh, Xh));
    if (!gs || gs->msh != msh) return fail(SEM_ERR_INVALID, "gs is NULL or built for another mesh");
    if (max_vectors < 1 || max_vectors > 256) return fail(SEM_ERR_INVALID, "max_vectors must be in 1..256");
    SEM_TRY(mesh_upload(msh));
    SEM_TRY(gs_upload(gs));
    sem_proj P = new (std::nothrow) sem_proj_s();
    if (!P) return fail(SEM_ERR_OOM, "out of host memory");
    P->coef = coef; P->msh = msh; P->Xh = Xh; P->gs = gs;
    P->m = max_vectors;
    P->n = coef->n;
    P->device = coef->device;
    const int64_t n = P->n;
    sem_status e = SEM_OK;
    if (n > 0) {
        if (e == SEM_OK) e = dalloc(&P->X, (size_t)P->m * n);
        if (e == SEM_OK) e = dalloc(&P->AX, (size_t)P->m * n);
        if (e == SEM_OK) e = dalloc(&P->x0, n);
        if (e == SEM_OK) e = dalloc(&P->r, n);
        if (e == SEM_OK) e = dalloc(&P->d, n);
        if (e == SEM_OK) e = dalloc(&P->w, n);
        if (e == SEM_OK) e = dalloc(&P->partial, (size_t)(ARN_MAXV + 1) * sem_arn_grid(n));
        if (e == SEM_OK) e = dalloc(&P->out, P->m + 1);
        if (e == SEM_OK && hipHostMalloc((void **)&P->h_out, sizeof(double) * P->m, hipHostMallocDefault) != hipSuccess)
            e = fail(SEM_ERR_OOM, "pinned host allocation failed");
    }
    if (e != SEM_OK) {
        proj_free(P);
        delete P;
        return e;
    }
    *proj = P;
    return SEM_OK;
}

sem_status sem_proj_size(sem_proj proj, int *count, int *max_vectors, int *restarts)
{
    if (!proj) return fail(SEM_ERR_INVALID, "proj is NULL");
    if (count) *count = proj->count;
    if (max_vectors) *max_vectors = proj->m;
    if (restarts) *restarts = proj->restarts;
    return SEM_OK;
}

sem_status sem_proj_reset(sem_proj proj)
{
    if (!proj) return fail(SEM_ERR_INVALID, "proj is NULL");
    proj->count = 0;
    proj->restarts = 0;
    return SEM_OK;
}

sem_status sem_proj_project(sem_proj proj, double *x0, double *r, const double *b, void *stream)
{
    SEM_TRY(proj_check(proj));
    if (proj->n == 0) return SEM_OK;
    if (!x0 || !r || !b) return fail(SEM_ERR_INVALID, "x0, r or b is NULL");
    const size_t bytes = (size_t)proj->n * 8;
    if (overlap(x0, bytes, r, bytes) || overlap(x0, bytes, b, bytes) || overlap(r, bytes, b, bytes))
        return fail(SEM_ERR_INVALID, "x0, r and b must not overlap");
    return proj_project(proj, x0, r, b, S(stream));
}

sem_status sem_proj_update(sem_proj proj, const double *x, const double *x0, int *added, void *stream)
{
    SEM_TRY(proj_check(proj));
    int dummy = 0;
    if (!added) added = &dummy;
    *added = 0;
    if (proj->n == 0) return SEM_OK;
    if (!x || !x0) return fail(SEM_ERR_INVALID, "x or x0 is NULL");
    return proj_update(proj, x, x0, added, S(stream));
}

sem_status sem_proj_solve(double *x, const double *b, sem_proj proj, const sem_pcg_params *params,
                          sem_pcg_info *info, void *stream)
{
    SEM_TRY(proj_check(proj));
    if (!params) return fail(SEM_ERR_INVALID, "params is NULL");
    if (!(params->rtol > 0.0)) return fail(SEM_ERR_INVALID, "projected solve needs rtol > 0");
    if (proj->n == 0) return SEM_OK;
    if (!x || !b) return fail(SEM_ERR_INVALID, "x or b is NULL");
    const size_t bytes = (size_t)proj->n * 8;
    if (overlap(x, bytes, b, bytes)) return fail(SEM_ERR_INVALID, "x and b overlap");
    hipStream_t st = S(stream);
    SEM_TRY(ensure_dinv(proj->coef, proj->gs, st));
    SEM_TRY(ensure_work(proj->coef, 1, params->mixed != 0));
    SEM_TRY(proj_project(proj, proj->x0, proj->r, b, st));
    double nb[2];
    SEM_TRY(proj_dots(proj, b, 1, b, &nb[0], st));
    SEM_TRY(proj_dots(proj, proj->r, 1, proj->r, &nb[1], st));
    const double bn = std::sqrt(nb[0]), rn = std::sqrt(nb[1]);
    // the correction solve A dx = r only needs |r - A dx| <= rtol |b|
    sem_pcg_params P2 = *params;
    P2.use_x0 = 0;
    sem_pcg_info i2{};
    sem_status st_solve = SEM_OK;
    if (rn > 0.0 && rn > params->rtol * bn) {
        P2.rtol = params->rtol * bn / rn;
        st_solve = sem_pcg_solve(x, proj->r, 1, proj->coef, proj->msh, proj->Xh, proj->gs, &P2, &i2, stream);
        if (st_solve != SEM_OK && st_solve != SEM_ERR_NOT_CONVERGED) return st_solve;
    } else {
        HIP_TRY(sem_launch_fill_f64(x, 0.0, proj->n, st));
    }
    const double one = 1.0;
    SEM_TRY(proj_comb(proj, x, nullptr, proj->x0, 1, &one, 1, st));
    double tr = 0.0;
    SEM_TRY(true_residual(proj->coef, proj->gs, 1, x, b, &tr, st));
    int added = 0;
    SEM_TRY(proj_update(proj, x, proj->x0, &added, st));
    if (info) {
        info->iters = i2.iters;
        info->inner_iters = i2.inner_iters;
        info->rel_res = bn > 0.0 ? i2.rel_res * (rn / bn) : 0.0;
        info->true_rel_res = tr;
        info->converged = (tr <= params->rtol) ? 1 : 0;
        if (rn <= params->rtol * bn) info->rel_res = bn > 0.0 ? rn / bn : 0.0;
    }
    if (st_solve == SEM_ERR_NOT_CONVERGED) return st_solve;
    return SEM_OK;
}

void sem_proj_destroy(sem_proj proj)
{
    if (!proj) return;
    proj_free(proj);
    delete proj;
}

// ------------------------------------------------------------------ two-level Schwarz
// Setup (host + a few launches): element lengths from the geometric factors, the
// 1-D extended operators and their eigen-decompositions, the coarse vertices and
// the Galerkin coarse matrix from eight probe applications of A_L.
static sem_status schwarz_setup(sem_coef c, sem_gs g, hipStream_t st)
{
    SchwarzData &Z = c->sz;
    if (Z.valid && Z.gs == (const void *)g) return SEM_OK;
    if (c->h1 || c->h2) return fail(SEM_ERR_UNSUPPORTED, "the Schwarz preconditioner needs scalar h1 and h2");
    Z.release();
    const int lx = c->lx, N = lx - 1, lx3 = lx * lx * lx;
    const int64_t E = c->nelv, n = c->n;
    const sem_space Xh = c->Xh;
    // element lengths: L_d = 2 / sqrt(mean over the element of G_dd / B), the sums
    // formed on the device
    std::vector<double> gb((size_t)3 * E);
    {
        double *d_gb = nullptr;
        SEM_TRY(dalloc(&d_gb, gb.size()));
        const hipError_t e1 = sem_launch_elem_gb(c->G, c->B, d_gb, E, lx3, st);
        const hipError_t e2 = e1 == hipSuccess
                                  ? hipMemcpyAsync(gb.data(), d_gb, sizeof(double) * gb.size(), hipMemcpyDeviceToHost, st)
                                  : e1;
        const hipError_t e3 = e2 == hipSuccess ? hipStreamSynchronize(st) : e2;
        dfree(d_gb);
        HIP_TRY(e3);
    }
    std::vector<double> Kref((size_t)lx * lx, 0.0);
    for (int m = 0; m < lx; ++m)
        for (int q = 0; q < lx; ++q)
            for (int i = 0; i < lx; ++i) Kref[m * lx + q] += Xh->w[i] * Xh->D[i * lx + m] * Xh->D[i * lx + q];
    const double dref = Xh->xi[1] - Xh->xi[0];
    std::vector<double> S((size_t)E * 3 * lx * lx), lam((size_t)E * 3 * lx);
    semh::parallel_for(E, [&](int64_t e0, int64_t e1) {
        std::vector<double> a((size_t)lx * lx), V((size_t)lx * lx), l(lx), M(lx);
        for (int64_t e = e0; e < e1; ++e) {
            for (int d = 0; d < 3; ++d) {
                const double L = 2.0 / std::sqrt(gb[(size_t)e * 3 + d] / lx3), J = L / 2.0, h = J * dref;
                for (int i = 0; i < lx; ++i) M[i] = Xh->w[i] * J;
                M[0] += h / 2.0;
                M[N] += h / 2.0;
                // C = M^{-1/2} K M^{-1/2}, K = Kref / J + 1/h on the two face diagonals
                for (int i = 0; i < lx; ++i)
                    for (int q = 0; q < lx; ++q) {
                        double k = Kref[i * lx + q] / J;
                        if (i == q && (i == 0 || i == N)) k += 1.0 / h;
                        a[i * lx + q] = k / std::sqrt(M[i] * M[q]);
                    }
                semh::sym_eig(lx, a.data(), V.data(), l.data());
                double *Sd = &S[((size_t)e * 3 + d) * lx * lx];
                for (int i = 0; i < lx; ++i)
                    for (int m = 0; m < lx; ++m) Sd[i * lx + m] = V[i * lx + m] / std::sqrt(M[i]);
                for (int m = 0; m < lx; ++m) lam[((size_t)e * 3 + d) * lx + m] = l[m];
            }
        }
    }, 64);
    // trilinear corner functions at the GLL points, corner c = a + 2 b + 4 cc
    std::vector<double> phi((size_t)8 * lx3);
    for (int cc = 0; cc < 2; ++cc)
        for (int bb = 0; bb < 2; ++bb)
            for (int aa = 0; aa < 2; ++aa) {
                const int c8 = aa + 2 * bb + 4 * cc;
                auto l1 = [&](int side, int i) { return side ? (1.0 + Xh->xi[i]) / 2.0 : (1.0 - Xh->xi[i]) / 2.0; };
                for (int k = 0; k < lx; ++k)
                    for (int j = 0; j < lx; ++j)
                        for (int i = 0; i < lx; ++i)
                            phi[(size_t)c8 * lx3 + i + lx * (j + lx * k)] = l1(aa, i) * l1(bb, j) * l1(cc, k);
            }
    std::vector<double> lin((size_t)2 * lx);
    for (int i = 0; i < lx; ++i) {
        lin[i] = (1.0 - Xh->xi[i]) / 2.0;
        lin[lx + i] = (1.0 + Xh->xi[i]) / 2.0;
    }
    // coarse vertices: the global ids of the element corners
    const sem_mesh msh = c->msh;
    std::vector<int64_t> cg((size_t)E * 8);
    int corner[8];
    for (int c8 = 0; c8 < 8; ++c8) {
        const int i = (c8 & 1) ? N : 0, j = (c8 & 2) ? N : 0, k = (c8 & 4) ? N : 0;
        corner[c8] = i + lx * (j + lx * k);
    }
    for (int64_t e = 0; e < E; ++e)
        for (int c8 = 0; c8 < 8; ++c8) cg[e * 8 + c8] = msh->glb[e * lx3 + corner[c8]];
    std::vector<int64_t> vid(cg);
    std::sort(vid.begin(), vid.end());
    vid.erase(std::unique(vid.begin(), vid.end()), vid.end());
    const int64_t nv = (int64_t)vid.size();
    std::vector<int32_t> cvert((size_t)E * 8);
    std::vector<uint8_t> vdir(nv, 0);
    for (int64_t q = 0; q < E * 8; ++q) {
        cvert[q] = (int32_t)(std::lower_bound(vid.begin(), vid.end(), cg[q]) - vid.begin());
        const int64_t e = q / 8;
        if (!msh->dir.empty() && msh->dir[e * lx3 + corner[q % 8]]) vdir[cvert[q]] = 1;
    }
    std::vector<int64_t> vptr(nv + 1, 0);
    for (int64_t q = 0; q < E * 8; ++q) vptr[cvert[q] + 1] += 1;
    for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
    std::vector<int32_t> vidx(E * 8);
    {
        std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
        for (int64_t q = 0; q < E * 8; ++q) vidx[fill[cvert[q]]++] = (int32_t)q;  // ascending e
    }
    // device data
    SEM_TRY(dalloc(&Z.S, S.size()));
    SEM_TRY(dalloc(&Z.lam, lam.size()));
    SEM_TRY(dalloc(&Z.phi, phi.size()));
    SEM_TRY(dalloc(&Z.lin, lin.size()));
    SEM_TRY(dalloc(&Z.cvert, cvert.size()));
    SEM_TRY(dalloc(&Z.v_ptr, vptr.size()));
    SEM_TRY(dalloc(&Z.v_idx, vidx.size()));
    SEM_TRY(dalloc(&Z.v_dir, vdir.size()));
    SEM_TRY(dalloc(&Z.part, (size_t)E * 8));
    SEM_TRY(dalloc(&Z.mult, (size_t)n));
    HIP_TRY(hipMemcpy(Z.S, S.data(), S.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.lam, lam.data(), lam.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.phi, phi.data(), phi.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.lin, lin.data(), lin.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.cvert, cvert.data(), cvert.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.v_ptr, vptr.data(), vptr.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.v_idx, vidx.data(), vidx.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.v_dir, vdir.data(), vdir.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.mult, g->m.mult.data(), (size_t)n, hipMemcpyHostToDevice));
    // Galerkin coarse matrix: element blocks A0_e[c'][c] = phi_c'^T A_L phi_c from probes
    SEM_TRY(ensure_work(c, 1, false));
    Work &W = c->ws;
    std::vector<double> Ae((size_t)E * 64), pe((size_t)E * 8);
    for (int c8 = 0; c8 < 8; ++c8) {
        HIP_TRY(sem_launch_probe(W.r, Z.phi, c8, E, lx3, st));
        SEM_TRY(launch_ax<double>(c, W.w, W.r, 1, st));
        CornerArgs CA{W.w, nullptr, Z.phi, Z.part, E, lx3};
        HIP_TRY(sem_launch_corner(&CA, st));
        HIP_TRY(hipMemcpyAsync(pe.data(), Z.part, sizeof(double) * E * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int64_t e = 0; e < E; ++e)
            for (int c2 = 0; c2 < 8; ++c2) Ae[(size_t)e * 64 + c2 * 8 + c8] = pe[e * 8 + c2];
    }
    // assemble row by row (rows in parallel): row v sums, per column, the element
    // blocks of the elements at v in ascending element order (v_idx lists them so);
    // columns ascending; Dirichlet rows and columns dropped, Dirichlet vertices keep
    // an identity row
    int64_t maxdeg = 1;
    for (int64_t v = 0; v < nv; ++v) maxdeg = std::max<int64_t>(maxdeg, vptr[v + 1] - vptr[v]);
    auto row_entries = [&](int64_t v, int32_t *cols, double *vals) -> int {
        if (vdir[v]) {
            cols[0] = (int32_t)v;
            vals[0] = 1.0;
            return 1;
        }
        int k = 0;
        for (int64_t q = vptr[v]; q < vptr[v + 1]; ++q) {
            const int64_t e = vidx[q] / 8;
            const int c2 = (int)(vidx[q] % 8);
            for (int c8 = 0; c8 < 8; ++c8) {
                const int32_t cc = cvert[e * 8 + c8];
                if (vdir[cc]) continue;
                int i = 0;
                while (i < k && cols[i] != cc) ++i;
                if (i == k) {
                    cols[k] = cc;
                    vals[k] = 0.0;
                    ++k;
                }
                vals[i] += Ae[(size_t)e * 64 + c2 * 8 + c8];
            }
        }
        for (int i = 1; i < k; ++i)  // insertion sort by column
            for (int j2 = i; j2 > 0 && cols[j2 - 1] > cols[j2]; --j2) {
                std::swap(cols[j2 - 1], cols[j2]);
                std::swap(vals[j2 - 1], vals[j2]);
            }
        return k;
    };
    std::vector<int64_t> rp(nv + 1, 0);
    semh::parallel_for(nv, [&](int64_t v0, int64_t v1) {
        std::vector<int32_t> cols((size_t)8 * maxdeg);
        std::vector<double> vals((size_t)8 * maxdeg);
        for (int64_t v = v0; v < v1; ++v) rp[v + 1] = row_entries(v, cols.data(), vals.data());
    }, 1024);
    for (int64_t v = 0; v < nv; ++v) rp[v + 1] += rp[v];
    std::vector<int32_t> ci((size_t)rp[nv]);
    std::vector<double> val((size_t)rp[nv]), dg(nv, 1.0);
    semh::parallel_for(nv, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v) {
            const int k = row_entries(v, ci.data() + rp[v], val.data() + rp[v]);
            for (int i = 0; i < k; ++i)
                if (ci[rp[v] + i] == v) dg[v] = val[rp[v] + i];
        }
    }, 1024);
    for (double &d : dg) d = (d != 0.0) ? 1.0 / d : 0.0;
    // ELL form, column-major: entry w of row v at w * nv + v; short rows padded with
    // value 0 and the row's own column
    int width = 1;
    for (int64_t v = 0; v < nv; ++v) width = std::max(width, (int)(rp[v + 1] - rp[v]));
    std::vector<int32_t> eci((size_t)width * nv);
    std::vector<double> evl((size_t)width * nv, 0.0);
    for (int64_t v = 0; v < nv; ++v)
        for (int w = 0; w < width; ++w) {
            const int64_t q = rp[v] + w;
            const bool in = q < rp[v + 1];
            eci[(size_t)w * nv + v] = in ? ci[q] : (int32_t)v;
            evl[(size_t)w * nv + v] = in ? val[q] : 0.0;
        }
    SEM_TRY(dalloc(&Z.ell_ci, eci.size()));
    SEM_TRY(dalloc(&Z.ell_val, evl.size()));
    SEM_TRY(dalloc(&Z.dinv0, (size_t)nv));
    SEM_TRY(dalloc(&Z.cv, (size_t)6 * nv));
    SEM_TRY(dalloc(&Z.cpart, (size_t)3 * ((nv + 255) / 256)));
    HIP_TRY(hipMemcpy(Z.ell_ci, eci.data(), eci.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.ell_val, evl.data(), evl.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.dinv0, dg.data(), dg.size() * 8, hipMemcpyHostToDevice));
    Z.width = width;
    Z.nv = nv;
    Z.gs = g;
    Z.valid = true;
    return SEM_OK;
}

// z = M^{-1} r: local solves summed over shared points and averaged, plus P e0 from
// coarse_iters Jacobi-CG steps on A0 e0 = P^T r; masked.  r assembled and masked.
static sem_status schwarz_apply(sem_coef c, sem_gs g, double *z, const double *r, int coarse_iters, hipStream_t st)
{
    SchwarzData &Z = c->sz;
    const int lx = c->lx;
    const FdmArgs F{z, r, Z.S, Z.lam, g->d_owner, Z.lin, Z.part, c->h1s, c->h2s, c->nelv};
    HIP_TRY(fns(lx).fdm(&F, st));
    SEM_TRY(launch_gs<double>(z, 1, g, nullptr, nullptr, st));
    const int64_t nv = Z.nv;
    double *x0 = Z.cv;
    const CoarseArgs CC{Z.ell_ci, Z.ell_val, Z.width, Z.dinv0, Z.part, Z.v_ptr, Z.v_idx, Z.v_dir,
                        x0, Z.cv + nv, Z.cv + 2 * nv, Z.cv + 3 * nv, Z.cv + 4 * nv, Z.cv + 5 * nv, Z.cpart, nv};
    HIP_TRY(sem_launch_coarse_cg(&CC, coarse_iters, st));
    const ProlongArgs PA{z, Z.mult, Z.lin, x0, Z.cvert, c->nelv};
    HIP_TRY(fns(lx).prolong(&PA, st));
    HIP_TRY(sem_launch_mask(z, 0, c->msh->d_dir_idx, (int64_t)c->msh->dir_idx.size(), c->n, 1, st));
    return SEM_OK;
}

sem_status sem_schwarz_apply(double *z, const double *r, sem_coef coef, sem_mesh msh, sem_space Xh, sem_gs gs,
                             int coarse_iters, void *stream)
{
    SEM_TRY(check_coef(coef, msh, Xh));
    if (!gs || gs->msh != msh) return fail(SEM_ERR_INVALID, "gs is NULL or built for another mesh");
    if (coarse_iters < 0 || coarse_iters > 10000) return fail(SEM_ERR_INVALID, "coarse_iters must be in 0..10000");
    const size_t bytes = (size_t)coef->n * 8;
    if (bytes == 0) return SEM_OK;
    if (!z || !r) return fail(SEM_ERR_INVALID, "z or r is NULL");
    if (overlap(z, bytes, r, bytes)) return fail(SEM_ERR_INVALID, "z and r overlap");
    hipStream_t st = S(stream);
    SEM_TRY(gs_upload(gs));
    SEM_TRY(mesh_upload(msh));
    SEM_TRY(schwarz_setup(coef, gs, st));
    return schwarz_apply(coef, gs, z, r, coarse_iters, st);
}

// ------------------------------------------------------------------ flexible GMRES
static sem_status gmres_apply(sem_coef c, sem_gs g, double *w, const double *z, hipStream_t st)
{
    SEM_TRY(launch_ax<double>(c, w, z, 1, st));
    SEM_TRY(launch_gs<double>(w, 1, g, nullptr, nullptr, st));
    HIP_TRY(sem_launch_mask(w, 0, c->msh->d_dir_idx, (int64_t)c->msh->dir_idx.size(), c->n, 1, st));
    return SEM_OK;
}

// z = M^{-1} v (0: point Jacobi; 1: two-level Schwarz)
static sem_status gmres_precond(sem_coef c, sem_gs g, const sem_gmres_params *P, double *z, const double *v,
                                hipStream_t st)
{
    if (P->precond == 1) return schwarz_apply(c, g, z, v, P->coarse_iters > 0 ? P->coarse_iters : 10, st);
    HIP_TRY(sem_launch_hadamard(z, c->dinv, v, c->n, st));
    return SEM_OK;
}

// One Arnoldi orthogonalisation of w against V_0..V_{m-1} (m <= ARN_MAXV) by classical
// Gram-Schmidt run twice, in three passes over the data and one host sync:
//   h = V^T w (and |w|^2);  w' = w - V h, h2 = V^T w', |w'|^2;
//   w'' = (w' - V h2) / |w''|, with |w''|^2 = |w'|^2 - |h2|^2.
// out holds two result rows of stride ostride (>= m + 3) on the device; on return
// h[i] = h_i + h2_i and *hn = |w''| (0 when w lies in the span: w'' is then 0).
static sem_status arnoldi_step(const VecCtx &X, const double *V, int64_t n, int m, double *w, double *out,
                               int ostride, double *h, double *hn, hipStream_t st)
{
    const int64_t G = sem_arn_grid(n);
    double *o1 = out, *o2 = out + ostride;
    ArnArgs A{V, n, m, w, w, X.owner, nullptr, nullptr, X.partial, n};
    HIP_TRY(sem_launch_arn(&A, 0, st));
    HIP_TRY(sem_launch_arn_finish(X.partial, G, m + 1, 0, o1, st));
    A.coef = o1;
    HIP_TRY(sem_launch_arn(&A, 1, st));
    HIP_TRY(sem_launch_arn_finish(X.partial, G, m + 1, 1, o2, st));
    A.coef = o2;
    A.scale = o2 + m + 2;
    HIP_TRY(sem_launch_arn(&A, 2, st));
    HIP_TRY(hipMemcpyAsync(X.h_out, out, sizeof(double) * (ostride + m + 3), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < m; ++i) h[i] = X.h_out[i] + X.h_out[ostride + i];
    *hn = X.h_out[ostride + m + 1];
    return SEM_OK;
}

// Apply the rotations 0..k-1 to column col (entries 0..k+1), then annihilate
// col[k+1] with a new rotation k and rotate g.  False on a zero or non-finite pivot.
static bool givens_column(double *col, int k, std::vector<double> &cs, std::vector<double> &sn,
                          std::vector<double> &gv)
{
    for (int i = 0; i < k; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
    }
    const double den = std::hypot(col[k], col[k + 1]);
    if (!(den > 0.0) || !std::isfinite(den)) return false;
    cs[k] = col[k] / den;
    sn[k] = col[k + 1] / den;
    col[k] = den;
    col[k + 1] = 0.0;
    gv[k + 1] = -sn[k] * gv[k];
    gv[k] = cs[k] * gv[k];
    return true;
}

// One GMRES cycle (restart m <= ARN_MAXV) with the delayed two-pass Gram-Schmidt
// step: V_0 = r / beta on entry.  At step j the basis vector u_j = V_j has been
// orthogonalised once; its second pass is made together with the first pass for
// w = A M^{-1} u_j (two passes over V_0..V_j, one host sync).  u_j then becomes the
// final q_j, and column j-1 of the Hessenberg matrix is completed with
// u_j = Q a + rho q_j; column j is tentative until the next step, and the cycle's
// last column is completed by one extra dot pass.  The stopping test uses the
// tentative column (it differs from the final one at rounding level).  On return the
// rotated columns 0..jj-1 are in H and g in gv.
static sem_status gmres_cycle_dcgs(sem_coef c, sem_gs g, const sem_gmres_params *P, const VecCtx &X, double *V,
                                   double *Z, int m, double beta, double bn, int &total, int &jj, bool &breakdown,
                                   std::vector<double> &H, std::vector<double> &gv, std::vector<double> &cs,
                                   std::vector<double> &sn, hipStream_t st)
{
    const int64_t n = X.n;
    const int64_t G = sem_arn_grid(n);
    std::vector<double> prev(m + 2, 0.0), col(m + 2, 0.0), t(m + 2, 0.0);
    double prev_nu = 0.0;
    std::fill(gv.begin(), gv.end(), 0.0);
    jj = 0;
    for (int j = 0; j < m && total < P->max_iter; ++j) {
        double *Vj = V + (int64_t)j * n, *Vn = V + (int64_t)(j + 1) * n, *Zj = Z + (int64_t)j * n;
        SEM_TRY(gmres_precond(c, g, P, Zj, Vj, st));
        SEM_TRY(gmres_apply(c, g, Vn, Zj, st));
        const int nq = 2 * j + 3;
        DcgsArgs D{V, n, j, Vj, Vn, X.owner, X.out + nq, X.partial, n};
        HIP_TRY(sem_launch_dcgs(&D, 0, st));
        HIP_TRY(sem_launch_dcgs_finish(X.partial, G, j, X.out, st));
        HIP_TRY(sem_launch_dcgs(&D, 1, st));
        HIP_TRY(hipMemcpyAsync(X.h_out, X.out, sizeof(double) * (nq + 2 * j + 6), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        total += 1;
        const double *a = X.h_out, *bq = X.h_out + j + 1, *cf = X.h_out + nq;
        const double rho = cf[2 * j + 3], gam = cf[2 * j + 4], nu = cf[2 * j + 5];
        if (j == 0) {
            gv[0] = beta * rho;  // r = beta u_0 = beta rho q_0
        } else {
            for (int i = 0; i < j; ++i) col[i] = prev[i] + prev_nu * a[i];
            col[j] = prev_nu * rho;
            if (!givens_column(col.data(), j - 1, cs, sn, gv)) {
                breakdown = true;
                jj = j - 1;
                return SEM_OK;
            }
            for (int i = 0; i < j; ++i) H[(size_t)i * m + (j - 1)] = col[i];
        }
        // tentative column j: A z_j = Q b + gamma q_j + nu u_{j+1}
        for (int i = 0; i < j; ++i) prev[i] = bq[i];
        prev[j] = gam;
        prev_nu = nu;
        jj = j + 1;
        for (int i = 0; i <= j; ++i) t[i] = prev[i];
        for (int i = 0; i < j; ++i) {
            const double tt = cs[i] * t[i] + sn[i] * t[i + 1];
            t[i + 1] = -sn[i] * t[i] + cs[i] * t[i + 1];
            t[i] = tt;
        }
        const double den = std::hypot(t[j], nu);
        const double est = den > 0.0 ? std::fabs(nu / den * gv[j]) : 0.0;
        const bool last = !(est > P->rtol * bn) || !(nu > 1e-300) || total >= P->max_iter || j == m - 1;
        if (last) {
            // complete column j: u_{j+1} = [q_0..q_j] a' + rho' q_{j+1}
            ArnArgs A{V, n, j + 1, Vn, Vn, X.owner, nullptr, nullptr, X.partial, n};
            HIP_TRY(sem_launch_arn(&A, 0, st));
            HIP_TRY(sem_launch_arn_finish(X.partial, G, j + 2, 0, X.out, st));
            HIP_TRY(hipMemcpyAsync(X.h_out, X.out, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            double rr = X.h_out[j + 1];
            for (int i = 0; i <= j; ++i) rr = std::fma(-X.h_out[i], X.h_out[i], rr);
            const double rho1 = rr > 0.0 ? std::sqrt(rr) : 0.0;
            for (int i = 0; i <= j; ++i) col[i] = prev[i] + nu * X.h_out[i];
            col[j + 1] = nu * rho1;
            if (!givens_column(col.data(), j, cs, sn, gv)) {
                breakdown = true;
                jj = j;
                return SEM_OK;
            }
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = col[i];
            return SEM_OK;
        }
    }
    return SEM_OK;
}

static sem_status gmres_run(double *x, const double *b, sem_coef c, sem_gs g, const sem_gmres_params *P,
                            sem_pcg_info *info, hipStream_t st)
{
    Work &W = c->ws;
    const int64_t n = c->n;
    const int m = P->restart;
    if (W.gm_m < m) {
        dfree(W.gm); dfree(W.gm_part); dfree(W.gm_out);
        if (W.gm_hout) (void)hipHostFree(W.gm_hout);
        W.gm_hout = nullptr;
        W.gm_m = 0;
        SEM_TRY(dalloc(&W.gm, (size_t)(2 * m + 2) * n));
        SEM_TRY(dalloc(&W.gm_part, std::max((size_t)PB * sem_vec_grid(n), (size_t)(2 * ARN_MAXV + 3) * sem_arn_grid(n))));
        const size_t nout = (size_t)std::max(2 * (m + 3), 4 * m + 16);
        SEM_TRY(dalloc(&W.gm_out, nout));
        HIP_TRY(hipHostMalloc((void **)&W.gm_hout, sizeof(double) * nout, hipHostMallocDefault));
        W.gm_m = m;
    }
    double *V = W.gm;                          // V_0 .. V_m
    double *Z = W.gm + (int64_t)(m + 1) * n;   // Z_0 .. Z_{m-1}
    double *wv = Z + (int64_t)m * n;           // work vector
    const VecCtx X{n, g->d_owner, W.gm_part, W.gm_out, W.gm_hout};
    double bb;
    SEM_TRY(vdots(X, b, n, 1, b, &bb, st));
    const double bn = std::sqrt(bb);
    if (!P->use_x0) HIP_TRY(sem_launch_fill_f64(x, 0.0, n, st));
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), h(m + 1), h2(m + 1), y(m);
    int total = 0, cycles = 0;
    double rel = 0.0;
    bool breakdown = false;
    for (;;) {
        // true residual r = b - A x into V_0 (zero on Dirichlet points)
        SEM_TRY(gmres_apply(c, g, wv, x, st));
        HIP_TRY(sem_launch_residual(V, b, wv, c->dinv, n, 1, st));
        double rr;
        SEM_TRY(vdots(X, V, n, 1, V, &rr, st));
        const double beta = std::sqrt(rr);
        rel = bn > 0.0 ? beta / bn : 0.0;
        if (!std::isfinite(rel)) { breakdown = true; break; }
        if (rel <= P->rtol || total >= P->max_iter || breakdown) break;
        cycles += 1;
        const double inv = 1.0 / beta;
        SEM_TRY(vcomb(X, V, nullptr, V, n, 1, &inv, 0, st));
        int jj = 0;
        if (m <= ARN_MAXV) {
            SEM_TRY(gmres_cycle_dcgs(c, g, P, X, V, Z, m, beta, bn, total, jj, breakdown, H, gv, cs, sn, st));
        } else {
            std::fill(gv.begin(), gv.end(), 0.0);
            gv[0] = beta;
            for (int j = 0; j < m && total < P->max_iter; ++j) {
                double *Vj = V + (int64_t)j * n, *Vn = V + (int64_t)(j + 1) * n, *Zj = Z + (int64_t)j * n;
                SEM_TRY(gmres_precond(c, g, P, Zj, Vj, st));
                SEM_TRY(gmres_apply(c, g, Vn, Zj, st));
                // classical Gram-Schmidt against V_0..V_j, twice; V_{j+1} normalised
                double hn;
                if (j + 1 <= ARN_MAXV) {
                    SEM_TRY(arnoldi_step(X, V, n, j + 1, Vn, W.gm_out, m + 3, h.data(), &hn, st));
                } else {
                    SEM_TRY(vdots(X, V, n, j + 1, Vn, h.data(), st));
                    for (int i = 0; i <= j; ++i) h2[i] = -h[i];
                    SEM_TRY(vcomb(X, Vn, nullptr, V, n, j + 1, h2.data(), 1, st));
                    SEM_TRY(vdots(X, V, n, j + 1, Vn, h2.data(), st));
                    for (int i = 0; i <= j; ++i) {
                        h[i] += h2[i];
                        h2[i] = -h2[i];
                    }
                    SEM_TRY(vcomb(X, Vn, nullptr, V, n, j + 1, h2.data(), 1, st));
                    double hh;
                    SEM_TRY(vdots(X, Vn, n, 1, Vn, &hh, st));
                    hn = std::sqrt(hh);
                    if (hn > 1e-300) {
                        const double ih = 1.0 / hn;
                        SEM_TRY(vcomb(X, Vn, nullptr, Vn, n, 1, &ih, 0, st));
                    }
                }
                total += 1;
                jj = j + 1;
                // rotate column j with the earlier Givens rotations, then annihilate H[j+1][j]
                for (int i = 0; i < j; ++i) {
                    const double t = cs[i] * h[i] + sn[i] * h[i + 1];
                    h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
                    h[i] = t;
                }
                const double den = std::hypot(h[j], hn);
                if (!(den > 0.0) || !std::isfinite(den)) { breakdown = true; jj = j; break; }
                cs[j] = h[j] / den;
                sn[j] = hn / den;
                h[j] = den;
                gv[j + 1] = -sn[j] * gv[j];
                gv[j] = cs[j] * gv[j];
                for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
                if (std::fabs(gv[j + 1]) <= P->rtol * bn || hn <= 1e-300) break;  // converged or invariant space
            }
        }
        if (jj == 0) break;
        // y = R^{-1} g (upper triangular), x += Z y
        for (int i = jj - 1; i >= 0; --i) {
            double sacc = gv[i];
            for (int k = i + 1; k < jj; ++k) sacc -= H[(size_t)i * m + k] * y[k];
            y[i] = sacc / H[(size_t)i * m + i];
        }
        SEM_TRY(vcomb(X, x, nullptr, Z, n, jj, y.data(), 1, st));
        if (breakdown) break;
    }
    HIP_TRY(hipStreamSynchronize(st));
    const bool conv = !breakdown && rel <= P->rtol;
    if (info) {
        info->iters = total;
        info->inner_iters = cycles;
        info->converged = conv ? 1 : 0;
        info->rel_res = rel;
        info->true_rel_res = rel;
    }
    if (breakdown) return fail(SEM_ERR_BREAKDOWN, "GMRES breakdown after %d steps", total);
    if (!conv) return fail(SEM_ERR_NOT_CONVERGED, "|r|/|b| = %.3e after %d GMRES steps", rel, total);
    return SEM_OK;
}

sem_status sem_gmres_solve(double *x, const double *b, sem_coef coef, sem_mesh msh, sem_space Xh, sem_gs gs,
                           const sem_gmres_params *params, sem_pcg_info *info, void *stream)
{
    SEM_TRY(check_coef(coef, msh, Xh));
    if (!gs || gs->msh != msh) return fail(SEM_ERR_INVALID, "gs is NULL or built for another mesh");
    if (!params) return fail(SEM_ERR_INVALID, "params is NULL");
    const sem_gmres_params &P = *params;
    if (!(P.rtol > 0.0) || !std::isfinite(P.rtol)) return fail(SEM_ERR_INVALID, "rtol must be > 0");
    if (P.max_iter < 1) return fail(SEM_ERR_INVALID, "max_iter must be >= 1");
    if (P.restart < 1 || P.restart > 200) return fail(SEM_ERR_INVALID, "restart must be in 1..200");
    if (P.precond != 0 && P.precond != 1) return fail(SEM_ERR_INVALID, "precond must be 0 or 1");
    if (P.coarse_iters < 0 || P.coarse_iters > 10000) return fail(SEM_ERR_INVALID, "coarse_iters must be in 0..10000");
    const size_t bytes = (size_t)coef->n * 8;
    if (bytes == 0) return SEM_OK;
    if (!x || !b) return fail(SEM_ERR_INVALID, "x or b is NULL");
    if (overlap(x, bytes, b, bytes)) return fail(SEM_ERR_INVALID, "x and b overlap");
    hipStream_t st = S(stream);
    SEM_TRY(gs_upload(gs));
    SEM_TRY(mesh_upload(msh));
    SEM_TRY(ensure_dinv(coef, gs, st));
    SEM_TRY(ensure_work(coef, 1, false));
    if (P.precond == 1) SEM_TRY(schwarz_setup(coef, gs, st));
    return gmres_run(x, b, coef, gs, &P, info, st);
}

}  // extern "C"
