// sem_noalloc.hip -- sem_pcg_solve_noalloc: the FP64 Jacobi-PCG solve of
// sem_pcg_solve (the velocity solve of Section 4 of arXiv 2107.01243) run on a fixed
// device workspace, for callers that cannot allocate device memory.
//
// The workspace is the file-scope device array `scratch` below.  Every GPU the
// library runs on holds its own copy for the life of the process.  Host code never
// uses the array's name as an address: the first call on a device looks the array
// up with hipGetSymbolAddress (with that device current) and keeps the pointer per
// device; kernels receive that pointer.  All calls on one GPU share the array, so
// calls that overlap in time on one GPU (two host threads, or two streams) race.
#include "sem_internal.h"

#include <mutex>

using namespace semi;

namespace {

constexpr int64_t kMaxPoints = SEM_NOALLOC_MAX_POINTS;  // n_p * nfields
constexpr int64_t kPartial = 1 << 17;                   // CG reduction partials (doubles)
constexpr int64_t kSmall = 512;                         // scalars, job, dots, flags (doubles)
// offsets in doubles: r, p, w (n_p * nfields each), dinv (n_p), partials, small block
constexpr int64_t kOffR = 0;
constexpr int64_t kOffP = kOffR + kMaxPoints;
constexpr int64_t kOffW = kOffP + kMaxPoints;
constexpr int64_t kOffDinv = kOffW + kMaxPoints;
constexpr int64_t kOffPartial = kOffDinv + kMaxPoints;
constexpr int64_t kOffSmall = kOffPartial + kPartial;
constexpr int64_t kWords = kOffSmall + kSmall;
// inside the small block (doubles): CgScalars[3], AlphaJob, dots[12], done[3]
constexpr int64_t kSmallScal = 0;
constexpr int64_t kSmallJob = 64;
constexpr int64_t kSmallDots = 128;
constexpr int64_t kSmallDone = 192;
static_assert(3 * sizeof(CgScalars) <= 8 * (kSmallJob - kSmallScal), "CgScalars block");
static_assert(sizeof(AlphaJob) <= 8 * (kSmallDots - kSmallJob), "AlphaJob slot");
static_assert(3 * sizeof(int) <= 8 * (kSmall - kSmallDone), "flag block");

}  // namespace

static_assert(kWords * 8 == SEM_NOALLOC_WORKSPACE_BYTES, "sem.h states the workspace size");

static __device__ __align__(256) double scratch[kWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device).
sem_status scratch_of(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(SEM_ERR_UNSUPPORTED, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        double *p = nullptr;
        HIP_TRY(hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SEM_ERR_HIP, "hipGetSymbolAddress returned NULL for the workspace");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SEM_OK;
}

}  // namespace

extern "C" sem_status sem_pcg_solve_noalloc(double *x, const double *b, int nfields, sem_coef coef, sem_mesh msh,
                                            sem_space Xh, sem_gs gs, const sem_pcg_params *params,
                                            sem_pcg_info *info, void *stream)
{
    SEM_TRY(check_pcg_args(x, b, nfields, coef, msh, Xh, gs, params));
    const sem_pcg_params &P = *params;
    if (P.mixed != 0 || P.variant != 0)
        return fail(SEM_ERR_INVALID, "the allocation-free solve is the FP64 two-reduction PCG (mixed = 0, variant = 0)");
    const int64_t nn = coef->n * (int64_t)nfields;
    if (nn > kMaxPoints)
        return fail(SEM_ERR_INVALID, "n_p * nfields = %lld exceeds the allocation-free workspace (%lld points)",
                    (long long)nn, (long long)kMaxPoints);
    if (nn == 0) return SEM_OK;
    if (gs->device < 0)
        return fail(SEM_ERR_INVALID, "gs handle not yet resident on a device: an allocating call that uses it "
                                     "(sem_gs_op, sem_jacobi_inverse, sem_pcg_solve) uploads it");
    SEM_TRY(check_device(gs->device));
    const int64_t nb = cg_partial_stride(coef);
    if ((4 * (int64_t)nfields + 3) * nb > kPartial)
        return fail(SEM_ERR_INVALID, "%lld reduction partials exceed the allocation-free workspace (%lld)",
                    (long long)((4 * (int64_t)nfields + 3) * nb), (long long)kPartial);
    int dev;
    SEM_TRY(current_device(&dev));
    double *base;
    SEM_TRY(scratch_of(dev, &base));
    hipStream_t st = S(stream);

    // the solver's scratch, all inside the workspace; host mirrors on this stack frame
    // (every copy into them is followed by a stream synchronisation before use)
    CgScalars h_scal[3];
    double h_dots[12];
    int h_done[3];
    double *small = base + kOffSmall;
    Work W;
    W.cap_n = coef->n;
    W.cap_f = nfields;
    W.r = base + kOffR;
    W.p = base + kOffP;
    W.w = base + kOffW;
    W.partial = base + kOffPartial;
    W.partial_len = (4 * (int64_t)nfields + 3) * nb;
    W.nb = nb;
    W.scal = (CgScalars *)(small + kSmallScal);
    W.job64 = (AlphaJob *)(small + kSmallJob);
    W.dots = small + kSmallDots;
    W.done = (int *)(small + kSmallDone);
    W.h_scal = h_scal;
    W.h_dots = h_dots;
    W.h_done = h_done;
    double *dinv = base + kOffDinv;

    // the gather-scatter folds the matvec partials into alpha through this job
    // (the copy's source lives until the solve's first synchronisation below)
    const AlphaJob job{W.partial, fns(coef->lx).nblk64(coef->nelv), W.scal};
    HIP_TRY(hipMemcpyAsync(W.job64, &job, sizeof(AlphaJob), hipMemcpyHostToDevice, st));
    // Jacobi inverse into the workspace (every element of it is written)
    SEM_TRY(compute_dinv(coef, gs, dinv, st));
    sem_pcg_params Q = P;
    if (Q.rtol > 0.0) Q.rtol *= SEM_RTOL_MARGIN;
    return pcg_fp64(x, b, nfields, coef, gs, &Q, info, W, dinv, st);
}
