// sem_proj.cpp -- the projection space of previous solutions (initial guesses of the
// pressure solve, Section 4 and Table 2 of arXiv 2107.01243) and the multi-vector
// inner products and combinations it shares with GMRES.
#include "sem_internal.h"

using namespace semi;

namespace __attribute__((visibility("hidden"))) semi {

// host_out[i] = (V_i, v) over unique nodes, i < l (V_i = V + i ld)
sem_status vdots(const VecCtx &X, const double *V, int64_t ld, int l, const double *v, double *host_out,
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
sem_status vcomb(const VecCtx &X, double *y, const double *src, const double *V, int64_t ld, int l,
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

}  // namespace semi

extern "C" {

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
    // the correction solve A dx = r only needs |r - A dx| <= rtol |b| (sem_pcg_solve
    // applies the margin SEM_RTOL_MARGIN to that target itself)
    sem_pcg_params P2 = *params;
    P2.use_x0 = 0;
    sem_pcg_info i2{};
    sem_status st_solve = SEM_OK;
    if (rn > 0.0 && rn > SEM_RTOL_MARGIN * params->rtol * bn) {
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
        if (rn <= SEM_RTOL_MARGIN * params->rtol * bn) info->rel_res = bn > 0.0 ? rn / bn : 0.0;
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

}  // extern "C"
