// sem_cg.cpp -- the Jacobi-preconditioned CG solvers behind sem_pcg_solve (the velocity
// solve of Section 4 of arXiv 2107.01243): FP64 two-reduction and single-reduction
// forms, FP32 iteration with FP64 reliable updates, and FP64 flexible CG around an
// FP32 inner solve ("other precision formats", Section 10).
#include "sem_internal.h"

using namespace semi;

namespace __attribute__((visibility("hidden"))) semi {

template <typename T>
sem_status cg_iterate(sem_coef c, Work &W, sem_gs g, int nf, T *x, T *r, T *p, T *w, const T *dinv, int max_iter,
                      int check_every, double *hist, int hist_len, hipStream_t st);

// Jacobi-PCG in precision T on nf fields.  x is the iterate (zeroed unless use_x0),
// b the assembled, masked right-hand side.  Per-field results land in W.h_scal.
template <typename T>
sem_status cg_run(sem_coef c, Work &W, sem_gs g, int nf, T *x, const T *b, bool use_x0, T *r, T *p, T *w,
                  const T *dinv, const double *rtol, int max_iter, int check_every, double *hist, int hist_len,
                  hipStream_t st)
{
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
    return cg_iterate<T>(c, W, g, nf, x, r, p, w, dinv, max_iter, check_every, hist, hist_len, st);
}

// Iterate the CG state held in W.scal until every field has stopped.
template <typename T>
sem_status cg_iterate(sem_coef c, Work &W, sem_gs g, int nf, T *x, T *r, T *p, T *w, const T *dinv, int max_iter,
                      int check_every, double *hist, int hist_len, hipStream_t st)
{
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
    M.deo = sizeof(T) == 8 ? c->deo64 : c->deo32;
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
sem_status true_residual(sem_coef c, Work &W, const double *dinv, sem_gs g, int nf, const double *x,
                         const double *b, double *rel, hipStream_t st)
{
    SEM_TRY(launch_ax<double>(c, W.w, x, nf, st));
    SEM_TRY(launch_gs<double>(W.w, nf, g, nullptr, nullptr, st));
    HIP_TRY(sem_launch_residual(W.r, b, W.w, dinv, c->n, nf, st));
    const double *a[2] = {W.r, b};
    double out[6];
    SEM_TRY(dots(c, W, g, nf, 2, a, a, out, st));
    for (int f = 0; f < nf; ++f) {
        const double rr = out[0 * nf + f], bb = out[1 * nf + f];
        rel[f] = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    }
    return SEM_OK;
}

sem_status true_residual(sem_coef c, sem_gs g, int nf, const double *x, const double *b, double *rel,
                         hipStream_t st)
{
    return true_residual(c, c->ws, c->dinv, g, nf, x, b, rel, st);
}

// FP64 two-reduction Jacobi-PCG on the scratch W and the Jacobi inverse dinv.
sem_status pcg_fp64(double *x, const double *b, int nf, sem_coef c, sem_gs g, const sem_pcg_params *P,
                    sem_pcg_info *info, Work &W, const double *dinv, hipStream_t st)
{
    const double rtol[3] = {P->rtol, P->rtol, P->rtol};
    SEM_TRY(cg_run<double>(c, W, g, nf, x, b, P->use_x0 != 0, W.r, W.p, W.w, dinv, rtol, P->max_iter,
                           P->check_every, nullptr, 0, st));
    // A field counts as converged only when its true residual |b - A x| / |b| meets
    // rtol.  When the recursive residual has drifted below it, the true residual
    // (left in W.r by true_residual) replaces it and the iteration continues with
    // its search direction.
    double tr[3];
    for (int round = 0;; ++round) {
        SEM_TRY(true_residual(c, W, dinv, g, nf, x, b, tr, st));
        bool any = false;
        for (int f = 0; f < nf; ++f) {
            const CgScalars &s = W.h_scal[f];
            W.h_done[f] = (s.status == 0 && P->rtol > 0 && s.bb > 0 && tr[f] > P->rtol && s.iter < P->max_iter) ? 1 : 0;
            any = any || W.h_done[f];
        }
        if (!any || round >= 16) break;
        const unsigned vg = sem_vec_grid(c->n);
        HIP_TRY(hipMemcpyAsync(W.done, W.h_done, sizeof(int) * nf, hipMemcpyHostToDevice, st));
        HIP_TRY(sem_launch_cg_replace_f64(W.r, dinv, g->d_owner, W.done, W.partial, c->n, nf, st));
        CgFinishArgs F{W.partial, (int64_t)vg, W.scal, nullptr, 0, nf};
        HIP_TRY(sem_launch_cg_resume(&F, W.done, st));
        SEM_TRY(cg_iterate<double>(c, W, g, nf, x, W.r, W.p, W.w, dinv, P->max_iter, P->check_every, nullptr, 0, st));
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

// Arguments of sem_pcg_solve (and of its allocation-free variant).
sem_status check_pcg_args(const double *x, const double *b, int nfields, sem_coef coef, sem_mesh msh, sem_space Xh,
                          sem_gs gs, const sem_pcg_params *params)
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
    return SEM_OK;
}

}  // namespace semi

extern "C" {

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
    M.deo = c->deo64;
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
    M.deo = c->deo32;
    CgUpdateArgs<float> U{W.y32, W.r32, W.p32, W.w32, c->dinv32, g->d_owner, W.scal, W.partial, n, nf};
    const unsigned ug = sem_update_grid(n, 1);
    CgFinishArgs F{W.partial, (int64_t)ug, W.scal, nullptr, 0, nf};
    const int check_every = std::max(1, P->check_every);
    const int64_t max_polls = (int64_t)P->max_iter + 64 * 64;  // every poll runs >= 1 iteration or ends a segment
    // Launches queued between polls after a segment has ended do no work but still
    // cost a pass over the vectors, so the next poll is placed where the current
    // segment is expected to end: at the length of the previous segment (check_every
    // before any has ended, check_every / 4 once the estimate is passed).
    int seg_len[3] = {0, 0, 0}, seg_start[3] = {0, 0, 0};
    for (int64_t poll = 0; poll < max_polls; ++poll) {
        HIP_TRY(hipMemcpyAsync(W.h_scal, W.scal, sizeof(CgScalars) * nf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(W.h_rel, W.rel, sizeof(RelState) * nf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        bool all_stopped = true, all_done = true;
        for (int f = 0; f < nf; ++f) {
            all_stopped = all_stopped && W.h_scal[f].stop;
            all_done = all_done && W.h_rel[f].done;
            if (W.h_rel[f].last_iter != seg_start[f]) {
                seg_len[f] = W.h_rel[f].last_iter - seg_start[f];
                seg_start[f] = W.h_rel[f].last_iter;
            }
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
        int todo = check_every;
        for (int f = 0; f < nf; ++f) {
            if (W.h_rel[f].done || W.h_scal[f].stop || seg_len[f] <= 0) continue;
            const int rem = seg_len[f] - (W.h_scal[f].iter - seg_start[f]);
            todo = std::min(todo, rem > 0 ? rem : std::max(1, check_every / 4));
        }
        for (int it = 0; it < todo; ++it) {
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
        SEM_TRY(cg_run<float>(c, W, g, nf, W.y32, W.r32, false, W.ri32, W.p32, W.w32, c->dinv32, tau,
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
    SEM_TRY(check_pcg_args(x, b, nfields, coef, msh, Xh, gs, params));
    const sem_pcg_params &P = *params;
    if ((size_t)coef->n * nfields == 0) return SEM_OK;
    hipStream_t st = S(stream);
    SEM_TRY(gs_upload(gs));
    SEM_TRY(ensure_dinv(coef, gs, st));
    SEM_TRY(ensure_work(coef, nfields, P.mixed != 0));
    // every stopping test below works on the target SEM_RTOL_MARGIN * rtol
    sem_pcg_params Q = P;
    if (Q.rtol > 0.0) Q.rtol *= SEM_RTOL_MARGIN;
    if (Q.mixed == 1) return pcg_mixed_reliable(x, b, nfields, coef, gs, &Q, info, st);
    if (Q.mixed == 2) return pcg_mixed(x, b, nfields, coef, gs, &Q, info, st);
    if (Q.variant == 1) return pcg_cg1(x, b, nfields, coef, gs, &Q, info, st);
    return pcg_fp64(x, b, nfields, coef, gs, &Q, info, coef->ws, coef->dinv, st);
}

}  // extern "C"
