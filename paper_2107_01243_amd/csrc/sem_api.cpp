// sem_api.cpp -- the C ABI of libsem: handles, validation, device residency, the
// operators (Jansson et al., arXiv 2107.01243: Eq. 9-10 operator, Section 3.2
// gather-scatter) and the shared device helpers of the solvers.
//
// Device residency: the mesh and gather-scatter handles are built on the host and
// uploaded on first device use, so their host logic (maps, counts, validation)
// is usable on machines without a GPU.  Everything numeric runs in the HIP
// kernels of ax_kernels.hip and vec_kernels.hip; the host code only sequences
// launches and polls a few device scalars.
#include "sem_internal.h"

using namespace semi;

namespace __attribute__((visibility("hidden"))) semi {

const LxFns &fns(int lx)
{
#define SEM_ROW(L)                                                                                 \
    {sem_launch_ax_f64_lx##L, sem_launch_ax_f32_lx##L, sem_launch_cg_f64_lx##L, sem_launch_cg_f32_lx##L, \
     sem_launch_cg1_f64_lx##L, sem_launch_fdm_lx##L, sem_launch_prolong_lx##L,                     \
     sem_launch_adj_f64_lx##L, sem_launch_adj_f32_lx##L, sem_launch_geom_lx##L, sem_launch_diag_lx##L,  \
     sem_cg_nblocks_f64_lx##L, sem_cg_nblocks_f32_lx##L, sem_deo_fill_lx##L},
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
    // one word per entry: the local index with bit 31 marking a group's first entry
    // (the kernel recovers positions and group sizes from these flags), padding all ones
    {
        std::vector<uint32_t> word(m.ent_idx.size());
        for (size_t q = 0; q < word.size(); ++q)
            word[q] = m.ent_idx[q] < 0 ? 0xffffffffu
                                       : ((uint32_t)m.ent_idx[q] | ((m.ent_meta[q] & 0xffu) == 0 ? 0x80000000u : 0u));
        SEM_TRY(dalloc(&g->d_ent_word, word.size()));
        if (!word.empty())
            HIP_TRY(hipMemcpy(g->d_ent_word, word.data(), word.size() * 4, hipMemcpyHostToDevice));
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

// dinv = 1 / QQ^T diag(A_L) (0 on Dirichlet points) into caller-provided memory.
sem_status compute_dinv(sem_coef c, sem_gs g, double *dinv, hipStream_t st)
{
    DiagArgs A;
    A.d = dinv;
    A.G = c->G;
    A.B = c->B;
    A.h1 = c->h1;
    A.h2 = c->h2;
    A.h1s = c->h1s;
    A.h2s = c->h2s;
    A.n = c->n;
    HIP_TRY(fns(c->lx).diag(&A, c->Xh->D, st));
    SEM_TRY(launch_gs<double>(dinv, 1, g, nullptr, nullptr, st));
    HIP_TRY(sem_launch_invert(dinv, c->msh->d_dir, c->n, st));
    return SEM_OK;
}

// Jacobi inverse (point Jacobi: exact assembled diagonal), cached per (coef, gs).
sem_status ensure_dinv(sem_coef c, sem_gs g, hipStream_t st)
{
    if (c->dinv_valid && c->dinv_gs == (const void *)g) return SEM_OK;
    if (!c->dinv) SEM_TRY(dalloc(&c->dinv, c->n));
    SEM_TRY(compute_dinv(c, g, c->dinv, st));
    if (c->flags & SEM_COEF_F32) {
        if (!c->dinv32) SEM_TRY(dalloc(&c->dinv32, c->n));
        HIP_TRY(sem_launch_cast_f32_f64(c->dinv32, c->dinv, 1.0, c->n, st));
    }
    c->dinv_valid = true;
    c->dinv_gs = g;
    return SEM_OK;
}

int64_t cg_partial_stride(sem_coef c)
{
    return std::max<int64_t>({fns(c->lx).nblk64(c->nelv), fns(c->lx).nblk32(c->nelv),
                              (int64_t)sem_vec_grid(c->n), (int64_t)sem_update_grid(c->n, 0),
                              (int64_t)sem_update_grid(c->n, 1)});
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
    const int64_t nb = cg_partial_stride(c);
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
sem_status dots(sem_coef c, Work &W, sem_gs g, int nf, int nd, const double *const *a, const double *const *b,
                double *host_out, hipStream_t st)
{
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

sem_status dots(sem_coef c, sem_gs g, int nf, int nd, const double *const *a, const double *const *b,
                double *host_out, hipStream_t st)
{
    return dots(c, c->ws, g, nf, nd, a, b, host_out, st);
}

}  // namespace semi

// ====================================================================== C ABI
extern "C" {

const char *sem_last_error(void) { return g_err.c_str(); }
const char *sem_version(void) { return "libsem 0.2 (gfx950)"; }
double sem_rtol_margin(void) { return SEM_RTOL_MARGIN; }

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
    dfree(gs->d_ent_word);
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
    {
        // the even-odd D of this lx in device memory (read by the kernels for lx >= 10)
        constexpr size_t b64 = sizeof(DEo<SEM_LX_MAX, double>), b32 = sizeof(DEo<SEM_LX_MAX, float>);
        unsigned char h64[b64] = {}, h32[b32] = {};
        fns(c->lx).deo(Xh->D, h64, h32);
        hipError_t e = hipSuccess;
        if ((s = dalloc((unsigned char **)&c->deo64, b64)) != SEM_OK ||
            (s = dalloc((unsigned char **)&c->deo32, b32)) != SEM_OK ||
            (e = hipMemcpy(c->deo64, h64, b64, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(c->deo32, h32, b32, hipMemcpyHostToDevice)) != hipSuccess) {
            sem_coef_destroy(c);
            return s != SEM_OK ? s : fail(SEM_ERR_HIP, "upload of D failed: %s", hipGetErrorString(e));
        }
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
    dfree(c->dinv); dfree(c->dinv32); dfree(c->deo64); dfree(c->deo32);
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
        AdjArgs<double> A{(double *)g, (const double *)u, (const double *)v, coef->G, coef->n, coef->nelv,
                          coef->deo64};
        e = fns(coef->lx).adj64(&A, Xh->D, S(stream));
    } else {
        AdjArgs<float> A{(float *)g, (const float *)u, (const float *)v, coef->G32, coef->n, coef->nelv,
                         coef->deo32};
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


}  // extern "C"
