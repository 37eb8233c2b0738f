// sem_gmres.cpp -- the pressure solver of Section 4 of arXiv 2107.01243: flexible
// GMRES with point-Jacobi or two-level additive Schwarz preconditioning (local
// fast-diagonalisation solves, Galerkin coarse space on linear elements).
#include "sem_internal.h"

using namespace semi;

extern "C" {

// ------------------------------------------------------------------ two-level Schwarz
// Per element and direction d, sum over the element of G_dd / B (formed on the
// device): the element length is L_d = 2 / sqrt(that sum / lx^3).
static sem_status elem_gb(sem_coef c, hipStream_t st, std::vector<double> &gb)
{
    const int lx3 = c->lx * c->lx * c->lx;
    gb.assign((size_t)3 * c->nelv, 0.0);
    double *d_gb = nullptr;
    SEM_TRY(dalloc(&d_gb, gb.size()));
    const hipError_t e1 = sem_launch_elem_gb(c->G, c->B, d_gb, c->nelv, lx3, st);
    const hipError_t e2 =
        e1 == hipSuccess ? hipMemcpyAsync(gb.data(), d_gb, sizeof(double) * gb.size(), hipMemcpyDeviceToHost, st) : e1;
    const hipError_t e3 = e2 == hipSuccess ? hipStreamSynchronize(st) : e2;
    dfree(d_gb);
    HIP_TRY(e3);
    return SEM_OK;
}

// 1-D GLL stiffness on [-1, 1]: Kref[m][q] = sum_i w_i D_im D_iq
static std::vector<double> ref_stiffness(sem_space Xh)
{
    const int lx = Xh->lx;
    std::vector<double> Kref((size_t)lx * lx, 0.0);
    for (int m = 0; m < lx; ++m)
        for (int q = 0; q < lx; ++q)
            for (int i = 0; i < lx; ++i) Kref[m * lx + q] += Xh->w[i] * Xh->D[i * lx + m] * Xh->D[i * lx + q];
    return Kref;
}

// Setup (host + a few launches): element lengths from the geometric factors, the
// 1-D extended operators and their eigen-decompositions, the coarse vertices and
// the Galerkin coarse matrix from eight probe applications of A_L.
static sem_status schwarz_setup_base(sem_coef c, sem_gs g, hipStream_t st)
{
    SchwarzData &Z = c->sz;
    if (Z.valid && Z.gs == (const void *)g) return SEM_OK;
    if (c->h1 || c->h2) return fail(SEM_ERR_UNSUPPORTED, "the Schwarz preconditioner needs scalar h1 and h2");
    Z.release();
    const int lx = c->lx, N = lx - 1, lx3 = lx * lx * lx;
    const int64_t E = c->nelv, n = c->n;
    const sem_space Xh = c->Xh;
    std::vector<double> gb;
    SEM_TRY(elem_gb(c, st, gb));
    const std::vector<double> Kref = ref_stiffness(Xh);
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
    SEM_TRY(dalloc(&Z.cpart, (size_t)(2 + sem_coarse_split()) * ((nv + 255) / 256)));
    HIP_TRY(hipMemcpy(Z.ell_ci, eci.data(), eci.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.ell_val, evl.data(), evl.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.dinv0, dg.data(), dg.size() * 8, hipMemcpyHostToDevice));
    Z.width = width;
    Z.nv = nv;
    Z.gs = g;
    Z.valid = true;
    return SEM_OK;
}

// The one-point overlap: the face-neighbour table, and per element and direction the
// 1-D operator on lx + 2 nodes (extension node, the element's GLL nodes, extension
// node).  Beyond a face with a neighbour the extension node is joined to the face node
// by a linear segment of the first GLL spacing and held by a Dirichlet condition one
// second GLL spacing further out; beyond a face without one, the face node keeps the
// first-spacing segment (Dirichlet at its end) and the extension node is decoupled
// (K = 1/h, M = h/2: its zero right-hand side gives zero there, so the own points see
// the element-only problem in that direction).
static sem_status schwarz_setup_overlap(sem_coef c, hipStream_t st)
{
    SchwarzData &Z = c->sz;
    if (Z.ov_valid) return SEM_OK;
    const int lx = c->lx, N = lx - 1, X = lx + 2, lx3 = lx * lx * lx;
    const int64_t E = c->nelv;
    const sem_space Xh = c->Xh;
    std::vector<int32_t> face;
    std::string msg;
    if (!semh::face_neighbours(E, lx, c->msh->glb.data(), face, msg)) return fail(SEM_ERR_INVALID, "%s", msg.c_str());
    std::vector<double> gb;
    SEM_TRY(elem_gb(c, st, gb));
    const std::vector<double> Kref = ref_stiffness(Xh);
    const int i2 = N >= 2 ? 2 : N;
    const double dref = Xh->xi[1] - Xh->xi[0], dref2 = Xh->xi[i2] - Xh->xi[i2 - 1];
    std::vector<double> S((size_t)E * 3 * X * X), lam((size_t)E * 3 * X);
    semh::parallel_for(E, [&](int64_t e0, int64_t e1) {
        std::vector<double> K((size_t)X * X), a((size_t)X * X), V((size_t)X * X), l(X), M(X);
        for (int64_t e = e0; e < e1; ++e) {
            for (int d = 0; d < 3; ++d) {
                const double L = 2.0 / std::sqrt(gb[(size_t)e * 3 + d] / lx3), J = L / 2.0;
                const double h = J * dref, h2 = J * dref2;
                std::fill(K.begin(), K.end(), 0.0);
                std::fill(M.begin(), M.end(), 0.0);
                for (int i = 0; i < lx; ++i) {
                    M[i + 1] = Xh->w[i] * J;
                    for (int q = 0; q < lx; ++q) K[(i + 1) * X + q + 1] = Kref[i * lx + q] / J;
                }
                for (int side = 0; side < 2; ++side) {
                    const bool has = face[((size_t)e * 6 + 2 * d + side) * 4] >= 0;
                    const int f = side ? lx : 1, xn = side ? X - 1 : 0;
                    K[f * X + f] += 1.0 / h;
                    M[f] += h / 2.0;
                    if (has) {
                        K[xn * X + xn] += 1.0 / h + 1.0 / h2;
                        K[xn * X + f] -= 1.0 / h;
                        K[f * X + xn] -= 1.0 / h;
                        M[xn] += h / 2.0 + h2 / 2.0;
                    } else {
                        K[xn * X + xn] = 1.0 / h;
                        M[xn] = h / 2.0;
                    }
                }
                for (int i = 0; i < X; ++i)
                    for (int q = 0; q < X; ++q) a[i * X + q] = K[i * X + q] / std::sqrt(M[i] * M[q]);
                semh::sym_eig(X, a.data(), V.data(), l.data());
                double *Sd = &S[((size_t)e * 3 + d) * X * X];
                for (int i = 0; i < X; ++i)
                    for (int m = 0; m < X; ++m) Sd[i * X + m] = V[i * X + m] / std::sqrt(M[i]);
                for (int m = 0; m < X; ++m) lam[((size_t)e * 3 + d) * X + m] = l[m];
            }
        }
    }, 64);
    dfree(Z.S_ov);  // left by an earlier setup that failed part way
    dfree(Z.lam_ov);
    dfree(Z.face);
    SEM_TRY(dalloc(&Z.S_ov, S.size()));
    SEM_TRY(dalloc(&Z.lam_ov, lam.size()));
    SEM_TRY(dalloc(&Z.face, face.size()));
    HIP_TRY(hipMemcpy(Z.S_ov, S.data(), S.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.lam_ov, lam.data(), lam.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Z.face, face.data(), face.size() * 4, hipMemcpyHostToDevice));
    Z.ov_valid = true;
    return SEM_OK;
}

static sem_status schwarz_setup(sem_coef c, sem_gs g, bool overlap, hipStream_t st)
{
    SEM_TRY(schwarz_setup_base(c, g, st));
    if (overlap) SEM_TRY(schwarz_setup_overlap(c, st));
    return SEM_OK;
}

// z = M^{-1} r: local solves (on the element's box, or with overlap on the box
// extended by one point, keeping the own points) summed over shared points and
// averaged, plus P e0 from coarse_iters Jacobi-CG steps on A0 e0 = P^T r; masked.
// r assembled and masked.
static sem_status schwarz_apply(sem_coef c, sem_gs g, double *z, const double *r, int coarse_iters, bool overlap,
                                hipStream_t st)
{
    SchwarzData &Z = c->sz;
    const int lx = c->lx;
    const FdmArgs F{z,      r,      overlap ? Z.S_ov : Z.S, overlap ? Z.lam_ov : Z.lam, g->d_owner,
                    Z.lin,  Z.part, overlap ? Z.face : nullptr, c->h1s, c->h2s, c->nelv};
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
                             int coarse_iters, int ov, void *stream)
{
    SEM_TRY(check_coef(coef, msh, Xh));
    if (!gs || gs->msh != msh) return fail(SEM_ERR_INVALID, "gs is NULL or built for another mesh");
    if (coarse_iters < 0 || coarse_iters > 10000) return fail(SEM_ERR_INVALID, "coarse_iters must be in 0..10000");
    if (ov != 0 && ov != 1) return fail(SEM_ERR_INVALID, "overlap must be 0 or 1");
    const size_t bytes = (size_t)coef->n * 8;
    if (bytes == 0) return SEM_OK;
    if (!z || !r) return fail(SEM_ERR_INVALID, "z or r is NULL");
    if (overlap(z, bytes, r, bytes)) return fail(SEM_ERR_INVALID, "z and r overlap");
    hipStream_t st = S(stream);
    SEM_TRY(gs_upload(gs));
    SEM_TRY(mesh_upload(msh));
    SEM_TRY(schwarz_setup(coef, gs, ov != 0, st));
    return schwarz_apply(coef, gs, z, r, coarse_iters, ov != 0, st);
}

// ------------------------------------------------------------------ flexible GMRES
static sem_status gmres_apply(sem_coef c, sem_gs g, double *w, const double *z, hipStream_t st)
{
    SEM_TRY(launch_ax<double>(c, w, z, 1, st));
    SEM_TRY(launch_gs<double>(w, 1, g, nullptr, nullptr, st));
    HIP_TRY(sem_launch_mask(w, 0, c->msh->d_dir_idx, (int64_t)c->msh->dir_idx.size(), c->n, 1, st));
    return SEM_OK;
}

// z = M^{-1} v (0: point Jacobi; 1: two-level Schwarz; 2: the same with one-point overlap)
static sem_status gmres_precond(sem_coef c, sem_gs g, const sem_gmres_params *P, double *z, const double *v,
                                hipStream_t st)
{
    if (P->precond == 1 || P->precond == 2)
        return schwarz_apply(c, g, z, v, P->coarse_iters > 0 ? P->coarse_iters : 10, P->precond == 2, st);
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
    if (P.precond < 0 || P.precond > 2) return fail(SEM_ERR_INVALID, "precond must be 0, 1 or 2");
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
    if (P.precond != 0) SEM_TRY(schwarz_setup(coef, gs, P.precond == 2, st));
    sem_gmres_params Q = P;  // cycles and convergence work on SEM_RTOL_MARGIN * rtol
    Q.rtol *= SEM_RTOL_MARGIN;
    return gmres_run(x, b, coef, gs, &Q, info, st);
}

}  // extern "C"
