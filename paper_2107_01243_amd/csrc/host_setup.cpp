// host_setup.cpp -- host-side setup of libsem: GLL space, synthetic box mesh,
// gather-scatter maps.  Pure C++ (no device calls), so it also runs on machines
// without a GPU.
//
// GLL space (Jansson et al., arXiv 2107.01243, Section 2, Eq. 7-9): points are
// -1, +1 and the zeros of L'_N, found with Newton's method on
// f(x) = x L_N(x) - L_{N-1}(x) (whose zeros in (-1,1) are those of L'_N because
// (1-x^2) L'_N = N (L_{N-1} - x L_N)), with f'(x) = (N+1) L_N(x); all in long
// double.  The derivative matrix uses barycentric weights,
// D_ij = (lambda_j / lambda_i) / (x_i - x_j), D_ii = -sum_{j != i} D_ij.
//
// Gather-scatter maps (Section 3.2): local indices are bucketed by global id
// (counting sort when the id range is compact, comparison sort otherwise), which
// keeps them in ascending local order inside each id.
#include "sem_host.h"

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

namespace semh {

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn, int64_t grain)
{
    unsigned nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 1;
    if (nt > 32) nt = 32;
    if (grain < 1) grain = 1;
    nt = (unsigned)std::min<int64_t>(nt, std::max<int64_t>(1, n / grain));
    if (nt == 1) {
        fn(0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t lo = t * chunk, hi = std::min<int64_t>(n, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([=, &fn] { fn(lo, hi); });
    }
    for (auto &x : th) x.join();
}

static void legendre_pair(int N, long double x, long double &LN, long double &LNm1)
{
    long double p0 = 1.0L, p1 = x;
    if (N == 0) { LN = 1.0L; LNm1 = 0.0L; return; }
    for (int k = 1; k < N; ++k) {
        const long double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
    }
    LN = p1;
    LNm1 = p0;
}

void gll_space(int lx, double *xi, double *w, double *D)
{
    const int N = lx - 1;
    std::vector<long double> x(lx), lam(lx);
    x[0] = -1.0L;
    x[N] = 1.0L;
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 1; i < N; ++i) {
        long double t = -cosl(pi * i / N);
        for (int it = 0; it < 60; ++it) {
            long double L, Lm;
            legendre_pair(N, t, L, Lm);
            const long double dt = (t * L - Lm) / ((N + 1) * L);
            t -= dt;
            if (fabsl(dt) < 1e-19L) break;
        }
        x[i] = t;
    }
    for (int i = 0; i < lx / 2; ++i) {  // exact symmetry about zero
        const long double a = 0.5L * (x[N - i] - x[i]);
        x[i] = -a;
        x[N - i] = a;
    }
    if (lx % 2) x[N / 2] = 0.0L;
    for (int i = 0; i < lx; ++i) {
        long double L, Lm;
        legendre_pair(N, x[i], L, Lm);
        xi[i] = (double)x[i];
        w[i] = (double)(2.0L / (N * (N + 1.0L) * L * L));
    }
    for (int j = 0; j < lx; ++j) {
        long double p = 1.0L;
        for (int k = 0; k < lx; ++k)
            if (k != j) p *= (x[j] - x[k]);
        lam[j] = 1.0L / p;
    }
    for (int i = 0; i < lx; ++i) {
        long double diag = 0.0L;
        for (int j = 0; j < lx; ++j) {
            if (j == i) continue;
            const long double v = (lam[j] / lam[i]) / (x[i] - x[j]);
            D[i * lx + j] = (double)v;
            diag -= v;
        }
        D[i * lx + i] = (double)diag;
    }
}

void box_mesh(int nx, int ny, int nz, int lx, double eps, const double *xi, int64_t *glb,
              uint8_t *dir, double *xyz)
{
    const int N = lx - 1;
    const int64_t Mx = (int64_t)nx * N + 1, My = (int64_t)ny * N + 1, Mz = (int64_t)nz * N + 1;
    const int64_t nelv = (int64_t)nx * ny * nz;
    const int64_t npe = (int64_t)lx * lx * lx;
    const int64_t n = nelv * npe;
    const double two_pi = 2.0 * M_PI;
    parallel_for(nelv, [&](int64_t e0, int64_t e1) {
        std::vector<double> sx(lx), sy(lx), sz(lx);
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / ((int64_t)nx * ny);
            for (int k = 0; k < lx; ++k)
                for (int j = 0; j < lx; ++j)
                    for (int i = 0; i < lx; ++i) {
                        const int64_t p = e * npe + i + (int64_t)lx * (j + (int64_t)lx * k);
                        const int64_t gx = ex * N + i, gy = ey * N + j, gz = ez * N + k;
                        if (glb) glb[p] = gx + Mx * (gy + My * gz);
                        if (dir)
                            dir[p] = (gx == 0 || gx == Mx - 1 || gy == 0 || gy == My - 1 || gz == 0 ||
                                      gz == Mz - 1);
                        if (xyz) {
                            const double X = (ex + 0.5 * (xi[i] + 1.0)) / nx;
                            const double Y = (ey + 0.5 * (xi[j] + 1.0)) / ny;
                            const double Z = (ez + 0.5 * (xi[k] + 1.0)) / nz;
                            const double sX = std::sin(two_pi * X), sY = std::sin(two_pi * Y),
                                         sZ = std::sin(two_pi * Z);
                            xyz[p] = X + eps * sY * sZ;
                            xyz[n + p] = Y + eps * sZ * sX;
                            xyz[2 * n + p] = Z + eps * sX * sY;
                        }
                    }
        }
    }, 256);
}

// Bucket local indices by global id; returns false (with msg) on invalid input.
bool build_gs_maps(int64_t n, const int64_t *glb, const uint8_t *dir, GsMaps &m, std::string &msg)
{
    m = GsMaps();
    m.n = n;
    if (n >= ((int64_t)1 << 31)) { msg = "gather-scatter needs n_local < 2^31"; return false; }
    int64_t gmax = -1;
    for (int64_t p = 0; p < n; ++p) {
        if (glb[p] < 0) { msg = "negative global id"; return false; }
        gmax = std::max(gmax, glb[p]);
    }
    std::vector<int32_t> order(n);
    std::vector<int64_t> start;  // group boundaries inside `order`
    std::vector<int64_t> gid;
    if (n > 0 && gmax <= 4 * n + 1024) {
        std::vector<int64_t> cnt(gmax + 2, 0);
        for (int64_t p = 0; p < n; ++p) cnt[glb[p] + 1] += 1;
        for (int64_t g = 0; g <= gmax; ++g) cnt[g + 1] += cnt[g];
        std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
        for (int64_t p = 0; p < n; ++p) order[pos[glb[p]]++] = (int32_t)p;
        for (int64_t g = 0; g <= gmax; ++g)
            if (cnt[g + 1] > cnt[g]) { start.push_back(cnt[g]); gid.push_back(g); }
        start.push_back(n);
    } else if (n > 0) {
        std::vector<std::pair<int64_t, int32_t>> s(n);
        for (int64_t p = 0; p < n; ++p) s[p] = {glb[p], (int32_t)p};
        std::sort(s.begin(), s.end());
        for (int64_t p = 0; p < n; ++p) {
            order[p] = s[p].second;
            if (p == 0 || s[p].first != s[p - 1].first) { start.push_back(p); gid.push_back(s[p].first); }
        }
        start.push_back(n);
    }
    m.mult.assign(n, 0);
    m.owner.assign(n, 0);
    const int64_t ng = (int64_t)gid.size();
    m.n_unique = ng;
    m.blk_ptr.push_back(0);
    m.big_ptr.push_back(0);
    for (int64_t g = 0; g < ng; ++g) {
        const int64_t lo = start[g], hi = start[g + 1], c = hi - lo;
        if (c > 255) { msg = "more than 255 copies of one global id"; return false; }
        if (dir) {
            for (int64_t q = lo + 1; q < hi; ++q)
                if ((dir[order[q]] != 0) != (dir[order[lo]] != 0)) {
                    msg = "Dirichlet flag differs between copies of one global id";
                    return false;
                }
        }
        m.owner[order[lo]] = 1;
        for (int64_t q = lo; q < hi; ++q) m.mult[order[q]] = (uint8_t)c;
        if (c >= 2 && c <= 64) {
            const int64_t used = (int64_t)m.ent_idx.size() % 64;
            if (used + c > 64)
                for (int64_t q = used; q < 64; ++q) { m.ent_idx.push_back(-1); m.ent_meta.push_back(0); }
            for (int64_t q = lo; q < hi; ++q) {
                m.ent_idx.push_back(order[q]);
                m.ent_meta.push_back((uint16_t)((q - lo) | (c << 8)));
            }
            m.max_group = std::max<int>(m.max_group, (int)c);
        } else if (c > 64) {
            for (int64_t q = lo; q < hi; ++q) m.big_idx.push_back(order[q]);
            m.big_ptr.push_back((int64_t)m.big_idx.size());
        }
        if (c == 2) {
            m.pairs.push_back(order[lo]);
            m.pairs.push_back(order[lo + 1]);
        } else if (c > 2) {
            for (int64_t q = lo; q < hi; ++q) m.blk_idx.push_back(order[q]);
            m.blk_ptr.push_back((int64_t)m.blk_idx.size());
        }
    }
    return true;
}

void element_order(const GsMaps &m, std::vector<int32_t> &pairs, std::vector<int64_t> &blk_ptr,
                   std::vector<int32_t> &blk_idx)
{
    const int64_t np = (int64_t)m.pairs.size() / 2;
    std::vector<int64_t> ord(np);
    for (int64_t q = 0; q < np; ++q) ord[q] = q;
    std::sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return m.pairs[2 * x] < m.pairs[2 * y]; });
    pairs.resize(2 * np);
    for (int64_t q = 0; q < np; ++q) {
        pairs[2 * q] = m.pairs[2 * ord[q]];
        pairs[2 * q + 1] = m.pairs[2 * ord[q] + 1];
    }
    const int64_t nb = (int64_t)m.blk_ptr.size() - 1;
    std::vector<int64_t> bo(nb);
    for (int64_t q = 0; q < nb; ++q) bo[q] = q;
    std::sort(bo.begin(), bo.end(), [&](int64_t x, int64_t y) { return m.blk_idx[m.blk_ptr[x]] < m.blk_idx[m.blk_ptr[y]]; });
    blk_ptr.assign(1, 0);
    blk_idx.clear();
    blk_idx.reserve(m.blk_idx.size());
    for (int64_t q = 0; q < nb; ++q) {
        for (int64_t c = m.blk_ptr[bo[q]]; c < m.blk_ptr[bo[q] + 1]; ++c) blk_idx.push_back(m.blk_idx[c]);
        blk_ptr.push_back((int64_t)blk_idx.size());
    }
}

void sym_eig(int n, double *a, double *V, double *lam)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
    double norm2 = 0.0;
    for (int i = 0; i < n * n; ++i) norm2 += a[i] * a[i];
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
        if (off <= 1e-32 * norm2) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[p * n + q];
                if (apq == 0.0) continue;
                const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = c * akp - s * akq;
                    a[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = c * apk - s * aqk;
                    a[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) lam[i] = a[i * n + i];
}

namespace {

// local index of the point with coordinate d equal to c and the two other
// coordinates (ascending direction order) equal to fa, fb
inline int64_t face_point(int lx, int d, int c, int fa, int fb)
{
    const int64_t l1 = lx, l2 = (int64_t)lx * lx;
    if (d == 0) return c + l1 * fa + l2 * fb;
    if (d == 1) return fa + l1 * c + l2 * fb;
    return fa + l1 * fb + l2 * c;
}

}  // namespace

bool face_neighbours(int64_t nelv, int lx, const int64_t *glb, std::vector<int32_t> &out, std::string &msg)
{
    const int N = lx - 1;
    const int64_t lx3 = (int64_t)lx * lx * lx;
    out.assign((size_t)nelv * 24, 0);
    for (int64_t q = 0; q < nelv * 6; ++q) out[(size_t)q * 4] = -1;
    if (nelv > 0x7fffffff / 6) {
        msg = "face_neighbours: too many elements";
        return false;
    }
    // faces keyed by their sorted corner ids
    struct Rec {
        int64_t key[4];
        int32_t ef;  // e * 6 + f
    };
    std::vector<Rec> rec((size_t)nelv * 6);
    parallel_for(nelv, [&](int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e)
            for (int f = 0; f < 6; ++f) {
                Rec &r = rec[(size_t)e * 6 + f];
                const int d = f / 2, c = (f & 1) ? N : 0;
                int q = 0;
                for (int fb = 0; fb <= N; fb += N)
                    for (int fa = 0; fa <= N; fa += N) r.key[q++] = glb[e * lx3 + face_point(lx, d, c, fa, fb)];
                std::sort(r.key, r.key + 4);
                r.ef = (int32_t)(e * 6 + f);
            }
    }, 4096);
    std::sort(rec.begin(), rec.end(), [](const Rec &x, const Rec &y) {
        return std::lexicographical_compare(x.key, x.key + 4, y.key, y.key + 4) ||
               (std::equal(x.key, x.key + 4, y.key) && x.ef < y.ef);
    });
    // for face A = (e, f) and its partner B = (e2, f2): B's inward point under A's
    // face point (fa, fb) is base + fa sa + fb sb, checked on every face point
    auto link = [&](int32_t A, int32_t B) -> bool {
        const int64_t e = A / 6, e2 = B / 6;
        const int f = A % 6, f2 = B % 6, d = f / 2, d2 = f2 / 2;
        const int c = (f & 1) ? N : 0, c2 = (f2 & 1) ? N : 0;
        // B's face coordinates of each of A's corners
        int img[3][2];
        const int ca[3][2] = {{0, 0}, {N, 0}, {0, N}};
        for (int m = 0; m < 3; ++m) {
            const int64_t g = glb[e * lx3 + face_point(lx, d, c, ca[m][0], ca[m][1])];
            bool hit = false;
            for (int gb = 0; gb <= N && !hit; gb += N)
                for (int ga = 0; ga <= N && !hit; ga += N)
                    if (glb[e2 * lx3 + face_point(lx, d2, c2, ga, gb)] == g) {
                        img[m][0] = ga;
                        img[m][1] = gb;
                        hit = true;
                    }
            if (!hit) return false;
        }
        const int64_t p0 = face_point(lx, d2, c2, img[0][0], img[0][1]);
        const int64_t pa = face_point(lx, d2, c2, img[1][0], img[1][1]);
        const int64_t pb = face_point(lx, d2, c2, img[2][0], img[2][1]);
        const int64_t sa = (pa - p0) / N, sb = (pb - p0) / N;
        if (sa * N != pa - p0 || sb * N != pb - p0) return false;
        for (int fb = 0; fb <= N; ++fb)
            for (int fa = 0; fa <= N; ++fa)
                if (glb[e * lx3 + face_point(lx, d, c, fa, fb)] != glb[e2 * lx3 + p0 + fa * sa + fb * sb])
                    return false;
        int64_t stride = 1;
        for (int k = 0; k < d2; ++k) stride *= lx;
        int32_t *o = &out[(size_t)A * 4];
        o[0] = (int32_t)e2;
        o[1] = (int32_t)(p0 + ((f2 & 1) ? -stride : stride));
        o[2] = (int32_t)sa;
        o[3] = (int32_t)sb;
        return true;
    };
    for (size_t q = 0; q < rec.size();) {
        size_t q2 = q + 1;
        while (q2 < rec.size() && std::equal(rec[q].key, rec[q].key + 4, rec[q2].key)) ++q2;
        if (q2 - q > 2) {
            msg = "face_neighbours: a face is shared by more than two elements";
            return false;
        }
        // an element holding both copies of a face (periodic, one element across) is not
        // its own neighbour
        if (q2 - q == 2 && rec[q].ef / 6 != rec[q + 1].ef / 6 &&
            (!link(rec[q].ef, rec[q + 1].ef) || !link(rec[q + 1].ef, rec[q].ef))) {
            msg = "face_neighbours: two elements share a face's corners but not its points as a grid";
            return false;
        }
        q = q2;
    }
    return true;
}

}  // namespace semh
