// sanitize_host_setup.cpp -- drives the host-side setup code of libsem (GLL space,
// box mesh, gather-scatter maps, element-order maps, the symmetric eigensolver of the
// Schwarz setup) on small and irregular inputs, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_sanitizers.py compiles it with g++ together
// with csrc/host_setup.cpp).  Every check failure prints a message and exits 1; the
// sanitizers abort on their own findings.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <random>
#include <string>
#include <vector>

#include "sem_host.h"

static int g_fail = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            std::fprintf(stderr, "CHECK failed: " #c " -- "); \
            std::fprintf(stderr, __VA_ARGS__);          \
            std::fprintf(stderr, "\n");                 \
            g_fail = 1;                                 \
        }                                              \
    } while (0)

static void check_space(int lx)
{
    std::vector<double> xi(lx), w(lx), D(lx * lx);
    semh::gll_space(lx, xi.data(), w.data(), D.data());
    double sw = 0;
    for (double v : w) sw += v;
    CHECK(std::fabs(sw - 2.0) < 1e-13, "lx=%d sum w = %.17g", lx, sw);
    for (int i = 0; i < lx; ++i) {  // D applied to x is 1, to a constant 0
        double d1 = 0, d0 = 0;
        for (int j = 0; j < lx; ++j) {
            d1 += D[i * lx + j] * xi[j];
            d0 += D[i * lx + j];
        }
        CHECK(std::fabs(d1 - 1.0) < 1e-10 && std::fabs(d0) < 1e-10, "lx=%d row %d", lx, i);
    }
}

static void check_maps(int nx, int ny, int nz, int lx)
{
    std::vector<double> xi(lx), w(lx), D(lx * lx);
    semh::gll_space(lx, xi.data(), w.data(), D.data());
    const int64_t n = (int64_t)nx * ny * nz * lx * lx * lx;
    std::vector<int64_t> glb(n);
    std::vector<uint8_t> dir(n);
    std::vector<double> xyz(3 * n);
    semh::box_mesh(nx, ny, nz, lx, 0.05, xi.data(), glb.data(), dir.data(), xyz.data());
    semh::GsMaps m;
    std::string msg;
    CHECK(semh::build_gs_maps(n, glb.data(), dir.data(), m, msg), "%s", msg.c_str());
    int64_t total = 0, owners = 0;
    for (int64_t i = 0; i < n; ++i) {
        total += 1;
        owners += m.owner[i];
    }
    const int64_t ux = (int64_t)nx * (lx - 1) + 1, uy = (int64_t)ny * (lx - 1) + 1, uz = (int64_t)nz * (lx - 1) + 1;
    CHECK(owners == ux * uy * uz, "%dx%dx%d lx=%d owners %lld", nx, ny, nz, lx, (long long)owners);
    CHECK(m.n_unique == ux * uy * uz, "n_unique %lld", (long long)m.n_unique);
    // every shared point appears exactly once among pairs, blocks and entries
    std::vector<int> seen(n, 0);
    for (int32_t v : m.pairs) seen[v] += 1;
    for (int32_t v : m.blk_idx) seen[v] += 1;
    for (int64_t i = 0; i < n; ++i) CHECK(seen[i] == (m.mult[i] > 1 ? 1 : 0), "point %lld", (long long)i);
    std::vector<int> seen_e(n, 0);
    for (size_t q = 0; q < m.ent_idx.size(); ++q)
        if (m.ent_idx[q] >= 0) seen_e[m.ent_idx[q]] += 1;
    for (int64_t i = 0; i < n; ++i) CHECK(seen_e[i] == (m.mult[i] > 1 ? 1 : 0), "entry %lld", (long long)i);
    std::vector<int32_t> pairs, blk_idx;
    std::vector<int64_t> blk_ptr;
    semh::element_order(m, pairs, blk_ptr, blk_idx);
    CHECK(pairs.size() == m.pairs.size() && blk_idx.size() == m.blk_idx.size(), "element order sizes");
    (void)total;
}

// Irregular ids: random global ids drawn from a small range (groups of any size,
// including groups above 64 copies, which take the CSR-only path).
static void check_random_ids(int64_t n, int64_t range, unsigned seed)
{
    std::mt19937_64 rng(seed);
    std::vector<int64_t> glb(n);
    for (auto &g : glb) g = (int64_t)(rng() % range) * 1000003;  // sparse id range
    semh::GsMaps m;
    std::string msg;
    CHECK(semh::build_gs_maps(n, glb.data(), nullptr, m, msg), "%s", msg.c_str());
    int64_t owners = 0;
    for (int64_t i = 0; i < n; ++i) owners += m.owner[i];
    CHECK(owners == m.n_unique, "random ids: owners %lld vs %lld", (long long)owners, (long long)m.n_unique);
}

static void check_eig(int n, unsigned seed)
{
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(-1, 1);
    std::vector<double> a(n * n), a0, V(n * n), lam(n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) a[i * n + j] = a[j * n + i] = U(rng);
    a0 = a;
    semh::sym_eig(n, a.data(), V.data(), lam.data());
    double err = 0, scale = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0;
            for (int k = 0; k < n; ++k) s += V[i * n + k] * lam[k] * V[j * n + k];
            err = std::fmax(err, std::fabs(s - a0[i * n + j]));
            scale = std::fmax(scale, std::fabs(a0[i * n + j]));
        }
    CHECK(err <= 1e-12 * n * scale, "sym_eig n=%d err %.3e", n, err);
}

// Face neighbours on a box mesh whose elements are each re-indexed by a random one of
// the 48 symmetries of the cube (axis permutation and flips): every face point's
// extension point must be the grid point one step outward along the face's global
// normal, present exactly when the element's face is inside the box.
static void check_faces(int nx, int ny, int nz, int lx, unsigned seed)
{
    std::vector<double> xi(lx), w(lx), D(lx * lx);
    semh::gll_space(lx, xi.data(), w.data(), D.data());
    const int N = lx - 1;
    const int64_t lx3 = (int64_t)lx * lx * lx, nelv = (int64_t)nx * ny * nz;
    std::vector<int64_t> g0(nelv * lx3), glb(nelv * lx3);
    semh::box_mesh(nx, ny, nz, lx, 0.0, xi.data(), g0.data(), nullptr, nullptr);
    const int64_t Mx = (int64_t)nx * N + 1, My = (int64_t)ny * N + 1;
    const int64_t gstride[3] = {1, Mx, Mx * My};
    const int nel[3] = {nx, ny, nz};
    std::mt19937_64 rng(seed);
    std::vector<int> perm((size_t)nelv * 3), flip((size_t)nelv * 3);
    for (int64_t e = 0; e < nelv; ++e) {
        int s[3] = {0, 1, 2};
        std::shuffle(s, s + 3, rng);
        for (int m = 0; m < 3; ++m) {
            perm[e * 3 + m] = s[m];
            flip[e * 3 + m] = (int)(rng() & 1);
        }
        for (int64_t p = 0; p < lx3; ++p) {
            const int c[3] = {(int)(p % lx), (int)((p / lx) % lx), (int)(p / (lx * lx))};
            int cn[3];
            for (int m = 0; m < 3; ++m) cn[m] = flip[e * 3 + m] ? N - c[perm[e * 3 + m]] : c[perm[e * 3 + m]];
            glb[e * lx3 + cn[0] + lx * (cn[1] + lx * cn[2])] = g0[e * lx3 + p];
        }
    }
    std::vector<int32_t> fn;
    std::string msg;
    const bool ok = semh::face_neighbours(nelv, lx, glb.data(), fn, msg);
    CHECK(ok, "%s", msg.c_str());
    if (!ok) return;
    for (int64_t e = 0; e < nelv; ++e) {
        const int64_t ec[3] = {e % nx, (e / nx) % ny, e / ((int64_t)nx * ny)};
        for (int f = 0; f < 6; ++f) {
            const int d = f / 2, side = f & 1;
            const int ga = perm[e * 3 + d];                           // global axis of the normal
            const int oldc = flip[e * 3 + d] ? N - side * N : side * N;  // old coordinate: 0 or N
            const int dirn = oldc == 0 ? -1 : 1;
            const bool inside = dirn < 0 ? ec[ga] > 0 : ec[ga] < nel[ga] - 1;
            const int32_t *o = &fn[(size_t)(e * 6 + f) * 4];
            CHECK((o[0] >= 0) == inside, "e %lld face %d neighbour %d", (long long)e, f, o[0]);
            if (o[0] < 0 || !inside) continue;
            for (int fb = 0; fb <= N; ++fb)
                for (int fa = 0; fa <= N; ++fa) {
                    int c[3];
                    c[d] = side * N;
                    c[d == 0 ? 1 : 0] = fa;
                    c[d == 2 ? 1 : 2] = fb;
                    const int64_t gp = glb[e * lx3 + c[0] + lx * (c[1] + lx * c[2])];
                    const int64_t q = o[1] + (int64_t)fa * o[2] + (int64_t)fb * o[3];
                    CHECK(q >= 0 && q < lx3, "e %lld face %d point (%d, %d): index %lld", (long long)e, f, fa, fb,
                          (long long)q);
                    if (q < 0 || q >= lx3) continue;
                    CHECK(glb[(int64_t)o[0] * lx3 + q] == gp + dirn * gstride[ga],
                          "e %lld face %d point (%d, %d): extension id %lld, want %lld", (long long)e, f, fa, fb,
                          (long long)glb[(int64_t)o[0] * lx3 + q], (long long)(gp + dirn * gstride[ga]));
                }
        }
    }
}

// Error paths of the face-neighbour builder: a face held by three elements (an element
// repeated twice more), and two elements whose shared face corners match while the
// points inside the face do not.
static void check_faces_invalid()
{
    const int lx = 3;
    const int64_t lx3 = 27;
    std::vector<double> xi(lx), w(lx), D(lx * lx);
    semh::gll_space(lx, xi.data(), w.data(), D.data());
    std::vector<int64_t> one(lx3), glb(3 * lx3);
    semh::box_mesh(1, 1, 1, lx, 0.0, xi.data(), one.data(), nullptr, nullptr);
    for (int r = 0; r < 3; ++r)
        for (int64_t p = 0; p < lx3; ++p) glb[r * lx3 + p] = one[p];
    std::vector<int32_t> fn;
    std::string msg;
    CHECK(!semh::face_neighbours(3, lx, glb.data(), fn, msg), "three elements on one face accepted");
    CHECK(msg.find("more than two") != std::string::npos, "message: %s", msg.c_str());
    std::vector<int64_t> two(2 * lx3);
    semh::box_mesh(2, 1, 1, lx, 0.0, xi.data(), two.data(), nullptr, nullptr);
    // the shared face of element 1 is i = 0; give its centre point a fresh id
    two[lx3 + 0 + lx * (1 + lx * 1)] = 1000000;
    msg.clear();
    CHECK(!semh::face_neighbours(2, lx, two.data(), fn, msg), "mismatched face interior accepted");
    CHECK(msg.find("not its points") != std::string::npos, "message: %s", msg.c_str());
    // one element, periodic in r (the i = lx - 1 face takes the ids of the i = 0 face): no
    // neighbour on either face
    std::vector<int64_t> per(one);
    for (int k = 0; k < lx; ++k)
        for (int j = 0; j < lx; ++j) per[(lx - 1) + lx * (j + lx * k)] = per[0 + lx * (j + lx * k)];
    msg.clear();
    CHECK(semh::face_neighbours(1, lx, per.data(), fn, msg), "%s", msg.c_str());
    CHECK(fn[0] == -1 && fn[4] == -1, "periodic self-neighbour: %d %d", fn[0], fn[4]);
}

int main()
{
    for (int lx = 2; lx <= 16; ++lx) check_space(lx);
    check_maps(1, 1, 1, 2);
    check_maps(2, 2, 2, 3);
    check_maps(3, 2, 1, 4);
    check_maps(4, 4, 4, 8);
    check_maps(2, 3, 5, 12);
    check_random_ids(1, 1, 1);
    check_random_ids(5000, 37, 2);     // large groups (> 64 copies)
    check_random_ids(20000, 9000, 3);  // mostly pairs and singletons
    for (int n : {1, 2, 5, 14, 18}) check_eig(n, 10 + n);
    check_faces(1, 1, 1, 3, 7);
    check_faces(2, 1, 1, 2, 8);
    check_faces(3, 2, 2, 4, 9);
    check_faces(3, 3, 3, 5, 10);
    check_faces(2, 3, 4, 8, 11);
    check_faces_invalid();
    std::vector<int64_t> hits(100000, 0);
    semh::parallel_for((int64_t)hits.size(), [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) hits[i] += 1;
    }, 1000);
    for (int64_t v : hits) CHECK(v == 1, "parallel_for coverage");
    if (g_fail) return 1;
    std::printf("host setup under sanitizers: ok\n");
    return 0;
}
