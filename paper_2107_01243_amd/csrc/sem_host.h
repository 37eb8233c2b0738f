// sem_host.h -- host-side helpers of libsem (internal).
#pragma once
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

namespace semh {

struct GsMaps {
    int64_t n = 0;
    int64_t n_unique = 0;
    std::vector<int32_t> pairs;    // (a, b) with a < b, ascending global id
    std::vector<int64_t> blk_ptr;  // CSR over blocks of >2 copies, ascending global id
    std::vector<int32_t> blk_idx;  // ascending local index inside a block
    std::vector<uint8_t> mult;     // copies of each local point's global id
    std::vector<uint8_t> owner;    // 1 on the lowest local index of every global id
    // Entry-parallel form of the same groups, ascending global id: one entry per
    // shared local point; a group never straddles a 64-entry (wave) boundary, gaps
    // are padding entries (index -1).  meta = position in group | (group size << 8).
    std::vector<int32_t> ent_idx;
    std::vector<uint16_t> ent_meta;
    int max_group = 0;             // largest group size among the entries
    // Groups with more than 64 copies (never in hexahedral box meshes) use CSR only.
    std::vector<int64_t> big_ptr;
    std::vector<int32_t> big_idx;
};

// fn(lo, hi) over [0, n) split across host threads, each taking at least `grain`
// items (serial below that).
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn, int64_t grain = 65536);
void gll_space(int lx, double *xi, double *w, double *D);
void box_mesh(int nx, int ny, int nz, int lx, double eps, const double *xi, int64_t *glb,
              uint8_t *dir, double *xyz);
bool build_gs_maps(int64_t n, const int64_t *glb, const uint8_t *dir, GsMaps &m, std::string &msg);
// The same groups reordered by their lowest local index (execution order on the device).
void element_order(const GsMaps &m, std::vector<int32_t> &pairs, std::vector<int64_t> &blk_ptr,
                   std::vector<int32_t> &blk_idx);

// Face neighbours of a conforming hexahedral mesh, from its global ids.  Face
// f = 2 d + side of an element holds the points whose local coordinate d is 0 (side 0)
// or lx - 1 (side 1); its face coordinates (fa, fb) are the two other local
// coordinates in ascending direction order.  out[(e * 6 + f) * 4 + 0..3] =
// {e2, base, sa, sb}: e2 the other element holding the face (every point of it, at
// matching grid positions), and, for face point (fa, fb), base + fa sa + fb sb the
// local index in e2 of the point one GLL index inside e2 from that point's copy;
// e2 = -1 (and zeros) where no other element holds the face (an element holding both
// copies of a periodic face is not its own neighbour).  Returns false (msg
// set) when a face is held by more than two elements or two elements share a face's
// corners but not its points.
bool face_neighbours(int64_t nelv, int lx, const int64_t *glb, std::vector<int32_t> &out, std::string &msg);

// Symmetric eigen-decomposition a = V diag(lam) V^T of the n x n row-major matrix a
// (destroyed) by cyclic Jacobi rotations; V row-major [row][mode].
void sym_eig(int n, double *a, double *V, double *lam);

}  // namespace semh
