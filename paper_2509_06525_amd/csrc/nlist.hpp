// Cell-list neighbour search on the GPU (internal).
//
// Atoms are binned into cells at least r_cut wide; an axis with fewer than
// three cells is scanned whole so no cell is visited twice.  Displacements are
// formed in FP64 under the minimum-image convention on periodic axes.
// Several independent structures ("segments", stacked along the atom index)
// can be binned at once: each has its own cell grid and its own range of
// global cell ids, and neighbours are only searched inside the segment.
#pragma once

#include "common.hpp"

namespace tbk {

// Cells are numbered in strips: the x axis is cut into strips of `strip`
// cells; cells are ordered by (z, strip, y, x within the strip), so cells that
// touch in y are `strip` ids apart and atoms sorted by cell id keep their
// neighbours close in memory.
struct CellGrid {
    double lo[3];       // origin of the binned range
    double len[3];      // length of the binned range
    int32_t nc[3];      // cells per axis (>= 1)
    int32_t periodic[3];
    double box[3];      // periodic lengths
    int32_t strip;      // cells per strip along x (>= 1)
    int32_t nstrip;     // ceil(nc[0] / strip)
    int64_t ncell;      // number of cell ids: nc[2] * nstrip * nc[1] * strip
    int64_t cell_off;   // first global cell id of this grid's segment
};

__host__ __device__ __forceinline__ int64_t cell_id(const CellGrid &g, int32_t cx, int32_t cy, int32_t cz) {
    const int32_t st = cx / g.strip, wx = cx - st * g.strip;
    return (((int64_t)cz * g.nstrip + st) * g.nc[1] + cy) * g.strip + wx;
}

// Device-side view of a built cell list.
struct CellList {
    const CellGrid *grids;      // [n_seg]
    const int32_t *seg_of;      // [n] segment of each atom
    const int32_t *cell_start;  // [ncell_total + 1]
    const int32_t *sorted;      // [n] atom indices, cell-major, ascending within a cell
};

__device__ __forceinline__ double min_image(double d, double L, int periodic) {
    return periodic ? __dsub_rn(d, __dmul_rn(L, rint(d / L))) : d;
}

__device__ __forceinline__ int32_t cell_coord(double x, const CellGrid &g, int k) {
    double u = (x - g.lo[k]) / g.len[k];
    if (g.periodic[k]) u -= floor(u);
    int32_t c = (int32_t)floor(u * (double)g.nc[k]);
    c = c < 0 ? 0 : c;
    c = c >= g.nc[k] ? g.nc[k] - 1 : c;
    return c;
}

// Calls f(j, r, dx, dy, dz) for every atom j != i of i's segment with
// |x_j - x_i| < r_cut (minimum image), visiting cells in a fixed order.
template <class F>
__device__ __forceinline__ void for_each_neighbor(const CellList &cl, const double *__restrict__ pos,
                                                  int32_t i, double r_cut, F &&f) {
    const CellGrid g = cl.grids[cl.seg_of[i]];
    const double xi = pos[3 * (int64_t)i], yi = pos[3 * (int64_t)i + 1], zi = pos[3 * (int64_t)i + 2];
    int32_t c[3] = {cell_coord(xi, g, 0), cell_coord(yi, g, 1), cell_coord(zi, g, 2)};
    int32_t lo[3], cnt[3];
    for (int k = 0; k < 3; ++k) {
        if (g.nc[k] >= 3) { lo[k] = c[k] - 1; cnt[k] = 3; }
        else { lo[k] = 0; cnt[k] = g.nc[k]; }
    }
    // Cheap pre-filter slightly above r_cut^2; the decision itself is r < r_cut.
    const double rc2_hi = r_cut * r_cut * (1.0 + 1e-12);
    for (int a = 0; a < cnt[2]; ++a) {
        int32_t cz = lo[2] + a;
        if (cz < 0 || cz >= g.nc[2]) {
            if (!g.periodic[2]) continue;
            cz = (cz + g.nc[2]) % g.nc[2];
        }
        for (int b = 0; b < cnt[1]; ++b) {
            int32_t cy = lo[1] + b;
            if (cy < 0 || cy >= g.nc[1]) {
                if (!g.periodic[1]) continue;
                cy = (cy + g.nc[1]) % g.nc[1];
            }
            for (int e = 0; e < cnt[0]; ++e) {
                int32_t cx = lo[0] + e;
                if (cx < 0 || cx >= g.nc[0]) {
                    if (!g.periodic[0]) continue;
                    cx = (cx + g.nc[0]) % g.nc[0];
                }
                const int64_t cid = g.cell_off + cell_id(g, cx, cy, cz);
                int32_t s0 = cl.cell_start[cid], s1 = cl.cell_start[cid + 1];
                for (int32_t s = s0; s < s1; ++s) {
                    int32_t j = cl.sorted[s];
                    if (j == i) continue;
                    double dx = min_image(pos[3 * (int64_t)j] - xi, g.box[0], g.periodic[0]);
                    double dy = min_image(pos[3 * (int64_t)j + 1] - yi, g.box[1], g.periodic[1]);
                    double dz = min_image(pos[3 * (int64_t)j + 2] - zi, g.box[2], g.periodic[2]);
                    // Uncontracted sum of squares: the same rounding for (i, j) and (j, i).
                    double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
                    if (r2 < rc2_hi) {
                        double r = sqrt(r2);
                        if (r < r_cut) f(j, r, dx, dy, dz);
                    }
                }
            }
        }
    }
}

// Owns the device buffers of a cell list built for stacked structures.
struct CellListOwner {
    CellList view{};
    int32_t n_seg = 0;
    DevBuf grids, seg_of, seg_atoms, cell_start, sorted;
    // Bins positions pos[n][3] of n_seg structures; structure s holds atoms
    // [seg_atoms[s], seg_atoms[s+1]) (host array) and, on periodic axes, the
    // box boxes[3 s .. 3 s + 2] (host).  Validates box lengths, finiteness and
    // (when species != nullptr) the species range.
    tbk_status build(const double *pos, const int32_t *species, int32_t n_species, int64_t n, int32_t n_seg,
                     const int64_t *seg_atoms, const double *boxes, const int32_t periodic[3], double r_cut,
                     hipStream_t s);
};

}  // namespace tbk
