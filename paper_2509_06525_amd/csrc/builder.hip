// Neighbour list and Hamiltonian assembly on the GPU (Eq. (1)).
//
// Build sequence for n_seg stacked structures (one structure = one segment):
//   1. k_segment_scan: per-segment coordinate range, NaN/Inf and species checks
//   2. cell list: cell id per atom (per-segment grids, global ids), counts,
//      exclusive scan, scatter, per-cell sort by atom index
//   3. k_degree: neighbours within r_cut per row
//   4. slice widths (max degree per slice) -> slice offsets (exclusive scan)
//   5. k_fill: columns and FP64 hoppings of each row, padding, in-row sort by
//      column, onsite, per-segment row Gershgorin bounds
// CSR is handled as SELL with slice height 1.  Rows of segment s occupy the
// segment's atom range, so stacked systems keep their own row blocks.
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstring>
#include <vector>

#include "builder.hpp"
#include "nlist.hpp"

namespace tbk {

namespace {

constexpr int kMaxDegree = 256;
constexpr int kMaxSpecies = 16;
constexpr int kCellStrip = 64;      // cells per strip of the row order

// seg_of[i] = s with seg_atoms[s] <= i < seg_atoms[s + 1] (offsets strictly
// increasing, so the binary search has one answer).
__global__ void k_seg_of(int64_t n, int32_t nseg, const int64_t *__restrict__ seg_atoms,
                         int32_t *__restrict__ seg_of) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (seg_atoms[mid] <= i) lo = mid;
        else hi = mid;
    }
    seg_of[i] = lo;
}

constexpr int kScanChunk = 16;      // atoms per thread in k_segment_scan

// Per-segment coordinate ranges and input checks over the whole grid.
// keys[(k n_seg + s) 2 + {0, 1}] = order-preserving keys of min / max of
// coordinate k over the finite coordinates of segment s (k_init_bounds start);
// flags[2 s] = 1 if some coordinate of s is NaN/Inf, flags[2 s + 1] = 1 if a
// species index is outside [0, n_species) (flags start at 0).  A block covers
// kScanChunk * kBlock consecutive atoms; a thread flushes its running range
// with atomics when its atoms cross into another segment, and the block folds
// the last ranges per segment before one atomic per segment and coordinate.
__global__ __launch_bounds__(kBlock) void k_segment_scan(const double *__restrict__ pos,
                                                         const int32_t *__restrict__ species, int64_t n,
                                                         const int32_t *__restrict__ seg_of, int32_t nseg,
                                                         int32_t n_species, int64_t *__restrict__ keys,
                                                         int32_t *__restrict__ flags) {
    const int64_t base = (int64_t)blockIdx.x * kBlock * kScanChunk;
    double mn[3], mx[3];
    int32_t cur = -1;
    auto reset = [&]() {
        for (int k = 0; k < 3; ++k) { mn[k] = INFINITY; mx[k] = -INFINITY; }
    };
    reset();
    for (int u = 0; u < kScanChunk; ++u) {
        const int64_t i = base + (int64_t)u * kBlock + threadIdx.x;
        if (i >= n) break;
        const int32_t sg = seg_of[i];
        if (sg != cur) {
            if (cur >= 0) {
                for (int k = 0; k < 3; ++k)
                    if (mn[k] <= mx[k]) {
                        atomicMin((long long *)&keys[2 * ((int64_t)k * nseg + cur)], (long long)dkey(mn[k]));
                        atomicMax((long long *)&keys[2 * ((int64_t)k * nseg + cur) + 1], (long long)dkey(mx[k]));
                    }
            }
            cur = sg;
            reset();
        }
        for (int k = 0; k < 3; ++k) {
            const double x = pos[3 * i + k];
            if (!isfinite(x)) flags[2 * sg] = 1;
            else { mn[k] = fmin(mn[k], x); mx[k] = fmax(mx[k], x); }
        }
        if (species) {
            const int32_t t = species[i];
            if (t < 0 || t >= n_species) flags[2 * sg + 1] = 1;
        }
    }
    for (int k = 0; k < 3; ++k) block_segment_bounds(mn[k], mx[k], cur < 0 ? -1 : k * nseg + cur, keys);
}

__global__ void k_cell_of(const double *__restrict__ pos, int64_t n, const CellGrid *__restrict__ grids,
                          const int32_t *__restrict__ seg_of, int32_t *__restrict__ cell,
                          int32_t *__restrict__ slot, int32_t *__restrict__ count) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const CellGrid g = grids[seg_of[i]];
    int32_t cx = cell_coord(pos[3 * i], g, 0);
    int32_t cy = cell_coord(pos[3 * i + 1], g, 1);
    int32_t cz = cell_coord(pos[3 * i + 2], g, 2);
    int32_t c = (int32_t)(g.cell_off + cell_id(g, cx, cy, cz));
    cell[i] = c;
    slot[i] = atomicAdd(&count[c], 1);
}

__global__ void k_scatter(int64_t n, const int32_t *__restrict__ cell, const int32_t *__restrict__ slot,
                          const int32_t *__restrict__ start, int32_t *__restrict__ sorted) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    sorted[start[cell[i]] + slot[i]] = (int32_t)i;
}

// Ascending atom order inside each cell (the scatter order depends on atomics).
__global__ void k_sort_cells(int64_t ncell, const int32_t *__restrict__ start, int32_t *__restrict__ sorted) {
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int32_t s0 = start[c], s1 = start[c + 1];
    for (int32_t a = s0 + 1; a < s1; ++a) {
        int32_t v = sorted[a];
        int32_t b = a - 1;
        while (b >= s0 && sorted[b] > v) { sorted[b + 1] = sorted[b]; --b; }
        sorted[b + 1] = v;
    }
}

__global__ void k_perm(int64_t n, int32_t reorder, const int32_t *__restrict__ sorted,
                       int32_t *__restrict__ perm, int32_t *__restrict__ iperm) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    int32_t a = reorder ? sorted[r] : (int32_t)r;
    perm[r] = a;
    iperm[a] = (int32_t)r;
}

__global__ void k_degree(CellList cl, const double *__restrict__ pos, int64_t n, double r_cut,
                         const int32_t *__restrict__ perm, int32_t *__restrict__ deg) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    int32_t cnt = 0;
    for_each_neighbor(cl, pos, perm[r], r_cut, [&](int32_t, double, double, double, double) { ++cnt; });
    deg[r] = cnt;
}

// Width of each slice (largest degree among its rows) and its stored entries.
__global__ void k_slice_width(int64_t n, int32_t slice, int64_t n_slices, const int32_t *__restrict__ deg,
                              int64_t *__restrict__ entries) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    int32_t w = 0;
    int64_t r1 = (s + 1) * slice < n ? (s + 1) * slice : n;
    for (int64_t r = s * slice; r < r1; ++r) w = deg[r] > w ? deg[r] : w;
    entries[s] = (int64_t)w * slice;
}

__global__ void k_init_bounds(int32_t n_seg, int64_t *__restrict__ keys) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_seg) return;
    keys[2 * s] = dkey(INFINITY);
    keys[2 * s + 1] = dkey(-INFINITY);
}

struct SpeciesTable {
    double onsite[kMaxSpecies];
    double t_pair[kMaxSpecies * kMaxSpecies];
};

template <class V>
__global__ void k_fill(CellList cl, const double *__restrict__ pos, const int32_t *__restrict__ species,
                       int64_t n, int32_t slice, double r_cut, double r0, double beta, int32_t n_species,
                       const SpeciesTable *__restrict__ tab, const int32_t *__restrict__ perm,
                       const int32_t *__restrict__ iperm, const int64_t *__restrict__ ptr,
                       int32_t *__restrict__ col, V *__restrict__ val, V *__restrict__ onsite,
                       int64_t *__restrict__ bound_keys, int64_t *__restrict__ val_keys,
                       int16_t *__restrict__ col16) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    double vlo = INFINITY, vhi = -INFINITY;   // range of the stored hoppings
    int32_t sg = -1;
    if (r < n) {
        const int64_t s = r / slice, lane = r - s * slice;
        const int64_t base = ptr[s] + lane;
        const int32_t w = (int32_t)((ptr[s + 1] - ptr[s]) / slice);
        const int32_t i = perm[r];
        const int32_t si = species[i];
        sg = cl.seg_of[i];
        int32_t k = 0;
        double asum = 0.0;
        for_each_neighbor(cl, pos, i, r_cut, [&](int32_t j, double rij, double, double, double) {
            double t = tab->t_pair[si * n_species + species[j]] * exp(-beta * (rij / r0 - 1.0));
            if (k < w) {
                col[base + (int64_t)k * slice] = iperm[j];
                val[base + (int64_t)k * slice] = (V)t;
            }
            vlo = fmin(vlo, (double)(V)t);
            vhi = fmax(vhi, (double)(V)t);
            asum += fabs(t);
            ++k;
        });
        for (int32_t q = k; q < w; ++q) {
            col[base + (int64_t)q * slice] = (int32_t)r;
            val[base + (int64_t)q * slice] = (V)0;
        }
        // Insertion sort of the row's real entries by column.
        int32_t kk = k < w ? k : w;
        for (int32_t a = 1; a < kk; ++a) {
            int32_t c = col[base + (int64_t)a * slice];
            V v = val[base + (int64_t)a * slice];
            int32_t b = a - 1;
            while (b >= 0 && col[base + (int64_t)b * slice] > c) {
                col[base + (int64_t)(b + 1) * slice] = col[base + (int64_t)b * slice];
                val[base + (int64_t)(b + 1) * slice] = val[base + (int64_t)b * slice];
                --b;
            }
            col[base + (int64_t)(b + 1) * slice] = c;
            val[base + (int64_t)(b + 1) * slice] = v;
        }
        if (col16) {    // 16-bit column offsets (escape -32768: read col)
            for (int32_t q = 0; q < w; ++q) {
                const int64_t d = (int64_t)col[base + (int64_t)q * slice] - r;
                col16[base + (int64_t)q * slice] = (d >= -32767 && d <= 32767) ? (int16_t)d : (int16_t)-32768;
            }
        }
        double eps = tab->onsite[si];
        onsite[r] = (V)eps;
        lo = eps - asum;
        hi = eps + asum;
    }
    block_segment_bounds(lo, hi, sg, bound_keys);
    block_segment_bounds(vlo, vhi, vlo <= vhi ? 0 : -1, val_keys);
}

template <class T>
tbk_status exclusive_scan(const T *in, T *out, int64_t n, hipStream_t s) {
    size_t tmp = 0;
    TBK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, in, out, (int)n, s));
    DevBuf t;
    TBK_HIP(t.alloc(tmp, s));
    TBK_HIP(hipcub::DeviceScan::ExclusiveSum(t.as<void>(), tmp, in, out, (int)n, s));
    return TBK_OK;
}

int32_t any_onsite(const tbk_tb_params *p) {
    for (int i = 0; i < p->n_species; ++i)
        if (p->onsite[i] != 0.0) return 1;
    return 0;
}

}  // namespace

tbk_status check_tb_params(const tbk_tb_params *p) {
    TBK_CHECK(p != nullptr, TBK_ERR_INVALID_ARG, "params is NULL");
    TBK_CHECK(std::isfinite(p->r_cut) && std::isfinite(p->r0) && std::isfinite(p->beta), TBK_ERR_NOT_FINITE,
              "r_cut, r0 or beta is not finite");
    TBK_CHECK(p->r_cut > 0 && p->r0 > 0 && p->beta >= 0, TBK_ERR_INVALID_ARG,
              "r_cut and r0 must be positive and beta non-negative");
    TBK_CHECK(p->n_species >= 1 && p->n_species <= kMaxSpecies, TBK_ERR_INVALID_ARG,
              "n_species must be in [1, %d]", kMaxSpecies);
    TBK_CHECK(p->onsite && p->t_pair, TBK_ERR_INVALID_ARG, "onsite/t_pair is NULL");
    for (int i = 0; i < p->n_species; ++i) {
        TBK_CHECK(std::isfinite(p->onsite[i]), TBK_ERR_NOT_FINITE, "onsite[%d] is not finite", i);
        for (int j = 0; j < p->n_species; ++j) {
            TBK_CHECK(std::isfinite(p->t_pair[i * p->n_species + j]), TBK_ERR_NOT_FINITE,
                      "t_pair[%d][%d] is not finite", i, j);
            TBK_CHECK(p->t_pair[i * p->n_species + j] == p->t_pair[j * p->n_species + i],
                      TBK_ERR_INVALID_ARG, "t_pair is not symmetric");
        }
    }
    return TBK_OK;
}

void decode_bounds(const std::vector<int64_t> &keys, int nseg, double *bounds) {
    for (int g = 0; g < nseg; ++g) {
        bounds[2 * g] = dunkey(keys[2 * g]);
        bounds[2 * g + 1] = dunkey(keys[2 * g + 1]);
    }
}

tbk_status init_bound_keys(DevBuf &keys, int nseg, hipStream_t s) {
    TBK_HIP(keys.alloc(sizeof(int64_t) * 2 * nseg, s));
    k_init_bounds<<<(nseg + 255) / 256, 256, 0, s>>>(nseg, keys.as<int64_t>());
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

tbk_status CellListOwner::build(const double *pos, const int32_t *species, int32_t n_species, int64_t n,
                                int32_t nseg, const int64_t *seg_atoms_h, const double *boxes,
                                const int32_t periodic[3], double r_cut, hipStream_t s) {
    TBK_CHECK(pos && boxes && periodic && seg_atoms_h, TBK_ERR_INVALID_ARG, "NULL position/box/periodic/segments");
    TBK_CHECK(n >= 1 && n < (int64_t)INT32_MAX, TBK_ERR_INVALID_ARG, "n = %lld out of [1, 2^31-1)", (long long)n);
    TBK_CHECK(nseg >= 1 && nseg <= (1 << 20), TBK_ERR_INVALID_ARG, "n_seg = %d out of [1, 2^20]", nseg);
    TBK_CHECK(seg_atoms_h[0] == 0 && seg_atoms_h[nseg] == n, TBK_ERR_INVALID_ARG,
              "segment offsets must start at 0 and end at n");
    for (int g = 0; g < nseg; ++g)
        TBK_CHECK(seg_atoms_h[g + 1] > seg_atoms_h[g], TBK_ERR_INVALID_ARG, "segment %d is empty or unordered", g);
    for (int k = 0; k < 3; ++k)
        TBK_CHECK(periodic[k] == 0 || periodic[k] == 1, TBK_ERR_INVALID_ARG, "periodic[%d] must be 0 or 1", k);
    for (int g = 0; g < nseg; ++g)
        for (int k = 0; k < 3; ++k)
            if (periodic[k]) {
                const double L = boxes[3 * g + k];
                TBK_CHECK(std::isfinite(L), TBK_ERR_NOT_FINITE, "box[%d] of segment %d is not finite", k, g);
                TBK_CHECK(L >= 2.0 * r_cut, TBK_ERR_INVALID_ARG,
                          "periodic length %g (axis %d, segment %d) is below 2 r_cut = %g", L, k, g, 2.0 * r_cut);
            }
    n_seg = nseg;
    TBK_HIP(seg_atoms.alloc(sizeof(int64_t) * (nseg + 1), s));
    TBK_HIP(seg_of.alloc(sizeof(int32_t) * n, s));
    TBK_HIP(hipMemcpyAsync(seg_atoms.as<int64_t>(), seg_atoms_h, sizeof(int64_t) * (nseg + 1),
                           hipMemcpyHostToDevice, s));
    const int gseg = (int)ceil_div(n, kBlock);
    k_seg_of<<<gseg, kBlock, 0, s>>>(n, nseg, seg_atoms.as<int64_t>(), seg_of.as<int32_t>());
    TBK_HIP(hipGetLastError());

    // 1. ranges and validity per segment
    DevBuf rkeys, rflags;
    TBK_HIP(rkeys.alloc(sizeof(int64_t) * 6 * nseg, s));
    TBK_HIP(rflags.alloc(sizeof(int32_t) * 2 * nseg, s));
    k_init_bounds<<<(3 * nseg + 255) / 256, 256, 0, s>>>(3 * nseg, rkeys.as<int64_t>());
    TBK_HIP(hipGetLastError());
    TBK_HIP(hipMemsetAsync(rflags.as<int32_t>(), 0, sizeof(int32_t) * 2 * nseg, s));
    k_segment_scan<<<(unsigned)ceil_div(n, (int64_t)kBlock * kScanChunk), kBlock, 0, s>>>(
        pos, species, n, seg_of.as<int32_t>(), nseg, n_species, rkeys.as<int64_t>(), rflags.as<int32_t>());
    TBK_HIP(hipGetLastError());
    std::vector<int64_t> hk(6 * (size_t)nseg);
    std::vector<int32_t> hf(2 * (size_t)nseg);
    TBK_HIP(hipMemcpyAsync(hk.data(), rkeys.as<int64_t>(), sizeof(int64_t) * 6 * nseg, hipMemcpyDeviceToHost, s));
    TBK_HIP(hipMemcpyAsync(hf.data(), rflags.as<int32_t>(), sizeof(int32_t) * 2 * nseg, hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    // hp[8 g + k] = min, hp[8 g + 3 + k] = max of coordinate k in segment g
    std::vector<double> hp(8 * (size_t)nseg);
    for (int g = 0; g < nseg; ++g) {
        TBK_CHECK(hf[2 * g] == 0, TBK_ERR_NOT_FINITE, "a coordinate of segment %d is NaN or Inf", g);
        TBK_CHECK(hf[2 * g + 1] == 0, TBK_ERR_INVALID_ARG, "a species index of segment %d is outside [0, %d)",
                  g, n_species);
        for (int k = 0; k < 3; ++k) {
            hp[8 * g + k] = dunkey(hk[2 * ((size_t)k * nseg + g)]);
            hp[8 * g + 3 + k] = dunkey(hk[2 * ((size_t)k * nseg + g) + 1]);
        }
    }

    // 2. one cell grid per segment, global cell ids
    std::vector<CellGrid> hg(nseg);
    int64_t off = 0;
    for (int g = 0; g < nseg; ++g) {
        CellGrid &c = hg[g];
        const int64_t na = seg_atoms_h[g + 1] - seg_atoms_h[g];
        int64_t ncell = 1;
        for (int k = 0; k < 3; ++k) {
            c.periodic[k] = periodic[k];
            c.box[k] = periodic[k] ? boxes[3 * g + k] : 0.0;
            if (periodic[k]) { c.lo[k] = 0.0; c.len[k] = boxes[3 * g + k]; }
            else { c.lo[k] = hp[8 * g + k]; c.len[k] = std::max(hp[8 * g + 3 + k] - hp[8 * g + k], 0.0) + 1e-9; }
            double ncd = std::floor(c.len[k] / r_cut);
            ncd = std::max(1.0, std::min(ncd, 1.0e6));
            c.nc[k] = (int32_t)ncd;
            ncell *= c.nc[k];
        }
        // Cap the cell count near the atom count (cells stay >= r_cut wide).
        while (ncell > 4 * na + 64) {
            int k = (c.nc[0] >= c.nc[1] && c.nc[0] >= c.nc[2]) ? 0 : (c.nc[1] >= c.nc[2] ? 1 : 2);
            ncell /= c.nc[k];
            c.nc[k] = std::max(1, c.nc[k] / 2);
            ncell *= c.nc[k];
        }
        c.strip = std::min<int32_t>(c.nc[0], kCellStrip);
        c.nstrip = (c.nc[0] + c.strip - 1) / c.strip;
        c.ncell = (int64_t)c.nc[2] * c.nstrip * c.nc[1] * c.strip;
        c.cell_off = off;
        off += c.ncell;
        TBK_CHECK(off < (int64_t)INT32_MAX, TBK_ERR_UNSUPPORTED, "too many cells");
    }
    const int64_t ncell = off;
    TBK_HIP(grids.alloc(sizeof(CellGrid) * nseg, s));
    TBK_HIP(hipMemcpyAsync(grids.as<CellGrid>(), hg.data(), sizeof(CellGrid) * nseg, hipMemcpyHostToDevice, s));

    DevBuf cell, slot, count;
    TBK_HIP(cell.alloc(sizeof(int32_t) * n, s));
    TBK_HIP(slot.alloc(sizeof(int32_t) * n, s));
    TBK_HIP(count.alloc(sizeof(int32_t) * (ncell + 1), s));
    TBK_HIP(cell_start.alloc(sizeof(int32_t) * (ncell + 1), s));
    TBK_HIP(sorted.alloc(sizeof(int32_t) * n, s));
    TBK_HIP(hipMemsetAsync(count.as<int32_t>(), 0, sizeof(int32_t) * (ncell + 1), s));
    const int gn = (int)ceil_div(n, kBlock);
    k_cell_of<<<gn, kBlock, 0, s>>>(pos, n, grids.as<CellGrid>(), seg_of.as<int32_t>(), cell.as<int32_t>(),
                                    slot.as<int32_t>(), count.as<int32_t>());
    TBK_HIP(hipGetLastError());
    tbk_status st = exclusive_scan(count.as<int32_t>(), cell_start.as<int32_t>(), ncell + 1, s);
    if (st != TBK_OK) return st;
    k_scatter<<<gn, kBlock, 0, s>>>(n, cell.as<int32_t>(), slot.as<int32_t>(), cell_start.as<int32_t>(),
                                    sorted.as<int32_t>());
    TBK_HIP(hipGetLastError());
    k_sort_cells<<<(int)ceil_div(ncell, kBlock), kBlock, 0, s>>>(ncell, cell_start.as<int32_t>(), sorted.as<int32_t>());
    TBK_HIP(hipGetLastError());
    view.grids = grids.as<CellGrid>();
    view.seg_of = seg_of.as<int32_t>();
    view.cell_start = cell_start.as<int32_t>();
    view.sorted = sorted.as<int32_t>();
    return TBK_OK;
}

tbk_status HamPlan::run(const double *pos, const int32_t *species, int64_t n, int32_t nseg, const int64_t *seg_atoms,
                        const double *boxes, const int32_t periodic[3], const tbk_tb_params *p, int32_t fmt,
                        int32_t slice_in, hipStream_t s) {
    tbk_status st = check_tb_params(p);
    if (st != TBK_OK) return st;
    TBK_CHECK(species != nullptr, TBK_ERR_INVALID_ARG, "species is NULL");
    TBK_CHECK(fmt == TBK_CSR_F64 || fmt == TBK_SELL_F64 || fmt == TBK_SELL_F32, TBK_ERR_INVALID_ARG,
              "unknown format %d", fmt);
    TBK_CHECK(p->reorder == 0 || p->reorder == 1, TBK_ERR_INVALID_ARG, "reorder must be 0 or 1");
    if (fmt == TBK_CSR_F64) slice = 1;
    else {
        TBK_CHECK(slice_in >= 1 && slice_in <= 1024 && (slice_in & (slice_in - 1)) == 0, TBK_ERR_INVALID_ARG,
                  "slice = %d is not a power of two in [1, 1024]", slice_in);
        slice = slice_in;
    }
    st = cells.build(pos, species, p->n_species, n, nseg, seg_atoms, boxes, periodic, p->r_cut, s);
    if (st != TBK_OK) return st;
    const int gn = (int)ceil_div(n, kBlock);
    TBK_HIP(perm.alloc(sizeof(int32_t) * n, s));
    TBK_HIP(iperm.alloc(sizeof(int32_t) * n, s));
    TBK_HIP(deg.alloc(sizeof(int32_t) * n, s));
    k_perm<<<gn, kBlock, 0, s>>>(n, p->reorder, cells.view.sorted, perm.as<int32_t>(), iperm.as<int32_t>());
    TBK_HIP(hipGetLastError());
    k_degree<<<gn, kBlock, 0, s>>>(cells.view, pos, n, p->r_cut, perm.as<int32_t>(), deg.as<int32_t>());
    TBK_HIP(hipGetLastError());
    n_slices = ceil_div(n, slice);
    DevBuf entries;
    TBK_HIP(entries.alloc(sizeof(int64_t) * (n_slices + 1), s));
    TBK_HIP(ptr.alloc(sizeof(int64_t) * (n_slices + 1), s));
    TBK_HIP(hipMemsetAsync(entries.as<int64_t>() + n_slices, 0, sizeof(int64_t), s));
    k_slice_width<<<(int)ceil_div(n_slices, kBlock), kBlock, 0, s>>>(n, slice, n_slices, deg.as<int32_t>(),
                                                                     entries.as<int64_t>());
    TBK_HIP(hipGetLastError());
    st = exclusive_scan(entries.as<int64_t>(), ptr.as<int64_t>(), n_slices + 1, s);
    if (st != TBK_OK) return st;
    // totals: max degree, degree sum, stored entries
    DevBuf red, t1, t2;
    TBK_HIP(red.alloc(sizeof(int64_t) * 2, s));
    int32_t *dmax = reinterpret_cast<int32_t *>(red.as<int64_t>());
    int64_t *dsum = red.as<int64_t>() + 1;
    size_t tmp = 0, tmp2 = 0;
    TBK_HIP(hipcub::DeviceReduce::Max(nullptr, tmp, deg.as<int32_t>(), dmax, (int)n, s));
    TBK_HIP(t1.alloc(tmp, s));
    TBK_HIP(hipcub::DeviceReduce::Max(t1.as<void>(), tmp, deg.as<int32_t>(), dmax, (int)n, s));
    TBK_HIP(hipcub::DeviceReduce::Sum(nullptr, tmp2, deg.as<int32_t>(), dsum, (int)n, s));
    TBK_HIP(t2.alloc(tmp2, s));
    TBK_HIP(hipcub::DeviceReduce::Sum(t2.as<void>(), tmp2, deg.as<int32_t>(), dsum, (int)n, s));
    int64_t host[2] = {0, 0};
    int64_t total = 0;
    TBK_HIP(hipMemcpyAsync(host, red.as<int64_t>(), sizeof(int64_t) * 2, hipMemcpyDeviceToHost, s));
    TBK_HIP(hipMemcpyAsync(&total, ptr.as<int64_t>() + n_slices, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    int32_t mxd;
    std::memcpy(&mxd, &host[0], sizeof(int32_t));
    max_degree = mxd;
    n_bonds = host[1] / 2;
    n_entries = total;
    TBK_CHECK(max_degree <= kMaxDegree, TBK_ERR_UNSUPPORTED, "max degree %d exceeds %d", max_degree, kMaxDegree);
    TBK_CHECK(n_entries < (int64_t)1 << 40, TBK_ERR_UNSUPPORTED, "too many entries");
    return TBK_OK;
}

tbk_status HamPlan::check_buffers(int64_t n, const tbk_ham *h) const {
    TBK_CHECK(h->n_rows >= n && h->n_ptr >= n_slices + 1 && h->n_entries >= n_entries,
              TBK_ERR_BUFFER_TOO_SMALL, "Hamiltonian buffers sized for n_rows=%lld n_ptr=%lld n_entries=%lld; "
              "need %lld, %lld, %lld", (long long)h->n_rows, (long long)h->n_ptr, (long long)h->n_entries,
              (long long)n, (long long)(n_slices + 1), (long long)n_entries);
    TBK_CHECK(h->ptr && h->col && h->val && h->onsite && h->perm, TBK_ERR_INVALID_ARG,
              "a Hamiltonian array pointer is NULL");
    return TBK_OK;
}

void HamPlan::set_sizes(int64_t n, const tbk_tb_params *p, tbk_ham *h) const {
    h->n_rows = n;
    h->n_ptr = n_slices + 1;
    h->n_entries = n_entries;
    h->n_bonds = n_bonds;
    h->max_degree = max_degree;
    h->has_onsite = any_onsite(p);
    h->n_seg = cells.n_seg;
    h->n_orb = 1;
    if (h->fmt == TBK_CSR_F64) h->slice = 1;
}

tbk_status HamPlan::fill(const double *pos, const int32_t *species, int64_t n, const tbk_tb_params *p, tbk_ham *h,
                         double *bounds, hipStream_t s) {
    tbk_status st = check_buffers(n, h);
    if (st != TBK_OK) return st;
    const int nseg = cells.n_seg;
    SpeciesTable tab{};
    for (int i = 0; i < p->n_species; ++i) {
        tab.onsite[i] = p->onsite[i];
        for (int j = 0; j < p->n_species; ++j) tab.t_pair[i * p->n_species + j] = p->t_pair[i * p->n_species + j];
    }
    DevBuf dtab, keys;
    TBK_HIP(dtab.alloc(sizeof(SpeciesTable), s));
    st = init_bound_keys(vkeys, 1, s);
    if (st != TBK_OK) return st;
    TBK_HIP(hipMemcpyAsync(dtab.as<void>(), &tab, sizeof(SpeciesTable), hipMemcpyHostToDevice, s));
    st = init_bound_keys(keys, nseg, s);
    if (st != TBK_OK) return st;
    const int gn = (int)ceil_div(n, kBlock);
    TBK_HIP(hipMemcpyAsync(h->ptr, ptr.as<int64_t>(), sizeof(int64_t) * (n_slices + 1), hipMemcpyDeviceToDevice, s));
    TBK_HIP(hipMemcpyAsync(h->perm, perm.as<int32_t>(), sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    if (h->fmt == TBK_SELL_F32) {
        k_fill<float><<<gn, kBlock, 0, s>>>(cells.view, pos, species, n, slice, p->r_cut, p->r0, p->beta,
                                            p->n_species, dtab.as<SpeciesTable>(), perm.as<int32_t>(),
                                            iperm.as<int32_t>(), h->ptr, h->col, static_cast<float *>(h->val),
                                            static_cast<float *>(h->onsite), keys.as<int64_t>(),
                                            vkeys.as<int64_t>(), h->col16);
    } else {
        k_fill<double><<<gn, kBlock, 0, s>>>(cells.view, pos, species, n, slice, p->r_cut, p->r0, p->beta,
                                             p->n_species, dtab.as<SpeciesTable>(), perm.as<int32_t>(),
                                             iperm.as<int32_t>(), h->ptr, h->col, static_cast<double *>(h->val),
                                             static_cast<double *>(h->onsite), keys.as<int64_t>(),
                                             vkeys.as<int64_t>(), h->col16);
    }
    TBK_HIP(hipGetLastError());
    return finish(keys, n, p, h, bounds, s);
}

tbk_status HamPlan::finish(DevBuf &keys, int64_t n, const tbk_tb_params *p, tbk_ham *h, double *bounds,
                           hipStream_t s) {
    const int nseg = cells.n_seg;
    std::vector<int64_t> hk(2 * (size_t)nseg);
    int64_t vk[2] = {0, 0};
    TBK_HIP(hipMemcpyAsync(hk.data(), keys.as<int64_t>(), sizeof(int64_t) * 2 * nseg, hipMemcpyDeviceToHost, s));
    if (vkeys.as<int64_t>())
        TBK_HIP(hipMemcpyAsync(vk, vkeys.as<int64_t>(), sizeof vk, hipMemcpyDeviceToHost, s));
    if (h->seg_rows)
        TBK_HIP(hipMemcpyAsync(h->seg_rows, cells.seg_atoms.as<int64_t>(), sizeof(int64_t) * (nseg + 1),
                               hipMemcpyDeviceToDevice, s));
    TBK_HIP(hipStreamSynchronize(s));
    decode_bounds(hk, nseg, bounds);
    set_sizes(n, p, h);
    // uniform hoppings: every stored value (as stored) equal, at least one entry
    h->uniform_hop = 0;
    h->hop_value = 0.0;
    if (vkeys.as<int64_t>() && vk[0] == vk[1] && dunkey(vk[0]) <= dunkey(vk[1])) {
        h->uniform_hop = 1;
        h->hop_value = dunkey(vk[0]);
    }
    return TBK_OK;
}

}  // namespace tbk

using namespace tbk;

namespace {

tbk_status size_common(const double *pos, const int32_t *species, int64_t n, int32_t nseg, const int64_t *seg_atoms,
                       const double *boxes, const int32_t periodic[3], const tbk_tb_params *p, tbk_ham *h,
                       void *stream) {
    TBK_CHECK(h != nullptr, TBK_ERR_INVALID_ARG, "h is NULL");
    hipStream_t s = as_stream(stream);
    HamPlan plan;
    tbk_status st = plan.run(pos, species, n, nseg, seg_atoms, boxes, periodic, p, h->fmt, h->slice, s);
    if (st != TBK_OK) return st;
    plan.set_sizes(n, p, h);
    return TBK_OK;
}

tbk_status build_common(const double *pos, const int32_t *species, int64_t n, int32_t nseg, const int64_t *seg_atoms,
                        const double *boxes, const int32_t periodic[3], const tbk_tb_params *p, tbk_ham *h,
                        double *bounds, void *stream) {
    TBK_CHECK(h != nullptr && bounds != nullptr, TBK_ERR_INVALID_ARG, "h or bounds is NULL");
    hipStream_t s = as_stream(stream);
    HamPlan plan;
    tbk_status st = plan.run(pos, species, n, nseg, seg_atoms, boxes, periodic, p, h->fmt, h->slice, s);
    if (st != TBK_OK) return st;
    return plan.fill(pos, species, n, p, h, bounds, s);
}

}  // namespace

extern "C" tbk_status tbk_hamiltonian_size(const double *pos, const int32_t *species, int64_t n,
                                           const double box[3], const int32_t periodic[3],
                                           const tbk_tb_params *p, tbk_ham *h, void *stream) {
    clear_error();
    TBK_CHECK(box != nullptr, TBK_ERR_INVALID_ARG, "box is NULL");
    const int64_t seg[2] = {0, n};
    return size_common(pos, species, n, 1, seg, box, periodic, p, h, stream);
}

extern "C" tbk_status tb_build_hamiltonian(const double *pos, const int32_t *species, int64_t n,
                                           const double box[3], const int32_t periodic[3],
                                           const tbk_tb_params *p, tbk_ham *h, double spec_bounds[2],
                                           void *stream) {
    clear_error();
    TBK_CHECK(box != nullptr, TBK_ERR_INVALID_ARG, "box is NULL");
    const int64_t seg[2] = {0, n};
    if (h) h->seg_rows = nullptr;
    return build_common(pos, species, n, 1, seg, box, periodic, p, h, spec_bounds, stream);
}

extern "C" tbk_status tbk_hamiltonian_size_batched(const double *pos, const int32_t *species, int32_t n_seg,
                                                   const int64_t *seg_atoms, const double *boxes,
                                                   const int32_t periodic[3], const tbk_tb_params *p, tbk_ham *h,
                                                   void *stream) {
    clear_error();
    TBK_CHECK(seg_atoms != nullptr && n_seg >= 1, TBK_ERR_INVALID_ARG, "bad segment table");
    return size_common(pos, species, seg_atoms[n_seg], n_seg, seg_atoms, boxes, periodic, p, h, stream);
}

extern "C" tbk_status tb_build_hamiltonian_batched(const double *pos, const int32_t *species, int32_t n_seg,
                                                   const int64_t *seg_atoms, const double *boxes,
                                                   const int32_t periodic[3], const tbk_tb_params *p, tbk_ham *h,
                                                   double *spec_bounds, void *stream) {
    clear_error();
    TBK_CHECK(seg_atoms != nullptr && n_seg >= 1, TBK_ERR_INVALID_ARG, "bad segment table");
    TBK_CHECK(h != nullptr && h->seg_rows != nullptr, TBK_ERR_INVALID_ARG, "h->seg_rows must hold n_seg+1 entries");
    return build_common(pos, species, seg_atoms[n_seg], n_seg, seg_atoms, boxes, periodic, p, h, spec_bounds, stream);
}
