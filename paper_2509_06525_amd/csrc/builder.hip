// Neighbour list and Hamiltonian assembly on the GPU (Eq. (1)).
//
// Build sequence for one structure:
//   1. k_scan_positions: per-axis range, NaN/Inf and species checks (block partials)
//   2. cell list: cell id per atom, counts, exclusive scan, scatter, per-cell sort
//   3. k_degree: neighbours within r_cut per row
//   4. slice widths (max degree per slice) -> slice offsets (exclusive scan)
//   5. k_fill: columns and FP64 hoppings of each row, padding, in-row sort by
//      column, onsite, row Gershgorin bounds (block partials)
// CSR is handled as SELL with slice height 1.
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstring>
#include <vector>

#include "nlist.hpp"

namespace tbk {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxDegree = 256;
constexpr int kMaxSpecies = 16;
constexpr int kCellStrip = 64;      // cells per strip of the row order

__global__ void k_scan_positions(const double *__restrict__ pos, const int32_t *__restrict__ species,
                                 int64_t n, int32_t n_species, double *__restrict__ part) {
    // part[block][8] = {min x, min y, min z, max x, max y, max z, bad coord, bad species}
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    double bad = 0.0, bad_sp = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < 3; ++k) {
            double x = pos[3 * i + k];
            if (!isfinite(x)) bad = 1.0;
            else { mn[k] = fmin(mn[k], x); mx[k] = fmax(mx[k], x); }
        }
        if (species) {
            int32_t s = species[i];
            if (s < 0 || s >= n_species) bad_sp = 1.0;
        }
    }
    __shared__ double red[8][kBlock];
    for (int k = 0; k < 3; ++k) { red[k][threadIdx.x] = mn[k]; red[3 + k][threadIdx.x] = mx[k]; }
    red[6][threadIdx.x] = bad;
    red[7][threadIdx.x] = bad_sp;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < 3; ++k)
                red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
            for (int k = 3; k < 8; ++k)
                red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) part[blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_cell_of(const double *__restrict__ pos, int64_t n, CellGrid g,
                          int32_t *__restrict__ cell, int32_t *__restrict__ slot,
                          int32_t *__restrict__ count) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t cx = cell_coord(pos[3 * i], g, 0);
    int32_t cy = cell_coord(pos[3 * i + 1], g, 1);
    int32_t cz = cell_coord(pos[3 * i + 2], g, 2);
    int32_t c = (int32_t)cell_id(g, cx, cy, cz);
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
                              int64_t *__restrict__ entries, int32_t *__restrict__ width) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    int32_t w = 0;
    int64_t r1 = (s + 1) * slice < n ? (s + 1) * slice : n;
    for (int64_t r = s * slice; r < r1; ++r) w = deg[r] > w ? deg[r] : w;
    width[s] = w;
    entries[s] = (int64_t)w * slice;
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
                       double *__restrict__ gersh) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (r < n) {
        const int64_t s = r / slice, lane = r - s * slice;
        const int64_t base = ptr[s] + lane;
        const int32_t w = (int32_t)((ptr[s + 1] - ptr[s]) / slice);
        const int32_t i = perm[r];
        const int32_t si = species[i];
        int32_t k = 0;
        double asum = 0.0;
        for_each_neighbor(cl, pos, i, r_cut, [&](int32_t j, double rij, double, double, double) {
            double t = tab->t_pair[si * n_species + species[j]] * exp(-beta * (rij / r0 - 1.0));
            if (k < w) {
                col[base + (int64_t)k * slice] = iperm[j];
                val[base + (int64_t)k * slice] = (V)t;
            }
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
        double eps = tab->onsite[si];
        onsite[r] = (V)eps;
        lo = eps - asum;
        hi = eps + asum;
    }
    __shared__ double red[2][kBlock];
    red[0][threadIdx.x] = lo;
    red[1][threadIdx.x] = hi;
    __syncthreads();
    for (int w2 = kBlock / 2; w2 > 0; w2 >>= 1) {
        if ((int)threadIdx.x < w2) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + w2]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w2]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { gersh[2 * blockIdx.x] = red[0][0]; gersh[2 * blockIdx.x + 1] = red[1][0]; }
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

tbk_status check_params(const tbk_tb_params *p) {
    TBK_CHECK(p != nullptr, TBK_ERR_INVALID_ARG, "params is NULL");
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

int32_t any_onsite(const tbk_tb_params *p) {
    for (int i = 0; i < p->n_species; ++i)
        if (p->onsite[i] != 0.0) return 1;
    return 0;
}

}  // namespace

tbk_status CellListOwner::build(const double *pos, const int32_t *species, int32_t n_species, int64_t n,
                                const double box[3], const int32_t periodic[3], double r_cut, hipStream_t s) {
    TBK_CHECK(pos && box && periodic, TBK_ERR_INVALID_ARG, "NULL position/box/periodic");
    TBK_CHECK(n >= 1 && n < (int64_t)INT32_MAX, TBK_ERR_INVALID_ARG, "n = %lld out of [1, 2^31-1)", (long long)n);
    for (int k = 0; k < 3; ++k) {
        TBK_CHECK(periodic[k] == 0 || periodic[k] == 1, TBK_ERR_INVALID_ARG, "periodic[%d] must be 0 or 1", k);
        if (periodic[k]) {
            TBK_CHECK(std::isfinite(box[k]), TBK_ERR_NOT_FINITE, "box[%d] is not finite", k);
            TBK_CHECK(box[k] >= 2.0 * r_cut, TBK_ERR_INVALID_ARG,
                      "periodic length box[%d] = %g is below 2 r_cut = %g", k, box[k], 2.0 * r_cut);
        }
    }
    // 1. ranges and validity
    const int nblk = (int)std::min<int64_t>(ceil_div(n, kBlock), 1024);
    DevBuf part;
    TBK_HIP(part.alloc(sizeof(double) * 8 * nblk, s));
    k_scan_positions<<<nblk, kBlock, 0, s>>>(pos, species, n, n_species, part.as<double>());
    TBK_HIP(hipGetLastError());
    std::vector<double> hp(8 * nblk);
    TBK_HIP(hipMemcpyAsync(hp.data(), part.as<double>(), sizeof(double) * 8 * nblk, hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    double bad = 0, bad_sp = 0;
    for (int b = 0; b < nblk; ++b) {
        for (int k = 0; k < 3; ++k) { mn[k] = std::min(mn[k], hp[8 * b + k]); mx[k] = std::max(mx[k], hp[8 * b + 3 + k]); }
        bad = std::max(bad, hp[8 * b + 6]);
        bad_sp = std::max(bad_sp, hp[8 * b + 7]);
    }
    TBK_CHECK(bad == 0.0, TBK_ERR_NOT_FINITE, "a coordinate is NaN or Inf");
    TBK_CHECK(bad_sp == 0.0, TBK_ERR_INVALID_ARG, "a species index is outside [0, %d)", n_species);

    // 2. cell grid
    CellGrid &g = view.g;
    int64_t ncell = 1;
    for (int k = 0; k < 3; ++k) {
        g.periodic[k] = periodic[k];
        g.box[k] = periodic[k] ? box[k] : 0.0;
        if (periodic[k]) { g.lo[k] = 0.0; g.len[k] = box[k]; }
        else { g.lo[k] = mn[k]; g.len[k] = std::max(mx[k] - mn[k], 0.0) + 1e-9; }
        double ncd = std::floor(g.len[k] / r_cut);
        ncd = std::max(1.0, std::min(ncd, 1.0e6));
        g.nc[k] = (int32_t)ncd;
        ncell *= g.nc[k];
    }
    // Cap the cell count near the atom count (cells stay >= r_cut wide).
    while (ncell > 4 * n + 64) {
        int k = (g.nc[0] >= g.nc[1] && g.nc[0] >= g.nc[2]) ? 0 : (g.nc[1] >= g.nc[2] ? 1 : 2);
        ncell /= g.nc[k];
        g.nc[k] = std::max(1, g.nc[k] / 2);
        ncell *= g.nc[k];
    }
    g.strip = std::min<int32_t>(g.nc[0], kCellStrip);
    g.nstrip = (g.nc[0] + g.strip - 1) / g.strip;
    ncell = (int64_t)g.nc[2] * g.nstrip * g.nc[1] * g.strip;
    g.ncell = ncell;
    TBK_CHECK(ncell < (int64_t)INT32_MAX, TBK_ERR_UNSUPPORTED, "too many cells");

    DevBuf cell, slot, count;
    TBK_HIP(cell.alloc(sizeof(int32_t) * n, s));
    TBK_HIP(slot.alloc(sizeof(int32_t) * n, s));
    TBK_HIP(count.alloc(sizeof(int32_t) * (ncell + 1), s));
    TBK_HIP(cell_start.alloc(sizeof(int32_t) * (ncell + 1), s));
    TBK_HIP(sorted.alloc(sizeof(int32_t) * n, s));
    TBK_HIP(hipMemsetAsync(count.as<int32_t>(), 0, sizeof(int32_t) * (ncell + 1), s));
    const int gn = (int)ceil_div(n, kBlock);
    k_cell_of<<<gn, kBlock, 0, s>>>(pos, n, g, cell.as<int32_t>(), slot.as<int32_t>(), count.as<int32_t>());
    TBK_HIP(hipGetLastError());
    tbk_status st = exclusive_scan(count.as<int32_t>(), cell_start.as<int32_t>(), ncell + 1, s);
    if (st != TBK_OK) return st;
    k_scatter<<<gn, kBlock, 0, s>>>(n, cell.as<int32_t>(), slot.as<int32_t>(), cell_start.as<int32_t>(),
                                    sorted.as<int32_t>());
    TBK_HIP(hipGetLastError());
    k_sort_cells<<<(int)ceil_div(ncell, kBlock), kBlock, 0, s>>>(ncell, cell_start.as<int32_t>(), sorted.as<int32_t>());
    TBK_HIP(hipGetLastError());
    view.cell_start = cell_start.as<int32_t>();
    view.sorted = sorted.as<int32_t>();
    return TBK_OK;
}

// Shared front half of the size query and the build: cell list, permutation,
// degrees, slice widths and offsets.
struct HamPlan {
    CellListOwner cells;
    DevBuf perm, iperm, deg, width, entries, ptr;
    int64_t n_slices = 0, n_entries = 0, n_bonds = 0;
    int32_t max_degree = 0;
    int32_t slice = 1;

    tbk_status run(const double *pos, const int32_t *species, int64_t n, const double box[3],
                   const int32_t periodic[3], const tbk_tb_params *p, int32_t fmt, int32_t slice_in,
                   hipStream_t s) {
        tbk_status st = check_params(p);
        if (st != TBK_OK) return st;
        TBK_CHECK(species != nullptr, TBK_ERR_INVALID_ARG, "species is NULL");
        TBK_CHECK(fmt == TBK_CSR_F64 || fmt == TBK_SELL_F64 || fmt == TBK_SELL_F32, TBK_ERR_INVALID_ARG,
                  "unknown format %d", fmt);
        TBK_CHECK(p->reorder == 0 || p->reorder == 1, TBK_ERR_INVALID_ARG, "reorder must be 0 or 1");
        if (fmt == TBK_CSR_F64) slice = 1;
        else {
            TBK_CHECK(slice_in >= 1 && slice_in <= 1024 && (slice_in & (slice_in - 1)) == 0,
                      TBK_ERR_INVALID_ARG, "slice = %d is not a power of two in [1, 1024]", slice_in);
            slice = slice_in;
        }
        st = cells.build(pos, species, p->n_species, n, box, periodic, p->r_cut, s);
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
        TBK_HIP(width.alloc(sizeof(int32_t) * n_slices, s));
        TBK_HIP(entries.alloc(sizeof(int64_t) * (n_slices + 1), s));
        TBK_HIP(ptr.alloc(sizeof(int64_t) * (n_slices + 1), s));
        TBK_HIP(hipMemsetAsync(entries.as<int64_t>() + n_slices, 0, sizeof(int64_t), s));
        k_slice_width<<<(int)ceil_div(n_slices, kBlock), kBlock, 0, s>>>(n, slice, n_slices, deg.as<int32_t>(),
                                                                         entries.as<int64_t>(), width.as<int32_t>());
        TBK_HIP(hipGetLastError());
        st = exclusive_scan(entries.as<int64_t>(), ptr.as<int64_t>(), n_slices + 1, s);
        if (st != TBK_OK) return st;
        // totals: entries, max degree, degree sum
        int32_t *dmax = nullptr;
        size_t tmp = 0;
        DevBuf red, t;
        TBK_HIP(red.alloc(sizeof(int64_t) * 2, s));
        TBK_HIP(hipcub::DeviceReduce::Max(nullptr, tmp, deg.as<int32_t>(), red.as<int32_t>(), (int)n, s));
        TBK_HIP(t.alloc(tmp, s));
        TBK_HIP(hipcub::DeviceReduce::Max(t.as<void>(), tmp, deg.as<int32_t>(), red.as<int32_t>(), (int)n, s));
        size_t tmp2 = 0;
        int64_t *dsum = red.as<int64_t>() + 1;
        TBK_HIP(hipcub::DeviceReduce::Sum(nullptr, tmp2, deg.as<int32_t>(), dsum, (int)n, s));
        DevBuf t2;
        TBK_HIP(t2.alloc(tmp2, s));
        TBK_HIP(hipcub::DeviceReduce::Sum(t2.as<void>(), tmp2, deg.as<int32_t>(), dsum, (int)n, s));
        (void)dmax;
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
};

}  // namespace tbk

using namespace tbk;

extern "C" tbk_status tbk_hamiltonian_size(const double *pos, const int32_t *species, int64_t n,
                                           const double box[3], const int32_t periodic[3],
                                           const tbk_tb_params *p, tbk_ham *h, void *stream) {
    clear_error();
    TBK_CHECK(h != nullptr, TBK_ERR_INVALID_ARG, "h is NULL");
    hipStream_t s = as_stream(stream);
    HamPlan plan;
    tbk_status st = plan.run(pos, species, n, box, periodic, p, h->fmt, h->slice, s);
    if (st != TBK_OK) return st;
    h->n_rows = n;
    h->n_ptr = plan.n_slices + 1;
    h->n_entries = plan.n_entries;
    h->n_bonds = plan.n_bonds;
    h->max_degree = plan.max_degree;
    h->has_onsite = any_onsite(p);
    h->n_seg = 1;
    if (h->fmt == TBK_CSR_F64) h->slice = 1;
    TBK_HIP(hipStreamSynchronize(s));
    return TBK_OK;
}

extern "C" tbk_status tb_build_hamiltonian(const double *pos, const int32_t *species, int64_t n,
                                           const double box[3], const int32_t periodic[3],
                                           const tbk_tb_params *p, tbk_ham *h, double spec_bounds[2],
                                           void *stream) {
    clear_error();
    TBK_CHECK(h != nullptr && spec_bounds != nullptr, TBK_ERR_INVALID_ARG, "h or spec_bounds is NULL");
    hipStream_t s = as_stream(stream);
    HamPlan plan;
    tbk_status st = plan.run(pos, species, n, box, periodic, p, h->fmt, h->slice, s);
    if (st != TBK_OK) return st;
    TBK_CHECK(h->n_rows >= n && h->n_ptr >= plan.n_slices + 1 && h->n_entries >= plan.n_entries,
              TBK_ERR_BUFFER_TOO_SMALL, "Hamiltonian buffers sized for n_rows=%lld n_ptr=%lld n_entries=%lld; "
              "need %lld, %lld, %lld", (long long)h->n_rows, (long long)h->n_ptr, (long long)h->n_entries,
              (long long)n, (long long)(plan.n_slices + 1), (long long)plan.n_entries);
    TBK_CHECK(h->ptr && h->col && h->val && h->onsite && h->perm, TBK_ERR_INVALID_ARG,
              "a Hamiltonian array pointer is NULL");

    SpeciesTable tab{};
    for (int i = 0; i < p->n_species; ++i) {
        tab.onsite[i] = p->onsite[i];
        for (int j = 0; j < p->n_species; ++j) tab.t_pair[i * p->n_species + j] = p->t_pair[i * p->n_species + j];
    }
    DevBuf dtab;
    TBK_HIP(dtab.alloc(sizeof(SpeciesTable), s));
    TBK_HIP(hipMemcpyAsync(dtab.as<void>(), &tab, sizeof(SpeciesTable), hipMemcpyHostToDevice, s));

    const int gn = (int)ceil_div(n, kBlock);
    DevBuf gersh;
    TBK_HIP(gersh.alloc(sizeof(double) * 2 * gn, s));
    TBK_HIP(hipMemcpyAsync(h->ptr, plan.ptr.as<int64_t>(), sizeof(int64_t) * (plan.n_slices + 1),
                           hipMemcpyDeviceToDevice, s));
    TBK_HIP(hipMemcpyAsync(h->perm, plan.perm.as<int32_t>(), sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    if (h->fmt == TBK_SELL_F32) {
        k_fill<float><<<gn, kBlock, 0, s>>>(plan.cells.view, pos, species, n, plan.slice, p->r_cut, p->r0, p->beta,
                                            p->n_species, dtab.as<SpeciesTable>(), plan.perm.as<int32_t>(),
                                            plan.iperm.as<int32_t>(), h->ptr, h->col,
                                            static_cast<float *>(h->val), static_cast<float *>(h->onsite),
                                            gersh.as<double>());
    } else {
        k_fill<double><<<gn, kBlock, 0, s>>>(plan.cells.view, pos, species, n, plan.slice, p->r_cut, p->r0, p->beta,
                                             p->n_species, dtab.as<SpeciesTable>(), plan.perm.as<int32_t>(),
                                             plan.iperm.as<int32_t>(), h->ptr, h->col,
                                             static_cast<double *>(h->val), static_cast<double *>(h->onsite),
                                             gersh.as<double>());
    }
    TBK_HIP(hipGetLastError());
    std::vector<double> hg(2 * gn);
    TBK_HIP(hipMemcpyAsync(hg.data(), gersh.as<double>(), sizeof(double) * 2 * gn, hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    double lo = INFINITY, hi = -INFINITY;
    for (int b = 0; b < gn; ++b) { lo = std::min(lo, hg[2 * b]); hi = std::max(hi, hg[2 * b + 1]); }
    spec_bounds[0] = lo;
    spec_bounds[1] = hi;
    h->n_rows = n;
    h->n_ptr = plan.n_slices + 1;
    h->n_entries = plan.n_entries;
    h->n_bonds = plan.n_bonds;
    h->max_degree = plan.max_degree;
    h->has_onsite = any_onsite(p);
    h->n_seg = 1;
    h->seg_rows = nullptr;
    return TBK_OK;
}
