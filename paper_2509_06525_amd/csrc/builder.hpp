// Internal plan of the Hamiltonian builder (shared by the plain, batched and
// learned assembly entry points).
#pragma once

#include <cstring>
#include <vector>

#include "common.hpp"
#include "nlist.hpp"

namespace tbk {

constexpr int kBlock = 256;

// Order-preserving map of doubles to signed 64-bit integers (for atomic min/max).
__host__ __device__ __forceinline__ int64_t dkey(double x) {
    int64_t b;
    std::memcpy(&b, &x, sizeof b);
    return b >= 0 ? b : (b ^ INT64_MAX);
}
__host__ __device__ __forceinline__ double dunkey(int64_t k) {
    int64_t b = k >= 0 ? k : (k ^ INT64_MAX);
    double x;
    std::memcpy(&x, &b, sizeof x);
    return x;
}

// Per-segment block reduction of row bounds [lo, hi] (sg = segment of the
// thread's row, -1 for none), then one atomic min and max per segment the
// block touches.  Every thread of the block must call it.
static __device__ __forceinline__ void block_segment_bounds(double lo, double hi, int32_t sg,
                                                            int64_t *bound_keys) {
    __shared__ int32_t sgr[2];
    __shared__ double red[2][kBlock];
    if (threadIdx.x == 0) { sgr[0] = INT32_MAX; sgr[1] = -1; }
    __syncthreads();
    if (sg >= 0) { atomicMin(&sgr[0], sg); atomicMax(&sgr[1], sg); }
    __syncthreads();
    const int32_t s0 = sgr[0], s1 = sgr[1];
    for (int32_t q = s0; q <= s1; ++q) {
        red[0][threadIdx.x] = (sg == q) ? lo : INFINITY;
        red[1][threadIdx.x] = (sg == q) ? hi : -INFINITY;
        __syncthreads();
        for (int w2 = kBlock / 2; w2 > 0; w2 >>= 1) {
            if ((int)threadIdx.x < w2) {
                red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + w2]);
                red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w2]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0 && red[0][0] <= red[1][0]) {
            atomicMin((long long *)&bound_keys[2 * q], (long long)dkey(red[0][0]));
            atomicMax((long long *)&bound_keys[2 * q + 1], (long long)dkey(red[1][0]));
        }
        __syncthreads();
    }
}

tbk_status check_tb_params(const tbk_tb_params *p);
void decode_bounds(const std::vector<int64_t> &keys, int nseg, double *bounds);
tbk_status init_bound_keys(DevBuf &keys, int nseg, hipStream_t s);

struct HamPlan {
    CellListOwner cells;
    DevBuf perm, iperm, deg, ptr;
    DevBuf vkeys;    // range of the stored hoppings (plain assembly only)
    int64_t n_slices = 0, n_entries = 0, n_bonds = 0;
    int32_t max_degree = 0;
    int32_t slice = 1;

    // Cell list, row order, degrees, slice offsets and totals.
    tbk_status run(const double *pos, const int32_t *species, int64_t n, int32_t nseg, const int64_t *seg_atoms,
                   const double *boxes, const int32_t periodic[3], const tbk_tb_params *p, int32_t fmt,
                   int32_t slice_in, hipStream_t s);
    // Columns, distance-formula values, onsite, per-segment Gershgorin bounds
    // (bounds: host [n_seg][2]); fills the size fields of h.
    tbk_status fill(const double *pos, const int32_t *species, int64_t n, const tbk_tb_params *p, tbk_ham *h,
                    double *bounds, hipStream_t s);
    tbk_status check_buffers(int64_t n, const tbk_ham *h) const;
    void set_sizes(int64_t n, const tbk_tb_params *p, tbk_ham *h) const;
    // Reads the bound keys back, copies the segment table, sets h's sizes.
    tbk_status finish(DevBuf &keys, int64_t n, const tbk_tb_params *p, tbk_ham *h, double *bounds, hipStream_t s);
};

}  // namespace tbk
