// Device helpers of the recurrence kernels (internal).
#pragma once

#include "common.hpp"

namespace tbk {

constexpr int kThreads = 256;

typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

template <bool NT, class T>
__device__ __forceinline__ T ld(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT, class T>
__device__ __forceinline__ void st(T *p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// VPT consecutive complex values of one row.
template <class VT, int VPT> struct Pack {
    VT re[VPT], im[VPT];
};

template <bool NT, class VT, int VPT>
__device__ __forceinline__ Pack<VT, VPT> load_pack(const VT *p) {
    Pack<VT, VPT> o;
    if constexpr (sizeof(VT) == 4 && VPT == 2) {
        f4v v = ld<NT>(reinterpret_cast<const f4v *>(p));
        o.re[0] = v.x; o.im[0] = v.y; o.re[1] = v.z; o.im[1] = v.w;
    } else if constexpr (sizeof(VT) == 4 && VPT == 1) {
        f2v v = ld<NT>(reinterpret_cast<const f2v *>(p));
        o.re[0] = v.x; o.im[0] = v.y;
    } else {
        static_assert(VPT == 1, "double packs hold one complex value");
        d2v v = ld<NT>(reinterpret_cast<const d2v *>(p));
        o.re[0] = v.x; o.im[0] = v.y;
    }
    return o;
}

template <bool NT, class VT, int VPT>
__device__ __forceinline__ void store_pack(VT *p, const Pack<VT, VPT> &o) {
    if constexpr (sizeof(VT) == 4 && VPT == 2) {
        f4v v = {o.re[0], o.im[0], o.re[1], o.im[1]};
        st<NT>(reinterpret_cast<f4v *>(p), v);
    } else if constexpr (sizeof(VT) == 4 && VPT == 1) {
        f2v v = {o.re[0], o.im[0]};
        st<NT>(reinterpret_cast<f2v *>(p), v);
    } else {
        d2v v = {o.re[0], o.im[0]};
        st<NT>(reinterpret_cast<d2v *>(p), v);
    }
}

// Block order over the XCDs (workgroup b runs on XCD b % 8).  Mode 0: dispatch
// order.  Mode 1: XCD x sweeps the contiguous eighth [x G/8, (x+1) G/8) of the
// blocks.  Modes 2 and 3: XCD x takes runs of xcd_run(mode) consecutive blocks
// and the 8 XCDs' runs lie side by side, so each XCD's neighbour rows stay in its
// own L2 while the chip as a whole still sweeps one front (one region of HBM and
// of the memory-side cache at a time).  The grid is a multiple of
// xcd_grid_multiple(mode); blocks past the last tile own none.
__host__ __device__ constexpr int64_t xcd_run(int mode) { return mode == 2 ? 16 : (mode == 3 ? 64 : 1); }
__host__ __device__ constexpr int64_t xcd_grid_multiple(int mode) {
    return mode == 0 ? 1 : (mode == 1 ? kNumXcd : kNumXcd * xcd_run(mode));
}

__device__ __forceinline__ int64_t logical_block(int xcd_remap) {
    const int64_t b = blockIdx.x, G = gridDim.x;
    if (xcd_remap == 1 && (G % kNumXcd) == 0) return (b % kNumXcd) * (G / kNumXcd) + b / kNumXcd;
    if (xcd_remap >= 2) {
        const int64_t C = xcd_run(xcd_remap);
        if (G % (kNumXcd * C) == 0) {
            const int64_t x = b % kNumXcd, j = b / kNumXcd;
            return (j / C) * (kNumXcd * C) + x * C + j % C;
        }
    }
    return b;
}

// Block reduction of acc[VPT] over rows sharing a vector slot; writes
// partial[lb][slot * VPT + q].
template <int L, int VPT>
__device__ __forceinline__ void block_reduce_store(double (&acc)[VPT], double *partial, int64_t lb) {
    __shared__ double red[kThreads / 64][64 * VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
#pragma unroll
        for (int off = L; off < 64; off <<= 1) acc[q] += __shfl_xor(acc[q], off);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < L) {
#pragma unroll
        for (int q = 0; q < VPT; ++q) red[wave][lane * VPT + q] = acc[q];
    }
    __syncthreads();
    if ((int)threadIdx.x < L * VPT) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) s += red[w][threadIdx.x];
        partial[lb * (L * VPT) + threadIdx.x] = s;
    }
}

// Counter-based random phase exp(i phi) of output k of SplitMix64 started at
// `seed` (Steele, Lea & Flood 2014): phi = 2 pi (x >> 11) 2^-53.
__device__ __forceinline__ void seeded_phase(uint64_t seed, uint64_t k, double &c, double &s) {
    uint64_t z = seed + (k + 1u) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    const double phi = 6.283185307179586 * ((double)(z >> 11) * 0x1p-53);
    sincos(phi, &s, &c);
}

}  // namespace tbk
