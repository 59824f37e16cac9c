// Chebyshev recurrence with fused moment accumulation (KPM, Sec. 2.4).
//
// One launch per recurrence step: every thread owns one row and VPT of the R
// vectors (L = R / VPT threads per row), gathers T_n over the row's stored
// entries, writes T_{n+1} = c1 (H - b) T_n - c0 T_{n-1} over T_{n-1} in place,
// and accumulates Re(conj(r) T_{n+1}) in double.  A block reduces its rows by
// wavefront shuffles and LDS and writes one partial per vector; a final kernel
// sums the partials in a fixed order (bitwise reproducible, no atomics).
//
// Tiles of 256 / L rows are mapped XCD-aware: workgroup b runs on XCD b % 8,
// XCD x owns the x-th contiguous eighth of the tiles, and its workgroups sweep
// that range round-robin so neighbouring rows are gathered from one L2.
#include <cmath>

#include "common.hpp"

namespace tbk {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxGrid = 2048;

template <class VT> struct C2;
template <> struct C2<float> { using T = float2; };
template <> struct C2<double> { using T = double2; };

// VPT consecutive complex values of one row.
template <class VT, int VPT> struct Pack {
    VT re[VPT], im[VPT];
};

template <class VT, int VPT>
__device__ __forceinline__ Pack<VT, VPT> load_pack(const VT *p) {
    Pack<VT, VPT> o;
    if constexpr (sizeof(VT) == 4 && VPT == 2) {
        float4 v = *reinterpret_cast<const float4 *>(p);
        o.re[0] = v.x; o.im[0] = v.y; o.re[1] = v.z; o.im[1] = v.w;
    } else if constexpr (sizeof(VT) == 4 && VPT == 1) {
        float2 v = *reinterpret_cast<const float2 *>(p);
        o.re[0] = v.x; o.im[0] = v.y;
    } else {
        static_assert(VPT == 1, "double packs hold one complex value");
        double2 v = *reinterpret_cast<const double2 *>(p);
        o.re[0] = v.x; o.im[0] = v.y;
    }
    return o;
}

template <class VT, int VPT>
__device__ __forceinline__ void store_pack(VT *p, const Pack<VT, VPT> &o) {
    if constexpr (sizeof(VT) == 4 && VPT == 2) {
        *reinterpret_cast<float4 *>(p) = make_float4(o.re[0], o.im[0], o.re[1], o.im[1]);
    } else if constexpr (sizeof(VT) == 4 && VPT == 1) {
        *reinterpret_cast<float2 *>(p) = make_float2(o.re[0], o.im[0]);
    } else {
        *reinterpret_cast<double2 *>(p) = make_double2(o.re[0], o.im[0]);
    }
}

template <class VT> struct StepArgs {
    const int64_t *ptr;      // slice offsets (slice height 1 = CSR)
    const int32_t *col;
    const VT *val;
    const VT *onsite;        // used when diag != 0
    int64_t n_rows;
    int32_t log2_slice;
    int32_t Rp;              // padded vector count = L * VPT
    const VT *tcur;          // T_n        [rows][Rp] complex
    const VT *tprev;         // T_{n-1}    (unused on the first step)
    VT *tnext;               // T_{n+1}    (may alias tprev)
    const VT *r;             // start vectors
    VT c1;                   // 2/a (1/a on the first step)
    VT shift;                // b
    double *partial;         // [gridDim.x][Rp] for this moment
};

// Block reduction of acc[VPT] over rows sharing a vector slot; writes
// partial[block][slot * VPT + q].
template <int L, int VPT>
__device__ __forceinline__ void block_reduce_store(double (&acc)[VPT], double *partial) {
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
        partial[(int64_t)blockIdx.x * (L * VPT) + threadIdx.x] = s;
    }
}

template <class VT, int L, int VPT, bool FIRST, bool DIAG>
__global__ __launch_bounds__(kThreads) void k_cheb_step(StepArgs<VT> a) {
    constexpr int RPB = kThreads / L;   // rows per tile
    const int lr = threadIdx.x / L;
    const int vs = threadIdx.x % L;
    const int64_t n_tiles = (a.n_rows + RPB - 1) / RPB;
    const int xcd = blockIdx.x % kNumXcd;
    const int nbx = gridDim.x / kNumXcd;
    const int jb = blockIdx.x / kNumXcd;
    const int64_t t0 = n_tiles * xcd / kNumXcd, t1 = n_tiles * (xcd + 1) / kNumXcd;
    const int64_t smask = ((int64_t)1 << a.log2_slice) - 1;
    const int Rp = a.Rp;
    const int voff = vs * VPT;

    double acc[VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) acc[q] = 0.0;

    for (int64_t t = t0 + jb; t < t1; t += nbx) {
        const int64_t i = t * RPB + lr;
        if (i >= a.n_rows) continue;
        const int64_t s = i >> a.log2_slice;
        const int64_t p0 = a.ptr[s], p1 = a.ptr[s + 1];
        const int64_t base = p0 + (i & smask);
        const int w = (int)((p1 - p0) >> a.log2_slice);
        const int64_t stride = smask + 1;
        Pack<VT, VPT> y;
#pragma unroll
        for (int q = 0; q < VPT; ++q) { y.re[q] = 0; y.im[q] = 0; }
        for (int k = 0; k < w; ++k) {
            const int32_t c = a.col[base + k * stride];
            const VT h = a.val[base + k * stride];
            Pack<VT, VPT> x = load_pack<VT, VPT>(a.tcur + 2 * ((int64_t)c * Rp + voff));
#pragma unroll
            for (int q = 0; q < VPT; ++q) { y.re[q] += h * x.re[q]; y.im[q] += h * x.im[q]; }
        }
        if constexpr (DIAG) {
            const VT d = (a.onsite ? a.onsite[i] : (VT)0) - a.shift;
            Pack<VT, VPT> x = load_pack<VT, VPT>(a.tcur + 2 * (i * Rp + voff));
#pragma unroll
            for (int q = 0; q < VPT; ++q) { y.re[q] += d * x.re[q]; y.im[q] += d * x.im[q]; }
        }
        const int64_t off = 2 * (i * Rp + voff);
        Pack<VT, VPT> o;
        if constexpr (FIRST) {
#pragma unroll
            for (int q = 0; q < VPT; ++q) { o.re[q] = a.c1 * y.re[q]; o.im[q] = a.c1 * y.im[q]; }
        } else {
            Pack<VT, VPT> pv = load_pack<VT, VPT>(a.tprev + off);
#pragma unroll
            for (int q = 0; q < VPT; ++q) {
                o.re[q] = a.c1 * y.re[q] - pv.re[q];
                o.im[q] = a.c1 * y.im[q] - pv.im[q];
            }
        }
        store_pack<VT, VPT>(a.tnext + off, o);
        Pack<VT, VPT> rv = load_pack<VT, VPT>(a.r + off);
#pragma unroll
        for (int q = 0; q < VPT; ++q)
            acc[q] += (double)rv.re[q] * (double)o.re[q] + (double)rv.im[q] * (double)o.im[q];
    }
    block_reduce_store<L, VPT>(acc, a.partial);
}

// r_int[i][v] = r[perm[i]][v] (v < R), 0 for padded vectors; partial sums of |r|^2.
template <class VT, int L, int VPT>
__global__ __launch_bounds__(kThreads) void k_prepare(const VT *__restrict__ r, const int32_t *__restrict__ perm,
                                                      int64_t n_rows, int32_t R, int32_t Rp,
                                                      VT *__restrict__ r_int, double *__restrict__ partial) {
    constexpr int RPB = kThreads / L;
    const int lr = threadIdx.x / L;
    const int vs = threadIdx.x % L;
    double acc[VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RPB + lr; i < n_rows; i += (int64_t)gridDim.x * RPB) {
        const int64_t src = perm ? (int64_t)perm[i] : i;
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int v = vs * VPT + q;
            VT re = 0, im = 0;
            if (v < R) { re = r[2 * (src * R + v)]; im = r[2 * (src * R + v) + 1]; }
            r_int[2 * (i * Rp + v)] = re;
            r_int[2 * (i * Rp + v) + 1] = im;
            acc[q] += (double)re * (double)re + (double)im * (double)im;
        }
    }
    block_reduce_store<L, VPT>(acc, partial);
}

// mu[v][n] = sum_b partial[n][b][v] in a fixed order; one block per moment.
__global__ __launch_bounds__(kThreads) void k_reduce_moments(const double *__restrict__ partial, int32_t G,
                                                             int32_t Rp, int32_t R, int32_t M,
                                                             double *__restrict__ mu) {
    __shared__ double red[kThreads];
    const int n = blockIdx.x;
    for (int v = 0; v < R; ++v) {
        double s = 0.0;
        for (int b = threadIdx.x; b < G; b += kThreads) s += partial[((int64_t)n * G + b) * Rp + v];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) mu[(int64_t)v * M + n] = red[0];
        __syncthreads();
    }
}

// flag = 1 if some |mu_n| exceeds mu_0 (1 + 1e-6) or is not finite.
__global__ void k_guard(const double *__restrict__ mu, int32_t R, int32_t M, int32_t *__restrict__ flag) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)R * M) return;
    int64_t v = idx / M;
    double m0 = mu[v * M];
    double m = mu[idx];
    if (!(fabs(m) <= m0 * (1.0 + 1e-6))) atomicOr(flag, 1);
}

int log2_exact(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return (1 << l) == x ? l : -1;
}

int pad_vectors(int R) {
    int p = 1;
    while (p < R) p <<= 1;
    return p;
}

struct Layout {
    int Rp, L, VPT, G;
    size_t elem;                 // bytes per real component
    size_t vec_bytes;            // one [rows][Rp] complex block
    size_t off_r, off_a, off_b, off_part, off_flag, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

tbk_status make_layout(const tbk_ham *h, int32_t R, int32_t M, int32_t precision, Layout &lay) {
    TBK_CHECK(h != nullptr, TBK_ERR_INVALID_ARG, "h is NULL");
    TBK_CHECK(R >= 1 && R <= 64, TBK_ERR_INVALID_ARG, "R = %d outside [1, 64]", R);
    TBK_CHECK(M >= 2, TBK_ERR_INVALID_ARG, "M = %d < 2", M);
    TBK_CHECK(h->n_rows >= 1, TBK_ERR_INVALID_ARG, "empty Hamiltonian");
    TBK_CHECK(precision == TBK_PREC_F64 || precision == TBK_PREC_C32, TBK_ERR_INVALID_ARG,
              "unknown precision %d", precision);
    if (precision == TBK_PREC_F64)
        TBK_CHECK(h->fmt == TBK_CSR_F64 || h->fmt == TBK_SELL_F64, TBK_ERR_INVALID_ARG,
                  "FP64 recurrence needs a double-valued Hamiltonian");
    else
        TBK_CHECK(h->fmt == TBK_SELL_F32, TBK_ERR_INVALID_ARG, "C32 recurrence needs a float SELL Hamiltonian");
    const int slice = h->fmt == TBK_CSR_F64 ? 1 : h->slice;
    TBK_CHECK(log2_exact(slice) >= 0, TBK_ERR_INVALID_ARG, "slice %d is not a power of two", slice);
    lay.Rp = pad_vectors(R);
    lay.elem = precision == TBK_PREC_F64 ? sizeof(double) : sizeof(float);
    lay.VPT = (precision == TBK_PREC_C32 && lay.Rp >= 2) ? 2 : 1;
    lay.L = lay.Rp / lay.VPT;
    const int64_t rpb = kThreads / lay.L;
    const int64_t tiles = (h->n_rows + rpb - 1) / rpb;
    int64_t G = std::min<int64_t>(kMaxGrid, tiles);
    G = ((G + kNumXcd - 1) / kNumXcd) * kNumXcd;
    lay.G = (int)G;
    lay.vec_bytes = align256((size_t)h->n_rows * lay.Rp * 2 * lay.elem);
    lay.off_r = 0;
    lay.off_a = lay.off_r + lay.vec_bytes;
    lay.off_b = lay.off_a + lay.vec_bytes;
    lay.off_part = lay.off_b + lay.vec_bytes;
    lay.off_flag = lay.off_part + align256((size_t)M * lay.G * lay.Rp * sizeof(double));
    lay.total = lay.off_flag + 256;
    return TBK_OK;
}

template <class VT, int L, int VPT>
void launch_step(bool first, bool diag, int G, hipStream_t s, const StepArgs<VT> &a) {
    if (first) {
        if (diag) k_cheb_step<VT, L, VPT, true, true><<<G, kThreads, 0, s>>>(a);
        else k_cheb_step<VT, L, VPT, true, false><<<G, kThreads, 0, s>>>(a);
    } else {
        if (diag) k_cheb_step<VT, L, VPT, false, true><<<G, kThreads, 0, s>>>(a);
        else k_cheb_step<VT, L, VPT, false, false><<<G, kThreads, 0, s>>>(a);
    }
}

template <class VT, int L, int VPT>
tbk_status run_moments(const tbk_ham *h, double a, double b, const VT *r, int32_t R, int32_t M,
                       const Layout &lay, char *work, double *mu, hipStream_t s) {
    VT *r_int = reinterpret_cast<VT *>(work + lay.off_r);
    VT *TA = reinterpret_cast<VT *>(work + lay.off_a);
    VT *TB = reinterpret_cast<VT *>(work + lay.off_b);
    double *part = reinterpret_cast<double *>(work + lay.off_part);
    int32_t *flag = reinterpret_cast<int32_t *>(work + lay.off_flag);
    const int G = lay.G;
    const int64_t stride = (int64_t)G * lay.Rp;

    k_prepare<VT, L, VPT><<<G, kThreads, 0, s>>>(r, h->perm, h->n_rows, R, lay.Rp, r_int, part);
    TBK_HIP(hipGetLastError());

    StepArgs<VT> sa{};
    sa.ptr = h->ptr;
    sa.col = h->col;
    sa.val = static_cast<const VT *>(h->val);
    sa.onsite = h->has_onsite ? static_cast<const VT *>(h->onsite) : nullptr;
    sa.n_rows = h->n_rows;
    sa.log2_slice = log2_exact(h->fmt == TBK_CSR_F64 ? 1 : h->slice);
    sa.Rp = lay.Rp;
    sa.r = r_int;
    sa.shift = (VT)b;
    const bool diag = h->has_onsite || b != 0.0;

    // n = 1: T_1 = Ht T_0 into TB
    sa.tcur = r_int; sa.tprev = nullptr; sa.tnext = TB; sa.c1 = (VT)(1.0 / a);
    sa.partial = part + stride;
    launch_step<VT, L, VPT>(true, diag, G, s, sa);
    TBK_HIP(hipGetLastError());
    sa.c1 = (VT)(2.0 / a);
    if (M > 2) {
        // n = 2: T_2 = 2 Ht T_1 - T_0 into TA
        sa.tcur = TB; sa.tprev = r_int; sa.tnext = TA;
        sa.partial = part + 2 * stride;
        launch_step<VT, L, VPT>(false, diag, G, s, sa);
        TBK_HIP(hipGetLastError());
    }
    for (int n = 3; n < M; ++n) {
        // T_n overwrites T_{n-2} in place
        VT *cur = (n & 1) ? TA : TB;     // T_{n-1}
        VT *old = (n & 1) ? TB : TA;     // T_{n-2} -> T_n
        sa.tcur = cur; sa.tprev = old; sa.tnext = old;
        sa.partial = part + n * stride;
        launch_step<VT, L, VPT>(false, diag, G, s, sa);
    }
    TBK_HIP(hipGetLastError());
    k_reduce_moments<<<M, kThreads, 0, s>>>(part, G, lay.Rp, R, M, mu);
    TBK_HIP(hipGetLastError());
    TBK_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    const int64_t nm = (int64_t)R * M;
    k_guard<<<(int)ceil_div(nm, 256), 256, 0, s>>>(mu, R, M, flag);
    TBK_HIP(hipGetLastError());
    int32_t hflag = 0;
    TBK_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    TBK_CHECK(hflag == 0, TBK_ERR_SPECTRUM,
              "a moment exceeds mu_0: the scale a = %g, shift b = %g do not bound the spectrum", a, b);
    return TBK_OK;
}

}  // namespace

}  // namespace tbk

using namespace tbk;

extern "C" tbk_status kpm_workspace_size(const tbk_ham *h, int32_t R, int32_t M, int32_t precision,
                                         int64_t *bytes) {
    clear_error();
    TBK_CHECK(bytes != nullptr, TBK_ERR_INVALID_ARG, "bytes is NULL");
    Layout lay;
    tbk_status st = make_layout(h, R, M, precision, lay);
    if (st != TBK_OK) return st;
    *bytes = (int64_t)lay.total;
    return TBK_OK;
}

extern "C" tbk_status kpm_moments(const tbk_ham *h, const double *a, const double *b, const void *r,
                                  int32_t R, int32_t M, int32_t precision, void *work, int64_t work_bytes,
                                  double *mu, void *stream) {
    clear_error();
    Layout lay;
    tbk_status st = make_layout(h, R, M, precision, lay);
    if (st != TBK_OK) return st;
    TBK_CHECK(a && b && r && work && mu, TBK_ERR_INVALID_ARG, "NULL argument");
    TBK_CHECK(h->n_seg == 1, TBK_ERR_UNSUPPORTED, "stacked systems go through kpm_moments_batched");
    TBK_CHECK(std::isfinite(a[0]) && std::isfinite(b[0]), TBK_ERR_NOT_FINITE, "a or b is not finite");
    TBK_CHECK(a[0] > 0, TBK_ERR_INVALID_ARG, "a = %g must be positive", a[0]);
    TBK_CHECK(work_bytes >= (int64_t)lay.total, TBK_ERR_BUFFER_TOO_SMALL,
              "work has %lld bytes, needs %lld", (long long)work_bytes, (long long)lay.total);
    TBK_CHECK(((uintptr_t)work & 255) == 0, TBK_ERR_INVALID_ARG, "work is not 256-byte aligned");
    TBK_CHECK(h->ptr && h->col && h->val && h->onsite, TBK_ERR_INVALID_ARG, "Hamiltonian array is NULL");
    hipStream_t s = as_stream(stream);
    char *w = static_cast<char *>(work);
    if (precision == TBK_PREC_F64) {
        const double *rr = static_cast<const double *>(r);
        switch (lay.L) {
        case 1: return run_moments<double, 1, 1>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 2: return run_moments<double, 2, 1>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 4: return run_moments<double, 4, 1>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 8: return run_moments<double, 8, 1>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 16: return run_moments<double, 16, 1>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 32: return run_moments<double, 32, 1>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 64: return run_moments<double, 64, 1>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        }
    } else {
        const float *rr = static_cast<const float *>(r);
        if (lay.VPT == 1) return run_moments<float, 1, 1>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        switch (lay.L) {
        case 1: return run_moments<float, 1, 2>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 2: return run_moments<float, 2, 2>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 4: return run_moments<float, 4, 2>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 8: return run_moments<float, 8, 2>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 16: return run_moments<float, 16, 2>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        case 32: return run_moments<float, 32, 2>(h, a[0], b[0], rr, R, M, lay, w, mu, s);
        }
    }
    return fail(TBK_ERR_UNSUPPORTED, "no kernel for R = %d", R);
}
