// Chebyshev recurrence with fused moment accumulation (KPM, Sec. 2.4).
//
// One launch per recurrence step.  A tile is 256 / L consecutive rows; every
// thread owns one row of the tile and VPT of the R vectors (L = R / VPT threads
// per row).  The thread gathers T_n over the row's stored entries, writes
// T_{n+1} = c1 (H - b) T_n - c0 T_{n-1} over T_{n-1} in place, and accumulates
// Re(conj(r) T_{n+1}) in double.  A block handles `tiles_per_block`
// consecutive tiles, reduces its rows by wavefront shuffles and LDS and writes
// one partial per vector; every few steps a reduction kernel folds the block
// partials in a fixed two-level order (bitwise reproducible, no float atomics).
//
// Launch shapes (tuned per problem): with xcd_remap, workgroup b (which the
// hardware dispatches to XCD b % 8) takes logical block (b % 8) G/8 + b / 8,
// so each XCD sweeps its own contiguous eighth of the rows; otherwise blocks
// take tiles in dispatch order.  With nontemporal, the streamed arrays
// (values, columns, T_{n-1}, r, T_{n+1}) bypass cache retention so that the
// L2 keeps the gathered T_n.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kpm.hpp"
#include "kpm_dev.hpp"

namespace tbk {

namespace {

constexpr int kReduceChunk = 2048;                 // partials per first-level reduction block
constexpr size_t kPartialBudget = 256ull << 20;    // bytes of block partials kept between reductions


// One recurrence step.  Each thread handles RPT rows (from RPT consecutive
// tiles of its block).  All loads of a row group are issued before any is
// used: the streamed operands, then the row's entries (KU at a time, or all W
// of them when every slice has the same width W), then the gathers of T_n, so
// a row costs two dependent memory round trips instead of one per entry.
// Rows past the end are clamped to the last row for their loads (always in
// bounds) and neither stored nor counted; entries past a slice's width are
// clamped to its last entry and weighted by zero.
template <class VT, int L, int VPT, bool FIRST, bool DIAG, bool NT, bool TIS, int RPT, int W, bool DBL>
__global__ __launch_bounds__(kThreads) void k_cheb_step(
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ col, const int16_t *__restrict__ col16,
    const VT *__restrict__ val, const VT *__restrict__ onsite, const VT *__restrict__ tcur, const VT *tprev,
    VT *tnext, const VT *__restrict__ r, double *__restrict__ partial, StepScalars<VT> a) {
    constexpr int RPB = kThreads / L;   // rows per tile
    constexpr int KU = W > 0 ? W : 4;   // entries per batch of loads
    const int lr = threadIdx.x / L;
    const int vs = threadIdx.x % L;
    const int64_t lb = logical_block(a.xcd_remap);
    const int64_t t0 = lb * a.tiles_per_block;
    const int64_t t1 = min(t0 + a.tiles_per_block, a.n_tiles);
    const int64_t smask = ((int64_t)1 << a.log2_slice) - 1;
    const int64_t stride = smask + 1;
    const int Rp = a.Rp;
    const int voff = vs * VPT;
    const int64_t last = a.n_rows - 1;

    constexpr int NA = DBL ? 2 * VPT : VPT;   // sums per thread
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;

    for (int64_t t = t0; t < t1; t += RPT) {
        int64_t i[RPT], base[RPT], off[RPT];
        int w[RPT];
        bool ok[RPT];
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int64_t tu = min(t + u, t1 - 1);
            const int64_t iu = (t + u) * RPB + lr;
            ok[u] = (t + u < t1) && (iu <= last);
            i[u] = min(tu * RPB + lr, last);
            off[u] = 2 * (i[u] * Rp + voff);
            int64_t p0, p1;
            if constexpr (TIS) {            // the tile is one slice: block-uniform offsets
                p0 = ptr[tu];
                p1 = ptr[tu + 1];
                base[u] = p0 + (i[u] & smask);
            } else {
                const int64_t sl = i[u] >> a.log2_slice;
                p0 = ptr[sl];
                p1 = ptr[sl + 1];
                base[u] = p0 + (i[u] & smask);
            }
            w[u] = W > 0 ? W : (int)((p1 - p0) >> a.log2_slice);
        }
        // streamed operands first: they do not depend on the entries
        Pack<VT, VPT> pv[RPT], rv[RPT];
        VT dg[RPT];
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            if constexpr (!FIRST) pv[u] = load_pack<NT, VT, VPT>(tprev + off[u]);
            // direct form: the start vector; doubling form: the row's own T_n
            if constexpr (DBL) rv[u] = load_pack<false, VT, VPT>(tcur + off[u]);
            else rv[u] = load_pack<NT, VT, VPT>(r + off[u]);
            if constexpr (DIAG) dg[u] = (onsite ? ld<NT>(onsite + i[u]) : (VT)0) - a.shift;
        }
        Pack<VT, VPT> y[RPT];
#pragma unroll
        for (int u = 0; u < RPT; ++u)
#pragma unroll
            for (int q = 0; q < VPT; ++q) { y[u].re[q] = 0; y[u].im[q] = 0; }
        int wmax = 0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) wmax = max(wmax, w[u]);
        for (int k0 = 0; k0 < wmax; k0 += KU) {
            int32_t c[RPT][KU];
            VT h[RPT][KU];
#pragma unroll
            for (int u = 0; u < RPT; ++u)
#pragma unroll
                for (int k = 0; k < KU; ++k) {
                    if constexpr (W > 0) {
                        if (a.compact) {
                            const int16_t d = ld<NT>(col16 + base[u] + k * stride);
                            c[u][k] = d == -32768 ? ld<NT>(col + base[u] + k * stride) : (int32_t)i[u] + d;
                        } else {
                            c[u][k] = ld<NT>(col + base[u] + k * stride);
                        }
                        if (a.uniform) h[u][k] = c[u][k] == (int32_t)i[u] ? (VT)0 : a.hop;   // padding: own row
                        else h[u][k] = ld<NT>(val + base[u] + k * stride);
                    } else {
                        // w[u] >= 1 here unless the whole slice is empty; then read the
                        // row's own diagonal position (entry 0 of a neighbouring slice
                        // is never read: kk is clamped below 0 -> use the row itself).
                        const int kk = min(k0 + k, w[u] - 1);
                        if (kk >= 0) {
                            if (a.compact) {
                                const int16_t d = ld<NT>(col16 + base[u] + kk * stride);
                                c[u][k] = d == -32768 ? ld<NT>(col + base[u] + kk * stride) : (int32_t)i[u] + d;
                            } else {
                                c[u][k] = ld<NT>(col + base[u] + kk * stride);
                            }
                            if (k0 + k >= w[u]) h[u][k] = 0;
                            else if (a.uniform) h[u][k] = c[u][k] == (int32_t)i[u] ? (VT)0 : a.hop;
                            else h[u][k] = ld<NT>(val + base[u] + kk * stride);
                        } else {
                            c[u][k] = (int32_t)i[u];
                            h[u][k] = 0;
                        }
                    }
                }
            Pack<VT, VPT> x[RPT][KU];
#pragma unroll
            for (int u = 0; u < RPT; ++u)
#pragma unroll
                for (int k = 0; k < KU; ++k)
                    x[u][k] = load_pack<false, VT, VPT>(tcur + 2 * ((int64_t)c[u][k] * Rp + voff));
#pragma unroll
            for (int u = 0; u < RPT; ++u)
#pragma unroll
                for (int k = 0; k < KU; ++k)
#pragma unroll
                    for (int q = 0; q < VPT; ++q) {
                        y[u].re[q] += h[u][k] * x[u][k].re[q];
                        y[u].im[q] += h[u][k] * x[u][k].im[q];
                    }
        }
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            if constexpr (DIAG) {
                Pack<VT, VPT> x = load_pack<false, VT, VPT>(tcur + off[u]);
#pragma unroll
                for (int q = 0; q < VPT; ++q) { y[u].re[q] += dg[u] * x.re[q]; y[u].im[q] += dg[u] * x.im[q]; }
            }
            Pack<VT, VPT> o;
#pragma unroll
            for (int q = 0; q < VPT; ++q) {
                if constexpr (FIRST) {
                    o.re[q] = a.c1 * y[u].re[q];
                    o.im[q] = a.c1 * y[u].im[q];
                } else {
                    o.re[q] = a.c1 * y[u].re[q] - pv[u].re[q];
                    o.im[q] = a.c1 * y[u].im[q] - pv[u].im[q];
                }
            }
            if (ok[u]) {
                store_pack<NT, VT, VPT>(tnext + off[u], o);
#pragma unroll
                for (int q = 0; q < VPT; ++q) {
                    const double cr = (double)rv[u].re[q] * (double)o.re[q] + (double)rv[u].im[q] * (double)o.im[q];
                    if constexpr (DBL) {
                        acc[q] += (double)o.re[q] * (double)o.re[q] + (double)o.im[q] * (double)o.im[q];
                        acc[VPT + q] += cr;
                    } else {
                        acc[q] += cr;
                    }
                }
            }
        }
    }
    block_reduce_store<L, NA>(acc, partial, lb);
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

// r_int[i][v] = r[perm[i]][v] (v < R), 0 for padded vectors; block partials of
// |r|^2 (in the doubling layout, each followed by VPT zeros).  With `seeded`
// the phases are generated for atom perm[i] (output perm[i] R + v) instead of
// being read from r.
template <class VT, int L, int VPT, bool DBL>
__global__ __launch_bounds__(kThreads) void k_prepare(const VT *__restrict__ r, const int32_t *__restrict__ perm,
                                                      int64_t n_rows, int32_t R, int32_t Rp, int32_t seeded,
                                                      uint64_t seed, VT *__restrict__ r_int,
                                                      double *__restrict__ partial) {
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
            if (v < R) {
                if (seeded) {
                    double c, sn;
                    seeded_phase(seed, (uint64_t)src * (uint64_t)R + (uint64_t)v, c, sn);
                    re = (VT)c;
                    im = (VT)sn;
                } else {
                    re = r[2 * (src * R + v)];
                    im = r[2 * (src * R + v) + 1];
                }
            }
            r_int[2 * (i * Rp + v)] = re;
            r_int[2 * (i * Rp + v) + 1] = im;
            acc[q] += (double)re * (double)re + (double)im * (double)im;
        }
    }
    if constexpr (DBL) {
        double acc2[2 * VPT];
#pragma unroll
        for (int q = 0; q < VPT; ++q) { acc2[q] = acc[q]; acc2[VPT + q] = 0.0; }
        block_reduce_store<L, 2 * VPT>(acc2, partial, blockIdx.x);
    } else {
        block_reduce_store<L, VPT>(acc, partial, blockIdx.x);
    }
}

// Block partials of Re <left|start> per vector slot (slot 0 of the first batch
// in the pair form of the recurrence); both vectors in row order, [rows][Rp].
template <class VT, int L, int VPT>
__global__ __launch_bounds__(kThreads) void k_pair_overlap(const VT *__restrict__ left,
                                                           const VT *__restrict__ start, int64_t n_rows,
                                                           int32_t Rp, double *__restrict__ partial) {
    constexpr int RPB = kThreads / L;
    const int lr = threadIdx.x / L;
    const int vs = threadIdx.x % L;
    double acc[VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RPB + lr; i < n_rows; i += (int64_t)gridDim.x * RPB) {
        const int64_t off = 2 * (i * Rp + vs * VPT);
        const Pack<VT, VPT> l = load_pack<false, VT, VPT>(left + off);
        const Pack<VT, VPT> t = load_pack<false, VT, VPT>(start + off);
#pragma unroll
        for (int q = 0; q < VPT; ++q)
            acc[q] += (double)l.re[q] * (double)t.re[q] + (double)l.im[q] * (double)t.im[q];
    }
    block_reduce_store<L, VPT>(acc, partial, blockIdx.x);
}

// Doubling identities for a Hermitian Ht (T_m T_n = (T_{m+n} + T_{|m-n|})/2):
// with a[v][k] = <T_k|T_k> and b[v][k] = Re <T_k|T_{k-1}> (k = 1..K; a[v][0] = mu_0),
//   mu_0 = a[v][0], mu_1 = b[v][1], mu_{2k} = 2 a[v][k] - mu_0, mu_{2k-1} = 2 b[v][k] - mu_1.
// raw is [Rv][K+1] over virtual vectors v' = (v / VPT) 2 VPT + (v % VPT) (+ VPT for b).
__global__ void k_doubling_combine(const double *__restrict__ raw, int32_t K, int32_t VPT, int32_t R, int32_t M,
                                   double *__restrict__ mu) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)R * M) return;
    const int v = (int)(idx / M), m = (int)(idx % M);
    const int va = (v / VPT) * 2 * VPT + (v % VPT), vb = va + VPT;
    const double *a = raw + (int64_t)va * (K + 1), *b = raw + (int64_t)vb * (K + 1);
    double out;
    if (m == 0) out = a[0];
    else if (m == 1) out = b[1];
    else if ((m & 1) == 0) out = 2.0 * a[m / 2] - a[0];
    else out = 2.0 * b[(m + 1) / 2] - b[1];
    mu[(int64_t)v * M + m] = out;
}

// First level: l1[n0 + k][v][c] = sum of partial[k][b][v] over b in chunk c.
// grid = (n_chunks, K).  Thread t reads vector v = t % Rp of blocks
// b0 + t / Rp, b0 + t / Rp + 256 / Rp, ..., so a wavefront reads whole rows of
// partial[k][b][0..Rp) (contiguous); the per-vector sums are then folded in LDS
// over the 256 / Rp thread groups in a fixed tree.
__global__ __launch_bounds__(kThreads) void k_reduce_l1(const double *__restrict__ partial, int64_t G, int32_t Rp,
                                                        int32_t R, int32_t n0, int32_t n_chunks,
                                                        double *__restrict__ l1) {
    __shared__ double red[kThreads];
    const int c = blockIdx.x;
    const int k = blockIdx.y;
    const int v = threadIdx.x % Rp;
    const int j = threadIdx.x / Rp;
    const int groups = kThreads / Rp;
    const double *p = partial + (int64_t)k * G * Rp;
    const int64_t b0 = (int64_t)c * kReduceChunk;
    const int64_t b1 = min(b0 + kReduceChunk, G);
    double s = 0.0;
    for (int64_t b = b0 + j; b < b1; b += groups) s += p[b * Rp + v];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int g = groups / 2; g > 0; g >>= 1) {
        if (j < g) red[threadIdx.x] += red[threadIdx.x + g * Rp];
        __syncthreads();
    }
    if (j == 0 && v < R) l1[((int64_t)(n0 + k) * R + v) * n_chunks + c] = red[v];
}

// Second level: mu[v][n] = sum over chunks of l1[n][v][c], in chunk order.
__global__ void k_reduce_l2(const double *__restrict__ l1, int32_t R, int32_t M, int32_t n_chunks,
                            double *__restrict__ mu) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)R * M) return;
    const int64_t n = idx / R, v = idx % R;
    const double *p = l1 + (n * R + v) * n_chunks;
    double s = 0.0;
    for (int c = 0; c < n_chunks; ++c) s += p[c];
    mu[v * M + n] = s;
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

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }


// rows_per_thread 4 is instantiated for one vector per row on width-3 slices
// (the latency-bound case: 44-56 B per row); elsewhere it runs as 2.
template <class VT, int L, int VPT, bool FIRST, bool DIAG, bool NT, bool TIS, int W, bool DBL>
void launch_step_d(const KpmPlan &pl, hipStream_t s, const StepPtrs<VT> &p, const StepScalars<VT> &a) {
    if constexpr (L == 1 && VPT == 1 && W == 3) {
        if (pl.cfg.rows_per_thread == 4) {
            k_cheb_step<VT, L, VPT, FIRST, DIAG, NT, TIS, 4, W, DBL><<<(unsigned)pl.G, kThreads, 0, s>>>(
                p.ptr, p.col, p.col16, p.val, p.onsite, p.tcur, p.tprev, p.tnext, p.r, p.partial, a);
            return;
        }
    }
    if (pl.cfg.rows_per_thread >= 2)
        k_cheb_step<VT, L, VPT, FIRST, DIAG, NT, TIS, 2, W, DBL><<<(unsigned)pl.G, kThreads, 0, s>>>(
            p.ptr, p.col, p.col16, p.val, p.onsite, p.tcur, p.tprev, p.tnext, p.r, p.partial, a);
    else
        k_cheb_step<VT, L, VPT, FIRST, DIAG, NT, TIS, 1, W, DBL><<<(unsigned)pl.G, kThreads, 0, s>>>(
            p.ptr, p.col, p.col16, p.val, p.onsite, p.tcur, p.tprev, p.tnext, p.r, p.partial, a);
}

template <class VT, int L, int VPT, bool FIRST, bool DIAG, bool NT, bool TIS, int W>
void launch_step_w(const KpmPlan &pl, hipStream_t s, const StepPtrs<VT> &p, const StepScalars<VT> &a) {
    if (pl.cfg.doubling) launch_step_d<VT, L, VPT, FIRST, DIAG, NT, TIS, W, true>(pl, s, p, a);
    else launch_step_d<VT, L, VPT, FIRST, DIAG, NT, TIS, W, false>(pl, s, p, a);
}

// Slices of one common width 3 (nearest-neighbour honeycomb) take a fully
// unrolled kernel; any other width pattern the general one (batches of four
// entries: an unrolled width-12 variant for s, p orbitals measured slower,
// its registers cut the occupancy).
template <class VT, int L, int VPT, bool FIRST, bool DIAG, bool NT, bool TIS>
void launch_step_rpt(const KpmPlan &pl, hipStream_t s, const StepPtrs<VT> &p, const StepScalars<VT> &a) {
    if (pl.uniform_width == 3) launch_step_w<VT, L, VPT, FIRST, DIAG, NT, TIS, 3>(pl, s, p, a);
    else launch_step_w<VT, L, VPT, FIRST, DIAG, NT, TIS, 0>(pl, s, p, a);
}

template <class VT, int L, int VPT, bool FIRST, bool DIAG>
void launch_step_nt(const KpmPlan &pl, hipStream_t s, const StepPtrs<VT> &p, const StepScalars<VT> &a) {
    const bool tis = pl.tile_is_slice;
    if (pl.cfg.nontemporal) {
        if (tis) launch_step_rpt<VT, L, VPT, FIRST, DIAG, true, true>(pl, s, p, a);
        else launch_step_rpt<VT, L, VPT, FIRST, DIAG, true, false>(pl, s, p, a);
    } else {
        if (tis) launch_step_rpt<VT, L, VPT, FIRST, DIAG, false, true>(pl, s, p, a);
        else launch_step_rpt<VT, L, VPT, FIRST, DIAG, false, false>(pl, s, p, a);
    }
}

template <class VT, int L, int VPT>
void launch_step(const KpmPlan &pl, bool first, bool diag, hipStream_t s, const StepPtrs<VT> &p,
                 const StepScalars<VT> &a) {
    if (first) {
        if (diag) launch_step_nt<VT, L, VPT, true, true>(pl, s, p, a);
        else launch_step_nt<VT, L, VPT, true, false>(pl, s, p, a);
    } else {
        if (diag) launch_step_nt<VT, L, VPT, false, true>(pl, s, p, a);
        else launch_step_nt<VT, L, VPT, false, false>(pl, s, p, a);
    }
}

void launch_reduce(const KpmPlan &pl, int n0, int count, int R, double *part, double *l1, hipStream_t s) {
    dim3 grid(pl.n_chunks, count);
    k_reduce_l1<<<grid, kThreads, 0, s>>>(part, pl.G, pl.Rp, R, n0, pl.n_chunks, l1);
}

// start/left (row order, [rows][Rp], both non-NULL) select the pair form:
// T_0 = start and mu_n = Re <left|T_n>, without the spectrum guard.
template <class VT, int L, int VPT, bool DBL>
tbk_status run_moments_t(const tbk_ham *h, const KpmPlan &pl, double a, double b, const VT *r, int32_t R,
                         int32_t M, char *work, double *mu, hipStream_t s, const VT *start, const VT *left) {
    const bool pair = left != nullptr;
    VT *r_int = reinterpret_cast<VT *>(work + pl.off_r);
    VT *TA = reinterpret_cast<VT *>(work + pl.off_a);
    VT *TB = reinterpret_cast<VT *>(work + pl.off_b);
    double *part = reinterpret_cast<double *>(work + pl.off_part);
    double *l1 = reinterpret_cast<double *>(work + pl.off_l1);
    double *raw = reinterpret_cast<double *>(work + pl.off_raw);
    int32_t *flag = reinterpret_cast<int32_t *>(work + pl.off_flag);
    const int Rv = pl.Rv;           // partial sums per block (per step)
    const int Mr = pl.Mr;           // reduced rows: moments (direct) or steps + 1 (doubling)
    const int Rout = DBL ? Rv : R;  // sums kept after the reduction
    const int64_t pstride = pl.G * Rv;
    const int K = pl.reduce_every;

    // row 0 goes through the same partial slots as the steps (slot 0 of the first batch)
    if (pair)
        k_pair_overlap<VT, L, VPT><<<(unsigned)pl.G, kThreads, 0, s>>>(left, start, h->n_rows, pl.Rp, part);
    else
        k_prepare<VT, L, VPT, DBL><<<(unsigned)pl.G, kThreads, 0, s>>>(r, h->perm, h->n_rows, R, pl.Rp,
                                                                        pl.seeded ? 1 : 0, pl.seed, r_int, part);
    TBK_HIP(hipGetLastError());
    const VT *t0 = pair ? start : r_int;

    StepPtrs<VT> sp{};
    sp.ptr = h->ptr;
    sp.col = h->col;
    sp.col16 = h->col16;
    sp.val = static_cast<const VT *>(h->val);
    sp.onsite = h->has_onsite ? static_cast<const VT *>(h->onsite) : nullptr;
    sp.r = pair ? left : r_int;
    StepScalars<VT> sa{};
    sa.n_rows = h->n_rows;
    sa.n_tiles = pl.n_tiles;
    sa.log2_slice = pl.log2_slice;
    sa.Rp = pl.Rp;
    sa.tiles_per_block = pl.cfg.tiles_per_block;
    sa.xcd_remap = pl.cfg.xcd_remap;
    sa.shift = (VT)b;
    sa.hop = (VT)h->hop_value;
    sa.uniform = pl.cfg.uniform_values;
    sa.compact = pl.cfg.compact_columns;
    const bool diag = h->has_onsite || b != 0.0;
    auto reduce = [&](int n0, int count) {
        dim3 grid(pl.n_chunks, count);
        k_reduce_l1<<<grid, kThreads, 0, s>>>(part, pl.G, Rv, Rout, n0, pl.n_chunks, l1);
    };

    int batch0 = 0;   // first row index of the pending batch
    for (int n = 1; n < Mr; ++n) {
        if (n - batch0 == K) {
            reduce(batch0, K);
            batch0 = n;
        }
        sp.partial = part + (int64_t)(n - batch0) * pstride;
        if (n == 1) {            // T_1 = Ht T_0 into TB
            sp.tcur = t0; sp.tprev = nullptr; sp.tnext = TB; sa.c1 = (VT)(1.0 / a);
        } else if (n == 2) {     // T_2 = 2 Ht T_1 - T_0 into TA
            sp.tcur = TB; sp.tprev = t0; sp.tnext = TA; sa.c1 = (VT)(2.0 / a);
        } else {                 // T_n overwrites T_{n-2} in place
            VT *cur = (n & 1) ? TA : TB;
            VT *old = (n & 1) ? TB : TA;
            sp.tcur = cur; sp.tprev = old; sp.tnext = old;
        }
        if (pl.block) {
            tbk_status st = launch_step_block<VT>(pl, n == 1, diag, s, sp, sa);
            if (st != TBK_OK) return st;
        } else {
            launch_step<VT, L, VPT>(pl, n == 1, diag, s, sp, sa);
        }
    }
    reduce(batch0, Mr - batch0);
    TBK_HIP(hipGetLastError());
    const int64_t nm = (int64_t)R * M;
    if constexpr (DBL) {
        k_reduce_l2<<<(unsigned)ceil_div((int64_t)Rv * Mr, 256), 256, 0, s>>>(l1, Rv, Mr, pl.n_chunks, raw);
        TBK_HIP(hipGetLastError());
        k_doubling_combine<<<(unsigned)ceil_div(nm, 256), 256, 0, s>>>(raw, Mr - 1, VPT, R, M, mu);
    } else {
        k_reduce_l2<<<(unsigned)ceil_div(nm, 256), 256, 0, s>>>(l1, R, M, pl.n_chunks, mu);
    }
    TBK_HIP(hipGetLastError());
    if (pair) return TBK_OK;     // no guard: |mu_n| <= mu_0 holds only for left = start
    TBK_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    k_guard<<<(unsigned)ceil_div(nm, 256), 256, 0, s>>>(mu, R, M, flag);
    TBK_HIP(hipGetLastError());
    int32_t hflag = 0;
    TBK_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    TBK_CHECK(hflag == 0, TBK_ERR_SPECTRUM,
              "a moment exceeds mu_0: the scale a = %g, shift b = %g do not bound the spectrum", a, b);
    return TBK_OK;
}

template <class VT, int L, int VPT>
tbk_status run_moments(const tbk_ham *h, const KpmPlan &pl, double a, double b, const VT *r, int32_t R,
                       int32_t M, char *work, double *mu, hipStream_t s, const VT *start, const VT *left) {
    if (pl.cfg.doubling) return run_moments_t<VT, L, VPT, true>(h, pl, a, b, r, R, M, work, mu, s, start, left);
    return run_moments_t<VT, L, VPT, false>(h, pl, a, b, r, R, M, work, mu, s, start, left);
}

}  // namespace

int pad_vectors(int R) {
    int p = 1;
    while (p < R) p <<= 1;
    return p;
}

tbk_kpm_config default_config(const tbk_ham *h, int32_t R, int32_t precision) {
    tbk_kpm_config c{};
    c.vectors_per_thread = (precision == TBK_PREC_C32 && pad_vectors(R) >= 2) ? 2 : 1;
    c.tiles_per_block = 2;
    c.nontemporal = 1;
    c.xcd_remap = 0;
    c.rows_per_thread = 1;
    c.persistent = 0;
    c.doubling = 0;
    c.uniform_values = 0;
    c.compact_columns = 0;
    c.atom_rows = (h && (h->fmt == TBK_BSELL4_F64 || h->fmt == TBK_BSELL4_F32 || h->fmt == TBK_BGEOM_F64 ||
                         h->fmt == TBK_BGEOM_F32))
                      ? 1
                      : 0;
    return c;
}

tbk_status make_plan(const tbk_ham *h, int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                     KpmPlan &pl) {
    TBK_CHECK(h != nullptr, TBK_ERR_INVALID_ARG, "h is NULL");
    TBK_CHECK(R >= 1 && R <= 64, TBK_ERR_INVALID_ARG, "R = %d outside [1, 64]", R);
    TBK_CHECK(M >= 2, TBK_ERR_INVALID_ARG, "M = %d < 2", M);
    TBK_CHECK(h->n_rows >= 1, TBK_ERR_INVALID_ARG, "empty Hamiltonian");
    TBK_CHECK(precision == TBK_PREC_F64 || precision == TBK_PREC_C32, TBK_ERR_INVALID_ARG,
              "unknown precision %d", precision);
    if (precision == TBK_PREC_F64)
        TBK_CHECK(h->fmt == TBK_CSR_F64 || h->fmt == TBK_SELL_F64 || h->fmt == TBK_BSELL4_F64 ||
                      h->fmt == TBK_BGEOM_F64,
                  TBK_ERR_INVALID_ARG, "FP64 recurrence needs a double-valued Hamiltonian");
    else
        TBK_CHECK(h->fmt == TBK_SELL_F32 || h->fmt == TBK_BSELL4_F32 || h->fmt == TBK_BGEOM_F32, TBK_ERR_INVALID_ARG,
                  "C32 recurrence needs a float SELL Hamiltonian");
    pl.geom = h->fmt == TBK_BGEOM_F64 || h->fmt == TBK_BGEOM_F32;
    pl.block = h->fmt == TBK_BSELL4_F64 || h->fmt == TBK_BSELL4_F32 || pl.geom;
    if (pl.geom) {
        for (int k = 0; k < 12; ++k) pl.geom_params[k] = h->sk_geom[k];
        TBK_CHECK(h->sk_geom[10] > 0 && std::isfinite(h->sk_geom[11]), TBK_ERR_INVALID_ARG,
                  "sk_geom: r0 must be positive and beta finite");
    }
    if (pl.block) {
        TBK_CHECK((h->n_orb == 4 || h->n_orb == 9) && h->n_rows % h->n_orb == 0, TBK_ERR_INVALID_ARG,
                  "a block Hamiltonian has 4 or 9 orbital rows per atom (n_orb = %d)", h->n_orb);
        pl.norb = h->n_orb;
    }
    const int slice = h->fmt == TBK_CSR_F64 ? 1 : h->slice;
    pl.log2_slice = log2_exact(slice);
    TBK_CHECK(pl.log2_slice >= 0, TBK_ERR_INVALID_ARG, "slice %d is not a power of two", slice);
    pl.cfg = cfg ? *cfg : default_config(h, R, precision);
    pl.Rp = pad_vectors(R);
    pl.elem = precision == TBK_PREC_F64 ? sizeof(double) : sizeof(float);
    TBK_CHECK(pl.cfg.vectors_per_thread == 1 || (pl.cfg.vectors_per_thread == 2 && precision == TBK_PREC_C32 &&
                                                 pl.Rp >= 2),
              TBK_ERR_INVALID_ARG, "vectors_per_thread must be 1, or 2 for the C32 recurrence with R >= 2");
    TBK_CHECK(pl.cfg.tiles_per_block >= 1 && pl.cfg.tiles_per_block <= (1 << 20), TBK_ERR_INVALID_ARG,
              "tiles_per_block = %d outside [1, 2^20]", pl.cfg.tiles_per_block);
    TBK_CHECK(pl.cfg.nontemporal == 0 || pl.cfg.nontemporal == 1, TBK_ERR_INVALID_ARG, "nontemporal must be 0/1");
    TBK_CHECK(pl.cfg.xcd_remap == 0 || pl.cfg.xcd_remap == 1, TBK_ERR_INVALID_ARG, "xcd_remap must be 0/1");
    TBK_CHECK(pl.cfg.rows_per_thread == 1 || pl.cfg.rows_per_thread == 2 || pl.cfg.rows_per_thread == 4,
              TBK_ERR_INVALID_ARG, "rows_per_thread must be 1, 2 or 4");
    TBK_CHECK(pl.cfg.persistent == 0 || pl.cfg.persistent == 1, TBK_ERR_INVALID_ARG, "persistent must be 0/1");
    TBK_CHECK(pl.cfg.doubling == 0 || pl.cfg.doubling == 1, TBK_ERR_INVALID_ARG, "doubling must be 0/1");
    TBK_CHECK(pl.cfg.uniform_values == 0 || pl.cfg.uniform_values == 1, TBK_ERR_INVALID_ARG,
              "uniform_values must be 0/1");
    TBK_CHECK(pl.cfg.uniform_values == 0 || h->uniform_hop == 1, TBK_ERR_INVALID_ARG,
              "uniform_values needs a Hamiltonian whose stored hoppings are all equal (h->uniform_hop)");
    TBK_CHECK(pl.cfg.compact_columns == 0 || pl.cfg.compact_columns == 1, TBK_ERR_INVALID_ARG,
              "compact_columns must be 0/1");
    TBK_CHECK(pl.cfg.compact_columns == 0 || h->col16 != nullptr, TBK_ERR_INVALID_ARG,
              "compact_columns needs the 16-bit column offsets h->col16");
    TBK_CHECK(!pl.block || (pl.cfg.uniform_values == 0 && pl.cfg.compact_columns == 0), TBK_ERR_INVALID_ARG,
              "uniform_values and compact_columns are not offered for block Hamiltonians");
    TBK_CHECK(pl.cfg.atom_rows == 0 || pl.cfg.atom_rows == 1, TBK_ERR_INVALID_ARG, "atom_rows must be 0/1");
    if (!pl.block) pl.cfg.atom_rows = 0;
    if (pl.geom) pl.cfg.atom_rows = 1;     // the displacement form has a thread per atom only
    pl.VPT = pl.cfg.vectors_per_thread;
    pl.L = pl.Rp / pl.VPT;
    const int64_t rpb = kThreads / pl.L;
    // tiles of rpb orbital rows, or of rpb atoms in the atom form of the block kernel
    const int64_t tiled = pl.cfg.atom_rows ? h->n_rows / pl.norb : h->n_rows;
    pl.n_tiles = (tiled + rpb - 1) / rpb;
    int64_t G = (pl.n_tiles + pl.cfg.tiles_per_block - 1) / pl.cfg.tiles_per_block;
    if (pl.cfg.xcd_remap) {
        // round up to a multiple of the XCD count; the extra blocks own no tile
        G = ((G + kNumXcd - 1) / kNumXcd) * kNumXcd;
    }
    TBK_CHECK(G < (int64_t)INT32_MAX, TBK_ERR_UNSUPPORTED, "grid too large");
    pl.G = G;
    pl.tile_is_slice = (slice == rpb);
    // every slice stores the same number of entries per row
    const int64_t n_slices = ceil_div(h->n_rows, slice);
    pl.uniform_width = (!pl.block && h->max_degree > 0 && h->n_entries == n_slices * slice * (int64_t)h->max_degree)
                           ? h->max_degree : 0;
    pl.n_chunks = (int)ceil_div(G, kReduceChunk);
    TBK_CHECK(pl.n_chunks < 65536, TBK_ERR_UNSUPPORTED, "too many blocks");
    pl.Rv = pl.cfg.doubling ? 2 * pl.Rp : pl.Rp;
    pl.Mr = pl.cfg.doubling ? M / 2 + 1 : M;
    const int Rout = pl.cfg.doubling ? pl.Rv : R;
    const size_t per_step = (size_t)G * pl.Rv * sizeof(double);
    pl.reduce_every = (int)std::max<size_t>(1, std::min<size_t>({kPartialBudget / per_step, (size_t)64, (size_t)pl.Mr}));
    TBK_CHECK(pl.reduce_every < 65536, TBK_ERR_UNSUPPORTED, "reduction grid too large");
    pl.vec_bytes = align256((size_t)h->n_rows * pl.Rp * 2 * pl.elem);
    pl.off_r = 0;
    pl.off_a = pl.off_r + pl.vec_bytes;
    pl.off_b = pl.off_a + pl.vec_bytes;
    pl.off_part = pl.off_b + pl.vec_bytes;
    // k_prepare writes one partial per block of its own grid (<= G blocks)
    pl.off_l1 = pl.off_part + align256((size_t)pl.reduce_every * per_step);
    pl.off_raw = pl.off_l1 + align256((size_t)pl.Mr * Rout * pl.n_chunks * sizeof(double));
    pl.off_flag = pl.off_raw + align256((size_t)pl.Mr * Rout * sizeof(double));
    pl.total = pl.off_flag + 256;
    return TBK_OK;
}

tbk_status run_plan(const tbk_ham *h, const KpmPlan &pl, double a, double b, const void *r, int32_t R,
                    int32_t M, int32_t precision, char *w, double *mu, hipStream_t s, const void *start,
                    const void *left) {
    const double *sd = static_cast<const double *>(start), *ld_ = static_cast<const double *>(left);
    const float *sf = static_cast<const float *>(start), *lf = static_cast<const float *>(left);
    if (precision == TBK_PREC_F64) {
        const double *rr = static_cast<const double *>(r);
        switch (pl.L) {
        case 1: return run_moments<double, 1, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 2: return run_moments<double, 2, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 4: return run_moments<double, 4, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 8: return run_moments<double, 8, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 16: return run_moments<double, 16, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 32: return run_moments<double, 32, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 64: return run_moments<double, 64, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        }
    } else {
        const float *rr = static_cast<const float *>(r);
        if (pl.VPT == 1) {
            switch (pl.L) {
            case 1: return run_moments<float, 1, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 2: return run_moments<float, 2, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 4: return run_moments<float, 4, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 8: return run_moments<float, 8, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 16: return run_moments<float, 16, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 32: return run_moments<float, 32, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 64: return run_moments<float, 64, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            }
        } else {
            switch (pl.L) {
            case 1: return run_moments<float, 1, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 2: return run_moments<float, 2, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 4: return run_moments<float, 4, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 8: return run_moments<float, 8, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 16: return run_moments<float, 16, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 32: return run_moments<float, 32, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            }
        }
    }
    return fail(TBK_ERR_UNSUPPORTED, "no kernel for R = %d", R);
}

// r[i][v] = the seeded phase of output i R + v (caller's atom order).
template <class VT>
__global__ void k_random_phase(uint64_t seed, int64_t n, int32_t R, VT *__restrict__ r) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * R) return;
    double c, sn;
    seeded_phase(seed, (uint64_t)idx, c, sn);
    r[2 * idx] = (VT)c;
    r[2 * idx + 1] = (VT)sn;
}

tbk_status check_moment_args(const tbk_ham *h, const KpmPlan &pl, const double *a, const double *b,
                             const void *r, void *work, int64_t work_bytes, double *mu) {
    TBK_CHECK(a && b && (r || pl.seeded) && work && mu, TBK_ERR_INVALID_ARG, "NULL argument");
    TBK_CHECK(h->n_seg == 1, TBK_ERR_UNSUPPORTED, "stacked systems go through kpm_moments_batched");
    TBK_CHECK(std::isfinite(a[0]) && std::isfinite(b[0]), TBK_ERR_NOT_FINITE, "a or b is not finite");
    TBK_CHECK(a[0] > 0, TBK_ERR_INVALID_ARG, "a = %g must be positive", a[0]);
    TBK_CHECK(work_bytes >= (int64_t)pl.total, TBK_ERR_BUFFER_TOO_SMALL,
              "work has %lld bytes, needs %lld", (long long)work_bytes, (long long)pl.total);
    TBK_CHECK(((uintptr_t)work & 255) == 0, TBK_ERR_INVALID_ARG, "work is not 256-byte aligned");
    TBK_CHECK(h->ptr && h->col && h->val && h->onsite, TBK_ERR_INVALID_ARG, "Hamiltonian array is NULL");
    return TBK_OK;
}

}  // namespace tbk

using namespace tbk;

extern "C" tbk_status kpm_default_config(const tbk_ham *h, int32_t R, int32_t precision, tbk_kpm_config *cfg) {
    clear_error();
    TBK_CHECK(cfg != nullptr, TBK_ERR_INVALID_ARG, "cfg is NULL");
    KpmPlan pl;
    tbk_status st = make_plan(h, R, 2, precision, nullptr, pl);
    if (st != TBK_OK) return st;
    *cfg = pl.cfg;
    return TBK_OK;
}

extern "C" tbk_status kpm_workspace_size(const tbk_ham *h, int32_t R, int32_t M, int32_t precision,
                                         int64_t *bytes) {
    return kpm_workspace_size_config(h, R, M, precision, nullptr, bytes);
}

extern "C" tbk_status kpm_workspace_size_config(const tbk_ham *h, int32_t R, int32_t M, int32_t precision,
                                                const tbk_kpm_config *cfg, int64_t *bytes) {
    clear_error();
    TBK_CHECK(bytes != nullptr, TBK_ERR_INVALID_ARG, "bytes is NULL");
    KpmPlan pl;
    tbk_status st = make_plan(h, R, M, precision, cfg, pl);
    if (st != TBK_OK) return st;
    *bytes = (int64_t)pl.total;
    return TBK_OK;
}

extern "C" tbk_status kpm_moments(const tbk_ham *h, const double *a, const double *b, const void *r,
                                  int32_t R, int32_t M, int32_t precision, void *work, int64_t work_bytes,
                                  double *mu, void *stream) {
    return kpm_moments_config(h, a, b, r, R, M, precision, nullptr, work, work_bytes, mu, stream);
}

extern "C" tbk_status kpm_moments_config(const tbk_ham *h, const double *a, const double *b, const void *r,
                                         int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                                         void *work, int64_t work_bytes, double *mu, void *stream) {
    clear_error();
    KpmPlan pl;
    tbk_status st = make_plan(h, R, M, precision, cfg, pl);
    if (st != TBK_OK) return st;
    st = check_moment_args(h, pl, a, b, r, work, work_bytes, mu);
    if (st != TBK_OK) return st;
    TBK_CHECK(pl.cfg.persistent == 0, TBK_ERR_INVALID_ARG, "the persistent launch is for kpm_moments_batched");
    return run_plan(h, pl, a[0], b[0], r, R, M, precision, static_cast<char *>(work), mu, as_stream(stream),
                    nullptr, nullptr);
}

extern "C" tbk_status kpm_moments_seeded(const tbk_ham *h, const double *a, const double *b, uint64_t seed,
                                         int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                                         void *work, int64_t work_bytes, double *mu, void *stream) {
    clear_error();
    KpmPlan pl;
    tbk_status st = make_plan(h, R, M, precision, cfg, pl);
    if (st != TBK_OK) return st;
    pl.seeded = true;
    pl.seed = seed;
    st = check_moment_args(h, pl, a, b, nullptr, work, work_bytes, mu);
    if (st != TBK_OK) return st;
    TBK_CHECK(pl.cfg.persistent == 0, TBK_ERR_INVALID_ARG, "the persistent launch is for kpm_moments_batched");
    return run_plan(h, pl, a[0], b[0], nullptr, R, M, precision, static_cast<char *>(work), mu, as_stream(stream),
                    nullptr, nullptr);
}

extern "C" tbk_status tbk_random_phase(uint64_t seed, int64_t n, int32_t R, int32_t precision, void *r,
                                       void *stream) {
    clear_error();
    TBK_CHECK(n >= 0 && R >= 1 && R <= 64, TBK_ERR_INVALID_ARG, "n = %lld, R = %d", (long long)n, R);
    TBK_CHECK(precision == TBK_PREC_F64 || precision == TBK_PREC_C32, TBK_ERR_INVALID_ARG, "bad precision");
    if (n == 0) return TBK_OK;
    TBK_CHECK(r != nullptr, TBK_ERR_INVALID_ARG, "r is NULL");
    hipStream_t s = as_stream(stream);
    const unsigned g = (unsigned)ceil_div(n * R, 256);
    if (precision == TBK_PREC_F64) k_random_phase<double><<<g, 256, 0, s>>>(seed, n, R, static_cast<double *>(r));
    else k_random_phase<float><<<g, 256, 0, s>>>(seed, n, R, static_cast<float *>(r));
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}
