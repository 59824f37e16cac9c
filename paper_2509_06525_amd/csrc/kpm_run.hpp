// Recurrence kernels and the driver of one run (T_0 .. T_{M-1} with fused
// moment sums, Sec. 2.4), templated on the vector type and the lane layout.
// Included by the kpm_inst_*.hip translation units, each of which instantiates
// run_moments_inst for some (VT, L, VPT), so that the many kernel variants
// compile in parallel.
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
#pragma once

#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kpm.hpp"
#include "kpm_dev.hpp"

namespace tbk {

namespace {

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

// r_int[i][v] = r[perm[i]][v] (v < R), 0 for padded vectors; block partials of
// |r|^2 (in the doubling layout, each followed by VPT zeros).  With `seeded`
// the phases are generated for atom perm[i] (output perm[i] R + v) instead of
// being read from r.  Rows are dealt to the first `blocks` workgroups (the
// blocks that own tiles), so the partition and the partial sums do not depend on
// how far the grid was rounded up for the XCD block order; the others write 0.
template <class VT, int L, int VPT, bool DBL>
__global__ __launch_bounds__(kThreads) void k_prepare(const VT *__restrict__ r, const int32_t *__restrict__ perm,
                                                      int64_t n_rows, int32_t R, int32_t Rp, int32_t seeded,
                                                      uint64_t seed, int64_t blocks, VT *__restrict__ r_int,
                                                      double *__restrict__ partial) {
    constexpr int RPB = kThreads / L;
    const int lr = threadIdx.x / L;
    const int vs = threadIdx.x % L;
    double acc[VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) acc[q] = 0.0;
    const int64_t i0 = blockIdx.x < blocks ? (int64_t)blockIdx.x * RPB + lr : n_rows;
    for (int64_t i = i0; i < n_rows; i += blocks * RPB) {
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
                                                           int32_t Rp, int64_t blocks, double *__restrict__ partial) {
    constexpr int RPB = kThreads / L;
    const int lr = threadIdx.x / L;
    const int vs = threadIdx.x % L;
    double acc[VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) acc[q] = 0.0;
    const int64_t i0 = blockIdx.x < blocks ? (int64_t)blockIdx.x * RPB + lr : n_rows;
    for (int64_t i = i0; i < n_rows; i += blocks * RPB) {
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

// Second level: mu[v][n] = sum over chunks of l1[n][v][c], in chunk order, for
// the moments n0 <= n < M.
__global__ void k_reduce_l2(const double *__restrict__ l1, int32_t R, int32_t M, int32_t n0, int32_t n_chunks,
                            double *__restrict__ mu) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)R * (M - n0)) return;
    const int64_t n = n0 + idx / R, v = idx % R;
    const double *p = l1 + (n * R + v) * n_chunks;
    double s = 0.0;
    for (int c = 0; c < n_chunks; ++c) s += p[c];
    mu[v * M + n] = s;
}

// flag = 1 if some |mu_n|, n0 <= n < M, exceeds mu_0 (1 + 1e-6) or is not
// finite.  A fresh run (n0 = 0) keeps mu_0 of every vector in mu0 for the
// runs that continue it; a continued run reads it from there.
__global__ void k_guard(const double *__restrict__ mu, int32_t R, int32_t M, int32_t n0, double *__restrict__ mu0,
                        int32_t *__restrict__ flag) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)R * (M - n0)) return;
    const int64_t v = idx / (M - n0), n = n0 + idx % (M - n0);
    const double m0 = n0 == 0 ? mu[v * M] : mu0[v];
    const double m = mu[v * M + n];
    if (n == 0) mu0[v] = m0;
    if (!(fabs(m) <= m0 * (1.0 + 1e-6))) atomicOr(flag, 1);
}

// x[0..n) = value (a kernel rather than a memset node, so the clears stay
// ordinary kernels under stream capture).
__global__ void k_fill_i32(int32_t *__restrict__ x, int32_t n, int32_t value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = value;
}

// Record of a completed run at the head of the workspace.
__global__ void k_store_state(KpmState st, KpmState *__restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = st;
}



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
    const int n_start = pl.n_start;   // 0, or >= 2 with T_{n_start-1}, T_{n_start-2} and r in the workspace
    KpmState *state = reinterpret_cast<KpmState *>(work + pl.off_state);
    double *mu0 = reinterpret_cast<double *>(work + pl.off_state + kStateMu0);
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

    // row 0 goes through the same partial slots as the steps (slot 0 of the first batch);
    // a continued run starts with the step n_start in slot 0
    if (pair)
        k_pair_overlap<VT, L, VPT><<<(unsigned)pl.G, kThreads, 0, s>>>(left, start, h->n_rows, pl.Rp, pl.G_real,
                                                                       part);
    else if (n_start == 0)
        k_prepare<VT, L, VPT, DBL><<<(unsigned)pl.G, kThreads, 0, s>>>(r, h->perm, h->n_rows, R, pl.Rp,
                                                                        pl.seeded ? 1 : 0, pl.seed, pl.G_real,
                                                                        r_int, part);
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

    StepTimer &timer = step_timer();
    const bool timed = timer.on && !pair;
    bool open = false;      // a timed stretch of step launches is open
    if (timed) timer.used = 0;
    int batch0 = n_start;   // first row index of the pending batch
    for (int n = n_start > 0 ? n_start : 1; n < Mr; ++n) {
        if (n - batch0 == K) {
            if (open) { TBK_HIP(timer.mark(s)); open = false; }
            reduce(batch0, K);
            batch0 = n;
        }
        if (timed && !open) { TBK_HIP(timer.mark(s)); open = true; }
        if (timed) ++timer.launches;
        sp.partial = part + (int64_t)(n - batch0) * pstride;
        if (n == 1) {            // T_1 = Ht T_0 into TB
            sp.tcur = t0; sp.tprev = nullptr; sp.tnext = TB; sa.c1 = (VT)(1.0 / a);
        } else if (n == 2) {     // T_2 = 2 Ht T_1 - T_0 into TA
            sp.tcur = TB; sp.tprev = t0; sp.tnext = TA; sa.c1 = (VT)(2.0 / a);
        } else {                 // T_n overwrites T_{n-2} in place (odd n in TB, even n in TA)
            VT *cur = (n & 1) ? TA : TB;
            VT *old = (n & 1) ? TB : TA;
            sp.tcur = cur; sp.tprev = old; sp.tnext = old; sa.c1 = (VT)(2.0 / a);
        }
        if (pl.block) {
            tbk_status st = launch_step_block<VT>(pl, n == 1, diag, s, sp, sa);
            if (st != TBK_OK) return st;
        } else {
            launch_step<VT, L, VPT>(pl, n == 1, diag, s, sp, sa);
        }
    }
    if (open) TBK_HIP(timer.mark(s));
    reduce(batch0, Mr - batch0);
    TBK_HIP(hipGetLastError());
    const int64_t nm = (int64_t)R * M;
    if constexpr (DBL) {
        k_reduce_l2<<<(unsigned)ceil_div((int64_t)Rv * Mr, 256), 256, 0, s>>>(l1, Rv, Mr, 0, pl.n_chunks, raw);
        TBK_HIP(hipGetLastError());
        k_doubling_combine<<<(unsigned)ceil_div(nm, 256), 256, 0, s>>>(raw, Mr - 1, VPT, R, M, mu);
    } else {
        const int64_t nw = (int64_t)R * (M - n_start);
        k_reduce_l2<<<(unsigned)ceil_div(nw, 256), 256, 0, s>>>(l1, R, M, n_start, pl.n_chunks, mu);
    }
    TBK_HIP(hipGetLastError());
    if (pair) return TBK_OK;     // no guard: |mu_n| <= mu_0 holds only for left = start
    k_fill_i32<<<1, 64, 0, s>>>(flag, 1, 0);
    if constexpr (DBL) {
        k_guard<<<(unsigned)ceil_div(nm, 256), 256, 0, s>>>(mu, R, M, 0, mu0, flag);
    } else {
        const int64_t nw = (int64_t)R * (M - n_start);
        k_guard<<<(unsigned)ceil_div(nw, 256), 256, 0, s>>>(mu, R, M, n_start, mu0, flag);
    }
    KpmState rec{};
    rec.magic = DBL ? 0 : kStateMagic;    // the doubling form keeps no state to continue from
    rec.n_rows = h->n_rows;
    rec.n_entries = h->n_entries;
    rec.R = R;
    rec.precision = sizeof(VT) == sizeof(double) ? TBK_PREC_F64 : TBK_PREC_C32;
    rec.fmt = h->fmt;
    rec.next_n = M;
    rec.a = a;
    rec.b = b;
    k_store_state<<<1, 64, 0, s>>>(rec, state);
    TBK_HIP(hipGetLastError());
    int32_t hflag = 0;
    TBK_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    if (timed) TBK_HIP(timer.collect());
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

template <class VT, int L, int VPT>
tbk_status run_moments_inst(const tbk_ham *h, const KpmPlan &pl, double a, double b, const VT *r, int32_t R,
                            int32_t M, char *work, double *mu, hipStream_t s, const VT *start, const VT *left) {
    return run_moments<VT, L, VPT>(h, pl, a, b, r, R, M, work, mu, s, start, left);
}

}  // namespace tbk
