// Chebyshev moments of many stacked structures in one recurrence launch per step.
//
// Each structure (segment) s owns the row range [seg_rows[s], seg_rows[s+1]) of
// the stacked Hamiltonian and has its own scale a_s and shift b_s.  Rows are
// cut into tiles of 256 / L rows that never straddle two segments (the last
// tile of a segment is partial); a tile table (first row, segment) drives the
// launch, so one launch advances every structure by one step.  Each tile's
// block writes one FP64 partial per vector; every few steps a reduction
// kernel sums each segment's tile partials in tile order (bitwise
// reproducible), giving mu[s][v][n].
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "common.hpp"
#include "kpm.hpp"
#include "kpm_dev.hpp"

namespace tbk {

namespace {

constexpr size_t kSegPartialBudget = 256ull << 20;
constexpr int kPersistMaxPerCU = 8;   // co-resident workgroups per CU planned for

// Poll limit of the persistent team barrier (about 2^26 polls of ~100 cycles,
// seconds); TBKPM_BARRIER_SPIN_LIMIT overrides it (tests force a timeout).
int64_t barrier_spin_limit() {
    const char *e = std::getenv("TBKPM_BARRIER_SPIN_LIMIT");
    if (e) {
        const long long v = std::atoll(e);
        if (v >= 1) return v;
    }
    return (int64_t)1 << 26;
}

// tile_row0[t], tile_seg[t] for the tiles of segment s (one block per segment).
__global__ void k_tile_table(const int64_t *__restrict__ seg_rows, const int64_t *__restrict__ tile_off, int32_t rpb,
                             int64_t *__restrict__ tile_row0, int32_t *__restrict__ tile_seg) {
    const int s = blockIdx.x;
    for (int64_t t = tile_off[s] + threadIdx.x; t < tile_off[s + 1]; t += blockDim.x) {
        tile_row0[t] = seg_rows[s] + (t - tile_off[s]) * rpb;
        tile_seg[t] = s;
    }
}

template <class VT> struct SegStep {
    const int64_t *ptr;
    const int32_t *col;
    const VT *val;
    const VT *onsite;        // may be null
    const VT *tcur;
    const VT *tprev;
    VT *tnext;
    const VT *r;
    double *partial;         // [n_tiles][Rp] of this moment
    const int64_t *tile_row0;
    const int32_t *tile_seg;
    const int64_t *seg_rows;
    const VT *c1;            // per segment: 1/a (first step) or 2/a
    const VT *shift;         // per segment: b
    int64_t n_tiles;
    int32_t log2_slice;
    int32_t Rp;
    int32_t tiles_per_block;
    int32_t xcd_remap;       // grid is a multiple of the XCD count when set
};

// One row of tile t for this thread: T_{n+1} of the row and its overlap with
// r added to acc.  Rows past the end of the tile's segment are clamped to the
// segment's last row for their loads and masked for the rest.
template <class VT, int L, int VPT, bool FIRST, bool DIAG, bool NT, int W>
__device__ __forceinline__ void seg_tile_row(const SegStep<VT> &a, int64_t t, double (&acc)[VPT]) {
    constexpr int KU = W > 0 ? W : 4;
    const int lr = threadIdx.x / L;
    const int vs = threadIdx.x % L;
    const int voff = vs * VPT;
    const int Rp = a.Rp;
    const int64_t smask = ((int64_t)1 << a.log2_slice) - 1;
    const int64_t stride = smask + 1;
    const int sg = a.tile_seg[t];
    const int64_t row_end = a.seg_rows[sg + 1];
    const int64_t iu = a.tile_row0[t] + lr;
    const bool ok = iu < row_end;
    const int64_t i = min(iu, row_end - 1);
    const int64_t off = 2 * (i * Rp + voff);
    const int64_t sl = i >> a.log2_slice;
    const int64_t p0 = a.ptr[sl], p1 = a.ptr[sl + 1];
    const int64_t base = p0 + (i & smask);
    const int w = W > 0 ? W : (int)((p1 - p0) >> a.log2_slice);
    const VT c1 = a.c1[sg];
    Pack<VT, VPT> pv, rv;
    VT dg = 0;
    if constexpr (!FIRST) pv = load_pack<NT, VT, VPT>(a.tprev + off);
    rv = load_pack<NT, VT, VPT>(a.r + off);
    if constexpr (DIAG) dg = (a.onsite ? ld<NT>(a.onsite + i) : (VT)0) - a.shift[sg];
    Pack<VT, VPT> y;
#pragma unroll
    for (int q = 0; q < VPT; ++q) { y.re[q] = 0; y.im[q] = 0; }
    for (int k0 = 0; k0 < w; k0 += KU) {
        int32_t c[KU];
        VT h[KU];
#pragma unroll
        for (int k = 0; k < KU; ++k) {
            if constexpr (W > 0) {
                c[k] = ld<NT>(a.col + base + k * stride);
                h[k] = ld<NT>(a.val + base + k * stride);
            } else {
                const int kk = min(k0 + k, w - 1);
                c[k] = ld<NT>(a.col + base + kk * stride);
                h[k] = (k0 + k < w) ? ld<NT>(a.val + base + kk * stride) : (VT)0;
            }
        }
        Pack<VT, VPT> x[KU];
#pragma unroll
        for (int k = 0; k < KU; ++k) x[k] = load_pack<false, VT, VPT>(a.tcur + 2 * ((int64_t)c[k] * Rp + voff));
#pragma unroll
        for (int k = 0; k < KU; ++k)
#pragma unroll
            for (int q = 0; q < VPT; ++q) { y.re[q] += h[k] * x[k].re[q]; y.im[q] += h[k] * x[k].im[q]; }
    }
    if constexpr (DIAG) {
        Pack<VT, VPT> x = load_pack<false, VT, VPT>(a.tcur + off);
#pragma unroll
        for (int q = 0; q < VPT; ++q) { y.re[q] += dg * x.re[q]; y.im[q] += dg * x.im[q]; }
    }
    Pack<VT, VPT> o;
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
        if constexpr (FIRST) { o.re[q] = c1 * y.re[q]; o.im[q] = c1 * y.im[q]; }
        else { o.re[q] = c1 * y.re[q] - pv.re[q]; o.im[q] = c1 * y.im[q] - pv.im[q]; }
    }
    if (ok) {
        store_pack<NT, VT, VPT>(a.tnext + off, o);
#pragma unroll
        for (int q = 0; q < VPT; ++q)
            acc[q] += (double)rv.re[q] * (double)o.re[q] + (double)rv.im[q] * (double)o.im[q];
    }
}

// One step for every segment: logical block b handles tiles_per_block
// consecutive tiles of the table and writes one partial per tile.  With
// xcd_remap each XCD sweeps a contiguous range of tiles, so the neighbour rows
// a tile gathers are mostly in that XCD's own L2; blocks past the last tile
// (grid rounded up to the XCD count) do nothing.
template <class VT, int L, int VPT, bool FIRST, bool DIAG, bool NT, int W>
__global__ __launch_bounds__(kThreads) void k_cheb_step_seg(SegStep<VT> a) {
    const int64_t t0 = logical_block(a.xcd_remap) * a.tiles_per_block;
    const int64_t t1 = min(t0 + a.tiles_per_block, a.n_tiles);
    for (int64_t t = t0; t < t1; ++t) {
        double acc[VPT];
#pragma unroll
        for (int q = 0; q < VPT; ++q) acc[q] = 0.0;
        seg_tile_row<VT, L, VPT, FIRST, DIAG, NT, W>(a, t, acc);
        block_reduce_store<L, VPT>(acc, a.partial, t);
        __syncthreads();   // the reduction's LDS is reused by the next tile
    }
}

// Persistent form: one launch runs all M - 1 steps.  Structure s is served by
// a team of workgroups [boff[s], boff[s+1]); each member owns a contiguous
// range of the structure's tiles and writes one partial per step
// (bpart[n][block][v]).  After each step the team meets at a barrier: a
// monotone counter per structure in global memory, incremented once per
// member and step, with agent-scope fences on both sides.  The wait is
// bounded: past `spin_limit` polls, or when another block has raised the
// abort flag, the block raises the flag and leaves, so every wave exits.
struct PersistArgs {
    const int32_t *block_seg;   // [G] structure of each workgroup
    const int64_t *boff;        // [n_seg + 1] team block ranges
    const int64_t *tile_off;    // [n_seg + 1] tile ranges
    double *bpart;              // [M][G][Rp]
    uint32_t *bar;              // [n_seg] step counters (zero at launch)
    int32_t *abort_flag;        // 0 at launch
    int32_t M;
    int64_t spin_limit;
};

template <class VT> struct PersistBufs {
    VT *r_int, *TA, *TB;
    const VT *c1f, *c1;
};

template <class VT, int L, int VPT, bool DIAG, bool NT, int W>
__global__ __launch_bounds__(kThreads) void k_cheb_persistent(SegStep<VT> a, PersistBufs<VT> bufs, PersistArgs pa) {
    __shared__ int32_t s_abort;
    const int64_t b = blockIdx.x;
    const int sg = pa.block_seg[b];
    const int64_t k = pa.boff[sg + 1] - pa.boff[sg], j = b - pa.boff[sg];
    const int64_t T0 = pa.tile_off[sg], Ts = pa.tile_off[sg + 1] - T0;
    const int64_t t0 = T0 + (Ts * j) / k, t1 = T0 + (Ts * (j + 1)) / k;
    const int64_t G = gridDim.x;
    for (int n = 1; n < pa.M; ++n) {
        SegStep<VT> st = a;
        if (n == 1) { st.tcur = bufs.r_int; st.tprev = nullptr; st.tnext = bufs.TB; st.c1 = bufs.c1f; }
        else if (n == 2) { st.tcur = bufs.TB; st.tprev = bufs.r_int; st.tnext = bufs.TA; st.c1 = bufs.c1; }
        else {
            VT *cur = (n & 1) ? bufs.TA : bufs.TB;
            VT *old = (n & 1) ? bufs.TB : bufs.TA;
            st.tcur = cur; st.tprev = old; st.tnext = old; st.c1 = bufs.c1;
        }
        double acc[VPT];
#pragma unroll
        for (int q = 0; q < VPT; ++q) acc[q] = 0.0;
        for (int64_t t = t0; t < t1; ++t) {
            if (n == 1) seg_tile_row<VT, L, VPT, true, DIAG, NT, W>(st, t, acc);
            else seg_tile_row<VT, L, VPT, false, DIAG, NT, W>(st, t, acc);
        }
        block_reduce_store<L, VPT>(acc, pa.bpart + ((int64_t)n * G) * a.Rp, b);
        if (n + 1 == pa.M) break;
        // team barrier
        __syncthreads();
        if (threadIdx.x == 0) {
            s_abort = 0;
            __threadfence();
            atomicAdd(&pa.bar[sg], 1u);
            const uint32_t target = (uint32_t)((int64_t)n * k);
            int64_t spins = 0;
            while (__hip_atomic_load(&pa.bar[sg], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (++spins > pa.spin_limit ||
                    __hip_atomic_load(pa.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    atomicOr(pa.abort_flag, 1);
                    s_abort = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __threadfence();
        }
        __syncthreads();
        if (s_abort) return;
    }
}

// mu[s][v][n] = sum over the team blocks of s of bpart[n][b][v], in block
// order; grid = (n_seg, ceil(M / 64)), one thread per (moment, vector).
__global__ void k_reduce_persistent(const double *__restrict__ bpart, int64_t G, const int64_t *__restrict__ boff,
                                    int32_t Rp, int32_t R, int32_t M, double *__restrict__ mu) {
    const int s = blockIdx.x;
    const int idx = R + blockIdx.y * blockDim.x + threadIdx.x;     // moments n >= 1
    if (idx >= M * R) return;
    const int n = idx / R, v = idx % R;
    double acc = 0.0;
    for (int64_t b = boff[s]; b < boff[s + 1]; ++b) acc += bpart[((int64_t)n * G + b) * Rp + v];
    mu[((int64_t)s * R + v) * M + n] = acc;
}

// r_int[i][v] = r[perm[i]][v] (v < R, zero for padded vectors) and the tile
// partials of |r|^2; one tile per block.
template <class VT, int L, int VPT>
__global__ __launch_bounds__(kThreads) void k_prepare_seg(const VT *__restrict__ r, const int32_t *__restrict__ perm,
                                                          const int64_t *__restrict__ tile_row0,
                                                          const int32_t *__restrict__ tile_seg,
                                                          const int64_t *__restrict__ seg_rows, int32_t R,
                                                          int32_t Rp, VT *__restrict__ r_int,
                                                          double *__restrict__ partial) {
    const int64_t t = blockIdx.x;
    const int lr = threadIdx.x / L, vs = threadIdx.x % L;
    const int64_t i = tile_row0[t] + lr;
    double acc[VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) acc[q] = 0.0;
    if (i < seg_rows[tile_seg[t] + 1]) {
        const int64_t src = perm[i];
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int v = vs * VPT + q;
            VT re = 0, im = 0;
            if (v < R) { re = r[2 * (src * R + v)]; im = r[2 * (src * R + v) + 1]; }
            r_int[2 * (i * Rp + v)] = re;
            r_int[2 * (i * Rp + v) + 1] = im;
            acc[q] = (double)re * (double)re + (double)im * (double)im;
        }
    }
    block_reduce_store<L, VPT>(acc, partial, t);
}

// mu[s][v][n0 + k] = sum over the tiles of segment s of partial[k][t][v], in
// tile order; grid = (n_seg, count).
__global__ __launch_bounds__(kThreads) void k_reduce_seg(const double *__restrict__ partial, int64_t n_tiles,
                                                         const int64_t *__restrict__ tile_off, int32_t Rp,
                                                         int32_t R, int32_t M, int32_t n0, double *__restrict__ mu) {
    __shared__ double red[kThreads];
    const int s = blockIdx.x, k = blockIdx.y;
    const int v = threadIdx.x % Rp, j = threadIdx.x / Rp, groups = kThreads / Rp;
    const double *p = partial + (int64_t)k * n_tiles * Rp;
    double acc = 0.0;
    for (int64_t t = tile_off[s] + j; t < tile_off[s + 1]; t += groups) acc += p[t * Rp + v];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int g = groups / 2; g > 0; g >>= 1) {
        if (j < g) red[threadIdx.x] += red[threadIdx.x + g * Rp];
        __syncthreads();
    }
    if (j == 0 && v < R) mu[((int64_t)s * R + v) * M + n0 + k] = red[v];
}

// flag = 0 (a kernel, not a memset node, so the clear stays an ordinary kernel under capture).
__global__ void k_fill_flag(int32_t *__restrict__ flag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0;
}

__global__ void k_guard_seg(const double *__restrict__ mu, int64_t rows, int32_t M, int32_t *__restrict__ flag) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= rows * M) return;
    const int64_t sv = idx / M;
    const double m0 = mu[sv * M];
    if (!(fabs(mu[idx]) <= m0 * (1.0 + 1e-6))) atomicOr(flag, 1);
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SegPlan {
    KpmPlan base;                    // vector layout and launch shape
    int32_t n_seg = 0;
    int64_t n_tiles = 0;
    std::vector<int64_t> seg_rows;   // host copy
    std::vector<int64_t> tile_off;   // host [n_seg + 1]
    int K = 1;
    // persistent launch
    bool persistent = false;
    int64_t Gp = 0;                  // workgroups of the persistent launch
    std::vector<int64_t> boff;       // [n_seg + 1] team block ranges
    std::vector<int32_t> block_seg;  // [Gp]
    size_t off_bpart = 0, off_boff = 0, off_bseg = 0, off_bar = 0;
    size_t off_r = 0, off_a = 0, off_b = 0, off_part = 0, off_row0 = 0, off_tseg = 0, off_toff = 0,
           off_c1f = 0, off_c1 = 0, off_shift = 0, off_flag = 0, total = 0;
};

// Teams of the persistent launch: at most gmax workgroups, one team per
// structure with at least one member, sizes proportional to tile counts.
tbk_status partition_teams(SegPlan &sp, int64_t gmax) {
    int64_t G = std::min<int64_t>(gmax, std::max<int64_t>(sp.n_tiles, sp.n_seg));
    TBK_CHECK(sp.n_seg <= G, TBK_ERR_UNSUPPORTED,
              "persistent launch needs one workgroup per structure (%d structures, %lld workgroups)", sp.n_seg,
              (long long)G);
    sp.boff.assign(sp.n_seg + 1, 0);
    std::vector<int64_t> ks(sp.n_seg);
    int64_t used = 0;
    for (int g = 0; g < sp.n_seg; ++g) {
        const int64_t Ts = sp.tile_off[g + 1] - sp.tile_off[g];
        ks[g] = 1 + ((G - sp.n_seg) * Ts) / std::max<int64_t>(sp.n_tiles, 1);
        ks[g] = std::min<int64_t>(ks[g], Ts);
        used += ks[g];
    }
    sp.Gp = used;
    sp.block_seg.resize(sp.Gp);
    for (int g = 0; g < sp.n_seg; ++g) {
        sp.boff[g + 1] = sp.boff[g] + ks[g];
        for (int64_t b = sp.boff[g]; b < sp.boff[g + 1]; ++b) sp.block_seg[b] = g;
    }
    return TBK_OK;
}

tbk_status make_seg_plan(const tbk_ham *h, int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                         hipStream_t s, SegPlan &sp) {
    TBK_CHECK(h != nullptr, TBK_ERR_INVALID_ARG, "h is NULL");
    TBK_CHECK(h->n_seg >= 1, TBK_ERR_INVALID_ARG, "n_seg = %d", h->n_seg);
    TBK_CHECK(h->seg_rows != nullptr, TBK_ERR_INVALID_ARG, "h->seg_rows is NULL");
    tbk_status st = make_plan(h, R, M, precision, cfg, sp.base);
    if (st != TBK_OK) return st;
    TBK_CHECK(sp.base.cfg.doubling == 0, TBK_ERR_UNSUPPORTED, "the doubling identities are not offered for stacked structures");
    TBK_CHECK(!sp.base.block, TBK_ERR_UNSUPPORTED, "block Hamiltonians are not offered for stacked structures");
    TBK_CHECK(sp.base.cfg.uniform_values == 0 && sp.base.cfg.compact_columns == 0, TBK_ERR_UNSUPPORTED,
              "uniform_values and compact_columns are not offered for stacked structures");
    sp.n_seg = h->n_seg;
    sp.seg_rows.resize(sp.n_seg + 1);
    TBK_HIP(hipMemcpyAsync(sp.seg_rows.data(), h->seg_rows, sizeof(int64_t) * (sp.n_seg + 1), hipMemcpyDeviceToHost,
                           s));
    TBK_HIP(hipStreamSynchronize(s));
    TBK_CHECK(sp.seg_rows[0] == 0 && sp.seg_rows[sp.n_seg] == h->n_rows, TBK_ERR_INVALID_ARG,
              "segment rows do not cover [0, n_rows)");
    const int rpb = kThreads / sp.base.L;
    sp.tile_off.assign(sp.n_seg + 1, 0);
    for (int g = 0; g < sp.n_seg; ++g) {
        const int64_t rows = sp.seg_rows[g + 1] - sp.seg_rows[g];
        TBK_CHECK(rows >= 1, TBK_ERR_INVALID_ARG, "segment %d is empty", g);
        sp.tile_off[g + 1] = sp.tile_off[g] + ceil_div(rows, rpb);
    }
    sp.n_tiles = sp.tile_off[sp.n_seg];
    const int64_t G = ceil_div(sp.n_tiles, sp.base.cfg.tiles_per_block);
    TBK_CHECK(G + kNumXcd < (int64_t)INT32_MAX && sp.n_tiles < (int64_t)INT32_MAX, TBK_ERR_UNSUPPORTED, "too many tiles");
    const size_t per_step = (size_t)sp.n_tiles * sp.base.Rp * sizeof(double);
    sp.K = (int)std::max<size_t>(1, std::min<size_t>({kSegPartialBudget / per_step, (size_t)64, (size_t)M}));
    const size_t vb = sp.base.vec_bytes, ve = sp.base.elem;
    sp.off_r = 0;
    sp.off_a = vb;
    sp.off_b = 2 * vb;
    sp.off_part = 3 * vb;
    sp.off_row0 = sp.off_part + a256((size_t)sp.K * per_step);
    sp.off_tseg = sp.off_row0 + a256(sizeof(int64_t) * sp.n_tiles);
    sp.off_toff = sp.off_tseg + a256(sizeof(int32_t) * sp.n_tiles);
    sp.off_c1f = sp.off_toff + a256(sizeof(int64_t) * (sp.n_seg + 1));
    sp.off_c1 = sp.off_c1f + a256(ve * sp.n_seg);
    sp.off_shift = sp.off_c1 + a256(ve * sp.n_seg);
    sp.off_flag = sp.off_shift + a256(ve * sp.n_seg);
    sp.total = sp.off_flag + 256;
    sp.persistent = sp.base.cfg.persistent != 0;
    if (sp.persistent) {
        int dev = 0, cus = 0;
        TBK_HIP(hipGetDevice(&dev));
        TBK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        // up to eight co-resident 256-thread workgroups per CU; the launch
        // re-partitions for what the kernel's occupancy allows (the
        // cooperative launch also refuses a grid that cannot be resident)
        st = partition_teams(sp, (int64_t)cus * kPersistMaxPerCU);
        if (st != TBK_OK) return st;
        const size_t bpart = (size_t)M * sp.Gp * sp.base.Rp * sizeof(double);
        TBK_CHECK(bpart <= (4ull << 30), TBK_ERR_UNSUPPORTED, "persistent partials would need %zu bytes", bpart);
        sp.off_bpart = sp.total;
        sp.off_boff = sp.off_bpart + a256(bpart);
        sp.off_bseg = sp.off_boff + a256(sizeof(int64_t) * (sp.n_seg + 1));
        sp.off_bar = sp.off_bseg + a256(sizeof(int32_t) * sp.Gp);
        sp.total = sp.off_bar + a256(sizeof(uint32_t) * sp.n_seg + 64);
    }
    return TBK_OK;
}

template <class VT, int L, int VPT, bool FIRST, bool DIAG>
void launch_seg(const SegPlan &sp, unsigned G, hipStream_t s, const SegStep<VT> &a) {
    const bool w3 = sp.base.uniform_width == 3;
    if (sp.base.cfg.nontemporal) {
        if (w3) k_cheb_step_seg<VT, L, VPT, FIRST, DIAG, true, 3><<<G, kThreads, 0, s>>>(a);
        else k_cheb_step_seg<VT, L, VPT, FIRST, DIAG, true, 0><<<G, kThreads, 0, s>>>(a);
    } else {
        if (w3) k_cheb_step_seg<VT, L, VPT, FIRST, DIAG, false, 3><<<G, kThreads, 0, s>>>(a);
        else k_cheb_step_seg<VT, L, VPT, FIRST, DIAG, false, 0><<<G, kThreads, 0, s>>>(a);
    }
}

template <class VT, int L, int VPT>
tbk_status run_seg(const tbk_ham *h, const SegPlan &sp, const double *a, const double *b, const VT *r, int32_t R,
                   int32_t M, char *w, double *mu, hipStream_t s) {
    const int ns = sp.n_seg;
    VT *r_int = reinterpret_cast<VT *>(w + sp.off_r);
    VT *TA = reinterpret_cast<VT *>(w + sp.off_a);
    VT *TB = reinterpret_cast<VT *>(w + sp.off_b);
    double *part = reinterpret_cast<double *>(w + sp.off_part);
    int64_t *row0 = reinterpret_cast<int64_t *>(w + sp.off_row0);
    int32_t *tseg = reinterpret_cast<int32_t *>(w + sp.off_tseg);
    int64_t *toff = reinterpret_cast<int64_t *>(w + sp.off_toff);
    VT *c1f = reinterpret_cast<VT *>(w + sp.off_c1f);
    VT *c1 = reinterpret_cast<VT *>(w + sp.off_c1);
    VT *shift = reinterpret_cast<VT *>(w + sp.off_shift);
    int32_t *flag = reinterpret_cast<int32_t *>(w + sp.off_flag);
    const int Rp = sp.base.Rp;
    const int64_t T = sp.n_tiles;
    const int64_t pstride = T * Rp;

    std::vector<VT> h1f(ns), h1(ns), hs(ns);
    bool diag = h->has_onsite != 0;
    for (int g = 0; g < ns; ++g) {
        h1f[g] = (VT)(1.0 / a[g]);
        h1[g] = (VT)(2.0 / a[g]);
        hs[g] = (VT)b[g];
        if (b[g] != 0.0) diag = true;
    }
    TBK_HIP(hipMemcpyAsync(toff, sp.tile_off.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, s));
    TBK_HIP(hipMemcpyAsync(c1f, h1f.data(), sizeof(VT) * ns, hipMemcpyHostToDevice, s));
    TBK_HIP(hipMemcpyAsync(c1, h1.data(), sizeof(VT) * ns, hipMemcpyHostToDevice, s));
    TBK_HIP(hipMemcpyAsync(shift, hs.data(), sizeof(VT) * ns, hipMemcpyHostToDevice, s));
    k_tile_table<<<ns, kThreads, 0, s>>>(h->seg_rows, toff, kThreads / L, row0, tseg);
    TBK_HIP(hipGetLastError());
    k_prepare_seg<VT, L, VPT><<<(unsigned)T, kThreads, 0, s>>>(r, h->perm, row0, tseg, h->seg_rows, R, Rp, r_int,
                                                               part);
    TBK_HIP(hipGetLastError());

    SegStep<VT> st{};
    st.ptr = h->ptr;
    st.col = h->col;
    st.val = static_cast<const VT *>(h->val);
    st.onsite = h->has_onsite ? static_cast<const VT *>(h->onsite) : nullptr;
    st.r = r_int;
    st.tile_row0 = row0;
    st.tile_seg = tseg;
    st.seg_rows = h->seg_rows;
    st.shift = shift;
    st.n_tiles = T;
    st.log2_slice = sp.base.log2_slice;
    st.Rp = Rp;
    st.tiles_per_block = sp.base.cfg.tiles_per_block;
    st.xcd_remap = sp.base.cfg.xcd_remap;
    if (sp.persistent) {
        // moment 0 from the tile partials of |r|^2
        {
            dim3 grid(ns, 1);
            k_reduce_seg<<<grid, kThreads, 0, s>>>(part, T, toff, Rp, R, M, 0, mu);
            TBK_HIP(hipGetLastError());
        }
        double *bpart = reinterpret_cast<double *>(w + sp.off_bpart);
        int64_t *boff = reinterpret_cast<int64_t *>(w + sp.off_boff);
        int32_t *bseg = reinterpret_cast<int32_t *>(w + sp.off_bseg);
        uint32_t *bar = reinterpret_cast<uint32_t *>(w + sp.off_bar);
        int32_t *abort_flag = reinterpret_cast<int32_t *>(bar + ns);
        TBK_HIP(hipMemsetAsync(bar, 0, sizeof(uint32_t) * ns + 64, s));
        PersistBufs<VT> bufs{r_int, TA, TB, c1f, c1};
        PersistArgs pa{bseg, boff, toff, bpart, bar, abort_flag, M, barrier_spin_limit()};
        void *args[] = {&st, &bufs, &pa};
        const bool w3 = sp.base.uniform_width == 3;
        const void *fn;
        if (sp.base.cfg.nontemporal)
            fn = diag ? (w3 ? (const void *)k_cheb_persistent<VT, L, VPT, true, true, 3>
                            : (const void *)k_cheb_persistent<VT, L, VPT, true, true, 0>)
                      : (w3 ? (const void *)k_cheb_persistent<VT, L, VPT, false, true, 3>
                            : (const void *)k_cheb_persistent<VT, L, VPT, false, true, 0>);
        else
            fn = diag ? (w3 ? (const void *)k_cheb_persistent<VT, L, VPT, true, false, 3>
                            : (const void *)k_cheb_persistent<VT, L, VPT, true, false, 0>)
                      : (w3 ? (const void *)k_cheb_persistent<VT, L, VPT, false, false, 3>
                            : (const void *)k_cheb_persistent<VT, L, VPT, false, false, 0>);
        int occ = 0, dev = 0, cus = 0;
        TBK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kThreads, 0));
        TBK_CHECK(occ >= 1, TBK_ERR_UNSUPPORTED, "the persistent kernel does not fit on a CU");
        TBK_HIP(hipGetDevice(&dev));
        TBK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        // the workspace was laid out for kPersistMaxPerCU workgroups per CU; fewer fit in the same space
        SegPlan tp = sp;
        tbk_status pst = partition_teams(tp, (int64_t)cus * std::min(occ, kPersistMaxPerCU));
        if (pst != TBK_OK) return pst;
        TBK_CHECK(tp.Gp <= sp.Gp, TBK_ERR_DEVICE, "persistent team layout exceeds its workspace");
        TBK_HIP(hipMemcpyAsync(boff, tp.boff.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, s));
        TBK_HIP(hipMemcpyAsync(bseg, tp.block_seg.data(), sizeof(int32_t) * tp.Gp, hipMemcpyHostToDevice, s));
        TBK_HIP(hipLaunchCooperativeKernel(fn, dim3((unsigned)tp.Gp), dim3(kThreads), args, 0, s));
        dim3 rg(ns, (unsigned)ceil_div((int64_t)(M - 1) * R, 256));
        k_reduce_persistent<<<rg, 256, 0, s>>>(bpart, tp.Gp, boff, Rp, R, M, mu);
        TBK_HIP(hipStreamSynchronize(s));    // the host team tables must outlive their transfers
        TBK_HIP(hipGetLastError());
        int32_t habort = 0;
        TBK_HIP(hipMemcpyAsync(&habort, abort_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TBK_HIP(hipStreamSynchronize(s));
        TBK_CHECK(habort == 0, TBK_ERR_DEVICE, "persistent recurrence: a team barrier timed out");
    } else {
    int64_t Gt = ceil_div(T, sp.base.cfg.tiles_per_block);
    Gt = ceil_div(Gt, xcd_grid_multiple(st.xcd_remap)) * xcd_grid_multiple(st.xcd_remap);
    const unsigned G = (unsigned)Gt;
    const int K = sp.K;
    auto reduce = [&](int n0, int count) {
        dim3 grid(ns, count);
        k_reduce_seg<<<grid, kThreads, 0, s>>>(part, T, toff, Rp, R, M, n0, mu);
    };
    StepTimer &timer = step_timer();
    bool open = false;      // a timed stretch of step launches is open
    if (timer.on) timer.used = 0;
    int batch0 = 0;
    for (int n = 1; n < M; ++n) {
        if (n - batch0 == K) {
            if (open) { TBK_HIP(timer.mark(s)); open = false; }
            reduce(batch0, K);
            batch0 = n;
        }
        if (timer.on && !open) { TBK_HIP(timer.mark(s)); open = true; }
        if (timer.on) ++timer.launches;
        st.partial = part + (int64_t)(n - batch0) * pstride;
        if (n == 1) {
            st.tcur = r_int; st.tprev = nullptr; st.tnext = TB; st.c1 = c1f;
        } else if (n == 2) {
            st.tcur = TB; st.tprev = r_int; st.tnext = TA; st.c1 = c1;
        } else {
            VT *cur = (n & 1) ? TA : TB;
            VT *old = (n & 1) ? TB : TA;
            st.tcur = cur; st.tprev = old; st.tnext = old;
        }
        if (n == 1) {
            if (diag) launch_seg<VT, L, VPT, true, true>(sp, G, s, st);
            else launch_seg<VT, L, VPT, true, false>(sp, G, s, st);
        } else {
            if (diag) launch_seg<VT, L, VPT, false, true>(sp, G, s, st);
            else launch_seg<VT, L, VPT, false, false>(sp, G, s, st);
        }
    }
    if (open) TBK_HIP(timer.mark(s));
    reduce(batch0, M - batch0);
    TBK_HIP(hipGetLastError());
    }
    k_fill_flag<<<1, 64, 0, s>>>(flag);
    const int64_t rows = (int64_t)ns * R;
    k_guard_seg<<<(unsigned)ceil_div(rows * M, 256), 256, 0, s>>>(mu, rows, M, flag);
    TBK_HIP(hipGetLastError());
    int32_t hflag = 0;
    TBK_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    if (step_timer().on) TBK_HIP(step_timer().collect());
    TBK_CHECK(hflag == 0, TBK_ERR_SPECTRUM, "a moment exceeds mu_0: some (a_s, b_s) does not bound its spectrum");
    return TBK_OK;
}

tbk_status dispatch_seg(const tbk_ham *h, const SegPlan &sp, const double *a, const double *b, const void *r,
                        int32_t R, int32_t M, int32_t precision, char *w, double *mu, hipStream_t s) {
    const int L = sp.base.L, VPT = sp.base.VPT;
    if (precision == TBK_PREC_F64) {
        const double *rr = static_cast<const double *>(r);
        switch (L) {
        case 1: return run_seg<double, 1, 1>(h, sp, a, b, rr, R, M, w, mu, s);
        case 2: return run_seg<double, 2, 1>(h, sp, a, b, rr, R, M, w, mu, s);
        case 4: return run_seg<double, 4, 1>(h, sp, a, b, rr, R, M, w, mu, s);
        case 8: return run_seg<double, 8, 1>(h, sp, a, b, rr, R, M, w, mu, s);
        case 16: return run_seg<double, 16, 1>(h, sp, a, b, rr, R, M, w, mu, s);
        case 32: return run_seg<double, 32, 1>(h, sp, a, b, rr, R, M, w, mu, s);
        case 64: return run_seg<double, 64, 1>(h, sp, a, b, rr, R, M, w, mu, s);
        }
    } else {
        const float *rr = static_cast<const float *>(r);
        if (VPT == 1) {
            switch (L) {
            case 1: return run_seg<float, 1, 1>(h, sp, a, b, rr, R, M, w, mu, s);
            case 2: return run_seg<float, 2, 1>(h, sp, a, b, rr, R, M, w, mu, s);
            case 4: return run_seg<float, 4, 1>(h, sp, a, b, rr, R, M, w, mu, s);
            case 8: return run_seg<float, 8, 1>(h, sp, a, b, rr, R, M, w, mu, s);
            case 16: return run_seg<float, 16, 1>(h, sp, a, b, rr, R, M, w, mu, s);
            case 32: return run_seg<float, 32, 1>(h, sp, a, b, rr, R, M, w, mu, s);
            case 64: return run_seg<float, 64, 1>(h, sp, a, b, rr, R, M, w, mu, s);
            }
        } else {
            switch (L) {
            case 1: return run_seg<float, 1, 2>(h, sp, a, b, rr, R, M, w, mu, s);
            case 2: return run_seg<float, 2, 2>(h, sp, a, b, rr, R, M, w, mu, s);
            case 4: return run_seg<float, 4, 2>(h, sp, a, b, rr, R, M, w, mu, s);
            case 8: return run_seg<float, 8, 2>(h, sp, a, b, rr, R, M, w, mu, s);
            case 16: return run_seg<float, 16, 2>(h, sp, a, b, rr, R, M, w, mu, s);
            case 32: return run_seg<float, 32, 2>(h, sp, a, b, rr, R, M, w, mu, s);
            }
        }
    }
    return fail(TBK_ERR_UNSUPPORTED, "no kernel for R = %d", R);
}

}  // namespace

}  // namespace tbk

using namespace tbk;

extern "C" tbk_status kpm_workspace_size_batched(const tbk_ham *h, int32_t R, int32_t M, int32_t precision,
                                                 const tbk_kpm_config *cfg, int64_t *bytes, void *stream) {
    clear_error();
    TBK_CHECK(bytes != nullptr, TBK_ERR_INVALID_ARG, "bytes is NULL");
    SegPlan sp;
    tbk_status st = make_seg_plan(h, R, M, precision, cfg, as_stream(stream), sp);
    if (st != TBK_OK) return st;
    *bytes = (int64_t)sp.total;
    return TBK_OK;
}

extern "C" tbk_status kpm_moments_batched(const tbk_ham *h, const double *a, const double *b, const void *r,
                                          int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                                          void *work, int64_t work_bytes, double *mu, void *stream) {
    clear_error();
    hipStream_t s = as_stream(stream);
    SegPlan sp;
    tbk_status st = make_seg_plan(h, R, M, precision, cfg, s, sp);
    if (st != TBK_OK) return st;
    TBK_CHECK(a && b && r && work && mu, TBK_ERR_INVALID_ARG, "NULL argument");
    for (int g = 0; g < sp.n_seg; ++g) {
        TBK_CHECK(std::isfinite(a[g]) && std::isfinite(b[g]), TBK_ERR_NOT_FINITE, "a or b of segment %d is not finite",
                  g);
        TBK_CHECK(a[g] > 0, TBK_ERR_INVALID_ARG, "a[%d] = %g must be positive", g, a[g]);
    }
    TBK_CHECK(work_bytes >= (int64_t)sp.total, TBK_ERR_BUFFER_TOO_SMALL, "work has %lld bytes, needs %lld",
              (long long)work_bytes, (long long)sp.total);
    TBK_CHECK(((uintptr_t)work & 255) == 0, TBK_ERR_INVALID_ARG, "work is not 256-byte aligned");
    TBK_CHECK(h->ptr && h->col && h->val && h->onsite && h->perm, TBK_ERR_INVALID_ARG, "Hamiltonian array is NULL");
    return dispatch_seg(h, sp, a, b, r, R, M, precision, static_cast<char *>(work), mu, s);
}
