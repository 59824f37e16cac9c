// Chebyshev recurrence step on a block Hamiltonian: NORB orbitals per atom
// (4: s, px, py, pz; 9: s, p and the five d), one NORB x NORB block per bond
// (the Slater-Koster blocks of the multi-orbital models), stored as a sliced
// ELL over atoms:
//   ptr[s]                      first block of atom slice s (slice = h->slice atoms),
//   col[q]                      neighbour atom row of block q (own row on padding),
//   val[NORB^2 q + NORB a + b]  <orbital a of the row atom| H |orbital b of col[q]>.
// Vectors keep the one-orbital layout over orbital rows NORB i + a, [rows][R_pad].
//
// A thread owns one orbital row (NORB i + a) and VPT vectors, like the
// one-orbital kernel.  Per neighbour block it reads the block's column (shared
// by the NORB rows of the atom: one address per atom in a wavefront), its row
// a of NORB values (one 16 B or 32 B load for NORB = 4), and the NORB orbital
// rows of the neighbour's T_n, which are contiguous.  Against the scalar
// expansion of the same matrix (NORB columns and NORB values per neighbour and
// orbital row) this reads 1/NORB of the column bytes and column loads.
#include <type_traits>

#include "common.hpp"
#include "kpm.hpp"
#include "kpm_dev.hpp"

namespace tbk {
namespace {

// Row a of a block: NORB values (vector loads for NORB = 4, whose rows are
// 16 B or 32 B aligned; scalar loads for NORB = 9).
template <int NORB, bool NT, class VT>
__device__ __forceinline__ void load_row(const VT *p, VT (&h)[NORB]) {
    if constexpr (NORB != 4) {
#pragma unroll
        for (int b = 0; b < NORB; ++b) h[b] = ld<NT>(p + b);
    } else if constexpr (sizeof(VT) == 4) {
        const f4v v = ld<NT>(reinterpret_cast<const f4v *>(p));
        h[0] = v.x; h[1] = v.y; h[2] = v.z; h[3] = v.w;
    } else {
        const d2v v0 = ld<NT>(reinterpret_cast<const d2v *>(p));
        const d2v v1 = ld<NT>(reinterpret_cast<const d2v *>(p) + 1);
        h[0] = v0.x; h[1] = v0.y; h[2] = v1.x; h[3] = v1.y;
    }
}

// KB neighbour blocks are loaded before any is used (three: the honeycomb's
// nearest neighbours in one batch); blocks past the atom's width are clamped
// to its last block and weighted by zero.
template <class VT, int NORB, int L, int VPT, bool FIRST, bool DIAG, bool NT, bool DBL>
__global__ __launch_bounds__(kThreads) void k_cheb_step_blk(
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ bcol, const VT *__restrict__ bval,
    const VT *__restrict__ onsite, const VT *__restrict__ tcur, const VT *tprev, VT *tnext,
    const VT *__restrict__ r, double *__restrict__ partial, StepScalars<VT> a) {
    constexpr int RPB = kThreads / L;   // orbital rows per tile
    constexpr int KB = 3;
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

    constexpr int NA = DBL ? 2 * VPT : VPT;
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;

    for (int64_t t = t0; t < t1; ++t) {
        const int64_t iu = t * RPB + lr;
        const bool ok = iu <= last;
        const int64_t i = min(iu, last);            // orbital row
        const int64_t at = i / NORB;                 // atom row
        const int orb = (int)(i - at * NORB);
        const int64_t off = 2 * (i * Rp + voff);
        const int64_t sl = at >> a.log2_slice;
        const int64_t p0 = ptr[sl], p1 = ptr[sl + 1];
        const int64_t base = p0 + (at & smask);
        const int w = (int)((p1 - p0) >> a.log2_slice);

        Pack<VT, VPT> pv, rv;
        VT dg = 0;
        if constexpr (!FIRST) pv = load_pack<NT, VT, VPT>(tprev + off);
        if constexpr (DBL) rv = load_pack<false, VT, VPT>(tcur + off);
        else rv = load_pack<NT, VT, VPT>(r + off);
        if constexpr (DIAG) dg = (onsite ? ld<NT>(onsite + i) : (VT)0) - a.shift;

        Pack<VT, VPT> y;
#pragma unroll
        for (int q = 0; q < VPT; ++q) { y.re[q] = 0; y.im[q] = 0; }
        for (int k0 = 0; k0 < w; k0 += KB) {
            int32_t c[KB];
            VT h[KB][NORB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int kk = min(k0 + k, w - 1);
                const int64_t q = base + (int64_t)kk * stride;
                c[k] = ld<NT>(bcol + q);
                load_row<NORB, NT, VT>(bval + (int64_t)NORB * NORB * q + NORB * orb, h[k]);
                if (k0 + k >= w) {
#pragma unroll
                    for (int b = 0; b < NORB; ++b) h[k][b] = 0;
                }
            }
            Pack<VT, VPT> x[KB][NORB];
#pragma unroll
            for (int k = 0; k < KB; ++k)
#pragma unroll
                for (int b = 0; b < NORB; ++b)
                    x[k][b] = load_pack<false, VT, VPT>(tcur + 2 * (((int64_t)NORB * c[k] + b) * Rp + voff));
#pragma unroll
            for (int k = 0; k < KB; ++k)
#pragma unroll
                for (int b = 0; b < NORB; ++b)
#pragma unroll
                    for (int q = 0; q < VPT; ++q) {
                        y.re[q] += h[k][b] * x[k][b].re[q];
                        y.im[q] += h[k][b] * x[k][b].im[q];
                    }
        }
        if constexpr (DIAG) {
            const Pack<VT, VPT> x = load_pack<false, VT, VPT>(tcur + off);
#pragma unroll
            for (int q = 0; q < VPT; ++q) { y.re[q] += dg * x.re[q]; y.im[q] += dg * x.im[q]; }
        }
        Pack<VT, VPT> o;
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            if constexpr (FIRST) {
                o.re[q] = a.c1 * y.re[q];
                o.im[q] = a.c1 * y.im[q];
            } else {
                o.re[q] = a.c1 * y.re[q] - pv.re[q];
                o.im[q] = a.c1 * y.im[q] - pv.im[q];
            }
        }
        if (ok) {
            store_pack<NT, VT, VPT>(tnext + off, o);
#pragma unroll
            for (int q = 0; q < VPT; ++q) {
                const double cr = (double)rv.re[q] * (double)o.re[q] + (double)rv.im[q] * (double)o.im[q];
                if constexpr (DBL) {
                    acc[q] += (double)o.re[q] * (double)o.re[q] + (double)o.im[q] * (double)o.im[q];
                    acc[VPT + q] += cr;
                } else {
                    acc[q] += cr;
                }
            }
        }
    }
    block_reduce_store<L, NA>(acc, partial, lb);
}

// Tiles from which the one-vector block kernels stage their rows by default
// (about eight workgroups per CU; fewer leave the barriers exposed).
constexpr int64_t kStageMinTiles = 2048;

// Last part of a one-vector step for the NORB rows of each atom of a tile
// (the thread's atom la, clamped atom row at): the tile's rows are one
// contiguous range, so T_{n-1}, r (T_n with the doubling identities) and the
// onsite energies are loaded, and T_{n+1} stored, through LDS as whole ranges;
// direct row accesses at a stride of NORB write every cache line several times
// in part.  y holds sum_q H_iq T_n(q) of the thread's rows.
template <class VT, int NORB, bool FIRST, bool DIAG, bool NT, bool DBL>
__device__ __forceinline__ void finish_rows_staged(const Pack<VT, 1> (&y)[NORB], const StepScalars<VT> &a, int64_t t,
                                                   int la, int64_t at, bool ok, const VT *__restrict__ onsite,
                                                   const VT *__restrict__ tcur, const VT *tprev, VT *tnext,
                                                   const VT *__restrict__ r, double (&acc)[DBL ? 2 : 1]) {
    constexpr int APB = kThreads;
    typedef std::conditional_t<sizeof(VT) == 4, f2v, d2v> C2;
    __shared__ C2 sbuf[NORB * kThreads];
    VT *sv = reinterpret_cast<VT *>(sbuf);
    const int64_t row0 = (int64_t)NORB * (t * APB);
    const int nrow = (int)min((int64_t)NORB * APB, a.n_rows - row0);
    const int mine = NORB * la;
    VT dg[NORB];
    C2 pv[NORB], rv[NORB];
    if constexpr (DIAG) {
        for (int e = threadIdx.x; e < nrow; e += kThreads) sv[e] = onsite ? ld<NT>(onsite + row0 + e) : (VT)0;
        __syncthreads();
#pragma unroll
        for (int o = 0; o < NORB; ++o) dg[o] = sv[mine + o] - a.shift;
        __syncthreads();
    }
    if constexpr (!FIRST) {
        const C2 *g = reinterpret_cast<const C2 *>(tprev) + row0;
        for (int e = threadIdx.x; e < nrow; e += kThreads) sbuf[e] = ld<NT>(g + e);
        __syncthreads();
#pragma unroll
        for (int o = 0; o < NORB; ++o) pv[o] = sbuf[mine + o];
        __syncthreads();
    }
    {
        const C2 *g = reinterpret_cast<const C2 *>(DBL ? tcur : r) + row0;
        for (int e = threadIdx.x; e < nrow; e += kThreads) sbuf[e] = DBL ? g[e] : ld<NT>(g + e);
        __syncthreads();
#pragma unroll
        for (int o = 0; o < NORB; ++o) rv[o] = sbuf[mine + o];
        __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < NORB; ++o) {
        VT yr = y[o].re[0], yi = y[o].im[0];
        if constexpr (DIAG) {
            C2 xs = rv[o];
            if constexpr (!DBL) xs = reinterpret_cast<const C2 *>(tcur)[(int64_t)NORB * at + o];
            yr += dg[o] * xs.x;
            yi += dg[o] * xs.y;
        }
        C2 ov;
        if constexpr (FIRST) {
            ov.x = a.c1 * yr;
            ov.y = a.c1 * yi;
        } else {
            ov.x = a.c1 * yr - pv[o].x;
            ov.y = a.c1 * yi - pv[o].y;
        }
        if (ok) {
            const double cr = (double)rv[o].x * (double)ov.x + (double)rv[o].y * (double)ov.y;
            if constexpr (DBL) {
                acc[0] += (double)ov.x * (double)ov.x + (double)ov.y * (double)ov.y;
                acc[1] += cr;
            } else {
                acc[0] += cr;
            }
        }
        sbuf[mine + o] = ov;
    }
    __syncthreads();
    {
        C2 *g = reinterpret_cast<C2 *>(tnext) + row0;
        for (int e = threadIdx.x; e < nrow; e += kThreads) st<NT>(g + e, sbuf[e]);
    }
    __syncthreads();
}

// Copies nbytes (a multiple of 4) from global memory to LDS with direct
// global-to-LDS loads: no register holds the data, and the copy completes at the
// issuing wave's next wait for all vector memory operations.  Every wave of the
// block takes 64-chunk runs of 16 bytes (the LDS destination of a run is uniform
// over the wave); the trailing words of a length that is not a multiple of 16 go
// through ordinary loads.
template <bool NT>
__device__ __forceinline__ void dma_to_lds(const void *g, void *l, int nbytes) {
    const int lane = threadIdx.x & 63;
    const int n16 = nbytes >> 4;
    for (int c0 = (int)(threadIdx.x >> 6) * 64; c0 < n16; c0 += kThreads)
        if (c0 + lane < n16)
            __builtin_amdgcn_global_load_lds(static_cast<const char *>(g) + 16 * (int64_t)(c0 + lane),
                                             (__attribute__((address_space(3))) void *)(static_cast<char *>(l) + 16 * c0),
                                             16, 0, NT ? 2 : 0);
    const int w0 = n16 * 4, nw = (nbytes >> 2) - w0;
    if ((int)threadIdx.x < nw)
        static_cast<int *>(l)[w0 + threadIdx.x] = static_cast<const int *>(g)[w0 + threadIdx.x];
}

// One-vector FP32 finish with prefetched streams: the tile's T_{n-1} and r (T_n
// in the doubling form) were copied to LDS (sprev, sr) when the tile started, so
// their round trip overlapped the bond loop; here the copies are awaited, the own
// rows of T_n (diagonal term) and the onsite energies are read, and T_{n+1} is
// staged through sprev for a contiguous store.
template <int NORB, bool FIRST, bool DIAG, bool NT, bool DBL>
__device__ __forceinline__ void finish_rows_prefetched(const Pack<float, 1> (&y)[NORB], const StepScalars<float> &a,
                                                       int64_t t, int la, int64_t at, bool ok,
                                                       const float *__restrict__ onsite, const float *__restrict__ tcur,
                                                       float *tnext, f2v *sprev, const f2v *sr,
                                                       double (&acc)[DBL ? 2 : 1]) {
    const int64_t row0 = (int64_t)NORB * (t * kThreads);
    const int nrow = (int)min((int64_t)NORB * kThreads, a.n_rows - row0);
    const int mine = NORB * la;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    f2v pv[NORB], rv[NORB], xs[NORB];
#pragma unroll
    for (int o = 0; o < NORB; ++o) {
        if constexpr (!FIRST) pv[o] = sprev[mine + o];
        rv[o] = sr[mine + o];
    }
    float dg[NORB];
    if constexpr (DIAG) {
        if constexpr (!DBL) {
#pragma unroll
            for (int o = 0; o < NORB; ++o) xs[o] = reinterpret_cast<const f2v *>(tcur)[(int64_t)NORB * at + o];
        }
        __syncthreads();                                  // sprev is read; its space takes the onsite energies
        float *sons = reinterpret_cast<float *>(sprev);
        if (onsite) dma_to_lds<NT>(onsite + row0, sons, nrow * 4);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll
        for (int o = 0; o < NORB; ++o) dg[o] = (onsite ? sons[mine + o] : 0.0f) - a.shift;
        __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < NORB; ++o) {
        float yr = y[o].re[0], yi = y[o].im[0];
        if constexpr (DIAG) {
            const f2v x = DBL ? rv[o] : xs[o];
            yr += dg[o] * x.x;
            yi += dg[o] * x.y;
        }
        f2v ov;
        if constexpr (FIRST) {
            ov.x = a.c1 * yr;
            ov.y = a.c1 * yi;
        } else {
            ov.x = a.c1 * yr - pv[o].x;
            ov.y = a.c1 * yi - pv[o].y;
        }
        if (ok) {
            const double cr = (double)rv[o].x * (double)ov.x + (double)rv[o].y * (double)ov.y;
            if constexpr (DBL) {
                acc[0] += (double)ov.x * (double)ov.x + (double)ov.y * (double)ov.y;
                acc[1] += cr;
            } else {
                acc[0] += cr;
            }
        }
        sprev[mine + o] = ov;
    }
    __syncthreads();
    f2v *g = reinterpret_cast<f2v *>(tnext) + row0;
    for (int e = threadIdx.x; e < nrow; e += kThreads) st<NT>(g + e, sprev[e]);
    __syncthreads();
}

// Atom form: a thread owns every orbital row of one atom (VPT vectors), so
// each neighbour's NORB orbital rows of T_n are gathered once per atom instead
// of once per orbital row; the block's rows are read one after the other
// (all L threads of an atom read the same values).  Rows of the atom are
// written, and their moment terms accumulated, in orbital order.
template <class VT, int NORB, int L, int VPT, bool FIRST, bool DIAG, bool NT, bool DBL>
__global__ __launch_bounds__(kThreads) void k_cheb_step_atom(
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ bcol, const VT *__restrict__ bval,
    const VT *__restrict__ onsite, const VT *__restrict__ tcur, const VT *tprev, VT *tnext,
    const VT *__restrict__ r, double *__restrict__ partial, StepScalars<VT> a, int stage) {
    constexpr int APB = kThreads / L;   // atoms per tile
    const int la = threadIdx.x / L;
    const int vs = threadIdx.x % L;
    const int64_t lb = logical_block(a.xcd_remap);
    const int64_t t0 = lb * a.tiles_per_block;
    const int64_t t1 = min(t0 + a.tiles_per_block, a.n_tiles);
    const int64_t smask = ((int64_t)1 << a.log2_slice) - 1;
    const int64_t stride = smask + 1;
    constexpr int Rp = L * VPT;       // padded vector count (a.Rp)
    const int voff = vs * VPT;
    const int64_t last = a.n_rows / NORB - 1;     // last atom row

    constexpr int NA = DBL ? 2 * VPT : VPT;
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;

    // float blocks with several lanes per atom: each lane loads a contiguous share
    // of the block (kFpl values, the last lane's share cut at NORB^2) and the atom's
    // lanes (all in one wavefront) read it whole from LDS, instead of every lane
    // loading all of it
    constexpr int kNB = NORB * NORB;
    constexpr bool kShare = sizeof(VT) == 4 && L >= 2 && L <= 16;
    constexpr int kFpl = kShare ? (kNB + L - 1) / L : 1;     // block values loaded per lane
    constexpr int kSS = (kNB + 3) / 4 * 4;                    // LDS stride per atom (16 B multiple)
    __shared__ __align__(16) VT sblk[kShare ? kSS * APB : 1];

    for (int64_t t = t0; t < t1; ++t) {
        const int64_t au = t * APB + la;
        const bool ok = au <= last;
        const int64_t at = min(au, last);
        const int64_t sl = at >> a.log2_slice;
        const int64_t p0 = ptr[sl], p1 = ptr[sl + 1];
        const int64_t base = p0 + (at & smask);
        const int w = (int)((p1 - p0) >> a.log2_slice);

        Pack<VT, VPT> y[NORB];
#pragma unroll
        for (int o = 0; o < NORB; ++o)
#pragma unroll
            for (int q = 0; q < VPT; ++q) { y[o].re[q] = 0; y[o].im[q] = 0; }
        // the next neighbour's column is loaded before this neighbour's block is
        // applied, so a neighbour waits for one memory round trip (its gathers)
        int32_t cn = w > 0 ? ld<NT>(bcol + base) : 0;
        for (int k = 0; k < w; ++k) {
            const int64_t qb = base + (int64_t)k * stride;
            const int32_t c = cn;
            Pack<VT, VPT> x[NORB];
#pragma unroll
            for (int b = 0; b < NORB; ++b)
                x[b] = load_pack<false, VT, VPT>(tcur + 2 * (((int64_t)NORB * c + b) * Rp + voff));
            if (k + 1 < w) cn = ld<NT>(bcol + qb + stride);
            const VT *bv = bval + (int64_t)NORB * NORB * qb;
            VT *sb = sblk + (kShare ? kSS * la : 0);
            if constexpr (kShare) {
                VT part[kFpl];
#pragma unroll
                for (int e = 0; e < kFpl; ++e)
                    if (kNB % L == 0 || vs * kFpl + e < kNB) part[e] = ld<NT>(bv + vs * kFpl + e);
                // the previous neighbour's reads of this atom's slots come before the writes
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int e = 0; e < kFpl; ++e)
                    if (kNB % L == 0 || vs * kFpl + e < kNB) sb[vs * kFpl + e] = part[e];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
#pragma unroll
            for (int o = 0; o < NORB; ++o) {
                VT h[NORB];
                if constexpr (kShare) {
#pragma unroll
                    for (int b = 0; b < NORB; ++b) h[b] = sb[NORB * o + b];
                } else {
                    load_row<NORB, NT, VT>(bv + NORB * o, h);
                }
#pragma unroll
                for (int b = 0; b < NORB; ++b)
#pragma unroll
                    for (int q = 0; q < VPT; ++q) {
                        y[o].re[q] += h[b] * x[b].re[q];
                        y[o].im[q] += h[b] * x[b].im[q];
                    }
            }
        }
        bool staged = false;
        if constexpr (L == 1 && VPT == 1) {
            if (stage) {
                finish_rows_staged<VT, NORB, FIRST, DIAG, NT, DBL>(y, a, t, la, at, ok, onsite, tcur, tprev, tnext,
                                                                  r, acc);
                staged = true;
            }
        }
        if (!staged) {
#pragma unroll
            for (int o = 0; o < NORB; ++o) {
                const int64_t i = (int64_t)NORB * at + o;
                const int64_t off = 2 * (i * Rp + voff);
                Pack<VT, VPT> pv, rv;
                if constexpr (!FIRST) pv = load_pack<NT, VT, VPT>(tprev + off);
                if constexpr (DBL) rv = load_pack<false, VT, VPT>(tcur + off);
                else rv = load_pack<NT, VT, VPT>(r + off);
                if constexpr (DIAG) {
                    const VT dg = (onsite ? ld<NT>(onsite + i) : (VT)0) - a.shift;
                    const Pack<VT, VPT> xs = DBL ? rv : load_pack<false, VT, VPT>(tcur + off);
#pragma unroll
                    for (int q = 0; q < VPT; ++q) { y[o].re[q] += dg * xs.re[q]; y[o].im[q] += dg * xs.im[q]; }
                }
                Pack<VT, VPT> ov;
#pragma unroll
                for (int q = 0; q < VPT; ++q) {
                    if constexpr (FIRST) {
                        ov.re[q] = a.c1 * y[o].re[q];
                        ov.im[q] = a.c1 * y[o].im[q];
                    } else {
                        ov.re[q] = a.c1 * y[o].re[q] - pv.re[q];
                        ov.im[q] = a.c1 * y[o].im[q] - pv.im[q];
                    }
                }
                if (ok) {
                    store_pack<NT, VT, VPT>(tnext + off, ov);
#pragma unroll
                    for (int q = 0; q < VPT; ++q) {
                        const double cr = (double)rv.re[q] * (double)ov.re[q] + (double)rv.im[q] * (double)ov.im[q];
                        if constexpr (DBL) {
                            acc[q] += (double)ov.re[q] * (double)ov.re[q] + (double)ov.im[q] * (double)ov.im[q];
                            acc[VPT + q] += cr;
                        } else {
                            acc[q] += cr;
                        }
                    }
                }
            }
        }
    }
    block_reduce_store<L, NA>(acc, partial, lb);
}

// Integrals and radial law of the displacement form, in the vector type.  The
// integrals are regrouped on the host into the combinations the projector form
// uses: ss, sp, pp_sigma - pp_pi, pp_pi, sd, pd_sigma, pd_pi / sqrt(3),
// dd_sigma - dd_delta, (dd_pi - dd_delta) / 3, dd_delta.
template <class VT> struct GeomParams {
    VT v[10];        // regrouped integrals at r0
    VT inv_r0;       // 1 / r0
    VT beta;         // decay exponent
    VT e0, e1;       // f(r) = 2^(e0 - e1 r): e0 = beta / ln 2, e1 = beta / (r0 ln 2)
};

// One bond's geometry for the projector form: the direction cosines c, sqrt(3) c,
// the d-orbital sigma vector u along c and the regrouped integrals scaled by f(r).
// Formed once per bond and used for both components of every vector.
template <class VT> struct BondFrame {
    VT k[10];
    VT l, m, n, sl, sm, sn;
    VT u[5];
};

// Direction cosines and f(r) from the displacement d (|d| > 0).  In FP32 the
// reciprocal square root and the power of two are single instructions (about one
// ulp each); in FP64 the correctly rounded sqrt, division and exp.
template <class VT>
__device__ __forceinline__ BondFrame<VT> bond_frame(const GeomParams<VT> &gp, VT dx, VT dy, VT dz, VT r2) {
    BondFrame<VT> b;
    VT inv, f;
    if constexpr (sizeof(VT) == 4) {
        inv = __builtin_amdgcn_rsqf(r2);
        f = __builtin_amdgcn_exp2f(gp.e0 - gp.e1 * (r2 * inv));
    } else {
        const VT rr = sqrt(r2);
        inv = (VT)1 / rr;
        f = exp(-gp.beta * (rr * gp.inv_r0 - (VT)1));
    }
#pragma unroll
    for (int q = 0; q < 10; ++q) b.k[q] = gp.v[q] * f;
    const VT s3 = (VT)1.7320508075688772;
    b.l = dx * inv;
    b.m = dy * inv;
    b.n = dz * inv;
    b.sl = s3 * b.l;
    b.sm = s3 * b.m;
    b.sn = s3 * b.n;
    b.u[0] = b.sl * b.m;
    b.u[1] = b.sm * b.n;
    b.u[2] = b.sn * b.l;
    b.u[3] = (VT)0.5 * (b.sl * b.l - b.sm * b.m);
    b.u[4] = b.n * b.n - (VT)0.5 * (b.l * b.l + b.m * b.m);
    return b;
}

// y += B x for the one-species Slater-Koster block B of a bond with direction
// cosines c = (l, m, n), without forming B: with u the d-orbital sigma vector
// along c (the s-d row of the table divided by V_sd_sigma) and J = du/dc (u is
// homogeneous of degree 2, so c.grad u_b = 2 u_b), the table's blocks are
//   p-p: V_pp_pi I + (V_pp_sigma - V_pp_pi) c c^T,
//   p-d: V_pd_sigma c u^T + V_pd_pi (J^T - 2 c u^T) / sqrt(3)    (d-p: minus its transpose),
//   d-d: V_dd_delta I + (V_dd_sigma - V_dd_delta) u u^T + (V_dd_pi - V_dd_delta) J (I - c c^T) J^T / 3,
// so one bond costs about 70 multiply-adds per vector component instead of the
// NORB^2 products plus the table.
template <class VT, int NORB>
__device__ __forceinline__ void sk_apply(const BondFrame<VT> &b, const VT (&x)[NORB], VT (&y)[NORB]) {
    const VT ss = b.k[0], sp = b.k[1], ppd = b.k[2], ppp = b.k[3];
    const VT l = b.l, m = b.m, n = b.n;
    const VT xs = x[0], xp0 = x[1], xp1 = x[2], xp2 = x[3];
    const VT cp = l * xp0 + m * xp1 + n * xp2;
    // every update is a chain of multiply-adds into y (one rounding per product)
    if constexpr (NORB == 4) {
        const VT t = ppd * cp - sp * xs;
        y[0] += ss * xs;
        y[0] += sp * cp;
        y[1] += ppp * xp0;
        y[1] += l * t;
        y[2] += ppp * xp1;
        y[2] += m * t;
        y[3] += ppp * xp2;
        y[3] += n * t;
    } else {
        const VT sd = b.k[4], pds = b.k[5], k1 = b.k[6], ddd_s = b.k[7], k2 = b.k[8], ddd = b.k[9];
        const VT sl = b.sl, sm = b.sm, sn = b.sn;
        const VT xd0 = x[4], xd1 = x[5], xd2 = x[6], xd3 = x[7], xd4 = x[8];
        const VT ud = b.u[0] * xd0 + b.u[1] * xd1 + b.u[2] * xd2 + b.u[3] * xd3 + b.u[4] * xd4;
        // G = J^T x_d, then (I - c c^T) G = G - 2 (u.x_d) c
        const VT nud2 = (VT)-2 * ud;
        const VT pl = sm * xd0 + sn * xd2 + sl * xd3 - l * xd4 + nud2 * l;
        const VT pm = sl * xd0 + sn * xd1 - sm * xd3 - m * xd4 + nud2 * m;
        const VT pn = sm * xd1 + sl * xd2 + (VT)2 * n * xd4 + nud2 * n;
        const VT t = ppd * cp + pds * ud - sp * xs;
        y[0] += ss * xs;
        y[0] += sp * cp;
        y[0] += sd * ud;
        y[1] += ppp * xp0;
        y[1] += l * t;
        y[1] += k1 * pl;
        y[2] += ppp * xp1;
        y[2] += m * t;
        y[2] += k1 * pm;
        y[3] += ppp * xp2;
        y[3] += n * t;
        y[3] += k1 * pn;
        // h = -k1 (x_p - c cp) + k2 (I - c c^T) G, then J h
        const VT hl = k2 * pl - k1 * (xp0 - l * cp);
        const VT hm = k2 * pm - k1 * (xp1 - m * cp);
        const VT hn = k2 * pn - k1 * (xp2 - n * cp);
        const VT w = sd * xs - pds * cp + ddd_s * ud;
        y[4] += ddd * xd0;
        y[4] += b.u[0] * w;
        y[4] += sm * hl;
        y[4] += sl * hm;
        y[5] += ddd * xd1;
        y[5] += b.u[1] * w;
        y[5] += sn * hm;
        y[5] += sm * hn;
        y[6] += ddd * xd2;
        y[6] += b.u[2] * w;
        y[6] += sn * hl;
        y[6] += sl * hn;
        y[7] += ddd * xd3;
        y[7] += b.u[3] * w;
        y[7] += sl * hl;
        y[7] -= sm * hm;
        y[8] += ddd * xd4;
        y[8] += b.u[4] * w;
        y[8] += (VT)2 * n * hn;
        y[8] -= l * hl;
        y[8] -= m * hm;
    }
}

// Displacement form (TBK_BGEOM_*): as the atom form, but each bond stores its
// displacement d = x_j - x_i (3 values) instead of its block.  The block is
// applied without being formed: r = |d|, direction cosines d / r, integrals
// scaled by f(r) = exp(-beta (r / r0 - 1)), then sk_apply in the vector type.
// Padding slots (d = 0) are skipped.  Per float bond this reads one 16-byte
// record (dx, dy, dz, the column's bits) instead of a column and 4 NORB^2 B;
// double bonds read the column and 24 B.  With one FP32 vector and staging, the
// finish's T_{n-1} and r are copied to LDS when the tile starts
// (finish_rows_prefetched).
template <class VT, int NORB, int L, int VPT, bool FIRST, bool DIAG, bool NT, bool DBL>
__global__ __launch_bounds__(kThreads) void k_cheb_step_geom(
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ bcol, const VT *__restrict__ geo,
    const VT *__restrict__ onsite, const VT *__restrict__ tcur, const VT *tprev, VT *tnext,
    const VT *__restrict__ r, double *__restrict__ partial, StepScalars<VT> a, GeomParams<VT> gp, int stage) {
    constexpr int APB = kThreads / L;   // atoms per tile
    const int la = threadIdx.x / L;
    const int vs = threadIdx.x % L;
    const int64_t lb = logical_block(a.xcd_remap);
    const int64_t t0 = lb * a.tiles_per_block;
    const int64_t t1 = min(t0 + a.tiles_per_block, a.n_tiles);
    const int64_t smask = ((int64_t)1 << a.log2_slice) - 1;
    const int64_t stride = smask + 1;
    constexpr int Rp = L * VPT;       // padded vector count (a.Rp)
    const int voff = vs * VPT;
    const int64_t last = a.n_rows / NORB - 1;     // last atom row

    constexpr int NA = DBL ? 2 * VPT : VPT;
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;

    // FP32 one-vector tiles with staging: the finish's streams are copied to LDS
    // when the tile starts (see finish_rows_prefetched)
    constexpr bool kPre = L == 1 && VPT == 1 && sizeof(VT) == 4;
    __shared__ f2v sprev[kPre ? NORB * kThreads : 1], sr[kPre ? NORB * kThreads : 1];
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t au = t * APB + la;
        const bool ok = au <= last;
        const int64_t at = min(au, last);
        const int64_t sl = at >> a.log2_slice;
        const int64_t p0 = ptr[sl], p1 = ptr[sl + 1];
        const int64_t base = p0 + (at & smask);
        const int w = (int)((p1 - p0) >> a.log2_slice);

        Pack<VT, VPT> y[NORB];
#pragma unroll
        for (int o = 0; o < NORB; ++o)
#pragma unroll
            for (int q = 0; q < VPT; ++q) { y[o].re[q] = 0; y[o].im[q] = 0; }
        // two bonds per pass: both bonds' columns, displacements and neighbour rows are
        // loaded before either block is applied (slots past the width repeat the last one
        // and are skipped, as are padding slots, d = 0).  The next pass's columns and
        // displacements are loaded before this pass's blocks are applied, so a pass waits
        // for one memory round trip (its gathers) instead of two.
        constexpr int KU = 2;
        int32_t cn[KU];
        VT dxn[KU], dyn[KU], dzn[KU];
        auto load_bonds = [&](int k0) {
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int64_t qb = base + (int64_t)max(0, min(k0 + u, w - 1)) * stride;
                if constexpr (sizeof(VT) == 4) {      // one 16-byte record (dx, dy, dz, column)
                    const f4v g = ld<NT>(reinterpret_cast<const f4v *>(geo) + qb);
                    dxn[u] = g.x;
                    dyn[u] = g.y;
                    dzn[u] = g.z;
                    cn[u] = __float_as_int(g.w);
                } else {
                    cn[u] = ld<NT>(bcol + qb);
                    dxn[u] = ld<NT>(geo + 3 * qb);
                    dyn[u] = ld<NT>(geo + 3 * qb + 1);
                    dzn[u] = ld<NT>(geo + 3 * qb + 2);
                }
            }
        };
        // the finish's streams (T_{n-1}, r) copied to LDS ahead of the bond loop
        auto prefetch_finish = [&]() {
            if constexpr (kPre) {
                if (stage) {
                    const int64_t row0 = (int64_t)NORB * (t * APB);
                    const int nbytes = 8 * (int)min((int64_t)NORB * APB, a.n_rows - row0);
                    if constexpr (!FIRST) dma_to_lds<NT>(reinterpret_cast<const f2v *>(tprev) + row0, sprev, nbytes);
                    dma_to_lds<NT && !DBL>(reinterpret_cast<const f2v *>(DBL ? tcur : r) + row0, sr, nbytes);
                }
            }
        };
        // one pass: the gathers of bonds k0, k0 + 1, the next pass's bond loads, then
        // both blocks
        auto pass = [&](int k0) {
            int32_t c[KU];
            VT dx[KU], dy[KU], dz[KU];
#pragma unroll
            for (int u = 0; u < KU; ++u) { c[u] = cn[u]; dx[u] = dxn[u]; dy[u] = dyn[u]; dz[u] = dzn[u]; }
            Pack<VT, VPT> x[KU][NORB];
#pragma unroll
            for (int u = 0; u < KU; ++u)
#pragma unroll
                for (int b = 0; b < NORB; ++b)
                    x[u][b] = load_pack<false, VT, VPT>(tcur + 2 * (((int64_t)NORB * c[u] + b) * Rp + voff));
            if (k0 + KU < w) load_bonds(k0 + KU);
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const VT r2 = dx[u] * dx[u] + dy[u] * dy[u] + dz[u] * dz[u];
                if (k0 + u >= w || !(r2 > (VT)0)) continue;
                const BondFrame<VT> bf = bond_frame(gp, dx[u], dy[u], dz[u], r2);
#pragma unroll
                for (int q = 0; q < VPT; ++q) {
                    VT xr[NORB], xi[NORB], yr[NORB], yi[NORB];
#pragma unroll
                    for (int b = 0; b < NORB; ++b) {
                        xr[b] = x[u][b].re[q];
                        xi[b] = x[u][b].im[q];
                        yr[b] = y[b].re[q];
                        yi[b] = y[b].im[q];
                    }
                    sk_apply<VT, NORB>(bf, xr, yr);
                    sk_apply<VT, NORB>(bf, xi, yi);
#pragma unroll
                    for (int b = 0; b < NORB; ++b) {
                        y[b].re[q] = yr[b];
                        y[b].im[q] = yi[b];
                    }
                }
            }
        };
        // the finish's copies go out with the first bond loads, whose round trip they share
        if (w > 0) load_bonds(0);
        prefetch_finish();
        for (int k0 = 0; k0 < w; k0 += KU) pass(k0);
        bool staged = false;
        if constexpr (kPre) {
            if (stage) {
                finish_rows_prefetched<NORB, FIRST, DIAG, NT, DBL>(y, a, t, la, at, ok, onsite, tcur, tnext, sprev, sr,
                                                                  acc);
                staged = true;
            }
        } else if constexpr (L == 1 && VPT == 1) {
            if (stage) {
                finish_rows_staged<VT, NORB, FIRST, DIAG, NT, DBL>(y, a, t, la, at, ok, onsite, tcur, tprev, tnext,
                                                                  r, acc);
                staged = true;
            }
        }
        if (!staged) {
#pragma unroll
            for (int o = 0; o < NORB; ++o) {
                const int64_t i = (int64_t)NORB * at + o;
                const int64_t off = 2 * (i * Rp + voff);
                Pack<VT, VPT> pv, rv;
                if constexpr (!FIRST) pv = load_pack<NT, VT, VPT>(tprev + off);
                if constexpr (DBL) rv = load_pack<false, VT, VPT>(tcur + off);
                else rv = load_pack<NT, VT, VPT>(r + off);
                if constexpr (DIAG) {
                    const VT dg = (onsite ? ld<NT>(onsite + i) : (VT)0) - a.shift;
                    const Pack<VT, VPT> xs = DBL ? rv : load_pack<false, VT, VPT>(tcur + off);
#pragma unroll
                    for (int q = 0; q < VPT; ++q) { y[o].re[q] += dg * xs.re[q]; y[o].im[q] += dg * xs.im[q]; }
                }
                Pack<VT, VPT> ov;
#pragma unroll
                for (int q = 0; q < VPT; ++q) {
                    if constexpr (FIRST) {
                        ov.re[q] = a.c1 * y[o].re[q];
                        ov.im[q] = a.c1 * y[o].im[q];
                    } else {
                        ov.re[q] = a.c1 * y[o].re[q] - pv.re[q];
                        ov.im[q] = a.c1 * y[o].im[q] - pv.im[q];
                    }
                }
                if (ok) {
                    store_pack<NT, VT, VPT>(tnext + off, ov);
#pragma unroll
                    for (int q = 0; q < VPT; ++q) {
                        const double cr = (double)rv.re[q] * (double)ov.re[q] + (double)rv.im[q] * (double)ov.im[q];
                        if constexpr (DBL) {
                            acc[q] += (double)ov.re[q] * (double)ov.re[q] + (double)ov.im[q] * (double)ov.im[q];
                            acc[VPT + q] += cr;
                        } else {
                            acc[q] += cr;
                        }
                    }
                }
            }
        }
    }
    block_reduce_store<L, NA>(acc, partial, lb);
}

template <class VT, int NORB, int L, int VPT, bool FIRST, bool DIAG>
void launch_fd(const KpmPlan &pl, hipStream_t s, const StepPtrs<VT> &p, const StepScalars<VT> &a) {
    const unsigned G = (unsigned)pl.G;
    // one-vector row staging through LDS (rows_per_thread: 1 = when the launch is large
    // enough to keep every CU busy between the staging barriers, 2 = always, 4 = never)
    const int stage = pl.cfg.rows_per_thread == 2 || (pl.cfg.rows_per_thread == 1 && pl.n_tiles >= kStageMinTiles);
    GeomParams<VT> gp;
    {
        // regroup the integrals (ss, sp, pp_sigma, pp_pi, sd, pd_sigma, pd_pi, dd_sigma,
        // dd_pi, dd_delta) into the projector form's combinations, in FP64
        const double *v = pl.geom_params;
        const double g[10] = {v[0], v[1], v[2] - v[3], v[3], v[4], v[5], v[6] / std::sqrt(3.0),
                              v[7] - v[9], (v[8] - v[9]) / 3.0, v[9]};
        for (int l = 0; l < 10; ++l) gp.v[l] = (VT)g[l];
        const double r0 = pl.geom_params[10], beta = pl.geom_params[11];
        gp.inv_r0 = r0 > 0 ? (VT)(1.0 / r0) : (VT)0;
        gp.beta = (VT)beta;
        gp.e0 = (VT)(beta / std::log(2.0));
        gp.e1 = r0 > 0 ? (VT)(beta / (r0 * std::log(2.0))) : (VT)0;
    }
#define TBK_BLK(NT, DBL)                                                                                    \
    do {                                                                                                    \
        if (pl.geom)                                                                                        \
            k_cheb_step_geom<VT, NORB, L, VPT, FIRST, DIAG, NT, DBL><<<G, kThreads, 0, s>>>(                \
                p.ptr, p.col, p.val, p.onsite, p.tcur, p.tprev, p.tnext, p.r, p.partial, a, gp, stage);     \
        else if (pl.cfg.atom_rows)                                                                          \
            k_cheb_step_atom<VT, NORB, L, VPT, FIRST, DIAG, NT, DBL><<<G, kThreads, 0, s>>>(                \
                p.ptr, p.col, p.val, p.onsite, p.tcur, p.tprev, p.tnext, p.r, p.partial, a, stage);         \
        else                                                                                                \
            k_cheb_step_blk<VT, NORB, L, VPT, FIRST, DIAG, NT, DBL><<<G, kThreads, 0, s>>>(                 \
                p.ptr, p.col, p.val, p.onsite, p.tcur, p.tprev, p.tnext, p.r, p.partial, a);                \
    } while (0)
    if (pl.cfg.nontemporal) {
        if (pl.cfg.doubling) TBK_BLK(true, true);
        else TBK_BLK(true, false);
    } else {
        if (pl.cfg.doubling) TBK_BLK(false, true);
        else TBK_BLK(false, false);
    }
#undef TBK_BLK
}

template <class VT, int NORB, int L, int VPT>
void launch_fdv(const KpmPlan &pl, bool first, bool diag, hipStream_t s, const StepPtrs<VT> &p,
                const StepScalars<VT> &a) {
    if (first) {
        if (diag) launch_fd<VT, NORB, L, VPT, true, true>(pl, s, p, a);
        else launch_fd<VT, NORB, L, VPT, true, false>(pl, s, p, a);
    } else {
        if (diag) launch_fd<VT, NORB, L, VPT, false, true>(pl, s, p, a);
        else launch_fd<VT, NORB, L, VPT, false, false>(pl, s, p, a);
    }
}

template <class VT, int L, int VPT>
void launch_lv(const KpmPlan &pl, bool first, bool diag, hipStream_t s, const StepPtrs<VT> &p,
               const StepScalars<VT> &a) {
    if (pl.norb == 9) launch_fdv<VT, 9, L, VPT>(pl, first, diag, s, p, a);
    else launch_fdv<VT, 4, L, VPT>(pl, first, diag, s, p, a);
}

}  // namespace

template <class VT>
tbk_status launch_step_block(const KpmPlan &pl, bool first, bool diag, hipStream_t s, const StepPtrs<VT> &p,
                             const StepScalars<VT> &a) {
    if constexpr (sizeof(VT) == 8) {
        switch (pl.L) {
        case 1: launch_lv<VT, 1, 1>(pl, first, diag, s, p, a); break;
        case 2: launch_lv<VT, 2, 1>(pl, first, diag, s, p, a); break;
        case 4: launch_lv<VT, 4, 1>(pl, first, diag, s, p, a); break;
        case 8: launch_lv<VT, 8, 1>(pl, first, diag, s, p, a); break;
        case 16: launch_lv<VT, 16, 1>(pl, first, diag, s, p, a); break;
        case 32: launch_lv<VT, 32, 1>(pl, first, diag, s, p, a); break;
        case 64: launch_lv<VT, 64, 1>(pl, first, diag, s, p, a); break;
        default: return fail(TBK_ERR_UNSUPPORTED, "no block kernel for L = %d", pl.L);
        }
    } else if (pl.VPT == 1) {
        switch (pl.L) {
        case 1: launch_lv<VT, 1, 1>(pl, first, diag, s, p, a); break;
        case 2: launch_lv<VT, 2, 1>(pl, first, diag, s, p, a); break;
        case 4: launch_lv<VT, 4, 1>(pl, first, diag, s, p, a); break;
        case 8: launch_lv<VT, 8, 1>(pl, first, diag, s, p, a); break;
        case 16: launch_lv<VT, 16, 1>(pl, first, diag, s, p, a); break;
        case 32: launch_lv<VT, 32, 1>(pl, first, diag, s, p, a); break;
        case 64: launch_lv<VT, 64, 1>(pl, first, diag, s, p, a); break;
        default: return fail(TBK_ERR_UNSUPPORTED, "no block kernel for L = %d", pl.L);
        }
    } else {
        switch (pl.L) {
        case 1: launch_lv<VT, 1, 2>(pl, first, diag, s, p, a); break;
        case 2: launch_lv<VT, 2, 2>(pl, first, diag, s, p, a); break;
        case 4: launch_lv<VT, 4, 2>(pl, first, diag, s, p, a); break;
        case 8: launch_lv<VT, 8, 2>(pl, first, diag, s, p, a); break;
        case 16: launch_lv<VT, 16, 2>(pl, first, diag, s, p, a); break;
        case 32: launch_lv<VT, 32, 2>(pl, first, diag, s, p, a); break;
        default: return fail(TBK_ERR_UNSUPPORTED, "no block kernel for L = %d", pl.L);
        }
    }
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

template tbk_status launch_step_block<float>(const KpmPlan &, bool, bool, hipStream_t, const StepPtrs<float> &,
                                             const StepScalars<float> &);
template tbk_status launch_step_block<double>(const KpmPlan &, bool, bool, hipStream_t, const StepPtrs<double> &,
                                              const StepScalars<double> &);

}  // namespace tbk
