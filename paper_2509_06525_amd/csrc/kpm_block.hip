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
#pragma unroll
            for (int o = 0; o < NORB; ++o) {
                VT h[NORB];
                load_row<NORB, NT, VT>(bv + NORB * o, h);
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

// Integrals and radial law of the displacement form, in the vector type.
template <class VT> struct GeomParams {
    VT v[10];        // integrals at r0
    VT inv_r0;       // 1 / r0
    VT beta;         // decay exponent
};

// y += B x for the one-species Slater-Koster block B of a bond with direction
// cosines c = (l, m, n) and integrals v (already scaled by f(r)), without
// forming B: with u the d-orbital sigma vector along c (the s-d row of the table
// divided by V_sd_sigma) and J = du/dc (u is homogeneous of degree 2, so
// c.grad u_b = 2 u_b), the table's blocks are
//   p-p: V_pp_pi I + (V_pp_sigma - V_pp_pi) c c^T,
//   p-d: V_pd_sigma c u^T + V_pd_pi (J^T - 2 c u^T) / sqrt(3)    (d-p: minus its transpose),
//   d-d: V_dd_delta I + (V_dd_sigma - V_dd_delta) u u^T + (V_dd_pi - V_dd_delta) J (I - c c^T) J^T / 3,
// so one bond costs about 76 multiply-adds per vector component instead of the
// NORB^2 products plus the table.
template <class VT, int NORB>
__device__ __forceinline__ void sk_apply(const VT (&v)[10], VT l, VT m, VT n, const VT (&x)[NORB], VT (&y)[NORB]) {
    const VT ss = v[0], sp = v[1], pps = v[2], ppp = v[3];
    const VT xs = x[0], xp0 = x[1], xp1 = x[2], xp2 = x[3];
    const VT cp = l * xp0 + m * xp1 + n * xp2;
    if constexpr (NORB == 4) {
        y[0] += ss * xs + sp * cp;
        const VT t = (pps - ppp) * cp - sp * xs;
        y[1] += ppp * xp0 + l * t;
        y[2] += ppp * xp1 + m * t;
        y[3] += ppp * xp2 + n * t;
    } else {
        const VT s3 = (VT)1.7320508075688772;
        const VT sd = v[4], pds = v[5], pdp = v[6], dds = v[7], ddp = v[8], ddd = v[9];
        const VT u0 = s3 * l * m, u1 = s3 * m * n, u2 = s3 * n * l;
        const VT u3 = (VT)0.5 * s3 * (l * l - m * m), u4 = n * n - (VT)0.5 * (l * l + m * m);
        const VT xd0 = x[4], xd1 = x[5], xd2 = x[6], xd3 = x[7], xd4 = x[8];
        const VT ud = u0 * xd0 + u1 * xd1 + u2 * xd2 + u3 * xd3 + u4 * xd4;
        // G = J^T x_d
        const VT gl = s3 * (m * xd0 + n * xd2 + l * xd3) - l * xd4;
        const VT gm = s3 * (l * xd0 + n * xd1 - m * xd3) - m * xd4;
        const VT gn = s3 * (m * xd1 + l * xd2) + (VT)2 * n * xd4;
        const VT ud2 = (VT)2 * ud;
        const VT pl = gl - ud2 * l, pm = gm - ud2 * m, pn = gn - ud2 * n;      // (I - c c^T) G
        const VT k1 = pdp / s3, k2 = (ddp - ddd) / (VT)3;
        y[0] += ss * xs + sp * cp + sd * ud;
        const VT t = (pps - ppp) * cp + pds * ud - sp * xs;
        y[1] += ppp * xp0 + l * t + k1 * pl;
        y[2] += ppp * xp1 + m * t + k1 * pm;
        y[3] += ppp * xp2 + n * t + k1 * pn;
        // h = -k1 (x_p - c cp) + k2 (I - c c^T) G, then J h
        const VT hl = k2 * pl - k1 * (xp0 - l * cp);
        const VT hm = k2 * pm - k1 * (xp1 - m * cp);
        const VT hn = k2 * pn - k1 * (xp2 - n * cp);
        const VT w = sd * xs - pds * cp + (dds - ddd) * ud;
        y[4] += ddd * xd0 + u0 * w + s3 * (m * hl + l * hm);
        y[5] += ddd * xd1 + u1 * w + s3 * (n * hm + m * hn);
        y[6] += ddd * xd2 + u2 * w + s3 * (n * hl + l * hn);
        y[7] += ddd * xd3 + u3 * w + s3 * (l * hl - m * hm);
        y[8] += ddd * xd4 + u4 * w + ((VT)2 * n * hn - l * hl - m * hm);
    }
}

// Displacement form (TBK_BGEOM_*): as the atom form, but each bond stores its
// displacement d = x_j - x_i (3 values) instead of its block.  The block is
// applied without being formed: r = |d|, direction cosines d / r, integrals
// scaled by f(r) = exp(-beta (r / r0 - 1)), then sk_apply in the vector type.
// Padding slots (d = 0) are skipped.  Per bond this reads 12 B (float) instead
// of 4 NORB^2 B.
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
                cn[u] = ld<NT>(bcol + qb);
                dxn[u] = ld<NT>(geo + 3 * qb);
                dyn[u] = ld<NT>(geo + 3 * qb + 1);
                dzn[u] = ld<NT>(geo + 3 * qb + 2);
            }
        };
        if (w > 0) load_bonds(0);
        for (int k0 = 0; k0 < w; k0 += KU) {
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
                const VT rr = sqrt(r2);
                const VT inv = (VT)1 / rr;
                const VT f = exp(-gp.beta * (rr * gp.inv_r0 - (VT)1));
                VT vf[10];
#pragma unroll
                for (int l = 0; l < 10; ++l) vf[l] = gp.v[l] * f;
                const VT cl = dx[u] * inv, cm = dy[u] * inv, cn = dz[u] * inv;
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
                    sk_apply<VT, NORB>(vf, cl, cm, cn, xr, yr);
                    sk_apply<VT, NORB>(vf, cl, cm, cn, xi, yi);
#pragma unroll
                    for (int b = 0; b < NORB; ++b) {
                        y[b].re[q] = yr[b];
                        y[b].im[q] = yi[b];
                    }
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

template <class VT, int NORB, int L, int VPT, bool FIRST, bool DIAG>
void launch_fd(const KpmPlan &pl, hipStream_t s, const StepPtrs<VT> &p, const StepScalars<VT> &a) {
    const unsigned G = (unsigned)pl.G;
    // one-vector row staging through LDS (rows_per_thread: 1 = when the launch is large
    // enough to keep every CU busy between the staging barriers, 2 = always, 4 = never)
    const int stage = pl.cfg.rows_per_thread == 2 || (pl.cfg.rows_per_thread == 1 && pl.n_tiles >= kStageMinTiles);
    GeomParams<VT> gp;
    for (int l = 0; l < 10; ++l) gp.v[l] = (VT)pl.geom_params[l];
    gp.inv_r0 = pl.geom_params[10] > 0 ? (VT)(1.0 / pl.geom_params[10]) : (VT)0;
    gp.beta = (VT)pl.geom_params[11];
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
