// Velocity autocorrelation (VAC) conductivity of Eq. (3) on the GPU.
//
//   sigma(E, t) = (2 e^2 / Omega) int_0^t Tr[delta(E - H) Re(V V(tau))] dtau,
//
// with V = (i / hbar)[H, X] and V(tau) = U(tau)^+ V U(tau), U = exp(-i H tau / hbar).
// The trace is estimated with random-phase vectors phi (Sec. 2.4):
//   phi_R(0) = phi, phi_L(0) = V phi; at each time step t_j = j dt
//     nu_m(t_j) = Re <phi_L(t_j)| T_m(Ht) V |phi_R(t_j)>     (pair form of the recurrence)
//   then phi_R, phi_L <- U(dt) (.), U(dt) by its Chebyshev-Bessel series
//     exp(-i H dt/hbar) = exp(-i b dt/hbar) sum_k (2 - delta_k0) (-i)^k J_k(a dt/hbar) T_k(Ht).
// delta(E - H) is the KPM expansion of the DOS, so the correlation at t_j is the
// DOS reconstruction of nu(t_j); the running time integral is the trapezoidal
// rule over the samples (lsqt_sigma in dos.hip).
//
// All vectors live in the builder's row order, [rows][R_pad] interleaved
// complex, like the recurrence's.  The kernels here are plain SELL sweeps with
// one thread per (row, vector) (for block Hamiltonians: per (orbital row,
// vector), over the atom's blocks); the M-1 recurrence steps per time step,
// which dominate, run in the tuned recurrence kernel, for B time steps at a
// time as one recurrence of R * B vectors (the moments of different time steps
// are independent: the phases are propagated B steps ahead and each step's
// start and left vectors take their own columns).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "kpm.hpp"

namespace tbk {
namespace {

constexpr double kHbar = 0.6582119569;   // eV fs
constexpr int kLsqtThreads = 256;

struct SellView {
    const int64_t *ptr;
    const int32_t *col;
    int32_t log2_slice;
};

__device__ __forceinline__ void row_range(const SellView &h, int64_t i, int64_t &base, int32_t &w,
                                          int64_t &stride) {
    const int64_t sl = i >> h.log2_slice;
    stride = (int64_t)1 << h.log2_slice;
    const int64_t p0 = h.ptr[sl], p1 = h.ptr[sl + 1];
    base = p0 + (i & (stride - 1));
    w = (int32_t)((p1 - p0) >> h.log2_slice);
}

// vx[q] = val[q] (x_j - x_i) / hbar for the stored entry q = (row i, column j),
// minimum-image displacement along `axis` between the rows' atoms; 0 on padding.
template <class V>
__global__ void k_velocity(SellView h, const V *__restrict__ val, const int32_t *__restrict__ perm, int32_t n_orb,
                           const double *__restrict__ pos, int64_t n, double L, int32_t periodic, int32_t axis,
                           V *__restrict__ vx) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    int64_t base, stride;
    int32_t w;
    row_range(h, r, base, w, stride);
    const double xi = pos[3 * (int64_t)(perm[r] / n_orb) + axis];
    for (int32_t k = 0; k < w; ++k) {
        const int64_t q = base + k * stride;
        const int32_t c = h.col[q];
        if (c == (int32_t)r) { vx[q] = (V)0; continue; }    // padding (no atom bonds to itself)
        double d = __dsub_rn(pos[3 * (int64_t)(perm[c] / n_orb) + axis], xi);
        if (periodic) d = __dsub_rn(d, __dmul_rn(L, rint(__ddiv_rn(d, L))));
        vx[q] = (V)__ddiv_rn(__dmul_rn((double)val[q], d), kHbar);
    }
}

// Block form: one atom row r per thread; every value of block q (neighbour
// atom col[q]) is scaled by the atoms' displacement (x_j - x_i) / hbar (the
// orbitals sit on their atom); padding blocks (col = own row) stay 0.
template <class V>
__global__ void k_velocity_blk(SellView h, const V *__restrict__ val, const int32_t *__restrict__ perm, int32_t norb,
                               const double *__restrict__ pos, int64_t n_atoms, double L, int32_t periodic,
                               int32_t axis, V *__restrict__ vx) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n_atoms) return;
    int64_t base, stride;
    int32_t w;
    row_range(h, r, base, w, stride);
    const int32_t nb = norb * norb;
    const double xi = pos[3 * (int64_t)(perm[norb * r] / norb) + axis];
    for (int32_t k = 0; k < w; ++k) {
        const int64_t q = base + k * stride;
        const int32_t c = h.col[q];
        double d = 0.0;
        if (c != (int32_t)r) {
            d = __dsub_rn(pos[3 * (int64_t)(perm[(int64_t)norb * c] / norb) + axis], xi);
            if (periodic) d = __dsub_rn(d, __dmul_rn(L, rint(__ddiv_rn(d, L))));
        }
        for (int32_t e = 0; e < nb; ++e)
            vx[nb * q + e] = (V)__ddiv_rn(__dmul_rn((double)val[nb * q + e], d), kHbar);
    }
}

// out[i][v] = r[perm[i]][v] for v < R, 0 for the padded vectors.
template <class VT>
__global__ void k_permute_in(const VT *__restrict__ r, const int32_t *__restrict__ perm, int64_t n, int32_t R,
                             int32_t Rp, VT *__restrict__ out) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * Rp) return;
    const int64_t i = idx / Rp;
    const int v = (int)(idx % Rp);
    VT re = 0, im = 0;
    if (v < R) {
        const int64_t src = 2 * ((int64_t)perm[i] * R + v);
        re = r[src];
        im = r[src + 1];
    }
    out[2 * idx] = re;
    out[2 * idx + 1] = im;
}

// dst[i][col0 + v] = src[i][v] for v < R: one time step's vectors into its
// columns of a batch ([rows][Rpb] interleaved complex, like every vector here).
template <class VT>
__global__ void k_insert_cols(const VT *__restrict__ src, int32_t Rp, int32_t R, int64_t n, int32_t Rpb,
                              int32_t col0, VT *__restrict__ dst) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * R) return;
    const int64_t i = idx / R;
    const int v = (int)(idx % R);
    const int64_t s = 2 * (i * Rp + v), d = 2 * (i * Rpb + col0 + v);
    dst[d] = src[s];
    dst[d + 1] = src[s + 1];
}

template <class VT>
__global__ void k_zero(int64_t m, VT *__restrict__ x) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx < m) x[idx] = (VT)0;
}

// y = V x, (V x)_i = i sum_q vx[q] x_col[q], for Rp vectors; x and y rows hold
// xld and yld vectors (the vectors may be columns of a wider block).
template <class VT>
__global__ void k_apply_velocity(SellView h, const VT *__restrict__ vx, const VT *__restrict__ x, int32_t xld,
                                 int64_t n, int32_t Rp, VT *__restrict__ y, int32_t yld) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * Rp) return;
    const int64_t i = idx / Rp;
    const int v = (int)(idx % Rp);
    int64_t base, stride;
    int32_t w;
    row_range(h, i, base, w, stride);
    VT sr = 0, si = 0;
    for (int32_t k = 0; k < w; ++k) {
        const int64_t q = base + k * stride;
        const VT c = vx[q];
        const int64_t xo = 2 * ((int64_t)h.col[q] * xld + v);
        sr += c * x[xo];
        si += c * x[xo + 1];
    }
    const int64_t yo = 2 * (i * yld + v);
    y[yo] = -si;
    y[yo + 1] = sr;
}

// (A x)_i for orbital row i of a block matrix (values a, norb x norb blocks
// over atom slices), vector v: sum over the atom's blocks and the neighbour's
// orbitals.
template <class VT>
__device__ __forceinline__ void block_row_product(const SellView &h, int32_t norb, const VT *__restrict__ a,
                                                  const VT *__restrict__ x, int64_t i, int v, int32_t Rp, VT &sr,
                                                  VT &si) {
    const int64_t at = i / norb;
    const int32_t orb = (int32_t)(i - at * norb);
    const int32_t nb = norb * norb;
    int64_t base, stride;
    int32_t w;
    row_range(h, at, base, w, stride);
    for (int32_t k = 0; k < w; ++k) {
        const int64_t q = base + k * stride;
        const int64_t c0 = (int64_t)norb * h.col[q];
        const VT *ar = a + nb * q + norb * orb;
        for (int32_t b = 0; b < norb; ++b) {
            const VT hv = ar[b];
            const int64_t xo = 2 * ((c0 + b) * Rp + v);
            sr += hv * x[xo];
            si += hv * x[xo + 1];
        }
    }
}

// y = V x on a block velocity operator (leading dimensions as k_apply_velocity).
template <class VT>
__global__ void k_apply_velocity_blk(SellView h, int32_t norb, const VT *__restrict__ vx, const VT *__restrict__ x,
                                     int32_t xld, int64_t n, int32_t Rp, VT *__restrict__ y, int32_t yld) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * Rp) return;
    const int64_t i = idx / Rp;
    const int v = (int)(idx % Rp);
    VT sr = 0, si = 0;
    block_row_product(h, norb, vx, x, i, v, xld, sr, si);
    const int64_t yo = 2 * (i * yld + v);
    y[yo] = -si;
    y[yo + 1] = sr;
}

// One term of the propagator series (as k_evolve_term) on NORB x NORB blocks,
// a thread per (atom, vector): the thread forms the atom's NORB rows of vector
// v, so each stored block and its column are read once per vector rather than
// once per orbital row, and the NORB rows' sums are independent chains.  tnext
// may alias tprev (a thread reads its own rows' old values before writing).
template <class VT, int NORB, bool FIRST>
__global__ __launch_bounds__(kLsqtThreads) void k_evolve_term_atom(
    SellView h, const VT *__restrict__ val, const VT *__restrict__ onsite, VT shift, VT c1,
    const VT *__restrict__ tcur, const VT *tprev, VT *tnext, VT *__restrict__ acc, double cr, double ci,
    int64_t n_atoms, int32_t Rp) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n_atoms * Rp) return;
    const int64_t at = idx / Rp;
    const int v = (int)(idx % Rp);
    VT yr[NORB], yi[NORB];
    for (int a = 0; a < NORB; ++a) {
        const int64_t i = (int64_t)NORB * at + a;
        const VT d = (onsite ? onsite[i] : (VT)0) - shift;
        yr[a] = d * tcur[2 * (i * Rp + v)];
        yi[a] = d * tcur[2 * (i * Rp + v) + 1];
    }
    int64_t base, stride;
    int32_t w;
    row_range(h, at, base, w, stride);
    for (int32_t k = 0; k < w; ++k) {
        const int64_t q = base + k * stride;
        const int64_t c0 = (int64_t)NORB * h.col[q];
        VT xr[NORB], xi[NORB];
        for (int b = 0; b < NORB; ++b) {
            const int64_t xo = 2 * ((c0 + b) * Rp + v);
            xr[b] = tcur[xo];
            xi[b] = tcur[xo + 1];
        }
        const VT *blk = val + (int64_t)NORB * NORB * q;
        for (int a = 0; a < NORB; ++a)
            for (int b = 0; b < NORB; ++b) {
                const VT hv = blk[NORB * a + b];
                yr[a] += hv * xr[b];
                yi[a] += hv * xi[b];
            }
    }
    for (int a = 0; a < NORB; ++a) {
        const int64_t o = 2 * (((int64_t)NORB * at + a) * Rp + v);
        VT tr = c1 * yr[a], ti = c1 * yi[a];
        if (!FIRST) {
            tr -= tprev[o];
            ti -= tprev[o + 1];
        }
        tnext[o] = tr;
        tnext[o + 1] = ti;
        acc[o] += (VT)(cr * (double)tr - ci * (double)ti);
        acc[o + 1] += (VT)(cr * (double)ti + ci * (double)tr);
    }
}

// One term of the propagator series: tnext = c1 (H - b) tcur - tprev (tprev
// absent on the first term), then acc += (cr + i ci) tnext.  A thread per row
// and pair of vectors (Rp even: phi_R and phi_L side by side), so each stored
// value and column is read once per pair and the pair's gathers are one
// 16-byte (C32) span.  tnext may alias tprev (each element reads its own old
// value before writing).
template <class VT, bool FIRST>
__global__ __launch_bounds__(kLsqtThreads) void k_evolve_term(SellView h, const VT *__restrict__ val,
                                                              const VT *__restrict__ onsite, VT shift, VT c1,
                                                              const VT *__restrict__ tcur, const VT *tprev, VT *tnext,
                                                              VT *__restrict__ acc, double cr, double ci, int64_t n,
                                                              int32_t Rp) {
    const int32_t hp = Rp / 2;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * hp) return;
    const int64_t i = idx / hp;
    const int64_t e = 2 * (i * Rp + 2 * (idx % hp));      // first of the pair's four values
    int64_t base, stride;
    int32_t w;
    row_range(h, i, base, w, stride);
    const VT d = (onsite ? onsite[i] : (VT)0) - shift;
    VT y[4];
    for (int c = 0; c < 4; ++c) y[c] = d * tcur[e + c];
    for (int32_t k = 0; k < w; ++k) {
        const int64_t q = base + k * stride;
        const VT hv = val[q];
        const int64_t xo = 2 * ((int64_t)h.col[q] * Rp) + (e - 2 * i * Rp);
        for (int c = 0; c < 4; ++c) y[c] += hv * tcur[xo + c];
    }
    for (int c = 0; c < 4; c += 2) {
        VT tr = c1 * y[c], ti = c1 * y[c + 1];
        if (!FIRST) {
            tr -= tprev[e + c];
            ti -= tprev[e + c + 1];
        }
        tnext[e + c] = tr;
        tnext[e + c + 1] = ti;
        acc[e + c] += (VT)(cr * (double)tr - ci * (double)ti);
        acc[e + c + 1] += (VT)(cr * (double)ti + ci * (double)tr);
    }
}

// y = (cr + i ci) x
template <class VT>
__global__ void k_cscale(const VT *__restrict__ x, double cr, double ci, int64_t m, VT *__restrict__ y) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= m) return;
    const double xr = x[2 * idx], xi = x[2 * idx + 1];
    y[2 * idx] = (VT)(cr * xr - ci * xi);
    y[2 * idx + 1] = (VT)(cr * xi + ci * xr);
}

__global__ void k_all_finite(const double *__restrict__ x, int64_t m, int32_t *__restrict__ flag) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx < m && !isfinite(x[idx])) *flag = 1;
}

int32_t log2_of(int32_t v) {
    int32_t l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Terms of the Chebyshev-Bessel series of exp(-i H dt/hbar): the first k past
// z = a dt/hbar with |J_k(z)| below 1e-15 (J_k decays faster than geometrically there).
int32_t default_terms(double z) {
    int32_t k = 1;
    while (k < 100000 && !(k > z && std::fabs(::jn(k, z)) < 1e-15)) ++k;
    return k + 1;
}

// Time steps whose recurrences run together as one recurrence of R * B vectors
// (their moments are independent, so batching only changes the summation
// tiling): 0 picks B = max(1, 16 / R).
int32_t time_batch_of(int32_t R, int32_t time_batch) {
    return time_batch > 0 ? time_batch : std::max(1, 16 / R);
}

struct LsqtLayout {
    KpmPlan pl;                 // recurrence of R * B vectors (B time steps)
    int32_t B = 1;              // time steps per recurrence
    size_t vec = 0, off_vec = 0;        // [rows][R_pad] vector units after the recurrence workspace
    size_t bvec = 0, off_batch = 0;     // start and left vectors of a batch, [rows][pad(R B)]
    size_t off_mu = 0, total = 0;       // a batch's moments [R B][M]
};

tbk_status make_layout(const tbk_ham *h, int32_t R, int32_t M, int32_t precision, int32_t time_batch,
                       const tbk_kpm_config *cfg, LsqtLayout &ly) {
    TBK_CHECK(R >= 1 && R <= 64, TBK_ERR_INVALID_ARG, "R = %d outside [1, 64]", R);
    TBK_CHECK(time_batch >= 0, TBK_ERR_INVALID_ARG, "time_batch = %d < 0", time_batch);
    ly.B = time_batch_of(R, time_batch);
    TBK_CHECK((int64_t)R * ly.B <= 64, TBK_ERR_INVALID_ARG, "R * time_batch = %lld exceeds 64 vectors",
              (long long)R * ly.B);
    tbk_status st = make_plan(h, R * ly.B, M, precision, cfg, ly.pl);
    if (st != TBK_OK) return st;
    TBK_CHECK(ly.pl.cfg.doubling == 0, TBK_ERR_INVALID_ARG,
              "the doubling identities need the same left and right vectors; VAC moments use the direct form");
    TBK_CHECK(h->n_seg == 1, TBK_ERR_UNSUPPORTED, "VAC conductivity takes one structure");
    TBK_CHECK(!ly.pl.geom, TBK_ERR_UNSUPPORTED, "VAC conductivity takes stored blocks, not the displacement form");
    TBK_CHECK(!ly.pl.block || ly.pl.norb == 4 || ly.pl.norb == 9, TBK_ERR_UNSUPPORTED,
              "VAC conductivity takes blocks of 4 or 9 orbitals, not %d", ly.pl.norb);
    TBK_CHECK(h->fmt != TBK_CSR_F64 || h->slice == 1, TBK_ERR_INVALID_ARG, "CSR needs slice 1");
    const size_t elem = precision == TBK_PREC_C32 ? sizeof(float) : sizeof(double);
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    ly.vec = a256((size_t)h->n_rows * pad_vectors(R) * 2 * elem);
    ly.off_vec = a256(ly.pl.total);
    ly.off_batch = ly.off_vec + 9 * ly.vec;
    ly.bvec = a256((size_t)h->n_rows * ly.pl.Rp * 2 * elem);
    ly.off_mu = ly.off_batch + 2 * ly.bvec;
    ly.total = ly.off_mu + a256((size_t)R * ly.B * M * sizeof(double));
    return TBK_OK;
}

template <class VT>
tbk_status run_vac(const tbk_ham *h, const VT *vx, double a, double b, const VT *r, int32_t R, int32_t M,
                   int32_t n_t, double dt, int32_t n_cheb, int32_t precision, const LsqtLayout &ly, char *work,
                   double *nu, hipStream_t s) {
    const KpmPlan &pl = ly.pl;
    const int32_t Rp = pad_vectors(R);
    const int32_t R2 = 2 * Rp;      // phi_R and phi_L side by side: both propagate in one sweep
    const int64_t n = h->n_rows;
    // vector units of [rows][Rp]: the [rows][2 Rp] blocks phi = (phi_R | phi_L), e1, e2, acc of the
    // propagation, and w = V phi_R
    auto unit = [&](int k) { return reinterpret_cast<VT *>(work + ly.off_vec + k * ly.vec); };
    VT *phi = unit(0), *e1 = unit(2), *e2 = unit(4), *acc = unit(6), *wv = unit(8);
    VT *phiL = phi + 2 * Rp;        // column Rp of phi
    const SellView sv{h->ptr, h->col, log2_of(h->fmt == TBK_CSR_F64 ? 1 : h->slice)};
    const VT *val = static_cast<const VT *>(h->val);
    const VT *ons = h->has_onsite ? static_cast<const VT *>(h->onsite) : nullptr;
    const int64_t nv = n * Rp, nv2 = n * R2;
    const unsigned g = (unsigned)ceil_div(nv, kLsqtThreads), g2 = (unsigned)ceil_div(nv2, kLsqtThreads);
    const unsigned gp = (unsigned)ceil_div(n * Rp, kLsqtThreads);     // a thread per row and pair of vectors

    // series coefficients of U(dt)
    const double z = a * dt / kHbar;
    std::vector<double> cre(n_cheb), cim(n_cheb);
    for (int32_t k = 0; k < n_cheb; ++k) {
        const double jk = (k == 0 ? 1.0 : 2.0) * ::jn(k, z);
        // (-i)^k: 1, -i, -1, i
        const int q = k & 3;
        cre[k] = q == 0 ? jk : (q == 2 ? -jk : 0.0);
        cim[k] = q == 1 ? -jk : (q == 3 ? jk : 0.0);
    }
    const double pr = std::cos(b * dt / kHbar), pi = -std::sin(b * dt / kHbar);   // exp(-i b dt / hbar)

    const bool blk = pl.block;
    const int32_t norb = pl.norb;
    auto term = [&](bool first, VT c1, const VT *tcur, const VT *tprev, VT *tnext, int32_t k) {
        if (blk) {
            const int64_t na = n / norb;
            const unsigned ga = (unsigned)ceil_div(na * R2, kLsqtThreads);
            if (norb == 4 && first)
                k_evolve_term_atom<VT, 4, true><<<ga, kLsqtThreads, 0, s>>>(sv, val, ons, (VT)b, c1, tcur, tprev,
                                                                             tnext, acc, cre[k], cim[k], na, R2);
            else if (norb == 4)
                k_evolve_term_atom<VT, 4, false><<<ga, kLsqtThreads, 0, s>>>(sv, val, ons, (VT)b, c1, tcur, tprev,
                                                                              tnext, acc, cre[k], cim[k], na, R2);
            else if (first)
                k_evolve_term_atom<VT, 9, true><<<ga, kLsqtThreads, 0, s>>>(sv, val, ons, (VT)b, c1, tcur, tprev,
                                                                             tnext, acc, cre[k], cim[k], na, R2);
            else
                k_evolve_term_atom<VT, 9, false><<<ga, kLsqtThreads, 0, s>>>(sv, val, ons, (VT)b, c1, tcur, tprev,
                                                                              tnext, acc, cre[k], cim[k], na, R2);
        } else {
            if (first)
                k_evolve_term<VT, true><<<gp, kLsqtThreads, 0, s>>>(sv, val, ons, (VT)b, c1, tcur, tprev, tnext, acc,
                                                                     cre[k], cim[k], n, R2);
            else
                k_evolve_term<VT, false><<<gp, kLsqtThreads, 0, s>>>(sv, val, ons, (VT)b, c1, tcur, tprev, tnext,
                                                                      acc, cre[k], cim[k], n, R2);
        }
    };
    // y = V x for the Rp vectors of x (rows of xld vectors) into y (rows of yld vectors)
    auto apply_v = [&](const VT *x, int32_t xld, VT *y, int32_t yld) {
        if (blk) k_apply_velocity_blk<VT><<<g, kLsqtThreads, 0, s>>>(sv, norb, vx, x, xld, n, Rp, y, yld);
        else k_apply_velocity<VT><<<g, kLsqtThreads, 0, s>>>(sv, vx, x, xld, n, Rp, y, yld);
    };

    // phi_R and phi_L <- U(dt) (.), together
    auto evolve = [&]() -> tbk_status {
        k_cscale<VT><<<g2, kLsqtThreads, 0, s>>>(phi, cre[0], cim[0], nv2, acc);
        if (n_cheb > 1) term(true, (VT)(1.0 / a), phi, nullptr, e1, 1);
        for (int32_t k = 2; k < n_cheb; ++k) {
            const VT *tcur = (k & 1) ? e2 : e1;
            const VT *tprev = k == 2 ? phi : ((k & 1) ? e1 : e2);
            VT *tnext = (k & 1) ? e1 : e2;
            term(false, (VT)(2.0 / a), tcur, tprev, tnext, k);
        }
        k_cscale<VT><<<g2, kLsqtThreads, 0, s>>>(acc, pr, pi, nv2, phi);
        TBK_HIP(hipGetLastError());
        return TBK_OK;
    };

    // phi_R(0) = r (padded vectors zero), phi_L(0) = V phi_R(0)
    k_permute_in<VT><<<g, kLsqtThreads, 0, s>>>(r, h->perm, n, R, Rp, wv);
    k_insert_cols<VT><<<g, kLsqtThreads, 0, s>>>(wv, Rp, Rp, n, R2, 0, phi);
    apply_v(phi, R2, phiL, R2);
    TBK_HIP(hipGetLastError());
    // B time steps at a time: V phi_R(t_j) and phi_L(t_j) of each step go into columns
    // q R .. q R + R - 1 of the batch's start and left vectors (unused columns of a
    // short last batch stay zero), then one pair-form recurrence of R B vectors gives
    // the batch's moments [q][v][m] = nu[j0 + q][v][m]
    const int32_t Rb = pl.Rp;
    VT *start = reinterpret_cast<VT *>(work + ly.off_batch);
    VT *left = reinterpret_cast<VT *>(work + ly.off_batch + ly.bvec);
    double *mub = reinterpret_cast<double *>(work + ly.off_mu);
    const int64_t nb_el = 2 * n * (int64_t)Rb;
    const unsigned gz = (unsigned)ceil_div(nb_el, kLsqtThreads);
    const unsigned gi = (unsigned)ceil_div(n * R, kLsqtThreads);
    for (int32_t j0 = 0; j0 < n_t; j0 += ly.B) {
        const int32_t nb = std::min(ly.B, n_t - j0);
        if (nb * R < Rb) {
            k_zero<VT><<<gz, kLsqtThreads, 0, s>>>(nb_el, start);
            k_zero<VT><<<gz, kLsqtThreads, 0, s>>>(nb_el, left);
        }
        for (int32_t q = 0; q < nb; ++q) {
            apply_v(phi, R2, wv, Rp);
            k_insert_cols<VT><<<gi, kLsqtThreads, 0, s>>>(wv, Rp, R, n, Rb, q * R, start);
            k_insert_cols<VT><<<gi, kLsqtThreads, 0, s>>>(phiL, R2, R, n, Rb, q * R, left);
            TBK_HIP(hipGetLastError());
            if (j0 + q + 1 < n_t) {
                tbk_status st = evolve();
                if (st != TBK_OK) return st;
            }
        }
        tbk_status st = run_plan(h, pl, a, b, nullptr, R * ly.B, M, precision, work, mub, s, start, left);
        if (st != TBK_OK) return st;
        TBK_HIP(hipMemcpyAsync(nu + (int64_t)j0 * R * M, mub, sizeof(double) * (size_t)nb * R * M,
                               hipMemcpyDeviceToDevice, s));
    }
    DevBuf flag;
    TBK_HIP(flag.alloc(sizeof(int32_t), s));
    TBK_HIP(hipMemsetAsync(flag.as<int32_t>(), 0, sizeof(int32_t), s));
    const int64_t m = (int64_t)n_t * R * M;
    k_all_finite<<<(unsigned)ceil_div(m, 256), 256, 0, s>>>(nu, m, flag.as<int32_t>());
    TBK_HIP(hipGetLastError());
    int32_t hf = 0;
    TBK_HIP(hipMemcpyAsync(&hf, flag.as<int32_t>(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    TBK_CHECK(hf == 0, TBK_ERR_SPECTRUM, "a correlation moment is not finite: (a, b) does not bound the spectrum");
    return TBK_OK;
}

}  // namespace
}  // namespace tbk

using namespace tbk;

extern "C" int32_t lsqt_chebyshev_terms(double a, double dt) {
    if (!(a > 0.0) || !(dt >= 0.0) || !std::isfinite(a * dt)) return -1;
    return default_terms(a * dt / kHbar);
}

extern "C" tbk_status tb_build_velocity(const double *pos, const double box[3], const int32_t periodic[3],
                                        int32_t axis, const tbk_ham *h, void *vx, void *stream) {
    clear_error();
    TBK_CHECK(pos && box && periodic && h && vx, TBK_ERR_INVALID_ARG, "NULL argument");
    TBK_CHECK(axis >= 0 && axis <= 2, TBK_ERR_INVALID_ARG, "axis = %d not in {0, 1, 2}", axis);
    TBK_CHECK(h->n_seg == 1, TBK_ERR_UNSUPPORTED, "the velocity operator is built for one structure");
    TBK_CHECK(h->fmt != TBK_BGEOM_F64 && h->fmt != TBK_BGEOM_F32, TBK_ERR_UNSUPPORTED,
              "the velocity operator is built for stored values, not the displacement form");
    TBK_CHECK(h->fmt == TBK_CSR_F64 || h->fmt == TBK_SELL_F64 || h->fmt == TBK_SELL_F32 ||
                  h->fmt == TBK_BSELL4_F64 || h->fmt == TBK_BSELL4_F32,
              TBK_ERR_INVALID_ARG, "unknown format %d", h->fmt);
    const bool blk = h->fmt == TBK_BSELL4_F64 || h->fmt == TBK_BSELL4_F32;
    TBK_CHECK(!blk || ((h->n_orb == 4 || h->n_orb == 9) && h->n_rows % h->n_orb == 0), TBK_ERR_INVALID_ARG,
              "a block Hamiltonian has 4 or 9 orbital rows per atom (n_orb = %d)", h->n_orb);
    TBK_CHECK(h->ptr && h->col && h->val && h->perm, TBK_ERR_INVALID_ARG, "a Hamiltonian array is NULL");
    TBK_CHECK(!periodic[axis] || (std::isfinite(box[axis]) && box[axis] > 0), TBK_ERR_INVALID_ARG,
              "periodic length along axis %d must be positive", axis);
    if (h->n_rows == 0) return TBK_OK;
    hipStream_t s = as_stream(stream);
    const SellView sv{h->ptr, h->col, log2_of(h->fmt == TBK_CSR_F64 ? 1 : h->slice)};
    const unsigned g = (unsigned)ceil_div(h->n_rows, kLsqtThreads);
    const int32_t n_orb = h->n_orb >= 1 ? h->n_orb : 1;
    if (blk) {
        const int64_t na = h->n_rows / n_orb;
        const unsigned ga = (unsigned)ceil_div(na, kLsqtThreads);
        if (h->fmt == TBK_BSELL4_F32)
            k_velocity_blk<float><<<ga, kLsqtThreads, 0, s>>>(sv, static_cast<const float *>(h->val), h->perm, n_orb,
                                                              pos, na, box[axis], periodic[axis], axis,
                                                              static_cast<float *>(vx));
        else
            k_velocity_blk<double><<<ga, kLsqtThreads, 0, s>>>(sv, static_cast<const double *>(h->val), h->perm,
                                                               n_orb, pos, na, box[axis], periodic[axis], axis,
                                                               static_cast<double *>(vx));
    } else if (h->fmt == TBK_SELL_F32)
        k_velocity<float><<<g, kLsqtThreads, 0, s>>>(sv, static_cast<const float *>(h->val), h->perm, n_orb, pos,
                                                     h->n_rows, box[axis], periodic[axis], axis,
                                                     static_cast<float *>(vx));
    else
        k_velocity<double><<<g, kLsqtThreads, 0, s>>>(sv, static_cast<const double *>(h->val), h->perm, n_orb, pos,
                                                      h->n_rows, box[axis], periodic[axis], axis,
                                                      static_cast<double *>(vx));
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

extern "C" tbk_status lsqt_workspace_size(const tbk_ham *h, int32_t R, int32_t M, int32_t precision,
                                          int32_t time_batch, const tbk_kpm_config *cfg, int64_t *bytes) {
    clear_error();
    TBK_CHECK(bytes != nullptr, TBK_ERR_INVALID_ARG, "bytes is NULL");
    LsqtLayout ly;
    tbk_status st = make_layout(h, R, M, precision, time_batch, cfg, ly);
    if (st != TBK_OK) return st;
    *bytes = (int64_t)ly.total;
    return TBK_OK;
}

extern "C" tbk_status lsqt_vac_moments(const tbk_ham *h, const void *vx, double a, double b, const void *r,
                                       int32_t R, int32_t M, int32_t n_t, double dt, int32_t n_cheb,
                                       int32_t precision, int32_t time_batch, const tbk_kpm_config *cfg,
                                       void *work, int64_t work_bytes, double *nu, void *stream) {
    clear_error();
    TBK_CHECK(h && vx && r && work && nu, TBK_ERR_INVALID_ARG, "NULL argument");
    TBK_CHECK(std::isfinite(a) && std::isfinite(b) && std::isfinite(dt), TBK_ERR_NOT_FINITE,
              "a, b or dt is not finite");
    TBK_CHECK(a > 0 && dt > 0, TBK_ERR_INVALID_ARG, "a = %g and dt = %g must be positive", a, dt);
    TBK_CHECK(n_t >= 1 && n_t <= 1000000, TBK_ERR_INVALID_ARG, "n_t = %d outside [1, 10^6]", n_t);
    if (n_cheb <= 0) n_cheb = default_terms(a * dt / kHbar);
    TBK_CHECK(n_cheb <= 100000, TBK_ERR_INVALID_ARG, "n_cheb = %d too large", n_cheb);
    LsqtLayout ly;
    tbk_status st = make_layout(h, R, M, precision, time_batch, cfg, ly);
    if (st != TBK_OK) return st;
    TBK_CHECK(work_bytes >= (int64_t)ly.total, TBK_ERR_BUFFER_TOO_SMALL, "work has %lld bytes, needs %lld",
              (long long)work_bytes, (long long)ly.total);
    TBK_CHECK(((uintptr_t)work & 255) == 0, TBK_ERR_INVALID_ARG, "work is not 256-byte aligned");
    hipStream_t s = as_stream(stream);
    char *w = static_cast<char *>(work);
    if (precision == TBK_PREC_C32)
        return run_vac<float>(h, static_cast<const float *>(vx), a, b, static_cast<const float *>(r), R, M, n_t, dt,
                              n_cheb, precision, ly, w, nu, s);
    return run_vac<double>(h, static_cast<const double *>(vx), a, b, static_cast<const double *>(r), R, M, n_t, dt,
                           n_cheb, precision, ly, w, nu, s);
}
