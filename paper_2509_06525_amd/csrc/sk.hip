// Multi-orbital Slater-Koster Hamiltonian (s, px, py, pz per atom) on the GPU.
//
// The paper's models attach several orbitals to each atom and form every
// atom-pair block from two-centre integrals and the bond direction (the SK
// conversion P_lambda(r_ij) of Sec. 3).  Here the s and p rows of the
// Slater-Koster table (Phys. Rev. 94, 1498 (1954), Table I) with one radial
// factor f(r) = exp(-beta (r/r0 - 1)) for every integral:
//   <s_i|s_j> = f V_ss_sigma, <s_i|p_j,b> = f c_b V_sp_sigma, <p_i,a|s_j> = -f c_a V_sp_sigma,
//   <p_i,a|p_j,b> = f [c_a c_b V_pp_sigma + (delta_ab - c_a c_b) V_pp_pi],
// c = bond direction cosines from i to j (minimum image).
//
// The orbital Hamiltonian (row 4 r + a for atom row r, orbital a = s, x, y, z)
// is stored either as an ordinary SELL matrix with 4 N rows (the recurrence,
// the DOS and the VAC path run on it unchanged) or as a block SELL over atoms
// with one 4x4 block per bond (a quarter of the column traffic; the block
// recurrence kernel in kpm_block.hip).  The neighbour search, the atom row
// order and the atom degrees come from the one-orbital builder's plan.
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <vector>

#include "builder.hpp"
#include "nlist.hpp"

namespace tbk {
namespace {

// entries[s] = C * max over the orbital rows of slice s of 4 * deg(atom row).
__global__ void k_sk_width(int64_t n_orb_rows, int32_t slice, int64_t n_slices, const int32_t *__restrict__ deg,
                           int64_t *__restrict__ entries) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    int32_t w = 0;
    const int64_t r1 = min((s + 1) * (int64_t)slice, n_orb_rows);
    for (int64_t R = s * (int64_t)slice; R < r1; ++R) w = max(w, 4 * deg[R >> 2]);
    entries[s] = (int64_t)slice * w;
}

// perm_orb[4 r + a] = 4 perm[r] + a
__global__ void k_sk_perm(int64_t n, const int32_t *__restrict__ perm, int32_t *__restrict__ perm_orb) {
    const int64_t R = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (R >= 4 * n) return;
    perm_orb[R] = 4 * perm[R >> 2] + (int32_t)(R & 3);
}

struct SkValues {
    double r0, beta, e_s, e_p;
    double v[4];   // V_ss_sigma, V_sp_sigma, V_pp_sigma, V_pp_pi at r0
};

// The 4x4 block of a bond of length r and vector (dx, dy, dz) from the row atom.
__device__ __forceinline__ void sk_block(const SkValues &sk, double r, double dx, double dy, double dz,
                                         double (&B)[4][4]) {
    const double c[3] = {dx / r, dy / r, dz / r};
    const double f = exp(-sk.beta * (r / sk.r0 - 1.0));
    B[0][0] = f * sk.v[0];
    for (int b = 0; b < 3; ++b) {
        B[0][b + 1] = f * c[b] * sk.v[1];
        B[b + 1][0] = -f * c[b] * sk.v[1];
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            B[a + 1][b + 1] = f * (c[a] * c[b] * sk.v[2] + ((a == b ? 1.0 : 0.0) - c[a] * c[b]) * sk.v[3]);
}

// One atom row r per thread: its four orbital rows, entry 4 q + b for the q-th
// neighbour (cell-list order) and its orbital b; padding (own row, value 0)
// up to the slice width; onsite; row Gershgorin bounds; 16-bit offsets.
template <class V>
__global__ void k_fill_sk(CellList cl, const double *__restrict__ pos, int64_t n, int32_t slice,
                          int32_t log2_slice, double r_cut, SkValues sk, const int32_t *__restrict__ perm,
                          const int32_t *__restrict__ iperm, const int64_t *__restrict__ ptr,
                          int32_t *__restrict__ col, V *__restrict__ val, V *__restrict__ onsite,
                          int16_t *__restrict__ col16, int64_t *__restrict__ bound_keys) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (r < n) {
        int64_t base[4];
        int32_t w[4];
        for (int a = 0; a < 4; ++a) {
            const int64_t R = 4 * r + a;
            const int64_t sl = R >> log2_slice;
            base[a] = ptr[sl] + (R & (slice - 1));
            w[a] = (int32_t)((ptr[sl + 1] - ptr[sl]) >> log2_slice);
        }
        const int32_t i = perm[r];
        double asum[4] = {0.0, 0.0, 0.0, 0.0};
        int32_t q = 0;
        for_each_neighbor(cl, pos, i, r_cut, [&](int32_t j, double rij, double dx, double dy, double dz) {
            double B[4][4];
            sk_block(sk, rij, dx, dy, dz, B);
            const int32_t cj = 4 * iperm[j];
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    const int32_t k = 4 * q + b;
                    if (k < w[a]) {
                        col[base[a] + (int64_t)k * slice] = cj + b;
                        val[base[a] + (int64_t)k * slice] = (V)B[a][b];
                    }
                    asum[a] += fabs(B[a][b]);
                }
            ++q;
        });
        for (int a = 0; a < 4; ++a) {
            const int64_t R = 4 * r + a;
            for (int32_t k = 4 * q; k < w[a]; ++k) {
                col[base[a] + (int64_t)k * slice] = (int32_t)R;
                val[base[a] + (int64_t)k * slice] = (V)0;
            }
            if (col16)
                for (int32_t k = 0; k < w[a]; ++k) {
                    const int64_t d = (int64_t)col[base[a] + (int64_t)k * slice] - R;
                    col16[base[a] + (int64_t)k * slice] =
                        (d >= -32767 && d <= 32767) ? (int16_t)d : (int16_t)-32768;
                }
            const double e = a == 0 ? sk.e_s : sk.e_p;
            onsite[R] = (V)e;
            lo = fmin(lo, e - asum[a]);
            hi = fmax(hi, e + asum[a]);
        }
    }
    block_segment_bounds(lo, hi, r < n ? 0 : -1, bound_keys);
}

// Block form: one atom row r per thread; block q (q-th neighbour, cell-list
// order) at slot base + q C of the atom slice, its 16 values row-major at
// 16 (base + q C); padding blocks (own row, zero) up to the slice width.
template <class V>
__global__ void k_fill_sk_blk(CellList cl, const double *__restrict__ pos, int64_t n, int32_t slice,
                              int32_t log2_slice, double r_cut, SkValues sk, const int32_t *__restrict__ perm,
                              const int32_t *__restrict__ iperm, const int64_t *__restrict__ ptr,
                              int32_t *__restrict__ bcol, V *__restrict__ bval, V *__restrict__ onsite,
                              int64_t *__restrict__ bound_keys) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (r < n) {
        const int64_t sl = r >> log2_slice;
        const int64_t base = ptr[sl] + (r & (slice - 1));
        const int32_t w = (int32_t)((ptr[sl + 1] - ptr[sl]) >> log2_slice);
        const int32_t i = perm[r];
        double asum[4] = {0.0, 0.0, 0.0, 0.0};
        int32_t q = 0;
        for_each_neighbor(cl, pos, i, r_cut, [&](int32_t j, double rij, double dx, double dy, double dz) {
            double B[4][4];
            sk_block(sk, rij, dx, dy, dz, B);
            if (q < w) {
                const int64_t slot = base + (int64_t)q * slice;
                bcol[slot] = iperm[j];
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) bval[16 * slot + 4 * a + b] = (V)B[a][b];
            }
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) asum[a] += fabs(B[a][b]);
            ++q;
        });
        for (int32_t k = q; k < w; ++k) {
            const int64_t slot = base + (int64_t)k * slice;
            bcol[slot] = (int32_t)r;
            for (int e = 0; e < 16; ++e) bval[16 * slot + e] = (V)0;
        }
        for (int a = 0; a < 4; ++a) {
            const double e = a == 0 ? sk.e_s : sk.e_p;
            onsite[4 * r + a] = (V)e;
            lo = fmin(lo, e - asum[a]);
            hi = fmax(hi, e + asum[a]);
        }
    }
    block_segment_bounds(lo, hi, r < n ? 0 : -1, bound_keys);
}

bool is_block(int32_t fmt) { return fmt == TBK_BSELL4_F64 || fmt == TBK_BSELL4_F32; }

tbk_status check_sk(const tbk_sk_params *sk) {
    TBK_CHECK(sk != nullptr, TBK_ERR_INVALID_ARG, "sk params are NULL");
    const double x[9] = {sk->r_cut, sk->r0, sk->beta, sk->e_s, sk->e_p,
                         sk->v_ss_sigma, sk->v_sp_sigma, sk->v_pp_sigma, sk->v_pp_pi};
    for (double v : x) TBK_CHECK(std::isfinite(v), TBK_ERR_NOT_FINITE, "an SK parameter is not finite");
    return TBK_OK;
}

// One-orbital plan of the atoms (cell list, row order, atom degrees) for the SK builder.
tbk_status atom_plan(const double *pos, const int32_t *species, int64_t n, const double box[3],
                     const int32_t periodic[3], const tbk_sk_params *sk, int32_t atom_slice, HamPlan &plan,
                     hipStream_t s) {
    tbk_status st = check_sk(sk);
    if (st != TBK_OK) return st;
    TBK_CHECK(box != nullptr, TBK_ERR_INVALID_ARG, "box is NULL");
    TBK_CHECK(n >= 1 && 4 * n < (int64_t)INT32_MAX, TBK_ERR_INVALID_ARG, "4 n = %lld orbital rows out of range",
              (long long)(4 * n));
    const double onsite0 = 0.0, t0 = 1.0;
    tbk_tb_params p{};
    p.r_cut = sk->r_cut;
    p.r0 = sk->r0;
    p.beta = sk->beta;
    p.n_species = 1;
    p.reorder = sk->reorder;
    p.onsite = &onsite0;
    p.t_pair = &t0;
    const int64_t seg[2] = {0, n};
    return plan.run(pos, species, n, 1, seg, box, periodic, &p, TBK_SELL_F64, atom_slice, s);
}

struct SkLayout {
    int64_t n_slices = 0, n_entries = 0;
    int32_t max_w = 0;
    DevBuf ptr;
};

tbk_status sk_layout(const HamPlan &plan, int64_t n, int32_t slice, SkLayout &ly, hipStream_t s) {
    const int64_t nr = 4 * n;
    ly.n_slices = ceil_div(nr, slice);
    DevBuf entries;
    TBK_HIP(entries.alloc(sizeof(int64_t) * (ly.n_slices + 1), s));
    TBK_HIP(ly.ptr.alloc(sizeof(int64_t) * (ly.n_slices + 1), s));
    TBK_HIP(hipMemsetAsync(entries.as<int64_t>() + ly.n_slices, 0, sizeof(int64_t), s));
    k_sk_width<<<(unsigned)ceil_div(ly.n_slices, kBlock), kBlock, 0, s>>>(nr, slice, ly.n_slices,
                                                                           plan.deg.as<int32_t>(),
                                                                           entries.as<int64_t>());
    TBK_HIP(hipGetLastError());
    size_t tmp = 0;
    TBK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, entries.as<int64_t>(), ly.ptr.as<int64_t>(),
                                             (int)(ly.n_slices + 1), s));
    DevBuf t;
    TBK_HIP(t.alloc(tmp, s));
    TBK_HIP(hipcub::DeviceScan::ExclusiveSum(t.as<void>(), tmp, entries.as<int64_t>(), ly.ptr.as<int64_t>(),
                                             (int)(ly.n_slices + 1), s));
    int64_t total = 0;
    TBK_HIP(hipMemcpyAsync(&total, ly.ptr.as<int64_t>() + ly.n_slices, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    ly.n_entries = total;
    ly.max_w = 4 * plan.max_degree;
    return TBK_OK;
}

int32_t log2i(int32_t v) {
    int32_t l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

tbk_status set_sk_sizes(int64_t n, const HamPlan &plan, const SkLayout &ly, const tbk_sk_params *sk, tbk_ham *h) {
    h->n_rows = 4 * n;
    if (is_block(h->fmt)) {      // blocks over atom slices
        h->n_ptr = plan.n_slices + 1;
        h->n_entries = plan.n_entries;
        h->max_degree = plan.max_degree;
    } else {
        h->n_ptr = ly.n_slices + 1;
        h->n_entries = ly.n_entries;
        h->max_degree = ly.max_w;
    }
    h->n_bonds = plan.n_bonds;
    h->has_onsite = (sk->e_s != 0.0 || sk->e_p != 0.0) ? 1 : 0;
    h->n_seg = 1;
    h->n_orb = 4;
    h->uniform_hop = 0;
    h->hop_value = 0.0;
    return TBK_OK;
}

}  // namespace
}  // namespace tbk

using namespace tbk;

extern "C" tbk_status tbk_hamiltonian_size_sk(const double *pos, const int32_t *species, int64_t n,
                                              const double box[3], const int32_t periodic[3],
                                              const tbk_sk_params *sk, tbk_ham *h, void *stream) {
    clear_error();
    TBK_CHECK(h != nullptr, TBK_ERR_INVALID_ARG, "h is NULL");
    TBK_CHECK(h->fmt == TBK_SELL_F32 || h->fmt == TBK_SELL_F64 || h->fmt == TBK_CSR_F64 || is_block(h->fmt),
              TBK_ERR_INVALID_ARG, "unknown format %d", h->fmt);
    const int32_t slice = h->fmt == TBK_CSR_F64 ? 1 : h->slice;
    TBK_CHECK(slice >= 1 && slice <= 1024 && (slice & (slice - 1)) == 0, TBK_ERR_INVALID_ARG,
              "slice = %d is not a power of two in [1, 1024]", slice);
    hipStream_t s = as_stream(stream);
    HamPlan plan;
    tbk_status st = atom_plan(pos, species, n, box, periodic, sk, is_block(h->fmt) ? slice : 1, plan, s);
    if (st != TBK_OK) return st;
    SkLayout ly;
    if (!is_block(h->fmt)) {
        st = sk_layout(plan, n, slice, ly, s);
        if (st != TBK_OK) return st;
    }
    if (h->fmt == TBK_CSR_F64) h->slice = 1;
    return set_sk_sizes(n, plan, ly, sk, h);
}

extern "C" tbk_status tb_build_hamiltonian_sk(const double *pos, const int32_t *species, int64_t n,
                                              const double box[3], const int32_t periodic[3],
                                              const tbk_sk_params *sk, tbk_ham *h, double spec_bounds[2],
                                              void *stream) {
    clear_error();
    TBK_CHECK(h != nullptr && spec_bounds != nullptr, TBK_ERR_INVALID_ARG, "h or bounds is NULL");
    TBK_CHECK(h->fmt == TBK_SELL_F32 || h->fmt == TBK_SELL_F64 || h->fmt == TBK_CSR_F64 || is_block(h->fmt),
              TBK_ERR_INVALID_ARG, "unknown format %d", h->fmt);
    const int32_t slice = h->fmt == TBK_CSR_F64 ? 1 : h->slice;
    TBK_CHECK(slice >= 1 && slice <= 1024 && (slice & (slice - 1)) == 0, TBK_ERR_INVALID_ARG,
              "slice = %d is not a power of two in [1, 1024]", slice);
    hipStream_t s = as_stream(stream);
    HamPlan plan;
    const bool blk = is_block(h->fmt);
    tbk_status st = atom_plan(pos, species, n, box, periodic, sk, blk ? slice : 1, plan, s);
    if (st != TBK_OK) return st;
    SkLayout ly;
    if (blk) {
        ly.n_slices = plan.n_slices;
        ly.n_entries = plan.n_entries;
    } else {
        st = sk_layout(plan, n, slice, ly, s);
        if (st != TBK_OK) return st;
    }
    TBK_CHECK(h->n_rows >= 4 * n && h->n_ptr >= ly.n_slices + 1 && h->n_entries >= ly.n_entries,
              TBK_ERR_BUFFER_TOO_SMALL, "buffers sized for n_rows=%lld n_ptr=%lld n_entries=%lld; need %lld, %lld, %lld",
              (long long)h->n_rows, (long long)h->n_ptr, (long long)h->n_entries, (long long)(4 * n),
              (long long)(ly.n_slices + 1), (long long)ly.n_entries);
    TBK_CHECK(h->ptr && h->col && h->val && h->onsite && h->perm, TBK_ERR_INVALID_ARG,
              "a Hamiltonian array pointer is NULL");
    TBK_HIP(hipMemcpyAsync(h->ptr, blk ? plan.ptr.as<int64_t>() : ly.ptr.as<int64_t>(),
                           sizeof(int64_t) * (ly.n_slices + 1), hipMemcpyDeviceToDevice, s));
    k_sk_perm<<<(unsigned)ceil_div(4 * n, kBlock), kBlock, 0, s>>>(n, plan.perm.as<int32_t>(), h->perm);
    TBK_HIP(hipGetLastError());
    DevBuf keys;
    st = init_bound_keys(keys, 1, s);
    if (st != TBK_OK) return st;
    SkValues v{sk->r0, sk->beta, sk->e_s, sk->e_p, {sk->v_ss_sigma, sk->v_sp_sigma, sk->v_pp_sigma, sk->v_pp_pi}};
    const unsigned g = (unsigned)ceil_div(n, kBlock);
    if (blk) {
        if (h->fmt == TBK_BSELL4_F32)
            k_fill_sk_blk<float><<<g, kBlock, 0, s>>>(plan.cells.view, pos, n, slice, log2i(slice), sk->r_cut, v,
                                                      plan.perm.as<int32_t>(), plan.iperm.as<int32_t>(), h->ptr,
                                                      h->col, static_cast<float *>(h->val),
                                                      static_cast<float *>(h->onsite), keys.as<int64_t>());
        else
            k_fill_sk_blk<double><<<g, kBlock, 0, s>>>(plan.cells.view, pos, n, slice, log2i(slice), sk->r_cut, v,
                                                       plan.perm.as<int32_t>(), plan.iperm.as<int32_t>(), h->ptr,
                                                       h->col, static_cast<double *>(h->val),
                                                       static_cast<double *>(h->onsite), keys.as<int64_t>());
    } else if (h->fmt == TBK_SELL_F32)
        k_fill_sk<float><<<g, kBlock, 0, s>>>(plan.cells.view, pos, n, slice, log2i(slice), sk->r_cut, v,
                                              plan.perm.as<int32_t>(), plan.iperm.as<int32_t>(), h->ptr, h->col,
                                              static_cast<float *>(h->val), static_cast<float *>(h->onsite),
                                              h->col16, keys.as<int64_t>());
    else
        k_fill_sk<double><<<g, kBlock, 0, s>>>(plan.cells.view, pos, n, slice, log2i(slice), sk->r_cut, v,
                                               plan.perm.as<int32_t>(), plan.iperm.as<int32_t>(), h->ptr, h->col,
                                               static_cast<double *>(h->val), static_cast<double *>(h->onsite),
                                               h->col16, keys.as<int64_t>());
    TBK_HIP(hipGetLastError());
    std::vector<int64_t> hk(2);
    TBK_HIP(hipMemcpyAsync(hk.data(), keys.as<int64_t>(), sizeof(int64_t) * 2, hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    decode_bounds(hk, 1, spec_bounds);
    if (h->fmt == TBK_CSR_F64) h->slice = 1;
    h->seg_rows = nullptr;
    return set_sk_sizes(n, plan, ly, sk, h);
}
