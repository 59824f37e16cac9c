// Multi-orbital Slater-Koster Hamiltonian (s, p or s, p, d per atom) on the GPU.
//
// The paper's models attach several orbitals to each atom and form every
// atom-pair block from two-centre integrals and the bond direction (the SK
// conversion P_lambda(r_ij) of Sec. 3).  Here the Slater-Koster table (Phys.
// Rev. 94, 1498 (1954), Table I) for s, p and d orbitals with one radial factor
// f(r) = exp(-beta (r/r0 - 1)) for every integral; c = bond direction cosines
// from i to j (minimum image); orbitals s, px, py, pz (and dxy, dyz, dzx,
// dx2-y2, d3z2-r2).
//
// The orbital Hamiltonian (row NORB r + a for atom row r, NORB = 4 or 9)
// is stored either as an ordinary SELL matrix with 4 N rows (the recurrence,
// the DOS and the VAC path run on it unchanged) or as a block SELL over atoms
// with one NORB x NORB block per bond (one column per block; the block
// recurrence kernel in kpm_block.hip).  The neighbour search, the atom row
// order and the atom degrees come from the one-orbital builder's plan.
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <vector>

#include "builder.hpp"
#include "nlist.hpp"
#include "sk_table.hpp"

namespace tbk {
namespace {

// entries[s] = C * max over the orbital rows of slice s of norb * deg(atom row).
__global__ void k_sk_width(int64_t n_orb_rows, int32_t norb, int32_t slice, int64_t n_slices,
                           const int32_t *__restrict__ deg, int64_t *__restrict__ entries) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    int32_t w = 0;
    const int64_t r1 = min((s + 1) * (int64_t)slice, n_orb_rows);
    for (int64_t R = s * (int64_t)slice; R < r1; ++R) w = max(w, norb * deg[R / norb]);
    entries[s] = (int64_t)slice * w;
}

// perm_orb[norb r + a] = norb perm[r] + a
__global__ void k_sk_perm(int64_t n, int32_t norb, const int32_t *__restrict__ perm,
                          int32_t *__restrict__ perm_orb) {
    const int64_t R = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (R >= norb * n) return;
    perm_orb[R] = norb * perm[R / norb] + (int32_t)(R % norb);
}

// bond_ptr[i] = first bond of atom i in (i, j)-sorted bonds (lower bound of i in bi), i = 0..n.
__global__ void k_bond_ptr(int64_t n, int64_t nb, const int32_t *__restrict__ bi, int64_t *__restrict__ bond_ptr) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i > n) return;
    int64_t lo = 0, hi = nb;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (bi[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    bond_ptr[i] = lo;
}

struct SkValues {
    double r0, beta, e_s, e_p, e_d;
    // at r0: ss_sigma, sp_sigma, pp_sigma, pp_pi, sd_sigma, pd_sigma, pd_pi, dd_sigma, dd_pi, dd_delta
    double v[10];
    // several species (pv != NULL): integrals pv[(s_i ns + s_j) 10 + l] of the ordered
    // species pair, onsite energies se[3 s + shell], species of the caller's atoms
    const double *pv = nullptr;
    const double *se = nullptr;
    const int32_t *species = nullptr;
    int32_t ns = 1;
    // onsite network (yon != NULL): yon[(s_i n_sh + shell) n_atoms + i] added to the onsite energy
    const float *yon = nullptr;
    int64_t n_atoms = 0;
    int32_t n_sh = 0;
};

// Per-bond scales of the two-centre integrals (learned form): bonds i < j of
// the hopping cutoff sorted by (i, j), bond_ptr[i] = first bond of atom i,
// y[l * nb + b] = output of network l for bond b; the bond's integral l is
// v[l] (1 + y).  y = NULL: the plain table.
struct BondScales {
    const int64_t *bond_ptr = nullptr;
    const int32_t *bj = nullptr;
    const float *y = nullptr;
    int64_t nb = 0;
    int32_t K = 0;
};

// The integrals of the bond i -> j (caller's atom indices): vu of the ordered
// species pair (s_i, s_j) and vl of (s_j, s_i), times the bond's learned scales.
// Both come back by value, so that no address of the parameter block is taken
// and the block stays out of per-lane memory.
__device__ __forceinline__ void bond_integrals(const BondScales &bs, const SkValues &sk, int32_t i, int32_t j,
                                               double (&vu)[10], double (&vl)[10]) {
    if (sk.pv) {
        const int32_t si = sk.species[i], sj = sk.species[j];
        const double *pu = sk.pv + 10 * ((int64_t)si * sk.ns + sj);
        const double *pl = sk.pv + 10 * ((int64_t)sj * sk.ns + si);
        for (int l = 0; l < 10; ++l) {
            vu[l] = pu[l];
            vl[l] = pl[l];
        }
    } else {
        for (int l = 0; l < 10; ++l) {
            vu[l] = sk.v[l];
            vl[l] = sk.v[l];
        }
    }
    if (!bs.y) return;
    const int32_t lo = min(i, j), hi = max(i, j);
    int64_t b = -1;
    for (int64_t q = bs.bond_ptr[lo]; q < bs.bond_ptr[lo + 1]; ++q)
        if (bs.bj[q] == hi) { b = q; break; }
    for (int l = 0; l < 10; ++l) {
        const double f = (b >= 0 && l < bs.K) ? 1.0 + (double)bs.y[(int64_t)l * bs.nb + b] : 1.0;
        vu[l] *= f;
        vl[l] *= f;
    }
}

// The NORB x NORB block of a bond of length r and vector (dx, dy, dz) from the
// row atom, integrals vu, vl (sk_table) at r0.
template <int NORB>
__device__ __forceinline__ void sk_block(const double *vu, const double *vl, const SkValues &sk, double r, double dx,
                                         double dy, double dz, double (&B)[NORB][NORB]) {
    sk_table<double, NORB>(vu, vl, dx / r, dy / r, dz / r, B);
    const double f = exp(-sk.beta * (r / sk.r0 - 1.0));
    for (int a = 0; a < NORB; ++a)
        for (int b = 0; b < NORB; ++b) B[a][b] *= f;
}

// Onsite energy of orbital a on atom i (caller's index).
__device__ __forceinline__ double sk_onsite(const SkValues &sk, int32_t i, int a) {
    const int sh = a == 0 ? 0 : (a < 4 ? 1 : 2);
    const double e = sk.pv ? sk.se[3 * sk.species[i] + sh] : (sh == 0 ? sk.e_s : (sh == 1 ? sk.e_p : sk.e_d));
    if (!sk.yon) return e;
    return e + (double)sk.yon[((int64_t)sk.species[i] * sk.n_sh + sh) * sk.n_atoms + i];
}

// One atom row r per thread: its NORB orbital rows, entry NORB q + b for the
// q-th neighbour (cell-list order) and its orbital b; padding (own row, value
// 0) up to the slice width; onsite; row Gershgorin bounds; 16-bit offsets.
template <class V, int NORB>
__global__ __launch_bounds__(kBlock) void k_fill_sk(CellList cl, const double *__restrict__ pos, int64_t n, int32_t slice,
                          int32_t log2_slice, double r_cut, SkValues sk, const int32_t *__restrict__ perm,
                          const int32_t *__restrict__ iperm, const int64_t *__restrict__ ptr,
                          int32_t *__restrict__ col, V *__restrict__ val, V *__restrict__ onsite,
                          int16_t *__restrict__ col16, int64_t *__restrict__ bound_keys, BondScales bs) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (r < n) {
        int64_t base[NORB];
        int32_t w[NORB];
        for (int a = 0; a < NORB; ++a) {
            const int64_t R = NORB * r + a;
            const int64_t sl = R >> log2_slice;
            base[a] = ptr[sl] + (R & (slice - 1));
            w[a] = (int32_t)((ptr[sl + 1] - ptr[sl]) >> log2_slice);
        }
        const int32_t i = perm[r];
        double asum[NORB];
        for (int a = 0; a < NORB; ++a) asum[a] = 0.0;
        int32_t q = 0;
        for_each_neighbor(cl, pos, i, r_cut, [&](int32_t j, double rij, double dx, double dy, double dz) {
            double B[NORB][NORB], vu[10], vl[10];
            bond_integrals(bs, sk, i, j, vu, vl);
            sk_block<NORB>(vu, vl, sk, rij, dx, dy, dz, B);
            const int32_t cj = NORB * iperm[j];
            for (int a = 0; a < NORB; ++a)
                for (int b = 0; b < NORB; ++b) {
                    const int32_t k = NORB * q + b;
                    if (k < w[a]) {
                        col[base[a] + (int64_t)k * slice] = cj + b;
                        val[base[a] + (int64_t)k * slice] = (V)B[a][b];
                    }
                    asum[a] += fabs(B[a][b]);
                }
            ++q;
        });
        for (int a = 0; a < NORB; ++a) {
            const int64_t R = NORB * r + a;
            for (int32_t k = NORB * q; k < w[a]; ++k) {
                col[base[a] + (int64_t)k * slice] = (int32_t)R;
                val[base[a] + (int64_t)k * slice] = (V)0;
            }
            if (col16)
                for (int32_t k = 0; k < w[a]; ++k) {
                    const int64_t d = (int64_t)col[base[a] + (int64_t)k * slice] - R;
                    col16[base[a] + (int64_t)k * slice] =
                        (d >= -32767 && d <= 32767) ? (int16_t)d : (int16_t)-32768;
                }
            const double e = sk_onsite(sk, i, a);
            onsite[R] = (V)e;
            lo = fmin(lo, e - asum[a]);
            hi = fmax(hi, e + asum[a]);
        }
    }
    block_segment_bounds(lo, hi, r < n ? 0 : -1, bound_keys);
}

// Block form: one atom row r per thread; block q (q-th neighbour, cell-list
// order) at slot base + q C of the atom slice, its NORB^2 values row-major at
// NORB^2 (base + q C); padding blocks (own row, zero) up to the slice width.
template <class V, int NORB>
__global__ __launch_bounds__(kBlock) void k_fill_sk_blk(CellList cl, const double *__restrict__ pos, int64_t n, int32_t slice,
                              int32_t log2_slice, double r_cut, SkValues sk, const int32_t *__restrict__ perm,
                              const int32_t *__restrict__ iperm, const int64_t *__restrict__ ptr,
                              int32_t *__restrict__ bcol, V *__restrict__ bval, V *__restrict__ onsite,
                              int64_t *__restrict__ bound_keys, BondScales bs, bool geom) {
    constexpr int NB = NORB * NORB;
    constexpr int GE = sizeof(V) == 4 ? 4 : 3;     // values per displacement slot
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (r < n) {
        const int64_t sl = r >> log2_slice;
        const int64_t base = ptr[sl] + (r & (slice - 1));
        const int32_t w = (int32_t)((ptr[sl + 1] - ptr[sl]) >> log2_slice);
        const int32_t i = perm[r];
        double asum[NORB];
        for (int a = 0; a < NORB; ++a) asum[a] = 0.0;
        int32_t q = 0;
        for_each_neighbor(cl, pos, i, r_cut, [&](int32_t j, double rij, double dx, double dy, double dz) {
            double B[NORB][NORB], vu[10], vl[10];
            bond_integrals(bs, sk, i, j, vu, vl);
            sk_block<NORB>(vu, vl, sk, rij, dx, dy, dz, B);
            if (q < w) {
                const int64_t slot = base + (int64_t)q * slice;
                bcol[slot] = iperm[j];
                if (geom) {              // the bond's displacement instead of its block
                    bval[GE * slot] = (V)dx;
                    bval[GE * slot + 1] = (V)dy;
                    bval[GE * slot + 2] = (V)dz;
                    if constexpr (GE == 4) bval[GE * slot + 3] = __int_as_float(iperm[j]);
                } else {
                    for (int a = 0; a < NORB; ++a)
                        for (int b = 0; b < NORB; ++b) bval[NB * slot + NORB * a + b] = (V)B[a][b];
                }
            }
            for (int a = 0; a < NORB; ++a)
                for (int b = 0; b < NORB; ++b) asum[a] += fabs(B[a][b]);
            ++q;
        });
        for (int32_t k = q; k < w; ++k) {
            const int64_t slot = base + (int64_t)k * slice;
            bcol[slot] = (int32_t)r;
            const int ne = geom ? 3 : NB;
            const int64_t e0 = (geom ? GE : NB) * slot;
            for (int e = 0; e < ne; ++e) bval[e0 + e] = (V)0;
            if constexpr (GE == 4)
                if (geom) bval[e0 + 3] = __int_as_float((int32_t)r);
        }
        for (int a = 0; a < NORB; ++a) {
            const double e = sk_onsite(sk, i, a);
            onsite[NORB * r + a] = (V)e;
            lo = fmin(lo, e - asum[a]);
            hi = fmax(hi, e + asum[a]);
        }
    }
    block_segment_bounds(lo, hi, r < n ? 0 : -1, bound_keys);
}

bool is_geom(int32_t fmt) { return fmt == TBK_BGEOM_F64 || fmt == TBK_BGEOM_F32; }
bool is_block(int32_t fmt) { return fmt == TBK_BSELL4_F64 || fmt == TBK_BSELL4_F32 || is_geom(fmt); }

tbk_status check_sk(const tbk_sk_params *sk) {
    TBK_CHECK(sk != nullptr, TBK_ERR_INVALID_ARG, "sk params are NULL");
    TBK_CHECK(sk->orbitals == 4 || sk->orbitals == 9, TBK_ERR_INVALID_ARG,
              "orbitals = %d (4 = s, p; 9 = s, p, d)", sk->orbitals);
    const double x[16] = {sk->r_cut, sk->r0, sk->beta, sk->e_s, sk->e_p, sk->e_d,
                          sk->v_ss_sigma, sk->v_sp_sigma, sk->v_pp_sigma, sk->v_pp_pi, sk->v_sd_sigma,
                          sk->v_pd_sigma, sk->v_pd_pi, sk->v_dd_sigma, sk->v_dd_pi, sk->v_dd_delta};
    for (double v : x) TBK_CHECK(std::isfinite(v), TBK_ERR_NOT_FINITE, "an SK parameter is not finite");
    if (!sk->pair_v) return TBK_OK;
    const int32_t ns = sk->n_species;
    TBK_CHECK(ns >= 1 && ns <= 16, TBK_ERR_INVALID_ARG, "n_species = %d outside [1, 16]", ns);
    TBK_CHECK(sk->species_e != nullptr, TBK_ERR_INVALID_ARG, "species_e is NULL");
    for (int64_t k = 0; k < (int64_t)ns * ns * 10; ++k)
        TBK_CHECK(std::isfinite(sk->pair_v[k]), TBK_ERR_NOT_FINITE, "pair_v[%lld] is not finite", (long long)k);
    for (int64_t k = 0; k < 3 * (int64_t)ns; ++k)
        TBK_CHECK(std::isfinite(sk->species_e[k]), TBK_ERR_NOT_FINITE, "species_e[%lld] is not finite",
                  (long long)k);
    // equal-l integrals (ss, pp, dd) do not depend on the order of the pair
    static const int same_l[6] = {0, 2, 3, 7, 8, 9};
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b)
            for (int l : same_l)
                TBK_CHECK(sk->pair_v[10 * (a * ns + b) + l] == sk->pair_v[10 * (b * ns + a) + l], TBK_ERR_INVALID_ARG,
                          "pair_v[%d][%d][%d] differs from pair_v[%d][%d][%d] (an equal-l integral)", a, b, l, b, a,
                          l);
    return TBK_OK;
}

int32_t species_count(const tbk_sk_params *sk) { return sk->pair_v ? sk->n_species : 1; }

// One-orbital plan of the atoms (cell list, row order, atom degrees) for the SK builder.
tbk_status atom_plan(const double *pos, const int32_t *species, int64_t n, const double box[3],
                     const int32_t periodic[3], const tbk_sk_params *sk, int32_t atom_slice, HamPlan &plan,
                     hipStream_t s) {
    tbk_status st = check_sk(sk);
    if (st != TBK_OK) return st;
    TBK_CHECK(box != nullptr, TBK_ERR_INVALID_ARG, "box is NULL");
    TBK_CHECK(n >= 1 && sk->orbitals * n < (int64_t)INT32_MAX, TBK_ERR_INVALID_ARG,
              "%lld orbital rows out of range", (long long)(sk->orbitals * n));
    // the one-orbital plan validates the species indices against n_species
    const int32_t ns = species_count(sk);
    std::vector<double> onsite0(ns, 0.0), t0((size_t)ns * ns, 1.0);
    tbk_tb_params p{};
    p.r_cut = sk->r_cut;
    p.r0 = sk->r0;
    p.beta = sk->beta;
    p.n_species = ns;
    p.reorder = sk->reorder;
    p.onsite = onsite0.data();
    p.t_pair = t0.data();
    const int64_t seg[2] = {0, n};
    return plan.run(pos, species, n, 1, seg, box, periodic, &p, TBK_SELL_F64, atom_slice, s);
}

struct SkLayout {
    int64_t n_slices = 0, n_entries = 0;
    int32_t max_w = 0;
    DevBuf ptr;
};

tbk_status sk_layout(const HamPlan &plan, int64_t n, int32_t norb, int32_t slice, SkLayout &ly, hipStream_t s) {
    const int64_t nr = norb * n;
    ly.n_slices = ceil_div(nr, slice);
    DevBuf entries;
    TBK_HIP(entries.alloc(sizeof(int64_t) * (ly.n_slices + 1), s));
    TBK_HIP(ly.ptr.alloc(sizeof(int64_t) * (ly.n_slices + 1), s));
    TBK_HIP(hipMemsetAsync(entries.as<int64_t>() + ly.n_slices, 0, sizeof(int64_t), s));
    k_sk_width<<<(unsigned)ceil_div(ly.n_slices, kBlock), kBlock, 0, s>>>(nr, norb, slice, ly.n_slices,
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
    ly.max_w = norb * plan.max_degree;
    return TBK_OK;
}

int32_t log2i(int32_t v) {
    int32_t l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

tbk_status set_sk_sizes(int64_t n, const HamPlan &plan, const SkLayout &ly, const tbk_sk_params *sk, tbk_ham *h,
                        bool learned_onsite = false) {
    const int32_t norb = sk->orbitals;
    h->n_rows = norb * n;
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
    h->has_onsite = (sk->e_s != 0.0 || sk->e_p != 0.0 || (norb == 9 && sk->e_d != 0.0)) ? 1 : 0;
    if (sk->pair_v) {
        h->has_onsite = 0;
        for (int64_t k = 0; k < 3 * (int64_t)sk->n_species; ++k)
            if ((k % 3 < 2 || norb == 9) && sk->species_e[k] != 0.0) h->has_onsite = 1;
    }
    if (learned_onsite) h->has_onsite = 1;
    h->n_seg = 1;
    h->n_orb = norb;
    h->uniform_hop = 0;
    h->hop_value = 0.0;
    return TBK_OK;
}

template <class V, int NORB>
void launch_fill(const HamPlan &plan, const double *pos, int64_t n, int32_t slice, double r_cut, const SkValues &v,
                 tbk_ham *h, int64_t *keys, const BondScales &bs, hipStream_t s) {
    const unsigned g = (unsigned)ceil_div(n, kBlock);
    if (is_block(h->fmt))
        k_fill_sk_blk<V, NORB><<<g, kBlock, 0, s>>>(plan.cells.view, pos, n, slice, log2i(slice), r_cut, v,
                                                    plan.perm.as<int32_t>(), plan.iperm.as<int32_t>(), h->ptr,
                                                    h->col, static_cast<V *>(h->val), static_cast<V *>(h->onsite),
                                                    keys, bs, is_geom(h->fmt));
    else
        k_fill_sk<V, NORB><<<g, kBlock, 0, s>>>(plan.cells.view, pos, n, slice, log2i(slice), r_cut, v,
                                                plan.perm.as<int32_t>(), plan.iperm.as<int32_t>(), h->ptr, h->col,
                                                static_cast<V *>(h->val), static_cast<V *>(h->onsite), h->col16,
                                                keys, bs);
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
        st = sk_layout(plan, n, sk->orbitals, slice, ly, s);
        if (st != TBK_OK) return st;
    }
    if (h->fmt == TBK_CSR_F64) h->slice = 1;
    return set_sk_sizes(n, plan, ly, sk, h);
}

namespace tbk {
namespace {

// Builds h; with a model, each bond's integrals are scaled by the outputs of
// one network per integral (bond features of the descriptor model, MLP
// forward of the learned-hopping path).
tbk_status build_sk(const double *pos, const int32_t *species, int64_t n, const double box[3],
                    const int32_t periodic[3], const tbk_sk_params *sk, const tbk_mlp_model *model,
                    const tbk_onsite_model *onsite, tbk_ham *h, double spec_bounds[2], float *bond_y,
                    int64_t bond_cap, int64_t *n_bonds, hipStream_t s) {
    TBK_CHECK(h != nullptr && spec_bounds != nullptr, TBK_ERR_INVALID_ARG, "h or bounds is NULL");
    TBK_CHECK(h->fmt == TBK_SELL_F32 || h->fmt == TBK_SELL_F64 || h->fmt == TBK_CSR_F64 || is_block(h->fmt),
              TBK_ERR_INVALID_ARG, "unknown format %d", h->fmt);
    const int32_t slice = h->fmt == TBK_CSR_F64 ? 1 : h->slice;
    TBK_CHECK(slice >= 1 && slice <= 1024 && (slice & (slice - 1)) == 0, TBK_ERR_INVALID_ARG,
              "slice = %d is not a power of two in [1, 1024]", slice);
    HamPlan plan;
    const bool blk = is_block(h->fmt);
    tbk_status st = atom_plan(pos, species, n, box, periodic, sk, blk ? slice : 1, plan, s);
    if (st != TBK_OK) return st;
    const int32_t norb = sk->orbitals;
    SkLayout ly;
    if (blk) {
        ly.n_slices = plan.n_slices;
        ly.n_entries = plan.n_entries;
    } else {
        st = sk_layout(plan, n, norb, slice, ly, s);
        if (st != TBK_OK) return st;
    }
    TBK_CHECK(h->n_rows >= norb * n && h->n_ptr >= ly.n_slices + 1 && h->n_entries >= ly.n_entries,
              TBK_ERR_BUFFER_TOO_SMALL, "buffers sized for n_rows=%lld n_ptr=%lld n_entries=%lld; need %lld, %lld, %lld",
              (long long)h->n_rows, (long long)h->n_ptr, (long long)h->n_entries, (long long)(norb * n),
              (long long)(ly.n_slices + 1), (long long)ly.n_entries);
    TBK_CHECK(h->ptr && h->col && h->val && h->onsite && h->perm, TBK_ERR_INVALID_ARG,
              "a Hamiltonian array pointer is NULL");
    TBK_HIP(hipMemcpyAsync(h->ptr, blk ? plan.ptr.as<int64_t>() : ly.ptr.as<int64_t>(),
                           sizeof(int64_t) * (ly.n_slices + 1), hipMemcpyDeviceToDevice, s));
    k_sk_perm<<<(unsigned)ceil_div(norb * n, kBlock), kBlock, 0, s>>>(n, norb, plan.perm.as<int32_t>(), h->perm);
    TBK_HIP(hipGetLastError());
    DevBuf keys;
    st = init_bound_keys(keys, 1, s);
    if (st != TBK_OK) return st;
    SkValues v{sk->r0, sk->beta, sk->e_s, sk->e_p, sk->e_d,
               {sk->v_ss_sigma, sk->v_sp_sigma, sk->v_pp_sigma, sk->v_pp_pi, sk->v_sd_sigma, sk->v_pd_sigma,
                sk->v_pd_pi, sk->v_dd_sigma, sk->v_dd_pi, sk->v_dd_delta}};
    DevBuf dpv, dse;
    if (sk->pair_v) {
        const int32_t ns = sk->n_species;
        TBK_HIP(dpv.alloc(sizeof(double) * 10 * ns * ns, s));
        TBK_HIP(dse.alloc(sizeof(double) * 3 * ns, s));
        TBK_HIP(hipMemcpyAsync(dpv.as<double>(), sk->pair_v, sizeof(double) * 10 * ns * ns, hipMemcpyHostToDevice, s));
        TBK_HIP(hipMemcpyAsync(dse.as<double>(), sk->species_e, sizeof(double) * 3 * ns, hipMemcpyHostToDevice, s));
        v.pv = dpv.as<double>();
        v.se = dse.as<double>();
        v.species = species;
        v.ns = ns;
    }
    DevBuf von, Xn, yon;
    if (onsite) {
        // node features -> one network per (species, shell)
        const int32_t ns = species_count(sk), nsh = norb == 4 ? 2 : 3;
        const int64_t seg[2] = {0, n};
        TBK_HIP(von.alloc(sizeof(double) * n * 8, s));
        TBK_HIP(Xn.alloc(sizeof(uint16_t) * 16 * n, s));
        TBK_HIP(yon.alloc(sizeof(float) * ns * nsh * n, s));
        st = onsite->c_nk ? tbk_descriptor_species(pos, species, 1, seg, box, periodic, onsite->r_cut, 8,
                                                   onsite->n_species, onsite->c_nk, von.as<double>(), s)
                          : tbk_descriptor(pos, 1, seg, box, periodic, onsite->r_cut, 8, von.as<double>(), s);
        if (st != TBK_OK) return st;
        st = tbk_node_features(n, von.as<double>(), 8, onsite->shift, onsite->scale, Xn.as<uint16_t>(), s);
        if (st != TBK_OK) return st;
        for (int32_t q = 0; q < ns * nsh; ++q) {
            st = tbk_mlp_forward(n, Xn.as<uint16_t>(), onsite->params + (int64_t)q * TBK_MLP_PARAMS,
                                 yon.as<float>() + (int64_t)q * n, s);
            if (st != TBK_OK) return st;
        }
        v.yon = yon.as<float>();
        v.n_atoms = n;
        v.n_sh = nsh;
        v.species = species;
    }
    BondScales bs;
    DevBuf vdesc, bi, bj, br, X, y, bptr;
    if (model) {
        // descriptor -> bonds of the hopping cutoff -> features -> one network per integral
        const int32_t K = norb == 4 ? 4 : 10;
        const int64_t nb = plan.n_bonds;
        const int64_t seg[2] = {0, n};
        if (n_bonds) *n_bonds = nb;
        TBK_CHECK(bond_y == nullptr || bond_cap >= K * nb, TBK_ERR_BUFFER_TOO_SMALL,
                  "bond_y holds %lld, needs %lld", (long long)bond_cap, (long long)(K * nb));
        TBK_HIP(vdesc.alloc(sizeof(double) * n * model->n_radial, s));
        st = model->c_nk ? tbk_descriptor_species(pos, species, 1, seg, box, periodic, model->r_cut, model->n_radial,
                                                  model->n_species, model->c_nk, vdesc.as<double>(), s)
                         : tbk_descriptor(pos, 1, seg, box, periodic, model->r_cut, model->n_radial,
                                          vdesc.as<double>(), s);
        if (st != TBK_OK) return st;
        const int64_t cap = std::max<int64_t>(nb, 1);
        TBK_HIP(bi.alloc(sizeof(int32_t) * cap, s));
        TBK_HIP(bj.alloc(sizeof(int32_t) * cap, s));
        TBK_HIP(br.alloc(sizeof(double) * cap, s));
        TBK_HIP(X.alloc(sizeof(uint16_t) * 16 * cap, s));
        TBK_HIP(y.alloc(sizeof(float) * K * cap, s));
        TBK_HIP(bptr.alloc(sizeof(int64_t) * (n + 1), s));
        int64_t nb2 = 0;
        st = tbk_bonds(pos, 1, seg, box, periodic, sk->r_cut, cap, bi.as<int32_t>(), bj.as<int32_t>(),
                       br.as<double>(), &nb2, s);
        if (st != TBK_OK) return st;
        TBK_CHECK(nb2 == nb, TBK_ERR_DEVICE, "bond count mismatch (%lld vs %lld)", (long long)nb2, (long long)nb);
        if (nb > 0) {
            st = model->c_nk
                     ? tbk_bond_features_species(nb, bi.as<int32_t>(), bj.as<int32_t>(), br.as<double>(), species,
                                                 vdesc.as<double>(), model->n_radial, model->r_cut, model->n_species,
                                                 model->c_nk, model->shift, model->scale, X.as<uint16_t>(), s)
                     : tbk_bond_features(nb, bi.as<int32_t>(), bj.as<int32_t>(), br.as<double>(), vdesc.as<double>(),
                                         model->n_radial, model->r_cut, model->shift, model->scale,
                                         X.as<uint16_t>(), s);
            if (st != TBK_OK) return st;
            for (int32_t l = 0; l < K; ++l) {
                st = tbk_mlp_forward(nb, X.as<uint16_t>(), model->params + (int64_t)l * TBK_MLP_PARAMS,
                                     y.as<float>() + (int64_t)l * nb, s);
                if (st != TBK_OK) return st;
            }
            if (bond_y)
                TBK_HIP(hipMemcpyAsync(bond_y, y.as<float>(), sizeof(float) * K * nb, hipMemcpyDeviceToDevice, s));
        }
        k_bond_ptr<<<(unsigned)ceil_div(n + 1, kBlock), kBlock, 0, s>>>(n, nb, bi.as<int32_t>(), bptr.as<int64_t>());
        TBK_HIP(hipGetLastError());
        bs.bond_ptr = bptr.as<int64_t>();
        bs.bj = bj.as<int32_t>();
        bs.y = y.as<float>();
        bs.nb = nb;
        bs.K = K;
    }
    const bool f32 = h->fmt == TBK_SELL_F32 || h->fmt == TBK_BSELL4_F32 || h->fmt == TBK_BGEOM_F32;
    if (is_geom(h->fmt)) {
        TBK_CHECK(!sk->pair_v && !model && !onsite, TBK_ERR_INVALID_ARG,
                  "the displacement format takes one species and fixed integrals");
        for (int l = 0; l < 10; ++l) h->sk_geom[l] = v.v[l];
        h->sk_geom[10] = sk->r0;
        h->sk_geom[11] = sk->beta;
    }
    if (norb == 4) {
        if (f32) launch_fill<float, 4>(plan, pos, n, slice, sk->r_cut, v, h, keys.as<int64_t>(), bs, s);
        else launch_fill<double, 4>(plan, pos, n, slice, sk->r_cut, v, h, keys.as<int64_t>(), bs, s);
    } else {
        if (f32) launch_fill<float, 9>(plan, pos, n, slice, sk->r_cut, v, h, keys.as<int64_t>(), bs, s);
        else launch_fill<double, 9>(plan, pos, n, slice, sk->r_cut, v, h, keys.as<int64_t>(), bs, s);
    }
    TBK_HIP(hipGetLastError());
    std::vector<int64_t> hk(2);
    TBK_HIP(hipMemcpyAsync(hk.data(), keys.as<int64_t>(), sizeof(int64_t) * 2, hipMemcpyDeviceToHost, s));
    TBK_HIP(hipStreamSynchronize(s));
    decode_bounds(hk, 1, spec_bounds);
    if (h->fmt == TBK_CSR_F64) h->slice = 1;
    h->seg_rows = nullptr;
    return set_sk_sizes(n, plan, ly, sk, h, onsite != nullptr);
}

}  // namespace
}  // namespace tbk

extern "C" tbk_status tb_build_hamiltonian_sk(const double *pos, const int32_t *species, int64_t n,
                                              const double box[3], const int32_t periodic[3],
                                              const tbk_sk_params *sk, tbk_ham *h, double spec_bounds[2],
                                              void *stream) {
    clear_error();
    return build_sk(pos, species, n, box, periodic, sk, nullptr, nullptr, h, spec_bounds, nullptr, 0, nullptr,
                    as_stream(stream));
}

extern "C" tbk_status tb_build_hamiltonian_sk_learned(const double *pos, const int32_t *species, int64_t n,
                                                      const double box[3], const int32_t periodic[3],
                                                      const tbk_sk_params *sk, const tbk_mlp_model *model,
                                                      const tbk_onsite_model *onsite, tbk_ham *h,
                                                      double spec_bounds[2], float *bond_y, int64_t bond_cap,
                                                      int64_t *n_bonds, void *stream) {
    clear_error();
    TBK_CHECK(model || onsite, TBK_ERR_INVALID_ARG, "neither a bond model nor an onsite model");
    if (model) {
        TBK_CHECK(model->params && model->shift && model->scale, TBK_ERR_INVALID_ARG, "model is incomplete");
        TBK_CHECK(model->n_radial == 8, TBK_ERR_INVALID_ARG, "n_radial = %d (must be 8)", model->n_radial);
        TBK_CHECK(std::isfinite(model->r_cut) && model->r_cut > 0, TBK_ERR_INVALID_ARG, "descriptor cutoff %g",
                  model->r_cut);
    }
    if (onsite) {
        TBK_CHECK(onsite->params && onsite->shift && onsite->scale, TBK_ERR_INVALID_ARG,
                  "onsite model is incomplete");
        TBK_CHECK(std::isfinite(onsite->r_cut) && onsite->r_cut > 0, TBK_ERR_INVALID_ARG,
                  "onsite descriptor cutoff %g", onsite->r_cut);
    }
    return build_sk(pos, species, n, box, periodic, sk, model, onsite, h, spec_bounds, bond_y, bond_cap, n_bonds,
                    as_stream(stream));
}
