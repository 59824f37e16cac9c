// Chebyshev recurrence with fused moment accumulation (KPM, Sec. 2.4): the
// run plan (workspace layout, launch shape), the dispatch to the kernel
// instances of kpm_run.hpp, checkpoint/resume of a run, and the C entry points.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "kpm.hpp"
#include "kpm_dev.hpp"

namespace tbk {

namespace {

int log2_exact(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return (1 << l) == x ? l : -1;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of kpm_moments_noalloc: one array per GPU, part of the loaded code
// object (no allocation call), shared by every call on that GPU.  Host code
// uses the device address hipGetSymbolAddress returns for the current device,
// never the array's name (a host-side stand-in).
constexpr size_t kScratchBytes = 64ull << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};

tbk_status scratch_address(void **out) {
    int dev = -1;
    TBK_HIP(hipGetDevice(&dev));
    TBK_CHECK(dev >= 0 && dev < kScratchDevices, TBK_ERR_UNSUPPORTED, "device %d: no workspace slot", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        TBK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        TBK_CHECK(p != nullptr, TBK_ERR_DEVICE, "no device address for the static workspace");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TBK_OK;
}

}  // namespace

StepTimer &step_timer() {
    static thread_local StepTimer t;
    return t;
}

hipError_t StepTimer::mark(hipStream_t s) {
    if (used == ev.size()) {
        hipEvent_t e;
        const hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        ev.push_back(e);
    }
    return hipEventRecord(ev[used++], s);
}

hipError_t StepTimer::collect() {
    for (size_t k = 0; k + 1 < used; k += 2) {
        float t = 0.f;
        const hipError_t err = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
        if (err != hipSuccess) return err;
        ms += t;
    }
    used = 0;
    return hipSuccess;
}

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
    c.xcd_remap = 2;            // runs of 16 blocks per XCD: never slower than dispatch order on MI355X
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
    TBK_CHECK(pl.cfg.xcd_remap >= 0 && pl.cfg.xcd_remap <= 3, TBK_ERR_INVALID_ARG, "xcd_remap must be 0..3");
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
    pl.G_real = G;
    {
        // round up to the block order's multiple; the extra blocks own no tile
        const int64_t mult = xcd_grid_multiple(pl.cfg.xcd_remap);
        G = ((G + mult - 1) / mult) * mult;
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
    // the state record and the vectors come first, at offsets that do not depend on M
    pl.off_state = 0;
    pl.off_r = kStateBytes;
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
        case 1: return run_moments_inst<double, 1, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 2: return run_moments_inst<double, 2, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 4: return run_moments_inst<double, 4, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 8: return run_moments_inst<double, 8, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 16: return run_moments_inst<double, 16, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 32: return run_moments_inst<double, 32, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        case 64: return run_moments_inst<double, 64, 1>(h, pl, a, b, rr, R, M, w, mu, s, sd, ld_);
        }
    } else {
        const float *rr = static_cast<const float *>(r);
        if (pl.VPT == 1) {
            switch (pl.L) {
            case 1: return run_moments_inst<float, 1, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 2: return run_moments_inst<float, 2, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 4: return run_moments_inst<float, 4, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 8: return run_moments_inst<float, 8, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 16: return run_moments_inst<float, 16, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 32: return run_moments_inst<float, 32, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 64: return run_moments_inst<float, 64, 1>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            }
        } else {
            switch (pl.L) {
            case 1: return run_moments_inst<float, 1, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 2: return run_moments_inst<float, 2, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 4: return run_moments_inst<float, 4, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 8: return run_moments_inst<float, 8, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 16: return run_moments_inst<float, 16, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
            case 32: return run_moments_inst<float, 32, 2>(h, pl, a, b, rr, R, M, w, mu, s, sf, lf);
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
    TBK_CHECK(a && b && (r || pl.seeded || pl.n_start > 0) && work && mu, TBK_ERR_INVALID_ARG, "NULL argument");
    TBK_CHECK(h->n_seg == 1, TBK_ERR_UNSUPPORTED, "stacked systems go through kpm_moments_batched");
    TBK_CHECK(std::isfinite(a[0]) && std::isfinite(b[0]), TBK_ERR_NOT_FINITE, "a or b is not finite");
    TBK_CHECK(a[0] > 0, TBK_ERR_INVALID_ARG, "a = %g must be positive", a[0]);
    TBK_CHECK(work_bytes >= (int64_t)pl.total, TBK_ERR_BUFFER_TOO_SMALL,
              "work has %lld bytes, needs %lld", (long long)work_bytes, (long long)pl.total);
    TBK_CHECK(((uintptr_t)work & 255) == 0, TBK_ERR_INVALID_ARG, "work is not 256-byte aligned");
    TBK_CHECK(h->ptr && h->col && h->val && h->onsite, TBK_ERR_INVALID_ARG, "Hamiltonian array is NULL");
    return TBK_OK;
}

// n_start is 0 or in [2, M), and only the direct form continues a run.
// A continued run (n_start > 0) needs the record a completed run of the same
// Hamiltonian, R, precision and (a, b) left at the head of `work`, ending at
// moment n_start - 1.  Reads it back (synchronises the stream).
tbk_status check_start(const KpmPlan &pl, int32_t M) {
    const int32_t n0 = pl.n_start;
    if (n0 == 0) return TBK_OK;
    TBK_CHECK(n0 >= 2 && n0 < M, TBK_ERR_INVALID_ARG, "n_start = %d: must be 0, or in [2, M) with M = %d", n0, M);
    TBK_CHECK(pl.cfg.doubling == 0, TBK_ERR_INVALID_ARG, "the doubling form cannot continue a run (n_start > 0)");
    return TBK_OK;
}

tbk_status check_resume(const tbk_ham *h, const KpmPlan &pl, double a, double b, int32_t R, int32_t M,
                        int32_t precision, const void *work, hipStream_t s) {
    const int32_t n0 = pl.n_start;
    if (n0 == 0) return TBK_OK;
    (void)M;
    KpmState st{};
    TBK_HIP(hipMemcpyAsync(&st, static_cast<const char *>(work) + pl.off_state, sizeof(st), hipMemcpyDeviceToHost,
                           s));
    TBK_HIP(hipStreamSynchronize(s));
    TBK_CHECK(st.magic == kStateMagic, TBK_ERR_INVALID_ARG,
              "n_start = %d: work holds no completed run of the direct recurrence to continue", n0);
    TBK_CHECK(st.n_rows == h->n_rows && st.n_entries == h->n_entries && st.fmt == h->fmt && st.R == R &&
                  st.precision == precision,
              TBK_ERR_INVALID_ARG, "n_start = %d: work holds a run of another Hamiltonian, R or precision", n0);
    TBK_CHECK(st.a == a && st.b == b, TBK_ERR_INVALID_ARG,
              "n_start = %d: work holds a run with another scale (a = %g, b = %g)", n0, st.a, st.b);
    TBK_CHECK(st.next_n == n0, TBK_ERR_INVALID_ARG,
              "n_start = %d: work holds the moments up to %d, so the run continues at n_start = %d", n0,
              st.next_n - 1, st.next_n);
    return TBK_OK;
}

}  // namespace tbk

using namespace tbk;

extern "C" tbk_status kpm_scale(int32_t n, const double *spec_bounds, double margin, double *a, double *b) {
    clear_error();
    TBK_CHECK(n >= 1 && spec_bounds && a && b, TBK_ERR_INVALID_ARG, "n = %d or a NULL argument", n);
    TBK_CHECK(std::isfinite(margin) && margin >= 1.0, TBK_ERR_INVALID_ARG, "margin = %g must be >= 1", margin);
    for (int32_t s = 0; s < n; ++s) {
        const double lo = spec_bounds[2 * s], hi = spec_bounds[2 * s + 1];
        TBK_CHECK(std::isfinite(lo) && std::isfinite(hi), TBK_ERR_NOT_FINITE, "bounds of system %d are not finite",
                  s);
        TBK_CHECK(hi > lo, TBK_ERR_INVALID_ARG,
                  "bounds of system %d: E_hi = %g <= E_lo = %g (a single-point spectrum has no Chebyshev scale)", s,
                  hi, lo);
    }
    for (int32_t s = 0; s < n; ++s) {
        const double lo = spec_bounds[2 * s], hi = spec_bounds[2 * s + 1];
        a[s] = margin * (hi - lo) / 2.0;
        b[s] = (hi + lo) / 2.0;
    }
    return TBK_OK;
}

extern "C" tbk_status kpm_step_timer(int32_t enable) {
    clear_error();
    TBK_CHECK(enable == 0 || enable == 1, TBK_ERR_INVALID_ARG, "enable must be 0 or 1");
    StepTimer &t = step_timer();
    t.on = enable == 1;
    t.ms = 0.0;
    t.launches = 0;
    t.used = 0;
    return TBK_OK;
}

extern "C" tbk_status kpm_step_timer_read(double *ms, int64_t *launches) {
    clear_error();
    TBK_CHECK(ms && launches, TBK_ERR_INVALID_ARG, "NULL argument");
    StepTimer &t = step_timer();
    *ms = t.ms;
    *launches = t.launches;
    t.ms = 0.0;
    t.launches = 0;
    return TBK_OK;
}

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
                                  int32_t R, int32_t M, int32_t precision, int32_t n_start, void *work,
                                  int64_t work_bytes, double *mu, void *stream) {
    return kpm_moments_config(h, a, b, r, R, M, precision, nullptr, n_start, work, work_bytes, mu, stream);
}

extern "C" tbk_status kpm_moments_config(const tbk_ham *h, const double *a, const double *b, const void *r,
                                         int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                                         int32_t n_start, void *work, int64_t work_bytes, double *mu,
                                         void *stream) {
    clear_error();
    KpmPlan pl;
    tbk_status st = make_plan(h, R, M, precision, cfg, pl);
    if (st != TBK_OK) return st;
    pl.n_start = n_start;
    st = check_start(pl, M);
    if (st != TBK_OK) return st;
    st = check_moment_args(h, pl, a, b, r, work, work_bytes, mu);
    if (st != TBK_OK) return st;
    TBK_CHECK(pl.cfg.persistent == 0, TBK_ERR_INVALID_ARG, "the persistent launch is for kpm_moments_batched");
    st = check_resume(h, pl, a[0], b[0], R, M, precision, work, as_stream(stream));
    if (st != TBK_OK) return st;
    return run_plan(h, pl, a[0], b[0], r, R, M, precision, static_cast<char *>(work), mu, as_stream(stream),
                    nullptr, nullptr);
}

extern "C" tbk_status kpm_moments_noalloc(const tbk_ham *h, const double *a, const double *b, const void *r,
                                          int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                                          int32_t n_start, double *mu, void *stream) {
    clear_error();
    KpmPlan pl;
    tbk_status st = make_plan(h, R, M, precision, cfg, pl);
    if (st != TBK_OK) return st;
    pl.n_start = n_start;
    st = check_start(pl, M);
    if (st != TBK_OK) return st;
    TBK_CHECK(pl.total <= kScratchBytes, TBK_ERR_BUFFER_TOO_SMALL,
              "kpm_moments_noalloc: this run needs %lld bytes of workspace, more than the %lld-byte static "
              "workspace (use kpm_moments_config with a caller-allocated workspace)",
              (long long)pl.total, (long long)kScratchBytes);
    void *work = nullptr;
    st = scratch_address(&work);
    if (st != TBK_OK) return st;
    st = check_moment_args(h, pl, a, b, r, work, (int64_t)kScratchBytes, mu);
    if (st != TBK_OK) return st;
    TBK_CHECK(pl.cfg.persistent == 0, TBK_ERR_INVALID_ARG, "the persistent launch is for kpm_moments_batched");
    st = check_resume(h, pl, a[0], b[0], R, M, precision, work, as_stream(stream));
    if (st != TBK_OK) return st;
    // the step timer's event pool may grow; this entry point makes no such call
    StepTimer &timer = step_timer();
    const bool was_on = timer.on;
    timer.on = false;
    st = run_plan(h, pl, a[0], b[0], r, R, M, precision, static_cast<char *>(work), mu, as_stream(stream),
                  nullptr, nullptr);
    timer.on = was_on;
    return st;
}

extern "C" tbk_status kpm_moments_seeded(const tbk_ham *h, const double *a, const double *b, uint64_t seed,
                                         int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                                         int32_t n_start, void *work, int64_t work_bytes, double *mu,
                                         void *stream) {
    clear_error();
    KpmPlan pl;
    tbk_status st = make_plan(h, R, M, precision, cfg, pl);
    if (st != TBK_OK) return st;
    pl.seeded = true;
    pl.seed = seed;
    pl.n_start = n_start;
    st = check_start(pl, M);
    if (st != TBK_OK) return st;
    st = check_moment_args(h, pl, a, b, nullptr, work, work_bytes, mu);
    if (st != TBK_OK) return st;
    TBK_CHECK(pl.cfg.persistent == 0, TBK_ERR_INVALID_ARG, "the persistent launch is for kpm_moments_batched");
    st = check_resume(h, pl, a[0], b[0], R, M, precision, work, as_stream(stream));
    if (st != TBK_OK) return st;
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
