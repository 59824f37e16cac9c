// Autotuner of the recurrence: SELL slice height and kernel launch shape.
//
// For one structure, every candidate slice height is built once; for each
// candidate launch shape a short recurrence (warm-up, then `steps` timed steps
// with HIP events on the caller's stream) is run on unit-modulus vectors, and
// the fastest (slice, shape) pair is returned.  Results are cached per device
// and problem class in memory and, when TBKPM_AUTOTUNE_CACHE names a file, in
// that file (one line per entry); TBKPM_AUTOTUNE=0 returns the defaults
// without timing.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "kpm.hpp"

namespace tbk {
namespace {

constexpr int kThreads = 256;

// Unit-modulus test vectors exp(i phi), phi from an integer hash of (row, vector).
template <class VT>
__global__ void k_tune_vectors(VT *r, int64_t n, int32_t R) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * R) return;
    uint64_t x = (uint64_t)idx * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    x ^= x >> 31;
    x *= 0xD6E8FEB86659FD93ull;
    x ^= x >> 32;
    const double phi = 6.283185307179586 * (double)(x & 0xFFFFFFFFull) / 4294967296.0;
    r[2 * idx] = (VT)cos(phi);
    r[2 * idx + 1] = (VT)sin(phi);
}

struct Key {
    std::string text;
    bool operator<(const Key &o) const { return text < o.text; }
};

std::mutex g_mu;
std::map<Key, tbk_tune_result> g_cache;
bool g_file_loaded = false;

std::string cache_path() {
    const char *p = std::getenv("TBKPM_AUTOTUNE_CACHE");
    return p ? std::string(p) : std::string();
}

void load_file_cache() {
    if (g_file_loaded) return;
    g_file_loaded = true;
    std::string path = cache_path();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        char key[512];
        tbk_tune_result r{};
        r.config.persistent = 0;
        r.config.doubling = 0;
        r.config.uniform_values = 0;
        int compact = 0;
        const int got = std::sscanf(line, "%511s %d %d %d %d %d %d %lf %d", key, &r.slice,
                                    &r.config.vectors_per_thread, &r.config.tiles_per_block,
                                    &r.config.nontemporal, &r.config.xcd_remap, &r.config.rows_per_thread,
                                    &r.ms_per_step, &compact);
        if (got == 8 || got == 9) {
            r.config.compact_columns = got == 9 ? compact : 0;
            r.from_cache = 1;
            r.config.doubling = std::strstr(key, "/dbl1") ? 1 : 0;
            r.config.uniform_values = std::strstr(key, "/uv1") ? 1 : 0;
            g_cache[Key{key}] = r;
        }
    }
    std::fclose(f);
}

void append_file_cache(const Key &k, const tbk_tune_result &r) {
    std::string path = cache_path();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d %d %.6f %d\n", k.text.c_str(), r.slice, r.config.vectors_per_thread,
                 r.config.tiles_per_block, r.config.nontemporal, r.config.xcd_remap, r.config.rows_per_thread,
                 r.ms_per_step, r.config.compact_columns);
    std::fclose(f);
}

Key make_key(int device, const char *arch, int64_t n, int32_t R, int32_t precision, int32_t fmt,
             const tbk_ham &h0, int32_t doubling, int32_t uniform_values) {
    int lg = 0;
    while (((int64_t)1 << (lg + 1)) <= n) ++lg;
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s/dev%d/n2^%d/R%d/p%d/f%d/deg%d/ons%d%s%s", arch, device, lg, R, precision,
                  fmt, h0.max_degree, h0.has_onsite, doubling ? "/dbl1" : "", uniform_values ? "/uv1" : "");
    return Key{buf};
}

// Owns the device arrays of one Hamiltonian built for tuning.
struct TuneHam {
    tbk_ham h{};
    DevBuf ptr, col, col16, val, onsite, perm;
};

tbk_status build_tune_ham(const double *pos, const int32_t *species, int64_t n, const double box[3],
                          const int32_t periodic[3], const tbk_tb_params *p, int32_t fmt, int32_t slice,
                          TuneHam &t, double bounds[2], hipStream_t s) {
    t.h = tbk_ham{};
    t.h.fmt = fmt;
    t.h.slice = slice;
    tbk_status st = tbk_hamiltonian_size(pos, species, n, box, periodic, p, &t.h, s);
    if (st != TBK_OK) return st;
    const size_t vb = fmt == TBK_SELL_F32 ? sizeof(float) : sizeof(double);
    TBK_HIP(t.ptr.alloc(sizeof(int64_t) * t.h.n_ptr, s));
    TBK_HIP(t.col.alloc(sizeof(int32_t) * std::max<int64_t>(t.h.n_entries, 1), s));
    TBK_HIP(t.val.alloc(vb * std::max<int64_t>(t.h.n_entries, 1), s));
    TBK_HIP(t.onsite.alloc(vb * n, s));
    TBK_HIP(t.perm.alloc(sizeof(int32_t) * n, s));
    TBK_HIP(t.col16.alloc(sizeof(int16_t) * std::max<int64_t>(t.h.n_entries, 1), s));
    t.h.col16 = t.col16.as<int16_t>();
    t.h.ptr = t.ptr.as<int64_t>();
    t.h.col = t.col.as<int32_t>();
    t.h.val = t.val.as<void>();
    t.h.onsite = t.onsite.as<void>();
    t.h.perm = t.perm.as<int32_t>();
    return tb_build_hamiltonian(pos, species, n, box, periodic, p, &t.h, bounds, s);
}

tbk_status time_shape(const tbk_ham &h, const tbk_kpm_config &cfg, int32_t R, int32_t steps, int32_t precision,
                      double a, double b, const void *r, double *mu, hipStream_t s, double *ms_out) {
    KpmPlan pl;
    const int M = cfg.doubling ? 2 * steps + 1 : steps + 1;   // `steps` launches either way
    tbk_status st = make_plan(&h, R, M, precision, &cfg, pl);
    if (st != TBK_OK) return st;
    DevBuf work;
    TBK_HIP(work.alloc(pl.total, s));
    char *w = work.as<char>();
    // warm-up, then the timed run
    st = run_plan(&h, pl, a, b, r, R, M, precision, w, mu, s);
    if (st != TBK_OK) return st;
    hipEvent_t e0, e1;
    TBK_HIP(hipEventCreate(&e0));
    TBK_HIP(hipEventCreate(&e1));
    TBK_HIP(hipEventRecord(e0, s));
    st = run_plan(&h, pl, a, b, r, R, M, precision, w, mu, s);
    TBK_HIP(hipEventRecord(e1, s));
    TBK_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    TBK_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != TBK_OK) return st;
    *ms_out = ms / steps;
    return TBK_OK;
}

}  // namespace
}  // namespace tbk

using namespace tbk;

namespace {

tbk_status autotune_impl(const double *pos, const int32_t *species, int64_t n, const double box[3],
                         const int32_t periodic[3], const tbk_tb_params *p, int32_t fmt, int32_t R,
                         int32_t precision, int32_t steps, int32_t doubling, int32_t uniform_values,
                         tbk_tune_result *out, void *stream) {
    TBK_CHECK(out != nullptr, TBK_ERR_INVALID_ARG, "out is NULL");
    TBK_CHECK(R >= 1 && R <= 64, TBK_ERR_INVALID_ARG, "R = %d outside [1, 64]", R);
    TBK_CHECK(steps >= 1 && steps <= 1000, TBK_ERR_INVALID_ARG, "steps = %d outside [1, 1000]", steps);
    TBK_CHECK(fmt == TBK_SELL_F32 || fmt == TBK_SELL_F64, TBK_ERR_INVALID_ARG, "tuning needs a SELL format");
    TBK_CHECK((precision == TBK_PREC_C32) == (fmt == TBK_SELL_F32), TBK_ERR_INVALID_ARG,
              "precision and format disagree");
    hipStream_t s = as_stream(stream);
    const int Rp = pad_vectors(R);
    const int vpt_max = (precision == TBK_PREC_C32 && Rp >= 2) ? 2 : 1;

    // A first build at the default slice gives the problem class for the cache key.
    TuneHam t0;
    double bounds[2];
    const int rpb1 = kThreads / (Rp / vpt_max);
    tbk_status st = build_tune_ham(pos, species, n, box, periodic, p, fmt, rpb1, t0, bounds, s);
    if (st != TBK_OK) return st;
    int dev = 0;
    TBK_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    TBK_HIP(hipGetDeviceProperties(&prop, dev));
    const Key key = make_key(dev, prop.gcnArchName, n, R, precision, fmt, t0.h, doubling, uniform_values);
    TBK_CHECK(uniform_values == 0 || t0.h.uniform_hop == 1, TBK_ERR_INVALID_ARG,
              "uniform_values: the structure's hoppings are not all equal");

    tbk_tune_result best{};
    best.slice = rpb1;
    best.config = default_config(&t0.h, R, precision);
    best.config.doubling = doubling;
    best.config.uniform_values = uniform_values;
    best.ms_per_step = -1.0;
    const char *env = std::getenv("TBKPM_AUTOTUNE");
    if (env && std::string(env) == "0") {
        *out = best;
        return TBK_OK;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_file_cache();
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            *out = it->second;
            out->from_cache = 1;
            return TBK_OK;
        }
    }

    const double a = 1.01 * (bounds[1] - bounds[0]) / 2.0, b = (bounds[1] + bounds[0]) / 2.0;
    const size_t elem = precision == TBK_PREC_C32 ? sizeof(float) : sizeof(double);
    DevBuf rbuf, mubuf;
    TBK_HIP(rbuf.alloc((size_t)n * R * 2 * elem, s));
    TBK_HIP(mubuf.alloc(sizeof(double) * R * (2 * steps + 1), s));
    const int64_t nv = n * R;
    if (precision == TBK_PREC_C32)
        k_tune_vectors<float><<<(unsigned)ceil_div(nv, 256), 256, 0, s>>>(rbuf.as<float>(), n, R);
    else
        k_tune_vectors<double><<<(unsigned)ceil_div(nv, 256), 256, 0, s>>>(rbuf.as<double>(), n, R);
    TBK_HIP(hipGetLastError());

    int tried = 0;
    for (int vpt = 1; vpt <= vpt_max; ++vpt) {
        const int rpb = kThreads / (Rp / vpt);
        for (int sf : {1, 4, 16}) {          // slice = rpb, rpb / 4, rpb / 16 (at least 1)
            const int slice = std::max(1, rpb / sf);
            TuneHam th;
            const tbk_ham *hp = &t0.h;
            if (slice != rpb1) {
                double bb[2];
                st = build_tune_ham(pos, species, n, box, periodic, p, fmt, slice, th, bb, s);
                if (st != TBK_OK) return st;
                hp = &th.h;
                TBK_CHECK(uniform_values == 0 || th.h.uniform_hop == 1, TBK_ERR_INVALID_ARG,
                          "uniform_values: the hoppings are not all equal at slice %d", slice);
            }
            for (int tpb : {1, 2, 4, 8})
                for (int rpt : {1, 2, 4}) {
                    if (rpt > tpb) continue;
                    if (rpt == 4 && (Rp / vpt != 1 || hp->max_degree != 3)) continue;   // see rows_per_thread
                    for (int nt : {0, 1})
                        for (int xr : {0, 1, 2, 3})
                        for (int cc : {0, 1}) {
                            tbk_kpm_config c{};
                            c.compact_columns = cc;
                            c.vectors_per_thread = vpt;
                            c.tiles_per_block = tpb;
                            c.rows_per_thread = rpt;
                            c.nontemporal = nt;
                            c.xcd_remap = xr;
                            c.persistent = 0;
                            c.doubling = doubling;
                            c.uniform_values = uniform_values;
                            double ms = 0.0;
                            st = time_shape(*hp, c, R, steps, precision, a, b, rbuf.as<void>(),
                                            mubuf.as<double>(), s, &ms);
                            if (st != TBK_OK) return st;
                            ++tried;
                            if (best.ms_per_step < 0 || ms < best.ms_per_step) {
                                best.ms_per_step = ms;
                                best.slice = slice;
                                best.config = c;
                            }
                        }
                }
            if (slice == 1) break;
        }
    }
    best.candidates = tried;
    best.from_cache = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = best;
        append_file_cache(key, best);
    }
    *out = best;
    return TBK_OK;
}

}  // namespace

extern "C" tbk_status tbk_autotune(const double *pos, const int32_t *species, int64_t n, const double box[3],
                                   const int32_t periodic[3], const tbk_tb_params *p, int32_t fmt, int32_t R,
                                   int32_t precision, int32_t steps, tbk_tune_result *out, void *stream) {
    clear_error();
    return autotune_impl(pos, species, n, box, periodic, p, fmt, R, precision, steps, 0, 0, out, stream);
}

extern "C" tbk_status tbk_autotune_form(const double *pos, const int32_t *species, int64_t n, const double box[3],
                                        const int32_t periodic[3], const tbk_tb_params *p, int32_t fmt, int32_t R,
                                        int32_t precision, int32_t steps, const tbk_kpm_config *form,
                                        tbk_tune_result *out, void *stream) {
    clear_error();
    const int32_t dbl = form ? form->doubling : 0, uv = form ? form->uniform_values : 0;
    TBK_CHECK(dbl == 0 || dbl == 1, TBK_ERR_INVALID_ARG, "form->doubling must be 0/1");
    TBK_CHECK(uv == 0 || uv == 1, TBK_ERR_INVALID_ARG, "form->uniform_values must be 0/1");
    return autotune_impl(pos, species, n, box, periodic, p, fmt, R, precision, steps, dbl, uv, out, stream);
}
