// Jackson-damped DOS reconstruction, Eq. (4), on the GPU (FP64), its integral
// (states below E), and the frame-averaged conductivity plateau and mobility.
//
// x = (E - b)/a, rho = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(x)] / (a pi sqrt(1 - x^2)),
// T_n(x) by the three-term recurrence, g_n of the Jackson kernel from its closed
// form.  A block serves 256 energies of one structure: the weights
// c_n = g_n mu_n (times 2 for n >= 1) are formed 256 at a time in LDS, one per
// thread, and every thread then runs the recurrence of its energy over them.
#include <cmath>

#include "common.hpp"

namespace tbk {
namespace {

constexpr int kDosThreads = 256;

// grid = (ceil(nE / 256), n_struct); structure s reads mu + s * M, its scale
// and shift (ab[s], ab[n_struct + s], or a0, b0 when ab is NULL),
// E + s * e_stride and writes rho + s * nE.
__global__ __launch_bounds__(kDosThreads) void k_dos(const double *__restrict__ mu, int32_t M, double a0, double b0,
                                                     const double *__restrict__ ab, int32_t kernel,
                                                     const double *__restrict__ E, int64_t e_stride, int32_t nE,
                                                     double *__restrict__ rho) {
    __shared__ double c[kDosThreads];
    const int s = blockIdx.y;
    const int e = blockIdx.x * kDosThreads + threadIdx.x;
    const double *m = mu + (int64_t)s * M;
    const double as = ab ? ab[s] : a0, bs = ab ? ab[gridDim.y + s] : b0;
    const double x = e < nE ? (E[(int64_t)s * e_stride + e] - bs) / as : 0.0;
    const bool inside = fabs(x) < 1.0;
    const double q = M_PI / (M + 1.0);
    const double cot_q = cos(q) / sin(q);
    double acc = 0.0, tm = 0.0, tn = 0.0;   // T_{n-1}, T_n of this thread's energy
    for (int n0 = 0; n0 < M; n0 += kDosThreads) {
        const int n = n0 + threadIdx.x;
        double w = 0.0;
        if (n < M) {
            double g = 1.0;
            if (kernel == 0) {
                double sn, cn;
                sincos(q * n, &sn, &cn);
                g = ((M - n + 1.0) * cn + sn * cot_q) / (M + 1.0);
            }
            w = (n == 0 ? 1.0 : 2.0) * g * m[n];
        }
        __syncthreads();
        c[threadIdx.x] = w;
        __syncthreads();
        const int cnt = min(kDosThreads, M - n0);
        for (int k = 0; k < cnt; ++k) {
            const int nn = n0 + k;
            double t;
            if (nn == 0) t = 1.0;
            else if (nn == 1) t = x;
            else t = 2.0 * x * tn - tm;
            acc += c[k] * t;
            tm = tn;
            tn = t;
        }
    }
    if (e < nE) rho[(int64_t)s * nE + e] = inside ? acc / (as * M_PI * sqrt(1.0 - x * x)) : 0.0;
}

// In place over sigma [n_t][nE] holding the correlation C_j(E): the running
// trapezoidal integral s_0 = 0, s_j = s_{j-1} + dt/2 (C_{j-1} + C_j).
__global__ void k_cumtrapz(double *__restrict__ sigma, int32_t n_t, int32_t nE, double dt) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    double prev = sigma[e], run = 0.0;
    sigma[e] = 0.0;
    for (int32_t j = 1; j < n_t; ++j) {
        const double cj = sigma[(int64_t)j * nE + e];
        run += 0.5 * dt * (prev + cj);
        sigma[(int64_t)j * nE + e] = run;
        prev = cj;
    }
}

// Integrated DOS N(E) of the damped expansion in closed form (x = cos theta):
//   N = g_0 mu_0 (1 - theta/pi) - (2/pi) sum_{n>=1} g_n mu_n sin(n theta) / n,
// 0 below the scaled interval and g_0 mu_0 above it.  sin(n theta) follows the
// same three-term recurrence as T_n (s_0 = 0, s_1 = sin theta); the weights
// are staged in LDS 256 at a time as in k_dos.
__global__ __launch_bounds__(kDosThreads) void k_integrated_dos(const double *__restrict__ mu, int32_t M, double a,
                                                                double b, int32_t kernel,
                                                                const double *__restrict__ E, int32_t nE,
                                                                double *__restrict__ N) {
    __shared__ double c[kDosThreads];
    const int e = blockIdx.x * kDosThreads + threadIdx.x;
    const double x = e < nE ? (E[e] - b) / a : 0.0;
    const double xc = fmin(1.0, fmax(-1.0, x));
    const double sth = sqrt(fmax(0.0, 1.0 - xc * xc));
    const double q = M_PI / (M + 1.0);
    const double cot_q = cos(q) / sin(q);
    double acc = 0.0, sm = 0.0, sn = 0.0;   // sin((n-1) theta), sin(n theta)
    double w0 = 0.0;
    for (int n0 = 0; n0 < M; n0 += kDosThreads) {
        const int n = n0 + threadIdx.x;
        double w = 0.0;
        if (n < M) {
            double g = 1.0;
            if (kernel == 0) {
                double sq, cq;
                sincos(q * n, &sq, &cq);
                g = ((M - n + 1.0) * cq + sq * cot_q) / (M + 1.0);
            }
            w = n == 0 ? g * mu[0] : 2.0 / M_PI * g * mu[n] / n;
        }
        __syncthreads();
        c[threadIdx.x] = w;
        __syncthreads();
        if (n0 == 0) w0 = c[0];
        const int cnt = min(kDosThreads, M - n0);
        for (int k = 0; k < cnt; ++k) {
            const int nn = n0 + k;
            if (nn == 0) continue;
            const double sv = nn == 1 ? sth : 2.0 * xc * sn - sm;
            acc += c[k] * sv;
            sm = sn;
            sn = sv;
        }
    }
    if (e < nE) N[e] = x <= -1.0 ? 0.0 : (x >= 1.0 ? w0 : w0 * (1.0 - acos(xc) / M_PI) - acc);
}

// Frame average, plateau and mobility, one thread per energy:
//   sigma_sc = max_j mean_f sigma[f][j][e], carriers = mean_f N[f][e] - n_ref,
//   mobility = 0.1 sigma_sc / |carriers| (cm^2/(V s); NaN where carriers = 0).
__global__ void k_mobility(const double *__restrict__ sigma, int32_t F, int32_t n_t, int32_t nE,
                           const double *__restrict__ N, double n_ref, double *__restrict__ sigma_sc,
                           double *__restrict__ carriers, double *__restrict__ mobility) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    double best = -INFINITY;
    for (int32_t j = 0; j < n_t; ++j) {
        double m = 0.0;
        for (int32_t f = 0; f < F; ++f) m += sigma[((int64_t)f * n_t + j) * nE + e];
        best = fmax(best, m / F);
    }
    double nb = 0.0;
    for (int32_t f = 0; f < F; ++f) nb += N[(int64_t)f * nE + e];
    nb = nb / F - n_ref;
    sigma_sc[e] = best;
    carriers[e] = nb;
    mobility[e] = nb != 0.0 ? 0.1 * best / fabs(nb) : __builtin_nan("");
}

// mean[s][n] = (1/R) sum_v mu[s][v][n], the sum over v in index order.
__global__ void k_mean_moments(const double *__restrict__ mu, int32_t n_seg, int32_t R, int32_t M,
                               double *__restrict__ mean) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_seg * M) return;
    const int64_t s = idx / M, n = idx % M;
    const double *p = mu + s * R * (int64_t)M + n;
    double acc = 0.0;
    for (int32_t v = 0; v < R; ++v) acc += p[(int64_t)v * M];
    mean[idx] = acc / R;
}

tbk_status check_dos(int32_t M, int32_t nE, int32_t kernel) {
    TBK_CHECK(M >= 1, TBK_ERR_INVALID_ARG, "M = %d < 1", M);
    TBK_CHECK(nE >= 0, TBK_ERR_INVALID_ARG, "nE = %d < 0", nE);
    TBK_CHECK(kernel == 0 || kernel == 1, TBK_ERR_INVALID_ARG, "kernel must be 0 (Jackson) or 1 (none)");
    return TBK_OK;
}

}  // namespace
}  // namespace tbk

using namespace tbk;

extern "C" tbk_status kpm_dos(const double *mu, int32_t M, double a, double b, int32_t kernel, const double *E,
                              int32_t nE, double *rho, void *stream) {
    clear_error();
    tbk_status st = check_dos(M, nE, kernel);
    if (st != TBK_OK) return st;
    TBK_CHECK(std::isfinite(a) && std::isfinite(b), TBK_ERR_NOT_FINITE, "a or b is not finite");
    TBK_CHECK(a > 0, TBK_ERR_INVALID_ARG, "a = %g must be positive", a);
    if (nE == 0) return TBK_OK;
    TBK_CHECK(mu && E && rho, TBK_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = as_stream(stream);
    k_dos<<<dim3((unsigned)ceil_div(nE, kDosThreads), 1), kDosThreads, 0, s>>>(mu, M, a, b, nullptr, kernel, E, 0,
                                                                               nE, rho);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

extern "C" tbk_status kpm_mean_moments(const double *mu, int32_t n_seg, int32_t R, int32_t M, double *mean,
                                       void *stream) {
    clear_error();
    TBK_CHECK(n_seg >= 1 && R >= 1 && M >= 1, TBK_ERR_INVALID_ARG, "n_seg = %d, R = %d, M = %d", n_seg, R, M);
    TBK_CHECK(mu && mean, TBK_ERR_INVALID_ARG, "NULL argument");
    const int64_t n = (int64_t)n_seg * M;
    k_mean_moments<<<(unsigned)ceil_div(n, 256), 256, 0, as_stream(stream)>>>(mu, n_seg, R, M, mean);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

extern "C" tbk_status kpm_dos_batched(const double *mu, int32_t M, int32_t n_struct, const double *a,
                                      const double *b, int32_t kernel, const double *E, int32_t nE, double *rho,
                                      void *stream) {
    clear_error();
    tbk_status st = check_dos(M, nE, kernel);
    if (st != TBK_OK) return st;
    TBK_CHECK(n_struct >= 1 && n_struct <= 65535, TBK_ERR_INVALID_ARG, "n_struct = %d outside [1, 65535]",
              n_struct);
    TBK_CHECK(a && b, TBK_ERR_INVALID_ARG, "a or b is NULL");
    for (int i = 0; i < n_struct; ++i) {
        TBK_CHECK(std::isfinite(a[i]) && std::isfinite(b[i]), TBK_ERR_NOT_FINITE, "a or b of structure %d", i);
        TBK_CHECK(a[i] > 0, TBK_ERR_INVALID_ARG, "a[%d] = %g must be positive", i, a[i]);
    }
    if (nE == 0) return TBK_OK;
    TBK_CHECK(mu && E && rho, TBK_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = as_stream(stream);
    DevBuf ab;
    TBK_HIP(ab.alloc(2 * sizeof(double) * n_struct, s));
    TBK_HIP(hipMemcpyAsync(ab.as<double>(), a, sizeof(double) * n_struct, hipMemcpyHostToDevice, s));
    TBK_HIP(hipMemcpyAsync(ab.as<double>() + n_struct, b, sizeof(double) * n_struct, hipMemcpyHostToDevice, s));
    k_dos<<<dim3((unsigned)ceil_div(nE, kDosThreads), (unsigned)n_struct), kDosThreads, 0, s>>>(
        mu, M, 0.0, 0.0, ab.as<double>(), kernel, E, nE, nE, rho);
    TBK_HIP(hipGetLastError());
    TBK_HIP(hipStreamSynchronize(s));    // the caller's a and b must outlive the transfer
    return TBK_OK;
}

extern "C" tbk_status lsqt_sigma(const double *nu, int32_t M, int32_t n_t, double dt, double a, double b,
                                 int32_t kernel, const double *E, int32_t nE, double *sigma, void *stream) {
    clear_error();
    tbk_status st = check_dos(M, nE, kernel);
    if (st != TBK_OK) return st;
    TBK_CHECK(n_t >= 1 && n_t <= 65535, TBK_ERR_INVALID_ARG, "n_t = %d outside [1, 65535]", n_t);
    TBK_CHECK(std::isfinite(a) && std::isfinite(b) && std::isfinite(dt), TBK_ERR_NOT_FINITE,
              "a, b or dt is not finite");
    TBK_CHECK(a > 0 && dt > 0, TBK_ERR_INVALID_ARG, "a and dt must be positive");
    if (nE == 0) return TBK_OK;
    TBK_CHECK(nu && E && sigma, TBK_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = as_stream(stream);
    k_dos<<<dim3((unsigned)ceil_div(nE, kDosThreads), (unsigned)n_t), kDosThreads, 0, s>>>(
        nu, M, a, b, nullptr, kernel, E, 0, nE, sigma);
    k_cumtrapz<<<(unsigned)ceil_div(nE, 256), 256, 0, s>>>(sigma, n_t, nE, dt);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

extern "C" tbk_status kpm_integrated_dos(const double *mu, int32_t M, double a, double b, int32_t kernel,
                                         const double *E, int32_t nE, double *N, void *stream) {
    clear_error();
    tbk_status st = check_dos(M, nE, kernel);
    if (st != TBK_OK) return st;
    TBK_CHECK(std::isfinite(a) && std::isfinite(b), TBK_ERR_NOT_FINITE, "a or b is not finite");
    TBK_CHECK(a > 0, TBK_ERR_INVALID_ARG, "a = %g must be positive", a);
    if (nE == 0) return TBK_OK;
    TBK_CHECK(mu && E && N, TBK_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = as_stream(stream);
    k_integrated_dos<<<(unsigned)ceil_div(nE, kDosThreads), kDosThreads, 0, s>>>(mu, M, a, b, kernel, E, nE, N);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}

extern "C" tbk_status lsqt_mobility(const double *sigma, int32_t n_frames, int32_t n_t, int32_t nE, const double *N,
                                    double n_ref, double *sigma_sc, double *carriers, double *mobility,
                                    void *stream) {
    clear_error();
    TBK_CHECK(n_frames >= 1 && n_t >= 1 && nE >= 0, TBK_ERR_INVALID_ARG, "n_frames = %d, n_t = %d, nE = %d",
              n_frames, n_t, nE);
    TBK_CHECK(std::isfinite(n_ref), TBK_ERR_NOT_FINITE, "n_ref is not finite");
    if (nE == 0) return TBK_OK;
    TBK_CHECK(sigma && N && sigma_sc && carriers && mobility, TBK_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = as_stream(stream);
    k_mobility<<<(unsigned)ceil_div(nE, 256), 256, 0, s>>>(sigma, n_frames, n_t, nE, N, n_ref, sigma_sc, carriers,
                                                           mobility);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}
