// Jackson-damped DOS reconstruction, Eq. (4), on the GPU (FP64).
//
// One thread per energy: x = (E - b)/a, Chebyshev polynomials T_n(x) by their
// three-term recurrence, damping factors g_n of the Jackson kernel computed from
// their closed form, rho = [g_0 mu_0 + 2 sum g_n mu_n T_n(x)] / (a pi sqrt(1 - x^2)).
#include <cmath>

#include "common.hpp"

namespace tbk {
namespace {

__global__ void k_dos(const double *__restrict__ mu, int32_t M, double a, double b, int32_t kernel,
                      const double *__restrict__ E, int32_t nE, double *__restrict__ rho) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    const double x = (E[e] - b) / a;
    if (!(fabs(x) < 1.0)) { rho[e] = 0.0; return; }
    const double q = M_PI / (M + 1.0);
    const double cot_q = cos(q) / sin(q);
    double s = mu[0];                       // g_0 = 1 for both kernels
    double tm = 1.0, tn = x;
    for (int n = 1; n < M; ++n) {
        double g = 1.0;
        if (kernel == 0) {
            double sn, cn;
            sincos(q * n, &sn, &cn);
            g = ((M - n + 1.0) * cn + sn * cot_q) / (M + 1.0);
        }
        s += 2.0 * g * mu[n] * tn;
        const double tp = 2.0 * x * tn - tm;
        tm = tn;
        tn = tp;
    }
    rho[e] = s / (a * M_PI * sqrt(1.0 - x * x));
}

}  // namespace
}  // namespace tbk

using namespace tbk;

extern "C" tbk_status kpm_dos(const double *mu, int32_t M, double a, double b, int32_t kernel, const double *E,
                              int32_t nE, double *rho, void *stream) {
    clear_error();
    TBK_CHECK(M >= 1, TBK_ERR_INVALID_ARG, "M = %d < 1", M);
    TBK_CHECK(nE >= 0, TBK_ERR_INVALID_ARG, "nE = %d < 0", nE);
    TBK_CHECK(kernel == 0 || kernel == 1, TBK_ERR_INVALID_ARG, "kernel must be 0 (Jackson) or 1 (none)");
    TBK_CHECK(std::isfinite(a) && std::isfinite(b), TBK_ERR_NOT_FINITE, "a or b is not finite");
    TBK_CHECK(a > 0, TBK_ERR_INVALID_ARG, "a = %g must be positive", a);
    if (nE == 0) return TBK_OK;
    TBK_CHECK(mu && E && rho, TBK_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = as_stream(stream);
    k_dos<<<(nE + 255) / 256, 256, 0, s>>>(mu, M, a, b, kernel, E, nE, rho);
    TBK_HIP(hipGetLastError());
    return TBK_OK;
}
