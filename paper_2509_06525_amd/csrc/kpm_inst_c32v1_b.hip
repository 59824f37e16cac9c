// Instances of the recurrence run for complex-float vectors, 1 vector per thread (kpm_run.hpp).
#include "kpm_run.hpp"

namespace tbk {
template tbk_status run_moments_inst<float, 8, 1>(const tbk_ham *, const KpmPlan &, double, double, const float *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const float *,
                                                   const float *);
template tbk_status run_moments_inst<float, 16, 1>(const tbk_ham *, const KpmPlan &, double, double, const float *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const float *,
                                                   const float *);
template tbk_status run_moments_inst<float, 32, 1>(const tbk_ham *, const KpmPlan &, double, double, const float *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const float *,
                                                   const float *);
template tbk_status run_moments_inst<float, 64, 1>(const tbk_ham *, const KpmPlan &, double, double, const float *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const float *,
                                                   const float *);
}  // namespace tbk
