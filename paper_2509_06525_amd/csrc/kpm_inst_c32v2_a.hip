// Instances of the recurrence run for complex-float vectors, 2 vectors per thread (kpm_run.hpp).
#include "kpm_run.hpp"

namespace tbk {
template tbk_status run_moments_inst<float, 1, 2>(const tbk_ham *, const KpmPlan &, double, double, const float *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const float *,
                                                   const float *);
template tbk_status run_moments_inst<float, 2, 2>(const tbk_ham *, const KpmPlan &, double, double, const float *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const float *,
                                                   const float *);
template tbk_status run_moments_inst<float, 4, 2>(const tbk_ham *, const KpmPlan &, double, double, const float *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const float *,
                                                   const float *);
}  // namespace tbk
