// Instances of the recurrence run for complex-double vectors, 1 vector per thread (kpm_run.hpp).
#include "kpm_run.hpp"

namespace tbk {
template tbk_status run_moments_inst<double, 8, 1>(const tbk_ham *, const KpmPlan &, double, double, const double *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const double *,
                                                   const double *);
template tbk_status run_moments_inst<double, 16, 1>(const tbk_ham *, const KpmPlan &, double, double, const double *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const double *,
                                                   const double *);
template tbk_status run_moments_inst<double, 32, 1>(const tbk_ham *, const KpmPlan &, double, double, const double *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const double *,
                                                   const double *);
template tbk_status run_moments_inst<double, 64, 1>(const tbk_ham *, const KpmPlan &, double, double, const double *,
                                                   int32_t, int32_t, char *, double *, hipStream_t, const double *,
                                                   const double *);
}  // namespace tbk
