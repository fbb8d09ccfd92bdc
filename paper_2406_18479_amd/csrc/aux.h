// Launchers of the small element-wise and reduction kernels (aux.hip).
#pragma once

#include "internal.h"

namespace green {

hipError_t launch_density(const double2* G, double2* gam, double2* gamT, int ns, int ntau, int nk, int nao,
                          hipStream_t s);
hipError_t launch_one_minus(double2* A, int n, int64_t batch, hipStream_t s);
hipError_t launch_minus_one(double2* A, int n, int64_t batch, hipStream_t s);
hipError_t launch_dyson_form(double2* A, const double2* S, const double2* H0, const double2* Sinf,
                             const double2* Sw, const double* wf, double mu, int ns, int nw, int nk, int nao,
                             hipStream_t s);
hipError_t launch_trace_prod(const double2* X, int64_t xs, const double2* Y, int64_t ydiv, int64_t ymod, int64_t ys,
                             int64_t ys2, int nao, int64_t nb, double2* tr, hipStream_t s);
hipError_t launch_weighted_sum(const double2* tr, int64_t n, const double2* w, int64_t wdiv, int64_t wmod,
                               int64_t wstride, double scale, double* out, hipStream_t s);
int mix_blocks(int64_t n);
hipError_t launch_mix(double2* S, const double2* Snew, double alpha, int64_t n, double* partial, double* out,
                      hipStream_t s);
hipError_t launch_herm(const double2* X, int64_t nmat, int nao, double* partial, double* out, hipStream_t s);
hipError_t launch_zero(double2* X, int64_t n, hipStream_t s);

}  // namespace green
