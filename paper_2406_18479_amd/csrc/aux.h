// Launchers of the small element-wise and reduction kernels (aux.hip).
#pragma once

#include "internal.h"

namespace green {

hipError_t launch_density(const double2* G, double2* gam, double2* gamT, int ns, int ntau, int nk, int nao,
                          hipStream_t s);
// dst[t] = src[nt - 1 - t]^T (conj: the conjugate transpose) for t in [t_lo, t_hi) (n x n complex matrices;
// src and dst may be the same array when the two t ranges do not overlap).
hipError_t launch_transpose_reverse(const double2* src, double2* dst, int n, int nt, int t_lo, int t_hi,
                                   hipStream_t s, bool conj = false);
// Momenta that are not contracted: for every block b < nblk and momentum k with kfill[k] != k,
// X[b][k] = X[b][kfill[k]] (kfill[k] < nk, a symmetry copy) or conj X[b][kfill[k] - nk] (time reversal), element by
// element (blocks of nk matrices of ne elements; kfill on the device, every source has kfill[src] == src).
hipError_t launch_fill_k(double2* X, int64_t nblk, int nk, int64_t ne, const int32_t* kfill, hipStream_t s);
// Hermitian partner slab: out[k][Q][i][j] = conj(in[kmap[k]][Q][j][i]) for k < nk (naux blocks of nao x nao per k).
hipError_t launch_herm_partner(const double2* in, double2* out, int nk, int naux, int nao, const int32_t* kmap,
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
// dst[b] = I - src[b] (n x n matrices), dst = src (n elements)
hipError_t launch_one_minus_copy(const double2* src, double2* dst, int n, int64_t batch, hipStream_t s);
hipError_t launch_copy(const double2* src, double2* dst, int64_t n, hipStream_t s);
// Input checks (asynchronous): `bit` is set in *status when the largest |difference| exceeds tol times the
// largest |value| (or a value is not finite).  partial: 512 doubles of scratch.
//   k:      X[b][k] against its source under kfill, as launch_fill_k (nblk blocks of nk matrices of ne elements)
//   herm:   X_b against X_b^dagger (nmat n x n matrices)
//   v:      V[q][k][Q] against V[-q][k+q][Q]^dagger (mode 0) or conj V[-q][-k][Q] (mode 1), on three Q
//   v_rot:  V[q][k][Q] against V[R q][R k][Q] for each of nops operations (krot[r nk + k] = R k), on three Q
hipError_t launch_check_k(const double2* X, int64_t nblk, int nk, int64_t ne, const int32_t* kfill, double tol,
                          int bit, double* partial, int* status, hipStream_t s);
hipError_t launch_check_herm(const double2* X, int64_t nmat, int n, double tol, int bit, double* partial, int* status,
                             hipStream_t s);
hipError_t launch_check_v(const double2* V, int nk, int naux, int nao, const int32_t* kadd, const int32_t* kneg,
                          int mode, double tol, int bit, double* partial, int* status, hipStream_t s);
hipError_t launch_check_v_rot(const double2* V, int nk, int naux, int nao, const int32_t* krot, int nops, double tol,
                              int bit, double* partial, int* status, hipStream_t s);

// DIIS: *out = sum Re(conj(a) b) (fixed-order reduction through partial[mix_blocks(n)]); r = x - old;
// out = sum_j c_j base[slot_j * stride + .] with *out_max = max |out_new - out_old|.
struct CombineCoefs {
  int32_t m;
  int32_t slot[16];
  double c[16];
};
hipError_t launch_dot_re(const double2* a, const double2* b, int64_t n, double* partial, double* out, hipStream_t s);
hipError_t launch_sub(double2* r, const double2* x, const double2* old, int64_t n, hipStream_t s);
hipError_t launch_combine(double2* out, const double2* base, int64_t stride, int64_t n, const CombineCoefs& cf,
                          double* partial, double* out_max, hipStream_t s);

}  // namespace green
