// Batched in-place inversion of complex FP64 matrices (n <= 512): blocked
// Gauss-Jordan elimination with partial pivoting, one workgroup per matrix.
//
// Used for the screening step [I - P~0(i W)]^{-1} (n = naux, Eq. tilde_P_omega)
// and for the Dyson inversion at every (s, k, i w_m) (n = nao, Eq. dyson).
//
// Per panel of nb columns (nb chosen so the n x nb panel fits in LDS):
//   1. the panel is eliminated in LDS column by column: pivot = largest |a_ik|
//      among the not yet pivoted rows (ties: lowest row), row swap, pivot-row
//      scaling and a rank-1 update of every other panel row; afterwards the
//      panel holds the nb columns of the accumulated elimination operator E;
//   2. every column j outside the panel is updated in one pass,
//        A[:, j] <- (P A[:, j] with the pivot rows zeroed) + E[:, panel] (P A)[panel rows, j],
//      where P is the panel's row permutation (read phase, barrier, write phase);
//   3. the panel is written back.
// After the last panel the columns are unscrambled (swaps undone in reverse order).
// Each panel reads and writes the matrix once, so the traffic is
// (n / nb) * 2 * 16 n^2 bytes per matrix.
#include <algorithm>

#include "internal.h"

namespace green {
namespace {

constexpr int kMaxN = 512;
constexpr int kCW = 8;             // columns per update block
constexpr int kMaxR = kMaxN / 32;  // rows per thread in the update phase

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(256) void zinv_kernel(double2* __restrict__ A, int n, int64_t stride, int nb,
                                                   int* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2* P = reinterpret_cast<double2*>(smem);  // [n][nb]
  double2* colc = P + (size_t)n * nb;             // [n]
  double2* prow = colc + n;                       // [nb]
  double2* BKs = prow + nb;                       // [nb][kCW]
  double* rv = reinterpret_cast<double*>(BKs + (size_t)nb * kCW);  // [4]
  int* ri = reinterpret_cast<int*>(rv + 4);                       // [4]
  int* pi = ri + 4;                                               // [n]
  int* perm = pi + n;                                             // [n]
  int* cols = perm + n;                                           // [n]

  double2* __restrict__ M = A + (int64_t)blockIdx.x * stride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double2 zero = make_double2(0.0, 0.0);
  bool any_swap = false;

  for (int k0 = 0; k0 < n; k0 += nb) {
    const int w = min(nb, n - k0);
    for (int idx = tid; idx < n * w; idx += 256) {
      const int i = idx / w, c = idx - i * w;
      P[i * nb + c] = M[(int64_t)i * n + k0 + c];
    }
    for (int i = tid; i < n; i += 256) pi[i] = i;
    __syncthreads();

    for (int c = 0; c < w; ++c) {
      const int k = k0 + c;
      double best = -1.0;
      int bi = n;
      for (int i = k + tid; i < n; i += 256) {
        const double2 v = P[i * nb + c];
        const double a = v.x * v.x + v.y * v.y;
        if (a > best) {
          best = a;
          bi = i;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_down(best, off);
        const int oi = __shfl_down(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) {
        rv[wave] = best;
        ri[wave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        double b = rv[0];
        int p = ri[0];
        for (int q = 1; q < 4; ++q)
          if (rv[q] > b || (rv[q] == b && ri[q] < p)) {
            b = rv[q];
            p = ri[q];
          }
        if (p >= n) p = k;
        perm[k] = p;
      }
      __syncthreads();
      const int p = perm[k];
      if (p != k) {
        any_swap = true;
        for (int cc = tid; cc < w; cc += 256) {
          const double2 t = P[k * nb + cc];
          P[k * nb + cc] = P[p * nb + cc];
          P[p * nb + cc] = t;
        }
        if (tid == 0) {
          const int t = pi[k];
          pi[k] = pi[p];
          pi[p] = t;
        }
      }
      __syncthreads();
      const double2 piv = P[k * nb + c];
      const double pa = piv.x * piv.x + piv.y * piv.y;
      double2 ipiv = zero;
      if (pa > 0.0 && pa <= 1.0e300) {
        ipiv = make_double2(piv.x / pa, -piv.y / pa);
      } else if (tid == 0) {
        atomicOr(status, 1);
      }
      if (tid < w) prow[tid] = (tid == c) ? ipiv : cmul(P[k * nb + tid], ipiv);
      for (int i = tid; i < n; i += 256) colc[i] = P[i * nb + c];
      __syncthreads();
      for (int idx = tid; idx < n * w; idx += 256) {
        const int i = idx / w, cc = idx - i * w;
        double2 v;
        if (i == k) {
          v = prow[cc];
        } else if (cc == c) {
          const double2 t = cmul(colc[i], ipiv);
          v = make_double2(-t.x, -t.y);
        } else {
          const double2 t = cmul(colc[i], prow[cc]);
          const double2 o = P[i * nb + cc];
          v = make_double2(o.x - t.x, o.y - t.y);
        }
        P[i * nb + cc] = v;
      }
      __syncthreads();
    }

    // ---- update all columns outside the panel
    if (w < n) {
      const int jj = tid & (kCW - 1);
      const int rg = tid >> 3;  // 32 row groups
      for (int j0 = 0; j0 < n; j0 += kCW) {
        if (j0 >= k0 && j0 + kCW <= k0 + w) continue;  // block entirely inside the panel
        const int j = j0 + jj;
        const bool jval = j < n && (j < k0 || j >= k0 + w);
        for (int idx = tid; idx < w * kCW; idx += 256) {
          const int cc = idx / kCW, j2 = idx - cc * kCW;
          const int jg = j0 + j2;
          const bool ok = jg < n && (jg < k0 || jg >= k0 + w);
          BKs[cc * kCW + j2] = ok ? M[(int64_t)pi[k0 + cc] * n + jg] : zero;
        }
        double2 old[kMaxR];
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
          const int i = rg + 32 * r;
          old[r] = (jval && i < n && (i < k0 || i >= k0 + w)) ? M[(int64_t)pi[i] * n + j] : zero;
        }
        __syncthreads();
        if (jval) {
#pragma unroll
          for (int r = 0; r < kMaxR; ++r) {
            const int i = rg + 32 * r;
            if (i < n) {
              double2 acc = old[r];
              for (int cc = 0; cc < w; ++cc) {
                const double2 t = cmul(P[i * nb + cc], BKs[cc * kCW + jj]);
                acc.x += t.x;
                acc.y += t.y;
              }
              M[(int64_t)i * n + j] = acc;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int idx = tid; idx < n * w; idx += 256) {
      const int i = idx / w, c = idx - i * w;
      M[(int64_t)i * n + k0 + c] = P[i * nb + c];
    }
    __syncthreads();
  }

  // ---- undo the row interchanges on the columns (reverse order)
  if (__syncthreads_or(any_swap ? 1 : 0)) {
    if (tid == 0) {
      for (int j = 0; j < n; ++j) cols[j] = j;
      for (int k = n - 1; k >= 0; --k) {
        const int p = perm[k];
        const int t = cols[k];
        cols[k] = cols[p];
        cols[p] = t;
      }
    }
    __syncthreads();
    const int rb = max(1, (256 * kMaxR) / n < 8 ? (256 * kMaxR) / n : 8);
    for (int i0 = 0; i0 < n; i0 += rb) {
      const int cnt = min(rb, n - i0) * n;
      double2 v[kMaxR];
#pragma unroll
      for (int r = 0; r < kMaxR; ++r) {
        const int idx = tid + 256 * r;
        if (idx < cnt) {
          const int i = i0 + idx / n, j = idx - (idx / n) * n;
          v[r] = M[(int64_t)i * n + cols[j]];
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kMaxR; ++r) {
        const int idx = tid + 256 * r;
        if (idx < cnt) {
          const int i = i0 + idx / n, j = idx - (idx / n) * n;
          M[(int64_t)i * n + j] = v[r];
        }
      }
      __syncthreads();
    }
  }
}

// LDS per workgroup for the panel.  Measured on MI355X: a wider panel (up to 150 KiB) cuts the number of
// full-matrix passes but costs occupancy and lengthens the serial column steps, and was slower for
// naux = 180 than this 56 KiB budget (which also needs no raised dynamic-LDS limit); at naux = 300 (1918 matrices
// per screening call) 100 and 150 KiB took the call from 82 ms to 100 and 97 ms.  Update blocks of 16 columns
// instead of kCW = 8 (half the barriers of the update phase) took it to 118 ms: the 32 rows each thread then holds
// leave one wave per SIMD.
size_t lds_budget() { return 56 * 1024; }

}  // namespace

hipError_t zinv_batched(double2* A, int n, int64_t stride, int batch, int* status, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (n <= 0 || n > kMaxN) return hipErrorInvalidValue;
  if (dryrun()) return hipSuccess;
  const size_t budget = lds_budget();
  int nb = (int)((budget - 32 * (size_t)n) / (16 * (size_t)n));
  nb = nb < 1 ? 1 : (nb > 32 ? 32 : nb);
  if (nb > n) nb = n;
  const size_t lds = 16 * ((size_t)n * nb + n + nb + (size_t)nb * kCW) + 8 * 4 + 4 * 4 + 4 * 3 * (size_t)n;
  hipLaunchKernelGGL(zinv_kernel, dim3(batch), dim3(256), lds, s, A, n, stride, nb, status);
  return hipGetLastError();
}

}  // namespace green
