// Batched complex FP64 GEMM on CDNA matrix cores (v_mfma_f64_16x16x4f64), 4M form.
//
// Every contraction of the GW hot path (the P~0 and Sigma~ stages, the
// Matsubara transforms, the Hartree-Fock terms) is a batched GEMM whose
// operands are strided views of the layouts in green_gw.h.  Two-level index
// maps let one kernel read "middle index" contractions such as
// X(Q) = A(Q) G, and per-batch tables supply the k+q / k-q lookups.
//
// Tiling: a 256-thread workgroup (4 waves in a 2 x 2 grid) computes a
// (32 WM) x (32 WN) tile; each wave owns WM x WN blocks of 16 x 16.  The K
// loop stages 8-deep complex slabs of A and B through LDS (double buffered,
// conjugation applied when staging), and each 4-deep sub-slab issues four
// real MFMAs per block:
//   C_re += A_re B_re - A_im B_im,   C_im += A_re B_im + A_im B_re.
#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "internal.h"

namespace green {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t map_idx(const IdxMap& m, int32_t x) {
  if (m.ext == kFlat) return (int64_t)x * m.s_in;
  const int32_t hi = x / m.ext;
  const int32_t lo = x - hi * m.ext;
  return (int64_t)lo * m.s_in + (int64_t)hi * m.s_out;
}

__device__ __forceinline__ int64_t batch_off(const BatchMap& b, int32_t x) {
  int32_t lo = x, hi = 0;
  if (b.ext_lo != kFlat) {
    hi = x / b.ext_lo;
    lo = x - hi * b.ext_lo;
  }
  const int64_t l = b.tab ? (int64_t)b.tab[lo] : (int64_t)lo;
  return l * b.s_lo + (int64_t)hi * b.s_hi;
}

template <int WM, int WN, Site SITE>
__global__ __launch_bounds__(256) void zgemm_f64_kernel(const ZGemm g) {
  constexpr int BM = 32 * WM, BN = 32 * WN, BK = 8;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  __shared__ double2 As[2][BK][BM];
  __shared__ double2 Bs[2][BK][BN];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tiles_m = (g.M + BM - 1) / BM;
  const int tiles_n = (g.N + BN - 1) / BN;
  const int64_t per_batch = (int64_t)tiles_m * tiles_n;
  const int64_t group = blockIdx.x / per_batch;  // = batch * ksplit + slice
  const int32_t tile = (int32_t)(blockIdx.x - group * per_batch);
  const int32_t batch = (int32_t)(group / g.ksplit);
  const int32_t slice = (int32_t)(group - (int64_t)batch * g.ksplit);
  const int tm = tile % tiles_m;
  const int tn = tile / tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  // K range of this slice (slices are multiples of BK)
  const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
  const int kbeg = slice * kchunk;
  const int kend = min(g.K, kbeg + kchunk);

  const double2* __restrict__ Ap = g.A.p + batch_off(g.A.b, batch);
  const double2* __restrict__ Bp = g.B.p + batch_off(g.B.b, batch);

  // ---- staging assignments (fixed rows of A / columns of B per thread)
  const bool a_kc = g.A.c.s_in == 1 && g.A.c.ext >= BK;  // K contiguous in A: threads along k
  const bool b_kc = !(g.B.c.s_in == 1 && g.B.c.ext >= 16) && g.B.r.s_in == 1;  // K contiguous in B
  int a_m[EA], a_k[EA];
  int64_t a_ro[EA];
  bool a_ok[EA];
#pragma unroll
  for (int e = 0; e < EA; ++e) {
    if (a_kc) {
      a_k[e] = tid & (BK - 1);
      a_m[e] = (tid >> 3) + 32 * e;
    } else {
      a_m[e] = tid % BM;
      a_k[e] = tid / BM + (256 / BM) * e;
    }
    const int gm = m0 + a_m[e];
    a_ok[e] = gm < g.M;
    a_ro[e] = a_ok[e] ? map_idx(g.A.r, gm) : 0;
  }
  int b_n[EB], b_k[EB];
  int64_t b_co[EB];
  bool b_ok[EB];
#pragma unroll
  for (int e = 0; e < EB; ++e) {
    if (b_kc) {
      b_k[e] = tid & (BK - 1);
      b_n[e] = (tid >> 3) + 32 * e;
    } else {
      b_n[e] = tid % BN;
      b_k[e] = tid / BN + (256 / BN) * e;
    }
    const int gn = n0 + b_n[e];
    b_ok[e] = gn < g.N;
    b_co[e] = b_ok[e] ? map_idx(g.B.c, gn) : 0;
  }
  const double asgn = g.A.conj ? -1.0 : 1.0;
  const double bsgn = g.B.conj ? -1.0 : 1.0;

  double2 ra[EA], rb[EB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int gk = k0 + a_k[e];
      double2 v = make_double2(0.0, 0.0);
      if (a_ok[e] && gk < kend) v = Ap[a_ro[e] + map_idx(g.A.c, gk)];
      v.y *= asgn;
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int gk = k0 + b_k[e];
      double2 v = make_double2(0.0, 0.0);
      if (b_ok[e] && gk < kend) v = Bp[map_idx(g.B.r, gk) + b_co[e]];
      v.y *= bsgn;
      rb[e] = v;
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) As[buf][a_k[e]][a_m[e]] = ra[e];
#pragma unroll
    for (int e = 0; e < EB; ++e) Bs[buf][b_k[e]][b_n[e]] = rb[e];
  };

  d4 acc_re[WM][WN], acc_im[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      acc_re[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      acc_im[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  const int wr = wave & 1, wc = wave >> 1;
  const int rowb = wr * 16 * WM, colb = wc * 16 * WN;
  const int nkt = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  load(kbeg);
  stage(0);
  __syncthreads();
  for (int it = 0; it < nkt; ++it) {
    const int buf = it & 1;
    if (it + 1 < nkt) load(kbeg + (it + 1) * BK);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int kr = 4 * s + (lane >> 4);
      double2 af[WM], bf[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) af[i] = As[buf][kr][rowb + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < WN; ++j) bf[j] = Bs[buf][kr][colb + 16 * j + (lane & 15)];
      // two passes over the blocks so that consecutive MFMAs never chain on one accumulator
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].x, bf[j].x, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].x, bf[j].y, acc_im[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-af[i].y, bf[j].y, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].y, bf[j].x, acc_im[i][j], 0, 0, 0);
        }
    }
    if (it + 1 < nkt) stage(buf ^ 1);
    __syncthreads();
  }

  // ---- epilogue: v_mfma_f64_16x16x4f64 leaves row (lane/16) + 4 r, column lane % 16 of each 16 x 16 block
  //      in element r of the lane's accumulator
  if (g.ksplit > 1) {
    double2* __restrict__ Pp = g.partial + ((int64_t)slice * g.batch + batch) * (int64_t)g.M * g.N;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + rowb + 16 * i + (lane >> 4) + 4 * r;
          const int gn = n0 + colb + 16 * j + (lane & 15);
          if (gm < g.M && gn < g.N) Pp[(int64_t)gm * g.N + gn] = make_double2(acc_re[i][j][r], acc_im[i][j][r]);
        }
    return;
  }
  double2* __restrict__ Cp = g.C + batch_off(g.cb, batch);
  const bool use_beta = g.beta.x != 0.0 || g.beta.y != 0.0;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + rowb + 16 * i + (lane >> 4) + 4 * r;
        const int gn = n0 + colb + 16 * j + (lane & 15);
        if (gm < g.M && gn < g.N) {
          const int64_t off = map_idx(g.cr, gm) + map_idx(g.cc, gn);
          const double vr = acc_re[i][j][r], vi = acc_im[i][j][r];
          double2 o;
          o.x = g.alpha.x * vr - g.alpha.y * vi;
          o.y = g.alpha.x * vi + g.alpha.y * vr;
          if (use_beta) {
            const double2 c = Cp[off];
            o.x += g.beta.x * c.x - g.beta.y * c.y;
            o.y += g.beta.x * c.y + g.beta.y * c.x;
          }
          Cp[off] = o;
        }
      }
}

// Second pass of split-K: C = alpha * sum_slices partial + beta * C, slices added in order.
__global__ __launch_bounds__(256) void zgemm_splitk_reduce(const ZGemm g) {
  const int64_t mn = (int64_t)g.M * g.N;
  const int64_t total = mn * g.batch;
  const bool use_beta = g.beta.x != 0.0 || g.beta.y != 0.0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = (int32_t)(x / mn);
    const int64_t e = x - (int64_t)b * mn;
    const int32_t gm = (int32_t)(e / g.N), gn = (int32_t)(e - (int64_t)(e / g.N) * g.N);
    double vr = 0.0, vi = 0.0;
    for (int sl = 0; sl < g.ksplit; ++sl) {
      const double2 v = g.partial[((int64_t)sl * g.batch + b) * mn + e];
      vr += v.x;
      vi += v.y;
    }
    double2* Cp = g.C + batch_off(g.cb, b);
    const int64_t off = map_idx(g.cr, gm) + map_idx(g.cc, gn);
    double2 o;
    o.x = g.alpha.x * vr - g.alpha.y * vi;
    o.y = g.alpha.x * vi + g.alpha.y * vr;
    if (use_beta) {
      const double2 c = Cp[off];
      o.x += g.beta.x * c.x - g.beta.y * c.y;
      o.y += g.beta.x * c.y + g.beta.y * c.x;
    }
    Cp[off] = o;
  }
}

}  // namespace

namespace {

struct Range {
  int64_t lo, hi;
};

// offsets x -> map(x) for x in [0, n): the box [lo, hi] that contains them
Range map_range(const IdxMap& m, int64_t n) {
  if (n <= 0) return {0, 0};
  if (m.ext == kFlat) {
    const int64_t e = (n - 1) * m.s_in;
    return {std::min<int64_t>(0, e), std::max<int64_t>(0, e)};
  }
  const int64_t nlo = std::min<int64_t>(m.ext, n) - 1;
  const int64_t nhi = (n - 1) / m.ext;
  const int64_t a = nlo * m.s_in, b = nhi * m.s_out;
  return {std::min<int64_t>(0, a) + std::min<int64_t>(0, b), std::max<int64_t>(0, a) + std::max<int64_t>(0, b)};
}

Range batch_range(const BatchMap& b, int64_t n, bool* ok) {
  *ok = true;
  if (n <= 0) return {0, 0};
  const int64_t ext = b.ext_lo == kFlat ? n : b.ext_lo;
  const int64_t nlo = std::min<int64_t>(ext, n);
  const int64_t nhi = (n - 1) / ext;
  int64_t lmin = 0, lmax = nlo - 1;
  if (b.tab) {
    if (!b.htab) {
      *ok = false;
      return {0, 0};
    }
    lmin = lmax = b.htab[0];
    for (int64_t i = 1; i < nlo; ++i) {
      lmin = std::min<int64_t>(lmin, b.htab[i]);
      lmax = std::max<int64_t>(lmax, b.htab[i]);
    }
  }
  const int64_t a1 = lmin * b.s_lo, a2 = lmax * b.s_lo, h = nhi * b.s_hi;
  return {std::min(a1, a2) + std::min<int64_t>(0, h), std::max(a1, a2) + std::max<int64_t>(0, h)};
}

bool check_operand(const char* name, const void* p, const Range& r1, const Range& r2, const Range& rb,
                   const Span& sp, char* why, int why_len) {
  if (!sp.base) {
    std::snprintf(why, why_len, "%s: no extent", name);
    return false;
  }
  const int64_t base = (static_cast<const char*>(p) - static_cast<const char*>(sp.base));
  if (base % 16) {
    std::snprintf(why, why_len, "%s: misaligned", name);
    return false;
  }
  const int64_t b0 = base / 16;
  const int64_t lo = b0 + r1.lo + r2.lo + rb.lo, hi = b0 + r1.hi + r2.hi + rb.hi;
  if (lo < 0 || hi >= sp.count) {
    std::snprintf(why, why_len, "%s: touches [%lld, %lld] of a %lld-element buffer", name, (long long)lo,
                  (long long)hi, (long long)sp.count);
    return false;
  }
  return true;
}

}  // namespace

bool dryrun() {
  const char* e = std::getenv("GREEN_DRYRUN");
  return e && e[0] == '1';
}

bool zgemm_in_bounds(const ZGemm& g, const Span& a, const Span& b, const Span& c, char* why, int why_len) {
  bool ok1 = true, ok2 = true, ok3 = true;
  const Range ba = batch_range(g.A.b, g.batch, &ok1), bb = batch_range(g.B.b, g.batch, &ok2),
              bc = batch_range(g.cb, g.batch, &ok3);
  if (!ok1 || !ok2 || !ok3) {
    std::snprintf(why, why_len, "batch table without host mirror");
    return false;
  }
  if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0) {
    std::snprintf(why, why_len, "empty or negative extent M=%d N=%d K=%d batch=%d", g.M, g.N, g.K, g.batch);
    return false;
  }
  if (g.ksplit < 1) {
    std::snprintf(why, why_len, "ksplit < 1");
    return false;
  }
  return check_operand("A", g.A.p, map_range(g.A.r, g.M), map_range(g.A.c, g.K), ba, a, why, why_len) &&
         check_operand("B", g.B.p, map_range(g.B.r, g.K), map_range(g.B.c, g.N), bb, b, why, why_len) &&
         check_operand("C", g.C, map_range(g.cr, g.M), map_range(g.cc, g.N), bc, c, why, why_len);
}

hipError_t zgemm(const ZGemm& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0) return hipErrorInvalidValue;
  if (dryrun()) return hipSuccess;
  if (g.ksplit < 1) return hipErrorInvalidValue;
  if (g.ksplit > 1 && !g.partial) return hipErrorInvalidValue;
  // tile shape: 32 x 32, 64 x 32, 32 x 64 or 64 x 64 (a dimension <= 32 gets a 32-wide tile)
  const int wm = g.M <= 32 ? 1 : 2, wn = g.N <= 32 ? 1 : 2;
  const int bm = 32 * wm, bn = 32 * wn;
  const int64_t tiles = (int64_t)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
  const dim3 grid((unsigned)(tiles * g.batch * g.ksplit)), block(256);
  const int shape = (wm - 1) * 2 + (wn - 1);
#define GREEN_SITE(S)                                                     \
  case Site::S:                                                          \
    switch (shape) {                                                     \
      case 0: zgemm_f64_kernel<1, 1, Site::S><<<grid, block, 0, s>>>(g); break; \
      case 1: zgemm_f64_kernel<1, 2, Site::S><<<grid, block, 0, s>>>(g); break; \
      case 2: zgemm_f64_kernel<2, 1, Site::S><<<grid, block, 0, s>>>(g); break; \
      default: zgemm_f64_kernel<2, 2, Site::S><<<grid, block, 0, s>>>(g); break; \
    }                                                                    \
    break;
  switch (g.site) {
    GREEN_SITE(P0_VG)
    GREEN_SITE(P0_VGrev)
    GREEN_SITE(P0_Contract)
    GREEN_SITE(Sig_PV)
    GREEN_SITE(Sig_XG)
    GREEN_SITE(Sig_YV)
    GREEN_SITE(HF)
    GREEN_SITE(Transform)
    default:
      GREEN_SITE(Generic)
  }
#undef GREEN_SITE
  if (g.ksplit > 1) {
    const int64_t total = (int64_t)g.M * g.N * g.batch;
    int64_t nb = (total + 255) / 256;
    if (nb > 65536) nb = 65536;
    zgemm_splitk_reduce<<<dim3((unsigned)nb), dim3(256), 0, s>>>(g);
  }
  return hipGetLastError();
}

}  // namespace green
