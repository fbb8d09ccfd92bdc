// Batched complex FP64 GEMM on CDNA matrix cores (v_mfma_f64_16x16x4f64), 3M form.
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
// conjugation applied when staging), and each 4-deep sub-slab issues three
// real MFMAs per block (3M form):
//   t1 += A_re B_re,  t2 += A_im B_im,  t3 += (A_re + A_im)(B_re + B_im);
//   C_re = t1 - t2,   C_im = t3 - t1 - t2.
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

// Running position k -> (k % ext, k / ext) of one staged element; advanced by a fixed step without
// divisions (the step never exceeds... any extent: the while loop handles ext < step).
struct KPos {
  int32_t k, lo, hi;
  __device__ __forceinline__ void init(const IdxMap& m, int32_t k0) {
    k = k0;
    if (m.ext == kFlat) {
      lo = k0;
      hi = 0;
    } else {
      hi = k0 / m.ext;
      lo = k0 - hi * m.ext;
    }
  }
  __device__ __forceinline__ int64_t off(const IdxMap& m) const { return (int64_t)lo * m.s_in + (int64_t)hi * m.s_out; }
  __device__ __forceinline__ void step(const IdxMap& m, int32_t d) {
    k += d;
    lo += d;
    if (m.ext != kFlat)
      while (lo >= m.ext) {
        lo -= m.ext;
        ++hi;
      }
  }
};

template <int WM, int WN>
__device__ __forceinline__ void f64_body(const ZGemm& g, int64_t bid) {
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
  const int64_t group = bid / per_batch;  // = batch * ksplit + slice
  const int32_t tile = (int32_t)(bid - group * per_batch);
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
  KPos apos[EA], bpos[EB];
#pragma unroll
  for (int e = 0; e < EA; ++e) apos[e].init(g.A.c, kbeg + a_k[e]);
#pragma unroll
  for (int e = 0; e < EB; ++e) bpos[e].init(g.B.r, kbeg + b_k[e]);
  // loads the next stage and advances the positions by BK
  auto load = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      double2 v = make_double2(0.0, 0.0);
      if (a_ok[e] && apos[e].k < kend) v = Ap[a_ro[e] + apos[e].off(g.A.c)];
      v.y *= asgn;
      ra[e] = v;
      apos[e].step(g.A.c, BK);
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      double2 v = make_double2(0.0, 0.0);
      if (b_ok[e] && bpos[e].k < kend) v = Bp[bpos[e].off(g.B.r) + b_co[e]];
      v.y *= bsgn;
      rb[e] = v;
      bpos[e].step(g.B.r, BK);
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) As[buf][a_k[e]][a_m[e]] = ra[e];
#pragma unroll
    for (int e = 0; e < EB; ++e) Bs[buf][b_k[e]][b_n[e]] = rb[e];
  };

  // 3M complex product (three real MFMA chains instead of four):
  //   t1 = sum a_re b_re,  t2 = sum a_im b_im,  t3 = sum (a_re + a_im)(b_re + b_im),
  //   C_re = t1 - t2,      C_im = t3 - t1 - t2.
  d4 t1[WM][WN], t2[WM][WN], t3[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      t1[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      t2[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      t3[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  const int wr = wave & 1, wc = wave >> 1;
  const int rowb = wr * 16 * WM, colb = wc * 16 * WN;
  const int nkt = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  load();
  stage(0);
  __syncthreads();
  for (int it = 0; it < nkt; ++it) {
    const int buf = it & 1;
    if (it + 1 < nkt) load();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int kr = 4 * s + (lane >> 4);
      double2 af[WM], bf[WN];
      double as[WM], bs[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        af[i] = As[buf][kr][rowb + 16 * i + (lane & 15)];
        as[i] = af[i].x + af[i].y;
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        bf[j] = Bs[buf][kr][colb + 16 * j + (lane & 15)];
        bs[j] = bf[j].x + bf[j].y;
      }
      // one pass per chain so that consecutive MFMAs never chain on one accumulator
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) t1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].x, bf[j].x, t1[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) t2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].y, bf[j].y, t2[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) t3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[i], bs[j], t3[i][j], 0, 0, 0);
    }
    if (it + 1 < nkt) stage(buf ^ 1);
    __syncthreads();
  }
  d4 acc_re[WM][WN], acc_im[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      acc_re[i][j] = t1[i][j] - t2[i][j];
      acc_im[i][j] = t3[i][j] - t1[i][j] - t2[i][j];
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
  int64_t coff[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int gn = n0 + colb + 16 * j + (lane & 15);
    coff[j] = gn < g.N ? map_idx(g.cc, gn) : 0;
  }
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + rowb + 16 * i + (lane >> 4) + 4 * r;
      if (gm >= g.M) continue;
      const int64_t roff = map_idx(g.cr, gm);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int gn = n0 + colb + 16 * j + (lane & 15);
        if (gn < g.N) {
          const int64_t off = roff + coff[j];
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
}

// ------------------------------------------------------------------------------------------------
// Mixed-precision variant: the same operands (complex FP64 in memory) are rounded while staging to
// LDS, either to FP32 (MODE 1, v_mfma_f32_16x16x4f32) or to a BF16 pair hi + lo with
// hi = bf16(x), lo = bf16(x - hi) (MODE 2, v_mfma_f32_16x16x32_bf16, products hi*hi + hi*lo + lo*hi).
// Complex numbers are laid out as (re, im) pairs along K, so one real MFMA chain gives
//   C_re = sum_k (re_a re_b - im_a im_b)   from A' = (re, -im) and B = (re, im),
//   C_im = sum_k (re_a im_b + im_a re_b)   from A  = (re,  im) and B' = (im, re).
// Accumulation is FP32 within a K slice (the split-K slices are combined in FP64).  For split BF16 the
// per-product rounding (about 2^-17 relative) is two orders above FP32 accumulation error.
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const __bf16 h = (__bf16)x;
  return (uint32_t)__builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float bf16_value(uint32_t b) {
  return __builtin_bit_cast(float, b << 16);
}
// (hi, lo) words of a complex value: low half = re, high half = im
__device__ __forceinline__ void split_pair(double re, double im, uint32_t& hi, uint32_t& lo) {
  const uint32_t hr = bf16_bits((float)re), hm = bf16_bits((float)im);
  const uint32_t lr = bf16_bits((float)(re - (double)bf16_value(hr)));
  const uint32_t lm = bf16_bits((float)(im - (double)bf16_value(hm)));
  hi = hr | (hm << 16);
  lo = lr | (lm << 16);
}
__device__ __forceinline__ u4 neg_im(u4 v) { return v ^ u4{0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u}; }
__device__ __forceinline__ u4 swap_re_im(u4 v) {
  return u4{(v.x >> 16) | (v.x << 16), (v.y >> 16) | (v.y << 16), (v.z >> 16) | (v.z << 16),
            (v.w >> 16) | (v.w << 16)};
}
__device__ __forceinline__ bf8 as_bf8(u4 v) { return __builtin_bit_cast(bf8, v); }
__device__ __forceinline__ int64_t elem_bytes_dev(int t) { return t == kC64 ? 16 : 8; }
__device__ __forceinline__ void split_pair_f(float re, float im, uint32_t& hi, uint32_t& lo) {
  const uint32_t hr = bf16_bits(re), hm = bf16_bits(im);
  hi = hr | (hm << 16);
  lo = bf16_bits(re - bf16_value(hr)) | (bf16_bits(im - bf16_value(hm)) << 16);
}
// a split-BF16 element of C (kCB16: 8 contiguous bytes; kCB16Q: its hi and lo words in its group of 4)
__device__ __forceinline__ void store_split(const ZGemm& g, int64_t off, uint2 w) {
  if (g.ctype == kCB16Q) {
    uint32_t* W = reinterpret_cast<uint32_t*>(g.C) + 2 * (off & ~(int64_t)3) + (off & 3);
    W[0] = w.x;
    W[4] = w.y;
  } else {
    reinterpret_cast<uint2*>(g.C)[off] = w;
  }
}
// C element store by the descriptor's ctype: v is the raw sum, alpha/beta applied here
__device__ __forceinline__ void store_c(const ZGemm& g, int64_t off, double2 v) {
  double2 o;
  o.x = g.alpha.x * v.x - g.alpha.y * v.y;
  o.y = g.alpha.x * v.y + g.alpha.y * v.x;
  const bool use_beta = g.beta.x != 0.0 || g.beta.y != 0.0;
  if (g.ctype == kC64) {
    double2* C = g.C + off;
    if (use_beta) {
      const double2 c = *C;
      o.x += g.beta.x * c.x - g.beta.y * c.y;
      o.y += g.beta.x * c.y + g.beta.y * c.x;
    }
    *C = o;
  } else if (g.ctype == kC32) {
    float2* C = reinterpret_cast<float2*>(g.C) + off;
    if (use_beta) {
      const float2 c = *C;
      o.x += g.beta.x * c.x - g.beta.y * c.y;
      o.y += g.beta.x * c.y + g.beta.y * c.x;
    }
    *C = make_float2((float)o.x, (float)o.y);
  } else {
    uint2 w;
    split_pair(o.x, o.y, w.x, w.y);
    store_split(g, off, w);
  }
}

// Store of an FP32 accumulator pair by the descriptor's ctype.  A split-BF16 output (beta == 0) is scaled and
// split in FP32 (the accumulator carries FP32 precision; hi + lo keeps 2^-17 of it); other outputs go through
// the FP64 path below.
__device__ __forceinline__ void store_cf(const ZGemm& g, int64_t off, float re, float im) {
  if (g.ctype == kCB16 || g.ctype == kCB16Q) {
    const float ar = (float)g.alpha.x, ai = (float)g.alpha.y;
    const float o_re = ar * re - ai * im, o_im = ar * im + ai * re;
    uint2 w;
    split_pair_f(o_re, o_im, w.x, w.y);
    store_split(g, off, w);
  } else {
    store_c(g, off, make_double2((double)re, (double)im));
  }
}
template <int MODE, int WM, int WN>
__device__ __forceinline__ void mx_body(const ZGemm& g, int64_t bid) {
  constexpr int BM = 32 * WM, BN = 32 * WN, BK = 16;  // BK complex K per stage
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  // LDS rows hold K contiguously, padded to spread banks
  constexpr int PW = MODE == 2 ? BK + 4 : 2 * BK + 4;  // row length in 32-bit words
  constexpr int APLANE = BM * PW, BPLANE = BN * PW;
  constexpr int NPL = MODE == 2 ? 2 : 1;  // planes per operand (hi, lo)
  __shared__ uint32_t As[2][NPL][APLANE];
  __shared__ uint32_t Bs[2][NPL][BPLANE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tiles_m = (g.M + BM - 1) / BM;
  const int tiles_n = (g.N + BN - 1) / BN;
  const int64_t per_batch = (int64_t)tiles_m * tiles_n;
  const int64_t group = bid / per_batch;
  const int32_t tile = (int32_t)(bid - group * per_batch);
  const int32_t batch = (int32_t)(group / g.ksplit);
  const int32_t slice = (int32_t)(group - (int64_t)batch * g.ksplit);
  const int tm = tile % tiles_m;
  const int tn = tile / tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
  const int kbeg = slice * kchunk;
  const int kend = min(g.K, kbeg + kchunk);

  const bool a_kc = g.A.c.s_in == 1 && g.A.c.ext >= BK;
  const bool b_kc = !(g.B.c.s_in == 1 && g.B.c.ext >= 16) && g.B.r.s_in == 1;
  int a_m[EA], a_k[EA];
  int64_t a_ro[EA];
  bool a_ok[EA];
#pragma unroll
  for (int e = 0; e < EA; ++e) {
    if (a_kc) {
      a_k[e] = tid & (BK - 1);
      a_m[e] = (tid >> 4) + 16 * e;
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
      b_n[e] = (tid >> 4) + 16 * e;
    } else {
      b_n[e] = tid % BN;
      b_k[e] = tid / BN + (256 / BN) * e;
    }
    const int gn = n0 + b_n[e];
    b_ok[e] = gn < g.N;
    b_co[e] = b_ok[e] ? map_idx(g.B.c, gn) : 0;
  }
  // raw element registers: a complex FP64 value, or the 8 bytes of a kC32 / kCB16 element in .x
  double2 ra[EA], rb[EB];
  const int ta = g.A.etype, tb = g.B.etype;
  auto fetch = [&](const char* base, int t, int64_t off) -> double2 {
    if (t == kC64) return reinterpret_cast<const double2*>(base)[off];
    const uint2 w = reinterpret_cast<const uint2*>(base)[off];
    return make_double2(__builtin_bit_cast(double, w), 0.0);
  };
  const char* Ab = reinterpret_cast<const char*>(g.A.p) + batch_off(g.A.b, batch) * elem_bytes_dev(ta);
  const char* Bb = reinterpret_cast<const char*>(g.B.p) + batch_off(g.B.b, batch) * elem_bytes_dev(tb);
  KPos apos[EA], bpos[EB];
#pragma unroll
  for (int e = 0; e < EA; ++e) apos[e].init(g.A.c, kbeg + a_k[e]);
#pragma unroll
  for (int e = 0; e < EB; ++e) bpos[e].init(g.B.r, kbeg + b_k[e]);
  auto load = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      ra[e] = (a_ok[e] && apos[e].k < kend) ? fetch(Ab, ta, a_ro[e] + apos[e].off(g.A.c)) : make_double2(0.0, 0.0);
      apos[e].step(g.A.c, BK);
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      rb[e] = (b_ok[e] && bpos[e].k < kend) ? fetch(Bb, tb, bpos[e].off(g.B.r) + b_co[e]) : make_double2(0.0, 0.0);
      bpos[e].step(g.B.r, BK);
    }
  };
  // raw element -> LDS words (conjugation applied here)
  auto put = [&](uint32_t* plane0, uint32_t* plane1, int idx, int t, double2 v, bool conj) {
    if (MODE == 2) {
      uint32_t hi, lo;
      if (t == kC64) {
        split_pair(v.x, conj ? -v.y : v.y, hi, lo);
      } else if (t == kC32) {
        const float2 f = __builtin_bit_cast(float2, v.x);
        split_pair_f(f.x, conj ? -f.y : f.y, hi, lo);
      } else {
        const uint2 w = __builtin_bit_cast(uint2, v.x);
        hi = conj ? (w.x ^ 0x80000000u) : w.x;
        lo = conj ? (w.y ^ 0x80000000u) : w.y;
      }
      plane0[idx] = hi;
      plane1[idx] = lo;
    } else {
      float re, im;
      if (t == kC64) {
        re = (float)v.x;
        im = (float)v.y;
      } else if (t == kC32) {
        const float2 f = __builtin_bit_cast(float2, v.x);
        re = f.x;
        im = f.y;
      } else {
        const uint2 w = __builtin_bit_cast(uint2, v.x);
        re = bf16_value(w.x & 0xffffu) + bf16_value(w.y & 0xffffu);
        im = bf16_value(w.x >> 16) + bf16_value(w.y >> 16);
      }
      plane0[2 * idx] = __builtin_bit_cast(uint32_t, re);
      plane0[2 * idx + 1] = __builtin_bit_cast(uint32_t, conj ? -im : im);
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = MODE == 2 ? a_m[e] * PW + a_k[e] : (a_m[e] * PW) / 2 + a_k[e];
      put(As[buf][0], As[buf][NPL - 1], idx, ta, ra[e], g.A.conj != 0);
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = MODE == 2 ? b_n[e] * PW + b_k[e] : (b_n[e] * PW) / 2 + b_k[e];
      put(Bs[buf][0], Bs[buf][NPL - 1], idx, tb, rb[e], g.B.conj != 0);
    }
  };

  f4 acc_re[WM][WN], acc_im[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      acc_re[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc_im[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }

  const int wr = wave & 1, wc = wave >> 1;
  const int rowb = wr * 16 * WM, colb = wc * 16 * WN;
  const int nkt = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  load();
  stage(0);
  __syncthreads();
  for (int it = 0; it < nkt; ++it) {
    const int buf = it & 1;
    if (it + 1 < nkt) load();
    if (MODE == 2) {
      const int koff = 4 * (lane >> 4);  // complex k offset of this lane's 8 bf16
      u4 ah[WM], al[WM], bh[WN], bl[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const int row = rowb + 16 * i + (lane & 15);
        ah[i] = *reinterpret_cast<const u4*>(&As[buf][0][row * PW + koff]);
        al[i] = *reinterpret_cast<const u4*>(&As[buf][1][row * PW + koff]);
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int col = colb + 16 * j + (lane & 15);
        bh[j] = *reinterpret_cast<const u4*>(&Bs[buf][0][col * PW + koff]);
        bl[j] = *reinterpret_cast<const u4*>(&Bs[buf][1][col * PW + koff]);
      }
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const bf8 anh = as_bf8(neg_im(ah[i])), anl = as_bf8(neg_im(al[i]));
        const bf8 aph = as_bf8(ah[i]), apl = as_bf8(al[i]);
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          const bf8 bph = as_bf8(bh[j]), bpl = as_bf8(bl[j]);
          const bf8 bsh = as_bf8(swap_re_im(bh[j])), bsl = as_bf8(swap_re_im(bl[j]));
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anh, bph, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aph, bsh, acc_im[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anh, bpl, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aph, bsl, acc_im[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anl, bph, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(apl, bsh, acc_im[i][j], 0, 0, 0);
        }
      }
    } else {
      const int kr = lane >> 4;  // real k within a 4-deep MFMA step
      const float sneg = (kr & 1) ? -1.0f : 1.0f;
#pragma unroll
      for (int st = 0; st < BK / 2; ++st) {
        const int w = 4 * st + kr;  // word index (re, im interleaved) of this lane's k
        float av[WM], an[WM], bv[WN], bw[WN];
#pragma unroll
        for (int i = 0; i < WM; ++i) {
          const int row = rowb + 16 * i + (lane & 15);
          av[i] = __builtin_bit_cast(float, As[buf][0][row * PW + w]);
          an[i] = sneg * av[i];
        }
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          const int col = colb + 16 * j + (lane & 15);
          bv[j] = __builtin_bit_cast(float, Bs[buf][0][col * PW + w]);
          bw[j] = __builtin_bit_cast(float, Bs[buf][0][col * PW + (w ^ 1)]);
        }
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) {
            acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(an[i], bv[j], acc_re[i][j], 0, 0, 0);
            acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bw[j], acc_im[i][j], 0, 0, 0);
          }
      }
    }
    if (it + 1 < nkt) stage(buf ^ 1);
    __syncthreads();
  }

  // epilogue: v_mfma_f32_16x16x4f32 / 16x16x32_bf16 leave row 4 (lane/16) + r, column lane % 16
  if (g.ksplit > 1) {
    double2* __restrict__ Pp = g.partial + ((int64_t)slice * g.batch + batch) * (int64_t)g.M * g.N;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + rowb + 16 * i + 4 * (lane >> 4) + r;
          const int gn = n0 + colb + 16 * j + (lane & 15);
          if (gm < g.M && gn < g.N)
            Pp[(int64_t)gm * g.N + gn] = make_double2((double)acc_re[i][j][r], (double)acc_im[i][j][r]);
        }
    return;
  }
  const int64_t cb = batch_off(g.cb, batch);
  int64_t coff[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int gn = n0 + colb + 16 * j + (lane & 15);
    coff[j] = gn < g.N ? map_idx(g.cc, gn) : 0;
  }
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + rowb + 16 * i + 4 * (lane >> 4) + r;
      if (gm >= g.M) continue;
      const int64_t roff = cb + map_idx(g.cr, gm);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int gn = n0 + colb + 16 * j + (lane & 15);
        if (gn < g.N) store_cf(g, roff + coff[j], acc_re[i][j][r], acc_im[i][j][r]);
      }
    }
}

// ------------------------------------------------------------------------------------------------
// Large-tile split-BF16 variant for the dominant contractions.  512 threads (8 waves, 4 along M x 2
// along N), each wave owning FM x FN blocks of 16 x 16, so a tile is (64 FM) x (32 FN).  Operands are
// stored pre-split (kCB16) and go to LDS unchanged, 32 complex K per stage (two MFMA K steps), double
// buffered (147 KB of LDS at 192 x 96).  The LDS rows are 128 bytes per plane with the 16-byte chunks
// XOR-swizzled by row, so the fragment reads of 16 rows at one K offset run without bank conflicts.  A is
// K-contiguous with a flat row map; B is K-contiguous with a flat column map, or N-contiguous with a flat
// K map.  Workgroups are renumbered so that each XCD (8 on MI355X, blocks dispatched round-robin)
// processes a contiguous range of tiles, whose operands then share its L2.
constexpr int kXcd = 8;

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t n) {
  const int64_t full = (n / kXcd) * kXcd;
  if (b >= full) return b;
  return (b % kXcd) * (n / kXcd) + b / kXcd;
}

// Offset of the K index of a staged element under a two-level map, advanced by a fixed step with no
// multiplications: the step and wrap increments are computed once per launch.
struct KCur {
  int32_t k, lo;
  int64_t off;
  __device__ __forceinline__ void init(const IdxMap& m, int32_t k0) {
    k = k0;
    if (m.ext == kFlat) {
      lo = k0;
      off = (int64_t)k0 * m.s_in;
    } else {
      const int32_t hi = k0 / m.ext;
      lo = k0 - hi * m.ext;
      off = (int64_t)lo * m.s_in + (int64_t)hi * m.s_out;
    }
  }
  __device__ __forceinline__ void step(const IdxMap& m, int32_t d, int64_t d_in, int64_t wrap) {
    k += d;
    lo += d;
    off += d_in;
    while (lo >= m.ext) {
      lo -= m.ext;
      off += wrap;
    }
  }
};

// K depth of a large tile: 32 complex when both double-buffered planes of the A and B tiles fit the
// 160 KB LDS at that depth, else 16.
constexpr int bt_bk(int FM, int FN) { return (64 * FM + 32 * FN) * 32 * 16 <= 160 * 1024 ? 32 : 16; }

// XOR pattern of the 16-byte chunks of row r for LDS rows of 64 or 128 bytes: with it the fragment reads (16
// rows at one chunk column per 16 lanes) run without bank conflicts on gfx950 (measured with
// SQ_LDS_BANK_CONFLICT; plain r & 7 or (r >> 1) & 7 leave 4 conflict cycles per read)
__device__ __forceinline__ int row_xor(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// word index of (row r, complex k) in a BK-word LDS plane row with swizzled 16-byte chunks
template <int BK>
__device__ __forceinline__ int bt_word(int r, int k) {
  if constexpr (BK == 32) return r * 32 + ((((k >> 2) ^ row_xor(r)) & 7) << 2) + (k & 3);
  else return r * 16 + ((((k >> 2) ^ row_xor(r)) & 3) << 2) + (k & 3);
}

// Output tile of a large-tile workgroup: XCD-aware renumbering, then (batch, K slice, tile); tiles in
// column order, or in bands of g.band tile rows each walked column by column.
struct LargeTile {
  int32_t batch, slice, m0, n0;
};
__device__ __forceinline__ LargeTile large_tile(const ZGemm& g, int64_t bid0, int64_t nblk, int BM, int BN) {
  const int tiles_m = (g.M + BM - 1) / BM;
  const int tiles_n = (g.N + BN - 1) / BN;
  const int64_t per_batch = (int64_t)tiles_m * tiles_n;
  const int64_t bid = xcd_block(bid0, nblk);
  const int64_t group = bid / per_batch;
  const int32_t tile = (int32_t)(bid - group * per_batch);
  LargeTile t;
  t.batch = (int32_t)(group / g.ksplit);
  t.slice = (int32_t)(group - (int64_t)t.batch * g.ksplit);
  int tm = tile % tiles_m;
  int tn = tile / tiles_m;
  if (g.band > 0 && g.band < tiles_m) {
    const int32_t per = g.band * tiles_n;
    const int32_t bi = tile / per, r = tile - bi * per;
    const int gb = min(g.band, tiles_m - bi * g.band);
    tn = r / gb;
    tm = bi * g.band + (r - tn * gb);
  }
  t.m0 = tm * BM;
  t.n0 = tn * BN;
  return t;
}

// Epilogue of a large tile: a wave's FM x FN fragments (16 x 16 each, rows from mw, columns from nw) to
// the split-K partial sums (FP64) or through the C maps.
template <int FM, int FN>
__device__ __forceinline__ void large_tile_store(const ZGemm& g, const f4 (&acc_re)[FM][FN], const f4 (&acc_im)[FM][FN],
                                                 int32_t batch, int32_t slice, int mw, int nw, int lane) {
  if (g.ksplit > 1) {
    double2* __restrict__ Pp = g.partial + ((int64_t)slice * g.batch + batch) * (int64_t)g.M * g.N;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = mw + 16 * i + 4 * (lane >> 4) + r;
        if (gm >= g.M) continue;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int gn = nw + 16 * j + (lane & 15);
          if (gn < g.N)
            Pp[(int64_t)gm * g.N + gn] = make_double2((double)acc_re[i][j][r], (double)acc_im[i][j][r]);
        }
      }
    return;
  }
  const int64_t cb = batch_off(g.cb, batch);
  int64_t coff[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int gn = nw + 16 * j + (lane & 15);
    coff[j] = gn < g.N ? map_idx(g.cc, gn) : 0;
  }
  // Split-BF16 output whose rows are contiguous (unit row stride, blocks of rows a multiple of 4, even
  // strides, 16-byte aligned): a lane's 4 consecutive rows of one column are 32 contiguous bytes, written as
  // two 16-byte stores
  const bool vec = g.ctype == kCB16 && g.cr.s_in == 1 && (g.cr.ext == kFlat || (g.cr.ext % 4 == 0 && g.cr.s_out % 2 == 0)) &&
                   g.cc.s_in % 2 == 0 && (g.cc.ext == kFlat || g.cc.s_out % 2 == 0) && cb % 2 == 0 &&
                   reinterpret_cast<uintptr_t>(g.C) % 16 == 0;
  const float ar = (float)g.alpha.x, ai = (float)g.alpha.y;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int gm0 = mw + 16 * i + 4 * (lane >> 4);
    if (vec && gm0 + 3 < g.M) {
      const int64_t roff = cb + map_idx(g.cr, gm0);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int gn = nw + 16 * j + (lane & 15);
        if (gn >= g.N) continue;
        uint32_t h[4], l[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float re = acc_re[i][j][r], im = acc_im[i][j][r];
          split_pair_f(ar * re - ai * im, ar * im + ai * re, h[r], l[r]);
        }
        u4* dst = reinterpret_cast<u4*>(reinterpret_cast<uint2*>(g.C) + roff + coff[j]);
        dst[0] = u4{h[0], l[0], h[1], l[1]};
        dst[1] = u4{h[2], l[2], h[3], l[3]};
      }
      continue;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = gm0 + r;
      if (gm >= g.M) continue;
      const int64_t roff = cb + map_idx(g.cr, gm);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int gn = nw + 16 * j + (lane & 15);
        if (gn < g.N) store_cf(g, roff + coff[j], acc_re[i][j][r], acc_im[i][j][r]);
      }
    }
  }
}

template <int FM, int FN, bool BNC>
__device__ __forceinline__ void bt_body(const ZGemm& g, int64_t bid0, int64_t nblk) {
  constexpr int BM = 64 * FM, BN = 32 * FN, BK = bt_bk(FM, FN);
  constexpr int EA = BM * BK / 512;
  constexpr int EB = BN * BK / 512;
  constexpr int RS = 512 / BK;  // rows staged per pass of the 512 threads
  static_assert(BK == 16 || BK == 32, "large-tile K depth");
  __shared__ uint32_t As[2][2][BM * BK];
  __shared__ uint32_t Bs[2][2][BN * BK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const LargeTile lt = large_tile(g, bid0, nblk, BM, BN);
  const int32_t batch = lt.batch, slice = lt.slice;
  const int m0 = lt.m0, n0 = lt.n0;
  const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
  const int kbeg = slice * kchunk;
  const int kend = min(g.K, kbeg + kchunk);

  const uint2* __restrict__ Ap = reinterpret_cast<const uint2*>(g.A.p) + batch_off(g.A.b, batch);
  const uint2* __restrict__ Bp = reinterpret_cast<const uint2*>(g.B.p) + batch_off(g.B.b, batch);
  constexpr bool b_kc = !BNC;  // BNC: B is N-contiguous, else K-contiguous
  // Rows (columns) beyond M (N) read row M-1 (column N-1) and lanes whose K index runs past the slice
  // read the slice's first K index: every load stays in bounds and carries no branch; such elements
  // are zeroed when staged.
  const int a_k = tid & (BK - 1);
  const int a_r0 = tid / BK;  // rows a_r0 + RS e
  // K-contiguous B: like A (BK consecutive K of 512 / BK columns per wave).  N-contiguous B: a wave stages
  // 16 consecutive columns at 4 consecutive K, so its LDS writes fall on distinct banks.
  int b_n[EB], b_k[EB];
#pragma unroll
  for (int e = 0; e < EB; ++e) {
    if constexpr (b_kc) {
      b_k[e] = tid & (BK - 1);
      b_n[e] = tid / BK + RS * e;
    } else {
      const int c = wave * EB + e;
      b_n[e] = 16 * (c % (BN / 16)) + (lane & 15);
      b_k[e] = 4 * (c / (BN / 16)) + (lane >> 4);
    }
  }
  // flat maps: A rows, B columns (K-contiguous B) or B K rows (N-contiguous B)
  const int64_t a_rs = g.A.r.s_in;
  const int64_t b_cs = g.B.c.s_in;
  int64_t b_col[BNC ? EB : 1];  // N-contiguous B: column offsets
#pragma unroll
  for (int e = 0; e < (BNC ? EB : 1); ++e) b_col[e] = BNC ? map_idx(g.B.c, min(n0 + b_n[e], g.N - 1)) : 0;
  const int64_t a_din = (int64_t)BK * g.A.c.s_in, a_wrap = g.A.c.s_out - (int64_t)g.A.c.ext * g.A.c.s_in;
  const int64_t b_din = (int64_t)BK * g.B.r.s_in, b_wrap = g.B.r.s_out - (int64_t)g.B.r.ext * g.B.r.s_in;
  KCur acur, bcur;
  acur.init(g.A.c, kbeg + a_k);
  // K-contiguous B: every element sits at this K; N-contiguous B: element e at this K + b_k[e] - (lane >> 4)
  bcur.init(g.B.r, kbeg + (b_kc ? b_k[0] : (lane >> 4)));
  const int64_t a_first = map_idx(g.A.c, kbeg), b_first = map_idx(g.B.r, kbeg);
  const uint32_t aflip = g.A.conj ? 0x80000000u : 0u, bflip = g.B.conj ? 0x80000000u : 0u;
  const int nkt = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;

  uint2 ra[EA], rb[EB];
  uint32_t okm = 0;  // bit 0: A elements inside the K range; bit 1 + e: B element e
  auto load = [&]() {
    const bool ak = acur.k < kend;
    const int64_t ao = ak ? acur.off : a_first;
    uint32_t m = ak ? 1u : 0u;
#pragma unroll
    for (int e = 0; e < EA; ++e) ra[e] = Ap[(int64_t)min(m0 + a_r0 + RS * e, g.M - 1) * a_rs + ao];
    if constexpr (b_kc) {
      const bool bk = bcur.k < kend;
      const int64_t bo = bk ? bcur.off : b_first;
#pragma unroll
      for (int e = 0; e < EB; ++e) rb[e] = Bp[bo + (int64_t)min(n0 + b_n[e], g.N - 1) * b_cs];
      m |= bk ? (((1u << EB) - 1u) << 1) : 0u;
    } else {
      // N-contiguous B: K rows bcur.k + (b_k[e] - (lane >> 4)) under a flat K map
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        const int dk = b_k[e] - (lane >> 4);
        const bool bk = bcur.k + dk < kend;
        rb[e] = Bp[(bk ? bcur.off + (int64_t)dk * g.B.r.s_in : b_first) + b_col[e]];
        m |= bk ? (2u << e) : 0u;
      }
    }
    okm = m;
    acur.step(g.A.c, BK, a_din, a_wrap);
    bcur.step(g.B.r, BK, b_din, b_wrap);
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const bool keep = (m0 + a_r0 + RS * e < g.M) && (okm & 1u);
      const int w = bt_word<BK>(a_r0 + RS * e, a_k);
      As[buf][0][w] = keep ? (ra[e].x ^ aflip) : 0u;
      As[buf][1][w] = keep ? (ra[e].y ^ aflip) : 0u;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const bool keep = (n0 + b_n[e] < g.N) && (okm & (2u << e));
      const int w = bt_word<BK>(b_n[e], b_k[e]);
      Bs[buf][0][w] = keep ? (rb[e].x ^ bflip) : 0u;
      Bs[buf][1][w] = keep ? (rb[e].y ^ bflip) : 0u;
    }
  };

  f4 acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc_re[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc_im[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  const int wm = wave & 3, wn = wave >> 2;
  const int rowb = wm * 16 * FM, colb = wn * 16 * FN;
  auto compute = [&](int buf, int sub) {
    {
      const int kq = 16 * sub + 4 * (lane >> 4);  // first complex K of this lane's 8 bf16
      u4 bh[FN], bl[FN];
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int w = bt_word<BK>(colb + 16 * j + (lane & 15), kq);
        bh[j] = *reinterpret_cast<const u4*>(&Bs[buf][0][w]);
        bl[j] = *reinterpret_cast<const u4*>(&Bs[buf][1][w]);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int w = bt_word<BK>(rowb + 16 * i + (lane & 15), kq);
        const u4 ah = *reinterpret_cast<const u4*>(&As[buf][0][w]);
        const u4 al = *reinterpret_cast<const u4*>(&As[buf][1][w]);
        const bf8 anh = as_bf8(neg_im(ah)), anl = as_bf8(neg_im(al));
        const bf8 aph = as_bf8(ah), apl = as_bf8(al);
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const bf8 bph = as_bf8(bh[j]), bpl = as_bf8(bl[j]);
          const bf8 bsh = as_bf8(swap_re_im(bh[j])), bsl = as_bf8(swap_re_im(bl[j]));
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anh, bph, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aph, bsh, acc_im[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anh, bpl, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aph, bsl, acc_im[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anl, bph, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(apl, bsh, acc_im[i][j], 0, 0, 0);
        }
      }
    }
  };

  // The next step's elements are staged into the other LDS buffer (last read before the previous
  // barrier) between the two MFMA K steps of the current one (BK = 32) or ahead of its one K step
  // (BK = 16), and the loads of the step after are issued right behind, so every load has a full
  // iteration to land.
  if (nkt > 0) {
    load();
    stage(0);
    __syncthreads();
    if (nkt > 1) load();
    for (int it = 0; it < nkt; ++it) {
      const int buf = it & 1;
      if constexpr (BK == 32) compute(buf, 0);
      if (it + 1 < nkt) stage(buf ^ 1);
      if (it + 2 < nkt) load();
      compute(buf, BK == 32 ? 1 : 0);
      __syncthreads();
    }
  }

  large_tile_store<FM, FN>(g, acc_re, acc_im, batch, slice, m0 + rowb, n0 + colb, lane);
}

// Split-BF16 large tiles fed by LDS DMA (K-contiguous A and B).  The tile (64 FM x 32 FN, 8 waves as
// 4 x 2, fragments as in the kernel above) advances 16 complex K per stage over a ring of three LDS
// stages: the global -> LDS copies of stage t + 2 are issued right after the barrier that opens stage
// t, so two stages of loads are always in flight and no register holds staged data.
//
// LDS rows hold the 16 complex K of one A row (B column) as 8 chunks of 16 bytes (2 complex, hi/lo
// interleaved as in memory); chunk c of row r sits at slot c ^ row_xor(r), which keeps the fragment
// reads free of bank conflicts.  One DMA instruction moves 1 KB: 8 rows of a
// stage, lane l writing slot l & 7 of row l >> 3 (so it reads the chunk that belongs there).  Rows
// (columns) beyond M (N) read row M-1 (column N-1); chunks past the slice's K end read the stage's
// first chunk and are zeroed in LDS once landed.  Requirements (checked on the host): K even, K maps
// flat or with an even extent of at least 16, even element strides, 16-byte aligned operands.
//
// Variant with stages of 32 complex K (BK = 32) and a two-slot ring (NS = 2): rows of 16 chunks (256 bytes,
// slot c ^ (r & 15)), four rows per DMA instruction, two MFMA K steps per barrier (half the barriers and
// waits per flop); the copies of stage t + 1 are issued after the barrier that opens stage t, so one stage of
// 32 K hides their latency.  K maps must be flat or of an extent of at least 32.

// wait until at most N vector-memory operations of this wave are outstanding (loads return in order)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
// workgroup barrier; memory operations are not moved across it, the counter waits are explicit
__device__ __forceinline__ void barrier_only() { asm volatile("s_barrier" ::: "memory"); }

__device__ __forceinline__ int bd_slot(int r, int c) { return c ^ row_xor(r); }

// One wave-wide 16-byte-per-lane copy global -> LDS (lane l lands at lds + 16 l bytes).  The LDS target is
// passed as a bare LDS address, so the compiler does not pair these copies with the fragment reads (it
// would otherwise wait for every copy in flight before each read); the waits are explicit.
__device__ __forceinline__ void dma16(const void* src, uint32_t* lds) {
  __builtin_amdgcn_global_load_lds(const_cast<void*>(src),
                                   (__attribute__((address_space(3))) void*)(uintptr_t)(uint32_t)(uintptr_t)lds, 16, 0,
                                   0);
}

template <int BK>
__device__ __forceinline__ int bd_slot_k(int r, int c) {
  if constexpr (BK == 16) return c ^ row_xor(r);
  else return c ^ (r & 15);
}

template <int FM, int FN, bool Q, int BK, int NS>
__device__ __forceinline__ void bd_body(const ZGemm& g, int64_t bid0, int64_t nblk) {
  constexpr int BM = 64 * FM, BN = 32 * FN;
  static_assert((BK == 16 && NS == 3) || (BK == 32 && NS == 2), "16-K stages in three slots or 32-K in two");
  constexpr int CPR = BK / 2;               // 16-byte chunks per LDS row
  constexpr int RPD = 64 / CPR;             // LDS rows per DMA instruction (1 KB)
  constexpr int W = 2 * BK;                 // 32-bit words per LDS row
  constexpr int DA = BM / RPD / 8, DB = BN / RPD / 8;  // DMA instructions per wave and stage
  static_assert(DB * RPD * 8 == BN && DA * RPD * 8 == BM, "tiles of whole DMA groups");
  constexpr int D = DA + DB;
  static_assert(NS * (BM + BN) * W * 4 <= 160 * 1024, "ring fits the LDS");
  __shared__ __attribute__((aligned(16))) uint32_t A0[BM * W], A1[BM * W], A2[NS == 3 ? BM * W : 4];
  __shared__ __attribute__((aligned(16))) uint32_t B0[BN * W], B1[BN * W], B2[NS == 3 ? BN * W : 4];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const LargeTile lt = large_tile(g, bid0, nblk, BM, BN);
  const int32_t batch = lt.batch, slice = lt.slice;
  const int m0 = lt.m0, n0 = lt.n0;
  const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
  const int kbeg = slice * kchunk;
  const int kend = min(g.K, kbeg + kchunk);
  const int nkt = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;

  const uint2* __restrict__ Ap = reinterpret_cast<const uint2*>(g.A.p) + batch_off(g.A.b, batch);
  const uint2* __restrict__ Bp = reinterpret_cast<const uint2*>(g.B.p) + batch_off(g.B.b, batch);
  // per lane and DMA instruction: row (column) offset and the chunk it carries
  // (32-K stages: twice the copies per stage, so the per-copy offsets are kept in 32 bits; the host allows those
  // tiles only where every element offset of an operand's batch slice fits)
  using off_t = typename std::conditional<BK == 32, int32_t, int64_t>::type;
  off_t a_ro[DA], b_co[DB];
  int a_c[DA], b_c[DB];
#pragma unroll
  for (int j = 0; j < DA; ++j) {
    const int r = RPD * (wave * DA + j) + lane / CPR;
    a_ro[j] = map_idx(g.A.r, min(m0 + r, g.M - 1));
    a_c[j] = bd_slot_k<BK>(r, lane % CPR);
  }
#pragma unroll
  for (int j = 0; j < DB; ++j) {
    const int r = RPD * (wave * DB + j) + lane / CPR;
    b_co[j] = map_idx(g.B.c, min(n0 + r, g.N - 1));
    b_c[j] = bd_slot_k<BK>(r, lane % CPR);
  }
  // stage K cursors (uniform): offset of the stage's first complex under each K map
  KCur acur, bcur;
  acur.init(g.A.c, kbeg);
  bcur.init(g.B.r, kbeg);
  const int64_t a_din = (int64_t)BK * g.A.c.s_in, a_wrap = g.A.c.s_out - (int64_t)g.A.c.ext * g.A.c.s_in;
  const int64_t b_din = (int64_t)BK * g.B.r.s_in, b_wrap = g.B.r.s_out - (int64_t)g.B.r.ext * g.B.r.s_in;
  // offset of 16-byte chunk c of the stage at the cursor (unit K stride): complex k0 + 2c (kCB16) or, for
  // kCB16Q, the hi (c even) or lo (c odd) words of the group at complex k0 + 4 (c / 2), which sit at the same
  // 8-byte element offset k0 + 2c; the stage's first chunk when that group lies past the slice's end
  auto chunk_off = [&](const KCur& cur, const IdxMap& m, int64_t wrap, int c) -> int64_t {
    const int dk = Q ? 4 * (c >> 1) : 2 * c;
    const int lo = cur.lo + dk;
    const int64_t off = cur.off + 2 * c + (lo >= m.ext ? wrap : 0);
    return cur.k + dk < kend ? off : cur.off;
  };
  // A stage whose 16 K all lie before the slice's end, under a K map that is flat or whose extent is a
  // multiple of 16 (stages start at multiples of 16, so they never straddle a wrap), needs no per-lane
  // checks: each lane adds its fixed chunk offset to the stage's uniform one.
  const bool a_whole = g.A.c.ext == kFlat || g.A.c.ext % BK == 0;
  const bool b_whole = g.B.r.ext == kFlat || g.B.r.ext % BK == 0;
  off_t a_lane[DA], b_lane[DB];
#pragma unroll
  for (int j = 0; j < DA; ++j) a_lane[j] = a_ro[j] + 2 * a_c[j];
#pragma unroll
  for (int j = 0; j < DB; ++j) b_lane[j] = b_co[j] + 2 * b_c[j];
  auto issue = [&](uint32_t* As, uint32_t* Bs) {
    if (a_whole && acur.k + BK <= kend) {
      const uint2* base = Ap + acur.off;
#pragma unroll
      for (int j = 0; j < DA; ++j) dma16(base + a_lane[j], As + (wave * DA + j) * 256);
    } else {
#pragma unroll
      for (int j = 0; j < DA; ++j)
        dma16(Ap + a_ro[j] + chunk_off(acur, g.A.c, a_wrap, a_c[j]), As + (wave * DA + j) * 256);
    }
    if (b_whole && bcur.k + BK <= kend) {
      const uint2* base = Bp + bcur.off;
#pragma unroll
      for (int j = 0; j < DB; ++j) dma16(base + b_lane[j], Bs + (wave * DB + j) * 256);
    } else {
#pragma unroll
      for (int j = 0; j < DB; ++j)
        dma16(Bp + b_co[j] + chunk_off(bcur, g.B.r, b_wrap, b_c[j]), Bs + (wave * DB + j) * 256);
    }
    acur.step(g.A.c, BK, a_din, a_wrap);
    bcur.step(g.B.r, BK, b_din, b_wrap);
  };

  f4 acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc_re[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc_im[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  const int wm = wave & 3, wn = wave >> 2;
  const int rowb = wm * 16 * FM, colb = wn * 16 * FN;
  const int g4 = lane >> 4, r16 = lane & 15;
  // hi and lo words of this lane's 4 complex K of MFMA step ks (chunks 8 ks + 2 g4 and + 1) of LDS row r
  auto frag = [&](const uint32_t* P, int r, int ks, u4& hi, u4& lo) {
    const u4 x = *reinterpret_cast<const u4*>(P + r * W + 4 * bd_slot_k<BK>(r, 8 * ks + 2 * g4));
    const u4 y = *reinterpret_cast<const u4*>(P + r * W + 4 * bd_slot_k<BK>(r, 8 * ks + 2 * g4 + 1));
    if constexpr (Q) {
      hi = x;
      lo = y;
    } else {
      hi = u4{x.x, x.z, y.x, y.z};
      lo = u4{x.y, x.w, y.y, y.w};
    }
  };
  auto compute = [&](const uint32_t* As, const uint32_t* Bs) {
#pragma unroll
    for (int ks = 0; ks < BK / 16; ++ks) {
    u4 bh[FN], bl[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) frag(Bs, colb + 16 * j + r16, ks, bh[j], bl[j]);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      u4 ah, al;
      frag(As, rowb + 16 * i + r16, ks, ah, al);
      const bf8 anh = as_bf8(neg_im(ah)), anl = as_bf8(neg_im(al));
      const bf8 aph = as_bf8(ah), apl = as_bf8(al);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const bf8 bph = as_bf8(bh[j]), bpl = as_bf8(bl[j]);
        const bf8 bsh = as_bf8(swap_re_im(bh[j])), bsl = as_bf8(swap_re_im(bl[j]));
        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anh, bph, acc_re[i][j], 0, 0, 0);
        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aph, bsh, acc_im[i][j], 0, 0, 0);
        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anh, bpl, acc_re[i][j], 0, 0, 0);
        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aph, bsl, acc_im[i][j], 0, 0, 0);
        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anl, bph, acc_re[i][j], 0, 0, 0);
        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(apl, bsh, acc_im[i][j], 0, 0, 0);
      }
    }
    // (two K steps per stage: the second step's reads are not hoisted over the first step's MFMAs, where
    // both steps' fragments together would not fit the registers)
    if constexpr (BK == 32) __builtin_amdgcn_sched_barrier(0);
    }
  };
  // chunks past the slice's K end in a landed stage -> 0 (every row of both tiles)
  const int kvalid_last = (kend - kbeg) - BK * (nkt - 1);  // complex K of the last stage, even
  auto zero_tail = [&](uint32_t* As, uint32_t* Bs) {
    for (int x = tid; x < (BM + BN) * CPR; x += 512) {
      const int r = x / CPR, c = x % CPR;
      if ((Q ? 4 * (c >> 1) : 2 * c) < kvalid_last) continue;
      uint32_t* P = r < BM ? As + r * W : Bs + (r - BM) * W;
      const int rr = r < BM ? r : r - BM;
      *reinterpret_cast<u4*>(P + 4 * bd_slot_k<BK>(rr, c)) = u4{0u, 0u, 0u, 0u};
    }
  };
  // one stage: own copies landed -> barrier (all copies landed, previous stage's buffer free) -> issue
  // stage t + 2 into that buffer -> MFMA
  // (NS = 2: own copies of stage t landed, nothing later in flight -> barrier -> issue stage t + 1 into the
  // slot stage t - 1 used -> MFMA)
  auto step = [&](uint32_t* As, uint32_t* Bs, uint32_t* An, uint32_t* Bn, int t) {
    if (NS == 3 && t + 1 < nkt) wait_vm<D>();
    else wait_vm<0>();
    if (t == nkt - 1 && kvalid_last < BK) {
      __syncthreads();
      zero_tail(As, Bs);
      __syncthreads();
    } else {
      barrier_only();
    }
    if (t + NS - 1 < nkt) issue(An, Bn);
    compute(As, Bs);
  };
  if (nkt > 0) {
    issue(A0, B0);
    if constexpr (NS == 3) {
      if (nkt > 1) issue(A1, B1);
      for (int it = 0; it < nkt; it += 3) {
        step(A0, B0, A2, B2, it);
        if (it + 1 < nkt) step(A1, B1, A0, B0, it + 1);
        if (it + 2 < nkt) step(A2, B2, A1, B1, it + 2);
      }
    } else {
      for (int it = 0; it < nkt; it += 2) {
        step(A0, B0, A1, B1, it);
        if (it + 1 < nkt) step(A1, B1, A0, B0, it + 1);
      }
    }
  }
  // every wave is done with the LDS stages before any wave of a persistent group starts another tile
  __syncthreads();
  large_tile_store<FM, FN>(g, acc_re, acc_im, batch, slice, m0 + rowb, n0 + colb, lane);
}

// LDS-DMA large tiles with the next stage's fragments prefetched: 512 threads (8 waves as WGM x 8/WGM over the
// tile, two per SIMD), each wave with FM x FN blocks of 16 x 16 and two sets of fragment registers.  DMA
// staging and LDS layout as in bd_body (a three-slot ring of 16 complex K); the fragments of stage t + 1 are
// read into the second register set right after the barrier that opens stage t, while the MFMAs of stage t
// run from the first, so the matrix cores do not wait for LDS after a barrier.  K maps must be flat or of an
// extent that is a multiple of 16 (no stage straddles a wrap).  The conjugated (re, -im) and swapped (im, re)
// forms that give the real and the imaginary part are made from the operand with fewer blocks per wave:
//   C_re = sum_k A (re, im) . B (re, -im),   C_im = sum_k A (re, im) . B (im, re)     (from B), or
//   C_re = sum_k A (re, -im) . B (re, im),   C_im = sum_k A (im, re) . B (re, im)     (from A).
__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt((0 << 8) | (7 << 4) | 15 | (3 << 14)); }

template <int FM, int FN, int WGM, int NS, int NW, bool Q>
__device__ __forceinline__ void bq_body(const ZGemm& g, int64_t bid0, int64_t nblk) {
  constexpr int WGN = NW / WGM;
  static_assert(WGM * WGN == NW && (NW == 4 || NW == 8), "four or eight waves");
  constexpr int NT = 64 * NW;
  constexpr int BM = 16 * FM * WGM, BN = 16 * FN * WGN, BK = 16;
  constexpr int DA = BM / (8 * NW), DB = BN / (8 * NW);  // DMA instructions per wave and stage (1 KB = 8 rows)
  static_assert(BM % (8 * NW) == 0 && BN % (8 * NW) == 0, "tile of whole DMA groups");
  constexpr int D = DA + DB;
  constexpr bool VB = FN <= FM;
  // one LDS array: slot s of A at word s SA, of B at NS SA + s SB (rows of 32 words: 16 complex, hi/lo)
  constexpr int SA = BM * 32, SB = BN * 32;
  static_assert(NS >= 3 && NS * (SA + SB) * 4 <= (NW == 4 ? 80 : 160) * 1024, "LDS ring");
  __shared__ __attribute__((aligned(16))) uint32_t lds[NS * (SA + SB)];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const LargeTile lt = large_tile(g, bid0, nblk, BM, BN);
  const int32_t batch = lt.batch, slice = lt.slice;
  const int m0 = lt.m0, n0 = lt.n0;
  const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
  const int kbeg = slice * kchunk;
  const int kend = min(g.K, kbeg + kchunk);
  const int nkt = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;

  const char* Ap = reinterpret_cast<const char*>(reinterpret_cast<const uint2*>(g.A.p) + batch_off(g.A.b, batch));
  const char* Bp = reinterpret_cast<const char*>(reinterpret_cast<const uint2*>(g.B.p) + batch_off(g.B.b, batch));
  // Copies: instruction j of this wave fills LDS row 8 (wave D + j) + (lane >> 3) of a slot, lane l writing slot
  // chunk (l & 7) there, i.e. memory chunk (l & 7) ^ row_xor(row) = c_even ^ ((wave D + j) & 1).  Element offsets
  // of a row (column) and of the K positions stay below 2^29 (checked on the host), so each lane carries 32-bit
  // byte offsets from a uniform base: a_lane[j] = (row offset + 2 chunk) * 8.
  const int c_even = (lane & 7) ^ (lane >> 3);
  uint32_t a_ro[DA], b_co[DB];
#pragma unroll
  for (int j = 0; j < DA; ++j)
    a_ro[j] = (uint32_t)map_idx(g.A.r, min(m0 + 8 * (wave * DA + j) + (lane >> 3), g.M - 1));
#pragma unroll
  for (int j = 0; j < DB; ++j)
    b_co[j] = (uint32_t)map_idx(g.B.c, min(n0 + 8 * (wave * DB + j) + (lane >> 3), g.N - 1));
  // K maps are flat or of an extent that is a multiple of 16 (checked on the host), so a stage never straddles
  // a wrap; only the slice's last stage can end early, and its chunks past the end copy the stage's first
  // chunk and are zeroed in LDS once landed
  KCur acur, bcur;
  acur.init(g.A.c, kbeg);
  bcur.init(g.B.r, kbeg);
  const int64_t a_din = (int64_t)BK * g.A.c.s_in, a_wrap = g.A.c.s_out - (int64_t)g.A.c.ext * g.A.c.s_in;
  const int64_t b_din = (int64_t)BK * g.B.r.s_in, b_wrap = g.B.r.s_out - (int64_t)g.B.r.ext * g.B.r.s_in;
  auto issue = [&](int slot) {
    uint32_t* As = lds + slot * SA;
    uint32_t* Bs = lds + NS * SA + slot * SB;
    // chunk part of this lane's element offset, for the two chunk parities
    uint32_t ca[2], cb[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int c = c_even ^ p;
      const int dk = Q ? 4 * (c >> 1) : 2 * c;
      ca[p] = acur.k + dk < kend ? 2u * c : 0u;
      cb[p] = bcur.k + dk < kend ? 2u * c : 0u;
    }
    const char* abase = Ap + acur.off * 8;
    const char* bbase = Bp + bcur.off * 8;
#pragma unroll
    for (int j = 0; j < DA; ++j) {
      uint32_t o = (a_ro[j] + ca[(wave * DA + j) & 1]) * 8u;
      asm volatile("" : "+v"(o));
      dma16(abase + o, As + (wave * DA + j) * 256);
    }
#pragma unroll
    for (int j = 0; j < DB; ++j) {
      uint32_t o = (b_co[j] + cb[(wave * DB + j) & 1]) * 8u;
      asm volatile("" : "+v"(o));
      dma16(bbase + o, Bs + (wave * DB + j) * 256);
    }
    acur.step(g.A.c, BK, a_din, a_wrap);
    bcur.step(g.B.r, BK, b_din, b_wrap);
  };
  const int kvalid_last = (kend - kbeg) - BK * (nkt - 1);  // complex K of the last stage, even
  // chunks past the slice's end in a landed stage -> 0 (every row of both tiles)
  auto zero_tail = [&](int slot) {
    uint32_t* As = lds + slot * SA;
    uint32_t* Bs = lds + NS * SA + slot * SB;
    for (int x = tid; x < (BM + BN) * 8; x += NT) {
      const int r = x >> 3, c = x & 7;
      if ((Q ? 4 * (c >> 1) : 2 * c) < kvalid_last) continue;
      uint32_t* P = r < BM ? As + r * 32 : Bs + (r - BM) * 32;
      const int rr = r < BM ? r : r - BM;
      *reinterpret_cast<u4*>(P + 4 * bd_slot(rr, c)) = u4{0u, 0u, 0u, 0u};
    }
  };

  f4 acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc_re[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc_im[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  const int wm = wave % WGM, wn = wave / WGM;
  const int rowb = wm * 16 * FM, colb = wn * 16 * FN;
  const int g4 = lane >> 4, r16 = lane & 15;
  // Fragment reads: row rowb + 16 i + r16 of a slot, chunks 2 g4 and 2 g4 + 1 under the swizzle c ^ row_xor(r),
  // and row_xor of those rows depends on r16 only, so one pair of lane offsets serves every block and slot
  // (the block and the slot are constant offsets)
  const int rx = row_xor(r16);
  const uint32_t fa0 = (uint32_t)((rowb + r16) * 32 + 4 * ((2 * g4) ^ rx));
  const uint32_t fa1 = (uint32_t)((rowb + r16) * 32 + 4 * ((2 * g4 + 1) ^ rx));
  const uint32_t fb0 = (uint32_t)((colb + r16) * 32 + 4 * ((2 * g4) ^ rx));
  const uint32_t fb1 = (uint32_t)((colb + r16) * 32 + 4 * ((2 * g4 + 1) ^ rx));
  struct Frags {
    u4 ah[FM], al[FM], bh[FN], bl[FN];
  };
  auto unpack = [&](u4 x, u4 y, u4& hi, u4& lo) {
    if constexpr (Q) {
      hi = x;
      lo = y;
    } else {
      hi = u4{x.x, x.z, y.x, y.z};
      lo = u4{x.y, x.w, y.y, y.w};
    }
  };
  auto read_frags = [&](int slot, Frags& f) {
    const uint32_t* As = lds + slot * SA;
    const uint32_t* Bs = lds + NS * SA + slot * SB;
#pragma unroll
    for (int j = 0; j < FN; ++j)
      unpack(*reinterpret_cast<const u4*>(Bs + fb0 + 512 * j), *reinterpret_cast<const u4*>(Bs + fb1 + 512 * j),
             f.bh[j], f.bl[j]);
#pragma unroll
    for (int i = 0; i < FM; ++i)
      unpack(*reinterpret_cast<const u4*>(As + fa0 + 512 * i), *reinterpret_cast<const u4*>(As + fa1 + 512 * i),
             f.ah[i], f.al[i]);
  };
  // the operand forms are made one block at a time, right before the MFMAs that use them
  auto compute = [&](const Frags& f) {
    if constexpr (VB) {
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const bf8 bch = as_bf8(neg_im(f.bh[j])), bcl = as_bf8(neg_im(f.bl[j]));
        const bf8 bsh = as_bf8(swap_re_im(f.bh[j])), bsl = as_bf8(swap_re_im(f.bl[j]));
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          const bf8 ah = as_bf8(f.ah[i]), al = as_bf8(f.al[i]);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bch, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bsh, acc_im[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bcl, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bsl, acc_im[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bch, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bsh, acc_im[i][j], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const bf8 ach = as_bf8(neg_im(f.ah[i])), acl = as_bf8(neg_im(f.al[i]));
        const bf8 ash = as_bf8(swap_re_im(f.ah[i])), asl = as_bf8(swap_re_im(f.al[i]));
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const bf8 bh = as_bf8(f.bh[j]), bl = as_bf8(f.bl[j]);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ach, bh, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ash, bh, acc_im[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ach, bl, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ash, bl, acc_im[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(acl, bh, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(asl, bh, acc_im[i][j], 0, 0, 0);
        }
      }
    }
  };
  // stage t (fragments in `cur`): own copies of stage t + 1 landed (those of up to NS - 2 later stages may be in
  // flight) and the fragment reads of stage t done -> barrier (every wave's copies of t + 1 landed, every wave
  // done reading the slot of stage t) -> stage t + NS copied into that slot -> fragments of t + 1 into `nxt` ->
  // MFMAs of stage t
  Frags f0, f1;
  auto wait_landed = [&](int later) {  // own copies outstanding beyond the stage waited for: `later` stages
    static_assert(NS <= 4, "ring depth");
    if constexpr (NS >= 4) {
      if (later >= 3) {
        wait_vm<3 * D>();
        return;
      }
    }
    if (later >= 2) wait_vm<2 * D>();
    else if (later >= 1) wait_vm<D>();
    else wait_vm<0>();
  };
  auto step = [&](int t, int rslot, int wslot, const Frags& cur, Frags& nxt) {
    if (t + 1 < nkt) {
      wait_landed(min(NS - 2, nkt - 2 - t));
      wait_lgkm0();
      barrier_only();
      if (t + NS < nkt) issue(wslot);
      if (t + 2 == nkt && kvalid_last < BK) {
        zero_tail(rslot);
        __syncthreads();
      }
      read_frags(rslot, nxt);
    } else {
      wait_lgkm0();
    }
    compute(cur);
  };
  if (nkt > 0) {
#pragma unroll
    for (int st = 0; st < NS; ++st)
      if (st < nkt) issue(st);
    wait_landed(min(NS - 1, nkt - 1));
    barrier_only();
    if (nkt == 1 && kvalid_last < BK) {
      zero_tail(0);
      __syncthreads();
    }
    read_frags(0, f0);
    // register sets alternate with the parity of t, slots rotate modulo NS (uniform); the loop body is always
    // two whole steps (one exit), an odd last step follows it
    int rs = 1, ws = 0, t = 0;
    for (; t + 2 <= nkt; t += 2) {
      step(t, rs, ws, f0, f1);
      rs = rs == NS - 1 ? 0 : rs + 1;
      ws = ws == NS - 1 ? 0 : ws + 1;
      step(t + 1, rs, ws, f1, f0);
      rs = rs == NS - 1 ? 0 : rs + 1;
      ws = ws == NS - 1 ? 0 : ws + 1;
    }
    if (t < nkt) step(t, rs, ws, f0, f1);
  }
  // every wave is done with the LDS stages before any wave of a persistent group starts another tile
  __syncthreads();
  large_tile_store<FM, FN>(g, acc_re, acc_im, batch, slice, m0 + rowb, n0 + colb, lane);
}

// Sigma~ stages 2 and 3 fused (split BF16).  For each (tt, k) of one tau chunk (one q, one spin):
//   S^T[j][i] = sum_{Q'} sum_b VT[k][Q'][j][b] Y^T[b][i],   Y^T[b][i] = sum_a GT[tt][k][b][a] X[tt][k][Q'][i][a]
// (Y = X G, S = Y V).  Y never leaves the registers: the 16 x 16 FP32 accumulator tile of Y^T that a lane
// holds (rows b = 4 (l >> 4) + r, column i = l & 15) is exactly its B operand of the second product (four
// consecutive K = b of column i), so it is split to BF16 hi + lo in place.  A workgroup owns (tt, k, slice of
// Q'); H waves share each 16-column block of i (wave w: columns 16 (w % NB) + ..., part h = w / NB of the
// b blocks), each summing over its own b blocks.  G^T and a ring of NS V^T blocks sit in LDS (rows padded
// to 16 NB); the V^T block (LDS DMA) and the X rows (registers) of Q' + NS - 1 are in flight while Q' is
// contracted (NS = 3, or 2 for the 80-row blocks, whose three slots would not fit 160 KB next to G^T).  Each
// (Q' slice, h) writes FP64 partial sums [slice H + h][k][j][tt][i] that the split-K pass adds in order.
//
// LDS rows of a block: K in groups of 4 complex, each group as a 16-byte unit of its 4 hi words then one of
// its 4 lo words (unit 2 g + 0 / 1), so that a fragment read is one 16-byte load per plane; unit u of row r
// sits at slot u ^ (r & 15) for rows of 256 or 512 bytes, u ^ row_xor(r) for rows of 128 bytes (the patterns
// that keep the fragment reads free of bank conflicts), and for rows of 640 bytes (NB = 5) at the XOR of its
// low three bits with (r >> 1) & 7, which stays inside the unit's aligned group of 8 and gives the 16 rows a
// fragment read touches 16 different bank offsets.  The map is its own inverse.
template <int NB>
__device__ __forceinline__ int xgv_swz(int r, int u) {
  constexpr int CH = 8 * NB;  // 16-byte units per row (16 NB complex)
  if constexpr (CH == 8) return u ^ row_xor(r);
  else if constexpr (CH % 16 == 0 && (CH & (CH - 1)) == 0) return u ^ (r & 15);
  else return (u & ~7) | ((u & 7) ^ ((r >> 1) & 7));
}
template <int NB>
__device__ __forceinline__ int xgv_word(int r, int u) {
  return (r * 8 * NB + xgv_swz<NB>(r, u)) * 4;
}
// complex 2 c, 2 c + 1 of row r (memory order: hi0, lo0, hi1, lo1) into their group's hi and lo units
template <int NB>
__device__ __forceinline__ void xgv_put(uint32_t* P, int r, int c, u4 v) {
  const int g = c >> 1, pos = 2 * (c & 1);
  *reinterpret_cast<uint2*>(&P[xgv_word<NB>(r, 2 * g) + pos]) = make_uint2(v.x, v.z);
  *reinterpret_cast<uint2*>(&P[xgv_word<NB>(r, 2 * g + 1) + pos]) = make_uint2(v.y, v.w);
}

template <int NB, int H, int NS>
__global__ __launch_bounds__(64 * NB * H) void sigma_xgv_kernel(const XgvArgs a) {
  constexpr int R = 16 * NB;       // padded rows and K of each block
  constexpr int NT = 64 * NB * H;  // threads
  constexpr int BH = NB / H;       // b blocks per wave
  static_assert(NB % H == 0, "b blocks split evenly");
  static_assert(NS == 2 || NS == 3, "V^T ring of two or three slots");
  constexpr int CH = 8 * NB;            // 16-byte units per LDS row
  constexpr int DV = 2 * NB / H;        // DMA instructions per wave and V^T block (R CH / 64 over NB H waves)
  constexpr int NX = 2 * NB;            // 16-byte X loads per lane and Q'
  static_assert((1 + NS) * R * R * 8 <= 160 * 1024, "G^T and the V^T ring fit the LDS");
  __shared__ __attribute__((aligned(16))) uint32_t Gs[R * R * 2];
  __shared__ __attribute__((aligned(16))) uint32_t Vs[NS][R * R * 2];

  const int tid = threadIdx.x, lane = tid & 63, w = (tid >> 6) % NB, h = (tid >> 6) / NB;
  const int g4 = lane >> 4, r16 = lane & 15;
  const int nao = a.nao, nch = nao / 2;  // nao even: a row of a block is nch 16-byte chunks
  const int vch = a.vs / 2;              // 16-byte chunks of a V^T row
  const int64_t nG = (int64_t)nao * nao, nVT = (int64_t)nao * a.vs;
  const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
  const int tt = (int)(bid % a.tcn);
  const int64_t rest = bid / a.tcn;
  const int sl = (int)(rest % a.qsplit);
  const int k = (int)(rest / a.qsplit);
  const int kk = a.kk[k];
  const int qc = (a.naux + a.qsplit - 1) / a.qsplit;
  const int q0 = min(a.naux, sl * qc), q1 = min(a.naux, q0 + qc);

  for (int x = tid; x < R * R / 2; x += NT) {
    reinterpret_cast<u4*>(Gs)[x] = u4{0u, 0u, 0u, 0u};
#pragma unroll
    for (int v = 0; v < NS; ++v) reinterpret_cast<u4*>(Vs[v])[x] = u4{0u, 0u, 0u, 0u};
  }
  __syncthreads();
  {
    const u4* src = reinterpret_cast<const u4*>(a.GT + tt * a.g_tt + (int64_t)kk * nG);
    for (int x = tid; x < nao * nch; x += NT) {
      const int r = x / nch, c = x - (x / nch) * nch;
      xgv_put<NB>(Gs, r, c, src[x]);
    }
  }
  // V^T block of one Q' (rows j, K = b; stored in memory in the LDS unit order: per group of 4 complex b, 16
  // bytes of hi words then 16 of lo words) copied by LDS DMA: instruction d of this wave fills the 64 LDS units
  // 64 (wave DV + d) + l (lane l), unit U being slot U % CH of row U / CH, i.e. the unit xgv_word places
  // there.  Units past the row (K padding, and the zero padding of the stored rows) and rows past nao read
  // unit 0 of row 0: finite values, multiplied by Y^T rows that are exactly 0 (b >= nao) or feeding outputs
  // that are not stored (j >= nao).
  // (80-row blocks: the blocks are stored as their LDS image, xgv_vimage, so copy d of a lane is the unit at
  // the same position in memory)
  const int64_t vblk = NB == 5 ? (int64_t)R * R : nVT;  // elements of one stored block
  const char* vbase = reinterpret_cast<const char*>(a.VT + (int64_t)kk * a.naux * vblk);
  int voff[NB == 5 ? 1 : DV];
  if constexpr (NB != 5) {
#pragma unroll
    for (int d = 0; d < DV; ++d) {
      const int U = 64 * ((tid >> 6) * DV + d) + lane;
      const int row = U / CH;
      const int u = xgv_swz<NB>(row, U - row * CH);
      voff[d] = row < nao && u < vch ? (row * a.vs + 2 * u) * 8 : 0;
    }
  }
  // (image copies: a wave-uniform base per copy plus one 32-bit lane offset, kept opaque so that the compiler
  // does not precompute a 64-bit address per copy)
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  uint32_t loff = lane * 16;
  asm volatile("" : "+v"(loff));
  auto vissue = [&](int qp, uint32_t* V) {
    const char* blk = vbase + (int64_t)qp * vblk * 8;
#pragma unroll
    for (int d = 0; d < DV; ++d) {
      if constexpr (NB == 5) dma16(blk + (int64_t)(wv * DV + d) * 1024 + loff, V + (wv * DV + d) * 256);
      else dma16(blk + voff[d], V + ((tid >> 6) * DV + d) * 256);
    }
  };
  // B operand of the first product: X^T (K = a, column i = 16 w + r16): complex a = 16 ab + 4 g4 .. + 3 of
  // row i, as two 16-byte chunks.  a >= nao reads a = 0 (finite; G^T is 0 there) and i >= nao reads row
  // nao - 1 (its results are not stored), so the loaded registers are used as they land.
  const int icl = min(16 * w + r16, nao - 1);
  // X of three consecutive Q' (NS = 3, loaded two Q' ahead) or one register set (NS = 2)
  u4 x0[NB][2], x1[NB][NS == 3 ? 2 : 1], x2[NB][NS == 3 ? 2 : 1];
  // (80-row blocks: a uniform block base and one opaque lane offset, the column clamped to nao - 2 per load, so
  // that no per-load address is kept across Q')
  uint32_t xlane = (uint32_t)icl * nao + 4 * g4;
  if constexpr (NB == 5) asm volatile("" : "+v"(xlane));
  auto xload = [&](int qp, u4 (&xv)[NB][2]) {
    if constexpr (NB == 5) {
      const uint2* blk = a.X + tt * a.x_tt + (int64_t)k * a.x_k + (int64_t)qp * nG;
#pragma unroll
      for (int ab = 0; ab < NB; ++ab)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t o = min(xlane + 16 * ab + 2 * h, (uint32_t)icl * nao + nao - 2);
          xv[ab][h] = *reinterpret_cast<const u4*>(blk + o);
        }
    } else {
      const uint2* row = a.X + tt * a.x_tt + (int64_t)k * a.x_k + (int64_t)qp * nG + (int64_t)icl * nao;
#pragma unroll
      for (int ab = 0; ab < NB; ++ab)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int a0 = 16 * ab + 4 * g4 + 2 * h;
          xv[ab][h] = *reinterpret_cast<const u4*>(row + (a0 < nao ? a0 : 0));
        }
    }
  };
  // A operand fragment: row r, K block kb (complex 16 kb + 4 g4 .. + 3) as hi and lo words
  // (80-row blocks: rows r = 16 b + r16 only, so the swizzle depends on r16 alone and a read is one of two lane
  // bases plus the constant (16 b CH + 8 kb) 4)
  const int sw5 = (r16 >> 1) & 7;
  const int wh5 = (r16 * CH + ((2 * g4) ^ sw5)) * 4, wl5 = (r16 * CH + ((2 * g4 + 1) ^ sw5)) * 4;
  auto frag = [&](const uint32_t* P, int r, int kb, u4& hi, u4& lo) {
    if constexpr (NB == 5) {
      const int c = ((r - r16) * CH + 8 * kb) * 4;
      hi = *reinterpret_cast<const u4*>(&P[wh5 + c]);
      lo = *reinterpret_cast<const u4*>(&P[wl5 + c]);
    } else {
      hi = *reinterpret_cast<const u4*>(&P[xgv_word<NB>(r, 8 * kb + 2 * g4)]);
      lo = *reinterpret_cast<const u4*>(&P[xgv_word<NB>(r, 8 * kb + 2 * g4 + 1)]);
    }
  };
  f4 s_re[NB], s_im[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    s_re[j] = f4{0.f, 0.f, 0.f, 0.f};
    s_im[j] = f4{0.f, 0.f, 0.f, 0.f};
  }
  // one Q': Y^T = G^T X^T, then S^T += V^T Y^T (B operands conjugated (re, -im) for the real part and swapped
  // (im, re) for the imaginary part, three split products each)
  // (NS = 2: xr is refilled with the X rows of Q' xnext once the first product has read it, so one register
  // set serves; the loads are in flight during the second product)
  auto contract = [&](const uint32_t* V, u4 (&xr)[NB][2], int xnext) {
    f4 y_re[BH], y_im[BH];
#pragma unroll
    for (int bb = 0; bb < BH; ++bb) {
      y_re[bb] = f4{0.f, 0.f, 0.f, 0.f};
      y_im[bb] = f4{0.f, 0.f, 0.f, 0.f};
    }
    // NB + BH steps (product 1 over the K blocks ab, product 2 over the b blocks bb), each on one group of
    // fragments from LDS; the next step's group is read before this step's MFMAs (double-buffered), so
    // LDS latency overlaps the matrix cores
    u4 fh[2][NB], fl[2][NB];
    auto read_group = [&](int st, u4 (&hh)[NB], u4 (&ll)[NB]) {
      if (st < NB) {
#pragma unroll
        for (int bb = 0; bb < BH; ++bb) frag(Gs, 16 * (h * BH + bb) + r16, st, hh[bb], ll[bb]);
      } else {
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) frag(V, 16 * jb + r16, h * BH + (st - NB), hh[jb], ll[jb]);
      }
    };
    read_group(0, fh[0], fl[0]);
#pragma unroll
    for (int st = 0; st < NB + BH; ++st) {
      if (st + 1 < NB + BH) read_group(st + 1, fh[(st + 1) & 1], fl[(st + 1) & 1]);
      const u4(&gh)[NB] = fh[st & 1];
      const u4(&gl)[NB] = fl[st & 1];
      if (st < NB) {
        const int ab = st;
        const u4 bh = u4{xr[ab][0].x, xr[ab][0].z, xr[ab][1].x, xr[ab][1].z};
        const u4 bl = u4{xr[ab][0].y, xr[ab][0].w, xr[ab][1].y, xr[ab][1].w};
        const bf8 bch = as_bf8(neg_im(bh)), bcl = as_bf8(neg_im(bl));
        const bf8 bsh = as_bf8(swap_re_im(bh)), bsl = as_bf8(swap_re_im(bl));
#pragma unroll
        for (int bb = 0; bb < BH; ++bb) {
          const bf8 xh = as_bf8(gh[bb]), xl = as_bf8(gl[bb]);
          y_re[bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, bch, y_re[bb], 0, 0, 0);
          y_im[bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, bsh, y_im[bb], 0, 0, 0);
          y_re[bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, bcl, y_re[bb], 0, 0, 0);
          y_im[bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, bsl, y_im[bb], 0, 0, 0);
          y_re[bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, bch, y_re[bb], 0, 0, 0);
          y_im[bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, bsh, y_im[bb], 0, 0, 0);
        }
        if constexpr (NS == 2) {
          if (st == NB - 1) xload(xnext, xr);
        }
      } else {
        const int bb = st - NB;
        uint32_t h0, h1, h2, h3, l0, l1, l2, l3;
        split_pair_f(y_re[bb][0], y_im[bb][0], h0, l0);
        split_pair_f(y_re[bb][1], y_im[bb][1], h1, l1);
        split_pair_f(y_re[bb][2], y_im[bb][2], h2, l2);
        split_pair_f(y_re[bb][3], y_im[bb][3], h3, l3);
        const u4 yh = u4{h0, h1, h2, h3}, yl = u4{l0, l1, l2, l3};
        const bf8 ych = as_bf8(neg_im(yh)), ycl = as_bf8(neg_im(yl));
        const bf8 ysh = as_bf8(swap_re_im(yh)), ysl = as_bf8(swap_re_im(yl));
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
          const bf8 vh = as_bf8(gh[jb]), vl = as_bf8(gl[jb]);
          s_re[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vh, ych, s_re[jb], 0, 0, 0);
          s_im[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vh, ysh, s_im[jb], 0, 0, 0);
          s_re[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vh, ycl, s_re[jb], 0, 0, 0);
          s_im[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vh, ysl, s_im[jb], 0, 0, 0);
          s_re[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vl, ych, s_re[jb], 0, 0, 0);
          s_im[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vl, ysh, s_im[jb], 0, 0, 0);
        }
      }
    }
  };
  // one Q' t: this wave's copies of V^T(t) and loads of X(t) landed (in flight behind them: those of t + 1
  // when NS = 3) -> barrier (every wave's copies landed; every wave done with step t - 1, whose LDS slot is
  // refilled next) -> V^T and X of t + NS - 1 issued -> contraction
  // With NS = 3 two groups are always in flight: past the slice's end the copies and loads repeat its last Q'
  // into a slot and registers nothing reads, so the counter waits are the same in every step.
  auto step = [&](int t, const uint32_t* V, uint32_t* V2, u4 (&xr)[NB][2], u4 (&xahead)[NB][2]) {
    if constexpr (NS == 3) {
      wait_vm<DV + NX>();
      barrier_only();
      vissue(min(t + 2, q1 - 1), V2);
      xload(min(t + 2, q1 - 1), xahead);
      contract(V, xr, -1);
    } else {
      wait_vm<0>();
      barrier_only();
      vissue(min(t + 1, q1 - 1), V2);
      contract(V, xr, min(t + 1, q1 - 1));
    }
  };
  if (q0 < q1) {
    vissue(q0, Vs[0]);
    xload(q0, x0);
    if constexpr (NS == 3) {
      vissue(min(q0 + 1, q1 - 1), Vs[1]);
      xload(min(q0 + 1, q1 - 1), x1);
      for (int qp = q0; qp < q1; qp += 3) {
        step(qp, Vs[0], Vs[2], x0, x2);
        if (qp + 1 >= q1) break;
        step(qp + 1, Vs[1], Vs[0], x1, x0);
        if (qp + 2 >= q1) break;
        step(qp + 2, Vs[2], Vs[1], x2, x1);
      }
    } else {
      for (int qp = q0; qp < q1; qp += 2) {
        step(qp, Vs[0], Vs[1], x0, x0);
        if (qp + 1 >= q1) break;
        step(qp + 1, Vs[1], Vs[0], x0, x0);
      }
    }
    wait_vm<0>();  // no copy into LDS outlives the workgroup
  }
  // S^T[j = 16 jb + 4 g4 + r][i = 16 w + r16] -> partial[((sl nk + k) nao + j) (tcn nao) + tt nao + i]
  const int i = 16 * w + r16;
  if (i < nao) {
    const int64_t ncol = (int64_t)a.tcn * nao;
    double2* P = a.partial + ((int64_t)(sl * H + h) * a.nk + k) * nao * ncol + (int64_t)tt * nao + i;
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = 16 * jb + 4 * g4 + r;
        if (j < nao) P[(int64_t)j * ncol] = make_double2((double)s_re[jb][r], (double)s_im[jb][r]);
      }
  }
}

// P~0 stage 1 in split BF16 without a tile loop: both V G products of a tau chunk,
//   P0_VG    T[tt][k][n][g]                 = sum_a V[vk(k)][n][a] G[t(tt)][gk(k)][a][g]        (n = (Q, d), g = b)
//   P0_VGrev T[tt][k][n / nao][g][n % nao]  = sum_c V[vk(k)][n][c] G[t(tt)][gk(k)][c][g]        (n = (Q', b), g = d)
// (the second stored transposed in its orbital pair).  A workgroup of W waves owns W RB 16 rows n of one k and a
// range of the chunk's tau nodes; each wave holds the split-BF16 fragments of its RB blocks of 16 rows (K = nao
// padded to 16 NB) in registers for the whole range, so V is read once per part of the chunk, and per tau node
// the G^T image of that node (16 NB rows g, K = a; zero past nao) is copied into one of two LDS buffers by LDS
// DMA while the other is contracted.  The work per node is NB x NB fragment groups (column block of 16 g, K block
// of 16 complex), each read once from LDS and applied to the RB row blocks with 6 MFMAs (three split products for
// each of C_re and C_im); the results are rounded to split BF16 and stored.  The bound is the HBM write of T
// (8 bytes per complex element against 8 nao complex MACs, all of it at the 16 NB padding of K and g).
// Products: P0_VG takes V as the A operand and the G^T image as B (B conjugated (re, -im) for the real part,
// swapped (im, re) for the imaginary part), P0_VGrev the image as A (with those variants) and V as B; either way
// the result tile has the row/column of the operand given as A.
// 16-row blocks of V per wave: 2 for P0_VG (all column blocks accumulated at once), 4 for P0_VGrev (3 with the
// 80-row images, whose V fragments take 5/4 of the registers); waves per workgroup: 4 (two workgroups per CU),
// 8 with the 80-row images (two 51 KB images per workgroup, one workgroup per CU)
constexpr int vg1_row_blocks(int nb, bool rev) { return rev ? (nb == 5 ? 3 : 4) : 2; }
constexpr int vg1_waves(int nb) { return nb == 5 ? 8 : 4; }

template <int NB, bool REV>
__global__ __launch_bounds__(64 * vg1_waves(NB), 8 / vg1_waves(NB)) void p0_vg1_kernel(const Vg1Args a) {
  constexpr int RB = vg1_row_blocks(NB, REV);  // 16-row blocks of V per wave
  constexpr int W = vg1_waves(NB);             // waves per workgroup
  constexpr int CH = 8 * NB;                   // 16-byte units per image row
  constexpr int UNITS = 16 * NB * CH;          // units per image
  constexpr int NCP = UNITS / 64;              // wave-wide 1 KB copies per image
  constexpr int CPW = (NCP + W - 1) / W;       // copies per wave (the last ones only where W does not divide NCP)
  static_assert(2 * UNITS * 16 * (8 / W) <= 160 * 1024, "the workgroups of a CU fit the LDS");
  __shared__ __attribute__((aligned(16))) uint32_t Gs[2][UNITS * 4];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g4 = lane >> 4, r16 = lane & 15;
  const int nao = a.nao, M = a.M;
  const int nrw = (M + 16 * RB * W - 1) / (16 * RB * W);
  const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
  const int rw = (int)(bid % nrw);
  const int64_t rest = bid / nrw;
  const int part = (int)(rest % a.tparts);
  const int k = (int)(rest / a.tparts);
  const int per = (a.tcn + a.tparts - 1) / a.tparts;
  const int tb = part * per, te = min(a.tcn, tb + per);
  if (tb >= te) return;  // uniform over the workgroup, before any barrier
  const int kv = a.vk ? a.vk[k] : k, kg = a.gk ? a.gk[k] : k;
  const int64_t nV = (int64_t)M * nao, nG = (int64_t)nao * nao;

  // image of chunk node tt: copy c (c = wv, wv + W, ...) moves units 64 c .. 64 c + 63, lane l the unit 64 c + l
  const char* img = reinterpret_cast<const char*>(a.img) + lane * 16;
  auto issue = [&](int tt, uint32_t* buf) {
    const char* src = img + ((int64_t)(a.t0 + a.tdir * tt) * a.nk + kg) * (UNITS * 16);
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int c = wv + W * j;
      if (NCP % W == 0 || c < NCP) dma16(src + c * 1024, buf + c * 256);
    }
  };
  issue(tb, Gs[0]);

  // this wave's rows n0 + 16 rb + r16 (rows past M read row M - 1; their results are not stored); complex
  // a = 16 s + 4 g4 .. + 3 of a row as two 16-byte loads (a >= nao reads a = 0: finite values facing image
  // zeros; nao even, so a pair never crosses the row end)
  const int n0 = (rw * W + wv) * 16 * RB;
  u4 vh[RB][NB], vl[RB][NB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int n = min(n0 + 16 * rb + r16, M - 1);
    const uint2* row = a.V + (int64_t)kv * nV + (int64_t)n * nao;
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      u4 x[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int a0 = 16 * s + 4 * g4 + 2 * h;
        x[h] = *reinterpret_cast<const u4*>(row + (a0 < nao ? a0 : 0));
      }
      vh[rb][s] = u4{x[0].x, x[0].z, x[1].x, x[1].z};
      vl[rb][s] = u4{x[0].y, x[0].w, x[1].y, x[1].w};
    }
  }
  wait_vm<0>();
  barrier_only();
  // byte offsets of this lane's results: P0_VG row n0 + 4 g4 (+ 16 rb + r), column r16 (+ 16 jt); P0_VGrev
  // column n = n0 + 16 rb + r16 at (n / nao) nao^2 + n % nao, row 4 g4 (+ 16 jt + r)
  uint32_t vofs0 = (uint32_t)(((int64_t)(n0 + 4 * g4) * nao + r16) * 8);
  uint32_t vofs[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int n = min(n0 + 16 * rb + r16, M - 1), qn = n / nao;
    vofs[rb] = (uint32_t)(((int64_t)qn * nG + (n - qn * nao) + 4 * g4 * nao) * 8);
    asm volatile("" : "+v"(vofs[rb]));
  }
  asm volatile("" : "+v"(vofs0));
  const int64_t rstep = (int64_t)nao * 8;  // bytes per row of nao elements
  // store bounds: P0_VG rows 16 rb + r < M - n0 - 4 g4, columns 16 jt < nao - r16; P0_VGrev columns
  // 16 rb < M - n0 - r16, rows 16 jt + r < nao - 4 g4
  const int rlim = REV ? M - n0 - r16 : M - n0 - 4 * g4;
  const int clim = REV ? nao - 4 * g4 : nao - r16;

  // image fragment of column block jt, K block s (rows 16 jt + r16, complex 16 s + 4 g4 .. + 3) as hi and lo
  // words; with the 80-row images the swizzle depends on r16 alone, so a read is one of two lane bases plus a
  // constant
  const int sw5 = (r16 >> 1) & 7;
  const int wh5 = (r16 * CH + ((2 * g4) ^ sw5)) * 4, wl5 = (r16 * CH + ((2 * g4 + 1) ^ sw5)) * 4;
  auto gfrag = [&](const uint32_t* G, int jt, int s, u4& hi, u4& lo) {
    if constexpr (NB == 5) {
      const int c = (16 * jt * CH + 8 * s) * 4;
      hi = *reinterpret_cast<const u4*>(&G[wh5 + c]);
      lo = *reinterpret_cast<const u4*>(&G[wl5 + c]);
    } else {
      const int r = 16 * jt + r16;
      hi = *reinterpret_cast<const u4*>(&G[xgv_word<NB>(r, 8 * s + 2 * g4)]);
      lo = *reinterpret_cast<const u4*>(&G[xgv_word<NB>(r, 8 * s + 2 * g4 + 1)]);
    }
  };

  for (int tt = tb; tt < te; ++tt) {
    const int cur = (tt - tb) & 1;
    // every wave's copies of this node's image landed (each wave waited for its own before its last stores of
    // the previous node) and every wave is done with the other buffer
    if (tt > tb) barrier_only();
    if (tt + 1 < te) issue(tt + 1, Gs[cur ^ 1]);
    const uint32_t* G = Gs[cur];
    char* out = reinterpret_cast<char*>(a.T + (int64_t)tt * a.nk * nV + (int64_t)k * nV);
    if constexpr (!REV) {
      // P0_VG: accumulators of every column block live (RB = 2), so that each row's results are stored by
      // consecutive instructions (a row of nao elements is complete when its lines leave the L2)
      f4 cre[RB][NB], cim[RB][NB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int jt = 0; jt < NB; ++jt) {
          cre[rb][jt] = f4{0.f, 0.f, 0.f, 0.f};
          cim[rb][jt] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
      for (int s = 0; s < NB; ++s)
#pragma unroll
        for (int jt = 0; jt < NB; ++jt) {
          u4 gh, gl;
          gfrag(G, jt, s, gh, gl);
          const bf8 gch = as_bf8(neg_im(gh)), gcl = as_bf8(neg_im(gl));
          const bf8 gsh = as_bf8(swap_re_im(gh)), gsl = as_bf8(swap_re_im(gl));
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            const bf8 xh = as_bf8(vh[rb][s]), xl = as_bf8(vl[rb][s]);
            f4& cr = cre[rb][jt];
            f4& ci = cim[rb][jt];
            cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, gch, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, gsh, ci, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, gcl, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, gsl, ci, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, gch, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, gsh, ci, 0, 0, 0);
          }
        }
      // result (n, g) = (n0 + 16 rb + 4 g4 + r, 16 jt + r16): row by row, the NB column blocks in turn.
      // Address: the output base plus a uniform offset that walks the rows plus a 32-bit lane offset; the bounds
      // are compared against lane limits kept opaque here, so that the compiler neither precomputes a scalar
      // address nor an exec mask per store.
      // (the copies of the next image were issued a whole node of MFMAs ago: waiting for them here, before the
      // stores, keeps the stores out of the wait)
      wait_vm<0>();
      int64_t o = 0;
      int lim = rlim, glim = clim;
      asm volatile("" : "+v"(lim), "+v"(glim));
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
          for (int jt = 0; jt < NB; ++jt) {
            uint32_t hi, lo;
            split_pair_f(cre[rb][jt][r], cim[rb][jt][r], hi, lo);
            if (16 * rb + r < lim && 16 * jt < glim)
              *reinterpret_cast<uint2*>(out + o + 16 * jt * 8 + vofs0) = make_uint2(hi, lo);
          }
          o += (r < 3 ? 1 : 13) * rstep;
          asm volatile("" : "+s"(o));
        }
    } else {
#pragma unroll
      for (int jt = 0; jt < NB; ++jt) {
        f4 cre[RB], cim[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          cre[rb] = f4{0.f, 0.f, 0.f, 0.f};
          cim[rb] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int s = 0; s < NB; ++s) {
          u4 gh, gl;
          gfrag(G, jt, s, gh, gl);
          const bf8 gch = as_bf8(neg_im(gh)), gcl = as_bf8(neg_im(gl));
          const bf8 gsh = as_bf8(swap_re_im(gh)), gsl = as_bf8(swap_re_im(gl));
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            const bf8 xh = as_bf8(vh[rb][s]), xl = as_bf8(vl[rb][s]);
            cre[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gch, xh, cre[rb], 0, 0, 0);
            cim[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gsh, xh, cim[rb], 0, 0, 0);
            cre[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gcl, xh, cre[rb], 0, 0, 0);
            cim[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gsl, xh, cim[rb], 0, 0, 0);
            cre[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gch, xl, cre[rb], 0, 0, 0);
            cim[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gsh, xl, cim[rb], 0, 0, 0);
          }
        }
        // result (g, n) = (16 jt + 4 g4 + r, n0 + 16 rb + r16) at (n / nao) nao^2 + g nao + n % nao: for each
        // row g the row blocks in turn (addressing and bounds as above)
        if (jt == NB - 1) wait_vm<0>();  // the next image landed (before the node's last stores, as above)
        int64_t o = (int64_t)16 * jt * rstep;
        int lim = rlim, glim = clim;
        asm volatile("" : "+v"(lim), "+v"(glim));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            uint32_t hi, lo;
            split_pair_f(cre[rb][r], cim[rb][r], hi, lo);
            if (16 * rb < lim && 16 * jt + r < glim) *reinterpret_cast<uint2*>(out + o + vofs[rb]) = make_uint2(hi, lo);
          }
          o += rstep;
          asm volatile("" : "+s"(o));
        }
      }
    }
  }
}

// Second pass of split-K: C = alpha * sum_slices partial + beta * C, slices added in order.
__device__ __forceinline__ void splitk_body(const ZGemm& g, int64_t x0, int64_t stride) {
  const int64_t mn = (int64_t)g.M * g.N;
  const int64_t total = mn * g.batch;
  for (int64_t x = x0; x < total; x += stride) {
    const int32_t b = (int32_t)(x / mn);
    const int64_t e = x - (int64_t)b * mn;
    const int32_t gm = (int32_t)(e / g.N), gn = (int32_t)(e - (int64_t)(e / g.N) * g.N);
    double vr = 0.0, vi = 0.0;
    for (int sl = 0; sl < g.ksplit; ++sl) {
      const double2 v = g.partial[((int64_t)sl * g.batch + b) * mn + e];
      vr += v.x;
      vi += v.y;
    }
    store_c(g, batch_off(g.cb, b) + map_idx(g.cr, gm) + map_idx(g.cc, gn), make_double2(vr, vi));
  }
}

__global__ __launch_bounds__(256) void zgemm_splitk_reduce(const ZGemm g) {
  splitk_body(g, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// ------------------------------------------------------------------------------------------------
// Kernels: one GEMM per launch (the call site is a template argument so that profilers attribute time
// per contraction), or a group of independent GEMMs of one variant in one persistent launch: a grid of
// workgroups walks the concatenated tile ranges of all descriptors.
template <int WM, int WN, Site SITE>
__global__ __launch_bounds__(256, 2) void zgemm_f64_kernel(const ZGemm g) {
  f64_body<WM, WN>(g, blockIdx.x);
}
template <int MODE, int WM, int WN, Site SITE>
__global__ __launch_bounds__(256) void zgemm_mx_kernel(const ZGemm g) {
  mx_body<MODE, WM, WN>(g, blockIdx.x);
}
template <int FM, int FN, bool BNC, Site SITE>
__global__ __launch_bounds__(512) void zgemm_bt_kernel(const ZGemm g) {
  bt_body<FM, FN, BNC>(g, blockIdx.x, gridDim.x);
}
template <int FM, int FN, bool Q, Site SITE>
__global__ __launch_bounds__(512) void zgemm_bd_kernel(const ZGemm g) {
  bd_body<FM, FN, Q, 16, 3>(g, blockIdx.x, gridDim.x);
}
// 32-K stages, two-slot ring
template <int FM, int FN, bool Q, Site SITE>
__global__ __launch_bounds__(512) void zgemm_bk_kernel(const ZGemm g) {
  bd_body<FM, FN, Q, 32, 2>(g, blockIdx.x, gridDim.x);
}
template <int FM, int FN, int WGM, int NS, int NW, bool Q, Site SITE>
__global__ __launch_bounds__(64 * NW, NW == 4 ? 2 : 1) void zgemm_bq_kernel(const ZGemm g) {
  bq_body<FM, FN, WGM, NS, NW, Q>(g, blockIdx.x, gridDim.x);
}

struct GroupArgs {
  const ZGemm* gs;       // device array of n descriptors
  const int64_t* start;  // device array of n + 1 tile offsets
  int32_t n;
  int64_t total;
};
template <class F>
__device__ __forceinline__ void group_loop(const GroupArgs& a, F&& body) {
  for (int64_t t = blockIdx.x; t < a.total; t += gridDim.x) {
    int d = 0;
    while (d + 1 < a.n && a.start[d + 1] <= t) ++d;
    // read the descriptor through the constant address space: its fields are invariant for the launch,
    // so they stay in scalar registers or the scalar cache across the body's barriers
    typedef const __attribute__((address_space(4))) ZGemm CZ;
    CZ* cg = (CZ*)(a.gs);
    body(*(const ZGemm*)(cg + d), t - a.start[d], a.start[d + 1] - a.start[d]);
  }
}
template <int WM, int WN>
__global__ __launch_bounds__(256, 2) void zgemm_f64_group(const GroupArgs a) {
  group_loop(a, [](const ZGemm& g, int64_t b, int64_t) { f64_body<WM, WN>(g, b); });
}
template <int MODE, int WM, int WN>
__global__ __launch_bounds__(256) void zgemm_mx_group(const GroupArgs a) {
  group_loop(a, [](const ZGemm& g, int64_t b, int64_t) { mx_body<MODE, WM, WN>(g, b); });
}
template <int FM, int FN, bool BNC>
__global__ __launch_bounds__(512) void zgemm_bt_group(const GroupArgs a) {
  group_loop(a, [](const ZGemm& g, int64_t b, int64_t n) { bt_body<FM, FN, BNC>(g, b, n); });
}
template <int FM, int FN, bool Q>
__global__ __launch_bounds__(512) void zgemm_bd_group(const GroupArgs a) {
  group_loop(a, [](const ZGemm& g, int64_t b, int64_t n) { bd_body<FM, FN, Q, 16, 3>(g, b, n); });
}
template <int FM, int FN, bool Q>
__global__ __launch_bounds__(512) void zgemm_bk_group(const GroupArgs a) {
  group_loop(a, [](const ZGemm& g, int64_t b, int64_t n) { bd_body<FM, FN, Q, 32, 2>(g, b, n); });
}
template <int FM, int FN, int WGM, int NS, int NW, bool Q>
__global__ __launch_bounds__(64 * NW, NW == 4 ? 2 : 1) void zgemm_bq_group(const GroupArgs a) {
  group_loop(a, [](const ZGemm& g, int64_t b, int64_t n) { bq_body<FM, FN, WGM, NS, NW, Q>(g, b, n); });
}
// split-K second pass of a group: descriptor blockIdx.y, elements strided over blockIdx.x
__global__ __launch_bounds__(256) void zgemm_splitk_reduce_group(const ZGemm* __restrict__ gs) {
  const ZGemm& g = gs[blockIdx.y];
  if (g.ksplit > 1) splitk_body(g, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// Transposing rounding: out[b][j][i] = round(in[b][i][j]).
__global__ void k_convert_c64_t(const double2* __restrict__ in, void* __restrict__ out, int32_t t, int n,
                                int64_t batch) {
  const int64_t nn = (int64_t)n * n, tot = nn * batch;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < tot; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = x / nn;
    const int e = (int)(x - b * nn);
    const int j = e / n, i = e - (e / n) * n;  // output element (j, i) <- input (i, j)
    const double2 v = in[b * nn + (int64_t)i * n + j];
    if (t == kC32) {
      reinterpret_cast<float2*>(out)[x] = make_float2((float)v.x, (float)v.y);
    } else {
      uint2 w;
      split_pair(v.x, v.y, w.x, w.y);
      reinterpret_cast<uint2*>(out)[x] = w;
    }
  }
}

// out[b][c][r] = rounded in[b][r][c] for rows x cols matrices: 32 x 32 tiles staged through LDS so that
// both the FP64 reads (along c) and the rounded writes (along r) are coalesced.  quad (kCB16, rows % 4 == 0):
// each output row stores its elements in groups of 4 as the 4 hi words, then the 4 lo words.
__global__ __launch_bounds__(256) void k_convert_c64_tr(const double2* __restrict__ in, void* __restrict__ out,
                                                        int32_t t, int rows, int cols, int quad, int rp) {
  __shared__ double2 tile[32][33];
  const int64_t b = blockIdx.z;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double2* src = in + b * rows * (int64_t)cols;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + ty + 8 * i, c = c0 + tx;
    if (r < rows && c < cols) tile[ty + 8 * i][tx] = src[(int64_t)r * cols + c];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = c0 + ty + 8 * i, r = r0 + tx;
    if (r >= rp || c >= cols) continue;
    const double2 v = r < rows ? tile[tx][ty + 8 * i] : make_double2(0.0, 0.0);
    const int64_t x = b * rp * (int64_t)cols + (int64_t)c * rp + r;
    if (t == kC32) {
      reinterpret_cast<float2*>(out)[x] = make_float2((float)v.x, (float)v.y);
    } else {
      uint2 w;
      split_pair(v.x, v.y, w.x, w.y);
      if (quad) {
        uint32_t* o = reinterpret_cast<uint32_t*>(out) + 2 * (x - r) + 8 * (r >> 2) + (r & 3);
        o[0] = w.x;
        o[4] = w.y;
      } else {
        reinterpret_cast<uint2*>(out)[x] = w;
      }
    }
  }
}

// LDS image of the transpose of n x n blocks (n = nao <= 16 NB), in the row layout of xgv_word<NB>: for block
// blk of `in` (element (b, j) at b nao + j), 16 NB rows j of 8 NB 16-byte units, unit u holding the hi (u even)
// or lo (u odd) words of the complex b = 4 (u / 2) .. + 3 of row j, stored at slot xgv_swz<NB>(j, u) of the row
// (the swizzle is its own inverse); zero past nao.  One thread per 16-byte unit.  NB = 5: the V^T blocks of the
// fused Sigma~ kernel (xgv_vimage); NB <= 4: the G^T images of the direct P~0 stage-1 kernel (vg1_image).
template <int NB>
__global__ __launch_bounds__(256) void k_tr_image(const double2* __restrict__ in, u4* __restrict__ out, int nao,
                                                  int64_t blocks) {
  constexpr int CH = 8 * NB, UNITS = 16 * NB * CH;
  const int64_t n = blocks * UNITS;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = x / UNITS;
    const int e = (int)(x - blk * UNITS), j = e / CH, sl = e - (e / CH) * CH;
    const int u = xgv_swz<NB>(j, sl);
    const int b0 = 4 * (u >> 1), plane = u & 1;
    const double2* src = in + blk * nao * (int64_t)nao;
    uint32_t w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int b = b0 + t;
      uint32_t hi = 0u, lo = 0u;
      if (j < nao && b < nao) {
        const double2 v = src[(int64_t)b * nao + j];
        split_pair(v.x, v.y, hi, lo);
      }
      w[t] = plane ? lo : hi;
    }
    out[x] = u4{w[0], w[1], w[2], w[3]};
  }
}

// Elementwise rounding of a complex FP64 array to kC32 or kCB16.
__global__ void k_convert_c64(const double2* __restrict__ in, void* __restrict__ out, int32_t t, int64_t n) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = in[x];
    if (t == kC32) {
      reinterpret_cast<float2*>(out)[x] = make_float2((float)v.x, (float)v.y);
    } else {
      uint2 w;
      split_pair(v.x, v.y, w.x, w.y);
      reinterpret_cast<uint2*>(out)[x] = w;
    }
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

bool check_operand(const char* name, const void* p, int32_t etype, const Range& r1, const Range& r2,
                   const Range& rb, const Span& sp, char* why, int why_len) {
  if (!sp.base) {
    std::snprintf(why, why_len, "%s: no extent", name);
    return false;
  }
  if (etype < kC64 || etype > kCB16Q) {
    std::snprintf(why, why_len, "%s: bad element type", name);
    return false;
  }
  const int64_t esz = elem_bytes(etype);
  const int64_t base = (static_cast<const char*>(p) - static_cast<const char*>(sp.base));
  if (base % esz) {
    std::snprintf(why, why_len, "%s: misaligned", name);
    return false;
  }
  // kCB16Q: the last element's whole group of 4 (groups counted from the pointer)
  const int64_t last = r1.hi + r2.hi + rb.hi;
  const int64_t lo = base + (r1.lo + r2.lo + rb.lo) * esz,
                hi = base + (etype == kCB16Q ? ((last | 3) + 1) * esz : last * esz + esz);
  if (lo < 0 || hi > sp.bytes) {
    std::snprintf(why, why_len, "%s: touches bytes [%lld, %lld) of a %lld-byte buffer", name, (long long)lo,
                  (long long)hi, (long long)sp.bytes);
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
  if (g.prec == 0 && (g.A.etype != kC64 || g.B.etype != kC64 || g.ctype != kC64)) {
    std::snprintf(why, why_len, "FP64 contraction with non-FP64 operands");
    return false;
  }
  if ((g.ctype == kCB16 || g.ctype == kCB16Q) && (g.beta.x != 0.0 || g.beta.y != 0.0)) {
    std::snprintf(why, why_len, "split-BF16 output cannot accumulate");
    return false;
  }
  return check_operand("A", g.A.p, g.A.etype, map_range(g.A.r, g.M), map_range(g.A.c, g.K), ba, a, why, why_len) &&
         check_operand("B", g.B.p, g.B.etype, map_range(g.B.r, g.K), map_range(g.B.c, g.N), bb, b, why, why_len) &&
         check_operand("C", g.C, g.ctype, map_range(g.cr, g.M), map_range(g.cc, g.N), bc, c, why, why_len);
}

// The large-tile kernel needs pre-split operands, a K-contiguous A, and B either K-contiguous or
// N-contiguous with the tile width dividing the 512 threads.
static bool big_ok(const ZGemm& g) {
  if (g.big < 1 || g.big > 4) return false;
  if (g.A.etype != kCB16 || g.B.etype != kCB16) return false;
  if (!(g.A.c.s_in == 1 && g.A.c.ext >= 16)) return false;
  const bool b_nc = g.B.c.s_in == 1 && g.B.c.ext >= 16;
  if (!b_nc && g.B.r.s_in != 1) return false;
  // row offsets of A, column offsets of a K-contiguous B and K offsets of an N-contiguous B are computed
  // as index * stride
  if (g.A.r.ext != kFlat) return false;
  if (!b_nc && g.B.c.ext != kFlat) return false;
  if (b_nc && g.B.r.ext != kFlat) return false;
  // the tall K-depth-16 tiles are built for a K-contiguous B only
  if (g.big >= 3 && b_nc) return false;
  return true;
}

// Large tiles (64 FM x 32 FN) by g.big: 1 = 192 x 96, 2 = 192 x 64, 3 = 320 x 64, 4 = 448 x 64.  The tall
// ones cover an M of 257..320 (448) in one tile row with at most 1/16 of it padding.
static void big_tile(int big, int* fm, int* fn) {
  static const int t[4][2] = {{3, 3}, {3, 2}, {5, 2}, {7, 2}};
  *fm = t[big - 1][0];
  *fn = t[big - 1][1];
}

// The LDS-DMA kernel: split-BF16 K-contiguous operands, even K, K maps flat or of even extent >= 16,
// even element strides and 16-byte aligned bases (every 2-complex chunk is one aligned 16-byte copy).
static bool even_map(const IdxMap& m) { return m.s_in % 2 == 0 && (m.ext == kFlat || m.s_out % 2 == 0); }
static bool even_batch(const BatchMap& b) { return b.s_lo % 2 == 0 && b.s_hi % 2 == 0; }
// kCB16Q operands (both or neither) need every row and every K block to start a group of 4: K, extents
// and strides multiples of 4.
static bool quad_map(const IdxMap& m) { return m.s_in % 4 == 0 && (m.ext == kFlat || m.s_out % 4 == 0); }
// largest |offset| an index map gives over [0, n)
static int64_t map_extent(const IdxMap& m, int64_t n) {
  if (n <= 0) return 0;
  if (m.ext == kFlat) return (n - 1) * std::abs(m.s_in);
  return (std::min<int64_t>(m.ext, n) - 1) * std::abs(m.s_in) + ((n - 1) / m.ext) * std::abs(m.s_out);
}
static bool dma_ok(const ZGemm& g) {
  if (g.big < 5 || g.big > 13) return false;
  // the prefetching kernel forms byte offsets from the operand's batch base in 32 bits: non-negative strides
  // and element offsets (row or column plus K) below 2^29
  if (g.big >= 7) {
    for (const IdxMap* m : {&g.A.r, &g.A.c, &g.B.r, &g.B.c})
      if (m->s_in < 0 || m->s_out < 0) return false;
    for (const IdxMap* m : {&g.A.c, &g.B.r})
      if (m->ext != kFlat && m->ext % 16 != 0) return false;
    const int64_t lim = (int64_t)1 << 29;
    if (map_extent(g.A.r, g.M) + map_extent(g.A.c, g.K) + 16 > lim) return false;
    if (map_extent(g.B.c, g.N) + map_extent(g.B.r, g.K) + 16 > lim) return false;
  }
  const bool q = g.A.etype == kCB16Q;
  if ((g.A.etype != kCB16 && !q) || g.B.etype != g.A.etype || g.A.conj || g.B.conj) return false;
  const int u = q ? 4 : 2;  // K granule of one 16-byte copy
  if (g.A.c.s_in != 1 || g.B.r.s_in != 1 || g.K % u != 0) return false;
  // (a K stage meets at most one wrap of a two-level K map: extents of at least the stage depth)
  const int kdepth = g.big >= 12 ? 32 : 16;
  for (const IdxMap* m : {&g.A.c, &g.B.r})
    if (m->ext != kFlat && (m->ext % u != 0 || m->ext < kdepth || m->s_out % u != 0)) return false;
  if (!even_map(g.A.r) || !even_map(g.B.c) || !even_batch(g.A.b) || !even_batch(g.B.b)) return false;
  if (q && (!quad_map(g.A.r) || !quad_map(g.B.c) || g.A.b.s_lo % 4 || g.A.b.s_hi % 4 || g.B.b.s_lo % 4 ||
            g.B.b.s_hi % 4))
    return false;
  return ((uintptr_t)g.A.p % 16 == 0) && ((uintptr_t)g.B.p % 16 == 0);
}

// LDS-DMA tiles by g.big (512 threads, 16 x 16 blocks per wave FM x FN): 5 = 320 x 64, 6 = 192 x 128; with the
// next stage's fragments prefetched: 7 = 320 x 64 (4 x 2 waves of 5 x 2 blocks, three-slot ring), 8 = 128 x 128
// (2 x 4 waves of 4 x 2 blocks, four-slot ring), 9 = 256 x 64 (4 x 2 waves of 4 x 2 blocks, four-slot ring);
// 256 threads, two workgroups per CU, three-slot ring: 10 = 128 x 64 (2 x 2 waves of 4 x 2 blocks), 11 = 64 x 128
// (1 x 4 waves of 4 x 2 blocks); stages of 32 complex K in a two-slot ring (512 threads, 4 x 2 waves): 12 = 128 x 128,
// 13 = 256 x 64.
static void dma_tile(int big, int* fm, int* fn) {
  static const int t[9][2] = {{5, 2}, {3, 4}, {5, 2}, {4, 2}, {4, 2}, {4, 2}, {4, 2}, {2, 4}, {4, 2}};
  *fm = t[big - 5][0];
  *fn = t[big - 5][1];
}

// Kernel variant of a descriptor: family (0: FP64, 1: FP32, 2: split BF16 64-wide tiles, 3: split BF16
// large tiles, 4: split BF16 large tiles fed by LDS DMA) and tile parameters.  g.shape (1..4) forces a 32/64-wide tile of the 256-thread kernels,
// 0 picks 32 along a dimension of at most 32, else 64.
Variant zgemm_variant(const ZGemm& g) {
  Variant v{};
  if (g.prec == 2 && dma_ok(g)) {
    v.family = g.big >= 12 ? 6 : g.big >= 7 ? 5 : 4;
    dma_tile(g.big, &v.p1, &v.p2);
    v.bnc = false;
    v.quad = g.A.etype == kCB16Q;
    if (v.family == 5) {
      const int nw = g.big >= 10 ? 4 : 8;
      const int wgm = g.big == 11 ? 1 : (g.big == 8 || g.big == 10) ? 2 : 4;
      v.threads = 64 * nw;
      v.bm = 16 * v.p1 * wgm;
      v.bn = 16 * v.p2 * (nw / wgm);
    } else {
      v.threads = 512;
      v.bm = 64 * v.p1;
      v.bn = 32 * v.p2;
    }
    return v;
  }
  if (g.A.etype == kCB16Q || g.B.etype == kCB16Q) {  // only the LDS-DMA kernel reads grouped operands
    v.family = -1;
    v.threads = 512;
    v.bm = v.bn = 64;
    return v;
  }
  // an LDS-DMA tile the operands do not allow falls back to a register-staged one: 320 x 64 to the same
  // tile, 192 x 128 and 128 x 128 to 192 x 96, the rest to 192 x 64
  ZGemm gb = g;
  if (gb.big >= 5)
    gb.big = (gb.big == 5 || gb.big == 7) ? 3 : (gb.big == 6 || gb.big == 8 || gb.big == 12) ? 1 : 2;
  if (g.prec == 2 && big_ok(gb)) {
    v.family = 3;
    big_tile(gb.big, &v.p1, &v.p2);
    v.bnc = g.B.c.s_in == 1 && g.B.c.ext >= 16;
    v.threads = 512;
    v.bm = 64 * v.p1;
    v.bn = 32 * v.p2;
    return v;
  }
  v.family = g.prec;  // 0, 1, 2
  if (g.shape >= 1 && g.shape <= 4) {
    v.p1 = (g.shape - 1) / 2 + 1;
    v.p2 = (g.shape - 1) % 2 + 1;
  } else {
    v.p1 = g.M <= 32 ? 1 : 2;
    v.p2 = g.N <= 32 ? 1 : 2;
  }
  v.bnc = false;
  v.threads = 256;
  v.bm = 32 * v.p1;
  v.bn = 32 * v.p2;
  return v;
}

bool same_variant(const Variant& a, const Variant& b) {
  return a.family == b.family && a.p1 == b.p1 && a.p2 == b.p2 && a.bnc == b.bnc && a.quad == b.quad &&
         a.threads == b.threads && a.bm == b.bm && a.bn == b.bn;
}

int zgemm_wgs_per_cu(const ZGemm& g) {
  const Variant v = zgemm_variant(g);
  if (v.family < 3) return 0;
  return v.family == 5 && v.threads == 256 ? 2 : 1;
}

void zgemm_tile(const ZGemm& g, int* bm, int* bn, int* threads) {
  const Variant v = zgemm_variant(g);
  *bm = v.bm;
  *bn = v.bn;
  *threads = v.threads;
}

int64_t zgemm_blocks(const ZGemm& g) {
  const Variant v = zgemm_variant(g);
  return (int64_t)((g.M + v.bm - 1) / v.bm) * ((g.N + v.bn - 1) / v.bn) * g.batch * g.ksplit;
}

namespace {

#define GREEN_SITES(X)     \
  switch (g.site) {        \
    case Site::P0_VG: X(P0_VG); break;             \
    case Site::P0_VGrev: X(P0_VGrev); break;       \
    case Site::P0_Contract: X(P0_Contract); break; \
    case Site::Sig_PV: X(Sig_PV); break;           \
    case Site::Sig_XG: X(Sig_XG); break;           \
    case Site::Sig_YV: X(Sig_YV); break;           \
    case Site::HF: X(HF); break;                   \
    case Site::Transform: X(Transform); break;     \
    case Site::GF2_VG: X(GF2_VG); break;           \
    case Site::GF2_Pair: X(GF2_Pair); break;       \
    case Site::GF2_Contract: X(GF2_Contract); break; \
    default: X(Generic); break;                    \
  }

template <int WM, int WN>
void launch_f64(const ZGemm& g, dim3 grid, hipStream_t s) {
#define X(S) zgemm_f64_kernel<WM, WN, Site::S><<<grid, dim3(256), 0, s>>>(g)
  GREEN_SITES(X)
#undef X
}
template <int MODE, int WM, int WN>
void launch_mx(const ZGemm& g, dim3 grid, hipStream_t s) {
#define X(S) zgemm_mx_kernel<MODE, WM, WN, Site::S><<<grid, dim3(256), 0, s>>>(g)
  GREEN_SITES(X)
#undef X
}
template <int FM, int FN, bool BNC>
void launch_bt(const ZGemm& g, dim3 grid, hipStream_t s) {
  switch (g.site) {
    case Site::P0_VG: zgemm_bt_kernel<FM, FN, BNC, Site::P0_VG><<<grid, dim3(512), 0, s>>>(g); break;
    case Site::P0_VGrev: zgemm_bt_kernel<FM, FN, BNC, Site::P0_VGrev><<<grid, dim3(512), 0, s>>>(g); break;
    case Site::P0_Contract: zgemm_bt_kernel<FM, FN, BNC, Site::P0_Contract><<<grid, dim3(512), 0, s>>>(g); break;
    case Site::Sig_PV: zgemm_bt_kernel<FM, FN, BNC, Site::Sig_PV><<<grid, dim3(512), 0, s>>>(g); break;
    case Site::GF2_Pair: zgemm_bt_kernel<FM, FN, BNC, Site::GF2_Pair><<<grid, dim3(512), 0, s>>>(g); break;
    default: zgemm_bt_kernel<FM, FN, BNC, Site::Generic><<<grid, dim3(512), 0, s>>>(g); break;
  }
}

template <int FM, int FN, int WGM, int NS, int NW, bool Q>
void launch_bq(const ZGemm& g, dim3 grid, hipStream_t s) {
  const dim3 b(64 * NW);
  switch (g.site) {
    case Site::P0_Contract: zgemm_bq_kernel<FM, FN, WGM, NS, NW, Q, Site::P0_Contract><<<grid, b, 0, s>>>(g); break;
    case Site::Sig_PV: zgemm_bq_kernel<FM, FN, WGM, NS, NW, Q, Site::Sig_PV><<<grid, b, 0, s>>>(g); break;
    default: zgemm_bq_kernel<FM, FN, WGM, NS, NW, Q, Site::Generic><<<grid, b, 0, s>>>(g); break;
  }
}

template <int FM, int FN, bool Q>
void launch_bd(const ZGemm& g, dim3 grid, hipStream_t s) {
  switch (g.site) {
    case Site::P0_Contract: zgemm_bd_kernel<FM, FN, Q, Site::P0_Contract><<<grid, dim3(512), 0, s>>>(g); break;
    case Site::Sig_PV: zgemm_bd_kernel<FM, FN, Q, Site::Sig_PV><<<grid, dim3(512), 0, s>>>(g); break;
    default: zgemm_bd_kernel<FM, FN, Q, Site::Generic><<<grid, dim3(512), 0, s>>>(g); break;
  }
}
template <int FM, int FN, bool Q>
void launch_bk(const ZGemm& g, dim3 grid, hipStream_t s) {
  switch (g.site) {
    case Site::P0_Contract: zgemm_bk_kernel<FM, FN, Q, Site::P0_Contract><<<grid, dim3(512), 0, s>>>(g); break;
    case Site::Sig_PV: zgemm_bk_kernel<FM, FN, Q, Site::Sig_PV><<<grid, dim3(512), 0, s>>>(g); break;
    default: zgemm_bk_kernel<FM, FN, Q, Site::Generic><<<grid, dim3(512), 0, s>>>(g); break;
  }
}

void launch_single(const Variant& v, const ZGemm& g, dim3 grid, hipStream_t s) {
  const int sh = (v.p1 - 1) * 2 + (v.p2 - 1);
  switch (v.family) {
    case 0:
      if (sh == 0) launch_f64<1, 1>(g, grid, s);
      else if (sh == 1) launch_f64<1, 2>(g, grid, s);
      else if (sh == 2) launch_f64<2, 1>(g, grid, s);
      else launch_f64<2, 2>(g, grid, s);
      break;
    case 1:
      if (sh == 0) launch_mx<1, 1, 1>(g, grid, s);
      else if (sh == 1) launch_mx<1, 1, 2>(g, grid, s);
      else if (sh == 2) launch_mx<1, 2, 1>(g, grid, s);
      else launch_mx<1, 2, 2>(g, grid, s);
      break;
    case 2:
      if (sh == 0) launch_mx<2, 1, 1>(g, grid, s);
      else if (sh == 1) launch_mx<2, 1, 2>(g, grid, s);
      else if (sh == 2) launch_mx<2, 2, 1>(g, grid, s);
      else launch_mx<2, 2, 2>(g, grid, s);
      break;
    case 4:
      if (v.p1 == 5) {
        if (v.quad) launch_bd<5, 2, true>(g, grid, s);
        else launch_bd<5, 2, false>(g, grid, s);
      } else {
        if (v.quad) launch_bd<3, 4, true>(g, grid, s);
        else launch_bd<3, 4, false>(g, grid, s);
      }
      break;
    case 6:
      if (v.p1 == 4) {
        if (v.quad) launch_bk<4, 2, true>(g, grid, s);
        else launch_bk<4, 2, false>(g, grid, s);
      } else {
        if (v.quad) launch_bk<2, 4, true>(g, grid, s);
        else launch_bk<2, 4, false>(g, grid, s);
      }
      break;
    case 5:
#define GREEN_BQ(...) (v.quad ? launch_bq<__VA_ARGS__, true>(g, grid, s) : launch_bq<__VA_ARGS__, false>(g, grid, s))
      switch (v.p1 * 100 + v.bm / 16 * 10 + v.threads / 64) {
        case 5 * 100 + 20 * 10 + 8: GREEN_BQ(5, 2, 4, 3, 8); break;   // 320 x 64
        case 4 * 100 + 16 * 10 + 8: GREEN_BQ(4, 2, 4, 4, 8); break;   // 256 x 64
        case 4 * 100 + 8 * 10 + 8: GREEN_BQ(4, 2, 2, 4, 8); break;    // 128 x 128
        case 4 * 100 + 8 * 10 + 4: GREEN_BQ(4, 2, 2, 3, 4); break;    // 128 x 64, two per CU
        default: GREEN_BQ(4, 2, 1, 3, 4); break;                      // 64 x 128, two per CU
      }
#undef GREEN_BQ
      break;
    default:
      if (v.p1 == 5) launch_bt<5, 2, false>(g, grid, s);
      else if (v.p1 == 7) launch_bt<7, 2, false>(g, grid, s);
      else if (v.p2 == 3) {
        if (v.bnc) launch_bt<3, 3, true>(g, grid, s);
        else launch_bt<3, 3, false>(g, grid, s);
      } else {
        if (v.bnc) launch_bt<3, 2, true>(g, grid, s);
        else launch_bt<3, 2, false>(g, grid, s);
      }
      break;
  }
}

void launch_group(const Variant& v, const GroupArgs& a, dim3 grid, hipStream_t s) {
  const int sh = (v.p1 - 1) * 2 + (v.p2 - 1);
  const dim3 b256(256), b512(512);
  switch (v.family) {
    case 0:
      if (sh == 0) zgemm_f64_group<1, 1><<<grid, b256, 0, s>>>(a);
      else if (sh == 1) zgemm_f64_group<1, 2><<<grid, b256, 0, s>>>(a);
      else if (sh == 2) zgemm_f64_group<2, 1><<<grid, b256, 0, s>>>(a);
      else zgemm_f64_group<2, 2><<<grid, b256, 0, s>>>(a);
      break;
    case 1:
      if (sh == 0) zgemm_mx_group<1, 1, 1><<<grid, b256, 0, s>>>(a);
      else if (sh == 1) zgemm_mx_group<1, 1, 2><<<grid, b256, 0, s>>>(a);
      else if (sh == 2) zgemm_mx_group<1, 2, 1><<<grid, b256, 0, s>>>(a);
      else zgemm_mx_group<1, 2, 2><<<grid, b256, 0, s>>>(a);
      break;
    case 2:
      if (sh == 0) zgemm_mx_group<2, 1, 1><<<grid, b256, 0, s>>>(a);
      else if (sh == 1) zgemm_mx_group<2, 1, 2><<<grid, b256, 0, s>>>(a);
      else if (sh == 2) zgemm_mx_group<2, 2, 1><<<grid, b256, 0, s>>>(a);
      else zgemm_mx_group<2, 2, 2><<<grid, b256, 0, s>>>(a);
      break;
    case 4:
      if (v.p1 == 5) {
        if (v.quad) zgemm_bd_group<5, 2, true><<<grid, b512, 0, s>>>(a);
        else zgemm_bd_group<5, 2, false><<<grid, b512, 0, s>>>(a);
      } else {
        if (v.quad) zgemm_bd_group<3, 4, true><<<grid, b512, 0, s>>>(a);
        else zgemm_bd_group<3, 4, false><<<grid, b512, 0, s>>>(a);
      }
      break;
    case 6:
      if (v.p1 == 4) {
        if (v.quad) zgemm_bk_group<4, 2, true><<<grid, b512, 0, s>>>(a);
        else zgemm_bk_group<4, 2, false><<<grid, b512, 0, s>>>(a);
      } else {
        if (v.quad) zgemm_bk_group<2, 4, true><<<grid, b512, 0, s>>>(a);
        else zgemm_bk_group<2, 4, false><<<grid, b512, 0, s>>>(a);
      }
      break;
    case 5:
#define GREEN_BQG(...) (v.quad ? zgemm_bq_group<__VA_ARGS__, true><<<grid, dim3(v.threads), 0, s>>>(a) \
                               : zgemm_bq_group<__VA_ARGS__, false><<<grid, dim3(v.threads), 0, s>>>(a))
      switch (v.p1 * 100 + v.bm / 16 * 10 + v.threads / 64) {
        case 5 * 100 + 20 * 10 + 8: GREEN_BQG(5, 2, 4, 3, 8); break;
        case 4 * 100 + 16 * 10 + 8: GREEN_BQG(4, 2, 4, 4, 8); break;
        case 4 * 100 + 8 * 10 + 8: GREEN_BQG(4, 2, 2, 4, 8); break;
        case 4 * 100 + 8 * 10 + 4: GREEN_BQG(4, 2, 2, 3, 4); break;
        default: GREEN_BQG(4, 2, 1, 3, 4); break;
      }
#undef GREEN_BQG
      break;
    default:
      if (v.p1 == 5) zgemm_bt_group<5, 2, false><<<grid, b512, 0, s>>>(a);
      else if (v.p1 == 7) zgemm_bt_group<7, 2, false><<<grid, b512, 0, s>>>(a);
      else if (v.p2 == 3) {
        if (v.bnc) zgemm_bt_group<3, 3, true><<<grid, b512, 0, s>>>(a);
        else zgemm_bt_group<3, 3, false><<<grid, b512, 0, s>>>(a);
      } else {
        if (v.bnc) zgemm_bt_group<3, 2, true><<<grid, b512, 0, s>>>(a);
        else zgemm_bt_group<3, 2, false><<<grid, b512, 0, s>>>(a);
      }
      break;
  }
}

bool launchable(const ZGemm& g) {
  if (g.ksplit < 1 || g.prec < 0 || g.prec > 2) return false;
  if (g.prec == 0 && (g.A.etype != kC64 || g.B.etype != kC64 || g.ctype != kC64)) return false;
  if (g.ksplit > 1 && !g.partial) return false;
  return zgemm_variant(g).family >= 0;
}

}  // namespace

hipError_t zgemm(const ZGemm& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0) return hipErrorInvalidValue;
  if (dryrun()) return hipSuccess;
  if (!launchable(g)) return hipErrorInvalidValue;
  const Variant v = zgemm_variant(g);
  launch_single(v, g, dim3((unsigned)zgemm_blocks(g)), s);
  if (g.ksplit > 1) {
    const int64_t total = (int64_t)g.M * g.N * g.batch;
    int64_t nb = (total + 255) / 256;
    if (nb > 65536) nb = 65536;
    zgemm_splitk_reduce<<<dim3((unsigned)nb), dim3(256), 0, s>>>(g);
  }
  return hipGetLastError();
}

hipError_t zgemm_group(const ZGemm* host, int n, const ZGemm* dev, const int64_t* dev_start, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (dryrun()) return hipSuccess;
  const Variant v = zgemm_variant(host[0]);
  int64_t total = 0, reduce_elems = 0;
  for (int i = 0; i < n; ++i) {
    const ZGemm& g = host[i];
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0 || g.K <= 0) return hipErrorInvalidValue;
    if (!launchable(g) || !same_variant(v, zgemm_variant(g))) return hipErrorInvalidValue;
    total += zgemm_blocks(g);
    if (g.ksplit > 1) reduce_elems = std::max<int64_t>(reduce_elems, (int64_t)g.M * g.N * g.batch);
  }
  GroupArgs a{dev, dev_start, n, total};
  // persistent grid: at most 8 workgroups per CU resident over 256 CUs
  const int64_t cap = (v.family >= 3 ? 1 : 4) * 256 * 8;
  launch_group(v, a, dim3((unsigned)std::min<int64_t>(total, cap)), s);
  if (reduce_elems > 0) {
    int64_t nb = (reduce_elems + 255) / 256;
    if (nb > 4096) nb = 4096;
    zgemm_splitk_reduce_group<<<dim3((unsigned)nb, (unsigned)n), dim3(256), 0, s>>>(dev);
  }
  return hipGetLastError();
}

hipError_t convert_c64_t(const double2* in, void* out, int32_t etype, int n, int64_t batch, hipStream_t s) {
  if (n <= 0 || batch <= 0) return hipSuccess;
  if (etype != kC32 && etype != kCB16) return hipErrorInvalidValue;
  if (dryrun()) return hipSuccess;
  const int64_t tot = (int64_t)n * n * batch;
  int64_t nb = (tot + 255) / 256;
  if (nb > 65536) nb = 65536;
  k_convert_c64_t<<<dim3((unsigned)nb), dim3(256), 0, s>>>(in, out, etype, n, batch);
  return hipGetLastError();
}

int xgv_halves(int nao) { return nao > 16 && nao <= 64 ? 2 : 1; }

hipError_t sigma_xgv(const XgvArgs& a, const ZGemm& reduce, hipStream_t s) {
  if (a.tcn <= 0 || a.nk <= 0 || a.naux <= 0) return hipSuccess;
  if (a.nao <= 0 || a.nao > kXgvMaxNao || a.nao % 2 != 0 || a.vs != xgv_vrow(a.nao) || a.qsplit < 1 ||
      reduce.ksplit != a.qsplit * xgv_halves(a.nao) || !a.partial)
    return hipErrorInvalidValue;
  if (dryrun()) return hipSuccess;
  const dim3 grid((unsigned)((int64_t)a.tcn * a.nk * a.qsplit));
  if (a.nao <= 16) sigma_xgv_kernel<1, 1, 3><<<grid, dim3(64), 0, s>>>(a);
  else if (a.nao <= 32) sigma_xgv_kernel<2, 2, 3><<<grid, dim3(256), 0, s>>>(a);
  else if (a.nao <= 64) sigma_xgv_kernel<4, 2, 3><<<grid, dim3(512), 0, s>>>(a);
  else sigma_xgv_kernel<5, 1, 2><<<grid, dim3(320), 0, s>>>(a);
  const int64_t total = (int64_t)reduce.M * reduce.N * reduce.batch;
  int64_t nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  zgemm_splitk_reduce<<<dim3((unsigned)nb), dim3(256), 0, s>>>(reduce);
  return hipGetLastError();
}

hipError_t convert_c64_tr(const double2* in, void* out, int32_t etype, int rows, int cols, int batch, hipStream_t s,
                          bool quad, int rows_out) {
  if (rows <= 0 || cols <= 0 || batch <= 0) return hipSuccess;
  const int rp = rows_out > rows ? rows_out : rows;
  if (etype != kC32 && etype != kCB16) return hipErrorInvalidValue;
  if (quad && (etype != kCB16 || rp % 4 != 0)) return hipErrorInvalidValue;
  if (batch > 65535 || (rp + 31) / 32 > 65535) return hipErrorInvalidValue;
  if (dryrun()) return hipSuccess;
  k_convert_c64_tr<<<dim3((unsigned)((cols + 31) / 32), (unsigned)((rp + 31) / 32), (unsigned)batch), dim3(256), 0,
                     s>>>(in, out, etype, rows, cols, quad ? 1 : 0, rp);
  return hipGetLastError();
}

hipError_t xgv_vimage(const double2* in, void* out, int nao, int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (nao <= 64 || nao > 80 || nao % 2 != 0) return hipErrorInvalidValue;
  if (dryrun()) return hipSuccess;
  int64_t nb = (blocks * 3200 + 255) / 256;
  if (nb > 65536) nb = 65536;
  k_tr_image<5><<<dim3((unsigned)nb), dim3(256), 0, s>>>(in, static_cast<u4*>(out), nao, blocks);
  return hipGetLastError();
}

int vg1_blocks(int nao) { return (nao + 15) / 16; }
bool vg1_ok(int nao) { return nao > 0 && nao % 2 == 0 && nao <= kVg1MaxNao; }
int64_t vg1_image_units(int nao) { return 128 * (int64_t)vg1_blocks(nao) * vg1_blocks(nao); }

hipError_t vg1_image(const double2* in, void* out, int nao, int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (!vg1_ok(nao)) return hipErrorInvalidValue;
  if (dryrun()) return hipSuccess;
  int64_t nb = (blocks * vg1_image_units(nao) + 255) / 256;
  if (nb > 65536) nb = 65536;
  u4* o = static_cast<u4*>(out);
  switch (vg1_blocks(nao)) {
    case 1: k_tr_image<1><<<dim3((unsigned)nb), dim3(256), 0, s>>>(in, o, nao, blocks); break;
    case 2: k_tr_image<2><<<dim3((unsigned)nb), dim3(256), 0, s>>>(in, o, nao, blocks); break;
    case 3: k_tr_image<3><<<dim3((unsigned)nb), dim3(256), 0, s>>>(in, o, nao, blocks); break;
    case 4: k_tr_image<4><<<dim3((unsigned)nb), dim3(256), 0, s>>>(in, o, nao, blocks); break;
    default: k_tr_image<5><<<dim3((unsigned)nb), dim3(256), 0, s>>>(in, o, nao, blocks); break;
  }
  return hipGetLastError();
}

hipError_t p0_vg1(const Vg1Args& a, bool rev, hipStream_t s) {
  if (a.tcn <= 0 || a.nk <= 0 || a.M <= 0) return hipSuccess;
  if (!vg1_ok(a.nao) || a.M % a.nao != 0 || (a.tdir != 1 && a.tdir != -1)) return hipErrorInvalidValue;
  // the kernel's 32-bit lane offsets address one k's M nao elements
  if ((int64_t)a.M * a.nao * 8 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (dryrun()) return hipSuccess;
  // workgroups: row groups x momenta x parts of the chunk, the chunk split until about 2048 workgroups (eight
  // per CU slot pair) or one node per part
  Vg1Args b = a;
  const int nb = vg1_blocks(a.nao);
  const int rows = 16 * vg1_row_blocks(nb, rev) * vg1_waves(nb);
  const int64_t nrw = (a.M + rows - 1) / rows;
  const int64_t target = 2048 * 4 / vg1_waves(nb);
  b.tparts = 1;
  while (b.tparts < a.tcn && nrw * a.nk * b.tparts < target) ++b.tparts;
  const dim3 grid((unsigned)(nrw * a.nk * b.tparts)), block(64 * vg1_waves(nb));
  switch (nb * 2 + (rev ? 1 : 0)) {
    case 2: p0_vg1_kernel<1, false><<<grid, block, 0, s>>>(b); break;
    case 3: p0_vg1_kernel<1, true><<<grid, block, 0, s>>>(b); break;
    case 4: p0_vg1_kernel<2, false><<<grid, block, 0, s>>>(b); break;
    case 5: p0_vg1_kernel<2, true><<<grid, block, 0, s>>>(b); break;
    case 6: p0_vg1_kernel<3, false><<<grid, block, 0, s>>>(b); break;
    case 7: p0_vg1_kernel<3, true><<<grid, block, 0, s>>>(b); break;
    case 8: p0_vg1_kernel<4, false><<<grid, block, 0, s>>>(b); break;
    case 9: p0_vg1_kernel<4, true><<<grid, block, 0, s>>>(b); break;
    case 10: p0_vg1_kernel<5, false><<<grid, block, 0, s>>>(b); break;
    default: p0_vg1_kernel<5, true><<<grid, block, 0, s>>>(b); break;
  }
  return hipGetLastError();
}

hipError_t convert_c64(const double2* in, void* out, int32_t etype, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (etype != kC32 && etype != kCB16) return hipErrorInvalidValue;
  if (dryrun()) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  k_convert_c64<<<dim3((unsigned)nb), dim3(256), 0, s>>>(in, out, etype, n);
  return hipGetLastError();
}

}  // namespace green
