// Small element-wise and reduction kernels of the GW iteration.
//
// Reductions are deterministic: a first pass writes one partial per block (a
// fixed tree inside the block), a second single-block pass combines the
// partials in index order, so results are bitwise reproducible for a given
// problem size.
#include "aux.h"

namespace green {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <typename T, typename Op>
__device__ T block_reduce(T v, Op op, T* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = op(sh[tid], sh[tid + s]);
    __syncthreads();
  }
  const T r = sh[0];
  __syncthreads();
  return r;
}

struct AddD {
  __device__ double operator()(double a, double b) const { return a + b; }
};
struct MaxD {
  __device__ double operator()(double a, double b) const { return a > b ? a : b; }
};

// gam[s][k] = -G[s][ntau-1][k];  gamT[s][k] = gam[s][k]^T   (G(0^-) = -G(beta^-))
__global__ void k_density(const double2* __restrict__ G, double2* __restrict__ gam, double2* __restrict__ gamT,
                          int ns, int ntau, int nk, int nao) {
  const int64_t nG = (int64_t)nao * nao;
  const int64_t total = (int64_t)ns * nk * nG;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sk = x / nG;
    const int e = (int)(x - sk * nG);
    const int i = e / nao, j = e - (e / nao) * nao;
    const int s = (int)(sk / nk), k = (int)(sk - (int64_t)s * nk);
    const double2 v = G[(((int64_t)s * ntau + (ntau - 1)) * nk + k) * nG + e];
    const double2 g = make_double2(-v.x, -v.y);
    gam[x] = g;
    if (gamT) gamT[sk * nG + (int64_t)j * nao + i] = g;
  }
}

// A[b] = I - A[b]  (n x n, batch stride n*n)
// dst[t][j][i] = src[nt - 1 - t][i][j] (conjugated if conj) for t in [t_lo, t_hi): one 32 x 32 tile of one t
// per block, transposed through LDS so that both the reads and the writes are row-contiguous.
// (src and dst may be one array, read and written on disjoint t ranges: no __restrict__.)
__global__ __launch_bounds__(256) void k_transpose_reverse(const double2* src, double2* dst, int n, int nt, int t_lo,
                                                           int conj) {
  __shared__ double2 tile[32][33];
  const int tiles = (n + 31) / 32;
  const int ti = blockIdx.x % tiles, tj = blockIdx.x / tiles;  // source tile rows ti, columns tj
  const int t = t_lo + blockIdx.y;
  const int64_t nn = (int64_t)n * n;
  const double2* S = src + (int64_t)(nt - 1 - t) * nn;
  double2* D = dst + (int64_t)t * nn;
  const int c = threadIdx.x & 31, r0 = threadIdx.x >> 5;
  for (int r = r0; r < 32; r += 8) {
    const int i = 32 * ti + r, j = 32 * tj + c;
    if (i < n && j < n) tile[r][c] = S[(int64_t)i * n + j];
  }
  __syncthreads();
  for (int r = r0; r < 32; r += 8) {
    const int j = 32 * tj + r, i = 32 * ti + c;  // destination row j, column i
    if (i < n && j < n) {
      const double2 v = tile[c][r];
      D[(int64_t)j * n + i] = conj ? make_double2(v.x, -v.y) : v;
    }
  }
}

__global__ void k_one_minus(double2* __restrict__ A, int n, int64_t batch) {
  const int64_t nn = (int64_t)n * n;
  const int64_t total = nn * batch;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(x % nn);
    const bool diag = (e / n) == (e % n);
    double2 v = A[x];
    v.x = (diag ? 1.0 : 0.0) - v.x;
    v.y = -v.y;
    A[x] = v;
  }
}

// A[b] = A[b] - I
__global__ void k_minus_one(double2* __restrict__ A, int n, int64_t batch) {
  const int64_t nn = (int64_t)n * n;
  const int64_t total = nn * batch;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(x % nn);
    if ((e / n) == (e % n)) A[x].x -= 1.0;
  }
}

// Dyson matrices A[s][m][k] = (i w_m + mu) S[k] - H0[s][k] - Sinf[s][k] - Sw[s][m][k]
__global__ void k_dyson_form(double2* __restrict__ A, const double2* __restrict__ S, const double2* __restrict__ H0,
                             const double2* __restrict__ Sinf, const double2* __restrict__ Sw,
                             const double* __restrict__ wf, double mu, int ns, int nw, int nk, int nao) {
  const int64_t nG = (int64_t)nao * nao;
  const int64_t total = (int64_t)ns * nw * nk * nG;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = x / nG;
    const int64_t e = x - b * nG;
    const int k = (int)(b % nk);
    const int64_t sm = b / nk;
    const int m = (int)(sm % nw);
    const int s = (int)(sm / nw);
    const double2 sv = S[(int64_t)k * nG + e];
    const double2 h = H0[((int64_t)s * nk + k) * nG + e];
    const double2 si = Sinf[((int64_t)s * nk + k) * nG + e];
    const double2 sw = Sw[x];
    const double w = wf[m];
    double2 v;
    // (mu + i w) * S
    v.x = mu * sv.x - w * sv.y;
    v.y = mu * sv.y + w * sv.x;
    v.x -= h.x + si.x + sw.x;
    v.y -= h.y + si.y + sw.y;
    A[x] = v;
  }
}

// tr[b] = sum_ij X_b[i][j] Y_{b'}[j][i],  X_b at X + xoff(b), Y at Y + yoff(b)
//   xoff(b) = b * xs;  yoff(b) = ((b / ydiv) % ymod) * ys + (b / (ydiv * ymod)) * ys2
__global__ __launch_bounds__(256) void k_trace_prod(const double2* __restrict__ X, int64_t xs,
                                                    const double2* __restrict__ Y, int64_t ydiv, int64_t ymod,
                                                    int64_t ys, int64_t ys2, int nao, double2* __restrict__ tr) {
  __shared__ double sh[256];
  const int64_t b = blockIdx.x;
  const double2* x = X + b * xs;
  const double2* y = Y + ((b / ydiv) % ymod) * ys + (b / (ydiv * ymod)) * ys2;
  double re = 0.0, im = 0.0;
  const int nn = nao * nao;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int i = e / nao, j = e - (e / nao) * nao;
    const double2 p = cmul(x[e], y[j * nao + i]);
    re += p.x;
    im += p.y;
  }
  re = block_reduce(re, AddD(), sh);
  im = block_reduce(im, AddD(), sh);
  if (threadIdx.x == 0) tr[b] = make_double2(re, im);
}

// out = scale * sum_b Re(w[(b / wdiv) % wmod] * tr[b])   (w == nullptr: weight 1); single block, fixed order.
__global__ __launch_bounds__(256) void k_weighted_sum(const double2* __restrict__ tr, int64_t n,
                                                      const double2* __restrict__ w, int64_t wdiv, int64_t wmod,
                                                      int64_t wstride, double scale, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < n; b += blockDim.x) {
    double2 t = tr[b];
    if (w) t = cmul(w[((b / wdiv) % wmod) * wstride], t);
    acc += t.x;
  }
  acc = block_reduce(acc, AddD(), sh);
  if (threadIdx.x == 0) *out = scale * acc;
}

// Mixing with diagnostics: S = alpha * Snew + (1 - alpha) * S; partial[block] = max |S_out - S_in|
__global__ __launch_bounds__(256) void k_mix(double2* __restrict__ S, const double2* __restrict__ Snew, double alpha,
                                             int64_t n, double* __restrict__ partial) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const double2 o = S[x];
    const double2 a = Snew[x];
    double2 v;
    if (alpha == 1.0) {
      v = a;
    } else {
      v.x = alpha * a.x + (1.0 - alpha) * o.x;
      v.y = alpha * a.y + (1.0 - alpha) * o.y;
    }
    const double dx = v.x - o.x, dy = v.y - o.y;
    const double d = sqrt(dx * dx + dy * dy);
    mx = (d > mx || d != d) ? d : mx;
    S[x] = v;
  }
  mx = block_reduce(mx, MaxD(), sh);
  if (partial && threadIdx.x == 0) partial[blockIdx.x] = mx;
}

// partial[block] = max |X_b[i][j] - conj X_b[j][i]| over matrices of size nao
__global__ __launch_bounds__(256) void k_herm(const double2* __restrict__ X, int64_t nmat, int nao,
                                              double* __restrict__ partial) {
  __shared__ double sh[256];
  const int64_t nG = (int64_t)nao * nao;
  const int64_t total = nmat * nG;
  double mx = 0.0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = x / nG;
    const int e = (int)(x - b * nG);
    const int i = e / nao, j = e - (e / nao) * nao;
    const double2 a = X[x];
    const double2 c = X[b * nG + (int64_t)j * nao + i];
    const double dx = a.x - c.x, dy = a.y + c.y;
    const double d = sqrt(dx * dx + dy * dy);
    mx = (d > mx || d != d) ? d : mx;
  }
  mx = block_reduce(mx, MaxD(), sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = mx;
}

__global__ __launch_bounds__(256) void k_max_partials(const double* __restrict__ partial, int n,
                                                      double* __restrict__ out) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int b = threadIdx.x; b < n; b += blockDim.x) {
    const double v = partial[b];
    mx = (v > mx || v != v) ? v : mx;
  }
  mx = block_reduce(mx, MaxD(), sh);
  if (threadIdx.x == 0) *out = mx;
}

// DIIS helpers.  partial[block] = sum Re(conj(a) b) over a grid-strided range (fixed grid: deterministic).
__global__ __launch_bounds__(256) void k_dot_re(const double2* __restrict__ a, const double2* __restrict__ b,
                                                int64_t n, double* __restrict__ partial) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const double2 u = a[x], v = b[x];
    acc += u.x * v.x + u.y * v.y;
  }
  acc = block_reduce(acc, AddD(), sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int n,
                                                      double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int b = threadIdx.x; b < n; b += blockDim.x) acc += partial[b];
  acc = block_reduce(acc, AddD(), sh);
  if (threadIdx.x == 0) *out = acc;
}

// r = x - old (old == nullptr: r = x)
__global__ void k_sub(double2* __restrict__ r, const double2* __restrict__ x, const double2* __restrict__ old,
                      int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = x[i];
    const double2 o = old ? old[i] : make_double2(0.0, 0.0);
    r[i] = make_double2(v.x - o.x, v.y - o.y);
  }
}

// out[i] = sum_j c_j base[slot_j * stride + i] (j in order); partial[block] = max |out_new - out_old|
__global__ __launch_bounds__(256) void k_combine(double2* __restrict__ out, const double2* __restrict__ base,
                                                 int64_t stride, int64_t n, CombineCoefs cf,
                                                 double* __restrict__ partial) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int j = 0; j < cf.m; ++j) {
      const double2 v = base[cf.slot[j] * stride + i];
      re += cf.c[j] * v.x;
      im += cf.c[j] * v.y;
    }
    const double2 o = out[i];
    const double dx = re - o.x, dy = im - o.y;
    const double d = sqrt(dx * dx + dy * dy);
    mx = (d > mx || d != d) ? d : mx;
    out[i] = make_double2(re, im);
  }
  mx = block_reduce(mx, MaxD(), sh);
  if (partial && threadIdx.x == 0) partial[blockIdx.x] = mx;
}

__global__ void k_zero(double2* __restrict__ X, int64_t n) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    X[x] = make_double2(0.0, 0.0);
}

// Momenta filled from a contracted one: for every block b < nblk and momentum k with kfill[k] != k,
// X[b][k] = X[b][kfill[k]] (kfill[k] < nk) or conj X[b][kfill[k] - nk] (kfill[k] >= nk).  Sources are contracted
// momenta (kfill[src] == src), so no block is both read and written.
__global__ void k_fill_k(double2* __restrict__ X, int64_t nblk, int nk, int64_t ne, const int32_t* __restrict__ kfill) {
  const int64_t n = nblk * nk * ne;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = x % ne;
    const int64_t bk = x / ne;
    const int k = (int)(bk % nk);
    const int f = kfill[k];
    if (f == k) continue;
    const int src = f < nk ? f : f - nk;
    const double2 v = X[(bk - k + src) * ne + e];
    X[x] = f < nk ? v : make_double2(v.x, -v.y);
  }
}

// 32 x 32 tiles of one (k, Q) block per workgroup, transposed through LDS (both sides row-contiguous).
__global__ __launch_bounds__(256) void k_herm_partner(const double2* __restrict__ in, double2* __restrict__ out,
                                                      int naux, int nao, const int32_t* __restrict__ kmap) {
  __shared__ double2 tile[32][33];
  const int tiles = (nao + 31) / 32;
  const int ti = blockIdx.x % tiles, tj = blockIdx.x / tiles;  // source tile rows ti, columns tj
  const int Q = blockIdx.y, k = blockIdx.z;
  const int64_t nG = (int64_t)nao * nao;
  const double2* S = in + ((int64_t)kmap[k] * naux + Q) * nG;
  double2* D = out + ((int64_t)k * naux + Q) * nG;
  const int c = threadIdx.x & 31, r0 = threadIdx.x >> 5;
  for (int r = r0; r < 32; r += 8) {
    const int i = 32 * ti + r, j = 32 * tj + c;
    if (i < nao && j < nao) tile[r][c] = S[(int64_t)i * nao + j];
  }
  __syncthreads();
  for (int r = r0; r < 32; r += 8) {
    const int j = 32 * tj + r, i = 32 * ti + c;  // destination row j, column i
    if (i < nao && j < nao) {
      const double2 v = tile[c][r];
      D[(int64_t)j * nao + i] = make_double2(v.x, -v.y);
    }
  }
}

// dst[b] = I - src[b]  (n x n, batch stride n*n; src and dst distinct)
__global__ void k_one_minus_copy(const double2* __restrict__ src, double2* __restrict__ dst, int n, int64_t batch) {
  const int64_t nn = (int64_t)n * n;
  const int64_t total = nn * batch;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(x % nn);
    const double2 v = src[x];
    dst[x] = make_double2(((e / n) == (e % n) ? 1.0 : 0.0) - v.x, -v.y);
  }
}

__global__ void k_copy(const double2* __restrict__ src, double2* __restrict__ dst, int64_t n) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    dst[x] = src[x];
}

// Input checks.  Each pass writes per block the largest |difference| and the largest |value| seen
// (partial[2 b], partial[2 b + 1]); k_check_finish compares them in block order and sets `bit` in *status when
// the difference exceeds tol times the largest value (or either is not finite).
constexpr int kCheckBlocks = 256;
__device__ __forceinline__ double cabs2(double2 v) { return sqrt(v.x * v.x + v.y * v.y); }
__device__ void check_store(double d, double m, double* partial) {
  __shared__ double sd[256], sm[256];
  d = block_reduce(d, MaxD(), sd);
  m = block_reduce(m, MaxD(), sm);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = d;
    partial[2 * blockIdx.x + 1] = m;
  }
}
// X[b][k][e] against its source under kfill (as k_fill_k: X[b][src] or conj X[b][src])
__global__ __launch_bounds__(256) void k_check_k(const double2* __restrict__ X, int64_t nblk, int nk, int64_t ne,
                                                 const int32_t* __restrict__ kfill, double* __restrict__ partial) {
  const int64_t total = nblk * nk * ne;
  double d = 0.0, m = 0.0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bk = x / ne, e = x - bk * ne;
    const int64_t b = bk / nk;
    const int k = (int)(bk - b * nk);
    const int f = kfill[k];
    const int src = f < nk ? f : f - nk;
    const double2 v = X[x], w = X[(b * nk + src) * ne + e];
    d = fmax(d, cabs2(make_double2(v.x - w.x, f < nk ? v.y - w.y : v.y + w.y)));
    m = fmax(m, cabs2(v));
  }
  check_store(d, m, partial);
}
// X_b[i][j] against conj X_b[j][i]
__global__ __launch_bounds__(256) void k_check_herm(const double2* __restrict__ X, int64_t nmat, int n,
                                                    double* __restrict__ partial) {
  const int64_t nn = (int64_t)n * n, total = nmat * nn;
  double d = 0.0, m = 0.0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = x / nn;
    const int e = (int)(x - b * nn), i = e / n, j = e - (e / n) * n;
    const double2 v = X[x], w = X[b * nn + (int64_t)j * n + i];
    d = fmax(d, cabs2(make_double2(v.x - w.x, v.y + w.y)));
    m = fmax(m, cabs2(v));
  }
  check_store(d, m, partial);
}
// V[q][k][Q] against its partner on three auxiliary indices Q in {0, naux / 2, naux - 1}:
//   pairing (mode 0):  V[-q][k + q][Q]^dagger   (V^{k2,k1}(Q) = V^{k1,k2}(Q)^dagger)
//   time reversal (1): conj V[-q][-k][Q]         (V^{-k1,-k2}(Q) = conj V^{k1,k2}(Q))
// kadd[q * nk + k] = k + q, kneg[k] = -k; every slab q of the full store is present.
__global__ __launch_bounds__(256) void k_check_v(const double2* __restrict__ V, int nk, int naux, int nao,
                                                 const int32_t* __restrict__ kadd, const int32_t* __restrict__ kneg,
                                                 int mode, double* __restrict__ partial) {
  const int64_t nG = (int64_t)nao * nao, nV = (int64_t)naux * nG;
  const int64_t total = (int64_t)nk * nk * 3 * nG;
  double d = 0.0, m = 0.0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = x / nG;
    const int e = (int)(x - blk * nG), i = e / nao, j = e - (e / nao) * nao;
    const int qi = (int)(blk % 3);
    const int64_t qk = blk / 3;
    const int k = (int)(qk % nk), q = (int)(qk / nk);
    const int Q = qi == 0 ? 0 : (qi == 1 ? naux / 2 : naux - 1);
    const double2 v = V[((int64_t)q * nk + k) * nV + Q * nG + e];
    double2 w;
    if (mode == 0)
      w = V[((int64_t)kneg[q] * nk + kadd[q * nk + k]) * nV + Q * nG + (int64_t)j * nao + i];
    else
      w = V[((int64_t)kneg[q] * nk + kneg[k]) * nV + Q * nG + e];
    d = fmax(d, cabs2(make_double2(v.x - w.x, v.y + w.y)));
    m = fmax(m, cabs2(v));
  }
  check_store(d, m, partial);
}
// V[q][k][Q] against V[R q][R k][Q] for every operation R (krot[r * nk + k] = R k) on three auxiliary indices
// Q in {0, naux / 2, naux - 1} (V^{R k1, R k2}(Q) = V^{k1,k2}(Q)); every slab q of the full store is present.
__global__ __launch_bounds__(256) void k_check_v_rot(const double2* __restrict__ V, int nk, int naux, int nao,
                                                     const int32_t* __restrict__ krot, int nops,
                                                     double* __restrict__ partial) {
  const int64_t nG = (int64_t)nao * nao, nV = (int64_t)naux * nG;
  const int64_t total = (int64_t)nops * nk * nk * 3 * nG;
  double d = 0.0, m = 0.0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = x / nG;
    const int e = (int)(x - blk * nG);
    const int qi = (int)(blk % 3);
    const int64_t rqk = blk / 3;
    const int k = (int)(rqk % nk);
    const int64_t rq = rqk / nk;
    const int q = (int)(rq % nk), r = (int)(rq / nk);
    const int Q = qi == 0 ? 0 : (qi == 1 ? naux / 2 : naux - 1);
    const int32_t* R = krot + (int64_t)r * nk;
    const double2 v = V[((int64_t)q * nk + k) * nV + Q * nG + e];
    const double2 w = V[((int64_t)R[q] * nk + R[k]) * nV + Q * nG + e];
    d = fmax(d, cabs2(make_double2(v.x - w.x, v.y - w.y)));
    m = fmax(m, cabs2(v));
  }
  check_store(d, m, partial);
}
__global__ __launch_bounds__(256) void k_check_finish(const double* __restrict__ partial, int nb, double tol, int bit,
                                                      int* __restrict__ status) {
  if (threadIdx.x != 0) return;
  double d = 0.0, m = 0.0;
  bool finite = true;
  for (int b = 0; b < nb; ++b) {
    finite = finite && isfinite(partial[2 * b]) && isfinite(partial[2 * b + 1]);
    d = fmax(d, partial[2 * b]);
    m = fmax(m, partial[2 * b + 1]);
  }
  if (!finite || !(d <= tol * m)) atomicOr(status, bit);
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_density(const double2* G, double2* gam, double2* gamT, int ns, int ntau, int nk, int nao,
                          hipStream_t s) {
  const int64_t n = (int64_t)ns * nk * nao * nao;
  hipLaunchKernelGGL(k_density, dim3(grid_for(n)), dim3(256), 0, s, G, gam, gamT, ns, ntau, nk, nao);
  return hipGetLastError();
}

hipError_t launch_transpose_reverse(const double2* src, double2* dst, int n, int nt, int t_lo, int t_hi,
                                   hipStream_t s, bool conj) {
  if (n <= 0 || t_hi <= t_lo) return hipSuccess;
  if (t_lo < 0 || t_hi > nt) return hipErrorInvalidValue;
  const int tiles = (n + 31) / 32;
  k_transpose_reverse<<<dim3((unsigned)(tiles * tiles), (unsigned)(t_hi - t_lo)), dim3(256), 0, s>>>(src, dst, n, nt,
                                                                                                    t_lo, conj ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_fill_k(double2* X, int64_t nblk, int nk, int64_t ne, const int32_t* kfill, hipStream_t s) {
  const int64_t n = nblk * nk * ne;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_k, dim3(grid_for(n)), dim3(256), 0, s, X, nblk, nk, ne, kfill);
  return hipGetLastError();
}

hipError_t launch_herm_partner(const double2* in, double2* out, int nk, int naux, int nao, const int32_t* kmap,
                               hipStream_t s) {
  if (nk <= 0 || naux <= 0 || nao <= 0) return hipSuccess;
  if (nk > 65535 || naux > 65535) return hipErrorInvalidValue;
  const int tiles = (nao + 31) / 32;
  k_herm_partner<<<dim3((unsigned)(tiles * tiles), (unsigned)naux, (unsigned)nk), dim3(256), 0, s>>>(in, out, naux,
                                                                                                    nao, kmap);
  return hipGetLastError();
}

hipError_t launch_one_minus(double2* A, int n, int64_t batch, hipStream_t s) {
  hipLaunchKernelGGL(k_one_minus, dim3(grid_for((int64_t)n * n * batch)), dim3(256), 0, s, A, n, batch);
  return hipGetLastError();
}

hipError_t launch_minus_one(double2* A, int n, int64_t batch, hipStream_t s) {
  hipLaunchKernelGGL(k_minus_one, dim3(grid_for((int64_t)n * n * batch)), dim3(256), 0, s, A, n, batch);
  return hipGetLastError();
}

hipError_t launch_dyson_form(double2* A, const double2* S, const double2* H0, const double2* Sinf,
                             const double2* Sw, const double* wf, double mu, int ns, int nw, int nk, int nao,
                             hipStream_t s) {
  const int64_t n = (int64_t)ns * nw * nk * nao * nao;
  hipLaunchKernelGGL(k_dyson_form, dim3(grid_for(n)), dim3(256), 0, s, A, S, H0, Sinf, Sw, wf, mu, ns, nw, nk, nao);
  return hipGetLastError();
}

hipError_t launch_trace_prod(const double2* X, int64_t xs, const double2* Y, int64_t ydiv, int64_t ymod, int64_t ys,
                             int64_t ys2, int nao, int64_t nb, double2* tr, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trace_prod, dim3((unsigned)nb), dim3(256), 0, s, X, xs, Y, ydiv, ymod, ys, ys2, nao, tr);
  return hipGetLastError();
}

hipError_t launch_weighted_sum(const double2* tr, int64_t n, const double2* w, int64_t wdiv, int64_t wmod,
                               int64_t wstride, double scale, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_weighted_sum, dim3(1), dim3(256), 0, s, tr, n, w, wdiv, wmod, wstride, scale, out);
  return hipGetLastError();
}

int mix_blocks(int64_t n) { return (int)grid_for(n) > 1024 ? 1024 : (int)grid_for(n); }

hipError_t launch_mix(double2* S, const double2* Snew, double alpha, int64_t n, double* partial, double* out,
                      hipStream_t s) {
  const int nb = mix_blocks(n);
  hipLaunchKernelGGL(k_mix, dim3(nb), dim3(256), 0, s, S, Snew, alpha, n, partial);
  if (partial && out) hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(256), 0, s, partial, nb, out);
  return hipGetLastError();
}

hipError_t launch_herm(const double2* X, int64_t nmat, int nao, double* partial, double* out, hipStream_t s) {
  const int nb = mix_blocks(nmat * nao * nao);
  hipLaunchKernelGGL(k_herm, dim3(nb), dim3(256), 0, s, X, nmat, nao, partial);
  hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(256), 0, s, partial, nb, out);
  return hipGetLastError();
}

hipError_t launch_dot_re(const double2* a, const double2* b, int64_t n, double* partial, double* out,
                         hipStream_t s) {
  const int nb = mix_blocks(n);
  hipLaunchKernelGGL(k_dot_re, dim3(nb), dim3(256), 0, s, a, b, n, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partial, nb, out);
  return hipGetLastError();
}

hipError_t launch_sub(double2* r, const double2* x, const double2* old, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(grid_for(n)), dim3(256), 0, s, r, x, old, n);
  return hipGetLastError();
}

hipError_t launch_combine(double2* out, const double2* base, int64_t stride, int64_t n, const CombineCoefs& cf,
                          double* partial, double* out_max, hipStream_t s) {
  if (cf.m < 1 || cf.m > 16) return hipErrorInvalidValue;
  const int nb = mix_blocks(n);
  hipLaunchKernelGGL(k_combine, dim3(nb), dim3(256), 0, s, out, base, stride, n, cf, partial);
  if (partial && out_max) hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(256), 0, s, partial, nb, out_max);
  return hipGetLastError();
}

hipError_t launch_one_minus_copy(const double2* src, double2* dst, int n, int64_t batch, hipStream_t s) {
  const int64_t total = (int64_t)n * n * batch;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_one_minus_copy, dim3(grid_for(total)), dim3(256), 0, s, src, dst, n, batch);
  return hipGetLastError();
}

hipError_t launch_copy(const double2* src, double2* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_check_k(const double2* X, int64_t nblk, int nk, int64_t ne, const int32_t* kfill, double tol,
                          int bit, double* partial, int* status, hipStream_t s) {
  if (nblk * nk * ne <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_k, dim3(kCheckBlocks), dim3(256), 0, s, X, nblk, nk, ne, kfill, partial);
  hipLaunchKernelGGL(k_check_finish, dim3(1), dim3(64), 0, s, partial, kCheckBlocks, tol, bit, status);
  return hipGetLastError();
}

hipError_t launch_check_herm(const double2* X, int64_t nmat, int n, double tol, int bit, double* partial, int* status,
                             hipStream_t s) {
  if (nmat * n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_herm, dim3(kCheckBlocks), dim3(256), 0, s, X, nmat, n, partial);
  hipLaunchKernelGGL(k_check_finish, dim3(1), dim3(64), 0, s, partial, kCheckBlocks, tol, bit, status);
  return hipGetLastError();
}

hipError_t launch_check_v(const double2* V, int nk, int naux, int nao, const int32_t* kadd, const int32_t* kneg,
                          int mode, double tol, int bit, double* partial, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_check_v, dim3(kCheckBlocks), dim3(256), 0, s, V, nk, naux, nao, kadd, kneg, mode, partial);
  hipLaunchKernelGGL(k_check_finish, dim3(1), dim3(64), 0, s, partial, kCheckBlocks, tol, bit, status);
  return hipGetLastError();
}

hipError_t launch_check_v_rot(const double2* V, int nk, int naux, int nao, const int32_t* krot, int nops, double tol,
                              int bit, double* partial, int* status, hipStream_t s) {
  if (nops <= 0 || nk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_v_rot, dim3(kCheckBlocks), dim3(256), 0, s, V, nk, naux, nao, krot, nops, partial);
  hipLaunchKernelGGL(k_check_finish, dim3(1), dim3(64), 0, s, partial, kCheckBlocks, tol, bit, status);
  return hipGetLastError();
}

hipError_t launch_zero(double2* X, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(256), 0, s, X, n);
  return hipGetLastError();
}

}  // namespace green
