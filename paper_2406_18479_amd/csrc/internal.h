// Internal declarations shared by the HIP translation units of libgreen_gw.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace green {

// Logical index x -> (x % ext) * s_in + (x / ext) * s_out  (a two-level strided map).
// A plain strided index uses ext = kFlat.
struct IdxMap {
  int32_t ext;
  int64_t s_in;
  int64_t s_out;
};
constexpr int32_t kFlat = 0x7fffffff;

static inline IdxMap flat(int64_t s) { return IdxMap{kFlat, s, 0}; }
static inline IdxMap two(int32_t ext, int64_t s_in, int64_t s_out) { return IdxMap{ext, s_in, s_out}; }

// Batch index b -> offset: lo = b % ext_lo, hi = b / ext_lo;
// offset = (tab ? tab[lo] : lo) * s_lo + hi * s_hi.
struct BatchMap {
  int32_t ext_lo;
  int64_t s_lo;
  const int32_t* tab;   // device, optional
  int64_t s_hi;
  const int32_t* htab;  // host mirror of tab (bounds validation only)
};
static inline BatchMap bnone() { return BatchMap{1, 0, nullptr, 0, nullptr}; }
static inline BatchMap bflat(int64_t s) { return BatchMap{kFlat, s, nullptr, 0, nullptr}; }
static inline BatchMap btwo(int32_t ext_lo, int64_t s_lo, const int32_t* tab, int64_t s_hi,
                            const int32_t* htab = nullptr) {
  return BatchMap{ext_lo, s_lo, tab, s_hi, htab};
}

// Storage type of a complex element.
enum ElemType : int32_t {
  kC64 = 0,   // double2 (re, im)                                         16 bytes
  kC32 = 1,   // float2 (re, im)                                           8 bytes
  kCB16 = 2,  // uint2 {hi, lo}: bf16 pairs (re | im << 16), x = hi + lo   8 bytes
  kCB16Q = 3, // as kCB16, elements grouped by 4 from the pointer passed: for element e the words at
              // 2 (e & ~3) + (e & 3) (hi) and that + 4 (lo), i.e. 16 bytes of hi words then 16 of lo words
              // per group.  Operands of this type are read by the LDS-DMA kernel only.
};
static inline int64_t elem_bytes(int32_t t) { return t == kC64 ? 16 : 8; }

// Complex operand of a batched GEMM: element (r, c) of batch b at p[batch(b) + r_map(r) + c_map(c)]
// (offsets in elements of type `etype`).
struct ZOp {
  const double2* p;
  IdxMap r, c;
  BatchMap b;
  int32_t conj;
  int32_t etype;
};

// Call sites of the batched GEMM.  Each site is its own kernel instantiation so that
// profilers attribute time per contraction.
enum class Site : int32_t {
  Generic = 0,
  P0_VG,        // P~0 stage 1: V^{k,k+q}(Q) G^{k+q}(tau)
  P0_VGrev,     // P~0 stage 1: V^{k+q,k}(Q') G^k(beta - tau)
  P0_Contract,  // P~0 stage 2: sum over (k, orbital pair) -> naux x naux
  Sig_PV,       // Sigma~ stage 1: P~(tau)^T V^{k,k-q}
  Sig_XG,       // Sigma~ stage 2: X G^{k-q}(tau)
  Sig_YV,       // Sigma~ stage 3: Y V^{k-q,k} summed over (Q', b)
  HF,           // Hartree-Fock terms
  Transform,    // Matsubara transforms and the energy quadrature
  GF2_VG,       // GF2 exchange: V^{a,a+q}(Q) G^{a+q} for every momentum pair
  GF2_Pair,     // GF2 exchange: four-index products summed over one auxiliary index
  GF2_Contract, // GF2 exchange: sum over (k1, k2) and three orbitals into Sigma
};

// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b]   (A: M x K, B: K x N, complex FP64).
// beta == 0 means C is not read.
//
// Split-K: with ksplit > 1 the K range is cut into ksplit slices; each slice writes its raw sum to
// partial[((slice * batch + b) * M + m) * N + n] and a second pass adds the slices in slice order
// (deterministic) and applies alpha, beta and the C maps.
struct ZGemm {
  Site site;
  int32_t M, N, K, batch;
  ZOp A, B;
  double2* C;
  IdxMap cr, cc;
  BatchMap cb;
  double2 alpha, beta;
  int32_t ksplit;
  double2* partial;
  int32_t prec;   // 0: FP64 MFMA, 1: FP32 MFMA, 2: split BF16 (hi + lo, three products) MFMA; prec 1 and 2
                  // accumulate in FP32 within a K slice, slices are combined in FP64
  int32_t ctype;  // ElemType of C (kCB16 requires beta == 0); prec 0 requires kC64 operands and output
  int32_t big;    // prec 2 with kCB16 operands, large-tile kernel: 1 = 192 x 96 tiles, 2 = 192 x 64,
                  // 3 = 320 x 64, 4 = 448 x 64 (3 and 4 need a K-contiguous B); LDS-DMA kernel (K-contiguous
                  // A and B, even K and strides, else as 3 and 1): 5 = 320 x 64, 6 = 192 x 128; LDS-DMA kernel
                  // with prefetched fragments (K maps flat or of extent a multiple of 16, else as 3, 1 and 2):
                  // 7 = 320 x 64, 8 = 128 x 128, 9 = 256 x 64, 10 = 128 x 64, 11 = 64 x 128 (two per CU);
                  // LDS-DMA kernel with 32-K stages in two slots (K maps flat or of extent >= 32, else as 1 and
                  // 2): 12 = 128 x 128, 13 = 256 x 64
  int32_t shape;  // 256-thread kernels: 0 = by size, 1..4 = 32x32, 32x64, 64x32, 64x64 tiles
  int32_t band;   // large-tile kernel: 0 = output tiles in column order; b > 0 = bands of b tile rows,
                  // each walked column by column (the A rows of a band stay in L2)
};

// Kernel variant a descriptor launches: family 0 FP64, 1 FP32, 2 split BF16 (256 threads), 3 split BF16
// large tiles (512 threads), 4 LDS-DMA large tiles (512 threads), 5 LDS-DMA large tiles with prefetched
// fragments (512 or 256 threads), 6 LDS-DMA large tiles with 32-K stages (512 threads); tile (bm, bn) =
// (32 p1, 32 p2), (64 p1, 32 p2) for families 3, 4 and 6.
struct Variant {
  int32_t family, p1, p2;  // family -1: no kernel reads these operands
  bool bnc;   // family 3: B is N-contiguous
  bool quad;  // family 4: kCB16Q operands
  int32_t threads, bm, bn;
};
Variant zgemm_variant(const ZGemm& g);
bool same_variant(const Variant& a, const Variant& b);
int64_t zgemm_blocks(const ZGemm& g);

// Tile of the GEMM variant the launcher will pick (for choosing split-K counts).
void zgemm_tile(const ZGemm& g, int* bm, int* bn, int* threads);
// Workgroups of the variant resident per CU for the large-tile kernels (1 or 2), 0 for the 256-thread kernels.
int zgemm_wgs_per_cu(const ZGemm& g);

hipError_t zgemm(const ZGemm& g, hipStream_t s);

// n independent GEMMs of one variant in one persistent launch (plus one grouped split-K pass when any
// has ksplit > 1).  `host` mirrors the n descriptors at `dev`; dev_start[i] is the first tile of
// descriptor i in the concatenated tile range (n + 1 entries, dev_start[0] = 0).
hipError_t zgemm_group(const ZGemm* host, int n, const ZGemm* dev, const int64_t* dev_start, hipStream_t s);

// Extent of a buffer in bytes: every element an operand touches must lie in [base, base + bytes).
struct Span {
  const void* base;
  int64_t bytes;
};

// Round a complex FP64 array to FP32 (kC32) or to split BF16 (kCB16), element for element.
hipError_t convert_c64(const double2* in, void* out, int32_t etype, int64_t n, hipStream_t s);
// out[b][j][i] = round(in[b][i][j]) for `batch` n x n matrices (kC32 or kCB16)
hipError_t convert_c64_t(const double2* in, void* out, int32_t etype, int n, int64_t batch, hipStream_t s);
// Sigma~ stages 2 and 3 fused for one tau chunk (split BF16, nao a multiple of 4 and at most 64):
//   partial[slice][k][j][tt][i] = sum over the slice's Q' of sum_{a,b} X[tt][k][Q'][i][a] GT[tt][kk(k)][b][a]
//                                  VT[kk(k)][Q'][j][b]
// then `reduce` (a split-K pass with ksplit = qsplit * xgv_halves(nao): rows j, columns (tt, i), batch k) adds
// the partial sums in order into Sigma with its alpha and beta.
struct XgvArgs {
  const uint2* X;      // element tt * x_tt + k * x_k + Q' * nao^2 + i * nao + a
  const uint2* GT;     // element tt * g_tt + kk * nao^2 + b * nao + a
  const uint2* VT;     // element kk * naux * nao * vs + Q' * nao * vs + j * vs + b, rows j of vs elements (nao
                       // rounded up to a multiple of 4, zero padded) in 4-element groups of hi words then lo words
                       // (convert_c64_tr with quad)
  const int32_t* kk;   // device: k -> block index of G and V
  double2* partial;    // qsplit * xgv_halves(nao) * nk * nao * tcn * nao elements
  int32_t nao, naux, nk, tcn, qsplit;
  int32_t vs;          // row length of the V^T blocks: xgv_vrow(nao)
  int64_t x_tt, x_k, g_tt;
};
// partial sums per Q' slice of the fused kernel (its b blocks split over that many waves: 2 for 16 < nao <= 64)
int xgv_halves(int nao);
// largest nao the fused kernel takes (even nao only), the padded row length of its V^T blocks, and the elements
// (8 bytes each) of one V^T block in memory: nao rows of xgv_vrow(nao) for nao <= 64, the 80 x 80 LDS image
// (xgv_vimage) above
constexpr int kXgvMaxNao = 80;
inline int xgv_vrow(int nao) { return (nao + 3) & ~3; }
inline int64_t xgv_vblock(int nao) { return nao > 64 ? 80 * 80 : (int64_t)nao * xgv_vrow(nao); }
// V^T blocks of the fused kernel for 64 < nao <= 80, written as the kernel's LDS image: for each of `blocks`
// (k, Q') blocks of `in` (nao x nao, element (b, j) at b nao + j, i.e. V^{k-q,k}_{bj}(Q')), 80 rows j of 40
// 16-byte units, unit (j, s) holding the hi (u even) or lo (u odd) words of the complex b = 4 (u / 2) .. + 3 of
// row j, u = s with its low three bits XORed with (j >> 1) & 7; zero past nao.
hipError_t xgv_vimage(const double2* in, void* out, int nao, int64_t blocks, hipStream_t s);
hipError_t sigma_xgv(const XgvArgs& a, const ZGemm& reduce, hipStream_t s);
// Stage 1 of P~0 in split BF16 for one tau chunk, as a dedicated kernel (even nao up to kVg1MaxNao):
//   rev = false (P0_VG):    T[tt][k][n][g]                = sum_a V[vk(k)][n][a] G[t(tt)][gk(k)][a][g]
//   rev = true  (P0_VGrev): T[tt][k][n / nao][g][n % nao] = sum_c V[vk(k)][n][c] G[t(tt)][gk(k)][c][g]
// with t(tt) = t0 + tdir tt, rows n < M = naux nao, g < nao; V and T kCB16, G read from its G^T images
// (vg1_image: one image of vg1_image_units(nao) 16-byte units per (t, k') of the spin, [t][k'] order).
struct Vg1Args {
  const uint2* V;      // element (kv nV + n) nao + a, nV = M nao
  const int32_t* vk;   // device: k -> kv (nullptr: kv = k)
  const void* img;     // G^T images, 16-byte aligned
  const int32_t* gk;   // device: k -> k' (nullptr: k' = k)
  uint2* T;            // tcn nk M nao elements
  int32_t t0, tdir;    // image node of chunk node tt: t0 + tdir tt (tdir = 1 or -1)
  int32_t tcn, tparts; // chunk nodes, and the parts of the chunk given to different workgroups (set by p0_vg1)
  int32_t nk, M, nao;
};
constexpr int kVg1MaxNao = 80;
int vg1_blocks(int nao);
bool vg1_ok(int nao);
int64_t vg1_image_units(int nao);
// G^T images of `blocks` nao x nao complex FP64 blocks of `in` (rows 16 vg1_blocks(nao) of the transpose, split BF16,
// zero past nao, swizzled as the kernel's LDS rows)
hipError_t vg1_image(const double2* in, void* out, int nao, int64_t blocks, hipStream_t s);
hipError_t p0_vg1(const Vg1Args& a, bool rev, hipStream_t s);
// out[b][c][r] = in[b][r][c] rounded to kC32 or kCB16 (rows x cols matrices, batch of them).  quad (kCB16,
// rows % 4 == 0): each output row holds its elements in groups of 4 as 4 hi words then 4 lo words.  rows_out >
// rows: output rows of rows_out elements, the ones past rows zero (out[b][c][r] over r < rows_out; quad needs
// rows_out % 4 == 0 instead).
hipError_t convert_c64_tr(const double2* in, void* out, int32_t etype, int rows, int cols, int batch, hipStream_t s,
                          bool quad = false, int rows_out = 0);

// Host-side bounds check of a GEMM descriptor against the buffers its operands point into (conservative:
// the box spanned by the index maps).  Returns false and fills `why` when an access could leave a buffer.
bool zgemm_in_bounds(const ZGemm& g, const Span& a, const Span& b, const Span& c, char* why, int why_len);

// GREEN_DRYRUN=1 in the environment: validate every launch and skip it (no device access at all).
bool dryrun();

// In-place inversion of `batch` complex n x n matrices at A + b*stride (row-major), Gauss-Jordan with
// partial pivoting.  A zero or non-finite pivot sets bit 0 of *status (the matrix is left finite).
hipError_t zinv_batched(double2* A, int n, int64_t stride, int batch, int* status, hipStream_t s);

}  // namespace green
