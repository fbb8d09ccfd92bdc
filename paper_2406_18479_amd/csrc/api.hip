// C ABI of libgreen_gw: plan, workspace layout and the orchestration of one
// self-consistent GW iteration (Sec. 2.3) from the batched kernels.
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/green_gw.h"
#include "aux.h"
#include "internal.h"

using green::BatchMap;
using green::IdxMap;
using green::ZGemm;
using green::ZOp;

namespace {

constexpr int kNumEvents = 9;

struct Region {
  size_t off = 0, bytes = 0;
};

// Autotuner: a contraction shape is identified by its call site, extents, arithmetic and element types;
// a candidate is a kernel tile choice plus a split-K count.
struct TuneKey {
  int32_t v[11];
  bool operator<(const TuneKey& o) const { return std::lexicographical_compare(v, v + 11, o.v, o.v + 11); }
};
struct TuneCand {
  int32_t shape, big, ksplit, band;
};
struct TuneEntry {
  std::vector<TuneCand> cands;
  std::vector<float> ms;  // time of each candidate's trial launch
  std::vector<hipEvent_t> ev;
  int trial = 0;          // next candidate to time; -1 before the untimed first call
  bool done = false;
  int chosen = 0;
  int64_t calls = 0;
};

}  // namespace

struct green_plan {
  green_dims d{};
  int nk = 0;
  int prec = GREEN_FP64;
  int tc = 1;  // tau nodes per contraction chunk
  int big_stage1 = 3;  // split-BF16 stage-1 kernel: 0 = 64 x 64 tiles, 1 = 192 x 96, 2 = 192 x 64, 3 = direct (p0_vg1,
                      // even nao up to 80; else 1)
  int big_p0 = 1;      // split-BF16 P~0 stage-2 kernel: 1 = 192 x 96 tiles, 2 = 192 x 64, 3 = 320 x 64, 4 = 448 x 64,
                       // LDS-DMA 5 = 320 x 64, 6 = 192 x 128
                       // (set at plan creation from naux)
  int big_sig = 6;     // split-BF16 Sigma~ stage-1 kernel (P~^T V over Q), the tiles of big_p0
  bool fuse_sig = false;  // split-BF16 plans, even nao up to 80: Sigma~ stages 2 and 3 in one kernel
  bool gf2 = false;       // the dynamic self-energy is GF2 (Eq. sigma2) instead of GW
  size_t chunk_bytes = 0;
  // GF2 exchange: per momentum triple (k, k1, k2), flattened ((k nk) + k1) nk + k2, the blocks of the V G
  // products and of V it reads: [0] V^{k,k1} G^{k1}(tau), [1] V^{k1,k3} G^{k3}(beta - tau), [2] V^{k3,k2} G^{k2}(tau),
  // [3] V^{k2,k}, with k3 = k1 + k2 - k (block index q nk + a of the pair V^{a,a+q})
  std::vector<int32_t> g2tab;
  std::vector<double> tau, wf, wb;
  std::vector<double2> TF_t2w, TF_w2t, TB_t2w, TB_w2t, Emass;
  std::vector<int32_t> kadd, ksub, kneg;  // [q][k]: k+q, k-q; [q]: -q
  std::vector<int32_t> qcan;              // momenta q with -q >= q (one of each +-q pair)
  // time reversal: the self-energy of -k is the complex conjugate of that of k
  bool trev = false;
  // point group acting on the k mesh (green_plan_set_kpoint_symmetry): krot[r][k] = R_r k; korb[k] = the
  // smallest momentum of the orbit of k (k itself without the group)
  bool ksym = false;
  int nrot = 0;
  std::vector<int32_t> krot, korb;
  // contracted momentum transfers qc of P~0 and the screening (one orbit of each pair {O, -O}, at its smallest
  // momentum; without the group, the q with -q >= q); for the others P~^q is the copy (qrel 1) or the transposed,
  // tau-reversed copy (qrel 2) of P~^{qsrc[q]}
  std::vector<int32_t> qc, qsrc, qrel;
  // contracted momenta kc of the self-energy (one per orbit, and with time reversal one orbit of each pair
  // {O, -O}; all k when neither applies); kfill[k] = k (contracted), the source momentum (copy) or the source + nk
  // (complex conjugate); ksubc[q][kk] = kc[kk] - q
  std::vector<int32_t> kc, kfill, ksubc;
  // Hermitian half store of V: the caller passes the slabs of the canonical q only (in qcan order); qslot[q] is
  // the slab of q there, -1 for the others (built from their partners on use)
  bool vhalf = false;
  std::vector<int32_t> qslot;
  // workspace regions
  Region r_TF_t2w, r_TF_w2t, r_TB_t2w, r_TB_w2t, r_Emass, r_wf, r_kadd, r_ksub, r_status, r_scal, r_partial;
  Region r_P, r_Pw, r_T1, r_T2, r_gam, r_gamT, r_D, r_Sinfn, r_Sign, r_Sw, r_A, r_tr, r_split, r_Vx, r_Ptx, r_Gx, r_GTx,
      r_Gimg;
  Region r_g2tab, r_Fp, r_Fm, r_X2, r_Z2;  // GF2 (empty until GREEN_OPT_GF2 is set)
  Region r_kneg, r_kc, r_ksubc, r_qc, r_kfill, r_krot;
  Region r_Vh;  // one partner slab of the half store (empty until GREEN_OPT_V_HALF is set)
  size_t ws_bytes = 0;
  void* bound_ws = nullptr;
  hipEvent_t ev[kNumEvents]{};
  bool events = false;
  void* clock = nullptr;  // KernelClock, created with the events
  // options
  int tune = 0;       // time the candidate kernels of every new contraction shape on its next calls
  int use_graph = 0;  // replay the Sigma evaluation of green_gw_iterate from a captured HIP graph
  std::map<TuneKey, TuneEntry> tuner;
  int64_t nops = 0;  // contractions of one Sigma evaluation
  // captured Sigma evaluation and the arguments it was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void* gargs[6] = {};
  double galpha = 0.0;
};

namespace {

template <typename T>
T* at(void* ws, const Region& r) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + r.off);
}

int hip_status(hipError_t e) { return e == hipSuccess ? GREEN_OK : GREEN_EHIP; }

#define HIP_TRY(expr)                          \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return GREEN_EHIP;   \
  } while (0)

#define GREEN_TRY(expr)              \
  do {                               \
    int r_ = (expr);                 \
    if (r_ != GREEN_OK) return r_;   \
  } while (0)

// Chebyshev-Lobatto check and energy quadrature E[t][t'] = int_0^beta l_t(tau) l_t'(tau) dtau
// (l_t: Lagrange basis of the nodes), from the DCT-I coefficients and W_lm = int T_l T_m dx.
bool build_mass_matrix(const std::vector<double>& tau, double beta, std::vector<double2>& E) {
  const int n = (int)tau.size();
  const int N = n - 1;
  for (int t = 0; t < n; ++t) {
    const double ref = 0.5 * beta * (1.0 - std::cos(M_PI * t / N));
    if (std::fabs(tau[t] - ref) > 1e-10 * beta) return false;
  }
  // C[l][t]: coefficient l of the interpolant from the value at node t; node t sits at x = cos(pi (N - t) / N)
  std::vector<double> C((size_t)n * n);
  for (int l = 0; l < n; ++l)
    for (int t = 0; t < n; ++t) {
      const int j = N - t;
      double c = (2.0 / N) * std::cos(M_PI * (double)l * j / N);
      if (j == 0 || j == N) c *= 0.5;
      if (l == 0 || l == N) c *= 0.5;
      C[(size_t)l * n + t] = c;
    }
  std::vector<double> W((size_t)n * n, 0.0);
  for (int l = 0; l < n; ++l)
    for (int m = 0; m < n; ++m)
      if (((l + m) & 1) == 0) {
        const double s = l + m, d = l - m;
        W[(size_t)l * n + m] = 1.0 / (1.0 - s * s) + 1.0 / (1.0 - d * d);
      }
  std::vector<double> WC((size_t)n * n, 0.0);  // W C
  for (int l = 0; l < n; ++l)
    for (int m = 0; m < n; ++m) {
      const double w = W[(size_t)l * n + m];
      if (w == 0.0) continue;
      for (int t = 0; t < n; ++t) WC[(size_t)l * n + t] += w * C[(size_t)m * n + t];
    }
  E.assign((size_t)n * n, make_double2(0.0, 0.0));
  for (int t = 0; t < n; ++t)
    for (int u = 0; u < n; ++u) {
      double acc = 0.0;
      for (int l = 0; l < n; ++l) acc += C[(size_t)l * n + t] * WC[(size_t)l * n + u];
      E[(size_t)t * n + u] = make_double2(0.5 * beta * acc, 0.0);
    }
  return true;
}

void kpoint(const int32_t* m, int k, int& a, int& b, int& c) {
  c = k % m[2];
  b = (k / m[2]) % m[1];
  a = k / (m[1] * m[2]);
}
int kflat(const int32_t* m, int a, int b, int c) {
  a = ((a % m[0]) + m[0]) % m[0];
  b = ((b % m[1]) + m[1]) % m[1];
  c = ((c % m[2]) + m[2]) % m[2];
  return (a * m[1] + b) * m[2] + c;
}

// Split-K scratch (a workspace region) and contraction precision of the current call, set by every
// entry point.
struct SplitBuf {
  double2* ptr = nullptr;
  int64_t cap = 0;  // complex elements
  int prec = 0;     // arithmetic of the P~0 stage-2 and Sigma~ stage-1 contractions
};
thread_local SplitBuf tl_split;
// plan of the current call (autotuner state) and whether launches are being captured into a graph
thread_local green_plan* tl_plan = nullptr;
thread_local bool tl_capturing = false;


int ensure_bound(green_plan* p, void* ws, hipStream_t s) {
  tl_split.ptr = reinterpret_cast<double2*>(static_cast<char*>(ws) + p->r_split.off);
  tl_split.cap = (int64_t)(p->r_split.bytes / sizeof(double2));
  tl_split.prec = p->prec;
  if (p->bound_ws == ws) return GREEN_OK;
  if (green::dryrun()) return GREEN_OK;
  auto up = [&](const Region& r, const void* src) {
    return hipMemcpyAsync(static_cast<char*>(ws) + r.off, src, r.bytes, hipMemcpyHostToDevice, s);
  };
  // index tables that may fill only part of their region
  auto upv = [&](const Region& r, const std::vector<int32_t>& v) {
    const size_t bytes = std::min(v.size() * 4, r.bytes);
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(static_cast<char*>(ws) + r.off, v.data(), bytes, hipMemcpyHostToDevice, s);
  };
  HIP_TRY(up(p->r_TF_t2w, p->TF_t2w.data()));
  HIP_TRY(up(p->r_TF_w2t, p->TF_w2t.data()));
  HIP_TRY(up(p->r_TB_t2w, p->TB_t2w.data()));
  HIP_TRY(up(p->r_TB_w2t, p->TB_w2t.data()));
  HIP_TRY(up(p->r_Emass, p->Emass.data()));
  HIP_TRY(up(p->r_wf, p->wf.data()));
  HIP_TRY(up(p->r_kadd, p->kadd.data()));
  HIP_TRY(up(p->r_ksub, p->ksub.data()));
  if (p->r_g2tab.bytes) HIP_TRY(up(p->r_g2tab, p->g2tab.data()));
  HIP_TRY(up(p->r_kneg, p->kneg.data()));
  HIP_TRY(upv(p->r_kc, p->kc));
  HIP_TRY(upv(p->r_ksubc, p->ksubc));
  HIP_TRY(upv(p->r_qc, p->qc));
  HIP_TRY(upv(p->r_kfill, p->kfill));
  HIP_TRY(upv(p->r_krot, p->krot));
  HIP_TRY(hipMemsetAsync(static_cast<char*>(ws) + p->r_status.off, 0, p->r_status.bytes, s));
  HIP_TRY(hipStreamSynchronize(s));
  p->bound_ws = ws;
  return GREEN_OK;
}

inline double2 cplx(double re, double im = 0.0) { return make_double2(re, im); }

// HIP-event timing of the two hot contraction launches (P~0 stage 2 and Sigma~ stage 1) inside
// green_gw_iterate: one event pair per launch, read after the iteration's final synchronisation.
struct KernelClock {
  std::vector<hipEvent_t> ev[2];
  int used[2] = {0, 0};
  double flops[2] = {0.0, 0.0};
  int begin(int slot, hipStream_t s) {
    const size_t need = 2 * (size_t)used[slot] + 2;
    while (ev[slot].size() < need) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return GREEN_EHIP;
      ev[slot].push_back(e);
    }
    return hip_status(hipEventRecord(ev[slot][2 * used[slot]], s));
  }
  int end(int slot, hipStream_t s, double f) {
    flops[slot] += f;
    const int e = hip_status(hipEventRecord(ev[slot][2 * used[slot] + 1], s));
    used[slot] += 1;
    return e;
  }
  void reset() {
    used[0] = used[1] = 0;
    flops[0] = flops[1] = 0.0;
  }
  int read(int slot, double* ms) const {
    double tot = 0.0;
    for (int i = 0; i < used[slot]; ++i) {
      float m = 0.f;
      if (hipEventElapsedTime(&m, ev[slot][2 * i], ev[slot][2 * i + 1]) != hipSuccess) return GREEN_EHIP;
      tot += m;
    }
    *ms = tot;
    return GREEN_OK;
  }
  ~KernelClock() {
    for (auto& v : ev)
      for (hipEvent_t e : v) (void)hipEventDestroy(e);
  }
};
thread_local KernelClock* tl_clock = nullptr;


// Recording: while tl_rec is set, gemm() and aux() append the launches of a call to a list instead of
// issuing them (the batched iteration replays the lists of several systems round by round).
struct Op {
  bool is_gemm = false;
  ZGemm g{};
  std::function<hipError_t(hipStream_t)> aux;
};
thread_local std::vector<Op>* tl_rec = nullptr;

// An auxiliary (non-GEMM) launch: issued now, or recorded.
template <class F>
int aux(hipStream_t s, F&& f) {
  if (tl_rec) {
    Op o;
    o.aux = std::function<hipError_t(hipStream_t)>(std::forward<F>(f));
    tl_rec->push_back(std::move(o));
    return GREEN_OK;
  }
  if (green::dryrun()) return GREEN_OK;
  return hip_status(f(s));
}

// GREEN_PROGRESS=1: long stages wait for each q-slab and report it on stderr (for runs of many minutes).
int progress(const char* stage, int q, int nq, hipStream_t s) {
  static const bool on = [] {
    const char* e = std::getenv("GREEN_PROGRESS");
    return e && e[0] == '1';
  }();
  if (!on || tl_rec || tl_capturing || green::dryrun()) return GREEN_OK;
  if (hipStreamSynchronize(s) != hipSuccess) return GREEN_EHIP;
  std::fprintf(stderr, "[green] %s q-slab %d/%d done\n", stage, q + 1, nq);
  std::fflush(stderr);
  return GREEN_OK;
}

// Split the K range when the output tiles alone cannot fill the GPU (256 CUs): aim for ~2048
// workgroups, keep every slice at least 64 deep, at most `cap` slices, and fit the partial sums into the
// scratch region.
int choose_ksplit(const ZGemm& g, int cap = 32) {
  const int M = g.M, N = g.N, K = g.K, batch = g.batch;
  int bm, bn, threads;
  green::zgemm_tile(g, &bm, &bn, &threads);
  const int64_t tiles = (int64_t)((M + bm - 1) / bm) * ((N + bn - 1) / bn) * batch;
  // 256-thread tiles: aim for ~2048 workgroups; large tiles (one or two workgroups per CU): ~1024 per slot
  const int per_cu = green::zgemm_wgs_per_cu(g);
  const int64_t target = per_cu ? 1024 * per_cu : 2048;
  if (tiles >= target / 2) return 1;
  int ks = (int)std::min<int64_t>((target + tiles - 1) / tiles, cap);
  ks = std::min(ks, std::max(1, K / 64));
  while (ks > 1 && (int64_t)ks * batch * M * N > tl_split.cap) --ks;
  return std::max(ks, 1);
}

void apply_cand(ZGemm& g, const TuneCand& c) {
  g.shape = c.shape;
  g.big = c.big;
  g.ksplit = c.ksplit;
  g.band = c.band;
  g.partial = c.ksplit > 1 ? tl_split.ptr : nullptr;
}

// Candidates for one contraction: the large-tile kernel (each tile shape) where the operands allow it,
// the 256-thread kernel at the size-picked tile and at 64 x 64, each at the default split-K count, twice
// and half of it (large tiles also at whole waves of workgroups).  The first candidate is the default.
std::vector<TuneCand> tune_candidates(const ZGemm& g0) {
  std::vector<TuneCand> out;
  auto add = [&](int shape, int big) {
    ZGemm g = g0;
    g.shape = shape;
    g.big = big;
    const int fam = green::zgemm_variant(g).family;
    if (fam < 0 || (big && fam != (big >= 7 ? 5 : big >= 5 ? 4 : 3))) return;
    g.ksplit = 1;
    const int ks0 = choose_ksplit(g);
    // large tiles run one workgroup per CU: also the split-K counts that fill one, two and three waves
    // of the 256 CUs as closely as possible from below
    int bm, bn, threads;
    green::zgemm_tile(g, &bm, &bn, &threads);
    const int per_cu = green::zgemm_wgs_per_cu(g);
    const bool whole = per_cu > 0;
    const int64_t tiles = (int64_t)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn) * g.batch;
    int opts[6] = {ks0, std::min(2 * ks0, 32), ks0 / 2, 0, 0, 0};
    if (whole)
      for (int w = 1; w <= 3; ++w) opts[2 + w] = (int)std::min<int64_t>(256 * per_cu * w / tiles, 32);
    for (int ks : opts) {
      if (ks < 1 || ks > std::max(1, g.K / 16)) continue;
      if (ks > 1 && (int64_t)ks * g.batch * g.M * g.N > tl_split.cap) continue;
      bool dup = false;
      for (const TuneCand& c : out)
        dup = dup || (c.shape == shape && c.big == big && c.ksplit == ks && c.band == 0);
      if (!dup) out.push_back(TuneCand{shape, big, ks, 0});
    }
    // large tiles over many tile rows: bands of 4 and 16 tile rows at the default split-K count
    if (whole && ks0 >= 1 && ks0 <= std::max(1, g.K / 16))
      for (int b : {4, 16})
        if ((g.M + bm - 1) / bm > b && (g.N + bn - 1) / bn > 1) out.push_back(TuneCand{shape, big, ks0, b});
  };
  // the default as launched untuned first (its split-K count may exceed what add() picks), then the
  // size-picked tile and the requested large tile
  if (green::zgemm_variant(g0).family >= 0) out.push_back(TuneCand{g0.shape, g0.big, g0.ksplit, 0});
  add(g0.shape, g0.big);
  if (g0.prec == 2) {
    add(0, 1);
    add(0, 2);
    // tall 320- and 448-row tiles where M needs more than one 192-row (320-row) tile
    if (g0.M > 192) add(0, 3);
    if (g0.M > 320) add(0, 4);
    // LDS-DMA tiles (where the operands allow them)
    add(0, 5);
    add(0, 6);
    add(0, 7);
    add(0, 8);
    add(0, 9);
    add(0, 10);
    add(0, 11);
    // (the 32-K-stage tiles 12 and 13 are plan options only: measured slower than the 16-K ring on the
    // contractions here, they would only lengthen tuning)
  }
  add(0, 0);
  add(4, 0);
  return out;
}

ZOp op(const void* ptr, IdxMap r, IdxMap c, BatchMap b, int etype = green::kC64, int conj = 0) {
  ZOp o;
  o.p = static_cast<const double2*>(ptr);
  o.r = r;
  o.c = c;
  o.b = b;
  o.conj = conj;
  o.etype = etype;
  return o;
}

int gemm(green::Site site, const char* label, const ZOp& A, const green::Span& sa, const ZOp& B, const green::Span& sb, void* C,
         const green::Span& sc, IdxMap cr, IdxMap cc, BatchMap cb, int M, int N, int K, int batch, double2 alpha,
         double2 beta, hipStream_t s, int prec = 0, int ctype = green::kC64, int big = 0, int ks_cap = 32) {
  ZGemm g;
  g.site = site;
  g.M = M;
  g.N = N;
  g.K = K;
  g.batch = batch;
  g.A = A;
  g.B = B;
  g.C = static_cast<double2*>(C);
  g.cr = cr;
  g.cc = cc;
  g.cb = cb;
  g.alpha = alpha;
  g.beta = beta;
  g.prec = prec;
  g.ctype = ctype;
  g.big = big;
  g.shape = 0;
  g.band = 0;
  g.ksplit = 1;
  g.ksplit = choose_ksplit(g, ks_cap);
  g.partial = g.ksplit > 1 ? tl_split.ptr : nullptr;
  char why[256];
  if (g.ksplit > 1 && (int64_t)g.ksplit * batch * M * N > tl_split.cap) return GREEN_EINVAL;
  if (!green::zgemm_in_bounds(g, sa, sb, sc, why, sizeof(why))) {
    std::fprintf(stderr, "green_gw: contraction '%s' rejected: %s\n", label, why);
    return GREEN_EINVAL;
  }
  // autotuned choice for this shape, or one trial launch of a candidate while tuning
  TuneEntry* te = nullptr;
  if (tl_plan) {
    const TuneKey key{{(int32_t)site, M, N, K, batch, prec, g.A.etype, g.B.etype, ctype, big, 0}};
    auto it = tl_plan->tuner.find(key);
    if (it != tl_plan->tuner.end() && it->second.done) {
      apply_cand(g, it->second.cands[it->second.chosen]);
    } else if (tl_plan->tune && !tl_rec && !tl_capturing && !green::dryrun()) {
      te = &tl_plan->tuner[key];
      if (te->cands.empty()) {
        te->cands = tune_candidates(g);
        te->ms.assign(te->cands.size(), 0.f);
        te->trial = -1;  // the first call runs the default untimed (code loading, first touch)
      }
      if (te->trial < 0) {
        te->trial = 0;
        te = nullptr;
      } else {
        apply_cand(g, te->cands[te->trial]);
      }
    }
  }
  if (te) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return GREEN_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return GREEN_EHIP;
    }
    te->ev.push_back(e0);
    te->ev.push_back(e1);
    HIP_TRY(hipEventRecord(e0, s));
    HIP_TRY(green::zgemm(g, s));
    HIP_TRY(hipEventRecord(e1, s));
    te->trial += 1;
    if (te->trial == (int)te->cands.size()) {
      HIP_TRY(hipEventSynchronize(e1));
      for (int c = 0; c < te->trial; ++c) HIP_TRY(hipEventElapsedTime(&te->ms[c], te->ev[2 * c], te->ev[2 * c + 1]));
      for (hipEvent_t e : te->ev) (void)hipEventDestroy(e);
      te->ev.clear();
      // the fastest candidate, unless it beats the default (candidate 0, the descriptor as launched untuned) by
      // less than 5 %: one timing per candidate carries a few per cent of noise (a candidate measured 3 % faster
      // once ran 2 % slower in the timed iterations), and keeping the default then keeps the choice stable from
      // run to run
      const int best = (int)(std::min_element(te->ms.begin(), te->ms.end()) - te->ms.begin());
      te->chosen = te->ms[best] < 0.95f * te->ms[0] ? best : 0;
      te->done = true;
    }
    return GREEN_OK;
  }
  if (tl_rec) {
    Op o;
    o.is_gemm = true;
    o.g = g;
    tl_rec->push_back(std::move(o));
    return GREEN_OK;
  }
  const int slot = site == green::Site::P0_Contract ? 0 : (site == green::Site::Sig_PV ? 1 : -1);
  KernelClock* clk = tl_clock;
  if (clk && slot >= 0 && !green::dryrun()) {
    GREEN_TRY(clk->begin(slot, s));
    GREEN_TRY(hip_status(green::zgemm(g, s)));
    GREEN_TRY(clk->end(slot, s, 8.0 * M * (double)N * K * batch));
    return GREEN_OK;
  }
  return hip_status(green::zgemm(g, s));
}

// extents in bytes: caller tensors are complex FP64 (count elements), workspace regions are raw bytes
green::Span span(const void* base, int64_t count) { return green::Span{base, count * (int64_t)sizeof(double2)}; }
green::Span span_ws(void* ws, const Region& r) {
  return green::Span{static_cast<char*>(ws) + r.off, (int64_t)r.bytes};
}
// element type of the contraction intermediates for a plan precision
int inter_type(int prec) { return prec == GREEN_FP64 ? green::kC64 : (prec == GREEN_FP32 ? green::kC32 : green::kCB16); }
// address of element `off` of an array of element type `etype`
const void* eptr(const void* base, int etype, int64_t off) {
  return static_cast<const char*>(base) + off * green::elem_bytes(etype);
}
void* eptr(void* base, int etype, int64_t off) { return static_cast<char*>(base) + off * green::elem_bytes(etype); }

using green::bflat;
using green::bnone;
using green::btwo;
using green::flat;
using green::two;

// Extents (complex elements) of the caller's tensors.
struct Extents {
  int64_t V, G, P, H, S, Sig;
};
Extents extents(const green_plan* p) {
  const green_dims& d = p->d;
  const int64_t nk = p->nk, nG = (int64_t)d.nao * d.nao, nV = (int64_t)d.naux * nG;
  Extents e;
  e.V = (p->vhalf ? (int64_t)p->qcan.size() : nk) * nk * nV;
  e.G = (int64_t)d.nspin * d.ntau * nk * nG;
  e.P = nk * d.ntau * (int64_t)d.naux * d.naux;
  e.H = (int64_t)d.nspin * nk * nG;
  e.S = nk * nG;
  e.Sig = e.G;
  return e;
}

// Split-BF16 plans whose Sigma~ stages 2 and 3 can run fused (even nao up to the fused kernel's 80).
bool fusable(int prec, int nao) { return prec == GREEN_BF16X3 && nao % 2 == 0 && nao <= green::kXgvMaxNao; }

// GF2 exchange tables of the contracted momenta kc (after the full tables: the four rows of every triple whose
// first momentum is contracted, in kc order).  The region holds room for every k.
void build_gf2_tail(green_plan* p) {
  if (p->g2tab.empty()) return;
  const int nk = p->nk;
  const int64_t ntrip = (int64_t)nk * nk * nk, nk2 = (int64_t)nk * nk;
  const int nkc = (int)p->kc.size();
  const int64_t nh = (int64_t)nkc * nk2;
  for (int w = 0; w < 4; ++w)
    for (int kk = 0; kk < nkc; ++kk)
      for (int64_t pr = 0; pr < nk2; ++pr)
        p->g2tab[4 * ntrip + w * nh + kk * nk2 + pr] = p->g2tab[w * ntrip + (int64_t)p->kc[kk] * nk2 + pr];
}

// Contracted sets and fill rules from the point group (if any) and time reversal.
//   Transfers: P~0^{R q} = P~0^q for R in the group (the sum over k is re-indexed by R), and
//   P~0^{-q}(tau) = P~0^q(beta - tau)^T always, so of each pair of orbits {O, -O} one is contracted, at its
//   smallest momentum c; the rest of O are copies of P~^c, the momenta of -O transposed, tau-reversed copies.
//   Momenta of the self-energy: Sigma~^{R k} = Sigma~^k; with time reversal Sigma~^{-k} = conj Sigma~^k as well.
void build_contracted_sets(green_plan* p) {
  const int nk = p->nk;
  std::vector<int32_t> orb(nk);
  for (int k = 0; k < nk; ++k) orb[k] = p->ksym ? p->korb[k] : k;
  p->qc.clear();
  p->qsrc.assign(nk, 0);
  p->qrel.assign(nk, 0);
  for (int q = 0; q < nk; ++q) {
    const int c = std::min(orb[q], orb[p->kneg[orb[q]]]);
    p->qsrc[q] = c;
    if (q == c) {
      p->qc.push_back(q);
      p->qrel[q] = 0;
    } else {
      p->qrel[q] = orb[q] == c ? 1 : 2;
    }
  }
  p->kc.clear();
  p->kfill.assign(nk, 0);
  for (int k = 0; k < nk; ++k) {
    const int c = p->trev ? std::min(orb[k], orb[p->kneg[orb[k]]]) : orb[k];
    if (k == c) {
      p->kc.push_back(k);
      p->kfill[k] = k;
    } else {
      p->kfill[k] = orb[k] == c ? c : c + nk;
    }
  }
  const int nkc = (int)p->kc.size();
  p->ksubc.resize((size_t)nk * nkc);
  for (int q = 0; q < nk; ++q)
    for (int kk = 0; kk < nkc; ++kk) p->ksubc[(size_t)q * nkc + kk] = p->ksub[(size_t)q * nk + p->kc[kk]];
  build_gf2_tail(p);
  p->bound_ws = nullptr;  // the tables are uploaded on the next call
}

// V slab of momentum transfer q, V[q][k] = V^{k,k+q}: the caller's array, or with the Hermitian half store the
// slot of a canonical q, or for the others the partner V^{k,k+q} = (V^{k+q,k})^dagger = (V[-q][k+q])^dagger
// written into the workspace (one slab at a time: of q and -q at most one is not canonical).
int v_slab(green_plan* p, const void* V, int q, void* ws, hipStream_t s, const void** ptr, green::Span* sp) {
  const int nk = p->nk, naux = p->d.naux, nao = p->d.nao;
  const int64_t slab = (int64_t)nk * naux * nao * nao;
  const Extents ex = extents(p);
  if (!p->vhalf || p->qslot[q] >= 0) {
    *ptr = eptr(V, green::kC64, (p->vhalf ? p->qslot[q] : q) * slab);
    *sp = span(V, ex.V);
    return GREEN_OK;
  }
  const int qn = p->kneg[q];
  if (p->qslot[qn] < 0 || (int64_t)p->r_Vh.bytes < slab * 16) return GREEN_EINVAL;
  const double2* in = static_cast<const double2*>(V) + p->qslot[qn] * slab;
  double2* out = at<double2>(ws, p->r_Vh);
  const int32_t* kmap = at<int32_t>(ws, p->r_kadd) + (size_t)q * nk;
  GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::launch_herm_partner(in, out, nk, naux, nao, kmap, st_); }));
  *ptr = out;
  *sp = span_ws(ws, p->r_Vh);
  return GREEN_OK;
}

// P[q][t] of the transfers that are not contracted, from the contracted ones: copies (qrel 1) or transposed,
// tau-reversed copies P[q][t] = P[qsrc][ntau - 1 - t]^T (qrel 2).
int fill_transfers(green_plan* p, double2* P, hipStream_t s) {
  const int nk = p->nk, naux = p->d.naux, ntau = p->d.ntau;
  const int64_t slab = (int64_t)ntau * naux * naux;
  for (int q = 0; q < nk; ++q) {
    if (p->qrel[q] == 0) continue;
    const double2* src = P + (int64_t)p->qsrc[q] * slab;
    double2* dst = P + (int64_t)q * slab;
    if (p->qrel[q] == 1)
      GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::launch_copy(src, dst, slab, st_); }));
    else
      GREEN_TRY(aux(s, [=](hipStream_t st_) {
        return green::launch_transpose_reverse(src, dst, naux, ntau, 0, ntau, st_);
      }));
  }
  return GREEN_OK;
}

// ---------------------------------------------------------------- polarization
int run_polarization(green_plan* p, const void* V, const void* G, void* P0, void* ws, hipStream_t s) {
  const green_dims& d = p->d;
  const int nk = p->nk, nao = d.nao, naux = d.naux, ntau = d.ntau, ns = d.nspin;
  const int64_t nG = (int64_t)nao * nao, nV = (int64_t)naux * nG, slab = (int64_t)nk * nV;
  const Extents ex = extents(p);
  const int32_t* kadd = at<int32_t>(ws, p->r_kadd);
  const int32_t* hadd = p->kadd.data();
  double2* T1 = at<double2>(ws, p->r_T1);
  double2* T2 = at<double2>(ws, p->r_T2);
  const green::Span sP = span(P0, ex.P);
  const green::Span sT1 = span_ws(ws, p->r_T1), sT2 = span_ws(ws, p->r_T2);
  double2* Pp = static_cast<double2*>(P0);
  const double w = ns == 1 ? 2.0 : 1.0;
  // Stage-1 operands: FP64 plans read V and G as given; FP32 plans round them while staging; split-BF16
  // plans round G once per call and each V slab once per q into the workspace, so that stage 1 runs on
  // the split-BF16 matrix cores as well.
  const bool bf = p->prec == GREEN_BF16X3;
  const int stage1 = p->prec == GREEN_FP64 ? 0 : (bf ? 2 : 1);
  const int st = bf ? green::kCB16 : green::kC64;  // storage of the stage-1 operands
  // storage of the stage-2 operands (kept interleaved: writing them in groups of 4 from the stage-1 epilogue
  // costs more in scattered 4-byte stores than the grouped reads save)
  const int tt = inter_type(p->prec);
  const void* Gs = G;
  green::Span sGs = span(G, ex.G);
  if (bf) {
    if ((int64_t)p->r_Gx.bytes < ex.G * 8 || (int64_t)p->r_Vx.bytes < 2 * slab * 8) return GREEN_EINVAL;
    GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64(static_cast<const double2*>(G), at<void>(ws, p->r_Gx), green::kCB16, ex.G, st_); }));
    Gs = at<void>(ws, p->r_Gx);
    sGs = span_ws(ws, p->r_Gx);
  }
  // split BF16, even nao up to 80: stage 1 by the direct kernel, which reads G from its G^T images
  const bool direct = bf && p->big_stage1 == 3 && green::vg1_ok(nao);
  const int64_t img_units = direct ? green::vg1_image_units(nao) : 0;
  if (direct) {
    if ((int64_t)p->r_Gimg.bytes < ex.G / nG * img_units * 16) return GREEN_EINVAL;
    void* img = at<void>(ws, p->r_Gimg);
    GREEN_TRY(aux(s, [=](hipStream_t st_) {
      return green::vg1_image(static_cast<const double2*>(G), img, nao, ex.G / nG, st_);
    }));
  }
  // P~0^{-q}(tau) = P~0^q(beta - tau)^T exactly (substitute k -> k + q and cycle the trace), and the grid is
  // symmetric (tau_{ntau-1-t} = beta - tau_t): only the transfers qc are contracted (q <= -q; with a point group
  // one orbit of each pair {O, -O}), the others are filled from them at the end; where -q lies in the orbit of q
  // (q = -q without a group) only the first half of the tau nodes is contracted, the second half is the
  // transposed, tau-reversed first half.
  // With time reversal also P~0^{-q}(tau) = conj P~0^q(tau), so P~0^q(beta - tau) = P~0^q(tau)^H: every q is
  // contracted on the first half of the tau nodes only, the second half is the conjugate transpose.
  const int nqc = (int)p->qc.size();
  for (int iq = 0; iq < nqc; ++iq) {
    const int q = p->qc[iq];
    const int qn = p->kneg[q];
    const bool self = p->qsrc[qn] == q && p->qrel[qn] != 2;  // -q in the orbit of q (or q itself)
    const int t_end = (self || p->trev) ? ntau / 2 : ntau;
    const void *Vq = nullptr, *Vqn = nullptr;
    green::Span sVs{}, sVn{};
    GREEN_TRY(v_slab(p, V, q, ws, s, &Vq, &sVs));
    GREEN_TRY(v_slab(p, V, qn, ws, s, &Vqn, &sVn));
    if (bf) {
      void* Vx = at<void>(ws, p->r_Vx);
      GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64(static_cast<const double2*>(Vq), Vx, green::kCB16, slab, st_); }));
      if (qn != q) GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64(static_cast<const double2*>(Vqn), eptr(Vx, green::kCB16, slab),
                                              green::kCB16, slab, st_); }));
      Vq = Vx;
      Vqn = qn != q ? eptr(Vx, green::kCB16, slab) : Vx;
      sVs = sVn = span_ws(ws, p->r_Vx);
    }
    for (int t0 = 0; t0 < t_end; t0 += p->tc) {
      const int tcn = std::min(p->tc, t_end - t0);
      for (int sp = 0; sp < ns; ++sp) {
        if (direct) {
          // T1[tt][k][(Q,d)][b] = sum_a V^{k,k+q}_{da}(Q) G^{k+q}_{ab}(tau_tt) and
          // T2[tt][k][Q'][d][b] = sum_c V^{k+q,k}_{bc}(Q') G^k_{cd}(beta - tau_tt), each V row read once per chunk
          // (every element read or written lies inside its region)
          if ((int64_t)tcn * nk * nV * 8 > (int64_t)std::min(p->r_T1.bytes, p->r_T2.bytes) ||
              (Vqn != Vq ? 2 : 1) * slab * 8 > (int64_t)p->r_Vx.bytes ||
              ((int64_t)(sp + 1) * ntau) * nk * img_units * 16 > (int64_t)p->r_Gimg.bytes)
            return GREEN_EINVAL;
          green::Vg1Args va{};
          va.img = static_cast<const char*>(at<void>(ws, p->r_Gimg)) + (int64_t)sp * ntau * nk * img_units * 16;
          va.tcn = tcn;
          va.tparts = 0;  // chosen by the launcher
          va.nk = nk;
          va.M = naux * nao;
          va.nao = nao;
          va.V = static_cast<const uint2*>(Vq);
          va.vk = nullptr;
          va.gk = kadd + q * nk;
          va.T = static_cast<uint2*>(static_cast<void*>(T1));
          va.t0 = t0;
          va.tdir = 1;
          GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::p0_vg1(va, false, st_); }));
          green::Vg1Args vr = va;
          vr.V = static_cast<const uint2*>(Vqn);
          vr.vk = kadd + q * nk;
          vr.gk = nullptr;
          vr.T = static_cast<uint2*>(static_cast<void*>(T2));
          vr.t0 = ntau - 1 - t0;
          vr.tdir = -1;
          GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::p0_vg1(vr, true, st_); }));
        }
        // T1[tt][k][(Q,d)][b] = sum_a V^{k,k+q}_{da}(Q) G^{k+q}_{ab}(tau_tt): one GEMM per k with the tau
        // nodes of the chunk folded into N = (tt, b), so each V block is read once per chunk
        if (!direct) GREEN_TRY(gemm(green::Site::P0_VG, "P0.VG", op(Vq, flat(nao), flat(1), bflat(nV), st), sVs,
                       op(eptr(Gs, st, ((int64_t)sp * ntau + t0) * nk * nG), flat(nao), two(nao, 1, (int64_t)nk * nG),
                          btwo(nk, nG, kadd + q * nk, 0, hadd + q * nk), st),
                       sGs, T1, sT1, flat(nao), two(nao, 1, (int64_t)nk * nV), bflat(nV), naux * nao, tcn * nao, nao,
                       nk, cplx(1), cplx(0), s, stage1, tt, bf ? (p->big_stage1 == 3 ? 1 : p->big_stage1) : 0));
        // T2[tt][k][Q'][d][b] = sum_c V^{k+q,k}_{bc}(Q') G^k_{cd}(beta - tau_tt)   (stored transposed in (b, d));
        // N = (tt, d), G(beta - tau) walks the grid backwards
        if (!direct) GREEN_TRY(gemm(green::Site::P0_VGrev, "P0.VGrev",
                       op(Vqn, flat(nao), flat(1), btwo(nk, nV, kadd + q * nk, 0, hadd + q * nk), st), sVn,
                       op(eptr(Gs, st, ((int64_t)sp * ntau + (ntau - 1 - t0)) * nk * nG), flat(nao),
                          two(nao, 1, -(int64_t)nk * nG), btwo(nk, nG, nullptr, 0), st),
                       sGs, T2, sT2, two(nao, 1, nG), two(nao, nao, (int64_t)nk * nV), bflat(nV), naux * nao,
                       tcn * nao, nao, nk, cplx(1), cplx(0), s, stage1, tt,
                       bf ? (p->big_stage1 == 3 ? 1 : p->big_stage1) : 0));
        // P0[q][t][Q][Q'] (+)= -(w/nk) sum_{k,(d,b)} T1[tt][k][Q][(d,b)] T2[tt][k][Q'][(d,b)]
        GREEN_TRY(gemm(green::Site::P0_Contract, "P0.contract",
                       op(T1, flat(nG), two((int32_t)nG, 1, nV), bflat((int64_t)nk * nV), tt), sT1,
                       op(T2, two((int32_t)nG, 1, nV), flat(nG), bflat((int64_t)nk * nV), tt), sT2,
                       Pp + ((int64_t)q * ntau + t0) * naux * naux, sP, flat(naux), flat(1),
                       bflat((int64_t)naux * naux), naux, naux, (int)(nk * nG), tcn, cplx(-w / nk),
                       cplx(sp == 0 ? 0.0 : 1.0), s, p->prec, green::kC64, bf ? p->big_p0 : 0));
      }
    }
    if (t_end < ntau) {
      double2* Pq = Pp + (int64_t)q * ntau * naux * naux;
      const bool cj = !self;  // time reversal
      GREEN_TRY(aux(s, [=](hipStream_t st_) {
        return green::launch_transpose_reverse(Pq, Pq, naux, ntau, ntau / 2, ntau, st_, cj);
      }));
    }
    GREEN_TRY(progress("polarization", iq, nqc, s));
  }
  return fill_transfers(p, Pp, s);
}

// ---------------------------------------------------------------- screening
int run_screen(green_plan* p, const void* P0, void* Pt, void* ws, hipStream_t s) {
  const green_dims& d = p->d;
  const int naux = d.naux, ntau = d.ntau, nwb = d.nw_b;
  const int64_t nP = (int64_t)naux * naux;
  const Extents ex = extents(p);
  double2* Pw = at<double2>(ws, p->r_Pw);
  const green::Span sPw = span_ws(ws, p->r_Pw);
  // The screening commutes with P(tau) -> P(beta - tau)^T (the bosonic transforms map it to P(i W) -> P(-i W)^T
  // on the symmetric grids, and [I - P]^{-1} P commutes with the transpose), so P~^{-q}(tau) = P~^q(beta - tau)^T,
  // and with copies: only the contracted transfers qc are screened, the others are filled from them as P~0 was.
  const int nc = (int)p->qc.size();
  const int32_t* qc = at<int32_t>(ws, p->r_qc);
  const int32_t* hqc = p->qc.data();
  // P0(i W_m) = sum_t TB_t2w[m][t] P0(tau_t)
  GREEN_TRY(gemm(green::Site::Transform, "screen.t2w", op(at<double2>(ws, p->r_TB_t2w), flat(ntau), flat(1), bnone()),
                 span_ws(ws, p->r_TB_t2w), op(P0, flat(nP), flat(1), btwo(nc, (int64_t)ntau * nP, qc, 0, hqc)),
                 span(P0, ex.P), Pw, sPw, flat(nP), flat(1), bflat((int64_t)nwb * nP), nwb, (int)nP, ntau, nc, cplx(1),
                 cplx(0), s));
  // P~(i W) = [I - P0]^{-1} P0, formed as a product with the inverse (not as [I - P0]^{-1} - I, which cancels
  // where |P0(i W)| << 1): per chunk of (q, m) matrices, B = I - P0 into T2 and inverted there, B P0 into T1,
  // copied back over P0
  if ((int64_t)nc * nwb * nP * 16 > (int64_t)p->r_Pw.bytes) return GREEN_EINVAL;
  {
    const int64_t per = (int64_t)(std::min(p->r_T1.bytes, p->r_T2.bytes) / (size_t)(nP * 16));
    if (per < 1) return GREEN_EINVAL;
    double2* T1 = at<double2>(ws, p->r_T1);
    double2* T2 = at<double2>(ws, p->r_T2);
    const green::Span sT1 = span_ws(ws, p->r_T1), sT2 = span_ws(ws, p->r_T2);
    const int64_t total = (int64_t)nc * nwb;
    for (int64_t b0 = 0; b0 < total; b0 += per) {
      const int nb = (int)std::min<int64_t>(per, total - b0);
      double2* P0w = Pw + b0 * nP;
      GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::launch_one_minus_copy(P0w, T2, naux, nb, st_); }));
      GREEN_TRY(aux(s, [=](hipStream_t st_) {
        return green::zinv_batched(T2, naux, nP, nb, at<int>(ws, p->r_status), st_);
      }));
      GREEN_TRY(gemm(green::Site::Generic, "screen.solve", op(T2, flat(naux), flat(1), bflat(nP)), sT2,
                     op(P0w, flat(naux), flat(1), bflat(nP)), sPw, T1, sT1, flat(naux), flat(1), bflat(nP), naux,
                     naux, naux, nb, cplx(1), cplx(0), s));
      GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::launch_copy(T1, P0w, (int64_t)nb * nP, st_); }));
    }
  }
  // P~(tau_t) = sum_m TB_w2t[t][m] P~(i W_m)
  GREEN_TRY(gemm(green::Site::Transform, "screen.w2t", op(at<double2>(ws, p->r_TB_w2t), flat(nwb), flat(1), bnone()),
                 span_ws(ws, p->r_TB_w2t), op(Pw, flat(nP), flat(1), bflat((int64_t)nwb * nP)), sPw, Pt,
                 span(Pt, ex.P), flat(nP), flat(1), btwo(nc, (int64_t)ntau * nP, qc, 0, hqc), ntau, (int)nP, nwb, nc,
                 cplx(1), cplx(0), s));
  return fill_transfers(p, static_cast<double2*>(Pt), s);
}

// ---------------------------------------------------------------- self-energy
int run_selfenergy(green_plan* p, const void* V, const void* G, const void* Pt, void* Sig, void* ws, hipStream_t s) {
  const green_dims& d = p->d;
  const int nk = p->nk, nao = d.nao, naux = d.naux, ntau = d.ntau, ns = d.nspin;
  const int64_t nG = (int64_t)nao * nao, nV = (int64_t)naux * nG, slab = (int64_t)nk * nV;
  const int64_t nP = (int64_t)naux * naux;
  const Extents ex = extents(p);
  const int32_t* ksub = at<int32_t>(ws, p->r_ksub);
  const int32_t* hsub = p->ksub.data();
  // With time reversal or a point group only the momenta kc[kk] are contracted: X, Y and the partial sums hold
  // kk = 0 .. nkx - 1, Sigma~ of the others is a copy or the complex conjugate of a contracted one's (filled at
  // the end).
  const bool tr = p->trev || p->ksym;
  const int nkx = tr ? (int)p->kc.size() : nk;
  const int32_t* kcan = at<int32_t>(ws, p->r_kc);
  const int32_t* hcan = p->kc.data();
  // k - q of each contracted momentum, and the Sigma~ block each one writes
  auto ktab = [&](int q) { return tr ? at<int32_t>(ws, p->r_ksubc) + (size_t)q * nkx : ksub + (size_t)q * nk; };
  auto hktab = [&](int q) { return tr ? p->ksubc.data() + (size_t)q * nkx : hsub + (size_t)q * nk; };
  const green::BatchMap sig_b = tr ? btwo(nkx, nG, kcan, 0, hcan) : bflat(nG);
  double2* T1 = at<double2>(ws, p->r_T1);
  double2* T2 = at<double2>(ws, p->r_T2);
  const green::Span sP = span(Pt, ex.P), sS = span(Sig, ex.Sig);
  const green::Span sT1 = span_ws(ws, p->r_T1), sT2 = span_ws(ws, p->r_T2);
  const double2* Pp = static_cast<const double2*>(Pt);
  double2* Sp = static_cast<double2*>(Sig);
  GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::launch_zero(Sp, ex.Sig, st_); }));
  // FP32 plans round the V slab of X = P~^T V to FP32 once per q and round the other operands while
  // staging; split-BF16 plans round G once per call, both V slabs of a q once, and keep X and Y in split
  // BF16, so every stage runs on the split-BF16 matrix cores.
  const bool mixed = p->prec != GREEN_FP64;
  const bool bf = p->prec == GREEN_BF16X3;
  const int vt = inter_type(p->prec);                                          // rounded V slabs
  const int xt = bf ? green::kCB16 : (mixed ? green::kC32 : green::kC64);      // X and Y
  const int gt = bf ? green::kCB16 : green::kC64;                              // G and the V of stage 3
  const int stage = p->prec == GREEN_FP64 ? 0 : (bf ? 2 : 1);
  // split-BF16 plans with an even naux run stage 1 on the LDS-DMA kernel (K-contiguous V slab)
  const bool vt_dma = bf && naux % 2 == 0;
  // with naux a multiple of 4 both of its operands hold the contraction index Q in groups of 4 (hi words, then
  // lo words), the order the LDS-DMA kernel reads its fragments in
  const bool pq = vt_dma && naux % 4 == 0;
  const int pvt = pq ? green::kCB16Q : green::kCB16;
  // ... and with nao a multiple of 4 up to 64, stages 2 and 3 in one kernel on G^T and per-block transposed
  // V slabs
  const bool fused = bf && p->fuse_sig;
  void* Vx = at<void>(ws, p->r_Vx);
  const green::Span sVx = span_ws(ws, p->r_Vx);
  void* Ptx = at<void>(ws, p->r_Ptx);
  const green::Span sPtx = span_ws(ws, p->r_Ptx);
  const void* Gs = G;
  green::Span sGs = span(G, ex.G);
  if (bf) {
    if ((int64_t)p->r_Gx.bytes < ex.G * 8) return GREEN_EINVAL;
    GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64(static_cast<const double2*>(G), at<void>(ws, p->r_Gx), green::kCB16, ex.G, st_); }));
    Gs = at<void>(ws, p->r_Gx);
    sGs = span_ws(ws, p->r_Gx);
  }
  if (fused) {
    if ((int64_t)p->r_GTx.bytes < ex.G * 8) return GREEN_EINVAL;
    GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64_tr(static_cast<const double2*>(G), at<void>(ws, p->r_GTx), green::kCB16, nao, nao, ns * ntau * nk, st_); }));
  }
  for (int q = 0; q < nk; ++q) {
    const int qn = p->kneg[q];
    const void* Vqn = nullptr;  // V^{k,k-q}: X = P~^T V
    const void* Vq = nullptr;   // V^{k-q,k}: Sigma += Y V
    green::Span sVa{}, sVb{};
    GREEN_TRY(v_slab(p, V, qn, ws, s, &Vqn, &sVa));
    GREEN_TRY(v_slab(p, V, q, ws, s, &Vq, &sVb));
    if (mixed) {
      if ((int64_t)p->r_Vx.bytes < (bf ? 2 : 1) * slab * green::elem_bytes(vt)) return GREEN_EINVAL;
      if (vt_dma) {
        // V^{k,k-q} stored [k][(i,a)][Q]: the contraction index Q runs contiguously for the LDS-DMA kernel
        GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64_tr(static_cast<const double2*>(Vqn), Vx, vt, naux, (int)nG, nk, st_, pq); }));
      } else {
        GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64(static_cast<const double2*>(Vqn), Vx, vt, slab, st_); }));
      }
      Vqn = Vx;
      sVa = sVx;
      if (bf) {
        const bool own = q != qn || vt_dma;  // stage 3 needs its own (untransposed) slab
        if (fused) {
          // V^{k-q,k}_{bj}(Q') stored [k][Q'][j][b] for the fused stages 2 and 3 (rows of b padded with zeros to a
          // multiple of 4)
          const int vs = green::xgv_vrow(nao);
          if (nao > 64)
            GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::xgv_vimage(static_cast<const double2*>(Vq), eptr(Vx, vt, slab), nao, (int64_t)nk * naux, st_); }));
          else
            GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64_tr(static_cast<const double2*>(Vq), eptr(Vx, vt, slab), vt, nao, nao, nk * naux, st_, true, vs); }));
        } else if (own) {
          GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64(static_cast<const double2*>(Vq), eptr(Vx, vt, slab), vt, slab, st_); }));
        }
        Vq = own || fused ? eptr(Vx, vt, slab) : Vx;
        sVb = sVx;
      }
    }
    if (bf) {
      // P~^q(tau)^T rounded to split BF16 for the large-tile kernel (K-contiguous rows)
      if ((int64_t)p->r_Ptx.bytes < (int64_t)ntau * nP * 8) return GREEN_EINVAL;
      if (pq)
        GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64_tr(Pp + (int64_t)q * ntau * nP, Ptx, green::kCB16, naux, naux, ntau, st_, true); }));
      else
        GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64_t(Pp + (int64_t)q * ntau * nP, Ptx, green::kCB16, naux, ntau, st_); }));
    }
    for (int t0 = 0; t0 < ntau; t0 += p->tc) {
      const int tcn = std::min(p->tc, ntau - t0);
      // X[tt][k][Q'][(i,a)] = sum_Q P~^q_{QQ'}(tau) V^{k,k-q}_{ia}(Q): the V slab is shared by the tau nodes
      // of the chunk, so they are stacked into the rows, M = (tt, Q') (no partial tiles at each naux edge)
      // (time reversal: one batch entry per contracted momentum, N = (i,a))
      const green::BatchMap vb = tr ? btwo(nkx, nV, kcan, 0, hcan) : bnone();
      GREEN_TRY(gemm(green::Site::Sig_PV, "Sigma.PV",
                     bf ? op(eptr(Ptx, pvt, (int64_t)t0 * nP), flat(naux), flat(1), bnone(), pvt)
                        : op(Pp + ((int64_t)q * ntau + t0) * nP, two(naux, 1, nP), flat(naux), bnone()),
                     bf ? sPtx : sP,
                     vt_dma ? op(Vqn, flat(1), flat(naux), vb, pvt)
                            : op(Vqn, flat(nG), tr ? flat(1) : two((int32_t)nG, 1, nV), vb,
                                 mixed ? vt : green::kC64),
                     sVa, T1, sT1, two(naux, nG, (int64_t)nkx * nV), tr ? flat(1) : two((int32_t)nG, 1, nV),
                     tr ? bflat(nV) : bnone(), tcn * naux, (int)(tr ? nG : nk * nG), naux, tr ? nkx : 1, cplx(1),
                     cplx(0), s, p->prec, xt, bf ? (vt_dma ? p->big_sig : 1) : 0));
      for (int sp = 0; sp < ns && fused; ++sp) {
        // Sigma[s][t][k][i][j] += -(1/nk) sum_{Q',b} (sum_a X[tt][k][Q'][i][a] G^{k-q}_{ab}(tau)) V^{k-q,k}_{bj}(Q'):
        // Q' slices of FP64 partial sums, added in slice order
        const int64_t blocks = (int64_t)tcn * nkx;
        const int hv = green::xgv_halves(nao);
        int qs = (int)std::min<int64_t>(16, std::max<int64_t>(1, (2560 + blocks - 1) / blocks));
        qs = std::min(qs, naux);
        while (qs > 1 && (int64_t)qs * hv * nkx * nG * tcn > tl_split.cap) --qs;
        if ((int64_t)qs * hv * nkx * nG * tcn > tl_split.cap) return GREEN_EINVAL;
        // every element the kernel reads lies inside its region
        if ((int64_t)tcn * nkx * nV * 8 > (int64_t)p->r_T1.bytes ||
            (int64_t)p->r_Vx.bytes < (slab + (int64_t)nk * naux * green::xgv_vblock(nao)) * 8 ||
            ((int64_t)sp * ntau + t0 + tcn) * nk * nG * 8 > (int64_t)p->r_GTx.bytes)
          return GREEN_EINVAL;
        green::XgvArgs xa{};
        xa.X = static_cast<const uint2*>(static_cast<const void*>(T1));
        xa.GT = static_cast<const uint2*>(at<void>(ws, p->r_GTx)) + ((int64_t)sp * ntau + t0) * nk * nG;
        xa.VT = static_cast<const uint2*>(Vq);
        xa.kk = ktab(q);
        xa.partial = tl_split.ptr;
        xa.nao = nao;
        xa.vs = green::xgv_vrow(nao);
        xa.naux = naux;
        xa.nk = nkx;
        xa.tcn = tcn;
        xa.qsplit = qs;
        xa.x_tt = (int64_t)nkx * nV;
        xa.x_k = nV;
        xa.g_tt = (int64_t)nk * nG;
        // the split-K pass: rows j, columns (tt, i), batch k; Sigma[s][t0 + tt][k][i][j]
        ZGemm rd{};
        rd.site = green::Site::Sig_YV;
        rd.M = nao;
        rd.N = tcn * nao;
        rd.K = naux;
        rd.batch = nkx;
        rd.C = Sp + ((int64_t)sp * ntau + t0) * nk * nG;
        rd.cr = flat(1);
        rd.cc = two(nao, nao, (int64_t)nk * nG);
        rd.cb = sig_b;
        rd.alpha = cplx(-1.0 / nk);
        rd.beta = cplx(1.0);
        rd.ksplit = qs * hv;
        rd.partial = tl_split.ptr;
        rd.prec = 2;
        rd.ctype = green::kC64;
        GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::sigma_xgv(xa, rd, st_); }));
      }
      for (int sp = 0; sp < ns && !fused; ++sp) {
        // Y[tt][k][(Q',i)][b] = sum_a X[tt][k][(Q',i)][a] G^{k-q}_{ab}(tau)
        GREEN_TRY(gemm(green::Site::Sig_XG, "Sigma.XG", op(T1, flat(nao), flat(1), bflat(nV), xt), sT1,
                       op(eptr(Gs, gt, ((int64_t)sp * ntau + t0) * nk * nG), flat(nao), flat(1),
                          btwo(nkx, nG, ktab(q), (int64_t)nk * nG, hktab(q)), gt),
                       sGs, T2, sT2, flat(nao), flat(1), bflat(nV), naux * nao, nao, nao, tcn * nkx, cplx(1), cplx(0),
                       s, stage, xt, bf ? 2 : 0));
        // Sigma[s][t][k][i][j] += -(1/nk) sum_{(Q',b)} Y[tt][k][Q'][i][b] V^{k-q,k}_{bj}(Q'): one GEMM per k
        // with the tau nodes folded into M = (tt, i), so each V block is read once per chunk
        GREEN_TRY(gemm(green::Site::Sig_YV, "Sigma.YV",
                       op(T2, two(nao, nao, (int64_t)nkx * nV), two(nao, 1, nG), bflat(nV), xt), sT2,
                       op(Vq, two(nao, nao, nG), flat(1), btwo(nkx, nV, ktab(q), 0, hktab(q)), gt), sVb,
                       Sp + ((int64_t)sp * ntau + t0) * nk * nG, sS, two(nao, nao, (int64_t)nk * nG), flat(1),
                       sig_b, tcn * nao, nao, naux * nao, nkx, cplx(-1.0 / nk), cplx(1.0), s, stage,
                       green::kC64));
      }
    }
    GREEN_TRY(progress("self-energy", q, nk, s));
  }
  if (tr) {
    const int32_t* kfill = at<int32_t>(ws, p->r_kfill);
    GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::launch_fill_k(Sp, (int64_t)ns * ntau, nk, nG, kfill, st_); }));
  }
  return GREEN_OK;
}

// ---------------------------------------------------------------- GF2 exchange term
// Adds the exchange part of Eq. sigma2 to Sig (G(-tau) = -G(beta - tau), prefactor 1/nk^2):
//   Sig[s][t][k] += -(1/nk^2) sum_{k1,k2} sum_{QQ'} F(k,k1)(Q) Fm(k1,k3)(Q') F(k3,k2)(Q) V^{k2,k}(Q'),
//   F(a,b) = V^{a,b} G^b_s(tau), Fm(a,b) = V^{a,b} G^b_s(beta - tau), k3 = k1 + k2 - k
// (the minus of the prefactor against the minus of the exchange term, and the minus of G(-tau)).  Per tau
// node the V G products of every momentum pair are formed once; per triple (k, k1, k2) the auxiliary
// indices are summed first, X[(i,q)][(m,l)] = sum_Q F(k,k1)_{iq}(Q) F(k3,k2)_{ml}(Q) and
// Z[(q,m)][(l,j)] = sum_Q' Fm(k1,k3)_{qm}(Q') V^{k2,k}_{lj}(Q'), then Sig_ij += X[i][(q,m,l)] Z[(q,m,l)][j]
// summed over the triples of a chunk as one contraction.
int run_gf2_exchange(green_plan* p, const void* V, const void* G, void* Sig, void* ws, hipStream_t s) {
  const green_dims& d = p->d;
  const int nk = p->nk, nao = d.nao, naux = d.naux, ntau = d.ntau, ns = d.nspin;
  const int64_t nG = (int64_t)nao * nao, nV = (int64_t)naux * nG, nG2 = nG * nG, n3 = nG * nao;
  const int nk2 = nk * nk;
  const Extents ex = extents(p);
  if (!p->gf2 || p->r_g2tab.bytes == 0 || p->vhalf) return GREEN_EINVAL;  // needs every V slab at once
  const int32_t* kadd = at<int32_t>(ws, p->r_kadd);
  const int32_t* hadd = p->kadd.data();
  const int64_t ntrip = (int64_t)nk2 * nk;
  // time reversal or a point group: only the triples of the contracted momenta kc (after the full tables), the
  // others' Sigma~ copied or conjugated at the end
  const bool tr = p->trev || p->ksym;
  const int nkx = tr ? (int)p->kc.size() : nk;
  const int64_t ntab = (int64_t)nkx * nk2;
  const int32_t* tab = at<int32_t>(ws, p->r_g2tab) + (tr ? 4 * ntrip : 0);
  const int32_t* htab = p->g2tab.data() + (tr ? 4 * ntrip : 0);
  const int32_t* kcan = at<int32_t>(ws, p->r_kc);
  const int32_t* hcan = p->kc.data();
  // Split-BF16 plans keep the pair products, V and the four-index products in split BF16, the operand of the
  // auxiliary sums that runs along the rows transposed (Q contiguous), so those sums run on the large-tile
  // kernel: F (Q-major) and F^T ([pair][(i,q)][Q]) share the first region, F'^T and the rounded V the second.
  const bool bf = p->prec == GREEN_BF16X3;
  const int et = bf ? green::kCB16 : green::kC64;
  const int64_t half = (int64_t)nk2 * nV;  // elements of one pair-product array
  void* Fp = at<void>(ws, p->r_Fp);
  void* Fm = at<void>(ws, p->r_Fm);
  void* FpT = bf ? eptr(Fp, et, half) : nullptr;
  void* Vr = bf ? eptr(Fm, et, half) : nullptr;
  void* X = at<void>(ws, p->r_X2);
  void* Z = at<void>(ws, p->r_Z2);
  const green::Span sV = span(V, ex.V), sG = span(G, ex.G), sS = span(Sig, ex.Sig);
  const green::Span sFp = span_ws(ws, p->r_Fp), sFm = span_ws(ws, p->r_Fm), sX = span_ws(ws, p->r_X2),
                    sZ = span_ws(ws, p->r_Z2);
  if (bf) {
    if ((int64_t)p->r_Fm.bytes < 2 * half * 8) return GREEN_EINVAL;
    GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::convert_c64(static_cast<const double2*>(V), Vr, green::kCB16, half, st_); }));
  }
  // triples per chunk: whole k (all nk^2 pairs) when they fit, else a run of pairs of one k; the contraction
  // depth (pairs) * nao^3 stays below 2^31
  const int64_t cap = (int64_t)(p->r_X2.bytes / (nG2 * green::elem_bytes(et)));
  int64_t pc_max = std::min<int64_t>(cap, (int64_t)nk2);
  pc_max = std::min<int64_t>(pc_max, ((int64_t)1 << 31) / n3 - 1);
  if (pc_max < 1) return GREEN_EINVAL;
  const int prec = p->prec;
  for (int sp = 0; sp < ns; ++sp)
    for (int t = 0; t < ntau; ++t) {
      // F[q][a] = V[q][a] G^{a+q}(tau) and F' with G(beta - tau): rows (Q, i), one batch entry per pair
      // (split BF16: F as given and transposed, F' transposed only)
      for (int pass = 0; pass < (bf ? 3 : 2); ++pass) {
        const bool rev = bf ? pass == 2 : pass == 1;
        const bool trans = bf && pass >= 1;  // stored transposed, [pair][(i,q)][Q]
        const int tn = rev ? ntau - 1 - t : t;
        void* C = rev ? Fm : (trans ? FpT : Fp);
        GREEN_TRY(gemm(green::Site::GF2_VG, rev ? "GF2.VGrev" : "GF2.VG", op(V, flat(nao), flat(1), bflat(nV)), sV,
                       op(static_cast<const double2*>(G) + ((int64_t)sp * ntau + tn) * nk * nG, flat(nao), flat(1),
                          btwo(nk2, nG, kadd, 0, hadd)),
                       sG, C, rev ? sFm : sFp, trans ? two(nao, (int64_t)nao * naux, 1) : flat(nao),
                       trans ? flat(naux) : flat(1), bflat(nV), naux * nao, nao, nao, nk2, cplx(1), cplx(0), s, prec,
                       et));
      }
      for (int k0 = 0; k0 < nkx;) {
        // chunk: kc whole momenta k (pc = nk^2 pairs each), or pairs [p0, p0 + pc) of one k
        const int kc = pc_max == nk2 ? (int)std::min<int64_t>(nkx - k0, std::max<int64_t>(1, cap / nk2)) : 1;
        for (int p0 = 0; p0 < nk2;) {
          const int pc = pc_max == nk2 ? nk2 : (int)std::min<int64_t>(nk2 - p0, pc_max);
          const int64_t b0 = (int64_t)k0 * nk2 + p0, nb = (int64_t)kc * pc;
          if (b0 + nb > ntab || nb * nG2 * green::elem_bytes(et) > (int64_t)p->r_X2.bytes) return GREEN_EINVAL;
          auto tb = [&](int which) { return btwo(green::kFlat, nV, tab + which * ntab + b0, 0, htab + which * ntab + b0); };
          // X[b][(i,q)][(m,l)] = sum_Q F(k,k1)[Q][(i,q)] F(k3,k2)[Q][(m,l)]
          GREEN_TRY(gemm(green::Site::GF2_Pair, "GF2.X",
                         bf ? op(FpT, flat(naux), flat(1), tb(0), et) : op(Fp, flat(1), flat(nG), tb(0)), sFp,
                         op(Fp, flat(nG), flat(1), tb(2), et), sFp, X, sX, flat(nG), flat(1), bflat(nG2), (int)nG,
                         (int)nG, naux, (int)nb, cplx(1), cplx(0), s, prec, et, bf ? 1 : 0));
          // Z[b][(q,m)][(l,j)] = sum_Q' F'(k1,k3)[Q'][(q,m)] V^{k2,k}[Q'][(l,j)]
          GREEN_TRY(gemm(green::Site::GF2_Pair, "GF2.Z",
                         bf ? op(Fm, flat(naux), flat(1), tb(1), et) : op(Fm, flat(1), flat(nG), tb(1)), sFm,
                         bf ? op(Vr, flat(nG), flat(1), tb(3), et) : op(V, flat(nG), flat(1), tb(3)), bf ? sFm : sV,
                         Z, sZ, flat(nG), flat(1), bflat(nG2), (int)nG, (int)nG, naux, (int)nb, cplx(1), cplx(0), s,
                         prec, et, bf ? 1 : 0));
          // Sig[s][t][k0 + kk][i][j] += -(1/nk^2) sum_{pair,(q,m,l)} X[kk pc + pair][i][(q,m,l)] Z[kk pc + pair][(q,m,l)][j]:
          // a few nao x nao outputs over a very deep K, so up to 256 K slices fill the GPU
          GREEN_TRY(gemm(green::Site::GF2_Contract, "GF2.contract",
                         op(X, flat(n3), two((int32_t)n3, 1, nG2), bflat((int64_t)pc * nG2), et), sX,
                         op(Z, two((int32_t)n3, nao, nG2), flat(1), bflat((int64_t)pc * nG2), et), sZ,
                         static_cast<double2*>(Sig) + (((int64_t)sp * ntau + t) * nk + (tr ? 0 : k0)) * nG, sS,
                         flat(nao), flat(1), tr ? btwo(kc, nG, kcan + k0, 0, hcan + k0) : bflat(nG), nao, nao,
                         (int)(pc * n3), kc, cplx(-1.0 / ((double)nk * nk)), cplx(1.0), s, prec, green::kC64, 0,
                         256));
          p0 += pc;
        }
        k0 += kc;
      }
    }
  if (tr) {
    const int32_t* kfill = at<int32_t>(ws, p->r_kfill);
    GREEN_TRY(aux(s, [=](hipStream_t st_) {
      return green::launch_fill_k(static_cast<double2*>(Sig), (int64_t)ns * ntau, nk, nG, kfill, st_);
    }));
  }
  return GREEN_OK;
}

// GF2 workspace and index tables (appended to the plan's workspace the first time GF2 is enabled).
void enable_gf2(green_plan* p) {
  if (p->r_g2tab.bytes) return;
  const green_dims& d = p->d;
  const int nk = p->nk;
  const int64_t nG = (int64_t)d.nao * d.nao, nV = (int64_t)d.naux * nG, nG2 = nG * nG;
  const int64_t ntrip = (int64_t)nk * nk * nk;
  p->g2tab.assign(4 * ntrip, 0);
  for (int k = 0; k < nk; ++k)
    for (int k1 = 0; k1 < nk; ++k1)
      for (int k2 = 0; k2 < nk; ++k2) {
        const int64_t b = ((int64_t)k * nk + k1) * nk + k2;
        const int k3 = p->ksub[(size_t)k * nk + p->kadd[(size_t)k2 * nk + k1]];  // (k1 + k2) - k
        auto blk = [&](int a, int bb) { return p->ksub[(size_t)a * nk + bb] * nk + a; };  // pair V^{a,bb}: q = bb - a
        p->g2tab[b] = blk(k, k1);
        p->g2tab[ntrip + b] = blk(k1, k3);
        p->g2tab[2 * ntrip + b] = blk(k3, k2);
        p->g2tab[3 * ntrip + b] = blk(k2, k);
      }
  // the same rows for the contracted momenta only, after the full tables (room for every k)
  p->g2tab.resize(8 * ntrip);
  build_gf2_tail(p);
  // four-index chunks: half the contraction budget each, between one triple and all of them
  const int64_t per = nG2 * 16;
  const int64_t want = std::max<int64_t>(1, (int64_t)(p->chunk_bytes / 2) / per);
  const int64_t trips = std::min<int64_t>(ntrip, want);
  size_t off = p->ws_bytes;
  auto take = [&](Region& r, size_t bytes) {
    r.off = off;
    r.bytes = bytes;
    off += (bytes + 255) & ~(size_t)255;
  };
  take(p->r_g2tab, p->g2tab.size() * 4);
  take(p->r_Fp, (size_t)nk * nk * nV * 16);
  take(p->r_Fm, (size_t)nk * nk * nV * 16);
  take(p->r_X2, (size_t)(trips * per));
  take(p->r_Z2, (size_t)(trips * per));
  p->ws_bytes = off;
  p->bound_ws = nullptr;  // the tables are uploaded on the next call
}

// ---------------------------------------------------------------- Hartree-Fock
int run_hf(green_plan* p, const void* V, const void* G, void* Sinf, void* ws, hipStream_t s) {
  const green_dims& d = p->d;
  const int nk = p->nk, nao = d.nao, naux = d.naux, ntau = d.ntau, ns = d.nspin;
  const int64_t nG = (int64_t)nao * nao, nV = (int64_t)naux * nG;
  const Extents ex = extents(p);
  const int32_t* ksub = at<int32_t>(ws, p->r_ksub);
  const int32_t* hsub = p->ksub.data();
  double2* gam = at<double2>(ws, p->r_gam);
  double2* gamT = at<double2>(ws, p->r_gamT);
  double2* D = at<double2>(ws, p->r_D);
  double2* T2 = at<double2>(ws, p->r_T2);
  const green::Span sV = span(V, ex.V), sH = span(Sinf, ex.H), sGam = span_ws(ws, p->r_gam),
                    sGamT = span_ws(ws, p->r_gamT), sD = span_ws(ws, p->r_D), sT2 = span_ws(ws, p->r_T2);
  const double2* Vp = static_cast<const double2*>(V);
  double2* Sp = static_cast<double2*>(Sinf);
  const double w = ns == 1 ? 2.0 : 1.0;
  GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::launch_density(static_cast<const double2*>(G), gam, gamT, ns, ntau, nk, nao, st_); }));
  // Hartree density D[Q] = (w/nk) sum_{s,k'} sum_{ab} V^{k'k'}_{ba}(Q) gamma^{k'}_{ab}
  for (int sp = 0; sp < ns; ++sp)
    GREEN_TRY(gemm(green::Site::HF, "HF.density", op(Vp, flat(nG), two((int32_t)nG, 1, nV), bnone()), sV,
                   op(gamT + (int64_t)sp * nk * nG, flat(1), flat(0), bnone()), sGamT, D, sD, flat(1), flat(0),
                   bnone(), naux, 1, (int)(nk * nG), 1, cplx(w / nk), cplx(sp == 0 ? 0.0 : 1.0), s));
  // Hartree term Sinf[s][k] = sum_Q D[Q] V^{kk}(Q)
  for (int sp = 0; sp < ns; ++sp)
    GREEN_TRY(gemm(green::Site::HF, "HF.hartree", op(D, flat(0), flat(1), bnone()), sD,
                   op(Vp, flat(nG), two((int32_t)nG, 1, nV), bnone()), sV, Sp + (int64_t)sp * nk * nG, sH, flat(0),
                   flat(1), bnone(), 1, (int)(nk * nG), naux, 1, cplx(1), cplx(0), s));
  // exchange: Sinf[s][k] -= (1/nk) sum_q sum_Q V^{k,k-q}(Q) gamma^{k-q} V^{k-q,k}(Q)
  // With time reversal or a point group it runs for the contracted momenta kk = 0 .. nkx - 1 only, as the
  // self-energy does: Sigma^inf(R k) = Sigma^inf(k) and Sigma^inf(-k) = conj Sigma^inf(k) hold for the Hartree term
  // as well (V^{Rk,Rk} = V^{k,k}, V^{-k,-k} = conj V^{k,k}), so the whole of Sigma^inf of the other momenta is filled
  // from the contracted ones at the end.
  const bool tr = p->trev || p->ksym;
  const int nkx = tr ? (int)p->kc.size() : nk;
  const int32_t* kcan = at<int32_t>(ws, p->r_kc);
  const int32_t* hcan = p->kc.data();
  auto ktab = [&](int q) { return tr ? at<int32_t>(ws, p->r_ksubc) + (size_t)q * nkx : ksub + (size_t)q * nk; };
  auto hktab = [&](int q) { return tr ? p->ksubc.data() + (size_t)q * nkx : hsub + (size_t)q * nk; };
  const green::BatchMap vn_b = tr ? btwo(nkx, nV, kcan, 0, hcan) : bflat(nV);
  const green::BatchMap hf_b = tr ? btwo(nkx, nG, kcan, 0, hcan) : bflat(nG);
  for (int q = 0; q < nk; ++q) {
    const int qn = p->kneg[q];
    const void *Vn = nullptr, *Vq = nullptr;
    green::Span sVn{}, sVq{};
    GREEN_TRY(v_slab(p, V, qn, ws, s, &Vn, &sVn));
    GREEN_TRY(v_slab(p, V, q, ws, s, &Vq, &sVq));
    for (int sp = 0; sp < ns; ++sp) {
      GREEN_TRY(gemm(green::Site::HF, "HF.Vgamma", op(Vn, flat(nao), flat(1), vn_b), sVn,
                     op(gam + (int64_t)sp * nk * nG, flat(nao), flat(1), btwo(nkx, nG, ktab(q), 0, hktab(q))),
                     sGam, T2, sT2, flat(nao), flat(1), bflat(nV), naux * nao, nao, nao, nkx, cplx(1), cplx(0), s));
      GREEN_TRY(gemm(green::Site::HF, "HF.exchange", op(T2, flat(nao), two(nao, 1, nG), bflat(nV)), sT2,
                     op(Vq, two(nao, nao, nG), flat(1), btwo(nkx, nV, ktab(q), 0, hktab(q))),
                     sVq, Sp + (int64_t)sp * nk * nG, sH, flat(nao), flat(1), hf_b, nao, nao, naux * nao, nkx,
                     cplx(-1.0 / nk), cplx(1.0), s));
    }
  }
  if (tr) {
    const int32_t* kfill = at<int32_t>(ws, p->r_kfill);
    GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::launch_fill_k(Sp, (int64_t)ns, nk, nG, kfill, st_); }));
  }
  return GREEN_OK;
}

// ---------------------------------------------------------------- Dyson + mu
// Bits of the device status word: a zero or non-finite pivot in a batched inversion, and inputs that break an
// assumption the plan relies on (time reversal, the point group; the debug checks of GREEN_CHECK=1).
constexpr int kStatusSingular = 1, kStatusTimeReversal = 2, kStatusInput = 4, kStatusSymmetry = 8;

int read_status_at(int* status, hipStream_t s) {
  if (green::dryrun()) return GREEN_OK;
  int st = 0;
  HIP_TRY(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (st) {
    HIP_TRY(hipMemsetAsync(status, 0, sizeof(int), s));
    return (st & (kStatusTimeReversal | kStatusInput | kStatusSymmetry)) ? GREEN_EINVAL : GREEN_ESINGULAR;
  }
  return GREEN_OK;
}
int read_status(green_plan* p, void* ws, hipStream_t s) { return read_status_at(at<int>(ws, p->r_status), s); }

// Device memory the Dyson step and the chemical-potential search work in: the plan's workspace regions,
// or the static scratch of the allocation-free entry point.
struct DysonMem {
  const double2 *TF_t2w, *TF_w2t;
  const double* wf;
  double2 *Sw, *A, *tr;
  double* scal;
  int* status;
  green::Span sTF_t2w, sTF_w2t, sSw, sA;
};
DysonMem dyson_mem(green_plan* p, void* ws) {
  DysonMem m;
  m.TF_t2w = at<double2>(ws, p->r_TF_t2w);
  m.TF_w2t = at<double2>(ws, p->r_TF_w2t);
  m.wf = at<double>(ws, p->r_wf);
  m.Sw = at<double2>(ws, p->r_Sw);
  m.A = at<double2>(ws, p->r_A);
  m.tr = at<double2>(ws, p->r_tr);
  m.scal = at<double>(ws, p->r_scal);
  m.status = at<int>(ws, p->r_status);
  m.sTF_t2w = green::Span{m.TF_t2w, (int64_t)p->r_TF_t2w.bytes};
  m.sTF_w2t = green::Span{m.TF_w2t, (int64_t)p->r_TF_w2t.bytes};
  m.sSw = green::Span{m.Sw, (int64_t)p->r_Sw.bytes};
  m.sA = green::Span{m.A, (int64_t)p->r_A.bytes};
  return m;
}

struct DysonCtx {
  green_plan* p;
  DysonMem m;
  hipStream_t s;
  const double2 *H0, *S, *Sinf;
  double nt;  // dry runs only: a stand-in electron count
};

// N(mu) = -(2/ns)(1/nk) sum_{s,m,k} Re( TF_w2t[ntau-1][m] Tr[G^k_s(i w_m; mu) S^k] )
int electron_count(const DysonCtx& c, double mu, double* n_out) {
  green_plan* p = c.p;
  const green_dims& d = p->d;
  const int nk = p->nk, nao = d.nao, ns = d.nspin, nw = d.nw_f, ntau = d.ntau;
  const int64_t nG = (int64_t)nao * nao;
  const int64_t nb = (int64_t)ns * nw * nk;
  if (green::dryrun()) {
    *n_out = (c.nt < 0 ? 1.0 : c.nt) + 0.5 * std::tanh(mu);
    return GREEN_OK;
  }
  double2* A = c.m.A;
  double2* tr = c.m.tr;
  double* scal = c.m.scal;
  HIP_TRY(green::launch_dyson_form(A, c.S, c.H0, c.Sinf, c.m.Sw, c.m.wf, mu, ns, nw, nk, nao, c.s));
  HIP_TRY(green::zinv_batched(A, nao, nG, (int)nb, c.m.status, c.s));
  HIP_TRY(green::launch_trace_prod(A, nG, c.S, 1, nk, nG, 0, nao, nb, tr, c.s));
  const double2* row = c.m.TF_w2t + (int64_t)(ntau - 1) * nw;
  HIP_TRY(green::launch_weighted_sum(tr, nb, row, nk, nw, 1, -(2.0 / ns) / nk, scal, c.s));
  HIP_TRY(hipMemcpyAsync(n_out, scal, sizeof(double), hipMemcpyDeviceToHost, c.s));
  HIP_TRY(hipStreamSynchronize(c.s));
  return GREEN_OK;
}

// Bracketing by doubling, then Illinois regula falsi (Sec. 2.3 step 3: fixed particle number).
int find_mu(const DysonCtx& c, double mu0, double nt, double* mu_out, double* n_out, int* evals) {
  const double tol = 1e-12 * std::max(1.0, std::fabs(nt));
  double n0;
  GREEN_TRY(electron_count(c, mu0, &n0));
  *evals = 1;
  if (!std::isfinite(n0)) return GREEN_ENAN;
  if (std::fabs(n0 - nt) <= tol) {
    *mu_out = mu0;
    *n_out = n0;
    return GREEN_OK;
  }
  double dlt = 1.0, lo = 0, hi = 0, nlo = 0, nhi = 0;
  bool ok = false;
  for (int i = 0; i < 60; ++i) {
    lo = mu0 - dlt;
    hi = mu0 + dlt;
    GREEN_TRY(electron_count(c, lo, &nlo));
    GREEN_TRY(electron_count(c, hi, &nhi));
    *evals += 2;
    if (!std::isfinite(nlo) || !std::isfinite(nhi)) return GREEN_ENAN;
    if (nlo <= nt && nt <= nhi) {
      ok = true;
      break;
    }
    dlt *= 2.0;
  }
  if (!ok) return GREEN_ENOCONV;
  double flo = nlo - nt, fhi = nhi - nt;
  if (std::fabs(flo) <= tol) {
    *mu_out = lo;
    *n_out = nlo;
    return GREEN_OK;
  }
  if (std::fabs(fhi) <= tol) {
    *mu_out = hi;
    *n_out = nhi;
    return GREEN_OK;
  }
  int side = 0;
  for (int it = 0; it < 200; ++it) {
    if (hi - lo < 1e-14) {
      const double mu = 0.5 * (lo + hi);
      double n;
      GREEN_TRY(electron_count(c, mu, &n));
      *evals += 1;
      *mu_out = mu;
      *n_out = n;
      return GREEN_OK;
    }
    double mu = (fhi != flo) ? (lo * fhi - hi * flo) / (fhi - flo) : 0.5 * (lo + hi);
    if (!(lo < mu && mu < hi)) mu = 0.5 * (lo + hi);
    double n;
    GREEN_TRY(electron_count(c, mu, &n));
    *evals += 1;
    if (!std::isfinite(n)) return GREEN_ENAN;
    const double f = n - nt;
    if (std::fabs(f) <= tol) {
      *mu_out = mu;
      *n_out = n;
      return GREEN_OK;
    }
    if (f < 0) {
      lo = mu;
      flo = f;
      if (side == -1) fhi *= 0.5;
      side = -1;
    } else {
      hi = mu;
      fhi = f;
      if (side == 1) flo *= 0.5;
      side = 1;
    }
  }
  return GREEN_ENOCONV;
}

int run_dyson_in(green_plan* p, const DysonMem& dm, const void* H0, const void* S, const void* Sinf, const void* Sig,
                 double nt, double* mu, void* G, double* n_out, int32_t* evals_out, hipStream_t s) {
  const green_dims& d = p->d;
  const int nk = p->nk, nao = d.nao, ns = d.nspin, nw = d.nw_f, ntau = d.ntau;
  const int64_t nG = (int64_t)nao * nao, nkG = (int64_t)nk * nG;
  const Extents ex = extents(p);
  // Sigma~(i w_m) = sum_t TF_t2w[m][t] Sigma~(tau_t)
  GREEN_TRY(gemm(green::Site::Transform, "dyson.t2w", op(dm.TF_t2w, flat(ntau), flat(1), bnone()), dm.sTF_t2w,
                 op(Sig, flat(nkG), flat(1), bflat((int64_t)ntau * nkG)), span(Sig, ex.Sig), dm.Sw, dm.sSw, flat(nkG),
                 flat(1), bflat((int64_t)nw * nkG), nw, (int)nkG, ntau, ns, cplx(1), cplx(0), s));
  DysonCtx c{p, dm, s, static_cast<const double2*>(H0), static_cast<const double2*>(S),
             static_cast<const double2*>(Sinf), nt};
  double m = *mu, n = 0.0;
  int evals = 0;
  if (nt >= 0) {
    GREEN_TRY(find_mu(c, *mu, nt, &m, &n, &evals));
  }
  // final Dyson at mu, then G(tau_t) = sum_m TF_w2t[t][m] G(i w_m)
  double nfinal;
  GREEN_TRY(electron_count(c, m, &nfinal));
  GREEN_TRY(gemm(green::Site::Transform, "dyson.w2t", op(dm.TF_w2t, flat(nw), flat(1), bnone()), dm.sTF_w2t,
                 op(dm.A, flat(nkG), flat(1), bflat((int64_t)nw * nkG)), dm.sA, G, span(G, ex.G), flat(nkG), flat(1),
                 bflat((int64_t)ntau * nkG), ntau, (int)nkG, nw, ns, cplx(1), cplx(0), s));
  GREEN_TRY(read_status_at(dm.status, s));
  *mu = m;
  if (n_out) *n_out = nfinal;
  if (evals_out) *evals_out = evals + 1;
  if (!std::isfinite(nfinal)) return GREEN_ENAN;
  return GREEN_OK;
}
int run_dyson(green_plan* p, const void* H0, const void* S, const void* Sinf, const void* Sig, double nt, double* mu,
              void* G, double* n_out, int32_t* evals_out, void* ws, hipStream_t s) {
  return run_dyson_in(p, dyson_mem(p, ws), H0, S, Sinf, Sig, nt, mu, G, n_out, evals_out, s);
}

// ---------------------------------------------------------------- energy (Galitskii-Migdal, with the new G)
int run_energy(green_plan* p, const void* H0, const void* G, const void* Sinf, const void* Sig, void* ws,
               hipStream_t s, green_report* rep) {
  const green_dims& d = p->d;
  const int nk = p->nk, nao = d.nao, ns = d.nspin, ntau = d.ntau;
  const int64_t nG = (int64_t)nao * nao, nkG = (int64_t)nk * nG;
  const Extents ex = extents(p);
  double2* gam = at<double2>(ws, p->r_gam);
  double2* tr = at<double2>(ws, p->r_tr);
  double* scal = at<double>(ws, p->r_scal);
  double2* Hm = at<double2>(ws, p->r_T1);
  const double2* Gp = static_cast<const double2*>(G);
  // Hm[s][t] = sum_t' E[t][t'] G[s][ntau-1-t']  (the interpolant of G(beta - tau) weighted by the mass matrix)
  GREEN_TRY(gemm(green::Site::Transform, "energy.mass", op(at<double2>(ws, p->r_Emass), flat(ntau), flat(1), bnone()),
                 span_ws(ws, p->r_Emass), op(Gp + (int64_t)(ntau - 1) * nkG, flat(-nkG), flat(1),
                                              bflat((int64_t)ntau * nkG)),
                 span(G, ex.G), Hm, span_ws(ws, p->r_T1), flat(nkG), flat(1), bflat((int64_t)ntau * nkG), ntau,
                 (int)nkG, ntau, ns, cplx(1), cplx(0), s));
  if (green::dryrun()) return GREEN_OK;
  HIP_TRY(green::launch_density(Gp, gam, nullptr, ns, ntau, nk, nao, s));
  // E_1b = (2/ns)(1/nk) sum Re Tr[gamma H0];  E_HF = (1/ns)(1/nk) sum Re Tr[gamma Sinf]
  HIP_TRY(green::launch_trace_prod(gam, nG, static_cast<const double2*>(H0), 1, (int64_t)ns * nk, nG, 0, nao,
                                   (int64_t)ns * nk, tr, s));
  HIP_TRY(green::launch_weighted_sum(tr, (int64_t)ns * nk, nullptr, 1, 1, 0, (2.0 / ns) / nk, scal + 0, s));
  HIP_TRY(green::launch_trace_prod(gam, nG, static_cast<const double2*>(Sinf), 1, (int64_t)ns * nk, nG, 0, nao,
                                   (int64_t)ns * nk, tr, s));
  HIP_TRY(green::launch_weighted_sum(tr, (int64_t)ns * nk, nullptr, 1, 1, 0, (1.0 / ns) / nk, scal + 1, s));
  // E_corr = -(1/ns)(1/nk) sum_{s,t,k} Re Tr[Sigma(tau_t) Hm[s][t]]
  const int64_t nb = (int64_t)ns * ntau * nk;
  HIP_TRY(green::launch_trace_prod(static_cast<const double2*>(Sig), nG, Hm, 1, nb, nG, 0, nao, nb, tr, s));
  HIP_TRY(green::launch_weighted_sum(tr, nb, nullptr, 1, 1, 0, -(1.0 / ns) / nk, scal + 2, s));
  HIP_TRY(green::launch_herm(static_cast<const double2*>(Sig), nb, nao, at<double>(ws, p->r_partial), scal + 3, s));
  double h[4];
  HIP_TRY(hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  rep->e_1b = h[0];
  rep->e_hf = h[1];
  rep->e_corr = h[2];
  rep->e_tot = h[0] + h[1] + h[2];
  rep->herm_err = h[3];
  (void)ex;
  return GREEN_OK;
}

int check_plan(green_plan* p, void* ws) {
  if (!p || !ws) return GREEN_EINVAL;
  return GREEN_OK;
}

// GREEN_CHECK=1: every entry point that reads G and V also checks the assumptions the method makes of them
// (G(tau) Hermitian per (s, t, k); the Hermitian pairing of V on a sample of auxiliary indices).
bool debug_checks() {
  static const bool on = [] {
    const char* e = std::getenv("GREEN_CHECK");
    return e && e[0] == '1';
  }();
  return on;
}

// Asynchronous checks of G and V against what the plan assumes; a violation is latched in the status word and
// reported (GREEN_EINVAL) by the next synchronising call.  With GREEN_OPT_TIME_REVERSAL: G^{-k}_s(tau) =
// conj G^k_s(tau) everywhere and V^{-k1,-k2}(Q) = conj V^{k1,k2}(Q) on three auxiliary indices of every pair
// (full store).  With a point group: G^k_s(tau) equal to G of the contracted momentum it is filled from (copy, or
// conjugate under time reversal) everywhere, and V^{R k1, R k2}(Q) = V^{k1,k2}(Q) for every operation on three
// auxiliary indices of every pair (full store).  Relative tolerance 1e-8 of the largest element.
int check_inputs(green_plan* p, const void* V, const void* G, void* ws, hipStream_t s) {
  const bool dbg = debug_checks();
  if (!p->trev && !p->ksym && !dbg) return GREEN_OK;
  const green_dims& d = p->d;
  const int nk = p->nk, nao = d.nao, naux = d.naux;
  const int64_t nG = (int64_t)nao * nao;
  const double2* Gp = static_cast<const double2*>(G);
  const double2* Vp = static_cast<const double2*>(V);
  double* part = at<double>(ws, p->r_partial);
  int* st = at<int>(ws, p->r_status);
  const int32_t* kneg = at<int32_t>(ws, p->r_kneg);
  const int32_t* kadd = at<int32_t>(ws, p->r_kadd);
  const int64_t nmat = (int64_t)d.nspin * d.ntau;
  const double tol = 1e-8;
  if (p->trev || p->ksym) {
    // G of every momentum that is not contracted against its source (orbit copies, time-reversal conjugates)
    const int32_t* kfill = at<int32_t>(ws, p->r_kfill);
    const int bit = p->ksym ? kStatusSymmetry : kStatusTimeReversal;
    GREEN_TRY(aux(s, [=](hipStream_t st_) {
      return green::launch_check_k(Gp, nmat, nk, nG, kfill, tol, bit, part, st, st_);
    }));
  }
  if (p->ksym && !p->vhalf) {
    const int32_t* krot = at<int32_t>(ws, p->r_krot);
    const int nrot = p->nrot;
    GREEN_TRY(aux(s, [=](hipStream_t st_) {
      return green::launch_check_v_rot(Vp, nk, naux, nao, krot, nrot, tol, kStatusSymmetry, part, st, st_);
    }));
  }
  if (p->trev) {
    if (!p->vhalf)
      GREEN_TRY(aux(s, [=](hipStream_t st_) {
        return green::launch_check_v(Vp, nk, naux, nao, kadd, kneg, 1, tol, kStatusTimeReversal, part, st, st_);
      }));
  }
  if (dbg) {
    GREEN_TRY(aux(s, [=](hipStream_t st_) {
      return green::launch_check_herm(Gp, nmat * nk, nao, tol, kStatusInput, part, st, st_);
    }));
    if (!p->vhalf)
      GREEN_TRY(aux(s, [=](hipStream_t st_) {
        return green::launch_check_v(Vp, nk, naux, nao, kadd, kneg, 0, tol, kStatusInput, part, st, st_);
      }));
  }
  return GREEN_OK;
}

// Sets the plan whose autotuner state gemm() consults for the lifetime of the scope.
struct PlanScope {
  green_plan* prev;
  explicit PlanScope(green_plan* p) : prev(tl_plan) { tl_plan = p; }
  ~PlanScope() { tl_plan = prev; }
};

int ensure_events(green_plan* p) {
  if (green::dryrun() || p->events) return GREEN_OK;
  for (int i = 0; i < kNumEvents; ++i)
    if (hipEventCreate(&p->ev[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(p->ev[j]);
      return GREEN_EHIP;
    }
  p->events = true;
  return GREEN_OK;
}

bool tuning_pending(const green_plan* p) {
  if (!p->tune) return false;
  if (p->tuner.empty()) return true;
  for (const auto& kv : p->tuner)
    if (!kv.second.done) return true;
  return false;
}

void drop_graph(green_plan* p) {
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
}

using MarkFn = std::function<hipError_t(int)>;

// The Sigma evaluation of one iteration (no host synchronisation, so it can be captured or recorded):
// Sigma^inf and Sigma~(tau) from (V, G) into the workspace, then mixed into the caller's Sinf and Sigma
// with weight alpha; max |Sigma~_new - Sigma~_old| lands in the scalar slot 8.
int sigma_eval(green_plan* p, const void* V, const void* G, void* Sinf, void* Sigma, double alpha, void* ws,
               hipStream_t s, const MarkFn* mark, bool mix = true) {
  const green_dims& d = p->d;
  const int64_t nG = (int64_t)d.nao * d.nao;
  const int64_t nsig = (int64_t)d.nspin * d.ntau * p->nk * nG, ninf = (int64_t)d.nspin * p->nk * nG;
  double2* P = at<double2>(ws, p->r_P);
  double2* Sinfn = at<double2>(ws, p->r_Sinfn);
  double2* Sign = at<double2>(ws, p->r_Sign);
  double* scal = at<double>(ws, p->r_scal);
  double* part = at<double>(ws, p->r_partial);
  auto m = [&](int i) { return mark ? hip_status((*mark)(i)) : GREEN_OK; };
  GREEN_TRY(check_inputs(p, V, G, ws, s));
  GREEN_TRY(run_hf(p, V, G, Sinfn, ws, s));
  GREEN_TRY(m(1));
  GREEN_TRY(run_polarization(p, V, G, P, ws, s));
  GREEN_TRY(m(2));
  // GF2: no screening, the bubble enters the self-energy bare (the direct term of Eq. sigma2), then the
  // exchange term is added
  if (!p->gf2) GREEN_TRY(run_screen(p, P, P, ws, s));
  GREEN_TRY(m(3));
  GREEN_TRY(run_selfenergy(p, V, G, P, Sign, ws, s));
  if (p->gf2) GREEN_TRY(run_gf2_exchange(p, V, G, Sign, ws, s));
  GREEN_TRY(m(4));
  if (!mix) return GREEN_OK;
  double2* Si = static_cast<double2*>(Sinf);
  double2* Sg = static_cast<double2*>(Sigma);
  GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::launch_mix(Si, Sinfn, alpha, ninf, nullptr, nullptr, st_); }));
  GREEN_TRY(aux(s, [=](hipStream_t st_) { return green::launch_mix(Sg, Sign, alpha, nsig, part, scal + 8, st_); }));
  return GREEN_OK;
}

// The rest of an iteration after the Sigma evaluation: Dyson with the chemical-potential search, the
// energy and the report (synchronises).
int close_iteration(green_plan* p, const void* H0, const void* S, void* G, void* Sinf, void* Sigma, double* mu,
                    double n_target, green_report* rep, void* ws, hipStream_t s, const MarkFn* mark = nullptr) {
  double n = 0.0;
  int32_t evals = 0;
  GREEN_TRY(run_dyson(p, H0, S, Sinf, Sigma, n_target, mu, G, &n, &evals, ws, s));
  if (mark) HIP_TRY((*mark)(6));
  GREEN_TRY(run_energy(p, H0, G, Sinf, Sigma, ws, s, rep));
  if (mark) HIP_TRY((*mark)(7));
  rep->n_elec = n;
  rep->mu = *mu;
  rep->mu_evals = evals;
  if (green::dryrun()) return GREEN_OK;
  double dsig = 0.0;
  HIP_TRY(hipMemcpyAsync(&dsig, at<double>(ws, p->r_scal) + 8, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  rep->max_dsigma = dsig;
  return GREEN_OK;
}

// Number of contractions the Sigma evaluation records (sizes the batched descriptor tables): a recording
// pass over stand-in addresses that are never dereferenced.
int count_ops(green_plan* p) {
  std::vector<Op> ops;
  char* fake = reinterpret_cast<char*>((uintptr_t)1 << 44);
  const SplitBuf saved = tl_split;
  tl_split.ptr = reinterpret_cast<double2*>(fake + p->r_split.off);
  tl_split.cap = (int64_t)(p->r_split.bytes / sizeof(double2));
  tl_split.prec = p->prec;
  green_plan* prev = tl_plan;
  tl_plan = nullptr;
  tl_rec = &ops;
  char* big = fake + ((uintptr_t)1 << 42);
  const int64_t step = (int64_t)1 << 40;
  const int st = sigma_eval(p, big, big + step, big + 2 * step, big + 3 * step, 1.0, fake, nullptr, nullptr);
  tl_rec = nullptr;
  tl_plan = prev;
  tl_split = saved;
  if (st != GREEN_OK) return st;
  int64_t n = 0;
  for (const Op& o : ops) n += o.is_gemm ? 1 : 0;
  p->nops = n;
  return GREEN_OK;
}

}  // namespace

// A recorded batched Sigma evaluation: per-system launch lists, the grouped schedule and its device tables.
struct BatchGroup {
  size_t first, count;  // descriptors [first, first + count)
  size_t start_off;     // tile offsets [start_off, start_off + count]
  bool solo = false;    // one contraction that fills the GPU on its own: its own (non-persistent) launch
};

struct green_batch {
  std::vector<green_plan*> plans;
  std::vector<green_system> sys;
  double alpha = 1.0;
  std::vector<std::vector<Op>> ops;
  std::vector<ZGemm> descs;
  std::vector<std::vector<BatchGroup>> groups;
  ZGemm* ddesc = nullptr;
  int64_t* dstart = nullptr;
  int use_graph = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~green_batch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// Pulay's constrained least squares for the DIIS coefficients: [[B, 1], [1^T, 0]] [c, l] = [0, 1] with B
// scaled by its largest diagonal element; Gaussian elimination with partial pivoting.  False if singular.
bool diis_solve(const double* B, int ld, int m, double* c) {
  double A[17][18];
  double dmax = 0.0;
  for (int i = 0; i < m; ++i) dmax = std::max(dmax, B[i * ld + i]);
  if (!(dmax > 0.0) || !std::isfinite(dmax)) return false;
  const int n = m + 1;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= n; ++j) A[i][j] = 0.0;
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < m; ++j) A[i][j] = B[i * ld + j] / dmax;
    A[i][m] = 1.0;
    A[m][i] = 1.0;
  }
  A[m][n] = 1.0;  // right-hand side column
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
    if (!(std::fabs(A[piv][col]) > 1e-300)) return false;
    if (piv != col)
      for (int j = 0; j <= n; ++j) std::swap(A[piv][j], A[col][j]);
    for (int r = col + 1; r < n; ++r) {
      const double f = A[r][col] / A[col][col];
      for (int j = col; j <= n; ++j) A[r][j] -= f * A[col][j];
    }
  }
  double x[17];
  for (int i = n - 1; i >= 0; --i) {
    double acc = A[i][n];
    for (int j = i + 1; j < n; ++j) acc -= A[i][j] * x[j];
    x[i] = acc / A[i][i];
  }
  for (int i = 0; i < m; ++i) {
    if (!std::isfinite(x[i])) return false;
    c[i] = x[i];
  }
  return true;
}

// ====================================================================== exported
extern "C" {

const char* green_strerror(int st) {
  switch (st) {
    case GREEN_OK: return "success";
    case GREEN_EINVAL: return "invalid argument";
    case GREEN_ENOMEM: return "workspace too small";
    case GREEN_EHIP: return "HIP runtime error";
    case GREEN_ESINGULAR: return "singular matrix in a batched inversion";
    case GREEN_ENOCONV: return "chemical potential not bracketed or not converged";
    case GREEN_ENAN: return "non-finite value";
    case GREEN_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

int green_plan_create(const green_dims* dims, const green_grid* grid, int prec, size_t chunk_bytes,
                      green_plan** out) {
  if (!dims || !grid || !out) return GREEN_EINVAL;
  *out = nullptr;
  const green_dims d = *dims;
  if (d.kmesh[0] < 1 || d.kmesh[1] < 1 || d.kmesh[2] < 1) return GREEN_EINVAL;
  if (d.nao < 1 || d.nao > 512 || d.naux < 1 || d.naux > 512) return GREEN_EINVAL;
  if (d.ntau < 4 || (d.ntau & 1) || d.nw_f != d.ntau || d.nw_b != d.ntau + 1) return GREEN_EINVAL;
  if (d.nspin != 1 && d.nspin != 2) return GREEN_EINVAL;
  if (!(d.beta > 0.0) || !std::isfinite(d.beta)) return GREEN_EINVAL;
  if (!grid->tau || !grid->wf || !grid->wb || !grid->TF_t2w || !grid->TF_w2t || !grid->TB_t2w || !grid->TB_w2t)
    return GREEN_EINVAL;
  if (prec != GREEN_FP64 && prec != GREEN_FP32 && prec != GREEN_BF16X3) return GREEN_EUNSUPPORTED;
  green_plan* p = new (std::nothrow) green_plan();
  if (!p) return GREEN_ENOMEM;
  p->d = d;
  p->nk = d.kmesh[0] * d.kmesh[1] * d.kmesh[2];
  p->prec = prec;
  const int nk = p->nk, ntau = d.ntau, nwf = d.nw_f, nwb = d.nw_b;
  p->tau.assign(grid->tau, grid->tau + ntau);
  p->wf.assign(grid->wf, grid->wf + nwf);
  p->wb.assign(grid->wb, grid->wb + nwb);
  auto cp = [](const void* src, size_t n, std::vector<double2>& dst) {
    dst.resize(n);
    std::memcpy(dst.data(), src, n * sizeof(double2));
  };
  cp(grid->TF_t2w, (size_t)nwf * ntau, p->TF_t2w);
  cp(grid->TF_w2t, (size_t)ntau * nwf, p->TF_w2t);
  cp(grid->TB_t2w, (size_t)nwb * ntau, p->TB_t2w);
  cp(grid->TB_w2t, (size_t)ntau * nwb, p->TB_w2t);
  for (int t = 0; t < ntau; ++t)
    if (std::fabs(p->tau[t] + p->tau[ntau - 1 - t] - d.beta) > 1e-10 * d.beta) {
      delete p;
      return GREEN_EINVAL;
    }
  if (!build_mass_matrix(p->tau, d.beta, p->Emass)) {
    delete p;
    return GREEN_EUNSUPPORTED;
  }
  p->kadd.resize((size_t)nk * nk);
  p->ksub.resize((size_t)nk * nk);
  p->kneg.resize(nk);
  for (int q = 0; q < nk; ++q) {
    int qa, qb, qc;
    kpoint(d.kmesh, q, qa, qb, qc);
    p->kneg[q] = kflat(d.kmesh, -qa, -qb, -qc);
    for (int k = 0; k < nk; ++k) {
      int a, b, c;
      kpoint(d.kmesh, k, a, b, c);
      p->kadd[(size_t)q * nk + k] = kflat(d.kmesh, a + qa, b + qb, c + qc);
      p->ksub[(size_t)q * nk + k] = kflat(d.kmesh, a - qa, b - qb, c - qc);
    }
  }
  for (int q = 0; q < nk; ++q)
    if (p->kneg[q] >= q) p->qcan.push_back(q);
  p->qslot.assign(nk, -1);
  for (size_t i = 0; i < p->qcan.size(); ++i) p->qslot[p->qcan[i]] = (int32_t)i;
  build_contracted_sets(p);
  // ---- workspace layout
  const int64_t nao = d.nao, naux = d.naux, ns = d.nspin;
  const int64_t nG = nao * nao, nV = naux * nG, nP = naux * naux;
  if (chunk_bytes == 0) chunk_bytes = (size_t)8 << 30;
  p->chunk_bytes = chunk_bytes;
  const size_t isz = prec == GREEN_FP64 ? 16 : 8;  // bytes of a stored contraction intermediate
  const size_t per_t = (size_t)2 * nk * nV * isz;
  int tc = (int)std::max<size_t>(1, chunk_bytes / per_t);
  tc = std::min(tc, ntau);
  p->tc = tc;
  // default tile of the split-BF16 P~0 contraction (naux x naux outputs): the least padded area, the
  // 192 x 96 tile (highest arithmetic intensity) counted at 90% of its area; 320 x 64 runs on the LDS-DMA
  // kernel where the operands allow it
  {
    static const int tile[4][2] = {{192, 96}, {192, 64}, {320, 64}, {448, 64}};
    double best = 0;
    for (int b = 0; b < 4; ++b) {
      const double a = (double)((naux + tile[b][0] - 1) / tile[b][0] * tile[b][0]) *
                       ((naux + tile[b][1] - 1) / tile[b][1] * tile[b][1]) * (b == 0 ? 0.9 : 1.0);
      if (b == 0 || a < best) {
        best = a;
        p->big_p0 = b + 1;
      }
    }
    if (p->big_p0 == 3) p->big_p0 = 5;
  }
  size_t off = 0;
  auto take = [&](Region& r, size_t bytes) {
    r.off = off;
    r.bytes = bytes;
    off += (bytes + 255) & ~(size_t)255;
  };
  take(p->r_TF_t2w, (size_t)nwf * ntau * 16);
  take(p->r_TF_w2t, (size_t)ntau * nwf * 16);
  take(p->r_TB_t2w, (size_t)nwb * ntau * 16);
  take(p->r_TB_w2t, (size_t)ntau * nwb * 16);
  take(p->r_Emass, (size_t)ntau * ntau * 16);
  take(p->r_wf, (size_t)nwf * 8);
  take(p->r_kadd, (size_t)nk * nk * 4);
  take(p->r_ksub, (size_t)nk * nk * 4);
  take(p->r_kneg, (size_t)nk * 4);
  take(p->r_kc, (size_t)nk * 4);
  take(p->r_ksubc, (size_t)nk * nk * 4);
  take(p->r_qc, (size_t)nk * 4);
  take(p->r_kfill, (size_t)nk * 4);
  take(p->r_status, 64);
  take(p->r_scal, 64 * 8);
  take(p->r_partial, 1024 * 8);
  take(p->r_P, (size_t)nk * ntau * nP * 16);
  take(p->r_Pw, p->qcan.size() * nwb * nP * 16);
  const size_t tbuf = std::max<size_t>((size_t)tc * nk * nV * isz, (size_t)ns * ntau * nk * nG * 16);
  take(p->r_T1, std::max<size_t>(tbuf, (size_t)nP * 16));
  take(p->r_T2, std::max<size_t>({(size_t)tc * nk * nV * isz, (size_t)nk * nV * 16, (size_t)nP * 16}));
  take(p->r_gam, (size_t)ns * nk * nG * 16);
  take(p->r_gamT, (size_t)ns * nk * nG * 16);
  take(p->r_D, (size_t)naux * 16);
  take(p->r_Sinfn, (size_t)ns * nk * nG * 16);
  take(p->r_Sign, (size_t)ns * ntau * nk * nG * 16);
  take(p->r_Sw, (size_t)ns * nwf * nk * nG * 16);
  take(p->r_A, (size_t)ns * nwf * nk * nG * 16);
  take(p->r_tr, (size_t)std::max<int64_t>(ns * nwf * nk, ns * ntau * nk) * 16);
  take(p->r_split, (size_t)1 << 30);
  p->fuse_sig = fusable(prec, (int)nao);
  // split BF16: two rounded V slabs (the second one with rows padded for the fused kernel)
  take(p->r_Vx, prec == GREEN_FP64 ? 0
                                   : prec == GREEN_BF16X3 ? (size_t)nk * naux * (nG + green::xgv_vblock((int)nao)) * 8
                                                          : (size_t)nk * nV * 8);
  take(p->r_Gx, prec == GREEN_BF16X3 ? (size_t)ns * ntau * nk * nG * 8 : 0);
  take(p->r_Ptx, prec == GREEN_BF16X3 ? (size_t)ntau * nP * 8 : 0);
  take(p->r_GTx, p->fuse_sig ? (size_t)ns * ntau * nk * nG * 8 : 0);
  // split BF16 with an even nao up to 80: G^T images of every (spin, t, k) for the direct stage-1 kernel
  take(p->r_Gimg, prec == GREEN_BF16X3 && green::vg1_ok((int)nao)
                      ? (size_t)ns * ntau * nk * green::vg1_image_units((int)nao) * 16 : 0);
  p->ws_bytes = off;
  if (count_ops(p) != GREEN_OK) {
    delete p;
    return GREEN_EINVAL;
  }
  *out = p;
  return GREEN_OK;
}

void green_plan_destroy(green_plan* p) {
  if (!p) return;
  drop_graph(p);
  for (auto& kv : p->tuner)
    for (hipEvent_t e : kv.second.ev) (void)hipEventDestroy(e);
  if (p->events)
    for (int i = 0; i < kNumEvents; ++i) (void)hipEventDestroy(p->ev[i]);
  delete static_cast<KernelClock*>(p->clock);
  delete p;
}

size_t green_workspace_bytes(const green_plan* p) { return p ? p->ws_bytes : 0; }

int green_gw_polarization(green_plan* p, const void* V, const void* G, void* P0, void* ws, void* stream) {
  GREEN_TRY(check_plan(p, ws));
  if (!V || !G || !P0) return GREEN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanScope scope(p);
  GREEN_TRY(ensure_bound(p, ws, s));
  GREEN_TRY(check_inputs(p, V, G, ws, s));
  return run_polarization(p, V, G, P0, ws, s);
}

int green_gw_screen(green_plan* p, const void* P0, void* Pt, void* ws, void* stream) {
  GREEN_TRY(check_plan(p, ws));
  if (!P0 || !Pt) return GREEN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanScope scope(p);
  GREEN_TRY(ensure_bound(p, ws, s));
  return run_screen(p, P0, Pt, ws, s);
}

int green_gw_selfenergy(green_plan* p, const void* V, const void* G, const void* Pt, void* Sigma, void* ws,
                        void* stream) {
  GREEN_TRY(check_plan(p, ws));
  if (!V || !G || !Pt || !Sigma) return GREEN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanScope scope(p);
  GREEN_TRY(ensure_bound(p, ws, s));
  GREEN_TRY(check_inputs(p, V, G, ws, s));
  return run_selfenergy(p, V, G, Pt, Sigma, ws, s);
}

int green_gf2_selfenergy(green_plan* p, const void* V, const void* G, void* Sigma, void* ws, void* stream) {
  GREEN_TRY(check_plan(p, ws));
  if (!V || !G || !Sigma || !p->gf2 || p->vhalf) return GREEN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanScope scope(p);
  GREEN_TRY(ensure_bound(p, ws, s));
  GREEN_TRY(check_inputs(p, V, G, ws, s));
  double2* P = at<double2>(ws, p->r_P);
  GREEN_TRY(run_polarization(p, V, G, P, ws, s));
  GREEN_TRY(run_selfenergy(p, V, G, P, Sigma, ws, s));
  return run_gf2_exchange(p, V, G, Sigma, ws, s);
}

int green_hf_static(green_plan* p, const void* V, const void* G, void* Sinf, void* ws, void* stream) {
  GREEN_TRY(check_plan(p, ws));
  if (!V || !G || !Sinf) return GREEN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanScope scope(p);
  GREEN_TRY(ensure_bound(p, ws, s));
  return run_hf(p, V, G, Sinf, ws, s);
}

int green_dyson(green_plan* p, const void* H0, const void* S, const void* Sinf, const void* Sigma, double n_target,
                double* mu, void* G, double* n_out, int32_t* evals_out, void* ws, void* stream) {
  GREEN_TRY(check_plan(p, ws));
  if (!H0 || !S || !Sinf || !Sigma || !mu || !G || !std::isfinite(*mu)) return GREEN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanScope scope(p);
  GREEN_TRY(ensure_bound(p, ws, s));
  return run_dyson(p, H0, S, Sinf, Sigma, n_target, mu, G, n_out, evals_out, ws, s);
}

int green_check_status(green_plan* p, void* ws, void* stream) {
  GREEN_TRY(check_plan(p, ws));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->bound_ws != ws) return GREEN_OK;  // nothing has run on this workspace
  return read_status(p, ws, s);
}

// ---------------------------------------------------------------- allocation-free Dyson
namespace {

// Device scratch of green_dyson_noalloc: every GPU the library runs on holds its own copy until the process
// ends, and every call on that GPU shares it.  In host code `scratch` names a host-side stand-in, never the
// device memory: its device address comes from hipGetSymbolAddress, once per device, and only that address
// reaches kernels and copies.
static __device__ __align__(256) unsigned char scratch[GREEN_NOALLOC_MAX_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's scratch (the current device; looked up on its first use).
int scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return GREEN_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GREEN_EHIP;
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return GREEN_OK;
}

// Byte offsets of the Dyson step's buffers inside the scratch (256-byte aligned).
struct NoallocLayout {
  size_t tf_t2w, tf_w2t, wf, sw, a, tr, scal, status, total;
};
NoallocLayout noalloc_layout(const green_plan* p) {
  const green_dims& d = p->d;
  const size_t nG = (size_t)d.nao * d.nao, nb = (size_t)d.nspin * d.nw_f * p->nk;
  NoallocLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  L.tf_t2w = take((size_t)d.nw_f * d.ntau * 16);
  L.tf_w2t = take((size_t)d.ntau * d.nw_f * 16);
  L.wf = take((size_t)d.nw_f * 8);
  L.sw = take(nb * nG * 16);
  L.a = take(nb * nG * 16);
  L.tr = take(nb * 16);
  L.scal = take(64 * 8);
  L.status = take(64);
  L.total = off;
  return L;
}

}  // namespace

int green_dyson_noalloc(green_plan* p, const void* H0, const void* S, const void* Sinf, const void* Sigma,
                        double n_target, double* mu, void* G, double* n_out, int32_t* evals_out, void* stream) {
  if (!p || !H0 || !S || !Sinf || !Sigma || !mu || !G || !std::isfinite(*mu)) return GREEN_EINVAL;
  const NoallocLayout L = noalloc_layout(p);
  if (L.total > (size_t)GREEN_NOALLOC_MAX_BYTES) return GREEN_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* base = nullptr;
  if (green::dryrun())
    base = reinterpret_cast<void*>((uintptr_t)1 << 40);  // validated against, never dereferenced
  else
    GREEN_TRY(scratch_address(&base));
  char* b = static_cast<char*>(base);
  DysonMem m;
  m.TF_t2w = reinterpret_cast<const double2*>(b + L.tf_t2w);
  m.TF_w2t = reinterpret_cast<const double2*>(b + L.tf_w2t);
  m.wf = reinterpret_cast<const double*>(b + L.wf);
  m.Sw = reinterpret_cast<double2*>(b + L.sw);
  m.A = reinterpret_cast<double2*>(b + L.a);
  m.tr = reinterpret_cast<double2*>(b + L.tr);
  m.scal = reinterpret_cast<double*>(b + L.scal);
  m.status = reinterpret_cast<int*>(b + L.status);
  m.sTF_t2w = green::Span{m.TF_t2w, (int64_t)(p->TF_t2w.size() * sizeof(double2))};
  m.sTF_w2t = green::Span{m.TF_w2t, (int64_t)(p->TF_w2t.size() * sizeof(double2))};
  m.sSw = green::Span{m.Sw, (int64_t)(L.a - L.sw)};
  m.sA = green::Span{m.A, (int64_t)(L.tr - L.a)};
  // no autotuner (its trials create events) and no split-K partial sums (no room for them)
  PlanScope scope(nullptr);
  struct SplitScope {
    SplitBuf saved;
    explicit SplitScope(int prec) : saved(tl_split) { tl_split = SplitBuf{nullptr, 0, prec}; }
    ~SplitScope() { tl_split = saved; }
  } split_scope(p->prec);
  if (!green::dryrun()) {
    // the scratch holds whatever the last call on this GPU left: the grid rows are copied in and the status
    // word cleared on every call
    HIP_TRY(hipMemcpyAsync(b + L.tf_t2w, p->TF_t2w.data(), p->TF_t2w.size() * sizeof(double2),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b + L.tf_w2t, p->TF_w2t.data(), p->TF_w2t.size() * sizeof(double2),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b + L.wf, p->wf.data(), p->wf.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(green::launch_zero(reinterpret_cast<double2*>(b + L.status), 4, s));
  }
  return run_dyson_in(p, m, H0, S, Sinf, Sigma, n_target, mu, G, n_out, evals_out, s);
}

// ---------------------------------------------------------------- k-path interpolation (Sec. 2.4)
// W[p][k] = (1/N_k) sum_R w(R) exp(2 pi i (khat_p - k) . R) over the R of the Born-von Karman supercell centred
// on 0; at an even mesh extent the zone-boundary term is split evenly between R = -n/2 and +n/2 (w = 1/2).
// The sum factorises over the three directions.
static void kpath_weights(const int32_t* mesh, const double* kfrac, int npath, std::vector<double2>& W) {
  const int nk = mesh[0] * mesh[1] * mesh[2];
  W.assign((size_t)npath * nk, make_double2(0.0, 0.0));
  std::vector<double2> f[3];
  for (int p = 0; p < npath; ++p) {
    for (int d = 0; d < 3; ++d) {
      const int n = mesh[d];
      f[d].assign(n, make_double2(0.0, 0.0));
      for (int m = 0; m < n; ++m) {
        double re = 0.0, im = 0.0;
        for (int R = -(n / 2); R <= n / 2; ++R) {
          const double w = (n % 2 == 0 && (R == n / 2 || R == -(n / 2))) ? 0.5 : 1.0;
          const double ph = 2.0 * M_PI * (kfrac[3 * p + d] - (double)m / n) * R;
          re += w * std::cos(ph);
          im += w * std::sin(ph);
        }
        f[d][m] = make_double2(re / n, im / n);
      }
    }
    for (int a = 0; a < mesh[0]; ++a)
      for (int b = 0; b < mesh[1]; ++b)
        for (int c = 0; c < mesh[2]; ++c) {
          const double2 x = f[0][a], y = f[1][b], z = f[2][c];
          const double2 xy = make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
          W[(size_t)p * nk + (a * mesh[1] + b) * mesh[2] + c] =
              make_double2(xy.x * z.x - xy.y * z.y, xy.x * z.y + xy.y * z.x);
        }
  }
}

int green_kpath_interpolate(green_plan* p, const double* kfrac, int npath, const void* Sinf, const void* Sigma,
                            void* Sinf_path, void* Sigma_path, void* ws, void* stream) {
  GREEN_TRY(check_plan(p, ws));
  if (!kfrac || npath <= 0 || !Sinf || !Sigma || !Sinf_path || !Sigma_path) return GREEN_EINVAL;
  for (int i = 0; i < 3 * npath; ++i)
    if (!std::isfinite(kfrac[i])) return GREEN_EINVAL;
  const green_dims& d = p->d;
  const int nk = p->nk, ns = d.nspin, ntau = d.ntau;
  const int64_t nG = (int64_t)d.nao * d.nao;
  if ((size_t)npath * nk * sizeof(double2) > p->r_T1.bytes) return GREEN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanScope scope(p);
  GREEN_TRY(ensure_bound(p, ws, s));
  std::vector<double2> W;
  kpath_weights(d.kmesh, kfrac, npath, W);
  double2* Wd = at<double2>(ws, p->r_T1);
  if (!green::dryrun()) {
    HIP_TRY(hipMemcpyAsync(Wd, W.data(), W.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  }
  const Extents ex = extents(p);
  const green::Span sW = span_ws(ws, p->r_T1);
  const int64_t pathG = (int64_t)npath * nG;
  // Sinf_path[s][p] = sum_k W[p][k] Sinf[s][k]
  GREEN_TRY(gemm(green::Site::Transform, "kpath.Sinf", op(Wd, flat(nk), flat(1), bnone()), sW,
                 op(Sinf, flat(nG), flat(1), bflat((int64_t)nk * nG)), span(Sinf, ex.H), Sinf_path,
                 span(Sinf_path, (int64_t)ns * pathG), flat(nG), flat(1), bflat(pathG), npath, (int)nG, nk, ns,
                 cplx(1), cplx(0), s));
  // Sigma_path[s][t][p] = sum_k W[p][k] Sigma~[s][t][k]
  GREEN_TRY(gemm(green::Site::Transform, "kpath.Sigma", op(Wd, flat(nk), flat(1), bnone()), sW,
                 op(Sigma, flat(nG), flat(1), bflat((int64_t)nk * nG)), span(Sigma, ex.Sig), Sigma_path,
                 span(Sigma_path, (int64_t)ns * ntau * pathG), flat(nG), flat(1), bflat(pathG), npath, (int)nG,
                 nk, ns * ntau, cplx(1), cplx(0), s));
  if (green::dryrun()) return GREEN_OK;
  HIP_TRY(hipStreamSynchronize(s));  // W lives in the workspace only for this call
  return GREEN_OK;
}

int green_gw_iterate(green_plan* p, const void* V, const void* H0, const void* S, void* G, void* Sinf, void* Sigma,
                     double* mu, double n_target, double alpha, green_report* rep, void* ws, void* stream) {
  GREEN_TRY(check_plan(p, ws));
  if (!V || !H0 || !S || !G || !Sinf || !Sigma || !mu || !rep || !std::isfinite(*mu)) return GREEN_EINVAL;
  if (!(alpha > 0.0 && alpha < 2.0)) return GREEN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanScope scope(p);
  GREEN_TRY(ensure_bound(p, ws, s));
  std::memset(rep, 0, sizeof(*rep));
  const bool dry = green::dryrun();
  GREEN_TRY(ensure_events(p));
  const MarkFn mark = [&](int i) { return dry ? hipSuccess : hipEventRecord(p->ev[i], s); };
  KernelClock* clk = nullptr;
  // the graph replays the Sigma evaluation once every contraction shape has its tuned kernel
  const bool graph = p->use_graph && !dry && s != nullptr && !tuning_pending(p);
  if (!dry && !graph) {
    if (!p->clock) p->clock = new (std::nothrow) KernelClock();
    clk = static_cast<KernelClock*>(p->clock);
    if (clk) clk->reset();
  }
  struct ClockScope {
    explicit ClockScope(KernelClock* c) { tl_clock = c; }
    ~ClockScope() { tl_clock = nullptr; }
  } clock_scope(clk);
  HIP_TRY(mark(0));
  if (graph) {
    const void* args[6] = {V, G, Sinf, Sigma, ws, nullptr};
    bool same = p->gexec != nullptr && p->galpha == alpha;
    for (int i = 0; i < 6 && same; ++i) same = p->gargs[i] == args[i];
    if (!same) {
      drop_graph(p);
      hipGraph_t gr = nullptr;
      HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      tl_capturing = true;
      const int st = sigma_eval(p, V, G, Sinf, Sigma, alpha, ws, s, nullptr);
      tl_capturing = false;
      const hipError_t ce = hipStreamEndCapture(s, &gr);
      if (st != GREEN_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return st;
      }
      if (ce != hipSuccess) return GREEN_EHIP;
      hipGraphExec_t ex = nullptr;
      if (hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return GREEN_EHIP;
      }
      p->graph = gr;
      p->gexec = ex;
      for (int i = 0; i < 6; ++i) p->gargs[i] = args[i];
      p->galpha = alpha;
    }
    HIP_TRY(hipGraphLaunch(p->gexec, s));
    for (int i = 1; i <= 4; ++i) HIP_TRY(mark(i));
  } else {
    GREEN_TRY(sigma_eval(p, V, G, Sinf, Sigma, alpha, ws, s, &mark));
  }
  HIP_TRY(mark(5));
  GREEN_TRY(close_iteration(p, H0, S, G, Sinf, Sigma, mu, n_target, rep, ws, s, &mark));
  if (dry) return GREEN_OK;
  for (int i = 0; i < 7; ++i) HIP_TRY(hipEventElapsedTime(&rep->ms[i], p->ev[i], p->ev[i + 1]));
  HIP_TRY(hipEventElapsedTime(&rep->ms[7], p->ev[0], p->ev[7]));
  if (clk)
    for (int slot = 0; slot < 2; ++slot) {
      GREEN_TRY(clk->read(slot, &rep->kern_ms[slot]));
      rep->kern_flops[slot] = clk->flops[slot];
      rep->kern_launches[slot] = clk->used[slot];
    }
  if (!std::isfinite(rep->e_tot) || !std::isfinite(rep->max_dsigma) || !std::isfinite(rep->herm_err))
    return GREEN_ENAN;
  return GREEN_OK;
}

size_t green_diis_history_bytes(const green_plan* p, int size) {
  if (!p || size < 2 || size > 16) return 0;
  const int64_t nG = (int64_t)p->d.nao * p->d.nao;
  const int64_t nv = (int64_t)p->d.nspin * p->nk * nG * (1 + p->d.ntau);  // Sigma^inf and Sigma~(tau)
  return (size_t)size * 2 * nv * sizeof(double2);
}

int green_gw_iterate_diis(green_plan* p, const void* V, const void* H0, const void* S, void* G, void* Sinf,
                          void* Sigma, double* mu, double n_target, double alpha, green_diis* dst, void* hist,
                          size_t hist_bytes, green_report* rep, void* ws, void* stream) {
  GREEN_TRY(check_plan(p, ws));
  if (!V || !H0 || !S || !G || !Sinf || !Sigma || !mu || !rep || !dst || !hist || !std::isfinite(*mu))
    return GREEN_EINVAL;
  if (!(alpha > 0.0 && alpha < 2.0)) return GREEN_EINVAL;
  if (dst->size < 2 || dst->size > 16 || dst->start < 0 || dst->count < 0 || dst->count > dst->size ||
      dst->next < 0 || dst->next >= dst->size || dst->iter < 0)
    return GREEN_EINVAL;
  if (hist_bytes < green_diis_history_bytes(p, dst->size)) return GREEN_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanScope scope(p);
  GREEN_TRY(ensure_bound(p, ws, s));
  std::memset(rep, 0, sizeof(*rep));
  const bool dry = green::dryrun();
  GREEN_TRY(ensure_events(p));
  const MarkFn mark = [&](int i) { return dry ? hipSuccess : hipEventRecord(p->ev[i], s); };
  HIP_TRY(mark(0));
  // Sigma[G]: x_n = (Sinf_new, Sigma_new) in the workspace, the caller's arrays still hold the input self-energy
  GREEN_TRY(sigma_eval(p, V, G, Sinf, Sigma, alpha, ws, s, &mark, false));
  const green_dims& d = p->d;
  const int64_t nG = (int64_t)d.nao * d.nao;
  const int64_t ninf = (int64_t)d.nspin * p->nk * nG, nsig = ninf * d.ntau, nv = ninf + nsig;
  double2* Sinfn = at<double2>(ws, p->r_Sinfn);
  double2* Sign = at<double2>(ws, p->r_Sign);
  double* scal = at<double>(ws, p->r_scal);
  double* part = at<double>(ws, p->r_partial);
  double2* Hb = static_cast<double2*>(hist);
  const int slot = dst->next;
  double2* x = Hb + (int64_t)slot * 2 * nv;  // x_n = [Sinf_new | Sigma_new]
  double2* r = x + nv;                        // r_n = x_n - (input self-energy)
  const int count = std::min(dst->count + 1, dst->size);
  // ring order, oldest first
  int slots[16];
  for (int j = 0; j < count; ++j) slots[j] = (slot - (count - 1) + j + dst->size) % dst->size;
  double brow[16] = {0.0};
  if (!dry) {
    HIP_TRY(hipMemcpyAsync(x, Sinfn, ninf * sizeof(double2), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(x + ninf, Sign, nsig * sizeof(double2), hipMemcpyDeviceToDevice, s));
    HIP_TRY(green::launch_sub(r, x, static_cast<const double2*>(Sinf), ninf, s));
    HIP_TRY(green::launch_sub(r + ninf, x + ninf, static_cast<const double2*>(Sigma), nsig, s));
    // new row of the Gram matrix, one fixed-order dot product per stored residual
    for (int j = 0; j < count; ++j) {
      const double2* rj = Hb + (int64_t)slots[j] * 2 * nv + nv;
      HIP_TRY(green::launch_dot_re(r, rj, nv, part, scal + 16 + j, s));
    }
    HIP_TRY(hipMemcpyAsync(brow, scal + 16, count * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  for (int j = 0; j < count; ++j) {
    dst->B[slot][slots[j]] = brow[j];
    dst->B[slots[j]][slot] = brow[j];
  }
  dst->count = count;
  dst->next = (slot + 1) % dst->size;
  const bool extrapolate = dst->iter >= dst->start && count >= 2;
  for (int j = 0; j < 16; ++j) dst->coef[j] = 0.0;
  if (extrapolate) {
    double Bm[16 * 16], c[16];
    for (int i = 0; i < count; ++i)
      for (int j = 0; j < count; ++j) Bm[i * 16 + j] = dst->B[slots[i]][slots[j]];
    if (!dry && !diis_solve(Bm, 16, count, c)) return GREEN_ESINGULAR;
    if (dry)
      for (int j = 0; j < count; ++j) c[j] = j == count - 1 ? 1.0 : 0.0;
    green::CombineCoefs cf{};
    cf.m = count;
    for (int j = 0; j < count; ++j) {
      cf.slot[j] = slots[j];
      cf.c[j] = c[j];
      dst->coef[j] = c[j];
    }
    if (!dry) {
      HIP_TRY(green::launch_combine(static_cast<double2*>(Sinf), Hb, 2 * nv, ninf, cf, nullptr, nullptr, s));
      HIP_TRY(green::launch_combine(static_cast<double2*>(Sigma), Hb + ninf, 2 * nv, nsig, cf, part, scal + 8, s));
    }
  } else if (!dry) {
    HIP_TRY(green::launch_mix(static_cast<double2*>(Sinf), Sinfn, alpha, ninf, nullptr, nullptr, s));
    HIP_TRY(green::launch_mix(static_cast<double2*>(Sigma), Sign, alpha, nsig, part, scal + 8, s));
  }
  dst->iter += 1;
  HIP_TRY(mark(5));
  GREEN_TRY(close_iteration(p, H0, S, G, Sinf, Sigma, mu, n_target, rep, ws, s, &mark));
  if (dry) return GREEN_OK;
  for (int i = 0; i < 7; ++i) HIP_TRY(hipEventElapsedTime(&rep->ms[i], p->ev[i], p->ev[i + 1]));
  HIP_TRY(hipEventElapsedTime(&rep->ms[7], p->ev[0], p->ev[7]));
  if (!std::isfinite(rep->e_tot) || !std::isfinite(rep->max_dsigma)) return GREEN_ENAN;
  return GREEN_OK;
}

int green_plan_set_option(green_plan* p, int option, int value) {
  if (!p) return GREEN_EINVAL;
  switch (option) {
    case GREEN_OPT_TUNE:
      if (value < 0 || value > 2) return GREEN_EINVAL;
      if (value == 2) p->tuner.clear();
      p->tune = value != 0;
      drop_graph(p);
      return GREEN_OK;
    case GREEN_OPT_GRAPH:
      if (value < 0 || value > 1) return GREEN_EINVAL;
      p->use_graph = value;
      if (!value) drop_graph(p);
      return GREEN_OK;
    case GREEN_OPT_P0_TILE:
      if (value < 1 || value > 13) return GREEN_EINVAL;
      p->big_p0 = value;
      drop_graph(p);
      return GREEN_OK;
    case GREEN_OPT_SIGMA_TILE:
      if (value < 1 || value > 13) return GREEN_EINVAL;
      p->big_sig = value;
      drop_graph(p);
      return GREEN_OK;
    case GREEN_OPT_STAGE1_TILE:
      if (value < 0 || value > 3) return GREEN_EINVAL;
      p->big_stage1 = value;
      drop_graph(p);
      return GREEN_OK;
    case GREEN_OPT_V_HALF:
      if (value < 0 || value > 1) return GREEN_EINVAL;
      if (value && p->gf2) return GREEN_EINVAL;
      if (value && p->r_Vh.bytes == 0) {
        const size_t bytes = (size_t)p->nk * p->d.naux * p->d.nao * p->d.nao * 16;
        p->r_Vh.off = p->ws_bytes;
        p->r_Vh.bytes = bytes;
        p->ws_bytes += (bytes + 255) & ~(size_t)255;
      }
      p->vhalf = value != 0;
      drop_graph(p);
      return count_ops(p);
    case GREEN_OPT_TIME_REVERSAL:
      if (value < 0 || value > 1) return GREEN_EINVAL;
      p->trev = value != 0;
      build_contracted_sets(p);
      drop_graph(p);
      return count_ops(p);
    case GREEN_OPT_GF2:
      if (value < 0 || value > 1) return GREEN_EINVAL;
      if (value && p->vhalf) return GREEN_EINVAL;
      if (value) enable_gf2(p);
      p->gf2 = value != 0;
      drop_graph(p);
      return count_ops(p);
    case GREEN_OPT_SIGMA_FUSED:
      if (value < 0 || value > 1) return GREEN_EINVAL;
      if (value && !fusable(p->prec, p->d.nao)) return GREEN_EINVAL;
      p->fuse_sig = value != 0;
      drop_graph(p);
      return GREEN_OK;
    default:
      return GREEN_EINVAL;
  }
}

int green_plan_set_kpoint_symmetry(green_plan* p, const int32_t* rot, int nops, int32_t* counts) {
  if (!p || nops < 0 || nops > GREEN_MAX_KPOINT_OPS || (nops > 0 && !rot)) return GREEN_EINVAL;
  const int nk = p->nk;
  const int32_t* m = p->d.kmesh;
  std::vector<int32_t> krot((size_t)nops * nk);
  for (int r = 0; r < nops; ++r) {
    const int32_t* R = rot + 9 * r;
    // well defined modulo the mesh: R maps m_j e_j into the lattice of mesh periods
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (((int64_t)R[3 * i + j] * m[j]) % m[i] != 0) return GREEN_EINVAL;
    std::vector<char> hit(nk, 0);
    for (int k = 0; k < nk; ++k) {
      int a, b, c;
      kpoint(m, k, a, b, c);
      int x[3];
      for (int i = 0; i < 3; ++i) {
        const int64_t v = (int64_t)R[3 * i] * a + (int64_t)R[3 * i + 1] * b + (int64_t)R[3 * i + 2] * c;
        x[i] = (int)(((v % m[i]) + m[i]) % m[i]);
      }
      const int img = kflat(m, x[0], x[1], x[2]);
      if (hit[img]) return GREEN_EINVAL;  // not one to one
      hit[img] = 1;
      krot[(size_t)r * nk + k] = img;
    }
  }
  // orbits of the generated group: k joined with R k for every operation, labelled by the smallest member
  std::vector<int32_t> root(nk);
  for (int k = 0; k < nk; ++k) root[k] = k;
  auto find = [&](int k) {
    while (root[k] != k) k = root[k] = root[root[k]];
    return k;
  };
  for (int r = 0; r < nops; ++r)
    for (int k = 0; k < nk; ++k) {
      const int a = find(k), b = find(krot[(size_t)r * nk + k]);
      if (a != b) root[std::max(a, b)] = std::min(a, b);
    }
  std::vector<int32_t> orb(nk);
  for (int k = 0; k < nk; ++k) orb[k] = find(k);
  if (nops > 0 && p->r_krot.bytes < krot.size() * 4) {
    const size_t bytes = (size_t)GREEN_MAX_KPOINT_OPS * nk * 4;
    p->r_krot.off = p->ws_bytes;
    p->r_krot.bytes = bytes;
    p->ws_bytes += (bytes + 255) & ~(size_t)255;
  }
  p->ksym = nops > 0;
  p->nrot = nops;
  p->krot.swap(krot);
  p->korb.swap(orb);
  build_contracted_sets(p);
  drop_graph(p);
  if (counts) {
    counts[0] = (int32_t)p->qc.size();
    counts[1] = (int32_t)p->kc.size();
  }
  return count_ops(p);
}

#ifndef GREEN_SOURCE_DIGEST
#define GREEN_SOURCE_DIGEST "unknown"
#endif
#ifndef GREEN_TARGET_ARCH
#define GREEN_TARGET_ARCH "unknown"
#endif
#define GREEN_STR2(x) #x
#define GREEN_STR(x) GREEN_STR2(x)
const char* green_build_info(void) {
  return "sources=" GREEN_SOURCE_DIGEST " arch=" GREEN_TARGET_ARCH " hip=" GREEN_STR(HIP_VERSION_MAJOR) "." GREEN_STR(
      HIP_VERSION_MINOR);
}

int green_plan_tuning_report(const green_plan* p, char* buf, size_t len) {
  if (!p || !buf || len == 0) return GREEN_EINVAL;
  std::string out;
  static const char* names[] = {"Generic", "P0_VG", "P0_VGrev", "P0_Contract", "Sig_PV", "Sig_XG", "Sig_YV",
                                "HF", "Transform", "GF2_VG", "GF2_Pair", "GF2_Contract"};
  for (const auto& kv : p->tuner) {
    const TuneKey& k = kv.first;
    const TuneEntry& e = kv.second;
    char line[256];
    const int site = k.v[0] >= 0 && k.v[0] <= 11 ? k.v[0] : 0;
    if (!e.done) {
      std::snprintf(line, sizeof(line), "%-12s M=%d N=%d K=%d batch=%d prec=%d: tuning (%d of %zu tried)\n",
                    names[site], k.v[1], k.v[2], k.v[3], k.v[4], k.v[5], e.trial, e.cands.size());
    } else {
      const TuneCand& c = e.cands[e.chosen];
      std::snprintf(line, sizeof(line),
                    "%-12s M=%d N=%d K=%d batch=%d prec=%d: shape=%d big=%d ksplit=%d band=%d %.1f us (default %.1f us)\n",
                    names[site], k.v[1], k.v[2], k.v[3], k.v[4], k.v[5], c.shape, c.big, c.ksplit, c.band,
                    1000.0 * e.ms[e.chosen], 1000.0 * e.ms[0]);
      out += line;
      // every candidate's time: shape/big/ksplit/band=us
      std::string all = "    candidates:";
      for (size_t i = 0; i < e.cands.size(); ++i) {
        char item[64];
        std::snprintf(item, sizeof(item), " %d/%d/%d/%d=%.0f", e.cands[i].shape, e.cands[i].big, e.cands[i].ksplit,
                      e.cands[i].band, 1000.0 * e.ms[i]);
        all += item;
      }
      all += "\n";
      out += all;
      continue;
    }
    out += line;
  }
  std::snprintf(buf, len, "%s", out.c_str());
  return out.size() + 1 > len ? GREEN_ENOMEM : GREEN_OK;
}

// ---------------------------------------------------------------- batched iteration
size_t green_batch_workspace_bytes(int nsys, green_plan* const* plans) {
  if (nsys <= 0 || !plans) return 0;
  size_t n = 0;
  for (int i = 0; i < nsys; ++i) {
    if (!plans[i]) return 0;
    n += (size_t)plans[i]->nops;
  }
  // one descriptor and one tile offset per recorded contraction, plus one closing offset per group
  return 256 + n * (sizeof(ZGemm) + 2 * sizeof(int64_t)) + 4096;
}

int green_batch_create(int nsys, green_plan* const* plans, const green_system* sys, double alpha, int use_graph,
                       void* batch_ws, size_t batch_ws_bytes, void* stream, green_batch** out) {
  if (!out) return GREEN_EINVAL;
  *out = nullptr;
  if (nsys <= 0 || !plans || !sys || !batch_ws) return GREEN_EINVAL;
  if (!(alpha > 0.0 && alpha < 2.0) || (use_graph != 0 && use_graph != 1)) return GREEN_EINVAL;
  if (batch_ws_bytes < green_batch_workspace_bytes(nsys, plans)) return GREEN_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool dry = green::dryrun();
  for (int i = 0; i < nsys; ++i) {
    const green_system& y = sys[i];
    GREEN_TRY(check_plan(plans[i], y.ws));
    if (!y.V || !y.H0 || !y.S || !y.G || !y.Sinf || !y.Sigma || !std::isfinite(y.mu)) return GREEN_EINVAL;
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i] || sys[j].ws == y.ws) return GREEN_EINVAL;  // systems need their own plan and workspace
  }
  std::unique_ptr<green_batch> bt(new (std::nothrow) green_batch());
  if (!bt) return GREEN_ENOMEM;
  bt->plans.assign(plans, plans + nsys);
  bt->sys.assign(sys, sys + nsys);
  bt->alpha = alpha;
  // 1. record the Sigma evaluation of every system
  bt->ops.resize(nsys);
  size_t rounds = 0;
  for (int i = 0; i < nsys; ++i) {
    PlanScope scope(plans[i]);
    GREEN_TRY(ensure_bound(plans[i], sys[i].ws, s));
    tl_rec = &bt->ops[i];
    const int st = sigma_eval(plans[i], sys[i].V, sys[i].G, sys[i].Sinf, sys[i].Sigma, alpha, sys[i].ws, s, nullptr);
    tl_rec = nullptr;
    GREEN_TRY(st);
    rounds = std::max(rounds, bt->ops[i].size());
  }
  // 2. schedule: round r holds the r-th launch of every system; its contractions are grouped by kernel variant
  std::vector<int64_t> starts;
  bt->groups.resize(rounds);
  for (size_t r = 0; r < rounds; ++r) {
    std::vector<int> pending;
    for (int i = 0; i < nsys; ++i) {
      const auto& ops = bt->ops[i];
      if (r < ops.size() && ops[r].is_gemm && ops[r].g.M > 0 && ops[r].g.N > 0) pending.push_back(i);
    }
    // a contraction whose tiles fill every CU at least twice runs as its own launch (the direct kernel keeps its
    // full rate); the others of the round share persistent launches per kernel variant
    {
      std::vector<int> rest;
      for (int i : pending) {
        const ZGemm& g = bt->ops[i][r].g;
        const int per_cu = green::zgemm_wgs_per_cu(g);
        if (green::zgemm_blocks(g) >= 2 * 256 * (int64_t)(per_cu ? per_cu : 4)) {
          BatchGroup gr{bt->descs.size(), 1, starts.size(), true};
          bt->descs.push_back(g);
          starts.push_back(0);
          starts.push_back(green::zgemm_blocks(g));
          bt->groups[r].push_back(gr);
        } else {
          rest.push_back(i);
        }
      }
      pending.swap(rest);
    }
    while (!pending.empty()) {
      const green::Variant v = green::zgemm_variant(bt->ops[pending[0]][r].g);
      BatchGroup gr{bt->descs.size(), 0, starts.size()};
      std::vector<int> rest;
      int64_t tiles = 0;
      starts.push_back(0);
      for (int i : pending) {
        const ZGemm& g = bt->ops[i][r].g;
        if (!green::same_variant(v, green::zgemm_variant(g))) {
          rest.push_back(i);
          continue;
        }
        bt->descs.push_back(g);
        tiles += green::zgemm_blocks(g);
        starts.push_back(tiles);
        gr.count += 1;
      }
      bt->groups[r].push_back(gr);
      pending.swap(rest);
    }
  }
  const size_t dbytes = (bt->descs.size() * sizeof(ZGemm) + 255) & ~(size_t)255;
  if (dbytes + starts.size() * sizeof(int64_t) > batch_ws_bytes) return GREEN_ENOMEM;
  char* base = static_cast<char*>(batch_ws);
  bt->ddesc = reinterpret_cast<ZGemm*>(base);
  bt->dstart = reinterpret_cast<int64_t*>(base + dbytes);
  if (!dry && !bt->descs.empty()) {
    HIP_TRY(hipMemcpyAsync(bt->ddesc, bt->descs.data(), bt->descs.size() * sizeof(ZGemm), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(bt->dstart, starts.data(), starts.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  bt->use_graph = use_graph && !dry && s != nullptr;
  if (!dry) {
    HIP_TRY(hipEventCreate(&bt->e0));
    HIP_TRY(hipEventCreate(&bt->e1));
  }
  *out = bt.release();
  return GREEN_OK;
}

int green_batch_iterate(green_batch* bt, green_system* sys, green_report* reps, void* stream) {
  if (!bt || !sys || !reps) return GREEN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool dry = green::dryrun();
  const int nsys = (int)bt->plans.size();
  for (int i = 0; i < nsys; ++i) {
    const green_system& a = sys[i];
    const green_system& b = bt->sys[i];
    if (a.V != b.V || a.H0 != b.H0 || a.S != b.S || a.G != b.G || a.Sinf != b.Sinf || a.Sigma != b.Sigma ||
        a.ws != b.ws || !std::isfinite(a.mu))
      return GREEN_EINVAL;  // the schedule was recorded for these buffers
    std::memset(&reps[i], 0, sizeof(green_report));
  }
  // replay round by round: one persistent launch per kernel variant, auxiliary launches per system
  auto replay = [&]() -> int {
    for (size_t r = 0; r < bt->groups.size(); ++r) {
      for (const BatchGroup& gr : bt->groups[r]) {
        if (gr.solo)
          HIP_TRY(green::zgemm(bt->descs[gr.first], s));
        else
          HIP_TRY(green::zgemm_group(bt->descs.data() + gr.first, (int)gr.count, bt->ddesc + gr.first,
                                     bt->dstart + gr.start_off, s));
      }
      for (int i = 0; i < nsys; ++i)
        if (r < bt->ops[i].size() && !bt->ops[i][r].is_gemm && !dry) HIP_TRY(bt->ops[i][r].aux(s));
    }
    return GREEN_OK;
  };
  for (int i = 0; i < nsys; ++i) GREEN_TRY(ensure_bound(bt->plans[i], sys[i].ws, s));
  if (!dry) HIP_TRY(hipEventRecord(bt->e0, s));
  if (bt->use_graph) {
    if (!bt->gexec) {
      hipGraph_t gr = nullptr;
      HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      tl_capturing = true;
      const int st = replay();
      tl_capturing = false;
      const hipError_t ce = hipStreamEndCapture(s, &gr);
      if (st != GREEN_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return st;
      }
      if (ce != hipSuccess) return GREEN_EHIP;
      if (hipGraphInstantiate(&bt->gexec, gr, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return GREEN_EHIP;
      }
      bt->graph = gr;
    }
    HIP_TRY(hipGraphLaunch(bt->gexec, s));
  } else {
    GREEN_TRY(replay());
  }
  if (!dry) HIP_TRY(hipEventRecord(bt->e1, s));
  // close every system's iteration: Dyson, chemical potential, energy
  for (int i = 0; i < nsys; ++i) {
    PlanScope scope(bt->plans[i]);
    GREEN_TRY(ensure_bound(bt->plans[i], sys[i].ws, s));
    GREEN_TRY(close_iteration(bt->plans[i], sys[i].H0, sys[i].S, sys[i].G, sys[i].Sinf, sys[i].Sigma, &sys[i].mu,
                              sys[i].n_target, &reps[i], sys[i].ws, s));
  }
  if (dry) return GREEN_OK;
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, bt->e0, bt->e1));
  for (int i = 0; i < nsys; ++i) {
    reps[i].ms[7] = ms;  // Sigma evaluation of the whole batch
    if (!std::isfinite(reps[i].e_tot) || !std::isfinite(reps[i].max_dsigma)) return GREEN_ENAN;
  }
  return GREEN_OK;
}

void green_batch_destroy(green_batch* bt) { delete bt; }

int green_gw_iterate_batched(int nsys, green_plan* const* plans, green_system* sys, double alpha,
                             green_report* reps, void* batch_ws, size_t batch_ws_bytes, void* stream) {
  if (nsys <= 0 || !plans || !sys || !reps) return GREEN_EINVAL;
  green_batch* bt = nullptr;
  GREEN_TRY(green_batch_create(nsys, plans, sys, alpha, 0, batch_ws, batch_ws_bytes, stream, &bt));
  const int st = green_batch_iterate(bt, sys, reps, stream);
  green_batch_destroy(bt);
  return st;
}

}  // extern "C"
