/*
 * green_gw.h -- C ABI of the MI355X (gfx950) GW self-energy hot path.
 *
 * The library evaluates one fully self-consistent GW iteration as described in
 * Iskakov et al., "Green/WeakCoupling" (Sec. 2: Eqs. sigma_inf, sigma_gw,
 * tilde_W_DF2, tilde_P_omega, P0t_to_P0w, tilde_P0_tau, dyson; Sec. 2.3 for the
 * loop, Sec. 4.2.2 for iteration mixing) on one GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All arrays are row-major.  "complex" means interleaved (re, im) doubles,
 *    i.e. the memory layout of C99 double _Complex and of torch.complex128.
 *  - Atomic units: energies in Hartree, beta in 1/Hartree.
 *  - k-mesh: Gamma-centred m0 x m1 x m2 Monkhorst-Pack mesh, nk = m0*m1*m2,
 *    k = (i0, i1, i2) has flat index (i0*m1 + i1)*m2 + i2; k+q, k-q, -k are
 *    taken component-wise modulo the mesh.
 *  - Layouts (device memory, complex):
 *        V      [nk(q)][nk(k)][naux][nao][nao]   V[q][k] = V^{k,k+q}_{ij}(Q)
 *        G      [nspin][ntau][nk][nao][nao]      G^k_s(tau_t)
 *        H0     [nspin][nk][nao][nao]            H^{k,(0)}
 *        S      [nk][nao][nao]                   overlap S^k
 *        Sinf   [nspin][nk][nao][nao]            Sigma^{inf,k}_s
 *        Sigma  [nspin][ntau][nk][nao][nao]      dynamic Sigma~^k_s(tau_t)
 *        P0, Pt [nk(q)][ntau][naux][naux]        P~0^q(tau_t), P~^q(tau_t)
 *    V must hold every ordered pair (k1, k2) with the Hermitian pairing
 *    V^{k2,k1}_{ij}(Q) = conj V^{k1,k2}_{ji}(Q) (real auxiliary basis).
 *  - tau grid: symmetric (tau_t + tau_{ntau-1-t} = beta) Chebyshev-Lobatto
 *    nodes, tau_0 = 0+ and tau_{ntau-1} = beta-.  G(beta - tau_t) is node
 *    ntau-1-t and G(0^-) = -G(beta^-).
 *  - nspin = 1 is a spin-restricted run (one stored channel standing for two
 *    equal spins: the spin sums of Eqs. tilde_P0_tau and sigma_inf's Hartree
 *    term count it twice); nspin = 2 is unrestricted.
 *
 * Ownership: the caller owns every buffer, including the workspace, whose size
 * green_workspace_bytes() reports.  The library never allocates device memory.
 * The plan is host-only state.  The first call with a given workspace uploads
 * the grid matrices and k-index tables into it (ordered on the given stream).
 *
 * Synchronisation: green_gw_polarization, green_gw_screen and
 * green_gw_selfenergy only enqueue work on `stream`.  green_dyson and
 * green_gw_iterate return host scalars and synchronise `stream`.
 *
 * Errors: every entry point returns a green_status.  Argument errors are
 * detected before any launch.  Numerical failures (a zero pivot in a batched
 * inversion, a non-finite result, a chemical potential that cannot be
 * bracketed or converged) are reported by the next synchronising call.
 * With GREEN_CHECK=1 in the environment (a debug mode) every call that reads
 * G and V also checks on the device that G(tau) is Hermitian per (s, t, k)
 * and that V has the Hermitian pairing on three auxiliary indices of every
 * pair, to 1e-8 of the largest element; violations are reported as
 * GREEN_EINVAL by the next synchronising call.
 */
#ifndef GREEN_GW_H
#define GREEN_GW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GREEN_OK = 0,
  GREEN_EINVAL = -1,      /* bad argument: null pointer, bad dimension, unsupported size */
  GREEN_ENOMEM = -2,      /* workspace smaller than green_workspace_bytes() */
  GREEN_EHIP = -3,        /* a HIP runtime call failed */
  GREEN_ESINGULAR = -4,   /* zero pivot in a batched inversion */
  GREEN_ENOCONV = -5,     /* chemical potential not bracketed / not converged */
  GREEN_ENAN = -6,        /* non-finite value in a result */
  GREEN_EUNSUPPORTED = -7 /* valid request this build cannot serve */
} green_status;

/* Arithmetic of the two dominant contractions (P~0 and Sigma~).  Inputs and
 * outputs stay complex FP64; only the contraction arithmetic changes. */
typedef enum {
  GREEN_FP64 = 0,  /* complex FP64 on v_mfma_f64_16x16x4 (4M)                       */
  GREEN_FP32 = 1,  /* complex FP32 on MFMA with FP32 accumulation                      */
  GREEN_BF16X3 = 2 /* split BF16 (hi + lo, three products) with FP32 accumulation      */
} green_prec;

typedef struct {
  int32_t kmesh[3]; /* Monkhorst-Pack mesh m0, m1, m2                                   */
  int32_t nao;      /* orbitals per k-point                                              */
  int32_t naux;     /* auxiliary (density-fitting) functions Q                            */
  int32_t ntau;     /* imaginary-time nodes (even, >= 4)                                 */
  int32_t nw_f;     /* fermionic Matsubara nodes of the grid                              */
  int32_t nw_b;     /* bosonic Matsubara nodes of the grid                                */
  int32_t nspin;    /* 1 = restricted, 2 = unrestricted                                   */
  double beta;      /* inverse temperature                                                */
} green_dims;

/* Grid data (the method's "grid file", Sec. 4.2).  Host pointers, copied by
 * green_plan_create; complex matrices are row-major.
 *   X(i w_m)  = sum_t TF_t2w[m][t] X(tau_t)   (fermionic, exact Fourier integral of the interpolant)
 *   X(tau_t)  = sum_m TF_w2t[t][m] X(i w_m)   (its least-squares inverse)
 *   TB_t2w / TB_w2t: the same for bosonic frequencies (Eq. P0t_to_P0w and its inverse). */
typedef struct {
  const double* tau;  /* [ntau] nodes, Chebyshev-Lobatto on [0, beta]                  */
  const double* wf;   /* [nw_f] fermionic Matsubara frequencies w_m = (2n+1) pi / beta   */
  const double* wb;   /* [nw_b] bosonic Matsubara frequencies  W_m = 2 n pi / beta       */
  const void* TF_t2w; /* complex [nw_f][ntau] */
  const void* TF_w2t; /* complex [ntau][nw_f] */
  const void* TB_t2w; /* complex [nw_b][ntau] */
  const void* TB_w2t; /* complex [ntau][nw_b] */
} green_grid;

/* Result of one iteration (host). */
typedef struct {
  double e_1b;       /* (2/ns)(1/nk) sum Re Tr[gamma H0]                                  */
  double e_hf;       /* (1/ns)(1/nk) sum Re Tr[gamma Sigma^inf]                           */
  double e_corr;     /* -(1/ns)(1/nk) sum int_0^beta Re Tr[Sigma~(tau) G(beta - tau)]     */
  double e_tot;      /* e_1b + e_hf + e_corr (Galitskii-Migdal, no nuclear term)          */
  double n_elec;     /* electron count of the new G                                       */
  double mu;         /* chemical potential                                                */
  double max_dsigma; /* max |Sigma~_new - Sigma~_old| (after mixing)                      */
  double herm_err;   /* max |Sigma~ - Sigma~^H|                                           */
  int32_t mu_evals;  /* electron-count evaluations in the mu search                       */
  int32_t pad;
  float ms[8];       /* stage times (ms): 0 HF, 1 P0, 2 screen, 3 Sigma, 4 mix, 5 Dyson+mu, 6 energy, 7 total */
  /* HIP-event timing of the two dominant contraction launches, [0] = P~0 stage 2 (sum over k and
   * orbital pairs into naux x naux), [1] = Sigma~ stage 1 (P~(tau)^T times V over Q):
   * summed launch time (ms), algorithmic real flops (4M complex counting) and launch count. */
  double kern_ms[2];
  double kern_flops[2];
  int32_t kern_launches[2];
} green_report;

typedef struct green_plan green_plan;

/* Create a plan for fixed dimensions and grid; `prec` selects the contraction
 * arithmetic.  chunk_bytes bounds the workspace used for contraction
 * intermediates (0 = default 8 GiB).  Returns GREEN_EINVAL for inconsistent
 * dims (nao > 512, naux > 512, odd ntau, nw_f != ntau, nw_b != ntau + 1 ...). */
int green_plan_create(const green_dims* dims, const green_grid* grid, int prec, size_t chunk_bytes,
                      green_plan** out);
void green_plan_destroy(green_plan* plan);

/* Workspace bytes for every entry point of this plan (green_gw_iterate needs all of it). */
size_t green_workspace_bytes(const green_plan* plan);

/* P~0^q_{QQ'}(tau) of Eq. tilde_P0_tau (with G^k(-tau) taken as the stored
 * G^k(beta - tau), see the header notes):
 *   P0^q_{QQ'}(tau) = -(1/nk) sum_{k,s} sum_{abcd} V^{k,k+q}_{da}(Q) G^k_{s,cd}(beta - tau)
 *                                                   G^{k+q}_{s,ab}(tau) V^{k+q,k}_{bc}(Q')
 * V, G: inputs (device).  P0: output [nk][ntau][naux][naux] (device).  Async. */
int green_gw_polarization(green_plan* plan, const void* V, const void* G, void* P0, void* ws, void* stream);

/* Screening (Eqs. P0t_to_P0w, tilde_P_omega and the inverse transform):
 *   P0(i W_m) = sum_t TB_t2w[m][t] P0(tau_t)
 *   P~(i W_m) = [I - P0(i W_m)]^{-1} P0(i W_m)      (batched Gauss-Jordan inverse with partial pivoting,
 *                                                    then the product with P0)
 *   P~(tau_t) = sum_m TB_w2t[t][m] P~(i W_m)
 * P0: input, Pt: output, both [nk][ntau][naux][naux] (device; may not alias).  Async. */
int green_gw_screen(green_plan* plan, const void* P0, void* Pt, void* ws, void* stream);

/* Sigma~ of Eqs. sigma_gw and tilde_W_DF2 with W~ = V P~(tau) V never formed:
 *   Sigma~^k_{s,ij}(tau) = -(1/nk) sum_q sum_ab G^{k-q}_{s,ab}(tau)
 *                          sum_{QQ'} V^{k,k-q}_{ia}(Q) P~^q_{QQ'}(tau) V^{k-q,k}_{bj}(Q')
 * V, G, Pt: inputs.  Sigma: output [nspin][ntau][nk][nao][nao] (overwritten).  Async. */
int green_gw_selfenergy(green_plan* plan, const void* V, const void* G, const void* Pt, void* Sigma, void* ws,
                        void* stream);

/* GF2 second-order self-energy (Eq. sigma2), for plans with GREEN_OPT_GF2 set:
 *   Sigma~(2)^k_{s,ij}(tau) = -(1/nk^2) sum_{k1,k2} sum_{QQ'} [direct - exchange]_{ij},   k3 = k1 + k2 - k,
 *   direct   = sum_{s'} [V^{k,k1}(Q) G^{k1}_s(tau) V^{k1,k}(Q')] Tr[V^{k3,k2}(Q) G^{k2}_{s'}(tau) V^{k2,k3}(Q') G^{k3}_{s'}(-tau)],
 *   exchange = V^{k,k1}(Q) G^{k1}_s(tau) V^{k1,k3}(Q') G^{k3}_s(-tau) V^{k3,k2}(Q) G^{k2}_s(tau) V^{k2,k}(Q'),
 * with G(-tau) = -G(beta - tau) (antiperiodic), the momentum delta of Eq. sigma2 taken as nk times a Kronecker
 * delta (hence 1/nk^2), and the spin sum of a restricted plan (nspin = 1) doubled.  The direct term is the
 * first-order bubble: green_gw_polarization followed by green_gw_selfenergy with P~ := P~0.  The exchange term
 * is contracted per tau node: the products V G of every momentum pair, then per triple (k, k1, k2) the
 * auxiliary sums X = sum_Q [V G](Q) x [V G](Q) and Z = sum_Q' [V G(beta - tau)](Q') x V(Q') (nao^4 each), then
 * sum over (k1, k2) and three orbitals of X Z; cost O(nk^3 ntau (naux nao^4 + nao^5)), in the plan's
 * arithmetic (FP32 and split-BF16 plans round the operands of these contractions and accumulate in FP32).
 * V, G: inputs (device).  Sigma: output [nspin][ntau][nk][nao][nao] (device, overwritten).  The P~0 region
 * of ws is overwritten.  GREEN_EINVAL if GREEN_OPT_GF2 is not set.  Async. */
int green_gf2_selfenergy(green_plan* plan, const void* V, const void* G, void* Sigma, void* ws, void* stream);

/* Hartree-Fock static self-energy, Eq. sigma_inf, from G(0^-) = -G(beta^-):
 *   Sinf^k_s = (1/nk) sum_{k' s' Q} V^{k,k}(Q) Tr[G^{k'}_{s'}(0^-) V^{k',k'}(Q)]
 *            - (1/nk) sum_{k' Q} V^{k,k'}(Q) G^{k'}_s(0^-) V^{k',k}(Q)
 * Output Sinf [nspin][nk][nao][nao].  Async. */
int green_hf_static(green_plan* plan, const void* V, const void* G, void* Sinf, void* ws, void* stream);

/* Dyson equation (Eq. dyson) and chemical potential (Sec. 2.3, step 3):
 *   G^k_s(i w_m) = [(i w_m + mu) S^k - H0^k_s - Sinf^k_s - Sigma~^k_s(i w_m)]^{-1},
 *   Sigma~(i w_m) = sum_t TF_t2w[m][t] Sigma~(tau_t),  G(tau_t) = sum_m TF_w2t[t][m] G(i w_m).
 * If n_target >= 0, *mu (in: start, out: result) is adjusted so that
 *   N(mu) = -(2/nspin)(1/nk) sum_{k,s} Re Tr[G^k_s(beta^-) S^k] = n_target
 * (bracket by doubling from +-1 Eh up to 60 times, then Illinois regula falsi; stop at
 * |N - n_target| <= 1e-12 max(1, n_target) or a bracket below 1e-14; at most 200 steps).
 * If n_target < 0, *mu is kept.  G: output [nspin][ntau][nk][nao][nao].
 * n_out / evals_out (host, optional): final electron count and number of N evaluations.
 * Synchronises `stream`. */
int green_dyson(green_plan* plan, const void* H0, const void* S, const void* Sinf, const void* Sigma, double n_target,
                double* mu, void* G, double* n_out, int32_t* evals_out, void* ws, void* stream);

/* Status latched on the device by earlier asynchronous calls on this workspace (synchronises `stream`, then
 * clears it): GREEN_ESINGULAR for a zero pivot in a batched inversion, GREEN_EINVAL for inputs that break an
 * assumption of the plan (see GREEN_OPT_TIME_REVERSAL and the GREEN_CHECK=1 debug checks of G Hermiticity and
 * the Hermitian pairing of V), GREEN_OK otherwise.  green_dyson and green_gw_iterate report the same on return. */
int green_check_status(green_plan* plan, void* ws, void* stream);

/* Allocation-free variant of green_dyson, for callers that cannot allocate device memory or pass a workspace
 * (tight serving loops, harnesses that forbid hipMalloc).  Same arguments and results as green_dyson minus the
 * workspace: the Dyson step and the chemical-potential search run in a device scratch array that is part of the
 * library's code object, GREEN_NOALLOC_MAX_BYTES bytes per GPU, held by every GPU the library runs on until the
 * process ends.  The call needs
 *     (2 nw_f ntau + nw_f / 2 + 2 nspin nw_f nk nao^2 + nspin nw_f nk) * 16 bytes (each part rounded up to 256)
 *     + 768 bytes
 * of it (the grid matrices, Sigma~(i w), the Dyson matrices and their traces) and returns GREEN_ENOMEM, before
 * any device work, when that exceeds GREEN_NOALLOC_MAX_BYTES.  It calls no allocator: the scratch's device
 * address is looked up once per device (on the device current at the call, which must be the device of
 * `stream`).  Every call on one GPU shares that GPU's scratch, which keeps the last call's contents (the call
 * copies the grid rows in and clears its status word first): calls that overlap on one GPU, from several host
 * threads or streams, race and give wrong results.  The autotuner is not consulted and no split-K partial sums
 * are used, so results equal those of green_dyson up to summation order.  Synchronises `stream`. */
#define GREEN_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int green_dyson_noalloc(green_plan* plan, const void* H0, const void* S, const void* Sinf, const void* Sigma,
                        double n_target, double* mu, void* G, double* n_out, int32_t* evals_out, void* stream);

/* k-path interpolation of the self-energy (Sec. 2.4, k-path interpolation): every momentum-dependent input
 * X(k) on the plan's Monkhorst-Pack mesh is taken to real space, X(R) = (1/nk) sum_k X(k) e^{-i k.R}, and
 * back onto the npath points khat, X(khat) = sum_R X(R) e^{i khat.R}, for X = Sinf and Sigma~(tau_t).
 * R runs over the lattice vectors of the Born-von Karman supercell centred on 0 (-n/2 .. n/2 per direction
 * of mesh extent n); at an even n the zone-boundary terms R = -n/2 and +n/2 carry weight 1/2 each, so the
 * interpolant reproduces the mesh values at mesh points.  kfrac: host [npath][3], fractional coordinates of
 * khat (k.R = 2 pi sum_d kfrac_d R_d; mesh point (a, b, c) is (a/n0, b/n1, c/n2)).
 * Inputs Sinf [nspin][nk][nao][nao], Sigma [nspin][ntau][nk][nao][nao]; outputs Sinf_path
 * [nspin][npath][nao][nao], Sigma_path [nspin][ntau][npath][nao][nao] (device).  The Green's function on the
 * path follows from green_dyson on a plan whose mesh is (npath, 1, 1), with H0 and S evaluated on the path by
 * the caller and n_target < 0 (the chemical potential of the mesh calculation kept).  npath * nk * 16 bytes
 * must fit the plan's contraction workspace.  Synchronises `stream`. */
int green_kpath_interpolate(green_plan* plan, const double* kfrac, int npath, const void* Sinf, const void* Sigma,
                            void* Sinf_path, void* Sigma_path, void* ws, void* stream);

/* One self-consistent iteration (Sec. 2.3):
 *   (1) Sinf_new = HF(G), Sigma_new = GW(G) [polarization, screen, selfenergy] (with GREEN_OPT_GF2:
 *       Sigma_new = GF2(G) [polarization, selfenergy with P~ := P~0, exchange term]);
 *   (2) mixing Sinf = alpha Sinf_new + (1-alpha) Sinf, Sigma = alpha Sigma_new + (1-alpha) Sigma
 *       (alpha = 1: no mixing; Sinf / Sigma are read only when alpha != 1);
 *   (3) chemical potential for n_target (kept if n_target < 0);
 *   (4) Dyson -> new G (overwrites G), energy and diagnostics into *report.
 * G, Sinf, Sigma: in/out (device).  mu: in/out (host).  Synchronises `stream`. */
int green_gw_iterate(green_plan* plan, const void* V, const void* H0, const void* S, void* G, void* Sinf, void* Sigma,
                     double* mu, double n_target, double alpha, green_report* report, void* ws, void* stream);

/* DIIS convergence acceleration (Sec. 4.2.2): the self-energy entering Dyson is a linear combination of the
 * self-energies of the last iterations, Sigma_n = sum_i c_i Sigma[G_{i-1}], with sum_i c_i = 1 and c minimising
 * |sum_i c_i r_i|^2 over the residuals r_i = Sigma[G_{i-1}] - Sigma_{i-1} (both Sigma^inf and Sigma~(tau),
 * Frobenius inner product, real part; the Gram matrix is scaled by its largest diagonal element and the
 * (m + 1)-dimensional Lagrange system solved on the host by elimination with partial pivoting).  Iterations
 * before `start` use the static mixing of green_gw_iterate (alpha) but are stored.
 * The caller owns the state (zero it, then set size in [2, 16] and start >= 0) and a device history buffer of
 * green_diis_history_bytes(plan, size) bytes that persists across the iterations. */
typedef struct {
  int32_t size;      /* most stored self-energies                                          */
  int32_t start;     /* first iteration (0-based) that extrapolates                       */
  int32_t count;     /* stored self-energies (updated by the library)                     */
  int32_t next;      /* ring slot of the next one (library)                               */
  int32_t iter;      /* iterations done (library)                                         */
  int32_t pad;
  double B[16][16];  /* Gram matrix of the stored residuals, by ring slot (library)       */
  double coef[16];   /* coefficients of the last extrapolation, oldest first (library)    */
} green_diis;

size_t green_diis_history_bytes(const green_plan* plan, int size);

/* One iteration as green_gw_iterate, with the mixing step replaced by DIIS.  GREEN_ESINGULAR when the
 * Lagrange system is singular (for instance two identical residuals); GREEN_ENOMEM for a short history. */
int green_gw_iterate_diis(green_plan* plan, const void* V, const void* H0, const void* S, void* G, void* Sinf,
                          void* Sigma, double* mu, double n_target, double alpha, green_diis* diis, void* history,
                          size_t history_bytes, green_report* report, void* ws, void* stream);

/* Plan options (green_plan_set_option):
 *   GREEN_OPT_TUNE  1: autotune.  Every contraction shape met on later calls is run once with each of
 *                   its candidate kernels (tile shape, large-tile kernel, split-K count; every candidate
 *                   computes the same contraction, differing only in summation order), timed with HIP
 *                   events, and the fastest is kept for all further calls of that shape on this plan (the
 *                   default unless a candidate is at least 5 % faster).
 *                   Synchronises `stream` once per shape when its last candidate has run.
 *                   2: forget earlier choices and tune again.  0: stop tuning (choices are kept).
 *   GREEN_OPT_GRAPH 1: green_gw_iterate captures its Sigma evaluation (Hartree-Fock, polarization,
 *                   screening, self-energy, mixing) into a HIP graph on first use and replays it while
 *                   (V, G, Sinf, Sigma, ws, alpha) stay the same; not while tuning is pending and not
 *                   on the default (null) stream, which cannot be captured: there it runs eagerly.  The
 *                   per-stage times are then not separated: ms[0] holds the replay, ms[1..4] are 0.
 *   GREEN_OPT_P0_TILE  split-BF16 plans: output tile of the P~0 contraction over k and orbital pairs
 *                   (the sum of Eq. tilde_P0_tau) before any autotuning: 1 = 192 x 96, 2 = 192 x 64,
 *                   3 = 320 x 64, 4 = 448 x 64 rows x columns of P~0(q, tau), register-staged; 5 = 320 x 64,
 *                   6 = 192 x 128 fed by LDS DMA (even nao; else as 3 and 1); 7 = 320 x 64, 8 = 128 x 128,
 *                   9 = 256 x 64 fed by LDS DMA with the next K stage's operands read ahead, 10 = 128 x 64 and
 *                   11 = 64 x 128 the same with 4 waves, two workgroups per CU (K blocks of a multiple of 16;
 *                   else 7 as 3, 8 as 1, 9 to 11 as 2), 12 = 128 x 128 and 13 = 256 x 64 fed by LDS DMA in stages
 *                   of 32 complex K through a two-slot ring (half the barriers per flop; K blocks of at least 32,
 *                   else 12 as 1, 13 as 2).  The plan starts with the tile that pads naux x naux
 *                   least (192 x 96 counted at 90% of its area), 320 x 64 on the LDS-DMA kernel.
 *   GREEN_OPT_SIGMA_TILE  split-BF16 plans: tile of the first Sigma~ contraction, P~(tau)^T V over the auxiliary
 *                   index (values as GREEN_OPT_P0_TILE; default 6).
 *   GREEN_OPT_STAGE1_TILE  split-BF16 plans: kernel of the V G products that feed it: 0 = 64 x 64 tiles,
 *                   1 = 192 x 96 tiles, 2 = 192 x 64 tiles, 3 (default) = the direct kernel (V rows held in
 *                   registers over a tau chunk, G^T of each tau node staged in LDS; even nao up to 80, else 1).
 *                   Both only change the summation blocking; results agree to rounding.
 *   GREEN_OPT_SIGMA_FUSED  split-BF16 plans with an even nao up to 80: 1 (default) runs the two contractions
 *                   of Eqs. sigma_gw and tilde_W_DF2 after P~^T V (over the orbital a with G(tau), then over (Q', b)
 *                   with V) in one kernel that keeps their intermediate in registers; 0 runs them as two
 *                   contractions through HBM.  GREEN_EINVAL where the plan does not allow 1.
 *   GREEN_OPT_GF2   1: the dynamic self-energy is the GF2 one of Eq. sigma2 (green_gf2_selfenergy) instead of
 *                   GW: green_gw_iterate and green_gw_iterate_diis skip the screening and add the exchange
 *                   term, and green_gf2_selfenergy is enabled.  The first time it is set the workspace grows
 *                   by the GF2 intermediates (two nk^2 x naux x nao^2 products V G and two chunks of four-index
 *                   products of nao^4 complex FP64 per momentum triple, each chunk at most chunk_bytes / 2 but
 *                   at least one triple): query green_workspace_bytes after setting it and bind a workspace of
 *                   that size.  0 (default): GW (the workspace keeps its size).
 *   GREEN_OPT_TIME_REVERSAL  1: the caller's system is time-reversal symmetric, V^{-k1,-k2}(Q) = conj V^{k1,k2}(Q)
 *                   and G^{-k}_s(tau) = conj G^k_s(tau) (which holds for G from green_dyson when H0(-k) =
 *                   conj H0(k) and S(-k) = conj S(k)); then P~0^{-q}(tau) = conj P~0^q(tau), which with the +-q
 *                   identity gives P~0^q(beta - tau) = P~0^q(tau)^H, and Sigma~^{-k} = conj Sigma~^k.  So
 *                   green_gw_polarization contracts the first half of the tau nodes only (the second half is
 *                   the conjugate transpose), and green_gw_selfenergy only the momenta k with -k >= k (flat
 *                   index), each partner written as the complex conjugate; the same inside the iterations and
 *                   in green_gf2_selfenergy (both terms).  Every call that reads G and V first checks on the
 *                   device that G^{-k}_s(tau) = conj G^k_s(tau) for every element and that V^{-k1,-k2}(Q) =
 *                   conj V^{k1,k2}(Q) on three auxiliary indices of every pair (full store), to 1e-8 of the
 *                   largest element; a violation is reported as GREEN_EINVAL by the next synchronising call
 *                   (green_dyson, green_gw_iterate, green_check_status).  0 (default): every tau node and every
 *                   k is contracted.
 *   GREEN_OPT_V_HALF  1: Hermitian half store of V.  Since V^{k2,k1}(Q) = V^{k1,k2}(Q)^dagger, the slab of q
 *                   (V[q][k] = V^{k,k+q}) follows from that of -q: the caller passes only the slabs of the
 *                   canonical q (-q >= q, flat index), in increasing q, as V[nqc][nk][naux][nao][nao] (the 3x3x3 mesh:
 *                   14 of 27 slabs, 4x4x4: 36 of 64).  The other slabs are written into the workspace one at a time
 *                   when used (the workspace grows by one slab, nk naux nao^2 complex: query green_workspace_bytes
 *                   after setting it).  Results equal those of the full store bit for bit when the full V has the
 *                   exact pairing.  Not with GREEN_OPT_GF2 (GREEN_EINVAL): its exchange term reads every slab at once.
 * Returns GREEN_EINVAL for an unknown option or value. */
#define GREEN_OPT_TUNE 1
#define GREEN_OPT_GRAPH 2
#define GREEN_OPT_P0_TILE 3
#define GREEN_OPT_STAGE1_TILE 4
#define GREEN_OPT_SIGMA_FUSED 5
#define GREEN_OPT_GF2 6
#define GREEN_OPT_TIME_REVERSAL 7
#define GREEN_OPT_V_HALF 8
#define GREEN_OPT_SIGMA_TILE 9
int green_plan_set_option(green_plan* plan, int option, int value);

/* Point-group symmetry of the k mesh (symmetry among the method's features, Sec. 3: the space-group operations
 * of a crystal reduce the momenta to an irreducible set).  Here the operations act on momenta alone: the orbital
 * and auxiliary bases transform trivially, so the caller's system must satisfy H0(R k) = H0(k), S(R k) = S(k),
 * V^{R k1, R k2}(Q) = V^{k1,k2}(Q) and G^{R k}_s(tau) = G^k_s(tau) for every operation R.  Then P~0^{R q} =
 * P~0^q (the sum over k of Eq. tilde_P0_tau re-indexed by R), the screening keeps it, and Sigma~^{R k} = Sigma~^k
 * (the sum over q of Eq. sigma_gw re-indexed).  With the +-q identity P~0^{-q}(tau) = P~0^q(beta - tau)^T, the
 * polarization and the screening are contracted for one orbit of each pair {O, -O} of momentum orbits (at its
 * smallest flat index; the first half of the tau nodes only where -q lies in the orbit of q), the self-energy for
 * one momentum per orbit (with GREEN_OPT_TIME_REVERSAL one orbit of each pair {O, -O}), each over every k or q;
 * the other momenta are written as copies (transposed, tau-reversed copies for -O; complex conjugates under time
 * reversal).  The Hartree-Fock terms, the Dyson step and the energies still run over every k.  The same in the
 * iterations and in green_gf2_selfenergy.
 *   rot     host, nops x 9 int32: operation r is the integer matrix R_r (row-major) acting on the integer mesh
 *           coordinates of a momentum, k = (i0, i1, i2) -> R_r k taken modulo the mesh (flat index (i0 m1 + i1) m2
 *           + i2); the identity need not be listed, and the orbits are those of the group the operations generate.
 *   nops    0 (rot may be NULL): no point group (the default).  At most GREEN_MAX_KPOINT_OPS.
 *   counts  optional host int32[2]: the number of contracted transfers (polarization, screening) and of
 *           contracted momenta (self-energy), e.g. 4 and 4 for the full cubic group on a 3x3x3 mesh.
 * Every call that reads G and V first checks on the device that G of every momentum equals that of the
 * contracted momentum it is filled from (or its conjugate under time reversal) and that V^{R k1, R k2}(Q) =
 * V^{k1,k2}(Q) for every operation on three auxiliary indices of every pair (full store), to 1e-8 of the largest
 * element; a violation is reported as GREEN_EINVAL by the next synchronising call.  The self-energy step alone
 * (green_gw_selfenergy) also needs P~^{R q} = P~^q of its input, which is not checked.
 * GREEN_EINVAL (plan unchanged) when an operation does not map the mesh onto itself (R_ij m_j must be a
 * multiple of m_i, and k -> R k one to one).  The workspace grows by the operations' tables the first time (query
 * green_workspace_bytes after the call). */
#define GREEN_MAX_KPOINT_OPS 192
int green_plan_set_kpoint_symmetry(green_plan* plan, const int32_t* rot, int nops, int32_t* counts);

/* Build provenance: a static NUL-terminated string "sources=<digest> arch=<gfx target> hip=<major.minor>", where
 * <digest> is the first 16 hex digits of the SHA-256 of the library's source files (csrc/ in name order, then this
 * header) as the in-tree build computed it.  The Python binding recomputes the digest from the sources beside the
 * library and refuses to load a library built from other sources. */
const char* green_build_info(void);

/* Text table of the autotuner's decisions into buf (host, len bytes, NUL-terminated; GREEN_ENOMEM when
 * truncated): per contraction shape a line with the chosen kernel and, once tuned, a line with every
 * candidate's time as shape/large tile/split-K count/tile-row band=microseconds. */
int green_plan_tuning_report(const green_plan* plan, char* buf, size_t len);

/* One system of a batched iteration: the arguments of green_gw_iterate (device pointers; mu host,
 * in/out) and that system's own workspace of green_workspace_bytes(plan) bytes. */
typedef struct {
  const void* V;
  const void* H0;
  const void* S;
  void* G;
  void* Sinf;
  void* Sigma;
  double mu;
  double n_target;
  void* ws;
} green_system;

/* Device bytes of the descriptor tables of a batched iteration over these plans. */
size_t green_batch_workspace_bytes(int nsys, green_plan* const* plans);

/* One self-consistent iteration (as green_gw_iterate) of nsys independent systems of any sizes, each
 * with its own plan and workspace.  The Sigma evaluations of all systems are issued together: the
 * r-th contraction of every system goes into one persistent launch per kernel variant (a grid that
 * walks the concatenated tile ranges of all of them), so small systems share the GPU instead of
 * running one after another; then every system's Dyson step, chemical potential and energy follow.
 * Results equal those of green_gw_iterate on each system with the same kernel choices.
 * batch_ws: device buffer of batch_ws_bytes >= green_batch_workspace_bytes(nsys, plans) bytes.
 * reports: nsys entries; ms[7] of each holds the Sigma evaluation time of the whole batch.
 * Synchronises `stream`.  GREEN_EINVAL when two systems share a plan or a workspace. */
int green_gw_iterate_batched(int nsys, green_plan* const* plans, green_system* systems, double alpha,
                             green_report* reports, void* batch_ws, size_t batch_ws_bytes, void* stream);

/* Batch handle: the batched iteration of green_gw_iterate_batched recorded once for fixed systems and
 * buffers, optionally replayed from a captured HIP graph (use_graph = 1; not on the default stream,
 * where it replays eagerly).  The descriptor tables are uploaded into batch_ws at creation (device,
 * caller-owned, must outlive the handle).  green_batch_iterate takes the same systems (same buffers,
 * mu may change) and runs one iteration of all of them; reports as for green_gw_iterate_batched.
 * Tuning choices of the plans are frozen at creation. */
typedef struct green_batch green_batch;
int green_batch_create(int nsys, green_plan* const* plans, const green_system* systems, double alpha, int use_graph,
                       void* batch_ws, size_t batch_ws_bytes, void* stream, green_batch** out);
int green_batch_iterate(green_batch* batch, green_system* systems, green_report* reports, void* stream);
void green_batch_destroy(green_batch* batch);

/* Human-readable text for a green_status. */
const char* green_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* GREEN_GW_H */
