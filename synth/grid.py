"""Imaginary-time / Matsubara grid data (the stand-in for the method's grid file).

The method takes its non-uniform imaginary-time grid and the matching
Matsubara-frequency transforms from an external grid file (Sec. 4.2, the
``--grid_file`` option, with IR and Chebyshev grids shipped).  Those files are
not available here, so this module builds an equivalent Chebyshev grid as
*input data*; nothing in it evaluates the self-energy method itself.

Grid (Chebyshev-Lobatto, symmetric):
    tau_t = beta/2 * (1 - cos(pi t / (ntau-1))),   t = 0 .. ntau-1
so tau_0 = 0, tau_{ntau-1} = beta and tau_t + tau_{ntau-1-t} = beta.

A function on the grid stands for its degree-(ntau-1) polynomial interpolant
p(tau) = sum_l c_l T_l(x), x = 2 tau / beta - 1.  The forward transforms are
exact Fourier integrals of that interpolant (Eq. P0t_to_P0w for the bosonic
case, the same integral with fermionic frequencies for G and Sigma):
    X(i nu) = int_0^beta p(tau) e^{i nu tau} dtau
            = beta/2 e^{i nu beta/2} sum_l c_l I_l(nu beta/2),
    I_l(a)  = int_{-1}^{1} T_l(x) e^{i a x} dx.
Fermionic nu = (2n+1) pi / beta, bosonic nu = 2 n pi / beta.

Sparse Matsubara nodes: positive candidates n < 300 plus 400 log-spaced values
up to 2e4 are ranked by greedy pivoted Gram-Schmidt on the real form of the
transform rows; ntau/2 positive nodes are kept and mirrored to +-.  Fermionic
grids have nw_f = ntau nodes; bosonic grids add Omega_0 = 0, nw_b = ntau + 1.
The inverse maps (frequency -> tau) are the least-squares pseudo-inverses.
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np
from scipy.special import jv


@dataclasses.dataclass(frozen=True)
class Grid:
    beta: float
    tau: np.ndarray  # [ntau]
    nf: np.ndarray  # [nw_f] fermionic Matsubara integers n  (omega = (2n+1) pi / beta)
    nb: np.ndarray  # [nw_b] bosonic Matsubara integers n    (Omega = 2 n pi / beta)
    TF_t2w: np.ndarray  # [nw_f, ntau] complex
    TF_w2t: np.ndarray  # [ntau, nw_f] complex
    TB_t2w: np.ndarray  # [nw_b, ntau] complex
    TB_w2t: np.ndarray  # [ntau, nw_b] complex

    @property
    def ntau(self) -> int:
        return int(self.tau.shape[0])

    @property
    def wf(self) -> np.ndarray:
        return (2 * self.nf + 1) * np.pi / self.beta

    @property
    def wb(self) -> np.ndarray:
        return 2 * self.nb * np.pi / self.beta


def lobatto_tau(ntau: int, beta: float) -> np.ndarray:
    t = np.arange(ntau)
    tau = 0.5 * beta * (1.0 - np.cos(np.pi * t / (ntau - 1)))
    tau[0] = 0.0
    tau[-1] = beta
    # exact mirror symmetry tau_t + tau_{n-1-t} = beta
    tau = 0.5 * (tau + (beta - tau[::-1]))
    return tau


def values_to_cheb(ntau: int) -> np.ndarray:
    """C[l, t] with c_l = sum_t C[l, t] f(tau_t) for the Lobatto nodes (DCT-I)."""
    N = ntau - 1
    t = np.arange(ntau)
    j = N - t  # x_t = cos(pi j / N)
    l = np.arange(ntau)
    C = (2.0 / N) * np.cos(np.pi * np.outer(l, j) / N)
    w = np.ones(ntau)
    w[0] = w[-1] = 0.5
    C *= w[None, :]  # endpoint weights in the sum over nodes (j = 0, N <=> t = N, 0)
    C[0, :] *= 0.5
    C[N, :] *= 0.5
    return C


def _cheb_fourier_small(a: float, n: int) -> np.ndarray:
    """I_l(a) for l < n from the Jacobi-Anger expansion (used for |a| < 1.25 n + 20).

    e^{iax} = sum_k eps_k i^k J_k(a) T_k(x) (eps_0 = 1, eps_k = 2), so
    I_l(a) = sum_k eps_k i^k J_k(a) W_lk with W_lk = int T_l T_k dx
           = 1/(1-(l+k)^2) + 1/(1-(l-k)^2) for l+k even, else 0.
    J_k(a) is negligible beyond k ~ a + 40 + 4 a^(1/3).
    """
    K = int(abs(a) + 40 + 4 * abs(a) ** (1.0 / 3.0))
    k = np.arange(K + 1)
    eps = np.where(k == 0, 1.0, 2.0)
    coef = eps * (1j ** k) * jv(k, a)
    l = np.arange(n)[:, None]
    s = (l + k[None, :]).astype(np.float64)
    d = (l - k[None, :]).astype(np.float64)
    with np.errstate(divide="ignore"):
        W = np.where((l + k[None, :]) % 2 == 0, 1.0 / (1.0 - s * s) + 1.0 / (1.0 - d * d), 0.0)
    return W @ coef


def _cheb_fourier_large(a: float, n: int) -> np.ndarray:
    """I_l(a) for l < n by the forward recurrence (stable for |a| >= 1.25 n).

    From T_l = (T'_{l+1}/(l+1) - T'_{l-1}/(l-1))/2 (l >= 2), T_1 = T'_2/4,
    T_0 = T'_1 and int T'_m e^{iax} = B_m - i a I_m, B_m = e^{ia} - (-1)^m e^{-ia}.
    """
    ia = 1j * a
    ep, em = np.exp(1j * a), np.exp(-1j * a)

    def B(m):
        return ep - (em if m % 2 == 0 else -em)

    I = np.zeros(max(n, 3), dtype=np.complex128)
    I[0] = 2.0 * np.sin(a) / a
    I[1] = (B(1) - I[0]) / ia
    I[2] = (B(2) - 4.0 * I[1]) / ia
    for l in range(2, n - 1):
        I[l + 1] = (l + 1) / ia * (B(l + 1) / (l + 1) - (B(l - 1) - ia * I[l - 1]) / (l - 1) - 2.0 * I[l])
    return I[:n]


def cheb_fourier(a: float, n: int) -> np.ndarray:
    """I_l(a) = int_{-1}^{1} T_l(x) e^{iax} dx, l = 0 .. n-1."""
    if a == 0.0:
        l = np.arange(n)
        out = np.zeros(n, dtype=np.complex128)
        ev = l % 2 == 0
        out[ev] = 2.0 / (1.0 - l[ev] ** 2)
        return out
    if a < 0:
        return np.conj(cheb_fourier(-a, n))
    if a < 1.25 * n + 20:
        return _cheb_fourier_small(a, n)
    return _cheb_fourier_large(a, n)


def transform_rows(nu: np.ndarray, tau_n: int, beta: float) -> np.ndarray:
    """Rows R[m, t]: X(i nu_m) = sum_t R[m, t] f(tau_t) for the interpolant of f."""
    C = values_to_cheb(tau_n)
    rows = np.empty((len(nu), tau_n), dtype=np.complex128)
    for m, v in enumerate(nu):
        a = 0.5 * v * beta
        I = cheb_fourier(a, tau_n)
        rows[m] = 0.5 * beta * np.exp(1j * a) * (I @ C)
    return rows


def _candidates() -> np.ndarray:
    c = np.concatenate([np.arange(300), np.unique(np.round(np.logspace(np.log10(300), np.log10(2.0e4), 400)))])
    return np.unique(c.astype(np.int64))


def _greedy_select(rows: np.ndarray, npick: int, forced: list[int]) -> list[int]:
    """Greedy pivoted Gram-Schmidt over 2-row real blocks [Re r; Im r].

    At each step the candidate whose block keeps the largest residual norm
    after projection on the rows already chosen is taken (rows unscaled, so
    the pick favours well-conditioned transforms).
    """
    R = np.concatenate([rows.real[:, None, :], rows.imag[:, None, :]], axis=1).copy()  # [nc, 2, ntau]
    picked: list[int] = []

    def add(c):
        for i in range(2):
            v = R[c, i].copy()
            nv = np.linalg.norm(v)
            if nv <= 1e-13 * max(1.0, np.abs(rows).max()):
                continue
            b = v / nv
            # remove b from every candidate row (modified Gram-Schmidt on residuals)
            R[:] -= np.einsum("cit,t->ci", R, b)[:, :, None] * b[None, None, :]
        picked.append(c)

    for c in forced:
        add(c)
    while len(picked) < npick + len(forced):
        score = np.einsum("cit,cit->c", R, R)
        score[picked] = -1.0
        add(int(np.argmax(score)))
    return picked


@functools.lru_cache(maxsize=16)
def _make_grid_cached(ntau: int, beta: float) -> Grid:
    if ntau < 4 or ntau % 2:
        raise ValueError("ntau must be even and >= 4")
    tau = lobatto_tau(ntau, beta)
    cand = _candidates()
    # fermionic
    rows_f = transform_rows((2 * cand + 1) * np.pi / beta, ntau, beta)
    pf = _greedy_select(rows_f, ntau // 2, [])
    npos = np.sort(cand[pf])
    nf = np.sort(np.concatenate([-npos - 1, npos]))
    TF_t2w = transform_rows((2 * nf + 1) * np.pi / beta, ntau, beta)
    # bosonic: Omega_0 forced, then ntau/2 positive nodes
    candb = cand[cand >= 0]
    rows_b = transform_rows(2 * candb * np.pi / beta, ntau, beta)
    zero = int(np.where(candb == 0)[0][0])
    pb = _greedy_select(rows_b, ntau // 2, [zero])
    bpos = np.sort(candb[[p for p in pb if p != zero]])
    nb = np.sort(np.concatenate([-bpos, [0], bpos]))
    TB_t2w = transform_rows(2 * nb * np.pi / beta, ntau, beta)
    TF_w2t = np.linalg.pinv(TF_t2w, rcond=1e-15)
    TB_w2t = np.linalg.pinv(TB_t2w, rcond=1e-15)
    for a in (tau, nf, nb, TF_t2w, TF_w2t, TB_t2w, TB_w2t):
        a.setflags(write=False)
    return Grid(float(beta), tau, nf, nb, TF_t2w, TF_w2t, TB_t2w, TB_w2t)


def make_grid(ntau: int, beta: float) -> Grid:
    """Chebyshev-Lobatto tau grid with sparse fermionic/bosonic Matsubara transforms."""
    return _make_grid_cached(int(ntau), float(beta))
