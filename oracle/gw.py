"""FP64 CPU oracle for the fully self-consistent GW iteration (test infrastructure).

This module is the reference that the HIP path is checked against.  It is
test infrastructure only: product code never imports it.  It shares no code
with the HIP path; both take the same seeded inputs from ``synth``.

Every step follows the paper (Iskakov et al., Green/WeakCoupling) literally,
with plain NumPy matrix products, in complex128:

  O1  gamma^k = G^k(0^-) = -G^k(beta^-)                     (Eq. sigma_inf, G at 0^-)
  O2  Sigma^inf: Hartree minus exchange                      (Eq. sigma_inf)
  O3  P0^q_{QQ'}(tau)                                         (Eq. tilde_P0_tau)
  O4  P0(i Omega) = int_0^beta P0(tau) e^{i Omega tau}       (Eq. P0t_to_P0w)
  O5  P~ = [I - P0]^{-1} P0                                   (Eq. tilde_P_omega)
  O6  P~(tau) from P~(i Omega)                                (inverse of Eq. P0t_to_P0w)
  O7  Sigma~^k(tau) = -(1/Nk) sum_q sum_ab G^{k-q} W~         (Eqs. sigma_gw, tilde_W_DF2)
  O8  Sigma mixing                                            (Sec. 4.2.2, iteration mixing)
  O9  Sigma~(i omega) from Sigma~(tau)
  O10 chemical potential for a fixed particle number           (Sec. 2.3, step 3)
  O11 Dyson G(i omega) and G(tau)                            (Eq. dyson)
  O12 Galitskii-Migdal energy (diagnostic; the paper names total energies
      but prints no formula)
  O13 k-path interpolation of Sigma^inf and Sigma~ (Sec. 2.4): to real
      space over the mesh, back onto arbitrary k
  O14 GF2 second-order self-energy, direct minus exchange    (Eq. sigma2)

Readings of the text (each listed with its reason in the design notes):
  * G1  In Eq. tilde_P0_tau the factor G^k(-tau) is the stored value at
        beta - tau.  With the antiperiodic G(-tau) = -G(beta-tau) fixed by
        Eq. dos_tau the printed sign would anti-screen; read this way the
        bubble equals the direct term of Eq. sigma2 (pinned in the tests).
  * G2  In Eq. sigma2 the momentum delta is Nk times a Kronecker delta, so
        the prefactor is effectively 1/Nk^2 (as in Eqs. sigma_gw and
        tilde_P0_tau); G(-tau) there is the antiperiodic -G(beta - tau).
  * G3  Spin-restricted runs (nspin = 1) hold one spin channel; the spin sums
        in Eq. tilde_P0_tau, the Hartree term and the direct term of Eq.
        sigma2 become a factor 2.
  * G7  The frequency -> tau maps are the grid's least-squares inverses.
  * G8  Node 0 is tau = 0^+, node ntau-1 is beta^-, G(0^-) = -G(beta^-).
  * G9  The one-body term of Eq. dyson is H^(0); Sigma^inf is recomputed
        from G every iteration.

Array layouts (row-major, complex128):
  V[q][k][Q][i][j] = V^{k,k+q}_{ij}(Q);  G[s][t][k][i][j];  H0[s][k][i][j];
  S[k][i][j];  P[q][t][Q][Q'];  Pw[q][m][Q][Q'];  Sigma_tau[s][t][k][i][j];
  Sigma_inf[s][k][i][j].
"""
from __future__ import annotations

import dataclasses

import numpy as np


# --------------------------------------------------------------------------- k-mesh helpers
def _kflat(kmesh, p):
    m1, m2, m3 = kmesh
    return ((p[0] % m1) * m2 + (p[1] % m2)) * m3 + (p[2] % m3)


def _kpoints(kmesh):
    return [(a, b, c) for a in range(kmesh[0]) for b in range(kmesh[1]) for c in range(kmesh[2])]


class KMesh:
    """Gamma-centred Monkhorst-Pack mesh with modular k +- q arithmetic."""

    def __init__(self, kmesh):
        self.kmesh = tuple(int(x) for x in kmesh)
        self.pts = _kpoints(self.kmesh)
        self.nk = len(self.pts)

    def add(self, k, q):
        a, b = self.pts[k], self.pts[q]
        return _kflat(self.kmesh, (a[0] + b[0], a[1] + b[1], a[2] + b[2]))

    def sub(self, k, q):
        a, b = self.pts[k], self.pts[q]
        return _kflat(self.kmesh, (a[0] - b[0], a[1] - b[1], a[2] - b[2]))


def V_pair(V: np.ndarray, km: KMesh, k1: int, k2: int) -> np.ndarray:
    """V^{k1,k2}(Q) [naux][nao][nao], looked up literally: V^{k1,k2} is stored at [q = k2 - k1][k1]."""
    return V[km.sub(k2, k1), k1]


def spin_weight(nspin: int) -> float:
    """Reading G3: a restricted run (one stored channel) stands for two equal spins."""
    return 2.0 if nspin == 1 else 1.0


# --------------------------------------------------------------------------- O1, O2
def density_matrix(G: np.ndarray) -> np.ndarray:
    """O1: gamma[s][k] = G^k_s(0^-) = -G^k_s(beta^-) (last grid node)."""
    return -G[:, -1]


def sigma_inf(V: np.ndarray, G: np.ndarray, kmesh) -> np.ndarray:
    """O2, Eq. sigma_inf.

    Hartree: (1/Nk) sum_{k' s' Q ab} V^{k,k}_{ij}(Q) G^{k'}_{s',ab}(0^-) V^{k',k'}_{ba}(Q)
    exchange: -(1/Nk) sum_{k' Q ab} V^{k,k'}_{ia}(Q) G^{k'}_{s,ab}(0^-) V^{k',k}_{bj}(Q)
    """
    km = KMesh(kmesh)
    ns = G.shape[0]
    nk = km.nk
    gam = density_matrix(G)  # [s][k]
    w = spin_weight(ns)
    naux = V.shape[2]
    nao = V.shape[3]
    # Hartree density per auxiliary index: sum_{k' s'} sum_ab gamma_ab V^{k'k'}_{ba}(Q)
    D = np.zeros(naux, dtype=np.complex128)
    for s in range(ns):
        for kp in range(nk):
            Vkk = V_pair(V, km, kp, kp)
            D += w * np.einsum("ab,Qba->Q", gam[s, kp], Vkk)
    D /= nk
    out = np.zeros((ns,) + G.shape[2:], dtype=np.complex128)
    for s in range(ns):
        for k in range(nk):
            hart = np.einsum("Qij,Q->ij", V_pair(V, km, k, k), D)
            exch = np.zeros_like(hart)
            for kp in range(nk):
                A = V_pair(V, km, k, kp)  # V^{k,k'}(Q)  [Q][i][a]
                B = V_pair(V, km, kp, k)  # V^{k',k}(Q)  [Q][b][j]
                Y = np.matmul(A, gam[s, kp])  # [Q][i][b] = sum_a V_ia gamma_ab
                exch += np.swapaxes(Y, 0, 1).reshape(nao, naux * nao) @ B.reshape(naux * nao, nao)
            out[s, k] = hart - exch / nk
    return out


# --------------------------------------------------------------------------- O3
def polarization(V: np.ndarray, G: np.ndarray, kmesh, ts=None, qs=None) -> np.ndarray:
    """O3, Eq. tilde_P0_tau with reading G1:

    P0^q_{QQ'}(tau) = -(1/Nk) sum_{k s} sum_{abcd} V^{k,k+q}_{da}(Q) G^k_{s,cd}(beta-tau)
                                                   G^{k+q}_{s,ab}(tau) V^{k+q,k}_{bc}(Q')
    (spin sum doubled for a restricted run).  Written as a trace,
    sum_{abcd} = sum_{d,b} [V^{k,k+q}(Q) G^{k+q}(tau)]_{db} [V^{k+q,k}(Q') G^k(beta-tau)]_{bd}.

    ts, qs: optional lists of grid nodes and momentum transfers to evaluate (default all); they only select.
    Returns P[q][t][Q][Q'] over qs x ts.
    """
    km = KMesh(kmesh)
    ns, ntau, nk, nao, _ = G.shape
    naux = V.shape[2]
    ts = list(range(ntau)) if ts is None else list(ts)
    qs = list(range(nk)) if qs is None else list(qs)
    w = spin_weight(ns)
    P = np.zeros((len(qs), len(ts), naux, naux), dtype=np.complex128)
    trev = [ntau - 1 - t for t in ts]  # beta - tau_t is node ntau-1-t on the symmetric grid
    for iq, q in enumerate(qs):
        for k in range(nk):
            kq = km.add(k, q)
            A = V_pair(V, km, k, kq).reshape(naux * nao, nao)  # V^{k,k+q}(Q), rows (Q, d), cols a
            B = V_pair(V, km, kq, k).reshape(naux * nao, nao)  # V^{k+q,k}(Q'), rows (Q', b), cols c
            for s in range(ns):
                for it, t in enumerate(ts):
                    # L[Q][d][b] = sum_a V^{k,k+q}_{da}(Q) G^{k+q}_{ab}(tau)
                    L = (A @ G[s, t, kq]).reshape(naux, nao * nao)  # cols (d, b)
                    # R[Q'][b][d] = sum_c V^{k+q,k}_{bc}(Q') G^k_{cd}(beta - tau)
                    R = (B @ G[s, trev[it], k]).reshape(naux, nao, nao)
                    Rf = np.swapaxes(R, 1, 2).reshape(naux, nao * nao)  # cols (d, b)
                    P[iq, it] += w * (L @ Rf.T)
    P *= -1.0 / nk
    return P


# --------------------------------------------------------------------------- O4 - O6
def to_bosonic(P: np.ndarray, TB_t2w: np.ndarray) -> np.ndarray:
    """O4, Eq. P0t_to_P0w on the grid: Pw[q][m] = sum_t TB_t2w[m, t] P[q][t]."""
    nq, ntau = P.shape[:2]
    rest = P.shape[2:]
    out = np.empty((nq, TB_t2w.shape[0]) + rest, dtype=np.complex128)
    for q in range(nq):
        out[q] = (TB_t2w @ P[q].reshape(ntau, -1)).reshape((TB_t2w.shape[0],) + rest)
    return out


def screen(Pw: np.ndarray) -> np.ndarray:
    """O5, Eq. tilde_P_omega: P~(i Omega) = [I - P0(i Omega)]^{-1} P0(i Omega), per (q, m)."""
    nq, nw, naux, _ = Pw.shape
    I = np.eye(naux)
    out = np.empty_like(Pw)
    for q in range(nq):
        for m in range(nw):
            out[q, m] = np.linalg.solve(I - Pw[q, m], Pw[q, m])
    return out


def from_bosonic(Pw: np.ndarray, TB_w2t: np.ndarray) -> np.ndarray:
    """O6: P~[q][t] = sum_m TB_w2t[t, m] P~w[q][m] (least-squares inverse of O4)."""
    nq, nw = Pw.shape[:2]
    rest = Pw.shape[2:]
    out = np.empty((nq, TB_w2t.shape[0]) + rest, dtype=np.complex128)
    for q in range(nq):
        out[q] = (TB_w2t @ Pw[q].reshape(nw, -1)).reshape((TB_w2t.shape[0],) + rest)
    return out


# --------------------------------------------------------------------------- O7
def selfenergy(V: np.ndarray, G: np.ndarray, Pt: np.ndarray, kmesh, ts=None, ks=None, qs=None) -> np.ndarray:
    """O7, Eqs. sigma_gw and tilde_W_DF2 (W~ evaluated on tau through P~(tau)):

    Sigma~^k_{s,ij}(tau) = -(1/Nk) sum_q sum_ab G^{k-q}_{s,ab}(tau)
                            sum_{QQ'} V^{k,k-q}_{ia}(Q) P~^q_{QQ'}(tau) V^{k-q,k}_{bj}(Q')
    evaluated as X(Q') = sum_Q P~_{QQ'} V^{k,k-q}(Q), then sum_{Q'} X(Q') G^{k-q} V^{k-q,k}(Q').

    Pt[q][t'] holds the nodes in ts (or all nodes).  qs: optional subset of the momentum transfers summed over (a
    selection only; the default is the whole sum).  Returns Sigma[s][t][k][i][j] over ts x ks.
    """
    km = KMesh(kmesh)
    ns, ntau, nk, nao, _ = G.shape
    naux = V.shape[2]
    ts = list(range(ntau)) if ts is None else list(ts)
    ks = list(range(nk)) if ks is None else list(ks)
    qs = list(range(nk)) if qs is None else list(qs)
    out = np.zeros((ns, len(ts), len(ks), nao, nao), dtype=np.complex128)
    for ik, k in enumerate(ks):
        for q in qs:
            kmq = km.sub(k, q)
            A = V_pair(V, km, k, kmq)  # V^{k,k-q}(Q)  [Q][i][a]
            B = V_pair(V, km, kmq, k)  # V^{k-q,k}(Q') [Q'][b][j]
            Af = A.reshape(naux, nao * nao)
            Bcat = B.reshape(naux * nao, nao)  # rows (Q', b)
            for it in range(len(ts)):
                t = ts[it]
                X = (Pt[q, it].T @ Af).reshape(naux * nao, nao)  # X[(Q', i)][a] = sum_Q P_{QQ'} A[Q][i][a]
                for s in range(ns):
                    Y = (X @ G[s, t, kmq]).reshape(naux, nao, nao)  # Y[Q'][i][b] = sum_a X_{ia} G_{ab}
                    Ycat = np.swapaxes(Y, 0, 1).reshape(nao, naux * nao)  # [i][(Q', b)]
                    out[s, it, ik] += Ycat @ Bcat
    out *= -1.0 / nk
    return out


# --------------------------------------------------------------------------- O14
def gf2_selfenergy(V: np.ndarray, G: np.ndarray, kmesh, ts=None, ks=None) -> np.ndarray:
    """O14, Eq. sigma2 with reading G2 (prefactor 1/Nk^2, k3 = k1 + k2 - k, G(-tau) = -G(beta - tau)):

    Sigma~(2)^k_{s,ij}(tau) = -(1/Nk^2) sum_{k1 k2} sum_{QQ'} [direct - exchange]_{ij}
      direct   = sum_{s'} [V^{k k1}(Q) G^{k1}_s(tau) V^{k1 k}(Q')]
                          * Tr[V^{k3 k2}(Q) G^{k2}_{s'}(tau) V^{k2 k3}(Q') G^{k3}_{s'}(-tau)]
      exchange = V^{k k1}(Q) G^{k1}_s(tau) V^{k1 k3}(Q') G^{k3}_s(-tau) V^{k3 k2}(Q) G^{k2}_s(tau) V^{k2 k}(Q')
    (the orbital sums of Eq. sigma2 written as matrix products and a trace; the spin sum of the direct
    term doubled for a restricted run).  For every (Q, Q') the matrix chain is formed whole and the pairs
    are summed last.  Returns Sigma[s][t][k][i][j] over ts x ks.
    """
    km = KMesh(kmesh)
    ns, ntau, nk, nao, _ = G.shape
    ts = list(range(ntau)) if ts is None else list(ts)
    ks = list(range(nk)) if ks is None else list(ks)
    w = spin_weight(ns)
    out = np.zeros((ns, len(ts), len(ks), nao, nao), dtype=np.complex128)
    for ik, k in enumerate(ks):
        for k1 in range(nk):
            for k2 in range(nk):
                k3 = km.sub(km.add(k1, k2), k)
                Va = V_pair(V, km, k, k1)    # V^{k k1}(Q)
                Vb = V_pair(V, km, k1, k)    # V^{k1 k}(Q')
                Vc = V_pair(V, km, k3, k2)   # V^{k3 k2}(Q)
                Vd = V_pair(V, km, k2, k3)   # V^{k2 k3}(Q')
                Ve = V_pair(V, km, k1, k3)   # V^{k1 k3}(Q')
                Vf = V_pair(V, km, k2, k)    # V^{k2 k}(Q')
                for it, t in enumerate(ts):
                    tm = ntau - 1 - t  # beta - tau on the symmetric grid
                    # bubble Tr[V^{k3 k2}(Q) G^{k2}(tau) V^{k2 k3}(Q') G^{k3}(-tau)], summed over spins
                    D = np.zeros((V.shape[2], V.shape[2]), dtype=np.complex128)
                    for sp in range(ns):
                        L = np.matmul(Vc, G[sp, t, k2])          # [Q][m][l]
                        R = np.matmul(Vd, -G[sp, tm, k3])        # [Q'][l][m]
                        D += w * np.einsum("Qml,Plm->QP", L, R)
                    for s in range(ns):
                        A1 = np.matmul(Va, G[s, t, k1])                        # [Q][i][q]
                        direct = np.matmul(A1[:, None], Vb[None, :])           # [Q][Q'][i][j]
                        direct = np.einsum("QP,QPij->ij", D, direct)
                        ch = np.matmul(A1[:, None], np.matmul(Ve, -G[s, tm, k3])[None, :])  # [Q][Q'][i][m]
                        ch = np.matmul(ch, np.matmul(Vc, G[s, t, k2])[:, None])            # [Q][Q'][i][l]
                        ch = np.matmul(ch, Vf[None, :])                                   # [Q][Q'][i][j]
                        out[s, it, ik] += direct - ch.sum(axis=(0, 1))
    out *= -1.0 / nk ** 2
    return out


# --------------------------------------------------------------------------- O8 - O11
def mix(new: np.ndarray, old: np.ndarray | None, alpha: float) -> np.ndarray:
    """O8: Sigma_n = alpha Sigma[G_{n-1}] + (1 - alpha) Sigma_{n-1} (alpha = 1: no mixing)."""
    if old is None or alpha == 1.0:
        return new.copy()
    return alpha * new + (1.0 - alpha) * old


def to_fermionic(X: np.ndarray, TF_t2w: np.ndarray) -> np.ndarray:
    """O9: X[s][m] = sum_t TF_t2w[m, t] X[s][t]  (also used for G)."""
    ns, ntau = X.shape[:2]
    rest = X.shape[2:]
    out = np.empty((ns, TF_t2w.shape[0]) + rest, dtype=np.complex128)
    for s in range(ns):
        out[s] = (TF_t2w @ X[s].reshape(ntau, -1)).reshape((TF_t2w.shape[0],) + rest)
    return out


def from_fermionic(Xw: np.ndarray, TF_w2t: np.ndarray) -> np.ndarray:
    """O11 (second half): X[s][t] = sum_m TF_w2t[t, m] X[s][m]."""
    ns, nw = Xw.shape[:2]
    rest = Xw.shape[2:]
    out = np.empty((ns, TF_w2t.shape[0]) + rest, dtype=np.complex128)
    for s in range(ns):
        out[s] = (TF_w2t @ Xw[s].reshape(nw, -1)).reshape((TF_w2t.shape[0],) + rest)
    return out


def dyson(H0, S, Sinf, Sw, wf, mu) -> np.ndarray:
    """O11, Eq. dyson: G(i w_m) = [(i w_m + mu) S - H0 - Sigma^inf - Sigma~(i w_m)]^{-1}."""
    ns, nw, nk, nao, _ = Sw.shape
    Gw = np.empty_like(Sw)
    for s in range(ns):
        for m in range(nw):
            for k in range(nk):
                A = (1j * wf[m] + mu) * S[k] - H0[s, k] - Sinf[s, k] - Sw[s, m, k]
                Gw[s, m, k] = np.linalg.inv(A)
    return Gw


def electron_number(Gw, S, TF_w2t, nspin) -> float:
    """N = -(2/ns)(1/Nk) sum_{s,k} Re Tr[G^k_s(beta^-) S^k], G(beta^-) from the last row of TF_w2t."""
    ns, nw, nk = Gw.shape[:3]
    row = TF_w2t[-1]  # [nw]
    Gb = np.einsum("m,smkij->skij", row, Gw)
    tr = np.einsum("skij,kji->", Gb, S)
    return float(-(2.0 / nspin) * tr.real / nk)


class MuSearchError(RuntimeError):
    pass


def find_mu(nfun, mu0: float, n_target: float, max_doublings: int = 60, max_steps: int = 200):
    """O10: chemical potential with N(mu) = n_target (Sec. 2.3, step 3).

    1. Accept mu0 if |N(mu0) - Nt| <= tol, tol = 1e-12 max(1, Nt).
    2. Bracket: [mu0 - d, mu0 + d] with d = 1, doubled up to 60 times until
       N(lo) <= Nt <= N(hi)  (N is non-decreasing in mu).
    3. Illinois regula falsi (secant kept inside the bracket, with the retained
       end's residual halved when the same end is kept twice); a step outside
       (lo, hi) falls back to bisection.  Stop at |N - Nt| <= tol or a bracket
       narrower than 1e-14; at most 200 steps.
    Returns (mu, N(mu), number of N evaluations).
    """
    tol = 1e-12 * max(1.0, abs(n_target))
    evals = 1
    n0 = nfun(mu0)
    if abs(n0 - n_target) <= tol:
        return mu0, n0, evals
    d = 1.0
    for _ in range(max_doublings):
        lo, hi = mu0 - d, mu0 + d
        nlo, nhi = nfun(lo), nfun(hi)
        evals += 2
        if nlo <= n_target <= nhi:
            break
        d *= 2.0
    else:
        raise MuSearchError("chemical potential not bracketed")
    flo, fhi = nlo - n_target, nhi - n_target
    if abs(flo) <= tol:
        return lo, nlo, evals
    if abs(fhi) <= tol:
        return hi, nhi, evals
    side = 0
    for _ in range(max_steps):
        if hi - lo < 1e-14:
            mu = 0.5 * (lo + hi)
            n = nfun(mu)
            return mu, n, evals + 1
        mu = (lo * fhi - hi * flo) / (fhi - flo) if fhi != flo else 0.5 * (lo + hi)
        if not (lo < mu < hi):
            mu = 0.5 * (lo + hi)
        n = nfun(mu)
        evals += 1
        f = n - n_target
        if abs(f) <= tol:
            return mu, n, evals
        if f < 0:
            lo, flo = mu, f
            if side == -1:
                fhi *= 0.5
            side = -1
        else:
            hi, fhi = mu, f
            if side == 1:
                flo *= 0.5
            side = 1
    raise MuSearchError("chemical potential search did not converge")


# --------------------------------------------------------------------------- O12
def _cheb_coeff_matrix(ntau: int) -> np.ndarray:
    """Values on the Lobatto nodes -> Chebyshev coefficients (DCT-I), nodes ordered tau ascending."""
    N = ntau - 1
    x = -np.cos(np.pi * np.arange(ntau) / N)  # x_t = 2 tau_t / beta - 1
    V = np.polynomial.chebyshev.chebvander(x, N)  # V[t, l] = T_l(x_t)
    return np.linalg.inv(V)


def tau_integral_product(F: np.ndarray, H: np.ndarray, beta: float) -> complex:
    """int_0^beta sum_ij F_ij(tau) H_ji(beta - tau) dtau for grid functions F[t][..][i][j], H[t][..][i][j].

    Exact for the degree-(ntau-1) interpolants: with Chebyshev coefficients
    a_l (of F) and b_m (of H), H(beta - tau) has coefficients (-1)^m b_m and
    int_0^beta = beta/2 sum_{lm} a_l (-1)^m b_m W_lm,
    W_lm = int_{-1}^{1} T_l T_m dx = 1/(1-(l+m)^2) + 1/(1-(l-m)^2) for l+m even.
    """
    ntau = F.shape[0]
    nao = F.shape[-1]
    Cinv = _cheb_coeff_matrix(ntau)
    a = np.tensordot(Cinv, F.reshape(ntau, -1, nao, nao), axes=(1, 0))  # [l][k][i][j]
    b = np.tensordot(Cinv, H.reshape(ntau, -1, nao, nao), axes=(1, 0))  # [m][k][i][j]
    l = np.arange(ntau)
    L, M = np.meshgrid(l, l, indexing="ij")
    with np.errstate(divide="ignore"):
        W = np.where((L + M) % 2 == 0, 1.0 / (1.0 - (L + M) ** 2.0) + 1.0 / (1.0 - (L - M) ** 2.0), 0.0)
    W = W * ((-1.0) ** M)
    # sum_ij F_ij H_ji per coefficient pair
    tr = np.einsum("lkij,mkji->lm", a, b)
    return complex(0.5 * beta * np.sum(W * tr))


def energy(G: np.ndarray, H0: np.ndarray, Sinf: np.ndarray, Sig: np.ndarray, beta: float) -> dict:
    """O12: Galitskii-Migdal energy of (G, Sigma), spin factors per reading G3.

    E_1b   = (2/ns)(1/Nk) sum_{k,s} Re Tr[gamma H0]
    E_HF   = (1/ns)(1/Nk) sum_{k,s} Re Tr[gamma Sigma^inf]
    E_corr = -(1/ns)(1/Nk) sum_{k,s} int_0^beta Re Tr[Sigma~(tau) G(beta - tau)] dtau
    """
    ns, ntau, nk = G.shape[:3]
    gam = density_matrix(G)
    e1 = (2.0 / ns) * np.einsum("skij,skji->", gam, H0).real / nk
    ehf = (1.0 / ns) * np.einsum("skij,skji->", gam, Sinf).real / nk
    ec = 0.0
    for s in range(ns):
        ec += tau_integral_product(Sig[s], G[s], beta).real
    ec = -(1.0 / ns) * ec / nk
    return dict(e_1b=float(e1), e_hf=float(ehf), e_corr=float(ec), e_tot=float(e1 + ehf + ec))


# --------------------------------------------------------------------------- one iteration
# --------------------------------------------------------------------------- O13: k-path interpolation
def lattice_vectors(kmesh):
    """Reading K1 of Sec. 2.4: the lattice vectors R of the Born-von Karman supercell centred on 0, with the
    weight of each; along a direction of even mesh extent n the zone-boundary vectors R = -n/2 and +n/2 both
    appear with weight 1/2 (the sum of the weights along a direction is n)."""
    axes = []
    for n in kmesh:
        h = n // 2
        axes.append([(R, 0.5 if (n % 2 == 0 and abs(R) == h) else 1.0) for R in range(-h, h + 1)
                     if n % 2 == 0 or abs(R) <= h])
    return [((a, b, c), wa * wb * wc) for a, wa in axes[0] for b, wb in axes[1] for c, wc in axes[2]]


def kpath_interpolate(X: np.ndarray, kmesh, kfrac) -> np.ndarray:
    """O13, Sec. 2.4: X(R) = (1/N_k) sum_k X(k) e^{-i k.R}, then X(khat) = sum_R X(R) e^{i khat.R}.

    X: [..., nk, nao, nao] on the mesh (mesh point (a, b, c) = fractional (a/n0, b/n1, c/n2)); kfrac:
    [npath][3] fractional coordinates; k.R = 2 pi sum_d k_d R_d.  Returns [..., npath, nao, nao]."""
    km = KMesh(kmesh)
    nk = len(km.pts)
    kf = np.asarray(kfrac, dtype=np.float64).reshape(-1, 3)
    kpts = np.array([[a / kmesh[0], b / kmesh[1], c / kmesh[2]] for (a, b, c) in km.pts])
    out_shape = X.shape[:-3] + (kf.shape[0],) + X.shape[-2:]
    out = np.zeros(out_shape, dtype=np.complex128)
    for R, w in lattice_vectors(kmesh):
        Rv = np.array(R, dtype=np.float64)
        XR = np.zeros(X.shape[:-3] + X.shape[-2:], dtype=np.complex128)
        for k in range(nk):
            XR += X[..., k, :, :] * np.exp(-2j * np.pi * (kpts[k] @ Rv))
        XR /= nk
        for p in range(kf.shape[0]):
            out[..., p, :, :] += w * XR * np.exp(2j * np.pi * (kf[p] @ Rv))
    return out


@dataclasses.dataclass
class State:
    G: np.ndarray
    Sinf: np.ndarray | None
    Sig: np.ndarray | None
    mu: float


def sigma_eval(V, G, kmesh, grid, method="gw"):
    """Sigma^inf and Sigma~ of G (steps O1 - O7; method "gf2": O14 in place of O3 - O7); also returns the
    intermediates."""
    Sinf = sigma_inf(V, G, kmesh)
    if method == "gf2":
        return Sinf, gf2_selfenergy(V, G, kmesh), {}
    P0 = polarization(V, G, kmesh)
    Pw = to_bosonic(P0, grid.TB_t2w)
    Ptw = screen(Pw)
    Pt = from_bosonic(Ptw, grid.TB_w2t)
    Sig = selfenergy(V, G, Pt, kmesh)
    return Sinf, Sig, dict(P0=P0, Pw=Pw, Ptw=Ptw, Pt=Pt)


def solve_dyson(H0, S, Sinf, Sig, grid, nspin, mu0, n_target):
    """Steps O9 - O11: Sigma~(i w), mu search (n_target < 0 keeps mu0) and G(tau)."""
    Sw = to_fermionic(Sig, grid.TF_t2w)
    wf = grid.wf

    def nfun(mu):
        return electron_number(dyson(H0, S, Sinf, Sw, wf, mu), S, grid.TF_w2t, nspin)

    if n_target is None or n_target < 0:
        mu, n = mu0, nfun(mu0)
    else:
        mu, n, _ = find_mu(nfun, mu0, n_target)
    Gw = dyson(H0, S, Sinf, Sw, wf, mu)
    G = from_fermionic(Gw, grid.TF_w2t)
    return G, mu, n


def iterate(system, state: State, alpha: float = 1.0, method: str = "gw"):
    """One self-consistency iteration (Sec. 2.3): Sigma[G] (GW, or GF2 with method "gf2"), mixing, mu,
    Dyson, energy."""
    sp = system.spec
    grid = system.grid
    Sinf_new, Sig_new, inter = sigma_eval(system.V, state.G, sp.kmesh, grid, method)
    Sinf = mix(Sinf_new, state.Sinf, alpha)
    Sig = mix(Sig_new, state.Sig, alpha)
    G, mu, n = solve_dyson(system.H0, system.S, Sinf, Sig, grid, sp.nspin, state.mu, system.n_target)
    e = energy(G, system.H0, Sinf, Sig, sp.beta)
    dsig = float(np.max(np.abs(Sig - state.Sig))) if state.Sig is not None else float(np.max(np.abs(Sig)))
    herm = float(np.max(np.abs(Sig - np.conj(np.swapaxes(Sig, -1, -2)))))
    report = dict(e, n_elec=n, mu=mu, max_dsigma=dsig, herm_err=herm)
    return State(G, Sinf, Sig, mu), report, inter


# ----------------------------------------------------------------------------- DIIS (Sec. 4.2.2)
@dataclasses.dataclass
class DiisHistory:
    """Self-energies of the last iterations for the DIIS extrapolation of Sec. 4.2.2.

    size: most stored vectors; start: first iteration (0-based) that extrapolates (earlier ones mix with
    alpha).  xs[i] = (Sinf, Sigma~) computed from G_{i-1}; rs[i] = xs[i] minus the self-energy that produced
    G_{i-1} (zero before the first iteration), the quantity that vanishes at self-consistency.
    """
    size: int
    start: int
    xs: list = dataclasses.field(default_factory=list)
    rs: list = dataclasses.field(default_factory=list)
    n: int = 0


def diis_coefficients(rs) -> np.ndarray:
    """Pulay's extrapolation: c minimises |sum_i c_i r_i|^2 subject to sum_i c_i = 1, from the Lagrange system
    [[B, 1], [1^T, 0]] [c, l] = [0, 1] with B_ij = Re <r_i, r_j> (both parts of each residual).  B is scaled by
    its largest diagonal element first (the solution does not change)."""
    m = len(rs)
    B = np.empty((m, m))
    for i in range(m):
        for j in range(m):
            B[i, j] = sum(float(np.vdot(a, b).real) for a, b in zip(rs[i], rs[j]))
    B = B / np.max(np.diag(B))
    A = np.zeros((m + 1, m + 1))
    A[:m, :m] = B
    A[:m, m] = 1.0
    A[m, :m] = 1.0
    rhs = np.zeros(m + 1)
    rhs[m] = 1.0
    return np.linalg.solve(A, rhs)[:m]


def iterate_diis(system, state: State, hist: DiisHistory, alpha: float = 1.0):
    """One iteration with DIIS (Sec. 4.2.2): the self-energy that enters Dyson is sum_i c_i Sigma_i over the
    stored self-energies once hist.start iterations have run (static mixing with alpha before)."""
    sp = system.spec
    grid = system.grid
    Sinf_new, Sig_new, inter = sigma_eval(system.V, state.G, sp.kmesh, grid)
    Sinf_old = state.Sinf if state.Sinf is not None else np.zeros_like(Sinf_new)
    Sig_old = state.Sig if state.Sig is not None else np.zeros_like(Sig_new)
    hist.xs.append((Sinf_new, Sig_new))
    hist.rs.append((Sinf_new - Sinf_old, Sig_new - Sig_old))
    if len(hist.xs) > hist.size:
        hist.xs.pop(0)
        hist.rs.pop(0)
    if hist.n >= hist.start and len(hist.xs) >= 2:
        c = diis_coefficients(hist.rs)
        Sinf = sum(ci * x[0] for ci, x in zip(c, hist.xs))
        Sig = sum(ci * x[1] for ci, x in zip(c, hist.xs))
    else:
        c = None
        Sinf = mix(Sinf_new, state.Sinf, alpha)
        Sig = mix(Sig_new, state.Sig, alpha)
    hist.n += 1
    G, mu, n = solve_dyson(system.H0, system.S, Sinf, Sig, grid, sp.nspin, state.mu, system.n_target)
    e = energy(G, system.H0, Sinf, Sig, sp.beta)
    dsig = float(np.max(np.abs(Sig - Sig_old)))
    herm = float(np.max(np.abs(Sig - np.conj(np.swapaxes(Sig, -1, -2)))))
    report = dict(e, n_elec=n, mu=mu, max_dsigma=dsig, herm_err=herm, diis_coef=c)
    return State(G, Sinf, Sig, mu), report, inter
