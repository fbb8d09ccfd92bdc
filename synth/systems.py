"""Seeded synthetic GW inputs shaped like the paper's workloads.

Stand-ins for the PySCF-prepared inputs of Sec. 4.1 (one-body Hamiltonian
H^(0)(k), overlap S(k), density-fitted integrals V^{k,k'}_{ij}(Q) of
Eq. CoulombDF, a mean-field starting G).  Every tensor is drawn from the
counter-based generator in ``synth.rng`` so that any block can be regenerated
on its own.

Conventions
-----------
* Gamma-centred m1 x m2 x m3 Monkhorst-Pack mesh; k = (i0, i1, i2) has flat
  index (i0*m2 + i1)*m3 + i2; k +- q and -k are taken component-wise modulo
  the mesh.
* V is stored as V[q][k][Q][i][j] = V^{k,k+q}_{ij}(Q): every ordered pair
  (k1, k2) appears exactly once, with q = k2 - k1.
* Hermitian pairing V^{k2,k1}_{ij}(Q) = conj V^{k1,k2}_{ji}(Q) (real auxiliary
  basis in the chemists'-notation integrals of Eq. Coulomb).
* G is stored as G[s][t][k][i][j] on the grid tau_t; node 0 is tau = 0+ and
  node ntau-1 is tau = beta-.
* Complex numbers are complex128 (interleaved re, im doubles).

Nothing here evaluates the self-energy method: the only physics is the
starting guess, the non-interacting G of Eq. dos_tau's sign convention for a
discrete spectrum (G(tau) = -C diag(e^{-(e-mu)tau}/(1+e^{-beta(e-mu)})) C^H),
which the paper's loop takes as an input.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

from . import rng
from .grid import Grid, make_grid


# --------------------------------------------------------------------------- k mesh
def kmesh_points(kmesh) -> np.ndarray:
    m = tuple(int(x) for x in kmesh)
    idx = np.array([(a, b, c) for a in range(m[0]) for b in range(m[1]) for c in range(m[2])], dtype=np.int64)
    return idx


def k_flat(kmesh, i0, i1, i2) -> int:
    m1, m2, m3 = kmesh
    return ((i0 % m1) * m2 + (i1 % m2)) * m3 + (i2 % m3)


def k_add_table(kmesh) -> np.ndarray:
    """add[k, q] = flat index of k + q."""
    pts = kmesh_points(kmesh)
    nk = len(pts)
    out = np.empty((nk, nk), dtype=np.int64)
    for a in range(nk):
        for b in range(nk):
            p = pts[a] + pts[b]
            out[a, b] = k_flat(kmesh, *p)
    return out


def k_sub_table(kmesh) -> np.ndarray:
    """sub[k, q] = flat index of k - q."""
    pts = kmesh_points(kmesh)
    nk = len(pts)
    out = np.empty((nk, nk), dtype=np.int64)
    for a in range(nk):
        for b in range(nk):
            p = pts[a] - pts[b]
            out[a, b] = k_flat(kmesh, *p)
    return out


def k_neg(kmesh) -> np.ndarray:
    pts = kmesh_points(kmesh)
    return np.array([k_flat(kmesh, *(-p)) for p in pts], dtype=np.int64)


# --------------------------------------------------------------------------- random matrices
def haar_unitary(key, n: int, real: bool = False) -> np.ndarray:
    if real:
        z = rng.normals(key, n * n).reshape(n, n)
    else:
        z = rng.complex_normals(key, (n, n))
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    ph = d / np.abs(d)
    return q * ph[None, :]


def random_hermitian_spectrum(seed: int, tag: int, spin: int, k: int, n: int, lo: float, hi: float,
                              real: bool) -> np.ndarray:
    """U diag(lambda) U^H with lambda ~ U[lo, hi] i.i.d. and U Haar (orthogonal if real)."""
    lam = lo + (hi - lo) * rng.uniforms(rng.stream_key(seed, tag, spin, k, 0, 1), 0, n)
    U = haar_unitary(rng.stream_key(seed, tag, spin, k, 0, 2), n, real=real)
    h = (U * lam[None, :]) @ U.conj().T
    return 0.5 * (h + h.conj().T)


# --------------------------------------------------------------------------- configs
@dataclasses.dataclass
class SystemSpec:
    name: str
    kmesh: tuple
    nao: int
    naux: int
    ntau: int
    beta: float
    nspin: int = 1  # 1 = spin-restricted, 2 = unrestricted
    seed: int = 18479
    band: float = 2.0  # eigenvalues of H0 uniform in [-band, band]
    v_decay: float = 0.05  # V ~ exp(-v_decay * Q)
    v_scale: float | None = None  # amplitude a (default 0.7 / nao)
    f_time_reversal: bool = True  # impose H0(-k) = conj H0(k)
    v_time_reversal: bool = False  # impose V^{-k1,-k2}(Q) = conj V^{k1,k2}(Q)
    s_identity: bool = True  # S = I, else I + 0.1 * (random Hermitian of unit norm)
    mu0: float = 0.0
    point_group: str = ""  # "" (none), "Oh" or "C3": inputs invariant under that group (synth.symmetry)

    @property
    def nk(self) -> int:
        return int(np.prod(self.kmesh))

    @property
    def amp(self) -> float:
        return self.v_scale if self.v_scale is not None else 0.7 / self.nao


@dataclasses.dataclass
class System:
    spec: SystemSpec
    grid: Grid
    H0: np.ndarray  # [ns][nk][nao][nao]
    S: np.ndarray  # [nk][nao][nao]
    V: np.ndarray  # [nk(q)][nk(k)][naux][nao][nao]  = V^{k,k+q}
    G0: np.ndarray  # [ns][ntau][nk][nao][nao]
    n_target: float
    mu0: float

    @property
    def dims(self) -> dict:
        s = self.spec
        return dict(kmesh=tuple(s.kmesh), nk=s.nk, nao=s.nao, naux=s.naux, ntau=s.ntau,
                    nw_f=len(self.grid.nf), nw_b=len(self.grid.nb), nspin=s.nspin, beta=s.beta)


def make_H0(spec: SystemSpec) -> np.ndarray:
    nk, nao, ns = spec.nk, spec.nao, spec.nspin
    neg = k_neg(spec.kmesh)
    H = np.zeros((ns, nk, nao, nao), dtype=np.complex128)
    for s in range(ns):
        for k in range(nk):
            if spec.f_time_reversal:
                kn = int(neg[k])
                if kn < k:
                    H[s, k] = H[s, kn].conj()
                    continue
                real = kn == k  # time-reversal-invariant momentum: H0 must be real
            else:
                real = False
            H[s, k] = random_hermitian_spectrum(spec.seed, rng.TAG_F, s, k, nao, -spec.band, spec.band, real)
    return H


def make_S(spec: SystemSpec) -> np.ndarray:
    nk, nao = spec.nk, spec.nao
    S = np.zeros((nk, nao, nao), dtype=np.complex128)
    neg = k_neg(spec.kmesh)
    for k in range(nk):
        if spec.s_identity:
            S[k] = np.eye(nao)
            continue
        kn = int(neg[k])
        if kn < k:
            S[k] = S[kn].conj()
            continue
        real = kn == k
        h = random_hermitian_spectrum(spec.seed, rng.TAG_S, 0, k, nao, -1.0, 1.0, real)
        S[k] = np.eye(nao) + 0.1 * h
    return S


def _v_block(spec: SystemSpec, k1: int, k2: int) -> np.ndarray:
    """Raw complex Gaussian block Z for the ordered pair (k1, k2), scaled by a e^{-decay Q}."""
    Z = rng.complex_normals(rng.stream_key(spec.seed, rng.TAG_V, 0, k1, k2), (spec.naux, spec.nao, spec.nao))
    env = spec.amp * np.exp(-spec.v_decay * np.arange(spec.naux))
    return Z * env[:, None, None]


def make_V(spec: SystemSpec) -> np.ndarray:
    """V[q][k] = V^{k,k+q}(Q) with Hermitian pairing V^{k2,k1}(Q) = V^{k1,k2}(Q)^H."""
    nk = spec.nk
    add = k_add_table(spec.kmesh)
    full = {}
    for k1 in range(nk):
        for k2 in range(k1, nk):
            Z = _v_block(spec, k1, k2)
            if k1 == k2:
                Z = 0.5 * (Z + np.conj(np.swapaxes(Z, 1, 2)))
            full[(k1, k2)] = Z
            if k1 != k2:
                full[(k2, k1)] = np.conj(np.swapaxes(Z, 1, 2))
    if spec.v_time_reversal:
        full = _impose_v_time_reversal(spec, full)
    V = np.empty((nk, nk, spec.naux, spec.nao, spec.nao), dtype=np.complex128)
    sub = k_sub_table(spec.kmesh)
    for q in range(nk):
        for k in range(nk):
            V[q, k] = full[(k, int(add[k, q]))]
    del sub
    return V


def _impose_v_time_reversal(spec: SystemSpec, full: dict) -> dict:
    """Group-average so that V^{-k1,-k2}(Q) = conj V^{k1,k2}(Q) and the Hermitian pairing both hold.

    The group {id, dagger-swap, conj-negate, transpose} acts on the set of
    blocks; averaging over each orbit keeps both symmetries exact.
    """
    neg = k_neg(spec.kmesh)
    out = {}
    for (k1, k2), Z in full.items():
        a = Z
        b = np.conj(np.swapaxes(full[(k2, k1)], 1, 2))  # dagger of the swapped block
        c = np.conj(full[(int(neg[k1]), int(neg[k2]))])  # conj of the negated pair
        d = np.swapaxes(full[(int(neg[k2]), int(neg[k1]))], 1, 2)  # transpose of the negated swap
        out[(k1, k2)] = 0.25 * (a + b + c + d)
    return out


def fermi(x: np.ndarray, beta: float) -> np.ndarray:
    return 0.5 * (1.0 - np.tanh(0.5 * beta * x))


def noninteracting_G(H0: np.ndarray, S: np.ndarray, tau: np.ndarray, beta: float, mu: float) -> np.ndarray:
    """Closed-form G0[s][t][k] = -C diag(e^{-x tau}/(1+e^{-beta x})) C^H, x = e - mu, H C = S C e."""
    ns, nk, nao, _ = H0.shape
    ntau = len(tau)
    G = np.zeros((ns, ntau, nk, nao, nao), dtype=np.complex128)
    for s in range(ns):
        for k in range(nk):
            e, C = scipy.linalg.eigh(H0[s, k], S[k])
            x = e - mu
            # e^{-x tau} / (1 + e^{-beta x}) computed without overflow
            logw = -np.outer(tau, x) - np.logaddexp(0.0, -beta * x)[None, :]
            w = np.exp(logw)  # [ntau, nao]
            G[s, :, k] = -np.einsum("ia,ta,ja->tij", C, w, C.conj())
    return G


def electron_count(H0: np.ndarray, S: np.ndarray, beta: float, mu: float) -> float:
    """N = (2/ns)(1/nk) sum_{s,k} sum_a f(e_a - mu): the electron count of the closed-form G0."""
    ns, nk = H0.shape[:2]
    tot = 0.0
    for s in range(ns):
        for k in range(nk):
            e = scipy.linalg.eigh(H0[s, k], S[k], eigvals_only=True)
            tot += fermi(e - mu, beta).sum()
    return 2.0 / ns * tot / nk


def make_system(spec: SystemSpec, with_V: bool = True) -> System:
    grid = make_grid(spec.ntau, spec.beta)
    H0 = make_H0(spec)
    S = make_S(spec)
    V = make_V(spec) if with_V else None
    G0 = noninteracting_G(H0, S, grid.tau, spec.beta, spec.mu0)
    n_target = electron_count(H0, S, spec.beta, spec.mu0)
    return System(spec, grid, H0, S, V, G0, n_target, spec.mu0)


def random_polarization(seed: int, nk: int, ntau: int, naux: int, scale: float = 0.05) -> np.ndarray:
    """A seeded Hermitian-in-(Q,Q') test input P[q][t][Q][Q'] for exercising the self-energy step alone."""
    P = np.empty((nk, ntau, naux, naux), dtype=np.complex128)
    for q in range(nk):
        for t in range(ntau):
            z = rng.complex_normals(rng.stream_key(seed, rng.TAG_P, 0, q, t), (naux, naux))
            P[q, t] = -scale * 0.5 * (z + z.conj().T) / np.sqrt(naux)
    return P


def random_green(seed: int, ns: int, ntau: int, nk: int, nao: int, scale: float = 0.1) -> np.ndarray:
    """A seeded Hermitian-per-(s,t,k) test input G[s][t][k] (not a physical Green's function)."""
    G = np.empty((ns, ntau, nk, nao, nao), dtype=np.complex128)
    for s in range(ns):
        for t in range(ntau):
            for k in range(nk):
                z = rng.complex_normals(rng.stream_key(seed, rng.TAG_G, s, t, k), (nao, nao))
                G[s, t, k] = -scale * 0.5 * (z + z.conj().T)
    return G
