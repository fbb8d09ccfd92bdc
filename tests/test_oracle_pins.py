"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU).

None of these re-types an oracle formula: each compares the oracle with a
closed form, an independent formulation (four-index pair space, the GF2
direct term of Eq. sigma2, explicit (ij|kl) integrals), a limit (MP2) or an
invariant.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

from oracle import gw
from synth import configs, grid as gridmod, systems


def _km(kmesh):
    return gw.KMesh(kmesh)


def _V4(V, km, k1, k2, k3, k4):
    """(k1 i, k2 j | k3 k, k4 l) = sum_Q V^{k1,k2}_{ij}(Q) V^{k3,k4}_{kl}(Q)  (Eq. CoulombDF)."""
    A = gw.V_pair(V, km, k1, k2)
    B = gw.V_pair(V, km, k3, k4)
    return np.einsum("Qij,Qkl->ijkl", A, B)


# ============================================================================ brute force (tiny)
@pytest.fixture(scope="module")
def tiny8():
    sp = configs.tiny(kmesh=(2, 2, 2), nao=2, naux=3, ntau=6, beta=5.0, seed=31)
    s = systems.make_system(sp)
    G = systems.random_green(77, 1, sp.ntau, sp.nk, sp.nao, scale=0.3)
    return s, G


def test_polarization_brute_force(tiny8):
    """Six-index loop over (k, a, b, c, d) per (q, t, Q, Q') with explicit momentum lookups."""
    s, G = tiny8
    km = _km(s.spec.kmesh)
    P = gw.polarization(s.V, G, s.spec.kmesh)
    nk, ntau, naux, nao = s.spec.nk, s.spec.ntau, s.spec.naux, s.spec.nao
    for q, t in [(0, 0), (3, 2), (7, 5), (5, 1)]:
        ref = np.zeros((naux, naux), dtype=complex)
        for Q, Qp, k in itertools.product(range(naux), range(naux), range(nk)):
            kq = km.add(k, q)
            Vl = gw.V_pair(s.V, km, k, kq)[Q]
            Vr = gw.V_pair(s.V, km, kq, k)[Qp]
            acc = 0.0
            for a, b, c, d in itertools.product(range(nao), repeat=4):
                acc += Vl[d, a] * G[0, ntau - 1 - t, k][c, d] * G[0, t, kq][a, b] * Vr[b, c]
            ref[Q, Qp] += -2.0 / nk * acc
        assert np.allclose(P[q, t], ref, atol=1e-14, rtol=1e-13)


def test_selfenergy_brute_force(tiny8):
    """Explicit four-index W~_{iabj} = sum_QQ' V V P V, then Sigma = -(1/Nk) sum_q sum_ab G W~ (Eq. sigma_gw)."""
    s, G = tiny8
    km = _km(s.spec.kmesh)
    nk, nao = s.spec.nk, s.spec.nao
    Pt = systems.random_polarization(5, nk, s.spec.ntau, s.spec.naux, scale=0.2)
    Sig = gw.selfenergy(s.V, G, Pt, s.spec.kmesh)
    for k, t in [(0, 0), (6, 3), (3, 5)]:
        ref = np.zeros((nao, nao), dtype=complex)
        for q in range(nk):
            kmq = km.sub(k, q)
            W = np.einsum("Qia,QR,Rbj->iabj", gw.V_pair(s.V, km, k, kmq), Pt[q, t], gw.V_pair(s.V, km, kmq, k))
            for i, j, a, b in itertools.product(range(nao), repeat=4):
                ref[i, j] += -1.0 / nk * G[0, t, kmq][a, b] * W[i, a, b, j]
        assert np.allclose(Sig[0, t, k], ref, atol=1e-15, rtol=1e-13)


def test_sigma_inf_against_explicit_coulomb(tiny8):
    """Eq. sigma_inf from explicit (ij|kl) integrals: J - K with G(0^-) = -G(beta^-)."""
    s, G = tiny8
    km = _km(s.spec.kmesh)
    nk, nao = s.spec.nk, s.spec.nao
    Sinf = gw.sigma_inf(s.V, G, s.spec.kmesh)
    gam = -G[0, -1]
    for k in range(nk):
        ref = np.zeros((nao, nao), dtype=complex)
        for kp in range(nk):
            J = _V4(s.V, km, k, k, kp, kp)  # (k i, k j | k' b, k' a)
            K = _V4(s.V, km, k, kp, kp, k)  # (k i, k' a | k' b, k j)
            ref += 2.0 / nk * np.einsum("ijba,ab->ij", J, gam[kp])
            ref -= 1.0 / nk * np.einsum("iabj,ab->ij", K, gam[kp])
        assert np.allclose(Sinf[0, k], ref, atol=1e-15, rtol=1e-13)


def test_unrestricted_spin_sums():
    """nspin = 2 with two equal channels reproduces the restricted run (spin factor reading)."""
    sp = configs.tiny(kmesh=(2, 1, 1), nao=3, naux=4, ntau=8, beta=6.0, seed=12)
    s = systems.make_system(sp)
    G1 = s.G0
    G2 = np.concatenate([G1, G1], axis=0)
    assert np.allclose(gw.polarization(s.V, G1, sp.kmesh), gw.polarization(s.V, G2, sp.kmesh), atol=1e-15)
    S1 = gw.sigma_inf(s.V, G1, sp.kmesh)
    S2 = gw.sigma_inf(s.V, G2, sp.kmesh)
    assert np.allclose(S2[0], S1[0], atol=1e-15) and np.allclose(S2[1], S1[0], atol=1e-15)


# ============================================================================ closed forms
def test_single_level_closed_form():
    """Nk = nao = naux = 1, real v, level e, mu = 0:
    P0 = -2 v^2 f (1-f) (constant), P~(tau) = P0 / (1 - beta P0), Sigma~(tau) = (1-f) e^{-e tau} v^2 P~."""
    for beta, eps, v, ntau in [(10.0, 0.3, 0.4, 8), (50.0, -0.05, 0.7, 20), (20.0, 0.0, 1.1, 12)]:
        g = gridmod.make_grid(ntau, beta)
        H0 = np.full((1, 1, 1, 1), eps, dtype=complex)
        S = np.ones((1, 1, 1), dtype=complex)
        V = np.full((1, 1, 1, 1, 1), v, dtype=complex)
        G0 = systems.noninteracting_G(H0, S, g.tau, beta, 0.0)
        f = 1.0 / (1.0 + np.exp(beta * eps))
        p0 = -2.0 * v * v * f * (1.0 - f)
        P0 = gw.polarization(V, G0, (1, 1, 1))
        assert np.allclose(P0[0, :, 0, 0], p0, rtol=1e-13, atol=1e-15)
        Pt = gw.from_bosonic(gw.screen(gw.to_bosonic(P0, g.TB_t2w)), g.TB_w2t)
        pt = p0 / (1.0 - beta * p0)
        assert np.allclose(Pt[0, :, 0, 0], pt, rtol=1e-11, atol=1e-15)
        Sig = gw.selfenergy(V, G0, Pt, (1, 1, 1))
        ref = (1.0 - f) * np.exp(-eps * g.tau) * v * v * pt
        assert np.allclose(Sig[0, :, 0, 0, 0], ref, rtol=1e-11, atol=1e-16)


def test_lindhard_closed_form():
    """Non-interacting bubble: P0^q(i W_n) = (2/Nk) sum_k sum_{a in k+q, c in k}
    M^Q_{ca} conj(M^{Q'}_{ca}) (f_a - f_c)/(e_a - e_c - i W_n), M^Q = C_c^H V^{k,k+q}(Q) C'_a,
    with the limit -beta f(1-f) at e_a = e_c, W = 0."""
    sp = configs.tiny(kmesh=(2, 2, 1), nao=3, naux=4, ntau=48, beta=10.0, band=1.0, seed=41)
    s = systems.make_system(sp)
    km = _km(sp.kmesh)
    P0 = gw.polarization(s.V, s.G0, sp.kmesh)
    Pw = gw.to_bosonic(P0, s.grid.TB_t2w)
    eig = [scipy.linalg.eigh(s.H0[0, k], s.S[k]) for k in range(sp.nk)]
    beta = sp.beta
    for q in range(sp.nk):
        for m in [0, len(s.grid.nb) // 2, len(s.grid.nb) // 2 + 3, len(s.grid.nb) - 1]:
            W = s.grid.wb[m]
            ref = np.zeros((sp.naux, sp.naux), dtype=complex)
            for k in range(sp.nk):
                kq = km.add(k, q)
                ec, Cc = eig[k]
                ea, Ca = eig[kq]
                fc = systems.fermi(ec, beta)
                fa = systems.fermi(ea, beta)
                M = np.einsum("ic,Qij,ja->Qca", Cc.conj(), gw.V_pair(s.V, km, k, kq), Ca)
                den = ea[None, :] - ec[:, None] - 1j * W
                with np.errstate(divide="ignore", invalid="ignore"):
                    fac = (fa[None, :] - fc[:, None]) / den
                deg = np.abs(den) < 1e-12
                fac[deg] = (-beta * fa[None, :] * (1 - fa[None, :]) * np.ones_like(den))[deg]
                ref += 2.0 / sp.nk * np.einsum("Qca,Rca,ca->QR", M, M.conj(), fac)
            assert np.max(np.abs(Pw[q, m] - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref)))


def test_pair_space_bubble_series():
    """RPA in the four-index pair space, with no auxiliary index: W~ = U_L chi [I - U chi]^{-1} U_R.

    For each q and bosonic node, chi^q_{(k',d,a),(k',b,c)}(i W) is the Fourier image of
    -(2/Nk) G^{k'}_{cd}(beta - tau) G^{k'+q}_{ab}(tau) and U, U_L, U_R are explicit (ij|kl)
    integrals.  By the push-through identity this equals sum_QQ' V P~ V of Eq. tilde_W_DF2.
    Sigma~ = -(1/Nk) sum_q sum_ab G^{k-q}(tau) W~(tau) is compared with the oracle.
    """
    sp = configs.tiny(kmesh=(2, 1, 1), nao=2, naux=3, ntau=12, beta=4.0, seed=51, v_scale=0.6)
    s = systems.make_system(sp)
    km = _km(sp.kmesh)
    nk, nao, ntau = sp.nk, sp.nao, sp.ntau
    g = s.grid
    G = s.G0
    Sinf, Sig, inter = gw.sigma_eval(s.V, G, sp.kmesh, g)
    npair = nk * nao * nao
    Wt = np.zeros((nk, nk, ntau, nao, nao, nao, nao), dtype=complex)  # [k][q][t][i][a][b][j]
    for q in range(nk):
        # chi(tau) in pair space, block diagonal over k'
        chi_t = np.zeros((ntau, npair, npair), dtype=complex)
        for kp in range(nk):
            kq = km.add(kp, q)
            for t in range(ntau):
                blk = -2.0 / nk * np.einsum("cd,ab->dabc", G[0, ntau - 1 - t, kp], G[0, t, kq])
                sl = slice(kp * nao * nao, (kp + 1) * nao * nao)
                chi_t[t, sl, sl] = blk.reshape(nao * nao, nao * nao)
        chi_w = np.einsum("mt,tab->mab", g.TB_t2w, chi_t)
        # U[(k',b,c),(k'',d,a)] = (k'+q b, k' c | k'' d, k''+q a)
        U = np.zeros((npair, npair), dtype=complex)
        for k1 in range(nk):
            for k2 in range(nk):
                blk = _V4(s.V, km, km.add(k1, q), k1, k2, km.add(k2, q))  # [b][c][d][a]
                U[k1 * nao * nao:(k1 + 1) * nao * nao, k2 * nao * nao:(k2 + 1) * nao * nao] = blk.reshape(
                    nao * nao, nao * nao)
        for k in range(nk):
            kmq = km.sub(k, q)
            # UL[(i,a),(k'',d,a')] = (k i, k-q a | k'' d, k''+q a');  UR[(k',b,c),(b',j)] = (k'+q b, k' c | k-q b', k j)
            UL = np.zeros((nao * nao, npair), dtype=complex)
            UR = np.zeros((npair, nao * nao), dtype=complex)
            for k2 in range(nk):
                UL[:, k2 * nao * nao:(k2 + 1) * nao * nao] = _V4(s.V, km, k, kmq, k2, km.add(k2, q)).reshape(
                    nao * nao, nao * nao)
                UR[k2 * nao * nao:(k2 + 1) * nao * nao, :] = _V4(s.V, km, km.add(k2, q), k2, kmq, k).reshape(
                    nao * nao, nao * nao)
            Ww = np.stack([UL @ chi_w[m] @ np.linalg.solve(np.eye(npair) - U @ chi_w[m], UR)
                           for m in range(chi_w.shape[0])])
            Wtau = np.einsum("tm,mab->tab", g.TB_w2t, Ww)  # [t][(i,a)][(b,j)]
            Wt[k, q] = Wtau.reshape(ntau, nao, nao, nao, nao)
    ref = np.zeros_like(Sig)
    for k in range(nk):
        for q in range(nk):
            kmq = km.sub(k, q)
            ref[0, :, k] += -1.0 / nk * np.einsum("tab,tiabj->tij", G[0, :, kmq], Wt[k, q])
    assert np.max(np.abs(Sig - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("kmesh", [(1, 1, 1), (2, 2, 2)])
def test_first_order_equals_gf2_direct(kmesh):
    """Feeding P~ := P0(tau) into Sigma~ gives the direct term of Eq. sigma2, evaluated literally with
    the antiperiodic G(-tau) = -G(beta - tau) and the lattice delta read as Nk times a Kronecker delta."""
    sp = configs.tiny(kmesh=kmesh, nao=2, naux=2, ntau=6, beta=3.0, seed=61)
    s = systems.make_system(sp)
    km = _km(kmesh)
    G = systems.random_green(8, 1, sp.ntau, sp.nk, sp.nao, scale=0.4)
    nk, nao, ntau = sp.nk, sp.nao, sp.ntau
    P0 = gw.polarization(s.V, G, kmesh)
    Sig = gw.selfenergy(s.V, G, P0, kmesh)
    for k, t in [(0, 1), (nk - 1, 4), (nk // 2, 0)]:
        ref = np.zeros((nao, nao), dtype=complex)
        for k1, k2, k3 in itertools.product(range(nk), repeat=3):
            if km.add(k, k3) != km.add(k1, k2):
                continue
            Gm = -G[0, ntau - 1 - t, k3]  # G^{k3}(-tau)
            for Q, Qp in itertools.product(range(sp.naux), repeat=2):
                Va = gw.V_pair(s.V, km, k1, k)[Qp]  # V^{k1 k}_{qj}(Q')
                Vb = gw.V_pair(s.V, km, k2, k3)[Qp]  # V^{k2 k3}_{ln}(Q')
                Vc = gw.V_pair(s.V, km, k, k1)[Q]  # V^{k k1}_{ip}(Q)
                Vd = gw.V_pair(s.V, km, k3, k2)[Q]  # V^{k3 k2}_{mk}(Q)
                for i, j in itertools.product(range(nao), repeat=2):
                    acc = 0.0
                    for kk, l, m, n, p, qq in itertools.product(range(nao), repeat=6):
                        acc += (Va[qq, j] * Vb[l, n] * Vc[i, p] * Vd[m, kk]
                                * G[0, t, k1][p, qq] * G[0, t, k2][kk, l] * Gm[n, m])
                    ref[i, j] += 2.0 * acc  # sum over sigma' (restricted)
        ref *= -1.0 / nk ** 2  # 1/Nk^3 times the lattice delta Nk
        assert np.allclose(Sig[0, t, k], ref, atol=1e-15, rtol=1e-12)


def test_mp2_direct_limit():
    """Gapped G0, Nk = 1, beta = 100: E_corr[Sigma^(1)[G0], G0] -> 2 E_MP2(direct),
    E_MP2(direct) = -2 sum_{ij occ, ab virt} (ia|jb)(ai|bj)/(e_a + e_b - e_i - e_j)
    (the Galitskii-Migdal interaction energy is twice the second-order energy)."""
    beta, ntau = 100.0, 104
    g = gridmod.make_grid(ntau, beta)
    rng = np.random.default_rng(3)
    e = np.array([-0.9, -0.55, -0.3, 0.3, 0.6, 1.0])
    n = len(e)
    U = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))[0]
    H0 = ((U * e) @ U.conj().T)[None, None]
    S = np.eye(n, dtype=complex)[None]
    Z = (rng.normal(size=(4, n, n)) + 1j * rng.normal(size=(4, n, n))) * 0.1
    V = (0.5 * (Z + np.conj(np.swapaxes(Z, 1, 2))))[None, None]
    G0 = systems.noninteracting_G(H0, S, g.tau, beta, 0.0)
    P0 = gw.polarization(V, G0, (1, 1, 1))
    Sig = gw.selfenergy(V, G0, P0, (1, 1, 1))
    E = gw.energy(G0, H0, np.zeros_like(H0), Sig, beta)
    Vmo = np.einsum("ia,Qij,jb->Qab", U.conj(), V[0, 0], U)
    occ, vir = [0, 1, 2], [3, 4, 5]
    emp2 = 0.0
    for i, j, a, b in itertools.product(occ, occ, vir, vir):
        iajb = np.sum(Vmo[:, i, a] * Vmo[:, j, b])
        aibj = np.sum(Vmo[:, a, i] * Vmo[:, b, j])
        emp2 += -2.0 * (iajb * aibj).real / (e[a] + e[b] - e[i] - e[j])
    assert abs(E["e_corr"] - 2.0 * emp2) < 1e-9 * abs(emp2) + 1e-13


def test_two_level_worked_example():
    """One occupied and one virtual level, one auxiliary function with V_ia = V_ai = v:
    E_corr -> -2 v^4 / (e_a - e_i) (twice the MP2 value -v^4 / (e_a - e_i))."""
    beta, ntau = 100.0, 104
    g = gridmod.make_grid(ntau, beta)
    ei, ea, v = -0.5, 0.4, 0.3
    H0 = np.diag([ei, ea]).astype(complex)[None, None]
    V = np.array([[[0.0, v], [v, 0.0]]], dtype=complex)[None, None]
    S = np.eye(2, dtype=complex)[None]
    G0 = systems.noninteracting_G(H0, S, g.tau, beta, 0.0)
    Sig = gw.selfenergy(V, G0, gw.polarization(V, G0, (1, 1, 1)), (1, 1, 1))
    E = gw.energy(G0, H0, np.zeros_like(H0), Sig, beta)
    assert abs(E["e_corr"] - (-2.0 * v ** 4 / (ea - ei))) < 1e-11


@pytest.mark.parametrize("kmesh,nspin,nao", [((1, 1, 1), 1, 3), ((3, 1, 1), 2, 2), ((2, 2, 1), 1, 2)])
def test_gf2_brute_force(kmesh, nspin, nao):
    """Eq. sigma2 as printed, with explicit loops over every momentum, orbital, spin and auxiliary index,
    the lattice delta read as Nk times a Kronecker delta and G(-tau) = -G(beta - tau)."""
    sp = configs.tiny(kmesh=kmesh, nao=nao, naux=2, ntau=6, beta=3.0, nspin=nspin, seed=83)
    s = systems.make_system(sp)
    km = _km(kmesh)
    G = systems.random_green(19, nspin, sp.ntau, sp.nk, nao, scale=0.4)
    nk, ntau = sp.nk, sp.ntau
    Sig = gw.gf2_selfenergy(s.V, G, kmesh)
    spins = [(sq, 1.0) for sq in range(nspin)] if nspin == 2 else [(0, 1.0), (0, 1.0)]  # sigma' channels
    for sig, k, t in [(0, 0, 1), (nspin - 1, nk - 1, 4), (0, nk // 2, 0)]:
        ref = np.zeros((nao, nao), dtype=complex)
        for k1, k2, k3 in itertools.product(range(nk), repeat=3):
            if km.add(k, k3) != km.add(k1, k2):
                continue
            for Q, Qp in itertools.product(range(sp.naux), repeat=2):
                V1 = gw.V_pair(s.V, km, k1, k)[Qp]   # V^{k1 k}_{qj}(Q')
                V2 = gw.V_pair(s.V, km, k2, k3)[Qp]  # V^{k2 k3}_{ln}(Q')
                V3 = gw.V_pair(s.V, km, k2, k)[Qp]   # V^{k2 k}_{lj}(Q')
                V4 = gw.V_pair(s.V, km, k1, k3)[Qp]  # V^{k1 k3}_{qn}(Q')
                V5 = gw.V_pair(s.V, km, k, k1)[Q]    # V^{k k1}_{ip}(Q)
                V6 = gw.V_pair(s.V, km, k3, k2)[Q]   # V^{k3 k2}_{mk}(Q)
                for ic, (sp2, _) in enumerate(spins):
                    same = (ic == 0) if nspin == 1 else (sp2 == sig)
                    G1 = G[sig, t, k1]
                    G2 = G[sp2, t, k2]
                    G3 = -G[sp2, ntau - 1 - t, k3]  # G^{k3}_{sigma'}(-tau)
                    for i, j in itertools.product(range(nao), repeat=2):
                        acc = 0.0
                        for kk, l, m, n, p_, qq in itertools.product(range(nao), repeat=6):
                            bra = V1[qq, j] * V2[l, n] - (V3[l, j] * V4[qq, n] if same else 0.0)
                            acc += bra * V5[i, p_] * V6[m, kk] * G1[p_, qq] * G2[kk, l] * G3[n, m]
                        ref[i, j] += acc
        ref *= -nk / nk ** 3  # 1/Nk^3 times the lattice delta Nk
        assert np.allclose(Sig[sig, t, k], ref, atol=1e-15, rtol=1e-12)


def test_gf2_single_orbital_closed_form():
    """One orbital, one k, restricted: the exchange term is half the direct one, so
    Sigma~(2)(tau) = -u^2 G(tau)^2 G(-tau) = u^2 G(tau)^2 G(beta - tau) with u = sum_Q V_Q^2."""
    sp = configs.tiny(kmesh=(1, 1, 1), nao=1, naux=3, ntau=8, beta=4.0, seed=5)
    s = systems.make_system(sp)
    G = systems.random_green(23, 1, sp.ntau, 1, 1, scale=0.5)
    Sig = gw.gf2_selfenergy(s.V, G, (1, 1, 1))
    u = np.sum(s.V[0, 0, :, 0, 0] ** 2)
    g = G[0, :, 0, 0, 0]
    ref = u ** 2 * g ** 2 * g[::-1]
    assert np.allclose(Sig[0, :, 0, 0, 0], ref, atol=1e-15, rtol=1e-12)


def _gapped_molecule(seed=3):
    rng = np.random.default_rng(seed)
    e = np.array([-0.9, -0.55, -0.3, 0.3, 0.6, 1.0])
    n = len(e)
    U = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))[0]
    H0 = ((U * e) @ U.conj().T)[None, None]
    Z = (rng.normal(size=(4, n, n)) + 1j * rng.normal(size=(4, n, n))) * 0.1
    V = (0.5 * (Z + np.conj(np.swapaxes(Z, 1, 2))))[None, None]
    return e, U, H0, V


def test_gf2_mp2_limit():
    """Gapped G0, Nk = 1, beta = 100: E_corr[Sigma(2)[G0], G0] -> 2 E_MP2 with the exchange term,
    E_MP2 = sum_{ij occ, ab virt} (ia|jb) [2 (ai|bj) - (bi|aj)] / (e_i + e_j - e_a - e_b),
    (pq|rs) = sum_Q V_pq(Q) V_rs(Q) in the eigenbasis of H0."""
    beta, ntau = 100.0, 104
    g = gridmod.make_grid(ntau, beta)
    e, U, H0, V = _gapped_molecule()
    n = len(e)
    S = np.eye(n, dtype=complex)[None]
    G0 = systems.noninteracting_G(H0, S, g.tau, beta, 0.0)
    Sig = gw.gf2_selfenergy(V, G0, (1, 1, 1))
    E = gw.energy(G0, H0, np.zeros_like(H0), Sig, beta)
    Vmo = np.einsum("ia,Qij,jb->Qab", U.conj(), V[0, 0], U)
    occ, vir = [0, 1, 2], [3, 4, 5]
    emp2 = 0.0
    for i, j, a, b in itertools.product(occ, occ, vir, vir):
        iajb = np.sum(Vmo[:, i, a] * Vmo[:, j, b])
        aibj = np.sum(Vmo[:, a, i] * Vmo[:, b, j])
        biaj = np.sum(Vmo[:, b, i] * Vmo[:, a, j])
        emp2 += (iajb * (2.0 * aibj - biaj)).real / (e[i] + e[j] - e[a] - e[b])
    assert abs(E["e_corr"] - 2.0 * emp2) < 1e-9 * abs(emp2) + 1e-13


def test_gf2_two_level_worked_example():
    """One occupied and one virtual level, one auxiliary function with V_ia = V_ai = v: the exchange term
    cancels half of the direct one, E_corr -> -v^4 / (e_a - e_i) (twice MP2's -v^4 / (2 (e_a - e_i)))."""
    beta, ntau = 100.0, 104
    g = gridmod.make_grid(ntau, beta)
    ei, ea, v = -0.5, 0.4, 0.3
    H0 = np.diag([ei, ea]).astype(complex)[None, None]
    V = np.array([[[0.0, v], [v, 0.0]]], dtype=complex)[None, None]
    S = np.eye(2, dtype=complex)[None]
    G0 = systems.noninteracting_G(H0, S, g.tau, beta, 0.0)
    Sig = gw.gf2_selfenergy(V, G0, (1, 1, 1))
    E = gw.energy(G0, H0, np.zeros_like(H0), Sig, beta)
    assert abs(E["e_corr"] - (-v ** 4 / (ea - ei))) < 1e-11


def test_gf2_direct_part_is_the_first_order_bubble():
    """The direct part of Eq. sigma2 is the first-order bubble: Sigma(2) plus (1/Nk^2) times the exchange
    part, the latter contracted from explicit four-index integrals (ab|cd) = sum_Q V_ab(Q) V_cd(Q), equals
    O7 fed P~ := P0."""
    sp = configs.tiny(kmesh=(2, 1, 1), nao=3, naux=4, ntau=6, beta=3.0, seed=29)
    s = systems.make_system(sp)
    km = _km(sp.kmesh)
    G = systems.random_green(41, 1, sp.ntau, sp.nk, sp.nao, scale=0.4)
    nk, ntau, nao = sp.nk, sp.ntau, sp.nao
    Sig2 = gw.gf2_selfenergy(s.V, G, sp.kmesh)
    first = gw.selfenergy(s.V, G, gw.polarization(s.V, G, sp.kmesh), sp.kmesh)
    for k, t in [(0, 2), (1, 5)]:
        ex = np.zeros((nao, nao), dtype=complex)
        for k1, k2 in itertools.product(range(nk), repeat=2):
            k3 = km.sub(km.add(k1, k2), k)
            # four-index integrals (ab|cd) = sum_Q V_ab(Q) V_cd(Q) of the exchange chain
            U1 = np.einsum("Qip,Qmk->ipmk", gw.V_pair(s.V, km, k, k1), gw.V_pair(s.V, km, k3, k2))
            U2 = np.einsum("Qqn,Qlj->qnlj", gw.V_pair(s.V, km, k1, k3), gw.V_pair(s.V, km, k2, k))
            ex += np.einsum("ipmk,qnlj,pq,kl,nm->ij", U1, U2, G[0, t, k1], G[0, t, k2],
                            -G[0, ntau - 1 - t, k3])
        # Sigma(2) = -(1/Nk^2)(direct - exchange)  =>  Sigma(2) - (1/Nk^2) exchange = first order
        assert np.allclose(Sig2[0, t, k] - ex / nk ** 2, first[0, t, k], atol=1e-15, rtol=1e-12)


def test_energy_integral_closed_form():
    """int_0^beta Tr[F(tau) H(beta - tau)] for F = e^{-x tau}, H = e^{-y tau} (1x1): closed form."""
    beta, ntau = 20.0, 64
    g = gridmod.make_grid(ntau, beta)
    x, y = 0.3, -0.2
    F = np.exp(-x * g.tau)[:, None, None, None].astype(complex)
    H = np.exp(-y * g.tau)[:, None, None, None].astype(complex)
    got = gw.tau_integral_product(F, H, beta)
    # int_0^beta e^{-x tau} e^{-y (beta - tau)} = e^{-y beta} (e^{(y - x) beta} - 1) / (y - x)
    ref = np.exp(-y * beta) * (np.exp((y - x) * beta) - 1.0) / (y - x)
    assert abs(got - ref) < 1e-11 * abs(ref)


def test_noninteracting_dyson_closed_form():
    """Sigma = 0: Dyson + mu search + TF_w2t reproduce G0(tau) = -C diag(e^{-x tau}/(1+e^{-beta x})) C^H
    for a general overlap S, N(mu*) = N_target, and G(0+) + G(beta-) = -S^{-1}."""
    sp = configs.tiny(kmesh=(2, 1, 1), nao=5, naux=3, ntau=48, beta=50.0, band=1.0, s_identity=False, seed=71)
    s = systems.make_system(sp)
    zero_inf = np.zeros_like(s.H0)
    zero_tau = np.zeros((1, sp.ntau, sp.nk, sp.nao, sp.nao), dtype=complex)
    G, mu, n = gw.solve_dyson(s.H0, s.S, zero_inf, zero_tau, s.grid, sp.nspin, 0.37, s.n_target)
    assert abs(n - s.n_target) <= 1e-12 * s.n_target
    assert abs(mu - 0.0) < 1e-8
    assert np.max(np.abs(G - s.G0)) < 1e-10
    for k in range(sp.nk):
        assert np.allclose(G[0, 0, k] + G[0, -1, k], -np.linalg.inv(s.S[k]), atol=1e-10)


def test_mu_search_hits_target():
    """Shifting the target electron count moves mu to the closed-form root of sum_a f(e_a - mu)."""
    sp = configs.tiny(kmesh=(1, 1, 1), nao=6, naux=3, ntau=48, beta=20.0, band=1.0, seed=81)
    s = systems.make_system(sp)
    e = np.linalg.eigvalsh(s.H0[0, 0])
    target = 2.0 * np.sum(systems.fermi(e - 0.123, sp.beta))
    z_inf = np.zeros_like(s.H0)
    z_tau = np.zeros((1, sp.ntau, 1, sp.nao, sp.nao), dtype=complex)
    G, mu, n = gw.solve_dyson(s.H0, s.S, z_inf, z_tau, s.grid, 1, 0.0, target)
    assert abs(mu - 0.123) < 1e-9
    assert abs(n - target) < 1e-11


# ============================================================================ invariants
@pytest.fixture(scope="module")
def physical():
    sp = configs.tiny(kmesh=(3, 1, 1), nao=4, naux=6, ntau=32, beta=10.0, band=1.5, seed=91, v_scale=0.3,
                      v_time_reversal=True)
    s = systems.make_system(sp)
    Sinf, Sig, inter = gw.sigma_eval(s.V, s.G0, sp.kmesh, s.grid)
    return s, Sinf, Sig, inter


def test_polarization_invariants(physical):
    s, _, _, inter = physical
    P0, Pw = inter["P0"], inter["Pw"]
    km = _km(s.spec.kmesh)
    neg = systems.k_neg(s.spec.kmesh)
    ntau = s.spec.ntau
    sc = np.max(np.abs(P0))
    # Hermitian in (Q, Q') at every tau
    assert np.max(np.abs(P0 - np.conj(np.swapaxes(P0, -1, -2)))) < 1e-14 * sc * 10
    # P0^q(beta - tau) = P0^{-q}(tau)^T
    for q in range(km.nk):
        assert np.max(np.abs(P0[q, ::-1] - np.swapaxes(P0[neg[q]], -1, -2))) < 1e-13 * sc
    # non-positive diagonal, and Hermitian part of P0(i W) negative semidefinite
    assert np.all(np.einsum("qtaa->qta", P0).real <= 1e-15)
    for q in range(km.nk):
        for m in range(Pw.shape[1]):
            h = 0.5 * (Pw[q, m] + Pw[q, m].conj().T)
            assert np.max(np.linalg.eigvalsh(h)) < 1e-12
            assert np.min(np.linalg.svd(np.eye(h.shape[0]) - Pw[q, m], compute_uv=False)) > 1.0 - 1e-12
    del ntau


def test_screening_residual(physical):
    _, _, _, inter = physical
    Pw, Ptw = inter["Pw"], inter["Ptw"]
    res = Ptw - Pw - np.matmul(Pw, Ptw)
    assert np.max(np.abs(res)) < 1e-14 * max(1.0, np.max(np.abs(Ptw)))


def test_screened_partner_momentum_identity():
    """P~^{-q}(tau) = P~^q(beta - tau)^T after the bosonic transforms and the screening, for inputs without
    time-reversal symmetry (the identity follows from relabelling k -> k + q in the trace and the reflection
    symmetry of the grid; the GPU path screens one q of each +-q pair and copies the partner)."""
    sp = configs.tiny(kmesh=(3, 2, 1), nao=4, naux=6, ntau=16, beta=10.0, seed=93, v_scale=0.3)
    s = systems.make_system(sp)
    neg = systems.k_neg(sp.kmesh)
    P0 = gw.polarization(s.V, s.G0, sp.kmesh)
    Pt = gw.from_bosonic(gw.screen(gw.to_bosonic(P0, s.grid.TB_t2w)), s.grid.TB_w2t)
    sc = np.max(np.abs(Pt))
    assert any(neg[q] != q for q in range(sp.nk))
    for q in range(sp.nk):
        assert np.max(np.abs(Pt[neg[q]] - np.swapaxes(Pt[q][::-1], -1, -2))) < 1e-13 * sc
        assert np.max(np.abs(P0[neg[q]] - np.swapaxes(P0[q][::-1], -1, -2))) < 1e-13 * np.max(np.abs(P0))


def test_selfenergy_symmetries(physical):
    """Hermiticity, causality (diagonal <= 0 with S = I) and time reversal Sigma^{-k} = conj Sigma^k."""
    s, Sinf, Sig, _ = physical
    sc = np.max(np.abs(Sig))
    assert np.max(np.abs(Sig - np.conj(np.swapaxes(Sig, -1, -2)))) < 1e-12 * sc
    assert np.all(np.einsum("stkii->stki", Sig).real <= 1e-15)
    neg = systems.k_neg(s.spec.kmesh)
    for k in range(s.spec.nk):
        assert np.max(np.abs(Sig[:, :, neg[k]] - np.conj(Sig[:, :, k]))) < 1e-12 * sc
        assert np.max(np.abs(Sinf[:, neg[k]] - np.conj(Sinf[:, k]))) < 1e-13


def test_iteration_runs_and_contracts():
    """Config-0-shaped system: 10 iterations, fixed N, shrinking max|dSigma|."""
    s = systems.make_system(configs.MOLECULE)
    st = gw.State(s.G0, None, None, 0.0)
    d = []
    for _ in range(10):
        st, rep, _ = gw.iterate(s, st)
        assert abs(rep["n_elec"] - s.n_target) < 1e-11
        d.append(rep["max_dsigma"])
    assert d[-1] < 1e-2 * d[1]


# ============================================================================ DIIS (Sec. 4.2.2)
def test_diis_two_vector_closed_form():
    """Two residuals: the constrained minimiser of |c r1 + (1 - c) r2| is c = (B22 - B12)/(B11 - 2 B12 + B22)."""
    rng = np.random.default_rng(3)
    r1 = (rng.normal(size=(2, 3)) + 1j * rng.normal(size=(2, 3)), rng.normal(size=4) + 1j * rng.normal(size=4))
    r2 = (rng.normal(size=(2, 3)) + 1j * rng.normal(size=(2, 3)), rng.normal(size=4) + 1j * rng.normal(size=4))
    dot = lambda a, b: sum(np.vdot(x, y).real for x, y in zip(a, b))  # noqa: E731
    B11, B22, B12 = dot(r1, r1), dot(r2, r2), dot(r1, r2)
    c = gw.diis_coefficients([r1, r2])
    assert abs(c[0] - (B22 - B12) / (B11 - 2 * B12 + B22)) < 1e-13
    assert abs(c.sum() - 1.0) < 1e-14
    # it is the minimum: any other affine combination has a larger residual norm
    f = lambda t: dot(tuple(t * a + (1 - t) * b for a, b in zip(r1, r2)), tuple(t * a + (1 - t) * b for a, b in zip(r1, r2)))  # noqa: E731
    assert f(c[0]) <= min(f(c[0] + 1e-3), f(c[0] - 1e-3))


def test_diis_solves_a_linear_fixed_point_in_dim_plus_one_steps():
    """With an unlimited subspace, DIIS on a linear map g(x) = A x + b (vectors x_i = g(y_i), residuals
    r_i = g(y_i) - y_i, next input y = sum c_i x_i) is a Krylov (GMRES-equivalent) method and reaches the
    fixed point after at most D + 1 evaluations, D the dimension of the space the coefficients span: the
    coefficients are real, so a complex d-vector counts as D = 2d real dimensions."""
    rng = np.random.default_rng(4)
    d = 5
    A = 0.3 * (rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d)))
    b = rng.normal(size=d) + 1j * rng.normal(size=d)
    xstar = np.linalg.solve(np.eye(d) - A, b)
    y = np.zeros(d, dtype=complex)
    xs, rs = [], []
    for it in range(2 * d + 1):
        gx = A @ y + b
        xs.append((gx,))
        rs.append((gx - y,))
        c = gw.diis_coefficients(rs) if len(rs) >= 2 else np.array([1.0])
        y = sum(ci * x[0] for ci, x in zip(c, xs))
        if it == 2 * d - 2:
            assert np.max(np.abs(y - xstar)) > 1e-6 * np.max(np.abs(xstar))  # not earlier
    assert np.max(np.abs(y - xstar)) < 1e-9 * np.max(np.abs(xstar))


def test_diis_iteration_converges_faster_than_plain():
    """DIIS reaches the same fixed point as the plain iteration in fewer iterations, and converges at a
    stronger coupling where the plain iteration oscillates."""
    def run(s, diis, n_max=25, tol=1e-9):
        st = gw.State(s.G0, None, None, 0.0)
        hist = gw.DiisHistory(size=5, start=2)
        for it in range(n_max):
            st, rep, _ = gw.iterate_diis(s, st, hist) if diis else gw.iterate(s, st)
            if rep["max_dsigma"] < tol:
                return it + 1, rep
        return n_max + 1, rep
    s = systems.make_system(configs.tiny(kmesh=(1, 1, 1), nao=6, naux=20, ntau=24, beta=20.0, seed=97))
    n_plain, rp = run(s, False)
    n_diis, rd = run(s, True)
    assert n_diis < n_plain <= 25
    assert abs(rp["e_tot"] - rd["e_tot"]) < 1e-8
    s = systems.make_system(configs.tiny(kmesh=(1, 1, 1), nao=6, naux=20, ntau=24, beta=20.0, seed=97,
                                         v_scale=0.2))
    n_plain, rp = run(s, False)
    n_diis, rd = run(s, True)
    assert n_plain > 25 and rp["max_dsigma"] > 1e-3
    assert n_diis <= 25


# ----------------------------------------------------------------------------------------------- k-path
@pytest.mark.parametrize("kmesh", [(2, 3, 1), (4, 1, 3)])
def test_kpath_interpolation_reproduces_mesh_values(kmesh):
    """At mesh points the interpolant of Sec. 2.4 (R over the centred supercell, zone-boundary terms split)
    returns the mesh values exactly."""
    rng = np.random.default_rng(11)
    nk = int(np.prod(kmesh))
    X = rng.normal(size=(2, nk, 3, 3)) + 1j * rng.normal(size=(2, nk, 3, 3))
    pts = [(a / kmesh[0], b / kmesh[1], c / kmesh[2]) for a in range(kmesh[0]) for b in range(kmesh[1])
           for c in range(kmesh[2])]
    Y = gw.kpath_interpolate(X, kmesh, pts)
    assert np.max(np.abs(Y - X)) < 1e-13


@pytest.mark.parametrize("kmesh", [(3, 3, 1), (4, 4, 2)])
def test_kpath_interpolation_exact_for_band_limited_functions(kmesh):
    """X(k) = sum_R C_R e^{2 pi i k.R} with every R strictly inside the supercell is interpolated exactly at
    arbitrary k (closed form)."""
    rng = np.random.default_rng(12)
    Rs = [R for R in itertools.product(*[range(-((n - 1) // 2), (n - 1) // 2 + 1) for n in kmesh])
          if all(abs(r) < n / 2 for r, n in zip(R, kmesh))]
    C = {R: rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2)) for R in Rs}

    def f(k):
        return sum(C[R] * np.exp(2j * np.pi * np.dot(k, R)) for R in Rs)
    mesh = [(a / kmesh[0], b / kmesh[1], c / kmesh[2]) for a in range(kmesh[0]) for b in range(kmesh[1])
            for c in range(kmesh[2])]
    X = np.stack([f(np.array(k)) for k in mesh])
    path = rng.uniform(-1.0, 1.0, size=(9, 3))
    Y = gw.kpath_interpolate(X, kmesh, path)
    ref = np.stack([f(k) for k in path])
    assert np.max(np.abs(Y - ref)) < 1e-12 * np.max(np.abs(ref))


def test_kpath_interpolation_against_fft():
    """The real-space coefficients X(R) = (1/N_k) sum_k X(k) e^{-i k.R} are NumPy's forward FFT over the mesh
    axes divided by N_k; summing them back with the boundary weights matches the oracle at arbitrary k."""
    kmesh = (4, 3, 2)
    rng = np.random.default_rng(13)
    nk = int(np.prod(kmesh))
    X = rng.normal(size=(nk, 2, 2)) + 1j * rng.normal(size=(nk, 2, 2))
    XR = np.fft.fftn(X.reshape(kmesh + (2, 2)), axes=(0, 1, 2)) / nk  # index R mod n
    path = rng.uniform(0.0, 1.0, size=(5, 3))
    ref = np.zeros((5, 2, 2), dtype=complex)
    for R in itertools.product(*[range(-(n // 2), n // 2 + 1) for n in kmesh]):
        w = np.prod([0.5 if (n % 2 == 0 and abs(r) == n // 2) else 1.0 for r, n in zip(R, kmesh)])
        if any(n % 2 == 1 and abs(r) > n // 2 for r, n in zip(R, kmesh)):
            continue
        idx = tuple(r % n for r, n in zip(R, kmesh))
        for p in range(5):
            ref[p] += w * XR[idx] * np.exp(2j * np.pi * np.dot(path[p], R))
    Y = gw.kpath_interpolate(X, kmesh, path)
    assert np.max(np.abs(Y - ref)) < 1e-13 * np.max(np.abs(ref))


# ============================================================================ energy, Dyson with a self-energy, mixing
def _eig_s(H, S):
    return scipy.linalg.eigh(H, S)


@pytest.mark.parametrize("kmesh,nspin,s_identity", [((1, 1, 1), 1, True), ((1, 1, 1), 1, False),
                                                    ((2, 1, 1), 2, True)])
def test_one_body_and_hartree_fock_energy_closed_form(kmesh, nspin, s_identity):
    """Galitskii-Migdal one-body and Hartree-Fock parts at the non-interacting G0, in the eigenbasis of
    H C = S C e (C^H S C = I, gamma = C f C^H):
      E_1b = (2/ns)(1/Nk) sum_{s,k} sum_i f_i e_i,
      E_HF = (1/ns)(1/Nk^2) sum_{s,k,k'} sum_{ij} f_{ski} f_{s'k'j} [(kk i i | k'k' j j) summed over s'
             (a restricted channel counted twice)  -  (k k' i j | k' k j i) at s' = s],
    with (k1 k2 i j | k3 k4 l m) = sum_Q (C^H V^{k1,k2}(Q) C)_{ij} (C^H V^{k3,k4}(Q) C)_{lm} built from
    explicit four-index integrals of Eq. CoulombDF."""
    sp = configs.tiny(kmesh=kmesh, nao=4, naux=5, ntau=24, beta=8.0, band=1.2, nspin=nspin,
                      s_identity=s_identity, seed=123)
    s = systems.make_system(sp)
    km = _km(kmesh)
    nk, ns, nao = sp.nk, sp.nspin, sp.nao
    Sinf = gw.sigma_inf(s.V, s.G0, kmesh)
    E = gw.energy(s.G0, s.H0, Sinf, np.zeros((ns, sp.ntau, nk, nao, nao), dtype=complex), sp.beta)
    C = np.empty((ns, nk, nao, nao), dtype=complex)
    f = np.empty((ns, nk, nao))
    e1 = 0.0
    for sp_ in range(ns):
        for k in range(nk):
            e, c = _eig_s(s.H0[sp_, k], s.S[k])
            C[sp_, k], f[sp_, k] = c, systems.fermi(e, sp.beta)
            e1 += np.sum(f[sp_, k] * e)
    e1 *= 2.0 / ns / nk
    ehf = 0.0
    for sa in range(ns):
        for k in range(nk):
            for sb in range(ns):
                for kp in range(nk):
                    A = np.einsum("ai,Qab,bj->Qij", C[sa, k].conj(), gw.V_pair(s.V, km, k, k), C[sa, k])
                    B = np.einsum("ai,Qab,bj->Qij", C[sb, kp].conj(), gw.V_pair(s.V, km, kp, kp), C[sb, kp])
                    J = np.einsum("Qii,Qjj->ij", A, B).real
                    ehf += (2.0 if ns == 1 else 1.0) * np.einsum("i,j,ij->", f[sa, k], f[sb, kp], J)
                    if sb == sa:
                        X = np.einsum("ai,Qab,bj->Qij", C[sa, k].conj(), gw.V_pair(s.V, km, k, kp), C[sa, kp])
                        Y = np.einsum("ai,Qab,bj->Qij", C[sa, kp].conj(), gw.V_pair(s.V, km, kp, k), C[sa, k])
                        K = np.einsum("Qij,Qji->ij", X, Y).real
                        ehf -= np.einsum("i,j,ij->", f[sa, k], f[sa, kp], K)
    ehf *= 1.0 / ns / nk ** 2
    assert abs(E["e_1b"] - e1) < 1e-12 * max(1.0, abs(e1))
    assert abs(E["e_hf"] - ehf) < 1e-13 * max(1.0, abs(ehf))
    assert E["e_corr"] == 0.0
    assert abs(E["e_tot"] - (e1 + ehf)) < 1e-12 * max(1.0, abs(e1 + ehf))


def _embedding(seed, nsys, nbath, spread=1.5, coupling=0.4):
    """A system block Hs (nsys x nsys, Hermitian), bath levels eb and couplings Wsb of a Hermitian
    (nsys + nbath) matrix whose bath block is diagonal."""
    rng = np.random.default_rng(seed)
    Z = rng.normal(size=(nsys, nsys)) + 1j * rng.normal(size=(nsys, nsys))
    Hs = 0.5 * spread * (Z + Z.conj().T) / np.sqrt(2 * nsys)
    eb = rng.uniform(-spread, spread, size=nbath)
    W = coupling * (rng.normal(size=(nsys, nbath)) + 1j * rng.normal(size=(nsys, nbath))) / np.sqrt(2)
    return Hs, eb, W


def _closed_form_G(H, tau, beta, mu):
    """-U diag(e^{-(E-mu)tau}/(1+e^{-beta(E-mu)})) U^H for a Hermitian H (S = I), per node."""
    E, U = np.linalg.eigh(H)
    x = E - mu
    w = np.exp(-np.outer(tau, x) - np.logaddexp(0.0, -beta * x)[None, :])
    return -np.einsum("ia,ta,ja->tij", U, w, U.conj())


@pytest.mark.parametrize("nspin,kmesh", [(1, (1, 1, 1)), (2, (2, 1, 1))])
def test_dyson_with_a_pole_self_energy(nspin, kmesh):
    """Eq. dyson with a non-zero Sigma~: a system coupled to a bath of levels eb through couplings W has the
    exact self-energy Sigma~(tau) = W g_b(tau) W^H, g_b the non-interacting bath G(tau) (a sum of poles), and
    its G is the system block of the non-interacting G of the whole Hermitian matrix [[Hs, W], [W^H, eb]]
    (Schur complement of the resolvent).  Hs is split as H0 + Sigma^inf, so both static terms enter with their
    sign.  Checks O9 (Sigma~(tau) -> Sigma~(i w)), O11 and, with a target electron count taken from the closed
    form at mu* = 0.17, the O10 root on an interacting G."""
    beta, ntau = 10.0, 64
    g = gridmod.make_grid(ntau, beta)
    nsys, nbath = 3, 4
    nk = int(np.prod(kmesh))
    H0 = np.empty((nspin, nk, nsys, nsys), dtype=complex)
    Sinf = np.empty_like(H0)
    Sig = np.empty((nspin, ntau, nk, nsys, nsys), dtype=complex)
    Gref = {}
    S = np.tile(np.eye(nsys, dtype=complex), (nk, 1, 1))
    mu_star = 0.17
    n_target = 0.0
    for s in range(nspin):
        for k in range(nk):
            Hs, eb, W = _embedding(1000 + 10 * s + k, nsys, nbath)
            rng = np.random.default_rng(77 + s + k)
            Z = rng.normal(size=(nsys, nsys)) + 1j * rng.normal(size=(nsys, nsys))
            Sinf[s, k] = 0.2 * (Z + Z.conj().T)
            H0[s, k] = Hs - Sinf[s, k]
            gb = -np.exp(-np.outer(g.tau, eb - mu_star) - np.logaddexp(0.0, -beta * (eb - mu_star))[None, :])
            Sig[s, :, k] = np.einsum("ib,tb,jb->tij", W, gb, W.conj())
            Hfull = np.block([[Hs, W], [W.conj().T, np.diag(eb)]])
            Gref[s, k] = _closed_form_G(Hfull, g.tau, beta, mu_star)[:, :nsys, :nsys]
            E, U = np.linalg.eigh(Hfull)
            n_target += (2.0 / nspin) / nk * np.sum(np.abs(U[:nsys]) ** 2 * systems.fermi(E - mu_star, beta)[None])
    # mu held at mu*: G(tau) of the embedded system
    G, mu, n = gw.solve_dyson(H0, S, Sinf, Sig, g, nspin, mu_star, -1.0)
    for s in range(nspin):
        for k in range(nk):
            assert np.max(np.abs(G[s, :, k] - Gref[s, k])) < 1e-10
    assert abs(n - n_target) < 1e-10
    # mu searched from 0 for the closed-form electron count of the system orbitals
    G2, mu2, n2 = gw.solve_dyson(H0, S, Sinf, Sig, g, nspin, 0.0, n_target)
    assert abs(mu2 - mu_star) < 1e-9
    assert np.max(np.abs(G2 - G)) < 1e-9


def test_mixing_at_alpha_below_one():
    """Sec. 4.2.2 damping: with 0 < alpha < 1 the self-energy that enters Dyson is alpha Sigma[G_{n-1}] +
    (1 - alpha) Sigma_{n-1} for both Sigma^inf and Sigma~.  Run one iteration at alpha = 0.6 from a state
    whose stored self-energies differ from Sigma[G]: the iteration must return the affine combination
    weighted towards the new self-energy, and its G must be the Dyson solution of that combination."""
    sp = configs.tiny(kmesh=(2, 1, 1), nao=3, naux=4, ntau=16, beta=6.0, seed=55)
    s = systems.make_system(sp)
    Sinf_new, Sig_new, _ = gw.sigma_eval(s.V, s.G0, sp.kmesh, s.grid)
    rng = np.random.default_rng(5)
    Sinf_old = Sinf_new + 0.05 * rng.normal(size=Sinf_new.shape)
    Sig_old = Sig_new + 0.05 * rng.normal(size=Sig_new.shape)
    st = gw.State(s.G0, Sinf_old, Sig_old, 0.0)
    alpha = 0.6
    st2, rep, _ = gw.iterate(s, st, alpha=alpha)
    # the new self-energy sits at the fraction alpha of the way from the old one: |S - S_old| = alpha |S_new - S_old|
    for got, new, old in [(st2.Sinf, Sinf_new, Sinf_old), (st2.Sig, Sig_new, Sig_old)]:
        d_new, d_got = new - old, got - old
        assert np.allclose(d_got, alpha * d_new, atol=1e-15, rtol=1e-13)
        assert np.linalg.norm(got - new) < np.linalg.norm(got - old)  # closer to the new self-energy
    # alpha -> 0 keeps the old self-energy, alpha = 1 takes the new one
    assert np.allclose(gw.mix(Sig_new, Sig_old, 1e-12), Sig_old, atol=1e-12)
    assert np.array_equal(gw.mix(Sig_new, Sig_old, 1.0), Sig_new)
    G, mu, _ = gw.solve_dyson(s.H0, s.S, st2.Sinf, st2.Sig, s.grid, sp.nspin, 0.0, s.n_target)
    assert np.max(np.abs(G - st2.G)) == 0.0 and mu == st2.mu
