"""Input generators and the Chebyshev grid (CPU)."""
import numpy as np
import pytest
import scipy.linalg

from synth import configs, grid as gridmod, rng, systems


# ----------------------------------------------------------------------------- rng
def test_splitmix64_reference_values():
    # Published SplitMix64 outputs for state 0 (first three outputs of the
    # sequence started at seed 0): 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F.
    state = np.uint64(0)
    outs = []
    for i in range(1, 4):
        outs.append(int(rng.splitmix64(np.uint64(0x9E3779B97F4A7C15 * (i - 1) % 2**64))))
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    del state


def test_rng_reproducible_and_independent():
    k1 = rng.stream_key(5, rng.TAG_V, 0, 1, 2)
    k2 = rng.stream_key(5, rng.TAG_V, 0, 2, 1)
    a = rng.complex_normals(k1, (1000,))
    b = rng.complex_normals(k1, (1000,))
    c = rng.complex_normals(k2, (1000,))
    assert np.array_equal(a, b)
    assert not np.allclose(a, c)
    z = rng.complex_normals(rng.stream_key(1, 2, 3), (200000,))
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 0.01
    assert abs(np.mean(z.real)) < 0.01 and abs(np.mean(z.imag)) < 0.01
    u = rng.uniforms(k1, 0, 100000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01


# ----------------------------------------------------------------------------- generators
@pytest.fixture(scope="module")
def sys222():
    return systems.make_system(configs.tiny(kmesh=(2, 2, 2), nao=4, naux=5, ntau=16, beta=10.0, seed=3))


def test_v_hermitian_pairing(sys222):
    V = sys222.V
    km = sys222.spec.kmesh
    add = systems.k_add_table(km)
    sub = systems.k_sub_table(km)
    nk = sys222.spec.nk
    for q in range(nk):
        for k in range(nk):
            kq = add[k, q]
            # V^{k+q,k} is stored at [q' = k - (k+q) = -q][k+q]
            back = V[sub[k, kq], kq]
            assert np.allclose(back, np.conj(np.swapaxes(V[q, k], 1, 2)), atol=0, rtol=0)


def test_h0_time_reversal_and_spectrum(sys222):
    H = sys222.H0
    neg = systems.k_neg(sys222.spec.kmesh)
    for k in range(sys222.spec.nk):
        assert np.array_equal(H[0, neg[k]], np.conj(H[0, k]))
        if neg[k] == k:  # every 2x2x2 point is time-reversal invariant -> real H0
            assert np.all(H[0, k].imag == 0)
        e = np.linalg.eigvalsh(H[0, k])
        assert e.min() >= -2.0 and e.max() <= 2.0
        assert np.allclose(H[0, k], H[0, k].conj().T)


def test_v_time_reversal_variant():
    s = systems.make_system(configs.tiny(kmesh=(3, 1, 1), nao=3, naux=4, ntau=8, seed=9, v_time_reversal=True))
    V = s.V
    km = s.spec.kmesh
    neg = systems.k_neg(km)
    add = systems.k_add_table(km)
    sub = systems.k_sub_table(km)
    for q in range(s.spec.nk):
        for k in range(s.spec.nk):
            kq = add[k, q]
            # V^{-k,-(k+q)} is stored at [q' = -q][-k]
            other = V[sub[neg[kq], neg[k]], neg[k]]
            assert np.allclose(other, np.conj(V[q, k]), atol=1e-15)
            back = V[sub[k, kq], kq]
            assert np.allclose(back, np.conj(np.swapaxes(V[q, k], 1, 2)), atol=1e-15)


def test_noninteracting_g_normalisation_general_S():
    sp = configs.tiny(kmesh=(2, 1, 1), nao=4, naux=3, ntau=12, beta=8.0, s_identity=False, seed=21)
    s = systems.make_system(sp)
    for k in range(sp.nk):
        lhs = s.G0[0, 0, k] + s.G0[0, -1, k]
        assert np.allclose(lhs, -np.linalg.inv(s.S[k]), atol=1e-13)
        assert np.min(np.linalg.eigvalsh(s.S[k])) > 0.5


def test_electron_count_matches_trace():
    sp = configs.tiny(kmesh=(2, 1, 1), nao=5, naux=3, ntau=12, beta=8.0, s_identity=False, seed=22)
    s = systems.make_system(sp)
    n = -(2.0 / sp.nspin) * sum(np.trace(s.G0[0, -1, k] @ s.S[k]).real for k in range(sp.nk)) / sp.nk
    assert abs(n - s.n_target) < 1e-12


def test_batch_draw_fits_hbm():
    specs = configs.batch_specs()
    assert len(specs) == 16
    tot = sum(sp.nk ** 2 * sp.naux * sp.nao ** 2 * 16 for sp in specs)
    assert tot < 200e9


# ----------------------------------------------------------------------------- grid
@pytest.mark.parametrize("ntau,beta", [(20, 50.0), (48, 50.0), (104, 100.0)])
def test_grid_structure(ntau, beta):
    g = gridmod.make_grid(ntau, beta)
    assert g.tau[0] == 0.0 and g.tau[-1] == beta
    assert np.allclose(g.tau + g.tau[::-1], beta, atol=1e-13, rtol=0)
    assert len(g.nf) == ntau and len(g.nb) == ntau + 1
    assert np.array_equal(np.sort(-g.nf - 1), g.nf)  # fermionic +- pairs
    assert np.array_equal(np.sort(-g.nb), g.nb) and 0 in g.nb
    assert np.allclose(g.TF_w2t @ g.TF_t2w, np.eye(ntau), atol=1e-11)
    assert np.allclose(g.TB_w2t @ g.TB_t2w, np.eye(ntau), atol=1e-11)
    assert np.linalg.cond(g.TF_t2w) < 1e4 and np.linalg.cond(g.TB_t2w) < 1e4


def _poly_fourier(coef, nu, beta):
    """Exact int_0^beta sum_p coef[p] tau^p e^{i nu tau} dtau by repeated integration by parts."""
    if nu == 0:
        return sum(c * beta ** (p + 1) / (p + 1) for p, c in enumerate(coef))
    tot = 0.0
    for p, c in enumerate(coef):
        # int_0^beta tau^p e^{i nu tau} = sum_j (-1)^j p!/(p-j)! tau^{p-j} e^{i nu tau}/(i nu)^{j+1} |_0^beta
        val = 0.0
        fact = 1.0
        for j in range(p + 1):
            if j > 0:
                fact *= p - j + 1
            term_b = beta ** (p - j) * np.exp(1j * nu * beta)
            term_0 = 1.0 if p - j == 0 else 0.0
            val += (-1) ** j * fact * (term_b - term_0) / (1j * nu) ** (j + 1)
        tot += c * val
    return tot


@pytest.mark.parametrize("ntau,beta", [(20, 50.0), (104, 100.0)])
def test_grid_transform_exact_on_polynomials(ntau, beta):
    g = gridmod.make_grid(ntau, beta)
    coef = [0.3, -0.2 / beta, 0.7 / beta ** 2, -0.4 / beta ** 3]
    f = sum(c * g.tau ** p for p, c in enumerate(coef))
    for rows, nus in ((g.TF_t2w, g.wf), (g.TB_t2w, g.wb)):
        got = rows @ f
        ref = np.array([_poly_fourier(coef, nu, beta) for nu in nus])
        assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, beta)


def test_grid_noninteracting_representation():
    """TF_t2w applied to the closed-form G0(tau) reproduces G0(i w) = sum_a C_a C_a^H / (i w - e_a)."""
    beta, ntau = 100.0, 104
    g = gridmod.make_grid(ntau, beta)
    e = np.array([-2.0, -0.7, -0.01, 0.02, 1.3, 2.0])
    U = scipy.linalg.qr(np.random.default_rng(1).normal(size=(6, 6)))[0]
    H = (U * e) @ U.T
    G0 = systems.noninteracting_G(H[None, None].astype(complex), np.eye(6)[None].astype(complex), g.tau, beta, 0.0)
    Gw = np.einsum("mt,tij->mij", g.TF_t2w, G0[0, :, 0])
    ref = np.einsum("ia,ma,ja->mij", U, 1.0 / (1j * g.wf[:, None] - e[None, :]), U)
    assert np.max(np.abs(Gw - ref)) < 1e-10
    # and back
    assert np.max(np.abs(np.einsum("tm,mij->tij", g.TF_w2t, ref) - G0[0, :, 0])) < 1e-9


# ----------------------------------------------------------------------------- device generator
def test_device_generator_matches_host():
    """The torch generator reproduces the NumPy integer stream bit for bit and V to rounding."""
    import torch

    from synth import device
    key = rng.stream_key(11, rng.TAG_V, 0, 1, 2)
    idx = np.arange(1000, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ref = rng.splitmix64(idx + key).astype(np.int64)
    got = device.splitmix64(torch.arange(1000, dtype=torch.int64) + device._i64(int(key))).numpy()
    assert np.array_equal(ref, got)
    assert np.array_equal(rng.uniforms(key, 0, 1000), device.uniforms(int(key), 1000, "cpu").numpy())
    sp = configs.tiny(kmesh=(2, 2, 1), nao=3, naux=5, ntau=8, seed=19)
    Vh = systems.make_V(sp)
    Vd = device.make_V(sp, device="cpu").numpy()
    assert np.max(np.abs(Vh - Vd)) < 1e-14 * np.max(np.abs(Vh))


def test_device_generator_time_reversal_variant():
    """The time-reversal-symmetric V from the torch generator matches the NumPy one to rounding and satisfies
    V^{-k1,-k2}(Q) = conj V^{k1,k2}(Q) and V^{k2,k1}(Q) = V^{k1,k2}(Q)^dagger to rounding."""
    from synth import device
    for kmesh in [(3, 2, 1), (2, 2, 2)]:
        sp = configs.tiny(kmesh=kmesh, nao=3, naux=5, ntau=8, seed=23, v_time_reversal=True)
        Vh = systems.make_V(sp)
        Vd = device.make_V(sp, device="cpu").numpy()
        scale = np.max(np.abs(Vh))
        assert np.max(np.abs(Vh - Vd)) < 1e-14 * scale
        sub, neg = systems.k_sub_table(kmesh), systems.k_neg(kmesh)

        def blk(k1, k2):
            return Vd[sub[k2, k1], k1]
        for k1 in range(sp.nk):
            for k2 in range(sp.nk):
                assert np.max(np.abs(blk(neg[k1], neg[k2]) - np.conj(blk(k1, k2)))) < 1e-15 * scale
                assert np.max(np.abs(blk(k2, k1) - np.conj(np.swapaxes(blk(k1, k2), 1, 2)))) < 1e-15 * scale
