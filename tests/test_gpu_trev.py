"""Time reversal (the self-energy contracted for k with -k >= k only, partners conjugated) on the GPU, on
time-reversal-symmetric systems (V^{-k1,-k2}(Q) = conj V^{k1,k2}(Q), H0(-k) = conj H0(k)).

Bar: FP64 iterations against the oracle (which contracts every k) at 1e-10; FP32 and split-BF16 plans with the
option against the same plans without it at 1e-6 relative (only the blocking of the first contraction
differs); the conjugate pairing holds exactly in the output.
"""
import numpy as np
import pytest

from oracle import gw as ogw
from synth import configs, systems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def say(*a):
    print("[gpu-case]", *a, flush=True)


CASES = [
    dict(kmesh=(3, 2, 1), nao=8, naux=24, ntau=8, nspin=1, seed=701),
    dict(kmesh=(2, 2, 2), nao=5, naux=13, ntau=6, nspin=2, seed=702),
]


def _system(c):
    sp = configs.tiny(kmesh=c["kmesh"], nao=c["nao"], naux=c["naux"], ntau=c["ntau"], beta=6.0, nspin=c["nspin"],
                      seed=c["seed"], v_scale=0.5 / c["nao"] ** 0.5, v_time_reversal=True)
    return systems.make_system(sp)


def _plan(s, prec, trev):
    from paper_2406_18479_amd.gw import Plan
    sp = s.spec
    p = Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin, prec=prec)
    p.set_option("time_reversal", int(trev))
    return p


def _partners_exact(Sig, kmesh):
    km = ogw.KMesh(kmesh)
    for k in range(km.nk):
        kn = km.sub(0, k)
        if kn < k:
            assert np.array_equal(Sig[:, :, k], np.conj(Sig[:, :, kn]))


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"k{c['kmesh']}_nao{c['nao']}_naux{c['naux']}_ns{c['nspin']}")
def test_time_reversal_iterations_match_oracle(c):
    _require_gpu()
    s = _system(c)
    sp = s.spec
    p = _plan(s, "fp64", True)
    V, H0, S = dev(s.V), dev(s.H0), dev(s.S)
    G = dev(s.G0)
    Sinf = torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0")
    Sig = torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0")
    st = ogw.State(s.G0, None, None, 0.0)
    mu = 0.0
    for it in range(2):
        say("time reversal iterate", c, it)
        mu, rep = p.iterate(V, H0, S, G, Sinf, Sig, mu, s.n_target, 1.0)
        st, orep, _ = ogw.iterate(s, st)
        hs = host(Sig)
        assert rel(hs, st.Sig) <= 1e-10, it
        assert rel(host(G), st.G) <= 1e-10, it
        assert rel(host(Sinf), st.Sinf) <= 1e-10, it  # Sigma^inf on the contracted momenta and their fill
        _partners_exact(hs, sp.kmesh)
        for key in ("e_1b", "e_hf", "e_corr", "e_tot"):
            assert abs(rep[key] - orep[key]) <= 1e-10, (it, key)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("c", CASES, ids=lambda c: f"k{c['kmesh']}_nao{c['nao']}_naux{c['naux']}_ns{c['nspin']}")
def test_time_reversal_mixed_precision(c, prec):
    """Split BF16 with nao = 8 runs the LDS-DMA stage 1 and the fused stages 2 + 3 on the contracted momenta;
    naux = 13 the register-staged path."""
    _require_gpu()
    s = _system(c)
    sp = s.spec
    say("time reversal", prec, c)
    V, G = dev(s.V), dev(s.G0)
    ref = _plan(s, prec, False)
    trp = _plan(s, prec, True)
    P0 = ref.polarization(V, G)
    # the time-reversal plan contracts half of the tau nodes and conjugate-transposes the rest
    assert rel(host(trp.polarization(V, G)), host(P0)) <= 1e-6
    Pt = ref.screen(P0)
    a = host(ref.selfenergy(V, G, Pt))
    b = host(trp.selfenergy(V, G, Pt))
    assert rel(b, a) <= 1e-6
    _partners_exact(b, sp.kmesh)


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"k{c['kmesh']}_nao{c['nao']}_naux{c['naux']}_ns{c['nspin']}")
def test_time_reversal_polarization_matches_oracle(c):
    _require_gpu()
    s = _system(c)
    sp = s.spec
    say("time reversal polarization", c)
    got = host(_plan(s, "fp64", True).polarization(dev(s.V), dev(s.G0)))
    assert rel(got, ogw.polarization(s.V, s.G0, sp.kmesh)) <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_time_reversal_gf2(prec):
    """GF2 (Eq. sigma2) with the option: both terms contracted for k with -k >= k, partners conjugated; FP64
    against the oracle at 1e-10, split BF16 against the same plan without the option at 1e-6."""
    _require_gpu()
    c = CASES[0]
    s = _system(c)
    sp = s.spec
    say("time reversal gf2", prec, c)
    V, G = dev(s.V), dev(s.G0)
    p = _plan(s, prec, True)
    p.set_option("gf2", 1)
    got = host(p.gf2_selfenergy(V, G))
    _partners_exact(got, sp.kmesh)
    if prec == "fp64":
        assert rel(got, ogw.gf2_selfenergy(s.V, s.G0, sp.kmesh)) <= 1e-10
    else:
        q = _plan(s, prec, False)
        q.set_option("gf2", 1)
        assert rel(got, host(q.gf2_selfenergy(V, G))) <= 1e-6
