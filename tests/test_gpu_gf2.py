"""GF2 self-energy (Eq. sigma2, direct minus exchange) on the GPU against the oracle, element by element.

Bar: FP64 plans max|GPU - oracle| / max|oracle| <= 1e-10; FP32 and split-BF16 plans (operands rounded,
FP32 accumulation within each contraction slice) <= 2e-5.  Shapes span ragged MFMA tiles (odd nao, naux),
both spin settings, a 3-point direction (k3 = k1 + k2 - k differs from k1 + k - k2 there) and forced
chunking of the momentum triples (one triple per chunk, and runs of pairs of one k).
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
    dict(kmesh=(1, 1, 1), nao=11, naux=37, ntau=8, nspin=1, chunk=0, seed=601),
    dict(kmesh=(2, 2, 2), nao=5, naux=13, ntau=6, nspin=1, chunk=0, seed=602),
    dict(kmesh=(3, 1, 1), nao=6, naux=10, ntau=6, nspin=2, chunk=0, seed=603),
    dict(kmesh=(3, 2, 1), nao=4, naux=9, ntau=6, nspin=1, chunk=1, seed=604),        # one triple per chunk
    dict(kmesh=(2, 2, 2), nao=5, naux=13, ntau=6, nspin=1, chunk=300_000, seed=605),  # 15 pairs of one k
]


def _system(c):
    sp = configs.tiny(kmesh=c["kmesh"], nao=c["nao"], naux=c["naux"], ntau=c["ntau"], beta=6.0, nspin=c["nspin"],
                      seed=c["seed"], v_scale=0.5 / c["nao"] ** 0.5)
    return systems.make_system(sp)


def _plan(s, prec, chunk):
    from paper_2406_18479_amd.gw import Plan
    sp = s.spec
    p = Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin, prec=prec, chunk_bytes=chunk)
    p.set_option("gf2", 1)
    return p


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"k{c['kmesh']}_nao{c['nao']}_naux{c['naux']}_ns{c['nspin']}_ch{c['chunk']}")
def test_gf2_selfenergy_parity(c):
    _require_gpu()
    s = _system(c)
    sp = s.spec
    say("gf2 fp64", c)
    G = systems.random_green(c["seed"] + 7, sp.nspin, sp.ntau, sp.nk, sp.nao, scale=0.4)
    ref = ogw.gf2_selfenergy(s.V, G, sp.kmesh)
    p = _plan(s, "fp64", c["chunk"])
    got = host(p.gf2_selfenergy(dev(s.V), dev(G)))
    assert rel(got, ref) <= 1e-10
    # the exchange term is not small against the direct one in these cases
    direct = ogw.selfenergy(s.V, G, ogw.polarization(s.V, G, sp.kmesh), sp.kmesh)
    assert np.max(np.abs(ref - direct)) > 1e-2 * np.max(np.abs(ref))


MIXED = [CASES[1], dict(kmesh=(2, 1, 1), nao=13, naux=37, ntau=6, nspin=1, chunk=0, seed=606)]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("c", MIXED, ids=lambda c: f"k{c['kmesh']}_nao{c['nao']}_naux{c['naux']}")
def test_gf2_mixed_precision(c, prec):
    """Split-BF16 plans run the auxiliary sums on the large-tile kernel (nao^2 = 169 rows and columns, a K of 37
    in two slices of 32); FP32 plans on the 256-thread kernel."""
    _require_gpu()
    s = _system(c)
    sp = s.spec
    say("gf2", prec, c)
    G = systems.random_green(c["seed"] + 7, sp.nspin, sp.ntau, sp.nk, sp.nao, scale=0.4)
    ref = ogw.gf2_selfenergy(s.V, G, sp.kmesh)
    p = _plan(s, prec, 0)
    err = rel(host(p.gf2_selfenergy(dev(s.V), dev(G))), ref)
    say("gf2", prec, "rel err", err)
    assert err <= 2e-5


def test_gf2_iteration_parity():
    """Two GF2 self-consistent iterations (Sec. 2.3 with the self-energy of Eq. sigma2) against the oracle."""
    _require_gpu()
    sp = configs.tiny(kmesh=(2, 1, 1), nao=5, naux=11, ntau=16, beta=10.0, seed=631, v_scale=0.2)
    s = systems.make_system(sp)
    p = _plan(s, "fp64", 0)
    V, H0, S = dev(s.V), dev(s.H0), dev(s.S)
    G = dev(s.G0)
    Sinf = torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0")
    Sig = torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0")
    st = ogw.State(s.G0, None, None, 0.0)
    mu = 0.0
    for it in range(2):
        say("gf2 iterate", it)
        mu, rep = p.iterate(V, H0, S, G, Sinf, Sig, mu, s.n_target, 1.0)
        st, orep, _ = ogw.iterate(s, st, method="gf2")
        assert rel(host(Sig), st.Sig) <= 1e-10, it
        assert rel(host(G), st.G) <= 1e-10, it
        assert abs(mu - orep["mu"]) <= 1e-10
        for key in ("e_1b", "e_hf", "e_corr", "e_tot"):
            assert abs(rep[key] - orep[key]) <= 1e-10, (it, key, rep[key], orep[key])
