"""Point-group reduction (green_plan_set_kpoint_symmetry) on the GPU, on systems invariant under the group.

The plan contracts one transfer per pair of orbits {O, -O} in P~0 and the screening and one momentum per orbit
(per pair under time reversal) in the self-energy, and writes the others as copies; the oracle contracts every
k and q.  Bar: FP64 against the oracle at 1e-10 (as the other FP64 paths); split BF16 with the group against the
same plan without it at 1e-6 relative (only the set of contracted blocks differs).  The full cubic group O_h on a
3x3x3 mesh leaves 4 of 27 momenta; C3 about the body diagonal (no inversion) exercises the transposed,
tau-reversed copies of -O and, with time reversal, the conjugate copies.
"""
import numpy as np
import pytest

from oracle import gw as ogw
from synth import configs
from synth import symmetry as sym

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GROUPS = {"Oh": sym.cubic_group, "C3": sym.threefold_group}


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


_CACHE = {}


def _system(group, trev, nspin=1, nao=6, naux=20, ntau=12):
    key = (group, trev, nspin, nao, naux, ntau)
    if key not in _CACHE:
        sp = configs.tiny(kmesh=(3, 3, 3), nao=nao, naux=naux, ntau=ntau, beta=8.0, nspin=nspin, seed=931,
                          v_scale=0.6 / nao ** 0.5, f_time_reversal=trev, v_time_reversal=trev)
        _CACHE[key] = sym.make_symmetric_system(sp, GROUPS[group]())
    return _CACHE[key]


def _plan(s, prec, group, trev):
    from paper_2406_18479_amd.gw import Plan
    sp = s.spec
    p = Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin, prec=prec)
    p.set_option("time_reversal", int(trev))
    counts = p.set_kpoint_symmetry(GROUPS[group]() if group else [])
    return p, counts


EXPECT = {("Oh", 0): (4, 4), ("Oh", 1): (4, 4), ("C3", 0): (6, 11), ("C3", 1): (6, 6)}
CASES = [("Oh", 0, 1), ("Oh", 1, 1), ("C3", 0, 1), ("C3", 1, 2)]


@pytest.mark.parametrize("group,trev,nspin", CASES, ids=lambda x: str(x))
def test_polarization_screening_selfenergy_match_oracle(group, trev, nspin):
    _require_gpu()
    s = _system(group, trev, nspin)
    sp = s.spec
    say("kpoint symmetry P0/screen/Sigma", group, "trev", trev, "nspin", nspin)
    p, counts = _plan(s, "fp64", group, trev)
    assert counts == EXPECT[(group, trev)]
    V, G = dev(s.V), dev(s.G0)
    P0 = p.polarization(V, G)
    ref_P0 = ogw.polarization(s.V, s.G0, sp.kmesh)
    assert rel(host(P0), ref_P0) <= 1e-10
    Pt = p.screen(P0)
    ref_Pt = ogw.from_bosonic(ogw.screen(ogw.to_bosonic(ref_P0, s.grid.TB_t2w)), s.grid.TB_w2t)
    assert rel(host(Pt), ref_Pt) <= 1e-10
    Sig = p.selfenergy(V, G, dev(ref_Pt))
    assert rel(host(Sig), ogw.selfenergy(s.V, s.G0, ref_Pt, sp.kmesh)) <= 1e-10
    p.check_status()


@pytest.mark.parametrize("group,trev,nspin", CASES, ids=lambda x: str(x))
def test_iterations_match_oracle(group, trev, nspin):
    _require_gpu()
    s = _system(group, trev, nspin)
    p, _ = _plan(s, "fp64", group, trev)
    V, H0, S = dev(s.V), dev(s.H0), dev(s.S)
    G = dev(s.G0)
    Sinf = torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0")
    Sig = torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0")
    st = ogw.State(s.G0, None, None, 0.0)
    mu = 0.0
    for it in range(2):
        say("kpoint symmetry iterate", group, "trev", trev, "nspin", nspin, "it", it)
        mu, rep = p.iterate(V, H0, S, G, Sinf, Sig, mu, s.n_target, 1.0)
        st, orep, _ = ogw.iterate(s, st)
        assert rel(host(Sig), st.Sig) <= 1e-10, it
        assert rel(host(G), st.G) <= 1e-10, it
        assert rel(host(Sinf), st.Sinf) <= 1e-10, it  # Sigma^inf on the contracted momenta and their fill
        for key in ("e_1b", "e_hf", "e_corr", "e_tot"):
            assert abs(rep[key] - orep[key]) <= 1e-10, (it, key)


@pytest.mark.parametrize("group,trev", [("Oh", 1), ("C3", 0)])
def test_gf2_matches_oracle(group, trev):
    _require_gpu()
    s = _system(group, trev, nao=4, naux=10, ntau=8)
    sp = s.spec
    say("kpoint symmetry gf2", group, "trev", trev)
    p, _ = _plan(s, "fp64", group, trev)
    p.set_option("gf2", 1)
    got = host(p.gf2_selfenergy(dev(s.V), dev(s.G0)))
    assert rel(got, ogw.gf2_selfenergy(s.V, s.G0, sp.kmesh)) <= 1e-10


@pytest.mark.parametrize("group,trev", [("Oh", 0), ("C3", 1)])
def test_split_bf16_with_the_group(group, trev):
    """nao = 8, naux = 24: the LDS-DMA stage 1 and the fused stages 2 + 3 on the contracted momenta."""
    _require_gpu()
    s = _system(group, trev, nao=8, naux=24)
    say("kpoint symmetry bf16x3", group, "trev", trev)
    V, G = dev(s.V), dev(s.G0)
    ref, _ = _plan(s, "bf16x3", None, 0)
    red, _ = _plan(s, "bf16x3", group, trev)
    P0 = ref.polarization(V, G)
    assert rel(host(red.polarization(V, G)), host(P0)) <= 1e-6
    Pt = ref.screen(P0)
    assert rel(host(red.screen(P0)), host(Pt)) <= 1e-6
    assert rel(host(red.selfenergy(V, G, Pt)), host(ref.selfenergy(V, G, Pt))) <= 1e-6


def test_v_half_store_with_the_group():
    _require_gpu()
    s = _system("C3", 0)
    say("kpoint symmetry v_half")
    full, _ = _plan(s, "fp64", "C3", 0)
    half, _ = _plan(s, "fp64", "C3", 0)
    half.set_option("v_half", 1)
    qcan = [q for q in range(s.spec.nk) if ogw.KMesh(s.spec.kmesh).sub(0, q) >= q]
    G = dev(s.G0)
    a = host(full.polarization(dev(s.V), G))
    b = host(half.polarization(dev(s.V[qcan]), G))
    assert np.array_equal(a, b)


def test_non_invariant_input_is_reported():
    """A G that breaks the group (one momentum's block scaled) latches GREEN_EINVAL instead of a wrong result."""
    _require_gpu()
    from paper_2406_18479_amd._lib import GreenError
    s = _system("Oh", 0)
    say("kpoint symmetry check")
    p, _ = _plan(s, "fp64", "Oh", 0)
    Gbad = s.G0.copy()
    Gbad[:, :, 5] *= 1.01
    p.polarization(dev(s.V), dev(Gbad))
    with pytest.raises(GreenError) as e:
        p.check_status()
    assert e.value.code == -1
    # a later good call is not affected
    p.polarization(dev(s.V), dev(s.G0))
    p.check_status()
