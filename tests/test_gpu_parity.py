"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on seeded inputs.

Bar: max|GPU - oracle| / max|oracle| <= 1e-10 for every FP64 result (Sigma~,
P~0, P~, G), |dE| <= 1e-10 Eh for energies.  Shapes span several MFMA tiles
with ragged tails (odd nao / naux), both spin settings and forced tau
chunking; the 2x2x2 production shape is checked in full for one iteration.
"""
import numpy as np
import pytest

from oracle import gw as ogw
from synth import configs, systems

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-10


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


def make_plan(s, prec="fp64", chunk_bytes=0):
    from paper_2406_18479_amd.gw import Plan
    sp = s.spec
    return Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin, prec=prec, chunk_bytes=chunk_bytes)


TINY = [
    dict(kmesh=(2, 2, 1), nao=5, naux=37, ntau=10, nspin=1, chunk=0, seed=101),
    dict(kmesh=(3, 1, 1), nao=3, naux=70, ntau=8, nspin=2, chunk=0, seed=102),
    dict(kmesh=(2, 1, 1), nao=17, naux=33, ntau=12, nspin=1, chunk=1, seed=103),
    dict(kmesh=(1, 1, 1), nao=34, naux=65, ntau=6, nspin=1, chunk=0, seed=104),
]


def _tiny_system(c):
    sp = configs.tiny(kmesh=c["kmesh"], nao=c["nao"], naux=c["naux"], ntau=c["ntau"], beta=6.0, nspin=c["nspin"],
                      seed=c["seed"], v_scale=0.5 / c["nao"] ** 0.5)
    return systems.make_system(sp)


@pytest.mark.parametrize("c", TINY, ids=lambda c: f"k{c['kmesh']}_nao{c['nao']}_naux{c['naux']}_ns{c['nspin']}")
def test_polarization_parity(c):
    _require_gpu()
    s = _tiny_system(c)
    sp = s.spec
    G = systems.random_green(c["seed"] + 1, sp.nspin, sp.ntau, sp.nk, sp.nao, scale=0.3)
    say("polarization", c)
    plan = make_plan(s, chunk_bytes=c["chunk"])
    P = host(plan.polarization(dev(s.V), dev(G)))
    ref = ogw.polarization(s.V, G, sp.kmesh)
    assert rel(P, ref) <= TOL


@pytest.mark.parametrize("c", TINY, ids=lambda c: f"k{c['kmesh']}_nao{c['nao']}_naux{c['naux']}_ns{c['nspin']}")
def test_selfenergy_parity(c):
    _require_gpu()
    s = _tiny_system(c)
    sp = s.spec
    G = systems.random_green(c["seed"] + 2, sp.nspin, sp.ntau, sp.nk, sp.nao, scale=0.3)
    Pt = systems.random_polarization(c["seed"] + 3, sp.nk, sp.ntau, sp.naux, scale=0.1)
    say("selfenergy", c)
    plan = make_plan(s, chunk_bytes=c["chunk"])
    Sig = host(plan.selfenergy(dev(s.V), dev(G), dev(Pt)))
    ref = ogw.selfenergy(s.V, G, Pt, sp.kmesh)
    assert rel(Sig, ref) <= TOL


@pytest.mark.parametrize("c", TINY, ids=lambda c: f"k{c['kmesh']}_nao{c['nao']}_naux{c['naux']}_ns{c['nspin']}")
def test_hf_static_parity(c):
    _require_gpu()
    s = _tiny_system(c)
    sp = s.spec
    G = systems.random_green(c["seed"] + 4, sp.nspin, sp.ntau, sp.nk, sp.nao, scale=0.3)
    say("hf_static", c)
    plan = make_plan(s)
    Sinf = host(plan.hf_static(dev(s.V), dev(G)))
    ref = ogw.sigma_inf(s.V, G, sp.kmesh)
    assert rel(Sinf, ref) <= TOL


@pytest.mark.parametrize("c", TINY[:3], ids=lambda c: f"k{c['kmesh']}_naux{c['naux']}")
def test_screen_parity(c):
    _require_gpu()
    s = _tiny_system(c)
    sp = s.spec
    P0 = ogw.polarization(s.V, s.G0, sp.kmesh)
    say("screen", c)
    plan = make_plan(s)
    Pt = host(plan.screen(dev(P0)))
    ref = ogw.from_bosonic(ogw.screen(ogw.to_bosonic(P0, s.grid.TB_t2w)), s.grid.TB_w2t)
    assert rel(Pt, ref) <= TOL


def test_screen_large_aux_parity():
    """naux = 300 (several inversion panels, row-interchange bookkeeping across panels)."""
    _require_gpu()
    sp = configs.tiny(kmesh=(2, 1, 1), nao=4, naux=300, ntau=8, beta=5.0, seed=111, v_scale=0.3)
    s = systems.make_system(sp)
    P0 = ogw.polarization(s.V, s.G0, sp.kmesh)
    P0 = P0 * (0.5 / np.max(np.abs(ogw.to_bosonic(P0, s.grid.TB_t2w))))  # keep [I - P0] well conditioned
    say("screen naux=300")
    plan = make_plan(s)
    Pt = host(plan.screen(dev(P0)))
    ref = ogw.from_bosonic(ogw.screen(ogw.to_bosonic(P0, s.grid.TB_t2w)), s.grid.TB_w2t)
    assert rel(Pt, ref) <= TOL


@pytest.mark.parametrize("nspin,s_identity", [(1, False), (2, True)])
def test_dyson_parity(nspin, s_identity):
    _require_gpu()
    sp = configs.tiny(kmesh=(2, 1, 1), nao=6, naux=5, ntau=24, beta=20.0, nspin=nspin, s_identity=s_identity,
                      seed=121)
    s = systems.make_system(sp)
    rng = np.random.default_rng(5)
    Sinf = 0.05 * (rng.normal(size=s.H0.shape) + 1j * rng.normal(size=s.H0.shape))
    Sinf = 0.5 * (Sinf + np.conj(np.swapaxes(Sinf, -1, -2)))
    Sig = systems.random_green(9, nspin, sp.ntau, sp.nk, sp.nao, scale=0.01)
    say("dyson", nspin, s_identity)
    plan = make_plan(s)
    G, mu, n, ev = plan.dyson(dev(s.H0), dev(s.S), dev(Sinf), dev(Sig), 0.05, n_target=s.n_target)
    G = host(G)
    Gr, mur, nr = ogw.solve_dyson(s.H0, s.S, Sinf, Sig, s.grid, nspin, 0.05, s.n_target)
    assert abs(n - s.n_target) <= 1e-12 * s.n_target
    assert abs(mu - mur) <= 1e-10
    assert rel(G, Gr) <= TOL


def test_iterate_molecule_ten_iterations():
    """Gamma-only molecule-like system (nk=1, nao=8, naux=32, ntau=20, beta=50): 10 iterations, each compared."""
    _require_gpu()
    s = systems.make_system(configs.MOLECULE)
    sp = s.spec
    plan = make_plan(s)
    V, H0, S = dev(s.V), dev(s.H0), dev(s.S)
    G = dev(s.G0)
    Sinf = torch.zeros(plan.shape_H, dtype=torch.complex128, device="cuda:0")
    Sig = torch.zeros(plan.shape_G, dtype=torch.complex128, device="cuda:0")
    st = ogw.State(s.G0, None, None, 0.0)
    mu = 0.0
    for it in range(10):
        say("iterate molecule", it)
        mu, rep = plan.iterate(V, H0, S, G, Sinf, Sig, mu, s.n_target, 1.0)
        st, orep, _ = ogw.iterate(s, st)
        assert rel(host(Sig), st.Sig) <= TOL, it
        assert rel(host(Sinf), st.Sinf) <= TOL, it
        assert rel(host(G), st.G) <= TOL, it
        assert abs(mu - orep["mu"]) <= 1e-10
        for key in ("e_1b", "e_hf", "e_corr", "e_tot"):
            assert abs(rep[key] - orep[key]) <= 1e-10, (it, key, rep[key], orep[key])
        assert abs(rep["n_elec"] - s.n_target) <= 1e-11
        assert abs(rep["max_dsigma"] - orep["max_dsigma"]) <= 1e-10 * max(1.0, orep["max_dsigma"])


def test_iterate_mixing_parity():
    _require_gpu()
    sp = configs.tiny(kmesh=(2, 1, 1), nao=5, naux=11, ntau=16, beta=10.0, seed=131, v_scale=0.2)
    s = systems.make_system(sp)
    plan = make_plan(s)
    V, H0, S = dev(s.V), dev(s.H0), dev(s.S)
    G = dev(s.G0)
    Sinf = torch.zeros(plan.shape_H, dtype=torch.complex128, device="cuda:0")
    Sig = torch.zeros(plan.shape_G, dtype=torch.complex128, device="cuda:0")
    st = ogw.State(s.G0, np.zeros(plan.shape_H, complex), np.zeros(plan.shape_G, complex), 0.0)
    mu = 0.0
    for it in range(3):
        say("iterate mixing", it)
        mu, rep = plan.iterate(V, H0, S, G, Sinf, Sig, mu, s.n_target, 0.6)
        st, orep, _ = ogw.iterate(s, st, alpha=0.6)
        assert rel(host(Sig), st.Sig) <= TOL
        assert abs(rep["e_tot"] - orep["e_tot"]) <= 1e-10


@pytest.fixture(scope="module")
def periodic2():
    return systems.make_system(configs.PERIODIC_2)


def test_iterate_periodic_2x2x2_full(periodic2):
    """nk=8 (2x2x2), nao=26, naux=180, ntau=104, beta=100: one full iteration, every output compared."""
    _require_gpu()
    s = periodic2
    plan = make_plan(s)
    V, H0, S = dev(s.V), dev(s.H0), dev(s.S)
    G = dev(s.G0)
    Sinf = torch.zeros(plan.shape_H, dtype=torch.complex128, device="cuda:0")
    Sig = torch.zeros(plan.shape_G, dtype=torch.complex128, device="cuda:0")
    say("iterate periodic 2x2x2")
    mu, rep = plan.iterate(V, H0, S, G, Sinf, Sig, 0.0, s.n_target, 1.0)
    st, orep, _ = ogw.iterate(s, ogw.State(s.G0, None, None, 0.0))
    assert rel(host(Sig), st.Sig) <= TOL
    assert rel(host(Sinf), st.Sinf) <= TOL
    assert rel(host(G), st.G) <= TOL
    assert abs(mu - orep["mu"]) <= 1e-10
    assert abs(rep["e_tot"] - orep["e_tot"]) <= 1e-10


def test_polarization_deterministic(periodic2):
    _require_gpu()
    s = periodic2
    plan = make_plan(s)
    V, G = dev(s.V), dev(s.G0)
    say("determinism")
    a = host(plan.polarization(V, G))
    b = host(plan.polarization(V, G))
    assert np.array_equal(a, b)


def test_nan_input_is_reported():
    _require_gpu()
    from paper_2406_18479_amd._lib import GreenError
    s = systems.make_system(configs.MOLECULE)
    plan = make_plan(s)
    G0 = s.G0.copy()
    G0[0, 3, 0, 1, 2] = np.nan
    G = dev(G0)
    Sinf = torch.zeros(plan.shape_H, dtype=torch.complex128, device="cuda:0")
    Sig = torch.zeros(plan.shape_G, dtype=torch.complex128, device="cuda:0")
    say("nan input")
    with pytest.raises(GreenError) as e:
        plan.iterate(dev(s.V), dev(s.H0), dev(s.S), G, Sinf, Sig, 0.0, s.n_target, 1.0)
    assert e.value.code in (-4, -5, -6)
