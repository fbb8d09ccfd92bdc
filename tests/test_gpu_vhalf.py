"""Hermitian half store of V (only the slabs of q with -q >= q passed; the others built from their partners on
use): iterations equal those with the full V bit for bit, since the synthetic V has the exact pairing
V^{k2,k1}(Q) = V^{k1,k2}(Q)^dagger; with time reversal on time-reversal-symmetric inputs (pairing exact only to
rounding) the iteration matches the oracle at 1e-10."""
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


def _plan(s, prec, half, trev=False):
    from paper_2406_18479_amd.gw import Plan
    sp = s.spec
    p = Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin, prec=prec)
    if half:
        p.set_option("v_half", 1)
    if trev:
        p.set_option("time_reversal", 1)
    return p


def _state(s, p, V):
    return dict(V=V, H0=dev(s.H0), S=dev(s.S), G=dev(s.G0),
                Sinf=torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0"),
                Sigma=torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0"), mu=0.0)


def _iterate(p, y, s):
    y["mu"], rep = p.iterate(y["V"], y["H0"], y["S"], y["G"], y["Sinf"], y["Sigma"], y["mu"], s.n_target, 1.0)
    return rep


CASES = [dict(kmesh=(3, 2, 1), nao=8, naux=20, ntau=8, nspin=1, seed=801),
         dict(kmesh=(3, 1, 2), nao=5, naux=13, ntau=6, nspin=2, seed=802)]  # (a 2x2x2 mesh has every q = -q)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("c", CASES, ids=lambda c: f"k{c['kmesh']}_nao{c['nao']}_ns{c['nspin']}")
def test_half_store_equals_full_store(c, prec):
    _require_gpu()
    s = systems.make_system(configs.tiny(kmesh=c["kmesh"], nao=c["nao"], naux=c["naux"], ntau=c["ntau"], beta=6.0,
                                         nspin=c["nspin"], seed=c["seed"], v_scale=0.5 / c["nao"] ** 0.5))
    pa, pb = _plan(s, prec, False), _plan(s, prec, True)
    Vh = s.V[pb.canonical_q]
    assert pb.shape_V == Vh.shape and Vh.shape[0] < s.V.shape[0]
    ya, yb = _state(s, pa, dev(s.V)), _state(s, pb, dev(Vh))
    for it in range(2):
        print(f"[gpu-case] half store {prec} {c} iteration {it}", flush=True)
        ra, rb = _iterate(pa, ya, s), _iterate(pb, yb, s)
        for key in ("G", "Sigma", "Sinf"):
            assert np.array_equal(host(ya[key]), host(yb[key])), (it, key)
        assert ra["e_tot"] == rb["e_tot"]


def test_half_store_with_time_reversal_matches_oracle():
    _require_gpu()
    sp = configs.tiny(kmesh=(3, 2, 1), nao=8, naux=20, ntau=8, beta=6.0, seed=803, v_scale=0.5 / 8 ** 0.5,
                      v_time_reversal=True)
    s = systems.make_system(sp)
    p = _plan(s, "fp64", True, trev=True)
    y = _state(s, p, dev(s.V[p.canonical_q]))
    st = ogw.State(s.G0, None, None, 0.0)
    for it in range(2):
        print(f"[gpu-case] half store + time reversal iteration {it}", flush=True)
        rep = _iterate(p, y, s)
        st, orep, _ = ogw.iterate(s, st)
        assert rel(host(y["Sigma"]), st.Sig) <= 1e-10
        assert rel(host(y["G"]), st.G) <= 1e-10
        assert abs(rep["e_tot"] - orep["e_tot"]) <= 1e-10
