"""Full-size checks on the 3x3x3 workload (nk=27, nao=52, naux=300, ntau=136, beta=100), the shape the
precision comparison is made on.  V (9.5 GB) is generated in device memory; the FP64 oracle evaluates
sampled outputs one by one from the same inputs copied to the host.
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


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def periodic3():
    _require_gpu()
    from synth import device
    spec = configs.PERIODIC_3
    s = systems.make_system(spec, with_V=False)
    say("generate V on device", spec.name)
    s.V_dev = device.make_V(spec, device="cuda:0")
    torch.cuda.synchronize()
    s.V = s.V_dev.cpu().numpy()
    return s


def _plan(s, prec):
    from paper_2406_18479_amd.gw import Plan
    sp = s.spec
    return Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin, prec=prec)


def test_polarization_sampled_tau(periodic3):
    """FP64 P~0 of the whole 3x3x3 workload at 12 tau nodes against the oracle: the FP64 plan contracts chunks of
    12 nodes (8 GiB of intermediates), so the nodes sit on both sides of chunk edges (11|12, 35|36, 59|60,
    131|132), and for q = 0 (its own partner) on both sides of the half the library contracts (67|68, the rest
    transposed from the first half); every q, with the partners -q of the +-q identity."""
    s = periodic3
    sp = s.spec
    say("polarization 3x3x3 fp64")
    p = _plan(s, "fp64")
    P = p.polarization(s.V_dev, torch.from_numpy(s.G0).to("cuda:0"))
    ts = [0, 11, 12, 35, 36, 59, 60, 67, 68, 100, 131, 132, 135]
    got = P[:, ts].cpu().numpy()
    del P, p
    torch.cuda.empty_cache()
    ref = ogw.polarization(s.V, s.G0, sp.kmesh, ts=ts)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("tile", [3, 4])
def test_polarization_tall_tiles_sampled_tau(periodic3, tile):
    """Split-BF16 P~0 with the 320- and 448-row output tiles at full size, sampled tau nodes against the
    oracle (same relative bound as the other split-BF16 contractions)."""
    s = periodic3
    sp = s.spec
    say("polarization 3x3x3 bf16x3 p0_tile", tile)
    p = _plan(s, "bf16x3")
    p.set_option("p0_tile", tile)
    P = p.polarization(s.V_dev, torch.from_numpy(s.G0).to("cuda:0"))
    ts = [1, 70]
    got = P[:, ts].cpu().numpy()
    del P, p
    torch.cuda.empty_cache()
    ref = ogw.polarization(s.V, s.G0, sp.kmesh, ts=ts)
    assert np.max(np.abs(got - ref)) <= 4e-5 * np.max(np.abs(ref))


def test_selfenergy_sampled_k_tau(periodic3):
    from synth import device
    s = periodic3
    sp = s.spec
    say("selfenergy 3x3x3 fp64")
    p = _plan(s, "fp64")
    G = systems.random_green(301, 1, sp.ntau, sp.nk, sp.nao, scale=0.05)
    Pt = device.random_polarization(302, sp.nk, sp.ntau, sp.naux, scale=0.02, device="cuda:0")
    Sig = p.selfenergy(s.V_dev, torch.from_numpy(G).to("cuda:0"), Pt)
    ks, ts = [0, 13, 26], [5, 100]
    got = Sig[:, ts][:, :, ks].cpu().numpy()
    Pt_h = Pt[:, ts].cpu().numpy()
    del Sig, Pt, p
    torch.cuda.empty_cache()
    ref = ogw.selfenergy(s.V, G, Pt_h, sp.kmesh, ts=ts, ks=ks)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_mixed_precision_bar_3x3x3(periodic3):
    """One iteration from identical inputs: FP32 and split BF16 within |dE| <= 1e-6 Eh, max|dSigma| <= 1e-5 Eh
    of the FP64 path; the FP64 iteration keeps the electron count."""
    s = periodic3
    out = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        say("iterate 3x3x3", prec)
        p = _plan(s, prec)
        G = torch.from_numpy(s.G0).to("cuda:0")
        Sinf = torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0")
        Sig = torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0")
        mu, rep = p.iterate(s.V_dev, torch.from_numpy(s.H0).to("cuda:0"), torch.from_numpy(s.S).to("cuda:0"), G,
                            Sinf, Sig, 0.0, s.n_target, 1.0)
        out[prec] = (Sig.cpu().numpy(), rep)
        say(prec, "ms", [round(x, 1) for x in rep["ms"]], "E_tot", rep["e_tot"])
        del p, G, Sinf, Sig
        torch.cuda.empty_cache()
    assert abs(out["fp64"][1]["n_elec"] - s.n_target) <= 1e-11 * s.n_target
    for prec in ("fp32", "bf16x3"):
        dE = abs(out[prec][1]["e_tot"] - out["fp64"][1]["e_tot"])
        dS = float(np.max(np.abs(out[prec][0] - out["fp64"][0])))
        say(f"{prec}: |dE| = {dE:.3e} Eh, max|dSigma| = {dS:.3e} Eh")
        assert dE <= 1e-6 and dS <= 1e-5
