"""k-path interpolation of the self-energy (Sec. 2.4) on the GPU against the oracle, and the Green's function
on the path from the Dyson equation with the interpolated self-energy."""
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


def _hermitian(rng, shape, scale):
    a = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    return scale * (a + np.swapaxes(a.conj(), -1, -2)) / 2


@pytest.mark.parametrize("kmesh,nspin", [((2, 3, 1), 1), ((4, 1, 3), 2)])
def test_kpath_interpolation_parity(kmesh, nspin):
    _require_gpu()
    from paper_2406_18479_amd.gw import Plan
    s = systems.make_system(configs.tiny(kmesh=kmesh, nao=5, naux=6, ntau=8, beta=10.0, seed=451, nspin=nspin))
    sp = s.spec
    print("[gpu-case] k-path interpolation", kmesh, nspin, flush=True)
    rng = np.random.default_rng(452)
    Sinf = _hermitian(rng, (nspin, sp.nk, sp.nao, sp.nao), 0.3)
    Sig = systems.random_green(453, nspin, sp.ntau, sp.nk, sp.nao, scale=0.1)
    path = np.vstack([rng.uniform(-0.5, 1.0, size=(11, 3)),
                      [[a / kmesh[0], b / kmesh[1], c / kmesh[2]] for a, b, c in [(0, 0, 0), (1, 0, 0)]]])
    p = Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=nspin, prec="fp64")
    Sinf_p, Sig_p = p.kpath_interpolate(path, dev(Sinf), dev(Sig))
    assert rel(host(Sinf_p), ogw.kpath_interpolate(Sinf, kmesh, path)) <= 1e-12
    assert rel(host(Sig_p), ogw.kpath_interpolate(Sig, kmesh, path)) <= 1e-12
    # the last two path points are mesh points: the mesh values come back
    assert np.max(np.abs(host(Sig_p)[:, :, -2] - Sig[:, :, 0])) <= 1e-13
    assert np.max(np.abs(host(Sig_p)[:, :, -1] - Sig[:, :, kmesh[1] * kmesh[2]])) <= 1e-13


def test_green_function_on_a_kpath():
    """One GW iteration on a 2x2x1 mesh, its self-energy interpolated onto 9 path points, H0 and S given on
    the path, Dyson at the mesh's chemical potential (kept): G on the path against the oracle."""
    _require_gpu()
    from paper_2406_18479_amd.gw import Plan
    s = systems.make_system(configs.tiny(kmesh=(2, 2, 1), nao=6, naux=14, ntau=20, beta=20.0, seed=461))
    sp = s.spec
    print("[gpu-case] G on a k-path", flush=True)
    p = Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin, prec="fp64")
    G = dev(s.G0)
    Sinf = torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0")
    Sig = torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0")
    mu, _ = p.iterate(dev(s.V), dev(s.H0), dev(s.S), G, Sinf, Sig, 0.0, s.n_target, 1.0)
    t = np.linspace(0.0, 1.0, 9)
    path = np.stack([0.5 * t, 0.25 * t, 0.0 * t], axis=1)
    Sinf_p, Sig_p = p.kpath_interpolate(path, Sinf, Sig)
    rng = np.random.default_rng(462)
    npath = path.shape[0]
    H0p = np.stack([s.H0[:, 0]] * npath, axis=1) + _hermitian(rng, (sp.nspin, npath, sp.nao, sp.nao), 0.05)
    Sp = np.stack([np.eye(sp.nao, dtype=complex)] * npath)
    pp = Plan((npath, 1, 1), sp.nao, 4, s.grid, nspin=sp.nspin, prec="fp64")
    Gp, mu_p, n_p, _ = pp.dyson(dev(H0p), dev(Sp), Sinf_p, Sig_p, mu, n_target=-1.0)
    assert mu_p == mu
    ref, _, _ = ogw.solve_dyson(H0p, Sp, host(Sinf_p), host(Sig_p), s.grid, sp.nspin, mu, -1.0)
    assert rel(host(Gp), ref) <= 1e-10
