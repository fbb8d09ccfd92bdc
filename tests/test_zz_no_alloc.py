"""green_dyson_noalloc (static device scratch, no workspace) against green_dyson on the same inputs.

Two calls in a row on different plans, the second with a smaller input, so the second call runs in a scratch
that still holds the first call's contents.  Bar: FP64, max|dG| / max|G| <= 1e-10, |d mu| <= 1e-10.
"""
import numpy as np
import pytest

from synth import configs, systems

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _case(kmesh, nao, ntau, nspin, seed):
    sp = configs.tiny(kmesh=kmesh, nao=nao, naux=4, ntau=ntau, beta=8.0, nspin=nspin, seed=seed, band=1.0,
                      s_identity=False)
    s = systems.make_system(sp, with_V=False)
    rng = np.random.default_rng(seed)
    nk = sp.nk
    Z = rng.normal(size=(nspin, nk, nao, nao)) + 1j * rng.normal(size=(nspin, nk, nao, nao))
    Sinf = 0.05 * (Z + np.conj(np.swapaxes(Z, -1, -2)))
    Sig = systems.random_green(seed + 1, nspin, ntau, nk, nao, scale=0.02)
    return s, Sinf, Sig


@pytest.mark.parametrize("n_target_mode", ["search", "fixed"])
def test_dyson_noalloc_equals_dyson(n_target_mode):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_18479_amd.gw import Plan
    for kmesh, nao, ntau, nspin, seed in [((2, 2, 1), 13, 24, 2, 5), ((1, 1, 1), 5, 12, 1, 6)]:
        print(f"[gpu-case] dyson_noalloc kmesh={kmesh} nao={nao} ntau={ntau} nspin={nspin} {n_target_mode}",
              flush=True)
        s, Sinf, Sig = _case(kmesh, nao, ntau, nspin, seed)
        sp = s.spec
        plan = Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin)
        H0, S, Sinf_d, Sig_d = _dev(s.H0), _dev(s.S), _dev(Sinf), _dev(Sig)
        nt = s.n_target if n_target_mode == "search" else -1.0
        G1, mu1, n1, ev1 = plan.dyson(H0, S, Sinf_d, Sig_d, 0.05, n_target=nt)
        G2, mu2, n2, ev2 = plan.dyson_noalloc(H0, S, Sinf_d, Sig_d, 0.05, n_target=nt)
        torch.cuda.synchronize()
        a, b = G2.cpu().numpy(), G1.cpu().numpy()
        err = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        assert err <= 1e-10, err
        assert abs(mu1 - mu2) <= 1e-10 and abs(n1 - n2) <= 1e-10 * max(1.0, abs(n1))
        assert ev1 == ev2
        plan.close()


def test_dyson_noalloc_rejects_a_plan_beyond_the_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_18479_amd import _lib
    from paper_2406_18479_amd.gw import Plan
    from synth import grid as gridmod
    g = gridmod.make_grid(40, 10.0)
    # Sigma~(i w) and the Dyson matrices: 2 x 40 x 8 x 96^2 x 16 B = 94 MB > 64 MiB
    plan = Plan((2, 2, 2), 96, 4, g, nspin=1)
    z = torch.zeros(plan.shape_H, dtype=torch.complex128, device="cuda:0")
    S = torch.eye(96, dtype=torch.complex128, device="cuda:0").repeat(8, 1, 1)
    Sig = torch.zeros(plan.shape_G, dtype=torch.complex128, device="cuda:0")
    with pytest.raises(_lib.GreenError) as e:
        plan.dyson_noalloc(z, S, z, Sig, 0.0)
    assert e.value.code == -2
    plan.close()
