"""The 4x4x4 target shape (nk 64, nao 78, naux 420, ntau 160, beta 200, two spins): one split-BF16 P~0 on the GPU
from the Hermitian half store of V (the 36 canonical-q slabs, 94 GB, generated in device memory), compared with the
oracle at sampled momentum transfers and tau nodes.  The oracle computes only the selected (q, tau) blocks, from the
slabs q and -q copied to the host."""
import numpy as np
import pytest

from oracle import gw as ogw
from synth import configs, systems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-case]", *a, flush=True)


class _Slabs:
    """V[q][k] for a few q only (host), indexable as the oracle indexes the full V."""

    def __init__(self, slabs, nk):
        self.slabs = slabs
        first = next(iter(slabs.values()))
        self.shape = (nk, nk) + tuple(first.shape[1:])

    def __getitem__(self, idx):
        q, k = idx
        return self.slabs[q][k]


def test_polarization_4x4x4_half_store_sampled():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_18479_amd.gw import Plan
    from synth import device
    spec = configs.LARGE_4
    s = systems.make_system(spec, with_V=False)
    plan = Plan(spec.kmesh, spec.nao, spec.naux, s.grid, nspin=spec.nspin, prec="bf16x3")
    plan.set_option("v_half", 1)
    qc = plan.canonical_q
    say("generate the half store of V on the device:", len(qc), "slabs")
    Vh = device.make_V(spec, device="cuda:0", qs=qc)
    G = torch.from_numpy(np.ascontiguousarray(s.G0)).to("cuda:0")
    say("polarization 4x4x4 bf16x3, half store")
    P = plan.polarization(Vh, G)
    # q = 0 is its own partner (contracted on the first 80 nodes, the rest transposed); q = 1 and its partner 3;
    # split-BF16 chunks of 3 tau nodes, so 2|3 is a chunk edge and 79|80 the half of q = 0
    qs, ts = [0, 1, 3], [2, 3, 79, 80]
    got = P[qs][:, ts].cpu().numpy()
    del P, Vh, plan
    torch.cuda.empty_cache()
    say("oracle slabs and sampled blocks")
    Vq = device.make_V(spec, device="cuda:0", qs=[0, 1, 3])
    slabs = {q: Vq[i].cpu().numpy() for i, q in enumerate([0, 1, 3])}
    del Vq
    torch.cuda.empty_cache()
    ref = ogw.polarization(_Slabs(slabs, spec.nk), s.G0, spec.kmesh, ts=ts, qs=qs)
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    say(f"4x4x4 split-BF16 P~0 vs oracle at q {qs} tau {ts}: max rel err {err:.3e}")
    assert err <= 4e-5
