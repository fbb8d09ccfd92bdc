"""Mixed-precision contractions (FP32 and split-BF16 hi+lo on MFMA, FP32 accumulation flushed to FP64)
against the FP64 path on the same inputs.

The contraction error bound follows from the arithmetic: FP32 rounds each
operand to 2^-24 relative; split BF16 keeps hi + lo to 2^-18 relative and
drops the lo*lo term, so each product carries up to ~3 * 2^-18 ~ 1.1e-5
relative error.  Sums of such products stay within that relative error of
the sum of magnitudes; the tests allow a factor ~3 margin on the max-norm.
The acceptance bar for a full iteration is |dE| <= 1e-6 Eh and
max|dSigma| <= 1e-5 Eh (checked on the 2x2x2 workload).
"""
import numpy as np
import pytest

from synth import configs, systems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

REL = {"fp32": 3e-6, "bf16x3": 4e-5}


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


def plan(s, prec):
    from paper_2406_18479_amd.gw import Plan
    sp = s.spec
    return Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin, prec=prec)


SMALL = [dict(kmesh=(2, 2, 1), nao=11, naux=53, ntau=12, seed=201),     # skinny stage-1 path, K <= 32
         dict(kmesh=(2, 1, 1), nao=40, naux=70, ntau=8, seed=202),      # K <= 64
         dict(kmesh=(1, 1, 1), nao=6, naux=200, ntau=6, seed=203)]      # naux > 192: two large tiles along M


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("c", SMALL, ids=lambda c: f"nao{c['nao']}_naux{c['naux']}")
def test_mixed_polarization_and_selfenergy(c, prec):
    _require_gpu()
    s = systems.make_system(configs.tiny(kmesh=c["kmesh"], nao=c["nao"], naux=c["naux"], ntau=c["ntau"], beta=8.0,
                                         seed=c["seed"], v_scale=0.5 / c["nao"] ** 0.5))
    print("[gpu-case] mixed contractions", prec, c, flush=True)
    V, G = dev(s.V), dev(s.G0)
    p64, pmx = plan(s, "fp64"), plan(s, prec)
    P64 = host(p64.polarization(V, G))
    Pmx = host(pmx.polarization(V, G))
    assert rel(Pmx, P64) <= REL[prec]
    Pt = dev(systems.random_polarization(7, s.spec.nk, s.spec.ntau, s.spec.naux, scale=0.1))
    S64 = host(p64.selfenergy(V, G, Pt))
    Smx = host(pmx.selfenergy(V, G, Pt))
    assert rel(Smx, S64) <= REL[prec]


@pytest.mark.parametrize("tile,nao", [(1, 10), (2, 10), (3, 10), (4, 10), (5, 10), (6, 10), (7, 10), (5, 12), (6, 12),
                                      (7, 12), (8, 12), (9, 12), (10, 12), (11, 12), (12, 10), (13, 10), (12, 12),
                                      (13, 12)])
def test_split_bf16_p0_tiles(tile, nao):
    """Every output tile of the split-BF16 P~0 contraction (register-staged 192 x 96, 192 x 64, 320 x 64,
    448 x 64; LDS-DMA 320 x 64, 192 x 128; LDS-DMA with operands read a stage ahead 320 x 64, 128 x 128,
    256 x 64, and two workgroups per CU 128 x 64, 64 x 128; LDS-DMA with 32-K stages 128 x 128, 256 x 64) on an
    naux that leaves ragged tiles along both P~0 dimensions, against the FP64 path.  nao = 10:
    K = nk nao^2 = 200, whose orbital-pair blocks (100) and end fall inside 16-wide K stages (the read-ahead
    kernel then falls back to the register-staged one); nao = 12: blocks of 144 that are whole stages."""
    _require_gpu()
    s = systems.make_system(configs.tiny(kmesh=(2, 1, 1), nao=nao, naux=350, ntau=6, beta=8.0, seed=204,
                                         v_scale=0.5 / nao ** 0.5))
    print("[gpu-case] split-BF16 P0 tile", tile, "nao", nao, flush=True)
    V, G = dev(s.V), dev(s.G0)
    p64, pmx = plan(s, "fp64"), plan(s, "bf16x3")
    pmx.set_option("p0_tile", tile)
    P64 = host(p64.polarization(V, G))
    Pmx = host(pmx.polarization(V, G))
    assert rel(Pmx, P64) <= REL["bf16x3"]


STAGE1 = [dict(kmesh=(2, 1, 1), nao=8, naux=40, ntau=10, nspin=1, seed=221),   # 16-wide blocks, ragged rows
          dict(kmesh=(3, 1, 1), nao=26, naux=50, ntau=8, nspin=2, seed=222),   # 32-wide blocks, two spins
          dict(kmesh=(2, 2, 1), nao=40, naux=30, ntau=12, nspin=1, seed=223),  # 48-wide blocks
          dict(kmesh=(2, 1, 1), nao=52, naux=70, ntau=6, nspin=1, seed=224),   # 64-wide blocks, padded
          dict(kmesh=(1, 1, 1), nao=64, naux=33, ntau=6, nspin=1, seed=225),   # 64-wide blocks, no padding
          dict(kmesh=(2, 2, 1), nao=64, naux=300, ntau=20, nspin=1, seed=226),  # 3 tau nodes per workgroup
          dict(kmesh=(2, 1, 1), nao=78, naux=40, ntau=6, nspin=2, seed=227),    # 80-wide blocks, two spins
          dict(kmesh=(1, 1, 1), nao=66, naux=31, ntau=6, nspin=1, seed=228),    # 80-wide blocks, mostly padding
          dict(kmesh=(2, 2, 1), nao=80, naux=400, ntau=12, nspin=1, seed=229),  # 80-wide, 4 nodes per workgroup
          dict(kmesh=(1, 1, 1), nao=2, naux=1, ntau=4, nspin=1, seed=230),     # smallest even nao, one aux row
          dict(kmesh=(3, 1, 1), nao=16, naux=9, ntau=6, nspin=1, seed=231),    # exactly one 16-wide block
          dict(kmesh=(2, 1, 1), nao=18, naux=7, ntau=6, nspin=2, seed=232),    # 32-wide, 2 valid in the last block
          dict(kmesh=(1, 2, 1), nao=48, naux=5, ntau=8, nspin=1, seed=233),    # exactly three blocks
          dict(kmesh=(2, 1, 1), nao=50, naux=6, ntau=6, nspin=1, seed=234)]    # 64-wide, 2 valid in the last block


@pytest.mark.parametrize("c", STAGE1, ids=lambda c: f"nao{c['nao']}_naux{c['naux']}_ns{c['nspin']}")
def test_split_bf16_stage1_direct(c):
    """The direct P~0 stage-1 kernel (V rows in registers over the tau chunk, G^T per node in LDS) against the
    192 x 96 tile kernel of the same split-BF16 plan (same products and roundings, other blocking) and against
    the FP64 path, for every block width (nao up to 16, 32, 48, 64, 80), ragged row counts (naux nao not a
    multiple of the rows of a workgroup), two spins, and shapes whose chunk is split into parts of several tau
    nodes."""
    _require_gpu()
    s = systems.make_system(configs.tiny(kmesh=c["kmesh"], nao=c["nao"], naux=c["naux"], ntau=c["ntau"], beta=8.0,
                                         nspin=c["nspin"], seed=c["seed"], v_scale=0.5 / c["nao"] ** 0.5))
    print("[gpu-case] direct stage-1 kernel", c, flush=True)
    V, G = dev(s.V), dev(s.G0)
    p64, pmx = plan(s, "fp64"), plan(s, "bf16x3")
    P64 = host(p64.polarization(V, G))
    pmx.set_option("stage1_tile", 3)
    Pd = host(pmx.polarization(V, G))
    pmx.set_option("stage1_tile", 1)
    Pt = host(pmx.polarization(V, G))
    assert rel(Pd, Pt) <= 2e-6
    assert rel(Pd, P64) <= REL["bf16x3"]


@pytest.mark.parametrize("tile", [5, 6, 7, 8, 9, 10, 11, 12, 13])
@pytest.mark.parametrize("naux", [300, 52, 64, 70])
def test_split_bf16_sigma_tiles(tile, naux):
    """Every LDS-DMA tile of the first split-BF16 Sigma~ contraction (P~^T V over the auxiliary index, K = naux)
    against the FP64 path: naux 300 and 52 end in a partial 16-wide K stage (12 and 4 left), 64 in whole stages,
    70 is not a multiple of 4 (operands in plain rather than grouped split-BF16 layout)."""
    _require_gpu()
    s = systems.make_system(configs.tiny(kmesh=(2, 1, 1), nao=8, naux=naux, ntau=10, beta=8.0, seed=209,
                                         v_scale=0.5 / 8 ** 0.5))
    print("[gpu-case] split-BF16 Sigma stage-1 tile", tile, "naux", naux, flush=True)
    V, G = dev(s.V), dev(s.G0)
    Pt = dev(systems.random_polarization(11, s.spec.nk, s.spec.ntau, s.spec.naux, scale=0.1))
    p64, pmx = plan(s, "fp64"), plan(s, "bf16x3")
    pmx.set_option("sigma_tile", tile)
    S64 = host(p64.selfenergy(V, G, Pt))
    Smx = host(pmx.selfenergy(V, G, Pt))
    assert rel(Smx, S64) <= REL["bf16x3"]


FUSED = [dict(kmesh=(2, 1, 1), nao=8, naux=40, ntau=10, seed=205),     # one 16-row block
         dict(kmesh=(3, 1, 1), nao=28, naux=90, ntau=8, seed=206),     # two blocks, padded
         dict(kmesh=(2, 1, 1), nao=40, naux=75, ntau=6, seed=207),     # four blocks, the last one empty
         dict(kmesh=(1, 1, 1), nao=64, naux=33, ntau=6, seed=208),     # four full blocks, odd naux
         dict(kmesh=(3, 1, 1), nao=26, naux=60, ntau=8, seed=209),     # V^T rows padded from 26 to 28
         dict(kmesh=(2, 1, 1), nao=78, naux=40, ntau=6, seed=210),     # 80-row blocks, two-slot ring
         dict(kmesh=(1, 1, 1), nao=66, naux=31, ntau=6, seed=211)]     # 80-row blocks, mostly padding


@pytest.mark.parametrize("c", FUSED, ids=lambda c: f"nao{c['nao']}_naux{c['naux']}")
def test_sigma_fused_stages(c):
    """Split-BF16 self-energy with stages 2 and 3 fused (intermediate in registers) against the same plan
    with the two stages through HBM (same roundings of the intermediate, other summation order) and
    against the FP64 path."""
    _require_gpu()
    s = systems.make_system(configs.tiny(kmesh=c["kmesh"], nao=c["nao"], naux=c["naux"], ntau=c["ntau"], beta=8.0,
                                         seed=c["seed"], v_scale=0.5 / c["nao"] ** 0.5))
    print("[gpu-case] fused sigma stages", c, flush=True)
    V, G = dev(s.V), dev(s.G0)
    Pt = dev(systems.random_polarization(9, s.spec.nk, s.spec.ntau, s.spec.naux, scale=0.1))
    p64, pmx = plan(s, "fp64"), plan(s, "bf16x3")
    S64 = host(p64.selfenergy(V, G, Pt))
    pmx.set_option("sigma_fused", 1)
    Sf = host(pmx.selfenergy(V, G, Pt))
    pmx.set_option("sigma_fused", 0)
    Su = host(pmx.selfenergy(V, G, Pt))
    assert rel(Sf, Su) <= 1e-5
    assert rel(Sf, S64) <= REL["bf16x3"]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_iteration_periodic_2x2x2(prec):
    """One iteration of the 2x2x2 workload from identical inputs: |dE| <= 1e-6 Eh, max|dSigma| <= 1e-5 Eh."""
    _require_gpu()
    s = systems.make_system(configs.PERIODIC_2)
    out = {}
    for pr in ("fp64", prec):
        print("[gpu-case] mixed iteration", pr, flush=True)
        p = plan(s, pr)
        G = dev(s.G0)
        Sinf = torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0")
        Sig = torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0")
        mu, rep = p.iterate(dev(s.V), dev(s.H0), dev(s.S), G, Sinf, Sig, 0.0, s.n_target, 1.0)
        out[pr] = (host(Sig), rep)
        del p
    dE = abs(out[prec][1]["e_tot"] - out["fp64"][1]["e_tot"])
    dS = float(np.max(np.abs(out[prec][0] - out["fp64"][0])))
    print(f"[gpu-case] {prec}: |dE| = {dE:.3e} Eh, max|dSigma| = {dS:.3e} Eh", flush=True)
    assert dE <= 1e-6
    assert dS <= 1e-5
