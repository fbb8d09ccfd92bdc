"""More GPU parity against the FP64 oracle: the screening on the production grid size and at weak coupling, two
spins at nao >= 26, GF2 on the multi-tile large-tile path, an uneven batch against per-system oracle iterations,
and the device checks of the plan's input assumptions.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import gw as ogw
from synth import configs, systems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def _plan(s, prec="fp64", chunk=0):
    from paper_2406_18479_amd.gw import Plan
    sp = s.spec
    return Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin, prec=prec, chunk_bytes=chunk)


def _screen_ref(P0, grid):
    return ogw.from_bosonic(ogw.screen(ogw.to_bosonic(P0, grid.TB_t2w)), grid.TB_w2t)


@pytest.fixture(scope="module")
def screen136():
    """P~0 of a small system on the 3x3x3 workload's grid (ntau 136, nw_b 137, beta 100), from the oracle."""
    sp = configs.tiny(kmesh=(3, 1, 1), nao=4, naux=40, ntau=136, beta=100.0, seed=701, band=2.0)
    s = systems.make_system(sp)
    P0 = ogw.polarization(s.V, s.G0, sp.kmesh)
    return s, P0


def test_screen_on_the_production_grid(screen136):
    """green_gw_screen at ntau = 136 / nw_b = 137 against the oracle's transform, solve and inverse transform."""
    _require_gpu()
    s, P0 = screen136
    say("screen ntau=136")
    Pt = host(_plan(s).screen(dev(P0)))
    assert rel(Pt, _screen_ref(P0, s.grid)) <= 1e-10


@pytest.mark.parametrize("scale", [1e-4, 1e-7])
def test_screen_relative_accuracy_at_weak_coupling(screen136, scale):
    """Where |P~0(i W)| << 1 (here at every node: P~0 scaled down) P~ = [I - P~0]^{-1} P~0 ~ P~0 must keep its
    relative accuracy; forming it as [I - P~0]^{-1} - I would lose about eps / |P~0| of it.  Checked element by
    element at 1e-11 of the largest element, and at every bosonic node (the largest |W| included) after the
    forward transform, at 1e-9 of that node's largest element."""
    _require_gpu()
    s, P0 = screen136
    P0s = P0 * scale
    say("screen weak coupling", scale)
    Pt = host(_plan(s).screen(dev(P0s)))
    ref = _screen_ref(P0s, s.grid)
    assert rel(Pt, ref) <= 1e-11
    Pw, Pw_ref = ogw.to_bosonic(Pt, s.grid.TB_t2w), ogw.to_bosonic(ref, s.grid.TB_t2w)
    for m in range(Pw.shape[1]):
        node = np.max(np.abs(Pw_ref[:, m]))
        assert np.max(np.abs(Pw[:, m] - Pw_ref[:, m])) <= 1e-9 * node, m


def test_two_spins_at_nao_26():
    """Unrestricted (two distinct spin channels) P~0, Sigma~ and one iteration at nao = 26 (MFMA tiles over the
    orbital pairs), against the oracle."""
    _require_gpu()
    sp = configs.tiny(kmesh=(2, 1, 1), nao=26, naux=64, ntau=10, beta=8.0, nspin=2, seed=702,
                      v_scale=0.5 / 26 ** 0.5)
    s = systems.make_system(sp)
    p = _plan(s)
    V, G = dev(s.V), dev(s.G0)
    say("two spins nao=26")
    P0 = ogw.polarization(s.V, s.G0, sp.kmesh)
    assert rel(host(p.polarization(V, G)), P0) <= 1e-10
    Pt = systems.random_polarization(703, sp.nk, sp.ntau, sp.naux, scale=0.05)
    assert rel(host(p.selfenergy(V, G, dev(Pt))), ogw.selfenergy(s.V, s.G0, Pt, sp.kmesh)) <= 1e-10
    Gd = dev(s.G0)
    Sinf = torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0")
    Sig = torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0")
    mu, rep = p.iterate(V, dev(s.H0), dev(s.S), Gd, Sinf, Sig, 0.0, s.n_target, 1.0)
    st, orep, _ = ogw.iterate(s, ogw.State(s.G0, None, None, 0.0))
    assert rel(host(Sig), st.Sig) <= 1e-10 and rel(host(Gd), st.G) <= 1e-10
    assert abs(mu - orep["mu"]) <= 1e-10 and abs(rep["e_tot"] - orep["e_tot"]) <= 1e-10


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x3", 2e-5)])
def test_gf2_multi_tile_orbital_pairs(prec, tol):
    """GF2 with nao^2 = 256 rows and columns in the auxiliary sums (more than one 192-row large tile in split
    BF16), against O14."""
    _require_gpu()
    sp = configs.tiny(kmesh=(2, 1, 1), nao=16, naux=24, ntau=6, beta=6.0, seed=704, v_scale=0.5 / 4.0)
    s = systems.make_system(sp)
    G = systems.random_green(705, 1, sp.ntau, sp.nk, sp.nao, scale=0.4)
    say("gf2 nao=16", prec)
    ref = ogw.gf2_selfenergy(s.V, G, sp.kmesh)
    p = _plan(s, prec)
    p.set_option("gf2", 1)
    assert rel(host(p.gf2_selfenergy(dev(s.V), dev(G))), ref) <= tol


BATCH = [dict(kmesh=(1, 1, 1), nao=8, naux=32, ntau=20, beta=50.0, seed=711),
         dict(kmesh=(2, 1, 1), nao=10, naux=40, ntau=16, beta=20.0, seed=712),
         dict(kmesh=(2, 2, 1), nao=7, naux=30, ntau=12, beta=10.0, seed=713, nspin=2),
         dict(kmesh=(3, 1, 1), nao=6, naux=36, ntau=16, beta=30.0, seed=714)]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_batched_iteration_against_the_oracle(prec):
    """One batched iteration of four uneven systems (green_gw_iterate_batched: grouped persistent launches)
    against the oracle's iteration of each system: FP64 at 1e-10 (Sigma~, G, E_tot), split BF16 within the
    accuracy bar (|dE| <= 1e-6 Eh, max|dSigma~| <= 1e-5 Eh)."""
    _require_gpu()
    from paper_2406_18479_amd.gw import iterate_batched
    ss = [systems.make_system(configs.tiny(**c)) for c in BATCH]
    plans = [_plan(s, prec) for s in ss]
    ys = []
    for s, p in zip(ss, plans):
        ys.append(dict(V=dev(s.V), H0=dev(s.H0), S=dev(s.S), G=dev(s.G0),
                       Sinf=torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0"),
                       Sigma=torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0"), mu=0.0,
                       n_target=s.n_target))
    say("batched vs oracle", prec)
    mus, reps = iterate_batched(plans, ys, 1.0)
    for s, y, mu, rep in zip(ss, ys, mus, reps):
        st, orep, _ = ogw.iterate(s, ogw.State(s.G0, None, None, 0.0))
        if prec == "fp64":
            assert rel(host(y["Sigma"]), st.Sig) <= 1e-10 and rel(host(y["G"]), st.G) <= 1e-10
            assert abs(rep["e_tot"] - orep["e_tot"]) <= 1e-10 and abs(mu - orep["mu"]) <= 1e-10
        else:
            assert abs(rep["e_tot"] - orep["e_tot"]) <= 1e-6
            assert float(np.max(np.abs(host(y["Sigma"]) - st.Sig))) <= 1e-5


def test_time_reversal_option_rejects_inputs_without_the_symmetry():
    """GREEN_OPT_TIME_REVERSAL on inputs that are not time-reversal symmetric: the device check latches the
    violation and the next synchronising call returns GREEN_EINVAL (instead of a wrong Sigma~); on symmetric
    inputs the same calls succeed."""
    _require_gpu()
    from paper_2406_18479_amd import _lib
    for tr_inputs in (False, True):
        sp = configs.tiny(kmesh=(3, 1, 1), nao=4, naux=10, ntau=8, beta=6.0, seed=715, v_time_reversal=tr_inputs)
        s = systems.make_system(sp)
        p = _plan(s)
        p.set_option("time_reversal", 1)
        say("time-reversal check, symmetric inputs:", tr_inputs)
        p.polarization(dev(s.V), dev(s.G0))
        if tr_inputs:
            p.check_status()
        else:
            with pytest.raises(_lib.GreenError) as e:
                p.check_status()
            assert e.value.code == -1
            p.check_status()  # cleared once reported


def test_debug_checks_flag_a_non_hermitian_g():
    """GREEN_CHECK=1 (a fresh process, the flag is read once): a G that is not Hermitian per (s, t, k) is
    reported as GREEN_EINVAL; the closed-form G0 passes."""
    _require_gpu()
    code = r'''
import sys
sys.path.insert(0, %r)
import numpy as np, torch
from synth import configs, systems
from paper_2406_18479_amd import _lib
from paper_2406_18479_amd.gw import Plan
sp = configs.tiny(kmesh=(2, 1, 1), nao=4, naux=8, ntau=8, beta=6.0, seed=716)
s = systems.make_system(sp)
p = Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=1)
dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
p.polarization(dev(s.V), dev(s.G0))
p.check_status()
G = s.G0.copy()
G[0, 3, 1, 0, 2] += 0.1
p.polarization(dev(s.V), dev(G))
try:
    p.check_status()
    print("NOT FLAGGED")
except _lib.GreenError as e:
    print("FLAGGED", e.code)
''' % ROOT
    env = dict(os.environ, GREEN_CHECK="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    say("debug-check subprocess:", out.stdout.strip()[-200:], out.stderr.strip()[-300:])
    assert out.returncode == 0 and "FLAGGED -1" in out.stdout
