"""Point-group reduction of the k sums (symmetry among the method's features, Sec. 3), on the CPU.

* The seeded generator of invariant systems: H0, S and V constant under the group (V^{R k1, R k2} = V^{k1,k2}),
  with the Hermitian pairing and, when asked, time reversal kept; the orbit counts of known meshes.
* The oracle on such a system (it contracts every k and q) shows the identities the library's fill rules use:
  P~0^{R q} = P~0^q, P~0^{-q}(tau) = P~0^q(beta - tau)^T, Sigma~^{R k} = Sigma~^k and, under time reversal,
  Sigma~^{-k} = conj Sigma~^k.
* The library's contracted sets (green_plan_set_kpoint_symmetry) and every launch in bounds (GREEN_DRYRUN=1).
"""
import ctypes

import numpy as np
import pytest

from oracle import gw as ogw
from synth import configs, systems
from synth import grid as gridmod
from synth import symmetry as sym


def _spec(kmesh=(3, 3, 3), nao=3, naux=5, ntau=8, trev=False, seed=911):
    return configs.tiny(kmesh=kmesh, nao=nao, naux=naux, ntau=ntau, beta=8.0, seed=seed, v_scale=0.6 / nao ** 0.5,
                        f_time_reversal=trev, v_time_reversal=trev)


GROUPS = {"Oh": sym.cubic_group, "C3": sym.threefold_group}


@pytest.mark.parametrize("kmesh,group,norb,order", [((3, 3, 3), "Oh", 4, 48), ((4, 4, 4), "Oh", 10, 48),
                                                    ((3, 3, 3), "C3", 11, 3), ((2, 2, 2), "Oh", 4, 6)])
def test_orbit_counts(kmesh, group, norb, order):
    """Irreducible points of Gamma-centred cubic meshes: 4 (3x3x3), 10 (4x4x4), 4 (2x2x2) under O_h; C3 about
    the body diagonal leaves the 3 diagonal points of 3x3x3 fixed and joins the other 24 in threes.  On the
    2x2x2 mesh the signs act trivially (-k = k), leaving the 6 axis permutations."""
    lab = sym.orbit_labels(kmesh, GROUPS[group]())
    assert len(set(lab.tolist())) == norb
    assert len(sym.group_closure(kmesh, GROUPS[group]())) == order


@pytest.mark.parametrize("trev", [False, True])
@pytest.mark.parametrize("group", ["Oh", "C3"])
def test_generator_is_invariant(group, trev):
    sp = _spec(trev=trev)
    s = sym.make_symmetric_system(sp, GROUPS[group]())
    km = ogw.KMesh(sp.kmesh)
    add = systems.k_add_table(sp.kmesh)
    for g in sym.group_closure(sp.kmesh, GROUPS[group]()):
        assert np.array_equal(s.H0[:, g], s.H0)
        assert np.array_equal(s.G0[:, :, g], s.G0)
        for k1 in range(km.nk):
            for k2 in range(km.nk):
                a = ogw.V_pair(s.V, km, k1, k2)
                b = ogw.V_pair(s.V, km, int(g[k1]), int(g[k2]))
                assert np.allclose(a, b, rtol=0, atol=1e-14 * np.max(np.abs(s.V)))
    # Hermitian pairing V^{k2,k1}(Q) = V^{k1,k2}(Q)^dagger
    for q in range(km.nk):
        for k in range(km.nk):
            k2 = int(add[k, q])
            assert np.allclose(ogw.V_pair(s.V, km, k2, k), np.conj(np.swapaxes(ogw.V_pair(s.V, km, k, k2), 1, 2)),
                               rtol=0, atol=1e-14 * np.max(np.abs(s.V)))
    if trev:
        neg = systems.k_neg(sp.kmesh)
        assert np.allclose(s.H0[:, neg], np.conj(s.H0), rtol=0, atol=1e-14)
        for k1 in range(km.nk):
            for k2 in range(km.nk):
                assert np.allclose(ogw.V_pair(s.V, km, int(neg[k1]), int(neg[k2])), np.conj(ogw.V_pair(s.V, km, k1, k2)),
                                   rtol=0, atol=1e-14 * np.max(np.abs(s.V)))


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("trev", [False, True])
@pytest.mark.parametrize("group", ["Oh", "C3"])
def test_oracle_shows_the_fill_identities(group, trev):
    """What the library copies instead of contracting, computed in full by the oracle."""
    sp = _spec(trev=trev)
    s = sym.make_symmetric_system(sp, GROUPS[group]())
    km = ogw.KMesh(sp.kmesh)
    nt = sp.ntau
    P0 = ogw.polarization(s.V, s.G0, sp.kmesh)
    neg = systems.k_neg(sp.kmesh)
    for g in sym.group_closure(sp.kmesh, GROUPS[group]()):
        assert _rel(P0[g], P0) <= 1e-12
    # the +-q identity (every system) and the time-reversal one
    assert _rel(P0[neg], np.swapaxes(P0[:, ::-1], 2, 3)) <= 1e-12
    if trev:
        assert _rel(P0[neg], np.conj(P0)) <= 1e-12
    Pw = ogw.screen(ogw.to_bosonic(P0, s.grid.TB_t2w))
    Pt = ogw.from_bosonic(Pw, s.grid.TB_w2t)
    for g in sym.group_closure(sp.kmesh, GROUPS[group]()):
        assert _rel(Pt[g], Pt) <= 1e-11
    assert _rel(Pt[neg], np.swapaxes(Pt[:, ::-1], 2, 3)) <= 1e-11
    Sig = ogw.selfenergy(s.V, s.G0, Pt, sp.kmesh)
    for g in sym.group_closure(sp.kmesh, GROUPS[group]()):
        assert _rel(Sig[:, :, g], Sig) <= 1e-11
    if trev:
        assert _rel(Sig[:, :, neg], np.conj(Sig)) <= 1e-11
    assert nt == Sig.shape[1] and km.nk == Sig.shape[2]


# ------------------------------------------------------------------------------------------- library (dry run)
BASE = 1 << 44
STEP = 1 << 40


@pytest.fixture
def lib(monkeypatch):
    monkeypatch.setenv("GREEN_DRYRUN", "1")
    from paper_2406_18479_amd import _lib
    return _lib


def _plan(lib, kmesh, nao, naux, ntau, nspin=1, prec=0):
    g = gridmod.make_grid(ntau, 50.0)
    d = lib.Dims((ctypes.c_int32 * 3)(*kmesh), nao, naux, ntau, len(g.nf), len(g.nb), nspin, 50.0)
    keep = [np.ascontiguousarray(a) for a in (g.tau, g.wf, g.wb)]
    keep += [np.ascontiguousarray(a, dtype=np.complex128) for a in (g.TF_t2w, g.TF_w2t, g.TB_t2w, g.TB_w2t)]
    gc = lib.GridC(*[a.ctypes.data for a in keep])
    h = ctypes.c_void_p()
    assert lib.LIB.green_plan_create(ctypes.byref(d), ctypes.byref(gc), prec, 0, ctypes.byref(h)) == 0
    return h


def _set(lib, h, ops):
    rot = np.ascontiguousarray(np.asarray(ops, dtype=np.int32).reshape(-1, 9))
    counts = (ctypes.c_int32 * 2)()
    ptr = rot.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if len(rot) else None
    st = lib.LIB.green_plan_set_kpoint_symmetry(h, ptr, len(rot), counts)
    return st, (int(counts[0]), int(counts[1]))


@pytest.mark.parametrize("kmesh,group,trev,counts", [
    ((3, 3, 3), "Oh", 0, (4, 4)), ((3, 3, 3), "Oh", 1, (4, 4)), ((4, 4, 4), "Oh", 0, (10, 10)),
    ((3, 3, 3), "C3", 0, (6, 11)), ((3, 3, 3), "C3", 1, (6, 6)), ((2, 2, 2), "Oh", 1, (4, 4))])
def test_contracted_sets(lib, kmesh, group, trev, counts):
    """Transfers: one orbit of each pair {O, -O}; momenta: one per orbit, per pair under time reversal (C3 on
    3x3x3: the diagonal gives {0} and {111, 222}, the 24 others 8 orbits in 4 pairs)."""
    h = _plan(lib, kmesh, 4, 8, 8)
    try:
        assert lib.LIB.green_plan_set_option(h, lib.OPT_TIME_REVERSAL, trev) == 0
        st, got = _set(lib, h, GROUPS[group]())
        assert st == 0 and got == counts
        # switching time reversal afterwards rebuilds the sets
        assert lib.LIB.green_plan_set_option(h, lib.OPT_TIME_REVERSAL, 1 - trev) == 0
        st, got2 = _set(lib, h, GROUPS[group]())
        assert st == 0 and got2[0] == counts[0]
        st, none = _set(lib, h, [])
        nk = int(np.prod(kmesh))
        assert st == 0 and none[0] == sum(1 for q in range(nk) if systems.k_neg(kmesh)[q] >= q)
    finally:
        lib.LIB.green_plan_destroy(h)


def test_rejects_operations_that_do_not_map_the_mesh(lib):
    h = _plan(lib, (2, 1, 1), 3, 4, 8)
    try:
        swap = np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1]])
        assert _set(lib, h, [swap])[0] == -1  # axes of different lengths
        assert _set(lib, h, [np.zeros((3, 3))])[0] == -1
        assert lib.LIB.green_plan_set_kpoint_symmetry(h, None, 1, None) == -1
        assert lib.LIB.green_plan_set_kpoint_symmetry(h, None, 193, None) == -1
        assert _set(lib, h, [np.eye(3)])[0] == 0  # trivial group: every k contracted
    finally:
        lib.LIB.green_plan_destroy(h)
    h = _plan(lib, (3, 3, 3), 3, 4, 8)
    try:
        assert _set(lib, h, [2 * np.eye(3)]) == (0, (14, 14))  # k -> 2k = -k on a 3-mesh: orbits {k, -k}
        assert _set(lib, h, [np.diag([1, 1, 3])])[0] == -1  # not one to one
    finally:
        lib.LIB.green_plan_destroy(h)


@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "bf16x3"])
@pytest.mark.parametrize("case", [dict(kmesh=(3, 3, 3), nao=52, naux=300, ntau=136, nspin=1, group="Oh"),
                                  dict(kmesh=(3, 3, 3), nao=8, naux=24, ntau=12, nspin=2, group="C3"),
                                  dict(kmesh=(4, 4, 4), nao=78, naux=420, ntau=160, nspin=2, group="Oh")],
                         ids=["k3_Oh", "k3_C3_ns2", "k4_Oh_ns2"])
@pytest.mark.parametrize("trev", [0, 1])
def test_symmetry_launches_in_bounds(lib, case, prec, trev):
    h = _plan(lib, case["kmesh"], case["nao"], case["naux"], case["ntau"], case["nspin"], prec)
    try:
        L = lib.LIB
        assert L.green_plan_set_option(h, lib.OPT_TIME_REVERSAL, trev) == 0
        assert _set(lib, h, GROUPS[case["group"]]())[0] == 0
        V, G, P0, Pt, Sig, H0, S, Sinf, ws = [BASE + i * STEP for i in range(9)]
        assert L.green_gw_polarization(h, V, G, P0, ws, None) == 0
        assert L.green_gw_screen(h, P0, Pt, ws, None) == 0
        assert L.green_gw_selfenergy(h, V, G, Pt, Sig, ws, None) == 0
        rep = lib.Report()
        mu = ctypes.c_double(0.0)
        assert L.green_gw_iterate(h, V, H0, S, G, Sinf, Sig, ctypes.byref(mu), 3.0, 1.0, ctypes.byref(rep), ws,
                                  None) == 0
        if case["nao"] <= 8:
            assert L.green_plan_set_option(h, lib.OPT_GF2, 1) == 0
            assert L.green_gf2_selfenergy(h, V, G, Sig, ws, None) == 0
        else:
            assert L.green_plan_set_option(h, lib.OPT_V_HALF, 1) == 0
            assert L.green_gw_iterate(h, V, H0, S, G, Sinf, Sig, ctypes.byref(mu), 3.0, 1.0, ctypes.byref(rep), ws,
                                      None) == 0
    finally:
        lib.LIB.green_plan_destroy(h)


@pytest.mark.parametrize("group,seed", [("Oh", 5), ("C3", 6)])
def test_device_generator_matches_host(group, seed):
    """synth.device.make_symmetric_V (the bench's generator, run here with torch on the CPU) builds the same V as
    the host generator: the same draws averaged over the same group, to rounding."""
    torch = pytest.importorskip("torch")
    from synth import device
    sp = configs.tiny(kmesh=(3, 3, 3), nao=3, naux=4, ntau=8, beta=8.0, seed=seed, v_scale=0.3)
    h = sym.make_symmetric_system(sp, GROUPS[group]())
    d = device.make_symmetric_V(sp, GROUPS[group](), device="cpu").numpy()
    assert _rel(d, h.V) <= 1e-13
    assert torch is not None
