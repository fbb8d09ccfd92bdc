"""Every contraction the library would launch stays inside its buffers (CPU, no device access).

With GREEN_DRYRUN=1 the library validates each batched-GEMM descriptor against
the extents of the buffers its operands point into and skips every launch.
The pointers below are fake, widely spaced addresses that are never
dereferenced, so production shapes (up to the 4x4x4, nao=78, naux=420 case)
are checked without allocating their memory.
"""
import ctypes
import os

import numpy as np
import pytest

from synth import grid as gridmod

CASES = [
    dict(kmesh=(1, 1, 1), nao=8, naux=32, ntau=20, beta=50.0, nspin=1, chunk=0),
    dict(kmesh=(2, 2, 2), nao=26, naux=180, ntau=104, beta=100.0, nspin=1, chunk=0),
    dict(kmesh=(2, 2, 2), nao=26, naux=180, ntau=104, beta=100.0, nspin=1, chunk=50_000_000),
    dict(kmesh=(3, 3, 3), nao=52, naux=300, ntau=136, beta=100.0, nspin=1, chunk=0),
    dict(kmesh=(4, 4, 4), nao=78, naux=420, ntau=160, beta=200.0, nspin=2, chunk=0),
    dict(kmesh=(3, 1, 1), nao=3, naux=70, ntau=8, beta=6.0, nspin=2, chunk=1),
    dict(kmesh=(2, 1, 1), nao=17, naux=33, ntau=12, beta=6.0, nspin=1, chunk=1),
]

BASE = 1 << 44
STEP = 1 << 40  # 1 TiB apart: no two fake buffers overlap


@pytest.fixture
def lib(monkeypatch):
    monkeypatch.setenv("GREEN_DRYRUN", "1")
    from paper_2406_18479_amd import _lib
    return _lib


def _plan(lib, c, prec=0):
    g = gridmod.make_grid(c["ntau"], c["beta"])
    d = lib.Dims((ctypes.c_int32 * 3)(*c["kmesh"]), c["nao"], c["naux"], c["ntau"], len(g.nf), len(g.nb),
                 c["nspin"], c["beta"])
    keep = [np.ascontiguousarray(a) for a in (g.tau, g.wf, g.wb)]
    keep += [np.ascontiguousarray(a, dtype=np.complex128) for a in (g.TF_t2w, g.TF_w2t, g.TB_t2w, g.TB_w2t)]
    gc = lib.GridC(*[a.ctypes.data for a in keep])
    h = ctypes.c_void_p()
    st = lib.LIB.green_plan_create(ctypes.byref(d), ctypes.byref(gc), prec, c["chunk"], ctypes.byref(h))
    assert st == 0, st
    return h


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("c", CASES, ids=lambda c: f"k{c['kmesh']}_nao{c['nao']}_naux{c['naux']}_ns{c['nspin']}_ch{c['chunk']}")
def test_all_launches_in_bounds(lib, c, prec):
    assert os.environ.get("GREEN_DRYRUN") == "1"
    h = _plan(lib, c, prec)
    try:
        ws_bytes = lib.LIB.green_workspace_bytes(h)
        assert ws_bytes > 0
        ptr = [BASE + i * STEP for i in range(10)]
        V, G, P0, Pt, Sig, H0, S, Sinf, G2, ws = ptr
        L = lib.LIB
        assert L.green_gw_polarization(h, V, G, P0, ws, None) == 0
        assert L.green_gw_screen(h, P0, Pt, ws, None) == 0
        assert L.green_gw_selfenergy(h, V, G, Pt, Sig, ws, None) == 0
        assert L.green_hf_static(h, V, G, Sinf, ws, None) == 0
        mu = ctypes.c_double(0.0)
        n = ctypes.c_double(0.0)
        ev = ctypes.c_int32(0)
        assert L.green_dyson(h, H0, S, Sinf, Sig, 3.0, ctypes.byref(mu), G2, ctypes.byref(n), ctypes.byref(ev), ws,
                             None) == 0
        rep = lib.Report()
        mu = ctypes.c_double(0.0)
        assert L.green_gw_iterate(h, V, H0, S, G, Sinf, Sig, ctypes.byref(mu), 3.0, 1.0, ctypes.byref(rep), ws,
                                  None) == 0
    finally:
        lib.LIB.green_plan_destroy(h)


@pytest.mark.parametrize("tiles", [(7, 7), (8, 8), (9, 9), (10, 10), (11, 11), (12, 12), (13, 13)])
@pytest.mark.parametrize("c", [CASES[1], CASES[3], CASES[4], CASES[6]],
                         ids=["k2x2x2", "k3x3x3", "k4x4x4", "nao17_ch1"])
def test_read_ahead_tiles_in_bounds(lib, c, tiles):
    """The split-BF16 contractions with the read-ahead LDS-DMA tiles forced (P~0 sum and Sigma~ stage 1) stay in
    their buffers on the production shapes (or fall back where the operands do not allow those tiles)."""
    h = _plan(lib, c, 2)
    try:
        L = lib.LIB
        assert L.green_plan_set_option(h, lib.OPT_P0_TILE, tiles[0]) == 0
        assert L.green_plan_set_option(h, lib.OPT_SIGMA_TILE, tiles[1]) == 0
        V, G, P0, Pt, Sig, ws = [BASE + i * STEP for i in range(6)]
        assert L.green_gw_polarization(h, V, G, P0, ws, None) == 0
        assert L.green_gw_selfenergy(h, V, G, Pt, Sig, ws, None) == 0
    finally:
        lib.LIB.green_plan_destroy(h)


@pytest.mark.parametrize("opts", ["plain", "options"])
@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "bf16x3"])
def test_batched_iteration_in_bounds(lib, prec, opts):
    """The batched iteration records every system's contractions with the same validation and
    groups them; with fake addresses nothing is launched.  "options": one system with time reversal, one
    with the GF2 self-energy."""
    cases = [CASES[0], CASES[1], CASES[5], CASES[6]]
    hs = [_plan(lib, c, prec) for c in cases]
    if opts == "options":
        assert lib.LIB.green_plan_set_option(hs[1], lib.OPT_TIME_REVERSAL, 1) == 0
        assert lib.LIB.green_plan_set_option(hs[2], lib.OPT_GF2, 1) == 0
    try:
        n = len(hs)
        handles = (ctypes.c_void_p * n)(*[h.value for h in hs])
        need = lib.LIB.green_batch_workspace_bytes(n, handles)
        assert need > 0
        systems = (lib.System * n)()
        for i in range(n):
            b = BASE + i * 16 * STEP
            systems[i] = lib.System(b, b + STEP, b + 2 * STEP, b + 3 * STEP, b + 4 * STEP, b + 5 * STEP, 0.0, 3.0,
                                    b + 6 * STEP)
        reps = (lib.Report * n)()
        bws = BASE + 100 * STEP
        L = lib.LIB
        assert L.green_gw_iterate_batched(n, handles, systems, 1.0, reps, bws, need, None) == 0
        assert L.green_gw_iterate_batched(n, handles, systems, 1.0, reps, bws, need - 1, None) == -2  # ENOMEM
        same_ws = (lib.System * 2)(systems[0], systems[0])
        two = (ctypes.c_void_p * 2)(hs[0].value, hs[1].value)
        assert L.green_gw_iterate_batched(2, two, same_ws, 1.0, reps, bws, need, None) == -1  # shared workspace
        assert L.green_gw_iterate_batched(n, handles, systems, 2.5, reps, bws, need, None) == -1  # alpha
    finally:
        for h in hs:
            lib.LIB.green_plan_destroy(h)


def test_plan_options_and_tuning_report(lib):
    h = _plan(lib, CASES[0], 0)
    try:
        L = lib.LIB
        assert L.green_plan_set_option(h, lib.OPT_TUNE, 1) == 0
        assert L.green_plan_set_option(h, lib.OPT_TUNE, 3) == -1
        assert L.green_plan_set_option(h, lib.OPT_GRAPH, 1) == 0
        assert L.green_plan_set_option(h, lib.OPT_GRAPH, 2) == -1
        for v in range(1, 14):
            assert L.green_plan_set_option(h, lib.OPT_P0_TILE, v) == 0
            assert L.green_plan_set_option(h, lib.OPT_SIGMA_TILE, v) == 0
        assert L.green_plan_set_option(h, lib.OPT_P0_TILE, 0) == -1
        assert L.green_plan_set_option(h, lib.OPT_P0_TILE, 14) == -1
        assert L.green_plan_set_option(h, lib.OPT_SIGMA_TILE, 0) == -1
        assert L.green_plan_set_option(h, lib.OPT_SIGMA_TILE, 14) == -1
        for v in (0, 1, 2, 3):
            assert L.green_plan_set_option(h, lib.OPT_STAGE1_TILE, v) == 0
        assert L.green_plan_set_option(h, lib.OPT_STAGE1_TILE, 4) == -1
        assert L.green_plan_set_option(h, lib.OPT_SIGMA_FUSED, 0) == 0
        assert L.green_plan_set_option(h, lib.OPT_SIGMA_FUSED, 2) == -1
        assert L.green_plan_set_option(h, 99, 0) == -1
        buf = ctypes.create_string_buffer(4096)
        assert L.green_plan_tuning_report(h, buf, len(buf)) == 0
        assert buf.value == b""  # nothing tuned without device runs
    finally:
        lib.LIB.green_plan_destroy(h)


def test_diis_iteration_in_bounds_and_argument_checks(lib):
    h = _plan(lib, CASES[1], 0)
    try:
        L = lib.LIB
        need = L.green_diis_history_bytes(h, 5)
        assert need > 0 and L.green_diis_history_bytes(h, 1) == 0 and L.green_diis_history_bytes(h, 17) == 0
        ptr = [BASE + i * STEP for i in range(10)]
        V, G, H0, S, Sinf, Sig, ws, hist = ptr[:8]
        st = lib.Diis()
        st.size, st.start = 5, 1
        rep = lib.Report()
        mu = ctypes.c_double(0.0)
        for it in range(7):
            assert L.green_gw_iterate_diis(h, V, H0, S, G, Sinf, Sig, ctypes.byref(mu), 3.0, 1.0, ctypes.byref(st),
                                           hist, need, ctypes.byref(rep), ws, None) == 0
            assert st.count == min(it + 1, 5) and st.iter == it + 1 and st.next == (it + 1) % 5
        assert L.green_gw_iterate_diis(h, V, H0, S, G, Sinf, Sig, ctypes.byref(mu), 3.0, 1.0, ctypes.byref(st),
                                       hist, need - 1, ctypes.byref(rep), ws, None) == -2  # short history
        bad = lib.Diis()
        bad.size = 1
        assert L.green_gw_iterate_diis(h, V, H0, S, G, Sinf, Sig, ctypes.byref(mu), 3.0, 1.0, ctypes.byref(bad),
                                       hist, need, ctypes.byref(rep), ws, None) == -1
    finally:
        lib.LIB.green_plan_destroy(h)


def test_kpath_interpolation_in_bounds_and_argument_checks(lib):
    """k-path interpolation: both contractions validated against their buffers; bad arguments rejected."""
    L = lib.LIB
    for c in (CASES[1], CASES[4]):
        h = _plan(lib, c, 0)
        try:
            Sinf, Sig, Sp, Sgp, ws = [BASE + i * STEP for i in range(5)]
            npath = 40
            k = (ctypes.c_double * (3 * npath))(*[0.01 * i for i in range(3 * npath)])
            assert L.green_kpath_interpolate(h, k, npath, Sinf, Sig, Sp, Sgp, ws, None) == 0
            assert L.green_kpath_interpolate(h, k, 0, Sinf, Sig, Sp, Sgp, ws, None) == -1
            assert L.green_kpath_interpolate(h, k, npath, None, Sig, Sp, Sgp, ws, None) == -1
            k[5] = float("nan")
            assert L.green_kpath_interpolate(h, k, npath, Sinf, Sig, Sp, Sgp, ws, None) == -1
        finally:
            L.green_plan_destroy(h)


@pytest.mark.parametrize("trev", [0, 1], ids=["all_k", "time_reversal"])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("ci", [0, 1, 2, 5, 6])
def test_gf2_in_bounds_and_argument_checks(lib, ci, prec, trev):
    """GF2 (Eq. sigma2): the option grows the workspace; every contraction of the exchange term, in whole-k
    and in partial-k chunks (chunk=1: one momentum triple per chunk), stays inside its buffers, standalone
    and inside the iteration; the entry point is refused without the option."""
    c = CASES[ci]
    L = lib.LIB
    h = _plan(lib, c, prec)
    try:
        V, G, Sig, H0, S, Sinf, ws = [BASE + i * STEP for i in range(7)]
        assert L.green_gf2_selfenergy(h, V, G, Sig, ws, None) == -1
        assert L.green_plan_set_option(h, lib.OPT_TIME_REVERSAL, trev) == 0
        ws0 = L.green_workspace_bytes(h)
        assert L.green_plan_set_option(h, lib.OPT_GF2, 2) == -1
        assert L.green_plan_set_option(h, lib.OPT_GF2, 1) == 0
        nk = int(np.prod(c["kmesh"]))
        nG2 = c["nao"] ** 4
        grow = L.green_workspace_bytes(h) - ws0
        assert grow >= 2 * nk * nk * c["naux"] * c["nao"] ** 2 * 16 + 2 * nG2 * 16
        assert L.green_gf2_selfenergy(h, V, G, Sig, ws, None) == 0
        assert L.green_gf2_selfenergy(h, None, G, Sig, ws, None) == -1
        rep = lib.Report()
        mu = ctypes.c_double(0.0)
        assert L.green_gw_iterate(h, V, H0, S, G, Sinf, Sig, ctypes.byref(mu), 3.0, 1.0, ctypes.byref(rep), ws,
                                  None) == 0
        # back to GW: the workspace keeps its size, the GF2 entry point is refused again
        assert L.green_plan_set_option(h, lib.OPT_GF2, 0) == 0
        assert L.green_workspace_bytes(h) == ws0 + grow
        assert L.green_gf2_selfenergy(h, V, G, Sig, ws, None) == -1
    finally:
        L.green_plan_destroy(h)


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("ci", [0, 1, 3, 4, 5, 6])
def test_time_reversal_in_bounds(lib, ci, prec):
    """Time reversal (only k with -k >= k contracted, partners conjugated): every contraction of the
    self-energy stays inside its buffers, standalone and inside the iteration, up to the 4x4x4 shape."""
    c = CASES[ci]
    L = lib.LIB
    h = _plan(lib, c, prec)
    try:
        V, G, Pt, Sig, H0, S, Sinf, ws = [BASE + i * STEP for i in range(8)]
        assert L.green_plan_set_option(h, lib.OPT_TIME_REVERSAL, 2) == -1
        assert L.green_plan_set_option(h, lib.OPT_TIME_REVERSAL, 1) == 0
        assert L.green_gw_selfenergy(h, V, G, Pt, Sig, ws, None) == 0
        rep = lib.Report()
        mu = ctypes.c_double(0.0)
        assert L.green_gw_iterate(h, V, H0, S, G, Sinf, Sig, ctypes.byref(mu), 3.0, 1.0, ctypes.byref(rep), ws,
                                  None) == 0
    finally:
        L.green_plan_destroy(h)


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("ci", [0, 1, 3, 4, 5, 6])
def test_v_half_store_in_bounds(lib, ci, prec):
    """Hermitian half store of V: with only the canonical-q slabs passed, every contraction of every entry point
    stays inside the smaller V (partner slabs come from the workspace), with and without time reversal; GF2 is
    refused with it."""
    c = CASES[ci]
    L = lib.LIB
    h = _plan(lib, c, prec)
    try:
        V, G, P0, Pt, Sig, H0, S, Sinf, G2, ws = [BASE + i * STEP for i in range(10)]
        ws0 = L.green_workspace_bytes(h)
        assert L.green_plan_set_option(h, lib.OPT_V_HALF, 1) == 0
        assert L.green_workspace_bytes(h) > ws0
        assert L.green_plan_set_option(h, lib.OPT_GF2, 1) == -1
        for trev in (0, 1):
            assert L.green_plan_set_option(h, lib.OPT_TIME_REVERSAL, trev) == 0
            assert L.green_gw_polarization(h, V, G, P0, ws, None) == 0
            assert L.green_gw_selfenergy(h, V, G, Pt, Sig, ws, None) == 0
            assert L.green_hf_static(h, V, G, Sinf, ws, None) == 0
            rep = lib.Report()
            mu = ctypes.c_double(0.0)
            assert L.green_gw_iterate(h, V, H0, S, G, Sinf, Sig, ctypes.byref(mu), 3.0, 1.0, ctypes.byref(rep), ws,
                                      None) == 0
    finally:
        L.green_plan_destroy(h)


@pytest.mark.parametrize("c,fits", [(CASES[0], True), (CASES[1], True), (CASES[3], False), (CASES[4], False),
                                    (CASES[5], True)],
                         ids=["molecule", "k2x2x2", "k3x3x3", "k4x4x4", "k3x1x1_ns2"])
def test_dyson_noalloc_bounds_and_limit(lib, c, fits):
    """The allocation-free Dyson step stays inside its static scratch, and plans whose Dyson buffers exceed
    GREEN_NOALLOC_MAX_BYTES are refused with GREEN_ENOMEM before any launch."""
    h = _plan(lib, c, 0)
    try:
        H0, S, Sinf, Sig, G = [BASE + i * STEP for i in range(5)]
        mu = ctypes.c_double(0.0)
        n = ctypes.c_double(0.0)
        ev = ctypes.c_int32(0)
        st = lib.LIB.green_dyson_noalloc(h, H0, S, Sinf, Sig, 3.0, ctypes.byref(mu), G, ctypes.byref(n),
                                         ctypes.byref(ev), None)
        nw, nk, nG = c["ntau"], int(np.prod(c["kmesh"])), c["nao"] ** 2
        need = 2 * c["nspin"] * nw * nk * nG * 16
        assert (need <= lib.NOALLOC_MAX_BYTES) == fits
        assert st == (0 if fits else -2)
        assert lib.LIB.green_dyson_noalloc(h, None, S, Sinf, Sig, 3.0, ctypes.byref(mu), G, None, None, None) == -1
    finally:
        lib.LIB.green_plan_destroy(h)
