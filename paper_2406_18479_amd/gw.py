"""Torch-facing wrappers of the GW entry points of libgreen_gw.

A :class:`Plan` owns the library plan and a workspace tensor; its methods
take device tensors (complex128, contiguous, on the plan's device) in the
layouts of include/green_gw.h and launch on the current torch stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: torch.Tensor, shape: tuple, name: str, device) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name}: expected complex128, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.device != device:
        raise ValueError(f"{name}: on {t.device}, plan is on {device}")
    return t.data_ptr()


class Plan:
    """Plan + workspace for fixed dimensions and grid (one GPU)."""

    def __init__(self, kmesh, nao, naux, grid, nspin=1, prec="fp64", chunk_bytes=0, device="cuda:0"):
        self.device = torch.device(device)
        self.kmesh = tuple(int(x) for x in kmesh)
        self.nk = int(np.prod(self.kmesh))
        self.nao, self.naux, self.nspin = int(nao), int(naux), int(nspin)
        self.ntau = int(grid.ntau)
        self.nw_f, self.nw_b = len(grid.nf), len(grid.nb)
        self.beta = float(grid.beta)
        d = _lib.Dims((ctypes.c_int32 * 3)(*self.kmesh), self.nao, self.naux, self.ntau, self.nw_f, self.nw_b,
                      self.nspin, self.beta)
        keep = [np.ascontiguousarray(a) for a in (grid.tau, grid.wf, grid.wb)]
        keep += [np.ascontiguousarray(a, dtype=np.complex128) for a in
                 (grid.TF_t2w, grid.TF_w2t, grid.TB_t2w, grid.TB_w2t)]
        g = _lib.GridC(*[a.ctypes.data for a in keep])
        h = ctypes.c_void_p()
        _lib.check(_lib.LIB.green_plan_create(ctypes.byref(d), ctypes.byref(g), _lib.PREC[prec], int(chunk_bytes),
                                              ctypes.byref(h)), "green_plan_create")
        self._h = h
        self.ws_bytes = int(_lib.LIB.green_workspace_bytes(h))
        with torch.cuda.device(self.device):
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    # shapes
    @property
    def canonical_q(self):
        """Momentum transfers q with -q >= q (flat index), in increasing order: the slabs of the half store."""
        m = self.kmesh
        out = []
        for q in range(self.nk):
            a, b, c = q // (m[1] * m[2]), (q // m[2]) % m[1], q % m[2]
            qn = (((-a) % m[0]) * m[1] + (-b) % m[1]) * m[2] + (-c) % m[2]
            if qn >= q:
                out.append(q)
        return out

    @property
    def shape_V(self):
        nq = len(self.canonical_q) if getattr(self, "v_half", False) else self.nk
        return (nq, self.nk, self.naux, self.nao, self.nao)

    @property
    def shape_G(self):
        return (self.nspin, self.ntau, self.nk, self.nao, self.nao)

    @property
    def shape_P(self):
        return (self.nk, self.ntau, self.naux, self.naux)

    @property
    def shape_H(self):
        return (self.nspin, self.nk, self.nao, self.nao)

    @property
    def shape_S(self):
        return (self.nk, self.nao, self.nao)

    def set_option(self, option: str, value: int) -> None:
        """option "tune" (0, 1, 2), "graph" (0, 1), "p0_tile" (1..13), "sigma_tile" (1..13), "stage1_tile" (0..3), "sigma_fused"
        (0, 1), "gf2" (0, 1), "time_reversal" (0, 1) or "v_half" (0, 1: V holds the canonical-q slabs only,
        shape_V follows); see green_plan_set_option.  The workspace is re-allocated when the option grows it."""
        code = {"tune": _lib.OPT_TUNE, "graph": _lib.OPT_GRAPH, "p0_tile": _lib.OPT_P0_TILE,
                "stage1_tile": _lib.OPT_STAGE1_TILE, "sigma_fused": _lib.OPT_SIGMA_FUSED,
                "gf2": _lib.OPT_GF2, "time_reversal": _lib.OPT_TIME_REVERSAL, "v_half": _lib.OPT_V_HALF,
                "sigma_tile": _lib.OPT_SIGMA_TILE}[option]
        _lib.check(_lib.LIB.green_plan_set_option(self._h, code, int(value)), "green_plan_set_option")
        if option == "v_half":
            self.v_half = bool(value)
        self._regrow()

    def _regrow(self) -> None:
        need = int(_lib.LIB.green_workspace_bytes(self._h))
        if need != self.ws_bytes:
            self.ws_bytes = need
            self.ws = None
            with torch.cuda.device(self.device):
                self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def set_kpoint_symmetry(self, rotations) -> tuple:
        """Point group acting on the k mesh (green_plan_set_kpoint_symmetry): `rotations` is a sequence of 3x3
        integer matrices acting on integer mesh coordinates (empty: none).  Returns the numbers of contracted
        momentum transfers and of contracted momenta."""
        rot = np.ascontiguousarray(np.asarray(rotations, dtype=np.int32).reshape(-1, 9))
        counts = (ctypes.c_int32 * 2)()
        ptr = rot.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if len(rot) else None
        _lib.check(_lib.LIB.green_plan_set_kpoint_symmetry(self._h, ptr, len(rot), counts),
                   "green_plan_set_kpoint_symmetry")
        self._regrow()
        return int(counts[0]), int(counts[1])

    def tuning_report(self) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        _lib.check(_lib.LIB.green_plan_tuning_report(self._h, buf, len(buf)), "green_plan_tuning_report")
        return buf.value.decode()

    def close(self):
        if getattr(self, "_h", None):
            _lib.LIB.green_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # entry points ------------------------------------------------------------------
    def polarization(self, V, G, P0=None):
        P0 = torch.empty(self.shape_P, dtype=torch.complex128, device=self.device) if P0 is None else P0
        _lib.check(_lib.LIB.green_gw_polarization(self._h, _ptr(V, self.shape_V, "V", self.device),
                                                  _ptr(G, self.shape_G, "G", self.device),
                                                  _ptr(P0, self.shape_P, "P0", self.device), self.ws.data_ptr(),
                                                  _stream(self.device)), "green_gw_polarization")
        return P0

    def screen(self, P0, Pt=None):
        Pt = torch.empty(self.shape_P, dtype=torch.complex128, device=self.device) if Pt is None else Pt
        _lib.check(_lib.LIB.green_gw_screen(self._h, _ptr(P0, self.shape_P, "P0", self.device),
                                            _ptr(Pt, self.shape_P, "Pt", self.device), self.ws.data_ptr(),
                                            _stream(self.device)), "green_gw_screen")
        return Pt

    def selfenergy(self, V, G, Pt, Sigma=None):
        Sigma = torch.empty(self.shape_G, dtype=torch.complex128, device=self.device) if Sigma is None else Sigma
        _lib.check(_lib.LIB.green_gw_selfenergy(self._h, _ptr(V, self.shape_V, "V", self.device),
                                                _ptr(G, self.shape_G, "G", self.device),
                                                _ptr(Pt, self.shape_P, "Pt", self.device),
                                                _ptr(Sigma, self.shape_G, "Sigma", self.device), self.ws.data_ptr(),
                                                _stream(self.device)), "green_gw_selfenergy")
        return Sigma

    def gf2_selfenergy(self, V, G, Sigma=None):
        """GF2 self-energy of Eq. sigma2 (direct minus exchange); needs set_option("gf2", 1)."""
        Sigma = torch.empty(self.shape_G, dtype=torch.complex128, device=self.device) if Sigma is None else Sigma
        _lib.check(_lib.LIB.green_gf2_selfenergy(self._h, _ptr(V, self.shape_V, "V", self.device),
                                                 _ptr(G, self.shape_G, "G", self.device),
                                                 _ptr(Sigma, self.shape_G, "Sigma", self.device), self.ws.data_ptr(),
                                                 _stream(self.device)), "green_gf2_selfenergy")
        return Sigma

    def hf_static(self, V, G, Sinf=None):
        Sinf = torch.empty(self.shape_H, dtype=torch.complex128, device=self.device) if Sinf is None else Sinf
        _lib.check(_lib.LIB.green_hf_static(self._h, _ptr(V, self.shape_V, "V", self.device),
                                            _ptr(G, self.shape_G, "G", self.device),
                                            _ptr(Sinf, self.shape_H, "Sinf", self.device), self.ws.data_ptr(),
                                            _stream(self.device)), "green_hf_static")
        return Sinf

    def dyson(self, H0, S, Sinf, Sigma, mu, n_target=-1.0, G=None):
        G = torch.empty(self.shape_G, dtype=torch.complex128, device=self.device) if G is None else G
        m = ctypes.c_double(mu)
        n = ctypes.c_double(0.0)
        ev = ctypes.c_int32(0)
        _lib.check(_lib.LIB.green_dyson(self._h, _ptr(H0, self.shape_H, "H0", self.device),
                                        _ptr(S, self.shape_S, "S", self.device),
                                        _ptr(Sinf, self.shape_H, "Sinf", self.device),
                                        _ptr(Sigma, self.shape_G, "Sigma", self.device), float(n_target),
                                        ctypes.byref(m), _ptr(G, self.shape_G, "G", self.device), ctypes.byref(n),
                                        ctypes.byref(ev), self.ws.data_ptr(), _stream(self.device)), "green_dyson")
        return G, m.value, n.value, ev.value

    def check_status(self):
        """Raise the error latched on the device by earlier calls (green_check_status); synchronises."""
        _lib.check(_lib.LIB.green_check_status(self._h, self.ws.data_ptr(), _stream(self.device)),
                   "green_check_status")

    def dyson_noalloc(self, H0, S, Sinf, Sigma, mu, n_target=-1.0, G=None):
        """dyson() through green_dyson_noalloc: the library works in its static device scratch (no workspace)."""
        G = torch.empty(self.shape_G, dtype=torch.complex128, device=self.device) if G is None else G
        m = ctypes.c_double(mu)
        n = ctypes.c_double(0.0)
        ev = ctypes.c_int32(0)
        _lib.check(_lib.LIB.green_dyson_noalloc(self._h, _ptr(H0, self.shape_H, "H0", self.device),
                                                _ptr(S, self.shape_S, "S", self.device),
                                                _ptr(Sinf, self.shape_H, "Sinf", self.device),
                                                _ptr(Sigma, self.shape_G, "Sigma", self.device), float(n_target),
                                                ctypes.byref(m), _ptr(G, self.shape_G, "G", self.device),
                                                ctypes.byref(n), ctypes.byref(ev), _stream(self.device)),
                   "green_dyson_noalloc")
        return G, m.value, n.value, ev.value

    def kpath_interpolate(self, kfrac, Sinf, Sigma):
        """Sinf and Sigma~(tau) interpolated from the mesh onto the points kfrac ([npath][3] fractional
        coordinates); returns (Sinf_path [nspin][npath][nao][nao], Sigma_path [nspin][ntau][npath][nao][nao]).
        The Green's function on the path: dyson() of a plan with kmesh (npath, 1, 1)."""
        import numpy as np
        kf = np.ascontiguousarray(np.asarray(kfrac, dtype=np.float64).reshape(-1, 3))
        npath = kf.shape[0]
        ns, nt, nao = self.nspin, self.ntau, self.nao
        Sinf_p = torch.empty((ns, npath, nao, nao), dtype=torch.complex128, device=self.device)
        Sig_p = torch.empty((ns, nt, npath, nao, nao), dtype=torch.complex128, device=self.device)
        _lib.check(_lib.LIB.green_kpath_interpolate(
            self._h, kf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), npath,
            _ptr(Sinf, self.shape_H, "Sinf", self.device), _ptr(Sigma, self.shape_G, "Sigma", self.device),
            Sinf_p.data_ptr(), Sig_p.data_ptr(), self.ws.data_ptr(), _stream(self.device)),
            "green_kpath_interpolate")
        return Sinf_p, Sig_p

    def iterate_diis(self, diis, V, H0, S, G, Sinf, Sigma, mu, n_target, alpha=1.0):
        """One iteration with DIIS (a DiisState of this plan); G, Sinf, Sigma updated in place."""
        m = ctypes.c_double(mu)
        rep = _lib.Report()
        _lib.check(_lib.LIB.green_gw_iterate_diis(self._h, _ptr(V, self.shape_V, "V", self.device),
                                                  _ptr(H0, self.shape_H, "H0", self.device),
                                                  _ptr(S, self.shape_S, "S", self.device),
                                                  _ptr(G, self.shape_G, "G", self.device),
                                                  _ptr(Sinf, self.shape_H, "Sinf", self.device),
                                                  _ptr(Sigma, self.shape_G, "Sigma", self.device), ctypes.byref(m),
                                                  float(n_target), float(alpha), ctypes.byref(diis.c),
                                                  diis.history.data_ptr(), diis.bytes, ctypes.byref(rep),
                                                  self.ws.data_ptr(), _stream(self.device)), "green_gw_iterate_diis")
        return m.value, rep.as_dict()

    def iterate(self, V, H0, S, G, Sinf, Sigma, mu, n_target, alpha=1.0):
        """One self-consistent iteration; G, Sinf, Sigma are updated in place.  Returns (mu, report dict)."""
        m = ctypes.c_double(mu)
        rep = _lib.Report()
        _lib.check(_lib.LIB.green_gw_iterate(self._h, _ptr(V, self.shape_V, "V", self.device),
                                             _ptr(H0, self.shape_H, "H0", self.device),
                                             _ptr(S, self.shape_S, "S", self.device),
                                             _ptr(G, self.shape_G, "G", self.device),
                                             _ptr(Sinf, self.shape_H, "Sinf", self.device),
                                             _ptr(Sigma, self.shape_G, "Sigma", self.device), ctypes.byref(m),
                                             float(n_target), float(alpha), ctypes.byref(rep), self.ws.data_ptr(),
                                             _stream(self.device)), "green_gw_iterate")
        return m.value, rep.as_dict()


class DiisState:
    """DIIS state and device history of one plan (green_gw_iterate_diis)."""

    def __init__(self, plan, size=5, start=2):
        self.c = _lib.Diis()
        self.c.size, self.c.start = int(size), int(start)
        self.bytes = int(_lib.LIB.green_diis_history_bytes(plan._h, int(size)))
        if self.bytes == 0:
            raise ValueError("DIIS size must be in [2, 16]")
        with torch.cuda.device(plan.device):
            self.history = torch.empty(self.bytes, dtype=torch.uint8, device=plan.device)

    @property
    def coefficients(self):
        return [self.c.coef[i] for i in range(self.c.count)]


def _systems_array(plans, systems):
    if len(plans) != len(systems) or not plans:
        raise ValueError("plans and systems must be non-empty lists of equal length")
    dev = plans[0].device
    n = len(plans)
    arr = (_lib.System * n)()
    for i, (p, y) in enumerate(zip(plans, systems)):
        if p.device != dev:
            raise ValueError("all plans must be on one device")
        arr[i] = _lib.System(_ptr(y["V"], p.shape_V, "V", dev), _ptr(y["H0"], p.shape_H, "H0", dev),
                             _ptr(y["S"], p.shape_S, "S", dev), _ptr(y["G"], p.shape_G, "G", dev),
                             _ptr(y["Sinf"], p.shape_H, "Sinf", dev), _ptr(y["Sigma"], p.shape_G, "Sigma", dev),
                             float(y["mu"]), float(y["n_target"]), p.ws.data_ptr())
    return dev, arr


def iterate_batched(plans, systems, alpha=1.0):
    """One iteration of several independent systems (green_gw_iterate_batched).

    plans: list of Plan (one per system, each with its own workspace), all on one device.
    systems: list of dicts with keys V, H0, S, G, Sinf, Sigma (tensors; G, Sinf, Sigma updated in place),
    mu (float) and n_target (float).  Returns (list of mu, list of report dicts).
    """
    dev, arr = _systems_array(plans, systems)
    n = len(plans)
    handles = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
    nbytes = int(_lib.LIB.green_batch_workspace_bytes(n, handles))
    with torch.cuda.device(dev):
        bws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    reps = (_lib.Report * n)()
    _lib.check(_lib.LIB.green_gw_iterate_batched(n, handles, arr, float(alpha), reps, bws.data_ptr(), nbytes,
                                                 _stream(dev)), "green_gw_iterate_batched")
    return [arr[i].mu for i in range(n)], [reps[i].as_dict() for i in range(n)]


class Batch:
    """A batched iteration recorded once for fixed systems (green_batch_create); `iterate` runs one
    iteration of every system, replayed from a HIP graph when use_graph (on a non-default stream)."""

    def __init__(self, plans, systems, alpha=1.0, use_graph=False):
        self.plans, self.systems = list(plans), list(systems)
        self.device, arr = _systems_array(self.plans, self.systems)
        n = len(self.plans)
        self._handles = (ctypes.c_void_p * n)(*[p._h.value for p in self.plans])
        nbytes = int(_lib.LIB.green_batch_workspace_bytes(n, self._handles))
        with torch.cuda.device(self.device):
            self.ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _lib.check(_lib.LIB.green_batch_create(n, self._handles, arr, float(alpha), int(bool(use_graph)),
                                               self.ws.data_ptr(), nbytes, _stream(self.device), ctypes.byref(h)),
                   "green_batch_create")
        self._h = h

    def iterate(self):
        """One iteration of all systems; updates G, Sinf, Sigma in place and each system's "mu".
        Returns the list of report dicts."""
        _, arr = _systems_array(self.plans, self.systems)
        n = len(self.plans)
        reps = (_lib.Report * n)()
        _lib.check(_lib.LIB.green_batch_iterate(self._h, arr, reps, _stream(self.device)), "green_batch_iterate")
        for i, y in enumerate(self.systems):
            y["mu"] = arr[i].mu
        return [reps[i].as_dict() for i in range(n)]

    def close(self):
        if getattr(self, "_h", None):
            _lib.LIB.green_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
