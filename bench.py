#!/usr/bin/env python
"""Benchmark: fully self-consistent GW iterations on one MI355X.

One step = one green_gw_iterate call (Sec. 2.3 loop: Hartree-Fock term, P~0,
bosonic transforms + screening, Sigma~, mixing, chemical potential, Dyson and
the energy) on a seeded synthetic system whose inputs are resident in HBM
before the timed region starts.

Metric: GW Sigma-eval TFLOP/s (algorithmic flops of the P~0 and Sigma~
contractions, 4M complex counting, divided by the time of the
polarization + screening + self-energy stages measured with HIP events inside
the library) and seconds per iteration (wall clock of the whole step).

Prints one JSON line (rank 0).  Only one GPU is supported: --gpus > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GW Sigma-eval TFLOP/s + s/iteration, mixed vs FP64 on 1 GPU at <=1e-6 Eh"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}  # MI355X dense matrix-core peaks per dtype


def contraction_flops(nk, nao, naux, ntau, nspin) -> float:
    """Algorithmic real flops of P~0 and Sigma~ per iteration: 2 contractions x
    ns nk^2 ntau (naux^2 nao^2 + 2 naux nao^3) complex MACs x 8 (4M)."""
    cmac = nspin * nk * nk * ntau * (naux * naux * nao * nao + 2 * naux * nao ** 3)
    return 2.0 * 8.0 * cmac


def executed_fraction(spec) -> float:
    """Share of the algorithmic contraction flops the library executes: P~0 is contracted for one orbit of each
    pair {O, -O} (one q of each +-q pair without a point group), on half the tau nodes where -q is in the orbit of q
    or with time reversal, and Sigma~ for one momentum per orbit (per orbit pair with time reversal)."""
    from synth import symmetry
    from synth.systems import k_neg
    neg = k_neg(spec.kmesh)
    nk = spec.nk
    tr = time_reversal_symmetric(spec)
    orb = symmetry.orbit_labels(spec.kmesh, symmetry.operations(spec.point_group)) if spec.point_group else \
        list(range(nk))
    p0 = sig = 0.0
    for q in range(nk):
        c = min(orb[q], orb[neg[orb[q]]])
        if q == c:
            p0 += 0.5 if (orb[neg[q]] == orb[q] or tr) else 1.0
        ck = min(orb[q], orb[neg[orb[q]]]) if tr else orb[q]
        sig += 1.0 if q == ck else 0.0
    return 0.5 * (p0 + sig) / nk


def workloads():
    from synth import configs
    return {"molecule": configs.MOLECULE, "periodic2": configs.PERIODIC_2, "periodic3": configs.PERIODIC_3,
            "periodic3tr": configs.PERIODIC_3_TR, "periodic3oh": configs.PERIODIC_3_OH, "large4": configs.LARGE_4}


def time_reversal_symmetric(spec) -> bool:
    """Synthetic systems built with V^{-k1,-k2} = conj V^{k1,k2} and H0(-k) = conj H0(k) (S = I): the plan may
    contract the self-energy for half of the momenta and conjugate the rest."""
    return bool(spec.v_time_reversal and spec.f_time_reversal)


def _host_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "host"


def oracle_full_iteration(spec) -> float:
    """Wall seconds of one whole FP64 oracle iteration (Sigma^inf, P~0, screening, Sigma~, mu search, Dyson,
    energy) from the closed-form starting G, on the host cores."""
    from oracle import gw as ogw
    from synth import systems
    s = systems.make_system(spec)
    t0 = time.perf_counter()
    ogw.iterate(s, ogw.State(s.G0, None, None, 0.0))
    return time.perf_counter() - t0


def oracle_contraction_sample(spec, V_slab, G0, target_s: float):
    """The oracle's two contractions on a sample of the workload: P~0 of one momentum transfer q (all k) and
    Sigma~ of one k summed over one q, each at a set of tau nodes sized to about target_s in total; returns the
    measured seconds, the sample's algorithmic flops and the extrapolated seconds of both whole contractions.
    V_slab(q) gives V[q] on the host (nk x naux x nao x nao)."""
    import numpy as np
    from oracle import gw as ogw
    sp = spec
    nk, ntau = sp.nk, sp.ntau
    km = ogw.KMesh(sp.kmesh)
    q = 1 if nk > 1 else 0
    qn, k = km.sub(0, q), 0
    slabs = {q: V_slab(q)}
    if qn != q:
        slabs[qn] = V_slab(qn)

    class Slabs:
        shape = (nk, nk, sp.naux, sp.nao, sp.nao)

        def __getitem__(self, idx):
            return slabs[idx[0]][idx[1]]

    V = Slabs()
    Pt = None

    def run(ts):
        nonlocal Pt
        t0 = time.perf_counter()
        P = ogw.polarization(V, G0, sp.kmesh, ts=ts, qs=[q])
        Pt = np.zeros((nk,) + P.shape[1:], dtype=np.complex128)
        Pt[q] = P[0]
        # Sigma~^k for k = 0 summed over the transfer q reads V^{k,k-q} = V[-q][k] and V^{k-q,k} = V[q][k-q]
        ogw.selfenergy(V, G0, Pt, sp.kmesh, ts=ts, ks=[k], qs=[q])
        return time.perf_counter() - t0

    one = run([0])
    nt = int(max(1, min(ntau, target_s / max(one, 1e-6))))
    ts = sorted(set(np.linspace(0, ntau - 1, nt).round().astype(int).tolist()))
    dt = run(ts)
    # per (q, k, tau, spin): naux^2 nao^2 + 2 naux nao^3 complex MACs for each contraction; the sample did nk of
    # them for P~0 (one q) and one for Sigma~ (one k, one q), at len(ts) nodes
    unit = sp.nspin * (sp.naux ** 2 * sp.nao ** 2 + 2 * sp.naux * sp.nao ** 3) * 8.0
    flops = unit * len(ts) * (nk + 1)
    full_s = dt * (2.0 * nk * nk * ntau) / ((nk + 1) * len(ts))
    return dt, flops, full_s, len(ts)


def cpu_baseline(system, target_s: float, full_configs=True):
    """The FP64 oracle on the host cores: the contraction rate on a bounded sample of this workload (the reported
    value, TFLOP/s), its extrapolation to one iteration of this workload, and whole oracle iterations of the
    molecule and 2x2x2 workloads (measured)."""
    import numpy as np
    from synth import configs
    sp = system.spec
    if getattr(system, "V_dev", None) is None:
        def V_slab(q):
            return system.V[q]
    elif getattr(system, "v_half", False):
        # half store: the canonical slabs in increasing q; the others from V^{k,k+q} = (V^{k+q,k})^dagger
        from synth.systems import k_add_table, k_neg
        canon = [q for q in range(sp.nk) if k_neg(sp.kmesh)[q] >= q]
        add = k_add_table(sp.kmesh)

        def V_slab(q):
            if q in canon:
                return system.V_dev[canon.index(q)].cpu().numpy()
            qn = int(k_neg(sp.kmesh)[q])
            part = system.V_dev[canon.index(qn)].cpu().numpy()
            return np.stack([np.conj(np.swapaxes(part[int(add[k, q])], -1, -2)) for k in range(sp.nk)])
    else:
        def V_slab(q):
            return system.V_dev[q].cpu().numpy()
    dt, flops, full_s, nts = oracle_contraction_sample(sp, V_slab, system.G0, target_s)
    out = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": _host_threads(), "kind": "oracle",
           "cpu_model": _cpu_model(),
           "sample": f"P~0 of one momentum transfer (all k) and Sigma~ of one k over one transfer, FP64 NumPy oracle, "
                     f"at {nts} of {sp.ntau} tau nodes of the {sp.name} workload: {dt:.1f} s",
           "seconds": dt,
           "s_per_iteration": {sp.name: {"seconds": round(full_s, 3), "how": "extrapolated from the sample (the two "
                                         "contractions; the rest of an iteration is < 1 % of them at this size)"}}}
    if full_configs:
        for c in (configs.MOLECULE, configs.PERIODIC_2):
            out["s_per_iteration"][c.name] = {"seconds": round(oracle_full_iteration(c), 3),
                                              "how": "measured, one whole oracle iteration"}
    return out


def tune_plan(plan, step, max_iters=60):
    """Run untimed iterations with the autotuner on until every contraction shape has its kernel."""
    plan.set_option("tune", 1)
    for i in range(max_iters):
        step()
        rep = plan.tuning_report()
        if rep and "tuning" not in rep:
            break
    plan.set_option("tune", 0)
    print(f"[bench] tuned in {i + 1} iterations:\n{plan.tuning_report()}", file=sys.stderr, flush=True)
    return i + 1


def time_kpath(plan, system, H0, S, Sinf, Sig, mu, npath):
    """Sec. 2.4 post-processing after the last iteration: Sinf and Sigma~ interpolated onto npath points of
    the straight path Gamma -> (1/2, 1/2, 1/2), then Dyson on the path at the kept chemical potential (H0 on
    the path stands in as the Gamma-point H0; S = I).  Returns the two times in ms."""
    import numpy as np
    import torch
    from paper_2406_18479_amd.gw import Plan
    spec = system.spec
    t = np.linspace(0.0, 0.5, npath)
    path = np.stack([t, t, t], axis=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Sinf_p, Sig_p = plan.kpath_interpolate(path, Sinf, Sig)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pp = Plan((npath, 1, 1), spec.nao, 4, system.grid, nspin=spec.nspin, prec="fp64")
    H0p = H0[:, :1].expand(spec.nspin, npath, spec.nao, spec.nao).contiguous()
    Sp = torch.eye(spec.nao, dtype=torch.complex128, device=H0.device).expand(npath, spec.nao, spec.nao).contiguous()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pp.dyson(H0p, Sp, Sinf_p, Sig_p, mu, n_target=-1.0)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    pp.close()
    return {"points": npath, "interpolation_ms": round((t1 - t0) * 1e3, 3), "dyson_ms": round((t3 - t2) * 1e3, 3)}


def time_reversal_leg(steps, warmup, tune=True):
    """The 3x3x3 shapes on time-reversal-symmetric inputs (plans with the time-reversal option): FP64 and split
    BF16, each tuned, one accuracy iteration, `warmup` + `steps` timed; returns a summary for the JSON line."""
    import numpy as np
    import torch
    from synth import configs, systems
    from synth import device as dgen
    spec = configs.PERIODIC_3_TR
    system = systems.make_system(spec, with_V=False)
    system.V_dev = dgen.make_V(spec, device="cuda:0")
    res = {p: run_precision(system, p, steps, warmup, tune=tune) for p in ("fp64", "bf16x3")}
    ref = res["fp64"]["first"]
    out = {"workload": spec.name, "precisions": {}}
    for p, r in res.items():
        dom = max(range(2), key=lambda i: r["kern"][i]["ms"])
        k = r["kern"][dom]
        out["precisions"][p] = {
            "s_per_iteration": round(r["s_per_iteration"], 6),
            "sigma_eval_tflops": round(r["sigma_eval_tflops"], 4),
            "d_energy_eh": abs(r["first"]["e_tot"] - ref["e_tot"]),
            "max_dsigma_vs_fp64_eh": float(np.max(np.abs(r["first"]["sigma"] - ref["sigma"]))),
            "stage_ms": r["stage_ms"],
            "dominant_kernel": {"kernel": r["kernel_names"][dom], "achieved_tflops": round(k["tflops"], 4),
                                "frac": round(k["tflops"] / PEAK_TFLOPS[p], 4),
                                "avg_launch_ms": round(k["ms"] / max(k["launches"], 1), 4)}}
    out["speedup_vs_fp64"] = round(res["fp64"]["s_per_iteration"] / res["bf16x3"]["s_per_iteration"], 3)
    system.V_dev = None
    del res
    torch.cuda.empty_cache()
    return out


def gf2_flops(nk, nao, naux, ntau, nspin) -> float:
    """Algorithmic real flops of one GF2 self-energy (Eq. sigma2): the direct term (the P~0 and Sigma~
    contractions) plus the exchange term, per spin and tau node 2 nk^2 naux nao^3 (V G products) +
    2 nk^3 naux nao^4 (auxiliary sums) + nk^3 nao^5 (final sum) complex MACs, x 8 (4M)."""
    ex = nspin * ntau * (2 * nk * nk * naux * nao ** 3 + 2 * nk ** 3 * naux * nao ** 4 + nk ** 3 * nao ** 5)
    return contraction_flops(nk, nao, naux, ntau, nspin) + 8.0 * ex


def time_gf2(precs, steps, tune=True):
    """GF2 self-energy (Eq. sigma2) on the 2x2x2 workload (nao 26, naux 180, ntau 104), inputs in HBM: each
    precision tuned in one untimed call, then `steps` calls timed; the error of each precision against FP64."""
    import numpy as np
    import torch
    from paper_2406_18479_amd.gw import Plan
    from synth import configs, systems
    from synth import device as dgen
    spec = configs.PERIODIC_2
    system = systems.make_system(spec, with_V=False)
    V = dgen.make_V(spec, device="cuda:0")
    G = torch.from_numpy(np.ascontiguousarray(system.G0)).to("cuda:0")
    flops = gf2_flops(spec.nk, spec.nao, spec.naux, spec.ntau, spec.nspin)
    out = {"workload": spec.name, "flops_per_call": flops, "precisions": {}}
    ref = None
    for prec in ["fp64"] + [p for p in precs if p != "fp64"]:
        plan = Plan(spec.kmesh, spec.nao, spec.naux, system.grid, nspin=spec.nspin, prec=prec)
        plan.set_option("gf2", 1)
        Sig = torch.empty(plan.shape_G, dtype=torch.complex128, device="cuda:0")
        if tune:
            plan.set_option("tune", 1)
            plan.gf2_selfenergy(V, G, Sig)
            plan.set_option("tune", 0)
        plan.gf2_selfenergy(V, G, Sig)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.gf2_selfenergy(V, G, Sig)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        r = {"ms_per_call": round(dt * 1e3, 3), "tflops": round(flops / dt / 1e12, 3),
             "frac_of_peak": round(flops / dt / 1e12 / PEAK_TFLOPS[prec], 4)}
        if ref is None:
            ref = Sig.clone()
        else:
            r["max_dsigma_vs_fp64"] = float((Sig - ref).abs().max())
        out["precisions"][prec] = r
        print(f"[bench] GF2 {prec}: {r}", file=sys.stderr, flush=True)
        del plan, Sig
        torch.cuda.empty_cache()
    return out


def run_precision(system, prec, steps, warmup, chunk_bytes=0, tune=False, graph=False, accuracy_point=True,
                  sample_max_bytes=1 << 30, kpath_points=0):
    """Time `steps` iterations (after `warmup`) at one contraction precision; returns a summary dict."""
    import numpy as np
    import torch

    def sample(Sig):
        """Sigma~ on the host: all of it, or for large systems a fixed subset of (spin, tau, k) blocks."""
        if Sig.numel() * 16 <= sample_max_bytes:
            return Sig.cpu().numpy()
        ns, nt, nk = Sig.shape[:3]
        ts = sorted({0, nt // 3, nt // 2, nt - 1})
        ks = sorted({0, nk // 2, nk - 1})
        return Sig[:, ts][:, :, ks].cpu().numpy()

    from paper_2406_18479_amd.gw import Plan

    spec = system.spec
    plan = Plan(spec.kmesh, spec.nao, spec.naux, system.grid, nspin=spec.nspin, prec=prec, chunk_bytes=chunk_bytes)
    if time_reversal_symmetric(spec):
        plan.set_option("time_reversal", 1)
    if spec.point_group:
        from synth import symmetry
        plan.set_kpoint_symmetry(symmetry.operations(spec.point_group))
    if getattr(system, "v_half", False):
        plan.set_option("v_half", 1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")  # noqa: E731
    V = system.V_dev
    H0, S = dev(system.H0), dev(system.S)

    def fresh():
        return (dev(system.G0), torch.zeros(plan.shape_H, dtype=torch.complex128, device="cuda:0"),
                torch.zeros(plan.shape_G, dtype=torch.complex128, device="cuda:0"))

    tuned = 0
    if tune:
        Gt, St, Sgt = fresh()
        box = [0.0]

        def tstep():
            box[0], _ = plan.iterate(V, H0, S, Gt, St, Sgt, box[0], system.n_target, 1.0)
        tuned = tune_plan(plan, tstep)
        del Gt, St, Sgt
    if graph:
        plan.set_option("graph", 1)
    # accuracy reference point: one iteration from the common starting G (with warmup = 0 and no separate
    # accuracy point, the first timed step is that iteration)
    first = None
    if accuracy_point or warmup > 0:
        G, Sinf, Sig = fresh()
        _, rep0 = plan.iterate(V, H0, S, G, Sinf, Sig, 0.0, system.n_target, 1.0)
        first = {"sigma": sample(Sig), "e_tot": rep0["e_tot"], "mu": rep0["mu"]}
        del G, Sinf, Sig
    # timed run
    G, Sinf, Sig = fresh()
    mu = 0.0
    for _ in range(warmup):
        mu, _ = plan.iterate(V, H0, S, G, Sinf, Sig, mu, system.n_target, 1.0)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for i in range(steps):
        mu, rep = plan.iterate(V, H0, S, G, Sinf, Sig, mu, system.n_target, 1.0)
        reps.append(rep)
        if first is None:
            first = {"sigma": sample(Sig), "e_tot": rep["e_tot"], "mu": rep["mu"]}
        print(f"[bench] {prec} step {i}: {rep['ms'][7]:.1f} ms  E_tot={rep['e_tot']:.10f}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    report = plan.tuning_report()
    kpath = time_kpath(plan, system, H0, S, Sinf, Sig, mu, kpath_points) if kpath_points > 0 else None
    plan.close()
    del plan, H0, S, G, Sinf, Sig
    torch.cuda.empty_cache()

    flops = contraction_flops(spec.nk, spec.nao, spec.naux, spec.ntau, spec.nspin)
    # Sigma evaluation: polarization + screening + self-energy stages (with a graph: the whole replay)
    sig_eval_s = sum((r["ms"][0] if graph else r["ms"][1] + r["ms"][2] + r["ms"][3]) for r in reps) / 1e3
    kern = []
    for slot in range(2):
        ms = sum(r["kern_ms"][slot] for r in reps)
        fl = sum(r["kern_flops"][slot] for r in reps)
        n = sum(r["kern_launches"][slot] for r in reps)
        kern.append(dict(ms=ms, flops=fl, launches=n, tflops=fl / (ms / 1e3) / 1e12 if ms > 0 else 0.0))
    return {
        "prec": prec,
        "sigma_eval_tflops": flops * steps / sig_eval_s / 1e12,
        "s_per_iteration": wall / steps,
        "sigma_eval_s_per_iteration": sig_eval_s / steps,
        "stage_ms": {k: round(sum(r["ms"][i] for r in reps) / steps, 3) for i, k in
                     enumerate(["hf", "polarization", "screen", "selfenergy", "mix", "dyson_mu", "energy",
                                "total"])},
        "kern": kern,
        "last": reps[-1],
        "first": first,
        "tune_iterations": tuned,
        "kpath": kpath,
        "kernel_names": [clocked_kernel_name("P0_Contract", prec, report, spec.naux, spec.nao),
                         clocked_kernel_name("Sig_PV", prec, report, spec.naux, spec.nao)],
    }


KERNEL_NAME = {"fp64": "zgemm_f64_kernel<2,2,Site::P0_Contract>",
               "fp32": "zgemm_mx_kernel<1,2,2,Site::P0_Contract>",
               "bf16x3": "zgemm_bt_kernel<3,3,false,Site::P0_Contract>"}
# large tiles of the split-BF16 kernel by its `big` selector: (FM, FN) of a 64 FM x 32 FN tile
BIG_TILE = {1: (3, 3), 2: (3, 2), 3: (5, 2), 4: (7, 2)}
DMA_TILE = {5: (5, 2), 6: (3, 4)}  # the LDS-DMA kernel's tiles
# the LDS-DMA kernel with fragments read ahead: (FM, FN, WGM, NS, NW) template arguments by `big`, and the
# register-staged tile it falls back to when a K map is not flat or of an extent that is a multiple of 16
READ_AHEAD = {7: (5, 2, 4, 3, 8), 8: (4, 2, 2, 4, 8), 9: (4, 2, 4, 4, 8), 10: (4, 2, 2, 3, 4), 11: (4, 2, 1, 3, 4)}
READ_AHEAD_FALLBACK = {7: 3, 8: 1, 9: 2, 10: 2, 11: 2}
# the LDS-DMA kernel with 32-K stages in a two-slot ring: (FM, FN) by `big`, register-staged fallback
DEEP_K = {12: (2, 4), 13: (4, 2)}
DEEP_K_FALLBACK = {12: 1, 13: 2}


def default_big(site: str, naux: int) -> int:
    """Large tile an untuned split-BF16 plan uses: Sigma~ stage 1 runs the LDS-DMA 192 x 128 tile on the
    transposed V slab (even naux), the P~0 sum the register-staged tile that pads naux x naux least (192 x 96
    counted at 90 % of its area, 320 x 64 on the LDS-DMA kernel), as the library's plan creation picks them."""
    if site == "Sig_PV":
        return 6 if naux % 2 == 0 else 1
    best, pick = None, 1
    for b, (fm, fn) in BIG_TILE.items():
        bm, bn = 64 * fm, 32 * fn
        a = -(-naux // bm) * bm * (-(-naux // bn) * bn) * (0.9 if b == 1 else 1.0)
        if best is None or a < best:
            best, pick = a, b
    return 5 if pick == 3 else pick  # 320 x 64 on the LDS-DMA kernel


def clocked_kernel_name(site: str, prec: str, report: str, naux: int, nao: int) -> str:
    """Template name of the kernel that runs a clocked contraction (the P~0 sum over k and orbital pairs,
    or Sigma~ stage 1): the autotuner's choice for the shape with the most tau nodes per launch, else the
    default one."""
    import re
    best = None
    for line in report.splitlines():
        m = re.match(site + r"\s+M=(\d+) N=(\d+) K=(\d+) batch=(\d+) prec=\d+: shape=(\d+) big=(\d+)", line)
        if m and (best is None or int(m.group(1)) * int(m.group(4)) > best[0]):
            best = (int(m.group(1)) * int(m.group(4)), int(m.group(1)), int(m.group(2)), int(m.group(5)),
                    int(m.group(6)))
    if best is None:
        if prec != "bf16x3":
            return KERNEL_NAME[prec].replace("P0_Contract", site)
        best = (0, 64, 64, 0, default_big(site, naux))
    _, M, N, shape, big = best
    # Sigma~ stage 1 reads an N-contiguous V slab unless naux is even (then a transposed one)
    bnc = "true" if site == "Sig_PV" and naux % 2 else "false"
    quad = site == "Sig_PV" and naux % 4 == 0  # operands in groups of 4 (hi, then lo words)
    if prec == "bf16x3" and big in READ_AHEAD:
        # K maps: Sigma~ stage 1 runs over Q (flat), the P~0 sum over (k, orbital pair) blocks of nao^2
        if site == "Sig_PV" or (nao * nao) % 16 == 0:
            return "zgemm_bq_kernel<{},{},{},{},{},{},Site::{}>".format(*READ_AHEAD[big], "true" if quad else "false",
                                                                       site)
        big = READ_AHEAD_FALLBACK[big]
    if prec == "bf16x3" and big in DEEP_K:
        if site == "Sig_PV" or nao * nao >= 32:
            return "zgemm_bk_kernel<{},{},{},Site::{}>".format(*DEEP_K[big], "true" if quad else "false", site)
        big = DEEP_K_FALLBACK[big]
    if prec == "bf16x3" and big in BIG_TILE:
        fm, fn = BIG_TILE[big]
        return f"zgemm_bt_kernel<{fm},{fn},{bnc},Site::{site}>"
    if prec == "bf16x3" and big in DMA_TILE:
        fm, fn = DMA_TILE[big]
        return f"zgemm_bd_kernel<{fm},{fn},{'true' if quad else 'false'},Site::{site}>"
    wm, wn = ((shape - 1) // 2 + 1, (shape - 1) % 2 + 1) if 1 <= shape <= 4 else (1 if M <= 32 else 2,
                                                                                    1 if N <= 32 else 2)
    if prec == "fp64":
        return f"zgemm_f64_kernel<{wm},{wn},Site::{site}>"
    return f"zgemm_mx_kernel<{1 if prec == 'fp32' else 2},{wm},{wn},Site::{site}>"


def run_batch(args):
    """The batching form: 16 independent systems of uneven sizes, one batched iteration per step (grouped
    persistent launches, optionally replayed from a HIP graph), against 16 sequential FP64 solves."""
    import numpy as np
    import torch

    from paper_2406_18479_amd.gw import Batch, Plan
    from synth import configs, systems
    from synth import device as dgen

    specs = configs.batch_specs()
    syss = []
    for sp in specs:
        y = systems.make_system(sp, with_V=False)
        y.V_dev = dgen.make_V(sp, device="cuda:0")
        syss.append(y)
    torch.cuda.synchronize()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")  # noqa: E731
    chunk = 1 << 30

    def fresh(y, p):
        return dict(V=y.V_dev, H0=dev(y.H0), S=dev(y.S), G=dev(y.G0),
                    Sinf=torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0"),
                    Sigma=torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0"), mu=0.0,
                    n_target=y.n_target)

    def step1(p, st):
        st["mu"], rep = p.iterate(st["V"], st["H0"], st["S"], st["G"], st["Sinf"], st["Sigma"], st["mu"],
                                  st["n_target"], 1.0)
        return rep

    flops = sum(contraction_flops(sp.nk, sp.nao, sp.naux, sp.ntau, sp.nspin) for sp in specs)
    # 16 sequential FP64 solves (plain per-system iterations, library-default kernels)
    seq = 0.0
    for y in syss:
        sp = y.spec
        p = Plan(sp.kmesh, sp.nao, sp.naux, y.grid, nspin=sp.nspin, prec="fp64", chunk_bytes=chunk)
        st = fresh(y, p)
        for _ in range(args.warmup):
            step1(p, st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step1(p, st)
        torch.cuda.synchronize()
        seq += (time.perf_counter() - t0) / args.steps
        p.close()
        del p, st
    print(f"[bench] 16 sequential FP64 solves: {seq:.3f} s/iteration", file=sys.stderr, flush=True)
    res = {}
    precs = ["fp64"] + [q for q in args.precisions.split(",") if q and q != "fp64"]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for prec in precs:
            plans = [Plan(y.spec.kmesh, y.spec.nao, y.spec.naux, y.grid, nspin=y.spec.nspin, prec=prec,
                          chunk_bytes=chunk) for y in syss]
            if args.tune:
                for p, y in zip(plans, syss):
                    st = fresh(y, p)
                    tune_plan(p, lambda: step1(p, st))
                    del st
            # accuracy point: one batched iteration from the common starting G of every system
            states = [fresh(y, p) for y, p in zip(syss, plans)]
            b = Batch(plans, states, use_graph=args.graph)
            reps = b.iterate()
            first = [(st["Sigma"].cpu().numpy(), r["e_tot"]) for st, r in zip(states, reps)]
            b.close()
            states = [fresh(y, p) for y, p in zip(syss, plans)]
            b = Batch(plans, states, use_graph=args.graph)
            for _ in range(args.warmup):
                b.iterate()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sig_ms = 0.0
            for i in range(args.steps):
                reps = b.iterate()
                sig_ms += reps[0]["ms"][7]
                print(f"[bench] batched {prec} step {i}: Sigma-eval {reps[0]['ms'][7]:.1f} ms", file=sys.stderr,
                      flush=True)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
            b.close()
            for p in plans:
                p.close()
            del b, plans, states
            torch.cuda.empty_cache()
            res[prec] = dict(s_per_iteration=wall, sigma_eval_s=sig_ms / 1e3 / args.steps, first=first)
    ref = res["fp64"]["first"]
    for prec, r in res.items():
        dE = max(abs(a[1] - b[1]) for a, b in zip(r["first"], ref))
        dS = max(float(np.max(np.abs(a[0] - b[0]))) for a, b in zip(r["first"], ref))
        r.update(d_energy_eh=dE, max_dsigma_vs_fp64_eh=dS, meets_bar=dE <= 1e-6 and dS <= 1e-5,
                 sigma_eval_tflops=flops / r["sigma_eval_s"] / 1e12)
    head = min((q for q in precs if res[q]["meets_bar"]), key=lambda q: res[q]["s_per_iteration"])
    h = res[head]
    return {
        "metric": METRIC,
        "value": round(h["sigma_eval_tflops"], 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["s_per_iteration"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[head],
        "data": "synthetic",
        "build": build_record(),
        "config": {"workload": "batch16_uneven_ntau104", "systems": [sp.name for sp in specs], "precision": head,
                   "graph": bool(args.graph), "tuned": bool(args.tune)},
        "s_per_iteration": round(h["s_per_iteration"], 6),
        "sequential_fp64_s_per_iteration": round(seq, 6),
        "speedup_vs_sequential_fp64": round(seq / h["s_per_iteration"], 3),
        "aggregate_flops_per_iteration": flops,
        "precisions": {q: {k: (round(v, 6) if isinstance(v, float) and not k.startswith(("d_", "max_d")) else v)
                           for k, v in r.items() if k != "first"}
                       for q, r in res.items()},
        "roofline": None,
        "cpu_baseline": None,
    }
def build_record() -> dict:
    """Provenance of the HIP library this run loaded: the digest of the sources it was built from (the binding
    refuses to load a library whose digest differs from the sources beside it), its target and HIP version."""
    from paper_2406_18479_amd import _lib
    rec = dict(kv.split("=", 1) for kv in _lib.BUILD_INFO.split())
    rec["library"] = os.path.relpath(_lib.LIB_PATH, os.path.dirname(os.path.abspath(__file__)))
    rec["sources_match"] = True
    return rec


# hardware MFMA products issued per algorithmic (4M) flop
MFMA_PER_ALG = {"fp64": 1.0, "fp32": 1.0, "bf16x3": 3.0}


def measured_traffic(workload: str, precision: str, kernel: str, chunk_mib: int = 0):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary (FETCH_SIZE +
    WRITE_SIZE, copy-calibrated), when it covers this workload, precision, kernel and contraction chunk (lines
    without a chunk_mib key were measured at the default chunk, 0); else None."""
    import glob
    for f in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md")):
        for line in open(f):
            if line.startswith("traffic_bytes_per_launch:"):
                tok = line.split()
                kv = dict(t.split("=", 1) for t in tok[2:])
                if (kv.get("workload") == workload and kv.get("precision") == precision and kv.get("kernel") == kernel
                        and int(kv.get("chunk_mib", "0")) == chunk_mib):
                    return float(tok[1])
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="periodic3", choices=sorted(workloads()) + ["batch16"])
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="skip the autotuner (by default every plan is tuned in untimed iterations first)")
    ap.add_argument("--save-sample", default="",
                    help="write the first-iteration energy and Sigma~ sample of each precision to this .npz")
    ap.add_argument("--reference-sample", default="",
                    help="FP64 first-iteration sample (.npz from --save-sample) to measure the errors against, "
                         "for workloads whose FP64 run is made in a separate process")
    ap.add_argument("--graph", action="store_true",
                    help="replay the Sigma evaluation from a HIP graph (runs on a non-default stream)")
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3",
                    help="comma list; fp64 is always run first as the accuracy reference")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the FP64 reference run (profiling runs of one precision; no accuracy fields)")
    ap.add_argument("--v-half", action="store_true",
                    help="pass V as the Hermitian half store (the canonical-q slabs only; GREEN_OPT_V_HALF)")
    ap.add_argument("--chunk-mib", type=int, default=0,
                    help="workspace bound for the contraction intermediates (0: library default)")
    ap.add_argument("--kpath", type=int, default=0,
                    help="after the timed steps, interpolate the self-energy onto this many k-path points and "
                         "solve Dyson there (Sec. 2.4 post-processing), timed separately")
    ap.add_argument("--tr", dest="tr_leg", action="store_true",
                    help="after the GW run, also run the time-reversal-symmetric 3x3x3 inputs with the time-reversal "
                         "option (FP64 and split BF16) into a `time_reversal` object (standalone: --workload periodic3tr)")
    ap.add_argument("--gf2", dest="gf2", action="store_true",
                    help="after the GW run, also time the GF2 self-energy (Eq. sigma2) on the 2x2x2 workload into a "
                         "`gf2` object (standalone: --gf2-only)")
    ap.add_argument("--gf2-only", action="store_true", help="time only the GF2 self-energy (prints its JSON)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU path is a design "
                                   "only (sharding over q, see the design notes)", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np

    from synth import systems

    if args.copy_calibration_mib > 0:
        import torch
        n = args.copy_calibration_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    import torch

    if args.gf2_only:
        print(json.dumps({"gf2": time_gf2([p for p in args.precisions.split(",") if p], max(args.steps, 1),
                                          tune=args.tune)}), flush=True)
        return
    if args.workload == "batch16":
        print(json.dumps(run_batch(args)), flush=True)
        return
    from synth import device as dgen
    spec = workloads()[args.workload]
    t0 = time.perf_counter()
    canon = [q for q in range(spec.nk) if systems.k_neg(spec.kmesh)[q] >= q]
    if spec.point_group:
        # inputs invariant under the group: H0 and G0 on the host, V averaged over the group in HBM
        from synth import symmetry
        system = symmetry.make_symmetric_system(spec, symmetry.operations(spec.point_group), with_V=False)
        system.V_dev = dgen.make_symmetric_V(spec, symmetry.operations(spec.point_group), device="cuda:0")
        if args.v_half:
            system.V_dev = system.V_dev[canon].contiguous()
    else:
        system = systems.make_system(spec, with_V=False)
        # generated in HBM (same draws as the host generator)
        system.V_dev = dgen.make_V(spec, device="cuda:0", qs=canon if args.v_half else None)
    system.v_half = bool(args.v_half)
    torch.cuda.synchronize()
    print(f"[bench] {spec.name}: V ({system.V_dev.numel() * 16 / 1e9:.1f} GB) generated on the device in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    asked = [p for p in args.precisions.split(",") if p]
    precs = asked if args.no_reference else ["fp64"] + [p for p in asked if p != "fp64"]
    side = torch.cuda.Stream() if args.graph else torch.cuda.current_stream()
    # the headline precision (the last one asked for, split BF16 by default) runs the requested steps; the
    # reference precisions before it at most 2 timed steps after at most 1 warm-up
    head_asked = asked[-1]
    with torch.cuda.stream(side):
        res = {p: run_precision(system, p, args.steps if p == head_asked else min(args.steps, 2),
                                args.warmup if p == head_asked else min(args.warmup, 1), args.chunk_mib << 20,
                                tune=args.tune, graph=args.graph, accuracy_point=not args.no_reference,
                                kpath_points=args.kpath) for p in precs}
    if args.save_sample:
        np.savez(args.save_sample, **{f"{p}_{k}": np.asarray(v) for p, r in res.items() for k, v in r["first"].items()},
                 **{f"{p}_s_per_iteration": r["s_per_iteration"] for p, r in res.items()})
    ref = res["fp64"]["first"] if "fp64" in res else None
    fp64_spi = res["fp64"]["s_per_iteration"] if "fp64" in res else None
    if ref is None and args.reference_sample:
        z = np.load(args.reference_sample)
        ref = {"sigma": z["fp64_sigma"], "e_tot": float(z["fp64_e_tot"])}
        fp64_spi = float(z["fp64_s_per_iteration"])
    for p, r in res.items():
        if ref is None:
            r["d_energy"] = r["max_dsigma_vs_fp64"] = None
            r["meets_bar"] = True
            continue
        r["d_energy"] = abs(r["first"]["e_tot"] - ref["e_tot"])
        r["max_dsigma_vs_fp64"] = float(np.max(np.abs(r["first"]["sigma"] - ref["sigma"])))
        r["meets_bar"] = r["d_energy"] <= 1e-6 and r["max_dsigma_vs_fp64"] <= 1e-5
    # headline: the fastest precision that meets the accuracy bar (fp64 always does)
    head = min((p for p in precs if res[p]["meets_bar"]), key=lambda p: res[p]["s_per_iteration"])
    h = res[head]
    # roofline of the clocked contraction that takes the most time (the P~0 sum or Sigma~ stage 1)
    dom = max(range(2), key=lambda i: h["kern"][i]["ms"])
    k = h["kern"][dom]
    peak = PEAK_TFLOPS[head]
    achieved = k["tflops"]
    out = {
        "metric": METRIC,
        "value": round(h["sigma_eval_tflops"], 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["s_per_iteration"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[head],
        "data": "synthetic",
        "build": build_record(),
        "config": {"workload": spec.name, "nk": spec.nk, "kmesh": list(spec.kmesh), "nao": spec.nao,
                   "naux": spec.naux, "ntau": spec.ntau, "nspin": spec.nspin, "beta": spec.beta,
                   "precision": head, "tuned": bool(args.tune), "graph": bool(args.graph),
                   "time_reversal": time_reversal_symmetric(spec), "point_group": spec.point_group or None,
                   "v_half_store": bool(args.v_half), "chunk_mib": args.chunk_mib or None},
        "flop_basis": "algorithmic: both contractions over every q, k and tau (4M counting)",
        "executed_tflops": round(h["sigma_eval_tflops"] * executed_fraction(spec), 4),
        "s_per_iteration": round(h["s_per_iteration"], 6),
        "fp64_s_per_iteration": round(fp64_spi, 6) if fp64_spi else None,
        "speedup_vs_fp64": round(fp64_spi / h["s_per_iteration"], 3) if fp64_spi else None,
        "precisions": {p: {"sigma_eval_tflops": round(r["sigma_eval_tflops"], 4),
                           "s_per_iteration": round(r["s_per_iteration"], 6),
                           "d_energy_eh": r["d_energy"], "max_dsigma_vs_fp64_eh": r["max_dsigma_vs_fp64"],
                           "meets_bar": r["meets_bar"], "stage_ms": r["stage_ms"],
                           "p0_contraction_tflops": round(r["kern"][0]["tflops"], 4),
                           "sigma_contraction_tflops": round(r["kern"][1]["tflops"], 4),
                           "p0_contraction_mfma_frac": round(r["kern"][0]["tflops"] * MFMA_PER_ALG[p]
                                                             / PEAK_TFLOPS[p], 4),
                           "sigma_contraction_mfma_frac": round(r["kern"][1]["tflops"] * MFMA_PER_ALG[p]
                                                                / PEAK_TFLOPS[p], 4),
                           **({"kpath": r["kpath"]} if r["kpath"] else {})}
                       for p, r in res.items()},
        "energy": {"e_tot": h["last"]["e_tot"], "e_corr": h["last"]["e_corr"], "mu": h["last"]["mu"],
                   "n_elec": h["last"]["n_elec"], "max_dsigma": h["last"]["max_dsigma"]},
        "roofline": {"bound": "mfma", "kernel": h["kernel_names"][dom], "achieved": round(achieved, 4), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "mfma_frac": round(achieved * MFMA_PER_ALG[head] / peak, 4),
                     "traffic": measured_traffic(spec.name, head, h["kernel_names"][dom], args.chunk_mib),
                     "launches": k["launches"], "avg_launch_ms": round(k["ms"] / max(k["launches"], 1), 4),
                     "flops_per_launch": k["flops"] / max(k["launches"], 1)},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(system, args.cpu_baseline_seconds,
                                           full_configs=args.workload in ("periodic3", "periodic2", "molecule"))
    if args.tr_leg or args.gf2:
        del res, h
        system.V_dev = None
        torch.cuda.empty_cache()
    if args.tr_leg and args.workload == "periodic3":
        out["time_reversal"] = time_reversal_leg(args.steps, args.warmup, tune=args.tune)
    if args.gf2:
        out["gf2"] = time_gf2(precs, max(args.steps, 1), tune=args.tune)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
