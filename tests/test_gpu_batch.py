"""Autotuner, HIP-graph replay and the batched iteration, each against the plain per-system iteration
on the same inputs."""
import numpy as np
import pytest

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


def plan(s, prec):
    from paper_2406_18479_amd.gw import Plan
    sp = s.spec
    return Plan(sp.kmesh, sp.nao, sp.naux, s.grid, nspin=sp.nspin, prec=prec)


def state(s, p):
    return dict(V=dev(s.V), H0=dev(s.H0), S=dev(s.S), G=dev(s.G0),
                Sinf=torch.zeros(p.shape_H, dtype=torch.complex128, device="cuda:0"),
                Sigma=torch.zeros(p.shape_G, dtype=torch.complex128, device="cuda:0"), mu=0.0, n_target=s.n_target)


def iterate(p, y, alpha=1.0):
    mu, rep = p.iterate(y["V"], y["H0"], y["S"], y["G"], y["Sinf"], y["Sigma"], y["mu"], y["n_target"], alpha)
    y["mu"] = mu
    return rep


# uneven sizes: molecule-like, small periodic meshes, odd orbital counts, two spins
BATCH = [dict(kmesh=(1, 1, 1), nao=8, naux=32, ntau=20, beta=50.0, seed=401),
         dict(kmesh=(2, 1, 1), nao=10, naux=60, ntau=16, beta=20.0, seed=402),
         dict(kmesh=(2, 2, 1), nao=13, naux=45, ntau=12, beta=10.0, seed=403, nspin=2),
         dict(kmesh=(1, 1, 1), nao=26, naux=150, ntau=20, beta=50.0, seed=404),
         dict(kmesh=(2, 2, 2), nao=6, naux=36, ntau=16, beta=30.0, seed=405)]


def _systems():
    return [systems.make_system(configs.tiny(**c)) for c in BATCH]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_batched_iteration_equals_per_system_iteration(prec):
    """Grouped persistent launches run the very same tiles in the same order: results are identical."""
    _require_gpu()
    from paper_2406_18479_amd.gw import iterate_batched
    sys_ = _systems()
    pa = [plan(s, prec) for s in sys_]
    pb = [plan(s, prec) for s in sys_]
    ya = [state(s, p) for s, p in zip(sys_, pa)]
    yb = [state(s, p) for s, p in zip(sys_, pb)]
    for it in range(2):
        print(f"[gpu-case] batched iteration {it} {prec} ({len(sys_)} systems)", flush=True)
        ra = [iterate(p, y) for p, y in zip(pa, ya)]
        mus, rb = iterate_batched(pb, yb)
        for i, (y1, y2) in enumerate(zip(ya, yb)):
            y2["mu"] = mus[i]
            for key in ("G", "Sigma", "Sinf"):
                a, b = host(y1[key]), host(y2[key])
                assert np.array_equal(a, b), (it, i, key, float(np.max(np.abs(a - b))))
            assert y1["mu"] == y2["mu"]
            assert ra[i]["e_tot"] == rb[i]["e_tot"]
            assert rb[i]["ms"][7] > 0.0


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_graph_replay_equals_eager(prec):
    """Every replay of the captured Sigma evaluation reproduces the eager iteration exactly, with eager
    work and synchronisations between the replays."""
    _require_gpu()
    s = systems.make_system(configs.tiny(kmesh=(2, 1, 1), nao=10, naux=60, ntau=16, beta=20.0, seed=411))
    pa, pb = plan(s, prec), plan(s, prec)
    pb.set_option("graph", 1)
    ya, yb = state(s, pa), state(s, pb)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for it in range(4):
            print(f"[gpu-case] graph replay {it} {prec}", flush=True)
            ra = iterate(pa, ya)
            rb = iterate(pb, yb)
            junk = torch.randn(1000, device="cuda:0").sum().item()  # eager work between replays
            assert np.isfinite(junk)
            for key in ("G", "Sigma", "Sinf"):
                assert np.array_equal(host(ya[key]), host(yb[key])), (it, key)
            assert ra["e_tot"] == rb["e_tot"] and ya["mu"] == yb["mu"]
        # new arguments: the graph is captured again
        yc = state(s, pb)
        yd = state(s, pa)
        rc = iterate(pb, yc)
        rd = iterate(pa, yd)
        assert np.array_equal(host(yc["Sigma"]), host(yd["Sigma"])) and rc["e_tot"] == rd["e_tot"]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_autotuner_settles_and_keeps_results(prec):
    """Tuning tries every candidate of every shape once, keeps the fastest, and every candidate computes
    the same contraction: each tuning iteration (a mix of trial kernels: tile shapes, split-K counts,
    tile-row bands) and the tuned plan give the default plan's iteration up to summation order."""
    import re
    _require_gpu()
    s = systems.make_system(configs.tiny(kmesh=(2, 2, 1), nao=26, naux=120, ntau=20, beta=30.0, seed=421))
    p0, p1 = plan(s, prec), plan(s, prec)
    tol = 1e-12 if prec == "fp64" else 1e-6
    ya = state(s, p0)
    ra = iterate(p0, ya)
    Sa = host(ya["Sigma"])

    def same(y, r):
        assert np.max(np.abs(host(y["Sigma"]) - Sa)) <= tol * np.max(np.abs(Sa))
        assert abs(r["e_tot"] - ra["e_tot"]) <= (1e-11 if prec == "fp64" else 1e-7)

    p1.set_option("tune", 1)
    for it in range(40):
        y = state(s, p1)
        same(y, iterate(p1, y))
        rep = p1.tuning_report()
        if rep and "tuning" not in rep:
            break
    print("[gpu-case] tuned after", it + 1, "iterations\n" + rep, flush=True)
    assert rep and "tuning" not in rep
    assert "band=" in rep
    if prec == "bf16x3":  # the large-tile candidates include tile-row bands
        assert re.search(r" \d+/\d+/\d+/4=", rep)
    for line in rep.strip().splitlines():
        m = re.search(r"band=\d+ ([0-9.]+) us \(default ([0-9.]+) us\)", line)
        if m:
            assert float(m.group(1)) <= float(m.group(2))
    yb = state(s, p1)
    same(yb, iterate(p1, yb))


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_batch_handle_graph_replay_equals_per_system(prec):
    """A recorded batch replayed from a HIP graph over several iterations equals per-system iterations."""
    _require_gpu()
    from paper_2406_18479_amd.gw import Batch
    sys_ = _systems()
    pa = [plan(s, prec) for s in sys_]
    pb = [plan(s, prec) for s in sys_]
    ya = [state(s, p) for s, p in zip(sys_, pa)]
    yb = [state(s, p) for s, p in zip(sys_, pb)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch = Batch(pb, yb, use_graph=True)
        for it in range(3):
            print(f"[gpu-case] batch graph replay {it} {prec}", flush=True)
            ra = [iterate(p, y) for p, y in zip(pa, ya)]
            rb = batch.iterate()
            junk = torch.randn(1000, device="cuda:0").sum().item()
            assert np.isfinite(junk)
            for i, (y1, y2) in enumerate(zip(ya, yb)):
                for key in ("G", "Sigma", "Sinf"):
                    assert np.array_equal(host(y1[key]), host(y2[key])), (it, i, key)
                assert y1["mu"] == y2["mu"] and ra[i]["e_tot"] == rb[i]["e_tot"]
        batch.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_batched_iteration_with_options(prec):
    """A batch mixing a time-reversal plan (on time-reversal-symmetric inputs), a GF2 plan and a plain plan
    equals the per-system iterations bit for bit."""
    _require_gpu()
    from paper_2406_18479_amd.gw import iterate_batched
    specs = [configs.tiny(kmesh=(3, 1, 1), nao=8, naux=24, ntau=12, beta=10.0, seed=411, v_time_reversal=True),
             configs.tiny(kmesh=(2, 1, 1), nao=6, naux=18, ntau=12, beta=10.0, seed=412),
             configs.tiny(kmesh=(1, 1, 1), nao=10, naux=40, ntau=16, beta=20.0, seed=413)]
    sys_ = [systems.make_system(sp) for sp in specs]

    def plans():
        ps = [plan(s, prec) for s in sys_]
        ps[0].set_option("time_reversal", 1)
        ps[1].set_option("gf2", 1)
        return ps
    pa, pb = plans(), plans()
    ya = [state(s, p) for s, p in zip(sys_, pa)]
    yb = [state(s, p) for s, p in zip(sys_, pb)]
    for it in range(2):
        print(f"[gpu-case] batched iteration with options {it} {prec}", flush=True)
        ra = [iterate(p, y) for p, y in zip(pa, ya)]
        mus, rb = iterate_batched(pb, yb)
        for i, (y1, y2) in enumerate(zip(ya, yb)):
            y2["mu"] = mus[i]
            for key in ("G", "Sigma", "Sinf"):
                assert np.array_equal(host(y1[key]), host(y2[key])), (it, i, key)
            assert ra[i]["e_tot"] == rb[i]["e_tot"]
