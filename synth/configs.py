"""The workload configurations (shapes, temperatures, seeds) of the synthetic inputs.

Each entry mirrors one of the problem sizes the GW hot path is measured on:
a Gamma-only molecule-like case, a 2x2x2 periodic case, a 3x3x3 precision
case, a batch of 16 uneven systems and a 4x4x4 spin-unrestricted case.  The
sizes stand in for PySCF inputs of the kind the paper's silicon example uses
(Sec. 6); the paper prints no timings for them.
"""
from __future__ import annotations

import numpy as np

from . import rng
from .systems import SystemSpec

MOLECULE = SystemSpec("molecule_nk1_nao8_naux32_ntau20", (1, 1, 1), nao=8, naux=32, ntau=20, beta=50.0,
                      seed=18479, band=1.0, v_decay=0.1, f_time_reversal=False)
PERIODIC_2 = SystemSpec("periodic_k2x2x2_nao26_naux180_ntau104", (2, 2, 2), nao=26, naux=180, ntau=104,
                        beta=100.0, seed=18480)
PERIODIC_3 = SystemSpec("periodic_k3x3x3_nao52_naux300_ntau136", (3, 3, 3), nao=52, naux=300, ntau=136,
                        beta=100.0, seed=18481)
# the same shapes with time-reversal-symmetric inputs (V^{-k1,-k2}(Q) = conj V^{k1,k2}(Q), H0(-k) = conj H0(k)),
# as in a non-magnetic crystal
PERIODIC_3_TR = SystemSpec("periodic_k3x3x3_nao52_naux300_ntau136_tr", (3, 3, 3), nao=52, naux=300, ntau=136,
                           beta=100.0, seed=18481, v_time_reversal=True)
# the 3x3x3 shapes on inputs invariant under the full cubic group (orbitals transforming trivially): the plan
# contracts 4 of the 27 momenta in each stage
PERIODIC_3_OH = SystemSpec("periodic_k3x3x3_nao52_naux300_ntau136_oh", (3, 3, 3), nao=52, naux=300, ntau=136,
                           beta=100.0, seed=18481, point_group="Oh")
LARGE_4 = SystemSpec("periodic_k4x4x4_nao78_naux420_ntau160_uhf", (4, 4, 4), nao=78, naux=420, ntau=160,
                     beta=200.0, nspin=2, seed=18483)

CONFIGS = {0: MOLECULE, 1: PERIODIC_2, 2: PERIODIC_3, 4: LARGE_4}


def batch_specs(seed: int = 18482, nsys: int = 16) -> list[SystemSpec]:
    """16 uneven systems: nao from {10,18,26,40,52,60}, naux = 6 nao, nk from {1,8,27}, beta from {50,100,200}."""
    u = rng.uniforms(rng.stream_key(seed, rng.TAG_DRAW, 0, 0, 0), 0, 3 * nsys).reshape(nsys, 3)
    naos = (10, 18, 26, 40, 52, 60)
    meshes = ((1, 1, 1), (2, 2, 2), (3, 3, 3))
    betas = (50.0, 100.0, 200.0)
    out = []
    for j in range(nsys):
        nao = naos[int(u[j, 0] * len(naos))]
        mesh = meshes[int(u[j, 1] * len(meshes))]
        beta = betas[int(u[j, 2] * len(betas))]
        out.append(SystemSpec(f"batch{j:02d}_k{'x'.join(map(str, mesh))}_nao{nao}", mesh, nao=nao, naux=6 * nao,
                              ntau=104, beta=beta, seed=1848200 + j))
    return out


def tiny(kmesh=(1, 1, 1), nao=3, naux=4, ntau=8, beta=10.0, nspin=1, seed=7, **kw) -> SystemSpec:
    """Small shapes for brute-force checks."""
    return SystemSpec(f"tiny_k{'x'.join(map(str, kmesh))}_nao{nao}_naux{naux}", tuple(kmesh), nao=nao, naux=naux,
                      ntau=ntau, beta=beta, nspin=nspin, seed=seed, **kw)


__all__ = ["CONFIGS", "MOLECULE", "PERIODIC_2", "PERIODIC_3", "PERIODIC_3_OH", "LARGE_4", "batch_specs", "tiny",
           "np"]
