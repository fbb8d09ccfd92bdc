"""Device-resident generation of the synthetic integrals V (same draws as ``synth.systems.make_V``).

The large workloads (3x3x3: 9.5 GB of V, 4x4x4: 167 GB) are generated directly
in device memory with torch: the SplitMix64 counter stream is reproduced
bit for bit in int64 arithmetic (two's-complement multiply, logical shifts by
masking), so every block uses the same integers as the NumPy generator; the
uniform -> normal transform (Box-Muller) runs in float64 torch ops and agrees
with the NumPy values to rounding.

Nothing here evaluates the GW method.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rng
from .systems import SystemSpec, k_add_table, k_neg, k_sub_table

_MASK64 = (1 << 64) - 1


def _i64(x: int) -> int:
    x &= _MASK64
    return x - (1 << 64) if x >= (1 << 63) else x


_GOLDEN = _i64(0x9E3779B97F4A7C15)
_M1 = _i64(0xBF58476D1CE4E5B9)
_M2 = _i64(0x94D049BB133111EB)


def _srl(x: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 values."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def splitmix64(x: torch.Tensor) -> torch.Tensor:
    z = x + _GOLDEN
    z = (z ^ _srl(z, 30)) * _M1
    z = (z ^ _srl(z, 27)) * _M2
    return z ^ _srl(z, 31)


def uniforms(key: int, count: int, device) -> torch.Tensor:
    idx = torch.arange(count, dtype=torch.int64, device=device)
    u = splitmix64(idx + _i64(int(key)))
    return _srl(u, 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def complex_normals(key: int, shape, device) -> torch.Tensor:
    n = int(np.prod(shape))
    u = uniforms(key, 4 * n, device).view(2 * n, 2)
    g = torch.sqrt(-2.0 * torch.log1p(-u[:, 0])) * torch.cos(2.0 * np.pi * u[:, 1])
    g = g.view(n, 2)
    z = torch.complex(g[:, 0], g[:, 1]) * np.sqrt(0.5)
    return z.view(shape)


def _block(spec: SystemSpec, k1: int, k2: int, env: torch.Tensor, device) -> torch.Tensor:
    key = int(rng.stream_key(spec.seed, rng.TAG_V, 0, k1, k2))
    Z = complex_normals(key, (spec.naux, spec.nao, spec.nao), device)
    return Z * env[:, None, None]


def _impose_time_reversal(spec: SystemSpec, V: torch.Tensor) -> None:
    """In place, the group average of synth.systems (same terms in the same order): every block becomes
    (a + b + c + d) / 4 over {itself, the dagger of the swapped pair, the conjugate of the negated pair, the
    transpose of the negated swapped pair}, so V^{-k1,-k2}(Q) = conj V^{k1,k2}(Q) and the Hermitian pairing
    hold to rounding.  Works orbit by orbit from saved originals."""
    nk = spec.nk
    neg = k_neg(spec.kmesh)
    sub = k_sub_table(spec.kmesh)

    def at(k1, k2):
        return V[int(sub[k2, k1]), k1]  # V^{k1,k2} is stored at [q = k2 - k1][k1]

    done = set()
    for k1 in range(nk):
        for k2 in range(nk):
            if (k1, k2) in done:
                continue
            orbit = {(k1, k2), (k2, k1), (int(neg[k1]), int(neg[k2])), (int(neg[k2]), int(neg[k1]))}
            orig = {m: at(*m).clone() for m in orbit}
            for (a1, a2) in orbit:
                a = orig[(a1, a2)]
                b = orig[(a2, a1)].transpose(1, 2).conj()
                c = orig[(int(neg[a1]), int(neg[a2]))].conj()
                d = orig[(int(neg[a2]), int(neg[a1]))].transpose(1, 2)
                at(a1, a2).copy_(0.25 * (a + b + c + d))
            done |= orbit


def make_V(spec: SystemSpec, device="cuda:0", out: torch.Tensor | None = None, qs=None) -> torch.Tensor:
    """V[q][k] = V^{k,k+q}(Q) on `device`, identical in construction to synth.systems.make_V.  qs: only the slabs
    of these momentum transfers, in that order (out[i] = slab qs[i]; not with time-reversal averaging, which
    mixes slabs)."""
    nk = spec.nk
    add = k_add_table(spec.kmesh)
    qs = list(range(nk)) if qs is None else list(qs)
    if spec.v_time_reversal and qs != list(range(nk)):
        raise ValueError("time-reversal-averaged V is generated whole")
    env = (spec.amp * torch.exp(-spec.v_decay * torch.arange(spec.naux, dtype=torch.float64))).to(device)
    if out is None:
        out = torch.empty((len(qs), nk, spec.naux, spec.nao, spec.nao), dtype=torch.complex128, device=device)
    for iq, q in enumerate(qs):
        for k in range(nk):
            k2 = int(add[k, q])
            if k == k2:
                Z = _block(spec, k, k, env, device)
                out[iq, k] = 0.5 * (Z + Z.conj().transpose(1, 2))
            elif k < k2:
                out[iq, k] = _block(spec, k, k2, env, device)
            else:
                out[iq, k] = _block(spec, k2, k, env, device).conj().transpose(1, 2)
    if spec.v_time_reversal:
        _impose_time_reversal(spec, out)
    return out


def make_symmetric_V(spec: SystemSpec, ops, device="cuda:0") -> torch.Tensor:
    """V of synth.symmetry.make_symmetric_system generated on `device`: the blocks of make_V averaged over the
    whole group the operations generate (V'^{k1,k2} = mean over R of V^{R k1, R k2}) and rescaled to the norm V had
    before (equal to the host construction up to summation order)."""
    from .symmetry import group_closure
    V = make_V(spec, device=device)
    nk = spec.nk
    add = torch.as_tensor(k_add_table(spec.kmesh), device=device)  # add[k, q] = k + q
    sub = torch.as_tensor(k_sub_table(spec.kmesh), device=device)  # sub[k, q] = k - q
    ks = torch.arange(nk, device=device)
    norm0 = torch.linalg.vector_norm(V)
    acc = torch.zeros_like(V)
    for g in group_closure(spec.kmesh, ops):
        gt = torch.as_tensor(g, device=device)
        # slab [q][k] holds the pair (k, k + q); its image (g k, g(k + q)) sits at [g(k + q) - g k][g k]
        k1 = gt[ks][None, :].expand(nk, nk)                 # [q][k] -> g k
        k2 = gt[add[ks][:, :].T]                            # [q][k] -> g(k + q)
        qi = sub[k2, k1]                                     # g(k + q) - g k
        acc += V[qi, k1]
    acc *= norm0 / torch.linalg.vector_norm(acc)
    del V
    return acc


def random_polarization(seed: int, nk: int, ntau: int, naux: int, scale: float = 0.05, device="cuda:0"):
    """Device twin of synth.systems.random_polarization (same counter streams)."""
    P = torch.empty((nk, ntau, naux, naux), dtype=torch.complex128, device=device)
    for q in range(nk):
        for t in range(ntau):
            z = complex_normals(int(rng.stream_key(seed, rng.TAG_P, 0, q, t)), (naux, naux), device)
            P[q, t] = -scale * 0.5 * (z + z.conj().T) / np.sqrt(naux)
    return P
