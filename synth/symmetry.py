"""Point groups acting on the k mesh, and seeded inputs invariant under them.

A crystal's point-group operations map the Monkhorst-Pack mesh onto itself;
here each operation is an integer 3x3 matrix R acting on the integer mesh
coordinates of a momentum, k -> R k modulo the mesh (Sec. 3 lists symmetry
among the method's features).  The orbital and auxiliary bases are taken to
transform trivially, so an invariant system has H0(R k) = H0(k),
S(R k) = S(k) and V^{R k1, R k2}(Q) = V^{k1,k2}(Q) (and hence G^{R k} = G^k
for the non-interacting G built from them).

Nothing here evaluates the self-energy method: this module only draws inputs.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import rng
from .systems import (System, SystemSpec, _impose_v_time_reversal, _v_block, electron_count, k_add_table, k_flat,
                      k_neg, kmesh_points, noninteracting_G, random_hermitian_spectrum)
from .grid import make_grid


def cubic_group() -> list[np.ndarray]:
    """The 48 operations of the full cubic group O_h: signed permutation matrices."""
    ops = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int32)
            for i in range(3):
                R[i, perm[i]] = signs[i]
            ops.append(R)
    return ops


def threefold_group() -> list[np.ndarray]:
    """C3 about the body diagonal: cyclic permutations of the three coordinates (no inversion)."""
    c = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], dtype=np.int32)
    return [np.eye(3, dtype=np.int32), c, c @ c]


def operations(name: str) -> list[np.ndarray]:
    """The operations of a named group ("Oh", "C3"; "" gives none)."""
    return {"": lambda: [], "Oh": cubic_group, "C3": threefold_group}[name]()


def act(kmesh, R: np.ndarray) -> np.ndarray:
    """The permutation k -> R k of the flat mesh indices."""
    m = np.asarray(kmesh)
    pts = kmesh_points(kmesh).astype(np.int64)  # [nk][3], integer coordinates
    img = (pts @ np.asarray(R, dtype=np.int64).T) % m
    out = np.array([k_flat(kmesh, *map(int, x)) for x in img], dtype=np.int64)
    assert len(set(out.tolist())) == len(out), "operation does not map the mesh onto itself"
    return out


def group_closure(kmesh, ops) -> list[np.ndarray]:
    """Every element of the group the operations generate, as permutations of the flat mesh indices."""
    nk = int(np.prod(kmesh))
    gens = [act(kmesh, R) for R in ops]
    seen = {tuple(range(nk))}
    todo = [np.arange(nk)]
    while todo:
        g = todo.pop()
        for h in gens:
            x = h[g]
            t = tuple(x.tolist())
            if t not in seen:
                seen.add(t)
                todo.append(x)
    return [np.array(t) for t in sorted(seen)]


def orbit_labels(kmesh, ops) -> np.ndarray:
    """Orbit of every momentum, labelled by its smallest flat index."""
    nk = int(np.prod(kmesh))
    lab = np.arange(nk)
    for g in group_closure(kmesh, ops):  # the orbit of k is {g(k)} over the whole group
        lab = np.minimum(lab, g)
    return lab


def _orbit_hermitian(spec: SystemSpec, tag: int, spin: int, k: int, lab, neg, lo, hi, out, conj_ok: bool):
    """Matrix of momentum k in a table that must be constant on orbits (and, when conj_ok, satisfy
    X(-k) = conj X(k)): copies from the orbit's first member or from the conjugate orbit, else a fresh draw."""
    r = int(lab[k])
    if r < k:
        return out[r]
    if conj_ok:
        rn = int(lab[neg[k]])
        if rn < k:
            return out[rn].conj()
        real = rn == k  # -k in the orbit of k: the matrix must be real
    else:
        real = False
    return random_hermitian_spectrum(spec.seed, tag, spin, k, spec.nao, lo, hi, real)


def make_symmetric_system(spec: SystemSpec, ops, with_V: bool = True) -> System:
    """A system invariant under the point group the operations generate (plus time reversal when the spec asks
    for it): H0 and S constant on orbits; V averaged over the group and rescaled to its former norm (with_V=False:
    V is left to synth.device.make_symmetric_V)."""
    nk, nao, ns = spec.nk, spec.nao, spec.nspin
    lab = orbit_labels(spec.kmesh, ops)
    neg = k_neg(spec.kmesh)
    H0 = np.zeros((ns, nk, nao, nao), dtype=np.complex128)
    for s in range(ns):
        for k in range(nk):
            H0[s, k] = _orbit_hermitian(spec, rng.TAG_F, s, k, lab, neg, -spec.band, spec.band, H0[s],
                                        spec.f_time_reversal)
    Sh = np.zeros((nk, nao, nao), dtype=np.complex128)
    if not spec.s_identity:
        for k in range(nk):
            Sh[k] = _orbit_hermitian(spec, rng.TAG_S, 0, k, lab, neg, -1.0, 1.0, Sh, spec.f_time_reversal)
    S = np.eye(nao)[None] + 0.1 * Sh
    grid = make_grid(spec.ntau, spec.beta)
    G0 = noninteracting_G(H0, S, grid.tau, spec.beta, spec.mu0)
    n_target = electron_count(H0, S, spec.beta, spec.mu0)
    if not with_V:
        return System(spec, grid, H0, S, None, G0, n_target, spec.mu0)
    # V: Hermitian pairing and (optionally) time reversal first, then the group average, which keeps both
    full = {}
    for k1 in range(nk):
        for k2 in range(k1, nk):
            Z = _v_block(spec, k1, k2)
            if k1 == k2:
                Z = 0.5 * (Z + np.conj(np.swapaxes(Z, 1, 2)))
            full[(k1, k2)] = Z
            if k1 != k2:
                full[(k2, k1)] = np.conj(np.swapaxes(Z, 1, 2))
    if spec.v_time_reversal:
        full = _impose_v_time_reversal(spec, full)
    group = group_closure(spec.kmesh, ops)
    norm0 = np.sqrt(sum(float(np.sum(np.abs(Z) ** 2)) for Z in full.values()))
    avg = {}
    for (k1, k2) in full:
        avg[(k1, k2)] = sum(full[(int(g[k1]), int(g[k2]))] for g in group) / len(group)
    norm1 = np.sqrt(sum(float(np.sum(np.abs(Z) ** 2)) for Z in avg.values()))
    add = k_add_table(spec.kmesh)
    V = np.empty((nk, nk, spec.naux, nao, nao), dtype=np.complex128)
    for q in range(nk):
        for k in range(nk):
            V[q, k] = avg[(k, int(add[k, q]))] * (norm0 / norm1)
    return System(spec, grid, H0, S, V, G0, n_target, spec.mu0)
