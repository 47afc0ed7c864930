"""Measurement side of the method, plainly (Sec. IV-F, Sec. V-A).

TEST INFRASTRUCTURE ONLY (like the rest of this package): it checks the
library's sampling, decoding and finite-shot estimate and shares no code
with it.

* ``born_sample``: inverse-CDF draws from |psi_i|^2 -- for a uniform u the
  index i with cdf(i-1) <= u * total < cdf(i), cdf the running sum;
* ``argmax``: the most probable basis state (smallest index on ties), the
  bitstring the paper decodes into a structure;
* ``qwc_groups``: qubit-wise-commuting groups of the off-diagonal terms,
  formed by first fit over the merged terms in ascending (x, z) order (each
  group gives every qubit one letter X, Y or Z);
* ``basis_rotate``: psi in a group's eigenbasis -- H on the qubits where the
  group has X, H S^dagger where it has Y (both map the letter to Z);
* ``energy_shots``: the shot estimate: the Z-only part as the mean of
  D(b) over samples of psi, each group as the sum of c_k times the sample
  mean of (-1)^{popcount(b & support_k)} over samples of the rotated psi.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def born_sample(psi: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Probabilities and their running sum in FP64, whatever the amplitudes'
    precision."""
    v = np.asarray(psi).astype(np.complex128)
    p = v.real * v.real + v.imag * v.imag
    cdf = np.cumsum(p)
    target = np.asarray(u, dtype=np.float64) * cdf[-1]
    idx = np.searchsorted(cdf, target, side="right")
    return np.minimum(idx, len(p) - 1).astype(np.uint64)


def argmax(psi: np.ndarray) -> int:
    v = np.asarray(psi).astype(np.complex128)
    return int(np.argmax(v.real * v.real + v.imag * v.imag))


def merge_terms(x, z, c):
    """Sum the coefficients of equal (x, z), drop zeros, ascending (x, z)."""
    acc = {}
    for xk, zk, ck in zip(np.asarray(x, dtype=np.uint64), np.asarray(z, dtype=np.uint64),
                          np.asarray(c, dtype=np.float64)):
        key = (int(xk), int(zk))
        acc[key] = acc.get(key, 0.0) + float(ck)
    return [(k[0], k[1], v) for k, v in sorted(acc.items()) if v != 0.0]


def _letters(x: int, z: int):
    """Per qubit of the term's support: 'X', 'Y' or 'Z'."""
    out = {}
    q = 0
    s = x | z
    while s >> q:
        if (s >> q) & 1:
            xb, zb = (x >> q) & 1, (z >> q) & 1
            out[q] = "Y" if (xb and zb) else ("X" if xb else "Z")
        q += 1
    return out


def qwc_groups(x, z, c) -> List[Tuple[int, int, int, List[Tuple[int, int, float]]]]:
    """[(X qubits, Y qubits, Z qubits, [(x, z, c), ...]), ...] of the merged
    off-diagonal terms, first fit in ascending (x, z) order."""
    groups = []
    for xk, zk, ck in merge_terms(x, z, c):
        if xk == 0:
            continue
        lk = _letters(xk, zk)
        for g in groups:
            if all(g["letters"].get(q, L) == L for q, L in lk.items()):
                g["letters"].update(lk)
                g["terms"].append((xk, zk, ck))
                break
        else:
            groups.append({"letters": dict(lk), "terms": [(xk, zk, ck)]})
    out = []
    for g in groups:
        xm = sum(1 << q for q, L in g["letters"].items() if L == "X")
        ym = sum(1 << q for q, L in g["letters"].items() if L == "Y")
        zm = sum(1 << q for q, L in g["letters"].items() if L == "Z")
        out.append((xm, ym, zm, g["terms"]))
    return out


def basis_rotate(psi: np.ndarray, n: int, xmask: int, ymask: int,
                 single: bool = False) -> np.ndarray:
    """H on the X qubits, H S^dagger on the Y qubits, as 2x2 matrices on the
    qubit's axis of the state tensor (qubit q = bit q of the index).

    single: the complex64 arithmetic of a complex64 state, qubit by qubit in
    ascending order: b <- -i b (Y only), then (h (a + b), h (a - b)) with
    h = 1/sqrt(2) rounded to float32 -- the precision in which a complex64
    engine decides which basis states the draws land on."""
    if single:
        h32 = np.float32(1.0 / np.sqrt(2.0))
        t = np.asarray(psi).astype(np.complex64).reshape([2] * n)
        for q in range(n):
            if not ((xmask | ymask) >> q) & 1:
                continue
            ax = n - 1 - q
            a = np.take(t, 0, axis=ax)
            b = np.take(t, 1, axis=ax)
            if (ymask >> q) & 1:
                b = (b.imag - 1j * b.real).astype(np.complex64)
            t = np.stack([h32 * (a + b), h32 * (a - b)], axis=ax).astype(np.complex64)
        return t.reshape(-1)
    h = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
    sdg = np.array([[1, 0], [0, -1j]], dtype=np.complex128)
    t = np.asarray(psi, dtype=np.complex128).reshape([2] * n)   # axis 0 = qubit n-1
    for q in range(n):
        if (ymask >> q) & 1:
            m = h @ sdg
        elif (xmask >> q) & 1:
            m = h
        else:
            continue
        ax = n - 1 - q
        t = np.moveaxis(np.tensordot(m, t, axes=([1], [ax])), 0, ax)
    return t.reshape(-1)


def energy_shots(n: int, psi: np.ndarray, x, z, c, u: np.ndarray, shots: int,
                 single: bool = False) -> float:
    """The finite-shot estimate; u holds (1 + groups) * shots uniforms: the
    first block for the Z-only part, then one block per group in order
    (single: the basis changes in complex64 arithmetic)."""
    terms = merge_terms(x, z, c)
    idx = np.arange(1 << n, dtype=np.uint64)
    d = np.zeros(1 << n)
    for xk, zk, ck in terms:
        if xk == 0:
            par = np.bitwise_count(idx & np.uint64(zk)) & 1
            d += ck * np.where(par, -1.0, 1.0)
    b = born_sample(psi, u[:shots])
    est = float(np.mean(d[b.astype(np.int64)]))
    for g, (xm, ym, _, gterms) in enumerate(qwc_groups(x, z, c)):
        rot = basis_rotate(psi, n, xm, ym, single)
        b = born_sample(rot, u[(g + 1) * shots:(g + 2) * shots])
        for xk, zk, ck in gterms:
            sup = np.uint64(xk | zk)
            par = np.bitwise_count(b & sup) & 1
            est += ck * float(np.mean(np.where(par, -1.0, 1.0)))
    return est
