"""Brute-force dense matrices for small n (n <= 8): every gate and every Pauli
string is built as a full 2^n x 2^n matrix from Kronecker products of the
textbook 2x2 matrices, U is their product, and E = psi^dagger H psi.

TEST INFRASTRUCTURE ONLY.  Independent of gv_oracle.c: no index tricks, no
bit masks inside the linear algebra; Pauli strings enter as letter labels.
Qubit q is bit q of the index, so it is the (n-1-q)-th factor from the left
of a Kronecker product.
"""
from __future__ import annotations

from functools import reduce
from typing import List, Sequence, Tuple

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
LETTER = {"I": I2, "X": X, "Y": Y, "Z": Z}


def ry(t: float) -> np.ndarray:
    """Eq. 7, first line."""
    c, s = np.cos(t / 2), np.sin(t / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(t: float) -> np.ndarray:
    """Eq. 7, second line."""
    return np.array([[np.exp(-0.5j * t), 0], [0, np.exp(0.5j * t)]], dtype=np.complex128)


def embed(n: int, ops: dict) -> np.ndarray:
    """Kronecker product with ops[q] on qubit q and identity elsewhere."""
    return reduce(np.kron, [ops.get(q, I2) for q in reversed(range(n))])


def cz(n: int, a: int, b: int) -> np.ndarray:
    # |0><0|_a (x) 1 + |1><1|_a (x) Z_b
    return embed(n, {a: P0}) + embed(n, {a: P1, b: Z})


def cnot(n: int, ctl: int, tgt: int) -> np.ndarray:
    # |0><0|_c (x) 1 + |1><1|_c (x) X_t
    return embed(n, {ctl: P0}) + embed(n, {ctl: P1, tgt: X})


def circuit(n: int, layers: int, ent: int, final_rotation: int = 0) -> List[Tuple]:
    """Gate list in application order: ('ry'|'rz', q, param) or ('cz'|'cnot', a, b).
    Layer l: RY on every qubit, RZ on every qubit, then the entangler; the
    optional final rotation layer has no entangler (EfficientSU2, Eq. 8)."""
    out = []
    for l in range(layers + final_rotation):
        base = l * 2 * n
        out += [("ry", q, base + q) for q in range(n)]
        out += [("rz", q, base + n + q) for q in range(n)]
        if l >= layers:
            break
        if ent in (1, 2):
            out += [("cz", q, q + 1) for q in range(n - 1)]
            if ent == 2 and n > 2:
                out.append(("cz", n - 1, 0))
        elif ent in (3, 4):
            if ent == 4 and n > 2:
                out.append(("cnot", n - 1, 0))
            out += [("cnot", q, q + 1) for q in range(n - 1)]
        elif ent == 5:      # full: every pair, first qubit outer
            out += [("cnot", i, j) for i in range(n) for j in range(i + 1, n)]
        elif ent == 6:      # reverse linear
            out += [("cnot", q, q + 1) for q in reversed(range(n - 1))]
        elif ent == 7:      # pairwise: even pairs, then odd pairs
            out += [("cnot", q, q + 1) for q in range(0, n - 1, 2)]
            out += [("cnot", q, q + 1) for q in range(1, n - 1, 2)]
        elif ent == 8:      # shifted circular alternating
            ring = ([(n - 1, 0)] + [(q, q + 1) for q in range(n - 1)]) if n > 2 else \
                [(q, q + 1) for q in range(n - 1)]
            if n > 2:
                s = l % len(ring)
                ring = ring[len(ring) - s:] + ring[:len(ring) - s]
            if l % 2:
                ring = [(b, a) for a, b in ring]
            out += [("cnot", a, b) for a, b in ring]
        elif ent != 0:
            raise ValueError("unknown entangler")
    return out


def unitary(n: int, layers: int, ent: int, theta, final_rotation: int = 0) -> np.ndarray:
    u = np.eye(1 << n, dtype=np.complex128)
    for g in circuit(n, layers, ent, final_rotation):
        if g[0] == "ry":
            m = embed(n, {g[1]: ry(theta[g[2]])})
        elif g[0] == "rz":
            m = embed(n, {g[1]: rz(theta[g[2]])})
        elif g[0] == "cz":
            m = cz(n, g[1], g[2])
        else:
            m = cnot(n, g[1], g[2])
        u = m @ u
    return u


def state(n, layers, ent, theta, final_rotation=0) -> np.ndarray:
    e0 = np.zeros(1 << n, dtype=np.complex128)
    e0[0] = 1.0
    return unitary(n, layers, ent, theta, final_rotation) @ e0


def label(n: int, x: int, z: int) -> str:
    """Letters of qubits n-1 ... 0 for P(x, z): x only -> X, z only -> Z,
    both -> Y (P(x, z) = i^{|x&z|} X^x Z^z and i X Z = Y)."""
    out = []
    for q in reversed(range(n)):
        xb, zb = (int(x) >> q) & 1, (int(z) >> q) & 1
        out.append({(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}[(xb, zb)])
    return "".join(out)


def pauli(lab: str) -> np.ndarray:
    """Matrix of a label written most significant qubit first."""
    return reduce(np.kron, [LETTER[ch] for ch in lab])


def hamiltonian(n: int, x: Sequence[int], z: Sequence[int], c: Sequence[float]) -> np.ndarray:
    """H = sum_k c_k P_k (Eq. 6) as a dense matrix."""
    h = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for xk, zk, ck in zip(x, z, c):
        h += ck * pauli(label(n, xk, zk))
    return h


def energy(n, layers, ent, theta, h, final_rotation=0) -> complex:
    psi = state(n, layers, ent, theta, final_rotation)
    return complex(np.vdot(psi, h @ psi))


def param_shift_grad(n, layers, ent, theta, h, final_rotation=0) -> np.ndarray:
    """Eq. 13 on the dense path."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros(theta.size)
    for j in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += np.pi / 2
        tm[j] -= np.pi / 2
        g[j] = 0.5 * (energy(n, layers, ent, tp, h, final_rotation).real
                      - energy(n, layers, ent, tm, h, final_rotation).real)
    return g
