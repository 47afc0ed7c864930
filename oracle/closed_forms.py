"""Closed-form energies and gradients that hold at any n.

TEST INFRASTRUCTURE ONLY.  These never touch a state vector, so they pin the
oracle (and the GPU path) at sizes where nothing else can:

* product states (no entangler): each qubit's Bloch vector is rotated by the
  SO(3) images of its RY and RZ gates (Eq. 7), and the expectation of a Pauli
  string is the product of the Bloch components it selects;
* computational basis states: RY(pi) on a set of qubits in the first layer,
  every other angle 0, gives +-|b>, whose energy is the diagonal entry D(b);
* the 1D cluster state (RY(pi/2) everywhere, then the CZ ladder) and the GHZ
  state (RY(pi/2) on qubit 0, then the CNOT ladder), with their textbook
  stabilizer expectations.
"""
from __future__ import annotations

import numpy as np


def so3_ry(t: float) -> np.ndarray:
    """Bloch-sphere image of RY(t): rotation by t about the y axis."""
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def so3_ry_d(t: float) -> np.ndarray:
    c, s = np.cos(t), np.sin(t)
    return np.array([[-s, 0.0, c], [0.0, 0.0, 0.0], [-c, 0.0, -s]])


def so3_rz(t: float) -> np.ndarray:
    """Bloch-sphere image of RZ(t): rotation by t about the z axis."""
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def so3_rz_d(t: float) -> np.ndarray:
    c, s = np.cos(t), np.sin(t)
    return np.array([[-s, -c, 0.0], [c, -s, 0.0], [0.0, 0.0, 0.0]])


def _pauli_index(x: int, z: int, q: int) -> int:
    """-1 for identity on qubit q, else 0/1/2 for X/Y/Z."""
    xb, zb = (x >> q) & 1, (z >> q) & 1
    return {(0, 0): -1, (1, 0): 0, (1, 1): 1, (0, 1): 2}[(xb, zb)]


def bloch_vectors(n: int, rot_layers: int, theta) -> np.ndarray:
    """Bloch vector of every qubit after rot_layers RY-then-RZ layers and no
    entangler; theta laid out as l*2n + g*n + q."""
    r = np.zeros((n, 3))
    for q in range(n):
        v = np.array([0.0, 0.0, 1.0])
        for l in range(rot_layers):
            v = so3_ry(theta[l * 2 * n + q]) @ v
            v = so3_rz(theta[l * 2 * n + n + q]) @ v
        r[q] = v
    return r


def product_energy_grad(n: int, rot_layers: int, theta, x, z, c):
    """Energy and gradient of the product state (entangler NONE) by the
    product rule.  rot_layers = layers + final_rotation."""
    theta = np.asarray(theta, dtype=np.float64)
    r = bloch_vectors(n, rot_layers, theta)
    # derivative of each qubit's Bloch vector by each of its angles
    dr = np.zeros((rot_layers, 2, n, 3))
    for q in range(n):
        mats = []
        for l in range(rot_layers):
            mats.append(("y", so3_ry(theta[l * 2 * n + q]), so3_ry_d(theta[l * 2 * n + q])))
            mats.append(("z", so3_rz(theta[l * 2 * n + n + q]), so3_rz_d(theta[l * 2 * n + n + q])))
        for k in range(len(mats)):
            v = np.array([0.0, 0.0, 1.0])
            for j, (_, m, md) in enumerate(mats):
                v = (md if j == k else m) @ v
            dr[k // 2, k % 2, q] = v
    e = 0.0
    grad = np.zeros(theta.size)
    for xk, zk, ck in zip(np.asarray(x, dtype=np.uint64), np.asarray(z, dtype=np.uint64), c):
        xk, zk = int(xk), int(zk)
        sup = [(q, _pauli_index(xk, zk, q)) for q in range(n)]
        sup = [(q, a) for q, a in sup if a >= 0]
        vals = [r[q, a] for q, a in sup]
        e += ck * float(np.prod(vals)) if vals else ck
        for t, (q, a) in enumerate(sup):
            rest = float(np.prod(vals[:t] + vals[t + 1:])) if len(vals) > 1 else 1.0
            for l in range(rot_layers):
                for g in range(2):
                    grad[l * 2 * n + g * n + q] += ck * dr[l, g, q, a] * rest
    return e, grad


def basis_theta(n: int, layers: int, bits: int, final_rotation: int = 0) -> np.ndarray:
    """Angles that prepare +-|bits>: RY(pi) on the set qubits of layer 0,
    every other angle 0 (RY(pi)|0> = |1> by Eq. 7)."""
    th = np.zeros(2 * n * (layers + final_rotation))
    for q in range(n):
        if (bits >> q) & 1:
            th[q] = np.pi
    return th


def diag_entry(bits: int, x, z, c) -> float:
    """D(b) = sum over Z-only terms of c_k (-1)^{popcount(b & z_k)}."""
    tot = 0.0
    for xk, zk, ck in zip(x, z, c):
        if int(xk) == 0:
            tot += ck * (-1.0 if bin(bits & int(zk)).count("1") % 2 else 1.0)
    return tot


def cluster_theta(n: int) -> np.ndarray:
    """One CZ layer after RY(pi/2) on every qubit: the 1D cluster state."""
    th = np.zeros(2 * n)
    th[:n] = np.pi / 2
    return th


def cluster_stabilizers(n: int):
    """(x, z) masks of X_0 Z_1, Z_{q-1} X_q Z_{q+1}, Z_{n-2} X_{n-1}: each has
    expectation +1 on the cluster state."""
    out = []
    for q in range(n):
        z = 0
        if q > 0:
            z |= 1 << (q - 1)
        if q < n - 1:
            z |= 1 << (q + 1)
        out.append((1 << q, z))
    return out


def ghz_theta(n: int) -> np.ndarray:
    """RY(pi/2) on qubit 0 only, then the linear CNOT ladder: GHZ state."""
    th = np.zeros(2 * n)
    th[0] = np.pi / 2
    return th
