"""CPU oracle for the Graph-VQE energy / gradient hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may use this package; the product path never does.  It shares no
code with the GPU library.

``gv_oracle.c`` holds the complex128 per-gate simulator (Sec. IV-B, Eq. 7-8),
the direct-sum diagonal and term-by-term Hamiltonian (Eq. 6), the energy
(Eq. 4) and the gate-by-gate adjoint gradient.  This module loads it with
ctypes and adds the parameter-shift gradient of Eq. 13 on top of it.
``dense`` (brute-force matrices, n <= 8) and ``closed_forms`` (product,
basis, cluster and GHZ states) are the independent pins the tests check the
oracle against.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gv_oracle.c")
LIB = os.path.join(HERE, "libgv_oracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    L = ctypes.CDLL(LIB)
    i32, i64, dbl, p = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    L.gvo_num_params.argtypes = [i32, i32, i32]
    L.gvo_num_params.restype = i32
    L.gvo_prepare.argtypes = [i32, i32, i32, i32, p, p]
    L.gvo_prepare.restype = i32
    L.gvo_apply_gates.argtypes = [i32, i32, i32, i32, p, i64, i64, i32, p]
    L.gvo_apply_gates.restype = i64
    L.gvo_num_gates.argtypes = [i32, i32, i32, i32]
    L.gvo_num_gates.restype = i64
    L.gvo_diag.argtypes = [i32, i64, p, p, p, p]
    L.gvo_diag.restype = None
    L.gvo_diag_at.argtypes = [i64, p, p, p, ctypes.c_uint64]
    L.gvo_diag_at.restype = dbl
    L.gvo_apply_h.argtypes = [i32, i64, p, p, p, p, p, p]
    L.gvo_apply_h.restype = None
    L.gvo_inner.argtypes = [i32, p, p, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.gvo_inner.restype = None
    L.gvo_energy_grad.argtypes = [i32, i32, i32, i32, p, i64, p, p, p, p, p, p, p]
    L.gvo_energy_grad.restype = i32
    L.gvo_adjoint_gates.argtypes = [i32, i32, i32, i32, p, i64, i64, p, p, p]
    L.gvo_adjoint_gates.restype = i64
    L.gvo_max_threads.argtypes = []
    L.gvo_max_threads.restype = i32
    L.gvo_set_threads.argtypes = [i32]
    L.gvo_set_threads.restype = None
    _lib = L
    return L


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _terms(x, z, c):
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    if not (x.shape == z.shape == c.shape):
        raise ValueError("x, z, c must have the same length")
    return x, z, c


def max_threads() -> int:
    """Host threads the oracle's parallel loops use."""
    return int(_load().gvo_max_threads())


def set_threads(n: int) -> None:
    """Threads for the oracle's parallel loops from now on."""
    _load().gvo_set_threads(int(n))


def num_params(n: int, layers: int, final_rotation: int = 0) -> int:
    return int(_load().gvo_num_params(n, layers, final_rotation))


def num_gates(n: int, layers: int, ent: int, final_rotation: int = 0) -> int:
    return int(_load().gvo_num_gates(n, layers, ent, final_rotation))


def prepare(n: int, layers: int, ent: int, theta, final_rotation: int = 0) -> np.ndarray:
    """psi = U(theta)|0...0> as complex128[2^n]."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    if theta.shape != (num_params(n, layers, final_rotation),):
        raise ValueError("wrong number of parameters")
    psi = np.empty(1 << n, dtype=np.complex128)
    rc = _load().gvo_prepare(n, layers, ent, final_rotation, _ptr(theta), _ptr(psi))
    if rc:
        raise ValueError(f"gvo_prepare failed ({rc})")
    return psi


def apply_gates(n, layers, ent, theta, psi, first, count, inverse=False, final_rotation=0):
    """Apply gates [first, first+count) of the circuit to psi in place."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.shape == (1 << n,)
    return int(_load().gvo_apply_gates(n, layers, ent, final_rotation, _ptr(theta),
                                       first, count, int(inverse), _ptr(psi)))


def adjoint_gates(n, layers, ent, theta, phi, lam, grad, first, count, final_rotation=0):
    """Reverse-mode steps for gates [first, first+count) (see gv_oracle.c)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    for a in (phi, lam):
        assert a.dtype == np.complex128 and a.flags.c_contiguous and a.shape == (1 << n,)
    assert grad.dtype == np.float64 and grad.flags.c_contiguous
    return int(_load().gvo_adjoint_gates(n, layers, ent, final_rotation, _ptr(theta),
                                         first, count, _ptr(phi), _ptr(lam), _ptr(grad)))


def diag(n: int, x, z, c) -> np.ndarray:
    """D_i = sum over Z-only terms of c_k (-1)^{popcount(i & z_k)} (direct sum)."""
    x, z, c = _terms(x, z, c)
    d = np.empty(1 << n, dtype=np.float64)
    _load().gvo_diag(n, len(c), _ptr(x), _ptr(z), _ptr(c), _ptr(d))
    return d


def diag_at(x, z, c, indices) -> np.ndarray:
    """D_i at the given indices, each by direct summation."""
    x, z, c = _terms(x, z, c)
    L = _load()
    return np.array([L.gvo_diag_at(len(c), _ptr(x), _ptr(z), _ptr(c), int(i))
                     for i in np.asarray(indices, dtype=np.uint64)], dtype=np.float64)


def apply_h(n: int, x, z, c, psi, d: Optional[np.ndarray] = None) -> np.ndarray:
    """H psi, term by term (Z-only terms through d when d is given)."""
    x, z, c = _terms(x, z, c)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty_like(psi)
    _load().gvo_apply_h(n, len(c), _ptr(x), _ptr(z), _ptr(c), _ptr(d), _ptr(psi), _ptr(out))
    return out


def inner(n: int, a, b) -> complex:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    re, im = ctypes.c_double(), ctypes.c_double()
    _load().gvo_inner(n, _ptr(a), _ptr(b), ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def energy(n, layers, ent, theta, x, z, c, d=None, final_rotation=0) -> complex:
    """<psi(theta)|H|psi(theta)> (Eq. 4); the imaginary part should vanish."""
    psi = prepare(n, layers, ent, theta, final_rotation)
    return inner(n, psi, apply_h(n, x, z, c, psi, d))


def energy_grad(n, layers, ent, theta, x, z, c, d=None, mask=None,
                final_rotation=0) -> Tuple[complex, np.ndarray]:
    """Energy and adjoint gradient (gate-by-gate reverse sweep)."""
    x, z, c = _terms(x, z, c)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    p = num_params(n, layers, final_rotation)
    if theta.shape != (p,):
        raise ValueError("wrong number of parameters")
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert mask.shape == (p,)
    e = np.zeros(2, dtype=np.float64)
    g = np.zeros(p, dtype=np.float64)
    rc = _load().gvo_energy_grad(n, layers, ent, final_rotation, _ptr(theta), len(c),
                                 _ptr(x), _ptr(z), _ptr(c), _ptr(d), _ptr(mask),
                                 _ptr(e), _ptr(g))
    if rc:
        raise ValueError(f"gvo_energy_grad failed ({rc})")
    return complex(e[0], e[1]), g


def param_shift_grad(n, layers, ent, theta, x, z, c, d=None, final_rotation=0,
                     indices=None) -> np.ndarray:
    """Eq. 13: dE/dtheta_j = (E(theta + pi/2 e_j) - E(theta - pi/2 e_j)) / 2,
    exact for RY and RZ (generators with eigenvalues +-1)."""
    theta = np.asarray(theta, dtype=np.float64)
    idx = range(theta.size) if indices is None else indices
    out = np.zeros(theta.size)
    for j in idx:
        tp = theta.copy()
        tp[j] += np.pi / 2
        tm = theta.copy()
        tm[j] -= np.pi / 2
        out[j] = 0.5 * (energy(n, layers, ent, tp, x, z, c, d, final_rotation).real
                        - energy(n, layers, ent, tm, x, z, c, d, final_rotation).real)
    return out


def param_mask(n: int, layers: int, qubit_mask: int, final_rotation: int = 0) -> np.ndarray:
    """Parameters of the qubits in qubit_mask: their RY and RZ angles in every
    layer (the block parameter set of Eq. 11)."""
    p = num_params(n, layers, final_rotation)
    m = np.zeros(p, dtype=np.uint8)
    for l in range(layers + final_rotation):
        for g in range(2):
            for q in range(n):
                if (qubit_mask >> q) & 1:
                    m[l * 2 * n + g * n + q] = 1
    return m
