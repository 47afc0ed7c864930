"""Seeded synthetic workloads: community-structured Pauli-sum Hamiltonians and
ansatz angles.

This module only draws random inputs.  It holds none of the method's
arithmetic (no state vector, no energy, no gradient), so both the GPU path and
the CPU oracle may take their inputs from it.

Why synthetic: the paper's Hamiltonians come from lattice protein folding
(Sec. IV-A, Eq. 1-6) built from contact potentials and penalties that are not
available here.  What the paper states about their structure is that they are
real-coefficient sums of Pauli strings (Eq. 6), sparse with high-weight
non-local terms, and that the qubits form weakly coupled communities that
Graph-VQE finds with Louvain on the interaction graph (Sec. IV-C, Eq. 9-10).
The recipe below plants such communities and draws terms on them.

Recipe (numpy ``default_rng(seed)``, draws in this order):
  1. communities: n qubits cut into K contiguous, near-equal blocks;
  2. graph: stochastic block model, intra-community edge p_in=0.6,
     inter-community edge p_out=0.05 (upper triangle, row-major order);
  3. diagonal terms: weight w ~ U{1..w_max}; a seed qubit uniform; the support
     grows one qubit at a time -- with probability 0.9 a uniform graph
     neighbour of the support not yet in it (when one exists), otherwise a
     uniform qubit not yet in it; duplicate supports are redrawn;
  4. off-diagonal terms (two-qubit XX/YY/XZ/ZY, grown the same way): see
     ``_offdiag_terms``;
  5. coefficients: N(0,1) when the whole support lies in one community,
     0.1*N(0,1) otherwise;
  6. angles: theta ~ U[-pi, pi) for every parameter (Eq. 7 range).

A Pauli string is stored as two bit masks over the qubits plus a real
coefficient: P(x, z) = i^{|x & z|} X^x Z^z, so Y on a qubit is x=z=1 there.
Qubit q is bit q of an amplitude index.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

# entangler codes shared with the C-ABI (same numeric values as gv_entangler)
ENT_NONE = 0
ENT_CZ_LINEAR = 1
ENT_CZ_CIRCULAR = 2
ENT_CNOT_LINEAR = 3
ENT_CNOT_CIRCULAR = 4
ENT_CNOT_FULL = 5
ENT_CNOT_REVERSE_LINEAR = 6
ENT_CNOT_PAIRWISE = 7
ENT_CNOT_SCA = 8

P_IN = 0.6
P_OUT = 0.05
P_NEIGHBOUR = 0.9


@dataclass
class Instance:
    """One energy/gradient problem: ansatz shape, Hamiltonian, angles."""
    n: int
    layers: int
    ent: int
    final_rotation: int
    x: np.ndarray          # uint64[M]
    z: np.ndarray          # uint64[M]
    c: np.ndarray          # float64[M]
    theta: np.ndarray      # float64[P]
    communities: List[List[int]] = field(default_factory=list)
    edges: Optional[np.ndarray] = None   # int32[E, 2]
    cluster_mask: int = 0  # qubits whose parameters a restricted update trains

    @property
    def num_params(self) -> int:
        return 2 * self.n * (self.layers + self.final_rotation)

    @property
    def num_terms(self) -> int:
        return int(self.c.shape[0])


def num_params(n: int, layers: int, final_rotation: int = 0) -> int:
    """P = 2 n (L + final_rotation); Eq. 8 is the final_rotation=1 case."""
    return 2 * n * (layers + final_rotation)


def communities_contiguous(n: int, k: int) -> List[List[int]]:
    k = max(1, min(k, n))
    bounds = [round(i * n / k) for i in range(k + 1)]
    return [list(range(bounds[i], bounds[i + 1])) for i in range(k)]


def _sbm_graph(rng, n, comm_of, p_in, p_out):
    adj = [set() for _ in range(n)]
    edges = []
    for a in range(n):
        for b in range(a + 1, n):
            p = p_in if comm_of[a] == comm_of[b] else p_out
            if rng.random() < p:
                adj[a].add(b)
                adj[b].add(a)
                edges.append((a, b))
    return adj, np.array(edges, dtype=np.int32).reshape(-1, 2)


def _grow_support(rng, n, adj, w):
    sup = [int(rng.integers(n))]
    inside = {sup[0]}
    while len(sup) < w:
        nb = sorted(set().union(*(adj[q] for q in sup)) - inside)
        if nb and rng.random() < P_NEIGHBOUR:
            q = nb[int(rng.integers(len(nb)))]
        else:
            rest = [q for q in range(n) if q not in inside]
            q = rest[int(rng.integers(len(rest)))]
        sup.append(q)
        inside.add(q)
    return sorted(sup)


def _diag_terms(rng, n, adj, m, w_max):
    seen = set()
    out = []
    w_hi = min(w_max, n)
    from math import comb
    if m > sum(comb(n, w) for w in range(1, w_hi + 1)):
        raise ValueError(f"{m} distinct Z-strings of weight 1..{w_hi} do not exist on {n} qubits")
    while len(out) < m:
        w = int(rng.integers(1, w_hi + 1))
        sup = _grow_support(rng, n, adj, w)
        mask = 0
        for q in sup:
            mask |= 1 << q
        if mask in seen:
            continue
        seen.add(mask)
        out.append(sup)
    return out


_PAULI_XZ = {"X": (1, 0), "Y": (1, 1), "Z": (0, 1)}


def _offdiag_terms(rng, n, adj, m, types: Sequence[str], groups: int = 0):
    """Two-qubit terms with at least one X or Y.

    A type such as "XZ" names an unordered pair of letters: either qubit of
    the support may carry the X.  (Read as ordered, the four types XX, YY,
    XZ, ZY would give at most 4 C(n, 2) distinct terms -- 1984 on 32 qubits,
    fewer than the 2000 the largest workload asks for.)

    groups == 0: each term draws its type uniformly from ``types``, a grown
    two-qubit support and a uniform orientation.
    groups > 0: ``groups`` random per-qubit bases (X, Y or Z on every qubit)
    are drawn first; each term picks a basis uniformly, then a grown support,
    and is kept when its two letters under that basis form one of ``types``.
    All terms of a basis commute qubit-wise, so the terms fall into at most
    ``groups`` qubit-wise-commuting sets.
    """
    allowed = {tuple(sorted(t)) for t in types}
    bases = None
    if groups > 0:
        letters = np.array(["X", "Y", "Z"])
        bases = [letters[rng.integers(0, 3, size=n)] for _ in range(groups)]
    seen = set()
    out = []
    guard = 0
    while len(out) < m:
        guard += 1
        if guard > 400 * m + 10000:
            raise RuntimeError("cannot draw enough distinct off-diagonal terms")
        sup = _grow_support(rng, n, adj, 2)
        if bases is None:
            t = types[int(rng.integers(len(types)))]
            if rng.integers(2):
                t = t[::-1]
        else:
            b = bases[int(rng.integers(groups))]
            t = str(b[sup[0]]) + str(b[sup[1]])
            if tuple(sorted(t)) not in allowed:
                continue
        x = z = 0
        for q, letter in zip(sup, t):
            xb, zb = _PAULI_XZ[letter]
            x |= xb << q
            z |= zb << q
        if (x, z) in seen:
            continue
        seen.add((x, z))
        out.append((sup, x, z))
    return out


def make_instance(n: int, layers: int, m_diag: int, w_max: int, k_comm: int,
                  seed: int = 0, m_off: int = 0,
                  off_types: Sequence[str] = ("XX", "YY", "XZ"),
                  off_groups: int = 0, ent: int = ENT_CZ_LINEAR,
                  final_rotation: int = 0, cluster: Optional[int] = None,
                  rng: Optional[np.random.Generator] = None) -> Instance:
    """Draw one planted-community instance (see the module docstring)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    comms = communities_contiguous(n, k_comm)
    comm_of = np.empty(n, dtype=np.int64)
    for ci, members in enumerate(comms):
        comm_of[members] = ci
    adj, edges = _sbm_graph(rng, n, comm_of, P_IN, P_OUT)
    dsup = _diag_terms(rng, n, adj, m_diag, w_max)
    osup = _offdiag_terms(rng, n, adj, m_off, off_types, off_groups) if m_off else []
    xs, zs, intra = [], [], []
    for sup in dsup:
        mask = 0
        for q in sup:
            mask |= 1 << q
        xs.append(0)
        zs.append(mask)
        intra.append(len({int(comm_of[q]) for q in sup}) == 1)
    for sup, x, z in osup:
        xs.append(x)
        zs.append(z)
        intra.append(len({int(comm_of[q]) for q in sup}) == 1)
    intra = np.array(intra, dtype=bool)
    coeff = rng.normal(0.0, 1.0, size=len(xs))
    coeff = np.where(intra, coeff, 0.1 * coeff)
    p = num_params(n, layers, final_rotation)
    theta = rng.uniform(-np.pi, np.pi, size=p)
    cmask = 0
    if cluster is not None:
        for q in comms[cluster % len(comms)]:
            cmask |= 1 << q
    return Instance(n=n, layers=layers, ent=ent, final_rotation=final_rotation,
                    x=np.array(xs, dtype=np.uint64), z=np.array(zs, dtype=np.uint64),
                    c=coeff.astype(np.float64), theta=theta.astype(np.float64),
                    communities=comms, edges=edges, cluster_mask=cmask)


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the five benchmark configurations of this
# engine; each is seeded (seed 0, the paper's fixed seed in Sec. V-A).
# ---------------------------------------------------------------------------

def workload_small(seed: int = 0) -> Instance:
    """n=10, L=2 CZ ladder (40 params), 200 Z-strings w 1-4, 4 communities."""
    return make_instance(10, 2, 200, 4, 4, seed=seed)


def workload_n22(seed: int = 0) -> Instance:
    """n=22, L=4 (176 params), 5000 Z-strings w 1-4 + 500 XX/YY/XZ, 8 communities."""
    return make_instance(22, 4, 5000, 4, 8, seed=seed, m_off=500,
                         off_types=("XX", "YY", "XZ"))


def workload_n28(seed: int = 0) -> Instance:
    """n=28, L=6 (336 params), 20000 Z-strings w 1-6, 16 communities."""
    return make_instance(28, 6, 20000, 6, 16, seed=seed)


def workload_n32(seed: int = 0) -> Instance:
    """n=32, L=4 (256 params), 50000 Z-strings w 1-6 + 2000 XX/YY/XZ/ZY in
    at most 64 qubit-wise-commuting groups, 32 communities."""
    return make_instance(32, 4, 50000, 6, 32, seed=seed, m_off=2000,
                         off_types=("XX", "YY", "XZ", "ZY"), off_groups=64)


def workload_batch(count: int = 256, seed: int = 0, n_lo: int = 12, n_hi: int = 20,
                   layer_choices: Sequence[int] = (3, 4, 5)) -> List[Instance]:
    """Uneven cluster instances: n ~ U{n_lo..n_hi}, L ~ U(layer_choices),
    50 n Z-strings (w 1-4) + 5 n XX/YY terms on a 2-4 community graph; instance
    i trains only the parameters of its community (i mod K_i)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        layers = int(layer_choices[int(rng.integers(len(layer_choices)))])
        k = int(rng.integers(2, 5))
        out.append(make_instance(n, layers, 50 * n, 4, k, m_off=5 * n,
                                 off_types=("XX", "YY"), cluster=i % k, rng=rng))
    return out


def random_theta(p: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-np.pi, np.pi, size=p)
