"""The seeded input generator: determinism, sizes and the structure the
workload recipe promises (distinct terms, weights, community coefficients,
qubit-wise-commuting group bound)."""
import numpy as np
import pytest

from paper_2607_02749_amd import synth


def greedy_qwc_groups(x, z, n):
    """Count of first-fit qubit-wise-commuting groups (per-qubit letter sets)."""
    groups = []
    for xk, zk in zip(x, z):
        letters = {q: (int(xk) >> q & 1, int(zk) >> q & 1) for q in range(n)
                   if (int(xk) | int(zk)) >> q & 1}
        for g in groups:
            if all(g.get(q, v) == v for q, v in letters.items()):
                g.update(letters)
                break
        else:
            groups.append(dict(letters))
    return len(groups)


def test_deterministic():
    a = synth.workload_small()
    b = synth.workload_small()
    for f in ("x", "z", "c", "theta"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = synth.workload_small(seed=1)
    assert not np.array_equal(a.c, c.c)


def test_small_workload_shape():
    w = synth.workload_small()
    assert w.n == 10 and w.layers == 2 and w.num_params == 40
    assert w.num_terms == 200 and np.all(w.x == 0)
    assert len(set(w.z.tolist())) == 200
    wts = np.array([bin(int(v)).count("1") for v in w.z])
    assert wts.min() >= 1 and wts.max() <= 4
    assert np.all(w.theta >= -np.pi) and np.all(w.theta < np.pi)


def test_n22_offdiag_types_and_coefficients():
    w = synth.workload_n22()
    off = w.x != 0
    assert off.sum() == 500 and (~off).sum() == 5000
    for xk, zk in zip(w.x[off], w.z[off]):
        sup = int(xk) | int(zk)
        assert bin(sup).count("1") == 2
    comm = np.zeros(w.n, int)
    for i, members in enumerate(w.communities):
        comm[members] = i
    for xk, zk, ck in zip(w.x, w.z, w.c):
        sup = [q for q in range(w.n) if (int(xk) | int(zk)) >> q & 1]
        if len({comm[q] for q in sup}) > 1:
            assert abs(ck) < 1.0  # 0.1 N(0,1): |c| >= 1 would be a 10-sigma draw


def test_n32_groups_bound():
    w = synth.make_instance(32, 4, 200, 6, 32, seed=0, m_off=2000,
                            off_types=("XX", "YY", "XZ", "ZY"), off_groups=64)
    off = w.x != 0
    assert off.sum() == 2000
    assert greedy_qwc_groups(w.x[off], w.z[off], 32) <= 64


def test_batch_workload():
    b = synth.workload_batch(count=12)
    assert len(b) == 12
    for i, inst in enumerate(b):
        assert 12 <= inst.n <= 20 and inst.layers in (3, 4, 5)
        assert inst.num_terms == 55 * inst.n
        assert inst.cluster_mask != 0
        assert 2 <= len(inst.communities) <= 4


def test_impossible_term_counts_raise():
    # 5 qubits hold only 30 distinct Z-strings of weight 1..4
    with pytest.raises(ValueError):
        synth.make_instance(5, 1, 31, 4, 2, seed=0)
    synth.make_instance(5, 1, 30, 4, 2, seed=0)
