"""Pins of the oracle's measurement functions (Sec. IV-F, Sec. V-A): Born
sampling against the distribution it draws from, basis states, the
qubit-wise-commuting grouping against its definition, the basis change
against dense Pauli matrices, and the shot estimate against the exact
energy (its limit) and against eigenstates (where it is exact)."""
import numpy as np
import pytest

import oracle
from oracle import dense
from oracle import measure as M
from paper_2607_02749_amd import synth


def test_born_sample_matches_distribution():
    rng = np.random.default_rng(1)
    psi = rng.normal(size=16) + 1j * rng.normal(size=16)
    psi /= np.linalg.norm(psi)
    u = rng.random(400000)
    b = M.born_sample(psi, u)
    freq = np.bincount(b.astype(np.int64), minlength=16) / len(u)
    p = np.abs(psi) ** 2
    assert np.abs(freq - p).max() < 5 * np.sqrt(p.max() / len(u)) + 1e-12
    # inverse CDF: u just below / at a cumulative sum picks that index / the next
    cdf = np.cumsum(p)
    for i in (0, 5, 14):
        assert M.born_sample(psi, [cdf[i] * (1 - 1e-12) / cdf[-1]])[0] == i
        assert M.born_sample(psi, [np.nextafter(cdf[i], 2) / cdf[-1]])[0] == i + 1
    # a basis state is always drawn
    e = np.zeros(32, complex)
    e[19] = 1j
    assert np.all(M.born_sample(e, rng.random(100)) == 19)


def test_argmax_ties_take_smallest_index():
    psi = np.array([0.1, 0.5, -0.5j, 0.2, 0.5, 0.4], dtype=complex)
    assert M.argmax(psi) == 1
    assert M.argmax(np.eye(8)[6]) == 6


def test_qwc_groups_definition():
    inst = synth.make_instance(8, 1, 10, 3, 2, seed=4, m_off=40, off_types=("XX", "YY", "XZ", "ZY"))
    groups = M.qwc_groups(inst.x, inst.z, inst.c)
    seen = []
    for xm, ym, zm, terms in groups:
        assert not (xm & ym) and not (xm & zm) and not (ym & zm)
        for xk, zk, _ in terms:
            for q, L in M._letters(xk, zk).items():
                assert ((xm >> q) & 1, (ym >> q) & 1, (zm >> q) & 1) == \
                    (int(L == "X"), int(L == "Y"), int(L == "Z"))
            seen.append((xk, zk))
        # pairwise: every two terms of a group commute (as dense matrices)
        for a in range(len(terms)):
            for b in range(a + 1, len(terms)):
                pa = dense.pauli(dense.label(8, terms[a][0], terms[a][1]))
                pb = dense.pauli(dense.label(8, terms[b][0], terms[b][1]))
                assert np.allclose(pa @ pb, pb @ pa)
    merged = [(xk, zk) for xk, zk, _ in M.merge_terms(inst.x, inst.z, inst.c) if xk]
    assert sorted(seen) == sorted(merged)


def test_basis_rotation_maps_group_terms_to_z_strings():
    n = 4
    for xm, ym in ((0b0011, 0b0100), (0b1000, 0b0011), (0, 0b1111)):
        rng = np.random.default_rng(xm * 16 + ym)
        psi = rng.normal(size=16) + 1j * rng.normal(size=16)
        v = np.column_stack([M.basis_rotate(col, n, xm, ym) for col in np.eye(16, dtype=complex)])
        assert np.allclose(v.conj().T @ v, np.eye(16))
        assert np.allclose(M.basis_rotate(psi, n, xm, ym), v @ psi)
        assert np.allclose(M.basis_rotate(psi, n, xm, ym, single=True), v @ psi, atol=1e-6)
        zm = (~(xm | ym)) & 0b1111
        for sub in range(16):                 # every term the basis allows
            x = sub & (xm | ym)
            z = (sub & ym) | (sub & zm)
            if not (x | z):
                continue
            p = dense.pauli(dense.label(n, x, z))
            zs = dense.pauli(dense.label(n, 0, x | z))
            assert np.allclose(v @ p @ v.conj().T, zs)


def test_energy_shots_converges_to_exact_energy():
    inst = synth.make_instance(6, 2, 20, 3, 2, seed=8, m_off=12, off_types=("XX", "YY", "XZ", "ZY"))
    psi = oracle.prepare(6, 2, inst.ent, inst.theta)
    e = oracle.energy(6, 2, inst.ent, inst.theta, inst.x, inst.z, inst.c).real
    ng = len(M.qwc_groups(inst.x, inst.z, inst.c))
    shots = 200000
    u = np.random.default_rng(3).random((1 + ng) * shots)
    est = M.energy_shots(6, psi, inst.x, inst.z, inst.c, u, shots)
    # each of the (1 + groups) sample means has variance <= (sum |c|)^2 / shots
    bound = 6 * np.abs(inst.c).sum() / np.sqrt(shots)
    assert abs(est - e) < bound, (est, e, bound)


def test_energy_shots_exact_on_basis_states():
    # |b> is an eigenstate of every Z-string: each shot returns D(b)
    inst = synth.make_instance(7, 1, 25, 3, 2, seed=9)
    from oracle import closed_forms as cf
    for b in (0, 37, 127):
        th = cf.basis_theta(7, 1, b)
        psi = oracle.prepare(7, 1, inst.ent, th)
        u = np.random.default_rng(b).random(500)
        est = M.energy_shots(7, psi, inst.x, inst.z, inst.c, u, 500)
        assert est == pytest.approx(cf.diag_entry(b, inst.x, inst.z, inst.c), abs=1e-12)
