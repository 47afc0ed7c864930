"""The Graph-VQE driver's host logic (Sec. IV-C to IV-E) against hand-computed
values: the interaction graph (Eq. 9), modularity (Eq. 10, also against
networkx's implementation), Louvain partitions of graphs whose best
partition is known, the S_min merge, and the sliding-window early stopping
of Eq. 14.  The GPU run of the whole driver is in tests/test_gpu_graphvqe.py."""
import numpy as np
import pytest

from paper_2607_02749_amd import graphvqe as G
from paper_2607_02749_amd import synth


def two_triangles():
    w = np.zeros((6, 6))
    for a, b in ((0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (2, 3)):
        w[a, b] = w[b, a] = 1.0
    return w


def test_interaction_graph_eq9():
    # Z0 Z1 (2), X1 X2 (-3), Z0 (1: one qubit, no edge), identity (5), Y0 Z2 (0.5),
    # X0 Y1 Z2 (-0.25: all three pairs)
    x = [0b000, 0b110, 0b000, 0, 0b001, 0b011]
    z = [0b011, 0b000, 0b001, 0, 0b101, 0b110]
    c = [2.0, -3.0, 1.0, 5.0, 0.5, -0.25]
    w = G.interaction_graph(3, x, z, c)
    want = np.array([[0, 2.25, 0.75], [2.25, 0, 3.25], [0.75, 3.25, 0]])
    assert np.allclose(w, want)


def test_modularity_eq10_hand_values():
    w = two_triangles()
    # m = 7, community degrees 7 and 7, 3 internal edges each:
    # Q = 2 (3/7 - (7/14)^2) = 5/14
    assert G.modularity(w, [0, 0, 0, 1, 1, 1]) == pytest.approx(5 / 14, abs=1e-15)
    # one community: Q = 1 - 1 = 0
    assert G.modularity(w, [0] * 6) == pytest.approx(0.0, abs=1e-15)
    # singletons: Q = -sum_i (k_i / 2m)^2 = -(4*4 + 2*9) / 196
    assert G.modularity(w, range(6)) == pytest.approx(-34 / 196, abs=1e-15)
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(3)
    a = rng.random((9, 9)) * (rng.random((9, 9)) < 0.5)
    a = np.triu(a, 1)
    a = a + a.T
    lab = rng.integers(0, 3, 9)
    g = nx.from_numpy_array(a)
    parts = [set(np.nonzero(lab == k)[0].tolist()) for k in range(3)]
    parts = [p for p in parts if p]
    assert G.modularity(a, lab) == pytest.approx(nx.community.modularity(g, parts), abs=1e-12)


def test_louvain_recovers_known_partitions():
    assert G.blocks_of(G.louvain(two_triangles())) == [[0, 1, 2], [3, 4, 5]]
    # four 5-cliques joined in a ring by single weak edges
    w = np.zeros((20, 20))
    for b in range(4):
        for i in range(5):
            for j in range(i + 1, 5):
                w[5 * b + i, 5 * b + j] = w[5 * b + j, 5 * b + i] = 1.0
        a, c = 5 * b + 4, (5 * (b + 1)) % 20
        w[a, c] = w[c, a] = 0.1
    for seed in range(4):
        blocks = G.blocks_of(G.louvain(w, seed=seed))
        assert blocks == [list(range(5 * b, 5 * b + 5)) for b in range(4)]
    # Louvain never returns a partition worse than the singletons or one block
    rng = np.random.default_rng(0)
    a = rng.random((12, 12))
    a = np.triu(a, 1)
    a = a + a.T
    lab = G.louvain(a)
    assert G.modularity(a, lab) >= max(G.modularity(a, range(12)), G.modularity(a, [0] * 12))


def test_louvain_on_planted_hamiltonian_graph():
    # the synthetic Hamiltonians plant communities with strong intra terms
    # (N(0,1) coefficients, edge p = 0.6) and weak inter terms (0.1 N(0,1));
    # the Eq. 9 graph of such a Hamiltonian should split along them
    inst = synth.make_instance(16, 1, 400, 3, 4, seed=2)
    w = G.interaction_graph(16, inst.x, inst.z, inst.c)
    lab = G.louvain(w, seed=0)
    truth = np.zeros(16, int)
    for k, comm in enumerate(inst.communities):
        truth[list(comm)] = k
    assert G.modularity(w, lab) >= G.modularity(w, truth) - 1e-9
    # every found block lies inside one planted community
    for b in G.blocks_of(lab):
        assert len(set(truth[b].tolist())) == 1


def test_merge_small_blocks():
    w = two_triangles()
    w[5, 0] = w[0, 5] = 0.5
    # block {3} has weight 1 to {0,1,2} (edge 2-3) and 2 to {4,5} (edges 3-4, 3-5)
    lab = np.array([0, 0, 0, 1, 2, 2])
    out = G.merge_small_blocks(w, lab, 2)
    assert G.blocks_of(out) == [[0, 1, 2], [3, 4, 5]]
    # S_min = 4: then both triangles are small; the one with the lower label
    # goes first and joins the other (weight 1 + 0.5)
    out = G.merge_small_blocks(w, lab, 4)
    assert G.blocks_of(out) == [[0, 1, 2, 3, 4, 5]]
    # equal weight to two neighbours: the lower label wins
    w3 = np.zeros((5, 5))
    w3[0, 1] = w3[1, 0] = w3[3, 4] = w3[4, 3] = 2.0
    w3[2, 1] = w3[1, 2] = w3[2, 3] = w3[3, 2] = 1.0
    out = G.merge_small_blocks(w3, [0, 0, 1, 2, 2], 2)
    assert G.blocks_of(out) == [[0, 1, 2], [3, 4]]
    # an isolated small block joins the smallest other block
    w2 = np.zeros((5, 5))
    w2[0, 1] = w2[1, 0] = w2[2, 3] = w2[3, 2] = 1.0
    out = G.merge_small_blocks(w2, [0, 0, 1, 1, 2], 2)
    assert sorted(map(len, G.blocks_of(out))) == [2, 3]
    # nothing below S_min: unchanged
    assert G.blocks_of(G.merge_small_blocks(w, [0, 0, 0, 1, 1, 1], 3)) == [[0, 1, 2], [3, 4, 5]]


def test_window_stopper_eq14():
    # W = 3: Delta_max at E_n covers t = n-3 .. n, four differences
    s = G.WindowStopper(tol=1e-3, window=3, patience=2)
    seq = [10.0, 9.0, 8.5, 8.4999, 8.4998, 8.4997, 8.4996, 8.4995]
    flags = [s.update(e) for e in seq]
    # Delta_max from E_2 on: 1, 1, 1, 1, 0.5, 1e-4 (check 1), 1e-4 (check 2)
    assert flags == [False] * 7 + [True]
    # a jump resets the patience (W = 1: two differences per check)
    s = G.WindowStopper(tol=1e-3, window=1, patience=2)
    out = [s.update(e) for e in (1.0, 1.0, 0.0, 0.0, 0.0, 0.0)]
    assert out == [False, False, False, False, False, True]


def test_param_index_matches_block_mask():
    # the driver's block parameter indices are the block's RY / RZ angles in
    # every layer (Sec. IV-D), as oracle.param_mask selects them
    import oracle

    class _A:
        n, layers, final_rotation = 7, 3, 1

    drv = G.GraphVQE.__new__(G.GraphVQE)
    drv.n, drv.ansatz = 7, _A()
    for block in ([0, 3], [1, 2, 6], [5]):
        idx = drv._param_index(block)
        m = oracle.param_mask(7, 3, G.qubit_mask(block), 1)
        assert np.array_equal(np.nonzero(m)[0], idx)
