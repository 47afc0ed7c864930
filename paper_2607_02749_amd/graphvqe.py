"""Graph-VQE's optimisation driver on top of the energy / gradient library
(Sec. IV-C to IV-E).

* ``interaction_graph``: the weighted qubit interaction graph of a Pauli sum,
  w_ij = sum of |c_k| over the terms acting on both qubits (Eq. 9).
* ``modularity``: Q of a partition of that graph (Eq. 10).
* ``louvain``: a Louvain community detection that maximises Q (local moves,
  then aggregation of the communities, repeated until Q stops improving),
  and ``merge_small_blocks``: blocks under S_min joined to the neighbour
  block they are most strongly coupled to (Sec. IV-C).
* ``WindowStopper``: the sliding-window criterion of Eq. 14 with patience.
* ``GraphVQE``: epochs of (1) blocks from the graph, (2) concurrent restricted
  block updates -- each block minimises the full-Hamiltonian energy over its
  own parameters with the others frozen (Eq. 11), every block running
  SciPy's L-BFGS-B in its own thread while one evaluation server gathers the
  blocks' pending energy / gradient requests into one batched library launch
  --, (3) a global L-BFGS-B refinement over all parameters (gradients from
  the library's reverse sweep, Eq. 13 defines the same gradient), with the
  energy optionally summed over Hamiltonian batches (Eq. 12), and (4) the
  epoch-level patience on the best energy, warm-starting every epoch from the
  best parameters found (Sec. IV-E).

Every energy and gradient comes from the HIP library (``gv``); this module
only plans and steers.  Sizes follow the paper's set-up: tolerance 1e-4,
patience 12 and window 40 for the early stopping, epoch patience 3.
"""
from __future__ import annotations

import threading
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np


# --------------------------------------------------------------- the graph

def interaction_graph(n: int, x, z, c) -> np.ndarray:
    """w_ij = sum_{k: P_k acts on i and on j} |c_k| for i != j (Eq. 9);
    zero diagonal."""
    w = np.zeros((n, n))
    for xk, zk, ck in zip(np.asarray(x, dtype=np.uint64), np.asarray(z, dtype=np.uint64),
                          np.asarray(c, dtype=np.float64)):
        sup = int(xk) | int(zk)
        qs = [q for q in range(n) if (sup >> q) & 1]
        for a in range(len(qs)):
            for b in range(a + 1, len(qs)):
                w[qs[a], qs[b]] += abs(ck)
                w[qs[b], qs[a]] += abs(ck)
    return w


def modularity(w: np.ndarray, labels: Sequence[int]) -> float:
    """Q = 1/(2m) sum_ij [w_ij - k_i k_j / (2m)] delta(c_i, c_j) (Eq. 10),
    m = half the sum of all w_ij, k_i = sum_j w_ij."""
    w = np.asarray(w, dtype=np.float64)
    two_m = w.sum()
    if two_m <= 0:
        return 0.0
    k = w.sum(axis=1)
    lab = np.asarray(labels)
    same = lab[:, None] == lab[None, :]
    return float(((w - np.outer(k, k) / two_m) * same).sum() / two_m)


def _local_moves(w: np.ndarray, order: np.ndarray) -> np.ndarray:
    """Louvain's first phase on a (possibly aggregated, self-looped) graph:
    every node starts alone; nodes are visited in `order` and moved to the
    neighbouring community with the largest modularity gain (staying put on
    ties), until a full sweep moves nothing.  Returns community labels."""
    nn = w.shape[0]
    two_m = w.sum()
    k = w.sum(axis=1)
    lab = np.arange(nn)
    tot = k.copy()                      # total degree per community
    moved = True
    while moved:
        moved = False
        for i in order:
            ci = lab[i]
            # weights from i to each community, without its self-loop
            links: Dict[int, float] = {}
            for j in np.nonzero(w[i])[0]:
                if j != i:
                    links[lab[j]] = links.get(lab[j], 0.0) + w[i, j]
            tot[ci] -= k[i]
            # gain of inserting i into community d (up to the common factor 1/m):
            # k_{i,d} - tot_d k_i / (2m)
            best, best_gain = ci, links.get(ci, 0.0) - tot[ci] * k[i] / two_m
            for d in sorted(links):
                g = links[d] - tot[d] * k[i] / two_m
                if g > best_gain + 1e-12:
                    best, best_gain = d, g
            tot[best] += k[i]
            if best != ci:
                lab[i] = best
                moved = True
    # renumber 0..K-1 in order of first appearance
    _, lab = np.unique(lab, return_inverse=True)
    return lab


def louvain(w: np.ndarray, seed: int = 0, max_levels: int = 32) -> np.ndarray:
    """Partition maximising modularity (Eq. 10) by the Louvain method: local
    moves, then each community becomes one node of an aggregated graph (its
    internal weight a self-loop), repeated while Q improves.  Node visiting
    order is a seeded permutation.  Returns a label per node."""
    w = np.asarray(w, dtype=np.float64)
    n = w.shape[0]
    if w.sum() <= 0:
        return np.arange(n)
    rng = np.random.default_rng(seed)
    labels = np.arange(n)
    g = w.copy()
    q_best = modularity(w, labels)
    for _ in range(max_levels):
        sub = _local_moves(g, rng.permutation(g.shape[0]))
        if sub.max() + 1 == g.shape[0]:
            break                                   # no node moved
        new_labels = sub[labels]
        q = modularity(w, new_labels)
        if q <= q_best + 1e-12:
            break
        labels, q_best = new_labels, q
        kc = sub.max() + 1
        agg = np.zeros((kc, kc))
        for a in range(g.shape[0]):
            for b in np.nonzero(g[a])[0]:
                agg[sub[a], sub[b]] += g[a, b]
        g = agg
    _, labels = np.unique(labels, return_inverse=True)
    return labels


def merge_small_blocks(w: np.ndarray, labels: Sequence[int], s_min: int) -> np.ndarray:
    """Join every block smaller than s_min to the neighbouring block it shares
    the most edge weight with (smallest block first; ties to the lower label),
    until none is left (Sec. IV-C).  A block with no edges to any other joins
    the smallest other block."""
    lab = np.array(labels)
    while True:
        ids, sizes = np.unique(lab, return_counts=True)
        small = [(s, b) for b, s in zip(ids, sizes) if s < s_min]
        if not small or len(ids) == 1:
            break
        _, b = min(small)
        inside = lab == b
        best, best_w = None, 0.0
        for o in ids:
            if o == b:
                continue
            cw = w[np.ix_(inside, lab == o)].sum()
            if cw > best_w + 1e-15:
                best, best_w = o, cw
        if best is None:
            others = [(s, o) for o, s in zip(ids, sizes) if o != b]
            best = min(others)[1]
        lab[inside] = best
    _, lab = np.unique(lab, return_inverse=True)
    return lab


def blocks_of(labels: Sequence[int]) -> List[List[int]]:
    """Qubit lists per block, ordered by their lowest qubit."""
    lab = np.asarray(labels)
    out = [sorted(np.nonzero(lab == b)[0].tolist()) for b in np.unique(lab)]
    return sorted(out, key=lambda b: b[0])


def qubit_mask(block: Sequence[int]) -> int:
    m = 0
    for q in block:
        m |= 1 << int(q)
    return m


# ----------------------------------------------------------- early stopping

class WindowStopper:
    """Eq. 14: after each new energy E_n, Delta_max = max of |E_t - E_{t-1}|
    over t in [n - W, n] (history indexed from 1); once Delta_max < tol for
    `patience` consecutive checks, ``stop`` becomes true."""

    def __init__(self, tol: float = 1e-4, window: int = 40, patience: int = 12):
        self.tol, self.window, self.patience = tol, window, patience
        self.history: List[float] = []
        self.quiet = 0
        self.stop = False

    def update(self, e: float) -> bool:
        self.history.append(float(e))
        h = self.history
        if len(h) >= 2:
            lo = max(1, len(h) - self.window - 1)   # 0-based index of E_{n-W}
            dmax = max(abs(h[t] - h[t - 1]) for t in range(lo, len(h)))
            self.quiet = self.quiet + 1 if dmax < self.tol else 0
            self.stop = self.quiet >= self.patience
        return self.stop


# ------------------------------------------------------------ the optimiser

class _Converged(Exception):
    pass


class _EvalServer:
    """Collects the energy / gradient requests of the block optimisers (one
    thread each) and answers all pending ones with one batched evaluation
    as soon as every block still running has asked."""

    def __init__(self, nblocks: int, evaluate: Callable):
        self.evaluate = evaluate
        self.alive = set(range(nblocks))
        self.pending: Dict[int, np.ndarray] = {}
        self.results: Dict[int, Tuple[float, np.ndarray]] = {}
        self.cv = threading.Condition()
        self.launches = 0
        self.error: Optional[BaseException] = None

    def request(self, bid: int, theta: np.ndarray):
        with self.cv:
            self.pending[bid] = theta
            self.cv.notify_all()
            while bid not in self.results and self.error is None:
                self.cv.wait()
            if self.error is not None:
                raise RuntimeError("batched evaluation failed") from self.error
            return self.results.pop(bid)

    def done(self, bid: int):
        with self.cv:
            self.alive.discard(bid)
            self.cv.notify_all()

    def serve(self):
        while True:
            with self.cv:
                while self.alive and set(self.pending) != self.alive:
                    self.cv.wait()
                if not self.alive:
                    return
                req = dict(self.pending)
                self.pending.clear()
            try:
                out = self.evaluate(req)
            except BaseException as e:      # wake every block thread, then re-raise
                with self.cv:
                    self.error = e
                    self.cv.notify_all()
                raise
            self.launches += 1
            with self.cv:
                self.results.update(out)
                self.cv.notify_all()


@dataclass
class EpochLog:
    epoch: int
    blocks: List[List[int]]
    modularity: float
    block_energy: float
    global_energy: float
    best_energy: float
    block_launches: int
    global_evals: int


@dataclass
class GraphVQEResult:
    theta: np.ndarray
    energy: float
    history: List[EpochLog] = field(default_factory=list)


class GraphVQE:
    """Graph-VQE on one GPU (Sec. IV).  ``ham``: (n, x, z, c) of the Pauli
    sum; ``ansatz``: a ``gv.Ansatz``.  Energies and gradients come from the
    library in `precision`."""

    def __init__(self, ansatz, x, z, c, precision="c64", s_min: int = 2, seed: int = 0,
                 tol: float = 1e-4, window: int = 40, patience_block: int = 12,
                 patience_global: int = 12, patience_epoch: int = 3, ftol: float = 1e-9,
                 block_maxiter: int = 50, global_maxiter: int = 50, ham_batches: int = 1,
                 device="cuda"):
        import torch

        from . import gv
        self.gv, self.torch = gv, torch
        self.ansatz = ansatz
        self.n = ansatz.n
        self.x = np.asarray(x, dtype=np.uint64)
        self.z = np.asarray(z, dtype=np.uint64)
        self.c = np.asarray(c, dtype=np.float64)
        self.precision = precision
        self.s_min, self.seed = s_min, seed
        self.tol, self.window = tol, window
        self.patience_block, self.patience_global = patience_block, patience_global
        self.patience_epoch = patience_epoch
        self.ftol, self.block_maxiter, self.global_maxiter = ftol, block_maxiter, global_maxiter
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        mode = "store" if self.n <= 26 else "uncompute"
        self.mode = mode
        self.state = gv.State(self.n, precision, "fused", ansatz, mode, device=self.device)
        # Hamiltonian batching (Eq. 12): E is the sum over the term subsets
        parts = np.array_split(np.arange(len(self.c)), max(1, ham_batches))
        self.hams = [gv.PauliSum(self.n, self.x[p], self.z[p], self.c[p]).prepare(self.state)
                     for p in parts if len(p)]
        self.global_evals = 0

    # full energy and gradient (sum over the Hamiltonian batches)
    def energy_grad(self, theta: np.ndarray, mask=None) -> Tuple[float, np.ndarray]:
        th = self.torch.tensor(theta, dtype=self.torch.float64, device=self.device)
        e_tot, g_tot = 0.0, np.zeros(theta.size)
        for h in self.hams:
            e, g = self.gv.energy_grad(self.state, h, th, self.ansatz, mask, self.mode)
            e_tot += e[0].item()
            g_tot += g.cpu().numpy()
        return e_tot, g_tot

    def partition(self) -> Tuple[List[List[int]], float]:
        w = interaction_graph(self.n, self.x, self.z, self.c)
        lab = merge_small_blocks(w, louvain(w, self.seed), self.s_min)
        return blocks_of(lab), modularity(w, lab)

    def _param_index(self, block: Sequence[int]) -> np.ndarray:
        n, R = self.n, self.ansatz.layers + self.ansatz.final_rotation
        return np.array(sorted(l * 2 * n + g * n + q for l in range(R) for g in range(2)
                               for q in block), dtype=np.int64)

    def _block_phase(self, theta0: np.ndarray, blocks: List[List[int]]):
        """Every block minimises E over its own parameters from theta0 (Eq.
        11), concurrently; returns the fused parameters and the server's
        launch count."""
        from scipy.optimize import minimize
        gv, torch = self.gv, self.torch
        nb = len(blocks)
        idx = [self._param_index(b) for b in blocks]
        use_batch = self.n >= 12 and self.ansatz.ent in (gv.ENT_NONE, gv.ENT_CZ_LINEAR,
                                                         gv.ENT_CZ_CIRCULAR)
        thetas = [torch.tensor(theta0, dtype=torch.float64, device=self.device) for _ in blocks]
        batch = None
        if use_batch:
            hb = gv.PauliSum(self.n, self.x, self.z, self.c)
            items = [(self.ansatz, thetas[i], hb, qubit_mask(blocks[i])) for i in range(nb)]
            batch = gv.Batch(items, self.precision, graph=True, device=self.device)
        masks = [gv.param_mask(self.n, self.ansatz.layers, qubit_mask(b),
                               self.ansatz.final_rotation, device=self.device) for b in blocks]

        def evaluate(req: Dict[int, np.ndarray]):
            out = {}
            if batch is not None:
                for bid, th in req.items():
                    thetas[bid].copy_(torch.from_numpy(th))
                batch.run()
                e = batch.energies[:, 0].cpu().numpy()
                for bid in req:
                    out[bid] = (float(e[bid]), batch.grads[bid].cpu().numpy())
            else:
                for bid, th in req.items():
                    thetas[bid].copy_(torch.from_numpy(th))
                    e, g = self.gv.energy_grad(self.state, self.hams[0], thetas[bid],
                                               self.ansatz, masks[bid], self.mode)
                    out[bid] = (e[0].item(), g.cpu().numpy())
            return out

        server = _EvalServer(nb, evaluate) if (batch is not None and len(self.hams) == 1) \
            else None
        results: List[Optional[np.ndarray]] = [None] * nb
        best_e = [np.inf] * nb

        def run_block(bid: int):
            full = theta0.copy()
            stop = WindowStopper(self.tol, self.window, self.patience_block)
            best = {"e": np.inf, "x": theta0[idx[bid]].copy()}

            def fun(xb):
                full[idx[bid]] = xb
                if server is not None:
                    e, g = server.request(bid, full.copy())
                else:
                    e, g = self.energy_grad(full, masks[bid])
                if e < best["e"]:
                    best["e"], best["x"] = e, xb.copy()
                return e, g[idx[bid]]

            def cb(intermediate_result):
                if stop.update(intermediate_result.fun):
                    raise StopIteration

            try:
                minimize(fun, theta0[idx[bid]], jac=True, method="L-BFGS-B", callback=cb,
                         options={"maxiter": self.block_maxiter, "ftol": self.ftol,
                                  "gtol": 0.1 * self.ftol})
            finally:
                if server is not None:
                    server.done(bid)
            results[bid] = best["x"]
            best_e[bid] = best["e"]

        if server is not None:
            threads = [threading.Thread(target=run_block, args=(b,)) for b in range(nb)]
            for t in threads:
                t.start()
            try:
                server.serve()
            finally:
                for t in threads:
                    t.join()
            launches = server.launches
        else:
            for b in range(nb):
                run_block(b)
            launches = 0
        fused = theta0.copy()
        for b in range(nb):
            fused[idx[b]] = results[b]
        return fused, launches

    def _global_phase(self, theta0: np.ndarray) -> Tuple[np.ndarray, float]:
        """L-BFGS-B over all parameters (ftol, gtol = 0.1 ftol), stopped by the
        window criterion with the global patience."""
        from scipy.optimize import minimize
        stop = WindowStopper(self.tol, self.window, self.patience_global)
        best = {"e": np.inf, "x": theta0.copy()}

        def fun(th):
            self.global_evals += 1
            e, g = self.energy_grad(th)
            if e < best["e"]:
                best["e"], best["x"] = e, th.copy()
            return e, g

        def cb(intermediate_result):
            if stop.update(intermediate_result.fun):
                raise StopIteration

        minimize(fun, theta0, jac=True, method="L-BFGS-B", callback=cb,
                 options={"maxiter": self.global_maxiter, "ftol": self.ftol,
                          "gtol": 0.1 * self.ftol})
        return best["x"], best["e"]

    def run(self, theta0: np.ndarray, epochs: int = 10, refine: bool = True) -> GraphVQEResult:
        best_theta = np.asarray(theta0, dtype=np.float64).copy()
        best_e, _ = self.energy_grad(best_theta)
        res = GraphVQEResult(best_theta.copy(), best_e)
        blocks, q = self.partition()
        stale = 0
        for ep in range(epochs):
            start = res.theta.copy()                 # warm start from the best so far
            fused, launches = self._block_phase(start, blocks)
            e_blk, _ = self.energy_grad(fused)
            evals0 = self.global_evals
            if refine:
                theta, e_glb = self._global_phase(fused)
            else:
                theta, e_glb = fused, e_blk
            if e_glb < res.energy - 1e-12:
                res.theta, res.energy = theta.copy(), e_glb
                stale = 0
            else:
                stale += 1
            res.history.append(EpochLog(ep, blocks, q, e_blk, e_glb, res.energy, launches,
                                        self.global_evals - evals0))
            if stale >= self.patience_epoch:
                break
        return res
