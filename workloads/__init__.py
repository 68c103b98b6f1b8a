"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random structures (graphs, edge weights, angle sets) with NumPy's
PCG64 generator. It holds none of the QAOA arithmetic: no cost function, no state, no
expectation value.

Workload families (the paper evaluates only on freshly drawn random graphs, Sec. 2 and
Sec. 4; MaxCut on random 3-regular graphs is the family of its prior-art comparison, Sec. 1):

* random d-regular graphs by the pairing (configuration) model, redrawn until simple;
* Erdos-Renyi G(n, 1/2) with optional integer edge weights U{lo..hi};
* angle sets beta, gamma ~ U(0, pi), stored per set as [beta_1..beta_p, gamma_1..gamma_p]
  (the angle layout of the paper's first code listing, Sec. 3).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Graph", "random_regular_graph", "erdos_renyi", "random_angles",
    "Workload", "workload", "WORKLOADS",
]


@dataclass
class Graph:
    """Undirected simple graph on vertices 0..n-1; edges sorted with u < v."""
    n: int
    u: np.ndarray          # int32 [m]
    v: np.ndarray          # int32 [m]
    w: np.ndarray          # int32 [m] (all ones when unweighted)

    @property
    def m(self) -> int:
        return int(self.u.size)

    @property
    def total_weight(self) -> int:
        return int(self.w.sum())

    def degrees(self) -> np.ndarray:
        d = np.zeros(self.n, dtype=np.int64)
        np.add.at(d, self.u, 1)
        np.add.at(d, self.v, 1)
        return d


def _edges_to_graph(n: int, edges, weights=None) -> Graph:
    edges = sorted((min(a, b), max(a, b)) for a, b in edges)
    u = np.array([e[0] for e in edges], dtype=np.int32)
    v = np.array([e[1] for e in edges], dtype=np.int32)
    if weights is None:
        w = np.ones(len(edges), dtype=np.int32)
    else:
        w = np.asarray(weights, dtype=np.int32)
    return Graph(n, u, v, w)


def random_regular_graph(n: int, d: int, seed: int, max_tries: int = 10000) -> Graph:
    """Uniform random simple d-regular graph by the pairing model with rejection.

    n*d points (d per vertex) are shuffled and paired consecutively; a pairing with a loop
    or a repeated edge is rejected and redrawn from the same generator.
    """
    if (n * d) % 2 != 0 or d >= n:
        raise ValueError("need n*d even and d < n")
    rng = np.random.default_rng(seed)
    points = np.repeat(np.arange(n), d)
    for _ in range(max_tries):
        perm = rng.permutation(points)
        a, b = perm[0::2], perm[1::2]
        if np.any(a == b):
            continue
        pairs = set()
        ok = True
        for x, y in zip(a.tolist(), b.tolist()):
            e = (min(x, y), max(x, y))
            if e in pairs:
                ok = False
                break
            pairs.add(e)
        if ok:
            return _edges_to_graph(n, pairs)
    raise RuntimeError("pairing model did not produce a simple graph")


def erdos_renyi(n: int, seed: int, prob: float = 0.5, weight_range: Optional[tuple] = None,
                rng: Optional[np.random.Generator] = None) -> Graph:
    """G(n, prob): pairs (i<j) in lexicographic order, each kept with probability prob.

    With weight_range=(lo, hi), integer weights U{lo..hi} are drawn for the kept edges in
    the same order, after all keep decisions.
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.size) < prob
    edges = list(zip(iu[keep].tolist(), ju[keep].tolist()))
    weights = None
    if weight_range is not None:
        lo, hi = weight_range
        weights = rng.integers(lo, hi + 1, size=len(edges))
    return _edges_to_graph(n, edges, weights)


def random_angles(p: int, n_sets: int, seed: int, lo: float = 0.0, hi: float = np.pi) -> np.ndarray:
    """float64 [n_sets, 2p]: row = [beta_1..beta_p, gamma_1..gamma_p], each ~ U(lo, hi)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n_sets, 2 * p))


@dataclass
class Workload:
    """One named workload: graphs, mixer, round count, angle sets."""
    name: str
    description: str
    graphs: List[Graph]
    p: int
    angles: np.ndarray             # [n_sets, 2p]
    mixer: str = "x"               # "x" (transverse field), "clique", "grover", "x_orders", "x_multiangle"
    hamming_k: int = -1            # feasible subspace weight, -1 = all 2^n states
    extra: dict = field(default_factory=dict)


def _maxcut_3reg(n, p, seed, n_sets=1):
    g = random_regular_graph(n, 3, seed)
    return g, random_angles(p, n_sets, seed + 1)


def workload(name: str, n_sets: Optional[int] = None) -> Workload:
    """Build one of the named workloads (seeds fixed here, recipe in the design notes)."""
    if name == "maxcut3reg_n10_p3":
        g, a = _maxcut_3reg(10, 3, 1001)
        return Workload(name, "MaxCut, random 3-regular n=10, X mixer, p=3, one angle set, forward",
                        [g], 3, a)
    if name == "maxcut3reg_n28_p8":
        g, a = _maxcut_3reg(28, 8, 2028)
        return Workload(name, "MaxCut, random 3-regular n=28, X mixer, p=8, fwd+grad",
                        [g], 8, a)
    if name == "batched_er_n12to20_p10":
        rng = np.random.default_rng(3000)
        graphs = []
        for _ in range(8):
            n = int(rng.integers(12, 21))
            graphs.append(erdos_renyi(n, 0, 0.5, (1, 4), rng=rng))
        ns = 256 if n_sets is None else n_sets
        return Workload(name, "8 weighted G(n,1/2) MaxCut, n~U{12..20}, 256 angle sets, p=10, fwd+grad",
                        graphs, 10, random_angles(10, ns, 3001))
    if name == "bisection_g16_k8_p6":
        g = erdos_renyi(16, 4016, 0.5)
        ns = 512 if n_sets is None else n_sets
        return Workload(name, "max-bisection G(16,1/2) on Hamming weight 8, clique mixer, p=6, 512 sets",
                        [g], 6, random_angles(6, ns, 4017), mixer="clique", hamming_k=8)
    if name == "grover_maxcut3reg_n40_p16":
        g, _ = _maxcut_3reg(40, 16, 6040)
        ns = 512 if n_sets is None else n_sets
        return Workload(name, "MaxCut, random 3-regular n=40, Grover mixer (table-free degeneracies), p=16, "
                              "512 sets", [g], 16, random_angles(16, ns, 6041), mixer="grover")
    if name == "angles_er_n12_p10":
        # the angle-finding study of Sec. 2.3: 50 unweighted G(12, 1/2) MaxCut instances, rounds
        # 1..10 of iterative basinhopping; the search draws its own angles (seed in extra)
        graphs = [erdos_renyi(12, 7000 + i, 0.5) for i in range(50 if n_sets is None else n_sets)]
        return Workload(name, "angle finding: 50 MaxCut G(12,1/2) instances, iterative basinhopping to p=10",
                        graphs, 10, np.zeros((0, 20)), extra={"seed": 7100, "n_chains": 8, "n_hops": 10})
    if name == "xorders_maxcut3reg_n24_p4":
        # mixer sum_i X_i + sum_{i<j} X_i X_j (orders 1 and 2, Eq. (2)), 16 angle sets per call
        g, _ = _maxcut_3reg(24, 4, 8024)
        ns = 16 if n_sets is None else n_sets
        return Workload(name, "MaxCut, random 3-regular n=24, mixer of all 1- and 2-body X products, p=4, "
                              "16 sets", [g], 4, random_angles(4, ns, 8025), mixer="x_orders",
                        extra={"orders": [1, 2]})
    if name == "multiangle_maxcut3reg_n24_p4":
        # per-qubit angles (one beta per qubit and layer), 16 angle sets per call; rows
        # [beta_{1,0..n-1}, ..., beta_{p,0..n-1}, gamma_1..gamma_p], each ~ U(0, pi)
        g, _ = _maxcut_3reg(24, 4, 8224)
        ns = 16 if n_sets is None else n_sets
        a = np.random.default_rng(8225).uniform(0.0, np.pi, size=(ns, 4 * (24 + 1)))
        return Workload(name, "MaxCut, random 3-regular n=24, per-qubit multi-angle X mixer, p=4, 16 sets",
                        [g], 4, a, mixer="x_multiangle")
    if name == "maxcut3reg_n32_p16":
        g, a = _maxcut_3reg(32, 16, 5032)
        return Workload(name, "MaxCut, random 3-regular n=32, X mixer, p=16, fwd+grad",
                        [g], 16, a)
    raise KeyError(name)


WORKLOADS = ["maxcut3reg_n10_p3", "maxcut3reg_n28_p8", "batched_er_n12to20_p10",
             "bisection_g16_k8_p6", "maxcut3reg_n32_p16", "grover_maxcut3reg_n40_p16", "angles_er_n12_p10",
             "xorders_maxcut3reg_n24_p4", "multiangle_maxcut3reg_n24_p4"]
