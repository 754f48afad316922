"""Pins for the oracle's adjacency and chart steps (CPU only).

The chart definition (Sec. "Chart Computation", Appendix "GPU Union Find",
Alg. 1) is checked against hand-worked fixtures and against an independent
disjoint-set union over the shared-vertex relation; adjacency against an
O(T^2) brute-force twin search.
"""
import json
import os

import numpy as np
import pytest

import oracle
from synth import scenes

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "small_meshes.json")))


def test_golden_adjacency_quad():
    q = GOLD["quad"]
    nbr = oracle.adjacency(np.array(q["indices"], np.int32))
    assert nbr.tolist() == q["nbr"]


@pytest.mark.parametrize("name", ["bowtie", "checker_2x2", "two_islands"])
def test_golden_charts(name):
    g = GOLD[name]
    idx = np.array(g["indices"], np.int32)
    V = int(idx.max()) + 1
    cot, cov, roots = oracle.charts(idx, V, np.array(g["visible"], np.uint8))
    assert cot.tolist() == g["chart_of_tri"]
    assert roots.tolist() == g["roots"]
    if "chart_of_vert" in g:
        assert cov.tolist() == g["chart_of_vert"]


def _brute_adjacency(idx):
    T = idx.shape[0]
    hes = []
    for t in range(T):
        for e in range(3):
            a, b = int(idx[t, e]), int(idx[t, (e + 1) % 3])
            hes.append((t, e, a, b))
    nbr = -np.ones((T, 3), np.int64)
    for (t, e, a, b) in hes:
        if a == b:
            continue
        same = sorted(3 * u + f for (u, f, c, d) in hes if c != d and {c, d} == {a, b})
        if len(same) < 2:
            continue
        k = same.index(3 * t + e)
        nbr[t, e] = same[(k + 1) % len(same)] // 3
    return nbr


def _random_mesh(rng, T, V, nonmanifold=True):
    idx = rng.integers(0, V, size=(T, 3)).astype(np.int32)
    if nonmanifold:  # force some shared edges and fans
        for t in range(1, T, 3):
            idx[t, 0], idx[t, 1] = idx[t - 1, 1], idx[t - 1, 0]
    return idx


@pytest.mark.parametrize("seed", range(6))
def test_adjacency_bruteforce(seed):
    rng = np.random.default_rng(seed)
    idx = _random_mesh(rng, 40, 12)
    assert np.array_equal(oracle.adjacency(idx), _brute_adjacency(idx))


def test_adjacency_grid_is_manifold():
    f = scenes.grid_frame(0)
    nbr = oracle.adjacency(f.indices)
    # twins are mutual on a manifold grid and boundary edges are exactly the rim
    T = f.num_triangles
    for t in range(0, T, 97):
        for e in range(3):
            u = nbr[t, e]
            if u >= 0:
                assert t in nbr[u]
    assert int((nbr < 0).sum()) == 4 * 64


class _DSU:
    def __init__(self, n):
        self.p = list(range(n))

    def find(self, x):
        while self.p[x] != x:
            self.p[x] = self.p[self.p[x]]
            x = self.p[x]
        return x

    def union(self, a, b):
        a, b = self.find(a), self.find(b)
        if a != b:
            self.p[max(a, b)] = min(a, b)


def _dsu_charts(idx, V, vis):
    T = idx.shape[0]
    d = _DSU(T)
    first = {}
    for t in range(T):
        if not vis[t]:
            continue
        for v in idx[t]:
            v = int(v)
            if v in first:
                d.union(first[v], t)
            else:
                first[v] = t
    labels = sorted({d.find(t) for t in range(T) if vis[t]})
    cidx = {l: i for i, l in enumerate(labels)}
    cot = [cidx[d.find(t)] if vis[t] else -1 for t in range(T)]
    cov = [-1] * V
    for t in range(T):
        if vis[t]:
            for v in idx[t]:
                cov[int(v)] = cot[t]
    return cot, cov, labels


@pytest.mark.parametrize("seed", range(10))
def test_charts_match_union_find(seed):
    rng = np.random.default_rng(100 + seed)
    T, V = int(rng.integers(5, 80)), int(rng.integers(6, 60))
    idx = _random_mesh(rng, T, V, nonmanifold=bool(seed % 2))
    vis = (rng.uniform(size=T) < 0.6).astype(np.uint8)
    cot, cov, roots = oracle.charts(idx, V, vis)
    ecot, ecov, eroots = _dsu_charts(idx, V, vis)
    assert cot.tolist() == ecot
    assert cov.tolist() == ecov
    assert roots.tolist() == eroots


def test_charts_grid_frame_invariants():
    f = scenes.grid_frame(3)
    cot, cov, roots = oracle.charts(f.indices, f.num_vertices, f.visible)
    vis = f.visible.astype(bool)
    assert (cot[~vis] == -1).all() and (cot[vis] >= 0).all()
    C = roots.shape[0]
    # label of each chart = its minimum triangle, and labels ascend with chart index
    for c in range(C):
        assert np.nonzero(cot == c)[0].min() == roots[c]
    assert (np.diff(roots) > 0).all()
    # each vertex of a visible triangle has that triangle's chart
    for k in range(3):
        assert (cov[f.indices[vis, k]] == cot[vis]).all()
    used = np.zeros(f.num_vertices, bool)
    used[f.indices[vis].ravel()] = True
    assert (cov[~used] == -1).all()
