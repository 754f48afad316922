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
@pytest.mark.parametrize("edge_only", [False, True])
def test_golden_charts(name, edge_only):
    g = GOLD[name]
    idx = np.array(g["indices"], np.int32)
    V = int(idx.max()) + 1
    cot, cov, roots = oracle.charts(idx, V, np.array(g["visible"], np.uint8), edge_only=edge_only)
    want = g["edge_only"] if edge_only else g
    assert cot.tolist() == want["chart_of_tri"]
    assert roots.tolist() == want["roots"]
    if "chart_of_vert" in want:
        assert cov.tolist() == want["chart_of_vert"]


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


# ---------------------------------------------------------------------------
# edge-connected charts (O3': joined across shared edges only)
# ---------------------------------------------------------------------------
def _brute_edge_charts(idx, V, vis):
    """O(T^2): triangles t, u are adjacent iff they share two distinct vertex
    indices (a shared undirected edge); components by repeated relabelling to
    the smallest label until nothing changes."""
    T = idx.shape[0]
    sets = [set(int(v) for v in idx[t]) for t in range(T)]
    lab = [t if vis[t] else -1 for t in range(T)]
    changed = True
    while changed:
        changed = False
        for t in range(T):
            if not vis[t]:
                continue
            for u in range(T):
                if u != t and vis[u] and len(sets[t] & sets[u]) >= 2 and lab[u] < lab[t]:
                    lab[t] = lab[u]
                    changed = True
    labels = sorted({lab[t] for t in range(T) if vis[t]})
    cidx = {l: i for i, l in enumerate(labels)}
    cot = [cidx[lab[t]] if vis[t] else -1 for t in range(T)]
    cov = [-1] * V
    for t in range(T):
        if vis[t]:
            for v in idx[t]:
                v = int(v)
                cov[v] = cot[t] if cov[v] < 0 else min(cov[v], cot[t])
    return cot, cov, labels


@pytest.mark.parametrize("seed", range(10))
def test_edge_charts_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    T, V = int(rng.integers(5, 70)), int(rng.integers(6, 40))
    idx = _random_mesh(rng, T, V, nonmanifold=bool(seed % 2))
    if seed % 3 == 0:
        idx[2] = [idx[2, 0], idx[2, 0], idx[2, 1]]  # a degenerate triangle
    vis = (rng.uniform(size=T) < 0.7).astype(np.uint8)
    cot, cov, roots = oracle.charts(idx, V, vis, edge_only=True)
    ecot, ecov, eroots = _brute_edge_charts(idx, V, vis)
    assert cot.tolist() == ecot
    assert cov.tolist() == ecov
    assert roots.tolist() == eroots


@pytest.mark.parametrize("maker", [lambda: scenes.grid_frame(3), lambda: scenes.orbit_frame(9)])
def test_edge_charts_refine_vertex_charts(maker):
    # every edge-connected chart lies inside one vertex-merged chart, and on
    # a frame with vertex-only contacts there are strictly more of them
    f = maker()
    cot_v, _, roots_v = oracle.charts(f.indices, f.num_vertices, f.visible)
    cot_e, cov_e, roots_e = oracle.charts(f.indices, f.num_vertices, f.visible, edge_only=True)
    vis = f.visible.astype(bool)
    assert np.array_equal(cot_e >= 0, vis)
    pairs = set(zip(cot_e[vis].tolist(), cot_v[vis].tolist()))
    assert len(pairs) == roots_e.shape[0]          # each edge chart maps to one vertex chart
    assert roots_e.shape[0] >= roots_v.shape[0]
    for c in range(roots_e.shape[0]):
        assert np.nonzero(cot_e == c)[0].min() == roots_e[c]
    # chart_of_vert: the smallest chart among the vertex's visible triangles
    want = np.full(f.num_vertices, np.iinfo(np.int32).max, np.int64)
    for k in range(3):
        np.minimum.at(want, f.indices[vis, k], cot_e[vis])
    want[want == np.iinfo(np.int32).max] = -1
    assert np.array_equal(cov_e, want)


def test_edge_charts_split_checkerboard():
    # a checkerboard of visible quads on the grid: neighbouring quads meet
    # only at corners, so edge-connected charts are single quads (the two
    # triangles of a quad share its diagonal) while vertex merging joins them
    f = scenes.grid_frame(0)
    T = f.num_triangles
    q = np.arange(T) // 2
    i, j = q // 64, q % 64
    vis = (((i + j) % 2) == 0).astype(np.uint8)
    _, _, roots_e = oracle.charts(f.indices, f.num_vertices, vis, edge_only=True)
    _, _, roots_v = oracle.charts(f.indices, f.num_vertices, vis)
    assert roots_e.shape[0] == 64 * 64 // 2
    assert roots_v.shape[0] == 1
