"""Pins for the oracle's packer: sizes, prefix-sum fold, overflow, mirrored
rows, push, selection (CPU only).

* a hand-worked example (tests/golden/fold_push_example.json);
* an independent re-implementation using division/modulo for the fold and a
  painted cell grid for the push (each box rises to just above every cell
  already painted in its columns);
* closed forms for one box, equal boxes and a single row;
* selection against an exhaustive exact-rational search over every j;
* pairwise non-overlap of the final placement.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import scenes

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fold_push_example.json")))
CONST = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "constants.json")))


def test_golden_fold_push():
    g = GOLD
    r = oracle.candidate(np.array(g["bw"], np.float32), np.array(g["bh"], np.float32), g["j"], g["J"],
                         g["omega"], g["gutter"], g["min_box"])
    e = g["expect"]
    assert r["a"].tolist() == e["a"] and r["b"].tolist() == e["b"]
    assert (r["m"], r["L"], r["H"], r["fit"], r["rows"]) == (e["m"], e["L"], e["H"], e["fit"], e["rows"])
    assert r["x"].tolist() == e["x"] and r["y"].tolist() == e["y"]


def painted_candidate(sbw, sbh, j, J, omega, g, mmin):
    """Independent statement of one candidate packing."""
    s = np.float32(j) / np.float32(J)
    a = [max(mmin, math.ceil(float(np.float32(w) * s))) + 2 * g for w in sbw]
    b = [max(mmin, math.ceil(float(np.float32(h) * s))) + 2 * g for h in sbh]
    C = len(a)
    X = [sum(a[:i]) for i in range(C)]
    row = [X[i] // omega for i in range(C)]
    off = [X[i] % omega for i in range(C)]
    m = max([0] + [off[i] + a[i] - omega for i in range(C)])
    L = omega + m
    res = dict(a=a, b=b, m=m, L=L, rows=(row[-1] + 1 if C else 0))
    if m > omega:
        res["fit"] = False
        return res
    x = [off[i] if row[i] % 3 == 0 else L - off[i] - a[i] for i in range(C)]
    top = [0] * L  # one past the highest painted cell per column
    y = [0] * C
    for r in sorted(set(row)):
        members = [i for i in range(C) if row[i] == r]
        for i in members:
            y[i] = max(top[c] for c in range(x[i], x[i] + a[i]))
        for i in members:
            for c in range(x[i], x[i] + a[i]):
                top[c] = max(top[c], y[i] + b[i])
    H = max([0] + [y[i] + b[i] for i in range(C)])
    res.update(x=x, y=y, H=H, fit=H <= L)
    return res


def _random_boxes(rng, C, omega, heavy=False):
    hi = omega * (1.5 if heavy else 0.4)
    w = rng.uniform(0, hi, C).astype(np.float32)
    h = rng.uniform(0, hi, C).astype(np.float32)
    bw, bh = np.minimum(w, h), np.maximum(w, h)
    key = np.minimum(np.ceil(bh).astype(np.int64), 8191)
    o = sorted(range(C), key=lambda c: (-key[c], c))
    return bw[o], bh[o]


@pytest.mark.parametrize("seed", range(12))
def test_candidate_matches_painted_grid(seed):
    rng = np.random.default_rng(seed)
    omega = [16, 32, 64][seed % 3]
    g = seed % 2
    C = int(rng.integers(1, 30))
    bw, bh = _random_boxes(rng, C, omega, heavy=seed % 4 == 3)
    J = [4, 16, 64][seed % 3]
    for j in range(1, J + 1, max(1, J // 8)):
        got = oracle.candidate(bw, bh, j, J, omega, g, 2)
        want = painted_candidate(bw, bh, j, J, omega, g, 2)
        assert got["a"].tolist() == want["a"] and got["b"].tolist() == want["b"]
        assert (got["m"], got["L"], got["rows"], got["fit"]) == (want["m"], want["L"], want["rows"], want["fit"])
        if "x" in want:
            assert got["x"].tolist() == want["x"] and got["y"].tolist() == want["y"]
            assert got["H"] == want["H"]


def _overlap(b1, b2):
    (x1, y1, a1, h1), (x2, y2, a2, h2) = b1, b2
    return x1 < x2 + a2 and x2 < x1 + a1 and y1 < y2 + h2 and y2 < y1 + h1


@pytest.mark.parametrize("seed", range(6))
def test_fitting_layout_has_no_overlap(seed):
    rng = np.random.default_rng(50 + seed)
    omega = 64
    C = int(rng.integers(2, 60))
    bw, bh = _random_boxes(rng, C, omega)
    for j in (8, 16, 32, 64):
        r = oracle.candidate(bw, bh, j, 64, omega, 1, 2)
        if not r["fit"]:
            continue
        boxes = list(zip(r["x"], r["y"], r["a"], r["b"]))
        for (p, q) in itertools.combinations(boxes, 2):
            assert not _overlap(p, q)
        for (x, y, a, b) in boxes:
            assert 0 <= x and x + a <= r["L"] and 0 <= y and y + b <= r["L"]


def test_closed_form_single_box():
    omega = 64
    for (w, h) in [(10.0, 20.0), (62.0, 62.0), (63.0, 10.0), (1.0, 1.0)]:
        bw, bh = min(w, h), max(w, h)
        r = oracle.candidate(np.array([bw], np.float32), np.array([bh], np.float32), 64, 64, omega, 0, 2)
        a, b = max(2, math.ceil(bw)), max(2, math.ceil(bh))
        assert (r["x"][0], r["y"][0]) == (0, 0)
        assert r["m"] == max(0, a - omega) and r["H"] == b
        assert r["fit"] == (a <= omega and b <= omega)


def test_closed_form_equal_boxes_grid():
    # n boxes of side s dividing omega: rows of omega/s boxes stacked exactly,
    # right-to-left rows flush right
    omega, side, n = 64, 8, 40
    r = oracle.candidate(np.full(n, side, np.float32), np.full(n, side, np.float32), 1, 1, omega, 0, 2)
    per = omega // side
    assert r["m"] == 0 and r["L"] == omega
    for i in range(n):
        row, k = divmod(i, per)
        col = k if row % 3 == 0 else per - 1 - k
        assert (r["x"][i], r["y"][i]) == (col * side, row * side)
    assert r["H"] == side * math.ceil(n / per) and r["fit"]


def test_closed_form_single_row():
    omega = 128
    bw = np.array([10, 9, 7, 5, 3], np.float32)
    bh = np.array([30, 20, 10, 6, 4], np.float32)
    r = oracle.candidate(bw, bh, 64, 64, omega, 1, 2)
    assert r["rows"] == 1 and r["m"] == 0 and (r["y"] == 0).all()
    assert r["x"].tolist() == np.concatenate([[0], np.cumsum(r["a"])[:-1]]).tolist()
    assert r["H"] == 32 and r["fit"]


def test_select_exhaustive():
    rng = np.random.default_rng(9)
    for trial in range(200):
        J = int(rng.integers(1, 70))
        table = np.zeros((J, 5), np.int64)
        for j in range(J):
            fit = rng.uniform() < 0.6
            L = int(rng.integers(64, 128))
            table[j] = [fit, L - 64, L, 0, 1]
        got = oracle.select(table)
        best = None
        for j in range(1, J + 1):
            if table[j - 1, 0]:
                eff = Fraction(j, table[j - 1, 2])
                if best is None or eff >= best[0]:
                    best = (eff, j)
        assert got == (best[1] if best else 0)


def test_constants_and_scale_set():
    # 64 candidate scales j/64, j = 1..64, all evaluated
    f = scenes.grid_frame(1)
    r = oracle.build_frame(f, J=CONST["num_scales"], want_occupancy=False)
    assert r["cand"].shape == (CONST["num_scales"], 5)
    key = r["key"]
    assert key.max() <= CONST["max_height"] - 1


@pytest.mark.parametrize("seed", [0, 7])
def test_selected_layout_full_path(seed):
    f = scenes.grid_frame(seed, atlas_size=256, rate=1.0)
    r = oracle.build_frame(f, want_occupancy=False)
    assert r["status"] == 0
    js = r["jstar"]
    # the chosen scale is the best fitting one
    effs = [(Fraction(j, int(r["cand"][j - 1, 2])), j) for j in range(1, 65) if r["cand"][j - 1, 0]]
    assert max(effs)[1] == js or max(effs)[0] == Fraction(js, r["L"])
    boxes = list(zip(r["x"], r["y"], r["a"], r["b"]))
    for (p, q) in itertools.combinations(boxes, 2):
        assert not _overlap(p, q)


def test_optimality_gap_report(capsys):
    """Report (not gated) how far the heuristic's scale is from the best
    uniform scale that admits any non-overlapping placement, on <= 4 boxes."""
    rng = np.random.default_rng(11)
    omega, J = 16, 16
    gaps = []
    for _ in range(8):
        C = int(rng.integers(1, 5))
        bw, bh = _random_boxes(rng, C, omega)
        cand = np.zeros((J, 5), np.int64)
        for j in range(1, J + 1):
            r = oracle.candidate(bw, bh, j, J, omega, 0, 2)
            cand[j - 1] = [r["fit"], r["m"], r["L"], r["H"], r["rows"]]
        js = oracle.select(cand)
        ours = Fraction(js, J) * Fraction(omega, int(cand[js - 1, 2])) if js else Fraction(0)
        best = Fraction(0)
        for j in range(J, 0, -1):
            s = np.float32(j) / np.float32(J)
            a = [max(2, math.ceil(float(np.float32(w) * s))) for w in bw]
            b = [max(2, math.ceil(float(np.float32(h) * s))) for h in bh]
            if _exhaustive_fits(a, b, omega):
                best = Fraction(j, J)
                break
        gaps.append(float(best - ours))
    print("optimality gap (best uniform scale - chosen):", gaps)


def _exhaustive_fits(a, b, omega):
    """Any non-overlapping placement (either orientation) inside omega^2?
    A feasible packing can be slid left/down until every box touches a wall
    or another box, so positions from {0} U {far edges of placed boxes}
    suffice."""
    C = len(a)
    placed = []

    def free(x, y, w, h):
        if x + w > omega or y + h > omega:
            return False
        return all(not _overlap((x, y, w, h), p) for p in placed)

    def rec(i):
        if i == C:
            return True
        xs = {0} | {p[0] + p[2] for p in placed}
        ys = {0} | {p[1] + p[3] for p in placed}
        for (w, h) in {(a[i], b[i]), (b[i], a[i])}:
            for y in sorted(ys):
                for x in sorted(xs):
                    if free(x, y, w, h):
                        placed.append((x, y, w, h))
                        if rec(i + 1):
                            return True
                        placed.pop()
        return False
    return rec(0)
