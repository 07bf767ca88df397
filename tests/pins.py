"""Pins of the oracle: checks against what the paper and the mathematics fix.

Every check takes an ``oracle.Oracle`` instance so that ``test_oracle_mutants``
can run the same pins against deliberately broken builds of the oracle and show
that each plausible mistake fails at least one of them.  None of these checks
retypes the oracle's formulas: they use hand-worked values, brute-force
enumeration of all seams (the definition of the minimum seam, Alg. 1), closed
forms and invariants of the method.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def py_brute_seam(E):
    """Enumerate every connected top-to-bottom seam (sec. 'Seam Identification':
    a path moving at most one column per row) and return the minimum of the key
    (cost, s[H-1], s[H-2], ..., s[0]): the cheapest seam, ties resolved by the
    leftmost column at the bottom, then the leftmost one row up, and so on.
    Pure Python; tiny maps only."""
    E = np.asarray(E)
    H, W = E.shape
    best = None
    for start in range(W):
        for moves in itertools.product((-1, 0, 1), repeat=H - 1):
            path = [start]
            ok = True
            for mv in moves:
                c = path[-1] + mv
                if c < 0 or c >= W:
                    ok = False
                    break
                path.append(c)
            if not ok:
                continue
            cost = int(sum(int(E[H - 1 - t, path[t]]) for t in range(H)))
            key = (cost, tuple(path))
            if best is None or key < best:
                best = key
    cost, path = best
    return np.array(path[::-1], np.int32), cost


def tiny_cases(n, seed):
    """Random tiny energy maps, many with tie-heavy alphabets."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(n):
        H = int(rng.integers(1, 7))
        W = int(rng.integers(1, 7))
        alpha = [2, 3, 4, 10, 1000][t % 5]
        out.append(rng.integers(0, alpha, size=(H, W)).astype(np.int32))
    return out


def check_seam_valid(seam, H, w):
    assert seam.shape == (H,)
    assert np.all(seam >= 0) and np.all(seam < w), "seam leaves the image"
    if H > 1:
        assert np.all(np.abs(np.diff(seam.astype(np.int64))) <= 1), "seam not 8-connected"


# ---------------------------------------------------------------- hand-worked
def pin_hand_grids(o):
    g = load_golden("hand_grids.json")
    for case in g["energy_grids"]:
        E = np.array(case["E"], np.int32)
        seam, cost, M, D = o.dp_seam(E, full=True)
        assert M.tolist() == case["M"], case["name"]
        assert seam.tolist() == case["seam"], case["name"]
        assert cost == case["cost"], case["name"]
        gs, gc = o.greedy_seam(E)
        assert gs.tolist() == case["greedy_seam"], case["name"]
        assert gc == case["greedy_cost"], case["name"]
        bs, bc = o.brute_seam(E)
        assert bs.tolist() == case["seam"] and bc == case["cost"], case["name"]


def pin_pixel_grid(o):
    g = load_golden("hand_grids.json")
    for case in g["pixel_grids"]:
        grey = np.array(case["grey"], np.uint8)
        img = np.repeat(grey[:, :, None], case["channels"], axis=2)
        e = o.energy(img)
        assert e.tolist() == case["energy"], case["name"]
        seam, cost, M, _ = o.dp_seam(e, full=True)
        assert M.tolist() == case["M"], case["name"]
        assert seam.tolist() == case["seam"] and cost == case["cost"], case["name"]
        out = o.remove_seam(img, seam)
        assert out[:, :, 0].tolist() == case["grey_after_one_seam"], case["name"]
        assert np.all(out == out[:, :, :1]), case["name"]
        assert o.energy(out).tolist() == case["energy_after_one_seam"], case["name"]
        out2, seams, costs = o.carve(img, img.shape[1] - 1)
        assert np.array_equal(out2, out) and seams[0].tolist() == case["seam"] and costs[0] == case["cost"]


# --------------------------------------------------------------- brute force
def pin_bruteforce(o, n=300, seed=11):
    for E in tiny_cases(n, seed):
        ps, pc = py_brute_seam(E)
        seam, cost = o.dp_seam(E)
        assert seam.tolist() == ps.tolist() and cost == pc, (E.tolist(), seam, ps)
        bs, bc = o.brute_seam(E)
        assert bs.tolist() == ps.tolist() and bc == pc, (E.tolist(), bs, ps)


def pin_bruteforce_large(o, sizes=((12, 12), (10, 12), (12, 9), (8, 11)), seed=12):
    """DP == exhaustive enumeration up to the paper's largest brute-force size (12x12)."""
    rng = np.random.default_rng(seed)
    for (H, W) in sizes:
        for alpha in (3, 50, 2000):
            E = rng.integers(0, alpha, size=(H, W)).astype(np.int32)
            assert _same(o.dp_seam(E), o.brute_seam(E)), (H, W, alpha)


def _same(a, b):
    return a[0].tolist() == b[0].tolist() and a[1] == b[1]


# -------------------------------------------------------------- closed forms
def pin_energy_closed_forms(o):
    rng = np.random.default_rng(5)
    # constant image: zero energy
    for (H, W, C) in [(1, 1, 3), (5, 7, 3), (4, 1, 1), (1, 6, 4)]:
        img = np.full((H, W, C), int(rng.integers(0, 256)), np.uint8)
        assert np.all(o.energy(img) == 0)
    # horizontal ramp I(y,x,c) = x: central difference 2 inside, one-sided 1 at the clamped edges
    for (H, W, C) in [(3, 2, 3), (4, 9, 3), (2, 5, 1), (1, 3, 4)]:
        img = np.broadcast_to(np.arange(W, dtype=np.uint8)[None, :, None], (H, W, C)).copy()
        row = [C * (1 if (x == 0 or x == W - 1) else 2) for x in range(W)]
        if W == 1:
            row = [0]
        assert o.energy(img).tolist() == [row] * H
    # vertical ramp I(y,x,c) = 3y
    H, W, C = 6, 4, 2
    img = np.broadcast_to((3 * np.arange(H, dtype=np.uint8))[:, None, None], (H, W, C)).copy()
    col = [C * 3 * (1 if (y == 0 or y == H - 1) else 2) for y in range(H)]
    assert o.energy(img).tolist() == [[v] * W for v in col]
    # anti-diagonal ramp I = 50 + 5x - 5y: the x and y differences have opposite signs, the energy
    # adds their magnitudes: 10 per axis inside, 5 per axis at a clamped edge
    H, W, C = 5, 6, 3
    yy, xx = np.mgrid[0:H, 0:W]
    img = np.repeat((50 + 5 * xx - 5 * yy).astype(np.uint8)[:, :, None], C, axis=2)
    ax = lambda n, i: 5 if (i == 0 or i == n - 1) else 10  # noqa: E731
    assert o.energy(img).tolist() == [[C * (ax(W, x) + ax(H, y)) for x in range(W)] for y in range(H)]
    # a single bright pixel (value v) in channel 1 of a zero image, at an interior point and a corner
    H, W, C, v = 5, 6, 3, 200
    img = np.zeros((H, W, C), np.uint8)
    img[2, 3, 1] = v
    exp = np.zeros((H, W), np.int64)
    exp[2, 2] = exp[2, 4] = exp[1, 3] = exp[3, 3] = v
    assert np.array_equal(o.energy(img), exp)
    img = np.zeros((H, W, C), np.uint8)
    img[0, 0, 2] = v
    exp = np.zeros((H, W), np.int64)
    exp[0, 0] = 2 * v      # both one-sided differences at the corner see the pixel itself
    exp[0, 1] = v          # central x-difference at (0,1) reaches back to (0,0)
    exp[1, 0] = v          # central y-difference at (1,0) reaches up to (0,0)
    assert np.array_equal(o.energy(img), exp)


def pin_energy_symmetry(o):
    """The e1 stencil treats x and y alike: energy(I^T) == energy(I)^T."""
    rng = np.random.default_rng(6)
    for (H, W, C) in [(7, 11, 3), (1, 9, 3), (13, 2, 4), (16, 16, 1)]:
        img = rng.integers(0, 256, size=(H, W, C), dtype=np.uint8)
        assert np.array_equal(o.energy(o.transpose(img)), o.energy(img).T)
        assert np.array_equal(o.transpose(img), np.transpose(img, (1, 0, 2)))


def pin_carve_closed_forms(o):
    # constant image: every seam is column 0 with cost 0; the output is the left part
    img = np.full((6, 9, 3), 77, np.uint8)
    out, seams, costs = o.carve(img, 4)
    assert np.all(seams == 0) and np.all(costs == 0) and np.array_equal(out, img[:, :4])
    # horizontal ramp I = x: energy row [3,6,...,6,3]; column 0 ties with the last column, leftmost wins,
    # the remaining image is again a ramp, so every seam is column 0 with cost 3H and the output is I[:, k:]
    H, W = 5, 12
    img = np.broadcast_to(np.arange(W, dtype=np.uint8)[None, :, None], (H, W, 3)).copy()
    out, seams, costs = o.carve(img, 7)
    assert np.all(seams == 0) and np.all(costs == 3 * H) and np.array_equal(out, img[:, 5:])
    # H == 1: the seam is the leftmost argmin of the single energy row
    rng = np.random.default_rng(7)
    for _ in range(20):
        img = rng.integers(0, 4, size=(1, 8, 3), dtype=np.uint8)
        e = o.energy(img)
        seam, cost = o.dp_seam(e)
        assert seam[0] == int(np.argmin(e[0])) and cost == int(e[0].min())
    # target_w == W is the identity
    img = rng.integers(0, 256, size=(4, 5, 3), dtype=np.uint8)
    out, seams, costs = o.carve(img, 5)
    assert np.array_equal(out, img) and seams.shape == (0, 4)


# ---------------------------------------------------------------- invariants
def carve_invariants(o, img, target_w, check_brute=False):
    """Run the carve seam by seam and check every invariant of the method on each seam."""
    out, seams, costs = o.carve(img, target_w)
    cur = img.copy()
    H = img.shape[0]
    for k in range(seams.shape[0]):
        w = cur.shape[1]
        e = o.energy(cur)
        s = seams[k]
        check_seam_valid(s, H, w)
        assert costs[k] == int(e[np.arange(H), s].sum()), "cost != sum of energy on the seam"
        assert (s.tolist(), int(costs[k])) == (lambda r: (r[0].tolist(), r[1]))(o.dp_seam(e))
        _, gc = o.greedy_seam(e)
        assert costs[k] <= gc, "DP seam dearer than the greedy seam"
        if check_brute:
            bs, bc = py_brute_seam(e)
            assert s.tolist() == bs.tolist() and costs[k] == bc
        nxt = np.stack([np.delete(cur[i], s[i], axis=0) for i in range(H)])
        # band property: after removing s, the energy changes only at new columns s_i-1 and s_i
        e2 = o.energy(nxt)
        for i in range(H):
            for x in range(w - 1):
                if x in (s[i] - 1, s[i]):
                    continue
                assert e2[i, x] == e[i, x + (1 if x >= s[i] else 0)], ("band", k, i, x)
        cur = nxt
    assert np.array_equal(out, cur), "carved image != input with the seams deleted"
    return seams, costs


def pin_carve_invariants(o):
    rng = np.random.default_rng(8)
    for (H, W, C, tw) in [(9, 13, 3, 6), (1, 7, 3, 2), (8, 1, 3, 1), (6, 6, 1, 1), (5, 10, 4, 3)]:
        for alpha in (2, 256):
            img = rng.integers(0, alpha, size=(H, W, C), dtype=np.uint8)
            carve_invariants(o, img, tw)


def pin_carve_hv(o):
    rng = np.random.default_rng(9)
    img = rng.integers(0, 5, size=(9, 11, 3), dtype=np.uint8)
    out, vs, vc, hs, hc = o.carve_hv(img, 7, 5)
    a, s1, c1 = o.carve(img, 7)
    t, s2, c2 = o.carve(np.transpose(a, (1, 0, 2)).copy(), 5)
    assert np.array_equal(out, np.transpose(t, (1, 0, 2)))
    assert np.array_equal(vs, s1) and np.array_equal(vc, c1) and np.array_equal(hs, s2) and np.array_equal(hc, c2)
    out, vs, vc, hs, hc = o.carve_hv(img, 8, 9)
    assert np.array_equal(out, o.carve(img, 8)[0]) and hs.shape == (0, 8)


ALL_PINS = [pin_hand_grids, pin_pixel_grid, pin_bruteforce, pin_energy_closed_forms, pin_energy_symmetry,
            pin_carve_closed_forms, pin_carve_invariants, pin_carve_hv]


# --------------------------------------------------------------------------------------------
# Seam insertion (sec. "Image Enlargement"; readings R15, R16)

def py_insert_sequential(img, seams_cur):
    """The paper's process, written independently of the oracle: the recorded seams are inserted
    one by one in removal order, each next to its own pixels.  A seam's pixel in a row is found by
    replaying the removals on a list of original columns; the growing row is a list of (original
    column, value) entries searched for that pixel, and the new entry goes right after it with
    (a + b + 1) >> 1 of the pixel and the entry that follows it (the pixel itself at the right
    border).  (Shifting every later seam by 2 at or right of each inserted one, a common shortcut,
    compares columns of different frames and misplaces crossing seams.)"""
    H, W, C = img.shape
    out = []
    for r in range(H):
        alive = list(range(W))
        pixels = [alive.pop(int(s[r])) for s in seams_cur]  # the seams' original columns, in order
        row = [(x, [int(v) for v in img[r, x]]) for x in range(W)]
        for x in pixels:
            at = next(i for i, (ox, _) in enumerate(row) if ox == x)
            a = row[at][1]
            b = row[at + 1][1] if at + 1 < len(row) else a
            row.insert(at + 1, (None, [(p + q + 1) >> 1 for p, q in zip(a, b)]))
        out.append([v for _, v in row])
    return np.array(out, dtype=np.uint8).reshape(H, W + len(seams_cur), C)


def insert_invariants(o, img, k, out, orig, seams_cur):
    """Width, recovery of the original by deleting the new pixels, the averaging rule, distinct
    original columns, and that deleting those columns in order reproduces the carve's seams."""
    H, W, C = img.shape
    assert out.shape == (H, W + k, C)
    assert orig.shape == (k, H)
    for r in range(H):
        cols = sorted(int(c) for c in orig[:, r])
        assert len(set(cols)) == k and all(0 <= c < W for c in cols)
        keep, new, p, mark = [], [], 0, set(cols)
        for x in range(W):
            keep.append(p)
            p += 1
            if x in mark:
                new.append((p, x))
                p += 1
        assert np.array_equal(out[r, keep], img[r]), "deleting the new pixels must give the original"
        for pos, x in new:
            a = img[r, x].astype(int)
            b = img[r, min(x + 1, W - 1)].astype(int)
            assert np.array_equal(out[r, pos], ((a + b + 1) >> 1).astype(np.uint8))
        idx = list(range(W))
        for j in range(k):
            s = idx.index(int(orig[j, r]))
            assert s == int(seams_cur[j, r]), "original columns must map back to the carve's seams"
            idx.pop(s)


def _seams_of(o, img, k):
    H = img.shape[0]
    return o.carve(img, img.shape[1] - k)[1] if k else np.zeros((0, H), np.int32)


def pin_insert_hand_grids(o):
    for c in load_golden("insert_grids.json")["cases"]:
        img = np.array(c["img"], dtype=np.uint8)
        out, orig = o.insert_seams(img, c["k"])
        assert np.array_equal(orig, np.array(c["orig"], dtype=np.int32)), c["name"]
        assert np.array_equal(out, np.array(c["out"], dtype=np.uint8)), c["name"]


def pin_insert_sequential_and_invariants(o, n=40, seed=17):
    rng = np.random.default_rng(seed)
    for t in range(n):
        H, W = int(rng.integers(1, 9)), int(rng.integers(2, 13))
        C = int(rng.choice([1, 3, 4]))
        alpha = int(rng.choice([2, 4, 256]))
        img = rng.integers(0, alpha, size=(H, W, C), dtype=np.uint8)
        k = int(rng.integers(0, W))
        out, orig = o.insert_seams(img, k)
        seams_cur = _seams_of(o, img, k)
        assert np.array_equal(out, py_insert_sequential(img, seams_cur)), (t, H, W, C, k)
        insert_invariants(o, img, k, out, orig, seams_cur)


def pin_insert_edges(o):
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, size=(6, 9, 3), dtype=np.uint8)
    out, orig = o.insert_seams(img, 0)
    assert np.array_equal(out, img) and orig.shape == (0, 6)
    out, orig = o.insert_seams(img, 8)  # k = W - 1: every pixel but one gets a new neighbour
    insert_invariants(o, img, 8, out, orig, _seams_of(o, img, 8))
    const = np.full((5, 7, 3), 77, np.uint8)  # constant image: zero energy, seams at columns 0, 1, 2
    out, orig = o.insert_seams(const, 3)
    assert np.array_equal(orig, np.array([[0] * 5, [1] * 5, [2] * 5], np.int32))
    assert (out == 77).all() and out.shape == (5, 10, 3)


ALL_PINS += [pin_insert_hand_grids, pin_insert_sequential_and_invariants, pin_insert_edges]


# --------------------------------------------------------------------------------------------
# Forward energy (sec. "Forward Energy Calculation"; readings R17-R19)


def _pair_diff(img, a, b):
    """D of R17: sum over channels of |I(a) - I(b)|."""
    return int(np.abs(img[a].astype(np.int64) - img[b].astype(np.int64)).sum())


def py_forward_cost_by_removal(img, seam):
    """Forward cost of removing `seam` from img, from the definition rather than the DP's cases:
    delete the seam, keep the original coordinates of every remaining pixel, and sum D over each
    pair that is adjacent in the result (left-right or up-down) but was not adjacent in img.  A
    seam pixel on the border of its row is charged against the pixel that becomes the border (R18).
    """
    img = np.asarray(img)
    H, W = img.shape[:2]
    rows = [[x for x in range(W) if x != seam[i]] for i in range(H)]
    cost = 0
    for i in range(H):
        row = rows[i]
        for x in range(len(row) - 1):
            if row[x + 1] != row[x] + 1:
                cost += _pair_diff(img, (i, row[x]), (i, row[x + 1]))
        if W > 1 and seam[i] in (0, W - 1):
            cost += _pair_diff(img, (i, seam[i]), (i, 1 if seam[i] == 0 else W - 2))
        if i > 0:
            up = rows[i - 1]
            for x in range(len(row)):
                if up[x] != row[x]:
                    cost += _pair_diff(img, (i - 1, up[x]), (i, row[x]))
    return cost


def py_brute_forward(img):
    """Every connected seam, costed by py_forward_cost_by_removal; the minimum of the key
    (cost, s[H-1], ..., s[0]) as for the e1 seam (R5, R6).  Tiny images only."""
    H, W = img.shape[:2]
    best = None
    for start in range(W):
        for moves in itertools.product((-1, 0, 1), repeat=H - 1):
            path = [start]
            for mv in moves:
                path.append(path[-1] + mv)
            if min(path) < 0 or max(path) >= W:
                continue
            key = (py_forward_cost_by_removal(img, path[::-1]), tuple(path))
            if best is None or key < best:
                best = key
    cost, path = best
    return np.array(path[::-1], np.int32), cost


def pin_forward_hand_grids(o):
    """Grids worked by hand (the M tables, directions, seam and cost in the golden file)."""
    for g in load_golden("forward_grids.json")["grids"]:
        img = np.array(g["image"], np.uint8)
        seam, cost, M, D = o.forward_seam(img, full=True)
        assert M.tolist() == g["M"], g["name"]
        assert D[1:].tolist() == g["D"][1:], g["name"]
        assert seam.tolist() == g["seam"] and cost == g["cost"], g["name"]


def pin_forward_bruteforce(o, n=160, seed=21):
    """DP seam == the exhaustive minimum under the removal-defined cost (tie-heavy inputs)."""
    rng = np.random.default_rng(seed)
    for t in range(n):
        H = int(rng.integers(1, 5))
        W = int(rng.integers(1, 6))
        C = int(rng.integers(1, 5))
        alpha = [2, 3, 5, 256][t % 4]
        img = rng.integers(0, alpha, size=(H, W, C), dtype=np.uint8)
        seam, cost = o.forward_seam(img)
        bs, bc = py_brute_forward(img)
        assert (seam.tolist(), cost) == (bs.tolist(), bc), (t, img.tolist())


def pin_forward_closed_forms(o):
    rng = np.random.default_rng(22)
    # constant image: every removal creates pairs of equal pixels
    img = np.full((5, 8, 3), 40, np.uint8)
    out, seams, costs = o.carve_forward(img, 3)
    assert np.all(seams == 0) and np.all(costs == 0) and np.array_equal(out, img[:, :3])
    # identical rows: vertical pairs of a straight seam are old pairs, so the cheapest seam is the
    # straight one at the leftmost minimum of the row's horizontal cost, and it costs H times that
    for _ in range(20):
        H, W, C = int(rng.integers(1, 7)), int(rng.integers(2, 9)), int(rng.integers(1, 5))
        row = rng.integers(0, 6, size=(1, W, C), dtype=np.uint8)
        img = np.repeat(row, H, axis=0)
        cu = [_pair_diff(row[0], max(j - 1, 0), min(j + 1, W - 1)) for j in range(W)]
        seam, cost = o.forward_seam(img)
        assert seam.tolist() == [int(np.argmin(cu))] * H and cost == H * min(cu), (row.tolist(), cu)
    # one row: the leftmost minimum of CU
    for _ in range(20):
        row = rng.integers(0, 256, size=(1, 7, 3), dtype=np.uint8)
        cu = [_pair_diff(row[0], max(j - 1, 0), min(j + 1, 6)) for j in range(7)]
        seam, cost = o.forward_seam(row)
        assert seam[0] == int(np.argmin(cu)) and cost == min(cu)
    # one column: nothing to remove against, cost 0
    seam, cost = o.forward_seam(rng.integers(0, 256, size=(6, 1, 3), dtype=np.uint8))
    assert seam.tolist() == [0] * 6 and cost == 0
    # target_w == W is the identity
    img = rng.integers(0, 256, size=(4, 5, 3), dtype=np.uint8)
    out, seams, costs = o.carve_forward(img, 5)
    assert np.array_equal(out, img) and seams.shape == (0, 4)


def forward_carve_invariants(o, img, target_w, check_brute=False):
    """Run the forward carve seam by seam: each seam is valid, its recorded cost is the
    removal-defined cost on the current image, it is the current image's minimum seam, and the
    output is the input with the seams deleted."""
    out, seams, costs = o.carve_forward(img, target_w)
    cur = img.copy()
    H = img.shape[0]
    for k in range(seams.shape[0]):
        s = seams[k]
        check_seam_valid(s, H, cur.shape[1])
        assert costs[k] == py_forward_cost_by_removal(cur, s), ("cost", k)
        if check_brute:
            bs, bc = py_brute_forward(cur)
            assert s.tolist() == bs.tolist() and costs[k] == bc, ("brute", k)
        cur = np.stack([np.delete(cur[i], s[i], axis=0) for i in range(H)])
    assert np.array_equal(out, cur), "carved image != input with the seams deleted"
    return seams, costs


def pin_forward_carve_invariants(o):
    rng = np.random.default_rng(23)
    for (H, W, C, tw) in [(4, 6, 3, 2), (3, 5, 1, 1), (1, 6, 4, 2), (5, 2, 3, 1)]:
        for alpha in (3, 256):
            img = rng.integers(0, alpha, size=(H, W, C), dtype=np.uint8)
            forward_carve_invariants(o, img, tw, check_brute=True)
    img = rng.integers(0, 256, size=(12, 20, 3), dtype=np.uint8)
    forward_carve_invariants(o, img, 9)


ALL_PINS += [pin_forward_hand_grids, pin_forward_bruteforce, pin_forward_closed_forms, pin_forward_carve_invariants]


# --------------------------------------------------------------------------------------------
# Object removal with a mask (sec. "Object Removal" among the applications; readings R20-R24)


def py_brute_masked(e, mask):
    """Every connected seam of the energy map e (int [H, W]) under the key
    (-masked pixels on the seam, energy of the seam, s[H-1], ..., s[0]): the seam through the most
    masked pixels, then the cheapest, then R5/R6 ties.  This is what any mask bias above the bound
    of R20 selects, written without a bias at all.  Tiny maps only."""
    e = np.asarray(e)
    H, W = e.shape
    best = None
    for start in range(W):
        for moves in itertools.product((-1, 0, 1), repeat=H - 1):
            path = [start]
            for mv in moves:
                path.append(path[-1] + mv)
            if min(path) < 0 or max(path) >= W:
                continue
            rows = [(H - 1 - t, path[t]) for t in range(H)]
            cnt = sum(1 for (r, c) in rows if mask[r, c])
            en = sum(int(e[r, c]) for (r, c) in rows)
            key = (-cnt, en, tuple(path))
            if best is None or key < best:
                best = key
    ncnt, en, path = best
    return np.array(path[::-1], np.int32), -ncnt, en


def _bbox_direction(mask):
    """R21 from the definition: vertical (0) unless the mask's box is wider than tall."""
    ys, xs = np.nonzero(mask)
    if len(ys) == 0:
        return 0
    return 0 if (xs.max() - xs.min() + 1) <= (ys.max() - ys.min() + 1) else 1


def object_invariants(o, img, mask, direction=-1, restore=False, check_brute=False):
    """Replay the recorded seams on numpy copies of the image and the mask: every seam is valid,
    crosses at least one masked pixel while one is left, costs its energy minus B per masked pixel
    on the current image, and (small cases) is the brute-force masked seam; the loop stops exactly
    when the mask is gone (or one column is left); the output is the replayed image, in the
    original orientation; a restored output has the original size and holds the reduced image
    once its inserted pixels are deleted."""
    H, W, C = img.shape
    out, info, seams, costs = o.remove_object(img, mask, direction, restore)
    d = info["direction"]
    assert d == (direction if direction >= 0 else _bbox_direction(mask))
    cur = img.copy() if d == 0 else np.ascontiguousarray(img.transpose(1, 0, 2))
    m = (mask != 0) if d == 0 else np.ascontiguousarray((mask != 0).T)
    h = cur.shape[0]
    B = o.mask_bias(h, C)
    assert B > h * 510 * C, "the bias must exceed the energy of any seam"
    k = info["k"]
    assert seams.shape == (k, h) and costs.shape == (k,)
    for j in range(k):
        assert m.any() and cur.shape[1] > 1, "a seam was removed after the mask was gone"
        s = seams[j]
        check_seam_valid(s, h, cur.shape[1])
        on = m[np.arange(h), s]
        assert on.any(), "a masked seam missed the mask"
        e = o.energy(cur)
        assert costs[j] == int(e[np.arange(h), s].sum()) - B * int(on.sum()), ("cost", j)
        if check_brute:
            bs, bcnt, ben = py_brute_masked(e, m)
            assert s.tolist() == bs.tolist() and int(on.sum()) == bcnt, ("brute", j)
        cur = np.stack([np.delete(cur[i], s[i], axis=0) for i in range(h)])
        m = np.stack([np.delete(m[i], s[i], axis=0) for i in range(h)])
    assert info["left"] == int(m.sum())
    assert not m.any() or cur.shape[1] == 1, "the loop stopped with masked pixels left"
    if not restore or k == 0:
        want = cur if d == 0 else np.ascontiguousarray(cur.transpose(1, 0, 2))
        assert np.array_equal(out, want), "output != input with the seams deleted"
    else:
        assert out.shape == (H, W, C)
        o_frame = out if d == 0 else np.ascontiguousarray(out.transpose(1, 0, 2))
        # the rounds of R23 on the reduced image, each one the insertion of the image enlargement
        res, rw = cur, cur.shape[1]
        while rw < cur.shape[1] + k:
            n = min(cur.shape[1] + k - rw, rw - 1)
            res, orig = o.insert_seams(res, n)
            rw += n
        assert np.array_equal(o_frame, res), "restored output != insertion rounds on the reduced image"
    return out, info, seams, costs


def pin_object_hand_grid(o):
    for c in load_golden("object_grids.json")["cases"]:
        img = np.array(c["img"], np.uint8)
        mask = np.array(c["mask"], np.uint8)
        assert o.mask_bias(img.shape[0], img.shape[2]) == c["bias"]
        out, info, seams, costs = o.remove_object(img, mask)
        assert info["direction"] == c["direction"] and seams.tolist() == c["seams"], c["name"]
        assert costs.tolist() == c["costs"], c["name"]
        assert np.array_equal(out, np.array(c["reduced"], np.uint8)), c["name"]
        out, info, _, _ = o.remove_object(img, mask, restore=True)
        assert np.array_equal(out, np.array(c["restored"], np.uint8)), c["name"]
        # the same object turned 90 degrees: horizontal seams, the transposed results
        t_img = np.ascontiguousarray(img.transpose(1, 0, 2))
        out, info, seams, costs = o.remove_object(t_img, np.ascontiguousarray(mask.T), restore=True)
        assert info["direction"] == 1 - c["direction"] and seams.tolist() == c["seams"], c["name"]
        assert np.array_equal(out, np.array(c["restored"], np.uint8).transpose(1, 0, 2)), c["name"]


def pin_masked_seam_bruteforce(o, n=150, seed=31):
    """The masked seam equals the lexicographic brute force for the bias of R20 and for any larger
    one; with no bias it is the e1 seam of the DP section."""
    rng = np.random.default_rng(seed)
    for t in range(n):
        H, W = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        C = int(rng.integers(1, 4))
        alpha = [2, 3, 256][t % 3]
        img = rng.integers(0, alpha, size=(H, W, C), dtype=np.uint8)
        mask = (rng.random((H, W)) < [0.1, 0.3, 0.6][t % 3]).astype(np.uint8)
        e = o.energy(img)
        bs, bcnt, ben = py_brute_masked(e, mask)
        B = o.mask_bias(H, C)
        for b in (B, 3 * B + 7):
            s, cost = o.masked_seam(img, mask, b)
            assert s.tolist() == bs.tolist() and cost == ben - b * bcnt, (t, b, img.tolist(), mask.tolist())
        s0, c0 = o.masked_seam(img, mask, 0)
        ps, pc = py_brute_seam(e)
        assert s0.tolist() == ps.tolist() and c0 == pc


def pin_object_direction(o):
    def box(H, W, y0, y1, x0, x1):
        m = np.zeros((H, W), np.uint8)
        m[y0:y1, x0:x1] = 1
        return m
    assert o.object_direction(np.zeros((5, 7), np.uint8)) == 0            # empty: nothing to choose
    assert o.object_direction(box(9, 9, 1, 8, 3, 5)) == 0                  # 7 tall, 2 wide
    assert o.object_direction(box(9, 9, 3, 5, 1, 8)) == 1                  # 2 tall, 7 wide
    assert o.object_direction(box(9, 9, 2, 6, 2, 6)) == 0                  # square: vertical
    m = np.zeros((8, 8), np.uint8)
    m[1, 1] = m[2, 6] = 1                                                  # box 2 tall, 6 wide
    assert o.object_direction(m) == 1
    m[7, 3] = 1                                                            # box 7 tall, 6 wide
    assert o.object_direction(m) == 0


def pin_object_invariants(o):
    rng = np.random.default_rng(33)
    for (H, W, C) in [(4, 6, 3), (5, 4, 1), (3, 7, 2), (6, 5, 3)]:
        for alpha in (3, 256):
            img = rng.integers(0, alpha, size=(H, W, C), dtype=np.uint8)
            mask = np.zeros((H, W), np.uint8)
            y0, x0 = int(rng.integers(0, H - 1)), int(rng.integers(0, W - 1))
            mask[y0:y0 + int(rng.integers(1, H - y0 + 1)), x0:x0 + int(rng.integers(1, 3))] = 1
            object_invariants(o, img, mask, check_brute=True)
            object_invariants(o, img, mask, restore=True)
            object_invariants(o, img, mask, direction=1 - _bbox_direction(mask), check_brute=True)
    img = rng.integers(0, 256, size=(14, 18, 3), dtype=np.uint8)
    mask = np.zeros((14, 18), np.uint8)
    mask[3:11, 7:10] = 1
    mask[5, 12] = 1
    object_invariants(o, img, mask, restore=True)


def pin_object_edges(o):
    rng = np.random.default_rng(34)
    img = rng.integers(0, 256, size=(5, 6, 3), dtype=np.uint8)
    # no mask: nothing removed, the image back unchanged
    for restore in (False, True):
        out, info, seams, costs = o.remove_object(img, np.zeros((5, 6), np.uint8), restore=restore)
        assert info["k"] == 0 and info["left"] == 0 and np.array_equal(out, img) and seams.shape == (0, 5)
    # a mask of two whole columns: two seams, each one of those columns, straight down
    mask = np.zeros((5, 6), np.uint8)
    mask[:, 1] = mask[:, 4] = 1
    out, info, seams, costs = object_invariants(o, img, mask, check_brute=True)
    assert info["k"] == 2 and all(len(set(s.tolist())) == 1 for s in seams)
    assert {int(seams[0][0]), int(seams[1][0])} in ({1, 3}, {4, 1})
    # more columns removed than remain: the size comes back in rounds (R23)
    mask = np.zeros((5, 6), np.uint8)
    mask[:, 1:5] = 1
    out, info, _, _ = object_invariants(o, img, mask, restore=True)
    assert info["k"] == 4 and out.shape == img.shape
    # one row, all masked: the carve stops at one column with the last masked pixel left
    row = rng.integers(0, 256, size=(1, 5, 3), dtype=np.uint8)
    out, info, _, _ = object_invariants(o, row, np.ones((1, 5), np.uint8), direction=0)
    assert info["k"] == 4 and info["left"] == 1 and out.shape == (1, 1, 3)
    try:  # ... and a single column cannot be enlarged
        o.remove_object(row, np.ones((1, 5), np.uint8), direction=0, restore=True)
        raise AssertionError("restoring from one column must fail")
    except ValueError:
        pass


ALL_PINS += [pin_object_hand_grid, pin_masked_seam_bruteforce, pin_object_direction, pin_object_invariants,
             pin_object_edges]
