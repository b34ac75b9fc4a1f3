"""Pins of the 2D oracle (quadtrees, D2Q9) against results fixed by plane
geometry: half-planes of a convex polygon, winding numbers, closed rectangles
whose edges pass through cell centres, slab and Cyrus-Beck entry parameters,
the 2:1 balance of the forest, and invariance under relabelling."""
import numpy as np
import pytest

import oracle
from synth import configs, polygons


def _centres2d(bcoord, L):
    t = np.arange(16)
    local = np.stack([t % 4, t // 4], axis=1)
    c = 4 * np.asarray(bcoord, dtype=np.int64)[:, None, :] + local[None]
    return np.ldexp(c.reshape(-1, 2) + 0.5, -L)


def _dirs2d():
    return np.array([[k % 3 - 1, k // 3 - 1] for k in range(9)])


def test_convex_polygon_solid_is_intersection_of_halfplanes():
    poly = polygons.circle(200, (32.3, 31.7), 10.0)
    n0 = (64, 64)
    for L in (0, 1):
        bc = oracle.level0_blocks2d(n0) if L == 0 else np.array(
            [[x, y] for y in range(12, 20) for x in range(12, 20)], dtype=np.int32)
        cells = oracle.classify_blocks2d(poly, n0, L, bc).reshape(-1).astype(bool)
        P = _centres2d(bc, L)
        a = poly.verts[poly.edges[:, 0]]
        b = poly.verts[poly.edges[:, 1]]
        e = b - a
        ok = np.ones(len(P), bool)
        for f in range(poly.ne):
            # left of every counter-clockwise edge
            g = e[f, 0] * (P[:, 1] - a[f, 1]) - e[f, 1] * (P[:, 0] - a[f, 0])
            assert np.abs(g).min() > 1e-9
            ok &= g >= 0
        assert np.array_equal(cells, ok)
        assert ok.sum() > 100


def test_nonconvex_solid_is_nonzero_winding_number():
    """Winding number by summed angles, for centres away from every edge."""
    w = configs.shapes2d_small()
    poly = w.poly
    bc = oracle.level0_blocks2d(w.n0)
    cells = oracle.classify_blocks2d(poly, w.n0, 0, bc).reshape(-1).astype(bool)
    P = _centres2d(bc, 0)
    a = poly.verts[poly.edges[:, 0]]
    b = poly.verts[poly.edges[:, 1]]
    wind = np.zeros(len(P))
    near = np.zeros(len(P), bool)
    for f in range(poly.ne):
        u = a[f][None] - P
        v = b[f][None] - P
        wind += np.arctan2(u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0], (u * v).sum(1))
        # distance to the segment
        e = b[f] - a[f]
        s = np.clip(((P - a[f]) @ e) / (e @ e), 0, 1)
        near |= np.hypot(*(P - (a[f] + s[:, None] * e)).T) < 1e-9
    inside = np.abs(wind) > np.pi
    assert np.array_equal(cells[~near], inside[~near])
    assert inside.sum() > 300 and (~inside).sum() > 1000


def test_rectangle_through_cell_centres_is_closed():
    """Edges and corners on level-0 centres: the solid cells are exactly the
    centres in the closed rectangle, (40.5-20.5+1) x (36.5-24.5+1) of them."""
    w = configs.square2d_small()
    bc = oracle.level0_blocks2d(w.n0)
    cells = oracle.classify_blocks2d(w.poly, w.n0, 0, bc).reshape(-1).astype(bool)
    P = _centres2d(bc, 0)
    ref = (P[:, 0] >= 20.5) & (P[:, 0] <= 40.5) & (P[:, 1] >= 24.5) & (P[:, 1] <= 36.5)
    assert np.array_equal(cells, ref)
    assert ref.sum() == 21 * 13


@pytest.mark.parametrize("name", ["square2d", "square2d_small"])
def test_rectangle_q_is_slab_entry(name):
    """Links into an axis-aligned rectangle from outside: q is the slab
    method's entry parameter max_a (lo_a or hi_a - x_a) / d_a."""
    w = configs.get(name)
    r = oracle.embed2d(w.poly, w.n0, w.lf, w.d_spec)
    lk, lv = r["links"], r["levels"][-1]
    lo, hi = w.poly.verts.min(0), w.poly.verts.max(0)
    h = 2.0 ** -w.lf
    D = _dirs2d()
    P = _centres2d(lv["bcoord"], w.lf)[lk["cell"]]
    d = D[lk["dir"]] * h
    tin = np.full(len(P), -np.inf)
    for a in range(2):
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(d[:, a] > 0, (lo[a] - P[:, a]) / d[:, a], np.where(d[:, a] < 0, (hi[a] - P[:, a]) / d[:, a], -np.inf))
        tin = np.maximum(tin, t)
    assert lk["n"] > 500
    assert np.abs(lk["q"] - tin).max() < 1e-9


def test_convex_polygon_q_is_cyrus_beck_entry():
    """Convex polygon: the first crossing is the largest entry parameter over
    the edges whose outward normal opposes the link."""
    poly = polygons.circle(200, (32.3, 31.7), 10.0)
    n0, L = (64, 64), 2
    bc = oracle.level0_blocks2d(n0)
    for lv in range(L):
        cells = oracle.classify_blocks2d(poly, n0, lv, bc)
        bc = oracle.refine2d(n0, lv, bc, cells, 1)["children"]
    lk = oracle.links2d(poly, n0, L, bc)
    a = poly.verts[poly.edges[:, 0]]
    b = poly.verts[poly.edges[:, 1]]
    e = b - a
    nrm = np.stack([e[:, 1], -e[:, 0]], axis=1)   # outward for counter-clockwise edges
    P = _centres2d(bc, L)[lk["cell"]]
    d = _dirs2d()[lk["dir"]] * 2.0 ** -L
    nd = d @ nrm.T                                  # [links, edges]
    num = ((a[None] - P[:, None, :]) * nrm[None]).sum(-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(nd < 0, num / nd, -np.inf)
    assert lk["n"] > 200
    assert np.abs(lk["q"] - t.max(1)).max() < 1e-9


def test_forest_two_to_one_and_coverage():
    """Every refined block's 8 neighbours exist on its level (so children
    differ from their neighbours by at most one level), and the children of a
    level tile exactly the refined blocks of the previous one."""
    w = configs.shapes2d_small()
    r = oracle.embed2d(w.poly, w.n0, w.lf, w.d_spec, with_links=False)
    for L, lv in enumerate(r["levels"][:-1]):
        bc = lv["bcoord"]
        have = {tuple(x) for x in bc}
        nbx, nby = (w.n0[0] // 4) << L, (w.n0[1] // 4) << L
        for b in np.nonzero(lv["refine"])[0]:
            for oy in (-1, 0, 1):
                for ox in (-1, 0, 1):
                    x, y = bc[b, 0] + ox, bc[b, 1] + oy
                    if 0 <= x < nbx and 0 <= y < nby:
                        assert (x, y) in have
        kids = r["levels"][L + 1]["bcoord"]
        par = {tuple(x) for x in bc[lv["refine"] != 0]}
        assert {(x // 2, y // 2) for x, y in kids} == par
        assert len(kids) == 4 * len(par)
        # every solid-boundary block is refined wherever it is eligible
        assert lv["refine"].sum() > 0


def test_relabelling_changes_nothing():
    """Reversing every edge and permuting the edge list leaves every flag and
    every q unchanged; the hit edges follow the permutation."""
    w = configs.cylinder2d_small()
    r0 = oracle.embed2d(w.poly, w.n0, w.lf, w.d_spec)
    perm = np.random.default_rng(2).permutation(w.poly.ne)
    p2 = polygons.Polygon(w.poly.verts.copy(), np.ascontiguousarray(w.poly.edges[perm][:, ::-1]))
    r1 = oracle.embed2d(p2, w.n0, w.lf, w.d_spec)
    for a, b in zip(r0["levels"], r1["levels"]):
        assert np.array_equal(a["solid"], b["solid"])
    l0, l1 = r0["links"], r1["links"]
    assert np.array_equal(l0["cell"], l1["cell"]) and np.array_equal(l0["dir"], l1["dir"])
    assert np.abs(l0["q"] - l1["q"]).max() < 1e-12
    ok = (l0["tied"] == 0) & (l1["tied"] == 0)
    assert np.array_equal(perm[l1["tri"][ok]], l0["tri"][ok])


def test_diamond_through_cell_centres_counts_vertices_once():
    """A diamond with its four vertices on level-0 centres: rows through the
    side vertices meet two edges there (one rising, one falling), and the
    solid cells are exactly the closed L1 ball |x - 32.5| + |y - 32.5| <= 12
    (so a vertex on the ray counts once)."""
    pts = np.array([[32.5, 20.5], [44.5, 32.5], [32.5, 44.5], [20.5, 32.5]])
    poly = polygons.Polygon(pts, np.array([[0, 1], [1, 2], [2, 3], [3, 0]], dtype=np.int32))
    n0 = (64, 64)
    bc = oracle.level0_blocks2d(n0)
    cells = oracle.classify_blocks2d(poly, n0, 0, bc).reshape(-1).astype(bool)
    P = _centres2d(bc, 0)
    ref = np.abs(P[:, 0] - 32.5) + np.abs(P[:, 1] - 32.5) <= 12
    assert np.array_equal(cells, ref)
    assert ref.sum() == 2 * 12 * 12 + 2 * 12 + 1
