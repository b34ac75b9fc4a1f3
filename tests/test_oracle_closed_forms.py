"""More pins of the CPU oracle against results that geometry fixes.

P3  icosphere: q against the entry root of the circumscribed sphere, within
    the gap between each facet plane and the sphere; solid count against the
    polyhedron's volume, within the number of cells the surface cuts.
P5  convex prism: q is the Cyrus-Beck entry parameter over the face planes.
P7  parity along all six axis directions agrees with the solid flags for
    centres that no surface comes near.
P11 a face on (or between) cell-centre planes: every face-interior column has
    5 (D3Q19) or 9 (D3Q27) cut links, all with q = (p_z - z0) / h.
Link sets: the (cell, direction) set of a convex body, D3Q19 and D3Q27,
    from half-space membership of every centre and of its neighbours.

Each test states the slip in the oracle it would catch.
"""
import numpy as np
import pytest

import oracle
from synth import configs, meshes


def _dirs():
    return np.array([[k % 3 - 1, (k // 3) % 3 - 1, k // 9 - 1] for k in range(27)])


def _planes(mesh):
    V = mesh.verts.astype(np.float64)
    T = mesh.tris
    a = V[T[:, 0]]
    n = np.cross(V[T[:, 1]] - a, V[T[:, 2]] - a)
    keep = np.abs(n).sum(1) > 0
    return a[keep], n[keep]


def _halfspace_inside(a, n, P):
    """Closed convex body as the intersection of the facet half-spaces
    n . (a - p) >= 0; asserts no point lies within 1e-9 of a facet plane, so
    the float64 signs are the exact ones."""
    ok = np.ones(len(P), bool)
    for f in range(len(a)):
        g = (a[f] - P) @ n[f]
        assert np.abs(g).min() > 1e-9
        ok &= g >= 0
    return ok


def _cyrus_beck(a, n, X, D):
    """Entry parameter of the segments X + t D into the convex body:
    max over the facets with n . D < 0 of n . (a - X) / (n . D); also the
    facet that attains it."""
    nd = D @ n.T
    num = np.einsum("fj,lfj->lf", n, a[None] - X[:, None])
    t = np.where(nd < 0, num / np.where(nd < 0, nd, 1.0), -np.inf)
    f = t.argmax(1)
    return t[np.arange(len(X)), f], f


# ----------------------------------------------------------------------------
# convex icosphere: link set by half-spaces (both lattices); true sphere
# ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def ico():
    w = configs.icosphere64()
    r = oracle.embed(w.mesh, w.n0, w.lf, w.lattice)
    return w, r


def _halfspace_link_set(w, lattice):
    """(cell, k) of every fluid centre of the 64^3 grid whose neighbour centre
    along c_k is solid, both by the half-space test on a dense grid of the
    centres (neighbours outside the domain are fluid); cells numbered
    64 * block + t as in the table."""
    a, n = _planes(w.mesh)
    N = w.n0[0]
    i = np.arange(N) + 0.5
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    inside = _halfspace_inside(a, n, np.stack([X, Y, Z], -1).reshape(-1, 3)).reshape(N, N, N)
    pad = np.zeros((N + 2,) * 3, bool)
    pad[1:-1, 1:-1, 1:-1] = inside
    D = _dirs()
    z, y, x = np.nonzero(~inside)
    cell = 64 * ((x // 4) + (N // 4) * ((y // 4) + (N // 4) * (z // 4))) + (x & 3) + 4 * (y & 3) + 16 * (z & 3)
    cells, dirs = [], []
    for k in oracle.lattice_dirs(lattice):
        cx, cy, cz = D[k]
        sel = pad[z + 1 + cz, y + 1 + cy, x + 1 + cx]
        cells.append(cell[sel])
        dirs.append(np.full(int(sel.sum()), k))
    cells, dirs = np.concatenate(cells), np.concatenate(dirs)
    order = np.lexsort((dirs, cells))
    return cells[order], dirs[order]


@pytest.mark.parametrize("lattice", [19, 27])
def test_icosphere_link_set_from_halfspaces(ico, lattice):
    """The oracle's link mask and table equal the set built from half-space
    membership alone.  Catches a wrong lattice filter (the D3Q27 corner
    directions dropped or the D3Q19 ones widened), a transposed halo index or
    a mask taken on solid instead of fluid cells."""
    w, r = ico
    bc = r["levels"][0]["bcoord"]
    Lk = r["links"] if lattice == w.lattice else oracle.links(w.mesh, w.n0, 0, bc, lattice)
    cells, dirs = _halfspace_link_set(w, lattice)
    assert Lk["n"] == len(cells)
    assert np.array_equal(Lk["cell"], cells) and np.array_equal(Lk["dir"], dirs)
    mask = np.zeros(len(bc) * 64, np.uint64)
    np.bitwise_or.at(mask, cells, np.left_shift(np.uint64(1), dirs.astype(np.uint64)))
    assert np.array_equal(Lk["mask"].reshape(-1).astype(np.uint64), mask)
    if lattice == 27:
        # the corner directions (|c|^2 = 3) add links only D3Q27 has
        assert (np.abs(_dirs()[dirs]).sum(1) == 3).sum() > 1000


def test_icosphere_d3q27_q_is_cyrus_beck(ico):
    """D3Q27 q on the convex icosphere (the corner directions included) is the
    Cyrus-Beck entry parameter."""
    w, r = ico
    bc = r["levels"][0]["bcoord"]
    Lk = oracle.links(w.mesh, w.n0, 0, bc, 27)
    a, n = _planes(w.mesh)
    X = oracle.cell_centres(bc, 0).reshape(-1, 3)[Lk["cell"]]
    t, _ = _cyrus_beck(a, n, X, _dirs()[Lk["dir"]].astype(float))
    np.testing.assert_allclose(Lk["q"], t, rtol=0, atol=1e-12)


def test_icosphere_q_against_true_sphere(ico):
    """The icosphere is inscribed in the sphere |x - c| = 12.  A link enters
    the sphere at t_s (smaller root of |X + t d - c|^2 = r^2) no later than it
    enters the polyhedron at q, and the polyhedron's entry facet f (plane
    n.x = d_f at distance d_f from c) satisfies n.(X + t_s d - c) <= r, so
      0 <= q - t_s <= (r - d_f) / |n . d|,  n the unit normal.
    The gap r - d_f (the sagitta) is computed from the mesh.  Catches a q
    taken at the far end, a missing 1/(n.d) scaling or a q in Euclidean units."""
    w, r = ico
    Lk, lv = r["links"], r["levels"][0]
    c = np.array([32.3, 31.7, 32.1])
    rad = 12.0
    a, n = _planes(w.mesh)
    nh = n / np.linalg.norm(n, axis=1)[:, None]
    d_f = np.einsum("ij,ij->i", nh, a - c)
    sag = rad - d_f
    assert (sag > 0).all() and sag.max() < 0.06           # a 3-times subdivided icosahedron at r = 12
    X = oracle.cell_centres(lv["bcoord"], 0).reshape(-1, 3)[Lk["cell"]]
    D = _dirs()[Lk["dir"]].astype(float)
    _, f = _cyrus_beck(a, n, X, D)
    Xc = X - c
    A = (D * D).sum(1)
    B = 2 * (Xc * D).sum(1)
    Cq = (Xc * Xc).sum(1) - rad * rad
    disc = B * B - 4 * A * Cq
    assert (disc > 0).all()                                # every link meets the sphere
    t_s = (-B - np.sqrt(disc)) / (2 * A)
    gap = Lk["q"] - t_s
    bound = sag[f] / np.abs(np.einsum("ij,ij->i", nh[f], D))
    assert (gap >= -1e-12).all()
    assert (gap <= bound + 1e-12).all()
    # the bound is not vacuous: links cross a shell far thinner than a cell
    assert np.median(bound) < 0.1


def _sat_meets(a, b, c, lo, hi, eps=1e-12):
    """Closed triangle (a, b, c) meets the closed box [lo, hi] (arrays of
    boxes), by the 13 separating axes; eps widens the box, so that a
    rounding error can only add boxes (the count is then an upper bound)."""
    ctr = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo) + eps
    v = [a - ctr, b - ctr, c - ctr]
    e = [b - a, c - b, a - c]
    axes = [np.eye(3)[i] for i in range(3)]
    axes.append(np.cross(e[0], e[1]))
    for ei in e:
        for i in range(3):
            axes.append(np.cross(np.eye(3)[i], ei))
    ok = np.ones(len(lo), bool)
    for ax in axes:
        if not np.any(ax):
            continue
        p = np.stack([vv @ ax for vv in v], 1)
        rr = (half * np.abs(ax)).sum(1)
        ok &= ~((p.min(1) > rr) | (p.max(1) < -rr))
    return ok


def test_icosphere_volume_within_cut_cells(ico):
    """A cell whose closed cube the surface does not meet lies wholly inside
    or wholly outside, so its flag counts its volume exactly; a cut cell errs
    by at most its volume.  Hence |N_solid - V_poly| <= N_cut, with V_poly by
    the divergence theorem and N_cut by triangle/cube separating axes."""
    w, r = ico
    V, T = w.mesh.verts, w.mesh.tris
    cut = set()
    for tri in T:
        a, b, c = V[tri]
        mn, mx = np.minimum(np.minimum(a, b), c), np.maximum(np.maximum(a, b), c)
        i0 = np.floor(mn - 1).astype(int)
        i1 = np.floor(mx).astype(int)
        g = np.stack(np.meshgrid(*[np.arange(i0[k], i1[k] + 1) for k in range(3)], indexing="ij"), -1).reshape(-1, 3)
        hit = _sat_meets(a, b, c, g.astype(float), g + 1.0)
        cut.update(map(tuple, g[hit]))
    n_cut = len(cut)
    v_poly = meshes.signed_volume(w.mesh)
    n_solid = int(r["levels"][0]["solid_cells"].sum())
    assert 4 / 3 * np.pi * 12 ** 3 * 0.98 < v_poly < 4 / 3 * np.pi * 12 ** 3
    assert abs(n_solid - v_poly) <= n_cut
    # the bound is about a third of the surface's cells, not the whole body
    assert n_cut < 0.5 * n_solid


# ----------------------------------------------------------------------------
# convex prism: Cyrus-Beck q over its face planes
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("lattice", [19, 27])
def test_prism_q_is_cyrus_beck(lattice):
    """64-gon prism (rim vertices on lattice points, caps on centre planes):
    convex, so every link's q is the entry parameter over its 66 face planes;
    exact for links entering through a cap (dyadic), within 1e-12 otherwise.
    Catches a q from the wrong one of two coplanar triangles' planes, an open
    instead of closed edge test where links graze rim vertices, or a missed
    hit through a shared edge."""
    w = configs.prism_small(lf=1)
    r = oracle.embed(w.mesh, w.n0, w.lf, lattice)
    Lk, lv = r["links"], r["levels"][-1]
    h = 0.5
    a, n = _planes(w.mesh)
    X = oracle.cell_centres(lv["bcoord"], 1).reshape(-1, 3)[Lk["cell"]]
    D = _dirs()[Lk["dir"]].astype(float) * h
    t, f = _cyrus_beck(a, n, X, D)
    assert len(t) > 1000
    np.testing.assert_allclose(Lk["q"], t, rtol=0, atol=1e-12)
    cap = np.abs(n[f][:, :2]).sum(1) == 0
    assert cap.sum() > 100
    assert np.array_equal(Lk["q"][cap], t[cap])


# ----------------------------------------------------------------------------
# a face on, or between, cell-centre planes: lattice counts per column
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("lattice,per_column", [(19, 5), (27, 9)])
@pytest.mark.parametrize("z_top", [36.5625, 36.3125])
def test_box_top_face_columns(lattice, per_column, z_top):
    """Box [20.5, z_top] (x, y in [20.5, 36.5625]), level 3 (h = 1/8).
    z_top = 36.5625 lies on a centre plane, 36.3125 between two.  Above each
    face-interior column exactly the lowest fluid centre has links, one per
    direction with c_z = -1 (5 in D3Q19, 9 in D3Q27), and each has
    q = (p_z - z_top) / h (the face is crossed at the same height whatever
    c_x, c_y).  Catches a lattice filter off by the corner directions and a
    q measured along |c| instead of along the link."""
    m = meshes.box((20.5, 20.5, 20.5), (36.5625, 36.5625, z_top))
    L = 3
    h = 2.0 ** -L
    # the blocks of level 3 around the top face, interior in x and y
    xs = np.arange(int(24 / (4 * h)), int(33 / (4 * h)))
    zb = int(np.floor(z_top / (4 * h)))
    bc = np.array([[x, y, z] for z in (zb - 1, zb, zb + 1) for y in xs for x in xs], np.int32)
    Lk = oracle.links(m, (64, 64, 64), L, bc, lattice)
    X = oracle.cell_centres(bc, L).reshape(-1, 3)[Lk["cell"]]
    c = _dirs()[Lk["dir"]]
    top = X[:, 2] > z_top
    p_z = h * (np.floor(z_top / h - 0.5) + 1.5)           # lowest centre above the face
    assert (X[top, 2] == p_z).all()
    assert (c[top, 2] == -1).all()
    assert np.array_equal(Lk["q"][top], np.full(top.sum(), (p_z - z_top) / h))
    cols = {}
    for x, y in X[top, :2]:
        cols[(x, y)] = cols.get((x, y), 0) + 1
    assert len(cols) == (len(xs) * 4) ** 2 and set(cols.values()) == {per_column}
    # every link below the face belongs to no column above it: none exist here
    assert top.sum() == Lk["n"]


# ----------------------------------------------------------------------------
# parity along the six axis directions
# ----------------------------------------------------------------------------

def _axis_parities(mesh, P, margin=1e-9):
    """Crossing parity of the rays from P along +e_a and -e_a for a = x, y, z,
    in float64 with barycentric coordinates; (point, axis) pairs whose ray
    comes within margin of an edge or whose crossing lies within margin of
    the point are reported as ambiguous.  Returns parities [n, 6] and an
    ambiguity mask [n, 3] per axis."""
    V = mesh.verts.astype(np.float64)
    T = mesh.tris
    A, B, C = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    par = np.zeros((len(P), 6), np.int64)
    amb = np.zeros((len(P), 3), bool)
    for ax in range(3):
        u, w = (ax + 1) % 3, (ax + 2) % 3
        area = (B[:, u] - A[:, u]) * (C[:, w] - A[:, w]) - (B[:, w] - A[:, w]) * (C[:, u] - A[:, u])
        ok = np.abs(area) > 1e-14
        a_, b_, c_, ar = A[ok], B[ok], C[ok], area[ok]
        for s in range(0, len(P), 1024):
            p = P[s:s + 1024]
            pu, pw = p[:, u][:, None], p[:, w][:, None]

            def cr(q0, q1):
                return (q1[:, u] - q0[:, u])[None] * (pw - q0[:, w][None]) - \
                       (q1[:, w] - q0[:, w])[None] * (pu - q0[:, u][None])
            l0 = cr(b_, c_) / ar[None]
            l1 = cr(c_, a_) / ar[None]
            l2 = cr(a_, b_) / ar[None]
            lm = np.minimum(np.minimum(l0, l1), l2)
            inside = lm > margin
            near = (np.abs(lm) <= margin)
            xh = l0 * a_[:, ax][None] + l1 * b_[:, ax][None] + l2 * c_[:, ax][None]
            dx = xh - p[:, ax][:, None]
            amb[s:s + 1024, ax] = near.any(1) | (inside & (np.abs(dx) <= margin)).any(1)
            par[s:s + 1024, 2 * ax] = (inside & (dx > 0)).sum(1) & 1
            par[s:s + 1024, 2 * ax + 1] = (inside & (dx < 0)).sum(1) & 1
    return par, amb


@pytest.mark.parametrize("name", ["star_small", "spheres_small"])
def test_parity_agrees_along_all_axes(name):
    """For the centres of 128 blocks per level (levels 0..1; half of them
    blocks the surface passes through), the crossing parities along each axis
    whose rays pass clear of every edge (both signs) agree with the oracle's
    flag, which uses the +x ray with a symbolic perturbation.  Rays through
    the projection of a mesh edge (a meridian seen end-on, for instance) are
    left out axis by axis.  Catches a wrong sign in the ahead-of-point test, a
    flipped edge-function rule or a lost triangle in the +x candidate lists."""
    w = configs.get(name)
    r = oracle.embed(w.mesh, w.n0, 1, w.lattice, with_links=False)
    rng = np.random.default_rng(7)
    total = 0
    for lv in r["levels"]:
        cells = lv["solid_cells"]
        # every cell of the blocks the surface passes through, and as many others
        mixed = np.nonzero((cells.min(1) == 0) & (cells.max(1) == 1))[0]
        pick = np.concatenate([rng.choice(mixed, min(len(mixed), 64), replace=False),
                               rng.choice(len(cells), 64, replace=False)])
        P = oracle.cell_centres(lv["bcoord"][pick], lv["level"]).reshape(-1, 3)
        par, amb = _axis_parities(w.mesh, P)
        got = cells[pick].reshape(-1).astype(np.int64)
        clear = np.repeat(~amb, 2, axis=1)                  # columns +a, -a share the axis
        assert ((par == got[:, None]) | ~clear).all()
        assert (clear.sum(1) >= 4).mean() > 0.99           # nearly every centre: two or three axes
        assert clear[:, 0].mean() > 0.98 and clear[:, 2].mean() > 0.98
        total += int(clear.sum())
        assert 0.1 < got.mean() < 0.9
    assert total > 6 * 14000


# ----------------------------------------------------------------------------
# hit parameter of a named triangle; the gradient's absolute-term scale
# ----------------------------------------------------------------------------

def test_q_given_on_three_crossings():
    """A thin slab x in [2.75, 3.0] and a box x in [3.25, 6.0] (both spanning
    y, z in [2.25, 6.75]): the level-0 link from (2.5, 3.5, 4.5) along +x (a
    fluid centre to the solid centre (3.5, 3.5, 4.5)) crosses the slab's two
    x faces at t = 1/4 and 1/2 and the box's low x face at t = 3/4, all
    dyadic, so the hit parameters are exact.  A triangle of each face named
    for the link gets its own t; only the slab's low face is a minimiser; a
    y face (never met) gets -1.  The oracle's own nearest triangles of the
    icosphere table are minimisers at the table's q.
    Slips caught: the named triangle's t taken from the nearest hit, is_min
    with the comparison reversed, a miss reported as t = 0."""
    slab = meshes.box((2.75, 2.25, 2.25), (3.0, 6.75, 6.75))
    body = meshes.box((3.25, 2.25, 2.25), (6.0, 6.75, 6.75))
    py, pz = 3.5, 4.5
    m = meshes.merge([slab, body])
    meshes.check_closed_oriented(m)
    V, T = m.verts.astype(np.float64), m.tris
    a = V[T[:, 0]]
    n = np.cross(V[T[:, 1]] - a, V[T[:, 2]] - a)
    xface = np.abs(n[:, 0]) > 0
    # (y, z) = (3.5, 4.5) lies on neither diagonal of these faces: one
    # triangle of each x face contains the crossing point; find it by the 2D
    # point-in-triangle test on (y, z)
    def holder(x0):
        for t in np.nonzero(xface & np.isclose(a[:, 0], x0))[0]:
            P = V[T[t]][:, 1:]
            d = np.array([(P[(i + 1) % 3][0] - P[i][0]) * (pz - P[i][1])
                          - (P[(i + 1) % 3][1] - P[i][1]) * (py - P[i][0]) for i in range(3)])
            if (d > 0).all() or (d < 0).all():
                return t
        raise AssertionError(x0)
    t_lo, t_hi, t_body = holder(2.75), holder(3.0), holder(3.25)
    yface = np.nonzero(np.abs(n[:, 1]) > 0)[0][0]
    cells = np.array([[2, 3, 4]] * 4, np.int32)
    dirs = np.array([14] * 4, np.uint8)          # c = (+1, 0, 0)
    r = oracle.q_given(m, (12, 12, 12), 0, cells, dirs, np.array([t_lo, t_hi, t_body, yface], np.int32))
    assert r["q"].tolist() == [0.25, 0.5, 0.75, -1.0]
    assert r["is_min"].tolist() == [True, False, False, False]
    near = oracle.q_points(m, (12, 12, 12), 0, cells[:1], dirs[:1])
    assert near["q"][0] == 0.25 and near["tri"][0] == t_lo
    w = configs.icosphere64()
    ref = oracle.embed(w.mesh, w.n0, w.lf, 19)
    Lk, lv = ref["links"], ref["levels"][-1]
    t = Lk["cell"] % 64
    cells = 4 * lv["bcoord"][Lk["cell"] // 64] + np.stack([t & 3, (t >> 2) & 3, t >> 4], 1)
    g = oracle.q_given(w.mesh, w.n0, 0, cells, Lk["dir"], Lk["tri"])
    assert np.array_equal(g["q"], Lk["q"]) and g["is_min"].all()


def test_grad_absolute_sums_to_the_translation_scale():
    """For one link with weight w and a hit inside its triangle (barycentrics
    lambda_j >= 0, summing to 1), the absolute-term gradient summed over the
    triangle's three vertices is |w| |n_a| / |n . d| per component (the
    signed sum is w n / (n . d), translation invariance).  With the weights of
    all links negated the absolute form is unchanged and the signed form
    flips.  Slips caught: abs taken of the summed gradient instead of each
    term, the weight's sign kept, a vertex's term dropped."""
    w = configs.icosphere64()
    ref = oracle.embed(w.mesh, w.n0, w.lf, 19)
    Lk, lv = ref["links"], ref["levels"][-1]
    ok = np.nonzero((Lk["tied"] == 0) & (Lk["q"] > 0.05) & (Lk["q"] < 0.95))[0]
    rng = np.random.default_rng(7)
    D = _dirs()
    for i in rng.choice(ok, 12, replace=False):
        wv = np.zeros(Lk["n"])
        wv[i] = -0.625
        ga = oracle.grad(w.mesh, w.n0, 0, lv["bcoord"], Lk["cell"], Lk["dir"], Lk["tri"], wv, absolute=True)
        gs = oracle.grad(w.mesh, w.n0, 0, lv["bcoord"], Lk["cell"], Lk["dir"], Lk["tri"], wv)
        vt = w.mesh.tris[Lk["tri"][i]]
        a, b, c = w.mesh.verts[vt]
        n = np.cross(b - a, c - a)
        d = D[Lk["dir"][i]].astype(np.float64)
        np.testing.assert_allclose(ga[vt].sum(0), 0.625 * np.abs(n) / abs(n.dot(d)), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(gs[vt].sum(0), -0.625 * n / n.dot(d), rtol=1e-12, atol=1e-15)
        assert (ga >= np.abs(gs) - 1e-15).all()
        others = np.setdiff1d(np.arange(len(ga)), vt)
        assert (ga[others] == 0).all()
    wv = rng.uniform(-1, 1, Lk["n"])
    ga = oracle.grad(w.mesh, w.n0, 0, lv["bcoord"], Lk["cell"], Lk["dir"], Lk["tri"], wv, absolute=True)
    gn = oracle.grad(w.mesh, w.n0, 0, lv["bcoord"], Lk["cell"], Lk["dir"], Lk["tri"], -wv, absolute=True)
    gs = oracle.grad(w.mesh, w.n0, 0, lv["bcoord"], Lk["cell"], Lk["dir"], Lk["tri"], wv)
    gsn = oracle.grad(w.mesh, w.n0, 0, lv["bcoord"], Lk["cell"], Lk["dir"], Lk["tri"], -wv)
    assert np.array_equal(ga, gn)
    np.testing.assert_allclose(gsn, -gs, rtol=0, atol=1e-12)
    assert (ga >= np.abs(gs) - 1e-12).all()
