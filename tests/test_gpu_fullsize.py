"""GPU parity at the full benchmark sizes.

star112k (112,000 triangles, 128^3 base, levels 0..3, D3Q19) and spheres64
(1,024,000 triangles, 256^3 base, levels 0..3, D3Q19): the whole forest
(every cell of every level, classes, marks, child maps) and the whole link
set of the finest level (the link mask of every cell, the link count, the
table's (cell, direction) order) against the oracle; q and the hit triangle
on a random sample of links.

star7m (7,200,000 triangles, float32 vertices, 256^3 base, levels 0..4,
D3Q27; the benchmark workload in the benchmark's launch configuration): the
whole forest and the whole link set in both forms; the oracle's own link
table (mask, cells, directions, q, hit triangles) on a sample of blocks that
includes blocks with no link-bin candidates; q on a random sample of links;
invariants that hold at any size.

The whole link set comes from the oracle's solid flags of the level and the
oracle's point rule for neighbour centres in no block (link_sets.py), so a
link or a block the GPU drops is found.
"""
import numpy as np
import pytest

import oracle
from synth import configs
from gpu_helpers import gpu_embed, say
from link_sets import level_link_set

pytestmark = pytest.mark.gpu

Q_TOL = 1e-5


def _cells_of(bcoord, blocks, t):
    return 4 * bcoord[blocks] + np.stack([t & 3, (t >> 2) & 3, t >> 4], 1)


def _check_forest(emb, ref):
    assert len(emb.levels) == len(ref["levels"])
    for g, r in zip(emb.levels, ref["levels"]):
        L = r["level"]
        assert np.array_equal(g.bcoord.cpu().numpy(), r["bcoord"]), f"blocks L{L}"
        gs = g.solid.cpu().numpy().view(np.uint64)
        assert np.array_equal(gs, r["solid"]), f"solid L{L}: {np.count_nonzero(gs != r['solid'])} blocks differ"
        if "refine" in r:
            assert np.array_equal(g.bclass.cpu().numpy(), r["bclass"]), f"bclass L{L}"
            assert np.array_equal(g.refine.cpu().numpy(), r["refine"]), f"refine L{L}"
            assert np.array_equal(g.child_map.cpu().numpy(), r["child_map"]), f"child_map L{L}"


def _check_link_set(emb, lset):
    """Every link of the level: count, (cell, direction) in table order, and
    the mask of every cell when the GPU wrote it."""
    Lk = emb.links
    n_ref = len(lset["cell"])
    assert Lk.n == n_ref, (Lk.n, n_ref)
    assert np.array_equal(Lk.cell.cpu().numpy().astype(np.int64), lset["cell"]), "link cells"
    assert np.array_equal(Lk.dir.cpu().numpy(), lset["dir"]), "link directions"
    if Lk.mask is not None:
        nb = int(emb.levels[-1].bcoord.shape[0])
        full = np.zeros((nb, 64), np.uint32)
        full[lset["blocks"]] = lset["masks"]
        gm = Lk.mask.cpu().numpy().view(np.uint32).reshape(nb, 64)
        assert np.array_equal(gm, full), f"link mask: {np.count_nonzero(gm != full)} cells differ"


def _check_links_sample(w, emb, rng, n):
    """q and hit triangle of n random links against the oracle's nearest hit;
    where the oracle finds several triangles at the minimum, the GPU's must
    be one of them."""
    lv = emb.levels[-1]
    L = lv.level
    bc = lv.bcoord.cpu().numpy()
    Lk = emb.links
    idx = rng.choice(Lk.n, min(n, Lk.n), replace=False)
    cell = Lk.cell.cpu().numpy()[idx]
    dirs = Lk.dir.cpu().numpy()[idx]
    cells = _cells_of(bc, cell // 64, cell % 64)
    ref = oracle.q_points(w.mesh, w.n0, L, cells, dirs)
    q = Lk.q.cpu().numpy()[idx].astype(np.float64)
    err = np.abs(q - ref["q"])
    assert err.max() <= Q_TOL, err.max()
    tri = Lk.tri.cpu().numpy()[idx]
    untied = ref["tied"] == 0
    assert np.array_equal(tri[untied], ref["tri"][untied])
    tied = np.nonzero(~untied)[0]
    if len(tied):
        g = oracle.q_given(w.mesh, w.n0, L, cells[tied], dirs[tied], tri[tied])
        assert g["is_min"].all(), f"{np.count_nonzero(~g['is_min'])} tied links name a triangle off the minimum"
    return float(err.max()), len(tied)


def _check_block_sample(w, emb, lset, rng, n_link_blocks, n_random, n_empty_bins):
    """The oracle's whole link table (mask, cells, directions, q, triangles)
    on a sample of blocks: blocks with links, random blocks, and candidate
    blocks (a fluid cell near a solid one) whose link bins are empty."""
    lv = emb.levels[-1]
    L = lv.level
    bc = lv.bcoord.cpu().numpy()
    nb = len(bc)
    gcell = emb.links.cell.cpu().numpy().astype(np.int64)
    gblk = gcell // 64
    with_links = np.unique(gblk)
    boff = emb.links.bins_off.cpu().numpy().astype(np.int64)
    empty = np.nonzero(boff[1:nb + 1] == boff[:nb])[0]
    empty_cand = np.intersect1d(empty, lset["blocks"])
    pick = [rng.choice(with_links, min(n_link_blocks, len(with_links)), replace=False),
            rng.choice(nb, min(n_random, nb), replace=False)]
    if len(empty_cand):
        pick.append(rng.choice(empty_cand, min(n_empty_bins, len(empty_cand)), replace=False))
    sel = np.unique(np.concatenate(pick))
    ref = oracle.links(w.mesh, w.n0, L, bc[sel], w.lattice)
    # the GPU's table restricted to the sampled blocks, in the same order
    lo = np.searchsorted(gblk, sel, side="left")
    hi = np.searchsorted(gblk, sel, side="right")
    rows = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)]) if len(sel) else np.zeros(0, np.int64)
    pos_in_sel = np.repeat(np.arange(len(sel)), hi - lo)
    got_cell = pos_in_sel * 64 + gcell[rows] % 64
    assert len(rows) == ref["n"], (len(rows), ref["n"])
    assert np.array_equal(got_cell, ref["cell"].astype(np.int64))
    assert np.array_equal(emb.links.dir.cpu().numpy()[rows], ref["dir"])
    q = emb.links.q.cpu().numpy()[rows].astype(np.float64)
    err = np.abs(q - ref["q"]) if ref["n"] else np.zeros(1)
    assert err.max() <= Q_TOL, err.max()
    untied = ref["tied"] == 0
    assert np.array_equal(emb.links.tri.cpu().numpy()[rows][untied], ref["tri"][untied])
    if emb.links.mask is not None:
        gm = emb.links.mask.cpu().numpy().view(np.uint32).reshape(nb, 64)[sel]
        assert np.array_equal(gm, ref["mask"])
    return {"blocks": len(sel), "empty_bin_candidates": int(len(empty_cand)), "links": int(ref["n"]),
            "max_dq": float(err.max())}


def _check_invariants(w, emb):
    lv = emb.levels
    for L in range(1, len(lv)):
        par = lv[L - 1].bcoord.cpu().numpy().astype(np.int64)
        dims = np.array(w.n0) // 4 * 2 ** (L - 1)
        key = lambda c: (c[:, 2] * dims[1] + c[:, 1]) * dims[0] + c[:, 0]
        pk = np.sort(key(par))
        ch = lv[L].bcoord.cpu().numpy().astype(np.int64)
        parents = np.unique(ch // 2, axis=0)
        # children come in complete octets, in parent order
        ref = lv[L - 1].refine.cpu().numpy().astype(bool)
        assert len(ch) == 8 * ref.sum()
        assert np.array_equal(ch[::8] // 2, par[ref])
        # 2:1 balance: every in-domain 26-neighbour of a refined parent exists
        for d in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).reshape(3, -1).T:
            q = parents + d
            ok = ((q >= 0) & (q < dims)).all(1)
            found = np.isin(key(q[ok]), pk)
            assert found.all(), f"level {L}: refined parent with a missing neighbour"
    # coverage: every vertex lies in a finest-level block
    L = len(lv) - 1
    dims = np.array(w.n0) // 4 * 2 ** L
    fb = lv[-1].bcoord.cpu().numpy().astype(np.int64)
    fk = np.sort((fb[:, 2] * dims[1] + fb[:, 1]) * dims[0] + fb[:, 0])
    vb = np.floor(w.mesh.verts.astype(np.float64) * 2 ** L / 4).astype(np.int64)
    vk = (vb[:, 2] * dims[1] + vb[:, 1]) * dims[0] + vb[:, 0]
    assert np.isin(vk, fk).all()
    # link table order (block, t, k)
    cell = emb.links.cell.cpu().numpy().astype(np.int64)
    dr = emb.links.dir.cpu().numpy().astype(np.int64)
    key = cell * 32 + dr
    assert (np.diff(key) > 0).all()


def _forest_and_links(w):
    say(f"[fullsize] {w.name}: oracle forest ...")
    ref = oracle.embed(w.mesh, w.n0, w.lf, w.lattice, w.d_spec, with_links=False)
    lv = ref["levels"][-1]
    say(f"[fullsize] {w.name}: link set from the oracle's flags ...")
    lset = level_link_set(w.mesh, w.n0, w.lf, lv["bcoord"], lv["solid"], w.lattice)
    say(f"[fullsize] {w.name}: {len(lset['cell'])} links in {len(lset['blocks'])} candidate blocks")
    return w, ref, lset


@pytest.fixture(scope="module")
def c1():
    return _forest_and_links(configs.star112k())


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_star112k_forest_and_link_set(c1, precision):
    w, ref, lset = c1
    say(f"[fullsize] star112k {precision}")
    emb, _, _ = gpu_embed(w, precision, with_mask=True)
    _check_forest(emb, ref)
    _check_link_set(emb, lset)
    _check_invariants(w, emb)
    e, nt = _check_links_sample(w, emb, np.random.default_rng(1), 20000)
    say(f"[fullsize] star112k {precision} ok: {emb.links.n} links, sampled max |dq| {e:.2e}, {nt} tied")


@pytest.fixture(scope="module")
def c2():
    return _forest_and_links(configs.star7m())


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_star7m_forest_and_link_set(c2, precision):
    w, ref, lset = c2
    say(f"[fullsize] star7m {precision}")
    emb, _, _ = gpu_embed(w, precision)
    _check_forest(emb, ref)
    _check_link_set(emb, lset)
    _check_invariants(w, emb)
    rng = np.random.default_rng(2)
    bs = _check_block_sample(w, emb, lset, rng, 4000, 2000, 1000)
    e, nt = _check_links_sample(w, emb, rng, 20000)
    st = emb.stats.cpu().numpy()
    say(f"[fullsize] star7m {precision} ok: {emb.links.n} links, block sample {bs}, sampled max |dq| {e:.2e}, "
        f"{nt} tied, stats {st.tolist()}")
    assert st[3] == 0


def test_star7m_bounce_back_properties():
    """Bounce-back over every link of the 7.2M-triangle star's finest level
    (D3Q27), float32 populations for all its blocks, checked by properties
    that hold at any size:
      simple bounce-back returns f*_p(x) into the reversed direction of x,
        for every link, and writes nothing else;
      a fluid at rest (f* = w_k) stays at rest under interpolated
        bounce-back: every returned population is exactly w of its direction
        (fp = fu = fb makes every form exact)."""
    import torch
    from paper_2512_01251_amd import geo_ibb, make_level
    from paper_2512_01251_amd.pipeline import links_dense
    from synth.populations import lattice_weights
    w = configs.star7m()
    say("[fullsize] star7m bounce-back")
    emb, _, _ = gpu_embed(w, "f32")
    dn = links_dense(emb)
    rec = emb.levels[-1]
    nb = int(rec.bcoord.shape[0])
    lvd = make_level(emb.n0, emb.lf, rec.bcoord, [lv.child_map for lv in emb.levels[:-1]])
    D = np.array([[k % 3 - 1, (k // 3) % 3 - 1, k // 9 - 1] for k in range(27)])
    rev = torch.tensor([int(np.nonzero(np.all(D == -D[k], axis=1))[0][0]) for k in range(27)], device="cuda")
    cell = emb.links.cell.long()
    k = emb.links.dir.long()
    b, t = cell // 64, cell % 64
    src = (b * 27 + k) * 64 + t          # D3Q27: slot = k
    dst = (b * 27 + rev[k]) * 64 + t
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    f_post = torch.empty((nb, 27, 64), dtype=torch.float32, device="cuda").uniform_(0.5, 1.0, generator=g)
    f_new = torch.full_like(f_post, -1.0)
    geo_ibb(lvd, rec.solid, dn.block_map, dn.q, dn.nbnd, 27, False, f_post, f_new)
    torch.cuda.synchronize()
    assert torch.equal(f_new.view(-1)[dst], f_post.view(-1)[src])
    assert int((f_new != -1.0).sum().item()) == emb.links.n
    wt = torch.tensor(lattice_weights(27), dtype=torch.float32, device="cuda")
    f_post.copy_(wt[None, :, None].expand_as(f_post))
    f_new.fill_(-1.0)
    d_fb = torch.zeros(1, dtype=torch.int64, device="cuda")
    geo_ibb(lvd, rec.solid, dn.block_map, dn.q, dn.nbnd, 27, True, f_post, f_new, d_fb)
    torch.cuda.synchronize()
    assert torch.equal(f_new.view(-1)[dst], wt[rev[k]])
    assert int((f_new != -1.0).sum().item()) == emb.links.n
    say(f"[fullsize] star7m bounce-back ok: {emb.links.n} links, {dn.nbnd} boundary blocks, "
        f"{int(d_fb.item())} fallbacks")


# ----------------------------------------------------------------------------
# degenerate and multi-body workloads at full size (256^3 base, levels 0..3,
# D3Q19): faces and vertices on cell-centre planes and lattice points, and 64
# disjoint bodies
# ----------------------------------------------------------------------------

_deg_cache = {}


def _deg_ref(name):
    if name not in _deg_cache:
        w = configs.get(name)
        say(f"[fullsize] {name} oracle ...")
        _deg_cache[name] = (w, oracle.embed(w.mesh, w.n0, w.lf, w.lattice, w.d_spec))
    return _deg_cache[name]


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("name", ["box256", "prism256"])
def test_degenerate_fullsize_exact(name, precision):
    from gpu_helpers import compare
    w, ref = _deg_ref(name)
    say(f"[fullsize] {name} {precision}")
    emb, _, _ = gpu_embed(w, precision)
    s = compare(w, emb, ref)
    _check_invariants(w, emb)
    say(f"[fullsize] {name} {precision} ok {s}")
    assert emb.stats.cpu().numpy()[3] == 0


@pytest.fixture(scope="module")
def c4():
    return _forest_and_links(configs.spheres64())


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_spheres64_forest_and_link_set(c4, precision):
    w, ref, lset = c4
    say(f"[fullsize] spheres64 {precision}")
    emb, _, _ = gpu_embed(w, precision, with_mask=True)
    _check_forest(emb, ref)
    _check_link_set(emb, lset)
    _check_invariants(w, emb)
    e, nt = _check_links_sample(w, emb, np.random.default_rng(5), 20000)
    say(f"[fullsize] spheres64 {precision} ok: {emb.links.n} links, sampled max |dq| {e:.2e}, {nt} tied")
