"""The 2D path (quadtrees, D2Q9) on the GPU against the 2D oracle, element by
element: blocks, solid flags, classes, refinement marks and child maps of
every level; the cut-link table's cells and directions exactly, q within
1e-5, the crossed edge wherever the oracle's is unique.  Includes the
paper's two 2D workloads at full size (512^2 root grid, levels 0..4)."""
import numpy as np
import pytest
import torch

import oracle
from synth import configs
from gpu_helpers import say

pytestmark = pytest.mark.gpu

NAMES = ["cylinder2d_small", "square2d_small", "shapes2d_small", "cylinder2d", "square2d"]
_refs = {}


def _ref(name):
    if name not in _refs:
        w = configs.get(name)
        _refs[name] = (w, oracle.embed2d(w.poly, w.n0, w.lf, w.d_spec))
    return _refs[name]


def _gpu(w, embedder=None):
    from paper_2512_01251_amd import pipeline2d
    V = torch.from_numpy(np.ascontiguousarray(w.poly.verts, dtype=np.float64)).cuda()
    E = torch.from_numpy(np.ascontiguousarray(w.poly.edges, dtype=np.int32)).cuda()
    e = embedder or pipeline2d.Embedder2D()
    return e.embed(V, E, w.n0, w.lf, w.d_spec)


def _compare(w, emb, ref):
    assert len(emb.levels) == len(ref["levels"])
    for g, r in zip(emb.levels, ref["levels"]):
        L = r["level"]
        assert np.array_equal(g.bcoord.cpu().numpy(), r["bcoord"]), f"blocks L{L}"
        gs = g.solid.cpu().numpy().view(np.uint16)
        assert np.array_equal(gs, r["solid"]), f"solid L{L}: {np.count_nonzero(gs != r['solid'])} blocks differ"
        if "refine" in r:
            assert np.array_equal(g.bclass.cpu().numpy(), r["bclass"]), f"bclass L{L}"
            assert np.array_equal(g.refine.cpu().numpy(), r["refine"]), f"refine L{L}"
            assert np.array_equal(g.child_map.cpu().numpy(), r["child_map"]), f"child_map L{L}"
    gl, rl = emb.links, ref["links"]
    assert gl.n == rl["n"], (gl.n, rl["n"])
    assert np.array_equal(gl.cell.cpu().numpy(), rl["cell"])
    assert np.array_equal(gl.dir.cpu().numpy(), rl["dir"])
    err = np.abs(gl.q.cpu().numpy().astype(np.float64) - rl["q"])
    if len(err) == 0:
        err = np.zeros(1)
    assert err.max() <= 1e-5, err.max()
    ge = gl.edge.cpu().numpy()
    sel = rl["tied"] == 0
    assert np.array_equal(ge[sel], rl["tri"][sel])
    return err.max()


@pytest.mark.parametrize("name", NAMES)
def test_2d_parity(name):
    w, ref = _ref(name)
    say(f"[2d] {name}")
    emb = _gpu(w)
    e = _compare(w, emb, ref)
    say(f"[2d] {name} ok: blocks {[int(l.bcoord.shape[0]) for l in emb.levels]}, {emb.links.n} links, "
        f"max |dq| {e:.2e}")


def test_2d_overflowed_buffers_are_redone_and_runs_identical():
    from paper_2512_01251_amd import pipeline2d
    w, ref = _ref("shapes2d_small")
    e = pipeline2d.Embedder2D()
    for L in range(w.lf + 1):
        e.caps[("rows", L)] = 1
    e.caps[("links", w.lf)] = 1
    e.caps[("links_table", w.lf)] = 1
    a = _gpu(w, e)
    assert e.caps[("rows", 0)] > 1 and e.caps[("links_table", w.lf)] > 1
    _compare(w, a, ref)
    b = _gpu(w, e)
    for f in ("cell", "dir", "q", "edge"):
        assert np.array_equal(getattr(a.links, f).cpu().numpy(), getattr(b.links, f).cpu().numpy()), f
