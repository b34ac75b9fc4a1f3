"""Shared helpers of the GPU tests: run the GPU path and the oracle on the
same seeded workload and compare element by element."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import numpy as np

import oracle


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_gpu(mesh):
    import torch
    V = torch.from_numpy(np.ascontiguousarray(mesh.verts)).cuda()
    T = torch.from_numpy(np.ascontiguousarray(mesh.tris, dtype=np.int32)).cuda()
    return V, T


def gpu_embed(w, precision, with_links=True, with_mask=None, check_contract=True):
    from paper_2512_01251_amd import pipeline
    V, T = to_gpu(w.mesh)
    if with_mask is None:
        with_mask = with_links and w.mesh.nt < 500000
    emb = pipeline.Embedder().embed(V, T, w.n0, w.lf, w.lattice, w.d_spec, precision, with_links,
                                    with_mask=with_links and with_mask, check_contract=check_contract)
    return emb, V, T


Q_TOL = 1e-5


def compare(w, emb, ref, check_links=True):
    """Bit-exact integer outputs, q within Q_TOL; returns a summary dict."""
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
    out = {"cells": sum(64 * len(r["bcoord"]) for r in ref["levels"])}
    if check_links:
        gl, rl = emb.links, ref["links"]
        if gl.mask is not None:
            gm = gl.mask.cpu().numpy().view(np.uint32)
            assert np.array_equal(gm, rl["mask"].reshape(-1)), "link mask"
        assert gl.n == rl["n"], (gl.n, rl["n"])
        assert np.array_equal(gl.cell.cpu().numpy(), rl["cell"]), "link cells"
        assert np.array_equal(gl.dir.cpu().numpy(), rl["dir"]), "link dirs"
        q = gl.q.cpu().numpy().astype(np.float64)
        err = np.abs(q - rl["q"])
        if len(err) == 0:
            err = np.zeros(1)
        assert err.max() <= Q_TOL, f"max |dq| = {err.max()}"
        tri = gl.tri.cpu().numpy()
        untied = rl["tied"] == 0
        bad = np.count_nonzero(tri[untied] != rl["tri"][untied])
        out.update(links=int(gl.n), q_maxerr=float(err.max()), q_p999=float(np.quantile(err, 0.999)) if len(err) else 0.0,
                   tri_mismatch=int(bad), tied=int((~untied).sum()))
        assert bad == 0, f"{bad} untied links hit a different triangle"
    return out
