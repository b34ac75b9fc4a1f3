"""Moving geometry on the GPU: a prescribed motion over several steps, each
step rebuilt with the same Embedder (remembered capacities, reused
workspace), compared with the oracle run from scratch on that step's
vertices: every flag of every level, the link table, the solid changes of
the finest level against the previous step, and the vertex gradient of a
weighted sum of q."""
import numpy as np
import pytest
import torch

import oracle
from synth import configs, meshes
from synth.weights import link_weights
from gpu_helpers import compare, say

pytestmark = pytest.mark.gpu


def _motion(mesh, s):
    """Step s of the prescribed motion: a rotation by 0.02 s about the z axis
    through the mesh centre, then a shift by s (0.31, -0.17, 0.23) cells."""
    V = mesh.verts.astype(np.float64)
    c = V.mean(axis=0)
    a = 0.02 * s
    R = np.array([[np.cos(a), -np.sin(a), 0.0], [np.sin(a), np.cos(a), 0.0], [0.0, 0.0, 1.0]])
    W = (V - c) @ R.T + c + s * np.array([0.31, -0.17, 0.23])
    return meshes.Mesh(W.astype(mesh.verts.dtype), mesh.tris.copy())


_refs = {}


def _oracle_step(w, m, s):
    if s not in _refs:
        _refs[s] = oracle.embed(m, w.n0, w.lf, w.lattice, w.d_spec)
    return _refs[s]


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_moving_geometry_steps_match_the_oracle(precision):
    from paper_2512_01251_amd import pipeline
    w = configs.star_small()
    e = pipeline.Embedder()
    T = torch.from_numpy(np.ascontiguousarray(w.mesh.tris, dtype=np.int32)).cuda()
    prev, prev_mesh, first = None, None, None
    for s in range(3):
        m = _motion(w.mesh, s)
        say(f"[moving] {precision} step {s}")
        ref = _oracle_step(w, m, s)
        V = torch.from_numpy(np.ascontiguousarray(m.verts)).cuda().requires_grad_(True)
        emb, q, ch = pipeline.shape_step(e, V, T, w.n0, w.lf, w.lattice, w.d_spec, precision, prev)
        compare(w, emb, ref)
        lv = ref["levels"][-1]
        if s == 0:
            assert ch is None
            first = (emb.links.cell.cpu().numpy().copy(), emb.links.q.cpu().numpy().copy())
        else:
            oc = oracle.solid_change(prev_mesh, w.n0, w.lf, lv["bcoord"], lv["solid_cells"])
            sp = ch.spawned.cpu().numpy().view(np.uint64)
            cv = ch.covered.cpu().numpy().view(np.uint64)
            assert np.array_equal(sp, oracle.pack_bits(oc["spawned"]))
            assert np.array_equal(cv, oracle.pack_bits(oc["covered"]))
            n_sp, n_cv = ch.counts.cpu().tolist()
            assert (n_sp, n_cv) == (oc["n_spawned"], oc["n_covered"])
            assert n_sp > 0 and n_cv > 0
            say(f"[moving] step {s}: {n_sp} cells uncovered, {n_cv} covered")
        # gradient of a weighted sum of q where the hit triangle is unique
        rl = ref["links"]
        wts = link_weights(w.lf, lv["bcoord"], rl["cell"], rl["dir"], seed=3 + s)
        wts[rl["tied"] != 0] = 0.0
        g_ref = oracle.grad(m, w.n0, w.lf, lv["bcoord"], rl["cell"], rl["dir"], rl["tri"], wts)
        (q.double() * torch.from_numpy(wts).cuda()).sum().backward()
        g = V.grad.cpu().numpy()
        assert np.abs(g - g_ref).max() <= 1e-4 * np.abs(g_ref).max()
        prev, prev_mesh = emb, m
    # back to the first position with the same Embedder: the same table
    V0 = torch.from_numpy(np.ascontiguousarray(_motion(w.mesh, 0).verts)).cuda()
    again = e.embed(V0, T, w.n0, w.lf, w.lattice, w.d_spec, precision, True)
    assert np.array_equal(again.links.cell.cpu().numpy(), first[0])
    assert np.array_equal(again.links.q.cpu().numpy(), first[1])
