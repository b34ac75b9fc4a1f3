"""The GPU path on edge cases (empty and degenerate geometry, bodies at the
ends of the coordinate range, single solid cells), element by element against
the oracle, in 3D (both arithmetic forms) and 2D."""
import numpy as np
import pytest

import oracle
from edge_cases import cases2d, cases3d
from gpu_helpers import compare, gpu_embed, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("name", ["empty", "between", "single", "flat", "edge_box"])
def test_edge_cases_3d(name, precision):
    w = cases3d()[name]
    say(f"[edge] {name} {precision}")
    ref = oracle.embed(w.mesh, w.n0, w.lf, w.lattice, w.d_spec)
    emb, _, _ = gpu_embed(w, precision)
    compare(w, emb, ref)
    say(f"[edge] {name} {precision} ok: {emb.links.n} links")


@pytest.mark.parametrize("name", ["empty2d", "single2d", "edge_rect2d"])
def test_edge_cases_2d(name):
    from test_gpu_2d import _compare, _gpu
    w = cases2d()[name]
    say(f"[edge] {name}")
    ref = oracle.embed2d(w.poly, w.n0, w.lf, w.d_spec)
    emb = _gpu(w)
    _compare(w, emb, ref)
    say(f"[edge] {name} ok: {emb.links.n} links")


def test_contract_counter_counts_each_bad_coordinate():
    """A coordinate meets the contract when it is 0 or lies in [1/4, n0] on its
    own axis.  Extra vertices that no triangle references reach only the
    checker: each bad coordinate is counted once per bin build, and every
    result equals that of the clean mesh."""
    import torch
    from paper_2512_01251_amd import GEO_STAT_CONTRACT, pipeline
    from synth import configs, meshes
    base = cases3d()["single"].mesh
    n0 = (32, 24, 16)   # distinct bounds per axis
    ok_extra = [[0.0, 0.25, 16.0], [32.0, 24.0, 0.25], [31.0, 23.5, 0.0]]
    one_bad = [[5.0, 25.0, 5.0]]                                 # y above 24
    many_bad = [[33.0, 5.0, 5.0], [5.0, 5.0, 17.0], [0.1, 0.2, 5.0], [float("nan"), -1.0, 8.0]]

    def run(extra):
        v = np.concatenate([base.verts, np.array(extra, dtype=np.float64).reshape(-1, 3)])
        m = meshes.Mesh(v, base.tris, "single_extra")
        w = configs.Workload("single_extra", m, n0, 2, 27)
        say(f"[contract] {len(extra)} extra vertices")
        emb, _, _ = gpu_embed(w, "f32", check_contract=False)
        torch.cuda.synchronize()
        return emb, int(emb.stats[GEO_STAT_CONTRACT].item())

    clean, c0 = run(ok_extra)
    _, c1 = run(ok_extra + one_bad)
    dirty, c6 = run(ok_extra + many_bad)
    assert c0 == 0
    assert c1 >= 1
    assert c6 == 6 * c1
    for a, b in zip(clean.levels, dirty.levels):
        assert torch.equal(a.solid, b.solid)
    assert clean.links.n == dirty.links.n
    assert torch.equal(clean.links.q, dirty.links.q) and torch.equal(clean.links.tri, dirty.links.tri)
    # by default the driver refuses to return results of such a mesh
    v = np.concatenate([base.verts, np.array(ok_extra + one_bad, dtype=np.float64)])
    w = configs.Workload("single_bad", meshes.Mesh(v, base.tris, "single_bad"), n0, 2, 27)
    with pytest.raises(ValueError, match="coordinate range"):
        gpu_embed(w, "f32")
