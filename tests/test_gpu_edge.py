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
