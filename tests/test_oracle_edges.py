"""The oracle on edge cases, pinned by closed forms: empty and degenerate
geometry gives an all-fluid grid with nothing refined and no links; boxes and
rectangles from the lowest allowed coordinate to the top of the domain, with
faces through cell centres, hold exactly the centres of the closed box; a body
around a single centre makes exactly that cell solid."""
import numpy as np
import pytest

import oracle
from edge_cases import cases2d, cases3d


@pytest.mark.parametrize("name", ["empty", "between", "flat"])
def test_no_solid_no_refinement_no_links(name):
    w = cases3d()[name]
    r = oracle.embed(w.mesh, w.n0, w.lf, w.lattice, w.d_spec)
    assert all(int(l["solid_cells"].sum()) == 0 for l in r["levels"])
    assert [len(l["bcoord"]) for l in r["levels"]][1:] == [0] * w.lf
    assert r["links"]["n"] == 0


def test_box_to_the_domain_top():
    w = cases3d()["edge_box"]
    r = oracle.embed(w.mesh, w.n0, 0, w.lattice, w.d_spec, with_links=False)
    # centres k + 1/2 in [0.25, 32] x [0.25, 9.5] x [0.25, 32]; 9.5 lies on a face
    assert int(r["levels"][0]["solid_cells"].sum()) == 32 * 10 * 32


def test_single_solid_centre():
    w = cases3d()["single"]
    bc = oracle.level0_blocks(w.n0)
    cells = oracle.classify_blocks(w.mesh, w.n0, 0, bc)
    P = oracle.cell_centres(bc, 0).reshape(-1, 3)[cells.reshape(-1) != 0]
    assert np.array_equal(P, [[10.5, 10.5, 10.5]])


def test_2d_edge_cases():
    c = cases2d()
    r = oracle.embed2d(c["empty2d"].poly, (32, 32), 2)
    assert all(int(l["solid_cells"].sum()) == 0 for l in r["levels"]) and r["links"]["n"] == 0
    w = c["edge_rect2d"]
    r = oracle.embed2d(w.poly, w.n0, 0, with_links=False)
    assert int(r["levels"][0]["solid_cells"].sum()) == 32 * 10
    w = c["single2d"]
    bc = oracle.level0_blocks2d(w.n0)
    cells = oracle.classify_blocks2d(w.poly, w.n0, 0, bc).reshape(-1)
    t = np.nonzero(cells)[0]
    assert len(t) == 1
    b, tt = divmod(int(t[0]), 16)
    assert (4 * bc[b, 0] + tt % 4, 4 * bc[b, 1] + tt // 4) == (10, 10)
