"""The link-set derivation used by the full-size GPU tests (link_sets.py),
checked against the oracle's own link table, which classifies every halo
centre by the point rule and finds each link by its q search.  Cases: the
single-level icosphere (neighbour blocks all present or outside the domain)
and refined stars whose finest level has missing neighbour blocks (their halo
centres go through the point rule), D3Q19 and D3Q27."""
import numpy as np
import pytest

import oracle
from synth import configs
from link_sets import BlockIndex, candidate_blocks, level_link_set


@pytest.mark.parametrize("name,lattice", [("icosphere", 19), ("icosphere", 27), ("star", 19), ("star", 27),
                                          ("star32", 27)])
def test_derived_link_set_equals_oracle_table(name, lattice):
    if name == "icosphere":
        w = configs.icosphere64()
    elif name == "star":
        w = configs.star_small()
    else:
        w = configs.star_small(n_theta=14, n_phi=16, n0=32, lf=1, dtype=np.float32)
    ref = oracle.embed(w.mesh, w.n0, w.lf, lattice, w.d_spec)
    lv = ref["levels"][-1]
    got = level_link_set(w.mesh, w.n0, w.lf, lv["bcoord"], lv["solid"], lattice)
    Lk = ref["links"]
    assert Lk["n"] > 0
    assert np.array_equal(got["cell"], Lk["cell"].astype(np.int64))
    assert np.array_equal(got["dir"], Lk["dir"])
    full = np.zeros((len(lv["bcoord"]), 64), np.uint32)
    full[got["blocks"]] = got["masks"]
    assert np.array_equal(full, Lk["mask"])
    # every block with a link is a candidate
    with_links = np.unique(Lk["cell"] // 64)
    assert np.isin(with_links, got["blocks"]).all()
    if name == "star":
        # this refined grid's finest level has candidate blocks with halo
        # centres in no block (the point-rule branch is exercised)
        idx = BlockIndex(w.n0, w.lf, lv["bcoord"])
        missing = 0
        for d in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
            i, inside = idx.find(idx.bc[got["blocks"]] + np.array(d))
            missing += int((inside & (i < 0)).sum())
        assert missing > 0


def test_candidate_blocks_leave_out_only_blocks_without_links():
    """Blocks outside the candidate set are all solid, or all fluid with
    all-fluid neighbours: none has a link in the oracle's table."""
    w = configs.star_small()
    ref = oracle.embed(w.mesh, w.n0, w.lf, 19, w.d_spec)
    lv = ref["levels"][-1]
    idx = BlockIndex(w.n0, w.lf, lv["bcoord"])
    cand = candidate_blocks(idx, lv["solid"])
    rest = np.setdiff1d(np.arange(len(lv["bcoord"])), cand)
    assert len(rest) > 0
    assert (ref["links"]["mask"][rest] == 0).all()
