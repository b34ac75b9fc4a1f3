"""Refinement with 0, 2 and 3 propagation passes (Eq. 3: N_prop grows with
d_spec) against the oracle.  The whole embedding of star_small at
d_spec = 6 and 12 (N_prop = 2 and 3) must equal the oracle's, and
geo_refine_flags with n_prop = 0, called through the C-ABI on each level of
the GPU's own forest, must give the oracle's classes, marks and children."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from synth import configs
from gpu_helpers import compare, gpu_embed, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d_spec,n_prop", [(6.0, 2), (12.0, 3)])
def test_more_propagation_passes_match_the_oracle(d_spec, n_prop):
    assert oracle.n_prop(d_spec) == n_prop
    w = dataclasses.replace(configs.star_small(), d_spec=d_spec)
    ref = oracle.embed(w.mesh, w.n0, w.lf, w.lattice, w.d_spec)
    say(f"[refine] star_small d_spec={d_spec} (N_prop = {n_prop})")
    emb, _, _ = gpu_embed(w, "f32")
    s = compare(w, emb, ref)
    say(f"[refine] d_spec={d_spec}: ok {s}")


def test_refine_without_propagation_through_the_c_abi():
    import paper_2512_01251_amd as geo
    w = configs.star_small()
    emb, _, _ = gpu_embed(w, "f32", with_links=False)
    for L, lv in enumerate(emb.levels[:-1]):
        bc = lv.bcoord
        nb = int(bc.shape[0])
        lvd = geo.make_level(w.n0, L, bc, [x.child_map for x in emb.levels[:L]])
        bclass = torch.empty(nb, dtype=torch.uint8, device="cuda")
        refine = torch.empty(nb, dtype=torch.uint8, device="cuda")
        cmap = torch.empty(nb, dtype=torch.int32, device="cuda")
        child = torch.empty((8 * nb, 3), dtype=torch.int32, device="cuda")
        d_n = torch.zeros(1, dtype=torch.int64, device="cuda")
        ws = torch.empty(geo.geo_workspace_size(geo.GEO_CALL_REFINE, nb, 0), dtype=torch.uint8, device="cuda")
        geo.geo_refine_flags(lvd, lv.solid, 0, bclass, refine, cmap, child, d_n, ws)
        torch.cuda.synchronize()
        words = lv.solid.cpu().numpy().view(np.uint64)
        cells = ((words[:, None] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.uint8)
        r = oracle.refine(w.n0, L, bc.cpu().numpy(), cells, 0)
        n = int(d_n.item())
        say(f"[refine] n_prop = 0, level {L}: {nb} blocks, {int(refine.sum().item())} refined")
        assert np.array_equal(bclass.cpu().numpy(), r["bclass"])
        assert np.array_equal(refine.cpu().numpy(), r["refine"])
        assert np.array_equal(cmap.cpu().numpy(), r["child_map"])
        assert n == len(r["children"]) and np.array_equal(child[:n].cpu().numpy(), r["children"])
