"""geo_cutlinks_noalloc (scratch in a fixed device array) against
geo_cutlinks (caller workspace) through the C ABI: identical outputs, on two
calls in a row, the second with a smaller level, so the second call runs on
scratch that still holds the first call's contents."""
import numpy as np
import pytest
import torch

from synth import configs
from paper_2512_01251_amd import GEO_NSTATS
from gpu_helpers import say, to_gpu

pytestmark = pytest.mark.gpu


def _level_inputs(w):
    """The finest level of an embedding and its bins, as C-ABI descriptors."""
    from paper_2512_01251_amd import (GEO_BINS_LINKS, GEO_BINS_ROWS, make_bins, make_level, make_mesh, pipeline)
    V, T = to_gpu(w.mesh)
    emb = pipeline.Embedder().embed(V, T, w.n0, w.lf, w.lattice, w.d_spec, "f32")
    rec = emb.levels[-1]
    child_maps = [lv.child_map for lv in emb.levels[:-1]]
    lvd = make_level(w.n0, w.lf, rec.bcoord, child_maps)
    nkeys = (w.n0[1] << w.lf) * (w.n0[2] << w.lf)
    d_rows = torch.tensor([rec.rows_val.numel()], dtype=torch.int64, device="cuda")
    d_links = torch.tensor([emb.links.bins_val.numel()], dtype=torch.int64, device="cuda")
    rows = make_bins(GEO_BINS_ROWS, nkeys, rec.rows_off, rec.rows_val, rec.rows_val.numel(), d_rows)
    links = make_bins(GEO_BINS_LINKS, lvd.nblocks, emb.links.bins_off, emb.links.bins_val,
                      emb.links.bins_val.numel(), d_links)
    keep = (V, T, rec, child_maps, d_rows, d_links, emb)
    return make_mesh(V, T), lvd, rows, links, emb.links.n, keep


def _outputs(nb, cap):
    z = lambda n, dt: torch.full((max(n, 1),), -7, dtype=dt, device="cuda")
    return {"mask": z(nb * 64, torch.int32), "cell": z(cap, torch.int32), "dir": z(cap, torch.uint8),
            "q": z(cap, torch.float32), "tri": z(cap, torch.int32),
            "n": torch.zeros(1, dtype=torch.int64, device="cuda"),
            "stats": torch.zeros(GEO_NSTATS, dtype=torch.int64, device="cuda")}


def _host(o, n):
    return {k: (v.cpu().numpy() if k in ("mask", "n", "stats") else v[:n].cpu().numpy()) for k, v in o.items()}


def test_noalloc_equals_workspace_call_on_two_calls():
    from paper_2512_01251_amd import (GEO_CALL_CUTLINKS, GEO_NOALLOC_SCRATCH_BYTES, GEO_PREC_F32_FALLBACK,
                                      geo_cutlinks, geo_cutlinks_noalloc, geo_workspace_size)
    cases = [configs.star_small(lattice=27),
             configs.star_small(n_theta=14, n_phi=16, n0=32, lf=1, dtype=np.float32)]
    sizes = []
    for w in cases:
        mesh, lvd, rows, links, n, keep = _level_inputs(w)
        nb, cap = lvd.nblocks, n + 100
        need = geo_workspace_size(GEO_CALL_CUTLINKS, nb, cap)
        assert need <= GEO_NOALLOC_SCRATCH_BYTES
        sizes.append((nb, n))
        say(f"[no-alloc] {w.name}: {nb} blocks, {n} links, workspace {need} bytes")
        a = _outputs(nb, cap)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        geo_cutlinks(mesh, lvd, rows, links, w.lattice, GEO_PREC_F32_FALLBACK, a["mask"], cap, a["n"], a["cell"],
                     a["dir"], a["q"], a["tri"], a["stats"], ws)
        b = _outputs(nb, cap)
        geo_cutlinks_noalloc(mesh, lvd, rows, links, w.lattice, GEO_PREC_F32_FALLBACK, b["mask"], cap, b["n"],
                             b["cell"], b["dir"], b["q"], b["tri"], b["stats"])
        torch.cuda.synchronize()
        ha, hb = _host(a, n), _host(b, n)
        assert int(ha["n"][0]) == n and int(hb["n"][0]) == n
        for k in ha:
            assert np.array_equal(ha[k], hb[k]), k
        del keep
    assert sizes[1][0] < sizes[0][0] and sizes[1][1] < sizes[0][1]


def test_noalloc_rejects_a_request_over_its_scratch():
    from paper_2512_01251_amd import GEO_ERR_TOO_LARGE, GeoError
    w = configs.star_small(n_theta=14, n_phi=16, n0=32, lf=1, dtype=np.float32)
    mesh, lvd, rows, links, n, keep = _level_inputs(w)
    from paper_2512_01251_amd import GEO_PREC_F32_FALLBACK, geo_cutlinks_noalloc
    o = _outputs(lvd.nblocks, 1)
    with pytest.raises(GeoError, match=str(GEO_ERR_TOO_LARGE)):
        geo_cutlinks_noalloc(mesh, lvd, rows, links, w.lattice, GEO_PREC_F32_FALLBACK, o["mask"], 1 << 26,
                             o["n"], o["cell"], o["dir"], o["q"], o["tri"], o["stats"])
