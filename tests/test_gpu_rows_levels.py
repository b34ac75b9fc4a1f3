"""ROWS bins of several levels from one call against one call per level.

The joint pass must give each level exactly the bins of the per-level call:
identical offsets and counts and the same entries in every line (the order
within a line is unspecified in both), with the same number of float64 and
exact predicate evaluations.  The solid flags that the pipeline builds from
the joint bins are checked against the oracle by the parity tests.  When one
level overflows its capacity, every level's count is still exact."""
import numpy as np
import pytest
import torch

from synth import configs
from gpu_helpers import say, to_gpu

pytestmark = pytest.mark.gpu

CASES = {
    "star_small": lambda: configs.star_small(),
    "star_small_f32verts": lambda: configs.star_small(dtype=np.float32, n_theta=30, n_phi=34),
    "box_small": lambda: configs.box_small(lf=3),
    "icosphere64": lambda: configs.icosphere64(),
}


def _nkeys(n0, L):
    return (n0[1] << L) * (n0[2] << L)


def _level_desc(geo, n0, L):
    lv = geo.geo_level()
    for a in range(3):
        lv.n0[a] = int(n0[a])
    lv.level = L
    lv.nblocks = 0
    return lv


def _alloc(geo, n0, L, cap, counter):
    nk = _nkeys(n0, L)
    off = torch.full((nk + 1,), -7, dtype=torch.int32, device="cuda")
    val = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    return off, val, geo.make_bins(geo.GEO_BINS_ROWS, nk, off, val, cap, counter)


def _per_level(geo, mesh, n0, L, prec, cap=None):
    if cap is None:  # sized by a first call that only counts
        cap = _per_level(geo, mesh, n0, L, prec, 0)[2]
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    stats = torch.zeros(geo.GEO_NSTATS, dtype=torch.int64, device="cuda")
    off, val, bins = _alloc(geo, n0, L, cap, cnt)
    ws = torch.empty(geo.geo_workspace_size(geo.GEO_CALL_BINS_ROWS, _nkeys(n0, L), cap), dtype=torch.uint8,
                     device="cuda")
    geo.geo_build_bins(mesh, _level_desc(geo, n0, L), geo.GEO_BINS_ROWS, prec, bins, stats, ws)
    torch.cuda.synchronize()
    return off.cpu().numpy(), val.cpu().numpy(), int(cnt.item()), stats.cpu().numpy()


def _joint(geo, mesh, n0, lmin, caps, prec):
    cnt = torch.zeros(len(caps), dtype=torch.int64, device="cuda")
    stats = torch.zeros(geo.GEO_NSTATS, dtype=torch.int64, device="cuda")
    outs, bins = [], []
    for i, cap in enumerate(caps):
        off, val, b = _alloc(geo, n0, lmin + i, cap, cnt[i:i + 1])
        outs.append((off, val))
        bins.append(b)
    nk = sum(_nkeys(n0, lmin + i) for i in range(len(caps)))
    ws = torch.empty(geo.geo_workspace_size(geo.GEO_CALL_BINS_ROWS_LEVELS, nk, sum(caps)), dtype=torch.uint8,
                     device="cuda")
    geo.geo_build_row_bins_levels(mesh, n0, lmin, prec, bins, stats, ws)
    torch.cuda.synchronize()
    return [(o.cpu().numpy(), v.cpu().numpy()) for o, v in outs], cnt.cpu().numpy().tolist(), stats.cpu().numpy()


def _canonical(off, val, n):
    """Entries sorted by (line, value): the bins' content with the order
    within each line removed."""
    line = np.repeat(np.arange(len(off) - 1), np.diff(off))
    v = val[:n]
    return v[np.lexsort((v, line))]


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("name", list(CASES))
def test_joint_row_bins_equal_the_per_level_calls(name, precision):
    import paper_2512_01251_amd as geo
    w = CASES[name]()
    prec = geo.GEO_PREC_F32_FALLBACK if precision == "f32" else geo.GEO_PREC_F64
    V, T = to_gpu(w.mesh)
    mesh = geo.make_mesh(V, T)
    say(f"[rows-levels] {name} {precision} nt={w.mesh.nt} n0={w.n0} levels 0..{w.lf}")
    ref = [_per_level(geo, mesh, w.n0, L, prec) for L in range(w.lf + 1)]
    counts = [r[2] for r in ref]
    assert all(c > 0 for c in counts)
    for lmin in sorted({0, min(1, w.lf)}):
        levels = range(lmin, w.lf + 1)
        got, gcnt, gst = _joint(geo, mesh, w.n0, lmin, [counts[L] + 5 for L in levels], prec)
        assert gcnt == [counts[L] for L in levels], (gcnt, counts)
        for (off, val), L in zip(got, levels):
            roff, rval, n, _ = ref[L]
            assert np.array_equal(off, roff), f"offsets of level {L}"
            assert np.array_equal(_canonical(off, val, n), _canonical(roff, rval, n)), f"entries of level {L}"
            assert (val[n:] == -7).all(), f"level {L} wrote beyond its count"
        st_ref = sum(ref[L][3] for L in levels)
        assert gst[0] == st_ref[0] and gst[1] == st_ref[1], (gst[:2], st_ref[:2])
    say(f"[rows-levels] {name} {precision}: entries per level {counts}")


def test_overflow_of_one_level_keeps_every_count_exact():
    import paper_2512_01251_amd as geo
    w = configs.star_small()
    V, T = to_gpu(w.mesh)
    mesh = geo.make_mesh(V, T)
    prec = geo.GEO_PREC_F32_FALLBACK
    counts = [_per_level(geo, mesh, w.n0, L, prec, 0)[2] for L in range(w.lf + 1)]
    caps = list(counts)
    caps[1] = counts[1] // 2
    say(f"[rows-levels] overflow: counts {counts}, caps {caps}")
    _, gcnt, _ = _joint(geo, mesh, w.n0, 0, caps, prec)
    assert gcnt == counts
    # capacity 0 on every level: nothing is written, every count exact
    got, gcnt, _ = _joint(geo, mesh, w.n0, 0, [0] * (w.lf + 1), prec)
    assert gcnt == counts
    assert all((v == -7).all() for _, v in got)
