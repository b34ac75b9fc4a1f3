"""Backward of q (float32 atomics) vs the oracle's closed-form gradient.

Tolerances, per vertex component: the float32 atomic sum against the
oracle's float64 sum within 1e-4 G_abs, where G_abs = sum_i |w_i| |dq_i/dv|
is the sum of the magnitudes of the same terms (the scale of the rounding of
any order of summation); float64 central differences of the oracle's q
against the oracle's closed form within 1e-6 G_abs."""
import numpy as np
import pytest
import torch

import oracle
from synth import configs
from synth.weights import link_weights
from gpu_helpers import gpu_embed, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_backward_matches_oracle_gradient(precision):
    from paper_2512_01251_amd import pipeline
    w = configs.star_small()
    ref = oracle.embed(w.mesh, w.n0, w.lf, w.lattice, w.d_spec)
    rl, lv = ref["links"], ref["levels"][-1]
    wts = link_weights(w.lf, lv["bcoord"], rl["cell"], rl["dir"], seed=3)
    wts[rl["tied"] != 0] = 0.0     # the hit triangle is not unique there
    g_ref = oracle.grad(w.mesh, w.n0, w.lf, lv["bcoord"], rl["cell"], rl["dir"], rl["tri"], wts)
    g_abs = oracle.grad(w.mesh, w.n0, w.lf, lv["bcoord"], rl["cell"], rl["dir"], rl["tri"], wts, absolute=True)
    say(f"[grad] {precision} links={rl['n']}")
    emb, V, T = gpu_embed(w, precision)
    Vg = V.clone().requires_grad_(True)
    q = pipeline.cut_link_q(Vg, T, emb)
    loss = (q.double() * torch.from_numpy(wts).cuda()).sum()
    loss.backward()
    g = Vg.grad.cpu().numpy()
    err = np.abs(g - g_ref)
    say(f"[grad] {precision} max err {err.max():.3e}, max err / G_abs {np.max(err / np.maximum(g_abs, 1e-300)):.3e}")
    assert (err <= 1e-4 * g_abs).all()


_q112k = {}


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_backward_star112k(precision):
    """Loss L = sum w_i q_i on the 112,000-triangle star (levels 0..3, D3Q19),
    w_i ~ U(-1, 1) seeded: the float32 atomic backward against the oracle's
    closed-form gradient at every vertex, and on 64 random vertices against
    float64 central differences (h = 1e-6) of the oracle's q."""
    from paper_2512_01251_amd import pipeline
    w = configs.star112k()
    say(f"[grad] star112k {precision}")
    emb, V, T = gpu_embed(w, precision)
    lv = emb.levels[-1]
    bc = lv.bcoord.cpu().numpy()
    cell = emb.links.cell.cpu().numpy()
    dirs = emb.links.dir.cpu().numpy()
    tri = emb.links.tri.cpu().numpy()
    wts = link_weights(w.lf, bc, cell, dirs, seed=3)
    # the oracle's own nearest hits decide which links have a unique triangle
    t = cell % 64
    cells = 4 * bc[cell // 64] + np.stack([t & 3, (t >> 2) & 3, t >> 4], 1)
    key = (cell.tobytes().__hash__(), dirs.tobytes().__hash__())
    if _q112k.get("key") != key:  # the same table in both forms: computed once
        _q112k.update(key=key, ref=oracle.q_points(w.mesh, w.n0, w.lf, cells, dirs))
    ref = _q112k["ref"]
    assert np.abs(emb.links.q.cpu().numpy() - ref["q"]).max() <= 1e-5
    keep = (ref["tied"] == 0) & (ref["tri"] == tri)
    wts[~keep] = 0.0
    g_ref = oracle.grad(w.mesh, w.n0, w.lf, bc, cell, dirs, tri, wts)
    g_abs = oracle.grad(w.mesh, w.n0, w.lf, bc, cell, dirs, tri, wts, absolute=True)
    Vg = V.clone().requires_grad_(True)
    q = pipeline.cut_link_q(Vg, T, emb)
    (q.double() * torch.from_numpy(wts).cuda()).sum().backward()
    g = Vg.grad.cpu().numpy()
    err = np.abs(g - g_ref)
    say(f"[grad] star112k {precision}: {emb.links.n} links, max |g - g_oracle| {err.max():.3e}, "
        f"max err / G_abs {np.max(err / np.maximum(g_abs, 1e-300)):.3e}")
    assert (err <= 1e-4 * g_abs).all()
    # central differences of the loss in float64 on 64 random vertices that
    # move some link; links whose nearest triangle changes within +-h are left out
    rng = np.random.default_rng(4)
    tris = w.mesh.tris
    touched = np.unique(tris[tri[wts != 0]])
    h = 1e-6
    checked = 0
    for v in rng.choice(touched, 64, replace=False):
        sel = np.nonzero((wts != 0) & np.isin(tri, np.nonzero((tris == v).any(1))[0]))[0]
        for a in range(3):
            qs, ok = [], True
            for sgn in (1.0, -1.0):
                m = w.mesh.__class__(verts=w.mesh.verts.astype(np.float64).copy(), tris=tris)
                m.verts[v, a] += sgn * h
                r = oracle.q_points(m, w.n0, w.lf, cells[sel], dirs[sel])
                ok &= bool(np.array_equal(r["tri"], tri[sel]))
                qs.append(r["q"])
            if not ok:
                continue
            fd = float(np.dot(wts[sel], (qs[0] - qs[1]) / (2 * h)))
            # the difference quotient's own rounding: each q is the float64
            # nearest to the exact value (|q| <= 1), so it carries 2^-53 / h
            floor = 2.0 ** -53 * float(np.abs(wts[sel]).sum()) / h
            assert abs(fd - g_ref[v, a]) <= 1e-6 * g_abs[v, a] + floor, (v, a, fd, g_ref[v, a], g_abs[v, a])
            assert abs(fd - g[v, a]) <= 1e-4 * g_abs[v, a] + floor, (v, a, fd, g[v, a], g_abs[v, a])
            checked += 1
    say(f"[grad] star112k {precision}: {checked} central differences agree")
    assert checked >= 96
