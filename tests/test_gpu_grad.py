"""Backward of q (float32 atomics) vs the oracle's closed-form gradient."""
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
    say(f"[grad] {precision} links={rl['n']}")
    emb, V, T = gpu_embed(w, precision)
    Vg = V.clone().requires_grad_(True)
    q = pipeline.cut_link_q(Vg, T, emb)
    loss = (q.double() * torch.from_numpy(wts).cuda()).sum()
    loss.backward()
    g = Vg.grad.cpu().numpy()
    scale = np.abs(g_ref).max()
    err = np.abs(g - g_ref)
    say(f"[grad] {precision} max err {err.max():.3e} scale {scale:.3e}")
    assert err.max() <= 1e-4 * scale
