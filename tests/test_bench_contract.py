"""bench.py on the host: more than one GPU is refused with a message (the
multi-GPU sharding is a design, not an implementation), before any device is
touched; and the HBM traffic figure is taken from the committed counter
profile only while the kernel it was measured on is unchanged."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr



def _copy_sources(sources, tmp_path, edit):
    """Copies of the q kernel's sources, the one named in edit changed."""
    out = []
    for p in sources:
        text = open(p, "rb").read()
        name = os.path.basename(p)
        if name in edit:
            text = edit[name](text)
        q = tmp_path / name
        q.write_bytes(text)
        out.append(str(q))
    return out


def test_traffic_is_taken_only_for_the_profiled_kernel(tmp_path, monkeypatch):
    """The counter profile names the sha256 of the kernel it was taken on:
    traffic is reported for that kernel and null once its device code (the
    kernel file, or the shared header above its host-side declarations)
    changes; a change to the host-side declarations alone keeps it."""
    import bench
    # a profile of the sources as they stand (the committed one may lag a
    # kernel change until the counters are taken again)
    prof = tmp_path / "profile.txt"
    prof.write_text(f"source_sha256: {bench.q_kernel_source_hash()}\ntraffic_bytes_per_launch: 123.0\n")
    monkeypatch.setattr(bench, "PMC_PROFILE", str(prof))
    c = bench.q_kernel_counters()
    assert c["traffic"] == 123.0, c["source"]

    marker = b"// host-side launchers"
    cases = {
        "kernel": ({"geo_cutlinks.hip": lambda t: t + b"\n// changed\n"}, False),
        "header device part": ({"geo_internal.h": lambda t: t.replace(marker, b"// changed\n" + marker, 1)}, False),
        "header host part": ({"geo_internal.h": lambda t: t + b"\n// changed\n"}, True),
    }
    sources = list(bench.Q_KERNEL_SOURCES)
    assert marker in open(sources[1], "rb").read()
    for name, (edit, kept) in cases.items():
        d = tmp_path / name.replace(" ", "_")
        d.mkdir()
        monkeypatch.setattr(bench, "Q_KERNEL_SOURCES", _copy_sources(sources, d, edit))
        c = bench.q_kernel_counters()
        assert (c["traffic"] is not None) == kept, (name, c["source"])


def test_cpu_baseline_leg_runs_on_the_host():
    """bench.py's cpu_baseline leg end to end on a small workload, fed the
    oracle's own embedding in place of the GPU's (CPU tensors): every field
    is produced, and the error against the oracle is zero on every output."""
    from types import SimpleNamespace as NS

    import numpy as np
    import torch

    import bench
    import oracle
    from synth import configs
    w = configs.star_small()
    ref = oracle.embed(w.mesh, w.n0, w.lf, w.lattice, w.d_spec)
    levels = [NS(level=r["level"], bcoord=torch.from_numpy(r["bcoord"]),
                 solid=torch.from_numpy(r["solid"].view(np.int64))) for r in ref["levels"]]
    rl = ref["links"]
    links = NS(n=rl["n"], cell=torch.from_numpy(rl["cell"]), dir=torch.from_numpy(rl["dir"]),
               q=torch.from_numpy(rl["q"].astype(np.float32)), tri=torch.from_numpy(rl["tri"]))
    res = bench.cpu_baseline(w, NS(levels=levels, links=links), chunk_blocks=40, min_seconds=0.0, max_chunks=1,
                             n_links=200, n_links_1t=50, n_blocks=20)
    assert res["kind"] == "oracle" and res["cores"] >= 1 and res["cpu_model"]
    for k in ("value", "mcells_per_s_1thread", "mlinks_per_s", "mlinks_per_s_1thread"):
        assert res[k] > 0, k
    e = res["error_vs_oracle"]
    assert e["solid_mismatches"] == 0 and e["link_set_mismatches"] == 0
    assert e["q_max_abs_err"] <= 1e-6 and e["tri_mismatches_untied"] == 0
