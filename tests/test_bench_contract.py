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
