"""bench.py contract checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "8", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _bench():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    return bench


def test_committed_counter_summaries_match_the_kernel_sources():
    # the roofline's traffic figures come from profiles/; they must describe the
    # kernels as committed (a summary for other sources reads as null)
    bench = _bench()
    assert bench.counter_traffic("k_push", "rmat22", "host", "partitioned", "bound") > 0
    assert bench.counter_traffic("k_step", "rmat22", "queued", "partitioned", "bound") > 0
    assert bench.batch_traffic("rmat22") > 0


def test_counter_summary_for_other_sources_or_settings_reads_as_none(tmp_path, monkeypatch):
    bench = _bench()
    assert bench.counter_traffic("k_push", "rmat22", "queued", "partitioned", "bound") is None
    assert bench.counter_traffic("k_push", "rmat22", "host", "plain", "bound") is None
    assert bench.counter_traffic("k_push", "grid2048", "host", "partitioned", "bound") is None
    # a copy of the tree whose batched kernel source differs by one byte
    fake = tmp_path / "root"
    (fake / "profiles").mkdir(parents=True)
    csrc = fake / "paper_2212_08200_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("gr_kernels.hip", "gr_device.h", "gr_internal.h", "gr_multi.hip", "gr_multi.h"):
        text = open(os.path.join(ROOT, "paper_2212_08200_amd", "csrc", f)).read()
        (csrc / f).write_text(text + (" " if f == "gr_multi.hip" else ""))
    name = "k_mq_batch_push_rmat22_counters.md"
    (fake / "profiles" / name).write_text(open(os.path.join(ROOT, "profiles", name)).read())
    monkeypatch.setattr(bench, "ROOT", str(fake))
    assert bench.batch_traffic("rmat22") is None
