"""bench.py's command line on the CPU: more than one GPU is refused with a
message, and the kernel-source digest that gates the counter record is
stable and covers the step kernel's sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_source_digest():
    sys.path.insert(0, ROOT)
    import bench
    d = bench.kernel_source_digest()
    assert len(d) == 64 and d == bench.kernel_source_digest()
    assert any(p.endswith("step_fused.hip") for p in bench.KERNEL_SOURCES)
    assert bench.measured_record("no-such-precision", "bytes", 48) is None
    assert bench.measured_record("fp32srf", "bytes", None) is None


def test_binding_limit():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.binding_limit(0.31, {"frac": 0.71}) == "valu"
    assert bench.binding_limit(0.80, {"frac": 0.40}) == "hbm"
    assert bench.binding_limit(0.31, None) is None


def test_counter_record_covers_the_autotuner_choices():
    """The committed counter record holds positive HBM bytes and VALU instructions per launch for every
    benchmarked storage mode at 32 to 80 rows, the segment lengths the autotuner picks on the batch."""
    sys.path.insert(0, ROOT)
    import bench
    rec = {}
    with open(bench.TRAFFIC_RECORD) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    assert len(rec["kernel_sources_sha256"]) == 64
    for prec in ("fp32srf", "fp32", "fp64"):
        for seg in range(32, 81, 8):
            for what in ("bytes", "valu_insts"):
                assert float(rec["%s_per_launch_%s_seg%d" % (what, prec, seg)]) > 0, (what, prec, seg)


def test_timed_schedule_and_what_it_runs():
    """The timed region of the default run is whole graph replays each with one residual step; with fewer
    timed steps than a graph holds, the graph and the residual interval shrink to the timed count and the
    warm-up rounds up to whole graphs."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.timed_schedule(20000, 100, 100, 100) == (100, 100, 100)
    ex = bench.executed(100, 20000, 100, 100)
    assert (ex["graph_replays"], ex["eager_steps"], ex["residual_steps"]) == (200, 0, 200)
    G, R, W = bench.timed_schedule(20, 5, 100, 100)
    assert (G, R, W) == (20, 20, 20)
    ex = bench.executed(W, 20, G, R)
    assert (ex["graph_replays"], ex["eager_steps"], ex["residual_steps"]) == (1, 0, 1)
    assert bench.timed_schedule(7, 5, 100, 100) == (6, 6, 6)
    # without the adjustment, 20 steps from step 5 run eagerly with no residual step
    ex = bench.executed(5, 20, 100, 100)
    assert (ex["graph_replays"], ex["eager_steps"], ex["residual_steps"]) == (0, 20, 0)
    # a replay starts only at a multiple of the graph size: 70 eager steps, one replay, 80 eager steps
    ex = bench.executed(30, 250, 100, 50)
    assert (ex["graph_replays"], ex["eager_steps"], ex["residual_steps"]) == (1, 150, 5)
    assert "1 replays of a 100-step HIP graph" in bench.describe(ex) and "150 eager steps" in bench.describe(ex)
