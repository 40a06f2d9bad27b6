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
