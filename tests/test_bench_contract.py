"""Host-side parts of the benchmark contract (no GPU): one GPU only, and the
committed counter summary carries the per-launch traffic of every stencil
class the roofline line can name."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_lines_for_every_roofline_class():
    b = _bench()
    for cls, name in b.TRAFFIC_KERNEL.items():
        t = b.stored_traffic(name, "C3")
        assert t is not None and t > 0, (cls, name)
    # the dominant kernel's traffic is above its algorithmic bytes (10.07 GB
    # per 12-RHS FP32 launch of the q-recursion form on 32^3x64) and below
    # three times them
    t = b.stored_traffic(b.TRAFFIC_KERNEL["dslash_mrq_f32"], "C3")
    alg = 32 * 32 * 32 * 64 * (48 * 4 + 12 * 24 * 4 * 4)
    assert alg < t < 3 * alg
    assert b.stored_traffic("no_such_kernel", "C3") is None
