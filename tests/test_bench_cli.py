"""bench.py's command line on the CPU: more than one GPU is refused with a
message (the path is built for one GPU), before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_iteration_byte_model_adds_up():
    # the per-level byte model used for the iteration-average rate: the
    # level-0 part at the 2D p=3 benchmark sizes is entry + 3 sweeps +
    # restriction + prolongation, and the parts sum to the total
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    sizes = [199712, 25657, 7215, 2210, 696, 217]
    nnzb = [797584, 161839, 48405, 14986, 4672, 1411]
    t = b.iteration_bytes(sizes, nnzb, 10)
    assert abs(t["total"] - sum(v for k, v in t.items() if k != "total")) < 1
    sweep = b.smoother_bytes(nnzb[0], sizes[0], 10, 4)
    n0, p2 = sizes[0], 100
    level0 = ((n0 * 10 * 8 + n0 * p2 * 4 + 2 * n0 * 10 * 4) + sweep + (sweep + n0 * p2 * 4)
              + (n0 * p2 * 4 + 2 * n0 * 10 * 4 + 4 * n0 + sizes[1] * 10 * 4) + 2 * sweep + n0 * 10 * 8)
    assert t["level0"] == level0
    assert t["outer"] == (n0 * 10 * 4 + 2 * n0 * 10 * 8) + b.spmv_bytes(nnzb[0], n0, 10) + 6 * n0 * 10 * 8
