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
    # restriction + prolongation on the facet-trace form (4 of 10 rows or
    # columns of each off-diagonal block stored; D^{-1} and the diagonal
    # blocks as upper triangles, 55 of 100 values; the transfers formed on the
    # fly), and the parts sum to the total
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    assert [b.facet_nodes(2, q) for q in (3, 6, 10)] == [2, 3, 4]
    assert [b.facet_nodes(3, q) for q in (4, 10, 20)] == [3, 6, 10]
    sizes = [199712, 25657, 7215, 2210, 696, 217]
    nnzb = [797584, 161839, 48405, 14986, 4672, 1411]
    t = b.iteration_bytes(sizes, nnzb, 10, 4, 3)
    assert abs(t["total"] - sum(v for k, v in t.items() if k != "total")) < 1
    n0, p2, pk, off = sizes[0], 100, 55, nnzb[0] - sizes[0]
    sweep = b.smoother_bytes(nnzb[0], n0, 10, 4, 4, 3)
    assert sweep == off * 40 * 4 + 15 * n0 + n0 * pk * 4 + 3 * n0 * 10 * 4
    assert b.smoother_bytes(nnzb[0], n0, 10, 4, 4, 3, sym=False) == sweep + n0 * (p2 - pk) * 4
    # the transfers form L_e from each element's 2 + 4 map values, its parent
    # index and the parents' 100 monomial coefficients
    tr = n0 * 6 * 4 + 4 * n0 + sizes[1] * p2 * 4
    restrict = off * 40 * 4 + 15 * n0 + n0 * pk * 4 + tr + 3 * n0 * 10 * 4 + n0 * 10 * 4
    level0 = ((n0 * 10 * 8 + n0 * pk * 4 + 2 * n0 * 10 * 4) + sweep + restrict
              + (tr + 2 * n0 * 10 * 4 + sizes[1] * 10 * 4) + 2 * sweep + n0 * 10 * 8)
    assert t["level0"] == level0
    spmv = n0 * pk * 8 + off * 40 * 8 + 15 * n0 + 3 * n0 * 10 * 8
    assert b.spmv_bytes(nnzb[0], n0, 10, 4, 3) == spmv
    assert t["outer"] == (n0 * 10 * 4 + 2 * n0 * 10 * 8) + spmv + 6 * n0 * 10 * 8


def test_byte_model_3d_p3_figures():
    # the 3D p = 3 (n_p = 20) workload of 384 000 tetrahedra, 1 900 800 block
    # slots and 22 569 level-1 aggregates: facet-trace blocks keep 10 of 20
    # rows or columns, the packed blocks 210 of 400 values, each element's
    # map 3 + 9 values; these are the per-launch figures the kernel-trace
    # summaries quote
    from paper_2012_08024_amd import bytemodel as bm
    n0, nnzb0, n1 = 384000, 1900800, 22569
    assert bm.facet_nodes(3, 20) == 10 and bm.row_block(20) == 210
    sweep = bm.smoother_bytes(nnzb0, n0, 20, 4, 10, 4)
    assert sweep == (nnzb0 - n0) * 20 * 10 * 4 + 5 * 4 * n0 + n0 * 210 * 4 + 3 * n0 * 20 * 4 == 1635840000
    tr = bm.transfer0_bytes(n0, n1, 20, 4, 4)
    assert tr == n0 * 12 * 4 + 4 * n0 + n1 * 400 * 4
    assert bm.restrict_bytes(nnzb0, n0, 20, 4, 10, 4, True, n1) + n0 * 20 * 4 == 1722638400
    assert bm.spmv_bytes(nnzb0, n0, 20, 10, 4) == 3264000000
