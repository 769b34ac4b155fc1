"""The host half of the library (topology, switch, greedy agglomeration, the
kappa-free element blocks, bases, transfers, Galerkin and flux plans and the
host-formed level operators) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on several meshes and options: no
sanitizer report, and the same results as the regular build (through the C
ABI).  CPU only."""
import importlib.util
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2012_08024_amd")

if shutil.which("g++") is None:  # pragma: no cover
    pytest.skip("no g++", allow_module_level=True)

import paper_2012_08024_amd as cm  # noqa: E402

# (dim, n, p, levels, coarsening, switch_mode, seed)
CASES = [
    (2, 12, 3, 4, 0, 0, 12),
    (2, 10, 2, 3, 1, 1, 7),
    (2, 9, 1, 5, 1, 0, 3),
    (3, 3, 2, 3, 0, 0, 13),
    (3, 3, 1, 3, 1, 1, 5),
    (3, 2, 3, 2, 0, 0, 17),
]


def _write_case(path, d, n, p, levels, coarsening, mode, seed):
    m = mesh2d_jittered_delaunay(n, seed % 5) if d == 2 else mesh3d_kuhn(n, seed % 5)
    kappa = np.random.default_rng(seed).uniform(0.5, 2.0, m.n_elem)
    with open(path, "wb") as fh:
        fh.write(struct.pack("<6iQqq", d, p, levels, coarsening, mode, 0, seed, m.coords.shape[0], m.n_elem))
        fh.write(np.ascontiguousarray(m.coords, dtype="<f8").tobytes())
        fh.write(np.ascontiguousarray(m.e2v, dtype="<i4").tobytes())
        fh.write(np.ascontiguousarray(m.face_bc, dtype="i1").tobytes())
        fh.write(np.ascontiguousarray(kappa, dtype="<f8").tobytes())
    return m, kappa


def _expected(m, kappa, d, p, levels, coarsening, mode, seed):
    """The driver's summaries from the regular library build."""
    out = []
    hosted = cm.switch(m, mode, seed).reshape(-1).astype(np.int64)
    w = np.arange(hosted.size) % 9973 + 1
    out.append(("switch", int(np.dot(hosted, w))))
    parents, sizes = cm.agglomerate(m, levels, seed, p=p)
    out.append(("levels", [int(x) for x in sizes]))
    for l in range(len(sizes)):
        rp, cols, blk = cm.debug_host_operator(m, p, kappa, parents, sizes, l, coarsening=coarsening,
                                               switch_mode=mode, switch_seed=seed)
        b = blk.reshape(-1)
        wb = np.arange(b.size) % 101 + 1
        wc = np.arange(cols.size) % 7 + 1
        out.append(("level", l, len(cols), int(np.dot(cols.astype(np.int64), wc)), float(np.abs(b).sum()),
                    float(np.dot(b, wb))))
    return out


def _parse(lines):
    out = []
    for ln in lines:
        t = ln.split()
        if t[0] == "switch":
            out.append(("switch", int(t[1])))
        elif t[0] == "levels":
            out.append(("levels", [int(x) for x in t[1:]]))
        elif t[0] == "level":
            out.append(("level", int(t[1]), int(t[3]), int(t[5]), float(t[7]), float(t[9])))
    return out


@pytest.fixture(scope="module")
def host_check(tmp_path_factory):
    spec = importlib.util.spec_from_file_location("_cdgmg_build", os.path.join(PKG, "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b.build_host_check(str(tmp_path_factory.mktemp("sanitize")))


def test_host_half_under_sanitizers(host_check, tmp_path):
    files, expected = [], []
    for k, case in enumerate(CASES):
        path = str(tmp_path / ("case%d.bin" % k))
        m, kappa = _write_case(path, *case)
        files.append(path)
        d, n, p, levels, coarsening, mode, seed = case
        expected.append(_expected(m, kappa, d, p, levels, coarsening, mode, seed))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([host_check] + files, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    blocks = r.stdout.split("case ")[1:]
    assert len(blocks) == len(CASES)
    for blk, exp in zip(blocks, expected):
        got = _parse(blk.strip().splitlines()[1:])
        assert len(got) == len(exp)
        for g, e in zip(got, exp):
            assert g[:4] == e[:4], (g, e)
            if g[0] == "level":
                assert abs(g[4] - e[4]) <= 1e-12 * abs(e[4]) and abs(g[5] - e[5]) <= 1e-12 * abs(e[4]), (g, e)
