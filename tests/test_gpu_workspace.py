"""The device workspace of the C ABI (caller-owned, sized by
cdgmg_workspace_size), run-to-run determinism, and the singular operator of a
problem with only Neumann boundaries."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2012_08024_amd as cm  # noqa: E402
from oracle.mesh import Topology  # noqa: E402
from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn, source_sine  # noqa: E402


def _raw_setup(mesh, p, kappa, parents, sizes, nbytes, ws_bytes, **kw):
    """cdgmg_setup through ctypes with a torch workspace of ws_bytes."""
    hm = cm.HostMesh.of(mesh)
    hier, keep = cm._hierarchy(parents, sizes)
    opts = cm.default_options(**kw)
    k = torch.tensor(kappa, dtype=torch.float64, device="cuda")
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    rc = cm.lib.cdgmg_setup(ctypes.byref(hm.c), p, k.data_ptr(), ctypes.byref(hier), ctypes.byref(opts),
                            ws.data_ptr(), ws_bytes, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                            ctypes.byref(h))
    return rc, h, ws


@pytest.mark.parametrize("d,n,p,levels,kw", [(2, 12, 3, 4, {}), (3, 4, 2, 3, {"mg_precision": cm.MG_FP64}),
                                             (2, 10, 2, 3, {"outer": cm.OUTER_GMRES, "restart": 7}),
                                             (2, 10, 3, 3, {"p_coarse": 1}),
                                             (2, 9, 2, 3, {"coarsening": cm.COARSEN_FLUX})])
def test_workspace_exact_size(d, n, p, levels, kw):
    mesh = mesh2d_jittered_delaunay(n, 1) if d == 2 else mesh3d_kuhn(n, 1)
    parents, sizes = cm.agglomerate(mesh, levels, 3, p=p)
    kappa = np.random.default_rng(1).uniform(0.5, 2.0, mesh.n_elem)
    kw = dict(kw, tol=1e-11)
    nbytes = cm.workspace_size(mesh, p, parents, sizes, **kw)
    print("case", d, n, p, kw, "workspace", nbytes, flush=True)
    # one byte short: refused before any kernel runs, naming the size needed
    rc, h, ws = _raw_setup(mesh, p, kappa, parents, sizes, nbytes, nbytes - 1, **kw)
    assert rc == -1 and not h.value
    assert str(nbytes) in cm.last_error()
    rc, h, ws = _raw_setup(mesh, p, kappa, parents, sizes, nbytes, nbytes, **kw)
    assert rc == 0
    cm.lib.cdgmg_destroy(h)
    # exactly the size: the solve equals the one of a Solver (own workspace)
    s = cm.Solver(mesh, p, kappa, parents, sizes, **kw)
    assert s.device_bytes() == nbytes and s.workspace.numel() == nbytes
    f = source_sine(s.node_coords().reshape(-1, d))
    u1, i1 = s.solve(f)
    s.close()
    rc, h, ws = _raw_setup(mesh, p, kappa, parents, sizes, nbytes, nbytes, **kw)
    assert rc == 0
    ft = torch.tensor(f, device="cuda")
    u2 = torch.empty_like(ft)
    info = cm._Info()
    assert cm.lib.cdgmg_solve(h, ft.data_ptr(), u2.data_ptr(), ctypes.byref(info)) == 0
    cm.lib.cdgmg_destroy(h)
    assert info.iterations == i1.iterations
    assert torch.equal(u1, u2)


def test_workspace_argument_checks():
    mesh = mesh2d_jittered_delaunay(6, 1)
    parents, sizes = cm.agglomerate(mesh, 2, 1, p=1)
    nbytes = cm.workspace_size(mesh, 1, parents, sizes)
    hm = cm.HostMesh.of(mesh)
    hier, keep = cm._hierarchy(parents, sizes)
    opts = cm.default_options()
    k = torch.ones(mesh.n_elem, dtype=torch.float64, device="cuda")
    ws = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    for ptr in (0, ws.data_ptr() + 8):  # null, misaligned
        rc = cm.lib.cdgmg_setup(ctypes.byref(hm.c), 1, k.data_ptr(), ctypes.byref(hier), ctypes.byref(opts),
                                ptr, nbytes, None, ctypes.byref(h))
        assert rc == -1 and not h.value


def test_two_solves_are_bitwise_identical():
    # fixed-order reductions and no atomics: the same solve twice, and on a
    # second handle, gives the same bits and the same iteration count
    mesh = mesh2d_jittered_delaunay(40, 3)
    parents, sizes = cm.agglomerate(mesh, 5, 12, p=3)
    kappa = np.random.default_rng(2).uniform(0.5, 2.0, mesh.n_elem)
    s1 = cm.Solver(mesh, 3, kappa, parents, sizes)
    f = source_sine(s1.node_coords().reshape(-1, 2))
    ua, ia = s1.solve(f, history=True)
    ub, ib = s1.solve(f, history=True)
    s2 = cm.Solver(mesh, 3, kappa, parents, sizes)
    uc, ic = s2.solve(f, history=True)
    assert ia.iterations == ib.iterations == ic.iterations
    assert torch.equal(ua, ub) and torch.equal(ua, uc)
    assert np.array_equal(ia.history, ib.history) and np.array_equal(ia.history, ic.history)
    g = s1.grad_kappa(ua, ub)
    assert torch.equal(g, s2.grad_kappa(ua, ub))
    s1.close()
    s2.close()


@pytest.mark.parametrize("levels", [1, 3])
def test_neumann_only_operator_is_singular(levels):
    # with Neumann conditions on the whole boundary the constants are in the
    # kernel of A (A 1 = 0): the coarsest operator is singular and setup says so
    mesh = mesh2d_jittered_delaunay(8, 1)
    face_bc = np.ones_like(mesh.face_bc)
    hm = cm.HostMesh(mesh.coords, mesh.e2v, face_bc)
    parents, sizes = cm.agglomerate(hm, levels, 5, p=2)
    with pytest.raises(cm.CdgmgError) as ei:
        cm.Solver(hm, 2, np.ones(mesh.n_elem), parents, sizes)
    assert ei.value.code == -4, str(ei.value)
    # one Dirichlet facet makes it definite again
    e, i = sorted(Topology(mesh.e2v, mesh.coords).boundary)[0]
    face_bc[e, i] = 0
    hm = cm.HostMesh(mesh.coords, mesh.e2v, face_bc)
    s = cm.Solver(hm, 2, np.ones(mesh.n_elem), parents, sizes)
    s.close()
