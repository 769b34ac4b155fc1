"""cdgmg_setup_static: the setup that allocates nothing (its device arrays in
the library's static per-GPU workspace) against cdgmg_setup with a
caller-owned workspace, through the C ABI."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2012_08024_amd as cm  # noqa: E402
from workloads import mesh2d_jittered_delaunay, source_sine  # noqa: E402

STATIC_BYTES = 64 << 20


def _static_setup(mesh, p, kappa, parents, sizes, **kw):
    hm = cm.HostMesh.of(mesh)
    hier, keep = cm._hierarchy(parents, sizes)
    opts = cm.default_options(**kw)
    k = torch.tensor(kappa, dtype=torch.float64, device="cuda")
    h = ctypes.c_void_p()
    rc = cm.lib.cdgmg_setup_static(ctypes.byref(hm.c), p, k.data_ptr(), ctypes.byref(hier), ctypes.byref(opts),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
    return rc, h


def _solve(h, f):
    ft = torch.tensor(f, device="cuda")
    u = torch.empty_like(ft)
    info = cm._Info()
    rc = cm.lib.cdgmg_solve(h, ft.data_ptr(), u.data_ptr(), ctypes.byref(info))
    return rc, u, info


@pytest.mark.parametrize("p", [2, 3])
def test_static_setup_matches_workspace_setup(p):
    # two calls in a row on this GPU, the second on a smaller mesh: each
    # solve equals the one with a caller-owned workspace, bit for bit
    for n, levels in ((16, 3), (9, 2)):
        mesh = mesh2d_jittered_delaunay(n, 1)
        parents, sizes = cm.agglomerate(mesh, levels, 11, p=p)
        kappa = np.random.default_rng(n).uniform(0.5, 2.0, mesh.n_elem)
        assert cm.workspace_size(mesh, p, parents, sizes) <= STATIC_BYTES
        print("static setup", n, p, list(sizes), flush=True)
        ref = cm.Solver(mesh, p, kappa, parents, sizes, tol=1e-11)
        f = source_sine(ref.node_coords().reshape(-1, 2))
        u_ref, i_ref = ref.solve(f)
        g_ref = ref.grad_kappa(u_ref, u_ref)
        ref.close()
        rc, h = _static_setup(mesh, p, kappa, parents, sizes, tol=1e-11)
        assert rc == 0, cm.last_error()
        # the array is held: another static setup on this GPU is refused
        rc2, h2 = _static_setup(mesh, p, kappa, parents, sizes)
        assert rc2 == -1 and not h2.value and "held" in cm.last_error()
        rc, u, info = _solve(h, f)
        assert rc == 0
        assert info.iterations == i_ref.iterations
        assert torch.equal(u, u_ref)
        g = torch.empty(mesh.n_elem, dtype=torch.float64, device="cuda")
        assert cm.lib.cdgmg_grad_kappa(h, u.data_ptr(), u.data_ptr(), g.data_ptr()) == 0
        assert torch.equal(g, g_ref)
        assert cm.lib.cdgmg_destroy(h) == 0


def test_static_setup_refuses_a_problem_beyond_its_size():
    mesh = mesh2d_jittered_delaunay(64, 1)
    parents, sizes = cm.agglomerate(mesh, 5, 11, p=3)
    need = cm.workspace_size(mesh, 3, parents, sizes)
    assert need > STATIC_BYTES
    rc, h = _static_setup(mesh, 3, np.ones(mesh.n_elem), parents, sizes)
    assert rc == -1 and not h.value
    assert str(STATIC_BYTES) in cm.last_error() and str(need) in cm.last_error()
    # the array is free again afterwards
    small = mesh2d_jittered_delaunay(8, 1)
    ps, ss = cm.agglomerate(small, 2, 11, p=1)
    s = cm.Solver(small, 1, np.ones(small.n_elem), ps, ss, static_workspace=True)
    assert s.workspace is None
    u, info = s.solve(np.ones(small.n_elem * 3))
    assert info.rel_residual <= 1e-10
    s.close()
