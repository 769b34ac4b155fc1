"""Python binding of libcdgmg (agglomeration multigrid for CDG on gfx950).

Argument marshalling only: every step of the discretisation and the solve
runs inside the shared library (host C++ setup and HIP kernels).  Device
arrays are torch tensors on the current CUDA (HIP) device; the library works
on torch's current stream.  Importing this package raises ImportError when
the compiled library is missing: there is no fallback path.
"""
import ctypes
import os

import numpy as np
# torch before the library: torch ships its own HIP runtime under the same
# soname, and whichever is loaded first serves the whole process, so loading
# torch first makes the library run on torch's runtime and device context
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libcdgmg.so")
if not os.path.exists(_LIBPATH):
    raise ImportError("libcdgmg.so is not built; run paper_2012_08024_amd/build.py "
                      "(or __graft_entry__.build()) first")
lib = ctypes.CDLL(_LIBPATH)

OK, NOT_CONVERGED = 0, 1
MG_FP64, MG_FP32 = 0, 1
OUTER_FCG, OUTER_PCG, OUTER_GMRES = 0, 1, 2
COARSEN_PRIMAL, COARSEN_FLUX = 0, 1
SWITCH_CONSISTENT, SWITCH_NATURAL = 0, 1
K_NAMES = ["spmv", "smooth0", "smooth", "restrict", "prolong", "coarse", "vector", "unused"]
NK = 8


class CdgmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("cdgmg error %d: %s" % (code, msg))
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_vert", ctypes.c_int64), ("coords", ctypes.c_void_p),
                ("n_elem", ctypes.c_int64), ("e2v", ctypes.c_void_p), ("face_bc", ctypes.c_void_p)]


class _Hier(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("level_sizes", ctypes.c_void_p), ("parent", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("omega", ctypes.c_double), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("mg_precision", ctypes.c_int), ("outer", ctypes.c_int),
                ("coarsening", ctypes.c_int), ("switch_mode", ctypes.c_int),
                ("switch_seed", ctypes.c_uint64), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("profile", ctypes.c_int), ("kernel_variant", ctypes.c_int), ("restart", ctypes.c_int),
                ("beta", ctypes.c_double), ("velocity", ctypes.c_double * 3), ("p_coarse", ctypes.c_int),
                ("p_jump", ctypes.c_int), ("coarse_group", ctypes.c_int), ("row_threads", ctypes.c_int),
                ("coarse_fp64", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("conv_factor", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double * NK), ("kernel_launches", ctypes.c_int64 * NK),
                ("history", ctypes.c_void_p), ("history_len", ctypes.c_int)]


_vp, _i, _i64, _u64, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
_SIGS = {
    "cdgmg_version": ([], _i),
    "cdgmg_last_error": ([], ctypes.c_char_p),
    "cdgmg_default_options": ([_vp], None),
    "cdgmg_agglomerate": ([_vp, _i, _i64, _i, _u64, _vp, _vp, _vp], _i),
    "cdgmg_switch": ([_vp, _i, _u64, _vp], _i),
    "cdgmg_workspace_size": ([_vp, _i, _vp, _vp, _vp], _i),
    "cdgmg_setup": ([_vp, _i, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp], _i),
    "cdgmg_setup_static": ([_vp, _i, _vp, _vp, _vp, _vp, _vp], _i),
    "cdgmg_update_kappa": ([_vp, _vp], _i),
    "cdgmg_solve": ([_vp, _vp, _vp, _vp], _i),
    "cdgmg_solve_rhs": ([_vp, _vp, _vp, _vp], _i),
    "cdgmg_solve_transpose": ([_vp, _vp, _vp, _vp], _i),
    "cdgmg_grad_kappa": ([_vp, _vp, _vp, _vp], _i),
    "cdgmg_apply_mass": ([_vp, _vp, _vp], _i),
    "cdgmg_apply_A": ([_vp, _i, _i, _vp, _vp], _i),
    "cdgmg_vcycle": ([_vp, _vp, _vp], _i),
    "cdgmg_level_info": ([_vp, _vp, _vp, _vp], _i),
    "cdgmg_launch_info": ([_vp, _vp, _vp, _vp, _vp, _vp], _i),
    "cdgmg_export_operator": ([_vp, _i, _vp, _vp, _vp, _vp], _i),
    "cdgmg_node_coords": ([_vp, _vp], _i),
    "cdgmg_device_bytes": ([_vp, _vp], _i),
    "cdgmg_set_profile": ([_vp, _i], _i),
    "cdgmg_destroy": ([_vp], _i),
    "cdgmg_debug_host_operator": ([_vp, _i, _vp, _vp, _vp, _i, _vp, _vp, _vp, _vp], _i),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = sorted(_SIGS)


def last_error():
    return lib.cdgmg_last_error().decode()


def _check(rc, allow_warning=False):
    if rc < 0 or (rc > 0 and not allow_warning):
        raise CdgmgError(rc, last_error())
    return rc


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def n_basis(dim, p):
    return (p + 1) * (p + 2) // 2 if dim == 2 else (p + 1) * (p + 2) * (p + 3) // 6


class HostMesh:
    """Contiguous host copies of a mesh (float64 coords, int32 e2v, int8 face_bc)."""

    def __init__(self, coords, e2v, face_bc):
        self.coords = np.ascontiguousarray(coords, dtype=np.float64)
        self.e2v = np.ascontiguousarray(e2v, dtype=np.int32)
        self.face_bc = np.ascontiguousarray(face_bc, dtype=np.int8)
        self.dim = self.coords.shape[1]
        self.n_elem = self.e2v.shape[0]
        self.c = _Mesh(self.dim, self.coords.shape[0], _ptr(self.coords).value, self.n_elem,
                       _ptr(self.e2v).value, _ptr(self.face_bc).value)

    @classmethod
    def of(cls, mesh):
        return cls(mesh.coords, mesh.e2v, mesh.face_bc)


def agglomerate(mesh, max_levels, seed, p=1, coarse_dofs=0):
    """Greedy agglomeration; returns (list of parent maps, level sizes)."""
    hm = mesh if isinstance(mesh, HostMesh) else HostMesh.of(mesh)
    parents = np.zeros(hm.n_elem * max(max_levels, 1), dtype=np.int32)
    sizes = np.zeros(max(max_levels, 1) + 1, dtype=np.int32)
    nl = ctypes.c_int(0)
    _check(lib.cdgmg_agglomerate(ctypes.byref(hm.c), max_levels, coarse_dofs, p, seed,
                                 _ptr(parents), _ptr(sizes), ctypes.byref(nl)))
    sizes = sizes[:nl.value].copy()
    out, off = [], 0
    for l in range(nl.value - 1):
        out.append(parents[off:off + sizes[l]].copy())
        off += sizes[l]
    return out, sizes


def switch(mesh, mode=SWITCH_CONSISTENT, seed=0):
    """Hosted-facet flags int8 [n_elem, dim+1] of the CDG switch."""
    hm = mesh if isinstance(mesh, HostMesh) else HostMesh.of(mesh)
    out = np.zeros((hm.n_elem, hm.dim + 1), dtype=np.int8)
    _check(lib.cdgmg_switch(ctypes.byref(hm.c), mode, seed, _ptr(out)))
    return out


def default_options(**kw):
    o = _Opts()
    lib.cdgmg_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k == "velocity":
            v = (list(v) + [0.0, 0.0, 0.0])[:3]
            o.velocity = (ctypes.c_double * 3)(*v)
        else:
            setattr(o, k, v)
    return o


def _hierarchy(parents, sizes):
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    par = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.int32) for x in parents])
                               if len(parents) else np.zeros(0, dtype=np.int32))
    return _Hier(len(sizes), _ptr(sizes).value, _ptr(par).value), (sizes, par)


def workspace_size(mesh, p, parents, sizes, options=None, **kw):
    """Device bytes cdgmg_setup needs (runs the host half of setup; no GPU)."""
    hm = mesh if isinstance(mesh, HostMesh) else HostMesh.of(mesh)
    hier, keep = _hierarchy(parents, sizes)
    opts = options if options is not None else default_options(**kw)
    nbytes = ctypes.c_size_t(0)
    _check(lib.cdgmg_workspace_size(ctypes.byref(hm.c), p, ctypes.byref(hier), ctypes.byref(opts),
                                    ctypes.byref(nbytes)))
    return nbytes.value


def debug_host_operator(mesh, p, kappa, parents, sizes, level, **options):
    """A_level formed on the host from the library's setup data (CPU test support).
    Returns (row_ptr, cols, blocks) in hierarchy numbering."""
    hm = mesh if isinstance(mesh, HostMesh) else HostMesh.of(mesh)
    npb = n_basis(hm.dim, p)
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    par = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.int32) for x in parents])
                               if len(parents) else np.zeros(0, dtype=np.int32))
    hier = _Hier(len(sizes), _ptr(sizes).value, _ptr(par).value)
    kappa = np.ascontiguousarray(kappa, dtype=np.float64)
    opts = default_options(**options)
    nnzb = ctypes.c_int64(0)
    args = (ctypes.byref(hm.c), p, _ptr(kappa), ctypes.byref(hier), ctypes.byref(opts), level)
    _check(lib.cdgmg_debug_host_operator(*args, ctypes.byref(nnzb), None, None, None))
    rp = np.zeros(int(sizes[level]) + 1, dtype=np.int64)
    cols = np.zeros(nnzb.value, dtype=np.int32)
    blocks = np.zeros((nnzb.value, npb, npb))
    _check(lib.cdgmg_debug_host_operator(*args, ctypes.byref(nnzb), _ptr(rp), _ptr(cols), _ptr(blocks)))
    return rp, cols, blocks


def bsr_to_scipy(rp, cols, blocks):
    import scipy.sparse as sp
    n = len(rp) - 1
    return sp.bsr_matrix((blocks, cols, rp), shape=(n * blocks.shape[1], n * blocks.shape[1])).tocsr()


class SolveInfo:
    def __init__(self, c, hist):
        self.iterations = c.iterations
        self.rel_residual = c.rel_residual
        self.conv_factor = c.conv_factor
        self.solve_ms = c.solve_ms
        self.kernel_ms = {K_NAMES[k]: c.kernel_ms[k] for k in range(NK)}
        self.kernel_launches = {K_NAMES[k]: c.kernel_launches[k] for k in range(NK)}
        self.history = hist[:self.iterations].copy() if hist is not None else None

    def __repr__(self):
        return "SolveInfo(iterations=%d, rel_residual=%.3e, conv_factor=%.3f, solve_ms=%.3f)" % (
            self.iterations, self.rel_residual, self.conv_factor, self.solve_ms)


class Solver:
    """setup(mesh, p, kappa, hierarchy) -> solve(f) -> u on the current GPU."""

    def __init__(self, mesh, p, kappa, parents, sizes, static_workspace=False, **options):
        import torch
        self.torch = torch
        self.hm = mesh if isinstance(mesh, HostMesh) else HostMesh.of(mesh)
        self.p = p
        self.np = n_basis(self.hm.dim, p)
        self.n_elem = self.hm.n_elem
        self.opts = default_options(**options)
        # degree of each p-level (hp front end: p down to 1, by one or in one
        # step); the agglomeration levels after them run at the last degree
        if self.opts.p_coarse == 1 and p >= 2:
            self.p_levels = [p, 1] if self.opts.p_jump else list(range(p, 0, -1))
        else:
            self.p_levels = [p]
        sizes = np.ascontiguousarray(sizes, dtype=np.int32)
        par = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.int32) for x in parents])
                                   if len(parents) else np.zeros(0, dtype=np.int32))
        self._sizes, self._par = sizes, par
        hier = _Hier(len(sizes), _ptr(sizes).value, _ptr(par).value)
        kappa = self._dev(kappa)
        self.handle = ctypes.c_void_p()
        stream = torch.cuda.current_stream().cuda_stream
        if static_workspace:
            # the library's static per-GPU workspace: nothing is allocated
            self.workspace = None
            _check(lib.cdgmg_setup_static(ctypes.byref(self.hm.c), p, kappa.data_ptr(), ctypes.byref(hier),
                                          ctypes.byref(self.opts), ctypes.c_void_p(stream),
                                          ctypes.byref(self.handle)))
        else:
            # the device memory of the handle: one torch-owned workspace
            nbytes = workspace_size(self.hm, p, parents, sizes, self.opts)
            self.workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
            _check(lib.cdgmg_setup(ctypes.byref(self.hm.c), p, kappa.data_ptr(), ctypes.byref(hier),
                                   ctypes.byref(self.opts), self.workspace.data_ptr(), nbytes,
                                   ctypes.c_void_p(stream), ctypes.byref(self.handle)))
        self._kappa = kappa.detach().clone()

    def _dev(self, a, dtype=None):
        torch = self.torch
        dtype = dtype or torch.float64
        if not isinstance(a, torch.Tensor):
            a = torch.as_tensor(np.asarray(a))
        return a.to(device="cuda", dtype=dtype).contiguous()

    def _vec(self, n=None, dtype=None):
        torch = self.torch
        return torch.empty((self.n_elem if n is None else n) * self.np, dtype=dtype or torch.float64, device="cuda")

    def _run_solve(self, fn, rhs, history, strict=False):
        info = _Info()
        hist = None
        if history:
            hist = np.zeros(max(self.opts.max_iter, 1))
            info.history = _ptr(hist).value
            info.history_len = len(hist)
        rhs = self._dev(rhs).reshape(-1)
        out = self._vec()
        rc = fn(self.handle, rhs.data_ptr(), out.data_ptr(), ctypes.byref(info))
        _check(rc, allow_warning=not strict)
        return out, SolveInfo(info, hist), rc

    def solve(self, f, history=False, strict=False):
        """u with A u = M_0 f (f nodal source, [n_elem * n_p]).  A solve that
        stops at max_iter returns its last iterate (CDGMG_NOT_CONVERGED is a
        warning) unless strict, which raises CdgmgError instead."""
        u, info, rc = self._run_solve(lib.cdgmg_solve, f, history, strict)
        return u, info

    def solve_rhs(self, b, history=False, strict=False):
        x, info, rc = self._run_solve(lib.cdgmg_solve_rhs, b, history, strict)
        return x, info

    def solve_transpose(self, g, history=False, strict=False):
        x, info, rc = self._run_solve(lib.cdgmg_solve_transpose, g, history, strict)
        return x, info

    def grad_kappa(self, u, lam):
        u, lam = self._dev(u).reshape(-1), self._dev(lam).reshape(-1)
        g = self.torch.empty(self.n_elem, dtype=self.torch.float64, device="cuda")
        _check(lib.cdgmg_grad_kappa(self.handle, u.data_ptr(), lam.data_ptr(), g.data_ptr()))
        return g

    def apply_mass(self, x):
        x = self._dev(x).reshape(-1)
        y = self._vec()
        _check(lib.cdgmg_apply_mass(self.handle, x.data_ptr(), y.data_ptr()))
        return y

    def update_kappa(self, kappa):
        kappa = self._dev(kappa)
        _check(lib.cdgmg_update_kappa(self.handle, kappa.data_ptr()))
        self._kappa = kappa.detach().clone()

    def ensure_kappa(self, kappa):
        """Rebuild the operators only if kappa differs from the current one."""
        kappa = self._dev(kappa)
        if kappa.shape != self._kappa.shape or not bool(self.torch.equal(kappa, self._kappa)):
            self.update_kappa(kappa)

    def level_info(self):
        nl = ctypes.c_int(0)
        _check(lib.cdgmg_level_info(self.handle, ctypes.byref(nl), None, None))
        ne = np.zeros(nl.value, dtype=np.int64)
        nz = np.zeros(nl.value, dtype=np.int64)
        _check(lib.cdgmg_level_info(self.handle, ctypes.byref(nl), _ptr(ne), _ptr(nz)))
        return ne, nz

    def launch_info(self):
        """Launch configuration per level: dict of int arrays lanes_sweep,
        lanes_restrict, row_threads, and the level-0 wavefronts per slice."""
        nl = ctypes.c_int(0)
        _check(lib.cdgmg_launch_info(self.handle, ctypes.byref(nl), None, None, None, None))
        ls = np.zeros(nl.value, dtype=np.int32)
        lr = np.zeros(nl.value, dtype=np.int32)
        rt = np.zeros(nl.value, dtype=np.int32)
        wf = ctypes.c_int(0)
        _check(lib.cdgmg_launch_info(self.handle, ctypes.byref(nl), _ptr(ls), _ptr(lr), _ptr(rt), ctypes.byref(wf)))
        return {"lanes_sweep": ls, "lanes_restrict": lr, "row_threads": rt, "wavefronts": wf.value}

    def apply_A(self, level, x, precision=0):
        torch = self.torch
        dt = torch.float64 if precision == 0 else torch.float32
        ne, _ = self.level_info()
        x = self._dev(x, dt).reshape(-1)
        y = torch.empty(int(ne[level]) * self.level_np(level), dtype=dt, device="cuda")
        _check(lib.cdgmg_apply_A(self.handle, level, precision, x.data_ptr(), y.data_ptr()))
        return y

    def level_np(self, level):
        """Block size n_p of the operator at a level."""
        return n_basis(self.hm.dim, self.p_levels[min(level, len(self.p_levels) - 1)])

    def vcycle(self, r):
        r = self._dev(r).reshape(-1)
        z = self._vec()
        _check(lib.cdgmg_vcycle(self.handle, r.data_ptr(), z.data_ptr()))
        return z

    def export_operator(self, level):
        """(row_ptr, cols, blocks[nnzb, n_p, n_p]) of A_level, FP64, hierarchy numbering."""
        ne, _ = self.level_info()
        nnzb = ctypes.c_int64(0)
        _check(lib.cdgmg_export_operator(self.handle, level, ctypes.byref(nnzb), None, None, None))
        rp = np.zeros(int(ne[level]) + 1, dtype=np.int64)
        cols = np.zeros(nnzb.value, dtype=np.int32)
        npl = self.level_np(level)
        blocks = np.zeros((nnzb.value, npl, npl))
        _check(lib.cdgmg_export_operator(self.handle, level, ctypes.byref(nnzb), _ptr(rp), _ptr(cols),
                                         _ptr(blocks)))
        return rp, cols, blocks

    def node_coords(self):
        out = np.zeros((self.n_elem, self.np, self.hm.dim))
        _check(lib.cdgmg_node_coords(self.handle, _ptr(out)))
        return out

    def set_profile(self, on):
        _check(lib.cdgmg_set_profile(self.handle, 1 if on else 0))

    def device_bytes(self):
        b = ctypes.c_size_t(0)
        _check(lib.cdgmg_device_bytes(self.handle, ctypes.byref(b)))
        return b.value

    def close(self):
        if self.handle:
            lib.cdgmg_destroy(self.handle)
            self.handle = ctypes.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
