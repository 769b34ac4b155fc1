"""The parity cases of the GPU tests and the kernel instantiations they reach.

test_gpu_parity.py compares the V-cycle with the oracle's for every case and
option listed here; the full-size tests check that each launch configuration
the benchmark workloads use (lanes per coarse row, thread-per-row workgroup
size, level-0 wavefronts per slice, per block size n_p and precision) lies in
COVERED.  Precision codes: 0 = FP64 V-cycle, 1 = FP32 V-cycle.
"""

CASES = {
    # name: (dim, n, p, levels, seed); sizes span several 64-row slices and a ragged tail
    "2d_p2": (2, 14, 2, 3, 11),
    "2d_p3": (2, 12, 3, 4, 12),
    "2d_p1": (2, 11, 1, 3, 5),
    "3d_p2": (3, 4, 2, 3, 13),
    "3d_p1": (3, 5, 1, 3, 7),
    # n_p = 20: one (automatic) or 2, 4, 5 wavefronts per level-0 slice (750 tetrahedra, 12 slices, ragged)
    "3d_p3": (3, 5, 3, 3, 17),
}
NP = {"2d_p1": 3, "2d_p2": 6, "2d_p3": 10, "3d_p1": 4, "3d_p2": 10, "3d_p3": 20}

# level-0 wavefronts per slice: kernel_variant values (0 = automatic: 1) run in
# FP64 on every case, and these in FP32
VARIANTS = [0, 1, 2, 4, 5]
FP32_VARIANT_CASES = [("2d_p3", 0), ("2d_p3", 1), ("2d_p3", 2), ("2d_p3", 5), ("3d_p2", 0), ("3d_p3", 0),
                      ("3d_p3", 2), ("3d_p3", 4), ("3d_p3", 5)]

# coarse levels: lanes per row of the sweep and of the residual + restriction,
# and the workgroup size of the thread-per-row transfer kernels
GROUPS = [8, 16, 32, 64]
ROW_THREADS = [64, 256]
GROUP_CASES = ["2d_p2", "2d_p3", "3d_p2", "3d_p3"]


def auto_wavefronts(npb):
    return 1


def _covered():
    wf = set()
    for c in CASES:
        for v in VARIANTS:
            if v == 0 or NP[c] % v == 0:
                wf.add((0, NP[c], v or auto_wavefronts(NP[c])))
    for c, v in FP32_VARIANT_CASES:
        wf.add((1, NP[c], v or auto_wavefronts(NP[c])))
    return {
        "group": {(mg, NP[c], g) for mg in (0, 1) for c in GROUP_CASES for g in GROUPS},
        "row_threads": {(mg, NP[c], t) for mg in (0, 1) for c in GROUP_CASES for t in ROW_THREADS},
        "wavefronts": wf,
    }


COVERED = _covered()


def uncovered(info, mg, npb):
    """Launch configurations of a handle (Solver.launch_info()) that no parity
    case reaches; empty when every one is covered."""
    out = []
    L = len(info["lanes_sweep"]) - 1
    for l in range(1, L):
        for key in ("lanes_sweep", "lanes_restrict"):
            if (mg, npb, int(info[key][l])) not in COVERED["group"]:
                out.append((key, l, int(info[key][l])))
    for l in range(L):
        if (mg, npb, int(info["row_threads"][l])) not in COVERED["row_threads"]:
            out.append(("row_threads", l, int(info["row_threads"][l])))
    if (mg, npb, int(info["wavefronts"])) not in COVERED["wavefronts"]:
        out.append(("wavefronts", 0, int(info["wavefronts"])))
    return out
