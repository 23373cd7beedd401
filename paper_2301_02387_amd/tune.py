"""Autotuner for the launch schedules of the two operator kernels.

Each candidate (sweep order, grid cap, and for the Poisson solve the long-row,
fused-direction, column-block and multigrid options) is applied with ``Operator.tune`` and timed on the
caller's own inputs: the orbital operator by the library's event-pair kernel
timing through ``rhs_apply`` (the frozen operator must be set), the Poisson
solve by the wall time of a ``poisson_pairs`` solve from zero.  The
fastest candidate is kept.  Results are cached in memory (and optionally in
a JSON file) per (mesh signature, degree, orbitals, instances).
"""
import json
import os

ORB_CANDIDATES = [(s, g) for s in (1, 0, 5, 4) for g in (2048, 8192, 65536)]
POI_CANDIDATES = ([(s, g) for s in (13, 12, 5, 4, 9, 1, 45, 44, 37, 36) for g in (2048, 8192)]
                  + [(s, 8192) for s in (21, 20, 29, 53, 52, 85, 84, 117, 116, 373, 372, 629, 628)])
# column blocking only changes anything at 32 or more columns (n >= 6 orbitals).
# On such wide column sets a Jacobi-preconditioned solve from zero takes
# seconds (about 1,000 iterations on the 1.5M-unknown water mesh, against
# about 15 with multigrid), so only one Jacobi schedule is timed there.
# Grid caps above 8192 give each workgroup of the sliced-ELL sweep one or two
# slices, so the hardware's in-order dispatch keeps the rows in flight on an
# XCD in one window (measured on the water mesh: CG pass 1.47 ms at 8192,
# 1.37 ms at 32768, 1.81 ms at 65536).  On those grids the sweep stays
# XCD-contiguous (bit 0): without it the operator pass fetches 9.2 instead of
# 6.7 GB per launch in the same time (the extra bytes come from the last-level
# cache), and the tuner's short solves from zero do not tell the two apart.
POI_CANDIDATES_WIDE = ([(13, 8192)]
                       + [(s, 8192) for s in (22, 20, 23, 21, 54, 52, 55, 53, 118, 116, 119, 117, 182, 214, 246,
                                               372, 628, 884)]
                       + [(s, g) for s in (117, 372, 373, 628) for g in (16384, 32768)])
# grid caps are per instance: a batch fills the chip with fewer workgroups each
ORB_CANDIDATES_BATCH = [(s, g) for s in (1, 0, 5, 4) for g in (256, 1024, 65536)]
POI_CANDIDATES_BATCH = ([(s, g) for s in (13, 12, 5, 4, 1, 45, 37, 36) for g in (256, 1024)]
                        + [(s, g) for s in (21, 20, 53, 52, 117, 116) for g in (256, 1024)]
                        + [(s, 2048) for s in (117, 116)])
_CACHE = {}


def _key(op):
    info = op.mesh.info
    return (f"{info['n_cells']}-{info['n_dof']}-{info['n_hang']}-p{info['p']}-n{op.n_orb}"
            f"-i{op.n_inst}-{op.n_dof}")


def _load(cache_file):
    if cache_file and os.path.exists(cache_file):
        with open(cache_file) as f:
            _CACHE.update({k: {kk: tuple(vv) if isinstance(vv, list) else vv for kk, vv in v.items()}
                           for k, v in json.load(f).items()})


def apply_cached(op, cache_file=None):
    """Apply the tuned schedules of this operator from the cache, if present."""
    key = _key(op)
    if key not in _CACHE:
        _load(cache_file)
    if key not in _CACHE:
        return None
    best = _CACHE[key]
    op.tune(0, *best["orbital"])
    op.tune(1, *best["poisson"])
    return best


def autotune(op, phi, W, reps=5, cache_file=None):
    """Pick and apply the fastest schedule for both operator kernels.

    phi: device orbitals [N_E][n] (consistent), W: device Poisson columns
    [N_F][n^2] holding a converged (or good) solution for phi; mh_freeze must
    have been called.  Returns {"orbital": (sched, grid), "poisson": (sched, grid),
    "timings": {...}}.
    """
    import torch
    key = _key(op)
    best = apply_cached(op, cache_file)
    if best is not None:
        return best
    out = torch.empty_like(phi)
    times = {"orbital": {}, "poisson": {}}
    batched = op.n_inst > 1
    for sched, grid in (ORB_CANDIDATES_BATCH if batched else ORB_CANDIDATES):
        op.tune(0, sched, grid)
        op.rhs_apply(phi, out)
        op.kernel_timing(0, True)
        for _ in range(reps):
            op.rhs_apply(phi, out)
        times["orbital"][(sched, grid)] = op.kernel_timing(0, False)[0]
    # Poisson: wall time of a full solve from zero on a scratch array (the
    # schedules differ in how many launches an iteration takes, and the
    # multigrid-preconditioned ones (bit 4) in the iteration count); the second
    # of two solves is timed, so a multigrid hierarchy is built before timing
    import time
    Wt = torch.zeros_like(W)
    wide = op.n_pair_cols >= 32 and op.n_pair_cols % 16 == 0
    for sched, grid in (POI_CANDIDATES_BATCH if batched else (POI_CANDIDATES_WIDE if wide else POI_CANDIDATES)):
        op.tune(1, sched, grid)
        for rep in range(2):
            Wt.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            op.poisson_pairs(phi, Wt, warm=False)
        times["poisson"][(sched, grid)] = (time.perf_counter() - t0) * 1e3
    del Wt
    best = {"orbital": min(times["orbital"], key=times["orbital"].get),
            "poisson": min(times["poisson"], key=times["poisson"].get)}
    op.tune(0, *best["orbital"])
    op.tune(1, *best["poisson"])
    best["timings_ms"] = {k: {f"{s}/{g}": v for (s, g), v in d.items()} for k, d in times.items()}
    _CACHE[key] = best
    if cache_file:
        data = {}
        if os.path.exists(cache_file):
            with open(cache_file) as f:
                data = json.load(f)
        data[key] = {"orbital": list(best["orbital"]), "poisson": list(best["poisson"])}
        with open(cache_file, "w") as f:
            json.dump(data, f, indent=1)
    return best
