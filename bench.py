#!/usr/bin/env python
"""Throughput of the MCTDHF orbital time step on one MI355X.

One step = the whole hot path at t_n: RDMs, pair Poisson solves (multipole
boundary values + multigrid-preconditioned CG on all pairs), mean field U
and the frozen operator G, m = 12 orbital right-hand-side evaluations inside
the short-iterative Arnoldi exponential, integrals and the CI Lanczos step,
and the observables.  `value` counts the Arnoldi right-hand-side evaluations
as DoF x orbitals per second of whole-step wall time, inputs resident in HBM.

Default workload: the H2O-shaped molecule, Q3 elements on [-40,40]^3, 16^3
coarse cells, 4 levels within 6.5 bohr of O and 3 of each H (1,517,876
unknowns), 8 orbitals, CAS(10e,8o) = 3,136 determinants, sin^2 800 nm pulse
of peak 0.0534 au, dt = 0.02, Krylov 12.  Its record also carries the H2
workload (Q3, [-30,30]^3, 12^3 cells, 3 levels in 1.5-bohr balls at
z = +-0.7, 66,635 unknowns, 2 orbitals, 4 determinants) under "h2", with the
forward+adjoint against plain forward comparison on that molecule and mesh,
and a measured device copy rate.
`--workload h2` runs the H2 record alone (with the oracle's whole steps as the
CPU baseline).  `--workload h2x64` runs 64 H2 instances of uneven meshes
(bond ~ U[1,2], refinement depth in {2,3,4}, E0 ~ U[0.02,0.06], seeded) as one
batch in the same kernel launches, and times 64 sequential single-instance
runs of the same instances on a bounded sample for the batched/sequential
ratio.
"""
import argparse
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _workload(name):
    from synth import workload
    return workload(name)


def initial_state(name, w, mesh, op, torch):
    import numpy as np
    from synth import h2_guess, h2o_guess, initial_guess, h2_ci_guess, random_ci
    xyz = mesh.coords()[:op.n_ext]
    if name == "h2":
        c = h2_guess(xyz, 0.7)
        C = h2_ci_guess()
    elif name in ("h2o", "h2o_q1"):
        c = h2o_guess(xyz)
        C = 0.9 * np.eye(1, op.n_ci, 0, dtype=complex)[0] + 0.1 * random_ci(op.n_ci, 7)
        C = C / np.linalg.norm(C)
    else:
        c = initial_guess(name, xyz)
        C = np.ones(1, dtype=complex)
    phi = torch.from_numpy(np.ascontiguousarray(c)).cuda()
    op.fill_hanging(phi)
    return phi, torch.from_numpy(np.ascontiguousarray(C)).cuda()


def stored_matrix_bytes(N, nnz, n_inst):
    """Bytes of the assembled Poisson operator read by one plain pass (column
    int32 + value per entry, row pointers): overhead of the assembled form,
    not part of the algorithmic bytes."""
    return 12 * nnz + 4 * (N + n_inst)


def poisson_algorithmic_bytes(info, op, fused=False):
    """Matrix-free bytes of one Poisson operator application on the pair
    columns (the Laplacian applied cell by cell from the 1D Gauss-Lobatto
    tables): operand rows read and result rows written once (8 B per column
    each), the cell->node maps (int32), the hanging-node constraint rows (int32
    index + weight) and h per cell.  With the CG direction formed in the same
    pass (schedule bit 3) also r and the previous direction read, the new
    direction written and the diagonal read."""
    P3 = (info["p"] + 1) ** 3
    N, ncol, nC = op.n_dof, op.n_pair_cols, info["n_cells"]
    b = 16 * ncol * N + 4 * P3 * nC + 12 * info["hang_nnz"] + 8 * nC
    if fused:
        b += 16 * ncol * N + 8 * N
    return b


def rhs_algorithmic_bytes(info, op, ecs=False):
    """B_G: bytes one orbital right-hand-side evaluation must move: the packed
    vector in and G v out (16 B per complex entry each), the per-node
    Hermitian mean-field matrix U (n^2 reals per full node), the per-node
    potential and dipole weights, the cell->node maps, the constraint rows and
    1/m of the unknowns.  The interface mass system is cache-resident.  With
    complex scaling the potential and field weights are complex and the row
    factor rho and a byte per cell join them."""
    P3 = (info["p"] + 1) ** 3
    n, N, NF, nC = op.n_orb, op.n_dof, info["n_full"], info["n_cells"]
    extra = 32 * op.n_ext + nC if ecs else 0
    return 32 * n * N + 8 * n * n * NF + 16 * NF + 4 * P3 * nC + 12 * info["hang_nnz"] + 8 * N + extra


def orbital_pass_bytes(info, op, ecs=False):
    """Algorithmic bytes of the orbital operator's node pass alone (kernel
    timing slot 0): orbitals in and out, U, the node tables (with complex
    scaling also the complex row factor, potential and field weights and the
    cells' scaled directions)."""
    P = info["p"] + 1
    nC, NE, N, n = info["n_cells"], op.n_ext, op.n_dof, op.n_orb
    meta = 32 * NE + 4 * P ** 3 * nC + 8 * nC + 4 * N
    extra = 32 * NE + nC if ecs else 0
    return 32 * n * NE + 8 * n * n * NE + 24 * NE + 8 * N + meta + extra


def copy_bandwidth(torch, gib=2, reps=10):
    """Measured device-to-device copy rate (a STREAM-copy figure): bytes read
    plus bytes written per second over `reps` copies of `gib` GiB, event-timed
    on the current stream."""
    a = torch.empty((gib << 30) // 8, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * (gib << 30) / (ms * 1e-3) / 1e9


def cpu_baseline_h2(w, budget_s):
    """The oracle, as it stands, on whole time steps of the H2 workload."""
    import numpy as np
    import psutil
    from oracle.mesh import Mesh, MeshDesc, Ball
    from oracle.fem import Operators
    from oracle.ci import CISpace
    from oracle.mctdhf import Propagator, orthonormalize
    from synth import h2_guess, h2_ci_guess, pulse
    mesh = Mesh(MeshDesc(w["lo"], w["hi"], w["n_coarse"], w["p"], [Ball(**b) for b in w["balls"]]))
    ops = Operators(mesh, w["nuclei"])
    cs = CISpace(w["n_orb"], w["n_alpha"], w["n_beta"])
    c = orthonormalize(ops, h2_guess(mesh.xyz[mesh.dof_nodes], 0.7))
    C = h2_ci_guess()
    pr = Propagator(ops, cs)
    pr.poisson.factor()            # one-off factorisation, as a warm-up would
    ops.gradient()                 # and the derivative matrices of the momentum record
    Tp = w["cycles"] * 2 * np.pi / 0.0569542
    proc = psutil.Process()
    c0 = proc.cpu_times()
    t0 = time.perf_counter()
    steps = 0
    while True:
        c, C, _ = pr.step(c, C, float(pulse(Tp / 2 + steps * w["dt"], w["E0"], w["cycles"])), w["dt"], w["krylov"])
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 3:
            break
    wall = time.perf_counter() - t0
    c1 = proc.cpu_times()
    cpu = (c1.user - c0.user) + (c1.system - c0.system)
    evals = steps * w["krylov"] * mesh.n_dof * w["n_orb"]
    return {"value": evals / wall, "unit": "DoF*orbitals/s", "cores": max(1, int(round(cpu / wall))),
            "kind": "oracle", "sample": f"{steps} full time step(s) of the same H2 workload "
                                        f"(Poisson LU factorisation done beforehand), {wall:.1f} s wall",
            "host_threads_available": os.cpu_count()}


def cpu_baseline_rhs_child(name, budget_s):
    """Child process of the CPU baseline: the oracle, as it stands, applying
    the frozen orbital right-hand side G of the workload.  Set-up first (its
    own mesh, operators, sparse LU of the mass matrix and the frozen operator
    with synthetic pair potentials: the oracle's direct Poisson solve does not
    fit at this size, and the cost of a G application does not depend on the
    potential values), then it waits for a line on stdin, so that its timed
    sample of about `budget_s` seconds runs after the GPU's timed work, and
    prints one JSON record."""
    import numpy as np
    import psutil
    from oracle.mesh import Mesh, MeshDesc, Ball
    from oracle.fem import Operators
    from oracle.ci import CISpace
    from oracle.mctdhf import Frozen, orthonormalize
    from synth import h2o_guess, random_ci
    w = _workload(name)
    t_set = time.perf_counter()
    mesh = Mesh(MeshDesc(w["lo"], w["hi"], w["n_coarse"], w["p"], [Ball(**b) for b in w["balls"]]))
    ops = Operators(mesh, w["nuclei"])
    n = w["n_orb"]
    cs = CISpace(n, w["n_alpha"], w["n_beta"])
    c = orthonormalize(ops, h2o_guess(mesh.xyz[mesh.dof_nodes]))
    gam, Gam = cs.rdms(random_ci(cs.dim, 7))
    r = np.linalg.norm(mesh.xyz, axis=1)
    W = {(a, b): (1.0 + 0.1 * (a + b)) / np.sqrt(r * r + 1.0) + 0j for a in range(n) for b in range(a, n)}
    ops.mass_solve(c[:, :1])       # one-off factorisation of the mass matrix
    fr = Frozen(ops, c, gam, Gam, 0.01, W)
    t_set = time.perf_counter() - t_set
    sys.stdin.readline()
    proc = psutil.Process()
    c0 = proc.cpu_times()
    t0 = time.perf_counter()
    k = 0
    while True:
        fr.G(c)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    wall = time.perf_counter() - t0
    c1 = proc.cpu_times()
    cpu = (c1.user - c0.user) + (c1.system - c0.system)
    print(json.dumps({
        "value": k * mesh.n_dof * n / wall, "unit": "DoF*orbitals/s", "cores": max(1, int(round(cpu / wall))),
        "kind": "oracle",
        "sample": f"{k} orbital right-hand-side evaluations (G applications) of the same {mesh.n_dof}-unknown, "
                  f"{n}-orbital workload, {wall:.1f} s wall, timed after the GPU's timed work; set-up "
                  f"({t_set:.0f} s: mesh, operators, mass-matrix LU, frozen operator) ran in a child process "
                  f"beside the GPU work; the oracle's direct Poisson solve does not fit at this size, so its "
                  f"whole-step rate is not measured",
        "setup_s": t_set, "host_threads_available": os.cpu_count()}), flush=True)


def start_cpu_baseline(name, budget_s):
    """Start the oracle's set-up in a child process (before this process
    touches the GPU); finish_cpu_baseline releases its timed sample."""
    import subprocess
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-child", name, str(budget_s)],
                            stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)


def finish_cpu_baseline(proc):
    out, _ = proc.communicate("go\n", timeout=1800)
    lines = [ln for ln in out.splitlines() if ln.startswith("{")]
    if proc.returncode != 0 or not lines:
        raise RuntimeError(f"CPU baseline child failed (exit {proc.returncode})")
    return json.loads(lines[-1])


def run_single(name, args, torch, with_adjoint, with_cpu):
    """Set-up, warm-up, autotuning and `args.steps` timed steps of one
    workload; returns the bench record."""
    import numpy as np
    import paper_2301_02387_amd as mh
    from synth import pulse, pulse_triangular, vector_potential_triangular, OMEGA_800NM

    w = _workload(name)
    gauge = w.get("gauge", "length")
    ecs = w.get("ecs")
    t_setup = time.perf_counter()
    mesh = mh.Mesh.from_workload(w)
    op = mh.Operator(mesh, w["nuclei"], w["n_orb"], w["n_alpha"], w["n_beta"],
                     polarization=w.get("polarization", (0.0, 0.0, 1.0)), poisson_rtol=1e-12, poisson_maxit=20000,
                     gauge=gauge, ecs=(ecs["theta"], ecs["inner"]) if ecs else None)
    t_setup = time.perf_counter() - t_setup
    log(f"{name}: set up in {t_setup:.1f} s, {op.n_dof} unknowns")
    info = mesh.info
    phi, Ci = initial_state(name, w, mesh, op, torch)
    W = torch.zeros((op.n_full, op.n_pair_cols), dtype=torch.float64, device="cuda")
    dt, m = w["dt"], w["krylov"]
    omega = w.get("omega", OMEGA_800NM)
    Tp = (w["cycles"] * 2 * np.pi / omega) if w["cycles"] else 1.0
    if args.tune_cache:   # schedules tuned by an earlier run on this workload, before the warm-up
        from paper_2301_02387_amd.tune import apply_cached
        apply_cached(op, args.tune_cache)
    # warm-up: imaginary-time relaxation steps, then one real-time step
    if args.warmup > 0:
        op.propagate(phi, Ci, W, [0.0] * (args.warmup + 1), 0.05, m=m, imaginary=True, final=False)
    t0 = Tp / 2   # the pulse peak
    if w.get("envelope") == "triangular":   # field values: E(t), or A(t) in the velocity gauge
        fv = vector_potential_triangular if gauge == "velocity" else pulse_triangular
        E = [float(fv(t0 + k * dt, w["E0"], omega)) for k in range(args.steps + 1)]
    else:
        E = [float(pulse(t0 + k * dt, w["E0"], w["cycles"], omega)) if w["cycles"] else 0.0
             for k in range(args.steps + 1)]
    op.propagate(phi, Ci, W, E[:2], dt, m=m, final=False)
    # schedules of the two operator kernels picked by the autotuner (untimed)
    from paper_2301_02387_amd.tune import autotune
    sched = autotune(op, phi, W, cache_file=args.tune_cache)
    log(f"{name}: warm-up and tuning done, schedules {sched['orbital']} {sched['poisson']}")
    # timed region: exactly `steps` steps
    op.kernel_timing(0, True)
    op.kernel_timing(1, True)
    torch.cuda.synchronize()
    t_a = time.perf_counter()
    rec = op.propagate(phi, Ci, W, E, dt, m=m, final=False, graph=args.graph, graph_step=args.graph_step)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_a
    k_orb = op.kernel_timing(0, False)
    k_poi = op.kernel_timing(1, False)
    log(f"{name}: {wall / args.steps * 1e3:.2f} ms per step")
    # Arnoldi step alone (G frozen at the last step), and G applications by
    # HIP event pairs on the stream the library launches on
    phi2 = phi.clone()
    reps = 5
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(reps):
        phi2.copy_(phi)
        op.arnoldi_step(phi2, dt, m)
    torch.cuda.synchronize()
    arnoldi_ms = (time.perf_counter() - ta) / reps * 1e3
    out = torch.empty_like(phi)
    reps_g = 20
    op.rhs_apply(phi, out)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps_g)]
    for k in range(reps_g):
        ev[2 * k].record()
        op.rhs_apply(phi, out)
        ev[2 * k + 1].record()
    torch.cuda.synchronize()
    rhs_ms = float(np.mean([ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(reps_g)]))

    evals = args.steps * m * op.n_dof * op.n_orb
    kern = {"stencil_orb": {"avg_ms": k_orb[0], "count": k_orb[1]},
            "poisson_spmv": {"avg_ms": k_poi[0], "count": k_poi[1]}}
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["count"])
    fused = bool(sched["poisson"][0] & 8)
    if dom == "poisson_spmv":
        byts = poisson_algorithmic_bytes(info, op, fused)
        over = stored_matrix_bytes(op.n_dof, op.n_poisson_nnz, op.n_inst)
    else:
        byts, over = orbital_pass_bytes(info, op, bool(ecs)), 0
    sched_tag = "/".join(map(str, sched["poisson"] if dom == "poisson_spmv" else sched["orbital"]))
    ach = byts / (kern[dom]["avg_ms"] * 1e-3) / 1e9 if kern[dom]["avg_ms"] > 0 else 0.0
    wl = (f"{name}_{op.n_dof}dof_{op.n_orb}orb" if name.endswith(f"_q{w['p']}")
          else f"{name}_q{w['p']}_{op.n_dof}dof_{op.n_orb}orb")
    bg = rhs_algorithmic_bytes(info, op, bool(ecs))
    rhs_ach = bg / (rhs_ms * 1e-3) / 1e9
    orb_b = orbital_pass_bytes(info, op, bool(ecs))
    orb_ach = orb_b / (k_orb[0] * 1e-3) / 1e9 if k_orb[0] > 0 else 0.0
    line = {
        "metric": "orbital-RHS evals/s (DoF x orbitals/s)",
        "value": evals / wall,
        "unit": "DoF*orbitals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": wl, "n_dof": op.n_dof, "n_full": info["n_full"], "n_cells": info["n_cells"],
                   "mesh": ("Kelly indicator of the nuclear potential, cell sizes "
                            + ", ".join(f"{(w['hi'] - w['lo']) / w['n_coarse'] / 2 ** l:g}"
                                        for l, c in enumerate(info["level_counts"]) if c)) if w.get("kelly")
                   else "ball refinement",
                   "gauge": gauge,
                   "absorber": (f"exterior complex scaling, {ecs['theta']} rad beyond |x_d| = "
                                + "/".join(f"{r:g}" for r in ecs["inner"])) if ecs else "none (Dirichlet box)",
                   "n_orb": op.n_orb, "n_ci": op.n_ci, "krylov": m, "dt": dt, "graph": bool(args.graph),
                   "graph_step": bool(args.graph_step), "parallelism": "none (one GPU)"},
        "arnoldi_step_ms": arnoldi_ms,
        "rhs_apply_ms": rhs_ms,
        "rhs_evals_per_s_isolated": op.n_dof * op.n_orb / (rhs_ms * 1e-3),
        "poisson_cg_iters_per_step": float(np.mean(rec["cg_iters"][:args.steps])),
        "setup_s": t_setup,
        "schedule": {"orbital": list(sched["orbital"]), "poisson": list(sched["poisson"]),
                     "tuning_ms": sched.get("timings_ms")},
        "kernels": kern,
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, wl, schedule=sched_tag),
                     "schedule": sched_tag,
                     "algorithmic_bytes_per_launch": byts,
                     "algorithmic_bytes": "matrix-free: operand and result rows, cell maps, constraint rows, h",
                     "stored_operator_bytes_per_launch": over},
        # one whole G application (node pass, stiffness, interface mass solve,
        # hanging fill) against B_G, by event pairs around each call
        "roofline_rhs": {"kernel": "rhs_apply (all launches of one G application)", "bound": "hbm",
                         "achieved": rhs_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": rhs_ach / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_launch": bg},
        # the orbital operator's node pass of every G application
        "roofline_orbital": {"kernel": "stencil_orb", "bound": "hbm", "achieved": orb_ach, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": orb_ach / HBM_PEAK_GBS,
                             "schedule": "/".join(map(str, sched["orbital"])), "algorithmic_bytes_per_launch": orb_b},
    }
    if with_adjoint:
        line["fwd_adjoint_vs_plain"] = adjoint_ratio(op, phi, Ci, w)
    if with_cpu:   # the H2 workload's oracle takes whole steps (its direct Poisson solve fits)
        line["cpu_baseline"] = cpu_baseline_h2(w, args.cpu_budget)
    del op, mesh
    return line


def main():
    if len(sys.argv) == 4 and sys.argv[1] == "--cpu-child":
        return cpu_baseline_rhs_child(sys.argv[2], float(sys.argv[3]))
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="h2o", choices=["h2", "h2o", "h2o_q1", "h_atom", "h2x64"])
    ap.add_argument("--batch", type=int, default=64, help="instances of the h2x64 workload")
    ap.add_argument("--seq-steps", type=int, default=None,
                    help="timed steps per instance of the sequential runs (default: --steps, the batch's own count)")
    ap.add_argument("--graph", action="store_true", help="replay each step's fixed part as a HIP graph")
    ap.add_argument("--graph-step", action="store_true",
                    help="replay whole steps (Poisson CG with a fixed iteration count included) as one HIP graph each")
    ap.add_argument("--no-sequential", action="store_true", help="h2x64: skip the sequential runs")
    ap.add_argument("--counters", action="store_true",
                    help="short run for hardware-counter passes: CG iterations and RHS applications on the "
                         "workload's mesh, then a 1 GiB elementwise multiply for calibration; prints no JSON")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward+adjoint vs plain comparison")
    ap.add_argument("--no-h2", action="store_true", help="h2o: skip the H2 workload's extra record")
    ap.add_argument("--no-q1", action="store_true",
                    help="h2o: skip the extra record of the Q1 water workload on its Kelly-refined mesh")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of tuned schedules: read if it holds this workload, else written after tuning")
    ap.add_argument("--poisson-schedule", default=None,
                    help="--counters: Poisson schedule/grid cap to count under (e.g. 117/32768) instead of the cache's")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the whole mesh lives on one MI355X; "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.counters:
        return run_counters(args)
    if args.workload == "h2x64":
        return run_batch(args)
    child = None
    if args.workload == "h2o" and not args.no_cpu_baseline:
        child = start_cpu_baseline(args.workload, args.cpu_budget)   # before this process touches the GPU
    import torch
    line = run_single(args.workload, args, torch, with_adjoint=(args.workload == "h2" and not args.no_adjoint),
                      with_cpu=(args.workload == "h2" and not args.no_cpu_baseline))
    if args.workload == "h2o" and not args.no_h2:
        # the H2 workload (also the differentiation workload's molecule and
        # mesh): whole-step record and forward+adjoint against plain forward
        h2 = run_single("h2", args, torch, with_adjoint=not args.no_adjoint, with_cpu=False)
        line["h2"] = {k: h2[k] for k in ("value", "ms_per_step", "config", "arnoldi_step_ms", "rhs_apply_ms",
                                         "poisson_cg_iters_per_step", "roofline", "roofline_rhs")}
        if "fwd_adjoint_vs_plain" in h2:
            line["fwd_adjoint_vs_plain"] = h2["fwd_adjoint_vs_plain"]
    if args.workload == "h2o" and not args.no_q1:
        # the water molecule as Sec. IV runs it: Q1 on a Kelly-refined mesh,
        # triangular 400 nm pulse along x, dt = 0.01
        q1 = run_single("h2o_q1", args, torch, with_adjoint=False, with_cpu=False)
        line["h2o_q1"] = {k: q1[k] for k in ("value", "ms_per_step", "config", "arnoldi_step_ms", "rhs_apply_ms",
                                             "poisson_cg_iters_per_step", "roofline", "roofline_rhs")}
    bw = copy_bandwidth(torch)
    line["hbm_copy_measured_GBs"] = bw
    for key in ("roofline", "roofline_rhs", "roofline_orbital"):
        line[key]["frac_of_measured_copy"] = line[key]["achieved"] / bw
    if child is not None:
        line["cpu_baseline"] = finish_cpu_baseline(child)
        line["rhs_isolated_vs_cpu_baseline"] = line["rhs_evals_per_s_isolated"] / line["cpu_baseline"]["value"]
    print(json.dumps(line))


def sources_sha1(root=None):
    """SHA-1 over the library sources and the workload generators (every file
    of paper_2301_02387_amd/csrc/ and synth/*.py, in name order, each as its
    relative path then its bytes): what fixes both the kernels and the data
    layout they stream (node numbering, operator copies, meshes)."""
    import hashlib
    root = root or ROOT
    files = (sorted(glob.glob(os.path.join(root, "paper_2301_02387_amd", "csrc", "*")))
             + sorted(glob.glob(os.path.join(root, "synth", "*.py"))))
    h = hashlib.sha1()
    for f in files:
        if os.path.isfile(f):
            h.update(os.path.relpath(f, root).encode() + b"\0")
            h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, workload, profiles_dir=None, root=None, schedule=None):
    """HBM bytes per launch of `kernel` on `workload` (under `schedule`) from the
    counter summaries under profiles/ (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0,
    calibrated), or None when none was taken or the library sources or
    workload generators have changed since (sources_sha1)."""
    sha = sources_sha1(root)
    for path in sorted(glob.glob(os.path.join(profiles_dir or os.path.join(ROOT, "profiles"), "*.md"))):
        for ln in open(path):
            if not ln.startswith("traffic:"):
                continue
            kv = dict(tok.split("=", 1) for tok in ln.split()[1:])
            if kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("sources_sha1") == sha \
                    and (schedule is None or kv.get("schedule", schedule) == schedule):
                return float(kv["bytes_per_launch"])
    return None


def adjoint_ratio(op, phi, Ci, w, steps=200, n_quad=8, harmonics=(5, 15)):
    """Forward + checkpointed recomputation + adjoint against the plain
    forward propagation on the differentiation workload's molecule and mesh
    (H2, Q3, 2 orbitals, 4 determinants): a window of `steps` real-time steps
    at the pulse peak, from the bench's current state, with the Frechet
    quadrature the tests use and the harmonic-band objective
    J = sum_h |sum_n d_n e^{-i h omega t_n} dt|^2 over the given harmonics of
    the pulse's frequency, whose gradient dJ/dd_n the adjoint takes."""
    import numpy as np
    import torch
    from synth import pulse, OMEGA_800NM
    dt, m = w["dt"], w["krylov"]
    Tp = w["cycles"] * 2 * np.pi / OMEGA_800NM
    t = Tp / 2 + dt * np.arange(steps + 1)
    E = pulse(t, w["E0"], w["cycles"])
    phi0, C0 = phi.clone(), Ci.clone()
    W = torch.zeros((op.n_full, op.n_pair_cols), dtype=torch.float64, device="cuda")
    d = op.propagate(phi0.clone(), C0.clone(), W, E, dt, m=m)["dipole"]
    g = np.zeros(steps + 1)
    for h in range(harmonics[0], harmonics[1] + 1):
        ph = np.exp(-1j * h * OMEGA_800NM * t)
        F = np.sum(d * ph) * dt
        g += 2.0 * np.real(np.conj(F) * ph) * dt

    def plain():
        W.zero_()
        op.propagate(phi0.clone(), C0.clone(), W, E, dt, m=m)

    def adjoint():
        plain()   # the forward pass that produced the dipoles
        W.zero_()
        op.propagate_adjoint(phi0, C0, W, E, dt, g, m=m, n_quad=n_quad)

    out = {}
    for name, fn in (("plain", plain), ("fwd_adjoint", adjoint)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        out[name + "_ms"] = (time.perf_counter() - t0) * 1e3
    out["ratio"] = out["fwd_adjoint_ms"] / out["plain_ms"]
    out["workload"] = (f"h2_q3_{op.n_dof}dof_2orb_4det (differentiation workload's molecule and mesh), "
                       f"{steps}-step window at the pulse peak, objective on harmonics {harmonics[0]}-{harmonics[1]}, "
                       f"{n_quad}-point Frechet quadrature, checkpoints every round(sqrt(N)) steps")
    return out


def run_counters(args):
    import numpy as np
    import torch
    import paper_2301_02387_amd as mh
    from synth import h2_guess, h2o_guess, random_ci
    if args.workload == "h2x64":
        _, _, op, _, phi, _ = batch_setup(args, maxit=24)
    else:
        w = _workload(args.workload)
        mesh = mh.Mesh.from_workload(w)
        ecs = w.get("ecs")
        op = mh.Operator(mesh, w["nuclei"], w["n_orb"], w["n_alpha"], w["n_beta"], poisson_maxit=24,
                         polarization=w.get("polarization", (0.0, 0.0, 1.0)), gauge=w.get("gauge", "length"),
                         ecs=(ecs["theta"], ecs["inner"]) if ecs else None)
        xyz = mesh.coords()[:op.n_ext]
        c = h2o_guess(xyz) if args.workload in ("h2o", "h2o_q1") else h2_guess(xyz, 0.7)
        phi = torch.from_numpy(np.ascontiguousarray(c)).cuda()
        op.fill_hanging(phi)
    if args.tune_cache:   # the schedules the bench run tuned for this workload
        from paper_2301_02387_amd.tune import apply_cached
        log(f"schedules from the cache: {apply_cached(op, args.tune_cache)}")
    if args.poisson_schedule:   # counters of another Poisson schedule than the tuned one
        sched, grid = map(int, args.poisson_schedule.split("/"))
        op.tune(1, sched, grid)
        log(f"Poisson schedule {sched}/{grid}")
    W = torch.zeros((op.n_full, op.n_pair_cols), dtype=torch.float64, device="cuda")
    it, _ = op.poisson_pairs(phi, W)
    log(f"cg iterations {it}")
    n, ni = op.n_orb, op.n_inst
    C = torch.from_numpy(np.stack([random_ci(op.n_ci, 3)] * ni)).cuda()
    g = torch.zeros((ni, n, n), dtype=torch.complex128, device="cuda")
    G = torch.zeros((ni,) + (n,) * 4, dtype=torch.complex128, device="cuda")
    op.ci_rdms(C, g, G)
    op.freeze(phi, g, G, 0.01, W)
    out = torch.empty_like(phi)
    for _ in range(10):
        op.rhs_apply(phi, out)
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 2.0, out=b)   # calibration: 1 GiB read and 1 GiB written per launch
    torch.cuda.synchronize()
    log("counters run done")


def batch_setup(args, maxit=20000):
    """The uneven H2 instances of the batch workload, their batched operator
    and the sigma_g / sigma_u start of every instance."""
    import numpy as np
    import torch
    import paper_2301_02387_amd as mh
    from synth import batch_instances, h2_guess
    ws = batch_instances(args.batch, seed=2301)
    w0 = ws[0]
    t_setup = time.perf_counter()
    meshes = [mh.Mesh.from_workload(w) for w in ws]
    op = mh.Operator.batch(meshes, [w["nuclei"] for w in ws], w0["n_orb"], w0["n_alpha"], w0["n_beta"],
                           field_scale=[w["E0"] for w in ws], poisson_rtol=1e-12, poisson_maxit=maxit)
    t_setup = time.perf_counter() - t_setup
    lay = op.layout()
    log(f"batch of {op.n_inst} set up in {t_setup:.1f} s: {op.n_dof} DoF in total")

    def guess(i, mesh):
        xyz = mesh.coords()[:lay[i, 1]]
        half = abs(ws[i]["nuclei"][0][1][2])
        return h2_guess(xyz, half)

    phi = torch.from_numpy(np.ascontiguousarray(np.concatenate([guess(i, m) for i, m in enumerate(meshes)]))).cuda()
    op.fill_hanging(phi)
    return ws, meshes, op, lay, phi, t_setup


def run_batch(args):
    """64 uneven H2 instances in one batch against 64 sequential plain runs."""
    import numpy as np
    import torch
    import paper_2301_02387_amd as mh
    from synth import h2_ci_guess, pulse
    from paper_2301_02387_amd.tune import autotune

    if args.seq_steps is None:
        args.seq_steps = args.steps
    ws, meshes, op, lay, phi, t_setup = batch_setup(args)
    w0 = ws[0]
    Ci = torch.from_numpy(np.stack([h2_ci_guess()] * op.n_inst)).cuda()
    W = torch.zeros((op.n_full, op.n_pair_cols), dtype=torch.float64, device="cuda")
    dt, m, cycles = w0["dt"], w0["krylov"], w0["cycles"]
    Tp = cycles * 2 * np.pi / 0.0569542
    if args.tune_cache:  # cached schedules already for the warm-up
        from paper_2301_02387_amd.tune import apply_cached
        log(f"schedules from the cache: {apply_cached(op, args.tune_cache)}")
    if args.warmup > 0:
        op.propagate(phi, Ci, W, [0.0] * (args.warmup + 1), 0.05, m=m, imaginary=True, final=False)
    t0 = Tp / 2
    # field shape for the batch's steps and the sequential runs' untimed + timed steps
    shape = [float(pulse(t0 + k * dt, 1.0, cycles)) for k in range(max(args.steps, args.seq_steps + 1) + 1)]
    op.propagate(phi, Ci, W, shape[:2], dt, m=m, final=False)
    sched = autotune(op, phi, W, cache_file=args.tune_cache)
    log(f"warm-up and tuning done: {sched['orbital']} {sched['poisson']}")
    op.kernel_timing(0, True)
    op.kernel_timing(1, True)
    torch.cuda.synchronize()
    t_a = time.perf_counter()
    rec = op.propagate(phi, Ci, W, shape[:args.steps + 1], dt, m=m, final=False, graph=args.graph,
                       graph_step=args.graph_step)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_a
    k_orb = op.kernel_timing(0, False)
    k_poi = op.kernel_timing(1, False)
    log(f"batched: {wall / args.steps * 1e3:.1f} ms per step, status {rec['status']}")
    # sequential baseline: each instance alone (plain operator, with the
    # schedules tuned on the first instance alone), from this batch's current
    # state, `seq_steps` timed steps after one untimed step
    seq_sched = None
    seq_step_s = 0.0
    seq_iters = []
    ph_all = phi.clone()
    C_all = Ci.clone()
    for i, mesh in enumerate(meshes):
        if args.no_sequential:
            break
        w = ws[i]
        one = mh.Operator(mesh, w["nuclei"], w["n_orb"], w["n_alpha"], w["n_beta"], poisson_rtol=1e-12,
                          poisson_maxit=20000)
        a, b = lay[i, 3], lay[i, 3] + lay[i, 1]
        Ei = [w["E0"] * v for v in shape[:args.seq_steps + 2]]

        def start():
            return (ph_all[a:b].clone(), C_all[i:i + 1].clone(),
                    torch.zeros((one.n_full, one.n_pair_cols), dtype=torch.float64, device="cuda"))
        if seq_sched is None:
            ph, C1, W1 = start()
            one.propagate(ph, C1, W1, Ei[:2], dt, m=m, final=False)
            seq_sched = autotune(one, ph, W1)
            log(f"sequential schedules (tuned on instance 0): {seq_sched['orbital']} {seq_sched['poisson']}")
        else:
            one.tune(0, *seq_sched["orbital"])
            one.tune(1, *seq_sched["poisson"])
        # the untimed step also builds what the schedules need on first use
        ph, C1, W1 = start()
        one.propagate(ph, C1, W1, Ei[:2], dt, m=m, final=False)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        r1 = one.propagate(ph, C1, W1, Ei[1:args.seq_steps + 2], dt, m=m, final=False)
        torch.cuda.synchronize()
        seq_step_s += (time.perf_counter() - ts) / args.seq_steps
        seq_iters.append(float(np.mean(r1["cg_iters"][:args.seq_steps])))
        del one
        if i % 8 == 7:
            log(f"sequential: {i + 1} instances, {seq_step_s * 1e3:.1f} ms per step so far")
    evals = args.steps * m * op.n_dof * op.n_orb
    n_cells = sum(mm.info["n_cells"] for mm in meshes)
    ncol = op.n_pair_cols
    # matrix-free bytes summed over the instances (one aggregate mesh record)
    agg = {"p": w0["p"], "n_cells": n_cells, "hang_nnz": sum(mm.info["hang_nnz"] for mm in meshes),
           "n_full": sum(mm.info["n_full"] for mm in meshes)}
    spmv_b = poisson_algorithmic_bytes(agg, op, bool(sched["poisson"][0] & 8))
    spmv_over = stored_matrix_bytes(op.n_dof, op.n_poisson_nnz, op.n_inst)
    P3 = (w0["p"] + 1) ** 3
    NE, N, n = op.n_ext, op.n_dof, op.n_orb
    orb_bytes = 32 * n * NE + 8 * n * n * NE + 24 * NE + 8 * N + 32 * NE + 4 * P3 * n_cells + 8 * n_cells + 4 * N
    kern = {"stencil_orb": {"avg_ms": k_orb[0], "count": k_orb[1], "algorithmic_bytes": orb_bytes},
            "poisson_spmv": {"avg_ms": k_poi[0], "count": k_poi[1], "algorithmic_bytes": spmv_b}}
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["count"])
    byts = kern[dom]["algorithmic_bytes"]
    ach = byts / (kern[dom]["avg_ms"] * 1e-3) / 1e9 if kern[dom]["avg_ms"] > 0 else 0.0
    batch_tag = "/".join(map(str, sched["poisson"] if dom == "poisson_spmv" else sched["orbital"]))
    ms_step = wall / args.steps * 1e3
    line = {
        "metric": "orbital-RHS evals/s (DoF x orbitals/s)",
        "value": evals / wall,
        "unit": "DoF*orbitals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"h2x{op.n_inst}_q3_{op.n_dof}dof_{op.n_orb}orb", "n_inst": op.n_inst,
                   "n_dof_total": op.n_dof, "n_dof_min": int(lay[:, 0].min()), "n_dof_max": int(lay[:, 0].max()),
                   "n_cells_total": n_cells, "krylov": m, "dt": dt, "graph": bool(args.graph),
                   "graph_step": bool(args.graph_step),
                   "parallelism": "none (one GPU, batch of instances)"},
        "batched_vs_sequential": (seq_step_s * 1e3 / ms_step) if not args.no_sequential else None,
        "sequential_ms_per_step": seq_step_s * 1e3,
        "sequential_sample": f"each of the {op.n_inst} instances alone, {args.seq_steps} timed step(s) after one "
                             f"untimed step, schedules tuned on instance 0 alone",
        "sequential_schedule": ({"orbital": list(seq_sched["orbital"]), "poisson": list(seq_sched["poisson"])}
                                if seq_sched else None),
        "poisson_cg_iters_per_step": float(np.mean(rec["cg_iters"][:args.steps])),
        "sequential_cg_iters_per_step_mean": float(np.mean(seq_iters)) if seq_iters else None,
        "setup_s": t_setup,
        "schedule": {"orbital": list(sched["orbital"]), "poisson": list(sched["poisson"]),
                     "tuning_ms": sched.get("timings_ms")},
        "kernels": kern,
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, f"h2x{op.n_inst}_q3_{op.n_dof}dof_{op.n_orb}orb",
                                                 schedule=batch_tag),
                     "schedule": batch_tag, "algorithmic_bytes_per_launch": byts,
                     "algorithmic_bytes": "matrix-free: operand and result rows, cell maps, constraint rows, h",
                     "stored_operator_bytes_per_launch": spmv_over if dom == "poisson_spmv" else 0},
        "roofline_orbital": {"kernel": "stencil_orb", "bound": "hbm",
                             "achieved": (orb_bytes / (k_orb[0] * 1e-3) / 1e9) if k_orb[0] > 0 else 0.0,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": ((orb_bytes / (k_orb[0] * 1e-3) / 1e9) if k_orb[0] > 0 else 0.0) / HBM_PEAK_GBS,
                             "algorithmic_bytes_per_launch": orb_bytes},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
