"""GPU parity of batched execution: several instances of uneven meshes
(different ball placements, nuclei and field amplitudes) propagated in the
same kernel launches, each compared with the CPU oracle run alone on its
own mesh; the graph-replayed step against the eager step; a batch of one
against the plain operator."""
import numpy as np
import pytest

from synth import random_ci, random_orbitals
from tests.lib_cases import Pair, rel_err_cols

pytestmark = pytest.mark.gpu

SEEDS = [0, 1, 2, 4]
E0 = [1.0, 0.5, 1.7, 0.8]


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


_CACHE = {}


def batch_case():
    """Pairs (library mesh + oracle) of the instances and the batched operator."""
    if "b" not in _CACHE:
        import paper_2301_02387_amd as mh
        pairs = [Pair("tiny_q3", seed=s, with_op=False) for s in SEEDS]
        w = pairs[0].w
        op = mh.Operator.batch([P.mesh for P in pairs], [P.w["nuclei"] for P in pairs], w["n_orb"], w["n_alpha"],
                               w["n_beta"], field_scale=E0, poisson_rtol=1e-13, poisson_maxit=20000)
        _CACHE["b"] = (pairs, op)
    return _CACHE["b"]


def initial_state(pairs, n_ci):
    from oracle.mctdhf import orthonormalize
    cs, Cs = [], []
    for i, P in enumerate(pairs):
        om = P.om
        c = random_orbitals(om.xyz[om.dof_nodes], P.w["n_orb"], 30 + i, spread=1.5)
        cs.append(orthonormalize(P.ops, c))
        Cs.append(random_ci(n_ci, 40 + i))
    return cs, Cs


def to_device(pairs, cs, Cs):
    torch = _torch()
    x = np.concatenate([P.to_lib_orb(c) for P, c in zip(pairs, cs)], axis=0)
    return torch.from_numpy(np.ascontiguousarray(x)).cuda(), torch.from_numpy(np.stack(Cs)).cuda()


def test_layout_is_concatenation():
    pairs, op = batch_case()
    lay = op.layout()
    assert op.n_inst == len(SEEDS)
    assert list(lay[:, 0]) == [P.N for P in pairs]
    assert list(lay[:, 1]) == [P.NE for P in pairs]
    assert list(lay[:, 2]) == [P.NF for P in pairs]
    assert list(lay[:, 3]) == list(np.concatenate([[0], np.cumsum(lay[:-1, 1])]))
    assert list(lay[:, 4]) == list(np.concatenate([[0], np.cumsum(lay[:-1, 2])]))
    assert len(set(lay[:, 0])) == len(SEEDS)  # uneven sizes


@pytest.mark.parametrize("imag,steps,orb,poi", [(False, 3, 1, 13), (True, 2, 1, 13), (False, 3, 4, 53),
                                                 (False, 3, 4, 117)])
def test_batch_propagate_matches_oracle(imag, steps, orb, poi):
    """Each instance of the batch against the oracle on its own mesh, with the
    default schedules and with those the batch bench tunes to (assembled
    orbital stiffness; multigrid CG with sliced-ELL rows)."""
    torch = _torch()
    from oracle.ci import CISpace
    from oracle.mctdhf import Propagator
    pairs, op = batch_case()
    op.tune(0, orb, 65536)
    op.tune(1, poi, 8192 if poi == 13 else 1024)
    w = pairs[0].w
    n = w["n_orb"]
    cs_space = CISpace(n, w["n_alpha"], w["n_beta"])
    cs, Cs = initial_state(pairs, cs_space.dim)
    x, Cd = to_device(pairs, cs, Cs)
    W = torch.zeros((op.n_full, n * n), dtype=torch.float64, device="cuda")
    dt = 0.02
    shape = [0.0 if imag else 0.05 * np.sin(0.3 * k) for k in range(steps + 1)]
    rec = op.propagate(x, Cd, W, shape, dt, m=12, imaginary=imag)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    Ch = Cd.cpu().numpy()
    lay = op.layout()
    for i, P in enumerate(pairs):
        pr = Propagator(P.ops, cs_space)
        cc, CC = cs[i].copy(), Cs[i].copy()
        recs = []
        for k in range(steps):
            cc, CC, ob = pr.step(cc, CC, E0[i] * shape[k], dt, 12, imaginary=imag)
            recs.append(ob)
        recs.append(pr.final_observables(cc, CC, E0[i] * shape[-1]))
        d_ref = np.array([r["dipole"] for r in recs])
        e_ref = np.array([r["energy"] for r in recs])
        assert np.max(np.abs(rec["dipole"][:, i] - d_ref)) <= 1e-8 * max(np.abs(d_ref).max(), 1e-3), i
        assert np.max(np.abs(rec["energy"][:, i] - e_ref)) <= 1e-8 * np.abs(e_ref).max(), i
        oE, NE = lay[i, 3], lay[i, 1]
        assert rel_err_cols(P.from_lib_dof(xh[oE:oE + NE]), cc) < 1e-8, i
        assert np.max(np.abs(Ch[i] - CC)) < 1e-8, i
    op.tune(0, 1, 65536)
    op.tune(1, 13, 8192)


def test_batch_multigrid_poisson():
    """Multigrid-preconditioned CG over the batch (a hierarchy per instance,
    the V-cycles in shared launches): every instance's pair potentials against
    the oracle's solve on its own mesh, in far fewer iterations than the
    Jacobi-preconditioned CG."""
    torch = _torch()
    from oracle.ci import CISpace
    from oracle.poisson import PoissonSolver
    pairs, op = batch_case()
    w = pairs[0].w
    n = w["n_orb"]
    cs, Cs = initial_state(pairs, CISpace(n, w["n_alpha"], w["n_beta"]).dim)
    x, _ = to_device(pairs, cs, Cs)
    lay = op.layout()
    refs = [PoissonSolver(P.ops).pair_potentials(c) for P, c in zip(pairs, cs)]
    its = {}
    try:
        for sched in (13, 21):
            op.tune(1, sched, 1024)
            for rep in range(2):  # the second solve reuses the hierarchies
                W = torch.zeros((op.n_full, n * n), dtype=torch.float64, device="cuda")
                it, rc = op.poisson_pairs(x, W)
                assert rc == 0, (sched, rep)
                its[sched] = it
                Wh = W.cpu().numpy()
                for i, P in enumerate(pairs):
                    oF, NF = lay[i, 4], lay[i, 2]
                    got = P.W_from_lib(Wh[oF:oF + NF], n)
                    for k, ref in refs[i].items():
                        num = np.sqrt(np.sum(P.ops.m * np.abs(got[k] - ref) ** 2))
                        den = np.sqrt(np.sum(P.ops.m * np.abs(ref) ** 2))
                        assert num / den < 1e-9, (sched, rep, i, k, num / den)
    finally:
        op.tune(1, 13, 8192)
    print("batch CG iterations jacobi / multigrid", its, flush=True)
    assert its[21] <= 60 and its[21] * 4 < its[13], its


@pytest.mark.parametrize("orb,poi", [(1, 13), (4, 53)])
def test_graph_replay_matches_eager(orb, poi):
    """The step replayed from a HIP graph against the eager step, with the
    default schedules and with those the batch bench tunes to (the assembled
    orbital stiffness inside the graph, multigrid CG before it)."""
    torch = _torch()
    pairs, op = batch_case()
    w = pairs[0].w
    n = w["n_orb"]
    from oracle.ci import CISpace
    cs, Cs = initial_state(pairs, CISpace(n, w["n_alpha"], w["n_beta"]).dim)
    shape = [0.05 * np.sin(0.3 * k) for k in range(6)]
    out = {}
    try:
        op.tune(0, orb, 65536)
        op.tune(1, poi, 8192 if poi == 13 else 1024)
        for graph in (False, True):
            x, Cd = to_device(pairs, cs, Cs)
            W = torch.zeros((op.n_full, n * n), dtype=torch.float64, device="cuda")
            rec = op.propagate(x, Cd, W, shape, 0.02, m=12, graph=graph)
            torch.cuda.synchronize()
            out[graph] = (rec, x.cpu().numpy(), Cd.cpu().numpy())
    finally:
        op.tune(0, 1, 65536)
        op.tune(1, 13, 8192)
    (r0, x0, c0), (r1, x1, c1) = out[False], out[True]
    # every replay (one per step) against the eager step, with host syncs
    # between replays.  Not bitwise: the Poisson boundary lift accumulates
    # with FP64 atomics, so even two eager runs differ in the last bits.
    for k in ("dipole", "energy"):
        assert np.max(np.abs(r0[k] - r1[k])) <= 1e-12 * np.abs(r0[k]).max(), k
    assert np.max(np.abs(x0 - x1)) <= 1e-12 * np.abs(x0).max()
    assert np.max(np.abs(c0 - c1)) <= 1e-12


def test_batch_of_one_equals_plain_operator():
    torch = _torch()
    import paper_2301_02387_amd as mh
    P = Pair("tiny_q3", seed=1)
    w = P.w
    plain = P.op
    one = mh.Operator.batch([P.mesh], [w["nuclei"]], w["n_orb"], w["n_alpha"], w["n_beta"])
    from oracle.ci import CISpace
    cs, Cs = initial_state([P], CISpace(w["n_orb"], w["n_alpha"], w["n_beta"]).dim)
    recs = []
    for op in (plain, one):
        x, Cd = to_device([P], cs, Cs)
        W = torch.zeros((op.n_full, w["n_orb"] ** 2), dtype=torch.float64, device="cuda")
        rec = op.propagate(x, Cd, W, [0.01, 0.02, 0.0], 0.02, m=10)
        torch.cuda.synchronize()
        recs.append((rec["dipole"], rec["energy"], x.cpu().numpy()))
    # same kernels and data; only the atomic order of the Poisson boundary lift differs
    assert np.max(np.abs(recs[0][0] - recs[1][0])) <= 1e-12 * np.abs(recs[0][0]).max()
    assert np.max(np.abs(recs[0][1] - recs[1][1])) <= 1e-12 * np.abs(recs[0][1]).max()
    assert np.max(np.abs(recs[0][2] - recs[1][2])) <= 1e-12 * np.abs(recs[0][2]).max()


def test_batch_multigrid_mixed_depths():
    """A batch whose instances have multigrid hierarchies of different depths,
    one of them a single level (an unrefined odd Q1 grid, solved by the dense
    inverse of its whole operator) beside refined Q1 meshes with several
    levels: every instance's pair potentials against the oracle, with the
    Jacobi, multigrid and sliced-ELL multigrid schedules."""
    torch = _torch()
    import paper_2301_02387_amd as mh
    from oracle.ci import CISpace
    from oracle.poisson import PoissonSolver
    pairs = [Pair("tiny_q1", seed=0, with_op=False), Pair("uniform_q1_odd", with_op=False),
             Pair("tiny_q1", seed=1, with_op=False)]
    assert pairs[1].Nh == 0 and pairs[0].Nh > 0
    w = pairs[0].w
    n = w["n_orb"]
    op = mh.Operator.batch([P.mesh for P in pairs], [P.w["nuclei"] for P in pairs], n, w["n_alpha"], w["n_beta"],
                           poisson_rtol=1e-13, poisson_maxit=20000)
    cs, Cs = initial_state(pairs, CISpace(n, w["n_alpha"], w["n_beta"]).dim)
    x, _ = to_device(pairs, cs, Cs)
    lay = op.layout()
    refs = [PoissonSolver(P.ops).pair_potentials(c) for P, c in zip(pairs, cs)]
    its = {}
    for sched in (13, 21, 53):
        op.tune(1, sched, 1024)
        for rep in range(2):
            W = torch.zeros((op.n_full, n * n), dtype=torch.float64, device="cuda")
            it, rc = op.poisson_pairs(x, W)
            assert rc == 0, (sched, rep)
            its[sched] = it
            Wh = W.cpu().numpy()
            for i, P in enumerate(pairs):
                oF, NF = lay[i, 4], lay[i, 2]
                got = P.W_from_lib(Wh[oF:oF + NF], n)
                for k, ref in refs[i].items():
                    num = np.sqrt(np.sum(P.ops.m * np.abs(got[k] - ref) ** 2))
                    den = np.sqrt(np.sum(P.ops.m * np.abs(ref) ** 2))
                    assert num / den < 1e-9, (sched, rep, i, k, num / den)
    print("mixed-depth batch CG iterations", its, flush=True)
    assert its[21] < its[13] and its[53] < its[13], its


def test_batch_workload_instances_equal_plain_runs():
    """Three instances of the 64-molecule workload itself (refinement depths
    2, 3 and 4: 45k-120k unknowns each) propagated as one batch and each on
    its own plain operator, with the same schedules (the interface mass block
    by Chebyshev on both sides) and the same inputs.  The two runs differ
    only in the order of FP64 atomic sums (Poisson boundary lift, CG
    accumulators), the Chebyshev count (the batch takes the largest) and the
    CG iteration count (the batch iterates until every instance has met the
    1e-13 target), so dipoles, energies, orbitals and CI vectors agree to the
    CG target, not bitwise: measured up to 2.4e-12 (orbitals, relative), 2e-13
    (CI vector), 7e-14 (energies, relative) and 6e-13 bohr (dipoles), so the
    gate is 1e-11."""
    torch = _torch()
    import paper_2301_02387_amd as mh
    from synth import batch_instances, h2_guess, h2_ci_guess
    ws, seen = [], set()
    for i, w in enumerate(batch_instances()):
        depth = w["balls"][0]["levels"]
        if depth not in seen:
            seen.add(depth)
            ws.append(w)
    assert sorted(w["balls"][0]["levels"] for w in ws) == [2, 3, 4]
    meshes = [mh.Mesh.from_workload(w) for w in ws]
    kw = dict(poisson_rtol=1e-13, poisson_maxit=20000)
    E0 = [w["E0"] for w in ws]
    batch = mh.Operator.batch(meshes, [w["nuclei"] for w in ws], 2, 1, 1, field_scale=E0, **kw)
    plains = [mh.Operator(m, w["nuclei"], 2, 1, 1, **kw) for m, w in zip(meshes, ws)]
    xs = []
    for m, w, op in zip(meshes, ws, plains):
        NE = op.n_ext
        xyz = m.coords()[:NE]
        x = torch.from_numpy(np.ascontiguousarray(h2_guess(xyz, w["nuclei"][0][1][2]))).cuda()
        op.fill_hanging(x)
        xs.append(x)
    shape = [np.sin(0.3 + 0.2 * k) for k in range(4)]
    for orb, poi in ((3, 13), (6, 53)):          # bit 1 of the orbital schedule: Chebyshev interface solve
        batch.tune(0, orb, 65536)
        batch.tune(1, poi, 1024)
        xb = torch.cat([x.clone() for x in xs], dim=0)
        Cb = torch.from_numpy(np.stack([h2_ci_guess()] * 3)).cuda()
        Wb = torch.zeros((batch.n_full, 4), dtype=torch.float64, device="cuda")
        rb = batch.propagate(xb, Cb, Wb, shape, 0.02, m=12)
        assert rb["status"] == 0
        lay = batch.layout()
        for i, op in enumerate(plains):
            op.tune(0, orb, 65536)
            op.tune(1, poi, 8192)
            x = xs[i].clone()
            C = torch.from_numpy(h2_ci_guess()[None, :].copy()).cuda()
            W = torch.zeros((op.n_full, 4), dtype=torch.float64, device="cuda")
            rp = op.propagate(x, C, W, [E0[i] * v for v in shape], 0.02, m=12)
            assert rp["status"] == 0
            torch.cuda.synchronize()
            # the field-induced dipole of these symmetric molecules is 1e-2 bohr
            # or less, a small difference of large contributions of either
            # sign, so its difference is taken in bohr (the molecules span
            # about one bohr)
            dd = np.max(np.abs(rb["dipole"][:, i] - rp["dipole"]))
            de = np.max(np.abs(rb["energy"][:, i] - rp["energy"])) / np.abs(rp["energy"]).max()
            oE, NE = lay[i, 3], lay[i, 1]
            xh = x.cpu().numpy()
            dx = np.abs(xb.cpu().numpy()[oE:oE + NE] - xh).max() / np.abs(xh).max()
            dc = np.abs(Cb.cpu().numpy()[i] - C.cpu().numpy()[0]).max()
            print(f"instance depth {ws[i]['balls'][0]['levels']} ({op.n_dof} unknowns), schedules {orb}/{poi}: "
                  f"dipole {dd:.2e} (max |d| {np.abs(rp['dipole']).max():.2e}) energy {de:.2e} "
                  f"orbitals {dx:.2e} CI {dc:.2e}", flush=True)
            assert max(dd, de, dx, dc) <= 1e-11, (i, orb, poi, dd, de, dx, dc)


@pytest.mark.parametrize("orb,poi", [(4, 53), (4, 117)])
def test_whole_step_graph_matches_eager(orb, poi):
    """Whole steps replayed from one HIP graph (MH_PROP_GRAPH_STEP: RDMs, CG
    start, pair Poisson solves with a fixed multigrid-CG count, boundary
    values, the step's field value from the device table, freeze, integrals,
    Arnoldi and CI steps) against the eager steps: from the fourth step on
    every step is one replay, with the host reading records between the
    replays.  Each replayed step's records and the final state equal the
    eager run's up to the CG target (the fixed count runs past it)."""
    torch = _torch()
    pairs, op = batch_case()
    w = pairs[0].w
    n = w["n_orb"]
    from oracle.ci import CISpace
    cs, Cs = initial_state(pairs, CISpace(n, w["n_alpha"], w["n_beta"]).dim)
    shape = [0.05 * np.sin(0.3 * k) for k in range(8)]
    out = {}
    try:
        op.tune(0, orb, 65536)
        op.tune(1, poi, 1024)
        for mode in ("eager", "graph_step"):
            x, Cd = to_device(pairs, cs, Cs)
            W = torch.zeros((op.n_full, n * n), dtype=torch.float64, device="cuda")
            rec = op.propagate(x, Cd, W, shape, 0.02, m=12, graph_step=(mode == "graph_step"))
            torch.cuda.synchronize()
            assert rec["status"] == 0, mode
            out[mode] = (rec, x.cpu().numpy(), Cd.cpu().numpy())
    finally:
        op.tune(0, 1, 65536)
        op.tune(1, 13, 8192)
    (r0, x0, c0), (r1, x1, c1) = out["eager"], out["graph_step"]
    print("cg iterations eager", r0["cg_iters"], "graph", r1["cg_iters"], flush=True)
    assert np.all(r1["cg_iters"][3:7] >= r0["cg_iters"][3:7])
    for k in ("dipole", "energy", "momentum"):
        assert np.max(np.abs(r0[k] - r1[k])) <= 1e-10 * max(np.abs(r0[k]).max(), 1e-3), k
    assert np.max(np.abs(x0 - x1)) <= 1e-10 * np.abs(x0).max()
    assert np.max(np.abs(c0 - c1)) <= 1e-10
