"""GPU parity: every entry point of the C ABI against the CPU oracle on the
same seeded inputs (small meshes spanning several cell tiles and a ragged
tail, plus the full H2 mesh).

Bar: operator applications (h1_apply, mass_solve, rhs_apply, arnoldi_step)
max over orbitals of |y_gpu - y_oracle|_2 / |y_oracle|_2 <= 1e-10, and
element-wise max_i |y_gpu - y_oracle| <= 1e-10 of each column's largest
entry; Poisson potentials <= 1e-10 in the m-weighted norm and element-wise
(CG driven to 1e-13 relative residual against the oracle's direct solve);
propagated dipoles and energies <= 1e-8.
"""
import numpy as np
import pytest

from synth import random_orbitals, random_ci
from tests.lib_cases import Pair, rel_err_cols, max_rel_cols, poisson_solver

pytestmark = pytest.mark.gpu

# kelly_*: meshes refined by Kelly's indicator of the nuclear potential (no
# balls; hanging faces at every level), with the field along x
SMALL = ["h_atom", "tiny_q3", "tiny_q1", "small_n3", "kelly_q1", "kelly_q2"]
# unrefined meshes: no hanging nodes, no interface mass block; on the odd Q1
# grid the multigrid hierarchy is the operator alone (dense inverse)
UNIFORM = ["uniform_q2", "uniform_q1_odd"]


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


_PAIRS = {}


def pair(name, **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _PAIRS:
        _PAIRS[key] = Pair(name, **kw)
    return _PAIRS[key]


def dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def orbitals(P, seed):
    om = P.om
    from oracle.mctdhf import orthonormalize
    c = random_orbitals(om.xyz[om.dof_nodes], P.w["n_orb"], seed, spread=1.5)
    return orthonormalize(P.ops, c)


@pytest.mark.parametrize("name", SMALL + UNIFORM)
def test_fill_hanging_and_mass_solve(name):
    torch = _torch()
    P = pair(name)
    n = P.w["n_orb"]
    c = orbitals(P, 1)
    x = dev(P.to_lib_orb(c))
    y = x.clone()
    y[P.N:] = 0
    P.op.fill_hanging(y)
    assert np.max(np.abs(host(y) - host(x))) < 1e-13 * np.abs(host(x)).max()
    f_or = (P.ops.M @ c)
    f = dev(np.ascontiguousarray(f_or[P.dof_or]))
    out = torch.zeros((P.NE, n), dtype=torch.complex128, device="cuda")
    P.op.mass_solve(f, out)
    ref = P.ops.mass_solve(f_or)
    o = host(out)
    assert rel_err_cols(P.from_lib_dof(o), ref) < 1e-12
    assert max_rel_cols(P.from_lib_dof(o), ref) < 1e-12
    if P.Nh:
        assert rel_err_cols(o[P.N:], (P.om.C @ ref)[P.perm[P.N:P.NE]]) < 1e-12


@pytest.mark.parametrize("name", SMALL + UNIFORM + ["h2"])
def test_h1_apply(name):
    torch = _torch()
    P = pair(name)
    n = P.w["n_orb"]
    c = orbitals(P, 2)
    E = 0.0317
    f = torch.zeros((P.N, n), dtype=torch.complex128, device="cuda")
    P.op.h1_apply(dev(P.to_lib_orb(c)), E, f)
    ref = P.ops.H1(E) @ c
    assert rel_err_cols(P.from_lib_dof(host(f)), ref) < 1e-10
    assert max_rel_cols(P.from_lib_dof(host(f)), ref) < 1e-10


def _poisson(P, c, rtol=1e-13):
    torch = _torch()
    n = P.w["n_orb"]
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    it, rc = P.op.poisson_pairs(dev(P.to_lib_orb(c)), W)
    return W, it, rc


@pytest.mark.parametrize("name", SMALL + UNIFORM + ["h2"])
def test_poisson_pairs(name):
    P = pair(name, poisson_rtol=1e-13, poisson_maxit=20000)
    n = P.w["n_orb"]
    c = orbitals(P, 3)
    W, it, rc = _poisson(P, c)
    assert rc == 0 and it > 0
    ref = poisson_solver(P.ops).pair_potentials(c)
    got = P.W_from_lib(host(W), n)
    worst = 0.0
    for k in ref:
        num = np.sqrt(np.sum(P.ops.m * np.abs(got[k] - ref[k]) ** 2))
        den = np.sqrt(np.sum(P.ops.m * np.abs(ref[k]) ** 2))
        el = np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max()
        worst = max(worst, num / den, el)
        assert num / den < 1e-10 and el < 1e-10, (k, num / den, el, it)
    print(name, "Poisson potentials: worst relative difference", worst, "after", it, "CG iterations", flush=True)


@pytest.mark.parametrize("name", ["tiny_q3", "small_n3", "tiny_n8"])
def test_poisson_every_schedule(name):
    """Each Poisson launch schedule (sweep order, column blocks, long rows by
    waves, direction fused into the operator pass, multigrid preconditioner,
    sliced-ELL short rows, float finest level, column blocks bound to XCDs,
    smoothing degrees 3 to 5) gives the oracle's potentials, cold and warm."""
    P = Pair(name, poisson_rtol=1e-13, poisson_maxit=20000)
    n = P.w["n_orb"]
    c = orbitals(P, 4)
    ref = poisson_solver(P.ops).pair_potentials(c)
    torch = _torch()
    x = dev(P.to_lib_orb(c))
    for sched in (884, 629, 372, 373, 277, 255, 246, 214, 182, 170, 130, 127, 117, 116, 85, 84, 63, 61, 53, 45, 44,
                  39, 37, 36, 33, 32, 31, 29, 22, 21, 20, 16, 15, 14, 13, 12, 9, 8, 7, 6, 5, 4, 2, 1, 0):
        for grid in (8, 2048):
            P.op.tune(1, sched, grid)
            W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
            it, rc = P.op.poisson_pairs(x, W)
            it2, rc2 = P.op.poisson_pairs(x, W, warm=True)
            assert rc == 0 and rc2 == 0 and it2 <= it
            got = P.W_from_lib(host(W), n)
            for k in ref:
                num = np.sqrt(np.sum(P.ops.m * np.abs(got[k] - ref[k]) ** 2))
                den = np.sqrt(np.sum(P.ops.m * np.abs(ref[k]) ** 2))
                assert num / den < 1e-9, (sched, grid, k, num / den)


@pytest.mark.parametrize("name,nci", [("tiny_q3", 4), ("small_n3", 9), ("beta_only", 2), ("full_alpha", 2)])
def test_ci_rdms(name, nci):
    torch = _torch()
    from oracle.ci import CISpace
    P = pair(name)
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    assert cs.dim == P.op.n_ci
    C = random_ci(cs.dim, 4)
    g = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    G = torch.zeros((n, n, n, n), dtype=torch.complex128, device="cuda")
    P.op.ci_rdms(dev(C), g, G)
    gr, Gr = cs.rdms(C)
    assert np.max(np.abs(host(g) - gr)) < 1e-13
    assert np.max(np.abs(host(G) - Gr)) < 1e-13


def _frozen(P, c, C, E):
    """Oracle frozen operator and the library frozen on the same inputs."""
    from oracle.ci import CISpace
    from oracle.mctdhf import Frozen
    torch = _torch()
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    gam, Gam = cs.rdms(C)
    W = poisson_solver(P.ops).pair_potentials(c)
    fr = Frozen(P.ops, c, gam, Gam, E, W)
    P.op.freeze(dev(P.to_lib_orb(c)), dev(gam), dev(Gam), E, dev(P.W_to_lib(W, n)))
    return fr, cs


@pytest.mark.parametrize("name", SMALL + UNIFORM + ["h2", "tiny_n8"])
def test_rhs_apply(name):
    """G applied to a random packed vector: interface mass block solved by the
    dense inverse (the default for one small instance) and by Chebyshev, the
    stiffness part node by node and by the assembled operator (from its CSR
    rows and from its sliced-ELL copy)."""
    torch = _torch()
    P = pair(name)
    for orb_sched in (1, 3, 5, 7):   # bit 1: Chebyshev interface solve, bit 2: assembled stiffness
        P.op.tune(0, orb_sched, 65536)
        _rhs_apply_case(P, name, torch)
    P.op.tune(1, 45, 8192)           # the assembled stiffness through the sliced-ELL rows
    for orb_sched in (5, 4):
        P.op.tune(0, orb_sched, 65536)
        _rhs_apply_case(P, name, torch)
    P.op.tune(1, 13, 8192)
    P.op.tune(0, 1, 65536)


def _rhs_apply_case(P, name, torch):
    n = P.w["n_orb"]
    c = orbitals(P, 5)
    from oracle.ci import CISpace
    dim = CISpace(n, P.w["n_alpha"], P.w["n_beta"]).dim
    fr, _ = _frozen(P, c, random_ci(dim, 6), 0.021)
    v = orbitals(P, 7)
    out = torch.zeros((P.NE, n), dtype=torch.complex128, device="cuda")
    P.op.rhs_apply(dev(P.to_lib_orb(v)), out)
    ref = fr.G(v)
    o = host(out)
    assert rel_err_cols(P.from_lib_dof(o), ref) < 1e-10
    assert max_rel_cols(P.from_lib_dof(o), ref) < 1e-10
    if P.Nh:
        assert rel_err_cols(o[P.N:], (P.om.C @ ref)[P.perm[P.N:P.NE]]) < 1e-10


@pytest.mark.parametrize("name,tau,m", [("tiny_q3", 0.02, 12), ("small_n3", 0.05, 12), ("h_atom", 0.02, 12),
                                        ("tiny_q3", -0.05j, 12), ("h2", 0.02, 12), ("tiny_q3", 0.02, 1),
                                        ("uniform_q2", 0.02, 2), ("uniform_q1_odd", 0.05, 12),
                                        ("h_atom", 0.02, 16), ("small_n3", 0.05, 24)])
def test_arnoldi_step(name, tau, m):
    from oracle.mctdhf import arnoldi_step
    P = pair(name)
    n = P.w["n_orb"]
    c = orbitals(P, 8)
    from oracle.ci import CISpace
    dim = CISpace(n, P.w["n_alpha"], P.w["n_beta"]).dim
    fr, _ = _frozen(P, c, random_ci(dim, 9), 0.013)
    x = dev(P.to_lib_orb(c))
    err, m_used = P.op.arnoldi_step(x, tau, m)
    ref, err_ref, m_ref, _ = arnoldi_step(P.ops, fr.G, c, tau, m)
    assert m_used == m_ref
    o = host(x)
    assert rel_err_cols(P.from_lib_dof(o), ref) < 1e-10
    assert max_rel_cols(P.from_lib_dof(o), ref) < 1e-10
    assert abs(err - err_ref) <= 1e-6 * err_ref + 1e-14


@pytest.mark.parametrize("name,steps,imag,sched", [("h_atom", 4, False, 13), ("tiny_q3", 4, False, 13),
                                                   ("small_n3", 3, False, 13), ("tiny_q3", 3, True, 13),
                                                   ("tiny_q3", 4, False, 21), ("small_n3", 3, False, 20),
                                                   ("tiny_q3", 4, False, 53), ("small_n3", 3, False, 52),
                                                   ("uniform_q2", 3, False, 13), ("uniform_q1_odd", 3, False, 53),
                                                   ("beta_one", 3, False, 13), ("full_alpha", 3, False, 13),
                                                   ("tiny_q3", 4, False, 117), ("small_n3", 3, False, 116),
                                                   ("kelly_q1", 3, False, 13), ("kelly_q2", 3, False, 117)])
def test_propagate_observables(name, steps, imag, sched):
    """Propagated dipoles, energies, orbitals and CI vectors against the
    oracle, with the default schedules (Poisson 13) and with the multigrid
    preconditioner (Poisson 20, 21; with the sliced-ELL rows 52, 53) and the
    assembled orbital stiffness."""
    torch = _torch()
    from oracle.ci import CISpace
    from oracle.mctdhf import Propagator
    P = pair(name, poisson_rtol=1e-13, poisson_maxit=20000)
    P.op.tune(1, sched, 8192)
    P.op.tune(0, 1 if sched == 13 else 5, 65536)   # with multigrid: the assembled orbital stiffness too
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    c = orbitals(P, 10)
    C = random_ci(cs.dim, 11)
    dt = 0.02
    E_steps = [0.0 if imag else 0.05 * np.sin(0.3 * k) for k in range(steps + 1)]
    x = dev(P.to_lib_orb(c))
    Cd = dev(C)
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    rec = P.op.propagate(x, Cd, W, E_steps, dt, m=12, imaginary=imag)
    pr = Propagator(P.ops, cs, poisson_solver(P.ops))
    recs = []
    cc, CC = c.copy(), C.copy()
    for k in range(steps):
        cc, CC, ob = pr.step(cc, CC, E_steps[k], dt, 12, imaginary=imag)
        recs.append(ob)
    recs.append(pr.final_observables(cc, CC, E_steps[-1]))
    d_ref = np.array([r["dipole"] for r in recs])
    e_ref = np.array([r["energy"] for r in recs])
    assert np.max(np.abs(rec["dipole"] - d_ref)) <= 1e-8 * max(np.abs(d_ref).max(), 1e-3)
    assert np.max(np.abs(rec["energy"] - e_ref)) <= 1e-8 * np.abs(e_ref).max()
    assert rel_err_cols(P.from_lib_dof(host(x)), cc) < 1e-8
    assert np.max(np.abs(host(Cd) - CC)) < 1e-8


def test_poisson_not_converged_status():
    torch = _torch()
    P = pair("tiny_q3", poisson_maxit=1)
    c = orbitals(P, 12)
    W, it, rc = _poisson(P, c)
    assert rc == 1 and it == 1


@pytest.mark.parametrize("name", ["tiny_q3", "small_n3", "h2", "kelly_q1", "kelly_q2"])
def test_multigrid_poisson(name):
    """The multigrid-preconditioned CG gives the oracle's potentials in a few
    tens of iterations, far fewer than the Jacobi-preconditioned one."""
    torch = _torch()
    P = Pair(name, poisson_rtol=1e-12, poisson_maxit=20000)
    n = P.w["n_orb"]
    c = orbitals(P, 4)
    ref = poisson_solver(P.ops).pair_potentials(c)
    x = dev(P.to_lib_orb(c))
    its = {}
    # Jacobi, multigrid, multigrid on float finest-level arrays (bit 6), and
    # multigrid with smoothing of degree 3 and 4 (bits 8-9)
    for sched in (13, 21, 85, 277, 533):
        P.op.tune(1, sched, 8192)
        W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
        it, rc = P.op.poisson_pairs(x, W)
        assert rc == 0
        its[sched] = it
        got = P.W_from_lib(host(W), n)
        for k in ref:
            num = np.sqrt(np.sum(P.ops.m * np.abs(got[k] - ref[k]) ** 2))
            den = np.sqrt(np.sum(P.ops.m * np.abs(ref[k]) ** 2))
            assert num / den < 1e-9, (sched, k, num / den)
    print(name, "CG iterations jacobi / multigrid / float / degree 3 / degree 4", its, flush=True)
    assert its[21] <= 60 and its[21] * 4 < its[13], its
    assert its[85] <= its[21] + 2, its
    assert its[533] <= its[277] <= its[21], its   # stronger smoothing, no more iterations


@pytest.mark.parametrize("name", UNIFORM)
def test_multigrid_poisson_unrefined(name):
    """Multigrid on unrefined meshes gives the oracle's potentials; on the odd
    Q1 grid the hierarchy is the operator itself, solved exactly by its dense
    inverse, so the preconditioned CG stops after its first iteration."""
    torch = _torch()
    P = Pair(name, poisson_rtol=1e-12, poisson_maxit=20000)
    assert P.Nh == 0
    n = P.w["n_orb"]
    c = orbitals(P, 4)
    ref = poisson_solver(P.ops).pair_potentials(c)
    x = dev(P.to_lib_orb(c))
    its = {}
    for sched in (13, 21, 53):
        P.op.tune(1, sched, 8192)
        W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
        it, rc = P.op.poisson_pairs(x, W)
        assert rc == 0
        its[sched] = it
        got = P.W_from_lib(host(W), n)
        for k in ref:
            num = np.sqrt(np.sum(P.ops.m * np.abs(got[k] - ref[k]) ** 2))
            den = np.sqrt(np.sum(P.ops.m * np.abs(ref[k]) ** 2))
            assert num / den < 1e-9, (sched, k, num / den)
    print(name, "CG iterations", its, flush=True)
    assert its[21] <= its[13] and its[53] <= its[13], its
    if name == "uniform_q1_odd":
        assert its[21] <= 2 and its[53] <= 2, its


def test_propagate_zero_steps():
    """A propagation of zero steps records the observables of the given state
    (and leaves it unchanged, its pair potentials solved into W); without the
    final record it does nothing."""
    torch = _torch()
    from oracle.ci import CISpace
    from oracle.mctdhf import Propagator
    P = pair("tiny_q3", poisson_rtol=1e-13, poisson_maxit=20000)
    P.op.tune(1, 13, 8192)
    P.op.tune(0, 1, 65536)
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    c = orbitals(P, 12)
    C = random_ci(cs.dim, 13)
    x = dev(P.to_lib_orb(c))
    Cd = dev(C)
    x0, C0 = host(x).copy(), host(Cd).copy()
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    rec = P.op.propagate(x, Cd, W, [0.013], 0.02)
    assert rec["status"] == 0 and rec["dipole"].shape == (1,)
    ref = Propagator(P.ops, cs).final_observables(c, C, 0.013)
    assert abs(rec["dipole"][0] - ref["dipole"]) <= 1e-8 * max(abs(ref["dipole"]), 1e-3)
    assert abs(rec["energy"][0] - ref["energy"]) <= 1e-8 * abs(ref["energy"])
    def unchanged():
        return (np.max(np.abs(host(x) - x0)) <= 1e-14 * np.abs(x0).max()
                and np.max(np.abs(host(Cd) - C0)) <= 1e-14 * np.abs(C0).max())

    assert unchanged()
    Wref = poisson_solver(P.ops).pair_potentials(c)
    got = P.W_from_lib(host(W), n)
    for k in Wref:
        num = np.sqrt(np.sum(P.ops.m * np.abs(got[k] - Wref[k]) ** 2))
        den = np.sqrt(np.sum(P.ops.m * np.abs(Wref[k]) ** 2))
        assert num / den < 1e-9, (k, num / den)
    W2 = torch.zeros_like(W)
    rec = P.op.propagate(x, Cd, W2, [0.013], 0.02, final=False)
    assert rec["status"] == 0
    assert unchanged()
    assert not host(W2).any()


def test_propagate_h2_full_mesh():
    """Three steps of the H2 workload itself (66,635 unknowns, Q3, two
    orbitals, four determinants) with the library's default schedules
    against the oracle: dipoles and energies <= 1e-8, orbitals and CI
    vector <= 1e-8."""
    torch = _torch()
    from oracle.ci import CISpace
    from oracle.mctdhf import Propagator
    P = pair("h2", poisson_rtol=1e-13, poisson_maxit=20000)
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    c = orbitals(P, 14)
    C = random_ci(cs.dim, 15)
    dt, steps = 0.02, 3
    E_steps = [0.0534 * np.sin(0.7 + 0.4 * k) for k in range(steps + 1)]
    x, Cd = dev(P.to_lib_orb(c)), dev(C)
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    rec = P.op.propagate(x, Cd, W, E_steps, dt, m=12)
    assert rec["status"] == 0
    pr = Propagator(P.ops, cs, poisson_solver(P.ops))
    recs = []
    cc, CC = c.copy(), C.copy()
    for k in range(steps):
        cc, CC, ob = pr.step(cc, CC, E_steps[k], dt, 12)
        recs.append(ob)
    recs.append(pr.final_observables(cc, CC, E_steps[-1]))
    d_ref = np.array([r["dipole"] for r in recs])
    e_ref = np.array([r["energy"] for r in recs])
    dd = np.max(np.abs(rec["dipole"] - d_ref)) / max(np.abs(d_ref).max(), 1e-3)
    de = np.max(np.abs(rec["energy"] - e_ref)) / np.abs(e_ref).max()
    print("h2 propagation: dipole", dd, "energy", de, flush=True)
    assert dd <= 1e-8 and de <= 1e-8
    assert rel_err_cols(P.from_lib_dof(host(x)), cc) < 1e-8
    assert np.max(np.abs(host(Cd) - CC)) < 1e-8
