"""GPU parity of the velocity gauge (Sec. II: the one-body operator carries
-i A(t).grad): the Gauss-Lobatto derivative term in its antisymmetric form,
applied node by node with the stiffness's line sums, against the oracle's
assembled matrices; the kinetic momentum record (velocity form of the
dipole) in both gauges.

Bars: operator applications <= 1e-10 relative per orbital and element-wise;
propagated dipoles, energies and momenta <= 1e-8."""
import numpy as np
import pytest

from synth import random_orbitals, random_ci
from tests.lib_cases import Pair, rel_err_cols, max_rel_cols, poisson_solver

pytestmark = pytest.mark.gpu

_PAIRS = {}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def pair(name, **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _PAIRS:
        from oracle.fem import Operators
        P = Pair(name, gauge="velocity", **kw)
        P.opv = Operators(P.om, P.w["nuclei"], gauge="velocity")   # the oracle in the velocity gauge
        _PAIRS[key] = P
    return _PAIRS[key]


def dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def orbitals(P, seed):
    from oracle.mctdhf import orthonormalize
    om = P.om
    return orthonormalize(P.ops, random_orbitals(om.xyz[om.dof_nodes], P.w["n_orb"], seed, spread=1.5))


@pytest.mark.parametrize("name", ["h_atom", "tiny_q3", "tiny_q1", "small_n3", "uniform_q2", "h2"])
def test_h1_apply_velocity(name):
    torch = _torch()
    P = pair(name)
    n = P.w["n_orb"]
    c = orbitals(P, 2)
    for A in (0.0, 0.37, -1.3):
        f = torch.zeros((P.N, n), dtype=torch.complex128, device="cuda")
        P.op.h1_apply(dev(P.to_lib_orb(c)), A, f)
        ref = P.opv.H1(A) @ c
        got = P.from_lib_dof(host(f))
        assert rel_err_cols(got, ref) < 1e-10 and max_rel_cols(got, ref) < 1e-10, A


@pytest.mark.parametrize("name", ["h_atom", "tiny_q3", "small_n3", "h2"])
def test_rhs_apply_velocity(name):
    """G with the velocity term; the orbital schedules that take the
    stiffness from the assembled operator fall back to the node pass."""
    torch = _torch()
    from oracle.ci import CISpace
    from oracle.mctdhf import Frozen
    P = pair(name)
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    c = orbitals(P, 5)
    C = random_ci(cs.dim, 6)
    gam, Gam = cs.rdms(C)
    W = poisson_solver(P.ops).pair_potentials(c)
    A = 0.21
    fr = Frozen(P.opv, c, gam, Gam, A, W)
    P.op.freeze(dev(P.to_lib_orb(c)), dev(gam), dev(Gam), A, dev(P.W_to_lib(W, n)))
    v = orbitals(P, 7)
    ref = fr.G(v)
    for orb_sched in (1, 3, 5):
        P.op.tune(0, orb_sched, 65536)
        out = torch.zeros((P.NE, n), dtype=torch.complex128, device="cuda")
        P.op.rhs_apply(dev(P.to_lib_orb(v)), out)
        got = P.from_lib_dof(host(out))
        assert rel_err_cols(got, ref) < 1e-10 and max_rel_cols(got, ref) < 1e-10, orb_sched
    P.op.tune(0, 1, 65536)


@pytest.mark.parametrize("name,steps", [("h_atom", 4), ("tiny_q3", 3), ("small_n3", 3)])
def test_propagate_velocity(name, steps):
    torch = _torch()
    from oracle.ci import CISpace
    from oracle.mctdhf import Propagator
    P = pair(name, poisson_rtol=1e-13, poisson_maxit=20000)
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    c = orbitals(P, 10)
    C = random_ci(cs.dim, 11)
    dt = 0.02
    A_steps = [0.3 * np.sin(0.5 * k + 0.2) for k in range(steps + 1)]
    x, Cd = dev(P.to_lib_orb(c)), dev(C)
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    rec = P.op.propagate(x, Cd, W, A_steps, dt, m=12)
    pr = Propagator(P.opv, cs, poisson_solver(P.ops))
    recs = []
    cc, CC = c.copy(), C.copy()
    for k in range(steps):
        cc, CC, ob = pr.step(cc, CC, A_steps[k], dt, 12)
        recs.append(ob)
    recs.append(pr.final_observables(cc, CC, A_steps[-1]))
    for key in ("dipole", "energy", "momentum"):
        ref = np.array([r[key] for r in recs])
        diff = np.max(np.abs(rec[key] - ref)) / max(np.abs(ref).max(), 1e-3)
        print(name, key, diff, flush=True)
        assert diff <= 1e-8, key
    assert rel_err_cols(P.from_lib_dof(host(x)), cc) < 1e-8
    assert np.max(np.abs(host(Cd) - CC)) < 1e-8


def test_momentum_record_length_gauge():
    """The kinetic momentum record in the length gauge (no A term) against the
    oracle, beside the dipole and energy."""
    torch = _torch()
    from oracle.ci import CISpace
    from oracle.mctdhf import Propagator
    P = Pair("small_n3", poisson_rtol=1e-13, poisson_maxit=20000)
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    c = orbitals(P, 12)
    C = random_ci(cs.dim, 13)
    E_steps = [0.05 * np.sin(0.3 * k) for k in range(4)]
    x, Cd = dev(P.to_lib_orb(c)), dev(C)
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    rec = P.op.propagate(x, Cd, W, E_steps, 0.02, m=12)
    _, _, recs = Propagator(P.ops, cs, poisson_solver(P.ops)).propagate(c, C, E_steps[:-1], 0.02, 12)
    ref = np.array([r["momentum"] for r in recs])
    assert np.max(np.abs(rec["momentum"] - ref)) <= 1e-8 * max(np.abs(ref).max(), 1e-3)


def test_adjoint_rejects_the_velocity_gauge():
    torch = _torch()
    import paper_2301_02387_amd as mh
    P = pair("tiny_q3")
    n = P.w["n_orb"]
    x = dev(P.to_lib_orb(orbitals(P, 3)))
    C = dev(random_ci(4, 2))
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    with pytest.raises(mh.MHError) as e:
        P.op.propagate_adjoint(x, C, W, [0.0, 0.1, 0.2], 0.02, np.ones(3))
    assert e.value.code == -6
