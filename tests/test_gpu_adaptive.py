"""GPU parity of the adaptive Krylov dimension (Sec. III.B: the space grows
until the error estimate meets a threshold, here the paper's 1e-10): the
dimension chosen and the result of an Arnoldi step, and a propagation's
records, against the oracle's adaptive step."""
import numpy as np
import pytest

from synth import random_orbitals, random_ci
from tests.lib_cases import Pair, rel_err_cols, max_rel_cols, poisson_solver

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def orbitals(P, seed):
    from oracle.mctdhf import orthonormalize
    om = P.om
    return orthonormalize(P.ops, random_orbitals(om.xyz[om.dof_nodes], P.w["n_orb"], seed, spread=1.5))


@pytest.mark.parametrize("name,tau", [("tiny_q3", 0.02), ("small_n3", 0.05), ("h_atom", 0.02), ("tiny_q3", -0.05j)])
def test_adaptive_arnoldi_step(name, tau):
    from oracle.ci import CISpace
    from oracle.mctdhf import Frozen, arnoldi_step
    P = Pair(name, krylov_tol=TOL)
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    c = orbitals(P, 8)
    gam, Gam = cs.rdms(random_ci(cs.dim, 9))
    W = poisson_solver(P.ops).pair_potentials(c)
    fr = Frozen(P.ops, c, gam, Gam, 0.013, W)
    P.op.freeze(dev(P.to_lib_orb(c)), dev(gam), dev(Gam), 0.013, dev(P.W_to_lib(W, n)))
    x = dev(P.to_lib_orb(c))
    err, m_used = P.op.arnoldi_step(x, tau, 24)
    ref, err_ref, m_ref, _ = arnoldi_step(P.ops, fr.G, c, tau, 24, tol=TOL)
    print(name, tau, "dimension", m_used, "oracle", m_ref, flush=True)
    assert m_used == m_ref and m_ref < 24
    got = P.from_lib_dof(host(x))
    assert rel_err_cols(got, ref) < 1e-10 and max_rel_cols(got, ref) < 1e-10
    assert err <= TOL and abs(err - err_ref) <= 1e-6 * err_ref + 1e-16


@pytest.mark.parametrize("name,steps", [("tiny_q3", 3), ("small_n3", 3)])
def test_adaptive_propagation(name, steps):
    torch = _torch()
    from oracle.ci import CISpace
    from oracle.mctdhf import Propagator
    P = Pair(name, krylov_tol=TOL, poisson_rtol=1e-13, poisson_maxit=20000)
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    c = orbitals(P, 10)
    C = random_ci(cs.dim, 11)
    E_steps = [0.05 * np.sin(0.3 * k) for k in range(steps + 1)]
    x, Cd = dev(P.to_lib_orb(c)), dev(C)
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    rec = P.op.propagate(x, Cd, W, E_steps, 0.02, m=20)
    pr = Propagator(P.ops, cs, poisson_solver(P.ops))
    recs = []
    cc, CC = c.copy(), C.copy()
    for k in range(steps):
        cc, CC, ob = pr.step(cc, CC, E_steps[k], 0.02, 20, krylov_tol=TOL)
        recs.append(ob)
    recs.append(pr.final_observables(cc, CC, E_steps[-1]))
    assert list(rec["krylov_dim"][:steps]) == [r["m"] for r in recs[:steps]], rec["krylov_dim"]
    assert max(rec["krylov_dim"][:steps]) < 20
    for key in ("dipole", "energy"):
        ref = np.array([r[key] for r in recs])
        assert np.max(np.abs(rec[key] - ref)) <= 1e-8 * max(np.abs(ref).max(), 1e-3), key
    assert rel_err_cols(P.from_lib_dof(host(x)), cc) < 1e-8
    assert np.max(np.abs(host(Cd) - CC)) < 1e-8


def test_adaptive_dimension_refuses_graph_replay():
    torch = _torch()
    import paper_2301_02387_amd as mh
    P = Pair("tiny_q3", krylov_tol=TOL)
    n = P.w["n_orb"]
    x = dev(P.to_lib_orb(orbitals(P, 3)))
    C = dev(random_ci(4, 2)[None, :])
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    with pytest.raises(mh.MHError) as e:
        P.op.propagate(x, C, W, [0.0, 0.0], 0.02, m=12, graph=True)
    assert e.value.code == -1
