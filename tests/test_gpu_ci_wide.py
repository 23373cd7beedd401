"""GPU parity on CI spaces wider than the 12-vector Lanczos space: eight
orbitals with 2 alpha + 2 beta electrons (784 determinants) and six orbitals
with 3 alpha + 3 beta (400 determinants), the shape class of the CAS(10e,8o)
water workload (Sec. II, Eqs. ci_eom and orb_eom; the CI exponential is then
truncated, not exact).  The library's own RDMs feed its frozen operator.

Bars: RDMs <= 1e-13 absolute (entries O(1)); operator applications <= 1e-10
relative per orbital and element-wise <= 1e-10 of each column's largest
entry; propagated dipoles and energies <= 1e-8.
"""
import numpy as np
import pytest

from synth import random_orbitals, random_ci
from tests.lib_cases import Pair, rel_err_cols, max_rel_cols, poisson_solver

pytestmark = pytest.mark.gpu

WIDE = ["tiny_n8_2a2b", "small_n6"]
_PAIRS = {}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def pair(name, **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _PAIRS:
        _PAIRS[key] = Pair(name, **kw)
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


@pytest.mark.parametrize("name", WIDE)
def test_ci_rdms_wide(name):
    torch = _torch()
    from oracle.ci import CISpace
    P = pair(name)
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    assert cs.dim == P.op.n_ci and cs.dim > 12
    for seed in (4, 5):
        C = random_ci(cs.dim, seed)
        g = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
        G = torch.zeros((n, n, n, n), dtype=torch.complex128, device="cuda")
        P.op.ci_rdms(dev(C), g, G)
        gr, Gr = cs.rdms(C)
        assert np.max(np.abs(host(g) - gr)) < 1e-13
        assert np.max(np.abs(host(G) - Gr)) < 1e-13


@pytest.mark.parametrize("name", WIDE)
def test_rhs_apply_with_library_rdms(name):
    """G frozen from the library's own RDMs (mh_ci_rdms) against the oracle's
    frozen operator built from the oracle's RDMs of the same CI vector."""
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
    fr = Frozen(P.ops, c, gam, Gam, 0.021, W)
    g = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    G = torch.zeros((n, n, n, n), dtype=torch.complex128, device="cuda")
    P.op.ci_rdms(dev(C), g, G)
    P.op.freeze(dev(P.to_lib_orb(c)), g, G, 0.021, dev(P.W_to_lib(W, n)))
    for orb_sched in (1, 5):
        P.op.tune(0, orb_sched, 65536)
        v = orbitals(P, 7)
        out = torch.zeros((P.NE, n), dtype=torch.complex128, device="cuda")
        P.op.rhs_apply(dev(P.to_lib_orb(v)), out)
        ref = fr.G(v)
        got = P.from_lib_dof(host(out))
        assert rel_err_cols(got, ref) < 1e-10
        assert max_rel_cols(got, ref) < 1e-10
    P.op.tune(0, 1, 65536)


@pytest.mark.parametrize("name,steps", [("tiny_n8_2a2b", 3), ("small_n6", 3)])
def test_propagate_wide_ci(name, steps):
    """Orbitals and CI vector advanced together with the CI exponential
    truncated at 12 Lanczos vectors (Sec. II ci_eom): dipoles, energies,
    orbitals and the CI vector against the oracle."""
    torch = _torch()
    from oracle.ci import CISpace
    from oracle.mctdhf import Propagator
    P = pair(name, poisson_rtol=1e-13, poisson_maxit=20000)
    n = P.w["n_orb"]
    cs = CISpace(n, P.w["n_alpha"], P.w["n_beta"])
    c = orbitals(P, 10)
    C = random_ci(cs.dim, 11)
    dt = 0.02
    E_steps = [0.05 * np.sin(0.3 * k) for k in range(steps + 1)]
    x, Cd = dev(P.to_lib_orb(c)), dev(C)
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    rec = P.op.propagate(x, Cd, W, E_steps, dt, m=12)
    pr = Propagator(P.ops, cs, poisson_solver(P.ops))
    recs = []
    cc, CC = c.copy(), C.copy()
    for k in range(steps):
        cc, CC, ob = pr.step(cc, CC, E_steps[k], dt, 12)
        recs.append(ob)
    recs.append(pr.final_observables(cc, CC, E_steps[-1]))
    d_ref = np.array([r["dipole"] for r in recs])
    e_ref = np.array([r["energy"] for r in recs])
    print(name, "dipole diff", np.max(np.abs(rec["dipole"] - d_ref)), "energy diff",
          np.max(np.abs(rec["energy"] - e_ref)), flush=True)
    assert np.max(np.abs(rec["dipole"] - d_ref)) <= 1e-8 * max(np.abs(d_ref).max(), 1e-3)
    assert np.max(np.abs(rec["energy"] - e_ref)) <= 1e-8 * np.abs(e_ref).max()
    assert rel_err_cols(P.from_lib_dof(host(x)), cc) < 1e-8
    assert np.max(np.abs(host(Cd) - CC)) < 1e-8
