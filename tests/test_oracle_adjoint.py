"""Pins of the reverse-mode reference (oracle/adjoint.py): its forward pass
reproduces the oracle's own propagation (mctdhf.Propagator) dipole by
dipole, its Poisson matrix reproduces the oracle's Poisson solve, and its
gradient agrees with central differences of the propagation."""
import numpy as np
import pytest
import torch

from oracle.adjoint import DenseModel, dipole_gradient, poisson_matrix, _t, CT
from oracle.ci import CISpace
from oracle.mctdhf import Propagator, orthonormalize
from oracle.poisson import PoissonSolver
from synth import random_orbitals, random_ci
from tests.oracle_cases import case

DT = 0.05


def _start(name, seed):
    w, mesh, ops = case(name)
    cs = CISpace(w["n_orb"], w["n_alpha"], w["n_beta"])
    c = orthonormalize(ops, random_orbitals(mesh.xyz[mesh.dof_nodes], w["n_orb"], seed, spread=1.2))
    C = random_ci(cs.dim, seed + 1)
    return ops, cs, c, C


def test_poisson_matrix_is_the_oracle_solve():
    ops, cs, c, C = _start("tiny_q1", 2)
    T = poisson_matrix(ops)
    phi = ops.to_full(c)
    rho = np.conj(phi[:, 0]) * phi[:, 1]
    ref = PoissonSolver(ops).solve_density(rho)
    assert np.linalg.norm(T @ rho - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", ["tiny_q1", "small_n3"])
def test_forward_matches_oracle_propagation(name):
    ops, cs, c, C = _start(name, 4)
    E = 0.05 * np.sin(0.7 * np.arange(4)) + 0.01
    _, _, recs = Propagator(ops, cs).propagate(c, C, E[:-1], DT, 12)
    ref = np.array([r["dipole"] for r in recs])
    model = DenseModel(ops, cs)
    with torch.no_grad():
        d = model.propagate(_t(c, CT), _t(C, CT), torch.tensor(E), DT, 12).numpy()
    assert np.max(np.abs(d - ref)) <= 1e-10 * max(1.0, np.abs(ref).max()), (d, ref)


def test_gradient_matches_central_differences():
    ops, cs, c, C = _start("tiny_q1", 6)
    E = 0.04 * np.cos(0.5 * np.arange(5))
    rng = np.random.default_rng(3)
    wts = rng.standard_normal(len(E))
    d, g = dipole_gradient(ops, cs, c, C, E, DT, wts)
    model = DenseModel(ops, cs)

    def J(Ev):
        with torch.no_grad():
            return float(torch.sum(_t(wts) * model.propagate(_t(c, CT), _t(C, CT), torch.tensor(Ev), DT, 12)))
    for k in range(2):
        delta = rng.standard_normal(len(E))
        delta[-1] = 0.0
        delta /= np.linalg.norm(delta)
        eps = 1e-4
        fd = (J(E + eps * delta) - J(E - eps * delta)) / (2 * eps)
        ad = float(g @ delta[:-1])
        assert abs(fd - ad) <= 1e-7 * max(abs(fd), 1e-3 * np.linalg.norm(g)), (fd, ad)
