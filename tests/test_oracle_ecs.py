"""Pins of the oracle's exterior complex scaling (Sec. IV: complex-scaled
coordinates outside an inner cuboid absorb what leaves the molecule).

What fixes the scaled operator here, other than the oracle itself:
  * angle zero is the unscaled operator;
  * scaling everything about the origin (no inner region) is uniform complex
    dilation x -> e^{i theta} x, under which the kinetic energy, a Coulomb
    potential centred at the origin, the length-gauge field and the first
    derivative acquire the exact factors e^{-2 i theta}, e^{-i theta},
    e^{i theta} and e^{-i theta};
  * on uniform Q1 cells with lumped mass the 1D Dirichlet spectrum is
    (4/h^2) sin^2(k pi / 2n), so scaling whole directions rotates exactly
    their share of every eigenvalue;
  * exterior scaling of a Cartesian product mesh separates: the 3D spectrum
    is the sum of 1D spectra of the textbook one-dimensional contour form
    (element mass times eta, element stiffness over eta), written out here
    independently, and that 1D form absorbs an outgoing wave packet without
    reflection while the unscaled one reflects it;
  * the scaled matrices are complex symmetric;
  * the continued Coulomb potential of a scaled cell equals a brute-force
    quadrature of its definition, with the contour written out here;
  * one electron in one orbital under complex scaling follows the dense
    exponential of the scaled one-body operator exactly, its orbital
    keeping unit norm while the CI coefficient carries the loss.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle.ecs import ECS
from oracle.fem import Operators, _regular_cells
from oracle.gll import operators_1d, lagrange_eval
from oracle.mesh import Ball, Mesh, MeshDesc
from oracle.ci import CISpace
from oracle import mctdhf
from synth import random_orbitals

TH = 0.35


def _dense_op(ops, A):
    """M_theta^{-1} A (dense)."""
    return np.linalg.solve(ops.M_theta.toarray(), A.toarray())


def _dense_plain(ops, A):
    return np.linalg.solve(ops.M.toarray(), A.toarray())


def test_zero_angle_is_unscaled():
    mesh = Mesh(MeshDesc(-6.0, 6.0, 3, 2, [Ball((0.2, -0.1, 0.3), 1.0, 1)]))
    nuc = [(1.0, (0.1, 0.2, -0.3))]
    for gauge in ("length", "velocity"):
        a = Operators(mesh, nuc, pol=(0.6, 0.0, 0.8), gauge=gauge)
        b = Operators(mesh, nuc, pol=(0.6, 0.0, 0.8), gauge=gauge, ecs=ECS(0.0, (2.0, 2.0, 2.0)))
        assert abs(b.M_theta - a.M).max() == 0.0
        d = abs(b.H1(0.07) - a.H1(0.07)).max()
        assert d < 1e-15 * abs(a.H1(0.07)).max()


def test_uniform_dilation_factors():
    """No inner region: z = e^{i theta} x everywhere (hanging nodes and a
    nucleus on a mesh node included)."""
    mesh = Mesh(MeshDesc(-4.0, 4.0, 4, 2, [Ball((0.0, 0.0, 0.0), 1.0, 1)]))
    assert mesh.info()["n_hang"] > 0
    nuc = [(1.0, (0.0, 0.0, 0.0))]
    pol = (0.0, 0.6, 0.8)
    a = Operators(mesh, nuc, pol=pol)
    b = Operators(mesh, nuc, pol=pol, ecs=ECS(TH, (0.0, 0.0, 0.0)))
    ph = np.exp(1j * TH)
    for At, Ap, f in ((b.K_theta, a.K, ph ** -2), (b.Vn_theta, a.Vn, ph ** -1), (b.Z_theta, a.Z, ph),
                      (b.Se_theta, a.Se, ph ** -1)):
        x, y = _dense_op(b, At), _dense_plain(a, Ap)
        assert np.abs(x - f * y).max() < 1e-12 * np.abs(y).max()


def _q1_lambda(n, h):
    k = np.arange(1, n)
    return (4.0 / h ** 2) * np.sin(k * np.pi / (2 * n)) ** 2


@pytest.mark.parametrize("scaled", [(1, 0, 0), (1, 1, 0), (0, 1, 1)])
def test_q1_whole_direction_scaling_closed_form(scaled):
    n, L = 6, 3.0
    h = 2 * L / n
    mesh = Mesh(MeshDesc(-L, L, n, 1, []))
    inner = [0.0 if s else L for s in scaled]
    ops = Operators(mesh, [], ecs=ECS(TH, inner))
    ev = np.linalg.eigvals(_dense_op(ops, 0.5 * ops.K_theta))
    lam = _q1_lambda(n, h)
    f = [np.exp(-2j * TH) if s else 1.0 for s in scaled]
    want = np.array([0.5 * (f[0] * a + f[1] * b + f[2] * c) for a in lam for b in lam for c in lam])
    d = np.abs(ev[:, None] - want[None, :])
    assert d.min(axis=1).max() < 1e-11 and d.min(axis=0).max() < 1e-11


def _contour_1d(p, edges, R, theta):
    """1D Gauss-Lobatto FEM on the given cell edges with contour scaling
    beyond |x| = R: element mass (h/2) w eta, stiffness (2/h) A / eta.
    Returns (mass diagonal, stiffness) on the interior nodes and their x."""
    xi, w, _, A = operators_1d(p)
    ncell = len(edges) - 1
    nn = ncell * p + 1
    m = np.zeros(nn, dtype=complex)
    K = np.zeros((nn, nn), dtype=complex)
    x = np.zeros(nn)
    for e in range(ncell):
        a, b = edges[e], edges[e + 1]
        h = b - a
        eta = np.exp(1j * theta) if (a >= R - 1e-12 or b <= -R + 1e-12) else 1.0
        idx = np.arange(e * p, e * p + p + 1)
        m[idx] += 0.5 * h * w * eta
        K[np.ix_(idx, idx)] += (2.0 / h) * A / eta
        x[idx] = a + 0.5 * h * (xi + 1.0)
    return m[1:-1], K[1:-1, 1:-1], x[1:-1]


@pytest.mark.parametrize("inner", [(2.0, 4.0, 4.0), (2.0, 2.0, 4.0)])
def test_exterior_scaling_separates_into_1d_contour_forms(inner):
    p, n, L = 2, 4, 4.0
    mesh = Mesh(MeshDesc(-L, L, n, p, []))
    ops = Operators(mesh, [], ecs=ECS(TH, inner))
    ev = np.linalg.eigvals(_dense_op(ops, 0.5 * ops.K_theta))
    edges = np.linspace(-L, L, n + 1)
    lams = []
    for d in range(3):
        m1, K1, _ = _contour_1d(p, edges, inner[d], TH)
        lams.append(np.linalg.eigvals(np.diag(1.0 / m1) @ K1))
    want = np.array([0.5 * (a + b + c) for a in lams[0] for b in lams[1] for c in lams[2]])
    d = np.abs(ev[:, None] - want[None, :])
    assert d.min(axis=1).max() < 1e-10 * np.abs(want).max()
    assert d.min(axis=0).max() < 1e-10 * np.abs(want).max()


@pytest.mark.parametrize("p", [1, 2])
def test_1d_contour_form_absorbs_an_outgoing_packet(p):
    """A packet leaving the inner region at speed 2 leaves less than 1e-3 of
    its norm behind with the contour, and is reflected back without it."""
    L, R = 40.0, 20.0
    edges = np.linspace(-L, L, int(2 * L / (0.1 * p)) + 1)
    left = {}
    for theta in (TH, 0.0):
        m, K, x = _contour_1d(p, edges, R, theta)
        _, _, xr = _contour_1d(p, edges, R, 0.0)
        mr, _, _ = _contour_1d(p, edges, R, 0.0)
        psi0 = np.exp(-x ** 2 / 8.0 + 2j * x)
        dt = 0.02
        H = 0.5 * K
        A = np.diag(m) + 0.5j * dt * H
        B = np.diag(m) - 0.5j * dt * H
        lu = sla.lu_factor(A)
        psi = psi0.copy()
        for _ in range(int(30.0 / dt)):
            psi = sla.lu_solve(lu, B @ psi)
        inner = np.abs(xr) < R
        left[theta] = np.sum(mr.real[inner] * np.abs(psi[inner]) ** 2) / np.sum(mr.real * np.abs(psi0) ** 2)
    assert left[TH] < 1e-3, left
    assert left[0.0] > 0.2, left


def test_scaled_matrices_are_complex_symmetric():
    mesh = Mesh(MeshDesc(-6.0, 6.0, 3, 2, [Ball((0.2, -0.1, 0.3), 1.0, 1)]))
    nuc = [(1.0, (0.1, 0.2, -0.3))]
    ops = Operators(mesh, nuc, pol=(0.6, 0.0, 0.8), gauge="velocity", ecs=ECS(TH, (2.0, 2.0, 2.0)))
    for A in (ops.K_theta, ops.M_theta, ops.Vn_theta, ops.Z_theta):
        assert abs(A - A.T).max() < 1e-15 * abs(A).max()
        assert abs(A - A.conj().T).max() > 1e-3 * abs(A).max()     # not Hermitian
    S = ops.Se_theta
    assert abs(S + S.T).max() < 1e-15 * abs(S).max()


def test_continued_potential_brute_force():
    """Scaled cells (x only; x and y) against a 24-point product rule of
    -Z J / sqrt(sum_d (z_d - R_d)^2) f_i with z written out here."""
    p = 2
    mesh = Mesh(MeshDesc(-6.0, 6.0, 3, p, []))
    Rn = np.array([0.3, -0.2, 0.1])
    inner = (2.0, 2.0, 6.0)
    ecs = ECS(TH, inner)
    eta = ecs.cell_eta(mesh)
    J = np.prod(eta, axis=1)
    org, hc = mesh.cell_origin(), mesh.cell_h()
    picks = [c for c in range(mesh.n_cells) if abs(eta[c, 0] - 1) > 0 and abs(eta[c, 1] - 1) == 0][:2] + \
            [c for c in range(mesh.n_cells) if abs(eta[c, 0] - 1) > 0 and abs(eta[c, 1] - 1) > 0][:2]
    assert len(picks) == 4
    got = _regular_cells(mesh, 1.0, Rn, np.array(picks), 16, ecs, J)   # the oracle's rule, 16 points
    g, gw = np.polynomial.legendre.leggauss(24)
    ph = np.exp(1j * TH)

    def z(xv, R):
        out = xv.astype(complex)
        far = np.abs(xv) > R
        out[far] = np.sign(xv[far]) * R + ph * (xv[far] - np.sign(xv[far]) * R)
        return out

    for k, c in enumerate(picks):
        h, o = hc[c], org[c]
        t = (g + 1.0) / 2.0
        X = [o[d] + h * t for d in range(3)]
        Zs = [z(X[d], inner[d]) - Rn[d] for d in range(3)]
        r = np.sqrt(Zs[0][:, None, None] ** 2 + Zs[1][None, :, None] ** 2 + Zs[2][None, None, :] ** 2)
        f = -J[c] / r * (gw[:, None, None] * gw[None, :, None] * gw[None, None, :]) * (h / 2) ** 3
        Lg = lagrange_eval(mesh.xi, g)                  # [P, 24]
        ref = np.einsum("aq,br,cs,qrs->cba", Lg, Lg, Lg, f).reshape(-1)
        assert np.abs(got[k] - ref).max() < 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("gauge", ["length", "velocity"])
def test_one_electron_under_scaling_is_the_scaled_tdse(gauge):
    mesh = Mesh(MeshDesc(-6.0, 6.0, 3, 2, [Ball((0.2, -0.1, 0.3), 1.0, 1)]))
    ops = Operators(mesh, [(1.0, (0.0, 0.0, 0.0))], pol=(0.6, 0.0, 0.8), gauge=gauge,
                    ecs=ECS(TH, (2.0, 2.0, 2.0)))
    cs = CISpace(1, 1, 0)
    c = mctdhf.orthonormalize(ops, random_orbitals(mesh.xyz[mesh.dof_nodes], 1, 9, spread=3.0))
    C = np.ones(1, dtype=complex)
    pr = mctdhf.Propagator(ops, cs)
    psi = c[:, 0].copy()
    Mt = ops.M_theta.toarray()
    dt = 0.05
    for E in (0.0, 0.3, -0.2, 0.5):
        c, C, _ = pr.step(c, C, E, dt, m=16)
        psi = sla.expm(-1j * dt * np.linalg.solve(Mt, ops.H1(E).toarray())) @ psi
        tot = C[0] * c[:, 0]
        assert np.sqrt(mctdhf.inner(ops, tot - psi, tot - psi).real) < 1e-10
        assert abs(np.sqrt(mctdhf.inner(ops, c, c).real) - 1.0) < 1e-3 * dt
    assert abs(C[0]) < 0.999          # the scaled region has absorbed part of the norm


def test_scaling_rejects_straddling_cells_and_bad_angles():
    mesh = Mesh(MeshDesc(-6.0, 6.0, 3, 1, []))
    with pytest.raises(ValueError):
        ECS(TH, (1.0, 2.0, 2.0)).cell_eta(mesh)
    with pytest.raises(ValueError):
        ECS(1.6, (2.0, 2.0, 2.0))
    with pytest.raises(ValueError):
        ECS(TH, (-1.0, 2.0, 2.0))


def test_projector_coefficients_are_the_generalised_fock_matrix():
    """With complex scaling (interface nodes in unscaled cells), the frozen
    lam equals h + gamma^{-1}-weighted two-electron integrals:
    lam_qp = h_qp + sum (gamma^{-1})_po Gamma_oq',rs g_qq'rs, which ties the
    scaled one-body form, its mass and the mean-field weights to the
    integrals of the energy."""
    from oracle.poisson import PoissonSolver
    from synth import random_ci
    mesh = Mesh(MeshDesc(-12.0, 12.0, 6, 2, [Ball((0.3, -0.2, 0.4), 1.0, 1)]))
    ops = Operators(mesh, [(1.0, (0.0, 0.0, 0.7)), (1.0, (0.0, 0.0, -0.7))], pol=(1.0, 0.0, 0.0),
                    ecs=ECS(TH, (8.0, 8.0, 8.0)))
    n = 2
    cs = CISpace(n, 1, 1)
    c = mctdhf.orthonormalize(ops, random_orbitals(mesh.xyz[mesh.dof_nodes], n, 3, spread=5.0))
    C = random_ci(cs.dim, 4)
    pr = mctdhf.Propagator(ops, cs, PoissonSolver(ops))
    E = 0.05
    fr = pr.freeze(c, C, E)
    h, g = mctdhf.integrals(ops, c, fr.Wfull, E)
    gi = mctdhf.gamma_reg_inv(fr.gamma)
    want = h + np.einsum("po,oars,qars->qp", gi, fr.Gamma, g)
    assert np.abs(fr.lam - want).max() < 1e-10 * np.abs(want).max()
