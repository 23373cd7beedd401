"""Pins of the oracle's Kelly indicator and Kelly refinement (Sec. III.A: cells
halved until Kelly's gradient-jump indicator of the nuclear potential meets a
threshold).

The pins fix the indicator by hand-derived values: a target the element space
reproduces has no gradient jumps at all; for x^2 on Q1 cells the interpolant's
slope on [a, a + h] is 2a + h, so every face jump, face integral and cell value
follows in closed form, on uniform meshes and across coarse-fine faces; faces
on the box boundary add nothing.  The refinement's own contract: no leaf left
above the threshold below the deepest level, 2:1 balance, and refinement only
adds to the ball mesh.
"""
import numpy as np
import pytest

from oracle.kelly import kelly_eta2, softened_coulomb
from oracle.mesh import balance_21, build_leaves, MeshDesc, Ball

LO, HI, NC = -2.0, 2.0, 4          # coarse cells of edge 1
UNIFORM = [(0, i, j, k) for i in range(NC) for j in range(NC) for k in range(NC)]
SQ3 = np.sqrt(3.0)


def x2(x, y, z):
    return x * x + 0.0 * y + 0.0 * z


def slope(a, h):
    """Slope of the Q1 interpolant of x^2 on [a, a + h]."""
    return 2.0 * a + h


@pytest.mark.parametrize("p", [1, 2, 3])
def test_reproduced_target_has_no_jumps(p):
    """A target in Q_p: the cell interpolants are the target itself, so no
    face carries a gradient jump, on a uniform mesh and across hanging faces."""
    f = lambda x, y, z: (x ** p + 0.5) * (y ** p - 0.25 * y) * (z - 0.3) ** p  # noqa: E731
    e = kelly_eta2(UNIFORM, LO, HI, NC, p, f)
    assert max(e.values()) < 1e-24
    L = set(UNIFORM) - {(0, 1, 1, 1)}
    L |= {(1, 2 + a, 2 + b, 2 + c) for a in (0, 1) for b in (0, 1) for c in (0, 1)}
    e = kelly_eta2(balance_21(L, NC), LO, HI, NC, p, f)
    assert max(e.values()) < 1e-22


def test_quadratic_on_uniform_q1_closed_form():
    """x^2 on unit Q1 cells: jump 2h = 2 on every x-face, none on y- and
    z-faces; an interior cell integrates 4 on each of its two x-faces, a cell
    on the box's x boundary only one of them."""
    e = kelly_eta2(UNIFORM, LO, HI, NC, 1, x2)
    h = 1.0
    for leaf, v in e.items():
        i = leaf[1]
        n_xfaces = (i > 0) + (i < NC - 1)
        want = SQ3 * h / 24.0 * n_xfaces * (2.0 * h) ** 2 * h * h
        assert abs(v - want) < 1e-13 * want, (leaf, v, want)


def test_quadratic_across_coarse_fine_faces_closed_form():
    """One unit cell split in eight: the coarse cell beside it meets four
    half-size faces, each with the jump between its slope and the fine
    cells' slope; a fine cell meets the coarse cell on one x-face and its
    sibling on the other."""
    L = set(UNIFORM) - {(0, 1, 1, 1)}
    L |= {(1, 2 + a, 2 + b, 2 + c) for a in (0, 1) for b in (0, 1) for c in (0, 1)}
    L = balance_21(L, NC)
    e = kelly_eta2(L, LO, HI, NC, 1, x2)
    # coarse cell x in [-2, -1] (box boundary on its left), fine cells x in [-1, -0.5]
    jump = slope(-2.0, 1.0) - slope(-1.0, 0.5)
    want = SQ3 * 1.0 / 24.0 * 4 * jump ** 2 * 0.25
    assert abs(e[(0, 0, 1, 1)] - want) < 1e-13 * want
    # coarse cell x in [0, 1] with the fine cells x in [-0.5, 0] on its left, a unit cell on its right
    jl = slope(0.0, 1.0) - slope(-0.5, 0.5)
    jr = slope(0.0, 1.0) - slope(1.0, 1.0)
    want = SQ3 * 1.0 / 24.0 * (4 * jl ** 2 * 0.25 + jr ** 2 * 1.0)
    assert abs(e[(0, 2, 1, 1)] - want) < 1e-13 * want
    # fine cell x in [-1, -0.5]: coarse neighbour left, fine sibling right
    j1 = slope(-1.0, 0.5) - slope(-2.0, 1.0)
    j2 = slope(-1.0, 0.5) - slope(-0.5, 0.5)
    want = SQ3 * 0.5 / 24.0 * (j1 ** 2 + j2 ** 2) * 0.25
    assert abs(e[(1, 2, 2, 2)] - want) < 1e-13 * want


def test_scaling_with_cell_size():
    """x^2 on Q1: the face jump is proportional to h, so an interior cell's
    eta^2 scales as h^5 when the whole mesh is refined once."""
    fine = [(1, i, j, k) for i in range(2 * NC) for j in range(2 * NC) for k in range(2 * NC)]
    e0 = kelly_eta2(UNIFORM, LO, HI, NC, 1, x2)[(0, 1, 1, 1)]
    e1 = kelly_eta2(fine, LO, HI, NC, 1, x2)[(1, 3, 3, 3)]
    assert abs(e1 / e0 - 2.0 ** -5) < 1e-12


NUC = [(1.0, (0.0, 0.0, 0.7)), (1.0, (0.0, 0.0, -0.7))]


def _ancestors(leaves):
    """Every leaf and every ancestor of a leaf."""
    return {(K[0] - s, K[1] >> s, K[2] >> s, K[3] >> s) for K in leaves for s in range(K[0] + 1)}


def _refined(p, tol, max_level, balls=()):
    desc = MeshDesc(-8.0, 8.0, 4, p, list(balls), kelly_nuclei=NUC, kelly_tol=tol, kelly_soft=0.1,
                    kelly_max_level=max_level)
    return desc, build_leaves(desc)


@pytest.mark.parametrize("p,tol", [(1, 0.01), (2, 0.005)])
def test_refinement_contract(p, tol):
    """After Kelly refinement every leaf below the deepest level meets the
    threshold, the tree is 2:1 balanced, and the mesh refines the ball mesh
    it started from."""
    balls = [Ball((0.0, 0.0, 0.0), 3.0, 1)]
    desc, leaves = _refined(p, tol, 3, balls)
    e = kelly_eta2(leaves, desc.lo, desc.hi, desc.n_coarse, p, softened_coulomb(NUC, 0.1))
    assert all(np.sqrt(v) <= tol for K, v in e.items() if K[0] < 3)
    assert sorted(balance_21(leaves, 4)) == sorted(leaves)
    assert max(K[0] for K in leaves) == 3
    base = build_leaves(MeshDesc(-8.0, 8.0, 4, p, balls))
    anc = _ancestors(leaves)
    assert all(K in anc for K in base)   # each ball leaf is a leaf or an ancestor of leaves


def test_refinement_is_symmetric():
    """The H2 target is symmetric under z -> -z and x <-> y, and so is the mesh."""
    desc, leaves = _refined(1, 0.01, 3)
    S = set(leaves)
    for (l, i, j, k) in leaves:
        n = 4 * 2 ** l
        assert (l, i, j, n - 1 - k) in S
        assert (l, j, i, k) in S

