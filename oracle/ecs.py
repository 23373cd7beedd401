"""Exterior complex scaling of the one-body operator (oracle).

Follows Sec. IV: outside an inner cuboid about the molecule the coordinates
are complex-scaled, which turns the box walls into an absorber; the paper
names the region and leaves the form to the literature.

Readings taken (the paper fixes none of them):
  * Cartesian scaling about the origin, one coordinate at a time: with the
    inner half-widths R_d and the angle theta,
        z_d(x) = x_d                                      for |x_d| <= R_d,
        z_d(x) = sign(x_d) R_d + e^{i theta} (x_d - sign(x_d) R_d)  beyond,
    so dz_d/dx_d = eta_d is 1 or e^{i theta}, constant in every cell (a cell
    may not straddle a plane x_d = +-R_d);
  * the one-body operator is continued along this contour: its Galerkin
    form on the bridged basis takes the contour's volume element
    J = eta_x eta_y eta_z, so per cell the mass carries J, the stiffness
    along d carries J / eta_d^2, the first derivative along d carries
    J / eta_d, the nuclear potential is V(z(x)) J (V continued with the
    principal square root) and the length-gauge field term E e.z(x) J;
  * the orbital equation's operator is M_theta^{-1} F_theta with
    M_theta = C^T diag(m_theta) C; the orbital inner product stays the
    Hermitian one of the real coordinates (M), so the projector, lam and
    h_pq are M inner products of M_theta^{-1} F_theta with the orbitals,
    and orthonormality is kept exactly while the CI norm carries the loss;
  * the pair potentials and the mean field stay on the real grid (the
    two-electron operator is not continued): the mean-field load is
    C^T[m_theta V C v], a pointwise product wherever J is uniform around a
    node;
  * the observables (dipole, momentum, orbital overlaps) use the real
    coordinates; the energy record is the real part of the complex
    expectation value.

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np


class ECS:
    """Scaling angle theta (radians, 0 <= theta < pi/2) and the inner
    half-widths (Rx, Ry, Rz) >= 0 of the unscaled cuboid about the origin."""

    def __init__(self, theta, inner):
        self.theta = float(theta)
        self.inner = np.asarray(inner, dtype=float).reshape(3)
        if not (0.0 <= self.theta < 0.5 * np.pi):
            raise ValueError("theta must lie in [0, pi/2)")
        if np.any(self.inner < 0.0):
            raise ValueError("inner half-widths must be >= 0")
        self.phase = np.exp(1j * self.theta)

    def contour(self, x, d):
        """z_d of real coordinates x (array) along direction d."""
        x = np.asarray(x, dtype=float)
        R = self.inner[d]
        s = np.sign(x)
        out = x.astype(complex)
        far = np.abs(x) > R
        out[far] = s[far] * R + self.phase * (x[far] - s[far] * R)
        return out

    def cell_eta(self, mesh, rtol=1e-12):
        """eta [n_cells, 3]: 1 or e^{i theta} per cell and direction."""
        h = mesh.cell_h()
        o = mesh.cell_origin()
        eta = np.ones((mesh.n_cells, 3), dtype=complex)
        for d in range(3):
            R = self.inner[d]
            lo, hi = o[:, d], o[:, d] + h
            tol = rtol * h
            out = (lo >= R - tol) | (hi <= -R + tol)
            ins = (lo >= -R - tol) & (hi <= R + tol)
            if np.any(~(out | ins)):
                raise ValueError("a cell straddles a scaling plane")
            eta[out, d] = self.phase
        return eta
