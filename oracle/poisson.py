"""Mean-field pair potentials by the Poisson equation (oracle).

Follows Sec. III.A (the Poisson equation that replaces Eq. mean-field, and
its Dirichlet condition): for each orbital pair r <= s,

    Laplace W_rs = -4 pi conj(phi_r) phi_s   in the box,
    W_rs = int conj(phi_r) phi_s / |x - x'|   on the box boundary.

Discretely, with rho at the full nodes and the Gauss-Lobatto mass m,

    K w = 4 pi C^T (m rho) - C^T K_full (CB W_B),   W = C w + CB W_B,

where CB injects boundary values (and their share in hanging-node rows).

The boundary integral is evaluated as the multipole expansion of its
Gauss-Lobatto quadrature about the box centre, truncated at l_max (a
reading: the paper does not say how the boundary integral is evaluated):

    W_B(x) = sum_{l<=lmax} 4pi/(2l+1) sum_m Q_lm S_lm(x^)/|x|^{l+1},
    Q_lm   = sum_i m_i rho_i |x_i|^l S_lm(x_i^)

with S_lm the orthonormal real spherical harmonics.  ``boundary_legendre``
evaluates the same truncated series through the Legendre addition theorem
as an independent check; ``boundary_direct`` is the untruncated quadrature.

The linear solve is exact up to rounding (sparse LU), since the solution of
the discrete Poisson problem has a plain definition.

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np
import scipy.sparse.linalg as spla
from scipy.special import sph_harm_y, eval_legendre

LMAX = 12


def real_sph(l, m, theta, phi):
    """Orthonormal real spherical harmonic S_lm (theta polar, phi azimuth)."""
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return np.sqrt(2.0) * (-1) ** m * np.real(y)
    return np.sqrt(2.0) * (-1) ** m * np.imag(y)


def _angles(x):
    r = np.linalg.norm(x, axis=1)
    safe = np.where(r > 0, r, 1.0)
    theta = np.arccos(np.clip(x[:, 2] / safe, -1.0, 1.0))
    phi = np.arctan2(x[:, 1], x[:, 0])
    return r, theta, phi


def multipole_moments(x, weights, lmax=LMAX):
    """Q[l][m+l] = sum_i weights_i |x_i|^l S_lm(x_i^)  (weights may be complex)."""
    r, th, ph = _angles(x)
    Q = []
    for l in range(lmax + 1):
        rl = r ** l
        Q.append(np.array([np.sum(weights * rl * real_sph(l, m, th, ph)) for m in range(-l, l + 1)]))
    return Q


def boundary_multipole(xb, Q, lmax=LMAX):
    r, th, ph = _angles(xb)
    out = np.zeros(len(xb), dtype=np.result_type(Q[0].dtype, float))
    for l in range(lmax + 1):
        pref = 4.0 * np.pi / (2 * l + 1) / r ** (l + 1)
        for m in range(-l, l + 1):
            out = out + pref * Q[l][m + l] * real_sph(l, m, th, ph)
    return out


def boundary_legendre(xb, x, weights, lmax=LMAX):
    """Same truncated series via 1/|x-y| = sum_l r_<^l / r_>^(l+1) P_l(cos g)."""
    rb = np.linalg.norm(xb, axis=1)
    r = np.linalg.norm(x, axis=1)
    out = np.zeros(len(xb), dtype=np.result_type(weights.dtype, float))
    for b in range(len(xb)):
        cosg = np.where(r > 0, (x @ xb[b]) / (np.where(r > 0, r, 1.0) * rb[b]), 1.0)
        s = 0.0
        for l in range(lmax + 1):
            s = s + (r ** l / rb[b] ** (l + 1)) * eval_legendre(l, cosg)
        out[b] = np.sum(weights * s)
    return out


def boundary_direct(xb, x, weights):
    """Untruncated quadrature sum_i weights_i / |x_b - x_i| (the node at x_b itself
    carries zero density, orbitals vanish on the boundary, and is skipped)."""
    out = np.zeros(len(xb), dtype=np.result_type(weights.dtype, float))
    for b in range(len(xb)):
        d = np.linalg.norm(x - xb[b], axis=1)
        keep = d > 0
        out[b] = np.sum(weights[keep] / d[keep])
    return out


class PoissonSolver:
    def __init__(self, ops, lmax=LMAX):
        self.ops = ops
        mesh = ops.mesh
        self.lmax = lmax
        self.center = np.full(3, 0.5 * (mesh.desc.lo + mesh.desc.hi))
        self.xb = mesh.xyz[mesh.bnd_nodes] - self.center
        self.xrel = mesh.xyz - self.center
        self._lu = None

    def factor(self):
        if self._lu is None:
            # symmetric minimum-degree ordering: same exact factorisation,
            # far less fill than the default column ordering on 3D meshes
            self._lu = spla.splu(self.ops.K.tocsc(), permc_spec="MMD_AT_PLUS_A",
                                 options=dict(SymmetricMode=True))
        return self._lu

    def _tables(self):
        """Regular solid harmonics at the full nodes, irregular ones (with the
        4pi/(2l+1) factor) at the boundary nodes; (lmax+1)^2 columns each."""
        if getattr(self, "_R", None) is None:
            r, th, ph = _angles(self.xrel)
            rb, thb, phb = _angles(self.xb)
            R, I = [], []
            for l in range(self.lmax + 1):
                for m in range(-l, l + 1):
                    R.append(r ** l * real_sph(l, m, th, ph))
                    I.append(4.0 * np.pi / (2 * l + 1) / rb ** (l + 1) * real_sph(l, m, thb, phb))
            self._R = np.stack(R, axis=1)
            self._I = np.stack(I, axis=1)
        return self._R, self._I

    def boundary_values(self, rho_full):
        R, I = self._tables()
        Q = (self.ops.m * rho_full) @ R
        return I @ Q

    def solve_density(self, rho_full, WB=None):
        """W at the full nodes for the density rho given at the full nodes."""
        ops, mesh = self.ops, self.ops.mesh
        if WB is None:
            WB = self.boundary_values(rho_full)
        gB = mesh.CB @ WB
        b = 4.0 * np.pi * (mesh.C.T @ (ops.m * rho_full)) - mesh.C.T @ (ops.Kfull @ gB)
        lu = self.factor()
        if np.iscomplexobj(b):
            w = lu.solve(np.ascontiguousarray(b.real)) + 1j * lu.solve(np.ascontiguousarray(b.imag))
        else:
            w = lu.solve(b)
        return mesh.C @ w + gB

    def pair_potentials(self, c):
        """W[(r, s)] for r <= s from orbital DoF coefficients c [N, n]."""
        phi = self.ops.to_full(c)
        n = c.shape[1]
        W = {}
        for r in range(n):
            for s in range(r, n):
                W[(r, s)] = self.solve_density(np.conj(phi[:, r]) * phi[:, s])
        return W


def full_pairs(W, n):
    """Dense W[r][s] over all pairs using W_sr = conj(W_rs)."""
    out = [[None] * n for _ in range(n)]
    for (r, s), w in W.items():
        out[r][s] = w
        out[s][r] = np.conj(w)
    return out
