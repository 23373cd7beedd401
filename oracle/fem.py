"""Discrete operators on the octree mesh (oracle).

Follows Sec. III.A: every integral uses the Gauss-Lobatto rule on each
cell's own nodes, so the full-node mass is diagonal, m_i = sum over cells
holding node i of (h/2)^3 w_a w_b w_c; the Galerkin one-body matrix
(H1)_{kl} = int b_k H1 b_l of Eq. discretized_eom is assembled through the
constraint matrix C (bridged basis b_k = sum_i C_ik f_i):

    M  = C^T diag(m) C                      (mass / overlap matrix)
    K  = C^T K_full C,  K_full = sum_cells (h/2)(A x W x W + W x A x W + W x W x A)
    H1(E) = K/2 + C^T diag(v + E m (e.x)) C (length gauge)
    H1(A) = K/2 + C^T diag(v) C - i A S_e   (velocity gauge, Sec. II: the
                                             one-body operator carries -i A(t).grad)

The first-derivative matrix of the velocity gauge is the Gauss-Lobatto
Galerkin form D_d = C^T D_full,d C with (D_full,d)_ij = sum_cells int f_i
d/dx_d f_j; by collocation (D_full,d u)_i = m_i (d u/d x_d)(x_i) for every u
of the element space whose derivative is continuous.  S_d = (D_d - D_d^T)/2
is its antisymmetric part (reading: the paper does not say how the term is
discretised; the antisymmetric part keeps H1 Hermitian, and it equals D_d
itself where no hanging nodes interrupt the face integrals, by summation by
parts of the Gauss-Lobatto rule), and S_e = sum_d e_d S_d along the field
direction e.  The A^2/2 term of the minimal coupling is dropped: it is a
constant in space and only adds a phase and N A^2/2 to the energy.

With exterior complex scaling (``ecs``: theta and the inner cuboid) every
cell integral above takes the contour's factors: the mass J, the stiffness
along d J / eta_d^2, the derivative along d J / eta_d, the potential
V(z(x)) J and the field e.z(x) J; ``ecs`` states the readings.

v is the lumped nuclear potential: v_i = sum_cells int_cell f_i V_nuc, the
row sum of the exact Galerkin potential matrix.  With a nucleus on a mesh
node, the Gauss-Lobatto value m_i V(x_i) is infinite; the lumped integral is
finite and equals m_i V(x_i) to quadrature accuracy for smooth V.  Cells
whose closure holds a nucleus use a six-pyramid Duffy rule with the apex on
the nucleus; every other cell uses tensor Gauss-Legendre with p+5 points
per direction.

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np
import scipy.sparse as sp

from .gll import operators_1d, lagrange_eval

DUFFY_POINTS = 16          # Gauss-Legendre points per pyramid direction


def local_index(P):
    return np.array([(a, b, c) for c in range(P) for b in range(P) for a in range(P)])


def full_mass(mesh, J=None):
    """m_i = sum over cells holding node i of J (h/2)^3 w_a w_b w_c (J = 1
    without complex scaling, else the cell's volume factor [n_cells])."""
    P = mesh.P
    _, w, _, _ = operators_1d(mesh.p)
    loc = local_index(P)
    wloc = w[loc[:, 0]] * w[loc[:, 1]] * w[loc[:, 2]]
    hc = mesh.cell_h()
    cw = (hc[:, None] / 2.0) ** 3 * wloc[None, :]
    if J is None:
        m = np.zeros(mesh.n_full)
    else:
        m = np.zeros(mesh.n_full, dtype=complex)
        cw = cw * J[:, None]
    np.add.at(m, mesh.cell_nodes, cw)
    return m


def full_stiffness(mesh, fac=None):
    """K_full = sum over cells of (h/2)(A x W x W + W x A x W + W x W x A);
    fac [n_cells, 3] (complex scaling) multiplies each cell's part along x,
    y and z."""
    P = mesh.P
    _, w, _, A = operators_1d(mesh.p)
    loc = local_index(P)
    rows, cols, vals, dirs = [], [], [], []
    for i, (a, b, c) in enumerate(loc):
        for a2 in range(P):
            j = a2 + P * (b + P * c)
            rows.append(i); cols.append(j); vals.append(A[a, a2] * w[b] * w[c]); dirs.append(0)
        for b2 in range(P):
            j = a + P * (b2 + P * c)
            rows.append(i); cols.append(j); vals.append(w[a] * A[b, b2] * w[c]); dirs.append(1)
        for c2 in range(P):
            j = a + P * (b + P * c2)
            rows.append(i); cols.append(j); vals.append(w[a] * w[b] * A[c, c2]); dirs.append(2)
    rows, cols, vals, dirs = map(np.array, (rows, cols, vals, dirs))
    hc = mesh.cell_h()
    R = mesh.cell_nodes[:, rows].ravel()
    Cc = mesh.cell_nodes[:, cols].ravel()
    V = (hc[:, None] / 2.0) * vals[None, :]
    if fac is not None:
        V = V * fac[:, dirs]
    return sp.csr_matrix((V.ravel(), (R, Cc)), shape=(mesh.n_full, mesh.n_full))


def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return (x + 1.0) / 2.0, w / 2.0          # on [0, 1]


def _regular_cells(mesh, Z, R, cells, q, ecs=None, J=None):
    """int_cell f_i(x) (-Z/|x-R|) dx by tensor Gauss-Legendre, q points/dim;
    with complex scaling, int_cell f_i(x) (-Z/r(z(x))) J dx, r the principal
    square root of sum_d (z_d - R_d)^2."""
    P = mesh.P
    g, gw = _gauss(q)
    Lg = lagrange_eval(mesh.xi, 2.0 * g - 1.0)           # [P, q]
    hc = mesh.cell_h()[cells]
    org = mesh.cell_origin()[cells]
    out = np.zeros((len(cells), P, P, P), dtype=float if ecs is None else complex)
    for s in range(0, len(cells), 4096):
        hh = hc[s:s + 4096]
        oo = org[s:s + 4096]
        X = oo[:, 0, None] + hh[:, None] * g[None, :]
        Y = oo[:, 1, None] + hh[:, None] * g[None, :]
        Zc = oo[:, 2, None] + hh[:, None] * g[None, :]
        if ecs is not None:
            X, Y, Zc = ecs.contour(X, 0), ecs.contour(Y, 1), ecs.contour(Zc, 2)
        r = np.sqrt((X[:, :, None, None] - R[0]) ** 2 + (Y[:, None, :, None] - R[1]) ** 2
                    + (Zc[:, None, None, :] - R[2]) ** 2)
        f = -Z / r * (gw[:, None, None] * gw[None, :, None] * gw[None, None, :])
        if ecs is not None:
            f = f * J[cells[s:s + 4096], None, None, None]
        t = np.einsum('aq,cqrs->cars', Lg, f)
        t = np.einsum('br,cars->cabs', Lg, t)
        t = np.einsum('cs,nabs->nabc', Lg, t)
        out[s:s + 4096] = t * (hh ** 3)[:, None, None, None]
    # local order: a (x) fastest -> index [c][b][a]
    return out.transpose(0, 3, 2, 1).reshape(len(cells), P ** 3)


def duffy_cell(mesh, Z, R, origin, h, n=DUFFY_POINTS, ecs=None, J=1.0):
    """int_cell f_i(x) (-Z/|x-R|) dx with R in the closed cell.

    The cube is split into six pyramids with apex R and a face as base;
    x = R + s (F(u,v) - R) gives dx = s^2 d h^2 ds du dv (d = apex height), so
    the 1/|x-R| singularity cancels.  Pyramids of zero height are skipped.
    With complex scaling the integrand is -Z J / r(z(x)): the real rule's
    weights times J |x - R| / r(z(x)).
    """
    P = mesh.P
    g, gw = _gauss(n)
    out = np.zeros((P, P, P), dtype=float if ecs is None else complex)
    for d in range(3):
        d1, d2 = [e for e in range(3) if e != d]
        for side in (0, 1):
            plane = origin[d] + side * h
            height = abs(R[d] - plane)
            if height <= 1e-14 * h:
                continue
            U, Vv = np.meshgrid(g, g, indexing='ij')
            F = np.zeros((n, n, 3))
            F[..., d] = plane
            F[..., d1] = origin[d1] + h * U
            F[..., d2] = origin[d2] + h * Vv
            dist = np.linalg.norm(F - np.asarray(R)[None, None, :], axis=-1)   # [u, v]
            X = np.asarray(R)[None, None, None, :] + g[:, None, None, None] * (F[None] - np.asarray(R))
            xi = 2.0 * (X - np.asarray(origin)) / h - 1.0                       # [s,u,v,3]
            Lx = lagrange_eval(mesh.xi, xi[..., 0].ravel()).reshape(P, n, n, n)
            Ly = lagrange_eval(mesh.xi, xi[..., 1].ravel()).reshape(P, n, n, n)
            Lz = lagrange_eval(mesh.xi, xi[..., 2].ravel()).reshape(P, n, n, n)
            wt = (gw[:, None, None] * gw[None, :, None] * gw[None, None, :]
                  * g[:, None, None] * height * h * h * (-Z) / dist[None, :, :])
            if ecs is not None:
                rz = np.sqrt(sum((ecs.contour(X[..., k], k) - R[k]) ** 2 for k in range(3)))
                wt = wt * J * np.linalg.norm(X - np.asarray(R), axis=-1) / rz
            out += np.einsum('asuv,bsuv,csuv,suv->abc', Lx, Ly, Lz, wt)
    return out.transpose(2, 1, 0).reshape(P ** 3)


def nuclear_lumped(mesh, nuclei, ecs=None):
    """v_i = sum_cells int_cell f_i V_nuc with V_nuc = -sum_a Z_a/|x - R_a|
    (with complex scaling: V_nuc(z(x)) J)."""
    J = None if ecs is None else np.prod(ecs.cell_eta(mesh), axis=1)
    v = np.zeros(mesh.n_full, dtype=float if ecs is None else complex)
    hc = mesh.cell_h()
    org = mesh.cell_origin()
    q = mesh.p + 5
    for (Z, R) in nuclei:
        R = np.asarray(R, dtype=float)
        tol = 1e-12 * hc
        inside = np.all((R[None, :] >= org - tol[:, None]) & (R[None, :] <= org + hc[:, None] + tol[:, None]), axis=1)
        reg = np.nonzero(~inside)[0]
        vals = _regular_cells(mesh, Z, R, reg, q, ecs, J)
        np.add.at(v, mesh.cell_nodes[reg], vals)
        for c in np.nonzero(inside)[0]:
            if ecs is None:
                np.add.at(v, mesh.cell_nodes[c], duffy_cell(mesh, Z, R, org[c], hc[c]))
            else:
                np.add.at(v, mesh.cell_nodes[c], duffy_cell(mesh, Z, R, org[c], hc[c], ecs=ecs, J=J[c]))
    return v


def full_gradient(mesh, fac=None):
    """[D_x, D_y, D_z] on the full nodes: (D_d)_ij = sum over cells of the
    Gauss-Lobatto quadrature of f_i d f_j / d x_d, i.e. per cell
    (h/2)^2 w_a w_b w_c l'_{a'}(xi_a) for nodes i = (a,b,c), j = (a',b,c)
    (x direction; likewise along y and z); fac [n_cells, 3] (complex
    scaling) multiplies each cell's part along d."""
    P = mesh.P
    _, w, D, _ = operators_1d(mesh.p)
    loc = local_index(P)
    hc = mesh.cell_h()
    out = []
    for d in range(3):
        rows, cols, vals = [], [], []
        for i, abc in enumerate(loc):
            for a2 in range(P):
                jabc = list(abc)
                jabc[d] = a2
                j = jabc[0] + P * (jabc[1] + P * jabc[2])
                rows.append(i); cols.append(j)
                vals.append(w[abc[0]] * w[abc[1]] * w[abc[2]] * D[abc[d], a2])
        rows, cols, vals = map(np.array, (rows, cols, vals))
        R = mesh.cell_nodes[:, rows].ravel()
        Cc = mesh.cell_nodes[:, cols].ravel()
        V = (hc[:, None] / 2.0) ** 2 * vals[None, :]
        if fac is not None:
            V = V * fac[:, d, None]
        out.append(sp.csr_matrix((V.ravel(), (R, Cc)), shape=(mesh.n_full, mesh.n_full)))
    return out


class Operators:
    """Assembled sparse operators of one mesh and one molecule.  gauge:
    "length" (field value E(t), term E m (e.x)) or "velocity" (field value
    A(t), term -i A S_e).  ecs: an ``ecs.ECS`` (complex scaling of the
    one-body operator) or None."""

    def __init__(self, mesh, nuclei, pol=(0.0, 0.0, 1.0), gauge="length", ecs=None):
        if gauge not in ("length", "velocity"):
            raise ValueError(gauge)
        self.mesh = mesh
        self.gauge = gauge
        self.ecs = ecs
        self.nuclei = [(float(Z), tuple(map(float, R))) for Z, R in nuclei]
        self.pol = np.asarray(pol, dtype=float)
        C = mesh.C
        self.m = full_mass(mesh)
        self.Kfull = full_stiffness(mesh)
        self.v = nuclear_lumped(mesh, self.nuclei)
        self.mz = self.m * (mesh.xyz @ self.pol)
        self.M = (C.T @ sp.diags(self.m) @ C).tocsc()
        self.K = (C.T @ self.Kfull @ C).tocsr()
        self.Vn = (C.T @ sp.diags(self.v) @ C).tocsr()
        self.Z = (C.T @ sp.diags(self.mz) @ C).tocsr()
        self._grad = None
        self._grad_theta = None
        self._Mlu = None
        self._Mtlu = None
        if ecs is not None:
            # the one-body operator on the scaled contour
            self.eta = ecs.cell_eta(mesh)
            self.J = np.prod(self.eta, axis=1)
            self.m_theta = full_mass(mesh, self.J)
            self.K_theta = (C.T @ full_stiffness(mesh, self.J[:, None] / self.eta ** 2) @ C).tocsr()
            self.v_theta = nuclear_lumped(mesh, self.nuclei, ecs)
            ez = sum(self.pol[d] * ecs.contour(mesh.xyz[:, d], d) for d in range(3))
            self.M_theta = (C.T @ sp.diags(self.m_theta) @ C).tocsc()
            self.Vn_theta = (C.T @ sp.diags(self.v_theta) @ C).tocsr()
            self.Z_theta = (C.T @ sp.diags(self.m_theta * ez) @ C).tocsr()
        else:
            self.m_theta = self.m

    def gradient(self):
        """(D_full, D, S, S_e): the first-derivative matrices, built on first use."""
        if self._grad is None:
            self._grad = self._derivatives(None)
        return self._grad

    def _derivatives(self, fac):
        C = self.mesh.C
        Dfull = full_gradient(self.mesh, fac)
        D = [(C.T @ Dd @ C).tocsr() for Dd in Dfull]
        S = [(0.5 * (Dd - Dd.T)).tocsr() for Dd in D]
        Se = sum(e * Sd for e, Sd in zip(self.pol, S)).tocsr()
        return (Dfull, D, S, Se)

    @property
    def Se(self):
        return self.gradient()[3]

    @property
    def Se_theta(self):
        """S_e on the scaled contour (per cell J / eta_d along d)."""
        if self.ecs is None:
            return self.Se
        if self._grad_theta is None:
            self._grad_theta = self._derivatives(self.J[:, None] / self.eta)
        return self._grad_theta[3]

    def H1(self, E):
        """One-body matrix at field value E: E(t) in the length gauge, A(t)
        in the velocity gauge (with complex scaling, its form on the scaled
        contour, to be inverted by M_theta)."""
        if self.ecs is not None:
            if self.gauge == "velocity":
                return (0.5 * self.K_theta + self.Vn_theta - 1j * E * self.Se_theta).tocsr()
            return (0.5 * self.K_theta + self.Vn_theta + E * self.Z_theta).tocsr()
        if self.gauge == "velocity":
            return (0.5 * self.K + self.Vn - 1j * E * self.Se).tocsr()
        return (0.5 * self.K + self.Vn + E * self.Z).tocsr()

    def theta_solve(self, f):
        """M_theta^{-1} f (the mass of the one-body operator's own form:
        M itself without complex scaling)."""
        if self.ecs is None:
            return self.mass_solve(f)
        if self._Mtlu is None:
            import scipy.sparse.linalg as spla
            self._Mtlu = spla.splu(self.M_theta)
        return self._Mtlu.solve(np.asarray(f, dtype=complex))

    def hermitian_load(self, f):
        """The load vector whose M^{-1} is M_theta^{-1} f: M M_theta^{-1} f
        (f itself without complex scaling), so that c^H of it is the M inner
        product of c with M_theta^{-1} f."""
        if self.ecs is None:
            return f
        return self.M @ self.theta_solve(f)

    def momentum(self):
        """Matrix of e.p = -i e.grad in the bridged basis (-i S_e)."""
        return (-1j * self.Se).tocsr()

    def mass_solve(self, f):
        """c = M^{-1} f by sparse LU (exact up to rounding)."""
        if self._Mlu is None:
            import scipy.sparse.linalg as spla
            self._Mlu = spla.splu(self.M)
        f = np.asarray(f)
        if np.iscomplexobj(f):
            return self._Mlu.solve(np.ascontiguousarray(f.real)) + 1j * self._Mlu.solve(np.ascontiguousarray(f.imag))
        return self._Mlu.solve(f)

    def to_full(self, c):
        """Full-node values C c (zero on the box boundary)."""
        return self.mesh.C @ c

    def nuclear_repulsion(self):
        e = 0.0
        nuc = self.nuclei
        for a in range(len(nuc)):
            for b in range(a + 1, len(nuc)):
                e += nuc[a][0] * nuc[b][0] / np.linalg.norm(np.subtract(nuc[a][1], nuc[b][1]))
        return e
