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


def full_mass(mesh):
    P = mesh.P
    _, w, _, _ = operators_1d(mesh.p)
    loc = local_index(P)
    wloc = w[loc[:, 0]] * w[loc[:, 1]] * w[loc[:, 2]]
    hc = mesh.cell_h()
    m = np.zeros(mesh.n_full)
    np.add.at(m, mesh.cell_nodes, (hc[:, None] / 2.0) ** 3 * wloc[None, :])
    return m


def full_stiffness(mesh):
    """K_full = sum over cells of (h/2)(A x W x W + W x A x W + W x W x A)."""
    P = mesh.P
    _, w, _, A = operators_1d(mesh.p)
    loc = local_index(P)
    rows, cols, vals = [], [], []
    for i, (a, b, c) in enumerate(loc):
        for a2 in range(P):
            j = a2 + P * (b + P * c)
            rows.append(i); cols.append(j); vals.append(A[a, a2] * w[b] * w[c])
        for b2 in range(P):
            j = a + P * (b2 + P * c)
            rows.append(i); cols.append(j); vals.append(w[a] * A[b, b2] * w[c])
        for c2 in range(P):
            j = a + P * (b + P * c2)
            rows.append(i); cols.append(j); vals.append(w[a] * w[b] * A[c, c2])
    rows, cols, vals = map(np.array, (rows, cols, vals))
    hc = mesh.cell_h()
    R = mesh.cell_nodes[:, rows].ravel()
    Cc = mesh.cell_nodes[:, cols].ravel()
    V = ((hc[:, None] / 2.0) * vals[None, :]).ravel()
    return sp.csr_matrix((V, (R, Cc)), shape=(mesh.n_full, mesh.n_full))


def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return (x + 1.0) / 2.0, w / 2.0          # on [0, 1]


def _regular_cells(mesh, Z, R, cells, q):
    """int_cell f_i(x) (-Z/|x-R|) dx by tensor Gauss-Legendre, q points/dim."""
    P = mesh.P
    g, gw = _gauss(q)
    Lg = lagrange_eval(mesh.xi, 2.0 * g - 1.0)           # [P, q]
    hc = mesh.cell_h()[cells]
    org = mesh.cell_origin()[cells]
    out = np.zeros((len(cells), P, P, P))
    for s in range(0, len(cells), 4096):
        hh = hc[s:s + 4096]
        oo = org[s:s + 4096]
        X = oo[:, 0, None] + hh[:, None] * g[None, :]
        Y = oo[:, 1, None] + hh[:, None] * g[None, :]
        Zc = oo[:, 2, None] + hh[:, None] * g[None, :]
        r = np.sqrt((X[:, :, None, None] - R[0]) ** 2 + (Y[:, None, :, None] - R[1]) ** 2
                    + (Zc[:, None, None, :] - R[2]) ** 2)
        f = -Z / r * (gw[:, None, None] * gw[None, :, None] * gw[None, None, :])
        t = np.einsum('aq,cqrs->cars', Lg, f)
        t = np.einsum('br,cars->cabs', Lg, t)
        t = np.einsum('cs,nabs->nabc', Lg, t)
        out[s:s + 4096] = t * (hh ** 3)[:, None, None, None]
    # local order: a (x) fastest -> index [c][b][a]
    return out.transpose(0, 3, 2, 1).reshape(len(cells), P ** 3)


def duffy_cell(mesh, Z, R, origin, h, n=DUFFY_POINTS):
    """int_cell f_i(x) (-Z/|x-R|) dx with R in the closed cell.

    The cube is split into six pyramids with apex R and a face as base;
    x = R + s (F(u,v) - R) gives dx = s^2 d h^2 ds du dv (d = apex height), so
    the 1/|x-R| singularity cancels.  Pyramids of zero height are skipped.
    """
    P = mesh.P
    g, gw = _gauss(n)
    out = np.zeros((P, P, P))
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
            out += np.einsum('asuv,bsuv,csuv,suv->abc', Lx, Ly, Lz, wt)
    return out.transpose(2, 1, 0).reshape(P ** 3)


def nuclear_lumped(mesh, nuclei):
    """v_i = sum_cells int_cell f_i V_nuc with V_nuc = -sum_a Z_a/|x - R_a|."""
    v = np.zeros(mesh.n_full)
    hc = mesh.cell_h()
    org = mesh.cell_origin()
    q = mesh.p + 5
    for (Z, R) in nuclei:
        R = np.asarray(R, dtype=float)
        tol = 1e-12 * hc
        inside = np.all((R[None, :] >= org - tol[:, None]) & (R[None, :] <= org + hc[:, None] + tol[:, None]), axis=1)
        reg = np.nonzero(~inside)[0]
        vals = _regular_cells(mesh, Z, R, reg, q)
        np.add.at(v, mesh.cell_nodes[reg], vals)
        for c in np.nonzero(inside)[0]:
            np.add.at(v, mesh.cell_nodes[c], duffy_cell(mesh, Z, R, org[c], hc[c]))
    return v


def full_gradient(mesh):
    """[D_x, D_y, D_z] on the full nodes: (D_d)_ij = sum over cells of the
    Gauss-Lobatto quadrature of f_i d f_j / d x_d, i.e. per cell
    (h/2)^2 w_a w_b w_c l'_{a'}(xi_a) for nodes i = (a,b,c), j = (a',b,c)
    (x direction; likewise along y and z)."""
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
        V = ((hc[:, None] / 2.0) ** 2 * vals[None, :]).ravel()
        out.append(sp.csr_matrix((V, (R, Cc)), shape=(mesh.n_full, mesh.n_full)))
    return out


class Operators:
    """Assembled sparse operators of one mesh and one molecule.  gauge:
    "length" (field value E(t), term E m (e.x)) or "velocity" (field value
    A(t), term -i A S_e)."""

    def __init__(self, mesh, nuclei, pol=(0.0, 0.0, 1.0), gauge="length"):
        if gauge not in ("length", "velocity"):
            raise ValueError(gauge)
        self.mesh = mesh
        self.gauge = gauge
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
        self._Mlu = None

    def gradient(self):
        """(D_full, D, S, S_e): the first-derivative matrices, built on first use."""
        if self._grad is None:
            C = self.mesh.C
            Dfull = full_gradient(self.mesh)
            D = [(C.T @ Dd @ C).tocsr() for Dd in Dfull]
            S = [(0.5 * (Dd - Dd.T)).tocsr() for Dd in D]
            Se = sum(e * Sd for e, Sd in zip(self.pol, S)).tocsr()
            self._grad = (Dfull, D, S, Se)
        return self._grad

    @property
    def Se(self):
        return self.gradient()[3]

    def H1(self, E):
        """One-body matrix at field value E: E(t) in the length gauge, A(t)
        in the velocity gauge."""
        if self.gauge == "velocity":
            return (0.5 * self.K + self.Vn - 1j * E * self.Se).tocsr()
        return (0.5 * self.K + self.Vn + E * self.Z).tocsr()

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
