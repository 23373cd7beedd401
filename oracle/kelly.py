"""Kelly's error indicator and the mesh refinement it drives (oracle).

Follows Sec. III.A: starting from uniform coarse cubes, cells are halved
until the error in every cell, estimated by Kelly's indicator from the jump
of a target function's gradient across the cell faces, is below a
threshold; the concluding section names the target: the Coulomb potential
of the nuclei.

Readings taken where the paper is silent:
  * the target is the softened potential V(r) = -sum_A Z_A / sqrt(|r - R_A|^2
    + a^2) with a stated length a > 0, so that nodal values stay finite where
    a node sits on a nucleus;
  * u_K is V interpolated at the Gauss-Lobatto nodes of cell K alone (no
    hanging-node constraint), with the degree p of the mesh;
  * eta_K^2 = (h_K / 24) * sum over the faces of K not on the box boundary of
    the integral over the face of (du_K/dn - du_N/dn)^2, N the neighbour leaf
    across each part of the face and h_K = sqrt(3) * edge the cell's
    diameter.  The integral runs over the smaller of the two faces (a face
    of a coarser neighbour is split into the four faces of its finer
    neighbours) with the (p+1)-point Gauss-Legendre rule per direction,
    exact for the integrand, a polynomial of degree 2p per direction;
  * every leaf with eta_K > tol whose level is below max_level is halved,
    the tree re-balanced 2:1 over all 26 neighbours, and the indicators
    recomputed, until no leaf is marked.

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np

from .gll import gll, lagrange_eval, lagrange_deriv


def softened_coulomb(nuclei, a):
    """f(x, y, z) = -sum Z / sqrt(|r - R|^2 + a^2) on arrays of coordinates."""
    def f(x, y, z):
        v = np.zeros(np.broadcast(x, y, z).shape)
        for Z, R in nuclei:
            v -= Z / np.sqrt((x - R[0]) ** 2 + (y - R[1]) ** 2 + (z - R[2]) ** 2 + a * a)
        return v
    return f


class _Leaves:
    """Leaf lookup of an octree given as a set of (level, i, j, k)."""

    def __init__(self, leaves, nc):
        self.set = set(leaves)
        self.nc = nc

    def holder(self, l, i, j, k):
        """The leaf of level <= l containing cell (l, i, j, k), or None."""
        for L in range(l, -1, -1):
            s = l - L
            key = (L, i >> s, j >> s, k >> s)
            if key in self.set:
                return key
        return None


def kelly_eta2(leaves, lo, hi, nc, p, f):
    """eta_K^2 of every leaf (dict leaf -> value) for the target f."""
    H = (hi - lo) / nc
    xi, _ = gll(p)
    gq, gw = np.polynomial.legendre.leggauss(p + 1)
    T = _Leaves(leaves, nc)
    cache = {}

    def geom(leaf):
        l, i, j, k = leaf
        h = H / 2 ** l
        return h, lo + h * np.array([i, j, k], dtype=float)

    def nodal(leaf):
        if leaf not in cache:
            h, o = geom(leaf)
            X = o[:, None] + h * (xi[None, :] + 1.0) / 2.0      # [3][P]
            cache[leaf] = f(X[0][:, None, None], X[1][None, :, None], X[2][None, None, :])  # U[a, b, c]
        return cache[leaf]

    def dgrad(leaf, d, pts):
        """d u_leaf / d x_d at physical points pts [m][3]."""
        h, o = geom(leaf)
        t = 2.0 * (pts - o[None, :]) / h - 1.0
        B = [lagrange_deriv(xi, t[:, e]) * (2.0 / h) if e == d else lagrange_eval(xi, t[:, e]) for e in range(3)]
        return np.einsum("abc,am,bm,cm->m", nodal(leaf), B[0], B[1], B[2])

    def face_points(d, xd, t0, t1, side):
        """Gauss points and weights on the square x_d = xd, tangential lower corner (t0, t1), edge `side`."""
        e1, e2 = [e for e in range(3) if e != d]
        u = t0 + side * (gq + 1.0) / 2.0
        v = t1 + side * (gq + 1.0) / 2.0
        U, Vv = np.meshgrid(u, v, indexing="ij")
        pts = np.zeros((U.size, 3))
        pts[:, d] = xd
        pts[:, e1] = U.ravel()
        pts[:, e2] = Vv.ravel()
        w = np.outer(gw, gw).ravel() * (side / 2.0) ** 2
        return pts, w

    eta2 = {}
    for leaf in leaves:
        l, i, j, k = leaf
        h, o = geom(leaf)
        idx = [i, j, k]
        n_l = nc * 2 ** l
        acc = 0.0
        for d in range(3):
            e1, e2 = [e for e in range(3) if e != d]
            for s in (-1, 1):
                nb = list(idx)
                nb[d] += s
                if nb[d] < 0 or nb[d] >= n_l:
                    continue                                  # box boundary: no contribution
                xd = o[d] + (h if s > 0 else 0.0)
                N = T.holder(l, *nb)
                if N is not None:                             # same level or coarser: K's whole face
                    parts = [(N, o[e1], o[e2], h)]
                else:                                         # four finer leaves across the face
                    parts = []
                    for a in (0, 1):
                        for b in (0, 1):
                            c = [0, 0, 0]
                            c[d] = 2 * nb[d] + (0 if s > 0 else 1)
                            c[e1] = 2 * idx[e1] + a
                            c[e2] = 2 * idx[e2] + b
                            child = (l + 1, c[0], c[1], c[2])
                            if child not in T.set:
                                raise ValueError("tree not 2:1 balanced across a face")
                            parts.append((child, o[e1] + a * h / 2, o[e2] + b * h / 2, h / 2))
                for (N, t0, t1, side) in parts:
                    pts, w = face_points(d, xd, t0, t1, side)
                    jump = dgrad(leaf, d, pts) - dgrad(N, d, pts)
                    acc += float(np.sum(w * jump * jump))
        eta2[leaf] = np.sqrt(3.0) * h / 24.0 * acc
    return eta2


def kelly_refine(leaves, lo, hi, nc, p, f, tol, max_level, balance):
    """Halve every leaf with eta > tol below max_level, re-balance with
    `balance` (a function of a leaf set), and repeat until none is marked.
    Returns (leaves, rounds)."""
    leaves = set(leaves)
    rounds = 0
    while True:
        eta2 = kelly_eta2(leaves, lo, hi, nc, p, f)
        marked = [K for K in leaves if K[0] < max_level and eta2[K] > tol * tol]
        if not marked:
            return sorted(leaves), rounds
        for (l, i, j, k) in marked:
            leaves.discard((l, i, j, k))
            leaves.update((l + 1, 2 * i + a, 2 * j + b, 2 * k + c) for a in (0, 1) for b in (0, 1) for c in (0, 1))
        leaves = set(balance(leaves))
        rounds += 1
