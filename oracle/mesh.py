"""Octree hexahedral mesh with hanging-node constraints (oracle).

Follows Sec. III.A: the box is first covered by uniform coarse cubes, which
are halved recursively where more resolution is needed; each cell carries
the tensor-product Lagrange basis on Gauss-Lobatto points, and continuity
across a refinement interface is restored by "bridged" basis functions.

Readings taken where the paper is silent:
  * refinement is geometric: a leaf of level l is split while it meets (its
    closest point lies strictly within radius r of) a ball whose level
    count exceeds l; then 2:1 balance is enforced over all 26 neighbours;
    a mesh may then be refined further by Kelly's indicator of the nuclear
    potential (``oracle/kelly.py`` states that criterion);
  * a full node is *hanging* iff the coarsest leaf whose closed box contains
    it does not have it as one of its own nodes; its value is that leaf's
    Lagrange interpolant at the node (the bridged function), with chains
    flattened so that masters are never hanging;
  * orbitals vanish on the box boundary (homogeneous Dirichlet), so DoFs are
    the full nodes that are neither hanging nor on the boundary.

Node identity is exact: per dimension a node coordinate is either a dyadic
rational of the coarse spacing (vertices, and the p=2 midpoints) or the
irrational Gauss-Lobatto offset of one specific cell, which no other cell
shares; both are encoded as integers.

Test infrastructure only (see ``oracle/__init__``).
"""
import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .gll import gll, lagrange_eval


@dataclass
class Ball:
    center: tuple
    radius: float
    levels: int


@dataclass
class MeshDesc:
    lo: float
    hi: float
    n_coarse: int
    p: int
    balls: list = field(default_factory=list)
    # Kelly refinement after the balls: nuclei [(Z, (x, y, z))], threshold,
    # softening length of the potential, deepest level (no nuclei: none)
    kelly_nuclei: list = field(default_factory=list)
    kelly_tol: float = 0.0
    kelly_soft: float = 0.0
    kelly_max_level: int = 0


def _cell_dist(lo, h, idx, c):
    """Distance from point c to the closed box [lo + h*idx, lo + h*(idx+1)]."""
    d2 = 0.0
    for t in range(3):
        a = lo + h * idx[t]
        b = a + h
        e = max(a - c[t], 0.0, c[t] - b)
        d2 += e * e
    return np.sqrt(d2)


def build_leaves(desc):
    """Ball refinement to a fixed point, then 26-neighbour 2:1 balance, then
    (when nuclei are given) Kelly refinement with re-balancing."""
    nc = desc.n_coarse
    H = (desc.hi - desc.lo) / nc
    leaves = {(0, i, j, k) for i in range(nc) for j in range(nc) for k in range(nc)}

    def children(l, i, j, k):
        return [(l + 1, 2 * i + a, 2 * j + b, 2 * k + c)
                for a in (0, 1) for b in (0, 1) for c in (0, 1)]

    changed = True
    while changed:
        changed = False
        nxt = set()
        for (l, i, j, k) in leaves:
            h = H / 2 ** l
            split = any(b.levels > l and _cell_dist(desc.lo, h, (i, j, k), b.center) < b.radius
                        for b in desc.balls)
            if split:
                nxt.update(children(l, i, j, k))
                changed = True
            else:
                nxt.add((l, i, j, k))
        leaves = nxt

    leaves = balance_21(leaves, nc)
    if desc.kelly_nuclei:
        from .kelly import kelly_refine, softened_coulomb
        f = softened_coulomb(desc.kelly_nuclei, desc.kelly_soft)
        leaves, _ = kelly_refine(leaves, desc.lo, desc.hi, nc, desc.p, f, desc.kelly_tol, desc.kelly_max_level,
                                 lambda L: balance_21(L, nc))
    return sorted(leaves)


def balance_21(leaves, nc):
    """Split leaves until no two leaves sharing a face, edge or corner differ
    by more than one level (all 26 neighbours)."""
    leaves = set(leaves)

    def children(l, i, j, k):
        return [(l + 1, 2 * i + a, 2 * j + b, 2 * k + c)
                for a in (0, 1) for b in (0, 1) for c in (0, 1)]

    def find_leaf(l, i, j, k):
        for L in range(l, -1, -1):
            s = l - L
            key = (L, i >> s, j >> s, k >> s)
            if key in leaves:
                return key
        return None

    offsets = [o for o in itertools.product((-1, 0, 1), repeat=3) if o != (0, 0, 0)]
    changed = True
    while changed:
        changed = False
        for (l, i, j, k) in sorted(leaves, reverse=True):
            if (l, i, j, k) not in leaves or l < 2:
                continue
            n_l = nc * 2 ** l
            for (di, dj, dk) in offsets:
                a, b, c = i + di, j + dj, k + dk
                if not (0 <= a < n_l and 0 <= b < n_l and 0 <= c < n_l):
                    continue
                nb = find_leaf(l, a, b, c)
                if nb is not None and nb[0] < l - 1:
                    leaves.discard(nb)
                    leaves.update(children(*nb))
                    changed = True
    return sorted(leaves)


class Mesh:
    """Leaves, full nodes, hanging constraints and DoF numbering."""

    def __init__(self, desc):
        self.desc = desc
        p = desc.p
        self.p = p
        P = p + 1
        self.P = P
        nc = desc.n_coarse
        self.H = (desc.hi - desc.lo) / nc
        cells = np.array(build_leaves(desc), dtype=np.int64)
        self.cells = cells
        self.n_cells = len(cells)
        Lmax = int(cells[:, 0].max())
        self.Lmax = Lmax
        self.level_counts = [int((cells[:, 0] == l).sum()) for l in range(Lmax + 1)]
        xi, w = gll(p)
        self.xi, self.w = xi, w
        s = (xi + 1.0) / 2.0                     # offsets in cell units
        # 2*s is an integer exactly for the dyadic offsets (ends, p=2 midpoint)
        dyadic = [a in (0, p) or (p == 2 and a == 1) for a in range(P)]
        two_s = [int(round(2 * s[a])) if dyadic[a] else -1 for a in range(P)]
        self._dyadic, self._two_s = dyadic, two_s
        self.NI = nc * 2 ** Lmax                 # finest cell count per dim
        self.top = nc * 2 ** (Lmax + 1)          # dyadic key of the upper box face

        lev = cells[:, 0]
        # per-dimension integer keys of every cell-local node coordinate
        keys = np.zeros((self.n_cells, 3, P), dtype=np.int64)
        for d in range(3):
            idx = cells[:, 1 + d]
            for a in range(P):
                if dyadic[a]:
                    keys[:, d, a] = (2 * idx + two_s[a]) << (Lmax - lev)
                else:
                    keys[:, d, a] = -(1 + ((lev * self.NI + idx) * P + a))
        self._cell_keys = keys
        off = 1 + (Lmax + 1) * self.NI * P
        S = 2 * off + 1
        self._key_off, self._key_S = off, S
        # local node index: a (x) fastest, then b (y), then c (z)
        loc = np.array([(a, b, c) for c in range(P) for b in range(P) for a in range(P)])
        full = ((keys[:, 0, loc[:, 0]] + off)
                + S * ((keys[:, 1, loc[:, 1]] + off) + S * (keys[:, 2, loc[:, 2]] + off)))
        uniq, inv = np.unique(full.ravel(), return_inverse=True)
        self.cell_nodes = inv.reshape(self.n_cells, P ** 3)
        self.n_full = len(uniq)
        kx = uniq % S - off
        ky = (uniq // S) % S - off
        kz = uniq // (S * S) - off
        self.node_keys = np.stack([kx, ky, kz], axis=1)
        self.xyz = np.stack([self._key_to_coord(self.node_keys[:, d]) for d in range(3)], axis=1)
        kk = self.node_keys
        self.is_bnd = np.any((kk == 0) | (kk == self.top), axis=1)
        self._classify_hanging()
        self._number_dofs()

    # -- exact coordinates ------------------------------------------------
    def _key_to_coord(self, k):
        t = np.zeros(len(k))
        dy = k >= 0
        t[dy] = k[dy] / 2.0 ** (self.Lmax + 1)
        code = -k[~dy] - 1
        a = code % self.P
        rest = code // self.P
        i = rest % self.NI
        l = rest // self.NI
        t[~dy] = (i + (self.xi[a] + 1.0) / 2.0) / 2.0 ** l
        return self.desc.lo + self.H * t

    def _key_t(self, k):
        """Position in coarse-cell units (exact for dyadic keys)."""
        return (self._key_to_coord(k) - self.desc.lo) / self.H

    def _candidates(self, k, L):
        """Level-L cell indices (per node, up to two) whose closed span holds key k."""
        n = len(k)
        c0 = np.full(n, -1, dtype=np.int64)
        c1 = np.full(n, -1, dtype=np.int64)
        dy = k >= 0
        sh = self.Lmax + 1 - L
        kd = k[dy]
        on = (kd & ((1 << sh) - 1)) == 0
        q = kd >> sh
        a0 = np.where(on, q - 1, q)
        a1 = np.where(on, q, -1)
        c0[dy], c1[dy] = a0, a1
        code = -k[~dy] - 1
        rest = code // self.P
        a = code % self.P
        i = rest % self.NI
        l = rest // self.NI
        fine = np.where(L <= l, i >> np.maximum(l - L, 0),
                        np.floor((i + (self.xi[a] + 1.0) / 2.0) * 2.0 ** (L - l)).astype(np.int64))
        c0[~dy] = fine
        nL = self.desc.n_coarse * 2 ** L
        c0[(c0 < 0) | (c0 >= nL)] = -1
        c1[(c1 < 0) | (c1 >= nL)] = -1
        return c0, c1

    def _classify_hanging(self):
        P, p = self.P, self.p
        leafcode = {tuple(c) for c in self.cells.tolist()}
        nF = self.n_full
        owner = np.full((nF, 4), -1, dtype=np.int64)       # coarsest containing leaf
        todo = np.arange(nF)
        for L in range(self.Lmax + 1):
            if len(todo) == 0:
                break
            cand = [self._candidates(self.node_keys[todo, d], L) for d in range(3)]
            found = np.zeros(len(todo), dtype=bool)
            for ci, cj, ck in itertools.product((0, 1), repeat=3):
                I, J, K = cand[0][ci], cand[1][cj], cand[2][ck]
                ok = (I >= 0) & (J >= 0) & (K >= 0) & ~found
                for t in np.nonzero(ok)[0]:
                    if (L, int(I[t]), int(J[t]), int(K[t])) in leafcode:
                        owner[todo[t]] = (L, I[t], J[t], K[t])
                        found[t] = True
            todo = todo[~found]
        assert len(todo) == 0, "node outside every leaf"
        self.node_owner = owner
        # is the node one of its coarsest leaf's own nodes?
        hang = np.zeros(nF, dtype=bool)
        match = np.full((nF, 3), -1, dtype=np.int64)
        for d in range(3):
            L = owner[:, 0]
            idx = owner[:, 1 + d]
            kd = self.node_keys[:, d]
            for a in range(P):
                if self._dyadic[a]:
                    lk = (2 * idx + self._two_s[a]) << (self.Lmax - L)
                else:
                    lk = -(1 + ((L * self.NI + idx) * P + a))
                match[kd == lk, d] = a
        hang = np.any(match < 0, axis=1)
        self.is_hang = hang
        # constraint rows: the coarsest leaf's interpolant evaluated at the node
        leaf_index = {tuple(c): n for n, c in enumerate(self.cells.tolist())}
        rows = {}
        for h in np.nonzero(hang)[0]:
            L, I, J, K = (int(v) for v in owner[h])
            cell = leaf_index[(L, I, J, K)]
            wd = []
            for d, idx in enumerate((I, J, K)):
                if match[h, d] >= 0:
                    e = np.zeros(P)
                    e[match[h, d]] = 1.0
                    wd.append(e)
                else:
                    t = self._key_t(self.node_keys[h:h + 1, d])[0]
                    xi_loc = 2.0 * (t * 2 ** L - idx) - 1.0
                    wd.append(lagrange_eval(self.xi, [xi_loc])[:, 0])
            row = {}
            for c in range(P):
                for b in range(P):
                    for a in range(P):
                        wv = wd[0][a] * wd[1][b] * wd[2][c]
                        if wv != 0.0:
                            nid = int(self.cell_nodes[cell, a + P * (b + P * c)])
                            row[nid] = row.get(nid, 0.0) + wv
            rows[int(h)] = row
        # flatten chains so that no master is itself hanging
        self.n_chain_subst = 0
        for _ in range(64):
            again = False
            for h, row in rows.items():
                if any(hang[m] for m in row):
                    new = {}
                    for m, wv in row.items():
                        if hang[m]:
                            for m2, w2 in rows[m].items():
                                new[m2] = new.get(m2, 0.0) + wv * w2
                            self.n_chain_subst += 1
                        else:
                            new[m] = new.get(m, 0.0) + wv
                    rows[h] = new
                    again = True
            if not again:
                break
        else:
            raise RuntimeError("constraint chains do not terminate")
        self.hang_rows = rows

    def _number_dofs(self):
        nF = self.n_full
        is_dof = ~self.is_hang & ~self.is_bnd
        self.dof_nodes = np.nonzero(is_dof)[0]
        self.n_dof = len(self.dof_nodes)
        self.dof_of = np.full(nF, -1, dtype=np.int64)
        self.dof_of[self.dof_nodes] = np.arange(self.n_dof)
        self.bnd_nodes = np.nonzero(self.is_bnd & ~self.is_hang)[0]
        self.bnd_of = np.full(nF, -1, dtype=np.int64)
        self.bnd_of[self.bnd_nodes] = np.arange(len(self.bnd_nodes))
        self.hang_nodes = np.nonzero(self.is_hang)[0]
        # C: full-node values from DoF values;  CB: from boundary values
        r, c, v, rb, cb, vb = [], [], [], [], [], []
        for k, n in enumerate(self.dof_nodes):
            r.append(n); c.append(k); v.append(1.0)
        for k, n in enumerate(self.bnd_nodes):
            rb.append(n); cb.append(k); vb.append(1.0)
        masters = set()
        self.hang_on_bnd = 0
        for h, row in self.hang_rows.items():
            if self.is_bnd[h]:
                self.hang_on_bnd += 1
            for m, wv in row.items():
                if self.dof_of[m] >= 0:
                    r.append(h); c.append(self.dof_of[m]); v.append(wv)
                    masters.add(int(self.dof_of[m]))
                else:
                    rb.append(h); cb.append(self.bnd_of[m]); vb.append(wv)
        self.C = sp.csr_matrix((v, (r, c)), shape=(nF, self.n_dof))
        self.CB = sp.csr_matrix((vb, (rb, cb)), shape=(nF, len(self.bnd_nodes)))
        self.masters = np.array(sorted(masters), dtype=np.int64)
        self.C_nnz_hang = sum(len(r) for r in self.hang_rows.values())

    def info(self):
        return dict(n_cells=self.n_cells, n_full=self.n_full, n_hang=int(self.is_hang.sum()),
                    n_bnd=int(self.is_bnd.sum()), n_dof=self.n_dof, n_masters=len(self.masters),
                    level_counts=self.level_counts, hang_nnz=self.C_nnz_hang,
                    chain_subst=self.n_chain_subst)

    def cell_h(self):
        return self.H / 2.0 ** self.cells[:, 0]

    def cell_origin(self):
        return self.desc.lo + self.cell_h()[:, None] * self.cells[:, 1:4]
