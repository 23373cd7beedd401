"""Helpers that pair a library mesh/operator with the oracle on the same
workload: node matching by coordinates and layout conversion.  Only
index bookkeeping lives here, no arithmetic of the method."""
import functools

import numpy as np

from tests.oracle_cases import case


def match_nodes(lib_xyz, or_xyz, tol=1e-9):
    """perm[i] = oracle full-node index of library full node i."""
    key = lambda x: tuple(np.round(np.asarray(x) / tol).astype(np.int64))  # noqa: E731
    table = {key(x): j for j, x in enumerate(or_xyz)}
    perm = np.array([table[key(x)] for x in lib_xyz], dtype=np.int64)
    assert len(set(perm.tolist())) == len(perm)
    return perm


class Pair:
    """Library mesh + operator and the oracle on one workload."""

    def __init__(self, name, seed=0, with_op=True, **op_kw):
        import paper_2301_02387_amd as mh
        self.w, self.om, self.ops = case(name, seed)
        self.mesh = mh.Mesh.from_workload(self.w)
        self.perm = match_nodes(self.mesh.coords(), self.om.xyz)
        info = self.mesh.info
        self.N, self.Nh, self.NF = info["n_dof"], info["n_hang"], info["n_full"]
        self.NE = self.N + self.Nh
        self.dof_or = self.om.dof_of[self.perm[:self.N]]        # oracle DoF of each library DoF
        assert np.all(self.dof_or >= 0)
        self.op = None
        if with_op:
            w = self.w
            op_kw.setdefault("polarization", w.get("polarization", (0.0, 0.0, 1.0)))
            self.op = mh.Operator(self.mesh, w["nuclei"], w["n_orb"], w["n_alpha"], w["n_beta"], **op_kw)

    # ---- layout conversion -------------------------------------------------
    def to_lib_orb(self, c_or):
        """Oracle DoF coefficients [N_or][n] -> library extended array [NE][n]."""
        full = self.om.C @ c_or
        return full[self.perm[:self.NE]]

    def from_lib_dof(self, x_lib):
        """Library DoF rows [N][n] -> oracle DoF order."""
        out = np.zeros((self.om.n_dof,) + x_lib.shape[1:], dtype=x_lib.dtype)
        out[self.dof_or] = x_lib[:self.N]
        return out

    def lib_full_to_oracle(self, a_lib):
        out = np.zeros((self.om.n_full,) + a_lib.shape[1:], dtype=a_lib.dtype)
        out[self.perm] = a_lib
        return out

    def W_to_lib(self, W, n):
        """Oracle pair potentials {(r,s): full-node array} -> [NF][n*n] real columns."""
        cols = []
        for r in range(n):
            for s in range(r, n):
                cols.append(W[(r, s)].real)
                if s != r:
                    cols.append(W[(r, s)].imag)
        A = np.stack(cols, axis=1)
        return np.ascontiguousarray(A[self.perm])

    def W_from_lib(self, Wl, n):
        A = self.lib_full_to_oracle(Wl)
        W, c = {}, 0
        for r in range(n):
            for s in range(r, n):
                if s == r:
                    W[(r, s)] = A[:, c].astype(complex)
                    c += 1
                else:
                    W[(r, s)] = A[:, c] + 1j * A[:, c + 1]
                    c += 2
        return W


def rel_err_cols(a, b):
    """max over columns of |a - b|_2 / |b|_2."""
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return max(np.linalg.norm(a[:, j] - b[:, j]) / max(np.linalg.norm(b[:, j]), 1e-300) for j in range(b.shape[1]))


def max_rel_cols(a, b):
    """max over columns of max_i |a_ij - b_ij| / max_i |b_ij|: an element-wise
    check beside the column 2-norms, so that a few wrong rows (hanging,
    master or boundary-lift rows) of a large mesh cannot hide in a norm."""
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return max(np.abs(a[:, j] - b[:, j]).max() / max(np.abs(b[:, j]).max(), 1e-300) for j in range(b.shape[1]))


_SOLVERS = {}


def poisson_solver(ops):
    """The oracle's Poisson solver of one operator set, factorised once and
    shared by the tests (the sparse LU of the H2 mesh takes tens of seconds)."""
    from oracle.poisson import PoissonSolver
    key = id(ops)
    if key not in _SOLVERS:
        _SOLVERS[key] = (ops, PoissonSolver(ops))
    return _SOLVERS[key][1]
