"""CI space, reduced density matrices and the CI Hamiltonian (oracle).

Follows Sec. II: the MCTDHF wave function is the full set of Slater
determinants over n spatial orbitals (a complete active space), with
spin-summed excitation operators E_pq = sum_sigma a+_{p sigma} a_{q sigma}.

Conventions (the paper's D and P are index permutations of these):
  gamma_pq       = <E_pq>
  Gamma_pq,rs    = <E_pq E_rs> - delta_qr <E_ps>
  H              = sum h_pq E_pq + 1/2 sum g_pqrs (E_pq E_rs - delta_qr E_ps)
  g_pqrs         = int conj(phi_p) phi_q W_rs  (chemists' order)
The paper's one-body matrix D^p_q equals gamma_qp and its two-body matrix
P^{pq}_{sr} equals Gamma_{sp,rq}.

A determinant is (alpha string, beta string); strings are bit masks of
occupied orbitals, ordered by integer value; the determinant index is
i_alpha * n_beta_strings + i_beta, and creation operators are ordered
alpha before beta, orbitals ascending.

Test infrastructure only (see ``oracle/__init__``).
"""
import itertools

import numpy as np
import scipy.sparse as sp


def strings(n, k):
    return sorted(sum(1 << o for o in occ) for occ in itertools.combinations(range(n), k))


def excite(s, p, q):
    """a+_p a_q acting on string s: return (sign, new string) or (0, None)."""
    if not (s >> q) & 1:
        return 0, None
    sign = -1 if bin(s & ((1 << q) - 1)).count('1') % 2 else 1
    s2 = s & ~(1 << q)
    if (s2 >> p) & 1:
        return 0, None
    if bin(s2 & ((1 << p) - 1)).count('1') % 2:
        sign = -sign
    return sign, s2 | (1 << p)


class CISpace:
    def __init__(self, n, n_alpha, n_beta):
        self.n, self.na, self.nb = n, n_alpha, n_beta
        self.sa = strings(n, n_alpha)
        self.sb = strings(n, n_beta)
        self.ia = {s: i for i, s in enumerate(self.sa)}
        self.ib = {s: i for i, s in enumerate(self.sb)}
        self.dim = len(self.sa) * len(self.sb)
        self._E = None

    def E_ops(self):
        """Sparse E_pq matrices, E[p][q][J, I] = <J|E_pq|I>."""
        if self._E is not None:
            return self._E
        n, NB = self.n, len(self.sb)
        E = [[None] * n for _ in range(n)]
        for p in range(n):
            for q in range(n):
                rows, cols, vals = [], [], []
                for ia, a in enumerate(self.sa):
                    sg, a2 = excite(a, p, q)
                    if sg:
                        ja = self.ia[a2]
                        for ib in range(NB):
                            rows.append(ja * NB + ib); cols.append(ia * NB + ib); vals.append(sg)
                for ib, b in enumerate(self.sb):
                    sg, b2 = excite(b, p, q)
                    if sg:
                        jb = self.ib[b2]
                        for ia in range(len(self.sa)):
                            rows.append(ia * NB + jb); cols.append(ia * NB + ib); vals.append(sg)
                E[p][q] = sp.csr_matrix((np.array(vals, dtype=float), (rows, cols)),
                                        shape=(self.dim, self.dim))
        self._E = E
        return E

    def rdms(self, C):
        """gamma [n,n] and Gamma [n,n,n,n] of the normalised-or-not vector C."""
        n = self.n
        E = self.E_ops()
        D = [[E[r][s] @ C for s in range(n)] for r in range(n)]
        gamma = np.array([[np.vdot(C, D[p][q]) for q in range(n)] for p in range(n)])
        Gamma = np.zeros((n, n, n, n), dtype=complex)
        for p, q, r, s in itertools.product(range(n), repeat=4):
            Gamma[p, q, r, s] = np.vdot(D[q][p], D[r][s]) - (gamma[p, s] if q == r else 0.0)
        return gamma, Gamma

    def hamiltonian(self, h, g):
        """Dense H_CI from one-electron h_pq and two-electron g_pqrs."""
        n = self.n
        E = self.E_ops()
        H = sp.csr_matrix((self.dim, self.dim), dtype=complex)
        for p, q in itertools.product(range(n), repeat=2):
            H = H + h[p, q] * E[p][q]
        for p, q, r, s in itertools.product(range(n), repeat=4):
            if g[p, q, r, s] == 0:
                continue
            term = E[p][q] @ E[r][s]
            if q == r:
                term = term - E[p][s]
            H = H + 0.5 * g[p, q, r, s] * term
        return H.toarray()

    def sigma(self, h, g, C):
        return self.hamiltonian(h, g) @ C
