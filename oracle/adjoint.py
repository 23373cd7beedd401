"""Reverse-mode reference for the gradient of the dipole record with respect
to the step fields (oracle).

A dense torch-CPU re-expression of the oracle's real-time propagation
(``mctdhf.Propagator.step``): per step, from the data at t_n (Sec. III.B,
first order),

    gamma, Gamma   = RDMs of the CI vector                 (Sec. II)
    W_rs           = T rho_rs, rho_rs = conj(phi_r) phi_s  (Sec. III.A Poisson
                     problem with its boundary integral, as one linear map)
    U, V, F, lam   as in ``mctdhf.Frozen``                 (Eq. orb_eom,
                                                            Eq. discretized_eom)
    c'             = short-iterative Arnoldi step of G     (Eq. packed_orb_eom:
                     the oracle's modified Gram-Schmidt with one
                     re-orthogonalisation, fixed dimension m, exp of the
                     Hessenberg matrix)
    C'             = exp(-i dt H_CI(h, g)) C               (Eq. ci_eom, X = 0;
                     the oracle's Lanczos with min(12, N_CI) vectors equals the
                     exact exponential up to rounding for N_CI <= 12)
    d_n            = sum_pq gamma_pq c_p^H Z c_q.

Every step is written with differentiable torch operations, so reverse-mode
automatic differentiation of J = sum_n w_n d_n gives dJ/dE_k.  The Poisson
map T is assembled densely from the oracle's own operators (K^-1 applied
to the load and boundary-lift columns), which limits this module to small
meshes.

Test infrastructure only (see ``oracle/__init__``).
"""
import itertools

import numpy as np
import scipy.sparse.linalg as spla
import torch

from .mctdhf import RDM_EPS
from .poisson import PoissonSolver

CT = torch.complex128


def _t(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype)


def poisson_matrix(ops, lmax=None):
    """Dense real T with W = T rho at the full nodes: the oracle's Poisson
    solve with multipole boundary values (``PoissonSolver.solve_density``)
    written as one matrix,

        T = C K^-1 (4 pi C^T diag(m) - C^T K_full CB I R^T diag(m)) + CB I R^T diag(m).
    """
    mesh = ops.mesh
    ps = PoissonSolver(ops) if lmax is None else PoissonSolver(ops, lmax)
    R, I = ps._tables()
    m = ops.m
    B = mesh.CB.toarray() @ (I @ (R.T * m[None, :]))                   # boundary lift per density column
    load = 4.0 * np.pi * (mesh.C.T.toarray() * m[None, :]) - mesh.C.T @ (ops.Kfull @ B)
    lu = spla.splu(ops.K.tocsc())
    w = lu.solve(np.asfortranarray(load))
    return mesh.C @ w + B


class DenseModel:
    """The oracle's operators of one mesh and CI space as dense torch tensors."""

    def __init__(self, ops, cispace):
        if getattr(ops, "ecs", None) is not None or ops.gauge != "length":
            raise ValueError("the dense model is the length-gauge operator without complex scaling")
        mesh = ops.mesh
        self.ops, self.ci = ops, cispace
        self.n = cispace.n
        self.M = _t(ops.M.toarray()).to(CT)
        self.Minv = torch.linalg.inv(self.M)
        self.H0 = _t((0.5 * ops.K + ops.Vn).toarray()).to(CT)
        self.Z = _t(ops.Z.toarray()).to(CT)
        self.C = _t(mesh.C.toarray()).to(CT)
        self.m = _t(ops.m)
        self.T = _t(poisson_matrix(ops)).to(CT)
        E = cispace.E_ops()
        n = self.n
        self.E = torch.stack([torch.stack([_t(E[p][q].toarray()) for q in range(n)]) for p in range(n)]).to(CT)
        # two-body operators E_pq E_rs - delta_qr E_ps
        E2 = torch.einsum('pqij,rsjk->pqrsik', self.E, self.E)
        for q in range(n):
            E2[:, q, q, :] = E2[:, q, q, :] - self.E
        self.E2 = E2
        self.vnn = ops.nuclear_repulsion()

    # ---- pieces of one step ------------------------------------------------
    def rdms(self, C):
        gamma = torch.einsum('i,pqij,j->pq', C.conj(), self.E, C)
        Gamma = torch.einsum('i,pqrsij,j->pqrs', C.conj(), self.E2, C)
        return gamma, Gamma

    def ginv(self, gamma):
        d, V = torch.linalg.eigh(0.5 * (gamma + gamma.conj().T))
        d = d + RDM_EPS * torch.exp(-d / RDM_EPS)
        return (V / d[None, :].to(CT)) @ V.conj().T

    def pair_potentials(self, phi):
        """Wf[r][s] at the full nodes for every ordered pair (W_sr = conj W_rs)."""
        n = self.n
        W = [[None] * n for _ in range(n)]
        for r in range(n):
            for s in range(r, n):
                W[r][s] = self.T @ (phi[:, r].conj() * phi[:, s])
                if s != r:
                    W[s][r] = W[r][s].conj()
        return W

    def frozen(self, c, gamma, Gamma, E, W):
        n = self.n
        U = torch.stack([torch.stack([sum(Gamma[o, q, r, s] * W[r][s] for r in range(n) for s in range(n))
                                      for q in range(n)], dim=-1) for o in range(n)], dim=-2)   # [NF, o, q]
        V = torch.einsum('po,xoq->xpq', self.ginv(gamma), U)
        H1 = self.H0 + E * self.Z

        def F(v):
            vf = self.C @ v
            mf = torch.einsum('xpq,xq->xp', V, vf) * self.m[:, None].to(CT)
            return H1 @ v + self.C.T @ mf

        lam = c.conj().T @ F(c)

        def G(v):
            return self.Minv @ F(v) - v @ lam
        return G, H1

    def inner(self, u, v):
        return torch.sum(u.conj() * (self.M @ v))

    def arnoldi(self, G, phi, tau, m, breakdown=1e-14):
        beta = torch.sqrt(self.inner(phi, phi).real)
        V = [phi / beta]
        Hcols = []
        m_eff = m
        for k in range(m):
            w = G(V[k])
            wn = torch.sqrt(self.inner(w, w).real)
            h = [torch.zeros((), dtype=CT) for _ in range(k + 1)]
            for _ in range(2):
                for j in range(k + 1):
                    hjk = self.inner(V[j], w)
                    h[j] = h[j] + hjk
                    w = w - hjk * V[j]
            hn = torch.sqrt(self.inner(w, w).real)
            Hcols.append((h, hn))
            if float(hn.detach()) <= breakdown * float(wn.detach()):
                m_eff = k + 1
                break
            V.append(w / hn)
        rows = []
        for k in range(m_eff):
            h, hn = Hcols[k]
            col = h + ([hn.to(CT)] if k + 1 < m_eff else [])
            col = col + [torch.zeros((), dtype=CT)] * (m_eff - len(col))
            rows.append(torch.stack(col))
        Hm = torch.stack(rows, dim=1)
        y = torch.linalg.matrix_exp(-1j * tau * Hm)[:, 0]
        return beta * sum(y[j] * V[j] for j in range(m_eff))

    def integrals(self, c, W, H1):
        n = self.n
        h = c.conj().T @ (H1 @ c)
        phi = self.C @ c
        g = torch.stack([torch.stack([torch.stack([torch.stack(
            [torch.sum(self.m * phi[:, p].conj() * phi[:, q] * W[r][s]) for s in range(n)])
            for r in range(n)]) for q in range(n)]) for p in range(n)])
        return h, g

    def hamiltonian(self, h, g):
        return torch.einsum('pq,pqij->ij', h, self.E) + 0.5 * torch.einsum('pqrs,pqrsij->ij', g, self.E2)

    def dipole(self, c, gamma):
        z = c.conj().T @ (self.Z @ c)
        return torch.sum(gamma * z).real

    def propagate(self, c, C, E_steps, dt, m=12):
        """Dipoles d_0 .. d_N for N = len(E_steps) - 1 steps (the last field
        value enters no dipole), as a differentiable function of E_steps."""
        ds = []
        N = len(E_steps) - 1
        for k in range(N + 1):
            gamma, Gamma = self.rdms(C)
            ds.append(self.dipole(c, gamma))
            if k == N:
                break
            phi = self.C @ c
            W = self.pair_potentials(phi)
            G, H1 = self.frozen(c, gamma, Gamma, E_steps[k], W)
            h, g = self.integrals(c, W, H1)
            c_next = self.arnoldi(G, c, dt, m)
            C = torch.linalg.matrix_exp(-1j * dt * self.hamiltonian(h, g)) @ C
            c = c_next
        return torch.stack(ds)


def dipole_gradient(ops, cispace, c0, C0, E_steps, dt, weights, m=12):
    """(d, dJ/dE) for J = sum_n weights_n d_n by reverse-mode autodiff of the
    dense re-expression; dJ/dE has len(E_steps) - 1 entries (E_N enters no
    dipole)."""
    model = DenseModel(ops, cispace)
    E = torch.tensor(np.asarray(E_steps, dtype=np.float64), requires_grad=True)
    d = model.propagate(_t(c0, CT), _t(C0, CT), E, dt, m)
    J = torch.sum(_t(weights) * d)
    J.backward()
    return d.detach().numpy(), E.grad.numpy()[:-1].copy()
