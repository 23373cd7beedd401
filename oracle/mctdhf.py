"""Frozen orbital operator G, short-iterative Arnoldi, CI step, propagation.

Follows Sec. II (Eqs. ci_eom and orb_eom with X = 0), the discretised
orbital equation (Eq. discretized_eom) and Sec. III.B (Eq. packed_orb_eom and
the frozen-operator exponential phi(t+dt) = exp(-i G dt) phi(t)).

Discrete frozen operator at t_n (orbitals c, RDMs, field E and the pair
potentials W all taken at t_n):

    U_oq(x)  = sum_rs Gamma_oq,rs W_rs(x)
    V(x)     = gamma^{-1} U(x)           (gamma regularised, see below)
    F_p(v)   = H1(E) v_p + C^T[ m * sum_q V_pq (C v_q) ]      (load vector)
    lam_qp   = c_q^H F_p(c)
    (G v)_p  = M^{-1} F_p(v) - sum_q lam_qp v_q

With exterior complex scaling (``ecs``) the load vector is the one-body
operator's contour form, M becomes M_theta in (G v)_p and in the mean-field
weights, and lam_qp = c_q^H M M_theta^{-1} F_p(c), the M inner product of
the unprojected right-hand side with the orbital (likewise h_pq).

The last line is the packed operator with its projector term read as a
frozen scalar lam_qp multiplying component q (at v = c it reproduces the
projector Q of Eq. orb_eom).  The mean-field index placement follows from
Eq. orb_eom with the paper's D and P written in terms of gamma and Gamma
(see ``ci``).  gamma is regularised in its eigenbasis as
d -> d + eps exp(-d/eps) with eps = 1e-10.

Arnoldi: inner product <U,V> = sum_p u_p^H M v_p over the packed vector;
modified Gram-Schmidt with one full re-orthogonalisation pass; happy
breakdown when h_{k+1,k} <= 1e-14 |G v_k|; phi' = beta V_m expm(-i tau H_m) e1
(tau = dt in real time, -i dtau in imaginary time); error estimate
beta h_{m+1,m} |e_m^T expm(-i tau H_m) e1|.  With an error threshold
(Sec. III.B: the dimension chosen adaptively against a threshold on the
error estimate) the space stops growing at the first dimension k whose
estimate beta h_{k+1,k} |e_k^T expm(-i tau H_k) e1| is at or below it, m
being then the largest dimension allowed.

CI: C' = expm(-i dt H_CI) C in the Krylov space of min(12, N_CI) vectors,
built with full re-orthogonalisation (the Arnoldi process, which for a
Hermitian H_CI is the Lanczos recursion and also serves the non-Hermitian
H_CI of complex scaling), from the same t_n integrals (orbitals and CI
advance together from t_n data).

Test infrastructure only (see ``oracle/__init__``).
"""
import itertools

import numpy as np
import scipy.linalg as sla

from .poisson import PoissonSolver, full_pairs

RDM_EPS = 1e-10


def gamma_reg_inv(gamma, eps=RDM_EPS):
    d, V = np.linalg.eigh(0.5 * (gamma + gamma.conj().T))
    d = d + eps * np.exp(-d / eps)
    return (V / d[None, :]) @ V.conj().T


def mean_field_U(Gamma, Wfull):
    """U[x, o, q] = sum_rs Gamma[o,q,r,s] W_rs(x) at the full nodes."""
    n = Gamma.shape[0]
    nF = len(Wfull[0][0])
    U = np.zeros((nF, n, n), dtype=complex)
    for o, q, r, s in itertools.product(range(n), repeat=4):
        if Gamma[o, q, r, s] != 0:
            U[:, o, q] += Gamma[o, q, r, s] * Wfull[r][s]
    return U


class Frozen:
    """G frozen at t_n."""

    def __init__(self, ops, c, gamma, Gamma, E, W):
        self.ops = ops
        self.c = c
        self.n = c.shape[1]
        self.E = E
        self.gamma, self.Gamma = gamma, Gamma
        self.Wfull = full_pairs(W, self.n)
        self.U = mean_field_U(Gamma, self.Wfull)
        self.ginv = gamma_reg_inv(gamma)
        self.V = np.einsum('po,xoq->xpq', self.ginv, self.U)
        self.H1 = ops.H1(E)
        self.lam = c.conj().T @ ops.hermitian_load(self.F(c))   # lam[q, p] = <c_q, M^-1 F_p(c)>_M

    def F(self, v):
        ops, C = self.ops, self.ops.mesh.C
        vf = C @ v
        mf = np.einsum('xpq,xq->xp', self.V, vf) * ops.m_theta[:, None]
        return self.H1 @ v + C.T @ mf

    def G(self, v):
        return self.ops.theta_solve(self.F(v)) - v @ self.lam


def inner(ops, u, v):
    return np.vdot(u, ops.M @ v)


def arnoldi_step(ops, Gop, phi, tau, m, breakdown=1e-14, tol=None):
    """One short-iterative Arnoldi step; returns (phi', err_estimate, m_used, H).
    tol: error threshold of the adaptive dimension (None: fixed dimension m)."""
    beta = np.sqrt(inner(ops, phi, phi).real)
    V = [phi / beta]
    Hm = np.zeros((m + 1, m), dtype=complex)
    m_eff = m
    for k in range(m):
        w = Gop(V[k])
        wn = np.sqrt(inner(ops, w, w).real)
        for _ in range(2):
            for j in range(k + 1):
                hjk = inner(ops, V[j], w)
                Hm[j, k] += hjk
                w = w - hjk * V[j]
        Hm[k + 1, k] = np.sqrt(inner(ops, w, w).real)
        if Hm[k + 1, k].real <= breakdown * wn:
            m_eff = k + 1
            break
        if tol is not None and k + 1 < m:
            yk = sla.expm(-1j * tau * Hm[:k + 1, :k + 1])[:, 0]
            if beta * abs(Hm[k + 1, k]) * abs(yk[k]) <= tol:
                m_eff = k + 1
                break
        V.append(w / Hm[k + 1, k])
    y = sla.expm(-1j * tau * Hm[:m_eff, :m_eff])[:, 0]
    out = beta * sum(y[j] * V[j] for j in range(m_eff))
    err = beta * abs(Hm[m_eff, m_eff - 1]) * abs(y[m_eff - 1])
    return out, err, m_eff, Hm[:m_eff + 1, :m_eff]


def lanczos_expm(H, C, tau, m=12):
    """expm(-i tau H) C in the Krylov space of m vectors, orthogonalised
    against all earlier ones twice (Lanczos for Hermitian H; the same
    Arnoldi process serves a non-Hermitian H)."""
    m = min(m, len(C))
    beta0 = np.linalg.norm(C)
    Q = [C / beta0]
    T = np.zeros((m, m), dtype=complex)
    m_eff = m
    for k in range(m):
        w = H @ Q[k]
        for j in range(k + 1):
            hjk = np.vdot(Q[j], w)
            T[j, k] += hjk
            w = w - hjk * Q[j]
        for j in range(k + 1):
            hjk = np.vdot(Q[j], w)
            T[j, k] += hjk
            w = w - hjk * Q[j]
        if k + 1 < m:
            b = np.linalg.norm(w)
            if b <= 1e-14 * max(1.0, abs(T[k, k])):
                m_eff = k + 1
                break
            T[k + 1, k] = b
            Q.append(w / b)
    y = sla.expm(-1j * tau * T[:m_eff, :m_eff])[:, 0]
    return beta0 * sum(y[j] * Q[j] for j in range(m_eff))


def integrals(ops, c, Wfull, E):
    """h_pq = <c_p, M^-1 H1(E) c_q>_M (= c_p^H H1(E) c_q without complex
    scaling) and g_pqrs = sum_F m conj(phi_p) phi_q W_rs."""
    n = c.shape[1]
    h = c.conj().T @ ops.hermitian_load(ops.H1(E) @ c)
    phi = ops.to_full(c)
    g = np.zeros((n, n, n, n), dtype=complex)
    for p, q in itertools.product(range(n), repeat=2):
        dens = ops.m * np.conj(phi[:, p]) * phi[:, q]
        for r, s in itertools.product(range(n), repeat=2):
            g[p, q, r, s] = np.sum(dens * Wfull[r][s])
    return h, g


def observables(ops, c, gamma, Gamma, h, g, E=0.0):
    """Dipole sum gamma_pq c_p^H Z c_q, energy, overlap, and the kinetic
    momentum along e: sum gamma_pq c_p^H (-i S_e) c_q, plus N A in the
    velocity gauge (E is then A(t)), the velocity form of the dipole."""
    zmat = c.conj().T @ (ops.Z @ c)
    dip = np.sum(gamma * zmat).real
    energy = (np.sum(h * gamma) + 0.5 * np.sum(g * Gamma)).real + ops.nuclear_repulsion()
    S = c.conj().T @ (ops.M @ c)
    pmat = c.conj().T @ (ops.momentum() @ c)
    mom = np.sum(gamma * pmat).real
    if ops.gauge == "velocity":
        mom += np.trace(gamma).real * E
    return dict(dipole=dip, energy=energy, overlap=S, momentum=mom)


def orthonormalize(ops, c):
    """Gram-Schmidt of the orbitals in the M inner product."""
    out = []
    for p in range(c.shape[1]):
        v = c[:, p].copy()
        for u in out:
            v = v - np.vdot(u, ops.M @ v) * u
        v = v / np.sqrt(np.vdot(v, ops.M @ v).real)
        out.append(v)
    return np.stack(out, axis=1)


class Propagator:
    """Time steps of the coupled orbital / CI equations."""

    def __init__(self, ops, cispace, poisson=None):
        self.ops = ops
        self.ci = cispace
        self.poisson = poisson or PoissonSolver(ops)

    def freeze(self, c, C, E):
        gamma, Gamma = self.ci.rdms(C)
        W = self.poisson.pair_potentials(c)
        fr = Frozen(self.ops, c, gamma, Gamma, E, W)
        return fr

    def step(self, c, C, E, dt, m=12, imaginary=False, krylov_tol=None):
        """Advance (c, C) by one step from t_n data; returns (c', C', info).
        krylov_tol: error threshold of the adaptive Krylov dimension (at most m)."""
        fr = self.freeze(c, C, E)
        h, g = integrals(self.ops, c, fr.Wfull, E)
        obs = observables(self.ops, c, fr.gamma, fr.Gamma, h, g, E)
        tau = -1j * dt if imaginary else dt
        c2, err, m_eff, _ = arnoldi_step(self.ops, fr.G, c, tau, m, tol=krylov_tol)
        Hci = self.ci.hamiltonian(h, g)
        C2 = lanczos_expm(Hci, C, tau, 12)
        if imaginary:
            c2 = orthonormalize(self.ops, c2)
            C2 = C2 / np.linalg.norm(C2)
        obs.update(err=err, m=m_eff)
        return c2, C2, obs

    def final_observables(self, c, C, E):
        fr = self.freeze(c, C, E)
        h, g = integrals(self.ops, c, fr.Wfull, E)
        return observables(self.ops, c, fr.gamma, fr.Gamma, h, g, E)

    def propagate(self, c, C, E_steps, dt, m=12, imaginary=False, krylov_tol=None):
        """Run len(E_steps) steps; returns final (c, C) and per-step records
        for t_0 .. t_N (the last one from a final freeze at E_steps[-1])."""
        recs = []
        for E in E_steps:
            c, C, obs = self.step(c, C, E, dt, m, imaginary, krylov_tol)
            recs.append(obs)
        recs.append(self.final_observables(c, C, E_steps[-1] if len(E_steps) else 0.0))
        return c, C, recs
