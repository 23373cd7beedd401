"""Differentiable dipole record: a ``torch.autograd.Function`` over
``Operator.propagate`` whose backward is the library's hand-written adjoint
(``mh_propagate_adjoint``: orbitals, mean field and CI vector, up to 4
orbitals and 12 determinants).

Forward: propagate from (phi0, C0) with the step fields E_steps and return
the dipole record d_0..d_N (CPU float64).  Backward: dJ/dE_k from the
incoming dJ/dd_n; E_N does not enter the dipoles and gets zero.  The adjoint
recomputes the orbitals from checkpoints (every ckpt_stride steps, default
round(sqrt(N))), so memory stays O(sqrt(N)) vectors.
"""
import numpy as np
import torch


class DipoleHistory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E_steps, op, phi0, C0, dt, m, n_quad, ckpt_stride):
        E = E_steps.detach().to("cpu", torch.float64).numpy().copy()
        phi = phi0.clone()
        C = C0.clone()
        W = torch.zeros((op.n_full, op.n_pair_cols), dtype=torch.float64, device=phi0.device)
        rec = op.propagate(phi, C, W, E, dt, m=m)
        ctx.save_for_backward(phi0, C0)
        ctx.op, ctx.E, ctx.dt, ctx.m, ctx.n_quad, ctx.stride = op, E, dt, m, n_quad, ckpt_stride
        return torch.from_numpy(rec["dipole"].copy())

    @staticmethod
    def backward(ctx, g):
        phi0, C0 = ctx.saved_tensors
        op = ctx.op
        W = torch.zeros((op.n_full, op.n_pair_cols), dtype=torch.float64, device=phi0.device)
        dJdE = op.propagate_adjoint(phi0, C0, W, ctx.E, ctx.dt, g.detach().to("cpu", torch.float64).numpy(),
                                    m=ctx.m, n_quad=ctx.n_quad, ckpt_stride=ctx.stride)
        grad = torch.zeros(len(ctx.E), dtype=torch.float64)
        grad[:-1] = torch.from_numpy(dJdE)
        return grad, None, None, None, None, None, None, None


def dipole_history(E_steps, op, phi0, C0, dt, m=12, n_quad=6, ckpt_stride=0):
    """Dipole record d_0..d_N as a differentiable function of E_steps (CPU tensor)."""
    return DipoleHistory.apply(E_steps, op, phi0, C0, dt, m, n_quad, ckpt_stride)


def field_at_steps(samples, t_samples, t_steps):
    """Piecewise-linear interpolation of field samples E(t_k) at the step times
    (differentiable in the samples; times outside the sample range clamp)."""
    t_samples = np.asarray(t_samples, dtype=np.float64)
    t_steps = np.clip(np.asarray(t_steps, dtype=np.float64), t_samples[0], t_samples[-1])
    idx = np.clip(np.searchsorted(t_samples, t_steps, side="right") - 1, 0, len(t_samples) - 2)
    w = (t_steps - t_samples[idx]) / (t_samples[idx + 1] - t_samples[idx])
    i0 = torch.from_numpy(idx)
    wt = torch.from_numpy(w)
    return (1.0 - wt) * samples[i0] + wt * samples[i0 + 1]


def harmonic_band_power(d, dt, omega0, lo=5.0, hi=15.0):
    """J = sum over DFT bins with lo <= omega_k / omega0 <= hi of |D_k|^2."""
    D = torch.fft.rfft(d)
    freqs = 2.0 * np.pi * np.arange(D.shape[0]) / (len(d) * dt)
    mask = torch.from_numpy((freqs / omega0 >= lo) & (freqs / omega0 <= hi))
    return (D.abs() ** 2)[mask].sum()
