"""The allocation-free mass solve (mh_mass_solve_noalloc) against
mh_mass_solve through the C ABI: calls in a row on different operators, the
second with a smaller interface system, each equal to the allocating entry
point's result (and to the oracle's sparse LU); also on a batch handle, whose
instances lie end to end in the static scratch array.  Collected last: it
must pass alone and after every other GPU test."""
import numpy as np
import pytest

from synth import random_orbitals
from tests.lib_cases import Pair, rel_err_cols, max_rel_cols

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _load(P, seed):
    from oracle.mctdhf import orthonormalize
    om = P.om
    c = orthonormalize(P.ops, random_orbitals(om.xyz[om.dof_nodes], P.w["n_orb"], seed, spread=1.5))
    return np.ascontiguousarray((P.ops.M @ c)[P.dof_or])


def _both(op, f, n_ext, n):
    torch = _torch()
    a = torch.zeros((n_ext, n), dtype=torch.complex128, device="cuda")
    b = torch.full((n_ext, n), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    op.mass_solve(f, a)
    op.mass_solve_noalloc(f, b)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_mass_solve_equals_mass_solve():
    torch = _torch()
    big, small = Pair("h2"), Pair("tiny_q3")
    assert small.om.masters.size < big.om.masters.size
    for P, seed in ((big, 1), (small, 2), (big, 3)):
        n = P.w["n_orb"]
        f = torch.from_numpy(_load(P, seed)).cuda()
        for sched in (1, 3):      # bit 1: Chebyshev interface solve even where a dense inverse is held
            P.op.tune(0, sched, 65536)
            a, b = _both(P.op, f, P.NE, n)
            assert np.isfinite(b).all()
            assert rel_err_cols(b, a) < 1e-12 and max_rel_cols(b, a) < 1e-12, (P.w["name"], sched)
            ref = P.ops.mass_solve(P.from_lib_dof(f.cpu().numpy()))     # the oracle's sparse LU
            assert rel_err_cols(P.from_lib_dof(b), ref) < 1e-12
        P.op.tune(0, 1, 65536)


def test_noalloc_mass_solve_on_a_batch():
    torch = _torch()
    import paper_2301_02387_amd as mh
    pairs = [Pair("tiny_q3", seed=s, with_op=False) for s in (0, 1, 2)]
    w = pairs[0].w
    op = mh.Operator.batch([P.mesh for P in pairs], [P.w["nuclei"] for P in pairs], w["n_orb"], w["n_alpha"],
                           w["n_beta"])
    lay = op.layout()
    n = w["n_orb"]
    f = np.zeros((op.n_ext, n), dtype=complex)
    for i, P in enumerate(pairs):
        f[lay[i, 3]:lay[i, 3] + P.N] = _load(P, 10 + i)
    fd = torch.from_numpy(f).cuda()
    for _ in range(2):
        a, b = _both(op, fd, op.n_ext, n)
        assert rel_err_cols(b, a) < 1e-12 and max_rel_cols(b, a) < 1e-12
