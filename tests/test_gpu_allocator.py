"""GPU: the library's own device workspaces from a registered allocator
(mh_set_allocator, here torch's caching allocator): an operator created
under it gives the same pair potentials and propagated observables as one on
hipMalloc, and hands every buffer back to it when destroyed."""
import gc

import numpy as np
import pytest

from synth import random_ci, random_orbitals
from tests.lib_cases import Pair

pytestmark = pytest.mark.gpu


def _run(torch):
    from oracle.ci import CISpace
    from oracle.mctdhf import orthonormalize
    P = Pair("tiny_q3", poisson_rtol=1e-13, poisson_maxit=20000)
    P.op.tune(1, 53, 8192)   # multigrid and sliced-ELL rows: workspaces built on first use
    w = P.w
    n = w["n_orb"]
    om = P.om
    c = orthonormalize(P.ops, random_orbitals(om.xyz[om.dof_nodes], n, 4, spread=1.5))
    x = torch.from_numpy(np.ascontiguousarray(P.to_lib_orb(c))).cuda()
    W = torch.zeros((P.NF, n * n), dtype=torch.float64, device="cuda")
    it, rc = P.op.poisson_pairs(x, W)
    assert rc == 0
    Cd = torch.from_numpy(random_ci(CISpace(n, w["n_alpha"], w["n_beta"]).dim, 5)).cuda()
    rec = P.op.propagate(x, Cd, W, [0.01, 0.02, 0.0], 0.02, m=10)
    torch.cuda.synchronize()
    out = (W.cpu().numpy(), np.asarray(rec["dipole"]), np.asarray(rec["energy"]), x.cpu().numpy())
    del P
    gc.collect()
    return out


def test_operator_on_registered_allocator():
    import torch
    import paper_2301_02387_amd as mh
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    counts = {"alloc": 0, "free": 0}
    live = {}

    def alloc(nbytes):
        p = torch.cuda.caching_allocator_alloc(int(nbytes))
        counts["alloc"] += 1
        live[p] = nbytes
        return p

    def free(ptr, nbytes):
        assert live.pop(ptr) == nbytes
        counts["free"] += 1
        torch.cuda.caching_allocator_delete(int(ptr))

    plain = _run(torch)
    try:
        mh.set_allocator(alloc, free)
        registered = _run(torch)
    finally:
        mh.set_allocator()
    assert counts["alloc"] > 50 and counts["free"] == counts["alloc"] and not live, (counts, len(live))
    for a, b in zip(plain, registered):
        assert np.max(np.abs(a - b)) <= 1e-12 * max(np.abs(a).max(), 1e-300)
