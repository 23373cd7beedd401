"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host mesh set-up equals the oracle's exactly
(integer counts, node sets, hanging-node constraint rows)."""
import os
import re

import numpy as np
import pytest

from tests.oracle_cases import case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2301_02387_amd as mh
    return mh, mh.load_library()


def test_library_exports_every_declared_symbol():
    mh, lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "mh.h")).read()
    names = set(re.findall(r"\b(mh_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(lib, n), n


@pytest.mark.parametrize("name", ["h_atom", "tiny_q3", "tiny_q1", "small_n3", "h2"])
def test_mesh_equals_oracle(name):
    mh, _ = _lib()
    from tests.lib_cases import match_nodes
    w, om, ops = case(name)
    M = mh.Mesh.from_workload(w)
    oi = om.info()
    for k in ("n_cells", "n_full", "n_dof", "n_hang", "n_masters", "hang_nnz"):
        assert M.info[k] == oi[k], k
    assert M.info["level_counts"] == oi["level_counts"]
    perm = match_nodes(M.coords(), om.xyz)
    N, Nh = M.info["n_dof"], M.info["n_hang"]
    # node classes agree
    assert np.all(om.dof_of[perm[:N]] >= 0)
    assert np.all(om.is_hang[perm[N:N + Nh]])
    assert np.all(om.is_bnd[perm[N + Nh:]] & ~om.is_hang[perm[N + Nh:]])
    # constraint rows agree (masters mapped through the node matching)
    ptr, col, wts = M.constraints()
    for h in range(0, Nh, max(1, Nh // 200)):
        mine = {int(perm[c]): wv for c, wv in zip(col[ptr[h]:ptr[h + 1]], wts[ptr[h]:ptr[h + 1]])}
        ref = om.hang_rows[int(perm[N + h])]
        assert set(mine) == set(ref)
        for k, v in ref.items():
            assert abs(mine[k] - v) < 1e-14


def test_h2o_mesh_counts():
    mh, _ = _lib()
    from synth import workload
    M = mh.Mesh.from_workload(workload("h2o"))
    # the 58,304-cell, ~1.5M-DoF H2O mesh under the geometric refinement rule
    assert M.info["n_cells"] == 58304
    assert M.info["n_dof"] == 1517876


def test_allocator_registration_arguments():
    """mh_set_allocator takes both functions or neither (no GPU work)."""
    mh, lib = _lib()
    from paper_2301_02387_amd._lib import _ALLOC_FN, _FREE_FN
    keep = _ALLOC_FN(lambda nbytes, ctx: None)
    assert lib.mh_set_allocator(keep, _FREE_FN(), None) == -1
    assert "both" in lib.mh_last_error().decode()
    assert lib.mh_set_allocator(_ALLOC_FN(), _FREE_FN(), None) == 0


def test_error_paths():
    mh, _ = _lib()
    with pytest.raises(mh.MHError) as e:
        mh.Mesh(-1, 1, 2, 4, [])
    assert e.value.code == -6
    with pytest.raises(mh.MHError) as e:
        mh.Mesh(1, -1, 2, 2, [])
    assert e.value.code == -1
