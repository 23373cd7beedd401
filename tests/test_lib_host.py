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


@pytest.mark.parametrize("name", ["h_atom", "tiny_q3", "tiny_q1", "small_n3", "h2", "uniform_q2", "uniform_q1_odd",
                                  "kelly_q1", "kelly_q2"])
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


@pytest.mark.parametrize("name", ["tiny_q3", "kelly_q2"])
def test_mesh_cells(name):
    """mh_mesh_cells: each cell's local node (a, b, c) sits at origin + edge
    (xi + 1) / 2 of the Gauss-Lobatto points, x fastest; every full node
    belongs to a cell; the leaves are the oracle's (same levels and corners)."""
    mh, _ = _lib()
    from oracle.gll import gll
    w, om, ops = case(name)
    M = mh.Mesh.from_workload(w)
    nodes, level, origin = M.cells()
    p = M.info["p"]
    xi, _ = gll(p)
    H = (w["hi"] - w["lo"]) / w["n_coarse"]
    edge = H / 2.0 ** level
    xyz = M.coords()
    t = (xi + 1.0) / 2.0
    loc = np.array([(t[a], t[b], t[c]) for c in range(p + 1) for b in range(p + 1) for a in range(p + 1)])
    want = origin[:, None, :] + edge[:, None, None] * loc[None, :, :]
    assert np.abs(xyz[nodes] - want).max() < 1e-12
    assert len(np.unique(nodes)) == M.info["n_full"]
    key = lambda l, o: (int(l),) + tuple(int(round(v * 1e6)) for v in o)  # noqa: E731
    lib_cells = sorted(key(l, o) for l, o in zip(level, origin))
    or_cells = sorted(key(l, [w["lo"] + H / 2.0 ** l * v for v in (i, j, k)]) for l, i, j, k in om.cells)
    assert lib_cells == or_cells


@pytest.mark.parametrize("p,tol", [(1, 0.05), (2, 0.02), (3, 0.02)])
def test_kelly_mesh_equals_oracle(p, tol):
    """The water nuclei's Kelly refinement (Sec. III.A) in the library and in
    the oracle: the same leaves (cell and level counts, the same node set)
    after the same number of refinement rounds, at degrees 1 to 3."""
    mh, _ = _lib()
    from tests.lib_cases import match_nodes
    from oracle.kelly import kelly_refine, softened_coulomb
    from oracle.mesh import Mesh as OMesh, MeshDesc, balance_21, build_leaves
    hx, hy = 1.42994, 1.10718
    nuc = [(8.0, (0.0, 0.0, 0.0)), (1.0, (hx, hy, 0.0)), (1.0, (-hx, hy, 0.0))]
    M = mh.Mesh(-16.0, 16.0, 4, p, [], kelly=dict(nuclei=nuc, tol=tol, soft=0.05, max_level=3))
    desc = MeshDesc(-16.0, 16.0, 4, p, [], kelly_nuclei=nuc, kelly_tol=tol, kelly_soft=0.05, kelly_max_level=3)
    om = OMesh(desc)
    base = build_leaves(MeshDesc(-16.0, 16.0, 4, p, []))
    _, rounds = kelly_refine(base, -16.0, 16.0, 4, p, softened_coulomb(nuc, 0.05), tol, 3,
                             lambda L: balance_21(L, 4))
    oi = om.info()
    for k in ("n_cells", "n_full", "n_dof", "n_hang", "n_masters", "hang_nnz"):
        assert M.info[k] == oi[k], k
    assert M.info["level_counts"] == oi["level_counts"]
    assert M.info["kelly_rounds"] == rounds > 0
    perm = match_nodes(M.coords(), om.xyz)
    assert len(perm) == om.n_full


def test_kelly_request_errors():
    mh, _ = _lib()
    nuc = [(1.0, (0.0, 0.0, 0.0))]
    for bad in (dict(tol=0.0, soft=0.1, max_level=2), dict(tol=0.01, soft=0.0, max_level=2),
                dict(tol=0.01, soft=0.1, max_level=-1)):
        with pytest.raises(mh.MHError):
            mh.Mesh(-4.0, 4.0, 2, 1, [], kelly=dict(nuclei=nuc, **bad))


def test_h2o_q1_mesh_levels():
    """The Q1 water workload's Kelly mesh spans six cell sizes, 4.0 down to
    0.125 bohr, as the mesh of Sec. IV does."""
    mh, _ = _lib()
    from synth import workload
    M = mh.Mesh.from_workload(workload("h2o_q1"))
    assert len(M.info["level_counts"]) == 6 and all(c > 0 for c in M.info["level_counts"])
    assert M.info["p"] == 1 and M.info["kelly_rounds"] == 5


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


def test_argument_errors_before_device_work():
    """Every entry point rejects a missing handle or a bad descriptor with its
    documented status before any device call (so this runs without a GPU):
    null handles give MH_INVALID_ARG (-1), out-of-range orbital counts and
    boundary orders MH_UNSUPPORTED (-6), inconsistent batches MH_INVALID_ARG."""
    import ctypes as C
    from synth import small_workload
    from paper_2301_02387_amd._lib import _OpDesc, _op_desc, _Sizes
    mh, lib = _lib()
    INVALID, UNSUP = -1, -6
    d = C.c_double(0.0)
    i32 = C.c_int32(0)
    i64 = C.c_int64(0)
    # op entry points with no handle
    assert lib.mh_fill_hanging(None, None, None) == INVALID
    assert lib.mh_mass_solve(None, None, None, None) == INVALID
    assert lib.mh_h1_apply(None, None, 0.0, None, None) == INVALID
    assert lib.mh_poisson_pairs(None, None, None, 0, C.byref(i32), None) == INVALID
    assert lib.mh_ci_rdms(None, None, None, None, None) == INVALID
    assert lib.mh_freeze(None, None, None, None, 0.0, None, None) == INVALID
    assert lib.mh_rhs_apply(None, None, None, None) == INVALID
    assert lib.mh_arnoldi_step(None, None, 0.01, 0.0, 8, C.byref(d), C.byref(i32), None) == INVALID
    assert lib.mh_propagate(None, None, None, None, None, 1, 0.01, 8, 0, None, None) == INVALID
    assert lib.mh_propagate_adjoint(None, None, None, None, None, 1, 0.01, 8, None, None, 2, 0, None) == INVALID
    assert lib.mh_op_sizes_get(None, C.byref(_Sizes())) == INVALID
    assert lib.mh_batch_layout(None, None) == INVALID
    assert lib.mh_kernel_timing(None, 0, 1, C.byref(d), C.byref(i64)) == INVALID
    assert lib.mh_tune(None, 1, 13, 8192) == INVALID
    assert lib.mh_op_destroy(None) == 0
    # mesh entry points with no handle
    assert lib.mh_mesh_info_get(None, None) == INVALID
    assert lib.mh_mesh_node_coords(None, None) == INVALID
    assert lib.mh_mesh_constraints(None, None, None, None) == INVALID
    assert lib.mh_mesh_destroy(None) == 0
    # descriptors rejected before the operator is built
    w = small_workload("tiny_q3", 0)
    M = mh.Mesh.from_workload(w)
    h = C.c_void_p()

    def desc(**kw):
        args = dict(nuclei=w["nuclei"], n_orb=w["n_orb"], n_alpha=w["n_alpha"], n_beta=w["n_beta"],
                    polarization=(0.0, 0.0, 1.0), lmax_bc=12, poisson_rtol=1e-12, poisson_maxit=100, rdm_eps=1e-10)
        args.update(kw)
        return _op_desc(**args)

    assert lib.mh_op_create(None, C.byref(desc()[0]), None, C.byref(h)) == INVALID
    for kw, code in [(dict(n_orb=9), UNSUP), (dict(n_orb=0), UNSUP), (dict(lmax_bc=13), UNSUP),
                     (dict(n_alpha=w["n_orb"] + 1), INVALID), (dict(n_alpha=0, n_beta=0), INVALID),
                     (dict(n_beta=-1), INVALID)]:
        dd, keep = desc(**kw)
        assert lib.mh_op_create(M._h, C.byref(dd), None, C.byref(h)) == code, kw
        assert lib.mh_last_error()
    dd, keep = desc()
    dd.charges = C.POINTER(C.c_double)()  # nuclei announced, charges missing
    assert lib.mh_op_create(M._h, C.byref(dd), None, C.byref(h)) == INVALID
    # batches: empty, too many, a null mesh, instances that disagree
    w1 = small_workload("tiny_q1", 0)
    M1 = mh.Mesh.from_workload(w1)
    d0, k0 = desc()
    d9, k9 = desc(n_orb=w["n_orb"] + 1, n_alpha=w["n_alpha"], n_beta=w["n_beta"])
    d1, k1 = desc()

    def batch(meshes, descs, n=None):
        hs = (C.c_void_p * len(meshes))(*[m._h.value if m is not None else None for m in meshes])
        ds = (_OpDesc * len(descs))(*descs)
        return lib.mh_batch_create(C.cast(hs, C.c_void_p), C.cast(ds, C.c_void_p), None,
                                   len(meshes) if n is None else n, None, C.byref(h))

    assert batch([M], [d0], n=0) == INVALID
    assert batch([M], [d0], n=5000) == UNSUP
    assert batch([M, None], [d0, d1]) == INVALID
    assert batch([M, M], [d0, d9]) == INVALID
    assert w1["p"] != w["p"]
    assert batch([M, M1], [d0, d1]) == INVALID
    assert "share p" in lib.mh_last_error().decode()


def test_header_compiles_as_c(tmp_path):
    """include/mh.h is a C header: it compiles with a C99 compiler alone."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    src = tmp_path / "use.c"
    src.write_text('#include "mh.h"\nint main(void) { return mh_mass_solve(0, 0, 0, 0) == MH_INVALID_ARG ? 0 : 1; }\n')
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-I", os.path.join(ROOT, "include"),
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
