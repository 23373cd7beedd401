"""Host logic of the schedule autotuner (no GPU): cached schedules are keyed
by mesh signature, degree, orbitals and instances, read back from the JSON
cache file and applied to the operator through its tune hook."""
import json

from paper_2301_02387_amd import tune


class _Mesh:
    def __init__(self, cells, dof, hang, p):
        self.info = {"n_cells": cells, "n_dof": dof, "n_hang": hang, "p": p}


class _Op:
    """Stand-in for an Operator: records the schedules it is given."""

    def __init__(self, cells=2736, dof=66635, hang=9240, p=3, n_orb=2, n_inst=1):
        self.mesh = _Mesh(cells, dof, hang, p)
        self.n_orb, self.n_inst, self.n_dof = n_orb, n_inst, dof
        self.calls = []

    def tune(self, which, sched, grid):
        self.calls.append((which, sched, grid))


def test_cached_schedules_are_applied(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "_CACHE", {})
    op = _Op()
    f = tmp_path / "tune.json"
    f.write_text(json.dumps({tune._key(op): {"orbital": [4, 65536], "poisson": [53, 8192]}}))
    best = tune.apply_cached(op, str(f))
    assert best["orbital"] == (4, 65536) and best["poisson"] == (53, 8192)
    assert op.calls == [(0, 4, 65536), (1, 53, 8192)]
    # a second operator of the same signature is served from memory
    op2 = _Op()
    assert tune.apply_cached(op2) == best and op2.calls == op.calls


def test_cache_key_separates_operators(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "_CACHE", {})
    f = tmp_path / "tune.json"
    f.write_text(json.dumps({tune._key(_Op()): {"orbital": [4, 65536], "poisson": [53, 8192]}}))
    for other in (_Op(n_orb=8), _Op(n_inst=64), _Op(p=2), _Op(dof=66636), _Op(hang=9241)):
        assert tune._key(other) != tune._key(_Op())
        assert tune.apply_cached(other, str(f)) is None and other.calls == []
    assert tune.apply_cached(_Op(), str(tmp_path / "missing.json")) is not None  # loaded above
    monkeypatch.setattr(tune, "_CACHE", {})
    assert tune.apply_cached(_Op(), str(tmp_path / "missing.json")) is None


def test_candidate_schedules_are_valid():
    """Every candidate is a schedule the library accepts (Poisson bits 0-9,
    orbital bits 0-2) with a grid cap in range."""
    for sched, grid in tune.ORB_CANDIDATES + tune.ORB_CANDIDATES_BATCH:
        assert 0 <= sched <= 7 and 8 <= grid <= 65536
    for sched, grid in tune.POI_CANDIDATES + tune.POI_CANDIDATES_WIDE + tune.POI_CANDIDATES_BATCH:
        assert 0 <= sched <= 1023 and 8 <= grid <= 65536
        assert not (sched & 64) or (sched & 16)   # float finest level only with the multigrid preconditioner
        assert not (sched & 128) or (sched & 2)   # column blocks bound to XCDs only with column blocks
        assert not (sched & 768) or (sched & 16)  # smoothing degree only with the multigrid preconditioner
