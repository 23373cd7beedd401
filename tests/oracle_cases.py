"""Shared, cached oracle set-ups for the tests (builds each mesh once)."""
import functools

import numpy as np

from oracle.mesh import Mesh, MeshDesc, Ball
from oracle.fem import Operators
from synth import workload, small_workload


def desc_of(w):
    k = w.get("kelly") or {}
    return MeshDesc(w["lo"], w["hi"], w["n_coarse"], w["p"], [Ball(**b) for b in w["balls"]],
                    kelly_nuclei=list(k.get("nuclei", [])), kelly_tol=k.get("tol", 0.0),
                    kelly_soft=k.get("soft", 0.0), kelly_max_level=k.get("max_level", 0))


# Degenerate meshes for the tests only: no refinement, so no hanging nodes and
# no interface block of the mass matrix.  On the odd Q1 grid the multigrid
# hierarchy has a single level (nothing coarser nests in it), solved by the
# dense inverse of the whole operator.
TEST_WORKLOADS = {
    "uniform_q2": dict(name="uniform_q2", lo=-5.0, hi=5.0, n_coarse=4, p=2, balls=[],
                       nuclei=[(1.0, (0.0, 0.0, 0.6)), (1.0, (0.0, 0.0, -0.6))], n_orb=2, n_alpha=1, n_beta=1),
    "uniform_q1_odd": dict(name="uniform_q1_odd", lo=-5.0, hi=5.0, n_coarse=5, p=1, balls=[],
                           nuclei=[(1.0, (0.3, -0.2, 0.1))], n_orb=2, n_alpha=1, n_beta=1),
    # CI spaces at their edges: no alpha electron (the empty string; with two
    # orbitals the 1-RDM of one electron has rank one, so that case only feeds
    # the RDM test, the one-orbital one the propagation), and a full alpha
    # shell (every orbital occupied) beside one beta electron
    "beta_one": dict(name="beta_one", lo=-6.0, hi=6.0, n_coarse=3, p=2,
                     balls=[dict(center=(0.3, -0.2, 0.4), radius=1.0, levels=1)],
                     nuclei=[(1.0, (0.0, 0.0, 0.0))], n_orb=1, n_alpha=0, n_beta=1),
    "beta_only": dict(name="beta_only", lo=-6.0, hi=6.0, n_coarse=3, p=2,
                      balls=[dict(center=(0.3, -0.2, 0.4), radius=1.0, levels=1)],
                      nuclei=[(1.0, (0.0, 0.0, 0.0))], n_orb=2, n_alpha=0, n_beta=1),
    "full_alpha": dict(name="full_alpha", lo=-6.0, hi=6.0, n_coarse=3, p=2,
                       balls=[dict(center=(0.3, -0.2, 0.4), radius=1.0, levels=1)],
                       nuclei=[(3.0, (0.0, 0.0, 0.0))], n_orb=2, n_alpha=2, n_beta=1),
}


@functools.lru_cache(maxsize=None)
def case(name, seed=0):
    if name in TEST_WORKLOADS:
        w = TEST_WORKLOADS[name]
    else:
        try:
            w = workload(name)
        except KeyError:
            w = small_workload(name, seed)
    mesh = Mesh(desc_of(w))
    ops = Operators(mesh, w["nuclei"], pol=w.get("polarization", (0.0, 0.0, 1.0)))
    return w, mesh, ops
