"""Shared, cached oracle set-ups for the tests (builds each mesh once)."""
import functools

import numpy as np

from oracle.mesh import Mesh, MeshDesc, Ball
from oracle.fem import Operators
from synth import workload, small_workload


def desc_of(w):
    return MeshDesc(w["lo"], w["hi"], w["n_coarse"], w["p"], [Ball(**b) for b in w["balls"]])


@functools.lru_cache(maxsize=None)
def case(name, seed=0):
    try:
        w = workload(name)
    except KeyError:
        w = small_workload(name, seed)
    mesh = Mesh(desc_of(w))
    ops = Operators(mesh, w["nuclei"])
    return w, mesh, ops
