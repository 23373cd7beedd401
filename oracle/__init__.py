"""Plain CPU oracle for the MCTDHF-on-adaptive-FEM hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
execute anything under this directory; only ``tests/``, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is written from the paper (Orimo, Sato & Ishikawa, arXiv
2301.02387) in plain NumPy/SciPy, in FP64 / complex128, with no blocking,
fusion or reordering beyond what the method states.  It shares no code with
the HIP path.  Each module header names the section or equation it follows.

Modules
-------
gll      Gauss-Lobatto-Legendre nodes, weights and 1D operators (Sec. III.A).
mesh     octree refinement, 2:1 balance, full nodes, hanging-node
         constraints and DoF numbering (Sec. III.A, "bridged functions").
fem      mass, stiffness, lumped nuclear potential, dipole and H1 matrices
         (Sec. III.A, Eq. discretized_eom and the GLL quadrature rule).
ecs      exterior complex scaling of the one-body operator (Sec. IV).
poisson  pair densities, multipole boundary values and the Poisson solve
         for the mean-field potentials (Sec. III.A, Poisson equation + BC).
ci       determinant strings, sigma vector, RDMs, CI Hamiltonian (Sec. II).
mctdhf   frozen operator G, short-iterative Arnoldi step, CI step,
         observables and time propagation (Sec. II Eqs. ci_eom / orb_eom,
         Sec. III.B Eq. packed_orb_eom).
"""
