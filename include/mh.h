/*
 * mh.h -- C ABI of the MI355X MCTDHF-on-octree-FEM hot path.
 *
 * Method: multiconfiguration time-dependent Hartree-Fock on an adaptive
 * finite-element mesh (Orimo, Sato & Ishikawa, arXiv 2301.02387).  The
 * library sets up the discretisation of Sec. III.A, applies the frozen
 * packed orbital operator G of Sec. III.B (Eq. packed_orb_eom), solves the
 * pair Poisson problems that give the mean-field potentials (Sec. III.A,
 * Poisson equation with its boundary integral), takes short-iterative
 * Arnoldi steps exp(-i G dt) and propagates orbitals and CI coefficients
 * together (Sec. II, Eqs. ci_eom and orb_eom with X = 0).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Status: every entry point returns int; 0 = MH_OK, 1 = MH_NOT_CONVERGED
 *    (outputs hold the last iterate), negative = failure.  The message of the
 *    last failure on the calling thread is returned by mh_last_error().  No
 *    C++ exception crosses this boundary.
 *  - Complex numbers are complex128, stored as interleaved (re, im) doubles;
 *    a "c128 array of length L" is 2L doubles.
 *  - Node order: the library numbers the full (Gauss-Lobatto) nodes as
 *    [0, N) unknown DoFs, [N, N + N_h) hanging nodes, [N + N_h, N_F) nodes on
 *    the box boundary.  N_E = N + N_h.
 *  - Orbital arrays are DEVICE c128 arrays [N_E][n] (orbital index fastest).
 *    Rows [0, N) are the DoF coefficients; rows [N, N_E) are the hanging-node
 *    values, which every output fills consistently (row h = sum_k c_hk row k)
 *    and every input must carry consistently (mh_fill_hanging does it).
 *    Boundary rows are not stored: orbitals vanish on the box boundary.
 *  - Device arrays are owned by the caller; the library never frees them.
 *    Handles (mh_mesh, mh_op) are owned by the library and freed by their
 *    destroy call.  Internal device workspaces are allocated by the library
 *    at mh_op_create.
 *  - Batches: an operator handle holds one or more independent instances
 *    (mh_op_create: one; mh_batch_create: several meshes and molecules of
 *    one orbital/electron space).  Every call then acts on all instances at
 *    once (one kernel launch covers them all).  A batch array is the
 *    per-instance arrays laid end to end: instance i owns rows
 *    [oE_i, oE_i + N_E,i) of every array over extended rows (orbitals, load
 *    vectors) and rows [oF_i, oF_i + N_F,i) of every array over full rows
 *    (pair potentials W); mh_batch_layout gives the offsets.  Small
 *    per-instance arrays (CI vectors, RDMs) are [n_inst][...].  Arrays
 *    documented below as [N][n] hold, for a batch, [sum N_E][n] with the
 *    extended-row offsets.  For a single instance every offset is 0.
 *  - Streams: every device call is enqueued on the hipStream_t given as
 *    `stream` (NULL = the default stream) and returns without synchronising,
 *    except where a call returns host results (noted per call), which
 *    synchronises that stream.  Asynchronous device errors surface at the next
 *    synchronising call.
 */
#ifndef MH_H
#define MH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MH_OK = 0,
  MH_NOT_CONVERGED = 1,
  MH_INVALID_ARG = -1,
  MH_OOM = -2,
  MH_HIP_ERROR = -3,
  MH_SINGULAR_RDM = -4,
  MH_NONFINITE = -5,
  MH_UNSUPPORTED = -6
};

typedef struct mh_mesh mh_mesh;
typedef struct mh_op mh_op;

/* A refinement ball: leaves of level l that come strictly closer than
 * `radius` to `center` are halved while l < levels (Sec. III.A: coarse cubes
 * halved recursively where resolution is needed; geometric criterion). */
typedef struct {
  double center[3];
  double radius;
  int32_t levels;
} mh_ball;

/* Box [lo, hi]^3 covered by n_coarse^3 cubes, Lagrange degree p (1..3) on
 * Gauss-Lobatto points (Sec. III.A), refined by the balls, then 2:1 balanced
 * over all 26 neighbours.
 *
 * Kelly refinement (Sec. III.A: cells halved until Kelly's indicator of the
 * nuclear Coulomb potential meets a threshold in every cell), when
 * n_kelly > 0, after the balls: u_K interpolates the softened potential
 * V = -sum Z / sqrt(|r - R|^2 + kelly_soft^2) at the Gauss-Lobatto nodes of
 * leaf K alone; eta_K^2 = (h_K / 24) * sum over K's interior faces of the
 * integral of the squared jump of du/dn (h_K = sqrt(3) * edge; each part of
 * a face shared with one neighbour integrated exactly by Gauss-Legendre).
 * Every leaf with eta_K > kelly_tol below level kelly_max_level is halved,
 * the tree re-balanced, and the indicators recomputed until none is marked.
 * MH_INVALID_ARG for kelly_soft <= 0, kelly_tol <= 0 or a negative level. */
typedef struct {
  double lo, hi;
  int32_t n_coarse;
  int32_t p;
  int32_t n_balls;
  const mh_ball* balls;          /* host array, read during the call only */
  int32_t n_kelly;               /* nuclei of the Kelly target (0: no Kelly refinement) */
  const double* kelly_nuclei;    /* host [n_kelly][4]: Z, x, y, z; read during the call only */
  double kelly_tol;              /* threshold on eta_K */
  double kelly_soft;             /* softening length (bohr) */
  int32_t kelly_max_level;       /* deepest level a Kelly split may create */
} mh_mesh_desc;

typedef struct {
  int64_t n_cells, n_full, n_dof, n_hang, n_bnd, n_masters, hang_nnz;
  int32_t p, max_level;
  int64_t level_counts[16];
  int32_t kelly_rounds;          /* Kelly refinement rounds taken (0 without Kelly) */
} mh_mesh_info;

/* Build the octree, nodes, hanging-node constraints (bridged basis of
 * Sec. III.A: a node is hanging iff the coarsest leaf containing it lacks it;
 * its value is that leaf's interpolant) and the node numbering above.
 * Host-only.  MH_UNSUPPORTED for p outside 1..3; MH_INVALID_ARG for an empty
 * box or a refinement deeper than the 19-bit octree index allows. */
int mh_mesh_create(const mh_mesh_desc* desc, mh_mesh** out);
int mh_mesh_info_get(const mh_mesh* mesh, mh_mesh_info* info);
/* Host double [N_F][3]: coordinates of every full node in library order. */
int mh_mesh_node_coords(const mh_mesh* mesh, double* xyz);
/* Host: hanging rows in CSR over full-node columns (masters are DoFs or
 * boundary nodes).  ptr: int64 [N_h + 1]; col: int64 [hang_nnz]; w: double
 * [hang_nnz].  Any pointer may be NULL to skip it. */
int mh_mesh_constraints(const mh_mesh* mesh, int64_t* ptr, int64_t* col, double* w);
/* Host: the leaves in library order (Morton order of the octree, Sec. III.A).
 * nodes: int32 [n_cells][(p+1)^3], the library index of each cell-local
 * Gauss-Lobatto node (a, b, c) at (c (p+1) + b) (p+1) + a, x fastest;
 * level: int32 [n_cells] refinement level (edge = (hi - lo) / n_coarse / 2^level);
 * origin: double [n_cells][3] lower corner.  Any pointer may be NULL. */
int mh_mesh_cells(const mh_mesh* mesh, int32_t* nodes, int32_t* level, double* origin);
int mh_mesh_destroy(mh_mesh* mesh);

/* Molecule and operator settings. */
typedef struct {
  int32_t n_nuclei;
  const double* charges;      /* host [n_nuclei] */
  const double* positions;    /* host [n_nuclei][3] */
  int32_t n_orb;              /* n spatial orbitals (1..8) */
  int32_t n_alpha, n_beta;    /* electrons per spin (full CAS over n orbitals) */
  double polarization[3];     /* unit field direction e (length gauge E(t) e.r) */
  int32_t lmax_bc;            /* multipole order of the Poisson boundary values (1..12;
                                 0 selects 12) */
  double poisson_rtol;        /* residual target of the pair Poisson CG: each column of an
                                 instance to |r| <= rtol x the largest |rhs| of its columns */
  int32_t poisson_maxit;      /* CG iteration cap */
  double rdm_eps;             /* regularisation of the 1-RDM inverse (<= 0 selects 1e-10) */
  int32_t gauge;              /* MH_GAUGE_LENGTH: field term E(t) e.r; MH_GAUGE_VELOCITY: term
                                 -i A(t) e.grad (Sec. II one-body operator), the field values
                                 passed to the calls below then being A(t) */
  double krylov_tol;          /* 0: Arnoldi steps use the Krylov dimension m they are given;
                                 > 0: adaptive dimension (Sec. III.B): the space stops growing
                                 at the first dimension whose error estimate is <= krylov_tol,
                                 m being the largest (one small synchronising read per vector) */
  double ecs_theta;           /* exterior complex scaling angle (0 <= theta < pi/2; 0: none) */
  double ecs_inner[3];        /* half-widths R_d of the unscaled cuboid |x_d| <= R_d about the origin */
} mh_op_desc;

/* Exterior complex scaling (Sec. IV: an absorbing boundary outside an inner
 * cuboid), when ecs_theta > 0.  Each coordinate beyond |x_d| = R_d continues
 * along z_d = sign(x_d) R_d + e^{i theta} (x_d - sign(x_d) R_d); the
 * one-body operator takes its Galerkin form on that contour (per cell the
 * volume factor J = prod_d dz_d/dx_d on the mass, J / eta_d^2 on the
 * stiffness along d, J / eta_d on the velocity-gauge derivative along d, the
 * Coulomb potential continued to V(z(x)) J with the principal square root,
 * and the length-gauge field e.z(x) J).  The orbital inner product stays the
 * Hermitian one of the real coordinates (M), the pair Poisson solves and the
 * mean field stay on the real grid, and the orbital operator is
 * M_theta^{-1} F_theta, M_theta the contour's mass.  The library hands that
 * on as the load vector M M_theta^{-1} F_theta (for the real mass solve),
 * which is what mh_h1_apply returns; h_pq and lam are then M inner products
 * and H_CI is non-Hermitian (the CI step's Krylov process orthogonalises
 * fully, so it needs no symmetry).  Dipole and momentum records use the
 * real coordinates; the energy record is the real part.  mh_op_create
 * returns MH_INVALID_ARG when a cell straddles a plane |x_d| = R_d, a
 * nucleus lies outside the open cuboid, or a hanging node or a master of
 * one touches a scaled cell; the adjoint returns MH_UNSUPPORTED. */

enum { MH_GAUGE_LENGTH = 0, MH_GAUGE_VELOCITY = 1 };

/* Operator set-up (Sec. III.A): Gauss-Lobatto masses, stiffness data, the
 * lumped nuclear potential v_i = sum_cells int f_i V_nuc (six-pyramid Duffy
 * rule in cells whose closure holds a nucleus, Gauss-Legendre with p+5
 * points elsewhere), dipole weights m (e.x), the hanging-interface block of
 * the mass matrix and the multipole tables; uploads everything and allocates
 * device workspaces.  Synchronises `stream`. */
int mh_op_create(const mh_mesh* mesh, const mh_op_desc* desc, void* stream, mh_op** out);
int mh_op_destroy(mh_op* op);

/* Hanging rows of an orbital array in place: x[h] = sum_k c_hk x[k]
 * (Sec. III.A bridged functions).  x: device c128 [N_E][n]. */
int mh_fill_hanging(mh_op* op, double* x, void* stream);

/* Mass solve of the discretised orbital equation (Eq. discretized_eom):
 * c = M^{-1} f with M = C^T diag(m) C (Gauss-Lobatto overlap of the bridged
 * basis).  f: device c128 [N][n] load vector (DoF rows only are read);
 * c: device c128 [N_E][n] output, hanging rows filled. */
int mh_mass_solve(mh_op* op, const double* f, double* c, void* stream);

/* Allocation-free variant of mh_mass_solve, for callers that cannot
 * allocate device memory during the call (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, result
 * and kernels as mh_mass_solve; the interface system's right-hand side,
 * iterate, residual and search directions live in a static device array of
 * 32 MiB that every GPU the library runs on holds until the process ends
 * (its address is taken when an operator is created on that device), instead
 * of the operator's own workspaces.  The call allocates nothing (no
 * hipMalloc, no registered allocator).  MH_UNSUPPORTED when the interface
 * system needs more than 32 MiB (5 x 16 x n bytes per interface unknown,
 * summed over the instances); MH_INVALID_ARG when called with another device
 * current than the one the operator was created on.  All calls on one GPU
 * share the array: calls that overlap in time on one GPU (two streams, two
 * threads) race and give wrong results; calls in one stream are ordered and
 * safe.  Nothing in the array needs clearing: each call writes every element
 * it reads before reading it. */
int mh_mass_solve_noalloc(mh_op* op, const double* f, double* c, void* stream);

/* One-body load vector f = H1 c in Galerkin form (Eq. discretized_eom):
 * length gauge H1(E) = K/2 + V_nuc + E (e.r); velocity gauge
 * H1(A) = K/2 + V_nuc - i A S_e, where the argument E is the vector
 * potential A(t) along e and S_e = sum_d e_d S_d, S_d the antisymmetric part
 * of the Gauss-Lobatto Galerkin derivative C^T D_d C (per cell
 * (h/2)^2 (Qs x W x W) along x, Qs = (W D - (W D)^T)/2 from the 1D
 * derivative matrix D and weights W; likewise along y and z; the A^2/2 term
 * is dropped, a spatial constant).  c: device c128 [N_E][n] (consistent);
 * f: device c128 [N][n]. */
int mh_h1_apply(mh_op* op, const double* c, double E, double* f, void* stream);

/* Pair Poisson solves (Sec. III.A): for every pair r <= s, solve
 * Laplace W_rs = -4 pi conj(phi_r) phi_s with Dirichlet values from the
 * multipole expansion (order lmax_bc, about the box centre) of the boundary
 * integral, by preconditioned CG on all pairs at once: the preconditioner is
 * the geometric multigrid V-cycle (Poisson schedule bit 4, the default and
 * the autotuner's choice on every workload measured) or the diagonal.
 * phi: device c128 [N_E][n] (consistent).
 * W:   device double [N_F][n*n] real columns, column order: for r = 0..n-1,
 *      s = r..n-1: (r == s) one column Re W_rr; (r < s) two columns Re W_rs,
 *      Im W_rs.  On entry W is the initial guess when `warm` != 0.
 * iters: host int32 [1] CG iterations taken (may be NULL).
 * Synchronises `stream`.  MH_NOT_CONVERGED if poisson_maxit is reached. */
int mh_poisson_pairs(mh_op* op, const double* phi, double* W, int32_t warm, int32_t* iters,
                     void* stream);

/* Reduced density matrices of a CI vector (Sec. II, spin-summed):
 * gamma_pq = <E_pq>, Gamma_pq,rs = <E_pq E_rs> - delta_qr gamma_ps.
 * Ci: device c128 [N_CI] (alpha-string major, strings ordered by bit mask);
 * gamma: device c128 [n][n]; Gamma: device c128 [n][n][n][n].  On a batch
 * handle each is one such block per instance ([n_inst][...]). */
int mh_ci_rdms(mh_op* op, const double* Ci, double* gamma, double* Gamma, void* stream);

/* Freeze G at t_n (Eqs. orb_eom, discretized_eom, packed_orb_eom with X = 0):
 * takes orbitals phi (device c128 [N_E][n]), RDMs (device c128, as above,
 * one block per instance on a batch handle), the field value E (times each
 * instance's field scale) and pair potentials W (device, layout of
 * mh_poisson_pairs); builds U_oq(x) = sum_rs Gamma_oq,rs W_rs(x), the
 * regularised gamma^{-1} and lam_qp = phi_q^H F_p(phi).  The frozen operator
 * is held by `op` until the next freeze.  MH_SINGULAR_RDM if gamma is not
 * positive after regularisation.  Synchronises `stream`. */
int mh_freeze(mh_op* op, const double* phi, const double* gamma, const double* Gamma, double E,
              const double* W, void* stream);

/* Frozen orbital right-hand side: (G v)_p = M^{-1} F_p(v) - sum_q lam_qp v_q,
 * F_p(v) = H1(E) v_p + C^T[m sum_q V_pq (C v_q)], V = gamma^{-1} U.
 * v, Gv: device c128 [N_E][n] (v consistent; Gv filled consistently). */
int mh_rhs_apply(mh_op* op, const double* v, double* Gv, void* stream);

/* Short-iterative Arnoldi step (Sec. III.B): phi <- exp(-i tau G) phi with
 * the frozen G, Krylov dimension m (<= 24), M-inner product over the packed
 * orbital vector, classical Gram-Schmidt with one re-orthogonalisation
 * (skipped when the first pass keeps at least a tenth of |w|),
 * happy breakdown at h_{k+1,k} <= 1e-14 |G v_k|.  tau = (tau_re, tau_im):
 * (dt, 0) real time, (0, -dtau) imaginary time.  err_est (host, may be
 * NULL) receives beta h_{m+1,m} |e_m^T expm(-i tau H_m) e_1|; m_used (host,
 * may be NULL) the Krylov dimension reached.  Synchronises when either host
 * pointer is non-NULL. */
int mh_arnoldi_step(mh_op* op, double* phi, double tau_re, double tau_im, int32_t m,
                    double* err_est, int32_t* m_used, void* stream);

/* Per-step observables written by mh_propagate, host arrays [n_steps + 1]
 * (dipole, energy, err_est, ortho: [n_steps + 1][n_inst], instance fastest). */
typedef struct {
  double* dipole;     /* sum_pq gamma_pq <phi_p|e.r|phi_q> */
  double* energy;     /* sum h gamma + 1/2 sum g Gamma + nuclear repulsion */
  double* err_est;    /* Arnoldi error estimate (0 for the final record) */
  double* ortho;      /* max |S - I|, S_pq = <phi_p|phi_q> */
  int32_t* cg_iters;  /* Poisson CG iterations (all instances iterate together) */
  double* momentum;   /* velocity form of the dipole: kinetic momentum along e,
                         sum_pq gamma_pq <phi_p|-i e.grad|phi_q> (+ N A(t) in the
                         velocity gauge), with the antisymmetric Gauss-Lobatto
                         derivative of the velocity-gauge term */
  int32_t* krylov_dim; /* Krylov dimension of each step's Arnoldi step (0 for the final record) */
} mh_observables;

/* Propagate orbitals and CI vector together for n_steps steps of size dt
 * (Sec. II Eqs. ci_eom / orb_eom with X = 0; Sec. III.B frozen-operator
 * exponential, first order): at t_n freeze G and the CI Hamiltonian from t_n
 * data with field E_steps[n], then phi <- exp(-i dt G) phi by Arnoldi (m)
 * and C <- exp(-i dt H_CI) C by Lanczos with min(12, N_CI) vectors.
 * flags: MH_PROP_IMAGINARY: dt is an imaginary-time step; orbitals are
 * then Gram-Schmidt orthonormalised in M and C normalised after every step.
 * MH_PROP_NO_FINAL: skip the final freeze at t_N (records [0, n_steps) only),
 * so that n_steps calls of one step do exactly n_steps freezes.
 * MH_PROP_GRAPH: capture the fixed launch sequence of a step that follows
 * the Poisson solve (freeze, integrals, observables, Arnoldi and CI steps)
 * once as a HIP graph on a stream of the library and replay it every step;
 * the Poisson CG, whose length depends on the data, stays eager.  Results
 * are those of the eager path.  Not with an adaptive Krylov dimension
 * (MH_INVALID_ARG).
 * MH_PROP_GRAPH_STEP (multigrid Poisson schedule, bit 4; not with
 * MH_PROP_GRAPH): from the fourth step of a call on, a whole step is one
 * replay of a HIP graph captured once per call: RDMs, the extrapolated CG
 * start, the pair Poisson solves with a fixed count of multigrid-
 * preconditioned CG iterations (three more than the third step took; no host
 * check inside the step), the boundary values, the step's field value from a
 * device copy of E_steps, then the step after the Poisson solve.  After each
 * replay the residual is checked on the host; a step whose CG stopped short
 * of the target makes the call return MH_NOT_CONVERGED (its records are
 * still filed).  The cg_iters record holds the fixed count for those steps.
 * phi: device c128 [N_E][n] in-out; Ci: device c128 [n_inst][N_CI] in-out;
 * E_steps: host double [n_steps + 1] (the last value is used for the final
 * record; in the velocity gauge these are values of A(t)); instance i sees
 * the field E0_i E_steps[k] (E0 = 1 for
 * mh_op_create).  obs: host arrays (any member may be NULL).  W_work: device
 * double [N_F][n*n] Poisson warm-start buffer (in-out, may hold zeros); the
 * first two steps of a call start CG from the previous solution (from W_work
 * at the first), the third from the linear extrapolation 2 W_n - W_{n-1} and
 * later steps from the quadratic extrapolation 3 W_n - 3 W_{n-1} + W_{n-2}
 * of the previous solutions.  MH_NONFINITE if an observable of a step is not
 * finite (NaN or Inf in the orbitals or CI vector).
 * Synchronises `stream`. */
enum { MH_PROP_IMAGINARY = 1, MH_PROP_NO_FINAL = 2, MH_PROP_GRAPH = 4, MH_PROP_GRAPH_STEP = 8 };
int mh_propagate(mh_op* op, double* phi, double* Ci, double* W_work, const double* E_steps,
                 int32_t n_steps, double dt, int32_t m, int32_t flags, mh_observables* obs,
                 void* stream);

/* Exact discrete adjoint of mh_propagate's dipole record with respect to
 * the field samples (reverse mode through the coupled orbital / CI steps of
 * Sec. II, Eqs. ci_eom and orb_eom with X = 0, and the first-order frozen
 * operator exponential of Sec. III.B).  Given g_n = dJ/dd_n for the record
 * d_0..d_N of mh_propagate (real time, same phi0, Ci0, E_steps, dt, m),
 * returns dJ/dE_k for k < N (E_N does not enter the dipoles).
 * Per step, backwards: the orbital adjoint nu (M-weighted, dJ = Re <nu, dc>_M)
 * is carried by exp(+i dt G^H), applied as the forward Arnoldi step of G with
 * its orbital mixing replaced and the orbitals conjugated by the regularised
 * 1-RDM; the CI adjoint kappa by exp(+i dt H_CI).  The Frechet derivatives
 * of both exponentials (n_quad-point Gauss-Legendre in s of
 * exp(-i(1-s)dt A) dA exp(-i s dt A)) give the sensitivities of the field,
 * of lambda, of the mean field V = gamma^-1 U and of the CI integrals h and g;
 * these are pushed back through U = Gamma W, through the pair Poisson solves
 * (one adjoint CG solve per step on all pair columns, with the transposed
 * multipole boundary lift) and the pair densities to the orbitals, and
 * through the RDMs to the CI vector.  Orbitals, CI vectors and pair
 * potentials are recomputed from checkpoints every ckpt_stride steps (<= 0:
 * round(sqrt(N))).  phi0: device c128 [N_E][n]; Ci0: device c128 [N_CI];
 * W_work: device double [N_F][n*n] warm-start buffer (overwritten);
 * E_steps: host [N + 1]; dJ_dd: host [N + 1]; dJ_dE: host out [N].
 * Allocates its checkpoint and work vectors per call.  MH_UNSUPPORTED for a
 * batch of several instances, more than 4 orbitals or more than 12
 * determinants (the CI exponential must be exact), or the velocity gauge;
 * MH_NOT_CONVERGED when a
 * Poisson solve stopped at the iteration cap (the gradient is still
 * returned).  Synchronises `stream`. */
int mh_propagate_adjoint(mh_op* op, const double* phi0, const double* Ci0, double* W_work,
                         const double* E_steps, int32_t n_steps, double dt, int32_t m,
                         const double* dJ_dd, double* dJ_dE, int32_t n_quad, int32_t ckpt_stride,
                         void* stream);

/* Sizes the caller needs to allocate device arrays. */
typedef struct {
  int64_t n_dof, n_ext, n_full, n_ci;
  int32_t n_orb, n_pair_cols;
  int64_t n_poisson_nnz;  /* entries of the assembled Poisson operator on the DoFs */
  int32_t n_inst;         /* instances in the handle (sizes above are batch totals) */
} mh_op_sizes;
int mh_op_sizes_get(const mh_op* op, mh_op_sizes* sizes);

/* Batch of independent instances sharing n_orb, n_alpha, n_beta, lmax_bc
 * and p (the many-molecule workload: one mesh and molecule per instance,
 * uneven sizes allowed).  meshes[i], descs[i]: as for mh_op_create;
 * field_scale: host [n_inst] (may be NULL = all 1): instance i sees the
 * field E0_i E.  Poisson tolerances and the RDM regularisation come from
 * descs[0].  The host set-up of the instances runs on several threads.
 * Every later call acts on all instances in the same kernel launches;
 * reductions are segmented per instance, and the CG, Arnoldi and Lanczos
 * scalars are per instance, so each instance evolves as it would alone
 * (up to the Chebyshev count of the interface mass solve, taken as the
 * largest over the batch, and the Poisson CG, which iterates until every
 * instance has converged).  Synchronises `stream`. */
int mh_batch_create(const mh_mesh* const* meshes, const mh_op_desc* descs, const double* field_scale,
                    int32_t n_inst, void* stream, mh_op** out);

/* Batch layout, host int64 [n_inst][6]: N, N_E, N_F, oE, oF, nnz of the
 * instance's assembled Poisson operator. */
int mh_batch_layout(const mh_op* op, int64_t* layout);

/* Timing hook for measurement: average duration (ms) of an operator kernel
 * over its launches since the last call, from HIP event pairs recorded on
 * the launch stream around each launch (no synchronisation while
 * recording; at most 4096 launches are recorded).  which: 0 = orbital
 * operator kernel (one-body + mean field), 1 = Poisson operator kernel.
 * enable: keep recording after this call.  Launches inside a captured
 * graph are not recorded.  Synchronises the device. */
int mh_kernel_timing(mh_op* op, int32_t which, int32_t enable, double* avg_ms, int64_t* count);

/* Launch schedule of an operator kernel, chosen by the autotuner.
 * which: 0 = orbital operator, 1 = Poisson operator.  sched bit 0: 1 =
 * XCD-contiguous sweep (XCD x of 8 owns a contiguous node range and its
 * workgroups walk it side by side), 0 = plain grid-stride sweep.  Orbital
 * only, sched bit 1: solve the interface block of the mass matrix by the
 * Chebyshev iteration even where the operator holds its dense inverse (a
 * single instance with at most 4096 interface unknowns holds one); bit 2:
 * the stiffness part of the orbital operator by the assembled Poisson
 * operator K~ applied to the 2n real columns of the orbitals (one sparse
 * pass with the Poisson schedule's long-row and sweep options), the node pass
 * adding only the diagonal and mean-field terms.  Poisson
 * only, sched bit 1: column blocking (16 columns per block on grid.z) when
 * the column count is a multiple of 16 and at least 32; bit 2: rows of the
 * assembled operator with more than 48
 * entries (hanging-node masters) taken by whole waves in reserved workgroups
 * of the same launch; bit 3: the CG direction formed inside the operator
 * pass (two launches per CG iteration instead of three; fewer launches, more
 * loads per entry); bit 4: CG preconditioned by the geometric multigrid
 * V-cycle instead of the diagonal (a hierarchy per instance, built on first
 * use; the V-cycles of a batch run level by level in shared launches); bit 5:
 * the rows of at most 48 entries read from a sliced-ELL copy of the operator
 * (built when the bit is first set: rows sorted by length within windows of
 * 4096, slices of 64 rows stored entry-major, so the lanes of a wave read
 * consecutive words), the longer rows by whole waves as with bit 2; bit 6
 * (with bit 4): the multigrid preconditioner's finest-level passes (smoothing,
 * residual and transfers) on float copies of their arrays (the residual, the
 * correction, the smoothing direction and the operator product); the CG
 * vectors, its own operator pass and every sum stay double, so the solution
 * meets the same residual target; bit 7 (with bit 1, when the number of
 * column blocks divides 8): the column blocks bound to XCDs, XCD x serving
 * block x mod the block count and the XCDs of one block splitting its rows
 * into contiguous ranges, so each XCD's L2 holds rows of one block only;
 * bits 8-9 (with bit 4): the degree of the Chebyshev smoothing on the finest
 * level before and after each coarse correction, 2 + their value (2 to 5;
 * more passes per cycle, fewer CG iterations); coarser levels smooth with
 * degree 2.
 * Default sched 13.  Allowed values: 0 to 7 (orbital); any combination of
 * bits 0 to 9 (Poisson).
 * grid_cap: maximum number of workgroups per instance (8..65536).  Results
 * do not depend on the schedule (the Poisson p.q partial sums change order
 * only). */
int mh_tune(mh_op* op, int32_t which, int32_t sched, int32_t grid_cap);

const char* mh_last_error(void);

/* Device workspace allocator.  The library's own device buffers (operator
 * tables, Krylov bases, CG and multigrid workspaces, adjoint scratch) come
 * from hipMalloc / hipFree unless an allocator is registered, e.g. a
 * framework's caching allocator, so that the library shares its memory pool.
 * alloc_fn(bytes, ctx) returns device memory of at least `bytes` bytes,
 * aligned to 256 bytes, or NULL on failure (the call that needed it then
 * returns MH_OOM); free_fn(ptr, bytes, ctx) returns it.  The registration is
 * process-wide and applies to allocations made after it; every buffer
 * records the pair that made it and is returned to that pair (on *_destroy,
 * or when a workspace is regrown), so the functions and ctx must stay valid
 * until every handle created while they were registered is destroyed.  Both
 * NULL restores hipMalloc / hipFree; exactly one NULL is MH_INVALID_ARG.  Not
 * to be called while another thread creates or runs a handle. */
typedef void* (*mh_alloc_fn)(size_t bytes, void* ctx);
typedef void (*mh_free_fn)(void* ptr, size_t bytes, void* ctx);
int mh_set_allocator(mh_alloc_fn alloc_fn, mh_free_fn free_fn, void* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MH_H */
