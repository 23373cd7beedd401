// Host-side data of the octree mesh and the operator set-up.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace mh {

// Gauss-Lobatto-Legendre nodes/weights on [-1,1], the 1D stiffness
// A_ab = sum_q w_q l_a'(x_q) l_b'(x_q) (Sec. III.A element basis/quadrature)
// and the antisymmetric part of the 1D first-derivative form,
// Qs_ab = (w_a l_b'(x_a) - w_b l_a'(x_b)) / 2 (velocity-gauge term).
struct Gll {
  int p = 0;
  std::vector<double> x, w, A, Qs;  // A, Qs row-major (p+1)^2
};
Gll make_gll(int p);
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);  // on [-1,1]
double lagrange(const std::vector<double>& nodes, int a, double x);

struct Ball {
  double c[3];
  double r;
  int levels;
};

struct Nucleus {
  double Z;
  double R[3];
};

// Kelly refinement request (Sec. III.A): leaves are halved while the Kelly
// indicator of the softened nuclear potential exceeds tol, up to max_level.
struct KellyReq {
  std::vector<Nucleus> nuclei;  // empty: no Kelly refinement
  double tol = 0.0, soft = 0.0;
  int max_level = 0;
};

struct Mesh {
  double lo = 0, hi = 0, H = 0;
  int nc = 0, p = 0, P = 0, Lmax = 0;
  int64_t n_cells = 0;
  std::vector<int32_t> cell_level;
  std::vector<int64_t> cell_ijk;     // 3 per cell
  std::vector<double> cell_h;        // edge length
  std::vector<double> cell_org;      // 3 per cell (lower corner)
  std::vector<int32_t> cell_nodes;   // n_cells * P^3, library node index
  int64_t nF = 0, N = 0, Nh = 0, Nb = 0;
  std::vector<double> xyz;           // nF * 3
  std::vector<int64_t> hang_ptr;     // Nh + 1 (row h <-> node N + h)
  std::vector<int64_t> hang_col;     // library node index of master (DoF or boundary)
  std::vector<double> hang_w;
  std::vector<int32_t> masters;      // DoF masters, ascending
  std::vector<int64_t> level_counts;
  std::vector<Ball> balls;           // the refinement request the mesh was built from
  KellyReq kelly;
  int kelly_rounds = 0;              // Kelly refinement rounds taken
  Gll gll;
};

// Returns "" on success, else an error message; `unsupported` set for
// configurations the library refuses (hanging node on the boundary, ...).
// kelly: optional Kelly refinement after the balls; level_cap >= 0: leaves
// deeper than level_cap are then replaced by their ancestors at that level;
// from: start from that mesh's leaves (same box) instead of the coarse cubes.
// The coarser multigrid levels of a Kelly mesh are its own leaves capped
// (from = the fine mesh), so each nests in the one above.
std::string build_mesh(double lo, double hi, int nc, int p, const std::vector<Ball>& balls,
                       Mesh& out, bool& unsupported, const KellyReq* kelly = nullptr, int level_cap = -1,
                       const Mesh* from = nullptr);

// Operator tables computed on the host at set-up.
// Exterior complex scaling of the one-body operator (Sec. IV absorber):
// coordinates beyond |x_d| = inner[d] continue along x_d -> sign(x_d) inner[d]
// + e^{i theta} (x_d - sign(x_d) inner[d]); theta = 0 leaves them real.
struct EcsReq {
  double theta = 0.0;
  double inner[3] = {0.0, 0.0, 0.0};
};

struct OpHost {
  std::vector<double> m, v, mz;            // nF: mass, lumped nuclear potential, m*(e.x)
  // complex scaling (ecs): the scaled directions of each cell (bit d), and per
  // extended row (re, im) the factor rho = m / m_theta, rho times the continued
  // lumped potential, and the continued field weights m (e.z)
  bool ecs = false;
  double ecs_theta = 0.0;
  std::vector<uint8_t> ecs_code;           // nC
  std::vector<double> ecs_rho, ecs_v, ecs_mz;  // NE x 2
  std::vector<uint64_t> owner_mask;        // per cell: local nodes whose diagonal terms it adds
  std::vector<int32_t> node_inc;           // NE x 8: cell*64 + local index of each incident cell, -1 padded
  // interface (hanging-master) block of the mass matrix, rows = masters
  std::vector<int32_t> ma_index;           // N: index into masters or -1
  std::vector<int32_t> ma_dof;             // DoF of each interface unknown (reverse Cuthill-McKee order)
  std::vector<int32_t> ma_ptr, ma_col;     // CSR over masters (columns = master index)
  std::vector<double> ma_val;
  std::vector<double> ma_dinv;             // 1 / diagonal
  double cheb_lo = 1, cheb_hi = 1;         // spectrum bounds of D^-1 A_Ma
  int cheb_iters = 0;
  std::vector<int32_t> ct_ptr, ct_row;     // per master: hanging rows (library index) constrained by it
  std::vector<double> ct_w;
  std::vector<double> inv_mass;            // N: 1/m_k for non-masters (0 for masters)
  // assembled Poisson operator C^T K_full C on the DoFs (homogeneous boundary), CSR
  std::vector<int32_t> kt_ptr, kt_col;
  std::vector<double> kt_val;
  std::vector<double> kdiag_inv;           // N: 1/diag(C^T K_full C)
  std::vector<int32_t> bnd_cells;          // cells touching boundary values
  std::vector<double> bnd_table;           // Nb x nharm multipole evaluation table
  int nharm = 0;
};

// ecs: complex scaling of the one-body operator (null or theta = 0: none);
// throws std::invalid_argument for a cell straddling a scaling plane, a
// nucleus outside the unscaled cuboid, or a hanging node or master touching a
// scaled cell.
void build_operator(const Mesh& mesh, const std::vector<Nucleus>& nuc, const double pol[3],
                    int lmax, OpHost& op, const EcsReq* ecs = nullptr);

// Geometric multigrid hierarchy for the assembled pair Poisson operator
// (homogeneous Dirichlet problem on the DoFs).  Level 0 is the operator's own
// mesh; level 1 is Q1 on the same leaves; then Q1 with every ball one level
// shallower, down to the uniform base grid; then base grids of half the cells
// per edge while the interior is larger than `max_coarse`.  The spaces are
// nested, so the prolongation is nodal interpolation of the coarse function at
// the fine DoF nodes (coarse hanging nodes expanded through their constraints,
// coarse boundary nodes zero) and the restriction its transpose.
struct MgLevel {
  int64_t N = 0;                           // DoFs
  std::vector<int32_t> k_ptr, k_col;       // operator (CSR over DoFs)
  std::vector<double> k_val, dinv;         // values, 1 / diagonal
  double lmax = 0;                         // largest eigenvalue of D^-1 K (power iteration, x 1.05)
  std::vector<int32_t> p_ptr, p_col;       // prolongation from level l+1: rows = DoFs of l
  std::vector<double> p_val;
  std::vector<int32_t> r_ptr, r_col;       // restriction to level l+1 (transpose): rows = DoFs of l+1
  std::vector<double> r_val;
};
struct MgHost {
  std::vector<MgLevel> lv;                 // lv[0] finest ... lv.back() coarsest
  std::vector<double> coarse_dense;        // the coarsest operator, dense row-major
};
// Levels stop at the first with at most max_coarse unknowns (or at the
// coarsest base grid of the plan).
void build_multigrid(const Mesh& fine, const OpHost& fop, MgHost& mg, int max_coarse = 400);

// Multipole harmonics shared by set-up and kernels: the order of the
// (l, m, cos/sin) terms.  Term count for lmax: (lmax+1)^2.
int multipole_terms(int lmax);

}  // namespace mh
