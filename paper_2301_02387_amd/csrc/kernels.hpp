// Device kernels of the hot path and their host launchers (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mh {

// Read-only mesh/operator data resident in HBM.
struct DevMesh {
  int P = 0, n = 0;                // nodes per cell edge, orbitals
  int64_t nC = 0, N = 0, NE = 0, NF = 0, Nh = 0, Nb = 0, nMa = 0;
  const int32_t* cell_nodes = nullptr;  // [nC][P^3]
  const double* cell_hh = nullptr;      // [nC] h/2
  const uint64_t* owner = nullptr;      // [nC] bit mask of owned local nodes
  const double* m = nullptr;            // [NF] Gauss-Lobatto full-node mass
  const double* v = nullptr;            // [NF] lumped nuclear potential
  const double* mz = nullptr;           // [NF] m (e.x)
  const int32_t* hang_ptr = nullptr;    // [Nh+1]
  const int32_t* hang_col = nullptr;    // library node index (DoF < N or boundary >= NE)
  const double* hang_w = nullptr;
  const int32_t* ma_index = nullptr;    // [N] master index or -1
  const int32_t* ma_dof = nullptr;      // [nMa] DoF of each master
  const int32_t* ma_ptr = nullptr;      // interface block CSR [nMa+1]
  const int32_t* ma_col = nullptr;
  const double* ma_val = nullptr;
  const double* ma_dinv = nullptr;
  const int32_t* ct_ptr = nullptr;      // per master: hanging rows it constrains
  const int32_t* ct_row = nullptr;
  const double* ct_w = nullptr;
  const double* inv_mass = nullptr;     // [N] 1/m for non-masters
  const double* kdiag_inv = nullptr;    // [N]
  const int32_t* node_inc = nullptr;    // [NE][8]: cell*64 + local index of each incident cell, -1 padded
  const int32_t* kt_ptr = nullptr;      // assembled Poisson operator on DoFs (CSR)
  const int32_t* kt_col = nullptr;
  const double* kt_val = nullptr;
  const int32_t* bnd_cells = nullptr;
  int64_t n_bnd_cells = 0;
  // launch schedules (set by mh_tune): bit 0 = XCD-contiguous sweep; grid caps
  int sched_orb = 1, sched_poi = 1, grid_orb = 65536, grid_poi = 8192;
  double A[16];                         // 1D stiffness (P x P, P <= 4)
  double w[4];                          // GLL weights
};

// ---- orbital-space operator -------------------------------------------------
// Node-centric operator (no atomics); diag_mode 0: K/2 only, 1: + v + E mz,
// 2: + mean field.  mode 0: load vector F; 1: M^-1 F; 2: M^-1 F - v lam.
// Non-master DoFs are final in out; masters and hanging nodes go to acc.
void launch_stencil_orb(const DevMesh& d, const double* u, double E, int diag_mode, const double* Upk,
                        const double* ginv, int mode, const double* lam, double* out, double* acc, hipStream_t s);
// Masters: acc_k + sum_h c_hk acc_h -> out (mode 0) or the interface rhs ma_b.
void launch_ma_gather_orb(const DevMesh& d, const double* acc, int mode, double* out, double* ma_b, hipStream_t s);
void launch_mass_direct(const DevMesh& d, const double* f, double* out, double* ma_b, hipStream_t s);
int launch_stencil_poisson(const DevMesh& d, const double* x, int ncol, double* q, double* acc, double* part,
                           hipStream_t s);
// Former scatter form (FP64 atomics), kept for the boundary-lift pass only.
// acc[node] += (K/2 + diag) u; diag_mode 0: none, 1: v + E mz, 2: + mean field
void launch_cell_orb(const DevMesh& d, const double* u, double* acc, double E, int diag_mode, const double* Upk,
                     const double* ginv, hipStream_t s);
// DoF epilogue.  mode 0: out = C^T acc (load vector); 1: out = M^-1 (C^T acc)
// on non-masters and master rhs into ma_b; 2: as 1 minus sum_q lam_qp v_q.
void launch_epi_orb(const DevMesh& d, double* acc, int mode, const double* v, const double* lam, double* out,
                    double* ma_b, hipStream_t s);
void launch_ma_solve(const DevMesh& d, const double* ma_b, double* x, double* r, double* dbuf0, double* dbuf1,
                     double lo, double hi, int iters, const double* v, const double* lam, double* out,
                     hipStream_t s);
void launch_fill_orb(const DevMesh& d, double* x, double* acc, hipStream_t s);
void launch_copy(const double* in, double* out, int64_t nd, hipStream_t s);
void launch_axpby(int64_t nd, double a, const double* x, double b, double* y, hipStream_t s);
void launch_zero(double* out, int64_t nd, hipStream_t s);

// ---- reductions ----------------------------------------------------------------
int gram_blocks(int64_t rows);
void launch_xgram(const double* X, int na, const double* Y, int nb, int yreal, const double* wt, int64_t rows,
                  double* part, int nblk, double* out, hipStream_t s);
void launch_gram(const double* a, const double* b, const double* wt, int64_t rows, int n, double* part,
                 int nblk, double* G, hipStream_t s);
int gint_blocks(const DevMesh& d);
void launch_gint_full(const DevMesh& d, const double* phi, const double* W, const int* colmap, double* part,
                      int nblk, double* Gtmp, double* g, hipStream_t s);
void launch_build_U_full(const DevMesh& d, const double* W, const double* Gamma, const int* colmap, double* Mr,
                         double* Upk, hipStream_t s);

// ---- Krylov ---------------------------------------------------------------------
struct Krylov {
  int m_max = 0;
  double* H = nullptr;       // device c128 [(m_max+1) x m_max], H[i + (m_max+1) j]
  double* hcur = nullptr;    // device c128 [m_max+1]
  double* scal = nullptr;    // [0]=beta [1]=next scale [2]=|w|^2 [3]=err [4]=m_eff [5]=1/beta
  double* y = nullptr;       // device c128 [m_max]
  double* part = nullptr;    // partial sums
  int nblk = 0;
};
void launch_norm_init(const DevMesh& d, const double* phi, Krylov& K, int m, hipStream_t s);
void launch_mdot(const DevMesh& d, double* const* V, int k, const double* w, Krylov& K, int pass, hipStream_t s);
void launch_orth_update(const DevMesh& d, double* const* V, int k, double* w, Krylov& K, int pass,
                        hipStream_t s);
void launch_krylov_scale(const DevMesh& d, const double* src, double* dst, Krylov& K, int which, int k,
                         hipStream_t s);
void launch_expm(Krylov& K, int m, double tau_re, double tau_im, hipStream_t s);
void launch_combine(const DevMesh& d, double* const* V, int m, double* phi, Krylov& K, hipStream_t s);

// ---- Poisson ---------------------------------------------------------------------
struct PoissonWs {
  int ncol = 0, nharm = 0, lmax = 0;
  double* acc = nullptr;   // [NE][ncol]
  double* p = nullptr;     // [NE][ncol]
  double* r = nullptr;     // [N][ncol]
  double* q = nullptr;     // [N][ncol]
  double* sc = nullptr;    // [8][ncol] scalars
  double* part = nullptr;  // partials
  double* part2 = nullptr; // partials of the master gather
  double* Q = nullptr;     // moments [nharm][ncol]
  double* mpart = nullptr; // moment partials
  int mblk = 0;
  const double* table = nullptr;  // [Nb][nharm]
  double center = 0;
  // optional timing of the stiffness (cell) kernel: event pairs recorded on
  // the launch stream around each launch, read after the timed region
  hipEvent_t* ev = nullptr;
  int ev_cap = 0, ev_used = 0;
};
enum { SC_RZ = 0, SC_PQ = 1, SC_ALPHA = 2, SC_BETA = 3, SC_RR = 4, SC_BB = 5, SC_RZN = 6 };
void launch_poisson_pipeline_moments(const DevMesh& d, const double* phi, const double* xyz, const int* colinfo,
                                     PoissonWs& P, hipStream_t s);
void launch_bnd_eval(const DevMesh& d, PoissonWs& P, double* W, hipStream_t s);
void launch_poisson_rhs_full(const DevMesh& d, const double* phi, double* W, const int* colinfo, double* rhs,
                             PoissonWs& P, hipStream_t s);
void launch_cg_start(const DevMesh& d, double* W, double* rhs_r, PoissonWs& P, int warm, hipStream_t s);
void launch_cg_step(const DevMesh& d, double* W, PoissonWs& P, hipStream_t s);
void launch_fill_real(const DevMesh& d, double* x, int ncol, int with_bnd, double* acc, hipStream_t s);
void launch_cell_poisson(const DevMesh& d, const double* x, double* acc, int ncol, int lift, hipStream_t s);

// ---- small dense work ----------------------------------------------------------------
void launch_ginv(const double* gamma, int n, double eps, double* ginv, int* flag, hipStream_t s);
void launch_observe(const double* gamma, const double* Gamma, const double* h, const double* g,
                    const double* zmat, const double* S, int n, double vnn, double* out, hipStream_t s);
void launch_orthonormalize_full(const DevMesh& d, const double* S, double* Rinv, double* x, hipStream_t s);

// ---- CI --------------------------------------------------------------------------------
struct CIDev {
  int n = 0, NA = 0, NB = 0, dim = 0;
  const int32_t* exa = nullptr;  // [NA][n*n]: I | (sign<0)<<30 with E_pq|I> = sign|J>, or -1
  const int32_t* exb = nullptr;  // [NB][n*n]
  double* D = nullptr;           // [dim][n*n] c128
  double* T = nullptr;           // [dim][n*n] c128
  double* hp = nullptr;          // h' [n*n] c128
  double* part = nullptr;
  double* w = nullptr;           // [dim] c128
};
void launch_ci_D(const CIDev& c, const double* C, hipStream_t s);
void launch_ci_rdm_full(const CIDev& c, const double* C, double* gamma, double* Gamma, double* Gtmp, hipStream_t s);
void launch_ci_hprime(const CIDev& c, const double* h, const double* g, hipStream_t s);
void launch_ci_sigma(const CIDev& c, const double* C, const double* g, double* sigma, hipStream_t s);
void launch_ci_lanczos(const CIDev& c, double* const* Qdev, double* const* Qhost, int m, const double* g,
                       double* Cvec, Krylov& K, double tau_re, double tau_im, int normalize, hipStream_t s);

}  // namespace mh
