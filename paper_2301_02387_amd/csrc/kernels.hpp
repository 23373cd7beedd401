// Device kernels of the hot path and their host launchers (gfx950, wave64).
//
// Every launch covers a batch of independent instances (one molecule and
// mesh each; a plain operator is a batch of one).  Instance i runs in the
// workgroups with blockIdx.y == i and finds its mesh and operator data in
// DevMesh dm[i].  Batch arrays are the per-instance arrays laid end to end:
// instance i owns rows [oE, oE + NE) of every array over extended rows,
// [oF, oF + NF) of arrays over full rows and [oMa, oMa + nMa) of arrays over
// interface masters.  Small per-instance results (Krylov matrices, CG
// scalars, moments, RDMs, integrals) are stored instance-major with a fixed
// stride, and every reduction is segmented: its partial sums never mix
// instances.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mh {

// Read-only mesh/operator data of one instance, resident in HBM.
// Largest Chebyshev smoothing degree of the multigrid cycle (Poisson schedule
// bits 8-9 choose 2 + their value).
constexpr int MG_MAX_DEG = 5;

struct DevMesh {
  // this instance's convergence flag in a batch's multigrid CG (nonzero: the
  // CG and multigrid launches skip the instance); zero outside the CG
  const int* cg_done = nullptr;
  int P = 0, n = 0;                // nodes per cell edge, orbitals
  int inst = 0;                    // instance index (== blockIdx.y of its workgroups)
  int64_t nC = 0, N = 0, NE = 0, NF = 0, Nh = 0, Nb = 0, nMa = 0;
  int64_t oE = 0, oF = 0, oMa = 0;      // first row in batch arrays (extended / full / master rows)
  const int32_t* cell_nodes = nullptr;  // [nC][P^3]
  const double* cell_hh = nullptr;      // [nC] h/2
  const double* m = nullptr;            // [NF] Gauss-Lobatto full-node mass
  const double* v = nullptr;            // [NF] lumped nuclear potential
  const double* mz = nullptr;           // [NF] m (e.x)
  const double* xyz = nullptr;          // [NF][3]
  const int32_t* hang_ptr = nullptr;    // [Nh+1]
  const int32_t* hang_col = nullptr;    // library node index (DoF < N or boundary >= NE)
  const double* hang_w = nullptr;
  const int32_t* ma_index = nullptr;    // [N] master index or -1
  const int32_t* ma_dof = nullptr;      // [nMa] DoF of each master
  const int32_t* ma_ptr = nullptr;      // interface block CSR [nMa+1]
  const int32_t* ma_col = nullptr;
  const double* ma_val = nullptr;
  const double* ma_dinv = nullptr;
  const double* cheb = nullptr;         // 1/theta, then (c1, c2) per Chebyshev iteration
  const double* ma_inv = nullptr;       // dense inverse of the interface block [nMa][nMa] (single small instances)
  const int32_t* ct_ptr = nullptr;      // per master: hanging rows it constrains
  const int32_t* ct_row = nullptr;
  const double* ct_w = nullptr;
  const double* inv_mass = nullptr;     // [N] 1/m for non-masters
  const double* kdiag_inv = nullptr;    // [N]
  const int32_t* node_inc = nullptr;    // [NE][8]: cell*64 + local index of each incident cell, -1 padded
  const int32_t* kt_ptr = nullptr;      // assembled Poisson operator on DoFs (CSR)
  const int32_t* kt_col = nullptr;
  const double* kt_val = nullptr;
  const int32_t* kt_long = nullptr;      // rows of the assembled operator with more than KT_LONG entries
  int64_t n_long = 0;
  // sliced-ELL copy of the other rows (Poisson schedule bit 5, built on first use):
  // slices of SELL_H row slots, rows sorted by length within windows of SELL_WINDOW;
  // entry t of slot r of slice s at sell_ptr[s] + SELL_H t + r (widths are
  // multiples of 4; padding entries hold coefficient 0 and a valid column)
  const int32_t* sell_ptr = nullptr;    // [n_slices + 1]
  const int32_t* sell_row = nullptr;    // [n_slices][SELL_H] row of each slot, -1 for none
  const int32_t* sell_col = nullptr;
  const double* sell_val = nullptr;
  int64_t n_slices = 0;
  // the same values rounded to float, read by the passes of the multigrid
  // preconditioner's finest level on float storage (Poisson schedule bit 6);
  // the CG's own operator pass reads the double values
  const float* kt_valf = nullptr;
  const float* sell_valf = nullptr;
  const int32_t* bnd_cells = nullptr;
  int64_t n_bnd_cells = 0;
  const double* bnd_table = nullptr;    // [Nb][nharm] multipole boundary table
  double center[3] = {0.0, 0.0, 0.0};   // multipole expansion centre
  double E0 = 1.0;                      // field amplitude of this instance (E = E0 x the step's field value)
  // multigrid level-0 Chebyshev coefficients: s0 = 1/theta, then (c1, c2) of
  // steps 1 .. MG_MAX_DEG - 1 of the three-term recurrence
  double mgc[2 * MG_MAX_DEG - 1] = {};
  double vnn = 0.0;                     // nuclear repulsion
  // launch schedules (set by mh_tune): bit 0 = XCD-contiguous sweep; orbital bit 1 = interface
  // solve by Chebyshev even where a dense inverse is held, bit 2 = stiffness part by the
  // assembled operator; Poisson bit 1 =
  // column blocks of 16, bit 2 = long rows by whole waves, bit 3 = CG direction formed
  // inside the operator pass, bit 4 = geometric multigrid preconditioner (a
  // hierarchy per instance), bit 5 = short rows from the sliced-ELL copy (long
  // rows by waves); grid caps (per instance)
  int sched_orb = 1, sched_poi = 13, grid_orb = 65536, grid_poi = 8192;
  double A[16];                         // 1D stiffness (P x P, P <= 4)
  double w[4];                          // GLL weights
  double Qs[16];                        // antisymmetric 1D first-derivative form (P x P)
  double pol[3] = {0.0, 0.0, 1.0};      // unit field direction e
  int gauge = 0;                        // 0: length (E(t) e.r), 1: velocity (-i A(t) e.grad)
  // exterior complex scaling of the one-body operator (ecs != 0): the scaled
  // directions of each cell (bit d); per extended row (re, im) rho = m / m_theta,
  // rho times the continued lumped potential and the continued field weights
  // m (e.z); ecs_pw[k] = e^{i (k - 2) theta} (re, im), k = 0..5: a cell with s
  // scaled directions carries e^{i (s - 2 b_d) theta} on its stiffness along d
  // and e^{i (s - b_d) theta} on its derivative along d (b_d: d scaled)
  int ecs = 0;
  const uint8_t* ecs_code = nullptr;
  const double* ecs_rho = nullptr;
  const double* ecs_v = nullptr;
  const double* ecs_mz = nullptr;
  double ecs_pw[12] = {};
};

// Rows of the assembled Poisson operator longer than this are handled by whole
// workgroups (the masters of hanging nodes: tens to hundreds of entries).
constexpr int KT_LONG = 48;
constexpr int SELL_H = 64;
constexpr int SELL_WINDOW = 4096;

// A batch as seen by the launchers: the device array of instances, and a host
// record with the shared parameters and the largest per-instance sizes (grid
// shapes are taken from these; workgroups beyond an instance's size idle).
struct Batch {
  const DevMesh* dm = nullptr;  // device [ni]
  int ni = 1;
  DevMesh mx;                   // host: shared fields, per-class maximum sizes
  int64_t tE = 0, tF = 0, tMa = 0;  // batch totals of extended, full and master rows
  int cheb_iters = 0;           // Chebyshev iterations (the largest instance count)
  // one instance: the Poisson operator passes leave their per-workgroup p.q
  // (r.z) sums here, [workgroup][column], folded by a second small launch
  // instead of every workgroup adding into the same accumulators
  double* spart = nullptr;
  int64_t spart_cap = 0;        // doubles
};

// ---- orbital-space operator -------------------------------------------------
// Node-centric operator (no atomics); diag_mode 0: K/2 only, 1: + v + E mz
// (length gauge) or + v - i A S_e (velocity gauge, the field value being A),
// 2: + mean field, 3: mz only, 4: -i S_e only (momentum along e).  mode 0:
// load vector F; 1: M^-1 F; 2: M^-1 F - v lam.  Non-master DoFs are final in
// out; masters and hanging nodes go to acc.  E is read from the device scalar
// *Ef (times each instance's E0).  Orbital schedule bit 2: the stiffness part
// by the assembled K~ (kq, kred scratch); not taken where the velocity term
// or the momentum is applied (those run node by node).
void launch_stencil_orb(const Batch& b, const double* u, const double* Ef, int diag_mode, const double* Upk,
                        const double* ginv, int mode, const double* lam, double* out, double* acc, double* kq,
                        double* kred, hipStream_t s);
// Masters: acc_k + sum_h c_hk acc_h -> out (mode 0) or the interface rhs ma_b.
void launch_ma_gather_orb(const Batch& b, const double* acc, int mode, double* out, double* ma_b, hipStream_t s);
void launch_mass_direct(const Batch& b, const double* f, double* out, double* ma_b, hipStream_t s);
void launch_ma_solve(const Batch& b, const double* ma_b, double* x, double* r, double* dbuf0, double* dbuf1,
                     const double* v, const double* lam, double* out, hipStream_t s);
void launch_fill_orb(const Batch& b, double* x, double* acc, hipStream_t s);
// In-place Gauss-Jordan inverse of a dense SPD matrix [n][n] (no pivoting), 3 n launches.
void launch_dense_inverse(double* A, int64_t n, hipStream_t s);
void launch_copy(const double* in, double* out, int64_t nd, hipStream_t s);
void launch_axpby(int64_t nd, double a, const double* x, double b, double* y, hipStream_t s);
void launch_zero(double* out, int64_t nd, hipStream_t s);
void launch_set(double* out, double value, hipStream_t s);
void launch_set_indexed(double* out, const double* table, const int* ctr, hipStream_t s);  // out = table[*ctr]
void launch_counter(int* ctr, int set, int value, hipStream_t s);                        // *ctr = value or += value
// x <- 2 x - xprev and xprev <- the old x (linear extrapolation in time) over nd doubles
void launch_extrapolate(double* x, double* xprev, int64_t nd, hipStream_t s);
// x <- 3 x - 3 p1 + p2 (quadratic extrapolation in time), then p2 <- p1 and p1 <- the old x
void launch_extrapolate2(double* x, double* p1, double* p2, int64_t nd, hipStream_t s);

// ---- reductions (segmented per instance) -----------------------------------------
enum { ROWS_DOF = 0, ROWS_EXT = 1 };
enum { WT_NONE = 0, WT_MASS = 1, WT_DIPOLE = 2 };
int gram_blocks(int64_t rows);
// G_i[a][b] = sum over rows of instance i of wt conj(A[row][a]) B[row][b]
// (A, B batch orbital arrays [tE][n]); G instance stride n*n.
void launch_gram(const Batch& b, const double* A, const double* B, int wsel, int rows, double* part, int nblk,
                 double* G, hipStream_t s);
// Same on flat per-instance arrays of `rows` rows: X [ni][rows][na], Y [ni][rows][nb].
void launch_xgram_flat(int ni, const double* X, int na, const double* Y, int nb, int64_t rows, double* part,
                       int nblk, double* out, hipStream_t s);
int gint_blocks(const Batch& b);
void launch_gint_full(const Batch& b, const double* phi, const double* W, const int* colmap, double* part, int nblk,
                      double* Gtmp, double* g, hipStream_t s);
void launch_build_U_full(const Batch& b, const double* W, const double* Gamma, const int* colmap, double* Mr,
                         double* Upk, hipStream_t s);

// ---- Krylov ---------------------------------------------------------------------
struct Krylov {
  int m_max = 0;
  double* H = nullptr;       // device c128 [ni][(m_max+1) x m_max], H[i + (m_max+1) j]
  double* hcur = nullptr;    // device c128 [ni][m_max+1]
  double* scal = nullptr;    // [ni][8]: [0]=beta [1]=next scale [2]=|w|^2 [3]=err [4]=m_eff [5]=1/beta
  double* y = nullptr;       // device c128 [ni][m_max]
  double* part = nullptr;    // partial sums [ni][nblk][...]
  int nblk = 0;
};
void launch_norm_init(const Batch& b, const double* phi, Krylov& K, int m, hipStream_t s);
void launch_mdot(const Batch& b, double* const* V, int k, const double* w, Krylov& K, int pass, hipStream_t s);
void launch_orth_update(const Batch& b, double* const* V, int k, double* w, Krylov& K, int pass, hipStream_t s);
// The first CGS2 update fused with the second pass's dots (w -= V hcur, then
// V^H M w finished into H and hcur as the second pass of launch_mdot).
void launch_orth_dot(const Batch& b, double* const* V, int k, double* w, Krylov& K, hipStream_t s);
void launch_krylov_scale(const Batch& b, const double* src, double* dst, Krylov& K, int which, hipStream_t s);
void launch_expm(int ni, Krylov& K, double tau_re, double tau_im, hipStream_t s);
// Adaptive dimension: where the error estimate of dimension m_try meets tol,
// the instance's dimension (scal[4]) becomes m_try.
void launch_krylov_check(int ni, Krylov& K, double tau_re, double tau_im, int m_try, double tol, hipStream_t s);
void launch_combine(const Batch& b, double* const* V, int m, double* phi, Krylov& K, hipStream_t s);

// ---- Poisson ---------------------------------------------------------------------
// Column arrays are real [rows][ncol]: acc, p, r, q over extended rows (batch
// offset oE), the potentials W over full rows (offset oF).
struct PoissonWs {
  int ncol = 0, nharm = 0, lmax = 0;
  double* acc = nullptr;   // [tE][ncol]
  double* p = nullptr;     // [tE][ncol] search direction (two buffers, alternating by iteration)
  double* p2 = nullptr;
  double* r = nullptr;     // [tE][ncol]
  double* q = nullptr;     // [tE][ncol]
  double* sc = nullptr;    // [ni][8][ncol] scalars
  double* red = nullptr;   // [ni][RED_SLOTS][ncol] atomic accumulators (rz x3, pq x2, rr x2; see stencil.hip)
  int it = 0;              // CG iteration within the running solve
  double* part = nullptr;  // partials [ni][grid][2 ncol]
  int64_t part_stride = 0;
  double* Q = nullptr;     // moments [ni][nharm][ncol]
  double* mpart = nullptr; // moment partials [ni][mblk][nharm ncol]
  int mblk = 0;
  // optional timing of the operator kernel: event pairs recorded on the
  // launch stream around each launch, read after the timed region
  hipEvent_t* ev = nullptr;
  int ev_cap = 0, ev_used = 0;
};
enum { SC_RZ = 0, SC_PQ = 1, SC_ALPHA = 2, SC_BETA = 3, SC_RR = 4, SC_BB = 5, SC_RZN = 6 };
// accumulator slots: r.D^-1 r of iteration k in RED_RZ + k % 3, p.q in RED_PQ + k % 2,
// r.r after iteration k in RED_RR + k % 2
enum { RED_RZ = 0, RED_PQ = 3, RED_RR = 5, RED_SLOTS = 8 };
// slot of r.r after the last iteration of a solve that took `it` iterations (it >= 1)
inline int red_rr_slot(int it) { return RED_RR + (it - 1) % 2; }
void launch_poisson_pipeline_moments(const Batch& b, const double* phi, const int* colinfo, PoissonWs& P,
                                     hipStream_t s);
void launch_bnd_eval(const Batch& b, PoissonWs& P, double* W, hipStream_t s);
void launch_poisson_rhs_full(const Batch& b, const double* phi, double* W, const int* colinfo, double* rhs,
                             PoissonWs& P, hipStream_t s);
void launch_cg_start(const Batch& b, double* W, double* rhs_r, PoissonWs& P, int warm, hipStream_t s);
void launch_cg_step(const Batch& b, double* W, PoissonWs& P, hipStream_t s);
// Pieces of a CG iteration with another preconditioner: q = K p with p.q into
// slot RED_PQ + k % 2, and the update pass (alpha_k = red[RED_RZ + k % 3] / p.q).
void launch_cg_apply_plain(const Batch& b, PoissonWs& P, const double* p, int k, hipStream_t s);
// rf (may be null): a float copy of the updated residual (Poisson schedule bit 6)
// Batch CG convergence flags (DevMesh::cg_done, device int [ni]): set an
// instance's flag once every column's r.r after iteration k is at most
// rtol^2 times its largest column's b.b; clear all flags.
void launch_cg_done(const Batch& b, const PoissonWs& P, int k, double rtol, hipStream_t s);
void launch_zero_int(int* x, int n, hipStream_t s);
// upd_x = 0: the x += alpha p of this iteration is left to the next direction
// pass (mg_dir with x) or to cg_xfinal after the last iteration.
void launch_cg_update(const Batch& b, double* W, PoissonWs& P, const double* p, int k, hipStream_t s,
                      float* rf = nullptr, int upd_x = 1);
void launch_to_float(const double* x, float* y, int64_t nd, hipStream_t s);
// Multigrid-preconditioned CG on the finest level, in operator passes (the
// Chebyshev coefficients are each instance's DevMesh::mgc; red: the CG
// accumulators [ni][RED_SLOTS][ncol]):
//  - the first two smoothing steps from z = 0 (z and d from r); clears red slot
//    rz_slot & 255; d is not stored when bit 8 of rz_slot is set (degree 2:
//    no third step reads it);
//  - smoothing step k (0 .. degree - 1) from zin into zout (d updated in
//    place); with rz_slot >= 0 (the last step after the coarse correction)
//    it also accumulates r.zout into that slot and leaves d alone.
void launch_mg_cheb0(const Batch& b, const double* r, double* z, double* d, double* red, int rz_slot, int ncol,
                     hipStream_t s);
void launch_mg_cheb_step(const Batch& b, const double* zin, const double* r, double* zout, double* d, double* red,
                         int ncol, int k, int rz_slot, hipStream_t s);
//  - the residual t = r - K z that the restriction to the next level reads
//    (red_scratch: accumulators the pass may touch, not the CG's).
void launch_mg_resid(const Batch& b, const double* z, const double* r, double* t, int ncol, double* red_scratch,
                     hipStream_t s);
// Poisson schedule bit 6: the finest multigrid level's passes on float arrays
void launch_mg_cheb0_f(const Batch& b, const float* r, float* z, float* d, double* red, int rz_slot, int ncol,
                       hipStream_t s);
void launch_mg_cheb_step_f(const Batch& b, const float* zin, const float* r, float* zout, float* d, double* red,
                           int ncol, int k, int rz_slot, hipStream_t s);
void launch_mg_resid_f(const Batch& b, const float* z, const float* r, float* t, int ncol, double* red_scratch,
                       hipStream_t s);
// Hanging rows of a real column array (xfull: x is over full rows, else extended).
void launch_fill_real(const Batch& b, double* x, int xfull, int ncol, int with_bnd, double* acc, hipStream_t s);

// ---- small dense work (one workgroup per instance) ------------------------------------
void launch_ginv(int ni, const double* gamma, int n, double eps, double* ginv, int* flag, hipStream_t s);
void launch_observe(const Batch& b, const double* gamma, const double* Gamma, const double* h, const double* g,
                    const double* zmat, const double* S, const double* pmat, const double* Ef, double* out,
                    hipStream_t s);
void launch_orthonormalize_full(const Batch& b, const double* S, double* Rinv, double* x, hipStream_t s);

// ---- CI (one space shared by the instances; vectors [ni][dim]) ---------------------------
struct CIDev {
  int n = 0, NA = 0, NB = 0, dim = 0;
  const int32_t* exa = nullptr;  // [NA][n*n]: I | (sign<0)<<30 with E_pq|I> = sign|J>, or -1
  const int32_t* exb = nullptr;  // [NB][n*n]
  double* D = nullptr;           // [ni][dim][n*n] c128
  double* T = nullptr;           // [ni][dim][n*n] c128
  double* hp = nullptr;          // h' [ni][n*n] c128
  double* part = nullptr;
  double* w = nullptr;           // [ni][dim] c128
};
void launch_ci_rdm_full(int ni, const CIDev& c, const double* C, double* gamma, double* Gamma, double* Gtmp,
                        hipStream_t s);
void launch_ci_hprime(int ni, const CIDev& c, const double* h, const double* g, hipStream_t s);
void launch_ci_lanczos(int ni, const CIDev& c, double* const* Qdev, double* const* Qhost, int m, const double* g,
                       double* Cvec, Krylov& K, double tau_re, double tau_im, int normalize, hipStream_t s);
void launch_ci_trdm(int ni, const CIDev& c, const double* A, const double* Bv, double* DA, double* DB,
                    double* gamma, double* Gamma, double* Gtmp, hipStream_t s);
void launch_ci_apply(int ni, const CIDev& c, const double* h, const double* g, const double* C, double* sigma,
                     hipStream_t s);

}  // namespace mh
