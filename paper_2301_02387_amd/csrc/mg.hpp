// Geometric multigrid preconditioner of the pair Poisson solves (mg.hip):
// per-instance hierarchies and the V-cycle over a whole batch.  Every pass over
// a level covers all instances in one launch (instance blockIdx.y); real
// [rows][ncol] arrays.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <vector>

namespace mh {

// Chebyshev smoothing interval [lmax / MG_RANGE, lmax] of D^-1 A
constexpr double MG_RANGE = 8.0;
constexpr int MG_RZ_BLOCKS = 256;

// One level of one instance.  `active`: smoothing and transfers run on this
// level (it is not the instance's coarsest); `coarse`: the level is the
// instance's coarsest, solved with the dense inverse cinv.
struct MgLevelDev {
  int64_t N = 0;                                                   // unknowns of the level
  int active = 0, coarse = 0;
  const int32_t* a_ptr = nullptr; const int32_t* a_col = nullptr;   // operator (CSR)
  const double* a_val = nullptr;
  const double* dinv = nullptr;                                    // 1 / diagonal
  double lmax = 0.0;                                               // bound of the spectrum of D^-1 A
  const int32_t* p_ptr = nullptr; const int32_t* p_col = nullptr;   // prolongation from level + 1 (rows N)
  const double* p_val = nullptr;
  const int32_t* r_ptr = nullptr; const int32_t* r_col = nullptr;   // restriction to level + 1 (its rows)
  const double* r_val = nullptr;
  const double* cinv = nullptr;                                    // dense inverse (coarse levels)
  double* r = nullptr;   // right-hand side [N][ncol] (level 0: the batch residual at this instance)
  double* z = nullptr;   // correction
  double* d = nullptr;   // Chebyshev direction
  double* t = nullptr;   // operator product scratch
  // level 0 on float storage (Poisson schedule bit 6): the residual copy, the
  // correction and the operator product the transfers read and write
  int f32 = 0;
  const int* done = nullptr;  // the instance's CG convergence flag (nonzero: skip)
  const float* rf = nullptr;
  float* zf = nullptr;
  float* tf = nullptr;
};

// The batch hierarchy: lv[l] = device array [ni] of level-l records (an
// instance with fewer levels has inactive records there); coarse = device
// array [ni] of each instance's coarsest level.  z0, t0: batch arrays of level
// 0 (extended-row layout, instance offsets as every Poisson array).
struct MgDev {
  int nlev = 0;
  std::vector<MgLevelDev*> lv;
  MgLevelDev* coarse = nullptr;
  int64_t max_n[32] = {};   // largest N of each level over the instances (grid shapes)
  int64_t max_coarse = 0;
  double* z0 = nullptr;
  double* z0b = nullptr;    // second level-0 correction array (the fused smoothing steps alternate)
  double* t0 = nullptr;
  double* d0 = nullptr;
  // the same level-0 arrays in float, with the float copy of the residual (schedule bit 6)
  float* z0f = nullptr;
  float* z0bf = nullptr;
  float* t0f = nullptr;
  float* d0f = nullptr;
  float* rf = nullptr;
  MgLevelDev* lv0_double = nullptr;  // device [ni] level-0 records on double / float storage
  MgLevelDev* lv0_float = nullptr;
  int nu = 2;               // finest level's smoothing steps before and after the coarse correction (Chebyshev degree)
};
// Level-0 passes over the batch (batch arrays): the residual t0 = r0 - A z0
// that the restriction reads, and the smoothing steps fused into the
// operator pass (degree nu >= 2): the two steps from zero (z0, d0 from r0),
// and step k (from the current correction into the other buffer; rz: the
// last step after the coarse correction, which also accumulates r.z).  The
// caller keeps the correction in z0 wherever the cycle reads it (residual
// pass, prolongation).
struct MgLevel0Ops {
  std::function<void(hipStream_t s)> resid;
  std::function<void(hipStream_t s)> cheb0;
  std::function<void(int k, bool rz, hipStream_t s)> cheb;
};

// z0 = B r0 for one symmetric V-cycle per instance (r0: the batch residual)
void mg_vcycle(const MgDev& mg, int ni, int ncol, const MgLevel0Ops& ops, hipStream_t s);
// red[i][slot][c] = sum over instance i's DoF rows of r[][c] z[][c] (part:
// ni * MG_RZ_BLOCKS * ncol doubles); dm: the batch instance records
struct DevMesh;
void mg_rz(const DevMesh* dm, int ni, int ncol, const double* r, const double* z, double* part, double* red,
           int slot, hipStream_t s);
// pcur = z + beta pprev per instance and column, beta = red[rz_cur] / red[rz_prev]
// (rz_prev < 0: beta = 0); clears red[rr_clear].  With x (not null, rz_prev >= 0):
// also the previous iteration's deferred x += (red[rz_prev] / red[pq_prev]) pprev.
void mg_dir(const DevMesh* dm, int ni, int64_t max_n, int ncol, const double* z, const double* pprev, double* pcur,
            double* red, int rz_cur, int rz_prev, int rr_clear, double* x, int pq_prev, hipStream_t s);
void mg_dir(const DevMesh* dm, int ni, int64_t max_n, int ncol, const float* z, const double* pprev, double* pcur,
            double* red, int rz_cur, int rz_prev, int rr_clear, double* x, int pq_prev, hipStream_t s);
// x += (red[rz_slot] / red[pq_slot]) p: the deferred update of the last iteration
void cg_xfinal(const DevMesh* dm, int ni, int64_t max_n, int ncol, double* x, const double* p, const double* red,
               int rz_slot, int pq_slot, hipStream_t s);

}  // namespace mh
