// Geometric multigrid preconditioner of the pair Poisson solves (mg.hip):
// device levels and the V-cycle.  One instance; real [rows][ncol] arrays.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <vector>

namespace mh {

// Chebyshev smoothing interval [lmax / MG_RANGE, lmax] of D^-1 A
constexpr double MG_RANGE = 8.0;
constexpr int MG_RZ_BLOCKS = 256;

struct MgLevelDev {
  int64_t N = 0;                                                   // unknowns of the level
  const int32_t* a_ptr = nullptr; const int32_t* a_col = nullptr;   // operator (CSR)
  const double* a_val = nullptr;
  const double* dinv = nullptr;                                    // 1 / diagonal
  double lmax = 0.0;                                               // bound of the spectrum of D^-1 A
  const int32_t* p_ptr = nullptr; const int32_t* p_col = nullptr;   // prolongation from level + 1 (rows N)
  const double* p_val = nullptr;
  const int32_t* r_ptr = nullptr; const int32_t* r_col = nullptr;   // restriction to level + 1 (its rows)
  const double* r_val = nullptr;
  double* r = nullptr;   // right-hand side (levels >= 1) [N][ncol]
  double* z = nullptr;   // correction (levels >= 1)
  double* d = nullptr;   // Chebyshev direction
  double* t = nullptr;   // operator product scratch
};
struct MgDev {
  std::vector<MgLevelDev> lv;   // lv[0] = the operator's own DoF space
  const double* cinv = nullptr; // dense inverse of the coarsest operator
  int nu = 2;                   // smoothing steps before and after the coarse correction
};
// y = A_lev x (level 0 may use the tuned Poisson operator kernel)
using MgSpmv = std::function<void(int lev, const double* x, double* y, hipStream_t s)>;

// z0 = B r0 for one symmetric V-cycle B (Chebyshev pre- and post-smoothing)
void mg_vcycle(const MgDev& mg, int ncol, const double* r0, double* z0, const MgSpmv& spmv, hipStream_t s);
void mg_level_spmv(const MgLevelDev& L, int ncol, const double* x, double* y, hipStream_t s);
// red[slot][c] = sum_i r[i][c] z[i][c] (part: MG_RZ_BLOCKS * ncol doubles)
void mg_rz(int64_t n, int ncol, const double* r, const double* z, double* part, double* red, int slot, hipStream_t s);
// pcur = z + beta pprev, beta = red[rz_cur] / red[rz_prev] per column (rz_prev < 0: beta = 0);
// clears red[rr_clear]
void mg_dir(int64_t n, int ncol, const double* z, const double* pprev, double* pcur, double* red, int rz_cur,
            int rz_prev, int rr_clear, hipStream_t s);

}  // namespace mh
