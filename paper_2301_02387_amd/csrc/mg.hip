// Geometric multigrid preconditioner for the pair Poisson solves (one
// instance): a V-cycle over the hierarchy built by build_multigrid (the
// operator's own Q_p space, Q1 on the same leaves, Q1 on shallower
// refinements, coarser base grids, a dense inverse at the bottom), with
// Chebyshev smoothing preconditioned by the diagonal.  All n^2 real pair
// columns go through every pass together ([rows][ncol] arrays).
#include <hip/hip_runtime.h>

#include <cmath>

#include "devutil.hpp"
#include "mg.hpp"

namespace mh {

// y = A (x - xm) (mode 0), y += A (x - xm) (mode 2); xm may be null.
__global__ void __launch_bounds__(NT) k_csr_mc(int64_t nrows, const int32_t* __restrict__ ptr,
                                               const int32_t* __restrict__ col, const double* __restrict__ val,
                                               const double* __restrict__ x, const double* __restrict__ xm,
                                               int ncol, double* __restrict__ y, int mode) {
  const int64_t total = nrows * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e / ncol;
    const int c = (int)(e - i * ncol);
    double s = 0.0;
    const int beg = ptr[i], end = ptr[i + 1];
    if (xm) {
      for (int t = beg; t < end; ++t) {
        const int64_t j = col[t];
        s += val[t] * (x[j * ncol + c] - xm[j * ncol + c]);
      }
    } else {
      for (int t = beg; t < end; ++t) s += val[t] * x[(int64_t)col[t] * ncol + c];
    }
    y[e] = mode == 2 ? y[e] + s : s;
  }
}
static void csr_mc(int64_t nrows, const int32_t* ptr, const int32_t* col, const double* val, const double* x,
                   const double* xm, int ncol, double* y, int mode, hipStream_t s) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_csr_mc, dim3(nblocks(nrows * ncol, NT, 16384)), dim3(NT), 0, s, nrows, ptr, col, val, x, xm,
                       ncol, y, mode);
}

// One Chebyshev step: res = r - Az (Az null: res = r), d = c1 d + c2 D^-1 res,
// z = d (zero_z) or z += d.
__global__ void __launch_bounds__(NT) k_cheb_mc(int64_t n, int ncol, const double* __restrict__ dinv,
                                                const double* __restrict__ r, const double* __restrict__ Az,
                                                double* __restrict__ d, double* __restrict__ z, double c1, double c2,
                                                int zero_z) {
  const int64_t total = n * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e / ncol;
    const double res = Az ? r[e] - Az[e] : r[e];
    const double dn = (c1 != 0.0 ? c1 * d[e] : 0.0) + c2 * dinv[i] * res;
    d[e] = dn;
    z[e] = zero_z ? dn : z[e] + dn;
  }
}

// z = Ainv r on the coarsest level (dense, row-major): one wave per (row,
// block of 8 columns), the lanes splitting the row's entries
__global__ void __launch_bounds__(NT) k_dense_mc(int64_t n, const double* __restrict__ Ainv,
                                                 const double* __restrict__ r, int ncol, double* __restrict__ z) {
  const int lane = threadIdx.x & 63;
  const int ncb = (ncol + 7) / 8;
  const int64_t items = n * ncb;
  for (int64_t w = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6; w < items; w += ((int64_t)gridDim.x * NT) >> 6) {
    const int64_t i = w / ncb;
    const int c0 = (int)(w - i * ncb) * 8;
    double acc[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[v] = 0.0;
    for (int64_t j = lane; j < n; j += 64) {
      const double a = Ainv[i * n + j];
#pragma unroll
      for (int v = 0; v < 8; ++v)
        if (c0 + v < ncol) acc[v] += a * r[j * ncol + c0 + v];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int v = 0; v < 8; ++v) acc[v] += __shfl_xor(acc[v], off, 64);
    if (lane < 8 && c0 + lane < ncol) {
      double out = 0.0;
#pragma unroll
      for (int v = 0; v < 8; ++v)
        if (v == lane) out = acc[v];
      z[i * ncol + c0 + lane] = out;
    }
  }
}

// Chebyshev smoother of degree nu on [lmax / MG_RANGE, lmax] for D^-1 A,
// applied to A z = r: from z = 0 (pre) or continuing from z (post).
static void smooth(const MgLevelDev& L, int ncol, const double* r, double* z, bool from_zero, int nu,
                   const MgSpmv& spmv, int lev, hipStream_t s) {
  const double b = L.lmax, a = L.lmax / MG_RANGE;
  const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
  const int g = nblocks(L.N * ncol, NT, 16384);
  double rho = 1.0 / sigma;
  for (int k = 0; k < nu; ++k) {
    const double* Az = nullptr;
    if (!(from_zero && k == 0)) {
      spmv(lev, z, L.t, s);
      Az = L.t;
    }
    double c1, c2;
    if (k == 0) {
      c1 = 0.0;
      c2 = 1.0 / theta;
    } else {
      const double rn = 1.0 / (2.0 * sigma - rho);
      c1 = rn * rho;
      c2 = 2.0 * rn / delta;
      rho = rn;
    }
    hipLaunchKernelGGL(k_cheb_mc, dim3(g), dim3(NT), 0, s, L.N, ncol, L.dinv, r, Az, L.d, z, c1, c2,
                       (from_zero && k == 0) ? 1 : 0);
  }
}

void mg_vcycle(const MgDev& mg, int ncol, const double* r0, double* z0, const MgSpmv& spmv, hipStream_t s) {
  const int nl = (int)mg.lv.size();
  for (int l = 0; l < nl; ++l) {
    const MgLevelDev& L = mg.lv[l];
    const double* r = l == 0 ? r0 : L.r;
    double* z = l == 0 ? z0 : L.z;
    if (l == nl - 1) {
      hipLaunchKernelGGL(k_dense_mc, dim3(nblocks(L.N * ((ncol + 7) / 8) * 64, NT, 4096)), dim3(NT), 0, s, L.N,
                         mg.cinv, r, ncol, z);
      break;
    }
    smooth(L, ncol, r, z, true, mg.nu, spmv, l, s);
    spmv(l, z, L.t, s);                                                  // t = A z
    const MgLevelDev& C = mg.lv[l + 1];
    csr_mc(C.N, L.r_ptr, L.r_col, L.r_val, r, L.t, ncol, C.r, 0, s);    // r_{l+1} = R (r - A z)
  }
  for (int l = nl - 2; l >= 0; --l) {
    const MgLevelDev& L = mg.lv[l];
    const MgLevelDev& C = mg.lv[l + 1];
    const double* r = l == 0 ? r0 : L.r;
    double* z = l == 0 ? z0 : L.z;
    csr_mc(L.N, L.p_ptr, L.p_col, L.p_val, C.z, nullptr, ncol, z, 2, s);  // z += P z_{l+1}
    smooth(L, ncol, r, z, false, mg.nu, spmv, l, s);
  }
}

void mg_level_spmv(const MgLevelDev& L, int ncol, const double* x, double* y, hipStream_t s) {
  csr_mc(L.N, L.a_ptr, L.a_col, L.a_val, x, nullptr, ncol, y, 0, s);
}

// PCG pieces: red[RZ + slot] = r . z per column (overwrites), and the
// direction p_k = z + beta_k p_{k-1} with beta_k = rz_k / rz_{k-1}; the
// direction pass also clears the r.r slot the update pass of iteration k fills.
__global__ void __launch_bounds__(NT) k_rz_parts(int64_t n, int ncol, const double* __restrict__ r,
                                                 const double* __restrict__ z, double* __restrict__ part) {
  // ncol consecutive threads take one row (coalesced), NT / ncol rows per pass
  __shared__ double lds[NT];
  const int groups = NT / ncol;
  const int g = threadIdx.x / ncol, c = threadIdx.x - g * ncol;
  double acc = 0.0;
  if (g < groups)
    for (int64_t i = (int64_t)blockIdx.x * groups + g; i < n; i += (int64_t)gridDim.x * groups)
      acc += r[i * ncol + c] * z[i * ncol + c];
  lds[threadIdx.x] = g < groups ? acc : 0.0;
  __syncthreads();
  if (threadIdx.x < (unsigned)ncol) {
    double t = 0.0;
    for (int q = 0; q < groups; ++q) t += lds[q * ncol + threadIdx.x];
    part[(int64_t)blockIdx.x * ncol + threadIdx.x] = t;
  }
}
__global__ void __launch_bounds__(NT) k_rz_finish(const double* __restrict__ part, int nblk, int ncol,
                                                  double* __restrict__ red, int slot) {
  __shared__ double lds4[4];
  const int c = blockIdx.x;
  const double v = sum_partials(part, nblk, ncol, c, lds4);
  if (threadIdx.x == 0) red[slot * ncol + c] = v;
}
void mg_rz(int64_t n, int ncol, const double* r, const double* z, double* part, double* red, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_rz_parts, dim3(MG_RZ_BLOCKS), dim3(NT), 0, s, n, ncol, r, z, part);
  hipLaunchKernelGGL(k_rz_finish, dim3(ncol), dim3(NT), 0, s, part, MG_RZ_BLOCKS, ncol, red, slot);
}

__global__ void __launch_bounds__(NT) k_mg_dir(int64_t n, int ncol, const double* __restrict__ z,
                                               const double* __restrict__ pprev, double* __restrict__ pcur,
                                               double* __restrict__ red, int rz_cur, int rz_prev, int rr_clear) {
  __shared__ double beta[64];
  if (threadIdx.x < (unsigned)ncol) {
    double bt = 0.0;
    if (rz_prev >= 0) {
      const double a = red[rz_cur * ncol + threadIdx.x], b = red[rz_prev * ncol + threadIdx.x];
      bt = b != 0.0 ? a / b : 0.0;
    }
    beta[threadIdx.x] = bt;
  }
  __syncthreads();
  const int64_t total = n * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int c = (int)(e % ncol);
    pcur[e] = z[e] + (beta[c] != 0.0 ? beta[c] * pprev[e] : 0.0);
  }
  if (blockIdx.x == 0 && threadIdx.x < (unsigned)ncol) red[rr_clear * ncol + threadIdx.x] = 0.0;
}
void mg_dir(int64_t n, int ncol, const double* z, const double* pprev, double* pcur, double* red, int rz_cur,
            int rz_prev, int rr_clear, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_dir, dim3(nblocks(n * ncol, NT, 8192)), dim3(NT), 0, s, n, ncol, z, pprev, pcur, red, rz_cur,
                     rz_prev, rr_clear);
}

}  // namespace mh
