// HIP kernels of the MCTDHF-on-octree-FEM hot path for gfx950 (wave64):
// interface mass solve, constraint fill, reductions, mean-field build,
// Krylov (Arnoldi) pieces, Poisson right-hand side and multipole boundary
// values, small dense work and the CI space.
//
// Orbital arrays are complex128 [rows][n] (orbital fastest); Poisson arrays
// are real [rows][ncol].  Row space of one instance: [0,N) DoFs, [N,NE)
// hanging nodes, [NE,NF) box-boundary nodes.  Batched launches: instance
// blockIdx.y, batch row offsets from its DevMesh (kernels.hpp).
#include <hip/hip_runtime.h>

#include <cmath>

#include "devutil.hpp"
#include "kernels.hpp"

namespace mh {

// Sum over a 256-thread block; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = lds[0] + lds[1] + lds[2] + lds[3];
  return t;
}

#define INSTANCE const DevMesh& d = dm[blockIdx.y]

// =====================================================================
// Chebyshev iteration on the interface block A_Ma (Jacobi-preconditioned,
// spectrum bounds from set-up): x_{k+1} = x_k + d_k, r_{k+1} = r_k - A d_k,
// d_{k+1} = c1_k d_k + c2_k D^-1 r_{k+1}; the per-instance coefficients
// (from that instance's bounds) are tabulated in d.cheb.
// =====================================================================
__global__ void __launch_bounds__(NT) k_cheb_init(const DevMesh* __restrict__ dm, const double2* __restrict__ b,
                                                  double2* __restrict__ x, double2* __restrict__ r,
                                                  double2* __restrict__ d0) {
  INSTANCE;
  const int n = d.n;
  const int64_t total = d.nMa * n, o = d.oMa * n;
  if (total == 0) return;
  const double inv_theta = d.cheb[0];
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t i = idx / n;
    double2 bi = b[o + idx];
    x[o + idx] = make_double2(0.0, 0.0);
    r[o + idx] = bi;
    d0[o + idx] = cscale(d.ma_dinv[i] * inv_theta, bi);
  }
}

// One row of the interface block per group of CHEB_G lanes: the lanes split
// the row's entries (tens per row) and combine by shuffles, all n orbitals
// at once.
constexpr int CHEB_G = 8;
__global__ void __launch_bounds__(NT) k_cheb_iter(const DevMesh* __restrict__ dm, double2* __restrict__ x,
                                                  double2* __restrict__ r, const double2* __restrict__ din,
                                                  double2* __restrict__ dout, int k) {
  INSTANCE;
  const int n = d.n;
  if (d.nMa == 0) return;
  const int64_t o = d.oMa * n;
  const double c1 = d.cheb[1 + 2 * k], c2 = d.cheb[2 + 2 * k];
  const double2* dI = din + o;
  const int g = (int)(threadIdx.x & (CHEB_G - 1));
  // XCD x sweeps the x-th eighth of the (band-ordered) rows, so its gathers
  // stay within that part of the vectors and hit its own L2
  const XcdSweep sw = xcd_sweep(d.nMa, NT / CHEB_G);
  for (int64_t i = sw.start + threadIdx.x / CHEB_G; i < sw.end; i += sw.step) {
    double sx[8], sy[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) { sx[p] = 0.0; sy[p] = 0.0; }
    const auto* mp = gbl(d.ma_ptr);
    for (int t = mp[i] + g; t < mp[i + 1]; t += CHEB_G) {
      const double a = gbl(d.ma_val)[t];
      const double2* row = dI + (int64_t)gbl(d.ma_col)[t] * n;
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (p < n) {
          const double2 v = row[p];
          sx[p] += a * v.x;
          sy[p] += a * v.y;
        }
    }
#pragma unroll
    for (int off = CHEB_G / 2; off > 0; off >>= 1)
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (p < n) {
          sx[p] += __shfl_xor(sx[p], off, CHEB_G);
          sy[p] += __shfl_xor(sy[p], off, CHEB_G);
        }
    const double gi = c2 * gbl(d.ma_dinv)[i];
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (p < n && p % CHEB_G == g) {
        const int64_t idx = o + i * n + p;
        const double2 dk = din[idx];
        x[idx] = cadd(x[idx], dk);
        const double2 rn = csub(r[idx], make_double2(sx[p], sy[p]));
        r[idx] = rn;
        dout[idx] = make_double2(c1 * dk.x + gi * rn.x, c1 * dk.y + gi * rn.y);
      }
  }
}

__global__ void __launch_bounds__(NT) k_cheb_finish(const DevMesh* __restrict__ dm, const double2* __restrict__ x,
                                                    const double2* __restrict__ dk, const double2* __restrict__ v,
                                                    const double2* __restrict__ lam, double2* __restrict__ out) {
  INSTANCE;
  const int n = d.n;
  const int64_t total = d.nMa * n, o = d.oMa * n, oe = d.oE * n;
  const double2* L = lam ? lam + (int64_t)blockIdx.y * n * n : nullptr;
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t i = idx / n;
    const int p = (int)(idx - i * n);
    const int64_t k = d.ma_dof[i];
    double2 xf = cadd(x[o + idx], dk[o + idx]);
    if (L)
      for (int q = 0; q < n; ++q) xf = csub(xf, cmul(L[q * n + p], v[oe + k * n + q]));
    out[oe + k * n + p] = xf;
  }
}

// Interface solve by the dense inverse (one instance): x = A^-1 b, one wave per
// row, the lanes splitting the row's columns (four strides of 64 per round,
// their loads in flight together); then the final value of each master DoF
// as in k_cheb_finish.  NP: the orbital count rounded up (2, 4 or 8).
template <int NP>
__global__ void __launch_bounds__(NT) k_ma_dense(const DevMesh* __restrict__ dm, const double2* __restrict__ b,
                                                 const double2* __restrict__ v, const double2* __restrict__ lam,
                                                 double2* __restrict__ out) {
  INSTANCE;
  const int n = d.n;
  const int64_t nMa = d.nMa, o = d.oMa * n, oe = d.oE * n;
  const auto* Ai = gbl(d.ma_inv);
  const int lane = threadIdx.x & 63;
  const double2* L = lam ? lam + (int64_t)blockIdx.y * n * n : nullptr;
  for (int64_t i = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6; i < nMa; i += ((int64_t)gridDim.x * NT) >> 6) {
    double sx[NP], sy[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) { sx[p] = 0.0; sy[p] = 0.0; }
    const auto* row = Ai + i * nMa;
    int64_t j = lane;
    for (; j + 192 < nMa; j += 256) {
      double a[4];
      double2 bj[4][NP];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = row[j + 64 * u];
#pragma unroll
        for (int p = 0; p < NP; ++p)
          if (p < n) bj[u][p] = ldg2(b, o + (j + 64 * u) * n + p);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int p = 0; p < NP; ++p)
          if (p < n) {
            sx[p] += a[u] * bj[u][p].x;
            sy[p] += a[u] * bj[u][p].y;
          }
    }
    for (; j < nMa; j += 64) {
      const double a = row[j];
#pragma unroll
      for (int p = 0; p < NP; ++p)
        if (p < n) {
          const double2 bj = ldg2(b, o + j * n + p);
          sx[p] += a * bj.x;
          sy[p] += a * bj.y;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int p = 0; p < NP; ++p)
        if (p < n) {
          sx[p] += __shfl_xor(sx[p], off, 64);
          sy[p] += __shfl_xor(sy[p], off, 64);
        }
    if (lane < n) {
      double2 xf = make_double2(0.0, 0.0);
#pragma unroll
      for (int p = 0; p < NP; ++p)
        if (p == lane) xf = make_double2(sx[p], sy[p]);
      const int64_t k = d.ma_dof[i];
      if (L)
        for (int q = 0; q < n; ++q) xf = csub(xf, cmul(L[q * n + lane], v[oe + k * n + q]));
      out[oe + k * n + lane] = xf;
    }
  }
}

// Gauss-Jordan step k on a dense SPD matrix: entries off row and column k
// (reading row and column k, which this launch does not write) ...
__global__ void __launch_bounds__(NT) k_gj_update(double* __restrict__ A, int64_t n, int64_t k) {
  const double inv = 1.0 / A[k * n + k];
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n * n; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e / n, j = e - i * n;
    if (i == k || j == k) continue;
    A[e] -= A[i * n + k] * A[k * n + j] * inv;
  }
}
// ... then row and column k (reading the pivot, written by the next launch) ...
__global__ void __launch_bounds__(NT) k_gj_rowcol(double* __restrict__ A, int64_t n, int64_t k) {
  const double inv = 1.0 / A[k * n + k];
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT) {
    if (t == k) continue;
    A[k * n + t] *= inv;
    A[t * n + k] *= -inv;
  }
}
// ... then the pivot itself.
__global__ void k_gj_pivot(double* __restrict__ A, int64_t n, int64_t k) {
  if (blockIdx.x == 0 && threadIdx.x == 0) A[k * n + k] = 1.0 / A[k * n + k];
}
void launch_dense_inverse(double* A, int64_t n, hipStream_t s) {
  const int g = nblocks(n * n, NT, 8192), g2 = nblocks(n, NT, 256);
  for (int64_t k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_gj_update, dim3(g), dim3(NT), 0, s, A, n, k);
    hipLaunchKernelGGL(k_gj_rowcol, dim3(g2), dim3(NT), 0, s, A, n, k);
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(64), 0, s, A, n, k);
  }
}

void launch_ma_solve(const Batch& b, const double* ma_b, double* x, double* r, double* dbuf0, double* dbuf1,
                     const double* v, const double* lam, double* out, hipStream_t s) {
  if (b.mx.nMa == 0) return;
  if (b.ni == 1 && b.mx.ma_inv && !(b.mx.sched_orb & 2)) {
    const dim3 g(nblocks(b.mx.nMa * 64, NT, 8192), 1);
    if (b.mx.n <= 2)
      hipLaunchKernelGGL(k_ma_dense<2>, g, dim3(NT), 0, s, b.dm, (const double2*)ma_b, (const double2*)v,
                         (const double2*)lam, (double2*)out);
    else if (b.mx.n <= 4)
      hipLaunchKernelGGL(k_ma_dense<4>, g, dim3(NT), 0, s, b.dm, (const double2*)ma_b, (const double2*)v,
                         (const double2*)lam, (double2*)out);
    else
      hipLaunchKernelGGL(k_ma_dense<8>, g, dim3(NT), 0, s, b.dm, (const double2*)ma_b, (const double2*)v,
                         (const double2*)lam, (double2*)out);
    return;
  }
  const dim3 g(nblocks(b.mx.nMa * b.mx.n), b.ni);
  hipLaunchKernelGGL(k_cheb_init, g, dim3(NT), 0, s, b.dm, (const double2*)ma_b, (double2*)x, (double2*)r,
                     (double2*)dbuf0);
  double* din = dbuf0;
  double* dout = dbuf1;
  const dim3 gi(xcd_grid(b.mx.nMa, NT / CHEB_G, 65536), b.ni);
  for (int k = 0; k < b.cheb_iters; ++k) {
    hipLaunchKernelGGL(k_cheb_iter, gi, dim3(NT), 0, s, b.dm, (double2*)x, (double2*)r, (const double2*)din,
                       (double2*)dout, k);
    double* t = din;
    din = dout;
    dout = t;
  }
  hipLaunchKernelGGL(k_cheb_finish, g, dim3(NT), 0, s, b.dm, (const double2*)x, (const double2*)din,
                     (const double2*)v, (const double2*)lam, (double2*)out);
}

// Hanging rows: x[h] = sum_k c_hk x[k] over DoF masters (boundary values of
// orbitals vanish); optionally zero the hanging rows of acc.
__global__ void __launch_bounds__(NT) k_fill_orb(const DevMesh* __restrict__ dm, double2* __restrict__ x,
                                                 double2* __restrict__ acc) {
  INSTANCE;
  const int n = d.n;
  const int64_t total = d.Nh * n, o = d.oE * n;
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t h = idx / n;
    const int p = (int)(idx - h * n);
    double2 s = make_double2(0.0, 0.0);
    const auto* hp = gbl(d.hang_ptr);
    for (int t = hp[h]; t < hp[h + 1]; ++t) {
      int col = gbl(d.hang_col)[t];
      if (col < d.N) {
        const double w = gbl(d.hang_w)[t];
        double2 v = x[o + (int64_t)col * n + p];
        s.x += w * v.x;
        s.y += w * v.y;
      }
    }
    x[o + (d.N + h) * n + p] = s;
    if (acc) acc[o + (d.N + h) * n + p] = make_double2(0.0, 0.0);
  }
}

void launch_fill_orb(const Batch& b, double* x, double* acc, hipStream_t s) {
  if (b.mx.Nh == 0) return;
  hipLaunchKernelGGL(k_fill_orb, dim3(nblocks(b.mx.Nh * b.mx.n), b.ni), dim3(NT), 0, s, b.dm, (double2*)x,
                     (double2*)acc);
}

__global__ void k_copy(const double* __restrict__ in, double* __restrict__ out, int64_t nd) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nd; i += (int64_t)gridDim.x * NT) out[i] = in[i];
}
__global__ void k_zero(double* __restrict__ out, int64_t nd) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nd; i += (int64_t)gridDim.x * NT) out[i] = 0.0;
}
__global__ void k_set(double* __restrict__ out, double value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = value;
}
void launch_copy(const double* in, double* out, int64_t nd, hipStream_t s) {
  if (nd > 0) hipLaunchKernelGGL(k_copy, dim3(nblocks(nd, NT, 8192)), dim3(NT), 0, s, in, out, nd);
}
void launch_zero(double* out, int64_t nd, hipStream_t s) {
  if (nd > 0) hipLaunchKernelGGL(k_zero, dim3(nblocks(nd, NT, 8192)), dim3(NT), 0, s, out, nd);
}
// x <- 2 x - xp and xp <- the old x (linear extrapolation in time, history shifted)
__global__ void k_extrapolate(double* __restrict__ x, double* __restrict__ xp, int64_t nd) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nd; i += (int64_t)gridDim.x * NT) {
    const double xi = x[i];
    x[i] = 2.0 * xi - xp[i];
    xp[i] = xi;
  }
}
void launch_extrapolate(double* x, double* xprev, int64_t nd, hipStream_t s) {
  if (nd > 0) hipLaunchKernelGGL(k_extrapolate, dim3(nblocks(nd, NT, 8192)), dim3(NT), 0, s, x, xprev, nd);
}
// x <- 3 x - 3 p1 + p2 (quadratic extrapolation in time), then p2 <- p1, p1 <- the old x
__global__ void k_extrapolate2(double* __restrict__ x, double* __restrict__ p1, double* __restrict__ p2, int64_t nd) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nd; i += (int64_t)gridDim.x * NT) {
    const double xi = x[i], a = p1[i];
    x[i] = 3.0 * (xi - a) + p2[i];
    p2[i] = a;
    p1[i] = xi;
  }
}
void launch_extrapolate2(double* x, double* p1, double* p2, int64_t nd, hipStream_t s) {
  if (nd > 0) hipLaunchKernelGGL(k_extrapolate2, dim3(nblocks(nd, NT, 8192)), dim3(NT), 0, s, x, p1, p2, nd);
}
void launch_set(double* out, double value, hipStream_t s) {
  hipLaunchKernelGGL(k_set, dim3(1), dim3(64), 0, s, out, value);
}
// A step counter on the device, so that a captured step reads its own field
// value from a table: out = table[*ctr]; ctr += add.
__global__ void k_set_indexed(double* __restrict__ out, const double* __restrict__ table,
                              const int* __restrict__ ctr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = table[ctr[0]];
}
__global__ void k_counter(int* __restrict__ ctr, int set, int value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctr[0] = set ? value : ctr[0] + value;
}
void launch_set_indexed(double* out, const double* table, const int* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_set_indexed, dim3(1), dim3(64), 0, s, out, table, ctr);
}
void launch_counter(int* ctr, int set, int value, hipStream_t s) {
  hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, ctr, set, value);
}

// =====================================================================
// Generic tiled reduction: out[a][b] = sum_i wt_i conj(X[i][a]) Y[i][b],
// one output set per instance.  Mesh mode (dm != null): X, Y are batch
// orbital arrays with na, nb columns, rows N or NE of the instance, weight
// none / m / m z.  Flat mode: X [ni][rows][na], Y [ni][rows][nb].
// Partials per block, then a finishing pass.  Deterministic.
// =====================================================================
constexpr int XG_CH = 16;
__global__ void __launch_bounds__(NT) k_xgram(const DevMesh* __restrict__ dm, int wsel, int rsel,
                                              const double2* __restrict__ X, int na, const double2* __restrict__ Y,
                                              int nb, int64_t frows, double2* __restrict__ part) {
  __shared__ double2 sx[XG_CH * 64];
  __shared__ double2 sy[XG_CH * 64];
  int64_t rows, xo, yo;
  const double* wt = nullptr;
  if (dm) {
    const DevMesh& d = dm[blockIdx.y];
    rows = rsel == ROWS_EXT ? d.NE : d.N;
    xo = d.oE * na;
    yo = d.oE * nb;
    wt = wsel == WT_MASS ? d.m : (wsel == WT_DIPOLE ? d.mz : nullptr);
  } else {
    rows = frows;
    xo = (int64_t)blockIdx.y * frows * na;
    yo = (int64_t)blockIdx.y * frows * nb;
  }
  X += xo;
  Y += yo;
  const int nout = na * nb;
  constexpr int MAXO = 16;  // outputs per thread (na*nb <= 4096)
  double2 accv[MAXO];
#pragma unroll
  for (int j = 0; j < MAXO; ++j) accv[j] = make_double2(0.0, 0.0);
  for (int64_t base = (int64_t)blockIdx.x * XG_CH; base < rows; base += (int64_t)gridDim.x * XG_CH) {
    const int cnt = (int)((rows - base) < XG_CH ? (rows - base) : XG_CH);
    __syncthreads();
    for (int e = threadIdx.x; e < XG_CH * na; e += NT) {
      int r = e / na, a = e - r * na;
      double2 v = make_double2(0.0, 0.0);
      if (r < cnt) {
        v = X[(base + r) * na + a];
        if (wt) v = cscale(gbl(wt)[base + r], v);
      }
      sx[r * na + a] = v;
    }
    for (int e = threadIdx.x; e < XG_CH * nb; e += NT) {
      int r = e / nb, bb = e - r * nb;
      sy[r * nb + bb] = (r < cnt) ? Y[(base + r) * nb + bb] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MAXO; ++j) {
      int o = threadIdx.x + j * NT;
      if (o >= nout) break;
      int a = o / nb, bb = o - a * nb;
      double2 s = accv[j];
      for (int r = 0; r < cnt; ++r) {
        double2 xv = sx[r * na + a], yv = sy[r * nb + bb];
        s.x += xv.x * yv.x + xv.y * yv.y;
        s.y += xv.x * yv.y - xv.y * yv.x;
      }
      accv[j] = s;
    }
  }
  double2* pb = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * nout;
#pragma unroll
  for (int j = 0; j < MAXO; ++j) {
    int o = threadIdx.x + j * NT;
    if (o < nout) pb[o] = accv[j];
  }
}

// The same for small output sets (na nb <= 16): every thread accumulates all
// outputs over a grid-stride set of rows (no staging, no barrier per chunk),
// then one reduction per workgroup (shuffles, then the four waves).
__global__ void __launch_bounds__(NT) k_xgram_small(const DevMesh* __restrict__ dm, int wsel, int rsel,
                                                    const double2* __restrict__ X, int na,
                                                    const double2* __restrict__ Y, int nb, int64_t frows,
                                                    double2* __restrict__ part) {
  __shared__ double2 lw[NT / 64][16];
  int64_t rows, xo, yo;
  const double* wt = nullptr;
  if (dm) {
    const DevMesh& d = dm[blockIdx.y];
    rows = rsel == ROWS_EXT ? d.NE : d.N;
    xo = d.oE * na;
    yo = d.oE * nb;
    wt = wsel == WT_MASS ? d.m : (wsel == WT_DIPOLE ? d.mz : nullptr);
  } else {
    rows = frows;
    xo = (int64_t)blockIdx.y * frows * na;
    yo = (int64_t)blockIdx.y * frows * nb;
  }
  X += xo;
  Y += yo;
  const int nout = na * nb;
  double2 acc[16];
#pragma unroll
  for (int o = 0; o < 16; ++o) acc[o] = make_double2(0.0, 0.0);
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < rows; i += (int64_t)gridDim.x * NT) {
    const double w = wt ? gbl(wt)[i] : 1.0;
#pragma unroll
    for (int o = 0; o < 16; ++o)
      if (o < nout) {
        const int a = o / nb, bb = o - a * nb;
        const double2 xv = cscale(w, X[i * na + a]), yv = Y[i * nb + bb];
        acc[o].x += xv.x * yv.x + xv.y * yv.y;
        acc[o].y += xv.x * yv.y - xv.y * yv.x;
      }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 0; o < 16; ++o)
    if (o < nout) {
      const double sx = wave_sum(acc[o].x), sy = wave_sum(acc[o].y);
      if (lane == 0) lw[wid][o] = make_double2(sx, sy);
    }
  __syncthreads();
  if (threadIdx.x < (unsigned)nout) {
    double2 t = lw[0][threadIdx.x];
    for (int w = 1; w < NT / 64; ++w) t = cadd(t, lw[w][threadIdx.x]);
    part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * nout + threadIdx.x] = t;
  }
}

// out[i][o] = sum_b part[i][b][o]; one workgroup per (output, instance)
__global__ void __launch_bounds__(NT) k_sum_parts(const double2* __restrict__ part, int nblk, int nout,
                                                  double2* __restrict__ out) {
  __shared__ double lds4[4];
  const double* pi = (const double*)(part + (int64_t)blockIdx.y * nblk * nout);
  const int o = blockIdx.x;
  const double sx = sum_partials(pi, nblk, 2 * nout, 2 * o, lds4);
  const double sy = sum_partials(pi, nblk, 2 * nout, 2 * o + 1, lds4);
  if (threadIdx.x == 0) out[(int64_t)blockIdx.y * nout + o] = make_double2(sx, sy);
}

int gram_blocks(int64_t rows) { return nblocks(rows, XG_CH, 512); }

void launch_gram(const Batch& b, const double* A, const double* B, int wsel, int rows, double* part, int nblk,
                 double* G, hipStream_t s) {
  const int n = b.mx.n;
  if (n * n <= 16)
    hipLaunchKernelGGL(k_xgram_small, dim3(nblk, b.ni), dim3(NT), 0, s, b.dm, wsel, rows, (const double2*)A, n,
                       (const double2*)B, n, (int64_t)0, (double2*)part);
  else
    hipLaunchKernelGGL(k_xgram, dim3(nblk, b.ni), dim3(NT), 0, s, b.dm, wsel, rows, (const double2*)A, n,
                       (const double2*)B, n, (int64_t)0, (double2*)part);
  hipLaunchKernelGGL(k_sum_parts, dim3(n * n, b.ni), dim3(NT), 0, s, (const double2*)part, nblk, n * n,
                     (double2*)G);
}

void launch_xgram_flat(int ni, const double* X, int na, const double* Y, int nb, int64_t rows, double* part,
                       int nblk, double* out, hipStream_t s) {
  if (na * nb <= 16)
    hipLaunchKernelGGL(k_xgram_small, dim3(nblk, ni), dim3(NT), 0, s, (const DevMesh*)nullptr, 0, 0,
                       (const double2*)X, na, (const double2*)Y, nb, rows, (double2*)part);
  else
    hipLaunchKernelGGL(k_xgram, dim3(nblk, ni), dim3(NT), 0, s, (const DevMesh*)nullptr, 0, 0, (const double2*)X, na,
                       (const double2*)Y, nb, rows, (double2*)part);
  hipLaunchKernelGGL(k_sum_parts, dim3(na * nb, ni), dim3(NT), 0, s, (const double2*)part, nblk, na * nb,
                     (double2*)out);
}

// Pair-product integrals: G[(p,q)][col] = sum_i m_i conj(phi_p) phi_q Wcol_i
// (X built on the fly as phi_p conj(phi_q) so that conj(X) = conj(phi_p) phi_q).
// Register tiles of GT_A pair products x GT_C columns per thread: every
// round of LDS reads (four products, four potentials) feeds 32 FMAs; tiles
// numbered column-tile fastest, at most NT of them (n <= 8).
constexpr int GT_A = 4, GT_C = 4;
__global__ void __launch_bounds__(NT) k_gint(const DevMesh* __restrict__ dm, const double2* __restrict__ phi,
                                             const double* __restrict__ W, int ncol, double2* __restrict__ part) {
  INSTANCE;
  __shared__ double2 sx[XG_CH * 64];
  __shared__ double sw[XG_CH * 64];
  const int n = d.n, na = n * n, nout = na * ncol;
  const int nap = (na + GT_A - 1) / GT_A * GT_A, ncp = (ncol + GT_C - 1) / GT_C * GT_C;
  phi += d.oE * n;
  W += d.oF * ncol;
  const int tiles_c = ncp / GT_C, tiles = (nap / GT_A) * tiles_c;
  const bool act = (int)threadIdx.x < tiles;
  const int a0 = act ? ((int)threadIdx.x / tiles_c) * GT_A : 0, c0 = act ? ((int)threadIdx.x % tiles_c) * GT_C : 0;
  double2 acc[GT_A][GT_C];
#pragma unroll
  for (int u = 0; u < GT_A; ++u)
#pragma unroll
    for (int v = 0; v < GT_C; ++v) acc[u][v] = make_double2(0.0, 0.0);
  const int64_t rows = d.NE;
  for (int64_t base = (int64_t)blockIdx.x * XG_CH; base < rows; base += (int64_t)gridDim.x * XG_CH) {
    const int cnt = (int)((rows - base) < XG_CH ? (rows - base) : XG_CH);
    __syncthreads();
    for (int e = threadIdx.x; e < XG_CH * nap; e += NT) {
      const int r = e / nap, a = e - r * nap;
      double2 v = make_double2(0.0, 0.0);
      if (r < cnt && a < na) {
        const int p = a / n, q = a - p * n;
        const int64_t i = base + r;
        const double2 fp = phi[i * n + p], fq = phi[i * n + q];
        // phi_p conj(phi_q) * m_i
        v = cscale(d.m[i], make_double2(fp.x * fq.x + fp.y * fq.y, fp.y * fq.x - fp.x * fq.y));
      }
      sx[r * nap + a] = v;
    }
    for (int e = threadIdx.x; e < XG_CH * ncp; e += NT) {
      const int r = e / ncp, c = e - r * ncp;
      sw[r * ncp + c] = (r < cnt && c < ncol) ? W[(base + r) * ncol + c] : 0.0;
    }
    __syncthreads();
    if (act)
      for (int r = 0; r < cnt; ++r) {
        double2 xv[GT_A];
        double yv[GT_C];
#pragma unroll
        for (int u = 0; u < GT_A; ++u) xv[u] = sx[r * nap + a0 + u];
#pragma unroll
        for (int v = 0; v < GT_C; ++v) yv[v] = sw[r * ncp + c0 + v];
#pragma unroll
        for (int u = 0; u < GT_A; ++u)
#pragma unroll
          for (int v = 0; v < GT_C; ++v) {
            acc[u][v].x += xv[u].x * yv[v];
            acc[u][v].y -= xv[u].y * yv[v];
          }
      }
  }
  if (!act) return;
  double2* pb = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * nout;
#pragma unroll
  for (int u = 0; u < GT_A; ++u)
#pragma unroll
    for (int v = 0; v < GT_C; ++v)
      if (a0 + u < na && c0 + v < ncol) pb[(a0 + u) * ncol + c0 + v] = acc[u][v];
}

// The same on the matrix cores (n >= 4): per chunk of GM_CH rows the real
// and imaginary parts of the products X and the potentials are staged in
// LDS, and Re G = sum Re X W, Im G = -sum Im X W accumulate in FP64 MFMA tiles
// of 16 products x 16 columns (the lane layout of k_moments_mfma), the tiles
// (real and imaginary product tiles x column tiles) dealt round-robin to the
// four waves, at most GM_TW per wave.
constexpr int GM_CH = 16, GM_TW = 8;
typedef double dvec4g_t __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(NT) k_gint_mfma(const DevMesh* __restrict__ dm, const double2* __restrict__ phi,
                                                  const double* __restrict__ W, int ncol,
                                                  double2* __restrict__ part) {
  INSTANCE;
  __shared__ double sxr[GM_CH * 64];
  __shared__ double sxi[GM_CH * 64];
  __shared__ double sw[GM_CH * 64];
  const int n = d.n, na = n * n, nout = na * ncol;
  phi += d.oE * n;
  W += d.oF * ncol;
  const int nat = (na + 15) / 16, nct = (ncol + 15) / 16, ntile = 2 * nat * nct;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  dvec4g_t acc[GM_TW];
#pragma unroll
  for (int j = 0; j < GM_TW; ++j) acc[j] = dvec4g_t{0.0, 0.0, 0.0, 0.0};
  const int64_t rows = d.NE;
  for (int64_t base = (int64_t)blockIdx.x * GM_CH; base < rows; base += (int64_t)gridDim.x * GM_CH) {
    const int cnt = (int)((rows - base) < GM_CH ? (rows - base) : GM_CH);
    __syncthreads();
    for (int e = threadIdx.x; e < GM_CH * 64; e += NT) {
      const int r = e >> 6, a = e & 63;
      double xr = 0.0, xi = 0.0, wv = 0.0;
      if (r < cnt) {
        const int64_t i = base + r;
        if (a < na) {
          const int p = a / n, q = a - p * n;
          const double2 fp = phi[i * n + p], fq = phi[i * n + q];
          const double mi = d.m[i];
          // m_i phi_p conj(phi_q)
          xr = mi * (fp.x * fq.x + fp.y * fq.y);
          xi = mi * (fp.y * fq.x - fp.x * fq.y);
        }
        if (a < ncol) wv = W[i * ncol + a];
      }
      sxr[e] = xr;
      sxi[e] = xi;
      sw[e] = wv;
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < GM_CH; k0 += 4) {
      const int kr = k0 + (lane >> 4), li = lane & 15;
#pragma unroll
      for (int j = 0; j < GM_TW; ++j) {
        const int tile = wave + 4 * j;
        if (tile < ntile) {
          const int u = tile % nct, ta = tile / nct;   // ta < nat: real tiles, then imaginary
          const int t = ta < nat ? ta : ta - nat;
          const double a = (ta < nat ? sxr : sxi)[kr * 64 + 16 * t + li];
          const double b = sw[kr * 64 + 16 * u + li];
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        }
      }
    }
  }
  double* pb = (double*)(part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * nout);
#pragma unroll
  for (int j = 0; j < GM_TW; ++j) {
    const int tile = wave + 4 * j;
    if (tile >= ntile) continue;
    const int u = tile % nct, ta = tile / nct;
    const bool im = ta >= nat;
    const int t = im ? ta - nat : ta;
    const int c = 16 * u + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * t + 4 * v + (lane >> 4);
      // conj(X) W: the imaginary part enters with a minus sign
      if (a < na && c < ncol) pb[2 * (a * ncol + c) + (im ? 1 : 0)] = im ? -acc[j][v] : acc[j][v];
    }
  }
}

// The same for n^2 x ncol <= 16 outputs (two orbitals): every thread
// accumulates all outputs over a grid-stride set of rows, then one reduction
// per workgroup.
__global__ void __launch_bounds__(NT) k_gint_small(const DevMesh* __restrict__ dm, const double2* __restrict__ phi,
                                                   const double* __restrict__ W, int ncol,
                                                   double2* __restrict__ part) {
  INSTANCE;
  __shared__ double2 lw[NT / 64][16];
  const int n = d.n, na = n * n, nout = na * ncol;
  phi += d.oE * n;
  W += d.oF * ncol;
  double2 acc[16];
#pragma unroll
  for (int o = 0; o < 16; ++o) acc[o] = make_double2(0.0, 0.0);
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < d.NE; i += (int64_t)gridDim.x * NT) {
    const double mi = gbl(d.m)[i];
#pragma unroll
    for (int o = 0; o < 16; ++o)
      if (o < nout) {
        const int a = o / ncol, c = o - a * ncol;
        const int p = a / n, q = a - p * n;
        const double2 fp = phi[i * n + p], fq = phi[i * n + q];
        // phi_p conj(phi_q) m_i, conjugated
        const double2 xv = cscale(mi, make_double2(fp.x * fq.x + fp.y * fq.y, fp.y * fq.x - fp.x * fq.y));
        const double yv = W[i * ncol + c];
        acc[o].x += xv.x * yv;
        acc[o].y -= xv.y * yv;
      }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 0; o < 16; ++o)
    if (o < nout) {
      const double sx = wave_sum(acc[o].x), sy = wave_sum(acc[o].y);
      if (lane == 0) lw[wid][o] = make_double2(sx, sy);
    }
  __syncthreads();
  if (threadIdx.x < (unsigned)nout) {
    double2 t = lw[0][threadIdx.x];
    for (int w = 1; w < NT / 64; ++w) t = cadd(t, lw[w][threadIdx.x]);
    part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * nout + threadIdx.x] = t;
  }
}

// Assemble g_pqrs from the pair-column integrals G[(p,q)][col].
__global__ void k_gint_assemble(const double2* __restrict__ G, int n, const int* __restrict__ colmap,
                                double2* __restrict__ g) {
  const int ncol = n * n, n4 = ncol * ncol;
  G += (int64_t)blockIdx.y * n4;
  g += (int64_t)blockIdx.y * n4;
  for (int o = blockIdx.x * NT + threadIdx.x; o < n4; o += gridDim.x * NT) {
    int s = o % n, r = (o / n) % n, pq = o / (n * n);
    int rr = r < s ? r : s, ss = r < s ? s : r;
    int cre = colmap[rr * n + ss];
    double2 val = G[pq * ncol + cre];
    if (rr != ss) {
      double2 im = G[pq * ncol + cre + 1];
      double sg = (r < s) ? 1.0 : -1.0;
      val = make_double2(val.x - sg * im.y, val.y + sg * im.x);
    }
    g[o] = val;
  }
}

// up to 2048 workgroups for the matrix-core form (n >= 4), 512 otherwise
int gint_blocks(const Batch& b) { return nblocks(b.mx.NE, XG_CH, b.mx.n >= 4 ? 2048 : 512); }

void launch_gint_full(const Batch& b, const double* phi, const double* W, const int* colmap, double* part, int nblk,
                      double* Gtmp, double* g, hipStream_t s) {
  const int n = b.mx.n, ncol = n * n;
  if (ncol * ncol <= 16)
    hipLaunchKernelGGL(k_gint_small, dim3(nblk, b.ni), dim3(NT), 0, s, b.dm, (const double2*)phi, W, ncol,
                       (double2*)part);
  else if (n >= 4)   // matrix cores: at least one full 16 x 16 tile
    hipLaunchKernelGGL(k_gint_mfma, dim3(nblk, b.ni), dim3(NT), 0, s, b.dm, (const double2*)phi, W, ncol,
                       (double2*)part);
  else
    hipLaunchKernelGGL(k_gint, dim3(nblk, b.ni), dim3(NT), 0, s, b.dm, (const double2*)phi, W, ncol,
                       (double2*)part);
  hipLaunchKernelGGL(k_sum_parts, dim3(ncol * ncol, b.ni), dim3(NT), 0, s, (const double2*)part, nblk, ncol * ncol,
                     (double2*)Gtmp);
  hipLaunchKernelGGL(k_gint_assemble, dim3(nblocks(ncol * ncol), b.ni), dim3(NT), 0, s, (const double2*)Gtmp, n,
                     colmap, (double2*)g);
}

// =====================================================================
// Mean field: U(x) = sum_rs Gamma_oq,rs W_rs(x), a real linear map of the
// n^2 real Poisson columns to the n^2 packed entries of the Hermitian U.
// =====================================================================
__global__ void k_build_Mreal(const double2* __restrict__ Gamma, int n, const int* __restrict__ colmap,
                              double* __restrict__ Mr) {
  const int nn = n * n;
  Gamma += (int64_t)blockIdx.y * nn * nn;
  Mr += (int64_t)blockIdx.y * nn * nn;
  for (int o = blockIdx.x * NT + threadIdx.x; o < nn * nn; o += gridDim.x * NT) {
    int out = o / nn, col = o - out * nn;
    int oi = out / n, qi = out - oi * n;  // packed position
    int ro = oi < qi ? oi : qi, co = oi < qi ? qi : oi;
    bool want_im = oi > qi;               // lower triangle holds the imaginary part
    // locate (r, s, part) of col
    int rr = 0, ss = 0, part = 0;
    for (int r = 0; r < n; ++r)
      for (int s = r; s < n; ++s) {
        int c0 = colmap[r * n + s];
        if (c0 == col) { rr = r; ss = s; part = 0; }
        if (r != s && c0 + 1 == col) { rr = r; ss = s; part = 1; }
      }
    // U_{ro,co} as a function of column value: Gamma_{ro co, rr ss} (a + i b) + Gamma_{ro co, ss rr} (a - i b)
    double2 g1 = Gamma[((ro * n + co) * n + rr) * n + ss];
    double2 g2 = Gamma[((ro * n + co) * n + ss) * n + rr];
    double2 coef;
    if (rr == ss) coef = g1;                                      // a only
    else if (part == 0) coef = cadd(g1, g2);                       // d U / d a
    else coef = make_double2(-(g1.y - g2.y), g1.x - g2.x);          // i (g1 - g2)
    Mr[o] = want_im ? coef.y : coef.x;
  }
}

// Upk[i][o] = sum_c Mr[o][c] W[i][c]: G lanes per node (G = n^2 rounded up
// to a power of two), lane o owning output o; the node's W row is read once,
// coalesced, and broadcast by shuffles; Mr is held transposed in LDS so the
// lanes of a group read consecutive words.
template <int G>
__global__ void __launch_bounds__(NT) k_build_U(const DevMesh* __restrict__ dm, const double* __restrict__ W,
                                                const double* __restrict__ Mr, double* __restrict__ Upk) {
  INSTANCE;
  __shared__ double sMT[64 * 64];
  const int nn = d.n * d.n;
  Mr += (int64_t)blockIdx.y * nn * nn;
  W += d.oF * nn;
  Upk += d.oE * nn;
  for (int e = threadIdx.x; e < nn * nn; e += NT) {
    const int o = e / nn, c = e - o * nn;
    sMT[c * nn + o] = Mr[e];
  }
  __syncthreads();
  const int o = (int)(threadIdx.x & (G - 1));
  for (int64_t i = ((int64_t)blockIdx.x * NT + threadIdx.x) / G; i < d.NE; i += ((int64_t)gridDim.x * NT) / G) {
    const double w = o < nn ? W[i * nn + o] : 0.0;
    double acc = 0.0;
    for (int c = 0; c < nn; ++c) {
      const double wc = __shfl(w, c, G);
      if (o < nn) acc += sMT[c * nn + o] * wc;
    }
    if (o < nn) Upk[i * nn + o] = acc;
  }
}

// Eight orbitals (64 x 64 map) on the matrix cores: per chunk of 64 rows, wave w takes rows
// 16 w .. 16 w + 15 and all four 16-output tiles, U = W M^T accumulated in
// FP64 MFMA tiles (lane layout of k_moments_mfma) over the 64 columns, four
// per instruction; W rows staged in LDS (row stride 65), M transposed in LDS.
typedef double dvec4u_t __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(NT) k_build_U64_mfma(const DevMesh* __restrict__ dm, const double* __restrict__ W,
                                                       const double* __restrict__ Mr, double* __restrict__ Upk) {
  INSTANCE;
  __shared__ double sMT[64 * 64];
  __shared__ double sW[64 * 65];
  Mr += (int64_t)blockIdx.y * 64 * 64;
  W += d.oF * 64;
  Upk += d.oE * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int o = e >> 6, c = e & 63;
    sMT[c * 64 + o] = Mr[e];
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  for (int64_t base = (int64_t)blockIdx.x * 64; base < d.NE; base += (int64_t)gridDim.x * 64) {
    const int cnt = (int)((d.NE - base) < 64 ? (d.NE - base) : 64);
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += NT) {
      const int r = e >> 6, c = e & 63;
      sW[r * 65 + c] = r < cnt ? W[(base + r) * 64 + c] : 0.0;
    }
    __syncthreads();
    dvec4u_t acc[4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) acc[ot] = dvec4u_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int c0 = 0; c0 < 64; c0 += 4) {
      const double a = sW[(16 * wave + li) * 65 + c0 + lk];
#pragma unroll
      for (int ot = 0; ot < 4; ++ot) {
        const double bv = sMT[(c0 + lk) * 64 + 16 * ot + li];
        acc[ot] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[ot], 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * wave + 4 * v + lk;
      if (r < cnt)
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) Upk[(base + r) * 64 + 16 * ot + li] = acc[ot][v];
    }
  }
}

void launch_build_U_full(const Batch& b, const double* W, const double* Gamma, const int* colmap, double* Mr,
                         double* Upk, hipStream_t s) {
  const int nn = b.mx.n * b.mx.n;
  hipLaunchKernelGGL(k_build_Mreal, dim3(nblocks(nn * nn), b.ni), dim3(NT), 0, s, (const double2*)Gamma, b.mx.n,
                     colmap, Mr);
  const int g = nblocks(b.mx.NE * 64, NT, 8192);
  if (nn <= 1) hipLaunchKernelGGL(k_build_U<1>, dim3(g, b.ni), dim3(NT), 0, s, b.dm, W, Mr, Upk);
  else if (nn <= 4) hipLaunchKernelGGL(k_build_U<4>, dim3(g, b.ni), dim3(NT), 0, s, b.dm, W, Mr, Upk);
  else if (nn <= 16) hipLaunchKernelGGL(k_build_U<16>, dim3(g, b.ni), dim3(NT), 0, s, b.dm, W, Mr, Upk);
  else if (nn < 64) hipLaunchKernelGGL(k_build_U<64>, dim3(g, b.ni), dim3(NT), 0, s, b.dm, W, Mr, Upk);
  else hipLaunchKernelGGL(k_build_U64_mfma, dim3(nblocks(b.mx.NE, 64, 8192), b.ni), dim3(NT), 0, s, b.dm, W, Mr, Upk);
}

// =====================================================================
// Krylov (Arnoldi) pieces.  M-inner product over the packed orbital vector:
// <u,v> = sum_i m_i sum_p conj(u_ip) v_ip on rows [0, NE) of each instance.
// Per-instance strides: H (m_max+1) m_max, hcur m_max+1, y m_max, scal 8,
// partials nblk (2 (m_max+1) + 1).
// =====================================================================
constexpr int KMAX = 25;

__device__ __forceinline__ int64_t kpart_stride(int nblk, int m_max) { return (int64_t)nblk * (2 * (m_max + 1) + 1); }

__global__ void __launch_bounds__(NT) k_mdot(const DevMesh* __restrict__ dm, const double2* const* __restrict__ V,
                                             int k, const double2* __restrict__ w, int with_norm, int m_max,
                                             double* __restrict__ part) {
  INSTANCE;
  __shared__ double lw[NT / 64][2 * KMAX + 1];
  const int n = d.n;
  const int64_t total = d.NE * n, o = d.oE * n;
  double hr[KMAX], hi[KMAX], nrm = 0.0;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) { hr[j] = 0.0; hi[j] = 0.0; }
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const double mi = gbl(d.m)[e / n];
    const double2 w0 = w[o + e];
    const double2 we = make_double2(mi * w0.x, mi * w0.y);
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j <= k) {
        double2 vj = ldg2(V[j], o + e);
        hr[j] += vj.x * we.x + vj.y * we.y;
        hi[j] += vj.x * we.y - vj.y * we.x;
      }
    }
    if (with_norm) nrm += we.x * w0.x + we.y * w0.y;
  }
  // every value reduced over its wave by shuffles, then the four waves
  // combined after one barrier
  const int nv = 2 * (k + 1) + 1;
  double* pb = part + blockIdx.y * kpart_stride(gridDim.x, m_max) + (int64_t)blockIdx.x * nv;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j <= k) {
      const double a = wave_sum(hr[j]), b = wave_sum(hi[j]);
      if (lane == 0) {
        lw[wid][2 * j] = a;
        lw[wid][2 * j + 1] = b;
      }
    }
  }
  const double c = wave_sum(nrm);
  if (lane == 0) lw[wid][nv - 1] = c;
  __syncthreads();
  if (threadIdx.x < (unsigned)nv) pb[threadIdx.x] = lw[0][threadIdx.x] + lw[1][threadIdx.x] + lw[2][threadIdx.x] + lw[3][threadIdx.x];
}

// Finish the dots, one workgroup per value: pass 1 sets column k of H, pass 2
// adds (re-orthogonalisation).
__global__ void __launch_bounds__(NT) k_mdot_finish(const double* __restrict__ part, int nblk, int k, int m_max,
                                                    int pass, double2* __restrict__ H, double2* __restrict__ hcur,
                                                    double* __restrict__ scal) {
  __shared__ double lds4[4];
  const int i = blockIdx.y, v = blockIdx.x;
  part += i * kpart_stride(nblk, m_max);
  H += (int64_t)i * (m_max + 1) * m_max;
  hcur += (int64_t)i * (m_max + 1);
  scal += 8 * i;
  const int nv = 2 * (k + 1) + 1;
  if (pass == 2 && scal[6] != 0.0) return;  // one Gram-Schmidt pass was enough (k_orth_decide)
  const double s = sum_partials(part, nblk, nv, v, lds4);
  if (threadIdx.x != 0) return;
  if (v == nv - 1) {
    if (pass == 1) scal[2] = s;
    return;
  }
  const int j = v >> 1;
  double* hc = (double*)&hcur[j];
  hc[v & 1] = s;
  double* hp = (double*)&H[j + (int64_t)(m_max + 1) * k];
  if (pass == 1) hp[v & 1] = s;
  else hp[v & 1] += s;
}

void launch_mdot(const Batch& b, double* const* V, int k, const double* w, Krylov& K, int pass, hipStream_t s) {
  hipLaunchKernelGGL(k_mdot, dim3(K.nblk, b.ni), dim3(NT), 0, s, b.dm, (const double2* const*)V, k,
                     (const double2*)w, pass == 1 ? 1 : 0, K.m_max, K.part);
  hipLaunchKernelGGL(k_mdot_finish, dim3(2 * (k + 1) + 1, b.ni), dim3(NT), 0, s, K.part, K.nblk, k, K.m_max, pass,
                     (double2*)K.H, (double2*)K.hcur, K.scal);
}

// Whether the first classical Gram-Schmidt pass suffices (the criterion of
// Daniel, Gragg, Kaufman and Stewart 1976, on the norm kept by the pass):
// with the basis orthonormal, |w - V h|^2 = |w|^2 - sum |h_j|^2 after the
// first pass.  One pass leaves the new vector orthogonal to the basis to about
// the dots' rounding error times |w| / |w - V h| (measured on random bases of
// 200,000 rows: 6e-16 at a kept fraction of 0.7, 5e-15 at 0.1), so while the
// pass keeps at least a tenth of |w| (1/100 of |w|^2) the second pass is
// skipped (scal[6] = 1): the fused update then forms the norm, and the second
// update and dot finish return at once.
__global__ void k_orth_decide(const double2* __restrict__ hcur, double* __restrict__ scal, int k, int m_max) {
  if (threadIdx.x != 0) return;
  const int i = blockIdx.x;
  hcur += (int64_t)i * (m_max + 1);
  scal += 8 * i;
  double hs = 0.0;
  for (int j = 0; j <= k; ++j) hs += hcur[j].x * hcur[j].x + hcur[j].y * hcur[j].y;
  const double w2 = scal[2];
  scal[6] = (w2 > 0.0 && w2 - hs >= 0.01 * w2) ? 1.0 : 0.0;
}

__global__ void __launch_bounds__(NT) k_orth_update(const DevMesh* __restrict__ dm,
                                                    const double2* const* __restrict__ V, int k,
                                                    double2* __restrict__ w, const double2* __restrict__ hcur,
                                                    int with_norm, int m_max, double* __restrict__ part,
                                                    const double* __restrict__ scal) {
  INSTANCE;
  if (with_norm && scal[8 * blockIdx.y + 6] != 0.0) return;  // the first pass was enough
  __shared__ double lds[8];
  const int n = d.n;
  const int64_t total = d.NE * n, o = d.oE * n;
  hcur += (int64_t)blockIdx.y * (m_max + 1);
  double2 h[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) h[j] = (j <= k) ? hcur[j] : make_double2(0.0, 0.0);
  double nrm = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    double2 we = w[o + e];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
      if (j <= k) we = csub(we, cmul(h[j], ldg2(V[j], o + e)));
    w[o + e] = we;
    if (with_norm) nrm += gbl(d.m)[e / n] * (we.x * we.x + we.y * we.y);
  }
  if (with_norm) {
    double c = block_sum(nrm, lds);
    if (threadIdx.x == 0) part[blockIdx.y * kpart_stride(gridDim.x, m_max) + blockIdx.x] = c;
  }
}

// The first update of CGS2 fused with the second pass's dot products:
// w -= sum_j V_j hcur_j, then the partials of V_j^H M w (layout of k_mdot,
// norm slot 0).  KM >= k + 1 sizes the register arrays.
template <int KM>
__global__ void __launch_bounds__(NT) k_orth_dot(const DevMesh* __restrict__ dm, const double2* const* __restrict__ V,
                                                 int k, double2* __restrict__ w, const double2* __restrict__ hcur,
                                                 int m_max, double* __restrict__ part, const double* __restrict__ scal) {
  INSTANCE;
  __shared__ double lw[NT / 64][2 * KM + 1];
  const int n = d.n;
  const int64_t total = d.NE * n, o = d.oE * n;
  hcur += (int64_t)blockIdx.y * (m_max + 1);
  if (scal[8 * blockIdx.y + 6] != 0.0) {
    // single pass: w -= sum_j V_j hcur_j and the partials of |w|_M^2 (layout of
    // the norm after the second update)
    double2 h[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) h[j] = (j <= k) ? hcur[j] : make_double2(0.0, 0.0);
    double nrm = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
      double2 we = w[o + e];
#pragma unroll
      for (int j = 0; j < KM; ++j)
        if (j <= k) we = csub(we, cmul(h[j], ldg2(V[j], o + e)));
      w[o + e] = we;
      nrm += gbl(d.m)[e / n] * (we.x * we.x + we.y * we.y);
    }
    const double c = block_sum(nrm, &lw[0][0]);
    if (threadIdx.x == 0) part[blockIdx.y * kpart_stride(gridDim.x, m_max) + blockIdx.x] = c;
    return;
  }
  double2 h[KM];
  double hr[KM], hi[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    h[j] = (j <= k) ? hcur[j] : make_double2(0.0, 0.0);
    hr[j] = 0.0;
    hi[j] = 0.0;
  }
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    double2 we = w[o + e];
    double2 vj[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j <= k) {
        vj[j] = ldg2(V[j], o + e);
        we = csub(we, cmul(h[j], vj[j]));
      }
    w[o + e] = we;
    const double mi = gbl(d.m)[e / n];
    const double2 wm = make_double2(mi * we.x, mi * we.y);
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j <= k) {
        hr[j] += vj[j].x * wm.x + vj[j].y * wm.y;
        hi[j] += vj[j].x * wm.y - vj[j].y * wm.x;
      }
  }
  const int nv = 2 * (k + 1) + 1;
  double* pb = part + blockIdx.y * kpart_stride(gridDim.x, m_max) + (int64_t)blockIdx.x * nv;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < KM; ++j)
    if (j <= k) {
      const double a = wave_sum(hr[j]), b = wave_sum(hi[j]);
      if (lane == 0) {
        lw[wid][2 * j] = a;
        lw[wid][2 * j + 1] = b;
      }
    }
  if (lane == 0) lw[wid][nv - 1] = 0.0;
  __syncthreads();
  if (threadIdx.x < (unsigned)nv)
    pb[threadIdx.x] = lw[0][threadIdx.x] + lw[1][threadIdx.x] + lw[2][threadIdx.x] + lw[3][threadIdx.x];
}

// h_{k+1,k} = |w|; happy breakdown when h <= 1e-14 |G v_k| (then scale 0).
__global__ void k_norm_finish(const double* __restrict__ part, int nblk, int k, int m_max, double2* __restrict__ H,
                              double* __restrict__ scal) {
  __shared__ double lds4[4];
  const int i = blockIdx.y;
  part += i * kpart_stride(nblk, m_max);
  H += (int64_t)i * (m_max + 1) * m_max;
  scal += 8 * i;
  const double s = sum_partials(part, nblk, 1, 0, lds4);
  if (threadIdx.x != 0) return;
  double h = sqrt(s);
  double wn = sqrt(scal[2]);
  H[(k + 1) + (int64_t)(m_max + 1) * k] = make_double2(h, 0.0);
  if (h <= 1e-14 * wn || !(h > 0.0)) {
    scal[1] = 0.0;
    if (scal[4] > k + 1) scal[4] = k + 1;
  } else {
    scal[1] = 1.0 / h;
  }
}

void launch_orth_update(const Batch& b, double* const* V, int k, double* w, Krylov& K, int pass, hipStream_t s) {
  hipLaunchKernelGGL(k_orth_update, dim3(K.nblk, b.ni), dim3(NT), 0, s, b.dm, (const double2* const*)V, k,
                     (double2*)w, (const double2*)K.hcur, pass == 2 ? 1 : 0, K.m_max, K.part, (const double*)K.scal);
  if (pass == 2)
    hipLaunchKernelGGL(k_norm_finish, dim3(1, b.ni), dim3(NT), 0, s, K.part, K.nblk, k, K.m_max, (double2*)K.H,
                       K.scal);
}

void launch_orth_dot(const Batch& b, double* const* V, int k, double* w, Krylov& K, hipStream_t s) {
  const dim3 g(K.nblk, b.ni);
  const auto* Vc = (const double2* const*)V;
  const double* sc = K.scal;
  hipLaunchKernelGGL(k_orth_decide, dim3(b.ni), dim3(64), 0, s, (const double2*)K.hcur, K.scal, k, K.m_max);
  if (k + 1 <= 4)
    hipLaunchKernelGGL(k_orth_dot<4>, g, dim3(NT), 0, s, b.dm, Vc, k, (double2*)w, (const double2*)K.hcur, K.m_max,
                       K.part, sc);
  else if (k + 1 <= 8)
    hipLaunchKernelGGL(k_orth_dot<8>, g, dim3(NT), 0, s, b.dm, Vc, k, (double2*)w, (const double2*)K.hcur, K.m_max,
                       K.part, sc);
  else if (k + 1 <= 13)
    hipLaunchKernelGGL(k_orth_dot<13>, g, dim3(NT), 0, s, b.dm, Vc, k, (double2*)w, (const double2*)K.hcur, K.m_max,
                       K.part, sc);
  else
    hipLaunchKernelGGL(k_orth_dot<KMAX>, g, dim3(NT), 0, s, b.dm, Vc, k, (double2*)w, (const double2*)K.hcur,
                       K.m_max, K.part, sc);
  hipLaunchKernelGGL(k_mdot_finish, dim3(2 * (k + 1) + 1, b.ni), dim3(NT), 0, s, K.part, K.nblk, k, K.m_max, 2,
                     (double2*)K.H, (double2*)K.hcur, K.scal);
}

__global__ void k_scale_by(const DevMesh* __restrict__ dm, const double2* __restrict__ src,
                           double2* __restrict__ dst, const double* __restrict__ scal, int which) {
  INSTANCE;
  const int64_t total = d.NE * d.n, o = d.oE * d.n;
  const double f = scal[8 * blockIdx.y + which];
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT)
    dst[o + e] = cscale(f, src[o + e]);
}

void launch_krylov_scale(const Batch& b, const double* src, double* dst, Krylov& K, int which, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_by, dim3(nblocks(b.mx.NE * b.mx.n, NT, 8192), b.ni), dim3(NT), 0, s, b.dm,
                     (const double2*)src, (double2*)dst, K.scal, which);
}

__global__ void __launch_bounds__(NT) k_norm_part(const DevMesh* __restrict__ dm, const double2* __restrict__ x,
                                                  int m_max, double* __restrict__ part) {
  INSTANCE;
  __shared__ double lds[8];
  const int n = d.n;
  const int64_t total = d.NE * n, o = d.oE * n;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const double2 v = x[o + e];
    s += gbl(d.m)[e / n] * (v.x * v.x + v.y * v.y);
  }
  double c = block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.y * kpart_stride(gridDim.x, m_max) + blockIdx.x] = c;
}

__global__ void k_beta_finish(const double* __restrict__ part, int nblk, int m, double* __restrict__ scal,
                              double2* __restrict__ H, int m_max) {
  const int i = blockIdx.y;
  part += i * kpart_stride(nblk, m_max);
  H += (int64_t)i * (m_max + 1) * m_max;
  scal += 8 * i;
  for (int t = threadIdx.x; t < (m_max + 1) * m_max; t += blockDim.x) H[t] = make_double2(0.0, 0.0);
  __shared__ double lds4[4];
  const double s = sum_partials(part, nblk, 1, 0, lds4);
  if (threadIdx.x != 0) return;
  double beta = sqrt(s);
  scal[0] = beta;
  scal[5] = beta > 0.0 ? 1.0 / beta : 0.0;
  scal[4] = m;
  scal[3] = 0.0;
}

void launch_norm_init(const Batch& b, const double* phi, Krylov& K, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_part, dim3(K.nblk, b.ni), dim3(NT), 0, s, b.dm, (const double2*)phi, K.m_max, K.part);
  hipLaunchKernelGGL(k_beta_finish, dim3(1, b.ni), dim3(NT), 0, s, K.part, K.nblk, m, K.scal, (double2*)K.H,
                     K.m_max);
}

// y = beta expm(A) e1, A = -i tau H_m (m = scal[4]); scaling and squaring
// with a degree-18 Taylor polynomial at |A/2^s|_1 <= 1/2 (remainder below
// 1e-22).  One workgroup per instance; matrices in LDS.
// m_try > 0 (adaptive dimension): only the error estimate of dimension m_try,
// beta h_{m_try+1,m_try} |e_{m_try}^T expm(A_{m_try}) e1|; where it is at or
// below tol the instance's dimension scal[4] becomes m_try (instances whose
// space already ended, by breakdown or an earlier estimate, are left alone).
__global__ void __launch_bounds__(NT) k_expm(const double2* __restrict__ H, int m_max, double tau_re, double tau_im,
                                             double* __restrict__ scal, double2* __restrict__ y, int m_try,
                                             double tol) {
  __shared__ double2 A[KMAX * KMAX], T[KMAX * KMAX], S[KMAX * KMAX];
  __shared__ int sh_s;
  __shared__ double sh_norm;
  const int inst = blockIdx.y;
  H += (int64_t)inst * (m_max + 1) * m_max;
  scal += 8 * inst;
  y += (int64_t)inst * m_max;
  if (m_try > 0 && (int)scal[4] <= m_try) return;  // uniform over the workgroup
  const int m = m_try > 0 ? m_try : (int)scal[4];
  const int mm = m * m;
  // A = -i tau H = (tau_im - i tau_re) H
  const double2 f = make_double2(tau_im, -tau_re);
  for (int e = threadIdx.x; e < mm; e += NT) {
    int i = e / m, j = e - i * m;
    A[e] = cmul(f, H[i + (int64_t)(m_max + 1) * j]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double nrm = 0.0;
    for (int j = 0; j < m; ++j) {
      double c = 0.0;
      for (int i = 0; i < m; ++i) c += hypot(A[i * m + j].x, A[i * m + j].y);
      nrm = fmax(nrm, c);
    }
    int s = 0;
    while (nrm > 0.5 && s < 60) { nrm *= 0.5; ++s; }
    sh_s = s;
    sh_norm = ldexp(1.0, -s);
  }
  __syncthreads();
  const int s = sh_s;
  for (int e = threadIdx.x; e < mm; e += NT) A[e] = cscale(sh_norm, A[e]);
  // Horner: T = I + A/18; T = I + A T / k for k = 17..1
  for (int e = threadIdx.x; e < mm; e += NT) {
    int i = e / m, j = e - i * m;
    T[e] = cscale(1.0 / 18.0, A[e]);
    if (i == j) T[e].x += 1.0;
  }
  __syncthreads();
  for (int k = 17; k >= 1; --k) {
    for (int e = threadIdx.x; e < mm; e += NT) {
      int i = e / m, j = e - i * m;
      double2 acc = make_double2(0.0, 0.0);
      for (int l = 0; l < m; ++l) acc = cadd(acc, cmul(A[i * m + l], T[l * m + j]));
      acc = cscale(1.0 / k, acc);
      if (i == j) acc.x += 1.0;
      S[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < mm; e += NT) T[e] = S[e];
    __syncthreads();
  }
  for (int q = 0; q < s; ++q) {
    for (int e = threadIdx.x; e < mm; e += NT) {
      int i = e / m, j = e - i * m;
      double2 acc = make_double2(0.0, 0.0);
      for (int l = 0; l < m; ++l) acc = cadd(acc, cmul(T[i * m + l], T[l * m + j]));
      S[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < mm; e += NT) T[e] = S[e];
    __syncthreads();
  }
  const double beta = scal[0];
  if (m_try > 0) {
    if (threadIdx.x == 0) {
      const double2 hlast = H[m + (int64_t)(m_max + 1) * (m - 1)];
      const double2 ylast = T[(m - 1) * m];
      if (beta * hypot(hlast.x, hlast.y) * hypot(ylast.x, ylast.y) <= tol) scal[4] = m;
    }
    return;
  }
  for (int i = threadIdx.x; i < m_max; i += NT) y[i] = (i < m) ? cscale(beta, T[i * m]) : make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    double2 hlast = H[m + (int64_t)(m_max + 1) * (m - 1)];
    double2 ylast = T[(m - 1) * m];
    scal[3] = beta * hypot(hlast.x, hlast.y) * hypot(ylast.x, ylast.y);
  }
}

void launch_expm(int ni, Krylov& K, double tau_re, double tau_im, hipStream_t s) {
  hipLaunchKernelGGL(k_expm, dim3(1, ni), dim3(NT), 0, s, (const double2*)K.H, K.m_max, tau_re, tau_im, K.scal,
                     (double2*)K.y, 0, 0.0);
}

void launch_krylov_check(int ni, Krylov& K, double tau_re, double tau_im, int m_try, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_expm, dim3(1, ni), dim3(NT), 0, s, (const double2*)K.H, K.m_max, tau_re, tau_im, K.scal,
                     (double2*)K.y, m_try, tol);
}

__global__ void __launch_bounds__(NT) k_combine(const DevMesh* __restrict__ dm, const double2* const* __restrict__ V,
                                                int m, int m_max, double2* __restrict__ phi,
                                                const double2* __restrict__ y) {
  INSTANCE;
  const int64_t total = d.NE * d.n, o = d.oE * d.n;
  y += (int64_t)blockIdx.y * m_max;
  double2 yy[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) yy[j] = (j < m) ? y[j] : make_double2(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
      if (j < m) s = cadd(s, cmul(yy[j], ldg2(V[j], o + e)));
    phi[o + e] = s;
  }
}

void launch_combine(const Batch& b, double* const* V, int m, double* phi, Krylov& K, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(nblocks(b.mx.NE * b.mx.n, NT, 8192), b.ni), dim3(NT), 0, s, b.dm,
                     (const double2* const*)V, m, K.m_max, (double2*)phi, (const double2*)K.y);
}

// =====================================================================
// Poisson: moments, boundary values, right-hand side.  Column c of the n^2
// real columns is (r, s, part) = colinfo[c].
// =====================================================================
constexpr int MP_CH = 32;

__device__ __forceinline__ double pair_density(const double2* phi, int n, int64_t i, int r, int s, int part) {
  double2 a = phi[i * n + r], b = phi[i * n + s];
  // conj(a) b
  return part == 0 ? (a.x * b.x + a.y * b.y) : (a.x * b.y - a.y * b.x);
}

// Multipole moments Q[t][c] = sum_i R_t(x_i) m_i rho_c(x_i) of the pair
// densities, per instance, with register tiles: each thread accumulates a
// tile of MT_H harmonics x MT_C columns, so every pair of LDS reads (one
// harmonic quadruple, one column quadruple) feeds 16 FMAs.  Tiles are
// numbered column-tile fastest; grid.z splits the tiles in sets of NT.
constexpr int MT_H = 4, MT_C = 4;
constexpr int MP_HP = 172;  // harmonics padded to a multiple of MT_H
__global__ void __launch_bounds__(NT) k_moments_rb(const DevMesh* __restrict__ dm, const double2* __restrict__ phi,
                                                   int lmax, int ncol, const int* __restrict__ colinfo,
                                                   double* __restrict__ part) {
  INSTANCE;
  __shared__ double sR[MP_CH * MP_HP];
  __shared__ double sW[MP_CH * 64];
  const int nh = (lmax + 1) * (lmax + 1);
  const int nhp = (nh + MT_H - 1) / MT_H * MT_H;
  const int ncp = (ncol + MT_C - 1) / MT_C * MT_C;
  const int nout = nh * ncol;
  const int n = d.n;
  phi += d.oE * n;
  const double cx = d.center[0], cy = d.center[1], cz = d.center[2];
  const int tiles_c = ncp / MT_C, tiles = (nhp / MT_H) * tiles_c;
  const int tile = blockIdx.z * NT + threadIdx.x;
  const bool act = tile < tiles;
  const int t0 = act ? (tile / tiles_c) * MT_H : 0, c0 = act ? (tile % tiles_c) * MT_C : 0;
  double acc[MT_H][MT_C];
#pragma unroll
  for (int a = 0; a < MT_H; ++a)
#pragma unroll
    for (int b = 0; b < MT_C; ++b) acc[a][b] = 0.0;
  const int64_t rows = d.NE;
  for (int64_t base = (int64_t)blockIdx.x * MP_CH; base < rows; base += (int64_t)gridDim.x * MP_CH) {
    const int cnt = (int)((rows - base) < MP_CH ? (rows - base) : MP_CH);
    __syncthreads();
    // harmonics of the chunk's rows, one (row, order m) per thread; padding zero
    for (int w = threadIdx.x; w < MP_CH * (lmax + 1); w += NT) {
      const int r = w / (lmax + 1), m = w - r * (lmax + 1);
      double* R = sR + r * nhp;
      if (r < cnt) {
        const int64_t i = base + r;
        solid_regular_m(d.xyz[3 * i] - cx, d.xyz[3 * i + 1] - cy, d.xyz[3 * i + 2] - cz, lmax, m, R);
      } else {
        for (int l = m; l <= lmax; ++l) {
          R[l * l + m] = 0.0;
          if (m > 0) R[l * l + l + m] = 0.0;
        }
      }
    }
    if (nhp > nh)
      for (int e = threadIdx.x; e < MP_CH * (nhp - nh); e += NT) sR[(e / (nhp - nh)) * nhp + nh + e % (nhp - nh)] = 0.0;
    for (int e = threadIdx.x; e < MP_CH * ncp; e += NT) {
      const int r = e / ncp, c = e - r * ncp;
      double v = 0.0;
      if (r < cnt && c < ncol) {
        const int64_t i = base + r;
        const int ci = colinfo[c];
        v = d.m[i] * pair_density(phi, n, i, ci & 255, (ci >> 8) & 255, ci >> 16);
      }
      sW[r * ncp + c] = v;
    }
    __syncthreads();
    if (act)
      for (int r = 0; r < cnt; ++r) {
        double hv[MT_H], wv[MT_C];
#pragma unroll
        for (int a = 0; a < MT_H; ++a) hv[a] = sR[r * nhp + t0 + a];
#pragma unroll
        for (int b = 0; b < MT_C; ++b) wv[b] = sW[r * ncp + c0 + b];
#pragma unroll
        for (int a = 0; a < MT_H; ++a)
#pragma unroll
          for (int b = 0; b < MT_C; ++b) acc[a][b] += hv[a] * wv[b];
      }
  }
  if (!act) return;
  double* pb = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * nout;
#pragma unroll
  for (int a = 0; a < MT_H; ++a)
#pragma unroll
    for (int b = 0; b < MT_C; ++b)
      if (t0 + a < nh && c0 + b < ncol) pb[(t0 + a) * ncol + c0 + b] = acc[a][b];
}
// The same moments on the matrix cores (16 or more columns): per chunk of
// MP_CH rows the harmonics R[row][h] and the weighted pair densities
// W[row][c] are staged in LDS once, and Q[h][c] += sum over rows of
// R[row][h] W[row][c] accumulates in FP64 MFMA tiles of 16 harmonics x 16
// columns, four rows per instruction.  The (harmonic tile, column tile)
// pairs are dealt round-robin to the four waves, at most MM_TW per wave.
// Lane layout of v_mfma_f64_16x16x4_f64 (measured): A[i][k] from lane 16 k + i,
// B[k][j] from lane 16 k + j, and accumulator v of lane l holds
// D[4 v + l / 16][l % 16].
constexpr int MM_HP = 176;  // harmonics padded to a multiple of 16 (lmax <= 12: 169)
constexpr int MM_TW = 11;   // 11 harmonic tiles x 4 column tiles over 4 waves
constexpr int MM_CH = 16;   // rows per chunk (30.5 KB of LDS: five workgroups per compute unit)
typedef double dvec4_t __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(NT) k_moments_mfma(const DevMesh* __restrict__ dm, const double2* __restrict__ phi,
                                                     int lmax, int ncol, const int* __restrict__ colinfo,
                                                     double* __restrict__ part) {
  INSTANCE;
  __shared__ double sR[MM_CH * MM_HP];
  __shared__ double sW[MM_CH * 64];
  const int nh = (lmax + 1) * (lmax + 1);
  const int nct = (ncol + 15) / 16, ntile = ((nh + 15) / 16) * nct;
  const int nout = nh * ncol;
  const int n = d.n;
  phi += d.oE * n;
  const double cx = d.center[0], cy = d.center[1], cz = d.center[2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  dvec4_t acc[MM_TW];
#pragma unroll
  for (int j = 0; j < MM_TW; ++j) acc[j] = dvec4_t{0.0, 0.0, 0.0, 0.0};
  const int64_t rows = d.NE;
  for (int64_t base = (int64_t)blockIdx.x * MM_CH; base < rows; base += (int64_t)gridDim.x * MM_CH) {
    const int cnt = (int)((rows - base) < MM_CH ? (rows - base) : MM_CH);
    __syncthreads();
    for (int w = threadIdx.x; w < MM_CH * (lmax + 1); w += NT) {
      const int r = w / (lmax + 1), m = w - r * (lmax + 1);
      double* R = sR + r * MM_HP;
      if (r < cnt) {
        const int64_t i = base + r;
        solid_regular_m(d.xyz[3 * i] - cx, d.xyz[3 * i + 1] - cy, d.xyz[3 * i + 2] - cz, lmax, m, R);
      } else {
        for (int l = m; l <= lmax; ++l) {
          R[l * l + m] = 0.0;
          if (m > 0) R[l * l + l + m] = 0.0;
        }
      }
    }
    for (int e = threadIdx.x; e < MM_CH * (MM_HP - nh); e += NT)
      sR[(e / (MM_HP - nh)) * MM_HP + nh + e % (MM_HP - nh)] = 0.0;
    for (int e = threadIdx.x; e < MM_CH * 64; e += NT) {
      const int r = e >> 6, c = e & 63;
      double v = 0.0;
      if (r < cnt && c < ncol) {
        const int64_t i = base + r;
        const int ci = colinfo[c];
        v = d.m[i] * pair_density(phi, n, i, ci & 255, (ci >> 8) & 255, ci >> 16);
      }
      sW[e] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < MM_CH; k0 += 4) {
      const int kr = k0 + (lane >> 4), li = lane & 15;
#pragma unroll
      for (int j = 0; j < MM_TW; ++j) {
        const int tile = wave + 4 * j;
        if (tile < ntile) {
          const int t = tile / nct, u = tile - t * nct;
          const double a = sR[kr * MM_HP + 16 * t + li];
          const double b = sW[kr * 64 + 16 * u + li];
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        }
      }
    }
  }
  double* pb = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * nout;
#pragma unroll
  for (int j = 0; j < MM_TW; ++j) {
    const int tile = wave + 4 * j;
    if (tile >= ntile) continue;
    const int t = tile / nct, u = tile - t * nct;
    const int c = 16 * u + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int h = 16 * t + 4 * v + (lane >> 4);
      if (h < nh && c < ncol) pb[h * ncol + c] = acc[j][v];
    }
  }
}

// out[i][o] = sum_b part[i][b][o]; one workgroup per (output, instance)
__global__ void __launch_bounds__(NT) k_sum_parts_real(const double* __restrict__ part, int nblk, int nout,
                                                       double* __restrict__ out) {
  __shared__ double lds4[4];
  const double s = sum_partials(part + (int64_t)blockIdx.y * nblk * nout, nblk, nout, blockIdx.x, lds4);
  if (threadIdx.x == 0) out[(int64_t)blockIdx.y * nout + blockIdx.x] = s;
}

// W[NE + b][c] = sum_t table[b][t] Q[t][c]
__global__ void k_bnd_eval(const DevMesh* __restrict__ dm, int nh, const double* __restrict__ Q, int ncol,
                           double* __restrict__ W) {
  INSTANCE;
  const int64_t total = d.Nb * ncol;
  Q += (int64_t)blockIdx.y * nh * ncol;
  W += d.oF * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    int64_t b = e / ncol;
    int c = (int)(e - b * ncol);
    double s = 0.0;
    for (int t = 0; t < nh; ++t) s += d.bnd_table[b * nh + t] * Q[t * ncol + c];
    W[(d.NE + b) * ncol + c] = s;
  }
}

// Boundary lift through the element stiffness: acc += K_full x over the
// listed boundary cells, with x the lift (boundary rows and the boundary-
// master share of hanging rows; DoF rows read as zero).  x over full rows,
// acc over extended rows; boundary rows of acc are skipped.
template <int P>
__global__ void __launch_bounds__(NT) k_lift_poisson(const DevMesh* __restrict__ dm, const double* __restrict__ x,
                                                     double* __restrict__ acc, int ncol) {
  INSTANCE;
  constexpr int P3 = P * P * P;
  __shared__ double sx[P3 * 64];
  __shared__ int snode[P3];
  x += d.oF * ncol;
  acc += d.oE * ncol;
  for (int64_t cb = blockIdx.x; cb < d.n_bnd_cells; cb += gridDim.x) {
    const int64_t e = d.bnd_cells[cb];
    __syncthreads();
    for (int t = threadIdx.x; t < P3; t += NT) snode[t] = d.cell_nodes[e * P3 + t];
    __syncthreads();
    for (int idx = threadIdx.x; idx < P3 * ncol; idx += NT) {
      int t = idx / ncol, c = idx - t * ncol;
      int node = snode[t];
      double v = 0.0;
      if (node >= d.NE) {
        v = x[(int64_t)node * ncol + c];
      } else if (node >= d.N) {
        int64_t h = node - d.N;
        for (int k = d.hang_ptr[h]; k < d.hang_ptr[h + 1]; ++k)
          if (d.hang_col[k] >= d.NE) v += d.hang_w[k] * x[(int64_t)d.hang_col[k] * ncol + c];
      }
      sx[c * P3 + t] = v;
    }
    __syncthreads();
    const double hh = d.cell_hh[e];
    for (int idx = threadIdx.x; idx < P3 * ncol; idx += NT) {
      int t = idx / ncol, c = idx - t * ncol;
      int node = snode[t];
      if (node >= d.NE) continue;
      int a = t % P, b = (t / P) % P, cc = t / (P * P);
      const double* xo = sx + c * P3;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        s0 += d.A[a * P + q] * xo[(cc * P + b) * P + q];
        s1 += d.A[b * P + q] * xo[(cc * P + q) * P + a];
        s2 += d.A[cc * P + q] * xo[(q * P + b) * P + a];
      }
      double y = hh * (d.w[b] * d.w[cc] * s0 + d.w[a] * d.w[cc] * s1 + d.w[a] * d.w[b] * s2);
      atomicAdd(acc + (int64_t)node * ncol + c, y);
    }
  }
}

static void launch_lift_poisson(const Batch& b, const double* x, double* acc, int ncol, hipStream_t s) {
  const int64_t ncell = b.mx.n_bnd_cells;
  if (ncell == 0) return;
  const dim3 g((unsigned)(ncell < 65536 ? ncell : 65536), b.ni);
  switch (b.mx.P) {
    case 2: hipLaunchKernelGGL(k_lift_poisson<2>, g, dim3(NT), 0, s, b.dm, x, acc, ncol); break;
    case 3: hipLaunchKernelGGL(k_lift_poisson<3>, g, dim3(NT), 0, s, b.dm, x, acc, ncol); break;
    default: hipLaunchKernelGGL(k_lift_poisson<4>, g, dim3(NT), 0, s, b.dm, x, acc, ncol);
  }
}

// Hanging rows of a real column array; with_bnd includes boundary masters.
__global__ void k_fill_real(const DevMesh* __restrict__ dm, double* __restrict__ x, int xfull, int ncol,
                            int with_bnd, double* __restrict__ acc) {
  INSTANCE;
  const int64_t total = d.Nh * ncol;
  x += (xfull ? d.oF : d.oE) * ncol;
  if (acc) acc += d.oE * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    int64_t h = e / ncol;
    int c = (int)(e - h * ncol);
    double s = 0.0;
    for (int t = d.hang_ptr[h]; t < d.hang_ptr[h + 1]; ++t) {
      int col = d.hang_col[t];
      if (col < d.N || with_bnd) s += d.hang_w[t] * x[(int64_t)col * ncol + c];
    }
    x[(d.N + h) * ncol + c] = s;
    if (acc) acc[(d.N + h) * ncol + c] = 0.0;
  }
}

void launch_fill_real(const Batch& b, double* x, int xfull, int ncol, int with_bnd, double* acc, hipStream_t s) {
  if (b.mx.Nh == 0) return;
  hipLaunchKernelGGL(k_fill_real, dim3(nblocks(b.mx.Nh * ncol), b.ni), dim3(NT), 0, s, b.dm, x, xfull, ncol,
                     with_bnd, acc);
}

// Zero rows [lo, hi) (lo, hi: 0 = 0, 1 = N, 2 = NE) of a real column array over extended rows.
__global__ void k_zero_rows(const DevMesh* __restrict__ dm, double* __restrict__ x, int ncol, int lo, int hi) {
  INSTANCE;
  const int64_t r0 = lo == 0 ? 0 : (lo == 1 ? d.N : d.NE), r1 = hi == 0 ? 0 : (hi == 1 ? d.N : d.NE);
  x += (d.oE + r0) * ncol;
  const int64_t total = (r1 - r0) * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) x[e] = 0.0;
}

// RHS: b = 4 pi C^T (m rho) - C^T acc;  partial |b|^2 (acc DoF rows zeroed).
__global__ void __launch_bounds__(NT) k_poisson_rhs(const DevMesh* __restrict__ dm, const double2* __restrict__ phi,
                                                    double* __restrict__ acc, int ncol,
                                                    const int* __restrict__ colinfo, double* __restrict__ rhs,
                                                    int64_t part_stride, double* __restrict__ part) {
  INSTANCE;
  __shared__ double lds[NT];
  const int groups = NT / ncol;
  const int g = threadIdx.x / ncol, c = threadIdx.x - g * ncol;
  const bool act = g < groups;
  double bb = 0.0;
  const int n = d.n;
  phi += d.oE * n;
  acc += d.oE * ncol;
  rhs += d.oE * ncol;
  const int ci = colinfo[act ? c : 0];
  const int r = ci & 255, s = (ci >> 8) & 255, pr = ci >> 16;
  if (act)
    for (int64_t k = (int64_t)blockIdx.x * groups + g; k < d.N; k += (int64_t)gridDim.x * groups) {
      double f = 4.0 * M_PI * d.m[k] * pair_density(phi, n, k, r, s, pr) - acc[k * ncol + c];
      acc[k * ncol + c] = 0.0;
      int mi = d.ma_index[k];
      if (mi >= 0)
        for (int t = d.ct_ptr[mi]; t < d.ct_ptr[mi + 1]; ++t) {
          int64_t h = d.ct_row[t];
          f += d.ct_w[t] * (4.0 * M_PI * d.m[h] * pair_density(phi, n, h, r, s, pr) - acc[h * ncol + c]);
        }
      rhs[k * ncol + c] = f;
      bb += f * f;
    }
  lds[threadIdx.x] = act ? bb : 0.0;
  __syncthreads();
  if (threadIdx.x < ncol) {
    double t = 0.0;
    for (int q = 0; q < groups; ++q) t += lds[q * ncol + threadIdx.x];
    part[blockIdx.y * part_stride + (int64_t)blockIdx.x * ncol + threadIdx.x] = t;
  }
}

// sc[i][slot][c] = sum_b part[i][b][c]; one workgroup per (column, instance)
__global__ void __launch_bounds__(NT) k_col_sum(const double* __restrict__ part, int64_t part_stride, int nblk,
                                                int ncol, double* __restrict__ sc, int slot) {
  __shared__ double lds4[4];
  const int c = blockIdx.x;
  const double s = sum_partials(part + blockIdx.y * part_stride, nblk, ncol, c, lds4);
  if (threadIdx.x == 0) sc[(int64_t)blockIdx.y * 8 * ncol + slot * ncol + c] = s;
}

static int rhs_blocks(const Batch& b, int ncol) { return nblocks(b.mx.N, NT / ncol, 1024); }

void launch_poisson_pipeline_moments(const Batch& b, const double* phi, const int* colinfo, PoissonWs& P,
                                     hipStream_t s) {
  const int nout = P.nharm * P.ncol;
  const double2* ph = (const double2*)phi;
  if (P.ncol >= 16 && P.ncol <= 64 && P.nharm <= MM_HP) {  // matrix cores: every tile in one workgroup
    hipLaunchKernelGGL(k_moments_mfma, dim3(P.mblk, b.ni), dim3(NT), 0, s, b.dm, ph, P.lmax, P.ncol, colinfo,
                       P.mpart);
  } else {
    // register tiles of 4 harmonics x 4 columns, sets of NT tiles over grid.z
    const int tiles = ((P.nharm + MT_H - 1) / MT_H) * ((P.ncol + MT_C - 1) / MT_C);
    const unsigned nz = (unsigned)((tiles + NT - 1) / NT);
    hipLaunchKernelGGL(k_moments_rb, dim3(P.mblk, b.ni, nz), dim3(NT), 0, s, b.dm, ph, P.lmax, P.ncol, colinfo,
                       P.mpart);
  }
  hipLaunchKernelGGL(k_sum_parts_real, dim3(nout, b.ni), dim3(NT), 0, s, P.mpart, P.mblk, nout, P.Q);
}

void launch_bnd_eval(const Batch& b, PoissonWs& P, double* W, hipStream_t s) {
  if (b.mx.Nb == 0) return;
  hipLaunchKernelGGL(k_bnd_eval, dim3(nblocks(b.mx.Nb * P.ncol), b.ni), dim3(NT), 0, s, b.dm, P.nharm, P.Q, P.ncol,
                     W);
}

void launch_poisson_rhs_full(const Batch& b, const double* phi, double* W, const int* colinfo, double* rhs,
                             PoissonWs& P, hipStream_t s) {
  const int ncol = P.ncol;
  launch_zero(P.acc, b.tE * ncol, s);  // the lift pass accumulates with atomics
  launch_lift_poisson(b, W, P.acc, ncol, s);
  const int nb = rhs_blocks(b, ncol);
  hipLaunchKernelGGL(k_poisson_rhs, dim3(nb, b.ni), dim3(NT), 0, s, b.dm, (const double2*)phi, P.acc, ncol, colinfo,
                     rhs, P.part_stride, P.part);
  hipLaunchKernelGGL(k_col_sum, dim3(ncol, b.ni), dim3(NT), 0, s, P.part, P.part_stride, nb, ncol, P.sc, (int)SC_BB);
  // hanging rows of acc back to zero
  if (b.mx.Nh > 0)
    hipLaunchKernelGGL(k_zero_rows, dim3(nblocks(b.mx.Nh * ncol, NT, 4096), b.ni), dim3(NT), 0, s, b.dm, P.acc,
                       ncol, 1, 2);
}

// =====================================================================
// Small dense kernels (one workgroup per instance, work on thread 0).
// =====================================================================
// Regularised inverse of the Hermitian 1-RDM: eigen-decomposition of the
// real 2n x 2n embedding [[Re, -Im], [Im, Re]] by Jacobi rotations, d -> d +
// eps exp(-d/eps), inverse from the eigenpairs.  One wave per instance with
// the matrices in LDS.  Each sweep runs 2n - 1 rounds of n disjoint pivot
// pairs (the round-robin ordering): the pairs' angles come from the entries
// at the start of the round, then all column rotations (of A and of the
// eigenvector matrix) and all row rotations are applied at once.  Disjoint
// rotations commute, so a round is the same as those rotations in sequence.
__device__ __forceinline__ double wave_sum_xor(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);  // every lane gets the same total
  return v;
}
__global__ void __launch_bounds__(64) k_ginv(const double2* __restrict__ gamma, int n, double eps,
                                             double2* __restrict__ ginv, int* __restrict__ flag) {
  __shared__ double a[16 * 16], V[16 * 16], dinv[16];
  __shared__ double rc[8], rs[8];
  __shared__ int rp[8], rq[8];
  __shared__ int badk[16];
  const int inst = blockIdx.x, lane = threadIdx.x;
  gamma += (int64_t)inst * n * n;
  ginv += (int64_t)inst * n * n;
  const int N2 = 2 * n, npair = n, m = N2 - 1;
  for (int e = lane; e < n * n; e += 64) {
    const int i = e / n, j = e - i * n;
    // Hermitian part
    const double re = 0.5 * (gamma[i * n + j].x + gamma[j * n + i].x);
    const double im = 0.5 * (gamma[i * n + j].y - gamma[j * n + i].y);
    a[i * N2 + j] = re;
    a[(i + n) * N2 + (j + n)] = re;
    a[i * N2 + (j + n)] = -im;
    a[(i + n) * N2 + j] = im;
  }
  for (int e = lane; e < N2 * N2; e += 64) V[e] = (e / N2 == e % N2) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = lane; e < N2 * N2; e += 64) {
      const double v = a[e];
      tot += v * v;
      if (e / N2 != e % N2) off += v * v;
    }
    off = wave_sum_xor(off);
    tot = wave_sum_xor(tot);
    // off-diagonal Frobenius norm at 1e-15 of the whole: above the rounding
    // floor of the rotations (about N2 eps^2 in the squares), so the sweeps stop
    // once converged instead of running to the cap on a stagnating remainder
    if (off <= 1e-30 * tot) break;
    for (int r = 0; r < m; ++r) {
      if (lane < npair) {
        // pair `lane` of round r: (N2 - 1, r) for lane 0, else (r + lane, r - lane) mod m
        int p = lane == 0 ? r : (r + lane) % m, q = lane == 0 ? N2 - 1 : (r - lane + m) % m;
        if (p > q) { const int t = p; p = q; q = t; }
        const double apq = a[p * N2 + q];
        double c = 1.0, sn = 0.0;
        if (fabs(apq) >= 1e-300) {
          const double theta = (a[q * N2 + q] - a[p * N2 + p]) / (2.0 * apq);
          const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          sn = t * c;
        }
        rp[lane] = p;
        rq[lane] = q;
        rc[lane] = c;
        rs[lane] = sn;
      }
      __syncthreads();
      for (int w = lane; w < npair * N2; w += 64) {  // columns p, q of a and V
        const int k = w / N2, i = w - k * N2;
        const int p = rp[k], q = rq[k];
        const double c = rc[k], sn = rs[k];
        const double aip = a[i * N2 + p], aiq = a[i * N2 + q];
        a[i * N2 + p] = c * aip - sn * aiq;
        a[i * N2 + q] = sn * aip + c * aiq;
        const double vip = V[i * N2 + p], viq = V[i * N2 + q];
        V[i * N2 + p] = c * vip - sn * viq;
        V[i * N2 + q] = sn * vip + c * viq;
      }
      __syncthreads();
      for (int w = lane; w < npair * N2; w += 64) {  // rows p, q of a
        const int k = w / N2, j = w - k * N2;
        const int p = rp[k], q = rq[k];
        const double c = rc[k], sn = rs[k];
        const double apj = a[p * N2 + j], aqj = a[q * N2 + j];
        a[p * N2 + j] = c * apj - sn * aqj;
        a[q * N2 + j] = sn * apj + c * aqj;
      }
      __syncthreads();
    }
  }
  if (lane < N2) {
    const double dk = a[lane * N2 + lane];
    const double dr = dk + eps * exp(-dk / eps);
    badk[lane] = (!(dr > 0.0) || !isfinite(dr)) ? 1 : 0;
    dinv[lane] = 1.0 / dr;
  }
  __syncthreads();
  for (int e = lane; e < n * n; e += 64) {
    const int i = e / n, j = e - i * n;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < N2; ++k) {
      re += V[i * N2 + k] * dinv[k] * V[j * N2 + k];
      im += V[(i + n) * N2 + k] * dinv[k] * V[j * N2 + k];
    }
    ginv[i * n + j] = make_double2(re, im);
  }
  if (lane == 0) {
    int bad = 0;
    for (int k = 0; k < N2; ++k) bad |= badk[k];
    flag[inst] = bad;
  }
}

void launch_ginv(int ni, const double* gamma, int n, double eps, double* ginv, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_ginv, dim3(ni), dim3(64), 0, s, (const double2*)gamma, n, eps, (double2*)ginv, flag);
}

// out[i]: [0] energy, [1] dipole, [2] max |S - I|, [3] kinetic momentum along
// e (sum gamma_pq <phi_p|-i S_e|phi_q>, plus N A in the velocity gauge)
__global__ void __launch_bounds__(NT) k_observe(const DevMesh* __restrict__ dm, const double2* __restrict__ gamma,
                                                const double2* __restrict__ Gamma, const double2* __restrict__ h,
                                                const double2* __restrict__ g, const double2* __restrict__ z,
                                                const double2* __restrict__ S, const double2* __restrict__ pm,
                                                const double* __restrict__ Ef, double* __restrict__ out) {
  __shared__ double lds4[4];
  const int inst = blockIdx.x;
  const DevMesh& d = dm[inst];
  const int n = d.n, nn = n * n;
  gamma += (int64_t)inst * nn;
  Gamma += (int64_t)inst * nn * nn;
  h += (int64_t)inst * nn;
  g += (int64_t)inst * nn * nn;
  z += (int64_t)inst * nn;
  S += (int64_t)inst * nn;
  pm += (int64_t)inst * nn;
  out += 8 * inst;
  // Re sum h gamma, Re sum gamma z, Re sum gamma p, tr gamma and Re sum g Gamma over the block
  double e1 = 0.0, e2 = 0.0, dip = 0.0, mom = 0.0, tr = 0.0;
  for (int i = threadIdx.x; i < nn; i += NT) {
    e1 += h[i].x * gamma[i].x - h[i].y * gamma[i].y;
    dip += gamma[i].x * z[i].x - gamma[i].y * z[i].y;
    mom += gamma[i].x * pm[i].x - gamma[i].y * pm[i].y;
    if (i % (n + 1) == 0) tr += gamma[i].x;
  }
  for (int i = threadIdx.x; i < nn * nn; i += NT) e2 += g[i].x * Gamma[i].x - g[i].y * Gamma[i].y;
  e1 = block_sum_all(e1, lds4);
  e2 = block_sum_all(e2, lds4);
  dip = block_sum_all(dip, lds4);
  mom = block_sum_all(mom, lds4);
  tr = block_sum_all(tr, lds4);
  if (threadIdx.x != 0) return;
  double orth = 0.0;
  for (int i = 0; i < nn; ++i) {
    const int p = i / n, q = i % n;
    const double dx = S[i].x - (p == q ? 1.0 : 0.0);
    orth = fmax(orth, hypot(dx, S[i].y));
  }
  out[0] = e1 + 0.5 * e2 + d.vnn;
  out[1] = dip;
  out[2] = orth;
  out[3] = mom + (d.gauge == 1 ? tr * Ef[0] * d.E0 : 0.0);
}

void launch_observe(const Batch& b, const double* gamma, const double* Gamma, const double* h, const double* g,
                    const double* zmat, const double* S, const double* pmat, const double* Ef, double* out,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_observe, dim3(b.ni), dim3(NT), 0, s, b.dm, (const double2*)gamma, (const double2*)Gamma,
                     (const double2*)h, (const double2*)g, (const double2*)zmat, (const double2*)S,
                     (const double2*)pmat, Ef, out);
}

// Gram-Schmidt in M as x <- x R^-1 with S = R^H R (Cholesky), R upper.
__global__ void k_chol_inv(const double2* __restrict__ S, int n, double2* __restrict__ Rinv) {
  if (threadIdx.x != 0) return;
  S += (int64_t)blockIdx.x * n * n;
  Rinv += (int64_t)blockIdx.x * n * n;
  double2 R[64], Ri[64];
  for (int i = 0; i < n * n; ++i) { R[i] = make_double2(0, 0); Ri[i] = make_double2(0, 0); }
  for (int j = 0; j < n; ++j) {
    // R_jj = sqrt(S_jj - sum_k |R_kj|^2); R_ji = (S_ji - sum_k conj(R_kj) R_ki) / R_jj
    double dd = S[j * n + j].x;
    for (int k = 0; k < j; ++k) dd -= R[k * n + j].x * R[k * n + j].x + R[k * n + j].y * R[k * n + j].y;
    double rjj = sqrt(fmax(dd, 1e-300));
    R[j * n + j] = make_double2(rjj, 0.0);
    for (int i = j + 1; i < n; ++i) {
      double2 s = S[j * n + i];
      for (int k = 0; k < j; ++k) s = csub(s, cjmul(R[k * n + j], R[k * n + i]));
      R[j * n + i] = cscale(1.0 / rjj, s);
    }
  }
  // invert upper triangular R
  for (int i = n - 1; i >= 0; --i) {
    Ri[i * n + i] = make_double2(1.0 / R[i * n + i].x, 0.0);
    for (int j = i + 1; j < n; ++j) {
      double2 s = make_double2(0, 0);
      for (int k = i + 1; k <= j; ++k) s = cadd(s, cmul(R[i * n + k], Ri[k * n + j]));
      Ri[i * n + j] = cscale(-1.0 / R[i * n + i].x, s);
    }
  }
  for (int i = 0; i < n * n; ++i) Rinv[i] = Ri[i];
}

__global__ void k_right_mul(const DevMesh* __restrict__ dm, double2* __restrict__ x, const double2* __restrict__ Ri) {
  INSTANCE;
  const int n = d.n;
  x += d.oE * n;
  Ri += (int64_t)blockIdx.y * n * n;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < d.NE; i += (int64_t)gridDim.x * NT) {
    double2 row[8], out[8];
    for (int p = 0; p < n; ++p) row[p] = x[i * n + p];
    for (int q = 0; q < n; ++q) {
      double2 s = make_double2(0, 0);
      for (int p = 0; p <= q; ++p) s = cadd(s, cmul(row[p], Ri[p * n + q]));
      out[q] = s;
    }
    for (int q = 0; q < n; ++q) x[i * n + q] = out[q];
  }
}

void launch_orthonormalize_full(const Batch& b, const double* S, double* Rinv, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv, dim3(b.ni), dim3(64), 0, s, (const double2*)S, b.mx.n, (double2*)Rinv);
  hipLaunchKernelGGL(k_right_mul, dim3(nblocks(b.mx.NE, NT, 4096), b.ni), dim3(NT), 0, s, b.dm, (double2*)x,
                     (const double2*)Rinv);
}

// =====================================================================
// CI: excitation-table sigma vector, RDMs, Lanczos in one workgroup per
// instance.  Tables: ex[J][p*n+q] = I | (sign<0) << 30 with E_pq |I> =
// sign |J>, or -1.  Vectors of instance i at offset i * dim.
// =====================================================================
__global__ void k_ci_D(CIDev c, const double2* __restrict__ C, double2* __restrict__ D) {
  const int nn = c.n * c.n;
  const int64_t total = (int64_t)c.dim * nn;
  C += (int64_t)blockIdx.y * c.dim;
  D += (int64_t)blockIdx.y * total;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    int J = (int)(e / nn), pq = (int)(e - (int64_t)J * nn);
    int Ja = J / c.NB, Jb = J - Ja * c.NB;
    double2 s = make_double2(0.0, 0.0);
    int ta = c.exa[Ja * nn + pq];
    if (ta >= 0) {
      double sg = (ta >> 30) ? -1.0 : 1.0;
      s = cadd(s, cscale(sg, C[(ta & 0x3fffffff) * c.NB + Jb]));
    }
    int tb = c.exb[Jb * nn + pq];
    if (tb >= 0) {
      double sg = (tb >> 30) ? -1.0 : 1.0;
      s = cadd(s, cscale(sg, C[Ja * c.NB + (tb & 0x3fffffff)]));
    }
    D[e] = s;  // D[J][pq] = (E_pq C)(J)
  }
}

static void launch_ci_D(int ni, const CIDev& c, const double* C, hipStream_t s) {
  hipLaunchKernelGGL(k_ci_D, dim3(nblocks((int64_t)c.dim * c.n * c.n), ni), dim3(NT), 0, s, c, (const double2*)C,
                     (double2*)c.D);
}

// Gamma[p][q][r][s] = sum_J conj(D[J][qp]) D[J][rs] - delta_qr gamma_ps, from G = D^H D
__global__ void k_ci_gamma2(const double2* __restrict__ G, const double2* __restrict__ gamma, int n,
                            double2* __restrict__ Gamma) {
  const int nn = n * n;
  G += (int64_t)blockIdx.y * nn * nn;
  gamma += (int64_t)blockIdx.y * nn;
  Gamma += (int64_t)blockIdx.y * nn * nn;
  for (int o = blockIdx.x * NT + threadIdx.x; o < nn * nn; o += gridDim.x * NT) {
    int s = o % n, r = (o / n) % n, q = (o / nn) % n, p = o / (nn * n);
    double2 v = G[(q * n + p) * nn + (r * n + s)];
    if (q == r) v = csub(v, gamma[p * n + s]);
    Gamma[o] = v;
  }
}

void launch_ci_rdm_full(int ni, const CIDev& c, const double* C, double* gamma, double* Gamma, double* Gtmp,
                        hipStream_t s) {
  const int nn = c.n * c.n;
  launch_ci_D(ni, c, C, s);
  int nb = gram_blocks(c.dim);
  launch_xgram_flat(ni, C, 1, c.D, nn, c.dim, c.part, nb, gamma, s);   // gamma[pq] = C^H D_pq
  launch_xgram_flat(ni, c.D, nn, c.D, nn, c.dim, c.part, nb, Gtmp, s);
  hipLaunchKernelGGL(k_ci_gamma2, dim3(nblocks(nn * nn), ni), dim3(NT), 0, s, (const double2*)Gtmp,
                     (const double2*)gamma, c.n, (double2*)Gamma);
}

// h'_pq = h_pq - 1/2 sum_q' g_pq'q'q
__global__ void k_ci_hprime(const double2* __restrict__ h, const double2* __restrict__ g, int n,
                            double2* __restrict__ hp) {
  const int nn = n * n;
  h += (int64_t)blockIdx.x * nn;
  g += (int64_t)blockIdx.x * nn * nn;
  hp += (int64_t)blockIdx.x * nn;
  for (int o = threadIdx.x; o < nn; o += blockDim.x) {
    int p = o / n, q = o % n;
    double2 s = h[o];
    for (int k = 0; k < n; ++k) s = csub(s, cscale(0.5, g[((p * n + k) * n + k) * n + q]));
    hp[o] = s;
  }
}
void launch_ci_hprime(int ni, const CIDev& c, const double* h, const double* g, hipStream_t s) {
  hipLaunchKernelGGL(k_ci_hprime, dim3(ni), dim3(64), 0, s, (const double2*)h, (const double2*)g, c.n,
                     (double2*)c.hp);
}

// T[J][pq] = h'_pq C[J] + 1/2 sum_rs g_pqrs D[J][rs]
__global__ void k_ci_T(CIDev c, const double2* __restrict__ C, const double2* __restrict__ g) {
  const int nn = c.n * c.n;
  const int64_t total = (int64_t)c.dim * nn;
  const int inst = blockIdx.y;
  C += (int64_t)inst * c.dim;
  g += (int64_t)inst * nn * nn;
  const double2* D = (const double2*)c.D + inst * total;
  const double2* hp = (const double2*)c.hp + (int64_t)inst * nn;
  double2* T = (double2*)c.T + inst * total;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    int J = (int)(e / nn), pq = (int)(e - (int64_t)J * nn);
    double2 s = cmul(hp[pq], C[J]);
    const double2* Dj = D + (int64_t)J * nn;
    const double2* gr = g + (int64_t)pq * nn;
    double2 t = make_double2(0.0, 0.0);
    for (int rs = 0; rs < nn; ++rs) t = cadd(t, cmul(gr[rs], Dj[rs]));
    T[e] = cadd(s, cscale(0.5, t));
  }
}

// sigma[J] = sum_pq (E_pq T_pq)(J)
__global__ void k_ci_sigma(CIDev c, double2* __restrict__ sigma) {
  const int nn = c.n * c.n;
  const int inst = blockIdx.y;
  const double2* T = (const double2*)c.T + (int64_t)inst * c.dim * nn;
  sigma += (int64_t)inst * c.dim;
  for (int J = blockIdx.x * NT + threadIdx.x; J < c.dim; J += gridDim.x * NT) {
    int Ja = J / c.NB, Jb = J - Ja * c.NB;
    double2 s = make_double2(0.0, 0.0);
    for (int pq = 0; pq < nn; ++pq) {
      int ta = c.exa[Ja * nn + pq];
      if (ta >= 0) {
        double sg = (ta >> 30) ? -1.0 : 1.0;
        s = cadd(s, cscale(sg, T[(int64_t)((ta & 0x3fffffff) * c.NB + Jb) * nn + pq]));
      }
      int tb = c.exb[Jb * nn + pq];
      if (tb >= 0) {
        double sg = (tb >> 30) ? -1.0 : 1.0;
        s = cadd(s, cscale(sg, T[(int64_t)(Ja * c.NB + (tb & 0x3fffffff)) * nn + pq]));
      }
    }
    sigma[J] = s;
  }
}

static void launch_ci_sigma(int ni, const CIDev& c, const double* C, const double* g, double* sigma, hipStream_t s) {
  const int nn = c.n * c.n;
  launch_ci_D(ni, c, C, s);
  hipLaunchKernelGGL(k_ci_T, dim3(nblocks((int64_t)c.dim * nn), ni), dim3(NT), 0, s, c, (const double2*)C,
                     (const double2*)g);
  hipLaunchKernelGGL(k_ci_sigma, dim3(nblocks(c.dim), ni), dim3(NT), 0, s, c, (double2*)sigma);
}

// Transition RDMs <A|E_pq|B> and <A|E_pq E_rs|B> - delta_qr <A|E_ps|B> (the
// RDMs above with different bra and ket), D tables in DA and DB.
void launch_ci_trdm(int ni, const CIDev& c, const double* A, const double* Bv, double* DA, double* DB,
                    double* gamma, double* Gamma, double* Gtmp, hipStream_t s) {
  const int nn = c.n * c.n;
  CIDev ca = c, cb = c;
  ca.D = DA;
  cb.D = DB;
  launch_ci_D(ni, ca, A, s);
  launch_ci_D(ni, cb, Bv, s);
  int nb = gram_blocks(c.dim);
  launch_xgram_flat(ni, A, 1, DB, nn, c.dim, c.part, nb, gamma, s);
  launch_xgram_flat(ni, DA, nn, DB, nn, c.dim, c.part, nb, Gtmp, s);
  hipLaunchKernelGGL(k_ci_gamma2, dim3(nblocks(nn * nn), ni), dim3(NT), 0, s, (const double2*)Gtmp,
                     (const double2*)gamma, c.n, (double2*)Gamma);
}

// sigma = (sum h_pq E_pq + 1/2 sum g_pqrs (E_pq E_rs - delta_qr E_ps)) C for
// general h and g; overwrites the shared h' of the CI space.
void launch_ci_apply(int ni, const CIDev& c, const double* h, const double* g, const double* C, double* sigma,
                     hipStream_t s) {
  launch_ci_hprime(ni, c, h, g, s);
  launch_ci_sigma(ni, c, C, g, sigma, s);
}

// One Lanczos/Arnoldi step on the CI space inside one workgroup: w is
// orthogonalised twice against Q_0..Q_k (full re-orthogonalisation),
// H column k filled, h_{k+1,k} = |w| (breakdown: scale 0, m_eff = k+1),
// Q_{k+1} = w / h.
__global__ void __launch_bounds__(1024) k_ci_lanczos_step(int dim, double2* const* __restrict__ Q, int k,
                                                          double2* __restrict__ w, double2* __restrict__ H, int m_max,
                                                          double* __restrict__ scal, int last) {
  __shared__ double red[32];
  __shared__ double2 hs[KMAX];
  const int inst = blockIdx.x;
  const int64_t vo = (int64_t)inst * dim;
  w += vo;
  H += (int64_t)inst * (m_max + 1) * m_max;
  scal += 8 * inst;
  auto bsum = [&](double v) -> double {
    v = wave_sum(v);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    __syncthreads();
    return t;
  };
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j <= k; ++j) {
      double re = 0.0, im = 0.0;
      for (int i = threadIdx.x; i < dim; i += blockDim.x) {
        double2 q = Q[j][vo + i], x = w[i];
        re += q.x * x.x + q.y * x.y;
        im += q.x * x.y - q.y * x.x;
      }
      re = bsum(re);
      im = bsum(im);
      if (threadIdx.x == 0) {
        hs[j] = make_double2(re, im);
        double2* hp = &H[j + (int64_t)(m_max + 1) * k];
        if (pass == 0) *hp = hs[j];
        else *hp = cadd(*hp, hs[j]);
      }
      __syncthreads();
    }
    for (int i = threadIdx.x; i < dim; i += blockDim.x) {
      double2 x = w[i];
      for (int j = 0; j <= k; ++j) x = csub(x, cmul(hs[j], Q[j][vo + i]));
      w[i] = x;
    }
    __syncthreads();
  }
  double nrm = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) nrm += w[i].x * w[i].x + w[i].y * w[i].y;
  nrm = sqrt(bsum(nrm));
  if (last) return;
  double hkk = 0.0;
  {
    double2 dd = H[k + (int64_t)(m_max + 1) * k];
    hkk = hypot(dd.x, dd.y);
  }
  bool brk = !(nrm > 1e-14 * fmax(1.0, hkk));
  double sc = brk ? 0.0 : 1.0 / nrm;
  if (threadIdx.x == 0) {
    H[(k + 1) + (int64_t)(m_max + 1) * k] = make_double2(brk ? 0.0 : nrm, 0.0);
    if (brk && scal[4] > k + 1) scal[4] = k + 1;
  }
  for (int i = threadIdx.x; i < dim; i += blockDim.x) Q[k + 1][vo + i] = cscale(sc, w[i]);
}

__global__ void __launch_bounds__(1024) k_ci_start(int dim, const double2* __restrict__ C, double2* __restrict__ Q0,
                                                   double* __restrict__ scal, int m, double2* __restrict__ H,
                                                   int m_max) {
  __shared__ double red[32];
  const int inst = blockIdx.x;
  C += (int64_t)inst * dim;
  Q0 += (int64_t)inst * dim;
  H += (int64_t)inst * (m_max + 1) * m_max;
  scal += 8 * inst;
  double s = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) s += C[i].x * C[i].x + C[i].y * C[i].y;
  s = wave_sum(s);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = s;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  double beta = sqrt(t);
  const double ib = beta > 0.0 ? 1.0 / beta : 0.0;  // a zero vector stays zero
  for (int i = threadIdx.x; i < dim; i += blockDim.x) Q0[i] = cscale(ib, C[i]);
  for (int i = threadIdx.x; i < (m_max + 1) * m_max; i += blockDim.x) H[i] = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    scal[0] = beta;
    scal[4] = m;
    scal[3] = 0.0;
  }
}

__global__ void __launch_bounds__(1024) k_ci_combine(int dim, double2* const* __restrict__ Q, int m, int m_max,
                                                     const double2* __restrict__ y, double2* __restrict__ C,
                                                     int normalize) {
  __shared__ double red[32];
  const int inst = blockIdx.x;
  const int64_t vo = (int64_t)inst * dim;
  y += (int64_t)inst * m_max;
  C += vo;
  double s2 = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) {
    double2 s = make_double2(0.0, 0.0);
    for (int j = 0; j < m; ++j) s = cadd(s, cmul(y[j], Q[j][vo + i]));
    C[i] = s;
    s2 += s.x * s.x + s.y * s.y;
  }
  if (!normalize) return;
  s2 = wave_sum(s2);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = s2;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  double f = 1.0 / sqrt(t);
  for (int i = threadIdx.x; i < dim; i += blockDim.x) C[i] = cscale(f, C[i]);
}

void launch_ci_lanczos(int ni, const CIDev& c, double* const* Qdev, double* const* Qhost, int m, const double* g,
                       double* Cvec, Krylov& K, double tau_re, double tau_im, int normalize, hipStream_t s) {
  hipLaunchKernelGGL(k_ci_start, dim3(ni), dim3(1024), 0, s, c.dim, (const double2*)Cvec, (double2*)Qhost[0], K.scal,
                     m, (double2*)K.H, K.m_max);
  for (int k = 0; k < m; ++k) {
    launch_ci_sigma(ni, c, Qhost[k], g, c.w, s);
    hipLaunchKernelGGL(k_ci_lanczos_step, dim3(ni), dim3(1024), 0, s, c.dim, (double2* const*)Qdev, k, (double2*)c.w,
                       (double2*)K.H, K.m_max, K.scal, (k == m - 1) ? 1 : 0);
  }
  hipLaunchKernelGGL(k_expm, dim3(1, ni), dim3(NT), 0, s, (const double2*)K.H, K.m_max, tau_re, tau_im, K.scal,
                     (double2*)K.y, 0, 0.0);
  hipLaunchKernelGGL(k_ci_combine, dim3(ni), dim3(1024), 0, s, c.dim, (double2* const*)Qdev, m, K.m_max,
                     (const double2*)K.y, (double2*)Cvec, normalize);
}

}  // namespace mh
