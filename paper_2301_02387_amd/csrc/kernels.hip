// HIP kernels of the MCTDHF-on-octree-FEM hot path for gfx950 (wave64).
//
// Orbital arrays are complex128 [rows][n] (orbital fastest); Poisson arrays
// are real [rows][ncol].  Row space: [0,N) DoFs, [N,NE) hanging nodes,
// [NE,NF) box-boundary nodes.
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


// =====================================================================
// Orbital cell operator: acc += (K/2 + v + E mz + m gamma^-1 U) u
// Sum-factorised per cell (Sec. III.A tensor-product basis): the element
// stiffness (h/2)(A x W x W + W x A x W + W x W x A) is applied line by
// line from LDS; node-diagonal terms are added once per node by its owner
// cell; results are scattered with FP64 atomics (boundary rows skipped).
// =====================================================================
template <int P>
__global__ void __launch_bounds__(NT) k_cell_orb(DevMesh d, const double2* __restrict__ u, double* __restrict__ acc,
                                                 double E, int diag_mode, const double* __restrict__ Upk,
                                                 const double2* __restrict__ ginv) {
  constexpr int P3 = P * P * P;
  constexpr int CPB = (NT / P3) > 0 ? NT / P3 : 1;
  __shared__ double2 su[CPB * 8 * P3];
  const int n = d.n;
  const int tid = threadIdx.x;
  const int ci = tid / P3, t = tid - ci * P3;
  const int64_t e = (int64_t)blockIdx.x * CPB + ci;
  const bool active = (ci < CPB) && (e < d.nC);
  const int node = active ? d.cell_nodes[e * P3 + t] : (int)d.NE;
  double2* my = su + ci * 8 * P3;
  if (ci < CPB) {
    for (int o = 0; o < n; ++o)
      my[o * P3 + t] = (active && node < d.NE) ? u[(int64_t)node * n + o] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (!active || node >= d.NE) return;
  const int a = t % P, b = (t / P) % P, c = t / (P * P);
  const double hh = d.cell_hh[e];
  const double wa = d.w[a], wb = d.w[b], wc = d.w[c];
  const double f0 = 0.5 * hh * wb * wc, f1 = 0.5 * hh * wa * wc, f2 = 0.5 * hh * wa * wb;
  double2 y[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) y[o] = make_double2(0.0, 0.0);
  for (int o = 0; o < n; ++o) {
    const double2* uo = my + o * P3;
    double2 s0 = make_double2(0, 0), s1 = make_double2(0, 0), s2 = make_double2(0, 0);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      double2 v0 = uo[(c * P + b) * P + q], v1 = uo[(c * P + q) * P + a], v2 = uo[(q * P + b) * P + a];
      double A0 = d.A[a * P + q], A1 = d.A[b * P + q], A2 = d.A[c * P + q];
      s0.x += A0 * v0.x; s0.y += A0 * v0.y;
      s1.x += A1 * v1.x; s1.y += A1 * v1.y;
      s2.x += A2 * v2.x; s2.y += A2 * v2.y;
    }
    y[o] = make_double2(f0 * s0.x + f1 * s1.x + f2 * s2.x, f0 * s0.y + f1 * s1.y + f2 * s2.y);
  }
  if (diag_mode >= 1 && ((d.owner[e] >> t) & 1ull)) {
    const double dg = d.v[node] + E * d.mz[node];
    for (int o = 0; o < n; ++o) {
      double2 uo = my[o * P3 + t];
      y[o].x += dg * uo.x;
      y[o].y += dg * uo.y;
    }
    if (diag_mode == 2) {
      // z = U u with U Hermitian packed: U_oo = Up[o][o], U_oq = Up[o][q] + i Up[q][o] (o < q)
      const double* Up = Upk + (int64_t)node * n * n;
      double2 z[8];
      for (int o = 0; o < n; ++o) {
        double2 s = make_double2(0.0, 0.0);
        for (int q = 0; q < n; ++q) {
          double2 Uoq;
          if (o == q) Uoq = make_double2(Up[o * n + o], 0.0);
          else if (o < q) Uoq = make_double2(Up[o * n + q], Up[q * n + o]);
          else Uoq = make_double2(Up[q * n + o], -Up[o * n + q]);
          s = cadd(s, cmul(Uoq, my[q * P3 + t]));
        }
        z[o] = s;
      }
      const double mi = d.m[node];
      for (int p = 0; p < n; ++p) {
        double2 s = make_double2(0.0, 0.0);
        for (int o = 0; o < n; ++o) s = cadd(s, cmul(ginv[p * n + o], z[o]));
        y[p].x += mi * s.x;
        y[p].y += mi * s.y;
      }
    }
  }
  double* dst = acc + (int64_t)node * n * 2;
  for (int o = 0; o < n; ++o) {
    atomicAdd(dst + 2 * o, y[o].x);
    atomicAdd(dst + 2 * o + 1, y[o].y);
  }
}

void launch_cell_orb(const DevMesh& d, const double* u, double* acc, double E, int diag_mode, const double* Upk,
                     const double* ginv, hipStream_t s) {
  switch (d.P) {
    case 2: {
      constexpr int CPB = NT / 8;
      hipLaunchKernelGGL(k_cell_orb<2>, dim3(nblocks(d.nC, CPB)), dim3(NT), 0, s, d, (const double2*)u, acc, E,
                         diag_mode, Upk, (const double2*)ginv);
      break;
    }
    case 3: {
      constexpr int CPB = NT / 27;
      hipLaunchKernelGGL(k_cell_orb<3>, dim3(nblocks(d.nC, CPB)), dim3(NT), 0, s, d, (const double2*)u, acc, E,
                         diag_mode, Upk, (const double2*)ginv);
      break;
    }
    default: {
      constexpr int CPB = NT / 64;
      hipLaunchKernelGGL(k_cell_orb<4>, dim3(nblocks(d.nC, CPB)), dim3(NT), 0, s, d, (const double2*)u, acc, E,
                         diag_mode, Upk, (const double2*)ginv);
    }
  }
}

// DoF epilogue: C^T (transposed constraints), then mass solve / projector.
__global__ void __launch_bounds__(NT) k_epi_orb(DevMesh d, double2* __restrict__ acc, int mode,
                                                const double2* __restrict__ v, const double2* __restrict__ lam,
                                                double2* __restrict__ out, double2* __restrict__ ma_b) {
  const int n = d.n;
  const int64_t total = d.N * n;
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t k = idx / n;
    const int p = (int)(idx - k * n);
    double2 f = acc[idx];
    acc[idx] = make_double2(0.0, 0.0);
    const int mi = d.ma_index[k];
    if (mi >= 0)
      for (int t = d.ct_ptr[mi]; t < d.ct_ptr[mi + 1]; ++t) {
        double2 a = acc[(int64_t)d.ct_row[t] * n + p];
        f.x += d.ct_w[t] * a.x;
        f.y += d.ct_w[t] * a.y;
      }
    if (mode == 0) {
      out[idx] = f;
      continue;
    }
    if (mi >= 0) {
      ma_b[(int64_t)mi * n + p] = f;
      continue;
    }
    double2 x = cscale(d.inv_mass[k], f);
    if (mode == 2)
      for (int q = 0; q < n; ++q) x = csub(x, cmul(lam[q * n + p], v[k * n + q]));
    out[idx] = x;
  }
}

void launch_epi_orb(const DevMesh& d, double* acc, int mode, const double* v, const double* lam, double* out,
                    double* ma_b, hipStream_t s) {
  hipLaunchKernelGGL(k_epi_orb, dim3(nblocks(d.N * d.n, NT, 8192)), dim3(NT), 0, s, d, (double2*)acc, mode,
                     (const double2*)v, (const double2*)lam, (double2*)out, (double2*)ma_b);
}

// Chebyshev iteration on the interface block A_Ma (Jacobi-preconditioned,
// spectrum bounds from set-up): x_{k+1} = x_k + d_k, r_{k+1} = r_k - A d_k,
// d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1}/delta) D^-1 r_{k+1}.
__global__ void __launch_bounds__(NT) k_cheb_init(DevMesh d, const double2* __restrict__ b, double2* __restrict__ x,
                                                  double2* __restrict__ r, double2* __restrict__ d0, double inv_theta) {
  const int n = d.n;
  const int64_t total = d.nMa * n;
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t i = idx / n;
    double2 bi = b[idx];
    x[idx] = make_double2(0.0, 0.0);
    r[idx] = bi;
    d0[idx] = cscale(d.ma_dinv[i] * inv_theta, bi);
  }
}

__global__ void __launch_bounds__(NT) k_cheb_iter(DevMesh d, double2* __restrict__ x, double2* __restrict__ r,
                                                  const double2* __restrict__ din, double2* __restrict__ dout,
                                                  double c1, double c2) {
  const int n = d.n;
  const int64_t total = d.nMa * n;
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t i = idx / n;
    const int p = (int)(idx - i * n);
    double2 s = make_double2(0.0, 0.0);
    for (int t = d.ma_ptr[i]; t < d.ma_ptr[i + 1]; ++t) {
      double2 v = din[(int64_t)d.ma_col[t] * n + p];
      s.x += d.ma_val[t] * v.x;
      s.y += d.ma_val[t] * v.y;
    }
    double2 dk = din[idx];
    x[idx] = cadd(x[idx], dk);
    double2 rn = csub(r[idx], s);
    r[idx] = rn;
    double g = c2 * d.ma_dinv[i];
    dout[idx] = make_double2(c1 * dk.x + g * rn.x, c1 * dk.y + g * rn.y);
  }
}

__global__ void __launch_bounds__(NT) k_cheb_finish(DevMesh d, const double2* __restrict__ x,
                                                    const double2* __restrict__ dk, const double2* __restrict__ v,
                                                    const double2* __restrict__ lam, double2* __restrict__ out) {
  const int n = d.n;
  const int64_t total = d.nMa * n;
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t i = idx / n;
    const int p = (int)(idx - i * n);
    const int64_t k = d.ma_dof[i];
    double2 xf = cadd(x[idx], dk[idx]);
    if (lam)
      for (int q = 0; q < n; ++q) xf = csub(xf, cmul(lam[q * n + p], v[k * n + q]));
    out[k * n + p] = xf;
  }
}

void launch_ma_solve(const DevMesh& d, const double* ma_b, double* x, double* r, double* dbuf0, double* dbuf1,
                     double lo, double hi, int iters, const double* v, const double* lam, double* out,
                     hipStream_t s) {
  if (d.nMa == 0) return;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  const int nb = nblocks(d.nMa * d.n);
  hipLaunchKernelGGL(k_cheb_init, dim3(nb), dim3(NT), 0, s, d, (const double2*)ma_b, (double2*)x, (double2*)r,
                     (double2*)dbuf0, 1.0 / theta);
  double rho = 1.0 / sigma;
  double* din = dbuf0;
  double* dout = dbuf1;
  for (int k = 0; k < iters; ++k) {
    double rho1 = 1.0 / (2.0 * sigma - rho);
    hipLaunchKernelGGL(k_cheb_iter, dim3(nb), dim3(NT), 0, s, d, (double2*)x, (double2*)r, (const double2*)din,
                       (double2*)dout, rho1 * rho, 2.0 * rho1 / delta);
    rho = rho1;
    double* t = din;
    din = dout;
    dout = t;
  }
  hipLaunchKernelGGL(k_cheb_finish, dim3(nb), dim3(NT), 0, s, d, (const double2*)x, (const double2*)din,
                     (const double2*)v, (const double2*)lam, (double2*)out);
}

// Hanging rows: x[h] = sum_k c_hk x[k] over DoF masters (boundary values of
// orbitals vanish); optionally zero the hanging rows of acc.
__global__ void __launch_bounds__(NT) k_fill_orb(DevMesh d, double2* __restrict__ x, double2* __restrict__ acc) {
  const int n = d.n;
  const int64_t total = d.Nh * n;
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t h = idx / n;
    const int p = (int)(idx - h * n);
    double2 s = make_double2(0.0, 0.0);
    for (int t = d.hang_ptr[h]; t < d.hang_ptr[h + 1]; ++t) {
      int col = d.hang_col[t];
      if (col < d.N) {
        double2 v = x[(int64_t)col * n + p];
        s.x += d.hang_w[t] * v.x;
        s.y += d.hang_w[t] * v.y;
      }
    }
    x[(d.N + h) * n + p] = s;
    if (acc) acc[(d.N + h) * n + p] = make_double2(0.0, 0.0);
  }
}

void launch_fill_orb(const DevMesh& d, double* x, double* acc, hipStream_t s) {
  if (d.Nh == 0) return;
  hipLaunchKernelGGL(k_fill_orb, dim3(nblocks(d.Nh * d.n)), dim3(NT), 0, s, d, (double2*)x, (double2*)acc);
}

__global__ void k_copy(const double* __restrict__ in, double* __restrict__ out, int64_t nd) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nd; i += (int64_t)gridDim.x * NT) out[i] = in[i];
}
__global__ void k_zero(double* __restrict__ out, int64_t nd) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nd; i += (int64_t)gridDim.x * NT) out[i] = 0.0;
}
void launch_copy(const double* in, double* out, int64_t nd, hipStream_t s) {
  if (nd > 0) hipLaunchKernelGGL(k_copy, dim3(nblocks(nd, NT, 8192)), dim3(NT), 0, s, in, out, nd);
}
void launch_zero(double* out, int64_t nd, hipStream_t s) {
  if (nd > 0) hipLaunchKernelGGL(k_zero, dim3(nblocks(nd, NT, 8192)), dim3(NT), 0, s, out, nd);
}

// =====================================================================
// Generic tiled reduction: out[a][b] = sum_i wt_i conj(X[i][a]) Y[i][b]
// X complex [rows][na]; Y complex or real [rows][nb].  Partials per block,
// then one finishing block.  Deterministic.
// =====================================================================
constexpr int XG_CH = 16;
__global__ void __launch_bounds__(NT) k_xgram(const double2* __restrict__ X, int na, const double* __restrict__ Y,
                                              int nb, int yreal, const double* __restrict__ wt, int64_t rows,
                                              double2* __restrict__ part) {
  __shared__ double2 sx[XG_CH * 64];
  __shared__ double2 sy[XG_CH * 64];
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
        if (wt) v = cscale(wt[base + r], v);
      }
      sx[r * na + a] = v;
    }
    for (int e = threadIdx.x; e < XG_CH * nb; e += NT) {
      int r = e / nb, bb = e - r * nb;
      double2 v = make_double2(0.0, 0.0);
      if (r < cnt) v = yreal ? make_double2(Y[(base + r) * nb + bb], 0.0) : ((const double2*)Y)[(base + r) * nb + bb];
      sy[r * nb + bb] = v;
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
#pragma unroll
  for (int j = 0; j < MAXO; ++j) {
    int o = threadIdx.x + j * NT;
    if (o < nout) part[(int64_t)blockIdx.x * nout + o] = accv[j];
  }
}

__global__ void k_sum_parts(const double2* __restrict__ part, int nblk, int nout, double2* __restrict__ out) {
  for (int o = blockIdx.x * NT + threadIdx.x; o < nout; o += gridDim.x * NT) {
    double2 s = make_double2(0.0, 0.0);
    for (int b = 0; b < nblk; ++b) s = cadd(s, part[(int64_t)b * nout + o]);
    out[o] = s;
  }
}

int gram_blocks(int64_t rows) { return nblocks(rows, XG_CH, 512); }

void launch_xgram(const double* X, int na, const double* Y, int nb, int yreal, const double* wt, int64_t rows,
                  double* part, int nblk, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_xgram, dim3(nblk), dim3(NT), 0, s, (const double2*)X, na, Y, nb, yreal, wt, rows,
                     (double2*)part);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblocks(na * nb)), dim3(NT), 0, s, (const double2*)part, nblk, na * nb,
                     (double2*)out);
}

void launch_gram(const double* a, const double* b, const double* wt, int64_t rows, int n, double* part, int nblk,
                 double* G, hipStream_t s) {
  launch_xgram(a, n, b, n, 0, wt, rows, part, nblk, G, s);
}

// Pair-product integrals: G[(p,q)][col] = sum_i m_i conj(phi_p) phi_q Wcol_i
// (X built on the fly as phi_p conj(phi_q) so that conj(X) = conj(phi_p) phi_q).
__global__ void __launch_bounds__(NT) k_gint(DevMesh d, const double2* __restrict__ phi,
                                             const double* __restrict__ W, int ncol, double2* __restrict__ part) {
  __shared__ double2 sx[XG_CH * 64];
  __shared__ double sw[XG_CH * 64];
  const int n = d.n, na = n * n, nout = na * ncol;
  constexpr int MAXO = 16;
  double2 accv[MAXO];
#pragma unroll
  for (int j = 0; j < MAXO; ++j) accv[j] = make_double2(0.0, 0.0);
  const int64_t rows = d.NE;
  for (int64_t base = (int64_t)blockIdx.x * XG_CH; base < rows; base += (int64_t)gridDim.x * XG_CH) {
    const int cnt = (int)((rows - base) < XG_CH ? (rows - base) : XG_CH);
    __syncthreads();
    for (int e = threadIdx.x; e < XG_CH * na; e += NT) {
      int r = e / na, a = e - r * na;
      int p = a / n, q = a - p * n;
      double2 v = make_double2(0.0, 0.0);
      if (r < cnt) {
        int64_t i = base + r;
        double2 fp = phi[i * n + p], fq = phi[i * n + q];
        // phi_p conj(phi_q) * m_i
        v = cscale(d.m[i], make_double2(fp.x * fq.x + fp.y * fq.y, fp.y * fq.x - fp.x * fq.y));
      }
      sx[r * na + a] = v;
    }
    for (int e = threadIdx.x; e < XG_CH * ncol; e += NT) {
      int r = e / ncol, c = e - r * ncol;
      sw[r * ncol + c] = (r < cnt) ? W[(base + r) * ncol + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MAXO; ++j) {
      int o = threadIdx.x + j * NT;
      if (o >= nout) break;
      int a = o / ncol, c = o - a * ncol;
      double2 s = accv[j];
      for (int r = 0; r < cnt; ++r) {
        double2 xv = sx[r * na + a];
        double yv = sw[r * ncol + c];
        s.x += xv.x * yv;
        s.y -= xv.y * yv;
      }
      accv[j] = s;
    }
  }
#pragma unroll
  for (int j = 0; j < MAXO; ++j) {
    int o = threadIdx.x + j * NT;
    if (o < nout) part[(int64_t)blockIdx.x * nout + o] = accv[j];
  }
}

// Assemble g_pqrs from the pair-column integrals G[(p,q)][col].
__global__ void k_gint_assemble(const double2* __restrict__ G, int n, const int* __restrict__ colmap,
                                double2* __restrict__ g) {
  const int ncol = n * n;
  for (int o = blockIdx.x * NT + threadIdx.x; o < n * n * n * n; o += gridDim.x * NT) {
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

int gint_blocks(const DevMesh& d) { return nblocks(d.NE, XG_CH, 512); }

void launch_gint_full(const DevMesh& d, const double* phi, const double* W, const int* colmap, double* part,
                      int nblk, double* Gtmp, double* g, hipStream_t s) {
  const int n = d.n, ncol = n * n;
  hipLaunchKernelGGL(k_gint, dim3(nblk), dim3(NT), 0, s, d, (const double2*)phi, W, ncol, (double2*)part);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblocks(ncol * ncol)), dim3(NT), 0, s, (const double2*)part, nblk,
                     ncol * ncol, (double2*)Gtmp);
  hipLaunchKernelGGL(k_gint_assemble, dim3(nblocks(ncol * ncol)), dim3(NT), 0, s, (const double2*)Gtmp, n, colmap,
                     (double2*)g);
}

// =====================================================================
// Mean field: U(x) = sum_rs Gamma_oq,rs W_rs(x), a real linear map of the
// n^2 real Poisson columns to the n^2 packed entries of the Hermitian U.
// =====================================================================
__global__ void k_build_Mreal(const double2* __restrict__ Gamma, int n, const int* __restrict__ colmap,
                              double* __restrict__ Mr) {
  const int nn = n * n;
  for (int o = blockIdx.x * NT + threadIdx.x; o < nn * nn; o += gridDim.x * NT) {
    int out = o / nn, col = o - out * nn;
    int oi = out / n, qi = out - oi * n;  // packed position
    int ro = oi < qi ? oi : qi, co = oi < qi ? qi : oi;
    bool want_im = oi > qi;               // lower triangle holds Im U_{co? }
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

__global__ void __launch_bounds__(NT) k_build_U(DevMesh d, const double* __restrict__ W, const double* __restrict__ Mr,
                                                double* __restrict__ Upk) {
  __shared__ double sM[64 * 64];
  const int nn = d.n * d.n;
  for (int e = threadIdx.x; e < nn * nn; e += NT) sM[e] = Mr[e];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < d.NE; i += (int64_t)gridDim.x * NT) {
    double wv[64];
    const double* wr = W + i * nn;
    for (int c = 0; c < nn; ++c) wv[c] = wr[c];
    double* ur = Upk + i * nn;
    for (int o = 0; o < nn; ++o) {
      double s = 0.0;
      const double* mrow = sM + o * nn;
      for (int c = 0; c < nn; ++c) s += mrow[c] * wv[c];
      ur[o] = s;
    }
  }
}

void launch_build_U_full(const DevMesh& d, const double* W, const double* Gamma, const int* colmap, double* Mr,
                         double* Upk, hipStream_t s) {
  const int nn = d.n * d.n;
  hipLaunchKernelGGL(k_build_Mreal, dim3(nblocks(nn * nn)), dim3(NT), 0, s, (const double2*)Gamma, d.n, colmap, Mr);
  hipLaunchKernelGGL(k_build_U, dim3(nblocks(d.NE, NT, 4096)), dim3(NT), 0, s, d, W, Mr, Upk);
}

// =====================================================================
// Krylov (Arnoldi) pieces.  M-inner product over the packed orbital vector:
// <u,v> = sum_i m_i sum_p conj(u_ip) v_ip on rows [0, NE).
// =====================================================================
constexpr int KMAX = 25;

__global__ void __launch_bounds__(NT) k_mdot(DevMesh d, const double2* const* __restrict__ V, int k,
                                             const double2* __restrict__ w, int with_norm, double* __restrict__ part) {
  __shared__ double lds[8];
  const int n = d.n;
  const int64_t total = d.NE * n;
  double hr[KMAX], hi[KMAX], nrm = 0.0;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) { hr[j] = 0.0; hi[j] = 0.0; }
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const double mi = d.m[e / n];
    const double2 w0 = w[e];
    const double2 we = make_double2(mi * w0.x, mi * w0.y);
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j <= k) {
        double2 vj = V[j][e];
        hr[j] += vj.x * we.x + vj.y * we.y;
        hi[j] += vj.x * we.y - vj.y * we.x;
      }
    }
    if (with_norm) nrm += we.x * w0.x + we.y * w0.y;
  }
  const int nv = 2 * (k + 1) + 1;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j <= k) {
      double a = block_sum(hr[j], lds);
      if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nv + 2 * j] = a;
      double b = block_sum(hi[j], lds);
      if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nv + 2 * j + 1] = b;
    }
  }
  double c = block_sum(nrm, lds);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nv + nv - 1] = c;
}

// Finish the dots: pass 1 sets column k of H, pass 2 adds (re-orthogonalisation).
__global__ void k_mdot_finish(const double* __restrict__ part, int nblk, int k, int m_max, int pass,
                              double2* __restrict__ H, double2* __restrict__ hcur, double* __restrict__ scal) {
  __shared__ double lds4[4];
  const int nv = 2 * (k + 1) + 1;
  for (int v = 0; v < nv; ++v) {
    const double s = sum_partials(part, nblk, nv, v, lds4);
    if (threadIdx.x != 0) continue;
    if (v == nv - 1) {
      if (pass == 1) scal[2] = s;
      continue;
    }
    int j = v >> 1;
    double* hc = (double*)&hcur[j];
    hc[v & 1] = s;
    double* hp = (double*)&H[j + (int64_t)(m_max + 1) * k];
    if (pass == 1) hp[v & 1] = s;
    else hp[v & 1] += s;
  }
}

void launch_mdot(const DevMesh& d, double* const* V, int k, const double* w, Krylov& K, int pass, hipStream_t s) {
  hipLaunchKernelGGL(k_mdot, dim3(K.nblk), dim3(NT), 0, s, d, (const double2* const*)V, k, (const double2*)w,
                     pass == 1 ? 1 : 0, K.part);
  hipLaunchKernelGGL(k_mdot_finish, dim3(1), dim3(NT), 0, s, K.part, K.nblk, k, K.m_max, pass, (double2*)K.H,
                     (double2*)K.hcur, K.scal);
}

__global__ void __launch_bounds__(NT) k_orth_update(DevMesh d, const double2* const* __restrict__ V, int k,
                                                    double2* __restrict__ w, const double2* __restrict__ hcur,
                                                    int with_norm, double* __restrict__ part) {
  __shared__ double lds[8];
  const int n = d.n;
  const int64_t total = d.NE * n;
  double2 h[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) h[j] = (j <= k) ? hcur[j] : make_double2(0.0, 0.0);
  double nrm = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    double2 we = w[e];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
      if (j <= k) we = csub(we, cmul(h[j], V[j][e]));
    w[e] = we;
    if (with_norm) nrm += d.m[e / n] * (we.x * we.x + we.y * we.y);
  }
  if (with_norm) {
    double c = block_sum(nrm, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = c;
  }
}

// h_{k+1,k} = |w|; happy breakdown when h <= 1e-14 |G v_k| (then scale 0).
__global__ void k_norm_finish(const double* __restrict__ part, int nblk, int k, int m_max,
                              double2* __restrict__ H, double* __restrict__ scal) {
  __shared__ double lds4[4];
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

void launch_orth_update(const DevMesh& d, double* const* V, int k, double* w, Krylov& K, int pass, hipStream_t s) {
  hipLaunchKernelGGL(k_orth_update, dim3(K.nblk), dim3(NT), 0, s, d, (const double2* const*)V, k, (double2*)w,
                     (const double2*)K.hcur, pass == 2 ? 1 : 0, K.part);
  if (pass == 2)
    hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(NT), 0, s, K.part, K.nblk, k, K.m_max, (double2*)K.H, K.scal);
}

__global__ void k_scale_by(const double2* __restrict__ src, double2* __restrict__ dst, int64_t total,
                           const double* __restrict__ scal, int which) {
  const double f = scal[which];
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT)
    dst[e] = cscale(f, src[e]);
}

void launch_krylov_scale(const DevMesh& d, const double* src, double* dst, Krylov& K, int which, int,
                         hipStream_t s) {
  const int64_t total = d.NE * d.n;
  hipLaunchKernelGGL(k_scale_by, dim3(nblocks(total, NT, 8192)), dim3(NT), 0, s, (const double2*)src,
                     (double2*)dst, total, K.scal, which);
}

__global__ void __launch_bounds__(NT) k_norm_part(DevMesh d, const double2* __restrict__ x,
                                                  double* __restrict__ part) {
  __shared__ double lds[8];
  const int n = d.n;
  const int64_t total = d.NE * n;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT)
    s += d.m[e / n] * (x[e].x * x[e].x + x[e].y * x[e].y);
  double c = block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = c;
}

__global__ void k_beta_finish(const double* __restrict__ part, int nblk, int m, double* __restrict__ scal,
                              double2* __restrict__ H, int m_max) {
  for (int i = threadIdx.x; i < (m_max + 1) * m_max; i += blockDim.x) H[i] = make_double2(0.0, 0.0);
  __shared__ double lds4[4];
  const double s = sum_partials(part, nblk, 1, 0, lds4);
  if (threadIdx.x != 0) return;
  double beta = sqrt(s);
  scal[0] = beta;
  scal[5] = beta > 0.0 ? 1.0 / beta : 0.0;
  scal[4] = m;
  scal[3] = 0.0;
}

void launch_norm_init(const DevMesh& d, const double* phi, Krylov& K, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_part, dim3(K.nblk), dim3(NT), 0, s, d, (const double2*)phi, K.part);
  hipLaunchKernelGGL(k_beta_finish, dim3(1), dim3(NT), 0, s, K.part, K.nblk, m, K.scal, (double2*)K.H, K.m_max);
}

// y = beta expm(A) e1, A = -i tau H_m (m = scal[4]); scaling and squaring
// with a degree-18 Taylor polynomial at |A/2^s|_1 <= 1/2 (remainder below
// 1e-22).  One workgroup; matrices in LDS.
__global__ void __launch_bounds__(NT) k_expm(const double2* __restrict__ H, int m_max, double tau_re, double tau_im,
                                             double* __restrict__ scal, double2* __restrict__ y) {
  __shared__ double2 A[KMAX * KMAX], T[KMAX * KMAX], S[KMAX * KMAX];
  __shared__ int sh_s;
  __shared__ double sh_norm;
  const int m = (int)scal[4];
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
  for (int i = threadIdx.x; i < m_max; i += NT) y[i] = (i < m) ? cscale(beta, T[i * m]) : make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    double2 hlast = H[m + (int64_t)(m_max + 1) * (m - 1)];
    double2 ylast = T[(m - 1) * m];
    scal[3] = beta * hypot(hlast.x, hlast.y) * hypot(ylast.x, ylast.y);
  }
}

void launch_expm(Krylov& K, int, double tau_re, double tau_im, hipStream_t s) {
  hipLaunchKernelGGL(k_expm, dim3(1), dim3(NT), 0, s, (const double2*)K.H, K.m_max, tau_re, tau_im, K.scal,
                     (double2*)K.y);
}

__global__ void __launch_bounds__(NT) k_combine(DevMesh d, const double2* const* __restrict__ V, int m,
                                                double2* __restrict__ phi, const double2* __restrict__ y) {
  const int64_t total = d.NE * d.n;
  double2 yy[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) yy[j] = (j < m) ? y[j] : make_double2(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
      if (j < m) s = cadd(s, cmul(yy[j], V[j][e]));
    phi[e] = s;
  }
}

void launch_combine(const DevMesh& d, double* const* V, int m, double* phi, Krylov& K, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(nblocks(d.NE * d.n, NT, 8192)), dim3(NT), 0, s, d, (const double2* const*)V, m,
                     (double2*)phi, (const double2*)K.y);
}

// =====================================================================
// Poisson: moments, boundary values, right-hand side, Jacobi PCG.
// Column c of the n^2 real columns is (r, s, part) = colinfo[c].
// =====================================================================
constexpr int MP_CH = 32;
constexpr int MP_MAXH = 169;  // (lmax+1)^2 for lmax <= 12

__device__ void solid_regular(double x, double y, double z, int lmax, double* R) {
  // R_lm = r^l P_l^m e^{i m phi} (no Condon-Shortley phase), cos then sin parts
  const double r2 = x * x + y * y + z * z;
  double pre = 1.0, pim = 0.0, dfact = 1.0;
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) {
      double t = pre * x - pim * y;
      pim = pre * y + pim * x;
      pre = t;
      dfact *= (2.0 * m - 1.0);
    }
    double a_re = dfact * pre, a_im = dfact * pim, b_re = 0.0, b_im = 0.0;  // a = R_{l-1}, b = R_{l-2}
    for (int l = m; l <= lmax; ++l) {
      double re, im;
      if (l == m) { re = a_re; im = a_im; }
      else if (l == m + 1) {
        re = (2.0 * m + 1.0) * z * a_re; im = (2.0 * m + 1.0) * z * a_im;
        b_re = a_re; b_im = a_im; a_re = re; a_im = im;
      } else {
        re = ((2.0 * l - 1.0) * z * a_re - (l + m - 1.0) * r2 * b_re) / (l - m);
        im = ((2.0 * l - 1.0) * z * a_im - (l + m - 1.0) * r2 * b_im) / (l - m);
        b_re = a_re; b_im = a_im; a_re = re; a_im = im;
      }
      R[l * l + m] = re;
      if (m > 0) R[l * l + l + m] = im;
    }
  }
}

__device__ __forceinline__ double pair_density(const double2* phi, int n, int64_t i, int r, int s, int part) {
  double2 a = phi[i * n + r], b = phi[i * n + s];
  // conj(a) b
  return part == 0 ? (a.x * b.x + a.y * b.y) : (a.x * b.y - a.y * b.x);
}

__global__ void __launch_bounds__(NT) k_moments(DevMesh d, const double2* __restrict__ phi, const double* __restrict__ xyz,
                                                double center, int lmax, int ncol, const int* __restrict__ colinfo,
                                                double* __restrict__ part) {
  __shared__ double sR[MP_CH * MP_MAXH];
  __shared__ double sW[MP_CH * 64];
  const int nh = (lmax + 1) * (lmax + 1);
  const int nout = nh * ncol;
  const int n = d.n;
  constexpr int MAXO = 48;
  double accv[MAXO];
#pragma unroll
  for (int j = 0; j < MAXO; ++j) accv[j] = 0.0;
  const int64_t rows = d.NE;
  for (int64_t base = (int64_t)blockIdx.x * MP_CH; base < rows; base += (int64_t)gridDim.x * MP_CH) {
    const int cnt = (int)((rows - base) < MP_CH ? (rows - base) : MP_CH);
    __syncthreads();
    if (threadIdx.x < MP_CH) {
      double* R = sR + threadIdx.x * nh;
      if ((int)threadIdx.x < cnt) {
        int64_t i = base + threadIdx.x;
        solid_regular(xyz[3 * i] - center, xyz[3 * i + 1] - center, xyz[3 * i + 2] - center, lmax, R);
      } else {
        for (int t = 0; t < nh; ++t) R[t] = 0.0;
      }
    }
    for (int e = threadIdx.x; e < MP_CH * ncol; e += NT) {
      int r = e / ncol, c = e - r * ncol;
      double v = 0.0;
      if (r < cnt) {
        int64_t i = base + r;
        int ci = colinfo[c];
        v = d.m[i] * pair_density(phi, n, i, ci & 255, (ci >> 8) & 255, ci >> 16);
      }
      sW[r * ncol + c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MAXO; ++j) {
      int o = threadIdx.x + j * NT;
      if (o >= nout) break;
      int t = o / ncol, c = o - t * ncol;
      double s = accv[j];
      for (int r = 0; r < cnt; ++r) s += sR[r * nh + t] * sW[r * ncol + c];
      accv[j] = s;
    }
  }
#pragma unroll
  for (int j = 0; j < MAXO; ++j) {
    int o = threadIdx.x + j * NT;
    if (o < nout) part[(int64_t)blockIdx.x * nout + o] = accv[j];
  }
}

__global__ void k_sum_parts_real(const double* __restrict__ part, int nblk, int nout, double* __restrict__ out) {
  for (int o = blockIdx.x * NT + threadIdx.x; o < nout; o += gridDim.x * NT) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * nout + o];
    out[o] = s;
  }
}

// W[NE + b][c] = sum_t table[b][t] Q[t][c]
__global__ void k_bnd_eval(DevMesh d, const double* __restrict__ table, int nh, const double* __restrict__ Q, int ncol,
                           double* __restrict__ W) {
  const int64_t total = d.Nb * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    int64_t b = e / ncol;
    int c = (int)(e - b * ncol);
    double s = 0.0;
    for (int t = 0; t < nh; ++t) s += table[b * nh + t] * Q[t * ncol + c];
    W[(d.NE + b) * ncol + c] = s;
  }
}

// Poisson cell operator on real columns: acc += K_full x.  lift = 1: only the
// listed boundary cells, with x taken as the boundary lift (boundary rows and
// the boundary-master share of hanging rows; DoF rows read as zero).
template <int P>
__global__ void __launch_bounds__(NT) k_cell_poisson(DevMesh d, const double* __restrict__ x, double* __restrict__ acc,
                                                     int ncol, int lift) {
  constexpr int P3 = P * P * P;
  __shared__ double sx[P3 * 64];
  __shared__ int snode[P3];
  const int64_t ncell = lift ? d.n_bnd_cells : d.nC;
  for (int64_t cb = blockIdx.x; cb < ncell; cb += gridDim.x) {
    const int64_t e = lift ? d.bnd_cells[cb] : cb;
    __syncthreads();
    for (int t = threadIdx.x; t < P3; t += NT) snode[t] = d.cell_nodes[e * P3 + t];
    __syncthreads();
    for (int idx = threadIdx.x; idx < P3 * ncol; idx += NT) {
      int t = idx / ncol, c = idx - t * ncol;
      int node = snode[t];
      double v = 0.0;
      if (!lift) {
        if (node < d.NE) v = x[(int64_t)node * ncol + c];
      } else if (node >= d.NE) {
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

void launch_cell_poisson(const DevMesh& d, const double* x, double* acc, int ncol, int lift, hipStream_t s) {
  int64_t ncell = lift ? d.n_bnd_cells : d.nC;
  if (ncell == 0) return;
  int nb = (int)(ncell < 65536 ? ncell : 65536);
  switch (d.P) {
    case 2: hipLaunchKernelGGL(k_cell_poisson<2>, dim3(nb), dim3(NT), 0, s, d, x, acc, ncol, lift); break;
    case 3: hipLaunchKernelGGL(k_cell_poisson<3>, dim3(nb), dim3(NT), 0, s, d, x, acc, ncol, lift); break;
    default: hipLaunchKernelGGL(k_cell_poisson<4>, dim3(nb), dim3(NT), 0, s, d, x, acc, ncol, lift);
  }
}

// Hanging rows of a real column array; with_bnd includes boundary masters.
__global__ void k_fill_real(DevMesh d, double* __restrict__ x, int ncol, int with_bnd, double* __restrict__ acc) {
  const int64_t total = d.Nh * ncol;
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

void launch_fill_real(const DevMesh& d, double* x, int ncol, int with_bnd, double* acc, hipStream_t s) {
  if (d.Nh == 0) return;
  hipLaunchKernelGGL(k_fill_real, dim3(nblocks(d.Nh * ncol)), dim3(NT), 0, s, d, x, ncol, with_bnd, acc);
}

// Column-wise partial sums over rows with thread layout (row group, column).
struct ColLayout {
  int ncol, groups;
};

// RHS: b = 4 pi C^T (m rho) - C^T acc;  r = b (cold start);  partial |b|^2.
__global__ void __launch_bounds__(NT) k_poisson_rhs(DevMesh d, const double2* __restrict__ phi, double* __restrict__ acc,
                                                    int ncol, const int* __restrict__ colinfo, double* __restrict__ rhs,
                                                    double* __restrict__ part) {
  __shared__ double lds[NT];
  const int groups = NT / ncol;
  const int g = threadIdx.x / ncol, c = threadIdx.x - g * ncol;
  const bool act = g < groups;
  double bb = 0.0;
  const int n = d.n;
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
    part[(int64_t)blockIdx.x * ncol + threadIdx.x] = t;
  }
}

// q = C^T acc (zeroing acc DoF rows); partial p.q
__global__ void __launch_bounds__(NT) k_cg_epi(DevMesh d, double* __restrict__ acc, const double* __restrict__ p,
                                               double* __restrict__ q, int ncol, double* __restrict__ part) {
  __shared__ double lds[NT];
  const int groups = NT / ncol;
  const int g = threadIdx.x / ncol, c = threadIdx.x - g * ncol;
  const bool act = g < groups;
  double pq = 0.0;
  if (act)
    for (int64_t k = (int64_t)blockIdx.x * groups + g; k < d.N; k += (int64_t)gridDim.x * groups) {
      double f = acc[k * ncol + c];
      acc[k * ncol + c] = 0.0;
      int mi = d.ma_index[k];
      if (mi >= 0)
        for (int t = d.ct_ptr[mi]; t < d.ct_ptr[mi + 1]; ++t) f += d.ct_w[t] * acc[(int64_t)d.ct_row[t] * ncol + c];
      q[k * ncol + c] = f;
      pq += f * p[k * ncol + c];
    }
  lds[threadIdx.x] = act ? pq : 0.0;
  __syncthreads();
  if (threadIdx.x < ncol) {
    double t = 0.0;
    for (int qq = 0; qq < groups; ++qq) t += lds[qq * ncol + threadIdx.x];
    part[(int64_t)blockIdx.x * ncol + threadIdx.x] = t;
  }
}

// scalar slots in sc[slot * ncol + c] (SC_* in kernels.hpp)

__global__ void k_col_finish(const double* __restrict__ part, int nblk, int ncol, double* __restrict__ sc, int slot,
                             int mode) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * ncol + c];
    if (mode == 0) {
      sc[slot * ncol + c] = s;
    } else if (mode == 1) {  // alpha = rz / pq
      sc[SC_PQ * ncol + c] = s;
      double rz = sc[SC_RZ * ncol + c];
      sc[SC_ALPHA * ncol + c] = (s != 0.0 && rz != 0.0) ? rz / s : 0.0;
    } else if (mode == 2) {  // beta = rz_new / rz (and rr from second half)
      double rz = sc[SC_RZ * ncol + c];
      sc[SC_BETA * ncol + c] = (rz != 0.0) ? s / rz : 0.0;
      sc[SC_RZ * ncol + c] = s;
    }
  }
}

// x += alpha p; r -= alpha q; z = D^-1 r; partials (r.z, r.r)
__global__ void __launch_bounds__(NT) k_cg_update(DevMesh d, double* __restrict__ x, double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ q, int ncol,
                                                  const double* __restrict__ sc, double* __restrict__ part) {
  __shared__ double lds[2 * NT];
  const int groups = NT / ncol;
  const int g = threadIdx.x / ncol, c = threadIdx.x - g * ncol;
  const bool act = g < groups;
  double rz = 0.0, rr = 0.0;
  if (act) {
    const double al = sc[SC_ALPHA * ncol + c];
    for (int64_t k = (int64_t)blockIdx.x * groups + g; k < d.N; k += (int64_t)gridDim.x * groups) {
      int64_t e = k * ncol + c;
      x[e] += al * p[e];
      double rn = r[e] - al * q[e];
      r[e] = rn;
      rz += rn * rn * d.kdiag_inv[k];
      rr += rn * rn;
    }
  }
  lds[threadIdx.x] = act ? rz : 0.0;
  lds[NT + threadIdx.x] = act ? rr : 0.0;
  __syncthreads();
  if (threadIdx.x < ncol) {
    double t = 0.0, u = 0.0;
    for (int qq = 0; qq < groups; ++qq) {
      t += lds[qq * ncol + threadIdx.x];
      u += lds[NT + qq * ncol + threadIdx.x];
    }
    part[(int64_t)blockIdx.x * 2 * ncol + threadIdx.x] = t;
    part[(int64_t)blockIdx.x * 2 * ncol + ncol + threadIdx.x] = u;
  }
}

__global__ void k_cg_finish2(const double* __restrict__ part, int nblk, int ncol, double* __restrict__ sc) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    double s = 0.0, u = 0.0;
    for (int b = 0; b < nblk; ++b) {
      s += part[(int64_t)b * 2 * ncol + c];
      u += part[(int64_t)b * 2 * ncol + ncol + c];
    }
    double rz = sc[SC_RZ * ncol + c];
    sc[SC_BETA * ncol + c] = (rz != 0.0) ? s / rz : 0.0;
    sc[SC_RZ * ncol + c] = s;
    sc[SC_RR * ncol + c] = u;
  }
}

// p = D^-1 r + beta p (DoF rows)
__global__ void k_cg_p(DevMesh d, const double* __restrict__ r, double* __restrict__ p, int ncol,
                       const double* __restrict__ sc) {
  const int64_t total = d.N * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    int64_t k = e / ncol;
    int c = (int)(e - k * ncol);
    p[e] = d.kdiag_inv[k] * r[e] + sc[SC_BETA * ncol + c] * p[e];
  }
}

static int col_blocks(const DevMesh& d, int ncol) {
  int groups = NT / ncol;
  return nblocks(d.N, groups, 1024);
}

void launch_poisson_pipeline_moments(const DevMesh& d, const double* phi, const double* xyz, const int* colinfo,
                                     PoissonWs& P, hipStream_t s) {
  const int nout = P.nharm * P.ncol;
  hipLaunchKernelGGL(k_moments, dim3(P.mblk), dim3(NT), 0, s, d, (const double2*)phi, xyz, P.center, P.lmax, P.ncol,
                     colinfo, P.mpart);
  hipLaunchKernelGGL(k_sum_parts_real, dim3(nblocks(nout)), dim3(NT), 0, s, P.mpart, P.mblk, nout, P.Q);
}

void launch_bnd_eval(const DevMesh& d, PoissonWs& P, double* W, hipStream_t s) {
  if (d.Nb == 0) return;
  hipLaunchKernelGGL(k_bnd_eval, dim3(nblocks(d.Nb * P.ncol)), dim3(NT), 0, s, d, P.table, P.nharm, P.Q, P.ncol, W);
}

void launch_poisson_rhs_full(const DevMesh& d, const double* phi, double* W, const int* colinfo, double* rhs,
                             PoissonWs& P, hipStream_t s) {
  const int ncol = P.ncol;
  launch_zero(P.acc, d.NE * ncol, s);  // the lift pass accumulates with atomics
  // boundary lift through the stiffness, then C^T and the density load
  launch_cell_poisson(d, W, P.acc, ncol, 1, s);
  int nb = col_blocks(d, ncol);
  hipLaunchKernelGGL(k_poisson_rhs, dim3(nb), dim3(NT), 0, s, d, (const double2*)phi, P.acc, ncol, colinfo, rhs,
                     P.part);
  hipLaunchKernelGGL(k_col_finish, dim3(1), dim3(64), 0, s, P.part, nb, ncol, P.sc, (int)SC_BB, 0);
  // hanging rows of acc back to zero
  launch_zero(P.acc + d.N * ncol, d.Nh * ncol, s);
}

// Operator apply q = K p (p DoF rows given; hanging rows filled here).
[[maybe_unused]] static void cg_apply_atomic(const DevMesh& d, PoissonWs& P, double* pvec, double* qvec, hipStream_t s) {
  const int ncol = P.ncol;
  launch_fill_real(d, pvec, ncol, 0, P.acc, s);
  const bool rec = P.ev && P.ev_used + 2 <= P.ev_cap;
  if (rec) (void)hipEventRecord(P.ev[P.ev_used], s);
  launch_cell_poisson(d, pvec, P.acc, ncol, 0, s);
  if (rec) {
    (void)hipEventRecord(P.ev[P.ev_used + 1], s);
    P.ev_used += 2;
  }
  int nb = col_blocks(d, ncol);
  hipLaunchKernelGGL(k_cg_epi, dim3(nb), dim3(NT), 0, s, d, P.acc, pvec, qvec, ncol, P.part);
  hipLaunchKernelGGL(k_col_finish, dim3(1), dim3(64), 0, s, P.part, nb, ncol, P.sc, (int)SC_PQ, 1);
}

__global__ void k_cg_start(DevMesh d, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ q,
                           double* __restrict__ p, int ncol, int warm) {
  const int64_t total = d.N * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    int64_t k = e / ncol;
    double rn = warm ? r[e] - q[e] : r[e];
    if (!warm) x[e] = 0.0;
    r[e] = rn;
    p[e] = d.kdiag_inv[k] * rn;
  }
}

__global__ void __launch_bounds__(NT) k_rz_part(DevMesh d, const double* __restrict__ r, int ncol,
                                                double* __restrict__ part) {
  __shared__ double lds[2 * NT];
  const int groups = NT / ncol;
  const int g = threadIdx.x / ncol, c = threadIdx.x - g * ncol;
  const bool act = g < groups;
  double rz = 0.0, rr = 0.0;
  if (act)
    for (int64_t k = (int64_t)blockIdx.x * groups + g; k < d.N; k += (int64_t)gridDim.x * groups) {
      double rn = r[k * ncol + c];
      rz += rn * rn * d.kdiag_inv[k];
      rr += rn * rn;
    }
  lds[threadIdx.x] = act ? rz : 0.0;
  lds[NT + threadIdx.x] = act ? rr : 0.0;
  __syncthreads();
  if (threadIdx.x < ncol) {
    double t = 0.0, u = 0.0;
    for (int qq = 0; qq < groups; ++qq) {
      t += lds[qq * ncol + threadIdx.x];
      u += lds[NT + qq * ncol + threadIdx.x];
    }
    part[(int64_t)blockIdx.x * 2 * ncol + threadIdx.x] = t;
    part[(int64_t)blockIdx.x * 2 * ncol + ncol + threadIdx.x] = u;
  }
}

__global__ void k_cg_start_finish(const double* __restrict__ part, int nblk, int ncol, double* __restrict__ sc) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    double s = 0.0, u = 0.0;
    for (int b = 0; b < nblk; ++b) {
      s += part[(int64_t)b * 2 * ncol + c];
      u += part[(int64_t)b * 2 * ncol + ncol + c];
    }
    sc[SC_RZ * ncol + c] = s;
    sc[SC_RR * ncol + c] = u;
  }
}

// Start: r = rhs - K x0 (warm) or rhs (cold, x0 = 0), p = z = D^-1 r.
void launch_cg_start_atomic(const DevMesh& d, double* W, double* rhs_r, PoissonWs& P, int warm, hipStream_t s) {
  const int ncol = P.ncol;
  if (warm) {
    // q = K x0 using p as staging for x0 (DoF rows)
    hipLaunchKernelGGL(k_copy, dim3(nblocks(d.N * ncol, NT, 8192)), dim3(NT), 0, s, W, P.p, d.N * ncol);
    cg_apply_atomic(d, P, P.p, P.q, s);
  }
  hipLaunchKernelGGL(k_cg_start, dim3(nblocks(d.N * ncol, NT, 8192)), dim3(NT), 0, s, d, W, rhs_r, P.q, P.p, ncol,
                     warm);
  int nb = col_blocks(d, ncol);
  hipLaunchKernelGGL(k_rz_part, dim3(nb), dim3(NT), 0, s, d, rhs_r, ncol, P.part);
  hipLaunchKernelGGL(k_cg_start_finish, dim3(1), dim3(64), 0, s, P.part, nb, ncol, P.sc);
}

void launch_cg_step_atomic(const DevMesh& d, double* W, PoissonWs& P, hipStream_t s) {
  const int ncol = P.ncol;
  cg_apply_atomic(d, P, P.p, P.q, s);
  int nb = col_blocks(d, ncol);
  hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(NT), 0, s, d, W, P.r, P.p, P.q, ncol, P.sc, P.part);
  hipLaunchKernelGGL(k_cg_finish2, dim3(1), dim3(64), 0, s, P.part, nb, ncol, P.sc);
  hipLaunchKernelGGL(k_cg_p, dim3(nblocks(d.N * ncol, NT, 8192)), dim3(NT), 0, s, d, P.r, P.p, ncol, P.sc);
}


// =====================================================================
// Small dense kernels (one workgroup / one thread).
// =====================================================================
// Regularised inverse of the Hermitian 1-RDM: eigen-decomposition of the
// real 2n x 2n embedding [[Re, -Im], [Im, Re]] by cyclic Jacobi, d -> d +
// eps exp(-d/eps), inverse from the eigenpairs.
__global__ void k_ginv(const double2* __restrict__ gamma, int n, double eps, double2* __restrict__ ginv,
                       int* __restrict__ flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int N2 = 2 * n;
  double a[16 * 16], V[16 * 16];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      // Hermitian part
      double re = 0.5 * (gamma[i * n + j].x + gamma[j * n + i].x);
      double im = 0.5 * (gamma[i * n + j].y - gamma[j * n + i].y);
      a[i * N2 + j] = re;
      a[(i + n) * N2 + (j + n)] = re;
      a[i * N2 + (j + n)] = -im;
      a[(i + n) * N2 + j] = im;
    }
  for (int i = 0; i < N2; ++i)
    for (int j = 0; j < N2; ++j) V[i * N2 + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < N2; ++i)
      for (int j = 0; j < N2; ++j) {
        tot += a[i * N2 + j] * a[i * N2 + j];
        if (i != j) off += a[i * N2 + j] * a[i * N2 + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < N2; ++p)
      for (int q = p + 1; q < N2; ++q) {
        double apq = a[p * N2 + q];
        if (fabs(apq) < 1e-300) continue;
        double theta = (a[q * N2 + q] - a[p * N2 + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < N2; ++k) {
          double akp = a[k * N2 + p], akq = a[k * N2 + q];
          a[k * N2 + p] = c * akp - s * akq;
          a[k * N2 + q] = s * akp + c * akq;
        }
        for (int k = 0; k < N2; ++k) {
          double apk = a[p * N2 + k], aqk = a[q * N2 + k];
          a[p * N2 + k] = c * apk - s * aqk;
          a[q * N2 + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < N2; ++k) {
          double vkp = V[k * N2 + p], vkq = V[k * N2 + q];
          V[k * N2 + p] = c * vkp - s * vkq;
          V[k * N2 + q] = s * vkp + c * vkq;
        }
      }
  }
  int bad = 0;
  double dinv[16];
  for (int k = 0; k < N2; ++k) {
    double dk = a[k * N2 + k];
    double dr = dk + eps * exp(-dk / eps);
    if (!(dr > 0.0) || !isfinite(dr)) bad = 1;
    dinv[k] = 1.0 / dr;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double re = 0.0, im = 0.0;
      for (int k = 0; k < N2; ++k) {
        re += V[i * N2 + k] * dinv[k] * V[j * N2 + k];
        im += V[(i + n) * N2 + k] * dinv[k] * V[j * N2 + k];
      }
      ginv[i * n + j] = make_double2(re, im);
    }
  *flag = bad;
}

void launch_ginv(const double* gamma, int n, double eps, double* ginv, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_ginv, dim3(1), dim3(64), 0, s, (const double2*)gamma, n, eps, (double2*)ginv, flag);
}

// out: [0] energy, [1] dipole, [2] max |S - I|, [3] sum |C|^2 (unused here)
__global__ void k_observe(const double2* __restrict__ gamma, const double2* __restrict__ Gamma,
                          const double2* __restrict__ h, const double2* __restrict__ g, const double2* __restrict__ z,
                          const double2* __restrict__ S, int n, double vnn, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double e1 = 0.0, e2 = 0.0, dip = 0.0, orth = 0.0;
  for (int i = 0; i < n * n; ++i) {
    e1 += h[i].x * gamma[i].x - h[i].y * gamma[i].y;
    dip += gamma[i].x * z[i].x - gamma[i].y * z[i].y;
    int p = i / n, q = i % n;
    double dx = S[i].x - (p == q ? 1.0 : 0.0);
    orth = fmax(orth, hypot(dx, S[i].y));
  }
  for (int i = 0; i < n * n * n * n; ++i) e2 += g[i].x * Gamma[i].x - g[i].y * Gamma[i].y;
  out[0] = e1 + 0.5 * e2 + vnn;
  out[1] = dip;
  out[2] = orth;
}

void launch_observe(const double* gamma, const double* Gamma, const double* h, const double* g, const double* zmat,
                    const double* S, int n, double vnn, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_observe, dim3(1), dim3(64), 0, s, (const double2*)gamma, (const double2*)Gamma,
                     (const double2*)h, (const double2*)g, (const double2*)zmat, (const double2*)S, n, vnn, out);
}

// Gram-Schmidt in M as x <- x R^-1 with S = R^H R (Cholesky), R upper.
__global__ void k_chol_inv(const double2* __restrict__ S, int n, double2* __restrict__ Rinv) {
  if (threadIdx.x != 0) return;
  double2 R[64], Ri[64];
  for (int i = 0; i < n * n; ++i) { R[i] = make_double2(0, 0); Ri[i] = make_double2(0, 0); }
  for (int j = 0; j < n; ++j) {
    // R_jj = sqrt(S_jj - sum_k |R_kj|^2); R_ji = (S_ji - sum_k conj(R_kj) R_ki) / R_jj
    double d = S[j * n + j].x;
    for (int k = 0; k < j; ++k) d -= R[k * n + j].x * R[k * n + j].x + R[k * n + j].y * R[k * n + j].y;
    double rjj = sqrt(fmax(d, 1e-300));
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

__global__ void k_right_mul(DevMesh d, double2* __restrict__ x, const double2* __restrict__ Ri) {
  const int n = d.n;
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

void launch_orthonormalize_full(const DevMesh& d, const double* S, double* Rinv, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(64), 0, s, (const double2*)S, d.n, (double2*)Rinv);
  hipLaunchKernelGGL(k_right_mul, dim3(nblocks(d.NE, NT, 4096)), dim3(NT), 0, s, d, (double2*)x,
                     (const double2*)Rinv);
}

// =====================================================================
// CI: excitation-table sigma vector, RDMs, Lanczos in one workgroup.
// Tables: ex[J][p*n+q] = I | (sign<0) << 30 with E_pq |I> = sign |J>, or -1.
// =====================================================================
__global__ void k_ci_D(CIDev c, const double2* __restrict__ C, double2* __restrict__ D) {
  const int nn = c.n * c.n;
  const int64_t total = (int64_t)c.dim * nn;
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

void launch_ci_D(const CIDev& c, const double* C, hipStream_t s) {
  hipLaunchKernelGGL(k_ci_D, dim3(nblocks((int64_t)c.dim * c.n * c.n)), dim3(NT), 0, s, c, (const double2*)C,
                     (double2*)c.D);
}

// Gamma[p][q][r][s] = sum_J conj(D[J][qp]) D[J][rs] - delta_qr gamma_ps, from G = D^H D
__global__ void k_ci_gamma2(const double2* __restrict__ G, const double2* __restrict__ gamma, int n,
                            double2* __restrict__ Gamma) {
  const int nn = n * n;
  for (int o = blockIdx.x * NT + threadIdx.x; o < nn * nn; o += gridDim.x * NT) {
    int s = o % n, r = (o / n) % n, q = (o / nn) % n, p = o / (nn * n);
    double2 v = G[(q * n + p) * nn + (r * n + s)];
    if (q == r) v = csub(v, gamma[p * n + s]);
    Gamma[o] = v;
  }
}

void launch_ci_rdm_full(const CIDev& c, const double* C, double* gamma, double* Gamma, double* Gtmp, hipStream_t s) {
  const int nn = c.n * c.n;
  launch_ci_D(c, C, s);
  int nb = gram_blocks(c.dim);
  launch_xgram(C, 1, c.D, nn, 0, nullptr, c.dim, c.part, nb, gamma, s);   // gamma[pq] = C^H D_pq
  launch_xgram(c.D, nn, c.D, nn, 0, nullptr, c.dim, c.part, nb, Gtmp, s);
  hipLaunchKernelGGL(k_ci_gamma2, dim3(nblocks(nn * nn)), dim3(NT), 0, s, (const double2*)Gtmp,
                     (const double2*)gamma, c.n, (double2*)Gamma);
}

// h'_pq = h_pq - 1/2 sum_q' g_pq'q'q
__global__ void k_ci_hprime(const double2* __restrict__ h, const double2* __restrict__ g, int n,
                            double2* __restrict__ hp) {
  for (int o = threadIdx.x; o < n * n; o += blockDim.x) {
    int p = o / n, q = o % n;
    double2 s = h[o];
    for (int k = 0; k < n; ++k) s = csub(s, cscale(0.5, g[((p * n + k) * n + k) * n + q]));
    hp[o] = s;
  }
}
void launch_ci_hprime(const CIDev& c, const double* h, const double* g, hipStream_t s) {
  hipLaunchKernelGGL(k_ci_hprime, dim3(1), dim3(64), 0, s, (const double2*)h, (const double2*)g, c.n, (double2*)c.hp);
}

// T[J][pq] = h'_pq C[J] + 1/2 sum_rs g_pqrs D[J][rs]
__global__ void k_ci_T(CIDev c, const double2* __restrict__ C, const double2* __restrict__ g) {
  const int nn = c.n * c.n;
  const int64_t total = (int64_t)c.dim * nn;
  const double2* D = (const double2*)c.D;
  const double2* hp = (const double2*)c.hp;
  double2* T = (double2*)c.T;
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
  const double2* T = (const double2*)c.T;
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

void launch_ci_sigma(const CIDev& c, const double* C, const double* g, double* sigma, hipStream_t s) {
  const int nn = c.n * c.n;
  launch_ci_D(c, C, s);
  hipLaunchKernelGGL(k_ci_T, dim3(nblocks((int64_t)c.dim * nn)), dim3(NT), 0, s, c, (const double2*)C,
                     (const double2*)g);
  hipLaunchKernelGGL(k_ci_sigma, dim3(nblocks(c.dim)), dim3(NT), 0, s, c, (double2*)sigma);
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
  double wn2 = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) wn2 += w[i].x * w[i].x + w[i].y * w[i].y;
  wn2 = bsum(wn2);
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j <= k; ++j) {
      double re = 0.0, im = 0.0;
      for (int i = threadIdx.x; i < dim; i += blockDim.x) {
        double2 q = Q[j][i], x = w[i];
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
      for (int j = 0; j <= k; ++j) x = csub(x, cmul(hs[j], Q[j][i]));
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
    double2 d = H[k + (int64_t)(m_max + 1) * k];
    hkk = hypot(d.x, d.y);
  }
  bool brk = !(nrm > 1e-14 * fmax(1.0, hkk));
  double sc = brk ? 0.0 : 1.0 / nrm;
  if (threadIdx.x == 0) {
    H[(k + 1) + (int64_t)(m_max + 1) * k] = make_double2(brk ? 0.0 : nrm, 0.0);
    if (brk && scal[4] > k + 1) scal[4] = k + 1;
  }
  for (int i = threadIdx.x; i < dim; i += blockDim.x) Q[k + 1][i] = cscale(sc, w[i]);
  (void)wn2;
}

__global__ void __launch_bounds__(1024) k_ci_start(int dim, const double2* __restrict__ C, double2* __restrict__ Q0,
                                                   double* __restrict__ scal, int m, double2* __restrict__ H,
                                                   int m_max) {
  __shared__ double red[32];
  double s = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) s += C[i].x * C[i].x + C[i].y * C[i].y;
  s = wave_sum(s);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = s;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  double beta = sqrt(t);
  for (int i = threadIdx.x; i < dim; i += blockDim.x) Q0[i] = cscale(1.0 / beta, C[i]);
  for (int i = threadIdx.x; i < (m_max + 1) * m_max; i += blockDim.x) H[i] = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    scal[0] = beta;
    scal[4] = m;
    scal[3] = 0.0;
  }
}

__global__ void __launch_bounds__(1024) k_ci_combine(int dim, double2* const* __restrict__ Q, int m,
                                                     const double2* __restrict__ y, double2* __restrict__ C,
                                                     int normalize) {
  __shared__ double red[32];
  double s2 = 0.0;
  for (int i = threadIdx.x; i < dim; i += blockDim.x) {
    double2 s = make_double2(0.0, 0.0);
    for (int j = 0; j < m; ++j) s = cadd(s, cmul(y[j], Q[j][i]));
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

void launch_ci_lanczos(const CIDev& c, double* const* Qdev, double* const* Qhost, int m, const double* g,
                       double* Cvec, Krylov& K, double tau_re, double tau_im, int normalize, hipStream_t s) {
  hipLaunchKernelGGL(k_ci_start, dim3(1), dim3(1024), 0, s, c.dim, (const double2*)Cvec, (double2*)Qhost[0], K.scal,
                     m, (double2*)K.H, K.m_max);
  for (int k = 0; k < m; ++k) {
    launch_ci_sigma(c, Qhost[k], g, c.w, s);
    hipLaunchKernelGGL(k_ci_lanczos_step, dim3(1), dim3(1024), 0, s, c.dim, (double2* const*)Qdev, k, (double2*)c.w,
                       (double2*)K.H, K.m_max, K.scal, (k == m - 1) ? 1 : 0);
  }
  hipLaunchKernelGGL(k_expm, dim3(1), dim3(NT), 0, s, (const double2*)K.H, K.m_max, tau_re, tau_im, K.scal,
                     (double2*)K.y);
  hipLaunchKernelGGL(k_ci_combine, dim3(1), dim3(1024), 0, s, c.dim, (double2* const*)Qdev, m, (const double2*)K.y,
                     (double2*)Cvec, normalize);
}


}  // namespace mh
