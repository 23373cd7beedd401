// Node-centric, atomic-free application of the one-body and Poisson
// operators (Sec. III.A tensor-product Lagrange basis on Gauss-Lobatto
// points; Eq. discretized_eom), and the Jacobi-preconditioned CG on the
// assembled Poisson operator.
//
// The element stiffness (h/2)(A x W x W + W x A x W + W x W x A) couples a
// node only to the nodes on its three coordinate lines inside each cell
// holding it (W is diagonal).  Each node therefore gathers its assembled
// value directly: for every incident cell (at most 8) it sums the three line
// contractions of the input, read straight from the cell's node map.  The
// result is written once, with no scatter and no atomics.  Node-diagonal
// terms (nuclear potential, field, mean field) are added by the same
// thread; for DoFs that are not hanging-node masters the mass solve and
// the projector term are applied in the same pass, so the output is final.
// Masters and hanging nodes hand their load values to a small gather
// kernel (the transposed constraints C^T) and the interface mass solve.
//
// Lane layout: L lanes per node (L a power of two >= the number of
// columns); lane = orbital (complex) or Poisson column (real).  Nodes are
// numbered in first-touch order over Morton-sorted cells, so the lines a
// wave reads are mostly shared with its neighbours and hit in L1/L2.
// Batched launches: instance blockIdx.y (kernels.hpp).
#include <hip/hip_runtime.h>

#include "devutil.hpp"
#include "kernels.hpp"

namespace mh {

#define INSTANCE const DevMesh& d = dm[blockIdx.y]

// --------------------------------------------------------------------------
// Orbital operator.  mode 0: F = load vector; 1: M^-1 F; 2: M^-1 F - v lam.
// Non-master DoFs get their final value in `out`; masters and hanging nodes
// store the load value in `acc`.
// --------------------------------------------------------------------------
template <int P, int L>
__global__ void __launch_bounds__(NT) k_stencil_orb(const DevMesh* __restrict__ dm, const double2* __restrict__ u,
                                                    const double* __restrict__ Ef, int diag_mode,
                                                    const double* __restrict__ Upk, const double2* __restrict__ ginv,
                                                    int mode, const double2* __restrict__ lam,
                                                    double2* __restrict__ out, double2* __restrict__ acc) {
  INSTANCE;
  constexpr int P3 = P * P * P;
  const int n = d.n;
  const int64_t o = d.oE * n;
  u += o;
  out += o;
  acc += o;
  Upk += d.oE * n * n;
  ginv += (int64_t)blockIdx.y * n * n;
  if (lam) lam += (int64_t)blockIdx.y * n * n;
  const double E = (diag_mode == 1 || diag_mode == 2) ? Ef[0] * d.E0 : 0.0;
  const XcdSweep sw = xcd_sweep(d.NE, NT / L, d.sched_orb & 1);
  // all L lanes of a node share i, so a node group enters and leaves together
  for (int64_t i = sw.start + threadIdx.x / L; i < sw.end; i += sw.step) {
    const int p = (int)(threadIdx.x & (L - 1));
    const bool act = p < n;
    double2 y = make_double2(0.0, 0.0), ui = make_double2(0.0, 0.0);
    if (act) ui = u[i * n + p];
    // the node's 8 incidence codes in two 16-byte loads (row of 32 bytes)
    const int4* inc4 = reinterpret_cast<const int4*>(d.node_inc + i * 8);
    int4 ca = inc4[0], cb = inc4[1];
    if (diag_mode == 3) ca = cb = make_int4(-1, -1, -1, -1);  // dipole weights only: no stiffness
    const int codes[8] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int code = codes[t];
      if (code < 0) continue;
      const int64_t K = code >> 6;
      const int loc = code & 63;
      const int a = loc % P, b = (loc / P) % P, c = loc / (P * P);
      const int32_t* cn = d.cell_nodes + K * P3;
      double2 s0 = make_double2(0.0, 0.0), s1 = s0, s2 = s0;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int j0 = cn[(c * P + b) * P + q], j1 = cn[(c * P + q) * P + a], j2 = cn[(q * P + b) * P + a];
        const double A0 = d.A[a * P + q], A1 = d.A[b * P + q], A2 = d.A[c * P + q];
        if (act) {
          if (j0 < d.NE) { const double2 v = u[(int64_t)j0 * n + p]; s0.x += A0 * v.x; s0.y += A0 * v.y; }
          if (j1 < d.NE) { const double2 v = u[(int64_t)j1 * n + p]; s1.x += A1 * v.x; s1.y += A1 * v.y; }
          if (j2 < d.NE) { const double2 v = u[(int64_t)j2 * n + p]; s2.x += A2 * v.x; s2.y += A2 * v.y; }
        }
      }
      const double hh = 0.5 * d.cell_hh[K];  // (1/2) K with K_cell = (h/2)(...)
      const double f0 = hh * d.w[b] * d.w[c], f1 = hh * d.w[a] * d.w[c], f2 = hh * d.w[a] * d.w[b];
      y.x += f0 * s0.x + f1 * s1.x + f2 * s2.x;
      y.y += f0 * s0.y + f1 * s1.y + f2 * s2.y;
    }
    if (diag_mode >= 1 && act) {
      const double dg = diag_mode == 3 ? d.mz[i] : d.v[i] + E * d.mz[i];
      y.x += dg * ui.x;
      y.y += dg * ui.y;
    }
    if (diag_mode == 2) {
      // z_p = sum_q U_pq u_q (U Hermitian, packed: Up[o][q] = Re U_oq, Up[q][o] = Im U_oq for o < q)
      const double* Up = Upk + i * n * n;
      double2 z = make_double2(0.0, 0.0);
      for (int q = 0; q < n; ++q) {
        const double2 uq = make_double2(__shfl(ui.x, q, L), __shfl(ui.y, q, L));
        if (act) {
          double2 Upq;
          if (p == q) Upq = make_double2(Up[p * n + p], 0.0);
          else if (p < q) Upq = make_double2(Up[p * n + q], Up[q * n + p]);
          else Upq = make_double2(Up[q * n + p], -Up[p * n + q]);
          z = cadd(z, cmul(Upq, uq));
        }
      }
      double2 wv = make_double2(0.0, 0.0);
      for (int oo = 0; oo < n; ++oo) {
        const double2 zo = make_double2(__shfl(z.x, oo, L), __shfl(z.y, oo, L));
        if (act) wv = cadd(wv, cmul(ginv[p * n + oo], zo));
      }
      if (act) {
        const double mi = d.m[i];
        y.x += mi * wv.x;
        y.y += mi * wv.y;
      }
    }
    double2 lm = make_double2(0.0, 0.0);
    if (mode == 2)
      for (int q = 0; q < n; ++q) {
        const double2 uq = make_double2(__shfl(ui.x, q, L), __shfl(ui.y, q, L));
        if (act) lm = cadd(lm, cmul(lam[q * n + p], uq));
      }
    if (!act) continue;
    const bool dof = i < d.N;
    const int mi = dof ? d.ma_index[i] : -1;
    if (dof && mi < 0) {
      if (mode == 0) out[i * n + p] = y;
      else out[i * n + p] = csub(cscale(d.inv_mass[i], y), lm);
    } else {
      acc[i * n + p] = y;
    }
  }
}

// Masters: load value = acc_k + sum_h c_hk acc_h (transposed constraints).
__global__ void __launch_bounds__(NT) k_ma_gather_orb(const DevMesh* __restrict__ dm, const double2* __restrict__ acc,
                                                      int mode, double2* __restrict__ out,
                                                      double2* __restrict__ ma_b) {
  INSTANCE;
  const int n = d.n;
  const int64_t total = d.nMa * n, o = d.oE * n, om = d.oMa * n;
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t i = idx / n;
    const int p = (int)(idx - i * n);
    const int64_t k = d.ma_dof[i];
    double2 f = acc[o + k * n + p];
    for (int t = d.ct_ptr[i]; t < d.ct_ptr[i + 1]; ++t) {
      const double2 a = acc[o + (int64_t)d.ct_row[t] * n + p];
      f.x += d.ct_w[t] * a.x;
      f.y += d.ct_w[t] * a.y;
    }
    if (mode == 0) out[o + k * n + p] = f;
    else ma_b[om + idx] = f;
  }
}

// Mass solve of a given load vector: non-masters 1/m, masters to ma_b.
__global__ void __launch_bounds__(NT) k_mass_direct(const DevMesh* __restrict__ dm, const double2* __restrict__ f,
                                                    double2* __restrict__ out, double2* __restrict__ ma_b) {
  INSTANCE;
  const int n = d.n;
  const int64_t total = d.N * n, o = d.oE * n, om = d.oMa * n;
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t k = idx / n;
    const int mi = d.ma_index[k];
    if (mi < 0) out[o + idx] = cscale(d.inv_mass[k], f[o + idx]);
    else ma_b[om + (int64_t)mi * n + (idx - k * n)] = f[o + idx];
  }
}

template <int P, int L>
static void launch_stencil_orb_t(const Batch& b, const double* u, const double* Ef, int diag_mode, const double* Upk,
                                 const double* ginv, int mode, const double* lam, double* out, double* acc,
                                 hipStream_t s) {
  const int grid = xcd_grid(b.mx.NE, NT / L, b.mx.grid_orb);
  hipLaunchKernelGGL((k_stencil_orb<P, L>), dim3(grid, b.ni), dim3(NT), 0, s, b.dm, (const double2*)u, Ef, diag_mode,
                     Upk, (const double2*)ginv, mode, (const double2*)lam, (double2*)out, (double2*)acc);
}

template <int P>
static void launch_stencil_orb_p(const Batch& b, const double* u, const double* Ef, int diag_mode, const double* Upk,
                                 const double* ginv, int mode, const double* lam, double* out, double* acc,
                                 hipStream_t s) {
  const int n = b.mx.n;
  if (n <= 1) launch_stencil_orb_t<P, 1>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, s);
  else if (n <= 2) launch_stencil_orb_t<P, 2>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, s);
  else if (n <= 4) launch_stencil_orb_t<P, 4>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, s);
  else launch_stencil_orb_t<P, 8>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, s);
}

void launch_stencil_orb(const Batch& b, const double* u, const double* Ef, int diag_mode, const double* Upk,
                        const double* ginv, int mode, const double* lam, double* out, double* acc, hipStream_t s) {
  switch (b.mx.P) {
    case 2: launch_stencil_orb_p<2>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, s); break;
    case 3: launch_stencil_orb_p<3>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, s); break;
    default: launch_stencil_orb_p<4>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, s);
  }
}

void launch_ma_gather_orb(const Batch& b, const double* acc, int mode, double* out, double* ma_b, hipStream_t s) {
  if (b.mx.nMa == 0) return;
  hipLaunchKernelGGL(k_ma_gather_orb, dim3(nblocks(b.mx.nMa * b.mx.n), b.ni), dim3(NT), 0, s, b.dm,
                     (const double2*)acc, mode, (double2*)out, (double2*)ma_b);
}

void launch_mass_direct(const Batch& b, const double* f, double* out, double* ma_b, hipStream_t s) {
  hipLaunchKernelGGL(k_mass_direct, dim3(nblocks(b.mx.N * b.mx.n, NT, 8192), b.ni), dim3(NT), 0, s, b.dm,
                     (const double2*)f, (double2*)out, (double2*)ma_b);
}

// --------------------------------------------------------------------------
// Assembled Poisson operator on the DoFs, K~ = C^T K_full C (CSR, built at
// set-up from the element line couplings): one dependent level per row
// (column index -> row of x), the hanging fill and the master gather folded
// into the matrix.  The matrix (about 12 B per entry, ~14 entries per row)
// is shared by all n^2 real columns, so it costs ~150 B per row against
// 8 n^2 B of x per row.  L lanes per row (lane = column); fused p.q
// partials.  x, q over extended rows (batch offset oE).
// --------------------------------------------------------------------------
template <int L>
__global__ void __launch_bounds__(NT) k_spmv_poisson(const DevMesh* __restrict__ dm, const double* __restrict__ x,
                                                     int ncol, double* __restrict__ q, int64_t part_stride,
                                                     double* __restrict__ part) {
  INSTANCE;
  __shared__ double lds[NT];
  x += d.oE * ncol;
  q += d.oE * ncol;
  const int c = (int)(threadIdx.x & (L - 1));
  const bool col_ok = c < ncol;
  double pq = 0.0;
  const XcdSweep sw = xcd_sweep(d.N, NT / L, d.sched_poi & 1);
  for (int64_t i = sw.start + threadIdx.x / L; i < sw.end; i += sw.step) {
    if (!col_ok) continue;
    const int beg = d.kt_ptr[i], end = d.kt_ptr[i + 1];
    double y0 = 0.0, y1 = 0.0;
    int t = beg;
    for (; t + 4 <= end; t += 4) {
      const int j0 = d.kt_col[t], j1 = d.kt_col[t + 1], j2 = d.kt_col[t + 2], j3 = d.kt_col[t + 3];
      const double x0 = x[(int64_t)j0 * ncol + c], x1 = x[(int64_t)j1 * ncol + c];
      const double x2 = x[(int64_t)j2 * ncol + c], x3 = x[(int64_t)j3 * ncol + c];
      y0 += d.kt_val[t] * x0 + d.kt_val[t + 2] * x2;
      y1 += d.kt_val[t + 1] * x1 + d.kt_val[t + 3] * x3;
    }
    for (; t < end; ++t) y0 += d.kt_val[t] * x[(int64_t)d.kt_col[t] * ncol + c];
    const double y = y0 + y1;
    q[i * ncol + c] = y;
    pq += y * x[i * ncol + c];
  }
  lds[threadIdx.x] = pq;
  __syncthreads();
  if (threadIdx.x < (unsigned)ncol) {
    double s = 0.0;
    for (int g = 0; g < NT / L; ++g) s += lds[g * L + threadIdx.x];
    part[blockIdx.y * part_stride + (int64_t)blockIdx.x * ncol + threadIdx.x] = s;
  }
}

// Same operator for an even number of columns: each lane owns V = 2 or 4
// adjacent columns (16-byte loads), so a wave keeps 64 V / ncol rows and
// their column loads in flight at once (the single-column form is bound by
// the latency of one row per wave).
template <int L, int V>
__global__ void __launch_bounds__(NT) k_spmv_poisson_v(const DevMesh* __restrict__ dm, const double* __restrict__ x,
                                                       int ncol, double* __restrict__ q, int64_t part_stride,
                                                       double* __restrict__ part) {
  INSTANCE;
  __shared__ double lds[NT * V];
  x += d.oE * ncol;
  q += d.oE * ncol;
  const int lane = (int)(threadIdx.x & (L - 1));
  const int c0 = lane * V;
  const bool col_ok = c0 < ncol;
  double pq[V];
#pragma unroll
  for (int v = 0; v < V; ++v) pq[v] = 0.0;
  const XcdSweep sw = xcd_sweep(d.N, NT / L, d.sched_poi & 1);
  for (int64_t i = sw.start + threadIdx.x / L; i < sw.end; i += sw.step) {
    if (!col_ok) continue;
    const int beg = d.kt_ptr[i], end = d.kt_ptr[i + 1];
    double y[V];
#pragma unroll
    for (int v = 0; v < V; ++v) y[v] = 0.0;
    int t = beg;
    for (; t + 4 <= end; t += 4) {
      double2 xv[4][V / 2];
      double av[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t j = d.kt_col[t + u];
        av[u] = d.kt_val[t + u];
        const double2* row = reinterpret_cast<const double2*>(x + j * ncol + c0);
#pragma unroll
        for (int v = 0; v < V / 2; ++v) xv[u][v] = row[v];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < V / 2; ++v) {
          y[2 * v] += av[u] * xv[u][v].x;
          y[2 * v + 1] += av[u] * xv[u][v].y;
        }
    }
    for (; t < end; ++t) {
      const double a = d.kt_val[t];
      const double2* row = reinterpret_cast<const double2*>(x + (int64_t)d.kt_col[t] * ncol + c0);
#pragma unroll
      for (int v = 0; v < V / 2; ++v) {
        const double2 r = row[v];
        y[2 * v] += a * r.x;
        y[2 * v + 1] += a * r.y;
      }
    }
    double2* qo = reinterpret_cast<double2*>(q + i * ncol + c0);
    const double2* xo = reinterpret_cast<const double2*>(x + i * ncol + c0);
#pragma unroll
    for (int v = 0; v < V / 2; ++v) {
      qo[v] = make_double2(y[2 * v], y[2 * v + 1]);
      const double2 xi = xo[v];
      pq[2 * v] += y[2 * v] * xi.x;
      pq[2 * v + 1] += y[2 * v + 1] * xi.y;
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v) lds[v * NT + threadIdx.x] = col_ok ? pq[v] : 0.0;
  __syncthreads();
  if (threadIdx.x < (unsigned)ncol) {
    const int cl = threadIdx.x / V, cv = threadIdx.x % V;
    double s = 0.0;
    for (int g = 0; g < NT / L; ++g) s += lds[cv * NT + g * L + cl];
    part[blockIdx.y * part_stride + (int64_t)blockIdx.x * ncol + threadIdx.x] = s;
  }
}

// Column-blocked form (ncol a multiple of 16, at most 4 blocks): the 8 XCDs
// are split evenly over the 16-column blocks and each XCD sweeps a
// contiguous share of the rows for its block only.  A row slice is then
// 128 B, so the band of neighbour rows one XCD touches fits its L2; the
// matrix is read once per column block.
__global__ void __launch_bounds__(NT) k_spmv_poisson_cb(const DevMesh* __restrict__ dm, const double* __restrict__ x,
                                                        int ncol, double* __restrict__ q, int64_t part_stride,
                                                        double* __restrict__ part) {
  INSTANCE;
  constexpr int L = 4, V = 4, CB = 16;
  __shared__ double lds[NT * V];
  x += d.oE * ncol;
  q += d.oE * ncol;
  const int nblk_c = ncol / CB;
  const int gpx = N_XCD / nblk_c;                 // XCDs per column block
  const int xcd = blockIdx.x % N_XCD, lb = blockIdx.x / N_XCD, nbx = gridDim.x / N_XCD;
  const int cblk = xcd / gpx, sub = xcd % gpx;
  const int64_t R = (d.N + gpx - 1) / gpx;
  const int64_t r0 = sub * R, r1 = (sub + 1) * R < d.N ? (sub + 1) * R : d.N;
  const int lane = (int)(threadIdx.x & (L - 1));
  const int c0 = cblk * CB + lane * V;
  double pq[V];
#pragma unroll
  for (int v = 0; v < V; ++v) pq[v] = 0.0;
  for (int64_t i = r0 + (int64_t)lb * (NT / L) + threadIdx.x / L; i < r1; i += (int64_t)nbx * (NT / L)) {
    const int beg = d.kt_ptr[i], end = d.kt_ptr[i + 1];
    double y[V];
#pragma unroll
    for (int v = 0; v < V; ++v) y[v] = 0.0;
    int t = beg;
    for (; t + 4 <= end; t += 4) {
      double2 xv[4][2];
      double av[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t j = d.kt_col[t + u];
        av[u] = d.kt_val[t + u];
        const double2* row = reinterpret_cast<const double2*>(x + j * ncol + c0);
        xv[u][0] = row[0];
        xv[u][1] = row[1];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        y[0] += av[u] * xv[u][0].x;
        y[1] += av[u] * xv[u][0].y;
        y[2] += av[u] * xv[u][1].x;
        y[3] += av[u] * xv[u][1].y;
      }
    }
    for (; t < end; ++t) {
      const double a = d.kt_val[t];
      const double2* row = reinterpret_cast<const double2*>(x + (int64_t)d.kt_col[t] * ncol + c0);
      const double2 r0v = row[0], r1v = row[1];
      y[0] += a * r0v.x;
      y[1] += a * r0v.y;
      y[2] += a * r1v.x;
      y[3] += a * r1v.y;
    }
    double2* qo = reinterpret_cast<double2*>(q + i * ncol + c0);
    const double2* xo = reinterpret_cast<const double2*>(x + i * ncol + c0);
    qo[0] = make_double2(y[0], y[1]);
    qo[1] = make_double2(y[2], y[3]);
    const double2 xa = xo[0], xb = xo[1];
    pq[0] += y[0] * xa.x;
    pq[1] += y[1] * xa.y;
    pq[2] += y[2] * xb.x;
    pq[3] += y[3] * xb.y;
  }
#pragma unroll
  for (int v = 0; v < V; ++v) lds[v * NT + threadIdx.x] = pq[v];
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += NT) {
    double s = 0.0;
    const int cc = c - cblk * CB;
    if (cc >= 0 && cc < CB) {
      const int cl = cc / V, cv = cc % V;
      for (int g = 0; g < NT / L; ++g) s += lds[cv * NT + g * L + cl];
    }
    part[blockIdx.y * part_stride + (int64_t)blockIdx.x * ncol + c] = s;
  }
}

template <int L, int V>
static int launch_spmv_poisson_v(const Batch& b, const double* x, int ncol, double* q, const PoissonWs& P,
                                 hipStream_t s) {
  if ((b.mx.sched_poi & 2) && ncol % 16 == 0 && (ncol == 16 || ncol == 32 || ncol == 64)) {
    const int grid = xcd_grid(b.mx.N * (ncol / 16), NT / 4, b.mx.grid_poi);
    hipLaunchKernelGGL(k_spmv_poisson_cb, dim3(grid, b.ni), dim3(NT), 0, s, b.dm, x, ncol, q, P.part_stride, P.part);
    return grid;
  }
  const int grid = xcd_grid(b.mx.N, NT / L, b.mx.grid_poi);
  hipLaunchKernelGGL((k_spmv_poisson_v<L, V>), dim3(grid, b.ni), dim3(NT), 0, s, b.dm, x, ncol, q, P.part_stride,
                     P.part);
  return grid;
}

template <int L>
static int launch_spmv_poisson_t(const Batch& b, const double* x, int ncol, double* q, const PoissonWs& P,
                                 hipStream_t s) {
  const int grid = xcd_grid(b.mx.N, NT / L, b.mx.grid_poi);
  hipLaunchKernelGGL((k_spmv_poisson<L>), dim3(grid, b.ni), dim3(NT), 0, s, b.dm, x, ncol, q, P.part_stride, P.part);
  return grid;
}

static int launch_spmv_poisson(const Batch& b, const double* x, int ncol, double* q, const PoissonWs& P,
                               hipStream_t s) {
  if (ncol % 2 == 0) {  // 16-byte column pairs
    if (ncol <= 4) return launch_spmv_poisson_v<2, 2>(b, x, ncol, q, P, s);
    if (ncol <= 16) return launch_spmv_poisson_v<4, 4>(b, x, ncol, q, P, s);
    if (ncol <= 32) return launch_spmv_poisson_v<8, 4>(b, x, ncol, q, P, s);
    return launch_spmv_poisson_v<16, 4>(b, x, ncol, q, P, s);
  }
  if (ncol <= 1) return launch_spmv_poisson_t<1>(b, x, ncol, q, P, s);
  if (ncol <= 2) return launch_spmv_poisson_t<2>(b, x, ncol, q, P, s);
  if (ncol <= 4) return launch_spmv_poisson_t<4>(b, x, ncol, q, P, s);
  if (ncol <= 8) return launch_spmv_poisson_t<8>(b, x, ncol, q, P, s);
  if (ncol <= 16) return launch_spmv_poisson_t<16>(b, x, ncol, q, P, s);
  if (ncol <= 32) return launch_spmv_poisson_t<32>(b, x, ncol, q, P, s);
  return launch_spmv_poisson_t<64>(b, x, ncol, q, P, s);
}

// --------------------------------------------------------------------------
// Jacobi-preconditioned CG, all columns of all instances at once with their
// own alpha and beta.  Scalars sc[i][slot][c] (SC_* in kernels.hpp).
// --------------------------------------------------------------------------
// alpha = rz / (p.q); one block per (column, instance)
__global__ void __launch_bounds__(NT) k_alpha_finish(const double* __restrict__ part, int64_t part_stride, int nb,
                                                     int ncol, double* __restrict__ sc) {
  __shared__ double lds4[4];
  const int c = blockIdx.x;
  part += blockIdx.y * part_stride;
  sc += (int64_t)blockIdx.y * 8 * ncol;
  const double s = sum_partials(part, nb, ncol, c, lds4);
  if (threadIdx.x == 0) {
    sc[SC_PQ * ncol + c] = s;
    const double rz = sc[SC_RZ * ncol + c];
    sc[SC_ALPHA * ncol + c] = (s != 0.0 && rz != 0.0) ? rz / s : 0.0;
  }
}

// x += alpha p; r -= alpha q; partial (r.D^-1 r, r.r).  x over full rows.
__global__ void __launch_bounds__(NT) k_cg_update2(const DevMesh* __restrict__ dm, double* __restrict__ x,
                                                   double* __restrict__ r, const double* __restrict__ p,
                                                   const double* __restrict__ q, int ncol,
                                                   const double* __restrict__ sc, int64_t part_stride,
                                                   double* __restrict__ part) {
  INSTANCE;
  __shared__ double lds[2 * NT];
  x += d.oF * ncol;
  r += d.oE * ncol;
  p += d.oE * ncol;
  q += d.oE * ncol;
  const int groups = NT / ncol;
  const int g = threadIdx.x / ncol, c = threadIdx.x - g * ncol;
  const bool act = g < groups;
  double rz = 0.0, rr = 0.0;
  if (act) {
    const double al = sc[(int64_t)blockIdx.y * 8 * ncol + SC_ALPHA * ncol + c];
    for (int64_t k = (int64_t)blockIdx.x * groups + g; k < d.N; k += (int64_t)gridDim.x * groups) {
      const int64_t e = k * ncol + c;
      x[e] += al * p[e];
      const double rn = r[e] - al * q[e];
      r[e] = rn;
      rz += rn * rn * d.kdiag_inv[k];
      rr += rn * rn;
    }
  }
  lds[threadIdx.x] = act ? rz : 0.0;
  lds[NT + threadIdx.x] = act ? rr : 0.0;
  __syncthreads();
  if (threadIdx.x < (unsigned)ncol) {
    double t = 0.0, u = 0.0;
    for (int gg = 0; gg < groups; ++gg) {
      t += lds[gg * ncol + threadIdx.x];
      u += lds[NT + gg * ncol + threadIdx.x];
    }
    double* pb = part + blockIdx.y * part_stride + (int64_t)blockIdx.x * 2 * ncol;
    pb[threadIdx.x] = t;
    pb[ncol + threadIdx.x] = u;
  }
}

// beta = rz_new / rz (mode 1) or initial rz (mode 0); rr.  One block per (column, instance).
__global__ void __launch_bounds__(NT) k_rz_finish(const double* __restrict__ part, int64_t part_stride, int nblk,
                                                  int ncol, double* __restrict__ sc, int mode) {
  __shared__ double lds4[4];
  const int c = blockIdx.x;
  part += blockIdx.y * part_stride;
  sc += (int64_t)blockIdx.y * 8 * ncol;
  const double s = sum_partials(part, nblk, 2 * ncol, c, lds4);
  const double u = sum_partials(part, nblk, 2 * ncol, ncol + c, lds4);
  if (threadIdx.x == 0) {
    if (mode == 1) {
      const double rz = sc[SC_RZ * ncol + c];
      sc[SC_BETA * ncol + c] = (rz != 0.0) ? s / rz : 0.0;
    }
    sc[SC_RZ * ncol + c] = s;
    sc[SC_RR * ncol + c] = u;
  }
}

// p = D^-1 r + beta p
__global__ void __launch_bounds__(NT) k_cg_p2(const DevMesh* __restrict__ dm, const double* __restrict__ r,
                                              double* __restrict__ p, int ncol, const double* __restrict__ sc) {
  INSTANCE;
  const int64_t total = d.N * ncol;
  r += d.oE * ncol;
  p += d.oE * ncol;
  const double* beta = sc + (int64_t)blockIdx.y * 8 * ncol + SC_BETA * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t k = e / ncol;
    const int c = (int)(e - k * ncol);
    p[e] = d.kdiag_inv[k] * r[e] + beta[c] * p[e];
  }
}

// start: r = rhs - q (warm) or rhs (cold, x = 0); p = D^-1 r; partial rz, rr.  x over full rows.
__global__ void __launch_bounds__(NT) k_cg_start2(const DevMesh* __restrict__ dm, double* __restrict__ x,
                                                  double* __restrict__ r, const double* __restrict__ q,
                                                  double* __restrict__ p, int ncol, int warm, int64_t part_stride,
                                                  double* __restrict__ part) {
  INSTANCE;
  __shared__ double lds[2 * NT];
  x += d.oF * ncol;
  r += d.oE * ncol;
  q += d.oE * ncol;
  p += d.oE * ncol;
  const int groups = NT / ncol;
  const int g = threadIdx.x / ncol, c = threadIdx.x - g * ncol;
  const bool act = g < groups;
  double rz = 0.0, rr = 0.0;
  if (act)
    for (int64_t k = (int64_t)blockIdx.x * groups + g; k < d.N; k += (int64_t)gridDim.x * groups) {
      const int64_t e = k * ncol + c;
      const double rn = warm ? r[e] - q[e] : r[e];
      if (!warm) x[e] = 0.0;
      r[e] = rn;
      p[e] = d.kdiag_inv[k] * rn;
      rz += rn * rn * d.kdiag_inv[k];
      rr += rn * rn;
    }
  lds[threadIdx.x] = act ? rz : 0.0;
  lds[NT + threadIdx.x] = act ? rr : 0.0;
  __syncthreads();
  if (threadIdx.x < (unsigned)ncol) {
    double t = 0.0, u = 0.0;
    for (int gg = 0; gg < groups; ++gg) {
      t += lds[gg * ncol + threadIdx.x];
      u += lds[NT + gg * ncol + threadIdx.x];
    }
    double* pb = part + blockIdx.y * part_stride + (int64_t)blockIdx.x * 2 * ncol;
    pb[threadIdx.x] = t;
    pb[ncol + threadIdx.x] = u;
  }
}

// DoF rows of x (full rows) into y (extended rows)
__global__ void __launch_bounds__(NT) k_copy_dofs(const DevMesh* __restrict__ dm, const double* __restrict__ x,
                                                  double* __restrict__ y, int ncol) {
  INSTANCE;
  const int64_t total = d.N * ncol;
  x += d.oF * ncol;
  y += d.oE * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) y[e] = x[e];
}

static int cg_blocks(const Batch& b, int ncol) { return nblocks(b.mx.N, NT / ncol, RED_BLOCKS); }

// q = K p, alpha from p.q
static void cg_apply2(const Batch& b, PoissonWs& P, double* pvec, double* qvec, hipStream_t s) {
  const int ncol = P.ncol;
  const bool rec = P.ev && P.ev_used + 2 <= P.ev_cap;
  if (rec) (void)hipEventRecord(P.ev[P.ev_used], s);
  const int nb1 = launch_spmv_poisson(b, pvec, ncol, qvec, P, s);
  if (rec) {
    (void)hipEventRecord(P.ev[P.ev_used + 1], s);
    P.ev_used += 2;
  }
  hipLaunchKernelGGL(k_alpha_finish, dim3(ncol, b.ni), dim3(NT), 0, s, P.part, P.part_stride, nb1, ncol, P.sc);
}

void launch_cg_start(const Batch& b, double* W, double* rhs_r, PoissonWs& P, int warm, hipStream_t s) {
  const int ncol = P.ncol;
  if (warm) {
    hipLaunchKernelGGL(k_copy_dofs, dim3(nblocks(b.mx.N * ncol, NT, 8192), b.ni), dim3(NT), 0, s, b.dm, W, P.p, ncol);
    cg_apply2(b, P, P.p, P.q, s);
  }
  const int nb = cg_blocks(b, ncol);
  hipLaunchKernelGGL(k_cg_start2, dim3(nb, b.ni), dim3(NT), 0, s, b.dm, W, rhs_r, P.q, P.p, ncol, warm, P.part_stride,
                     P.part);
  hipLaunchKernelGGL(k_rz_finish, dim3(ncol, b.ni), dim3(NT), 0, s, P.part, P.part_stride, nb, ncol, P.sc, 0);
}

void launch_cg_step(const Batch& b, double* W, PoissonWs& P, hipStream_t s) {
  const int ncol = P.ncol;
  cg_apply2(b, P, P.p, P.q, s);
  const int nb = cg_blocks(b, ncol);
  hipLaunchKernelGGL(k_cg_update2, dim3(nb, b.ni), dim3(NT), 0, s, b.dm, W, P.r, P.p, P.q, ncol, P.sc, P.part_stride,
                     P.part);
  hipLaunchKernelGGL(k_rz_finish, dim3(ncol, b.ni), dim3(NT), 0, s, P.part, P.part_stride, nb, ncol, P.sc, 1);
  hipLaunchKernelGGL(k_cg_p2, dim3(nblocks(b.mx.N * ncol, NT, 8192), b.ni), dim3(NT), 0, s, b.dm, P.r, P.p, ncol,
                     P.sc);
}

// y = a x + b y over nd doubles (a, b real)
__global__ void __launch_bounds__(NT) k_axpby(int64_t nd, double a, const double* __restrict__ x, double b,
                                              double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nd; i += (int64_t)gridDim.x * NT)
    y[i] = a * x[i] + b * y[i];
}
void launch_axpby(int64_t nd, double a, const double* x, double b, double* y, hipStream_t s) {
  if (nd > 0) hipLaunchKernelGGL(k_axpby, dim3(nblocks(nd, NT, 8192)), dim3(NT), 0, s, nd, a, x, b, y);
}

}  // namespace mh
