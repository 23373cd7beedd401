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

#include <algorithm>
#include <type_traits>

#include "devutil.hpp"
#include "kernels.hpp"

namespace mh {

#define INSTANCE const DevMesh& d = dm[blockIdx.y]

// --------------------------------------------------------------------------
// Orbital operator.  mode 0: F = load vector; 1: M^-1 F; 2: M^-1 F - v lam.
// Non-master DoFs get their final value in `out`; masters and hanging nodes
// store the load value in `acc`.
// --------------------------------------------------------------------------
// ASM: the stiffness part is taken from kq, the assembled K~ u on the DoF
// rows (constraints folded in, so hanging rows carry no stiffness and the
// masters already hold their hanging neighbours' share); the node then only
// adds its diagonal and mean-field terms.
// VEL: the first-derivative term -i a.S u of the velocity gauge (a = A(t) e,
// or e alone for the momentum, diag_mode 4), S the Gauss-Lobatto Galerkin
// derivative in its antisymmetric form: per cell (h/2)^2 (Qs x W x W) along x
// and likewise along y and z, so its line sums share the stiffness's loads.
// ECS: exterior complex scaling of the one-body part (diag_mode 0..2, on
// instances that carry it): each cell's stiffness and derivative loads along
// d take the contour factors e^{i (s - 2 b_d) theta} and e^{i (s - b_d) theta}
// (s scaled directions, b_d whether d is one), the node's cell sum is
// multiplied by rho = m / m_theta, and the potential and field weights are the
// continued complex ones, so the load is in units of the real mass; the
// mean-field load is unchanged.
template <int P, int L, bool ASM, bool VEL, bool ECS>
__global__ void __launch_bounds__(NT) k_stencil_orb(const DevMesh* __restrict__ dm, const double2* __restrict__ u,
                                                    const double* __restrict__ Ef, int diag_mode,
                                                    const double* __restrict__ Upk, const double2* __restrict__ ginv,
                                                    int mode, const double2* __restrict__ lam,
                                                    double2* __restrict__ out, double2* __restrict__ acc,
                                                    const double2* __restrict__ kq) {
  INSTANCE;
  constexpr int P3 = P * P * P;
  // per wave: the packed mean-field matrices of its 64 / L nodes (at most 64 doubles each)
  __shared__ double sU[NT / 64][512];
  const int n = d.n;
  const int64_t o = d.oE * n;
  u += o;
  out += o;
  acc += o;
  if (ASM) kq += o;
  Upk += d.oE * n * n;
  ginv += (int64_t)blockIdx.y * n * n;
  if (lam) lam += (int64_t)blockIdx.y * n * n;
  const double E = (diag_mode == 1 || diag_mode == 2) ? Ef[0] * d.E0 : 0.0;
  // velocity term: vector potential a = A e (diag_mode 4: a = e); no stiffness for diag_mode 4
  const double av = diag_mode == 4 ? 1.0 : E;
  const double ax = VEL ? av * d.pol[0] : 0.0, ay = VEL ? av * d.pol[1] : 0.0, az = VEL ? av * d.pol[2] : 0.0;
  const bool stiff = diag_mode <= 2;
  const double Elen = d.gauge == 1 ? 0.0 : E;   // the length-gauge term only in the length gauge
  const bool ecs_i = ECS && d.ecs && diag_mode <= 2;
  // e^{i k theta}, k = -2..3, staged in LDS: the cells pick their factors by a per-lane index
  __shared__ double2 spw[6];
  if (ECS) {
    if (threadIdx.x < 6) spw[threadIdx.x] = make_double2(d.ecs_pw[2 * threadIdx.x], d.ecs_pw[2 * threadIdx.x + 1]);
    __syncthreads();
  }
  auto pw = [&](int k) { return spw[k + 2]; };
  const XcdSweep sw = xcd_sweep(d.NE, NT / L, d.sched_orb & 1);
  // all L lanes of a node share i, so a node group enters and leaves together
  for (int64_t i = sw.start + threadIdx.x / L; i < sw.end; i += sw.step) {
    const int p = (int)(threadIdx.x & (L - 1));
    const bool act = p < n;
    double2 y = make_double2(0.0, 0.0), ui = make_double2(0.0, 0.0);
    if (act) ui = u[i * n + p];
    // the node's 8 incidence codes in two 16-byte loads (row of 32 bytes)
    typedef int ivec4_t __attribute__((ext_vector_type(4)));
    const auto* inc4 = reinterpret_cast<const __attribute__((address_space(1))) ivec4_t*>(gbl(d.node_inc) + i * 8);
    ivec4_t ca = ivec4_t{-1, -1, -1, -1}, cb = ca;
    if (!ASM) {
      ca = inc4[0];
      cb = inc4[1];
    } else if (diag_mode != 3 && i < d.N && act) {
      y = cscale(0.5, kq[i * n + p]);  // (1/2) K~ u
    }
    if (diag_mode == 3) ca = cb = ivec4_t{-1, -1, -1, -1};  // dipole weights only: no stiffness
    const int codes[8] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int code = codes[t];
      if (code < 0) continue;
      const int64_t K = code >> 6;
      const int loc = code & 63;
      const int a = loc % P, b = (loc / P) % P, c = loc / (P * P);
      const auto* cn = gbl(d.cell_nodes) + K * P3;
      double2 s0 = make_double2(0.0, 0.0), s1 = s0, s2 = s0;
      double2 t0 = s0, t1 = s0, t2 = s0;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int j0 = cn[(c * P + b) * P + q], j1 = cn[(c * P + q) * P + a], j2 = cn[(q * P + b) * P + a];
        const double A0 = d.A[a * P + q], A1 = d.A[b * P + q], A2 = d.A[c * P + q];
        // the point q of a line through the node that is the node itself
        // (q == a along x, ...) takes its value from the register, not memory
        if (act) {
          if (j0 < d.NE) {
            double2 v;
            if (q == a) v = ui;
            else v = u[(int64_t)j0 * n + p];
            s0.x += A0 * v.x; s0.y += A0 * v.y;
            if (VEL) { const double Q = d.Qs[a * P + q]; t0.x += Q * v.x; t0.y += Q * v.y; }
          }
          if (j1 < d.NE) {
            double2 v;
            if (q == b) v = ui;
            else v = u[(int64_t)j1 * n + p];
            s1.x += A1 * v.x; s1.y += A1 * v.y;
            if (VEL) { const double Q = d.Qs[b * P + q]; t1.x += Q * v.x; t1.y += Q * v.y; }
          }
          if (j2 < d.NE) {
            double2 v;
            if (q == c) v = ui;
            else v = u[(int64_t)j2 * n + p];
            s2.x += A2 * v.x; s2.y += A2 * v.y;
            if (VEL) { const double Q = d.Qs[c * P + q]; t2.x += Q * v.x; t2.y += Q * v.y; }
          }
        }
      }
      const double hk = gbl(d.cell_hh)[K];  // h/2
      int sc = 0, b0 = 0, b1 = 0, b2 = 0;    // scaled directions of the cell (complex scaling)
      if (ecs_i) {
        const int code = gbl(d.ecs_code)[K];
        b0 = code & 1;
        b1 = (code >> 1) & 1;
        b2 = (code >> 2) & 1;
        sc = b0 + b1 + b2;
      }
      if (stiff) {
        const double hh = 0.5 * hk;  // (1/2) K with K_cell = (h/2)(...)
        const double f0 = hh * d.w[b] * d.w[c], f1 = hh * d.w[a] * d.w[c], f2 = hh * d.w[a] * d.w[b];
        if (ecs_i && sc) {
          y = cadd(y, cscale(f0, cmul(pw(sc - 2 * b0), s0)));
          y = cadd(y, cscale(f1, cmul(pw(sc - 2 * b1), s1)));
          y = cadd(y, cscale(f2, cmul(pw(sc - 2 * b2), s2)));
        } else {
          y.x += f0 * s0.x + f1 * s1.x + f2 * s2.x;
          y.y += f0 * s0.y + f1 * s1.y + f2 * s2.y;
        }
      }
      if (VEL) {  // y += -i (h/2)^2 (ax Wb Wc t0 + ay Wa Wc t1 + az Wa Wb t2)
        const double h2 = hk * hk;
        const double g0 = h2 * ax * d.w[b] * d.w[c], g1 = h2 * ay * d.w[a] * d.w[c], g2 = h2 * az * d.w[a] * d.w[b];
        if (ecs_i && sc) {
          t0 = cmul(pw(sc - b0), t0);
          t1 = cmul(pw(sc - b1), t1);
          t2 = cmul(pw(sc - b2), t2);
        }
        y.x += g0 * t0.y + g1 * t1.y + g2 * t2.y;
        y.y -= g0 * t0.x + g1 * t1.x + g2 * t2.x;
      }
    }
    if (ecs_i && act) {
      const auto* rho = gbl(d.ecs_rho);
      y = cmul(make_double2(rho[2 * i], rho[2 * i + 1]), y);
    }
    if (diag_mode >= 1 && diag_mode <= 3 && act) {
      if (ecs_i && diag_mode != 3) {
        const auto* vc = gbl(d.ecs_v);
        const auto* zc = gbl(d.ecs_mz);
        const double2 dg = make_double2(vc[2 * i] + Elen * zc[2 * i], vc[2 * i + 1] + Elen * zc[2 * i + 1]);
        y = cadd(y, cmul(dg, ui));
      } else {
        const double dg = diag_mode == 3 ? gbl(d.mz)[i] : gbl(d.v)[i] + Elen * gbl(d.mz)[i];
        y.x += dg * ui.x;
        y.y += dg * ui.y;
      }
    }
    if (diag_mode == 2) {
      // z_p = sum_q U_pq u_q (U Hermitian, packed: Up[o][q] = Re U_oq, Up[q][o] = Im U_oq for o < q).
      // The node's n^2 packed values are read by its L lanes in consecutive
      // words and staged in the wave's LDS slice, where each lane then finds
      // the entries of its row and column.
      double* Up = &sU[threadIdx.x >> 6][((threadIdx.x & 63) / L) * (n * n)];
      {
        const auto* Ug = gbl(Upk) + i * n * n;
        for (int f = (int)(threadIdx.x & (L - 1)); f < n * n; f += L) Up[f] = Ug[f];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
      __builtin_amdgcn_wave_barrier();  // the slice is rewritten for the wave's next nodes
      double2 wv = make_double2(0.0, 0.0);
      for (int oo = 0; oo < n; ++oo) {
        const double2 zo = make_double2(__shfl(z.x, oo, L), __shfl(z.y, oo, L));
        if (act) wv = cadd(wv, cmul(ginv[p * n + oo], zo));
      }
      if (act) {
        const double mi = gbl(d.m)[i];
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
    const int mi = dof ? gbl(d.ma_index)[i] : -1;
    if (dof && mi < 0) {
      if (mode == 0) out[i * n + p] = y;
      else out[i * n + p] = csub(cscale(gbl(d.inv_mass)[i], y), lm);
    } else {
      acc[i * n + p] = y;
    }
  }
}

// Masters: load value = acc_k + sum_h c_hk acc_h (transposed constraints).
// One master per group of GATHER_G lanes splitting its hanging rows (about
// fifty), combined by shuffles; all n orbitals at once.
constexpr int GATHER_G = 16;
__global__ void __launch_bounds__(NT) k_ma_gather_orb(const DevMesh* __restrict__ dm, const double2* __restrict__ acc,
                                                      int mode, double2* __restrict__ out,
                                                      double2* __restrict__ ma_b) {
  INSTANCE;
  const int n = d.n;
  const int64_t o = d.oE * n, om = d.oMa * n;
  const int g = (int)(threadIdx.x & (GATHER_G - 1));
  const int64_t groups = (int64_t)gridDim.x * (NT / GATHER_G);
  for (int64_t i = ((int64_t)blockIdx.x * NT + threadIdx.x) / GATHER_G; i < d.nMa; i += groups) {
    const int64_t k = gbl(d.ma_dof)[i];
    double fx[8], fy[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) { fx[p] = 0.0; fy[p] = 0.0; }
    if (g == 0) {
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (p < n) {
          const double2 a = acc[o + k * n + p];
          fx[p] = a.x;
          fy[p] = a.y;
        }
    }
    const auto* ctp = gbl(d.ct_ptr);
    for (int t = ctp[i] + g; t < ctp[i + 1]; t += GATHER_G) {
      const double w = gbl(d.ct_w)[t];
      const double2* row = acc + o + (int64_t)gbl(d.ct_row)[t] * n;
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (p < n) {
          const double2 a = row[p];
          fx[p] += w * a.x;
          fy[p] += w * a.y;
        }
    }
#pragma unroll
    for (int off = GATHER_G / 2; off > 0; off >>= 1)
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (p < n) {
          fx[p] += __shfl_xor(fx[p], off, GATHER_G);
          fy[p] += __shfl_xor(fy[p], off, GATHER_G);
        }
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (p < n && p % GATHER_G == g) {
        const double2 f = make_double2(fx[p], fy[p]);
        if (mode == 0) out[o + k * n + p] = f;
        else ma_b[om + i * n + p] = f;
      }
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
    const int mi = gbl(d.ma_index)[k];
    if (mi < 0) out[o + idx] = cscale(gbl(d.inv_mass)[k], f[o + idx]);
    else ma_b[om + (int64_t)mi * n + (idx - k * n)] = f[o + idx];
  }
}

static void launch_spmv_poisson(const Batch& b, const double* x, const double* pprev, double* pout, int ncol,
                                double* q, const PoissonWs& P, int k, hipStream_t s);

template <int P, int L>
static void launch_stencil_orb_t(const Batch& b, const double* u, const double* Ef, int diag_mode, const double* Upk,
                                 const double* ginv, int mode, const double* lam, double* out, double* acc,
                                 const double* kq, hipStream_t s) {
  const int grid = xcd_grid(b.mx.NE, NT / L, b.mx.grid_orb);
  const bool vel = diag_mode == 4 || (b.mx.gauge == 1 && (diag_mode == 1 || diag_mode == 2));
  const bool ecs = b.mx.ecs && diag_mode <= 2;
  if (kq)
    hipLaunchKernelGGL((k_stencil_orb<P, L, true, false, false>), dim3(grid, b.ni), dim3(NT), 0, s, b.dm,
                       (const double2*)u, Ef, diag_mode, Upk, (const double2*)ginv, mode, (const double2*)lam,
                       (double2*)out, (double2*)acc, (const double2*)kq);
  else if (vel && ecs)
    hipLaunchKernelGGL((k_stencil_orb<P, L, false, true, true>), dim3(grid, b.ni), dim3(NT), 0, s, b.dm,
                       (const double2*)u, Ef, diag_mode, Upk, (const double2*)ginv, mode, (const double2*)lam,
                       (double2*)out, (double2*)acc, (const double2*)nullptr);
  else if (vel)
    hipLaunchKernelGGL((k_stencil_orb<P, L, false, true, false>), dim3(grid, b.ni), dim3(NT), 0, s, b.dm,
                       (const double2*)u, Ef, diag_mode, Upk, (const double2*)ginv, mode, (const double2*)lam,
                       (double2*)out, (double2*)acc, (const double2*)nullptr);
  else if (ecs)
    hipLaunchKernelGGL((k_stencil_orb<P, L, false, false, true>), dim3(grid, b.ni), dim3(NT), 0, s, b.dm,
                       (const double2*)u, Ef, diag_mode, Upk, (const double2*)ginv, mode, (const double2*)lam,
                       (double2*)out, (double2*)acc, (const double2*)nullptr);
  else
    hipLaunchKernelGGL((k_stencil_orb<P, L, false, false, false>), dim3(grid, b.ni), dim3(NT), 0, s, b.dm,
                       (const double2*)u, Ef, diag_mode, Upk, (const double2*)ginv, mode, (const double2*)lam,
                       (double2*)out, (double2*)acc, (const double2*)nullptr);
}

template <int P>
static void launch_stencil_orb_p(const Batch& b, const double* u, const double* Ef, int diag_mode, const double* Upk,
                                 const double* ginv, int mode, const double* lam, double* out, double* acc,
                                 const double* kq, hipStream_t s) {
  const int n = b.mx.n;
  if (n <= 1) launch_stencil_orb_t<P, 1>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, kq, s);
  else if (n <= 2) launch_stencil_orb_t<P, 2>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, kq, s);
  else if (n <= 4) launch_stencil_orb_t<P, 4>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, kq, s);
  else launch_stencil_orb_t<P, 8>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, kq, s);
}

// Orbital schedule bit 2: the stiffness part by the assembled Poisson
// operator K~ applied to the 2n real columns of the orbital array (the tuned
// SpMV, long rows by waves), then the node pass adds the diagonal and
// mean-field terms; kq [tE][n] and kred (RED_SLOTS x 2n per instance) are
// scratch.
void launch_stencil_orb(const Batch& b, const double* u, const double* Ef, int diag_mode, const double* Upk,
                        const double* ginv, int mode, const double* lam, double* out, double* acc, double* kq,
                        double* kred, hipStream_t s) {
  // the velocity term, the momentum and complex scaling run node by node (their line sums
  // share the stiffness's loads; the scaled stiffness is complex)
  const bool vel = diag_mode == 4 || (b.mx.gauge == 1 && (diag_mode == 1 || diag_mode == 2));
  const bool asm_k = (b.mx.sched_orb & 4) && kq && kred && !vel && !(b.mx.ecs && diag_mode <= 2);
  if (asm_k && diag_mode != 3) {
    PoissonWs Pk;
    Pk.red = kred;
    // at 2n <= 16 columns the stiffness pass runs best on at most 8192
    // workgroups, whatever cap the Poisson schedule of the pair columns takes
    Batch bk = b;
    bk.mx.grid_poi = std::min(b.mx.grid_poi, 8192);
    launch_spmv_poisson(bk, u, u, kq, 2 * b.mx.n, kq, Pk, -1, s);
  }
  const double* q = asm_k ? kq : nullptr;
  switch (b.mx.P) {
    case 2: launch_stencil_orb_p<2>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, q, s); break;
    case 3: launch_stencil_orb_p<3>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, q, s); break;
    default: launch_stencil_orb_p<4>(b, u, Ef, diag_mode, Upk, ginv, mode, lam, out, acc, q, s);
  }
}

void launch_ma_gather_orb(const Batch& b, const double* acc, int mode, double* out, double* ma_b, hipStream_t s) {
  if (b.mx.nMa == 0) return;
  hipLaunchKernelGGL(k_ma_gather_orb, dim3(nblocks(b.mx.nMa * GATHER_G), b.ni), dim3(NT), 0, s, b.dm,
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
// into the matrix.  The matrix (about 12 B per entry, ~22 entries per row)
// is shared by all n^2 real columns.  L lanes per row, each owning V
// adjacent columns (16-byte loads for V >= 2); fused p.q partials.  x, q
// over extended rows (batch offset oE).
//
// Row lengths are very uneven: the masters of hanging nodes carry the
// constrained neighbourhood (up to several hundred entries against a median
// near 13).  Left to L lanes, such a row would keep its workgroup waiting
// for hundreds of dependent loads.  So the first `nlb` workgroups take the
// rows longer than KT_LONG, one row at a time per workgroup with all its
// NT / L lane groups splitting the entries and an LDS reduction; the other
// workgroups sweep the remaining rows.
// --------------------------------------------------------------------------
// Operator pass modes: plain q = K x (SP_PLAIN); the CG direction formed on
// the fly (SP_CG); and the two Chebyshev smoothing passes of the multigrid
// cycle on the finest level, which replace q by the smoother's update:
// SP_CHEB0 runs the first two steps from z = 0 (its operand s0 D^-1 r is
// formed on the fly), SP_CHEB runs one step on a given z into another array.
// SP_CHEB_RZ is the second SP_CHEB step with r.z accumulated for the
// multigrid-preconditioned CG.  SP_RES writes the residual r - K z that the
// restriction to the next multigrid level reads.
enum { SP_PLAIN = 0, SP_CG = 1, SP_CHEB0 = 2, SP_CHEB = 3, SP_CHEB_RZ = 4, SP_RES = 5 };

// Value of the operand at row j, columns c0 .. c0+V: x itself; (SP_CG) the CG
// direction p_j = D^-1_j r_j + beta p_prev,j formed on the fly (x = r then);
// (SP_CHEB0) beta D^-1_j x_j (x = r, beta = s0).
// T: storage type of the operand arrays (double; float for the finest-level
// multigrid arrays of Poisson schedule bit 6).  Arithmetic is in double.
template <int V, int MODE, class T>
__device__ __forceinline__ void operand_row(const __attribute__((address_space(1))) T* xg,
                                            const __attribute__((address_space(1))) T* pg,
                                            const __attribute__((address_space(1))) double* dinv, const double* beta,
                                            int64_t j, int ld, int c0, double* out) {
  load_vals<V>(xg + j * ld + c0, out);  // 16-byte loads (ncol and c0 multiples of V)
  if constexpr (MODE == SP_CHEB0) {
    const double dj = dinv[j];
#pragma unroll
    for (int v = 0; v < V; ++v) out[v] = beta[v] * dj * out[v];
  }
  if constexpr (MODE == SP_CG) {
    const double dj = dinv[j];
    double pv[V];
    load_vals<V>(pg + j * ld + c0, pv);
#pragma unroll
    for (int v = 0; v < V; ++v) out[v] = dj * out[v] + (beta[v] != 0.0 ? beta[v] * pv[v] : 0.0);
  }
}

// y += sum over entries t = beg, beg + stride, ... < end of val[t] operand(col[t]);
// four entries per round with all their loads issued together.  Past the end
// the index is clamped to the row's last entry (every row holds its diagonal)
// and the coefficient zeroed, so the loads need no branch.
template <int V, int MODE, class T>
__device__ __forceinline__ void spmv_row_part(const DevMesh& d, const T* __restrict__ x,
                                              const T* __restrict__ pprev, const double* beta, int ld, int c0,
                                              int beg, int end, int stride, double* y) {
  const auto* kcol = gbl(d.kt_col);
  const auto* kval = gbl(d.kt_val);
  const auto* kvalf = gbl(d.kt_valf);   // the float passes read the float copy
  const auto* xg = gbl(x);
  const auto* pg = gbl(pprev);
  const auto* dinv = gbl(d.kdiag_inv);
  for (int t = beg; t < end; t += 4 * stride) {
    double av[4];
    double xv[4][V];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int tt = t + u * stride;
      const int tc = tt < end ? tt : end - 1;
      const int64_t j = kcol[tc];
      double a;
      if constexpr (std::is_same<T, float>::value) a = kvalf[tc];
      else a = kval[tc];
      av[u] = tt < end ? a : 0.0;
      operand_row<V, MODE, T>(xg, pg, dinv, beta, j, ld, c0, xv[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < V; ++v) y[v] += av[u] * xv[u][v];
  }
}

// Row i done, y = (K operand)_i.  SP_PLAIN / SP_CG: q_i = y, (SP_CG) p_i =
// the operand of row i, and the p.q partial.
// Chebyshev passes (x: the operand's source, pprev = r, pout = z out, q = d,
// cf = the instance's coefficients s0, c1, c2; step k of SP_CHEB, step 1 for
// SP_CHEB_RZ):
//   SP_CHEB0: d0 = s0 D^-1 r, d = c1 d0 + c2 D^-1 (r - y), z = d0 + d (d not
//             stored when bit 8 of k is set: no further step reads it);
//   SP_CHEB:  d = c1 d + c D^-1 (r - y) (k = 0: c1 d dropped, c = s0; else
//             c1, c = c2 of step k), z = x + d; SP_CHEB_RZ also the r.z
//             partial (in pq), its step being k >> 4 (its slot k & 15); it is
//             the last step of a smoothing, so d is not stored.
// cf: s0, then (c1, c2) of each step from 1 on.
// SP_RES (x = z, pprev = r): q_i = r_i - y.
template <int V, int MODE, class T>
__device__ __forceinline__ void spmv_store(const DevMesh& d, T* __restrict__ q, T* __restrict__ pout,
                                           const T* __restrict__ x, const T* __restrict__ pprev,
                                           const double* beta, int64_t i, int ld, int c0, const double* y,
                                           double* pq, const double* cf, int k) {
  if constexpr (MODE == SP_RES) {
    double rv[V];
    operand_row<V, SP_PLAIN, T>(gbl(pprev), gbl(pprev), gbl(d.kdiag_inv), beta, i, ld, c0, rv);
    T* qo = q + i * ld + c0;
#pragma unroll
    for (int v = 0; v < V; ++v) qo[v] = (T)(rv[v] - y[v]);
  } else if constexpr (MODE == SP_CHEB0 || MODE == SP_CHEB || MODE == SP_CHEB_RZ) {
    const int step = MODE == SP_CHEB_RZ ? k >> 4 : k;
    const double di = gbl(d.kdiag_inv)[i];
    double rv[V], xv[V], dv[V];
    operand_row<V, SP_PLAIN, T>(gbl(pprev), gbl(pprev), gbl(d.kdiag_inv), beta, i, ld, c0, rv);
    if constexpr (MODE != SP_CHEB0) {
      operand_row<V, SP_PLAIN, T>(gbl(x), gbl(x), gbl(d.kdiag_inv), beta, i, ld, c0, xv);
      if (step > 0) operand_row<V, SP_PLAIN, T>(gbl((const T*)q), gbl(x), gbl(d.kdiag_inv), beta, i, ld, c0, dv);
    }
    T* qo = q + i * ld + c0;
    T* po = pout + i * ld + c0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if constexpr (MODE == SP_CHEB0) {
        const double d0 = cf[0] * di * rv[v];
        const double dn = cf[1] * d0 + cf[2] * di * (rv[v] - y[v]);  // step 1
        if (!(k & 256)) qo[v] = (T)dn;
        po[v] = (T)(d0 + dn);
      } else {
        const double dn = (step > 0 ? cf[2 * step - 1] * dv[v] + cf[2 * step] * di * (rv[v] - y[v])
                                    : cf[0] * di * (rv[v] - y[v]));
        const double zn = xv[v] + dn;
        if constexpr (MODE != SP_CHEB_RZ) qo[v] = (T)dn;
        po[v] = (T)zn;
        if constexpr (MODE == SP_CHEB_RZ) pq[v] += rv[v] * zn;
      }
    }
  } else {
    double pi[V];
    operand_row<V, MODE, T>(gbl(x), gbl(pprev), gbl(d.kdiag_inv), beta, i, ld, c0, pi);
    T* qo = q + i * ld + c0;
    T* po = pout + i * ld + c0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      qo[v] = (T)y[v];
      if constexpr (MODE == SP_CG) po[v] = (T)pi[v];
      pq[v] += y[v] * pi[v];
    }
  }
}

// Columns [col0, col0 + nc) of arrays with ld columns per row, col0 = blockIdx.z * nc
// (nc = ld without column blocking).  SELL: the short rows come from the
// sliced-ELL copy, a wave taking 64 / L slots of one slice (one width for all
// its rows), so each round of entries is read as consecutive words.
// MODE: SP_*; red: the CG accumulators ([ni][RED_SLOTS][ld]); k: the CG
// iteration (SP_CG; see launch_spmv_poisson for SP_PLAIN), the
// smoothing step (SP_CHEB) or the r.z slot (SP_CHEB0 clears it, SP_CHEB_RZ
// accumulates into slot k & 15 at step k >> 4).
template <int L, int V, int MODE, bool SELL, class T>
__global__ void __launch_bounds__(NT) k_spmv_poisson(const DevMesh* __restrict__ dm, const T* __restrict__ x,
                                                     const T* __restrict__ pprev, T* __restrict__ pout,
                                                     int ld, int nc, T* __restrict__ q, int nlb,
                                                     double* __restrict__ red, int k, double* __restrict__ part) {
  constexpr bool FUSE = MODE == SP_CG;
  INSTANCE;
  if (d.cg_done && *d.cg_done) return;  // converged instance of a batch CG (batches take no partials)
  __shared__ double lds[NT * V];
  // column block: blockIdx.z, or with schedule bit 7 the XCD's (xcd_sweep_cols;
  // the grid then runs all column blocks along x)
  const int nb_col = ld / nc;
  const bool aff = (d.sched_poi & 128) && nb_col > 1 && N_XCD % nb_col == 0;
  const int col0 = (aff ? ((int)blockIdx.x % N_XCD) % nb_col : (int)blockIdx.z) * nc;
  // one workgroup per column block clears the slots below (workgroup 0 of the
  // block's z slice; with bit 7 workgroups 0 .. nb_col - 1, one per block)
  const bool first_wg = aff ? (int)blockIdx.x < nb_col : blockIdx.x == 0;
  x += d.oE * ld + col0;
  q += d.oE * ld + col0;
  pprev += d.oE * ld + col0;
  pout += d.oE * ld + col0;
  double cf[2 * MG_MAX_DEG - 1];
#pragma unroll
  for (int j = 0; j < 2 * MG_MAX_DEG - 1; ++j) cf[j] = d.mgc[j];
  red += (int64_t)blockIdx.y * RED_SLOTS * ld + col0;
  const int lane = (int)(threadIdx.x & (L - 1));
  const int c0 = lane * V;
  const bool col_ok = c0 < nc;
  // beta_k = rz_k / rz_{k-1} per column (0 at the first iteration); s0 for SP_CHEB0
  double beta[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    beta[v] = MODE == SP_CHEB0 ? cf[0] : 0.0;
    if (FUSE && k > 0 && c0 + v < nc) {
      const double rzk = red[(RED_RZ + k % 3) * ld + c0 + v], rzp = red[(RED_RZ + (k + 2) % 3) * ld + c0 + v];
      beta[v] = rzp != 0.0 ? rzk / rzp : 0.0;
    }
  }
  double pq[V];
#pragma unroll
  for (int v = 0; v < V; ++v) pq[v] = 0.0;
  if ((int)blockIdx.x < nlb) {
    // long rows: one per wave at a time, its 64 / L lane groups splitting the
    // entries, combined by shuffles (no workgroup barrier)
    constexpr int SEG = 64 / L;
    const int wave = threadIdx.x >> 6, seg = (threadIdx.x & 63) / L;
    // the long-row workgroups of this column block: all of them, or with column
    // blocks bound to XCDs those on this XCD's group (index gi of ng)
    int gi = (int)blockIdx.x, ng = nlb;
    if (aff) {
      const int G = N_XCD / nb_col;
      gi = ((int)blockIdx.x / N_XCD) * G + ((int)blockIdx.x % N_XCD) / nb_col;
      ng = nlb / N_XCD * G;
    }
    for (int64_t lr = (int64_t)gi * (NT / 64) + wave; lr < d.n_long; lr += (int64_t)ng * (NT / 64)) {
      const int64_t i = gbl(d.kt_long)[lr];
      const int beg = gbl(d.kt_ptr)[i], end = gbl(d.kt_ptr)[i + 1];
      double y[V];
#pragma unroll
      for (int v = 0; v < V; ++v) y[v] = 0.0;
      if (col_ok) spmv_row_part<V, MODE, T>(d, x, pprev, beta, ld, c0, beg + seg, end, SEG, y);
#pragma unroll
      for (int off = L; off < 64; off <<= 1)
#pragma unroll
        for (int v = 0; v < V; ++v) y[v] += __shfl_xor(y[v], off, 64);
      if (seg == 0 && col_ok) spmv_store<V, MODE, T>(d, q, pout, x, pprev, beta, i, ld, c0, y, pq, cf, k);
    }
  } else if constexpr (SELL) {
    constexpr int R = 64 / L;  // slots per wave
    const int wave = threadIdx.x >> 6, slot_in = (threadIdx.x & 63) / L;
    const XcdSweep sw =
        aff ? xcd_sweep_cols(d.n_slices * L, NT / 64, nb_col, (int)blockIdx.x - nlb, (int)gridDim.x - nlb)
            : xcd_sweep(d.n_slices * L, NT / 64, d.sched_poi & 1, (int)blockIdx.x - nlb, (int)gridDim.x - nlb);
    const auto* sptr = gbl(d.sell_ptr);
    const auto* srow = gbl(d.sell_row);
    const auto* scol = gbl(d.sell_col);
    const auto* sval = gbl(d.sell_val);
    const auto* svalf = gbl(d.sell_valf);   // the float passes read the float copy
    const auto* xg = gbl(x);
    const auto* pg = gbl(pprev);
    const auto* dinv = gbl(d.kdiag_inv);
    for (int64_t u = sw.start + wave; u < sw.end; u += sw.step) {
      const int64_t sl = u / L;
      const int slot = (int)(u - sl * L) * R + slot_in;
      const int i = srow[sl * SELL_H + slot];
      if (i < 0 || !col_ok) continue;
      const int base = sptr[sl], width = (sptr[sl + 1] - base) / SELL_H;
      double y[V];
#pragma unroll
      for (int v = 0; v < V; ++v) y[v] = 0.0;
      for (int t = 0; t < width; t += 4) {
        double av[4];
        double xv[4][V];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int e = base + (t + h) * SELL_H + slot;
          if constexpr (std::is_same<T, float>::value) av[h] = svalf[e];
          else av[h] = sval[e];
          operand_row<V, MODE, T>(xg, pg, dinv, beta, (int64_t)scol[e], ld, c0, xv[h]);
        }
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
          for (int v = 0; v < V; ++v) y[v] += av[h] * xv[h][v];
      }
      spmv_store<V, MODE, T>(d, q, pout, x, pprev, beta, i, ld, c0, y, pq, cf, k);
    }
  } else {
    const XcdSweep sw = aff ? xcd_sweep_cols(d.N, NT / L, nb_col, (int)blockIdx.x - nlb, (int)gridDim.x - nlb)
                            : xcd_sweep(d.N, NT / L, d.sched_poi & 1, (int)blockIdx.x - nlb, (int)gridDim.x - nlb);
    for (int64_t i = sw.start + threadIdx.x / L; i < sw.end; i += sw.step) {
      if (!col_ok) continue;
      const int beg = gbl(d.kt_ptr)[i], end = gbl(d.kt_ptr)[i + 1];
      if (nlb > 0 && end - beg > KT_LONG) continue;  // taken by the long-row workgroups
      double y[V];
#pragma unroll
      for (int v = 0; v < V; ++v) y[v] = 0.0;
      spmv_row_part<V, MODE, T>(d, x, pprev, beta, ld, c0, beg, end, 1, y);
      spmv_store<V, MODE, T>(d, q, pout, x, pprev, beta, i, ld, c0, y, pq, cf, k);
    }
  }
  if constexpr (MODE == SP_CHEB0 || MODE == SP_CHEB || MODE == SP_RES) {
    if (MODE == SP_CHEB0 && first_wg && threadIdx.x < (unsigned)nc) red[(k & 255) * ld + threadIdx.x] = 0.0;
    return;
  }
  // p.q (r.z for SP_CHEB_RZ) of the workgroup: shuffles over the rows of each wave, then 4 waves
#pragma unroll
  for (int off = L; off < 64; off <<= 1)
#pragma unroll
    for (int v = 0; v < V; ++v) pq[v] += __shfl_xor(pq[v], off, 64);
  if ((threadIdx.x & 63) < (unsigned)L)
#pragma unroll
    for (int v = 0; v < V; ++v) lds[(threadIdx.x >> 6) * (L * V) + lane * V + v] = col_ok ? pq[v] : 0.0;
  __syncthreads();
  if (threadIdx.x < (unsigned)nc) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) sum += lds[w * (L * V) + threadIdx.x];
    if (part) {
      part[(int64_t)blockIdx.x * nc + threadIdx.x] = sum;  // folded by k_fold_parts
    } else if constexpr (MODE == SP_CHEB_RZ) {
      atomicAdd(red + (k & 15) * ld + threadIdx.x, sum);  // r.z of this instance and column
    } else {
      // iteration of this pass: k (fused), -2 - k (plain pass of a CG iteration), 0 (k = -1: start)
      const int kk = k >= 0 ? k : (k <= -2 ? -2 - k : 0);
      atomicAdd(red + (RED_PQ + kk % 2) * ld + threadIdx.x, sum);  // p.q of this instance and column
    }
    if (FUSE && first_wg) {  // clear what the update pass of this iteration accumulates into
      red[(RED_RZ + (k + 1) % 3) * ld + threadIdx.x] = 0.0;
      red[(RED_RR + k % 2) * ld + threadIdx.x] = 0.0;
    }
  }
}

// dst[c] += sum over the rows workgroups w of part[w][c] (one instance; nc
// divides NT): the per-workgroup sums of an operator pass, added with a few
// hundred atomics where the pass itself would issue one per workgroup and
// column, all on the same nc addresses.
__global__ void __launch_bounds__(NT) k_fold_parts(const double* __restrict__ part, int rows, int nc,
                                                   double* __restrict__ dst) {
  __shared__ double lds[NT];
  const int per = NT / nc;
  const int c = (int)threadIdx.x % nc, g = (int)threadIdx.x / nc;
  double s = 0.0;
  for (int64_t w = (int64_t)blockIdx.x * per + g; w < rows; w += (int64_t)gridDim.x * per) s += part[w * nc + c];
  lds[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < (unsigned)nc) {
    double t = 0.0;
    for (int j = 0; j < per; ++j) t += lds[j * nc + threadIdx.x];
    atomicAdd(dst + threadIdx.x, t);
  }
}

// Workgroups reserved for the long rows when schedule bit 2 or 5 is set:
// about two rows per wave, a multiple of 8 (so the XCD of the sweeping
// workgroups is unchanged).
static int long_row_blocks(const Batch& b) {
  if (b.mx.n_long == 0 || !(b.mx.sched_poi & (4 | 32))) return 0;
  const int64_t nb = std::min<int64_t>((b.mx.n_long + 2 * (NT / 64) - 1) / (2 * (NT / 64)), 2048);
  return (int)((nb + N_XCD - 1) / N_XCD * N_XCD);
}

// Set by the timed operator pass: the end event, recorded right after the pass
// kernel and before its fold, so the event pair spans that kernel alone.
static thread_local hipEvent_t t_pass_end = nullptr;

template <int L, int V, int MODE, class T>
static void launch_spmv_m(const Batch& b, const T* x, const T* pprev, T* pout, int ld, int nc, T* q, double* red,
                          int k, hipStream_t s) {
  // schedule bit 7 with column blocks: the blocks ride along x, bound to XCDs
  // (the kernel takes the column block from the XCD), each block the whole sweep
  const int nbc = ld / nc;
  if ((b.mx.sched_poi & 128) && nbc > 1 && N_XCD % nbc == 0) {
    const int nlb = long_row_blocks(b) * nbc;
    const int sweep = (b.mx.sched_poi & 32) ? xcd_grid(b.mx.n_slices * L, NT / 64, b.mx.grid_poi)
                                            : xcd_grid(b.mx.N, NT / L, b.mx.grid_poi);
    const dim3 g(nlb + sweep * nbc, b.ni, 1);
    if (b.mx.sched_poi & 32)
      hipLaunchKernelGGL((k_spmv_poisson<L, V, MODE, true, T>), g, dim3(NT), 0, s, b.dm, x, pprev, pout, ld, nc, q,
                         nlb, red, k, (double*)nullptr);
    else
      hipLaunchKernelGGL((k_spmv_poisson<L, V, MODE, false, T>), g, dim3(NT), 0, s, b.dm, x, pprev, pout, ld, nc, q,
                         nlb, red, k, (double*)nullptr);
    if (t_pass_end) (void)hipEventRecord(t_pass_end, s);
    return;
  }
  const int nlb = long_row_blocks(b);
  const bool sell = b.mx.sched_poi & 32;
  const int gx = nlb + (sell ? xcd_grid(b.mx.n_slices * L, NT / 64, b.mx.grid_poi) : xcd_grid(b.mx.N, NT / L, b.mx.grid_poi));
  // one instance: per-workgroup sums to the partial buffer, then one fold
  double* part = nullptr;
  if constexpr (MODE == SP_PLAIN || MODE == SP_CG || MODE == SP_CHEB_RZ)
    if (b.spart && b.ni == 1 && nc == ld && NT % nc == 0 && (int64_t)gx * nc <= b.spart_cap) part = b.spart;
  const dim3 g(gx, b.ni, ld / nc);
  if (sell)
    hipLaunchKernelGGL((k_spmv_poisson<L, V, MODE, true, T>), g, dim3(NT), 0, s, b.dm, x, pprev, pout, ld, nc, q,
                       nlb, red, k, part);
  else
    hipLaunchKernelGGL((k_spmv_poisson<L, V, MODE, false, T>), g, dim3(NT), 0, s, b.dm, x, pprev, pout, ld, nc, q,
                       nlb, red, k, part);
  if (t_pass_end) (void)hipEventRecord(t_pass_end, s);
  if (part) {
    const int kk = k >= 0 ? k : (k <= -2 ? -2 - k : 0);
    const int slot = MODE == SP_CHEB_RZ ? (k & 15) : RED_PQ + kk % 2;
    const int fb = (int)std::max<int64_t>(1, std::min<int64_t>(256, (int64_t)gx / (NT / nc * 16)));
    hipLaunchKernelGGL(k_fold_parts, dim3(fb), dim3(NT), 0, s, part, gx, nc, red + (int64_t)slot * ld);
  }
}
template <int L, int V, class T>
static void launch_spmv_t(const Batch& b, const T* x, const T* pprev, T* pout, int ld, int nc, T* q, double* red,
                          int mode, int k, hipStream_t s) {
  switch (mode) {
    case SP_PLAIN: return launch_spmv_m<L, V, SP_PLAIN, T>(b, x, pprev, pout, ld, nc, q, red, k, s);
    case SP_CG:  // the CG direction: double arrays only
      if constexpr (sizeof(T) == sizeof(double)) return launch_spmv_m<L, V, SP_CG, T>(b, x, pprev, pout, ld, nc, q, red, k, s);
      return;
    case SP_CHEB0: return launch_spmv_m<L, V, SP_CHEB0, T>(b, x, pprev, pout, ld, nc, q, red, k, s);
    case SP_CHEB: return launch_spmv_m<L, V, SP_CHEB, T>(b, x, pprev, pout, ld, nc, q, red, k, s);
    case SP_RES: return launch_spmv_m<L, V, SP_RES, T>(b, x, pprev, pout, ld, nc, q, red, k, s);
    default: return launch_spmv_m<L, V, SP_CHEB_RZ, T>(b, x, pprev, pout, ld, nc, q, red, k, s);
  }
}

// q = K x (k < 0: k = -1 at the CG start, -2 - j for the plain pass of iteration j),
// or for CG iteration k >= 0: p_k = D^-1 r + beta_k p_{k-1} formed on the fly from
// x = r and pprev, written to pout, and q = K p_k.
// Schedule bit 1 (column blocking): with 32 or more columns in multiples of 16,
// grid.z runs over blocks of 16 columns, so a row slice is 128 B and the band of
// neighbour rows a sweep touches stays in L2 (the matrix is read once per block).
template <class T>
static void launch_spmv_mode(const Batch& b, const T* x, const T* pprev, T* pout, int ncol, T* q, double* red,
                             int mode, int k, hipStream_t s);
static void launch_spmv_poisson(const Batch& b, const double* x, const double* pprev, double* pout, int ncol,
                                double* q, const PoissonWs& P, int k, hipStream_t s) {
  launch_spmv_mode(b, x, pprev, pout, ncol, q, P.red, k >= 0 ? SP_CG : SP_PLAIN, k, s);
}
template <class T>
static void launch_spmv_mode(const Batch& b, const T* x, const T* pprev, T* pout, int ncol, T* q, double* red,
                             int mode, int k, hipStream_t s) {
  if ((b.mx.sched_poi & 2) && ncol >= 32 && ncol % 16 == 0)
    return launch_spmv_t<4, 4, T>(b, x, pprev, pout, ncol, 16, q, red, mode, k, s);
  if (ncol % 4 == 0 && ncol > 4) {  // 4 columns per lane (two 16-byte loads; one for float)
    if (ncol <= 16) return launch_spmv_t<4, 4, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
    if (ncol <= 32) return launch_spmv_t<8, 4, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
    return launch_spmv_t<16, 4, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
  }
  if (ncol % 2 == 0) {  // column pairs
    if (ncol <= 4) return launch_spmv_t<2, 2, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
    if (ncol <= 8) return launch_spmv_t<4, 2, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
    if (ncol <= 16) return launch_spmv_t<8, 2, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
    if (ncol <= 32) return launch_spmv_t<16, 2, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
    return launch_spmv_t<32, 2, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
  }
  if (ncol <= 1) return launch_spmv_t<1, 1, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
  if (ncol <= 2) return launch_spmv_t<2, 1, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
  if (ncol <= 4) return launch_spmv_t<4, 1, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
  if (ncol <= 8) return launch_spmv_t<8, 1, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
  if (ncol <= 16) return launch_spmv_t<16, 1, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
  if (ncol <= 32) return launch_spmv_t<32, 1, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
  return launch_spmv_t<64, 1, T>(b, x, pprev, pout, ncol, ncol, q, red, mode, k, s);
}

// --------------------------------------------------------------------------
// Jacobi-preconditioned CG, all columns of all instances at once with their
// own alpha and beta.  Scalars sc[i][slot][c] (SC_* in kernels.hpp).
// --------------------------------------------------------------------------
// One CG iteration is two launches.  The operator pass forms the direction
// p_k = D^-1 r_k + beta_k p_{k-1} on the fly for every row it reads (beta_k =
// rz_k / rz_{k-1} from the accumulators), writes p_k to the other direction
// buffer, and accumulates p.q with FP64 atomics per instance and column.  The
// update pass takes alpha_k = rz_k / p.q, updates x and r, and accumulates
// rz_{k+1} and r.r.  The accumulators rotate (rz over three slots, p.q and
// r.r over two), and each pass clears only slots that no workgroup of the
// same launch reads, so no launch overwrites a value its own workgroups use.

// x += alpha p; r -= alpha q; accumulate (r.D^-1 r, r.r).  x over full rows.
__global__ void __launch_bounds__(NT) k_cg_update2(const DevMesh* __restrict__ dm, double* __restrict__ x,
                                                   double* __restrict__ r, const double* __restrict__ p,
                                                   const double* __restrict__ q, int ncol, double* __restrict__ red,
                                                   int k, float* __restrict__ rf, int upd_x) {
  INSTANCE;
  if (d.cg_done && *d.cg_done) return;
  __shared__ double lds[2 * NT];
  x += d.oF * ncol;
  if (rf) rf += d.oE * ncol;
  r += d.oE * ncol;
  p += d.oE * ncol;
  q += d.oE * ncol;
  red += (int64_t)blockIdx.y * RED_SLOTS * ncol;
  const int groups = NT / ncol;
  const int g = threadIdx.x / ncol, c = threadIdx.x - g * ncol;
  const bool act = g < groups;
  const auto* dinv = gbl(d.kdiag_inv);
  double rz = 0.0, rr = 0.0;
  if (act) {
    const double pq = red[(RED_PQ + k % 2) * ncol + c], rz0 = red[(RED_RZ + k % 3) * ncol + c];
    const double al = (pq != 0.0 && rz0 != 0.0) ? rz0 / pq : 0.0;
    for (int64_t kk = (int64_t)blockIdx.x * groups + g; kk < d.N; kk += (int64_t)gridDim.x * groups) {
      const int64_t e = kk * ncol + c;
      if (upd_x) x[e] += al * p[e];   // else deferred to the next direction pass
      const double rn = r[e] - al * q[e];
      r[e] = rn;
      if (rf) rf[e] = (float)rn;  // the finest multigrid level's float copy (Poisson schedule bit 6)
      rz += rn * rn * dinv[kk];
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
    atomicAdd(red + (RED_RZ + (k + 1) % 3) * ncol + threadIdx.x, t);
    atomicAdd(red + (RED_RR + k % 2) * ncol + threadIdx.x, u);
    if (blockIdx.x == 0) red[(RED_PQ + (k + 1) % 2) * ncol + threadIdx.x] = 0.0;  // for the next operator pass
  }
}

// Direction pass for schedules without bit 3: p_k = D^-1 r_k + beta_k p_{k-1}
// into pcur; workgroup 0 clears the slots the update pass of iteration k
// accumulates into (the operator pass does this when it forms p_k itself).
__global__ void __launch_bounds__(NT) k_cg_dir(const DevMesh* __restrict__ dm, const double* __restrict__ r,
                                               const double* __restrict__ pprev, double* __restrict__ pcur, int ncol,
                                               double* __restrict__ red, int k) {
  INSTANCE;
  __shared__ double beta[64];
  const int64_t total = d.N * ncol;
  r += d.oE * ncol;
  pprev += d.oE * ncol;
  pcur += d.oE * ncol;
  red += (int64_t)blockIdx.y * RED_SLOTS * ncol;
  if (threadIdx.x < (unsigned)ncol) {
    double bt = 0.0;
    if (k > 0) {
      const double rzk = red[(RED_RZ + k % 3) * ncol + threadIdx.x], rzp = red[(RED_RZ + (k + 2) % 3) * ncol + threadIdx.x];
      bt = rzp != 0.0 ? rzk / rzp : 0.0;
    }
    beta[threadIdx.x] = bt;
  }
  __syncthreads();
  const auto* dinv = gbl(d.kdiag_inv);
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t kk = e / ncol;
    const int c = (int)(e - kk * ncol);
    const double bt = beta[c];
    pcur[e] = dinv[kk] * r[e] + (bt != 0.0 ? bt * pprev[e] : 0.0);
  }
  if (blockIdx.x == 0 && threadIdx.x < (unsigned)ncol) {
    red[(RED_RZ + (k + 1) % 3) * ncol + threadIdx.x] = 0.0;
    red[(RED_RR + k % 2) * ncol + threadIdx.x] = 0.0;
  }
}

// Initial rz, rr from the start partials (rz_0 into slot RED_RZ, r.r also
// into SC_RR); the other accumulators cleared.
__global__ void __launch_bounds__(NT) k_rz_start(const double* __restrict__ part, int64_t part_stride, int nblk,
                                                 int ncol, double* __restrict__ sc, double* __restrict__ red) {
  __shared__ double lds4[4];
  const int c = blockIdx.x;
  part += blockIdx.y * part_stride;
  sc += (int64_t)blockIdx.y * 8 * ncol;
  red += (int64_t)blockIdx.y * RED_SLOTS * ncol;
  const double s = sum_partials(part, nblk, 2 * ncol, c, lds4);
  const double u = sum_partials(part, nblk, 2 * ncol, ncol + c, lds4);
  if (threadIdx.x == 0) {
    for (int slot = 0; slot < RED_SLOTS; ++slot) red[slot * ncol + c] = 0.0;
    red[RED_RZ * ncol + c] = s;
    sc[SC_RZ * ncol + c] = s;
    sc[SC_RR * ncol + c] = u;
  }
}

// start: r = rhs - q (warm) or rhs (cold, x = 0); partial rz, rr.  x over full rows.
__global__ void __launch_bounds__(NT) k_cg_start2(const DevMesh* __restrict__ dm, double* __restrict__ x,
                                                  double* __restrict__ r, const double* __restrict__ q, int ncol,
                                                  int warm, int64_t part_stride, double* __restrict__ part) {
  INSTANCE;
  __shared__ double lds[2 * NT];
  x += d.oF * ncol;
  r += d.oE * ncol;
  q += d.oE * ncol;
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
      const double di = gbl(d.kdiag_inv)[k];
      rz += rn * rn * di;
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

// Workgroups of the CG start and update passes: about 32 elements per thread,
// at least RED_BLOCKS (small meshes: few partial sums) and at most 2048 (eight
// per compute unit), so the passes over large meshes keep enough loads in flight.
static int cg_blocks(const Batch& b, int ncol) {
  const int64_t want = std::min<int64_t>(std::max<int64_t>(b.mx.N * ncol / (NT * 32), RED_BLOCKS), 2048);
  return nblocks(b.mx.N, NT / ncol, (int)want);
}

// the operator pass with optional event timing on the launch stream
static void cg_apply2(const Batch& b, PoissonWs& P, const double* x, const double* pprev, double* pout, double* q,
                      int k, hipStream_t s) {
  const bool rec = P.ev && P.ev_used + 2 <= P.ev_cap;
  if (rec) {
    (void)hipEventRecord(P.ev[P.ev_used], s);
    t_pass_end = P.ev[P.ev_used + 1];
  }
  launch_spmv_poisson(b, x, pprev, pout, P.ncol, q, P, k, s);
  if (rec) {
    t_pass_end = nullptr;
    P.ev_used += 2;
  }
}

void launch_cg_start(const Batch& b, double* W, double* rhs_r, PoissonWs& P, int warm, hipStream_t s) {
  const int ncol = P.ncol;
  if (warm) {  // q = K x0, x0 = the DoF rows of W (staged in the first direction buffer)
    hipLaunchKernelGGL(k_copy_dofs, dim3(nblocks(b.mx.N * ncol, NT, 8192), b.ni), dim3(NT), 0, s, b.dm, W, P.p, ncol);
    cg_apply2(b, P, P.p, P.p2, P.p2, P.q, -1, s);
  }
  const int nb = cg_blocks(b, ncol);
  hipLaunchKernelGGL(k_cg_start2, dim3(nb, b.ni), dim3(NT), 0, s, b.dm, W, rhs_r, P.q, ncol, warm, P.part_stride,
                     P.part);
  hipLaunchKernelGGL(k_rz_start, dim3(ncol, b.ni), dim3(NT), 0, s, P.part, P.part_stride, nb, ncol, P.sc, P.red);
  P.it = 0;
}

void launch_cg_step(const Batch& b, double* W, PoissonWs& P, hipStream_t s) {
  const int ncol = P.ncol, k = P.it;
  double* pcur = (k % 2) ? P.p2 : P.p;
  double* pprev = (k % 2) ? P.p : P.p2;
  if (b.mx.sched_poi & 8) {
    cg_apply2(b, P, P.r, pprev, pcur, P.q, k, s);  // direction formed inside the operator pass
  } else {
    hipLaunchKernelGGL(k_cg_dir, dim3(nblocks(b.mx.N * ncol, NT, 8192), b.ni), dim3(NT), 0, s, b.dm, P.r, pprev, pcur,
                       ncol, P.red, k);
    cg_apply2(b, P, pcur, pprev, pcur, P.q, -2 - k, s);  // plain operator pass of iteration k
  }
  const int nb = cg_blocks(b, ncol);
  hipLaunchKernelGGL(k_cg_update2, dim3(nb, b.ni), dim3(NT), 0, s, b.dm, W, P.r, pcur, P.q, ncol, P.red, k,
                     (float*)nullptr, 1);
  P.it = k + 1;
}

// Chebyshev smoothing on the finest multigrid level fused into the operator
// pass (the spmv_store comment gives the updates): the first two steps from
// zero (z, d from r), and one further step from zin into zout.
// t = r - K z on the finest level (the residual the restriction reads)
void launch_mg_resid(const Batch& b, const double* z, const double* r, double* t, int ncol, double* red_scratch,
                     hipStream_t s) {
  launch_spmv_mode(b, z, r, t, ncol, t, red_scratch, SP_RES, -1, s);
}
void launch_mg_resid_f(const Batch& b, const float* z, const float* r, float* t, int ncol, double* red_scratch,
                       hipStream_t s) {
  launch_spmv_mode<float>(b, z, r, t, ncol, t, red_scratch, SP_RES, -1, s);
}
void launch_mg_cheb0(const Batch& b, const double* r, double* z, double* d, double* red, int rz_slot, int ncol,
                     hipStream_t s) {
  launch_spmv_mode(b, r, r, z, ncol, d, red, SP_CHEB0, rz_slot, s);
}
void launch_mg_cheb_step(const Batch& b, const double* zin, const double* r, double* zout, double* d, double* red,
                         int ncol, int k, int rz_slot, hipStream_t s) {
  if (rz_slot >= 0) launch_spmv_mode(b, zin, r, zout, ncol, d, red, SP_CHEB_RZ, rz_slot | (k << 4), s);
  else launch_spmv_mode(b, zin, r, zout, ncol, d, red, SP_CHEB, k, s);
}

// The same finest-level passes on float storage (Poisson schedule bit 6):
// operand, residual copy, corrections and directions in float, sums in
// double.  These passes are not event-timed (the timing slot holds the
// double passes of the CG itself).
void launch_mg_cheb0_f(const Batch& b, const float* r, float* z, float* d, double* red, int rz_slot, int ncol,
                       hipStream_t s) {
  launch_spmv_mode<float>(b, r, r, z, ncol, d, red, SP_CHEB0, rz_slot, s);
}
void launch_mg_cheb_step_f(const Batch& b, const float* zin, const float* r, float* zout, float* d, double* red,
                           int ncol, int k, int rz_slot, hipStream_t s) {
  if (rz_slot >= 0) launch_spmv_mode<float>(b, zin, r, zout, ncol, d, red, SP_CHEB_RZ, rz_slot | (k << 4), s);
  else launch_spmv_mode<float>(b, zin, r, zout, ncol, d, red, SP_CHEB, k, s);
}

// The plain operator pass of CG iteration k on the direction p (q = K p, p.q
// accumulated for the update pass), and the update pass itself.
void launch_cg_apply_plain(const Batch& b, PoissonWs& P, const double* p, int k, hipStream_t s) {
  cg_apply2(b, P, p, p, const_cast<double*>(p), P.q, -2 - k, s);
}
// Convergence flags of a batch's multigrid CG (the host test of the same
// solve, on the device): after the update pass of iteration k an instance is
// done once every column's r.r is at most rtol^2 times its largest column's
// b.b.  Its r.r is then copied into the other r.r slot as well, so the final
// test reads a converged value whichever iteration the solve stops after,
// and its later CG and multigrid launches return at once.  One wave per
// instance (ncol <= 64).
__global__ void k_cg_done(const DevMesh* __restrict__ dm, const double* __restrict__ sc, double* __restrict__ red,
                          int ncol, int k, double rtol2) {
  INSTANCE;
  if (!d.cg_done || *d.cg_done) return;
  sc += (int64_t)blockIdx.y * 8 * ncol;
  red += (int64_t)blockIdx.y * RED_SLOTS * ncol;
  const int c = threadIdx.x;
  double bb = c < ncol ? sc[SC_BB * ncol + c] : 0.0;
  for (int off = 32; off > 0; off >>= 1) bb = fmax(bb, __shfl_xor(bb, off, 64));
  const double rr = c < ncol ? red[(RED_RR + k % 2) * ncol + c] : 0.0;
  const bool ok = c >= ncol || rr <= rtol2 * bb;
  if (__all(ok)) {
    if (c < ncol) red[(RED_RR + (k + 1) % 2) * ncol + c] = rr;
    if (c == 0) *const_cast<int*>(d.cg_done) = 1;
  }
}
void launch_cg_done(const Batch& b, const PoissonWs& P, int k, double rtol, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_done, dim3(1, b.ni), dim3(64), 0, s, b.dm, P.sc, P.red, P.ncol, k, rtol * rtol);
}
__global__ void k_zero_int(int* __restrict__ x, int n) {
  for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) x[i] = 0;
}
void launch_zero_int(int* x, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_zero_int, dim3(nblocks(n)), dim3(NT), 0, s, x, n);
}

void launch_cg_update(const Batch& b, double* W, PoissonWs& P, const double* p, int k, hipStream_t s, float* rf,
                      int upd_x) {
  const int nb = cg_blocks(b, P.ncol);
  hipLaunchKernelGGL(k_cg_update2, dim3(nb, b.ni), dim3(NT), 0, s, b.dm, W, P.r, p, P.q, P.ncol, P.red, k, rf, upd_x);
}

__global__ void __launch_bounds__(NT) k_to_float(const double* __restrict__ x, float* __restrict__ y, int64_t nd) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nd; i += (int64_t)gridDim.x * NT) y[i] = (float)x[i];
}
void launch_to_float(const double* x, float* y, int64_t nd, hipStream_t s) {
  if (nd > 0) hipLaunchKernelGGL(k_to_float, dim3(nblocks(nd, NT, 8192)), dim3(NT), 0, s, x, y, nd);
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
