// Kernels of the reverse sweep of the dipole record (exact discrete adjoint
// of one real-time step of the coupled orbital / CI equations, Sec. II Eqs.
// ci_eom and orb_eom with the frozen operator of Sec. III.B; one instance,
// at most 4 orbitals).  The orchestration is in api.hip.
//
// Conventions: a sensitivity K_Y of a complex quantity Y means
// dJ = Re sum K_Y dY; orbital adjoints nu are M-weighted, dJ = Re <nu, dc>_M.
// Orbital arrays complex [NE][n], Poisson column arrays real [rows][ncol]
// (pair r <= s: Re and, for r < s, Im of W_rs), small matrices row-major.
#include <hip/hip_runtime.h>

#include <cmath>

#include "adjoint.hpp"
#include "devutil.hpp"

namespace mh {

#define INSTANCE const DevMesh& d = dm[blockIdx.y]
constexpr int AN = 4;  // largest orbital count of the adjoint

// out = beta out + in X  (per row: out_q = sum_p in_p X[p][q])
__global__ void __launch_bounds__(NT) k_mix(const DevMesh* __restrict__ dm, const double2* __restrict__ in,
                                            const double2* __restrict__ X, double beta, double2* __restrict__ out) {
  INSTANCE;
  const int n = d.n;
  in += d.oE * n;
  out += d.oE * n;
  X += (int64_t)blockIdx.y * n * n;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < d.NE; i += (int64_t)gridDim.x * NT) {
    double2 row[AN], res[AN];
    for (int p = 0; p < n; ++p) row[p] = in[i * n + p];
    for (int q = 0; q < n; ++q) {
      double2 s = beta != 0.0 ? cscale(beta, out[i * n + q]) : make_double2(0.0, 0.0);
      for (int p = 0; p < n; ++p) s = cadd(s, cmul(row[p], X[p * n + q]));
      res[q] = s;
    }
    for (int q = 0; q < n; ++q) out[i * n + q] = res[q];
  }
}
void launch_mix(const Batch& b, const double* in, const double* X, double beta, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mix, dim3(nblocks(b.mx.NE, NT, 4096), b.ni), dim3(NT), 0, s, b.dm, (const double2*)in,
                     (const double2*)X, beta, (double2*)out);
}

// Q[i][p][q] += omega m_i conj(A_ip) B_iq
__global__ void __launch_bounds__(NT) k_q_accum(const DevMesh* __restrict__ dm, const double2* __restrict__ A,
                                                const double2* __restrict__ B, double wr, double wi,
                                                double2* __restrict__ Q) {
  INSTANCE;
  const int n = d.n, nn = n * n;
  A += d.oE * n;
  B += d.oE * n;
  Q += d.oE * nn;
  const double2 w = make_double2(wr, wi);
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < d.NE; i += (int64_t)gridDim.x * NT) {
    const double2 wm = cscale(d.m[i], w);
    double2 a[AN], bv[AN];
    for (int p = 0; p < n; ++p) {
      a[p] = A[i * n + p];
      bv[p] = B[i * n + p];
    }
    for (int p = 0; p < n; ++p) {
      const double2 wa = cmul(wm, make_double2(a[p].x, -a[p].y));
      for (int q = 0; q < n; ++q) Q[i * nn + p * n + q] = cadd(Q[i * nn + p * n + q], cmul(wa, bv[q]));
    }
  }
}
void launch_q_accum(const Batch& b, const double* A, const double* B, double wr, double wi, double* Q,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_q_accum, dim3(nblocks(b.mx.NE, NT, 4096), b.ni), dim3(NT), 0, s, b.dm, (const double2*)A,
                     (const double2*)B, wr, wi, (double2*)Q);
}

// W_rs (every ordered pair) of one node from its real columns.
__device__ __forceinline__ void node_pairs(const double* wrow, const int* colmap, int n, double2* Wc) {
  for (int r = 0; r < n; ++r)
    for (int s = r; s < n; ++s) {
      const int c0 = colmap[r * n + s];
      if (r == s) {
        Wc[r * n + r] = make_double2(wrow[c0], 0.0);
      } else {
        Wc[r * n + s] = make_double2(wrow[c0], wrow[c0 + 1]);
        Wc[s * n + r] = make_double2(wrow[c0], -wrow[c0 + 1]);
      }
    }
}

// Complex sensitivities K[r][s] of the ordered pair potentials -> real columns
// (W_sr = conj W_rs): K_Re += Re(K_rs + K_sr), K_Im += Im(K_sr - K_rs).
__device__ __forceinline__ void pairs_to_cols(const double2* K, const int* colmap, int n, double* out) {
  for (int r = 0; r < n; ++r)
    for (int s = r; s < n; ++s) {
      const int c0 = colmap[r * n + s];
      if (r == s) {
        out[c0] += K[r * n + r].x;
      } else {
        out[c0] += K[r * n + s].x + K[s * n + r].x;
        out[c0 + 1] += K[s * n + r].y - K[r * n + s].y;
      }
    }
}

// Per node: the mean-field sensitivity Q (of V = gamma^-1 U) and the
// two-electron integral sensitivity Kg turned into sensitivities of the pair
// potential columns (Kw, rows < NE) and of the orbital values (Phib, the
// conjugated sensitivity of phi at the node, Kg part only).
//   K_U = ginv^T Q,  K_Upacked -> Kw = Mr^T K_Upacked,
//   K_W[r][s] += m sum_pq Kg[pqrs] conj(phi_p) phi_q,
//   Phib_p = m sum_qrs Kg[pqrs] phi_q W_rs + m sum_ars conj(Kg[a p r s]) phi_a conj(W_rs).
__global__ void __launch_bounds__(NT) k_adj_mf(const DevMesh* __restrict__ dm, const double2* __restrict__ Q,
                                               const double* __restrict__ W, const double2* __restrict__ phi,
                                               const double2* __restrict__ ginv, const double* __restrict__ Mr,
                                               const double2* __restrict__ Kg, const int* __restrict__ colmap,
                                               double* __restrict__ Kw, double2* __restrict__ Phib) {
  INSTANCE;
  const int n = d.n, nn = n * n;
  __shared__ double sMr[AN * AN * AN * AN];
  __shared__ double2 sKg[AN * AN * AN * AN];
  __shared__ double2 sG[AN * AN];
  __shared__ int sCm[AN * AN];
  for (int e = threadIdx.x; e < nn * nn; e += NT) {
    sMr[e] = Mr[(int64_t)blockIdx.y * nn * nn + e];
    sKg[e] = Kg[(int64_t)blockIdx.y * nn * nn + e];
  }
  for (int e = threadIdx.x; e < nn; e += NT) {
    sG[e] = ginv[(int64_t)blockIdx.y * nn + e];
    sCm[e] = colmap[e];
  }
  __syncthreads();
  Q += d.oE * nn;
  W += d.oF * nn;
  Kw += d.oF * nn;
  phi += d.oE * n;
  Phib += d.oE * n;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < d.NE; i += (int64_t)gridDim.x * NT) {
    const double mi = d.m[i];
    double2 q[AN * AN], ph[AN], Wc[AN * AN];
    double wrow[AN * AN], kw[AN * AN];
    for (int e = 0; e < nn; ++e) {
      q[e] = Q[i * nn + e];
      wrow[e] = W[i * nn + e];
      kw[e] = 0.0;
    }
    for (int p = 0; p < n; ++p) ph[p] = phi[i * n + p];
    node_pairs(wrow, sCm, n, Wc);
    // K_U[o][q] = sum_p ginv[p][o] Q[p][q]; packed: [o][o] Re, [o][q] Re(K_oq + K_qo), [q][o] Im(K_qo - K_oq)
    double2 ku[AN * AN];
    for (int o = 0; o < n; ++o)
      for (int qq = 0; qq < n; ++qq) {
        double2 s = make_double2(0.0, 0.0);
        for (int p = 0; p < n; ++p) s = cadd(s, cmul(sG[p * n + o], q[p * n + qq]));
        ku[o * n + qq] = s;
      }
    double kup[AN * AN];
    for (int o = 0; o < n; ++o) {
      kup[o * n + o] = ku[o * n + o].x;
      for (int qq = o + 1; qq < n; ++qq) {
        kup[o * n + qq] = ku[o * n + qq].x + ku[qq * n + o].x;
        kup[qq * n + o] = ku[qq * n + o].y - ku[o * n + qq].y;
      }
    }
    for (int c = 0; c < nn; ++c) {
      double s = 0.0;
      for (int o = 0; o < nn; ++o) s += sMr[o * nn + c] * kup[o];
      kw[c] = s;
    }
    // two-electron integral part
    double2 kwg[AN * AN];
    for (int rs = 0; rs < nn; ++rs) {
      double2 s = make_double2(0.0, 0.0);
      for (int p = 0; p < n; ++p)
        for (int qq = 0; qq < n; ++qq) s = cadd(s, cmul(sKg[(p * n + qq) * nn + rs], cjmul(ph[p], ph[qq])));
      kwg[rs] = cscale(mi, s);
    }
    pairs_to_cols(kwg, sCm, n, kw);
    for (int c = 0; c < nn; ++c) Kw[i * nn + c] = kw[c];
    for (int p = 0; p < n; ++p) {
      double2 s = make_double2(0.0, 0.0);
      for (int qq = 0; qq < n; ++qq)
        for (int rs = 0; rs < nn; ++rs) s = cadd(s, cmul(sKg[(p * n + qq) * nn + rs], cmul(ph[qq], Wc[rs])));
      for (int a = 0; a < n; ++a)
        for (int rs = 0; rs < nn; ++rs) {
          const double2 k = sKg[(a * n + p) * nn + rs];
          // conj(k) phi_a conj(W_rs) = conj(k W_rs) phi_a
          const double2 kwv = cmul(k, Wc[rs]);
          s = cadd(s, cmul(make_double2(kwv.x, -kwv.y), ph[a]));
        }
      Phib[i * n + p] = cscale(mi, s);
    }
  }
}
void launch_adj_mf(const Batch& b, const double* Q, const double* W, const double* phi, const double* ginv,
                   const double* Mr, const double* Kg, const int* colmap, double* Kw, double* Phib, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_mf, dim3(nblocks(b.mx.NE, NT, 4096), b.ni), dim3(NT), 0, s, b.dm, (const double2*)Q, W,
                     (const double2*)phi, (const double2*)ginv, Mr, (const double2*)Kg, colmap, Kw, (double2*)Phib);
}

// G2[a][j] = sum_{i < NE} Q[i][a] W[i][j] (a, j < n^2): block partials, then
// one workgroup per output.
constexpr int QW_BLOCKS = 256;
__global__ void __launch_bounds__(NT) k_qw_gram(const DevMesh* __restrict__ dm, const double2* __restrict__ Q,
                                                const double* __restrict__ W, double* __restrict__ part) {
  INSTANCE;
  const int nn = d.n * d.n, nout = nn * nn;
  Q += d.oE * nn;
  W += d.oF * nn;
  const int o = threadIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  if (o < nout) {
    const int a = o / nn, j = o - a * nn;
    for (int64_t i = blockIdx.x; i < d.NE; i += gridDim.x) acc = cadd(acc, cscale(W[i * nn + j], Q[i * nn + a]));
  }
  double* pb = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 2 * nout;
  if (o < nout) {
    pb[2 * o] = acc.x;
    pb[2 * o + 1] = acc.y;
  }
}
__global__ void __launch_bounds__(NT) k_cpart_finish(const double* __restrict__ part, int nblk, int nout,
                                                     double* __restrict__ out) {
  __shared__ double lds4[4];
  part += (int64_t)blockIdx.y * nblk * 2 * nout;
  const int o = blockIdx.x;
  const double re = sum_partials(part, nblk, 2 * nout, 2 * o, lds4);
  const double im = sum_partials(part, nblk, 2 * nout, 2 * o + 1, lds4);
  if (threadIdx.x == 0) {
    out[((int64_t)blockIdx.y * nout + o) * 2] = re;
    out[((int64_t)blockIdx.y * nout + o) * 2 + 1] = im;
  }
}
void launch_qw_gram(const Batch& b, const double* Q, const double* W, double* part, double* G2, hipStream_t s) {
  const int nn = b.mx.n * b.mx.n;
  hipLaunchKernelGGL(k_qw_gram, dim3(QW_BLOCKS, b.ni), dim3(NT), 0, s, b.dm, (const double2*)Q, W, part);
  hipLaunchKernelGGL(k_cpart_finish, dim3(nn * nn, b.ni), dim3(NT), 0, s, part, QW_BLOCKS, nn * nn, G2);
}
int64_t qw_part_doubles(const Batch& b) { return (int64_t)b.ni * QW_BLOCKS * 2 * (int64_t)b.mx.n * b.mx.n * b.mx.n * b.mx.n; }

// ------------------------------------------------------------------------
// Small per-instance work on one thread (n <= 4).  Small block layout
// (complex, n^2 each unless noted): see AdjSmall in adjoint.hpp.
// ------------------------------------------------------------------------
__device__ void cinv(const double2* A, int n, double2* out) {
  double2 a[AN * AN], b[AN * AN];
  for (int i = 0; i < n * n; ++i) {
    a[i] = A[i];
    b[i] = make_double2((i / n) == (i % n) ? 1.0 : 0.0, 0.0);
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = hypot(a[c * n + c].x, a[c * n + c].y);
    for (int r = c + 1; r < n; ++r) {
      const double v = hypot(a[r * n + c].x, a[r * n + c].y);
      if (v > best) { best = v; piv = r; }
    }
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        double2 t = a[c * n + k]; a[c * n + k] = a[piv * n + k]; a[piv * n + k] = t;
        t = b[c * n + k]; b[c * n + k] = b[piv * n + k]; b[piv * n + k] = t;
      }
    const double2 d = a[c * n + c];
    const double dd = d.x * d.x + d.y * d.y;
    const double2 inv = make_double2(d.x / dd, -d.y / dd);
    for (int k = 0; k < n; ++k) {
      a[c * n + k] = cmul(a[c * n + k], inv);
      b[c * n + k] = cmul(b[c * n + k], inv);
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double2 f = a[r * n + c];
      for (int k = 0; k < n; ++k) {
        a[r * n + k] = csub(a[r * n + k], cmul(f, a[c * n + k]));
        b[r * n + k] = csub(b[r * n + k], cmul(f, b[c * n + k]));
      }
    }
  }
  for (int i = 0; i < n * n; ++i) out[i] = b[i];
}

__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// gr = inverse of the regularised gamma^-1; Xg = ginv^T; Xr = gr^T;
// lam2 = gr^T lam^H ginv^T (the mixing of the adjoint operator conjugated by gr^T).
__global__ void k_adj_prep(const double2* __restrict__ ginv, const double2* __restrict__ lam, int n,
                           double2* __restrict__ sm) {
  if (threadIdx.x != 0) return;
  const int nn = n * n;
  double2 gr[AN * AN], t[AN * AN];
  cinv(ginv, n, gr);
  double2* Xg = sm + ADJ_XG * nn;
  double2* Xr = sm + ADJ_XR * nn;
  double2* L2 = sm + ADJ_LAM2 * nn;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      Xg[a * n + b] = ginv[b * n + a];
      Xr[a * n + b] = gr[b * n + a];
    }
  for (int a = 0; a < n; ++a)  // t = gr^T lam^H
    for (int b = 0; b < n; ++b) {
      double2 s = make_double2(0.0, 0.0);
      for (int k = 0; k < n; ++k) s = cadd(s, cmul(gr[k * n + a], cconj(lam[b * n + k])));
      t[a * n + b] = s;
    }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double2 s = make_double2(0.0, 0.0);
      for (int k = 0; k < n; ++k) s = cadd(s, cmul(t[a * n + k], ginv[b * n + k]));
      L2[a * n + b] = s;
    }
}

// One Frechet quadrature node of the orbital exponential: ebar += Re(w tr Gz),
// Lbar[q][p] -= w Sm[p][q].
__global__ void k_adj_quad(const double2* __restrict__ Gz, const double2* __restrict__ Sm, double wr, double wi,
                           int n, double* __restrict__ ebar, double2* __restrict__ sm) {
  if (threadIdx.x != 0) return;
  const double2 w = make_double2(wr, wi);
  double2 tr = make_double2(0.0, 0.0);
  for (int p = 0; p < n; ++p) tr = cadd(tr, Gz[p * n + p]);
  ebar[0] += cmul(w, tr).x;
  double2* Lb = sm + ADJ_LBAR * n * n;
  for (int q = 0; q < n; ++q)
    for (int p = 0; p < n; ++p) Lb[q * n + p] = csub(Lb[q * n + p], cmul(w, Sm[p * n + q]));
}

// Field and mixing terms of the lambda, h and dipole sensitivities:
// ebar += Re sum Lbar_qp z_qp + Re sum Kh_pq z_pq; XL1 = Lbar^T, XL2 = conj(Lbar),
// Xh = Kh^T + conj(Kh), Xd = 2 g gamma^T; Kgam += g z.
__global__ void k_adj_terms(const double2* __restrict__ z, const double2* __restrict__ gam, double g, int n,
                            double* __restrict__ ebar, double2* __restrict__ sm) {
  if (threadIdx.x != 0) return;
  const int nn = n * n;
  const double2* Lb = sm + ADJ_LBAR * nn;
  const double2* Kh = sm + ADJ_KH * nn;
  double e = 0.0;
  for (int i = 0; i < nn; ++i) e += cmul(Lb[i], z[i]).x + cmul(Kh[i], z[i]).x;
  ebar[0] += e;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      sm[ADJ_XL1 * nn + a * n + b] = Lb[b * n + a];
      sm[ADJ_XL2 * nn + a * n + b] = cconj(Lb[a * n + b]);
      sm[ADJ_XH * nn + a * n + b] = cadd(Kh[b * n + a], cconj(Kh[a * n + b]));
      sm[ADJ_XD * nn + a * n + b] = cscale(2.0 * g, gam[b * n + a]);
      sm[ADJ_KGAM * nn + a * n + b] = cadd(sm[ADJ_KGAM * nn + a * n + b], cscale(g, z[a * n + b]));
    }
}

// From G2 = sum_x Q(x) W(x)^T: the sensitivities of ginv (pushed to gamma:
// Kgam -= ginv^T K_ginv ginv^T) and of the column map Mr (pushed to Gamma,
// the adjoint of the Mr construction from Gamma).
__global__ void k_adj_mf_small(const double2* __restrict__ G2, const double* __restrict__ Mr,
                               const double2* __restrict__ ginv, const int* __restrict__ colmap, int n,
                               double2* __restrict__ sm, double2* __restrict__ KGam) {
  if (threadIdx.x != 0) return;
  const int nn = n * n;
  // U_oq = sum_j Uc[oq][j] W_j (W_j real columns), from the packed rows of Mr
  auto Uc = [&](int o, int q, int j) -> double2 {
    if (o == q) return make_double2(Mr[(o * n + o) * nn + j], 0.0);
    if (o < q) return make_double2(Mr[(o * n + q) * nn + j], Mr[(q * n + o) * nn + j]);
    return make_double2(Mr[(q * n + o) * nn + j], -Mr[(o * n + q) * nn + j]);
  };
  double2 Kgi[AN * AN];
  for (int p = 0; p < n; ++p)
    for (int o = 0; o < n; ++o) {
      double2 s = make_double2(0.0, 0.0);
      for (int q = 0; q < n; ++q)
        for (int j = 0; j < nn; ++j) s = cadd(s, cmul(Uc(o, q, j), G2[(p * n + q) * nn + j]));
      Kgi[p * n + o] = s;
    }
  double2* Kgam = sm + ADJ_KGAM * nn;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double2 s = make_double2(0.0, 0.0);
      for (int p = 0; p < n; ++p)
        for (int o = 0; o < n; ++o) s = cadd(s, cmul(cmul(ginv[p * n + a], Kgi[p * n + o]), ginv[b * n + o]));
      Kgam[a * n + b] = csub(Kgam[a * n + b], s);
    }
  for (int e = 0; e < nn * nn; ++e) KGam[e] = make_double2(0.0, 0.0);
  for (int j = 0; j < nn; ++j) {
    // K_U^(j) = ginv^T G2[:, j] (as n x n), then packed like U
    double2 ku[AN * AN];
    for (int o = 0; o < n; ++o)
      for (int q = 0; q < n; ++q) {
        double2 s = make_double2(0.0, 0.0);
        for (int p = 0; p < n; ++p) s = cadd(s, cmul(ginv[p * n + o], G2[(p * n + q) * nn + j]));
        ku[o * n + q] = s;
      }
    for (int out = 0; out < nn; ++out) {
      const int oi = out / n, qi = out - oi * n;
      double kmr;
      if (oi == qi) kmr = ku[oi * n + oi].x;
      else if (oi < qi) kmr = ku[oi * n + qi].x + ku[qi * n + oi].x;
      else kmr = ku[oi * n + qi].y - ku[qi * n + oi].y;
      // Mr[out][j] = Re(phase coef): coef from Gamma entries g1, g2 of column j's pair
      const int ro = oi < qi ? oi : qi, co = oi < qi ? qi : oi;
      const bool want_im = oi > qi;
      int rr = 0, ss = 0, part = 0;
      for (int r = 0; r < n; ++r)
        for (int s = r; s < n; ++s) {
          const int c0 = colmap[r * n + s];
          if (c0 == j) { rr = r; ss = s; part = 0; }
          if (r != s && c0 + 1 == j) { rr = r; ss = s; part = 1; }
        }
      const double2 ph = want_im ? make_double2(0.0, -1.0) : make_double2(1.0, 0.0);
      const double2 k = cscale(kmr, ph);
      const int i1 = ((ro * n + co) * n + rr) * n + ss, i2 = ((ro * n + co) * n + ss) * n + rr;
      if (rr == ss) {
        KGam[i1] = cadd(KGam[i1], k);
      } else if (part == 0) {
        KGam[i1] = cadd(KGam[i1], k);
        KGam[i2] = cadd(KGam[i2], k);
      } else {
        const double2 ik = make_double2(-k.y, k.x);  // i k
        KGam[i1] = cadd(KGam[i1], ik);
        KGam[i2] = csub(KGam[i2], ik);
      }
    }
  }
}

// CI sensitivities of the RDMs as an operator on the CI vector:
// h = Kgam + Kgam^H, g = 2 (KGam[pqrs] + conj(KGam[srqp])).
__global__ void k_adj_ciprep(const double2* __restrict__ sm, const double2* __restrict__ KGam, int n,
                             double2* __restrict__ h, double2* __restrict__ g) {
  if (threadIdx.x != 0) return;
  const int nn = n * n;
  const double2* Kgam = sm + ADJ_KGAM * nn;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) h[a * n + b] = cadd(Kgam[a * n + b], cconj(Kgam[b * n + a]));
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      for (int r = 0; r < n; ++r)
        for (int s = 0; s < n; ++s)
          g[((p * n + q) * n + r) * n + s] =
              cscale(2.0, cadd(KGam[((p * n + q) * n + r) * n + s], cconj(KGam[((s * n + r) * n + q) * n + p])));
}

// y += (wr + i wi) x over cnt complex values
__global__ void k_caxpy(int64_t cnt, double wr, double wi, const double2* __restrict__ x, double2* __restrict__ y) {
  const double2 w = make_double2(wr, wi);
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * NT)
    y[i] = cadd(y[i], cmul(w, x[i]));
}
void launch_caxpy(int64_t cnt, double wr, double wi, const double* x, double* y, hipStream_t s) {
  if (cnt > 0)
    hipLaunchKernelGGL(k_caxpy, dim3(nblocks(cnt, NT, 4096)), dim3(NT), 0, s, cnt, wr, wi, (const double2*)x,
                       (double2*)y);
}

void launch_adj_prep(const double* ginv, const double* lam, int n, double* sm, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_prep, dim3(1), dim3(64), 0, s, (const double2*)ginv, (const double2*)lam, n,
                     (double2*)sm);
}
void launch_adj_quad(const double* Gz, const double* Sm, double wr, double wi, int n, double* ebar, double* sm,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_adj_quad, dim3(1), dim3(64), 0, s, (const double2*)Gz, (const double2*)Sm, wr, wi, n, ebar,
                     (double2*)sm);
}
void launch_adj_terms(const double* z, const double* gam, double g, int n, double* ebar, double* sm, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_terms, dim3(1), dim3(64), 0, s, (const double2*)z, (const double2*)gam, g, n, ebar,
                     (double2*)sm);
}
void launch_adj_mf_small(const double* G2, const double* Mr, const double* ginv, const int* colmap, int n,
                         double* sm, double* KGam, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_mf_small, dim3(1), dim3(64), 0, s, (const double2*)G2, Mr, (const double2*)ginv, colmap,
                     n, (double2*)sm, (double2*)KGam);
}
void launch_adj_ciprep(const double* sm, const double* KGam, int n, double* h, double* g, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_ciprep, dim3(1), dim3(64), 0, s, (const double2*)sm, (const double2*)KGam, n,
                     (double2*)h, (double2*)g);
}

// ------------------------------------------------------------------------
// Adjoint of the pair Poisson solves.  Forward: W = C w + CB W_B with
// K w = 4 pi C^T (m rho) - C^T K_full CB W_B and W_B = table (sum_i m_i rho_i R(x_i)).
// Reverse, for a column sensitivity Kw: z = K^-1 C^T Kw (a CG solve with this
// right-hand side), then
//   K_rho = 4 pi m (C z) + m R(x) table^T [CB^T Kw - CB^T K_full C z].
// ------------------------------------------------------------------------
// y = C^T Kw on the DoF rows (Kw over full rows, y over extended rows)
__global__ void __launch_bounds__(NT) k_ctrans_real(const DevMesh* __restrict__ dm, const double* __restrict__ Kw,
                                                    int ncol, double* __restrict__ y) {
  INSTANCE;
  Kw += d.oF * ncol;
  y += d.oE * ncol;
  const int64_t total = d.N * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t k = e / ncol;
    const int c = (int)(e - k * ncol);
    double f = Kw[k * ncol + c];
    const int mi = d.ma_index[k];
    if (mi >= 0)
      for (int t = d.ct_ptr[mi]; t < d.ct_ptr[mi + 1]; ++t) f += d.ct_w[t] * Kw[(int64_t)d.ct_row[t] * ncol + c];
    y[k * ncol + c] = f;
  }
}
// sc[SC_BB][c] = sum over DoF rows of y^2, one workgroup per (column, instance)
__global__ void __launch_bounds__(NT) k_colsq(const DevMesh* __restrict__ dm, const double* __restrict__ y, int ncol,
                                              double* __restrict__ sc) {
  INSTANCE;
  __shared__ double lds4[4];
  y += d.oE * ncol;
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < d.N; k += NT) s += y[k * ncol + c] * y[k * ncol + c];
  s = block_sum_all(s, lds4);
  if (threadIdx.x == 0) sc[(int64_t)blockIdx.y * 8 * ncol + SC_BB * ncol + c] = s;
}
void launch_adj_poisson_rhs(const Batch& b, const double* Kw, int ncol, double* y, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrans_real, dim3(nblocks(b.mx.N * ncol, NT, 8192), b.ni), dim3(NT), 0, s, b.dm, Kw, ncol, y);
  hipLaunchKernelGGL(k_colsq, dim3(ncol, b.ni), dim3(NT), 0, s, b.dm, y, ncol, sc);
}

// tb[b] += CB^T Kw: hanging rows with boundary masters pass their share on
__global__ void __launch_bounds__(NT) k_cbT(const DevMesh* __restrict__ dm, const double* __restrict__ Kw, int ncol,
                                            double* __restrict__ tb) {
  INSTANCE;
  Kw += d.oF * ncol;
  const int64_t total = d.Nh * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t h = e / ncol;
    const int c = (int)(e - h * ncol);
    const double v = Kw[(d.N + h) * ncol + c];
    for (int t = d.hang_ptr[h]; t < d.hang_ptr[h + 1]; ++t) {
      const int col = d.hang_col[t];
      if (col >= d.NE) atomicAdd(tb + (int64_t)(col - d.NE) * ncol + c, d.hang_w[t] * v);
    }
  }
}

// tb[b] -= CB^T K_full u over the boundary cells (u = C z over full rows with
// zero boundary rows): the transpose of the boundary lift of the forward solve.
template <int P>
__global__ void __launch_bounds__(NT) k_liftT(const DevMesh* __restrict__ dm, const double* __restrict__ u, int ncol,
                                              double* __restrict__ tb) {
  INSTANCE;
  constexpr int P3 = P * P * P;
  __shared__ double sx[P3 * 16];
  __shared__ int snode[P3];
  u += d.oF * ncol;
  for (int64_t cb = blockIdx.x; cb < d.n_bnd_cells; cb += gridDim.x) {
    const int64_t e = d.bnd_cells[cb];
    __syncthreads();
    for (int t = threadIdx.x; t < P3; t += NT) snode[t] = d.cell_nodes[e * P3 + t];
    __syncthreads();
    for (int idx = threadIdx.x; idx < P3 * ncol; idx += NT) {
      const int t = idx / ncol, c = idx - t * ncol;
      const int node = snode[t];
      sx[c * P3 + t] = node < d.NE ? u[(int64_t)node * ncol + c] : 0.0;
    }
    __syncthreads();
    const double hh = d.cell_hh[e];
    for (int idx = threadIdx.x; idx < P3 * ncol; idx += NT) {
      const int t = idx / ncol, c = idx - t * ncol;
      const int node = snode[t];
      if (node < d.N) continue;
      const int a = t % P, b = (t / P) % P, cc = t / (P * P);
      const double* xo = sx + c * P3;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        s0 += d.A[a * P + q] * xo[(cc * P + b) * P + q];
        s1 += d.A[b * P + q] * xo[(cc * P + q) * P + a];
        s2 += d.A[cc * P + q] * xo[(q * P + b) * P + a];
      }
      const double y = hh * (d.w[b] * d.w[cc] * s0 + d.w[a] * d.w[cc] * s1 + d.w[a] * d.w[b] * s2);
      if (node >= d.NE) {
        atomicAdd(tb + (int64_t)(node - d.NE) * ncol + c, -y);
      } else {
        const int64_t h = node - d.N;
        for (int k = d.hang_ptr[h]; k < d.hang_ptr[h + 1]; ++k)
          if (d.hang_col[k] >= d.NE) atomicAdd(tb + (int64_t)(d.hang_col[k] - d.NE) * ncol + c, -d.hang_w[k] * y);
      }
    }
  }
}

// qlm[t][c] = sum_b table[b][t] tb[b][c]; one workgroup per (term, column)
__global__ void __launch_bounds__(NT) k_qlm(const DevMesh* __restrict__ dm, const double* __restrict__ tb, int ncol,
                                            int nh, double* __restrict__ qlm) {
  INSTANCE;
  __shared__ double lds4[4];
  const int t = blockIdx.x / ncol, c = blockIdx.x - t * ncol;
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < d.Nb; b += NT) s += d.bnd_table[b * nh + t] * tb[b * ncol + c];
  s = block_sum_all(s, lds4);
  if (threadIdx.x == 0) qlm[((int64_t)blockIdx.y * nh + t) * ncol + c] = s;
}

void launch_adj_bnd(const Batch& b, const double* Kw, const double* u, int ncol, int nh, double* tb, double* qlm,
                    hipStream_t s) {
  if (b.mx.Nb == 0) return;
  if (b.mx.Nh > 0)
    hipLaunchKernelGGL(k_cbT, dim3(nblocks(b.mx.Nh * ncol, NT, 4096), b.ni), dim3(NT), 0, s, b.dm, Kw, ncol, tb);
  const int64_t ncell = b.mx.n_bnd_cells;
  if (ncell > 0) {
    const dim3 g((unsigned)(ncell < 65536 ? ncell : 65536), b.ni);
    switch (b.mx.P) {
      case 2: hipLaunchKernelGGL(k_liftT<2>, g, dim3(NT), 0, s, b.dm, u, ncol, tb); break;
      case 3: hipLaunchKernelGGL(k_liftT<3>, g, dim3(NT), 0, s, b.dm, u, ncol, tb); break;
      default: hipLaunchKernelGGL(k_liftT<4>, g, dim3(NT), 0, s, b.dm, u, ncol, tb);
    }
  }
  hipLaunchKernelGGL(k_qlm, dim3(nh * ncol, b.ni), dim3(NT), 0, s, b.dm, tb, ncol, nh, qlm);
}

// K_rho at the extended rows and its orbital part: for pair (r, s) with
// K = K_Re - i K_Im (r < s) or K_Re (r = s): Phib_r += K phi_s,
// Phib_s += conj(K) phi_r (r = s: Phib_r += 2 K phi_r).
constexpr int KR_CH = 16;
__global__ void __launch_bounds__(NT) k_krho(const DevMesh* __restrict__ dm, const double* __restrict__ z,
                                             const double* __restrict__ qlm, int lmax, int ncol,
                                             const int* __restrict__ colmap, const double2* __restrict__ phi,
                                             double2* __restrict__ Phib) {
  INSTANCE;
  __shared__ double sR[KR_CH * 169];
  __shared__ double sK[KR_CH * AN * AN];
  __shared__ double sq[169 * AN * AN];
  __shared__ int sCm[AN * AN];
  const int n = d.n, nh = (lmax + 1) * (lmax + 1);
  z += d.oF * ncol;
  phi += d.oE * n;
  Phib += d.oE * n;
  qlm += (int64_t)blockIdx.y * nh * ncol;
  for (int e = threadIdx.x; e < nh * ncol; e += NT) sq[e] = qlm[e];
  for (int e = threadIdx.x; e < n * n; e += NT) sCm[e] = colmap[e];
  const double cx = d.center[0], cy = d.center[1], cz = d.center[2];
  for (int64_t base = (int64_t)blockIdx.x * KR_CH; base < d.NE; base += (int64_t)gridDim.x * KR_CH) {
    const int cnt = (int)((d.NE - base) < KR_CH ? (d.NE - base) : KR_CH);
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const int64_t i = base + threadIdx.x;
      solid_regular(d.xyz[3 * i] - cx, d.xyz[3 * i + 1] - cy, d.xyz[3 * i + 2] - cz, lmax, sR + threadIdx.x * nh);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < cnt * ncol; e += NT) {
      const int r = e / ncol, c = e - r * ncol;
      const int64_t i = base + r;
      double s = 0.0;
      for (int t = 0; t < nh; ++t) s += sR[r * nh + t] * sq[t * ncol + c];
      sK[r * ncol + c] = d.m[i] * (4.0 * M_PI * z[i * ncol + c] + s);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < cnt * n; e += NT) {
      const int r = e / n, p = e - r * n;
      const int64_t i = base + r;
      double2 acc = Phib[i * n + p];
      for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) {
          const int c0 = sCm[a * n + b];
          if (a == b) {
            if (p == a) acc = cadd(acc, cscale(2.0 * sK[r * ncol + c0], phi[i * n + a]));
          } else {
            const double2 K = make_double2(sK[r * ncol + c0], -sK[r * ncol + c0 + 1]);
            if (p == a) acc = cadd(acc, cmul(K, phi[i * n + b]));
            if (p == b) acc = cadd(acc, cmul(cconj(K), phi[i * n + a]));
          }
        }
      Phib[i * n + p] = acc;
    }
  }
}
void launch_krho(const Batch& b, const double* z, const double* qlm, int lmax, int ncol, const int* colmap,
                 const double* phi, double* Phib, hipStream_t s) {
  hipLaunchKernelGGL(k_krho, dim3(nblocks(b.mx.NE, KR_CH, 4096), b.ni), dim3(NT), 0, s, b.dm, z, qlm, lmax, ncol,
                     colmap, (const double2*)phi, (double2*)Phib);
}

// Split a full-node load vector (extended rows) the way the operator pass
// does: non-master DoFs get their mass-solved value in out, masters and
// hanging rows go to acc (gathered and solved on the interface afterwards).
__global__ void __launch_bounds__(NT) k_load_split(const DevMesh* __restrict__ dm, const double2* __restrict__ f,
                                                   double2* __restrict__ out, double2* __restrict__ acc) {
  INSTANCE;
  const int n = d.n;
  const int64_t o = d.oE * n, total = d.NE * n;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e / n;
    const double2 v = f[o + e];
    if (i < d.N && d.ma_index[i] < 0) out[o + e] = cscale(d.inv_mass[i], v);
    else acc[o + e] = v;
  }
}
void launch_load_split(const Batch& b, const double* f, double* out, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_load_split, dim3(nblocks(b.mx.NE * b.mx.n, NT, 8192), b.ni), dim3(NT), 0, s, b.dm,
                     (const double2*)f, (double2*)out, (double2*)acc);
}

}  // namespace mh
