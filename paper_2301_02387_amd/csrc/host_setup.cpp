// Operator set-up on the host: Gauss-Lobatto masses, lumped nuclear
// potential, dipole weights, the hanging-interface block of the mass matrix
// with its Chebyshev spectrum bounds, the Jacobi diagonal of the Poisson
// stiffness, and the multipole boundary table.
//
// Sec. III.A: all integrals by the Gauss-Lobatto rule on each cell, so the
// full-node mass is diagonal and the mass matrix of the bridged basis is
// M = C^T diag(m) C, diagonal except on DoFs that are masters of hanging
// nodes.  The nuclear potential is lumped: v_i = sum_cells int f_i V_nuc,
// evaluated by a six-pyramid Duffy rule (apex on the nucleus, 16 Gauss
// points per direction) in cells whose closure holds a nucleus and by tensor
// Gauss-Legendre with p+5 points per direction elsewhere.
#include <algorithm>
#include <cmath>
#include <complex>
#include <functional>
#include <map>
#include <stdexcept>

#include "host.hpp"

namespace mh {

int multipole_terms(int lmax) { return (lmax + 1) * (lmax + 1); }

namespace {

// y = (h/2) (A x W x W + W x A x W + W x W x A) x   on one cell (local order a fastest)
void elem_stiff(int P, const std::vector<double>& A, const std::vector<double>& w, double h, const double* x,
                double* y) {
  double s = 0.5 * h;
  for (int c = 0; c < P; ++c)
    for (int b = 0; b < P; ++b)
      for (int a = 0; a < P; ++a) {
        double t = 0.0;
        for (int q = 0; q < P; ++q) {
          t += A[a * P + q] * w[b] * w[c] * x[(c * P + b) * P + q];
          t += w[a] * A[b * P + q] * w[c] * x[(c * P + q) * P + a];
          t += w[a] * w[b] * A[c * P + q] * x[(q * P + b) * P + a];
        }
        y[(c * P + b) * P + a] = s * t;
      }
}

void cell_regular(const Mesh& M, int64_t e, double Z, const double* R, int q, const std::vector<double>& g,
                  const std::vector<double>& gw, const std::vector<double>& Lg, double* out) {
  const int P = M.P;
  const double h = M.cell_h[e];
  const double* o = &M.cell_org[3 * e];
  std::vector<double> f(q * q * q), t1(P * q * q), t2(P * P * q);
  for (int k = 0; k < q; ++k)
    for (int j = 0; j < q; ++j)
      for (int i = 0; i < q; ++i) {
        double dx = o[0] + h * g[i] - R[0], dy = o[1] + h * g[j] - R[1], dz = o[2] + h * g[k] - R[2];
        f[(k * q + j) * q + i] = -Z / std::sqrt(dx * dx + dy * dy + dz * dz) * gw[i] * gw[j] * gw[k];
      }
  for (int a = 0; a < P; ++a)
    for (int k = 0; k < q; ++k)
      for (int j = 0; j < q; ++j) {
        double s = 0.0;
        for (int i = 0; i < q; ++i) s += Lg[a * q + i] * f[(k * q + j) * q + i];
        t1[(a * q + k) * q + j] = s;
      }
  for (int a = 0; a < P; ++a)
    for (int b = 0; b < P; ++b)
      for (int k = 0; k < q; ++k) {
        double s = 0.0;
        for (int j = 0; j < q; ++j) s += Lg[b * q + j] * t1[(a * q + k) * q + j];
        t2[(a * P + b) * q + k] = s;
      }
  const double vol = h * h * h;
  for (int c = 0; c < P; ++c)
    for (int b = 0; b < P; ++b)
      for (int a = 0; a < P; ++a) {
        double s = 0.0;
        for (int k = 0; k < q; ++k) s += Lg[c * q + k] * t2[(a * P + b) * q + k];
        out[(c * P + b) * P + a] += vol * s;
      }
}

// The same integral on a complex-scaled cell: int f_i (-Z / r(z(x))) J dx,
// z the contour of each coordinate, r the principal square root of
// sum_d (z_d - R_d)^2 (the continuation of |x - R|).
void cell_regular_scaled(const Mesh& M, int64_t e, double Z, const double* R, int q, const std::vector<double>& g,
                         const std::vector<double>& gw, const std::vector<double>& Lg,
                         const std::function<std::complex<double>(double, int)>& zc, std::complex<double> J,
                         std::complex<double>* out) {
  typedef std::complex<double> cd;
  const int P = M.P;
  const double h = M.cell_h[e];
  const double* o = &M.cell_org[3 * e];
  std::vector<cd> f(q * q * q), t1(P * q * q), t2(P * P * q);
  std::vector<cd> zx(q), zy(q), zz(q);
  for (int i = 0; i < q; ++i) {
    zx[i] = zc(o[0] + h * g[i], 0) - R[0];
    zy[i] = zc(o[1] + h * g[i], 1) - R[1];
    zz[i] = zc(o[2] + h * g[i], 2) - R[2];
  }
  for (int k = 0; k < q; ++k)
    for (int j = 0; j < q; ++j)
      for (int i = 0; i < q; ++i)
        f[(k * q + j) * q + i] = -Z * J / std::sqrt(zx[i] * zx[i] + zy[j] * zy[j] + zz[k] * zz[k]) * (gw[i] * gw[j] * gw[k]);
  for (int a = 0; a < P; ++a)
    for (int k = 0; k < q; ++k)
      for (int j = 0; j < q; ++j) {
        cd s = 0.0;
        for (int i = 0; i < q; ++i) s += Lg[a * q + i] * f[(k * q + j) * q + i];
        t1[(a * q + k) * q + j] = s;
      }
  for (int a = 0; a < P; ++a)
    for (int b = 0; b < P; ++b)
      for (int k = 0; k < q; ++k) {
        cd s = 0.0;
        for (int j = 0; j < q; ++j) s += Lg[b * q + j] * t1[(a * q + k) * q + j];
        t2[(a * P + b) * q + k] = s;
      }
  const double vol = h * h * h;
  for (int c = 0; c < P; ++c)
    for (int b = 0; b < P; ++b)
      for (int a = 0; a < P; ++a) {
        cd s = 0.0;
        for (int k = 0; k < q; ++k) s += Lg[c * q + k] * t2[(a * P + b) * q + k];
        out[(c * P + b) * P + a] += vol * s;
      }
}

void cell_duffy(const Mesh& M, int64_t e, double Z, const double* R, double* out) {
  const int P = M.P, n = 16;
  const double h = M.cell_h[e];
  const double* o = &M.cell_org[3 * e];
  std::vector<double> g, gw;
  gauss_legendre(n, g, gw);
  for (int i = 0; i < n; ++i) { g[i] = 0.5 * (g[i] + 1.0); gw[i] *= 0.5; }
  double Lx[8], Ly[8], Lz[8];
  for (int d = 0; d < 3; ++d) {
    int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    for (int side = 0; side < 2; ++side) {
      double plane = o[d] + side * h;
      double height = std::fabs(R[d] - plane);
      if (height <= 1e-14 * h) continue;
      for (int iu = 0; iu < n; ++iu)
        for (int iv = 0; iv < n; ++iv) {
          double F[3];
          F[d] = plane;
          F[d1] = o[d1] + h * g[iu];
          F[d2] = o[d2] + h * g[iv];
          double dist = std::sqrt((F[0] - R[0]) * (F[0] - R[0]) + (F[1] - R[1]) * (F[1] - R[1]) +
                                  (F[2] - R[2]) * (F[2] - R[2]));
          for (int is = 0; is < n; ++is) {
            double s = g[is];
            double X[3];
            for (int k = 0; k < 3; ++k) X[k] = R[k] + s * (F[k] - R[k]);
            double wt = gw[is] * gw[iu] * gw[iv] * s * height * h * h * (-Z) / dist;
            for (int a = 0; a < P; ++a) {
              Lx[a] = lagrange(M.gll.x, a, 2.0 * (X[0] - o[0]) / h - 1.0);
              Ly[a] = lagrange(M.gll.x, a, 2.0 * (X[1] - o[1]) / h - 1.0);
              Lz[a] = lagrange(M.gll.x, a, 2.0 * (X[2] - o[2]) / h - 1.0);
            }
            for (int c = 0; c < P; ++c)
              for (int b = 0; b < P; ++b) {
                double wb = wt * Lz[c] * Ly[b];
                for (int a = 0; a < P; ++a) out[(c * P + b) * P + a] += wb * Lx[a];
              }
          }
        }
    }
  }
}

// Eigenvalues of a small symmetric matrix by cyclic Jacobi rotations.
std::vector<double> sym_eigs(std::vector<double> a, int n) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += a[i * n + j] * a[i * n + j];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  std::vector<double> ev(n);
  for (int i = 0; i < n; ++i) ev[i] = a[i * n + i];
  std::sort(ev.begin(), ev.end());
  return ev;
}

}  // namespace

void build_operator(const Mesh& M, const std::vector<Nucleus>& nuc, const double pol[3], int lmax, OpHost& op,
                    const EcsReq* ecs) {
  typedef std::complex<double> cd;
  const int P = M.P, P3 = P * P * P;
  const int64_t nC = M.n_cells, nF = M.nF, N = M.N, NE = M.N + M.Nh;
  const std::vector<double>& w = M.gll.w;

  // ---- complex scaling: the scaled directions of every cell ---------------------
  op.ecs = ecs && ecs->theta > 0.0;
  op.ecs_theta = op.ecs ? ecs->theta : 0.0;
  const cd ph = std::polar(1.0, op.ecs_theta);
  auto zc = [&](double x, int d) -> cd {
    const double R = ecs->inner[d];
    if (std::fabs(x) <= R) return cd(x, 0.0);
    const double sg = x > 0 ? 1.0 : -1.0;
    return sg * R + ph * (x - sg * R);
  };
  if (op.ecs) {
    op.ecs_code.assign(nC, 0);
    for (int64_t e = 0; e < nC; ++e) {
      const double h = M.cell_h[e], tol = 1e-12 * h;
      for (int d = 0; d < 3; ++d) {
        const double lo = M.cell_org[3 * e + d], hi = lo + h, R = ecs->inner[d];
        const bool out = lo >= R - tol || hi <= -R + tol;
        const bool in = lo >= -R - tol && hi <= R + tol;
        if (!out && !in) throw std::invalid_argument("a cell straddles a complex-scaling plane");
        if (out) op.ecs_code[e] |= (uint8_t)(1 << d);
      }
    }
    for (const Nucleus& nu : nuc)
      for (int d = 0; d < 3; ++d)
        if (!(std::fabs(nu.R[d]) < ecs->inner[d]))
          throw std::invalid_argument("complex scaling: every nucleus must lie inside the unscaled cuboid");
  }
  std::vector<cd> vt;  // continued lumped potential (complex scaling only)
  if (op.ecs) vt.assign(nF, cd(0.0, 0.0));

  // ---- masses and dipole weights --------------------------------------------
  op.m.assign(nF, 0.0);
  for (int64_t e = 0; e < nC; ++e) {
    double s = 0.125 * M.cell_h[e] * M.cell_h[e] * M.cell_h[e];
    for (int c = 0; c < P; ++c)
      for (int b = 0; b < P; ++b)
        for (int a = 0; a < P; ++a) op.m[M.cell_nodes[e * P3 + (c * P + b) * P + a]] += s * w[a] * w[b] * w[c];
  }
  op.mz.assign(nF, 0.0);
  for (int64_t n = 0; n < nF; ++n)
    op.mz[n] = op.m[n] * (pol[0] * M.xyz[3 * n] + pol[1] * M.xyz[3 * n + 1] + pol[2] * M.xyz[3 * n + 2]);

  // ---- lumped nuclear potential ----------------------------------------------
  op.v.assign(nF, 0.0);
  {
    int q = M.p + 5;
    std::vector<double> g, gw;
    gauss_legendre(q, g, gw);
    for (int i = 0; i < q; ++i) { g[i] = 0.5 * (g[i] + 1.0); gw[i] *= 0.5; }
    std::vector<double> Lg(P * q);
    for (int a = 0; a < P; ++a)
      for (int i = 0; i < q; ++i) Lg[a * q + i] = lagrange(M.gll.x, a, 2.0 * g[i] - 1.0);
    std::vector<double> cellv(P3);
    std::vector<cd> cellc(P3);
    for (int64_t e = 0; e < nC; ++e) {
      std::fill(cellv.begin(), cellv.end(), 0.0);
      const double h = M.cell_h[e];
      const double* o = &M.cell_org[3 * e];
      for (const Nucleus& nu : nuc) {
        double tol = 1e-12 * h;
        bool inside = true;
        for (int d = 0; d < 3; ++d)
          if (nu.R[d] < o[d] - tol || nu.R[d] > o[d] + h + tol) inside = false;
        if (inside) cell_duffy(M, e, nu.Z, nu.R, cellv.data());
        else cell_regular(M, e, nu.Z, nu.R, q, g, gw, Lg, cellv.data());
      }
      for (int t = 0; t < P3; ++t) op.v[M.cell_nodes[e * P3 + t]] += cellv[t];
      if (!op.ecs) continue;
      if (op.ecs_code[e] == 0) {
        for (int t = 0; t < P3; ++t) vt[M.cell_nodes[e * P3 + t]] += cellv[t];
        continue;
      }
      // a scaled cell holds no nucleus (they lie inside the unscaled cuboid)
      std::fill(cellc.begin(), cellc.end(), cd(0.0, 0.0));
      const cd J = std::pow(ph, (double)__builtin_popcount(op.ecs_code[e]));
      for (const Nucleus& nu : nuc) cell_regular_scaled(M, e, nu.Z, nu.R, q, g, gw, Lg, zc, J, cellc.data());
      for (int t = 0; t < P3; ++t) vt[M.cell_nodes[e * P3 + t]] += cellc[t];
    }
  }

  // ---- ownership of node-diagonal terms ---------------------------------------
  op.owner_mask.assign(nC, 0ull);
  {
    std::vector<char> taken(NE, 0);
    for (int64_t e = 0; e < nC; ++e)
      for (int t = 0; t < P3; ++t) {
        int32_t n = M.cell_nodes[e * P3 + t];
        if (n < NE && !taken[n]) { taken[n] = 1; op.owner_mask[e] |= (1ull << t); }
      }
  }

  // ---- node -> incident cells (at most 8: one leaf per octant around a point)
  op.node_inc.assign((size_t)NE * 8, -1);
  {
    std::vector<uint8_t> cnt(NE, 0);
    for (int64_t e = 0; e < nC; ++e)
      for (int t = 0; t < P3; ++t) {
        int32_t nd = M.cell_nodes[e * P3 + t];
        if (nd >= NE) continue;
        if (cnt[nd] >= 8) throw std::runtime_error("a node lies in more than 8 cells");
        op.node_inc[(size_t)nd * 8 + cnt[nd]++] = (int32_t)(e * 64 + t);
      }
  }

  // ---- interface block of the mass matrix ------------------------------------
  const int64_t nMa = (int64_t)M.masters.size();
  op.ma_index.assign(N, -1);
  for (int64_t i = 0; i < nMa; ++i) op.ma_index[M.masters[i]] = (int32_t)i;
  std::vector<std::map<int32_t, double>> rows(nMa);
  for (int64_t i = 0; i < nMa; ++i) rows[i][(int32_t)i] += op.m[M.masters[i]];
  std::vector<std::vector<std::pair<int32_t, double>>> ct(nMa);
  for (int64_t h = 0; h < M.Nh; ++h) {
    double mh = op.m[N + h];
    for (int64_t a = M.hang_ptr[h]; a < M.hang_ptr[h + 1]; ++a) {
      int64_t ka = M.hang_col[a];
      if (ka >= N) continue;
      int32_t ia = op.ma_index[ka];
      ct[ia].push_back({(int32_t)(N + h), M.hang_w[a]});
      for (int64_t b = M.hang_ptr[h]; b < M.hang_ptr[h + 1]; ++b) {
        int64_t kb = M.hang_col[b];
        if (kb >= N) continue;
        rows[ia][op.ma_index[kb]] += mh * M.hang_w[a] * M.hang_w[b];
      }
    }
  }
  // Order the interface unknowns by reverse Cuthill-McKee on the block's own
  // graph (every connected piece from a node of least degree, neighbours by
  // increasing degree), so that the rows a workgroup sweeps gather their
  // neighbours from a narrow band of the interface vectors.
  std::vector<int32_t> order;  // new index -> original index
  {
    order.reserve(nMa);
    std::vector<char> seen(nMa, 0);
    std::vector<int32_t> by_deg(nMa);
    for (int64_t i = 0; i < nMa; ++i) by_deg[i] = (int32_t)i;
    std::stable_sort(by_deg.begin(), by_deg.end(),
                     [&](int32_t a, int32_t b) { return rows[a].size() < rows[b].size(); });
    for (int32_t root : by_deg) {
      if (seen[root]) continue;
      size_t head = order.size();
      order.push_back(root);
      seen[root] = 1;
      while (head < order.size()) {
        const int32_t u = order[head++];
        std::vector<int32_t> nb;
        for (auto& kv : rows[u])
          if (!seen[kv.first]) { nb.push_back(kv.first); seen[kv.first] = 1; }
        std::stable_sort(nb.begin(), nb.end(),
                         [&](int32_t a, int32_t b) { return rows[a].size() < rows[b].size(); });
        order.insert(order.end(), nb.begin(), nb.end());
      }
    }
    std::reverse(order.begin(), order.end());
  }
  std::vector<int32_t> newidx(nMa);
  for (int64_t i = 0; i < nMa; ++i) newidx[order[i]] = (int32_t)i;
  op.ma_dof.resize(nMa);
  for (int64_t i = 0; i < nMa; ++i) {
    op.ma_dof[i] = M.masters[order[i]];
    op.ma_index[op.ma_dof[i]] = (int32_t)i;
  }
  op.ma_ptr.assign(nMa + 1, 0);
  op.ma_col.clear();
  op.ma_val.clear();
  op.ma_dinv.assign(nMa, 0.0);
  for (int64_t i = 0; i < nMa; ++i) {
    std::map<int32_t, double> r;
    for (auto& kv : rows[order[i]]) r[newidx[kv.first]] = kv.second;
    for (auto& kv : r) {
      op.ma_col.push_back(kv.first);
      op.ma_val.push_back(kv.second);
      if (kv.first == i) op.ma_dinv[i] = 1.0 / kv.second;
    }
    op.ma_ptr[i + 1] = (int32_t)op.ma_col.size();
  }
  op.ct_ptr.assign(nMa + 1, 0);
  op.ct_row.clear();
  op.ct_w.clear();
  for (int64_t i = 0; i < nMa; ++i) {
    for (auto& rw : ct[order[i]]) { op.ct_row.push_back(rw.first); op.ct_w.push_back(rw.second); }
    op.ct_ptr[i + 1] = (int32_t)op.ct_row.size();
  }
  // spectrum of D^-1/2 A D^-1/2 by Lanczos, then Chebyshev iteration count
  op.cheb_lo = op.cheb_hi = 1.0;
  op.cheb_iters = 0;
  if (nMa > 0) {
    int k = (int)std::min<int64_t>(nMa, 80);
    std::vector<std::vector<double>> Q;
    std::vector<double> alpha, beta;
    std::vector<double> v(nMa), wv(nMa);
    for (int64_t i = 0; i < nMa; ++i) v[i] = 1.0 + 0.37 * std::sin(1.7 * i + 0.3);
    double nv = 0.0;
    for (double x : v) nv += x * x;
    nv = std::sqrt(nv);
    for (double& x : v) x /= nv;
    for (int it = 0; it < k; ++it) {
      Q.push_back(v);
      for (int64_t i = 0; i < nMa; ++i) {
        double s = 0.0;
        for (int32_t t = op.ma_ptr[i]; t < op.ma_ptr[i + 1]; ++t)
          s += op.ma_val[t] * std::sqrt(op.ma_dinv[i] * op.ma_dinv[op.ma_col[t]]) * v[op.ma_col[t]];
        wv[i] = s;
      }
      double a = 0.0;
      for (int64_t i = 0; i < nMa; ++i) a += wv[i] * v[i];
      alpha.push_back(a);
      for (int pass = 0; pass < 2; ++pass)
        for (auto& qv : Q) {
          double d = 0.0;
          for (int64_t i = 0; i < nMa; ++i) d += qv[i] * wv[i];
          for (int64_t i = 0; i < nMa; ++i) wv[i] -= d * qv[i];
        }
      double b = 0.0;
      for (double x : wv) b += x * x;
      b = std::sqrt(b);
      if (b < 1e-12 || it == k - 1) break;
      beta.push_back(b);
      for (int64_t i = 0; i < nMa; ++i) v[i] = wv[i] / b;
    }
    int m = (int)alpha.size();
    std::vector<double> T(m * m, 0.0);
    for (int i = 0; i < m; ++i) {
      T[i * m + i] = alpha[i];
      if (i + 1 < m) T[i * m + i + 1] = T[(i + 1) * m + i] = beta[i];
    }
    std::vector<double> ev = sym_eigs(T, m);
    op.cheb_lo = ev.front() * 0.95;
    op.cheb_hi = ev.back() * 1.05;
    double kappa = op.cheb_hi / op.cheb_lo;
    double r = (std::sqrt(kappa) - 1.0) / (std::sqrt(kappa) + 1.0);
    // error target 1e-14 of the initial error in the block's energy norm:
    // four orders below the 1e-10 to which G applications are compared
    op.cheb_iters = (int)std::ceil(std::log(1e-14 / 2.0) / std::log(r)) + 1;
  }
  op.inv_mass.assign(N, 0.0);
  for (int64_t k = 0; k < N; ++k)
    if (op.ma_index[k] < 0) op.inv_mass[k] = 1.0 / op.m[k];

  // ---- complex scaling: the load vector in units of the real mass -------------
  // The scaled operator is M_theta^-1 F_theta with M_theta = C^T diag(m_theta) C;
  // the orbital product stays the real one (M).  When no hanging node or
  // master touches a scaled cell, M and M_theta share the interface block and
  // M M_theta^-1 = diag(rho), rho = m / m_theta (1 on the interface), so
  // rho F_theta is a load vector for the real mass solve, and the products
  // c^H (rho F_theta) are M inner products: rho multiplies the stiffness and
  // derivative loads and the potential; the field weights become m (e.z) and
  // the mean-field load m V u is unchanged.
  if (op.ecs) {
    auto touches_scaled = [&](int64_t nd) {
      for (int t = 0; t < 8; ++t) {
        const int32_t code = op.node_inc[(size_t)nd * 8 + t];
        if (code < 0) break;
        if (op.ecs_code[code >> 6]) return true;
      }
      return false;
    };
    for (int64_t r = N; r < NE; ++r)
      if (touches_scaled(r)) throw std::invalid_argument("complex scaling: a hanging node touches a scaled cell");
    for (int64_t i = 0; i < nMa; ++i)
      if (touches_scaled(op.ma_dof[i])) throw std::invalid_argument("complex scaling: a master touches a scaled cell");
    std::vector<cd> mt(nF, cd(0.0, 0.0));
    for (int64_t e = 0; e < nC; ++e) {
      const cd J = std::pow(ph, (double)__builtin_popcount(op.ecs_code[e]));
      const double s = 0.125 * M.cell_h[e] * M.cell_h[e] * M.cell_h[e];
      for (int c = 0; c < P; ++c)
        for (int b = 0; b < P; ++b)
          for (int a = 0; a < P; ++a)
            mt[M.cell_nodes[e * P3 + (c * P + b) * P + a]] += (op.ecs_code[e] ? J : cd(1.0, 0.0)) * (s * w[a] * w[b] * w[c]);
    }
    op.ecs_rho.assign(2 * NE, 0.0);
    op.ecs_v.assign(2 * NE, 0.0);
    op.ecs_mz.assign(2 * NE, 0.0);
    for (int64_t r = 0; r < NE; ++r) {
      const cd rho = op.m[r] / mt[r];
      const cd vr = rho * vt[r];
      cd ez(0.0, 0.0);
      for (int d = 0; d < 3; ++d) ez += pol[d] * zc(M.xyz[3 * r + d], d);
      const cd mzr = op.m[r] * ez;
      op.ecs_rho[2 * r] = rho.real();
      op.ecs_rho[2 * r + 1] = rho.imag();
      op.ecs_v[2 * r] = vr.real();
      op.ecs_v[2 * r + 1] = vr.imag();
      op.ecs_mz[2 * r] = mzr.real();
      op.ecs_mz[2 * r + 1] = mzr.imag();
    }
  }

  // ---- assembled Poisson operator K~ = C^T K_full C on the DoFs --------------
  // Row k of K_full is the sum over k's cells of its three line couplings
  // (h/2) A (x) W (x) W etc.; rows of masters also collect c_hk times the
  // rows of the hanging nodes they constrain; columns are expanded through
  // C onto DoFs (boundary columns drop: the CG unknowns are homogeneous).
  {
    const std::vector<double>& A = M.gll.A;
    op.kt_ptr.assign(N + 1, 0);
    op.kt_col.clear();
    op.kt_val.clear();
    std::vector<std::pair<int32_t, double>> ent;
    auto add_row = [&](int64_t nd, double s) {
      for (int t = 0; t < 8; ++t) {
        const int32_t code = op.node_inc[(size_t)nd * 8 + t];
        if (code < 0) break;
        const int64_t e = code >> 6;
        const int loc = code & 63;
        const int a = loc % P, b = (loc / P) % P, c = loc / (P * P);
        const int32_t* cn = &M.cell_nodes[e * P3];
        const double hh = 0.5 * M.cell_h[e];
        for (int q = 0; q < P; ++q) {
          const int32_t js[3] = {cn[(c * P + b) * P + q], cn[(c * P + q) * P + a], cn[(q * P + b) * P + a]};
          const double cf[3] = {hh * A[a * P + q] * w[b] * w[c], hh * w[a] * A[b * P + q] * w[c],
                                hh * w[a] * w[b] * A[c * P + q]};
          for (int l = 0; l < 3; ++l) {
            const int64_t j = js[l];
            const double v = s * cf[l];
            if (j < N) {
              ent.push_back({(int32_t)j, v});
            } else if (j < NE) {
              for (int64_t r = M.hang_ptr[j - N]; r < M.hang_ptr[j - N + 1]; ++r)
                if (M.hang_col[r] < N) ent.push_back({(int32_t)M.hang_col[r], v * M.hang_w[r]});
            }
          }
        }
      }
    };
    for (int64_t k = 0; k < N; ++k) {
      ent.clear();
      add_row(k, 1.0);
      const int32_t mi = op.ma_index[k];
      if (mi >= 0)
        for (int32_t t = op.ct_ptr[mi]; t < op.ct_ptr[mi + 1]; ++t) add_row(op.ct_row[t], op.ct_w[t]);
      std::sort(ent.begin(), ent.end(),
                [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                  return x.first < y.first;
                });
      for (size_t t = 0; t < ent.size();) {
        size_t u = t;
        double v = 0.0;
        while (u < ent.size() && ent[u].first == ent[t].first) v += ent[u++].second;
        op.kt_col.push_back(ent[t].first);
        op.kt_val.push_back(v);
        t = u;
      }
      if (op.kt_col.size() >= (size_t)INT32_MAX) throw std::runtime_error("Poisson operator too large");
      op.kt_ptr[k + 1] = (int32_t)op.kt_col.size();
    }
  }

  // ---- Jacobi diagonal of C^T K_full C --------------------------------------
  {
    std::vector<double> kdiag(N, 0.0);
    std::vector<double> x(P3), y(P3);
    for (int64_t e = 0; e < nC; ++e) {
      const int32_t* cn = &M.cell_nodes[e * P3];
      bool simple = true;
      for (int t = 0; t < P3; ++t)
        if (cn[t] >= N && cn[t] < NE) simple = false;
      if (simple) {
        // element diagonal: (h/2)(A_aa w_b w_c + w_a A_bb w_c + w_a w_b A_cc)
        for (int c = 0; c < P; ++c)
          for (int b = 0; b < P; ++b)
            for (int a = 0; a < P; ++a) {
              int32_t n = cn[(c * P + b) * P + a];
              if (n >= N) continue;
              kdiag[n] += 0.5 * M.cell_h[e] *
                          (M.gll.A[a * P + a] * w[b] * w[c] + w[a] * M.gll.A[b * P + b] * w[c] +
                           w[a] * w[b] * M.gll.A[c * P + c]);
            }
        continue;
      }
      // DoFs reached from this cell, with their local weight vectors
      std::map<int64_t, std::vector<double>> wk;
      for (int t = 0; t < P3; ++t) {
        int64_t n = cn[t];
        if (n < N) {
          auto& vv = wk[n];
          if (vv.empty()) vv.assign(P3, 0.0);
          vv[t] += 1.0;
        } else if (n < NE) {
          for (int64_t a = M.hang_ptr[n - N]; a < M.hang_ptr[n - N + 1]; ++a) {
            int64_t k = M.hang_col[a];
            if (k >= N) continue;
            auto& vv = wk[k];
            if (vv.empty()) vv.assign(P3, 0.0);
            vv[t] += M.hang_w[a];
          }
        }
      }
      for (auto& kv : wk) {
        elem_stiff(P, M.gll.A, w, M.cell_h[e], kv.second.data(), y.data());
        double s = 0.0;
        for (int t = 0; t < P3; ++t) s += kv.second[t] * y[t];
        kdiag[kv.first] += s;
      }
    }
    op.kdiag_inv.assign(N, 0.0);
    for (int64_t k = 0; k < N; ++k) op.kdiag_inv[k] = 1.0 / kdiag[k];
  }

  // ---- cells that see boundary values -----------------------------------------
  op.bnd_cells.clear();
  {
    std::vector<char> hang_bnd(M.Nh, 0);
    for (int64_t h = 0; h < M.Nh; ++h)
      for (int64_t a = M.hang_ptr[h]; a < M.hang_ptr[h + 1]; ++a)
        if (M.hang_col[a] >= NE) hang_bnd[h] = 1;
    for (int64_t e = 0; e < nC; ++e) {
      bool touch = false;
      for (int t = 0; t < P3; ++t) {
        int64_t n = M.cell_nodes[e * P3 + t];
        if (n >= NE || (n >= N && hang_bnd[n - N])) touch = true;
      }
      if (touch) op.bnd_cells.push_back((int32_t)e);
    }
  }

  // ---- multipole evaluation table at the boundary nodes -----------------------
  // Regular harmonics R_lm = r^l P_l^m(cos t) e^{i m phi} (no Condon-Shortley
  // phase) by R_mm = (2m-1)!! (x+iy)^m, R_{m+1,m} = (2m+1) z R_mm,
  // (l-m) R_lm = (2l-1) z R_{l-1,m} - (l+m-1) r^2 R_{l-2,m}; irregular
  // I_lm = R_lm / r^(2l+1).  Addition theorem: 1/|x-y| = sum_{l, m>=0}
  // eps_m (l-m)!/(l+m)! Re[R_lm(y) conj(I_lm(x))], eps_0 = 1, eps_m = 2.
  // Term order within l: cos m = 0..l, then sin m = 1..l (offset l^2).
  op.nharm = multipole_terms(lmax);
  op.bnd_table.assign((size_t)M.Nb * op.nharm, 0.0);
  double ctr = 0.5 * (M.lo + M.hi);
  for (int64_t b = 0; b < M.Nb; ++b) {
    int64_t n = NE + b;
    double x = M.xyz[3 * n] - ctr, y = M.xyz[3 * n + 1] - ctr, z = M.xyz[3 * n + 2] - ctr;
    double r2 = x * x + y * y + z * z;
    double r = std::sqrt(r2);
    double* row = &op.bnd_table[(size_t)b * op.nharm];
    double pre = 1.0, pim = 0.0;  // (x+iy)^m
    double dfact = 1.0;           // (2m-1)!!
    for (int m = 0; m <= lmax; ++m) {
      if (m > 0) {
        double t = pre * x - pim * y;
        pim = pre * y + pim * x;
        pre = t;
        dfact *= (2.0 * m - 1.0);
      }
      double rm2_re = 0, rm2_im = 0, rm1_re = dfact * pre, rm1_im = dfact * pim;
      for (int l = m; l <= lmax; ++l) {
        double re, im;
        if (l == m) { re = rm1_re; im = rm1_im; }
        else if (l == m + 1) {
          re = (2.0 * m + 1.0) * z * rm1_re; im = (2.0 * m + 1.0) * z * rm1_im;
          rm2_re = rm1_re; rm2_im = rm1_im; rm1_re = re; rm1_im = im;
        } else {
          re = ((2.0 * l - 1.0) * z * rm1_re - (l + m - 1.0) * r2 * rm2_re) / (l - m);
          im = ((2.0 * l - 1.0) * z * rm1_im - (l + m - 1.0) * r2 * rm2_im) / (l - m);
          rm2_re = rm1_re; rm2_im = rm1_im; rm1_re = re; rm1_im = im;
        }
        double fr = 1.0;  // (l-m)!/(l+m)!
        for (int t = l - m + 1; t <= l + m; ++t) fr /= t;
        double eps = (m == 0) ? 1.0 : 2.0;
        double sc = eps * fr / std::pow(r, 2 * l + 1);
        row[l * l + m] = sc * re;
        if (m > 0) row[l * l + l + m] = sc * im;
      }
    }
  }
}

}  // namespace mh
