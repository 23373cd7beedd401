// Host set-up of the geometric multigrid hierarchy for the pair Poisson
// operator: coarse meshes, their assembled operators, the interpolation
// between consecutive levels, smoother bounds and the dense coarsest inverse.
#include <algorithm>
#include <cmath>
#include <map>
#include <stdexcept>
#include <unordered_map>

#include "host.hpp"

namespace mh {

namespace {

uint64_t leaf_key(int l, int64_t i, int64_t j, int64_t k) {
  return ((uint64_t)l << 60) | ((uint64_t)i << 40) | ((uint64_t)j << 20) | (uint64_t)k;
}

// Leaf of mesh C containing point x (on a shared face any adjacent leaf does:
// the coarse function is continuous there).
int64_t locate(const Mesh& C, const std::unordered_map<uint64_t, int64_t>& leaves, const double* x) {
  for (int l = 0; l <= C.Lmax; ++l) {
    const int64_t n = (int64_t)C.nc << l;
    const double h = (C.hi - C.lo) / (double)n;
    int64_t ijk[3];
    for (int d = 0; d < 3; ++d) {
      int64_t t = (int64_t)std::floor((x[d] - C.lo) / h);
      ijk[d] = std::min<int64_t>(std::max<int64_t>(t, 0), n - 1);
    }
    auto it = leaves.find(leaf_key(l, ijk[0], ijk[1], ijk[2]));
    if (it != leaves.end()) return it->second;
  }
  return -1;
}

// Prolongation rows: for each DoF node of F, the coarse function's value there
// as a combination of C's DoFs.
void prolongation(const Mesh& F, const Mesh& C, MgLevel& out) {
  std::unordered_map<uint64_t, int64_t> leaves;
  leaves.reserve(C.n_cells * 2);
  for (int64_t e = 0; e < C.n_cells; ++e)
    leaves[leaf_key(C.cell_level[e], C.cell_ijk[3 * e], C.cell_ijk[3 * e + 1], C.cell_ijk[3 * e + 2])] = e;
  const int P = C.P;
  const int64_t NEc = C.N + C.Nh;
  out.p_ptr.assign(F.N + 1, 0);
  out.p_col.clear();
  out.p_val.clear();
  std::map<int64_t, double> row;
  for (int64_t i = 0; i < F.N; ++i) {
    const double* x = &F.xyz[3 * i];
    const int64_t e = locate(C, leaves, x);
    if (e < 0) throw std::runtime_error("multigrid: fine node outside the coarse mesh");
    double w1[3][4];
    for (int d = 0; d < 3; ++d) {
      const double xi = 2.0 * (x[d] - C.cell_org[3 * e + d]) / C.cell_h[e] - 1.0;
      for (int a = 0; a < P; ++a) w1[d][a] = lagrange(C.gll.x, a, xi);
    }
    row.clear();
    for (int c = 0; c < P; ++c)
      for (int b = 0; b < P; ++b)
        for (int a = 0; a < P; ++a) {
          const double w = w1[0][a] * w1[1][b] * w1[2][c];
          if (std::fabs(w) < 1e-15) continue;
          const int64_t nd = C.cell_nodes[(e * P + c) * P * P + b * P + a];
          if (nd < C.N) {
            row[nd] += w;
          } else if (nd < NEc) {  // hanging: its constraint row (boundary masters carry zero)
            const int64_t h = nd - C.N;
            for (int64_t t = C.hang_ptr[h]; t < C.hang_ptr[h + 1]; ++t)
              if (C.hang_col[t] < C.N) row[C.hang_col[t]] += w * C.hang_w[t];
          }
        }
    for (const auto& kv : row)
      if (std::fabs(kv.second) > 1e-14) {
        out.p_col.push_back((int32_t)kv.first);
        out.p_val.push_back(kv.second);
      }
    out.p_ptr[i + 1] = (int32_t)out.p_col.size();
  }
  // transpose
  const int64_t Nc = C.N;
  out.r_ptr.assign(Nc + 1, 0);
  for (int32_t c : out.p_col) out.r_ptr[c + 1]++;
  for (int64_t c = 0; c < Nc; ++c) out.r_ptr[c + 1] += out.r_ptr[c];
  out.r_col.assign(out.p_col.size(), 0);
  out.r_val.assign(out.p_col.size(), 0.0);
  std::vector<int32_t> fill(out.r_ptr.begin(), out.r_ptr.end() - 1);
  for (int64_t i = 0; i < F.N; ++i)
    for (int32_t t = out.p_ptr[i]; t < out.p_ptr[i + 1]; ++t) {
      const int32_t c = out.p_col[t];
      out.r_col[fill[c]] = (int32_t)i;
      out.r_val[fill[c]++] = out.p_val[t];
    }
}

void csr_apply(const MgLevel& L, const std::vector<double>& x, std::vector<double>& y) {
  y.assign(L.N, 0.0);
  for (int64_t i = 0; i < L.N; ++i) {
    double s = 0.0;
    for (int32_t t = L.k_ptr[i]; t < L.k_ptr[i + 1]; ++t) s += L.k_val[t] * x[L.k_col[t]];
    y[i] = s;
  }
}

// Largest eigenvalue of D^-1 K by power iteration (a fixed seed-free start).
double lambda_max(const MgLevel& L) {
  std::vector<double> x(L.N), y;
  for (int64_t i = 0; i < L.N; ++i) x[i] = 1.0 + 0.5 * std::sin(0.7 * (double)i);
  double lam = 0.0;
  for (int it = 0; it < 40; ++it) {
    csr_apply(L, x, y);
    double nrm = 0.0;
    for (int64_t i = 0; i < L.N; ++i) {
      y[i] *= L.dinv[i];
      nrm += y[i] * y[i];
    }
    nrm = std::sqrt(nrm);
    double xn = 0.0;
    for (double v : x) xn += v * v;
    lam = nrm / std::sqrt(xn);
    for (int64_t i = 0; i < L.N; ++i) x[i] = y[i] / nrm;
  }
  return lam;
}

void take_operator(const OpHost& H, int64_t N, MgLevel& L) {
  L.N = N;
  L.k_ptr = H.kt_ptr;
  L.k_col = H.kt_col;
  L.k_val = H.kt_val;
  L.dinv = H.kdiag_inv;
}

}  // namespace

void build_multigrid(const Mesh& fine, const OpHost& fop, MgHost& mg, int max_coarse) {
  mg.lv.clear();
  std::vector<Mesh> meshes;
  meshes.push_back(fine);
  MgLevel L0;
  take_operator(fop, fine.N, L0);
  mg.lv.push_back(std::move(L0));
  // coarser meshes: Q1 on the same leaves, then shallower balls (a Kelly mesh:
  // its leaves capped one level shallower at a time, so every level nests in
  // the one above), then coarser base grids
  struct Plan {
    int nc;
    std::vector<Ball> balls;
    int cap;  // level cap of a Kelly mesh, -1 otherwise
  };
  std::vector<Plan> plan;
  const bool kelly = !fine.kelly.nuclei.empty();
  if (kelly) {
    for (int cap = fine.Lmax; cap >= 0; --cap) plan.push_back({fine.nc, {}, cap});
  } else {
    int maxlev = 0;
    for (const Ball& b : fine.balls) maxlev = std::max(maxlev, b.levels);
    for (int drop = 0; drop <= maxlev; ++drop) {
      std::vector<Ball> bl;
      for (Ball b : fine.balls) {
        b.levels = std::max(0, b.levels - drop);
        if (b.levels > 0) bl.push_back(b);
      }
      plan.push_back({fine.nc, bl, -1});
    }
  }
  for (int nc = fine.nc; nc % 2 == 0 && (int64_t)(nc - 1) * (nc - 1) * (nc - 1) > max_coarse;) {
    nc /= 2;
    plan.push_back({nc, {}, -1});
  }
  const double pol[3] = {0.0, 0.0, 1.0};
  for (size_t pi = 0; pi < plan.size(); ++pi) {
    const auto& pl = plan[pi];
    Mesh C;
    bool uns = false;
    std::string err = pl.cap >= 0 ? build_mesh(fine.lo, fine.hi, pl.nc, 1, {}, C, uns, nullptr, pl.cap, &fine)
                                  : build_mesh(fine.lo, fine.hi, pl.nc, 1, pl.balls, C, uns);
    if (!err.empty()) throw std::runtime_error("multigrid coarse mesh: " + err);
    const Mesh& F = meshes.back();
    if (F.p == 1 && C.n_cells == F.n_cells && C.nc == F.nc) continue;  // same mesh as the level above
    // a level that removes less than 40 % of the unknowns costs launches without
    // coarsening much; skip it (the meshes are nested, so the next one still is)
    if (pi + 1 < plan.size() && (double)C.N > 0.6 * (double)mg.lv.back().N) continue;
    if (C.N == 0) break;
    OpHost HC;
    build_operator(C, {}, pol, 0, HC);
    prolongation(F, C, mg.lv.back());
    MgLevel LC;
    take_operator(HC, C.N, LC);
    mg.lv.push_back(std::move(LC));
    meshes.push_back(std::move(C));
    if (mg.lv.back().N <= max_coarse) break;  // small enough for the dense solve
  }
  for (MgLevel& L : mg.lv) L.lmax = 1.05 * lambda_max(L);
  // the coarsest operator as a dense row-major matrix (inverted on the device)
  const MgLevel& Lc = mg.lv.back();
  const int64_t n = Lc.N;
  mg.coarse_dense.assign(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t t = Lc.k_ptr[i]; t < Lc.k_ptr[i + 1]; ++t) mg.coarse_dense[i * n + Lc.k_col[t]] = Lc.k_val[t];
}

}  // namespace mh
