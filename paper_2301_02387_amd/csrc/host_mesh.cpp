// Octree mesh, Gauss-Lobatto nodes and hanging-node constraints (host).
//
// Sec. III.A: uniform coarse cubes halved recursively; tensor-product
// Lagrange basis on Gauss-Lobatto points in each cell; continuity across
// refinement interfaces through bridged basis functions.  Here a node is
// hanging iff the coarsest leaf whose closed box contains it does not have
// it as one of its own nodes, and its value is that leaf's interpolant.
//
// Node identity is exact: per dimension a node coordinate is either a dyadic
// multiple of H / 2^(Lmax+1) (cell ends; the p = 2 midpoint) or an interior
// Gauss-Lobatto offset (p = 3), which belongs to exactly one (level, index,
// offset) triple; both kinds are encoded as 64-bit integers.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <unordered_set>

#include "host.hpp"

namespace mh {

// ---------------------------------------------------------------- GLL ----
static double legendre_p(int n, double x, double* dp) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) {
    if (dp) *dp = 0.0;
    return 1.0;
  }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    double d2 = d0 + (2.0 * k - 1.0) * p1;  // P_k' = P_{k-2}' + (2k-1) P_{k-1}
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  if (dp) *dp = d1;
  return p1;
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double dp;
      double pz = legendre_p(n, z, &dp);
      double dz = pz / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double dp;
    legendre_p(n, z, &dp);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

double lagrange(const std::vector<double>& nodes, int a, double x) {
  double v = 1.0;
  for (size_t b = 0; b < nodes.size(); ++b)
    if ((int)b != a) v *= (x - nodes[b]) / (nodes[a] - nodes[b]);
  return v;
}

static double lagrange_d(const std::vector<double>& nodes, int a, double x) {
  double s = 0.0;
  int n = (int)nodes.size();
  for (int c = 0; c < n; ++c) {
    if (c == a) continue;
    double t = 1.0 / (nodes[a] - nodes[c]);
    for (int b = 0; b < n; ++b)
      if (b != a && b != c) t *= (x - nodes[b]) / (nodes[a] - nodes[b]);
    s += t;
  }
  return s;
}

Gll make_gll(int p) {
  Gll g;
  g.p = p;
  int P = p + 1;
  g.x.assign(P, 0.0);
  g.w.assign(P, 0.0);
  g.x[0] = -1.0;
  g.x[p] = 1.0;
  // interior nodes: roots of P_p', by Newton from Chebyshev-Lobatto guesses,
  // using (1 - x^2) P_p'' = 2x P_p' - p(p+1) P_p.
  for (int i = 1; i < p; ++i) {
    double z = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double dp;
      double pz = legendre_p(p, z, &dp);
      double d2 = (2.0 * z * dp - p * (p + 1.0) * pz) / (1.0 - z * z);
      double dz = dp / d2;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    g.x[i] = z;
  }
  for (int i = 0; i < P; ++i) {
    double pz = legendre_p(p, g.x[i], nullptr);
    g.w[i] = 2.0 / (p * (p + 1.0) * pz * pz);
  }
  g.A.assign(P * P, 0.0);
  for (int a = 0; a < P; ++a)
    for (int b = 0; b < P; ++b) {
      double s = 0.0;
      for (int q = 0; q < P; ++q) s += g.w[q] * lagrange_d(g.x, a, g.x[q]) * lagrange_d(g.x, b, g.x[q]);
      g.A[a * P + b] = s;
    }
  g.Qs.assign(P * P, 0.0);
  for (int a = 0; a < P; ++a)
    for (int b = 0; b < P; ++b)
      g.Qs[a * P + b] = 0.5 * (g.w[a] * lagrange_d(g.x, b, g.x[a]) - g.w[b] * lagrange_d(g.x, a, g.x[b]));
  return g;
}

// ---------------------------------------------------------- octree ----
namespace {

constexpr int kIdxBits = 19;
inline uint64_t pack(int l, int64_t i, int64_t j, int64_t k) {
  return ((uint64_t)l << (3 * kIdxBits)) | ((uint64_t)i << (2 * kIdxBits)) | ((uint64_t)j << kIdxBits) |
         (uint64_t)k;
}
struct Leaf {
  int l;
  int64_t i, j, k;
};
inline Leaf unpack(uint64_t c) {
  const uint64_t m = (1ull << kIdxBits) - 1;
  return Leaf{(int)(c >> (3 * kIdxBits)), (int64_t)((c >> (2 * kIdxBits)) & m), (int64_t)((c >> kIdxBits) & m),
              (int64_t)(c & m)};
}

inline uint64_t spread3(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}

struct Key3 {
  int64_t k[3];
  bool operator==(const Key3& o) const { return k[0] == o.k[0] && k[1] == o.k[1] && k[2] == o.k[2]; }
};
struct Key3Hash {
  size_t operator()(const Key3& a) const {
    uint64_t h = 1469598103934665603ull;
    for (int d = 0; d < 3; ++d) {
      h ^= (uint64_t)a.k[d] + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
      h *= 1099511628211ull;
    }
    return (size_t)h;
  }
};

}  // namespace

// Kelly's indicator (Sec. III.A) of the softened nuclear potential
// V = -sum Z / sqrt(|r - R|^2 + a^2) on every leaf: u_K interpolates V at the
// leaf's own Gauss-Lobatto nodes, and eta_K^2 = (h_K / 24) sum over the
// leaf's interior faces of the integral of the squared jump of du/dn, h_K =
// sqrt(3) edge.  Each face is integrated on its parts shared with one
// neighbour (the whole face against a leaf of the same or the next coarser
// level, else the four faces of the finer leaves across it) by the tensor
// Gauss-Legendre rule of p + 1 points, exact for the polynomial jump squared.
static void kelly_indicators(const std::vector<uint64_t>& leaves, const std::unordered_set<uint64_t>& set, double lo,
                             double H, int nc, int p, const std::vector<double>& xi, const KellyReq& kr,
                             std::vector<double>& eta2) {
  const int P = p + 1;
  std::vector<double> gq, gw;
  gauss_legendre(P, gq, gw);
  auto holder = [&](int l, int64_t a, int64_t b, int64_t c) -> int {
    for (int L = l; L >= 0; --L) {
      const int s = l - L;
      if (set.count(pack(L, a >> s, b >> s, c >> s))) return L;
    }
    return -1;
  };
  auto pot = [&](double x, double y, double z) {
    double v = 0.0;
    for (const Nucleus& n : kr.nuclei) {
      const double dx = x - n.R[0], dy = y - n.R[1], dz = z - n.R[2];
      v -= n.Z / std::sqrt(dx * dx + dy * dy + dz * dz + kr.soft * kr.soft);
    }
    return v;
  };
  struct Cell {
    double h, o[3];
    std::vector<double> U;  // U[(c P + b) P + a] = V at node (a, b, c)
  };
  auto make_cell = [&](int l, int64_t i, int64_t j, int64_t k) {
    Cell C;
    C.h = H / std::ldexp(1.0, l);
    const int64_t idx[3] = {i, j, k};
    for (int d = 0; d < 3; ++d) C.o[d] = lo + C.h * idx[d];
    C.U.resize(P * P * P);
    for (int c = 0; c < P; ++c)
      for (int b = 0; b < P; ++b)
        for (int a = 0; a < P; ++a)
          C.U[(c * P + b) * P + a] = pot(C.o[0] + C.h * (xi[a] + 1.0) / 2.0, C.o[1] + C.h * (xi[b] + 1.0) / 2.0,
                                         C.o[2] + C.h * (xi[c] + 1.0) / 2.0);
    return C;
  };
  // d u_C / d x_d at a physical point
  auto dgrad = [&](const Cell& C, int d, const double* x) {
    double B[3][4];
    for (int e = 0; e < 3; ++e) {
      const double t = 2.0 * (x[e] - C.o[e]) / C.h - 1.0;
      for (int a = 0; a < P; ++a) B[e][a] = e == d ? lagrange_d(xi, a, t) * (2.0 / C.h) : lagrange(xi, a, t);
    }
    double s = 0.0;
    for (int c = 0; c < P; ++c)
      for (int b = 0; b < P; ++b) {
        double r = 0.0;
        for (int a = 0; a < P; ++a) r += C.U[(c * P + b) * P + a] * B[0][a];
        s += r * B[1][b] * B[2][c];
      }
    return s;
  };
  eta2.assign(leaves.size(), 0.0);
  for (size_t n = 0; n < leaves.size(); ++n) {
    const Leaf L = unpack(leaves[n]);
    const Cell K = make_cell(L.l, L.i, L.j, L.k);
    const int64_t idx[3] = {L.i, L.j, L.k};
    const int64_t n_l = (int64_t)nc << L.l;
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) {
      const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int64_t nb[3] = {idx[0], idx[1], idx[2]};
        nb[d] += sgn;
        if (nb[d] < 0 || nb[d] >= n_l) continue;  // box boundary
        const double xd = K.o[d] + (sgn > 0 ? K.h : 0.0);
        struct Part {
          Cell N;
          double t0, t1, side;
        };
        std::vector<Part> parts;
        const int Lh = holder(L.l, nb[0], nb[1], nb[2]);
        if (Lh >= 0) {
          const int s = L.l - Lh;
          parts.push_back({make_cell(Lh, nb[0] >> s, nb[1] >> s, nb[2] >> s), K.o[e1], K.o[e2], K.h});
        } else {
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
              int64_t c[3];
              c[d] = 2 * nb[d] + (sgn > 0 ? 0 : 1);
              c[e1] = 2 * idx[e1] + a;
              c[e2] = 2 * idx[e2] + b;
              parts.push_back({make_cell(L.l + 1, c[0], c[1], c[2]), K.o[e1] + a * K.h / 2, K.o[e2] + b * K.h / 2,
                               K.h / 2});
            }
        }
        for (const Part& pt : parts) {
          for (int u = 0; u < P; ++u)
            for (int v = 0; v < P; ++v) {
              double x[3];
              x[d] = xd;
              x[e1] = pt.t0 + pt.side * (gq[u] + 1.0) / 2.0;
              x[e2] = pt.t1 + pt.side * (gq[v] + 1.0) / 2.0;
              const double jump = dgrad(K, d, x) - dgrad(pt.N, d, x);
              acc += gw[u] * gw[v] * (pt.side / 2.0) * (pt.side / 2.0) * jump * jump;
            }
        }
      }
    }
    eta2[n] = std::sqrt(3.0) * K.h / 24.0 * acc;
  }
}

std::string build_mesh(double lo, double hi, int nc, int p, const std::vector<Ball>& balls, Mesh& M,
                       bool& unsupported, const KellyReq* kelly, int level_cap, const Mesh* from) {
  unsupported = false;
  if (p < 1 || p > 3) {
    unsupported = true;
    return "degree p must be 1, 2 or 3";
  }
  if (!(hi > lo) || nc < 1) return "invalid box";
  const int P = p + 1;
  M.lo = lo; M.hi = hi; M.nc = nc; M.p = p; M.P = P;
  M.balls = balls;
  M.H = (hi - lo) / nc;
  M.gll = make_gll(p);
  const double H = M.H;

  // ---- ball refinement to a fixed point --------------------------------
  std::vector<uint64_t> cur;
  if (from) {  // start from another mesh's leaves (same box)
    if (from->nc != nc || from->lo != lo || from->hi != hi) return "leaves of a mesh on another box";
    for (int64_t e = 0; e < from->n_cells; ++e)
      cur.push_back(pack(from->cell_level[e], from->cell_ijk[3 * e], from->cell_ijk[3 * e + 1],
                         from->cell_ijk[3 * e + 2]));
  } else {
    for (int64_t k = 0; k < nc; ++k)
      for (int64_t j = 0; j < nc; ++j)
        for (int64_t i = 0; i < nc; ++i) cur.push_back(pack(0, i, j, k));
  }
  for (;;) {
    bool changed = false;
    std::vector<uint64_t> nxt;
    nxt.reserve(cur.size());
    for (uint64_t c : cur) {
      Leaf L = unpack(c);
      double h = H / std::ldexp(1.0, L.l);
      bool split = false;
      for (const Ball& b : balls) {
        if (b.levels <= L.l) continue;
        double d2 = 0.0;
        int64_t idx[3] = {L.i, L.j, L.k};
        for (int d = 0; d < 3; ++d) {
          double a0 = lo + h * idx[d], a1 = a0 + h;
          double e = std::max(std::max(a0 - b.c[d], 0.0), b.c[d] - a1);
          d2 += e * e;
        }
        if (std::sqrt(d2) < b.r) { split = true; break; }
      }
      if (split) {
        if (L.l + 1 > 12 || ((int64_t)nc << (L.l + 1)) >= (1ll << kIdxBits)) return "refinement too deep";
        for (int c3 = 0; c3 < 8; ++c3)
          nxt.push_back(pack(L.l + 1, 2 * L.i + (c3 & 1), 2 * L.j + ((c3 >> 1) & 1), 2 * L.k + (c3 >> 2)));
        changed = true;
      } else {
        nxt.push_back(c);
      }
    }
    cur.swap(nxt);
    if (!changed) break;
  }

  // ---- 2:1 balance over 26 neighbours ------------------------------------
  std::unordered_set<uint64_t> set(cur.begin(), cur.end());
  auto coarsest_holder = [&](int l, int64_t a, int64_t b, int64_t c) -> int {
    for (int L = l; L >= 0; --L) {
      int s = l - L;
      if (set.count(pack(L, a >> s, b >> s, c >> s))) return L;
    }
    return -1;
  };
  auto balance = [&]() {
    for (;;) {
      bool changed = false;
      std::vector<uint64_t> snap(set.begin(), set.end());
      std::sort(snap.begin(), snap.end());
      for (uint64_t c : snap) {
        if (!set.count(c)) continue;
        Leaf L = unpack(c);
        if (L.l < 2) continue;
        int64_t nl = (int64_t)nc << L.l;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              if (!dx && !dy && !dz) continue;
              int64_t a = L.i + dx, b = L.j + dy, cc = L.k + dz;
              if (a < 0 || b < 0 || cc < 0 || a >= nl || b >= nl || cc >= nl) continue;
              int Lh = coarsest_holder(L.l, a, b, cc);
              if (Lh >= 0 && Lh < L.l - 1) {
                int s = L.l - Lh;
                int64_t ia = a >> s, ib = b >> s, ic = cc >> s;
                set.erase(pack(Lh, ia, ib, ic));
                for (int c3 = 0; c3 < 8; ++c3)
                  set.insert(pack(Lh + 1, 2 * ia + (c3 & 1), 2 * ib + ((c3 >> 1) & 1), 2 * ic + (c3 >> 2)));
                changed = true;
              }
            }
      }
      if (!changed) break;
    }
  };
  balance();

  // ---- Kelly refinement ----------------------------------------------------
  M.kelly = KellyReq();
  M.kelly_rounds = 0;
  if (kelly && !kelly->nuclei.empty()) {
    if (!(kelly->soft > 0.0) || !(kelly->tol > 0.0) || kelly->max_level < 0) return "invalid Kelly refinement request";
    M.kelly = *kelly;
    std::vector<double> eta2;
    for (;;) {
      std::vector<uint64_t> cur_leaves(set.begin(), set.end());
      std::sort(cur_leaves.begin(), cur_leaves.end());
      kelly_indicators(cur_leaves, set, lo, H, nc, p, M.gll.x, *kelly, eta2);
      std::vector<uint64_t> marked;
      for (size_t n = 0; n < cur_leaves.size(); ++n)
        if (unpack(cur_leaves[n]).l < kelly->max_level && eta2[n] > kelly->tol * kelly->tol)
          marked.push_back(cur_leaves[n]);
      if (marked.empty()) break;
      for (uint64_t c : marked) {
        const Leaf L = unpack(c);
        if (L.l + 1 > 12 || ((int64_t)nc << (L.l + 1)) >= (1ll << kIdxBits)) return "refinement too deep";
        set.erase(c);
        for (int c3 = 0; c3 < 8; ++c3)
          set.insert(pack(L.l + 1, 2 * L.i + (c3 & 1), 2 * L.j + ((c3 >> 1) & 1), 2 * L.k + (c3 >> 2)));
      }
      balance();
      ++M.kelly_rounds;
    }
  }

  // ---- level cap: ancestors at level_cap replace deeper leaves ---------------
  if (level_cap >= 0) {
    std::unordered_set<uint64_t> capped;
    for (uint64_t c : set) {
      const Leaf L = unpack(c);
      if (L.l <= level_cap) {
        capped.insert(c);
      } else {
        const int s = L.l - level_cap;
        capped.insert(pack(level_cap, L.i >> s, L.j >> s, L.k >> s));
      }
    }
    set.swap(capped);
  }

  // ---- Morton order of the leaves -----------------------------------------
  std::vector<uint64_t> leaves(set.begin(), set.end());
  int Lmax = 0;
  for (uint64_t c : leaves) Lmax = std::max(Lmax, unpack(c).l);
  M.Lmax = Lmax;
  std::vector<std::pair<uint64_t, uint64_t>> order;
  order.reserve(leaves.size());
  for (uint64_t c : leaves) {
    Leaf L = unpack(c);
    int s = Lmax - L.l;
    uint64_t code = spread3((uint64_t)L.i << s) | (spread3((uint64_t)L.j << s) << 1) |
                    (spread3((uint64_t)L.k << s) << 2);
    order.push_back({code, c});
  }
  std::sort(order.begin(), order.end());
  const int64_t nC = (int64_t)order.size();
  M.n_cells = nC;
  M.cell_level.resize(nC);
  M.cell_ijk.resize(3 * nC);
  M.cell_h.resize(nC);
  M.cell_org.resize(3 * nC);
  M.level_counts.assign(Lmax + 1, 0);
  for (int64_t e = 0; e < nC; ++e) {
    Leaf L = unpack(order[e].second);
    M.cell_level[e] = L.l;
    M.cell_ijk[3 * e] = L.i; M.cell_ijk[3 * e + 1] = L.j; M.cell_ijk[3 * e + 2] = L.k;
    double h = H / std::ldexp(1.0, L.l);
    M.cell_h[e] = h;
    M.cell_org[3 * e] = lo + h * L.i; M.cell_org[3 * e + 1] = lo + h * L.j; M.cell_org[3 * e + 2] = lo + h * L.k;
    M.level_counts[L.l]++;
  }

  // ---- per-dimension node keys --------------------------------------------
  const int64_t NI = (int64_t)nc << Lmax;
  const int64_t top = (int64_t)nc << (Lmax + 1);
  std::vector<int> two_s(P, -1);  // 2 * offset for dyadic offsets, -1 otherwise
  for (int a = 0; a < P; ++a) {
    if (a == 0) two_s[a] = 0;
    else if (a == p) two_s[a] = 2;
    else if (p == 2 && a == 1) two_s[a] = 1;
  }
  auto dim_key = [&](int l, int64_t idx, int a) -> int64_t {
    if (two_s[a] >= 0) return (2 * idx + two_s[a]) << (Lmax - l);
    return -(1 + ((l * NI + idx) * P + a));
  };
  auto key_t = [&](int64_t k) -> double {  // position in coarse-cell units
    if (k >= 0) return std::ldexp((double)k, -(Lmax + 1));
    int64_t code = -k - 1;
    int a = (int)(code % P);
    int64_t rest = code / P;
    int64_t idx = rest % NI;
    int l = (int)(rest / NI);
    return (idx + 0.5 * (M.gll.x[a] + 1.0)) / std::ldexp(1.0, l);
  };

  // ---- nodes in first-touch order over Morton-sorted cells -----------------
  std::unordered_map<Key3, int64_t, Key3Hash> nodemap;
  nodemap.reserve((size_t)nC * P * P * P / 2);
  std::vector<Key3> keys;
  std::vector<int64_t> tmp_nodes(nC * P * P * P);
  for (int64_t e = 0; e < nC; ++e) {
    int l = M.cell_level[e];
    for (int c = 0; c < P; ++c)
      for (int b = 0; b < P; ++b)
        for (int a = 0; a < P; ++a) {
          Key3 K{{dim_key(l, M.cell_ijk[3 * e], a), dim_key(l, M.cell_ijk[3 * e + 1], b),
                  dim_key(l, M.cell_ijk[3 * e + 2], c)}};
          auto it = nodemap.find(K);
          int64_t id;
          if (it == nodemap.end()) {
            id = (int64_t)keys.size();
            nodemap.emplace(K, id);
            keys.push_back(K);
          } else {
            id = it->second;
          }
          tmp_nodes[(e * P + c) * P * P + b * P + a] = id;
        }
  }
  int64_t nF = (int64_t)keys.size();

  // ---- breadth-first cell order (Cuthill-McKee on cells sharing a node) -------
  // Starting from the first Morton cell (a box corner), cells are visited
  // level set by level set, so cells that share nodes sit near each other in
  // the cell order (the node-centric passes read the data of a node's
  // incident cells).  The nodes get a provisional first-touch numbering here;
  // the library numbering below orders them by position.
  {
    const int P3 = P * P * P;
    std::vector<int64_t> cptr(nF + 1, 0), cidx((size_t)nC * P3);
    for (int64_t t = 0; t < nC * P3; ++t) cptr[tmp_nodes[t] + 1]++;
    for (int64_t v = 0; v < nF; ++v) cptr[v + 1] += cptr[v];
    {
      std::vector<int64_t> fillp(cptr.begin(), cptr.end() - 1);
      for (int64_t e = 0; e < nC; ++e)
        for (int t = 0; t < P3; ++t) cidx[fillp[tmp_nodes[e * P3 + t]]++] = e;
    }
    std::vector<int64_t> order;
    order.reserve(nC);
    std::vector<char> seen(nC, 0);
    for (int64_t s0 = 0; s0 < nC; ++s0) {
      if (seen[s0]) continue;
      seen[s0] = 1;
      size_t head = order.size();
      order.push_back(s0);
      while (head < order.size()) {
        const int64_t e = order[head++];
        for (int t = 0; t < P3; ++t) {
          const int64_t v = tmp_nodes[e * P3 + t];
          for (int64_t k = cptr[v]; k < cptr[v + 1]; ++k) {
            const int64_t f = cidx[k];
            if (!seen[f]) {
              seen[f] = 1;
              order.push_back(f);
            }
          }
        }
      }
    }
    // permute cells and renumber nodes by first touch in the new order
    std::vector<int32_t> lvl(nC);
    std::vector<int64_t> ijk(3 * nC);
    std::vector<double> ch(nC), co(3 * nC);
    std::vector<int64_t> newid(nF, -1), tn2(tmp_nodes.size());
    std::vector<Key3> keys2(nF);
    int64_t next = 0;
    for (int64_t e2 = 0; e2 < nC; ++e2) {
      const int64_t e = order[e2];
      lvl[e2] = M.cell_level[e];
      ch[e2] = M.cell_h[e];
      for (int d = 0; d < 3; ++d) {
        ijk[3 * e2 + d] = M.cell_ijk[3 * e + d];
        co[3 * e2 + d] = M.cell_org[3 * e + d];
      }
      for (int t = 0; t < P3; ++t) {
        const int64_t v = tmp_nodes[e * P3 + t];
        if (newid[v] < 0) {
          newid[v] = next;
          keys2[next] = keys[v];
          ++next;
        }
        tn2[e2 * P3 + t] = newid[v];
      }
    }
    M.cell_level.swap(lvl);
    M.cell_ijk.swap(ijk);
    M.cell_h.swap(ch);
    M.cell_org.swap(co);
    tmp_nodes.swap(tn2);
    keys.swap(keys2);
    nF = next;
  }

  // ---- classification --------------------------------------------------------
  std::unordered_map<uint64_t, int64_t> leaf_id;
  leaf_id.reserve(nC * 2);
  for (int64_t e = 0; e < nC; ++e)
    leaf_id[pack(M.cell_level[e], M.cell_ijk[3 * e], M.cell_ijk[3 * e + 1], M.cell_ijk[3 * e + 2])] = e;
  std::vector<char> is_bnd(nF, 0), is_hang(nF, 0);
  std::vector<std::vector<std::pair<int64_t, double>>> rows(nF);
  for (int64_t n = 0; n < nF; ++n) {
    const Key3& K = keys[n];
    for (int d = 0; d < 3; ++d)
      if (K.k[d] == 0 || K.k[d] == top) is_bnd[n] = 1;
    // coarsest leaf containing the node
    int64_t owner = -1;
    int Lown = -1;
    for (int L = 0; L <= Lmax && owner < 0; ++L) {
      int64_t cand[3][2];
      int ncand[3];
      int64_t nL = (int64_t)nc << L;
      for (int d = 0; d < 3; ++d) {
        int64_t k = K.k[d];
        ncand[d] = 0;
        if (k >= 0) {
          int sh = Lmax + 1 - L;
          int64_t q = k >> sh;
          if ((k & ((1ll << sh) - 1)) == 0) {
            if (q - 1 >= 0) cand[d][ncand[d]++] = q - 1;
            if (q < nL) cand[d][ncand[d]++] = q;
          } else {
            cand[d][ncand[d]++] = q;
          }
        } else {
          int64_t code = -k - 1;
          int a = (int)(code % P);
          int64_t rest = code / P;
          int64_t idx = rest % NI;
          int l = (int)(rest / NI);
          int64_t q = (L <= l) ? (idx >> (l - L))
                               : (int64_t)std::floor((idx + 0.5 * (M.gll.x[a] + 1.0)) * std::ldexp(1.0, L - l));
          cand[d][ncand[d]++] = q;
        }
      }
      for (int x = 0; x < ncand[0] && owner < 0; ++x)
        for (int y = 0; y < ncand[1] && owner < 0; ++y)
          for (int z = 0; z < ncand[2] && owner < 0; ++z) {
            auto it = leaf_id.find(pack(L, cand[0][x], cand[1][y], cand[2][z]));
            if (it != leaf_id.end()) { owner = it->second; Lown = L; }
          }
    }
    if (owner < 0) return "node outside every leaf";
    int match[3];
    bool hang = false;
    for (int d = 0; d < 3; ++d) {
      match[d] = -1;
      for (int a = 0; a < P; ++a)
        if (dim_key(Lown, M.cell_ijk[3 * owner + d], a) == K.k[d]) match[d] = a;
      if (match[d] < 0) hang = true;
    }
    if (!hang) continue;
    is_hang[n] = 1;
    double wd[3][8];
    for (int d = 0; d < 3; ++d) {
      for (int a = 0; a < P; ++a) wd[d][a] = 0.0;
      if (match[d] >= 0) {
        wd[d][match[d]] = 1.0;
      } else {
        double t = key_t(K.k[d]);
        double xi = 2.0 * (t * std::ldexp(1.0, Lown) - (double)M.cell_ijk[3 * owner + d]) - 1.0;
        for (int a = 0; a < P; ++a) wd[d][a] = lagrange(M.gll.x, a, xi);
      }
    }
    for (int c = 0; c < P; ++c)
      for (int b = 0; b < P; ++b)
        for (int a = 0; a < P; ++a) {
          double wv = wd[0][a] * wd[1][b] * wd[2][c];
          if (wv != 0.0) rows[n].push_back({tmp_nodes[(owner * P + c) * P * P + b * P + a], wv});
        }
  }
  // flatten chains: substitute hanging masters until none remain
  for (int pass = 0;; ++pass) {
    if (pass > 64) return "constraint chains do not terminate";
    bool again = false;
    for (int64_t n = 0; n < nF; ++n) {
      if (!is_hang[n]) continue;
      bool has = false;
      for (auto& mw : rows[n]) if (is_hang[mw.first]) { has = true; break; }
      if (!has) continue;
      again = true;
      std::vector<std::pair<int64_t, double>> nr;
      for (auto& mw : rows[n]) {
        if (is_hang[mw.first]) {
          for (auto& m2 : rows[mw.first]) nr.push_back({m2.first, mw.second * m2.second});
        } else {
          nr.push_back(mw);
        }
      }
      std::sort(nr.begin(), nr.end());
      std::vector<std::pair<int64_t, double>> merged;
      for (auto& t : nr) {
        if (!merged.empty() && merged.back().first == t.first) merged.back().second += t.second;
        else merged.push_back(t);
      }
      rows[n].swap(merged);
    }
    if (!again) break;
  }
  // A hanging node on the box boundary keeps its constraint row (its masters
  // lie on the same boundary face): zero for orbitals, the interpolated
  // boundary value for the Poisson potentials.

  // ---- library numbering: DoFs, hanging, boundary -----------------------------
  // Each group in the Morton order of the node positions (21 bits per axis
  // over the box).  A node's line neighbours in every incident cell are then
  // near it in index space for all but the few entries that cross a Morton
  // jump (H2O: 90 % of the operator entries within 1,500 rows, against 90,000
  // in the first-touch order of the breadth-first cell visit), so a pass that
  // walks the rows in order finds the rows it gathers in cache.
  std::vector<int64_t> lib(nF, -1);
  int64_t N = 0, Nh = 0, Nb = 0;
  {
    auto group = [&](int64_t n) { return is_hang[n] ? 1 : (is_bnd[n] ? 2 : 0); };
    std::vector<uint64_t> code(nF);
    const double scale = std::ldexp(1.0, 21) / nc;   // key_t is in coarse-cell units, 0 .. nc
    for (int64_t n = 0; n < nF; ++n) {
      uint64_t q[3];
      for (int d = 0; d < 3; ++d) {
        const double t = key_t(keys[n].k[d]) * scale;
        q[d] = t <= 0.0 ? 0 : std::min<uint64_t>((uint64_t)t, (1ull << 21) - 1);
      }
      code[n] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
    }
    std::vector<int64_t> idx(nF);
    for (int64_t n = 0; n < nF; ++n) idx[n] = n;
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
      const int ga = group(a), gb = group(b);
      return ga != gb ? ga < gb : code[a] < code[b];
    });
    for (int64_t k = 0; k < nF; ++k) lib[idx[k]] = k;
    for (int64_t n = 0; n < nF; ++n) {
      const int g = group(n);
      if (g == 0) ++N;
      else if (g == 1) ++Nh;
      else ++Nb;
    }
  }
  M.nF = nF; M.N = N; M.Nh = Nh; M.Nb = Nb;
  M.cell_nodes.resize(tmp_nodes.size());
  for (size_t t = 0; t < tmp_nodes.size(); ++t) M.cell_nodes[t] = (int32_t)lib[tmp_nodes[t]];
  M.xyz.resize(3 * nF);
  for (int64_t n = 0; n < nF; ++n)
    for (int d = 0; d < 3; ++d) M.xyz[3 * lib[n] + d] = lo + H * key_t(keys[n].k[d]);
  std::vector<int64_t> hang_of(Nh);
  for (int64_t n = 0; n < nF; ++n) if (is_hang[n]) hang_of[lib[n] - N] = n;
  M.hang_ptr.assign(Nh + 1, 0);
  M.hang_col.clear();
  M.hang_w.clear();
  std::vector<char> is_master(N, 0);
  for (int64_t h = 0; h < Nh; ++h) {
    auto r = rows[hang_of[h]];
    for (auto& mw : r) mw.first = lib[mw.first];
    std::sort(r.begin(), r.end());
    for (auto& mw : r) {
      M.hang_col.push_back(mw.first);
      M.hang_w.push_back(mw.second);
      if (mw.first < N) is_master[mw.first] = 1;
    }
    M.hang_ptr[h + 1] = (int64_t)M.hang_col.size();
  }
  M.masters.clear();
  for (int64_t k = 0; k < N; ++k) if (is_master[k]) M.masters.push_back((int32_t)k);
  if (nF >= (1ll << 31)) return "mesh too large for 32-bit node indices";
  return "";
}

}  // namespace mh
