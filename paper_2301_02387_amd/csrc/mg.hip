// Geometric multigrid preconditioner for the pair Poisson solves: a V-cycle
// per instance over the hierarchy built by build_multigrid (the operator's own
// Q_p space, Q1 on the same leaves, Q1 on shallower refinements, coarser base
// grids, a dense inverse at the bottom), with Chebyshev smoothing
// preconditioned by the diagonal.  All n^2 real pair columns go through every
// pass together ([rows][ncol] arrays), and every pass covers all instances of
// a batch in one launch: blockIdx.y selects the instance's level record, and
// records of levels an instance does not have are inactive.
#include <hip/hip_runtime.h>

#include <cmath>

#include "devutil.hpp"
#include "kernels.hpp"
#include "mg.hpp"

namespace mh {

#define INSTANCE const DevMesh& d = dm[blockIdx.y]

// sum of val[t] (x[col[t] ncol + c] - xm[col[t] ncol + c]) (SUB; else x alone)
// over t = beg, beg + stride, ... < end, for end > beg.  Rounds of 8 entries:
// the indices and coefficients of the next round are requested before this
// round's gathers, so each round waits for one memory latency.  Entries past
// the end repeat the last one with coefficient 0 (in-bounds loads, no branch).
template <bool SUB, class IP, class DP, class XP>
__device__ __forceinline__ double row_gather_dot(IP col, DP val, int beg, int end, int stride, XP x, XP xm, int ncol,
                                                 int c) {
  double s = 0.0;
  int jn[8];
  double an[8];
#pragma unroll
  for (int h = 0; h < 8; ++h) {
    const int tt = beg + h * stride;
    const int tc = tt < end ? tt : end - 1;
    jn[h] = col[tc];
    an[h] = tt < end ? val[tc] : 0.0;
  }
  for (int t = beg; t < end; t += 8 * stride) {
    int jc[8];
    double ac[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      jc[h] = jn[h];
      ac[h] = an[h];
    }
    if (t + 8 * stride < end) {
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int tt = t + (8 + h) * stride;
        const int tc = tt < end ? tt : end - 1;
        jn[h] = col[tc];
        an[h] = tt < end ? val[tc] : 0.0;
      }
    }
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int64_t j = (int64_t)jc[h] * ncol + c;
      s += ac[h] * (SUB ? (double)x[j] - (double)xm[j] : (double)x[j]);
    }
  }
  return s;
}

// The same with V adjacent columns per lane (c0 .. c0 + V, 16-byte loads;
// ncol and c0 multiples of V): s[v] += the entries' sum for column c0 + v.
template <int V, bool SUB, class IP, class DP, class XP>
__device__ __forceinline__ void row_gather_v(IP col, DP val, int beg, int end, int stride, XP x, XP xm, int ncol,
                                             int c0, double* s) {
  int jn[8];
  double an[8];
#pragma unroll
  for (int h = 0; h < 8; ++h) {
    const int tt = beg + h * stride;
    const int tc = tt < end ? tt : end - 1;
    jn[h] = col[tc];
    an[h] = tt < end ? val[tc] : 0.0;
  }
  for (int t = beg; t < end; t += 8 * stride) {
    int jc[8];
    double ac[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      jc[h] = jn[h];
      ac[h] = an[h];
    }
    if (t + 8 * stride < end) {
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int tt = t + (8 + h) * stride;
        const int tc = tt < end ? tt : end - 1;
        jn[h] = col[tc];
        an[h] = tt < end ? val[tc] : 0.0;
      }
    }
    double xv[8][V];
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      load_vals<V>(x + (int64_t)jc[h] * ncol + c0, xv[h]);
      if constexpr (SUB) {
        double mv[V];
        load_vals<V>(xm + (int64_t)jc[h] * ncol + c0, mv);
#pragma unroll
        for (int v = 0; v < V; ++v) xv[h][v] -= mv[v];
      }
    }
#pragma unroll
    for (int h = 0; h < 8; ++h)
#pragma unroll
      for (int v = 0; v < V; ++v) s[v] += ac[h] * xv[h][v];
  }
}

// coarse.r = R (fine.r - fine.t) for each instance whose fine record is
// active (tres: fine.t holds the residual r - A z already, R fine.t).  A
// restriction row gathers every fine node in the support of a coarse basis
// function (up to 343 entries from Q3 to Q1), so one wave takes a row: groups
// of cw lanes (a power of two >= ncol) split its entries, lane c of a group
// holds column c, and the groups are combined by shuffles.
__global__ void __launch_bounds__(NT) k_mg_restrict(const MgLevelDev* __restrict__ fine,
                                                    const MgLevelDev* __restrict__ coarse, int ncol, int cw,
                                                    int tres) {
  const MgLevelDev& F = fine[blockIdx.y];
  if (!F.active || (F.done && *F.done)) return;
  const MgLevelDev& C = coarse[blockIdx.y];
  const auto* ptr = gbl(F.r_ptr);
  const auto* col = gbl(F.r_col);
  const auto* val = gbl(F.r_val);
  const auto* r = gbl((const double*)F.r);
  const auto* t = gbl((const double*)F.t);
  const auto* rf = gbl(F.rf);
  const auto* tf = gbl((const float*)F.tf);
  const bool f32 = F.f32 != 0;
  auto* y = gblw(C.r);
  const int lane = threadIdx.x & 63;
  const int grp = lane / cw, c = lane - grp * cw, ngrp = 64 / cw;
  const int64_t nrow = C.N;
  for (int64_t w = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6; w < nrow; w += ((int64_t)gridDim.x * NT) >> 6) {
    double s = 0.0;
    if (c < ncol) {
      const int beg = ptr[w] + grp, end = ptr[w + 1];
      if (end > beg) {
        if (tres)
          s = f32 ? row_gather_dot<false>(col, val, beg, end, ngrp, tf, tf, ncol, c)
                  : row_gather_dot<false>(col, val, beg, end, ngrp, t, t, ncol, c);
        else
          s = f32 ? row_gather_dot<true>(col, val, beg, end, ngrp, rf, tf, ncol, c)
                  : row_gather_dot<true>(col, val, beg, end, ngrp, r, t, ncol, c);
      }
    }
    for (int off = 32; off >= cw; off >>= 1) s += __shfl_xor(s, off, 64);
    if (grp == 0 && c < ncol) y[w * ncol + c] = s;
  }
}

// The restriction with V columns per lane (ncol a multiple of V, cw a power
// of two >= ncol / V lanes per group): 64 / cw groups split a row's entries,
// each with eight entries in flight, and the coarse rows are swept by XCD.
// TRES as tres of k_mg_restrict.
template <int V, bool TRES>
__global__ void __launch_bounds__(NT) k_mg_restrict_v(const MgLevelDev* __restrict__ fine,
                                                      const MgLevelDev* __restrict__ coarse, int ncol, int cw) {
  const MgLevelDev& F = fine[blockIdx.y];
  if (!F.active || (F.done && *F.done)) return;
  const MgLevelDev& C = coarse[blockIdx.y];
  const auto* ptr = gbl(F.r_ptr);
  const auto* col = gbl(F.r_col);
  const auto* val = gbl(F.r_val);
  const auto* r = gbl((const double*)F.r);
  const auto* t = gbl((const double*)F.t);
  const auto* rf = gbl(F.rf);
  const auto* tf = gbl((const float*)F.tf);
  const bool f32 = F.f32 != 0;
  auto* y = gblw(C.r);
  const int lane = threadIdx.x & 63;
  const int grp = lane / cw, c0 = (lane - grp * cw) * V, ngrp = 64 / cw;
  const bool act = c0 < ncol;
  const XcdSweep sw = xcd_sweep(C.N, NT / 64);
  for (int64_t w = sw.start + (threadIdx.x >> 6); w < sw.end; w += sw.step) {
    double s[V];
#pragma unroll
    for (int v = 0; v < V; ++v) s[v] = 0.0;
    const int beg = ptr[w] + grp, end = ptr[w + 1];
    if (act && end > beg) {
      if constexpr (TRES) {
        if (f32) row_gather_v<V, false>(col, val, beg, end, ngrp, tf, tf, ncol, c0, s);
        else row_gather_v<V, false>(col, val, beg, end, ngrp, t, t, ncol, c0, s);
      } else {
        if (f32) row_gather_v<V, true>(col, val, beg, end, ngrp, rf, tf, ncol, c0, s);
        else row_gather_v<V, true>(col, val, beg, end, ngrp, r, t, ncol, c0, s);
      }
    }
    for (int off = 32; off >= cw; off >>= 1)
#pragma unroll
      for (int v = 0; v < V; ++v) s[v] += __shfl_xor(s[v], off, 64);
    if (grp == 0 && act)
#pragma unroll
      for (int v = 0; v < V; ++v) y[w * ncol + c0 + v] = s[v];
  }
}

// fine.z += P coarse.z with V columns per lane and L lanes per row (a power
// of two >= ncol / V), so a wave takes 64 / L rows at once; rows swept by XCD.
template <int V, int L>
__global__ void __launch_bounds__(NT) k_mg_prolong_v(const MgLevelDev* __restrict__ fine,
                                                     const MgLevelDev* __restrict__ coarse, int ncol) {
  const MgLevelDev& F = fine[blockIdx.y];
  if (!F.active || (F.done && *F.done)) return;
  const MgLevelDev& C = coarse[blockIdx.y];
  const auto* ptr = gbl(F.p_ptr);
  const auto* col = gbl(F.p_col);
  const auto* val = gbl(F.p_val);
  const auto* x = gbl((const double*)C.z);
  auto* z = gblw(F.z);
  auto* zf = gblw(F.zf);
  const bool f32 = F.f32 != 0;
  const int c0 = (int)(threadIdx.x & (L - 1)) * V;
  const bool act = c0 < ncol;
  const XcdSweep sw = xcd_sweep(F.N, NT / L);
  for (int64_t i = sw.start + threadIdx.x / L; i < sw.end; i += sw.step) {
    const int beg = ptr[i], end = ptr[i + 1];
    if (!act || end <= beg) continue;
    double s[V];
#pragma unroll
    for (int v = 0; v < V; ++v) s[v] = 0.0;
    row_gather_v<V, false>(col, val, beg, end, 1, x, x, ncol, c0, s);
    const int64_t e = i * ncol + c0;
    double zo[V];
    if (f32) {
      load_vals<V>(zf + e, zo);
#pragma unroll
      for (int v = 0; v < V; ++v) zf[e + v] = (float)(zo[v] + s[v]);
    } else {
      load_vals<V>(z + e, zo);
#pragma unroll
      for (int v = 0; v < V; ++v) z[e + v] = zo[v] + s[v];
    }
  }
}

// fine.z += P coarse.z for each instance whose fine record is active
__global__ void __launch_bounds__(NT) k_mg_prolong(const MgLevelDev* __restrict__ fine,
                                                   const MgLevelDev* __restrict__ coarse, int ncol) {
  const MgLevelDev& F = fine[blockIdx.y];
  if (!F.active || (F.done && *F.done)) return;
  const MgLevelDev& C = coarse[blockIdx.y];
  const int64_t total = F.N * ncol;
  const auto* ptr = gbl(F.p_ptr);
  const auto* col = gbl(F.p_col);
  const auto* val = gbl(F.p_val);
  const auto* x = gbl((const double*)C.z);
  auto* z = gblw(F.z);
  auto* zf = gblw(F.zf);
  const bool f32 = F.f32 != 0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e / ncol;
    const int c = (int)(e - i * ncol);
    const int beg = ptr[i], end = ptr[i + 1];
    if (end > beg) {
      const double v = row_gather_dot<false>(col, val, beg, end, 1, x, x, ncol, c);
      if (f32) zf[e] = (float)((double)zf[e] + v);
      else z[e] += v;
    }
  }
}

// z = Ainv r on each instance's coarsest level (dense, row-major): one wave
// per (row, block of 8 columns), the lanes splitting the row's entries
__global__ void __launch_bounds__(NT) k_mg_coarse(const MgLevelDev* __restrict__ co, int ncol) {
  const MgLevelDev& L = co[blockIdx.y];
  if (L.done && *L.done) return;
  const int64_t n = L.N;
  const auto* Ainv = gbl(L.cinv);
  const auto* r = gbl((const double*)L.r);
  auto* z = gblw(L.z);
  const int lane = threadIdx.x & 63;
  const int ncb = (ncol + 7) / 8;
  const int64_t items = n * ncb;
  for (int64_t w = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6; w < items; w += ((int64_t)gridDim.x * NT) >> 6) {
    const int64_t i = w / ncb;
    const int c0 = (int)(w - i * ncb) * 8;
    double acc[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[v] = 0.0;
    // four strides of 64 per round, their loads in flight together
    int64_t j = lane;
    for (; j + 192 < n; j += 256) {
      double a[4], rv[4][8];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Ainv[i * n + j + 64 * u];
#pragma unroll
        for (int v = 0; v < 8; ++v) rv[u][v] = c0 + v < ncol ? r[(j + 64 * u) * ncol + c0 + v] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[v] += a[u] * rv[u][v];
    }
    for (; j < n; j += 64) {
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

static dim3 level_grid(int64_t n, int ncol, int ni) { return dim3(nblocks(n * ncol, NT, 16384), ni); }

// Coarse-level passes with the operator product fused in, LN lanes per row
// and V adjacent columns per lane (16-byte loads for V = 4):
//  - MODE 0, one Chebyshev smoothing step k (the recurrence of k_mg_cheb):
//    res = r - A zin (res = r for the first step from zero), d = c1 d +
//    c2 D^-1 res, zout = zin + d (zout = d for the first step from zero).
//    The smoothing has degree 2 (k = 0, 1): d is stored only by step 0 from
//    a nonzero z; from zero, step 1 takes d from its zin, which step 0 wrote.
//    zin and zout are the level's z and t arrays (into_t: z -> t, else
//    t -> z), so the rows gathered from zin are never the rows written.
//  - MODE 1, the residual t = r - A z that the restriction reads.
template <int MODE, int V, int LN>
__global__ void __launch_bounds__(NT) k_mg_level_pass(const MgLevelDev* __restrict__ lv, int ncol, int k,
                                                      int from_zero, int into_t) {
  const MgLevelDev& L = lv[blockIdx.y];
  if (!L.active || (L.done && *L.done)) return;
  const double b = L.lmax, a = L.lmax / MG_RANGE;
  const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
  double c1 = 0.0, c2 = 1.0 / theta;
  double rho = 1.0 / sigma;
  for (int j = 1; j <= k; ++j) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    c1 = rn * rho;
    c2 = 2.0 * rn / delta;
    rho = rn;
  }
  const bool first = MODE == 0 && from_zero && k == 0;
  const auto* ptr = gbl(L.a_ptr);
  const auto* col = gbl(L.a_col);
  const auto* val = gbl(L.a_val);
  const auto* dinv = gbl(L.dinv);
  const auto* r = gbl((const double*)L.r);
  const auto* zin = gbl((const double*)(MODE == 1 || into_t ? L.z : L.t));
  auto* zout = gblw(MODE == 1 || into_t ? L.t : L.z);
  auto* dd = gblw(L.d);
  const int c0 = (int)(threadIdx.x % LN) * V;
  const bool act = c0 < ncol;
  for (int64_t i = ((int64_t)blockIdx.x * NT + threadIdx.x) / LN; i < L.N; i += (int64_t)gridDim.x * NT / LN) {
    if (!act) continue;
    double y[V];
#pragma unroll
    for (int v = 0; v < V; ++v) y[v] = 0.0;
    if (!first) {
      const int beg = ptr[i], end = ptr[i + 1];
      if (end > beg) row_gather_v<V, false>(col, val, beg, end, 1, zin, zin, ncol, c0, y);
    }
    const int64_t e = i * ncol + c0;
    double rv[V];
    load_vals<V>(r + e, rv);
    if constexpr (MODE == 1) {
#pragma unroll
      for (int v = 0; v < V; ++v) zout[e + v] = rv[v] - y[v];
    } else {
      const double di = dinv[i];
      double dv[V], zv[V];
      if (!first) load_vals<V>(zin + e, zv);
      if (k > 0) {
        if (from_zero) {  // the first step's d is its zout, this step's zin
#pragma unroll
          for (int v = 0; v < V; ++v) dv[v] = zv[v];
        } else {
          load_vals<V>(dd + e, dv);
        }
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double dn = (k > 0 ? c1 * dv[v] : 0.0) + c2 * di * (rv[v] - y[v]);
        if (k == 0 && !from_zero) dd[e + v] = dn;   // the only d a later step reads
        zout[e + v] = first ? dn : zv[v] + dn;
      }
    }
  }
}

template <int MODE>
static void coarse_pass(const MgDev& mg, int l, int ni, int ncol, int k, int from_zero, int into_t, hipStream_t s) {
  auto go = [&](auto kern, int ln) {
    hipLaunchKernelGGL(kern, dim3(nblocks(mg.max_n[l] * ln, NT, 16384), ni), dim3(NT), 0, s, mg.lv[l], ncol, k,
                       from_zero, into_t);
  };
  if (ncol >= 16 && ncol % 4 == 0) {
    if (ncol > 32) go(k_mg_level_pass<MODE, 4, 16>, 16);
    else if (ncol > 16) go(k_mg_level_pass<MODE, 4, 8>, 8);
    else go(k_mg_level_pass<MODE, 4, 4>, 4);
  } else if (ncol <= 1) go(k_mg_level_pass<MODE, 1, 1>, 1);
  else if (ncol <= 2) go(k_mg_level_pass<MODE, 1, 2>, 2);
  else if (ncol <= 4) go(k_mg_level_pass<MODE, 1, 4>, 4);
  else if (ncol <= 8) go(k_mg_level_pass<MODE, 1, 8>, 8);
  else if (ncol <= 16) go(k_mg_level_pass<MODE, 1, 16>, 16);
  else if (ncol <= 32) go(k_mg_level_pass<MODE, 1, 32>, 32);
  else go(k_mg_level_pass<MODE, 1, 64>, 64);
}

static void smooth(const MgDev& mg, int l, int ni, int ncol, bool from_zero, const MgLevel0Ops& ops, hipStream_t s) {
  if (l == 0) {  // fused into the level-0 operator passes (degree mg.nu >= 2)
    if (from_zero) {
      ops.cheb0(s);                                   // steps 0 and 1
      for (int k = 2; k < mg.nu; ++k) ops.cheb(k, false, s);
    } else {
      for (int k = 0; k < mg.nu; ++k) ops.cheb(k, k == mg.nu - 1, s);
    }
    return;
  }
  // coarser levels: Chebyshev degree 2 with the products fused into the
  // steps; the first step writes t, the second brings the correction back to z
  coarse_pass<0>(mg, l, ni, ncol, 0, from_zero ? 1 : 0, 1, s);
  coarse_pass<0>(mg, l, ni, ncol, 1, from_zero ? 1 : 0, 0, s);
}

void mg_vcycle(const MgDev& mg, int ni, int ncol, const MgLevel0Ops& ops, hipStream_t s) {
  const int nl = mg.nlev;
  // 4 columns per lane in the transfers when the column count is a multiple of
  // 4: for the restriction from 16 columns on (at 4 columns its 64 lane groups
  // spend more on combining than they gain), for the prolongation from 4 on
  const bool wide = ncol >= 16 && ncol % 4 == 0;
  const bool wide_p = ncol % 4 == 0;
  for (int l = 0; l + 1 < nl; ++l) {
    smooth(mg, l, ni, ncol, true, ops, s);
    // the residual r - A z that the restriction reads: the level-0 residual
    // pass, or the coarse level's fused pass
    const int tres = 1;
    if (l > 0) coarse_pass<1>(mg, l, ni, ncol, 0, 0, 1, s);
    else ops.resid(s);
    if (wide) {
      int cw = 1;
      while (cw * 4 < ncol) cw *= 2;
      const dim3 g(xcd_grid(mg.max_n[l + 1], NT / 64, 16384), ni);
      if (tres) hipLaunchKernelGGL((k_mg_restrict_v<4, true>), g, dim3(NT), 0, s, mg.lv[l], mg.lv[l + 1], ncol, cw);
      else hipLaunchKernelGGL((k_mg_restrict_v<4, false>), g, dim3(NT), 0, s, mg.lv[l], mg.lv[l + 1], ncol, cw);
    } else {
      int cw = 1;
      while (cw < ncol) cw *= 2;
      hipLaunchKernelGGL(k_mg_restrict, dim3(nblocks(mg.max_n[l + 1] * 64, NT, 16384), ni), dim3(NT), 0, s,
                         mg.lv[l], mg.lv[l + 1], ncol, cw, tres);
    }
  }
  hipLaunchKernelGGL(k_mg_coarse, dim3(nblocks(mg.max_coarse * ((ncol + 7) / 8) * 64, NT, 4096), ni), dim3(NT), 0, s,
                     mg.coarse, ncol);
  for (int l = nl - 2; l >= 0; --l) {
    if (wide_p && ncol > 32)
      hipLaunchKernelGGL((k_mg_prolong_v<4, 16>), dim3(xcd_grid(mg.max_n[l], NT / 16, 16384), ni), dim3(NT), 0, s,
                         mg.lv[l], mg.lv[l + 1], ncol);
    else if (wide_p && ncol > 16)
      hipLaunchKernelGGL((k_mg_prolong_v<4, 8>), dim3(xcd_grid(mg.max_n[l], NT / 8, 16384), ni), dim3(NT), 0, s,
                         mg.lv[l], mg.lv[l + 1], ncol);
    else if (wide_p && ncol > 4)
      hipLaunchKernelGGL((k_mg_prolong_v<4, 4>), dim3(xcd_grid(mg.max_n[l], NT / 4, 16384), ni), dim3(NT), 0, s,
                         mg.lv[l], mg.lv[l + 1], ncol);
    else if (wide_p)
      hipLaunchKernelGGL((k_mg_prolong_v<4, 1>), dim3(xcd_grid(mg.max_n[l], NT, 16384), ni), dim3(NT), 0, s,
                         mg.lv[l], mg.lv[l + 1], ncol);
    else
      hipLaunchKernelGGL(k_mg_prolong, level_grid(mg.max_n[l], ncol, ni), dim3(NT), 0, s, mg.lv[l], mg.lv[l + 1],
                         ncol);
    smooth(mg, l, ni, ncol, false, ops, s);
  }
}

// PCG pieces: red[i][slot] = r . z per instance and column (overwrites), and
// the direction p_k = z + beta_k p_{k-1} with beta_k = rz_k / rz_{k-1}; the
// direction pass also clears the r.r slot the update pass of iteration k fills.
__global__ void __launch_bounds__(NT) k_rz_parts(const DevMesh* __restrict__ dm, int ncol, const double* __restrict__ r,
                                                 const double* __restrict__ z, double* __restrict__ part) {
  INSTANCE;
  // ncol consecutive threads take one row (coalesced), NT / ncol rows per pass
  __shared__ double lds[NT];
  r += d.oE * ncol;
  z += d.oE * ncol;
  const int groups = NT / ncol;
  const int g = threadIdx.x / ncol, c = threadIdx.x - g * ncol;
  double acc = 0.0;
  if (g < groups)
    for (int64_t i = (int64_t)blockIdx.x * groups + g; i < d.N; i += (int64_t)gridDim.x * groups)
      acc += r[i * ncol + c] * z[i * ncol + c];
  lds[threadIdx.x] = g < groups ? acc : 0.0;
  __syncthreads();
  if (threadIdx.x < (unsigned)ncol) {
    double t = 0.0;
    for (int q = 0; q < groups; ++q) t += lds[q * ncol + threadIdx.x];
    part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * ncol + threadIdx.x] = t;
  }
}
__global__ void __launch_bounds__(NT) k_rz_finish(const double* __restrict__ part, int nblk, int ncol,
                                                  double* __restrict__ red, int slot) {
  __shared__ double lds4[4];
  const int c = blockIdx.x;
  part += (int64_t)blockIdx.y * nblk * ncol;
  red += (int64_t)blockIdx.y * RED_SLOTS * ncol;
  const double v = sum_partials(part, nblk, ncol, c, lds4);
  if (threadIdx.x == 0) red[slot * ncol + c] = v;
}
void mg_rz(const DevMesh* dm, int ni, int ncol, const double* r, const double* z, double* part, double* red, int slot,
           hipStream_t s) {
  hipLaunchKernelGGL(k_rz_parts, dim3(MG_RZ_BLOCKS, ni), dim3(NT), 0, s, dm, ncol, r, z, part);
  hipLaunchKernelGGL(k_rz_finish, dim3(ncol, ni), dim3(NT), 0, s, part, MG_RZ_BLOCKS, ncol, red, slot);
}

template <class Z>
// With x (deferred solution update): also x += alpha_{k-1} p_{k-1}, alpha from
// the r.z slot rz_prev and the p.q slot pq_prev of the previous iteration,
// while p_{k-1} is read for the direction anyway.
__global__ void __launch_bounds__(NT) k_mg_dir(const DevMesh* __restrict__ dm, int ncol, const Z* __restrict__ z,
                                               const double* __restrict__ pprev, double* __restrict__ pcur,
                                               double* __restrict__ red, int rz_cur, int rz_prev, int rr_clear,
                                               double* __restrict__ x, int pq_prev) {
  INSTANCE;
  if (d.cg_done && *d.cg_done) return;  // converged instance of a batch CG
  __shared__ double beta[64], alpha[64];
  red += (int64_t)blockIdx.y * RED_SLOTS * ncol;
  const bool upd = x != nullptr && rz_prev >= 0;
  if (threadIdx.x < (unsigned)ncol) {
    double bt = 0.0, al = 0.0;
    if (rz_prev >= 0) {
      const double a = red[rz_cur * ncol + threadIdx.x], b = red[rz_prev * ncol + threadIdx.x];
      bt = b != 0.0 ? a / b : 0.0;
      if (upd) {
        const double pq = red[pq_prev * ncol + threadIdx.x];
        al = (pq != 0.0 && b != 0.0) ? b / pq : 0.0;
      }
    }
    beta[threadIdx.x] = bt;
    alpha[threadIdx.x] = al;
  }
  __syncthreads();
  z += d.oE * ncol;
  pprev += d.oE * ncol;
  pcur += d.oE * ncol;
  if (upd) x += d.oF * ncol;
  const int64_t total = d.N * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int c = (int)(e % ncol);
    const double pp = pprev[e];
    pcur[e] = (double)z[e] + (beta[c] != 0.0 ? beta[c] * pp : 0.0);
    if (upd) x[e] += alpha[c] * pp;
  }
  if (blockIdx.x == 0 && threadIdx.x < (unsigned)ncol) red[rr_clear * ncol + threadIdx.x] = 0.0;
}

// The deferred solution update of the last CG iteration: x += alpha p with
// alpha from the r.z slot rz_slot and the p.q slot pq_slot.
__global__ void __launch_bounds__(NT) k_cg_xfinal(const DevMesh* __restrict__ dm, int ncol, double* __restrict__ x,
                                                  const double* __restrict__ p, const double* __restrict__ red,
                                                  int rz_slot, int pq_slot) {
  INSTANCE;
  __shared__ double alpha[64];
  red += (int64_t)blockIdx.y * RED_SLOTS * ncol;
  if (threadIdx.x < (unsigned)ncol) {
    const double rz = red[rz_slot * ncol + threadIdx.x], pq = red[pq_slot * ncol + threadIdx.x];
    alpha[threadIdx.x] = (pq != 0.0 && rz != 0.0) ? rz / pq : 0.0;
  }
  __syncthreads();
  x += d.oF * ncol;
  p += d.oE * ncol;
  const int64_t total = d.N * ncol;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT)
    x[e] += alpha[e % ncol] * p[e];
}
void cg_xfinal(const DevMesh* dm, int ni, int64_t max_n, int ncol, double* x, const double* p, const double* red,
               int rz_slot, int pq_slot, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_xfinal, dim3(nblocks(max_n * ncol, NT, 8192), ni), dim3(NT), 0, s, dm, ncol, x, p, red,
                     rz_slot, pq_slot);
}
void mg_dir(const DevMesh* dm, int ni, int64_t max_n, int ncol, const double* z, const double* pprev, double* pcur,
            double* red, int rz_cur, int rz_prev, int rr_clear, double* x, int pq_prev, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_dir<double>, dim3(nblocks(max_n * ncol, NT, 8192), ni), dim3(NT), 0, s, dm, ncol, z, pprev,
                     pcur, red, rz_cur, rz_prev, rr_clear, x, pq_prev);
}
void mg_dir(const DevMesh* dm, int ni, int64_t max_n, int ncol, const float* z, const double* pprev, double* pcur,
            double* red, int rz_cur, int rz_prev, int rr_clear, double* x, int pq_prev, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_dir<float>, dim3(nblocks(max_n * ncol, NT, 8192), ni), dim3(NT), 0, s, dm, ncol, z, pprev,
                     pcur, red, rz_cur, rz_prev, rr_clear, x, pq_prev);
}

}  // namespace mh
