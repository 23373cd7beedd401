// Device helpers shared by the kernel translation units (wave64, 256 threads).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mh {

#ifndef NT
#define NT 256
#endif

// Array pointers read from an instance record in memory are generic to the
// compiler, which then emits flat loads (tracked by both wait counters, so
// dependent loads serialise).  They all point to device global memory; this
// cast lets the compiler emit global loads instead.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gbl(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gblw(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// 16-byte global load of element i of a double2 array (double2 is a class
// type that does not copy from another address space; the native vector type does).
typedef double dvec2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ldg2(const double2* p, int64_t i) {
  const dvec2_t v = ((const __attribute__((address_space(1))) dvec2_t*)p)[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ double2 ldg2(const double* p, int64_t i) {
  return ldg2(reinterpret_cast<const double2*>(p), i);
}

// V consecutive values of a global row as doubles, in 16-byte loads (double
// pairs or float quads; the row is aligned to V elements).
typedef float fvec2_t __attribute__((ext_vector_type(2)));
typedef float fvec4_t __attribute__((ext_vector_type(4)));
template <int V>
__device__ __forceinline__ void load_vals(const __attribute__((address_space(1))) double* row, double* out) {
  if constexpr (V == 1) {
    out[0] = row[0];
  } else {
#pragma unroll
    for (int v = 0; v < V / 2; ++v) {
      const double2 r2 = ldg2((const double*)row, v);
      out[2 * v] = r2.x;
      out[2 * v + 1] = r2.y;
    }
  }
}
template <int V>
__device__ __forceinline__ void load_vals(const __attribute__((address_space(1))) float* row, double* out) {
  if constexpr (V == 1) {
    out[0] = row[0];
  } else if constexpr (V == 2) {
    const fvec2_t f = *(const __attribute__((address_space(1))) fvec2_t*)row;
    out[0] = f.x;
    out[1] = f.y;
  } else {
#pragma unroll
    for (int v = 0; v < V / 4; ++v) {
      const fvec4_t f = ((const __attribute__((address_space(1))) fvec4_t*)row)[v];
      out[4 * v] = f.x;
      out[4 * v + 1] = f.y;
      out[4 * v + 2] = f.z;
      out[4 * v + 3] = f.w;
    }
  }
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cjmul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Sum over a 256-thread block; the result is returned to every thread.
__device__ __forceinline__ double block_sum_all(double v, double* lds4) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds4[wid] = v;
  __syncthreads();
  return lds4[0] + lds4[1] + lds4[2] + lds4[3];
}

// Deterministic sum of part[b * stride + o] over b < nblk by one 256-thread block.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nblk, int stride, int o,
                                               double* lds4) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += NT) s += part[(int64_t)b * stride + o];
  return block_sum_all(s, lds4);
}

// Regular solid harmonics R_lm(x) of the multipole expansion, (lmax+1)^2 values:
// index l*l + m holds the cos part, l*l + l + m (m > 0) the sin part.
__device__ inline void solid_regular(double x, double y, double z, int lmax, double* R) {
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

// The order-m terms of solid_regular alone (l = m .. lmax), with the same
// arithmetic: (x + i y)^m and (2m - 1)!! by the same recurrence, then the
// recurrence in l.
__device__ inline void solid_regular_m(double x, double y, double z, int lmax, int m, double* R) {
  const double r2 = x * x + y * y + z * z;
  double pre = 1.0, pim = 0.0, dfact = 1.0;
  for (int k = 1; k <= m; ++k) {
    double t = pre * x - pim * y;
    pim = pre * y + pim * x;
    pre = t;
    dfact *= (2.0 * k - 1.0);
  }
  double a_re = dfact * pre, a_im = dfact * pim, b_re = 0.0, b_im = 0.0;
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

static inline int nblocks(int64_t work, int per = NT, int cap = 1 << 20) {
  int64_t b = (work + per - 1) / per;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

// XCD-aware sweep of [0, total) in chunks of `per_block` items.  Workgroups
// are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8),
// each with its own L2.  XCD x takes the contiguous range [x R, (x+1) R)
// and its blocks walk it side by side, so the items in flight on one XCD
// lie in a window of (blocks per XCD) * per_block consecutive items whose
// neighbours are mostly in that XCD's L2.  gridDim.x must be a multiple of 8.
constexpr int N_XCD = 8;
struct XcdSweep {
  int64_t start, end, step;
};
// (bx, gx): this workgroup's index and the number of workgroups taking part
// (a launch may reserve its first workgroups for other work; the reserved
// count is a multiple of 8, so bx % 8 is still the XCD).
__device__ __forceinline__ XcdSweep xcd_sweep(int64_t total, int per_block, bool xcd, int bx, int gx) {
  if (!xcd) {  // plain grid-stride sweep
    XcdSweep s;
    s.start = (int64_t)bx * per_block;
    s.end = total;
    s.step = (int64_t)gx * per_block;
    return s;
  }
  const int x = bx % N_XCD;
  const int lb = bx / N_XCD;
  const int nbx = gx / N_XCD;
  const int64_t R = (total + N_XCD - 1) / N_XCD;
  XcdSweep s;
  s.start = x * R + (int64_t)lb * per_block;
  s.end = (x + 1) * R < total ? (x + 1) * R : total;
  s.step = (int64_t)nbx * per_block;
  return s;
}
__device__ __forceinline__ XcdSweep xcd_sweep(int64_t total, int per_block, bool xcd = true) {
  return xcd_sweep(total, per_block, xcd, (int)blockIdx.x, (int)gridDim.x);
}
// Column blocks bound to XCDs: with B column blocks (B divides 8), XCD x
// serves column block x % B and the 8 / B XCDs of one column block split the
// items into contiguous ranges, so each L2 holds one column block's rows.
// (bx, gx) as in xcd_sweep.
__device__ __forceinline__ XcdSweep xcd_sweep_cols(int64_t total, int per_block, int B, int bx, int gx) {
  const int x = bx % N_XCD;
  const int G = N_XCD / B;   // XCDs per column block
  const int xg = x / B;      // this XCD's rank among them
  const int lb = bx / N_XCD;
  const int nbx = gx / N_XCD;
  const int64_t R = (total + G - 1) / G;
  XcdSweep s;
  s.start = xg * R + (int64_t)lb * per_block;
  s.end = (xg + 1) * R < total ? (xg + 1) * R : total;
  s.step = (int64_t)nbx * per_block;
  return s;
}
static inline int xcd_grid(int64_t items, int per_block, int cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b > cap) b = cap;
  b = ((b + N_XCD - 1) / N_XCD) * N_XCD;
  return (int)(b < N_XCD ? N_XCD : b);
}

// Blocks for grid-stride reductions: about one per compute unit.
constexpr int RED_BLOCKS = 256;
// Grid cap of the node-centric Poisson operator (its p.q partial sums).
constexpr int STENCIL_BLOCKS = 8192;

}  // namespace mh
