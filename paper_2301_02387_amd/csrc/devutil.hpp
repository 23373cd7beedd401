// Device helpers shared by the kernel translation units (wave64, 256 threads).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mh {

#ifndef NT
#define NT 256
#endif

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
__device__ __forceinline__ XcdSweep xcd_sweep(int64_t total, int per_block, bool xcd = true) {
  if (!xcd) {  // plain grid-stride sweep
    XcdSweep s;
    s.start = (int64_t)blockIdx.x * per_block;
    s.end = total;
    s.step = (int64_t)gridDim.x * per_block;
    return s;
  }
  const int x = blockIdx.x % N_XCD;
  const int lb = blockIdx.x / N_XCD;
  const int nbx = gridDim.x / N_XCD;
  const int64_t R = (total + N_XCD - 1) / N_XCD;
  XcdSweep s;
  s.start = x * R + (int64_t)lb * per_block;
  s.end = (x + 1) * R < total ? (x + 1) * R : total;
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
