// Device helpers shared by the kernels of libgps: complex arithmetic,
// deterministic FP64 block reductions, slot lookup.
#pragma once

#include <type_traits>

#include "gps_internal.h"

namespace gps {

template <typename T>
__device__ __forceinline__ cplx<T> cmk(T x, T y) { cplx<T> c; c.x = x; c.y = y; return c; }
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return cmk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return cmk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return cmk(a.x * s, a.y * s); }

// Sum of v over the work-group, identical in every thread.  Fixed reduction
// tree (wavefront butterfly, then waves in index order): the result depends
// only on the inputs, never on timing.  Any block size up to 1024 threads.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double wsum[16];
  __shared__ double total;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) wsum[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += wsum[w];
    total = s;
  }
  __syncthreads();
  double r = total;
  __syncthreads();   // the shared words may be reused by the next call
  return r;
}

// Sum of v over the wavefront, in every lane (fixed butterfly: the result
// depends only on the inputs).  No barrier: a kernel whose work-groups hold
// several wavefronts writes one partial per wavefront.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic sum of n partials spaced by `stride` doubles: four
// independent loads in flight per thread, fixed combination order.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n,
                                               int stride = 1) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const int step = blockDim.x;
  int i = threadIdx.x;
  for (; i + 3 * step < n; i += 4 * step) {
    const double a = part[(size_t)i * stride];
    const double b = part[(size_t)(i + step) * stride];
    const double c = part[(size_t)(i + 2 * step) * stride];
    const double d = part[(size_t)(i + 3 * step) * stride];
    s0 += a;
    s1 += b;
    s2 += c;
    s3 += d;
  }
  for (; i < n; i += step) s0 += part[(size_t)i * stride];
  return block_sum((s0 + s1) + (s2 + s3));
}

// Tile processed by work-group `bid` of a G-group launch.  Work-groups are
// dealt round-robin to the 8 XCDs (each with its own L2); this bijection
// gives every XCD a contiguous range of tiles, so tiles that share cache
// lines (neighbouring pencils, rows of one plane) meet in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int G) {
  constexpr int X = 8;
  const int q = G / X, r = G % X;
  const int xcd = bid % X, local = bid / X;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Ghost index on an axis of n points: wrapped (periodic) or edge-replicated.
__device__ __forceinline__ int ghost_index(int i, int n, int periodic) {
  if (periodic) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  return min(max(i, 0), n - 1);
}

// Element at a 32-bit byte offset from a work-group-uniform base pointer.
// The address is then the scalar base plus a 32-bit vector offset, with no
// 64-bit vector arithmetic.  Callers guarantee offsets below 4 GiB.
template <typename V>
__device__ __forceinline__ V& at_bytes(V* base, unsigned off) {
  return *reinterpret_cast<V*>(reinterpret_cast<
      typename std::conditional<std::is_const<V>::value, const char, char>::type*>(base) + off);
}

// Stop flag of a solve, for the y, z and x-inverse passes.  Its writers are
// the x-forward head (loss of definiteness) and work-group 0 of the y-inverse
// pass (the stop decision), which it reads only at the end: so the flag is
// the same for every wavefront of a launch, except in the y-inverse pass of
// the last iteration, where the other work-groups' results are unused either
// way.  stop_flag_issue is called right after
// the pass's operand loads: every lane loads the flag through a vector load
// (the zero offset comes from an instruction the compiler cannot fold), so it
// travels with the operands and the wait for them covers it, instead of a
// scalar load issued after that wait.  stop_flag_set reads lane 0's copy as a
// scalar.
__device__ __forceinline__ int stop_flag_issue(const SolveState* st) {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return reinterpret_cast<const int*>(&st->done)[z];
}
__device__ __forceinline__ bool stop_flag_set(int v) {
  return __builtin_amdgcn_readfirstlane(v) != 0;
}

// Plain scalar read of the stop flag (generic passes).
__device__ __forceinline__ int solve_stopped(const SolveState* st) { return st->done; }

}  // namespace gps
