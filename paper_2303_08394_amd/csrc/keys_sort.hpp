// Device building blocks shared by the point re-sort and the device tree
// build: Morton keys of points (the host build's rule, in FP64 without
// contraction), a stable LSD radix sort of 64-bit keys with 32-bit values,
// an exclusive scan of 32-bit counts, and helpers.  Every kernel and helper
// lives in an anonymous namespace: each including source gets its own copy.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "common.hpp"
#include "hip_check.hpp"

namespace kifmm {
namespace {

constexpr int kThreads = 256;   // = the 256 digits of a pass
constexpr int kItems = 16;      // keys per thread and block tile
constexpr int kTile = kThreads * kItems;
typedef unsigned long long u64;

__device__ inline u64 spread3(u64 v) {  // bit k of v -> bit 3k (k < 21)
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
__device__ inline u64 morton3(u64 x, u64 y, u64 z) { return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z); }

struct Frame {
  double lo[3];
  double r0;  // root half-width
  int L;      // key level
};

// A point outside the closed root cube (t outside [0, 1] on some axis, or
// not a number) is counted in *outside: the update is then refused, as the
// clamp would put it in a boundary leaf beyond that leaf's equivalent surface.
__global__ void key_kernel(const double* __restrict__ xyz, int64_t n, Frame f, u64* __restrict__ keys,
                           int32_t* __restrict__ idx, unsigned long long* __restrict__ outside) {
#pragma clang fp contract(off)
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double cells = double(int64_t(1) << f.L), maxi = cells - 1.0;
  u64 ix[3];
  bool inside = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double t = (xyz[3 * i + d] - f.lo[d]) / (2.0 * f.r0);
    inside = inside && t >= 0.0 && t <= 1.0;
    double c = floor(t * cells);
    if (!(c >= 0.0)) c = 0.0;
    if (c > maxi) c = maxi;
    ix[d] = u64(c);
  }
  keys[i] = morton3(ix[0], ix[1], ix[2]);
  idx[i] = int32_t(i);
  if (!inside) atomicAdd(outside, 1ull);
}

// Digit counts of each block's tile, stored digit-major: hist[digit][block].
__global__ void radix_hist_kernel(const u64* __restrict__ keys, int64_t n, int shift,
                                  uint32_t* __restrict__ hist, int nblk) {
  __shared__ uint32_t h[kThreads];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kTile;
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k * kThreads + tid;
    if (i < n) atomicAdd(&h[unsigned(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[int64_t(tid) * nblk + blockIdx.x] = h[tid];
}

// Exclusive prefix sum of a[0..m) in place, in three launches: each block
// of 1024 threads scans its chunk (wave shuffles, then the waves' totals) and
// records the chunk's total; one block scans those totals; every element
// then adds its chunk's offset.
__global__ __launch_bounds__(1024) void scan_chunks_kernel(uint32_t* a, int64_t m, uint32_t* totals) {
  __shared__ uint32_t wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t i = int64_t(blockIdx.x) * 1024 + tid;
  const uint32_t v = i < m ? a[i] : 0u;
  uint32_t s = v;  // inclusive scan within the wave
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(s, off, 64);
    if (lane >= off) s += t;
  }
  if (lane == 63) wsum[w] = s;
  __syncthreads();
  uint32_t before = 0;
  for (int k = 0; k < w; ++k) before += wsum[k];
  if (i < m) a[i] = before + s - v;
  if (tid == 1023) totals[blockIdx.x] = before + s;
}

__global__ __launch_bounds__(1024) void scan_totals_kernel(uint32_t* totals, int n) {
  // n <= 1024 * 64: each thread scans a run of consecutive totals
  __shared__ uint32_t part[1024];
  const int tid = threadIdx.x, per = (n + 1023) / 1024;
  const int b = tid * per, e = min(n, b + per);
  uint32_t sum = 0;
  for (int k = b; k < e; ++k) sum += totals[k];
  part[tid] = sum;
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int k = 0; k < 1024; ++k) {
      const uint32_t x = part[k];
      part[k] = run;
      run += x;
    }
  }
  __syncthreads();
  uint32_t run = part[tid];
  for (int k = b; k < e; ++k) {
    const uint32_t x = totals[k];
    totals[k] = run;
    run += x;
  }
}

__global__ void scan_add_kernel(uint32_t* a, int64_t m, const uint32_t* totals) {
  const int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  if (i < m) a[i] += totals[blockIdx.x];
}

// Stable scatter of one pass.  Each block walks its tile in chunks of 256
// keys (one per thread, in order); a key's place is its digit's running base
// for the block + the counts of its digit in lower waves of the chunk + its
// rank among the lanes of its wave with the same digit (found with ballots).
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const u64* __restrict__ kin, const int32_t* __restrict__ vin, int64_t n, int shift,
    const uint32_t* __restrict__ hist, int nblk, u64* __restrict__ kout, int32_t* __restrict__ vout) {
  constexpr int NW = kThreads / 64;
  __shared__ uint32_t base[kThreads];
  __shared__ uint32_t wcnt[NW][kThreads];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  base[tid] = hist[int64_t(tid) * nblk + blockIdx.x];
  const int64_t t0 = int64_t(blockIdx.x) * kTile;
  for (int k = 0; k < kItems; ++k) {
#pragma unroll
    for (int q = 0; q < NW; ++q) wcnt[q][tid] = 0;
    __syncthreads();
    const int64_t i = t0 + k * kThreads + tid;
    const bool valid = i < n;  // invalid lanes only follow valid ones
    const u64 key = valid ? kin[i] : ~0ull;
    const int32_t val = valid ? vin[i] : 0;
    const uint32_t d = unsigned(key >> shift) & 255u;
    unsigned long long peers = ~0ull;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const unsigned long long lower = peers & ((1ull << lane) - 1ull);
    if (lower == 0ull) wcnt[w][d] = uint32_t(__popcll(peers));
    __syncthreads();
    uint32_t pos = base[d] + uint32_t(__popcll(lower));
    for (int q = 0; q < w; ++q) pos += wcnt[q][d];
    if (valid) {
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) add += wcnt[q][tid];
    base[tid] += add;
    __syncthreads();
  }
}

// Sorted raw coordinates of every sorted point.
__global__ void gather_sorted_kernel(const double* __restrict__ xyz, const int32_t* __restrict__ perm, int64_t n,
                                     double* __restrict__ sorted_xyz) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = perm[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) sorted_xyz[3 * i + d] = xyz[3 * j + d];
}


__device__ inline int64_t lower_bound_u64(const u64* a, int64_t n, u64 v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}


template <class T>
T* dalloc(std::vector<void*>& owned, size_t count) {
  alloc_hook("hipMalloc");
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) raise(KIFMM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  owned.push_back(p);
  return static_cast<T*>(p);
}

// Exclusive scan of a[0..m) in place (three launches); totals holds
// (m + 1023) / 1024 words, at most 1024 * 64 of them.
inline void scan_exclusive(uint32_t* a, int64_t m, uint32_t* totals, hipStream_t s) {
  if (m <= 0) return;
  const int nchunk = int((m + 1023) / 1024);
  if (nchunk > 1024 * 64) raise(KIFMM_EUNSUPPORTED, "scan: too many entries");
  hipLaunchKernelGGL(scan_chunks_kernel, dim3(unsigned(nchunk)), dim3(1024), 0, s, a, m, totals);
  LAUNCHCHECK("scan_chunks_kernel");
  hipLaunchKernelGGL(scan_totals_kernel, dim3(1), dim3(1024), 0, s, totals, nchunk);
  LAUNCHCHECK("scan_totals_kernel");
  hipLaunchKernelGGL(scan_add_kernel, dim3(unsigned(nchunk)), dim3(1024), 0, s, a, m, totals);
  LAUNCHCHECK("scan_add_kernel");
}

// Stable sort of n (key, value) pairs on the low `bits` bits of the keys, 8
// bits per pass, ping-ponging between (k0, v0) and (k1, v1); hist holds
// 256 * ceil(n / kTile) words and totals that many / 1024 (rounded up).
// Returns true if the sorted pairs ended in (k1, v1).
inline bool radix_sort_pairs(u64* k0, int32_t* v0, u64* k1, int32_t* v1, int64_t n, int bits, uint32_t* hist,
                             uint32_t* totals, hipStream_t s) {
  if (n <= 0) return false;
  const int nblk = int((n + kTile - 1) / kTile);
  const int64_t m = int64_t(kThreads) * nblk;
  const int passes = (bits + 7) / 8;
  u64 *kin = k0, *kout = k1;
  int32_t *vin = v0, *vout = v1;
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nblk), dim3(kThreads), 0, s, kin, n, 8 * p, hist, nblk);
    LAUNCHCHECK("radix_hist_kernel");
    scan_exclusive(hist, m, totals, s);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblk), dim3(kThreads), 0, s, kin, vin, n, 8 * p, hist, nblk,
                       kout, vout);
    LAUNCHCHECK("radix_scatter_kernel");
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  return kin == k1;
}

}  // namespace
}  // namespace kifmm
