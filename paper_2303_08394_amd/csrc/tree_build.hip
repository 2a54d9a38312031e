// The octree and its interaction lists built on the GPU from device
// coordinates (section "Data-oriented design of PyExaFMM": a linear octree
// whose points are sorted by Morton key and whose boxes are ranges of that
// order; the U, V, W, X lists of section "Computational structure of FMM
// operators", defined as in Ying et al. 2004).  The result equals the host
// build (build_host_tree) integer for integer: keys, point order, boxes,
// numbering and lists.
//
//   root        min / max of the coordinates reduced on the device, the root
//               box then derived by the host's own rule (set_tree_root);
//   keys, order key_kernel and the stable radix sort of keys_sort.hpp;
//   refinement  level by level: a box splits by the host's rule; its
//               non-empty children are found by binary search of their key
//               ranges in the sorted keys and compacted by a scan, so every
//               level stays in Morton order;
//   balance     finest level first, as on the host: every leaf of the level
//               looks up its 26 neighbour cells (the deepest existing box
//               holding each, by binary search per level); a leaf more than
//               one level coarser is split, and the lookup repeats until no
//               leaf is split;
//   numbering   level by level, Morton order within a level;
//   lists       one thread per box enumerates its lists as the host does
//               (the same candidates and tests; the descent into finer
//               boxes without a stack), in a counting pass and a filling
//               pass, then sorts each of its slices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "device.hpp"
#include "hip_check.hpp"
#include "host_tree.hpp"
#include "keys_sort.hpp"

namespace kifmm {
namespace {

constexpr int kMaxLevels = 21;  // levels 0..20

__device__ inline u64 compact3(u64 v) {  // every third bit of v -> the low 21 bits
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
  v = (v ^ (v >> 32)) & 0x1fffffull;
  return v;
}

// Per-block minima, maxima and non-finite count of n points [n][3]:
// part[block] = (mn x, y, z, mx x, y, z, count, unused).
__global__ __launch_bounds__(256) void minmax_kernel(const double* __restrict__ xyz, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double s[8][256];
  const int tid = threadIdx.x;
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  double bad = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + tid; i < n; i += int64_t(gridDim.x) * 256)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double v = xyz[3 * i + d];
      if (!isfinite(v)) {
        bad += 1.0;
      } else {
        mn[d] = fmin(mn[d], v);
        mx[d] = fmax(mx[d], v);
      }
    }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    s[d][tid] = mn[d];
    s[3 + d][tid] = mx[d];
  }
  s[6][tid] = bad;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        s[d][tid] = fmin(s[d][tid], s[d][tid + h]);
        s[3 + d][tid] = fmax(s[3 + d][tid], s[3 + d][tid + h]);
      }
      s[6][tid] += s[6][tid + h];
    }
    __syncthreads();
  }
  if (tid < 8) part[8 * blockIdx.x + tid] = tid < 7 ? s[tid][0] : 0.0;
}

// The boxes of one level during refinement and balance: Morton code at the
// level (ascending), source and target ranges, leaf flag, and a mark used by
// the split passes.
struct Level {
  int64_t n = 0;
  u64* code = nullptr;
  int32_t *sb = nullptr, *se = nullptr, *tb = nullptr, *te = nullptr;
  int32_t *leaf = nullptr, *mark = nullptr;
};

// Split flags of refinement (the host's rule): uniform trees split every box
// above the depth; adaptive ones boxes holding more than ncrit sources or
// more than ncrit targets, above max_depth.
__global__ void want_split_kernel(int64_t n, int l, int uniform_depth, int ncrit, int max_depth,
                                  const int32_t* __restrict__ sb, const int32_t* __restrict__ se,
                                  const int32_t* __restrict__ tb, const int32_t* __restrict__ te,
                                  int32_t* __restrict__ want, int32_t* __restrict__ leaf) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool w = uniform_depth >= 0 ? l < uniform_depth
                                    : ((se[i] - sb[i] > ncrit || te[i] - tb[i] > ncrit) && l < max_depth);
  want[i] = w ? 1 : 0;
  leaf[i] = w ? 0 : 1;
}

__device__ inline int32_t lower_bound_in(const u64* __restrict__ a, int32_t b, int32_t e, u64 v) {
  while (b < e) {
    const int32_t mid = b + ((e - b) >> 1);
    if (a[mid] < v) b = mid + 1;
    else e = mid;
  }
  return b;
}

// Candidate children (8 per box) of the boxes whose flag is set: their key
// ranges in the sorted sources and targets; cnt = 1 for a non-empty child.
__global__ void child_ranges_kernel(int64_t n, int l, int L, const u64* __restrict__ code,
                                    const int32_t* __restrict__ sb, const int32_t* __restrict__ se,
                                    const int32_t* __restrict__ tb, const int32_t* __restrict__ te,
                                    const int32_t* __restrict__ flag, const u64* __restrict__ skey,
                                    const u64* __restrict__ tkey, int4* __restrict__ rng,
                                    uint32_t* __restrict__ cnt) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= 8 * n) return;
  const int64_t i = g >> 3;
  if (!flag[i]) {
    cnt[g] = 0;
    return;
  }
  const u64 m = (code[i] << 3) | u64(g & 7);
  const int sh = 3 * (L - l - 1);
  const u64 klo = m << sh, khi = (m + 1) << sh;
  const int32_t s0 = lower_bound_in(skey, sb[i], se[i], klo);
  const int32_t s1 = lower_bound_in(skey, s0, se[i], khi);
  const int32_t t0 = lower_bound_in(tkey, tb[i], te[i], klo);
  const int32_t t1 = lower_bound_in(tkey, t0, te[i], khi);
  rng[g] = make_int4(s0, s1, t0, t1);
  cnt[g] = (s1 > s0 || t1 > t0) ? 1u : 0u;
}

// Non-empty candidates to their places (pos: exclusive scan of the
// candidates' counts) in the child level's arrays, from entry `base` on; new
// boxes are leaves.  A candidate is taken if the scan advances after it; the
// last one is placed by child_last_kernel.
__global__ void child_scatter_kernel(int64_t n8, const u64* __restrict__ code, const int4* __restrict__ rng,
                                     const uint32_t* __restrict__ pos, int64_t base, Level out) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= n8 - 1 || pos[g + 1] == pos[g]) return;
  const int4 r = rng[g];
  const int64_t j = base + pos[g];
  out.code[j] = (code[g >> 3] << 3) | u64(g & 7);
  out.sb[j] = r.x;
  out.se[j] = r.y;
  out.tb[j] = r.z;
  out.te[j] = r.w;
  out.leaf[j] = 1;
  out.mark[j] = 0;
}

// The last candidate, whose emptiness the scan alone does not show (cnt_last:
// its count, copied before the scan).
__global__ void child_last_kernel(int64_t n8, const u64* __restrict__ code, const int4* __restrict__ rng,
                                  const uint32_t* __restrict__ pos, const uint32_t* __restrict__ cnt_last,
                                  int64_t base, Level out) {
  if (threadIdx.x != 0 || *cnt_last == 0) return;
  const int64_t g = n8 - 1;
  const int4 r = rng[g];
  const int64_t j = base + pos[g];
  out.code[j] = (code[g >> 3] << 3) | u64(g & 7);
  out.sb[j] = r.x;
  out.se[j] = r.y;
  out.tb[j] = r.z;
  out.te[j] = r.w;
  out.leaf[j] = 1;
  out.mark[j] = 0;
}

__global__ void copy_last_kernel(const uint32_t* __restrict__ a, int64_t i, uint32_t* __restrict__ out) {
  if (threadIdx.x == 0) *out = a[i];
}

// The tables of all levels, for lookups across levels.
struct LevelTable {
  const u64* code[kMaxLevels];
  int32_t* leaf[kMaxLevels];
  int32_t* mark[kMaxLevels];
  int32_t n[kMaxLevels];
};

__device__ inline int32_t find_code(const u64* __restrict__ a, int32_t n, u64 v) {
  const int32_t p = lower_bound_in(a, 0, n, v);
  return (p < n && a[p] == v) ? p : -1;
}

// Balance at level l: every leaf of the level looks up its 26 neighbour
// cells; the deepest existing box holding a cell, if a leaf more than one
// level coarser, is marked for splitting.
__global__ void balance_mark_kernel(LevelTable T, int l, unsigned* __restrict__ any) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T.n[l] || !T.leaf[l][i]) return;
  const u64 m = T.code[l][i];
  const int64_t ax = int64_t(compact3(m >> 2)), ay = int64_t(compact3(m >> 1)), az = int64_t(compact3(m));
  const int64_t side = int64_t(1) << l;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        if (!dx && !dy && !dz) continue;
        const int64_t nx = ax + dx, ny = ay + dy, nz = az + dz;
        if (nx < 0 || ny < 0 || nz < 0 || nx >= side || ny >= side || nz >= side) continue;
        const u64 cell = morton3(u64(nx), u64(ny), u64(nz));
        int k = l - 1, c = -1;
        for (; k >= 0; --k) {
          c = find_code(T.code[k], T.n[k], cell >> (3 * (l - k)));
          if (c >= 0) break;
        }
        if (c < 0 || k >= l - 1 || !T.leaf[k][c]) continue;
        T.mark[k][c] = 1;
        atomicOr(any, 1u);
      }
}

// Boxes split by balance stop being leaves.
__global__ void unleaf_marked_kernel(int64_t n, const int32_t* __restrict__ mark, int32_t* __restrict__ leaf) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && mark[i]) leaf[i] = 0;
}

__global__ void iota_kernel(int32_t* __restrict__ v, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) v[i] = int32_t(i);
}

// Entries of a level in the order `idx` (after sorting its codes).
__global__ void gather_level_kernel(int64_t n, const int32_t* __restrict__ idx, Level in, Level out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t k = idx[i];
  out.code[i] = in.code[k];
  out.sb[i] = in.sb[k];
  out.se[i] = in.se[k];
  out.tb[i] = in.tb[k];
  out.te[i] = in.te[k];
  out.leaf[i] = in.leaf[k];
  out.mark[i] = 0;
}

// The final box table: all levels back to back (level-major, Morton order
// inside a level); lookups of (level, code) by binary search inside the level.
struct Boxes {
  int32_t nbox = 0, depth = 0;
  int32_t start[kMaxLevels + 1];  // first box of each level, start[depth + 1] = nbox
  const u64* code;
  const int32_t *sb, *se, *tb, *te, *leaf;
  int32_t *level, *parent, *octant, *anchor, *child_begin, *child_count;
};

__device__ inline int32_t find_box(const Boxes& B, int l, int64_t x, int64_t y, int64_t z) {
  if (l > B.depth) return -1;
  const int64_t n = int64_t(1) << l;
  if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return -1;
  const int32_t b = B.start[l], e = B.start[l + 1];
  const u64 v = morton3(u64(x), u64(y), u64(z));
  const int32_t p = lower_bound_in(B.code, b, e, v);
  return (p < e && B.code[p] == v) ? p : -1;
}

// Level, parent, octant, anchor and children of every box.
__global__ void finalize_kernel(Boxes B) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= B.nbox) return;
  int l = 0;
  while (B.start[l + 1] <= g) ++l;
  const u64 m = B.code[g];
  B.level[g] = l;
  B.octant[g] = int32_t(m & 7);
  B.anchor[3 * g] = int32_t(compact3(m >> 2));
  B.anchor[3 * g + 1] = int32_t(compact3(m >> 1));
  B.anchor[3 * g + 2] = int32_t(compact3(m));
  B.parent[g] = l == 0 ? -1 : lower_bound_in(B.code, B.start[l - 1], B.start[l], m >> 3);
  if (l < B.depth) {
    const int32_t b = lower_bound_in(B.code, B.start[l + 1], B.start[l + 2], m << 3);
    const int32_t e = lower_bound_in(B.code, b, B.start[l + 2], (m + 1) << 3);
    B.child_begin[g] = e > b ? b : -1;
    B.child_count[g] = e - b;
  } else {
    B.child_begin[g] = -1;
    B.child_count[g] = 0;
  }
}

__device__ inline bool adjacent_boxes(const Boxes& B, int32_t a, int32_t b) {
  const int la = B.level[a], lb = B.level[b];
  const int L = max(la, lb);
  const int64_t sa = int64_t(1) << (L - la), sbb = int64_t(1) << (L - lb);
  for (int d = 0; d < 3; ++d) {
    const int64_t alo = int64_t(B.anchor[3 * a + d]) * sa, blo = int64_t(B.anchor[3 * b + d]) * sbb;
    if (max(alo, blo) > min(alo + sa, blo + sbb)) return false;
  }
  return true;
}

struct ListOut {
  uint32_t* cnt;        // [4][nbox] (counting pass)
  const uint32_t* off;  // [4][nbox] exclusive scans of cnt (filling pass)
  int32_t* items[4];
};

// The lists of box g, as the host enumerates them; FILL writes them at their
// offsets and sorts each slice, otherwise only their lengths are counted.
template <bool FILL>
__global__ void lists_kernel(Boxes B, ListOut o) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= B.nbox) return;
  uint32_t n[4] = {0u, 0u, 0u, 0u};
  const int64_t nb = B.nbox;
  auto emit = [&](int k, int32_t c) {
    if constexpr (FILL) o.items[k][o.off[k * nb + g] + n[k]] = c;
    ++n[k];
  };
  auto nsrc = [&](int32_t c) { return B.se[c] - B.sb[c]; };
  if (B.te[g] > B.tb[g]) {  // no targets below the box: no lists
    const int l = B.level[g];
    const int64_t a[3] = {B.anchor[3 * g], B.anchor[3 * g + 1], B.anchor[3 * g + 2]};
    if (B.leaf[g]) {
      // U: coarser or same-level leaves touching the box (the box included)
      for (int l2 = 0; l2 <= l; ++l2) {
        const int64_t s = int64_t(1) << (l - l2), n2 = int64_t(1) << l2;
        int64_t lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
          lo[d] = max((a[d] + s - 1) / s - 1, int64_t(0));
          hi[d] = min((a[d] + 1) / s, n2 - 1);
        }
        for (int64_t x = lo[0]; x <= hi[0]; ++x)
          for (int64_t y = lo[1]; y <= hi[1]; ++y)
            for (int64_t z = lo[2]; z <= hi[2]; ++z) {
              const int32_t c = find_box(B, l2, x, y, z);
              if (c >= 0 && B.leaf[c] && nsrc(c) > 0) emit(0, c);
            }
      }
      // finer boxes: the subtrees of the non-leaf colleagues, descended while
      // they touch the box (leaves that touch it: U; boxes that do not: W).
      // Depth first without a stack: children are contiguous, so the next
      // box is the first child, else the next sibling of the box or of its
      // nearest ancestor below the colleague.
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            if (!dx && !dy && !dz) continue;
            const int32_t c = find_box(B, l, a[0] + dx, a[1] + dy, a[2] + dz);
            if (c < 0 || B.leaf[c]) continue;
            int32_t d = B.child_begin[c];
            while (d >= 0) {
              bool down = false;
              if (nsrc(d) > 0) {
                if (adjacent_boxes(B, d, g)) {
                  if (B.leaf[d]) emit(0, d);
                  else down = true;
                } else {
                  emit(2, d);
                }
              }
              if (down) {
                d = B.child_begin[d];
                continue;
              }
              for (;;) {
                const int32_t p = B.parent[d];
                if (d + 1 < B.child_begin[p] + B.child_count[p]) {
                  ++d;
                  break;
                }
                if (p == c) {
                  d = -1;
                  break;
                }
                d = p;
              }
            }
          }
    }
    if (l >= 2) {
      // V: children of the parent's colleagues not touching the box
      const int32_t P = B.parent[g];
      const int64_t pa[3] = {B.anchor[3 * P], B.anchor[3 * P + 1], B.anchor[3 * P + 2]};
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            const int32_t c = find_box(B, l - 1, pa[0] + dx, pa[1] + dy, pa[2] + dz);
            if (c < 0) continue;
            for (int k = 0; k < B.child_count[c]; ++k) {
              const int32_t A = B.child_begin[c] + k;
              if (nsrc(A) > 0 && !adjacent_boxes(B, A, g)) emit(1, A);
            }
          }
    }
    if (l >= 1) {
      // X: leaves coarser than the box touching its parent but not the box
      const int32_t P = B.parent[g];
      const int64_t pa[3] = {B.anchor[3 * P], B.anchor[3 * P + 1], B.anchor[3 * P + 2]};
      const int lp = l - 1;
      for (int l2 = 0; l2 <= lp; ++l2) {
        const int64_t s = int64_t(1) << (lp - l2), n2 = int64_t(1) << l2;
        int64_t lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
          lo[d] = max((pa[d] + s - 1) / s - 1, int64_t(0));
          hi[d] = min((pa[d] + 1) / s, n2 - 1);
        }
        for (int64_t x = lo[0]; x <= hi[0]; ++x)
          for (int64_t y = lo[1]; y <= hi[1]; ++y)
            for (int64_t z = lo[2]; z <= hi[2]; ++z) {
              const int32_t c = find_box(B, l2, x, y, z);
              if (c >= 0 && B.leaf[c] && nsrc(c) > 0 && !adjacent_boxes(B, c, g)) emit(3, c);
            }
      }
    }
  }
  if constexpr (!FILL) {
    for (int k = 0; k < 4; ++k) o.cnt[k * nb + g] = n[k];
  } else {
    // each slice in ascending box order, as the host sorts it
    for (int k = 0; k < 4; ++k) {
      int32_t* v = o.items[k] + o.off[k * nb + g];
      for (uint32_t i = 1; i < n[k]; ++i) {
        const int32_t x = v[i];
        uint32_t j = i;
        for (; j > 0 && v[j - 1] > x; --j) v[j] = v[j - 1];
        v[j] = x;
      }
    }
  }
}

// Device arrays owned by one build, freed together.
struct Pool {
  std::vector<void*> owned;
  template <class T>
  T* get(int64_t count) {
    alloc_hook("build_tree_device");
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, size_t(std::max<int64_t>(count, 1)) * sizeof(T));
    if (e != hipSuccess) raise(KIFMM_ENOMEM, std::string("build_tree_device: hipMalloc: ") + hipGetErrorString(e));
    owned.push_back(p);
    return static_cast<T*>(p);
  }
  ~Pool() {
    for (void* p : owned) (void)hipFree(p);
  }
};

inline unsigned blocks(int64_t n, int t = 256) { return unsigned(std::max<int64_t>((n + t - 1) / t, 1)); }

Level alloc_level(Pool& P, int64_t n) {
  Level v;
  v.n = n;
  v.code = P.get<u64>(n);
  v.sb = P.get<int32_t>(n);
  v.se = P.get<int32_t>(n);
  v.tb = P.get<int32_t>(n);
  v.te = P.get<int32_t>(n);
  v.leaf = P.get<int32_t>(n);
  v.mark = P.get<int32_t>(n);
  return v;
}

// Sorted keys, order and coordinates of one point set.
struct SortedPoints {
  u64* key = nullptr;
  int32_t* perm = nullptr;
  double* xyz = nullptr;
};

}  // namespace

HostTree* build_tree_device(const double* src, int64_t nsrc, const double* tgt, int64_t ntgt,
                            const kifmm_tree_params& prm, void* stream) {
  if (!src || !tgt) raise(KIFMM_EINVAL, "build_tree: null point array");
  validate_tree_params(nsrc, ntgt, prm);
  for (const double* p : {src, tgt}) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      raise(KIFMM_EINVAL, "build_tree_device: coordinates must be device memory");
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  Pool P;
  const bool same = tgt == src && ntgt == nsrc;

  // non-finite coordinates and the bounding box
  constexpr int kRedBlocks = 512;
  double* part = P.get<double>(8 * kRedBlocks);
  std::vector<double> hp(8 * kRedBlocks);
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = 0; k < (same ? 1 : 2); ++k) {
    const double* x = k == 0 ? src : tgt;
    const int64_t n = k == 0 ? nsrc : ntgt;
    hipLaunchKernelGGL(minmax_kernel, dim3(kRedBlocks), dim3(256), 0, s, x, n, part);
    LAUNCHCHECK("minmax_kernel");
    HIPCHECK(hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    double bad = 0;
    for (int b = 0; b < kRedBlocks; ++b) {
      for (int d = 0; d < 3; ++d) {
        mn[d] = std::min(mn[d], hp[8 * b + d]);
        mx[d] = std::max(mx[d], hp[8 * b + 3 + d]);
      }
      bad += hp[8 * b + 6];
    }
    if (bad > 0)
      raise(KIFMM_EINVAL, k == 0 ? "build_tree: non-finite source coordinate" : "build_tree: non-finite target coordinate");
  }
  auto Tp = std::make_unique<HostTree>();
  HostTree& T = *Tp;
  T.nsrc = nsrc;
  T.ntgt = ntgt;
  set_tree_root(T, prm, mn, mx);
  T.tgt_is_src = same;
  const int L = T.key_level;

  // keys and sorted order of each point set
  const int64_t nmax = std::max(nsrc, ntgt);
  const int nblk = int((nmax + kTile - 1) / kTile);
  const int64_t nhist = int64_t(kThreads) * std::max(nblk, 1);
  // (the sort's digit counts later serve the scans of the box candidates)
  const int64_t nscan = std::max<int64_t>(nhist, 16 * nmax + 8);
  uint32_t* hist = P.get<uint32_t>(nscan);
  uint32_t* totals = P.get<uint32_t>((nscan + 1023) / 1024);
  unsigned long long* outside = P.get<unsigned long long>(1);
  HIPCHECK(hipMemsetAsync(outside, 0, 8, s));
  u64* k0 = P.get<u64>(nmax);
  int32_t* v0 = P.get<int32_t>(nmax);
  SortedPoints sp[2];
  for (int k = 0; k < (same ? 1 : 2); ++k) {
    const double* x = k == 0 ? src : tgt;
    const int64_t n = k == 0 ? nsrc : ntgt;
    SortedPoints& o = sp[k];
    o.key = P.get<u64>(n);
    o.perm = P.get<int32_t>(n);
    o.xyz = P.get<double>(3 * n);
    Frame f;
    for (int d = 0; d < 3; ++d) f.lo[d] = T.lo[d];
    f.r0 = T.r0;
    f.L = L;
    hipLaunchKernelGGL(key_kernel, dim3(blocks(n)), dim3(256), 0, s, x, n, f, k0, v0, outside);
    LAUNCHCHECK("key_kernel");
    if (!radix_sort_pairs(k0, v0, o.key, o.perm, n, 3 * L, hist, totals, s)) {
      HIPCHECK(hipMemcpyAsync(o.key, k0, size_t(n) * 8, hipMemcpyDeviceToDevice, s));
      HIPCHECK(hipMemcpyAsync(o.perm, v0, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(gather_sorted_kernel, dim3(blocks(n)), dim3(256), 0, s, x, o.perm, n, o.xyz);
    LAUNCHCHECK("gather_sorted_kernel");
  }
  if (same) sp[1] = sp[0];
  if (prm.root_halfwidth > 0) {
    unsigned long long h = 0;
    HIPCHECK(hipMemcpyAsync(&h, outside, 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (h != 0) raise(KIFMM_EINVAL, "build_tree: a point lies outside the given root box");
  }

  // refinement, level by level
  std::vector<Level> lv;
  {
    Level root = alloc_level(P, 1);
    const u64 zero = 0;
    const int32_t r4[4] = {0, int32_t(nsrc), 0, int32_t(ntgt)};
    HIPCHECK(hipMemcpyAsync(root.code, &zero, 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(root.sb, &r4[0], 4, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(root.se, &r4[1], 4, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(root.tb, &r4[2], 4, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(root.te, &r4[3], 4, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemsetAsync(root.mark, 0, 4, s));
    lv.push_back(root);
  }
  // candidates: 8 per box of a level, and a level holds at most one box per
  // point (boxes are never empty)
  const int64_t max_cand = 16 * nmax + 8;
  int4* rng = P.get<int4>(max_cand);
  uint32_t* cnt = hist;  // (the sort is done: its scratch serves the scans)
  uint32_t* last = P.get<uint32_t>(1);
  // children of the boxes of level l whose `flag` is set, appended to level
  // l + 1 (created if absent); returns how many
  auto split_level = [&](int l, const int32_t* flag) -> int64_t {
    const Level& a = lv[l];
    const int64_t n8 = 8 * a.n;
    if (n8 > max_cand) raise(KIFMM_EINVAL, "build_tree_device: more boxes on a level than points");
    hipLaunchKernelGGL(child_ranges_kernel, dim3(blocks(n8)), dim3(256), 0, s, a.n, l, L, a.code, a.sb, a.se,
                       a.tb, a.te, flag, sp[0].key, sp[1].key, rng, cnt);
    LAUNCHCHECK("child_ranges_kernel");
    hipLaunchKernelGGL(copy_last_kernel, dim3(1), dim3(64), 0, s, cnt, n8 - 1, last);
    LAUNCHCHECK("copy_last_kernel");
    scan_exclusive(cnt, n8, totals, s);
    uint32_t h[2];
    HIPCHECK(hipMemcpyAsync(&h[0], cnt + n8 - 1, 4, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(&h[1], last, 4, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const int64_t added = int64_t(h[0]) + h[1];
    if (added == 0) return 0;
    const int64_t old = int(lv.size()) > l + 1 ? lv[l + 1].n : 0;
    Level nx = alloc_level(P, old + added);
    if (old > 0) {
      const Level& o = lv[l + 1];
      HIPCHECK(hipMemcpyAsync(nx.code, o.code, old * 8, hipMemcpyDeviceToDevice, s));
      for (auto pr : {std::make_pair(nx.sb, o.sb), std::make_pair(nx.se, o.se), std::make_pair(nx.tb, o.tb),
                      std::make_pair(nx.te, o.te), std::make_pair(nx.leaf, o.leaf)})
        HIPCHECK(hipMemcpyAsync(pr.first, pr.second, old * 4, hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(child_scatter_kernel, dim3(blocks(n8)), dim3(256), 0, s, n8, a.code, rng, cnt, old, nx);
    LAUNCHCHECK("child_scatter_kernel");
    hipLaunchKernelGGL(child_last_kernel, dim3(1), dim3(64), 0, s, n8, a.code, rng, cnt, last, old, nx);
    LAUNCHCHECK("child_last_kernel");
    if (old > 0) {
      // a level that gained boxes by balance: back into Morton order
      u64* kk = P.get<u64>(old + added);
      int32_t* ix = P.get<int32_t>(old + added);
      int32_t* iy = P.get<int32_t>(old + added);
      u64* ky = P.get<u64>(old + added);
      HIPCHECK(hipMemcpyAsync(kk, nx.code, (old + added) * 8, hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(iota_kernel, dim3(blocks(old + added)), dim3(256), 0, s, ix, old + added);
      LAUNCHCHECK("iota_kernel");
      const bool in_y = radix_sort_pairs(kk, ix, ky, iy, old + added, 3 * (l + 1), hist, totals, s);
      Level sorted = alloc_level(P, old + added);
      hipLaunchKernelGGL(gather_level_kernel, dim3(blocks(old + added)), dim3(256), 0, s, old + added,
                         in_y ? iy : ix, nx, sorted);
      LAUNCHCHECK("gather_level_kernel");
      nx = sorted;
    }
    if (int(lv.size()) > l + 1) lv[l + 1] = nx;
    else lv.push_back(nx);
    return added;
  };
  for (int l = 0;; ++l) {
    Level& a = lv[l];
    int32_t* want = P.get<int32_t>(a.n);
    hipLaunchKernelGGL(want_split_kernel, dim3(blocks(a.n)), dim3(256), 0, s, a.n, l, prm.uniform_depth, prm.ncrit,
                       prm.max_depth, a.sb, a.se, a.tb, a.te, want, a.leaf);
    LAUNCHCHECK("want_split_kernel");
    if (l >= L || split_level(l, want) == 0) break;
  }

  // 2:1 balance (adaptive trees), finest level first
  if (prm.uniform_depth < 0 && prm.balance) {
    unsigned* any = P.get<unsigned>(1);
    const int maxl = int(lv.size()) - 1;
    for (int l = maxl; l >= 2; --l) {
      for (;;) {
        LevelTable tab{};
        for (int k = 0; k < int(lv.size()); ++k) {
          tab.code[k] = lv[k].code;
          tab.leaf[k] = lv[k].leaf;
          tab.mark[k] = lv[k].mark;
          tab.n[k] = int32_t(lv[k].n);
          HIPCHECK(hipMemsetAsync(lv[k].mark, 0, size_t(lv[k].n) * 4, s));
        }
        HIPCHECK(hipMemsetAsync(any, 0, 4, s));
        hipLaunchKernelGGL(balance_mark_kernel, dim3(blocks(lv[l].n)), dim3(256), 0, s, tab, l, any);
        LAUNCHCHECK("balance_mark_kernel");
        unsigned h = 0;
        HIPCHECK(hipMemcpyAsync(&h, any, 4, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        if (!h) break;
        // split the marked leaves (levels l-2..0), deepest first: the marks of
        // a level are used before its arrays are replaced (re-sorted with the
        // children of the level above)
        for (int k = l - 2; k >= 0; --k) {
          split_level(k, lv[k].mark);
          hipLaunchKernelGGL(unleaf_marked_kernel, dim3(blocks(lv[k].n)), dim3(256), 0, s, lv[k].n, lv[k].mark,
                             lv[k].leaf);
          LAUNCHCHECK("unleaf_marked_kernel");
        }
      }
    }
  }

  // numbering: all levels back to back
  const int depth = int(lv.size()) - 1;
  int64_t nb64 = 0;
  for (auto& v : lv) nb64 += v.n;
  if (nb64 > (int64_t(1) << 31) - 1) raise(KIFMM_EUNSUPPORTED, "build_tree_device: too many boxes");
  const int32_t nb = int32_t(nb64);
  Boxes B{};
  B.nbox = nb;
  B.depth = depth;
  u64* gcode = P.get<u64>(nb);
  int32_t* g4[5];
  for (auto& p : g4) p = P.get<int32_t>(nb);
  {
    int64_t at = 0;
    for (int l = 0; l <= depth; ++l) {
      B.start[l] = int32_t(at);
      const Level& v = lv[l];
      HIPCHECK(hipMemcpyAsync(gcode + at, v.code, v.n * 8, hipMemcpyDeviceToDevice, s));
      const int32_t* srcs[5] = {v.sb, v.se, v.tb, v.te, v.leaf};
      for (int k = 0; k < 5; ++k) HIPCHECK(hipMemcpyAsync(g4[k] + at, srcs[k], v.n * 4, hipMemcpyDeviceToDevice, s));
      at += v.n;
    }
    for (int l = depth + 1; l <= kMaxLevels; ++l) B.start[l] = int32_t(at);
  }
  B.code = gcode;
  B.sb = g4[0];
  B.se = g4[1];
  B.tb = g4[2];
  B.te = g4[3];
  B.leaf = g4[4];
  B.level = P.get<int32_t>(nb);
  B.parent = P.get<int32_t>(nb);
  B.octant = P.get<int32_t>(nb);
  B.anchor = P.get<int32_t>(3 * int64_t(nb));
  B.child_begin = P.get<int32_t>(nb);
  B.child_count = P.get<int32_t>(nb);
  hipLaunchKernelGGL(finalize_kernel, dim3(blocks(nb)), dim3(256), 0, s, B);
  LAUNCHCHECK("finalize_kernel");

  // interaction lists: count, scan, fill (and sort)
  const int64_t n4 = 4 * int64_t(nb);
  uint32_t* lcnt = P.get<uint32_t>(n4);
  ListOut lo{};
  lo.cnt = lcnt;
  hipLaunchKernelGGL((lists_kernel<false>), dim3(blocks(nb, 128)), dim3(128), 0, s, B, lo);
  LAUNCHCHECK("lists_kernel");
  std::vector<uint32_t> counts(n4);
  HIPCHECK(hipMemcpyAsync(counts.data(), lcnt, n4 * 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  int64_t tot[4] = {0, 0, 0, 0};
  for (int k = 0; k < 4; ++k) {
    T.off[k].assign(nb + 1, 0);
    for (int32_t b = 0; b < nb; ++b) T.off[k][b + 1] = T.off[k][b] + counts[int64_t(k) * nb + b];
    tot[k] = T.off[k][nb];
    if (tot[k] > int64_t(UINT32_MAX)) raise(KIFMM_EUNSUPPORTED, "build_tree_device: interaction list too long");
  }
  {
    // per-list exclusive offsets as 32-bit words for the filling pass
    std::vector<uint32_t> offs(n4);
    for (int k = 0; k < 4; ++k)
      for (int32_t b = 0; b < nb; ++b) offs[int64_t(k) * nb + b] = uint32_t(T.off[k][b]);
    HIPCHECK(hipMemcpyAsync(lcnt, offs.data(), n4 * 4, hipMemcpyHostToDevice, s));
    lo.off = lcnt;
    for (int k = 0; k < 4; ++k) lo.items[k] = P.get<int32_t>(tot[k]);
    hipLaunchKernelGGL((lists_kernel<true>), dim3(blocks(nb, 128)), dim3(128), 0, s, B, lo);
    LAUNCHCHECK("lists_kernel");
    for (int k = 0; k < 4; ++k) {
      T.items[k].resize(tot[k]);
      if (tot[k]) HIPCHECK(hipMemcpyAsync(T.items[k].data(), lo.items[k], tot[k] * 4, hipMemcpyDeviceToHost, s));
    }
    HIPCHECK(hipStreamSynchronize(s));  // (offs stays alive until here)
  }

  // the host copy
  T.nbox = nb;
  T.depth = depth;
  auto down32 = [&](std::vector<int32_t>& v, const int32_t* d, int64_t n) {
    v.resize(n);
    HIPCHECK(hipMemcpyAsync(v.data(), d, n * 4, hipMemcpyDeviceToHost, s));
  };
  down32(T.level, B.level, nb);
  down32(T.parent, B.parent, nb);
  down32(T.octant, B.octant, nb);
  down32(T.leaf, B.leaf, nb);
  down32(T.anchor, B.anchor, 3 * int64_t(nb));
  down32(T.child_begin, B.child_begin, nb);
  down32(T.child_count, B.child_count, nb);
  std::vector<int32_t> r4[4];
  down32(r4[0], B.sb, nb);
  down32(r4[1], B.se, nb);
  down32(r4[2], B.tb, nb);
  down32(r4[3], B.te, nb);
  std::vector<int32_t> perm32[2];
  for (int k = 0; k < 2; ++k) {
    const int64_t n = k == 0 ? nsrc : ntgt;
    down32(perm32[k], sp[k].perm, n);
    (k == 0 ? T.skey : T.tkey).resize(n);
    HIPCHECK(hipMemcpyAsync((k == 0 ? T.skey : T.tkey).data(), sp[k].key, n * 8, hipMemcpyDeviceToHost, s));
    (k == 0 ? T.sxyz : T.txyz).resize(3 * n);
    HIPCHECK(hipMemcpyAsync((k == 0 ? T.sxyz : T.txyz).data(), sp[k].xyz, 3 * n * 8, hipMemcpyDeviceToHost, s));
  }
  HIPCHECK(hipStreamSynchronize(s));
  T.sbeg.assign(r4[0].begin(), r4[0].end());
  T.send.assign(r4[1].begin(), r4[1].end());
  T.tbeg.assign(r4[2].begin(), r4[2].end());
  T.tend.assign(r4[3].begin(), r4[3].end());
  T.sperm.assign(perm32[0].begin(), perm32[0].end());
  T.tperm.assign(perm32[1].begin(), perm32[1].end());
  T.level_start.assign(depth + 2, 0);
  for (int l = 0; l <= depth + 1; ++l) T.level_start[l] = B.start[l];
  T.leaves.clear();
  for (int32_t g = 0; g < nb; ++g)
    if (T.leaf[g]) T.leaves.push_back(g);
  return Tp.release();
}

}  // namespace kifmm
