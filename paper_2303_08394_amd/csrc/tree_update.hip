// New point positions sorted into an existing tree on the GPU: the part of
// the tree build that depends on the points (section "Data-oriented design":
// the linear octree keeps its points sorted by the Morton key of their leaf,
// and boxes as ranges of that order).  While every point stays in a leaf of
// its kind (sources, targets) that was occupied before, and no occupied leaf
// empties, the boxes, interaction lists and tile plans do not change; only
// the point order, the leaf-relative coordinates and the box ranges do.
// Every rule follows the host build exactly (FP64, no contraction).
//
//   key      clamp(floor(t * 2^L), 0, 2^L - 1) per axis, t = (x - lo) / (2 r0),
//            interleaved x-major at the key level L (the uniform depth, or the
//            maximum depth of an adaptive tree: up to 60 bits);
//   order    stable LSD radix sort of the keys, 8 bits per pass, ties in the
//            caller's order;
//   ranges   box b at level l holds the keys [m << 3(L-l), (m+1) << 3(L-l))
//            of its Morton code m;
//   frame    (x - c) / r of the leaf's centre c and half-width r.
#include <hip/hip_runtime.h>

#include <algorithm>
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

// Leaf-frame coordinates (x - c) / r of the points of each leaf (one block
// per leaf box; c and r from its anchor and level, as the host computes them).
__global__ void leaf_frame_kernel(const int32_t* __restrict__ leaves, const int32_t* __restrict__ anchor,
                                  const int32_t* __restrict__ level, const int2* __restrict__ ranges, Frame f,
                                  const double* __restrict__ sorted_xyz, double4* __restrict__ rel) {
#pragma clang fp contract(off)
  const int g = leaves[blockIdx.x];
  const int2 rg = ranges[g];
  const double r = f.r0 / double(int64_t(1) << level[g]);
  double c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) c[d] = f.lo[d] + (2.0 * double(anchor[3 * g + d]) + 1.0) * r;
  for (int i = rg.x + threadIdx.x; i < rg.y; i += blockDim.x)
    rel[i] = make_double4((sorted_xyz[3 * i] - c[0]) / r, (sorted_xyz[3 * i + 1] - c[1]) / r,
                          (sorted_xyz[3 * i + 2] - c[2]) / r, 0.0);
}

// New point range of every box; flags a leaf whose emptiness changed (occ:
// 1 for the leaves that held points of this kind) and counts the points that
// fall in leaves.
__global__ void ranges_kernel(const int32_t* __restrict__ anchor, const int32_t* __restrict__ level,
                              const int32_t* __restrict__ is_leaf, const uint8_t* __restrict__ occ,
                              int32_t nbox, int L, const u64* __restrict__ skeys, int64_t n,
                              int2* __restrict__ out, unsigned* __restrict__ flag,
                              unsigned long long* __restrict__ in_leaves) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nbox) return;
  const int l = level[g];
  const u64 m = morton3(u64(anchor[3 * g]), u64(anchor[3 * g + 1]), u64(anchor[3 * g + 2]));
  const int sh = 3 * (L - l);
  const int64_t b = lower_bound_u64(skeys, n, m << sh);
  const int64_t e = lower_bound_u64(skeys, n, (m + 1) << sh);
  out[g] = make_int2(int(b), int(e));
  if (is_leaf[g]) {
    if ((e > b) != (occ[g] != 0)) atomicOr(flag, 1u);
    atomicAdd(in_leaves, (unsigned long long)(e - b));
  }
}


}  // namespace

// One sorted point set.
struct SortedSet {
  u64* keys = nullptr;         // [n] sorted leaf keys
  int32_t* perm = nullptr;     // [n] sorted position -> caller index
  double* xyz = nullptr;       // [n][3] sorted coordinates
  double4* rel = nullptr;      // [n] leaf-frame coordinates
  int2* ranges = nullptr;      // [nbox]
};

// Per-tree device state of the re-sort, kept between updates: the tree's box
// table and leaf occupancy (uploaded once), sort scratch, and two output sets
// per kind, so that a rejected update leaves the last accepted one intact.
struct PendingPoints {
  int device = -1;
  int32_t nbox = 0;
  int64_t nsrc = 0, ntgt = 0;
  int nleaves = 0, nblk = 0, nchunk = 0;
  int32_t *anchor = nullptr, *level = nullptr, *leaf = nullptr, *leaves = nullptr;
  uint8_t *occ_src = nullptr, *occ_tgt = nullptr;
  u64* k0 = nullptr;
  int32_t* v0 = nullptr;
  uint32_t *hist = nullptr, *totals = nullptr;
  unsigned long long* stat = nullptr;  // [4]: flag, source count, target count, points outside the root
  SortedSet src[2], tgt[2];
  int cur = -1;             // output set of the last accepted update
  bool stale_host = false;  // the host copy of the tree lags set `cur`
  bool tgt_sep = false;     // set `cur` has its own targets
  std::vector<void*> allocs;
  ~PendingPoints() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

static void alloc_set(PendingPoints& P, SortedSet& S, int64_t n) {
  S.keys = dalloc<u64>(P.allocs, n);
  S.perm = dalloc<int32_t>(P.allocs, n);
  S.xyz = dalloc<double>(P.allocs, size_t(n) * 3);
  S.rel = dalloc<double4>(P.allocs, n);
  S.ranges = dalloc<int2>(P.allocs, P.nbox);
}

PendingPoints* sort_state_create(const HostTree& T) {
  auto P = std::make_unique<PendingPoints>();
  P->device = current_device();
  P->nbox = T.nbox;
  P->nsrc = T.nsrc;
  P->ntgt = T.ntgt;
  const int64_t nmax = std::max(T.nsrc, T.ntgt);
  P->nblk = int((nmax + kTile - 1) / kTile);
  const int64_t m = int64_t(kThreads) * P->nblk;
  P->nchunk = int((m + 1023) / 1024);
  if (P->nchunk > 1024 * 64) raise(KIFMM_EUNSUPPORTED, "update_points: too many points for one sort");
  std::vector<int32_t> isleaf(T.leaf.begin(), T.leaf.end()), leaves;
  std::vector<uint8_t> os(T.nbox, 0), ot(T.nbox, 0);
  for (int32_t g = 0; g < T.nbox; ++g) {
    if (T.leaf[g]) leaves.push_back(g);
    os[g] = T.send[g] > T.sbeg[g] ? 1 : 0;
    ot[g] = T.tend[g] > T.tbeg[g] ? 1 : 0;
  }
  P->nleaves = int(leaves.size());
  P->anchor = dalloc<int32_t>(P->allocs, T.anchor.size());
  P->level = dalloc<int32_t>(P->allocs, T.level.size());
  P->leaf = dalloc<int32_t>(P->allocs, isleaf.size());
  P->leaves = dalloc<int32_t>(P->allocs, leaves.size());
  P->occ_src = dalloc<uint8_t>(P->allocs, os.size());
  P->occ_tgt = dalloc<uint8_t>(P->allocs, ot.size());
  HIPCHECK(hipMemcpy(P->anchor, T.anchor.data(), T.anchor.size() * 4, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(P->level, T.level.data(), T.level.size() * 4, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(P->leaf, isleaf.data(), isleaf.size() * 4, hipMemcpyHostToDevice));
  if (!leaves.empty()) HIPCHECK(hipMemcpy(P->leaves, leaves.data(), leaves.size() * 4, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(P->occ_src, os.data(), os.size(), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(P->occ_tgt, ot.data(), ot.size(), hipMemcpyHostToDevice));
  P->k0 = dalloc<u64>(P->allocs, nmax);
  P->v0 = dalloc<int32_t>(P->allocs, nmax);
  P->hist = dalloc<uint32_t>(P->allocs, size_t(m));
  P->totals = dalloc<uint32_t>(P->allocs, P->nchunk);
  P->stat = dalloc<unsigned long long>(P->allocs, 4);
  for (int k = 0; k < 2; ++k) alloc_set(*P, P->src[k], T.nsrc);
  return P.release();
}

static void sort_set(PendingPoints& P, const HostTree& T, const double* xyz, int64_t n, const uint8_t* occ,
                     hipStream_t s, SortedSet& S, unsigned long long* d_count) {
  Frame f;
  for (int d = 0; d < 3; ++d) f.lo[d] = T.lo[d];
  f.r0 = T.r0;
  f.L = T.key_level;
  const unsigned grid = unsigned((n + 255) / 256);
  hipLaunchKernelGGL(key_kernel, dim3(grid), dim3(256), 0, s, xyz, n, f, P.k0, P.v0, P.stat + 3);
  LAUNCHCHECK("key_kernel");
  const bool in_set = radix_sort_pairs(P.k0, P.v0, S.keys, S.perm, n, 3 * T.key_level, P.hist, P.totals, s);
  // the set keeps its own sorted keys and order
  if (!in_set) {
    HIPCHECK(hipMemcpyAsync(S.keys, P.k0, size_t(n) * 8, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipMemcpyAsync(S.perm, P.v0, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
  }
  hipLaunchKernelGGL(gather_sorted_kernel, dim3(grid), dim3(256), 0, s, xyz, S.perm, n, S.xyz);
  LAUNCHCHECK("gather_sorted_kernel");
  hipLaunchKernelGGL(ranges_kernel, dim3(unsigned((T.nbox + 255) / 256)), dim3(256), 0, s, P.anchor, P.level,
                     P.leaf, occ, T.nbox, T.key_level, S.keys, n, S.ranges,
                     reinterpret_cast<unsigned*>(P.stat), d_count);
  LAUNCHCHECK("ranges_kernel");
  if (P.nleaves > 0) {
    hipLaunchKernelGGL(leaf_frame_kernel, dim3(unsigned(P.nleaves)), dim3(64), 0, s, P.leaves, P.anchor,
                       P.level, S.ranges, f, S.xyz, S.rel);
    LAUNCHCHECK("leaf_frame_kernel");
  }
}

void update_points_device(PendingPoints& P, const HostTree& T, EvalState* st, const double* src,
                          const double* tgt, void* stream) {
  if (!src) raise(KIFMM_EINVAL, "update_points: null source coordinates");
  if (!tgt && !T.tgt_is_src)
    raise(KIFMM_EINVAL, "update_points: the tree has separate targets; pass their coordinates");
  if (P.device != current_device() || P.nbox != T.nbox || P.nsrc != T.nsrc || P.ntgt != T.ntgt)
    raise(KIFMM_EINVAL, "update_points: sort state of another device or tree");
  for (const double* p : {src, tgt}) {
    if (!p) continue;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      raise(KIFMM_EINVAL, "update_points: coordinates must be device memory");
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nxt = P.cur == 0 ? 1 : 0;  // the set not holding the last accepted update
  if (tgt && !P.tgt[nxt].keys) alloc_set(P, P.tgt[nxt], T.ntgt);
  HIPCHECK(hipMemsetAsync(P.stat, 0, 4 * sizeof(unsigned long long), s));
  sort_set(P, T, src, T.nsrc, P.occ_src, s, P.src[nxt], P.stat + 1);
  if (tgt) sort_set(P, T, tgt, T.ntgt, P.occ_tgt, s, P.tgt[nxt], P.stat + 2);
  unsigned long long stat[4];
  HIPCHECK(hipMemcpyAsync(stat, P.stat, sizeof(stat), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (stat[3] != 0)
    raise(KIFMM_EINVAL, "update_points: " + std::to_string(stat[3]) +
                            " point(s) outside the tree's root box (rebuild the tree on the host)");
  if ((stat[0] & 0xffffffffull) != 0 || int64_t(stat[1]) != T.nsrc || (tgt && int64_t(stat[2]) != T.ntgt))
    raise(KIFMM_EINVAL,
          "update_points: the points occupy other leaves than the tree's (rebuild the tree on the host)");
  // the evaluation state resident on this device takes the new order in place
  const SortedSet& ss = P.src[nxt];
  const SortedSet& ts = tgt ? P.tgt[nxt] : ss;
  DevPointView v = st ? dev_point_view(*st) : DevPointView{};
  if (v.device == P.device && v.nbox == T.nbox) {
    HIPCHECK(hipMemcpyAsync(v.box_src, ss.ranges, size_t(T.nbox) * 8, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipMemcpyAsync(v.src64, ss.rel, size_t(T.nsrc) * 32, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipMemcpyAsync(v.src_perm, ss.perm, size_t(T.nsrc) * 4, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipMemcpyAsync(v.box_tgt, ts.ranges, size_t(T.nbox) * 8, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipMemcpyAsync(v.tgt64, ts.rel, size_t(T.ntgt) * 32, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipMemcpyAsync(v.tgt_perm, ts.perm, size_t(T.ntgt) * 4, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipStreamSynchronize(s));
  }
  P.cur = nxt;
  P.tgt_sep = tgt != nullptr;
  P.stale_host = true;
}

static void set_to_host(const SortedSet& S, int64_t n, int32_t nbox, std::vector<int64_t>& perm,
                        std::vector<double>& xyz, std::vector<uint64_t>& keys, std::vector<int64_t>& beg,
                        std::vector<int64_t>& end) {
  std::vector<u64> k(n);
  std::vector<int32_t> p(n);
  std::vector<int2> r(nbox);
  xyz.resize(3 * size_t(n));
  HIPCHECK(hipMemcpy(k.data(), S.keys, size_t(n) * 8, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(p.data(), S.perm, size_t(n) * 4, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(xyz.data(), S.xyz, size_t(n) * 24, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(r.data(), S.ranges, size_t(nbox) * 8, hipMemcpyDeviceToHost));
  keys.assign(k.begin(), k.end());
  perm.assign(p.begin(), p.end());
  for (int32_t g = 0; g < nbox; ++g) {
    beg[g] = r[g].x;
    end[g] = r[g].y;
  }
}

void pending_to_host(PendingPoints& P, HostTree& T) {
  if (!P.stale_host) return;
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev != P.device) HIPCHECK(hipSetDevice(P.device));
  const SortedSet& ss = P.src[P.cur];
  set_to_host(ss, P.nsrc, P.nbox, T.sperm, T.sxyz, T.skey, T.sbeg, T.send);
  const SortedSet& ts = P.tgt_sep ? P.tgt[P.cur] : ss;
  set_to_host(ts, P.ntgt, P.nbox, T.tperm, T.txyz, T.tkey, T.tbeg, T.tend);
  if (dev != P.device) HIPCHECK(hipSetDevice(dev));
  P.stale_host = false;
}

bool pending_stale(const PendingPoints* P) { return P && P->stale_host; }
int pending_device(const PendingPoints* P) { return P ? P->device : -1; }
void pending_free(PendingPoints* P) { delete P; }

}  // namespace kifmm
