// Host octree build: Morton keys, sort, uniform or adaptive refinement, 2:1
// balance, and the U, V, W, X interaction lists (section "Computational
// structure of FMM operators"; lists as defined by Ying et al. 2004, to which
// the paper defers).
//
// Geometric rules, all in FP64 (compiled without FP contraction):
//   root        given, or the bounding cube of all points: c0 = (min+max)/2,
//               r0 = (max extent / 2) * (1 + 2^-20), r0 = 0.5 if all coincide;
//   box index   clamp(floor(t * 2^l), 0, 2^l - 1), t = (x - (c0 - r0)) / (2 r0);
//               keys are taken at the finest level and shifted for coarser ones,
//               which equals evaluating the formula at each level since
//               t * 2^L is exactly (t * 2^l) * 2^(L-l);
//   refinement  uniform: split every non-empty box above the given depth;
//               adaptive: split while > ncrit sources or > ncrit targets and
//               below max_depth; only non-empty children are created;
//   balance     touching leaves (face, edge, corner) differ by <= 1 level;
//   adjacency   closed cubes intersect.
#include "host_tree.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.hpp"

namespace kifmm {
namespace {

inline uint64_t spread3(uint64_t v) {
  // spreads the low 21 bits of v to every third bit
  v &= 0x1fffff;
  v = (v | (v << 32)) & 0x1f00000000ffffULL;
  v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}
inline uint64_t compact3(uint64_t v) {
  v &= 0x1249249249249249ULL;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ULL;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00fULL;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffULL;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffULL;
  v = (v ^ (v >> 32)) & 0x1fffff;
  return v;
}
// Morton code: x in the most significant position of each 3-bit group, so the
// octant of a child is (x_bit << 2) | (y_bit << 1) | z_bit.
inline uint64_t morton(uint64_t x, uint64_t y, uint64_t z) {
  return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}
// A code unique over (level, cell): a sentinel bit above the 3*level key bits.
inline uint64_t cell_code(int level, uint64_t m) { return (uint64_t(1) << (3 * level)) | m; }

struct Builder {
  const kifmm_tree_params& prm;
  HostTree& T;
  // boxes under construction (DFS order)
  struct Box {
    int level;
    uint64_t m;  // Morton code at its level
    int parent;
    int64_t sb, se, tb, te;
    bool leaf;
  };
  std::vector<Box> boxes;
  std::unordered_map<uint64_t, int> index;  // cell_code -> position in boxes

  Builder(const kifmm_tree_params& p, HostTree& t) : prm(p), T(t) {}

  bool wants_split(const Box& b) const {
    if (prm.uniform_depth >= 0) return b.level < prm.uniform_depth;
    return (b.se - b.sb > prm.ncrit || b.te - b.tb > prm.ncrit) && b.level < prm.max_depth;
  }

  // Creates the non-empty children of box i; returns their positions.
  std::vector<int> split(int i) {
    Box b = boxes[i];
    int l = b.level + 1;
    int sh = 3 * (T.key_level - l);
    std::vector<int> out;
    for (uint64_t o = 0; o < 8; ++o) {
      uint64_t m = (b.m << 3) | o;
      uint64_t klo = m << sh, khi = (m + 1) << sh;
      auto sb = std::lower_bound(T.skey.begin() + b.sb, T.skey.begin() + b.se, klo) - T.skey.begin();
      auto se = std::lower_bound(T.skey.begin() + sb, T.skey.begin() + b.se, khi) - T.skey.begin();
      auto tb = std::lower_bound(T.tkey.begin() + b.tb, T.tkey.begin() + b.te, klo) - T.tkey.begin();
      auto te = std::lower_bound(T.tkey.begin() + tb, T.tkey.begin() + b.te, khi) - T.tkey.begin();
      if (se == sb && te == tb) continue;
      Box c{l, m, i, sb, se, tb, te, true};
      index[cell_code(l, m)] = static_cast<int>(boxes.size());
      boxes.push_back(c);
      out.push_back(static_cast<int>(boxes.size()) - 1);
    }
    boxes[i].leaf = out.empty();
    return out;
  }

  int find(int level, int64_t x, int64_t y, int64_t z) const {
    int64_t n = int64_t(1) << level;
    if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return -1;
    auto it = index.find(cell_code(level, morton(x, y, z)));
    return it == index.end() ? -1 : it->second;
  }

  void refine() {
    boxes.push_back(Box{0, 0, -1, 0, T.nsrc, 0, T.ntgt, true});
    index[cell_code(0, 0)] = 0;
    std::vector<int> stack{0};
    while (!stack.empty()) {
      int b = stack.back();
      stack.pop_back();
      if (wants_split(boxes[b])) {
        auto ch = split(b);
        stack.insert(stack.end(), ch.begin(), ch.end());
      }
    }
  }

  // 2:1 balance: for each leaf B (finest level first), every coarse leaf that
  // contains one of B's 26 neighbour cells and is more than one level coarser
  // is split, repeatedly.  Leaves created here are coarser than B and are
  // handled when the sweep reaches their level.
  void balance() {
    int maxl = 0;
    for (auto& b : boxes) maxl = std::max(maxl, b.level);
    for (int l = maxl; l >= 2; --l) {
      std::vector<int> lv;
      for (int i = 0; i < static_cast<int>(boxes.size()); ++i)
        if (boxes[i].leaf && boxes[i].level == l) lv.push_back(i);
      for (int i : lv) {
        uint64_t m = boxes[i].m;
        int64_t ax = compact3(m >> 2), ay = compact3(m >> 1), az = compact3(m);
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
              if (!dx && !dy && !dz) continue;
              int64_t nx = ax + dx, ny = ay + dy, nz = az + dz;
              int64_t n = int64_t(1) << l;
              if (nx < 0 || ny < 0 || nz < 0 || nx >= n || ny >= n || nz >= n) continue;
              for (;;) {
                // deepest existing box containing the neighbour cell, at level <= l-1
                int k = l - 1, c = -1;
                for (; k >= 0; --k) {
                  c = find(k, nx >> (l - k), ny >> (l - k), nz >> (l - k));
                  if (c >= 0) break;
                }
                if (c < 0 || k >= l - 1 || !boxes[c].leaf) break;
                split(c);
              }
            }
      }
    }
  }
};

inline bool adjacent(const HostTree& T, int32_t a, int32_t b) {
  int la = T.level[a], lb = T.level[b];
  int L = std::max(la, lb);
  int64_t sa = int64_t(1) << (L - la), sb = int64_t(1) << (L - lb);
  for (int d = 0; d < 3; ++d) {
    int64_t alo = int64_t(T.anchor[3 * a + d]) * sa, blo = int64_t(T.anchor[3 * b + d]) * sb;
    if (std::max(alo, blo) > std::min(alo + sa, blo + sb)) return false;
  }
  return true;
}

}  // namespace

void HostTree::center(int32_t b, double c[3]) const {
  double r = halfwidth(level[b]);
  for (int d = 0; d < 3; ++d) c[d] = lo[d] + (2.0 * double(anchor[3 * b + d]) + 1.0) * r;
}

static void sort_points(const double* xyz, int64_t n, const double lo[3], double r0, int L,
                        std::vector<int64_t>& perm, std::vector<double>& sorted,
                        std::vector<uint64_t>& keys) {
  std::vector<std::pair<uint64_t, int64_t>> kv(n);
  const double cells = double(int64_t(1) << L);
  const double maxi = cells - 1.0;
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      uint64_t ix[3];
      for (int d = 0; d < 3; ++d) {
        double t = (xyz[3 * i + d] - lo[d]) / (2.0 * r0);
        double f = std::floor(t * cells);
        if (!(f >= 0.0)) f = 0.0;
        if (f > maxi) f = maxi;
        ix[d] = static_cast<uint64_t>(f);
      }
      kv[i] = {morton(ix[0], ix[1], ix[2]), i};
    }
  });
  std::sort(kv.begin(), kv.end());
  perm.resize(n);
  sorted.resize(3 * n);
  keys.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    perm[i] = kv[i].second;
    keys[i] = kv[i].first;
    for (int d = 0; d < 3; ++d) sorted[3 * i + d] = xyz[3 * kv[i].second + d];
  }
}

static void build_lists(HostTree& T, const std::unordered_map<uint64_t, int32_t>& idx) {
  auto find = [&](int level, int64_t x, int64_t y, int64_t z) -> int32_t {
    int64_t n = int64_t(1) << level;
    if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return -1;
    auto it = idx.find(cell_code(level, morton(x, y, z)));
    return it == idx.end() ? -1 : it->second;
  };
  const int32_t nb = T.nbox;
  std::array<std::vector<std::vector<int32_t>>, 4> lists;
  for (auto& l : lists) l.assign(nb, {});

  parallel_for(nb, [&](int64_t b0, int64_t b1) {
    std::vector<int32_t> cand;
    for (int64_t bi = b0; bi < b1; ++bi) {
      int32_t B = static_cast<int32_t>(bi);
      if (T.ntgt_of(B) == 0) continue;  // no targets below B: no lists needed
      int l = T.level[B];
      const int32_t* a = &T.anchor[3 * B];
      if (T.leaf[B]) {
        auto& U = lists[LIST_U][B];
        auto& W = lists[LIST_W][B];
        // coarser or same-level leaves touching B (B included)
        for (int l2 = 0; l2 <= l; ++l2) {
          int64_t s = int64_t(1) << (l - l2), n2 = int64_t(1) << l2;
          int64_t lo[3], hi[3];
          for (int d = 0; d < 3; ++d) {
            lo[d] = std::max<int64_t>((a[d] + s - 1) / s - 1, 0);
            hi[d] = std::min<int64_t>((a[d] + 1) / s, n2 - 1);
          }
          for (int64_t x = lo[0]; x <= hi[0]; ++x)
            for (int64_t y = lo[1]; y <= hi[1]; ++y)
              for (int64_t z = lo[2]; z <= hi[2]; ++z) {
                int32_t c = find(l2, x, y, z);
                if (c >= 0 && T.leaf[c] && T.nsrc_of(c) > 0) U.push_back(c);
              }
        }
        // finer boxes: descend the subtrees of B's non-leaf colleagues
        cand.clear();
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
              if (!dx && !dy && !dz) continue;
              int32_t c = find(l, a[0] + dx, a[1] + dy, a[2] + dz);
              if (c >= 0 && !T.leaf[c])
                for (int k = 0; k < T.child_count[c]; ++k) cand.push_back(T.child_begin[c] + k);
            }
        while (!cand.empty()) {
          int32_t c = cand.back();
          cand.pop_back();
          if (T.nsrc_of(c) == 0) continue;
          if (adjacent(T, c, B)) {
            if (T.leaf[c]) {
              U.push_back(c);
            } else {
              for (int k = 0; k < T.child_count[c]; ++k) cand.push_back(T.child_begin[c] + k);
            }
          } else {
            W.push_back(c);
          }
        }
        std::sort(U.begin(), U.end());
        std::sort(W.begin(), W.end());
      }
      if (l >= 2) {
        auto& V = lists[LIST_V][B];
        const int32_t P = T.parent[B];
        const int32_t* pa = &T.anchor[3 * P];
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
              int32_t c = find(l - 1, pa[0] + dx, pa[1] + dy, pa[2] + dz);
              if (c < 0) continue;
              for (int k = 0; k < T.child_count[c]; ++k) {
                int32_t A = T.child_begin[c] + k;
                if (T.nsrc_of(A) > 0 && !adjacent(T, A, B)) V.push_back(A);
              }
            }
        std::sort(V.begin(), V.end());
      }
      if (l >= 1) {
        // X(B): leaves coarser than B touching B's parent but not B
        auto& X = lists[LIST_X][B];
        const int32_t P = T.parent[B];
        const int32_t* pa = &T.anchor[3 * P];
        int lp = l - 1;
        for (int l2 = 0; l2 <= lp; ++l2) {
          int64_t s = int64_t(1) << (lp - l2), n2 = int64_t(1) << l2;
          int64_t lo[3], hi[3];
          for (int d = 0; d < 3; ++d) {
            lo[d] = std::max<int64_t>((pa[d] + s - 1) / s - 1, 0);
            hi[d] = std::min<int64_t>((pa[d] + 1) / s, n2 - 1);
          }
          for (int64_t x = lo[0]; x <= hi[0]; ++x)
            for (int64_t y = lo[1]; y <= hi[1]; ++y)
              for (int64_t z = lo[2]; z <= hi[2]; ++z) {
                int32_t c = find(l2, x, y, z);
                if (c >= 0 && T.leaf[c] && T.nsrc_of(c) > 0 && !adjacent(T, c, B)) X.push_back(c);
              }
        }
        std::sort(X.begin(), X.end());
      }
    }
  }, 64);

  for (int k = 0; k < 4; ++k) {
    T.off[k].assign(nb + 1, 0);
    for (int32_t b = 0; b < nb; ++b) T.off[k][b + 1] = T.off[k][b] + int64_t(lists[k][b].size());
    T.items[k].resize(T.off[k][nb]);
    for (int32_t b = 0; b < nb; ++b)
      std::copy(lists[k][b].begin(), lists[k][b].end(), T.items[k].begin() + T.off[k][b]);
  }
}

void validate_tree_params(int64_t nsrc, int64_t ntgt, const kifmm_tree_params& prm) {
  if (nsrc < 1 || ntgt < 1) raise(KIFMM_EINVAL, "build_tree: n_src and n_tgt must be >= 1");
  if (nsrc > (int64_t(1) << 31) - 1 || ntgt > (int64_t(1) << 31) - 1)
    raise(KIFMM_EINVAL, "build_tree: at most 2^31-1 points");
  if (prm.uniform_depth > 20) raise(KIFMM_EINVAL, "build_tree: uniform_depth must be <= 20");
  if (prm.uniform_depth < -1) raise(KIFMM_EINVAL, "build_tree: uniform_depth must be >= -1");
  if (prm.uniform_depth < 0) {
    if (prm.ncrit < 1) raise(KIFMM_EINVAL, "build_tree: ncrit must be >= 1");
    if (prm.max_depth < 0 || prm.max_depth > 20)
      raise(KIFMM_EINVAL, "build_tree: max_depth must be in [0, 20]");
  }
  if (prm.root_halfwidth < 0 || !std::isfinite(prm.root_halfwidth))
    raise(KIFMM_EINVAL, "build_tree: root_halfwidth must be finite and >= 0");
  if (prm.root_halfwidth > 0)
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(prm.root_center[d])) raise(KIFMM_EINVAL, "build_tree: non-finite root centre");
}

void set_tree_root(HostTree& T, const kifmm_tree_params& prm, const double mn[3], const double mx[3]) {
  if (prm.root_halfwidth > 0) {
    for (int d = 0; d < 3; ++d) T.c0[d] = prm.root_center[d];
    T.r0 = prm.root_halfwidth;
  } else {
    double ext = 0;
    for (int d = 0; d < 3; ++d) {
      T.c0[d] = 0.5 * (mn[d] + mx[d]);
      ext = std::max(ext, mx[d] - mn[d]);
    }
    double r = 0.5 * ext * (1.0 + std::ldexp(1.0, -20));
    T.r0 = r > 0 ? r : 0.5;
  }
  for (int d = 0; d < 3; ++d) T.lo[d] = T.c0[d] - T.r0;
  T.key_level = prm.uniform_depth >= 0 ? prm.uniform_depth : prm.max_depth;
}

HostTree* build_host_tree(const double* src, int64_t nsrc, const double* tgt, int64_t ntgt,
                          const kifmm_tree_params& prm) {
  if (!src || !tgt) raise(KIFMM_EINVAL, "build_tree: null point array");
  validate_tree_params(nsrc, ntgt, prm);
  for (int64_t i = 0; i < 3 * nsrc; ++i)
    if (!std::isfinite(src[i])) raise(KIFMM_EINVAL, "build_tree: non-finite source coordinate");
  for (int64_t i = 0; i < 3 * ntgt; ++i)
    if (!std::isfinite(tgt[i])) raise(KIFMM_EINVAL, "build_tree: non-finite target coordinate");

  alloc_hook("build_tree");
  auto* Tp = new HostTree();
  HostTree& T = *Tp;
  try {
    T.nsrc = nsrc;
    T.ntgt = ntgt;
    double mn[3], mx[3];
    for (int d = 0; d < 3; ++d) mn[d] = mx[d] = src[d];
    if (prm.root_halfwidth <= 0) {
      auto upd = [&](const double* x, int64_t n) {
        for (int64_t i = 0; i < n; ++i)
          for (int d = 0; d < 3; ++d) {
            mn[d] = std::min(mn[d], x[3 * i + d]);
            mx[d] = std::max(mx[d], x[3 * i + d]);
          }
      };
      upd(src, nsrc);
      upd(tgt, ntgt);
    }
    set_tree_root(T, prm, mn, mx);
    if (prm.root_halfwidth > 0) {
      // a point outside the given root cube would be clamped into a boundary
      // leaf, beyond that leaf's equivalent surface: refused
      auto inside = [&](const double* x, int64_t n) {
        for (int64_t i = 0; i < n; ++i)
          for (int d = 0; d < 3; ++d) {
            const double t = (x[3 * i + d] - T.lo[d]) / (2.0 * T.r0);
            if (!(t >= 0.0 && t <= 1.0)) return false;
          }
        return true;
      };
      if (!inside(src, nsrc) || !inside(tgt, ntgt))
        raise(KIFMM_EINVAL, "build_tree: a point lies outside the given root box");
    }
    T.tgt_is_src = tgt == src && ntgt == nsrc;

    sort_points(src, nsrc, T.lo, T.r0, T.key_level, T.sperm, T.sxyz, T.skey);
    sort_points(tgt, ntgt, T.lo, T.r0, T.key_level, T.tperm, T.txyz, T.tkey);

    Builder B(prm, T);
    B.refine();
    if (prm.uniform_depth < 0 && prm.balance) B.balance();

    // final numbering: by (level, Morton)
    const int nb = static_cast<int>(B.boxes.size());
    std::vector<int> order(nb);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int x, int y) {
      if (B.boxes[x].level != B.boxes[y].level) return B.boxes[x].level < B.boxes[y].level;
      return B.boxes[x].m < B.boxes[y].m;
    });
    std::vector<int> newid(nb);
    for (int i = 0; i < nb; ++i) newid[order[i]] = i;
    T.nbox = nb;
    T.level.resize(nb);
    T.parent.resize(nb);
    T.octant.resize(nb);
    T.leaf.resize(nb);
    T.anchor.resize(3 * nb);
    T.child_begin.assign(nb, -1);
    T.child_count.assign(nb, 0);
    T.sbeg.resize(nb);
    T.send.resize(nb);
    T.tbeg.resize(nb);
    T.tend.resize(nb);
    std::unordered_map<uint64_t, int32_t> idx;
    idx.reserve(nb * 2);
    T.depth = 0;
    for (int i = 0; i < nb; ++i) {
      const auto& b = B.boxes[order[i]];
      T.level[i] = b.level;
      T.parent[i] = b.parent < 0 ? -1 : newid[b.parent];
      T.octant[i] = static_cast<int32_t>(b.m & 7);
      T.leaf[i] = b.leaf ? 1 : 0;
      T.anchor[3 * i + 0] = static_cast<int32_t>(compact3(b.m >> 2));
      T.anchor[3 * i + 1] = static_cast<int32_t>(compact3(b.m >> 1));
      T.anchor[3 * i + 2] = static_cast<int32_t>(compact3(b.m));
      T.sbeg[i] = b.sb;
      T.send[i] = b.se;
      T.tbeg[i] = b.tb;
      T.tend[i] = b.te;
      T.depth = std::max(T.depth, b.level);
      idx[cell_code(b.level, b.m)] = i;
    }
    for (int i = 0; i < nb; ++i) {
      int p = T.parent[i];
      if (p < 0) continue;
      if (T.child_begin[p] < 0 || i < T.child_begin[p]) T.child_begin[p] = i;
      T.child_count[p]++;
    }
    T.level_start.assign(T.depth + 2, 0);
    for (int i = 0; i < nb; ++i) T.level_start[T.level[i] + 1]++;
    for (int l = 0; l <= T.depth; ++l) T.level_start[l + 1] += T.level_start[l];
    for (int i = 0; i < nb; ++i)
      if (T.leaf[i]) T.leaves.push_back(i);

    build_lists(T, idx);
  } catch (...) {
    delete Tp;
    throw;
  }
  return Tp;
}

}  // namespace kifmm
