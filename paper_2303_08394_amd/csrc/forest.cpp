// Forest assembly and gathered-GEMM tile plans.
#include "forest.hpp"

#include <algorithm>
#include <array>
#include <map>
#include <memory>
#include <set>

#include "common.hpp"

namespace kifmm {
namespace {

// Groups `boxes` by key, keeps the given order inside a group, and cuts each
// group into tiles of TB columns.
template <class KeyF>
std::vector<std::vector<int32_t>> group_tiles(const std::vector<int32_t>& boxes, int TB, KeyF key) {
  std::map<int64_t, std::vector<int32_t>> groups;
  for (int32_t b : boxes) groups[key(b)].push_back(b);
  std::vector<std::vector<int32_t>> tiles;
  for (auto& g : groups)
    for (size_t i = 0; i < g.second.size(); i += TB)
      tiles.emplace_back(g.second.begin() + i,
                         g.second.begin() + std::min(g.second.size(), i + size_t(TB)));
  return tiles;
}

// Appends one tile whose column j takes, at each step, the source given by
// src(j, step) (or -1).
void add_tile(Plan& P, const std::vector<int32_t>& cols, const std::vector<int32_t>& ops,
              const std::vector<std::vector<int32_t>>& srcs) {
  const int TB = P.TB;
  for (int j = 0; j < TB; ++j) P.tile_cols.push_back(j < int(cols.size()) ? cols[j] : -1);
  for (size_t s = 0; s < ops.size(); ++s) {
    P.step_op.push_back(ops[s]);
    for (int j = 0; j < TB; ++j) {
      int32_t v = j < int(cols.size()) ? srcs[s][j] : -1;
      P.step_src.push_back(v);
      if (v >= 0) P.useful_pairs++;
    }
  }
  P.step_beg.push_back(int32_t(P.step_op.size()));
  P.ntile++;
}

Plan new_plan(int TB) {
  Plan P;
  P.TB = TB;
  P.step_beg.push_back(0);
  return P;
}

}  // namespace

void check_operand_limits(int64_t nbox, int n_rhs, int n) {
  const int64_t ld = (int64_t(n) + 31) / 32 * 32;
  // widest element of a column: three 16-bit parts (6 bytes) or FP64 (8)
  const int64_t bytes = (nbox + 1) * int64_t(n_rhs) * ld * 8;
  if (nbox < 0 || n_rhs < 1 || n < 1 || bytes / 16 > (int64_t(1) << 32))
    raise(KIFMM_EUNSUPPORTED, "evaluate: density columns beyond 64 GiB (boxes x right-hand sides x operator rows)");
}

HostForest* build_forest(const HostTree* const* trees, int n, const HostOps& ops, int TB, int TBm,
                         bool split, double pair_fill, int64_t max_pairs, bool per_level) {
  alloc_hook("evaluate (plans)");
  std::unique_ptr<HostForest> Fp(new HostForest());
  HostForest& F = *Fp;
  F.nprob = n;
  F.src_off.assign(n + 1, 0);
  F.tgt_off.assign(n + 1, 0);
  F.box_off.assign(n + 1, 0);
  for (int k = 0; k < n; ++k) {
    F.src_off[k + 1] = F.src_off[k] + trees[k]->nsrc;
    F.tgt_off[k + 1] = F.tgt_off[k] + trees[k]->ntgt;
    F.box_off[k + 1] = F.box_off[k] + trees[k]->nbox;
    F.depth = std::max(F.depth, trees[k]->depth);
  }
  F.nsrc = F.src_off[n];
  F.ntgt = F.tgt_off[n];
  F.nbox = F.box_off[n];
  if (F.nsrc > (int64_t(1) << 31) - 1 || F.ntgt > (int64_t(1) << 31) - 1)
    raise(KIFMM_EUNSUPPORTED, "forest: more than 2^31-1 points");
  const int32_t NB = F.nbox;
  F.box_geo.resize(4 * size_t(NB));
  F.box_r.resize(NB);
  F.box_src.resize(2 * size_t(NB));
  F.box_tgt.resize(2 * size_t(NB));
  F.box_parent.resize(NB);
  F.box_octant.resize(NB);
  F.box_leaf.resize(NB);
  F.src_f64.resize(4 * size_t(F.nsrc));
  F.tgt_f64.resize(4 * size_t(F.ntgt));
  F.src_perm.resize(F.nsrc);
  F.tgt_perm.resize(F.ntgt);

  std::vector<int32_t> boxes_by_level_src, tmp;
  std::vector<std::vector<int32_t>> lvl_boxes(F.depth + 1);
  for (int k = 0; k < n; ++k) {
    const HostTree& T = *trees[k];
    const int32_t bo = F.box_off[k];
    const int64_t so = F.src_off[k], to = F.tgt_off[k];
    for (int32_t b = 0; b < T.nbox; ++b) {
      int32_t g = bo + b;
      for (int d = 0; d < 3; ++d) F.box_geo[4 * size_t(g) + d] = T.anchor[3 * b + d];
      F.box_geo[4 * size_t(g) + 3] = T.level[b];
      F.box_r[g] = T.halfwidth(T.level[b]);
      F.box_src[2 * size_t(g)] = int32_t(so + T.sbeg[b]);
      F.box_src[2 * size_t(g) + 1] = int32_t(so + T.send[b]);
      F.box_tgt[2 * size_t(g)] = int32_t(to + T.tbeg[b]);
      F.box_tgt[2 * size_t(g) + 1] = int32_t(to + T.tend[b]);
      F.box_parent[g] = T.parent[b] < 0 ? -1 : bo + T.parent[b];
      F.box_octant[g] = T.octant[b];
      F.box_leaf[g] = T.leaf[b];
      lvl_boxes[T.level[b]].push_back(g);
      if (T.leaf[b]) {
        double c[3], r = T.halfwidth(T.level[b]);
        T.center(b, c);
        for (int64_t i = T.sbeg[b]; i < T.send[b]; ++i)
          for (int d = 0; d < 3; ++d) F.src_f64[4 * (so + i) + d] = (T.sxyz[3 * i + d] - c[d]) / r;
        for (int64_t i = T.tbeg[b]; i < T.tend[b]; ++i)
          for (int d = 0; d < 3; ++d) F.tgt_f64[4 * (to + i) + d] = (T.txyz[3 * i + d] - c[d]) / r;
      }
    }
    for (int64_t i = 0; i < T.nsrc; ++i) F.src_perm[so + i] = int32_t(T.sperm[i]);
    for (int64_t i = 0; i < T.ntgt; ++i) F.tgt_perm[to + i] = int32_t(T.tperm[i]);
  }

  auto nsrc_of = [&](int32_t g) { return F.box_src[2 * size_t(g) + 1] - F.box_src[2 * size_t(g)]; };
  auto ntgt_of = [&](int32_t g) { return F.box_tgt[2 * size_t(g) + 1] - F.box_tgt[2 * size_t(g)]; };

  // leaf work lists and the U, W, X lists in global ids
  F.u_off.push_back(0);
  F.w_off.push_back(0);
  F.x_off.push_back(0);
  for (int k = 0; k < n; ++k) {
    const HostTree& T = *trees[k];
    const int32_t bo = F.box_off[k];
    for (int32_t b = 0; b < T.nbox; ++b) {
      const int32_t g = bo + b;
      if (T.leaf[b] && T.level[b] >= 2 && T.nsrc_of(b) > 0) F.p2m_boxes.push_back(g);
      if (T.leaf[b] && T.ntgt_of(b) > 0) {
        F.leaf_boxes.push_back(g);
        for (int64_t e = T.off[LIST_U][b]; e < T.off[LIST_U][b + 1]; ++e) {
          int32_t a = T.items[LIST_U][e];
          F.u_items.push_back(bo + a);
          F.p2p_interactions += T.ntgt_of(b) * T.nsrc_of(a);
        }
        for (int64_t e = T.off[LIST_W][b]; e < T.off[LIST_W][b + 1]; ++e)
          F.w_items.push_back(bo + T.items[LIST_W][e]);
        F.u_off.push_back(int32_t(F.u_items.size()));
        F.w_off.push_back(int32_t(F.w_items.size()));
      }
      if (T.off[LIST_X][b + 1] > T.off[LIST_X][b] && T.ntgt_of(b) > 0) {
        F.x_boxes.push_back(g);
        for (int64_t e = T.off[LIST_X][b]; e < T.off[LIST_X][b + 1]; ++e)
          F.x_items.push_back(bo + T.items[LIST_X][e]);
        F.x_off.push_back(int32_t(F.x_items.size()));
      }
      F.n_v_pairs += T.off[LIST_V][b + 1] - T.off[LIST_V][b];
    }
  }
  F.n_u_pairs = int64_t(F.u_items.size());
  F.n_w_pairs = int64_t(F.w_items.size());
  F.n_x_pairs = int64_t(F.x_items.size());

  // plans
  const int D = F.depth;
  F.m2m.assign(D + 1, new_plan(TB));
  F.m2m_sum.assign(D + 1, {});
  F.uc2e.assign(D + 1, new_plan(TB));
  F.l2l.assign(D + 1, new_plan(TB));
  F.dc2e.assign(D + 1, new_plan(TB));
  F.m2l = new_plan(TBm);
  for (int l = 2; l <= D; ++l) {
    // M2M: per-child contributions, then a per-parent sum in octant order
    std::vector<int32_t> parents, withsrc, withtgt;
    for (int32_t g : lvl_boxes[l]) {
      if (nsrc_of(g) > 0) withsrc.push_back(g);
      if (ntgt_of(g) > 0) withtgt.push_back(g);
      if (!F.box_leaf[g] && nsrc_of(g) > 0) parents.push_back(g);
    }
    if (!parents.empty()) {
      // children with sources of the non-leaf parents of this level
      std::map<std::pair<int32_t, int>, int32_t> child;
      std::vector<int32_t> kids;
      for (int32_t g : lvl_boxes[l + 1 <= D ? l + 1 : l])
        if (l + 1 <= D && nsrc_of(g) > 0) {
          child[{F.box_parent[g], F.box_octant[g]}] = g;
          kids.push_back(g);
        }
      for (auto& tile : group_tiles(kids, TB, [&](int32_t g) { return int64_t(F.box_octant[g]); }))
        add_tile(F.m2m[l], tile, {F.box_octant[tile[0]]}, {tile});
      for (int32_t par : parents) {
        F.m2m_sum[l].push_back(par);
        for (int o = 0; o < 8; ++o) {
          auto it = child.find({par, o});
          F.m2m_sum[l].push_back(it != child.end() ? it->second : -1);
        }
      }
    }
    for (auto& tile : group_tiles(withsrc, TB, [](int32_t) { return int64_t(0); }))
      add_tile(F.uc2e[l], tile, {0}, {tile});
    for (auto& tile : group_tiles(withtgt, TB, [](int32_t) { return int64_t(0); }))
      add_tile(F.dc2e[l], tile, {0}, {tile});
    if (l >= 3) {
      for (auto& tile : group_tiles(withtgt, TB, [&](int32_t g) { return int64_t(F.box_octant[g]); })) {
        std::vector<int32_t> par(tile.size());
        for (size_t j = 0; j < tile.size(); ++j) par[j] = F.box_parent[tile[j]];
        add_tile(F.l2l[l], tile, {F.box_octant[tile[0]]}, {par});
      }
    }
  }
  // M2L: targets grouped by (level, octant), steps = union of the tile's offsets
  {
    std::vector<int32_t> tg;
    // V lists per global box
    std::vector<std::vector<std::pair<int32_t, int32_t>>> vl(NB);  // (op, source)
    for (int k = 0; k < n; ++k) {
      const HostTree& T = *trees[k];
      const int32_t bo = F.box_off[k];
      for (int32_t b = 0; b < T.nbox; ++b) {
        if (T.ntgt_of(b) == 0 || T.off[LIST_V][b + 1] == T.off[LIST_V][b]) continue;
        const int32_t g = bo + b;
        tg.push_back(g);
        for (int64_t e = T.off[LIST_V][b]; e < T.off[LIST_V][b + 1]; ++e) {
          int32_t a = T.items[LIST_V][e];
          int dx = T.anchor[3 * a] - T.anchor[3 * b];
          int dy = T.anchor[3 * a + 1] - T.anchor[3 * b + 1];
          int dz = T.anchor[3 * a + 2] - T.anchor[3 * b + 2];
          int op = ops.m2l_index[(dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)];
          if (op < 0) raise(KIFMM_EINVAL, "forest: V-list offset outside the M2L table");
          vl[g].push_back({op, bo + a});
        }
      }
    }
    // Targets of one (level, octant) class are ordered by the set of offsets
    // of their V list (then Morton order), so that a tile holds boxes with the
    // same or similar offsets and few steps run with empty columns; boxes
    // away from the domain boundary all share the full set.
    std::vector<std::vector<uint64_t>> mask(NB);
    for (int32_t g : tg) {
      mask[g].assign((kNumM2L + 63) / 64, 0);
      for (auto& e : vl[g]) mask[g][e.first >> 6] |= uint64_t(1) << (e.first & 63);
    }
    std::stable_sort(tg.begin(), tg.end(), [&](int32_t x, int32_t y) {
      int64_t kx = int64_t(F.box_geo[4 * size_t(x) + 3]) * 8 + F.box_octant[x];
      int64_t ky = int64_t(F.box_geo[4 * size_t(y) + 3]) * 8 + F.box_octant[y];
      if (kx != ky) return kx < ky;
      if (mask[x] != mask[y]) return mask[x] > mask[y];
      return x < y;
    });
    auto class_key = [&](int32_t g) { return int64_t(F.box_geo[4 * size_t(g) + 3]) * 8 + F.box_octant[g]; };
    // Fill of each problem's own tiles: V-list pairs over (union of the
    // tile's offsets) x tile width, for tiles of 64 boxes whatever TBm is.  A
    // problem below pair_fill runs M2L pair by pair; the choice depends on
    // the problem alone (not on the batch it is in, nor on the number of
    // right-hand sides), so results match across those bitwise.
    constexpr int kFillTB = 64;
    auto prob_of = [&](int32_t g) {
      return int(std::upper_bound(F.box_off.begin(), F.box_off.end(), g) - F.box_off.begin()) - 1;
    };
    std::vector<char> as_pairs(n, 0);
    if (pair_fill > 0.0) {
      std::vector<std::vector<int32_t>> per(n);
      for (int32_t g : tg) per[prob_of(g)].push_back(g);
      for (int k = 0; k < n; ++k) {
        int64_t useful = 0, slots = 0;
        for (auto& tile : group_tiles(per[k], kFillTB, class_key)) {
          std::vector<uint64_t> u((kNumM2L + 63) / 64, 0);
          for (int32_t g : tile) {
            useful += int64_t(vl[g].size());
            for (size_t w = 0; w < u.size(); ++w) u[w] |= mask[g][w];
          }
          int64_t cnt = 0;
          for (uint64_t w : u) cnt += __builtin_popcountll(w);
          slots += cnt * kFillTB;
        }
        as_pairs[k] = slots > 0 && double(useful) < pair_fill * double(slots);
      }
      int64_t np = 0;
      for (int32_t g : tg)
        if (as_pairs[prob_of(g)]) np += int64_t(vl[g].size());
      if (np > max_pairs) std::fill(as_pairs.begin(), as_pairs.end(), 0);
    }
    std::vector<int32_t> tg_pairs;
    {
      std::vector<int32_t> dense;
      for (int32_t g : tg) (as_pairs[prob_of(g)] ? tg_pairs : dense).push_back(g);
      tg.swap(dense);
    }
    auto tiles = group_tiles(tg, TBm, class_key);
    // Step order inside a tile: by the parity of the offset, then by
    // operator.  The targets of one tile share their octant, so the parity of
    // the offset fixes the parity class of every source box the step reads;
    // the blocks on one XCD then sweep one class (1/8 of the level's
    // densities) after another and find them in that XCD's L2.
    auto step_key = [&](int32_t op) {
      const int32_t* d = &ops.m2l_offset[3 * size_t(op)];
      return int32_t((((d[0] & 1) << 2) | ((d[1] & 1) << 1) | (d[2] & 1)) * kNumM2L + op);
    };
    struct Part {
      std::vector<int32_t> cols, opl;
      std::vector<std::vector<int32_t>> srcs;
      int cls;
    };
    std::array<std::vector<Part>, 8> q;  // per octant class
    for (auto& tile : tiles) {
      std::map<int32_t, std::vector<int32_t>> steps;  // keyed by step_key
      for (size_t j = 0; j < tile.size(); ++j)
        for (auto& e : vl[tile[j]]) {
          auto& s = steps[step_key(e.first)];
          if (s.empty()) s.assign(tile.size(), -1);
          s[j] = e.second;
        }
      Part whole{tile, {}, {}, F.box_octant[tile[0]]};
      for (auto& s : steps) {
        whole.opl.push_back(s.first % kNumM2L);
        whole.srcs.push_back(s.second);
      }
      // The step list is cut in two parts run by two blocks (twice the
      // blocks the level's tiles alone give); both add into the zeroed
      // output, so each value is the sum of at most two terms and does not
      // depend on their order.  The cut is at a fixed offset property (x
      // offset even / odd: the first four parity classes) and every tile is
      // cut, so a box's two partial sums do not depend on which boxes share
      // its tile (batches and multi-RHS runs reproduce single runs bitwise).
      const size_t ns = whole.opl.size();
      size_t h = 0;
      while (h < ns && step_key(whole.opl[h]) < 4 * kNumM2L) ++h;
      if (split && h > 0 && h < ns) {
        Part a{tile, {whole.opl.begin(), whole.opl.begin() + h}, {whole.srcs.begin(), whole.srcs.begin() + h}, whole.cls};
        Part b{tile, {whole.opl.begin() + h, whole.opl.end()}, {whole.srcs.begin() + h, whole.srcs.end()}, whole.cls};
        q[whole.cls].push_back(std::move(a));
        q[whole.cls ^ 4].push_back(std::move(b));
      } else {
        q[whole.cls].push_back(std::move(whole));
      }
    }
    // Launch order: blocks are dealt to the 8 XCDs round-robin, so part t is
    // taken from queue t % 8 while every queue has parts left.  Queue k holds
    // the even-x parts of octant k and the odd-x parts of octant k ^ 4: a
    // step of offset parity class c reads source boxes of parity class
    // octant ^ c, so both kinds of part sweep the same four source classes
    // in the same order (k, k ^ 1, k ^ 2, k ^ 3), and the blocks resident on
    // one XCD read one class of densities at a time from that XCD's L2
    // (queued by octant alone, the two halves of a tile would keep two
    // classes live).  Inside a queue, parts with more steps go first.
    for (auto& v : q)
      std::stable_sort(v.begin(), v.end(), [](const Part& x, const Part& y) { return x.opl.size() > y.opl.size(); });
    std::array<size_t, 8> pos{};
    for (bool any = true; any;) {
      any = false;
      for (int o = 0; o < 8; ++o)
        if (pos[o] < q[o].size()) {
          Part& t = q[o][pos[o]++];
          if (per_level) {
            const int32_t lev_off = F.box_geo[4 * size_t(t.cols[0]) + 3] * kNumM2L;
            std::vector<int32_t> ops(t.opl);
            for (auto& v : ops) v += lev_off;
            add_tile(F.m2l, t.cols, ops, t.srcs);
          } else {
            add_tile(F.m2l, t.cols, t.opl, t.srcs);
          }
          any = true;
        }
    }
    F.m2l.atomic = true;
    F.m2l.split = split;
    F.per_level = per_level;

    // Pair-by-pair M2L of the sparse problems: pairs sorted by offset, then
    // target; tiles of TBm pairs of one offset (one step each); pair p writes
    // column p of the pair buffer.  The offsets are dealt to 8 queues
    // (fewest tiles first) and the queues interleaved, so that consecutive
    // blocks, which go to different XCDs, take their operators from
    // different queues and each operator is read by one XCD's L2.
    F.m2l_pair = new_plan(TBm);
    F.pair_fill = pair_fill;
    F.max_pairs = max_pairs;
    struct PairE {
      int32_t op, t, s;
    };
    std::vector<PairE> pe;
    for (int32_t g : tg_pairs)
      for (auto& e : vl[g]) pe.push_back({e.first, g, e.second});
    std::sort(pe.begin(), pe.end(), [](const PairE& x, const PairE& y) {
      return x.op != y.op ? x.op < y.op : x.t < y.t;
    });
    F.n_pairs = int64_t(pe.size());
    if (F.n_pairs > (int64_t(1) << 31) - 1) raise(KIFMM_EUNSUPPORTED, "forest: too many M2L pairs");
    std::vector<std::vector<std::pair<int32_t, int32_t>>> per_op(kNumM2L);  // tile ranges in pe
    auto level_of = [&](int32_t g) { return F.box_geo[4 * size_t(g) + 3]; };
    for (size_t i = 0; i < pe.size();) {
      size_t j = i;
      // (with operators per level a tile also keeps to one level)
      while (j < pe.size() && pe[j].op == pe[i].op && j - i < size_t(TBm) &&
             (!per_level || level_of(pe[j].t) == level_of(pe[i].t)))
        ++j;
      per_op[pe[i].op].push_back({int32_t(i), int32_t(j)});
      i = j;
    }
    std::vector<int32_t> op_order(kNumM2L);
    for (int o = 0; o < kNumM2L; ++o) op_order[o] = o;
    std::stable_sort(op_order.begin(), op_order.end(),
                     [&](int32_t x, int32_t y) { return per_op[x].size() > per_op[y].size(); });
    std::array<std::vector<std::pair<int32_t, int32_t>>, 8> pq;
    std::array<size_t, 8> load{};
    for (int32_t o : op_order) {
      if (per_op[o].empty()) continue;
      int qi = int(std::min_element(load.begin(), load.end()) - load.begin());
      for (auto& r : per_op[o]) pq[qi].push_back(r);
      load[qi] += per_op[o].size();
    }
    std::array<size_t, 8> qpos{};
    for (bool any = true; any;) {
      any = false;
      for (int qi = 0; qi < 8; ++qi)
        if (qpos[qi] < pq[qi].size()) {
          auto r = pq[qi][qpos[qi]++];
          std::vector<int32_t> cols, srcs;
          for (int32_t i = r.first; i < r.second; ++i) {
            cols.push_back(i);
            srcs.push_back(pe[i].s);
          }
          const int32_t op = pe[r.first].op + (per_level ? level_of(pe[r.first].t) * kNumM2L : 0);
          add_tile(F.m2l_pair, cols, {op}, {srcs});
          any = true;
        }
    }
    // per target: its pairs in offset order
    std::map<int32_t, std::vector<int32_t>> of_tgt;
    for (size_t i = 0; i < pe.size(); ++i) of_tgt[pe[i].t].push_back(int32_t(i));
    F.pair_off.push_back(0);
    for (auto& kv : of_tgt) {
      F.pair_tgt.push_back(kv.first);
      F.pair_items.insert(F.pair_items.end(), kv.second.begin(), kv.second.end());
      F.pair_off.push_back(int32_t(F.pair_items.size()));
    }
  }
  return Fp.release();
}

}  // namespace kifmm
