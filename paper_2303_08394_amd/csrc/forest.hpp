// A forest: one or more host trees merged into the flat arrays the device
// kernels read, plus the tile plans of the gathered GEMMs (M2M, L2L, the
// check-to-equivalent solves and M2L).
//
// Box "columns": every box b owns n_rhs columns of a density or check
// potential buffer, column (b * n_rhs + r) of length ld (ld = n rounded up to
// 16, padding rows zero).
#pragma once

#include <cstdint>
#include <vector>

#include "host_tree.hpp"
#include "precompute.hpp"

namespace kifmm {

// out[tile_cols[t][j]] (+)= sum over the tile's steps s of
//   op[step_op[s]] * in[step_src[s][j]]      (j < TB; -1 entries are skipped)
struct Plan {
  int32_t ntile = 0, TB = 0;
  std::vector<int32_t> tile_cols;  // [ntile][TB]
  std::vector<int32_t> step_beg;   // [ntile + 1]
  std::vector<int32_t> step_op;    // [nstep]
  std::vector<int32_t> step_src;   // [nstep][TB]
  int64_t nstep() const { return int64_t(step_op.size()); }
  int64_t useful_pairs = 0;        // (column, step) pairs with a source
  // Tiles add into the output with atomics instead of read-add-write; a
  // column then appears in at most two tiles and the output starts at zero.
  bool atomic = false;
  bool split = false;              // tiles cut in two (plan cache key)
};

struct HostForest {
  int32_t nprob = 0, nbox = 0, depth = 0;
  int64_t nsrc = 0, ntgt = 0;
  std::vector<int64_t> src_off, tgt_off;  // per problem point ranges [nprob + 1]
  std::vector<int32_t> box_off;           // per problem box ranges [nprob + 1]
  // per box
  std::vector<int32_t> box_geo;     // [nbox][4] anchor x, y, z, level
  std::vector<double> box_r;        // [nbox] half-width
  std::vector<int32_t> box_src;     // [nbox][2] global sorted source range
  std::vector<int32_t> box_tgt;     // [nbox][2]
  std::vector<int32_t> box_parent;  // global id or -1
  std::vector<int32_t> box_octant, box_leaf;
  // points, sorted, coordinates relative to their leaf: (x - c) / r, w = 0
  std::vector<double> src_f64, tgt_f64;  // [n][4]
  std::vector<int32_t> src_perm, tgt_perm;  // sorted -> caller index (within problem)
  // leaf work lists
  std::vector<int32_t> p2m_boxes;   // leaves at level >= 2 holding sources
  std::vector<int32_t> leaf_boxes;  // leaves holding targets
  std::vector<int32_t> u_off, u_items, w_off, w_items;  // CSR over leaf_boxes
  std::vector<int32_t> x_boxes, x_off, x_items;         // boxes with a non-empty X list
  // per-level plans (index = level) and the all-level M2L plan.  The M2M
  // plan of level l has one step per child (at level l + 1, tiled by octant):
  // it writes that child's contribution M2M[octant] * up_eq[child] to the
  // child's own column of a scratch buffer, and m2m_sum[l] ([nparent][9]:
  // parent, then its child of octant 0..7 or -1) adds them up per parent.
  std::vector<Plan> m2m, uc2e, l2l, dc2e;
  std::vector<std::vector<int32_t>> m2m_sum;
  Plan m2l;
  // Problems whose M2L tiles would be sparse (the tiles' fill, V-list pairs
  // over tile columns x steps, below pair_fill: adaptive trees of surfaces)
  // run M2L pair by pair instead: m2l_pair has one step per tile, TBm
  // (target, source) pairs of one offset, and writes pair p's product to
  // column p of a pair buffer; then each target's check potential is the sum
  // of its pairs (pair_items[pair_off[k] .. pair_off[k + 1]) for target
  // pair_tgt[k]), in the order of the offsets.
  Plan m2l_pair;
  std::vector<int32_t> pair_tgt, pair_off, pair_items;
  int64_t n_pairs = 0;
  double pair_fill = 0.0;          // the threshold the plans were built for
  int64_t max_pairs = 0;           // and the pair count cap
  // M2L operator indices include the level (level * 316 + offset): operator
  // tables per level, as the screened kernel needs
  bool per_level = false;
  // statistics of the lists (for work counts)
  int64_t n_u_pairs = 0, n_v_pairs = 0, n_w_pairs = 0, n_x_pairs = 0;
  int64_t p2p_interactions = 0;  // sum over U pairs of n_tgt(B) * n_src(A)
};

// Builds the forest of `n` trees for operator set `ops`: plan width TB boxes
// per tile for M2M, L2L and the solves, TBm for M2L.  With split, every M2L
// tile is run as two blocks (even and odd x offsets).  Problems whose M2L
// tiles fill less than pair_fill of their slots run M2L pair by pair, unless
// that makes more than max_pairs pairs (then none does).  per_level: M2L
// operator indices carry the target level (tables per level).
HostForest* build_forest(const HostTree* const* trees, int n, const HostOps& ops, int TB, int TBm,
                         bool split, double pair_fill, int64_t max_pairs, bool per_level = false);

// Raises KIFMM_EUNSUPPORTED unless the density columns of a forest of nbox
// boxes (plus the zero box) with n_rhs right-hand sides at operator size n,
// split into up to three 16-bit parts or held in FP64, span at most 2^32
// units of 16 bytes (64 GiB): the gathered GEMM addresses them with 32-bit
// unit offsets.
void check_operand_limits(int64_t nbox, int n_rhs, int n);

}  // namespace kifmm
