// Host octree and interaction lists (sections "The Fast Multipole Method" and
// "Computational structure of FMM operators"; linear octree of section
// "Data-oriented design": boxes are rows of flat arrays, found by key).
#pragma once

#include <array>
#include <cstdint>
#include <unordered_map>
#include <vector>

#include "kifmm.h"

namespace kifmm {

enum ListKind { LIST_U = 0, LIST_V = 1, LIST_W = 2, LIST_X = 3 };

struct HostTree {
  // inputs (sorted by Morton key of the finest level)
  int64_t nsrc = 0, ntgt = 0;
  std::vector<int64_t> sperm, tperm;  // sorted position -> caller index
  std::vector<double> sxyz, txyz;     // sorted coordinates [n][3]
  std::vector<uint64_t> skey, tkey;   // sorted Morton keys at level key_level

  double c0[3] = {0, 0, 0}, r0 = 0, lo[3] = {0, 0, 0};
  int key_level = 0;  // level of the point keys (uniform depth or max depth)
  bool tgt_is_src = false;  // the targets were given as the source array
  int depth = 0;      // deepest level holding a box

  // boxes: numbered level by level, Morton order inside a level
  int32_t nbox = 0;
  std::vector<int32_t> level, parent, octant, leaf, anchor;  // anchor [nbox][3]
  std::vector<int32_t> child_begin, child_count;             // children contiguous
  std::vector<int64_t> sbeg, send, tbeg, tend;               // ranges in sorted points
  std::vector<int32_t> level_start;                          // [depth + 2]
  std::vector<int32_t> leaves;                               // leaf box ids, ascending

  // interaction lists, CSR over boxes (source boxes without sources skipped)
  std::array<std::vector<int64_t>, 4> off;
  std::array<std::vector<int32_t>, 4> items;

  double halfwidth(int l) const { return r0 / double(int64_t(1) << l); }
  void center(int32_t b, double c[3]) const;
  int64_t nsrc_of(int32_t b) const { return send[b] - sbeg[b]; }
  int64_t ntgt_of(int32_t b) const { return tend[b] - tbeg[b]; }
};

// Argument checks shared by the host and the device build (EINVAL).
void validate_tree_params(int64_t nsrc, int64_t ntgt, const kifmm_tree_params& prm);
// Root box (given, or the bounding cube of the points' per-axis minima mn and
// maxima mx), lower corner and key level of T.
void set_tree_root(HostTree& T, const kifmm_tree_params& prm, const double mn[3], const double mx[3]);

// Builds the tree and its lists.  Throws kifmm::Error on bad input.
HostTree* build_host_tree(const double* src, int64_t nsrc, const double* tgt, int64_t ntgt,
                          const kifmm_tree_params& prm);

}  // namespace kifmm
