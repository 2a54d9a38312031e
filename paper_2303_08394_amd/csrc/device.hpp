// Device-side state of an evaluation: the forest and operator tables in HBM,
// the work buffers, and the entry into the evaluation pipeline.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>
#include <memory>
#include <vector>

#include "forest.hpp"
#include "host_tree.hpp"
#include "kifmm.h"

namespace kifmm {

struct DevPlan {
  int32_t ntile = 0, TB = 0;
  int32_t *tile_cols = nullptr, *step_beg = nullptr, *step_op = nullptr, *step_src = nullptr;
  int64_t nstep = 0, useful_pairs = 0;
  int32_t max_tile_steps = 0;  // longest step list of one tile
  bool atomic = false;         // tiles add into the output with atomics
};

struct DevForest;   // defined in evaluate.hip
struct DevOps;
struct DevWork;

// Everything one evaluation needs on one device: built on first use.
struct EvalState {
  int device = -1;
  std::unique_ptr<HostForest> host;
  DevForest* forest = nullptr;
  ~EvalState();
};

// Uploads (once) and returns the device operator tables of `ops` for `device`.
struct OpsCache {
  std::map<int, DevOps*> per_device;
  ~OpsCache();
};

// Runs the evaluation; throws kifmm::Error.
// With grad, potentials[k] holds [n_rhs][4][n_tgt]: the potential and its
// gradient (d/dx, d/dy, d/dz) at every target.
void evaluate_forest(EvalState& st, const HostOps& hops, OpsCache& ocache,
                     const void* const* charges, void* const* potentials, int n_rhs,
                     bool io_fp64, kifmm_precision prec, void* stream, bool grad = false);

// Bytes of the allocation-free entry point's work-buffer array on each device.
constexpr size_t kNoAllocScratchBytes = size_t(256) << 20;

// The evaluation of one tree with every work buffer taken from a fixed
// device array (kifmm_evaluate_noalloc): no device allocation, eager
// launches on `stream`.  The tree's device state and the operator tables of
// `prec` must already be on the current device.  Throws kifmm::Error.
void evaluate_forest_noalloc(EvalState& st, const HostOps& hops, OpsCache& oc, const void* charges,
                             void* potentials, int n_rhs, bool io_fp64, kifmm_precision prec, void* stream);

// Host-memory convenience: copies charges in, evaluates in FP32 with FP64
// input/output on the default stream, copies potentials out, synchronously.
void evaluate_simple_host(EvalState& st, const HostOps& hops, OpsCache& oc, const double* q,
                          int64_t nsrc, double* pot, int64_t ntgt);

// Copies a cached work buffer to the host as FP64 (see kifmm_debug_buffer).
void debug_buffer(EvalState& st, int which, bool fp64, int n_rhs, double* out, int64_t n_out);

int current_device();

// Device arrays of a single-tree forest that new point positions rewrite in
// place (kifmm_tree_update_points); device -1 when no forest is resident.
struct DevPointView {
  int device = -1;
  int32_t nbox = 0;
  void* box_src = nullptr;  // int2 [nbox]: sorted point range of each box
  void* box_tgt = nullptr;
  void* src64 = nullptr;    // double4 [n]: leaf-frame coordinates
  void* tgt64 = nullptr;
  int32_t* src_perm = nullptr;  // [n]: sorted position -> caller index
  int32_t* tgt_perm = nullptr;
};
DevPointView dev_point_view(const EvalState& st);

// Device state of the point re-sort of one tree (see tree_update.hip): the
// tree's boxes and leaf occupancy on the device, sort scratch, and the last
// accepted sorted order, kept between updates.
struct PendingPoints;
PendingPoints* sort_state_create(const HostTree& T);
// Sorts src (and tgt; null: the sources) into T's leaves on the current
// device and, if st has a forest resident there, rewrites it in place.
// Throws Error EINVAL if a point falls outside the leaves of its kind that
// were occupied, or one of those empties (T, st and the last accepted order
// unchanged).  Synchronises the stream.
void update_points_device(PendingPoints& P, const HostTree& T, EvalState* st, const double* src,
                          const double* tgt, void* stream);
// Copies the last accepted order, coordinates, keys and box ranges into T
// (if it lags them).
void pending_to_host(PendingPoints& P, HostTree& T);
bool pending_stale(const PendingPoints* p);
int pending_device(const PendingPoints* p);
void pending_free(PendingPoints* p);

// The tree of build_host_tree built on the current device from DEVICE
// coordinates src [nsrc][3] and tgt [ntgt][3] (tgt == src: the same array):
// equal to the host build integer for integer; synchronises the stream.
// Throws Error (EINVAL as build_host_tree, or for host pointers).
HostTree* build_tree_device(const double* src, int64_t nsrc, const double* tgt, int64_t ntgt,
                            const kifmm_tree_params& prm, void* stream);

// smallest order at which FP32-bulk modes evaluate L2P/M2P terms in FP64
void set_far_fp64_min_p(int p);
// smallest order at which FP32/FP16 M2L runs on check potentials with the
// operators folded with UC2E
void set_m2l_check_min_p(int p);
// capture evaluations on non-default streams into hipGraphs (default on)
void set_use_graphs(bool on);
// evaluation graphs captured so far in this process
int64_t graph_captures();
void set_near_fork(int v);
// split-precision M2L plans of 65..128 columns on the wide-tile kernel (default off)
void set_m2l_wide(bool on);
void set_m2l_async(bool on);
// operator rows per M2L block: 160, 128, or 0 = the one padding the least
void set_m2l_rows(int rows);
// smallest order at which FP32-accumulating M2L sums its steps in FP64
void set_m2l_fp64_sum_min_p(int p);

// profiling
void set_profiling(bool on);
int n_phases();
const char* phase_name(int i);
void get_phase_times(double* ms, int64_t* launches);

}  // namespace kifmm
