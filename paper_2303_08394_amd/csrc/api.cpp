// The C ABI (include/kifmm.h): argument checks, handle ownership, caching of
// device state, and translation of internal errors into status codes.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "device.hpp"
#include "forest.hpp"
#include "host_tree.hpp"
#include "precompute.hpp"

struct kifmm_tree {
  std::unique_ptr<kifmm::HostTree> host;
  std::unique_ptr<kifmm::EvalState> state;  // single-tree forest + device state
  int state_n = 0;  // operator size the cached forest was built for
  // device state of the point re-sort (the host copy may lag its last order)
  kifmm::PendingPoints* sort = nullptr;
  ~kifmm_tree() {
    if (sort) kifmm::pending_free(sort);
  }
};

struct kifmm_ops {
  std::unique_ptr<kifmm::HostOps> host;
  kifmm::OpsCache cache;
};

namespace kifmm {

static thread_local std::string t_last_error;

kifmm_status fail(kifmm_status st, const std::string& msg) {
  t_last_error = msg;
  return st;
}

// Batch forests, keyed by the ordered tree handles and the operator set.
struct BatchKey {
  std::vector<const kifmm_tree*> trees;
  const kifmm_ops* ops;
  bool operator<(const BatchKey& o) const {
    if (ops != o.ops) return ops < o.ops;
    return trees < o.trees;
  }
};
static std::mutex g_batch_mu;
static std::map<BatchKey, std::unique_ptr<EvalState>> g_batches;

static void purge_batches(const kifmm_tree* t, const kifmm_ops* o) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (auto it = g_batches.begin(); it != g_batches.end();) {
    bool hit = (o && it->first.ops == o) ||
               (t && std::find(it->first.trees.begin(), it->first.trees.end(), t) != it->first.trees.end());
    it = hit ? g_batches.erase(it) : std::next(it);
  }
}

static int plan_width(int n_rhs) { return std::max(1, 64 / n_rhs); }

// tuning (see kifmm_set_tuning)
static std::atomic<int> g_m2l_tile_cols{64};
static int m2l_plan_width(int n_rhs) { return std::max(1, g_m2l_tile_cols.load() / n_rhs); }
static std::atomic<int> g_m2l_split{1};
static std::atomic<int> g_m2l_pair_fill{40};  // percent, at operators of 160 rows
// Tile-fill threshold below which a problem runs M2L pair by pair.  The pair
// scheme moves n_rhs x ld values per pair through HBM on top of the products
// the tiles also compute, so it pays at higher fills as the operators grow:
// the threshold scales with sqrt(ld / 160) (measured crossovers of the split
// modes on surface trees: ~0.4 at p = 6, ~0.57 at p = 8, ~0.73 at p = 10).
static double pair_fill(int n) {
  const int v = g_m2l_pair_fill.load();
  if (v >= 101) return 2.0;  // always
  const int ld = (n + 31) / 32 * 32;
  return v / 100.0 * std::sqrt(ld / 160.0);
}
// The pair buffer holds n_pairs x n_rhs x ld values of up to 8 bytes; plans
// keep it under 64 GiB (beyond that every problem runs gathered tiles).
static int64_t max_pairs(int n, int n_rhs) {
  const int64_t ld = (n + 31) / 32 * 32;
  return (int64_t(64) << 30) / (ld * n_rhs * 8);
}
// a cached plan is reused only if it was cut the way the tuning asks now
static bool plan_current(const HostForest& F, int TB, int TBm, int n, int n_rhs, bool per_level) {
  return F.dc2e.back().TB == TB && F.m2l.TB == TBm && F.m2l.split == (g_m2l_split.load() != 0) &&
         F.pair_fill == pair_fill(n) && F.max_pairs == max_pairs(n, n_rhs) && F.per_level == per_level;
}

// Operators of the screened kernel are tied to a root box size and a depth.
static void check_kernel(const HostTree& T, const HostOps& O) {
  if (O.kernel == 0) return;
  if (T.r0 != O.r0)
    raise(KIFMM_EINVAL, "evaluate: screened-kernel operators were precomputed for another root half-width");
  if (T.depth > O.levels - 1)
    raise(KIFMM_EINVAL, "evaluate: the tree is deeper than the screened-kernel operators' max_level");
}

template <class F>
static kifmm_status guard(F&& f) {
  try {
    f();
    return KIFMM_OK;
  } catch (const Error& e) {
    return fail(e.status, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(KIFMM_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(KIFMM_EDEVICE, e.what());
  } catch (...) {
    return fail(KIFMM_EDEVICE, "unknown internal error");
  }
}

// The host copy of a tree, refreshed first from a device point update.
static const HostTree& host_of(const kifmm_tree* tree) {
  auto* t = const_cast<kifmm_tree*>(tree);
  if (pending_stale(t->sort)) pending_to_host(*t->sort, *t->host);
  return *t->host;
}

static void check_eval_args(const kifmm_tree* tree, const kifmm_ops* ops, int32_t n_rhs,
                            kifmm_precision prec) {
  if (!tree || !ops) raise(KIFMM_EINVAL, "evaluate: null tree or ops handle");
  if (n_rhs < 1) raise(KIFMM_EINVAL, "evaluate: n_rhs must be >= 1");
  if (n_rhs > 64) raise(KIFMM_EUNSUPPORTED, "evaluate: at most 64 right-hand sides per call");
  if (prec < KIFMM_FP64 || prec > KIFMM_FP64_M2L_F16X3) raise(KIFMM_EINVAL, "evaluate: unknown precision");
}

}  // namespace kifmm

using namespace kifmm;

extern "C" {

const char* kifmm_last_error(void) { return t_last_error.c_str(); }

kifmm_status kifmm_build_tree(const double* src_xyz, int64_t n_src, const double* tgt_xyz,
                              int64_t n_tgt, const kifmm_tree_params* params, kifmm_tree** out) {
  if (!out) return fail(KIFMM_EINVAL, "build_tree: null output handle");
  if (!params) return fail(KIFMM_EINVAL, "build_tree: null params");
  return guard([&] {
    auto t = std::make_unique<kifmm_tree>();
    t->host.reset(build_host_tree(src_xyz, n_src, tgt_xyz, n_tgt, *params));
    *out = t.release();
  });
}

kifmm_status kifmm_build_tree_device(const double* src_xyz, int64_t n_src, const double* tgt_xyz,
                                     int64_t n_tgt, const kifmm_tree_params* params, void* hip_stream,
                                     kifmm_tree** out) {
  if (!out) return fail(KIFMM_EINVAL, "build_tree_device: null output handle");
  if (!params) return fail(KIFMM_EINVAL, "build_tree_device: null params");
  return guard([&] {
    auto t = std::make_unique<kifmm_tree>();
    t->host.reset(build_tree_device(src_xyz, n_src, tgt_xyz, n_tgt, *params, hip_stream));
    *out = t.release();
  });
}

kifmm_status kifmm_tree_get_info(const kifmm_tree* tree, kifmm_tree_info* info) {
  if (!tree || !info) return fail(KIFMM_EINVAL, "tree_get_info: null argument");
  const HostTree& T = *tree->host;
  std::memset(info, 0, sizeof(*info));
  info->n_src = T.nsrc;
  info->n_tgt = T.ntgt;
  info->depth = T.depth;
  info->n_boxes = T.nbox;
  info->n_leaves = int32_t(T.leaves.size());
  info->n_u = int64_t(T.items[LIST_U].size());
  info->n_v = int64_t(T.items[LIST_V].size());
  info->n_w = int64_t(T.items[LIST_W].size());
  info->n_x = int64_t(T.items[LIST_X].size());
  for (int d = 0; d < 3; ++d) info->root_center[d] = T.c0[d];
  info->root_halfwidth = T.r0;
  return KIFMM_OK;
}

kifmm_status kifmm_tree_export_boxes(const kifmm_tree* tree, int32_t* level, int32_t* anchor,
                                     int32_t* parent, int32_t* is_leaf, int64_t* src_range,
                                     int64_t* tgt_range) {
  if (!tree) return fail(KIFMM_EINVAL, "tree_export_boxes: null tree");
  return guard([&] {
  const HostTree& T = host_of(tree);
  for (int32_t b = 0; b < T.nbox; ++b) {
    if (level) level[b] = T.level[b];
    if (anchor)
      for (int d = 0; d < 3; ++d) anchor[3 * b + d] = T.anchor[3 * b + d];
    if (parent) parent[b] = T.parent[b];
    if (is_leaf) is_leaf[b] = T.leaf[b];
    if (src_range) {
      src_range[2 * b] = T.sbeg[b];
      src_range[2 * b + 1] = T.send[b];
    }
    if (tgt_range) {
      tgt_range[2 * b] = T.tbeg[b];
      tgt_range[2 * b + 1] = T.tend[b];
    }
  }
  });
}

kifmm_status kifmm_tree_export_list(const kifmm_tree* tree, int32_t which, int64_t* offsets,
                                    int32_t* items) {
  if (!tree || !offsets) return fail(KIFMM_EINVAL, "tree_export_list: null argument");
  if (which < 0 || which > 3) return fail(KIFMM_EINVAL, "tree_export_list: which must be 0..3");
  const HostTree& T = *tree->host;
  std::copy(T.off[which].begin(), T.off[which].end(), offsets);
  if (items) std::copy(T.items[which].begin(), T.items[which].end(), items);
  return KIFMM_OK;
}

kifmm_status kifmm_tree_export_perm(const kifmm_tree* tree, int64_t* src_perm, int64_t* tgt_perm) {
  if (!tree) return fail(KIFMM_EINVAL, "tree_export_perm: null tree");
  return guard([&] {
    const HostTree& T = host_of(tree);
    if (src_perm) std::copy(T.sperm.begin(), T.sperm.end(), src_perm);
    if (tgt_perm) std::copy(T.tperm.begin(), T.tperm.end(), tgt_perm);
  });
}

kifmm_status kifmm_tree_update_points(kifmm_tree* tree, const double* src_xyz, const double* tgt_xyz,
                                      void* hip_stream) {
  return guard([&] {
    if (!tree) raise(KIFMM_EINVAL, "tree_update_points: null tree");
    if (!src_xyz) raise(KIFMM_EINVAL, "tree_update_points: null source coordinates");
    if (tree->sort && pending_device(tree->sort) != current_device()) {
      // the sort state lives on another device: bring the host copy up to
      // date, then start over on this one
      host_of(tree);
      pending_free(tree->sort);
      tree->sort = nullptr;
    }
    if (!tree->sort) tree->sort = sort_state_create(*tree->host);
    EvalState* st = tree->state.get();
    update_points_device(*tree->sort, *tree->host, st, src_xyz, tgt_xyz, hip_stream);
    purge_batches(tree, nullptr);
    if (tgt_xyz && tgt_xyz != src_xyz) tree->host->tgt_is_src = false;
    // no forest on this device took the new order in place: refresh the
    // host copy now, and build the evaluation state from it when needed
    if (!st || dev_point_view(*st).device != current_device()) {
      host_of(tree);
      tree->state.reset();
    }
  });
}

kifmm_status kifmm_precompute_operators(int32_t p, double rcond, kifmm_ops** out) {
  if (!out) return fail(KIFMM_EINVAL, "precompute_operators: null output handle");
  return guard([&] {
    auto o = std::make_unique<kifmm_ops>();
    o->host.reset(build_host_ops(p, rcond));
    *out = o.release();
  });
}

kifmm_status kifmm_precompute_operators_ex(int32_t p, double rcond, int32_t flags, kifmm_ops** out) {
  if (!out) return fail(KIFMM_EINVAL, "precompute_operators_ex: null output handle");
  if (flags & ~int32_t(KIFMM_PRECOMPUTE_DEVICE_SVD))
    return fail(KIFMM_EINVAL, "precompute_operators_ex: unknown flag");
  return guard([&] {
    auto o = std::make_unique<kifmm_ops>();
    o->host.reset(build_host_ops(p, rcond, (flags & KIFMM_PRECOMPUTE_DEVICE_SVD) != 0));
    *out = o.release();
  });
}

kifmm_status kifmm_precompute_operators_screened(int32_t p, double rcond, double kappa,
                                                 double root_halfwidth, int32_t max_level, int32_t flags,
                                                 kifmm_ops** out) {
  if (!out) return fail(KIFMM_EINVAL, "precompute_operators_screened: null output handle");
  if (flags & ~int32_t(KIFMM_PRECOMPUTE_DEVICE_SVD))
    return fail(KIFMM_EINVAL, "precompute_operators_screened: unknown flag");
  if (!(kappa > 0.0)) return fail(KIFMM_EINVAL, "precompute_operators_screened: kappa must be > 0");
  return guard([&] {
    auto o = std::make_unique<kifmm_ops>();
    o->host.reset(build_host_ops(p, rcond, (flags & KIFMM_PRECOMPUTE_DEVICE_SVD) != 0, kappa, root_halfwidth,
                                 max_level));
    *out = o.release();
  });
}

kifmm_status kifmm_ops_save(const kifmm_ops* ops, const char* path) {
  if (!ops) return fail(KIFMM_EINVAL, "ops_save: null ops");
  return guard([&] { save_host_ops(*ops->host, path); });
}

kifmm_status kifmm_ops_load(const char* path, int32_t p, double rcond, kifmm_ops** out) {
  if (!out) return fail(KIFMM_EINVAL, "ops_load: null output handle");
  return guard([&] {
    auto o = std::make_unique<kifmm_ops>();
    o->host.reset(load_host_ops(path, p, rcond));
    *out = o.release();
  });
}

int32_t kifmm_ops_n(const kifmm_ops* ops) { return ops ? ops->host->n : -1; }

int32_t kifmm_ops_levels(const kifmm_ops* ops) { return ops ? ops->host->levels : -1; }

kifmm_status kifmm_ops_export(const kifmm_ops* ops, int32_t which, double* out, int64_t n_out) {
  if (!ops || !out) return fail(KIFMM_EINVAL, "ops_export: null argument");
  const HostOps& H = *ops->host;
  std::vector<double> off;
  const std::vector<double>* v = nullptr;
  switch (which) {
    case 0: v = &H.surf; break;
    case 1: v = &H.uc2e; break;
    case 2: v = &H.dc2e; break;
    case 3: v = &H.m2m; break;
    case 4: v = &H.l2l; break;
    case 5: v = &H.m2l; break;
    case 6:
      off.assign(H.m2l_offset.begin(), H.m2l_offset.end());
      v = &off;
      break;
    default: return fail(KIFMM_EINVAL, "ops_export: which must be 0..6");
  }
  if (n_out < int64_t(v->size())) return fail(KIFMM_EINVAL, "ops_export: output too small");
  std::copy(v->begin(), v->end(), out);
  return KIFMM_OK;
}

}  // extern "C"

static kifmm_status evaluate_impl(const kifmm_tree* tree, const kifmm_ops* ops, const void* charges,
                                  int32_t n_rhs, void* potentials, int32_t io_fp64,
                                  kifmm_precision precision, void* hip_stream, bool grad) {
  return guard([&] {
    check_eval_args(tree, ops, n_rhs, precision);
    if (!charges || !potentials) raise(KIFMM_EINVAL, "evaluate: null charges or potentials");
    auto* t = const_cast<kifmm_tree*>(tree);
    const int TB = plan_width(n_rhs), TBm = m2l_plan_width(n_rhs);
    const int n = ops->host->n;
    const bool per_level = ops->host->kernel != 0;
    check_kernel(*t->host, *ops->host);
    bool rebuild =
        !t->state || t->state_n != n || !plan_current(*t->state->host, TB, TBm, n, n_rhs, per_level);
    if (pending_stale(t->sort) && (rebuild || dev_point_view(*t->state).device != current_device())) {
      // the device-updated points live only in the resident forest: a new
      // forest (new plans, or another device) is built from the host copy
      host_of(t);
      rebuild = true;
    }
    if (rebuild) {
      // the new state replaces the old one only once its plans exist
      std::unique_ptr<EvalState> st(new EvalState());
      const HostTree* one = t->host.get();
      st->host.reset(build_forest(&one, 1, *ops->host, TB, TBm, g_m2l_split.load() != 0, pair_fill(n),
                                  max_pairs(n, n_rhs), per_level));
      t->state = std::move(st);
      t->state_n = ops->host->n;
    }
    check_operand_limits(t->state->host->nbox, n_rhs, n);
    const void* q[1] = {charges};
    void* o[1] = {potentials};
    evaluate_forest(*t->state, *ops->host, const_cast<kifmm_ops*>(ops)->cache, q, o, n_rhs,
                    io_fp64 != 0, precision, hip_stream, grad);
  });
}

extern "C" {

kifmm_status kifmm_evaluate(const kifmm_tree* tree, const kifmm_ops* ops, const void* charges,
                            int32_t n_rhs, void* potentials, int32_t io_fp64,
                            kifmm_precision precision, void* hip_stream) {
  return evaluate_impl(tree, ops, charges, n_rhs, potentials, io_fp64, precision, hip_stream, false);
}

kifmm_status kifmm_evaluate_noalloc(const kifmm_tree* tree, const kifmm_ops* ops, const void* charges,
                                    int32_t n_rhs, void* potentials, int32_t io_fp64,
                                    kifmm_precision precision, void* hip_stream) {
  return guard([&] {
    check_eval_args(tree, ops, n_rhs, precision);
    if (!charges || !potentials) raise(KIFMM_EINVAL, "evaluate_noalloc: null charges or potentials");
    auto* t = const_cast<kifmm_tree*>(tree);
    const int n = ops->host->n;
    check_kernel(*t->host, *ops->host);
    // the forest (plans and device arrays) must be the one kifmm_evaluate
    // would use now: building another allocates
    if (!t->state || t->state_n != n ||
        !plan_current(*t->state->host, plan_width(n_rhs), m2l_plan_width(n_rhs), n, n_rhs, ops->host->kernel != 0))
      raise(KIFMM_EINVAL, "evaluate_noalloc: no evaluation state for these operators, right-hand sides and "
                          "tuning (run kifmm_evaluate once)");
    if (pending_stale(t->sort) && dev_point_view(*t->state).device != current_device())
      raise(KIFMM_EINVAL, "evaluate_noalloc: updated points are not on this device (run kifmm_evaluate once)");
    check_operand_limits(t->state->host->nbox, n_rhs, n);
    evaluate_forest_noalloc(*t->state, *ops->host, const_cast<kifmm_ops*>(ops)->cache, charges, potentials,
                            n_rhs, io_fp64 != 0, precision, hip_stream);
  });
}

kifmm_status kifmm_evaluate_gradient(const kifmm_tree* tree, const kifmm_ops* ops,
                                     const void* charges, int32_t n_rhs, void* out,
                                     int32_t io_fp64, kifmm_precision precision,
                                     void* hip_stream) {
  return evaluate_impl(tree, ops, charges, n_rhs, out, io_fp64, precision, hip_stream, true);
}

kifmm_status kifmm_evaluate_batch(int32_t n_prob, const kifmm_tree* const* trees,
                                  const kifmm_ops* ops, const void* const* charges,
                                  void* const* potentials, int32_t io_fp64,
                                  kifmm_precision precision, void* hip_stream) {
  return guard([&] {
    if (n_prob < 1) raise(KIFMM_EINVAL, "evaluate_batch: n_prob must be >= 1");
    if (!trees || !charges || !potentials) raise(KIFMM_EINVAL, "evaluate_batch: null array");
    for (int k = 0; k < n_prob; ++k) {
      check_eval_args(trees[k], ops, 1, precision);
      if (!charges[k] || !potentials[k]) raise(KIFMM_EINVAL, "evaluate_batch: null buffer");
    }
    BatchKey key{std::vector<const kifmm_tree*>(trees, trees + n_prob), ops};
    EvalState* st = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_batch_mu);
      auto& slot = g_batches[key];
      const int n = ops->host->n;
      const bool per_level = ops->host->kernel != 0;
      for (int k = 0; k < n_prob; ++k) check_kernel(*trees[k]->host, *ops->host);
      if (slot && !plan_current(*slot->host, plan_width(1), m2l_plan_width(1), n, 1, per_level)) slot.reset();
      if (!slot) {
        std::vector<const HostTree*> hts(n_prob);
        for (int k = 0; k < n_prob; ++k) hts[k] = &host_of(trees[k]);
        auto s = std::make_unique<EvalState>();
        s->host.reset(build_forest(hts.data(), n_prob, *ops->host, plan_width(1), m2l_plan_width(1),
                                   g_m2l_split.load() != 0, pair_fill(n), max_pairs(n, 1), per_level));
        slot = std::move(s);
      }
      st = slot.get();
    }
    check_operand_limits(st->host->nbox, 1, ops->host->n);
    evaluate_forest(*st, *ops->host, const_cast<kifmm_ops*>(ops)->cache, charges, potentials, 1,
                    io_fp64 != 0, precision, hip_stream);
  });
}

kifmm_status kifmm_evaluate_simple(const double* src, const double* q, int64_t n_src,
                                   const double* tgt, int64_t n_tgt, int32_t p, double* pot) {
  if (!src || !q || !tgt || !pot) return fail(KIFMM_EINVAL, "evaluate_simple: null argument");
  return guard([&] {
    kifmm_tree_params prm{};
    prm.uniform_depth = -1;
    prm.ncrit = 64;
    prm.max_depth = 20;
    prm.balance = 1;
    std::unique_ptr<HostTree> ht(build_host_tree(src, n_src, tgt, n_tgt, prm));
    std::unique_ptr<HostOps> ho(build_host_ops(p, 1e-9));
    for (int64_t i = 0; i < n_src; ++i)
      if (!std::isfinite(q[i])) raise(KIFMM_EINVAL, "evaluate_simple: non-finite charge");
    EvalState st;
    const HostTree* one = ht.get();
    st.host.reset(build_forest(&one, 1, *ho, plan_width(1), m2l_plan_width(1), g_m2l_split.load() != 0,
                              pair_fill(ho->n), max_pairs(ho->n, 1)));
    OpsCache oc;
    evaluate_simple_host(st, *ho, oc, q, n_src, pot, n_tgt);
  });
}

kifmm_status kifmm_debug_buffer(const kifmm_tree* tree, int32_t which, int32_t fp64,
                                int32_t n_rhs, double* out, int64_t n_out) {
  if (!tree || !out) return fail(KIFMM_EINVAL, "debug_buffer: null argument");
  return guard([&] {
    if (!tree->state) raise(KIFMM_EINVAL, "debug_buffer: no evaluation has run on this tree");
    debug_buffer(*tree->state, which, fp64 != 0, n_rhs, out, n_out);
  });
}

void kifmm_tree_destroy(kifmm_tree* tree) {
  if (!tree) return;
  purge_batches(tree, nullptr);
  delete tree;
}

void kifmm_ops_destroy(kifmm_ops* ops) {
  if (!ops) return;
  purge_batches(nullptr, ops);
  delete ops;
}

static kifmm_status set_tuning_impl(const char* key, int32_t value);

// The values of the knobs whose state lives with the evaluation kernels, as
// last set here (their defaults until then), for kifmm_get_tuning.
static std::atomic<int> g_near_fork_set{4}, g_graph_set{1}, g_fp64_sum_min_p_set{10},
    g_check_min_p_set{10}, g_far_fp64_min_p_set{10}, g_m2l_wide_set{0}, g_m2l_rows_set{0}, g_m2l_async_set{1};

static std::atomic<int>* tuning_slot(const char* key) {
  static const struct {
    const char* key;
    std::atomic<int>* v;
  } slots[] = {{"m2l_tile_cols", &g_m2l_tile_cols},
               {"m2l_pair_fill", &g_m2l_pair_fill},
               {"m2l_split", &g_m2l_split},
               {"near_fork", &g_near_fork_set},
               {"graph", &g_graph_set},
               {"m2l_fp64_sum_min_p", &g_fp64_sum_min_p_set},
               {"m2l_check_min_p", &g_check_min_p_set},
               {"far_fp64_min_p", &g_far_fp64_min_p_set},
               {"m2l_wide", &g_m2l_wide_set},
               {"m2l_rows", &g_m2l_rows_set},
               {"m2l_async", &g_m2l_async_set}};
  for (const auto& sl : slots)
    if (std::strcmp(key, sl.key) == 0) return sl.v;
  return nullptr;
}

kifmm_status kifmm_get_tuning(const char* key, int32_t* value) {
  if (!key || !value) return fail(KIFMM_EINVAL, "get_tuning: null argument");
  std::atomic<int>* v = tuning_slot(key);
  if (!v) return fail(KIFMM_EINVAL, std::string("get_tuning: unknown key ") + key);
  *value = v->load();
  return KIFMM_OK;
}

kifmm_status kifmm_set_tuning(const char* key, int32_t value) {
  if (!key) return fail(KIFMM_EINVAL, "set_tuning: null key");
  const kifmm_status st = set_tuning_impl(key, value);
  if (st == KIFMM_OK) *tuning_slot(key) = value;
  return st;
}

static kifmm_status set_tuning_impl(const char* key, int32_t value) {
  if (std::strcmp(key, "m2l_tile_cols") == 0) {
    if (value != 64 && value != 96 && value != 128 && value != 160 && value != 192)
      return fail(KIFMM_EINVAL, "set_tuning: m2l_tile_cols must be 64, 96, 128, 160 or 192");
    g_m2l_tile_cols = value;
    return KIFMM_OK;
  }
  if (std::strcmp(key, "m2l_pair_fill") == 0) {
    if (value < 0 || value > 101) return fail(KIFMM_EINVAL, "set_tuning: m2l_pair_fill must be 0..101");
    g_m2l_pair_fill = value;
    return KIFMM_OK;
  }
  if (std::strcmp(key, "m2l_split") == 0) {
    if (value != 0 && value != 1) return fail(KIFMM_EINVAL, "set_tuning: m2l_split must be 0 or 1");
    g_m2l_split = value;
    return KIFMM_OK;
  }
  if (std::strcmp(key, "near_fork") == 0) {
    if (value < 0 || value > 4) return fail(KIFMM_EINVAL, "set_tuning: near_fork must be 0..4");
    set_near_fork(value);
    return KIFMM_OK;
  }
  if (std::strcmp(key, "graph") == 0) {
    if (value != 0 && value != 1) return fail(KIFMM_EINVAL, "set_tuning: graph must be 0 or 1");
    set_use_graphs(value != 0);
    return KIFMM_OK;
  }
  if (std::strcmp(key, "m2l_fp64_sum_min_p") == 0) {
    if (value < 2 || value > 17) return fail(KIFMM_EINVAL, "set_tuning: m2l_fp64_sum_min_p must be in [2, 17]");
    set_m2l_fp64_sum_min_p(value);
    return KIFMM_OK;
  }
  if (std::strcmp(key, "m2l_check_min_p") == 0) {
    if (value < 2 || value > 17) return fail(KIFMM_EINVAL, "set_tuning: m2l_check_min_p must be in [2, 17]");
    set_m2l_check_min_p(value);
    return KIFMM_OK;
  }
  if (std::strcmp(key, "far_fp64_min_p") == 0) {
    if (value < 2 || value > 17) return fail(KIFMM_EINVAL, "set_tuning: far_fp64_min_p must be in [2, 17]");
    set_far_fp64_min_p(value);
    return KIFMM_OK;
  }
  if (std::strcmp(key, "m2l_rows") == 0) {
    if (value != 0 && value != 128 && value != 160)
      return fail(KIFMM_EINVAL, "set_tuning: m2l_rows must be 0, 128 or 160");
    set_m2l_rows(value);
    return KIFMM_OK;
  }
  if (std::strcmp(key, "m2l_wide") == 0) {
    if (value != 0 && value != 1) return fail(KIFMM_EINVAL, "set_tuning: m2l_wide must be 0 or 1");
    set_m2l_wide(value != 0);
    return KIFMM_OK;
  }
  if (std::strcmp(key, "m2l_async") == 0) {
    if (value != 0 && value != 1) return fail(KIFMM_EINVAL, "set_tuning: m2l_async must be 0 or 1");
    set_m2l_async(value != 0);
    return KIFMM_OK;
  }
  return fail(KIFMM_EINVAL, std::string("set_tuning: unknown key ") + key);
}

kifmm_status kifmm_set_profiling(int32_t enable) {
  set_profiling(enable != 0);
  return KIFMM_OK;
}
int64_t kifmm_graph_captures(void) { return graph_captures(); }

void kifmm_debug_fail_allocations(int64_t after) { alloc_fail_counter() = after < 0 ? -1 : after; }
int32_t kifmm_n_phases(void) { return n_phases(); }
const char* kifmm_phase_name(int32_t i) { return phase_name(i); }
kifmm_status kifmm_get_phase_times(double* ms, int64_t* launches) {
  return guard([&] { get_phase_times(ms, launches); });
}

}  // extern "C"
