// Host-side code of the library (tree and interaction lists, operator
// precompute and its cache file, the forest's launch plans) driven under
// AddressSanitizer and UndefinedBehaviorSanitizer.  Built with g++ from the
// host sources only (no HIP): the two device-side precompute entry points are
// replaced by stubs that are never called (device_svd stays off).  Prints
// "host_sanitize ok" after the checks; any sanitizer report aborts first.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <random>
#include <string>
#include <vector>

#include "common.hpp"
#include "forest.hpp"
#include "host_tree.hpp"
#include "precompute.hpp"

namespace kifmm {
std::vector<double> m2l_check_form_device(const HostOps&) { raise(KIFMM_EUNSUPPORTED, "no device here"); }
std::vector<double> pinv_truncated_device(const double*, int, double, int*) {
  raise(KIFMM_EUNSUPPORTED, "no device here");
}
}  // namespace kifmm

using namespace kifmm;

static int failures = 0;
#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++failures;                                                   \
    }                                                               \
  } while (0)

static std::vector<double> cube(int n, unsigned seed) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::vector<double> x(3 * size_t(n));
  for (auto& v : x) v = u(g);
  return x;
}

static std::vector<double> sphere(int n, unsigned seed, double jitter) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> x(3 * size_t(n));
  for (int i = 0; i < n; ++i) {
    double a = nd(g), b = nd(g), c = nd(g);
    const double s = (1.0 + jitter * nd(g)) / std::sqrt(a * a + b * b + c * c);
    x[3 * i] = a * s, x[3 * i + 1] = b * s, x[3 * i + 2] = c * s;
  }
  return x;
}

static kifmm_tree_params params(int depth, int ncrit, int maxd, bool unit_cube) {
  kifmm_tree_params p{};
  p.uniform_depth = depth;
  p.ncrit = ncrit;
  p.max_depth = maxd;
  p.balance = 1;
  if (unit_cube) {
    p.root_center[0] = p.root_center[1] = p.root_center[2] = 0.5;
    p.root_halfwidth = 0.5;
  }
  return p;
}

// every source point lies in exactly one leaf, inside the leaf's range
static void check_tree(const HostTree& t) {
  CHECK(t.nbox > 0 && int(t.level.size()) == t.nbox);
  int64_t covered = 0;
  for (int32_t b : t.leaves) covered += t.nsrc_of(b);
  CHECK(covered == t.nsrc);
  for (int k = 0; k < 4; ++k) CHECK(t.off[k].size() == size_t(t.nbox) + 1);
}

int main() {
  // trees: uniform, adaptive on a surface with and without jitter,
  // separate targets, a single point, coincident points
  std::vector<std::unique_ptr<HostTree>> trees;
  {
    auto x = cube(20000, 1);
    trees.emplace_back(build_host_tree(x.data(), 20000, x.data(), 20000, params(3, 0, 0, true)));
  }
  {
    auto x = sphere(30000, 2, 1e-3);
    trees.emplace_back(build_host_tree(x.data(), 30000, x.data(), 30000, params(-1, 32, 12, false)));
  }
  {
    auto x = sphere(12000, 3, 0.0);
    trees.emplace_back(build_host_tree(x.data(), 12000, x.data(), 12000, params(-1, 24, 14, false)));
  }
  {
    auto x = cube(5000, 4), y = cube(3000, 5);
    trees.emplace_back(build_host_tree(x.data(), 5000, y.data(), 3000, params(-1, 16, 10, true)));
  }
  {
    double one[3] = {0.25, 0.5, 0.75};
    trees.emplace_back(build_host_tree(one, 1, one, 1, params(-1, 8, 6, true)));
  }
  {
    std::vector<double> same(3 * 200, 0.3);
    trees.emplace_back(build_host_tree(same.data(), 200, same.data(), 200, params(-1, 8, 5, true)));
  }
  for (auto& t : trees) check_tree(*t);

  // bad inputs are errors, not crashes
  {
    double nanp[3] = {0.1, NAN, 0.2};
    bool threw = false;
    try {
      std::unique_ptr<HostTree> t(build_host_tree(nanp, 1, nanp, 1, params(-1, 8, 6, false)));
    } catch (const Error& e) {
      threw = e.status == KIFMM_EINVAL;
    }
    CHECK(threw);
    threw = false;
    try {
      auto x = cube(10, 6);
      std::unique_ptr<HostTree> t(build_host_tree(x.data(), 10, x.data(), 10, params(-1, 8, 21, false)));
    } catch (const Error& e) {
      threw = e.status == KIFMM_EINVAL;
    }
    CHECK(threw);
  }

  // injected allocation failures: ENOMEM, nothing leaked (leak detection on),
  // the hook disarmed after firing
  {
    auto enomem = [](auto&& f) {
      alloc_fail_counter() = 0;
      bool threw = false;
      try {
        f();
      } catch (const Error& e) {
        threw = e.status == KIFMM_ENOMEM;
      }
      return threw && alloc_fail_counter() == -1;
    };
    auto x = cube(3000, 9);
    CHECK(enomem([&] { std::unique_ptr<HostTree> t(build_host_tree(x.data(), 3000, x.data(), 3000, params(-1, 16, 8, true))); }));
    CHECK(enomem([&] { std::unique_ptr<HostOps> o(build_host_ops(3, 1e-9)); }));
    std::unique_ptr<HostOps> o3(build_host_ops(3, 1e-9));
    const HostTree* one = trees[0].get();
    CHECK(enomem([&] { std::unique_ptr<HostForest> f(build_forest(&one, 1, *o3, 64, 64, true, 0.4, 1 << 30)); }));
    alloc_fail_counter() = 3;  // armed, not reached by one build
    std::unique_ptr<HostTree> t(build_host_tree(x.data(), 3000, x.data(), 3000, params(-1, 16, 8, true)));
    CHECK(alloc_fail_counter() == 2);
    alloc_fail_counter() = -1;
  }

  // density columns the GEMM can address with 32-bit counts of 16-byte units
  {
    auto refused = [](int64_t nbox, int n_rhs, int n) {
      try {
        check_operand_limits(nbox, n_rhs, n);
      } catch (const Error& e) {
        return e.status == KIFMM_EUNSUPPORTED;
      }
      return false;
    };
    // 1M points at depth 5 (37,449 boxes), p = 10 (n = 488), 64 right-hand
    // sides: 2.5e9 split elements, past 2^31, but 1.2e9 units of 16 bytes
    CHECK(!refused(37449, 64, 488));
    // p = 16 (n = 1352, ld = 1376), 64 right-hand sides: the largest box
    // count that fits, and one more
    const int64_t ld16 = 1376, cap = (int64_t(1) << 36) / (64 * ld16 * 8) - 1;
    CHECK(!refused(cap, 64, 1352));
    CHECK(refused(cap + 1, 64, 1352));
    CHECK(refused(-1, 1, 152) && refused(10, 0, 152));
  }

  // operators, the cache file and its rejections
  std::unique_ptr<HostOps> ops(build_host_ops(4, 1e-9));
  const std::string path = "host_sanitize_ops.bin";
  save_host_ops(*ops, path.c_str());
  {
    std::unique_ptr<HostOps> back(load_host_ops(path.c_str(), 4, 1e-9));
    CHECK(back->uc2e == ops->uc2e && back->m2l == ops->m2l && back->m2m == ops->m2m);
    bool threw = false;
    try {
      std::unique_ptr<HostOps> other(load_host_ops(path.c_str(), 5, 1e-9));
    } catch (const Error&) {
      threw = true;
    }
    CHECK(threw);
    // a truncated file
    if (FILE* w = std::fopen(path.c_str(), "wb")) {
      std::fputs("KIFM", w);
      std::fclose(w);
    }
    threw = false;
    try {
      std::unique_ptr<HostOps> bad(load_host_ops(path.c_str(), 4, 1e-9));
    } catch (const Error&) {
      threw = true;
    }
    CHECK(threw);
    std::remove(path.c_str());
  }
  std::unique_ptr<HostOps> scr(build_host_ops(3, 1e-9, false, 5.0, 1.0, 16));
  CHECK(scr->levels > 0);

  // plans: one tree, a batch, both M2L schemes, split on and off, all widths
  for (auto& t : trees) {
    const HostTree* one = t.get();
    for (int TBm : {64, 128, 192})
      for (double fill : {0.0, 0.4, 1.01})
        for (bool split : {true, false}) {
          std::unique_ptr<HostForest> f(build_forest(&one, 1, *ops, 64, TBm, split, fill, int64_t(1) << 40));
          CHECK(f->nprob == 1);
        }
  }
  {
    std::vector<const HostTree*> all;
    for (auto& t : trees) all.push_back(t.get());
    std::unique_ptr<HostForest> f(build_forest(all.data(), int(all.size()), *ops, 64, 64, true, 0.4, int64_t(1) << 40));
    CHECK(f->nprob == int(all.size()));
    std::unique_ptr<HostForest> g(build_forest(all.data(), int(all.size()), *scr, 64, 64, true, 0.4, int64_t(1) << 40,
                                               true));
    CHECK(g->per_level);
  }
  if (failures) {
    std::fprintf(stderr, "host_sanitize: %d failed checks\n", failures);
    return 1;
  }
  std::printf("host_sanitize ok\n");
  return 0;
}
