// KIFMM evaluation on one CDNA4 GPU: device state, kernels and the pipeline.
//
// Pipeline (sections "The Fast Multipole Method" and "Computational
// structure of FMM operators"): gather charges into Morton order; P2M at the
// leaves; M2M + UC2E level by level upward; P2L (X lists) and M2L (V lists)
// for all levels in one launch each; L2L + DC2E level by level downward; one
// fused leaf kernel for L2P + M2P (W lists) + near field (U lists) with the
// per-target sum in FP64; scatter back to the caller's order.
//
// Units: coordinates are relative to a box centre in units of its half-width
// r.  A "scaled" check potential is r times the check potential; with it every
// translation operator is the same at all levels (the kernel is homogeneous
// of degree -1), and the particle kernels work on O(1) numbers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <type_traits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "device.hpp"
#include "hip_check.hpp"

namespace kifmm {

static constexpr double kInv4Pi = 0.0795774715459476678844418816863;
static constexpr double kRin = 1.05, kRout = 2.95;
// FP16 split M2L: operators are stored times 2^kF16OpExp (their entries are
// O(1e-2), so both parts stay normal FP16 numbers); densities are scaled by
// 2^e with e chosen from their largest magnitude so that it maps below 2^14.
constexpr int kF16OpExp = 10;

// Exponent e of the FP16 density scale 2^e: the largest magnitude (absmax
// word, float bits) lands in [2^13, 2^14).
__device__ inline int f16_density_exp(const unsigned* absmax) {
  const float mx = __uint_as_float(*absmax);
  int e = 0;
  if (mx > 0.0f) {
    (void)frexpf(mx, &e);  // mx in [2^(e-1), 2^e)
    e = 14 - e;
  }
  return e;
}

// ------------------------------------------------------------------------
// device state
// ------------------------------------------------------------------------

// Every DevOps gets a new generation number: a captured evaluation graph is
// keyed by it, never by the DevOps address, which a later operator set can
// reuse after this one is destroyed.
static std::atomic<uint64_t> g_ops_generation{0};

struct DevOps {
  int n = 0, ld = 0, p = 0;
  uint64_t generation = ++g_ops_generation;
  // table sets: 1 (Laplace), or one per level (screened kernel, exp(-kappa d)
  // / (4 pi d)); every table below holds `levels` sets back to back
  int levels = 1;
  double kappa = 0.0;
  double *uc2e = nullptr, *dc2e = nullptr;               // [ld][ld]
  float *m2m32 = nullptr, *l2l32 = nullptr, *m2l32 = nullptr;  // [k][ld][ld]
  double *m2m64 = nullptr, *l2l64 = nullptr, *m2l64 = nullptr;
  // split tables, [316][ld][2][ld]: each operator row as high part, low part
  uint16_t* m2l_b = nullptr;    // BF16 parts of M2L
  uint16_t* m2l_h = nullptr;    // FP16 parts of 2^10 M2L
  // check-potential form (M2L folded with UC2E): FP32 and FP16 parts
  float* m2lc32 = nullptr;
  uint16_t* m2lc_h = nullptr;
  double4* surf = nullptr;                               // [n] unit-cube surface
  std::vector<void*> allocs;
  ~DevOps() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

struct DevWork {
  int n_rhs = 0;
  bool fp64 = false;
  void* qs = nullptr;       // [n_rhs][nsrc]
  void* up_chk = nullptr;   // [nbox][n_rhs][ld]
  void* up_eq = nullptr;
  void* dn_chk = nullptr;
  void* dn_eq = nullptr;
  // FP32-bulk gradient evaluations: the downward check potentials in FP64
  // from L2L on (see pipeline)
  double* dn_chk64 = nullptr;
  double* pot = nullptr;    // [n_rhs][ntgt]
  unsigned* absmax = nullptr;  // [4] scratch word for the FP16 density scale
  size_t col_bytes = 0;
  void* split = nullptr;       // split-precision M2L operand, up to 3 16-bit parts per element
  size_t split_bytes = 0;
  void* pairs = nullptr;       // pair-by-pair M2L products [n_pairs][n_rhs][ld]
  size_t pair_bytes = 0;
  std::vector<void*> allocs;
  ~DevWork() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

struct DevForest {
  int32_t nbox = 0, nprob = 0, depth = 0;
  int64_t nsrc = 0, ntgt = 0;
  int ld = 0, n = 0;
  int4* box_geo = nullptr;
  double* box_r = nullptr;
  int2 *box_src = nullptr, *box_tgt = nullptr;
  double4 *src64 = nullptr, *tgt64 = nullptr;
  int32_t *src_perm = nullptr, *tgt_perm = nullptr;
  int64_t *src_off = nullptr, *tgt_off = nullptr;
  int32_t *p2m_boxes = nullptr, *leaf_boxes = nullptr, *u_off = nullptr, *u_items = nullptr;
  int32_t *w_off = nullptr, *w_items = nullptr, *x_boxes = nullptr, *x_off = nullptr, *x_items = nullptr;
  int32_t n_p2m = 0, n_leaf = 0, n_x = 0;
  int64_t max_src_per_prob = 0, max_tgt_per_prob = 0;
  std::vector<DevPlan> m2m, uc2e, l2l, dc2e;
  std::vector<int32_t*> m2m_sum;     // per level [n][9], see HostForest
  std::vector<int32_t> n_m2m_sum;
  DevPlan m2l;
  // pair-by-pair M2L of sparse problems (see HostForest::m2l_pair)
  DevPlan m2l_pair;
  int32_t *pair_tgt = nullptr, *pair_off = nullptr, *pair_items = nullptr;
  int32_t n_pair_tgt = 0;
  int64_t n_pairs = 0;
  std::vector<void*> allocs;
  std::map<std::pair<int, int>, DevWork*> work;  // (fp64, n_rhs)
  // the last captured evaluation and what it was captured for
  hipGraphExec_t graph = nullptr;
  std::vector<const void*> graph_key;
  ~DevForest() {
    if (graph) (void)hipGraphExecDestroy(graph);
    for (auto& w : work) delete w.second;
    for (void* p : allocs) (void)hipFree(p);
  }
};

EvalState::~EvalState() { delete forest; }

DevPointView dev_point_view(const EvalState& st) {
  DevPointView v;
  const DevForest* F = st.forest;
  if (!F || F->nprob != 1) return v;
  v.device = st.device;
  v.nbox = F->nbox;
  v.box_src = F->box_src;
  v.box_tgt = F->box_tgt;
  v.src64 = F->src64;
  v.tgt64 = F->tgt64;
  v.src_perm = F->src_perm;
  v.tgt_perm = F->tgt_perm;
  return v;
}
OpsCache::~OpsCache() {
  for (auto& kv : per_device) delete kv.second;
}

int current_device() {
  int d = 0;
  HIPCHECK(hipGetDevice(&d));
  return d;
}

template <class T>
static T* dev_alloc(std::vector<void*>& allocs, size_t count) {
  if (count == 0) count = 1;
  alloc_hook("hipMalloc");
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) raise(KIFMM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  allocs.push_back(p);
  return static_cast<T*>(p);
}

template <class D, class S>
static D* dev_upload(std::vector<void*>& allocs, const std::vector<S>& v) {
  static_assert(sizeof(D) % sizeof(S) == 0 || sizeof(S) % sizeof(D) == 0, "layout");
  size_t bytes = v.size() * sizeof(S);
  size_t count = (bytes + sizeof(D) - 1) / sizeof(D);
  D* p = dev_alloc<D>(allocs, count);
  if (bytes) HIPCHECK(hipMemcpy(p, v.data(), bytes, hipMemcpyHostToDevice));
  return p;
}

// Absent sources (-1) become the zero box, so the GEMM never branches on them.
static DevPlan upload_plan(std::vector<void*>& allocs, const Plan& P, int32_t zero_box) {
  DevPlan d;
  d.ntile = P.ntile;
  d.TB = P.TB;
  d.nstep = P.nstep();
  d.useful_pairs = P.useful_pairs;
  d.atomic = P.atomic;
  for (int32_t t = 0; t < P.ntile; ++t)
    d.max_tile_steps = std::max(d.max_tile_steps, P.step_beg[t + 1] - P.step_beg[t]);
  if (P.ntile == 0) return d;
  d.tile_cols = dev_upload<int32_t>(allocs, P.tile_cols);
  d.step_beg = dev_upload<int32_t>(allocs, P.step_beg);
  d.step_op = dev_upload<int32_t>(allocs, P.step_op);
  std::vector<int32_t> src(P.step_src);
  for (auto& v : src)
    if (v < 0) v = zero_box;
  d.step_src = dev_upload<int32_t>(allocs, src);
  return d;
}

// Leading dimension of density columns and operators: n rounded up to the
// GEMM k-chunk (32), padding rows and columns zero.
static int round32(int n) { return (n + 31) / 32 * 32; }

static DevForest* upload_forest(const HostForest& F, int n) {
  auto* D = new DevForest();
  try {
    D->nbox = F.nbox;
    D->nprob = F.nprob;
    D->depth = F.depth;
    D->nsrc = F.nsrc;
    D->ntgt = F.ntgt;
    D->n = n;
    D->ld = round32(n);
    auto& A = D->allocs;
    D->box_geo = dev_upload<int4>(A, F.box_geo);
    D->box_r = dev_upload<double>(A, F.box_r);
    D->box_src = dev_upload<int2>(A, F.box_src);
    D->box_tgt = dev_upload<int2>(A, F.box_tgt);
    D->src64 = dev_upload<double4>(A, F.src_f64);
    D->tgt64 = dev_upload<double4>(A, F.tgt_f64);
    D->src_perm = dev_upload<int32_t>(A, F.src_perm);
    D->tgt_perm = dev_upload<int32_t>(A, F.tgt_perm);
    D->src_off = dev_upload<int64_t>(A, F.src_off);
    D->tgt_off = dev_upload<int64_t>(A, F.tgt_off);
    for (int k = 0; k < F.nprob; ++k) {
      D->max_src_per_prob = std::max(D->max_src_per_prob, F.src_off[k + 1] - F.src_off[k]);
      D->max_tgt_per_prob = std::max(D->max_tgt_per_prob, F.tgt_off[k + 1] - F.tgt_off[k]);
    }
    D->p2m_boxes = dev_upload<int32_t>(A, F.p2m_boxes);
    D->n_p2m = int32_t(F.p2m_boxes.size());
    D->leaf_boxes = dev_upload<int32_t>(A, F.leaf_boxes);
    D->n_leaf = int32_t(F.leaf_boxes.size());
    D->u_off = dev_upload<int32_t>(A, F.u_off);
    D->u_items = dev_upload<int32_t>(A, F.u_items);
    D->w_off = dev_upload<int32_t>(A, F.w_off);
    D->w_items = dev_upload<int32_t>(A, F.w_items);
    D->x_boxes = dev_upload<int32_t>(A, F.x_boxes);
    D->n_x = int32_t(F.x_boxes.size());
    D->x_off = dev_upload<int32_t>(A, F.x_off);
    D->x_items = dev_upload<int32_t>(A, F.x_items);
    for (auto& p : F.m2m) D->m2m.push_back(upload_plan(A, p, F.nbox));
    for (auto& t : F.m2m_sum) {
      D->m2m_sum.push_back(t.empty() ? nullptr : dev_upload<int32_t>(A, t));
      D->n_m2m_sum.push_back(int32_t(t.size() / 9));
    }
    for (auto& p : F.uc2e) D->uc2e.push_back(upload_plan(A, p, F.nbox));
    for (auto& p : F.l2l) D->l2l.push_back(upload_plan(A, p, F.nbox));
    for (auto& p : F.dc2e) D->dc2e.push_back(upload_plan(A, p, F.nbox));
    D->m2l = upload_plan(A, F.m2l, F.nbox);
    D->m2l_pair = upload_plan(A, F.m2l_pair, F.nbox);
    D->n_pairs = F.n_pairs;
    D->n_pair_tgt = int32_t(F.pair_tgt.size());
    if (D->n_pair_tgt > 0) {
      D->pair_tgt = dev_upload<int32_t>(A, F.pair_tgt);
      D->pair_off = dev_upload<int32_t>(A, F.pair_off);
      D->pair_items = dev_upload<int32_t>(A, F.pair_items);
    }
  } catch (...) {
    delete D;
    throw;
  }
  return D;
}

// pads a row-major [k][n][n] table to [k][ld][ld] with zeros
template <class T>
static std::vector<T> pad_table(const std::vector<double>& src, int k, int n, int ld) {
  std::vector<T> out(size_t(k) * ld * ld, T(0));
  for (int m = 0; m < k; ++m)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        out[(size_t(m) * ld + i) * ld + j] = T(src[(size_t(m) * n + i) * n + j]);
  return out;
}

// float -> bfloat16 bits, round to nearest even (finite inputs)
static uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
static double bf16_value(uint16_t b) {
  uint32_t u = uint32_t(b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

static uint16_t f16_bits(double x) {
  _Float16 h = _Float16(float(x));
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}
static double f16_value(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, 2);
  return double(float(h));
}

// M2L runs on check potentials with the folded operators from this order on
// (their cancellation is ~10x smaller than the densities' at p = 10, larger
// at p <= 8).
static int g_m2l_check_min_p = 10;
void set_m2l_check_min_p(int p) { g_m2l_check_min_p = p; }
// FP32-accumulating M2L moves its sums into FP64 after every operator step
// from this order on (it costs occupancy; at p = 10 it cuts the error ~10x).
static int g_m2l_fp64_sum_min_p = 10;
void set_m2l_fp64_sum_min_p(int p) { g_m2l_fp64_sum_min_p = p; }

// Interleaves the high and low parts of every operator row in blocks of the
// GEMM k-chunk (32): [k][ld rows][ld / 32][2][32], so that the two parts of
// one row's chunk are one 128-byte line.
template <class Split>
static uint16_t* upload_split(DevOps* O, const std::vector<double>& pad, Split split) {
  const size_t ld = size_t(O->ld), rows = pad.size() / ld;
  std::vector<uint16_t> out(2 * pad.size());
  for (size_t r = 0; r < rows; ++r)
    for (size_t j = 0; j < ld; ++j) {
      uint16_t hi, lo;
      split(pad[r * ld + j], hi, lo);
      const size_t base = ((r * (ld / 32) + j / 32) * 2) * 32 + j % 32;
      out[base] = hi;
      out[base + 32] = lo;
    }
  return dev_upload<uint16_t>(O->allocs, out);
}
static uint16_t* upload_split16(DevOps* O, const std::vector<double>& pad) {
  const double sc = std::ldexp(1.0, kF16OpExp);
  return upload_split(O, pad, [&](double x, uint16_t& hi, uint16_t& lo) {
    const double v = x * sc;
    hi = f16_bits(v);
    lo = f16_bits(v - f16_value(hi));
  });
}

// Which tables an evaluation needs: bulk type (FP32 or FP64 M2M/L2L), and the
// M2L operand: FP64, FP32, BF16 split or FP16 split, in density or check form.
struct OpsNeed {
  bool bulk64 = false, m2l64 = false, m2l32 = false, bf16 = false, f16 = false, check_form = false;
  bool l2l64 = false;  // FP64 L2L in an FP32-bulk evaluation (gradients)
};

static DevOps* ops_for_device(OpsCache& oc, const HostOps& H, int dev, const OpsNeed& need) {
  DevOps* O = nullptr;
  if (auto it = oc.per_device.find(dev); it != oc.per_device.end()) O = it->second;
  if (!O) {
    // the base tables first, entered into the cache only when complete; the
    // optional tables below are each set only once uploaded
    std::unique_ptr<DevOps> Op(new DevOps());
    O = Op.get();
    O->n = H.n;
    O->p = H.p;
    O->ld = round32(H.n);
    O->levels = H.levels;
    O->kappa = H.kappa;
    O->uc2e = dev_upload<double>(O->allocs, pad_table<double>(H.uc2e, H.levels, H.n, O->ld));
    O->dc2e = dev_upload<double>(O->allocs, pad_table<double>(H.dc2e, H.levels, H.n, O->ld));
    std::vector<double> s4(4 * size_t(H.n), 0.0);
    for (int i = 0; i < H.n; ++i)
      for (int d = 0; d < 3; ++d) s4[4 * i + d] = H.surf[3 * i + d];
    O->surf = dev_upload<double4>(O->allocs, s4);
    oc.per_device[dev] = Op.release();
  }
  if (need.bulk64 && !O->m2m64)
    O->m2m64 = dev_upload<double>(O->allocs, pad_table<double>(H.m2m, 8 * H.levels, H.n, O->ld));
  if ((need.bulk64 || need.l2l64) && !O->l2l64)
    O->l2l64 = dev_upload<double>(O->allocs, pad_table<double>(H.l2l, 8 * H.levels, H.n, O->ld));
  if (!need.bulk64 && !O->m2m32) {
    O->m2m32 = dev_upload<float>(O->allocs, pad_table<float>(H.m2m, 8 * H.levels, H.n, O->ld));
    O->l2l32 = dev_upload<float>(O->allocs, pad_table<float>(H.l2l, 8 * H.levels, H.n, O->ld));
  }
  if (need.m2l64 && !O->m2l64)
    O->m2l64 = dev_upload<double>(O->allocs, pad_table<double>(H.m2l, kNumM2L * H.levels, H.n, O->ld));
  if (need.check_form) {
    if ((need.f16 && !O->m2lc_h) || (need.m2l32 && !O->m2lc32)) {
      std::vector<double> pad = pad_table<double>(m2l_check_form_device(H), kNumM2L, H.n, O->ld);
      if (need.f16 && !O->m2lc_h) O->m2lc_h = upload_split16(O, pad);
      if (need.m2l32 && !O->m2lc32) {
        std::vector<float> f(pad.begin(), pad.end());
        O->m2lc32 = dev_upload<float>(O->allocs, f);
      }
    }
  } else {
    if (need.m2l32 && !O->m2l32)
      O->m2l32 = dev_upload<float>(O->allocs, pad_table<float>(H.m2l, kNumM2L * H.levels, H.n, O->ld));
    if (need.f16 && !O->m2l_h)
      O->m2l_h = upload_split16(O, pad_table<double>(H.m2l, kNumM2L * H.levels, H.n, O->ld));
  }
  if (need.bf16 && !O->m2l_b)
    O->m2l_b = upload_split(O, pad_table<double>(H.m2l, kNumM2L * H.levels, H.n, O->ld),
                            [](double x, uint16_t& hi, uint16_t& lo) {
                              hi = bf16_bits(float(x));
                              lo = bf16_bits(float(x - bf16_value(hi)));
                            });
  return O;
}

static DevWork* work_for(DevForest& F, bool fp64, int n_rhs, bool grad = false) {
  // (buffers of gradient evaluations are kept apart: 4 values per target)
  const std::pair<int, int> key{(fp64 ? 1 : 0) | (grad ? 2 : 0), n_rhs};
  auto found = F.work.find(key);
  if (found != F.work.end()) return found->second;
  // built aside and entered only when every buffer exists (an allocation
  // failure leaves no half-made entry behind)
  std::unique_ptr<DevWork> Wp(new DevWork());
  DevWork* W = Wp.get();
  W->n_rhs = n_rhs;
  W->fp64 = fp64;
  size_t es = fp64 ? 8 : 4;
  // one extra box: the zero columns that empty GEMM slots read
  size_t cols = size_t(F.nbox + 1) * n_rhs * F.ld;
  W->col_bytes = cols * es;
  auto alloc_bytes = [&](size_t bytes) {
    void* p = dev_alloc<unsigned char>(W->allocs, bytes);
    HIPCHECK(hipMemset(p, 0, bytes));
    return p;
  };
  W->qs = alloc_bytes(size_t(n_rhs) * F.nsrc * es);
  W->up_chk = alloc_bytes(W->col_bytes);
  W->up_eq = alloc_bytes(W->col_bytes);
  W->dn_chk = alloc_bytes(W->col_bytes);
  W->dn_eq = alloc_bytes(W->col_bytes);
  W->pot = static_cast<double*>(alloc_bytes(size_t(n_rhs) * (grad ? 4 : 1) * F.ntgt * 8));
  if (grad && !fp64) W->dn_chk64 = static_cast<double*>(alloc_bytes(cols * 8));
  W->absmax = static_cast<unsigned*>(alloc_bytes(16));
  F.work[key] = Wp.release();
  return W;
}

// The split M2L operand ([columns][ld / 32][parts][32] of 16-bit values),
// allocated on first use by a split-precision mode (outside graph capture).
static void ensure_split(DevForest& F, DevWork* W) {
  if (W->split) return;
  const size_t cols = size_t(F.nbox + 1) * W->n_rhs * F.ld;
  W->split_bytes = cols * 3 * 2;
  W->split = dev_alloc<unsigned char>(W->allocs, W->split_bytes);
  HIPCHECK(hipMemset(W->split, 0, W->split_bytes));
}

// The pair buffer of the pair-by-pair M2L, allocated on first use (outside
// graph capture).
static void ensure_pairs(DevForest& F, DevWork* W) {
  if (W->pairs || F.n_pairs == 0) return;
  W->pair_bytes = size_t(F.n_pairs) * W->n_rhs * F.ld * (W->fp64 ? 8 : 4);
  W->pairs = dev_alloc<unsigned char>(W->allocs, W->pair_bytes);
}

// ------------------------------------------------------------------------
// profiling: HIP events around each phase on the evaluation stream
// ------------------------------------------------------------------------

// Phases hold only their own launches (the M2L phase is the gathered GEMM
// alone; zeroing its output and the FP16 density scale are "m2l_prep").  While profiling
// is on, the near field runs on the evaluation stream instead of the
// auxiliary one, so no two phases overlap and each one's events time it alone.
enum Phase { PH_GATHER, PH_P2M, PH_M2M, PH_UC2E, PH_M2L_PREP, PH_M2L, PH_M2L_PAIR, PH_P2L, PH_L2L,
             PH_DC2E, PH_NEAR, PH_FAR, PH_SCATTER, PH_N };
static const char* kPhaseNames[PH_N] = {"gather", "p2m", "m2m", "uc2e", "m2l_prep", "m2l", "m2l_pair",
                                        "p2l", "l2l", "dc2e", "near", "far", "scatter"};

struct Profiler {
  bool on = false;
  struct Rec {
    int ph;
    hipEvent_t a, b;
    int launches;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipStream_t stream = nullptr;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    return e;
  }
};
static Profiler g_prof;

struct PhaseScope {
  int ph;
  hipStream_t s;
  hipEvent_t a{};
  int launches = 0;
  PhaseScope(int ph_, hipStream_t s_) : ph(ph_), s(s_) {
    if (g_prof.on) {
      a = g_prof.get();
      HIPCHECK(hipEventRecord(a, s));
    }
  }
  ~PhaseScope() noexcept(false) {
    if (g_prof.on) {
      hipEvent_t b = g_prof.get();
      HIPCHECK(hipEventRecord(b, s));
      g_prof.recs.push_back({ph, a, b, launches});
      g_prof.stream = s;
    }
  }
};

void set_profiling(bool on) { g_prof.on = on; }
int n_phases() { return PH_N; }
const char* phase_name(int i) { return (i >= 0 && i < PH_N) ? kPhaseNames[i] : nullptr; }
void get_phase_times(double* ms, int64_t* launches) {
  for (int i = 0; i < PH_N; ++i) {
    if (ms) ms[i] = 0;
    if (launches) launches[i] = 0;
  }
  if (!g_prof.recs.empty()) HIPCHECK(hipEventSynchronize(g_prof.recs.back().b));
  for (auto& r : g_prof.recs) {
    float t = 0;
    HIPCHECK(hipEventElapsedTime(&t, r.a, r.b));
    if (ms) ms[r.ph] += t;
    if (launches) launches[r.ph] += r.launches;
    g_prof.pool.push_back(r.a);
    g_prof.pool.push_back(r.b);
  }
  g_prof.recs.clear();
}

// ------------------------------------------------------------------------
// kernels
// ------------------------------------------------------------------------

template <class T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };

__device__ inline float rinv(float r2) { return r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f; }
__device__ inline double rinv(double r2) { return r2 > 0.0 ? rsqrt(r2) : 0.0; }
// for pairs that cannot coincide (r2 > 0)
__device__ inline float rinv_nonzero(float r2) { return __builtin_amdgcn_rsqf(r2); }
__device__ inline double rinv_nonzero(double r2) { return rsqrt(r2); }

constexpr int kMaxProb = 64;
struct PtrPack {
  const void* p[kMaxProb];
};

template <class TI, class T>
__global__ void gather_kernel(PtrPack q, int prob0, const int64_t* __restrict__ src_off,
                              const int32_t* __restrict__ perm, int n_rhs, int64_t nsrc,
                              T* __restrict__ qs) {
  const int k = blockIdx.y;
  const int64_t b = src_off[prob0 + k], e = src_off[prob0 + k + 1];
  const int64_t i = b + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= e) return;
  const int64_t nk = e - b;
  const TI* src = static_cast<const TI*>(q.p[k]);
  const int64_t ci = perm[i];
  for (int r = 0; r < n_rhs; ++r) qs[int64_t(r) * nsrc + i] = T(src[int64_t(r) * nk + ci]);
}

template <class TO>
__global__ void scatter_kernel(PtrPack out, int prob0, const int64_t* __restrict__ tgt_off,
                               const int32_t* __restrict__ perm, int n_rhs, int64_t ntgt,
                               const double* __restrict__ pot) {
  const int k = blockIdx.y;
  const int64_t b = tgt_off[prob0 + k], e = tgt_off[prob0 + k + 1];
  const int64_t i = b + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= e) return;
  const int64_t nk = e - b;
  TO* dst = static_cast<TO*>(const_cast<void*>(out.p[k]));
  const int64_t ci = perm[i];
  for (int r = 0; r < n_rhs; ++r) dst[int64_t(r) * nk + ci] = TO(pot[int64_t(r) * ntgt + i]);
}

// Block-wide maximum of m (>= 0), then one atomic per block: atomics from
// every wave onto the single result word serialize in L2.
__device__ inline void block_max_to(float m, unsigned* out) {
  __shared__ float s_m[16];
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) s_m[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < nw; ++i) m = fmaxf(m, s_m[i]);
    atomicMax(out, __float_as_uint(m));
  }
}

// Largest |x| over n4 float4 values, into *out as float bits (all values >= 0,
// so unsigned order equals float order); *out must start at 0.
__global__ void absmax_kernel(const float4* __restrict__ p, int64_t n4, unsigned* __restrict__ out) {
  float m = 0.0f;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += int64_t(gridDim.x) * blockDim.x) {
    float4 v = p[i];
    m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
  }
  block_max_to(m, out);
}

__global__ void absmax_kernel64(const double2* __restrict__ p, int64_t n2, unsigned* __restrict__ out) {
  float m = 0.0f;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n2; i += int64_t(gridDim.x) * blockDim.x) {
    double2 v = p[i];
    m = fmaxf(m, float(fmax(fabs(v.x), fabs(v.y))));
  }
  block_max_to(m, out);
}

// Pair-by-pair M2L, second half: the downward check potential of each target
// of a sparse problem is the sum of its pairs' products (pair buffer columns
// of n_rhs * ld elements), taken in the order the plan lists them (by
// offset), in FP64, rounded once.  The targets' columns receive nothing else
// before P2L, so the sum is stored.  One thread per 16-byte unit of a
// target's columns; eight pairs' loads are issued before they are added (in
// order).  Grid-stride over (target, unit).
template <class T>
__global__ void m2l_pair_sum_kernel(const int32_t* __restrict__ tgt, const int32_t* __restrict__ off,
                                    const int32_t* __restrict__ items, int ntgt, int64_t units,
                                    const uint4* __restrict__ pairs, uint4* __restrict__ out) {
  constexpr int E = 16 / sizeof(T), U = 8;
  const int64_t tot = int64_t(ntgt) * units;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < tot;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t k = i / units, w = i - k * units;
    double acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.0;
    const int e0 = off[k], e1 = off[k + 1];
    for (int b = e0; b < e1; b += U) {
      uint4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (b + u < e1) v[u] = pairs[int64_t(items[b + u]) * units + w];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (b + u < e1) {
          const T* x = reinterpret_cast<const T*>(&v[u]);
#pragma unroll
          for (int e = 0; e < E; ++e) acc[e] += double(x[e]);
        }
    }
    uint4 r;
    T* y = reinterpret_cast<T*>(&r);
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = T(acc[e]);
    out[int64_t(tgt[k]) * units + w] = r;
  }
}

// M2M, second half: the upward check potential of each parent is the sum of
// its children's contributions (written per child by the gathered GEMM),
// added in octant order.  tab is [npar][9]: parent, children 0..7 or -1.
// Columns are ld elements, ld a multiple of 32, so 16-byte units tile them.
template <class T>
__global__ void m2m_sum_kernel(const int32_t* __restrict__ tab, int npar, int64_t units_per_box,
                               const uint4* __restrict__ part, uint4* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(npar) * units_per_box) return;
  const int64_t k = i / units_per_box, u = i - k * units_per_box;
  const int32_t* t = tab + 9 * k;
  constexpr int E = 16 / sizeof(T);
  T acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = T(0);
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int c = t[1 + o];
    if (c >= 0) {
      const uint4 v = part[int64_t(c) * units_per_box + u];
      const T* x = reinterpret_cast<const T*>(&v);
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] += x[e];
    }
  }
  uint4 r;
  T* y = reinterpret_cast<T*>(&r);
#pragma unroll
  for (int e = 0; e < E; ++e) y[e] = acc[e];
  out[int64_t(t[0]) * units_per_box + u] = r;
}

// FP32 -> FP64 copy of n values (grid-stride)
__global__ void widen_kernel(const float* __restrict__ in, double* __restrict__ out, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    out[i] = double(in[i]);
}

__global__ void zero_kernel(uint4* __restrict__ p, int64_t n16) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = make_uint4(0, 0, 0, 0);
}

// --- P2P-shaped operators -------------------------------------------------
// One block per target box.  Targets are particles (LEAF) or surface points
// (P2M: upward check, P2L: downward check); sources are "segments": the
// particles of a leaf, or the equivalent surface of a box with its density.
// Every source is moved into the target box's frame once, while it is staged
// into LDS; targets are split into chunks (64 lanes for surface targets; of
// equal width up to 64 lanes, chosen per leaf, for particles) and the
// 256 / width lane groups ("slices") stride over the staged sources, then
// reduce in FP64.

// LEAF: near + far in one pass; NEAR: U lists only (writes the sums);
// FAR: W lists and the own downward surface (adds to the sums).
enum { MODE_P2M = 0, MODE_P2L = 1, MODE_LEAF = 2, MODE_NEAR = 3, MODE_FAR = 4 };
enum { SEG_POINTS = 0, SEG_UP_EQUIV = 1, SEG_DN_EQUIV = 2 };

template <class T>
struct P2PArgs {
  const int4* box_geo;
  const double* box_r;
  const int2* box_src;
  const int2* box_tgt;
  const double4* src64;
  const double4* tgt64;
  const T* qs;
  int64_t nsrc;
  int n_rhs;
  const double4* surf;
  int n, ld;
  const T* up_eq;
  const T* dn_eq;
  T* out_col;
  double* pot;
  int64_t ntgt;
  const int32_t* work;
  const int32_t* l1_off;
  const int32_t* l1_items;
  const int32_t* l2_off;
  const int32_t* l2_items;
  int grad;  // leaf kernel: also the gradient (pot holds [n_rhs][4][ntgt])
  double kappa;  // screened kernel exp(-kappa d) / (4 pi d); 0: Laplace
};

template <class T, int RC, bool LO = false>
struct P2PCfg {
  static constexpr int NT = 256;
  // staged source: position (+ the charge in w when RC == 1), charges of RC > 1
  // columns; with LO the FP32 rounding error of the position as well
  static constexpr int PB = int(sizeof(typename V4<T>::type)) + (RC > 1 ? RC * int(sizeof(T)) : 0) +
                            (LO ? int(sizeof(typename V4<T>::type)) : 0);
  // The batch size depends on T only, so every right-hand side sees the same
  // summation order whatever RC is (multi-RHS columns equal single runs bitwise).
  static constexpr int CAP = sizeof(T) == 4 ? 1024 : 512;
  static constexpr int BYTES = CAP * PB;
};

// (A -> B) frame change: shift = (c_A - c_B) / r_B, ratio = r_A / r_B.
__device__ inline double4 frame(int4 a, int4 b) {
  double ratio = ldexp(1.0, b.w - a.w);
  double4 g;
  g.x = (2.0 * a.x + 1.0) * ratio - (2.0 * b.x + 1.0);
  g.y = (2.0 * a.y + 1.0) * ratio - (2.0 * b.y + 1.0);
  g.z = (2.0 * a.z + 1.0) * ratio - (2.0 * b.z + 1.0);
  g.w = ratio;
  return g;
}

constexpr int kMaxSeg = 160, kNch = 4;  // segment window (any count is processed in windows)

struct SegTable {
  int pre[kMaxSeg + 1];
  int id[kMaxSeg];
  int kind[kMaxSeg];
  double4 geo[kMaxSeg];
  int self_k;  // index of the target box's own particle segment, or -1
};

// Source segment si of work item wi (target box B) for the given mode.
template <class T, int MODE>
__device__ inline void segment_info(const P2PArgs<T>& a, int wi, int B, int4 gB, int nU, int si,
                                    int& kind, int& id, int& size, double4& g) {
  if (MODE == MODE_P2M) {
    int2 sr = a.box_src[B];
    kind = SEG_POINTS;
    id = sr.x;
    size = sr.y - sr.x;
    g = make_double4(0.0, 0.0, 0.0, 1.0);
  } else if (si < nU) {
    int A = a.l1_items[a.l1_off[wi] + si];
    int2 sr = a.box_src[A];
    kind = SEG_POINTS;
    id = sr.x;
    size = sr.y - sr.x;
    g = frame(a.box_geo[A], gB);
  } else if (MODE != MODE_P2L && si < nU + (a.l2_off[wi + 1] - a.l2_off[wi])) {
    int A = a.l2_items[a.l2_off[wi] + (si - nU)];
    kind = SEG_UP_EQUIV;
    id = A;
    size = a.n;
    g = frame(a.box_geo[A], gB);
    g.w *= kRin;
  } else {
    kind = SEG_DN_EQUIV;
    id = B;
    size = a.n;
    g = make_double4(0.0, 0.0, 0.0, kRout);
  }
}

// Accumulates the sources of segments [s0, s1) into acc, computing pair terms
// in precision U (staging in LDS, FP32/FP64 partials folded into FP64).  With
// GRAD (one right-hand side), gacc also sums q (x - y) / |x - y|^3 per axis.
template <class U, class T, int MODE, int RC, int TCH, bool GRAD = false, bool SCR = false>
__device__ void p2p_phase(const P2PArgs<T>& a, unsigned char* smem, SegTable& st, int wi, int B,
                          int4 gB, int nU, int s0, int s1, int rhs0, const double (&tx)[kNch],
                          const double (&ty)[kNch], const double (&tz)[kNch], int nchunks,
                          double (&acc)[kNch][RC], double (&gacc)[kNch][3], double kB, int j0, int SL) {
  // j0: this lane's first staged source (its lane group; past every source
  // for lanes outside the SL lane groups), SL: lane groups striding over them
  // SCR: the screened kernel, exp(-kB d) / d in the target box's units
  // (kB = kappa r_B); its factor multiplies 1 / d
  const U ukB = U(kB);
  static_assert(!GRAD || RC == 1, "gradients are summed for one right-hand side per block");
  // Gradient terms cancel strongly between neighbours (points on a surface):
  // in FP32 the differences x - y then take the positions as two-float sums
  // (hi + lo), so that they are not limited by the rounding of coordinates.
  constexpr bool LO = GRAD && sizeof(U) == 4;
  using C = P2PCfg<U, RC, LO>;
  using V = typename V4<U>::type;
  constexpr int NT = 256, CAP = C::CAP;
  V* s_pos = reinterpret_cast<V*>(smem);
  U* s_q = reinterpret_cast<U*>(smem + CAP * sizeof(V));
  V* s_lo = reinterpret_cast<V*>(smem + CAP * sizeof(V));  // (LO only, RC == 1)
  const int tid = threadIdx.x;
  U ux[kNch], uy[kNch], uz[kNch], lx[kNch], ly[kNch], lz[kNch];
#pragma unroll
  for (int c = 0; c < kNch; ++c) {
    ux[c] = U(tx[c]);
    uy[c] = U(ty[c]);
    uz[c] = U(tz[c]);
    lx[c] = U(tx[c] - double(ux[c]));
    ly[c] = U(ty[c] - double(uy[c]));
    lz[c] = U(tz[c] - double(uz[c]));
  }
  for (int sw = s0; sw < s1; sw += kMaxSeg) {
    const int nw = min(kMaxSeg, s1 - sw);
    __syncthreads();
    if (tid == 0) {
      st.pre[0] = 0;
      st.self_k = -1;
    }
    __syncthreads();
    if (tid < nw) {
      int kind, id, size;
      double4 g;
      segment_info<T, MODE>(a, wi, B, gB, nU, sw + tid, kind, id, size, g);
      st.kind[tid] = kind;
      st.id[tid] = id;
      st.geo[tid] = g;
      st.pre[tid + 1] = size;
      // the segment whose coincidence test differs from the others': near
      // field, the target box's own particles (the only sources that can
      // coincide with targets: equal points always share a leaf); far field,
      // the box's own downward equivalent surface (at 2.95 r, never within
      // 1.95 r of its particles)
      if constexpr (MODE == MODE_LEAF || MODE == MODE_NEAR) {
        if (kind == SEG_POINTS && size > 0 && id == a.box_src[B].x) st.self_k = tid;
      } else if constexpr (MODE == MODE_FAR) {
        if (kind == SEG_DN_EQUIV && size > 0) st.self_k = tid;
      }
    }
    __syncthreads();
    for (int off = 1; off < nw; off <<= 1) {
      int v = (tid < nw && tid >= off) ? st.pre[tid + 1 - off] : 0;
      __syncthreads();
      if (tid < nw) st.pre[tid + 1] += v;
      __syncthreads();
    }
    const int total = st.pre[nw];
    for (int b0 = 0; b0 < total; b0 += CAP) {
      const int nb = min(CAP, total - b0);
      for (int j = tid; j < nb; j += NT) {
        const int gidx = b0 + j;
        int lo = 0, hi = nw - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (st.pre[mid] <= gidx) lo = mid;
          else hi = mid - 1;
        }
        const int local = gidx - st.pre[lo];
        const int kind = st.kind[lo];
        const double4 g = st.geo[lo];
        double px, py, pz;
        U q0 = U(0);  // first right-hand side (staged with the position when RC == 1)
        if (kind == SEG_POINTS) {
          const int64_t pi = int64_t(st.id[lo]) + local;
          double4 p = a.src64[pi];
          px = g.x + g.w * p.x;
          py = g.y + g.w * p.y;
          pz = g.z + g.w * p.z;
#pragma unroll
          for (int r = 0; r < RC; ++r) {
            int rr = rhs0 + r;
            const U qv = rr < a.n_rhs ? U(a.qs[int64_t(rr) * a.nsrc + pi]) : U(0);
            if (r == 0) q0 = qv;
            if constexpr (RC > 1) s_q[r * CAP + j] = qv;
          }
        } else {
          double4 s = a.surf[local];
          px = g.x + g.w * s.x;
          py = g.y + g.w * s.y;
          pz = g.z + g.w * s.z;
          const T* dens = kind == SEG_UP_EQUIV ? a.up_eq : a.dn_eq;
          const int64_t col0 = int64_t(st.id[lo]) * a.n_rhs;
#pragma unroll
          for (int r = 0; r < RC; ++r) {
            int rr = rhs0 + r;
            const U qv = rr < a.n_rhs ? U(dens[(col0 + rr) * a.ld + local]) : U(0);
            if (r == 0) q0 = qv;
            if constexpr (RC > 1) s_q[r * CAP + j] = qv;
          }
        }
        V v;
        v.x = U(px);
        v.y = U(py);
        v.z = U(pz);
        v.w = q0;  // one right-hand side: the charge rides along with the position
        s_pos[j] = v;
        if constexpr (LO) {
          V l;
          l.x = U(px - double(v.x));
          l.y = U(py - double(v.y));
          l.z = U(pz - double(v.z));
          l.w = U(0);
          s_lo[j] = l;
        }
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < kNch; ++c) {
        if (c < nchunks) {
          U part[RC], gpart[3] = {U(0), U(0), U(0)};
#pragma unroll
          for (int r = 0; r < RC; ++r) part[r] = U(0);
          const U x = ux[c], y = uy[c], z = uz[c], xl = lx[c], yl = ly[c], zl = lz[c];
          // sources j = j0, j0 + SL, ... in order; four per trip so that their
          // LDS reads are in flight together (same summation order)
          auto pair = [&](const V& s, int j, auto checked) __attribute__((always_inline)) {
            U dx = x - s.x, dy = y - s.y, dz = z - s.z;
            if constexpr (LO) {
              const V l = s_lo[j];
              dx += xl - l.x;
              dy += yl - l.y;
              dz += zl - l.z;
            }
            const U r2 = dx * dx + dy * dy + dz * dz;
            U ri;
            if constexpr (decltype(checked)::value) ri = rinv(r2);   // coincident pair -> 0
            else ri = rinv_nonzero(r2);
            // gradient factor: 1/d^3, screened (1 + kB d) exp(-kB d) / d^3
            U gf = U(0);
            if constexpr (GRAD) gf = ri * ri;
            if constexpr (SCR) {
              const U kd = ukB * (r2 * ri);
              U e;
              if constexpr (sizeof(U) == 4) e = __expf(-kd);
              else e = exp(-kd);
              ri *= e;
              if constexpr (GRAD) gf *= U(1) + kd;
            }
            if constexpr (RC == 1) {
              part[0] += s.w * ri;
              if constexpr (GRAD) {
                const U qr3 = s.w * ri * gf;
                gpart[0] += qr3 * dx;
                gpart[1] += qr3 * dy;
                gpart[2] += qr3 * dz;
              }
            } else {
#pragma unroll
              for (int r = 0; r < RC; ++r) part[r] += s_q[r * CAP + j] * ri;
            }
          };
          // staged sources [j, end) with stride SL, in order
          auto run = [&](int j, int end, auto checked) __attribute__((always_inline)) {
            for (; j + 3 * SL < end; j += 4 * SL) {
              const V s0 = s_pos[j], s1 = s_pos[j + SL], s2 = s_pos[j + 2 * SL], s3 = s_pos[j + 3 * SL];
              pair(s0, j, checked);
              pair(s1, j + SL, checked);
              pair(s2, j + 2 * SL, checked);
              pair(s3, j + 3 * SL, checked);
            }
            for (; j < end; j += SL) pair(s_pos[j], j, checked);
            return j;
          };
          const std::true_type chk;
          const std::false_type nochk;
          // the ranges keep the order j = j0, j0 + SL, ...
          int lo = nb, hi = nb;
          if (st.self_k >= 0) {
            lo = min(max(st.pre[st.self_k] - b0, 0), nb);
            hi = min(max(st.pre[st.self_k + 1] - b0, 0), nb);
          }
          if constexpr (MODE == MODE_LEAF || MODE == MODE_NEAR) {
            // only the target box's own particles need the coincidence test
            int j = run(j0, lo, nochk);
            j = run(j, hi, chk);
            run(j, nb, nochk);
          } else if constexpr (MODE == MODE_FAR) {
            // all but the box's own downward surface need it
            int j = run(j0, lo, chk);
            j = run(j, hi, nochk);
            run(j, nb, chk);
          } else if constexpr (MODE == MODE_P2M) {
            // check surface at 2.95 r, sources inside the box: never coincide
            run(j0, nb, nochk);
          } else {
            run(j0, nb, chk);
          }
#pragma unroll
          for (int r = 0; r < RC; ++r) acc[c][r] += double(part[r]);
          if constexpr (GRAD) {
#pragma unroll
            for (int k = 0; k < 3; ++k) gacc[c][k] += double(gpart[k]);
          }
        }
      }
      __syncthreads();
    }
  }
}

// --- P2P-shaped operators -------------------------------------------------
// One block per target box.  Targets are particles (LEAF) or surface points
// (P2M: upward check, P2L: downward check); sources are "segments": the
// particles of a leaf, or the equivalent surface of a box with its density.
// Every source is moved into the target box's frame once, while it is staged
// into LDS; targets are split into chunks (TCH lanes, or for leaves of equal
// width chosen per leaf, see below) and the lane groups stride over the
// staged sources, then reduce in FP64.  Particle
// segments are computed in T, equivalent-surface segments (L2P, M2P) in TF:
// FP64 at high order, where the equivalent densities cancel strongly.
template <class T, class TF, int MODE, int RC, int TCH, bool GRAD = false, bool SCR = false>
__global__ __launch_bounds__(256) void p2p_kernel(P2PArgs<T> a) {
  constexpr int NT = 256;
  static_assert(!GRAD || (MODE == MODE_LEAF && RC == 1), "gradients: leaf kernel, one right-hand side");
  constexpr int SMEM0 = P2PCfg<T, RC, GRAD>::BYTES > P2PCfg<TF, RC, GRAD>::BYTES ? P2PCfg<T, RC, GRAD>::BYTES
                                                                                 : P2PCfg<TF, RC, GRAD>::BYTES;
  constexpr int NV = RC + (GRAD ? 3 : 0);  // reduced values per target
  constexpr int RED = NT * NV * 8;
  __shared__ __align__(16) unsigned char smem[SMEM0 > RED ? SMEM0 : RED];
  __shared__ SegTable st;
  double* s_red = reinterpret_cast<double*>(smem);

  const int tid = threadIdx.x;
  const int wi = blockIdx.x;
  const int B = a.work[wi];
  const int rhs0 = blockIdx.y * RC;
  const int4 gB = a.box_geo[B];

  int nU = 0, nseg = 0, nnear = 0;
  if (MODE == MODE_P2M) {
    nseg = nnear = 1;
  } else if (MODE == MODE_P2L) {
    nU = a.l1_off[wi + 1] - a.l1_off[wi];
    nseg = nnear = nU;
  } else {
    nU = a.l1_off[wi + 1] - a.l1_off[wi];
    const int nW = a.l2_off[wi + 1] - a.l2_off[wi];
    nnear = nU;
    nseg = MODE == MODE_NEAR ? nU : nU + nW + (gB.w >= 2 ? 1 : 0);
  }
  constexpr bool LEAFLIKE = MODE == MODE_LEAF || MODE == MODE_NEAR || MODE == MODE_FAR;
  int nt, tbase = 0;
  double trad = 0.0;
  if (LEAFLIKE) {
    int2 tr = a.box_tgt[B];
    tbase = tr.x;
    nt = tr.y - tr.x;
  } else {
    nt = a.n;
    trad = MODE == MODE_P2M ? kRout : kRin;
  }

  // Lanes per target chunk: TCH for surface targets; for leaves, the
  // leaf's targets in ceil(nt / 64) chunks of equal width (at least 8 lanes;
  // 64 past kNch such chunks), so that a leaf of 33 to 64 points does not pad
  // to 64 target slots nor one of 65 to 96 to 128.  The 256 / tch lane
  // groups (the rest of the threads idle) stride over the staged sources.
  // The split depends only on the box, so runs stay deterministic.  (Surface
  // targets, 152 at p = 6, measured slower in 3 chunks of 51 than of 64.)
  int tch = TCH;
  if constexpr (LEAFLIKE) {
    const int nch = (nt + 63) / 64;
    tch = nch <= kNch ? max((nt + nch - 1) / max(nch, 1), 8) : 64;
  }
  const int ti = tid % tch, sl = tid / tch, SL = NT / tch;
  const int j0 = sl < SL ? sl : (1 << 30);
  for (int t0 = 0; t0 < nt; t0 += tch * kNch) {
    double tx[kNch], ty[kNch], tz[kNch];
    double acc[kNch][RC], gacc[kNch][3];
#pragma unroll
    for (int c = 0; c < kNch; ++c) {
      int t = t0 + c * tch + ti;
      tx[c] = ty[c] = tz[c] = 0.0;
      if (t < nt) {
        if (LEAFLIKE) {
          double4 p = a.tgt64[tbase + t];
          tx[c] = p.x;
          ty[c] = p.y;
          tz[c] = p.z;
        } else {
          double4 s = a.surf[t];
          tx[c] = trad * s.x;
          ty[c] = trad * s.y;
          tz[c] = trad * s.z;
        }
      }
#pragma unroll
      for (int r = 0; r < RC; ++r) acc[c][r] = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) gacc[c][k] = 0.0;
    }
    const int nchunks = (min(nt - t0, tch * kNch) + tch - 1) / tch;
    const double kB = SCR ? a.kappa * a.box_r[B] : 0.0;
    if (MODE != MODE_FAR)
      p2p_phase<T, T, MODE, RC, TCH, GRAD, SCR>(a, smem, st, wi, B, gB, nU, 0, nnear, rhs0, tx, ty, tz,
                                                nchunks, acc, gacc, kB, j0, SL);
    if (MODE != MODE_NEAR && nseg > nnear)
      p2p_phase<TF, T, MODE, RC, TCH, GRAD, SCR>(a, smem, st, wi, B, gB, nU, nnear, nseg, rhs0, tx, ty, tz,
                                                 nchunks, acc, gacc, kB, j0, SL);

    // reduce the slices of each chunk and write
    const double rB = a.box_r[B];
#pragma unroll
    for (int c = 0; c < kNch; ++c) {
      if (c < nchunks) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RC; ++r) s_red[(sl * tch + ti) * NV + r] = acc[c][r];
        if constexpr (GRAD) {
#pragma unroll
          for (int k = 0; k < 3; ++k) s_red[(sl * tch + ti) * NV + 1 + k] = gacc[c][k];
        }
        __syncthreads();
        if (sl == 0) {
          const int t = t0 + c * tch + ti;
          if (t < nt) {
            if constexpr (GRAD) {
              // potentials then gradients: component k of right-hand side
              // rr at pot[(4 rr + k) ntgt + target]; the frame's unit is r_B,
              // so d/dx = (1 / r_B) d/dx~, and d/dx~ 1/|x~ - y~| = -(x~ - y~) / |x~ - y~|^3
              const int rr = rhs0;
              if (rr < a.n_rhs) {
                double v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                  v[k] = 0.0;
                  for (int s2 = 0; s2 < SL; ++s2) v[k] += s_red[(s2 * tch + ti) * NV + k];
                }
                double* o = a.pot + int64_t(4 * rr) * a.ntgt + tbase + t;
                o[0] = v[0] * (kInv4Pi / rB);
#pragma unroll
                for (int k = 1; k < 4; ++k) o[int64_t(k) * a.ntgt] = -v[k] * (kInv4Pi / (rB * rB));
              }
            } else {
#pragma unroll
            for (int r = 0; r < RC; ++r) {
              double sum = 0.0;
              for (int s2 = 0; s2 < SL; ++s2) sum += s_red[(s2 * tch + ti) * NV + r];
              const int rr = rhs0 + r;
              if (rr < a.n_rhs) {
                if (MODE == MODE_LEAF || MODE == MODE_NEAR) {
                  a.pot[int64_t(rr) * a.ntgt + tbase + t] = sum * (kInv4Pi / rB);
                } else if (MODE == MODE_FAR) {
                  a.pot[int64_t(rr) * a.ntgt + tbase + t] += sum * (kInv4Pi / rB);
                } else {
                  T* o = a.out_col + (int64_t(B) * a.n_rhs + rr) * a.ld + t;
                  if (MODE == MODE_P2M) *o = T(sum * kInv4Pi);
                  else *o += T(sum * kInv4Pi);
                }
              }
            }
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// --- gathered GEMM on the matrix cores ------------------------------------
// out[col] (+)= sum_steps op[step] * in[src col] over the tiles of a Plan.
//
// A block (4 waves) owns TC = 64*CB output columns and one group of up to 160
// rows; wave w owns CB column blocks of 16 and 10 row blocks of 16.  The k
// dimension advances in chunks of KC: lane group g = lane/16 always carries
// the KC/4 consecutive k values [g*KC/4, (g+1)*KC/4) of a chunk, for both
// operands, so each fragment is one or two 128-bit LDS reads.  That is a
// valid assignment of k to the MFMA's k slots because A and B use the same
// one.  Operator and gathered-column chunks are double-buffered in LDS: the
// next chunk's global loads are in flight while the current one feeds the
// matrix cores, with one barrier per chunk.
//
// Modes: FP32 (16x16x4 f32), FP64 (16x16x4 f64), and split BF16 on the
// 16x16x32 bf16 instruction with FP32 accumulation: BF3 = A_h x_h + A_h x_l
// + A_l x_h, BF5 additionally splits x three ways and adds A_l x_m + A_h x_l.

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));  // 16-byte staging unit
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

enum { GM_F32 = 0, GM_F64 = 1, GM_BF3 = 2, GM_BF5 = 3, GM_H3 = 4 };



template <int MODE> struct GT;
template <> struct GT<GM_F32> {
  using TA = float;       // LDS element of both operands
  using acc = f32x4;
  static constexpr int KC = 32, NB = 1;
  // output layout of 16x16 products: lane l, register v -> D[row(l,v)][l%16]
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static constexpr bool ROWS4 = true;  // a lane's four registers are consecutive rows
};
template <> struct GT<GM_F64> {
  using TA = double;
  using acc = f64x4;
  static constexpr int KC = 16, NB = 1;
  __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
  static constexpr bool ROWS4 = false;
};
template <> struct GT<GM_BF3> {
  using TA = __bf16;
  using acc = f32x4;
  static constexpr int KC = 32, NB = 2;
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static constexpr bool ROWS4 = true;
};
template <> struct GT<GM_BF5> {
  using TA = __bf16;
  using acc = f32x4;
  static constexpr int KC = 32, NB = 3;
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static constexpr bool ROWS4 = true;
};
template <> struct GT<GM_H3> {
  using TA = _Float16;
  using acc = f32x4;
  static constexpr int KC = 32, NB = 2;
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static constexpr bool ROWS4 = true;
};

struct GemmArgs {
  const void* ops;      // [nop][ld rows][ld / KC][NA parts][KC]; NA = 2 for split modes (high, low)
  int64_t op_stride;    // elements between operators (0: one operator)
  int ld, n_rhs, accumulate, TB;
  const void* in;       // columns [ncol][ld] of TI
  void* out;            // columns [ncol][ld] of TO
  const int32_t* tile_cols;
  const int32_t* step_beg;
  const int32_t* step_op;
  const int32_t* step_src;
  const unsigned* absmax;  // FP16 split: bits of max |input| (non-negative float)
  int zero_box;            // box index of the all-zero columns (the forest's nbox)
  int atomic;              // add into the output with atomics (see Plan::atomic)
  int ntile;               // tiles of the plan
};

constexpr int kRB = 10, kROWS = kRB * 16;
constexpr int kFewTiles = 128;  // below this, non-M2L plans use 32-row blocks
constexpr int kMaxTileSteps = 320;  // >= 316, the M2L offsets a tile can hold

template <int MODE, class TI, class TO, int CB, int CG = 1, int RB = kRB>
struct GemmCfg {
  using G = GT<MODE>;
  using TA = typename G::TA;
  // RB row blocks of 16 per block (kRB = 10: all 160 rows; 2: 32-row groups,
  // five blocks per tile, for plans with few tiles)
  static constexpr int ROWS = RB * 16;
  // CG column groups of 4 waves: NT threads, TC output columns per block
  static constexpr int KC = G::KC, NB = G::NB, TC = 64 * CB * CG, NT = 256 * CG;
  static constexpr int NA = (MODE == GM_BF3 || MODE == GM_BF5 || MODE == GM_H3) ? 2 : 1;  // operator tables
  // per buffer: NA operator tiles [ROWS][KC] and NB column tiles [TC][KC] of TA
  // operator part tables sit A_TSTRIDE elements apart: 128 bytes more than a
  // multiple of 256, so the two parts of one row land in different banks
  static constexpr int A_TSTRIDE = ROWS * KC + (NA > 1 ? 128 / int(sizeof(TA)) : 0);
  static constexpr int B_TSTRIDE = TC * KC + (NB > 1 ? 128 / int(sizeof(TA)) : 0);  // likewise
  static constexpr int A_ELEMS = NA * A_TSTRIDE, B_ELEMS = NB * B_TSTRIDE;
  static constexpr int BUF_BYTES = (A_ELEMS + B_ELEMS) * int(sizeof(TA));
  // 16-byte global units per chunk
  static constexpr int A_UNITS_ROW = KC * int(sizeof(TA)) / 16;         // per table row
  static constexpr int A_UNITS = NA * ROWS * A_UNITS_ROW;
  static constexpr int A_PER_T = (A_UNITS + NT - 1) / NT;  // units past A_UNITS repeat earlier ones
  // split modes read densities already split into NB 16-bit parts,
  // chunk-interleaved like the operators ([column][ld / KC][NB][KC])
  static constexpr bool SPLIT = NA > 1;
  static constexpr int B_UNITS_COL = SPLIT ? NB * KC * int(sizeof(TA)) / 16 : KC * int(sizeof(TI)) / 16;
  static constexpr int B_UNITS = TC * B_UNITS_COL;
  static constexpr int B_PER_T = (B_UNITS + NT - 1) / NT;
  // LDS rows are KC elements with no padding; the 16-byte chunks of a row are
  // XOR-swizzled so that one chunk column of consecutive rows (a fragment
  // read: lane = row) and the staging stores avoid bank conflicts.  Both
  // patterns were chosen by measurement (LDS bank-conflict counter at zero):
  // 64-byte rows: chunk ^ ((row / 2) mod 4); 128-byte rows: chunk ^ h(row)
  // with h a bijection of row mod 8 that also separates rows r and r + 8.
  static constexpr int EPC = 16 / int(sizeof(TA));            // elements per chunk
  static constexpr int CPR = KC * int(sizeof(TA)) / 16;       // chunks per row
  static_assert(CPR == 4 || CPR == 8, "LDS rows of 64 or 128 bytes");
  __device__ static int swz(int row, int chunk) {
    if constexpr (CPR == 4) return chunk ^ ((row >> 1) & 3);
    else return chunk ^ (((row ^ (row >> 3)) & 1) | (row & 6));
  }
  __device__ static int off(int row, int chunk) { return row * KC + swz(row, chunk) * EPC; }
};

// The M2L operand of the split modes: every density x (times 2^e for FP16,
// from the absmax word) becomes NB low-precision parts h = H(x),
// m = H(x - h), l = H(x - h - m), stored like the operator tables: element
// k of column c, part t at c*ld*NB + (k/32)*NB*32 + t*32 + k%32.  One thread
// converts 8 consecutive elements of a column (a 16-byte chunk per part).
template <class T, class H, int NB>
__global__ void split_kernel(const T* __restrict__ in, H* __restrict__ out, int64_t ngroups, int ld,
                             const unsigned* __restrict__ absmax, T* __restrict__ zero_out) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= ngroups) return;
  const float scale = absmax ? ldexpf(1.0f, f16_density_exp(absmax)) : 1.0f;
  const int gpc = ld / 8;
  const int64_t col = gi / gpc;
  const int k = int(gi - col * gpc) * 8;
  // the same elements of the M2L output (the downward check potentials),
  // which the split M2L adds into, start at zero
#pragma unroll
  for (int i = 0; i < 8; ++i) zero_out[col * ld + k + i] = T(0);
  const T* src = in + col * ld + k;
  H* dst = out + col * int64_t(ld) * NB + (k / 32) * NB * 32 + k % 32;
  typedef H vec8 __attribute__((ext_vector_type(8)));
  vec8 part[NB];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float x = float(src[i]) * scale;
    const H h = H(x);
    const float r = x - float(h);
    const H m = H(r);
    part[0][i] = h;
    part[1][i] = m;
    if constexpr (NB == 3) part[2][i] = H(r - float(m));
  }
#pragma unroll
  for (int t = 0; t < NB; ++t) *reinterpret_cast<vec8*>(dst + t * 32) = part[t];
}

// TAG separates the M2L launches into their own symbols: 1 = M2L, 2 = M2L
// with FP32 sums moved into FP64 registers after every operator step.
// LDS buffering of the gathered GEMM.  Two buffers let one chunk be staged
// while the previous one is read (one barrier per chunk); one buffer costs a
// second barrier per chunk but halves the LDS, so three blocks fit on a CU.
// One buffer where the registers allow three blocks (32-bit operands, no
// FP64 sums): measured faster there, as the staging latency is what bounds
// the split-precision M2L.
template <int MODE, class TO, int CB, int TAG, int CG = 1>
struct GemmOcc {
  // blocks of CG > 1 column groups (3 x 4 waves, one block per CU) share one
  // operator staging among 192 columns; only for 32-bit outputs, no FP64 sums
  static constexpr bool WIDE_OK = CB == 1 && TAG != 2 && MODE != GM_F64 && sizeof(TO) == 4;
  static constexpr bool THREE = CG == 1 && WIDE_OK;
  static constexpr int NBUF = THREE ? 1 : 2;
  static constexpr int MINB = CG > 1 ? 1 : (THREE ? 3 : 2);
};

template <int MODE, class TI, class TO, int CB, int TAG, int CG = 1, int RB = kRB>
__global__ __launch_bounds__(256 * CG, (GemmOcc<MODE, TO, CB, TAG, CG>::MINB)) void gemm_kernel(GemmArgs a) {
  using Cfg = GemmCfg<MODE, TI, TO, CB, CG, RB>;
  static_assert(RB % 2 == 0, "row blocks are split between two waves");
  constexpr int NT = Cfg::NT;
  using G = GT<MODE>;
  using TA = typename Cfg::TA;
  using ACC = typename G::acc;
  constexpr int KC = Cfg::KC, NB = Cfg::NB, TC = Cfg::TC, NA = Cfg::NA;
  constexpr bool BF = (MODE == GM_BF3 || MODE == GM_BF5 || MODE == GM_H3);  // split modes
  constexpr int NBUF = GemmOcc<MODE, TO, CB, TAG, CG>::NBUF;
  static_assert(CG == 1 || GemmOcc<MODE, TO, CB, TAG, CG>::WIDE_OK, "wide blocks need 32-bit outputs");
  __shared__ __align__(16) unsigned char smem[NBUF * Cfg::BUF_BYTES];
  __shared__ int s_ops[kMaxTileSteps];  // the tile's operator indices
  // FP16 split: the densities arrive scaled by 2^e and the operators by
  // 2^kF16OpExp; the epilogue undoes both (exact powers of two)
  float out_scale = 1.0f;
  if constexpr (MODE == GM_H3) out_scale = ldexpf(1.0f, -f16_density_exp(a.absmax) - kF16OpExp);

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, r16 = lane & 15;
  // waves form a 2 x 2 grid: wr picks half of the row blocks, wc half of the
  // column blocks, so each operator fragment is read by two waves, not four
  constexpr int RBW = RB / 2, CBW = 2 * CB;
  const int wr = (wave & 3) >> 1, wc = wave & 1;
  // first column of this wave's column group; a plan wider than the block
  // is covered by blockIdx.z slices of TC columns
  const int col0 = blockIdx.z * TC;
  const int cbase = col0 + (wave >> 2) * 64 * CB;
  const int tile = blockIdx.x;
  const int row0 = blockIdx.y * Cfg::ROWS;
  const int nrb = min(RB, (a.ld - row0) / 16);
  const int ld = a.ld;
  const int ncols = a.TB * a.n_rhs;
  const int sb = a.step_beg[tile], se = a.step_beg[tile + 1];
  const int kcs = ld / KC;  // chunks per step
  const int nchunks = (se - sb) * kcs;

  ACC acc[RBW][CBW];
#pragma unroll
  for (int i = 0; i < RBW; ++i)
#pragma unroll
    for (int c = 0; c < CBW; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][c][v] = 0;
  // TAG 2: after every operator step the FP32 sums are moved into FP64
  // registers, so FP32 rounding spans one step (one n x n product) only
  constexpr bool FLUSH = TAG == 2 && MODE != GM_F64;
  f64x4 acc64[FLUSH ? RBW : 1][FLUSH ? CBW : 1];
  if constexpr (FLUSH) {
#pragma unroll
    for (int i = 0; i < RBW; ++i)
#pragma unroll
      for (int c = 0; c < CBW; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc64[i][c][v] = 0.0;
  }

  // registers of the chunk in flight from global memory
  // two register sets: chunk c is loaded into set c % 2 two chunks before
  // it is computed, and moved to LDS one chunk before
  u32x4 ra[2][Cfg::A_PER_T], rb[2][Cfg::B_PER_T];

  // Per-thread staging addresses, fixed for the whole tile: operator units
  // (row, part, split part) and the LDS slots they land in.  Operator rows
  // past ld are clamped to a valid row: they only feed output rows that the
  // epilogue discards.
  static_assert(Cfg::B_UNITS % NT == 0, "staging units per thread");
  static_assert(NA == 1 || KC == 32, "split operator tables are interleaved in blocks of 32");
  int a_goff[Cfg::A_PER_T], a_loff[Cfg::A_PER_T];
#pragma unroll
  for (int j = 0; j < Cfg::A_PER_T; ++j) {
    // consecutive lanes: the chunks of a row, then the next row, then the
    // next part table, then the next pair of rows
    const int u = (tid + j * NT) % Cfg::A_UNITS;
    const int part = u % Cfg::CPR, rsub = (u / Cfg::CPR) & 1, t = (u / (2 * Cfg::CPR)) % NA;
    const int rl = (u / (2 * Cfg::CPR * NA)) * 2 + rsub;
    const int rg = min(row0 + rl, ld - 1);
    a_goff[j] = rg * ld * NA + t * KC + part * Cfg::EPC;
    a_loff[j] = t * Cfg::A_TSTRIDE + Cfg::off(rl, part);
  }
  // B staging units of this thread: output slot (column of the tile), part
  // table and 16-byte chunk.  Split modes use the operators' lane order (the
  // chunks of a slot, the next slot, the next part, the next slot pair),
  // which keeps the LDS stores free of bank conflicts.
  auto b_unit = [&](int u, int& slot, int& t, int& c) __attribute__((always_inline)) {
    if constexpr (Cfg::SPLIT) {
      c = u % 4;
      t = (u / 8) % NB;
      slot = (u / (8 * NB)) * 2 + ((u / 4) & 1);
    } else {
      slot = u / Cfg::B_UNITS_COL;
      c = u % Cfg::B_UNITS_COL;
      t = 0;
    }
  };
  int b_loff[Cfg::SPLIT ? Cfg::B_PER_T : 1];
  if constexpr (Cfg::SPLIT) {
#pragma unroll
    for (int j = 0; j < Cfg::B_PER_T; ++j) {
      int slot, t, c;
      b_unit(tid + j * NT, slot, t, c);
      b_loff[j] = t * Cfg::B_TSTRIDE + Cfg::off(slot, c);
    }
  }
  // Step bookkeeping of the chunk being loaded: its step, its chunk within
  // the step, and the step's operator and source columns.  The operator
  // index and the source boxes of the following step are fetched a whole
  // step ahead (the tile's operator list sits in LDS), so no load latency is
  // exposed when the step changes.  Slots past the tile's columns read the
  // all-zero box.
  // b_goff counts 16-byte units from the start of the input columns: the
  // operand of a wide multi-RHS problem passes 2^31 elements (1M points,
  // p = 10, 64 right-hand sides, split parts: 2.5e9), while 2^32 units of
  // 16 bytes cover 64 GiB (run_gemm refuses larger operands)
  int ld_st = sb, ld_kc = 0;
  int cur_op = 0, nxt_op = 0;
  int nxt_src[Cfg::B_PER_T];
  uint32_t b_goff[Cfg::B_PER_T];
  // The prefetch loads are unconditional (indices clamped into the tile, a
  // step past the end re-reads the last one) so that they land directly in
  // the registers that carry them to the next step; slots past the tile's
  // columns are replaced by the zero box where the value is used.
  auto fetch_step = [&](int st) __attribute__((always_inline)) {
    const int sc = min(st, se - 1);
    nxt_op = s_ops[sc - sb];
#pragma unroll
    for (int j = 0; j < Cfg::B_PER_T; ++j) {
      int s, t, c;
      b_unit(tid + j * NT, s, t, c);
      s += col0;
      nxt_src[j] = a.step_src[int64_t(sc) * a.TB + min(s / a.n_rhs, a.TB - 1)];
    }
  };
  auto begin_step = [&]() __attribute__((always_inline)) {
    cur_op = nxt_op;
#pragma unroll
    for (int j = 0; j < Cfg::B_PER_T; ++j) {
      int s, t, c;
      b_unit(tid + j * NT, s, t, c);
      s += col0;
      const int box = s < ncols ? nxt_src[j] : a.zero_box;
      const uint32_t col = uint32_t(box) * uint32_t(a.n_rhs) + uint32_t(s % a.n_rhs);
      if constexpr (Cfg::SPLIT)
        b_goff[j] = col * uint32_t(ld * NB * int(sizeof(TI)) / 16) + uint32_t((t * KC) / Cfg::EPC + c);
      else
        b_goff[j] = col * uint32_t(ld * int(sizeof(TI)) / 16) + uint32_t(c);
    }
  };
  auto load_regs = [&](auto P) __attribute__((always_inline)) {
    constexpr int R = decltype(P)::value;
    const int k0 = ld_kc * KC;
    const TA* opb = static_cast<const TA*>(a.ops) + int64_t(cur_op) * a.op_stride + NA * k0;
#pragma unroll
    for (int j = 0; j < Cfg::A_PER_T; ++j) ra[R][j] = *reinterpret_cast<const u32x4*>(opb + a_goff[j]);
    const u32x4* inb = reinterpret_cast<const u32x4*>(static_cast<const TI*>(a.in) + (Cfg::SPLIT ? NB * k0 : k0));
#pragma unroll
    for (int j = 0; j < Cfg::B_PER_T; ++j) rb[R][j] = inb[b_goff[j]];
  };
  auto advance = [&]() __attribute__((always_inline)) {
    if (++ld_kc == kcs) {
      ld_kc = 0;
      ++ld_st;
      begin_step();
      fetch_step(ld_st + 1);
    }
  };

  auto store_lds = [&](auto P, int buf) __attribute__((always_inline)) {
    constexpr int R = decltype(P)::value;
    TA* As = reinterpret_cast<TA*>(smem + (NBUF == 2 ? buf : 0) * Cfg::BUF_BYTES);
    TA* Bs = As + Cfg::A_ELEMS;
#pragma unroll
    for (int j = 0; j < Cfg::A_PER_T; ++j) *reinterpret_cast<u32x4*>(As + a_loff[j]) = ra[R][j];
    if constexpr (Cfg::SPLIT) {
#pragma unroll
      for (int j = 0; j < Cfg::B_PER_T; ++j) *reinterpret_cast<u32x4*>(Bs + b_loff[j]) = rb[R][j];
    } else {
      constexpr int EPU = 16 / int(sizeof(TI));  // input elements per unit
#pragma unroll
      for (int j = 0; j < Cfg::B_PER_T; ++j) {
        const int u = tid + j * NT;
        const int s = u / Cfg::B_UNITS_COL, part = u % Cfg::B_UNITS_COL;
        const TI* vals = reinterpret_cast<const TI*>(&rb[R][j]);
        // input unit `part` holds k = part*EPU .. part*EPU + EPU - 1
        constexpr int EPC = Cfg::EPC;
        if constexpr (EPU >= EPC) {
          // one or more whole LDS chunks
#pragma unroll
          for (int q = 0; q < EPU / EPC; ++q) {
            TA* d = Bs + Cfg::off(s, part * (EPU / EPC) + q);
#pragma unroll
            for (int x = 0; x < EPC; ++x) d[x] = TA(vals[q * EPC + x]);
          }
        } else {
          // part of one LDS chunk
          const int k0 = part * EPU;
          TA* d = Bs + Cfg::off(s, k0 / EPC) + k0 % EPC;
#pragma unroll
          for (int x = 0; x < EPU; ++x) d[x] = TA(vals[x]);
        }
      }
    }
  };

  auto compute = [&](int buf) __attribute__((always_inline)) {
    const TA* As = reinterpret_cast<const TA*>(smem + (NBUF == 2 ? buf : 0) * Cfg::BUF_BYTES);
    const TA* Bs = As + Cfg::A_ELEMS;
    constexpr int KL = KC / 4;  // k values per lane per chunk
    if constexpr (!BF) {
      // all fragments of the chunk first, then k-outer / row-block-inner so
      // that consecutive MFMAs accumulate into different registers.  Lane
      // group g carries k = g*KL .. g*KL + KL - 1: chunks g*KL/EPC onwards.
      constexpr int EPC = Cfg::EPC, NCH = KL / EPC;
      TA bv[CBW][KL], av[RBW][KL];
#pragma unroll
      for (int c = 0; c < CBW; ++c) {
        const int col = cbase - col0 + wc * 16 * CBW + c * 16 + r16;
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
          const TA* p = Bs + Cfg::off(col, g * NCH + q);
#pragma unroll
          for (int x = 0; x < EPC; ++x) bv[c][q * EPC + x] = p[x];
        }
      }
      // rows past ld are staged as zeros, so every row block is computed
      // unconditionally; only the epilogue skips them
#pragma unroll
      for (int i = 0; i < RBW; ++i) {
        const int arow = (wr * RBW + i) * 16 + r16;
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
          const TA* p = As + Cfg::off(arow, g * NCH + q);
#pragma unroll
          for (int x = 0; x < EPC; ++x) av[i][q * EPC + x] = p[x];
        }
      }
#pragma unroll
      for (int e = 0; e < KL; ++e)
#pragma unroll
        for (int i = 0; i < RBW; ++i)
#pragma unroll
            for (int c = 0; c < CBW; ++c) {
              if constexpr (MODE == GM_F32)
                acc[i][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][e], bv[c][e], acc[i][c], 0, 0, 0);
              else
                acc[i][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][e], bv[c][e], acc[i][c], 0, 0, 0);
            }
    } else {
      using vec8 = typename std::conditional<MODE == GM_H3, f16x8, bf16x8>::type;
      auto mma = [](vec8 x, vec8 y, f32x4 c) {
        if constexpr (MODE == GM_H3) return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
        else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
      };
      vec8 bh[CBW], bm[CBW], bl[CBW];
#pragma unroll
      for (int c = 0; c < CBW; ++c) {
        const int col = cbase - col0 + wc * 16 * CBW + c * 16 + r16;
        const int o = Cfg::off(col, g);
        bh[c] = *reinterpret_cast<const vec8*>(Bs + o);
        bl[c] = *reinterpret_cast<const vec8*>(Bs + (NB - 1) * Cfg::B_TSTRIDE + o);
        if constexpr (NB == 3) bm[c] = *reinterpret_cast<const vec8*>(Bs + Cfg::B_TSTRIDE + o);
      }
#pragma unroll
      for (int i = 0; i < RBW; ++i) {
        const int o = Cfg::off((wr * RBW + i) * 16 + r16, g);
        const vec8 ah = *reinterpret_cast<const vec8*>(As + o);
        const vec8 al = *reinterpret_cast<const vec8*>(As + Cfg::A_TSTRIDE + o);
#pragma unroll
        for (int c = 0; c < CBW; ++c) {
          acc[i][c] = mma(ah, bh[c], acc[i][c]);
          acc[i][c] = mma(al, bh[c], acc[i][c]);
          if constexpr (NB == 3) {
            acc[i][c] = mma(ah, bm[c], acc[i][c]);
            acc[i][c] = mma(al, bm[c], acc[i][c]);
          }
          acc[i][c] = mma(ah, bl[c], acc[i][c]);
        }
      }
    }
    // keep the staging of later chunks (which waits for their global loads)
    // behind this chunk's matrix instructions
    __builtin_amdgcn_sched_barrier(0);
  };

  auto flush = [&]() __attribute__((always_inline)) {
    if constexpr (FLUSH) {
#pragma unroll
      for (int i = 0; i < RBW; ++i)
#pragma unroll
        for (int c = 0; c < CBW; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            acc64[i][c][v] += double(acc[i][c][v]);
            acc[i][c][v] = 0;
          }
    }
  };

  if (nchunks > 0) {
    for (int i = tid; i < se - sb; i += NT) s_ops[i] = a.step_op[sb + i];
    __syncthreads();
    fetch_step(sb);
    begin_step();
    fetch_step(sb + 1);
    const std::integral_constant<int, 0> R0;
    const std::integral_constant<int, 1> R1;
    auto issue = [&](auto P) __attribute__((always_inline)) {  // the next chunk in order
      advance();
      load_regs(P);
    };
    int cm_kc = 0;  // chunk within the step, on the compute side
    auto step_end = [&]() __attribute__((always_inline)) {
      if (++cm_kc == kcs) {
        cm_kc = 0;
        flush();
      }
    };
    load_regs(R0);
    store_lds(R0, 0);
    if (nchunks > 1) issue(R1);
    __syncthreads();
    // Chunk c is computed from LDS buffer c % 2; while it is, chunk c + 2 is
    // loaded into register set c % 2 and chunk c + 1 moves from set
    // (c + 1) % 2 into the other buffer.  The loop runs two chunks at a time
    // with no branches around loads and stores; the last one to three chunks
    // follow it.
    int ch = 0;
    // with one LDS buffer, every wave must be done reading it before the
    // next chunk is stored
    auto reuse = [&]() __attribute__((always_inline)) {
      if constexpr (NBUF == 1) __syncthreads();
    };
    for (; ch + 3 < nchunks; ch += 2) {
      issue(R0);
      compute(0);
      step_end();
      reuse();
      store_lds(R1, 1);
      __syncthreads();
      issue(R1);
      compute(1);
      step_end();
      reuse();
      store_lds(R0, 0);
      __syncthreads();
    }
    if (ch + 2 < nchunks) issue(R0);
    compute(0);
    step_end();
    if (ch + 1 < nchunks) {
      reuse();
      store_lds(R1, 1);
      __syncthreads();
      compute(1);
      step_end();
      if (ch + 2 < nchunks) {
        reuse();
        store_lds(R0, 0);
        __syncthreads();
        compute(0);
        step_end();
      }
    }
  }

#pragma unroll
  for (int c = 0; c < CBW; ++c) {
    const int s = cbase + wc * 16 * CBW + c * 16 + r16;
    if (s < ncols) {
      const int b = s / a.n_rhs, r = s % a.n_rhs;
      const int box = a.tile_cols[int64_t(tile) * a.TB + b];
      if (box >= 0) {
        TO* o = static_cast<TO*>(a.out) + (int64_t(box) * a.n_rhs + r) * ld;
#pragma unroll
        for (int i = 0; i < RBW; ++i) {
          if (wr * RBW + i < nrb) {
            // summed in the wider of the accumulator and output types
            using TAcc = typename std::conditional<(sizeof(TO) > sizeof(acc[0][0][0])), TO,
                                                   decltype(acc[0][0][0] + 0)>::type;
            TAcc val[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              val[v] = TAcc(acc[i][c][v]);
              if constexpr (FLUSH) val[v] = TAcc(acc64[i][c][v] + double(acc[i][c][v]));
              if constexpr (MODE == GM_H3) val[v] *= TAcc(out_scale);
            }
            const int rbase = row0 + (wr * RBW + i) * 16;
            if (a.atomic) {
#pragma unroll
              for (int v = 0; v < 4; ++v) unsafeAtomicAdd(o + rbase + G::row(lane, v), TO(val[v]));
            } else if constexpr (G::ROWS4 && sizeof(TO) == 4) {
              // the lane's four rows are consecutive: one 16-byte access
              f32x4* o4 = reinterpret_cast<f32x4*>(o + rbase + G::row(lane, 0));
              f32x4 w;
              if (a.accumulate) w = *o4;
#pragma unroll
              for (int v = 0; v < 4; ++v) w[v] = a.accumulate ? float(val[v] + TAcc(w[v])) : float(val[v]);
              *o4 = w;
            } else {
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int row = rbase + G::row(lane, v);
                TAcc x = val[v];
                if (a.accumulate) x += TAcc(o[row]);
                o[row] = TO(x);
              }
            }
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------------
// pipeline
// ------------------------------------------------------------------------

// Split-precision M2L with wide tiles (BF16x3 and FP16x3: two operator parts,
// two density parts).  A block owns 160 rows x 128 output columns; its four
// waves each own 80 rows x 64 columns (5 x 4 MFMA blocks of 16 x 16), so a
// wave reads 10 KB of operator fragments from LDS per 60 MFMAs instead of
// 14 KB per 30 in gemm_kernel's 80 x 32 wave tiles.  Only the operator goes
// through LDS, double-buffered (one barrier per 32-wide k chunk); every lane
// loads its density fragments (8 consecutive k of one column, both parts)
// straight from the chunk-interleaved split operand into registers, one
// chunk ahead.  Same plans, same arithmetic and summation order per column
// as gemm_kernel, so the results are bitwise equal to it.
template <int MODE, class TO>
__global__ __launch_bounds__(256, 2) void m2l_wide_kernel(GemmArgs a) {
  using G = GT<MODE>;
  using TA = typename G::TA;
  static_assert(G::NB == 2 && (MODE == GM_BF3 || MODE == GM_H3), "two density parts");
  using Cfg = GemmCfg<MODE, TA, TO, 2, 1, kRB>;  // the operator side of the 160-row tile
  constexpr int KC = 32, RBW = kRB / 2, CBW = 4, NT = 256;
  constexpr int A_BYTES = Cfg::A_ELEMS * int(sizeof(TA));
  using vec8 = typename std::conditional<MODE == GM_H3, f16x8, bf16x8>::type;
  __shared__ __align__(16) unsigned char smem[2 * A_BYTES];
  __shared__ int s_ops[kMaxTileSteps];
  float out_scale = 1.0f;
  if constexpr (MODE == GM_H3) out_scale = ldexpf(1.0f, -f16_density_exp(a.absmax) - kF16OpExp);

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, r16 = lane & 15;
  const int wr = wave >> 1, wc = wave & 1;
  const int tile = blockIdx.x;
  const int row0 = blockIdx.y * Cfg::ROWS;
  const int nrb = min(kRB, (a.ld - row0) / 16);
  const int ld = a.ld;
  const int ncols = a.TB * a.n_rhs;
  const int sb = a.step_beg[tile], se = a.step_beg[tile + 1];
  const int kcs = ld / KC;
  const int nchunks = (se - sb) * kcs;

  f32x4 acc[RBW][CBW];
#pragma unroll
  for (int i = 0; i < RBW; ++i)
#pragma unroll
    for (int c = 0; c < CBW; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][c][v] = 0.0f;

  // operator staging: the same units and LDS slots as gemm_kernel's
  int a_goff[Cfg::A_PER_T], a_loff[Cfg::A_PER_T];
#pragma unroll
  for (int j = 0; j < Cfg::A_PER_T; ++j) {
    const int u = (tid + j * NT) % Cfg::A_UNITS;
    const int part = u % Cfg::CPR, rsub = (u / Cfg::CPR) & 1, t = (u / (2 * Cfg::CPR)) % 2;
    const int rl = (u / (2 * Cfg::CPR * 2)) * 2 + rsub;
    const int rg = min(row0 + rl, ld - 1);
    a_goff[j] = rg * ld * 2 + t * KC + part * Cfg::EPC;
    a_loff[j] = t * Cfg::A_TSTRIDE + Cfg::off(rl, part);
  }
  u32x4 ra[Cfg::A_PER_T];
  // density fragments of two chunks: [set][column block][part]
  u32x4 rb[2][CBW][2];
  const u32x4* inb = static_cast<const u32x4*>(a.in);
  const uint32_t col_units = uint32_t(ld * 2 * int(sizeof(TA)) / 16);  // 16-byte units per column
  // the lane's column of each column block (within the tile), and the 16-byte
  // unit of its k group in that column of the step being loaded
  // (the source boxes of the next step are fetched a whole step ahead)
  uint32_t b_base[CBW];
  int nxt_src[CBW];
  int ld_st = sb, ld_kc = 0;  // step and chunk of the chunk being loaded
  int cur_op = 0;
  auto fetch_src = [&](int st) __attribute__((always_inline)) {
    const int sc = min(st, se - 1);
#pragma unroll
    for (int c = 0; c < CBW; ++c) {
      const int s = wc * 64 + c * 16 + r16;
      nxt_src[c] = s < ncols ? a.step_src[int64_t(sc) * a.TB + s / a.n_rhs] : a.zero_box;
    }
  };
  auto begin_step = [&]() __attribute__((always_inline)) {
    cur_op = s_ops[min(ld_st, se - 1) - sb];
#pragma unroll
    for (int c = 0; c < CBW; ++c) {
      const int s = wc * 64 + c * 16 + r16;
      b_base[c] = (uint32_t(nxt_src[c]) * uint32_t(a.n_rhs) + uint32_t(s % a.n_rhs)) * col_units + uint32_t(g);
    }
  };
  auto load = [&](int set) __attribute__((always_inline)) {
    const TA* opb = static_cast<const TA*>(a.ops) + int64_t(cur_op) * a.op_stride + 2 * (ld_kc * KC);
#pragma unroll
    for (int j = 0; j < Cfg::A_PER_T; ++j) ra[j] = *reinterpret_cast<const u32x4*>(opb + a_goff[j]);
#pragma unroll
    for (int c = 0; c < CBW; ++c)
#pragma unroll
      for (int t = 0; t < 2; ++t) rb[set][c][t] = inb[b_base[c] + uint32_t(ld_kc * 8 + t * 4)];
  };
  auto advance = [&]() __attribute__((always_inline)) {
    if (++ld_kc == kcs) {
      ld_kc = 0;
      ++ld_st;
      begin_step();
      fetch_src(ld_st + 1);
    }
  };
  auto store_a = [&](int buf) __attribute__((always_inline)) {
    TA* As = reinterpret_cast<TA*>(smem + buf * A_BYTES);
#pragma unroll
    for (int j = 0; j < Cfg::A_PER_T; ++j) *reinterpret_cast<u32x4*>(As + a_loff[j]) = ra[j];
  };
  auto mma = [](vec8 x, vec8 y, f32x4 c) __attribute__((always_inline)) {
    if constexpr (MODE == GM_H3) return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
  };
  auto compute = [&](int buf, int set) __attribute__((always_inline)) {
    const TA* As = reinterpret_cast<const TA*>(smem + buf * A_BYTES);
#pragma unroll
    for (int i = 0; i < RBW; ++i) {
      const int o = Cfg::off((wr * RBW + i) * 16 + r16, g);
      const vec8 ah = *reinterpret_cast<const vec8*>(As + o);
      const vec8 al = *reinterpret_cast<const vec8*>(As + Cfg::A_TSTRIDE + o);
#pragma unroll
      for (int c = 0; c < CBW; ++c) {
        const vec8 bh = __builtin_bit_cast(vec8, rb[set][c][0]);
        const vec8 bl = __builtin_bit_cast(vec8, rb[set][c][1]);
        acc[i][c] = mma(ah, bh, acc[i][c]);
        acc[i][c] = mma(al, bh, acc[i][c]);
        acc[i][c] = mma(ah, bl, acc[i][c]);
      }
    }
  };

  if (nchunks > 0) {
    for (int i = tid; i < se - sb; i += NT) s_ops[i] = a.step_op[sb + i];
    __syncthreads();
    fetch_src(sb);
    begin_step();
    fetch_src(sb + 1);
    load(0);
    store_a(0);
    if (nchunks > 1) {
      advance();
      load(1);
    }
    __syncthreads();
    // chunk c: computed from LDS buffer c % 2 and register set c % 2; its
    // operator for chunk c + 1 goes to the other buffer, then chunk c + 2 is
    // loaded into the freed register set
    const std::integral_constant<int, 0> S0;
    const std::integral_constant<int, 1> S1;
    auto iteration = [&](int c, auto SET) __attribute__((always_inline)) {
      constexpr int set = decltype(SET)::value;
      compute(set, set);
      if (c + 1 < nchunks) store_a(set ^ 1);
      if (c + 2 < nchunks) {
        advance();
        load(set);
      }
      __syncthreads();
    };
    int c = 0;
    for (; c + 1 < nchunks; c += 2) {
      iteration(c, S0);
      iteration(c + 1, S1);
    }
    if (c < nchunks) iteration(c, S0);
  }

#pragma unroll
  for (int cb = 0; cb < CBW; ++cb) {
    const int s = wc * 64 + cb * 16 + r16;
    if (s < ncols) {
      const int b = s / a.n_rhs, r = s % a.n_rhs;
      const int box = a.tile_cols[int64_t(tile) * a.TB + b];
      if (box >= 0) {
        TO* o = static_cast<TO*>(a.out) + (int64_t(box) * a.n_rhs + r) * ld;
#pragma unroll
        for (int i = 0; i < RBW; ++i) {
          if (wr * RBW + i < nrb) {
            const int rbase = row0 + (wr * RBW + i) * 16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              float val = acc[i][cb][v];
              if constexpr (MODE == GM_H3) val *= out_scale;
              unsafeAtomicAdd(o + rbase + G::row(lane, v), TO(val));
            }
          }
        }
      }
    }
  }
}

// Split-precision M2L with asynchronous staging (BF16x3 and FP16x3, tiles of
// 16 NCB columns: 64, 128 or 160).  Operator and density chunks go from
// global memory straight into LDS (global_load_lds, 16 bytes a lane, no
// registers on the way) in two stages: while chunk c feeds the matrix cores
// from one stage, chunk c + 1 lands in the other, and one barrier per chunk
// hands the stages over.  With no staging registers, a wave reads all
// fragments of its chunk first and then issues its MFMAs back to back.
// Block shape (four waves in a 2 x 2 grid, wave tiles of 8 RB x 8 NCB), plans,
// arithmetic and summation order per column are gemm_kernel's, so the
// results are bitwise equal to it.  Gathered tiles add into the output with
// atomics (two terms a value); pair tiles store their products.
//
// LDS traffic is arranged in 1 KB blocks (16 rows or columns of one part,
// 64 bytes each): a stage holds 2 RB operator blocks and 2 NCB density
// blocks (80 KB a block at RB = NCB = 10, so two blocks fill a CU's 160 KB),
// and wave w fills operator blocks w, w + 4, ... and the density blocks
// (both parts) of column blocks w, w + 4, w + 8.  One load instruction
// writes one block, lane i to its 16-byte slot i, so each lane fetches the
// global chunk that the XOR swizzle of the layout puts in that slot (the
// swizzle is an involution).
template <int MODE, class TO, int RB, int NCB, bool FLUSH = false>
__global__ __launch_bounds__(256, 2) void m2l_async_kernel(GemmArgs a) {
  using G = GT<MODE>;
  using TA = typename G::TA;
  static_assert(G::NB == 2 && (MODE == GM_BF3 || MODE == GM_H3), "two density parts");
  static_assert(G::KC == 32 && sizeof(TA) == 2, "64-byte LDS rows");
  static_assert(NCB % 2 == 0 && NCB <= 12 && RB % 2 == 0, "two wave columns, two wave rows");
  constexpr int KC = 32, RBW = RB / 2, CBW = NCB / 2;
  static_assert((2 * RB) % 4 == 0, "operator blocks are dealt evenly to the four waves");
  constexpr int A_PER_W = 2 * RB / 4;
  constexpr int B_PER_W = (NCB + 3) / 4;   // column blocks per wave (the last may be absent)
  constexpr int BLK = 16 * KC;              // elements of a 1 KB block
  constexpr int A_PART = RB * 16 * KC;      // operator part table of a stage
  constexpr int B_PART = NCB * 16 * KC;     // density part table of a stage
  constexpr int A_ELEMS = 2 * A_PART, STAGE = A_ELEMS + 2 * B_PART;
  constexpr int EPC = 8;                    // elements per 16-byte chunk
  // chunk of a 64-byte row, XOR-swizzled so that a fragment read (lane =
  // row, one chunk column) meets no bank conflicts
  auto swz = [](int row, int chunk) __attribute__((always_inline)) { return chunk ^ ((row >> 1) & 3); };
  auto off = [&](int row, int chunk) __attribute__((always_inline)) { return row * KC + swz(row, chunk) * EPC; };
  using vec8 = typename std::conditional<MODE == GM_H3, f16x8, bf16x8>::type;
  __shared__ __align__(16) TA stage0[STAGE];
  __shared__ __align__(16) TA stage1[STAGE];
  float out_scale = 1.0f;
  if constexpr (MODE == GM_H3) out_scale = ldexpf(1.0f, -f16_density_exp(a.absmax) - kF16OpExp);

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, r16 = lane & 15;
  const int wr = wave >> 1, wc = wave & 1;
  // Blocks are dealt to the 8 XCDs round-robin.  The grid is 1-D over the
  // tiles (padded to a multiple of 8) times the row blocks, row block
  // slowest, numbered so that XCD x receives tiles x, x + 8, ... (the plan's
  // XCD queues) in every row block: the blocks running together then share
  // one row slice of each operator.  (Running a tile's row blocks together
  // instead, to share its density columns, measured slower.)
  const int T8 = (a.ntile + 7) / 8;  // groups of 8 tiles
  const int xcd = int(blockIdx.x & 7), kx = int(blockIdx.x >> 3);
  const int tile = (kx % T8) * 8 + xcd;
  if (tile >= a.ntile) return;  // padding of the last group of 8 tiles
  const int row0 = (kx / T8) * RB * 16;
  const int nrb = min(RB, (a.ld - row0) / 16);
  const int ld = a.ld;
  const int ncols = a.TB * a.n_rhs;
  const int sb = a.step_beg[tile], se = a.step_beg[tile + 1];
  const int kcs = ld / KC;
  const int nchunks = (se - sb) * kcs;

  f32x4 acc[RBW][CBW];
#pragma unroll
  for (int i = 0; i < RBW; ++i)
#pragma unroll
    for (int c = 0; c < CBW; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][c][v] = 0.0f;
  // FLUSH (FP64 sums, as gemm_kernel's TAG 2): after every operator step the
  // FP32 sums move into FP64 registers
  f64x4 acc64[FLUSH ? RBW : 1][FLUSH ? CBW : 1];
  if constexpr (FLUSH) {
#pragma unroll
    for (int i = 0; i < RBW; ++i)
#pragma unroll
      for (int c = 0; c < CBW; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc64[i][c][v] = 0.0;
  }

  // operator blocks of this wave: element offsets in an operator (chunk 0)
  // and the blocks' places in a stage.  Rows past ld are clamped to a valid
  // row; they only feed output rows the epilogue discards.
  uint32_t a_goff[A_PER_W];
  int a_dst[A_PER_W];
#pragma unroll
  for (int j = 0; j < A_PER_W; ++j) {
    const int q = wave + 4 * j, t = q / RB, rb = q % RB;
    const int rl = rb * 16 + (lane >> 2);
    const int rg = min(row0 + rl, ld - 1);
    a_goff[j] = uint32_t(rg * ld * 2 + t * KC + swz(rl, lane & 3) * EPC);
    a_dst[j] = t * A_PART + rb * BLK;
  }
  // density blocks: column slots 16 (wave + 4 m) + lane / 4 of the tile
  int slot[B_PER_W];
  uint32_t b_chunk[B_PER_W];
#pragma unroll
  for (int m = 0; m < B_PER_W; ++m) {
    slot[m] = 16 * (wave + 4 * m) + (lane >> 2);
    b_chunk[m] = uint32_t(swz(slot[m], lane & 3));
  }
  auto has_block = [&](int m) __attribute__((always_inline)) { return wave + 4 * m < NCB; };
  const uint32_t col_units = uint32_t(ld * 2 * int(sizeof(TA)) / 16);  // 16-byte units per column
  uint32_t b_goff[B_PER_W];  // 16-byte unit of the slot's column, chunk 0, part 0
  // Step and chunk of the next chunk to request.  The operator index and the
  // source boxes of the following step are fetched a whole step ahead (the
  // step's loads complete at a handover, before they are used).  Slots past
  // the tile's columns load the last column's boxes: they only feed output
  // columns that the epilogue drops.
  int ld_st = sb, ld_kc = 0, cur_op = 0, nxt_op = 0, nxt_src[B_PER_W];
  auto fetch_step = [&](int st) __attribute__((always_inline)) {
    const int sc = min(st, se - 1);
    nxt_op = a.step_op[sc];
#pragma unroll
    for (int m = 0; m < B_PER_W; ++m)
      nxt_src[m] = a.step_src[int64_t(sc) * a.TB + min(slot[m] / a.n_rhs, a.TB - 1)];
  };
  auto begin_step = [&]() __attribute__((always_inline)) {
    cur_op = nxt_op;
#pragma unroll
    for (int m = 0; m < B_PER_W; ++m)
      b_goff[m] = (uint32_t(nxt_src[m]) * uint32_t(a.n_rhs) + uint32_t(slot[m] % a.n_rhs)) * col_units + b_chunk[m];
  };
  auto advance = [&]() __attribute__((always_inline)) {
    if (++ld_kc == kcs) {
      ld_kc = 0;
      ++ld_st;
      begin_step();
      fetch_step(ld_st + 1);
    }
  };
  // the loads of the chunk (ld_st, ld_kc) into stage S
  auto issue = [&](auto S) __attribute__((always_inline)) {
    TA* st = decltype(S)::value == 0 ? stage0 : stage1;
    const TA* opb = static_cast<const TA*>(a.ops) + int64_t(cur_op) * a.op_stride + 2 * (ld_kc * KC);
#pragma unroll
    for (int j = 0; j < A_PER_W; ++j)
      __builtin_amdgcn_global_load_lds((void*)(opb + a_goff[j]), (void*)(st + a_dst[j]), 16, 0, 0);
#pragma unroll
    for (int m = 0; m < B_PER_W; ++m) {
      if (has_block(m)) {
        const u32x4* inb = static_cast<const u32x4*>(a.in) + b_goff[m] + uint32_t(ld_kc * 8);
#pragma unroll
        for (int t = 0; t < 2; ++t)
          __builtin_amdgcn_global_load_lds((void*)(inb + 4 * t),
                                           (void*)(st + A_ELEMS + t * B_PART + (wave + 4 * m) * BLK), 16, 0, 0);
      }
    }
  };
  // this wave's loads have landed, then every wave's (and every wave is done
  // with the chunk before); no instruction crosses this point (the scheduler
  // would otherwise move the MFMAs of the chunk before it behind the wait)
  auto handover = [&]() __attribute__((always_inline)) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  };
  auto mma = [](vec8 x, vec8 y, f32x4 c) __attribute__((always_inline)) {
    if constexpr (MODE == GM_H3) return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
  };
  auto compute = [&](auto S) __attribute__((always_inline)) {
    // the loads issued before stay ahead of this chunk's work
    __builtin_amdgcn_sched_barrier(0);
    const TA* As = decltype(S)::value == 0 ? stage0 : stage1;
    const TA* Bs = As + A_ELEMS;
    vec8 bh[CBW], bl[CBW], ah[RBW], al[RBW];
#pragma unroll
    for (int c = 0; c < CBW; ++c) {
      const int o = off(wc * 16 * CBW + c * 16 + r16, g);
      bh[c] = *reinterpret_cast<const vec8*>(Bs + o);
      bl[c] = *reinterpret_cast<const vec8*>(Bs + B_PART + o);
    }
#pragma unroll
    for (int i = 0; i < RBW; ++i) {
      const int o = off((wr * RBW + i) * 16 + r16, g);
      ah[i] = *reinterpret_cast<const vec8*>(As + o);
      al[i] = *reinterpret_cast<const vec8*>(As + A_PART + o);
    }
    // per accumulator A_h x_h, A_l x_h, A_h x_l (gemm_kernel's order);
    // consecutive products go to different accumulators
#pragma unroll
    for (int i = 0; i < RBW; ++i)
#pragma unroll
      for (int c = 0; c < CBW; ++c) {
        acc[i][c] = mma(ah[i], bh[c], acc[i][c]);
        acc[i][c] = mma(al[i], bh[c], acc[i][c]);
        acc[i][c] = mma(ah[i], bl[c], acc[i][c]);
      }
    // every fragment read first (in the order above, so the first products
    // wait for the first reads only), then the products
    __builtin_amdgcn_sched_group_barrier(0x100, 2 * (CBW + RBW), 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 3 * CBW * RBW, 0);
  };

  int cm_kc = 0;  // chunk within the step, on the compute side
  auto step_end = [&]() __attribute__((always_inline)) {
    if constexpr (FLUSH) {
      if (++cm_kc == kcs) {
        cm_kc = 0;
#pragma unroll
        for (int i = 0; i < RBW; ++i)
#pragma unroll
          for (int c = 0; c < CBW; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              acc64[i][c][v] += double(acc[i][c][v]);
              acc[i][c][v] = 0.0f;
            }
      }
    }
  };

  if (nchunks > 0) {
    fetch_step(sb);
    begin_step();
    fetch_step(sb + 1);
    const std::integral_constant<int, 0> S0;
    const std::integral_constant<int, 1> S1;
    issue(S0);
    int c = 0;
    for (; c + 1 < nchunks; c += 2) {
      handover();
      advance();
      issue(S1);
      compute(S0);
      step_end();
      handover();
      if (c + 2 < nchunks) {
        advance();
        issue(S0);
      }
      compute(S1);
      step_end();
    }
    if (c < nchunks) {
      handover();
      compute(S0);
      step_end();
    }
  }

#pragma unroll
  for (int cb = 0; cb < CBW; ++cb) {
    const int s = wc * 16 * CBW + cb * 16 + r16;
    if (s < ncols) {
      const int b = s / a.n_rhs, r = s % a.n_rhs;
      const int box = a.tile_cols[int64_t(tile) * a.TB + b];
      if (box >= 0) {
        TO* o = static_cast<TO*>(a.out) + (int64_t(box) * a.n_rhs + r) * ld;
#pragma unroll
        for (int i = 0; i < RBW; ++i) {
          if (wr * RBW + i < nrb) {
            const int rbase = row0 + (wr * RBW + i) * 16;
            // summed in the wider of FP32 and the output type (gemm_kernel's rule)
            using TAcc = typename std::conditional<(sizeof(TO) > 4), TO, float>::type;
            TAcc val[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              val[v] = TAcc(acc[i][cb][v]);
              if constexpr (FLUSH) val[v] = TAcc(acc64[i][cb][v] + double(acc[i][cb][v]));
              if constexpr (MODE == GM_H3) val[v] *= TAcc(out_scale);
            }
            if (a.atomic) {
#pragma unroll
              for (int v = 0; v < 4; ++v) unsafeAtomicAdd(o + rbase + G::row(lane, v), TO(val[v]));
            } else if constexpr (sizeof(TO) == 4) {
              // pair tiles: every output written once; the lane's four rows
              // are consecutive, one 16-byte store
              static_assert(G::ROWS4, "four consecutive rows a lane");
              f32x4 w;
#pragma unroll
              for (int v = 0; v < 4; ++v) w[v] = float(val[v]);
              *reinterpret_cast<f32x4*>(o + rbase + G::row(lane, 0)) = w;
            } else {
#pragma unroll
              for (int v = 0; v < 4; ++v) o[rbase + G::row(lane, v)] = TO(val[v]);
            }
          }
        }
      }
    }
  }
}

// Split-precision M2L plans of up to 160 columns run m2l_async_kernel (1) or
// gemm_kernel (0); the two give bitwise equal results.
static bool g_m2l_async = true;
void set_m2l_async(bool on) { g_m2l_async = on; }

// Split-precision M2L plans of 65..128 columns run m2l_wide_kernel (1) or
// gemm_kernel (0); the two give bitwise equal results.
static bool g_m2l_wide = false;
void set_m2l_wide(bool on) { g_m2l_wide = on; }

// Operator rows per M2L block: 160 or 128, or 0 to take the one that pads
// the operator's ld rows the least (160 at ld = 160 and 320; 128 at ld = 64,
// 128, 224 and 512, i.e. p = 4, 5, 7 and 10).  Rows are independent
// outputs, so the choice does not change any result.
static int g_m2l_rows = 0;
void set_m2l_rows(int rows) { g_m2l_rows = rows; }
static int m2l_block_rows(int ld) {
  if (g_m2l_rows) return g_m2l_rows;
  const int c160 = (ld + 159) / 160 * 160, c128 = (ld + 127) / 128 * 128;
  return c128 < c160 ? 128 : 160;
}

// 16-byte units spanned by the input columns of a gathered GEMM (boxes
// 0..zero_box, n_rhs columns each of ld rows, split modes NB parts a row)
template <int MODE, class TI>
uint64_t gemm_in_units(int64_t zero_box, int64_t n_rhs, int64_t ld) {
  using Cfg = GemmCfg<MODE, TI, float, 1, 1, kRB>;
  const uint64_t parts = Cfg::SPLIT ? uint64_t(Cfg::NB) : 1u;
  return uint64_t(zero_box + 1) * uint64_t(n_rhs) * uint64_t(ld) * parts * sizeof(TI) / 16;
}

// zero_box: the forest's box count; the columns of that box in every buffer
// are allocated, zero, and never written.
template <int MODE, class TI, class TO, int TAG = 0>
static void run_gemm(const DevPlan& P, const void* ops, int64_t op_stride, int ld, int zero_box,
                     int n_rhs, const TI* in, TO* out, bool accumulate, hipStream_t s,
                     PhaseScope& ps, const unsigned* absmax = nullptr) {
  if (P.ntile == 0) return;
  const int ncols = P.TB * n_rhs;
  if (ncols > 192) raise(KIFMM_EUNSUPPORTED, "plan width exceeds the GEMM tile");
  if (ld % 32) raise(KIFMM_EINVAL, "operator leading dimension must be a multiple of 32");
  if (P.max_tile_steps > kMaxTileSteps) raise(KIFMM_EUNSUPPORTED, "GEMM tile with too many operator steps");
  // the kernel addresses its input columns in 32-bit counts of 16-byte units
  if (gemm_in_units<MODE, TI>(zero_box, n_rhs, ld) > (uint64_t(1) << 32))
    raise(KIFMM_EUNSUPPORTED, "GEMM operand beyond 64 GiB (boxes x right-hand sides x rows)");
  GemmArgs g{ops, op_stride, ld, n_rhs, accumulate ? 1 : 0, P.TB, in, out,
             P.tile_cols, P.step_beg, P.step_op, P.step_src, absmax, zero_box, P.atomic ? 1 : 0,
             int(P.ntile)};
  // split-precision M2L tiles of up to 160 columns (gathered tiles adding
  // with atomics, or pair tiles storing their products): the
  // asynchronous-staging kernel or (65..128 columns) the wide-tile kernel
  if constexpr ((MODE == GM_BF3 || MODE == GM_H3) && (TAG == 1 || TAG == 2)) {
    // with FP64 sums (TAG 2) the FP64 accumulators fit the registers of
    // tiles of up to 96 columns (128-row blocks) or 64 (160-row blocks)
    constexpr bool FL = TAG == 2;
    const bool r128 = m2l_block_rows(ld) == 128;
    if (g_m2l_async && ncols <= (FL ? (r128 ? 96 : 64) : 160) && (P.atomic || !accumulate)) {
      // 1-D grids: tiles padded to a multiple of 8, times the row blocks
      const unsigned t8 = unsigned((P.ntile + 7) / 8 * 8);
      const dim3 g128(t8 * unsigned((ld + 127) / 128)), g160(t8 * unsigned((ld + kROWS - 1) / kROWS));
      auto launch = [&](auto ncb) {
        constexpr int NCB = decltype(ncb)::value;
        if constexpr (!FL || NCB <= 6) {
          if (r128)
            hipLaunchKernelGGL((m2l_async_kernel<MODE, TO, 8, NCB, FL>), g128, dim3(256), 0, s, g);
          else if constexpr (!FL || NCB == 4)
            hipLaunchKernelGGL((m2l_async_kernel<MODE, TO, kRB, NCB, FL>), g160, dim3(256), 0, s, g);
        }
      };
      if (ncols <= 64) launch(std::integral_constant<int, 4>());
      else if (ncols <= 96) launch(std::integral_constant<int, 6>());
      else if (ncols <= 128) launch(std::integral_constant<int, 8>());
      else launch(std::integral_constant<int, 10>());
      LAUNCHCHECK("m2l_async_kernel");
      ps.launches++;
      return;
    }
  }
  if constexpr ((MODE == GM_BF3 || MODE == GM_H3) && TAG == 1) {
    if (g_m2l_wide && ncols > 64 && ncols <= 128 && P.atomic) {
      dim3 grid(P.ntile, (ld + kROWS - 1) / kROWS);
      hipLaunchKernelGGL((m2l_wide_kernel<MODE, TO>), grid, dim3(256), 0, s, g);
      LAUNCHCHECK("m2l_wide_kernel");
      ps.launches++;
      return;
    }
  }
  // plans with few tiles (the coarse levels of M2M, L2L and the solves) run
  // 32-row blocks: five times the blocks, a fifth of the work per block
  if constexpr (TAG == 0) {
    if (P.ntile < kFewTiles && ncols <= 64) {
      dim3 grid(P.ntile, (ld + 31) / 32);
      hipLaunchKernelGGL((gemm_kernel<MODE, TI, TO, 1, TAG, 1, 2>), grid, dim3(256), 0, s, g);
      LAUNCHCHECK("gemm_kernel");
      ps.launches++;
      return;
    }
  }
  // blocks of RB x 16 operator rows: 160 (10 row blocks) or, for M2L, 128
  // rows where fewer padded rows result (see m2l_block_rows)
  auto dispatch = [&](auto rb_tag) {
    constexpr int RB = decltype(rb_tag)::value;
    dim3 grid(P.ntile, (ld + RB * 16 - 1) / (RB * 16));
    if (ncols > 128) {
      if constexpr (GemmOcc<MODE, TO, 1, TAG, 3>::WIDE_OK) {
        hipLaunchKernelGGL((gemm_kernel<MODE, TI, TO, 1, TAG, 3, RB>), grid, dim3(768), 0, s, g);
      } else {
        grid.z = (ncols + 63) / 64;  // 64-column slices of the wide tiles
        hipLaunchKernelGGL((gemm_kernel<MODE, TI, TO, 1, TAG, 1, RB>), grid, dim3(256), 0, s, g);
      }
    } else if (ncols > 64) {
      hipLaunchKernelGGL((gemm_kernel<MODE, TI, TO, 2, TAG, 1, RB>), grid, dim3(256), 0, s, g);
    } else {
      hipLaunchKernelGGL((gemm_kernel<MODE, TI, TO, 1, TAG, 1, RB>), grid, dim3(256), 0, s, g);
    }
  };
  if constexpr (TAG != 0) {
    if (m2l_block_rows(ld) == 128) dispatch(std::integral_constant<int, 8>());
    else dispatch(std::integral_constant<int, kRB>());
  } else {
    dispatch(std::integral_constant<int, kRB>());
  }
  LAUNCHCHECK("gemm_kernel");
  ps.launches++;
}

template <class T, class TF, int MODE, int RC, int TCH, bool GRAD = false, bool SCR = false>
static void run_p2p(const P2PArgs<T>& args, int nwork, int n_rhs, hipStream_t s, PhaseScope& ps) {
  if (nwork == 0) return;
  dim3 grid(nwork, (n_rhs + RC - 1) / RC);
  hipLaunchKernelGGL((p2p_kernel<T, TF, MODE, RC, TCH, GRAD, SCR>), grid, dim3(256), 0, s, args);
  LAUNCHCHECK("p2p_kernel");
  ps.launches++;
}

// Equivalent-surface terms (L2P, M2P) can run in FP64 at high order: the
// equivalent densities cancel more strongly as p grows (the pseudo-inverse
// keeps singular values down to rcond), so FP32 kernel values limit the far
// field to ~1e-5 at p = 10.
static int g_far_fp64_min_p = 10;
void set_far_fp64_min_p(int p) { g_far_fp64_min_p = p; }

template <class T, int MODE, int TCH, bool SCR>
static void run_p2p_rhs(const P2PArgs<T>& args, int nwork, int n_rhs, bool far64, hipStream_t s,
                        PhaseScope& ps) {
  if (far64) {
    if (n_rhs == 1) run_p2p<T, double, MODE, 1, TCH, false, SCR>(args, nwork, n_rhs, s, ps);
    else run_p2p<T, double, MODE, 8, TCH, false, SCR>(args, nwork, n_rhs, s, ps);
  } else {
    if (n_rhs == 1) run_p2p<T, T, MODE, 1, TCH, false, SCR>(args, nwork, n_rhs, s, ps);
    else run_p2p<T, T, MODE, 8, TCH, false, SCR>(args, nwork, n_rhs, s, ps);
  }
}

template <class T, int MODE, int TCH>
static void run_p2p_rc(const P2PArgs<T>& args, int nwork, int n_rhs, bool far64, hipStream_t s,
                       PhaseScope& ps) {
  if constexpr (MODE == MODE_LEAF) {
    if (args.grad) {
      // potential and gradient: one right-hand side per block
      if (args.kappa != 0.0) {
        if (far64) run_p2p<T, double, MODE, 1, TCH, true, true>(args, nwork, n_rhs, s, ps);
        else run_p2p<T, T, MODE, 1, TCH, true, true>(args, nwork, n_rhs, s, ps);
      } else {
        if (far64) run_p2p<T, double, MODE, 1, TCH, true>(args, nwork, n_rhs, s, ps);
        else run_p2p<T, T, MODE, 1, TCH, true>(args, nwork, n_rhs, s, ps);
      }
      return;
    }
  }
  if (args.kappa != 0.0) run_p2p_rhs<T, MODE, TCH, true>(args, nwork, n_rhs, far64, s, ps);
  else run_p2p_rhs<T, MODE, TCH, false>(args, nwork, n_rhs, far64, s, ps);
}

// Where the near field forks off the evaluation stream: 0 right after the
// gather, 2 after P2M (it then overlaps the latency-bound M2M / C2E chain
// rather than P2M), 1 just before M2L, 3 right after M2L (overlapping the
// L2L / C2E chain); 4 (default): no fork, near and far field as one kernel
// at the end.  Measured on 1M points: the concurrent near field takes the
// compute units the chain kernels would use, so the forked schedules are no
// faster than running everything in order, and the one merged kernel saves
// the far field's own pass over the leaves.
static int g_near_fork = 4;
void set_near_fork(int v) { g_near_fork = v; }

// Per-device auxiliary stream and fork/join events of the pipeline (default
// priority, non-blocking; created once and kept for the process).
struct Aux {
  hipStream_t stream = nullptr;
  hipEvent_t forked = nullptr, joined = nullptr;
};
static Aux& aux_for(int dev) {
  static std::map<int, Aux> m;
  Aux& x = m[dev];
  if (!x.stream) {
    HIPCHECK(hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&x.forked, hipEventDisableTiming));
    HIPCHECK(hipEventCreateWithFlags(&x.joined, hipEventDisableTiming));
  }
  return x;
}

template <class T, class TIO>
static void pipeline(DevForest& F, DevOps& O, DevWork& W, const void* const* charges,
                     void* const* potentials, int n_rhs, kifmm_precision prec, bool check_form,
                     bool grad, hipStream_t s) {
  constexpr int GF = sizeof(T) == 8 ? GM_F64 : GM_F32;
  const int ld = F.ld;
  Aux& aux = aux_for(current_device());
  const int64_t nn = int64_t(ld) * ld;
  T* qs = static_cast<T*>(W.qs);
  T* up_chk = static_cast<T*>(W.up_chk);
  T* up_eq = static_cast<T*>(W.up_eq);
  T* dn_chk = static_cast<T*>(W.dn_chk);
  T* dn_eq = static_cast<T*>(W.dn_eq);
  const T* m2m = nullptr;
  const T* l2l = nullptr;
  if constexpr (sizeof(T) == 8) {
    m2m = O.m2m64;
    l2l = O.l2l64;
  } else {
    m2m = O.m2m32;
    l2l = O.l2l32;
  }
  // the operator set of level l (one set for the Laplace kernel)
  if (O.levels > 1 && F.depth > O.levels - 1)
    raise(KIFMM_EINVAL, "evaluate: the forest is deeper than the operators' levels");
  auto set = [&](int l) { return int64_t(O.levels > 1 ? l : 0); };

  {
    PhaseScope ps(PH_GATHER, s);
    for (int k0 = 0; k0 < F.nprob; k0 += kMaxProb) {
      int nk = std::min(kMaxProb, F.nprob - k0);
      PtrPack pk{};
      for (int k = 0; k < nk; ++k) pk.p[k] = charges[k0 + k];
      dim3 grid(unsigned((F.max_src_per_prob + 255) / 256), nk);
      hipLaunchKernelGGL((gather_kernel<TIO, T>), grid, dim3(256), 0, s, pk, k0, F.src_off,
                         F.src_perm, n_rhs, F.nsrc, qs);
      LAUNCHCHECK("gather_kernel");
      ps.launches++;
    }
  }
  P2PArgs<T> base{};
  base.box_geo = F.box_geo;
  base.box_r = F.box_r;
  base.box_src = F.box_src;
  base.box_tgt = F.box_tgt;
  base.src64 = F.src64;
  base.tgt64 = F.tgt64;
  base.qs = qs;
  base.nsrc = F.nsrc;
  base.n_rhs = n_rhs;
  base.surf = O.surf;
  base.n = O.n;
  base.ld = ld;
  base.up_eq = up_eq;
  base.dn_eq = dn_eq;
  base.pot = W.pot;
  base.ntgt = F.ntgt;
  base.grad = grad ? 1 : 0;
  base.kappa = O.kappa;
  // The near field needs only the gathered charges; it runs on the
  // auxiliary stream, forked after the gather (g_near_fork 0), after P2M (2),
  // before M2L (1) or after it (3), and is joined before the far field.  With
  // g_near_fork 4 near and far field run as one kernel at the end.
  // (gradients always take the merged leaf kernel)
  const int near_fork = grad ? 4 : g_near_fork;
  const bool merged_leaf = near_fork == 4;
  auto fork_near = [&]() {
    HIPCHECK(hipEventRecord(aux.forked, s));
    HIPCHECK(hipStreamWaitEvent(aux.stream, aux.forked, 0));
    const hipStream_t ns = g_prof.on ? s : aux.stream;
    {
      PhaseScope ps(PH_NEAR, ns);
      P2PArgs<T> a = base;
      a.work = F.leaf_boxes;
      a.l1_off = F.u_off;
      a.l1_items = F.u_items;
      a.l2_off = F.w_off;
      a.l2_items = F.w_items;
      run_p2p_rc<T, MODE_NEAR, 32>(a, F.n_leaf, n_rhs, false, ns, ps);
    }
    HIPCHECK(hipEventRecord(aux.joined, aux.stream));
  };
  if (near_fork == 0) fork_near();
  {
    PhaseScope ps(PH_P2M, s);
    P2PArgs<T> a = base;
    a.work = F.p2m_boxes;
    a.out_col = up_chk;
    run_p2p_rc<T, MODE_P2M, 64>(a, F.n_p2m, n_rhs, false, s, ps);
  }
  if (near_fork == 2) fork_near();
  for (int l = F.depth; l >= 2; --l) {
    {
      PhaseScope ps(PH_M2M, s);
      // per-child contributions into the (not yet used) downward check
      // columns, then the per-parent sums into the upward check potentials
      run_gemm<GF, T, T>(F.m2m[l], m2m + set(l) * 8 * nn, nn, ld, F.nbox, n_rhs, up_eq, dn_chk, false, s, ps);
      const int npar = F.n_m2m_sum[l];
      if (npar > 0) {
        const int64_t upb = int64_t(n_rhs) * ld * int64_t(sizeof(T)) / 16;
        const int64_t tot = npar * upb;
        hipLaunchKernelGGL(m2m_sum_kernel<T>, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s,
                           F.m2m_sum[l], npar, upb, reinterpret_cast<const uint4*>(dn_chk),
                           reinterpret_cast<uint4*>(up_chk));
        LAUNCHCHECK("m2m_sum_kernel");
        ps.launches++;
      }
    }
    {
      PhaseScope ps(PH_UC2E, s);
      run_gemm<GM_F64, T, T>(F.uc2e[l], O.uc2e + set(l) * nn, 0, ld, F.nbox, n_rhs, up_chk, up_eq, false, s, ps);
    }
  }
  if (near_fork == 1) fork_near();
  {
    // operand of M2L: upward densities, or (check form) upward check potentials
    const T* m2l_in = check_form ? up_chk : up_eq;
    const bool split_mode = prec == KIFMM_M2L_F16X3 || prec == KIFMM_FP64_M2L_F16X3 ||
                            prec == KIFMM_M2L_BF16X3 || prec == KIFMM_M2L_BF16X5;
    if (!split_mode) {
      // M2L adds its tiles into zeroed downward check potentials with
      // atomics (two terms at most per value); P2L and L2L add afterwards.
      // (The split pass of the split modes zeroes them itself.)
      PhaseScope ps(PH_M2L_PREP, s);
      int64_t n16 = int64_t(W.col_bytes / 16);
      hipLaunchKernelGGL(zero_kernel, dim3(2048), dim3(256), 0, s, static_cast<uint4*>(W.dn_chk), n16);
      LAUNCHCHECK("zero_kernel");
      ps.launches++;
    }
    auto scale16 = [&]() {
      PhaseScope ps(PH_M2L_PREP, s);
      hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<uint4*>(W.absmax), int64_t(1));
      LAUNCHCHECK("zero_kernel");
      if constexpr (sizeof(T) == 8)
        hipLaunchKernelGGL(absmax_kernel64, dim3(512), dim3(256), 0, s,
                           reinterpret_cast<const double2*>(m2l_in), int64_t(W.col_bytes / 16), W.absmax);
      else
        hipLaunchKernelGGL(absmax_kernel, dim3(512), dim3(256), 0, s,
                           reinterpret_cast<const float4*>(m2l_in), int64_t(W.col_bytes / 16), W.absmax);
      LAUNCHCHECK("absmax_kernel");
      ps.launches += 2;
    };
    const bool f16 = prec == KIFMM_M2L_F16X3 || prec == KIFMM_FP64_M2L_F16X3;
    if (f16) scale16();
    // split modes: the operand is split into its 16-bit parts once
    auto split_in = [&](auto mode_tag, const T* in, const unsigned* amax) {
      constexpr int MODE = decltype(mode_tag)::value;
      using H = typename GT<MODE>::TA;
      PhaseScope pp(PH_M2L_PREP, s);
      const int64_t ngroups = int64_t(F.nbox + 1) * n_rhs * ld / 8;
      if (int64_t(sizeof(H)) * GT<MODE>::NB * ngroups * 8 > int64_t(W.split_bytes))
        raise(KIFMM_EINVAL, "evaluate: split operand buffer too small");
      hipLaunchKernelGGL((split_kernel<T, H, GT<MODE>::NB>), dim3(unsigned((ngroups + 255) / 256)), dim3(256), 0,
                         s, in, static_cast<H*>(W.split), ngroups, ld, amax, dn_chk);
      LAUNCHCHECK("split_kernel");
      pp.launches++;
    };
    if (f16) split_in(std::integral_constant<int, GM_H3>(), m2l_in, W.absmax);
    if constexpr (sizeof(T) == 4) {
      if (prec == KIFMM_M2L_BF16X3) split_in(std::integral_constant<int, GM_BF3>(), up_eq, nullptr);
      if (prec == KIFMM_M2L_BF16X5) split_in(std::integral_constant<int, GM_BF5>(), up_eq, nullptr);
    }
    const bool fp64_sum = O.p >= g_m2l_fp64_sum_min_p;
    // one M2L plan: the gathered tiles (adding into dn_chk with atomics), or
    // the pair tiles (storing into the pair buffer)
    auto run_m2l = [&](const DevPlan& P, T* out, PhaseScope& ps) {
      auto run_m2l_impl = [&](auto mode_tag, const void* opa, const unsigned* amax) {
        constexpr int MODE = decltype(mode_tag)::value;
        constexpr bool split = !(MODE == GM_F32 || MODE == GM_F64);
        using TIn = typename std::conditional<split, typename GT<MODE>::TA, T>::type;
        const TIn* in = split ? static_cast<const TIn*>(W.split) : reinterpret_cast<const TIn*>(m2l_in);
        constexpr int64_t parts = split ? 2 : 1;
        if (fp64_sum)
          run_gemm<MODE, TIn, T, 2>(P, opa, parts * nn, ld, F.nbox, n_rhs, in, out, false, s, ps, amax);
        else
          run_gemm<MODE, TIn, T, 1>(P, opa, parts * nn, ld, F.nbox, n_rhs, in, out, false, s, ps, amax);
      };
      const void* op32 = check_form ? static_cast<const void*>(O.m2lc32) : static_cast<const void*>(O.m2l32);
      const void* oph = check_form ? O.m2lc_h : O.m2l_h;
      if (prec == KIFMM_FP64) {
        run_gemm<GM_F64, T, T, 1>(P, O.m2l64, nn, ld, F.nbox, n_rhs, m2l_in, out, false, s, ps);
      } else if (prec == KIFMM_FP32 || prec == KIFMM_FP64_M2L_FP32) {
        run_m2l_impl(std::integral_constant<int, GM_F32>(), op32, nullptr);
      } else if (f16) {
        run_m2l_impl(std::integral_constant<int, GM_H3>(), oph, W.absmax);
      } else if constexpr (sizeof(T) == 4) {
        if (prec == KIFMM_M2L_BF16X3)
          run_m2l_impl(std::integral_constant<int, GM_BF3>(), O.m2l_b, nullptr);
        else
          run_m2l_impl(std::integral_constant<int, GM_BF5>(), O.m2l_b, nullptr);
      }
    };
    {
      PhaseScope ps(PH_M2L, s);
      run_m2l(F.m2l, dn_chk, ps);
    }
    if (F.m2l_pair.ntile > 0) {
      // sparse problems: one product per pair, then each target's sum
      PhaseScope ps(PH_M2L_PAIR, s);
      if (W.pairs == nullptr) raise(KIFMM_EINVAL, "evaluate: pair buffer missing");
      T* pairs = static_cast<T*>(W.pairs);
      run_m2l(F.m2l_pair, pairs, ps);
      const int64_t units = int64_t(n_rhs) * ld * int64_t(sizeof(T)) / 16;
      const int64_t tot = int64_t(F.n_pair_tgt) * units;
      const unsigned nblk = unsigned(std::min<int64_t>((tot + 255) / 256, 65536));
      hipLaunchKernelGGL(m2l_pair_sum_kernel<T>, dim3(nblk), dim3(256), 0, s, F.pair_tgt, F.pair_off,
                         F.pair_items, F.n_pair_tgt, units, reinterpret_cast<const uint4*>(pairs),
                         reinterpret_cast<uint4*>(dn_chk));
      LAUNCHCHECK("m2l_pair_sum_kernel");
      ps.launches++;
    }
  }
  if (near_fork == 3) fork_near();
  {
    PhaseScope ps(PH_P2L, s);
    P2PArgs<T> a = base;
    a.work = F.x_boxes;
    a.l1_off = F.x_off;
    a.l1_items = F.x_items;
    a.out_col = dn_chk;
    run_p2p_rc<T, MODE_P2L, 64>(a, F.n_x, n_rhs, false, s, ps);
  }
  // Gradients in the FP32-bulk modes: from here on the downward check
  // potentials are FP64 (M2L and P2L added into the FP32 columns above; L2L
  // runs in FP64 and adds into the FP64 copy; DC2E reads it).  Gradients of
  // the leaf stage amplify rounding noise on the check surface: a check
  // potential stored in FP32 alone moves the gradient of points near a
  // jittered surface by ~3e-6, the FP32 L2L sums by ~2e-5.
  const bool down64 = sizeof(T) == 4 && W.dn_chk64 != nullptr;
  if (down64) {
    PhaseScope ps(PH_L2L, s);
    const int64_t nv = int64_t(W.col_bytes / sizeof(T));
    hipLaunchKernelGGL(widen_kernel, dim3(2048), dim3(256), 0, s, reinterpret_cast<const float*>(dn_chk),
                       W.dn_chk64, nv);
    LAUNCHCHECK("widen_kernel");
    ps.launches++;
  }
  for (int l = 2; l <= F.depth; ++l) {
    if (l >= 3) {
      PhaseScope ps(PH_L2L, s);
      if (down64)
        run_gemm<GM_F64, T, double>(F.l2l[l], O.l2l64 + set(l) * 8 * nn, nn, ld, F.nbox, n_rhs, dn_eq,
                                    W.dn_chk64, true, s, ps);
      else
        run_gemm<GF, T, T>(F.l2l[l], l2l + set(l) * 8 * nn, nn, ld, F.nbox, n_rhs, dn_eq, dn_chk, true, s, ps);
    }
    {
      PhaseScope ps(PH_DC2E, s);
      if (down64)
        run_gemm<GM_F64, double, T>(F.dc2e[l], O.dc2e + set(l) * nn, 0, ld, F.nbox, n_rhs, W.dn_chk64, dn_eq,
                                    false, s, ps);
      else
        run_gemm<GM_F64, T, T>(F.dc2e[l], O.dc2e + set(l) * nn, 0, ld, F.nbox, n_rhs, dn_chk, dn_eq, false, s, ps);
    }
  }
  {
    // join the near field, then add the far field (L2P + M2P); or both in
    // one kernel
    if (!merged_leaf) HIPCHECK(hipStreamWaitEvent(s, aux.joined, 0));
    PhaseScope ps(PH_FAR, s);
    P2PArgs<T> a = base;
    a.work = F.leaf_boxes;
    a.l1_off = F.u_off;
    a.l1_items = F.u_items;
    a.l2_off = F.w_off;
    a.l2_items = F.w_items;
    const bool far64 = sizeof(T) == 4 && O.p >= g_far_fp64_min_p;
    if (merged_leaf) run_p2p_rc<T, MODE_LEAF, 32>(a, F.n_leaf, n_rhs, far64, s, ps);
    else run_p2p_rc<T, MODE_FAR, 32>(a, F.n_leaf, n_rhs, far64, s, ps);
  }
  {
    PhaseScope ps(PH_SCATTER, s);
    for (int k0 = 0; k0 < F.nprob; k0 += kMaxProb) {
      int nk = std::min(kMaxProb, F.nprob - k0);
      PtrPack pk{};
      for (int k = 0; k < nk; ++k) pk.p[k] = potentials[k0 + k];
      dim3 grid(unsigned((F.max_tgt_per_prob + 255) / 256), nk);
      // (gradients: 4 columns per right-hand side, potential then d/dx, d/dy, d/dz)
      hipLaunchKernelGGL((scatter_kernel<TIO>), grid, dim3(256), 0, s, pk, k0, F.tgt_off,
                         F.tgt_perm, n_rhs * (grad ? 4 : 1), F.ntgt, W.pot);
      LAUNCHCHECK("scatter_kernel");
      ps.launches++;
    }
  }
}

// Evaluations on a non-default stream are captured once into a hipGraph and
// replayed with one launch while the inputs of the capture stay the same.
static bool g_use_graphs = true;
static std::atomic<int64_t> g_graph_captures{0};  // evaluation graphs captured so far
void set_use_graphs(bool on) { g_use_graphs = on; }

void evaluate_forest(EvalState& st, const HostOps& hops, OpsCache& oc, const void* const* charges,
                     void* const* potentials, int n_rhs, bool io_fp64, kifmm_precision prec,
                     void* stream, bool grad) {
  const int dev = current_device();
  if (!st.forest || st.device != dev) {
    delete st.forest;
    st.forest = nullptr;
    st.forest = upload_forest(*st.host, hops.n);
    st.device = dev;
  }
  const bool fp64 = prec == KIFMM_FP64 || prec == KIFMM_FP64_M2L_FP32 || prec == KIFMM_FP64_M2L_F16X3;
  OpsNeed need;
  need.bulk64 = fp64;
  need.m2l64 = prec == KIFMM_FP64;
  need.m2l32 = prec == KIFMM_FP32 || prec == KIFMM_FP64_M2L_FP32;
  need.bf16 = prec == KIFMM_M2L_BF16X3 || prec == KIFMM_M2L_BF16X5;
  need.f16 = prec == KIFMM_M2L_F16X3 || prec == KIFMM_FP64_M2L_F16X3;
  // folded check form for the FP32 / FP16 M2L operands at high order
  need.check_form = (need.m2l32 || need.f16) && hops.p >= g_m2l_check_min_p && hops.kernel == 0;
  need.l2l64 = grad && !fp64;
  DevOps* O = ops_for_device(oc, hops, dev, need);
  DevForest& F = *st.forest;
  if (F.n != hops.n) raise(KIFMM_EINVAL, "evaluate: operator order differs from the cached forest");
  if ((hops.kernel != 0) != st.host->per_level)
    raise(KIFMM_EINVAL, "evaluate: the cached plans were built for another kernel");
  DevWork* W = work_for(F, fp64, n_rhs, grad);
  if (need.bf16 || need.f16) ensure_split(F, W);
  ensure_pairs(F, W);
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto launch_all = [&]() {
    if (fp64) {
      if (io_fp64) pipeline<double, double>(F, *O, *W, charges, potentials, n_rhs, prec, need.check_form, grad, s);
      else pipeline<double, float>(F, *O, *W, charges, potentials, n_rhs, prec, need.check_form, grad, s);
    } else {
      if (io_fp64) pipeline<float, double>(F, *O, *W, charges, potentials, n_rhs, prec, need.check_form, grad, s);
      else pipeline<float, float>(F, *O, *W, charges, potentials, n_rhs, prec, need.check_form, grad, s);
    }
  };
  if (!g_use_graphs || g_prof.on || s == nullptr) {
    launch_all();
    return;
  }
  // everything the captured launches depend on
  std::vector<const void*> key = {reinterpret_cast<const void*>(intptr_t(prec)),
                                  reinterpret_cast<const void*>(intptr_t(n_rhs)),
                                  reinterpret_cast<const void*>(intptr_t(io_fp64)), s,
                                  reinterpret_cast<const void*>(uintptr_t(O->generation)), W,
                                  reinterpret_cast<const void*>(intptr_t(g_far_fp64_min_p)),
                                  reinterpret_cast<const void*>(intptr_t(g_m2l_check_min_p)),
                                  reinterpret_cast<const void*>(intptr_t(g_m2l_fp64_sum_min_p)),
                                  reinterpret_cast<const void*>(intptr_t(g_near_fork)),
                                  reinterpret_cast<const void*>(intptr_t(g_m2l_wide)),
                                  reinterpret_cast<const void*>(intptr_t(g_m2l_async)),
                                  reinterpret_cast<const void*>(intptr_t(g_m2l_rows)),
                                  reinterpret_cast<const void*>(intptr_t(grad))};
  for (int k = 0; k < F.nprob; ++k) {
    key.push_back(charges[k]);
    key.push_back(potentials[k]);
  }
  if (!F.graph || F.graph_key != key) {
    if (F.graph) {
      HIPCHECK(hipGraphExecDestroy(F.graph));
      F.graph = nullptr;
    }
    hipGraph_t g = nullptr;
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      launch_all();
    } catch (...) {
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHECK(hipStreamEndCapture(s, &g));
    hipError_t ie = hipGraphInstantiate(&F.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      F.graph = nullptr;
      raise(KIFMM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    F.graph_key = key;
    ++g_graph_captures;
  }
  HIPCHECK(hipGraphLaunch(F.graph, s));
}

int64_t graph_captures() { return g_graph_captures.load(); }

// ------------------------------------------------------------------------
// allocation-free evaluation
// ------------------------------------------------------------------------

// The work buffers of kifmm_evaluate_noalloc, carved from this array on every
// call.  Every device that runs the library holds its own copy until the
// process ends; host code uses the per-device address from
// hipGetSymbolAddress, never the array's name.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, unsigned char*> g_scratch_addr;

// Device address of `scratch` on the current device (looked up once per device).
static unsigned char* scratch_address(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    raise(KIFMM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_addr[dev] = static_cast<unsigned char*>(p);
  return static_cast<unsigned char*>(p);
}

void evaluate_forest_noalloc(EvalState& st, const HostOps& hops, OpsCache& oc, const void* charges,
                             void* potentials, int n_rhs, bool io_fp64, kifmm_precision prec, void* stream) {
  const int dev = current_device();
  if (!st.forest || st.device != dev)
    raise(KIFMM_EINVAL, "evaluate_noalloc: the tree has no device state on this device (run kifmm_evaluate once)");
  if (g_prof.on) raise(KIFMM_EINVAL, "evaluate_noalloc: phase profiling is on (it creates events)");
  const bool fp64 = prec == KIFMM_FP64 || prec == KIFMM_FP64_M2L_FP32 || prec == KIFMM_FP64_M2L_F16X3;
  OpsNeed need;
  need.m2l32 = prec == KIFMM_FP32 || prec == KIFMM_FP64_M2L_FP32;
  need.bf16 = prec == KIFMM_M2L_BF16X3 || prec == KIFMM_M2L_BF16X5;
  need.f16 = prec == KIFMM_M2L_F16X3 || prec == KIFMM_FP64_M2L_F16X3;
  need.check_form = (need.m2l32 || need.f16) && hops.p >= g_m2l_check_min_p && hops.kernel == 0;
  auto it = oc.per_device.find(dev);
  DevOps* O = it == oc.per_device.end() ? nullptr : it->second;
  const bool ready =
      O && (fp64 ? (O->m2m64 && O->l2l64) : (O->m2m32 && O->l2l32)) && (prec != KIFMM_FP64 || O->m2l64) &&
      (!need.m2l32 || (need.check_form ? O->m2lc32 : O->m2l32) != nullptr) &&
      (!need.f16 || (need.check_form ? O->m2lc_h : O->m2l_h) != nullptr) && (!need.bf16 || O->m2l_b);
  if (!ready)
    raise(KIFMM_EINVAL,
          "evaluate_noalloc: the operator tables of this precision are not on this device (run kifmm_evaluate once)");
  DevForest& F = *st.forest;
  if (F.n != hops.n) raise(KIFMM_EINVAL, "evaluate_noalloc: operator order differs from the cached forest");
  if ((hops.kernel != 0) != st.host->per_level)
    raise(KIFMM_EINVAL, "evaluate_noalloc: the cached plans were built for another kernel");

  // layout: the regions that must start at zero first, then the rest
  const size_t es = fp64 ? 8 : 4;
  const size_t cols = size_t(F.nbox + 1) * n_rhs * F.ld;
  auto up256 = [](size_t b) { return (b + 255) / 256 * 256; };
  DevWork W;
  W.n_rhs = n_rhs;
  W.fp64 = fp64;
  W.col_bytes = cols * es;
  W.split_bytes = (need.bf16 || need.f16) ? cols * 3 * 2 : 0;
  W.pair_bytes = size_t(F.n_pairs) * n_rhs * F.ld * es;
  size_t off = 0;
  size_t at[8];
  const size_t sizes[8] = {W.col_bytes, W.col_bytes, W.col_bytes, W.col_bytes, W.split_bytes, 256,
                           size_t(n_rhs) * F.nsrc * es, size_t(n_rhs) * F.ntgt * 8};
  for (int k = 0; k < 8; ++k) {
    at[k] = off;
    off += up256(sizes[k]);
  }
  const size_t zero_bytes = at[6];  // four column buffers, split operand, absmax word
  const size_t pairs_at = off;
  off += up256(W.pair_bytes);
  if (off > kNoAllocScratchBytes)
    raise(KIFMM_EUNSUPPORTED, "evaluate_noalloc: this evaluation needs " + std::to_string(off >> 20) +
                                  " MiB of work buffers; the allocation-free entry point holds " +
                                  std::to_string(kNoAllocScratchBytes >> 20) + " MiB");
  unsigned char* base = scratch_address(dev);
  W.up_chk = base + at[0];
  W.up_eq = base + at[1];
  W.dn_chk = base + at[2];
  W.dn_eq = base + at[3];
  W.split = W.split_bytes ? base + at[4] : nullptr;
  W.absmax = reinterpret_cast<unsigned*>(base + at[5]);
  W.qs = base + at[6];
  W.pot = reinterpret_cast<double*>(base + at[7]);
  W.pairs = W.pair_bytes ? base + pairs_at : nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the array keeps the previous call's values: padding rows and the zero
  // box's columns must read zero (a fill kernel, not a memset, so that a
  // caller can capture the call into a graph)
  hipLaunchKernelGGL(zero_kernel, dim3(2048), dim3(256), 0, s, reinterpret_cast<uint4*>(base),
                     int64_t(zero_bytes / 16));
  LAUNCHCHECK("zero_kernel");
  const void* q[1] = {charges};
  void* o[1] = {potentials};
  if (fp64) {
    if (io_fp64) pipeline<double, double>(F, *O, W, q, o, n_rhs, prec, need.check_form, false, s);
    else pipeline<double, float>(F, *O, W, q, o, n_rhs, prec, need.check_form, false, s);
  } else {
    if (io_fp64) pipeline<float, double>(F, *O, W, q, o, n_rhs, prec, need.check_form, false, s);
    else pipeline<float, float>(F, *O, W, q, o, n_rhs, prec, need.check_form, false, s);
  }
}

void debug_buffer(EvalState& st, int which, bool fp64, int n_rhs, double* out, int64_t n_out) {
  if (!st.forest) raise(KIFMM_EINVAL, "debug_buffer: no evaluation has run on this tree");
  DevForest& F = *st.forest;
  auto it = F.work.find({fp64 ? 1 : 0, n_rhs});
  if (it == F.work.end()) raise(KIFMM_EINVAL, "debug_buffer: no evaluation with this precision and n_rhs");
  DevWork& W = *it->second;
  HIPCHECK(hipDeviceSynchronize());
  const size_t es = fp64 ? 8 : 4;
  if (which == 4) {
    size_t cnt = size_t(n_rhs) * F.ntgt;
    if (n_out < int64_t(cnt)) raise(KIFMM_EINVAL, "debug_buffer: output too small");
    HIPCHECK(hipMemcpy(out, W.pot, cnt * 8, hipMemcpyDeviceToHost));
    return;
  }
  void* src = which == 0 ? W.up_chk : which == 1 ? W.up_eq : which == 2 ? W.dn_chk : which == 3 ? W.dn_eq : nullptr;
  if (!src) raise(KIFMM_EINVAL, "debug_buffer: which must be 0..4");
  const size_t cols = size_t(F.nbox) * n_rhs;
  if (n_out < int64_t(cols * F.n)) raise(KIFMM_EINVAL, "debug_buffer: output too small");
  std::vector<unsigned char> h(cols * F.ld * es);
  HIPCHECK(hipMemcpy(h.data(), src, h.size(), hipMemcpyDeviceToHost));
  for (size_t c = 0; c < cols; ++c)
    for (int k = 0; k < F.n; ++k) {
      size_t i = c * F.ld + k;
      out[c * F.n + k] = fp64 ? reinterpret_cast<double*>(h.data())[i] : double(reinterpret_cast<float*>(h.data())[i]);
    }
}

void evaluate_simple_host(EvalState& st, const HostOps& hops, OpsCache& oc, const double* q,
                          int64_t nsrc, double* pot, int64_t ntgt) {
  std::vector<void*> bufs;
  struct Free {
    std::vector<void*>& b;
    ~Free() {
      for (void* p : b) (void)hipFree(p);
    }
  } fr{bufs};
  double* dq = dev_alloc<double>(bufs, size_t(nsrc));
  double* dp = dev_alloc<double>(bufs, size_t(ntgt));
  HIPCHECK(hipMemcpy(dq, q, size_t(nsrc) * 8, hipMemcpyHostToDevice));
  const void* qa[1] = {dq};
  void* pa[1] = {dp};
  evaluate_forest(st, hops, oc, qa, pa, 1, true, KIFMM_FP32, nullptr, false);
  HIPCHECK(hipStreamSynchronize(nullptr));
  HIPCHECK(hipMemcpy(pot, dp, size_t(ntgt) * 8, hipMemcpyDeviceToHost));
}

}  // namespace kifmm
