// FP64 operator precomputation: surfaces, one-sided Jacobi SVD, truncated
// pseudo-inverses and the translation operator tables on a reference box.
#include "precompute.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>

#include "common.hpp"

namespace kifmm {

static constexpr double kInv4Pi = 0.0795774715459476678844418816863;  // 1/(4 pi)

// Points of the p x p x p lattice {-1 + 2i/(p-1)}^3 on the boundary of [-1,1]^3:
// p^3 - (p-2)^3 = 6(p-1)^2 + 2 of them (the count n_e given in the paper).
static std::vector<double> surface_points(int p) {
  std::vector<double> g(p);
  for (int i = 0; i < p; ++i) g[i] = -1.0 + 2.0 * double(i) / double(p - 1);
  g[0] = -1.0;
  g[p - 1] = 1.0;
  std::vector<double> s;
  for (int a = 0; a < p; ++a)
    for (int b = 0; b < p; ++b)
      for (int c = 0; c < p; ++c)
        if (a == 0 || a == p - 1 || b == 0 || b == p - 1 || c == 0 || c == p - 1) {
          s.push_back(g[a]);
          s.push_back(g[b]);
          s.push_back(g[c]);
        }
  return s;
}

// K[i][j] = 1/(4 pi |x_i - y_j|) for x_i = xs + xr * s_i, y_j = ys + yr * s_j.
// out[i][j] = G(x_i, y_j), x_i = xs + xr s_i, y_j = ys + yr s_j, for the
// Laplace kernel 1 / (4 pi d) (lambda = 0) or the screened kernel
// exp(-lambda d) / (4 pi d) in box units (lambda = kappa times the box size).
static void kernel_block(const std::vector<double>& s, int n, const double xs[3], double xr,
                         const double ys[3], double yr, double* out, double lambda = 0.0) {
  for (int i = 0; i < n; ++i) {
    double x0 = xs[0] + xr * s[3 * i], x1 = xs[1] + xr * s[3 * i + 1], x2 = xs[2] + xr * s[3 * i + 2];
    for (int j = 0; j < n; ++j) {
      double d0 = x0 - (ys[0] + yr * s[3 * j]);
      double d1 = x1 - (ys[1] + yr * s[3 * j + 1]);
      double d2 = x2 - (ys[2] + yr * s[3 * j + 2]);
      const double d = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      out[size_t(i) * n + j] = lambda == 0.0 ? kInv4Pi / d : kInv4Pi * std::exp(-lambda * d) / d;
    }
  }
}

void jacobi_svd(const double* a, int n, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& V) {
  // Column-major working copies: W holds the columns of a, Q accumulates V.
  std::vector<double> W(size_t(n) * n), Q(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) W[size_t(j) * n + i] = a[size_t(i) * n + j];
  for (int j = 0; j < n; ++j) Q[size_t(j) * n + j] = 1.0;
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
    int64_t rotations = 0;
    for (int i = 0; i < n - 1; ++i) {
      double* wi = &W[size_t(i) * n];
      double* qi = &Q[size_t(i) * n];
      for (int j = i + 1; j < n; ++j) {
        double* wj = &W[size_t(j) * n];
        double al = 0, be = 0, ga = 0;
        for (int k = 0; k < n; ++k) {
          al += wi[k] * wi[k];
          be += wj[k] * wj[k];
          ga += wi[k] * wj[k];
        }
        if (ga == 0.0 || std::fabs(ga) <= tol * std::sqrt(al * be)) continue;
        ++rotations;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int k = 0; k < n; ++k) {
          double x = wi[k], y = wj[k];
          wi[k] = c * x - sn * y;
          wj[k] = sn * x + c * y;
        }
        double* qj = &Q[size_t(j) * n];
        for (int k = 0; k < n; ++k) {
          double x = qi[k], y = qj[k];
          qi[k] = c * x - sn * y;
          qj[k] = sn * x + c * y;
        }
      }
    }
    if (rotations == 0) break;
  }
  std::vector<double> nrm(n);
  for (int j = 0; j < n; ++j) {
    double acc = 0;
    for (int k = 0; k < n; ++k) acc += W[size_t(j) * n + k] * W[size_t(j) * n + k];
    nrm[j] = std::sqrt(acc);
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
  U.assign(size_t(n) * n, 0.0);
  V.assign(size_t(n) * n, 0.0);
  s.assign(n, 0.0);
  for (int c = 0; c < n; ++c) {
    int j = ord[c];
    s[c] = nrm[j];
    for (int k = 0; k < n; ++k) {
      U[size_t(k) * n + c] = nrm[j] > 0 ? W[size_t(j) * n + k] / nrm[j] : 0.0;
      V[size_t(k) * n + c] = Q[size_t(j) * n + k];
    }
  }
}

std::vector<double> pinv_truncated(const double* a, int n, double rcond, int* rank) {
  std::vector<double> U, s, V;
  jacobi_svd(a, n, U, s, V);
  int r = 0;
  while (r < n && s[r] > 0 && s[r] >= rcond * s[0]) ++r;
  if (rank) *rank = r;
  std::vector<double> P(size_t(n) * n, 0.0);
  // P = V_r diag(1/s_r) U_r^T
  parallel_for(n, [&](int64_t b, int64_t e) {
    std::vector<double> row(r);
    for (int64_t i = b; i < e; ++i) {
      for (int k = 0; k < r; ++k) row[k] = V[size_t(i) * n + k] / s[k];
      for (int j = 0; j < n; ++j) {
        double acc = 0;
        for (int k = 0; k < r; ++k) acc += row[k] * U[size_t(j) * n + k];
        P[size_t(i) * n + j] = acc;
      }
    }
  }, 8);
  return P;
}

HostOps* build_host_ops(int p, double rcond, bool device_svd, double kappa, double r0, int max_level) {
  if (p < 2 || p > 16) raise(KIFMM_EINVAL, "precompute_operators: p must be in [2, 16]");
  if (!(rcond > 0.0 && rcond < 1.0)) raise(KIFMM_EINVAL, "precompute_operators: rcond must be in (0, 1)");
  const bool screened = kappa != 0.0;
  if (screened) {
    if (!(kappa > 0.0) || !std::isfinite(kappa)) raise(KIFMM_EINVAL, "precompute_operators: kappa must be > 0");
    if (!(r0 > 0.0) || !std::isfinite(r0)) raise(KIFMM_EINVAL, "precompute_operators: root half-width must be > 0");
    if (max_level < 2 || max_level > 20) raise(KIFMM_EINVAL, "precompute_operators: max_level must be in [2, 20]");
  }
  alloc_hook("precompute_operators");
  auto* O = new HostOps();
  try {
    O->p = p;
    O->rcond = rcond;
    O->device_svd = device_svd;
    O->kernel = screened ? 1 : 0;
    O->kappa = kappa;
    O->r0 = screened ? r0 : 0.0;
    O->levels = screened ? max_level + 1 : 1;
    O->surf = surface_points(p);
    const int n = O->n = static_cast<int>(O->surf.size() / 3);
    const size_t nn = size_t(n) * n;
    const int L = O->levels;
    const double zero[3] = {0, 0, 0};
    std::vector<double> k(nn);
    auto pinv = [&](const double* a) {
      return device_svd ? pinv_truncated_device(a, n, rcond) : pinv_truncated(a, n, rcond);
    };
    O->uc2e.assign(L * nn, 0.0);
    O->dc2e.assign(L * nn, 0.0);
    O->m2m.assign(8 * L * nn, 0.0);
    O->l2l.assign(8 * L * nn, 0.0);
    O->m2l.assign(size_t(kNumM2L) * L * nn, 0.0);
    std::fill(std::begin(O->m2l_index), std::end(O->m2l_index), -1);
    for (int dx = -3; dx <= 3; ++dx)
      for (int dy = -3; dy <= 3; ++dy)
        for (int dz = -3; dz <= 3; ++dz) {
          if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
          O->m2l_index[(dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)] = int32_t(O->m2l_offset.size() / 3);
          O->m2l_offset.push_back(dx);
          O->m2l_offset.push_back(dy);
          O->m2l_offset.push_back(dz);
        }
    // Table set t: one set for the Laplace kernel (level independent with
    // scaled check potentials); for the screened kernel one per level l >= 2,
    // with lambda = kappa r_l in the level's box units (levels 0, 1 unused).
    for (int t = screened ? 2 : 0; t < L; ++t) {
      const double lam = screened ? kappa * (r0 / double(int64_t(1) << t)) : 0.0;
      // UC2E: upward check (outer) <- upward equivalent (inner)
      kernel_block(O->surf, n, zero, kRadiusOuter, zero, kRadiusInner, k.data(), lam);
      std::vector<double> u = pinv(k.data());
      std::copy(u.begin(), u.end(), O->uc2e.begin() + t * nn);
      // DC2E: downward check (inner) <- downward equivalent (outer)
      kernel_block(O->surf, n, zero, kRadiusInner, zero, kRadiusOuter, k.data(), lam);
      u = pinv(k.data());
      std::copy(u.begin(), u.end(), O->dc2e.begin() + t * nn);
      for (int o = 0; o < 8; ++o) {
        // M2M in the parent's units (parent at level t), L2L in the child's
        // (child at level t): child centre relative to the parent +-1/2
        double sh[3] = {(((o >> 2) & 1) ? 0.5 : -0.5), (((o >> 1) & 1) ? 0.5 : -0.5),
                        ((o & 1) ? 0.5 : -0.5)};
        kernel_block(O->surf, n, zero, kRadiusOuter, sh, 0.5 * kRadiusInner, &O->m2m[(size_t(t) * 8 + o) * nn], lam);
        // parent centre relative to the child, in child half-widths: -+1
        double ps[3] = {-2 * sh[0], -2 * sh[1], -2 * sh[2]};
        kernel_block(O->surf, n, zero, kRadiusInner, ps, 2.0 * kRadiusOuter, &O->l2l[(size_t(t) * 8 + o) * nn], lam);
      }
      for (int idx = 0; idx < kNumM2L; ++idx) {
        const int32_t* d = &O->m2l_offset[3 * size_t(idx)];
        double sh[3] = {2.0 * d[0], 2.0 * d[1], 2.0 * d[2]};
        kernel_block(O->surf, n, zero, kRadiusInner, sh, kRadiusInner,
                     &O->m2l[(size_t(t) * kNumM2L + idx) * nn], lam);
      }
    }
  } catch (...) {
    delete O;
    throw;
  }
  return O;
}

// --- persistent cache ------------------------------------------------------
// Layout (little-endian): "KIFMMOPS", u32 version, i32 p, i32 n, f64 rcond,
// f64 inner radius, f64 outer radius, i32 number of M2L offsets, u32 flags
// (bit 0: GPU SVD), then surf, uc2e, dc2e, m2m, l2l, m2l (f64), m2l_offset
// and m2l_index (i32), then the FNV-1a 64 hash of all preceding bytes.
namespace {

constexpr char kMagic[8] = {'K', 'I', 'F', 'M', 'M', 'O', 'P', 'S'};
constexpr uint32_t kVersion = 1;

struct Fnv {
  uint64_t h = 1469598103934665603ULL;
  void add(const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ULL;
    }
  }
};

}  // namespace

void save_host_ops(const HostOps& O, const char* path) {
  if (!path) raise(KIFMM_EINVAL, "ops_save: null path");
  if (O.kernel != 0) raise(KIFMM_EUNSUPPORTED, "ops_save: the cache holds Laplace-kernel operators only");
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) raise(KIFMM_EINVAL, std::string("ops_save: cannot write ") + tmp);
  Fnv h;
  bool ok = true;
  auto put = [&](const void* p, size_t n) {
    if (n == 0) return;
    h.add(p, n);
    ok = ok && std::fwrite(p, 1, n, f) == n;
  };
  const uint32_t version = kVersion, flags = O.device_svd ? 1u : 0u;
  const int32_t p = O.p, n = O.n, nm2l = kNumM2L;
  const double rin = kRadiusInner, rout = kRadiusOuter;
  put(kMagic, 8);
  put(&version, 4);
  put(&p, 4);
  put(&n, 4);
  put(&O.rcond, 8);
  put(&rin, 8);
  put(&rout, 8);
  put(&nm2l, 4);
  put(&flags, 4);
  for (const std::vector<double>* v : {&O.surf, &O.uc2e, &O.dc2e, &O.m2m, &O.l2l, &O.m2l})
    put(v->data(), v->size() * 8);
  put(O.m2l_offset.data(), O.m2l_offset.size() * 4);
  put(O.m2l_index, sizeof(O.m2l_index));
  const uint64_t sum = h.h;
  ok = ok && std::fwrite(&sum, 1, 8, f) == 8;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    raise(KIFMM_EINVAL, std::string("ops_save: writing ") + path + " failed");
  }
}

HostOps* load_host_ops(const char* path, int p, double rcond) {
  if (!path) raise(KIFMM_EINVAL, "ops_load: null path");
  alloc_hook("ops_load");
  FILE* f = std::fopen(path, "rb");
  if (!f) raise(KIFMM_EINVAL, std::string("ops_load: cannot read ") + path);
  std::unique_ptr<HostOps> O(new HostOps());
  Fnv h;
  bool ok = true;
  auto get = [&](void* q, size_t n) {
    if (n == 0 || !ok) return;
    ok = std::fread(q, 1, n, f) == n;
    if (ok) h.add(q, n);
  };
  auto bad = [&](const std::string& why) {
    std::fclose(f);
    raise(KIFMM_EINVAL, std::string("ops_load: ") + path + ": " + why);
  };
  char magic[8];
  uint32_t version = 0, flags = 0;
  int32_t fp = 0, fn = 0, nm2l = 0;
  double frcond = 0, rin = 0, rout = 0;
  get(magic, 8);
  if (!ok || std::memcmp(magic, kMagic, 8) != 0) bad("not an operator cache file");
  get(&version, 4);
  if (!ok || version != kVersion) bad("unknown format version");
  get(&fp, 4);
  get(&fn, 4);
  get(&frcond, 8);
  get(&rin, 8);
  get(&rout, 8);
  get(&nm2l, 4);
  get(&flags, 4);
  if (!ok) bad("truncated header");
  if (fp != p || frcond != rcond || rin != kRadiusInner || rout != kRadiusOuter || nm2l != kNumM2L)
    bad("holds operators of another key (p, rcond or surface radii)");
  const int n = p * p * p - (p - 2) * (p - 2) * (p - 2);
  if (fn != n) bad("surface size does not match p");
  O->p = p;
  O->n = n;
  O->rcond = rcond;
  O->device_svd = (flags & 1u) != 0;
  const size_t nn = size_t(n) * n;
  O->surf.resize(3 * size_t(n));
  O->uc2e.resize(nn);
  O->dc2e.resize(nn);
  O->m2m.resize(8 * nn);
  O->l2l.resize(8 * nn);
  O->m2l.resize(size_t(kNumM2L) * nn);
  O->m2l_offset.resize(3 * size_t(kNumM2L));
  for (std::vector<double>* v : {&O->surf, &O->uc2e, &O->dc2e, &O->m2m, &O->l2l, &O->m2l})
    get(v->data(), v->size() * 8);
  get(O->m2l_offset.data(), O->m2l_offset.size() * 4);
  get(O->m2l_index, sizeof(O->m2l_index));
  uint64_t sum = 0;
  const uint64_t want = h.h;
  if (ok) ok = std::fread(&sum, 1, 8, f) == 8;
  if (!ok) bad("truncated");
  char extra;
  if (std::fread(&extra, 1, 1, f) != 0) bad("trailing bytes");
  if (sum != want) bad("checksum mismatch (damaged file)");
  std::fclose(f);
  return O.release();
}

}  // namespace kifmm
