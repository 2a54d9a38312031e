// FP64 operator precomputation: surfaces, one-sided Jacobi SVD, truncated
// pseudo-inverses and the translation operator tables on a reference box.
#include "precompute.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

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
static void kernel_block(const std::vector<double>& s, int n, const double xs[3], double xr,
                         const double ys[3], double yr, double* out) {
  for (int i = 0; i < n; ++i) {
    double x0 = xs[0] + xr * s[3 * i], x1 = xs[1] + xr * s[3 * i + 1], x2 = xs[2] + xr * s[3 * i + 2];
    for (int j = 0; j < n; ++j) {
      double d0 = x0 - (ys[0] + yr * s[3 * j]);
      double d1 = x1 - (ys[1] + yr * s[3 * j + 1]);
      double d2 = x2 - (ys[2] + yr * s[3 * j + 2]);
      out[size_t(i) * n + j] = kInv4Pi / std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
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

std::vector<double> m2l_check_form(const HostOps& O) {
  const int n = O.n;
  const size_t nn = size_t(n) * n;
  std::vector<double> out(size_t(kNumM2L) * nn, 0.0);
  parallel_for(kNumM2L, [&](int64_t b, int64_t e) {
    for (int64_t k = b; k < e; ++k) {
      const double* A = &O.m2l[size_t(k) * nn];
      double* C = &out[size_t(k) * nn];
      for (int i = 0; i < n; ++i)
        for (int l = 0; l < n; ++l) {
          const double a = A[size_t(i) * n + l];
          const double* Br = &O.uc2e[size_t(l) * n];
          double* Cr = &C[size_t(i) * n];
          for (int j = 0; j < n; ++j) Cr[j] += a * Br[j];
        }
    }
  }, 1);
  return out;
}

HostOps* build_host_ops(int p, double rcond) {
  if (p < 2 || p > 16) raise(KIFMM_EINVAL, "precompute_operators: p must be in [2, 16]");
  if (!(rcond > 0.0 && rcond < 1.0)) raise(KIFMM_EINVAL, "precompute_operators: rcond must be in (0, 1)");
  auto* O = new HostOps();
  try {
    O->p = p;
    O->rcond = rcond;
    O->surf = surface_points(p);
    const int n = O->n = static_cast<int>(O->surf.size() / 3);
    const size_t nn = size_t(n) * n;
    const double zero[3] = {0, 0, 0};
    std::vector<double> k(nn);
    // UC2E: upward check (outer) <- upward equivalent (inner)
    kernel_block(O->surf, n, zero, kRadiusOuter, zero, kRadiusInner, k.data());
    O->uc2e = pinv_truncated(k.data(), n, rcond);
    // DC2E: downward check (inner) <- downward equivalent (outer)
    kernel_block(O->surf, n, zero, kRadiusInner, zero, kRadiusOuter, k.data());
    O->dc2e = pinv_truncated(k.data(), n, rcond);
    O->m2m.resize(8 * nn);
    O->l2l.resize(8 * nn);
    for (int o = 0; o < 8; ++o) {
      // child centre relative to the parent, in parent half-widths: +-1/2
      double sh[3] = {(((o >> 2) & 1) ? 0.5 : -0.5), (((o >> 1) & 1) ? 0.5 : -0.5),
                      ((o & 1) ? 0.5 : -0.5)};
      kernel_block(O->surf, n, zero, kRadiusOuter, sh, 0.5 * kRadiusInner, &O->m2m[o * nn]);
      // parent centre relative to the child, in child half-widths: -+1
      double ps[3] = {-2 * sh[0], -2 * sh[1], -2 * sh[2]};
      kernel_block(O->surf, n, zero, kRadiusInner, ps, 2.0 * kRadiusOuter, &O->l2l[o * nn]);
    }
    std::fill(std::begin(O->m2l_index), std::end(O->m2l_index), -1);
    O->m2l.resize(size_t(kNumM2L) * nn);
    int idx = 0;
    for (int dx = -3; dx <= 3; ++dx)
      for (int dy = -3; dy <= 3; ++dy)
        for (int dz = -3; dz <= 3; ++dz) {
          if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
          O->m2l_offset.push_back(dx);
          O->m2l_offset.push_back(dy);
          O->m2l_offset.push_back(dz);
          O->m2l_index[(dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)] = idx;
          double sh[3] = {2.0 * dx, 2.0 * dy, 2.0 * dz};
          kernel_block(O->surf, n, zero, kRadiusInner, sh, kRadiusInner, &O->m2l[size_t(idx) * nn]);
          ++idx;
        }
  } catch (...) {
    delete O;
    throw;
  }
  return O;
}

}  // namespace kifmm
