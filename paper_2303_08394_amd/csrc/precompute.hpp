// Operator precomputation on the host in FP64 (section "Computational
// structure of FMM operators": surfaces of n_e = 6(p-1)^2 + 2 points and
// check-to-equivalent solves; section "Parallelization strategies for FMM
// operators": M2M/L2L precomputed once and scaled per level).
#pragma once

#include <cstdint>
#include <vector>

namespace kifmm {

constexpr double kRadiusInner = 1.05;  // upward equivalent / downward check
constexpr double kRadiusOuter = 2.95;  // upward check / downward equivalent
constexpr int kNumM2L = 316;           // offsets in {-3..3}^3 minus {-1..1}^3

struct HostOps {
  int p = 0, n = 0;
  double rcond = 0;
  std::vector<double> surf;  // [n][3] unit-cube surface points
  // Reference operators (box half-width 1), row-major [rows][cols]:
  //   uc2e, dc2e  [n][n]    scaled check potential -> density
  //   m2m [8][n][n]         child density -> parent scaled check (parent r = 1)
  //   l2l [8][n][n]         parent density -> child scaled check (child r = 1)
  //   m2l [316][n][n]       source density -> target scaled check (same level)
  // A "scaled" check potential is r times the check potential of a box of
  // half-width r; with it every translation is independent of the level,
  // because the kernel is homogeneous of degree -1 and pinv(K / r) = r pinv(K).
  std::vector<double> uc2e, dc2e, m2m, l2l, m2l;
  std::vector<int32_t> m2l_offset;  // [316][3] source anchor - target anchor
  int32_t m2l_index[343];           // (dx+3)*49 + (dy+3)*7 + (dz+3) -> op, or -1
  bool device_svd = false;          // pseudo-inverses from the GPU SVD
  // Kernel: 0 Laplace (one table set); 1 screened, exp(-kappa d) / (4 pi d):
  // not homogeneous, so one table set per level l (index l, stacked in every
  // table above: uc2e [levels][n][n], m2m [levels][8][n][n], m2l
  // [levels][316][n][n]), for boxes of half-width r0 / 2^l; sets 0 and 1 are
  // zero (unused).
  int kernel = 0;
  double kappa = 0.0, r0 = 0.0;
  int levels = 1;
};

// device_svd: the two pseudo-inverses on the GPU (pinv_truncated_device);
// everything else on the host.  kappa > 0: the screened kernel, tables for
// levels 2..max_level of a tree whose root half-width is r0.
HostOps* build_host_ops(int p, double rcond, bool device_svd = false, double kappa = 0.0, double r0 = 0.0,
                        int max_level = 0);

// Persistent operator cache: a binary file holding every table of a HostOps
// with its key (p, rcond, the surface radii) and an FNV-1a checksum.
// save throws Error(EINVAL) if the file cannot be written; load throws
// Error(EINVAL) if it cannot be read, is not such a file, is damaged, or holds
// operators of another key.
void save_host_ops(const HostOps& ops, const char* path);
HostOps* load_host_ops(const char* path, int p, double rcond);

// M2L folded with the upward solve: m2l[o] * uc2e for every offset, FP64,
// [316][n][n], on the current GPU (one batched FP64 GEMM).  Maps a source
// box's scaled upward check potential straight to the target's scaled
// downward check potential.
std::vector<double> m2l_check_form_device(const HostOps& ops);

// pinv_truncated on the GPU: rocSOLVER SVD, truncated product in one kernel.
std::vector<double> pinv_truncated_device(const double* a, int n, double rcond, int* rank = nullptr);


// One-sided Jacobi SVD of the square row-major matrix a [n][n]:
// a = U diag(s) V^T; outputs U, V row-major [n][n], s descending.
void jacobi_svd(const double* a, int n, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& V);

// Pseudo-inverse of a [n][n] from the SVD, dropping s_i < rcond * s_max.
std::vector<double> pinv_truncated(const double* a, int n, double rcond, int* rank = nullptr);

}  // namespace kifmm
