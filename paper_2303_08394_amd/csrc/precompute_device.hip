// The check-to-equivalent pseudo-inverses of the operator precomputation on
// the GPU (section "Computational structure of FMM operators": the upward and
// downward solves; the regularised pseudo-inverse drops singular values below
// rcond * sigma_max, as the host path does).  The SVD is rocSOLVER's (FP64,
// bidiagonalisation + QR iteration); the truncated product V S^+ U^T is one
// small kernel.  A different SVD algorithm from the host's one-sided Jacobi,
// so the two pseudo-inverses agree to the conditioning of the kept part
// (~1e-9 relative at rcond = 1e-9), not bitwise.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <string>
#include <vector>

#include "hip_check.hpp"
#include "precompute.hpp"

namespace kifmm {
namespace {

// P = V S^+ U^T for the column-major SVD M = U diag(s) V^T (vt holds V^T):
// P[i + j n] = sum_k vt[k + i n] inv(s_k) u[j + k n], inv(s) = 1/s for kept
// values, 0 for dropped ones.
__global__ void pinv_product_kernel(const double* __restrict__ u, const double* __restrict__ s,
                                    const double* __restrict__ vt, int n, double cut, double* __restrict__ p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) {
    const double sk = s[k];
    if (sk >= cut) acc += vt[k + int64_t(i) * n] * (u[j + int64_t(k) * n] / sk);
  }
  p[i + int64_t(j) * n] = acc;
}

void rbcheck(rocblas_status st, const char* what) {
  if (st != rocblas_status_success)
    raise(KIFMM_EDEVICE, std::string(what) + ": rocBLAS/rocSOLVER status " + std::to_string(int(st)));
}

}  // namespace

std::vector<double> pinv_truncated_device(const double* a, int n, double rcond, int* rank) {
  // a is row-major, i.e. the column-major buffer of M = a^T; the column-major
  // buffer of pinv(M) is the row-major buffer of pinv(a) = pinv(M)^T.
  const size_t nn = size_t(n) * n;
  std::vector<void*> bufs;
  struct Free {
    std::vector<void*>& b;
    rocblas_handle h = nullptr;
    ~Free() {
      if (h) rocblas_destroy_handle(h);
      for (void* p : b) (void)hipFree(p);
    }
  } guard{bufs};
  auto alloc = [&](size_t bytes) {
    alloc_hook("precompute (device)");
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) raise(KIFMM_ENOMEM, std::string("precompute (device): hipMalloc: ") + hipGetErrorString(e));
    bufs.push_back(p);
    return static_cast<double*>(p);
  };
  double* dA = alloc(nn * 8);
  double* dU = alloc(nn * 8);
  double* dV = alloc(nn * 8);
  double* dS = alloc(size_t(n) * 8);
  double* dE = alloc(size_t(n) * 8);
  double* dP = alloc(nn * 8);
  rocblas_int* dinfo = static_cast<rocblas_int*>(static_cast<void*>(alloc(8)));
  HIPCHECK(hipMemcpy(dA, a, nn * 8, hipMemcpyHostToDevice));
  rbcheck(rocblas_create_handle(&guard.h), "rocblas_create_handle");
  rbcheck(rocsolver_dgesvd(guard.h, rocblas_svect_all, rocblas_svect_all, n, n, dA, n, dS, dU, n, dV, n, dE,
                           rocblas_outofplace, dinfo),
          "rocsolver_dgesvd");
  HIPCHECK(hipDeviceSynchronize());
  rocblas_int info = 0;
  std::vector<double> s(n);
  HIPCHECK(hipMemcpy(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(s.data(), dS, size_t(n) * 8, hipMemcpyDeviceToHost));
  if (info != 0) raise(KIFMM_EDEVICE, "rocsolver_dgesvd did not converge");
  const double cut = rcond * s[0];
  if (rank) {
    int r = 0;
    for (double v : s) r += v >= cut ? 1 : 0;
    *rank = r;
  }
  hipLaunchKernelGGL(pinv_product_kernel, dim3(unsigned((n + 127) / 128), unsigned(n)), dim3(128), 0, 0, dU, dS,
                     dV, n, cut, dP);
  LAUNCHCHECK("pinv_product_kernel");
  std::vector<double> out(nn);
  HIPCHECK(hipMemcpy(out.data(), dP, nn * 8, hipMemcpyDeviceToHost));
  return out;
}

// The M2L check form on the GPU: the 316 products M2L_o * UC2E (row-major n x n,
// FP64) as one strided-batched rocBLAS DGEMM.  In column-major terms the
// row-major product C = A B is C^T = B^T A^T, i.e. gemm(B, A) on the same
// buffers.
std::vector<double> m2l_check_form_device(const HostOps& O) {
  const int n = O.n;
  const size_t nn = size_t(n) * n;
  std::vector<void*> bufs;
  struct Free {
    std::vector<void*>& b;
    rocblas_handle h = nullptr;
    ~Free() {
      if (h) rocblas_destroy_handle(h);
      for (void* p : b) (void)hipFree(p);
    }
  } guard{bufs};
  auto alloc = [&](size_t bytes) {
    alloc_hook("precompute (device)");
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) raise(KIFMM_ENOMEM, std::string("precompute (device): hipMalloc: ") + hipGetErrorString(e));
    bufs.push_back(p);
    return static_cast<double*>(p);
  };
  double* dA = alloc(size_t(kNumM2L) * nn * 8);
  double* dB = alloc(nn * 8);
  double* dC = alloc(size_t(kNumM2L) * nn * 8);
  HIPCHECK(hipMemcpy(dA, O.m2l.data(), size_t(kNumM2L) * nn * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(dB, O.uc2e.data(), nn * 8, hipMemcpyHostToDevice));
  rbcheck(rocblas_create_handle(&guard.h), "rocblas_create_handle");
  const double one = 1.0, zero = 0.0;
  rbcheck(rocblas_dgemm_strided_batched(guard.h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, dB,
                                        n, 0, dA, n, rocblas_stride(nn), &zero, dC, n, rocblas_stride(nn),
                                        kNumM2L),
          "rocblas_dgemm_strided_batched");
  std::vector<double> out(size_t(kNumM2L) * nn);
  HIPCHECK(hipMemcpy(out.data(), dC, out.size() * 8, hipMemcpyDeviceToHost));
  return out;
}

}  // namespace kifmm
