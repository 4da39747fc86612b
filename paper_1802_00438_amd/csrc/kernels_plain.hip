// kernels_plain.hip -- one-step-per-launch kernels, fill kernels and the launch dispatch.
#include "launch.hpp"

// Fill kernel used instead of hipMemsetAsync (clears memory inside captured graphs too).
__global__ void fill_kernel(float* p, size_t n, float v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}
__global__ void fill_int_kernel(int* p, size_t n, int v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}


namespace {
const int kK2D[] = {4, 8, 12, 16, 20, 24};
const int kK2H[] = {4, 8, 12, 16};
const int kK2A[] = {4, 8, 12};
const int kK3D[] = {1, 2, 3, 4, 5, 6};
const int kK3H[] = {1, 2, 3, 4};
const int kK3A[] = {1, 2, 3, 4};
}  // namespace

int tb_instantiated(int ndim, KMode m, const int** ks) {
  if (ndim == 2) {
    if (m == KM_DIFF) { *ks = kK2D; return 6; }
    if (m == KM_HOT || m == KM_PHYS) { *ks = kK2H; return 4; }
    *ks = kK2A; return 3;  // transposed steps
  }
  if (m == KM_DIFF) { *ks = kK3D; return 6; }
  if (m == KM_HOT) { *ks = kK3H; return 4; }
  *ks = kK3A; return 4;
}

int tb_max_k(int ndim, KMode m) {
  const int* ks;
  const int n = tb_instantiated(ndim, m, &ks);
  return ks[n - 1];
}

hipError_t launch_tb2d(int K, KMode m, bool full, const Tb2dArgs& a, hipStream_t s) {
  switch (m) {
    case KM_DIFF: return launch_tb2d_diff(K, full, a, s);
    case KM_HOT: return launch_tb2d_hot(K, full, a, s);
    case KM_ADJ: return launch_tb2d_adj(K, false, full, a, s);
    case KM_ADJ_ACC: return launch_tb2d_adj(K, true, full, a, s);
    case KM_PHYS: return launch_tb2d_phys(K, full, a, s);
    case KM_PHYS_ADJ: return launch_tb2d_phys_adj(K, false, full, a, s);
    case KM_PHYS_ADJ_ACC: return launch_tb2d_phys_adj(K, true, full, a, s);
    case KM_STAR: break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_tb3d(int K, KMode m, bool full, const Tb3dArgs& a, hipStream_t s) {
  switch (m) {
    case KM_DIFF: return launch_tb3d_diff(K, full, a, s);
    case KM_HOT: return launch_tb3d_hot(K, full, a, s);
    case KM_ADJ: return launch_tb3d_adj(K, false, full, a, s);
    case KM_ADJ_ACC: return launch_tb3d_adj(K, true, full, a, s);
    case KM_PHYS:
    case KM_PHYS_ADJ:
    case KM_PHYS_ADJ_ACC:
    case KM_STAR: break;  // 2D only
  }
  return hipErrorInvalidValue;
}

hipError_t launch_plain(KMode m, const PlainArgs& a, hipStream_t s) {
  const int nb = plain_blocks(a);
  switch (m) {
    case KM_DIFF: hipLaunchKernelGGL((plain_kernel<false, false, false>), dim3(nb), dim3(64), 0, s, a); break;
    case KM_HOT: hipLaunchKernelGGL((plain_kernel<true, false, false>), dim3(nb), dim3(64), 0, s, a); break;
    case KM_ADJ: hipLaunchKernelGGL((plain_kernel<false, true, false>), dim3(nb), dim3(64), 0, s, a); break;
    case KM_ADJ_ACC: hipLaunchKernelGGL((plain_kernel<false, true, true>), dim3(nb), dim3(64), 0, s, a); break;
    case KM_PHYS:
      if (a.ndim != 2) return hipErrorInvalidValue;
      hipLaunchKernelGGL((plain_kernel<true, false, false, true>), dim3(nb), dim3(64), 0, s, a);
      break;
    case KM_PHYS_ADJ:
      if (a.ndim != 2) return hipErrorInvalidValue;
      hipLaunchKernelGGL((plain_kernel<false, true, false, true>), dim3(nb), dim3(64), 0, s, a);
      break;
    case KM_PHYS_ADJ_ACC:
      if (a.ndim != 2) return hipErrorInvalidValue;
      hipLaunchKernelGGL((plain_kernel<false, true, true, true>), dim3(nb), dim3(64), 0, s, a);
      break;
    case KM_STAR: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill(float* p, size_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_int(int* p, size_t n, int v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Bitwise comparison of two device arrays; adds the number of differing cells to *counter.
__global__ void count_mismatch_kernel(const float* a, const float* b, size_t n, int* counter) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  int local = 0;
  for (; i < n; i += stride) local += (__float_as_uint(a[i]) != __float_as_uint(b[i])) ? 1 : 0;
  if (local) atomicAdd(counter, local);
}

hipError_t launch_count_mismatch(const float* a, const float* b, size_t n, int* counter, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(count_mismatch_kernel, dim3((unsigned)nb), dim3(256), 0, s, a, b, n, counter);
  return hipGetLastError();
}
