// Calibration kernels: the device's practical streaming and MFMA rates,
// measured with code of this library rather than the runtime's copies, so
// that each kernel's roofline fraction can be set against what the same
// kind of code reaches on the same device.
//   copy   16-byte loads and stores, grid-stride, non-temporal: read and
//          write bytes once each (four independent loads per lane in flight
//          measured slower: 4.69 against 5.17 TB/s);
//   read   16-byte loads summed per lane, one partial per workgroup;
//   mfma   back-to-back MFMA on register operands, eight independent
//          accumulators per wave (no memory traffic).
#include "plan.h"

namespace bst {

namespace {
typedef double dbl2v __attribute__((ext_vector_type(2)));
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kCalibGrid = 256 * 8;   // eight workgroups of 256 lanes per compute unit

__global__ __launch_bounds__(256) void calib_copy_kernel(const dbl2v* __restrict__ src,
                                                         dbl2v* __restrict__ dst, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ __launch_bounds__(256) void calib_read_kernel(const dbl2v* __restrict__ src, int64_t n2,
                                                         double* __restrict__ partial) {
  __shared__ double red[4];
  const int64_t stride = (int64_t)gridDim.x * 256;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += stride) {
    const dbl2v v = __builtin_nontemporal_load(src + i);
    s += v.x + v.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// iters rounds of 8 independent MFMAs per wave; the accumulators are summed
// and written so that nothing is optimised away.
__global__ __launch_bounds__(256) void calib_mfma_f64_kernel(int64_t iters, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  double a = 1.0 + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
  dbl4 acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = dbl4{0, 0, 0, 0};
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void calib_mfma_bf16_kernel(int64_t iters, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1.0f + 0.001f * (float)(lane + e));
    b[e] = (__bf16)(1.0f - 0.001f * (float)(lane - e));
  }
  flt4 acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = flt4{0, 0, 0, 0};
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = (double)s;
}
// Reads only, so that the lines it leaves in the caches are clean and their
// eviction costs no write-back later.  The buffer holds zeros: the store that
// keeps the loads alive never happens.
__global__ __launch_bounds__(256) void cache_flush_kernel(dbl2v* __restrict__ buf, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += stride) {
    const dbl2v v = buf[i];
    s += v.x + v.y;
  }
  if (s == 1.0) buf[0] = dbl2v{s, s};
}
}  // namespace

hipError_t launch_cache_flush(double* buf, int64_t n, hipStream_t s) {
  if (!buf || n < 2) return hipSuccess;
  hipLaunchKernelGGL(cache_flush_kernel, dim3(kCalibGrid), dim3(256), 0, s, reinterpret_cast<dbl2v*>(buf),
                     n / 2);
  return hipGetLastError();
}

}  // namespace bst

using namespace bst;

extern "C" {

int32_t bst_calib_grid(void) { return kCalibGrid; }

bst_status bst_calib_copy(const void* src, void* dst, size_t bytes, void* stream) {
  BST_TRY
  if (!src || !dst || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(src) & 15) ||
      (reinterpret_cast<uintptr_t>(dst) & 15))
    fail(BST_E_INVALID, "copy buffers must be 16-byte aligned, bytes a multiple of 16");
  hipLaunchKernelGGL(calib_copy_kernel, dim3(kCalibGrid), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const dbl2v*>(src), static_cast<dbl2v*>(dst), (int64_t)(bytes / 16));
  check_hip(hipGetLastError(), "calibration copy");
  BST_CATCH
}

bst_status bst_calib_read(const void* src, size_t bytes, double* partial, void* stream) {
  BST_TRY
  if (!src || !partial || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(src) & 15))
    fail(BST_E_INVALID, "read buffer must be 16-byte aligned, bytes a multiple of 16");
  hipLaunchKernelGGL(calib_read_kernel, dim3(kCalibGrid), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const dbl2v*>(src), (int64_t)(bytes / 16), partial);
  check_hip(hipGetLastError(), "calibration read");
  BST_CATCH
}

bst_status bst_calib_mfma(bst_precision form, int64_t iters, double* out, double* flops, void* stream) {
  BST_TRY
  if (!out || !flops || iters < 1 || (form != BST_FP64 && form != BST_BF16X3))
    fail(BST_E_INVALID, "form must be BST_FP64 or BST_BF16X3, iters >= 1");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // 16x16x4 float64: 2048 flops; 16x16x32 bfloat16: 16384 flops per wave
  // instruction; 8 per round, 4 waves per workgroup
  const double per = form == BST_FP64 ? 2048.0 : 16384.0;
  *flops = per * 8.0 * (double)iters * (double)kCalibGrid * 4.0;
  if (form == BST_FP64)
    hipLaunchKernelGGL(calib_mfma_f64_kernel, dim3(kCalibGrid), dim3(256), 0, s, iters, out);
  else
    hipLaunchKernelGGL(calib_mfma_bf16_kernel, dim3(kCalibGrid), dim3(256), 0, s, iters, out);
  check_hip(hipGetLastError(), "calibration mfma");
  BST_CATCH
}

}  // extern "C"
