// ctu_stream.hip -- plain streaming kernels that measure what this GPU's HBM delivers to
// accesses shaped like the CTU sweeps' (one 8-byte element per lane, 64 consecutive
// elements per wavefront), nothing of the method itself: a read-only sum, a copy, a 2:1
// add and a 5:1 combine (five input arrays, one output, the read:write mix of the fused
// update).  The achieved-bandwidth ceiling and the counter calibration of the roofline come
// from these.
#include "ctu_kernels.hpp"

namespace ctu {

namespace {

constexpr int kStreamUnroll = 4;  // elements per lane, blockDim apart (independent loads)

__device__ __forceinline__ double stream_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// out[blockIdx.x] = sum of the block's elements: every element is read once.
__global__ __launch_bounds__(256) void k_stream_read(const double* __restrict__ a, size_t n,
                                                     double* __restrict__ out) {
  const size_t base = (size_t)blockIdx.x * (256 * kStreamUnroll) + threadIdx.x;
  double v[kStreamUnroll];
#pragma unroll
  for (int k = 0; k < kStreamUnroll; ++k) {
    const size_t i = base + (size_t)k * 256;
    v[k] = i < n ? a[i] : 0.0;
  }
  double s = (v[0] + v[1]) + (v[2] + v[3]);
  s = stream_wave_sum(s);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ __launch_bounds__(256) void k_stream_copy(const double* __restrict__ a, size_t n,
                                                     double* __restrict__ c) {
  const size_t base = (size_t)blockIdx.x * (256 * kStreamUnroll) + threadIdx.x;
  double v[kStreamUnroll];
#pragma unroll
  for (int k = 0; k < kStreamUnroll; ++k) {
    const size_t i = base + (size_t)k * 256;
    v[k] = i < n ? a[i] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < kStreamUnroll; ++k) {
    const size_t i = base + (size_t)k * 256;
    if (i < n) c[i] = v[k];
  }
}

__global__ __launch_bounds__(256) void k_stream_add(const double* __restrict__ a,
                                                    const double* __restrict__ b, size_t n,
                                                    double* __restrict__ c) {
  const size_t base = (size_t)blockIdx.x * (256 * kStreamUnroll) + threadIdx.x;
  double v[kStreamUnroll];
#pragma unroll
  for (int k = 0; k < kStreamUnroll; ++k) {
    const size_t i = base + (size_t)k * 256;
    v[k] = i < n ? a[i] + b[i] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < kStreamUnroll; ++k) {
    const size_t i = base + (size_t)k * 256;
    if (i < n) c[i] = v[k];
  }
}

// c[i] = a[i] + a[n + i] + ... + a[4n + i]: five input arrays laid out one after another
// (as the fields of a state are), one output.
__global__ __launch_bounds__(256) void k_stream_combine5(const double* __restrict__ a, size_t n,
                                                         double* __restrict__ c) {
  const size_t base = (size_t)blockIdx.x * (256 * kStreamUnroll) + threadIdx.x;
  double v[kStreamUnroll];
#pragma unroll
  for (int k = 0; k < kStreamUnroll; ++k) {
    const size_t i = base + (size_t)k * 256;
    double s = 0.0;
    if (i < n) {
#pragma unroll
      for (int f = 0; f < 5; ++f) s += a[(size_t)f * n + i];
    }
    v[k] = s;
  }
#pragma unroll
  for (int k = 0; k < kStreamUnroll; ++k) {
    const size_t i = base + (size_t)k * 256;
    if (i < n) c[i] = v[k];
  }
}

}  // namespace

size_t stream_probe_blocks(size_t n) { return (n + 256 * kStreamUnroll - 1) / (256 * kStreamUnroll); }

hipError_t launch_stream_probe(int kind, const double* a, const double* b, double* c, size_t n,
                               hipStream_t stream) {
  const size_t nb = stream_probe_blocks(n);
  if (nb == 0 || nb > 0x7fffffffULL) return hipErrorInvalidValue;
  const dim3 G((unsigned)nb), B(256);
  switch (kind) {
    case STREAM_READ:
      hipLaunchKernelGGL(k_stream_read, G, B, 0, stream, a, n, c);
      break;
    case STREAM_COPY:
      hipLaunchKernelGGL(k_stream_copy, G, B, 0, stream, a, n, c);
      break;
    case STREAM_ADD:
      hipLaunchKernelGGL(k_stream_add, G, B, 0, stream, a, b, n, c);
      break;
    case STREAM_COMBINE5:
      hipLaunchKernelGGL(k_stream_combine5, G, B, 0, stream, a, n, c);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ctu
