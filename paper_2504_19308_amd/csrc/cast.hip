// Element type conversion between row-major matrices of float32, bfloat16
// and float16 at any row pitch (the described operands of the C ABI):
// widening is exact, narrowing rounds to nearest even.  Rows whose length,
// pitches and addresses allow it move eight elements per thread (16-byte
// 16-bit words, two float4 of float32); the rest one element per thread.
#include "amm_internal.hpp"

namespace amm {
namespace {

__device__ __forceinline__ float load_as_f32(const void* p, int dtype, int64_t i) {
  if (dtype == AMM_BF16) return __uint_as_float((uint32_t)static_cast<const uint16_t*>(p)[i] << 16);
  if (dtype == AMM_F16) return __half2float(static_cast<const __half*>(p)[i]);
  return static_cast<const float*>(p)[i];
}

__device__ __forceinline__ uint16_t bf16_bits(float v) {
  const uint32_t b = __float_as_uint(v);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (uint16_t)((b >> 16) | 0x40u);   // NaN stays NaN
  return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);                                          // nearest even
}

__device__ __forceinline__ void store_from_f32(void* p, int dtype, int64_t i, float v) {
  if (dtype == AMM_BF16) static_cast<uint16_t*>(p)[i] = bf16_bits(v);
  else if (dtype == AMM_F16) static_cast<__half*>(p)[i] = __float2half_rn(v);
  else static_cast<float*>(p)[i] = v;
}

__global__ void cast_matrix_kernel(const void* __restrict__ src, int sdt, int64_t sld, int64_t rows, int64_t cols,
                                   void* __restrict__ dst, int ddt, int64_t dld) {
  // blockIdx.y strides over rows, threads over the columns of a row
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x)
      store_from_f32(dst, ddt, r * dld + c, load_as_f32(src, sdt, r * sld + c));
}

// eight elements of a row as float32
__device__ __forceinline__ void load8(const void* p, int dt, int64_t i, float (&v)[8]) {
  if (dt == AMM_F32) {
    const float4 a = *reinterpret_cast<const float4*>(static_cast<const float*>(p) + i);
    const float4 b = *reinterpret_cast<const float4*>(static_cast<const float*>(p) + i + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
    const uint4 w = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(p) + i);
    const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (dt == AMM_BF16) {
        v[2 * k] = __uint_as_float(u[k] << 16);
        v[2 * k + 1] = __uint_as_float(u[k] & 0xFFFF0000u);
      } else {
        v[2 * k] = __half2float(__ushort_as_half((unsigned short)(u[k] & 0xFFFFu)));
        v[2 * k + 1] = __half2float(__ushort_as_half((unsigned short)(u[k] >> 16)));
      }
    }
  }
}

__device__ __forceinline__ void store8(void* p, int dt, int64_t i, const float (&v)[8]) {
  if (dt == AMM_F32) {
    *reinterpret_cast<float4*>(static_cast<float*>(p) + i) = float4{v[0], v[1], v[2], v[3]};
    *reinterpret_cast<float4*>(static_cast<float*>(p) + i + 4) = float4{v[4], v[5], v[6], v[7]};
  } else {
    uint32_t u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t lo, hi;
      if (dt == AMM_BF16) {
        lo = bf16_bits(v[2 * k]);
        hi = bf16_bits(v[2 * k + 1]);
      } else {
        lo = __half_as_ushort(__float2half_rn(v[2 * k]));
        hi = __half_as_ushort(__float2half_rn(v[2 * k + 1]));
      }
      u[k] = lo | (hi << 16);
    }
    *reinterpret_cast<uint4*>(static_cast<uint16_t*>(p) + i) = uint4{u[0], u[1], u[2], u[3]};
  }
}

__global__ void cast_matrix8_kernel(const void* __restrict__ src, int sdt, int64_t sld, int64_t rows, int64_t cols8,
                                    void* __restrict__ dst, int ddt, int64_t dld) {
  const int64_t total = rows * cols8;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / cols8, c = (t - r * cols8) * 8;
    float v[8];
    load8(src, sdt, r * sld + c, v);
    store8(dst, ddt, r * dld + c, v);
  }
}

}  // namespace

amm_status cast_matrix(const void* src, int src_dtype, int64_t src_ld, int64_t rows, int64_t cols, void* dst,
                       int dst_dtype, int64_t dst_ld, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return AMM_OK;
  TimedLaunch tl("cast_matrix", s);
  const size_t ss = src_dtype == AMM_F32 ? 4 : 2, ds = dst_dtype == AMM_F32 ? 4 : 2;
  const bool wide = cols % 8 == 0 && src_ld % 8 == 0 && dst_ld % 8 == 0 && ((uintptr_t)src % (8 * ss)) == 0 &&
                    ((uintptr_t)dst % (8 * ds)) == 0 && ((uintptr_t)src % 16) == 0 && ((uintptr_t)dst % 16) == 0;
  if (wide) {
    const int64_t total = rows * (cols / 8);
    const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(cast_matrix8_kernel, dim3(grid), dim3(256), 0, s, src, src_dtype, src_ld, rows, cols / 8, dst,
                       dst_dtype, dst_ld);
  } else {
    const unsigned gx = (unsigned)std::min<int64_t>((cols + 255) / 256, 64);
    const unsigned gy = (unsigned)std::min<int64_t>(rows, 8192);
    hipLaunchKernelGGL(cast_matrix_kernel, dim3(gx, gy), dim3(256), 0, s, src, src_dtype, src_ld, rows, cols, dst,
                       dst_dtype, dst_ld);
  }
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

}  // namespace amm
