// Dominant-entry sparsification and the sparse products (eq. (2.4) of the
// paper, abstract; Sec. 2.4 "may require exploitation of sparse data
// structures").
//
// Reading: S keeps the nnz entries of largest |a| (ties to the smaller
// row-major index), stored as CSR; R = A - S is the dense residue.
//
// Extraction is a radix select on the IEEE bit pattern of |a| (for finite
// floats the order of |a| equals the unsigned order of (bits & 0x7fffffff)):
// four 8-bit digit passes from the top narrow down the threshold key T with
//   #{key > T} < nnz <= #{key >= T},
// the entries with key == T are then taken in row-major order until nnz is
// reached.  A per-row pass writes CSR rows (column order) and R.
#include <algorithm>
#include <utility>
#include <vector>

#include "amm_internal.hpp"

namespace amm {
namespace {

__device__ __forceinline__ uint32_t key_of(float a) { return __float_as_uint(a) & 0x7fffffffu; }

// histogram of digit `shift` among keys whose bits above the digit equal prefix
__global__ void radix_hist(const float* __restrict__ A, int64_t count, uint32_t prefix,
                           uint32_t hi_mask, int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const uint32_t k = key_of(A[i]);
    if ((k & hi_mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// per-row counts of key > T and key == T
__global__ void row_counts(const float* __restrict__ A, int64_t n, uint32_t T,
                           int32_t* __restrict__ gt, int32_t* __restrict__ eq) {
  const int64_t row = blockIdx.x;
  const float* a = A + row * n;
  int cg = 0, ce = 0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const uint32_t k = key_of(a[j]);
    cg += k > T;
    ce += k == T;
  }
  __shared__ int sg[256], se[256];
  sg[threadIdx.x] = cg;
  se[threadIdx.x] = ce;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      sg[threadIdx.x] += sg[threadIdx.x + off];
      se[threadIdx.x] += se[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    gt[row] = sg[0];
    eq[row] = se[0];
  }
}

// Block-wide exclusive scan of 0/1 flags (256 threads, 4 waves of 64).
__device__ __forceinline__ int block_excl_scan(int flag, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  const int in_wave = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) wsum[wave] = __popcll(m);
  __syncthreads();
  int before = 0, tot = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) before += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return before + in_wave;
}

// One block per row: write the kept entries (column order) and R = A - S.
__global__ void __launch_bounds__(256)
fill_rows(const float* __restrict__ A, int64_t n, uint32_t T, const int32_t* __restrict__ take_eq,
          const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col, float* __restrict__ val,
          float* __restrict__ R) {
  __shared__ int wsum[4];
  const int64_t row = blockIdx.x;
  const float* a = A + row * n;
  float* r = R + row * n;
  int eq_seen = 0, out_pos = row_ptr[row];
  const int eq_cap = take_eq[row];
  for (int64_t j0 = 0; j0 < n; j0 += 256) {
    const int64_t j = j0 + threadIdx.x;
    float v = 0.f;
    uint32_t k = 0;
    if (j < n) {
      v = a[j];
      k = key_of(v);
    }
    const int is_eq = (j < n) && (k == T);
    int eq_tot;
    const int eq_rank = eq_seen + block_excl_scan(is_eq, wsum, &eq_tot);
    const int keep = (j < n) && (k > T || (is_eq && eq_rank < eq_cap));
    int keep_tot;
    const int pos = out_pos + block_excl_scan(keep, wsum, &keep_tot);
    if (keep) {
      col[pos] = (int32_t)j;
      val[pos] = v;
    }
    if (j < n) r[j] = keep ? 0.f : v;
    eq_seen += eq_tot;
    out_pos += keep_tot;
  }
}

// S B with S in CSR.  B is cut into slices of 64 columns; a block owns one
// slice of 16 output rows, each row handled by 16 lanes holding 4 adjacent
// columns, which walk the row's stored entries and gather the matching 256-byte
// slice rows of B (4 gathers in flight, summed in entry order).  Blocks are
// dealt so that every XCD sweeps whole slices: all rows of a slice run on one
// XCD, whose L2 then holds that slice of B (n x 256 bytes) while it is reused
// by every stored entry.  A row's entries are taken from rng[row * stride +
// blk] to rng[row * stride + blk + 1]: the whole row (rng = row_ptr, stride 1)
// or, for long inner dimensions, the part of the row in one block of inner
// indices, launched block after block with the later blocks accumulating, so
// that the slice of B an XCD holds is 4096 x 256 bytes.
constexpr int SW = 64;    // columns per slice
constexpr int RPB = 16;   // rows per block

__global__ void __launch_bounds__(256)
spmm_slices(const int32_t* __restrict__ rng, int stride, int blk, const int32_t* __restrict__ col,
            const float* __restrict__ val, const float* __restrict__ B, int64_t ldb, int64_t rows, int64_t p,
            float* __restrict__ out, int64_t ldo, int accumulate, int nslices, int rgroups, int vec) {
  const int bid = blockIdx.x;
  int slice, rg;
  if ((nslices & 7) == 0) {
    const int xcd = bid & 7, local = bid >> 3;
    slice = xcd * (nslices >> 3) + local / rgroups;
    rg = local % rgroups;
  } else {
    slice = bid / rgroups;
    rg = bid % rgroups;
  }
  const int64_t row = (int64_t)rg * RPB + (threadIdx.x >> 4);
  const int64_t c0 = (int64_t)slice * SW + (threadIdx.x & 15) * 4;
  if (row >= rows || c0 >= p) return;
  const int e0 = rng[row * stride + blk], e1 = rng[row * stride + blk + 1];
  float* o = out + row * ldo + c0;
  if (vec) {  // p, ldb, ldo % 4 == 0 and 16-byte aligned B / out: c0 + 3 < p
    float4 acc{0.f, 0.f, 0.f, 0.f};
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
      float v[4];
      float4 x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[u] = val[e + u];
        x[u] = *reinterpret_cast<const float4*>(B + (int64_t)col[e + u] * ldb + c0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc.x += v[u] * x[u].x; acc.y += v[u] * x[u].y; acc.z += v[u] * x[u].z; acc.w += v[u] * x[u].w;
      }
    }
    for (; e < e1; ++e) {
      const float v = val[e];
      const float4 x = *reinterpret_cast<const float4*>(B + (int64_t)col[e] * ldb + c0);
      acc.x += v * x.x; acc.y += v * x.y; acc.z += v * x.z; acc.w += v * x.w;
    }
    if (accumulate) {
      const float4 z = *reinterpret_cast<const float4*>(o);
      acc = float4{acc.x + z.x, acc.y + z.y, acc.z + z.z, acc.w + z.w};
    }
    *reinterpret_cast<float4*>(o) = acc;
  } else {
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int e = e0; e < e1; ++e) {
      const float v = val[e];
      const float* b = B + (int64_t)col[e] * ldb + c0;
      for (int q = 0; q < 4 && c0 + q < p; ++q) acc[q] += v * b[q];
    }
    for (int q = 0; q < 4 && c0 + q < p; ++q) o[q] = accumulate ? o[q] + acc[q] : acc[q];
  }
}

constexpr int SWN = 32;   // columns per slice, narrow form
constexpr int RPBN = 32;  // rows per block, narrow form
// entries per round (two per lane): 4.75 ms against 5.3 ms for 8 at n = 16384
// (cross-lane swizzles instead of the LDS hand-over: 4.95 ms)
constexpr int kNarrowRound = 16;

// S B with S in CSR, float4 path (p, ldb, ldo % 4 == 0, 16-byte aligned B and
// out).  Slices of 32 columns, 8 lanes per row (a float4 each), whole rows in
// one pass: a slice of B is n x 128 bytes (2 MiB at n = 16384), held in one
// XCD's L2 while that XCD sweeps the slice's rows (blocks are dealt so that
// every XCD owns whole slices), and each gathered row is one 128-byte line.
// A row's stored entries come G at a time, one or two per lane, in one
// coalesced read of the indices and one of the values, issued a round ahead;
// each round's entries are handed to the row's lanes through LDS: every lane
// stores its (column, value) pairs in its group's slot and every lane reads
// the round back two entries at a time (the 8 lanes of a group read the same
// address, a broadcast).  A wave's LDS operations complete in order, so the
// group's stores are visible to its reads without a barrier; wave barriers
// keep the compiler from moving them across each other.  With `add` the
// result is out = S B + add (add with row pitch ld_add), else out (+)= S B.
template <int G>
__global__ void __launch_bounds__(256)
spmm_narrow(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const float* __restrict__ val,
                const float* __restrict__ B, int64_t ldb, int64_t rows, int64_t p, float* __restrict__ out,
                int64_t ldo, int accumulate, const float* __restrict__ add, int64_t ld_add, int nslices,
                int rgroups) {
  static_assert(G == 8 || G == 16, "one or two entries per lane and round");
  constexpr int H = G / 8;
  __shared__ __align__(16) int2 ent[256 / 8][G];
  const int bid = blockIdx.x;
  int slice, rg;
  if ((nslices & 7) == 0) {
    const int xcd = bid & 7, local = bid >> 3;
    slice = xcd * (nslices >> 3) + local / rgroups;
    rg = local % rgroups;
  } else {
    slice = bid / rgroups;
    rg = bid % rgroups;
  }
  const int lane8 = threadIdx.x & 7;
  int2* my = ent[threadIdx.x >> 3];
  const int64_t row = (int64_t)rg * RPBN + (threadIdx.x >> 3);
  if (row >= rows) return;            // a row's 8 lanes leave together
  const int64_t c0 = (int64_t)slice * SWN + lane8 * 4;
  const bool ok = c0 < p;
  const int e0 = row_ptr[row], e1 = row_ptr[row + 1];
  int nc[H], nv[H];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int e = e0 + 8 * h + lane8;
    nc[h] = 0;
    nv[h] = 0;
    if (e < e1) {
      nc[h] = col[e];
      nv[h] = __float_as_int(val[e]);
    }
  }
  float4 acc{0.f, 0.f, 0.f, 0.f};
  for (int base = e0; base < e1; base += G) {
#pragma unroll
    for (int h = 0; h < H; ++h) my[8 * h + lane8] = int2{nc[h], nv[h]};
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int e = base + G + 8 * h + lane8;
      nc[h] = 0;
      nv[h] = 0;
      if (e < e1) {
        nc[h] = col[e];
        nv[h] = __float_as_int(val[e]);
      }
    }
    const int cnt = e1 - base;
    float4 x[G];
    float v[G];
#pragma unroll
    for (int j = 0; j < G; j += 2) {
      const int4 q = *reinterpret_cast<const int4*>(&my[j]);
      v[j] = __int_as_float(q.y);
      v[j + 1] = __int_as_float(q.w);
      x[j] = (j < cnt && ok) ? *reinterpret_cast<const float4*>(B + (int64_t)q.x * ldb + c0)
                             : float4{0.f, 0.f, 0.f, 0.f};
      x[j + 1] = (j + 1 < cnt && ok) ? *reinterpret_cast<const float4*>(B + (int64_t)q.z * ldb + c0)
                                     : float4{0.f, 0.f, 0.f, 0.f};
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < G; ++j) {
      acc.x += v[j] * x[j].x;
      acc.y += v[j] * x[j].y;
      acc.z += v[j] * x[j].z;
      acc.w += v[j] * x[j].w;
    }
  }
  if (!ok) return;
  float4* o = reinterpret_cast<float4*>(out + row * ldo + c0);
  if (add) {
    const float4 z = *reinterpret_cast<const float4*>(add + row * ld_add + c0);
    acc = float4{acc.x + z.x, acc.y + z.y, acc.z + z.z, acc.w + z.w};
  } else if (accumulate) {
    const float4 z = *o;
    acc = float4{acc.x + z.x, acc.y + z.y, acc.z + z.z, acc.w + z.w};
  }
  *o = acc;
}

// out (cols x rows, row pitch ldo) (+)= Y^T for Y rows x cols (row pitch ldy),
// through 32 x 33 LDS tiles
__global__ void transpose_acc_kernel(const float* __restrict__ Y, int64_t ldy, int64_t rows, int64_t cols,
                                     float* __restrict__ out, int64_t ldo, int accumulate) {
  __shared__ float tile[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[i][threadIdx.x] = Y[r * ldy + c];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int64_t c = c0 + i, r = r0 + threadIdx.x;
    if (r < rows && c < cols) {
      float* o = out + c * ldo + r;
      *o = accumulate ? *o + tile[threadIdx.x][i] : tile[threadIdx.x][i];
    }
  }
}

__global__ void fill_kernel(float* __restrict__ p, int64_t count, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

}  // namespace

__global__ void transpose_kernel(const float* __restrict__ src, int64_t lds_, int64_t rows, int64_t cols,
                                 float* __restrict__ dst, int64_t ldd) {
  __shared__ float tile[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[i][threadIdx.x] = src[r * lds_ + c];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int64_t c = c0 + i, r = r0 + threadIdx.x;
    if (r < rows && c < cols) dst[c * ldd + r] = tile[threadIdx.x][i];
  }
}

amm_status transpose_ld_f32(const float* src, int64_t ld_src, int64_t rows, int64_t cols, float* dst,
                            int64_t ld_dst, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return AMM_OK;
  if ((rows + 31) / 32 > 65535) return fail(AMM_EUNSUPPORTED, "transpose too tall");
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32)),
                     dim3(32, 8), 0, s, src, ld_src, rows, cols, dst, ld_dst);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

amm_status transpose_f32(const float* src, int64_t rows, int64_t cols, float* dst, hipStream_t s) {
  return transpose_ld_f32(src, cols, rows, cols, dst, rows, s);
}

amm_status transpose_acc_ld_f32(const float* Y, int64_t ldy, int64_t rows, int64_t cols, float* out, int64_t ldo,
                                bool accumulate, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return AMM_OK;
  if ((rows + 31) / 32 > 65535 || (cols + 31) / 32 > 65535) return fail(AMM_EUNSUPPORTED, "transpose too large");
  hipLaunchKernelGGL(transpose_acc_kernel, dim3((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32)),
                     dim3(32, 8), 0, s, Y, ldy, rows, cols, out, ldo, accumulate ? 1 : 0);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

amm_status transpose_acc_f32(const float* Y, int64_t rows, int64_t cols, float* out, bool accumulate,
                             hipStream_t s) {
  return transpose_acc_ld_f32(Y, cols, rows, cols, out, rows, accumulate, s);
}

// Row pitch (in floats) for a scratch copy of a matrix with `cols` columns
// whose gathers or column reads would otherwise all fall on one L2 channel:
// pitches that are large multiples of a power of two (16384 floats = 64 KiB,
// say) put every row of a column slice at the same address bits; 64 extra
// floats shift consecutive rows by 256 bytes.
int64_t spread_pitch(int64_t cols) { return (cols >= 2048 && cols % 2048 == 0) ? cols + 64 : cols; }

// dst (rows x cols, row pitch ld_dst) = src (rows x cols, contiguous)
__global__ void repitch_kernel(const float4* __restrict__ src, int64_t lds4, int64_t rows, int64_t cols4,
                               float4* __restrict__ dst, int64_t ld4) {
  const int64_t total = rows * cols4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols4, c = i - r * cols4;
    dst[r * ld4 + c] = src[r * lds4 + c];
  }
}

amm_status repitch_f32(const float* src, int64_t ld_src, int64_t rows, int64_t cols, float* dst, int64_t ld_dst,
                       hipStream_t s) {
  if (rows <= 0 || cols <= 0) return AMM_OK;
  if (cols % 4 || ld_dst % 4 || ld_src % 4 || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16))
    return fail(AMM_EINVAL, "repitch needs float4-aligned rows");
  TimedLaunch tl("repitch", s);
  const int64_t cols4 = cols / 4, total = rows * cols4;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(repitch_kernel, dim3(grid), dim3(256), 0, s, reinterpret_cast<const float4*>(src), ld_src / 4,
                     rows, cols4, reinterpret_cast<float4*>(dst), ld_dst / 4);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

amm_status fill_f32(float* p, int64_t count, float v, hipStream_t s) {
  if (count <= 0) return AMM_OK;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

amm_status sparse_extract(amm_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t nnz,
                          amm_dec* d, float* R, hipStream_t s) {
  (void)ctx;
  const int64_t count = m * n;
  if (m > 0x7fffffff || nnz > 0x7fffffff) return fail(AMM_EUNSUPPORTED, "sparse part too large for int32 CSR");
  d->nnz = nnz;
  AMM_TRY(d->row_ptr.alloc((m + 1) * 4));
  AMM_TRY(d->col.alloc(std::max<int64_t>(nnz, 1) * 4));
  AMM_TRY(d->val.alloc(std::max<int64_t>(nnz, 1) * 4));

  // radix select of the threshold key
  uint32_t prefix = 0, hi_mask = 0;
  int64_t remaining = nnz;  // how many of the keys matching the prefix are still needed
  DevBuf hist;
  AMM_TRY(hist.alloc(256 * 4));
  uint32_t T = 0xffffffffu;  // nnz == 0: nothing passes key > T or == T
  if (nnz > 0) {
    const unsigned grid = (unsigned)std::min<int64_t>((count + 255) / 256, 4096);
    for (int shift = 24; shift >= 0; shift -= 8) {
      AMM_HIP(hipMemsetAsync(hist.ptr, 0, 256 * 4, s));
      hipLaunchKernelGGL(radix_hist, dim3(grid), dim3(256), 0, s, A, count, prefix, hi_mask, shift,
                         hist.as<uint32_t>());
      AMM_HIP(hipGetLastError());
      uint32_t h[256];
      AMM_HIP(hipMemcpyAsync(h, hist.ptr, sizeof(h), hipMemcpyDeviceToHost, s));
      AMM_HIP(hipStreamSynchronize(s));
      int digit = 255;
      for (; digit >= 0; --digit) {
        if ((int64_t)h[digit] >= remaining) break;
        remaining -= h[digit];
      }
      if (digit < 0) return fail(AMM_EDEVICE, "radix select lost count");
      prefix |= (uint32_t)digit << shift;
      hi_mask |= 255u << shift;
    }
    T = prefix;
  }
  // remaining = number of entries equal to T that must be taken
  DevBuf gt, eq, take, rp;
  AMM_TRY(gt.alloc(m * 4));
  AMM_TRY(eq.alloc(m * 4));
  AMM_TRY(take.alloc(m * 4));
  std::vector<int32_t> hgt(m), heq(m), htake(m), hrp(m + 1);
  if (nnz > 0) {
    hipLaunchKernelGGL(row_counts, dim3((unsigned)m), dim3(256), 0, s, A, n, T, gt.as<int32_t>(), eq.as<int32_t>());
    AMM_HIP(hipGetLastError());
    AMM_HIP(hipMemcpyAsync(hgt.data(), gt.ptr, m * 4, hipMemcpyDeviceToHost, s));
    AMM_HIP(hipMemcpyAsync(heq.data(), eq.ptr, m * 4, hipMemcpyDeviceToHost, s));
    AMM_HIP(hipStreamSynchronize(s));
  }
  int64_t eq_left = remaining, pos = 0;
  for (int64_t i = 0; i < m; ++i) {
    const int64_t tk = std::min<int64_t>(eq_left, heq[i]);
    htake[i] = (int32_t)tk;
    eq_left -= tk;
    hrp[i] = (int32_t)pos;
    pos += hgt[i] + tk;
  }
  hrp[m] = (int32_t)pos;
  if (pos != nnz) return fail(AMM_EDEVICE, "sparse count mismatch %lld vs %lld", (long long)pos, (long long)nnz);
  AMM_HIP(hipMemcpyAsync(take.ptr, htake.data(), m * 4, hipMemcpyHostToDevice, s));
  AMM_HIP(hipMemcpyAsync(d->row_ptr.ptr, hrp.data(), (m + 1) * 4, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(fill_rows, dim3((unsigned)m), dim3(256), 0, s, A, n, T, take.as<int32_t>(),
                     d->row_ptr.as<int32_t>(), d->col.as<int32_t>(), d->val.as<float>(), R);
  AMM_HIP(hipGetLastError());
  AMM_TRY(build_csc(d, s));
  // norms for reporting: ||A||_F^2 = ||S||^2 + ||R||^2 is left to the caller
  return AMM_OK;
}

namespace {


// out = S B (+ out if acc, or + add when add != nullptr: float4 path only)
amm_status spmm_launch(const int32_t* row_ptr, const int32_t* col, const float* val, int64_t rows,
                       const float* B, int64_t ldb, int64_t p, float* out, int64_t ldo, bool acc, hipStream_t s,
                       const int32_t* blk_ptr, int blocks, const float* add = nullptr, int64_t ld_add = 0) {
  if (rows <= 0 || p <= 0) return AMM_OK;
  const int64_t nslices = (p + SW - 1) / SW, rgroups = (rows + RPB - 1) / RPB;
  if (nslices * rgroups > 0x7fffffff || rgroups > 0x7fffffff) return fail(AMM_EUNSUPPORTED, "SpMM grid too large");
  if (blocks > 1 && !blk_ptr) return fail(AMM_EINVAL, "blocked SpMM without block ranges");
  const int vec = (p % 4 == 0 && ldb % 4 == 0 && ldo % 4 == 0 && ((uintptr_t)B % 16) == 0 &&
                   ((uintptr_t)out % 16) == 0) ? 1 : 0;
  if (vec) {
    const int64_t ns = (p + SWN - 1) / SWN, rgs = (rows + RPBN - 1) / RPBN;
    if (ns * rgs > 0x7fffffff) return fail(AMM_EUNSUPPORTED, "SpMM grid too large");
    if (add && (ld_add % 4 || ((uintptr_t)add % 16))) return fail(AMM_EINVAL, "SpMM addend not float4 aligned");
    hipLaunchKernelGGL(spmm_narrow<kNarrowRound>, dim3((unsigned)(ns * rgs)), dim3(256), 0, s, row_ptr, col, val, B,
                       ldb, rows, p, out, ldo, acc ? 1 : 0, add, ld_add, (int)ns, (int)rgs);
    AMM_HIP(hipGetLastError());
    return AMM_OK;
  }
  if (add) return fail(AMM_EINVAL, "SpMM with an addend needs the float4 path");
  const int32_t* rng = blocks <= 1 ? row_ptr : blk_ptr;
  const int stride = blocks <= 1 ? 1 : blocks + 1;
  for (int b = 0; b < std::max(blocks, 1); ++b) {
    const int a = (acc || b > 0) ? 1 : 0;
    hipLaunchKernelGGL(spmm_slices, dim3((unsigned)(nslices * rgroups)), dim3(256), 0, s, rng, stride, b, col,
                         val, B, ldb, rows, p, out, ldo, a, (int)nslices, (int)rgroups, vec);
    AMM_HIP(hipGetLastError());
  }
  return AMM_OK;
}

}  // namespace

amm_status spmm_raw(const int32_t* row_ptr, const int32_t* col, const float* val, int64_t rows,
                    const float* B, int64_t p, float* out, bool acc, hipStream_t s, const int32_t* blk_ptr,
                    int blocks, int64_t ldb, int64_t ldo) {
  TimedLaunch tl("spmm_csr", s);
  return spmm_launch(row_ptr, col, val, rows, B, ldb > 0 ? ldb : p, p, out, ldo > 0 ? ldo : p, acc, s, blk_ptr,
                     blocks);
}

amm_status spmm_csr(const amm_dec* d, const float* B, int64_t ldb, int64_t p, float* out, bool acc, hipStream_t s,
                    const float* add, int64_t ld_add, int64_t ldo) {
  TimedLaunch tl("spmm_csr", s);
  return spmm_launch(d->row_ptr.as<int32_t>(), d->col.as<int32_t>(), d->val.as<float>(), d->m, B, ldb, p, out,
                     ldo > 0 ? ldo : p, acc, s, d->csr_blk.as<int32_t>(), d->csr_blocks, add, ld_add);
}

// out (rows x p) (+)= X S for X rows x n and S n x p sparse:
//   (X S)^T = S^T X^T, and S^T in CSR is S in CSC, so the product is the row
//   gather above on X^T, transposed back into out.  The transposed scratch
//   copies get a pitch that spreads their rows over the L2 channels.
amm_status dense_times_csr(amm_ctx* ctx, const float* X, int64_t rows, const amm_dec* d, float* out,
                           bool acc, hipStream_t s) {
  const int64_t n = d->m, p = d->n;
  if (rows <= 0 || p <= 0) return AMM_OK;
  if ((rows + 31) / 32 > 65535 || (p + 31) / 32 > 65535) return fail(AMM_EUNSUPPORTED, "sparse operand too large");
  const int64_t ld = spread_pitch(rows);
  AMM_TRY(ctx->scratch[6].reserve((size_t)n * ld * sizeof(float)));
  AMM_TRY(ctx->scratch[7].reserve((size_t)p * ld * sizeof(float)));
  float* Xt = ctx->scratch[6].as<float>();
  float* Y = ctx->scratch[7].as<float>();
  TimedLaunch tl("dense_times_csr", s);
  AMM_TRY(transpose_ld_f32(X, n, rows, n, Xt, ld, s));
  AMM_TRY(spmm_launch(d->csc_ptr.as<int32_t>(), d->csc_row.as<int32_t>(), d->csc_val.as<float>(), p, Xt, ld, rows, Y,
                      ld, false, s, d->csc_blk.as<int32_t>(), d->csc_blocks));
  return transpose_acc_ld_f32(Y, ld, p, rows, out, p, acc, s);
}

}  // namespace amm
