// Batched truncated-SVD products with bfloat16 components (Sec. 2.2 of the
// paper, one zeroth-order product U_i S_i (V_i^T B_i) per pair): the factors
// and the activations B_i are bfloat16, every product accumulates in float32.
//
// Three launches cover all pairs:
//   panel:  G_i = V_i^T B_i      (k x p, float32; split reductions as partials)
//   split:  the partials summed in split order and G_i carried as hi + lo
//           bfloat16 pairs (hi = bf16(g), lo = bf16(g - hi)), once per pair
//   output: out_i = (U_i S_i) G_i, so the second product sees G_i to ~2^-17
//           relative and only the stored components are bfloat16.
// Matrix cores: v_mfma_f32_16x16x32_bf16, lane l holding a[j] = A[l%16][8(l/16)+j],
// b[j] = B[8(l/16)+j][l%16] and d[r] = D[4(l/16)+r][l%16].  Both operands are
// staged k-contiguous in LDS (row stride 40 bf16: 16-byte aligned rows whose
// 16-byte reads by 8 consecutive lanes fall in distinct banks).
#include "amm_internal.hpp"

namespace amm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // vector types keep staging in registers

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int KS = 32;    // reduction step (rows of B per stage)
constexpr int FS = 32;    // factor chunk of the output kernel
constexpr int PT = 128;   // panel columns per workgroup
constexpr int OT16 = 128; // output tile
constexpr int LS = 40;    // LDS row stride (bf16) of 32-wide chunks
constexpr int MAXB = 256;

struct PanelJobB {
  const __bf16* Vt;   // k x n
  const __bf16* B;    // n x p
  int64_t n, p;
  int ntiles, splits;
  float* Gt;          // splits x (p x k)
  int64_t split_stride;
};

struct RedJobB {
  const float* Gt;    // splits x (p x k)
  int splits;
  int64_t split_stride;
  int64_t count;      // p x k
  __bf16* Gh;         // p x k
  __bf16* Gl;
};

struct OutJobB {
  int64_t m, p;
  const __bf16* US;   // m x k
  const __bf16* Gh;   // p x k, hi and lo parts of G^T
  const __bf16* Gl;
  float* out;         // m x p
};

__device__ __forceinline__ int xcd_tile16(int bid, int nblk) {
  if (nblk % 8) return bid;
  return (bid % 8) * (nblk / 8) + bid / 8;
}

__device__ __forceinline__ int find_job16(const int* start, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int K>
__global__ void __launch_bounds__(256)
panel_bf16_kernel(const PanelJobB* __restrict__ jobs, const int* __restrict__ start, int count) {
  constexpr int FB = K / 16;                       // factor blocks
  constexpr int VQ = (K * 4 + 255) / 256;          // 16-byte V loads per thread
  __shared__ int st[MAXB + 1];
  __shared__ __align__(16) __bf16 Bs[PT * LS];    // [col][r]
  __shared__ __align__(16) __bf16 Vs[K * LS];     // [f][r]
  for (int i = threadIdx.x; i <= count; i += blockDim.x) st[i] = start[i];
  __syncthreads();
  const int bid = blockIdx.x;
  const int jx = find_job16(st, count, bid);
  const PanelJobB jb = jobs[jx];
  const int local = xcd_tile16(bid - st[jx], st[jx + 1] - st[jx]);
  const int tile = local / jb.splits, split = local % jb.splits;
  const int64_t j0 = (int64_t)tile * PT;
  const int64_t per = jb.n / jb.splits;           // multiple of KS (host-checked)
  const int64_t rb = (int64_t)split * per, re = rb + per;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, li = lane & 15, lg = lane >> 4;
  const int rp = t & 15, cc = t >> 4;             // B staging: rows 2rp, 2rp+1; columns 8cc..8cc+7

  f32x4 acc[FB][2];
#pragma unroll
  for (int f = 0; f < FB; ++f) acc[f][0] = acc[f][1] = f32x4{0.f, 0.f, 0.f, 0.f};

  u32x4 x0, x1;   // eight bf16 of rows 2rp and 2rp + 1, element u in half (u & 1) of word u / 2
  u32x4 vr[VQ];
  auto fetch = [&](int64_t r0) {
    x0 = *reinterpret_cast<const u32x4*>(jb.B + (r0 + 2 * rp) * jb.p + j0 + 8 * cc);
    x1 = *reinterpret_cast<const u32x4*>(jb.B + (r0 + 2 * rp + 1) * jb.p + j0 + 8 * cc);
#pragma unroll
    for (int q = 0; q < VQ; ++q) {
      const int e = t + 256 * q;
      if (e < K * 4) vr[q] = *reinterpret_cast<const u32x4*>(jb.Vt + (int64_t)(e >> 2) * jb.n + r0 + 8 * (e & 3));
    }
  };
  auto stash = [&]() {
    unsigned int* bw = reinterpret_cast<unsigned int*>(Bs);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const unsigned int h0 = (x0[u >> 1] >> (16 * (u & 1))) & 0xffffu;
      const unsigned int h1 = (x1[u >> 1] >> (16 * (u & 1))) & 0xffffu;
      bw[((8 * cc + u) * LS + 2 * rp) >> 1] = h0 | (h1 << 16);
    }
#pragma unroll
    for (int q = 0; q < VQ; ++q) {
      const int e = t + 256 * q;
      if (e < K * 4) *reinterpret_cast<u32x4*>(Vs + (e >> 2) * LS + 8 * (e & 3)) = vr[q];
    }
  };

  if (rb < re) fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += KS) {
    __syncthreads();
    stash();
    __syncthreads();
    if (r0 + KS < re) fetch(r0 + KS);
    bf16x8 b[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
      b[cb] = *reinterpret_cast<const bf16x8*>(Bs + (32 * wave + 16 * cb + li) * LS + 8 * lg);
#pragma unroll
    for (int f = 0; f < FB; ++f) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(Vs + (16 * f + li) * LS + 8 * lg);
      acc[f][0] = mfma_bf16(a, b[0], acc[f][0]);
      acc[f][1] = mfma_bf16(a, b[1], acc[f][1]);
    }
  }
  // lane holds G[16f + 4lg + r][j0 + 32 wave + 16 cb + li]; Gt is p x K
  float* Gt = jb.Gt + (int64_t)split * jb.split_stride;
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int64_t c = j0 + 32 * wave + 16 * cb + li;
      *reinterpret_cast<float4*>(Gt + c * K + 16 * f + 4 * lg) =
          float4{acc[f][cb][0], acc[f][cb][1], acc[f][cb][2], acc[f][cb][3]};
    }
}

// G^T of every pair: split partials summed in split order, then hi + lo bf16
__global__ void __launch_bounds__(256)
g_split_kernel(const RedJobB* __restrict__ jobs, const int* __restrict__ start, int count) {
  __shared__ int st[MAXB + 1];
  for (int i = threadIdx.x; i <= count; i += blockDim.x) st[i] = start[i];
  __syncthreads();
  const int bid = blockIdx.x;
  const int jx = find_job16(st, count, bid);
  const RedJobB jb = jobs[jx];
  const int64_t i = ((int64_t)(bid - st[jx]) * 256 + threadIdx.x) * 4;
  if (i >= jb.count) return;
  f32x4 v = *reinterpret_cast<const f32x4*>(jb.Gt + i);
  for (int s = 1; s < jb.splits; ++s) v += *reinterpret_cast<const f32x4*>(jb.Gt + s * jb.split_stride + i);
  __bf16 h[4], l[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    h[r] = (__bf16)v[r];
    l[r] = (__bf16)(v[r] - (float)h[r]);
  }
  *reinterpret_cast<uint2*>(jb.Gh + i) = *reinterpret_cast<const uint2*>(h);
  *reinterpret_cast<uint2*>(jb.Gl + i) = *reinterpret_cast<const uint2*>(l);
}

template <int K>
__global__ void __launch_bounds__(256)
out_bf16_kernel(const OutJobB* __restrict__ jobs, const int* __restrict__ start, int count) {
  __shared__ int st[MAXB + 1];
  __shared__ __align__(16) __bf16 Us[OT16 * LS];   // [row][f]
  __shared__ __align__(16) __bf16 Gh[OT16 * LS];   // [col][f]
  __shared__ __align__(16) __bf16 Gl[OT16 * LS];
  for (int i = threadIdx.x; i <= count; i += blockDim.x) st[i] = start[i];
  __syncthreads();
  const int bid = blockIdx.x;
  const int jx = find_job16(st, count, bid);
  const OutJobB jb = jobs[jx];
  const int tile = xcd_tile16(bid - st[jx], st[jx + 1] - st[jx]);
  const int ntn = (int)(jb.p / OT16);
  const int64_t m0 = (int64_t)(tile / ntn) * OT16, n0 = (int64_t)(tile % ntn) * OT16;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, li = lane & 15, lg = lane >> 4;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  f32x4 acc[4][4];   // [column block][row block], computed transposed
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  // 128 rows (columns of G) x 32 bf16 per chunk and operand: 8 bf16 per load
  u32x4 ur[2], hr[2], lr[2];
  auto fetch = [&](int f0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = t + 256 * q;
      ur[q] = *reinterpret_cast<const u32x4*>(jb.US + (m0 + (e >> 2)) * K + f0 + 8 * (e & 3));
      hr[q] = *reinterpret_cast<const u32x4*>(jb.Gh + (n0 + (e >> 2)) * K + f0 + 8 * (e & 3));
      lr[q] = *reinterpret_cast<const u32x4*>(jb.Gl + (n0 + (e >> 2)) * K + f0 + 8 * (e & 3));
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = t + 256 * q, off = (e >> 2) * LS + 8 * (e & 3);
      *reinterpret_cast<u32x4*>(Us + off) = ur[q];
      *reinterpret_cast<u32x4*>(Gh + off) = hr[q];
      *reinterpret_cast<u32x4*>(Gl + off) = lr[q];
    }
  };

  fetch(0);
  for (int f0 = 0; f0 < K; f0 += FS) {
    __syncthreads();
    stash();
    __syncthreads();
    if (f0 + FS < K) fetch(f0 + FS);
    bf16x8 u[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) u[rb] = *reinterpret_cast<const bf16x8*>(Us + (wm + 16 * rb + li) * LS + 8 * lg);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const bf16x8 gh = *reinterpret_cast<const bf16x8*>(Gh + (wn + 16 * cb + li) * LS + 8 * lg);
      const bf16x8 gl = *reinterpret_cast<const bf16x8*>(Gl + (wn + 16 * cb + li) * LS + 8 * lg);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        acc[cb][rb] = mfma_bf16(gh, u[rb], acc[cb][rb]);
        acc[cb][rb] = mfma_bf16(gl, u[rb], acc[cb][rb]);
      }
    }
  }
  // lane holds out[m0 + wm + 16 rb + li][n0 + wn + 16 cb + 4 lg + r]
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
      *reinterpret_cast<float4*>(jb.out + (m0 + wm + 16 * rb + li) * jb.p + n0 + wn + 16 * cb + 4 * lg) =
          float4{acc[cb][rb][0], acc[cb][rb][1], acc[cb][rb][2], acc[cb][rb][3]};
}

// dst (cols x rows) = bf16(src^T) for src rows x cols float32
__global__ void bf16_transpose_kernel(const float* __restrict__ src, int64_t rows, int64_t cols,
                                      __bf16* __restrict__ dst) {
  __shared__ float tile[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[i][threadIdx.x] = src[r * cols + c];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int64_t c = c0 + i, r = r0 + threadIdx.x;
    if (r < rows && c < cols) dst[c * rows + r] = (__bf16)tile[threadIdx.x][i];
  }
}

__global__ void bf16_convert_kernel(const float* __restrict__ src, int64_t count, __bf16* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = (__bf16)src[i];
}

template <int K>
amm_status launch_bf16(const amm_batch_plan* bp, hipStream_t s) {
  const int count = (int)bp->items.size();
  {
    TimedLaunch tl("batch_panel_bf16", s);
    hipLaunchKernelGGL((panel_bf16_kernel<K>), dim3((unsigned)bp->panel_blocks), dim3(256), 0, s,
                       reinterpret_cast<const PanelJobB*>(bp->pjobs), (const int*)bp->pstart, count);
    AMM_HIP(hipGetLastError());
  }
  {
    TimedLaunch tl("batch_split_bf16", s);
    hipLaunchKernelGGL(g_split_kernel, dim3((unsigned)bp->red_blocks), dim3(256), 0, s,
                       reinterpret_cast<const RedJobB*>(bp->rjobs), (const int*)bp->rstart, count);
    AMM_HIP(hipGetLastError());
  }
  TimedLaunch tl("batch_out_bf16", s);
  hipLaunchKernelGGL((out_bf16_kernel<K>), dim3((unsigned)bp->out_blocks), dim3(256), 0, s,
                     reinterpret_cast<const OutJobB*>(bp->ojobs), (const int*)bp->ostart, count);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

}  // namespace

bool batch_item_ok_bf16(int64_t m, int64_t n, int64_t p, int k) {
  return (k == 32 || k == 64 || k == 128) && m > 0 && p > 0 && n > 0 && m % OT16 == 0 && p % PT == 0 &&
         n % KS == 0 && (m / OT16) * (p / OT16) < (int64_t)1 << 30;
}

// Plan-owned bfloat16 copies of the factors: Vt_i = bf16(V_i^T) (k x n_i) and
// US_i = bf16(U_i S_i) (m_i x k).
amm_status batch_convert_bf16(amm_batch_plan* bp, const std::vector<const float*>& V,
                              const std::vector<const float*>& US, hipStream_t s) {
  const int k = bp->k;
  size_t total = 0;
  for (const auto& it : bp->items) total += (size_t)k * (it.n + it.m);
  AMM_TRY(bp->fac16.alloc(std::max<size_t>(total, 1) * sizeof(__bf16)));
  __bf16* base = bp->fac16.as<__bf16>();
  size_t off = 0;
  for (size_t i = 0; i < bp->items.size(); ++i) {
    auto& it = bp->items[i];
    __bf16* vt = base + off;
    off += (size_t)k * it.n;
    __bf16* us = base + off;
    off += (size_t)k * it.m;
    if ((it.n + 31) / 32 > 65535) return fail(AMM_EUNSUPPORTED, "factor too tall");
    hipLaunchKernelGGL(bf16_transpose_kernel, dim3((unsigned)((k + 31) / 32), (unsigned)((it.n + 31) / 32)),
                       dim3(32, 8), 0, s, V[i], it.n, (int64_t)k, vt);
    AMM_HIP(hipGetLastError());
    const int64_t cnt = (int64_t)k * it.m;
    hipLaunchKernelGGL(bf16_convert_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, US[i], cnt, us);
    AMM_HIP(hipGetLastError());
    it.Vt16 = vt;
    it.US16 = us;
  }
  return AMM_OK;
}

amm_status batch_build_bf16(amm_batch_plan* bp, int target_blocks) {
  const int count = (int)bp->items.size();
  const int k = bp->k;
  std::vector<PanelJobB> pj(count);
  std::vector<OutJobB> oj(count);
  std::vector<RedJobB> rj(count);
  std::vector<int> ps(count + 1, 0), os(count + 1, 0), rs(count + 1, 0), splits(count);
  int64_t total_tiles = 0;
  for (auto& it : bp->items) total_tiles += it.p / PT;
  size_t part_floats = 0;
  for (int i = 0; i < count; ++i) {
    const auto& it = bp->items[i];
    int sp = 1;
    while (sp < 8 && total_tiles * sp * 2 <= target_blocks && it.n % (KS * sp * 2) == 0 && it.n / (sp * 2) >= 512)
      sp *= 2;
    splits[i] = sp;
    part_floats += (size_t)sp * k * it.p;
    ps[i + 1] = ps[i] + (int)(it.p / PT) * sp;
    os[i + 1] = os[i] + (int)((it.m / OT16) * (it.p / OT16));
    rs[i + 1] = rs[i] + (int)(((int64_t)k * it.p / 4 + 255) / 256);
  }
  size_t g_elems = 0;
  for (const auto& it : bp->items) g_elems += (size_t)k * it.p;
  AMM_TRY(bp->partials.reserve(part_floats * sizeof(float)));
  AMM_TRY(bp->gsplit.reserve(std::max<size_t>(g_elems, 1) * 2 * sizeof(__bf16)));
  size_t off = 0, goff = 0;
  for (int i = 0; i < count; ++i) {
    const auto& it = bp->items[i];
    float* G = bp->partials.as<float>() + off;
    off += (size_t)splits[i] * k * it.p;
    __bf16* gh = bp->gsplit.as<__bf16>() + goff;
    __bf16* gl = gh + g_elems;
    goff += (size_t)k * it.p;
    pj[i] = PanelJobB{static_cast<const __bf16*>(it.Vt16), static_cast<const __bf16*>(it.B16), it.n, it.p,
                      (int)(it.p / PT), splits[i], G, (int64_t)k * it.p};
    rj[i] = RedJobB{G, splits[i], (int64_t)k * it.p, (int64_t)k * it.p, gh, gl};
    oj[i] = OutJobB{it.m, it.p, static_cast<const __bf16*>(it.US16), gh, gl, it.out};
  }
  const size_t tbytes = count * (sizeof(PanelJobB) + sizeof(OutJobB) + sizeof(RedJobB)) + 3 * (count + 1) * sizeof(int);
  AMM_TRY(bp->tables.reserve(tbytes + 64));
  char* base = bp->tables.as<char>();
  bp->pjobs = base;
  bp->ojobs = base + count * sizeof(PanelJobB);
  bp->rjobs = base + count * (sizeof(PanelJobB) + sizeof(OutJobB));
  bp->pstart = reinterpret_cast<int*>(base + count * (sizeof(PanelJobB) + sizeof(OutJobB) + sizeof(RedJobB)));
  bp->ostart = bp->pstart + count + 1;
  bp->rstart = bp->ostart + count + 1;
  AMM_HIP(hipMemcpy(bp->pjobs, pj.data(), count * sizeof(PanelJobB), hipMemcpyHostToDevice));
  AMM_HIP(hipMemcpy(bp->ojobs, oj.data(), count * sizeof(OutJobB), hipMemcpyHostToDevice));
  AMM_HIP(hipMemcpy(bp->rjobs, rj.data(), count * sizeof(RedJobB), hipMemcpyHostToDevice));
  AMM_HIP(hipMemcpy(bp->pstart, ps.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice));
  AMM_HIP(hipMemcpy(bp->ostart, os.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice));
  AMM_HIP(hipMemcpy(bp->rstart, rs.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice));
  bp->panel_blocks = ps[count];
  bp->out_blocks = os[count];
  bp->red_blocks = rs[count];
  bp->splits = splits;
  bp->target_blocks = target_blocks;
  return AMM_OK;
}

amm_status batch_launch_bf16(const amm_batch_plan* bp, hipStream_t s) {
  switch (bp->k) {
    case 32: return launch_bf16<32>(bp, s);
    case 64: return launch_bf16<64>(bp, s);
    case 128: return launch_bf16<128>(bp, s);
    default: return fail(AMM_EUNSUPPORTED, "bf16 batch rank %d", bp->k);
  }
}

}  // namespace amm
