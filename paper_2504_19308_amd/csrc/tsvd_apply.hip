// Truncated-SVD products on the matrix cores (Sec. 2.2 of the paper).
//
//   zeroth order  M0 = U_A S_A (V_A^T B)
//   first order   M1 = M0 + Delta A Btil
//                    = U_A S_A (V_A^T Delta B) + (A U_B)(S_B V_B^T)
// (expand Atil B + (A - Atil) Btil = Atil (B - Btil) + A Btil).  With Delta B
// kept by B's decomposition the first-order product needs no k x k correction
// term: one "panel" launch computes the two skinny products
//   G = V_A^T Delta B  (k_A x p, streams Delta B once)
//   H = A U_B          (m x k_B, streams A once)
// and one output GEMM with the short inner dimension k_A + k_B writes
//   M1 = [U_A S_A | H] [G ; S_B V_B^T].
// Both launches stream their large operand from HBM exactly once; the factor
// matrices (<= 2 MiB) stay in L2.
//
// panel_kernel: C (a x b) = X^T Y for a tall X (n x a, a <= 128) and a tall
// view Y (n x b); one workgroup owns TB = 16 columns of C and the whole
// reduction over n, its four waves splitting every 64-row slab; partial sums
// meet in LDS at the end (fixed order, deterministic).
//
// out_kernel: C (M x N) = [A1 | A2][B1 ; B2] with K1 + K2 <= 256; 128 x 128
// tiles, the K extent staged through LDS in slabs of 64 with the next slab
// prefetched into registers.
#include "amm_internal.hpp"

namespace amm {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Tile order that keeps neighbouring tiles on one XCD (blocks are dealt to
// the 8 XCDs round-robin); identity unless the count divides evenly.
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
  if (nblk % 8) return bid;
  return (bid % 8) * (nblk / 8) + bid / 8;
}

// One skinny product  C (a x TB tile) = X^T Y  over the rows [r_begin, r_end)
// of the reduction.  X: n x A row-major (the factor), Y: the large operand.
//  YROW:  Y(i, j) = Y[i * y_ld + j0 + j]   (a column slab of a row-major matrix)
//  !YROW: Y(i, j) = Y[(j0 + j) * y_ld + i] (TB rows of a row-major matrix)
// Y is staged k-contiguous per column (Yt[j][i]) so that both the loads and the
// per-lane MFMA operand reads are conflict-free.
template <int A, int TB> struct PanelCfg {
  static constexpr int BK = (A * TB <= 32 * 16) ? 128 : ((A * TB <= 64 * 32) ? 64 : 32);
  // X rows: stride 16 or 48 (mod 64) words so the 4 k-rows of an operand read
  // fall in disjoint bank groups; Yt rows: stride 4 (mod 64) words
  static constexpr int XS = ((A + 16) % 32 == 16) ? A + 16 : A + 32;
  static constexpr int YS = BK + 4;
  static constexpr int XN4 = (BK * A / 4 + 255) / 256;
  static constexpr int YN4 = (BK * TB / 4 + 255) / 256;
  static constexpr int SMEM = BK * XS + TB * YS;
  static constexpr int RED = 4 * A * TB;
  static constexpr int SMEM_ALL = SMEM > RED ? SMEM : RED;
};

struct PanelJob {
  const float* X;
  const float* Y;
  int64_t y_ld;
  int64_t n;          // reduction length
  int ntiles;         // column tiles
  int splits;         // reduction splits (blockIdx -> tile, split)
  float* C;
  int64_t c_rs, c_cs, c_split;
};

template <int A, int TB, bool YROW>
__device__ __forceinline__ void panel_tile(const PanelJob& jb, int bid, int nblk, float* smem) {
  using Cfg = PanelCfg<A, TB>;
  constexpr int BK = Cfg::BK, XS = Cfg::XS, YS = Cfg::YS, XN4 = Cfg::XN4, YN4 = Cfg::YN4;
  float* Xs = smem;
  float* Yt = smem + BK * XS;
  const int lin = xcd_tile(bid, nblk);
  const int tile = lin / jb.splits, split = lin % jb.splits;
  const int64_t j0 = (int64_t)tile * TB;
  const int64_t per = (jb.n + jb.splits - 1) / jb.splits;
  const int64_t rb = (int64_t)split * per;
  const int64_t re = (rb + per < jb.n) ? rb + per : jb.n;
  const float* __restrict__ X = jb.X;
  const float* __restrict__ Y = jb.Y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;

  float4 xr[XN4], yr[YN4];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < XN4; ++q) {
      const int e = tid + q * 256;
      const int row = e / (A / 4), c4 = e % (A / 4);
      xr[q] = (e < BK * A / 4 && r0 + row < re)
                  ? *reinterpret_cast<const float4*>(X + (r0 + row) * A + c4 * 4)
                  : float4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int q = 0; q < YN4; ++q) {
      const int e = tid + q * 256;
      float4 v{0.f, 0.f, 0.f, 0.f};
      if (e < BK * TB / 4) {
        if (YROW) {
          const int row = e / (TB / 4), c4 = e % (TB / 4);
          if (r0 + row < re) v = *reinterpret_cast<const float4*>(Y + (r0 + row) * jb.y_ld + j0 + c4 * 4);
        } else {
          const int j = e / (BK / 4), i4 = e % (BK / 4);
          if (r0 + i4 * 4 < re) v = *reinterpret_cast<const float4*>(Y + (j0 + j) * jb.y_ld + r0 + i4 * 4);
        }
      }
      yr[q] = v;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < XN4; ++q) {
      const int e = tid + q * 256;
      if (e < BK * A / 4) *reinterpret_cast<float4*>(Xs + (e / (A / 4)) * XS + (e % (A / 4)) * 4) = xr[q];
    }
#pragma unroll
    for (int q = 0; q < YN4; ++q) {
      const int e = tid + q * 256;
      if (e < BK * TB / 4) {
        if (YROW) {
          const int row = e / (TB / 4), c4 = e % (TB / 4);
          Yt[(c4 * 4 + 0) * YS + row] = yr[q].x;
          Yt[(c4 * 4 + 1) * YS + row] = yr[q].y;
          Yt[(c4 * 4 + 2) * YS + row] = yr[q].z;
          Yt[(c4 * 4 + 3) * YS + row] = yr[q].w;
        } else {
          const int j = e / (BK / 4), i4 = e % (BK / 4);
          *reinterpret_cast<float4*>(Yt + j * YS + i4 * 4) = yr[q];
        }
      }
    }
  };

  constexpr int IB = A / 16, JB = TB / 16;
  f32x4 acc[IB][JB];
#pragma unroll
  for (int a = 0; a < IB; ++a)
#pragma unroll
    for (int b = 0; b < JB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  if (rb < re) fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += BK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (r0 + BK < re) fetch(r0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; kk += 4) {
      const int k = wave * (BK / 4) + kk + lk;
      float bv[JB];
#pragma unroll
      for (int b = 0; b < JB; ++b) bv[b] = Yt[(b * 16 + li) * YS + k];
#pragma unroll
      for (int a = 0; a < IB; ++a) {
        const float av = Xs[k * XS + a * 16 + li];
#pragma unroll
        for (int b = 0; b < JB; ++b) acc[a][b] = mfma16(av, bv[b], acc[a][b]);
      }
    }
  }
  __syncthreads();
  float* red = smem;
#pragma unroll
  for (int a = 0; a < IB; ++a)
#pragma unroll
    for (int b = 0; b < JB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(wave * A + a * 16 + lk * 4 + r) * TB + b * 16 + li] = acc[a][b][r];
  __syncthreads();
  float* C = jb.C + (int64_t)split * jb.c_split;
  for (int e = tid; e < A * TB; e += 256) {
    const float v = red[e] + red[A * TB + e] + red[2 * A * TB + e] + red[3 * A * TB + e];
    const int i = e / TB, j = e % TB;
    C[i * jb.c_rs + (j0 + j) * jb.c_cs] = v;
  }
}

constexpr int G_TB = 32;   // column slab of the row-streamed operand (128-byte rows)
constexpr int H_TB = 16;   // rows of the column-streamed operand

// Blocks [0, nG) run job g (Y rows streamed, YROW), the rest run job h.
template <int AG, int AH>
__global__ void __launch_bounds__(256)
panel2_kernel(PanelJob g, PanelJob h) {
  constexpr int SG = AG > 0 ? PanelCfg<(AG > 0 ? AG : 16), G_TB>::SMEM_ALL : 0;
  constexpr int SH = AH > 0 ? PanelCfg<(AH > 0 ? AH : 16), H_TB>::SMEM_ALL : 0;
  __shared__ __align__(16) float smem[(SG > SH ? SG : SH) > 0 ? (SG > SH ? SG : SH) : 4];
  const int nG = AG > 0 ? g.ntiles * g.splits : 0;
  if ((int)blockIdx.x < nG) {
    if constexpr (AG > 0) panel_tile<AG, G_TB, true>(g, blockIdx.x, nG, smem);
  } else {
    if constexpr (AH > 0) panel_tile<AH, H_TB, false>(h, blockIdx.x - nG, gridDim.x - nG, smem);
  }
}

// ---- short-K output GEMM -------------------------------------------------------
constexpr int OT = 128;   // tile
constexpr int OKC = 32;   // K slab
constexpr int OAS = OKC + 4, OBS = OT + 16;

// A2 and B1 may each be the sum of `a2s` / `b1s` partial slabs (split
// reductions of the panel launch), added here in a fixed order.
struct OutJob {
  int64_t M, N;
  int K1, K2;
  const float* A1; int64_t lda1;
  const float* A2; int64_t lda2; int a2s; int64_t a2_stride;
  const float* B1; int64_t ldb1; int b1s; int64_t b1_stride;
  const float* B2; int64_t ldb2;
  float* C; int64_t ldc;
};

__device__ __forceinline__ void out_tile(const OutJob& jb, int tile, float* As, float* Bs) {
  const int64_t M = jb.M, N = jb.N;
  const int K1 = jb.K1, K2 = jb.K2;
  const float* __restrict__ A1 = jb.A1;
  const float* __restrict__ A2 = jb.A2;
  const float* __restrict__ B1 = jb.B1;
  const float* __restrict__ B2 = jb.B2;
  float* __restrict__ C = jb.C;
  const int64_t lda1 = jb.lda1, lda2 = jb.lda2, ldb1 = jb.ldb1, ldb2 = jb.ldb2, ldc = jb.ldc;
  const int a2s = jb.a2s, b1s = jb.b1s;
  const int64_t a2_stride = jb.a2_stride, b1_stride = jb.b1_stride;
  (void)M;
  const int ntn = (int)(N / OT);
  const int64_t m0 = (int64_t)(tile / ntn) * OT, n0 = (int64_t)(tile % ntn) * OT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int K = K1 + K2;

  constexpr int AN = OT * OKC / 4 / 256, BN4 = OKC * OT / 4 / 256;
  float4 ar[AN], br[BN4];
  auto add4 = [](float4 a, float4 b) { return float4{a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w}; };
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < AN; ++q) {
      const int e = tid + q * 256;
      const int row = e / (OKC / 4), k4 = e % (OKC / 4);
      const int k = k0 + k4 * 4;
      float4 v{0.f, 0.f, 0.f, 0.f};
      if (k < K1) {
        v = *reinterpret_cast<const float4*>(A1 + (m0 + row) * lda1 + k);
      } else if (k < K) {
        const float* src = A2 + (m0 + row) * lda2 + (k - K1);
        v = *reinterpret_cast<const float4*>(src);
        for (int t = 1; t < a2s; ++t) v = add4(v, *reinterpret_cast<const float4*>(src + t * a2_stride));
      }
      ar[q] = v;
    }
#pragma unroll
    for (int q = 0; q < BN4; ++q) {
      const int e = tid + q * 256;
      const int kr = e / (OT / 4), j4 = e % (OT / 4);
      const int k = k0 + kr;
      float4 v{0.f, 0.f, 0.f, 0.f};
      if (k < K1) {
        const float* src = B1 + (int64_t)k * ldb1 + n0 + j4 * 4;
        v = *reinterpret_cast<const float4*>(src);
        for (int t = 1; t < b1s; ++t) v = add4(v, *reinterpret_cast<const float4*>(src + t * b1_stride));
      } else if (k < K) {
        v = *reinterpret_cast<const float4*>(B2 + (int64_t)(k - K1) * ldb2 + n0 + j4 * 4);
      }
      br[q] = v;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < AN; ++q) {
      const int e = tid + q * 256;
      *reinterpret_cast<float4*>(As + (e / (OKC / 4)) * OAS + (e % (OKC / 4)) * 4) = ar[q];
    }
#pragma unroll
    for (int q = 0; q < BN4; ++q) {
      const int e = tid + q * 256;
      *reinterpret_cast<float4*>(Bs + (e / (OT / 4)) * OBS + (e % (OT / 4)) * 4) = br[q];
    }
  };

  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  fetch(0);
  for (int k0 = 0; k0 < K; k0 += OKC) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + OKC < K) fetch(k0 + OKC);
    const int kend = (K - k0) < OKC ? (K - k0) : OKC;
    for (int kk = 0; kk < kend; kk += 4) {
      float av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[(wm + a * 16 + li) * OAS + kk + lk];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[(kk + lk) * OBS + wn + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma16(av[a], bv[b], acc[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        C[(m0 + wm + a * 16 + lk * 4 + r) * ldc + n0 + wn + b * 16 + li] = acc[a][b][r];
}

__global__ void __launch_bounds__(256) out_kernel(OutJob jb) {
  __shared__ __align__(16) float As[OT * OAS];
  __shared__ __align__(16) float Bs[OKC * OBS];
  out_tile(jb, xcd_tile(blockIdx.x, gridDim.x), As, Bs);
}

// ---- batches: one launch covers the tiles of many products --------------------
// Block b belongs to the job j with start[j] <= b < start[j + 1] (start has
// count + 1 entries); the search is over a short table in LDS.
constexpr int MAX_BATCH = 256;

__device__ __forceinline__ int find_job(const int* __restrict__ start, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int A>
__global__ void __launch_bounds__(256)
panel_batch_kernel(const PanelJob* __restrict__ jobs, const int* __restrict__ start, int count) {
  __shared__ __align__(16) float smem[PanelCfg<A, G_TB>::SMEM_ALL];
  __shared__ int st[MAX_BATCH + 1];
  for (int i = threadIdx.x; i <= count; i += blockDim.x) st[i] = start[i];
  __syncthreads();
  const int b = blockIdx.x;
  const int j = find_job(st, count, b);
  const PanelJob jb = jobs[j];
  panel_tile<A, G_TB, true>(jb, b - st[j], st[j + 1] - st[j], smem);
}

__global__ void __launch_bounds__(256)
out_batch_kernel(const OutJob* __restrict__ jobs, const int* __restrict__ start, int count) {
  __shared__ __align__(16) float As[OT * OAS];
  __shared__ __align__(16) float Bs[OKC * OBS];
  __shared__ int st[MAX_BATCH + 1];
  for (int i = threadIdx.x; i <= count; i += blockDim.x) st[i] = start[i];
  __syncthreads();
  const int b = blockIdx.x;
  const int j = find_job(st, count, b);
  const OutJob jb = jobs[j];
  out_tile(jb, xcd_tile(b - st[j], st[j + 1] - st[j]), As, Bs);
}

template <int AG, int AH>
amm_status launch_panel2(const PanelJob& g, const PanelJob& h, hipStream_t s) {
  const int64_t nb = (AG > 0 ? (int64_t)g.ntiles * g.splits : 0) + (AH > 0 ? (int64_t)h.ntiles * h.splits : 0);
  if (nb <= 0) return AMM_OK;
  if (nb > 0x7fffffff) return fail(AMM_EUNSUPPORTED, "panel grid too large");
  TimedLaunch tl("panel", s);
  hipLaunchKernelGGL((panel2_kernel<AG, AH>), dim3((unsigned)nb), dim3(256), 0, s, g, h);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

template <int AG>
amm_status dispatch_h(int ah, const PanelJob& g, const PanelJob& h, hipStream_t s) {
  switch (ah) {
    case 0:
      if constexpr (AG == 0) return fail(AMM_EUNSUPPORTED, "empty panel");
      else return launch_panel2<AG, 0>(g, h, s);
    case 16: return launch_panel2<AG, 16>(g, h, s);
    case 32: return launch_panel2<AG, 32>(g, h, s);
    case 48: return launch_panel2<AG, 48>(g, h, s);
    case 64: return launch_panel2<AG, 64>(g, h, s);
    case 128: return launch_panel2<AG, 128>(g, h, s);
    default: return fail(AMM_EUNSUPPORTED, "panel rank %d", ah);
  }
}

amm_status dispatch_panel(int ag, int ah, const PanelJob& g, const PanelJob& h, hipStream_t s) {
  switch (ag) {
    case 0: return dispatch_h<0>(ah, g, h, s);
    case 16: return dispatch_h<16>(ah, g, h, s);
    case 32: return dispatch_h<32>(ah, g, h, s);
    case 48: return dispatch_h<48>(ah, g, h, s);
    case 64: return dispatch_h<64>(ah, g, h, s);
    case 128: return dispatch_h<128>(ah, g, h, s);
    default: return fail(AMM_EUNSUPPORTED, "panel rank %d", ag);
  }
}

int pick_splits(int64_t tiles, int64_t n) {
  // aim for >= 1024 workgroups, each reducing at least 512 rows, with split
  // boundaries on multiples of 4 rows (float4 loads never straddle a split)
  int sp = 1;
  while (sp < 4 && tiles * sp < 1024 && n / (sp * 2) >= 512 && n % (8 * sp) == 0) sp *= 2;
  return sp;
}

}  // namespace

bool tsvd_fast_shapes(int64_t m, int64_t n, int64_t p, int ka, int kb) {
  auto rank_ok = [](int k) { return k == 0 || k == 16 || k == 32 || k == 48 || k == 64 || k == 128; };
  return m % OT == 0 && p % OT == 0 && n % 4 == 0 && m > 0 && p > 0 && rank_ok(ka) && rank_ok(kb) &&
         ka + kb > 0 && ka + kb <= 256;
}

// Products of the truncated-SVD path on the fast shapes:
//   ka > 0:  G = V_A^T Y   (Y n x p; split partials in Gp, summed by the output GEMM)
//   kb > 0:  H = X U_B     (X m x n)
//   out = [US_A | H] [G ; VSt_B]
amm_status tsvd_fast_product(int64_t m, int64_t n, int64_t p, int ka, int kb, const float* V_A,
                             const float* US_A, const float* Y, const float* X, const float* U_B,
                             const float* VSt_B, float* Gp, size_t gp_floats, float* H,
                             size_t h_floats, float* out, hipStream_t s) {
  PanelJob g{}, h{};
  int gs = 1, hs = 1;
  if (ka > 0) {
    g.ntiles = (int)(p / G_TB);
    gs = pick_splits(g.ntiles, n);
    if ((size_t)gs * ka * p > gp_floats) return fail(AMM_EINVAL, "panel scratch too small");
    g = PanelJob{V_A, Y, p, n, (int)(p / G_TB), gs, Gp, p, 1, (int64_t)ka * p};
  }
  if (kb > 0) {
    const int tiles = (int)(m / H_TB);
    hs = pick_splits(tiles, n);
    if ((size_t)hs * kb * m > h_floats) return fail(AMM_EINVAL, "panel scratch too small");
    h = PanelJob{U_B, X, n, n, tiles, hs, H, 1, kb, (int64_t)kb * m};
  }
  AMM_TRY(dispatch_panel(ka, kb, g, h, s));
  const int64_t tiles = (m / OT) * (p / OT);
  if (tiles > 0x7fffffff) return fail(AMM_EUNSUPPORTED, "output too large");
  TimedLaunch tl("gemm_out", s);
  OutJob oj{m, p, ka, kb, US_A, (int64_t)ka, H, (int64_t)kb, hs, (int64_t)kb * m, Gp, p, gs,
            (int64_t)ka * p, VSt_B, p, out, p};
  hipLaunchKernelGGL(out_kernel, dim3((unsigned)tiles), dim3(256), 0, s, oj);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

int tsvd_fast_splits(int64_t tiles, int64_t n) { return pick_splits(tiles, n); }

namespace {
bool rank_supported(int a) { return a == 16 || a == 32 || a == 48 || a == 64 || a == 128; }
}

bool panel_full_ok(int a, int64_t ncols) { return rank_supported(a) && ncols % G_TB == 0 && ncols > 0; }

// C (a x ncols, row-major) = X^T Y, X n_red x a, Y n_red x ncols; one reduction split
amm_status panel_full(int a, int64_t n_red, const float* X, const float* Y, int64_t ncols, float* C,
                      hipStream_t s) {
  if (!panel_full_ok(a, ncols)) return fail(AMM_EUNSUPPORTED, "panel shape");
  PanelJob g{X, Y, ncols, n_red, (int)(ncols / G_TB), 1, C, ncols, 1, 0};
  PanelJob h{};
  return dispatch_panel(a, 0, g, h, s);
}

bool gemm_short_ok(int64_t M, int64_t N, int K) { return M % OT == 0 && N % OT == 0 && K % 4 == 0 && K > 0 && M > 0 && N > 0; }

// C (M x N) = A (M x K) B (K x N), all row-major and contiguous
amm_status gemm_short(int64_t M, int64_t N, int K, const float* A, const float* B, float* C, hipStream_t s) {
  if (!gemm_short_ok(M, N, K)) return fail(AMM_EUNSUPPORTED, "short-K GEMM shape");
  const int64_t tiles = (M / OT) * (N / OT);
  TimedLaunch tl("gemm_out", s);
  OutJob oj{M, N, K, 0, A, (int64_t)K, nullptr, 0, 1, 0, B, N, 1, 0, nullptr, 0, C, N};
  hipLaunchKernelGGL(out_kernel, dim3((unsigned)tiles), dim3(256), 0, s, oj);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}


// ---- batch plans ---------------------------------------------------------------
namespace {

template <int A>
amm_status launch_panel_batch(const PanelJob* jobs, const int* start, int count, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((panel_batch_kernel<A>), dim3((unsigned)blocks), dim3(256), 0, s, jobs, start, count);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

amm_status panel_batch(int a, const PanelJob* jobs, const int* start, int count, int blocks, hipStream_t s) {
  switch (a) {
    case 16: return launch_panel_batch<16>(jobs, start, count, blocks, s);
    case 32: return launch_panel_batch<32>(jobs, start, count, blocks, s);
    case 48: return launch_panel_batch<48>(jobs, start, count, blocks, s);
    case 64: return launch_panel_batch<64>(jobs, start, count, blocks, s);
    case 128: return launch_panel_batch<128>(jobs, start, count, blocks, s);
    default: return fail(AMM_EUNSUPPORTED, "batch rank %d", a);
  }
}

}  // namespace

amm_status batch_build(amm_batch_plan* bp, int target_blocks) {
  const int count = (int)bp->items.size();
  std::vector<PanelJob> pj(count);
  std::vector<OutJob> oj(count);
  std::vector<int> ps(count + 1, 0), os(count + 1, 0);
  std::vector<int> splits(count);
  size_t part_floats = 0;
  int64_t total_tiles = 0;
  for (auto& it : bp->items) total_tiles += it.p / G_TB;
  for (int i = 0; i < count; ++i) {
    const auto& it = bp->items[i];
    const int tiles = (int)(it.p / G_TB);
    int sp = 1;
    while (sp < 8 && total_tiles * sp * 2 <= target_blocks && it.n / (sp * 2) >= 256 && it.n % (8 * sp) == 0) sp *= 2;
    splits[i] = sp;
    part_floats += (size_t)sp * bp->k * it.p;
    ps[i + 1] = ps[i] + tiles * sp;
    os[i + 1] = os[i] + (int)((it.m / OT) * (it.p / OT));
  }
  AMM_TRY(bp->partials.reserve(part_floats * sizeof(float)));
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    const auto& it = bp->items[i];
    float* G = bp->partials.as<float>() + off;
    off += (size_t)splits[i] * bp->k * it.p;
    pj[i] = PanelJob{it.V, it.B, it.p, it.n, (int)(it.p / G_TB), splits[i], G, it.p, 1, (int64_t)bp->k * it.p};
    oj[i] = OutJob{it.m, it.p, bp->k, 0, it.US, (int64_t)bp->k, nullptr, 0, 1, 0, G, it.p, splits[i],
                   (int64_t)bp->k * it.p, nullptr, 0, it.out, it.p};
  }
  AMM_TRY(bp->tables.reserve(count * (sizeof(PanelJob) + sizeof(OutJob)) + 2 * (count + 1) * sizeof(int) + 64));
  char* base = bp->tables.as<char>();
  bp->pjobs = base;
  bp->ojobs = base + count * sizeof(PanelJob);
  bp->pstart = reinterpret_cast<int*>(base + count * (sizeof(PanelJob) + sizeof(OutJob)));
  bp->ostart = bp->pstart + count + 1;
  AMM_HIP(hipMemcpy(bp->pjobs, pj.data(), count * sizeof(PanelJob), hipMemcpyHostToDevice));
  AMM_HIP(hipMemcpy(bp->ojobs, oj.data(), count * sizeof(OutJob), hipMemcpyHostToDevice));
  AMM_HIP(hipMemcpy(bp->pstart, ps.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice));
  AMM_HIP(hipMemcpy(bp->ostart, os.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice));
  bp->panel_blocks = ps[count];
  bp->out_blocks = os[count];
  bp->splits = splits;
  bp->target_blocks = target_blocks;
  return AMM_OK;
}

amm_status batch_launch(amm_batch_plan* bp, hipStream_t s) {
  const int count = (int)bp->items.size();
  {
    TimedLaunch tl("batch_panel", s);
    AMM_TRY(panel_batch(bp->k, reinterpret_cast<const PanelJob*>(bp->pjobs), bp->pstart, count, bp->panel_blocks, s));
  }
  TimedLaunch tl("batch_out", s);
  hipLaunchKernelGGL(out_batch_kernel, dim3((unsigned)bp->out_blocks), dim3(256), 0, s,
                     reinterpret_cast<const OutJob*>(bp->ojobs), (const int*)bp->ostart, count);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

bool batch_item_ok(int64_t m, int64_t n, int64_t p, int k) {
  return tsvd_fast_shapes(m, n, p, k, 0) && p % G_TB == 0 && k > 0;
}

int batch_max_items() { return MAX_BATCH; }

}  // namespace amm
