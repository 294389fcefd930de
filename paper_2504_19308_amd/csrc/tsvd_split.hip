// Truncated-SVD products (Sec. 2.2 of the paper) on the fast shapes:
//
//   zeroth order  out = U_A S_A (V_A^T B)
//   first order   out = U_A S_A (V_A^T Delta B) + (A U_B)(S_B V_B^T)
//
// in three launches:
//   panels   G = V_A^T Y (k_A x p) and H = X U_B (m x k_B), Y = B or Delta B,
//            X = A, float32 matrix cores, the large operands streamed once
//            straight into MFMA registers;
//   reduce   the split partial sums of G and H, in a fixed order;
//   output   out = [U_A S_A | H] [G ; S_B V_B^T] with a short inner dimension
//            (k_A + k_B <= 128), on the bfloat16 matrix cores with every
//            float32 operand split into three bfloat16 parts
//            x = hi + mid + lo (each part the rounding of what is left); the
//            six products hi*hi, hi*mid, mid*hi, hi*lo, lo*hi, mid*mid carry
//            every term above 2^-24 relative, so the result has float32
//            accuracy (products accumulate in float32).
//
// Panel layouts.  v_mfma_f32_16x16x4f32 takes a[k = l/16][i = l%16] and
// b[k = l/16][j = l%16].  G job: lane (g, t) = (l/16, l%16) loads the float4
// Y[r + g][j0 + 4t .. 4t+3]; component s is the B operand of MFMA s, whose
// columns are j0 + 4t + s, so the four MFMAs cover 64 columns per wave.  H job:
// lane (g, t) loads X[row0 + 16b + t][c + 4g .. 4g+3]; component s is the A
// operand of MFMA s with reduction index c + 4g + s.  The four waves of a
// workgroup split its reduction range and meet in LDS; workgroups split the
// reduction S ways and leave S partials.
#include <map>
#include <mutex>

#include "amm_internal.hpp"

namespace amm {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int xcd_order(int bid, int nblk) {
  if (nblk % 8) return bid;
  return (bid % 8) * (nblk / 8) + bid / 8;
}

constexpr int PW = 4;    // waves per panel workgroup

// Load batch of a panel wave: DG 4-row groups (G job) or DH 16-column groups
// (H job).  The plain form loads a batch and multiplies it; the deep form
// keeps three batches in registers and issues a batch's loads two batches
// before its MFMAs (software pipeline), trading occupancy for loads in flight;
// it is used for ranks 32.
constexpr int DG = 4, DH = 2;

// G (as Gt, p x KA) partial of split `split`: rows [split*per*PW, ...) of Y
template <int KA, bool DEEP>
__device__ __forceinline__ void g_job(const float* __restrict__ X, const float* __restrict__ Y, int64_t p,
                                      int64_t n, int S, float* __restrict__ Gt, int bid, int nblk, float* red) {
  constexpr int IB = KA / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = lane & 15, g = lane >> 4;
  const int ncb = (int)(p / 64);
  const int b = xcd_order(bid, nblk);
  const int cb = b % ncb, split = b / ncb;
  const int64_t j0 = (int64_t)cb * 64;
  const int64_t per = n / ((int64_t)S * PW);
  const int64_t rb = ((int64_t)split * PW + wave) * per, re = rb + per;
  f32x4 acc[IB][4];
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[i][q] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto load = [&](int64_t r, float4(&y)[DG], float(&xv)[DG][IB]) {
#pragma unroll
    for (int d = 0; d < DG; ++d) {
      const int64_t row = r + 4 * d + g;
      y[d] = *reinterpret_cast<const float4*>(Y + row * p + j0 + 4 * t);
#pragma unroll
      for (int i = 0; i < IB; ++i) xv[d][i] = X[row * KA + i * 16 + t];
    }
  };
  auto comp = [&](const float4(&y)[DG], const float(&xv)[DG][IB]) {
#pragma unroll
    for (int d = 0; d < DG; ++d)
#pragma unroll
      for (int i = 0; i < IB; ++i) {
        acc[i][0] = mfma_f32(xv[d][i], y[d].x, acc[i][0]);
        acc[i][1] = mfma_f32(xv[d][i], y[d].y, acc[i][1]);
        acc[i][2] = mfma_f32(xv[d][i], y[d].z, acc[i][2]);
        acc[i][3] = mfma_f32(xv[d][i], y[d].w, acc[i][3]);
      }
  };
  constexpr int STEP = 4 * DG;
  if constexpr (!DEEP) {
    for (int64_t r = rb; r < re; r += STEP) {
      float4 y[DG];
      float xv[DG][IB];
      load(r, y, xv);
      comp(y, xv);
    }
  } else {
    // batches b = 0, 1, ... of STEP rows (per is a multiple of STEP) rotate
    // through three register sets; batches b + 1 and b + 2 are in flight
    // while batch b is multiplied
    const int64_t nb = per / STEP;
    float4 y0[DG], y1[DG], y2[DG];
    float x0[DG][IB], x1[DG][IB], x2[DG][IB];
    load(rb, y0, x0);
    if (nb > 1) load(rb + STEP, y1, x1);
    for (int64_t b = 0; b < nb; b += 3) {
      if (b + 2 < nb) load(rb + (b + 2) * STEP, y2, x2);
      comp(y0, x0);
      if (b + 3 < nb) load(rb + (b + 3) * STEP, y0, x0);
      if (b + 1 < nb) comp(y1, x1);
      if (b + 4 < nb) load(rb + (b + 4) * STEP, y1, x1);
      if (b + 2 < nb) comp(y2, x2);
    }
  }
  // lane: acc[i][q][rr] = G[16i + 4g + rr][j0 + 4t + q]
  if (wave > 0) {
#pragma unroll
    for (int i = 0; i < IB; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<float4*>(red + ((wave - 1) * 64 + 4 * t + q) * KA + 16 * i + 4 * g) =
            float4{acc[i][q][0], acc[i][q][1], acc[i][q][2], acc[i][q][3]};
  }
  __syncthreads();
  if (wave > 0) return;
  float* dst = Gt + (int64_t)split * p * KA;
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float4 v{acc[i][q][0], acc[i][q][1], acc[i][q][2], acc[i][q][3]};
      for (int w = 1; w < PW; ++w) {
        const float4 o = *reinterpret_cast<const float4*>(red + ((w - 1) * 64 + 4 * t + q) * KA + 16 * i + 4 * g);
        v = float4{v.x + o.x, v.y + o.y, v.z + o.z, v.w + o.w};
      }
      *reinterpret_cast<float4*>(dst + (j0 + 4 * t + q) * KA + 16 * i + 4 * g) = v;
    }
}

// H (m x KB) partial of split `split`: columns [split*per*PW, ...) of X
template <int KB, bool DEEP>
__device__ __forceinline__ void h_job(const float* __restrict__ U, const float* __restrict__ X, int64_t m,
                                      int64_t n, int S, float* __restrict__ H, int bid, int nblk, float* red) {
  constexpr int CB = KB / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = lane & 15, g = lane >> 4;
  const int nrb = (int)(m / 64);
  const int b = xcd_order(bid, nblk);
  const int rbk = b % nrb, split = b / nrb;
  const int64_t row0 = (int64_t)rbk * 64;
  const int64_t per = n / ((int64_t)S * PW);
  const int64_t c0s = ((int64_t)split * PW + wave) * per, ce = c0s + per;
  f32x4 acc[4][CB];
#pragma unroll
  for (int bb = 0; bb < 4; ++bb)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[bb][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto load = [&](int64_t c0, float4(&a)[DH][4], float(&u)[DH][4][CB]) {
#pragma unroll
    for (int d = 0; d < DH; ++d) {
      const int64_t cc = c0 + 16 * d + 4 * g;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) a[d][bb] = *reinterpret_cast<const float4*>(X + (row0 + 16 * bb + t) * n + cc);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < CB; ++c) u[d][q][c] = U[(cc + q) * KB + c * 16 + t];
    }
  };
  auto comp = [&](const float4(&a)[DH][4], const float(&u)[DH][4][CB]) {
#pragma unroll
    for (int d = 0; d < DH; ++d)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          acc[bb][c] = mfma_f32(a[d][bb].x, u[d][0][c], acc[bb][c]);
          acc[bb][c] = mfma_f32(a[d][bb].y, u[d][1][c], acc[bb][c]);
          acc[bb][c] = mfma_f32(a[d][bb].z, u[d][2][c], acc[bb][c]);
          acc[bb][c] = mfma_f32(a[d][bb].w, u[d][3][c], acc[bb][c]);
        }
  };
  constexpr int STEP = 16 * DH;
  if constexpr (!DEEP) {
    for (int64_t c0 = c0s; c0 < ce; c0 += STEP) {
      float4 a[DH][4];
      float u[DH][4][CB];
      load(c0, a, u);
      comp(a, u);
    }
  } else {
    const int64_t nb = per / STEP;
    float4 a0[DH][4], a1[DH][4], a2[DH][4];
    float u0[DH][4][CB], u1[DH][4][CB], u2[DH][4][CB];
    load(c0s, a0, u0);
    if (nb > 1) load(c0s + STEP, a1, u1);
    for (int64_t b = 0; b < nb; b += 3) {
      if (b + 2 < nb) load(c0s + (b + 2) * STEP, a2, u2);
      comp(a0, u0);
      if (b + 3 < nb) load(c0s + (b + 3) * STEP, a0, u0);
      if (b + 1 < nb) comp(a1, u1);
      if (b + 4 < nb) load(c0s + (b + 4) * STEP, a1, u1);
      if (b + 2 < nb) comp(a2, u2);
    }
  }
  // lane: acc[bb][c][rr] = H[row0 + 16bb + 4g + rr][16c + t]
  if (wave > 0) {
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) red[((wave - 1) * 64 + 16 * bb + 4 * g + rr) * KB + 16 * c + t] = acc[bb][c][rr];
  }
  __syncthreads();
  if (wave > 0) return;
  float* dst = H + (int64_t)split * m * KB;
#pragma unroll
  for (int bb = 0; bb < 4; ++bb)
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        float v = acc[bb][c][rr];
        for (int w = 1; w < PW; ++w) v += red[((w - 1) * 64 + 16 * bb + 4 * g + rr) * KB + 16 * c + t];
        dst[(row0 + 16 * bb + 4 * g + rr) * KB + 16 * c + t] = v;
      }
}

struct PanelArgs {
  const float* VA;   // n x KA
  const float* Y;    // n x p
  const float* UB;   // n x KB
  const float* X;    // m x n
  int64_t m, n, p;
  int SG, SH;
  float* Gt;         // SG x (p x KA)
  float* H;          // SH x (m x KB)
};

template <int KA, int KB, bool DEEP>
__global__ void __launch_bounds__(256) split_panels_kernel(PanelArgs a) {
  constexpr int KM = KA > KB ? KA : KB;
  __shared__ __align__(16) float red[(PW - 1) * 64 * KM];
  const int nG = (int)(a.p / 64) * a.SG;
  if ((int)blockIdx.x < nG) g_job<KA, DEEP>(a.VA, a.Y, a.p, a.n, a.SG, a.Gt, blockIdx.x, nG, red);
  else if constexpr (KB > 0) h_job<KB, DEEP>(a.UB, a.X, a.m, a.n, a.SH, a.H, blockIdx.x - nG, gridDim.x - nG, red);
}

// sum S partial slabs of `count` floats (fixed order); two regions per launch
__global__ void split_reduce_kernel(const float* __restrict__ g_src, int gs, int64_t g_count, float* __restrict__ g_dst,
                                    const float* __restrict__ h_src, int hs, int64_t h_count, float* __restrict__ h_dst) {
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  const float* src;
  float* dst;
  int S;
  int64_t count;
  if (i < g_count) {
    src = g_src; dst = g_dst; S = gs; count = g_count;
  } else {
    i -= g_count;
    if (i >= h_count) return;
    src = h_src; dst = h_dst; S = hs; count = h_count;
  }
  float4 v = *reinterpret_cast<const float4*>(src + i);
  for (int s = 1; s < S; ++s) {
    const float4 w = *reinterpret_cast<const float4*>(src + s * count + i);
    v = float4{v.x + w.x, v.y + w.y, v.z + w.z, v.w + w.w};
  }
  *reinterpret_cast<float4*>(dst + i) = v;
}

// ---- output: C (M x N) = [A1 | A2] [B1 | B2]^T, operands k-contiguous float32 --------
constexpr int OT = 128;   // output tile
constexpr int KC = 32;    // inner chunk
constexpr int LS = 40;    // LDS row stride (bf16): 16-byte aligned rows, conflict-free 16-byte reads

__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  const float r1 = x - (float)h;
  m = (__bf16)r1;
  l = (__bf16)(r1 - (float)m);
}

union B4 {
  uint2 v;
  __bf16 e[4];
};

template <int K1, int K2>
__global__ void __launch_bounds__(256)
split_out_kernel(const float* __restrict__ A1, const float* __restrict__ A2, const float* __restrict__ B1,
                 const float* __restrict__ B2, int64_t M, int64_t N, float* __restrict__ C) {
  constexpr int NCH = (K1 + K2) / KC;
  __shared__ __align__(16) __bf16 As[3][OT * LS];
  __shared__ __align__(16) __bf16 Bs[3][OT * LS];
  const int ntn = (int)(N / OT);
  const int tile = xcd_order(blockIdx.x, gridDim.x);
  const int64_t m0 = (int64_t)(tile / ntn) * OT, n0 = (int64_t)(tile % ntn) * OT;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, li = lane & 15, lg = lane >> 4;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x4 acc[4][4];   // [column block][row block], computed transposed
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  float4 ar[4], br[4];
  auto fetch = [&](int ch) {
    const int k0 = ch * KC;
    const bool first = k0 < K1;
    const float* Ap = first ? A1 : A2;
    const float* Bp = first ? B1 : B2;
    const int ld = first ? K1 : K2;
    const int kk = first ? k0 : k0 - K1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;   // 128 rows x 8 float4
      ar[q] = *reinterpret_cast<const float4*>(Ap + (m0 + (e >> 3)) * ld + kk + 4 * (e & 7));
      br[q] = *reinterpret_cast<const float4*>(Bp + (n0 + (e >> 3)) * ld + kk + 4 * (e & 7));
    }
  };
  auto stash = [&](float4 v, __bf16 (*dst)[OT * LS], int e) {
    B4 h, m, l;
    split3(v.x, h.e[0], m.e[0], l.e[0]);
    split3(v.y, h.e[1], m.e[1], l.e[1]);
    split3(v.z, h.e[2], m.e[2], l.e[2]);
    split3(v.w, h.e[3], m.e[3], l.e[3]);
    const int off = (e >> 3) * LS + 4 * (e & 7);
    *reinterpret_cast<uint2*>(&dst[0][off]) = h.v;
    *reinterpret_cast<uint2*>(&dst[1][off]) = m.v;
    *reinterpret_cast<uint2*>(&dst[2][off]) = l.v;
  };
  fetch(0);
#pragma unroll 1
  for (int ch = 0; ch < NCH; ++ch) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      stash(ar[q], As, t + 256 * q);
      stash(br[q], Bs, t + 256 * q);
    }
    __syncthreads();
    if (ch + 1 < NCH) fetch(ch + 1);
    bf16x8 u[3][4];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) u[s][rb] = *reinterpret_cast<const bf16x8*>(&As[s][(wm + 16 * rb + li) * LS + 8 * lg]);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      bf16x8 g[3];
#pragma unroll
      for (int s = 0; s < 3; ++s) g[s] = *reinterpret_cast<const bf16x8*>(&Bs[s][(wn + 16 * cb + li) * LS + 8 * lg]);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        f32x4 c = acc[cb][rb];
        c = mfma_bf16(g[1], u[1][rb], c);   // smallest terms first
        c = mfma_bf16(g[2], u[0][rb], c);
        c = mfma_bf16(g[0], u[2][rb], c);
        c = mfma_bf16(g[1], u[0][rb], c);
        c = mfma_bf16(g[0], u[1][rb], c);
        c = mfma_bf16(g[0], u[0][rb], c);
        acc[cb][rb] = c;
      }
    }
  }
  // lane holds C[m0 + wm + 16 rb + li][n0 + wn + 16 cb + 4 lg + r]
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
      *reinterpret_cast<float4*>(C + (m0 + wm + 16 * rb + li) * N + n0 + wn + 16 * cb + 4 * lg) =
          float4{acc[cb][rb][0], acc[cb][rb][1], acc[cb][rb][2], acc[cb][rb][3]};
}

// largest S in {8, 4, 2, 1} keeping about `target` workgroups and whole load batches per wave
int pick_s(int64_t blocks1, int64_t n, int quantum, int target) {
  int S = 8;
  while (S > 1 && (blocks1 * S > 2 * target || n % ((int64_t)S * PW * quantum) != 0)) S /= 2;
  return S;
}

template <int KA, int KB>
amm_status launch_panels(const PanelArgs& a, bool deep, hipStream_t s) {
  const int64_t blocks = (a.p / 64) * a.SG + (KB > 0 ? (a.m / 64) * a.SH : 0);
  TimedLaunch tl("panel", s);
  if constexpr (KA == 32 && KB <= 32) {
    if (deep) {
      hipLaunchKernelGGL((split_panels_kernel<KA, KB, true>), dim3((unsigned)blocks), dim3(256), 0, s, a);
      AMM_HIP(hipGetLastError());
      return AMM_OK;
    }
  }
  hipLaunchKernelGGL((split_panels_kernel<KA, KB, false>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

template <int K1, int K2>
amm_status launch_out(const float* A1, const float* A2, const float* B1, const float* B2, int64_t M, int64_t N,
                      float* C, hipStream_t s) {
  TimedLaunch tl("gemm_out", s);
  hipLaunchKernelGGL((split_out_kernel<K1, K2>), dim3((unsigned)((M / OT) * (N / OT))), dim3(256), 0, s, A1, A2, B1,
                     B2, M, N, C);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

amm_status dispatch_panels(int ka, int kb, const PanelArgs& a, bool deep, hipStream_t s) {
#define AMM_P(A, B) \
  if (ka == A && kb == B) return launch_panels<A, B>(a, deep, s);
  AMM_P(32, 0) AMM_P(64, 0) AMM_P(32, 32) AMM_P(32, 64) AMM_P(64, 32) AMM_P(64, 64) AMM_P(128, 0) AMM_P(128, 128)
#undef AMM_P
  return fail(AMM_EUNSUPPORTED, "split panel ranks %d, %d", ka, kb);
}

amm_status dispatch_out(int k1, int k2, const float* A1, const float* A2, const float* B1, const float* B2,
                        int64_t M, int64_t N, float* C, hipStream_t s) {
#define AMM_O(X, Y) \
  if (k1 == X && k2 == Y) return launch_out<X, Y>(A1, A2, B1, B2, M, N, C, s);
  AMM_O(32, 0) AMM_O(64, 0) AMM_O(32, 32) AMM_O(32, 64) AMM_O(64, 32) AMM_O(64, 64) AMM_O(128, 0) AMM_O(128, 128)
#undef AMM_O
  return fail(AMM_EUNSUPPORTED, "split output ranks %d, %d", k1, k2);
}

// deep (pipelined) panels for rank-32 operands when the reduction length splits
// into whole deep batches; they want fewer, longer workgroups
bool use_deep(int64_t n, int ka, int kb) {
  return ka == 32 && kb <= 32 && n % (PW * 16 * DH) == 0 && n % (PW * 4 * DG) == 0;
}

void plan_splits(int64_t m, int64_t n, int64_t p, int ka, int kb, int* SG, int* SH, bool* deep) {
  *deep = use_deep(n, ka, kb);
  // deep panels: about one workgroup per CU in total (the G and H jobs of a
  // first-order product side by side), each wave with three batches of loads
  // in flight; doubling the splits measured slower (more partial traffic,
  // shorter pipelines)
  const int target = *deep ? (kb > 0 ? 64 : 128) : 512;
  const int qg = 4 * DG, qh = 16 * DH;
  *SG = pick_s(p / 64, n, qg, target);
  *SH = kb > 0 ? pick_s(m / 64, n, qh, target) : 1;
}

}  // namespace

bool tsvd_split_shapes(int64_t m, int64_t n, int64_t p, int ka, int kb) {
  const bool ranks = ((ka == 32 || ka == 64) && (kb == 0 || kb == 32 || kb == 64)) ||
                     (ka == 128 && (kb == 0 || kb == 128));
  return ranks && m > 0 && p > 0 && m % OT == 0 &&
         p % OT == 0 && n % (PW * 16 * DH) == 0 && n % (PW * 4 * DG) == 0 && n > 0 &&
         (m / OT) * (p / OT) < ((int64_t)1 << 31);
}

// ---- fixed device scratch for callers that cannot allocate -------------------
// One array per device, for the whole process: the split partials and the
// reduced G and H of amm_approx_matmul_static.  In host code `scratch` names a
// host-side stand-in, never the device memory: the device address comes from
// hipGetSymbolAddress, looked up once per device (with that device current)
// when a context is created there, and only that pointer reaches the kernels.
static __device__ __align__(256) float scratch[kStaticScratchFloats];

namespace {
std::mutex g_static_mtx;
std::map<int, std::pair<hipError_t, float*>> g_static;   // device -> (lookup status, address)
}  // namespace

void static_scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_static_mtx);
  if (g_static.count(device)) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_static[device] = {e, e == hipSuccess ? static_cast<float*>(ptr) : nullptr};
}

amm_status static_scratch(int device, float** out) {
  std::lock_guard<std::mutex> lk(g_static_mtx);
  const auto it = g_static.find(device);
  if (it == g_static.end()) return fail(AMM_ESTATE, "no context was created on device %d", device);
  if (it->second.first != hipSuccess) return hip_fail(it->second.first, "hipGetSymbolAddress(scratch)");
  *out = it->second.second;
  return AMM_OK;
}

size_t tsvd_split_scratch(int64_t m, int64_t n, int64_t p, int ka, int kb) {
  int SG, SH;
  bool deep;
  plan_splits(m, n, p, ka, kb, &SG, &SH, &deep);
  return (size_t)(SG + 1) * ka * p + (size_t)(SH + 1) * kb * m + 64;
}

// out = US_A (V_A^T Y)        (kb == 0)
// out = US_A (V_A^T Y) + (X U_B) VS_B^T
// V_A n x ka, US_A m x ka, Y n x p, X m x n, U_B n x kb, VS_B p x kb; scratch as sized above
amm_status tsvd_split_product(int64_t m, int64_t n, int64_t p, int ka, int kb, const float* V_A, const float* US_A,
                              const float* Y, const float* X, const float* U_B, const float* VS_B, float* scratch,
                              size_t scratch_floats, float* out, hipStream_t s) {
  if (!tsvd_split_shapes(m, n, p, ka, kb)) return fail(AMM_EUNSUPPORTED, "split product shape");
  if (scratch_floats < tsvd_split_scratch(m, n, p, ka, kb)) return fail(AMM_EINVAL, "split product scratch too small");
  PanelArgs a{};
  bool deep;
  plan_splits(m, n, p, ka, kb, &a.SG, &a.SH, &deep);
  a.VA = V_A; a.Y = Y; a.UB = U_B; a.X = X;
  a.m = m; a.n = n; a.p = p;
  float* Gp = scratch;
  float* Hp = Gp + (size_t)a.SG * ka * p;
  float* G = Hp + (size_t)a.SH * kb * m;
  float* H = G + (size_t)ka * p;
  a.Gt = a.SG > 1 ? Gp : G;
  a.H = a.SH > 1 ? Hp : H;
  AMM_TRY(dispatch_panels(ka, kb, a, deep, s));
  const int64_t gc = a.SG > 1 ? (int64_t)ka * p : 0, hc = (kb > 0 && a.SH > 1) ? (int64_t)kb * m : 0;
  if (gc + hc > 0) {
    TimedLaunch tl("reduce", s);
    const int64_t quads = (gc + hc) / 4;
    hipLaunchKernelGGL(split_reduce_kernel, dim3((unsigned)((quads + 255) / 256)), dim3(256), 0, s, Gp, a.SG, gc, G,
                       Hp, a.SH, hc, H);
    AMM_HIP(hipGetLastError());
  }
  return dispatch_out(ka, kb, US_A, H, G, VS_B, m, p, out, s);
}

}  // namespace amm
