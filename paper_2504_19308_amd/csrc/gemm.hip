// Dense GEMM on the CDNA matrix cores, for the truncated-SVD factor products
// (Sec. 2.2: U (S (V^T B)), and the first-order factor products) and for the
// float64 randomized SVD (Alg. 2.1).
//
//   C[M x N] = alpha * A[M x K] B[K x N] + beta * C
//
// A and B are strided views (element (i,j) at p[i*rs + j*cs]) so transposed
// factors need no copies.  Block tile BM x BN x 16 with 256 threads: four
// waves in a 2 x 2 grid, each owning a (BM/2) x (BN/2) patch of 16 x 16
// v_mfma_*_16x16x4 tiles.  Operand tiles are staged through LDS k-major so
// that the per-lane MFMA operand reads are unit stride across lanes.  The next
// K-slab is fetched into registers while the current one is multiplied.
// Split-K (gridDim.z > 1) writes alpha-scaled partial sums to a workspace that
// a second kernel reduces in a fixed order (deterministic, no atomics).
#include "amm_internal.hpp"

namespace amm {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using acc_t = f32x4;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  using acc_t = f64x4;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// k-slab depth: 16 float32 or 32 float64 values (64 B rows of a slab either way)
template <typename T>
constexpr int kBK = sizeof(T) == 8 ? 32 : 16;
constexpr int NT = 256;

// BM, BN in {32, 64, 128}; each wave: (BM/2) x (BN/2) = TM x TN MFMA tiles.
template <typename T, int BM, int BN>
__global__ void __launch_bounds__(NT)
gemm_kernel(int64_t M, int64_t N, int64_t K, T alpha, const T* __restrict__ A, int64_t a_rs,
            int64_t a_cs, const T* __restrict__ B, int64_t b_rs, int64_t b_cs, T beta,
            T* __restrict__ C, int64_t ldc, int64_t k_split, T* __restrict__ part) {
  constexpr int BK = kBK<T>;
  constexpr int TM = BM / 32, TN = BN / 32;
  constexpr int APT = BM * BK / NT;  // A elements per thread per slab
  constexpr int BPT = BN * BK / NT;
  constexpr int PAD = sizeof(T) == 4 ? 16 : 8;   // spreads the 4 k-rows of an MFMA read over banks
  __shared__ T As[BK][BM + PAD];
  __shared__ T Bs[BK][BN + PAD];

  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * k_split;
  const int64_t kend = (kbeg + k_split < K) ? kbeg + k_split : K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);

  // Loader mapping: choose the contiguous direction of each operand so that
  // neighbouring threads read neighbouring addresses.
  const bool a_kfast = (a_cs == 1);
  const bool b_nfast = (b_cs == 1) || (b_rs != 1);

  T ra[APT], rb[BPT];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < APT; ++e) {
      const int idx = tid + e * NT;
      int i, k;
      if (a_kfast) { k = idx % BK; i = idx / BK; } else { i = idx % BM; k = idx / BM; }
      const int64_t gi = m0 + i, gk = k0 + k;
      ra[e] = (gi < M && gk < kend) ? A[gi * a_rs + gk * a_cs] : T(0);
    }
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
      const int idx = tid + e * NT;
      int j, k;
      if (b_nfast) { j = idx % BN; k = idx / BN; } else { k = idx % BK; j = idx / BK; }
      const int64_t gj = n0 + j, gk = k0 + k;
      rb[e] = (gj < N && gk < kend) ? B[gk * b_rs + gj * b_cs] : T(0);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < APT; ++e) {
      const int idx = tid + e * NT;
      int i, k;
      if (a_kfast) { k = idx % BK; i = idx / BK; } else { i = idx % BM; k = idx / BM; }
      As[k][i] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
      const int idx = tid + e * NT;
      int j, k;
      if (b_nfast) { j = idx % BN; k = idx / BN; } else { k = idx % BK; j = idx / BK; }
      Bs[k][j] = rb[e];
    }
  };

  using acc_t = typename Mfma<T>::acc_t;
  acc_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  const int li = lane & 15, lk = lane >> 4;
  if (kbeg < kend) fetch(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[kk + lk][wm + a * 16 + li];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = Bs[kk + lk][wn + b * 16 + li];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = Mfma<T>::op(av[a], bv[b], acc[a][b]);
    }
  }

  // D layout, lane l, element r, col l%16:  f32 16x16x4 -> row 4*(l/16) + r;
  // f64 16x16x4 -> row 4*r + l/16 (checked on gfx950 with a lane probe)
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = m0 + wm + a * 16 + (sizeof(T) == 4 ? lk * 4 + r : r * 4 + lk);
        const int64_t gj = n0 + wn + b * 16 + li;
        if (gi < M && gj < N) {
          const T v = alpha * acc[a][b][r];
          if (part) {
            part[(int64_t)blockIdx.z * M * N + gi * N + gj] = v;
          } else {
            T* c = C + gi * ldc + gj;
            *c = (beta == T(0)) ? v : v + beta * *c;
          }
        }
      }
}

template <typename T>
__global__ void splitk_reduce(int64_t M, int64_t N, int splits, const T* __restrict__ part,
                              T beta, T* __restrict__ C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t i = idx / N, j = idx % N;
  // eight partials' loads in flight at a time (a plain loop waits for each)
  T s = 0;
  int z = 0;
  for (; z + 8 <= splits; z += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(z + u) * M * N + idx];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; z < splits; ++z) s += part[(int64_t)z * M * N + idx];
  T* c = C + i * ldc + j;
  *c = (beta == T(0)) ? s : s + beta * *c;
}

// Split-K workspace: the calling context's grow-only area.  Every library
// entry point that multiplies sets it, so a GEMM outside a context call is an
// internal error rather than a shared buffer that two contexts' streams could
// race on.
amm_status part_ws(DevBuf** ws) {
  if (!g_gemm_part) return fail(AMM_EINVAL, "internal: split-K GEMM outside a context call");
  *ws = g_gemm_part;
  return AMM_OK;
}

template <typename T>
amm_status gemm_any(int64_t M, int64_t N, int64_t K, T alpha, const T* A, int64_t a_rs,
                    int64_t a_cs, const T* B, int64_t b_rs, int64_t b_cs, T beta, T* C,
                    int64_t ldc, hipStream_t s, const char* tag) {
  if (M <= 0 || N <= 0) return AMM_OK;
  if (K <= 0) {
    // C = beta C
    if (beta == T(1)) return AMM_OK;
    return fail(AMM_EUNSUPPORTED, "gemm with K = 0 and beta != 1");
  }
  // tile shape: small output dimension -> narrow tiles
  int BM = 64, BN = 64;
  if (M <= 32) BM = 32;
  if (N <= 32) BN = 32;
  if (sizeof(T) == 4 && M >= 1024 && N >= 1024) { BM = 128; BN = 128; }
  const int64_t gm = (M + BM - 1) / BM, gn = (N + BN - 1) / BN;
  // split K when the output grid cannot fill the chip
  int64_t splits = 1;
  const int64_t target = 1024;
  constexpr int BK = kBK<T>;
  if (gm * gn < target && K >= 512) {
    splits = (target + gm * gn - 1) / (gm * gn);
    // float64: down to two slabs per split (small outputs such as an l x l
    // Gram matrix are latency-bound); float32: at least 256 per split
    const int64_t maxs = sizeof(T) == 8 ? K / (2 * BK) : K / 256;
    if (splits > maxs) splits = maxs;
    if (splits < 1) splits = 1;
  }
  int64_t k_split = (K + splits - 1) / splits;
  k_split = ((k_split + BK - 1) / BK) * BK;
  splits = (K + k_split - 1) / k_split;
  T* part = nullptr;
  if (splits > 1) {
    DevBuf* ws = nullptr;
    AMM_TRY(part_ws(&ws));
    AMM_TRY(ws->reserve((size_t)splits * M * N * sizeof(T)));
    part = ws->as<T>();
  }
  if (gm > 65535 || splits > 65535) return fail(AMM_EUNSUPPORTED, "gemm grid too large");
  dim3 grid((unsigned)gn, (unsigned)gm, (unsigned)splits), block(NT);
  {
  TimedLaunch tl(tag, s);
#define AMM_GEMM_LAUNCH(bm, bn)                                                                \
  hipLaunchKernelGGL((gemm_kernel<T, bm, bn>), grid, block, 0, s, M, N, K, alpha, A, a_rs,  \
                     a_cs, B, b_rs, b_cs, beta, C, ldc, k_split, part)
  if (BM == 128 && BN == 128) AMM_GEMM_LAUNCH(128, 128);
  else if (BM == 64 && BN == 64) AMM_GEMM_LAUNCH(64, 64);
  else if (BM == 32 && BN == 64) AMM_GEMM_LAUNCH(32, 64);
  else if (BM == 64 && BN == 32) AMM_GEMM_LAUNCH(64, 32);
  else AMM_GEMM_LAUNCH(32, 32);
#undef AMM_GEMM_LAUNCH
  }
  AMM_HIP(hipGetLastError());
  if (splits > 1) {
    const int64_t tot = M * N;
    TimedLaunch tl("splitk_reduce", s);
    hipLaunchKernelGGL((splitk_reduce<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       M, N, (int)splits, part, beta, C, ldc);
    AMM_HIP(hipGetLastError());
  }
  return AMM_OK;
}

}  // namespace

amm_status gemm_f32(int64_t M, int64_t N, int64_t Kd, float alpha, MatView A, MatView B,
                    float beta, float* C, int64_t ldc, hipStream_t s, const char* tag) {
  return gemm_any<float>(M, N, Kd, alpha, A.p, A.rs, A.cs, B.p, B.rs, B.cs, beta, C, ldc, s, tag);
}

amm_status gemm_f64(int64_t M, int64_t N, int64_t Kd, double alpha, const double* A,
                    int64_t a_rs, int64_t a_cs, const double* B, int64_t b_rs, int64_t b_cs,
                    double beta, double* C, int64_t ldc, hipStream_t s) {
  return gemm_any<double>(M, N, Kd, alpha, A, a_rs, a_cs, B, b_rs, b_cs, beta, C, ldc, s, "gemm_f64");
}

}  // namespace amm
