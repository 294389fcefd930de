// Circulant-component product, fused in one kernel per column tile.
//
// Alg. 2.3 step 5 with the shift trick of Sec. 2.3.2:
//   Atil b = F^-1 ( sum_t  diag(L_t) C^{k_t} F b ),   (C^k X)[p] = X[(p-k) mod n],
// so each operand column needs one forward FFT, K complex multiply-adds per
// frequency bin and one inverse FFT.  Atil is real (frequency set closed
// under k -> n-k), hence complex-linear on complex vectors: two real columns
// b1, b2 are packed as b1 + i b2, transformed together, and the real and
// imaginary parts of the result are Atil b1 and Atil b2.
//
// One workgroup owns C packed columns (2C real columns) and keeps their whole
// spectra in LDS (layout [bin][col], one padding slot per 16 bins):
//   load tile -> forward Stockham stages -> shifted MAC into registers ->
//   inverse stages -> store (1/n folded in).
// Row mode is the same pipeline applied to pairs of rows of X, used for the
// first-order term  Delta A Btil = (Btil^T Delta A^T)^T, whose operator is the
// adjoint list (conj L_t[p + k_t], shift -k_t).
#include "amm_internal.hpp"
#include "fft_core.hpp"

#include <hip/hip_fp16.h>

namespace amm {
namespace {

constexpr int kH16MinLog2 = 10;   // float16 lists: n >= 1024

template <int LOG2N> struct CdCfg {
  static constexpr int N = 1 << LOG2N;
  // packed columns per workgroup.  n = 1024 and 2048 hold ~70 KiB of spectra
  // (two workgroups per CU overlap their load, transform and store phases,
  // measured faster than one 139 KiB tile); from n = 4096 up a tile fills
  // ~139 KiB (n = 16384 holds a single packed column pair).
  static constexpr int C = LOG2N <= 9 ? 16 : (LOG2N >= 12 ? (1 << (14 - LOG2N)) : (LOG2N == 10 ? 8 : 4));
  static constexpr int T = LOG2N <= 8 ? 256 : (LOG2N <= 11 ? 512 : 1024);  // threads
  static constexpr int CPL = C < 4 ? C : 4;                             // cols per MAC lane
  static constexpr int G = C / CPL;
  static constexpr int BL = T / G;                                      // MAC bin lanes
  static constexpr int NBINS = (N + BL - 1) / BL;
  static constexpr int LDS_SLOTS = (N + N / 16 + 1) * C;
  // stage twiddles W^e, e < N, as W^(e_hi 2^TWB) W^(e_lo): two LDS tables of
  // TWL and TWH entries copied from the float32 table (one product, no global
  // loads inside the transform); n <= 256 keeps the whole table
  static constexpr int TWB = LOG2N <= 8 ? LOG2N : (LOG2N + 1) / 2;
  static constexpr int TWL = 1 << TWB, TWH = N >> TWB;
};

__device__ __forceinline__ int pad_bin(int bin) { return bin + (bin >> 4); }

// LDS slot of (bin, col): the C packed columns of a bin sit together
// ([bin][col], one padding slot per 16 bins) in both modes.
template <int LOG2N, bool ROWS>
__device__ __forceinline__ int slot(int bin, int col) {
  using Cfg = CdCfg<LOG2N>;
  return pad_bin(bin) * Cfg::C + col;
}

template <int R, int SIGN, int LOG2N, int Ns, bool ROWS>
__device__ __forceinline__ void lds_stage(float2* lds, const float2* twl, const float2* twh) {
  using Cfg = CdCfg<LOG2N>;
  constexpr int N = Cfg::N, C = Cfg::C, T = Cfg::T;
  constexpr int NBF = (N / R) * C;
  constexpr int NB = (NBF + T - 1) / T;
  float2 v[NB][R];
  constexpr int twstep = N / (Ns * R);
  // Opaque copy of the thread index: keeps the compiler from hoisting every
  // stage's LDS addresses out of the kernel and holding them in registers.
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tid + i * T;
    if (NBF % T == 0 || b < NBF) {
      const int col = b % C, j = b / C;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds[slot<LOG2N, ROWS>(j + r * (N / R), col)];
      if constexpr (Ns > 1) {
        const unsigned k = (unsigned)j & (Ns - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const unsigned e = (unsigned)r * k * (unsigned)twstep;   // < N
          float2 w = twl[e & (Cfg::TWL - 1)];
          if constexpr (Cfg::TWH > 1) w = cmul(twh[e >> Cfg::TWB], w);
          if (SIGN > 0) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      dftR<R, SIGN>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tid + i * T;
    if (NBF % T == 0 || b < NBF) {
      const int col = b % C, j = b / C;
      const int k = j & (Ns - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[slot<LOG2N, ROWS>(base + r * Ns, col)] = v[i][r];
    }
  }
  __syncthreads();
}

template <int SIGN, int LOG2N, bool ROWS, int ST = 0, int Ns = 1>
__device__ __forceinline__ void lds_fft(float2* lds, const float2* twl, const float2* twh) {
  if constexpr (ST < stage_count(LOG2N)) {
    constexpr int lr = stage_log2r(LOG2N, ST);
    lds_stage<(1 << lr), SIGN, LOG2N, Ns, ROWS>(lds, twl, twh);
    lds_fft<SIGN, LOG2N, ROWS, ST + 1, (Ns << lr)>(lds, twl, twh);
  }
}

// ROWS = false: tile = real columns [2 C tile, 2 C tile + 2C) of an N x p matrix.
// ROWS = true:  tile = real rows [2 C tile, ...) of a rows x N matrix.
// SPEC = true (column mode only): store the forward spectrum of each packed
// column pair instead of the product, unscaled, in the same row-major slots
// (bin p, pair c) -> out[p * extent + 2c + {re, im}].
// H16: the eigenvalue lists are stored as float16 pairs (the spectral
// multipliers of the product in half precision); they are widened on load and
// every product and sum stays float32.
template <bool H16>
__device__ __forceinline__ float2 list_at(const void* __restrict__ L, int64_t i) {
  if constexpr (H16) return __half22float2(reinterpret_cast<const __half2*>(L)[i]);
  else return reinterpret_cast<const float2*>(L)[i];
}

template <int LOG2N, bool ROWS, bool SPEC = false, bool H16 = false>
__global__ void __launch_bounds__(CdCfg<LOG2N>::T)
cd_apply_kernel(const float* __restrict__ X, float* __restrict__ out, int64_t extent,
                int K, const int32_t* __restrict__ shifts, const void* __restrict__ L,
                const float2* __restrict__ tw, int accumulate, int vec4, CdPairs pr) {
  using Cfg = CdCfg<LOG2N>;
  constexpr int N = Cfg::N, C = Cfg::C, T = Cfg::T;
  __shared__ __align__(16) float2 lds[Cfg::LDS_SLOTS];
  __shared__ float2 twl[Cfg::TWL], twh[Cfg::TWH];
  float* ldsf = reinterpret_cast<float*>(lds);
  for (int i = threadIdx.x; i < Cfg::TWL + Cfg::TWH; i += T) {
    if (i < Cfg::TWL) twl[i] = tw[i];
    else twh[i - Cfg::TWL] = tw[(i - Cfg::TWL) << Cfg::TWB];
  }

  // XCD-aware tile order: consecutive tiles land on the same XCD so that the
  // row segments they share stay in one L2.
  const int nblk = gridDim.x;
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const int per = (nblk + 7) / 8;
  int tile = xcd * per + slot;
  if ((nblk & 7) != 0) tile = blockIdx.x;   // only remap when it is a bijection
  const int64_t first = (int64_t)tile * 2 * C;  // first real column / row

  // ---- load -----------------------------------------------------------------
  // All global loads of a thread are issued before its first LDS store.
  if (!ROWS) {
    if (2 * C >= 4 && vec4) {
      constexpr int V = 2 * C >= 4 ? 2 * C / 4 : 1;      // float4 per row
      constexpr int TOT = N * V, NL = (TOT + T - 1) / T;
      float4 r[NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int e = threadIdx.x + q * T;
        const int row = e / V, v = e % V;
        const int64_t c = first + 4 * v;
        r[q] = (e < TOT && c < extent) ? *reinterpret_cast<const float4*>(X + (int64_t)row * extent + c)
                                       : float4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int e = threadIdx.x + q * T;
        if (e < TOT) *reinterpret_cast<float4*>(&lds[pad_bin(e / V) * C + 2 * (e % V)]) = r[q];
      }
    } else {
      for (int e = threadIdx.x; e < N * 2 * C; e += T) {
        const int rc = e % (2 * C), row = e / (2 * C);
        const int64_t c = first + rc;
        ldsf[(pad_bin(row) * C + (rc >> 1)) * 2 + (rc & 1)] = c < extent ? X[(int64_t)row * extent + c] : 0.f;
      }
    }
  } else {
    for (int e = threadIdx.x; e < N * 2 * C; e += T) {
      const int q = e % N, rl = e / N;
      const int64_t r = first + rl;
      ldsf[(pad_bin(q) * C + (rl >> 1)) * 2 + (rl & 1)] = r < extent ? X[r * N + q] : 0.f;
    }
  }
  __syncthreads();

  lds_fft<-1, LOG2N, ROWS>(lds, twl, twh);

  if constexpr (!SPEC) {
  // ---- shifted spectral MAC: Y[p] = sum_t L_t[p] X[(p - k_t) mod N] ---------
  constexpr int CPL = Cfg::CPL, G = Cfg::G, BL = Cfg::BL, NBINS = Cfg::NBINS;
  // lanes = (bin, column group); the packed columns of a group are read together
  const int cg = threadIdx.x % G;
  const int bl = threadIdx.x / G;
  auto load_x = [&](int q, float2 (&x)[CPL]) {
    const float2* src = &lds[pad_bin(q & (N - 1)) * C + cg * CPL];
    if constexpr (CPL == 4) {
      const float4 x01 = reinterpret_cast<const float4*>(src)[0], x23 = reinterpret_cast<const float4*>(src)[1];
      x[0] = float2{x01.x, x01.y};
      x[1] = float2{x01.z, x01.w};
      x[2] = float2{x23.x, x23.y};
      x[3] = float2{x23.z, x23.w};
    } else if constexpr (CPL == 2) {
      const float4 x01 = reinterpret_cast<const float4*>(src)[0];
      x[0] = float2{x01.x, x01.y};
      x[1] = float2{x01.z, x01.w};
    } else {
      x[0] = src[0];
    }
  };
  auto cmac = [](float2& a, float2 l, float2 x) {
    a.x += l.x * x.x - l.y * x.y;
    a.y += l.x * x.y + l.y * x.x;
  };
  float2 acc[NBINS][CPL];
#pragma unroll
  for (int i = 0; i < NBINS; ++i)
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[i][c] = float2{0.f, 0.f};

  // Paired form (real operator, frequency set closed under k -> N-k): the list
  // of N-k is L_{N-k}[p] = conj(L_k[-p]), so one read of L_k at a bin and at
  // its mirror serves both members of the pair.  A lane then owns bin pairs
  // (b, N-b) -- b = 0 goes with the other self-mirrored bin N/2 -- and reads
  // half as many list entries.
  constexpr bool CAN_PAIR = (NBINS % 2 == 0) && (N % BL == 0);
  constexpr int NH = NBINS / 2;
  const bool paired = CAN_PAIR && pr.npairs >= 0;
  auto pair_bins = [&](int i, int& b1, int& b2) {
    b1 = bl + i * BL;
    b2 = b1 == 0 ? N / 2 : N - b1;
  };
  if (paired) {
    for (int u = 0; u < pr.npairs; ++u) {
      const int2 pk = pr.pairs[u];
      const int k = pk.x;
      const int64_t Lt = (int64_t)pk.y * N;
#pragma unroll
      for (int i = 0; i < NH; ++i) {
        int b1, b2;
        pair_bins(i, b1, b2);
        const float2 l1 = list_at<H16>(L, Lt + b1), l2 = list_at<H16>(L, Lt + b2);
        const bool self = b1 == 0;                  // 0 and N/2 are their own mirrors
        const float2 m1 = self ? l1 : l2, m2 = self ? l2 : l1;
        const float2 c1 = float2{m1.x, -m1.y}, c2 = float2{m2.x, -m2.y};
        float2 x[CPL], y[CPL];
        load_x(b1 - k, x);
        load_x(b1 + k, y);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          cmac(acc[i][c], l1, x[c]);
          cmac(acc[i][c], c1, y[c]);
        }
        load_x(b2 - k, x);
        load_x(b2 + k, y);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          cmac(acc[NH + i][c], l2, x[c]);
          cmac(acc[NH + i][c], c2, y[c]);
        }
      }
    }
    for (int v = 0; v < pr.nsingles; ++v) {
      const int2 sk = pr.singles[v];
      const int k = sk.x;
      const int64_t Lt = (int64_t)sk.y * N;
#pragma unroll
      for (int i = 0; i < NH; ++i) {
        int b1, b2;
        pair_bins(i, b1, b2);
        float2 x[CPL];
        load_x(b1 - k, x);
        const float2 l1 = list_at<H16>(L, Lt + b1);
#pragma unroll
        for (int c = 0; c < CPL; ++c) cmac(acc[i][c], l1, x[c]);
        load_x(b2 - k, x);
        const float2 l2 = list_at<H16>(L, Lt + b2);
#pragma unroll
        for (int c = 0; c < CPL; ++c) cmac(acc[NH + i][c], l2, x[c]);
      }
    }
  } else {
    for (int t = 0; t < K; ++t) {
      const int k = shifts[t];
      const int64_t Lt = (int64_t)t * N;
#pragma unroll
      for (int i = 0; i < NBINS; ++i) {
        const int p = bl + i * BL;
        if (N % BL == 0 || p < N) {
          const float2 l = list_at<H16>(L, Lt + p);
          float2 x[CPL];
          load_x(p - k, x);
#pragma unroll
          for (int c = 0; c < CPL; ++c) cmac(acc[i][c], l, x[c]);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NBINS; ++i) {
    int p = bl + i * BL;
    if (paired) {
      int b1, b2;
      pair_bins(i < NH ? i : i - NH, b1, b2);
      p = i < NH ? b1 : b2;
    }
    if (N % BL == 0 || p < N) {
      float2* dst = &lds[pad_bin(p) * C + cg * CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) dst[c] = acc[i][c];
    }
  }
  __syncthreads();

  lds_fft<+1, LOG2N, ROWS>(lds, twl, twh);
  }

  // ---- store ----------------------------------------------------------------
  const float scale = SPEC ? 1.0f : 1.0f / (float)N;
  if (!ROWS) {
    if (2 * C >= 4 && vec4) {
      constexpr int V = 2 * C >= 4 ? 2 * C / 4 : 1;
      constexpr int TOT = N * V, NL = (TOT + T - 1) / T;
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int e = threadIdx.x + q * T;
        const int row = e / V, v = e % V;
        const int64_t c = first + 4 * v;
        if (e < TOT && c < extent) {
          float4 y = *reinterpret_cast<const float4*>(&lds[pad_bin(row) * C + 2 * v]);
          y = float4{y.x * scale, y.y * scale, y.z * scale, y.w * scale};
          float4* o = reinterpret_cast<float4*>(out + (int64_t)row * extent + c);
          if (accumulate) {
            const float4 z = *o;
            y = float4{y.x + z.x, y.y + z.y, y.z + z.z, y.w + z.w};
          }
          *o = y;
        }
      }
    } else {
      for (int e = threadIdx.x; e < N * 2 * C; e += T) {
        const int rc = e % (2 * C), row = e / (2 * C);
        const int64_t c = first + rc;
        if (c < extent) {
          const float v = ldsf[(pad_bin(row) * C + (rc >> 1)) * 2 + (rc & 1)] * scale;
          float* o = out + (int64_t)row * extent + c;
          *o = accumulate ? *o + v : v;
        }
      }
    }
  } else {
    for (int e = threadIdx.x; e < N * 2 * C; e += T) {
      const int q = e % N, rl = e / N;
      const int64_t r = first + rl;
      if (r < extent) {
        const float v = ldsf[(pad_bin(q) * C + (rl >> 1)) * 2 + (rl & 1)] * scale;
        float* o = out + r * N + q;
        *o = accumulate ? *o + v : v;
      }
    }
  }
}

// ---- sides that are not powers of two (n <= 2048), fused ---------------------
// The length-n DFT of sign s is Bluestein's chirp convolution,
//   X[k] = ch_k sum_j (x_j ch_j) conj(ch_{k-j}),   ch_t = exp(s pi i t^2 / n),
// done as a cyclic convolution of length M = 2^LOG2M >= 2n - 1 in LDS:
// chirp, forward FFT, times H (the FFT of the wrapped conj(ch), over M), inverse
// FFT, chirp.  The forward DFT, the shifted spectral MAC over n bins (indices
// mod n) and the inverse DFT (conjugate chirp, its own H, 1/n) run in one
// kernel per tile of 2C real columns (or rows), as cd_apply_kernel does for
// powers of two.  tab = [ch (n) | H_fwd / M (M) | H_inv / M (M)].
template <int LOG2M, bool ROWS, bool H16>
__global__ void __launch_bounds__(CdCfg<LOG2M>::T)
cd_chirp_kernel(const float* __restrict__ X, float* __restrict__ out, int64_t extent, int n, int K,
                const int32_t* __restrict__ shifts, const void* __restrict__ L, const float2* __restrict__ tab,
                const float2* __restrict__ tw, int accumulate) {
  using Cfg = CdCfg<LOG2M>;
  constexpr int M = Cfg::N, C = Cfg::C, T = Cfg::T;
  __shared__ __align__(16) float2 lds[Cfg::LDS_SLOTS];
  __shared__ float2 twl[Cfg::TWL], twh[Cfg::TWH];
  float* ldsf = reinterpret_cast<float*>(lds);
  for (int i = threadIdx.x; i < Cfg::TWL + Cfg::TWH; i += T) {
    if (i < Cfg::TWL) twl[i] = tw[i];
    else twh[i - Cfg::TWL] = tw[(i - Cfg::TWL) << Cfg::TWB];
  }
  const float2* ch = tab;
  const float2* Hf = tab + n;
  const float2* Hb = tab + n + M;
  const int nblk = gridDim.x;
  const int xcd = blockIdx.x % 8, slot_ = blockIdx.x / 8;
  int tile = xcd * ((nblk + 7) / 8) + slot_;
  if ((nblk & 7) != 0) tile = blockIdx.x;
  const int64_t first = (int64_t)tile * 2 * C;

  // load (bins >= n are the zero padding)
  if (!ROWS) {
    for (int e = threadIdx.x; e < M * 2 * C; e += T) {
      const int rc = e % (2 * C), row = e / (2 * C);
      const int64_t c = first + rc;
      ldsf[(pad_bin(row) * C + (rc >> 1)) * 2 + (rc & 1)] = (row < n && c < extent) ? X[(int64_t)row * extent + c] : 0.f;
    }
  } else {
    for (int e = threadIdx.x; e < M * 2 * C; e += T) {
      const int q = e % M, rl = e / M;
      const int64_t r = first + rl;
      ldsf[(pad_bin(q) * C + (rl >> 1)) * 2 + (rl & 1)] = (q < n && r < extent) ? X[r * n + q] : 0.f;
    }
  }
  __syncthreads();
  // a (bins < n) times w (tw_conj: use conj(w))
  auto scale_bins = [&](int count, const float2* w, bool conj_w) {
    for (int e = threadIdx.x; e < count * C; e += T) {
      const int bin = e / C, col = e % C;
      float2 f = w[bin];
      if (conj_w) f.y = -f.y;
      float2& v = lds[pad_bin(bin) * C + col];
      v = cmul(v, f);
    }
    __syncthreads();
  };
  // forward DFT of length n
  scale_bins(n, ch, false);
  lds_fft<-1, LOG2M, ROWS>(lds, twl, twh);
  scale_bins(M, Hf, false);
  lds_fft<+1, LOG2M, ROWS>(lds, twl, twh);
  scale_bins(n, ch, false);

  // shifted spectral MAC over n bins: Y[p] = sum_t L_t[p] X[(p - k_t) mod n]
  constexpr int CPL = Cfg::CPL, G = Cfg::G, BL = Cfg::BL;
  constexpr int NB = (M / 2 + BL - 1) / BL;    // n <= M / 2
  const int cg = threadIdx.x % G, bl = threadIdx.x / G;
  float2 acc[NB][CPL];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[i][c] = float2{0.f, 0.f};
  for (int t = 0; t < K; ++t) {
    const int k = shifts[t];
    const int64_t Lt = (int64_t)t * n;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int p = bl + i * BL;
      if (p < n) {
        const float2 l = list_at<H16>(L, Lt + p);
        int q = p - k;
        if (q < 0) q += n;
        const float2* src = &lds[pad_bin(q) * C + cg * CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          const float2 x = src[c];
          acc[i][c].x += l.x * x.x - l.y * x.y;
          acc[i][c].y += l.x * x.y + l.y * x.x;
        }
      }
    }
  }
  __syncthreads();
  // inverse DFT of length n (conjugate chirp), padding re-zeroed
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int p = bl + i * BL;
    if (p < n) {
#pragma unroll
      for (int c = 0; c < CPL; ++c) lds[pad_bin(p) * C + cg * CPL + c] = acc[i][c];
    }
  }
  for (int e = threadIdx.x; e < (M - n) * C; e += T) lds[pad_bin(n + e / C) * C + e % C] = float2{0.f, 0.f};
  __syncthreads();
  scale_bins(n, ch, true);
  lds_fft<-1, LOG2M, ROWS>(lds, twl, twh);
  scale_bins(M, Hb, false);
  lds_fft<+1, LOG2M, ROWS>(lds, twl, twh);
  scale_bins(n, ch, true);

  // store y / n
  const float sc = 1.0f / (float)n;
  if (!ROWS) {
    for (int e = threadIdx.x; e < n * 2 * C; e += T) {
      const int rc = e % (2 * C), row = e / (2 * C);
      const int64_t c = first + rc;
      if (c < extent) {
        const float v = ldsf[(pad_bin(row) * C + (rc >> 1)) * 2 + (rc & 1)] * sc;
        float* o = out + (int64_t)row * extent + c;
        *o = accumulate ? *o + v : v;
      }
    }
  } else {
    for (int e = threadIdx.x; e < n * 2 * C; e += T) {
      const int q = e % n, rl = e / n;
      const int64_t r = first + rl;
      if (r < extent) {
        const float v = ldsf[(pad_bin(q) * C + (rl >> 1)) * 2 + (rl & 1)] * sc;
        float* o = out + r * n + q;
        *o = accumulate ? *o + v : v;
      }
    }
  }
}

template <int LOG2M>
amm_status launch_chirp(bool rows, const float* X, float* out, int64_t extent, int n, int K, const int32_t* shifts,
                        const void* L, bool h16, const float2* tab, const float2* tw, bool acc, hipStream_t s) {
  using Cfg = CdCfg<LOG2M>;
  const int64_t tiles = (extent + 2 * Cfg::C - 1) / (2 * Cfg::C);
  if (tiles == 0) return AMM_OK;
  if (tiles > 0x7fffffff) return fail(AMM_EUNSUPPORTED, "too many column tiles");
  TimedLaunch tl(rows ? "cd_apply_rows" : "cd_apply_columns", s);
  const dim3 grid((unsigned)tiles), block(Cfg::T);
  if (h16) {
    if constexpr (LOG2M >= 12) {   // float16 lists: n > 1024
      if (rows)
        hipLaunchKernelGGL((cd_chirp_kernel<LOG2M, true, true>), grid, block, 0, s, X, out, extent, n, K, shifts, L,
                           tab, tw, acc ? 1 : 0);
      else
        hipLaunchKernelGGL((cd_chirp_kernel<LOG2M, false, true>), grid, block, 0, s, X, out, extent, n, K, shifts, L,
                           tab, tw, acc ? 1 : 0);
    } else {
      return fail(AMM_EUNSUPPORTED, "float16 lists need n >= 1024");
    }
  } else if (rows)
    hipLaunchKernelGGL((cd_chirp_kernel<LOG2M, true, false>), grid, block, 0, s, X, out, extent, n, K, shifts, L, tab,
                       tw, acc ? 1 : 0);
  else
    hipLaunchKernelGGL((cd_chirp_kernel<LOG2M, false, false>), grid, block, 0, s, X, out, extent, n, K, shifts, L, tab,
                       tw, acc ? 1 : 0);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

template <int LOG2N>
amm_status launch_cd(bool rows, const float* X, float* out, int64_t extent, int K,
                     const int32_t* shifts, const void* L, const float2* tw, bool acc,
                     hipStream_t s, bool spec, CdPairs pr, bool h16) {
  using Cfg = CdCfg<LOG2N>;
  const int64_t tiles = (extent + 2 * Cfg::C - 1) / (2 * Cfg::C);
  if (tiles == 0) return AMM_OK;
  if (tiles > 0x7fffffff) return fail(AMM_EUNSUPPORTED, "too many column tiles");
  dim3 grid((unsigned)tiles), block(Cfg::T);
  TimedLaunch tl(spec ? "cd_spectrum" : (rows ? "cd_apply_rows" : "cd_apply_columns"), s);
  // float4 path: whole float4 groups inside a row and 16-byte aligned rows
  const int vec4 = (!rows && 2 * Cfg::C >= 4 && extent % 4 == 0 && ((uintptr_t)X % 16) == 0 &&
                    ((uintptr_t)out % 16) == 0) ? 1 : 0;
  if (spec)
    hipLaunchKernelGGL((cd_apply_kernel<LOG2N, false, true>), grid, block, 0, s, X, out, extent, 0,
                       shifts, L, tw, 0, vec4, pr);
  else if (h16) {
    if constexpr (LOG2N >= kH16MinLog2) {
      if (rows)
        hipLaunchKernelGGL((cd_apply_kernel<LOG2N, true, false, true>), grid, block, 0, s, X, out, extent, K,
                           shifts, L, tw, acc ? 1 : 0, 0, pr);
      else
        hipLaunchKernelGGL((cd_apply_kernel<LOG2N, false, false, true>), grid, block, 0, s, X, out, extent, K,
                           shifts, L, tw, acc ? 1 : 0, vec4, pr);
    } else {
      return fail(AMM_EUNSUPPORTED, "float16 lists need n >= %d", 1 << kH16MinLog2);
    }
  } else if (rows)
    hipLaunchKernelGGL((cd_apply_kernel<LOG2N, true>), grid, block, 0, s, X, out, extent, K,
                       shifts, L, tw, acc ? 1 : 0, 0, pr);
  else
    hipLaunchKernelGGL((cd_apply_kernel<LOG2N, false>), grid, block, 0, s, X, out, extent, K,
                       shifts, L, tw, acc ? 1 : 0, vec4, pr);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

amm_status dispatch_cd(bool rows, int log2n, const float* X, float* out, int64_t extent, int K,
                       const int32_t* shifts, const void* L, const float2* tw, bool acc,
                       hipStream_t s, bool spec, CdPairs pr, bool h16 = false) {
  switch (log2n) {
#define AMM_CASE(L2) \
  case L2: return launch_cd<L2>(rows, X, out, extent, K, shifts, L, tw, acc, s, spec, pr, h16);
    AMM_CASE(1) AMM_CASE(2) AMM_CASE(3) AMM_CASE(4) AMM_CASE(5) AMM_CASE(6)
    AMM_CASE(7) AMM_CASE(8) AMM_CASE(9) AMM_CASE(10) AMM_CASE(11) AMM_CASE(12)
    AMM_CASE(13) AMM_CASE(14)
#undef AMM_CASE
    default: return fail(AMM_EUNSUPPORTED, "circulant product needs 2 <= n <= 16384, n a power of two");
  }
}

}  // namespace

amm_status cd_apply_columns(amm_ctx* ctx, int log2n, int K, const int32_t* shifts,
                            const float2* L, const float* B, int64_t p, float* out,
                            bool accumulate, hipStream_t s, CdPairs pr, const __half2* L16) {
  const float2* tw = nullptr;
  AMM_TRY(twiddles32(ctx, log2n, &tw));
  if (L16) return dispatch_cd(false, log2n, B, out, p, K, shifts, L16, tw, accumulate, s, false, pr, true);
  return dispatch_cd(false, log2n, B, out, p, K, shifts, L, tw, accumulate, s, false, pr);
}

amm_status cd_spectrum_columns(amm_ctx* ctx, int log2n, const float* B, int64_t p, float* spec,
                               hipStream_t s) {
  const float2* tw = nullptr;
  AMM_TRY(twiddles32(ctx, log2n, &tw));
  return dispatch_cd(false, log2n, B, spec, p, 0, nullptr, nullptr, tw, false, s, true, CdPairs{});
}

// Fused chirp-convolution product for 3 <= n <= 2048, n not a power of two:
// rows = false: out (n x extent) (+)= Atil X for X n x extent; rows = true:
// out (extent x n) (+)= the operator applied to each row of X (extent x n).
amm_status cd_chirp_apply(amm_ctx* ctx, bool rows, int n, int K, const int32_t* shifts, const float2* L,
                          const float* X, int64_t extent, float* out, bool accumulate, hipStream_t s,
                          const __half2* L16) {
  if (n < 3 || n > kChirpFusedMax) return fail(AMM_EUNSUPPORTED, "fused chirp product needs 3 <= n <= %d", kChirpFusedMax);
  int lM = 0;
  while ((1 << lM) < 2 * n - 1) ++lM;
  const float2* tab = nullptr;
  AMM_TRY(chirp_tables32(ctx, n, s, &tab));
  const float2* tw = nullptr;
  AMM_TRY(twiddles32(ctx, lM, &tw));
  switch (lM) {
#define AMM_CASE(L2) \
  case L2: return launch_chirp<L2>(rows, X, out, extent, n, K, shifts, L16 ? (const void*)L16 : (const void*)L, \
                                   L16 != nullptr, tab, tw, accumulate, s);
    AMM_CASE(3) AMM_CASE(4) AMM_CASE(5) AMM_CASE(6) AMM_CASE(7) AMM_CASE(8) AMM_CASE(9) AMM_CASE(10)
    AMM_CASE(11) AMM_CASE(12)
#undef AMM_CASE
    default: return fail(AMM_EUNSUPPORTED, "fused chirp product length %d", n);
  }
}

amm_status cd_apply_rows(amm_ctx* ctx, int log2n, int K, const int32_t* shifts,
                         const float2* L, const float* X, int64_t rows, float* out,
                         bool accumulate, hipStream_t s, CdPairs pr, const __half2* L16) {
  const float2* tw = nullptr;
  AMM_TRY(twiddles32(ctx, log2n, &tw));
  if (L16) return dispatch_cd(true, log2n, X, out, rows, K, shifts, L16, tw, accumulate, s, false, pr, true);
  return dispatch_cd(true, log2n, X, out, rows, K, shifts, L, tw, accumulate, s, false, pr);
}

}  // namespace amm
