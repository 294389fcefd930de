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
// H16 = true: float16 spectral products.  The lists are float16 pairs scaled
// by a power of two (l16_inv undoes it).  After the forward transform the
// tile's spectrum is scaled by the power of two that puts its largest
// component in [2^14, 2^15), rounded to float16 pairs and laid out without
// padding, twice in a row (bins 0 .. 2N-1, bin q + N a copy of bin q): every
// shifted read (p - k or p + k) then lands inside the doubled range without a
// modulo, and a lane's reads for one shift are one base plus constant offsets.
// Each complex product is two v_dot2_f32_f16 (two float16 products summed
// into a float32 accumulator); both transforms, the sums and the output stay
// float32.
template <bool H16>
__device__ __forceinline__ float2 list_at(const void* __restrict__ L, int64_t i) {
  if constexpr (H16) return __half22float2(reinterpret_cast<const __half2*>(L)[i]);
  else return reinterpret_cast<const float2*>(L)[i];
}

// float32 multipliers: a list value times a spectrum value, complex.
struct MulF { float2 v; };
__device__ __forceinline__ MulF mul_plain(float2 l) { return MulF{l}; }
__device__ __forceinline__ MulF mul_conj(float2 l) { return MulF{float2{l.x, -l.y}}; }
__device__ __forceinline__ void mac(float2& a, const MulF& m, float2 x) {
  a.x += m.v.x * x.x - m.v.y * x.y;
  a.y += m.v.x * x.y + m.v.y * x.x;
}

typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// float16 multipliers.  A value is (re, im) in the two halves of a 32-bit word
// (re low).  m x = (mr xr - mi xi) + i (mi xr + mr xi): the real part dots x
// with m, the high product negated, the imaginary part with m's halves swapped;
// conj(m) x = (mr xr + mi xi) + i (mr xi - mi xr): m itself, and the swapped
// word with the low product negated.  The negations are operand modifiers of
// v_dot2_f32_f16 (two float16 products summed into a float32 accumulator), so
// a list value costs one swap; the compiler does not fold sign flips of
// float16 pairs into these modifiers, hence the instruction is written out.
struct MulH { uint32_t m, sw; };    // value and its swapped halves
struct MulHc { uint32_t m, sw; };   // the same, applied conjugated
__device__ __forceinline__ uint32_t swap_halves(uint32_t u) { return (u >> 16) | (u << 16); }
__device__ __forceinline__ MulH mul_plain(uint32_t l) { return MulH{l, swap_halves(l)}; }
__device__ __forceinline__ MulHc mul_conj(uint32_t l) { return MulHc{l, swap_halves(l)}; }
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2(__builtin_bit_cast(half2v, a), __builtin_bit_cast(half2v, b), c, false);
}
__device__ __forceinline__ float dot2_neg_hi(uint32_t a, uint32_t b, float c) {
  asm("v_dot2_f32_f16 %0, %1, %2, %0 neg_hi:[1,0,0]" : "+v"(c) : "v"(a), "v"(b));
  return c;
}
__device__ __forceinline__ float dot2_neg_lo(uint32_t a, uint32_t b, float c) {
  asm("v_dot2_f32_f16 %0, %1, %2, %0 neg_lo:[1,0,0]" : "+v"(c) : "v"(a), "v"(b));
  return c;
}
__device__ __forceinline__ void mac(float2& a, const MulH& m, uint32_t x) {
  a.x = dot2_neg_hi(m.m, x, a.x);
  a.y = dot2(m.sw, x, a.y);
}
__device__ __forceinline__ void mac(float2& a, const MulHc& m, uint32_t x) {
  a.x = dot2(m.m, x, a.x);
  a.y = dot2_neg_lo(m.sw, x, a.y);
}

template <bool H16> struct ListVal { using type = float2; };
template <> struct ListVal<true> { using type = uint32_t; };
template <bool H16>
__device__ __forceinline__ typename ListVal<H16>::type list_val(const void* __restrict__ L, int64_t i) {
  if constexpr (H16) return reinterpret_cast<const uint32_t*>(L)[i];
  else return reinterpret_cast<const float2*>(L)[i];
}

// CPL float16 spectrum values of one bin (consecutive words from word w)
template <int CPL>
__device__ __forceinline__ void read_h(const uint32_t* hs, int w, uint32_t (&x)[CPL]) {
  if constexpr (CPL == 4) {
    const uint4 v = *reinterpret_cast<const uint4*>(hs + w);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  } else if constexpr (CPL == 2) {
    const uint2 v = *reinterpret_cast<const uint2*>(hs + w);
    x[0] = v.x; x[1] = v.y;
  } else {
    x[0] = hs[w];
  }
}

// JOBS: a batched launch; each workgroup takes its product's operands from
// the job table (jobs sorted by tile0) instead of the arguments.
template <int LOG2N, bool ROWS, bool SPEC = false, bool H16 = false, bool JOBS = false>
__global__ void __launch_bounds__(CdCfg<LOG2N>::T)
cd_apply_kernel(const float* __restrict__ X, int64_t ldx, float* __restrict__ out, int64_t ldo, int64_t extent,
                int K, const int32_t* __restrict__ shifts, const void* __restrict__ L,
                const float2* __restrict__ tw, int accumulate, int vec4, CdPairs pr, float l16_inv,
                const CdJob* __restrict__ jobs = nullptr, int njobs = 0) {
  using Cfg = CdCfg<LOG2N>;
  constexpr int N = Cfg::N, C = Cfg::C, T = Cfg::T;
  const uint16_t* Xh = nullptr;   // bfloat16 rows (batched launches)
  int rows_in = N, rows_out = N;
  int job_tile = 0;
  if constexpr (JOBS) {
    // the launch's tiles in XCD-aware order (consecutive tiles, which share a
    // product's lists, on one XCD), then the last job with tile0 <= that tile
    int gt = blockIdx.x;
    if ((gridDim.x & 7) == 0) gt = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].tile0 <= gt) lo = mid;
      else hi = mid - 1;
    }
    const CdJob& J = jobs[lo];
    if (J.x_bf16) Xh = static_cast<const uint16_t*>(J.X);
    else X = static_cast<const float*>(J.X);
    out = J.out;
    ldx = J.ldx;
    ldo = J.ldo;
    extent = J.extent;
    K = J.K;
    shifts = J.shifts;
    L = J.L;
    pr = J.pr;
    l16_inv = J.l16_inv;
    accumulate = J.accumulate;
    vec4 = J.vec4;
    rows_in = J.rows_in;
    rows_out = J.rows_out;
    job_tile = gt - J.tile0;
  }
  __shared__ __align__(16) float2 lds[Cfg::LDS_SLOTS];
  __shared__ float2 twl[Cfg::TWL], twh[Cfg::TWH];
  __shared__ float red[(T + 63) / 64];
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
  if constexpr (JOBS) tile = job_tile;      // batched: consecutive tiles of one product
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
        if constexpr (JOBS) {
          const bool in = e < TOT && c < extent && row < rows_in;
          if (Xh) {
            // four bfloat16 values (8 bytes) widened exactly
            const uint2 h = in ? *reinterpret_cast<const uint2*>(Xh + (int64_t)row * ldx + c) : uint2{0u, 0u};
            r[q] = float4{__uint_as_float(h.x << 16), __uint_as_float(h.x & 0xFFFF0000u), __uint_as_float(h.y << 16),
                          __uint_as_float(h.y & 0xFFFF0000u)};
          } else {
            r[q] = in ? *reinterpret_cast<const float4*>(X + (int64_t)row * ldx + c) : float4{0.f, 0.f, 0.f, 0.f};
          }
        } else {
          r[q] = (e < TOT && c < extent) ? *reinterpret_cast<const float4*>(X + (int64_t)row * ldx + c)
                                         : float4{0.f, 0.f, 0.f, 0.f};
        }
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
        float x = 0.f;
        if constexpr (JOBS) {
          if (c < extent && row < rows_in)
            x = Xh ? __uint_as_float((uint32_t)Xh[(int64_t)row * ldx + c] << 16) : X[(int64_t)row * ldx + c];
        } else {
          x = c < extent ? X[(int64_t)row * ldx + c] : 0.f;
        }
        ldsf[(pad_bin(row) * C + (rc >> 1)) * 2 + (rc & 1)] = x;
      }
    }
  } else {
    for (int e = threadIdx.x; e < N * 2 * C; e += T) {
      const int q = e % N, rl = e / N;
      const int64_t r = first + rl;
      ldsf[(pad_bin(q) * C + (rl >> 1)) * 2 + (rl & 1)] = r < extent ? X[r * ldx + q] : 0.f;
    }
  }
  __syncthreads();

  lds_fft<-1, LOG2N, ROWS>(lds, twl, twh);

  float scale = SPEC ? 1.0f : 1.0f / (float)N;
  if constexpr (!SPEC) {
  // ---- shifted spectral MAC: Y[p] = sum_t L_t[p] X[(p - k_t) mod N] ---------
  constexpr int CPL = Cfg::CPL, G = Cfg::G, BL = Cfg::BL, NBINS = Cfg::NBINS;
  using LV = typename ListVal<H16>::type;
  // lanes = (bin, column group); the packed columns of a group are read together
  const int cg = threadIdx.x % G;
  const int bl = threadIdx.x / G;
  uint32_t* hs = reinterpret_cast<uint32_t*>(lds);

  if constexpr (H16) {
    // scale, round and double the spectrum (see above)
    constexpr int NV = (N * C + T - 1) / T;
    float2 v[NV];
    float mx = 0.f;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = threadIdx.x + q * T;   // bin * C + column
      if ((N * C) % T == 0 || e < N * C) {
        v[q] = lds[pad_bin(e / C) * C + e % C];
        mx = fmaxf(mx, fmaxf(fabsf(v[q].x), fabsf(v[q].y)));
      }
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();    // also: every thread has read its values
    mx = red[0];
    for (int w = 1; w < (T + 63) / 64; ++w) mx = fmaxf(mx, red[w]);
    int ex = 0;
    (void)frexpf(mx, &ex);                        // mx < 2^ex
    const int sh = min(max(15 - ex, -100), 100);  // mx 2^sh < 2^15
    const float sx = ldexpf(1.0f, sh);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = threadIdx.x + q * T;
      if ((N * C) % T == 0 || e < N * C) {
        const uint32_t u = __builtin_bit_cast(uint32_t, __floats2half2_rn(v[q].x * sx, v[q].y * sx));
        hs[e] = u;
        hs[e + N * C] = u;
      }
    }
    __syncthreads();
    scale = ldexpf(l16_inv / (float)N, -sh);
  }

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
  // word offset of bin q (0 <= q < 2N) in the doubled float16 spectrum
  auto hw = [&](int q) { return q * C + cg * CPL; };
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
    constexpr int NHA = NH > 0 ? NH : 1;
    auto fetch = [&](int u, LV (&v1)[NHA], LV (&v2)[NHA]) {
      const int64_t Lt = (int64_t)pr.pairs[u].y * N;
#pragma unroll
      for (int i = 0; i < NH; ++i) {
        int b1, b2;
        pair_bins(i, b1, b2);
        v1[i] = list_val<H16>(L, Lt + b1);
        v2[i] = list_val<H16>(L, Lt + b2);
      }
    };
    // both members of the pair (k, N - k) at the lane's bins, lists v1 = L_k[b1], v2 = L_k[b2]
    auto apply = [&](int k, const LV (&v1)[NHA], const LV (&v2)[NHA]) {
      // float16 reads: b1 -+ k step +BL with i; b2 -+ k step -BL (bases at
      // i = NH-1); lane 0's partner of bin 0 is N/2
      const int wx1 = hw(bl - k + N), wy1 = hw(bl + k);
      const int wx2 = hw(2 * N - bl - (NH - 1) * BL - k), wy2 = hw(N - bl - (NH - 1) * BL + k);
      const int sx2 = hw(N / 2 - k + N), sy2 = hw(N / 2 + k);
#pragma unroll
      for (int i = 0; i < NH; ++i) {
        int b1, b2;
        pair_bins(i, b1, b2);
        const bool self = b1 == 0;                  // 0 and N/2 are their own mirrors
        const LV l1 = v1[i], l2 = v2[i];
        const LV m1 = self ? l1 : l2, m2 = self ? l2 : l1;
        if constexpr (H16) {
          // swap each list value once; the conjugated uses are m1 = l2 and m2 = l1
          // except at the self-mirrored bins
          const uint32_t s1 = swap_halves(l1), s2 = swap_halves(l2);
          const MulH p1{l1, s1}, p2{l2, s2};
          const MulHc q1{m1, self ? s1 : s2}, q2{m2, self ? s2 : s1};
          uint32_t x[CPL], y[CPL];
          read_h<CPL>(hs, wx1 + i * BL * C, x);
          read_h<CPL>(hs, wy1 + i * BL * C, y);
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            mac(acc[i][c], p1, x[c]);
            mac(acc[i][c], q1, y[c]);
          }
          int ax = wx2 + (NH - 1 - i) * BL * C, ay = wy2 + (NH - 1 - i) * BL * C;
          if (i == 0 && bl == 0) {
            ax = sx2;
            ay = sy2;
          }
          read_h<CPL>(hs, ax, x);
          read_h<CPL>(hs, ay, y);
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            mac(acc[NH + i][c], p2, x[c]);
            mac(acc[NH + i][c], q2, y[c]);
          }
        } else {
          const auto p1 = mul_plain(l1), q1 = mul_conj(m1), p2 = mul_plain(l2), q2 = mul_conj(m2);
          float2 x[CPL], y[CPL];
          load_x(b1 - k, x);
          load_x(b1 + k, y);
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            mac(acc[i][c], p1, x[c]);
            mac(acc[i][c], q1, y[c]);
          }
          load_x(b2 - k, x);
          load_x(b2 + k, y);
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            mac(acc[NH + i][c], p2, x[c]);
            mac(acc[NH + i][c], q2, y[c]);
          }
        }
      }
    };
    LV c1[NHA], c2[NHA];
    for (int u = 0; u < pr.npairs; ++u) {
      fetch(u, c1, c2);
      apply(pr.pairs[u].x, c1, c2);
    }
    for (int v = 0; v < pr.nsingles; ++v) {
      const int2 sk = pr.singles[v];
      const int k = sk.x;
      const int64_t Lt = (int64_t)sk.y * N;
#pragma unroll
      for (int i = 0; i < NH; ++i) {
        int b1, b2;
        pair_bins(i, b1, b2);
        const auto p1 = mul_plain(list_val<H16>(L, Lt + b1)), p2 = mul_plain(list_val<H16>(L, Lt + b2));
        if constexpr (H16) {
          uint32_t x[CPL];
          read_h<CPL>(hs, hw(b1 - k + N), x);
#pragma unroll
          for (int c = 0; c < CPL; ++c) mac(acc[i][c], p1, x[c]);
          read_h<CPL>(hs, hw(b2 - k + N), x);
#pragma unroll
          for (int c = 0; c < CPL; ++c) mac(acc[NH + i][c], p2, x[c]);
        } else {
          float2 x[CPL];
          load_x(b1 - k, x);
#pragma unroll
          for (int c = 0; c < CPL; ++c) mac(acc[i][c], p1, x[c]);
          load_x(b2 - k, x);
#pragma unroll
          for (int c = 0; c < CPL; ++c) mac(acc[NH + i][c], p2, x[c]);
        }
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
          const auto m = mul_plain(list_val<H16>(L, Lt + p));
          if constexpr (H16) {
            uint32_t x[CPL];
            read_h<CPL>(hs, hw(p - k + N), x);
#pragma unroll
            for (int c = 0; c < CPL; ++c) mac(acc[i][c], m, x[c]);
          } else {
            float2 x[CPL];
            load_x(p - k, x);
#pragma unroll
            for (int c = 0; c < CPL; ++c) mac(acc[i][c], m, x[c]);
          }
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
  if (!ROWS) {
    if (2 * C >= 4 && vec4) {
      constexpr int V = 2 * C >= 4 ? 2 * C / 4 : 1;
      constexpr int TOT = N * V, NL = (TOT + T - 1) / T;
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int e = threadIdx.x + q * T;
        const int row = e / V, v = e % V;
        const int64_t c = first + 4 * v;
        if (e < TOT && c < extent && (!JOBS || row < rows_out)) {
          float4 y = *reinterpret_cast<const float4*>(&lds[pad_bin(row) * C + 2 * v]);
          y = float4{y.x * scale, y.y * scale, y.z * scale, y.w * scale};
          float4* o = reinterpret_cast<float4*>(out + (int64_t)row * ldo + c);
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
        if (c < extent && (!JOBS || row < rows_out)) {
          const float v = ldsf[(pad_bin(row) * C + (rc >> 1)) * 2 + (rc & 1)] * scale;
          float* o = out + (int64_t)row * ldo + c;
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
        float* o = out + r * ldo + q;
        *o = accumulate ? *o + v : v;
      }
    }
  }
}

// ---- n = 16384, float16 products, columns: two column pairs per workgroup -----
// At n = 16384 a float32 spectrum fills the LDS, so the kernel above holds one
// packed column pair and streams every eigenvalue list once per pair.  This
// form keeps two pairs (four real columns) per workgroup: the LDS holds one
// float32 spectrum at a time for the transforms, and the other pair waits in
// registers (its raw columns during the first forward transform, its
// float16 spectrum during the first MAC, its finished columns during the
// second inverse transform).  The MACs run one pair after the other, each
// against that pair's doubled float16 spectrum (the affine reads of the
// one-pair kernel; reading both pairs side by side with wrapped indices
// measured slower, 2.0 against 1.3 ms for K = 64 at p = 16384).  Loads and
// stores move 16 bytes per row (storing each pair as soon as it is done, 8
// bytes per row, measured slower).  Each pair has its own power-of-two scale.
// The kernel runs at the 128-register limit with a few spilled values outside
// the MAC loop.

// The thread's bins tid + q T of the float32 spectrum in LDS, scaled by the
// power of two that puts the block's largest component in [2^14, 2^15) and
// rounded to float16 words; returns the exponent of that scale.  Ends with a
// barrier: every thread has read its bins.
template <int LOG2N>
__device__ __forceinline__ int spectrum_to_half(const float2* lds, float* red, uint32_t (&h)[CdCfg<LOG2N>::N /
                                                                                       CdCfg<LOG2N>::T]) {
  using Cfg = CdCfg<LOG2N>;
  constexpr int T = Cfg::T, NV = Cfg::N / T;
  float2 v[NV];
  float mx = 0.f;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    v[q] = lds[pad_bin(threadIdx.x + q * T)];
    mx = fmaxf(mx, fmaxf(fabsf(v[q].x), fabsf(v[q].y)));
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = red[0];
  for (int w = 1; w < T / 64; ++w) mx = fmaxf(mx, red[w]);
  int ex = 0;
  (void)frexpf(mx, &ex);
  const int sh = min(max(15 - ex, -100), 100);
  const float sx = ldexpf(1.0f, sh);
#pragma unroll
  for (int q = 0; q < NV; ++q)
    h[q] = __builtin_bit_cast(uint32_t, __floats2half2_rn(v[q].x * sx, v[q].y * sx));
  __syncthreads();
  return sh;
}

// The float16 MAC of one packed column pair (C = 1) against the doubled,
// unpadded spectrum hs (words 0 .. 2N-1, word q + N a copy of word q): the
// same arithmetic as the float16 branch of cd_apply_kernel, whose lane owns
// bins b1 = tid + i T and their mirrors.
template <int LOG2N>
__device__ __forceinline__ void mac_h16_doubled(const uint32_t* hs, const void* __restrict__ L, CdPairs pr, int K,
                                                const int32_t* __restrict__ shifts,
                                                float2 (&acc)[CdCfg<LOG2N>::N / CdCfg<LOG2N>::T]) {
  using Cfg = CdCfg<LOG2N>;
  constexpr int N = Cfg::N, T = Cfg::T, NV = N / T, BL = T, NH = NV / 2;
  const int bl = threadIdx.x;
  const uint32_t* Lw = reinterpret_cast<const uint32_t*>(L);
  auto pair_bins = [&](int i, int& b1, int& b2) {
    b1 = bl + i * BL;
    b2 = b1 == 0 ? N / 2 : N - b1;
  };
  if (pr.npairs >= 0) {
    for (int u = 0; u < pr.npairs; ++u) {
      const int k = pr.pairs[u].x;
      const int64_t Lt = (int64_t)pr.pairs[u].y * N;
      // b1 -+ k step +BL with i; b2 -+ k step -BL (bases at i = NH-1); lane
      // 0's partner of bin 0 is N/2.  Lists in two halves of the lane's bins
      // (register pressure).
      const int wx1 = bl - k + N, wy1 = bl + k;
      const int wx2 = 2 * N - bl - (NH - 1) * BL - k, wy2 = N - bl - (NH - 1) * BL + k;
#pragma unroll
      for (int hb = 0; hb < NH; hb += NH / 2) {
        uint32_t l1v[NH / 2], l2v[NH / 2];
#pragma unroll
        for (int j = 0; j < NH / 2; ++j) {
          int b1, b2;
          pair_bins(hb + j, b1, b2);
          l1v[j] = Lw[Lt + b1];
          l2v[j] = Lw[Lt + b2];
        }
#pragma unroll
        for (int j = 0; j < NH / 2; ++j) {
          const int i = hb + j;
          const bool self = i == 0 && bl == 0;
          const uint32_t l1 = l1v[j], l2 = l2v[j];
          const uint32_t s1 = swap_halves(l1), s2 = swap_halves(l2);
          const MulH p1{l1, s1}, p2{l2, s2};
          const MulHc q1{self ? l1 : l2, self ? s1 : s2}, q2{self ? l2 : l1, self ? s2 : s1};
          mac(acc[i], p1, hs[wx1 + i * BL]);
          mac(acc[i], q1, hs[wy1 + i * BL]);
          int ax = wx2 + (NH - 1 - i) * BL, ay = wy2 + (NH - 1 - i) * BL;
          if (self) {
            ax = N / 2 - k + N;
            ay = N / 2 + k;
          }
          mac(acc[NH + i], p2, hs[ax]);
          mac(acc[NH + i], q2, hs[ay]);
        }
      }
    }
    for (int v = 0; v < pr.nsingles; ++v) {
      const int k = pr.singles[v].x;
      const int64_t Lt = (int64_t)pr.singles[v].y * N;
#pragma unroll
      for (int i = 0; i < NH; ++i) {
        int b1, b2;
        pair_bins(i, b1, b2);
        mac(acc[i], mul_plain(Lw[Lt + b1]), hs[b1 - k + N]);
        mac(acc[NH + i], mul_plain(Lw[Lt + b2]), hs[b2 - k + N]);
      }
    }
  } else {
    for (int t = 0; t < K; ++t) {
      const int k = shifts[t];
      const int64_t Lt = (int64_t)t * N;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        int b1, b2;
        pair_bins(i < NH ? i : i - NH, b1, b2);
        const int b = i < NH ? b1 : b2;
        mac(acc[i], mul_plain(Lw[Lt + b]), hs[b - k + N]);
      }
    }
  }
}

template <int LOG2N>
__global__ void __launch_bounds__(CdCfg<LOG2N>::T)
cd_pair2_h16_kernel(const float* __restrict__ X, int64_t ldx, float* __restrict__ out, int64_t ldo,
                    int64_t extent, int K, const int32_t* __restrict__ shifts, const void* __restrict__ L,
                    const float2* __restrict__ tw, int accumulate, CdPairs pr, float l16_inv) {
  using Cfg = CdCfg<LOG2N>;
  constexpr int N = Cfg::N, T = Cfg::T;
  static_assert(Cfg::C == 1 && N % T == 0, "one float32 spectrum per LDS tile");
  constexpr int NV = N / T, BL = T, NH = NV / 2;
  __shared__ __align__(16) float2 lds[Cfg::LDS_SLOTS];
  __shared__ float2 twl[Cfg::TWL], twh[Cfg::TWH];
  __shared__ float red[T / 64];
  for (int i = threadIdx.x; i < Cfg::TWL + Cfg::TWH; i += T) {
    if (i < Cfg::TWL) twl[i] = tw[i];
    else twh[i - Cfg::TWL] = tw[(i - Cfg::TWL) << Cfg::TWB];
  }
  const int nblk = gridDim.x;
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  int tile = xcd * ((nblk + 7) / 8) + slot;
  if ((nblk & 7) != 0) tile = blockIdx.x;
  const int64_t first = (int64_t)tile * 4;   // first real column
  const int tid = threadIdx.x;

  // ---- load: pair 0 (columns first, first + 1) into LDS, pair 1 kept --------
  float2 keep[NV];
  {
    const bool whole = first + 3 < extent;
#pragma unroll
    for (int q0 = 0; q0 < NV; q0 += NV / 2) {   // two halves of the rows (register pressure)
      float4 r[NV / 2];
#pragma unroll
      for (int j = 0; j < NV / 2; ++j) {
        const float* src = X + (int64_t)(tid + (q0 + j) * T) * ldx + first;
        if (whole) {
          r[j] = *reinterpret_cast<const float4*>(src);
        } else {
          r[j] = float4{first < extent ? src[0] : 0.f, first + 1 < extent ? src[1] : 0.f,
                        first + 2 < extent ? src[2] : 0.f, 0.f};
        }
      }
#pragma unroll
      for (int j = 0; j < NV / 2; ++j) {
        lds[pad_bin(tid + (q0 + j) * T)] = float2{r[j].x, r[j].y};
        keep[q0 + j] = float2{r[j].z, r[j].w};
      }
    }
  }
  __syncthreads();
  lds_fft<-1, LOG2N, false>(lds, twl, twh);
  uint32_t h0[NV];
  const int sh0 = spectrum_to_half<LOG2N>(lds, red, h0);
#pragma unroll
  for (int q = 0; q < NV; ++q) lds[pad_bin(tid + q * T)] = keep[q];
  __syncthreads();
  lds_fft<-1, LOG2N, false>(lds, twl, twh);
  uint32_t h1[NV];
  const int sh1 = spectrum_to_half<LOG2N>(lds, red, h1);
  // ---- the MAC, one pair at a time against its doubled float16 spectrum -------
  float2 acc[NV][2];
  uint32_t* hs = reinterpret_cast<uint32_t*>(lds);
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    float2 a[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) a[i] = float2{0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const uint32_t w = pair == 0 ? h0[q] : h1[q];
      hs[tid + q * T] = w;
      hs[tid + q * T + N] = w;
    }
    __syncthreads();
    mac_h16_doubled<LOG2N>(hs, L, pr, K, shifts, a);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i][pair] = a[i];
  }
  auto pair_bins = [&](int i, int& b1, int& b2) {
    b1 = tid + i * BL;
    b2 = b1 == 0 ? N / 2 : N - b1;
  };

  // ---- inverse transforms, pair 0 then pair 1; store 16 bytes per row --------
  auto put = [&](int pair) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      int b1, b2;
      pair_bins(i < NH ? i : i - NH, b1, b2);
      lds[pad_bin(i < NH ? b1 : b2)] = acc[i][pair];
    }
  };
  put(0);
  __syncthreads();
  lds_fft<+1, LOG2N, false>(lds, twl, twh);
  float2 res0[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) res0[q] = lds[pad_bin(tid + q * T)];
  __syncthreads();
  put(1);
  __syncthreads();
  lds_fft<+1, LOG2N, false>(lds, twl, twh);
  const float s0 = ldexpf(l16_inv / (float)N, -sh0), s1 = ldexpf(l16_inv / (float)N, -sh1);
  const bool whole = first + 3 < extent;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const float2 y1 = lds[pad_bin(tid + q * T)];
    float4 y{res0[q].x * s0, res0[q].y * s0, y1.x * s1, y1.y * s1};
    float* dst = out + (int64_t)(tid + q * T) * ldo + first;
    if (whole) {
      if (accumulate) {
        const float4 z = *reinterpret_cast<const float4*>(dst);
        y = float4{y.x + z.x, y.y + z.y, y.z + z.z, y.w + z.w};
      }
      *reinterpret_cast<float4*>(dst) = y;
    } else {
      const float yv[3] = {y.x, y.y, y.z};
      for (int j = 0; j < 3; ++j)
        if (first + j < extent) dst[j] = accumulate ? dst[j] + yv[j] : yv[j];
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
                const float2* __restrict__ tw, int accumulate, float l16_inv) {
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

  // store y / n (float16 lists: also undo their power-of-two scale)
  const float sc = (H16 ? l16_inv : 1.0f) / (float)n;
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
                        const void* L, bool h16, float l16_inv, const float2* tab, const float2* tw, bool acc,
                        hipStream_t s) {
  using Cfg = CdCfg<LOG2M>;
  const int64_t tiles = (extent + 2 * Cfg::C - 1) / (2 * Cfg::C);
  if (tiles == 0) return AMM_OK;
  if (tiles > 0x7fffffff) return fail(AMM_EUNSUPPORTED, "too many column tiles");
  TimedLaunch tl(rows ? "cd_apply_rows" : "cd_apply_columns", s);
  const dim3 grid((unsigned)tiles), block(Cfg::T);
  const int a = acc ? 1 : 0;
  if (h16) {
    if constexpr (LOG2M >= 12) {   // float16 lists: n > 1024
      if (rows)
        hipLaunchKernelGGL((cd_chirp_kernel<LOG2M, true, true>), grid, block, 0, s, X, out, extent, n, K, shifts, L,
                           tab, tw, a, l16_inv);
      else
        hipLaunchKernelGGL((cd_chirp_kernel<LOG2M, false, true>), grid, block, 0, s, X, out, extent, n, K, shifts, L,
                           tab, tw, a, l16_inv);
    } else {
      return fail(AMM_EUNSUPPORTED, "float16 lists need n >= 1024");
    }
  } else if (rows)
    hipLaunchKernelGGL((cd_chirp_kernel<LOG2M, true, false>), grid, block, 0, s, X, out, extent, n, K, shifts, L, tab,
                       tw, a, 1.0f);
  else
    hipLaunchKernelGGL((cd_chirp_kernel<LOG2M, false, false>), grid, block, 0, s, X, out, extent, n, K, shifts, L, tab,
                       tw, a, 1.0f);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

#ifndef AMM_CD_ONEPAIR
#define AMM_CD_ONEPAIR 0
#endif

template <int LOG2N, bool ROWS, bool H16>
void launch_cd_kernel(dim3 grid, dim3 block, hipStream_t s, const float* X, int64_t ldx, float* out, int64_t ldo,
                      int64_t extent, int K, const int32_t* shifts, const void* L, const float2* tw, int acc, int vec4,
                      CdPairs pr, float l16_inv) {
  hipLaunchKernelGGL((cd_apply_kernel<LOG2N, ROWS, false, H16>), grid, block, 0, s, X, ldx, out, ldo,
                     extent, K, shifts, L, tw, acc, vec4, pr, l16_inv);
}

template <int LOG2N>
amm_status launch_cd(bool rows, const float* X, int64_t ldx, float* out, int64_t ldo, int64_t extent, int K,
                     const int32_t* shifts, const void* L, const float2* tw, bool acc,
                     hipStream_t s, bool spec, CdPairs pr, bool h16, float l16_inv) {
  using Cfg = CdCfg<LOG2N>;
  const int64_t tiles = (extent + 2 * Cfg::C - 1) / (2 * Cfg::C);
  if (tiles == 0) return AMM_OK;
  if (tiles > 0x7fffffff) return fail(AMM_EUNSUPPORTED, "too many column tiles");
  dim3 grid((unsigned)tiles), block(Cfg::T);
  TimedLaunch tl(spec ? "cd_spectrum" : (rows ? "cd_apply_rows" : "cd_apply_columns"), s);
  // float4 path: whole float4 groups inside a row and 16-byte aligned rows
  const int vec4 = (!rows && 2 * Cfg::C >= 4 && extent % 4 == 0 && ldx % 4 == 0 && ldo % 4 == 0 &&
                    ((uintptr_t)X % 16) == 0 && ((uintptr_t)out % 16) == 0) ? 1 : 0;
  const int a = acc ? 1 : 0;
  if (spec)
    hipLaunchKernelGGL((cd_apply_kernel<LOG2N, false, true>), grid, block, 0, s, X, ldx, out, ldo, extent, 0,
                       shifts, L, tw, 0, vec4, pr, 1.0f);
  else if (h16) {
    if constexpr (LOG2N == 14 && !AMM_CD_ONEPAIR) {
      // two column pairs per workgroup (16-byte row accesses)
      if (!rows && ldx % 4 == 0 && ldo % 4 == 0 && ((uintptr_t)X % 16) == 0 && ((uintptr_t)out % 16) == 0) {
        const int64_t t4 = (extent + 3) / 4;
        hipLaunchKernelGGL((cd_pair2_h16_kernel<LOG2N>), dim3((unsigned)t4), block, 0, s, X, ldx, out, ldo, extent, K,
                           shifts, L, tw, a, pr, l16_inv);
        AMM_HIP(hipGetLastError());
        return AMM_OK;
      }
    }
    if constexpr (LOG2N >= kH16MinLog2) {
      if (rows)
        launch_cd_kernel<LOG2N, true, true>(grid, block, s, X, ldx, out, ldo, extent, K, shifts, L, tw, a, 0, pr,
                                            l16_inv);
      else
        launch_cd_kernel<LOG2N, false, true>(grid, block, s, X, ldx, out, ldo, extent, K, shifts, L, tw, a, vec4, pr,
                                             l16_inv);
    } else {
      return fail(AMM_EUNSUPPORTED, "float16 spectral products need n >= %d", 1 << kH16MinLog2);
    }
  } else if (rows)
    launch_cd_kernel<LOG2N, true, false>(grid, block, s, X, ldx, out, ldo, extent, K, shifts, L, tw, a, 0, pr, 1.0f);
  else
    launch_cd_kernel<LOG2N, false, false>(grid, block, s, X, ldx, out, ldo, extent, K, shifts, L, tw, a, vec4, pr,
                                          1.0f);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

amm_status dispatch_cd(bool rows, int log2n, const float* X, int64_t ldx, float* out, int64_t ldo, int64_t extent,
                       int K, const int32_t* shifts, const void* L, const float2* tw, bool acc,
                       hipStream_t s, bool spec, CdPairs pr, bool h16 = false, float l16_inv = 1.0f) {
  switch (log2n) {
#define AMM_CASE(L2) \
  case L2: return launch_cd<L2>(rows, X, ldx, out, ldo, extent, K, shifts, L, tw, acc, s, spec, pr, h16, l16_inv);
    AMM_CASE(1) AMM_CASE(2) AMM_CASE(3) AMM_CASE(4) AMM_CASE(5) AMM_CASE(6)
    AMM_CASE(7) AMM_CASE(8) AMM_CASE(9) AMM_CASE(10) AMM_CASE(11) AMM_CASE(12)
    AMM_CASE(13) AMM_CASE(14)
#undef AMM_CASE
    default: return fail(AMM_EUNSUPPORTED, "circulant product needs 2 <= n <= 16384, n a power of two");
  }
}

template <int LOG2N>
amm_status launch_cd_jobs(bool h16, const CdJob* jobs, int njobs, int tiles, const float2* tw, hipStream_t s) {
  using Cfg = CdCfg<LOG2N>;
  dim3 grid((unsigned)tiles), block(Cfg::T);
  TimedLaunch tl("cd_apply_batched", s);
  if (h16) {
    if constexpr (LOG2N >= kH16MinLog2)
      hipLaunchKernelGGL((cd_apply_kernel<LOG2N, false, false, true, true>), grid, block, 0, s, (const float*)nullptr,
                         (int64_t)0, (float*)nullptr, (int64_t)0, (int64_t)0, 0, (const int32_t*)nullptr,
                         (const void*)nullptr, tw, 0, 0, CdPairs{}, 1.0f, jobs, njobs);
    else
      return fail(AMM_EUNSUPPORTED, "float16 spectral products need n >= %d", 1 << kH16MinLog2);
  } else {
    hipLaunchKernelGGL((cd_apply_kernel<LOG2N, false, false, false, true>), grid, block, 0, s, (const float*)nullptr,
                       (int64_t)0, (float*)nullptr, (int64_t)0, (int64_t)0, 0, (const int32_t*)nullptr,
                       (const void*)nullptr, tw, 0, 0, CdPairs{}, 1.0f, jobs, njobs);
  }
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

}  // namespace

int cd_tile_columns(int log2n) {
  switch (log2n) {
#define AMM_CASE(L2) \
  case L2: return 2 * CdCfg<L2>::C;
    AMM_CASE(6) AMM_CASE(7) AMM_CASE(8) AMM_CASE(9) AMM_CASE(10) AMM_CASE(11) AMM_CASE(12) AMM_CASE(13) AMM_CASE(14)
#undef AMM_CASE
    default: return 0;
  }
}

amm_status cd_apply_jobs(amm_ctx* ctx, int log2n, bool h16, const CdJob* jobs, int njobs, int tiles, hipStream_t s) {
  if (njobs <= 0 || tiles <= 0) return AMM_OK;
  const float2* tw = nullptr;
  AMM_TRY(twiddles32(ctx, log2n, &tw));
  switch (log2n) {
#define AMM_CASE(L2) \
  case L2: return launch_cd_jobs<L2>(h16, jobs, njobs, tiles, tw, s);
    AMM_CASE(6) AMM_CASE(7) AMM_CASE(8) AMM_CASE(9) AMM_CASE(10) AMM_CASE(11) AMM_CASE(12) AMM_CASE(13) AMM_CASE(14)
#undef AMM_CASE
    default: return fail(AMM_EUNSUPPORTED, "batched circulant launches need 64 <= n <= 16384");
  }
}

amm_status cd_apply_columns(amm_ctx* ctx, int log2n, int K, const int32_t* shifts,
                            const float2* L, const float* B, int64_t p, float* out,
                            bool accumulate, hipStream_t s, CdPairs pr, const __half2* L16, float l16_inv,
                            int64_t ldb, int64_t ldo) {
  const float2* tw = nullptr;
  AMM_TRY(twiddles32(ctx, log2n, &tw));
  const int64_t ldx = ldb > 0 ? ldb : p, ldy = ldo > 0 ? ldo : p;
  if (L16)
    return dispatch_cd(false, log2n, B, ldx, out, ldy, p, K, shifts, L16, tw, accumulate, s, false, pr, true, l16_inv);
  return dispatch_cd(false, log2n, B, ldx, out, ldy, p, K, shifts, L, tw, accumulate, s, false, pr);
}

amm_status cd_spectrum_columns(amm_ctx* ctx, int log2n, const float* B, int64_t p, float* spec,
                               hipStream_t s) {
  const float2* tw = nullptr;
  AMM_TRY(twiddles32(ctx, log2n, &tw));
  return dispatch_cd(false, log2n, B, p, spec, p, p, 0, nullptr, nullptr, tw, false, s, true, CdPairs{});
}

// Fused chirp-convolution product for 3 <= n <= 2048, n not a power of two:
// rows = false: out (n x extent) (+)= Atil X for X n x extent; rows = true:
// out (extent x n) (+)= the operator applied to each row of X (extent x n).
amm_status cd_chirp_apply(amm_ctx* ctx, bool rows, int n, int K, const int32_t* shifts, const float2* L,
                          const float* X, int64_t extent, float* out, bool accumulate, hipStream_t s,
                          const __half2* L16, float l16_inv) {
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
                                   L16 != nullptr, l16_inv, tab, tw, accumulate, s);
    AMM_CASE(3) AMM_CASE(4) AMM_CASE(5) AMM_CASE(6) AMM_CASE(7) AMM_CASE(8) AMM_CASE(9) AMM_CASE(10)
    AMM_CASE(11) AMM_CASE(12)
#undef AMM_CASE
    default: return fail(AMM_EUNSUPPORTED, "fused chirp product length %d", n);
  }
}

amm_status cd_apply_rows(amm_ctx* ctx, int log2n, int K, const int32_t* shifts,
                         const float2* L, const float* X, int64_t rows, float* out,
                         bool accumulate, hipStream_t s, CdPairs pr, const __half2* L16, float l16_inv) {
  const float2* tw = nullptr;
  AMM_TRY(twiddles32(ctx, log2n, &tw));
  const int64_t n = int64_t{1} << log2n;
  if (L16)
    return dispatch_cd(true, log2n, X, n, out, n, rows, K, shifts, L16, tw, accumulate, s, false, pr, true, l16_inv);
  return dispatch_cd(true, log2n, X, n, out, n, rows, K, shifts, L, tw, accumulate, s, false, pr);
}

}  // namespace amm
