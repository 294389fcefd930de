// Circulant decomposition and products for sizes that are not powers of two.
//
// A length-n DFT with sign s, X[k] = sum_j x_j exp(s 2 pi i j k / n), is
// evaluated as Bluestein's chirp convolution: with ch_t = exp(s pi i t^2 / n),
//   j k = (j^2 + k^2 - (k - j)^2) / 2   =>   X[k] = ch_k sum_j (x_j ch_j) conj(ch_{k-j}),
// a linear convolution done as a cyclic one of power-of-two length N >= 2n - 1
// through the float64 Stockham passes.  t^2 is reduced mod 2n in integers
// before the angle is formed, so the chirp is exact to rounding for every t.
//
// The product  out = sum_t R_t D^{k_t} B = F^-1 sum_t diag(L_t) C^{k_t} F B
// (Alg. 2.3 step 5, W D^k W* = C^k) then runs as three float64 steps over the
// columns of B, two real columns packed into one complex column (the
// truncated operator is real, hence complex-linear): forward DFT, the
// spectral multiply-accumulate of the kept shifted spectra, inverse DFT.
// Up to n = 2048 the product runs instead as one fused float32 kernel (the
// chirp convolutions in LDS, cd_chirp_kernel) fed by the float32 tables built
// here; larger sides take the float64 steps, which keep the float32 parity
// bar with room to spare.
#include "amm_internal.hpp"

namespace amm {
namespace {

__device__ __forceinline__ double2 cmul64(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ __forceinline__ double2 chirp(int64_t t, int n, int sign) {
  const int64_t r = (t * t) % (2 * (int64_t)n);
  double sn, cs;
  sincospi((double)sign * (double)r / (double)n, &sn, &cs);
  return double2{cs, sn};
}

// b[t] = conj(ch_t) for t < n, b[N - t] = conj(ch_t) for 0 < t < n, else 0
__global__ void chirp_kernel_vec(double2* __restrict__ b, int n, int N, int sign) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  int u = -1;
  if (t < n) u = t;
  else if (t > N - n) u = N - t;
  if (u < 0) {
    b[t] = double2{0.0, 0.0};
  } else {
    const double2 c = chirp(u, n, sign);
    b[t] = double2{c.x, -c.y};
  }
}

// P[v][t] = x_v[t] ch_t (t < n), 0 (n <= t < N), for v in [v0, v0 + nv)
__global__ void bluestein_pad(const double2* __restrict__ x, int n, int64_t es, int64_t bs, int64_t v0, int64_t nv,
                              int N, int sign, double2* __restrict__ P) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nv * N) return;
  const int64_t v = id % nv, t = id / nv;   // v fastest: neighbouring threads read neighbouring columns
  double2 r{0.0, 0.0};
  if (t < n) r = cmul64(x[(v0 + v) * bs + t * es], chirp(t, n, sign));
  P[v * N + t] = r;
}

__global__ void pointwise_mul(double2* __restrict__ P, const double2* __restrict__ Bh, int N, int64_t count) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= count) return;
  P[id] = cmul64(P[id], Bh[id % N]);
}

// x_v[k] = P[v][k] ch_k scale for k < n
__global__ void bluestein_unpad(const double2* __restrict__ P, int n, int N, int sign, double scale, int64_t es,
                                int64_t bs, int64_t v0, int64_t nv, double2* __restrict__ x) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nv * n) return;
  const int64_t v = id % nv, k = id / nv;
  const double2 r = cmul64(P[v * N + k], chirp(k, n, sign));
  x[(v0 + v) * bs + k * es] = double2{r.x * scale, r.y * scale};
}

// Z[q][c] = B[q][2c] + i B[q][2c + 1] (a missing odd column is zero)
__global__ void pack_pairs(const float* __restrict__ B, int64_t n, int64_t p, int64_t P2, double2* __restrict__ Z) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * P2) return;
  const int64_t q = id / P2, c = id % P2;
  const double re = B[q * p + 2 * c];
  const double im = (2 * c + 1 < p) ? (double)B[q * p + 2 * c + 1] : 0.0;
  Z[id] = double2{re, im};
}

// Y[q][c] = sum_t L_t[q] X[(q - k_t) mod n][c]
__global__ void spectral_mac(const double2* __restrict__ X, int n, int64_t P2, int K, const int32_t* __restrict__ shifts,
                             const float2* __restrict__ L, double2* __restrict__ Y) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)n * P2) return;
  const int q = (int)(id / P2);
  const int64_t c = id % P2;
  double2 acc{0.0, 0.0};
  for (int t = 0; t < K; ++t) {
    int src = q - shifts[t];
    if (src < 0) src += n;
    const float2 l = L[(int64_t)t * n + q];
    const double2 a = cmul64(double2{(double)l.x, (double)l.y}, X[(int64_t)src * P2 + c]);
    acc.x += a.x;
    acc.y += a.y;
  }
  Y[id] = acc;
}

// out[q][2c] (+)= re Y[q][c], out[q][2c + 1] (+)= im Y[q][c]
__global__ void unpack_pairs(const double2* __restrict__ Y, int64_t n, int64_t p, int64_t P2, float* __restrict__ out,
                             int accumulate) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * P2) return;
  const int64_t q = id / P2, c = id % P2;
  const double2 y = Y[id];
  float* o = out + q * p + 2 * c;
  o[0] = accumulate ? o[0] + (float)y.x : (float)y.x;
  if (2 * c + 1 < p) o[1] = accumulate ? o[1] + (float)y.y : (float)y.y;
}

// X[q][2c], X[q][2c + 1] = re, im of Z[q][c] (float32)
__global__ void spectrum_to_f32(const double2* __restrict__ Z, int64_t count, float* __restrict__ X) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= count) return;
  const double2 z = Z[id];
  X[2 * id] = (float)z.x;
  X[2 * id + 1] = (float)z.y;
}

int ceil_log2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

unsigned blocks_for(int64_t count) { return (unsigned)((count + 255) / 256); }

// float32 tables of the fused product: tab[t] = ch_t (sign -1), then the two
// kernel spectra scaled by 1/N
__global__ void chirp_tables_f32(const double2* __restrict__ Bf, const double2* __restrict__ Bb, int n, int N,
                                 float2* __restrict__ tab) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n + 2 * N) return;
  double2 v;
  if (id < n) v = chirp(id, n, -1);
  else if (id < n + N) v = double2{Bf[id - n].x / N, Bf[id - n].y / N};
  else v = double2{Bb[id - n - N].x / N, Bb[id - n - N].y / N};
  tab[id] = float2{(float)v.x, (float)v.y};
}

// FFT_N of the wrapped conj(ch) for (n, sign), computed once per context
amm_status chirp_spectrum64(amm_ctx* ctx, int n, int sign, hipStream_t s, const double2** out) {
  const int lN = std::max(ceil_log2(2 * (int64_t)n - 1), 1);
  const int N = 1 << lN;
  const int64_t key = 2 * (int64_t)n + (sign > 0 ? 1 : 0);
  auto it = ctx->chirp64.find(key);
  if (it == ctx->chirp64.end()) {
    const double2* tw = nullptr;
    AMM_TRY(twiddles64(ctx, lN, &tw));
    DevBuf bk, bt;
    AMM_TRY(bk.alloc((size_t)N * sizeof(double2)));
    AMM_TRY(bt.alloc((size_t)N * sizeof(double2)));
    hipLaunchKernelGGL(chirp_kernel_vec, dim3(blocks_for(N)), dim3(256), 0, s, bk.as<double2>(), n, N, sign);
    AMM_HIP(hipGetLastError());
    double2 *kc = bk.as<double2>(), *kt = bt.as<double2>();
    AMM_TRY(fft64_transform(kc, kt, lN, 1, N, 1, false, -1, 1.0, tw, s));
    AMM_HIP(hipStreamSynchronize(s));   // the other buffer is released on return
    // the passes ping-pong: keep whichever buffer holds the spectrum
    it = ctx->chirp64.emplace(key, std::move(kc == bk.as<double2>() ? bk : bt)).first;
  }
  *out = it->second.as<double2>();
  return AMM_OK;
}

}  // namespace

amm_status chirp_tables32(amm_ctx* ctx, int n, hipStream_t s, const float2** tab) {
  auto it = ctx->chirp32.find(n);
  if (it == ctx->chirp32.end()) {
    const int N = 1 << std::max(ceil_log2(2 * (int64_t)n - 1), 1);
    const double2 *Bf = nullptr, *Bb = nullptr;
    AMM_TRY(chirp_spectrum64(ctx, n, -1, s, &Bf));
    AMM_TRY(chirp_spectrum64(ctx, n, +1, s, &Bb));
    DevBuf t;
    AMM_TRY(t.alloc((size_t)(n + 2 * N) * sizeof(float2)));
    hipLaunchKernelGGL(chirp_tables_f32, dim3(blocks_for(n + 2 * N)), dim3(256), 0, s, Bf, Bb, n, N, t.as<float2>());
    AMM_HIP(hipGetLastError());
    AMM_HIP(hipStreamSynchronize(s));
    it = ctx->chirp32.emplace(n, std::move(t)).first;
  }
  *tab = it->second.as<float2>();
  return AMM_OK;
}

amm_status dft64_any(amm_ctx* ctx, double2* x, int n, int64_t es, int64_t bs, int64_t batch, int sign, double scale,
                     hipStream_t s, bool sync) {
  if (n < 1 || batch <= 0) return AMM_OK;
  const int lN = ceil_log2(2 * (int64_t)n - 1);
  if (lN > 15) return fail(AMM_EUNSUPPORTED, "DFT length %d too large", n);
  const int N = 1 << std::max(lN, 1);
  const double2* tw = nullptr;
  AMM_TRY(twiddles64(ctx, std::max(lN, 1), &tw));
  // kernel spectrum Bh = FFT_N(b), computed once per (n, sign) and kept by the context
  const double2* Bh = nullptr;
  AMM_TRY(chirp_spectrum64(ctx, n, sign, s, &Bh));
  // vectors in chunks of at most ~512 MiB of padded data, in the context's work areas
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(batch, ((int64_t)512 << 20) / ((int64_t)N * 16)));
  AMM_TRY(ctx->scratch[10].reserve((size_t)chunk * N * sizeof(double2)));
  AMM_TRY(ctx->scratch[11].reserve((size_t)chunk * N * sizeof(double2)));
  for (int64_t v0 = 0; v0 < batch; v0 += chunk) {
    const int64_t nv = std::min(chunk, batch - v0);
    double2 *cur = ctx->scratch[10].as<double2>(), *tmp = ctx->scratch[11].as<double2>();
    hipLaunchKernelGGL(bluestein_pad, dim3(blocks_for(nv * N)), dim3(256), 0, s, x, n, es, bs, v0, nv, N, sign, cur);
    AMM_HIP(hipGetLastError());
    AMM_TRY(fft64_transform(cur, tmp, std::max(lN, 1), 1, N, nv, false, -1, 1.0, tw, s));
    hipLaunchKernelGGL(pointwise_mul, dim3(blocks_for(nv * N)), dim3(256), 0, s, cur, Bh, N, nv * N);
    AMM_HIP(hipGetLastError());
    AMM_TRY(fft64_transform(cur, tmp, std::max(lN, 1), 1, N, nv, false, +1, 1.0 / N, tw, s));
    hipLaunchKernelGGL(bluestein_unpad, dim3(blocks_for(nv * n)), dim3(256), 0, s, cur, n, N, sign, scale, es, bs, v0,
                       nv, x);
    AMM_HIP(hipGetLastError());
  }
  if (sync) AMM_HIP(hipStreamSynchronize(s));
  return AMM_OK;
}

amm_status cd_apply_general(amm_ctx* ctx, int n, int K, const int32_t* shifts, const float2* L, const float* B,
                            int64_t p, float* out, bool acc, hipStream_t s, const __half2* L16,
                            float l16_inv) {
  if (p <= 0) return AMM_OK;
  if (K == 0) {
    if (!acc) return fill_f32(out, (int64_t)n * p, 0.f, s);
    return AMM_OK;
  }
  if (n >= 3 && n <= kChirpFusedMax) return cd_chirp_apply(ctx, false, n, K, shifts, L, B, p, out, acc, s, L16, l16_inv);
  const int64_t P2 = (p + 1) / 2, cnt = (int64_t)n * P2;
  AMM_TRY(ctx->scratch[8].reserve(cnt * sizeof(double2)));
  AMM_TRY(ctx->scratch[9].reserve(cnt * sizeof(double2)));
  double2 *z = ctx->scratch[8].as<double2>(), *y = ctx->scratch[9].as<double2>();
  TimedLaunch tl("cd_apply_general", s);
  hipLaunchKernelGGL(pack_pairs, dim3(blocks_for(cnt)), dim3(256), 0, s, B, (int64_t)n, p, P2, z);
  AMM_HIP(hipGetLastError());
  AMM_TRY(dft64_any(ctx, z, n, P2, 1, P2, -1, 1.0, s, false));
  hipLaunchKernelGGL(spectral_mac, dim3(blocks_for(cnt)), dim3(256), 0, s, z, n, P2, K, shifts, L, y);
  AMM_HIP(hipGetLastError());
  AMM_TRY(dft64_any(ctx, y, n, P2, 1, P2, +1, 1.0 / n, s, false));
  hipLaunchKernelGGL(unpack_pairs, dim3(blocks_for(cnt)), dim3(256), 0, s, y, (int64_t)n, p, P2, out, acc ? 1 : 0);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

// Packed forward spectra of B's column pairs for any n (p even): X (n x p
// floats) holds F(b_2c + i b_2c+1)[q] at X[q][2c], X[q][2c + 1]
amm_status spectrum_columns_general(amm_ctx* ctx, int n, const float* B, int64_t p, float* X, hipStream_t s) {
  if (p <= 0) return AMM_OK;
  const int64_t P2 = p / 2, cnt = (int64_t)n * P2;
  AMM_TRY(ctx->scratch[8].reserve(cnt * sizeof(double2)));
  double2* z = ctx->scratch[8].as<double2>();
  hipLaunchKernelGGL(pack_pairs, dim3(blocks_for(cnt)), dim3(256), 0, s, B, (int64_t)n, p, P2, z);
  AMM_HIP(hipGetLastError());
  AMM_TRY(dft64_any(ctx, z, n, P2, 1, P2, -1, 1.0, s, false));
  hipLaunchKernelGGL(spectrum_to_f32, dim3(blocks_for(cnt)), dim3(256), 0, s, z, cnt, X);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

// out (rows x n) (+)= X Btil for X (rows x n): the column form on X^T with the
// adjoint lists, transposed back
amm_status cd_apply_rows_general(amm_ctx* ctx, int n, int K, const int32_t* shifts_adj, const float2* Ladj,
                                 const float* X, int64_t rows, float* out, bool acc, hipStream_t s,
                                 const __half2* Ladj16, float l16_inv) {
  if (rows <= 0) return AMM_OK;
  if (n >= 3 && n <= kChirpFusedMax) {
    if (K == 0) return acc ? AMM_OK : fill_f32(out, (int64_t)n * rows, 0.f, s);
    return cd_chirp_apply(ctx, true, n, K, shifts_adj, Ladj, X, rows, out, acc, s, Ladj16, l16_inv);
  }
  AMM_TRY(ctx->scratch[12].reserve((size_t)n * rows * sizeof(float)));
  AMM_TRY(ctx->scratch[13].reserve((size_t)n * rows * sizeof(float)));
  float *xt = ctx->scratch[12].as<float>(), *yt = ctx->scratch[13].as<float>();
  AMM_TRY(transpose_f32(X, rows, n, xt, s));
  AMM_TRY(cd_apply_general(ctx, n, K, shifts_adj, Ladj, xt, rows, yt, false, s));
  AMM_TRY(transpose_acc_f32(yt, n, rows, out, acc, s));
  return AMM_OK;
}

}  // namespace amm
