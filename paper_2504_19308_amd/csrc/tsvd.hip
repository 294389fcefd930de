// Randomized truncated SVD, float64 on the device (Alg. 2.1 of the paper,
// after Halko, Martinsson and Tropp).
//
// Alg. 2.1 sketches Y = A phi with k random columns, orthonormalises Y and
// takes the SVD of Q^T A.  Without oversampling that does not return the best
// rank-k approximation, so the sketch carries `oversample` extra columns and
// `power_iters` subspace iterations (Y <- A A^T Y with re-orthonormalisation),
// both from the same reference; the leading k triplets are kept.
//
// Device work: the tall GEMMs (float64 MFMA), the sketch generator and the
// l x l steps.  For l = k + oversample <= 96 the CholeskyQR factors and the
// Jacobi eigensolver of the Gram matrix (Q^T A)(Q^T A)^T run in one
// workgroup each: the whole decomposition is enqueued without a host round
// trip and read back once at the end.  Up to 2048 columns a blocked
// CholeskyQR and a block one-sided Jacobi on the Cholesky factor take over
// (one flag read per Jacobi sweep, the eigenvalues sorted on the host);
// beyond that, and for k = 0, the l x l steps run on the host.
// Intermediate orthonormalisations of the subspace iteration take one
// shifted CholeskyQR pass (they only need a well-conditioned basis of the
// same span); the final basis takes three (shifted CholeskyQR3).
//
// The sketch entries are N(0,1) from Philox4x32-10 (Salmon et al., 2011) with
// the Box-Muller transform: counter = (element pair index, seed), key fixed.
#include <algorithm>
#include <cmath>
#include <vector>

#include "amm_internal.hpp"

namespace amm {
namespace {

__device__ __forceinline__ void philox_round(uint32_t* c, const uint32_t* k) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__device__ __forceinline__ void philox4x32_10(uint32_t* c, uint32_t k0, uint32_t k1) {
  uint32_t k[2] = {k0, k1};
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
}

__global__ void gaussian_sketch(double* __restrict__ out, int64_t count, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // pair index
  if (2 * i >= count) return;
  uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)seed, (uint32_t)(seed >> 32)};
  philox4x32_10(c, 0x1BD11BDAu, 0x6A09E667u);
  // two uniforms in (0, 1] from 53-bit words
  const uint64_t a = ((uint64_t)c[0] << 21) ^ (uint64_t)(c[1] >> 11);
  const uint64_t b = ((uint64_t)c[2] << 21) ^ (uint64_t)(c[3] >> 11);
  const double u1 = ((double)(a & ((1ull << 53) - 1)) + 1.0) * (1.0 / 9007199254740992.0);
  const double u2 = ((double)(b & ((1ull << 53) - 1)) + 0.5) * (1.0 / 9007199254740992.0);
  const double r = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  out[2 * i] = r * cs;
  if (2 * i + 1 < count) out[2 * i + 1] = r * sn;
}

__global__ void widen_f32(const float* __restrict__ a, double* __restrict__ b, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) b[i] = (double)a[i];
}

__global__ void sumsq_partial(const float* __restrict__ a, int64_t count, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const double v = a[i];
    s += v * v;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void diff_sumsq_partial(const float* __restrict__ x, const float* __restrict__ y, int64_t count,
                                   double* __restrict__ part) {
  __shared__ double sd[256], sx[256];
  double d = 0.0, a = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const double u = x[i], v = u - (double)y[i];
    a += u * u;
    d += v * v;
  }
  sd[threadIdx.x] = d;
  sx[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      sd[threadIdx.x] += sd[threadIdx.x + off];
      sx[threadIdx.x] += sx[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sd[0];
    part[2 * blockIdx.x + 1] = sx[0];
  }
}

// out[i*ldo + j] = (float)(src[i*lds + perm[j]] * (scale ? scale[perm[j]] : 1))
__global__ void pick_columns(const double* __restrict__ src, int64_t rows, int64_t lds,
                             const int32_t* __restrict__ perm, const double* __restrict__ scale,
                             int k, float* __restrict__ out, float* __restrict__ out_scaled,
                             const double* __restrict__ sig) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * k) return;
  const int64_t i = idx / k;
  const int j = (int)(idx % k);
  double v = src[i * lds + perm[j]];
  if (scale) v *= scale[perm[j]];
  out[idx] = (float)v;
  out_scaled[idx] = (float)(v * sig[j]);
}

// Orthonormalise the columns of Y (rows x l, row-major) in place into Q via
// CholeskyQR2 (a shifted first pass guards against a numerically rank-deficient
// sketch).  tmp: rows x l scratch.
amm_status orthonormalise(double* Y, double* tmp, int64_t rows, int l, DevBuf& gram, hipStream_t s) {
  std::vector<double> G(l * l);
  for (int pass = 0; pass < 3; ++pass) {
    AMM_TRY(gemm_f64(l, l, rows, 1.0, Y, 1, l, Y, l, 1, 0.0, gram.as<double>(), l, s));
    AMM_HIP(hipMemcpyAsync(G.data(), gram.ptr, l * l * sizeof(double), hipMemcpyDeviceToHost, s));
    AMM_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < l; ++i)
      for (int j = 0; j < i; ++j) G[i * l + j] = G[j * l + i] = 0.5 * (G[i * l + j] + G[j * l + i]);
    // the first pass is always shifted; a later pass is shifted only if its
    // plain factorisation fails (an exactly rank-deficient operand: the extra
    // columns then carry singular values at rounding level)
    double nrm = 0.0;
    for (int i = 0; i < l; ++i) nrm += G[i * l + i];
    const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 1.1102230246251565e-16 * nrm;
    std::vector<double> G0;
    if (pass > 0) G0 = G;
    if (pass == 0)
      for (int i = 0; i < l; ++i) G[i * l + i] += shift;
    if (!cholesky_upper(G, l)) {
      if (pass == 0) return fail(AMM_EDEVICE, "CholeskyQR broke down (sketch rank-deficient)");
      G = G0;
      for (int i = 0; i < l; ++i) G[i * l + i] += shift;
      if (!cholesky_upper(G, l)) return fail(AMM_EDEVICE, "CholeskyQR broke down (sketch rank-deficient)");
    }
    std::vector<double> Ri = inv_upper(G, l);
    AMM_HIP(hipMemcpyAsync(gram.ptr, Ri.data(), l * l * sizeof(double), hipMemcpyHostToDevice, s));
    AMM_TRY(gemm_f64(rows, l, l, 1.0, Y, l, 1, gram.as<double>(), l, 1, 0.0, tmp, l, s));
    AMM_HIP(hipMemcpyAsync(Y, tmp, rows * l * sizeof(double), hipMemcpyDeviceToDevice, s));
    AMM_HIP(hipStreamSynchronize(s));
  }
  return AMM_OK;
}

}  // namespace

amm_status sumsq_f32(const float* x, int64_t count, hipStream_t s, double* out) {
  *out = 0.0;
  if (count <= 0) return AMM_OK;
  const int blocks = (int)std::min<int64_t>(1024, (count + 255) / 256);
  DevBuf part;
  AMM_TRY(part.alloc(blocks * sizeof(double)));
  hipLaunchKernelGGL(sumsq_partial, dim3(blocks), dim3(256), 0, s, x, count, part.as<double>());
  AMM_HIP(hipGetLastError());
  std::vector<double> h(blocks);
  AMM_HIP(hipMemcpyAsync(h.data(), part.ptr, blocks * sizeof(double), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipStreamSynchronize(s));
  double t = 0.0;
  for (double v : h) t += v;
  *out = t;
  return AMM_OK;
}

amm_status diff_sumsq_f32(const float* x, const float* y, int64_t count, hipStream_t s, double* dd, double* xx) {
  *dd = *xx = 0.0;
  if (count <= 0) return AMM_OK;
  const int blocks = (int)std::min<int64_t>(1024, (count + 255) / 256);
  DevBuf part;
  AMM_TRY(part.alloc(2 * blocks * sizeof(double)));
  hipLaunchKernelGGL(diff_sumsq_partial, dim3(blocks), dim3(256), 0, s, x, y, count, part.as<double>());
  AMM_HIP(hipGetLastError());
  std::vector<double> h(2 * blocks);
  AMM_HIP(hipMemcpyAsync(h.data(), part.ptr, 2 * blocks * sizeof(double), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < blocks; ++b) {
    *dd += h[2 * b];
    *xx += h[2 * b + 1];
  }
  return AMM_OK;
}

namespace {

amm_status tsvd_decompose_host(amm_ctx* ctx, const float* A, int64_t m, int64_t n, int k,
                               const amm_opts* o, amm_dec* dec, hipStream_t s) {
  const int64_t mn = std::min(m, n);
  const int l = (int)std::min<int64_t>(mn, (int64_t)k + std::max(o->oversample, 0));
  const int q = std::max(o->power_iters, 0);
  dec->K_eff = k;
  // ||A||_F
  {
    double t = 0.0;
    AMM_TRY(sumsq_f32(A, m * n, s, &t));
    dec->norm_A = std::sqrt(t);
  }
  const int64_t kk = std::max(k, 1);
  AMM_TRY(dec->U.alloc(m * kk * 4));
  AMM_TRY(dec->US.alloc(m * kk * 4));
  AMM_TRY(dec->V.alloc(n * kk * 4));
  AMM_TRY(dec->VS.alloc(n * kk * 4));
  AMM_TRY(dec->VSt.alloc(n * kk * 4));
  AMM_TRY(dec->Vt.alloc(n * kk * 4));
  AMM_TRY(dec->sigma.alloc(kk * 4));
  if (k == 0 || dec->norm_A == 0.0) {
    // nothing to keep (a zero operand has no nonzero singular triplet)
    dec->K_eff = 0;
    dec->norm_residual = dec->norm_A;
    if (dec->norm_A == 0.0) dec->sigma_next = 0.0;
    return AMM_OK;
  }
  // work buffers come from the context's grow-only areas: repeated decompositions
  // allocate (and free) nothing once the areas have grown
  DevBuf* ws = ctx->rsvd;
  DevBuf &A64 = ws[0], &Om = ws[1], &Y = ws[2], &Z = ws[3], &T1 = ws[4], &gram = ws[5], &Bs = ws[6];
  AMM_TRY(A64.reserve(m * n * sizeof(double)));
  AMM_TRY(Om.reserve(n * l * sizeof(double)));
  AMM_TRY(Y.reserve(m * l * sizeof(double)));
  AMM_TRY(Z.reserve(n * l * sizeof(double)));
  AMM_TRY(T1.reserve(std::max(m, n) * l * sizeof(double)));
  AMM_TRY(gram.reserve(l * l * sizeof(double)));
  AMM_TRY(Bs.reserve(l * n * sizeof(double)));
  hipLaunchKernelGGL(widen_f32, dim3((unsigned)((m * n + 255) / 256)), dim3(256), 0, s, A, A64.as<double>(), m * n);
  const int64_t cnt = n * l;
  hipLaunchKernelGGL(gaussian_sketch, dim3((unsigned)((cnt / 2 + 256) / 256)), dim3(256), 0, s, Om.as<double>(), cnt, o->seed);
  AMM_HIP(hipGetLastError());
  const double* Ad = A64.as<double>();
  // Y = A Omega
  AMM_TRY(gemm_f64(m, l, n, 1.0, Ad, n, 1, Om.as<double>(), l, 1, 0.0, Y.as<double>(), l, s));
  AMM_TRY(orthonormalise(Y.as<double>(), T1.as<double>(), m, l, gram, s));
  for (int it = 0; it < q; ++it) {
    // Z = A^T Q, orthonormalise; Y = A Z, orthonormalise
    AMM_TRY(gemm_f64(n, l, m, 1.0, Ad, 1, n, Y.as<double>(), l, 1, 0.0, Z.as<double>(), l, s));
    AMM_TRY(orthonormalise(Z.as<double>(), T1.as<double>(), n, l, gram, s));
    AMM_TRY(gemm_f64(m, l, n, 1.0, Ad, n, 1, Z.as<double>(), l, 1, 0.0, Y.as<double>(), l, s));
    AMM_TRY(orthonormalise(Y.as<double>(), T1.as<double>(), m, l, gram, s));
  }
  // Bs = Q^T A  (l x n)
  AMM_TRY(gemm_f64(l, n, m, 1.0, Y.as<double>(), 1, l, Ad, n, 1, 0.0, Bs.as<double>(), n, s));
  // Gram = Bs Bs^T = W diag(lam) W^T  (host Jacobi)
  AMM_TRY(gemm_f64(l, l, n, 1.0, Bs.as<double>(), n, 1, Bs.as<double>(), 1, n, 0.0, gram.as<double>(), l, s));
  std::vector<double> G(l * l), lam, W;
  AMM_HIP(hipMemcpyAsync(G.data(), gram.ptr, l * l * sizeof(double), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < l; ++i)
    for (int j = 0; j < i; ++j) G[i * l + j] = G[j * l + i] = 0.5 * (G[i * l + j] + G[j * l + i]);
  jacobi_eig(G, l, lam, W);
  std::vector<int32_t> order(l);
  for (int i = 0; i < l; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return lam[a] > lam[b]; });
  std::vector<double> sig(l), inv_sig(l, 0.0);
  for (int i = 0; i < l; ++i) {
    sig[i] = std::sqrt(std::max(lam[i], 0.0));
    inv_sig[i] = sig[i] > 0 ? 1.0 / sig[i] : 0.0;
  }
  std::vector<double> sig_k(k);
  std::vector<float> sig_f(k);
  double kept = 0.0;
  for (int j = 0; j < k; ++j) {
    sig_k[j] = sig[order[j]];
    sig_f[j] = (float)sig_k[j];
    kept += sig_k[j] * sig_k[j];
  }
  dec->norm_residual = std::sqrt(std::max(dec->norm_A * dec->norm_A - kept, 0.0));
  dec->sigma64 = sig_k;
  // the sketch's (k+1)-th singular value estimates ||Delta A||_2 (Thm. 3.8)
  if (k < l) dec->sigma_next = sig[order[k]];
  else if (k == mn) dec->sigma_next = 0.0;
  // U_full = Q W (m x l), V_full = Bs^T W diag(1/sig) (n x l)
  DevBuf &Wd = ws[7], &Uf = ws[8], &Vf = ws[9];
  DevBuf perm, isg, sgk;
  AMM_TRY(Wd.reserve(l * l * sizeof(double)));
  AMM_TRY(Uf.reserve(m * l * sizeof(double)));
  AMM_TRY(Vf.reserve(n * l * sizeof(double)));
  AMM_TRY(perm.alloc(l * 4));
  AMM_TRY(isg.alloc(l * sizeof(double)));
  AMM_TRY(sgk.alloc(k * sizeof(double)));
  AMM_HIP(hipMemcpyAsync(Wd.ptr, W.data(), l * l * sizeof(double), hipMemcpyHostToDevice, s));
  AMM_HIP(hipMemcpyAsync(perm.ptr, order.data(), l * 4, hipMemcpyHostToDevice, s));
  AMM_HIP(hipMemcpyAsync(isg.ptr, inv_sig.data(), l * sizeof(double), hipMemcpyHostToDevice, s));
  AMM_HIP(hipMemcpyAsync(sgk.ptr, sig_k.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
  AMM_TRY(gemm_f64(m, l, l, 1.0, Y.as<double>(), l, 1, Wd.as<double>(), l, 1, 0.0, Uf.as<double>(), l, s));
  AMM_TRY(gemm_f64(n, l, l, 1.0, Bs.as<double>(), 1, n, Wd.as<double>(), l, 1, 0.0, Vf.as<double>(), l, s));
  hipLaunchKernelGGL(pick_columns, dim3((unsigned)((m * k + 255) / 256)), dim3(256), 0, s, Uf.as<double>(), m,
                     (int64_t)l, perm.as<int32_t>(), (const double*)nullptr, k, dec->U.as<float>(),
                     dec->US.as<float>(), sgk.as<double>());
  hipLaunchKernelGGL(pick_columns, dim3((unsigned)((n * k + 255) / 256)), dim3(256), 0, s, Vf.as<double>(), n,
                     (int64_t)l, perm.as<int32_t>(), isg.as<double>(), k, dec->V.as<float>(),
                     dec->VS.as<float>(), sgk.as<double>());
  AMM_HIP(hipGetLastError());
  AMM_TRY(transpose_f32(dec->VS.as<float>(), n, k, dec->VSt.as<float>(), s));
  AMM_TRY(transpose_f32(dec->V.as<float>(), n, k, dec->Vt.as<float>(), s));
  AMM_HIP(hipMemcpyAsync(dec->sigma.ptr, sig_f.data(), k * 4, hipMemcpyHostToDevice, s));
  AMM_HIP(hipStreamSynchronize(s));
  return AMM_OK;
}

// Orthonormalise the columns of *cur (rows x l) through `passes` CholeskyQR
// passes on the device (the first shifted); each pass writes Q = Y R^-1 into
// the other buffer and swaps the two.
// Work of the l x l steps: rinv (l x l) for sketches up to 96 columns; R
// (l x l), the inverse diagonal blocks E and a panel P for larger ones.
struct SmallWork {
  double* rinv;
  double* R;
  double* E;
  double* P;
  int* status;
};

amm_status orthonormalise_dev(double** cur, double** alt, int64_t rows, int l, int passes, double* gram,
                              const SmallWork& w, hipStream_t s) {
  for (int pass = 0; pass < passes; ++pass) {
    AMM_TRY(gemm_f64(l, l, rows, 1.0, *cur, 1, l, *cur, l, 1, 0.0, gram, l, s));
    if (l <= kSmallEigMax) {
      AMM_TRY(chol_qr_factor(gram, l, rows, pass == 0 ? 0 : 1, w.rinv, w.status, s));
      AMM_TRY(gemm_f64(rows, l, l, 1.0, *cur, l, 1, w.rinv, l, 1, 0.0, *alt, l, s));
    } else {
      AMM_TRY(chol_qr_blocked(gram, l, rows, pass == 0, w.R, w.E, w.status, s));
      AMM_TRY(chol_qr_apply(*cur, rows, l, w.R, w.E, *alt, w.P, s));
    }
    std::swap(*cur, *alt);
  }
  return AMM_OK;
}

__global__ void set_i32(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// The decomposition with every step on the device and, for sketches up to 96
// columns, a single read-back of the singular values, the norm partial sums
// and the breakdown flag at the end (larger sketches read the flag of each
// Jacobi sweep and the eigenvalues, which they sort on the host).
amm_status tsvd_decompose_device(amm_ctx* ctx, const float* A, int64_t m, int64_t n, int k, int l, int q,
                                 const amm_opts* o, amm_dec* dec, hipStream_t s) {
  const int64_t mn = std::min(m, n);
  DevBuf* ws = ctx->rsvd;
  DevBuf &A64 = ws[0], &Om = ws[1], &Y = ws[2], &Z = ws[3], &Y2 = ws[4], &gram = ws[5], &Bs = ws[6];
  DevBuf &Wd = ws[7], &Uf = ws[8], &Vf = ws[9], &Z2 = ws[10], &small = ws[11], &big = ws[12];
  constexpr int kParts = 1024;
  AMM_TRY(A64.reserve(m * n * sizeof(double)));
  AMM_TRY(Om.reserve(n * l * sizeof(double)));
  AMM_TRY(Y.reserve(m * l * sizeof(double)));
  AMM_TRY(Y2.reserve(m * l * sizeof(double)));
  AMM_TRY(Z.reserve(n * l * sizeof(double)));
  AMM_TRY(Z2.reserve(n * l * sizeof(double)));
  AMM_TRY(gram.reserve(l * l * sizeof(double)));
  AMM_TRY(Bs.reserve(l * n * sizeof(double)));
  AMM_TRY(Wd.reserve(l * l * sizeof(double)));
  AMM_TRY(Uf.reserve(m * l * sizeof(double)));
  AMM_TRY(Vf.reserve(n * l * sizeof(double)));
  // small: [sig_sorted l | norm partials kParts | isg l | sgk l | rinv l*l] doubles, then perm l, status 1 int32
  const size_t nd = (size_t)3 * l + kParts + (size_t)l * l;
  AMM_TRY(small.reserve(nd * sizeof(double) + (l + 1) * sizeof(int32_t)));
  double* sig_sorted = small.as<double>();
  double* parts = sig_sorted + l;
  double* isg = parts + kParts;
  double* sgk = isg + l;
  double* rinv = sgk + l;
  int32_t* perm = reinterpret_cast<int32_t*>(rinv + (size_t)l * l);
  int* status = perm + l;
  SmallWork w{rinv, nullptr, nullptr, nullptr, status};
  const bool large = l > kSmallEigMax;
  if (large) {
    // R (l x l), E (64 x 64 per diagonal block), P (l x 64), the sweep flag
    const size_t nr = (size_t)l * l, ne = (size_t)chol_blocks(l) * 64 * 64, npn = (size_t)l * 64;
    AMM_TRY(big.reserve((nr + ne + npn) * sizeof(double) + 16));
    w.R = big.as<double>();
    w.E = w.R + nr;
    w.P = w.E + ne;
  }
  int* flag = large ? reinterpret_cast<int*>(w.P + (size_t)l * 64) : nullptr;
  hipLaunchKernelGGL(set_i32, dim3(1), dim3(64), 0, s, status, 0);
  // ||A||_F partial sums (read with the results)
  const int blocks = (int)std::min<int64_t>(kParts, (m * n + 255) / 256);
  hipLaunchKernelGGL(sumsq_partial, dim3(blocks), dim3(256), 0, s, A, m * n, parts);
  hipLaunchKernelGGL(widen_f32, dim3((unsigned)((m * n + 255) / 256)), dim3(256), 0, s, A, A64.as<double>(), m * n);
  const int64_t cnt = n * l;
  hipLaunchKernelGGL(gaussian_sketch, dim3((unsigned)((cnt / 2 + 256) / 256)), dim3(256), 0, s, Om.as<double>(), cnt,
                     o->seed);
  AMM_HIP(hipGetLastError());
  const double* Ad = A64.as<double>();
  double *y = Y.as<double>(), *y2 = Y2.as<double>(), *z = Z.as<double>(), *z2 = Z2.as<double>();
  // Y = A Omega
  AMM_TRY(gemm_f64(m, l, n, 1.0, Ad, n, 1, Om.as<double>(), l, 1, 0.0, y, l, s));
  AMM_TRY(orthonormalise_dev(&y, &y2, m, l, q > 0 ? 1 : 3, gram.as<double>(), w, s));
  for (int it = 0; it < q; ++it) {
    // Z = A^T Q, orthonormalise; Y = A Z, orthonormalise (three passes for the final basis)
    AMM_TRY(gemm_f64(n, l, m, 1.0, Ad, 1, n, y, l, 1, 0.0, z, l, s));
    AMM_TRY(orthonormalise_dev(&z, &z2, n, l, 1, gram.as<double>(), w, s));
    AMM_TRY(gemm_f64(m, l, n, 1.0, Ad, n, 1, z, l, 1, 0.0, y, l, s));
    AMM_TRY(orthonormalise_dev(&y, &y2, m, l, it + 1 == q ? 3 : 1, gram.as<double>(), w, s));
  }
  // Bs = Q^T A (l x n); its Gram matrix Bs Bs^T = W diag(lam) W^T
  AMM_TRY(gemm_f64(l, n, m, 1.0, y, 1, l, Ad, n, 1, 0.0, Bs.as<double>(), n, s));
  AMM_TRY(gemm_f64(l, l, n, 1.0, Bs.as<double>(), n, 1, Bs.as<double>(), 1, n, 0.0, gram.as<double>(), l, s));
  // W element (i, j) = component i of eigenvector j: row-major from the one-workgroup solver,
  // contiguous eigenvectors (column-major) from the one-sided Jacobi
  int64_t w_rs = l, w_cs = 1;
  if (!large) {
    AMM_TRY(gram_eig(gram.as<double>(), l, n, k, Wd.as<double>(), perm, isg, sgk, dec->sigma.as<float>(), sig_sorted,
                     status, s));
  } else {
    std::vector<double> lam;
    AMM_TRY(gram_eig_large(gram.as<double>(), l, n, w.R, w.E, Wd.as<double>(), rinv, flag, status, lam, nullptr, s));
    // descending order (ties by index), sigma = sqrt(lam), 1/sigma, the leading k
    std::vector<int32_t> order(l);
    for (int i = 0; i < l; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lam[a] > lam[b]; });
    std::vector<double> ss(l), inv(l), sk(std::max(k, 1));
    std::vector<float> sf(std::max(k, 1));
    for (int j = 0; j < l; ++j) ss[j] = std::sqrt(std::max(lam[order[j]], 0.0));
    for (int i = 0; i < l; ++i) {
      const double sg = std::sqrt(std::max(lam[i], 0.0));
      inv[i] = sg > 0.0 ? 1.0 / sg : 0.0;
    }
    for (int j = 0; j < k; ++j) {
      sk[j] = ss[j];
      sf[j] = (float)ss[j];
    }
    AMM_HIP(hipMemcpyAsync(perm, order.data(), l * sizeof(int32_t), hipMemcpyHostToDevice, s));
    AMM_HIP(hipMemcpyAsync(isg, inv.data(), l * sizeof(double), hipMemcpyHostToDevice, s));
    AMM_HIP(hipMemcpyAsync(sgk, sk.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
    AMM_HIP(hipMemcpyAsync(sig_sorted, ss.data(), l * sizeof(double), hipMemcpyHostToDevice, s));
    AMM_HIP(hipMemcpyAsync(dec->sigma.ptr, sf.data(), k * sizeof(float), hipMemcpyHostToDevice, s));
    w_rs = 1;
    w_cs = l;
  }
  // U_full = Q W (m x l), V_full = Bs^T W diag(1/sig) (n x l); the leading k columns in descending order
  AMM_TRY(gemm_f64(m, l, l, 1.0, y, l, 1, Wd.as<double>(), w_rs, w_cs, 0.0, Uf.as<double>(), l, s));
  AMM_TRY(gemm_f64(n, l, l, 1.0, Bs.as<double>(), 1, n, Wd.as<double>(), w_rs, w_cs, 0.0, Vf.as<double>(), l, s));
  hipLaunchKernelGGL(pick_columns, dim3((unsigned)((m * k + 255) / 256)), dim3(256), 0, s, Uf.as<double>(), m,
                     (int64_t)l, perm, (const double*)nullptr, k, dec->U.as<float>(), dec->US.as<float>(), sgk);
  hipLaunchKernelGGL(pick_columns, dim3((unsigned)((n * k + 255) / 256)), dim3(256), 0, s, Vf.as<double>(), n,
                     (int64_t)l, perm, isg, k, dec->V.as<float>(), dec->VS.as<float>(), sgk);
  AMM_HIP(hipGetLastError());
  AMM_TRY(transpose_f32(dec->VS.as<float>(), n, k, dec->VSt.as<float>(), s));
  AMM_TRY(transpose_f32(dec->V.as<float>(), n, k, dec->Vt.as<float>(), s));
  // one read-back: singular values, norm partial sums, breakdown flag
  std::vector<double> h((size_t)l + blocks);
  int st = 0;
  AMM_HIP(hipMemcpyAsync(h.data(), sig_sorted, ((size_t)l + blocks) * sizeof(double), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipStreamSynchronize(s));
  double a2 = 0.0;
  for (int b = 0; b < blocks; ++b) a2 += h[l + b];
  dec->norm_A = std::sqrt(a2);
  if (dec->norm_A == 0.0) {
    // a zero operand has no nonzero singular triplet
    dec->K_eff = 0;
    dec->norm_residual = 0.0;
    dec->sigma_next = 0.0;
    return AMM_OK;
  }
  if (st != 0) return fail(AMM_EDEVICE, "CholeskyQR broke down (sketch rank-deficient)");
  std::vector<double> sig_k(h.begin(), h.begin() + k);
  double kept = 0.0;
  for (double v : sig_k) kept += v * v;
  dec->norm_residual = std::sqrt(std::max(dec->norm_A * dec->norm_A - kept, 0.0));
  dec->sigma64 = sig_k;
  // the sketch's (k+1)-th singular value estimates ||Delta A||_2 (Thm. 3.8)
  if (k < l) dec->sigma_next = h[k];
  else if (k == mn) dec->sigma_next = 0.0;
  return AMM_OK;
}

}  // namespace

constexpr int kLargeSketchMax = 2048;

amm_status tsvd_decompose(amm_ctx* ctx, const float* A, int64_t m, int64_t n, int k, const amm_opts* o, amm_dec* dec,
                          hipStream_t s) {
  const int64_t mn = std::min(m, n);
  const int l = (int)std::min<int64_t>(mn, (int64_t)k + std::max(o->oversample, 0));
  const int q = std::max(o->power_iters, 0);
  // the host path remains for k = 0 (nothing to keep) and sketches beyond kLargeSketchMax
  if (k == 0 || l > kLargeSketchMax) return tsvd_decompose_host(ctx, A, m, n, k, o, dec, s);
  dec->K_eff = k;
  const int64_t kk = std::max(k, 1);
  AMM_TRY(dec->U.alloc(m * kk * 4));
  AMM_TRY(dec->US.alloc(m * kk * 4));
  AMM_TRY(dec->V.alloc(n * kk * 4));
  AMM_TRY(dec->VS.alloc(n * kk * 4));
  AMM_TRY(dec->VSt.alloc(n * kk * 4));
  AMM_TRY(dec->Vt.alloc(n * kk * 4));
  AMM_TRY(dec->sigma.alloc(kk * 4));
  return tsvd_decompose_device(ctx, A, m, n, k, l, q, o, dec, s);
}

}  // namespace amm
