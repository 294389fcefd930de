// Backward of the approximate product with a frozen truncation structure.
//
// For a layer Y = P(W) X, where P maps W to its truncation with the structure
// held fixed (kept circulant frequencies S, singular subspaces U_k / V_k, the
// sparse pattern Omega), P is linear, so
//     dX = P(W)^T dY,      dW = P^T(dY X^T).
// The circulant and SVD projections are orthogonal (Rem. 1.2 of the paper for
// the circulant case), hence self-adjoint:
//   SVD:        P(G) = U U^T G V V^T
//               dX = V S (U^T dY),  dW = U [(U^T dY)(V^T X)^T] V^T
//   circulant:  P(G) = sum_{k in S} R_k(G) D^k; the needed eigenvalue lists of
//               P(dY X^T) are the kept wrapped diagonals of F (dY X^T) F^-1:
//                 Lg_k[p] = (1/n) sum_c Yh_c[p] conj(Xh_c[(p - k) mod n]),
//               a sampled product of the column spectra of dY and X (no m x n
//               product is formed); dW = sum_t R^G_t D^{k_t} is then the same
//               spectral operator applied to the identity.
//   sparse:     P(G) = G o Omega + P_in(G o Omega^c), with adjoint
//               G o Omega + P_in(G) o Omega^c; dX = S^T dY + P_in(W_R)^T dY.
#include <vector>

#include "amm_internal.hpp"

namespace amm {
namespace {

__global__ void set_identity(float* __restrict__ I, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * n) I[i] = (i / n == i % n) ? 1.f : 0.f;
}

// Lg_t[p] = 1/(2n) sum_pairs [ Zy[p] conj(Zx[q]) + conj(Zy[-p]) Zx[-q] ],  q = p - k_t,
// where Zy, Zx are the spectra of packed column pairs (two real columns per
// complex column): the sum over the two real columns of a pair equals half of
// the bracket.  One block per bin p; threads stride over the pairs.
__global__ void __launch_bounds__(256)
spectral_sddmm(const float2* __restrict__ Zy, const float2* __restrict__ Zx, int n, int64_t pairs,
               int K, const int32_t* __restrict__ shifts, float2* __restrict__ Lg) {
  __shared__ float2 red[256];
  const int p = blockIdx.x;
  const int pm = p == 0 ? 0 : n - p;
  const float2* yp = Zy + (int64_t)p * pairs;
  const float2* ym = Zy + (int64_t)pm * pairs;
  const float sc = 0.5f / (float)n;
  for (int t = 0; t < K; ++t) {
    int q = p - shifts[t];
    if (q < 0) q += n;
    const int qm = q == 0 ? 0 : n - q;
    const float2* xq = Zx + (int64_t)q * pairs;
    const float2* xm = Zx + (int64_t)qm * pairs;
    float ar = 0.f, ai = 0.f;
    for (int64_t c = threadIdx.x; c < pairs; c += blockDim.x) {
      const float2 a = yp[c], b = xq[c], u = ym[c], v = xm[c];
      // a conj(b) + conj(u) v
      ar += a.x * b.x + a.y * b.y + u.x * v.x + u.y * v.y;
      ai += a.y * b.x - a.x * b.y + u.x * v.y - u.y * v.x;
    }
    red[threadIdx.x] = float2{ar, ai};
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        red[threadIdx.x].x += red[threadIdx.x + off].x;
        red[threadIdx.x].y += red[threadIdx.x + off].y;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) Lg[(int64_t)t * n + p] = float2{red[0].x * sc, red[0].y * sc};
    __syncthreads();
  }
}

// dW[i, j] = sum_c dY[i, c] X[j, c] for the stored entries (i, j) of a CSR
// pattern; one block per row i with dY's row staged in LDS.
__global__ void __launch_bounds__(256)
pattern_sddmm(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
              const float* __restrict__ dY, const float* __restrict__ X, int64_t p, int64_t ldw,
              float* __restrict__ dW) {
  extern __shared__ float yrow[];
  __shared__ float red[256];
  const int64_t i = blockIdx.x;
  for (int64_t c = threadIdx.x; c < p; c += blockDim.x) yrow[c] = dY[i * p + c];
  __syncthreads();
  for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    const int64_t j = col[e];
    float acc = 0.f;
    for (int64_t c = threadIdx.x; c < p; c += blockDim.x) acc += yrow[c] * X[j * p + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) dW[i * ldw + j] = red[0];
    __syncthreads();
  }
}

// zero the stored positions of a CSR pattern in a dense matrix
__global__ void pattern_zero(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                             int64_t rows, int64_t ldw, float* __restrict__ W) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (i >= rows) return;
  for (int e = row_ptr[i] + threadIdx.x; e < row_ptr[i + 1]; e += blockDim.x) W[i * ldw + col[e]] = 0.f;
}

amm_status bw_tsvd(amm_ctx* ctx, const amm_dec* d, const float* X, const float* dY, int64_t p,
                   float* dX, float* dW, bool acc_dx, hipStream_t s) {
  const int64_t m = d->m, n = d->n;
  const int k = d->K_eff;
  if (k == 0) {
    if (dX && !acc_dx) AMM_TRY(fill_f32(dX, n * p, 0.f, s));
    if (dW) AMM_TRY(fill_f32(dW, m * n, 0.f, s));
    return AMM_OK;
  }
  AMM_TRY(ctx->scratch[0].reserve((size_t)k * p * sizeof(float)));
  float* Gy = ctx->scratch[0].as<float>();
  // Gy = U^T dY  (k x p)
  if (panel_full_ok(k, p)) AMM_TRY(panel_full(k, m, d->U.as<float>(), dY, p, Gy, s));
  else AMM_TRY(gemm_f32(k, p, m, 1.f, MatView{d->U.as<float>(), 1, k}, MatView{dY, p, 1}, 0.f, Gy, p, s, "gemm_UtdY"));
  if (dX) {
    // dX (+)= (V S) Gy
    if (!acc_dx && gemm_short_ok(n, p, k)) AMM_TRY(gemm_short(n, p, k, d->VS.as<float>(), Gy, dX, s));
    else AMM_TRY(gemm_f32(n, p, k, 1.f, MatView{d->VS.as<float>(), k, 1}, MatView{Gy, p, 1}, acc_dx ? 1.f : 0.f, dX, p, s, "gemm_out"));
  }
  if (dW) {
    AMM_TRY(ctx->scratch[1].reserve((size_t)k * p * sizeof(float)));
    AMM_TRY(ctx->scratch[3].reserve((size_t)k * k * sizeof(float)));
    AMM_TRY(ctx->scratch[2].reserve((size_t)m * k * sizeof(float)));
    float* Gx = ctx->scratch[1].as<float>();
    float* core = ctx->scratch[3].as<float>();
    float* UC = ctx->scratch[2].as<float>();
    // Gx = V^T X (k x p);  core = Gy Gx^T (k x k);  UC = U core;  dW = UC V^T
    if (panel_full_ok(k, p)) AMM_TRY(panel_full(k, n, d->V.as<float>(), X, p, Gx, s));
    else AMM_TRY(gemm_f32(k, p, n, 1.f, MatView{d->V.as<float>(), 1, k}, MatView{X, p, 1}, 0.f, Gx, p, s, "gemm_VtX"));
    AMM_TRY(gemm_f32(k, k, p, 1.f, MatView{Gy, p, 1}, MatView{Gx, 1, p}, 0.f, core, k, s, "gemm_core"));
    AMM_TRY(gemm_f32(m, k, k, 1.f, MatView{d->U.as<float>(), k, 1}, MatView{core, k, 1}, 0.f, UC, k, s, "gemm_small"));
    if (gemm_short_ok(m, n, k) && d->Vt.ptr) AMM_TRY(gemm_short(m, n, k, UC, d->Vt.as<float>(), dW, s));
    else AMM_TRY(gemm_f32(m, n, k, 1.f, MatView{UC, k, 1}, MatView{d->V.as<float>(), 1, k}, 0.f, dW, n, s, "gemm_dW"));
  }
  return AMM_OK;
}

int ilog2(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}

amm_status bw_circulant(amm_ctx* ctx, const amm_dec* d, const float* X, const float* dY, int64_t p,
                        float* dX, float* dW, bool acc_dx, hipStream_t s) {
  const int64_t n = d->n;
  const bool pow2 = (n & (n - 1)) == 0;   // other sides: the chirp-convolution path
  const int l2 = ilog2(n);
  const int K = d->K_eff;
  if (dX) {
    if (K == 0) {
      if (!acc_dx) AMM_TRY(fill_f32(dX, n * p, 0.f, s));
    } else if (pow2) {
      AMM_TRY(cd_apply_columns(ctx, l2, K, d->shifts_adj.as<int32_t>(), d->Ladj.as<float2>(), dY, p, dX, acc_dx, s,
                               d->pairs_of(true), d->lists16(true), d->l16_inv));
    } else {
      AMM_TRY(cd_apply_general(ctx, (int)n, K, d->shifts_adj.as<int32_t>(), d->Ladj.as<float2>(), dY, p, dX, acc_dx,
                               s));
    }
  }
  if (dW) {
    if (K == 0) return fill_f32(dW, n * n, 0.f, s);
    if (p % 2) return fail(AMM_EUNSUPPORTED, "circulant dW needs an even number of columns");
    AMM_TRY(ctx->scratch[0].reserve((size_t)n * p * sizeof(float)));
    AMM_TRY(ctx->scratch[1].reserve((size_t)n * p * sizeof(float)));
    AMM_TRY(ctx->scratch[2].reserve((size_t)n * n * sizeof(float)));
    AMM_TRY(ctx->scratch[3].reserve((size_t)K * n * sizeof(float2)));
    float* Zy = ctx->scratch[0].as<float>();
    float* Zx = ctx->scratch[1].as<float>();
    float* I = ctx->scratch[2].as<float>();
    float2* Lg = ctx->scratch[3].as<float2>();
    if (pow2) {
      AMM_TRY(cd_spectrum_columns(ctx, l2, dY, p, Zy, s));
      AMM_TRY(cd_spectrum_columns(ctx, l2, X, p, Zx, s));
    } else {
      AMM_TRY(spectrum_columns_general(ctx, (int)n, dY, p, Zy, s));
      AMM_TRY(spectrum_columns_general(ctx, (int)n, X, p, Zx, s));
    }
    {
      TimedLaunch tl("spectral_sddmm", s);
      hipLaunchKernelGGL(spectral_sddmm, dim3((unsigned)n), dim3(256), 0, s, (const float2*)Zy, (const float2*)Zx,
                         (int)n, p / 2, K, d->shifts.as<int32_t>(), Lg);
      AMM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(set_identity, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, I, n);
    AMM_HIP(hipGetLastError());
    if (pow2) AMM_TRY(cd_apply_columns(ctx, l2, K, d->shifts.as<int32_t>(), Lg, I, n, dW, false, s));
    else AMM_TRY(cd_apply_general(ctx, (int)n, K, d->shifts.as<int32_t>(), Lg, I, n, dW, false, s));
  }
  return AMM_OK;
}

amm_status bw_any(amm_ctx* ctx, const amm_dec* d, const float* X, const float* dY, int64_t p, float* dX,
                  float* dW, bool acc_dx, hipStream_t s);

amm_status bw_sparse(amm_ctx* ctx, const amm_dec* d, const float* X, const float* dY, int64_t p, float* dX,
                     float* dW, bool acc_dx, hipStream_t s) {
  const int64_t m = d->m, n = d->n;
  if (dX) {
    // S^T dY: the CSC arrays are the CSR of S^T (n rows)
    AMM_TRY(spmm_raw(d->csc_ptr.as<int32_t>(), d->csc_row.as<int32_t>(), d->csc_val.as<float>(), n, dY, p, dX,
                     acc_dx, s, d->csc_blk.as<int32_t>(), d->csc_blocks));
  }
  if (dW) {
    if (d->inner) {
      AMM_TRY(bw_any(ctx, d->inner, X, dY, p, nullptr, dW, false, s));
      if (d->nnz > 0) {
        dim3 blk(64, 4);
        hipLaunchKernelGGL(pattern_zero, dim3((unsigned)((m + 3) / 4)), blk, 0, s, d->row_ptr.as<int32_t>(),
                           d->col.as<int32_t>(), m, n, dW);
        AMM_HIP(hipGetLastError());
      }
    } else {
      AMM_TRY(fill_f32(dW, m * n, 0.f, s));
    }
    if (d->nnz > 0) {
      const size_t lds = (size_t)p * sizeof(float);
      if (lds > 150 * 1024) return fail(AMM_EUNSUPPORTED, "too many columns for the pattern product");
      if (lds > 64 * 1024)
        AMM_HIP(hipFuncSetAttribute((const void*)pattern_sddmm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      TimedLaunch tl("pattern_sddmm", s);
      hipLaunchKernelGGL(pattern_sddmm, dim3((unsigned)m), dim3(256), lds, s, d->row_ptr.as<int32_t>(),
                         d->col.as<int32_t>(), dY, X, p, n, dW);
      AMM_HIP(hipGetLastError());
    }
  }
  if (dX && d->inner) AMM_TRY(bw_any(ctx, d->inner, X, dY, p, dX, nullptr, true, s));
  return AMM_OK;
}

amm_status bw_any(amm_ctx* ctx, const amm_dec* d, const float* X, const float* dY, int64_t p, float* dX,
                  float* dW, bool acc_dx, hipStream_t s) {
  if (d->kind & AMM_SPARSE) return bw_sparse(ctx, d, X, dY, p, dX, dW, acc_dx, s);
  if (d->kind == AMM_CIRCULANT) return bw_circulant(ctx, d, X, dY, p, dX, dW, acc_dx, s);
  if (d->kind == AMM_TSVD) return bw_tsvd(ctx, d, X, dY, p, dX, dW, acc_dx, s);
  return fail(AMM_EUNSUPPORTED, "no backward for this decomposition kind");
}

}  // namespace

amm_status approx_backward(amm_ctx* ctx, const amm_dec* d, const float* X, const float* dY, int64_t p,
                           float* dX, float* dW, hipStream_t s) {
  return bw_any(ctx, d, X, dY, p, dX, dW, false, s);
}

}  // namespace amm
