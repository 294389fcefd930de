// Circulant decomposition on the device, float64 (Thm. 1.1, Alg. 2.2,
// Alg. 2.3 steps 2-4 and step 6's residual).
//
// The paper forms the cycle matrix (cycle j in column j, Alg. A.2), takes the
// DFT of every cycle to get all coefficients r_{j,k} (Alg. 2.2) and then the
// eigenvalue lists L_k = F r_{.,k} (Alg. 2.3 step 4).  Substituting the cycle
// index j = (row - col) mod n gives the same numbers from the two-sided
// transform  Ahat = F A F^-1  (DFT down the columns, inverse DFT along the
// rows -- the 2-D relation the paper notes in Sec. 2.3.1):
//     L_k[p] = Ahat[p, (p - k) mod n],
// i.e. the k-th component lives on the k-th wrapped diagonal of Ahat.  Both
// transforms then run along contiguous or column-batched directions of the
// row-major input instead of along the wrapped diagonals that the cycle
// gather reads.  The component energy is, by Parseval,
//     ||R_k||_F^2 = n sum_j |r_{j,k}|^2 = sum_p |L_k[p]|^2,
// the quantity Alg. 2.3 ranks by (its T[k] is the square root of this / n).
// Removing the kept diagonals of Ahat and transforming back gives
// Delta A = A - sum_{t} R_{k_t} D^{k_t} (step 6) without the O(K n^2) sum.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "amm_internal.hpp"
#include "fft_core.hpp"

namespace amm {
namespace {

__global__ void widen_real(const float* __restrict__ A, double2* __restrict__ Z, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) Z[i] = double2{(double)A[i], 0.0};
}

__global__ void real_part_f32(const double2* __restrict__ Z, float* __restrict__ out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (float)Z[i].x;
}

// One Stockham pass over `batch` complex vectors of length n.  Element e of
// vector b lives at b*bs + e*es.  batch_fast picks the thread order so that
// neighbouring threads touch neighbouring addresses (columns: batch index
// fastest; rows: element index fastest).
template <int R, int SIGN>
__global__ void fft64_pass(const double2* __restrict__ in, double2* __restrict__ out, int n,
                           int Ns, int64_t es, int64_t bs, int64_t batch,
                           const double2* __restrict__ tw, double scale, int batch_fast) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = n / R;
  if (gid >= nb * batch) return;
  int64_t b, j;
  if (batch_fast) { b = gid % batch; j = gid / batch; }
  else { j = gid % nb; b = gid / nb; }
  const double2* src = in + b * bs;
  double2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = src[(j + (int64_t)r * nb) * es];
  const int k = (int)(j & (Ns - 1));
  if (Ns > 1) {
    const int step = n / (Ns * R);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      double2 w = tw[(unsigned)(r * k * step)];
      if (SIGN > 0) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
  }
  dftR<R, SIGN>(v);
  double2* dst = out + b * bs;
  const int64_t base = (j - k) * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[(base + (int64_t)r * Ns) * es] = cscale(v[r], scale);
}

// E_part[chunk][k] = sum over rows p of the chunk of |Ahat[p, (p - k) mod n]|^2
// One Stockham pass of radix R = 16 R2 (R2 = 2 ... 16) as two levels in a
// workgroup of 16 lanes x 16: with r = r1 + 16 r2 and q = a + R2 b,
//   X[q] = sum_r1 w16^(r1 b) w_R^(r1 a) [sum_r2 v[r1 + 16 r2] w_R2^(r2 a)],
// thread (lane, r1) loads its R2 inputs, applies the stage twiddles, takes the
// R2-point DFT and the w_R^(r1 a) twiddles; one LDS exchange; thread (lane, a)
// takes the 16-point DFT over r1 and stores X[a + R2 b].  Half the global
// round trips of two radix-16 passes.  The 16 lanes run along the contiguous
// index: MODE 0, 16 consecutive vectors (bs = 1, batch % 16 == 0); MODE 1,
// 16 consecutive groups j of one vector (es = 1, (n / R) % 16 == 0, Ns >= 16,
// so the outputs of a given q are contiguous too); MODE 2, the same with
// Ns = 1, whose outputs (j R + q) are staged through LDS and stored as one
// contiguous run of 16 R elements.  With `rin` the input is real float32 at
// the same positions (the first pass over a real operand, which then needs no
// widened copy).
template <int R2, int SIGN, int MODE>
__global__ void __launch_bounds__(256)
fft64_pass2(const double2* __restrict__ in, double2* __restrict__ out, int n, int Ns, int64_t es, int64_t bs,
            int64_t batch, const double2* __restrict__ tw, double scale, const float* __restrict__ rin) {
  constexpr int R = 16 * R2, P = 17;   // LDS pitch over r1 (odd in 16-byte units)
  __shared__ double2 sh[16 * R2 * P];
  const int c = threadIdx.x & 15, r1 = threadIdx.x >> 4;
  const int64_t nb = n / R;
  int64_t b, j, j0 = 0;
  if constexpr (MODE == 0) {
    const int64_t gpb = batch / 16;
    j = blockIdx.x / gpb;
    b = (blockIdx.x % gpb) * 16 + c;
  } else {
    const int64_t per = nb / 16;
    b = blockIdx.x / per;
    j0 = (blockIdx.x % per) * 16;
    j = j0 + c;
  }
  const int k = (int)(j & (Ns - 1));
  double2 v[R2];
  if (rin) {
    const float* rsrc = rin + b * bs;
#pragma unroll
    for (int r2 = 0; r2 < R2; ++r2) v[r2] = double2{(double)rsrc[(j + (int64_t)(r1 + 16 * r2) * nb) * es], 0.0};
  } else {
    const double2* src = in + b * bs;
#pragma unroll
    for (int r2 = 0; r2 < R2; ++r2) v[r2] = src[(j + (int64_t)(r1 + 16 * r2) * nb) * es];
  }
  if (Ns > 1) {
    const int step = n / (Ns * R);
#pragma unroll
    for (int r2 = 0; r2 < R2; ++r2) {
      double2 w = tw[(unsigned)((r1 + 16 * r2) * k * step)];
      if (SIGN > 0) w.y = -w.y;
      v[r2] = cmul(v[r2], w);
    }
  }
  dftR<R2, SIGN>(v);
  const int inner = n / R;
#pragma unroll
  for (int a = 1; a < R2; ++a) {
    double2 w = tw[(unsigned)(r1 * a * inner)];
    if (SIGN > 0) w.y = -w.y;
    v[a] = cmul(v[a], w);
  }
#pragma unroll
  for (int a = 0; a < R2; ++a) sh[(c * R2 + a) * P + r1] = v[a];
  __syncthreads();
  const int a = threadIdx.x >> 4;   // second level: thread (lane, a), a < R2
  double2 z[16];
  if (a < R2) {
#pragma unroll
    for (int t = 0; t < 16; ++t) z[t] = sh[(c * R2 + a) * P + t];
    dftR<16, SIGN>(z);              // z[bq] = X[a + R2 bq]
  }
  double2* dst = out + b * bs;
  if constexpr (MODE == 2) {
    __syncthreads();
    if (a < R2)
#pragma unroll
      for (int bq = 0; bq < 16; ++bq) sh[c * R + a + R2 * bq] = z[bq];
    __syncthreads();
    for (int idx = threadIdx.x; idx < 16 * R; idx += 256) dst[j0 * R + idx] = cscale(sh[idx], scale);
  } else {
    if (a < R2) {
      const int64_t base = (j - k) * R + k;
#pragma unroll
      for (int bq = 0; bq < 16; ++bq) dst[(base + (int64_t)(a + R2 * bq) * Ns) * es] = cscale(z[bq], scale);
    }
  }
}

// *out = max over the list entries of max(|x|, |y|), as the bits of a
// non-negative float (integer order = float order)
__global__ void list_absmax(const float2* __restrict__ L, int64_t count, unsigned* __restrict__ out) {
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fmaxf(fabsf(L[i].x), fabsf(L[i].y)));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// Check (pass, ta, tb) of blockIdx.y: *fail = 1 unless list tb of the pass
// (L, or Ladj for pass 1) is the mirrored conjugate of list ta,
// L_b[p] = conj(L_a[-p]), to tol at every p.
__global__ void mirror_check(const float2* __restrict__ L, const float2* __restrict__ La, int64_t n,
                             const int4* __restrict__ checks, float tol, int* __restrict__ fail) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int4 ck = checks[blockIdx.y];
  const float2* Ls = ck.x == 0 ? L : La;
  const float2 a = Ls[(int64_t)ck.y * n + (p == 0 ? 0 : n - p)], b = Ls[(int64_t)ck.z * n + p];
  if (fabsf(b.x - a.x) > tol || fabsf(b.y + a.y) > tol) atomicOr(fail, 1);
}

__global__ void zero_words(unsigned* p, int count) {
  if ((int)threadIdx.x < count) p[threadIdx.x] = 0u;
}

__global__ void energy_partial(const double2* __restrict__ Ahat, int n, int rows_per_chunk,
                               double* __restrict__ part) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  if (k >= n) return;
  const int p0 = chunk * rows_per_chunk;
  const int p1 = min(n, p0 + rows_per_chunk);
  double s = 0.0;
  for (int p = p0; p < p1; ++p) {
    const int q = p - k;
    const double2 v = Ahat[(int64_t)p * n + (q < 0 ? q + n : q)];
    s += v.x * v.x + v.y * v.y;
  }
  part[(int64_t)chunk * n + k] = s;
}

__global__ void energy_reduce(const double* __restrict__ part, int chunks, int n,
                              double* __restrict__ E) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * n + k];
  E[k] = s;
}

// L_t[p] = Ahat[p, (p - k_t) mod n];  Ladj_t[p] = conj(L_t[(p + k_t) mod n])
__global__ void gather_lists(const double2* __restrict__ Ahat, int n,
                             const int32_t* __restrict__ shifts, float2* __restrict__ L,
                             float2* __restrict__ Ladj) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (p >= n) return;
  const int k = shifts[t];
  const int q = p - k, r = p + k;
  const double2 a = Ahat[(int64_t)p * n + (q < 0 ? q + n : q)];
  L[(int64_t)t * n + p] = float2{(float)a.x, (float)a.y};
  const double2 b = Ahat[(int64_t)(r >= n ? r - n : r) * n + p];
  Ladj[(int64_t)t * n + p] = float2{(float)b.x, (float)-b.y};
}

// X[p] = sum over dropped k of |L_k[p]|^2 = sum_q |Ahat[p, q]|^2 - sum_t |Ahat[p, (p - k_t) mod n]|^2:
// the energy of Fourier mode p left in Delta A.  One workgroup of 256 per row.
__global__ void __launch_bounds__(256) mode_energy_rows(const double2* __restrict__ Ahat, int n,
                                                        const int32_t* __restrict__ shifts, int K,
                                                        double* __restrict__ X) {
  __shared__ double sh[256];
  const int p = blockIdx.x;
  const double2* row = Ahat + (int64_t)p * n;
  double s = 0.0;
  for (int q = threadIdx.x; q < n; q += 256) {
    const double2 v = row[q];
    s += v.x * v.x + v.y * v.y;
  }
  for (int t = threadIdx.x; t < K; t += 256) {
    const int q = p - shifts[t];
    const double2 v = row[q < 0 ? q + n : q];
    s -= v.x * v.x + v.y * v.y;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) X[p] = sh[0];
}

__global__ void lists_to_half(const float2* __restrict__ src, __half2* __restrict__ dst, int64_t count,
                              float scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = __floats2half2_rn(src[i].x * scale, src[i].y * scale);
}

__global__ void zero_diagonals(double2* __restrict__ Ahat, int n, const int32_t* __restrict__ shifts) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (p >= n) return;
  const int q = p - shifts[t];
  Ahat[(int64_t)p * n + (q < 0 ? q + n : q)] = double2{0.0, 0.0};
}

template <int SIGN>
amm_status launch_pass(int log2r, const double2* in, double2* out, int n, int Ns, int64_t es,
                       int64_t bs, int64_t batch, const double2* tw, double scale,
                       bool batch_fast, hipStream_t s) {
  const int R = 1 << log2r;
  const int64_t threads = (int64_t)(n / R) * batch;
  dim3 grid((unsigned)((threads + 255) / 256)), block(256);
  const int bf = batch_fast ? 1 : 0;
  switch (R) {
    case 16: hipLaunchKernelGGL((fft64_pass<16, SIGN>), grid, block, 0, s, in, out, n, Ns, es, bs, batch, tw, scale, bf); break;
    case 8: hipLaunchKernelGGL((fft64_pass<8, SIGN>), grid, block, 0, s, in, out, n, Ns, es, bs, batch, tw, scale, bf); break;
    case 4: hipLaunchKernelGGL((fft64_pass<4, SIGN>), grid, block, 0, s, in, out, n, Ns, es, bs, batch, tw, scale, bf); break;
    case 2: hipLaunchKernelGGL((fft64_pass<2, SIGN>), grid, block, 0, s, in, out, n, Ns, es, bs, batch, tw, scale, bf); break;
    default: return fail(AMM_EUNSUPPORTED, "bad radix");
  }
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

}  // namespace

namespace {

template <int SIGN, int MODE>
amm_status launch_pass2(int log2r, const double2* in, double2* out, int n, int Ns, int64_t es, int64_t bs,
                        int64_t batch, const double2* tw, double scale, const float* rin, hipStream_t s) {
  const int64_t groups = (int64_t)(n >> log2r) * batch;   // one workgroup per 16 groups
  dim3 grid((unsigned)(groups / 16)), block(256);
  switch (log2r) {
    case 8: hipLaunchKernelGGL((fft64_pass2<16, SIGN, MODE>), grid, block, 0, s, in, out, n, Ns, es, bs, batch, tw, scale, rin); break;
    case 7: hipLaunchKernelGGL((fft64_pass2<8, SIGN, MODE>), grid, block, 0, s, in, out, n, Ns, es, bs, batch, tw, scale, rin); break;
    case 6: hipLaunchKernelGGL((fft64_pass2<4, SIGN, MODE>), grid, block, 0, s, in, out, n, Ns, es, bs, batch, tw, scale, rin); break;
    case 5: hipLaunchKernelGGL((fft64_pass2<2, SIGN, MODE>), grid, block, 0, s, in, out, n, Ns, es, bs, batch, tw, scale, rin); break;
    default: return fail(AMM_EUNSUPPORTED, "bad two-level radix");
  }
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

template <int SIGN>
amm_status launch_any2(int log2r, int mode, const double2* in, double2* out, int n, int Ns, int64_t es,
                       int64_t bs, int64_t batch, const double2* tw, double scale, const float* rin,
                       hipStream_t s) {
  if (mode == 0) return launch_pass2<SIGN, 0>(log2r, in, out, n, Ns, es, bs, batch, tw, scale, rin, s);
  if (mode == 1) return launch_pass2<SIGN, 1>(log2r, in, out, n, Ns, es, bs, batch, tw, scale, rin, s);
  return launch_pass2<SIGN, 2>(log2r, in, out, n, Ns, es, bs, batch, tw, scale, rin, s);
}

}  // namespace

// Passes of up to 256 points as two levels in a workgroup (fft64_pass2)
// where the lanes can run along a contiguous index: columns of 16 or more
// vectors at unit batch stride, or rows with at least 16 groups per pass;
// radix-16 passes (and one smaller) otherwise and for the last few bits.
amm_status fft64_transform(double2*& cur, double2*& tmp, int log2n, int64_t es, int64_t bs, int64_t batch,
                           bool batch_fast, int sign, double scale, const double2* tw, hipStream_t s,
                           const float* real_src) {
  const int n = 1 << log2n;
  const bool cols2 = batch_fast && bs == 1 && batch % 16 == 0;
  const bool rows2 = !batch_fast && es == 1;
  std::vector<std::pair<int, bool>> plan;   // (log2 radix, two-level)
  for (int bits = log2n; bits > 0;) {
    const int lr2 = std::min({8, bits, rows2 ? log2n - 4 : 8});
    if ((cols2 || rows2) && lr2 >= 5) {
      plan.push_back({lr2, true});
      bits -= lr2;
    } else {
      const int lr = std::min(4, bits);
      plan.push_back({lr, false});
      bits -= lr;
    }
  }
  // a real input that the first pass cannot read directly is widened into cur first
  if (real_src && !plan[0].second) {
    const int64_t count = (batch - 1) * bs + ((int64_t)n - 1) * es + 1;
    hipLaunchKernelGGL(widen_real, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, real_src, cur, count);
    AMM_HIP(hipGetLastError());
    real_src = nullptr;
  }
  int Ns = 1;
  for (size_t st = 0; st < plan.size(); ++st) {
    const int lr = plan[st].first;
    const double sc = (st + 1 == plan.size()) ? scale : 1.0;
    if (plan[st].second) {
      const int mode = cols2 ? 0 : (Ns == 1 ? 2 : 1);
      if (mode == 1 && Ns < 16) return fail(AMM_EUNSUPPORTED, "internal: two-level row pass needs Ns >= 16");
      const float* rin = st == 0 ? real_src : nullptr;
      if (sign < 0) AMM_TRY(launch_any2<-1>(lr, mode, cur, tmp, n, Ns, es, bs, batch, tw, sc, rin, s));
      else AMM_TRY(launch_any2<+1>(lr, mode, cur, tmp, n, Ns, es, bs, batch, tw, sc, rin, s));
    } else {
      if (sign < 0) AMM_TRY(launch_pass<-1>(lr, cur, tmp, n, Ns, es, bs, batch, tw, sc, batch_fast, s));
      else AMM_TRY(launch_pass<+1>(lr, cur, tmp, n, Ns, es, bs, batch, tw, sc, batch_fast, s));
    }
    std::swap(cur, tmp);
    Ns <<= lr;
  }
  return AMM_OK;
}

namespace {

// Transform all n vectors of the n x n array in `cur` along one axis; result
// ends in `cur` (buffers are swapped as needed).  columns: vectors run down
// the columns.  sign -1 forward; `scale` multiplies the final pass.
amm_status transform_axis(double2*& cur, double2*& tmp, int log2n, bool columns, int sign,
                          double scale, const double2* tw, hipStream_t s) {
  const int n = 1 << log2n;
  return fft64_transform(cur, tmp, log2n, columns ? n : 1, columns ? 1 : n, n, columns, sign, scale, tw, s);
}

}  // namespace

// float16 copies of L and Ladj, scaled by the power of two that puts the
// largest list component in [2^13, 2^14) (the lists of a small residue would
// otherwise sit among the float16 subnormals); l16_inv undoes the scale.
amm_status cd_make_half_lists(amm_dec* dec, const std::vector<float2>& Lh, hipStream_t s) {
  float mx = 0.f;
  for (const float2& v : Lh) mx = std::max(mx, std::max(std::fabs(v.x), std::fabs(v.y)));
  return cd_make_half_lists_mx(dec, mx, s);
}

amm_status cd_make_half_lists_mx(amm_dec* dec, float mx, hipStream_t s) {
  int ex = 0;
  (void)std::frexp(mx, &ex);                         // mx < 2^ex
  const int sh = std::min(std::max(14 - ex, -100), 100);
  const int64_t cnt = (int64_t)dec->K_eff * dec->n;
  AMM_TRY(dec->L16.alloc(cnt * sizeof(__half2)));
  AMM_TRY(dec->Ladj16.alloc(cnt * sizeof(__half2)));
  const float sc = std::ldexp(1.0f, sh);
  hipLaunchKernelGGL(lists_to_half, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, dec->L.as<float2>(),
                     dec->L16.as<__half2>(), cnt, sc);
  hipLaunchKernelGGL(lists_to_half, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, dec->Ladj.as<float2>(),
                     dec->Ladj16.as<__half2>(), cnt, sc);
  AMM_HIP(hipGetLastError());
  dec->l16_inv = std::ldexp(1.0f, -sh);
  dec->fp16 = true;
  return AMM_OK;
}

// Pair tables from the device lists: the largest component (for the
// tolerance 1e-5 max + 1e-30, as with host lists), then every mirror test the
// closed set needs in one launch and one flag.
amm_status cd_build_pairs_dev(amm_dec* dec, float* mx, hipStream_t s) {
  const int64_t n = dec->n;
  const int K = dec->K_eff;
  *mx = 0.f;
  dec->npairs = dec->npairs_adj = -1;
  dec->nsingles = dec->nsingles_adj = 0;
  if (K == 0) return AMM_OK;
  DevBuf words;
  AMM_TRY(words.alloc(2 * sizeof(unsigned)));
  unsigned* w = words.as<unsigned>();
  hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, s, w, 2);
  const int64_t cnt = (int64_t)K * n;
  hipLaunchKernelGGL(list_absmax, dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 2048)), dim3(256), 0, s,
                     dec->L.as<float2>(), cnt, w);
  AMM_HIP(hipGetLastError());
  unsigned bits = 0;
  AMM_HIP(hipMemcpyAsync(&bits, w, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipStreamSynchronize(s));
  std::memcpy(mx, &bits, sizeof(float));
  // the tests the closed set needs (recorded; the tables assume they pass)
  std::vector<int4> checks;
  AMM_TRY(cd_pair_tables(dec, [&](int pass, int ta, int tb) {
    checks.push_back(int4{pass, ta, tb, 0});
    return true;
  }));
  if (dec->npairs < 0 || checks.empty()) return AMM_OK;   // not closed
  DevBuf ck;
  AMM_TRY(ck.alloc(checks.size() * sizeof(int4)));
  AMM_HIP(hipMemcpyAsync(ck.ptr, checks.data(), checks.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  const float tol = 1e-5f * *mx + 1e-30f;
  hipLaunchKernelGGL(mirror_check, dim3((unsigned)((n + 255) / 256), (unsigned)checks.size()), dim3(256), 0, s,
                     dec->L.as<float2>(), dec->Ladj.as<float2>(), n, ck.as<int4>(), tol,
                     reinterpret_cast<int*>(w + 1));
  AMM_HIP(hipGetLastError());
  unsigned failed = 0;
  AMM_HIP(hipMemcpyAsync(&failed, w + 1, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipStreamSynchronize(s));
  if (failed) {
    dec->npairs = dec->npairs_adj = -1;
    dec->nsingles = dec->nsingles_adj = 0;
    dec->pair_buf.release();
  }
  return AMM_OK;
}

amm_status cd_decompose(amm_ctx* ctx, const float* A, int n, int K, bool keep_residual,
                        amm_dec* dec, hipStream_t s, bool fp16) {
  const bool pow2 = (n & (n - 1)) == 0;
  int log2n = 0;
  while ((1 << log2n) < n) ++log2n;
  const int64_t nn = (int64_t)n * n;
  const double2* tw = nullptr;
  if (pow2) AMM_TRY(twiddles64(ctx, log2n, &tw));
  // transform of all n rows or columns; other sizes through the chirp convolution
  auto xform = [&](double2*& cur, double2*& tmp, bool columns, int sign, double scale) -> amm_status {
    if (pow2) return transform_axis(cur, tmp, log2n, columns, sign, scale, tw, s);
    return dft64_any(ctx, cur, n, columns ? n : 1, columns ? 1 : n, n, sign, scale, s);
  };
  DevBuf z0, z1;
  AMM_TRY(z0.alloc(nn * sizeof(double2)));
  AMM_TRY(z1.alloc(nn * sizeof(double2)));
  double2* cur = z0.as<double2>();
  double2* tmp = z1.as<double2>();
  if (pow2) {
    // the first column pass reads A (real float32) directly
    AMM_TRY(fft64_transform(cur, tmp, log2n, n, 1, n, true, -1, 1.0, tw, s, A));
  } else {
    hipLaunchKernelGGL(widen_real, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, A, cur, nn);
    AMM_HIP(hipGetLastError());
    AMM_TRY(xform(cur, tmp, /*columns=*/true, -1, 1.0));
  }
  AMM_TRY(xform(cur, tmp, /*columns=*/false, +1, 1.0 / n));

  // energies ||R_k||_F^2
  const int rows_per_chunk = 64;
  const int chunks = (n + rows_per_chunk - 1) / rows_per_chunk;
  DevBuf part;
  AMM_TRY(part.alloc((size_t)chunks * n * sizeof(double)));
  AMM_TRY(dec->energies.alloc((size_t)n * sizeof(double)));
  hipLaunchKernelGGL(energy_partial, dim3((unsigned)((n + 255) / 256), (unsigned)chunks), dim3(256), 0, s,
                     cur, n, rows_per_chunk, part.as<double>());
  hipLaunchKernelGGL(energy_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     part.as<double>(), chunks, n, dec->energies.as<double>());
  AMM_HIP(hipGetLastError());
  std::vector<double> E(n);
  AMM_HIP(hipMemcpyAsync(E.data(), dec->energies.ptr, n * sizeof(double), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipStreamSynchronize(s));
  dec->has_energies = true;

  // selection (Alg. 2.3 steps 2-3, closed under conjugate pairs)
  dec->freqs = select_closed(E, K);
  dec->K_eff = (int)dec->freqs.size();
  double total = 0.0, kept = 0.0;
  for (int k = 0; k < n; ++k) total += E[k];
  for (int k : dec->freqs) kept += E[k];
  dec->norm_A = std::sqrt(std::max(total, 0.0));
  dec->norm_residual = std::sqrt(std::max(total - kept, 0.0));

  const int Ke = dec->K_eff;
  std::vector<int32_t> adj(Ke);
  for (int t = 0; t < Ke; ++t) adj[t] = (n - dec->freqs[t]) % n;
  const size_t kb = (size_t)std::max(Ke, 1) * sizeof(int32_t);
  AMM_TRY(dec->shifts.alloc(kb));
  AMM_TRY(dec->shifts_adj.alloc(kb));
  AMM_TRY(dec->L.alloc((size_t)std::max(Ke, 1) * n * sizeof(float2)));
  AMM_TRY(dec->Ladj.alloc((size_t)std::max(Ke, 1) * n * sizeof(float2)));
  if (Ke > 0) {
    AMM_HIP(hipMemcpyAsync(dec->shifts.ptr, dec->freqs.data(), Ke * sizeof(int32_t), hipMemcpyHostToDevice, s));
    AMM_HIP(hipMemcpyAsync(dec->shifts_adj.ptr, adj.data(), Ke * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(gather_lists, dim3((unsigned)((n + 255) / 256), (unsigned)Ke), dim3(256), 0, s,
                       cur, n, dec->shifts.as<int32_t>(), dec->L.as<float2>(), dec->Ladj.as<float2>());
    AMM_HIP(hipGetLastError());
    float mx = 0.f;
    AMM_TRY(cd_build_pairs_dev(dec, &mx, s));
    if (fp16 && n >= 1024 && (pow2 || n <= kChirpFusedMax)) AMM_TRY(cd_make_half_lists_mx(dec, mx, s));
  }

  // spectral concentration of Delta A (circulant residual theorem of Sec. 3):
  // mu = max_p X_p / (||Delta A||_F^2 / n)
  {
    DevBuf X;
    AMM_TRY(X.alloc((size_t)n * sizeof(double)));
    hipLaunchKernelGGL(mode_energy_rows, dim3((unsigned)n), dim3(256), 0, s, cur, n, dec->shifts.as<int32_t>(), Ke,
                       X.as<double>());
    AMM_HIP(hipGetLastError());
    std::vector<double> Xh(n);
    AMM_HIP(hipMemcpyAsync(Xh.data(), X.ptr, n * sizeof(double), hipMemcpyDeviceToHost, s));
    AMM_HIP(hipStreamSynchronize(s));
    double xmax = 0.0;
    for (double v : Xh) xmax = std::max(xmax, v);
    const double r2 = dec->norm_residual * dec->norm_residual;
    dec->mu = r2 > 0.0 ? xmax * n / r2 : 1.0;
  }

  if (keep_residual) {
    // Delta A = F^-1 (Ahat with the kept diagonals removed) F
    if (Ke > 0) {
      hipLaunchKernelGGL(zero_diagonals, dim3((unsigned)((n + 255) / 256), (unsigned)Ke), dim3(256), 0, s,
                         cur, n, dec->shifts.as<int32_t>());
      AMM_HIP(hipGetLastError());
    }
    AMM_TRY(xform(cur, tmp, /*columns=*/false, -1, 1.0));
    AMM_TRY(xform(cur, tmp, /*columns=*/true, +1, 1.0 / n));
    AMM_TRY(dec->residual.alloc(nn * sizeof(float)));
    hipLaunchKernelGGL(real_part_f32, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, cur,
                       dec->residual.as<float>(), nn);
    AMM_HIP(hipGetLastError());
  }
  // the temporaries are released on return; make sure no kernel still uses them
  AMM_HIP(hipStreamSynchronize(s));
  return AMM_OK;
}

}  // namespace amm
