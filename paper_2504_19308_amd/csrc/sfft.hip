// Fourier-domain sparsification (Sec. 2.4 of the paper, Alg. 2.4 and 2.5).
//
// With F[p, q] = exp(-2 pi i p q / n) (unnormalised) and W = F / sqrt(n):
//   AB = (A W*)(W B) = (1/n) (A conj(F)) (F B).
// Decomposition (float64 on the device, selection on the host as for the
// circulant kind):
//   left role  (A, m x n, n = 2^a):  H = A conj(F) by rows; each row keeps the
//     closed set of at most K frequencies {q, n-q} with the most energy;
//     stored as CSR with values H / n (float32 complex), and the residual's
//     half spectrum R[q][i] = H[i, q] / n for dropped q <= n/2 (transposed,
//     (n/2 + 1) x m float32 complex).
//   right role (B, n x p, n = 2^b): G = F B by columns; each column keeps its
//     closed set; stored per column as the representatives q <= n/2 with the
//     values w_q G[q, j] (w = 2 for a pair, 1 for q = 0 and q = n/2).
// Products:
//   zeroth  M0 = (1/n) Re(Atil conj(F)... ) computed as a complex SpMM of the
//           CSR against the packed spectrum X_c = F(b_2c + i b_2c+1): for a
//           closed row selection the sum splits into a real part (column 2c)
//           and an imaginary part (column 2c + 1).
//   first   M0 + Re((A W* - Atil) Btil): for closed selections on both sides
//           the conjugate pairs fold onto the half spectrum, so column j of
//           the term is sum over representatives q of Re(R[q][.] w_q G[q, j]);
//           computed transposed (a second SpMM with real output) and added
//           back transposed.
#include <type_traits>

#include "amm_internal.hpp"

namespace amm {
namespace {

__global__ void real_to_c64(const float* __restrict__ A, double2* __restrict__ Z, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) Z[i] = double2{(double)A[i], 0.0};
}

__global__ void abs2_c64(const double2* __restrict__ Z, double* __restrict__ E, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) E[i] = Z[i].x * Z[i].x + Z[i].y * Z[i].y;
}

// val[e] = H[row(e) * rs + idx[e] * cs] * scale (float32 complex)
__global__ void gather_entries(const double2* __restrict__ H, const int32_t* __restrict__ ptr,
                               const int32_t* __restrict__ idx, const int32_t* __restrict__ wt, int64_t rows,
                               int64_t rs, int64_t cs, double scale, float2* __restrict__ val) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (r >= rows) return;
  for (int e = ptr[r] + threadIdx.x; e < ptr[r + 1]; e += blockDim.x) {
    const double2 h = H[r * rs + (int64_t)idx[e] * cs];
    const double w = wt ? (double)wt[e] * scale : scale;
    val[e] = float2{(float)(h.x * w), (float)(h.y * w)};
  }
}

// R[q][i] = H[i, q] * scale for q in [0, half), i in [0, m): transposed through LDS tiles
__global__ void half_spectrum_t(const double2* __restrict__ H, int64_t m, int64_t n, int64_t half, double scale,
                                float2* __restrict__ R) {
  __shared__ float2 tile[32][33];
  const int64_t q0 = (int64_t)blockIdx.x * 32, i0 = (int64_t)blockIdx.y * 32;
  for (int t = threadIdx.y; t < 32; t += 8) {
    const int64_t i = i0 + t, q = q0 + threadIdx.x;
    if (i < m && q < half) {
      const double2 h = H[i * n + q];
      tile[t][threadIdx.x] = float2{(float)(h.x * scale), (float)(h.y * scale)};
    }
  }
  __syncthreads();
  for (int t = threadIdx.y; t < 32; t += 8) {
    const int64_t q = q0 + t, i = i0 + threadIdx.x;
    if (i < m && q < half) R[q * m + i] = tile[threadIdx.x][t];
  }
}

// R[q][i] = 0 for the kept entries (i, q) with q < half
__global__ void zero_kept(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx, int64_t m, int64_t half,
                          float2* __restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  for (int e = ptr[i]; e < ptr[i + 1]; ++e)
    if (idx[e] < half) R[(int64_t)idx[e] * m + i] = float2{0.f, 0.f};
}

// Complex SpMM over slices of a dense complex operand D (rows indexed by the
// CSR column ids, W complex columns, row stride ld floats).  For output row r:
//   PACKED: out[r][2c], out[r][2c+1] = re, im of sum_e val[e] * D[idx[e]][c]
//   REAL:   out[r][c] = re of the same sum
// One wave per output row and slice of 64 * V complex columns (V = 2: a lane
// owns two neighbouring complex columns, one 16-byte load per entry); entries
// are taken four at a time with their loads issued together.  Blocks of one
// XCD sweep whole slices so a slice of D stays in that XCD's L2.
template <bool PACKED, int V>
__global__ void __launch_bounds__(256) cspmm_slices(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                                    const float2* __restrict__ val, const float* __restrict__ D,
                                                    int64_t ld, int64_t W, int64_t rows, float* __restrict__ out,
                                                    int64_t ldo, int accumulate, int nslices, int rgroups) {
  constexpr int RPB = 16;   // output rows per block (4 waves x 4)
  const int nblk = nslices * rgroups;
  int b = blockIdx.x;
  if (nblk % 8 == 0) b = (b % 8) * (nblk / 8) + b / 8;
  const int slice = b / rgroups, rg = b % rgroups;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c = ((int64_t)slice * 64 + lane) * V;   // first complex column of this lane
  if (c >= W) return;
  typedef typename std::conditional<V == 2, float4, float2>::type vec_t;
  for (int k = 0; k < RPB / 4; ++k) {
    const int64_t r = (int64_t)rg * RPB + wave * (RPB / 4) + k;
    if (r >= rows) break;
    float ar[V], ai[V];
#pragma unroll
    for (int v = 0; v < V; ++v) ar[v] = ai[v] = 0.f;
    const int e0 = ptr[r], e1 = ptr[r + 1];
    auto mac = [&](float2 a, const vec_t& d) {
      if constexpr (V == 2) {
        ar[0] += a.x * d.x - a.y * d.y;
        ai[0] += a.x * d.y + a.y * d.x;
        ar[1] += a.x * d.z - a.y * d.w;
        ai[1] += a.x * d.w + a.y * d.z;
      } else {
        ar[0] += a.x * d.x - a.y * d.y;
        ai[0] += a.x * d.y + a.y * d.x;
      }
    };
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
      vec_t d[4];
      float2 a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = val[e + u];
        d[u] = *reinterpret_cast<const vec_t*>(D + (int64_t)idx[e + u] * ld + 2 * c);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) mac(a[u], d[u]);
    }
    for (; e < e1; ++e) mac(val[e], *reinterpret_cast<const vec_t*>(D + (int64_t)idx[e] * ld + 2 * c));
    if (PACKED) {
      vec_t* o = reinterpret_cast<vec_t*>(out + r * ldo + 2 * c);
      vec_t v;
      if constexpr (V == 2) v = float4{ar[0], ai[0], ar[1], ai[1]};
      else v = float2{ar[0], ai[0]};
      if (accumulate) {
        const vec_t w = *o;
        if constexpr (V == 2) v = float4{v.x + w.x, v.y + w.y, v.z + w.z, v.w + w.w};
        else v = float2{v.x + w.x, v.y + w.y};
      }
      *o = v;
    } else {
      if constexpr (V == 2) {
        float2* o = reinterpret_cast<float2*>(out + r * ldo + c);
        float2 v{ar[0], ar[1]};
        if (accumulate) {
          const float2 w = *o;
          v = float2{v.x + w.x, v.y + w.y};
        }
        *o = v;
      } else {
        float* o = out + r * ldo + c;
        *o = accumulate ? *o + ar[0] : ar[0];
      }
    }
  }
}

amm_status launch_cspmm(bool packed, const int32_t* ptr, const int32_t* idx, const float2* val, const float* D,
                        int64_t ld, int64_t W, int64_t rows, float* out, int64_t ldo, bool acc, hipStream_t s) {
  if (rows <= 0 || W <= 0) return AMM_OK;
  // two complex columns per lane when every access stays 16-byte (packed) or 8-byte (real) aligned
  const bool v2 = (W % 2 == 0) && (ld % 4 == 0) && (packed ? (ldo % 4 == 0) : (ldo % 2 == 0)) &&
                  ((uintptr_t)D % 16 == 0) && ((uintptr_t)out % (packed ? 16 : 8) == 0);
  const int64_t per = v2 ? 128 : 64;
  const int64_t nslices = (W + per - 1) / per, rgroups = (rows + 15) / 16;
  if (nslices * rgroups > 0x7fffffff) return fail(AMM_EUNSUPPORTED, "SpMM grid too large");
  const dim3 grid((unsigned)(nslices * rgroups)), block(256);
  const int a = acc ? 1 : 0;
#define AMM_CS(P, V) \
  hipLaunchKernelGGL((cspmm_slices<P, V>), grid, block, 0, s, ptr, idx, val, D, ld, W, rows, out, ldo, a, (int)nslices, \
                     (int)rgroups)
  if (packed) {
    if (v2) AMM_CS(true, 2);
    else AMM_CS(true, 1);
  } else {
    if (v2) AMM_CS(false, 2);
    else AMM_CS(false, 1);
  }
#undef AMM_CS
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

// Closed top-K of one energy vector (the select_closed rule, with a partial
// sort of the pair classes: only the leading K/2 are needed)
void closed_topk(const double* E, int n, int K, std::vector<int32_t>& out) {
  out.clear();
  K = std::min(K, n);
  std::vector<int> singles{0};
  if (n % 2 == 0 && n > 1) singles.push_back(n / 2);
  std::vector<int> pairs;
  pairs.reserve(n / 2);
  for (int k = 1; k < (n + 1) / 2; ++k) pairs.push_back(k);
  const size_t need = std::min<size_t>(pairs.size(), (size_t)(K / 2));
  auto cmp = [&](int a, int b) {
    const double ea = E[a] + E[n - a], eb = E[b] + E[n - b];
    if (ea != eb) return ea > eb;
    return a < b;
  };
  std::partial_sort(pairs.begin(), pairs.begin() + need, pairs.end(), cmp);
  std::vector<std::vector<int>> subsets{{}};
  for (int sgl : singles) subsets.push_back({sgl});
  if (singles.size() == 2) subsets.push_back(singles);
  bool have = false;
  double best_total = 0.0;
  size_t best_size = 0;
  for (const auto& U : subsets) {
    if ((int)U.size() > K) continue;
    std::vector<int32_t> members(U.begin(), U.end());
    const size_t np = std::min(need, (size_t)(K - (int)U.size()) / 2);
    for (size_t i = 0; i < np; ++i) {
      members.push_back(pairs[i]);
      members.push_back(n - pairs[i]);
    }
    double total = 0.0;
    for (int m : members) total += E[m];
    if (!have || total > best_total || (total == best_total && members.size() > best_size)) {
      have = true;
      best_total = total;
      best_size = members.size();
      out = members;
    }
  }
  std::sort(out.begin(), out.end());
}

int ilog2_exact(int64_t v) {
  if (v < 1 || (v & (v - 1))) return -1;
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

}  // namespace

bool sfft_left_ok(int64_t n) { return n >= 2 && n <= 16384; }

amm_status sfft_decompose(amm_ctx* ctx, const float* A, int64_t m, int64_t n, int K, bool keep_residual, amm_dec* d,
                          hipStream_t s) {
  const int ln = ilog2_exact(n), lm = ilog2_exact(m);
  const bool left = n >= 2 && n <= 16384, right = m >= 2 && m <= 16384;
  if (!left && !right) return fail(AMM_EUNSUPPORTED, "Fourier sparsification needs m or n in [2, 16384]");
  if (K < 0) return fail(AMM_EINVAL, "K = %d", K);
  const int64_t mn = m * n;
  DevBuf z0, z1, E;
  AMM_TRY(z0.alloc(mn * sizeof(double2)));
  AMM_TRY(z1.alloc(mn * sizeof(double2)));
  AMM_TRY(E.alloc(mn * sizeof(double)));
  std::vector<double> Eh(mn);
  const unsigned g = (unsigned)((mn + 255) / 256);
  double tot = 0.0;
  if (left) {
    // H = A conj(F) along rows
    double2 *cur = z0.as<double2>(), *tmp = z1.as<double2>();
    hipLaunchKernelGGL(real_to_c64, dim3(g), dim3(256), 0, s, A, cur, mn);
    AMM_HIP(hipGetLastError());
    if (ln > 0) {
      const double2* tw = nullptr;
      AMM_TRY(twiddles64(ctx, ln, &tw));
      AMM_TRY(fft64_transform(cur, tmp, ln, 1, n, m, false, +1, 1.0, tw, s));
    } else {
      AMM_TRY(dft64_any(ctx, cur, (int)n, 1, n, m, +1, 1.0, s));
    }
    hipLaunchKernelGGL(abs2_c64, dim3(g), dim3(256), 0, s, cur, E.as<double>(), mn);
    AMM_HIP(hipGetLastError());
    AMM_HIP(hipMemcpyAsync(Eh.data(), E.ptr, mn * sizeof(double), hipMemcpyDeviceToHost, s));
    AMM_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> ptr(m + 1, 0), idx, sel;
    idx.reserve((size_t)m * std::min<int64_t>(K, n));
    double kept = 0.0;
    for (int64_t i = 0; i < m; ++i) {
      const double* Ei = Eh.data() + i * n;
      closed_topk(Ei, (int)n, K, sel);
      for (int q : sel) {
        idx.push_back(q);
        kept += Ei[q];
      }
      ptr[i + 1] = (int32_t)idx.size();
    }
    for (double v : Eh) tot += v;
    const int64_t nnz = (int64_t)idx.size();
    AMM_TRY(d->sf_rptr.alloc((m + 1) * sizeof(int32_t)));
    AMM_TRY(d->sf_ridx.alloc(std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
    AMM_TRY(d->sf_rval.alloc(std::max<int64_t>(nnz, 1) * sizeof(float2)));
    AMM_HIP(hipMemcpyAsync(d->sf_rptr.ptr, ptr.data(), (m + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (nnz) AMM_HIP(hipMemcpyAsync(d->sf_ridx.ptr, idx.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(gather_entries, dim3((unsigned)((m + 3) / 4)), dim3(64, 4), 0, s, cur, d->sf_rptr.as<int32_t>(),
                       d->sf_ridx.as<int32_t>(), (const int32_t*)nullptr, m, n, (int64_t)1, 1.0 / (double)n,
                       d->sf_rval.as<float2>());
    AMM_HIP(hipGetLastError());
    if (keep_residual) {
      const int64_t half = n / 2 + 1;
      AMM_TRY(d->sf_Rt.alloc(half * m * sizeof(float2)));
      hipLaunchKernelGGL(half_spectrum_t, dim3((unsigned)((half + 31) / 32), (unsigned)((m + 31) / 32)), dim3(32, 8), 0,
                         s, cur, m, n, half, 1.0 / (double)n, d->sf_Rt.as<float2>());
      hipLaunchKernelGGL(zero_kept, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, d->sf_rptr.as<int32_t>(),
                         d->sf_ridx.as<int32_t>(), m, half, d->sf_Rt.as<float2>());
      AMM_HIP(hipGetLastError());
    }
    AMM_HIP(hipStreamSynchronize(s));
    d->sf_left = true;
    d->nnz = nnz;
    // ||A||_F^2 = sum |H|^2 / n (Parseval), ||Delta A||_F^2 = (sum - kept) / n
    d->norm_A = std::sqrt(std::max(tot, 0.0) / (double)n);
    d->norm_residual = std::sqrt(std::max(tot - kept, 0.0) / (double)n);
  }
  if (right) {
    // G = F A along columns (A as the right operand: inner dimension m)
    double2 *cur = z0.as<double2>(), *tmp = z1.as<double2>();
    hipLaunchKernelGGL(real_to_c64, dim3(g), dim3(256), 0, s, A, cur, mn);
    AMM_HIP(hipGetLastError());
    if (lm > 0) {
      const double2* tw = nullptr;
      AMM_TRY(twiddles64(ctx, lm, &tw));
      AMM_TRY(fft64_transform(cur, tmp, lm, n, 1, n, true, -1, 1.0, tw, s));
    } else {
      AMM_TRY(dft64_any(ctx, cur, (int)m, n, 1, n, -1, 1.0, s));
    }
    hipLaunchKernelGGL(abs2_c64, dim3(g), dim3(256), 0, s, cur, E.as<double>(), mn);
    AMM_HIP(hipGetLastError());
    AMM_HIP(hipMemcpyAsync(Eh.data(), E.ptr, mn * sizeof(double), hipMemcpyDeviceToHost, s));
    AMM_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> ptr(n + 1, 0), idx, wt, sel;
    std::vector<double> col(m);
    double kept = 0.0, total = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      for (int64_t q = 0; q < m; ++q) col[q] = Eh[q * n + j];
      closed_topk(col.data(), (int)m, K, sel);
      for (int q : sel) {
        kept += col[q];
        if (q <= m / 2) {   // representative of its class
          idx.push_back(q);
          wt.push_back((q == 0 || 2 * q == m) ? 1 : 2);
        }
      }
      for (int64_t q = 0; q < m; ++q) total += col[q];
      ptr[j + 1] = (int32_t)idx.size();
    }
    const int64_t nr = (int64_t)idx.size();
    AMM_TRY(d->sf_cptr.alloc((n + 1) * sizeof(int32_t)));
    AMM_TRY(d->sf_cidx.alloc(std::max<int64_t>(nr, 1) * sizeof(int32_t)));
    AMM_TRY(d->sf_cval.alloc(std::max<int64_t>(nr, 1) * sizeof(float2)));
    DevBuf wdev;
    AMM_TRY(wdev.alloc(std::max<int64_t>(nr, 1) * sizeof(int32_t)));
    AMM_HIP(hipMemcpyAsync(d->sf_cptr.ptr, ptr.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (nr) {
      AMM_HIP(hipMemcpyAsync(d->sf_cidx.ptr, idx.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice, s));
      AMM_HIP(hipMemcpyAsync(wdev.ptr, wt.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    // entry (column j, q): G[q * n + j]  -> row stride 1 (over j), index stride n
    hipLaunchKernelGGL(gather_entries, dim3((unsigned)((n + 3) / 4)), dim3(64, 4), 0, s, cur, d->sf_cptr.as<int32_t>(),
                       d->sf_cidx.as<int32_t>(), wdev.as<int32_t>(), n, (int64_t)1, n, 1.0, d->sf_cval.as<float2>());
    AMM_HIP(hipGetLastError());
    AMM_HIP(hipStreamSynchronize(s));
    d->sf_right = true;
    if (!left) {
      d->norm_A = std::sqrt(std::max(total, 0.0) / (double)m);
      d->norm_residual = std::sqrt(std::max(total - kept, 0.0) / (double)m);
    }
  }
  return AMM_OK;
}

// out (m x p) (+)= Atil W* W B for the left role; B n x p, p even, through the
// packed spectrum of B's column pairs
amm_status sfft_left_apply(amm_ctx* ctx, const amm_dec* d, const float* B, int64_t p, float* out, bool acc,
                           hipStream_t s) {
  const int64_t m = d->m, n = d->n;
  if (!d->sf_left) return fail(AMM_EUNSUPPORTED, "handle has no row sparsification (n out of range)");
  if (p % 2) return fail(AMM_EUNSUPPORTED, "Fourier-sparsified products need an even column count");
  AMM_TRY(ctx->scratch[6].reserve((size_t)n * p * sizeof(float)));
  float* X = ctx->scratch[6].as<float>();
  const int ln = ilog2_exact(n);
  if (ln > 0) AMM_TRY(cd_spectrum_columns(ctx, ln, B, p, X, s));
  else AMM_TRY(spectrum_columns_general(ctx, (int)n, B, p, X, s));
  TimedLaunch tl("sfft_spmm", s);
  return launch_cspmm(true, d->sf_rptr.as<int32_t>(), d->sf_ridx.as<int32_t>(), d->sf_rval.as<float2>(), X, p, p / 2,
                      m, out, p, acc, s);
}

// out (m x p) += Re((A W* - Atil) Btil) for dA, dB both sparsified (dA left, dB right)
amm_status sfft_first_order_term(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, float* out, hipStream_t s) {
  const int64_t m = dA->m, n = dA->n, p = dB->n;
  if (!dA->sf_Rt.ptr) return fail(AMM_ESTATE, "left operand keeps no spectral residual (decompose with keep_residual)");
  if (!dB->sf_right) return fail(AMM_EUNSUPPORTED, "right operand has no column sparsification (m out of range)");
  if (dB->m != n) return fail(AMM_ESHAPE, "inner dimensions differ");
  AMM_TRY(ctx->scratch[7].reserve((size_t)p * m * sizeof(float)));
  float* Y = ctx->scratch[7].as<float>();   // p x m: row j = column j of the term
  {
    TimedLaunch tl("sfft_dense_sparse", s);
    AMM_TRY(launch_cspmm(false, dB->sf_cptr.as<int32_t>(), dB->sf_cidx.as<int32_t>(), dB->sf_cval.as<float2>(),
                         dA->sf_Rt.as<float>(), 2 * m, m, p, Y, m, false, s));
  }
  return transpose_acc_f32(Y, p, m, out, true, s);
}

}  // namespace amm
