// Fourier-domain sparsification (Sec. 2.4 of the paper, Alg. 2.4 and 2.5).
//
// With F[p, q] = exp(-2 pi i p q / n) (unnormalised) and W = F / sqrt(n):
//   AB = (A W*)(W B) = (1/n) (A conj(F)) (F B).
// Decomposition (float64 on the device, the per-row / per-column closed
// selection too):
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

// ---- closed top-K selection on the device ------------------------------------
// One workgroup per vector (a row of H for the left role, a column of G for
// the right role) applies the selection rule to its energies E (length len):
// the kept set is closed under q -> len - q and holds at most K members;
// among the candidates "singles U (a subset of {0, len/2}) plus the np
// highest-energy pairs {k, len - k}" (ties to the smaller k) it keeps the one
// with the most energy, then the larger one.  Pair energies go to LDS; the
// need-th largest (need = min(#pairs, K/2)) is found by an 8-bit radix select
// on their float64 bit patterns (nonnegative, so the patterns order like the
// values); every candidate takes either the top need pairs or the top
// need - 1, so the totals follow from that sum and the threshold value.
// Output per vector (slot of K entries, ascending frequency):
//   left role:  every member;
//   right role: the class representatives q <= len/2 with weight 1 (a
//               single) or 2 (a pair);
// plus the member count, the kept energy and the vector's total energy.
constexpr int kSelThreads = 256;
constexpr int kSelMaxPairs = 8192;   // len <= 16384

__device__ __forceinline__ uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }

__device__ double sel_block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__device__ int sel_block_count(int v, int* redi) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) redi[threadIdx.x >> 6] = v;
  __syncthreads();
  return redi[0] + redi[1] + redi[2] + redi[3];
}

// Exclusive prefix over the block's threads (in thread order) of v.
__device__ int sel_block_exclusive(int v, int* redi) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  __syncthreads();
  if (lane == 63) redi[wave] = incl;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wave; ++w) base += redi[w];
  return base + incl - v;
}

__global__ void __launch_bounds__(kSelThreads) closed_topk_kernel(const double* __restrict__ E, int64_t count, int len,
                                                                  int64_t vec_step, int64_t elem_stride, int K,
                                                                  int slot, int right_role,
                                                                  int32_t* __restrict__ slot_idx,
                                                                  int32_t* __restrict__ slot_wt,
                                                                  int32_t* __restrict__ slot_cnt,
                                                                  double* __restrict__ kept_out,
                                                                  double* __restrict__ total_out) {
  __shared__ double pe[kSelMaxPairs];
  __shared__ unsigned char flag[2 * kSelMaxPairs];
  __shared__ int hist[256];
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ int sel_digit, sel_remaining;
  const int64_t v = blockIdx.x;
  if (v >= count) return;
  const double* e = E + v * vec_step;
  const int tid = threadIdx.x;
  const int npairs = (len + 1) / 2 - 1;          // classes {k, len - k}, 1 <= k < (len + 1) / 2
  const bool even = (len % 2 == 0) && len > 1;
  const double e0 = e[0], eh = even ? e[(int64_t)(len / 2) * elem_stride] : 0.0;
  double part = 0.0;
  for (int k = 1 + tid; k <= npairs; k += kSelThreads) {
    const double x = e[(int64_t)k * elem_stride] + e[(int64_t)(len - k) * elem_stride];
    pe[k - 1] = x;
    part += x;
  }
  for (int q = tid; q < len; q += kSelThreads) flag[q] = 0;
  const double total = sel_block_sum(part, red) + e0 + eh;   // (its barriers also publish pe and flag)
  const int Kc = min(K, len);
  const int need = min(npairs, Kc / 2);
  // the need-th largest pair energy T and how many of the pairs equal to T are taken
  uint64_t prefix = 0, mask = 0;
  int take_eq = 0;
  double top = 0.0, T = 0.0;
  if (need > 0) {
    int remaining = need;
    for (int shift = 56; shift >= 0; shift -= 8) {
      hist[tid] = 0;   // 256 threads, 256 bins
      __syncthreads();
      for (int k = tid; k < npairs; k += kSelThreads) {
        const uint64_t b = dbits(pe[k]);
        if ((b & mask) == prefix) atomicAdd(&hist[(b >> shift) & 255], 1);
      }
      __syncthreads();
      if (tid < 64) {
        // lane L holds bins 255 - 4L .. 252 - 4L (descending digits); inclusive scan over lanes
        int c4[4], s4 = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c4[u] = hist[255 - 4 * tid - u];
          s4 += c4[u];
        }
        int incl = s4;
        for (int off = 1; off < 64; off <<= 1) {
          const int t = __shfl_up(incl, off, 64);
          if (tid >= off) incl += t;
        }
        const int excl = incl - s4;
        // the lane whose range crosses `remaining` picks the digit
        if (excl < remaining && incl >= remaining) {
          int cum = excl;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (cum + c4[u] >= remaining && cum < remaining) {
              sel_digit = 255 - 4 * tid - u;
              sel_remaining = remaining - cum;
            }
            cum += c4[u];
          }
        }
      }
      __syncthreads();
      prefix |= (uint64_t)sel_digit << shift;
      mask |= (uint64_t)255 << shift;
      remaining = sel_remaining;
      __syncthreads();   // every thread has read the pick before the next pass rewrites it
    }
    take_eq = remaining;   // pairs equal to T among the top need (>= 1)
    T = __longlong_as_double((long long)prefix);
    double gt = 0.0;
    for (int k = tid; k < npairs; k += kSelThreads)
      if (dbits(pe[k]) > prefix) gt += pe[k];
    top = sel_block_sum(gt, red) + (double)take_eq * T;   // energy of the top need pairs
  }
  // best candidate: singles U, then np = need or need - 1 pairs
  double best = 0.0;
  int best_size = -1, best_u = 0, best_np = 0;
  for (int u = 0; u < 4; ++u) {
    const bool has0 = (u & 1) != 0, hash = (u & 2) != 0;
    if (hash && !even) continue;
    const int us = (has0 ? 1 : 0) + (hash ? 1 : 0);
    if (us > Kc) continue;
    const int np = min(need, (Kc - us) / 2);
    double tot = (has0 ? e0 : 0.0) + (hash ? eh : 0.0);
    tot += (np == need) ? top : top - T;   // np is need or need - 1
    const int size = us + 2 * np;
    if (best_size < 0 || tot > best || (tot == best && size > best_size)) {
      best = tot;
      best_size = size;
      best_u = u;
      best_np = np;
    }
  }
  // members: pairs above T, then the first (take_eq or take_eq - 1) pairs equal to T by index
  const int take = (best_np == need) ? take_eq : take_eq - 1;
  {
    // contiguous chunk of pair indices per thread, so the ties are counted in index order
    const int chunk = (npairs + kSelThreads - 1) / kSelThreads;
    const int k0 = tid * chunk, k1 = min(npairs, k0 + chunk);
    int eq = 0;
    if (best_np > 0)
      for (int k = k0; k < k1; ++k) eq += (dbits(pe[k]) == prefix) ? 1 : 0;
    int before = sel_block_exclusive(eq, redi);
    if (best_np > 0)
      for (int k = k0; k < k1; ++k) {
        const uint64_t b = dbits(pe[k]);
        bool in = b > prefix;
        if (b == prefix) in = before++ < take;
        if (in) {
          const int q = k + 1;
          flag[q] = 2;                          // a pair's representative
          if (!right_role) flag[len - q] = 2;
        }
      }
  }
  if (tid == 0) {
    if (best_u & 1) flag[0] = 1;
    if (best_u & 2) flag[len / 2] = 1;
  }
  __syncthreads();
  // compaction in ascending frequency order
  {
    const int chunk = (len + kSelThreads - 1) / kSelThreads;
    const int q0 = tid * chunk, q1 = min(len, q0 + chunk);
    int c = 0;
    for (int q = q0; q < q1; ++q) c += flag[q] ? 1 : 0;
    int pos = sel_block_exclusive(c, redi);
    for (int q = q0; q < q1; ++q)
      if (flag[q]) {
        slot_idx[v * slot + pos] = q;
        if (right_role) slot_wt[v * slot + pos] = flag[q];
        ++pos;
      }
    const int cnt = sel_block_count(c, redi);
    if (tid == 0) {
      slot_cnt[v] = cnt;
      kept_out[v] = best;
      total_out[v] = total;
    }
  }
}

// Slots of K entries per vector -> CSR (ptr from the counts' prefix sums).
__global__ void slots_to_csr(const int32_t* __restrict__ slot_idx, const int32_t* __restrict__ slot_wt,
                             const int32_t* __restrict__ ptr, int64_t count, int K, int32_t* __restrict__ idx,
                             int32_t* __restrict__ wt) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (v >= count) return;
  const int b = ptr[v], c = ptr[v + 1] - b;
  for (int t = threadIdx.x; t < c; t += blockDim.x) {
    idx[b + t] = slot_idx[v * K + t];
    if (wt) wt[b + t] = slot_wt[v * K + t];
  }
}

// Closed selection of `count` vectors of E; builds ptr/idx (and wt for the
// right role) in d's buffers, returns the summed kept and total energies.
amm_status select_closed_device(const double* E, int64_t count, int len, int64_t vec_step, int64_t elem_stride, int K,
                                bool right_role, DevBuf& ptr_buf, DevBuf& idx_buf, DevBuf* wt_buf, int64_t* nnz_out,
                                double* kept_sum, double* total_sum, hipStream_t s) {
  const int slot = std::max(1, std::min(K, len));   // entries per vector at most
  DevBuf slots, swt, cnt, kept, tot;
  AMM_TRY(slots.alloc((size_t)count * slot * sizeof(int32_t)));
  AMM_TRY(swt.alloc(right_role ? (size_t)count * slot * sizeof(int32_t) : 4));
  AMM_TRY(cnt.alloc((size_t)count * sizeof(int32_t)));
  AMM_TRY(kept.alloc((size_t)count * sizeof(double)));
  AMM_TRY(tot.alloc((size_t)count * sizeof(double)));
  {
    TimedLaunch tl("sfft_select", s);
    hipLaunchKernelGGL(closed_topk_kernel, dim3((unsigned)count), dim3(kSelThreads), 0, s, E, count, len, vec_step,
                       elem_stride, K, slot, right_role ? 1 : 0, slots.as<int32_t>(), swt.as<int32_t>(), cnt.as<int32_t>(),
                       kept.as<double>(), tot.as<double>());
    AMM_HIP(hipGetLastError());
  }
  std::vector<int32_t> hc(count);
  std::vector<double> hk(count), ht(count);
  AMM_HIP(hipMemcpyAsync(hc.data(), cnt.ptr, count * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipMemcpyAsync(hk.data(), kept.ptr, count * sizeof(double), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipMemcpyAsync(ht.data(), tot.ptr, count * sizeof(double), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> ptr(count + 1, 0);
  double ks = 0.0, ts = 0.0;
  for (int64_t v = 0; v < count; ++v) {
    ptr[v + 1] = ptr[v] + hc[v];
    ks += hk[v];
    ts += ht[v];
  }
  const int64_t nnz = ptr[count];
  AMM_TRY(ptr_buf.alloc((count + 1) * sizeof(int32_t)));
  AMM_TRY(idx_buf.alloc(std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
  if (wt_buf) AMM_TRY(wt_buf->alloc(std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
  AMM_HIP(hipMemcpyAsync(ptr_buf.ptr, ptr.data(), (count + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(slots_to_csr, dim3((unsigned)((count + 3) / 4)), dim3(64, 4), 0, s, slots.as<int32_t>(),
                     swt.as<int32_t>(), ptr_buf.as<int32_t>(), count, slot, idx_buf.as<int32_t>(),
                     wt_buf ? wt_buf->as<int32_t>() : (int32_t*)nullptr);
  AMM_HIP(hipGetLastError());
  AMM_HIP(hipStreamSynchronize(s));   // the slot buffers are released on return
  *nnz_out = nnz;
  *kept_sum = ks;
  *total_sum = ts;
  return AMM_OK;
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
    int64_t nnz = 0;
    double kept = 0.0;
    AMM_TRY(select_closed_device(E.as<double>(), m, (int)n, n, 1, K, false, d->sf_rptr, d->sf_ridx, nullptr, &nnz,
                                 &kept, &tot, s));
    AMM_TRY(d->sf_rval.alloc(std::max<int64_t>(nnz, 1) * sizeof(float2)));
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
    int64_t nr = 0;
    double kept = 0.0, total = 0.0;
    DevBuf wdev;
    AMM_TRY(select_closed_device(E.as<double>(), n, (int)m, 1, n, K, true, d->sf_cptr, d->sf_cidx, &wdev, &nr, &kept,
                                 &total, s));
    AMM_TRY(d->sf_cval.alloc(std::max<int64_t>(nr, 1) * sizeof(float2)));
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
