// The l x l steps of the randomized SVD (Alg. 2.1 with oversampling and
// subspace iteration) on the device, one workgroup each, so the
// decomposition makes no host round trip between its GEMMs:
//
//   chol_inv_kernel   Gram matrix G = Y^T Y of a sketch -> R^-1 with
//                     G (+ shift) = R^T R (CholeskyQR's factor, inverted);
//   gram_eig_kernel   G = B B^T of the projected operand -> eigenvectors W
//                     and eigenvalues (parallel cyclic Jacobi), sorted into
//                     the singular values and column order that the factor
//                     assembly uses.
//
// Both hold their l x l matrices in LDS (l <= kSmallEigMax: two 96 x 97
// float64 arrays at an odd row pitch, 146 KiB of the 160 KiB a workgroup may
// use).  A larger sketch keeps the host path.
#include <algorithm>
#include <cmath>
#include <vector>

#include "amm_internal.hpp"

namespace amm {
namespace {

constexpr int NT = 256;
constexpr int LM = kSmallEigMax;
constexpr int LS = LM * (LM + 1);   // an l x l array at the odd row pitch ld = l | 1

// Row pitch of an l x l LDS array: odd, so that a column walk (lanes on
// consecutive rows) spreads its 8-byte reads over the banks.
__device__ __forceinline__ int pitch_of(int l) { return l | 1; }

__device__ __forceinline__ double block_sum(double v, double* red) {
  // 256 threads: four waves, shuffles inside a wave, LDS across waves
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// S[i][c] = (G[i][c] + G[c][i]) / 2, plus `shift` on the diagonal, for
// i, c < n (G at pitch ldg) into LDS at pitch ld.  Thread (g, c) takes rows
// g, g + ng, ...: eight rows' loads (clamped addresses, so unconditional) are
// in flight before their stores, where a plain loop would wait for each.
__device__ void load_sym_lds(const double* __restrict__ G, int64_t ldg, int n, double shift, double* S, int ld) {
  const int ng = NT / n, g = (int)threadIdx.x / n, c = (int)threadIdx.x % n;
  if (g >= ng) return;
  for (int i0 = g; i0 < n; i0 += 8 * ng) {
    double u[8], v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = min(i0 + t * ng, n - 1);
      u[t] = G[i * ldg + c];
      v[t] = G[c * ldg + i];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = i0 + t * ng;
      if (i < n) S[i * ld + c] = 0.5 * (u[t] + v[t]) + (i == c ? shift : 0.0);
    }
  }
}

// Upper Cholesky factor R of S (l x l at pitch ld, symmetric, only the upper
// triangle is read; S = R^T R) by row elimination, applied at the same time
// to E = I: the row operations that turn S into R turn I into R^-T (E S = R,
// so E = R S^-1 = R^-T), with no serial back substitution.  On return the
// upper part of S holds R and E (lower triangular) holds R^-T.  Returns
// false (uniformly over the block) at a non-positive pivot.  Thread (g, c)
// owns column c of the rows g, g + ng, ... (no division inside the loops).
// One barrier per step: step j reads row j unscaled and scales on the fly;
// the scaled row j is stored during step j + 1, when no thread reads it.
__device__ bool cholesky_inv_lds(double* S, double* E, int l, int ld) {
  const int ng = NT / l, g = (int)threadIdx.x / l, c = (int)threadIdx.x % l;
  const bool active = g < ng;
  if (active)
    for (int a = g; a < l; a += ng) E[a * ld + c] = (a == c) ? 1.0 : 0.0;
  int pend = -1;   // row whose scaled values thread (0, c) still has to store
  double pend_s = 0.0, pend_e = 0.0;
  for (int j = 0; j < l; ++j) {
    __syncthreads();
    if (g == 0 && pend >= 0) {
      if (c >= pend) S[pend * ld + c] = pend_s;
      if (c <= pend) E[pend * ld + c] = pend_e;
    }
    const double d = S[j * ld + j];
    if (!(d > 0.0)) return false;
    const double ir = 1.0 / sqrt(d);
    if (active) {
      const double xs = S[j * ld + c] * ir, xe = E[j * ld + c] * ir;   // row j of R and of R^-T
      // rows a > j: minus R[j][a] times row j (S: columns >= a; E: columns
      // <= j), four rows per pass; the loads are unconditional (rows past
      // the end clamped) so all twelve are in flight together
      for (int a0 = j + 1 + g; a0 < l; a0 += 4 * ng) {
        double f[4], ts[4], te[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int a = min(a0 + u * ng, l - 1);
          f[u] = S[j * ld + a] * ir;
          ts[u] = S[a * ld + c];
          te[u] = E[a * ld + c];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int a = a0 + u * ng;
          if (a < l) {
            if (c >= a) S[a * ld + c] = ts[u] - f[u] * xs;
            else if (c <= j) E[a * ld + c] = te[u] - f[u] * xe;
          }
        }
      }
      if (g == 0) {
        pend = j;
        pend_s = xs;
        pend_e = xe;
      }
    }
  }
  __syncthreads();
  if (g == 0 && pend >= 0) {
    if (c >= pend) S[pend * ld + c] = pend_s;
    if (c <= pend) E[pend * ld + c] = pend_e;
  }
  __syncthreads();
  return true;
}

// The same factorisation held in registers, for l <= 64: thread (wave w,
// lane c) keeps column c of rows w, w + 4, ..., w + 60 of S (s[16]) and of E
// (e[16]); rows and columns past l are the identity (a block-diagonal
// padding that the factor keeps).  Step j: the wave holding row j takes the
// pivot from lane j, scales the row and publishes rows j of R and of E
// through LDS (double-buffered: a buffer is rewritten two steps later, after
// a barrier every reader has passed, so one barrier per step); every thread
// then subtracts R[j][a] times them from its rows a > j.  Every register
// index is a constant of the unrolled loops.  Returns false (uniformly) at a
// non-positive pivot.
constexpr int LR = 64;
__device__ bool cholesky_inv_regs(double (&s)[16], double (&e)[16], int l, double (*Rrow)[LR], double (*Erow)[LR],
                                  int* fail_flag) {
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < 16; ++m) e[m] = (w + 4 * m == c) ? 1.0 : 0.0;
  if (threadIdx.x == 0) *fail_flag = 0;
  __syncthreads();
  // step j = 4 mm + w4: the register index mm is a constant of the unrolled
  // outer loop, the inner loop stays rolled (a quarter of the code)
#pragma unroll
  for (int mm = 0; mm < LR / 4; ++mm) {
    if (4 * mm >= l) break;
    for (int w4 = 0; w4 < 4; ++w4) {
      const int j = 4 * mm + w4;
      if (j >= l) break;   // uniform
      const int buf = j & 1;
      if (w == w4) {
        const double v = s[mm];
        const double d = __shfl(v, j, 64);
        if (!(d > 0.0) && c == 0) *fail_flag = 1;
        const double ir = 1.0 / sqrt(d);   // not a number after a failed pivot: the flag decides
        const double rv = c >= j ? v * ir : 0.0;
        const double ev = e[mm] * ir;
        s[mm] = rv;
        e[mm] = ev;
        Rrow[buf][c] = rv;
        Erow[buf][c] = ev;
      }
      __syncthreads();
      const double rc = Rrow[buf][c], ec = Erow[buf][c];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        if (w + 4 * m > j) {   // uniform over the wave
          const double f = Rrow[buf][w + 4 * m];
          s[m] -= f * rc;
          e[m] -= f * ec;
        }
      }
    }
  }
  __syncthreads();
  const bool ok = *fail_flag == 0;
  __syncthreads();   // every thread has read the flag before a retry clears it
  return ok;
}

// Rows w + 4 m, column c of G (pitch ldg; + shift on the diagonal) into s;
// the identity past l.
__device__ __forceinline__ void load_gram_regs(double (&s)[16], const double* __restrict__ gram, int64_t ldg, int l,
                                               double shift) {
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cc = min(c, l - 1);
  double u[16], v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {   // clamped addresses: all 32 loads in flight together
    const int ac = min(w + 4 * m, l - 1);
    u[m] = gram[ac * ldg + cc];
    v[m] = gram[cc * ldg + ac];
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int a = w + 4 * m;
    s[m] = (a < l && c < l) ? 0.5 * (u[m] + v[m]) + (a == c ? shift : 0.0) : (a == c ? 1.0 : 0.0);
  }
}

// chol_inv_kernel's contract for l <= 64, with the factorisation in registers.
__global__ void __launch_bounds__(NT) chol_inv_reg_kernel(const double* __restrict__ gram, int l, int64_t rows,
                                                          int mode, double* __restrict__ rinv,
                                                          int* __restrict__ status) {
  __shared__ double Rrow[2][LR], Erow[2][LR];
  __shared__ double red[4];
  __shared__ int fail_flag;
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  double tr = 0.0;
  for (int i = threadIdx.x; i < l; i += NT) tr += gram[i * l + i];
  tr = block_sum(tr, red);
  const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 1.1102230246251565e-16 * tr;
  double s[16], e[16];
  load_gram_regs(s, gram, l, l, mode == 0 ? shift : 0.0);
  bool ok = cholesky_inv_regs(s, e, l, Rrow, Erow, &fail_flag);
  if (!ok && mode != 0) {
    load_gram_regs(s, gram, l, l, shift);
    ok = cholesky_inv_regs(s, e, l, Rrow, Erow, &fail_flag);
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int a = w + 4 * m;
    // R^-1 = E^T (upper): rinv[c][a] = E[a][c] for a >= c; the identity on a breakdown
    if (a < l && c < l) rinv[c * l + a] = ok ? (a >= c ? e[m] : 0.0) : (a == c ? 1.0 : 0.0);
  }
  if (!ok && threadIdx.x == 0) *status = 1;
}

// mode 0: G + shift (the first CholeskyQR pass, always shifted); mode 1: G,
// shifted only if its plain factorisation fails.  shift = 11 (rows l +
// l (l + 1)) u tr(G), u = 2^-53 (shifted CholeskyQR3, Fukaya et al. 2020).
// rinv (l x l, row-major) receives R^-1 (zero below the diagonal).  On a
// breakdown *status is set to 1 and rinv holds the identity.
__global__ void __launch_bounds__(NT) chol_inv_kernel(const double* __restrict__ gram, int l, int64_t rows,
                                                      int mode, double* __restrict__ rinv, int* __restrict__ status) {
  __shared__ double S[LS];
  __shared__ double E[LS];
  __shared__ double red[4];
  const int tid = threadIdx.x, ld = pitch_of(l);
  const int ng = NT / l, g = tid / l, c = tid % l;
  auto load = [&](double shift) {
    __syncthreads();
    load_sym_lds(gram, l, l, shift, S, ld);
  };
  double tr = 0.0;
  for (int i = tid; i < l; i += NT) tr += gram[i * l + i];
  tr = block_sum(tr, red);
  const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 1.1102230246251565e-16 * tr;
  load(mode == 0 ? shift : 0.0);
  bool ok = cholesky_inv_lds(S, E, l, ld);
  if (!ok && mode != 0) {
    load(shift);
    ok = cholesky_inv_lds(S, E, l, ld);
  }
  if (!ok) {
    if (tid == 0) *status = 1;
    if (g < ng)
      for (int i = g; i < l; i += ng) rinv[i * l + c] = (i == c) ? 1.0 : 0.0;
    return;
  }
  // R^-1 = E^T (upper)
  if (g < ng)
    for (int i = g; i < l; i += ng) rinv[i * l + c] = (c >= i) ? E[c * ld + i] : 0.0;
}

// Player at seat `pos` of round `r` of a round-robin over `np` players (np
// even): seat 0 keeps player 0, the others rotate.
__device__ __forceinline__ int seat(int pos, int r, int np) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % (np - 1); }

// Lane-exchange steps of a butterfly over 4 or 8 adjacent lanes (DPP: quad
// permutations [1,0,3,2] and [2,3,0,1], then the mirror within 8 lanes),
// applied to both halves of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int LPP>
__device__ __forceinline__ double lane_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (LPP == 8) v += dpp_f64<0x141>(v);   // row_half_mirror: the other quad of the 8
  return v;
}

// One sweep (np - 1 rounds) of one-sided Jacobi on the rows of S (l x l at
// pitch ld): lane li of pair group pi rotates elements li, li + LPP, ...
// (at most EM of them) of the pair's rows p, q, both held in registers; the
// LPP lanes of a pair are adjacent in one wave and reduce the dot products by
// a butterfly (commutative at every step, so every one of them computes the
// same rotation).  A rotation sets *any_rot.
template <int LPP, int EM>
__device__ void ojac_sweep(double* S, int ld, int l, int np, int pi, int li, bool on, double tol, int* any_rot) {
  for (int r = 0; r < np - 1; ++r) {
    __syncthreads();
    if (!on) continue;
    int p = seat(pi, r, np), q = seat(np - 1 - pi, r, np);
    if (p > q) {
      const int t = p;
      p = q;
      q = t;
    }
    if (q >= l) continue;   // the dummy row of an odd l (uniform over the pair's lanes)
    double x[EM], y[EM];
#pragma unroll
    for (int t = 0; t < EM; ++t) {   // clamped loads (all in flight together), zeroed past the row
      const int e = li + t * LPP, ec = min(e, l - 1);
      const double xv = S[p * ld + ec], yv = S[q * ld + ec];
      x[t] = e < l ? xv : 0.0;
      y[t] = e < l ? yv : 0.0;
    }
    double a = 0.0, b = 0.0, d = 0.0;
#pragma unroll
    for (int t = 0; t < EM; ++t) {
      a += x[t] * x[t];
      b += y[t] * y[t];
      d += x[t] * y[t];
    }
    a = lane_sum<LPP>(a);
    b = lane_sum<LPP>(b);
    d = lane_sum<LPP>(d);
    if (!(fabs(d) > tol * sqrt(a * b))) continue;   // orthogonal to rounding (or not a number)
    const double zeta = (b - a) / (2.0 * d);
    const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
#pragma unroll
    for (int u = 0; u < EM; ++u) {
      const int e = li + u * LPP;
      if (e < l) {
        S[p * ld + e] = cs * x[u] - sn * y[u];
        S[q * ld + e] = sn * x[u] + cs * y[u];
      }
    }
    if (li == 0) *any_rot = 1;
  }
}

// Eigen-decomposition of the symmetric positive semi-definite G = B B^T (l x
// l, the Gram matrix of `rows`-long rows) through its Cholesky factor:
// G + delta I = R^T R with delta = 11 (rows l + l (l + 1)) u tr(G), which keeps
// the factorisation defined for a singular G and moves no eigenvector; then
// one-sided (Hestenes) Jacobi on the rows of R (the columns of R^T): each
// round rotates l/2 disjoint row pairs (round-robin ordering, a group of LPP
// adjacent lanes per pair, dot products reduced by shuffles, both rows held
// in registers) until they are orthogonal to tol = max(1e-15, l u); a sweep
// is l - 1 rounds, sweeps run until one rotates nothing (at most 40).  Then
// R^T V = U Sigma: row j of R holds sigma_j u_j, so the eigenvalues are
// ||row_j||^2 - delta and the eigenvectors the normalised rows, with no
// rotation matrix formed.  On the triangular factor the sweeps are about
// half those of the same iteration on G.  Outputs, with the eigenvalues
// sorted descending (order[j] = index of the j-th largest; ties by index):
//   W (l x l, row-major) eigenvectors by original index, W[i l + j] =
//   component i of eigenvector j; perm[j] = order[j];
//   isg[i] = 1 / sqrt(lam_i) (0 for lam_i <= 0), by original index;
//   sgk[j] = sqrt(lam_order[j]) for j < k (float64) and sigma_f (float32);
//   sig_sorted[j] = sqrt(max(lam_order[j], 0)) for j < l.
// A failed factorisation (G not positive semi-definite to rounding) sets
// *status and leaves W = I and zero eigenvalues.
__global__ void __launch_bounds__(NT) gram_eig_kernel(const double* __restrict__ gram, int l, int64_t rows, int k,
                                                      double* __restrict__ Wout, int32_t* __restrict__ perm,
                                                      double* __restrict__ isg, double* __restrict__ sgk,
                                                      float* __restrict__ sigma_f, double* __restrict__ sig_sorted,
                                                      int* __restrict__ status) {
  __shared__ double S[LS];
  __shared__ double E[LS];   // R^-T from the factorisation (not used here)
  __shared__ double Rrow[2][LR], Erow[2][LR];
  __shared__ double red[4];
  __shared__ double lam[LM], inv_norm[LM];
  __shared__ int any_rot, fail_flag;
  const int tid = threadIdx.x, ld = pitch_of(l);
  const int ng = NT / l, g = tid / l, c = tid % l;
  const bool active = g < ng;
  double tr = 0.0;
  for (int i = tid; i < l; i += NT) tr += gram[i * l + i];
  tr = block_sum(tr, red);
  const double delta = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 1.1102230246251565e-16 * tr;
  bool ok;
  if (l <= LR) {
    // factor in registers, then R (upper) into S
    double sr[16], er[16];
    load_gram_regs(sr, gram, l, l, delta);
    ok = cholesky_inv_regs(sr, er, l, Rrow, Erow, &fail_flag);
    const int cr = tid & 63, wr = tid >> 6;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int a = wr + 4 * m;
      if (a < l && cr < l) S[a * ld + cr] = ok ? (cr >= a ? sr[m] : 0.0) : (a == cr ? 1.0 : 0.0);
    }
  } else {
    load_sym_lds(gram, l, l, delta, S, ld);
    ok = cholesky_inv_lds(S, E, l, ld);
    // R: the upper part of S; clear the rest (identity on a breakdown)
    if (active) {
      for (int i = g; i < l; i += ng) {
        if (!ok)
          S[i * ld + c] = (i == c) ? 1.0 : 0.0;
        else if (c < i)
          S[i * ld + c] = 0.0;
      }
    }
  }
  if (!ok && tid == 0) *status = 1;
  const double shift = ok ? delta : 1.0;
  const int np = l + (l & 1);   // an odd l gets a dummy row l (its pairs are skipped)
  const int npairs = np / 2, LPP = npairs <= NT / 8 ? 8 : 4;
  const int pi = tid / LPP, li = tid % LPP;
  const bool on = ok && pi < npairs;
  const double tol = fmax(1e-15, l * 1.1102230246251565e-16);
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) any_rot = 0;
    // uniform branch: every thread takes the same sweep (and its barriers)
    if (l <= 32)
      ojac_sweep<8, 4>(S, ld, l, np, pi, li, on, tol, &any_rot);
    else if (LPP == 8)
      ojac_sweep<8, 8>(S, ld, l, np, pi, li, on, tol, &any_rot);
    else
      ojac_sweep<4, (LM + 3) / 4>(S, ld, l, np, pi, li, on, tol, &any_rot);
    __syncthreads();
    const int rot = any_rot;
    __syncthreads();   // every thread has read any_rot before it is cleared
    if (!rot) break;
  }
  // eigenvalues ||row_j||^2 - shift, eigenvectors the normalised rows
  for (int j = tid / 64; j < l; j += NT / 64) {
    double a = 0.0;
    for (int e = tid % 64; e < l; e += 64) a += S[j * ld + e] * S[j * ld + e];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (tid % 64 == 0) {
      lam[j] = fmax(a - shift, 0.0);
      inv_norm[j] = a > 0.0 ? 1.0 / sqrt(a) : 0.0;
    }
  }
  __syncthreads();
  for (int i = tid; i < l; i += NT) {
    const double li2 = lam[i];
    int rank = 0;
    for (int j = 0; j < l; ++j) rank += (lam[j] > li2 || (lam[j] == li2 && j < i)) ? 1 : 0;
    const double sg = sqrt(li2);
    perm[rank] = i;
    isg[i] = sg > 0.0 ? 1.0 / sg : 0.0;
    sig_sorted[rank] = sg;
    if (rank < k) {
      sgk[rank] = sg;
      sigma_f[rank] = (float)sg;
    }
  }
  if (active)
    for (int i = g; i < l; i += ng) Wout[i * l + c] = S[c * ld + i] * inv_norm[c];
}

// ---- sketches above 96 columns ---------------------------------------------------
// G (l x l, pitch ld) + shift on the diagonal, shift = 11 (rows l + l (l + 1))
// u tr(G): the first CholeskyQR pass's, as in the one-workgroup form.  One
// workgroup.
__global__ void __launch_bounds__(NT) add_shift_kernel(double* __restrict__ G, int l, int64_t ld, int64_t rows,
                                                       double* __restrict__ shift_out) {
  __shared__ double red[4];
  double tr = 0.0;
  for (int i = threadIdx.x; i < l; i += NT) tr += G[i * ld + i];
  tr = block_sum(tr, red);
  const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 1.1102230246251565e-16 * tr;
  for (int i = threadIdx.x; i < l; i += NT) G[i * ld + i] += shift;
  if (shift_out && threadIdx.x == 0) *shift_out = shift;
}

// Cholesky factor of the b x b diagonal block at G (pitch ldg, b <= 64), in
// registers: R_jj (upper) into R (pitch ldr), R_jj^-T (lower) into E (pitch
// b).  A non-positive pivot sets *status (R_jj = E = I).
constexpr int kCholBlock = 64;
static_assert(kCholBlock <= LR, "diagonal blocks factor in registers");
__global__ void __launch_bounds__(NT) chol_block_kernel(const double* __restrict__ G, int64_t ldg, int b,
                                                        double* __restrict__ R, int64_t ldr, double* __restrict__ E,
                                                        int* __restrict__ status) {
  __shared__ double Rrow[2][LR], Erow[2][LR];
  __shared__ int fail_flag;
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  double sr[16], er[16];
  load_gram_regs(sr, G, ldg, b, 0.0);
  const bool ok = cholesky_inv_regs(sr, er, b, Rrow, Erow, &fail_flag);
  if (!ok && threadIdx.x == 0) *status = 1;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int a = w + 4 * m;
    if (a < b && c < b) {
      R[a * ldr + c] = ok ? (c >= a ? sr[m] : 0.0) : (a == c ? 1.0 : 0.0);
      E[a * b + c] = ok ? (c <= a ? er[m] : 0.0) : (a == c ? 1.0 : 0.0);
    }
  }
}

__global__ void fill_f64_kernel(double* __restrict__ p, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// One round of block one-sided (Hestenes) Jacobi on the columns of M (l x l;
// column j contiguous at M + j l).  The columns form blocks of BS; the
// workgroup of block pair (P, Q) of round r stages their (up to) 2 BS columns
// in LDS (dynamic, 2 BS (l | 1) doubles: one batch of loads), forms their
// Gram matrix H = M_c^T M_c, runs one cyclic two-sided Jacobi sweep on H
// (rotating a pair unless |h_pq| <= tol sqrt(h_pp h_qq)) while accumulating
// the rotations in J, and writes M_c J back.  Any rotation sets *rotated.
// Repeated sweeps until none rotates leave every column pair orthogonal to
// tol: M V with V orthogonal and never formed.  Slots past column l stay zero
// and are never rotated.
template <int BS>
__global__ void __launch_bounds__(NT) bjac_round_kernel(double* __restrict__ M, int l, int nb, int r, int npb,
                                                        double tol, int* __restrict__ rotated) {
  constexpr int W = 2 * BS;   // slots; W * W <= NT
  static_assert(W * W <= NT && W % 4 == 0, "block shape");
  extern __shared__ double X[];   // W x lp: slot a's column at X + a lp
  __shared__ double H[W * (W + 1)], J[W * (W + 1)];
  __shared__ int col[W];
  __shared__ int total_rot;
  int P = seat(blockIdx.x, r, npb), Q = seat(npb - 1 - blockIdx.x, r, npb);
  if (P >= nb || Q >= nb) return;   // the dummy block of an odd count (uniform over the workgroup)
  const int tid = threadIdx.x, lp = l | 1;   // odd pitch: the W slots of one row fall in distinct banks
  if (tid < W) {
    const int c = (tid < BS ? P * BS + tid : Q * BS + tid - BS);
    col[tid] = c < l ? c : -1;
  }
  if (tid == 0) total_rot = 0;
  __syncthreads();
  // Each block's columns are one contiguous range of M: eight loads in flight
  // per thread per batch, then their LDS stores; the slots of a partial
  // block's missing columns are zero.
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int blk = h == 0 ? P : Q, wb = min(BS, l - blk * BS);
    const double* src = M + (int64_t)blk * BS * l;
    const int count = wb * l;
    for (int base = 0; base < count; base += 8 * NT) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + tid + u * NT;
        v[u] = idx < count ? src[idx] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + tid + u * NT;
        if (idx < count) {
          const int sl = idx / l, k = idx - sl * l;
          X[(h * BS + sl) * lp + k] = v[u];
        }
      }
    }
    for (int idx = count + tid; idx < BS * l; idx += NT) {
      const int sl = idx / l, k = idx - sl * l;
      X[(h * BS + sl) * lp + k] = 0.0;
    }
  }
  __syncthreads();
  // H = M_c^T M_c in 4 x 4 tiles: thread (tile, split) sums rows split,
  // split + S, ... of its tile (the S splits of a tile are adjacent lanes,
  // reduced by shuffles)
  {
    constexpr int TI = W / 4, S = NT / (TI * TI);
    static_assert(S <= 64 && (S & (S - 1)) == 0, "tile split");
    const int tile = tid / S, sp = tid % S, ti = tile / TI, tj = tile % TI;
    double acc[4][4] = {};
    for (int k = sp; k < l; k += S) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = X[(4 * ti + u) * lp + k];
        b[u] = X[(4 * tj + u) * lp + k];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
#pragma unroll
    for (int off = 1; off < S; off <<= 1)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += __shfl_xor(acc[u][v], off, 64);
    if (sp == 0)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int hi = 4 * ti + u, hj = 4 * tj + v;
          H[hi * (W + 1) + hj] = acc[u][v];
          J[hi * (W + 1) + hj] = (hi == hj) ? 1.0 : 0.0;
        }
  }
  // One cyclic Jacobi sweep on H, rotations accumulated in J (new column p =
  // c x_p - s x_q, new column q = s x_p + c x_q; H <- J_r^T H J_r, J <- J
  // J_r).  Thread (i, j) computes the rotations of the pairs holding i and j
  // itself (bitwise the same as every other thread that computes them), so
  // a round needs only the barriers around its stores.  One sweep per visit:
  // the outer sweeps converge in about as many visits as with a fully
  // diagonalised H, at a fraction of the inner rounds.
  const int i = tid / W, j = tid % W;
  const bool el = tid < W * W;
  for (int rr = 0; rr < W - 1; ++rr) {
    __syncthreads();
    double hn = 0.0, jn = 0.0;
    if (el) {
      double cs2[2], cp2[2];
      int pt2[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int x = e == 0 ? i : j;
        // position of slot x in the round-robin seating of round rr, its partner's slot
        const int pos = x == 0 ? 0 : (x - 1 - rr + 2 * (W - 1)) % (W - 1) + 1;
        const int y = seat(W - 1 - pos, rr, W);
        const int p = min(x, y), q = max(x, y);
        const double hpp = H[p * (W + 1) + p], hqq = H[q * (W + 1) + q], hpq = H[p * (W + 1) + q];
        double cc = 1.0, ss = 0.0;
        if (fabs(hpq) > tol * sqrt(hpp * hqq)) {
          const double zeta = (hqq - hpp) / (2.0 * hpq);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          cc = 1.0 / sqrt(1.0 + t * t);
          ss = cc * t;
          total_rot = 1;
        }
        cs2[e] = cc;
        cp2[e] = x == p ? -ss : ss;
        pt2[e] = y;
      }
      const int pi = pt2[0], pj = pt2[1];
      const double si = cs2[0], ti = cp2[0], sj = cs2[1], tj = cp2[1];
      hn = si * (sj * H[i * (W + 1) + j] + tj * H[i * (W + 1) + pj]) +
           ti * (sj * H[pi * (W + 1) + j] + tj * H[pi * (W + 1) + pj]);
      jn = sj * J[i * (W + 1) + j] + tj * J[i * (W + 1) + pj];
    }
    __syncthreads();
    if (el) {
      H[i * (W + 1) + j] = hn;
      J[i * (W + 1) + j] = jn;
    }
  }
  __syncthreads();
  if (!total_rot) return;   // read after the last barrier: uniform
  if (tid == 0) atomicOr(rotated, 1);
  // M_c <- M_c J from the staged copy: thread (group of 4 output columns,
  // row), NT / (W / 4) consecutive rows per pass; each staged value feeds 4
  // outputs
  constexpr int G4 = W / 4, RP = NT / G4;
  const int bg = tid / RP, rsub = tid % RP;
  double jc[W][4];
#pragma unroll
  for (int a = 0; a < W; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) jc[a][v] = J[a * (W + 1) + 4 * bg + v];
  int cb[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) cb[v] = col[4 * bg + v];
  for (int k = rsub; k < l; k += RP) {
    double y[4] = {};
#pragma unroll
    for (int a = 0; a < W; ++a) {
      const double x = X[a * lp + k];
#pragma unroll
      for (int v = 0; v < 4; ++v) y[v] += x * jc[a][v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (cb[v] >= 0) M[(int64_t)cb[v] * l + k] = y[v];
  }
}

// Column j of M (l x l, contiguous columns) = sigma_j u_j with sigma_j^2 the
// eigenvalue of G + shift: lam[j] = max(||m_j||^2 - shift, 0) and column j of
// W = m_j / ||m_j|| (one workgroup per column).
__global__ void __launch_bounds__(NT) eig_finish_kernel(const double* __restrict__ M, int l,
                                                        const double* __restrict__ shift, double* __restrict__ W,
                                                        double* __restrict__ lam) {
  __shared__ double red[4];
  const double* m = M + (int64_t)blockIdx.x * l;
  double a = 0.0;
  for (int k = threadIdx.x; k < l; k += NT) a += m[k] * m[k];
  a = block_sum(a, red);
  const double inv = a > 0.0 ? 1.0 / sqrt(a) : 0.0;
  for (int k = threadIdx.x; k < l; k += NT) W[(int64_t)blockIdx.x * l + k] = m[k] * inv;
  if (threadIdx.x == 0) lam[blockIdx.x] = fmax(a - *shift, 0.0);
}

__global__ void set_flag_kernel(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

}  // namespace

amm_status chol_qr_factor(const double* gram, int l, int64_t rows, int mode, double* rinv, int* status,
                          hipStream_t s) {
  if (l < 1 || l > kSmallEigMax) return fail(AMM_EUNSUPPORTED, "device CholeskyQR factor needs 1 <= l <= %d", kSmallEigMax);
  TimedLaunch tl("rsvd_chol", s);
  if (l <= LR)
    hipLaunchKernelGGL(chol_inv_reg_kernel, dim3(1), dim3(NT), 0, s, gram, l, rows, mode, rinv, status);
  else
    hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(NT), 0, s, gram, l, rows, mode, rinv, status);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}

amm_status gram_eig(const double* gram, int l, int64_t rows, int k, double* W, int32_t* perm, double* isg,
                    double* sgk, float* sigma_f, double* sig_sorted, int* status, hipStream_t s) {
  if (l < 1 || l > kSmallEigMax || k > l) return fail(AMM_EUNSUPPORTED, "device Gram eigensolver needs k <= l <= %d", kSmallEigMax);
  TimedLaunch tl("rsvd_eig", s);
  hipLaunchKernelGGL(gram_eig_kernel, dim3(1), dim3(NT), 0, s, gram, l, rows, k, W, perm, isg, sgk, sigma_f,
                     sig_sorted, status);
  AMM_HIP(hipGetLastError());
  return AMM_OK;
}


// ---- sketches above 96 columns: blocked CholeskyQR, one-sided Jacobi ------------

int chol_blocks(int l) { return (l + kCholBlock - 1) / kCholBlock; }

// Upper Cholesky factor R of G (+ the shift when `shift`; G l x l, overwritten
// by the trailing updates) in blocks of 64.  The passes after a shifted one
// factor a basis whose condition the shift has bounded, so they run unshifted
// (a non-positive pivot there sets *status, which the caller reports).  Blocks: each diagonal block in one workgroup (R_jj and
// R_jj^-T into E, 64 x 64 per block), the block row of R beside it by one
// GEMM with R_jj^-T, the trailing matrix by one more.
amm_status chol_qr_blocked(double* G, int l, int64_t rows, bool shift, double* R, double* E, int* status,
                           hipStream_t s, double* shift_out) {
  const int nb = chol_blocks(l);
  if (shift) hipLaunchKernelGGL(add_shift_kernel, dim3(1), dim3(NT), 0, s, G, l, (int64_t)l, rows, shift_out);
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)std::min<int64_t>(((int64_t)l * l + 255) / 256, 4096)), dim3(256),
                     0, s, R, (int64_t)l * l, 0.0);
  AMM_HIP(hipGetLastError());
  for (int jb = 0; jb < nb; ++jb) {
    const int j0 = jb * kCholBlock, b = std::min(kCholBlock, l - j0), j1 = j0 + b;
    double* Ej = E + (size_t)jb * kCholBlock * kCholBlock;
    {
      TimedLaunch tl("rsvd_chol", s);
      hipLaunchKernelGGL(chol_block_kernel, dim3(1), dim3(NT), 0, s, G + (int64_t)j0 * l + j0, (int64_t)l, b,
                         R + (int64_t)j0 * l + j0, (int64_t)l, Ej, status);
      AMM_HIP(hipGetLastError());
    }
    if (j1 < l) {
      const int w = l - j1;
      // R[j0:j1, j1:l] = R_jj^-T G[j0:j1, j1:l]
      AMM_TRY(gemm_f64(b, w, b, 1.0, Ej, b, 1, G + (int64_t)j0 * l + j1, l, 1, 0.0, R + (int64_t)j0 * l + j1, l, s));
      // G[j1:l, j1:l] -= R[j0:j1, j1:l]^T R[j0:j1, j1:l]
      AMM_TRY(gemm_f64(w, w, b, -1.0, R + (int64_t)j0 * l + j1, 1, l, R + (int64_t)j0 * l + j1, l, 1, 1.0,
                       G + (int64_t)j1 * l + j1, l, s));
    }
  }
  return AMM_OK;
}

// Q = Y R^-1 by block columns: Q_j = Y_j X_jj - Q_{<j} (R_{<j, j} X_jj), X_jj =
// R_jj^-1 = (R_jj^-T)^T.  P: scratch of l x 64.
amm_status chol_qr_apply(const double* Y, int64_t rows, int l, const double* R, const double* E, double* Q, double* P,
                         hipStream_t s) {
  const int nb = chol_blocks(l);
  for (int jb = 0; jb < nb; ++jb) {
    const int j0 = jb * kCholBlock, b = std::min(kCholBlock, l - j0);
    const double* Ej = E + (size_t)jb * kCholBlock * kCholBlock;   // X_jj(i, k) = Ej[k b + i]
    AMM_TRY(gemm_f64(rows, b, b, 1.0, Y + j0, l, 1, Ej, 1, b, 0.0, Q + j0, l, s));
    if (j0 > 0) {
      AMM_TRY(gemm_f64(j0, b, b, 1.0, R + j0, l, 1, Ej, 1, b, 0.0, P, b, s));
      AMM_TRY(gemm_f64(rows, b, j0, -1.0, Q, l, 1, P, b, 1, 1.0, Q + j0, l, s));
    }
  }
  return AMM_OK;
}

// Eigen-decomposition of the symmetric positive semi-definite G = B B^T (l x
// l, the Gram matrix of `rows`-long rows; overwritten): G + shift = R^T R by
// the blocked Cholesky factorisation (R into R, E its scratch), then block
// one-sided Jacobi on the columns of R^T (the rows of R, contiguous in the
// row-major R; the lower-triangular orientation converges in about half the
// sweeps of the same iteration on G): R^T V = U Sigma with U the eigenvectors
// of G and Sigma^2 - shift its eigenvalues.  Sweeps (8-column blocks, 4 above
// 1024 columns; round-robin block pairs, one launch per round) run until one
// rotates nothing (at most 40).  W (l x l) receives the eigenvectors as contiguous
// columns, lam_host the eigenvalues (unsorted); dev (2 + l doubles) is device
// scratch.
amm_status gram_eig_large(double* G, int l, int64_t rows, double* R, double* E, double* W, double* dev, int* flag,
                          int* status, std::vector<double>& lam_host, int* sweeps_out, hipStream_t s) {
  double* shift = dev;
  double* lam = dev + 2;
  AMM_TRY(chol_qr_blocked(G, l, rows, true, R, E, status, s, shift));
  // 8-column blocks while the staged pair fits in LDS (l <= 1024), 4 beyond
  const int BS = l <= 1024 ? 8 : 4;
  const int nb = (l + BS - 1) / BS, npb = nb + (nb & 1);
  const size_t lds = (size_t)2 * BS * (l | 1) * sizeof(double);
  if (lds > 140 * 1024) return fail(AMM_EUNSUPPORTED, "sketch of %d columns too wide for the device eigensolver", l);
  const void* kern = BS == 8 ? (const void*)bjac_round_kernel<8> : (const void*)bjac_round_kernel<4>;
  if (lds > 64 * 1024) AMM_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const double tol = std::max(1e-15, l * 1.1102230246251565e-16);
  int sweep = 0, h = 1;
  TimedLaunch tl("rsvd_eig", s);
  for (; sweep < 40 && h; ++sweep) {
    hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(64), 0, s, flag);
    for (int r = 0; r < npb - 1; ++r) {
      if (BS == 8)
        hipLaunchKernelGGL(bjac_round_kernel<8>, dim3((unsigned)(npb / 2)), dim3(NT), lds, s, R, l, nb, r, npb, tol,
                           flag);
      else
        hipLaunchKernelGGL(bjac_round_kernel<4>, dim3((unsigned)(npb / 2)), dim3(NT), lds, s, R, l, nb, r, npb, tol,
                           flag);
    }
    AMM_HIP(hipGetLastError());
    AMM_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    AMM_HIP(hipStreamSynchronize(s));
  }
  hipLaunchKernelGGL(eig_finish_kernel, dim3((unsigned)l), dim3(NT), 0, s, R, l, shift, W, lam);
  AMM_HIP(hipGetLastError());
  lam_host.resize(l);
  AMM_HIP(hipMemcpyAsync(lam_host.data(), lam, l * sizeof(double), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipStreamSynchronize(s));
  if (sweeps_out) *sweeps_out = sweep;
  return AMM_OK;
}

}  // namespace amm
