// C ABI of the approximate-product library: handles, validation, dispatch.
//
// Combination rules (eq. (2.1)-(2.3) of the paper):
//   zeroth order  out = Atil B
//   first order   out = Atil B + Delta A Btil
// "left" products (Atil B) and "right" products (X Btil for a dense X) are
// dispatched per decomposition kind; a sparse handle contributes its CSR part
// and then its truncated residue.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <functional>
#include <map>

#include "amm_internal.hpp"

namespace amm {

namespace {
thread_local char g_msg[512] = "";
}

thread_local KernelTimer* g_timer = nullptr;

namespace {
// Routes the launches of one API call to the context's timer when enabled.
// Per API call: the context's launch timer (if timing is on) and its
// allocator for every device buffer the call makes.
struct TimerScope {
  KernelTimer* prev;
  const AllocFns* prev_alloc;
  DevBuf* prev_part;
  explicit TimerScope(amm_ctx* ctx) : prev(g_timer), prev_alloc(g_alloc), prev_part(g_gemm_part) {
    g_timer = (ctx && ctx->timing) ? &ctx->timer : nullptr;
    g_alloc = ctx ? &ctx->alloc : nullptr;
    g_gemm_part = ctx ? &ctx->gemm_part : nullptr;
  }
  // calls on a handle alone allocate with the handle's allocator
  explicit TimerScope(const amm_dec* d) : prev(g_timer), prev_alloc(g_alloc), prev_part(g_gemm_part) {
    g_timer = nullptr;
    g_alloc = d ? &d->alloc : nullptr;
    g_gemm_part = nullptr;
  }
  ~TimerScope() {
    g_timer = prev;
    g_alloc = prev_alloc;
    g_gemm_part = prev_part;
  }
};
}  // namespace

amm_status fail(amm_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
  va_end(ap);
  return st;
}

amm_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(AMM_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(AMM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

thread_local const AllocFns* g_alloc = nullptr;
thread_local DevBuf* g_gemm_part = nullptr;

amm_status DevBuf::alloc(size_t b) {
  release();
  fns = AllocFns{};
  if (b == 0) return AMM_OK;
  if (g_alloc && g_alloc->alloc) {
    ptr = g_alloc->alloc(b, g_alloc->device, g_alloc->user);
    if (!ptr) return fail(AMM_ENOMEM, "caller's allocator returned NULL for %zu bytes", b);
    fns = *g_alloc;
  } else {
    hipError_t e = hipMalloc(&ptr, b);
    if (e != hipSuccess) {
      ptr = nullptr;
      return hip_fail(e, "hipMalloc");
    }
  }
  bytes = b;
  return AMM_OK;
}

amm_status DevBuf::reserve(size_t b) {
  if (b <= bytes) return AMM_OK;
  return alloc(b);
}

namespace {

int log2_exact(int64_t n) {
  if (n < 2 || (n & (n - 1)) != 0) return -1;
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

// circulant handles of any side n in [2, 16384]; powers of two run the fused
// single-kernel product, other sides the float64 chirp-convolution steps
bool circ_side_ok(int64_t n) { return n >= 2 && n <= 16384; }

amm_status circ_columns(amm_ctx* ctx, const amm_dec* b, const float* B, int64_t p, float* out, bool acc,
                        hipStream_t s, int64_t ldb = 0, int64_t ldo = 0) {
  if (b->K_eff == 0) {
    if (!acc) AMM_TRY(fill_f32(out, b->n * p, 0.f, s));
    return AMM_OK;
  }
  if (is_pow2(b->n))
    return cd_apply_columns(ctx, log2_exact(b->n), b->K_eff, b->shifts.as<int32_t>(), b->L.as<float2>(), B, p, out, acc,
                            s, b->pairs_of(false), b->lists16(false), b->l16_inv, ldb, ldo);
  if ((ldb && ldb != p) || (ldo && ldo != p)) return fail(AMM_EUNSUPPORTED, "strided operands need n a power of two");
  return cd_apply_general(ctx, (int)b->n, b->K_eff, b->shifts.as<int32_t>(), b->L.as<float2>(), B, p, out, acc, s,
                          b->lists16(false), b->l16_inv);
}

// exp(-2 pi i m / n) with the angle reduced to the first octant, so every entry
// is the correctly rounded value of an exactly representable fraction m / n.
void twiddle_value(int64_t m, int64_t n, long double* c, long double* s) {
  // angle = 2 pi m / n; use m/n in [0, 1)
  const long double pi = 3.141592653589793238462643383279502884L;
  const int64_t q = m * 8;           // position in eighths of a turn
  const int64_t oct = q / n;         // octant 0..7
  const int64_t rem = q - oct * n;   // remainder within the octant, times n
  long double a = (long double)rem / (long double)n * (pi / 4);  // in [0, pi/4)
  long double cs, sn;
  // in octant o, angle = o * pi/4 + a
  switch (oct) {
    case 0: cs = cosl(a); sn = sinl(a); break;
    case 1: cs = sinl(pi / 4 - a); sn = cosl(pi / 4 - a); break;
    case 2: cs = -sinl(a); sn = cosl(a); break;
    case 3: cs = -cosl(pi / 4 - a); sn = sinl(pi / 4 - a); break;
    case 4: cs = -cosl(a); sn = -sinl(a); break;
    case 5: cs = -sinl(pi / 4 - a); sn = -cosl(pi / 4 - a); break;
    case 6: cs = sinl(a); sn = -cosl(a); break;
    default: cs = cosl(pi / 4 - a); sn = -sinl(pi / 4 - a); break;
  }
  *c = cs;
  *s = -sn;  // exp(-i angle)
}

}  // namespace

amm_status twiddles32(amm_ctx* ctx, int log2n, const float2** out) {
  auto it = ctx->tw32.find(log2n);
  if (it == ctx->tw32.end()) {
    const int64_t n = int64_t(1) << log2n;
    std::vector<float2> h(n);
    for (int64_t m = 0; m < n; ++m) {
      long double c, s;
      twiddle_value(m, n, &c, &s);
      h[m] = float2{(float)c, (float)s};
    }
    DevBuf b;
    AMM_TRY(b.alloc(n * sizeof(float2)));
    AMM_HIP(hipMemcpy(b.ptr, h.data(), n * sizeof(float2), hipMemcpyHostToDevice));
    it = ctx->tw32.emplace(log2n, std::move(b)).first;
  }
  *out = it->second.as<float2>();
  return AMM_OK;
}

amm_status twiddles64(amm_ctx* ctx, int log2n, const double2** out) {
  auto it = ctx->tw64.find(log2n);
  if (it == ctx->tw64.end()) {
    const int64_t n = int64_t(1) << log2n;
    std::vector<double2> h(n);
    for (int64_t m = 0; m < n; ++m) {
      long double c, s;
      twiddle_value(m, n, &c, &s);
      h[m] = double2{(double)c, (double)s};
    }
    DevBuf b;
    AMM_TRY(b.alloc(n * sizeof(double2)));
    AMM_HIP(hipMemcpy(b.ptr, h.data(), n * sizeof(double2), hipMemcpyHostToDevice));
    it = ctx->tw64.emplace(log2n, std::move(b)).first;
  }
  *out = it->second.as<double2>();
  return AMM_OK;
}

amm_status tsvd_residual(const float* A, int64_t m, int64_t n, int k, const float* US, const float* V,
                         float* dst, hipStream_t s) {
  AMM_HIP(hipMemcpyAsync(dst, A, m * n * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (k > 0) AMM_TRY(gemm_f32(m, n, k, -1.f, MatView{US, k, 1}, MatView{V, 1, k}, 1.f, dst, n, s, "gemm_residual"));
  return AMM_OK;
}

// ---- product dispatch ---------------------------------------------------------
namespace {

bool is_circ(const amm_dec* d) { return d->kind == AMM_CIRCULANT; }
bool is_tsvd(const amm_dec* d) { return d->kind == AMM_TSVD; }
bool is_sparse(const amm_dec* d) { return (d->kind & AMM_SPARSE) != 0; }
bool is_sfft(const amm_dec* d) { return d->kind == AMM_SFFT; }

// Rectangular circulant operand: out (m x p) = Atil B block by block.  Row
// blocks write their s output rows (the last block's overhang goes to the
// scratch and only the valid rows are copied); column blocks accumulate over
// the matching row slices of B (the last slice, zero-padded, from scratch).
// scratch: s x p floats.
amm_status blocked_apply(amm_ctx* ctx, const amm_dec* d, const float* B, int64_t p, float* out, float* scratch,
                         hipStream_t s) {
  const int64_t sd = d->block_rows ? d->n : d->m;
  const int nb = (int)d->blocks.size();
  for (int j = 0; j < nb; ++j) {
    const amm_dec* b = d->blocks[j];
    const int64_t lo = (int64_t)j * sd;
    const int64_t valid = std::min<int64_t>(sd, (d->block_rows ? d->m : d->n) - lo);
    const bool acc = !d->block_rows && j > 0;
    if (d->block_rows) {
      float* dst = valid == sd ? out + lo * p : scratch;
      AMM_TRY(circ_columns(ctx, b, B, p, dst, false, s));
      if (valid < sd)
        AMM_HIP(hipMemcpyAsync(out + lo * p, scratch, valid * p * sizeof(float), hipMemcpyDeviceToDevice, s));
    } else {
      const float* src = B + lo * p;
      if (valid < sd) {
        AMM_TRY(fill_f32(scratch, sd * p, 0.f, s));
        AMM_HIP(hipMemcpyAsync(scratch, src, valid * p * sizeof(float), hipMemcpyDeviceToDevice, s));
        src = scratch;
      }
      if (b->K_eff == 0) {
        if (!acc) AMM_TRY(fill_f32(out, d->m * p, 0.f, s));
      } else {
        AMM_TRY(circ_columns(ctx, b, src, p, out, acc, s));
      }
    }
  }
  return AMM_OK;
}

// out (m x p) (+)= Atil B
amm_status left_apply(amm_ctx* ctx, const amm_dec* d, const float* B, int64_t p, float* out,
                      bool acc, hipStream_t s) {
  if (!d->blocks.empty()) {
    if (acc) return fail(AMM_EUNSUPPORTED, "blocked circulant operand inside a sum");
    const int64_t sd = d->block_rows ? d->n : d->m;
    AMM_TRY(ctx->scratch[6].reserve((size_t)sd * p * sizeof(float)));
    return blocked_apply(ctx, d, B, p, out, ctx->scratch[6].as<float>(), s);
  }
  if (is_sparse(d)) {
    // The row gathers of the sparse part (and the column reads and writes of
    // a circulant residue) at a row pitch that is a large power of two all
    // land on one L2 channel: both read a copy of B at a spread pitch, the
    // residue's product goes to a spread-pitch buffer, and the sparse part
    // writes out = S B + that buffer.
    const int64_t sp = spread_pitch(p);
    const amm_dec* in = d->inner;
    if (sp != p && d->nnz > 0 && ((uintptr_t)B % 16) == 0 && ((uintptr_t)out % 16) == 0) {
      AMM_TRY(ctx->scratch[14].reserve((size_t)d->n * sp * sizeof(float)));
      float* Bs = ctx->scratch[14].as<float>();
      AMM_TRY(repitch_f32(B, p, d->n, p, Bs, sp, s));
      if (!acc && in && is_circ(in) && in->blocks.empty() && is_pow2(in->n) && in->K_eff > 0) {
        AMM_TRY(ctx->scratch[15].reserve((size_t)d->m * sp * sizeof(float)));
        float* Y = ctx->scratch[15].as<float>();
        AMM_TRY(cd_apply_columns(ctx, log2_exact(in->n), in->K_eff, in->shifts.as<int32_t>(), in->L.as<float2>(), Bs,
                                 p, Y, false, s, in->pairs_of(false), in->lists16(false), in->l16_inv, sp, sp));
        return spmm_csr(d, Bs, sp, p, out, false, s, Y, sp);
      }
      if (in) {
        AMM_TRY(left_apply(ctx, in, B, p, out, acc, s));
        acc = true;
      }
      return spmm_csr(d, Bs, sp, p, out, acc, s);
    }
    if (in) {
      AMM_TRY(left_apply(ctx, in, B, p, out, acc, s));
      acc = true;
    }
    return spmm_csr(d, B, p, p, out, acc, s);
  }
  if (is_sfft(d)) return sfft_left_apply(ctx, d, B, p, out, acc, s);
  if (is_circ(d)) return circ_columns(ctx, d, B, p, out, acc, s);
  if (is_tsvd(d)) {
    const int k = d->K_eff;
    if (k == 0) {
      if (!acc) AMM_TRY(fill_f32(out, d->m * p, 0.f, s));
      return AMM_OK;
    }
    AMM_TRY(ctx->scratch[0].reserve((size_t)k * p * sizeof(float)));
    float* G = ctx->scratch[0].as<float>();
    if (!acc && tsvd_split_shapes(d->m, d->n, p, k, 0)) {
      const size_t need = tsvd_split_scratch(d->m, d->n, p, k, 0);
      AMM_TRY(ctx->scratch[4].reserve(need * sizeof(float)));
      return tsvd_split_product(d->m, d->n, p, k, 0, d->V.as<float>(), d->US.as<float>(), B, nullptr, nullptr,
                                nullptr, ctx->scratch[4].as<float>(), need, out, s);
    }
    if (!acc && tsvd_fast_shapes(d->m, d->n, p, k, 0)) {
      const size_t gp = (size_t)4 * k * p;
      AMM_TRY(ctx->scratch[4].reserve(gp * sizeof(float)));
      return tsvd_fast_product(d->m, d->n, p, k, 0, d->V.as<float>(), d->US.as<float>(), B, nullptr,
                               nullptr, nullptr, ctx->scratch[4].as<float>(), gp, nullptr, 0, out, s);
    }
    // G = V^T B  (k x p)
    AMM_TRY(gemm_f32(k, p, d->n, 1.f, MatView{d->V.as<float>(), 1, k}, MatView{B, p, 1}, 0.f, G, p, s, "gemm_VtB"));
    // out = (U S) G
    AMM_TRY(gemm_f32(d->m, p, k, 1.f, MatView{d->US.as<float>(), k, 1}, MatView{G, p, 1},
                     acc ? 1.f : 0.f, out, p, s, "gemm_out"));
    return AMM_OK;
  }
  return fail(AMM_EINVAL, "unknown decomposition kind %d", d->kind);
}

// out (rows x p) (+)= X Btil, X dense rows x n
amm_status right_apply(amm_ctx* ctx, const float* X, int64_t rows, const amm_dec* d, float* out,
                       bool acc, hipStream_t s) {
  const int64_t n = d->m, p = d->n;  // Btil is n x p
  if (is_sfft(d)) return fail(AMM_EUNSUPPORTED, "a Fourier-sparsified right operand pairs only with one on the left");
  if (is_sparse(d)) {
    AMM_TRY(dense_times_csr(ctx, X, rows, d, out, acc, s));
    if (d->inner) AMM_TRY(right_apply(ctx, X, rows, d->inner, out, true, s));
    return AMM_OK;
  }
  if (is_circ(d)) {
    if (d->K_eff == 0) {
      if (!acc) AMM_TRY(fill_f32(out, rows * p, 0.f, s));
      return AMM_OK;
    }
    if (!is_pow2(d->n))
      return cd_apply_rows_general(ctx, (int)d->n, d->K_eff, d->shifts_adj.as<int32_t>(), d->Ladj.as<float2>(), X,
                                   rows, out, acc, s, d->lists16(true), d->l16_inv);
    return cd_apply_rows(ctx, log2_exact(d->n), d->K_eff, d->shifts_adj.as<int32_t>(),
                         d->Ladj.as<float2>(), X, rows, out, acc, s, d->pairs_of(true), d->lists16(true), d->l16_inv);
  }
  if (is_tsvd(d)) {
    const int k = d->K_eff;
    if (k == 0) {
      if (!acc) AMM_TRY(fill_f32(out, rows * p, 0.f, s));
      return AMM_OK;
    }
    AMM_TRY(ctx->scratch[1].reserve((size_t)rows * k * sizeof(float)));
    float* T = ctx->scratch[1].as<float>();
    // T = X U  (rows x k), out (+)= (T S) V^T = T (V S)^T
    AMM_TRY(gemm_f32(rows, k, n, 1.f, MatView{X, n, 1}, MatView{d->U.as<float>(), k, 1}, 0.f, T, k, s));
    AMM_TRY(gemm_f32(rows, p, k, 1.f, MatView{T, k, 1}, MatView{d->VS.as<float>(), 1, k},
                     acc ? 1.f : 0.f, out, p, s));
    return AMM_OK;
  }
  return fail(AMM_EINVAL, "unknown decomposition kind %d", d->kind);
}

// Pointer to Delta A (m x n) for the left operand, materialised in scratch[2]
// when the handle only borrows A.
amm_status residual_of(amm_ctx* ctx, const amm_dec* d, const float** out, hipStream_t s) {
  if (d->residual.ptr) {
    *out = d->residual.as<float>();
    return AMM_OK;
  }
  if (is_sparse(d)) {
    if (d->inner && (d->inner->residual.ptr || d->inner->A_borrowed))
      return residual_of(ctx, d->inner, out, s);
    return fail(AMM_ESTATE, "sparse handle has no residual for a first-order product");
  }
  if (is_tsvd(d) && d->A_borrowed) {
    const int64_t mn = d->m * d->n;
    AMM_TRY(ctx->scratch[2].reserve(mn * sizeof(float)));
    float* R = ctx->scratch[2].as<float>();
    AMM_HIP(hipMemcpyAsync(R, d->A_borrowed, mn * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (d->K_eff > 0)
      AMM_TRY(gemm_f32(d->m, d->n, d->K_eff, -1.f, MatView{d->US.as<float>(), d->K_eff, 1},
                       MatView{d->V.as<float>(), 1, d->K_eff}, 1.f, R, d->n, s));
    *out = R;
    return AMM_OK;
  }
  return fail(AMM_ESTATE, "left operand keeps no Delta A (decompose with keep_residual or pass A)");
}

}  // namespace
}  // namespace amm

using namespace amm;

amm_dec::~amm_dec() {
  if (inner) delete inner;
  for (amm_dec* b : blocks) delete b;
}

amm_batch_plan::~amm_batch_plan() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (own) (void)hipStreamDestroy(own);
}

extern "C" {

void amm_opts_default(amm_opts* o) {
  if (!o) return;
  o->sparse_frac = 0.01;
  o->sparse_nnz = -1;
  o->oversample = 16;
  o->power_iters = 2;
  o->seed = 0;
  o->keep_residual = 1;
  o->spectral_fp16 = 0;
}

const char* amm_last_error(void) { return g_msg; }

amm_status amm_ctx_create(amm_ctx** ctx, int device) { return amm_ctx_create_with_allocator(ctx, device, nullptr); }

amm_status amm_ctx_create_with_allocator(amm_ctx** ctx, int device, const amm_allocator* alloc) {
  if (!ctx) return fail(AMM_EINVAL, "ctx is NULL");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(AMM_EINVAL, "allocator needs both functions");
  int count = 0;
  AMM_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(AMM_EINVAL, "device %d out of range (%d devices)", device, count);
  AMM_HIP(hipSetDevice(device));
  static_scratch_init(device);   // the fixed scratch's address on this device
  amm_ctx* c = new amm_ctx();
  c->device = device;
  if (alloc) c->alloc = AllocFns{alloc->alloc, alloc->free, alloc->user, device};
  {
    const char* e = std::getenv("AMM_DEBUG");
    c->debug = e && *e && std::strcmp(e, "0") != 0;
    const char* tc = std::getenv("AMM_TUNE_CACHE");
    if (tc) c->tune_cache = tc;
  }
  *ctx = c;
  return AMM_OK;
}

void amm_ctx_destroy(amm_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  delete ctx;
}

void amm_dec_destroy(amm_dec* dec) { delete dec; }

amm_status amm_ctx_set_timing(amm_ctx* ctx, int enable) {
  if (!ctx) return fail(AMM_EINVAL, "ctx is NULL");
  ctx->timing = enable != 0;
  return AMM_OK;
}

amm_status amm_ctx_timings(amm_ctx* ctx, char* names, int name_len, double* total_ms,
                           int64_t* launches, int cap, int* count) {
  if (!ctx || !count) return fail(AMM_EINVAL, "NULL argument");
  KernelTimer& t = ctx->timer;
  for (auto& p : t.pending) {
    float ms = 0.f;
    AMM_HIP(hipEventSynchronize(p.b));
    AMM_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    auto& acc = t.totals[p.name];
    acc.first += ms;
    acc.second += 1;
  }
  t.pending.clear();
  t.used = 0;   // every pooled event is resolved: reuse them
  *count = (int)t.totals.size();
  if (names || total_ms || launches) {
    if (cap < (int)t.totals.size()) return fail(AMM_EINVAL, "capacity %d < %d", cap, (int)t.totals.size());
    int i = 0;
    for (auto& kv : t.totals) {
      if (names && name_len > 0) {
        std::snprintf(names + (size_t)i * name_len, name_len, "%s", kv.first.c_str());
      }
      if (total_ms) total_ms[i] = kv.second.first;
      if (launches) launches[i] = kv.second.second;
      ++i;
    }
    t.totals.clear();
  }
  return AMM_OK;
}

amm_status amm_dec_query(const amm_dec* d, amm_dec_info* info) {
  if (!d || !info) return fail(AMM_EINVAL, "NULL argument");
  info->kind = d->kind;
  info->m = d->m;
  info->n = d->n;
  info->K = d->K;
  info->K_eff = d->K_eff;
  info->nnz = d->nnz;
  info->has_residual = (d->residual.ptr || d->A_borrowed ||
                        (d->inner && (d->inner->residual.ptr || d->inner->A_borrowed))) ? 1 : 0;
  info->blocks = (int)d->blocks.size();
  {
    const amm_dec* c = (d->inner ? d->inner : d);
    info->spectral_fp16 = (c->fp16 || (!c->blocks.empty() && c->blocks[0]->fp16)) ? 1 : 0;
  }
  info->norm_A = d->norm_A;
  info->norm_residual = d->norm_residual;
  {
    const amm_dec* c = (d->inner ? d->inner : d);
    info->mu = c->mu;
    info->sigma_next = c->sigma_next;
  }
  return AMM_OK;
}

amm_status amm_dec_block(const amm_dec* d, int j, const amm_dec** block) {
  if (!d || !block) return fail(AMM_EINVAL, "NULL argument");
  if (j < 0 || j >= (int)d->blocks.size()) return fail(AMM_EINVAL, "block %d out of [0, %d)", j, (int)d->blocks.size());
  *block = d->blocks[j];
  return AMM_OK;
}

amm_status amm_dec_frequencies(const amm_dec* d, int32_t* out_host, int cap, int* count) {
  if (!d || !count) return fail(AMM_EINVAL, "NULL argument");
  const amm_dec* c = is_sparse(d) ? d->inner : d;
  if (!c || !is_circ(c)) return fail(AMM_ESTATE, "not a circulant decomposition");
  *count = (int)c->freqs.size();
  if (out_host) {
    if (cap < (int)c->freqs.size()) return fail(AMM_EINVAL, "capacity %d < %d", cap, (int)c->freqs.size());
    std::memcpy(out_host, c->freqs.data(), c->freqs.size() * sizeof(int32_t));
  }
  return AMM_OK;
}

amm_status amm_dec_circulant_lists(const amm_dec* d, double* eig_host, int64_t cap) {
  if (!d || !eig_host) return fail(AMM_EINVAL, "NULL argument");
  const amm_dec* c = is_sparse(d) ? d->inner : d;
  if (!c || !is_circ(c)) return fail(AMM_ESTATE, "not a circulant decomposition");
  if (!c->blocks.empty()) return fail(AMM_EINVAL, "blocked circulant handle: read the lists of each block");
  const int64_t cnt = (int64_t)c->K_eff * c->n;
  if (cap < cnt) return fail(AMM_EINVAL, "capacity %lld < %lld", (long long)cap, (long long)cnt);
  if (cnt == 0) return AMM_OK;
  std::vector<float2> L((size_t)cnt);
  AMM_HIP(hipMemcpy(L.data(), c->L.ptr, cnt * sizeof(float2), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < cnt; ++i) {
    eig_host[2 * i] = L[i].x;
    eig_host[2 * i + 1] = L[i].y;
  }
  return AMM_OK;
}

amm_status amm_dec_energies(const amm_dec* d, double* out_host, int64_t cap) {
  if (!d || !out_host) return fail(AMM_EINVAL, "NULL argument");
  const amm_dec* c = is_sparse(d) ? d->inner : d;
  if (!c || !c->has_energies) return fail(AMM_ESTATE, "no energies stored");
  if (cap < c->n) return fail(AMM_EINVAL, "capacity too small");
  AMM_HIP(hipMemcpy(out_host, c->energies.ptr, c->n * sizeof(double), hipMemcpyDeviceToHost));
  return AMM_OK;
}

amm_status amm_dec_tsvd_factors(const amm_dec* d, float* U_host, float* sigma_host, float* V_host) {
  if (!d) return fail(AMM_EINVAL, "NULL argument");
  const amm_dec* c = is_sparse(d) ? d->inner : d;
  if (!c || !is_tsvd(c)) return fail(AMM_ESTATE, "not an SVD decomposition");
  const int k = c->K_eff;
  if (U_host) AMM_HIP(hipMemcpy(U_host, c->U.ptr, c->m * k * sizeof(float), hipMemcpyDeviceToHost));
  if (sigma_host) AMM_HIP(hipMemcpy(sigma_host, c->sigma.ptr, k * sizeof(float), hipMemcpyDeviceToHost));
  if (V_host) AMM_HIP(hipMemcpy(V_host, c->V.ptr, c->n * k * sizeof(float), hipMemcpyDeviceToHost));
  return AMM_OK;
}

amm_status amm_dec_sparse_part(const amm_dec* d, int32_t* row_ptr_host, int32_t* col_host, float* val_host) {
  if (!d || !is_sparse(d)) return fail(AMM_ESTATE, "not a sparse decomposition");
  if (row_ptr_host) AMM_HIP(hipMemcpy(row_ptr_host, d->row_ptr.ptr, (d->m + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (d->nnz > 0) {
    if (col_host) AMM_HIP(hipMemcpy(col_host, d->col.ptr, d->nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (val_host) AMM_HIP(hipMemcpy(val_host, d->val.ptr, d->nnz * sizeof(float), hipMemcpyDeviceToHost));
  }
  return AMM_OK;
}

}  // extern "C"

namespace amm {

// Pair structure of a closed frequency set (see CdPairs), for the lists L
// (shifts k_t) and for the adjoint lists Ladj_t[p] = conj(L_t[p + k_t])
// (shifts -k_t).  Left unset (plain loop) when the set is not closed or the
// lists are not those of a real operator to float32 rounding: `mirror(pass,
// ta, tb)` tells whether list tb of the pass (0: L, 1: Ladj) is the mirrored
// conjugate of list ta, L_b[p] = conj(L_a[-p]) to the tolerance.
amm_status cd_pair_tables(amm_dec* d, const std::function<bool(int, int, int)>& mirror) {
  d->npairs = d->npairs_adj = -1;
  d->nsingles = d->nsingles_adj = 0;
  const int64_t n = d->n;
  const int K = d->K_eff;
  if (K == 0) return AMM_OK;
  std::map<int64_t, int> idx;
  for (int t = 0; t < K; ++t) idx[d->freqs[t]] = t;
  for (int t = 0; t < K; ++t)
    if (!idx.count((n - d->freqs[t]) % n)) return AMM_OK;
  std::vector<int64_t> ka(K);
  for (int t = 0; t < K; ++t) ka[t] = d->freqs[t] == 0 ? 0 : n - d->freqs[t];
  std::vector<int2> pairs, singles, pairs_a, singles_a;
  for (int pass = 0; pass < 2; ++pass) {
    auto& P = pass == 0 ? pairs : pairs_a;
    auto& S = pass == 0 ? singles : singles_a;
    std::map<int64_t, int> at;
    for (int t = 0; t < K; ++t) at[pass == 0 ? (int64_t)d->freqs[t] : ka[t]] = t;
    for (const auto& kv : at) {
      const int64_t k = kv.first, kk = (n - k) % n;
      const int t = kv.second, tt = at[kk];
      if (k == kk) {
        if (!mirror(pass, t, t)) return AMM_OK;
        S.push_back(int2{(int)k, t});
      } else if (k < kk) {
        if (!mirror(pass, t, tt)) return AMM_OK;
        P.push_back(int2{(int)k, t});
      }
    }
  }
  std::vector<int2> all;
  all.insert(all.end(), pairs.begin(), pairs.end());
  all.insert(all.end(), singles.begin(), singles.end());
  all.insert(all.end(), pairs_a.begin(), pairs_a.end());
  all.insert(all.end(), singles_a.begin(), singles_a.end());
  AMM_TRY(d->pair_buf.alloc(all.size() * sizeof(int2)));
  AMM_HIP(hipMemcpy(d->pair_buf.ptr, all.data(), all.size() * sizeof(int2), hipMemcpyHostToDevice));
  d->npairs = (int)pairs.size();
  d->nsingles = (int)singles.size();
  d->npairs_adj = (int)pairs_a.size();
  d->nsingles_adj = (int)singles_a.size();
  return AMM_OK;
}

// The same with the mirror test on host copies of the lists (imported
// eigenvalues).
amm_status cd_build_pairs(amm_dec* d, const std::vector<float2>& Lh) {
  const int64_t n = d->n;
  const int K = d->K_eff;
  if (K == 0 || (int64_t)Lh.size() < (int64_t)K * n) {
    d->npairs = d->npairs_adj = -1;
    d->nsingles = d->nsingles_adj = 0;
    return AMM_OK;
  }
  float mx = 0.f;
  for (const float2& v : Lh) mx = std::max(mx, std::max(std::fabs(v.x), std::fabs(v.y)));
  const float tol = 1e-5f * mx + 1e-30f;
  // adjoint lists on the host: La_t[p] = conj(L_t[(p + k) mod n]) (the index
  // wraps once, so the two ranges run without a modulo)
  std::vector<float2> La((size_t)K * n);
  for (int t = 0; t < K; ++t) {
    const int64_t k = d->freqs[t];
    const float2* src = Lh.data() + (size_t)t * n;
    float2* dst = La.data() + (size_t)t * n;
    for (int64_t p = 0; p < n - k; ++p) dst[p] = float2{src[p + k].x, -src[p + k].y};
    for (int64_t p = n - k; p < n; ++p) dst[p] = float2{src[p + k - n].x, -src[p + k - n].y};
  }
  // L_b[p] == conj(L_a[-p]) for every p (index -p is 0 at p = 0, else n - p)
  auto mirror = [&](int pass, int ta, int tb) {
    const std::vector<float2>& Ls = pass == 0 ? Lh : La;
    const float2* la = Ls.data() + (size_t)ta * n;
    const float2* lb = Ls.data() + (size_t)tb * n;
    if (std::fabs(lb[0].x - la[0].x) > tol || std::fabs(lb[0].y + la[0].y) > tol) return false;
    bool ok = true;
    for (int64_t p = 1; p < n; ++p) {
      const float2 a = la[n - p], b = lb[p];
      ok &= !(std::fabs(b.x - a.x) > tol || std::fabs(b.y + a.y) > tol);
    }
    return ok;
  };
  return cd_pair_tables(d, mirror);
}

}  // namespace amm

extern "C" {

amm_status amm_dec_import_circulant(amm_ctx* ctx, int64_t n, int K, const int32_t* freqs,
                                    const double* eig, const float* residual, double norm_A,
                                    double norm_residual, amm_dec** out) {
  TimerScope ts(ctx);
  if (!ctx || !out) return fail(AMM_EINVAL, "NULL argument");
  if (!circ_side_ok(n)) return fail(AMM_EUNSUPPORTED, "circulant path needs n in [2, 16384], got %lld", (long long)n);
  if (K < 0 || K > n) return fail(AMM_EINVAL, "K = %d out of [0, n]", K);
  if (K > 0 && (!freqs || !eig)) return fail(AMM_EINVAL, "NULL frequencies or eigenvalues");
  for (int t = 0; t < K; ++t)
    if (freqs[t] < 0 || freqs[t] >= n) return fail(AMM_EINVAL, "frequency %d out of range", freqs[t]);
  AMM_HIP(hipSetDevice(ctx->device));
  amm_dec* d = new amm_dec();
  d->kind = AMM_CIRCULANT;
  d->m = d->n = n;
  d->K = d->K_eff = K;
  d->device = ctx->device;
  d->norm_A = norm_A;
  d->norm_residual = norm_residual;
  d->freqs.assign(freqs, freqs + K);
  std::vector<float2> L((size_t)std::max(K, 1) * n), La((size_t)std::max(K, 1) * n);
  std::vector<int32_t> sh(std::max(K, 1)), sa(std::max(K, 1));
  for (int t = 0; t < K; ++t) {
    const int64_t k = freqs[t];
    sh[t] = (int32_t)k;
    sa[t] = (int32_t)((n - k) % n);
    for (int64_t p = 0; p < n; ++p) {
      const double* e = eig + 2 * ((int64_t)t * n + p);
      L[(size_t)t * n + p] = float2{(float)e[0], (float)e[1]};
      const double* f = eig + 2 * ((int64_t)t * n + ((p + k) % n));
      La[(size_t)t * n + p] = float2{(float)f[0], (float)-f[1]};
    }
  }
  amm_status st;
  if ((st = d->L.alloc(L.size() * sizeof(float2))) != AMM_OK ||
      (st = d->Ladj.alloc(La.size() * sizeof(float2))) != AMM_OK ||
      (st = d->shifts.alloc(sh.size() * sizeof(int32_t))) != AMM_OK ||
      (st = d->shifts_adj.alloc(sa.size() * sizeof(int32_t))) != AMM_OK) {
    delete d;
    return st;
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(d->L.ptr, L.data(), L.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d->Ladj.ptr, La.data(), La.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d->shifts.ptr, sh.data(), sh.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d->shifts_adj.ptr, sa.data(), sa.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    L.resize((size_t)K * n);
    if ((st = cd_build_pairs(d, L)) != AMM_OK) {
      delete d;
      return st;
    }
  }
  if (e == hipSuccess && residual) {
    if ((st = d->residual.alloc(n * n * sizeof(float))) != AMM_OK) { delete d; return st; }
    e = hipMemcpy(d->residual.ptr, residual, n * n * sizeof(float), hipMemcpyDeviceToDevice);
  }
  if (e != hipSuccess) {
    delete d;
    return hip_fail(e, "import circulant");
  }
  *out = d;
  return AMM_OK;
}

amm_status amm_dec_import_tsvd(amm_ctx* ctx, int64_t m, int64_t n, int k, const double* U,
                               const double* sigma, const double* V, const float* A, amm_dec** out) {
  TimerScope ts(ctx);
  if (!ctx || !out) return fail(AMM_EINVAL, "NULL argument");
  if (m <= 0 || n <= 0 || k < 0 || k > std::min(m, n)) return fail(AMM_ESHAPE, "bad SVD shape m=%lld n=%lld k=%d", (long long)m, (long long)n, k);
  if (k > 0 && (!U || !sigma || !V)) return fail(AMM_EINVAL, "NULL factor");
  AMM_HIP(hipSetDevice(ctx->device));
  amm_dec* d = new amm_dec();
  d->kind = AMM_TSVD;
  d->m = m;
  d->n = n;
  d->K = d->K_eff = k;
  d->device = ctx->device;
  d->A_borrowed = A;
  const int64_t kk = std::max(k, 1);
  std::vector<float> hU(m * kk, 0.f), hUS(m * kk, 0.f), hV(n * kk, 0.f), hVS(n * kk, 0.f), hs(kk, 0.f);
  double s2 = 0.0;
  for (int j = 0; j < k; ++j) { hs[j] = (float)sigma[j]; s2 += sigma[j] * sigma[j]; }
  d->sigma64.assign(sigma, sigma + k);
  for (int64_t i = 0; i < m; ++i)
    for (int j = 0; j < k; ++j) {
      hU[i * k + j] = (float)U[i * k + j];
      hUS[i * k + j] = (float)(U[i * k + j] * sigma[j]);
    }
  for (int64_t i = 0; i < n; ++i)
    for (int j = 0; j < k; ++j) {
      hV[i * k + j] = (float)V[i * k + j];
      hVS[i * k + j] = (float)(V[i * k + j] * sigma[j]);
    }
  amm_status st;
  std::vector<float> hVSt(n * kk, 0.f), hVt(n * kk, 0.f);
  for (int64_t i = 0; i < n; ++i)
    for (int j = 0; j < k; ++j) {
      hVSt[(int64_t)j * n + i] = hVS[i * k + j];
      hVt[(int64_t)j * n + i] = hV[i * k + j];
    }
  if ((st = d->U.alloc(hU.size() * 4)) != AMM_OK || (st = d->US.alloc(hUS.size() * 4)) != AMM_OK ||
      (st = d->V.alloc(hV.size() * 4)) != AMM_OK || (st = d->VS.alloc(hVS.size() * 4)) != AMM_OK ||
      (st = d->VSt.alloc(hVSt.size() * 4)) != AMM_OK || (st = d->Vt.alloc(hVt.size() * 4)) != AMM_OK ||
      (st = d->sigma.alloc(hs.size() * 4)) != AMM_OK) {
    delete d;
    return st;
  }
  hipError_t e = hipMemcpy(d->U.ptr, hU.data(), hU.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d->US.ptr, hUS.data(), hUS.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d->V.ptr, hV.data(), hV.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d->VS.ptr, hVS.data(), hVS.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d->VSt.ptr, hVSt.data(), hVSt.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d->Vt.ptr, hVt.data(), hVt.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d->sigma.ptr, hs.data(), hs.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    delete d;
    return hip_fail(e, "import tsvd");
  }
  // norms for the error estimates: known only with A
  d->norm_A = NAN;
  d->norm_residual = NAN;
  (void)s2;
  if (A) {
    amm_status st2 = d->residual.alloc(m * n * sizeof(float));
    if (st2 == AMM_OK) st2 = tsvd_residual(A, m, n, k, d->US.as<float>(), d->V.as<float>(), d->residual.as<float>(), 0);
    if (st2 == AMM_OK && hipDeviceSynchronize() != hipSuccess) st2 = fail(AMM_EDEVICE, "residual");
    double a2 = 0.0, r2 = 0.0;
    if (st2 == AMM_OK) st2 = sumsq_f32(A, m * n, 0, &a2);
    if (st2 == AMM_OK) st2 = sumsq_f32(d->residual.as<float>(), m * n, 0, &r2);
    if (st2 != AMM_OK) {
      delete d;
      return st2;
    }
    d->norm_A = std::sqrt(a2);
    d->norm_residual = std::sqrt(r2);
  }
  *out = d;
  return AMM_OK;
}

amm_status amm_dec_import_sparse(amm_ctx* ctx, int64_t m, int64_t n, int64_t nnz,
                                 const int32_t* row_ptr, const int32_t* col, const float* val,
                                 amm_dec* residue, const float* A, amm_dec** out) {
  TimerScope ts(ctx);
  if (!ctx || !out) return fail(AMM_EINVAL, "NULL argument");
  if (m <= 0 || n <= 0 || nnz < 0 || nnz > m * n) return fail(AMM_ESHAPE, "bad sparse shape");
  if (!row_ptr || (nnz > 0 && (!col || !val))) return fail(AMM_EINVAL, "NULL CSR array");
  if (row_ptr[0] != 0 || row_ptr[m] != nnz) return fail(AMM_EINVAL, "row_ptr does not span [0, nnz]");
  for (int64_t i = 0; i < m; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return fail(AMM_EINVAL, "row_ptr not monotone");
  for (int64_t e = 0; e < nnz; ++e)
    if (col[e] < 0 || col[e] >= n) return fail(AMM_EINVAL, "column index out of range");
  if (residue && (residue->m != m || residue->n != n)) return fail(AMM_ESHAPE, "residue shape differs");
  AMM_HIP(hipSetDevice(ctx->device));
  amm_dec* d = new amm_dec();
  d->kind = AMM_SPARSE | (residue ? residue->kind : 0);
  d->m = m;
  d->n = n;
  d->nnz = nnz;
  d->device = ctx->device;
  d->A_borrowed = A;
  amm_status st;
  if ((st = d->row_ptr.alloc((m + 1) * 4)) != AMM_OK || (st = d->col.alloc(std::max<int64_t>(nnz, 1) * 4)) != AMM_OK ||
      (st = d->val.alloc(std::max<int64_t>(nnz, 1) * 4)) != AMM_OK) {
    delete d;
    return st;
  }
  hipError_t e = hipMemcpy(d->row_ptr.ptr, row_ptr, (m + 1) * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && nnz) e = hipMemcpy(d->col.ptr, col, nnz * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && nnz) e = hipMemcpy(d->val.ptr, val, nnz * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    delete d;
    return hip_fail(e, "import sparse");
  }
  if ((st = build_csc(d, nullptr)) != AMM_OK) {
    delete d;
    return st;
  }
  d->inner = residue;
  if (residue) d->K = d->K_eff = residue->K_eff;
  d->norm_A = d->norm_residual = NAN;   // not known from the parts
  *out = d;
  return AMM_OK;
}

static amm_status decompose_body(amm_ctx* ctx, const float* A, int64_t m, int64_t n, int kind, int K,
                         const amm_opts* opts, void* stream, amm_dec** out) {
  if (!ctx || !A || !out) return fail(AMM_EINVAL, "NULL argument");
  if (m <= 0 || n <= 0) return fail(AMM_ESHAPE, "empty operand");
  amm_opts o;
  amm_opts_default(&o);
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  TimerScope ts(ctx);
  AMM_HIP(hipSetDevice(ctx->device));
  const int base = kind & ~AMM_SPARSE;
  if (kind & AMM_SPARSE) {
    if (base != 0 && base != AMM_CIRCULANT && base != AMM_TSVD) return fail(AMM_EINVAL, "bad kind %d", kind);
    int64_t nnz = o.sparse_nnz >= 0 ? o.sparse_nnz : (int64_t)llround(o.sparse_frac * (double)m * (double)n);
    if (nnz < 0 || nnz > m * n) return fail(AMM_EINVAL, "sparse count %lld out of range", (long long)nnz);
    amm_dec* d = new amm_dec();
    d->kind = kind;
    d->m = m;
    d->n = n;
    d->K = K;
    d->device = ctx->device;
    DevBuf R;
    amm_status st = R.alloc(m * n * sizeof(float));
    if (st == AMM_OK) st = sparse_extract(ctx, A, m, n, nnz, d, R.as<float>(), s);
    // ||A||_F, and ||Delta A||_F = ||R||_F without an inner truncation
    double a2 = 0.0, r2 = 0.0;
    if (st == AMM_OK) st = sumsq_f32(A, m * n, s, &a2);
    if (st == AMM_OK && base == 0) st = sumsq_f32(R.as<float>(), m * n, s, &r2);
    d->norm_A = std::sqrt(a2);
    d->norm_residual = std::sqrt(r2);
    if (st == AMM_OK && base != 0) {
      amm_dec* in = nullptr;
      st = amm_decompose(ctx, R.as<float>(), m, n, base, K, &o, stream, &in);
      if (st == AMM_OK) {
        d->inner = in;
        d->K_eff = in->K_eff;
        d->norm_residual = in->norm_residual;   // Delta A = R - trunc(R)
        // R is a temporary: the inner handle keeps its own Delta R, never R
        in->A_borrowed = nullptr;
      }
    } else if (st == AMM_OK && o.keep_residual) {
      d->residual = std::move(R);
    }
    if (st == AMM_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(AMM_EDEVICE, "sync");
    if (st != AMM_OK) {
      delete d;
      return st;
    }
    *out = d;
    return AMM_OK;
  }
  if (kind == AMM_CIRCULANT && m != n) {
    // square blocks of side s = min(m, n) along the longer dimension
    const int64_t sd = std::min(m, n), lg = std::max(m, n);
    if (!circ_side_ok(sd)) return fail(AMM_EUNSUPPORTED, "circulant blocks need min(m, n) in [2, 16384]");
    if (K < 0 || K > sd) return fail(AMM_EINVAL, "K = %d out of [0, %lld]", K, (long long)sd);
    const int nb = (int)((lg + sd - 1) / sd);
    amm_dec* d = new amm_dec();
    d->kind = AMM_CIRCULANT;
    d->m = m;
    d->n = n;
    d->K = K;
    d->device = ctx->device;
    d->block_rows = m > n;
    DevBuf blk;
    amm_status st = blk.alloc((size_t)sd * sd * sizeof(float));
    amm_opts ob = o;
    ob.keep_residual = 0;
    double a2 = 0.0, r2 = 0.0;
    for (int j = 0; j < nb && st == AMM_OK; ++j) {
      const int64_t lo = (int64_t)j * sd, valid = std::min(sd, lg - lo);
      float* bp = blk.as<float>();
      if (valid < sd) st = fill_f32(bp, sd * sd, 0.f, s);
      if (st != AMM_OK) break;
      hipError_t e;
      if (d->block_rows)   // rows lo..lo+valid of A (n columns)
        e = hipMemcpy2DAsync(bp, sd * sizeof(float), A + lo * n, n * sizeof(float), sd * sizeof(float), valid,
                             hipMemcpyDeviceToDevice, s);
      else                 // columns lo..lo+valid of A (m rows)
        e = hipMemcpy2DAsync(bp, sd * sizeof(float), A + lo, n * sizeof(float), valid * sizeof(float), sd,
                             hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) { st = hip_fail(e, "hipMemcpy2DAsync"); break; }
      amm_dec* b = new amm_dec();
      b->kind = AMM_CIRCULANT;
      b->m = b->n = sd;
      b->K = K;
      b->device = ctx->device;
      st = cd_decompose(ctx, bp, (int)sd, K, false, b, s, o.spectral_fp16 != 0);
      if (st != AMM_OK) { delete b; break; }
      d->blocks.push_back(b);
      d->K_eff += b->K_eff;
      a2 += b->norm_A * b->norm_A;
      r2 += b->norm_residual * b->norm_residual;
    }
    if (st != AMM_OK) {
      delete d;
      return st;
    }
    d->norm_A = std::sqrt(a2);
    d->norm_residual = std::sqrt(r2);
    *out = d;
    return AMM_OK;
  }
  if (kind == AMM_SFFT) {
    amm_dec* d = new amm_dec();
    d->kind = AMM_SFFT;
    d->m = m;
    d->n = n;
    d->K = K;
    d->device = ctx->device;
    amm_status st = sfft_decompose(ctx, A, m, n, K, o.keep_residual != 0, d, s);
    if (st != AMM_OK) {
      delete d;
      return st;
    }
    d->K_eff = K;
    *out = d;
    return AMM_OK;
  }
  if (kind == AMM_CIRCULANT) {
    if (!circ_side_ok(n)) return fail(AMM_EUNSUPPORTED, "circulant path needs n in [2, 16384]");
    if (K < 0 || K > n) return fail(AMM_EINVAL, "K = %d out of [0, n]", K);
    amm_dec* d = new amm_dec();
    d->kind = AMM_CIRCULANT;
    d->m = d->n = n;
    d->K = K;
    d->device = ctx->device;
    amm_status st = cd_decompose(ctx, A, (int)n, K, o.keep_residual != 0, d, s, o.spectral_fp16 != 0);
    if (st != AMM_OK) {
      delete d;
      return st;
    }
    *out = d;
    return AMM_OK;
  }
  if (kind == AMM_TSVD) {
    if (K < 0 || K > std::min(m, n)) return fail(AMM_EINVAL, "rank %d out of range", K);
    amm_dec* d = new amm_dec();
    d->kind = AMM_TSVD;
    d->m = m;
    d->n = n;
    d->K = K;
    d->device = ctx->device;
    amm_status st = tsvd_decompose(ctx, A, m, n, K, &o, d, s);
    if (st == AMM_OK && o.keep_residual) {
      st = d->residual.alloc(m * n * sizeof(float));
      if (st == AMM_OK) st = tsvd_residual(A, m, n, d->K_eff, d->US.as<float>(), d->V.as<float>(), d->residual.as<float>(), s);
      if (st == AMM_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(AMM_EDEVICE, "residual");
    }
    if (st != AMM_OK) {
      delete d;
      return st;
    }
    if (o.keep_residual) d->A_borrowed = A;
    *out = d;
    return AMM_OK;
  }
  return fail(AMM_EINVAL, "bad kind %d", kind);
}

static amm_status matmul_body(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, const float* B,
                             int64_t n, int64_t p, float* out, void* stream) {
  if (!ctx || !dA) return fail(AMM_EINVAL, "NULL argument");
  if (n != dA->n) return fail(AMM_ESHAPE, "B has %lld rows, A has %lld columns", (long long)n, (long long)dA->n);
  if (p < 0) return fail(AMM_ESHAPE, "negative column count");
  if (p == 0) return AMM_OK;   // empty product: nothing to write
  if (!B || !out) return fail(AMM_EINVAL, "NULL argument");
  if (dB && (dB->m != n || dB->n != p)) return fail(AMM_ESHAPE, "dB describes a %lldx%lld operand, B is %lldx%lld",
                                                    (long long)dB->m, (long long)dB->n, (long long)n, (long long)p);
  if (B == out) return fail(AMM_EINVAL, "out aliases B");
  hipStream_t s = (hipStream_t)stream;
  AMM_HIP(hipSetDevice(ctx->device));
  if (dB && (!dA->blocks.empty() || !dB->blocks.empty() || (dA->inner && !dA->inner->blocks.empty()) ||
             (dB->inner && !dB->inner->blocks.empty())))
    return fail(AMM_EUNSUPPORTED, "first-order products of blocked circulant operands are not supported");
  if (dB && (is_sfft(dA) || is_sfft(dB))) {
    if (!(is_sfft(dA) && is_sfft(dB)))
      return fail(AMM_EUNSUPPORTED, "first order with Fourier sparsification needs it on both operands");
    if (!dA->sf_left || !dA->sf_Rt.ptr)
      return fail(AMM_ESTATE, "left operand keeps no spectral residual (n a power of two, keep_residual)");
    if (!dB->sf_right) return fail(AMM_EUNSUPPORTED, "right operand has no column sparsification");
    if (p % 2) return fail(AMM_EUNSUPPORTED, "Fourier-sparsified products need an even column count");
    TimerScope ts(ctx);
    AMM_TRY(left_apply(ctx, dA, B, p, out, false, s));
    return sfft_first_order_term(ctx, dA, dB, out, s);
  }
  if (dB) {
    // validate the residual source before any launch
    if (!(is_tsvd(dA) && is_tsvd(dB) && dA->A_borrowed)) {
      bool ok = dA->residual.ptr || (is_tsvd(dA) && dA->A_borrowed) ||
                (is_sparse(dA) && dA->inner && (dA->inner->residual.ptr || dA->inner->A_borrowed));
      if (!ok) return fail(AMM_ESTATE, "left operand keeps no Delta A (decompose with keep_residual or pass A)");
    }
  }
  TimerScope ts(ctx);
  if (!dB) return left_apply(ctx, dA, B, p, out, false, s);
  if (is_tsvd(dA) && is_tsvd(dB) && dA->A_borrowed && dB->residual.ptr &&
      tsvd_split_shapes(dA->m, n, p, dA->K_eff, dB->K_eff)) {
    // M1 = U_A S_A (V_A^T Delta B) + (A U_B)(S_B V_B^T): panels, reduce, split output GEMM
    const size_t need = tsvd_split_scratch(dA->m, n, p, dA->K_eff, dB->K_eff);
    AMM_TRY(ctx->scratch[4].reserve(need * sizeof(float)));
    return tsvd_split_product(dA->m, n, p, dA->K_eff, dB->K_eff, dA->V.as<float>(), dA->US.as<float>(),
                              dB->residual.as<float>(), dA->A_borrowed, dB->U.as<float>(), dB->VS.as<float>(),
                              ctx->scratch[4].as<float>(), need, out, s);
  }
  if (is_tsvd(dA) && is_tsvd(dB) && dA->A_borrowed && dB->residual.ptr &&
      tsvd_fast_shapes(dA->m, n, p, dA->K_eff, dB->K_eff)) {
    // M1 = U_A S_A (V_A^T Delta B) + (A U_B)(S_B V_B^T): two panels, one output GEMM
    const int ka = dA->K_eff, kb = dB->K_eff;
    const int64_t m = dA->m;
    const size_t gp = (size_t)4 * std::max(ka, 1) * p, hp = (size_t)4 * std::max(kb, 1) * m;
    AMM_TRY(ctx->scratch[4].reserve(gp * sizeof(float)));
    AMM_TRY(ctx->scratch[5].reserve(hp * sizeof(float)));
    return tsvd_fast_product(m, n, p, ka, kb, dA->V.as<float>(), dA->US.as<float>(), dB->residual.as<float>(),
                             dA->A_borrowed, dB->U.as<float>(), dB->VSt.as<float>(), ctx->scratch[4].as<float>(),
                             gp, ctx->scratch[5].as<float>(), hp, out, s);
  }
  if (is_tsvd(dA) && is_tsvd(dB) && dA->A_borrowed) {
    // M1 = U_A S_A (V_A^T B) + (A U_B - U_A S_A (V_A^T U_B)) S_B V_B^T
    //    = [U_A S_A | H] [V_A^T B ; S_B V_B^T]   -- one output GEMM, no Delta A
    const int ka = dA->K_eff, kb = dB->K_eff, kc = ka + kb;
    const int64_t m = dA->m;
    if (kc == 0) return fill_f32(out, m * p, 0.f, s);
    AMM_TRY(ctx->scratch[0].reserve((size_t)kc * p * sizeof(float)));
    AMM_TRY(ctx->scratch[1].reserve((size_t)m * kc * sizeof(float)));
    AMM_TRY(ctx->scratch[3].reserve((size_t)std::max(ka, 1) * std::max(kb, 1) * sizeof(float)));
    float* Gc = ctx->scratch[0].as<float>();   // kc x p
    float* Uc = ctx->scratch[1].as<float>();   // m x kc
    float* Sm = ctx->scratch[3].as<float>();   // ka x kb
    if (ka > 0) {
      AMM_TRY(gemm_f32(ka, p, n, 1.f, MatView{dA->V.as<float>(), 1, ka}, MatView{B, p, 1}, 0.f, Gc, p, s, "gemm_VtB"));
      AMM_HIP(hipMemcpy2DAsync(Uc, kc * sizeof(float), dA->US.ptr, ka * sizeof(float), ka * sizeof(float), m,
                               hipMemcpyDeviceToDevice, s));
    }
    if (kb > 0) {
      AMM_HIP(hipMemcpyAsync(Gc + (int64_t)ka * p, dB->VSt.ptr, (size_t)kb * p * sizeof(float),
                             hipMemcpyDeviceToDevice, s));
      AMM_TRY(gemm_f32(m, kb, n, 1.f, MatView{dA->A_borrowed, n, 1}, MatView{dB->U.as<float>(), kb, 1}, 0.f,
                       Uc + ka, kc, s, "gemm_AU"));
      if (ka > 0) {
        AMM_TRY(gemm_f32(ka, kb, n, 1.f, MatView{dA->V.as<float>(), 1, ka}, MatView{dB->U.as<float>(), kb, 1}, 0.f,
                         Sm, kb, s, "gemm_small"));
        AMM_TRY(gemm_f32(m, kb, ka, -1.f, MatView{dA->US.as<float>(), ka, 1}, MatView{Sm, kb, 1}, 1.f, Uc + ka, kc,
                         s, "gemm_small"));
      }
    }
    return gemm_f32(m, p, kc, 1.f, MatView{Uc, kc, 1}, MatView{Gc, p, 1}, 0.f, out, p, s, "gemm_out");
  }
  AMM_TRY(left_apply(ctx, dA, B, p, out, false, s));
  const float* dAres = nullptr;
  AMM_TRY(residual_of(ctx, dA, &dAres, s));
  return right_apply(ctx, dAres, dA->m, dB, out, true, s);
}

static amm_status strided_body(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, const float* B,
                                     int64_t n, int64_t p, int64_t ldb, float* out, int64_t ldo, void* stream) {
  if (!ctx || !dA) return fail(AMM_EINVAL, "NULL argument");
  if (ldb < p || ldo < p) return fail(AMM_ESHAPE, "row pitches %lld, %lld below %lld columns", (long long)ldb,
                                      (long long)ldo, (long long)p);
  if (ldb == p && ldo == p) return amm_approx_matmul(ctx, dA, dB, B, n, p, out, stream);
  if (n != dA->n) return fail(AMM_ESHAPE, "B has %lld rows, A has %lld columns", (long long)n, (long long)dA->n);
  if (p == 0) return AMM_OK;
  if (!B || !out) return fail(AMM_EINVAL, "NULL argument");
  const int64_t m = dA->m;
  if (panels_overlap(B, n, ldb, out, m, ldo, p)) return fail(AMM_EINVAL, "out overlaps B");
  hipStream_t s = (hipStream_t)stream;
  AMM_HIP(hipSetDevice(ctx->device));
  TimerScope ts(ctx);
  const amm_dec* in = dA->inner;
  const bool f4 = ((uintptr_t)B % 16) == 0 && ((uintptr_t)out % 16) == 0 && ldb % 4 == 0 && ldo % 4 == 0 && p % 4 == 0;
  if (!dB && dA->blocks.empty() && is_circ(dA) && is_pow2(dA->n))
    return circ_columns(ctx, dA, B, p, out, false, s, ldb, ldo);   // the product reads and writes at the pitches
  if (!dB && dA->blocks.empty() && is_sparse(dA) && dA->nnz > 0 && f4 && in && is_circ(in) && in->blocks.empty() &&
      is_pow2(in->n) && in->K_eff > 0) {
    // B to a spread pitch (from ldb), the residue's product there, S B + it written at ldo
    const int64_t sp = spread_pitch(p);
    AMM_TRY(ctx->scratch[14].reserve((size_t)n * sp * sizeof(float)));
    AMM_TRY(ctx->scratch[15].reserve((size_t)m * sp * sizeof(float)));
    float* Bs = ctx->scratch[14].as<float>();
    float* Y = ctx->scratch[15].as<float>();
    AMM_TRY(repitch_f32(B, ldb, n, p, Bs, sp, s));
    AMM_TRY(cd_apply_columns(ctx, log2_exact(in->n), in->K_eff, in->shifts.as<int32_t>(), in->L.as<float2>(), Bs, p, Y,
                             false, s, in->pairs_of(false), in->lists16(false), in->l16_inv, sp, sp));
    return spmm_csr(dA, Bs, sp, p, out, false, s, Y, sp, ldo);
  }
  // other kinds: packed copies in and out around the contiguous product
  const float* Bp = B;
  if (ldb != p) {
    AMM_TRY(ctx->scratch[16].reserve((size_t)n * p * sizeof(float)));
    AMM_HIP(hipMemcpy2DAsync(ctx->scratch[16].ptr, p * sizeof(float), B, ldb * sizeof(float), p * sizeof(float), n,
                             hipMemcpyDeviceToDevice, s));
    Bp = ctx->scratch[16].as<float>();
  }
  float* Op = out;
  if (ldo != p) {
    AMM_TRY(ctx->scratch[17].reserve((size_t)m * p * sizeof(float)));
    Op = ctx->scratch[17].as<float>();
  }
  AMM_TRY(amm_approx_matmul(ctx, dA, dB, Bp, n, p, Op, stream));
  if (ldo != p)
    AMM_HIP(hipMemcpy2DAsync(out, ldo * sizeof(float), Op, p * sizeof(float), p * sizeof(float), m,
                             hipMemcpyDeviceToDevice, s));
  return AMM_OK;
}

}  // extern "C"

namespace {
bool dtype_ok(int t) { return t == AMM_F32 || t == AMM_BF16 || t == AMM_F16; }
size_t dtype_size(int t) { return t == AMM_F32 ? 4 : 2; }

amm_status check_matrix(const amm_matrix* M, const char* name, int64_t rows, int64_t cols) {
  if (!M) return fail(AMM_EINVAL, "%s is NULL", name);
  if (!dtype_ok(M->dtype)) return fail(AMM_EINVAL, "%s: unknown element type %d", name, M->dtype);
  if (M->rows != rows || M->cols != cols)
    return fail(AMM_ESHAPE, "%s is %lldx%lld, expected %lldx%lld", name, (long long)M->rows, (long long)M->cols,
                (long long)rows, (long long)cols);
  if (M->ld < cols) return fail(AMM_ESHAPE, "%s: pitch %lld below %lld columns", name, (long long)M->ld, (long long)cols);
  if (rows > 0 && cols > 0 && !M->data) return fail(AMM_EINVAL, "%s has no data", name);
  return AMM_OK;
}

// byte ranges of two described matrices meet
bool matrices_overlap(const amm_matrix* a, const amm_matrix* b) {
  if (!a || !b || a->rows == 0 || a->cols == 0 || b->rows == 0 || b->cols == 0) return false;
  const uintptr_t a0 = (uintptr_t)a->data, a1 = a0 + (uintptr_t)((a->rows - 1) * a->ld + a->cols) * dtype_size(a->dtype);
  const uintptr_t b0 = (uintptr_t)b->data, b1 = b0 + (uintptr_t)((b->rows - 1) * b->ld + b->cols) * dtype_size(b->dtype);
  return a0 < b1 && b0 < a1;
}

// A float32 packed view of M: M itself when it already is one, else a
// widened copy in `buf`.
amm_status packed_input(const amm_matrix* M, DevBuf& buf, const float** out, hipStream_t s) {
  if (M->dtype == AMM_F32 && M->ld == M->cols) {
    *out = static_cast<const float*>(M->data);
    return AMM_OK;
  }
  AMM_TRY(buf.reserve((size_t)M->rows * M->cols * sizeof(float)));
  AMM_TRY(cast_matrix(M->data, M->dtype, M->ld, M->rows, M->cols, buf.ptr, AMM_F32, M->cols, s));
  *out = buf.as<float>();
  return AMM_OK;
}

// Where a float32 result for M is written: M itself when packed float32,
// else `buf` (copied out by finish_output).
amm_status packed_output(const amm_matrix* M, DevBuf& buf, float** out) {
  if (M->dtype == AMM_F32 && M->ld == M->cols) {
    *out = static_cast<float*>(M->data);
    return AMM_OK;
  }
  AMM_TRY(buf.reserve((size_t)M->rows * M->cols * sizeof(float)));
  *out = buf.as<float>();
  return AMM_OK;
}

amm_status finish_output(const amm_matrix* M, const float* res, hipStream_t s) {
  if (res == M->data) return AMM_OK;
  return cast_matrix(res, AMM_F32, M->cols, M->rows, M->cols, M->data, M->dtype, M->ld, s);
}
}  // namespace

extern "C" {

amm_status amm_approx_matmul_ex(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, const amm_matrix* B,
                                const amm_matrix* out, void* stream) {
  if (!ctx || !dA || !B || !out) return fail(AMM_EINVAL, "NULL argument");
  const int64_t n = dA->n, p = B->cols, m = dA->m;
  AMM_TRY(check_matrix(B, "B", n, p));
  AMM_TRY(check_matrix(out, "out", m, p));
  if (p == 0) return AMM_OK;
  if (matrices_overlap(B, out)) return fail(AMM_EINVAL, "out overlaps B");
  if (B->dtype == AMM_F32 && out->dtype == AMM_F32)
    return amm_approx_matmul_strided(ctx, dA, dB, static_cast<const float*>(B->data), n, p, B->ld,
                                     static_cast<float*>(out->data), out->ld, stream);
  if (dB && (dB->m != n || dB->n != p)) return fail(AMM_ESHAPE, "dB describes a %lldx%lld operand, B is %lldx%lld",
                                                    (long long)dB->m, (long long)dB->n, (long long)n, (long long)p);
  hipStream_t s = (hipStream_t)stream;
  AMM_HIP(hipSetDevice(ctx->device));
  TimerScope ts(ctx);
  const float* Bp = nullptr;
  float* Op = nullptr;
  AMM_TRY(packed_input(B, ctx->scratch[16], &Bp, s));
  AMM_TRY(packed_output(out, ctx->scratch[17], &Op));
  AMM_TRY(amm_approx_matmul(ctx, dA, dB, Bp, n, p, Op, stream));
  return finish_output(out, Op, s);
}

amm_status amm_approx_matmul_backward_ex(amm_ctx* ctx, const amm_dec* dW, const amm_matrix* X, const amm_matrix* dY,
                                         const amm_matrix* dX, const amm_matrix* dW_out, void* stream) {
  if (!ctx || !dW || !X || !dY) return fail(AMM_EINVAL, "NULL argument");
  const int64_t m = dW->m, n = dW->n, p = X->cols;
  AMM_TRY(check_matrix(X, "X", n, p));
  AMM_TRY(check_matrix(dY, "dY", m, p));
  if (dX) AMM_TRY(check_matrix(dX, "dX", n, p));
  if (dW_out) AMM_TRY(check_matrix(dW_out, "dW", m, n));
  if (!dX && !dW_out) return AMM_OK;
  for (const amm_matrix* o : {dX, dW_out})
    if (o && (matrices_overlap(o, X) || matrices_overlap(o, dY))) return fail(AMM_EINVAL, "an output overlaps an input");
  if (dX && dW_out && matrices_overlap(dX, dW_out)) return fail(AMM_EINVAL, "dX overlaps dW");
  hipStream_t s = (hipStream_t)stream;
  AMM_HIP(hipSetDevice(ctx->device));
  TimerScope ts(ctx);
  const float *Xp = nullptr, *Yp = nullptr;
  float *dXp = nullptr, *dWp = nullptr;
  AMM_TRY(packed_input(X, ctx->scratch[16], &Xp, s));
  AMM_TRY(packed_input(dY, ctx->scratch[18], &Yp, s));
  if (dX) AMM_TRY(packed_output(dX, ctx->scratch[17], &dXp));
  if (dW_out) AMM_TRY(packed_output(dW_out, ctx->scratch[19], &dWp));
  AMM_TRY(amm_approx_matmul_backward(ctx, dW, Xp, Yp, p, dXp, dWp, stream));
  if (dX) AMM_TRY(finish_output(dX, dXp, s));
  if (dW_out) AMM_TRY(finish_output(dW_out, dWp, s));
  return AMM_OK;
}

}  // extern "C"

extern "C" {

amm_status amm_approx_matmul_static(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, const float* B, int64_t n,
                                    int64_t p, float* out, void* stream) {
  if (!ctx || !dA) return fail(AMM_EINVAL, "NULL argument");
  if (n != dA->n) return fail(AMM_ESHAPE, "B has %lld rows, A has %lld columns", (long long)n, (long long)dA->n);
  if (p < 0) return fail(AMM_ESHAPE, "negative column count");
  if (p == 0) return AMM_OK;
  if (!B || !out) return fail(AMM_EINVAL, "NULL argument");
  if (dB && (dB->m != n || dB->n != p)) return fail(AMM_ESHAPE, "dB describes a %lldx%lld operand, B is %lldx%lld",
                                                    (long long)dB->m, (long long)dB->n, (long long)n, (long long)p);
  if (B == out) return fail(AMM_EINVAL, "out aliases B");
  if (!is_tsvd(dA) || (dB && !is_tsvd(dB)))
    return fail(AMM_EUNSUPPORTED, "the fixed-scratch product takes truncated-SVD handles only");
  if (dB && !(dA->A_borrowed && dB->residual.ptr))
    return fail(AMM_ESTATE, "first order needs A borrowed by dA and Delta B kept by dB");
  const int ka = dA->K_eff, kb = dB ? dB->K_eff : 0;
  if (!tsvd_split_shapes(dA->m, n, p, ka, kb))
    return fail(AMM_EUNSUPPORTED, "the fixed-scratch product needs ranks 32/64 (or 128 with 0 or 128), m, p "
                                  "multiples of 128 and n a multiple of 128");
  const size_t need = tsvd_split_scratch(dA->m, n, p, ka, kb);
  if (need > kStaticScratchFloats)
    return fail(AMM_EUNSUPPORTED, "the product needs %zu scratch floats, more than the fixed %zu", need,
                kStaticScratchFloats);
  float* scr = nullptr;
  AMM_TRY(static_scratch(ctx->device, &scr));
  hipStream_t s = (hipStream_t)stream;
  AMM_HIP(hipSetDevice(ctx->device));
  if (!dB)
    return tsvd_split_product(dA->m, n, p, ka, 0, dA->V.as<float>(), dA->US.as<float>(), B, nullptr, nullptr,
                              nullptr, scr, kStaticScratchFloats, out, s);
  return tsvd_split_product(dA->m, n, p, ka, kb, dA->V.as<float>(), dA->US.as<float>(), dB->residual.as<float>(),
                            dA->A_borrowed, dB->U.as<float>(), dB->VS.as<float>(), scr, kStaticScratchFloats, out, s);
}

static amm_status backward_body(amm_ctx* ctx, const amm_dec* dW, const float* X, const float* dY,
                                      int64_t p, float* dX, float* dW_out, void* stream) {
  if (!ctx || !dW || !X || !dY) return fail(AMM_EINVAL, "NULL argument");
  if (p <= 0) return fail(AMM_ESHAPE, "X has no columns");
  if (!dX && !dW_out) return AMM_OK;
  if (dX && (dX == dY || dX == X)) return fail(AMM_EINVAL, "dX aliases an input");
  if (dW_out && (dW_out == dY || dW_out == X)) return fail(AMM_EINVAL, "dW aliases an input");
  const amm_dec* c = dW;
  while (c) {
    if (c->kind == AMM_CIRCULANT && (c->m != c->n)) return fail(AMM_ESHAPE, "circulant handle not square");
    if (c->kind == AMM_TSVD && !c->Vt.ptr && dW_out) return fail(AMM_ESTATE, "SVD handle lacks V^T");
    c = c->inner;
  }
  hipStream_t s = (hipStream_t)stream;
  AMM_HIP(hipSetDevice(ctx->device));
  TimerScope ts(ctx);
  return approx_backward(ctx, dW, X, dY, p, dX, dW_out, s);
}

}  // extern "C"

namespace {

// circulant entries: the zeroth-order product of each entry in turn, blocked
// operands through the plan-owned scratch (so a captured graph never points
// into the context's growable buffers)
// The job table of a circulant plan: every power-of-two block product with
// side in [64, 16384] becomes one job (row blocks write their valid rows,
// column blocks read theirs and accumulate from the second block on, one
// launch phase per block index); other entries stay per-entry launches.
amm_status circ_build_jobs(amm_batch_plan* bp, bool x_bf16) {
  struct Key {
    int log2n, h16, phase;
    bool operator<(const Key& o) const {
      if (log2n != o.log2n) return log2n < o.log2n;
      if (h16 != o.h16) return h16 < o.h16;
      return phase < o.phase;
    }
  };
  std::map<Key, std::vector<CdJob>> groups;
  for (size_t i = 0; i < bp->items.size(); ++i) {
    const amm_dec* d = bp->decs[i];
    const auto& it = bp->items[i];
    const int64_t sd = d->blocks.empty() ? d->n : std::min(d->m, d->n);
    const int l2 = is_pow2(sd) ? log2_exact(sd) : -1;
    if (l2 < 0 || cd_tile_columns(l2) == 0) {
      if (x_bf16) return fail(AMM_EUNSUPPORTED, "entry %zu: side %lld outside the batched launches", i, (long long)sd);
      bp->cloose.push_back((int)i);
      continue;
    }
    const size_t esz = x_bf16 ? 2 : 4;
    const char* X = static_cast<const char*>(x_bf16 ? it.B16 : static_cast<const void*>(it.B));
    const int64_t p = it.p;
    auto job = [&](const amm_dec* b, const char* Xb, float* ob, int rows_in, int rows_out, int acc) {
      CdJob j{};
      j.X = Xb;
      j.out = ob;
      j.ldx = p;
      j.ldo = p;
      j.extent = p;
      j.shifts = b->shifts.as<int32_t>();
      j.L = b->lists16(false) ? static_cast<const void*>(b->lists16(false)) : static_cast<const void*>(b->L.as<float2>());
      j.pr = b->pairs_of(false);
      j.l16_inv = b->l16_inv;
      j.K = b->K_eff;
      j.accumulate = acc;
      j.x_bf16 = x_bf16 ? 1 : 0;
      const size_t xal = x_bf16 ? 8 : 16;
      j.vec4 = (p % 4 == 0 && ((uintptr_t)Xb % xal) == 0 && ((uintptr_t)ob % 16) == 0) ? 1 : 0;
      j.rows_in = rows_in;
      j.rows_out = rows_out;
      return j;
    };
    if (d->blocks.empty()) {
      groups[{l2, d->lists16(false) != nullptr, 0}].push_back(job(d, X, it.out, (int)sd, (int)sd, 0));
      continue;
    }
    for (size_t jb = 0; jb < d->blocks.size(); ++jb) {
      const amm_dec* b = d->blocks[jb];
      const int64_t lo = (int64_t)jb * sd;
      const int h = b->lists16(false) != nullptr;
      if (d->block_rows) {
        const int valid = (int)std::min<int64_t>(sd, d->m - lo);
        groups[{l2, h, 0}].push_back(job(b, X, it.out + lo * p, (int)sd, valid, 0));
      } else {
        const int valid = (int)std::min<int64_t>(sd, d->n - lo);
        groups[{l2, h, (int)jb}].push_back(job(b, X + (size_t)lo * p * esz, it.out, valid, (int)sd, jb > 0 ? 1 : 0));
      }
    }
  }
  // phases in order (the map's order is side, precision, phase: accumulation
  // phases of one group follow their first phase)
  for (auto& kv : groups) {
    amm_batch_plan::CircGroup g{kv.first.log2n, kv.first.h16 != 0, (int)bp->cjobs_host.size(), (int)kv.second.size(), 0};
    const int tc = cd_tile_columns(g.log2n);
    for (auto& j : kv.second) {
      j.tile0 = g.tiles;
      g.tiles += (int)((j.extent + tc - 1) / tc);
      bp->cjobs_host.push_back(j);
    }
    bp->cgroups.push_back(g);
  }
  if (!bp->cjobs_host.empty()) {
    AMM_TRY(bp->cjobs.alloc(bp->cjobs_host.size() * sizeof(CdJob)));
    AMM_HIP(hipMemcpy(bp->cjobs.ptr, bp->cjobs_host.data(), bp->cjobs_host.size() * sizeof(CdJob),
                      hipMemcpyHostToDevice));
  }
  return AMM_OK;
}

amm_status circ_one(amm_batch_plan* bp, size_t i, hipStream_t s);

amm_status circ_job_launches(amm_batch_plan* bp, hipStream_t s) {
  const CdJob* jobs = bp->cjobs.as<CdJob>();
  for (const auto& g : bp->cgroups)
    AMM_TRY(cd_apply_jobs(bp->ctx, g.log2n, g.h16, jobs + g.first_job, g.njobs, g.tiles, s));
  for (int i : bp->cloose) AMM_TRY(circ_one(bp, (size_t)i, s));
  return AMM_OK;
}

amm_status circ_launches(amm_batch_plan* bp, hipStream_t s) {
  if (bp->circ_mode == 1) return circ_job_launches(bp, s);
  for (size_t i = 0; i < bp->items.size(); ++i) AMM_TRY(circ_one(bp, i, s));
  return AMM_OK;
}

amm_status circ_one(amm_batch_plan* bp, size_t i, hipStream_t s) {
  {
    const amm_dec* d = bp->decs[i];
    const auto& it = bp->items[i];
    if (!d->blocks.empty()) {
      AMM_TRY(blocked_apply(bp->ctx, d, it.B, it.p, it.out, bp->partials.as<float>(), s));
    } else if (d->K_eff == 0) {
      AMM_TRY(fill_f32(it.out, it.m * it.p, 0.f, s));
    } else if (!is_pow2(d->n)) {
      AMM_TRY(cd_chirp_apply(bp->ctx, false, (int)d->n, d->K_eff, d->shifts.as<int32_t>(), d->L.as<float2>(), it.B,
                             it.p, it.out, false, s, d->lists16(false), d->l16_inv));
    } else {
      AMM_TRY(cd_apply_columns(bp->ctx, log2_exact(d->n), d->K_eff, d->shifts.as<int32_t>(), d->L.as<float2>(), it.B,
                               it.p, it.out, false, s, d->pairs_of(false), d->lists16(false), d->l16_inv));
    }
  }
  return AMM_OK;
}

amm_status plan_build(amm_batch_plan* bp, int t) {
  if (bp->launches) return AMM_OK;
  return bp->bf16 ? batch_build_bf16(bp, t) : batch_build(bp, t);
}
amm_status plan_launch(amm_batch_plan* bp, hipStream_t s) {
  if (bp->launches) return circ_launches(bp, s);
  return bp->bf16 ? batch_launch_bf16(bp, s) : batch_launch(bp, s);
}

// Autotune the reduction split policy by timing each candidate on the caller's
// stream, then capture the two launches once on a plan-owned stream; runs
// replay the graph.  Deletes the plan on failure.
// ---- tune cache ----------------------------------------------------------------
// A plan's tuned choice keyed by everything the timing depended on: the
// device (architecture, compute units), the plan kind and every entry's
// shape, rank or kept frequencies and list precision.  One text line per
// entry: "AMMTUNE1 <key> <choice> <ms> <ms_entry> <ms_table>"; the last line
// for a key wins, appends are single writes.
uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

uint64_t plan_key(const amm_batch_plan* bp) {
  uint64_t h = 1469598103934665603ull;
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, bp->ctx->device) == hipSuccess) {
    h = fnv1a(h, prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
    h = fnv1a(h, &prop.multiProcessorCount, sizeof(int));
  }
  const int head[3] = {bp->launches ? 1 : 0, bp->bf16 ? 1 : 0, bp->k};
  h = fnv1a(h, head, sizeof(head));
  for (size_t i = 0; i < bp->items.size(); ++i) {
    const auto& it = bp->items[i];
    const int64_t dims[3] = {it.m, it.n, it.p};
    h = fnv1a(h, dims, sizeof(dims));
    if (bp->launches) {
      const amm_dec* d = bp->decs[i];
      const amm_dec* b = d->blocks.empty() ? d : d->blocks[0];
      const int info[3] = {b->K_eff, b->lists16(false) ? 1 : 0, (int)d->blocks.size()};
      h = fnv1a(h, info, sizeof(info));
    }
  }
  return h;
}

bool tune_lookup(const std::string& path, uint64_t key, int* choice, double* ms, double* ms0, double* ms1) {
  if (path.empty()) return false;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    unsigned long long k = 0;
    int c = 0;
    double a = 0, b = 0, e = 0;
    if (std::sscanf(line, "AMMTUNE1 %llx %d %lf %lf %lf", &k, &c, &a, &b, &e) == 5 && k == key) {
      *choice = c;
      *ms = a;
      *ms0 = b;
      *ms1 = e;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void tune_store(const std::string& path, uint64_t key, int choice, double ms, double ms0, double ms1) {
  if (path.empty()) return;
  char line[256];
  const int len = std::snprintf(line, sizeof(line), "AMMTUNE1 %016llx %d %.6g %.6g %.6g\n", (unsigned long long)key,
                                choice, ms, ms0, ms1);
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;   // the cache is an optimisation: a file that cannot be written is skipped
  (void)std::fwrite(line, 1, (size_t)len, f);
  std::fclose(f);
}

// (Re)capture the plan's launches into its graph on its own stream.
amm_status plan_capture(amm_batch_plan* bp) {
  if (bp->exec) (void)hipGraphExecDestroy(bp->exec);
  if (bp->graph) (void)hipGraphDestroy(bp->graph);
  bp->exec = nullptr;
  bp->graph = nullptr;
  KernelTimer* saved = g_timer;
  g_timer = nullptr;
  amm_status st = AMM_OK;
  if (hipStreamBeginCapture(bp->own, hipStreamCaptureModeThreadLocal) != hipSuccess) st = fail(AMM_EDEVICE, "capture");
  if (st == AMM_OK) {
    amm_status ls = plan_launch(bp, bp->own);
    hipError_t ce = hipStreamEndCapture(bp->own, &bp->graph);
    if (ls != AMM_OK) st = ls;
    else if (ce != hipSuccess) st = hip_fail(ce, "hipStreamEndCapture");
  }
  if (st == AMM_OK && hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0) != hipSuccess)
    st = fail(AMM_EDEVICE, "hipGraphInstantiate");
  g_timer = saved;
  return st;
}

amm_status plan_finish(amm_batch_plan* bp, hipStream_t s, amm_batch_plan** plan) {
  const int candidates[] = {256, 512, 1024, 2048, 4096};
  double best = 1e30;
  int best_t = 1024;
  hipEvent_t e0, e1;
  amm_status st = AMM_OK;
  const uint64_t key = plan_key(bp);
  int cached = 0;
  double cms = 0, c0 = -1, c1 = -1;
  const bool hit = tune_lookup(bp->ctx->tune_cache, key, &cached, &cms, &c0, &c1) &&
                   (bp->launches ? (cached == 0 || cached == 1) && !(cached == 1 && bp->cgroups.empty()) &&
                                       !(cached == 0 && bp->bf16)
                                 : cached > 0);
  if (hit) {
    // the choice a tuning run stored for this device and these shapes
    bp->from_cache = true;
    if (bp->launches) {
      bp->circ_mode = cached;
      bp->circ_ms[0] = c0;
      bp->circ_ms[1] = c1;
    } else {
      best_t = cached;
    }
    best = 3.0 * cms;
  }
  if (!hit && hipEventCreate(&e0) != hipSuccess) st = fail(AMM_EDEVICE, "event");
  if (!hit && st == AMM_OK && hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); st = fail(AMM_EDEVICE, "event"); }
  if (hit) {
    // nothing to time
  } else if (st == AMM_OK && bp->launches) {
    // circulant plans: time the per-entry launches and the job-table launches
    // (a warm-up and three runs each) and keep the faster; bfloat16 plans
    // have only the job table
    for (int mode = bp->bf16 ? 1 : 0; mode <= (bp->cgroups.empty() ? 0 : 1) && st == AMM_OK; ++mode) {
      bp->circ_mode = mode;
      st = plan_launch(bp, s);
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < 3 && st == AMM_OK; ++r) st = plan_launch(bp, s);
      (void)hipEventRecord(e1, s);
      float ms = 0.f;
      if (st == AMM_OK && hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
      bp->circ_ms[mode] = ms / 3.0;
    }
    const bool table = bp->circ_ms[1] >= 0.0 && (bp->circ_ms[0] < 0.0 || bp->circ_ms[1] <= bp->circ_ms[0]);
    bp->circ_mode = table ? 1 : 0;
    best = 3.0 * bp->circ_ms[bp->circ_mode];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  } else if (st == AMM_OK) {
    for (int t : candidates) {
      if ((st = plan_build(bp, t)) != AMM_OK) break;
      if ((st = plan_launch(bp, s)) != AMM_OK) break;  // warm-up
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < 3 && st == AMM_OK; ++r) st = plan_launch(bp, s);
      (void)hipEventRecord(e1, s);
      if (st != AMM_OK) break;
      if (hipEventSynchronize(e1) != hipSuccess) { st = fail(AMM_EDEVICE, "tuning"); break; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) { best = ms; best_t = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  if (st == AMM_OK) st = plan_build(bp, best_t);
  bp->tuned_ms = best / 3.0;
  if (st == AMM_OK && !hit)
    tune_store(bp->ctx->tune_cache, key, bp->launches ? bp->circ_mode : best_t, bp->tuned_ms, bp->circ_ms[0],
               bp->circ_ms[1]);
  if (st == AMM_OK && hipStreamCreateWithFlags(&bp->own, hipStreamNonBlocking) != hipSuccess) st = fail(AMM_EDEVICE, "stream");
  if (st == AMM_OK) st = plan_capture(bp);
  if (st == AMM_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(AMM_EDEVICE, "sync");
  if (st != AMM_OK) {
    delete bp;
    return st;
  }
  *plan = bp;
  return AMM_OK;
}

// shared argument checks: one rank, truncated-SVD handles, shapes on the path
amm_status plan_check(int count, const amm_dec* const* dA, const void* const* B, const int64_t* p,
                      float* const* out, bool bf16, int* k_out) {
  if (count <= 0 || count > batch_max_items()) return fail(AMM_EINVAL, "batch size %d out of [1, %d]", count, batch_max_items());
  int k = -1;
  for (int i = 0; i < count; ++i) {
    const amm_dec* d = dA[i];
    if (!d || !B[i] || !out[i]) return fail(AMM_EINVAL, "NULL entry %d", i);
    if (d->kind == AMM_CIRCULANT && dA[0]->kind == AMM_CIRCULANT) {
      if (p[i] <= 0) return fail(AMM_ESHAPE, "entry %d has no columns", i);
      const int64_t side = d->blocks.empty() ? d->n : std::min(d->m, d->n);
      if (bf16 && !(is_pow2(side) && cd_tile_columns(log2_exact(side)) > 0))
        return fail(AMM_EUNSUPPORTED, "entry %d: bfloat16 circulant plans need power-of-two sides in [64, 16384]", i);
      if (!is_pow2(side) && !(side >= 3 && side <= kChirpFusedMax))
        return fail(AMM_EUNSUPPORTED, "entry %d: circulant plans need power-of-two sides or sides up to %d", i,
                    kChirpFusedMax);
      continue;
    }
    if (d->kind != AMM_TSVD || dA[0]->kind != AMM_TSVD)
      return fail(AMM_EUNSUPPORTED, "batch entries must be all truncated-SVD or all circulant handles");
    if (k < 0) k = d->K_eff;
    if (d->K_eff != k) return fail(AMM_EUNSUPPORTED, "batch entries must share one rank");
    const bool ok = bf16 ? batch_item_ok_bf16(d->m, d->n, p[i], k) : batch_item_ok(d->m, d->n, p[i], k);
    if (!ok)
      return fail(AMM_EUNSUPPORTED, "entry %d: shape %lldx%lld by %lld columns, rank %d not on the batched path", i,
                  (long long)d->m, (long long)d->n, (long long)p[i], k);
  }
  *k_out = k;
  return AMM_OK;
}

}  // namespace

extern "C" {

amm_status amm_batch_plan_create(amm_ctx* ctx, int count, const amm_dec* const* dA, const float* const* B,
                                 const int64_t* p, float* const* out, void* stream, amm_batch_plan** plan) {
  TimerScope ts(ctx);
  if (!ctx || !dA || !B || !p || !out || !plan) return fail(AMM_EINVAL, "NULL argument");
  int k = 0;
  AMM_TRY(plan_check(count, dA, reinterpret_cast<const void* const*>(B), p, out, false, &k));
  AMM_HIP(hipSetDevice(ctx->device));
  amm_batch_plan* bp = new amm_batch_plan();
  bp->ctx = ctx;
  bp->k = k;
  if (dA[0]->kind == AMM_CIRCULANT) {
    // circulant entries: plan-owned scratch and every twiddle table made now,
    // so that running (or capturing) the plan allocates nothing
    bp->launches = true;
    size_t scratch = 1;
    for (int i = 0; i < count; ++i) {
      const amm_dec* d = dA[i];
      bp->items.push_back({d->m, d->n, p[i], nullptr, nullptr, B[i], out[i]});
      bp->decs.push_back(d);
      const int64_t sd = d->blocks.empty() ? d->n : std::min(d->m, d->n);
      if (!d->blocks.empty()) scratch = std::max(scratch, (size_t)sd * p[i]);
      const float2* tw = nullptr;
      amm_status st;
      if (is_pow2(sd)) {
        st = twiddles32(ctx, log2_exact(sd), &tw);
      } else {   // the fused chirp-convolution kernel: its twiddles and chirp tables
        int lM = 0;
        while ((int64_t(1) << lM) < 2 * sd - 1) ++lM;
        const float2* tab = nullptr;
        st = twiddles32(ctx, lM, &tw);
        if (st == AMM_OK) st = chirp_tables32(ctx, (int)sd, (hipStream_t)stream, &tab);
      }
      if (st != AMM_OK) {
        delete bp;
        return st;
      }
    }
    amm_status st = bp->partials.alloc(scratch * sizeof(float));
    if (st == AMM_OK) st = circ_build_jobs(bp, false);
    if (st != AMM_OK) {
      delete bp;
      return st;
    }
    return plan_finish(bp, (hipStream_t)stream, plan);
  }
  for (int i = 0; i < count; ++i)
    bp->items.push_back({dA[i]->m, dA[i]->n, p[i], dA[i]->V.as<float>(), dA[i]->US.as<float>(), B[i], out[i]});
  return plan_finish(bp, (hipStream_t)stream, plan);
}

amm_status amm_batch_plan_create_bf16(amm_ctx* ctx, int count, const amm_dec* const* dA, const void* const* B,
                                      const int64_t* p, float* const* out, void* stream, amm_batch_plan** plan) {
  TimerScope ts(ctx);
  if (!ctx || !dA || !B || !p || !out || !plan) return fail(AMM_EINVAL, "NULL argument");
  int k = 0;
  AMM_TRY(plan_check(count, dA, B, p, out, true, &k));
  AMM_HIP(hipSetDevice(ctx->device));
  amm_batch_plan* bp = new amm_batch_plan();
  bp->ctx = ctx;
  bp->k = k;
  bp->bf16 = true;
  if (dA[0]->kind == AMM_CIRCULANT) {
    // bfloat16 B_i read by the batched launches (widened in the load), float32 products
    bp->launches = true;
    amm_status st = AMM_OK;
    for (int i = 0; i < count && st == AMM_OK; ++i) {
      amm_batch_plan::Item it{dA[i]->m, dA[i]->n, p[i], nullptr, nullptr, nullptr, out[i]};
      it.B16 = B[i];
      bp->items.push_back(it);
      bp->decs.push_back(dA[i]);
      const int64_t sd = dA[i]->blocks.empty() ? dA[i]->n : std::min(dA[i]->m, dA[i]->n);
      const float2* tw = nullptr;
      st = twiddles32(ctx, log2_exact(sd), &tw);
    }
    if (st == AMM_OK) st = circ_build_jobs(bp, true);
    if (st != AMM_OK) {
      delete bp;
      return st;
    }
    return plan_finish(bp, (hipStream_t)stream, plan);
  }
  std::vector<const float*> V, US;
  for (int i = 0; i < count; ++i) {
    amm_batch_plan::Item it{dA[i]->m, dA[i]->n, p[i], nullptr, nullptr, nullptr, out[i]};
    it.B16 = B[i];
    bp->items.push_back(it);
    V.push_back(dA[i]->V.as<float>());
    US.push_back(dA[i]->US.as<float>());
  }
  hipStream_t s = (hipStream_t)stream;
  amm_status st = batch_convert_bf16(bp, V, US, s);
  if (st != AMM_OK) {
    delete bp;
    return st;
  }
  return plan_finish(bp, s, plan);
}

static amm_status batch_run_body(amm_batch_plan* plan, int use_graph, void* stream) {
  if (!plan) return fail(AMM_EINVAL, "NULL plan");
  hipStream_t s = (hipStream_t)stream;
  TimerScope ts(plan->ctx);
  if (use_graph && plan->exec && !g_timer) {
    AMM_HIP(hipGraphLaunch(plan->exec, s));
    return AMM_OK;
  }
  return plan_launch(plan, s);
}

amm_status amm_batch_circulant_set_mode(amm_batch_plan* plan, int job_table) {
  if (!plan) return fail(AMM_EINVAL, "NULL plan");
  if (!plan->launches) return fail(AMM_ESTATE, "not a circulant plan");
  if (job_table && plan->cgroups.empty()) return fail(AMM_EUNSUPPORTED, "no entry runs in the batched launches");
  if (!job_table && plan->bf16) return fail(AMM_EUNSUPPORTED, "bfloat16 plans run only the batched launches");
  TimerScope ts(plan->ctx);
  AMM_HIP(hipSetDevice(plan->ctx->device));
  AMM_HIP(hipStreamSynchronize(plan->own));
  plan->circ_mode = job_table ? 1 : 0;
  return plan_capture(plan);
}

amm_status amm_batch_circulant_schedule(const amm_batch_plan* plan, int* job_table, int* launches,
                                        double* entry_ms, double* table_ms) {
  if (!plan) return fail(AMM_EINVAL, "NULL plan");
  if (!plan->launches) return fail(AMM_ESTATE, "not a circulant plan");
  if (job_table) *job_table = plan->circ_mode;
  if (launches)
    *launches = plan->circ_mode == 1 ? (int)(plan->cgroups.size() + plan->cloose.size()) : (int)plan->items.size();
  if (entry_ms) *entry_ms = plan->circ_ms[0];
  if (table_ms) *table_ms = plan->circ_ms[1];
  return AMM_OK;
}

amm_status amm_batch_info(const amm_batch_plan* plan, int* target_blocks, int* panel_blocks, int* out_blocks,
                          double* tuned_ms) {
  if (!plan) return fail(AMM_EINVAL, "NULL plan");
  if (target_blocks) *target_blocks = plan->target_blocks;
  if (panel_blocks) *panel_blocks = plan->panel_blocks;
  if (out_blocks) *out_blocks = plan->out_blocks;
  if (tuned_ms) *tuned_ms = plan->tuned_ms;
  return AMM_OK;
}

void amm_batch_plan_destroy(amm_batch_plan* plan) {
  if (!plan) return;
  if (plan->own) (void)hipStreamSynchronize(plan->own);
  delete plan;
}

}  // extern "C"

// ---- error estimates (Sec. 2.5, Sec. 3) ------------------------------------
namespace {

const amm_dec* core_of(const amm_dec* d) { return (d->kind & AMM_SPARSE) ? d->inner : d; }

bool is_finite(double x) { return std::isfinite(x); }

// Thm. 3.6 without its vanishing term: the norm ratio, times 4/(3 sqrt n) for U(0, a) entries
double prior_of(double nA, double nB, double dA, double dB, int64_t n, int entries) {
  if (!is_finite(nA) || !is_finite(nB) || !is_finite(dA) || !is_finite(dB)) return NAN;
  if (nA == 0.0 || nB == 0.0) return (dA * dB == 0.0) ? 0.0 : INFINITY;
  const double ratio = dA * dB / (nA * nB);
  return entries == AMM_ENTRIES_UNSIGNED_UNIFORM ? 4.0 / (3.0 * std::sqrt((double)n)) * ratio : ratio;
}

}  // namespace

extern "C" {

amm_status amm_dec_set_spectral_fp16(amm_dec* dec, int enable) {
  TimerScope ts(static_cast<const amm_dec*>(dec));
  if (!dec) return fail(AMM_EINVAL, "NULL handle");
  amm_dec* c = is_sparse(dec) ? dec->inner : dec;
  if (!c || c->kind != AMM_CIRCULANT) return fail(AMM_EINVAL, "not a circulant handle (or sparse with a circulant residue)");
  std::vector<amm_dec*> parts;
  if (c->blocks.empty()) parts.push_back(c);
  else parts.assign(c->blocks.begin(), c->blocks.end());
  for (amm_dec* b : parts) {
    const bool pow2 = is_pow2(b->n);
    if (enable && (b->n < 1024 || (!pow2 && b->n > kChirpFusedMax)))
      return fail(AMM_EUNSUPPORTED, "float16 spectral products need n >= 1024 (a power of two, or at most %d)",
                  kChirpFusedMax);
  }
  AMM_HIP(hipSetDevice(c->device));
  for (amm_dec* b : parts) {
    if (!enable) {
      b->fp16 = false;
      continue;
    }
    if (b->fp16 || b->K_eff == 0) continue;
    std::vector<float2> Lh((size_t)b->K_eff * b->n);
    AMM_HIP(hipMemcpy(Lh.data(), b->L.ptr, Lh.size() * sizeof(float2), hipMemcpyDeviceToHost));
    AMM_TRY(cd_make_half_lists(b, Lh, nullptr));
    AMM_HIP(hipStreamSynchronize(nullptr));
  }
  return AMM_OK;
}

amm_status amm_dec_set_sigma_next(amm_dec* dec, double sigma_next) {
  if (!dec) return fail(AMM_EINVAL, "NULL argument");
  amm_dec* c = (dec->kind & AMM_SPARSE) ? dec->inner : dec;
  if (!c || c->kind != AMM_TSVD) return fail(AMM_EINVAL, "not a truncated-SVD handle");
  if (!(sigma_next >= 0.0)) return fail(AMM_EINVAL, "sigma_next must be >= 0");
  c->sigma_next = sigma_next;
  return AMM_OK;
}

amm_status amm_estimate_error(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, const float* M, int64_t m,
                              int64_t p, int entries, void* stream, amm_error_estimate* out) {
  TimerScope ts(ctx);
  if (!ctx || !dA || !dB || !out) return fail(AMM_EINVAL, "NULL argument");
  if (entries != AMM_ENTRIES_SIGNED && entries != AMM_ENTRIES_UNSIGNED_UNIFORM)
    return fail(AMM_EINVAL, "entries = %d", entries);
  if (dA->n != dB->m) return fail(AMM_ESHAPE, "inner dimensions differ (%lld, %lld)", (long long)dA->n,
                                  (long long)dB->m);
  if (M && (m != dA->m || p != dB->n)) return fail(AMM_ESHAPE, "M is %lld x %lld, product is %lld x %lld",
                                                   (long long)m, (long long)p, (long long)dA->m, (long long)dB->n);
  AMM_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = dA->n;
  amm_error_estimate e;
  e.norm_A = dA->norm_A;
  e.norm_B = dB->norm_A;
  e.norm_dA = dA->norm_residual;
  e.norm_dB = dB->norm_residual;
  e.prior = prior_of(e.norm_A, e.norm_B, e.norm_dA, e.norm_dB, n, entries);
  e.norm_M = NAN;
  if (M) {
    double t = 0.0;
    AMM_TRY(sumsq_f32(M, m * p, s, &t));
    e.norm_M = std::sqrt(t);
  }
  const double num = e.norm_dA * e.norm_dB;
  auto over_M = [&](double v) {
    if (!is_finite(v) || !is_finite(e.norm_M)) return (double)NAN;
    if (e.norm_M == 0.0) return v == 0.0 ? 0.0 : (double)INFINITY;
    return v / e.norm_M;
  };
  // Cor. 3.7
  e.posterior = over_M(num / std::sqrt((double)n));
  const amm_dec* ca = core_of(dA);
  const amm_dec* cb = core_of(dB);
  // Thm. 3.8 with ||Delta||_2 = sigma_{k+1}
  e.spec_dA = (ca && ca->kind == AMM_TSVD) ? ca->sigma_next : NAN;
  e.spec_dB = (cb && cb->kind == AMM_TSVD) ? cb->sigma_next : NAN;
  e.svd_bound = over_M(std::sqrt(e.spec_dA * e.spec_dB * num));
  // circulant residual theorem, used as an estimate
  const bool cda = ca && ca->kind == AMM_CIRCULANT && ca->blocks.empty();
  const bool cdb = cb && cb->kind == AMM_CIRCULANT && cb->blocks.empty();
  e.mu_A = cda ? ca->mu : NAN;
  e.mu_B = cdb ? cb->mu : NAN;
  e.cd_estimate = over_M(std::pow(e.mu_A * e.mu_B, 0.25) / std::sqrt((double)n) * num);
  *out = e;
  return AMM_OK;
}

amm_status amm_estimate_sketch(amm_ctx* ctx, const float* A, const float* B, const float* M, const float* G,
                               int64_t m, int64_t n, int64_t p, int64_t l, void* stream, double* est) {
  TimerScope ts(ctx);
  if (!ctx || !A || !B || !M || !G || !est) return fail(AMM_EINVAL, "NULL argument");
  if (m <= 0 || n <= 0 || p <= 0 || l <= 0) return fail(AMM_ESHAPE, "empty sketch shape");
  AMM_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  DevBuf Y, N, MG;
  AMM_TRY(Y.alloc(n * l * sizeof(float)));
  AMM_TRY(N.alloc(m * l * sizeof(float)));
  AMM_TRY(MG.alloc(m * l * sizeof(float)));
  AMM_TRY(gemm_f32(n, l, p, 1.f, MatView{B, p, 1}, MatView{G, l, 1}, 0.f, Y.as<float>(), l, s, "sketch_gemm"));
  AMM_TRY(gemm_f32(m, l, n, 1.f, MatView{A, n, 1}, MatView{Y.as<float>(), l, 1}, 0.f, N.as<float>(), l, s,
                   "sketch_gemm"));
  AMM_TRY(gemm_f32(m, l, p, 1.f, MatView{M, p, 1}, MatView{G, l, 1}, 0.f, MG.as<float>(), l, s, "sketch_gemm"));
  double dd = 0.0, xx = 0.0;
  AMM_TRY(diff_sumsq_f32(N.as<float>(), MG.as<float>(), m * l, s, &dd, &xx));
  *est = xx > 0.0 ? std::sqrt(dd / xx) : 0.0;
  return AMM_OK;
}

amm_status amm_choose_rank(const amm_dec* dA, const amm_dec* dB, double tau, int entries, int* K) {
  if (!dA || !dB || !K) return fail(AMM_EINVAL, "NULL argument");
  if (!(tau >= 0.0)) return fail(AMM_EINVAL, "tolerance must be >= 0");
  if (entries != AMM_ENTRIES_SIGNED && entries != AMM_ENTRIES_UNSIGNED_UNIFORM)
    return fail(AMM_EINVAL, "entries = %d", entries);
  if (dA->n != dB->m) return fail(AMM_ESHAPE, "inner dimensions differ");
  const int64_t n = dA->n;
  if (dA->kind == AMM_CIRCULANT && dB->kind == AMM_CIRCULANT) {
    if (!dA->has_energies || !dB->has_energies || !dA->blocks.empty() || !dB->blocks.empty() || dA->n != dB->n)
      return fail(AMM_EUNSUPPORTED, "rank choice needs square circulant handles made by amm_decompose");
    std::vector<double> EA(n), EB(n);
    AMM_HIP(hipMemcpy(EA.data(), dA->energies.ptr, n * sizeof(double), hipMemcpyDeviceToHost));
    AMM_HIP(hipMemcpy(EB.data(), dB->energies.ptr, n * sizeof(double), hipMemcpyDeviceToHost));
    const std::vector<double> RA = retained_all(EA), RB = retained_all(EB);
    double ta = 0.0, tb = 0.0;
    for (double v : EA) ta += v;
    for (double v : EB) tb += v;
    for (int64_t k = 0; k <= n; ++k) {
      const double pr = prior_of(std::sqrt(ta), std::sqrt(tb), std::sqrt(std::max(ta - RA[k], 0.0)),
                                 std::sqrt(std::max(tb - RB[k], 0.0)), n, entries);
      if (pr <= tau) {
        *K = (int)k;
        return AMM_OK;
      }
    }
    *K = (int)n;
    return AMM_OK;
  }
  if (dA->kind == AMM_TSVD && dB->kind == AMM_TSVD) {
    if (!is_finite(dA->norm_A) || !is_finite(dB->norm_A))
      return fail(AMM_ESTATE, "norms unknown (import the factors with A)");
    const int kmax = std::min({dA->K_eff, dB->K_eff, (int)dA->sigma64.size(), (int)dB->sigma64.size()});
    const std::vector<double>& sa = dA->sigma64;
    const std::vector<double>& sb = dB->sigma64;
    double ka = 0.0, kb = 0.0;
    for (int k = 0; k <= kmax; ++k) {
      if (k > 0) {
        ka += sa[k - 1] * sa[k - 1];
        kb += sb[k - 1] * sb[k - 1];
      }
      const double pr = prior_of(dA->norm_A, dB->norm_A, std::sqrt(std::max(dA->norm_A * dA->norm_A - ka, 0.0)),
                                 std::sqrt(std::max(dB->norm_A * dB->norm_A - kb, 0.0)), n, entries);
      if (pr <= tau) {
        *K = k;
        return AMM_OK;
      }
    }
    *K = kmax;
    return AMM_OK;
  }
  return fail(AMM_EUNSUPPORTED, "rank choice for two circulant or two truncated-SVD handles");
}

}  // extern "C"

// ---- debug mode: argument pointers checked, every call synchronised ----------
namespace {

// In debug mode a pointer the device would dereference must be device (or
// managed, or mapped host) memory reachable from the context's device.
amm_status debug_pointer(const amm_ctx* ctx, const void* ptr, const char* name) {
  if (!ctx || !ctx->debug || !ptr) return AMM_OK;
  hipPointerAttribute_t a{};
  const hipError_t e = hipPointerGetAttributes(&a, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();   // the query's failure is not a device error
    return fail(AMM_EINVAL, "%s (%p) is not device memory", name, ptr);
  }
  const bool device_side = a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged ||
                           (a.type == hipMemoryTypeHost && a.devicePointer);
  if (!device_side) return fail(AMM_EINVAL, "%s (%p) is not device memory", name, ptr);
  if (a.type == hipMemoryTypeDevice && a.device != ctx->device)
    return fail(AMM_EINVAL, "%s lives on device %d, the context on device %d", name, a.device, ctx->device);
  return AMM_OK;
}

// In debug mode wait for the call's work and report any device error as the call's.
amm_status debug_finish(const amm_ctx* ctx, hipStream_t s, amm_status st, const char* what) {
  if (!ctx || !ctx->debug || st != AMM_OK) return st;
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(AMM_EDEVICE, "%s: device error after the call: %s", what, hipGetErrorString(e));
  return AMM_OK;
}

}  // namespace

extern "C" {

amm_status amm_ctx_set_tune_cache(amm_ctx* ctx, const char* path) {
  if (!ctx) return fail(AMM_EINVAL, "NULL context");
  ctx->tune_cache = path ? path : "";
  return AMM_OK;
}

amm_status amm_batch_tuned_from_cache(const amm_batch_plan* plan, int* from_cache) {
  if (!plan || !from_cache) return fail(AMM_EINVAL, "NULL argument");
  *from_cache = plan->from_cache ? 1 : 0;
  return AMM_OK;
}

amm_status amm_ctx_set_debug(amm_ctx* ctx, int enable) {
  if (!ctx) return fail(AMM_EINVAL, "NULL context");
  ctx->debug = enable != 0;
  return AMM_OK;
}

amm_status amm_decompose(amm_ctx* ctx, const float* A, int64_t m, int64_t n, int kind, int K, const amm_opts* opts,
                         void* stream, amm_dec** out) {
  AMM_TRY(debug_pointer(ctx, A, "A"));
  return debug_finish(ctx, (hipStream_t)stream, decompose_body(ctx, A, m, n, kind, K, opts, stream, out),
                      "amm_decompose");
}

amm_status amm_approx_matmul(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, const float* B, int64_t n, int64_t p,
                             float* out, void* stream) {
  AMM_TRY(debug_pointer(ctx, B, "B"));
  AMM_TRY(debug_pointer(ctx, out, "out"));
  return debug_finish(ctx, (hipStream_t)stream, matmul_body(ctx, dA, dB, B, n, p, out, stream), "amm_approx_matmul");
}

amm_status amm_approx_matmul_strided(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, const float* B, int64_t n,
                                     int64_t p, int64_t ldb, float* out, int64_t ldo, void* stream) {
  AMM_TRY(debug_pointer(ctx, B, "B"));
  AMM_TRY(debug_pointer(ctx, out, "out"));
  return debug_finish(ctx, (hipStream_t)stream, strided_body(ctx, dA, dB, B, n, p, ldb, out, ldo, stream),
                      "amm_approx_matmul_strided");
}

amm_status amm_approx_matmul_backward(amm_ctx* ctx, const amm_dec* dW, const float* X, const float* dY, int64_t p,
                                      float* dX, float* dW_out, void* stream) {
  AMM_TRY(debug_pointer(ctx, X, "X"));
  AMM_TRY(debug_pointer(ctx, dY, "dY"));
  AMM_TRY(debug_pointer(ctx, dX, "dX"));
  AMM_TRY(debug_pointer(ctx, dW_out, "dW"));
  return debug_finish(ctx, (hipStream_t)stream, backward_body(ctx, dW, X, dY, p, dX, dW_out, stream),
                      "amm_approx_matmul_backward");
}

amm_status amm_batch_run(amm_batch_plan* plan, int use_graph, void* stream) {
  return debug_finish(plan ? plan->ctx : nullptr, (hipStream_t)stream, batch_run_body(plan, use_graph, stream),
                      "amm_batch_run");
}

}  // extern "C"
