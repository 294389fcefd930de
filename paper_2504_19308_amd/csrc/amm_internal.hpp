// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <map>
#include <string>
#include <functional>
#include <vector>

#include "host_logic.hpp"
#include <cmath>

#include "amm.h"

namespace amm {

// ---- error reporting -------------------------------------------------------
amm_status fail(amm_status st, const char* fmt, ...);
amm_status hip_fail(hipError_t e, const char* what);

#define AMM_HIP(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return amm::hip_fail(e_, #call); \
  } while (0)

#define AMM_TRY(call)                    \
  do {                                   \
    amm_status s_ = (call);              \
    if (s_ != AMM_OK) return s_;         \
  } while (0)

// ---- device buffers ---------------------------------------------------------
// Device allocations go through the allocator of the context the current API
// call works for (amm_ctx_create_with_allocator), else hipMalloc; a buffer
// keeps the functions it was allocated with and frees through them.
struct AllocFns {
  void* (*alloc)(size_t bytes, int device, void* user) = nullptr;
  void (*free)(void* ptr, size_t bytes, int device, void* user) = nullptr;
  void* user = nullptr;
  int device = 0;
};
extern thread_local const AllocFns* g_alloc;

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  AllocFns fns{};
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), bytes(o.bytes), fns(o.fns) { o.ptr = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      ptr = o.ptr;
      bytes = o.bytes;
      fns = o.fns;
      o.ptr = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (ptr) {
      if (fns.free) fns.free(ptr, bytes, fns.device, fns.user);
      else (void)hipFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
  }
  amm_status alloc(size_t b);          // exact-size allocation (frees old)
  amm_status reserve(size_t b);        // grow-only
  template <typename T> T* as() const { return static_cast<T*>(ptr); }
};

// ---- optional per-launch timing ---------------------------------------------
// When a context has timing enabled, every kernel launch made on its behalf is
// bracketed by hipEventRecord on the launch stream; amm_ctx_timings() resolves
// the events and reports the total and count per kernel name.
struct KernelTimer {
  struct Pending { const char* name; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::map<std::string, std::pair<double, long>> totals;  // ms, launches
  // events are created once and reused, so a timed launch adds two records
  // and no event creation to the host's launch path.  They only carry
  // timestamps (the host waits on the stream, not on them), so they are made
  // without the system-scope fence, which would write back the caches at
  // every marker and bill that to the kernel between them.
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~KernelTimer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};
extern thread_local KernelTimer* g_timer;
// split-K partial sums of the GEMMs: the work area of the context the current
// API call works for (nullptr outside a context call)
extern thread_local DevBuf* g_gemm_part;

struct TimedLaunch {
  hipEvent_t b_ = nullptr;
  hipStream_t s_;
  const char* name_;
  TimedLaunch(const char* name, hipStream_t s) : s_(s), name_(name) {
    if (!g_timer) return;
    hipEvent_t a = g_timer->take();
    b_ = a ? g_timer->take() : nullptr;
    if (!b_) return;
    (void)hipEventRecord(a, s_);
    g_timer->pending.push_back({name_, a, b_});
  }
  ~TimedLaunch() {
    if (b_) (void)hipEventRecord(b_, s_);
  }
};

// Optional pair structure of a real operator's closed frequency set:
// pairs[u] = {k, t} for each pair {k, N-k} (t the list index of k), singles
// for the self-paired 0 and N/2.  npairs < 0: use the plain K-term loop.
struct CdPairs {
  const int2* pairs = nullptr;
  int npairs = -1;
  const int2* singles = nullptr;
  int nsingles = 0;
};

// One product of a batched circulant launch (column mode): out (N x extent)
// (+)= Atil X for one square block, over the launch's workgroups tile0 ..
// tile0 + tiles - 1.  Rows of X at or past rows_in read as zero (the padded
// last block of a column-blocked operand); rows of out at or past rows_out
// are not written (the overhang of a row-blocked one).
struct CdJob {
  const void* X;            // float32, or bfloat16 when x_bf16
  float* out;
  int64_t ldx, ldo, extent;
  const int32_t* shifts;
  const void* L;            // float2 lists, or the float16 ones of a float16 launch
  CdPairs pr;
  float l16_inv;
  int K, accumulate, vec4, x_bf16;
  int rows_in, rows_out;
  int tile0;
};
}  // namespace amm

struct amm_ctx {
  int device = 0;
  amm::AllocFns alloc;                 // caller's allocator (alloc == NULL: hipMalloc)
  std::map<int, amm::DevBuf> tw32;     // per log2 n: n float2, exp(-2 pi i m / n)
  std::map<int, amm::DevBuf> tw64;     // per log2 n: n double2
  amm::DevBuf scratch[20];             // grow-only work areas for products (8-13: chirp-convolution path,
                                       // 14, 15: B and the residue's product at a spread row pitch for
                                       // sparse products; 16-19: packed float32 copies of strided or
                                       // 16-bit operands)
  std::map<int64_t, amm::DevBuf> chirp64;   // per (n, sign): float64 spectrum of the chirp kernel
  std::map<int, amm::DevBuf> chirp32;       // per n: float32 chirp and kernel spectra of the fused product
  amm::DevBuf rsvd[14];                     // grow-only work areas of the randomized SVD
  amm::DevBuf gemm_part;                    // grow-only split-K partial sums
  amm::KernelTimer timer;
  bool timing = false;
  bool debug = false;
  std::string tune_cache;              // file of tuned batch-plan choices ("" = none)                  // check argument pointers, synchronise after every call
};

struct amm_dec {
  amm_dec() {
    if (amm::g_alloc) alloc = *amm::g_alloc;   // the allocator of the call that makes the handle
  }
  int kind = 0;
  int64_t m = 0, n = 0;
  int K = 0;
  int K_eff = 0;
  double norm_A = 0.0;
  double norm_residual = 0.0;
  // residual statistics for the error estimates (NaN: not available)
  double mu = NAN;           // circulant: max_i X_i / (||Delta A||_F^2 / n)
  double sigma_next = NAN;   // truncated SVD: estimate of sigma_{k+1} = ||Delta A||_2
  std::vector<double> sigma64;  // truncated SVD: the kept singular values in float64 (host)
  int device = 0;
  amm::AllocFns alloc;          // allocator of the context that made the handle

  // Fourier-domain sparsification: left role (rows of A conj(F) / n, CSR)
  // and its residual half spectrum ((n/2+1) x m, transposed); right role
  // (columns of F A: half-spectrum representatives with their pair weight)
  amm::DevBuf sf_rptr, sf_ridx, sf_rval, sf_Rt, sf_cptr, sf_cidx, sf_cval;
  bool sf_left = false, sf_right = false;

  // circulant (n x n): kept frequencies, float32 eigenvalue lists and the
  // adjoint lists  Ladj_t[p] = conj(L_t[(p + k_t) mod n]) with shift -k_t.
  std::vector<int32_t> freqs;
  amm::DevBuf shifts;      // K_eff int32: k_t
  amm::DevBuf shifts_adj;  // K_eff int32: (n - k_t) mod n
  amm::DevBuf L;           // K_eff x n float2
  amm::DevBuf Ladj;        // K_eff x n float2
  amm::DevBuf energies;    // n double (decompose only)
  // float16 copies of L and Ladj used by the products when requested (n >= 1024)
  amm::DevBuf L16, Ladj16;
  bool fp16 = false;
  float l16_inv = 1.0f;   // the float16 lists hold L / l16_inv (a power of two)
  const __half2* lists16(bool adjoint) const {
    if (!fp16) return nullptr;
    return adjoint ? Ladj16.as<__half2>() : L16.as<__half2>();
  }
  // pair structure for the paired spectral MAC (npairs < 0: not available)
  amm::DevBuf pair_buf;     // int2: pairs, singles, pairs_adj, singles_adj
  int npairs = -1, nsingles = 0, npairs_adj = -1, nsingles_adj = 0;
  amm::CdPairs pairs_of(bool adjoint) const {
    const int2* b = pair_buf.as<int2>();
    if (adjoint) {
      if (npairs_adj < 0) return amm::CdPairs{};
      const int2* p = b + npairs + nsingles;
      return amm::CdPairs{p, npairs_adj, p + npairs_adj, nsingles_adj};
    }
    if (npairs < 0) return amm::CdPairs{};
    return amm::CdPairs{b, npairs, b + npairs, nsingles};
  }
  bool has_energies = false;

  // SVD: U m x k, V n x k, sigma k (float32), US = U diag(sigma), VS = V diag(sigma),
  // VSt = (V diag(sigma))^T  (k x n, for the fused first-order output GEMM)
  amm::DevBuf U, V, sigma, US, VS, VSt, Vt;

  // sparse part: CSR (row_ptr m+1, col, val) and its transpose as CSC
  // (csc_ptr n+1, csc_row, csc_val) for products with S on the right
  int64_t nnz = 0;
  amm::DevBuf row_ptr, col, val;
  amm::DevBuf csc_ptr, csc_row, csc_val;
  // entry ranges of each CSR row (CSC column) per block of 4096 inner indices,
  // (blocks + 1) offsets per row; blocks = 1 keeps row_ptr (csc_ptr) alone
  amm::DevBuf csr_blk, csc_blk;
  int csr_blocks = 1, csc_blocks = 1;
  amm_dec* inner = nullptr;

  // rectangular circulant operand: square blocks of side s = min(m, n) along
  // the longer dimension (the last one zero-padded), each its own circulant
  // decomposition; block_rows: blocks stacked down the rows (m > n)
  std::vector<amm_dec*> blocks;
  bool block_rows = false;

  // Delta A: owned (circulant) or borrowed A (SVD / sparse)
  amm::DevBuf residual;        // m x n float32, owned
  const float* A_borrowed = nullptr;

  ~amm_dec();
};

struct amm_batch_plan {
  struct Item {
    int64_t m, n, p;
    const float* V;    // n x k
    const float* US;   // m x k
    const float* B;    // n x p
    float* out;        // m x p
    const void* B16 = nullptr;   // bfloat16 plans: B (n x p), V^T (k x n), U S (m x k)
    const void* Vt16 = nullptr;
    const void* US16 = nullptr;
  };
  amm_ctx* ctx = nullptr;
  int k = 0;
  bool bf16 = false;            // bfloat16 components, float32 accumulation
  bool launches = false;        // circulant entries: one product launch sequence per entry
  std::vector<const amm_dec*> decs;
  amm::DevBuf fac16;            // plan-owned bfloat16 factor copies
  std::vector<Item> items;
  std::vector<int> splits;
  int target_blocks = 0;
  int panel_blocks = 0, out_blocks = 0;
  amm::DevBuf partials, tables;
  amm::DevBuf gsplit;           // bfloat16 plans: hi and lo parts of every G^T
  void* pjobs = nullptr;
  void* ojobs = nullptr;
  void* rjobs = nullptr;
  int* pstart = nullptr;
  int* ostart = nullptr;
  int* rstart = nullptr;
  int red_blocks = 0;
  // circulant plans: batched launches over a job table, one per (side,
  // list precision, accumulation phase) group, and the entries they do not
  // cover (other sides) launched one by one
  struct CircGroup {
    int log2n;
    bool h16;
    int first_job, njobs, tiles;
  };
  std::vector<amm::CdJob> cjobs_host;
  std::vector<CircGroup> cgroups;
  std::vector<int> cloose;
  amm::DevBuf cjobs;
  int circ_mode = 0;            // 0: every entry launched by itself; 1: the job-table launches
  double circ_ms[2] = {-1.0, -1.0};   // tuner's time of one run in each mode (-1: not timed)
  bool from_cache = false;      // the tuned choice came from the context's tune cache
  hipStream_t own = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double tuned_ms = 0.0;
  ~amm_batch_plan();
};

namespace amm {

// ---- kernel launchers (defined in the .hip files) ---------------------------
amm_status twiddles32(amm_ctx* ctx, int log2n, const float2** out);
amm_status twiddles64(amm_ctx* ctx, int log2n, const double2** out);

// Circulant product through the fused LDS FFT kernel.
//  column mode: out (n x p) [+]= Atil B, B (n x p) row-major, along columns.
//  row mode:    out (rows x n) [+]= X Btil^T-side operator applied to each
//               row of X (rows x n):  out_row = (op(row^T))^T.
// L16 (optional, n >= 1024): the lists as float16 pairs scaled by a power of
// two (l16_inv = its inverse); the spectral products then run in float16 with
// float32 sums (see cd_apply_kernel).
// ldb, ldo: row pitches of B and out in floats (0 = p).
amm_status cd_apply_columns(amm_ctx* ctx, int log2n, int K, const int32_t* shifts,
                            const float2* L, const float* B, int64_t p, float* out,
                            bool accumulate, hipStream_t s, CdPairs pr = CdPairs{},
                            const __half2* L16 = nullptr, float l16_inv = 1.0f, int64_t ldb = 0,
                            int64_t ldo = 0);
// Batched column-mode products over a job table (device memory, sorted by
// tile0, covering workgroups 0 .. tiles - 1); cd_tile_columns: real columns
// per workgroup at side 2^log2n (0 outside 64 .. 16384).
amm_status cd_apply_jobs(amm_ctx* ctx, int log2n, bool h16, const CdJob* jobs, int njobs, int tiles, hipStream_t s);
int cd_tile_columns(int log2n);
amm_status cd_apply_rows(amm_ctx* ctx, int log2n, int K, const int32_t* shifts,
                         const float2* L, const float* X, int64_t rows, float* out,
                         bool accumulate, hipStream_t s, CdPairs pr = CdPairs{},
                         const __half2* L16 = nullptr, float l16_inv = 1.0f);

// Forward spectra of the packed column pairs of B (n x p, p even): spec
// (n x p floats) holds complex bin values at [p][2c], [p][2c + 1].
amm_status cd_spectrum_columns(amm_ctx* ctx, int log2n, const float* B, int64_t p, float* spec,
                               hipStream_t s);

// Circulant decomposition, float64 on the device.
// Builds dec->pair_buf from host copies of the lists when the frequency set
// is closed and the lists satisfy L_{n-k}[p] = conj(L_k[-p]).
amm_status cd_build_pairs(amm_dec* dec, const std::vector<float2>& L_host);
// The same with the lists on the device only (the mirror test and the
// largest list component |x|, |y| computed there; *mx receives the latter).
amm_status cd_build_pairs_dev(amm_dec* dec, float* mx, hipStream_t s);
// The table builder shared by both: mirror(pass, ta, tb) is the list test.
amm_status cd_pair_tables(amm_dec* d, const std::function<bool(int, int, int)>& mirror);

// float16 copies of dec->L and dec->Ladj (host copy of L given) with a
// power-of-two scale; sets dec->fp16 and dec->l16_inv.
amm_status cd_make_half_lists(amm_dec* dec, const std::vector<float2>& L_host, hipStream_t s);
// the same given the largest list component
amm_status cd_make_half_lists_mx(amm_dec* dec, float mx, hipStream_t s);

amm_status cd_decompose(amm_ctx* ctx, const float* A, int n, int K,
                        bool keep_residual, amm_dec* dec, hipStream_t s, bool fp16 = false);

// Any-length float64 DFT of `batch` vectors in place (element e of vector b
// at b*bs + e*es), sign -1: exp(-2 pi i jk/n); result times `scale`.
// Lengths that are not powers of two go through Bluestein's chirp convolution.
// sync = false leaves the work queued on s (the chirp-convolution products,
// whose results only kernels on s read)
amm_status dft64_any(amm_ctx* ctx, double2* x, int n, int64_t es, int64_t bs, int64_t batch, int sign, double scale,
                     hipStream_t s, bool sync = true);
// Circulant products for sizes that are not powers of two (float64 steps):
// out (n x p) (+)= Atil B, and out (rows x n) (+)= X Btil with the adjoint lists.
// Circulant products for sides that are not powers of two: fused float32
// chirp-convolution kernel up to kChirpFusedMax, float64 steps above.
constexpr int kChirpFusedMax = 2048;
// [ch (n) | H_fwd / M (M) | H_inv / M (M)] in float32, M = 2^ceil(log2(2n - 1)), cached per n
amm_status chirp_tables32(amm_ctx* ctx, int n, hipStream_t s, const float2** tab);
// L16 (optional, n >= 1024): the lists as float16 pairs scaled by 1 / l16_inv,
// widened on load (float32 products)
amm_status cd_chirp_apply(amm_ctx* ctx, bool rows, int n, int K, const int32_t* shifts, const float2* L,
                          const float* X, int64_t extent, float* out, bool accumulate, hipStream_t s,
                          const __half2* L16 = nullptr, float l16_inv = 1.0f);
amm_status cd_apply_general(amm_ctx* ctx, int n, int K, const int32_t* shifts, const float2* L, const float* B,
                            int64_t p, float* out, bool acc, hipStream_t s, const __half2* L16 = nullptr,
                            float l16_inv = 1.0f);
amm_status spectrum_columns_general(amm_ctx* ctx, int n, const float* B, int64_t p, float* X, hipStream_t s);
amm_status cd_apply_rows_general(amm_ctx* ctx, int n, int K, const int32_t* shifts_adj, const float2* Ladj,
                                 const float* X, int64_t rows, float* out, bool acc, hipStream_t s,
                                 const __half2* Ladj16 = nullptr, float l16_inv = 1.0f);

// Float64 Stockham FFT over `batch` vectors of length 2^log2n (element e of
// vector b at b*bs + e*es); sign -1: exp(-2 pi i jk/n), +1: its conjugate;
// `scale` multiplies the result, which ends in `cur` (buffers swapped).
amm_status fft64_transform(double2*& cur, double2*& tmp, int log2n, int64_t es, int64_t bs, int64_t batch,
                           bool batch_fast, int sign, double scale, const double2* tw, hipStream_t s, const float* real_src = nullptr);


// Dense float32 GEMM on MFMA: C = alpha * op(A) op(B) + beta * C, with
// general element strides (row-major or transposed views).
struct MatView {
  const float* p;
  int64_t rs, cs;  // element (i, j) at p[i*rs + j*cs]
};
amm_status gemm_f32(int64_t M, int64_t N, int64_t Kd, float alpha, MatView A, MatView B,
                    float beta, float* C, int64_t ldc, hipStream_t s, const char* tag = "gemm_f32");
amm_status gemm_f64(int64_t M, int64_t N, int64_t Kd, double alpha, const double* A,
                    int64_t a_rs, int64_t a_cs, const double* B, int64_t b_rs,
                    int64_t b_cs, double beta, double* C, int64_t ldc, hipStream_t s);

// SVD path: skinny panels and the short-K output GEMM (tsvd_apply.hip)
bool tsvd_fast_shapes(int64_t m, int64_t n, int64_t p, int ka, int kb);
bool tsvd_split_shapes(int64_t m, int64_t n, int64_t p, int ka, int kb);
size_t tsvd_split_scratch(int64_t m, int64_t n, int64_t p, int ka, int kb);
// Fixed per-device scratch of amm_approx_matmul_static (floats).
constexpr size_t kStaticScratchFloats = size_t{8} << 20;   // 32 MiB
// Look up the device address of the fixed scratch on `device` (current);
// once per device, from amm_ctx_create.
void static_scratch_init(int device);
// Its device address on `device`, or an error if the lookup failed or never ran.
amm_status static_scratch(int device, float** out);
amm_status tsvd_split_product(int64_t m, int64_t n, int64_t p, int ka, int kb, const float* V_A, const float* US_A,
                              const float* Y, const float* X, const float* U_B, const float* VS_B, float* scratch,
                              size_t scratch_floats, float* out, hipStream_t s);
int tsvd_fast_splits(int64_t tiles, int64_t n);
amm_status tsvd_fast_product(int64_t m, int64_t n, int64_t p, int ka, int kb, const float* V_A,
                             const float* US_A, const float* Y, const float* X, const float* U_B,
                             const float* VSt_B, float* Gp, size_t gp_floats, float* H,
                             size_t h_floats, float* out, hipStream_t s);
// Skinny and short-K products on the matrix cores (shapes: see tsvd_apply.hip)
amm_status panel_full(int a, int64_t n_red, const float* X, const float* Y, int64_t ncols, float* C,
                      hipStream_t s);
bool panel_full_ok(int a, int64_t ncols);
amm_status gemm_short(int64_t M, int64_t N, int K, const float* A, const float* B, float* C, hipStream_t s);
bool gemm_short_ok(int64_t M, int64_t N, int K);
// Raw CSR x dense: out (rows x p) (+)= S B
// rows of S from row_ptr, or per block of 4096 inner indices from blk_ptr
// ((blocks + 1) offsets per row) when blocks > 1
// (ldb, ldo: row pitches of B and out in floats; 0 = p)
amm_status spmm_raw(const int32_t* row_ptr, const int32_t* col, const float* val, int64_t rows,
                    const float* B, int64_t p, float* out, bool accumulate, hipStream_t s,
                    const int32_t* blk_ptr = nullptr, int blocks = 1, int64_t ldb = 0, int64_t ldo = 0);

// Delta A = A - (U S) V^T into dst (m x n)
amm_status tsvd_residual(const float* A, int64_t m, int64_t n, int k, const float* US, const float* V,
                         float* dst, hipStream_t s);
amm_status tsvd_decompose(amm_ctx* ctx, const float* A, int64_t m, int64_t n, int k,
                          const amm_opts* o, amm_dec* dec, hipStream_t s);

// Fourier-domain sparsification (sfft.hip)
bool sfft_left_ok(int64_t n);
amm_status sfft_decompose(amm_ctx* ctx, const float* A, int64_t m, int64_t n, int K, bool keep_residual, amm_dec* d,
                          hipStream_t s);
amm_status sfft_left_apply(amm_ctx* ctx, const amm_dec* d, const float* B, int64_t p, float* out, bool acc,
                           hipStream_t s);
amm_status sfft_first_order_term(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, float* out, hipStream_t s);

// Sparse path
amm_status sparse_extract(amm_ctx* ctx, const float* A, int64_t m, int64_t n, int64_t nnz,
                          amm_dec* dec, float* R_out, hipStream_t s);
// out (m x p, contiguous) (+)= S B, B with row pitch ldb (floats); with
// `add` (row pitch ld_add; float4-aligned operands only) out = S B + add
amm_status spmm_csr(const amm_dec* d, const float* B, int64_t ldb, int64_t p, float* out, bool accumulate,
                    hipStream_t s, const float* add = nullptr, int64_t ld_add = 0, int64_t ldo = 0);
amm_status dense_times_csr(amm_ctx* ctx, const float* X, int64_t rows, const amm_dec* d, float* out,
                           bool accumulate, hipStream_t s);

amm_status fill_f32(float* p, int64_t count, float v, hipStream_t s);
// out (cols x rows) (+)= Y^T for Y (rows x cols)
amm_status transpose_acc_f32(const float* Y, int64_t rows, int64_t cols, float* out, bool accumulate,
                             hipStream_t s);
// sum of squares of count floats, accumulated in float64 (synchronises s)
amm_status sumsq_f32(const float* x, int64_t count, hipStream_t s, double* out);
// l x l steps of the randomized SVD on the device (rsvd_small.hip)
constexpr int kSmallEigMax = 96;
amm_status chol_qr_factor(const double* gram, int l, int64_t rows, int mode, double* rinv, int* status,
                          hipStream_t s);
amm_status gram_eig(const double* gram, int l, int64_t rows, int k, double* W, int32_t* perm, double* isg,
                    double* sgk, float* sigma_f, double* sig_sorted, int* status, hipStream_t s);
// larger sketches: blocked CholeskyQR (E: chol_blocks(l) blocks of 64 x 64,
// P: l x 64) and block one-sided Jacobi on the Cholesky factor (one launch
// per round of block pairs)
int chol_blocks(int l);
amm_status chol_qr_blocked(double* G, int l, int64_t rows, bool shift, double* R, double* E, int* status,
                           hipStream_t s, double* shift_out = nullptr);
amm_status chol_qr_apply(const double* Y, int64_t rows, int l, const double* R, const double* E, double* Q, double* P,
                         hipStream_t s);
amm_status gram_eig_large(double* G, int l, int64_t rows, double* R, double* E, double* W, double* dev, int* flag,
                          int* status, std::vector<double>& lam_host, int* sweeps_out, hipStream_t s);
// ||x - y||_F^2 and ||x||_F^2 of count floats, float64 (synchronises s)
amm_status diff_sumsq_f32(const float* x, const float* y, int64_t count, hipStream_t s, double* dd, double* xx);
amm_status transpose_f32(const float* src, int64_t rows, int64_t cols, float* dst, hipStream_t s);
// the same with row pitches (floats) on both sides
amm_status transpose_ld_f32(const float* src, int64_t ld_src, int64_t rows, int64_t cols, float* dst,
                            int64_t ld_dst, hipStream_t s);
amm_status transpose_acc_ld_f32(const float* Y, int64_t ldy, int64_t rows, int64_t cols, float* out, int64_t ldo,
                                bool accumulate, hipStream_t s);
// Row pitch for a scratch copy of a matrix with `cols` columns that spreads a
// column slice's rows over the L2 channels (cols + 64 for multiples of 2048).
int64_t spread_pitch(int64_t cols);
// dst (rows x cols, row pitch ld_dst) = src (rows x cols, contiguous); float4 aligned
// Element-wise copy between row-major matrices of element types
// AMM_F32 / AMM_BF16 / AMM_F16 (widening exact, narrowing rounds to nearest even).
amm_status cast_matrix(const void* src, int src_dtype, int64_t src_ld, int64_t rows, int64_t cols, void* dst,
                       int dst_dtype, int64_t dst_ld, hipStream_t s);
amm_status repitch_f32(const float* src, int64_t ld_src, int64_t rows, int64_t cols, float* dst, int64_t ld_dst,
                       hipStream_t s);
amm_status approx_backward(amm_ctx* ctx, const amm_dec* d, const float* X, const float* dY, int64_t p,
                           float* dX, float* dW, hipStream_t s);
// Batched truncated-SVD products (tsvd_apply.hip)
amm_status batch_build(amm_batch_plan* bp, int target_blocks);
amm_status batch_launch(amm_batch_plan* bp, hipStream_t s);
bool batch_item_ok(int64_t m, int64_t n, int64_t p, int k);
int batch_max_items();
bool batch_item_ok_bf16(int64_t m, int64_t n, int64_t p, int k);
amm_status batch_convert_bf16(amm_batch_plan* bp, const std::vector<const float*>& V,
                              const std::vector<const float*>& US, hipStream_t s);
amm_status batch_build_bf16(amm_batch_plan* bp, int target_blocks);
amm_status batch_launch_bf16(const amm_batch_plan* bp, hipStream_t s);
// Build the CSC copy of a CSR part held on the device (host transpose).
// column-major copy of a sparse part and the block ranges of both (csc_build.hip)
constexpr int64_t kSpBlock = 4096;   // inner indices per block of a blocked sparse product
amm_status build_csc(amm_dec* d, hipStream_t s);

}  // namespace amm
