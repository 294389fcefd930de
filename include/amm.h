/*
 * amm.h -- approximate matrix multiplication from truncated decompositions,
 * MI355X (gfx950) library.  C ABI: every entry point is extern "C", takes plain
 * host or device pointers and sizes, and returns an amm_status.  No exception
 * crosses the ABI.  A non-OK status leaves every output untouched and sets a
 * thread-local message readable with amm_last_error().
 *
 * The operation (paper: "Efficient approximations of matrix multiplication
 * using truncated decompositions", Sec. 2.1, eq. (2.1)-(2.3)):
 *   A = Atil + Delta A,  B = Btil + Delta B,
 *   zeroth order  M0 = Atil B,
 *   first order   M1 = Atil B + Delta A Btil   (= AB - Delta A Delta B).
 * Atil is one of
 *   - a truncated circulant decomposition  sum_{k in S} R_k D^k  (Thm. 1.1,
 *     Alg. 2.2 / 2.3), applied through FFTs: FFT(B) -> sum_t diag(L_t) C^k_t
 *     -> one inverse FFT (Alg. 2.3 step 5);
 *   - a truncated SVD  U_k S_k V_k^T  (Sec. 2.2, Alg. 2.1), applied as
 *     U_k (S_k (V_k^T B));
 *   - a sparse part of dominant entries plus a truncated dense residue,
 *     S + trunc(A - S)  (eq. (2.4), abstract).
 *
 * Conventions shared by all calls
 *   - Matrices are row-major, contiguous (leading dimension = column count),
 *     float32, in device memory unless stated otherwise.
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     All device work of a call is enqueued on it.  amm_approx_matmul never
 *     synchronises the host; amm_decompose synchronises `stream` (it reads
 *     the per-frequency energies or the sketch back to pick components).
 *   - The caller owns A, B, out and the streams.  A decomposition handle owns
 *     its component buffers; it is immutable after creation and may be used
 *     from several streams, but must outlive the work enqueued with it.
 *   - Circulant decompositions take square operands (or square blocks) of
 *     side 2 <= n <= 16384.  Powers of two run the fused single-kernel
 *     product; other sides transform through Bluestein's chirp convolution:
 *     one fused float32 kernel up to n = 2048 (float16 lists and batch
 *     plans included), float64 steps above.
 */
#ifndef AMM_H
#define AMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amm_ctx amm_ctx;
typedef struct amm_dec amm_dec;
typedef struct amm_batch_plan amm_batch_plan;

typedef enum {
  AMM_OK = 0,
  AMM_EINVAL = 1,       /* NULL pointer, negative size, bad enum value */
  AMM_ESHAPE = 2,       /* operand shapes do not conform */
  AMM_EUNSUPPORTED = 3, /* valid request outside what the GPU path covers */
  AMM_ENOMEM = 4,       /* device allocation failed */
  AMM_EDEVICE = 5,      /* a HIP call failed; message holds hipGetErrorString */
  AMM_ESTATE = 6        /* handle in the wrong state (e.g. no residual kept) */
} amm_status;

/* Decomposition kinds. AMM_SPARSE may be OR-ed with AMM_CIRCULANT or
 * AMM_TSVD, which then truncates the dense residue A - S. */
enum { AMM_CIRCULANT = 1, AMM_TSVD = 2, AMM_SPARSE = 4, AMM_SFFT = 8 };

/* Element types of described operands. */
enum { AMM_F32 = 0, AMM_BF16 = 1, AMM_F16 = 2 };

/* A row-major device matrix: element (r, c) at data + (r ld + c) elements
 * of `dtype`; ld >= cols.  The caller owns the memory. */
typedef struct {
  void* data;
  int64_t rows, cols, ld;
  int dtype;
} amm_matrix;

typedef struct {
  double sparse_frac;  /* AMM_SPARSE: keep round(frac*m*n) entries of largest |a| */
  int64_t sparse_nnz;  /* AMM_SPARSE: if >= 0, overrides sparse_frac */
  int oversample;      /* AMM_TSVD: extra sketch columns (default 16) */
  int power_iters;     /* AMM_TSVD: subspace iterations (default 2) */
  uint64_t seed;       /* AMM_TSVD: counter-based sketch seed (Philox4x32-10) */
  int keep_residual;   /* keep Delta A on the device so that this handle can
                          be the left operand of a first-order product */
  int spectral_fp16;   /* AMM_CIRCULANT with n >= 1024 (a power of two, or at
                          most 2048): float16 spectral products (Alg. 2.3
                          step 5 with half-precision multiplicands).  The
                          eigenvalue lists are stored as float16 pairs scaled
                          by a power of two; powers of two also round each
                          tile's forward spectrum to float16 (scaled by a
                          power of two per tile) and form every list-times-
                          spectrum product in half precision with float32
                          sums; both FFTs and the output stay float32.
                          Other sides widen the float16 lists and multiply in
                          float32.  Each multiplicand carries a relative
                          rounding of 2^-11, so the circulant term differs
                          from its float32 value by about 1e-3 relative
                          (default 0) */
} amm_opts;

/* Fill `o` with the defaults (frac 0.01, nnz -1, oversample 16, power 2,
 * seed 0, keep_residual 1, spectral_fp16 0). */
void amm_opts_default(amm_opts* o);

typedef struct {
  int kind;              /* AMM_CIRCULANT / AMM_TSVD, possibly | AMM_SPARSE */
  int64_t m, n;          /* operand shape */
  int K;                 /* requested components (frequencies or rank) */
  int K_eff;             /* components kept (circulant: K or K-1, pairs closed) */
  int64_t nnz;           /* sparse entries (0 if not sparse) */
  int has_residual;      /* Delta A available for first-order use */
  double norm_A;         /* ||A||_F  (float64) */
  double norm_residual;  /* ||Delta A||_F from the dropped energy/spectrum
                            (blocked operands: over the zero-padded blocks) */
  int blocks;            /* square circulant blocks of a rectangular operand (0: none) */
  int spectral_fp16;     /* circulant products use float16 spectral products */
  double mu;             /* circulant: spectral concentration of Delta A (see
                            amm_estimate_error); NaN if not computed */
  double sigma_next;     /* truncated SVD: sigma_{k+1} estimate (= ||Delta A||_2);
                            NaN if unknown */
} amm_dec_info;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` (made current for the call).
 * Owns per-size twiddle tables and grow-only work areas; not thread-safe.
 * Calls on one context share its work areas, so calls enqueued on different
 * streams must be ordered by the caller (or use one context per stream);
 * contexts never share work areas with each other. */
amm_status amm_ctx_create(amm_ctx** ctx, int device);

/* Debug mode (also on when the environment variable AMM_DEBUG is set to
 * anything but "0" at context creation): every product, gradient,
 * decomposition and batch run of the context first checks that the matrix
 * pointers it is given are device memory of the context's device
 * (AMM_EINVAL otherwise, before any launch), and afterwards synchronises
 * its stream, so a device fault is reported by the call that caused it
 * (AMM_EDEVICE).  Costs a host round trip per call. */
amm_status amm_ctx_set_debug(amm_ctx* ctx, int enable);

/* Tune cache: batch plans of this context look their tuned choice (the
 * split target of a truncated-SVD plan, the schedule of a circulant plan) up
 * in the text file `path`, keyed by the device's architecture and compute
 * units and every entry's shape, rank or kept frequencies and list
 * precision, and skip their timing runs on a hit; a miss tunes and appends
 * one line.  NULL or "" turns it off (the default unless AMM_TUNE_CACHE is
 * set at context creation).  A file that cannot be read or written only
 * disables the cache.  Processes may share one file (single-line appends). */
amm_status amm_ctx_set_tune_cache(amm_ctx* ctx, const char* path);
void amm_ctx_destroy(amm_ctx* ctx);

/* Device allocator supplied by the caller (e.g. a framework's caching
 * allocator): alloc returns `bytes` of device memory on `device` (NULL on
 * failure, reported as AMM_ENOMEM), free returns it.  Both must be callable
 * from the thread that calls the library and stay valid while any buffer they
 * made lives: until the context and every handle and plan made on it are
 * destroyed.  free can be called while work queued earlier on the call's
 * stream still reads the buffer (a work area grown inside a call, a handle
 * destroyed after its last product was queued): the allocator must reuse
 * memory in stream order (as torch's caching allocator does for the stream
 * the library launches on) or wait for the device itself. */
typedef struct {
  void* (*alloc)(size_t bytes, int device, void* user);
  void (*free)(void* ptr, size_t bytes, int device, void* user);
  void* user;
} amm_allocator;

/* amm_ctx_create with every device buffer of the context, of the handles and
 * plans made on it (component buffers, work areas, tables) taken from
 * `alloc` instead of hipMalloc.  alloc == NULL: as amm_ctx_create.  The
 * structure is copied.  The fixed scratch of amm_approx_matmul_static is
 * not an allocation and is unaffected. */
amm_status amm_ctx_create_with_allocator(amm_ctx** ctx, int device, const amm_allocator* alloc);

/* Per-launch timing for measurement.  With timing enabled, every kernel that
 * a call on `ctx` enqueues is bracketed by hipEventRecord on the same stream.
 * amm_ctx_timings waits for the recorded events, then reports per kernel name
 * the summed duration (ms) and launch count, and clears the totals.  With all
 * output pointers NULL it only reports *count (the number of names).
 * names: cap slots of name_len bytes each, NUL-terminated. */
amm_status amm_ctx_set_timing(amm_ctx* ctx, int enable);
amm_status amm_ctx_timings(amm_ctx* ctx, char* names, int name_len, double* total_ms,
                           int64_t* launches, int cap, int* count);

/* Message for the last non-OK status on this thread ("" if none). */
const char* amm_last_error(void);

/* ---- decomposition ------------------------------------------------------ */

/* Decompose the m x n float32 device matrix A.
 *  kind = AMM_CIRCULANT: for m != n, A is cut into square blocks of side
 *    s = min(m, n) along the longer dimension, the last
 *    block zero-padded (Sec. 2.3: rectangular matrices through square
 *    blocks), and each block is decomposed as below with its own K; such
 *    handles serve zeroth-order products only.  For each square operand it computes every circulant
 *    coefficient (Thm. 1.1 / Alg. 2.2) in float64 on the device through the
 *    two-sided transform F A F^-1, ranks the frequencies by energy
 *    ||R_k||_F^2 (Alg. 2.3 steps 2-3) and keeps the closed set of at most K
 *    frequencies {k, n-k} with the most energy, then stores the eigenvalue
 *    lists L_t = F r_{.,k_t} (Alg. 2.3 step 4).  With keep_residual it also
 *    keeps Delta A = A - sum_{t} R_t D^{k_t}  (Alg. 2.3 step 6) in float32.
 *  kind = AMM_TSVD: rank-K randomized SVD (Alg. 2.1, with oversampling and
 *    subspace iterations), float64 on the device; K <= min(m, n).  A zero
 *    operand gives K_eff = 0; an operand of rank below K keeps its extra
 *    components with singular values at rounding level.  With
 *    keep_residual it borrows A (see amm_dec_import_tsvd) -- the caller must
 *    keep A alive and unchanged while the handle is used as a left operand.
 *  kind = AMM_SFFT: Fourier-domain sparsification (Sec. 2.4, Alg. 2.4/2.5).
 *    With W the unitary DFT of the inner dimension, AB = (A W*)(W B).  As a
 *    left operand (2 <= n <= 16384) each row of A W* keeps its
 *    K dominant frequencies; as a right operand (2 <= m <= 16384) each column
 *    of W A keeps its K dominant frequencies.  Both are computed in float64 on
 *    the device (sizes that are not powers of two through Bluestein's chirp
 *    convolution); the kept sets are closed under q -> n-q (the most energy in
 *    at most K members, as for the circulant kind), which keeps products real.
 *    Stored: the kept entries in float32 (CSR by rows, and by columns as
 *    half-spectrum representatives), and with keep_residual the residual half
 *    spectrum of A W* ((n/2+1) x m, float32 complex).  Products need an even
 *    column count p; first order needs both operands of this kind.  Cannot be
 *    combined with AMM_SPARSE.
 *  kind |= AMM_SPARSE: first splits A = S + R with S the round(frac*m*n)
 *    entries of largest |a| (ties to the smaller row-major index), stored as
 *    CSR, then truncates R with the other kind (K may be 0 for none).
 * `opts` may be NULL (defaults).  On success *out owns a new handle. */
amm_status amm_decompose(amm_ctx* ctx, const float* A, int64_t m, int64_t n,
                         int kind, int K, const amm_opts* opts, void* stream,
                         amm_dec** out);

/* Import a circulant truncation computed elsewhere.
 *  freqs_host: K int32 frequencies in [0, n) (host).
 *  eig_host:   K x n complex float64, interleaved (re, im), row t holds
 *              L_t[p] = sum_j r_{j,k_t} exp(-2 pi i p j / n)  (host).
 *  residual:   optional n x n float32 Delta A on the device, copied.
 *  norm_A, norm_residual: stored for amm_dec_query (may be 0).
 * The set should be closed under k -> n-k for a real product. */
amm_status amm_dec_import_circulant(amm_ctx* ctx, int64_t n, int K,
                                    const int32_t* freqs_host,
                                    const double* eig_host,
                                    const float* residual, double norm_A,
                                    double norm_residual, amm_dec** out);

/* Import a truncated SVD: U (m x k), sigma (k), V (n x k), float64 host
 * arrays, row-major.  A (m x n, device) is optional and borrowed: it is needed
 * only when this handle is the left operand of a first-order product. */
amm_status amm_dec_import_tsvd(amm_ctx* ctx, int64_t m, int64_t n, int k,
                               const double* U_host, const double* sigma_host,
                               const double* V_host, const float* A,
                               amm_dec** out);

/* Import a sparse part (CSR on the host: row_ptr m+1, col nnz ascending per
 * row, val nnz) plus an optional truncated residue handle, whose ownership
 * passes to the new handle.  A (device, borrowed) as in amm_dec_import_tsvd.
 * Rows whose columns are not ascending are accepted (index range and row_ptr
 * are checked, AMM_EINVAL otherwise); products with them keep the one-pass
 * gather instead of the blocked one used when n > 8192, and sum a row's
 * entries in stored order. */
amm_status amm_dec_import_sparse(amm_ctx* ctx, int64_t m, int64_t n,
                                 int64_t nnz, const int32_t* row_ptr_host,
                                 const int32_t* col_host, const float* val_host,
                                 amm_dec* residue, const float* A,
                                 amm_dec** out);

amm_status amm_dec_query(const amm_dec* dec, amm_dec_info* info);

/* Block j of a rectangular circulant decomposition (a square circulant
 * handle of side min(m, n)), borrowed: valid while `dec` lives, never passed
 * to amm_dec_destroy. */
amm_status amm_dec_block(const amm_dec* dec, int j, const amm_dec** block);

/* Copy the kept circulant frequencies (ascending) to `out_host` (capacity
 * `cap`); *count receives K_eff. Circulant handles (or sparse ones with a
 * circulant residue) only. */
amm_status amm_dec_frequencies(const amm_dec* dec, int32_t* out_host, int cap,
                               int* count);

/* Copy the eigenvalue lists L_t = F r_{.,k_t} of a square circulant handle
 * (or the circulant residue of a sparse one) to the host: K_eff x n complex
 * values, interleaved (re, im), row t for the t-th frequency that
 * amm_dec_frequencies reports (Alg. 2.3 step 4).  The lists the products use
 * are float32; they are widened exactly, so amm_dec_import_circulant of these
 * values rebuilds the same float32 lists.  cap counts complex values. */
amm_status amm_dec_circulant_lists(const amm_dec* dec, double* eig_host, int64_t cap);

/* Copy the float64 per-frequency energies ||R_k||_F^2 (n values) of a
 * circulant decomposition made by amm_decompose to the host. */
amm_status amm_dec_energies(const amm_dec* dec, double* out_host, int64_t cap);

/* Copy the truncated-SVD factors as float32 (U m x k, sigma k, V n x k). */
amm_status amm_dec_tsvd_factors(const amm_dec* dec, float* U_host,
                                float* sigma_host, float* V_host);

/* Copy the sparse part (row_ptr m+1, col nnz, val nnz) to the host. */
amm_status amm_dec_sparse_part(const amm_dec* dec, int32_t* row_ptr_host,
                               int32_t* col_host, float* val_host);

/* Serialise a handle to a host buffer (a checkpoint of a decomposition made
 * offline, as the paper treats the weights' decomposition, Sec. 4.5; its
 * circulant lists, SVD factors and sparse arrays are the float32 values the
 * products use, with their derived tables).  buf == NULL: *bytes receives the
 * size needed.  Otherwise *bytes is buf's capacity (AMM_EINVAL if too small)
 * and receives the size written.  Device -> host copies; synchronous.  A
 * borrowed operand (A of a truncated SVD) is not included: pass it again to
 * amm_dec_import.  The blob is plain host bytes (same-endian hosts). */
amm_status amm_dec_export(const amm_dec* dec, void* buf, size_t* bytes);

/* Rebuild a handle from amm_dec_export's bytes on ctx's device: every buffer
 * is copied back verbatim, so products of the imported handle equal those of
 * the exported one bit for bit.  A (device, may be NULL) is borrowed again by
 * the nodes that borrowed an operand when exported (first-order left operands
 * of the truncated-SVD kind).  AMM_EINVAL on a malformed or truncated blob,
 * AMM_EUNSUPPORTED on another format version.  Synchronous. */
amm_status amm_dec_import(amm_ctx* ctx, const void* buf, size_t bytes, const float* A,
                          amm_dec** out);

void amm_dec_destroy(amm_dec* dec);

/* ---- product ------------------------------------------------------------ */

/* out (m x p) = Atil B                 when dB == NULL   (zeroth order)
 * out (m x p) = Atil B + Delta A Btil  when dB != NULL   (first order)
 * B is n x p on the device, dA describes an m x n operand.  dB must describe
 * B's own decomposition (n x p) and dA must hold Delta A (circulant:
 * keep_residual; SVD/sparse: borrowed A).  out is overwritten; it must not
 * alias B.  p == 0 is an empty product: AMM_OK, nothing is read or written
 * (B and out may then be NULL).  Nothing is allocated per call except the SVD
 * and sparse intermediates, which come from the context's reusable scratch. */
amm_status amm_approx_matmul(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB,
                             const float* B, int64_t n, int64_t p, float* out,
                             void* stream);

/* amm_approx_matmul on operands with row pitches (Alg. 2.3 step 5 and
 * eq. (2.1), (2.4) as above): B is n x p with row r at B + r ldb, out is
 * m x p with row r at out + r ldo, e.g. column panels of larger row-major
 * matrices.  ldb >= p and ldo >= p (AMM_ESHAPE otherwise); the two panels
 * may share no element (AMM_EINVAL; with equal pitches the test is exact, so
 * two column panels of one matrix are accepted, with different pitches the
 * address ranges must be disjoint); columns between p and the pitch are
 * neither read nor written.  ldb == ldo == p is amm_approx_matmul.  A zeroth-order
 * product of a circulant handle with n a power of two, and of a sparse
 * handle over such a circulant residue (16-byte aligned pointers, pitches and
 * p multiples of 4), reads and writes at the pitches directly; other
 * requests pass through packed copies in the context's scratch (one
 * device-to-device 2-D copy each way).  Same stream and error behaviour as
 * amm_approx_matmul. */
amm_status amm_approx_matmul_strided(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB,
                                     const float* B, int64_t n, int64_t p, int64_t ldb,
                                     float* out, int64_t ldo, void* stream);

/* amm_approx_matmul on described operands of any element type: B (n x p)
 * and out (m x p), each float32, bfloat16 or float16, with its own pitch.
 * The arithmetic is the float32 product's: 16-bit B is widened once into
 * the context's scratch (exactly: every bfloat16 and float16 value is a
 * float32 value), a 16-bit out receives the float32 result rounded once to
 * nearest even.  All-float32 operands take amm_approx_matmul_strided.
 * Shapes must conform (AMM_ESHAPE), dtype be one of the three (AMM_EINVAL),
 * and B and out must not overlap (AMM_EINVAL). */
amm_status amm_approx_matmul_ex(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, const amm_matrix* B,
                                const amm_matrix* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as amm_approx_matmul for truncated-SVD handles, through the split
 * path only (dA of rank 32 or 64 with dB NULL or of rank 32/64, or rank 128
 * with dB NULL or of rank 128; m, p and n multiples of 128).  Its
 * intermediates live in one fixed array of 32 MiB per device (8 Mi floats,
 * reserved on a device when the library's code is first loaded there -- at
 * the latest by amm_ctx_create, which looks up its address -- and held until
 * the process ends; the
 * request's need is (S_G + 1) k_A p + (S_H + 1) k_B m + 64 floats for the
 * split counts S the product picks), so the call allocates nothing and never
 * synchronises.  Larger needs return AMM_EUNSUPPORTED, other handle kinds
 * AMM_EUNSUPPORTED, a first-order request without A borrowed by dA or
 * Delta B kept by dB AMM_ESTATE, a device on which no context was created
 * AMM_ESTATE.  Every call on a device shares that device's array: calls that
 * overlap on one device (two streams, two threads) race and must be ordered
 * by the caller.  Nothing in the array needs to start at zero; each call
 * overwrites what it reads. */
amm_status amm_approx_matmul_static(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB,
                                    const float* B, int64_t n, int64_t p, float* out,
                                    void* stream);

/* ---- batches of products ---------------------------------------------------- */

/* Plan `count` zeroth-order products out_i = Atil_i B_i of truncated-SVD
 * handles that share one rank k (16, 32, 48, 64 or 128) -- e.g. the linear
 * layers of a model -- executed as two launches for the whole batch: one
 * covering every V_i^T B_i reduction and one covering every output tile.
 * Shapes: m_i and p_i multiples of 128, n_i a multiple of 4; up to 256
 * entries.  B[i] (n_i x p[i]) and out[i] (m_i x p[i]) are device pointers bound
 * to the plan: later runs read and write the same buffers (the caller keeps
 * them alive and does not overlap runs of one plan).  Creation times several
 * reduction-split policies on `stream` (out_i are written while tuning),
 * keeps the fastest, and captures the two launches in a HIP graph.
 * Circulant handles (square, or rectangular in square blocks; any mix of
 * sizes) plan instead the fused product launch(es) of each entry, with
 * plan-owned scratch and all twiddle (and chirp) tables created up front,
 * captured in one HIP graph; their sides are powers of two or at most 2048
 * (AMM_EUNSUPPORTED otherwise). */
amm_status amm_batch_plan_create(amm_ctx* ctx, int count, const amm_dec* const* dA,
                                 const float* const* B, const int64_t* p, float* const* out,
                                 void* stream, amm_batch_plan** plan);
/* The same plan with bfloat16 components and float32 accumulation: B[i] are
 * bfloat16 device matrices (n_i x p[i], row-major, caller-owned and bound to
 * the plan), the plan keeps bfloat16 copies V_i^T and U_i S_i of each
 * handle's factors (rounded to nearest even), and out[i] are float32.  The
 * intermediate V_i^T B_i is accumulated in float32 and enters the second
 * product as a hi + lo pair of bfloat16 values, so the rounding of the stored
 * components is the only bfloat16 loss.  Shapes: rank 32, 64 or 128, m_i and
 * p[i] multiples of 128, n_i a multiple of 32; up to 256 entries.
 * Circulant handles (all entries circulant, power-of-two sides or square
 * blocks of side 64 .. 16384): the batched launches read the bfloat16 B_i
 * directly and widen them exactly in the load, everything after is the
 * float32 (or float16-list) product of the float32 plan. */
amm_status amm_batch_plan_create_bf16(amm_ctx* ctx, int count, const amm_dec* const* dA,
                                      const void* const* B, const int64_t* p, float* const* out,
                                      void* stream, amm_batch_plan** plan);
/* Run the plan on `stream`; use_graph != 0 replays the captured graph
 * (ignored while the context has timing enabled: then the launches are
 * issued directly so that they can be timed). */
amm_status amm_batch_run(amm_batch_plan* plan, int use_graph, void* stream);
/* Chosen split policy (target workgroups), launch sizes and the tuned time
 * of one run in ms. */
amm_status amm_batch_info(const amm_batch_plan* plan, int* target_blocks, int* panel_blocks,
                          int* out_blocks, double* tuned_ms);
/* Circulant plans: the schedule the plan's tuner kept.  Power-of-two block
 * products with sides 64 .. 16384 can run as batched launches over a job
 * table (one launch per side, list precision and accumulation phase -- a
 * column-blocked operand's second and later blocks accumulate in later
 * phases), the rest one launch sequence per entry; the tuner times both
 * (a warm-up and three runs each) at plan creation and keeps the faster.
 * job_table: 1 if the job-table launches were kept; launches: kernel
 * launch sequences per run; entry_ms, table_ms: the tuner's time of one run
 * in each mode (-1 when not timed; bfloat16 plans time only the job table).
 * AMM_ESTATE for a truncated-SVD plan. */
amm_status amm_batch_circulant_schedule(const amm_batch_plan* plan, int* job_table, int* launches,
                                        double* entry_ms, double* table_ms);
/* Override the tuner: job_table 1 runs the batched launches (AMM_EUNSUPPORTED
 * if no entry is eligible), 0 every entry by itself (AMM_EUNSUPPORTED for a
 * bfloat16 plan); the plan's graph is captured again.  Waits for the plan's
 * own stream; work the caller enqueued with the old schedule may still run. */
amm_status amm_batch_circulant_set_mode(amm_batch_plan* plan, int job_table);
/* 1 if the plan's tuned choice came from the context's tune cache. */
amm_status amm_batch_tuned_from_cache(const amm_batch_plan* plan, int* from_cache);
void amm_batch_plan_destroy(amm_batch_plan* plan);

/* ---- backward ------------------------------------------------------------ */

/* Gradients of Y = Wtil X (Wtil: the truncation held by dW, m x n; X: n x p;
 * dY: m x p, all device float32) with the truncation structure frozen -- the
 * kept circulant frequencies, the singular subspaces U_k and V_k, and the
 * sparse pattern are constants, so Wtil = P(W) with P linear:
 *   dX  = Wtil^T dY          (n x p)   written when dX != NULL,
 *   dWo = P^T(dY X^T)        (m x n)   written when dWo != NULL.
 * For the circulant and SVD kinds P is an orthogonal projection (the
 * Frobenius orthogonality of the components, Rem. 1.2 of the paper; the
 * orthonormal singular subspaces), so P^T = P.  The circulant gradient is
 * formed from the column spectra of dY and X without the m x n product
 * dY X^T.  Circulant dWo needs p even.  Outputs are overwritten and must not
 * alias the inputs. */
/* amm_approx_matmul_backward on described operands of any element type
 * (see amm_approx_matmul_ex): X (n x p), dY (m x p), dX (n x p) and dWo
 * (m x n) each float32, bfloat16 or float16 with its own pitch; dX or dWo
 * may be NULL (not computed).  16-bit inputs are widened once, outputs are
 * the float32 gradients rounded once. */
amm_status amm_approx_matmul_backward_ex(amm_ctx* ctx, const amm_dec* dW, const amm_matrix* X,
                                         const amm_matrix* dY, const amm_matrix* dX,
                                         const amm_matrix* dW_out, void* stream);

amm_status amm_approx_matmul_backward(amm_ctx* ctx, const amm_dec* dW, const float* X,
                                      const float* dY, int64_t p, float* dX, float* dWo,
                                      void* stream);

/* ---- error estimates (Sec. 2.5 and Sec. 3) ------------------------------- */

/* Entry model for the a priori estimate (Thm. 3.6). */
enum {
  AMM_ENTRIES_SIGNED = 0,            /* mean-zero entries / Haar singular vectors */
  AMM_ENTRIES_UNSIGNED_UNIFORM = 1   /* entries U(0, a) */
};

/* Estimates of the relative error ||AB - M||_F / ||AB||_F = ||Delta A Delta B||_F / ||AB||_F
 * of the first-order product M = Atil B + Delta A Btil (eq. (2.1)), n the inner
 * dimension.  Fields that cannot be formed are NaN. */
typedef struct {
  double norm_A, norm_B;     /* ||A||_F, ||B||_F as held by the handles */
  double norm_dA, norm_dB;   /* ||Delta A||_F, ||Delta B||_F */
  double norm_M;             /* ||M||_F of the given product (float64 sum) */
  double prior;              /* Thm. 3.6 without its vanishing term: ||dA|| ||dB|| / (||A|| ||B||),
                                times 4 / (3 sqrt(n)) for AMM_ENTRIES_UNSIGNED_UNIFORM */
  double posterior;          /* Cor. 3.7: ||dA|| ||dB|| / (sqrt(n) ||M||) */
  double svd_bound;          /* Thm. 3.8 over ||M||: sqrt(||dA||_2 ||dB||_2 ||dA|| ||dB||) / ||M||,
                                both operands truncated SVDs (plain or as the residue of a sparse
                                split) with ||dA||_2 = sigma_next.  For exact factors ||M|| <= ||AB||
                                (proof of Cor. 3.7), so this bounds the relative error */
  double cd_estimate;        /* circulant residual theorem of Sec. 3 over ||M||:
                                (mu_A mu_B)^(1/4) ||dA|| ||dB|| / (sqrt(n) ||M||), both operands square
                                circulant.  Its inequality does not hold for every input, so it is an
                                estimate, not a bound */
  double spec_dA, spec_dB;   /* sigma_next of the two truncated SVDs */
  double mu_A, mu_B;         /* circulant concentration: mu = max_i X_i / (||dA||_F^2 / n),
                                X_i = sum over dropped k of |lambda_i(R_k)|^2 */
} amm_error_estimate;

/* Fill *out from the norms and statistics the handles carry (decomposed
 * handles, circulant imports with their norms, truncated-SVD imports with A);
 * with M (m x p float32, device, the product of dA and dB) also ||M||_F and the
 * estimates that divide by it.  Synchronises `stream` when M is given.
 * Errors: AMM_ESHAPE if dA->n != dB->m or M's shape differs from the product. */
amm_status amm_estimate_error(amm_ctx* ctx, const amm_dec* dA, const amm_dec* dB, const float* M, int64_t m,
                              int64_t p, int entries, void* stream, amm_error_estimate* out);

/* Randomized estimate of the relative error (Sec. 2.5, last item):
 *   *est = ||A (B G) - M G||_F / ||A (B G)||_F
 * A (m x n), B (n x p), M (m x p) and the sketch G (p x l, N(0, 1) or
 * Rademacher entries drawn by the caller) are float32 row-major device arrays.
 * The three products run on the matrix cores in float32, the norms in float64;
 * the cost is 2 l (n p + m n + m p) flops.  Synchronises `stream`. */
amm_status amm_estimate_sketch(amm_ctx* ctx, const float* A, const float* B, const float* M, const float* G,
                               int64_t m, int64_t n, int64_t p, int64_t l, void* stream, double* est);

/* The smallest truncation K (the same for A and B) whose a priori estimate
 * (Thm. 3.6, as in amm_estimate_error) is <= tau (Sec. 2.5: add components
 * while the estimate is not small enough).  Two square circulant handles made
 * by amm_decompose: any K in [0, n], from their n energies and the pair-closed
 * selection (||Delta A(K)||^2 = sum E - retained(K)); decompose again with the
 * returned K.  Two truncated-SVD handles: K <= min(k_A, k_B) from the kept
 * singular values (||Delta A(k)||^2 = ||A||^2 - sum_{i<k} sigma_i^2); returns
 * that maximum when no smaller rank meets tau.  Host work only. */
amm_status amm_choose_rank(const amm_dec* dA, const amm_dec* dB, double tau, int entries, int* K);

/* Switch float16 spectral products (see amm_opts.spectral_fp16) on or off
 * for a circulant handle (or the circulant residue of a sparse handle; every
 * block of a rectangular one), e.g. after amm_dec_import_circulant.  Builds
 * the scaled float16 lists from the float32 ones on the handle's device
 * (synchronous); call it before the handle is used in enqueued work.
 * AMM_EUNSUPPORTED for sides below 1024 or, not powers of two, above 2048. */
amm_status amm_dec_set_spectral_fp16(amm_dec* dec, int enable);

/* Record sigma_{k+1} (>= 0) for an imported truncated SVD whose next singular
 * value the caller knows (decomposed handles carry their sketch's estimate). */
amm_status amm_dec_set_sigma_next(amm_dec* dec, double sigma_next);

#ifdef __cplusplus
}
#endif
#endif /* AMM_H */
