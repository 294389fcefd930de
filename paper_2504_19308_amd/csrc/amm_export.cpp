// Export and import of decomposition handles (host code).
//
// A handle is written as a self-contained blob: a header, then the root node
// and, recursively, its truncated residue (sparse handles) and its square
// blocks (rectangular circulant handles).  A node holds the scalar state of
// the handle and every device buffer the products read, copied verbatim
// (float32 lists, factors and sparse arrays exactly as the products use them,
// the derived tables included), so an imported handle gives the same products
// as the exported one, bit for bit.  A borrowed operand (A of a truncated SVD
// used as the left operand of a first-order product) is not part of the blob;
// the import takes it again.
#include <cstring>
#include <vector>

#include "amm_internal.hpp"

using namespace amm;

namespace {

constexpr uint32_t kMagic = 0x584d4d41u;   // "AMMX"
constexpr uint32_t kVersion = 1;

enum : uint32_t {
  F_FP16 = 1u << 0,
  F_ENERGIES = 1u << 1,
  F_BLOCK_ROWS = 1u << 2,
  F_SF_LEFT = 1u << 3,
  F_SF_RIGHT = 1u << 4,
  F_BORROWED_A = 1u << 5,
  F_INNER = 1u << 6,
};

// the device buffers of a node, in a fixed order (the tag is the index)
std::vector<DevBuf*> buffers_of(amm_dec* d) {
  return {&d->shifts, &d->shifts_adj, &d->L,       &d->Ladj,    &d->energies, &d->L16,     &d->Ladj16,
          &d->pair_buf, &d->U,        &d->V,       &d->sigma,   &d->US,       &d->VS,      &d->VSt,
          &d->Vt,       &d->row_ptr,  &d->col,     &d->val,     &d->csc_ptr,  &d->csc_row, &d->csc_val,
          &d->csr_blk,  &d->csc_blk,  &d->residual, &d->sf_rptr, &d->sf_ridx, &d->sf_rval, &d->sf_Rt,
          &d->sf_cptr,  &d->sf_cidx,  &d->sf_cval};
}

struct Writer {
  std::vector<unsigned char> out;
  template <typename T> void put(const T& v) {
    const auto* p = reinterpret_cast<const unsigned char*>(&v);
    out.insert(out.end(), p, p + sizeof(T));
  }
  void bytes(const void* p, size_t n) {
    const auto* c = static_cast<const unsigned char*>(p);
    out.insert(out.end(), c, c + n);
  }
};

struct Reader {
  const unsigned char* p;
  size_t left;
  bool ok = true;
  template <typename T> T get() {
    T v{};
    if (left < sizeof(T)) {
      ok = false;
      return v;
    }
    std::memcpy(&v, p, sizeof(T));
    p += sizeof(T);
    left -= sizeof(T);
    return v;
  }
  const unsigned char* take(size_t n) {
    if (left < n) {
      ok = false;
      return nullptr;
    }
    const unsigned char* q = p;
    p += n;
    left -= n;
    return q;
  }
};

amm_status write_node(const amm_dec* dc, Writer& w) {
  amm_dec* d = const_cast<amm_dec*>(dc);   // only read
  uint32_t flags = 0;
  if (d->fp16) flags |= F_FP16;
  if (d->has_energies) flags |= F_ENERGIES;
  if (d->block_rows) flags |= F_BLOCK_ROWS;
  if (d->sf_left) flags |= F_SF_LEFT;
  if (d->sf_right) flags |= F_SF_RIGHT;
  if (d->A_borrowed) flags |= F_BORROWED_A;
  if (d->inner) flags |= F_INNER;
  w.put<int32_t>(d->kind);
  w.put<int32_t>(d->K);
  w.put<int32_t>(d->K_eff);
  w.put<uint32_t>(flags);
  w.put<int64_t>(d->m);
  w.put<int64_t>(d->n);
  w.put<int64_t>(d->nnz);
  w.put<double>(d->norm_A);
  w.put<double>(d->norm_residual);
  w.put<double>(d->mu);
  w.put<double>(d->sigma_next);
  w.put<float>(d->l16_inv);
  w.put<int32_t>(d->npairs);
  w.put<int32_t>(d->nsingles);
  w.put<int32_t>(d->npairs_adj);
  w.put<int32_t>(d->nsingles_adj);
  w.put<int32_t>(d->csr_blocks);
  w.put<int32_t>(d->csc_blocks);
  w.put<int32_t>((int32_t)d->blocks.size());
  w.put<uint64_t>(d->sigma64.size());
  w.bytes(d->sigma64.data(), d->sigma64.size() * sizeof(double));
  w.put<uint64_t>(d->freqs.size());
  w.bytes(d->freqs.data(), d->freqs.size() * sizeof(int32_t));
  const auto bufs = buffers_of(d);
  uint32_t nb = 0;
  for (DevBuf* b : bufs) nb += b->ptr ? 1 : 0;
  w.put<uint32_t>(nb);
  std::vector<unsigned char> host;
  for (uint32_t tag = 0; tag < bufs.size(); ++tag) {
    const DevBuf* b = bufs[tag];
    if (!b->ptr) continue;
    w.put<uint32_t>(tag);
    w.put<uint64_t>(b->bytes);
    host.resize(b->bytes);
    AMM_HIP(hipMemcpy(host.data(), b->ptr, b->bytes, hipMemcpyDeviceToHost));
    w.bytes(host.data(), b->bytes);
  }
  if (d->inner) AMM_TRY(write_node(d->inner, w));
  for (const amm_dec* b : d->blocks) AMM_TRY(write_node(b, w));
  return AMM_OK;
}

amm_status read_node(Reader& r, int device, const float* A, amm_dec** out, int depth) {
  if (depth > 4) return fail(AMM_EINVAL, "decomposition blob nests too deep");
  amm_dec* d = new amm_dec();
  d->device = device;
  auto bad = [&](const char* what) {
    delete d;
    return fail(AMM_EINVAL, "decomposition blob: %s", what);
  };
  d->kind = r.get<int32_t>();
  d->K = r.get<int32_t>();
  d->K_eff = r.get<int32_t>();
  const uint32_t flags = r.get<uint32_t>();
  d->m = r.get<int64_t>();
  d->n = r.get<int64_t>();
  d->nnz = r.get<int64_t>();
  d->norm_A = r.get<double>();
  d->norm_residual = r.get<double>();
  d->mu = r.get<double>();
  d->sigma_next = r.get<double>();
  d->l16_inv = r.get<float>();
  d->npairs = r.get<int32_t>();
  d->nsingles = r.get<int32_t>();
  d->npairs_adj = r.get<int32_t>();
  d->nsingles_adj = r.get<int32_t>();
  d->csr_blocks = r.get<int32_t>();
  d->csc_blocks = r.get<int32_t>();
  const int32_t nblocks = r.get<int32_t>();
  const uint64_t ns = r.get<uint64_t>();
  if (!r.ok || ns > r.left / sizeof(double)) return bad("truncated header");
  d->sigma64.resize(ns);
  if (ns) std::memcpy(d->sigma64.data(), r.take(ns * sizeof(double)), ns * sizeof(double));
  const uint64_t nf = r.get<uint64_t>();
  if (!r.ok || nf > r.left / sizeof(int32_t)) return bad("truncated frequency list");
  d->freqs.resize(nf);
  if (nf) std::memcpy(d->freqs.data(), r.take(nf * sizeof(int32_t)), nf * sizeof(int32_t));
  const int base = d->kind & ~AMM_SPARSE;
  if (d->kind <= 0 || (base != 0 && base != AMM_CIRCULANT && base != AMM_TSVD && base != AMM_SFFT) ||
      d->m <= 0 || d->n <= 0 || d->K_eff < 0 || nblocks < 0 || nblocks > 1024)
    return bad("bad node header");
  d->fp16 = (flags & F_FP16) != 0;
  d->has_energies = (flags & F_ENERGIES) != 0;
  d->block_rows = (flags & F_BLOCK_ROWS) != 0;
  d->sf_left = (flags & F_SF_LEFT) != 0;
  d->sf_right = (flags & F_SF_RIGHT) != 0;
  if (flags & F_BORROWED_A) d->A_borrowed = A;
  const auto bufs = buffers_of(d);
  const uint32_t nb = r.get<uint32_t>();
  if (!r.ok || nb > bufs.size()) return bad("bad buffer count");
  for (uint32_t i = 0; i < nb; ++i) {
    const uint32_t tag = r.get<uint32_t>();
    const uint64_t bytes = r.get<uint64_t>();
    if (!r.ok || tag >= bufs.size() || bufs[tag]->ptr || bytes > r.left) return bad("bad buffer record");
    const unsigned char* src = r.take(bytes);
    amm_status st = bufs[tag]->alloc(bytes);
    if (st != AMM_OK) {
      delete d;
      return st;
    }
    const hipError_t e = hipMemcpy(bufs[tag]->ptr, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      delete d;
      return hip_fail(e, "import copy");
    }
  }
  // the buffers the products index must match the shape they claim
  const size_t lists = (size_t)d->K_eff * d->n * sizeof(float2);
  if (d->kind == AMM_CIRCULANT && nblocks == 0 && d->K_eff > 0 &&
      (d->L.bytes < lists || d->Ladj.bytes < lists || d->shifts.bytes < d->K_eff * sizeof(int32_t)))
    return bad("circulant lists shorter than K_eff x n");
  if (d->kind & AMM_SPARSE) {
    if (d->row_ptr.bytes < (size_t)(d->m + 1) * sizeof(int32_t) || d->col.bytes < d->nnz * sizeof(int32_t) ||
        d->val.bytes < d->nnz * sizeof(float))
      return bad("sparse arrays shorter than the entry count");
  }
  if (flags & F_INNER) {
    amm_status st = read_node(r, device, A, &d->inner, depth + 1);
    if (st != AMM_OK) {
      delete d;
      return st;
    }
  }
  for (int j = 0; j < nblocks; ++j) {
    amm_dec* b = nullptr;
    amm_status st = read_node(r, device, A, &b, depth + 1);
    if (st != AMM_OK) {
      delete d;
      return st;
    }
    d->blocks.push_back(b);
  }
  *out = d;
  return AMM_OK;
}

}  // namespace

extern "C" {

amm_status amm_dec_export(const amm_dec* dec, void* buf, size_t* bytes) {
  if (!dec || !bytes) return fail(AMM_EINVAL, "NULL argument");
  AMM_HIP(hipSetDevice(dec->device));
  Writer w;
  w.put<uint32_t>(kMagic);
  w.put<uint32_t>(kVersion);
  w.put<uint64_t>(0);   // total size, patched below
  AMM_TRY(write_node(dec, w));
  const uint64_t total = w.out.size();
  std::memcpy(w.out.data() + 8, &total, sizeof(total));
  if (!buf) {
    *bytes = total;
    return AMM_OK;
  }
  if (*bytes < total) return fail(AMM_EINVAL, "export buffer of %zu bytes, %llu needed", *bytes,
                                  (unsigned long long)total);
  std::memcpy(buf, w.out.data(), total);
  *bytes = total;
  return AMM_OK;
}

amm_status amm_dec_import(amm_ctx* ctx, const void* buf, size_t bytes, const float* A, amm_dec** out) {
  if (!ctx || !buf || !out) return fail(AMM_EINVAL, "NULL argument");
  Reader r{static_cast<const unsigned char*>(buf), bytes};
  const uint32_t magic = r.get<uint32_t>(), version = r.get<uint32_t>();
  const uint64_t total = r.get<uint64_t>();
  if (!r.ok || magic != kMagic) return fail(AMM_EINVAL, "not a decomposition blob");
  if (version != kVersion) return fail(AMM_EUNSUPPORTED, "decomposition blob version %u", version);
  if (total != bytes) return fail(AMM_EINVAL, "blob size %zu, header says %llu", bytes, (unsigned long long)total);
  AMM_HIP(hipSetDevice(ctx->device));
  // buffers come from the context's allocator (if it has one)
  struct Scope {
    const AllocFns* prev = g_alloc;
    DevBuf* prev_part = g_gemm_part;
    explicit Scope(amm_ctx* c) {
      g_alloc = &c->alloc;
      g_gemm_part = &c->gemm_part;
    }
    ~Scope() {
      g_alloc = prev;
      g_gemm_part = prev_part;
    }
  } scope(ctx);
  amm_dec* d = nullptr;
  AMM_TRY(read_node(r, ctx->device, A, &d, 0));
  if (r.left != 0) {
    delete d;
    return fail(AMM_EINVAL, "decomposition blob has %zu trailing bytes", r.left);
  }
  *out = d;
  return AMM_OK;
}

}  // extern "C"
