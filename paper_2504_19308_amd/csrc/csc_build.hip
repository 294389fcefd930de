// Column-major copy (CSC) of a sparse part and the per-row entry ranges of
// the blocked sparse products, built on the device.
//
// The CSC is the CSR transposed with the entries of each column in row order:
// a stable radix sort of the entries by column (the CSR order is row-major,
// so equal columns keep their row order), the column starts by binary search
// in the sorted columns, the rows and values unpacked.  The block ranges give,
// per row of an index-sorted CSR (or CSC), the first entry of every block of
// kSpBlock inner indices.
#include <hipcub/hipcub.hpp>

#include "amm_internal.hpp"

namespace amm {
namespace {

// packed[e] = (row << 32) | bits(val[e]) for the entries e of every row
__global__ void pack_rows(const int32_t* __restrict__ rp, int64_t rows, const float* __restrict__ val,
                          uint64_t* __restrict__ packed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x)
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
      packed[e] = ((uint64_t)(uint32_t)i << 32) | (uint64_t)__float_as_uint(val[e]);
}

// cp[c] = first position of column c in the sorted columns (c = 0 .. n)
__global__ void col_starts(const int32_t* __restrict__ sorted, int64_t nnz, int64_t n, int32_t* __restrict__ cp) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n; c += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (sorted[mid] < c) lo = mid + 1;
      else hi = mid;
    }
    cp[c] = (int32_t)lo;
  }
}

__global__ void unpack_rows(const uint64_t* __restrict__ packed, int64_t nnz, int32_t* __restrict__ rr,
                            float* __restrict__ cv) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t v = packed[e];
    rr[e] = (int32_t)(v >> 32);
    cv[e] = __uint_as_float((uint32_t)v);
  }
}

// *unsorted = 1 if some row's indices decrease
__global__ void check_sorted(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx, int64_t rows,
                             int* __restrict__ unsorted) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x) {
    bool bad = false;
    for (int32_t e = ptr[i] + 1; e < ptr[i + 1]; ++e) bad |= idx[e] < idx[e - 1];
    if (bad) atomicOr(unsorted, 1);
  }
}

__global__ void set_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// h[i (nb + 1) + b] = first entry of row i with index >= b kSpBlock; h[i (nb + 1) + nb] = end of row i
__global__ void row_block_starts(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx, int64_t rows,
                                 int nb, int32_t* __restrict__ h) {
  const int64_t total = rows * (nb + 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / (nb + 1);
    const int b = (int)(t - i * (nb + 1));
    int32_t lo = ptr[i], hi = ptr[i + 1];
    if (b < nb) {
      const int64_t key = (int64_t)b * kSpBlock;
      while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (idx[mid] < key) lo = mid + 1;
        else hi = mid;
      }
    }
    h[t] = b < nb ? lo : ptr[i + 1];
  }
}

unsigned grid_for(int64_t items) { return (unsigned)std::min<int64_t>(std::max<int64_t>((items + 255) / 256, 1), 8192); }

// Entry ranges per block of kSpBlock inner indices, or blocks = 1 when the
// inner dimension is short (up to 2 kSpBlock, where a whole slice of B stays
// in an XCD's L2) or a row's indices are not sorted.
amm_status block_ranges(const int32_t* ptr, const int32_t* idx, int64_t rows, int64_t inner, int* flag,
                        amm::DevBuf* out, int* blocks, hipStream_t s) {
  *blocks = 1;
  if (inner <= 2 * kSpBlock) return AMM_OK;
  hipLaunchKernelGGL(set_int, dim3(1), dim3(64), 0, s, flag, 0);
  hipLaunchKernelGGL(check_sorted, dim3(grid_for(rows)), dim3(256), 0, s, ptr, idx, rows, flag);
  AMM_HIP(hipGetLastError());
  int unsorted = 0;
  AMM_HIP(hipMemcpyAsync(&unsorted, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  AMM_HIP(hipStreamSynchronize(s));
  if (unsorted) return AMM_OK;
  const int nb = (int)((inner + kSpBlock - 1) / kSpBlock);
  AMM_TRY(out->alloc((size_t)rows * (nb + 1) * 4));
  hipLaunchKernelGGL(row_block_starts, dim3(grid_for(rows * (nb + 1))), dim3(256), 0, s, ptr, idx, rows, nb,
                     out->as<int32_t>());
  AMM_HIP(hipGetLastError());
  *blocks = nb;
  return AMM_OK;
}

}  // namespace

amm_status build_csc(amm_dec* d, hipStream_t s) {
  const int64_t m = d->m, n = d->n, nnz = d->nnz;
  if (nnz > INT32_MAX || m > INT32_MAX || n >= INT32_MAX) return fail(AMM_ESHAPE, "sparse part too large");
  AMM_TRY(d->csc_ptr.alloc((n + 1) * 4));
  AMM_TRY(d->csc_row.alloc(std::max<int64_t>(nnz, 1) * 4));
  AMM_TRY(d->csc_val.alloc(std::max<int64_t>(nnz, 1) * 4));
  DevBuf packed, packed_out, cols_out, temp, flag;
  AMM_TRY(flag.alloc(sizeof(int)));
  if (nnz > 0) {
    AMM_TRY(packed.alloc(nnz * 8));
    AMM_TRY(packed_out.alloc(nnz * 8));
    AMM_TRY(cols_out.alloc(nnz * 4));
    hipLaunchKernelGGL(pack_rows, dim3(grid_for(m)), dim3(256), 0, s, d->row_ptr.as<int32_t>(), m,
                       d->val.as<float>(), packed.as<uint64_t>());
    AMM_HIP(hipGetLastError());
    int end_bit = 1;
    while (end_bit < 31 && (int64_t(1) << end_bit) < n) ++end_bit;
    size_t temp_bytes = 0;
    AMM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, d->col.as<int32_t>(), cols_out.as<int32_t>(),
                                               packed.as<uint64_t>(), packed_out.as<uint64_t>(), (int)nnz, 0,
                                               end_bit, s));
    AMM_TRY(temp.alloc(std::max<size_t>(temp_bytes, 1)));
    AMM_HIP(hipcub::DeviceRadixSort::SortPairs(temp.ptr, temp_bytes, d->col.as<int32_t>(), cols_out.as<int32_t>(),
                                               packed.as<uint64_t>(), packed_out.as<uint64_t>(), (int)nnz, 0,
                                               end_bit, s));
    hipLaunchKernelGGL(unpack_rows, dim3(grid_for(nnz)), dim3(256), 0, s, packed_out.as<uint64_t>(), nnz,
                       d->csc_row.as<int32_t>(), d->csc_val.as<float>());
  }
  hipLaunchKernelGGL(col_starts, dim3(grid_for(n + 1)), dim3(256), 0, s, cols_out.as<int32_t>(), nnz, n,
                     d->csc_ptr.as<int32_t>());
  AMM_HIP(hipGetLastError());
  AMM_TRY(block_ranges(d->row_ptr.as<int32_t>(), d->col.as<int32_t>(), m, n, flag.as<int>(), &d->csr_blk,
                       &d->csr_blocks, s));
  AMM_TRY(block_ranges(d->csc_ptr.as<int32_t>(), d->csc_row.as<int32_t>(), n, m, flag.as<int>(), &d->csc_blk,
                       &d->csc_blocks, s));
  // the local buffers are released on return
  AMM_HIP(hipStreamSynchronize(s));
  return AMM_OK;
}

}  // namespace amm
