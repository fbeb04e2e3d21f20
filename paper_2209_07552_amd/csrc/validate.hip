// msrep_validate: O(nnz) structure checks of a matrix descriptor on the GPU.
// The first offence (lowest position) is reported.
#include <mutex>
#include <vector>

#include "common.hpp"

namespace msrep {
namespace {

enum : int64_t {
  kPtrStart = 1,  // ptr[0] != 0
  kPtrOrder = 2,  // ptr[i] > ptr[i+1]
  kPtrEnd = 3,    // ptr[rows] != nnz
  kIdxRange = 4,  // minor index out of range
  kRowOrder = 5,  // COO row indices decrease
  kRowRange = 6,  // COO row index out of range
  kColOrder = 7,  // column-sorted COO column indices decrease
};

__device__ __forceinline__ void report(unsigned long long *first, int64_t pos, int64_t code) {
  atomicMin(first, static_cast<unsigned long long>(pos) * 8ull + static_cast<unsigned long long>(code));
}

__global__ void check_compressed(const int32_t *__restrict__ ptr, int32_t rows,
                                 const int32_t *__restrict__ idx, int64_t nnz, int32_t minor,
                                 unsigned long long *first) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i <= rows; i += stride) {
    if (i == 0 && ptr[0] != 0) report(first, 0, kPtrStart);
    if (i < rows && ptr[i] > ptr[i + 1]) report(first, i, kPtrOrder);
    if (i == rows && ptr[rows] != nnz) report(first, rows, kPtrEnd);
  }
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < nnz; k += stride)
    if (static_cast<uint32_t>(idx[k]) >= static_cast<uint32_t>(minor)) report(first, k, kIdxRange);
}

// order: 0 any, 1 rows non-decreasing, 2 columns non-decreasing
__global__ void check_coo(const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                          int64_t nnz, int32_t m, int32_t n, int order,
                          unsigned long long *first) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < nnz; k += stride) {
    if (static_cast<uint32_t>(row[k]) >= static_cast<uint32_t>(m)) report(first, k, kRowRange);
    if (order == 1 && k > 0 && row[k - 1] > row[k]) report(first, k, kRowOrder);
    if (order == 2 && k > 0 && col[k - 1] > col[k]) report(first, k, kColOrder);
    if (static_cast<uint32_t>(col[k]) >= static_cast<uint32_t>(n)) report(first, k, kIdxRange);
  }
}

__global__ void set_u64(unsigned long long *p, unsigned long long v) { *p = v; }

// One small result word per device, allocated on first use and kept.
unsigned long long *result_word(int dev) {
  static std::mutex mu;
  static std::vector<unsigned long long *> words;
  std::lock_guard<std::mutex> g(mu);
  if (static_cast<int>(words.size()) <= dev) words.resize(dev + 1, nullptr);
  if (!words[dev]) {
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(unsigned long long)) != hipSuccess) return nullptr;
    words[dev] = static_cast<unsigned long long *>(p);
  }
  return words[dev];
}

}  // namespace
}  // namespace msrep

using namespace msrep;

extern "C" msrep_status msrep_validate(const msrep_mat *A, void *stream) {
  if (msrep_status st = check_mat(A, "msrep_validate")) return st;
  int dev = 0;
  MSREP_HIP(hipGetDevice(&dev));
  unsigned long long *word = result_word(dev);
  if (!word) return fail(MSREP_ERR_HIP, "msrep_validate: cannot allocate the result word");
  hipStream_t s = as_stream(stream);
  const unsigned long long none = ~0ull;
  hipLaunchKernelGGL(set_u64, dim3(1), dim3(1), 0, s, word, none);
  MSREP_LAUNCHED("set_u64");
  const int64_t work = (A->nnz > A->m ? A->nnz : A->m) + 1;
  const int grid = static_cast<int>((work + 255) / 256 < 8192 ? (work + 255) / 256 : 8192);
  if (A->fmt == MSREP_COO || A->fmt == MSREP_COO_ANY || A->fmt == MSREP_COO_COL) {
    if (A->nnz > 0) {
      const int order = A->fmt == MSREP_COO ? 1 : A->fmt == MSREP_COO_COL ? 2 : 0;
      hipLaunchKernelGGL(check_coo, dim3(grid), dim3(256), 0, s, A->idx, A->idx2, A->nnz, A->m,
                         A->n, order, word);
      MSREP_LAUNCHED("check_coo");
    }
  } else {
    const int32_t rows = major_dim(A), minor = A->fmt == MSREP_CSR ? A->n : A->m;
    hipLaunchKernelGGL(check_compressed, dim3(grid), dim3(256), 0, s, A->ptr, rows, A->idx,
                       A->nnz, minor, word);
    MSREP_LAUNCHED("check_compressed");
  }
  unsigned long long host = none;
  MSREP_HIP(hipMemcpyAsync(&host, word, sizeof host, hipMemcpyDeviceToHost, s));
  MSREP_HIP(hipStreamSynchronize(s));
  if (host == none) return ok();
  const long long pos = static_cast<long long>(host / 8);
  static const char *what[8] = {"",
                               "pointer does not start at 0",
                               "pointer decreases",
                               "pointer does not end at nnz",
                               "index out of range",
                               "COO row indices are not sorted",
                               "COO row index out of range",
                               "COO column indices are not sorted"};
  return fail(MSREP_ERR_FORMAT, "msrep_validate: %s at position %lld", what[host % 8], pos);
}
