// fill.hip -- device fills and a one-word device copy.
#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

__global__ void k_copy1(uint32_t *dst, const uint32_t *src) { *dst = *src; }

__global__ void k_fill(uint32_t *p, uint32_t v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_zero_spans(ZeroSpans z) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (int k = 0; k < z.count; k++)
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < z.n[k]; i += stride) z.p[k][i] = 0;
}

}  // namespace

void copy_u32(uint32_t *dst, const uint32_t *src, hipStream_t s) {
  PCBZ_LAUNCH(k_copy1, dim3(1), dim3(1), 0, s, dst, src);
}

void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  PCBZ_LAUNCH(k_fill, dim3((uint32_t)blocks), dim3(256), 0, s, p, v, n);
}

void zero_spans(const ZeroSpans &z, hipStream_t s) {
  size_t most = 0;
  for (int k = 0; k < z.count; k++) most = z.n[k] > most ? z.n[k] : most;
  if (most == 0) return;
  size_t blocks = (most + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  PCBZ_LAUNCH(k_zero_spans, dim3((uint32_t)blocks), dim3(256), 0, s, z);
}

}  // namespace pcbz
