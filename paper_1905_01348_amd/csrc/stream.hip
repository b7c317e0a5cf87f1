// Bandwidth probes: read-only, write-only and in-place streams over a device
// buffer, 16 bytes per lane per access in a grid-stride loop, with the same
// non-temporal hints the pair passes use on their pair volume.  They give the
// DRAM rates a kernel of this library can expect on the device it runs on,
// against which the pass kernels' achieved rates are read.
#include <algorithm>

#include "common.hpp"

namespace fx {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// the XOR of everything read; written out (by a vector store of one lane)
// only if it equals a value no data of the probe produces, so that the loads
// cannot be dropped
__global__ void __launch_bounds__(256) k_stream_read(const u32x4* __restrict__ p, size_t n, u32x4* __restrict__ sink) {
  u32x4 acc = {0u, 0u, 0u, 0u};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    acc ^= __builtin_nontemporal_load(p + i);
  if (acc.x == 0x9e3779b9u && acc.y == 0x7f4a7c15u && acc.z == 0x85ebca6bu && acc.w == 0xc2b2ae35u)
    sink[threadIdx.x] = acc;
}

__global__ void __launch_bounds__(256) k_stream_write(u32x4* __restrict__ p, size_t n, unsigned int v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const u32x4 w = {v, v ^ (unsigned int)i, v, v};
    __builtin_nontemporal_store(w, p + i);
  }
}

__global__ void __launch_bounds__(256) k_stream_inplace(u32x4* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    // every lane of the word changes, so that the whole 16 bytes are loaded
    // and stored (changing one lane lets the compiler narrow both to 4 bytes)
    u32x4 w = __builtin_nontemporal_load(p + i);
    w += 1u;
    __builtin_nontemporal_store(w, p + i);
  }
}

}  // namespace fx

using namespace fx;

extern "C" {

fx_status fx_debug_stream(fx_ctx* ctx, int32_t mode, void* buf, size_t bytes, int32_t iters, void* stream,
                          double* gbps) {
  clear_error();
  if (!ctx) FX_FAIL(FX_ERR_INVALID, "ctx is NULL");
  if (!buf || !gbps) FX_FAIL(FX_ERR_INVALID, "buf and gbps must be non-NULL");
  if (mode < 0 || mode > 2) FX_FAIL(FX_ERR_INVALID, "mode = %d not in {0, 1, 2}", mode);
  if (bytes < 4096 || bytes % 16 || ((uintptr_t)buf % 16)) FX_FAIL(FX_ERR_INVALID, "bytes must be >= 4096, a multiple of 16, on a 16-byte aligned buffer");
  if (iters < 1) FX_FAIL(FX_ERR_INVALID, "iters = %d must be >= 1", iters);
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  FX_HIP(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const size_t n = bytes / 16;
  // the read probe's sink: the first 4 KiB of the buffer itself (written only
  // on a match no data of the probe produces)
  u32x4* p = reinterpret_cast<u32x4*>(buf);
  // many short-lived workgroups: the grid that streamed fastest in a sweep of 2048-65536
  const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  auto launch = [&]() {
    if (mode == 0)
      hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, st, p, n, p);
    else if (mode == 1)
      hipLaunchKernelGGL(k_stream_write, dim3(grid), dim3(256), 0, st, p, n, 0x5a5a5a5au);
    else
      hipLaunchKernelGGL(k_stream_inplace, dim3(grid), dim3(256), 0, st, p, n);
  };
  launch();  // warm-up
  FX_LAUNCH_CHECK();
  hipEvent_t e0, e1;
  FX_HIP(hipEventCreate(&e0));
  FX_HIP(hipEventCreate(&e1));
  FX_HIP(hipEventRecord(e0, st));
  for (int i = 0; i < iters; ++i) launch();
  FX_HIP(hipEventRecord(e1, st));
  FX_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  FX_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  FX_LAUNCH_CHECK();
  const double moved = (mode == 2 ? 2.0 : 1.0) * (double)bytes * iters;
  *gbps = ms > 0.f ? moved / (ms * 1e-3) / 1e9 : 0.0;
  return FX_OK;
}

}  // extern "C"
