// lc_search_noalloc: the first stage of the search with its workspace in a
// fixed device array of the library instead of caller memory, for callers
// that cannot allocate device memory (include/lc.h).
//
// The array is a file-scope device variable, so every GPU the library runs on
// holds its own copy for the life of the process.  Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device
// (kept per device below): the variable's name on the host is not a device
// address.
#include <mutex>

#include "lc_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(LC_NOALLOC_SCRATCH_BYTES);
constexpr size_t kCounterBytes = 256;  // the walk's queue counters at the head of a workspace
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static_assert(kScratchBytes % 16 == 0, "the fill kernel writes 16-byte words");

// Zero n16 16-byte words (a kernel, not a memset, so that a captured call
// records no memset node).
__global__ void zero_words_kernel(uint4 *p, size_t n16) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += size_t(gridDim.x) * blockDim.x)
    p[i] = z;
}

struct DeviceScratch {
  void *ptr = nullptr;  // device address of `scratch` on this device
};

std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

// The array's address on the current device, found (and the whole array
// zeroed on `st`) at the first call on that device.
int scratch_on(int dev, hipStream_t st, void **out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (dev < 0 || dev >= kMaxDevices) return LC_EINVAL;
  DeviceScratch &d = g_dev[dev];
  if (!d.ptr) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LC_EHIP;
    hipLaunchKernelGGL(zero_words_kernel, dim3(1024), dim3(256), 0, st, static_cast<uint4 *>(p),
                       kScratchBytes / 16);
    if (hipGetLastError() != hipSuccess) return LC_EHIP;
    d.ptr = p;
  }
  *out = d.ptr;
  return LC_OK;
}

}  // namespace

extern "C" int lc_search_noalloc(const lc_index *ix, const void *lut, int lut_dtype, const float *lut_scale,
                                 int64_t nq, const int32_t *ef, int32_t ef_max, int32_t S, int32_t *cand_ids,
                                 float *cand_adc, int32_t *cand_n, int32_t *stats, void *stream) {
  if (!ix || nq < 0 || ef_max < 1 || S < 1) return LC_EINVAL;
  if (ef_max > 4096 || S > 4096) return LC_ENOTSUP;
  if (lut_dtype != LC_LUT_F32 && lut_dtype != LC_LUT_F16) return LC_EINVAL;
  if (nq == 0) return LC_OK;
  if (nq > int64_t(0x7FFFFFFF)) return LC_EINVAL;
  if (!lut || !cand_ids || !cand_adc || !cand_n) return LC_EINVAL;
  if (lut_dtype == LC_LUT_F16 && !lut_scale) return LC_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LC_EHIP;
  if (dev != ix->device) return LC_EINVAL;  // the array used is the current device's
  hipStream_t st = static_cast<hipStream_t>(stream);
  void *ptr = nullptr;
  int rc = scratch_on(dev, st, &ptr);
  if (rc != LC_OK) return rc;
  // the queue counters start at zero; a walk that ran to its end left every
  // visited bitset and id list behind them zero-filled
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, static_cast<uint4 *>(ptr), kCounterBytes / 16);
  if (hipGetLastError() != hipSuccess) return LC_EHIP;
  return lc_launch_walk(ix, lut, lut_dtype, lut_scale, nq, ef, ef_max, S, 0, nullptr, cand_ids, cand_adc, cand_n,
                        stats, ptr, kScratchBytes, nullptr, st, /*fit_ws=*/true);
}
