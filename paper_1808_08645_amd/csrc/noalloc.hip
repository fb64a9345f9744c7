// Entry points for callers that cannot allocate: the per-block partial sums of the FP64
// norm reduction live in a fixed device array of the library instead of a context buffer,
// and a second kernel adds them on the device, so a call allocates and synchronises
// nothing.
//
// The array's host-side name is not a device address: set-up (bbwadg_create, with the
// context's device current) asks HIP for this device's address of it once and keeps it per
// device; kernels only ever receive that address.
#include <atomic>

#include "bbwadg_internal.hpp"

namespace bbw {

// [kScratchBlocks][4] per-block partial sums; every GPU holds its own copy until the
// process ends. Calls on one GPU share it, so calls that overlap on one GPU race.
static __device__ __align__(256) double scratch[kScratchBlocks * 4];

namespace {

constexpr int kMaxScratchDevices = 64;
std::atomic<double*> g_scratch[kMaxScratchDevices];

// out[f] = sum over b of partial[b][f], b ascending: the order of the host-side sum of
// bbwadg_l2norm2, so both give the same bits.
__global__ __launch_bounds__(64) void sum_partials_kernel(const double* partial, int nblocks, double* out) {
  const int f = threadIdx.x;
  if (f < 4) {
    double acc = 0.0;
    for (int b = 0; b < nblocks; ++b) acc += partial[(size_t)b * 4 + f];
    out[f] = acc;
  }
}

}  // namespace

int scratch_init() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= kMaxScratchDevices) return (int)hipErrorInvalidDevice;
  if (g_scratch[dev].load(std::memory_order_acquire)) return 0;
  double* p = nullptr;
  e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
  if (e != hipSuccess) return (int)e;
  g_scratch[dev].store(p, std::memory_order_release);  // the same value if two threads race here
  return 0;
}

int l2norm2_noalloc(int N, int dtype, const void* q, int64_t K, const double* J, const double* mass, int nblocks,
                    double* out, void* stream) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  double* p = (dev >= 0 && dev < kMaxScratchDevices) ? g_scratch[dev].load(std::memory_order_acquire) : nullptr;
  if (!p) return (int)hipErrorNotInitialized;
  if (nblocks <= 0 || nblocks > kScratchBlocks) return (int)hipErrorInvalidValue;
  int r = launch_l2norm(N, dtype, q, K, J, mass, p, nblocks, stream);
  if (r) return r;
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, (const double*)p, nblocks, out);
  return (int)hipGetLastError();
}

}  // namespace bbw
