// LDS read bandwidth of the whole chip, measured (the ceiling the decoders' LDS traffic is
// compared with).  Every workgroup fills 32 KB of LDS and then reads it back in a loop with
// bank-conflict-free accesses (consecutive lanes, consecutive words), 4 or 16 bytes per lane
// per instruction; the reads are folded into a value per thread that is stored, so that none
// of them can be dropped.  Not part of the decoders: a measurement aid built beside them.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kThreads = 256;
constexpr int kWords = 8192;  // 32 KB of LDS per workgroup

template <int WIDTH>
__global__ __launch_bounds__(kThreads) void lds_read_kernel(uint32_t* __restrict__ out, int reps) {
  __shared__ uint32_t buf[kWords];
  const int t = threadIdx.x;
  for (int j = t; j < kWords; j += kThreads) buf[j] = (uint32_t)j * 2654435761u;
  __syncthreads();
  // The base moves by whole wavefront rows (lanes stay contiguous) and stays low enough that
  // the unrolled reads are base + constant: immediate offsets, no address arithmetic per read.
  uint32_t acc0 = 0u, acc1 = 0u;
  if constexpr (WIDTH == 16) {
    const uint4* v = reinterpret_cast<const uint4*>(buf);  // 2048 entries
    for (int r = 0; r < reps; ++r) {
      const int base = t + 64 * (r & 7);  // <= 703
#pragma unroll
      for (int u = 0; u < 4; ++u) {  // <= 703 + 768 < 2048
        const uint4 x = v[base + u * kThreads];
        acc0 = acc0 + x.x + x.y;  // three-input adds: one vector instruction per pair
        acc1 = acc1 + x.z + x.w;
      }
    }
  } else {
    for (int r = 0; r < reps; ++r) {
      const int base = t + 64 * (r & 7);  // <= 703
#pragma unroll
      for (int u = 0; u < 8; u += 4) {  // <= 703 + 7 * 1024 < 8192
        acc0 = acc0 + buf[base + u * 1024] + buf[base + (u + 1) * 1024];
        acc1 = acc1 + buf[base + (u + 2) * 1024] + buf[base + (u + 3) * 1024];
      }
    }
  }
  out[(size_t)blockIdx.x * kThreads + t] = acc0 + acc1;
}

}  // namespace

// Reads LDS with `width_bytes` (4 or 16) per lane per instruction on every CU and returns the
// rate in bytes per second (`bytes_per_s`) and the mean launch time (`ms`) over `launches`
// timed launches after one untimed one.  Allocates and frees its own output buffer on the
// current device.  Returns 0, or -1 for a bad argument, or the HIP error code.
extern "C" int lds_peak_measure(int width_bytes, int launches, double* bytes_per_s, double* ms) {
  if ((width_bytes != 4 && width_bytes != 16) || launches < 1 || !bytes_per_s || !ms) return -1;
  int dev = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return (int)e;
  const int blocks = prop.multiProcessorCount * 16;
  const int reps = 8192;  // a few milliseconds per launch
  uint32_t* out = nullptr;
  e = hipMalloc(&out, (size_t)blocks * kThreads * sizeof(uint32_t));
  if (e != hipSuccess) return (int)e;
  hipEvent_t a = nullptr, b = nullptr;
  e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  float total = 0.f;
  for (int k = 0; e == hipSuccess && k <= launches; ++k) {
    if (k == 1) e = hipEventRecord(a, nullptr);
    if (e != hipSuccess) break;
    if (width_bytes == 16)
      hipLaunchKernelGGL(lds_read_kernel<16>, dim3(blocks), dim3(kThreads), 0, nullptr, out, reps);
    else
      hipLaunchKernelGGL(lds_read_kernel<4>, dim3(blocks), dim3(kThreads), 0, nullptr, out, reps);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(b, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(&total, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(out);
  if (e != hipSuccess) return (int)e;
  const double per = (double)total / launches;
  // per thread and repetition: 4 reads of 16 bytes, or 8 reads of 4 bytes
  const double bytes = (double)blocks * kThreads * reps * (width_bytes == 16 ? 4.0 : 8.0) * width_bytes;
  *ms = per;
  *bytes_per_s = bytes / (per * 1e-3);
  return 0;
}
