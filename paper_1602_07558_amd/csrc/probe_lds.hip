// LDS read bandwidth of the device, measured (the roofline peak that the
// stage kernels' LDS traffic is compared with). Built as its own small
// library (libswept2d_probe.so) for the benchmark; the swept2d library does
// not use it.
//
// Every thread streams reads of W-byte words from a 64 KB LDS buffer, eight
// distinct addresses per iteration, consecutive lanes on consecutive words
// (no bank conflicts), and adds every loaded word into an accumulator that
// is stored behind a data-dependent test, so no read can be dropped or
// merged. Two workgroups of 1024 threads per compute unit keep 32 waves
// issuing LDS reads.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

constexpr int kThreads = 1024;
constexpr int kBufBytes = 65536;

template <class T>
__global__ __launch_bounds__(kThreads) void k_lds_read(int iters, unsigned* sink) {
  constexpr int N = kBufBytes / (int)sizeof(T);  // a power of two
  constexpr int WORDS = (int)sizeof(T) / 4;
  __shared__ T buf[N];
  for (int i = threadIdx.x; i < N; i += kThreads) {
    T v;
    unsigned* p = reinterpret_cast<unsigned*>(&v);
#pragma unroll
    for (int k = 0; k < WORDS; ++k) p[k] = (unsigned)(i * 131 + k);
    buf[i] = v;
  }
  __syncthreads();
  unsigned acc = 0;
  int idx = (int)threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const T v = buf[(idx + u * (N / 8)) & (N - 1)];
      const unsigned* p = reinterpret_cast<const unsigned*>(&v);
#pragma unroll
      for (int k = 0; k < WORDS; ++k) acc += p[k];
    }
    idx = (idx + 64 + (int)(acc & 0)) & (N - 1);
    __asm__ volatile("" : "+v"(idx));
  }
  if (acc == 0x9E3779B9u) sink[blockIdx.x] = acc;
}

template <class T>
int run(int cus, int iters, double* bytes_per_s) {
  unsigned* sink = nullptr;
  if (hipMalloc(&sink, sizeof(unsigned) * 4 * cus) != hipSuccess) return -1;
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  const int blocks = 2 * cus;
  hipLaunchKernelGGL(k_lds_read<T>, dim3(blocks), dim3(kThreads), 0, 0, 8, sink);
  hipEventRecord(a, 0);
  hipLaunchKernelGGL(k_lds_read<T>, dim3(blocks), dim3(kThreads), 0, 0, iters, sink);
  hipEventRecord(b, 0);
  hipError_t e = hipEventSynchronize(b);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  hipEventDestroy(a);
  hipEventDestroy(b);
  hipFree(sink);
  if (e != hipSuccess || ms <= 0) return -2;
  *bytes_per_s = (double)blocks * kThreads * (double)iters * 8.0 * sizeof(T) / (ms * 1e-3);
  return 0;
}

}  // namespace

// Measured LDS read bandwidth of the current device in bytes per second, with
// 8-byte words (ds_read_b64, as the FP64 stage kernels use) and 16-byte words
// (ds_read_b128). Returns 0, or a negative code when a HIP call failed.
extern "C" int lds_probe_read_bandwidth(double* b64_bytes_per_s, double* b128_bytes_per_s, int* cus) {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -3;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return -3;
  *cus = n;
  int rc = run<uint2>(n, 4000, b64_bytes_per_s);
  if (rc == 0) rc = run<uint4>(n, 4000, b128_bytes_per_s);
  return rc;
}
