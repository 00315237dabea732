// Kernel of one launch class of the phased batch (window pitch
// SWEPT_BATCH_WC, workgroup size SWEPT_BATCH_NT, set by the build: one object
// per class).
#include "stages.hpp"

#if !defined(SWEPT_BATCH_WC) || !defined(SWEPT_BATCH_NT)
#error "build with -DSWEPT_BATCH_WC=<pitch> -DSWEPT_BATCH_NT=<threads>"
#endif

template struct swept::BatchPhase<SWEPT_BATCH_WC, SWEPT_BATCH_NT>;

#if defined(SWEPT2D_BUILD_PERSISTENT_BATCH) && SWEPT_BATCH_WC == 66
namespace swept {
hipError_t launch_batch(const BatchSched& s, int blocks, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_batch, dim3(blocks), dim3(kBatchThreads), lds, st, s);
  return hipGetLastError();
}

hipError_t launch_batch_reset(unsigned* done, int ngrids, unsigned long long* head, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3((ngrids + 255) / 256 + 1), dim3(256), 0, st, done, ngrids, head);
  return hipGetLastError();
}

hipError_t batch_blocks_per_cu(size_t lds, int* out) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_batch, kBatchThreads, lds);
}
}  // namespace swept
#endif
