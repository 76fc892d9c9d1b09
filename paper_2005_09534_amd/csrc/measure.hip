// Attainable HBM bandwidth: a plain device copy with 16-byte vector loads and
// stores over a grid-stride loop, timed with HIP events on the caller's
// stream.  It gives the copy rate that the step kernel's achieved bandwidth
// is set beside (the peak of the HBM3E stacks is not reachable by any
// kernel).
#include <algorithm>

#include "internal.h"

namespace polfed {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void k_stream_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                              long long n16) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

double stream_copy_gbs(hipStream_t st, const void *src, void *dst, long long bytes, int reps,
                       int num_cu) {
  const long long n16 = bytes / 16;
  if (n16 <= 0 || reps <= 0) return 0.0;
  const int th = 256;
  const long long nwg = std::min<long long>((n16 + th - 1) / th, (long long)num_cu * 16);
  hipEvent_t e0, e1;
  PF_HIP(hipEventCreate(&e0));
  PF_HIP(hipEventCreate(&e1));
  k_stream_copy<<<(unsigned)nwg, th, 0, st>>>(static_cast<const u32x4 *>(src),
                                               static_cast<u32x4 *>(dst), n16);  // warm
  check_launch("k_stream_copy");
  PF_HIP(hipEventRecord(e0, st));
  for (int k = 0; k < reps; ++k)
    k_stream_copy<<<(unsigned)nwg, th, 0, st>>>(static_cast<const u32x4 *>(src),
                                                 static_cast<u32x4 *>(dst), n16);
  PF_HIP(hipEventRecord(e1, st));
  PF_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  PF_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return 2.0 * 16.0 * (double)n16 * reps / (1e-3 * ms) / 1e9;
}

}  // namespace polfed
