// The Gram product for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
// polfed_gram_static keeps its partial tiles in a fixed device array instead
// of the context's growable workspace.
//
// The array below, `scratch`, is a file-scope __device__ variable: every
// GPU the library runs on holds its own copy until the process ends.  In
// host code its name is a host-side stand-in, not a device address; the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device (with that device current) at context creation and kept
// in g_scratch_ptr.  Only that pointer is handed to kernels.
//
// Every call on one GPU shares that GPU's array and leaves the last call's
// partial tiles in it; the Gram kernels overwrite every tile they sum, so
// nothing needs clearing.  Calls that overlap in time on one GPU (from two
// streams or two contexts) race on the array.
#include <mutex>
#include <string>

#include "internal.h"

namespace polfed {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kGramScratchDoubles];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

void init_gram_scratch(int device) {
  PF_REQUIRE(device >= 0 && device < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void *ptr = nullptr;
  PF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  g_scratch_ptr[device] = static_cast<double *>(ptr);
}

__global__ void k_fill_block(int p, int q, double *C, long long ldc, double v) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)p * q) return;
  C[(e / q) * ldc + (e % q)] = v;
}

void launch_gram_static(hipStream_t st, int device, long long n, int p, int q, const double *X,
                        long long ldx, const double *Y, long long ldy, double *C,
                        long long ldc, int num_cu) {
  PF_REQUIRE(device >= 0 && device < kMaxDevices, "device index out of range");
  double *part = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    part = g_scratch_ptr[device];
  }
  PF_REQUIRE(part != nullptr, "polfed_gram_static: scratch not set up on this device");
  PF_REQUIRE((long long)p * q <= (long long)kGramScratchDoubles,
             "polfed_gram_static: p * q = " + std::to_string((long long)p * q) +
                 " exceeds the fixed scratch of " + std::to_string(kGramScratchDoubles) +
                 " doubles");
  if (n == 0) {  // no rows: C = 0, by a fill kernel
    const long long tot = (long long)p * q;
    k_fill_block<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(p, q, C, ldc, 0.0);
    check_launch("k_fill_block");
    return;
  }
  long long rows_per_chunk = 0;
  const long long nchunks =
      gram_chunks(n, p, q, num_cu, (long long)kGramScratchDoubles, rows_per_chunk);
  launch_gram_parts(st, n, p, q, X, ldx, Y, ldy, C, ldc, part, rows_per_chunk, nchunks);
}

}  // namespace polfed
