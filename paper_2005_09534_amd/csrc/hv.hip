// FP64 instantiations of the fused Chebyshev step (hv_kernels.h), and the
// small layout kernels of the filter: slice packing and precision casts.
#include "hv_kernels.h"

namespace polfed {

template void launch_step_batched<double>(hipStream_t, int, const StepArgs<double> &,
                                   const BatchItem<double> *, int, long long, long long,
                                   long long, const BatchTables &, const StepShape &, int);
template long long batched_tile_rows<double>(int, const StepShape &);
template void launch_step<double>(hipStream_t, int, const StepArgs<double> &,
                                  const StepShape &, int);

// -------------------------------------------------------------- casts --

template <class T>
__global__ void k_pack_slices(long long n, int S, int sw, const T *X, long long ldx, T *out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * S) return;
  const long long r = i / S;
  const int c = (int)(i - r * S);
  const int sl = c / sw;
  out[(size_t)sl * n * sw + (size_t)r * sw + (c - sl * sw)] = X[(size_t)r * ldx + c];
}

template <class T>
void launch_pack_slices(hipStream_t st, long long n, int S, int nslices, const T *X,
                        long long ldx, T *out) {
  const long long tot = n * S;
  if (tot <= 0) return;
  const int th = 256;
  k_pack_slices<T><<<(unsigned)((tot + th - 1) / th), th, 0, st>>>(n, S, S / nslices, X, ldx, out);
  check_launch("k_pack_slices");
}

template void launch_pack_slices<float>(hipStream_t, long long, int, int, const float *,
                                        long long, float *);
template void launch_pack_slices<double>(hipStream_t, long long, int, int, const double *,
                                         long long, double *);

template <class Tin, class Tout>
__global__ void k_cast(long long n, int S, const Tin *in, long long ldin, Tout *out,
                       long long ldout) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * S) return;
  long long r = i / S;
  int c = (int)(i - r * S);
  out[(size_t)r * ldout + c] = (Tout)in[(size_t)r * ldin + c];
}

template <class Tin, class Tout>
void launch_cast(hipStream_t st, long long n, int S, const Tin *in, long long ldin, Tout *out,
                 long long ldout) {
  long long tot = n * S;
  if (tot <= 0) return;
  int th = 256;
  k_cast<Tin, Tout><<<(unsigned)((tot + th - 1) / th), th, 0, st>>>(n, S, in, ldin, out, ldout);
  check_launch("k_cast");
}

template void launch_cast<double, float>(hipStream_t, long long, int, const double *, long long,
                                         float *, long long);
template void launch_cast<float, double>(hipStream_t, long long, int, const float *, long long,
                                         double *, long long);
template void launch_cast<double, double>(hipStream_t, long long, int, const double *,
                                          long long, double *, long long);

}  // namespace polfed
