// Matrix-free application of H~ fused with one three-term Chebyshev step.
//
//   out[r,:] = alpha X[r,:] + dscale dt[r] V[r,:] + sum_bonds w_l V[r',:]
//              + gamma W[r,:]
//
// H of eq. (XXZ) has, in row r (state s), the diagonal d_r and an entry J_l/2
// at the row r' of s with an antiparallel pair (i, i+l mod L) swapped
// (Supplement, "Technical details": the off-diagonal values are all equal,
// so nothing but the pattern is needed -- and here not even the pattern is
// stored: it is regenerated from s).  H is symmetric, so y = Hx is a pure
// row gather: no atomics.
//
// One Clenshaw step b_k = c_k X + 2 H~ b_{k+1} - b_{k+2} is this kernel with
// alpha = c_k, V = b_{k+1}, dscale = 2 (dt = a d + b), w_l = a J_l, W =
// b_{k+2}, gamma = -1; the last step Y = (c_0 X + H~ b_1 - b_2)/D uses
// alpha = c_0/D, dscale = 1/D, w_l = a J_l/(2D), gamma = -1/D.
//
// Layout: blocks are row-major (the s values of a row contiguous), so one
// gathered neighbour is one contiguous s * sizeof(T) segment.  A row is
// owned by G lanes, each moving VEC = 16/sizeof(T) * LPL elements with 16-byte
// vector loads; 64/G rows share a wavefront.  Workgroups are persistent and
// each owns a contiguous range of rows; the workgroup index is remapped so
// that the ranges of one XCD are adjacent (consecutive workgroup ids land on
// different XCDs), which keeps the near-diagonal gathers inside one L2.
// The rank tables are staged in LDS once per workgroup.
#include "internal.h"

namespace polfed {

template <class T, int N>
struct alignas(sizeof(T) * N) VecT {
  T v[N];
};

template <class T, int S, int LPL>
struct StepCfg {
  static constexpr int kV16 = 16 / (int)sizeof(T);             // elements per 16 B
  static constexpr int VEC = (S >= kV16 * LPL) ? kV16 * LPL : (S >= kV16 ? kV16 : S);
  static constexpr int G = S / VEC;                               // lanes per row
  static_assert(G >= 1 && G <= 64, "row must fit a wavefront");
  static constexpr int RPW = 64 / G;                              // rows per wave
  static constexpr int NLD = (VEC * (int)sizeof(T) >= 16) ? VEC * (int)sizeof(T) / 16 : 1;
  static constexpr int LDV = (VEC * (int)sizeof(T) >= 16) ? 16 / (int)sizeof(T) : VEC;
};

template <class T, int VEC, int LDV>
__device__ __forceinline__ void load_row(const T *__restrict__ p, T (&v)[VEC]) {
#pragma unroll
  for (int k = 0; k < VEC; k += LDV) {
    VecT<T, LDV> t = *reinterpret_cast<const VecT<T, LDV> *>(p + k);
#pragma unroll
    for (int e = 0; e < LDV; ++e) v[k + e] = t.v[e];
  }
}

template <class T, int VEC, int LDV>
__device__ __forceinline__ void store_row(T *__restrict__ p, const T (&v)[VEC]) {
#pragma unroll
  for (int k = 0; k < VEC; k += LDV) {
    VecT<T, LDV> t;
#pragma unroll
    for (int e = 0; e < LDV; ++e) t.v[e] = v[k + e];
    *reinterpret_cast<VecT<T, LDV> *>(p + k) = t;
  }
}

// Neighbours gathered per batch: enough loads in flight per lane for memory-
// level parallelism while the batch stays within ~32 registers of data.
template <int VEC>
struct Chunk {
  static constexpr int value = (32 / VEC) > 8 ? 8 : ((32 / VEC) < 2 ? 2 : 32 / VEC);
};

template <class T, int S, int LPL, bool LDS_TAB, int MAXT>
__global__ __launch_bounds__(MAXT) void k_step(StepArgs<T> a) {
  using C = StepCfg<T, S, LPL>;
  constexpr int VEC = C::VEC, G = C::G, RPW = C::RPW, LDV = C::LDV;
  constexpr int kChunk = Chunk<VEC>::value;
  extern __shared__ int32_t s_tab[];

  const int32_t *tA = a.tabA;
  const int32_t *tB = a.tabB;
  const int tsz = 1 << a.half;
  if (LDS_TAB) {
    for (int i = threadIdx.x; i < tsz; i += blockDim.x) {
      s_tab[i] = a.tabA[i];
      s_tab[tsz + i] = a.tabB[i];
    }
    __syncthreads();
    tA = s_tab;
    tB = s_tab + tsz;
  }

  // XCD-aware remap: physical id b runs on XCD b % 8; give each XCD one
  // contiguous run of logical ranges.
  const unsigned nwg = gridDim.x;
  const unsigned b = blockIdx.x;
  unsigned logical = b;
  if ((nwg & 7u) == 0u) logical = (b & 7u) * (nwg >> 3) + (b >> 3);

  const long long r_begin = (long long)logical * a.rows_per_wg;
  long long r_end = r_begin + a.rows_per_wg;
  if (r_end > a.n) r_end = a.n;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int slot = lane / G;
  const int col = (lane % G) * VEC;
  const long long rows_per_iter = (long long)(blockDim.x >> 6) * RPW;
  const int L = a.L;
  const uint32_t fullmask = a.fullmask;
  const uint32_t lomask = a.lomask;
  const int half = a.half;

  for (long long base = r_begin; base < r_end; base += rows_per_iter) {
    const long long r = base + (long long)wave * RPW + slot;
    if (r >= r_end) continue;

    T acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = T(0);

    if (a.V != nullptr) {
      const uint32_t s = a.states[r];
      T self[VEC];
      load_row<T, VEC, LDV>(a.V + (size_t)r * a.ldv + col, self);
      const T dd = a.dscale * a.dt[r];
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] = dd * self[e];

      // antiparallel bonds: bit i of s ^ rot_l(s) marks the pair (i, i+l)
      const uint32_t rot1 = ((s >> 1) | (s << (L - 1))) & fullmask;
      unsigned long long mm = (unsigned long long)(s ^ rot1);
      if (a.has_j2) {
        const uint32_t rot2 = ((s >> 2) | (s << (L - 2))) & fullmask;
        mm |= (unsigned long long)(s ^ rot2) << 32;
      }
      while (mm) {
        int32_t idx[kChunk];
        bool two[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          idx[u] = -1;
          two[u] = false;
          if (mm) {
            const int bit = __ffsll((long long)mm) - 1;
            mm &= mm - 1ull;
            const int l = (bit >= 32) ? 2 : 1;
            const int i = bit & 31;
            int j = i + l;
            if (j >= L) j -= L;
            const uint32_t f = s ^ ((1u << i) | (1u << j));
            idx[u] = tA[f >> half] + tB[f & lomask];
            two[u] = (l == 2);
          }
        }
        T nb[kChunk][VEC];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          if (idx[u] >= 0) load_row<T, VEC, LDV>(a.V + (size_t)idx[u] * a.ldv + col, nb[u]);
        }
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          if (idx[u] >= 0) {
            const T w = two[u] ? a.w2 : a.w1;
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] += w * nb[u][e];
          }
        }
      }
    }

    if (a.X != nullptr) {
      T x[VEC];
      load_row<T, VEC, LDV>(a.X + (size_t)r * a.ldx + col, x);
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] += a.alpha * x[e];
    }
    if (a.W != nullptr) {
      T w[VEC];
      load_row<T, VEC, LDV>(a.W + (size_t)r * a.ldw + col, w);
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] += a.gamma * w[e];
    }
    store_row<T, VEC, LDV>(a.out + (size_t)r * a.ldo + col, acc);
  }
}

template <class T, int S, int LPL>
static void launch_step_s(hipStream_t st, const StepArgs<T> &a0, const StepShape &shape,
                          int num_cu) {
  using C = StepCfg<T, S, LPL>;
  StepArgs<T> a = a0;
  const int threads = shape.threads;
  const long long rows_per_iter = (long long)(threads / 64) * C::RPW;
  long long want = (long long)num_cu * shape.wg_per_cu;
  long long iters_total = (a.n + rows_per_iter - 1) / rows_per_iter;
  long long iters_per_wg = (iters_total + want - 1) / want;
  if (iters_per_wg < 1) iters_per_wg = 1;
  a.rows_per_wg = iters_per_wg * rows_per_iter;
  long long nwg = (a.n + a.rows_per_wg - 1) / a.rows_per_wg;
  // a multiple of 8 lets the kernel apply its XCD remap; extra groups exit
  nwg = ((nwg + 7) / 8) * 8;
  const bool lds = shape.lds_tables && a.L <= kMaxLdsTableL;
  size_t shm = lds ? (size_t)2 * sizeof(int32_t) * ((size_t)1 << a.half) : 0;
  if (threads > 256) {
    if (threads != 1024) throw Error(POLFED_EINVAL, "step kernel: threads must be 256 or 1024");
    if (lds)
      k_step<T, S, LPL, true, 1024><<<(unsigned)nwg, threads, shm, st>>>(a);
    else
      k_step<T, S, LPL, false, 1024><<<(unsigned)nwg, threads, 0, st>>>(a);
  } else {
    if (threads != 256) throw Error(POLFED_EINVAL, "step kernel: threads must be 256 or 1024");
    if (lds)
      k_step<T, S, LPL, true, 256><<<(unsigned)nwg, threads, shm, st>>>(a);
    else
      k_step<T, S, LPL, false, 256><<<(unsigned)nwg, threads, 0, st>>>(a);
  }
  check_launch("k_step");
}

template <class T, int S>
static void launch_step_lpl(hipStream_t st, const StepArgs<T> &a, const StepShape &shape,
                            int num_cu) {
  switch (shape.lpl) {
    case 2: launch_step_s<T, S, 2>(st, a, shape, num_cu); break;
    case 4: launch_step_s<T, S, 4>(st, a, shape, num_cu); break;
    default: launch_step_s<T, S, 1>(st, a, shape, num_cu); break;
  }
}

template <class T>
void launch_step(hipStream_t st, int S, const StepArgs<T> &a, const StepShape &shape,
                 int num_cu) {
  if (a.n <= 0) return;
  switch (S) {
    case 1: launch_step_lpl<T, 1>(st, a, shape, num_cu); break;
    case 2: launch_step_lpl<T, 2>(st, a, shape, num_cu); break;
    case 4: launch_step_lpl<T, 4>(st, a, shape, num_cu); break;
    case 8: launch_step_lpl<T, 8>(st, a, shape, num_cu); break;
    case 16: launch_step_lpl<T, 16>(st, a, shape, num_cu); break;
    case 32: launch_step_lpl<T, 32>(st, a, shape, num_cu); break;
    case 64: launch_step_lpl<T, 64>(st, a, shape, num_cu); break;
    default: throw Error(POLFED_EINVAL, "block width must be a power of two in [1, 64]");
  }
}

template void launch_step<float>(hipStream_t, int, const StepArgs<float> &, const StepShape &,
                                 int);
template void launch_step<double>(hipStream_t, int, const StepArgs<double> &,
                                  const StepShape &, int);

// -------------------------------------------------------------- casts --

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
