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
// vector loads; 64/G rows share a wavefront.  Workgroups are persistent;
// each XCD sweeps one contiguous eighth of the rows with all its groups in
// step (see the tile schedule below), which keeps the gathers of a row's
// own bit segment inside that XCD's L2.  The rank tables are staged in LDS
// once per workgroup.
#include <algorithm>

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

// Streaming rows (X, W in, the output out) are touched once per step:
// non-temporal accesses keep them from displacing the gathered block in L2.
template <class T, int VEC, int LDV>
__device__ __forceinline__ void load_row_nt(const T *__restrict__ p, T (&v)[VEC]) {
#pragma unroll
  for (int k = 0; k < VEC; ++k) v[k] = __builtin_nontemporal_load(p + k);
}

template <class T, int VEC, int LDV>
__device__ __forceinline__ void store_row_nt(T *__restrict__ p, const T (&v)[VEC]) {
#pragma unroll
  for (int k = 0; k < VEC; ++k) __builtin_nontemporal_store(v[k], p + k);
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

// One row of the fused step: out[r,:] for the lanes (col .. col+VEC) this
// thread owns.  tA / tB are the rank tables (LDS or global).
template <class T, int S, int LPL>
__device__ __forceinline__ void step_row(const StepArgs<T> &a, long long r, int col,
                                         const int32_t *__restrict__ tA,
                                         const int32_t *__restrict__ tB) {
  using C = StepCfg<T, S, LPL>;
  constexpr int VEC = C::VEC, LDV = C::LDV;
  constexpr int kChunk = Chunk<VEC>::value;
  const int L = a.L;
  const uint32_t fullmask = a.fullmask;
  const uint32_t lomask = a.lomask;
  const int half = a.half;

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
    load_row_nt<T, VEC, LDV>(a.X + (size_t)r * a.ldx + col, x);
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] += a.alpha * x[e];
  }
  if (a.W != nullptr) {
    T w[VEC];
    load_row_nt<T, VEC, LDV>(a.W + (size_t)r * a.ldw + col, w);
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] += a.gamma * w[e];
  }
  store_row_nt<T, VEC, LDV>(a.out + (size_t)r * a.ldo + col, acc);
}

// Stage the two rank tables in LDS (when LDS_TAB) and return their bases.
template <bool LDS_TAB>
__device__ __forceinline__ void stage_tables(const int32_t *gA, const int32_t *gB, int half,
                                             int32_t *s_tab, const int32_t *&tA,
                                             const int32_t *&tB) {
  tA = gA;
  tB = gB;
  if (LDS_TAB) {
    const int tsz = 1 << half;
    for (int i = threadIdx.x; i < tsz; i += blockDim.x) {
      s_tab[i] = gA[i];
      s_tab[tsz + i] = gB[i];
    }
    __syncthreads();
    tA = s_tab;
    tB = s_tab + tsz;
  }
}

// Tile range of physical group b of nwg over ntiles tiles.  Physical group b
// runs on XCD b % 8 (groups are dealt to the XCDs round-robin); XCD x owns
// the contiguous tile range [x TX, (x+1) TX) and its W = nwg/8 groups stride
// through it together, so the rows in flight on one XCD form one contiguous
// window: the neighbours a row gathers from its own bit segment (and, in a
// batch, its own realisation) are then mostly in that XCD's L2.
__device__ __forceinline__ void xcd_tiles(long long ntiles, long long &t_begin, long long &t_end,
                                          long long &t_step) {
  const unsigned nwg = gridDim.x;
  const unsigned b = blockIdx.x;
  if ((nwg & 7u) == 0u) {
    const long long W = nwg >> 3;
    const long long TX = (ntiles + 7) / 8;
    const long long x = b & 7u, slot_g = b >> 3;
    t_begin = x * TX + slot_g;
    t_end = (x + 1) * TX < ntiles ? (x + 1) * TX : ntiles;
    t_step = W;
  } else {
    t_begin = b;
    t_end = ntiles;
    t_step = nwg;
  }
}

template <class T, int S, int LPL, bool LDS_TAB, int MAXT>
__global__ __launch_bounds__(MAXT) void k_step(StepArgs<T> a) {
  using C = StepCfg<T, S, LPL>;
  constexpr int VEC = C::VEC, G = C::G, RPW = C::RPW;
  extern __shared__ int32_t s_tab[];
  const int32_t *tA, *tB;
  stage_tables<LDS_TAB>(a.tabA, a.tabB, a.half, s_tab, tA, tB);

  const long long rows_per_iter = (long long)(blockDim.x >> 6) * RPW;
  const long long ntiles = (a.n + rows_per_iter - 1) / rows_per_iter;
  long long t_begin, t_end, t_step;
  xcd_tiles(ntiles, t_begin, t_end, t_step);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int slot = lane / G;
  const int col = (lane % G) * VEC;
  for (long long t = t_begin; t < t_end; t += t_step) {
    const long long r = t * rows_per_iter + (long long)wave * RPW + slot;
    if (r >= a.n) continue;
    step_row<T, S, LPL>(a, r, col, tA, tB);
  }
}

// Batched Clenshaw step for B realisations of one chain length L (same
// basis, block width S): realisation i has its own diagonal, coefficients,
// order K_i and buffers.  At global step j (0 <= j <= Kmax), realisation i
// is at local step j_i = j - (Kmax - K_i) (idle while j_i < 0), so that all
// end together; step Kmax is the final combination Y = (c_0 X + H~ b_1 -
// b_2)/D.  Tiles run realisation-major, so an XCD works through whole
// realisations.
template <class T, int S, int LPL, bool LDS_TAB, int MAXT>
__global__ __launch_bounds__(MAXT) void k_step_batched(StepArgs<T> base, const BatchItem<T> *items,
                                                       int B, long long j, long long Kmax) {
  using C = StepCfg<T, S, LPL>;
  constexpr int VEC = C::VEC, G = C::G, RPW = C::RPW;
  extern __shared__ int32_t s_tab[];
  const int32_t *tA, *tB;
  stage_tables<LDS_TAB>(base.tabA, base.tabB, base.half, s_tab, tA, tB);

  const long long n = base.n;
  const long long rows_per_iter = (long long)(blockDim.x >> 6) * RPW;
  const long long tper = (n + rows_per_iter - 1) / rows_per_iter;
  long long t_begin, t_end, t_step;
  xcd_tiles(tper * B, t_begin, t_end, t_step);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int slot = lane / G;
  const int col = (lane % G) * VEC;
  for (long long t = t_begin; t < t_end; t += t_step) {
    const int i = (int)(t / tper);
    const BatchItem<T> it = items[i];
    const long long ji = j - (Kmax - it.K);
    if (!it.active || ji < 0) continue;
    const long long r = (t - (long long)i * tper) * rows_per_iter + (long long)wave * RPW + slot;
    if (r >= n) continue;
    StepArgs<T> a = base;
    a.dt = it.dt;
    const size_t blk = (size_t)n * S;
    T *bufs[3] = {it.buf, it.buf + blk, it.buf + 2 * blk};
    a.ldv = a.ldw = a.ldo = a.ldx = S;
    if (j < Kmax) {
      const long long k = it.K - ji;
      a.out = bufs[ji % 3];
      a.V = (ji >= 1) ? bufs[(ji - 1) % 3] : nullptr;
      a.W = (ji >= 2) ? bufs[(ji - 2) % 3] : nullptr;
      const double ck = it.coef[k];
      a.X = (ck != 0.0) ? it.X : nullptr;
      a.alpha = (T)ck;
      a.dscale = T(2);
      a.w1 = it.w1;
      a.w2 = it.w2;
      a.gamma = T(-1);
    } else {
      a.out = it.Y;
      a.X = it.X;
      a.alpha = (T)(it.coef[0] * it.Dinv);
      a.V = (it.K >= 1) ? bufs[(it.K - 1) % 3] : nullptr;
      a.W = (it.K >= 2) ? bufs[(it.K - 2) % 3] : nullptr;
      a.dscale = (T)it.Dinv;
      a.w1 = (T)(0.5 * (double)it.w1 * it.Dinv);
      a.w2 = (T)(0.5 * (double)it.w2 * it.Dinv);
      a.gamma = (T)(-it.Dinv);
    }
    step_row<T, S, LPL>(a, r, col, tA, tB);
  }
}

// Grid-wide barrier of a cooperative launch (every group resident).  Each
// group arrives once per barrier on a counter that only grows; barrier number
// `target / gridDim.x` is passed when the counter reaches `target`.  Every
// wave waits for its own memory operations; then one thread releases the
// group's stores at device scope (the L2s of the XCDs are not coherent with
// each other), arrives, waits, and acquires for the group.
// The wait is bounded by the device wall clock: a group that waits longer
// than `timeout` ticks (or sees the flag set) sets sync[1] and returns false,
// so every group leaves the kernel at its next barrier.
__device__ __forceinline__ bool grid_barrier(unsigned *sync, unsigned target,
                                             unsigned long long timeout) {
  __shared__ int s_fail;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's loads and stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    // one device-scope release (L2 write-back) per group, after every wave's
    // stores have left it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long t0 = wall_clock64();
    int fail = 0;
    while (__hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          wall_clock64() - t0 > timeout) {
        __hip_atomic_store(sync + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        fail = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    s_fail = fail;
    // one device-scope acquire per group: invalidates this CU's L1 and the
    // XCD's L2 lines for every wave of the group
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return s_fail == 0;
}

// All K + 1 Clenshaw steps of one filter application in one launch (see
// FusedArgs): step j < K computes b_k, k = K - j, into buffer j mod 3 from
// b_{k+1} (buffer j-1) and b_{k+2} (buffer j-2); step K writes Y.  The rank
// tables are staged once for all steps; each group keeps the same row tiles
// in every step.
template <class T, int S, int LPL, bool LDS_TAB, int MAXT>
__global__ __launch_bounds__(MAXT) void k_filter_fused(FusedArgs<T> f) {
  using C = StepCfg<T, S, LPL>;
  constexpr int VEC = C::VEC, G = C::G, RPW = C::RPW;
  extern __shared__ int32_t s_tab[];
  const int32_t *tA, *tB;
  stage_tables<LDS_TAB>(f.base.tabA, f.base.tabB, f.base.half, s_tab, tA, tB);

  const long long n = f.base.n;
  const long long rows_per_iter = (long long)(blockDim.x >> 6) * RPW;
  const long long ntiles = (n + rows_per_iter - 1) / rows_per_iter;
  long long t_begin, t_end, t_step;
  xcd_tiles(ntiles, t_begin, t_end, t_step);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int slot = lane / G;
  const int col = (lane % G) * VEC;
  const size_t blk = (size_t)n * S;
  T *bufs[3] = {f.buf, f.buf + blk, f.buf + 2 * blk};
  const long long K = f.K;
  for (long long j = 0; j <= K; ++j) {
    StepArgs<T> a = f.base;
    a.ldv = a.ldw = S;
    if (j < K) {
      const double ck = f.coef[K - j];
      a.out = bufs[j % 3];
      a.ldo = S;
      a.V = (j >= 1) ? bufs[(j - 1) % 3] : nullptr;
      a.W = (j >= 2) ? bufs[(j - 2) % 3] : nullptr;
      a.X = (ck != 0.0) ? f.X : nullptr;
      a.ldx = f.ldx;
      a.alpha = (T)ck;
      a.dscale = T(2);
      a.w1 = (T)f.w1;
      a.w2 = (T)f.w2;
      a.gamma = T(-1);
    } else {
      a.out = f.Y;
      a.ldo = f.ldy;
      a.X = f.X;
      a.ldx = f.ldx;
      a.alpha = (T)(f.coef[0] * f.Dinv);
      a.V = (K >= 1) ? bufs[(K - 1) % 3] : nullptr;
      a.W = (K >= 2) ? bufs[(K - 2) % 3] : nullptr;
      a.dscale = (T)f.Dinv;
      a.w1 = (T)(0.5 * f.w1 * f.Dinv);
      a.w2 = (T)(0.5 * f.w2 * f.Dinv);
      a.gamma = (T)(-f.Dinv);
    }
    for (long long t = t_begin; t < t_end; t += t_step) {
      const long long r = t * rows_per_iter + (long long)wave * RPW + slot;
      if (r < n) step_row<T, S, LPL>(a, r, col, tA, tB);
    }
    if (j < K && !grid_barrier(f.sync, (unsigned)((j + 1) * gridDim.x), f.timeout_ticks)) return;
  }
}

template <class T, int S, int LPL, bool LDS_TAB, int MAXT>
static bool launch_fused_k(hipStream_t st, const FusedArgs<T> &f, const StepShape &shape,
                           int num_cu, size_t shm) {
  using C = StepCfg<T, S, LPL>;
  auto kern = k_filter_fused<T, S, LPL, LDS_TAB, MAXT>;
  int per_cu = 0;
  PF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, MAXT, shm));
  const long long rows_per_iter = (long long)(MAXT / 64) * C::RPW;
  const long long tiles = (f.base.n + rows_per_iter - 1) / rows_per_iter;
  long long nwg = (long long)num_cu * std::min(per_cu, shape.wg_per_cu);
  nwg = std::min(nwg, ((tiles + 7) / 8) * 8);
  nwg = (nwg / 8) * 8;  // the per-XCD tile schedule wants a multiple of 8
  if (nwg < 8 || (double)(f.K + 1) * (double)nwg >= 4.0e9) return false;
  FusedArgs<T> arg = f;
  void *params[] = {&arg};
  PF_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3((unsigned)nwg),
                                    dim3(MAXT), params, (unsigned)shm, st));
  check_launch("k_filter_fused");
  return true;
}

// The fused kernel keeps its per-step state in registers; it is built for
// 256-thread groups only (1024-thread groups would spill), a 1024-thread
// shape running as four times as many 256-thread groups.
template <class T, int S, int LPL>
static bool launch_fused_s(hipStream_t st, const FusedArgs<T> &f, const StepShape &shape,
                           int num_cu) {
  const bool lds = shape.lds_tables && f.base.L <= kMaxLdsTableL;
  const size_t shm = lds ? (size_t)2 * sizeof(int32_t) * ((size_t)1 << f.base.half) : 0;
  if (shape.threads != 256 && shape.threads != 1024)
    throw Error(POLFED_EINVAL, "step kernel: threads must be 256 or 1024");
  StepShape sh = shape;
  if (sh.threads == 1024) {
    sh.threads = 256;
    sh.wg_per_cu *= 4;
  }
  return lds ? launch_fused_k<T, S, LPL, true, 256>(st, f, sh, num_cu, shm)
             : launch_fused_k<T, S, LPL, false, 256>(st, f, sh, num_cu, 0);
}

template <class T>
bool launch_filter_fused(hipStream_t st, int S, const FusedArgs<T> &f, const StepShape &shape,
                         int num_cu) {
  if (f.base.n <= 0) return true;
#define PF_FUSED_CASE(SS)                                                   \
  case SS:                                                                  \
    if (shape.lpl == 2) return launch_fused_s<T, SS, 2>(st, f, shape, num_cu); \
    if (shape.lpl == 4) return launch_fused_s<T, SS, 4>(st, f, shape, num_cu); \
    return launch_fused_s<T, SS, 1>(st, f, shape, num_cu);
  switch (S) {
    PF_FUSED_CASE(1)
    PF_FUSED_CASE(2)
    PF_FUSED_CASE(4)
    PF_FUSED_CASE(8)
    PF_FUSED_CASE(16)
    PF_FUSED_CASE(32)
    PF_FUSED_CASE(64)
    default: throw Error(POLFED_EINVAL, "block width must be a power of two in [1, 64]");
  }
#undef PF_FUSED_CASE
}

template bool launch_filter_fused<float>(hipStream_t, int, const FusedArgs<float> &,
                                         const StepShape &, int);
template bool launch_filter_fused<double>(hipStream_t, int, const FusedArgs<double> &,
                                          const StepShape &, int);

template <class T, int S, int LPL>
static void launch_step_s(hipStream_t st, const StepArgs<T> &a0, const StepShape &shape,
                          int num_cu) {
  using C = StepCfg<T, S, LPL>;
  StepArgs<T> a = a0;
  const int threads = shape.threads;
  const long long rows_per_iter = (long long)(threads / 64) * C::RPW;
  long long want = (long long)num_cu * shape.wg_per_cu;
  long long tiles = (a.n + rows_per_iter - 1) / rows_per_iter;
  long long nwg = std::min(want, tiles);
  // a multiple of 8 lets the kernel apply its per-XCD schedule; extra
  // groups find no tile and exit
  nwg = ((nwg + 7) / 8) * 8;
  a.rows_per_wg = rows_per_iter;
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

template <class T, int S, int LPL>
static void launch_batched_s(hipStream_t st, const StepArgs<T> &a, const BatchItem<T> *items,
                             int B, long long j, long long Kmax, const StepShape &shape,
                             int num_cu) {
  using C = StepCfg<T, S, LPL>;
  const int threads = shape.threads;
  const long long rows_per_iter = (long long)(threads / 64) * C::RPW;
  const long long tiles = ((a.n + rows_per_iter - 1) / rows_per_iter) * B;
  long long nwg = std::min((long long)num_cu * shape.wg_per_cu, tiles);
  nwg = ((nwg + 7) / 8) * 8;
  const bool lds = shape.lds_tables && a.L <= kMaxLdsTableL;
  size_t shm = lds ? (size_t)2 * sizeof(int32_t) * ((size_t)1 << a.half) : 0;
  if (threads > 256) {
    if (lds)
      k_step_batched<T, S, LPL, true, 1024><<<(unsigned)nwg, threads, shm, st>>>(a, items, B, j, Kmax);
    else
      k_step_batched<T, S, LPL, false, 1024><<<(unsigned)nwg, threads, 0, st>>>(a, items, B, j, Kmax);
  } else {
    if (lds)
      k_step_batched<T, S, LPL, true, 256><<<(unsigned)nwg, threads, shm, st>>>(a, items, B, j, Kmax);
    else
      k_step_batched<T, S, LPL, false, 256><<<(unsigned)nwg, threads, 0, st>>>(a, items, B, j, Kmax);
  }
  check_launch("k_step_batched");
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

template <class T>
void launch_step_batched(hipStream_t st, int S, const StepArgs<T> &a, const BatchItem<T> *items,
                         int B, long long j, long long Kmax, const StepShape &shape, int num_cu) {
  if (a.n <= 0 || B <= 0) return;
  if (shape.threads != 256 && shape.threads != 1024)
    throw Error(POLFED_EINVAL, "step kernel: threads must be 256 or 1024");
#define PF_BATCH_CASE(SS)                                                              \
  case SS:                                                                             \
    if (shape.lpl == 2)                                                                \
      launch_batched_s<T, SS, 2>(st, a, items, B, j, Kmax, shape, num_cu);             \
    else if (shape.lpl == 4)                                                           \
      launch_batched_s<T, SS, 4>(st, a, items, B, j, Kmax, shape, num_cu);             \
    else                                                                               \
      launch_batched_s<T, SS, 1>(st, a, items, B, j, Kmax, shape, num_cu);             \
    break;
  switch (S) {
    PF_BATCH_CASE(1)
    PF_BATCH_CASE(2)
    PF_BATCH_CASE(4)
    PF_BATCH_CASE(8)
    PF_BATCH_CASE(16)
    PF_BATCH_CASE(32)
    PF_BATCH_CASE(64)
    default: throw Error(POLFED_EINVAL, "block width must be a power of two in [1, 64]");
  }
#undef PF_BATCH_CASE
}

template void launch_step_batched<float>(hipStream_t, int, const StepArgs<float> &,
                                         const BatchItem<float> *, int, long long, long long,
                                         const StepShape &, int);
template void launch_step_batched<double>(hipStream_t, int, const StepArgs<double> &,
                                          const BatchItem<double> *, int, long long, long long,
                                          const StepShape &, int);

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
