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
//
// Ranks of neighbours come from the two tables (rank mode RM = 0), or
// (RM = 1) incrementally
// from the row's own rank: in the colex rank sum_t C(p_t, t), moving the
// particle with q particles below it from bit i to bit i+1 adds C(i, q)
// (Pascal's rule on its one term); a hop from i to i+2 adds C(i, q) +
// C(i+1, q + n_{i+1}) (two such moves, the second one over or past the
// particle at i+1); the reverse moves subtract the same.  Bonds that wrap
// round the chain renumber every particle and take the tables.  RM = 2 reads
// them from a stored pattern instead (the paper's own matrix form: column
// indices only, the value J_l/2 implied by the bond range, which the top bit
// of an index marks), built once per chain length in the same bond order, so
// all three modes add the same terms in the same order.
//
// The forward three-term form t_{k+1} = 2 H~ t_k - t_{k-1} (the sum of
// c_k T_k(H~) X accumulated term by term) is this kernel with W = t_{k-1}
// and the fused accumulation acc = cin src + cacc out.
#pragma once
// Included by hv.hip (FP64 instantiations, casts) and hv_f32.hip (FP32
// instantiations), which compile in parallel.
#include <algorithm>
#include <climits>
#include <type_traits>

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
template <class T, int S, int LPL, bool EARLY, int RM>
__device__ __forceinline__ void step_row(const StepArgs<T> &a, long long r, int col,
                                         const int32_t *__restrict__ tA,
                                         const uint16_t *__restrict__ tB,
                                         const int32_t *__restrict__ tC) {
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
  // EARLY: the streamed operands do not depend on the gathers; issuing their
  // loads first overlaps their latency with the neighbour rounds (a gain
  // where a step is one round of latency, small chains) at the cost of
  // registers held across the gathers.  Either way they are added last, in
  // the same order, so the result does not depend on EARLY.
  T x[VEC], w[VEC];
  if (EARLY) {
    if (a.X != nullptr) load_row_nt<T, VEC, LDV>(a.X + (size_t)r * a.ldx + col, x);
    if (a.W != nullptr) load_row_nt<T, VEC, LDV>(a.W + (size_t)r * a.ldw + col, w);
  }

  if (a.V != nullptr) {
    const uint32_t s = (RM == 2) ? 0u : a.states[r];
    T self[VEC];
    load_row<T, VEC, LDV>(a.V + (size_t)r * a.ldv + col, self);
    const T dd = a.dscale * a.dt[r];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = dd * self[e];

    // antiparallel bonds: bit i of s ^ rot_l(s) marks the pair (i, i+l);
    // with the stored pattern, the row's index range [q, qe)
    unsigned long long mm = 0ull;
    long long q = 0, qe = 0;
    if (RM == 2) {
      q = a.csr_ptr[r];
      qe = a.csr_ptr[r + 1];
    } else {
      const uint32_t rot1 = ((s >> 1) | (s << (L - 1))) & fullmask;
      mm = (unsigned long long)(s ^ rot1);
      if (a.has_j2) {
        const uint32_t rot2 = ((s >> 2) | (s << (L - 2))) & fullmask;
        mm |= (unsigned long long)(s ^ rot2) << 32;
      }
    }
    auto remaining = [&]() { return (RM == 2) ? (q < qe) : (mm != 0ull); };
    // Neighbours go in chunks of kChunk: the rank-table lookups of chunk c+1
    // are issued right after the gathers of chunk c, so each chunk costs one
    // round of memory latency (lookups and gathers overlap) rather than two.
    // Bits are taken in the same order either way, so the sum is unchanged.
    // (bit u of `two` marks a J2 bond in slot u)
    auto fill = [&](int32_t(&idx)[kChunk], uint32_t &two) {
      two = 0u;
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        idx[u] = -1;
        if (RM == 2) {
          if (q < qe) {
            const uint32_t e = (uint32_t)a.csr_col[q++];
            idx[u] = (int32_t)(e & 0x7fffffffu);
            if (e >> 31) two |= 1u << u;
          }
        } else if (mm) {
          const int bit = __ffsll((long long)mm) - 1;
          mm &= mm - 1ull;
          const int l = (bit >= 32) ? 2 : 1;
          const int i = bit & 31;
          int j = i + l;
          if (j >= L) j -= L;
          if (RM == 1 && j > i) {
            const int q = __popc(s & ((1u << i) - 1u));
            int d = tC[32 * i + q];
            if (l == 2) d += tC[32 * (i + 1) + q + (int)((s >> (i + 1)) & 1u)];
            idx[u] = ((s >> i) & 1u) ? (int32_t)r + d : (int32_t)r - d;
          } else {
            const uint32_t f = s ^ ((1u << i) | (1u << j));
            idx[u] = tA[f >> half] + (int32_t)tB[f & lomask];
          }
          if (l == 2) two |= 1u << u;
        }
      }
    };
    int32_t idx[kChunk];
    uint32_t two;
    fill(idx, two);
    for (;;) {
      T nb[kChunk][VEC];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        if (idx[u] >= 0) load_row<T, VEC, LDV>(a.V + (size_t)idx[u] * a.ldv + col, nb[u]);
      }
      const bool more = remaining();
      int32_t idx2[kChunk];
      uint32_t two2;
      fill(idx2, two2);  // no-op lookups when nothing is left
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        if (idx[u] >= 0) {
          const T w = ((two >> u) & 1u) ? a.w2 : a.w1;
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[e] += w * nb[u][e];
        }
      }
      if (!more) break;
#pragma unroll
      for (int u = 0; u < kChunk; ++u) idx[u] = idx2[u];
      two = two2;
    }
  }

  if (a.X != nullptr) {
    if (!EARLY) load_row_nt<T, VEC, LDV>(a.X + (size_t)r * a.ldx + col, x);
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] += a.alpha * x[e];
  }
  if (a.W != nullptr) {
    if (!EARLY) load_row_nt<T, VEC, LDV>(a.W + (size_t)r * a.ldw + col, w);
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] += a.gamma * w[e];
  }
  if (!a.skip_out) store_row_nt<T, VEC, LDV>(a.out + (size_t)r * a.ldo + col, acc);
  if (a.acc != nullptr) {
    T src[VEC];
    load_row_nt<T, VEC, LDV>(a.src + (size_t)r * a.ldsrc + col, src);
#pragma unroll
    for (int e = 0; e < VEC; ++e) src[e] = a.cin * src[e] + a.cacc * acc[e];
    store_row_nt<T, VEC, LDV>(a.acc + (size_t)r * a.ldacc + col, src);
  }
}

// Stage the two rank tables in LDS (when LDS_TAB) and return their bases.
// LDS layout (bytes): tabA (2^half int32), tabB (2^half uint16), then the
// 32 x 32 binomials (int32) when RANKI.
template <bool LDS_TAB, bool RANKI>
__device__ __forceinline__ void stage_tables(const int32_t *gA, const uint16_t *gB,
                                             const int32_t *gC, int half, int32_t *s_tab,
                                             const int32_t *&tA, const uint16_t *&tB,
                                             const int32_t *&tC) {
  tA = gA;
  tB = gB;
  tC = gC;
  if (LDS_TAB) {
    const int tsz = 1 << half;
    uint16_t *sB = reinterpret_cast<uint16_t *>(s_tab + tsz);
    for (int i = threadIdx.x; i < tsz; i += blockDim.x) {
      s_tab[i] = gA[i];
      sB[i] = gB[i];
    }
    int32_t *sC = s_tab + tsz + tsz / 2;  // tsz >= 4, so 4-byte aligned
    if (RANKI)
      for (int i = threadIdx.x; i < 32 * 32; i += blockDim.x) sC[i] = gC[i];
    __syncthreads();
    tA = s_tab;
    tB = sB;
    if (RANKI) tC = sC;
  }
}

// Tile range and column slice of physical group b of nwg.  Physical group b
// runs on XCD b % 8 (groups are dealt to the XCDs round-robin).  With
// nslices column slices, XCD x works on slice x % nslices and on part
// x / nslices of the rows: the tile range [p TX, (p+1) TX) of the 8 /
// nslices parts, which its W = nwg/8 groups stride through together, so the
// rows in flight on one XCD form one contiguous window.  The neighbours a
// row gathers from its own bit segment are then mostly in that XCD's L2;
// with fewer parts the window covers more of the chain (with nslices = 8,
// every XCD sweeps all rows of its own slice and no gathered line is shared
// between XCDs), and the L2 holds more rows of the narrower slice.
__device__ __forceinline__ void xcd_tiles(long long ntiles, int nslices, int &slice,
                                          long long &t_begin, long long &t_end,
                                          long long &t_step, bool interleave = false) {
  const unsigned nwg = gridDim.x;
  const unsigned b = blockIdx.x;
  slice = 0;
  if ((nwg & 7u) == 0u) {
    const long long W = nwg >> 3;
    const int x = (int)(b & 7u);
    slice = x & (nslices - 1);
    const int parts = 8 / nslices;
    const int part = x / nslices;
    if (interleave) {
      // the parts take every parts-th tile, so all XCDs of a slice sweep one
      // row window together (one window for the Infinity Cache to hold
      // instead of `parts`)
      t_begin = (long long)part + (long long)parts * (long long)(b >> 3);
      t_end = ntiles;
      t_step = (long long)parts * W;
    } else {
      const long long TX = (ntiles + parts - 1) / parts;
      t_begin = (long long)part * TX + (long long)(b >> 3);
      t_end = ((long long)part + 1) * TX < ntiles ? ((long long)part + 1) * TX : ntiles;
      t_step = W;
    }
  } else {  // (the launchers always round the grid to a multiple of 8)
    t_begin = b;
    t_end = ntiles;
    t_step = nwg;
  }
}

template <class T, int S, int LPL, bool LDS_TAB, int MAXT, bool EARLY, int RM>
__global__ __launch_bounds__(MAXT) void k_step(StepArgs<T> a) {
  using C = StepCfg<T, S, LPL>;
  constexpr int VEC = C::VEC, G = C::G, RPW = C::RPW;
  extern __shared__ int32_t s_tab[];
  const int32_t *tA, *tC;
  const uint16_t *tB;
  stage_tables<LDS_TAB && RM != 2, RM == 1>(a.tabA, a.tabB, a.binom, a.half, s_tab, tA, tB, tC);

  const long long rows_per_iter = (long long)(blockDim.x >> 6) * RPW;
  const long long ntiles = (a.n + rows_per_iter - 1) / rows_per_iter;
  long long t_begin, t_end, t_step;
  int slice;
  xcd_tiles(ntiles, a.nslices, slice, t_begin, t_end, t_step, a.interleave != 0);
  if (slice != 0) {  // this group's column slice of every operand
    if (a.X) a.X += slice * a.xss;
    if (a.V) a.V += slice * a.vss;
    if (a.W) a.W += slice * a.wss;
    a.out += slice * a.oss;
    if (a.acc) a.acc += slice * a.accss;
    if (a.src) a.src += slice * a.srcss;
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int slot = lane / G;
  const int col = (lane % G) * VEC;
  for (long long t = t_begin; t < t_end; t += t_step) {
    const long long r = t * rows_per_iter + (long long)wave * RPW + slot;
    if (r >= a.n) continue;
    step_row<T, S, LPL, EARLY, RM>(a, r, col, tA, tB, tC);
  }
}

// Batched Clenshaw step for B realisations of one block width S (chain
// lengths may differ): realisation i has its own chain, diagonal,
// coefficients, order K_i and buffers.  At global step j (0 <= j <= Kmax),
// realisation i is at local step j_i = j - (Kmax - K_i) (idle while j_i <
// 0), so that all end together; step Kmax is the final combination Y = (c_0
// X + H~ b_1 - b_2)/D.  The tiles of all realisations form one range
// (realisation-major, item i from its tile0), so an XCD works through whole
// realisations, and short chains share each launch with long ones.
template <class T, int S, int LPL, bool LDS_TAB, int MAXT, bool EARLY>
__global__ __launch_bounds__(MAXT) void k_step_batched(StepArgs<T> base, const BatchItem<T> *items,
                                                       int B, long long j, long long Kmax,
                                                       long long ntiles, BatchTables bt) {
  using C = StepCfg<T, S, LPL>;
  constexpr int VEC = C::VEC, G = C::G, RPW = C::RPW;
  extern __shared__ int32_t s_tab[];
  const int32_t *tC = base.binom;
  if (LDS_TAB) {  // every distinct chain length's tables
    for (int k = 0; k < bt.count; ++k) {
      const int tsz = 1 << bt.half[k];
      int32_t *sA = s_tab + bt.off[k];
      uint16_t *sB = reinterpret_cast<uint16_t *>(sA + tsz);
      for (int i = threadIdx.x; i < tsz; i += blockDim.x) {
        sA[i] = bt.A[k][i];
        sB[i] = bt.B[k][i];
      }
    }
    __syncthreads();
  }

  const long long rows_per_iter = (long long)(blockDim.x >> 6) * RPW;
  long long t_begin, t_end, t_step;
  int slice;
  const int ns = base.nslices;  // column slices: S is one slice's width
  xcd_tiles(ntiles, ns, slice, t_begin, t_end, t_step);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int slot = lane / G;
  const int col = (lane % G) * VEC;
  // the realisation holding tile t is the last item with tile0 <= t: a
  // binary search for this group's first tile, then, as t only grows, a
  // forward scan (the tile range of one realisation spans many steps of t)
  int i = 0;
  {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].tile0 <= t_begin)
        lo = mid;
      else
        hi = mid - 1;
    }
    i = lo;
  }
  long long next0 = (i + 1 < B) ? items[i + 1].tile0 : LLONG_MAX;
  for (long long t = t_begin; t < t_end; t += t_step) {
    while (t >= next0) {
      ++i;
      next0 = (i + 1 < B) ? items[i + 1].tile0 : LLONG_MAX;
    }
    const BatchItem<T> it = items[i];
    const long long ji = j - (Kmax - it.K);
    if (!it.active || ji < 0) {
      // the realisation idles at this step: jump past the rest of its tiles
      // (a batch spends many steps with most of its members idle)
      if (next0 >= t_end) break;
      t += ((next0 - t + t_step - 1) / t_step - 1) * t_step;
      continue;
    }
    const long long r = (t - it.tile0) * rows_per_iter + (long long)wave * RPW + slot;
    if (r >= it.n) continue;
    StepArgs<T> a = base;
    a.states = it.states;
    a.n = it.n;
    a.L = it.L;
    a.half = it.half;
    a.lomask = it.lomask;
    a.fullmask = it.fullmask;
    a.dt = it.dt;
    // recurrence buffers: three blocks of n x (ns S), each slice-major (this
    // group's slice: n x S at slice n S); X and Y row-major, this slice's
    // columns at offset slice S
    const size_t blk = (size_t)it.n * S * ns;
    const size_t soff = (size_t)slice * it.n * S;
    T *bufs[3] = {it.buf + soff, it.buf + blk + soff, it.buf + 2 * blk + soff};
    a.ldv = a.ldw = S;
    a.ldx = it.ldx;
    if (j < Kmax) {
      const long long k = it.K - ji;
      a.out = bufs[ji % 3];
      a.ldo = S;
      a.V = (ji >= 1) ? bufs[(ji - 1) % 3] : nullptr;
      a.W = (ji >= 2) ? bufs[(ji - 2) % 3] : nullptr;
      const double ck = it.coef[k];
      a.X = (ck != 0.0) ? it.X + (size_t)slice * S : nullptr;
      a.alpha = (T)ck;
      a.dscale = T(2);
      a.w1 = it.w1;
      a.w2 = it.w2;
      a.gamma = T(-1);
    } else {
      a.out = it.Y + (size_t)slice * S;
      a.ldo = it.ldy;
      a.X = it.X + (size_t)slice * S;
      a.alpha = (T)(it.coef[0] * it.Dinv);
      a.V = (it.K >= 1) ? bufs[(it.K - 1) % 3] : nullptr;
      a.W = (it.K >= 2) ? bufs[(it.K - 2) % 3] : nullptr;
      a.dscale = (T)it.Dinv;
      a.w1 = (T)(0.5 * (double)it.w1 * it.Dinv);
      a.w2 = (T)(0.5 * (double)it.w2 * it.Dinv);
      a.gamma = (T)(-it.Dinv);
    }
    if (LDS_TAB) {
      const int32_t *tA = s_tab + it.taboff;
      step_row<T, S, LPL, EARLY, 0>(a, r, col, tA,
                                    reinterpret_cast<const uint16_t *>(tA + (1 << it.half)), tC);
    } else {
      step_row<T, S, LPL, EARLY, 0>(a, r, col, it.tabA, it.tabB, tC);
    }
  }
}

// Calls f.template operator()<LDS_TAB, MAXT, EARLY, RM>() for the runtime
// choice (rank modes other than the tables only where the launcher uses
// them; the stored pattern needs no tables in LDS).
template <bool MODES_USED, class F>
static void dispatch_shape(bool lds, int threads, bool early, int rank_mode, F &&f) {
  if (threads != 256 && threads != 512 && threads != 1024)
    throw Error(POLFED_EINVAL, "step kernel: threads must be 256, 512 or 1024");
  auto with_rank = [&](auto lds_c, auto thr_c, auto early_c) {
    constexpr bool LD = decltype(lds_c)::value;
    constexpr int TH = decltype(thr_c)::value;
    constexpr bool EA = decltype(early_c)::value;
    if (MODES_USED && rank_mode == 1)
      f.template operator()<LD, TH, EA, MODES_USED ? 1 : 0>();
    else if (MODES_USED && rank_mode == 2)
      f.template operator()<false, TH, EA, MODES_USED ? 2 : 0>();
    else
      f.template operator()<LD, TH, EA, 0>();
  };
  auto with_threads = [&](auto lds_c, auto early_c) {
    if (threads == 1024)
      with_rank(lds_c, std::integral_constant<int, 1024>{}, early_c);
    else if (threads == 512)
      with_rank(lds_c, std::integral_constant<int, 512>{}, early_c);
    else
      with_rank(lds_c, std::integral_constant<int, 256>{}, early_c);
  };
  using T_ = std::true_type;
  using F_ = std::false_type;
  if (lds)
    early ? with_threads(T_{}, T_{}) : with_threads(T_{}, F_{});
  else
    early ? with_threads(F_{}, T_{}) : with_threads(F_{}, F_{});
}

// Launchers of the two step kernels for one (T, S, LPL), called by
// dispatch_shape with the remaining template parameters.
template <class T, int S, int LPL>
struct StepLaunch {
  hipStream_t st;
  const StepArgs<T> &a;
  long long nwg;
  int threads;
  size_t shm;
  template <bool LDS_TAB, int MAXT, bool EARLY, int RM>
  void operator()() const {
    // L = 28 tables (96 KB) exceed the default 64 KB of dynamic LDS per
    // group
    if (LDS_TAB && shm > 65536)
      PF_HIP(hipFuncSetAttribute(
          reinterpret_cast<const void *>(k_step<T, S, LPL, LDS_TAB, MAXT, EARLY, RM>),
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    k_step<T, S, LPL, LDS_TAB, MAXT, EARLY, RM>
        <<<(unsigned)nwg, threads, LDS_TAB ? shm : 0, st>>>(a);
  }
};

template <class T, int S, int LPL>
struct BatchedLaunch {
  hipStream_t st;
  const StepArgs<T> &a;
  const BatchItem<T> *items;
  int B;
  long long j, Kmax, ntiles, nwg;
  const BatchTables &bt;
  int threads;
  size_t shm;
  template <bool LDS_TAB, int MAXT, bool EARLY, int RM>
  void operator()() const {
    if (LDS_TAB && shm > 65536)
      PF_HIP(hipFuncSetAttribute(
          reinterpret_cast<const void *>(k_step_batched<T, S, LPL, LDS_TAB, MAXT, EARLY>),
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    k_step_batched<T, S, LPL, LDS_TAB, MAXT, EARLY>
        <<<(unsigned)nwg, threads, LDS_TAB ? shm : 0, st>>>(a, items, B, j, Kmax, ntiles, bt);
  }
};

template <class T, int S, int LPL>
static void launch_step_s(hipStream_t st, const StepArgs<T> &a0, const StepShape &shape,
                          int num_cu) {
  using C = StepCfg<T, S, LPL>;
  StepArgs<T> a = a0;
  const int threads = shape.threads;
  const long long rows_per_iter = (long long)(threads / 64) * C::RPW;
  long long want = (long long)num_cu * shape.wg_per_cu;
  long long tiles = (a.n + rows_per_iter - 1) / rows_per_iter;
  long long nwg = std::min(want, tiles * a.nslices);
  // a multiple of 8 lets the kernel apply its per-XCD schedule; extra
  // groups find no tile and exit
  nwg = ((nwg + 7) / 8) * 8;
  a.rows_per_wg = rows_per_iter;
  const int mode = shape.rank_incr;
  if (mode == 2 && (a.csr_ptr == nullptr || a.csr_col == nullptr))
    throw Error(POLFED_EINVAL, "step kernel: stored neighbour pattern not built");
  const bool lds = shape.lds_tables && a.L <= kMaxLdsTableL && mode != 2;
  const size_t shm =
      lds ? (size_t)6 * ((size_t)1 << a.half) + (mode == 1 ? sizeof(int32_t) * 32 * 32 : 0) : 0;
  dispatch_shape<true>(lds, threads, shape.early_loads != 0, mode,
                       StepLaunch<T, S, LPL>{st, a, nwg, threads, shm});
  check_launch("k_step");
}

template <class T, int S, int LPL>
static void launch_batched_s(hipStream_t st, const StepArgs<T> &a, const BatchItem<T> *items,
                             int B, long long j, long long Kmax, long long ntiles,
                             const BatchTables &bt, const StepShape &shape, int num_cu) {
  const int threads = shape.threads;
  long long nwg = std::min((long long)num_cu * shape.wg_per_cu, ntiles * a.nslices);
  nwg = ((nwg + 7) / 8) * 8;
  const bool lds = shape.lds_tables && bt.count > 0;
  const size_t shm = lds ? sizeof(int32_t) * (size_t)bt.ints : 0;
  dispatch_shape<false>(lds, threads, shape.early_loads != 0, 0,
                        BatchedLaunch<T, S, LPL>{st, a, items, B, j, Kmax, ntiles, nwg, bt,
                                                 threads, shm});
  check_launch("k_step_batched");
}

// Loads per lane beyond what a row of S values holds change nothing (the
// row is then one lane's), so only distinct kernels are built.
template <class T, int S>
constexpr int max_lpl() {
  return (S * (int)sizeof(T) >= 64) ? 4 : (S * (int)sizeof(T) >= 32 ? 2 : 1);
}

template <class T, int S>
static void launch_step_lpl(hipStream_t st, const StepArgs<T> &a, const StepShape &shape,
                            int num_cu) {
  constexpr int M = max_lpl<T, S>();
  const int lpl = std::min(shape.lpl, M);
  if constexpr (M >= 4)
    if (lpl == 4) return launch_step_s<T, S, 4>(st, a, shape, num_cu);
  if constexpr (M >= 2)
    if (lpl == 2) return launch_step_s<T, S, 2>(st, a, shape, num_cu);
  launch_step_s<T, S, 1>(st, a, shape, num_cu);
}

template <class T>
void launch_step(hipStream_t st, int S, const StepArgs<T> &a0, const StepShape &shape,
                 int num_cu) {
  if (a0.n <= 0) return;
  StepArgs<T> a = a0;
  if (a.nslices < 1) a.nslices = 1;
  if (a.nslices != 1 && a.nslices != 2 && a.nslices != 4 && a.nslices != 8)
    throw Error(POLFED_EINVAL, "step kernel: column slices must be 1, 2, 4 or 8");
  if (S % a.nslices != 0) throw Error(POLFED_EINVAL, "step kernel: width not divisible by slices");
  // blocks beyond the Infinity Cache (256 MB) are swept as one row window
  // by all the XCDs of a slice; smaller ones keep a window per XCD
  a.interleave = ((double)a.n * S * sizeof(T) > 256.0 * 1024.0 * 1024.0) ? 1 : 0;
  S /= a.nslices;  // the kernel's template width is one slice
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
                         int B, long long j, long long Kmax, long long total_tiles,
                         const BatchTables &tables, const StepShape &shape, int num_cu) {
  if (total_tiles <= 0 || B <= 0) return;
  if (shape.threads != 256 && shape.threads != 512 && shape.threads != 1024)
    throw Error(POLFED_EINVAL, "step kernel: threads must be 256, 512 or 1024");
  const int ns = shape.xcd_slices;
  if (ns != 1 && ns != 2 && ns != 4 && ns != 8)
    throw Error(POLFED_EINVAL, "step kernel: column slices must be 1, 2, 4 or 8");
  if (S % ns != 0) throw Error(POLFED_EINVAL, "step kernel: width not divisible by slices");
  StepArgs<T> a0 = a;
  a0.nslices = ns;
  S /= ns;  // the kernel's template width is one slice
#define PF_BATCH_CASE(SS)                                                                  \
  case SS: {                                                                               \
    constexpr int M = max_lpl<T, SS>();                                                    \
    const int lpl = std::min(shape.lpl, M);                                                \
    if constexpr (M >= 4)                                                                  \
      if (lpl == 4) {                                                                      \
        launch_batched_s<T, SS, 4>(st, a0, items, B, j, Kmax, total_tiles, tables, shape,   \
                                   num_cu);                                                \
        break;                                                                             \
      }                                                                                    \
    if constexpr (M >= 2)                                                                  \
      if (lpl == 2) {                                                                      \
        launch_batched_s<T, SS, 2>(st, a0, items, B, j, Kmax, total_tiles, tables, shape,   \
                                   num_cu);                                                \
        break;                                                                             \
      }                                                                                    \
    launch_batched_s<T, SS, 1>(st, a0, items, B, j, Kmax, total_tiles, tables, shape,       \
                               num_cu);                                                    \
    break;                                                                                 \
  }
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

// Rows per tile of the batched kernel: the workgroup's waves times the rows
// a wave covers at the loads per lane the launcher picks for this width
// (split into the shape's column slices).
template <class T>
long long batched_tile_rows(int S, const StepShape &shape) {
  if (shape.xcd_slices > 1 && S % shape.xcd_slices == 0) S /= shape.xcd_slices;
  auto rows = [&](auto s_c) -> long long {
    constexpr int SS = decltype(s_c)::value;
    constexpr int M = max_lpl<T, SS>();
    const int lpl = std::min(shape.lpl, M);
    const int rpw = (lpl >= 4 && M >= 4) ? StepCfg<T, SS, (M >= 4 ? 4 : 1)>::RPW
                    : (lpl >= 2 && M >= 2) ? StepCfg<T, SS, (M >= 2 ? 2 : 1)>::RPW
                                           : StepCfg<T, SS, 1>::RPW;
    return (long long)(shape.threads / 64) * rpw;
  };
  switch (S) {
    case 1: return rows(std::integral_constant<int, 1>{});
    case 2: return rows(std::integral_constant<int, 2>{});
    case 4: return rows(std::integral_constant<int, 4>{});
    case 8: return rows(std::integral_constant<int, 8>{});
    case 16: return rows(std::integral_constant<int, 16>{});
    case 32: return rows(std::integral_constant<int, 32>{});
    case 64: return rows(std::integral_constant<int, 64>{});
    default: throw Error(POLFED_EINVAL, "block width must be a power of two in [1, 64]");
  }
}

}  // namespace polfed
