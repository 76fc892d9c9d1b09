// Sz=0 basis of the spin chain: enumeration, ranking and the diagonal of H.
//
// The sector of zero magnetisation holds the C(L, L/2) L-bit integers with
// L/2 set bits (paper, "Benchmark models").  Row r is the r-th such integer
// in ascending order; ascending order of fixed-weight bit strings is the
// colexicographic order of their set-bit positions p_1 < ... < p_{L/2}, whose
// rank is sum_t C(p_t, t).  Unranking inverts that sum greedily from the top
// bit.  Ranking uses two tables split at bit `half` = L/2: the low half
// contributes sum over its own set bits, and the high half's bits have
// known index t = (L/2 - popcount(hi)) + u, so each half's term is a table
// lookup and rank(s) = tabA[hi] + tabB[lo].  tabB[lo] is a rank among the
// C(half, popcount(lo)) <= C(15, 7) low patterns and fits 16 bits.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace polfed {

__constant__ uint32_t c_binom[33][33];  // C(n, k), n, k <= 32 (C(32,16) < 2^32)

void upload_binomials(int device) {
  static bool done[64] = {false};
  if (device >= 0 && device < 64 && done[device]) return;
  uint32_t tab[33][33];
  for (int n = 0; n <= 32; ++n)
    for (int k = 0; k <= 32; ++k) {
      if (k > n) tab[n][k] = 0;
      else if (k == 0 || k == n) tab[n][k] = 1;
      else tab[n][k] = tab[n - 1][k - 1] + tab[n - 1][k];
    }
  PF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_binom), tab, sizeof(tab)));
  if (device >= 0 && device < 64) done[device] = true;
}

__global__ void k_unrank(uint32_t *states, long long n, int L) {
  long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  uint32_t rem = (uint32_t)r;
  uint32_t s = 0;
  int p = L - 1;
  for (int t = L / 2; t >= 1; --t) {
    while (c_binom[p][t] > rem) --p;  // stops at p >= t-1, where C(p,t) = 0
    s |= 1u << p;
    rem -= c_binom[p][t];
    --p;
  }
  states[r] = s;
}

// tabB[lo] = sum over set bits q (ascending, index t = 1, 2, ...) of C(q, t)
// tabA[hi] = sum over set bits q of hi (index t continuing after the
//            L/2 - popcount(hi) bits below) of C(half + q, t)
__global__ void k_rank_tables(int32_t *tabA, uint16_t *tabB, int L, int half) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (1 << half)) return;
  int t = 0;
  uint32_t sb = 0;
  for (int q = 0; q < half; ++q)
    if ((x >> q) & 1) sb += c_binom[q][++t];
  tabB[x] = (uint16_t)sb;
  int below = L / 2 - __popc((uint32_t)x);
  uint32_t sa = 0;
  if (below >= 0) {
    t = below;
    for (int q = 0; q < L - half; ++q)
      if ((x >> q) & 1) sa += c_binom[half + q][++t];
  }
  tabA[x] = (int32_t)sa;
}

__global__ void k_rank(const uint32_t *states, int32_t *ranks, long long n, const int32_t *tabA,
                       const uint16_t *tabB, int L, int half) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t s = states[i];
  bool ok = (L >= 32 || (s >> L) == 0) && __popc(s) == L / 2;
  ranks[i] = ok ? tabA[s >> half] + tabB[s & ((1u << half) - 1u)] : -1;
}

__global__ void k_binom_table(int32_t *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 32 * 32) out[i] = (int32_t)c_binom[i >> 5][i & 31];  // C(31, k) < 2^31
}

void build_basis(hipStream_t st, Basis &b, int L) {
  b.L = L;
  b.half = L / 2;
  b.n = polfed_dim(L);
  b.states.ensure(sizeof(uint32_t) * b.n);
  b.tabA.ensure(sizeof(int32_t) << b.half);
  b.tabB.ensure(sizeof(uint16_t) << b.half);
  int th = 256;
  k_unrank<<<(unsigned)((b.n + th - 1) / th), th, 0, st>>>(b.states.as<uint32_t>(), b.n, L);
  check_launch("k_unrank");
  k_rank_tables<<<(unsigned)(((1 << b.half) + th - 1) / th), th, 0, st>>>(
      b.tabA.as<int32_t>(), b.tabB.as<uint16_t>(), L, b.half);
  check_launch("k_rank_tables");
  b.binom.ensure(sizeof(int32_t) * 32 * 32);
  k_binom_table<<<4, 256, 0, st>>>(b.binom.as<int32_t>());
  check_launch("k_binom_table");
}

void launch_rank(hipStream_t st, const Basis &b, long long n, const uint32_t *states,
                 int32_t *ranks) {
  if (n <= 0) return;
  int th = 256;
  k_rank<<<(unsigned)((n + th - 1) / th), th, 0, st>>>(states, ranks, n, b.tabA.as<int32_t>(),
                                                      b.tabB.as<uint16_t>(), b.L, b.half);
  check_launch("k_rank");
}

// ---- stored neighbour pattern (rank mode 2 of the step kernel) ----------

__device__ __forceinline__ unsigned long long bond_mask(uint32_t s, int L, int has_j2) {
  const uint32_t full = (L >= 32) ? 0xffffffffu : ((1u << L) - 1u);
  const uint32_t rot1 = ((s >> 1) | (s << (L - 1))) & full;
  unsigned long long mm = (unsigned long long)(s ^ rot1);
  if (has_j2) {
    const uint32_t rot2 = ((s >> 2) | (s << (L - 2))) & full;
    mm |= (unsigned long long)(s ^ rot2) << 32;
  }
  return mm;
}

// counts of one block of 1024 rows: cnt[r] and the block total
__global__ __launch_bounds__(1024) void k_pattern_count(const uint32_t *states, long long n,
                                                         int L, int has_j2, long long *ptr,
                                                         long long *bsum) {
  __shared__ long long sh[1024];
  const long long r = (long long)blockIdx.x * 1024 + threadIdx.x;
  const long long c = (r < n) ? (long long)__popcll(bond_mask(states[r], L, has_j2)) : 0;
  sh[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {  // exclusive scan of the block, in order
    long long run = 0;
    for (int i = 0; i < 1024; ++i) {
      const long long v = sh[i];
      sh[i] = run;
      run += v;
    }
    bsum[blockIdx.x] = run;
  }
  __syncthreads();
  if (r < n) ptr[r] = sh[threadIdx.x];
}

__global__ void k_pattern_offsets(long long n, const long long *boff, long long *ptr,
                                  long long nnz) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) ptr[r] += boff[r / 1024];
  if (r == n) ptr[n] = nnz;
}

// col[ptr[r] ..]: the neighbours of row r in the step kernel's bond order
__global__ void k_pattern_fill(const uint32_t *states, long long n, int L, int half, int has_j2,
                               const int32_t *tabA, const uint16_t *tabB, const long long *ptr,
                               int32_t *col) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t s = states[r];
  unsigned long long mm = bond_mask(s, L, has_j2);
  const uint32_t lomask = (1u << half) - 1u;
  long long q = ptr[r];
  while (mm) {
    const int bit = __ffsll((long long)mm) - 1;
    mm &= mm - 1ull;
    const int l = (bit >= 32) ? 2 : 1;
    const int i = bit & 31;
    int j = i + l;
    if (j >= L) j -= L;
    const uint32_t f = s ^ ((1u << i) | (1u << j));
    const int32_t rk = tabA[f >> half] + (int32_t)tabB[f & lomask];
    col[q++] = (l == 2) ? (int32_t)((uint32_t)rk | 0x80000000u) : rk;
  }
}

void build_pattern(hipStream_t st, const Basis &b, bool has_j2, Pattern &pat) {
  const long long n = b.n;
  const long long nb = (n + 1023) / 1024;
  pat.n = n;
  long long *ptr = static_cast<long long *>(pat.ptr.ensure(sizeof(long long) * (n + 1)));
  DevBuf bsum;
  long long *dsum = static_cast<long long *>(bsum.ensure(sizeof(long long) * nb));
  k_pattern_count<<<(unsigned)nb, 1024, 0, st>>>(b.states.as<uint32_t>(), n, b.L, has_j2 ? 1 : 0,
                                                 ptr, dsum);
  check_launch("k_pattern_count");
  std::vector<long long> hs(nb), ho(nb);
  PF_HIP(hipMemcpyAsync(hs.data(), dsum, sizeof(long long) * nb, hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
  long long run = 0;
  for (long long i = 0; i < nb; ++i) {
    ho[i] = run;
    run += hs[i];
  }
  PF_REQUIRE(run < (1LL << 40), "pattern too large");
  pat.nnz = run;
  PF_HIP(hipMemcpyAsync(dsum, ho.data(), sizeof(long long) * nb, hipMemcpyHostToDevice, st));
  const int th = 256;
  k_pattern_offsets<<<(unsigned)((n + 1 + th - 1) / th), th, 0, st>>>(n, dsum, ptr, run);
  check_launch("k_pattern_offsets");
  int32_t *col = static_cast<int32_t *>(pat.col.ensure(sizeof(int32_t) * std::max<long long>(1, run)));
  k_pattern_fill<<<(unsigned)((n + th - 1) / th), th, 0, st>>>(
      b.states.as<uint32_t>(), n, b.L, b.half, has_j2 ? 1 : 0, b.tabA.as<int32_t>(),
      b.tabB.as<uint16_t>(), ptr, col);
  check_launch("k_pattern_fill");
  PF_HIP(hipStreamSynchronize(st));  // bsum is freed on return
}

struct DiagArgs {
  double h[32];
  double J1, J2, Delta;
  int L;
};

// H[r][r] = sum_l (J_l Delta / 4) (L - 2 popcount(s ^ rot_l(s)))
//           + sum_{i set} h_i - (1/2) sum_i h_i
// where bit i of s ^ rot_l(s) marks an antiparallel bond (i, i+l mod L);
// each bond contributes +1/4 (parallel) or -1/4 (antiparallel) times J_l
// Delta, and the field term is h_i S^z_i with S^z = n_i - 1/2.
__global__ void k_diag(const uint32_t *states, double *d, long long n, DiagArgs a) {
  long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  uint32_t s = states[r];
  int L = a.L;
  uint32_t mask = (L >= 32) ? 0xffffffffu : ((1u << L) - 1u);
  uint32_t rot1 = ((s >> 1) | (s << (L - 1))) & mask;
  int anti1 = __popc(s ^ rot1);
  double v = 0.25 * a.J1 * a.Delta * (double)(L - 2 * anti1);
  if (a.J2 != 0.0) {
    uint32_t rot2 = ((s >> 2) | (s << (L - 2))) & mask;
    int anti2 = __popc(s ^ rot2);
    v += 0.25 * a.J2 * a.Delta * (double)(L - 2 * anti2);
  }
  double hs = 0.0, htot = 0.0;
  for (int i = 0; i < L; ++i) {
    htot += a.h[i];
    if ((s >> i) & 1u) hs += a.h[i];
  }
  d[r] = v + hs - 0.5 * htot;
}

void launch_diag(hipStream_t st, const Chain &c, double *d) {
  DiagArgs a;
  for (int i = 0; i < 32; ++i) a.h[i] = (i < c.L) ? c.h[i] : 0.0;
  a.J1 = c.J1;
  a.J2 = c.J2;
  a.Delta = c.Delta;
  a.L = c.L;
  long long n = c.basis->n;
  int th = 256;
  k_diag<<<(unsigned)((n + th - 1) / th), th, 0, st>>>(c.basis->states.as<uint32_t>(), d, n, a);
  check_launch("k_diag");
}

// dt[r] = a d[r] + b, rounded to T: the diagonal of H~ = aH + b.
template <class T>
__global__ void k_scaled_diag(long long n, const double *d, double a, double b, T *out) {
  long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[r] = (T)(a * d[r] + b);
}

template <class T>
void launch_scaled_diag(hipStream_t st, long long n, const double *d, double a, double b,
                        T *out) {
  int th = 256;
  k_scaled_diag<T><<<(unsigned)((n + th - 1) / th), th, 0, st>>>(n, d, a, b, out);
  check_launch("k_scaled_diag");
}

template void launch_scaled_diag<float>(hipStream_t, long long, const double *, double, double,
                                        float *);
template void launch_scaled_diag<double>(hipStream_t, long long, const double *, double, double,
                                         double *);

}  // namespace polfed
