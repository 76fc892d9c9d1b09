// Observables of the returned eigenpairs (main text, "Entanglement entropy
// and level statistics"): the entanglement entropy of an eigenvector for a
// bipartition of the ring into two halves, and the mean gap ratio of the
// eigenvalues.
//
// Cut x (a bit offset): the first half holds bits x .. x+h-1 (mod L), h =
// L/2, the second the other h bits in ring order.  With t = s rotated right
// by x, a = t & (2^h - 1) and b = t >> h.  A state of zero magnetisation has
// popcount(a) = n and popcount(b) = h - n, so the coefficient matrix
// psi[a][b] is block diagonal by n: block n is C(h, n) x C(h, n), and the
// blocks hold exactly the C(L, h) coefficients (Vandermonde's identity).
// The squared Schmidt coefficients are the eigenvalues of the blocks' Gram
// matrices M_n^T M_n; S_E = -sum lambda ln lambda.
//
// Device steps: scatter each (vector, cut) into its blocks (row and column
// by the colex rank of a and b among patterns of their weight), form the
// block Gram matrices, take their eigenvalues with the batched LDS Jacobi
// (all blocks of one size at once; blocks up to 128 x 128, i.e. L <= 18),
// and sum -lambda ln lambda per (vector, cut).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace polfed {

__device__ __forceinline__ int colex_rank(uint32_t pat, int bits, const int32_t *binom) {
  int r = 0, t = 0;
  for (int q = 0; q < bits; ++q)
    if ((pat >> q) & 1u) r += binom[32 * q + (++t)];
  return r;
}

// out[p][off[n] + rb * d_n + ra] = V[r][j], pair p = j * ncut + c.
__global__ void k_ent_scatter(long long n, int L, const uint32_t *states, const double *V,
                              long long ldv, int ncut, const int *cuts, const int32_t *binom,
                              const long long *off, double *out, int p0) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int p = p0 + (int)blockIdx.y;
  const int j = p / ncut, c = p % ncut;
  const int h = L / 2;
  const int x = cuts[c];
  const uint32_t full = (L >= 32) ? 0xffffffffu : ((1u << L) - 1u);
  const uint32_t s = states[r];
  const uint32_t t = x ? (((s >> x) | (s << (L - x))) & full) : s;
  const uint32_t a = t & ((1u << h) - 1u), b = t >> h;
  const int na = __popc(a);
  const int d = binom[32 * h + na];
  const int ra = colex_rank(a, h, binom), rb = colex_rank(b, L - h, binom);
  out[(size_t)blockIdx.y * n + off[na] + (size_t)rb * d + ra] = V[(size_t)r * ldv + j];
}

// Gram matrix of block na for every pair: G[p][i][k] = sum_b M[p][b][i] M[p][b][k]
// (one workgroup per pair).
__global__ void k_ent_gram(long long n, int d, long long offn, const double *M, double *G) {
  const int p = blockIdx.x;
  const double *Mb = M + (size_t)p * n + offn;
  double *Gb = G + (size_t)p * d * d;
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const int i = e / d, k = e % d;
    if (k < i) continue;
    double acc = 0.0;
    for (int bb = 0; bb < d; ++bb) acc += Mb[(size_t)bb * d + i] * Mb[(size_t)bb * d + k];
    Gb[(size_t)i * d + k] = acc;
    Gb[(size_t)k * d + i] = acc;
  }
}

__global__ void k_eye_batch(int d, int B, double *V) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)B * d * d) return;
  const int w = (int)(e % ((long long)d * d));
  V[e] = (w / d == w % d) ? 1.0 : 0.0;
}

// S[p] += -sum_k lambda_k ln lambda_k over the d eigenvalues of pair p.
__global__ void k_ent_sum(int d, int B, const double *w, double *S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B) return;
  double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    const double lam = w[(size_t)p * d + k];
    if (lam > 1e-300) acc -= lam * log(lam);
  }
  S[p] += acc;
}

void entanglement_entropy(hipStream_t st, const Basis &bs, int nvec, const double *V,
                          long long ldv, const std::vector<int> &cuts, double *S_host,
                          DevBuf &work) {
  const int L = bs.L, h = L / 2;
  const long long n = bs.n;
  PF_REQUIRE(L >= 2 && L <= 18, "entanglement: L must be in [2, 18] (blocks up to 128 x 128)");
  const int ncut = (int)cuts.size();
  const long long npairs = (long long)nvec * ncut;
  std::vector<long long> d(h + 1), off(h + 2, 0);
  for (int k = 0; k <= h; ++k) {
    long long c = 1;
    for (int i = 1; i <= k; ++i) c = c * (h - k + i) / i;  // C(h, k)
    d[k] = c;
    off[k + 1] = off[k] + c * c;
  }
  PF_REQUIRE(off[h + 1] == n, "entanglement: block sizes do not add up to the sector");
  // pairs in chunks, each chunk's blocks, Gram matrices and eigenvalues
  // within a bounded workspace
  const long long chunk = std::max<long long>(1, std::min<long long>(npairs, 512));
  // workspace: S per pair, block offsets, cuts, then four 256-byte aligned
  // regions of n doubles per pair of the chunk
  const size_t small = sizeof(double) * npairs + sizeof(long long) * (h + 2) + sizeof(int) * ncut;
  const size_t per = sizeof(double) * (size_t)n;  // blocks of one pair
  char *ws = static_cast<char *>(work.ensure(small + 4 * per * chunk + 256));
  double *dS = reinterpret_cast<double *>(ws);
  long long *doff = reinterpret_cast<long long *>(ws + sizeof(double) * npairs);
  int *dcut = reinterpret_cast<int *>(ws + sizeof(double) * npairs + sizeof(long long) * (h + 2));
  double *M = reinterpret_cast<double *>(
      (reinterpret_cast<uintptr_t>(ws + small) + 255) & ~(uintptr_t)255);
  double *G = M + (size_t)n * chunk;
  double *Vs = G + (size_t)n * chunk;
  double *Vo = Vs + (size_t)n * chunk;
  PF_HIP(hipMemcpyAsync(doff, off.data(), sizeof(long long) * (h + 2), hipMemcpyHostToDevice, st));
  PF_HIP(hipMemcpyAsync(dcut, cuts.data(), sizeof(int) * ncut, hipMemcpyHostToDevice, st));
  launch_fill(st, dS, npairs, 0.0);
  for (long long p0 = 0; p0 < npairs; p0 += chunk) {
    const int B = (int)std::min<long long>(chunk, npairs - p0);
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)B);
    k_ent_scatter<<<grid, 256, 0, st>>>(n, L, bs.states.as<uint32_t>(), V, ldv, ncut, dcut,
                                        bs.binom.as<int32_t>(), doff, M, (int)p0);
    check_launch("k_ent_scatter");
    for (int k = 0; k <= h; ++k) {
      // block k of every pair: Gram matrices (G), starting vectors (Vs),
      // eigenvectors and then eigenvalues (Vo): B (dk^2 + dk) <= B n doubles,
      // as the largest block appears twice in the sector (h >= 3) or fills it
      const int dk = (int)d[k];
      k_ent_gram<<<B, 256, 0, st>>>(n, dk, off[k], M, G);
      check_launch("k_ent_gram");
      const long long tot = (long long)B * dk * dk;
      k_eye_batch<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(dk, B, Vs);
      check_launch("k_eye_batch");
      double *w = Vo + (size_t)B * dk * dk;
      if (!sym_eig_batched(st, dk, B, G, Vs, w, Vo))
        throw Error(POLFED_EINVAL, "entanglement: block of size " + std::to_string(dk) +
                                       " beyond the batched eigensolver (L <= 18)");
      k_ent_sum<<<(B + 255) / 256, 256, 0, st>>>(dk, B, w, dS + p0);
      check_launch("k_ent_sum");
    }
  }
  PF_HIP(hipMemcpyAsync(S_host, dS, sizeof(double) * npairs, hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
}

}  // namespace polfed

namespace polfed {

double mean_gap_ratio(const double *E, int n) {
  std::vector<double> e(E, E + n);
  std::sort(e.begin(), e.end());
  double acc = 0.0;
  for (int i = 0; i + 2 < n; ++i) {
    const double g1 = e[i + 1] - e[i], g2 = e[i + 2] - e[i + 1];
    const double lo = std::min(g1, g2), hi = std::max(g1, g2);
    acc += (hi > 0.0) ? lo / hi : 0.0;
  }
  return acc / (n - 2);
}

}  // namespace polfed
