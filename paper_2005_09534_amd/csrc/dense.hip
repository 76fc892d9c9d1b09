// Dense FP64 kernels of the block-Lanczos side of POLFED.
//
// * Tall-skinny products on the matrix cores (v_mfma_f64_16x16x4f64):
//     gram   C = X^T Y   (A_j = Q_j^T U_j of eq. (Lan1), the projections
//                         Qm^T U of the full reorthogonalisation, U^T U of
//                         the QR step and U^T H~ U of Rayleigh-Ritz)
//     update Y = alpha X C + beta Y  (U - Q_{j-1} B_j^T, U - Q_j A_j,
//                         U - Qm (Qm^T U), Q = U R^{-1}, Ritz vectors Qm T)
//   The reduction of gram over rows is two-stage (per-workgroup partials,
//   then a fixed-order sum), so results are bitwise reproducible.
// * A cyclic Jacobi eigensolver (round-robin parallel ordering) for T_m and
//   the Rayleigh-Ritz matrix: one launch per round over the whole matrix,
//   double-buffered so that every workgroup derives the round's rotations
//   from an unmodified input; the host checks the off-diagonal norm between
//   sweeps.
// * Cholesky of the s x s Gram matrix for CholeskyQR.
// * Column reductions, Philox4x32-10 start vectors, and the single-vector
//   Lanczos helpers for the spectral bounds.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace polfed {

typedef double d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ gram --
//
// Workgroup = 4 waves; it owns a 64 (columns of X) x 64 (columns of Y)
// output tile and a contiguous chunk of rows.  Wave w owns output rows
// [16w, 16w+16) of the tile, i.e. 1 x 4 MFMA tiles of 16 x 16.  One MFMA
// step contracts 4 rows: lane l supplies A[i=l%16][k=l/16] = X[row0+k][ci]
// and B[k=l/16][j=l%16] = Y[row0+k][cj]; the result tile holds
// D[l/16 + 4v][l%16] in component v of lane l (checked on gfx950).

constexpr int kGramTM = 64, kGramTN = 64;

__global__ __launch_bounds__(256) void k_gram(long long n, int p, int q, const double *X,
                                              long long ldx, const double *Y, long long ldy,
                                              double *part, long long rows_per_chunk,
                                              int tiles_m, int tiles_n) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int t = blockIdx.x;
  const int tm = t % tiles_m;
  t /= tiles_m;
  const int tn = t % tiles_n;
  const int chunk = t / tiles_n;
  const long long r0 = (long long)chunk * rows_per_chunk;
  long long r1 = r0 + rows_per_chunk;
  if (r1 > n) r1 = n;

  const int ci = tm * kGramTM + wave * 16 + (lane & 15);  // X column for A operand
  const int kk = lane >> 4;                                // row within the 4-row step
  const bool ci_ok = ci < p;
  int cj[4];
  bool cj_ok[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    cj[u] = tn * kGramTN + u * 16 + (lane & 15);
    cj_ok[u] = cj[u] < q;
  }
  d4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = (d4){0.0, 0.0, 0.0, 0.0};

  long long r = r0;
  for (; r + 16 <= r1; r += 16) {
    double av[4], bv[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const long long row = r + 4 * s + kk;
      av[s] = ci_ok ? X[row * ldx + ci] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) bv[s][u] = cj_ok[u] ? Y[row * ldy + cj[u]] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s][u], acc[u], 0, 0, 0);
  }
  for (; r < r1; r += 4) {
    const long long row = r + kk;
    const bool rok = row < r1;
    const double a = (rok && ci_ok) ? X[row * ldx + ci] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double bb = (rok && cj_ok[u]) ? Y[row * ldy + cj[u]] : 0.0;
      acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc[u], 0, 0, 0);
    }
  }
  // partial tile -> part[chunk][i][j] (p x q, row-major)
  double *out = part + (size_t)chunk * p * q;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = tn * kGramTN + u * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = tm * kGramTM + wave * 16 + (lane >> 4) + 4 * v;
      if (i < p && j < q) out[(size_t)i * q + j] = acc[u][v];
    }
  }
}

// C[i][j] = sum over chunks c of part[c][i][j]: one wavefront per output
// element, lane l adding chunks l, l + 64, ... in order, then a fixed
// butterfly over the lanes, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_gram_reduce(int p, int q, int nchunks,
                                                     const double *part, double *C,
                                                     long long ldc) {
  const long long e = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= (long long)p * q) return;
  const size_t pq = (size_t)p * q;
  double s = 0.0;
  for (int c = lane; c < nchunks; c += 64) s += part[(size_t)c * pq + e];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
  if (lane == 0) {
    const int i = (int)(e / q), j = (int)(e % q);
    C[(size_t)i * ldc + j] = s;
  }
}

// Row chunks of the Gram product for n rows and a p x q output: about four
// workgroups per CU in all, at least 256 rows a chunk, and (cap > 0) no
// more chunks than cap / (p q) partial tiles hold.
long long gram_chunks(long long n, int p, int q, int num_cu, long long cap,
                      long long &rows_per_chunk) {
  const int tiles_m = (p + kGramTM - 1) / kGramTM;
  const int tiles_n = (q + kGramTN - 1) / kGramTN;
  long long want = std::max<long long>(1, (4LL * num_cu) / (tiles_m * tiles_n));
  if (cap > 0) want = std::min<long long>(want, cap / ((long long)p * q));
  want = std::max<long long>(want, 1);
  rows_per_chunk = std::max<long long>(256, (n + want - 1) / want);
  rows_per_chunk = ((rows_per_chunk + 15) / 16) * 16;
  return std::max<long long>(1, (n + rows_per_chunk - 1) / rows_per_chunk);
}

void launch_gram_parts(hipStream_t st, long long n, int p, int q, const double *X,
                       long long ldx, const double *Y, long long ldy, double *C, long long ldc,
                       double *part, long long rows_per_chunk, long long nchunks) {
  const int tiles_m = (p + kGramTM - 1) / kGramTM;
  const int tiles_n = (q + kGramTN - 1) / kGramTN;
  const long long nblk = nchunks * tiles_m * tiles_n;
  k_gram<<<(unsigned)nblk, 256, 0, st>>>(n, p, q, X, ldx, Y, ldy, part, rows_per_chunk, tiles_m,
                                         tiles_n);
  check_launch("k_gram");
  const long long tot = (long long)p * q;
  k_gram_reduce<<<(unsigned)((tot + 3) / 4), 256, 0, st>>>(p, q, (int)nchunks, part, C, ldc);
  check_launch("k_gram_reduce");
}

void launch_gram(hipStream_t st, long long n, int p, int q, const double *X, long long ldx,
                 const double *Y, long long ldy, double *C, long long ldc, DevBuf &partials,
                 int num_cu) {
  if (p <= 0 || q <= 0) return;
  long long rows_per_chunk = 0;
  const long long nchunks = gram_chunks(n, p, q, num_cu, 0, rows_per_chunk);
  double *part = static_cast<double *>(partials.ensure(sizeof(double) * nchunks * p * q));
  launch_gram_parts(st, n, p, q, X, ldx, Y, ldy, C, ldc, part, rows_per_chunk, nchunks);
}

// ---------------------------------------------------------------- update --
//
// Workgroup = 4 waves, 64 rows; wave w owns rows [16w, 16w+16) and all q
// (<= 64) columns as up to 4 MFMA tiles.  Lane l supplies
// A[i=l%16][k=l/16] = X[row0+i][k0+k] and B[k=l/16][j=l%16] = C[k0+k][j];
// result component v of lane l is D[l/16 + 4v][l%16].

__global__ __launch_bounds__(256) void k_update(long long n, int p, int q, double alpha,
                                                const double *X, long long ldx, const double *C,
                                                long long ldc, double beta, double *Y,
                                                long long ldy) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const long long row0 = (long long)blockIdx.x * 64 + wave * 16;
  const long long ra = row0 + (lane & 15);
  const bool ra_ok = ra < n;
  const int kk = lane >> 4;
  const int ntile = (q + 15) / 16;
  d4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < p; k0 += 4) {
    const int k = k0 + kk;
    const bool k_ok = k < p;
    const double a = (ra_ok && k_ok) ? X[ra * ldx + k] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < ntile) {
        const int j = u * 16 + (lane & 15);
        const double b = (k_ok && j < q) ? C[(size_t)k * ldc + j] : 0.0;
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (u < ntile) {
      const int j = u * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long long row = row0 + (lane >> 4) + 4 * v;
        if (row < n && j < q) {
          double *y = Y + row * ldy + j;
          *y = (beta == 0.0) ? alpha * acc[u][v] : alpha * acc[u][v] + beta * (*y);
        }
      }
    }
  }
}

void launch_update(hipStream_t st, long long n, int p, int q, double alpha, const double *X,
                   long long ldx, const double *C, long long ldc, double beta, double *Y,
                   long long ldy) {
  if (n <= 0 || q <= 0) return;
  if (q > 64) throw Error(POLFED_EINVAL, "update: q must be <= 64");
  if (p <= 0) {
    // Y = beta Y
    launch_update(st, n, 1, q, 0.0, X, ldx, C, ldc, beta, Y, ldy);
    return;
  }
  k_update<<<(unsigned)((n + 63) / 64), 256, 0, st>>>(n, p, q, alpha, X, ldx, C, ldc, beta, Y,
                                                      ldy);
  check_launch("k_update");
}

// --------------------------------------------------------- small gemm --

__global__ void k_small_gemm(int m, int l, int k, const double *A, int lda, const double *B,
                             int ldb, double *C, int ldc, int transA) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * k) return;
  int i = e / k, j = e % k;
  double s = 0.0;
  for (int t = 0; t < l; ++t) {
    double a = transA ? A[(size_t)t * lda + i] : A[(size_t)i * lda + t];
    s += a * B[(size_t)t * ldb + j];
  }
  C[(size_t)i * ldc + j] = s;
}

void launch_small_gemm(hipStream_t st, int m, int l, int k, const double *A, int lda,
                       const double *B, int ldb, double *C, int ldc, int transA) {
  if (m <= 0 || k <= 0) return;
  int tot = m * k;
  k_small_gemm<<<(tot + 255) / 256, 256, 0, st>>>(m, l, k, A, lda, B, ldb, C, ldc, transA);
  check_launch("k_small_gemm");
}

// -------------------------------------------------------------- cholesky --
//
// G = L L^T (s <= 64, one workgroup, G staged in LDS).  Writes B = L^T
// (upper triangular, the R factor of U = Q R) and Rinv = L^{-T}, so that
// Q = U Rinv.  flag[0] = 1 + index of the first pivot <= rel_tol * max
// diag(G) (0 if none).

__global__ __launch_bounds__(256) void k_chol(int s, const double *G, double *Rinv, double *B,
                                              int *flag, double rel_tol) {
  __shared__ double a[64 * 64];
  __shared__ double dmax;
  __shared__ int bad;
  const int t = threadIdx.x;
  for (int e = t; e < s * s; e += blockDim.x) a[e] = G[e];
  if (t == 0) {
    double m = 0.0;
    for (int i = 0; i < s; ++i) m = fmax(m, G[i * s + i]);
    dmax = m;
    bad = 0;
  }
  __syncthreads();
  for (int k = 0; k < s; ++k) {
    if (t == 0) {
      double d = a[k * s + k];
      if (!(d > rel_tol * dmax) && bad == 0) bad = k + 1;
      a[k * s + k] = (d > 0.0 && bad == 0) ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double lkk = a[k * s + k];
    for (int i = k + 1 + t; i < s; i += blockDim.x) a[i * s + k] /= lkk;
    __syncthreads();
    for (int e = t; e < (s - k - 1) * (s - k - 1); e += blockDim.x) {
      int i = k + 1 + e / (s - k - 1), j = k + 1 + e % (s - k - 1);
      if (j <= i) a[i * s + j] -= a[i * s + k] * a[j * s + k];
    }
    __syncthreads();
  }
  // column j of L^{-1} by forward substitution, one column per thread,
  // stored transposed: Rinv[j][i] = (L^{-1})[i][j]  (upper triangular)
  for (int j = t; j < s; j += blockDim.x) {
    double *row = Rinv + (size_t)j * s;
    for (int i = 0; i < j; ++i) row[i] = 0.0;
    row[j] = 1.0 / a[j * s + j];
    for (int i = j + 1; i < s; ++i) {
      double sum = 0.0;
      for (int k = j; k < i; ++k) sum += a[i * s + k] * row[k];
      row[i] = -sum / a[i * s + i];
    }
  }
  for (int e = t; e < s * s; e += blockDim.x) {
    int i = e / s, j = e % s;
    B[e] = (j >= i) ? a[j * s + i] : 0.0;  // L^T
  }
  if (t == 0) flag[0] = bad;
}

void launch_chol(hipStream_t st, int s, const double *G, double *Rinv, double *B, int *flag,
                 double rel_tol) {
  if (s > 64) throw Error(POLFED_EINVAL, "cholesky: s must be <= 64");
  k_chol<<<1, 256, 0, st>>>(s, G, Rinv, B, flag, rel_tol);
  check_launch("k_chol");
}

// out = in^T (s x s, row-major);  sym: in = (in + in^T)/2 in place
__global__ void k_small_transpose(int m, int k, const double *in, int ldi, double *out, int ldo) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * k) return;
  int i = e / k, j = e % k;
  out[(size_t)j * ldo + i] = in[(size_t)i * ldi + j];
}

__global__ void k_symmetrize(int s, double *A, int lda) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s * s) return;
  int i = e / s, j = e % s;
  if (j <= i) return;
  double v = 0.5 * (A[(size_t)i * lda + j] + A[(size_t)j * lda + i]);
  A[(size_t)i * lda + j] = v;
  A[(size_t)j * lda + i] = v;
}

void launch_small_transpose(hipStream_t st, int m, int k, const double *in, int ldi, double *out,
                            int ldo) {
  if (m <= 0 || k <= 0) return;
  k_small_transpose<<<(m * k + 255) / 256, 256, 0, st>>>(m, k, in, ldi, out, ldo);
  check_launch("k_small_transpose");
}

void launch_symmetrize(hipStream_t st, int s, double *A, int lda) {
  if (s <= 0) return;
  k_symmetrize<<<(s * s + 255) / 256, 256, 0, st>>>(s, A, lda);
  check_launch("k_symmetrize");
}

// ---------------------------------------------------------------- jacobi --
//
// Cyclic Jacobi with the round-robin ("tournament") ordering: with m = n
// rounded up to even, round r pairs position 0 with position m-1 and k
// with m-1-k, where position i >= 1 holds index 1 + (i - 1 + r) mod (m-1);
// over m-1 rounds every pair meets once.  A round computes the n/2
// rotations from the current A, then applies J^T A J block-wise (each
// 2 x 2 block of rows {p1,q1} x cols {p2,q2} is owned by one thread) and
// V <- V J.  The rotation J = [[c, s], [-s, c]] on (p, q) annihilates
// a_pq with t = sign(th)/(|th| + sqrt(th^2+1)), th = (a_qq - a_pp)/(2 a_pq).

__device__ __forceinline__ int rr_index(int i, int r, int m) {
  return (i == 0) ? 0 : 1 + (i - 1 + r) % (m - 1);
}

// Rotation of pair k in round r, computed from the round's input matrix
// (which no thread of the round writes), so every workgroup that needs it
// gets the same (p, q, c, s).
__device__ __forceinline__ void jacobi_rotation(const double *A, int n, int m, int r, int k,
                                                int &p, int &q, double &c, double &s) {
  p = rr_index(k, r, m);
  q = rr_index(m - 1 - k, r, m);
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
  c = 1.0;
  s = 0.0;
  if (q < n) {
    const double apq = A[(size_t)p * n + q];
    if (apq != 0.0) {
      const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
      const double th = (aqq - app) / (2.0 * apq);
      double tt = 1.0 / (fabs(th) + sqrt(th * th + 1.0));
      if (th < 0.0) tt = -tt;
      c = 1.0 / sqrt(tt * tt + 1.0);
      s = tt * c;
    }
  }
}

// One round over the whole matrix: Aout = J^T Ain J (2 x 2 blocks, one per
// thread, 16 x 16 pair-blocks per workgroup) and V <- V J in place (16 rows
// x 16 pairs per workgroup).  Workgroups [0, nta) do A tiles, the rest V.
constexpr int kJT = 16;
// Largest matrix the batched LDS Jacobi takes (n^2 doubles + 16 KB of LDS).
constexpr int kLdsEigMax = 128;

__global__ __launch_bounds__(256) void k_jacobi_round(int n, int r, const double *Ain,
                                                      double *Aout, double *V, int tiles_a) {
  __shared__ int sp[2][kJT], sq[2][kJT];
  __shared__ double sc[2][kJT], ss[2][kJT];
  const int m = n + (n & 1);
  const int npair = m / 2;
  const int tp = (npair + kJT - 1) / kJT;
  const int t = threadIdx.x;
  const int ty = t / kJT, tx = t % kJT;
  int blk = blockIdx.x;
  if (blk < tiles_a) {
    const int tk1 = blk / tp, tk2 = blk % tp;
    if (t < 2 * kJT) {
      const int which = t / kJT, i = t % kJT;
      const int k = (which == 0 ? tk1 : tk2) * kJT + i;
      int p = 0, q = n;
      double c = 1.0, s = 0.0;
      if (k < npair) jacobi_rotation(Ain, n, m, r, k, p, q, c, s);
      sp[which][i] = p; sq[which][i] = q; sc[which][i] = c; ss[which][i] = s;
    }
    __syncthreads();
    const int k1 = tk1 * kJT + ty, k2 = tk2 * kJT + tx;
    if (k1 >= npair || k2 >= npair) return;
    const int p1 = sp[0][ty], q1 = sq[0][ty], p2 = sp[1][tx], q2 = sq[1][tx];
    const double c1 = sc[0][ty], s1 = ss[0][ty], c2 = sc[1][tx], s2 = ss[1][tx];
    const bool q1ok = q1 < n, q2ok = q2 < n;
    const double a00 = Ain[(size_t)p1 * n + p2];
    const double a01 = q2ok ? Ain[(size_t)p1 * n + q2] : 0.0;
    const double a10 = q1ok ? Ain[(size_t)q1 * n + p2] : 0.0;
    const double a11 = (q1ok && q2ok) ? Ain[(size_t)q1 * n + q2] : 0.0;
    // rows: R1^T = [[c1, -s1], [s1, c1]]; cols: R2 = [[c2, s2], [-s2, c2]]
    const double b00 = c1 * a00 - s1 * a10, b01 = c1 * a01 - s1 * a11;
    const double b10 = s1 * a00 + c1 * a10, b11 = s1 * a01 + c1 * a11;
    Aout[(size_t)p1 * n + p2] = b00 * c2 - b01 * s2;
    if (q2ok) Aout[(size_t)p1 * n + q2] = b00 * s2 + b01 * c2;
    if (q1ok) Aout[(size_t)q1 * n + p2] = b10 * c2 - b11 * s2;
    if (q1ok && q2ok) Aout[(size_t)q1 * n + q2] = b10 * s2 + b11 * c2;
  } else {
    blk -= tiles_a;
    const int ti = blk / tp, tk = blk % tp;
    if (t < kJT) {
      const int k = tk * kJT + t;
      int p = 0, q = n;
      double c = 1.0, s = 0.0;
      if (k < npair) jacobi_rotation(Ain, n, m, r, k, p, q, c, s);
      sp[0][t] = p; sq[0][t] = q; sc[0][t] = c; ss[0][t] = s;
    }
    __syncthreads();
    const int i = ti * kJT + ty, k = tk * kJT + tx;
    if (i >= n || k >= npair) return;
    const int p = sp[0][tx], q = sq[0][tx];
    if (q >= n) return;
    const double c = sc[0][tx], s = ss[0][tx];
    const double vp = V[(size_t)i * n + p], vq = V[(size_t)i * n + q];
    V[(size_t)i * n + p] = c * vp - s * vq;
    V[(size_t)i * n + q] = s * vp + c * vq;
  }
}

// Batched cyclic Jacobi for many small symmetric matrices of one size: one
// workgroup per matrix with the matrix in LDS, the eigenvectors accumulated
// in global memory.  The rotations (round-robin pairs, same formula as
// jacobi_rotation), the in-place 2 x 2 block updates and the stopping rule
// are those of sym_eig, applied to each matrix on its own, so that many
// Lanczos convergence checks of one batch run in a single launch.
__global__ __launch_bounds__(1024) void k_jacobi_lds(int n, double *A, double *V, double *w,
                                                     double *Vout, int max_sweeps) {
  extern __shared__ double sA[];  // n * n, then 2 * 1024 for reductions
  __shared__ int sp[kLdsEigMax / 2], sq[kLdsEigMax / 2];
  __shared__ double sc[kLdsEigMax / 2], ss[kLdsEigMax / 2];
  __shared__ int s_stop;
  double *red = sA + (size_t)n * n;
  const int t = threadIdx.x, nt = blockDim.x;
  const size_t nn = (size_t)n * n;
  double *Ab = A + (size_t)blockIdx.x * nn;
  double *Vb = V + (size_t)blockIdx.x * nn;
  for (size_t e = t; e < nn; e += nt) sA[e] = Ab[e];
  __syncthreads();
  const int m = n + (n & 1);
  const int npair = m / 2;
  double prev = -1.0;
  for (int sweep = 0; sweep < max_sweeps && n > 1; ++sweep) {
    for (int r = 0; r < m - 1; ++r) {
      if (t < npair) {
        int p, q;
        double c, sn;
        jacobi_rotation(sA, n, m, r, t, p, q, c, sn);
        sp[t] = p;
        sq[t] = q;
        sc[t] = c;
        ss[t] = sn;
      }
      __syncthreads();
      // A <- J^T A J: the 2 x 2 blocks (pair k1 rows, pair k2 columns) are
      // disjoint, each read and written by one thread
      for (int idx = t; idx < npair * npair; idx += nt) {
        const int k1 = idx / npair, k2 = idx % npair;
        const int p1 = sp[k1], q1 = sq[k1], p2 = sp[k2], q2 = sq[k2];
        const double c1 = sc[k1], s1 = ss[k1], c2 = sc[k2], s2 = ss[k2];
        const bool q1ok = q1 < n, q2ok = q2 < n;
        const double a00 = sA[(size_t)p1 * n + p2];
        const double a01 = q2ok ? sA[(size_t)p1 * n + q2] : 0.0;
        const double a10 = q1ok ? sA[(size_t)q1 * n + p2] : 0.0;
        const double a11 = (q1ok && q2ok) ? sA[(size_t)q1 * n + q2] : 0.0;
        const double b00 = c1 * a00 - s1 * a10, b01 = c1 * a01 - s1 * a11;
        const double b10 = s1 * a00 + c1 * a10, b11 = s1 * a01 + c1 * a11;
        sA[(size_t)p1 * n + p2] = b00 * c2 - b01 * s2;
        if (q2ok) sA[(size_t)p1 * n + q2] = b00 * s2 + b01 * c2;
        if (q1ok) sA[(size_t)q1 * n + p2] = b10 * c2 - b11 * s2;
        if (q1ok && q2ok) sA[(size_t)q1 * n + q2] = b10 * s2 + b11 * c2;
      }
      // V <- V J (columns p, q of every row)
      for (int idx = t; idx < n * npair; idx += nt) {
        const int i = idx / npair, k = idx % npair;
        const int p = sp[k], q = sq[k];
        if (q >= n) continue;
        const double c = sc[k], sn = ss[k];
        const double vp = Vb[(size_t)i * n + p], vq = Vb[(size_t)i * n + q];
        Vb[(size_t)i * n + p] = c * vp - sn * vq;
        Vb[(size_t)i * n + q] = sn * vp + c * vq;
      }
      __syncthreads();
    }
    // off-diagonal and diagonal sums of squares
    double off = 0.0, dg = 0.0;
    for (size_t e = t; e < nn; e += nt) {
      const double v = sA[e];
      if (e / n == e % n) dg += v * v; else off += v * v;
    }
    red[t] = off;
    red[1024 + t] = dg;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
      if (t < h && t + h < nt) {
        red[t] += red[t + h];
        red[1024 + t] += red[1024 + t + h];
      }
      __syncthreads();
    }
    if (t == 0) {
      const double o = red[0], d = red[1024];
      int stop = (!(o > 1e-28 * d) || o == 0.0) ? 1 : 0;
      if (prev >= 0.0 && sweep >= 3 && o > 0.5 * prev) stop = 1;
      s_stop = stop;
      red[0] = o;  // kept for prev
    }
    __syncthreads();
    prev = red[0];
    const int stop = s_stop;
    __syncthreads();
    if (stop) break;
  }
  // eigenvalues ascending (ties by index) and the matching columns of V
  double *wb = w + (size_t)blockIdx.x * n;
  double *Vo = Vout + (size_t)blockIdx.x * nn;
  for (int i = t; i < n; i += nt) {
    const double di = sA[(size_t)i * n + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = sA[(size_t)j * n + j];
      rank += (dj < di || (dj == di && j < i)) ? 1 : 0;
    }
    wb[rank] = di;
    for (int row = 0; row < n; ++row) Vo[(size_t)row * n + rank] = Vb[(size_t)row * n + i];
  }
}

bool sym_eig_batched(hipStream_t st, int n, int B, double *A, double *V, double *w,
                     double *Vout) {
  if (n < 1 || n > kLdsEigMax || B < 1) return false;
  const size_t shm = sizeof(double) * ((size_t)n * n + 2 * 1024);
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_jacobi_lds),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  k_jacobi_lds<<<B, 1024, shm, st>>>(n, A, V, w, Vout, 40);
  check_launch("k_jacobi_lds");
  return true;
}

// off-diagonal and diagonal sums of squares -> out[0], out[1] (one block)
__global__ __launch_bounds__(1024) void k_offnorm(int n, const double *A, double *out) {
  __shared__ double red[2][1024];
  const int t = threadIdx.x;
  double off = 0.0, dg = 0.0;
  for (long long e = t; e < (long long)n * n; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const double v = A[e];
    if (i == j) dg += v * v; else off += v * v;
  }
  red[0][t] = off;
  red[1][t] = dg;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) {
      red[0][t] += red[0][t + w];
      red[1][t] += red[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

__global__ void k_eye(int n, double *V) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  V[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
}

// Sort eigenvalues ascending (ties by index) and permute V's columns.
__global__ void k_eig_sort(int n, const double *A, const double *Vin, double *w, double *Vout) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double x = A[(size_t)t * n + t];
  int rk = 0;
  for (int j = 0; j < n; ++j) {
    const double y = A[(size_t)j * n + j];
    if (y < x || (y == x && j < t)) ++rk;
  }
  w[rk] = x;
  for (int i = 0; i < n; ++i) Vout[(size_t)i * n + rk] = Vin[(size_t)i * n + t];
}

// W = blockdiag(V0, I): V0 is n0 x n0 (ld n0), W is n x n.
__global__ void k_embed_block(int n, int n0, const double *V0, double *W) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  W[e] = (i < n0 && j < n0) ? V0[(size_t)i * n0 + j] : (i == j ? 1.0 : 0.0);
}

void launch_embed_block(hipStream_t st, int n, int n0, const double *V0, double *W) {
  const long long nn = (long long)n * n;
  if (nn <= 0) return;
  k_embed_block<<<(unsigned)((nn + 255) / 256), 256, 0, st>>>(n, n0, V0, W);
  check_launch("k_embed_block");
}

void sym_eig(hipStream_t st, int n, double *A, double *w, double *V, DevBuf &work,
             const double *V0) {
  if (n <= 0) return;
  if (n > 4096) throw Error(POLFED_EINVAL, "sym_eig: n must be <= 4096");
  const size_t nn = (size_t)n * n;
  double *base = static_cast<double *>(work.ensure(sizeof(double) * (2 * nn + 4)));
  double *Vw = base;
  double *A2 = base + nn;
  double *off = base + 2 * nn;
  double *buf[2] = {A, A2};
  if (V0) {
    // warm start: A is already V0^T A_orig V0, rotations accumulate onto V0
    PF_HIP(hipMemcpyAsync(Vw, V0, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
  } else {
    k_eye<<<(unsigned)((nn + 255) / 256), 256, 0, st>>>(n, Vw);
    check_launch("k_eye");
  }
  // up to 128 x 128 the matrix fits one workgroup's LDS: the same sweeps
  // and stopping rule in a single launch, without a host round trip per
  // sweep
  if (n <= kLdsEigMax && sym_eig_batched(st, n, 1, A, Vw, w, V)) return;
  const int m = n + (n & 1);
  const int npair = m / 2;
  const int tp = (npair + kJT - 1) / kJT;
  const int tiles_a = tp * tp;
  const int tiles_v = ((n + kJT - 1) / kJT) * tp;
  int cur = 0;
  double host[2] = {0.0, 0.0};
  double prev = -1.0;
  for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
    for (int r = 0; r < m - 1; ++r) {
      k_jacobi_round<<<tiles_a + tiles_v, 256, 0, st>>>(n, r, buf[cur], buf[cur ^ 1], Vw, tiles_a);
      cur ^= 1;
    }
    check_launch("k_jacobi_round");
    k_offnorm<<<1, 1024, 0, st>>>(n, buf[cur], off);
    check_launch("k_offnorm");
    PF_HIP(hipMemcpyAsync(host, off, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    PF_HIP(hipStreamSynchronize(st));
    // stop at a relative off-diagonal Frobenius norm of 1e-14, or when the
    // rounding floor is reached (no further decrease)
    if (!(host[0] > 1e-28 * host[1]) || host[0] == 0.0) break;
    if (prev >= 0.0 && sweep >= 3 && host[0] > 0.5 * prev) break;
    prev = host[0];
  }
  k_eig_sort<<<(n + 255) / 256, 256, 0, st>>>(n, buf[cur], Vw, w, V);
  check_launch("k_eig_sort");
}

// ------------------------------------------------------------- philox --
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
// (c0,c1,c2,c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)), with the key bumped by the Weyl constants between rounds.

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += W0;
    k1 += W1;
  }
  return c;
}

__global__ void k_philox_fill(long long n, int S, double *X, long long ld, uint32_t k0,
                              uint32_t k1, uint32_t sid) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * S) return;
  const long long r = e / S;
  const int c = (int)(e % S);
  U4 o = philox4x32_10(U4{(uint32_t)r, (uint32_t)(r >> 32), (uint32_t)c, sid}, k0, k1);
  const unsigned long long bits = ((unsigned long long)o.x << 21) ^ ((unsigned long long)o.y >> 11);
  const double u = (double)(bits & ((1ull << 53) - 1)) * (1.0 / 9007199254740992.0);
  X[r * ld + c] = 2.0 * u - 1.0;
}

void launch_philox_fill(hipStream_t st, long long n, int S, double *X, long long ld,
                        unsigned long long seed, unsigned stream_id) {
  long long tot = n * S;
  if (tot <= 0) return;
  k_philox_fill<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(
      n, S, X, ld, (uint32_t)seed, (uint32_t)(seed >> 32), stream_id);
  check_launch("k_philox_fill");
}

// ----------------------------------------------------- column reductions --
//
// Grid: nblk row-chunks x ceil(q/64) column groups; lane = column, the 4
// waves stride over the rows of the chunk; partials[blk][col] then a
// fixed-order sum.

template <int MODE>  // 0: sum x^2; 1: sum (hv - e v)^2
__global__ __launch_bounds__(256) void k_colsq(long long n, int q, const double *X,
                                               long long ldx, const double *V, long long ldv,
                                               const double *E, double *part,
                                               long long rows_per_blk) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cg = blockIdx.y;
  const int col = cg * 64 + lane;
  const long long r0 = (long long)blockIdx.x * rows_per_blk;
  long long r1 = r0 + rows_per_blk;
  if (r1 > n) r1 = n;
  double s = 0.0;
  if (col < q) {
    const double e = (MODE == 1) ? E[col] : 0.0;
    for (long long r = r0 + wave; r < r1; r += 4) {
      double x = X[r * ldx + col];
      if (MODE == 1) x -= e * V[r * ldv + col];
      s += x * x;
    }
  }
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && col < q)
    part[(size_t)blockIdx.x * q + col] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__global__ void k_colsum_final(int q, int nblk, const double *part, double *out, int do_sqrt) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= q) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * q + j];
  out[j] = do_sqrt ? sqrt(s) : s;
}

static void colsq(hipStream_t st, int mode, long long n, int q, const double *X, long long ldx,
                  const double *V, long long ldv, const double *E, double *out,
                  DevBuf &partials, int num_cu) {
  if (q <= 0) return;
  long long want = std::max<long long>(1, 2LL * num_cu / ((q + 63) / 64));
  long long rows = std::max<long long>(64, (n + want - 1) / want);
  long long nblk = std::max<long long>(1, (n + rows - 1) / rows);
  double *part = static_cast<double *>(partials.ensure(sizeof(double) * nblk * q));
  dim3 grid((unsigned)nblk, (unsigned)((q + 63) / 64));
  if (mode == 0)
    k_colsq<0><<<grid, 256, 0, st>>>(n, q, X, ldx, V, ldv, E, part, rows);
  else
    k_colsq<1><<<grid, 256, 0, st>>>(n, q, X, ldx, V, ldv, E, part, rows);
  check_launch("k_colsq");
  k_colsum_final<<<(q + 255) / 256, 256, 0, st>>>(q, (int)nblk, part, out, 1);
  check_launch("k_colsum_final");
}

void launch_colnorms(hipStream_t st, long long n, int q, const double *X, long long ldx,
                     double *out, DevBuf &partials, int num_cu) {
  colsq(st, 0, n, q, X, ldx, nullptr, 0, nullptr, out, partials, num_cu);
}

void launch_resid_norms(hipStream_t st, long long n, int q, const double *HV, long long ldhv,
                        const double *V, long long ldv, const double *E, double *out,
                        DevBuf &partials, int num_cu) {
  colsq(st, 1, n, q, HV, ldhv, V, ldv, E, out, partials, num_cu);
}

// argmax |x| per column, lowest row on ties -> f[j] = sign of that entry
__global__ __launch_bounds__(256) void k_colargmax(long long n, int q, const double *X,
                                                   long long ldx, double *pv, long long *pi,
                                                   long long rows_per_blk) {
  __shared__ double bv[4][64];
  __shared__ long long bi[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = blockIdx.y * 64 + lane;
  const long long r0 = (long long)blockIdx.x * rows_per_blk;
  long long r1 = r0 + rows_per_blk;
  if (r1 > n) r1 = n;
  double best = -1.0;
  long long bidx = -1;
  if (col < q) {
    for (long long r = r0 + wave; r < r1; r += 4) {
      const double a = fabs(X[r * ldx + col]);
      if (a > best) { best = a; bidx = r; }  // rows visited ascending: keeps lowest on ties
    }
  }
  bv[wave][lane] = best;
  bi[wave][lane] = bidx;
  __syncthreads();
  if (wave == 0 && col < q) {
    for (int w = 1; w < 4; ++w) {
      const double v = bv[w][lane];
      const long long i = bi[w][lane];
      if (v > best || (v == best && i >= 0 && (bidx < 0 || i < bidx))) { best = v; bidx = i; }
    }
    pv[(size_t)blockIdx.x * q + col] = best;
    pi[(size_t)blockIdx.x * q + col] = bidx;
  }
}

__global__ void k_sign_final(int q, int nblk, const double *pv, const long long *pi,
                             const double *X, long long ldx, double *f) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= q) return;
  double best = -1.0;
  long long bidx = -1;
  for (int b = 0; b < nblk; ++b) {
    const double v = pv[(size_t)b * q + j];
    const long long i = pi[(size_t)b * q + j];
    if (v > best || (v == best && i >= 0 && (bidx < 0 || i < bidx))) { best = v; bidx = i; }
  }
  f[j] = (bidx >= 0 && X[bidx * ldx + j] < 0.0) ? -1.0 : 1.0;
}

void launch_sign_factors(hipStream_t st, long long n, int q, const double *X, long long ldx,
                         double *f, DevBuf &partials, int num_cu) {
  if (q <= 0) return;
  long long want = std::max<long long>(1, 2LL * num_cu / ((q + 63) / 64));
  long long rows = std::max<long long>(64, (n + want - 1) / want);
  long long nblk = std::max<long long>(1, (n + rows - 1) / rows);
  char *base = static_cast<char *>(partials.ensure((sizeof(double) + sizeof(long long)) * nblk * q));
  double *pv = reinterpret_cast<double *>(base);
  long long *pi = reinterpret_cast<long long *>(base + sizeof(double) * nblk * q);
  dim3 grid((unsigned)nblk, (unsigned)((q + 63) / 64));
  k_colargmax<<<grid, 256, 0, st>>>(n, q, X, ldx, pv, pi, rows);
  check_launch("k_colargmax");
  k_sign_final<<<(q + 255) / 256, 256, 0, st>>>(q, (int)nblk, pv, pi, X, ldx, f);
  check_launch("k_sign_final");
}

__global__ void k_scale_cols(long long n, int q, double *X, long long ldx, const double *f) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * q) return;
  long long r = e / q;
  int j = (int)(e % q);
  X[r * ldx + j] *= f[j];
}

void launch_scale_cols(hipStream_t st, long long n, int q, double *X, long long ldx,
                       const double *f) {
  long long tot = n * q;
  if (tot <= 0) return;
  k_scale_cols<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(n, q, X, ldx, f);
  check_launch("k_scale_cols");
}

// out[j * n + r] = X[r * ldx + j] through a 32 x 32 LDS tile
__global__ void k_to_colmajor(long long n, int q, const double *X, long long ldx, double *out) {
  __shared__ double tile[32][33];
  const long long r0 = (long long)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const long long r = r0 + k;
    const int c = c0 + tx;
    tile[k][tx] = (r < n && c < q) ? X[r * ldx + c] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k;
    const long long r = r0 + tx;
    if (r < n && c < q) out[(size_t)c * n + r] = tile[tx][k];
  }
}

void launch_to_colmajor(hipStream_t st, long long n, int q, const double *X, long long ldx,
                        double *out) {
  if (n <= 0 || q <= 0) return;
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((q + 31) / 32));
  k_to_colmajor<<<grid, 256, 0, st>>>(n, q, X, ldx, out);
  check_launch("k_to_colmajor");
}

__global__ void k_gather_cols(long long n, int q, const double *X, long long ldx, const int *idx,
                              double *out, long long ldo) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * q) return;
  long long r = e / q;
  int j = (int)(e % q);
  out[r * ldo + j] = X[r * ldx + idx[j]];
}

void launch_gather_cols(hipStream_t st, long long n, int q, const double *X, long long ldx,
                        const int *idx, double *out, long long ldo) {
  long long tot = n * q;
  if (tot <= 0) return;
  k_gather_cols<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(n, q, X, ldx, idx, out, ldo);
  check_launch("k_gather_cols");
}

__global__ void k_fill(double *x, long long count, double v) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) x[e] = v;
}

void launch_fill(hipStream_t st, double *x, long long count, double v) {
  if (count <= 0) return;
  k_fill<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(x, count, v);
  check_launch("k_fill");
}

// ----------------------------------------------- single-vector Lanczos --
//
// One step of the bounds Lanczos (w = H v_k already computed):
//   alpha_k = v_k . w;  w <- w - alpha_k v_k - beta_k v_{k-1};
//   beta_{k+1} = ||w||;  v_{k+1} = w / beta_{k+1}.
// Scalars stay on the device; every block of a kernel re-reduces the same
// partial array in the same order, so all blocks agree bitwise.

constexpr int kRedThreads = 256;

__device__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double sum_partials(const double *part, int nblk, double *sh) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[b];
  return block_sum(s, sh);
}

__global__ __launch_bounds__(kRedThreads) void k_dot_partials(long long n, const double *x,
                                                              const double *y, double *part) {
  __shared__ double sh[kRedThreads];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_lanczos_update(long long n, double *w,
                                                                const double *v,
                                                                const double *vprev,
                                                                const double *part, int nblk,
                                                                double *alpha,
                                                                const double *beta_prev,
                                                                double *part2) {
  __shared__ double sh[kRedThreads];
  const double a = sum_partials(part, nblk, sh);
  const double b = (vprev != nullptr) ? beta_prev[0] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) alpha[0] = a;
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double x = w[i] - a * v[i];
    if (vprev != nullptr) x -= b * vprev[i];
    w[i] = x;
    s += x * x;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part2[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_lanczos_normalize(long long n, const double *w,
                                                                   double *vnext,
                                                                   const double *part2, int nblk,
                                                                   double *beta) {
  __shared__ double sh[kRedThreads];
  const double b = sqrt(sum_partials(part2, nblk, sh));
  if (blockIdx.x == 0 && threadIdx.x == 0) beta[0] = b;
  const double inv = (b > 1e-300) ? 1.0 / b : 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    vnext[i] = w[i] * inv;
}

void launch_dot_partials(hipStream_t st, long long n, const double *x, const double *y,
                         double *part, int nblk) {
  k_dot_partials<<<nblk, kRedThreads, 0, st>>>(n, x, y, part);
  check_launch("k_dot_partials");
}

void launch_lanczos_update(hipStream_t st, long long n, double *w, const double *v,
                           const double *vprev, const double *part, int nblk, double *alpha,
                           const double *beta_prev, double *part2) {
  k_lanczos_update<<<nblk, kRedThreads, 0, st>>>(n, w, v, vprev, part, nblk, alpha, beta_prev,
                                                 part2);
  check_launch("k_lanczos_update");
}

void launch_lanczos_normalize(hipStream_t st, long long n, const double *w, double *vnext,
                              const double *part2, int nblk, double *beta) {
  k_lanczos_normalize<<<nblk, kRedThreads, 0, st>>>(n, w, vnext, part2, nblk, beta);
  check_launch("k_lanczos_normalize");
}

}  // namespace polfed
