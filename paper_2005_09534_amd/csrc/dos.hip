// Density of states of H~ by the kernel polynomial method: the Chebyshev
// moments mu_n = Tr T_n(H~) / N estimated from random vectors (Silver et al.,
// the iterative estimator the paper names for the DOS of an arbitrary sparse
// matrix, where the order K is chosen; main text, "POLFED algorithm").
//
// Each block of vectors r runs the forward recurrence t_0 = r, t_1 = H~ r,
// t_{k+1} = 2 H~ t_k - t_{k-1} with the fused step kernel, and after each
// step a deterministic two-stage reduction takes <t_k, t_k> and
// <t_k, t_{k-1}> over all rows and columns.  With T_{2k} = 2 T_k^2 - 1 and
// T_{2k+1} = 2 T_{k+1} T_k - T_1, m steps give the moments up to 2m:
//   <r|T_{2k}|r>   = 2 <t_k, t_k> - <r, r>,
//   <r|T_{2k+1}|r> = 2 <t_{k+1}, t_k> - <t_1, t_0>,
// and mu_n is their sum over the vectors divided by sum <r, r>.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace polfed {

constexpr int kDotThreads = 256;

// part[2 blk] = sum x^2, part[2 blk + 1] = sum x y over this workgroup's
// elements of the tot contiguous ones (y may be null: 0).  Each lane
// strides over the elements, then a fixed butterfly per wave and a fixed
// order over the four waves.
__global__ __launch_bounds__(kDotThreads) void k_dual_dot(long long tot, const double *x,
                                                        const double *y, double *part) {
  __shared__ double red[2][kDotThreads / 64];
  const long long stride = (long long)gridDim.x * kDotThreads;
  double a0 = 0.0, a1 = 0.0;
  for (long long i = (long long)blockIdx.x * kDotThreads + threadIdx.x; i < tot; i += stride) {
    const double v = x[i];
    a0 += v * v;
    if (y) a1 += v * y[i];
  }
  for (int o = 32; o >= 1; o >>= 1) {
    a0 += __shfl_xor(a0, o);
    a1 += __shfl_xor(a1, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = a0;
    red[1][wave] = a1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < kDotThreads / 64; ++w) {
      s0 += red[0][w];
      s1 += red[1][w];
    }
    part[2 * blockIdx.x] = s0;
    part[2 * blockIdx.x + 1] = s1;
  }
}

// out[0..1] = sums of the nblk partial pairs (one wave, fixed order).
__global__ __launch_bounds__(64) void k_dual_final(int nblk, const double *part, double *out) {
  double a0 = 0.0, a1 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) {
    a0 += part[2 * b];
    a1 += part[2 * b + 1];
  }
  for (int o = 32; o >= 1; o >>= 1) {
    a0 += __shfl_xor(a0, o);
    a1 += __shfl_xor(a1, o);
  }
  if (threadIdx.x == 0) {
    out[0] = a0;
    out[1] = a1;
  }
}

// Columns c < cnt of X (n x ld): x -> -1 where x < 0, else +1.
__global__ void k_rademacher(long long n, int cnt, double *X, long long ld) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * cnt) return;
  const long long r = e / cnt;
  const int c = (int)(e % cnt);
  double &x = X[r * ld + c];
  x = (x < 0.0) ? -1.0 : 1.0;
}

static void dual_dot(hipStream_t st, long long tot, const double *x, const double *y,
                     double *part, int nblk, double *out) {
  k_dual_dot<<<nblk, kDotThreads, 0, st>>>(tot, x, y, part);
  check_launch("k_dual_dot");
  k_dual_final<<<1, 64, 0, st>>>(nblk, part, out);
  check_launch("k_dual_final");
}

void dos_moments(polfed_ctx *ctx, const Chain &c, double a, double b, int nmom, int nvec,
                 const double *R, unsigned long long seed, std::vector<double> &mu) {
  PF_REQUIRE(nmom >= 1 && nmom <= (1 << 20), "dos moments: nmom must be in [1, 2^20]");
  PF_REQUIRE(nvec >= 1, "dos moments: nvec must be >= 1");
  hipStream_t st = ctx->stream;
  const long long n = c.basis->n;
  const int m = nmom / 2;  // steps: t_0 .. t_m
  int S = 1;
  while (S < nvec && S < 64) S <<= 1;
  const int nchunk = (nvec + S - 1) / S;
  const long long tot = n * S;
  const int nblk = (int)std::max<long long>(
      1, std::min<long long>(4LL * ctx->num_cu, (tot + kDotThreads - 1) / kDotThreads));

  double *dt = static_cast<double *>(ctx->buf("dos_dt").ensure(sizeof(double) * n));
  double *ring = static_cast<double *>(ctx->buf("dos_t").ensure(sizeof(double) * 3 * (size_t)tot));
  double *part = static_cast<double *>(ctx->buf("dos_part").ensure(sizeof(double) * 2 * nblk));
  const size_t ndots = (size_t)nchunk * (m + 1) * 2;
  double *dots = static_cast<double *>(ctx->buf("dos_dots").ensure(sizeof(double) * ndots));
  launch_scaled_diag<double>(st, n, c.diag.as<double>(), a, b, dt);
  double *t[3] = {ring, ring + tot, ring + 2 * tot};
  const StepShape shape = [&] {
    auto it = ctx->shapes.find(std::make_tuple(c.L, S, 8));
    return it != ctx->shapes.end() ? it->second : default_shape(c.L, S, false);
  }();
  if (shape.rank_incr == 2 && !c.pattern) c.pattern = &ctx->pattern(c.L, c.J2 != 0.0);

  for (int ch = 0; ch < nchunk; ++ch) {
    const int c0 = ch * S;
    const int cnt = std::min(S, nvec - c0);
    if (cnt < S) launch_fill(st, t[0], tot, 0.0);
    if (R) {
      PF_HIP(hipMemcpy2DAsync(t[0], sizeof(double) * S, R + c0, sizeof(double) * nvec,
                              sizeof(double) * cnt, (size_t)n, hipMemcpyDeviceToDevice, st));
    } else {
      launch_philox_fill(st, n, cnt, t[0], S, seed, 0x444f53u + (unsigned)ch);
      const long long e = n * cnt;
      k_rademacher<<<(unsigned)((e + 255) / 256), 256, 0, st>>>(n, cnt, t[0], S);
      check_launch("k_rademacher");
    }
    double *d = dots + (size_t)ch * (m + 1) * 2;
    dual_dot(st, tot, t[0], nullptr, part, nblk, d);
    for (int k = 1; k <= m; ++k) {
      StepArgs<double> sa;
      std::memset(&sa, 0, sizeof(sa));
      const Basis &bs = *c.basis;
      sa.states = bs.states.as<uint32_t>();
      sa.dt = dt;
      sa.tabA = bs.tabA.as<int32_t>();
      sa.tabB = bs.tabB.as<uint16_t>();
      sa.n = n;
      sa.L = c.L;
      sa.half = bs.half;
      sa.lomask = (1u << bs.half) - 1u;
      sa.fullmask = (c.L >= 32) ? 0xffffffffu : ((1u << c.L) - 1u);
      sa.has_j2 = (c.J2 != 0.0) ? 1 : 0;
      sa.binom = bs.binom.as<int32_t>();
      sa.nslices = 1;
      if (c.pattern) {
        sa.csr_ptr = c.pattern->ptr.as<long long>();
        sa.csr_col = c.pattern->col.as<int32_t>();
      }
      sa.V = t[(k - 1) % 3];
      sa.ldv = S;
      sa.out = t[k % 3];
      sa.ldo = S;
      if (k == 1) {  // t_1 = H~ t_0
        sa.dscale = 1.0;
        sa.w1 = 0.5 * a * c.J1;
        sa.w2 = 0.5 * a * c.J2;
      } else {  // t_k = 2 H~ t_{k-1} - t_{k-2}
        sa.W = t[(k - 2) % 3];
        sa.ldw = S;
        sa.dscale = 2.0;
        sa.w1 = a * c.J1;
        sa.w2 = a * c.J2;
        sa.gamma = -1.0;
      }
      launch_step<double>(st, S, sa, shape, ctx->num_cu);
      dual_dot(st, tot, t[k % 3], t[(k - 1) % 3], part, nblk, d + 2 * k);
    }
  }
  std::vector<double> h(ndots);
  PF_HIP(hipMemcpyAsync(h.data(), dots, sizeof(double) * ndots, hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
  ctx->buf("dos_t").release();  // 3 n S values: not kept for the solve that follows
  // sums over the chunks, in chunk order
  std::vector<double> d0(m + 1, 0.0), d1(m + 1, 0.0);
  for (int ch = 0; ch < nchunk; ++ch)
    for (int k = 0; k <= m; ++k) {
      d0[k] += h[((size_t)ch * (m + 1) + k) * 2];
      d1[k] += h[((size_t)ch * (m + 1) + k) * 2 + 1];
    }
  PF_REQUIRE(d0[0] > 0.0, "dos moments: the random vectors are all zero");
  mu.assign(nmom, 0.0);
  for (int j = 0; j < nmom; ++j) {
    const int k = j / 2;
    const double tr = (j % 2 == 0) ? 2.0 * d0[k] - d0[0] : 2.0 * d1[k + 1] - d1[1];
    mu[j] = (j == 0) ? 1.0 : tr / d0[0];
  }
}

}  // namespace polfed
