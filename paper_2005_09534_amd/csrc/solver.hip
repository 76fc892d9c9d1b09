// POLFED solve on one GPU: host control loop around the device kernels.
//
// Steps (main text, "POLFED algorithm"; Supplement, "Convergence of POLFED"):
//  1. Lanczos on H for the extremes E0, E1, widened by their residual bound
//     and a margin eta (E1 - E0): a Chebyshev series of order K grows like
//     cosh(K sqrt(2 delta)) at a distance delta outside [-1, 1].
//  2. H~ = a H + b; target sigma~ = a sigma_H + b.
//  3. K from the density of states for a window of N_win = ceil(f N_ev)
//     eigenvalues (f = 1.5 by default: the Gaussian estimate can exceed the
//     local density, and K ~ 1/N_win keeps the filter work unchanged).
//  4. Q_1: Philox start block, orthonormalised.
//  5. Block Lanczos on P(H~), eqs. (Lan1)-(Lan2):
//        U = P Q_j - Q_{j-1} B_j^T ; A_j = sym(Q_j^T U) ; U -= Q_j A_j ;
//        U -= Qm (Qm^T U) twice (full reorthogonalisation, not fed into T) ;
//        Q_{j+1} B_{j+1} = U by CholeskyQR2 (diag(B) > 0).
//     T_m is block tridiagonal with A_j, B_{j+1} below and B_{j+1}^T above.
//  6. Eigenpairs (theta_i, t_i) of T_m; converged when theta_i >= p and
//     ||B_{j+1} t~_i|| <= tau; stop once N_ev have converged.
//  7. Ritz vectors Qm t_i for theta_i >= p; Rayleigh-Ritz of H~ on their span
//     (eps_i = u_i^T H~ u_i when the theta_i are distinct; P is even around
//     sigma locally, so pairs sigma +- d share theta and need the joint
//     projection); the N_ev values nearest sigma; residuals ||Hv - Ev||.
// In FP32 mode the filter runs in FP32 (X and the recurrence vectors), and
// everything else in FP64; a refinement in FP64 follows (see refine()).
#include <algorithm>
#include <chrono>
#include <iterator>
#include <map>
#include <set>
#include <memory>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cstdint>
#include <numeric>

#include "internal.h"

namespace polfed {

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ operators --

// Step arguments for a chain with the given diagonal (in T) and weights.
template <class T>
static StepArgs<T> base_args(const Chain &c, const T *dt) {
  StepArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  const Basis &b = *c.basis;
  a.states = b.states.as<uint32_t>();
  a.dt = dt;
  a.tabA = b.tabA.as<int32_t>();
  a.tabB = b.tabB.as<uint16_t>();
  a.n = b.n;
  a.L = c.L;
  a.half = b.half;
  a.lomask = (1u << b.half) - 1u;
  a.fullmask = (c.L >= 32) ? 0xffffffffu : ((1u << c.L) - 1u);
  a.has_j2 = (c.J2 != 0.0) ? 1 : 0;
  a.binom = b.binom.as<int32_t>();
  a.nslices = 1;
  if (c.pattern) {
    a.csr_ptr = c.pattern->ptr.as<long long>();
    a.csr_col = c.pattern->col.as<int32_t>();
  }
  return a;
}

// The stored neighbour pattern of the chain, built on first use, where the
// shape reads neighbours from it (rank mode 2).  Before any graph capture.
static void attach_pattern(polfed_ctx *ctx, const Chain &c, const StepShape &shape) {
  if (shape.rank_incr == 2 && !c.pattern) c.pattern = &ctx->pattern(c.L, c.J2 != 0.0);
}

// Algorithmic bytes of one step launch: each streamed block once (out, the
// gathered V, W, X, and the accumulator's source and destination), plus the
// state word and diagonal of every row when H~ is applied -- or, when the
// neighbours come from the stored pattern (rank mode 2), the diagonal, the
// row pointers and every column index instead of the state word.
template <class T>
static double step_bytes(const StepArgs<T> &st, int S, int rank_mode = 0,
                         const Pattern *pat = nullptr) {
  const int streams = (st.skip_out ? 0 : 1) + (st.V ? 1 : 0) + (st.W ? 1 : 0) +
                      (st.X ? 1 : 0) + (st.acc ? 2 : 0);
  double b = (double)st.n * (S * (double)sizeof(T) * streams);
  if (st.V) {
    if (rank_mode == 2 && pat)
      b += (double)st.n * (8.0 + sizeof(T)) + 8.0 + 4.0 * (double)pat->nnz;
    else
      b += (double)st.n * (4.0 + sizeof(T));
  }
  return b;
}

static StepShape shape_for(const polfed_ctx *ctx, int L, int S, bool fp32) {
  auto it = ctx->shapes.find(std::make_tuple(L, S, fp32 ? 4 : 8));
  if (it != ctx->shapes.end()) return it->second;
  return default_shape(L, S, fp32);
}

// out = scale * (dt .* V + sum w_l V[nbr]) for a block of `width` columns,
// split into power-of-two chunks of at most 64 columns.
template <class T>
static void apply_op(polfed_ctx *ctx, const Chain &c, const T *dt, double wscale1,
                     double wscale2, const T *V, long long ldv, T *out, long long ldo, int width,
                     bool fp32) {
  int off = 0;
  while (off < width) {
    int S = 64;
    while (S > width - off) S >>= 1;
    attach_pattern(ctx, c, shape_for(ctx, c.L, S, fp32));
    StepArgs<T> a = base_args<T>(c, dt);
    a.V = V + off;
    a.ldv = ldv;
    a.out = out + off;
    a.ldo = ldo;
    a.dscale = T(1);
    a.w1 = (T)wscale1;
    a.w2 = (T)wscale2;
    launch_step<T>(ctx->stream, S, a, shape_for(ctx, c.L, S, fp32), ctx->num_cu);
    off += S;
  }
}

// Y = P^K_sigma(H~) X = (sum_k c_k T_k(H~) X) / D by the forward three-term
// recurrence: t_0 = X, t_1 = H~ X, t_{k+1} = 2 H~ t_k - t_{k-1}, each t_k
// added to Y with weight c_k / D as it is made (steps after the last
// non-zero c_k are not run).  Returns the algorithmic bytes of the launches;
// with launch = false only counts them.
template <class T>
static double queue_filter_forward(hipStream_t stream, int num_cu, const StepShape &shape,
                                   const Chain &c, const T *dt, double a, int S, const T *X,
                                   long long ldx, T *Y, long long ldy, long long K,
                                   const std::vector<double> &coef, double D, T *buf3,
                                   bool launch) {
  const long long n = c.basis->n;
  T *bufs[3] = {buf3, buf3 + (size_t)n * S, buf3 + (size_t)2 * n * S};
  const double Dinv = 1.0 / D;
  double moved = 0.0;
  long long klast = 0;
  for (long long k = K; k >= 1; --k)
    if (coef[k] != 0.0) {
      klast = k;
      break;
    }
  if (klast == 0) {  // Y = c_0 X / D
    StepArgs<T> st = base_args<T>(c, dt);
    st.out = Y;
    st.ldo = ldy;
    st.X = X;
    st.ldx = ldx;
    st.alpha = (T)(coef[0] * Dinv);
    if (launch) launch_step<T>(stream, S, st, shape, num_cu);
    return step_bytes(st, S, shape.rank_incr, c.pattern);
  }
  for (long long k = 1; k <= klast; ++k) {
    StepArgs<T> st = base_args<T>(c, dt);
    st.out = bufs[(k - 1) % 3];
    st.ldo = S;
    st.skip_out = (k == klast) ? 1 : 0;
    if (k == 1) {  // t_1 = H~ X
      st.V = X;
      st.ldv = ldx;
      st.dscale = T(1);
      st.w1 = (T)(0.5 * a * c.J1);
      st.w2 = (T)(0.5 * a * c.J2);
      st.acc = Y;
      st.ldacc = ldy;
      st.src = X;
      st.ldsrc = ldx;
      st.cin = (T)(coef[0] * Dinv);
      st.cacc = (T)(coef[1] * Dinv);
    } else {  // t_k = 2 H~ t_{k-1} - t_{k-2}
      st.V = bufs[(k - 2) % 3];
      st.ldv = S;
      if (k == 2) {
        st.W = X;
        st.ldw = ldx;
      } else {
        st.W = bufs[(k - 3) % 3];
        st.ldw = S;
      }
      st.dscale = T(2);
      st.w1 = (T)(a * c.J1);
      st.w2 = (T)(a * c.J2);
      st.gamma = T(-1);
      if (coef[k] != 0.0) {
        st.acc = Y;
        st.ldacc = ldy;
        st.src = Y;
        st.ldsrc = ldy;
        st.cin = T(1);
        st.cacc = (T)(coef[k] * Dinv);
      }
    }
    if (launch) launch_step<T>(stream, S, st, shape, num_cu);
    moved += step_bytes(st, S, shape.rank_incr, c.pattern);
  }
  return moved;
}

// Y = P^K_sigma(H~) X by Clenshaw:  b_k = c_k X + 2 H~ b_{k+1} - b_{k+2},
// k = K..1, then Y = (c_0 X + H~ b_1 - b_2) / D (or by the forward form,
// per `form`).  dt = a d + b in T.  Returns the algorithmic bytes of the
// launches it queues; with launch = false only counts them.
// Column slices of the Clenshaw filter for this shape and width (1 when
// the shape asks for none or the width does not split).
static int filter_slices(const StepShape &shape, int S) {
  const int ns = shape.xcd_slices;
  return (ns > 1 && ns <= S && S % ns == 0) ? ns : 1;
}

template <class T>
static double queue_filter(hipStream_t stream, int num_cu, const StepShape &shape, const Chain &c,
                           const T *dt, double a, int S, const T *X, long long ldx, T *Y,
                           long long ldy, long long K, const std::vector<double> &coef, double D,
                           T *buf3, int form, T *xpack, bool launch = true) {
  if (form == POLFED_FORM_FORWARD)
    return queue_filter_forward<T>(stream, num_cu, shape, c, dt, a, S, X, ldx, Y, ldy, K, coef,
                                   D, buf3, launch);
  const long long n = c.basis->n;
  T *bufs[3] = {buf3, buf3 + (size_t)n * S, buf3 + (size_t)2 * n * S};
  // With XCD column slices the recurrence blocks and a copy of X are held
  // slice-major (each slice an n x S/ns block), so that one XCD's rows of
  // its slice are contiguous; only Y, written once, stays row-major.
  const int ns = filter_slices(shape, S);
  const long long sw = S / ns;
  const long long bss = (ns > 1) ? n * sw : 0;  // slice stride of a packed block
  const long long bld = (ns > 1) ? sw : S;      // its leading dimension
  const T *Xin = X;
  long long ldxin = ldx, xss = 0;
  if (ns > 1) {
    if (launch) launch_pack_slices<T>(stream, n, S, ns, X, ldx, xpack);
    Xin = xpack;
    ldxin = sw;
    xss = n * sw;
  }
  double moved = 0.0;
  for (long long j = 0; j < K; ++j) {
    const long long k = K - j;
    StepArgs<T> st = base_args<T>(c, dt);
    st.nslices = ns;
    st.out = bufs[j % 3];
    st.ldo = bld;
    st.oss = bss;
    if (j >= 1) {
      st.V = bufs[(j - 1) % 3];
      st.ldv = bld;
      st.vss = bss;
    }
    if (j >= 2) {
      st.W = bufs[(j - 2) % 3];
      st.ldw = bld;
      st.wss = bss;
    }
    if (coef[k] != 0.0) {
      st.X = Xin;
      st.ldx = ldxin;
      st.xss = xss;
    }
    st.alpha = (T)coef[k];
    st.dscale = T(2);
    st.w1 = (T)(a * c.J1);
    st.w2 = (T)(a * c.J2);
    st.gamma = T(-1);
    if (launch) launch_step<T>(stream, S, st, shape, num_cu);
    moved += step_bytes(st, S, shape.rank_incr, c.pattern);
  }
  StepArgs<T> st = base_args<T>(c, dt);
  st.nslices = ns;
  st.out = Y;
  st.ldo = ldy;
  st.oss = (ns > 1) ? sw : 0;
  st.X = Xin;
  st.ldx = ldxin;
  st.xss = xss;
  // (products with 1/D, as in the batched kernel)
  const double Dinv = 1.0 / D;
  st.alpha = (T)(coef[0] * Dinv);
  if (K >= 1) {
    st.V = bufs[(K - 1) % 3];
    st.ldv = bld;
    st.vss = bss;
  }
  if (K >= 2) {
    st.W = bufs[(K - 2) % 3];
    st.ldw = bld;
    st.wss = bss;
  }
  st.dscale = (T)Dinv;
  st.w1 = (T)(0.5 * (a * c.J1) * Dinv);
  st.w2 = (T)(0.5 * (a * c.J2) * Dinv);
  st.gamma = (T)(-Dinv);
  if (launch) launch_step<T>(stream, S, st, shape, num_cu);
  moved += step_bytes(st, S, shape.rank_incr, c.pattern);
  return moved;
}

// Graphs pay off where a step is short (launch-bound): blocks up to 64 MB
// and K up to 2^17 launches per graph.
template <class T>
static bool graph_worthwhile(long long n, int S, long long K) {
  return K >= 16 && K <= (1LL << 17) && (double)n * S * sizeof(T) <= 64.0 * (1 << 20);
}

template <class T>
static void run_filter(polfed_ctx *ctx, const Chain &c, const T *dt, double a, int S,
                       const T *X, long long ldx, T *Y, long long ldy, long long K,
                       const std::vector<double> &coef, double D, T *buf3, bool fp32,
                       double *bytes, bool reused = true) {
  const long long n = c.basis->n;
  StepShape shape = shape_for(ctx, c.L, S, fp32);
  attach_pattern(ctx, c, shape);
  if (!ctx->ev_start) {
    PF_HIP(hipEventCreate(&ctx->ev_start));
    PF_HIP(hipEventCreate(&ctx->ev_stop));
  }
  double moved = 0.0;
  const int form = ctx->filter_form;
  // the slice-major copy of X (allocated before any capture)
  T *xpack = nullptr;
  if (form == POLFED_FORM_CLENSHAW && filter_slices(shape, S) > 1)
    xpack = static_cast<T *>(ctx->buf("xpack").ensure(sizeof(T) * (size_t)n * S));
  // a graph pays for its capture only when it is replayed: filters run once
  // (the refinement passes, each with its own order) launch directly
  if (reused && ctx->use_graphs && graph_worthwhile<T>(n, S, K)) {
    // key: every value baked into the launches
    std::vector<unsigned long long> key = {
        (unsigned long long)sizeof(T), (unsigned long long)S, (unsigned long long)n,
        (unsigned long long)c.L, (unsigned long long)(uintptr_t)X, (unsigned long long)ldx,
        (unsigned long long)(uintptr_t)Y, (unsigned long long)ldy, (unsigned long long)K,
        (unsigned long long)(uintptr_t)dt, (unsigned long long)(uintptr_t)buf3,
        (unsigned long long)(uintptr_t)c.basis->states.p,
        (unsigned long long)shape.threads, (unsigned long long)shape.lpl,
        (unsigned long long)shape.wg_per_cu, (unsigned long long)shape.lds_tables,
        (unsigned long long)shape.early_loads, (unsigned long long)shape.rank_incr,
        (unsigned long long)shape.xcd_slices, (unsigned long long)(uintptr_t)xpack,
        (unsigned long long)form};
    auto bits = [](double v) {
      unsigned long long u;
      std::memcpy(&u, &v, sizeof(u));
      return u;
    };
    key.push_back(bits(a));
    key.push_back(bits(c.J1));
    key.push_back(bits(c.J2));
    key.push_back(bits(D));
    unsigned long long hsh = 1469598103934665603ull;  // FNV-1a over the coefficients
    for (double v : coef) {
      hsh ^= bits(v);
      hsh *= 1099511628211ull;
    }
    key.push_back(hsh);
    if (!(ctx->filter_graph && ctx->filter_graph_key == key)) {
      if (ctx->filter_graph) {
        PF_HIP(hipGraphExecDestroy(ctx->filter_graph));
        ctx->filter_graph = nullptr;
      }
      // capture on the context's own stream (the null stream cannot be
      // captured); the graph is launched on the working stream
      hipGraph_t g = nullptr;
      PF_HIP(hipStreamBeginCapture(ctx->own_stream, hipStreamCaptureModeThreadLocal));
      try {
        queue_filter<T>(ctx->own_stream, ctx->num_cu, shape, c, dt, a, S, X, ldx, Y, ldy, K, coef,
                        D, buf3, form, xpack);
      } catch (...) {
        hipGraph_t dummy = nullptr;
        (void)hipStreamEndCapture(ctx->own_stream, &dummy);
        if (dummy) (void)hipGraphDestroy(dummy);
        throw;
      }
      PF_HIP(hipStreamEndCapture(ctx->own_stream, &g));
      hipError_t e = hipGraphInstantiate(&ctx->filter_graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      PF_HIP(e);
      ctx->filter_graph_key = key;
    }
    PF_HIP(hipEventRecord(ctx->ev_start, ctx->stream));
    PF_HIP(hipGraphLaunch(ctx->filter_graph, ctx->stream));
    // same byte model as the direct path
    moved = queue_filter<T>(ctx->own_stream, ctx->num_cu, shape, c, dt, a, S, X, ldx, Y, ldy, K,
                            coef, D, buf3, form, xpack, false);
  } else {
    PF_HIP(hipEventRecord(ctx->ev_start, ctx->stream));
    moved = queue_filter<T>(ctx->stream, ctx->num_cu, shape, c, dt, a, S, X, ldx, Y, ldy, K, coef,
                            D, buf3, form, xpack);
  }
  if (bytes) *bytes += moved;
  PF_HIP(hipEventRecord(ctx->ev_stop, ctx->stream));
  PF_HIP(hipEventSynchronize(ctx->ev_stop));
  float ms = 0.0f;
  PF_HIP(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop));
  ctx->filter_gpu_s += 1e-3 * ms;
  long long launches = K + 1;
  if (form == POLFED_FORM_FORWARD) {  // steps 1 .. last non-zero c_k, at least one
    launches = 1;
    for (long long k = K; k >= 1; --k)
      if (coef[k] != 0.0) {
        launches = k;
        break;
      }
  }
  ctx->filter_launches += (double)launches;
  ctx->filter_bytes += moved;
}

// ------------------------------------------------------- chain helpers --

static void validate_model(const polfed_model *m) {
  PF_REQUIRE(m != nullptr, "model is NULL");
  PF_REQUIRE(m->L % 2 == 0, "L must be even");
  PF_REQUIRE(m->L >= 4 && m->L <= 30, "L must be in [4, 30]");
  PF_REQUIRE(!(m->J2 != 0.0 && m->L < 6), "J2 != 0 needs L >= 6");
  PF_REQUIRE(m->h != nullptr, "h is NULL");
  for (int i = 0; i < m->L; ++i) PF_REQUIRE(std::isfinite(m->h[i]), "h must be finite");
  PF_REQUIRE(std::isfinite(m->J1) && std::isfinite(m->J2) && std::isfinite(m->Delta),
             "couplings must be finite");
}

void make_chain(polfed_ctx *ctx, const polfed_model *m, Chain &c) {
  validate_model(m);
  c.L = m->L;
  c.J1 = m->J1;
  c.J2 = m->J2;
  c.Delta = m->Delta;
  for (int i = 0; i < 32; ++i) c.h[i] = (i < m->L) ? m->h[i] : 0.0;
  c.basis = &ctx->basis(m->L);
  c.diag.ensure(sizeof(double) * c.basis->n);
  launch_diag(ctx->stream, c, c.diag.as<double>());
}

// ------------------------------------------------------------ bounds --

void run_bounds(polfed_ctx *ctx, const Chain &c, int steps, unsigned long long seed, double &E0,
                double &E1, double &r0, double &r1) {
  const long long n = c.basis->n;
  steps = (int)std::min<long long>(steps, n - 1);
  if (steps < 1) steps = 1;
  hipStream_t st = ctx->stream;
  double *vec = static_cast<double *>(ctx->buf("bnd_vec").ensure(sizeof(double) * 4 * n));
  double *v[3] = {vec, vec + n, vec + 2 * n};
  double *w = vec + 3 * n;
  const int nblk = (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 4LL * ctx->num_cu));
  double *sc = static_cast<double *>(
      ctx->buf("bnd_scal").ensure(sizeof(double) * (2 * (size_t)steps + 2 + 2 * (size_t)nblk)));
  double *alpha = sc;
  double *beta = sc + steps;  // beta[0..steps]
  double *part = sc + 2 * steps + 1;
  double *part2 = part + nblk;
  launch_fill(st, beta, 1, 0.0);
  launch_philox_fill(st, n, 1, v[0], 1, seed, 0x5eedu);
  launch_dot_partials(st, n, v[0], v[0], part2, nblk);
  launch_lanczos_normalize(st, n, v[0], v[0], part2, nblk, beta + steps);  // scratch beta slot
  launch_fill(st, beta, 1, 0.0);
  attach_pattern(ctx, c, shape_for(ctx, c.L, 1, false));
  for (int k = 0; k < steps; ++k) {
    double *vk = v[k % 3];
    double *vprev = (k >= 1) ? v[(k + 2) % 3] : nullptr;
    double *vnext = v[(k + 1) % 3];
    StepArgs<double> a = base_args<double>(c, c.diag.as<double>());
    a.V = vk;
    a.ldv = 1;
    a.out = w;
    a.ldo = 1;
    a.dscale = 1.0;
    a.w1 = 0.5 * c.J1;
    a.w2 = 0.5 * c.J2;
    launch_step<double>(st, 1, a, shape_for(ctx, c.L, 1, false), ctx->num_cu);
    launch_dot_partials(st, n, vk, w, part, nblk);
    launch_lanczos_update(st, n, w, vk, vprev, part, nblk, alpha + k, beta + k, part2);
    launch_lanczos_normalize(st, n, w, vnext, part2, nblk, beta + k + 1);
  }
  std::vector<double> ha(steps), hb(steps + 1);
  PF_HIP(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * steps, hipMemcpyDeviceToHost, st));
  PF_HIP(hipMemcpyAsync(hb.data(), beta, sizeof(double) * (steps + 1), hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
  std::vector<double> off(steps, 0.0);
  for (int k = 1; k < steps; ++k) off[k] = hb[k];
  double ylo, yhi;
  tridiag_extremes(ha, off, E0, E1, ylo, yhi);
  r0 = std::fabs(hb[steps] * ylo);
  r1 = std::fabs(hb[steps] * yhi);
}

// ------------------------------------------------------------- the solve --

static int next_pow2_le(int x) {
  int s = 1;
  while (s * 2 <= x) s *= 2;
  return s;
}

int choose_block(int L, int nev, int precision);

// Block size: the autotuner's entry for (L, precision, nev) if the context
// holds one, else the built-in rule.
static int block_for(const polfed_ctx *ctx, int L, int nev, int precision) {
  auto it = ctx->blocks.find(std::make_tuple(L, precision, nev));
  if (it != ctx->blocks.end()) return it->second;
  return choose_block(L, nev, precision);
}

static polfed_opts resolve_opts(const polfed_opts *in) {
  polfed_opts o;
  polfed_default_opts(&o);
  if (in) o = *in;
  if (o.p <= 0.0) o.p = 0.17;
  if (o.window_factor <= 0.0) o.window_factor = 1.5;
  if (o.tol <= 0.0) o.tol = 1e-10;
  if (o.eta <= 0.0) o.eta = 1e-3;
  if (o.bounds_steps <= 0) o.bounds_steps = 200;
  if (o.dos_moments <= 0) o.dos_moments = 256;
  if (o.dos_vectors <= 0) o.dos_vectors = 4;
  PF_REQUIRE(o.dos == POLFED_DOS_GAUSS || o.dos == POLFED_DOS_KPM, "dos must be 0 or 1");
  PF_REQUIRE(o.damping == POLFED_DAMP_NONE || o.damping == POLFED_DAMP_JACKSON,
             "damping must be 0 or 1");
  PF_REQUIRE(o.dos_moments <= (1 << 20), "dos_moments must be at most 2^20");
  PF_REQUIRE(o.precision == 0 || o.precision == 1, "precision must be 0 or 1");
  PF_REQUIRE(o.target_kind == 0 || o.target_kind == 1, "target_kind must be 0 or 1");
  if (o.target_kind == 0) PF_REQUIRE(o.target > 0.0 && o.target < 1.0, "eps target must be in (0,1)");
  return o;
}

// The state of one POLFED solve (one realisation): setup, then alternately
// filter_X() / [the filter, alone or batched] / lanczos_step() until done,
// then finalize().  Device state that must live across Lanczos steps is
// owned here; scratch that is consumed within one step is the context's.
// Residual bar of returned pairs in FP32-filter mode: a result whose FP64
// refinement could not bring every residual to 1e-8 ||H|| (this happens when
// the Gaussian density of states overestimated the window, so that wanted
// values sit below p where the filter separates them poorly) is recomputed
// with the FP64 filter; info->refine_passes is then -1.
constexpr double kFp32ResidBar = 1e-8;
// Widest filter window (in units of N_ev) the solve grows to when the
// Gaussian DOS has sized it too narrow: the default 1.5 doubled three times.
constexpr double kMaxWindowFactor = 12.0;
// Largest automatic filter order of the FP32 filter: its rounding error
// relative to the FP64 filter, measured at about 3.5 eps32 sqrt(K) with
// eps32 = 2^-24, stays below 1e-4 up to K ~ 2.3e5; 2e5 keeps a margin.
constexpr long long kFp32MaxOrder = 200000;
// Retries with the bounds margin eta doubled after a filter left [-1, 1].
constexpr int kBoundsRetries = 3;

template <class T>
struct Realization {
  polfed_ctx *ctx = nullptr;
  Chain c;
  polfed_opts o;
  int nev = 0;
  bool fp32 = sizeof(T) == 4;
  long long n = 0;
  int s = 0, P = 0, m_max = 0, nwin = 0;
  double E0 = 0, E1 = 0, r0 = 0, r1 = 0, E0w = 0, E1w = 0, a = 0, b = 0;
  double sigma_H = 0, sigma = 0, normH = 0, tau = 0;
  long long K = 0;
  std::vector<double> coef;
  double D = 1.0;
  DevBuf Qb, Tmb, dtb, Xb, Yb, Bb, coefb, chebb;
  // eigenvectors of the T_m of the last convergence check (ms_prev x ms_prev),
  // the warm start of the next check's eigensolve
  DevBuf Vprevb, thprevb, Wb;
  int ms_prev = 0;
  int m_done = 0, nconv = 0, refills = 0;
  // batch member that failed with an error of its own (bounds, breakdown,
  // invalid target): its status, and it takes no further part
  int err = 0;
  int above = 0;  // Ritz values with theta >= p at the last convergence check
  bool done = false;
  double t_start = 0, t_bounds = 0, t_filter = 0, t_orth = 0, t_eig = 0, bytes = 0;
  double filter_gpu_s = 0, filter_launches = 0;

  double *Q() const { return Qb.as<double>(); }
  double *Tm() const { return Tmb.as<double>(); }
  T *dt() const { return dtb.as<T>(); }
  T *Xs() const { return Xb.as<T>(); }
  T *Ys() const { return Yb.as<T>(); }
  double *Bcur() const { return Bb.as<double>(); }
  double *BT() const { return Bb.as<double>() + (size_t)s * s; }

  void setup(polfed_ctx *ctx_, const polfed_model *model, const polfed_opts &o_, int nev_);
  const T *filter_X();
  void lanczos_step();
  // lanczos_step in parts, for the batch driver: the block (Lan1,
  // reorthogonalisation, QR, T_m), returning whether a convergence check is
  // due; the check's eigenproblem (T_m, or W^T T_m W for a warm start, into
  // A and its starting vectors into V0, both ms x ms); and the check itself
  // from the eigenpairs (th ascending, Vt columns).
  bool lanczos_block();
  int check_size() const { return m_done * s; }
  void check_prepare(double *A, double *V0);
  void check_finish(const double *th, const double *Vt);
  void check_single();  // prepare, sym_eig, finish
  int finalize(double *evals, double *evecs, double *resid, polfed_info *info);
  // finalize in phases, for the batch driver (which runs the refinement
  // filters of its members as batched launches): the Rayleigh-Ritz step on
  // the final T_m's candidates, returning whether an FP64 refinement pass is
  // wanted; a pass's input Vn and coefficients; the pass's filter UR =
  // P^{K_r}(H~) Vn alone; its orthonormalisation and Rayleigh-Ritz,
  // returning whether another pass is wanted; the outputs.
  bool fin_begin();
  void refine_prepare();
  void refine_filter_single();
  bool refine_finish();
  int fin_end(double *evals, double *evecs, double *resid, polfed_info *info);
  // state of the phases: the Rayleigh-Ritz space UR, its Ritz vectors WR,
  // a pass's input Vn, the returned vectors Vout, and H~'s diagonal in FP64
  DevBuf URb, WRb, Vnb, Voutb, dt64b;
  int nc = 0, q = 0, qpad = 0, ldr = 0, ldo = 0, nout = 0, passes = 0;
  bool converged_fin = false;
  std::vector<double> Efin, Esel, rres, coef_r;
  double D_r = 1.0, rmax = 0.0, refine_target = 0.0, t3 = 0.0, tr0 = 0.0;
  double t_refine = 0.0, refine_bytes = 0.0, rr_apps = 0.0, ctx_gpu0 = 0.0, ctx_launch0 = 0.0;
  long long K_r = 0;
  // The filter window held fewer than nev Ritz values with theta >= p at
  // the last check: the order K from the Gaussian DOS made the main lobe too
  // narrow for nev eigenvalues (a DOS that is low at the target, as in short
  // strongly disordered chains), and outside the lobe theta is no measure of
  // nearness to the target.  Only for an automatic K.
  bool window_short() const { return o.K <= 0 && above < nev; }

 private:
  double finish(const double *X, long long ldx, const std::vector<int> &idx,
                const std::vector<double> &Ev);
  std::vector<int> nearest(const std::vector<double> &E, const std::vector<char> &ok, int k) const;
  double rayleigh_ritz(int k);
  int cholqr2(double *X, double *out, long long ldo);
  void refill_block(const double *Uorig, double *out, long long ldo, int pc, int j);
};

template <class T>
void Realization<T>::setup(polfed_ctx *ctx_, const polfed_model *model, const polfed_opts &o_,
                           int nev_) {
  ctx = ctx_;
  o = o_;
  nev = nev_;
  hipStream_t st = ctx->stream;
  t_start = now_s();
  make_chain(ctx, model, c);
  n = c.basis->n;
  PF_REQUIRE(nev >= 1 && nev <= n, "nev must be in [1, dim]");
  if (o.block_size == 0) o.block_size = block_for(ctx, c.L, nev, o.precision);
  PF_REQUIRE(o.block_size >= 1 && o.block_size <= 64 &&
                 (o.block_size & (o.block_size - 1)) == 0,
             "block_size must be a power of two in [1, 64]");
  s = o.block_size;

  // spectral bounds, widened by the residual bounds and eta (E1 - E0)
  run_bounds(ctx, c, o.bounds_steps, o.seed ^ 0xb0b0ull, E0, E1, r0, r1);
  const double width = E1 - E0;
  PF_REQUIRE(width > 0.0, "spectrum has zero width");
  E0w = E0 - r0 - o.eta * width;
  E1w = E1 + r1 + o.eta * width;
  a = 2.0 / (E1w - E0w);
  b = -(E0w + E1w) / (E1w - E0w);
  sigma_H = (o.target_kind == 0) ? E0 + o.target * width : o.target;
  sigma = a * sigma_H + b;
  PF_REQUIRE(std::fabs(sigma) < 1.0, "target lies outside the spectral bounds");
  normH = std::max(std::fabs(E0), std::fabs(E1));
  t_bounds = now_s() - t_start;

  // order from the density of states for a window of N_win eigenvalues
  nwin = (int)std::min<long long>((long long)std::ceil(o.window_factor * nev), n);
  K = o.K;
  if (K <= 0) {
    // FP32 filter: its rounding error grows like eps32 sqrt(K); beyond the
    // cap the window is widened until K fits (the wider window then counts
    // as one wider than the default for the stop rule)
    const long long cap = (o.max_order > 0) ? o.max_order : kFp32MaxOrder;
    const int nwin0 = nwin;
    if (o.dos == POLFED_DOS_KPM) {
      // kernel polynomial DOS from Chebyshev moments of this H~
      std::vector<double> mu;
      dos_moments(ctx, c, a, b, o.dos_moments, o.dos_vectors, nullptr, o.seed ^ 0xd05d05ull, mu);
      K = choose_order_kpm(mu, n, sigma, nwin, o.p, o.damping);
      if (fp32 && K > cap)
        nwin = capped_window_kpm(mu, n, sigma, nwin, o.p, cap, &K, o.damping);
    } else {
      double rho = 0.0;
      const double Gamma = dos_gamma(c.L, c.J1, c.J2, c.Delta, c.h);
      const double Ebar = trace_mean(c.L, c.J1, c.J2, c.Delta);
      K = choose_order(n, Ebar, Gamma, E0w, E1w, sigma, nwin, o.p, &rho, o.damping);
      if (fp32 && K > cap)
        nwin = capped_window(n, Ebar, Gamma, E0w, E1w, sigma, nwin, o.p, cap, &K, o.damping);
    }
    if (nwin != nwin0) o.window_factor = std::max(o.window_factor, (double)nwin / nev);
  }
  cheb_coeffs(sigma, K, coef, D, o.damping);
  // column cap: 8 N_win + 8 s in whole blocks, at most n, and the Lanczos
  // basis within half of the device memory free now (the Rayleigh-Ritz
  // step needs room for three more blocks of the candidates' width)
  long long cols = (o.max_cols > 0) ? o.max_cols : 8LL * nwin + 8LL * s;
  cols = std::min<long long>(cols, (n / s) * s);
  {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) {
      const long long cols_mem = ((long long)(0.5 * (double)free_b / (8.0 * (double)n)) / s) * s;
      if (cols_mem >= s) cols = std::min(cols, cols_mem);
    }
  }
  m_max = (int)std::max<long long>(1, cols / s);
  P = m_max * s;
  // convergence threshold on ||B t~||: FP64 filter 1e-10; FP32 filter
  // eps32 sqrt(K), the size of its rounding errors.  The rounding errors are
  // spread over the whole spectrum and the FP64 refinement removes them in one
  // short pass; what it removes slowly is mixing with eigenvectors just
  // outside the window, which only Lanczos convergence itself suppresses, so
  // the FP32 run is taken down to this level rather than stopped above it.
  tau = fp32 ? std::max(1e-10, 1.1920929e-7 * std::sqrt((double)K)) : 1e-10;

  Qb.ensure(sizeof(double) * (size_t)n * P);
  Tmb.ensure(sizeof(double) * (size_t)P * P);
  dtb.ensure(sizeof(T) * n);
  Xb.ensure(sizeof(T) * (size_t)n * s);
  Yb.ensure(sizeof(T) * (size_t)n * s);
  Bb.ensure(sizeof(double) * 2 * (size_t)s * s);
  launch_scaled_diag<T>(st, n, c.diag.as<double>(), a, b, dt());
  launch_fill(st, Tm(), (long long)P * P, 0.0);

  // start block Q_1: Philox entries, orthonormalised
  double *U = static_cast<double *>(ctx->buf("U").ensure(sizeof(double) * (size_t)n * s));
  launch_philox_fill(st, n, s, U, s, o.seed, 1u);
  if (cholqr2(U, Q(), P) != 0) throw Error(POLFED_EBREAKDOWN, "start block is rank deficient");
}

// CholeskyQR2 of X (n x s, ld s) into out (ld ldo); Bcur = its R factor.
// Returns the flag of the first pivot below 1e-14 of the largest diagonal
// of the Gram matrix (0 = fine): beyond a condition number of ~1e7
// CholeskyQR2 no longer restores orthogonality, and the refill path takes
// over.
template <class T>
int Realization<T>::cholqr2(double *X, double *out, long long ldo) {
  hipStream_t st = ctx->stream;
  DevBuf &partials = ctx->buf("partials");
  double *sm = static_cast<double *>(ctx->buf("cqr").ensure(sizeof(double) * 5 * 64 * 64));
  double *G = sm, *Rinv1 = sm + 4096, *B1 = sm + 2 * 4096, *Rinv2 = sm + 3 * 4096, *B2 = sm + 4 * 4096;
  double *U2 = static_cast<double *>(ctx->buf("U2").ensure(sizeof(double) * (size_t)n * s));
  int *flag = static_cast<int *>(ctx->buf("flag").ensure(64));
  launch_gram(st, n, s, s, X, s, X, s, G, s, partials, ctx->num_cu);
  launch_chol(st, s, G, Rinv1, B1, flag, 1e-14);
  launch_update(st, n, s, s, 1.0, X, s, Rinv1, s, 0.0, U2, s);
  launch_gram(st, n, s, s, U2, s, U2, s, G, s, partials, ctx->num_cu);
  launch_chol(st, s, G, Rinv2, B2, flag + 1, 1e-14);
  launch_update(st, n, s, s, 1.0, U2, s, Rinv2, s, 0.0, out, ldo);
  launch_small_gemm(st, s, s, s, B2, s, B1, s, Bcur(), s, 0);
  int hf[2] = {0, 0};
  PF_HIP(hipMemcpyAsync(hf, flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
  return hf[0] ? hf[0] : hf[1];
}

// The block lost rank (the Krylov space is nearly exhausted, which happens
// when n is small).  Keep the well-conditioned directions of U and refill
// the rest with random vectors orthogonal to Qm; then B_{j+1} = Q_{j+1}^T U,
// so that U = Q_{j+1} B_{j+1} still holds on the kept directions (B is no
// longer triangular; T_m does not need it to be).
template <class T>
void Realization<T>::refill_block(const double *Uorig, double *out, long long ldo, int pc, int j) {
  hipStream_t st = ctx->stream;
  DevBuf &partials = ctx->buf("partials");
  ++refills;
  double *Wg = static_cast<double *>(ctx->buf("Wg").ensure(sizeof(double) * ((size_t)s * s * 4 + 2 * s)));
  double *G = Wg + (size_t)3 * s * s;
  double *U = static_cast<double *>(ctx->buf("U").ensure(sizeof(double) * (size_t)n * s));
  double *U2 = static_cast<double *>(ctx->buf("U2").ensure(sizeof(double) * (size_t)n * s));
  double *Cproj = static_cast<double *>(ctx->buf("Cproj").ensure(sizeof(double) * (size_t)P * s));
  launch_gram(st, n, s, s, Uorig, s, Uorig, s, G, s, partials, ctx->num_cu);
  launch_symmetrize(st, s, G, s);
  double *lam = Wg + (size_t)2 * s * s, *W = Wg;
  sym_eig(st, s, G, lam, W, ctx->buf("eigwork_small"));
  std::vector<double> hl(s), hW((size_t)s * s);
  PF_HIP(hipMemcpyAsync(hl.data(), lam, sizeof(double) * s, hipMemcpyDeviceToHost, st));
  PF_HIP(hipMemcpyAsync(hW.data(), W, sizeof(double) * s * s, hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
  const double lmax = std::max(hl[s - 1], 0.0);
  // kept directions: U w_i / sqrt(lambda_i) for lambda_i > 1e-20 lambda_max
  std::vector<double> M((size_t)s * s, 0.0);
  int r = 0;
  for (int i = s - 1; i >= 0; --i) {
    if (!(hl[i] > 1e-20 * lmax) || lmax == 0.0) continue;
    for (int k = 0; k < s; ++k) M[(size_t)k * s + r] = hW[(size_t)k * s + i] / std::sqrt(hl[i]);
    ++r;
  }
  double *Md = Wg + (size_t)s * s;
  PF_HIP(hipMemcpyAsync(Md, M.data(), sizeof(double) * s * s, hipMemcpyHostToDevice, st));
  launch_update(st, n, s, s, 1.0, Uorig, s, Md, s, 0.0, U2, s);  // columns >= r are zero
  if ((long long)pc + s > n) {
    // no room for s new directions (only at the last block of a tiny
    // problem, where only B_{j+1} is used): keep the r directions
    launch_cast<double, double>(st, n, s, U2, s, out, ldo);
    launch_gram(st, n, s, s, out, ldo, Uorig, s, Bcur(), s, partials, ctx->num_cu);
    return;
  }
  // random columns r..s-1, then the whole block against Qm (twice) and QR
  launch_philox_fill(st, n, s - r, U2 + r, s, o.seed + 977ull * (j + 1) + 13ull * refills, 2u);
  for (int pass = 0; pass < 2; ++pass) {
    launch_gram(st, n, pc, s, Q(), P, U2, s, Cproj, s, partials, ctx->num_cu);
    launch_update(st, n, pc, s, -1.0, Q(), P, Cproj, s, 1.0, U2, s);
  }
  PF_HIP(hipMemcpyAsync(U, U2, sizeof(double) * n * s, hipMemcpyDeviceToDevice, st));
  if (cholqr2(U, out, ldo) != 0)
    throw Error(POLFED_EBREAKDOWN, "Lanczos block lost rank and could not be refilled");
  launch_gram(st, n, s, s, out, ldo, Uorig, s, Bcur(), s, partials, ctx->num_cu);
}

// Stage Q_j (j = m_done) as the filter input in T (a fixed buffer, so that a
// captured filter graph stays valid from block to block).
template <class T>
const T *Realization<T>::filter_X() {
  launch_cast<double, T>(ctx->stream, n, s, Q() + (size_t)m_done * s, P, Xs(), s);
  return Xs();
}

// One block-Lanczos step on the filtered block Y = P(H~) Q_j (in Ys()):
// eqs. (Lan1)-(Lan2) with full reorthogonalisation, T_m, and the
// convergence test on the eigenpairs of T_m.
template <class T>
bool Realization<T>::lanczos_block() {
  hipStream_t st = ctx->stream;
  DevBuf &partials = ctx->buf("partials");
  const int j = m_done;
  double t1 = now_s();
  double *U = static_cast<double *>(ctx->buf("U").ensure(sizeof(double) * (size_t)n * s));
  double *Usave = static_cast<double *>(ctx->buf("Usave").ensure(sizeof(double) * (size_t)n * s));
  double *Cproj = static_cast<double *>(ctx->buf("Cproj").ensure(sizeof(double) * (size_t)P * s));
  double *Ablk = static_cast<double *>(ctx->buf("Ablk").ensure(sizeof(double) * 64 * 64));
  launch_cast<T, double>(st, n, s, Ys(), s, U, s);
  double *Qj = Q() + (size_t)j * s;
  // Lan1: U -= Q_{j-1} B_j^T ; A_j = sym(Q_j^T U) ; U -= Q_j A_j
  if (j > 0) launch_update(st, n, s, s, -1.0, Q() + (size_t)(j - 1) * s, P, BT(), s, 1.0, U, s);
  launch_gram(st, n, s, s, Qj, P, U, s, Ablk, s, partials, ctx->num_cu);
  launch_symmetrize(st, s, Ablk, s);
  {
    // bounds guard: A_j = Q_j^T P(H~) Q_j has entries of size <= max|P| on
    // the spectrum, about 1 when [E0w, E1w] encloses it; outside [-1, 1] the
    // Chebyshev terms grow like cosh(K acosh|x|), so an eigenvalue beyond the
    // widened bounds shows up here as huge or non-finite entries
    std::vector<double> ha((size_t)s * s);
    PF_HIP(hipMemcpyAsync(ha.data(), Ablk, sizeof(double) * s * s, hipMemcpyDeviceToHost, st));
    PF_HIP(hipStreamSynchronize(st));
    for (double v : ha)
      if (!(std::fabs(v) <= 4.0))
        throw Error(POLFED_EBOUNDS,
                    "filter left [-1, 1]: the spectrum extends beyond the widened Lanczos "
                    "bounds (raise bounds_steps or eta)");
  }
  launch_update(st, n, s, s, -1.0, Qj, P, Ablk, s, 1.0, U, s);
  PF_HIP(hipMemcpy2DAsync(Tm() + (size_t)j * s * P + j * s, sizeof(double) * P, Ablk,
                          sizeof(double) * s, sizeof(double) * s, s, hipMemcpyDeviceToDevice, st));
  // full reorthogonalisation against Q_1..Q_j, twice
  const int pc = (j + 1) * s;
  for (int pass = 0; pass < 2; ++pass) {
    launch_gram(st, n, pc, s, Q(), P, U, s, Cproj, s, partials, ctx->num_cu);
    launch_update(st, n, pc, s, -1.0, Q(), P, Cproj, s, 1.0, U, s);
  }
  // Lan2: Q_{j+1} B_{j+1} = U  (after the last block Q_{j+1} lands in U:
  // only B_{j+1} is needed)
  double *Qnext = (j + 1 < m_max) ? Q() + (size_t)(j + 1) * s : U;
  const long long ldq = (j + 1 < m_max) ? P : s;
  PF_HIP(hipMemcpyAsync(Usave, U, sizeof(double) * n * s, hipMemcpyDeviceToDevice, st));
  if (cholqr2(U, Qnext, ldq) != 0) refill_block(Usave, Qnext, ldq, pc, j);
  launch_small_transpose(st, s, s, Bcur(), s, BT(), s);
  if (j + 1 < m_max) {
    PF_HIP(hipMemcpy2DAsync(Tm() + (size_t)(j + 1) * s * P + j * s, sizeof(double) * P, Bcur(),
                            sizeof(double) * s, sizeof(double) * s, s, hipMemcpyDeviceToDevice, st));
    PF_HIP(hipMemcpy2DAsync(Tm() + (size_t)j * s * P + (j + 1) * s, sizeof(double) * P, BT(),
                            sizeof(double) * s, sizeof(double) * s, s, hipMemcpyDeviceToDevice, st));
  }
  double t2 = now_s();
  t_orth += t2 - t1;
  m_done = j + 1;
  const int ms = m_done * s;
  const int check_from = std::max(s, std::min(nev, P));
  const bool due = (ms >= check_from || m_done == m_max);
  if (!due && m_done >= m_max) done = true;
  return due;
}

template <class T>
void Realization<T>::check_prepare(double *A, double *V0) {
  hipStream_t st = ctx->stream;
  const int ms = m_done * s;
  PF_HIP(hipMemcpy2DAsync(A, sizeof(double) * ms, Tm(), sizeof(double) * P, sizeof(double) * ms, ms,
                          hipMemcpyDeviceToDevice, st));
  if (ms_prev > 0 && ms_prev == ms - s) {
    // warm start: T_m = [[T_{m-1}, C], [C^T, A_m]] and T_{m-1} = V D V^T
    // from the last check, so W^T T_m W with W = blockdiag(V, I) is diagonal
    // but for its last s rows and columns; Jacobi on it needs far fewer
    // sweeps
    double *tmp = static_cast<double *>(Wb.ensure(sizeof(double) * (size_t)P * P));
    launch_embed_block(st, ms, ms_prev, Vprevb.as<double>(), V0);
    launch_small_gemm(st, ms, ms, ms, A, ms, V0, ms, tmp, ms, 0);
    launch_small_gemm(st, ms, ms, ms, V0, ms, tmp, ms, A, ms, 1);
    launch_symmetrize(st, ms, A, ms);
  } else {
    launch_embed_block(st, ms, 0, nullptr, V0);  // identity
  }
}

template <class T>
void Realization<T>::check_finish(const double *th, const double *Vt) {
  hipStream_t st = ctx->stream;
  DevBuf &partials = ctx->buf("partials");
  const int ms = m_done * s;
  const double t2 = now_s();
  Vprevb.ensure(sizeof(double) * (size_t)P * P);
  thprevb.ensure(sizeof(double) * (size_t)P);
  PF_HIP(hipMemcpyAsync(thprevb.p, th, sizeof(double) * (size_t)ms, hipMemcpyDeviceToDevice, st));
  PF_HIP(hipMemcpyAsync(Vprevb.p, Vt, sizeof(double) * (size_t)ms * ms, hipMemcpyDeviceToDevice, st));
  ms_prev = ms;
  // residual_i = ||B_{j+1} t~_i||, t~_i the last s components of t_i
  double *Rres = static_cast<double *>(ctx->buf("Rres").ensure(sizeof(double) * (size_t)64 * P));
  double *tr = static_cast<double *>(ctx->buf("tres").ensure(sizeof(double) * (size_t)P));
  launch_small_gemm(st, s, s, ms, Bcur(), s, Vt + (size_t)(ms - s) * ms, ms, Rres, ms, 0);
  launch_colnorms(st, s, ms, Rres, ms, tr, partials, ctx->num_cu);
  std::vector<double> theta(ms), tres(ms);
  PF_HIP(hipMemcpyAsync(theta.data(), th, sizeof(double) * ms, hipMemcpyDeviceToHost, st));
  PF_HIP(hipMemcpyAsync(tres.data(), tr, sizeof(double) * ms, hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
  // converged: theta_i >= p and ||B t~_i|| <= tau; when fewer than nev
  // Ritz values exceed p (the Gaussian DOS overestimated the window), the
  // nev largest theta take their place
  double thr = o.p;
  above = 0;
  for (int i = 0; i < ms; ++i) above += theta[i] >= o.p;
  if (above < nev) thr = theta[std::max(0, ms - nev)];  // ascending order
  // a window wider than the default 1.5 N_ev (a widened rerun, or the
  // caller's choice) holds many eigenvalues where P is nearly flat, and N_ev
  // converged pairs anywhere in it need not be the N_ev nearest: there the
  // nev largest theta must be the converged ones
  if (o.window_factor > 1.5 + 1e-9 && ms >= nev) thr = std::max(thr, theta[ms - nev]);
  nconv = 0;
  int nconv_loose = 0;
  for (int i = 0; i < ms; ++i) {
    if (theta[i] >= thr && tres[i] <= tau) ++nconv;
    if (theta[i] >= thr && tres[i] <= 30.0 * tau) ++nconv_loose;
  }
  // FP32 filter at the column cap: a Ritz pair whose estimate stalls above
  // eps32 sqrt(K) (its rounding floor) still counts if it is within 30x of
  // it; the FP64 refinement and the residual bar decide the result's
  // accuracy (and an FP64 re-solve follows if it misses the bar)
  if (fp32 && m_done >= m_max && nconv < nev && nconv_loose >= nev) nconv = nconv_loose;
  t_eig += now_s() - t2;
  if (nconv >= nev || m_done >= m_max) done = true;
  if (std::getenv("POLFED_VERBOSE"))
    fprintf(stderr, "[polfed] L=%d block %d/%d: %d of %d converged (filter %.2f s so far)\n", c.L,
            m_done, m_max, nconv, nev, t_filter);
}


template <class T>
void Realization<T>::lanczos_step() {
  if (lanczos_block()) check_single();
}

template <class T>
void Realization<T>::check_single() {
  const double t2 = now_s();
  const int ms = m_done * s;
  double *Tw = static_cast<double *>(ctx->buf("Tw").ensure(sizeof(double) * (size_t)P * P));
  double *Vt = static_cast<double *>(ctx->buf("Vt").ensure(sizeof(double) * (size_t)P * P));
  double *V0 = static_cast<double *>(ctx->buf("V0").ensure(sizeof(double) * (size_t)P * P));
  double *th = static_cast<double *>(ctx->buf("theta").ensure(sizeof(double) * (size_t)P));
  check_prepare(Tw, V0);
  sym_eig(ctx->stream, ms, Tw, th, Vt, ctx->buf("eigwork"), V0);
  t_eig += now_s() - t2;
  check_finish(th, Vt);
}

// Vout (n x nout, ld ldo) <- columns idx of X (ld ldx); then normalise, fix
// signs and compute ||H v - E v||.  Returns the largest residual.
template <class T>
double Realization<T>::finish(const double *X, long long ldx, const std::vector<int> &idx,
                              const std::vector<double> &Ev) {
  hipStream_t st = ctx->stream;
  DevBuf &partials = ctx->buf("partials");
  double *Vout = Voutb.as<double>();
  double *HV = static_cast<double *>(ctx->buf("HV").ensure(sizeof(double) * (size_t)n * ldo));
  double *vecs = static_cast<double *>(ctx->buf("vecs").ensure(sizeof(double) * 4 * (size_t)ldo));
  double *nrm = vecs, *Ed = vecs + ldo, *rd = vecs + 2 * ldo, *sg = vecs + 3 * ldo;
  int *didx = static_cast<int *>(ctx->buf("idx").ensure(sizeof(int) * (size_t)(P + 64) * 2));
  nout = (int)idx.size();
  Esel = Ev;
  rres.assign(nout, 0.0);
  PF_HIP(hipMemcpyAsync(didx, idx.data(), sizeof(int) * nout, hipMemcpyHostToDevice, st));
  launch_gather_cols(st, n, nout, X, ldx, didx, Vout, ldo);
  launch_colnorms(st, n, nout, Vout, ldo, nrm, partials, ctx->num_cu);
  std::vector<double> hn(nout);
  PF_HIP(hipMemcpyAsync(hn.data(), nrm, sizeof(double) * nout, hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < nout; ++i) hn[i] = 1.0 / hn[i];
  PF_HIP(hipMemcpyAsync(nrm, hn.data(), sizeof(double) * nout, hipMemcpyHostToDevice, st));
  launch_scale_cols(st, n, nout, Vout, ldo, nrm);
  launch_sign_factors(st, n, nout, Vout, ldo, sg, partials, ctx->num_cu);
  launch_scale_cols(st, n, nout, Vout, ldo, sg);
  apply_op<double>(ctx, c, c.diag.as<double>(), 0.5 * c.J1, 0.5 * c.J2, Vout, ldo, HV, ldo, nout,
                   false);
  rr_apps += nout;
  PF_HIP(hipMemcpyAsync(Ed, Esel.data(), sizeof(double) * nout, hipMemcpyHostToDevice, st));
  launch_resid_norms(st, n, nout, HV, ldo, Vout, ldo, Ed, rd, partials, ctx->num_cu);
  PF_HIP(hipMemcpyAsync(rres.data(), rd, sizeof(double) * nout, hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
  double rm = 0.0;
  for (int i = 0; i < nout; ++i) rm = std::max(rm, rres[i]);
  return rm;
}

// indices of the k values of E nearest sigma_H (ties -> lower E), taken
// from those with ok[i]; returned ascending in E
template <class T>
std::vector<int> Realization<T>::nearest(const std::vector<double> &E,
                                         const std::vector<char> &ok, int k) const {
  std::vector<int> ord;
  for (int i = 0; i < (int)E.size(); ++i)
    if (ok[i]) ord.push_back(i);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    const double dx = std::fabs(E[x] - sigma_H), dy = std::fabs(E[y] - sigma_H);
    if (dx != dy) return dx < dy;
    return E[x] < E[y];
  });
  if ((int)ord.size() > k) ord.resize(k);
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return E[x] < E[y]; });
  return ord;
}

// Rayleigh-Ritz of H~ on span(UR[:, :k]) (orthonormal): WR = UR Y, the nev
// nearest the target selected and finished; returns their largest residual.
template <class T>
double Realization<T>::rayleigh_ritz(int k) {
  hipStream_t st = ctx->stream;
  DevBuf &partials = ctx->buf("partials");
  DevBuf &eigwork = ctx->buf("eigwork");
  double *UR = URb.as<double>(), *WR = WRb.as<double>();
  double *Gr = static_cast<double *>(ctx->buf("Gr").ensure(sizeof(double) * (size_t)ldr * ldr * 3 + 16));
  double *Yr = Gr + (size_t)ldr * ldr;
  double *epsd = static_cast<double *>(ctx->buf("epsd").ensure(sizeof(double) * (size_t)ldr));
  apply_op<double>(ctx, c, dt64b.as<double>(), 0.5 * a * c.J1, 0.5 * a * c.J2, UR, ldr, WR, ldr, k,
                   false);
  rr_apps += k;
  launch_gram(st, n, k, k, UR, ldr, WR, ldr, Gr, k, partials, ctx->num_cu);
  launch_symmetrize(st, k, Gr, k);
  sym_eig(st, k, Gr, epsd, Yr, eigwork);
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int w = std::min(64, k - c0);
    launch_update(st, n, k, w, 1.0, UR, ldr, Yr + c0, k, 0.0, WR + c0, ldr);
  }
  std::vector<double> eps(k);
  PF_HIP(hipMemcpyAsync(eps.data(), epsd, sizeof(double) * k, hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
  Efin.resize(k);
  for (int i = 0; i < k; ++i) Efin[i] = (eps[i] - b) / a;
  const std::vector<int> sel = nearest(Efin, std::vector<char>(k, 1), nev);
  std::vector<double> Ev;
  for (int i : sel) Ev.push_back(Efin[i]);
  return finish(WR, ldr, sel, Ev);
}

// The final T_m's eigenpairs, the Rayleigh-Ritz step on the candidates and
// the selection of the nev nearest the target.  Returns whether an FP64
// refinement pass is wanted (FP32 filter, residuals above its target).
template <class T>
bool Realization<T>::fin_begin() {
  hipStream_t st = ctx->stream;
  DevBuf &eigwork = ctx->buf("eigwork");
  const int ms = m_done * s;
  converged_fin = nconv >= nev;
  double *Qp = Q();
  // the eigenpairs of the final T_m
  double *Tw = static_cast<double *>(ctx->buf("Tw").ensure(sizeof(double) * (size_t)P * P));
  double *Vt = static_cast<double *>(ctx->buf("Vt").ensure(sizeof(double) * (size_t)P * P));
  double *th = static_cast<double *>(ctx->buf("theta").ensure(sizeof(double) * (size_t)P * 2));
  if (ms_prev == ms) {
    // the last convergence check decomposed this very T_m
    PF_HIP(hipMemcpyAsync(Vt, Vprevb.p, sizeof(double) * (size_t)ms * ms, hipMemcpyDeviceToDevice,
                          st));
    PF_HIP(hipMemcpyAsync(th, thprevb.p, sizeof(double) * (size_t)ms, hipMemcpyDeviceToDevice, st));
  } else {
    PF_HIP(hipMemcpy2DAsync(Tw, sizeof(double) * ms, Tm(), sizeof(double) * P, sizeof(double) * ms,
                            ms, hipMemcpyDeviceToDevice, st));
    sym_eig(st, ms, Tw, th, Vt, eigwork);
  }
  std::vector<double> theta(ms);
  PF_HIP(hipMemcpyAsync(theta.data(), th, sizeof(double) * ms, hipMemcpyDeviceToHost, st));
  PF_HIP(hipStreamSynchronize(st));
  // 7: Rayleigh-Ritz of H~, selection of the nev nearest the target, and
  // residuals with the unscaled H
  t3 = now_s();
  ctx_gpu0 = ctx->filter_gpu_s;
  ctx_launch0 = ctx->filter_launches;
  dt64b.ensure(sizeof(double) * n);
  launch_scaled_diag<double>(st, n, c.diag.as<double>(), a, b, dt64b.as<double>());
  const int nout_max = std::min<long long>(nev, ms);
  ldo = ((nout_max + 7) / 8) * 8;
  Voutb.ensure(sizeof(double) * (size_t)n * ldo);
  int *didx = static_cast<int *>(ctx->buf("idx").ensure(sizeof(int) * (size_t)(P + 64) * 2));

  // candidates: theta >= p (else the nev largest theta); their Ritz vectors
  // Qm t_i span the Rayleigh-Ritz space
  std::vector<int> cand;
  for (int i = 0; i < ms; ++i)
    if (theta[i] >= o.p) cand.push_back(i);
  // at least nev candidates (the nev largest theta when fewer pass p)
  const int want = nev;
  if ((int)cand.size() < want) {
    cand.clear();
    for (int i = ms - 1; i >= 0 && (int)cand.size() < want; --i) cand.push_back(i);
    std::sort(cand.begin(), cand.end());
  }
  nc = (int)cand.size();
  // refined columns (FP32 mode): all candidates, so that every in-window
  // error direction lies in the Rayleigh-Ritz space; padded to kernel
  // widths: whole 64-column launches, then the remainder rounded up to a
  // power of two
  q = nc;
  qpad = 64 * (q / 64);
  if (q % 64) {
    int w = 1;
    while (w < q % 64) w *= 2;
    qpad += w;
  }
  ldr = std::max(((nc + 7) / 8) * 8, qpad);
  PF_HIP(hipMemcpyAsync(didx, cand.data(), sizeof(int) * nc, hipMemcpyHostToDevice, st));
  double *Tsel = static_cast<double *>(ctx->buf("Tsel").ensure(sizeof(double) * (size_t)ms * ldr));
  launch_gather_cols(st, ms, nc, Vt, ms, didx, Tsel, ldr);
  URb.ensure(sizeof(double) * (size_t)n * ldr);
  WRb.ensure(sizeof(double) * (size_t)n * ldr);
  for (int c0 = 0; c0 < nc; c0 += 64) {
    const int w = std::min(64, nc - c0);
    launch_update(st, n, ms, w, 1.0, Qp, P, Tsel + c0, ldr, 0.0, URb.as<double>() + c0, ldr);
  }
  rmax = rayleigh_ritz(nc);
  if (std::getenv("POLFED_VERBOSE"))
    fprintf(stderr, "[polfed] rr: %d candidates, max resid / ||H|| = %.3e\n", nc, rmax / normH);
  // the Lanczos basis and T_m are no longer needed (a batch holds many)
  Qb.release();
  Tmb.release();

  // FP64 refinement of the FP32-filter mode.  The FP32 rounding of the
  // recurrence leaves errors ~eps32 sqrt(K) in the Ritz vectors, spread
  // over the whole spectrum.  Subspace iteration with the FP64 filter
  // P^{K_r}(H~) on the q candidate Ritz vectors damps a component at
  // angular distance u from the target by ~1/(K_r u) relative to the wanted
  // ones, so a short filter removes that spread (K_r = K/4 first); the
  // slower near-window part (damped by theta_k / theta_i per pass) is small
  // because the FP32 Lanczos ran to convergence at the rounding level.
  // Rayleigh-Ritz on the filtered span removes the mixing among candidates.
  // K_r = K/4, K/2, then K, at most 8 passes; target 8e-9 ||H|| (or tol if
  // looser), under the 1e-8 ||H|| bar for returned residuals (the returned
  // residuals are recomputed exactly, so the bar is met, not estimated).
  refine_target = std::max(o.tol, 8e-9) * normH;
  K_r = std::max<long long>(16, K / 4);
  passes = 0;
  return fp32 && rmax > refine_target;
}

// Vn <- the q Ritz vectors nearest the target (padding columns zero), and
// the coefficients of this pass's filter P^{K_r}.
template <class T>
void Realization<T>::refine_prepare() {
  hipStream_t st = ctx->stream;
  tr0 = now_s();
  if (!Vnb.p) {
    Vnb.ensure(sizeof(double) * (size_t)n * ldr);
    launch_fill(st, Vnb.as<double>(), (long long)n * ldr, 0.0);  // padding columns stay zero
  }
  int *didx = static_cast<int *>(ctx->buf("idx").ensure(sizeof(int) * (size_t)(P + 64) * 2));
  const std::vector<int> near = nearest(Efin, std::vector<char>(Efin.size(), 1), q);
  PF_HIP(hipMemcpyAsync(didx, near.data(), sizeof(int) * q, hipMemcpyHostToDevice, st));
  launch_gather_cols(st, n, q, WRb.as<double>(), ldr, didx, Vnb.as<double>(), ldr);
  cheb_coeffs(sigma, K_r, coef_r, D_r, o.damping);
}

// UR <- P^{K_r}(H~) Vn with the single-chain FP64 filter, in whole
// 64-column launches and the power-of-two remainder.
template <class T>
void Realization<T>::refine_filter_single() {
  double *cheb64 =
      static_cast<double *>(ctx->buf("cheb64").ensure(sizeof(double) * 3 * (size_t)n * 64));
  for (int c0 = 0; c0 < qpad; c0 += 64) {
    const int w = std::min(64, qpad - c0);  // 64, or the power-of-two remainder
    run_filter<double>(ctx, c, dt64b.as<double>(), a, w, Vnb.as<double>() + c0, ldr,
                       URb.as<double>() + c0, ldr, K_r, coef_r, D_r, cheb64, false, &refine_bytes,
                       false);
  }
}

// After the pass's filter: SVQB orthonormalisation of UR, Rayleigh-Ritz,
// and the stall check.  Returns whether another pass is wanted.
template <class T>
bool Realization<T>::refine_finish() {
  hipStream_t st = ctx->stream;
  DevBuf &partials = ctx->buf("partials");
  DevBuf &eigwork = ctx->buf("eigwork");
  double *UR = URb.as<double>(), *WR = WRb.as<double>();
  double *Gr = static_cast<double *>(ctx->buf("Gr").ensure(sizeof(double) * (size_t)ldr * ldr * 3 + 16));
  double *Yr = Gr + (size_t)ldr * ldr;
  double *Mr = Yr + (size_t)ldr * ldr;
  double *epsd = static_cast<double *>(ctx->buf("epsd").ensure(sizeof(double) * (size_t)ldr));
  rr_apps += (double)(K_r + 1) * q;
  // SVQB orthonormalisation of UR[:, :q] (twice): UR <- UR W Lambda^{-1/2}
  for (int it = 0; it < 2; ++it) {
    launch_gram(st, n, q, q, UR, ldr, UR, ldr, Gr, q, partials, ctx->num_cu);
    launch_symmetrize(st, q, Gr, q);
    sym_eig(st, q, Gr, epsd, Yr, eigwork);
    std::vector<double> lam(q), W((size_t)q * q);
    PF_HIP(hipMemcpyAsync(lam.data(), epsd, sizeof(double) * q, hipMemcpyDeviceToHost, st));
    PF_HIP(hipMemcpyAsync(W.data(), Yr, sizeof(double) * q * q, hipMemcpyDeviceToHost, st));
    PF_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < q; ++i) {
      const double f = (lam[i] > 1e-28 * lam[q - 1]) ? 1.0 / std::sqrt(lam[i]) : 0.0;
      for (int k = 0; k < q; ++k) W[(size_t)k * q + i] *= f;
    }
    PF_HIP(hipMemcpyAsync(Mr, W.data(), sizeof(double) * q * q, hipMemcpyHostToDevice, st));
    for (int c0 = 0; c0 < q; c0 += 64) {
      const int w = std::min(64, q - c0);
      launch_update(st, n, q, w, 1.0, UR, ldr, Mr + c0, q, 0.0, WR + c0, ldr);
    }
    PF_HIP(hipMemcpy2DAsync(UR, sizeof(double) * ldr, WR, sizeof(double) * ldr,
                            sizeof(double) * q, n, hipMemcpyDeviceToDevice, st));
  }
  PF_HIP(hipStreamSynchronize(st));
  t_refine += now_s() - tr0;
  ++passes;
  const double rprev = rmax;
  rmax = rayleigh_ritz(q);
  if (std::getenv("POLFED_VERBOSE"))
    fprintf(stderr, "[polfed] refine pass %d: K_r %lld, %d vectors, max resid / ||H|| = %.3e\n",
            passes, K_r, q, rmax / normH);
  // a pass at (about) the full order K that gains less than 10% has
  // stalled (a wanted direction missing from, or barely separated
  // within, the refined span); more passes would not reach the target,
  // and the caller's FP64 re-solve is cheaper than running them out
  if (2 * K_r > K && rmax > 0.9 * rprev) return false;
  K_r = std::min<long long>(2 * K_r, K);
  return rmax > refine_target && passes < 8;
}

template <class T>
int Realization<T>::fin_end(double *evals, double *evecs, double *resid, polfed_info *info) {
  hipStream_t st = ctx->stream;
  if (evecs) {
    double *cm = static_cast<double *>(ctx->buf("colmajor").ensure(sizeof(double) * (size_t)n * nout));
    launch_to_colmajor(st, n, nout, Voutb.as<double>(), ldo, cm);
    PF_HIP(hipMemcpyAsync(evecs, cm, sizeof(double) * (size_t)n * nout, hipMemcpyDeviceToHost, st));
  }
  PF_HIP(hipStreamSynchronize(st));
  const double t_rr = now_s() - t3 - t_refine;
  filter_gpu_s += ctx->filter_gpu_s - ctx_gpu0;
  filter_launches += ctx->filter_launches - ctx_launch0;

  for (int i = 0; i < nout; ++i) {
    evals[i] = Esel[i];
    resid[i] = rres[i];
  }
  for (int i = nout; i < nev; ++i) {
    evals[i] = NAN;
    resid[i] = NAN;
  }
  int n_ok = 0;
  double rm = 0.0;
  for (int i = 0; i < nout; ++i) {
    // FP32 mode is held to the FP32 residual bar (its refinement target)
    if (rres[i] <= (fp32 ? std::max(o.tol, kFp32ResidBar) : o.tol) * normH) ++n_ok;
    rm = std::max(rm, rres[i]);
  }
  polfed_info inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.t_bounds = t_bounds;
  inf.E0 = E0;
  inf.E1 = E1;
  inf.E0w = E0w;
  inf.E1w = E1w;
  inf.sigma_energy = sigma_H;
  inf.sigma_tilde = sigma;
  inf.normH = normH;
  inf.K = K;
  inf.nev_window = nwin;
  inf.block_size = s;
  inf.m = m_done;
  inf.n_conv = n_ok;
  inf.refine_passes = passes;
  inf.t_refine = t_refine;
  inf.max_resid = rm;
  inf.t_filter = t_filter;
  inf.t_orth = t_orth;
  inf.t_eig = t_eig;
  inf.t_rr = t_rr;
  inf.t_total = now_s() - t_start;
  inf.hv_apps = (double)(K + 1) * (m_done * s) + rr_apps + o.bounds_steps;
  inf.filter_bytes = bytes + refine_bytes;
  inf.filter_gpu_s = filter_gpu_s;
  inf.filter_launches = filter_launches;
  if (info) *info = inf;
  // the refinement's device state is no longer needed
  URb.release();
  WRb.release();
  Vnb.release();
  Voutb.release();
  dt64b.release();
  // OK only when every returned pair meets the accuracy bar: a run can stop
  // with N_ev converged Ritz pairs and still select an unconverged one as
  // one of the N_ev nearest (its residual then shows it)
  bool all_ok = nout == nev;
  for (int i = 0; i < nout; ++i)
    if (!(rres[i] <= std::max(o.tol, kFp32ResidBar) * normH)) all_ok = false;
  return (converged_fin && all_ok) ? POLFED_OK : POLFED_NOT_CONVERGED;
}

template <class T>
int Realization<T>::finalize(double *evals, double *evecs, double *resid, polfed_info *info) {
  if (fin_begin()) {
    do {
      refine_prepare();
      refine_filter_single();
    } while (refine_finish());
  }
  return fin_end(evals, evecs, resid, info);
}


// ------------------------------------------------------------- drivers --

template <class T>
static int solve_single(polfed_ctx *ctx, const polfed_model *model, const polfed_opts &o, int nev,
                        double *evals, double *evecs, double *resid, polfed_info *info,
                        bool *short_window = nullptr, double *window_factor_used = nullptr) {
  Realization<T> R;
  R.setup(ctx, model, o, nev);
  if (window_factor_used) *window_factor_used = R.o.window_factor;
  T *cheb = static_cast<T *>(ctx->buf("cheb").ensure(sizeof(T) * 3 * (size_t)R.n * R.s));
  while (!R.done) {
    const double t0 = now_s();
    const double g0 = ctx->filter_gpu_s, l0 = ctx->filter_launches;
    const T *X = R.filter_X();
    run_filter<T>(ctx, R.c, R.dt(), R.a, R.s, X, R.s, R.Ys(), R.s, R.K, R.coef, R.D, cheb,
                  R.fp32, &R.bytes);
    R.filter_gpu_s += ctx->filter_gpu_s - g0;
    R.filter_launches += ctx->filter_launches - l0;
    R.t_filter += now_s() - t0;
    R.lanczos_step();
  }
  if (short_window) *short_window = R.window_short();
  return R.finalize(evals, evecs, resid, info);
}


// Info of an FP64 re-solve (i64) after a failed FP32 attempt (first):
// refine_passes = -1, and the attempt's time and work added in.
static void merge_resolve_info(polfed_info &i64, const polfed_info &first) {
  i64.refine_passes = -1;
  i64.t_total += first.t_total;
  i64.t_refine += first.t_total;  // the abandoned FP32 attempt
  i64.hv_apps += first.hv_apps;
  i64.filter_bytes += first.filter_bytes;
  i64.filter_gpu_s += first.filter_gpu_s;
  i64.filter_launches += first.filter_launches;
}

// Time and work of an abandoned attempt added to the info of the result.
static void add_attempt(polfed_info &info, const polfed_info &prev) {
  info.t_total += prev.t_total;
  info.hv_apps += prev.hv_apps;
  info.filter_bytes += prev.filter_bytes;
  info.filter_gpu_s += prev.filter_gpu_s;
  info.filter_launches += prev.filter_launches;
}

// A solve in precision T, repeated with the window sized for twice as many
// eigenvalues (o.window_factor doubled, so K about halves) while the window
// turns out too narrow, up to kMaxWindowFactor; a window still too narrow
// there makes the status NOT_CONVERGED.  o is left at the factor used.
template <class T>
static int solve_widened(polfed_ctx *ctx, const polfed_model *model, polfed_opts &o, int nev,
                         double *evals, double *evecs, double *resid, polfed_info *info) {
  polfed_info prev;
  bool have_prev = false;
  for (;;) {
    bool short_window = false;
    double wf = o.window_factor;
    int rc = solve_single<T>(ctx, model, o, nev, evals, evecs, resid, info, &short_window, &wf);
    o.window_factor = wf;  // the FP32 order cap may have widened it
    if (have_prev) add_attempt(*info, prev);
    if (!short_window) return rc;
    if (2.0 * o.window_factor > kMaxWindowFactor)
      return rc == POLFED_OK ? POLFED_NOT_CONVERGED : rc;
    prev = *info;
    have_prev = true;
    o.window_factor *= 2.0;
  }
}

int solve_one(polfed_ctx *ctx, const polfed_model *model, const polfed_opts *opts_in, int nev,
              double *evals, double *evecs, double *resid, polfed_info *info) {
  polfed_opts o = resolve_opts(opts_in);
  PF_REQUIRE(evals != nullptr && resid != nullptr, "evals and resid must not be NULL");
  polfed_info inf;
  std::memset(&inf, 0, sizeof(inf));
  int rc;
  // a filter that left [-1, 1] (the widened Lanczos bounds still missed part
  // of the spectrum) ends the attempt with POLFED_EBOUNDS: the bounds margin
  // eta is doubled and the solve repeated, three times at most
  for (int attempt = 0;; ++attempt) {
    try {
      if (o.precision == 1) {
        rc = solve_widened<float>(ctx, model, o, nev, evals, evecs, resid, &inf);
        if (inf.max_resid > kFp32ResidBar * inf.normH) {
          // the FP32 result misses the bar: recompute with the FP64 filter
          polfed_opts o64 = o;
          o64.precision = 0;
          polfed_info i64;
          std::memset(&i64, 0, sizeof(i64));
          rc = solve_widened<double>(ctx, model, o64, nev, evals, evecs, resid, &i64);
          merge_resolve_info(i64, inf);
          inf = i64;
        }
      } else {
        rc = solve_widened<double>(ctx, model, o, nev, evals, evecs, resid, &inf);
      }
      break;
    } catch (const Error &e) {
      if (e.code != POLFED_EBOUNDS || attempt == kBoundsRetries) throw;
      o.eta *= 2.0;
    }
  }
  if (info) *info = inf;
  return rc;
}

// Batched solve: realisations are grouped by block size and J2 != 0 (chain
// lengths may mix); each group advances in lock step, one Lanczos block at a
// time, with the filter of all its active members in one persistent launch
// per Chebyshev step (k_step_batched), the K_max + 1 launches of a block
// captured once in a HIP graph and replayed for every block.  Members whose
// order K_i is below K_max idle for the first K_max - K_i steps; members
// that converged are switched off in the device descriptor table.
// Launch shape of the batched step kernel: the context's entry, else the
// single-chain default with the tables as rank method and no column slices.
static StepShape batch_shape_for(const polfed_ctx *ctx, int L, int S, bool fp32) {
  auto it = ctx->batch_shapes.find(std::make_tuple(L, S, fp32 ? 4 : 8));
  if (it != ctx->batch_shapes.end()) return it->second;
  return default_batch_shape(L, S, fp32);
}

// Algorithmic bytes of one realisation's batched Clenshaw filter (the byte
// model of the single-chain filter: each streamed block once per step, the
// state word and diagonal of every row where H~ is applied).
template <class T>
static double batched_filter_bytes(long long n, int S, long long K, const std::vector<double> &coef) {
  double mv = 0.0;
  for (long long jj = 0; jj < K; ++jj) {
    const int streams = 1 + (jj >= 1) + (jj >= 2) + (coef[K - jj] != 0.0);
    mv += (double)n * (S * (double)sizeof(T) * streams + (jj >= 1 ? 4.0 + sizeof(T) : 0.0));
  }
  mv += (double)n * (S * (double)sizeof(T) * (2 + (K >= 1) + (K >= 2)) +
                     (K >= 1 ? 4.0 + sizeof(T) : 0.0));
  return mv;
}

// Fill the chain fields and tile offsets of batch items (rows per tile rpi);
// returns the launch's total tiles.
template <class T>
static long long fill_batch_chains(std::vector<BatchItem<T>> &items,
                                   const std::vector<const Chain *> &chains, long long rpi) {
  long long tiles = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    const Chain &c = *chains[i];
    const Basis &b = *c.basis;
    BatchItem<T> &it = items[i];
    it.states = b.states.as<uint32_t>();
    it.tabA = b.tabA.as<int32_t>();
    it.tabB = b.tabB.as<uint16_t>();
    it.n = b.n;
    it.L = c.L;
    it.half = b.half;
    it.lomask = (1u << b.half) - 1u;
    it.fullmask = (c.L >= 32) ? 0xffffffffu : ((1u << c.L) - 1u);
    it.tile0 = tiles;
    tiles += (b.n + rpi - 1) / rpi;
  }
  return tiles;
}

// The distinct rank tables of a batched launch's chains, to be staged in
// LDS (each item's tab set): at most kMaxBatchTables lengths, each L <=
// kMaxLdsTableL, 96 KB in all; otherwise count = 0 and every realisation
// reads its tables from global memory.
template <class T>
static BatchTables batch_tables(std::vector<BatchItem<T>> &items,
                                const std::vector<const Chain *> &chains) {
  BatchTables bt;
  std::memset(&bt, 0, sizeof(bt));
  std::map<const Basis *, int> idx;
  for (size_t i = 0; i < items.size(); ++i) {
    const Basis *b = chains[i]->basis;
    auto f = idx.find(b);
    if (f == idx.end()) {
      if (bt.count == kMaxBatchTables || chains[i]->L > kMaxLdsTableL) {
        std::memset(&bt, 0, sizeof(bt));
        return bt;
      }
      const int k = bt.count++;
      bt.A[k] = b->tabA.as<int32_t>();
      bt.B[k] = b->tabB.as<uint16_t>();
      bt.half[k] = b->half;
      bt.off[k] = bt.ints;
      bt.ints += (1 << b->half) + (1 << b->half) / 2;
      f = idx.emplace(b, k).first;
    }
    items[i].taboff = bt.off[f->second];
  }
  if ((size_t)bt.ints * sizeof(int32_t) > (size_t)96 * 1024) std::memset(&bt, 0, sizeof(bt));
  return bt;
}

// The FP64 refinement filters UR = P^{K_r}(H~) Vn of the members `ids`
// (after their refine_prepare), as batched Clenshaw launches: per 64-column
// chunk of the refined block, the members with that chunk, in sub-batches
// whose recurrence buffers stay within 4 GiB.  The kernel time is shared
// among the members in proportion to their rows times steps.
template <class T>
static void refine_batched(polfed_ctx *ctx, std::vector<std::unique_ptr<Realization<T>>> &rs,
                           const std::vector<int> &ids) {
  hipStream_t st = ctx->stream;
  std::map<std::pair<int, int>, std::vector<int>> chunks;  // (first column, width) -> members
  for (int i : ids)
    for (int c0 = 0; c0 < rs[i]->qpad; c0 += 64)
      chunks[std::make_pair(c0, std::min(64, rs[i]->qpad - c0))].push_back(i);
  hipEvent_t e0, e1;
  PF_HIP(hipEventCreate(&e0));
  PF_HIP(hipEventCreate(&e1));
  try {
    for (auto &ch : chunks) {
      const int c0 = ch.first.first, w = ch.first.second;
      const std::vector<int> &all = ch.second;
      size_t k0 = 0;
      while (k0 < all.size()) {
        size_t k1 = k0, tot = 0;
        while (k1 < all.size()) {
          const size_t need = sizeof(double) * 3 * (size_t)rs[all[k1]]->n * w;
          if (k1 > k0 && tot + need > ((size_t)4 << 30)) break;
          tot += need;
          ++k1;
        }
        const int B = (int)(k1 - k0);
        double *cheb = static_cast<double *>(ctx->buf("ref_cheb").ensure(tot));
        size_t ncoef = 0;
        int Lmax = 0;
        long long Kmax = 0;
        for (size_t k = k0; k < k1; ++k) {
          const Realization<T> &r = *rs[all[k]];
          ncoef += r.coef_r.size();
          Lmax = std::max(Lmax, r.c.L);
          Kmax = std::max(Kmax, r.K_r);
        }
        double *coefs = static_cast<double *>(ctx->buf("ref_coef").ensure(sizeof(double) * ncoef));
        std::vector<BatchItem<double>> items(B);
        std::vector<const Chain *> chains(B);
        size_t co = 0, bo = 0;
        const Realization<T> *rmax_L = rs[all[k0]].get();
        for (int k = 0; k < B; ++k) {
          Realization<T> &r = *rs[all[k0 + k]];
          if (r.c.L == Lmax) rmax_L = &r;
          PF_HIP(hipMemcpyAsync(coefs + co, r.coef_r.data(), sizeof(double) * r.coef_r.size(),
                                hipMemcpyHostToDevice, st));
          BatchItem<double> &it = items[k];
          std::memset(&it, 0, sizeof(it));
          it.dt = r.dt64b.template as<double>();
          it.X = r.Vnb.template as<double>() + c0;
          it.ldx = r.ldr;
          it.buf = cheb + bo;
          it.Y = r.URb.template as<double>() + c0;
          it.ldy = r.ldr;
          it.coef = coefs + co;
          it.Dinv = 1.0 / r.D_r;
          it.w1 = r.a * r.c.J1;
          it.w2 = r.a * r.c.J2;
          it.K = r.K_r;
          it.active = 1;
          chains[k] = &r.c;
          co += r.coef_r.size();
          bo += (size_t)3 * r.n * w;
        }
        const StepShape shape = batch_shape_for(ctx, Lmax, w, false);
        const long long total = fill_batch_chains(items, chains, batched_tile_rows<double>(w, shape));
        const BatchTables bt = batch_tables(items, chains);
        BatchItem<double> *itemsd = static_cast<BatchItem<double> *>(
            ctx->buf("ref_items").ensure(sizeof(BatchItem<double>) * B));
        PF_HIP(hipMemcpyAsync(itemsd, items.data(), sizeof(BatchItem<double>) * B,
                              hipMemcpyHostToDevice, st));
        StepArgs<double> base = base_args<double>(rmax_L->c, rmax_L->dt64b.template as<double>());
        PF_HIP(hipEventRecord(e0, st));
        for (long long j = 0; j <= Kmax; ++j)
          launch_step_batched<double>(st, w, base, itemsd, B, j, Kmax, total, bt, shape,
                                      ctx->num_cu);
        PF_HIP(hipEventRecord(e1, st));
        PF_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        PF_HIP(hipEventElapsedTime(&ms, e0, e1));
        double wsum = 0.0;
        for (int k = 0; k < B; ++k) wsum += (double)items[k].n * (items[k].K + 1);
        if (std::getenv("POLFED_VERBOSE"))
          fprintf(stderr, "[polfed] batched refinement filter: %d members, width %d, K_max %lld: "
                          "%.2f s\n", B, w, Kmax, 1e-3 * ms);
        for (int k = 0; k < B; ++k) {
          Realization<T> &r = *rs[all[k0 + k]];
          const double f = (double)items[k].n * (items[k].K + 1) / wsum;
          r.filter_gpu_s += 1e-3 * ms * f;
          r.filter_launches += (double)(Kmax + 1) * f;
          r.refine_bytes += batched_filter_bytes<double>(r.n, w, r.K_r, r.coef_r);
        }
        k0 = k1;
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  PF_HIP(hipEventDestroy(e0));
  PF_HIP(hipEventDestroy(e1));
}

template <class T>
static int solve_batch_impl(polfed_ctx *ctx, int R, const polfed_model *models,
                            const polfed_opts &o, int nev, double *evals, double *evecs,
                            double *resid, polfed_info *infos, int *status) {
  hipStream_t st = ctx->stream;
  // evecs offsets of every realisation
  std::vector<size_t> voff(R + 1, 0);
  for (int r = 0; r < R; ++r) {
    const long long d = polfed_dim(models[r].L);
    PF_REQUIRE(d > 0, "invalid L in batch");
    voff[r + 1] = voff[r] + (size_t)d * nev;
  }
  // every argument is checked before any work, so that an error leaves the
  // outputs untouched
  for (int r = 0; r < R; ++r) {
    validate_model(&models[r]);
    PF_REQUIRE(nev >= 1 && nev <= polfed_dim(models[r].L), "nev must be in [1, dim] for every model");
  }
  // group by (block size, J2 != 0): a group's realisations share every
  // batched launch whatever their L (each brings its own basis); the bond
  // set of the launch (with or without J2) is common to the group
  std::map<std::pair<int, int>, std::vector<int>> groups;
  for (int r = 0; r < R; ++r) {
    const int s = o.block_size ? o.block_size : block_for(ctx, models[r].L, nev, o.precision);
    groups[std::make_pair(s, models[r].J2 != 0.0 ? 1 : 0)].push_back(r);
  }
  int worst = POLFED_OK;
  // errors that belong to one realisation end that member only; the others
  // complete (errors of the device or its memory end the call)
  auto member_error = [](const Error &e) {
    return e.code == POLFED_EBOUNDS || e.code == POLFED_EBREAKDOWN || e.code == POLFED_EINVAL;
  };
  for (auto &g : groups) {
    const std::vector<int> &mem = g.second;
    const int B = (int)mem.size();
    const double tg0 = now_s();
    std::vector<std::unique_ptr<Realization<T>>> rs(B);
    polfed_opts og = o;
    og.block_size = g.first.first;
    long long Kmax = 0;
    int first_ok = -1;
    for (int i = 0; i < B; ++i) {
      rs[i].reset(new Realization<T>());
      try {
        rs[i]->setup(ctx, &models[mem[i]], og, nev);
      } catch (const Error &e) {
        if (!member_error(e)) throw;
        rs[i]->err = e.code;
        rs[i]->done = true;
        continue;
      }
      Kmax = std::max(Kmax, rs[i]->K);
      if (first_ok < 0) first_ok = i;
    }
    if (first_ok < 0) {  // every member of the group failed in its setup
      for (int i = 0; i < B; ++i) status[mem[i]] = rs[i]->err;
      if (worst == POLFED_OK) worst = POLFED_NOT_CONVERGED;
      continue;
    }
    // the longest chain of the group names the launch shape
    int rL = first_ok;
    for (int i = 0; i < B; ++i)
      if (!rs[i]->err && rs[i]->c.L > rs[rL]->c.L) rL = i;
    const Realization<T> &r0 = *rs[rL];
    const int S = r0.s;
    // per-member recurrence buffers, coefficients and descriptors
    size_t nbuf = 0, ncoef = 0;
    for (auto &r : rs) {
      nbuf += (size_t)3 * r->n * S;
      ncoef += r->coef.size();
    }
    DevBuf cheb, coefs, itemsd;
    cheb.ensure(sizeof(T) * nbuf);
    coefs.ensure(sizeof(double) * ncoef);
    std::vector<BatchItem<T>> items(B);
    std::vector<const Chain *> chains(B);
    size_t co = 0, bo = 0;
    for (int i = 0; i < B; ++i) {
      Realization<T> &r = *rs[i];
      PF_HIP(hipMemcpyAsync(coefs.as<double>() + co, r.coef.data(), sizeof(double) * r.coef.size(),
                            hipMemcpyHostToDevice, st));
      BatchItem<T> &it = items[i];
      std::memset(&it, 0, sizeof(it));
      it.dt = r.dt();
      it.X = r.Xs();
      it.ldx = S;
      it.buf = cheb.as<T>() + bo;
      it.Y = r.Ys();
      it.ldy = S;
      it.coef = coefs.as<double>() + co;
      it.Dinv = 1.0 / r.D;
      it.w1 = (T)(r.a * r.c.J1);
      it.w2 = (T)(r.a * r.c.J2);
      it.K = r.K;
      it.active = r.err ? 0 : 1;
      chains[i] = r.err ? &r0.c : &r.c;
      if (r.err) it.K = 0;
      co += r.coef.size();
      bo += (size_t)3 * r.n * S;
    }
    const StepShape shape = batch_shape_for(ctx, r0.c.L, S, r0.fp32);
    const long long total = fill_batch_chains(items, chains, batched_tile_rows<T>(S, shape));
    const BatchTables bt = batch_tables(items, chains);
    itemsd.ensure(sizeof(BatchItem<T>) * B);
    StepArgs<T> base = base_args<T>(r0.c, r0.dt());
    hipGraphExec_t graph = nullptr;
    hipEvent_t e0, e1;
    PF_HIP(hipEventCreate(&e0));
    PF_HIP(hipEventCreate(&e1));
    double gfilter = 0.0, glaunch = 0.0;
    try {
      for (;;) {
        int nact = 0;
        for (int i = 0; i < B; ++i) {
          items[i].active = rs[i]->done ? 0 : 1;
          if (!rs[i]->done) {
            rs[i]->filter_X();
            ++nact;
          }
        }
        if (nact == 0) break;
        PF_HIP(hipMemcpyAsync(itemsd.p, items.data(), sizeof(BatchItem<T>) * B,
                              hipMemcpyHostToDevice, st));
        if (!graph && ctx->use_graphs && Kmax <= (1LL << 17)) {
          hipGraph_t gr = nullptr;
          PF_HIP(hipStreamBeginCapture(ctx->own_stream, hipStreamCaptureModeThreadLocal));
          try {
            for (long long j = 0; j <= Kmax; ++j)
              launch_step_batched<T>(ctx->own_stream, S, base, itemsd.as<BatchItem<T>>(), B, j, Kmax,
                                     total, bt, shape, ctx->num_cu);
          } catch (...) {
            hipGraph_t dummy = nullptr;
            (void)hipStreamEndCapture(ctx->own_stream, &dummy);
            if (dummy) (void)hipGraphDestroy(dummy);
            throw;
          }
          PF_HIP(hipStreamEndCapture(ctx->own_stream, &gr));
          hipError_t e = hipGraphInstantiate(&graph, gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          PF_HIP(e);
        }
        const double tf0 = now_s();
        PF_HIP(hipEventRecord(e0, st));
        if (graph) {
          PF_HIP(hipGraphLaunch(graph, st));
        } else {
          for (long long j = 0; j <= Kmax; ++j)
            launch_step_batched<T>(st, S, base, itemsd.as<BatchItem<T>>(), B, j, Kmax, total,
                                   bt, shape, ctx->num_cu);
        }
        PF_HIP(hipEventRecord(e1, st));
        PF_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        PF_HIP(hipEventElapsedTime(&ms, e0, e1));
        gfilter += 1e-3 * ms;
        glaunch += (double)(Kmax + 1);
        // algorithmic bytes of the active members (same model as one filter)
        for (int i = 0; i < B; ++i)
          if (items[i].active) rs[i]->bytes += batched_filter_bytes<T>(rs[i]->n, S, rs[i]->K, rs[i]->coef);
        const double tf = now_s() - tf0;
        for (int i = 0; i < B; ++i)
          if (items[i].active) rs[i]->t_filter += tf / nact;
        // every active member's block, then their convergence checks: the
        // members due at one T_m size run their eigenproblems in one batched
        // launch when small enough
        std::vector<int> due;
        for (int i = 0; i < B; ++i) {
          if (!items[i].active) continue;
          try {
            if (rs[i]->lanczos_block()) due.push_back(i);
          } catch (const Error &e) {
            if (!member_error(e)) throw;
            rs[i]->err = e.code;
            rs[i]->done = true;
          }
        }
        std::map<int, std::vector<int>> by_size;
        for (int i : due) by_size[rs[i]->check_size()].push_back(i);
        for (auto &bs : by_size) {
          const int msz = bs.first;
          const std::vector<int> &dz = bs.second;
          bool batched = false;
          if (dz.size() > 1 && msz <= 128) {
            const double te0 = now_s();
            const size_t mm = (size_t)msz * msz, nd = dz.size();
            double *Aall = static_cast<double *>(ctx->buf("bat_eig").ensure(
                sizeof(double) * (3 * mm + msz) * nd));
            double *V0all = Aall + mm * nd, *Vall = V0all + mm * nd, *wall = Vall + mm * nd;
            for (size_t k = 0; k < nd; ++k) rs[dz[k]]->check_prepare(Aall + k * mm, V0all + k * mm);
            batched = sym_eig_batched(st, msz, (int)nd, Aall, V0all, wall, Vall);
            if (batched) {
              PF_HIP(hipStreamSynchronize(st));
              const double share = (now_s() - te0) / nd;
              for (size_t k = 0; k < nd; ++k) {
                rs[dz[k]]->t_eig += share;
                rs[dz[k]]->check_finish(wall + k * msz, Vall + k * mm);
              }
            }
          }
          if (!batched)
            for (int i : dz) rs[i]->check_single();
        }
      }
    } catch (...) {
      if (graph) (void)hipGraphExecDestroy(graph);
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    if (graph) PF_HIP(hipGraphExecDestroy(graph));
    PF_HIP(hipEventDestroy(e0));
    PF_HIP(hipEventDestroy(e1));
    cheb.release();
    const double tg1 = now_s();
    // Rayleigh-Ritz of every member, then the FP64 refinement passes of
    // those that want them, each pass's filters batched
    std::vector<int> ref;
    for (int i = 0; i < B; ++i) {
      if (rs[i]->err) continue;
      rs[i]->filter_gpu_s = gfilter / B;
      rs[i]->filter_launches = glaunch / B;
      if (rs[i]->fin_begin()) ref.push_back(i);
    }
    const double tb1 = now_s();
    double t_prep = 0.0, t_rfilt = 0.0, t_fin = 0.0;
    while (!ref.empty()) {
      const double ta = now_s();
      for (int i : ref) rs[i]->refine_prepare();
      const double tb = now_s();
      refine_batched<T>(ctx, rs, ref);
      const double tc = now_s();
      std::vector<int> more;
      for (int i : ref)
        if (rs[i]->refine_finish()) more.push_back(i);
      ref.swap(more);
      t_prep += tb - ta;
      t_rfilt += tc - tb;
      t_fin += now_s() - tc;
    }
    ctx->buf("ref_cheb").release();  // up to 4 GiB of refinement recurrence buffers
    if (std::getenv("POLFED_VERBOSE"))
      fprintf(stderr, "[polfed] batch finalize: Rayleigh-Ritz %.2f s, refinement prepare %.2f s, "
                      "filters %.2f s, orthonormalisation and Rayleigh-Ritz %.2f s\n",
              tb1 - tg1, t_prep, t_rfilt, t_fin);
    // members whose window was too narrow, and members whose FP32 result
    // misses the bar, each with its first attempt
    std::vector<int> widen, redo;
    std::vector<polfed_info> first_w, first;
    const bool can_widen = 2.0 * og.window_factor <= kMaxWindowFactor;
    for (int i = 0; i < B; ++i) {
      const int r = mem[i];
      if (rs[i]->err) {  // outputs of a failed member stay untouched
        status[r] = rs[i]->err;
        if (worst == POLFED_OK) worst = POLFED_NOT_CONVERGED;
        continue;
      }
      polfed_info ir;
      int rc = rs[i]->fin_end(evals + (size_t)r * nev, evecs ? evecs + voff[r] : nullptr,
                              resid + (size_t)r * nev, &ir);
      if (rs[i]->window_short()) {
        if (can_widen) {
          widen.push_back(r);
          first_w.push_back(ir);
          continue;
        }
        if (rc == POLFED_OK) rc = POLFED_NOT_CONVERGED;
      } else if (rs[i]->fp32 && ir.max_resid > kFp32ResidBar * ir.normH) {
        redo.push_back(r);
        first.push_back(ir);
        continue;
      }
      if (infos) infos[r] = ir;
      status[r] = rc;
      if (rc > 0 && worst == POLFED_OK) worst = rc;
    }
    std::set<int> Ls;
    for (auto &r : rs)
      if (!r->err) Ls.insert(r->c.L);
    rs.clear();  // the group's device state is no longer needed
    // a sub-batch of the members `ids` with options `os` (in FP64 when
    // fp64); results go to their places, each info merged with the member's
    // first attempt by `merge`
    auto rerun = [&](const std::vector<int> &ids, const std::vector<polfed_info> &firsts,
                     const polfed_opts &os, bool fp64, void (*merge)(polfed_info &, const polfed_info &)) {
      const int nr = (int)ids.size();
      std::vector<polfed_model> sub(nr);
      size_t tot = 0;
      for (int k = 0; k < nr; ++k) {
        sub[k] = models[ids[k]];
        tot += (size_t)polfed_dim(sub[k].L) * nev;
      }
      std::vector<double> ev((size_t)nr * nev), rsd((size_t)nr * nev);
      std::vector<double> vv(evecs ? tot : 0);
      std::vector<polfed_info> inf(nr);
      std::vector<int> stt(nr);
      if (fp64)
        solve_batch_impl<double>(ctx, nr, sub.data(), os, nev, ev.data(),
                                 evecs ? vv.data() : nullptr, rsd.data(), inf.data(), stt.data());
      else
        solve_batch_impl<T>(ctx, nr, sub.data(), os, nev, ev.data(), evecs ? vv.data() : nullptr,
                            rsd.data(), inf.data(), stt.data());
      size_t off = 0;
      for (int k = 0; k < nr; ++k) {
        const int r = ids[k];
        const size_t len = (size_t)polfed_dim(sub[k].L) * nev;
        std::memcpy(evals + (size_t)r * nev, ev.data() + (size_t)k * nev, sizeof(double) * nev);
        std::memcpy(resid + (size_t)r * nev, rsd.data() + (size_t)k * nev, sizeof(double) * nev);
        if (evecs) std::memcpy(evecs + voff[r], vv.data() + off, sizeof(double) * len);
        off += len;
        polfed_info ir = inf[k];
        merge(ir, firsts[k]);
        if (infos) infos[r] = ir;
        status[r] = stt[k];
        if (stt[k] > 0 && worst == POLFED_OK) worst = stt[k];
      }
    };

    if (!widen.empty()) {
      // too narrow a window: the same solve with the window sized for twice
      // as many eigenvalues, as one batch of its own (same block size)
      polfed_opts ow = og;
      ow.window_factor *= 2.0;
      rerun(widen, first_w, ow, false, add_attempt);
    }
    if (!redo.empty()) {
      // the FP64 re-solves of this group as one batch of their own (same
      // block size), each result as a single FP64 re-solve would report it
      polfed_opts o64 = og;
      o64.precision = 0;
      rerun(redo, first, o64, true, merge_resolve_info);
    }

    if (std::getenv("POLFED_VERBOSE")) {
      std::string ls;
      for (int L : Ls) ls += (ls.empty() ? "" : ",") + std::to_string(L);
      fprintf(stderr,
              "[polfed] batch group L=%s s=%d: %d members, Lanczos %.2f s (filter kernels "
              "%.2f s), finalize %.2f s\n",
              ls.c_str(), g.first.first, B, tg1 - tg0, gfilter, now_s() - tg1);
    }
  }
  return worst;
}

int solve_batch(polfed_ctx *ctx, int R, const polfed_model *models, const polfed_opts *opts_in,
                int nev, double *evals, double *evecs, double *resid, polfed_info *infos,
                int *status) {
  polfed_opts o = resolve_opts(opts_in);
  PF_REQUIRE(R >= 1 && models && status && evals && resid, "invalid batch arguments");
  // the batched kernel is Clenshaw's; the members' single-chain filters (the
  // refinement) follow it, whatever the context's setting
  struct FormGuard {
    polfed_ctx *c;
    int saved;
    ~FormGuard() { c->filter_form = saved; }
  } guard{ctx, ctx->filter_form};
  ctx->filter_form = POLFED_FORM_CLENSHAW;
  auto run = [&](int n, const polfed_model *ms, const polfed_opts &oo, double *ev, double *vv,
                 double *rs, polfed_info *inf, int *st) {
    return oo.precision == 1 ? solve_batch_impl<float>(ctx, n, ms, oo, nev, ev, vv, rs, inf, st)
                             : solve_batch_impl<double>(ctx, n, ms, oo, nev, ev, vv, rs, inf, st);
  };
  int worst = run(R, models, o, evals, evecs, resid, infos, status);
  // members whose filter left [-1, 1] (POLFED_EBOUNDS): again as a batch of
  // their own with the bounds margin eta doubled, three times at most
  for (int attempt = 0; attempt < kBoundsRetries; ++attempt) {
    std::vector<int> ids;
    for (int r = 0; r < R; ++r)
      if (status[r] == POLFED_EBOUNDS) ids.push_back(r);
    if (ids.empty()) break;
    o.eta *= 2.0;
    std::vector<size_t> voff(R + 1, 0);
    for (int r = 0; r < R; ++r) voff[r + 1] = voff[r] + (size_t)polfed_dim(models[r].L) * nev;
    const int nr = (int)ids.size();
    std::vector<polfed_model> sub(nr);
    size_t tot = 0;
    for (int k = 0; k < nr; ++k) {
      sub[k] = models[ids[k]];
      tot += (size_t)polfed_dim(sub[k].L) * nev;
    }
    std::vector<double> ev((size_t)nr * nev), rs((size_t)nr * nev), vv(evecs ? tot : 0);
    std::vector<polfed_info> inf(nr);
    std::vector<int> st(nr);
    run(nr, sub.data(), o, ev.data(), evecs ? vv.data() : nullptr, rs.data(), inf.data(),
        st.data());
    size_t off = 0;
    for (int k = 0; k < nr; ++k) {
      const int r = ids[k];
      const size_t len = (size_t)polfed_dim(sub[k].L) * nev;
      status[r] = st[k];
      if (st[k] >= 0) {  // outputs of a member that failed again stay untouched
        std::memcpy(evals + (size_t)r * nev, ev.data() + (size_t)k * nev, sizeof(double) * nev);
        std::memcpy(resid + (size_t)r * nev, rs.data() + (size_t)k * nev, sizeof(double) * nev);
        if (evecs) std::memcpy(evecs + voff[r], vv.data() + off, sizeof(double) * len);
        if (infos) infos[r] = inf[k];
      }
      off += len;
    }
    worst = POLFED_OK;
    for (int r = 0; r < R; ++r)
      if (status[r] != POLFED_OK) worst = POLFED_NOT_CONVERGED;
  }
  return worst;
}

// ------------------------------------------------- stage-call helpers --

template <class T>
void stage_apply_h(polfed_ctx *ctx, const Chain &c, int nvec, const T *X, T *Y) {
  const long long n = c.basis->n;
  T *dt = static_cast<T *>(ctx->buf("stage_dt").ensure(sizeof(T) * n));
  launch_scaled_diag<T>(ctx->stream, n, c.diag.as<double>(), 1.0, 0.0, dt);
  apply_op<T>(ctx, c, dt, 0.5 * c.J1, 0.5 * c.J2, X, nvec, Y, nvec, nvec, sizeof(T) == 4);
}

template <class T>
void stage_apply_filter(polfed_ctx *ctx, const Chain &c, double E0, double E1, double sigma,
                        long long K, int nvec, const T *X, T *Y) {
  const long long n = c.basis->n;
  const double a = 2.0 / (E1 - E0), b = -(E0 + E1) / (E1 - E0);
  T *dt = static_cast<T *>(ctx->buf("stage_dt").ensure(sizeof(T) * n));
  launch_scaled_diag<T>(ctx->stream, n, c.diag.as<double>(), a, b, dt);
  T *bufs = static_cast<T *>(ctx->buf("stage_cheb").ensure(sizeof(T) * 3 * (size_t)n * nvec));
  std::vector<double> coef;
  double D;
  cheb_coeffs(sigma, K, coef, D, ctx->filter_damping);
  run_filter<T>(ctx, c, dt, a, nvec, X, nvec, Y, nvec, K, coef, D, bufs, sizeof(T) == 4, nullptr);
}

template void stage_apply_h<float>(polfed_ctx *, const Chain &, int, const float *, float *);
template void stage_apply_h<double>(polfed_ctx *, const Chain &, int, const double *, double *);
template void stage_apply_filter<float>(polfed_ctx *, const Chain &, double, double, double,
                                        long long, int, const float *, float *);
template void stage_apply_filter<double>(polfed_ctx *, const Chain &, double, double, double,
                                         long long, int, const double *, double *);

// ----------------------------------------------------------- tuning --

StepShape default_shape(int L, int S, bool fp32) {
  // From sweeps of (threads, loads per lane, groups per CU, LDS tables,
  // early streamed loads, column slices) on gfx950 boxes: eight 256-thread
  // groups per CU with the rank tables in LDS lead up to L = 20; short rows
  // (L <= 16, and FP32 at L = 18) want one 16-byte load per lane, the rest
  // two; FP32 at L = 22 prefers two 1024-thread groups per CU.  At L >= 22
  // splitting the block's columns over the XCDs pays in FP64 (L = 22: two
  // slices, 231 against 244 us a step at s = 32; L = 26: four slices, 9.4
  // against 10.4 ms at s = 64) and at L = 26 in FP32 (two slices, 4.46
  // against 4.63 ms at s = 64).  Short chains (L <= 16) sit near the launch
  // floor (~5-6 us a step).
  StepShape sh;
  sh.lds_tables = 1;
  sh.lpl = 2;
  sh.threads = 256;
  sh.wg_per_cu = 8;
  if (L <= 16 || (L == 18 && fp32)) {
    sh.lpl = 1;
  } else if (L >= 24 && fp32) {
    sh.threads = 512;
    sh.wg_per_cu = 2;
    sh.xcd_slices = 2;
  } else if (L >= 24) {
    sh.wg_per_cu = 2;
    sh.xcd_slices = 4;
  } else if (L >= 22 && fp32) {
    sh.threads = 1024;
    sh.wg_per_cu = 2;
  } else if (L >= 22) {
    sh.threads = 512;
    sh.wg_per_cu = 4;
    sh.early_loads = 1;
    sh.xcd_slices = 2;
  }
  (void)S;
  return sh;
}

StepShape default_batch_shape(int L, int S, bool fp32) {
  // The single-chain default with the tables as rank method and no column
  // slices.  (Four slices for the FP64 refinement filters of the 512-
  // realisation batch, which would keep one L = 18 realisation's gathered
  // slice in an XCD's L2, measured slower at 32 columns (64-byte slices of
  // 128-byte lines: 7.9 against 6.4 s for one pass) and even at 64.)
  StepShape sh = default_shape(L, S, fp32);
  sh.rank_incr = 0;
  sh.xcd_slices = 1;
  return sh;
}

int choose_block(int L, int nev, int precision) {
  int s = next_pow2_le(std::max(1, nev / 4));
  s = std::min(s, precision ? 32 : 16);
  if (L <= 14) s = std::min(s, 8);
  return std::max(1, s);
}

}  // namespace polfed
