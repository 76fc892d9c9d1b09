// C-ABI entry points of libpolfed (declared in include/polfed.h).
//
// Every entry point converts internal exceptions into a status code and
// records the message on the context; nothing throws across the ABI.
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "internal.h"

namespace polfed {

void make_chain(polfed_ctx *ctx, const polfed_model *m, Chain &c);
int solve_one(polfed_ctx *ctx, const polfed_model *model, const polfed_opts *opts, int nev,
              double *evals, double *evecs, double *resid, polfed_info *info);
int solve_batch(polfed_ctx *ctx, int R, const polfed_model *models, const polfed_opts *opts,
                int nev, double *evals, double *evecs, double *resid, polfed_info *infos,
                int *status);
void run_bounds(polfed_ctx *ctx, const Chain &c, int steps, unsigned long long seed, double &E0,
                double &E1, double &r0, double &r1);
template <class T>
void stage_apply_h(polfed_ctx *ctx, const Chain &c, int nvec, const T *X, T *Y);
template <class T>
void stage_apply_filter(polfed_ctx *ctx, const Chain &c, double E0, double E1, double sigma,
                        long long K, int nvec, const T *X, T *Y);

void check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    throw Error(POLFED_EDEVICE, std::string("launch of ") + what + ": " + hipGetErrorString(e));
}

DevBuf::~DevBuf() {
  if (p) (void)hipFree(p);
}

void DevBuf::release() {
  if (!p) return;
  PF_HIP(hipDeviceSynchronize());
  PF_HIP(hipFree(p));
  p = nullptr;
  bytes = 0;
}

void *DevBuf::ensure(size_t nbytes) {
  if (nbytes == 0) nbytes = 1;
  if (nbytes <= bytes) return p;
  if (p) {
    // queued kernels may still use the old block
    PF_HIP(hipDeviceSynchronize());
    PF_HIP(hipFree(p));
    p = nullptr;
    bytes = 0;
  }
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw Error(POLFED_ENOMEM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed");
  }
  bytes = nbytes;
  return p;
}

static bool pow2_block(int s) { return s >= 1 && s <= 64 && (s & (s - 1)) == 0; }

template <class F>
static int guarded(polfed_ctx *ctx, F &&f) {
  if (!ctx) return POLFED_EINVAL;
  try {
    PF_HIP(hipSetDevice(ctx->device));
    ctx->last_error.clear();
    return f();
  } catch (const Error &e) {
    ctx->last_error = e.what();
    return e.code;
  } catch (const std::exception &e) {
    ctx->last_error = e.what();
    return POLFED_EDEVICE;
  }
}

}  // namespace polfed

using namespace polfed;

const Pattern &polfed_ctx::pattern(int L, bool has_j2) {
  auto &p = patterns[{L, has_j2 ? 1 : 0}];
  if (!p) {
    p.reset(new Pattern());
    build_pattern(stream, basis(L), has_j2, *p);
  }
  return *p;
}

const Basis &polfed_ctx::basis(int L) {
  auto &p = bases[L];
  if (!p) {
    p.reset(new Basis());
    build_basis(stream, *p, L);
  }
  return *p;
}

extern "C" {

long long polfed_dim(int L) {
  if (L < 2 || L > 30 || (L & 1)) return -1;
  long long r = 1;
  for (int k = 1; k <= L / 2; ++k) r = r * (L / 2 + k) / k;
  return r;
}

void polfed_default_opts(polfed_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->target_kind = 0;
  o->target = 0.5;
  o->block_size = 0;
  o->K = 0;
  o->p = 0.17;
  o->precision = 0;
  o->window_factor = 1.5;
  o->max_cols = 0;
  o->tol = 1e-10;
  o->eta = 1e-3;
  o->bounds_steps = 200;
  o->seed = 12345;
  o->max_order = 0;
  o->dos = POLFED_DOS_GAUSS;
  o->dos_moments = 256;
  o->dos_vectors = 4;
  o->damping = POLFED_DAMP_NONE;
}

// Message of the last failed polfed_create on this host thread (there is no
// context to hold it).
static thread_local std::string t_create_error;

int polfed_create(int device, polfed_ctx **out) {
  t_create_error.clear();
  if (!out) {
    t_create_error = "polfed_create: out is NULL";
    return POLFED_EINVAL;
  }
  *out = nullptr;
  polfed_ctx *ctx = new polfed_ctx();
  ctx->device = device;
  try {
    int ndev = 0;
    PF_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) {
      delete ctx;
      t_create_error = "polfed_create: device " + std::to_string(device) + " out of range (" +
                       std::to_string(ndev) + " visible)";
      return POLFED_EINVAL;
    }
    PF_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    PF_HIP(hipGetDeviceProperties(&prop, device));
    ctx->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    PF_HIP(hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking));
    ctx->stream = ctx->own_stream;
    ctx->use_graphs = std::getenv("POLFED_NO_GRAPH") ? 0 : 1;
    upload_binomials(device);
    init_gram_scratch(device);
  } catch (const Error &e) {
    delete ctx;
    t_create_error = e.what();
    return e.code;
  }
  *out = ctx;
  return POLFED_OK;
}

int polfed_destroy(polfed_ctx *ctx) {
  if (!ctx) return POLFED_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->patterns.clear();
  ctx->bases.clear();
  ctx->bufs.clear();
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
  if (ctx->filter_graph) (void)hipGraphExecDestroy(ctx->filter_graph);
  if (ctx->ev_start) (void)hipEventDestroy(ctx->ev_start);
  if (ctx->ev_stop) (void)hipEventDestroy(ctx->ev_stop);
  delete ctx;
  return POLFED_OK;
}

const char *polfed_last_error(const polfed_ctx *ctx) {
  return ctx ? ctx->last_error.c_str() : t_create_error.c_str();
}

int polfed_set_stream(polfed_ctx *ctx, void *stream) {
  return guarded(ctx, [&] {
    ctx->stream = static_cast<hipStream_t>(stream);
    return POLFED_OK;
  });
}

int polfed_synchronize(polfed_ctx *ctx) {
  return guarded(ctx, [&] {
    PF_HIP(hipStreamSynchronize(ctx->stream));
    return POLFED_OK;
  });
}

int polfed_cheb_coeffs(double sigma, long long K, double *c, double *D) {
  if (!c || !D || K < 0 || !(std::fabs(sigma) < 1.0)) return POLFED_EINVAL;
  std::vector<double> v;
  double d;
  cheb_coeffs(sigma, K, v, d);
  std::memcpy(c, v.data(), sizeof(double) * (size_t)(K + 1));
  *D = d;
  return POLFED_OK;
}

int polfed_filter_coeffs(double sigma, long long K, int damping, double *c, double *D) {
  if (!c || !D || K < 0 || !(std::fabs(sigma) < 1.0) ||
      (damping != POLFED_DAMP_NONE && damping != POLFED_DAMP_JACKSON))
    return POLFED_EINVAL;
  std::vector<double> v;
  double d;
  cheb_coeffs(sigma, K, v, d, damping);
  std::memcpy(c, v.data(), sizeof(double) * (size_t)(K + 1));
  *D = d;
  return POLFED_OK;
}

int polfed_filter_order_damped(const polfed_model *m, double E0w, double E1w, double sigma,
                               int nwin, double p, int damping, long long max_order,
                               int *nwin_out, long long *K) {
  if (!m || !m->h || !K || !nwin_out || nwin < 1 || !(E1w > E0w) || !(std::fabs(sigma) < 1.0) ||
      !(p > 0.0) || (damping != POLFED_DAMP_NONE && damping != POLFED_DAMP_JACKSON))
    return POLFED_EINVAL;
  long long n = polfed_dim(m->L);
  if (n < 0) return POLFED_EINVAL;
  const double Gamma = dos_gamma(m->L, m->J1, m->J2, m->Delta, m->h);
  const double Ebar = trace_mean(m->L, m->J1, m->J2, m->Delta);
  const int nw = (int)std::min<long long>(nwin, n);
  *K = choose_order(n, Ebar, Gamma, E0w, E1w, sigma, nw, p, nullptr, damping);
  *nwin_out = nw;
  if (max_order > 0 && *K > max_order)
    *nwin_out = capped_window(n, Ebar, Gamma, E0w, E1w, sigma, nw, p, max_order, K, damping);
  return POLFED_OK;
}

int polfed_filter_order(const polfed_model *m, double E0w, double E1w, double sigma, int nwin,
                        double p, long long *K, double *rho) {
  if (!m || !m->h || !K || nwin < 1 || !(E1w > E0w) || !(std::fabs(sigma) < 1.0) || !(p > 0.0))
    return POLFED_EINVAL;
  long long n = polfed_dim(m->L);
  if (n < 0) return POLFED_EINVAL;
  const double Gamma = dos_gamma(m->L, m->J1, m->J2, m->Delta, m->h);
  const double Ebar = trace_mean(m->L, m->J1, m->J2, m->Delta);
  double r = 0.0;
  *K = choose_order(n, Ebar, Gamma, E0w, E1w, sigma, nwin, p, &r);
  if (rho) *rho = r;
  return POLFED_OK;
}

int polfed_window_order(const polfed_model *m, double E0w, double E1w, double sigma, int nwin,
                        double p, long long max_order, int *nwin_out, long long *K) {
  if (!m || !m->h || !K || !nwin_out || nwin < 1 || !(E1w > E0w) || !(std::fabs(sigma) < 1.0) ||
      !(p > 0.0))
    return POLFED_EINVAL;
  long long n = polfed_dim(m->L);
  if (n < 0) return POLFED_EINVAL;
  const double Gamma = dos_gamma(m->L, m->J1, m->J2, m->Delta, m->h);
  const double Ebar = trace_mean(m->L, m->J1, m->J2, m->Delta);
  *nwin_out = capped_window(n, Ebar, Gamma, E0w, E1w, sigma, (int)std::min<long long>(nwin, n), p,
                            max_order, K);
  return POLFED_OK;
}

int polfed_kpm_count(const double *mu, int nmom, long long N, double x_lo, double x_hi,
                     double *count) {
  if (!mu || !count || nmom < 1 || N < 0 || !(x_lo <= x_hi)) return POLFED_EINVAL;
  *count = kpm_count(std::vector<double>(mu, mu + nmom), N, x_lo, x_hi);
  return POLFED_OK;
}

int polfed_kpm_order(const double *mu, int nmom, long long N, double sigma, int nwin, double p,
                     int damping, long long max_order, int *nwin_out, long long *K) {
  if (!mu || !K || !nwin_out || nmom < 1 || N < 1 || nwin < 1 || !(std::fabs(sigma) < 1.0) ||
      !(p > 0.0) || (damping != POLFED_DAMP_NONE && damping != POLFED_DAMP_JACKSON))
    return POLFED_EINVAL;
  const std::vector<double> m(mu, mu + nmom);
  const int nw = (int)std::min<long long>(nwin, N);
  *K = choose_order_kpm(m, N, sigma, nw, p, damping);
  *nwin_out = nw;
  if (max_order > 0 && *K > max_order)
    *nwin_out = capped_window_kpm(m, N, sigma, nw, p, max_order, K, damping);
  return POLFED_OK;
}

int polfed_dos_moments(polfed_ctx *ctx, const polfed_model *m, double E0w, double E1w, int nmom,
                       int nvec, const double *R, unsigned long long seed, double *mu) {
  return guarded(ctx, [&] {
    PF_REQUIRE(mu != nullptr, "mu is NULL");
    PF_REQUIRE(E1w > E0w, "E1w must exceed E0w");
    PF_REQUIRE(nmom >= 1 && nmom <= (1 << 20), "dos moments: nmom must be in [1, 2^20]");
    PF_REQUIRE(nvec >= 1, "dos moments: nvec must be >= 1");
    Chain c;
    make_chain(ctx, m, c);
    const double a = 2.0 / (E1w - E0w), b = -(E0w + E1w) / (E1w - E0w);
    std::vector<double> out;
    dos_moments(ctx, c, a, b, nmom, nvec, R, seed, out);
    std::copy(out.begin(), out.end(), mu);
    return POLFED_OK;
  });
}

int polfed_basis(polfed_ctx *ctx, int L, uint32_t *states) {
  return guarded(ctx, [&] {
    PF_REQUIRE(polfed_dim(L) > 0 && L >= 2, "L must be even in [2, 30]");
    PF_REQUIRE(states != nullptr, "states is NULL");
    const Basis &b = ctx->basis(L);
    PF_HIP(hipMemcpyAsync(states, b.states.p, sizeof(uint32_t) * b.n, hipMemcpyDeviceToDevice,
                          ctx->stream));
    return POLFED_OK;
  });
}

int polfed_rank(polfed_ctx *ctx, int L, long long n, const uint32_t *states, int32_t *ranks) {
  return guarded(ctx, [&] {
    PF_REQUIRE(polfed_dim(L) > 0 && L >= 2, "L must be even in [2, 30]");
    PF_REQUIRE(n >= 0, "n must be >= 0");
    PF_REQUIRE(n == 0 || (states && ranks), "states/ranks NULL");
    launch_rank(ctx->stream, ctx->basis(L), n, states, ranks);
    return POLFED_OK;
  });
}

int polfed_diag(polfed_ctx *ctx, const polfed_model *m, double *d) {
  return guarded(ctx, [&] {
    PF_REQUIRE(d != nullptr, "d is NULL");
    Chain c;
    make_chain(ctx, m, c);
    PF_HIP(hipMemcpyAsync(d, c.diag.p, sizeof(double) * c.basis->n, hipMemcpyDeviceToDevice,
                          ctx->stream));
    PF_HIP(hipStreamSynchronize(ctx->stream));  // c.diag is freed on return
    return POLFED_OK;
  });
}

int polfed_apply_h(polfed_ctx *ctx, const polfed_model *m, int precision, int nvec, const void *X,
                   void *Y) {
  return guarded(ctx, [&] {
    PF_REQUIRE(precision == 0 || precision == 1, "precision must be 0 or 1");
    PF_REQUIRE(pow2_block(nvec), "nvec must be a power of two in [1, 64]");
    PF_REQUIRE(X && Y && X != Y, "X, Y must be distinct non-NULL device pointers");
    Chain c;
    make_chain(ctx, m, c);
    if (precision == 0)
      stage_apply_h<double>(ctx, c, nvec, static_cast<const double *>(X), static_cast<double *>(Y));
    else
      stage_apply_h<float>(ctx, c, nvec, static_cast<const float *>(X), static_cast<float *>(Y));
    PF_HIP(hipStreamSynchronize(ctx->stream));
    return POLFED_OK;
  });
}

int polfed_apply_filter(polfed_ctx *ctx, const polfed_model *m, double E0, double E1,
                        double sigma, long long K, int precision, int nvec, const void *X,
                        void *Y) {
  return guarded(ctx, [&] {
    PF_REQUIRE(precision == 0 || precision == 1, "precision must be 0 or 1");
    PF_REQUIRE(pow2_block(nvec), "nvec must be a power of two in [1, 64]");
    PF_REQUIRE(X && Y && X != Y, "X, Y must be distinct non-NULL device pointers");
    PF_REQUIRE(E1 > E0, "E1 must exceed E0");
    PF_REQUIRE(std::fabs(sigma) < 1.0, "|sigma_tilde| must be < 1");
    PF_REQUIRE(K >= 0 && K <= (1LL << 26), "K must be in [0, 2^26]");
    Chain c;
    make_chain(ctx, m, c);
    if (precision == 0)
      stage_apply_filter<double>(ctx, c, E0, E1, sigma, K, nvec, static_cast<const double *>(X),
                                 static_cast<double *>(Y));
    else
      stage_apply_filter<float>(ctx, c, E0, E1, sigma, K, nvec, static_cast<const float *>(X),
                                static_cast<float *>(Y));
    PF_HIP(hipStreamSynchronize(ctx->stream));
    return POLFED_OK;
  });
}

int polfed_gram(polfed_ctx *ctx, long long n, int p, int q, const double *X, long long ldx,
                const double *Y, long long ldy, double *C, long long ldc) {
  return guarded(ctx, [&] {
    PF_REQUIRE(n >= 0 && p >= 1 && q >= 1, "need n >= 0, p, q >= 1");
    PF_REQUIRE(ldx >= p && ldy >= q && ldc >= q, "leading dimensions too small");
    PF_REQUIRE(X && Y && C, "NULL operand");
    if (n == 0) {
      for (int i = 0; i < p; ++i)
        PF_HIP(hipMemsetAsync(C + (size_t)i * ldc, 0, sizeof(double) * q, ctx->stream));
      return POLFED_OK;
    }
    launch_gram(ctx->stream, n, p, q, X, ldx, Y, ldy, C, ldc, ctx->buf("partials"), ctx->num_cu);
    return POLFED_OK;
  });
}

int polfed_gram_static(polfed_ctx *ctx, long long n, int p, int q, const double *X,
                       long long ldx, const double *Y, long long ldy, double *C, long long ldc) {
  return guarded(ctx, [&] {
    PF_REQUIRE(n >= 0 && p >= 1 && q >= 1, "need n >= 0, p, q >= 1");
    PF_REQUIRE(ldx >= p && ldy >= q && ldc >= q, "leading dimensions too small");
    PF_REQUIRE(C && (n == 0 || (X && Y)), "NULL operand");
    launch_gram_static(ctx->stream, ctx->device, n, p, q, X, ldx, Y, ldy, C, ldc, ctx->num_cu);
    return POLFED_OK;
  });
}

int polfed_update(polfed_ctx *ctx, long long n, int p, int q, double alpha, const double *X,
                  long long ldx, const double *C, long long ldc, double beta, double *Y,
                  long long ldy) {
  return guarded(ctx, [&] {
    PF_REQUIRE(n >= 0 && p >= 1 && q >= 1 && q <= 64, "need n >= 0, p >= 1, 1 <= q <= 64");
    PF_REQUIRE(ldx >= p && ldc >= q && ldy >= q, "leading dimensions too small");
    PF_REQUIRE(X && C && Y, "NULL operand");
    launch_update(ctx->stream, n, p, q, alpha, X, ldx, C, ldc, beta, Y, ldy);
    return POLFED_OK;
  });
}

int polfed_sym_eig(polfed_ctx *ctx, int n, double *A, double *w, double *V) {
  return guarded(ctx, [&] {
    PF_REQUIRE(n >= 1 && n <= 4096, "n must be in [1, 4096]");
    PF_REQUIRE(A && w && V, "NULL operand");
    sym_eig(ctx->stream, n, A, w, V, ctx->buf("eigwork"));
    PF_HIP(hipStreamSynchronize(ctx->stream));
    return POLFED_OK;
  });
}

int polfed_bounds(polfed_ctx *ctx, const polfed_model *m, int steps, unsigned long long seed,
                  double *E0, double *E1, double *r0, double *r1) {
  return guarded(ctx, [&] {
    PF_REQUIRE(steps >= 1, "steps must be >= 1");
    PF_REQUIRE(E0 && E1, "NULL output");
    Chain c;
    make_chain(ctx, m, c);
    double a, b, ra, rb;
    run_bounds(ctx, c, steps, seed, a, b, ra, rb);
    *E0 = a;
    *E1 = b;
    if (r0) *r0 = ra;
    if (r1) *r1 = rb;
    return POLFED_OK;
  });
}

int polfed_set_step_shape(polfed_ctx *ctx, int L, int nvec, int precision, int threads, int lpl,
                          int wg_per_cu, int lds_tables, int early_loads, int rank_incremental,
                          int xcd_slices) {
  return guarded(ctx, [&] {
    PF_REQUIRE(polfed_dim(L) > 0 && L >= 4, "L must be even in [4, 30]");
    PF_REQUIRE(pow2_block(nvec), "nvec must be a power of two in [1, 64]");
    PF_REQUIRE(precision == 0 || precision == 1, "precision must be 0 or 1");
    PF_REQUIRE(threads == 256 || threads == 512 || threads == 1024,
               "threads must be 256, 512 or 1024");
    PF_REQUIRE(lpl == 1 || lpl == 2 || lpl == 4, "lpl must be 1, 2 or 4");
    PF_REQUIRE(rank_incremental >= 0 && rank_incremental <= 2,
               "rank mode must be 0 (tables), 1 (incremental) or 2 (stored pattern)");
    PF_REQUIRE(wg_per_cu >= 1 && wg_per_cu <= 32, "wg_per_cu must be in [1, 32]");
    PF_REQUIRE(xcd_slices == 1 || xcd_slices == 2 || xcd_slices == 4 || xcd_slices == 8,
               "xcd_slices must be 1, 2, 4 or 8");
    StepShape sh;
    sh.threads = threads;
    sh.lpl = lpl;
    sh.wg_per_cu = wg_per_cu;
    sh.lds_tables = lds_tables ? 1 : 0;
    sh.early_loads = early_loads ? 1 : 0;
    sh.rank_incr = rank_incremental;
    sh.xcd_slices = xcd_slices;
    ctx->shapes[std::make_tuple(L, nvec, precision ? 4 : 8)] = sh;
    return POLFED_OK;
  });
}

int polfed_set_batch_shape(polfed_ctx *ctx, int L, int nvec, int precision, int threads, int lpl,
                           int wg_per_cu, int lds_tables, int early_loads, int xcd_slices) {
  return guarded(ctx, [&] {
    PF_REQUIRE(polfed_dim(L) > 0 && L >= 4, "L must be even in [4, 30]");
    PF_REQUIRE(pow2_block(nvec), "nvec must be a power of two in [1, 64]");
    PF_REQUIRE(precision == 0 || precision == 1, "precision must be 0 or 1");
    PF_REQUIRE(threads == 256 || threads == 512 || threads == 1024,
               "threads must be 256, 512 or 1024");
    PF_REQUIRE(lpl == 1 || lpl == 2 || lpl == 4, "lpl must be 1, 2 or 4");
    PF_REQUIRE(wg_per_cu >= 1 && wg_per_cu <= 32, "wg_per_cu must be in [1, 32]");
    PF_REQUIRE((xcd_slices == 1 || xcd_slices == 2 || xcd_slices == 4 || xcd_slices == 8) &&
                   xcd_slices <= nvec,
               "xcd_slices must be 1, 2, 4 or 8 and at most nvec");
    StepShape sh;
    sh.threads = threads;
    sh.lpl = lpl;
    sh.wg_per_cu = wg_per_cu;
    sh.lds_tables = lds_tables ? 1 : 0;
    sh.early_loads = early_loads ? 1 : 0;
    sh.rank_incr = 0;
    sh.xcd_slices = xcd_slices;
    ctx->batch_shapes[std::make_tuple(L, nvec, precision ? 4 : 8)] = sh;
    return POLFED_OK;
  });
}

int polfed_get_batch_shape(polfed_ctx *ctx, int L, int nvec, int precision, int *threads,
                           int *lpl, int *wg_per_cu, int *lds_tables, int *early_loads,
                           int *xcd_slices) {
  return guarded(ctx, [&] {
    PF_REQUIRE(polfed_dim(L) > 0 && L >= 4, "L must be even in [4, 30]");
    PF_REQUIRE(pow2_block(nvec), "nvec must be a power of two in [1, 64]");
    PF_REQUIRE(precision == 0 || precision == 1, "precision must be 0 or 1");
    PF_REQUIRE(threads && lpl && wg_per_cu && lds_tables && early_loads && xcd_slices,
               "NULL output");
    StepShape sh;
    auto it = ctx->batch_shapes.find(std::make_tuple(L, nvec, precision ? 4 : 8));
    if (it != ctx->batch_shapes.end()) {
      sh = it->second;
    } else {
      sh = default_batch_shape(L, nvec, precision == 1);
    }
    *xcd_slices = sh.xcd_slices;
    *threads = sh.threads;
    *lpl = sh.lpl;
    *wg_per_cu = sh.wg_per_cu;
    *lds_tables = sh.lds_tables;
    *early_loads = sh.early_loads;
    return POLFED_OK;
  });
}

int polfed_get_step_shape(polfed_ctx *ctx, int L, int nvec, int precision, int *threads, int *lpl,
                          int *wg_per_cu, int *lds_tables, int *early_loads,
                          int *rank_incremental, int *xcd_slices) {
  return guarded(ctx, [&] {
    PF_REQUIRE(polfed_dim(L) > 0 && L >= 4, "L must be even in [4, 30]");
    PF_REQUIRE(pow2_block(nvec), "nvec must be a power of two in [1, 64]");
    PF_REQUIRE(precision == 0 || precision == 1, "precision must be 0 or 1");
    PF_REQUIRE(threads && lpl && wg_per_cu && lds_tables && early_loads && rank_incremental &&
                   xcd_slices,
               "NULL output");
    auto it = ctx->shapes.find(std::make_tuple(L, nvec, precision ? 4 : 8));
    const StepShape sh = (it != ctx->shapes.end()) ? it->second : default_shape(L, nvec, precision != 0);
    *threads = sh.threads;
    *lpl = sh.lpl;
    *wg_per_cu = sh.wg_per_cu;
    *lds_tables = sh.lds_tables;
    *early_loads = sh.early_loads;
    *rank_incremental = sh.rank_incr;
    *xcd_slices = sh.xcd_slices;
    return POLFED_OK;
  });
}

int polfed_set_block_size(polfed_ctx *ctx, int L, int precision, int nev, int block_size) {
  return guarded(ctx, [&] {
    PF_REQUIRE(polfed_dim(L) > 0 && L >= 4, "L must be even in [4, 30]");
    PF_REQUIRE(precision == 0 || precision == 1, "precision must be 0 or 1");
    PF_REQUIRE(nev >= 1, "nev must be >= 1");
    PF_REQUIRE(pow2_block(block_size), "block_size must be a power of two in [1, 64]");
    ctx->blocks[std::make_tuple(L, precision, nev)] = block_size;
    return POLFED_OK;
  });
}

int polfed_set_graphs(polfed_ctx *ctx, int on) {
  return guarded(ctx, [&] {
    ctx->use_graphs = on ? 1 : 0;
    return POLFED_OK;
  });
}

int polfed_set_filter_form(polfed_ctx *ctx, int form) {
  return guarded(ctx, [&] {
    PF_REQUIRE(form == POLFED_FORM_CLENSHAW || form == POLFED_FORM_FORWARD,
               "form must be POLFED_FORM_CLENSHAW or POLFED_FORM_FORWARD");
    ctx->filter_form = form;
    return POLFED_OK;
  });
}

int polfed_set_filter_damping(polfed_ctx *ctx, int damping) {
  return guarded(ctx, [&] {
    PF_REQUIRE(damping == POLFED_DAMP_NONE || damping == POLFED_DAMP_JACKSON,
               "damping must be POLFED_DAMP_NONE or POLFED_DAMP_JACKSON");
    ctx->filter_damping = damping;
    return POLFED_OK;
  });
}

int polfed_filter_stats(polfed_ctx *ctx, double *gpu_s, double *launches, double *bytes,
                        int reset) {
  return guarded(ctx, [&] {
    if (gpu_s) *gpu_s = ctx->filter_gpu_s;
    if (launches) *launches = ctx->filter_launches;
    if (bytes) *bytes = ctx->filter_bytes;
    if (reset) {
      ctx->filter_gpu_s = 0.0;
      ctx->filter_launches = 0.0;
      ctx->filter_bytes = 0.0;
    }
    return POLFED_OK;
  });
}

int polfed_entanglement(polfed_ctx *ctx, int L, int nvec, const double *V, long long ldv,
                        int ncut, const int *cuts, double *S) {
  return guarded(ctx, [&] {
    PF_REQUIRE(polfed_dim(L) > 0 && L >= 2 && L <= 18, "L must be even in [2, 18]");
    PF_REQUIRE(nvec >= 1 && ldv >= nvec, "need nvec >= 1 and ldv >= nvec");
    PF_REQUIRE(ncut >= 1 && cuts && V && S, "NULL argument or no cuts");
    std::vector<int> cv(cuts, cuts + ncut);
    for (int x : cv) PF_REQUIRE(x >= 0 && x < L, "cut offsets must be in [0, L)");
    entanglement_entropy(ctx->stream, ctx->basis(L), nvec, V, ldv, cv, S, ctx->buf("ent"));
    return POLFED_OK;
  });
}

int polfed_gap_ratio(const double *E, int n, double *rbar) {
  if (!E || !rbar || n < 3) return POLFED_EINVAL;
  *rbar = mean_gap_ratio(E, n);
  return POLFED_OK;
}

double polfed_s_rmt(int L) {
  return 0.5 * L * std::log(2.0) + 0.5 * (0.5 + std::log(0.5)) - 0.5;
}

int polfed_stream_copy(polfed_ctx *ctx, const void *src, void *dst, long long bytes, int reps,
                       double *gbs) {
  return guarded(ctx, [&] {
    PF_REQUIRE(src && dst && gbs, "NULL argument");
    PF_REQUIRE(bytes >= 16 && bytes % 16 == 0, "bytes must be a positive multiple of 16");
    PF_REQUIRE(reps >= 1, "reps must be >= 1");
    PF_REQUIRE((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 == 0,
               "src and dst must be 16-byte aligned");
    *gbs = stream_copy_gbs(ctx->stream, src, dst, bytes, reps, ctx->num_cu);
    return POLFED_OK;
  });
}

int polfed_solve(polfed_ctx *ctx, const polfed_model *model, const polfed_opts *opts, int nev,
                 double *evals, double *evecs, double *resid, polfed_info *info) {
  return guarded(ctx, [&] { return solve_one(ctx, model, opts, nev, evals, evecs, resid, info); });
}

int polfed_solve_batch(polfed_ctx *ctx, int R, const polfed_model *models,
                       const polfed_opts *opts, int nev, double *evals, double *evecs,
                       double *resid, polfed_info *infos, int *status) {
  return guarded(ctx, [&] {
    return solve_batch(ctx, R, models, opts, nev, evals, evecs, resid, infos, status);
  });
}

}  // extern "C"
