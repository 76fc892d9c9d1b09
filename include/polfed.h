/*
 * polfed.h -- C ABI of libpolfed: the POLFED hot path on AMD MI355X (gfx950).
 *
 * POLFED (polynomially filtered exact diagonalisation; Sierant, Lewenstein,
 * Zakrzewski, arXiv:2005.09534) finds the N_ev eigenpairs nearest an energy
 * target of the disordered spin-1/2 chain of eq. (XXZ) in its Sz=0 sector:
 * block Lanczos, eqs. (Lan1)-(Lan2), applied to the Chebyshev filter
 * P^K_sigma(H~) of eq. (polyTransf), with full reorthogonalisation and a final
 * Rayleigh-Ritz step (main text, "POLFED algorithm"; Supplement,
 * "Convergence of POLFED" and "Technical details").
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: every call returns int.  0 = POLFED_OK; >0 = warning, outputs
 *   written but flagged; <0 = error, outputs untouched.  The message of the
 *   last error on a context is returned by polfed_last_error().
 * - Basis: a Sz=0 basis state is an L-bit integer, bit i <-> site i+1, bit
 *   set <-> S^z = +1/2.  Rows of H are ordered by ascending state integer, so
 *   row r holds the r-th smallest L-bit integer with L/2 set bits.
 * - H: the literal double sum of eq. (XXZ) over l = 1,2 and i = 1..L with
 *   periodic sites; off-diagonal elements +J_l/2 between states that differ
 *   by swapping an antiparallel pair (Supplement, "Technical details").
 * - Rescaled operator: H~ = a H + b with a = 2/(E1-E0), b = -(E0+E1)/(E1-E0)
 *   (main text, "POLFED algorithm").  sigma_tilde is a target in H~ units.
 * - Vector blocks passed to stage calls are DEVICE pointers, row-major
 *   (n rows x nvec columns, row r's nvec values contiguous), FP64 (double)
 *   or FP32 (float) as the precision argument says.  Stage calls are
 *   asynchronous on the context's stream (polfed_set_stream) unless stated.
 * - Ownership: callers allocate every input and output.  The library
 *   allocates and frees only device workspace held by the context.  A
 *   context is used by one host thread at a time.
 * - Sizes: L even, 4 <= L <= 30 (J2 != 0 needs L >= 6).  Block widths
 *   (nvec, block_size) are powers of two from 1 to 64.
 */
#ifndef POLFED_H
#define POLFED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum polfed_status {
  POLFED_OK = 0,
  POLFED_NOT_CONVERGED = 1, /* best pairs returned; info->n_conv met tol */
  POLFED_EINVAL = -1,       /* invalid argument (message says which)     */
  POLFED_ENOMEM = -2,       /* device allocation failed                  */
  POLFED_EDEVICE = -3,      /* HIP runtime error                         */
  POLFED_EBOUNDS = -4,      /* spectral bounds too tight: filter blew up
                               (checked on every Lanczos block; the solve
                               calls retry with the margin eta doubled,
                               three times, before returning it)          */
  POLFED_EBREAKDOWN = -5    /* Lanczos block could not be refilled       */
};

typedef struct polfed_ctx polfed_ctx;

/* The chain of eq. (XXZ).  h: caller-owned host array of length L, read
 * during the call only. */
typedef struct {
  int L;
  double J1, J2, Delta;
  const double *h;
} polfed_model;

/* Solver options.  polfed_default_opts() fills the defaults named here. */
typedef struct {
  int target_kind;        /* 0: target = rescaled energy eps in (0,1),
                             sigma_H = E0 + eps (E1 - E0) with the Lanczos
                             extremes; 1: target = absolute energy sigma_H  */
  double target;          /* default 0.5 (middle of the spectrum)          */
  int block_size;         /* s in {1,2,4,...,64}; 0 = autotuned             */
  long long K;            /* filter order; 0 = from the density of states  */
  double p;               /* threshold on theta; 0 -> 0.17                  */
  int precision;          /* 0: FP64 filter; 1: FP32 filter, FP64 Lanczos,
                             Rayleigh-Ritz and residuals + FP64 refinement  */
  double window_factor;   /* filter window sized for ceil(f N_ev)
                             eigenvalues; 0 -> 1.5.  With K = 0 it is
                             doubled (up to 12) while a run ends with fewer
                             than N_ev Ritz values at theta >= p           */
  int max_cols;           /* Lanczos columns; 0 -> 8 N_win + 8 s           */
  double tol;             /* residual target relative to ||H||; 0 -> 1e-10 */
  double eta;             /* bounds margin, fraction of E1-E0; 0 -> 1e-3   */
  int bounds_steps;       /* bounds Lanczos steps; 0 -> 200                 */
  unsigned long long seed;/* start-block generator key                     */
  long long max_order;    /* FP32 filter with automatic K: the largest order
                             it may take (0 -> 200000); beyond it the
                             window is widened until K fits (N_ev -> a N_ev
                             gives K -> K/a at about the same filter work;
                             Supplement, "Benchmark for disorder spin
                             chains"), and info->nev_window reports it    */
  int dos;                /* density of states of the order rule (K = 0):
                             POLFED_DOS_GAUSS (default) the Gaussian of
                             polfed_filter_order; POLFED_DOS_KPM the kernel
                             polynomial estimate from dos_moments Chebyshev
                             moments of H~ on dos_vectors random +-1
                             vectors (polfed_dos_moments), for chains whose
                             DOS is not Gaussian at the target            */
  int dos_moments;        /* KPM moments M; 0 -> 256                       */
  int dos_vectors;        /* KPM random vectors; 0 -> 4                    */
  int damping;            /* POLFED_DAMP_NONE (default: the paper's raw
                             delta expansion of eq. (polyTransf)) or
                             POLFED_DAMP_JACKSON: c_n g_n with the Jackson
                             factors of the K+1 coefficients, which removes
                             the side lobes and widens the main lobe about
                             twofold; the order rule then counts states in
                             the damped filter's lobe (polfed_filter_coeffs,
                             polfed_filter_order_damped)                  */
} polfed_opts;

enum polfed_dos { POLFED_DOS_GAUSS = 0, POLFED_DOS_KPM = 1 };
enum polfed_damping { POLFED_DAMP_NONE = 0, POLFED_DAMP_JACKSON = 1 };

/* Per-solve record (all times in seconds, wall clock on the host). */
typedef struct {
  double E0, E1;          /* Lanczos extremes of H                          */
  double E0w, E1w;        /* widened bounds used for H~                     */
  double sigma_energy;    /* target in H units                              */
  double sigma_tilde;     /* target in H~ units                             */
  double normH;           /* max(|E0|, |E1|)                                */
  long long K;            /* filter order used                              */
  int nev_window;         /* eigenvalues the window was sized for           */
  int block_size;         /* s used                                         */
  int m;                  /* Lanczos blocks at stop                         */
  int n_conv;             /* pairs with residual <= tol ||H|| (FP32 mode:
                             max(tol, 1e-8) ||H||)                          */
  int refine_passes;      /* FP64 refinement passes (precision 1); -1 when
                             the FP32 result missed 1e-8 ||H|| and was
                             recomputed with the FP64 filter               */
  double max_resid;       /* max returned residual (H units)                */
  double t_bounds, t_filter, t_orth, t_eig, t_rr, t_refine, t_total;
  double hv_apps;         /* H~ applications to single vectors              */
  double filter_bytes;    /* algorithmic bytes moved by the filter kernels  */
  double filter_gpu_s;    /* filter kernel time by HIP events on the stream */
  double filter_launches; /* Chebyshev step kernels launched                */
} polfed_info;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` (hipSetDevice is called).  The
 * context owns a non-blocking stream and its device workspace. */
int polfed_create(int device, polfed_ctx **out);
int polfed_destroy(polfed_ctx *ctx);
/* Message of the last error on ctx ("" if none); owned by ctx.  With
 * ctx == NULL: the message of the last failed polfed_create on the calling
 * host thread (thread-local storage of the library). */
const char *polfed_last_error(const polfed_ctx *ctx);
/* Run subsequent calls on `stream` (a hipStream_t; NULL is HIP's null
 * stream).  Until this is called, calls run on the context's own
 * non-blocking stream. */
int polfed_set_stream(polfed_ctx *ctx, void *stream);
/* Wait for all work the context queued. */
int polfed_synchronize(polfed_ctx *ctx);

/* ---- host-side helpers (no device work) -------------------------------- */

/* C(L, L/2), the Sz=0 sector size ("Benchmark models"); -1 if L is odd or
 * outside [2, 30]. */
long long polfed_dim(int L);
void polfed_default_opts(polfed_opts *opts);

/* Chebyshev coefficients of eq. (polyTransf): c[n] = sqrt(4 - 3 delta_n0)
 * cos(n arccos sigma_tilde), n = 0..K (c: host array of K+1), and *D with
 * P(sigma_tilde) = 1.  |sigma_tilde| < 1. */
int polfed_cheb_coeffs(double sigma_tilde, long long K, double *c, double *D);

/* Filter order from the density of states (main text "POLFED algorithm",
 * Supplement "Convergence"): K = max{K : n_P(K) >= nwin}, where n_P is the
 * number of states of the Gaussian DOS (centre Tr H / N, width Gamma with
 * Gamma^2 = L (J1^2+J2^2)(2+Delta^2)/16 + sum h_i^2/4) inside the main lobe
 * {x : P_K(x) >= p} around sigma_tilde, for H~ built with bounds E0w, E1w.
 * Writes *K and the density rho~(sigma_tilde) (states per unit of H~). */
int polfed_filter_order(const polfed_model *model, double E0w, double E1w,
                        double sigma_tilde, int nwin, double p,
                        long long *K, double *rho);

/* Filter coefficients with optional damping: c[n] = c_n of
 * polfed_cheb_coeffs times g_n, where for damping = POLFED_DAMP_JACKSON
 * g_n = [(M-n+1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))]/(M+1),
 * M = K+1 (Jackson's kernel; Weisse et al., Rev. Mod. Phys. 78, 275), and
 * g_n = 1 for POLFED_DAMP_NONE; *D = sum_n c[n] T_n(sigma_tilde), so that
 * P(sigma_tilde) = 1.  c: host array of K+1.  The damped P is non-negative
 * on [-1, 1]. */
int polfed_filter_coeffs(double sigma_tilde, long long K, int damping, double *c, double *D);
/* polfed_filter_order and polfed_window_order for a damped filter: the
 * main lobe {P_K >= p} is that of the damped P (in closed form: with x =
 * cos theta, sigma_tilde = cos alpha, P(x) = [F(theta-alpha) +
 * F(theta+alpha)]/[F(0) + F(2 alpha)], F(u) = (E(u+beta) + E(u-beta))^2,
 * E(u) = sin(M u/2)/sin(u/2), beta = pi/(M+1)); *K the order and *nwin_out
 * the window after the cap max_order (<= 0: no cap). */
int polfed_filter_order_damped(const polfed_model *model, double E0w, double E1w,
                               double sigma_tilde, int nwin, double p, int damping,
                               long long max_order, int *nwin_out, long long *K);

/* The order cap of the FP32 filter (polfed_opts.max_order): the smallest
 * window count *nwin_out >= nwin whose order from polfed_filter_order is at
 * most max_order, and that order *K (max_order <= 0: no cap, the window
 * stays nwin).  The window never exceeds the sector size. */
int polfed_window_order(const polfed_model *model, double E0w, double E1w,
                        double sigma_tilde, int nwin, double p, long long max_order,
                        int *nwin_out, long long *K);

/* Kernel polynomial method (the iterative DOS estimator the paper names
 * for arbitrary sparse matrices, where K is chosen; main text "POLFED
 * algorithm"): with Chebyshev moments mu[0..nmom-1] of H~ (from
 * polfed_dos_moments) and Jackson damping
 *   g_n = [(M-n+1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))]/(M+1),
 * M = nmom, the number of states of an N-state sector in [x_lo, x_hi]
 * (H~ units, clamped to [-1, 1]) is
 *   N/pi [g_0 mu_0 (t_lo - t_hi) + 2 sum_{n>=1} g_n mu_n (sin n t_lo - sin n t_hi)/n],
 * t = arccos x.  polfed_kpm_count writes it to *count. */
int polfed_kpm_count(const double *mu, int nmom, long long N, double x_lo, double x_hi,
                     double *count);
/* The order rule of polfed_filter_order with the KPM count in place of the
 * Gaussian: *K = max{K : count(main lobe {P_K >= p} around sigma_tilde) >=
 * nwin}, the lobe that of the filter with the given damping
 * (POLFED_DAMP_*); with max_order > 0 and that K above it, the smallest
 * window *nwin_out >= nwin whose order is at most max_order, as in
 * polfed_window_order (else *nwin_out = nwin). */
int polfed_kpm_order(const double *mu, int nmom, long long N, double sigma_tilde, int nwin,
                     double p, int damping, long long max_order, int *nwin_out, long long *K);

/* ---- stage calls (device pointers, async on the context stream) -------- */

/* states[r] = the r-th Sz=0 state (uint32, length polfed_dim(L)). */
int polfed_basis(polfed_ctx *ctx, int L, uint32_t *states);
/* ranks[i] = row of states[i] in the Sz=0 basis, or -1 if states[i] is not
 * an L-bit integer with L/2 set bits.  n >= 0 entries. */
int polfed_rank(polfed_ctx *ctx, int L, long long n, const uint32_t *states,
                int32_t *ranks);
/* d[r] = H[r][r] in FP64 (length polfed_dim(L)). */
int polfed_diag(polfed_ctx *ctx, const polfed_model *model, double *d);
/* Y = H X (unscaled H), X and Y n x nvec row-major, n = polfed_dim(L);
 * precision 0: double, 1: float.  X and Y must not overlap. */
int polfed_apply_h(polfed_ctx *ctx, const polfed_model *model, int precision,
                   int nvec, const void *X, void *Y);
/* Y = P^K_sigma(H~) X, with H~ built from E0, E1 (used as given), by the
 * Clenshaw recurrence (Supplement, "Technical details") or by the forward
 * recurrence that accumulates c_k T_k(H~) X term by term, as the context's
 * polfed_set_filter_form says; precision 0: double, 1: float; K >= 0.
 * X and Y must not overlap. */
int polfed_apply_filter(polfed_ctx *ctx, const polfed_model *model, double E0,
                        double E1, double sigma_tilde, long long K,
                        int precision, int nvec, const void *X, void *Y);

/* Chebyshev moments of H~ = a H + b, a = 2/(E1w - E0w), b = -(E0w + E1w)/
 * (E1w - E0w), for the kernel polynomial DOS (Silver et al.):
 *   mu[j] = sum_r <r|T_j(H~)|r> / sum_r <r|r>,  j = 0 .. nmom-1,
 * over the nvec columns r of R (device, n x nvec row-major, n =
 * polfed_dim(L), read only), or, with R = NULL, of nvec vectors of +-1
 * entries drawn from Philox4x32-10 keyed by seed.  With +-1 entries mu[j]
 * estimates Tr T_j(H~) / n.  FP64; the moments come from floor(nmom/2)
 * three-term steps by T_2k = 2 T_k^2 - 1 and T_2k+1 = 2 T_k+1 T_k - T_1;
 * mu[0] = 1.  mu: host array of nmom.  1 <= nmom <= 2^20, nvec >= 1.
 * Blocks the host until done; deterministic for fixed inputs. */
int polfed_dos_moments(polfed_ctx *ctx, const polfed_model *model, double E0w, double E1w,
                       int nmom, int nvec, const double *R, unsigned long long seed,
                       double *mu);

/* Tall-skinny FP64 products on the matrix cores (block Gram-Schmidt and
 * projection of eqs. (Lan1)-(Lan2) and the Ritz step).  All operands are
 * device, row-major, with leading dimensions in elements:
 *   polfed_gram:   C (p x q, ldc) = X^T Y,  X: n x p, Y: n x q
 *   polfed_update: Y (n x q) = alpha X C + beta Y,  X: n x p, C: p x q
 * p, q >= 1; polfed_update needs q <= 64.  Results are deterministic. */
int polfed_gram(polfed_ctx *ctx, long long n, int p, int q, const double *X,
                long long ldx, const double *Y, long long ldy, double *C,
                long long ldc);
/* polfed_gram for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same product, C (p x q, ldc) = X^T Y, with its partial tiles in a
 * fixed 16 MiB device array of the library (one per GPU, held until the
 * process ends) instead of the context's workspace; it calls no hipMalloc,
 * hipFree or allocating routine.  The number of row chunks is limited so
 * that their partial tiles fit the array, so results equal polfed_gram's to
 * rounding (bitwise when the chunking is the same) and are deterministic.
 * Needs p * q <= 2^21 (else POLFED_EINVAL with a message); n = 0 writes
 * C = 0 (X and Y may then be NULL).  Calls that overlap in time on one GPU
 * (two streams or two contexts) race on the array. */
int polfed_gram_static(polfed_ctx *ctx, long long n, int p, int q, const double *X,
                       long long ldx, const double *Y, long long ldy, double *C,
                       long long ldc);
int polfed_update(polfed_ctx *ctx, long long n, int p, int q, double alpha,
                  const double *X, long long ldx, const double *C,
                  long long ldc, double beta, double *Y, long long ldy);

/* Symmetric eigendecomposition on the device (cyclic Jacobi, FP64):
 * A (n x n, row-major, symmetric; overwritten) -> w[n] eigenvalues in
 * ascending order and V (n x n, row-major) with eigenvector i in column i.
 * Used for T_m and the Rayleigh-Ritz matrix.  1 <= n <= 4096.  Blocks the
 * host until done (it reads the convergence flag). */
int polfed_sym_eig(polfed_ctx *ctx, int n, double *A, double *w, double *V);

/* Spectral bounds: `steps` of single-vector FP64 Lanczos on H from a
 * seeded start vector (main text: E0, E1 from the Lanczos algorithm).
 * Writes the extreme Ritz values and their residual bounds |beta_k y_k|.
 * Blocks the host until done. */
int polfed_bounds(polfed_ctx *ctx, const polfed_model *model, int steps,
                  unsigned long long seed, double *E0, double *E1,
                  double *r0, double *r1);

/* ---- tuning and measurement -------------------------------------------- */

/* Launch shape of the fused Chebyshev-step kernel for chains of length L,
 * block width nvec (power of two, 1..64) and precision (0: FP64, 1: FP32):
 * threads per workgroup (256, 512 or 1024), 16-byte loads per lane per gathered
 * row (lpl: 1, 2 or 4), persistent workgroups per compute unit (1..32),
 * whether the rank tables are staged in LDS (ignored for L > 28), whether
 * the streamed operands are loaded before the neighbour gathers
 * (early_loads != 0), and how neighbour ranks are found (rank_incremental
 * = 0: the two rank tables for every bond; 1: from the row's own rank by a
 * binomial step for bonds that do not wrap round the chain, the tables for
 * the rest; 2: from a stored pattern of the off-diagonal entries -- column
 * indices only, the value J_l/2 implied, the paper's own matrix form
 * (Supplement, "Technical details") -- built on the device at the first
 * use for a chain length (4 bytes per entry, 8 per row), whose index
 * reads the filter's byte count then includes; the batched solve always
 * uses the tables), and
 * into how many column slices the block is split across the eight XCDs
 * (xcd_slices = 1, 2, 4 or 8; the workgroups of XCD x work on slice
 * x % xcd_slices over 8 / xcd_slices of the rows, so that each XCD's L2
 * holds more rows of a narrower slice; the Clenshaw filter then keeps its
 * recurrence blocks slice-major; a width that does not split runs
 * unsliced; single H applications and the forward form are never sliced).
 * Results are identical for every shape.  Entries live in the context;
 * without one the library's built-in default is used.  The autotuner
 * (paper_2005_09534_amd/autotune.py) searches this space. */
int polfed_set_step_shape(polfed_ctx *ctx, int L, int nvec, int precision, int threads,
                          int lpl, int wg_per_cu, int lds_tables, int early_loads,
                          int rank_incremental, int xcd_slices);
/* The step shape in force for (L, nvec, precision): the context's entry,
 * else the built-in default.  Outputs as in polfed_set_step_shape. */
int polfed_get_step_shape(polfed_ctx *ctx, int L, int nvec, int precision, int *threads,
                          int *lpl, int *wg_per_cu, int *lds_tables, int *early_loads,
                          int *rank_incremental, int *xcd_slices);
/* Launch shape of the batched step kernel of polfed_solve_batch (its
 * Lanczos filters and FP64 refinement filters) for a launch whose longest
 * chain has length L, at block width nvec and precision: threads, loads per
 * lane, workgroups per CU, LDS tables, early loads and column slices as in
 * polfed_set_step_shape (the batched kernel always ranks with the tables;
 * the tables of every chain length in a launch go to LDS together).
 * Separate from the single-chain shape: a batched launch walks many chains,
 * where the best shape differs.  Without an entry a built-in default is
 * used (the single-chain default without column slices). */
int polfed_set_batch_shape(polfed_ctx *ctx, int L, int nvec, int precision, int threads,
                           int lpl, int wg_per_cu, int lds_tables, int early_loads,
                           int xcd_slices);
int polfed_get_batch_shape(polfed_ctx *ctx, int L, int nvec, int precision, int *threads,
                           int *lpl, int *wg_per_cu, int *lds_tables, int *early_loads,
                           int *xcd_slices);
/* Block size used when opts->block_size is 0 for chains of length L at the
 * given precision and N_ev (the autotuner's choice); without an entry a
 * built-in rule is used (about N_ev/4, capped at 16 in FP64 and 32 in FP32,
 * at 8 for L <= 14). */
int polfed_set_block_size(polfed_ctx *ctx, int L, int precision, int nev, int block_size);
/* Capture each filter application (its K+1 step launches) in a HIP graph
 * that is replayed for every Lanczos block (on != 0, the default unless the
 * environment sets POLFED_NO_GRAPH), or launch the steps one by one.  Used
 * where a step is short (blocks up to 64 MB, K <= 2^17).  Results are
 * identical either way. */
int polfed_set_graphs(polfed_ctx *ctx, int on);
/* Recurrence that evaluates the filter sum_k c_k T_k(H~) X / D (eq.
 * (polyTransf)) in polfed_apply_filter and in polfed_solve (its Lanczos
 * blocks and FP64 refinement): POLFED_FORM_CLENSHAW (the default; Clenshaw's
 * backward recurrence, Supplement, "Technical details") or
 * POLFED_FORM_FORWARD (t_{k+1} = 2 H~ t_k - t_{k-1}, with c_k/D times each
 * t_k added to Y in the same launch; two more streamed blocks per step).
 * The two agree to rounding.  polfed_solve_batch always uses Clenshaw. */
#define POLFED_FORM_CLENSHAW 0
#define POLFED_FORM_FORWARD 1
int polfed_set_filter_form(polfed_ctx *ctx, int form);
/* Damping of the filter coefficients in polfed_apply_filter
 * (POLFED_DAMP_NONE, the default, or POLFED_DAMP_JACKSON; polfed_solve takes
 * it from its options). */
int polfed_set_filter_damping(polfed_ctx *ctx, int damping);
/* Filter counters accumulated by the context since the last reset (or the
 * start of the last polfed_solve): kernel time of the Chebyshev steps by HIP
 * events on the context's stream (seconds), step launches, and algorithmic
 * bytes (each vector element counted once per stream it is read or
 * written: n [nvec b (streams) + 4 + b] per step, b = 4 or 8).  Any output
 * pointer may be NULL.  reset != 0 zeroes the counters after reading. */
int polfed_filter_stats(polfed_ctx *ctx, double *gpu_s, double *launches, double *bytes,
                        int reset);

/* ---- observables of the eigenpairs (main text, "Entanglement entropy and
 * level statistics") ----------------------------------------------------- */

/* Entanglement entropy S_E = -sum_i alpha_i^2 ln(alpha_i^2) over the Schmidt
 * coefficients alpha_i of each of nvec vectors (DEVICE, row-major
 * polfed_dim(L) x nvec with leading dimension ldv >= nvec, unit norm, in the
 * basis order of the header) for the bipartition of the ring at each of
 * ncut cuts: cut x (host array cuts[c], 0 <= x < L) puts bits x .. x+L/2-1
 * (mod L), i.e. sites x+1 .. x+L/2, in the first half.  S (HOST, nvec x
 * ncut) receives S[j * ncut + c].  The coefficient matrix is block diagonal
 * by the magnetisation of the first half; the blocks' Gram matrices are
 * diagonalised on the device.  2 <= L <= 18 (blocks up to 128 x 128).
 * Blocks the host until done. */
int polfed_entanglement(polfed_ctx *ctx, int L, int nvec, const double *V, long long ldv,
                        int ncut, const int *cuts, double *S);
/* Mean gap ratio of n >= 3 levels E (host; any order): the average over
 * consecutive sorted levels of r_i = min(g_i, g_{i+1}) / max(g_i, g_{i+1}),
 * g_i = E_{i+1} - E_i. */
int polfed_gap_ratio(const double *E, int n, double *rbar);
/* S_RMT(L) = (L/2) ln 2 + (1/2 + ln(1/2))/2 - 1/2, the entropy of a chaotic
 * chain in the zero-magnetisation sector, by which S_E is scaled. */
double polfed_s_rmt(int L);

/* Attainable device-memory bandwidth, for setting the step kernel's
 * achieved rate beside it: copies `bytes` bytes (a positive multiple of 16;
 * src and dst device pointers, 16-byte aligned, not overlapping) with a
 * plain kernel of 16-byte non-temporal loads and stores, once to warm up and
 * then `reps` times, timed with HIP events on the context's stream.  Writes
 * *gbs = (read + written bytes) / seconds / 1e9.  Blocks until done.  The
 * copy should be much larger than the 256 MB Infinity Cache. */
int polfed_stream_copy(polfed_ctx *ctx, const void *src, void *dst, long long bytes, int reps,
                       double *gbs);

/* ---- the solve --------------------------------------------------------- */

/* The nev eigenpairs of H nearest the target.  Outputs are HOST arrays the
 * caller allocates: evals[nev] ascending (H units); evecs (nullable)
 * [dim x nev] column-major (eigenvector i contiguous at evecs + i*dim),
 * each of unit norm with its largest-|.| entry positive (lowest index on
 * ties); resid[nev] = ||H v - E v||_2.  info nullable.  opts NULL means
 * defaults.  With an automatic order (K = 0), a run whose filter window
 * turns out to hold fewer than nev Ritz values at theta >= p (the Gaussian
 * density of states overestimated the density at the target) is repeated
 * with the window doubled (info->nev_window reports the final one).  In FP32
 * mode a result whose largest residual misses 1e-8 ||H|| after the
 * refinement is recomputed with the FP64 filter (info->refine_passes = -1).
 * Returns POLFED_NOT_CONVERGED (with the best nev pairs) when the Lanczos
 * column cap is reached first, when the window is still too narrow at
 * 12 N_ev, or when a returned residual exceeds max(tol, 1e-8) ||H||.
 * Blocks until done. */
int polfed_solve(polfed_ctx *ctx, const polfed_model *model,
                 const polfed_opts *opts, int nev, double *evals,
                 double *evecs, double *resid, polfed_info *info);

/* R independent realisations (paper, "Benchmark": disorder averages are
 * many independent runs) solved together: models[R] may mix L.  evals and
 * resid are [R x nev] (realisation-major); evecs NULL or the concatenation
 * of the per-realisation [dim_r x nev] column-major blocks; infos (nullable)
 * [R]; status[R] per realisation: POLFED_OK, POLFED_NOT_CONVERGED, or the
 * member's own error (POLFED_EBOUNDS after the retries below,
 * POLFED_EBREAKDOWN, POLFED_EINVAL), which ends that member only, its
 * outputs left untouched.  Returns POLFED_OK when every member is OK, else
 * POLFED_NOT_CONVERGED; an error of the device or its memory ends the call
 * and is returned.  R >= 1 and
 * 1 <= nev <= dim_r for every model, checked before any work (else
 * POLFED_EINVAL with the outputs untouched).  Window doubling and FP64
 * re-solves as in polfed_solve, each run for the members concerned as a
 * batch of its own; a member whose filter left [-1, 1] is solved again with
 * the bounds margin eta doubled (three times at most), as in polfed_solve.
 * Realisations with one block size and the same J2 != 0
 * share every filter launch whatever their L (one batched step kernel walks
 * all their row tiles), and the FP64 refinement filters of the FP32 mode
 * run batched in the same way.  With opts->block_size = 0 each chain
 * length takes its own block size (polfed_set_block_size, else the
 * built-in rule). */
int polfed_solve_batch(polfed_ctx *ctx, int R, const polfed_model *models,
                       const polfed_opts *opts, int nev, double *evals,
                       double *evecs, double *resid, polfed_info *infos,
                       int *status);

#ifdef __cplusplus
}
#endif

#endif /* POLFED_H */
