// Internal declarations of libpolfed (host C++ and HIP device code).
// Not part of the ABI; the public contract is include/polfed.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <tuple>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/polfed.h"

namespace polfed {

// ---------------------------------------------------------------- errors --

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define PF_HIP(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::polfed::Error(POLFED_EDEVICE, std::string(#expr) + ": " +       \
                                                hipGetErrorString(e_));       \
  } while (0)

#define PF_REQUIRE(cond, msg)                                                 \
  do {                                                                        \
    if (!(cond)) throw ::polfed::Error(POLFED_EINVAL, (msg));                 \
  } while (0)

// Check the launch that was just queued.
void check_launch(const char *what);

// ----------------------------------------------------------- device memory --

// Owning device buffer (hipMalloc / hipFree); grows on demand.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf();
  void *ensure(size_t nbytes);  // contents not preserved on growth
  void release();               // free now (after the device is done with it)
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// ------------------------------------------------------- chain on the GPU --

// Device-resident description of the Sz=0 basis of one chain length L:
// states[n] ascending, and the two rank tables with
//   rank(s) = tabA[s >> half] + tabB[s & (2^half - 1)]
// (tabA int32, tabB uint16: a rank among at most C(15, 7) low patterns)
// (the colexicographic rank sum_t C(p_t, t) split at bit `half`; each half
// contributes a term that depends only on its own bits once the total
// popcount is fixed at L/2).
struct Basis {
  int L = 0;
  int half = 0;
  long long n = 0;
  DevBuf states, tabA, tabB;
  DevBuf binom;  // int32 C(n, k) at [32 n + k], n, k < 32
};

// Stored off-diagonal pattern of H (rank mode 2): per row, the column
// indices of its neighbours in the kernel's bond order (J1 bonds by
// ascending bit, then J2 bonds), the top bit of an index marking a J2 bond;
// its values J_l/2 are implied.  One per (L, J2 != 0).
struct Pattern {
  long long n = 0, nnz = 0;
  DevBuf ptr, col;  // int64 [n + 1], int32 [nnz]
};

// One chain (model + basis + diagonal in FP64).
struct Chain {
  int L;
  double J1, J2, Delta;
  double h[32];
  const Basis *basis;
  mutable const Pattern *pattern = nullptr;  // attached where a launch uses rank mode 2
  DevBuf diag;  // FP64 H[r][r]
};

// Maximum L handled with the rank tables in LDS (6 * 2^(L/2) bytes: 96 KB
// at L = 28, within the 160 KB of a CU).
constexpr int kMaxLdsTableL = 28;

// --------------------------------------------------------------- kernels --

// basis.hip
void upload_binomials(int device);
void build_basis(hipStream_t st, Basis &b, int L);
void launch_rank(hipStream_t st, const Basis &b, long long n, const uint32_t *states,
                 int32_t *ranks);
void launch_diag(hipStream_t st, const Chain &c, double *d);
void build_pattern(hipStream_t st, const Basis &b, bool has_j2, Pattern &pat);
template <class T>
void launch_scaled_diag(hipStream_t st, long long n, const double *d, double a, double b, T *out);

// hv.hip: the fused Chebyshev step / H~ application
//   out[r,:] = alpha X[r,:] + dscale dt[r] V[r,:] + sum_bonds w_l V[nbr,:]
//              + gamma W[r,:]
// X, W may be null (alpha / gamma ignored); V may be null (no operator
// term).  Rows are row-major with the given leading dimensions.
template <class T>
struct StepArgs {
  const uint32_t *states;
  const T *dt;
  const int32_t *tabA;
  const uint16_t *tabB;
  const T *X;
  long long ldx;
  const T *V;
  long long ldv;
  const T *W;
  long long ldw;
  T *out;
  long long ldo;
  T alpha, dscale, w1, w2, gamma;
  long long n;
  int L, half;
  uint32_t lomask, fullmask;
  int has_j2;
  long long rows_per_wg;
  const int32_t *binom;  // C(n, k) at [32 n + k] (incremental ranks)
  // optional fused accumulation (forward recurrence):
  //   acc[r,:] = cin * src[r,:] + cacc * out[r,:]   (src may be acc itself)
  T *acc;
  long long ldacc;
  const T *src;
  long long ldsrc;
  T cin, cacc;
  int skip_out;  // the step's own output is not stored (only acc is)
  // XCD column slices (1, 2, 4 or 8): the block's S columns are split into
  // nslices slices of S / nslices columns; the workgroups of XCD x work on
  // slice x % nslices only, over the rows of part x / nslices.  Each operand
  // gives the element offset from one slice to the next (a row-major block:
  // the slice width; a slice-major block: n times the slice width) -- its
  // leading dimension is then that of the slice.
  int nslices;
  long long xss, vss, wss, oss, accss, srcss;
  // the parts of the rows an XCD group covers are interleaved tile by tile
  // rather than contiguous (set by the launcher for blocks larger than the
  // Infinity Cache)
  int interleave;
  // stored neighbour pattern (rank mode 2): row r's neighbours are
  // csr_col[csr_ptr[r] .. csr_ptr[r+1]), the top bit marking a J2 bond
  const long long *csr_ptr;
  const int32_t *csr_col;
};

// Launch shape of the step kernel (the autotuner's search space).
struct StepShape {
  int threads = 256;     // workgroup size: 256, 512 or 1024
  int lpl = 1;           // 16-byte loads per lane per gathered row
  int wg_per_cu = 8;     // persistent workgroups per CU
  int lds_tables = 1;    // stage rank tables in LDS
  int early_loads = 0;   // issue the streamed loads before the gathers
  int rank_incr = 0;     // neighbour ranks: 0 tables, 1 incremental for bonds
                         // that do not wrap, 2 the stored pattern
  int xcd_slices = 1;    // column slices, one per XCD group (1, 2, 4, 8)
};

template <class T>
void launch_step(hipStream_t st, int S, const StepArgs<T> &a, const StepShape &shape, int num_cu);

// One realisation of a batched filter (device-resident descriptor).  The
// realisations of one launch share the block width and whether J2 != 0;
// each brings its own chain length and basis.
template <class T>
struct BatchItem {
  const T *dt;         // a d + b
  const T *X;          // n x S input block (leading dimension ldx)
  T *buf;              // 3 n x S recurrence buffers (leading dimension S)
  T *Y;                // n x S output (leading dimension ldy)
  const double *coef;  // c_0 .. c_K (device)
  double Dinv;         // 1 / D
  T w1, w2;            // a J1, a J2
  long long K;
  int active;
  // the realisation's chain: Sz=0 states and rank tables, dimension, L
  const uint32_t *states;
  const int32_t *tabA;
  const uint16_t *tabB;
  long long n;
  int L, half;
  uint32_t lomask, fullmask;
  long long ldx, ldy;
  // first row tile of this realisation in the launch's tile range (tiles of
  // batched_tile_rows rows, realisations in item order)
  long long tile0;
  int taboff;  // int32 offset of its tables in the launch's LDS staging (BatchTables.off)
};

// The distinct rank tables of a batched launch (one per chain length), all
// staged in LDS: set k at int32 offset off[k] (tabA, then tabB as uint16).
// count = 0: every realisation reads its own tables from global memory.
constexpr int kMaxBatchTables = 8;
struct BatchTables {
  const int32_t *A[kMaxBatchTables];
  const uint16_t *B[kMaxBatchTables];
  int half[kMaxBatchTables];
  int off[kMaxBatchTables];
  int count;
  int ints;  // LDS size in int32 words
};

// Rows per tile of the batched step kernel for this width and shape.
template <class T>
long long batched_tile_rows(int S, const StepShape &shape);

// One batched Clenshaw step j (0..Kmax) for the B realisations of items
// (device array, tile0 filled for batched_tile_rows; total_tiles = the
// tiles of all of them).  a: the launch's common arguments (has_j2, binom);
// tables: the rank tables staged in LDS (count 0: none).
template <class T>
void launch_step_batched(hipStream_t st, int S, const StepArgs<T> &a, const BatchItem<T> *items,
                         int B, long long j, long long Kmax, long long total_tiles,
                         const BatchTables &tables, const StepShape &shape, int num_cu);
// Built-in default shapes (used when the context holds no tuned entry) of
// the single-chain and the batched step kernel.
StepShape default_shape(int L, int S, bool fp32);
StepShape default_batch_shape(int L, int S, bool fp32);

// out (slice-major: nslices blocks of n x (S / nslices), each row's slice
// contiguous) <- X (n x S, row-major, leading dimension ldx).
template <class T>
void launch_pack_slices(hipStream_t st, long long n, int S, int nslices, const T *X,
                        long long ldx, T *out);

template <class Tin, class Tout>
void launch_cast(hipStream_t st, long long n, int S, const Tin *in, long long ldin, Tout *out,
                 long long ldout);

// dense.hip: FP64 tall-skinny products and small dense kernels
void launch_gram(hipStream_t st, long long n, int p, int q, const double *X, long long ldx,
                 const double *Y, long long ldy, double *C, long long ldc, DevBuf &partials,
                 int num_cu);
// The Gram product in its two launches, on partial tiles the caller
// provides: gram_chunks picks the row chunks (about four workgroups per CU,
// >= 256 rows each; cap > 0 limits them to cap / (p q) partial tiles) and
// launch_gram_parts runs the MFMA kernel and the fixed-order chunk sum.
long long gram_chunks(long long n, int p, int q, int num_cu, long long cap,
                      long long &rows_per_chunk);
void launch_gram_parts(hipStream_t st, long long n, int p, int q, const double *X,
                       long long ldx, const double *Y, long long ldy, double *C, long long ldc,
                       double *part, long long rows_per_chunk, long long nchunks);
// noalloc.hip: the Gram product on the partial tiles of a fixed device
// array of kGramScratchDoubles doubles (16 MiB), one copy per device;
// init_gram_scratch(device) takes the array's device address once per
// device, with the device current, before any call.
constexpr size_t kGramScratchDoubles = (size_t)2 << 20;
void init_gram_scratch(int device);
void launch_gram_static(hipStream_t st, int device, long long n, int p, int q, const double *X,
                        long long ldx, const double *Y, long long ldy, double *C,
                        long long ldc, int num_cu);
void launch_update(hipStream_t st, long long n, int p, int q, double alpha, const double *X,
                   long long ldx, const double *C, long long ldc, double beta, double *Y,
                   long long ldy);
// Jacobi eigensolver; A (n x n) overwritten; w ascending, V columns.
// V0 (nullable, n x n): warm start -- A holds V0^T A_orig V0 and the
// returned V are eigenvectors of A_orig (rotations accumulate onto V0).
void sym_eig(hipStream_t st, int n, double *A, double *w, double *V, DevBuf &work,
             const double *V0 = nullptr);
// B symmetric n x n matrices at once (n <= 128, one workgroup each, matrix
// in LDS): A (B x n x n, destroyed), V (B x n x n) the starting vectors
// (identity, or a warm start with A already rotated), outputs w (B x n,
// ascending) and Vout (B x n x n, columns = eigenvectors).  Returns false
// (nothing launched) when n is too large or the LDS cannot be granted.
bool sym_eig_batched(hipStream_t st, int n, int B, double *A, double *V, double *w,
                     double *Vout);
// W = blockdiag(V0 (n0 x n0), identity) as an n x n row-major matrix.
void launch_embed_block(hipStream_t st, int n, int n0, const double *V0, double *W);
// Cholesky of the s x s Gram matrix G (device, row-major, ld s):
// writes Rinv = L^{-T} (upper) and B = L^T (upper), and flag[0] = index+1
// of the first non-positive pivot (0 if fine).
void launch_chol(hipStream_t st, int s, const double *G, double *Rinv, double *B, int *flag,
                 double rel_tol);
// C = A * B for small row-major matrices (device), C: m x k, A: m x l, B: l x k.
void launch_small_gemm(hipStream_t st, int m, int l, int k, const double *A, int lda,
                       const double *B, int ldb, double *C, int ldc, int transA);
// Fill X (n x S, ld) with uniform [-1,1) from Philox4x32-10 keyed by seed,
// counter (row, col, stream).
void launch_philox_fill(hipStream_t st, long long n, int S, double *X, long long ld,
                        unsigned long long seed, unsigned stream_id);
// Column 2-norms of X (n x q): out[q] (two-stage, deterministic).
void launch_colnorms(hipStream_t st, long long n, int q, const double *X, long long ldx,
                     double *out, DevBuf &partials, int num_cu);
// Residual norms ||HV - V diag(E)|| columns: HV, V (n x q), E[q] -> out[q].
void launch_resid_norms(hipStream_t st, long long n, int q, const double *HV, long long ldhv,
                        const double *V, long long ldv, const double *E, double *out,
                        DevBuf &partials, int num_cu);
// Scale columns: X[:, j] *= f[j].
void launch_scale_cols(hipStream_t st, long long n, int q, double *X, long long ldx,
                       const double *f);
// Sign normalisation factors: f[j] = sign of the largest-|.| entry of
// column j (lowest row on ties).
void launch_sign_factors(hipStream_t st, long long n, int q, const double *X, long long ldx,
                         double *f, DevBuf &partials, int num_cu);
// Transpose row-major X (n x q) into column-major out (out[j*n + r]).
void launch_to_colmajor(hipStream_t st, long long n, int q, const double *X, long long ldx,
                        double *out);
// Gather columns: out[:, j] = X[:, idx[j]].
void launch_gather_cols(hipStream_t st, long long n, int q, const double *X, long long ldx,
                        const int *idx, double *out, long long ldo);
void launch_fill(hipStream_t st, double *x, long long count, double v);
void launch_small_transpose(hipStream_t st, int m, int k, const double *in, int ldi, double *out,
                            int ldo);
void launch_symmetrize(hipStream_t st, int s, double *A, int lda);

// Bounds Lanczos helpers (single vector, FP64, scalars on device).
void launch_dot_partials(hipStream_t st, long long n, const double *x, const double *y,
                         double *part, int nblk);
void launch_lanczos_update(hipStream_t st, long long n, double *w, const double *v,
                           const double *vprev, const double *part, int nblk, double *alpha,
                           const double *beta_prev, double *part2);
void launch_lanczos_normalize(hipStream_t st, long long n, const double *w, double *vnext,
                              const double *part2, int nblk, double *beta);

// observables.hip: S_E of nvec device vectors (row-major n x nvec, ld ldv)
// for each cut (bit offset), into S_host[j * ncut + c] (L <= 18); and the
// mean gap ratio of n >= 3 levels (host).
void entanglement_entropy(hipStream_t st, const Basis &bs, int nvec, const double *V,
                          long long ldv, const std::vector<int> &cuts, double *S_host,
                          DevBuf &work);
double mean_gap_ratio(const double *E, int n);

// measure.hip: copy rate (read + write bytes per second / 1e9) of a plain
// 16-byte-vector device copy of `bytes` bytes, repeated reps times.
double stream_copy_gbs(hipStream_t st, const void *src, void *dst, long long bytes, int reps,
                       int num_cu);

// ------------------------------------------------------------ host math --

// plan.cpp
// (damping: POLFED_DAMP_NONE, the paper's raw delta expansion, or
// POLFED_DAMP_JACKSON; the order rules then use the damped filter's lobe)
void cheb_coeffs(double sigma, long long K, std::vector<double> &c, double &D, int damping = 0);
double dos_gamma(int L, double J1, double J2, double Delta, const double *h);
double trace_mean(int L, double J1, double J2, double Delta);
long long choose_order(long long N, double Ebar, double Gamma, double E0w, double E1w,
                       double sigma, int nwin, double p, double *rho, int damping = 0);
int capped_window(long long N, double Ebar, double Gamma, double E0w, double E1w, double sigma,
                  int nwin, double p, long long K_cap, long long *K, int damping = 0);
// Kernel polynomial method (density of states from Chebyshev moments mu of
// H~, Jackson damping): the number of states in [x_lo, x_hi], the density at
// x, and the order rule and FP32 cap with that density in place of the
// Gaussian.
void jackson(int M, std::vector<double> &g);
double kpm_count(const std::vector<double> &mu, long long N, double x_lo, double x_hi);
double kpm_density(const std::vector<double> &mu, double x);
long long choose_order_kpm(const std::vector<double> &mu, long long N, double sigma, int nwin,
                           double p, int damping = 0);
int capped_window_kpm(const std::vector<double> &mu, long long N, double sigma, int nwin,
                      double p, long long K_cap, long long *K, int damping = 0);
// dos.hip: Chebyshev moments mu_0 .. mu_{nmom-1} of H~ = aH + b from the nvec
// columns of R (device, n x nvec row-major; NULL: +-1 entries from Philox
// keyed by seed), mu_n = sum_r <r|T_n|r> / sum_r <r|r>, into mu (host).
void dos_moments(polfed_ctx *ctx, const Chain &c, double a, double b, int nmom, int nvec,
                 const double *R, unsigned long long seed, std::vector<double> &mu);
// Extreme eigenvalues of the symmetric tridiagonal (alpha[k], beta[k] for
// k=1..k-1 off-diagonal) and the last components of their unit
// eigenvectors.
void tridiag_extremes(const std::vector<double> &alpha, const std::vector<double> &beta,
                      double &lo, double &hi, double &ylo_last, double &yhi_last);

}  // namespace polfed

// ---------------------------------------------------------------- context --

struct polfed_ctx {
  int device = 0;
  int num_cu = 256;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  std::string last_error;
  std::map<int, std::unique_ptr<polfed::Basis>> bases;  // per L
  std::map<std::pair<int, int>, std::unique_ptr<polfed::Pattern>> patterns;  // per (L, J2 != 0)
  std::map<std::string, std::unique_ptr<polfed::DevBuf>> bufs;
  // HIP-event timing of the filter kernels (Chebyshev steps), accumulated
  // over a solve: GPU seconds between the first and last step of each
  // filter application, and the number of step launches
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  double filter_gpu_s = 0.0;
  double filter_launches = 0.0;
  double filter_bytes = 0.0;
  // launch shapes of the step kernel chosen by the autotuner, keyed by
  // (L, block width, precision bytes)
  std::map<std::tuple<int, int, int>, polfed::StepShape> shapes;
  // launch shapes of the batched step kernel (same key); its rank mode is
  // always the tables and its column slices 1
  std::map<std::tuple<int, int, int>, polfed::StepShape> batch_shapes;
  // block sizes chosen by the autotuner, keyed by (L, precision, nev)
  std::map<std::tuple<int, int, int>, int> blocks;
  // cached HIP graph of one whole filter application (K+1 step launches),
  // replayed for every Lanczos block; keyed by everything baked into it
  hipGraphExec_t filter_graph = nullptr;
  std::vector<unsigned long long> filter_graph_key;
  int use_graphs = 1;
  int filter_form = 0;  // POLFED_FORM_CLENSHAW or POLFED_FORM_FORWARD
  int filter_damping = 0;  // POLFED_DAMP_* of polfed_apply_filter
  polfed::DevBuf &buf(const std::string &name) {
    auto &p = bufs[name];
    if (!p) p.reset(new polfed::DevBuf());
    return *p;
  }
  const polfed::Basis &basis(int L);
  const polfed::Pattern &pattern(int L, bool has_j2);
};
