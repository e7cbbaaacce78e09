/*
 * rpchol: bistochastic kernel eigendecomposition by randomly pivoted partial
 * Cholesky, for AMD Instinct MI355X (gfx950).
 *
 * The method is that of Vales & Giannakis, "Accelerated decomposition of
 * bistochastic kernel matrices by low rank approximation":
 *   - rpchol_factor   : Algorithm 2 (accelerated randomly pivoted Cholesky,
 *                       ARPC) with Algorithm 3 (its accept/reject check), on
 *                       the Gaussian kernel K_ij = exp(-|x_i - x_j|^2 / eps)
 *                       of the Application section (eq. data-kernel), which
 *                       is never formed;
 *   - bistoch_degrees : the normalisation vectors d~ = diag(F F^T 1) and
 *                       q~ = diag(F F^T D~^{-1} 1) of Algorithm 1 and the
 *                       section "Bistochastic normalization";
 *   - bistoch_eig     : the rest of Algorithm 1 (QR of D~^{-1} F, EVD of the
 *                       small inner matrix R C R^T with C = F^T Q~^{-1} F,
 *                       eigenvectors U = Q V), top nev eigenpairs;
 *   - nystrom_extend  : the Nystrom extension of the section "Nystrom method
 *                       connection", applied to P~, at new points.
 *
 * Conventions shared by every entry point:
 *   - Every data pointer is a DEVICE pointer owned by the caller.  The
 *     library allocates nothing on these paths; scratch memory comes from
 *     a caller-provided workspace whose size the *_workspace_size call
 *     returns.  Workspaces may not be shared by calls that overlap in time.
 *   - Every call is stream-ordered and asynchronous on `stream` (0 = the
 *     null stream), with one exception: for r > 96, bistoch_eig and
 *     bistoch_lowmem read the small eigensolver's convergence flag back to
 *     the host after each of its Rayleigh-Ritz steps (one synchronisation of
 *     `stream` each, usually one in all), and issue its retries and fallback
 *     only when needed; while the stream is being captured into a graph, or
 *     inside the batched form, they issue those launches unconditionally
 *     (each returns at once after convergence) and never synchronise.  The
 *     return value reports host-side argument checks and launch errors
 *     only.
 *   - Failures found on the device (a degree <= 0, a Cholesky breakdown,
 *     non-finite input) are written to the device int32 *dev_status, which
 *     the caller clears to 0 before the call and reads after a sync
 *     (rpc_status_sync does both the sync and the read).  The first error
 *     written wins.
 *   - The accepted pivot count k lives in device memory (int32) so that no
 *     call needs a host synchronisation; columns of F at index >= k are 0.
 *   - Layouts: X is row-major N x d (float32, float64 or bf16, leading
 *     dimension ldx >= d).
 *     F is column-major N x r with leading dimension ldf >= N, ldf a
 *     multiple of 8.  U is column-major N x nev (leading dimension ldu >= N,
 *     a multiple of 8).  Phi is column-major M x nev (ldphi >= M).
 *   - Nothing throws across the ABI.  Calls on distinct buffers and
 *     workspaces may run concurrently on different streams.
 */
#ifndef RPCHOL_H_
#define RPCHOL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* rpc_stream_t; /* a hipStream_t */

typedef enum {
  RPC_OK = 0,
  RPC_EINVAL = -1,      /* bad argument: r > N, b < 1, greedy with b != 1, eps <= 0, nev > r, NULL, dtype */
  RPC_EWORKSPACE = -2,  /* workspace smaller than *_workspace_size reported */
  RPC_EHIP = -3,        /* HIP launch or runtime error */
  RPC_EDEGREE = -4,     /* device: an entry of d~ = diag(F F^T 1) is not > 0 (Algorithm 1 assert) */
  RPC_EQDEGREE = -5,    /* device: an entry of q~ = diag(F F^T D~^{-1} 1) is not > 0 (Algorithm 1 assert) */
  RPC_EBREAKDOWN = -6,  /* device: Cholesky of a Gram or a replayed pivot block not positive definite */
  RPC_ENONFINITE = -7,  /* device: non-finite value in the input points */
  RPC_ENOCONV = -8      /* device: the small eigensolver hit its iteration limit */
} rpc_status;

/* RPC_F32_SPLIT16: float32 data whose products run on the fp16 MFMA pipe,
 * each operand split as hi = fp16(x) plus lo = fp16(x - hi) and each product
 * taken as hi hi + hi lo + lo hi (about 2^-22 relative per product: 22 of
 * float32's 24 significand bits, so a form of its own between bf16 and
 * float32, not float32-grade); accepted as gemm_dtype and as gram_dtype, in
 * both cases with a float32 factor. */
typedef enum { RPC_F64 = 0, RPC_F32 = 1, RPC_BF16 = 2, RPC_F32_SPLIT16 = 3 } rpc_dtype;

typedef enum {
  RPC_SAMPLED = 0, /* Algorithm 2: b iid proposals per round from rho / sum(rho) */
  RPC_GREEDY = 1,  /* deterministic pivoting: argmax rho (lowest index on ties); needs b = 1 */
  RPC_REPLAY = 2   /* the ordered pivots in `replay` are taken, all accepted */
} rpc_mode;

/* Points: N rows of dimension d, row-major, and the bandwidth eps of
 * k(x, y) = exp(-|x - y|^2 / eps).  dtype is the element type of X:
 * RPC_F32, RPC_F64 or RPC_BF16 (others: RPC_EINVAL).  The float64 arithmetic
 * of the method sees the stored values exactly; bf16 distance products of
 * float64 points round them through float32.  The learned-surrogate calls
 * take RPC_F32 points only. */
typedef struct {
  int64_t N;
  int64_t d;
  int64_t ldx;
  const void* X; /* device, ldx elements per row */
  double eps;
  int32_t dtype; /* rpc_dtype of X */
} rpc_points;

/* Options of rpchol_factor (Algorithm 2).
 *  r, b         rank budget and block size; t = ceil(r / b) rounds, the last
 *               proposes r - (t - 1) b pivots.
 *  gemm_dtype   arithmetic of the kernel-column distance products:
 *               F64 (points upcast exactly), F32, or BF16 (points rounded to
 *               bf16; squared norms of the rounded points in fp32; the result
 *               is the exact Gaussian kernel of the rounded points up to fp32
 *               accumulation), or F32_SPLIT16 (float32 points, the inner
 *               products as split fp16 pairs after scaling both operands by
 *               one power of two chosen from max |x| (exact): columns at
 *               the fp16 MFMA rate with about 22 of float32's 24
 *               significand bits per product; the Schur update is split
 *               likewise, the pivot-block solve stays float64; needs
 *               factor_dtype F32).
 *               The pivot block H uses the same points in float64.
 *  factor_dtype F64 or F32: storage of F and arithmetic of the Schur update.
 *               Pivot selection, the pivot-block Cholesky, the triangular
 *               solve and the residual diagonal are float64 in every mode.
 *  tau          a proposal whose updated pivot H(i, i) <= tau is rejected.
 *  uniforms     device doubles in [0, 1), multiples of 2^-53; round i uses
 *               uniforms[2 b i + j] for proposal j and uniforms[2 b i + b + j]
 *               for its accept test; n_uniforms >= 2 b ceil(r / b)
 *               (SAMPLED only).
 *  replay       device int64 ordered pivots (REPLAY only), n_replay <= r.
 *  round_accepted  optional device int32 array of ceil(r / b) entries (or
 *               ceil(n_replay / b) in replay mode) receiving the number of
 *               pivots accepted in each round; may be NULL.
 *  round_trace  optional device double array of as many entries receiving
 *               after each round the relative trace error
 *               tr(K - F F^T) / tr(K) = sum(rho) / N of the factor so far
 *               (the error Algorithm 2 reduces round by round; Theorem 1
 *               bounds its expectation); may be NULL.
 *  flags        RPC_FACTOR_UNFUSED: evaluate the kernel columns and the Schur
 *               update W -= F F_S^T in two kernels (W written, then read
 *               back) instead of one fused kernel where both products share
 *               an accumulator; results agree to rounding.  Meant for timing
 *               the kernel-column evaluation on its own.
 *               RPC_FACTOR_SHARED_X: the job may share its kernel-column pass
 *               with other jobs on the same points (rpchol_factor_group,
 *               rpc_batched_run); the factorisation then uses the two-kernel
 *               arithmetic of RPC_FACTOR_UNFUSED, so a job factorised alone
 *               with this bit equals the same job factorised in a group, bit
 *               for bit.
 *               RPC_FACTOR_LOW_MEMORY: the low-memory form (the paper's
 *               appendix on randomly pivoted Cholesky): the N x r factor is
 *               never stored; F receives only F(S, :), the r x r lower
 *               triangular factor rows of the pivots in pivot order (ldf >= r;
 *               rows and columns >= k are zero), from which any row follows as
 *               F(x, :) = K(x, X_S) F(S, :)^{-T}.  Each round evaluates again
 *               the kernel columns of every earlier round in place of reading
 *               F (round i makes i extra column passes), keeping the memory at
 *               O(N (d + b) + r^2) beyond the points.  Needs factor_dtype F64;
 *               not with RPC_FACTOR_SHARED_X.  Pivots, k, rho and
 *               round_accepted are as in the full form (to rounding).
 *               RPC_FACTOR_SPLIT_SOLVE: the pivot-block solve G = W L^{-T}
 *               runs on the fp16 MFMA pipe as split hi/lo pairs (about 2^-22
 *               per product) instead of in float64; only with BF16 products
 *               and a float32 factor, not with RPC_FACTOR_LOW_MEMORY.  Without
 *               it the solve is float64 in every form, as the method's
 *               precision form asks.
 *               Other bits: RPC_EINVAL. */
#define RPC_FACTOR_UNFUSED 1
#define RPC_FACTOR_SHARED_X 2
#define RPC_FACTOR_LOW_MEMORY 4
#define RPC_FACTOR_SPLIT_SOLVE 8
typedef struct {
  int32_t r;
  int32_t b;
  int32_t mode;         /* rpc_mode */
  int32_t gemm_dtype;   /* rpc_dtype */
  int32_t factor_dtype; /* RPC_F64 or RPC_F32 */
  int32_t flags;        /* RPC_FACTOR_* bits, 0 by default */
  double tau;
  const double* uniforms;
  int64_t n_uniforms;
  const int64_t* replay;
  int64_t n_replay;
  int32_t* round_accepted;
  double* round_trace;
} rpc_factor_opts;

/* Options of bistoch_eig (Algorithm 1 after the factorisation).
 *  nev        number of leading eigenpairs returned (1 <= nev <= r).
 *  gamma      regulariser added to the entries (i, i), i < k, of D~^{-1} F
 *             before the QR (the stabilised QR of the "Numerical experiments"
 *             section); default 0.  The decomposition is then that of
 *             B' C B'^T with B' = D~^{-1} F + gamma E_k (E_k: ones at (i, i),
 *             i < k): G_B gains gamma (B_k + B_k^T) + gamma^2 I_k and U rows
 *             i < k gain gamma (R^{-1} V)[i, :], so U stays orthonormal; the
 *             eigenvalues carry a floor of order gamma^2 (the paper's 1e-8
 *             floor).  ext_E satisfies U = B' ext_E, so the extension of a
 *             training row i < k differs from U[i, :] by gamma ext_E[i, :].
 *  fix_const  if nonzero, U(:, 0) is set to 1/sqrt(N) and U re-orthonormalised
 *             by a QR with positive diag(R) (Algorithm 1, optional lines).
 *  gram_dtype F64, F32 or F32_SPLIT16: arithmetic of the two N-long Gram
 *             products (float64 accumulation across row chunks in all cases);
 *             F32_SPLIT16 needs a float32 factor (RPC_EINVAL otherwise) and
 *             is otherwise the F32 form (r x r stages, scales and U).
 *  u_dtype    F64 or F32 storage of U.
 *  normalization  RPC_BISTOCHASTIC (default), or RPC_SYMMETRIC: the
 *             eigenpairs of L~ = D~^{-1/2} K~ D~^{-1/2} (the paper's symmetric
 *             normalisation), computed with B = D~^{-1/2} F and C = I (one
 *             Gram product instead of two; q~ is not read).  Its leading
 *             eigenpair is (1, D~^{1/2} 1 / |D~^{1/2} 1|).  fix_const is not
 *             defined for it (RPC_EINVAL); ext_E is then R^T V Lambda^{-1}, the
 *             matrix of the extension f(y)^T E / sqrt(c^T f(y)), which
 *             nystrom_extend_symmetric applies. */
typedef enum {
  RPC_BISTOCHASTIC = 0, /* P~ = D~^{-1} K~ Q~^{-1} K~ D~^{-1} (Algorithm 1) */
  RPC_SYMMETRIC = 1     /* L~ = D~^{-1/2} K~ D~^{-1/2} (symmetric normalisation) */
} rpc_normalization;

/* QR of B in Algorithm 1 (the paper suggests CGS2 or Cholesky QR2):
 *  RPC_QR_CHOLQR   Cholesky QR in Gram space: G_B = B^T B = R^T R (column
 *                  equilibrated), Q = B R^{-1} never formed (default; one
 *                  N-long Gram product, exact to the Gram's rounding times
 *                  cond(B)^2).
 *  RPC_QR_CHOLQR2  Cholesky QR2: Q1 = B R1^{-1} is formed in float64 (N x r
 *                  workspace), its Gram G2 = Q1^T Q1 = R2^T R2 factored
 *                  again, R = R2 R1, U = Q1 R2^{-1} V: orthogonality to
 *                  rounding for B with cond(B) up to about u^{-1/2}, at the
 *                  cost of one N x r x r product and one more Gram. */
typedef enum { RPC_QR_CHOLQR = 0, RPC_QR_CHOLQR2 = 1 } rpc_qr_mode;

typedef struct {
  int32_t nev;
  int32_t fix_const;
  int32_t gram_dtype;
  int32_t u_dtype;
  int32_t normalization; /* rpc_normalization */
  int32_t qr_mode;       /* rpc_qr_mode */
  double gamma;
} rpc_eig_opts;

/* ---- Algorithm 2 (ARPC) with Algorithm 3 ------------------------------
 * Outputs: F (N x r, column-major, dtype factor_dtype; columns >= k are 0),
 * pivots (r int64 in acceptance order, entries >= k set to -1), rho (N
 * doubles: the final residual diagonal diag(K - F F^T), clamped >= 0, zero at
 * pivots), k_out (device int32: accepted pivot count).  The relative trace
 * error of the approximation is sum(rho) / N. */
int rpchol_factor_workspace_size(const rpc_points* X, const rpc_factor_opts* opts, size_t* bytes);
int rpchol_factor(const rpc_points* X, const rpc_factor_opts* opts, void* F, int64_t ldf,
                  int64_t* pivots, double* rho, int32_t* k_out, void* workspace,
                  size_t workspace_bytes, int32_t* dev_status, rpc_stream_t stream);

/* ---- Algorithm 2 for several bandwidths on the same points ------------
 * The data sets of the method are often decomposed at several bandwidths
 * (the batched form's 8 per data set).  rpchol_factor_group runs n_group
 * (1..16) factorisations of the same points X (X->eps is ignored) with
 * bandwidths eps[g] (host array) and options opts[g] (host array of host
 * pointers) in lockstep: the points are converted once, and each round's
 * kernel columns of all jobs are computed in one launch whose workgroups for
 * one tile of rows run together, so X is read from HBM once per round for the
 * group (per-column bandwidth in the exp epilogue).  Every job must use the
 * same r, b, mode (SAMPLED or GREEDY), gemm_dtype, factor_dtype, tau and
 * flags, with RPC_FACTOR_SHARED_X set, and a gemm_dtype other than
 * F32_SPLIT16; uniforms and round_accepted may differ.
 * Outputs are per job (host arrays of device pointers), each exactly what
 * rpchol_factor returns for that job alone (bit for bit); F leading
 * dimension ldf is common.  The workspace holds the converted points once and
 * the round state of every job. */
int rpchol_factor_group_workspace_size(const rpc_points* X, const rpc_factor_opts* opts,
                                       int32_t n_group, size_t* bytes);
int rpchol_factor_group(const rpc_points* X, const double* eps, const rpc_factor_opts* const* opts,
                        int32_t n_group, void* const* F, int64_t ldf, int64_t* const* pivots,
                        double* const* rho, int32_t* const* k_out, int32_t* const* dev_status,
                        void* workspace, size_t workspace_bytes, rpc_stream_t stream);

/* ---- Algorithm 1: normalisation vectors -------------------------------
 * c = F^T 1 (r doubles), d~ = F c (N doubles, asserted > 0, RPC_EDEGREE),
 * w = F^T (1/d~), q~ = F w (N doubles, asserted > 0, RPC_EQDEGREE).  Only the
 * first *k columns of F are read. */
int bistoch_degrees_workspace_size(int64_t N, int32_t r, size_t* bytes);
int bistoch_degrees(const void* F, int32_t f_dtype, int64_t N, int64_t ldf, int32_t r,
                    const int32_t* k, double* c, double* d_tilde, double* q_tilde,
                    void* workspace, size_t workspace_bytes, int32_t* dev_status,
                    rpc_stream_t stream);

/* ---- bistoch_degrees for callers that cannot allocate ------------------
 * For code that may not call hipMalloc or pass a workspace (work under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same computation and results as bistoch_degrees, bit for bit, with the
 * scratch taken from a library-owned static device array of about 9 MiB
 * (each GPU the library runs on holds one copy until the process ends).
 * Limits: N <= 1048576 and r <= 1024; larger sizes return RPC_EWORKSPACE
 * without launching anything.  `stream` must belong to the current device
 * (RPC_EINVAL otherwise).  Every call on a GPU shares that GPU's array, so
 * calls that overlap in time on one GPU (different streams, or host
 * threads) race and give undefined results; calls in one stream are
 * ordered and safe.  Allocates no device or host memory. */
int bistoch_degrees_noalloc(const void* F, int32_t f_dtype, int64_t N, int64_t ldf, int32_t r,
                            const int32_t* k, double* c, double* d_tilde, double* q_tilde,
                            int32_t* dev_status, rpc_stream_t stream);

/* ---- Algorithm 1: factored EVD ----------------------------------------
 * With B = D~^{-1} F (+ gamma on its leading diagonal, see rpc_eig_opts) and
 * C = F^T Q~^{-1} F:
 * G_B = B^T B = R^T R (Cholesky QR, R upper triangular with positive
 * diagonal, so Q = B R^{-1} is never formed), M = R C R^T, M = V Lambda V^T,
 * U = B R^{-1} V(:, :nev).  Outputs: U (N x nev, column-major, u_dtype;
 * each column signed so its largest-magnitude entry, lowest index on ties,
 * is positive), lambda (nev doubles, decreasing), ext_E (r x nev doubles,
 * column-major: E = C R^T V Lambda^{-1} with rows >= k zero), which
 * nystrom_extend consumes. */
int bistoch_eig_workspace_size(int64_t N, int32_t r, const rpc_eig_opts* opts, size_t* bytes);
int bistoch_eig(const void* F, int32_t f_dtype, int64_t N, int64_t ldf, int32_t r,
                const int32_t* k, const double* c, const double* d_tilde, const double* q_tilde,
                const rpc_eig_opts* opts, void* U, int64_t ldu, double* lambda, double* ext_E,
                void* workspace, size_t workspace_bytes, int32_t* dev_status, rpc_stream_t stream);

/* ---- Nystrom extension to new points ----------------------------------
 * For each row y of Y (M x d float32, row-major, same d and eps as X):
 * f(y) = F(S, :)^{-1} k(X_S, y) with S the accepted pivots (F(S, :) is lower
 * triangular in pivot order), d~(y) = c^T f(y), and
 * Phi(y, :) = f(y)^T E / d~(y).  At a training point this reproduces the row
 * of U.  Phi is column-major M x nev float64. */
int nystrom_extend_workspace_size(int64_t M, int64_t d, int32_t r, int32_t nev, size_t* bytes);
int nystrom_extend(const rpc_points* Y, const rpc_points* X, const int64_t* pivots,
                   const int32_t* k, const void* F, int32_t f_dtype, int64_t ldf, int32_t r,
                   const double* c, const double* ext_E, int32_t nev, double* Phi, int64_t ldphi,
                   void* workspace, size_t workspace_bytes, int32_t* dev_status,
                   rpc_stream_t stream);

/* ---- Nystrom extension for the symmetric normalisation -----------------
 * The eigenvectors of L~ = D~^{-1/2} K~ D~^{-1/2} (bistoch_eig with
 * normalization RPC_SYMMETRIC) at new points, from L~ U = U Lambda and the
 * Nystrom extension of the section "Nystrom method connection":
 * Phi(y, :) = f(y)^T E / sqrt(d~(y)), f(y) = F(S, :)^{-1} k(X_S, y),
 * d~(y) = c^T f(y), E = R^T V Lambda^{-1} (the ext_E of that call).  At a
 * training point it reproduces the row of U.  Arguments, layouts, workspace
 * (nystrom_extend_workspace_size) and errors as nystrom_extend. */
int nystrom_extend_symmetric(const rpc_points* Y, const rpc_points* X, const int64_t* pivots,
                             const int32_t* k, const void* F, int32_t f_dtype, int64_t ldf,
                             int32_t r, const double* c, const double* ext_E, int32_t nev,
                             double* Phi, int64_t ldphi, void* workspace, size_t workspace_bytes,
                             int32_t* dev_status, rpc_stream_t stream);

/* ---- Algorithm 1 from the low-memory factor ------------------------------
 * The whole of Algorithm 1 (bistoch_degrees then bistoch_eig) for a factor
 * from rpchol_factor with RPC_FACTOR_LOW_MEMORY, which keeps only
 * FS = F(S, :) (r x r float64, row i = pivot i, leading dimension ldfs >= r;
 * entries with an index >= k are ignored).  The N x r factor is never
 * stored: F F^T interpolates K on the pivots, so every row follows from the
 * points as F(x, :) = K(x, X_S) FS^{-T} (the appendix on randomly pivoted
 * Cholesky and its low-memory remark), and each pass over the factor
 * recomputes it block by block, block_rows rows at a time (0: 65536; else a
 * multiple of 8192, at least r unless N is smaller): an MFMA distance
 * product with an exp epilogue and a product with FS^{-T}.  Five passes:
 * c; d~ and w; q~; the two Grams; U.  Memory O(N (d + nev) + r^2 +
 * block_rows (r + d)) beyond the points.  Float64 throughout.  X is the
 * points and bandwidth of the factorisation; pivots and k as it returned.
 * Options as bistoch_eig with gram_dtype RPC_F64 and qr_mode RPC_QR_CHOLQR
 * (the second pass of Cholesky QR2 needs Q1 = B R1^{-1}, an N x r matrix):
 * others give RPC_EINVAL.  Outputs as bistoch_degrees (c, d_tilde, q_tilde;
 * q_tilde may be NULL with the symmetric normalisation) and bistoch_eig (U,
 * lambda, ext_E); device-side failures as those two calls report them. */
int bistoch_lowmem_workspace_size(const rpc_points* X, int32_t r, const rpc_eig_opts* opts,
                                  int64_t block_rows, size_t* bytes);
int bistoch_lowmem(const rpc_points* X, const int64_t* pivots, const int32_t* k, const double* FS,
                   int64_t ldfs, int32_t r, const rpc_eig_opts* opts, int64_t block_rows,
                   double* c, double* d_tilde, double* q_tilde, void* U, int64_t ldu,
                   double* lambda, double* ext_E, void* workspace, size_t workspace_bytes,
                   int32_t* dev_status, rpc_stream_t stream);

/* ---- Nystrom extension from the low-memory factor -------------------------
 * nystrom_extend (normalization RPC_BISTOCHASTIC) or nystrom_extend_symmetric
 * (RPC_SYMMETRIC) with F(S, :) given directly as FS (r x r float64, row i =
 * pivot i, ldfs >= r), as rpchol_factor returns it with
 * RPC_FACTOR_LOW_MEMORY; c and ext_E from bistoch_lowmem.  Workspace
 * nystrom_extend_workspace_size; other arguments and errors as
 * nystrom_extend. */
int nystrom_extend_lowmem(const rpc_points* Y, const rpc_points* X, const int64_t* pivots,
                          const int32_t* k, const double* FS, int64_t ldfs, int32_t r,
                          const double* c, const double* ext_E, int32_t nev, int32_t normalization,
                          double* Phi, int64_t ldphi, void* workspace, size_t workspace_bytes,
                          int32_t* dev_status, rpc_stream_t stream);

/* ---- Batched form: many independent decompositions ----------------------
 * A job is one full decomposition of its own points (rpchol_factor, then
 * bistoch_degrees, then bistoch_eig, exactly as the three calls made one
 * after the other) with its own output buffers, all device memory owned by
 * the caller.  Small problems cannot fill the chip one at a time, so
 * rpc_batched_run forks `stream` onto n_streams (1..32) internal streams
 * (created on first use per device, default priority, kept until the process
 * ends; HIP maps them onto GPU_MAX_HW_QUEUES hardware queues, four unless the
 * process sets that variable before HIP starts),
 * assigns the jobs longest-first (estimated N r (2 d + 3 r)) to the stream
 * with the least assigned work, and joins them back into `stream`.  Jobs on
 * one stream run in sequence and share one slice of the workspace.  Each
 * job's dev_status is cleared when the job starts.  Results equal those of
 * the single calls bit for bit.  On a host-side error the jobs issued before
 * it still run and the first error is returned.
 *
 * rpc_batched_graph_create captures the same issue into a HIP graph (stream
 * must not be the null stream; profiling must be off); every launch of the
 * graph recomputes all jobs from their current inputs.  Buffers named in the
 * job table must stay valid while the graph exists. */
typedef struct {
  rpc_points X;           /* points and bandwidth */
  rpc_factor_opts factor; /* rank budget, block size, mode, dtypes, uniforms */
  rpc_eig_opts eig;       /* nev, gamma, fix_const, dtypes */
  void* F;                /* N x r, column-major, ldf (multiple of 8, >= N) */
  int64_t ldf;
  int64_t* pivots;        /* r */
  double* rho;            /* N */
  int32_t* k;             /* 1 */
  double* c;              /* r */
  double* d_tilde;        /* N */
  double* q_tilde;        /* N */
  void* U;                /* N x nev, column-major, ldu */
  int64_t ldu;
  double* lambda;         /* nev */
  double* ext_E;          /* r x nev */
  int32_t* dev_status;    /* 1, required */
} rpc_job;

typedef struct rpc_graph_s* rpc_graph;

int rpc_job_workspace_size(const rpc_job* job, size_t* bytes);
int rpc_batched_workspace_size(const rpc_job* jobs, int32_t n_jobs, int32_t n_streams,
                               size_t* bytes);
int rpc_batched_run(const rpc_job* jobs, int32_t n_jobs, int32_t n_streams, void* workspace,
                    size_t workspace_bytes, rpc_stream_t stream);
int rpc_batched_graph_create(const rpc_job* jobs, int32_t n_jobs, int32_t n_streams,
                             void* workspace, size_t workspace_bytes, rpc_stream_t stream,
                             rpc_graph* graph);
int rpc_batched_graph_launch(rpc_graph graph, rpc_stream_t stream);
int rpc_batched_graph_destroy(rpc_graph graph);

/* Any rpc_graph (batched jobs or surrogate training epochs): launch on
 * `stream` (stream-ordered; the graph's work runs after what precedes it on
 * the stream), or destroy (the handle is invalid afterwards). */
int rpc_graph_launch(rpc_graph graph, rpc_stream_t stream);
int rpc_graph_destroy(rpc_graph graph);

/* Block-size autotuning: runs the job once untimed and `reps` times timed
 * (HIP events on `stream`, synchronising) for each candidate block size b
 * (the job's own b is ignored), writes the mean milliseconds to ms[i] (if
 * non-NULL) and the fastest candidate to *best_b.  Overwrites the job's
 * outputs; the workspace must cover every candidate. */
int rpc_autotune_block(const rpc_job* job, const int32_t* candidates, int32_t n_candidates,
                       int32_t reps, void* workspace, size_t workspace_bytes, rpc_stream_t stream,
                       int32_t* best_b, double* ms);

/* ---- Learned surrogate of the Nystrom extension -------------------------
 * The Nystrom extension above maps a new state y to the values of the
 * approximate eigenvectors at y.  The surrogate is a multilayer perceptron
 * trained to reproduce sqrt(N) U (eigenfunction values of order one) at the
 * training states:
 *     z1 = W1 x + b1, a1 = gelu(z1), z2 = W2 a1 + b2, a2 = gelu(z2),
 *     y  = W3 a2 + b3 (n_out outputs),  res = wr . a2 + br,
 * with x the state standardised per feature, gelu(t) = t Phi(t) (exact erf
 * form, Hendrycks & Gimpel 2016), and res a predicted log10 of the RMS error
 * of y against the exact extension, used to fall back to nystrom_extend per
 * point.  Products run on bf16 MFMA with fp32 accumulation: the standardised
 * input, the weights, the hidden activations and the back-propagated errors
 * are rounded to bf16; biases, pre-activations, the loss and the optimiser
 * state stay fp32.  Training: mean squared error over batch and outputs,
 * AdamW (Loshchilov & Hutter 2019; decoupled decay on every trained entry,
 * bias-corrected moments).  Phase 0 trains W1..b3 against the targets;
 * phase 1 trains only the residual head (wr, br) against log10 RMS errors.
 *
 * Parameter vector (float32, caller-owned, sur_layout offsets, each a
 * multiple of 64 elements): W1 h x d row-major, b1 (h), W2 h x h, b2 (h),
 * W3 n3 x h with n3 = n_out + 1 rounded up to 16 (rows 0..n_out-1: output
 * layer; row n_out: wr; the rest zero), b3 (n3; entry n_out is br).  The
 * AdamW moments m and v use the same layout; `wbf16` holds the bf16 copy of
 * the parameter vector (same offsets) that the products read. */
typedef struct {
  int32_t d;     /* input width, 8 <= d <= 4096, multiple of 8 */
  int32_t h;     /* hidden width, 64 <= h <= 4096, multiple of 64 */
  int32_t n_out; /* outputs, 1 <= n_out <= 255 */
} sur_shape;

typedef struct {
  int64_t W1, b1, W2, b2, W3, b3; /* element offsets into the parameter vector */
  int64_t total;                  /* elements of the vector (and of m, v, wbf16) */
  int32_t n3;                     /* rows of W3 (output layer + residual head + zero pad) */
} sur_layout;

typedef struct {
  double lr, beta1, beta2, eps, weight_decay; /* AdamW hyper-parameters */
  int64_t step;   /* AdamW step number t >= 1, counted per phase */
  int32_t phase;  /* 0: W1..b3 on the targets; 1: residual head only */
  int32_t splits; /* batch splits of the weight-gradient sums, 1..64 (0 = 8) */
} sur_train_opts;

/* Host only.  RPC_EINVAL for a shape outside the limits above. */
int surrogate_layout(const sur_shape* shape, sur_layout* out);

/* Initialisation.  With `uniforms` (device doubles in [0, 1), at least
 * surrogate_init_uniforms() of them; fewer: RPC_EINVAL) every weight and bias
 * becomes (2 u - 1) / sqrt(fan_in), u taken in the order W1, b1, W2, b2, W3,
 * b3, wr, br (row-major within a matrix); with uniforms == NULL `params`
 * already holds the initial values.  Pad entries are zeroed, both AdamW
 * moments zeroed and the bf16 copy written. */
int surrogate_init_uniforms(const sur_shape* shape, int64_t* count);
int surrogate_init(const sur_shape* shape, const double* uniforms, int64_t n_uniforms,
                   float* params, float* adam_m, float* adam_v, uint16_t* wbf16,
                   rpc_stream_t stream);

/* Per-feature mean and 1/(population standard deviation) of the N x d
 * float32 rows X (row-major, ldx >= d), in float64 (two passes); a constant
 * feature gets scale 1. */
int surrogate_standardize_workspace_size(int64_t N, int64_t d, size_t* bytes);
int surrogate_standardize(const float* X, int64_t N, int64_t d, int64_t ldx, double* mean,
                          double* rstd, void* workspace, size_t workspace_bytes,
                          rpc_stream_t stream);

/* One AdamW step on the batch rows idx[0..batch) (device int64, each in
 * [0, N) of X; out-of-range indices set RPC_EINVAL in *dev_status and leave
 * the step's outputs undefined).  Targets: phase 0, target(b, j) =
 * tscale * T[idx[b] + j ldt] for j < n_out (column-major, t_dtype F32 or
 * F64, e.g. U of bistoch_eig with tscale = sqrt(N)); phase 1, target(b) =
 * T[idx[b]] (per-point log10 RMS error).  Updates params, adam_m, adam_v and
 * wbf16 in place.  Optional outputs (NULL to skip): grad (float32, parameter
 * layout: the summed gradient of the step, zero for entries the phase does
 * not train) and loss (one device double: the batch loss before the step).
 * 1 <= batch <= 65536. */
int surrogate_train_workspace_size(const sur_shape* shape, int64_t batch, int32_t splits,
                                   size_t* bytes);
int surrogate_train_step(const sur_shape* shape, const sur_train_opts* opts, const float* X,
                         int64_t ldx, int64_t N, const double* mean, const double* rstd,
                         const int64_t* idx, int64_t batch, const void* T, int32_t t_dtype,
                         int64_t ldt, double tscale, float* params, float* adam_m,
                         float* adam_v, uint16_t* wbf16, float* grad, double* loss,
                         void* workspace, size_t workspace_bytes, int32_t* dev_status,
                         rpc_stream_t stream);

/* ceil(n_idx / batch) steps of surrogate_train_step over consecutive slices
 * of idx (the last one ragged), with step numbers opts->step, opts->step + 1,
 * ...; loss, if non-NULL, receives one device double per step.  The
 * workspace is that of surrogate_train_step for `batch`. */
int surrogate_train_epoch(const sur_shape* shape, const sur_train_opts* opts, const float* X,
                          int64_t ldx, int64_t N, const double* mean, const double* rstd,
                          const int64_t* idx, int64_t n_idx, int64_t batch, const void* T,
                          int32_t t_dtype, int64_t ldt, double tscale, float* params,
                          float* adam_m, float* adam_v, uint16_t* wbf16, double* loss,
                          void* workspace, size_t workspace_bytes, int32_t* dev_status,
                          rpc_stream_t stream);

/* One training epoch captured as a graph: the launches of
 * surrogate_train_epoch (ceil(n_idx / batch) AdamW steps over consecutive
 * slices of idx) recorded once; each rpc_graph_launch runs one more epoch on
 * the current contents of every buffer named here (rewrite idx in place with
 * the next epoch's permutation between launches).  The AdamW step number is
 * read from and advanced in device memory: step_counter (int64) holds the
 * number of steps taken so far in this phase and grows by one per step, so
 * every launch continues the bias correction where the last one stopped;
 * o->step is ignored.  Replays equal surrogate_train_epoch calls bit for bit.
 * stream must not be the null stream and profiling must be off (RPC_EINVAL);
 * other arguments as surrogate_train_epoch.  For callers whose training is
 * launch-bound (one step is about ten small launches). */
int surrogate_train_graph_create(const sur_shape* shape, const sur_train_opts* opts,
                                 const float* X, int64_t ldx, int64_t N, const double* mean,
                                 const double* rstd, const int64_t* idx, int64_t n_idx,
                                 int64_t batch, const void* T, int32_t t_dtype, int64_t ldt,
                                 double tscale, float* params, float* adam_m, float* adam_v,
                                 uint16_t* wbf16, double* loss, int64_t* step_counter,
                                 void* workspace, size_t workspace_bytes, int32_t* dev_status,
                                 rpc_stream_t stream, rpc_graph* graph);

/* Forward pass over the M rows of Y (float32 row-major, ldy >= d): Phi (M x
 * n_out float32, column-major, ldphi >= M) and, if non-NULL, res (M float32,
 * the residual head).  Rows are processed in chunks of at most 65536. */
int surrogate_infer_workspace_size(const sur_shape* shape, int64_t M, size_t* bytes);
int surrogate_infer(const sur_shape* shape, const float* params, const uint16_t* wbf16,
                    const float* Y, int64_t ldy, int64_t M, const double* mean,
                    const double* rstd, float* Phi, int64_t ldphi, float* res, void* workspace,
                    size_t workspace_bytes, int32_t* dev_status, rpc_stream_t stream);

/* Residual-head targets for phase 1: out[m] = log10 of the RMS over j <
 * n_out of Phi_s(m, j) - scale * Phi_n(m, j) (Phi_s float32 and Phi_n
 * float64, both column-major); out is float64.  A zero difference gives
 * log10 of the smallest normal double, -307.65. */
int surrogate_residual_target(const float* Phi_s, int64_t lds, const double* Phi_n,
                              int64_t ldn, double scale, int64_t M, int32_t n_out, double* out,
                              rpc_stream_t stream);

/* Hybrid extension: the surrogate everywhere, then the exact Nystrom
 * extension (scaled by `scale`, normally sqrt(N)) at the points whose
 * residual head predicts res > log10_threshold.  The surrogate's n_out must
 * not exceed nev.  Synchronises `stream` once (to size the fallback set);
 * *n_fallback (host) receives its size.  The workspace covers both parts. */
int surrogate_extend_workspace_size(const sur_shape* shape, int64_t M, int64_t d, int32_t r,
                                    int32_t nev, size_t* bytes);
int surrogate_extend(const sur_shape* shape, const float* params, const uint16_t* wbf16,
                     const double* mean, const double* rstd, double log10_threshold,
                     const rpc_points* Y, const rpc_points* X, const int64_t* pivots,
                     const int32_t* k, const void* F, int32_t f_dtype, int64_t ldf, int32_t r,
                     const double* c, const double* ext_E, int32_t nev, double scale,
                     float* Phi, int64_t ldphi, float* res, int64_t* n_fallback,
                     void* workspace, size_t workspace_bytes, int32_t* dev_status,
                     rpc_stream_t stream);

/* ---- Per-kernel timing (diagnostics for benchmarking) ------------------
 * When enabled, the library brackets each launch of its main kernel classes
 * with HIP events on the launching stream.  rpc_profile_read synchronises on
 * the recorded events and returns, for one class, the summed duration in ms
 * and the number of launches since the last reset.  Classes: 0 kernel
 * columns, 1 Schur update, 2 triangular solve + downdate, 3 pivot draw,
 * 4 pivot block + accept/reject, 5 degrees, 6 Gram partial products,
 * 7 r x r work (Gram row scales, chunk reduction and finish, Cholesky, inner
 * product), 8 eigenvector formation, 9 Nystrom extension, 10 inner
 * eigensolver, 11 surrogate training step, 12 surrogate inference.
 * Process-global state, not
 * thread-safe; returns RPC_EWORKSPACE if the event pool overflowed. */
int rpc_profile_enable(int on);
int rpc_profile_reset(void);
int rpc_profile_read(int32_t kind, double* total_ms, int64_t* launches);

/* Synchronise `stream` and return the device status word (or RPC_EHIP). */
int rpc_status_sync(const int32_t* dev_status, rpc_stream_t stream);

/* Library version string. */
const char* rpc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RPCHOL_H_ */
