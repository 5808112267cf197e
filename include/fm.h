/*
 * fm.h -- C ABI of the structured linear operator library (MI355X, gfx950).
 *
 * A linear operator A (m x n) is applied forward, y = A x (the forward
 * transform of eq. (3)), or backward, x = A^H y (the backward transform of
 * eq. (4)), to a block of column vectors at once, as in the paper's section
 * "Software description" (operators act on arrays of several vectors, and the
 * number of vectors processed together is a calibration parameter there).
 *
 * Conventions that hold for every entry point:
 *
 *  - Blocks are column-major: column j of a block with leading dimension ld
 *    starts at ptr + j*ld elements; ld >= rows. In PyTorch terms a block is a
 *    contiguous tensor of shape (ncols, rows).
 *  - Data pointers are DEVICE pointers on the current HIP device, in the
 *    operator's element type: FM_C64 = interleaved float (re, im),
 *    FM_C128 = interleaved double, FM_I32 = int32_t, FM_I64 = int64_t.
 *  - Operators are immutable once created (section "General Matrix-free
 *    Representations": precomputations stay valid only because instances never
 *    change). Handles are reference counted; fm_op_compose and fm_op_adjoint
 *    retain their children, so callers may release children afterwards.
 *  - Creation copies every parameter array (the caller may free it on return)
 *    and performs the precomputation (spectra, twiddle tables) on `stream`;
 *    creation synchronises that stream before it returns.
 *  - fm_apply enqueues kernels on `stream` and returns without synchronising.
 *    It allocates nothing when a large enough workspace is passed.
 *  - Every entry point validates its arguments first and returns a status
 *    before anything is enqueued. On error, fm_last_error() describes it.
 *    Device faults surface as FM_E_DEVICE at the next synchronising call.
 *  - Streams are passed as `void*` holding a hipStream_t (NULL: the null
 *    stream), so this header does not depend on the HIP headers.
 */
#ifndef FM_H
#define FM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fm_op_s* fm_op;
typedef struct fm_batch_s* fm_batch;

typedef enum { FM_C64 = 1, FM_C128 = 2, FM_I32 = 3, FM_I64 = 4 } fm_dtype;

/* FM_FWD: y = A x (eq. 3).  FM_ADJ: y = A^H x (eq. 4). */
typedef enum { FM_FWD = 0, FM_ADJ = 1 } fm_dir;

typedef enum { FM_PRODUCT = 0, FM_SUM = 1, FM_KRON = 2, FM_BLKDIAG = 3 } fm_compose_kind;

typedef enum {
  FM_OK = 0,
  FM_E_INVALID = 1,     /* NULL handle/pointer, non-positive size, bad enum  */
  FM_E_SHAPE = 2,       /* inconsistent shapes, ld < rows, index out of range */
  FM_E_DTYPE = 3,       /* dtype mismatch or not supported by this operator  */
  FM_E_ALIAS = 4,       /* x and y overlap                                    */
  FM_E_UNSUPPORTED = 5, /* valid request the library does not implement       */
  FM_E_WORKSPACE = 6,   /* workspace given but smaller than fm_workspace_size */
  FM_E_NOMEM = 7,       /* device allocation failed                           */
  FM_E_DEVICE = 8,      /* HIP runtime error (launch failure, device fault)   */
  FM_E_RELEASED = 9     /* handle already released                            */
} fm_status;

/* ------------------------------------------------------------------ creation
 * Parameter arrays are device pointers in dtype `dt`.
 */

/* Unnormalised DFT matrix F_n, F[i,k] = exp(-2 pi j i k / n), eq. (1) read with
 * 0-based indices. 1 <= n <= 2^20 for powers of two (Stockham transforms);
 * other n up to 2^19 through Bluestein's identity F = D T D, with
 * D = diag(exp(-pi j i^2 / n)) and the Toeplitz T[i,k] = exp(pi j (i-k)^2 / n)
 * (chirps from FP64 with exact angle reduction). Complex dtypes; the
 * non-power-of-two form allocates device memory and synchronises. */
fm_status fm_op_create_fourier(fm_op* out, int64_t n, fm_dtype dt);

/* Walsh-Hadamard matrix H_n in natural (Sylvester) order, entries +-1,
 * H[i,j] = (-1)^popcount(i AND j); n a power of two. All four dtypes; integer
 * results wrap modulo 2^32 / 2^64 (two's complement), so they are exact and
 * independent of the order of additions. */
fm_status fm_op_create_hadamard(fm_op* out, int64_t n, fm_dtype dt);

/* Diag(d), n x n with d on the diagonal (the Diag factor of eq. (7)).
 * Complex dtypes. */
fm_status fm_op_create_diag(fm_op* out, int64_t n, const void* d, fm_dtype dt, void* stream);

/* Dense m x n matrix, column-major with leading dimension lda >= m (the plain
 * product of eq. (2)); used mainly as a Kronecker factor. Complex dtypes.
 * complex64 products of at most 64 x 64 with 64 or more vectors run on the
 * matrix cores (FM_DENSE_MFMA=0 keeps them on the vector units). */
fm_status fm_op_create_dense(fm_op* out, int64_t m, int64_t n, const void* a, int64_t lda,
                             fm_dtype dt, void* stream);

/* Circulant C(c): y = c cyclically convolved with x (eq. (5)), c = first column,
 * C[i,j] = c[(i-j) mod n]. The spectrum DFT(c) is computed once here in FP64
 * (section "General Matrix-free Representations": FFT(c) is precomputed at
 * initialisation). 1 <= n <= 2^20 for powers of two; other n up to 2^19 are
 * created as the n x n Toeplitz with first column c and first row
 * (c_0, c_{n-1}, ..., c_1), applied through its power-of-two embedding (the
 * handle then behaves as a Toeplitz: no fused Gramian or inverse).
 * Complex dtypes. */
fm_status fm_op_create_circulant(fm_op* out, int64_t n, const void* c, fm_dtype dt, void* stream);

/* Circulant whose generator is the +-1 output of a linear feedback shift
 * register (the LFSR circulant of the operator zoo): `order` bits, taps and a
 * nonzero start state in the low `order` bits. Step k outputs s_k = +1 when
 * bit 0 of the register is 0 and -1 when it is 1, then shifts the register
 * right by one and sets bit order-1 to the parity of (register & taps) taken
 * before the shift, i.e. bit i of the register holds s_{k+i} and
 * s_{k+order} = XOR of s_{k+i} over the set bits i of taps. c = (s_0, ...,
 * s_{n-1}), n = 2^order - 1 (the period when x^order + sum_{i in taps} x^i is
 * primitive). 2 <= order <= 19. Complex dtypes. */
fm_status fm_op_create_lfsr_circulant(fm_op* out, int32_t order, uint64_t taps, uint64_t state, fm_dtype dt,
                                      void* stream);

/* Toeplitz m x n (a non-circular convolution): T[i,j] = col[i-j] for i >= j,
 * row[j-i] for i < j. col has m entries and defines the diagonal; row has n
 * entries and row[0] is ignored. Applied through a cyclic convolution of length
 * L with zero padding and cropping (the embedding described for eq. (7)); L is
 * the smallest length >= m + n - 1 among the powers of two and, above 4096,
 * 4096 * n2 for n2 in {3, 5, 6, 9, 10, 12, 20, 24, 30} (any L >= m + n - 1
 * gives the same matrix; these lengths waste less than the next power of two
 * and have fast transforms here); the environment variable FM_EMBED=pow2 keeps
 * powers of two. m + n - 1 <= 2^20. Complex dtypes. */
fm_status fm_op_create_toeplitz(fm_op* out, int64_t m, int64_t n, const void* col,
                                const void* row, fm_dtype dt, void* stream);

/* Multilevel (block-) Toeplitz of `levels` levels with n_per_level[l] entries
 * per level (square, size prod n_l), the 2-level structure of the blocks H_ij
 * of eq. (7). t holds prod(2 n_l - 1) values, row-major (last level fastest),
 * offset o_l at index o_l + n_l - 1:
 *   T[(i_1..i_d),(j_1..j_d)] = t[i_1-j_1, ..., i_d-j_d].
 * 1 <= levels <= 3. Complex dtypes. */
fm_status fm_op_create_mltoeplitz(fm_op* out, int32_t levels, const int64_t* n_per_level,
                                  const void* t, fm_dtype dt, void* stream);

/* Row selection S (m x n_in), S[r, idx[r]] = 1 (the Partial operator, and the
 * row selections of Psi in eq. (9)). idx: DEVICE int32 array of m distinct
 * indices in [0, n_in); validated here (FM_E_SHAPE on a duplicate or an index
 * out of range). Forward gathers; the adjoint writes every one of the n_in
 * outputs once, through an inverse index map the handle keeps (n_in int32,
 * -1 for rows not selected), with zeros where no row is selected. All dtypes. */
fm_status fm_op_create_select_rows(fm_op* out, int64_t n_in, int64_t m, const int32_t* idx,
                                   fm_dtype dt, void* stream);

/* Composite of `nterms` operators, all of one dtype (section "General
 * Matrix-free Representations": composites are applied only through their
 * terms' transforms):
 *   FM_PRODUCT  terms[0] * terms[1] * ... (applied right to left),
 *   FM_SUM      terms[0] + terms[1] + ... (equal shapes),
 *   FM_KRON     terms[0] (x) terms[1] (x) ... (first factor slowest, eq. (7)),
 *   FM_BLKDIAG  block diagonal of the terms (the BlkDiag of eq. (9)).
 * Retains the terms. */
fm_status fm_op_compose(fm_op* out, fm_compose_kind kind, int32_t nterms, const fm_op* terms);

/* Block matrix H = [A_ij], i < nbr, j < nbc: the N1 x N1 block structure of
 * the ultrasound model (section "Application to Ultrasonic Nondestructive
 * Testing", the block matrix of eq. (6)'s H with 2-level Toeplitz blocks of
 * eq. (7), and the Blocks operator of the listing next to it).
 * terms: nbr * nbc handles, row-major (terms[i * nbc + j] = A_ij), one dtype;
 * every block of a block row has the same number of rows, every block of a
 * block column the same number of columns (FM_E_SHAPE otherwise). A handle may
 * appear several times. Forward y_i = sum_j A_ij x_j, adjoint
 * x_j = sum_i A_ij^H y_i, where x_j / y_i are the row slices of the columns.
 * When every block is a multilevel Toeplitz of one geometry, each input slice
 * is transformed once, the blocks are mixed per frequency bin and each output
 * slice is transformed back once (2 (nbr + nbc) transforms instead of
 * 2 nbr nbc). Retains the terms. */
fm_status fm_op_create_blocks(fm_op* out, int32_t nbr, int32_t nbc, const fm_op* terms);

/* Hermitian transpose A^H as an operator (shares A's storage, retains A). */
fm_status fm_op_adjoint(fm_op* out, fm_op a);

/* Shape (m rows, n columns) and dtype of an operator. Any pointer may be NULL. */
/* Views and derived operators of the base-class feature table (section
 * "General Matrix-free Representations": transpose, Hermitian transpose,
 * complex conjugate, Gramian, inverse). Each returns a new immutable handle
 * that retains what it is built from.
 *   fm_op_conj:    conj(A), applied as conj(A conj(x)); the transpose is
 *                  fm_op_adjoint of it (A^T = conj(A)^H). Integer operators
 *                  are their own conjugates.
 *   fm_op_gram:    A^H A. Built from the structure where one exists: a
 *                  circulant gives the circulant of spectrum |c_hat|^2 (one
 *                  convolution), Fourier and Hadamard give n I, a diagonal
 *                  diag(|d|^2), a row selection the diagonal of its indices,
 *                  Kron and BlkDiag the Kron / BlkDiag of the terms' Gramians,
 *                  conj(A) conj(A^H A); anything else the product A^H A.
 *                  Complex dtypes.
 *   fm_op_inverse: A^-1 for square operators with a structured inverse:
 *                  Circulant (spectrum 1/c_hat), Diag (1/d), Fourier (F^H / n),
 *                  Hadamard (H / n), square row selections (permutations:
 *                  S^H), square Toeplitz (applied by Levinson recursion,
 *                  O(n^2) per vector, one work-group per vector; a vector
 *                  whose system has a singular leading minor comes out NaN),
 *                  and Kron, BlkDiag, Product, adjoint and conj views of
 *                  those. FM_E_INVALID for a singular circulant or diagonal,
 *                  FM_E_SHAPE for non-square, FM_E_UNSUPPORTED for other kinds.
 *                  Complex dtypes; synchronises the device. */
fm_status fm_op_conj(fm_op* out, fm_op a);
fm_status fm_op_gram(fm_op* out, fm_op a);
fm_status fm_op_inverse(fm_op* out, fm_op a);
/* Run-time calibration of the evaluation path, after the paper's runtime
 * path optimisation (section "Software description": algorithms are timed at
 * run time and the faster one is kept per size and number of vectors). For
 * an operator of at most 64 x 64 (any kind, composites included) the library
 * can apply its structured transforms or a dense product with the
 * operator's matrix, materialised once through the operator's own complex128
 * transforms applied to the identity and rounded once for complex64.
 *   fm_op_calibrate times both paths on ncols columns on `stream` (2 warm-up
 *   and 5 timed applications each, HIP events), keeps the faster for every
 *   later application of this handle and reports both times (ms per
 *   application; any output pointer may be NULL). choice: 0 structured,
 *   1 dense.
 *   fm_op_set_path forces a path (0 or 1).
 * The operator's value does not change (within the precision of either
 * path), only how it is evaluated; calls serialise on a library mutex and
 * synchronise. Complex dtypes; FM_E_UNSUPPORTED above 64 x 64. */
fm_status fm_op_calibrate(fm_op a, int64_t ncols, int32_t* choice, double* ms_fast, double* ms_dense, void* stream);
fm_status fm_op_set_path(fm_op a, int32_t path);

/* Calibration model (the same run-time path optimisation, measured once per
 * device instead of per handle): for three operator classes -- circulant,
 * Toeplitz (square) and Fourier -- in complex64 and complex128, the times of
 * the structured and of the dense evaluation on a grid of sizes n = 8, 16,
 * 32, 48, 64 and column counts 1, 16, 256, 4096, 65536 (the dense product of
 * complex64 runs on the matrix cores when there are 64 vectors or more).
 *   fm_calibration_build measures the grid on the current device with
 *   operators of deterministic test values (synchronises; about a second);
 *   fm_calibration_entries copies the table out (out may be NULL to get the
 *   count; cap: room in out); fm_calibration_load installs a saved table on
 *   the current device (reuse across processes); fm_op_choose_path sets a
 *   handle's path from the model without timing it: the log ratio of the two
 *   times is interpolated bilinearly in (size, log2 ncols) between the grid
 *   points around (max(m, n), ncols), clamped to the grid, and the dense path
 *   is taken where it is negative. FM_E_INVALID without a model,
 *   FM_E_UNSUPPORTED for other kinds (fm_op_calibrate times any kind). */
enum { FM_CAL_CIRCULANT = 0, FM_CAL_TOEPLITZ = 1, FM_CAL_FOURIER = 2 };
typedef struct {
  int32_t cls;      /* FM_CAL_* */
  int32_t dt;       /* FM_C64 or FM_C128 */
  int32_t n;        /* operator size */
  int32_t reserved; /* 0 */
  int64_t ncols;
  double ms_fast;   /* structured transforms, ms per application */
  double ms_dense;  /* dense product, ms per application */
} fm_calib_entry;
fm_status fm_calibration_build(void* stream);
fm_status fm_calibration_entries(fm_calib_entry* out, int32_t cap, int32_t* count);
fm_status fm_calibration_load(const fm_calib_entry* in, int32_t count);
fm_status fm_op_choose_path(fm_op a, int64_t ncols, int32_t* choice);

fm_status fm_op_shape(fm_op a, int64_t* m, int64_t* n, fm_dtype* dt);

/* Cyclic length L the operator's transforms run at (section "Circulant
 * Matrices", eq. (5), and the Toeplitz embedding of eq. (7)): n for Fourier
 * and power-of-two Circulant, the embedding length for Toeplitz (the rule
 * stated at fm_op_create_toeplitz; a Circulant whose size is not a power of
 * two is built as a Toeplitz and reports its embedding; a Fourier whose size
 * is not a power of two runs as D T D with a Toeplitz T and reports T's), 0
 * for every other kind. *L must not be NULL. */
fm_status fm_op_transform_length(fm_op a, int64_t* L);

/* Drops one reference; storage is freed when the last reference goes. */
fm_status fm_op_release(fm_op a);

/* ------------------------------------------------------------------ application */

/* Workspace bytes fm_apply needs for (a, dir, ncols). */
fm_status fm_workspace_size(fm_op a, fm_dir dir, int64_t ncols, size_t* bytes);

/* y = A x (FM_FWD) or y = A^H x (FM_ADJ) for ncols columns.
 * FWD: x is n x ncols (ldx >= n), y is m x ncols (ldy >= m); ADJ swaps m, n.
 * ws/ws_bytes: device workspace of at least fm_workspace_size bytes; with
 * ws == NULL and ws_bytes == 0 the library takes stream-ordered memory
 * (hipMallocAsync/hipFreeAsync) itself. x and y must not overlap (FM_E_ALIAS).
 * ncols == 0 is a no-op. */
fm_status fm_apply(fm_op a, fm_dir dir, int64_t ncols, const void* x, int64_t ldx, void* y,
                   int64_t ldy, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fm_apply
 * with its workspace taken from a fixed array of FM_NOALLOC_SCRATCH_BYTES
 * (64 MiB) that the library holds on every device it runs on until the
 * process ends. Same arguments, layout and results as fm_apply (the same
 * kernels: identical bits). Makes no hipMalloc / hipFree call and no other
 * allocation; the operator's twiddle tables are created with the operator.
 * A call whose workspace (fm_workspace_size) exceeds the array returns
 * FM_E_WORKSPACE before anything is enqueued. The array's device address is
 * looked up on the first call on each device. All calls on one device share
 * that device's array and its contents stay from the last call: calls that
 * overlap in time on one device (different streams or threads without
 * ordering) race on it and must be serialised by the caller. Stream-ordered. */
#define FM_NOALLOC_SCRATCH_BYTES (64u << 20)
fm_status fm_apply_noalloc(fm_op a, fm_dir dir, int64_t ncols, const void* x, int64_t ldx, void* y,
                           int64_t ldy, void* stream);

/* ------------------------------------------------------------------ FISTA / ISTA
 * Per column j of b (each column is its own problem), minimise
 *   1/2 ||A x_j - b_j||_2^2 + lambda_j ||x_j||_1
 * (eq. (8) with the conventional factor 1/2, i.e. tau = 2 lambda), by the
 * constant-step proximal-gradient iteration the paper runs (ISTA) and its
 * accelerated form it cites (FISTA, Beck-Teboulle):
 *   g = A^H (A y_k - b); x_{k+1} = soft(y_k - g/L, lambda/L);
 *   t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2;
 *   y_{k+1} = x_{k+1} + ((t_k - 1)/t_{k+1}) (x_{k+1} - x_k)   (ISTA: y = x).
 * soft() shrinks the complex modulus (|z| <= s gives exactly 0).
 */
typedef struct {
  int32_t max_iters;       /* iterations K (>= 0)                               */
  int32_t momentum;        /* 1 FISTA, 0 ISTA                                   */
  int32_t x0_given;        /* 1: x holds the start x_0 on entry; 0: x_0 = 0     */
  int32_t power_max_iters; /* power iteration cap when L <= 0 (e.g. 500)        */
  double lambda_abs;       /* > 0: lambda_j = lambda_abs for every column       */
  double lambda_rel;       /* used when lambda_abs <= 0:
                              lambda_j = lambda_rel * ||A^H b_j||_inf           */
  double L;                /* > 0: step constant; <= 0: FP64 power iteration    */
  double stop_tol;         /* > 0: freeze column j after the first k with
                              ||x_k - x_{k-1}|| <= stop_tol * ||x_k||; 0: fixed K */
  double power_tol;        /* relative change that ends the power iteration     */
  uint64_t seed;           /* start vector of the power iteration (SplitMix64)  */
} fm_fista_opts;

typedef struct {
  int32_t iters_done;  /* iterations applied to this column                     */
  int32_t status;      /* 0 ok, 1 non-finite values met (column frozen)         */
  double L_used;       /* step constant used                                    */
  double lambda_used;  /* lambda_j used                                         */
} fm_fista_stat;

/* Runs the iteration on `stream`; b is m x ncols, x is n x ncols (output; also
 * the start when x0_given). stats: HOST array of ncols entries, filled after the
 * single synchronisation at the end (may be NULL). Workspace as in fm_apply
 * (size from fm_fista_workspace_size). Complex dtypes.
 * For A = C or A = S C (C a circulant or Toeplitz leaf, S a row selection) the
 * iteration runs in the convolution's own passes, with the residual and the
 * update in their loads and stores, replayed from HIP graphs of 10 iterations
 * (A = S C with one or two columns and a power-of-two C of length >= 65536:
 * with 1024-point rows in the four-step split instead of 4096);
 * other operators run the general loop (products through fm_apply's executor,
 * then the update). Environment: FM_FISTA_FUSED=0 sends every operator through
 * the general loop; FM_FISTA_GRAPH=k captures k iterations per graph (0: direct
 * launches); FM_FISTA_NARROW=0 keeps 4096-point rows. All forms give the same
 * iterates up to rounding. */
fm_status fm_fista(fm_op a, int64_t ncols, const void* b, int64_t ldb, void* x, int64_t ldx,
                   const fm_fista_opts* opts, fm_fista_stat* stats, void* ws, size_t ws_bytes,
                   void* stream);
fm_status fm_fista_workspace_size(fm_op a, int64_t ncols, const fm_fista_opts* opts, size_t* bytes);

/* L = ||A||_2^2 by power iteration on A^H A in complex128 (FP64) whatever the
 * operator's dtype: v <- v/||v||, repeat w = A^H A v, L_k = ||A v||^2,
 * v <- w/||w|| until |L_k - L_{k-1}| <= tol * L_k or max_iters. v0: DEVICE
 * complex128 start vector of n entries, or NULL for the SplitMix64 vector of
 * `seed` (entry i = (u(2i) - 1/2) + j (u(2i+1) - 1/2), u(k) the k-th SplitMix64
 * output of `seed` scaled to [0,1) by its top 53 bits). Synchronises `stream`
 * once every 16 iterations (the stopping test is applied to every iteration
 * in order from a device history of the norms; iterations past the stop are
 * discarded); the chunks of 16 after the first replay one HIP graph captured
 * per call (direct launches under FM_FISTA_GRAPH=0; the same bits either way).
 * For A = S C (C a circulant or Toeplitz of power-of-two length >= 65536, S a
 * row selection) the products run through fm_fista's passes with 1024-point
 * rows (FM_FISTA_FUSED=0 or FM_FISTA_NARROW=0: through fm_apply's executor).
 * iters_out may be NULL. */
fm_status fm_power_iteration(fm_op a, const void* v0, uint64_t seed, int32_t max_iters, double tol,
                             double* L_out, int32_t* iters_out, void* stream);

/* Orthogonal matching pursuit, the greedy sparse recovery the paper runs
 * beside FISTA on the ultrasound model (section "Application to Ultrasonic
 * Nondestructive Testing"), per column b_j of b (each column one problem):
 * k times (or until ||r|| <= tol ||b_j||): c = A^H r, pick the unchosen index
 * of largest |c_i| (first on ties; correlations are not normalised by column
 * norms), solve the least-squares problem on the chosen columns, r = b - A x.
 * The least squares are kept as A_S = Q R (Gram-Schmidt applied twice against
 * the chosen columns) and solved by back substitution at the end.
 * x (n x ncols, ldx): the solution, zero outside the support. support: DEVICE
 * int32 array of ncols * k entries (column j at support + j*k, atoms in
 * selection order, -1 after the last) or NULL. stats: HOST array of ncols
 * entries or NULL; status 0 ok, 1 non-finite value, 2 stopped early because
 * the chosen column depends on the earlier ones (that atom is not kept).
 * 1 <= k <= min(m, n, 1024). Workspace as for fm_fista (size from
 * fm_omp_workspace_size; NULL and 0: allocated on the stream). Synchronises
 * `stream` when stats is given. Complex dtypes. */
typedef struct {
  int32_t atoms;    /* chosen atoms kept */
  int32_t status;
  double res_norm;  /* ||b - A x||_2 at the end */
} fm_omp_stat;
fm_status fm_omp(fm_op a, int64_t ncols, const void* b, int64_t ldb, int32_t k, double tol, void* x, int64_t ldx,
                 int32_t* support, fm_omp_stat* stats, void* ws, size_t ws_bytes, void* stream);
fm_status fm_omp_workspace_size(fm_op a, int64_t ncols, int32_t k, size_t* bytes);

/* ------------------------------------------------------------------ batching
 * Many independent Circulant / Toeplitz operators of uneven sizes applied
 * together (the batch-of-operators extension of the per-column evaluation of
 * Sec. 2). At creation the library cuts every transform into 4096-value work
 * items and lays them out in a software-pipelined sequence of kernel launches
 * ("stages"): operators whose embedding length is <= 4096 take one item per
 * column; longer ones take three passes of a four-step split, chunked so
 * that the intermediate buffers of three chunks in flight stay in a fixed
 * device pool. One direction is a few stage launches on `stream`, with no
 * host synchronisation and no waits between workgroups; after its first use
 * with a given set of pointers the sequence is replayed from a captured HIP
 * graph (FM_BATCH_GRAPH=0 disables capture). ops: composite-free
 * Circulant or Toeplitz operators of one complex dtype on the current device;
 * ncols[i] >= 1 columns of operator i. The batch holds references to its
 * operators until fm_batch_release. */
fm_status fm_batch_create(fm_batch* out, int32_t nops, const fm_op* ops, const int64_t* ncols);
/* x[i], y[i]: device blocks of operator i with leading dimensions ldx[i], ldy[i]
 * (host arrays of nops entries). */
fm_status fm_batch_apply(fm_batch b, fm_dir dir, const void* const* x, const int64_t* ldx,
                         void* const* y, const int64_t* ldy, void* stream);
/* FISTA / ISTA for every column of every operator of the batch (opts shared;
 * b[i] is m_i x ncols[i], x[i] is n_i x ncols[i]). With opts->L <= 0 each
 * operator uses max_k |DFT_L(g)_k|^2 of its cyclic embedding, an upper bound
 * of its ||A||_2^2. Columns meeting the stopping rule are frozen and their work
 * is skipped from then on. stats: host array with one entry per column of
 * every operator, in batch order (may be NULL). Synchronises the stream once at
 * the end. */
fm_status fm_batch_fista(fm_batch b, const void* const* bvec, const int64_t* ldb, void* const* x,
                         const int64_t* ldx, const fm_fista_opts* opts, fm_fista_stat* stats,
                         void* stream);
fm_status fm_batch_release(fm_batch b);

/* Schedule of a batch (see fm_batch_tune). */
typedef struct {
  int32_t max_fuse;    /* strided four-step factors up to 2^max_fuse are folded into the row pass */
  int32_t region_mib;  /* slot region of one chunk of four-step columns (three rotate), MiB */
  int32_t graphs;      /* 1: the stage sequence is replayed from captured HIP graphs */
  int32_t stages;      /* kernel launches per direction (output only) */
  double ms;           /* measured milliseconds per direction (fm_batch_tune), else 0 */
} fm_batch_schedule;

/* Autotuner, in the spirit of the paper's run-time calibration (Sec. 2.1):
 * times fm_batch_apply(dir) on the caller's blocks for every candidate
 * schedule (max_fuse 0..5 x slot regions of 24, 48 and 96 MiB), `reps`
 * timed runs each after one warm-up, then times the four fastest and the
 * schedule in use on entry again in two interleaved rounds of 2 * reps runs,
 * and keeps the fastest by each candidate's minimum (a candidate replaces the
 * best so far only when it is more than 1 % faster). The default schedule
 * is (3, 96 MiB). y receives the
 * correct result. Synchronises the device. A schedule whose max_fuse differs
 * from the per-operator path's default (3, FM_MAX_FUSE) computes the same
 * products with a different rounding order, so results then agree with
 * fm_apply to rounding rather than bit for bit. `chosen` may be NULL. */
fm_status fm_batch_tune(fm_batch b, fm_dir dir, const void* const* x, const int64_t* ldx,
                        void* const* y, const int64_t* ldy, int32_t reps, fm_batch_schedule* chosen,
                        void* stream);
/* The batch's current schedule. */
fm_status fm_batch_get_schedule(fm_batch b, fm_batch_schedule* out);
/* Sets the schedule (max_fuse 0..5, region_mib 16..1024; graphs and ms are
 * ignored). Synchronises the device. */
fm_status fm_batch_set_schedule(fm_batch b, const fm_batch_schedule* sc);

/* ------------------------------------------------------------------ differentiation
 * Building blocks of reverse-mode differentiation through operator
 * applications and unrolled FISTA (an extension; the paper has no autodiff).
 * Gradients follow PyTorch's convention for complex tensors: for a real loss
 * and an upstream gradient G of an output s, the gradient of an input z is
 * G conj(ds/dz) + conj(G) ds/dz*. The gradient of x for y = A x is A^H G, so
 * fm_apply in the other direction serves it.
 *
 * Generator of a circulant C(c) (n x n, c its first column; the cyclic
 * convolution y = c (*) x of eq. (5)), summed over the ncols columns:
 *   use = FM_FWD, y = C(c) in:    grad_c[k] (+)= sum_j sum_i g_j[i] conj(in_j[(i-k) mod n])
 *   use = FM_ADJ, w = C(c)^H in:  grad_c[k] (+)= sum_j sum_i in_j[i] conj(g_j[(i-k) mod n])
 * (circular cross-correlations, computed through length-n DFTs and summed over
 * the columns in the frequency domain). in, g: DEVICE blocks of ncols columns
 * of n entries (leading dimensions ld_in, ld_g >= n); grad_c: DEVICE vector of
 * n entries, overwritten (accumulate = 0) or added to; it must not overlap the
 * inputs. n: power of two <= 2^20; complex dtypes. ncols = 0 leaves grad_c
 * unchanged (accumulate) or zeroes it. Takes its own workspace from the
 * stream-ordered allocator (hipMallocAsync / hipFreeAsync on `stream`) and
 * does not wait on the host; the column sum is deterministic (a fixed grouping
 * of the columns, groups added in order). */
fm_status fm_circulant_grad_generator(int64_t n, int64_t ncols, fm_dir use, const void* in,
                                      int64_t ld_in, const void* g, int64_t ld_g, void* grad_c,
                                      int32_t accumulate, fm_dtype dt, void* stream);

/* Momentum weight of FISTA iteration `iter` (0-based: the weight applied
 * after the (iter+1)-th gradient step), the accelerated form of the solver of
 * eq. (8): t_1 = 1, t_{j+1} = (1 + sqrt(1 + 4 t_j^2))/2, beta = (t_{iter+1} - 1)
 * / t_{iter+2} (0 for iter = 0), formed in FP64 by the recurrence; 0 when
 * momentum = 0 (ISTA). The same value fm_fista, fm_batch_fista and
 * fm_fista_step use. beta: HOST output. */
fm_status fm_fista_momentum(int32_t iter, int32_t momentum, double* beta);

/* One proximal-gradient step of the solver of eq. (8) on DEVICE blocks of
 * ncols columns of n entries (all with leading dimension ld), given the
 * gradient g = A^H (A y - b), as iteration `iter` (0-based) of the solve:
 *   z = y - g / L,  x_new = soft(z, lam[j] / L),  y_new = x_new + beta (x_new - x_old)
 * with beta the momentum weight of that iteration (fm_fista_momentum; 0 when
 * momentum = 0). soft(z, s) = z (|z| - s)/|z| for |z| > s, else 0 (complex
 * modulus). lam: DEVICE array of ncols doubles. z_out (may be NULL) receives
 * z. x_new may be x_old and y_new may be y (elementwise in place); x_new, y_new
 * and z_out must not overlap each other. The arithmetic is that of fm_fista's
 * update, so a step recomputed from the same inputs gives the same bits.
 * iter < 0 or L <= 0 is rejected. Stream-ordered. */
fm_status fm_fista_step(int64_t n, int64_t ncols, const void* y, const void* g, const void* x_old,
                        void* x_new, void* y_new, void* z_out, int64_t ld, const double* lam,
                        double L, int32_t iter, int32_t momentum, fm_dtype dt, void* stream);

/* Vector-Jacobian product of fm_fista_step (iteration `iter`, momentum weight
 * beta as there). Given z of the forward step and
 * the upstream gradients gx_new, gy_new of x_new, y_new, with
 * xt = gx_new + (1 + beta) gy_new and s = lam[j]/L:
 *   gz     = xt (1 - s/(2|z|)) + conj(xt) s z^2 / (2 |z|^3)   if |z| > s, else 0
 *   gg     = -gz / L               (gradient of g; may be NULL)
 *   gx_old = -beta gy_new          (gradient of x_old; may be NULL)
 * and the gradient of y is gz (z = y - g/L). gz may be gx_new or gy_new,
 * gg and gx_old may be gx_new or gy_new (elementwise in place); other overlaps
 * are rejected. Same layout rules as fm_fista_step. Stream-ordered. */
fm_status fm_fista_step_vjp(int64_t n, int64_t ncols, const void* z, const void* gx_new,
                            const void* gy_new, void* gz, void* gg, void* gx_old, int64_t ld,
                            const double* lam, double L, int32_t iter, int32_t momentum, fm_dtype dt,
                            void* stream);

/* out = alpha x + beta y on DEVICE blocks (real alpha, beta; complex dtypes).
 * out may be x or y with the same leading dimension. Stream-ordered. */
fm_status fm_axpby(int64_t n, int64_t ncols, double alpha, const void* x, int64_t ldx, double beta,
                   const void* y, int64_t ldy, void* out, int64_t ldo, fm_dtype dt, void* stream);

/* Upper bound of ||A||_2^2 from the operator's structure, in FP64: n for
 * Fourier and Hadamard, 1 for a row selection, max |d|^2 for Diag, the
 * squared Frobenius norm for a dense matrix, max_k |DFT_L(g)_k|^2 for
 * Circulant / Toeplitz / multilevel Toeplitz (g the cyclic embedding), the
 * product over the terms of a Product or Kronecker product, (sum of square
 * roots)^2 for a Sum, the maximum over the blocks of BlkDiag. A valid FISTA
 * step constant. Synchronises the stream. */
fm_status fm_op_norm_bound(fm_op a, double* bound, void* stream);

/* ------------------------------------------------------------------ misc */
/* Thread-local description of the last error; valid until the next fm_* call
 * on this thread. */
const char* fm_last_error(void);
/* Library version, e.g. "0.1.0". */
const char* fm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FM_H */
