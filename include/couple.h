/*
 * couple.h -- C ABI of libcouple: MASTER mode-coupling matrices on MI355X.
 *
 * Computes, for a survey window with power spectra W_TT, W_TP, W_PP,
 *
 *   K^X_{l1 l2} = (2 l2 + 1) Xi_X(l1, l2),
 *   Xi_X(l1, l2) = 1/(4 pi) sum_{l3} (2 l3 + 1) W^X_{l3} S^X(l1, l2, l3),
 *
 *   S^TT = (l1 l2 l3; 0 0 0)^2                              Sec. 2, eq. K_TT
 *   S^TE = [(1+(-1)^L)/2] (l1 l2 l3; 0 0 0)(l1 l2 l3; -2 2 0)   App. A, eq. Sig_TE
 *   S^EE = S^BB = [(1+(-1)^L)/2]^2 (l1 l2 l3; -2 2 0)^2      Sec. 2, eq. K_EE; App. A
 *
 * (L = l1 + l2 + l3; W^TT = W_TT, W^TE = W_TP, W^EE = W^BB = W_PP), with every
 * 3j value taken from look-up tables of g(p) = (2p)!/(2^{2p} (p!)^2) built by
 * the recurrence of Sec. 3.1 (eqs. 000_sq_main, gdef, g_rec), and the
 * (-2 2 0) symbol reduced to the (0 0 0) one in closed form (Sec. 3.2,
 * App. B.3, eq. 022_linear_closedform).
 *
 * Conventions for every entry point
 *   - Return value: COUPLE_OK (0) on success, a negative COUPLE_E* code on
 *     failure.  Nothing throws or aborts.  couple_last_error() gives the text
 *     of the last failure on that context.
 *   - Pointers to window spectra and outputs are DEVICE pointers (e.g. the
 *     data_ptr() of a torch-ROCm tensor on the context's device), owned by the
 *     caller, float64, contiguous.  The library never frees them.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL means
 *     the legacy default stream); results are ready when the stream is.
 *     Argument errors are detected on the host before anything is enqueued.
 *   - Calls on one context must not overlap in time on different streams:
 *     they share the context's workspace.
 *   - Output layout: out[n_spec][lmax+1][lmax+1], row-major (row l1, column
 *     l2), spectra in the order TT, TE, EE, BB restricted to those requested.
 *     Polarization rows and columns 0 and 1 are exactly 0 (the (-2 2 0)
 *     symbol vanishes for l < 2).  K^BB is bitwise equal to K^EE.
 */
#ifndef COUPLE_H
#define COUPLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct couple_ctx couple_ctx;

enum couple_status {
    COUPLE_OK = 0,
    COUPLE_EINVAL = -1,   /* bad argument (detected on the host, nothing enqueued) */
    COUPLE_ENOMEM = -2,   /* device or host allocation failed (couple_init only)   */
    COUPLE_EDEVICE = -3,  /* a HIP runtime call or kernel launch failed            */
    COUPLE_ENOTSUP = -4   /* valid request the library does not implement          */
};

/* spectra bit mask; outputs are written in this order */
enum couple_spectrum {
    COUPLE_TT = 1,
    COUPLE_TE = 2,
    COUPLE_EE = 4,
    COUPLE_BB = 8,
    COUPLE_EB = 16, /* odd-L leakage kernel of App. A: S^EB = [(1-(-1)^L)/2]^2 (l1 l2 l3; -2 2 0)^2
                       with W_PP (the E-B mixing block of the MASTER polarization matrix) */
    COUPLE_XI = 256 /* output-form flag, OR-ed into spectra: write the symmetric kernels
                       Xi_X(l1, l2) of App. A instead of K^X = (2 l2 + 1) Xi_X, same layout.
                       Evaluated on the power spectrum of the squared mask, these are the
                       kernels of the approximate pseudo-C_l covariance (Sec. 2; band-limited
                       form Sec. 4.3).  For the same inputs and precision, K^X equals the
                       float64 product (2 l2 + 1) * Xi_X bit for bit. */
};

/* arithmetic of the l3 reduction */
enum couple_precision {
    COUPLE_FP64 = 0,   /* float64 throughout                                          */
    COUPLE_FP32C = 1,  /* float32 terms with compensated accumulation; float64 tables,
                          window scaling and final rescale.  Each block of terms is
                          scaled by a power of two from the largest |W'| it can meet,
                          so windows far outside float32's range are handled       */
    COUPLE_MFMA_FP32 = 2, /* batched form only: float32 matrix-core contraction of the
                             3j^2 tiles against the windows, Kahan-flushed accumulators;
                             W' = (2l+1) W_l / 4 pi is rounded to float32 unscaled, so
                             terms whose W' lies below its normal range are lost     */
    COUPLE_MFMA_BF16X3 = 3 /* batched form only: the same contraction on bfloat16
                              matrix cores with both operands split hi + lo and three
                              products (hi*hi + hi*lo + lo*hi) accumulated in float32;
                              relative error per term at most 3 * 2^-16 (4.6e-5),
                              bfloat16 keeping 8 significant bits.  A 2e-5-class
                              form (measured 1.4e-5 .. 2.0e-5): it does not meet
                              the 1e-6 of COUPLE_FP32C and COUPLE_MFMA_FP32      */
};

/*
 * couple_init -- build the look-up tables on the current HIP device and size
 * the workspace for every later call with lmax <= lmax_max.
 *   lmax_max : 0 <= lmax_max <= COUPLE_LMAX_LIMIT.
 *   ctx      : receives the new context (owned by the caller; release with
 *              couple_free).
 * Tables (Sec. 3.1): g(p) for p <= lmax_max and 1/((2p+1) g(p)) for
 * p <= 2 lmax_max (the paper's 1/(J+1) factor folded in, J + 1 = 2p + 1),
 * plus c_l = [(l-1) l (l+1) (l+2)]^{-1/2} (the 1/(lambda eta) factor of
 * App. B.3).  They are generated on the device by the g recurrence in
 * double-double arithmetic and rounded once to float64 and float32.
 * Workspace: 4 (lmax_max+1)(lmax_max+2)/2 float64 for the symmetric kernels
 * Xi (TT, TE, EE, EB) plus 6 (2 lmax_max + 1) words for the scaled windows.
 * If the environment variable COUPLE_MAX_DEVICE_BYTES holds a positive decimal
 * byte count, a context whose tables and workspace (and, later, batched
 * workspace) would exceed it is refused with ENOMEM before any allocation.
 * Errors: EINVAL (bad lmax_max, NULL ctx), ENOMEM (allocation failed, or the
 * byte cap above), EDEVICE (no usable device, or a device error -- including
 * one left by earlier work on the device, which HIP reports on the next call).
 */
#define COUPLE_LMAX_LIMIT 16384
int couple_init(int lmax_max, couple_ctx **ctx);

/* couple_free -- release a context (NULL is a no-op).  Synchronises the whole
 * device first (hipDeviceSynchronize: work of other contexts and streams on it
 * is waited for too), since the context does not track the streams its calls
 * were enqueued on. */
void couple_free(couple_ctx *ctx);

/* couple_last_error -- NUL-terminated text of the last failure on ctx (owned
 * by ctx, valid until the next call on it); "" if none.  ctx may be NULL, in
 * which case the text of the last failed couple_init is returned. */
const char *couple_last_error(const couple_ctx *ctx);

/*
 * couple_matrix -- full coupling matrices (Sec. 2 eqs. K_TT, K_EE; App. A).
 *   W_TT, W_TP, W_PP : device float64 window spectra W_l, l = 0 .. w_len-1.
 *                      Only those the requested spectra use must be non-NULL
 *                      (TT -> W_TT, TE -> W_TP, EE/BB/EB -> W_PP).
 *                      With COUPLE_XI in spectra, Xi_X is written instead of K^X.
 *   w_len            : >= 2*lmax + 1 (W_L is needed for L <= 2 lmax, Sec. 4).
 *   lmax             : 0 <= lmax <= lmax_max of ctx.
 *   spectra          : non-empty OR of COUPLE_TT/TE/EE/BB/EB; output i is the
 *                      i-th requested spectrum in the order TT, TE, EE, BB, EB.
 *                      EB (odd L) is a second pass over the triangle.
 *   precision        : COUPLE_FP64 or COUPLE_FP32C.
 *   out              : device float64, popcount(spectra) * (lmax+1)^2 entries,
 *                      8-byte aligned; fully overwritten.
 *   stream           : hipStream_t to enqueue on.
 * Errors: EINVAL (NULL ctx/out/needed window, lmax or w_len out of range,
 * empty or unknown spectra bits, unknown precision, misaligned out), EDEVICE.
 */
int couple_matrix(couple_ctx *ctx, const double *W_TT, const double *W_TP, const double *W_PP,
                  int w_len, int lmax, unsigned spectra, int precision, double *out, void *stream);

/*
 * couple_band -- band-limited coupling matrices (Sec. 4.3): only
 * l3_lo <= l3 <= l3_hi enters the l3 sum, which is exact when W vanishes
 * outside that band.  Elements with |l1 - l2| > l3_hi are exactly 0 and
 * cost nothing.
 *   l3_lo, l3_hi : 0 <= l3_lo <= l3_hi.
 *   bin_edges    : NULL for the unbinned [n_spec][lmax+1][lmax+1] output, or a
 *                  HOST array of n_bins+1 strictly increasing multipoles with
 *                  0 <= bin_edges[0] and bin_edges[n_bins] <= lmax+1; bin b is
 *                  [bin_edges[b], bin_edges[b+1]).  Binned output is
 *                  out[n_spec][n_bins][n_bins] with
 *                  K_{b b'} = (1/n_b) sum_{l1 in b} sum_{l2 in b'} K_{l1 l2}
 *                  (uniform average over the row bin, sum over the column bin).
 *   other arguments as couple_matrix (w_len >= min(l3_hi, 2 lmax) + 1).
 * Asynchronous on stream, no allocation.  With n_bins <= 512 the bin edges
 * travel in the kernel arguments, so the call only enqueues kernels (it can
 * be captured in a graph); longer bin lists are staged through the
 * context's pinned buffer after a synchronisation of stream.
 * Errors: as couple_matrix, plus EINVAL for a bad band or bin list.
 */
int couple_band(couple_ctx *ctx, int l3_lo, int l3_hi, const double *W_TT, const double *W_TP,
                const double *W_PP, int w_len, int lmax, unsigned spectra, int precision,
                const int *bin_edges, int n_bins, double *out, void *stream);

/*
 * couple_band_batched -- couple_band for n_masks windows in one call.  Up to
 * four masks (three in FP32C, two in FP64 when TE is asked for) share one
 * strip launch, and with EB one odd-L launch as well: the g/h factors and the
 * (-2 2 0) polynomial of each term are formed once for them, and each mask's
 * sums are those of couple_band (the results are bitwise equal, in
 * COUPLE_FP64 and COUPLE_FP32C).  Such a group needs its Xi triangles of
 * diagonals 0 .. min(lmax, l3_hi) in the context's workspace, 3 per mask (4
 * with EB); the group is cut to what fits, and where a single mask is left the
 * per-mask launches run, as they do for FP32C with EB when the band has fewer
 * than 8192 strip items of 256 rows (couple_band's strip then runs 128-row
 * items, whose EB sums round differently).
 *   W_TT, W_TP, W_PP : HOST arrays of n_masks DEVICE pointers (an array may
 *                      be NULL when no requested spectrum uses it).
 *   out              : device float64, n_masks consecutive outputs of the
 *                      couple_band layout (mask-major).
 *   other arguments as couple_band; every mask shares lmax, band and bins.
 * Errors: as couple_band (the message names the offending mask), EINVAL for
 * n_masks < 1.
 */
int couple_band_batched(couple_ctx *ctx, int n_masks, int l3_lo, int l3_hi, const double *const *W_TT,
                        const double *const *W_TP, const double *const *W_PP, int w_len, int lmax,
                        unsigned spectra, int precision, const int *bin_edges, int n_bins, double *out,
                        void *stream);

/*
 * couple_reserve_batched -- size the context's batched workspace for a batch
 * of n_masks windows with the given lmax (HOST array).  Allocates (this is the
 * one entry point besides couple_init that does); later batched calls of the
 * same or smaller size allocate nothing.  When the workspace grows it first
 * synchronises the whole device (hipDeviceSynchronize, as couple_free), since
 * earlier batched calls on any stream may still read the old workspace.
 * Size: 3 (lmax_m+1)(lmax_m+2)/2 float64 per mask (its Xi),
 * plus, per group of 16 masks sorted by lmax (L = the group's largest), the
 * larger of the two W' tables: 3 (2L+33) x 16 float32 or
 * 3 x 2 x 2 x 16 x (L+64 rounded up to 8) bfloat16.
 * Errors: EINVAL (NULL ctx/lmax_i, n_masks outside [1, 64], lmax > lmax_max),
 * ENOMEM (allocation failed, or above COUPLE_MAX_DEVICE_BYTES, see couple_init).
 */
int couple_reserve_batched(couple_ctx *ctx, int n_masks, const int *lmax_i);

/*
 * couple_matrix_batched -- full coupling matrices for n_masks windows of
 * uneven lmax in one call (Sec. 2 eqs. K_TT, K_EE; App. A, per mask).
 *   lmax_i, w_len_i : HOST arrays of n_masks ints (w_len_i[m] >= 2 lmax_i[m] + 1).
 *   W_TT, W_TP, W_PP: HOST arrays of n_masks DEVICE float64 pointers (an
 *                     array may be NULL when no requested spectrum uses it).
 *   out             : HOST array of n_masks DEVICE float64 pointers; mask m
 *                     gets popcount(spectra) (lmax_i[m]+1)^2 entries in the
 *                     couple_matrix layout.
 *   precision       : COUPLE_MFMA_FP32 or COUPLE_MFMA_BF16X3 (no EB: ENOTSUP) -- one
 *                     contraction launch for the whole batch (plus a window
 *                     table kernel before and one fill kernel after): masks
 *                     sorted by lmax in groups of 16 share every generated
 *                     3j^2 tile on the matrix cores; needs
 *                     couple_reserve_batched first.  No allocation, no host
 *                     synchronisation: the call can be captured in a graph.
 *                     COUPLE_FP64 / COUPLE_FP32C -- each mask's result is
 *                     couple_matrix's, bitwise.  Masks sorted by
 *                     lmax run in groups of four (with TE three in FP32C,
 *                     two in FP64) through one strip launch each (and one
 *                     odd-L launch with EB), over the grid of the group's
 *                     largest lmax, sharing each term's g/h factors and
 *                     (-2 2 0) polynomial; their Xi stores go to the batched
 *                     workspace when couple_reserve_batched sized it for the
 *                     batch, else to the context's (in turns of what fits),
 *                     and one fill launch follows per turn.  FP32C with EB
 *                     groups only masks whose lmax agree mod 4, and runs
 *                     masks of lmax below 1792 (where couple_matrix's strip
 *                     runs 128-row items) through couple_matrix one by one.
 *                     Kernels only, no allocation or host synchronisation:
 *                     capturable in a graph.
 * Errors: EINVAL (as couple_matrix, naming the mask; workspace too small),
 * EDEVICE.
 */
int couple_matrix_batched(couple_ctx *ctx, int n_masks, const int *lmax_i, const double *const *W_TT,
                          const double *const *W_TP, const double *const *W_PP, const int *w_len_i,
                          unsigned spectra, int precision, double *const *out, void *stream);

/*
 * Tile shape of a batched matrix-core kernel (precision COUPLE_MFMA_FP32 or
 * COUPLE_MFMA_BF16X3, each keeps its own), and how often the float32
 * matrix-core accumulators are flushed into the running sums:
 *   row_tiles 1, 2, 4: the 16-mask form -- masks sorted by lmax in column groups
 *     of 16, each group run to its largest lmax; row_tiles 16-row tiles of one
 *     diagonal per wavefront; flush = MFMA steps between flushes (1..16; a
 *     float32 step covers 4 l3 values, a BF16x3 step 32).
 *   row_tiles 64, 128 (COUPLE_MFMA_FP32 only): the 4-mask form -- every work
 *     item runs tiles of four masks, each only as far as its largest lmax, on
 *     4 x 4 x 1 blocks; row_tiles rows of one diagonal per wavefront; flush =
 *     groups of 16 l3 values between flushes (1..4).
 *   Defaults: float32 (2, 8), BF16x3 (2, 4).
 *
 * couple_autotune_batched times the candidate shapes -- float32: row_tiles
 * 1, 2, 4 with flush 4 and 8, and 64, 128 with flush 2; BF16x3: row_tiles 1,
 * 2, 4 with flush 2 and 4 -- on the given batch (same arguments as
 * couple_matrix_batched; out is overwritten), keeps the fastest in ctx for
 * later batched calls of that precision and returns it through the optional
 * HOST pointers.  Synchronises the stream.
 * Errors: as couple_matrix_batched; EINVAL for a bad tile shape or a
 * precision without one.
 */
int couple_set_batched_tiles(couple_ctx *ctx, int precision, int row_tiles, int flush);
int couple_get_batched_tiles(couple_ctx *ctx, int precision, int *row_tiles, int *flush);
int couple_autotune_batched(couple_ctx *ctx, int precision, int n_masks, const int *lmax_i,
                            const double *const *W_TT, const double *const *W_TP, const double *const *W_PP,
                            const int *w_len_i, unsigned spectra, double *const *out, void *stream,
                            int *best_row_tiles, int *best_flush, float *best_ms);

/*
 * couple_threej_rows -- rows of Wigner 3j symbols (l1 l2 l3; -m m 0) for
 * m = 0, 1, 2 over every l3 = |l1-l2| .. l1+l2, evaluated from the context's
 * g(p) tables in closed form: the (0 0 0) symbol by eq. 000_sq_main (Sec. 3.1),
 * the (-1 1 0) family by App. B (eq. joneodd for odd L; eq. joneeven, whose
 * two terms collapse to one product, for even L) and the (-2 2 0) family by
 * App. B.3 (eq. 022_linear_closedform, and eq. 022_rearranged for odd L).
 * These are the symbols of the lensing and aberration weights the paper
 * names (Sec. 1) as well as of the coupling matrices.  float64.
 *   m        : 0, 1 or 2.
 *   l1, l2   : DEVICE int32 arrays of n_pairs multipoles.  A pair outside
 *              [0, lmax_max] gives a row of NaN (checked on the device).
 *   out      : device float64 [n_pairs][stride]; out[p][i] is the symbol at
 *              l3 = |l1-l2| + i for i < 2 min(l1, l2) + 1 and 0 beyond; rows
 *              longer than stride are cut at stride.
 * Only enqueues one kernel (no allocation, graph-capturable).
 * Errors: EINVAL (NULL ctx or pointer, misalignment, m, n_pairs or stride out
 * of range), EDEVICE.
 */
int couple_threej_rows(couple_ctx *ctx, int m, int n_pairs, const int *l1, const int *l2, double *out,
                       long long stride, void *stream);

/*
 * couple_threej_rows_m -- rows of Wigner 3j symbols (l1 l2 l3; m1 m2 m3),
 * m3 = -m1 - m2, over every l3 = |l1-l2| .. l1+l2, for the small magnetic
 * numbers whose two entries of equal sign (zero counts as either) are at most
 * 2 in magnitude: the (1 1 -2) and (2 2 -4) families that the Conclusion
 * names for the stochastic gravitational-wave background, their m-flips
 * (-1 -1 2), (-2 -2 4) and column permutations such as (2 -1 -1), mixed
 * ones such as (2 1 -3), and the (-m m 0), m <= 2, rows of couple_threej_rows.
 * Each symbol is one table product in closed form: the App. B forms of the
 * (0 -1 1) and (0 -2 2) families carried to (a b -a-b) by the lowering
 * relation of E57 Sec. 3.7 and collapsed symbolically to
 *   (x y z; a b -a-b) = T N_ab(x(x+1), y(y+1), z(z+1)) / (2 D_ab),
 * T the (0 0 0) symbol of eq. 000_sq_main (even L) or its odd-L counterpart,
 * N_ab an integer polynomial evaluated exactly, D_ab^2 a product of factorial
 * ratios; so no cancellation, and no recursion along the row.  float64.
 *   m1, m2   : the magnetic numbers of the l1 and l2 columns.
 *   l1, l2   : DEVICE int32 arrays of n_pairs multipoles.  A pair outside
 *              [0, lmax_max] gives a row of NaN (checked on the device).
 *   out      : device float64 [n_pairs][stride]; out[p][i] is the symbol at
 *              l3 = |l1-l2| + i for i < 2 min(l1, l2) + 1 and 0 beyond (also 0
 *              where a selection rule |m| <= l fails); rows longer than stride
 *              are cut at stride.
 * Only enqueues one kernel (no allocation, graph-capturable).
 * Errors: EINVAL (NULL ctx or pointer, misalignment, magnetic numbers outside
 * the families above, n_pairs or stride out of range), EDEVICE.
 */
int couple_threej_rows_m(couple_ctx *ctx, int m1, int m2, int n_pairs, const int *l1, const int *l2, double *out,
                         long long stride, void *stream);

/*
 * Binned MASTER solve (Sec. 2, eq. pseudo_cl).  The pseudo-spectra are linear
 * in the true spectra,
 *   <C~^TT> = K^TT C^TT,
 *   <C~^EE> = K^EE C^EE + K^EB C^BB,   <C~^BB> = K^EB C^EE + K^BB C^BB
 * (the B-mode line by the structure of App. A: Xi_BB has the form of Xi_EE and
 * Xi_BE = Xi_EB).  Binned with the couple_band rule (row-bin average,
 * column-bin sum, C_l constant inside a bin) this is K_{b b'} C_{b'} = C~_b.
 *
 * couple_bin_spectra -- C~_b = (1/n_b) sum_{l in b} C~_l for n_spec spectra.
 *   cl        : device float64 [n_spec][cl_len].
 *   bin_edges : HOST array of n_bins+1 strictly increasing multipoles,
 *               0 <= bin_edges[0], bin_edges[n_bins] <= cl_len,
 *               1 <= n_bins <= lmax_max+1 (as couple_band).
 *   out       : device float64 [n_spec][n_bins].
 *   Up to 512 bins only enqueues a kernel; longer lists synchronise stream
 *   and stage the edges as couple_band does.
 *
 * couple_master_solve -- solve the binned system for n_rhs right-hand sides.
 *   pol = 0 : K = [n][n] (e.g. binned K^TT); m = n unknowns.
 *   pol = 1 : K = [3][n][n], the binned K^EE, K^BB, K^EB in that order (the
 *             output of couple_band with spectra EE|BB|EB); the system is
 *             [K^EE K^EB; K^EB K^BB] of m = 2n unknowns (C^EE then C^BB).
 *   rhs  : device float64 [n_rhs][m] (binned pseudo-spectra, EE then BB).
 *   work : device float64 workspace of m * (m + n_rhs) entries, overwritten.
 *   x    : device float64 [n_rhs][m], the solution.
 *   m + n_rhs <= 15840.  Gaussian elimination with partial pivoting in
 *   float64; K and rhs are not modified.  Below 400 unknowns one work-group
 *   runs it all (one kernel).  From 400 on, outer panels of 32 columns are
 *   factorised by one work-group each while the row exchanges, U12 and the
 *   trailing updates are spread over the chip (3 kernels per panel); x serves
 *   as the scratch for each panel's pivots until the back substitution
 *   writes it.  A singular system (a zero pivot column) gives NaN in every
 *   entry of x.  Only enqueues kernels (no allocation, graph-capturable).
 * Errors (both): EINVAL (NULL ctx or pointer, misaligned pointer, sizes or
 * edges out of range), EDEVICE.
 */
int couple_bin_spectra(couple_ctx *ctx, int n_spec, const double *cl, int cl_len, const int *bin_edges,
                       int n_bins, double *out, void *stream);
int couple_master_solve(couple_ctx *ctx, int pol, int n, const double *K, int n_rhs, const double *rhs,
                        double *work, double *x, void *stream);

/*
 * couple_master_solve_noalloc -- couple_master_solve without the `work`
 * argument, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * [m][m + n_rhs] workspace is a file-scope device array of
 * COUPLE_NOALLOC_SOLVE_DOUBLES float64 (32 MiB) that every GPU the library
 * runs on holds until the process ends; couple_init resolves its address on
 * the context's device.  Arguments, layout, result and errors are those of
 * couple_master_solve; in addition m * (m + n_rhs) must not exceed
 * COUPLE_NOALLOC_SOLVE_DOUBLES (EINVAL otherwise, before any launch; with one
 * right-hand side that is m <= 2047 unknowns).  The call allocates nothing and
 * only enqueues the same kernels on `stream`.  All calls on one GPU share its
 * array: calls that may overlap on one GPU (other streams, other threads or
 * contexts) race and must be ordered by the caller.  Every entry the solve
 * reads is written earlier in the same call, so nothing needs clearing.
 */
#define COUPLE_NOALLOC_SOLVE_DOUBLES (1LL << 22)
int couple_master_solve_noalloc(couple_ctx *ctx, int pol, int n, const double *K, int n_rhs,
                                const double *rhs, double *x, void *stream);

/*
 * couple_tables -- copy the context's look-up tables to HOST buffers (for
 * inspection and tests).  Any pointer may be NULL to skip that table.
 *   g    : lmax_max + 1 float64,   g[p] = g(p)                  (eq. gdef)
 *   h    : 2 lmax_max + 1 float64, h[p] = 1/((2p+1) g(p))        (eq. 000_sq_main)
 *   cl   : lmax_max + 1 float64,   cl[l] = [(l-1) l (l+1)(l+2)]^{-1/2}, 0 for l < 2
 *   gf, hf : float32 roundings of g and h (lengths as g and h)
 * Synchronises the device.  Errors: EINVAL (NULL ctx), EDEVICE.
 */
int couple_tables(const couple_ctx *ctx, double *g, double *h, double *cl, float *gf, float *hf);

/* couple_lmax_max -- the lmax_max ctx was built for, or -1 for NULL. */
int couple_lmax_max(const couple_ctx *ctx);

/*
 * Measurement hooks (not part of the method).  couple_profile(ctx, 1) clears
 * the counters and makes every later call record a HIP event pair around each
 * of its kernels on the call's stream; couple_profile(ctx, 0) stops.
 * couple_profile_read waits for the recorded events and returns, per stage,
 * the summed kernel milliseconds and the number of launches:
 *   stage 0 = window scaling, 1 = l3 reduction (strip kernel),
 *   2 = fill / bin.
 * ms and counts are HOST arrays of COUPLE_N_STAGES entries (either may be
 * NULL).  Errors: EINVAL (NULL ctx), EDEVICE.
 */
#define COUPLE_N_STAGES 3
int couple_profile(couple_ctx *ctx, int enable);
int couple_profile_read(couple_ctx *ctx, double *ms, int *counts);

#ifdef __cplusplus
}
#endif

#endif /* COUPLE_H */
