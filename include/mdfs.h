/*
 * mdfs.h -- C ABI of the MI355X (gfx950) k-tuple information-gain sweep of MDFS
 * ("MDFS - MultiDimensional Feature Selection", Piliszek, Mnich, Migacz, Tabaszewski, Sulecki,
 * Polewko-Klim, Rudnicki).
 *
 * The library computes, for every variable x_i of an information system with N objects, p
 * variables and a binary decision y,
 *
 *     IG^k_max(y; x_i) = N max_{m, r} ( H(y | x_m1..x_m(k-1)) - H(y | x_i, x_m1..x_m(k-1)) )
 *
 * (equation IGmax, section "Theory"), the maximum over every (k-1)-tuple m of other variables
 * and over n_disc random discretisations r (section "Algorithm and implementation", the
 * paragraphs on range/shares and on multiple discretisations), together with the tuple and the
 * discretisation where it is attained (the optional tuple output of ComputeMaxInfoGains,
 * section "Package functions introduction").  Entropies use pseudocounted class probabilities
 * p^d = (N^d_v + beta^d) / (N^0_v + beta^0 + N^1_v + beta^1), beta^d = xi N^d / min(N^0, N^1)
 * (the class-probability and pseudocount equations), natural logarithms, and voxel weights
 * n_v / N.
 *
 * Conventions shared by every entry point
 *   * Pointers named "device" are HIP device pointers on the current device; the caller owns
 *     every buffer, including the workspace.  The library never allocates device memory.
 *   * data   : float32, variable-major [n_var][n_obj] (R's column-major N x p matrix).
 *   * y      : uint8 [n_obj], values in {0, 1}, both classes non-empty.
 *   * codes  : uint8 [n_disc][n_var][n_obj], each in [0, divisions].
 *   * stream : a hipStream_t passed as void*; NULL is the default stream.
 *   * Argument errors are detected on the host before anything is enqueued and returned as a
 *     negative mdfs_status; mdfs_last_error() then describes them (thread-local string).
 *   * Calls that read the decision synchronise `stream` once at entry (to validate y and
 *     size the launch) and once at exit (to check the device status word); all kernels run
 *     on `stream`.
 *   * Supported sizes: 2 <= n_obj <= 16384 and n_obj >= divisions+1; each class < 32768
 *     objects; k in {1, 2, 3, 4, 5} (the paper's limit); divisions in {1, 2, 4} (2, 3 or 5
 *     classes); n_disc >= 1; disc_offset >= 0; for k = 3, n_var <= 8192; for k = 4,
 *     n_var <= 2048; for k = 5, n_var <= 512 (the partner tuple of a k >= 4 candidate travels
 *     as its 32-bit lexicographic rank); the k >= 4 engines keep the entropy tables (16 bytes per
 *     object) in LDS, which bounds n_obj near 8000 there.  Beyond these, MDFS_E_LIMIT.
 */
#ifndef MDFS_H
#define MDFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MDFS_OK = 0,
    MDFS_E_ARG = -1,     /* null pointer, bad size, range outside [0,1], xi < 0, ... */
    MDFS_E_Y = -2,       /* y has a value outside {0,1}, or one class is empty */
    MDFS_E_K = -3,       /* k not supported */
    MDFS_E_DIV = -4,     /* divisions not supported */
    MDFS_E_NAN = -5,     /* data holds a NaN */
    MDFS_E_NOMEM = -6,   /* workspace smaller than mdfs_workspace_size() */
    MDFS_E_HIP = -7,     /* a HIP runtime call failed */
    MDFS_E_CANCELLED = -8, /* the caller's cancel word was set while the sweep ran; outputs undefined */
    MDFS_E_OVERFLOW = -9,  /* candidate buffer overflow (pathological mass ties); results invalid */
    MDFS_E_LIMIT = -10     /* a size beyond the supported maximum */
} mdfs_status;

typedef enum {
    MDFS_ENGINE_AUTO = 0,     /* k=2: fp4 MFMA if both classes < 4096 objects, else int8 MFMA;
                                 k=3: fp4 MFMA for 2 or 3 classes under the same condition, else
                                 bitset; k=4: bitset for 2 or 3 classes, else histogram; k=5:
                                 bitset for 2 classes, else histogram */
    MDFS_ENGINE_MFMA = 1,     /* one-hot int8 contraction on the matrix cores */
    MDFS_ENGINE_BITSET = 2,   /* per-class bitsets, AND + popcount; k=3, k=4 with 2 or 3 classes,
                                 k=5 with 2 classes (there every cell follows from the counts of
                                 the objects in the first bin of each subset of the tuple, by
                                 inclusion-exclusion) */
    MDFS_ENGINE_MFMA_FP4 = 3, /* one-hot E2M1 (fp4) contraction, float32 accumulation (exact
                                 integers); k=2, or k=3 with divisions 1 or 2; each class < 4096
                                 objects, else MDFS_E_LIMIT */
    MDFS_ENGINE_HIST = 4      /* per-tuple histogram of the class-sorted codes, every cell counted
                                 directly; k = 4 or 5, any class count ("auto" for k = 5 with 3
                                 or 5 classes and for k = 4 with five classes) */
} mdfs_engine;

/* Problem description.  Fields follow the arguments of ComputeMaxInfoGains
 * (section "Canonical package usage": dimensions, divisions, discretizations, range,
 * pseudo.count, seed). */
typedef struct {
    int64_t n_obj;       /* N, objects */
    int64_t n_var;       /* p, variables */
    int32_t k;           /* dimensions: tuple size 1 to 5 (k = 1: each variable alone) */
    int32_t divisions;   /* classes per variable = divisions + 1 */
    int32_t n_disc;      /* number of random discretisations */
    int32_t disc_offset; /* index of the first discretisation (run r uses index disc_offset+r) */
    double range;        /* share spread: shares ~ U(1-range, 1+range), 0 <= range <= 1 */
    double pseudocount;  /* xi in beta^d = xi N^d / min(N^0,N^1); xi >= 0 */
    uint64_t seed;       /* seed of the counter-based SplitMix64 draws of the shares */
    int32_t engine;      /* mdfs_engine */
    int32_t flags;       /* bitwise OR of mdfs_flags; other bits must be 0 */
    int32_t workgroups;  /* workgroups of the persistent sweep kernels: 0 = the whole GPU, else
                            8..4096; smaller grids let concurrent calls on other streams share
                            the GPU (results do not depend on it) */
    int32_t tile;        /* launch shape of the pair sweep, 0 = default (results do not depend on
                            it; the autotuner picks it): bits 0-7 the super-tile side in tiles
                            (2, 4, 8 or 16: the tiles whose operand panels share an XCD's L2),
                            bits 8-11 the waves per workgroup with three classes (4 or 8);
                            other bits must be 0 */
    const volatile uint32_t *cancel;
                         /* nullable: a caller-owned word in host-mapped memory (hipHostMalloc);
                            while it reads non-zero, the persistent sweep kernels stop taking work
                            (each checks it every 16 work items and exits normally) and the call
                            returns MDFS_E_CANCELLED (mdfs_check_status for asynchronous calls).
                            The library never writes it; the caller clears it. */
} mdfs_params;

typedef enum {
    /* record HIP events on the call's stream around each phase; read with mdfs_phase_times */
    MDFS_FLAG_TIMING = 1
} mdfs_flags;

/* Bytes of device workspace that mdfs_discretize / mdfs_max_ig need for `prm` (0 when the
 * parameters are invalid; mdfs_last_error() says why).  The workspace holds the class-sorted
 * one-hot (or bitset) encoding of every discretisation, per-variable marginals, entropy
 * lookup tables and the candidate buffer of the max reduction. */
size_t mdfs_workspace_size(const mdfs_params *prm);

/* Randomised rank-based discretisation (section "Algorithm and implementation": shares drawn
 * from U(1-range, 1+range), divisions distinct cut positions, the variable sorted and the
 * values at the cut positions used as thresholds).  For discretisation index
 * q = disc_offset + r and variable v: shares s_j = (1-range) + 2 range u_j with u_j from
 * SplitMix64 keyed by (seed, q, v, j); cut t_j = floor(N cum_j / S) clamped into [1, N-1] and
 * made strictly increasing; threshold v_j = sort(x_v)[t_j]; code = #{j : x >= v_j}.
 *   data  : device float32 [n_var][n_obj] (input)
 *   codes : device uint8 [n_disc][n_var][n_obj] (output)
 *   ws    : device workspace of at least mdfs_workspace_size(prm) bytes
 * Returns MDFS_E_NAN if data holds a NaN (codes then undefined).  Synchronises `stream`. */
int mdfs_discretize(const mdfs_params *prm, const float *data, uint8_t *codes, void *ws,
                    size_t ws_bytes, void *stream);

/* IG^k_max(y; x_i) for every variable (equation IGmax), maximised over all k-tuples and all
 * n_disc discretisations, with the argmax.  k = 1 is the one-dimensional analysis:
 * IG(x_i) = N (H(y) - H(y | x_i)) in binary64, maximised over the discretisations only (argmax
 * is not written).
 *   data        : device float32 [n_var][n_obj] (input)
 *   y           : device uint8 [n_obj] (input, decision)
 *   ig_max      : device float32 [n_var] (output): the maximum IG, in nats, evaluated in
 *                 binary64 for the maximising tuple and rounded to float32
 *   argmax      : device int32 [n_var][k-1] (output, nullable): the other members of the
 *                 maximising tuple, ascending variable indices
 *   argmax_disc : device int32 [n_var] (output, nullable): absolute discretisation index
 *                 (disc_offset + r) of the maximum
 *   ws          : device workspace of at least mdfs_workspace_size(prm) bytes
 * Ties: candidates within tau = 1e-9 max(1,|max|) of the maximum are tied; the smallest
 * discretisation index wins, then the lexicographically smallest tuple.
 * Synchronises `stream` at entry (reads y) and at exit (device status). */
int mdfs_max_ig(const mdfs_params *prm, const float *data, const uint8_t *y, float *ig_max,
                int32_t *argmax, int32_t *argmax_disc, void *ws, size_t ws_bytes, void *stream);

/* mdfs_max_ig without any host synchronisation, for callers that enqueue many calls or capture
 * the launch sequence in a HIP graph (the batching of many problems behind one replay):
 *   n1     : number of objects with y = 1 (known to the caller, e.g. when y was uploaded); the
 *            launch is sized from it and y is checked against it on the device.  A mismatch or a
 *            y value outside {0, 1} writes nothing and is reported by mdfs_check_status (MDFS_E_Y).
 *   other arguments as mdfs_max_ig; outputs are defined once the stream reaches them.
 * Nothing is read back: the candidate-overflow collect pass is always enqueued and exits on the
 * device when not needed; NaN data, bad y and a final overflow are reported by mdfs_check_status.
 * MDFS_FLAG_TIMING is refused.  Every engine runs as in mdfs_max_ig (the k = 3 matrix-core tile
 * list is built on the device).
 * Argument errors are returned before anything is enqueued, as for the other calls. */
int mdfs_max_ig_async(const mdfs_params *prm, const float *data, const uint8_t *y, int64_t n1, float *ig_max,
                      int32_t *argmax, int32_t *argmax_disc, void *ws, size_t ws_bytes, void *stream);

/* mdfs_max_ig_async for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same computation and outputs, with the
 * workspace taken from a device array inside the library (128 MiB per GPU, held from the first
 * use until the process ends) instead of a caller buffer.  No device or host memory is allocated
 * by the call.
 *   prm, data, y, n1, ig_max, argmax, argmax_disc, stream : as mdfs_max_ig_async
 *   status_out : device int32 [1] (nullable): written on `stream` after the outputs with the code
 *                mdfs_check_status would return (MDFS_OK, MDFS_E_Y, MDFS_E_NAN, MDFS_E_OVERFLOW)
 * Returns MDFS_E_NOMEM when mdfs_workspace_size(prm) exceeds 128 MiB (e.g. N = 2000, p = 500,
 * three classes and 30 discretisations need 92 MiB at k = 2, 112 MiB at k = 3), other argument
 * errors as mdfs_max_ig_async, before anything is enqueued.  Every call on one GPU uses that GPU's
 * one array: calls that overlap in time on one GPU (other streams, other host threads) race and
 * must be serialised by the caller; each call starts by clearing what it needs cleared. */
int mdfs_max_ig_noalloc(const mdfs_params *prm, const float *data, const uint8_t *y, int64_t n1, float *ig_max,
                        int32_t *argmax, int32_t *argmax_disc, int32_t *status_out, void *stream);

/* Several problems (datasets of uneven N and p, their own discretisation counts) in one
 * asynchronous call.  k = 2: the maximum pass is ONE persistent launch over the concatenated
 * tiles of all problems, so small problems share the GPU instead of leaving it idle between
 * launches, and each problem's own kernels (encoding, collect pass, re-score) run on one of four
 * streams.  Other k: each problem's calls run on one of four streams (the caller's and three
 * side streams of a per-thread pool, forked from and joined back into `stream`), so problems that
 * do not fill the GPU run concurrently.
 *   n               : 1 <= n <= 12 problems, all with the same k; for k = 2 also the same
 *                     divisions, the same encoding (every class < 4096 objects for fp4, or
 *                     engine mfma for int8) and the same super-tile side (tile bits 0-7; the
 *                     wave bits are not used here)
 *   prm[i], data[i], y[i], n1[i], ig_max[i], argmax[i], argmax_disc[i], ws[i], ws_bytes[i]:
 *                     problem i, as for mdfs_max_ig_async (its own workspace)
 *   batch_ws        : device memory of mdfs_batch_workspace_size() bytes (the work counters of
 *                     the k = 2 fused launch)
 * Per-problem status: mdfs_check_status(&prm[i], ws[i], ...).  Returns MDFS_E_K for mixed k,
 * MDFS_E_LIMIT for mixed divisions, encodings or super-tiles at k = 2; other argument errors as
 * mdfs_max_ig_async, before anything is enqueued.  Enqueued on `stream` with no host
 * synchronisation (capturable once a call outside capture has created the thread's streams). */
size_t mdfs_batch_workspace_size(void);
int mdfs_max_ig_batch(int n, const mdfs_params *prm, const float *const *data, const uint8_t *const *y,
                      const int64_t *n1, float *const *ig_max, int32_t *const *argmax, int32_t *const *argmax_disc,
                      void *const *ws, const size_t *ws_bytes, void *batch_ws, size_t batch_ws_bytes, void *stream);

/* Status of the last call that used workspace `ws` with parameters `prm` (synchronises `stream`):
 * MDFS_OK, or MDFS_E_Y / MDFS_E_NAN / MDFS_E_ARG (codes out of range) / MDFS_E_OVERFLOW as the
 * device flagged it. */
int mdfs_check_status(const mdfs_params *prm, const void *ws, size_t ws_bytes, void *stream);

/* mdfs_max_ig from caller-supplied codes instead of the randomised discretisation, so that a
 * discretised dataset can stay resident (or come from another discretiser): the same sweep,
 * outputs, ties and error behaviour.  range and seed of `prm` are unused.
 *   codes : device uint8 [n_disc][n_var][n_obj], each in [0, divisions]; a larger value makes the
 *           call return MDFS_E_ARG (detected on the device, reported at exit)
 * Discretisation index disc_offset + r names codes[r] in argmax_disc. */
int mdfs_max_ig_codes(const mdfs_params *prm, const uint8_t *codes, const uint8_t *y, float *ig_max,
                      int32_t *argmax, int32_t *argmax_disc, void *ws, size_t ws_bytes, void *stream);

/* Per-class voxel counts of every pair under one discretisation, as produced by the k=2 count
 * engine (the counters N^d of section "Algorithm and implementation").  Requires k = 2 in
 * `prm`; `disc` selects the discretisation (0 <= disc < n_disc).
 *   counts : device int32 [n_var][n_var][2][c][c], c = divisions+1, class-major; entry
 *            [i][j][d][a][b] counts objects of class d with code a in x_i and b in x_j; only
 *            i < j is written (other entries untouched).
 * The directly counted cells come from the maximum pass of mdfs_max_ig itself (the same kernel
 * body, encoding and table capacity, with a store added); the cells of each variable's dropped
 * last bin are completed from the marginals.  For tests and inspection: O(p^2 c^2) output.
 * Synchronises `stream`. */
int mdfs_pair_counts(const mdfs_params *prm, const float *data, const uint8_t *y, int32_t disc,
                     int32_t *counts, void *ws, size_t ws_bytes, void *stream);

/* Per-class voxel counts of the triples (i_sel, j, l), i_sel < j < l, under one discretisation, as
 * produced by the k = 3 count engine that `prm` selects (bitset, or the matrix cores for two and
 * three classes; the counters N^d of section "Algorithm and implementation").  Requires k = 3;
 * 0 <= disc < n_disc; 0 <= i_sel <= n_var - 3.
 *   counts : device int32 [n_var][n_var][2][c][c][c], c = divisions+1, class-major; entry
 *            [j][l][d][a][b][e] counts objects of class d with codes a, b, e in x_i_sel, x_j, x_l;
 *            only i_sel < j < l is written (other entries untouched).
 * The directly counted cells come from the very sweep that mdfs_max_ig runs (the same kernel body,
 * table capacity and encoding, with a store added); the cells of each variable's dropped last bin
 * are completed from the pair tables and marginals of that discretisation.  For tests and
 * inspection: O(p^2 c^3) output.  Synchronises `stream`. */
int mdfs_triple_counts(const mdfs_params *prm, const float *data, const uint8_t *y, int32_t disc, int32_t i_sel,
                       int32_t *counts, void *ws, size_t ws_bytes, void *stream);

/* ComputeInterestingTuples (section "Canonical package usage": the tuples whose information
 * gain is at least a threshold, with the gain per member): every (variable i, partner tuple m,
 * discretisation q) with IG(i | m) >= ig_thr, IG per equation IGmax in binary64 (the same value
 * mdfs_max_ig maximises).  One sweep in collect mode appends every tuple whose float32 IG lies
 * within the screen window of ig_thr; candidates are re-scored in binary64 and filtered.
 *   ig_thr   : threshold (not NaN; -inf lists every tuple and member, subject to capacity).
 *   var      : device int32 [max_out] variable i of each record.
 *   partners : device int32 [max_out][k-1] the partner tuple m, ascending.
 *   disc     : device int32 [max_out] discretisation index q (disc_offset-based).
 *   ig       : device double [max_out] IG(i | m).
 *   n_found  : host int64 (output): records found; when it exceeds max_out only max_out were
 *              written.  Record order is unspecified.
 * Returns MDFS_E_OVERFLOW (n_found = candidates appended) when more candidates lie near the
 * threshold than the workspace holds (max(256 n_var, 2^20) records).  Synchronises `stream`. */
int mdfs_interesting_tuples(const mdfs_params *prm, const float *data, const uint8_t *y, double ig_thr,
                            int32_t *var, int32_t *partners, int32_t *disc, double *ig, int64_t max_out,
                            int64_t *n_found, void *ws, size_t ws_bytes, void *stream);

/* AddContrastVariables (section "Package functions introduction": variables known to be
 * irrelevant, for the fit of the IG_max distribution; they are left out of the p-value
 * adjustment).  The paper cites the construction without defining it; here contrast variable c
 * copies original variable src(c) = SplitMix64(seed, c, 0x5352434) mod n_var with its objects
 * permuted by a keyed 4-round Feistel network on 2h-bit indices (2^(2h) >= n_obj), cycle-walked
 * into [0, n_obj): out[n_var + c][n] = data[src(c)][perm_c(n)].
 *   data : device float32 [n_var][n_obj] (input)
 *   out  : device float32 [n_var + n_contrast][n_obj] (output): the originals, then the contrast
 *          variables; must not overlap data
 *   src  : host int32 [n_contrast] (output, nullable): src(c) of every contrast variable
 * Enqueued on `stream` (no synchronisation).  Returns MDFS_E_ARG for null pointers, overlap or
 * sizes outside 1 <= n_obj <= 2^30, 1 <= n_var < 2^31, 0 <= n_contrast <= 2^24. */
int mdfs_add_contrast(const float *data, int64_t n_obj, int64_t n_var, int64_t n_contrast, uint64_t seed,
                      float *out, int32_t *src, void *stream);

/* ---- Significance of IG^k_max (host-side, binary64; host pointers, no device work) ----
 * Section "Theory", the paragraphs after equation IGmax: for an irrelevant variable and one
 * k-tuple, 2 IG is chi-square distributed (natural logarithms); IG^k_max, the largest of many
 * such values, follows an extreme value distribution whose one free parameter, the number of
 * independent tests n_eff, is fitted to the irrelevant part of the data; this yields p-values,
 * IG_lim for a significance level, and p-values adjusted by Holm or Benjamini-Hochberg(-Yekutieli)
 * (section "Canonical package usage": ComputePValue, then p.adjust).  Model used here:
 * Pr(IG_max <= x) = F(2x)^n_eff, F the chi-square CDF with mdfs_chi2_df(k, divisions) degrees of
 * freedom; n_eff by maximum likelihood, n_eff = -m / sum_v ln F(2 IG_v) over the m selected
 * variables with IG_v > 0. */

typedef enum {
    MDFS_ADJ_NONE = 0,   /* p-values unchanged */
    MDFS_ADJ_HOLM = 1,   /* Holm step-down (FWER) */
    MDFS_ADJ_BH = 2,     /* Benjamini-Hochberg (FDR) */
    MDFS_ADJ_BY = 3      /* Benjamini-Hochberg-Yekutieli (FDR under dependence) */
} mdfs_adjust;

/* Degrees of freedom of 2 IG for one tuple of irrelevant variables and a binary decision:
 * (c - 1) c^(k-1), c = divisions + 1.  Returns the df (> 0), or MDFS_E_K / MDFS_E_DIV for k
 * outside [1, 5] or divisions outside [1, 15]. */
int mdfs_chi2_df(int k, int divisions);

/* p-value of every variable's IG^k_max.
 *   ig          : host double [n], IG^k_max in nats (the values mdfs_max_ig returns)
 *   fit_mask    : host uint8 [n] or NULL: the variables taken as irrelevant for the fit of n_eff
 *                 (1 = use); NULL = all variables.  Variables with IG <= 0 never enter the fit.
 *   n_eff_fixed : > 0 uses this n_eff (e.g. 1 for a single tuple and discretisation), <= 0 fits it
 *   p_out       : host double [n] (output) 1 - F(2 IG)^n_eff, accurate far below 1e-16; 1 for IG <= 0
 *   n_eff_out   : host double (output, nullable) the n_eff used
 * Returns MDFS_E_ARG for null pointers, n < 1, a NaN IG or no usable variable in the fit. */
int mdfs_pvalues(const double *ig, int64_t n, int k, int divisions, const uint8_t *fit_mask, double n_eff_fixed,
                 double *p_out, double *n_eff_out);

/* IG_lim: the IG^k_max whose p-value is alpha under n_eff (0 < alpha < 1, 0 < n_eff < inf).
 *   ig_lim : host double (output).  Returns MDFS_E_ARG for arguments out of range. */
int mdfs_ig_lim(int k, int divisions, double n_eff, double alpha, double *ig_lim);

/* Adjusted p-values (method: mdfs_adjust), the definitions of R's p.adjust: Holm
 * max_{j<=i} min(1, (n-j+1) p_(j)); BH min_{j>=i} min(1, n/j p_(j)); BY as BH times sum_{j<=n} 1/j.
 *   p : host double [n] in [0, 1];  out : host double [n] (output; may alias p).
 * Returns MDFS_E_ARG for null pointers, n < 1, an unknown method or a p outside [0, 1]. */
int mdfs_p_adjust(const double *p, int64_t n, int method, double *out);

/* The float32 screening maxima of the sweep before the binary64 re-score: for every variable
 * the largest float32 IG over all tuples and discretisations, and the float32 error bound E
 * that the re-score window is built from (|IG_f32 - IG| <= E for every tuple).
 *   ig32 : device float32 [n_var] (output);  err_bound : host double* (output, nullable).
 * Synchronises `stream`. */
int mdfs_screen_max(const mdfs_params *prm, const float *data, const uint8_t *y, float *ig32,
                    double *err_bound, void *ws, size_t ws_bytes, void *stream);

/* Phase durations of the last call on this thread that ran with MDFS_FLAG_TIMING, measured
 * with HIP events recorded on that call's stream: [0] setup (status, class order, entropy
 * tables), [1] discretise + encode, [2] tuple sweep, [3] re-score and outputs.
 *   ms : host float[n_max] (output, milliseconds).  Returns the number of phases written
 *        (0 when no timed call has completed on this thread). */
int mdfs_phase_times(float *ms, int n_max);

/* Thread-local description of the last error returned on this thread ("" after success). */
const char *mdfs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MDFS_H */
