// api.hip -- the extern "C" entry points declared in include/mdfs.h.
//
// Host side only: argument validation, class sizes and pseudocounts (beta^d = xi N^d /
// min(N^0, N^1), section "Algorithm and implementation"), the float32 screen error bound, the
// workspace layout, and the launch sequence on the caller's stream.  All arithmetic of the
// path runs in the kernels.
#include "../../include/mdfs.h"
#include "mdfs_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <mutex>
#include <vector>

using namespace mdfs;

// the thread's last error message (a fixed buffer: reporting an error allocates nothing)
static thread_local char g_err[512];

namespace mdfs {
void set_error(const char *msg) { snprintf(g_err, sizeof g_err, "%s", msg); }
}

static int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

static int hip_fail(hipError_t e, const char *what)
{
    return fail(MDFS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char *mdfs_last_error(void) { return g_err; }

// ---- optional per-phase timing with HIP events on the call's stream
constexpr int N_PHASE = 4;
static thread_local float g_phase_ms[N_PHASE];
static thread_local int g_n_phase = 0;

struct PhaseTimer {
    hipEvent_t ev[N_PHASE + 1] = {};
    bool on = false;
    hipStream_t s = nullptr;
    PhaseTimer(bool enable, hipStream_t stream) : on(enable), s(stream)
    {
        if (!on) return;
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) on = false;
    }
    void mark(int i)
    {
        if (on) (void)hipEventRecord(ev[i], s);
    }
    // after the stream has been synchronised
    void publish()
    {
        if (!on) return;
        for (int i = 0; i < N_PHASE; ++i)
            if (hipEventElapsedTime(&g_phase_ms[i], ev[i], ev[i + 1]) != hipSuccess) g_phase_ms[i] = -1.f;
        g_n_phase = N_PHASE;
    }
    ~PhaseTimer()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

extern "C" int mdfs_phase_times(float *ms, int n_max)
{
    int n = g_n_phase < n_max ? g_n_phase : n_max;
    for (int i = 0; i < n; ++i) ms[i] = g_phase_ms[i];
    return ms ? n : 0;
}

// Validate everything that does not need the data or the decision.
static int check_params(const mdfs_params *prm, bool sweep = true)
{
    if (!prm) return fail(MDFS_E_ARG, "params is NULL");
    if (prm->flags & ~MDFS_FLAG_TIMING) return fail(MDFS_E_ARG, "unknown flag bits 0x%x", prm->flags);
    if (prm->k < 1 || prm->k > 5) return fail(MDFS_E_K, "k=%d: supported tuple sizes are 1 to 5", prm->k);
    if (prm->divisions != 1 && prm->divisions != 2 && prm->divisions != 4)
        return fail(MDFS_E_DIV, "divisions=%d: supported are 1, 2, 4", prm->divisions);
    if (prm->n_obj < 2 || prm->n_obj < prm->divisions + 1)
        return fail(MDFS_E_ARG, "n_obj=%lld too small for %d classes", (long long)prm->n_obj, prm->divisions + 1);
    if (prm->n_obj > MAX_NOBJ) return fail(MDFS_E_LIMIT, "n_obj=%lld > %d", (long long)prm->n_obj, MAX_NOBJ);
    if (prm->n_var < prm->k) return fail(MDFS_E_ARG, "n_var=%lld < k", (long long)prm->n_var);
    if (prm->k == 3 && prm->n_var > MAX_K3_VARS)
        return fail(MDFS_E_LIMIT, "k=3 with n_var=%lld > %d", (long long)prm->n_var, MAX_K3_VARS);
    if (prm->k == 4 && prm->n_var > MAX_K4_VARS)
        return fail(MDFS_E_LIMIT, "k=4 with n_var=%lld > %d", (long long)prm->n_var, MAX_K4_VARS);
    if (prm->k == 5 && prm->n_var > MAX_K5_VARS)
        return fail(MDFS_E_LIMIT, "k=5 with n_var=%lld > %d", (long long)prm->n_var, MAX_K5_VARS);
    if (sweep && prm->k == 4 && prm->engine != MDFS_ENGINE_AUTO && prm->engine != MDFS_ENGINE_HIST &&
        !(prm->engine == MDFS_ENGINE_BITSET && prm->divisions <= 2))
        return fail(MDFS_E_LIMIT, "k=4 runs on the bitset engine (2 or 3 classes) or the histogram engine");
    if (sweep && prm->k == 5 && prm->engine != MDFS_ENGINE_AUTO && prm->engine != MDFS_ENGINE_HIST &&
        !(prm->engine == MDFS_ENGINE_BITSET && prm->divisions == 1))
        return fail(MDFS_E_LIMIT, "k=5 runs on the bitset engine (2 classes) or the histogram engine");
    if (sweep && prm->k <= 3 && prm->engine == MDFS_ENGINE_HIST)
        return fail(MDFS_E_LIMIT, "the histogram engine is built for k = 4 and 5");
    if (sweep && prm->k == 3 && prm->engine == MDFS_ENGINE_MFMA)
        return fail(MDFS_E_LIMIT, "k=3 on the matrix cores uses the fp4 encoding (engine mfma_fp4)");
    if (sweep && prm->k == 3 && prm->engine == MDFS_ENGINE_MFMA_FP4 && prm->divisions != 1 && prm->divisions != 2)
        return fail(MDFS_E_LIMIT, "k=3 on the matrix cores is built for divisions=1 or 2 (2 or 3 classes)");
    if (sweep && prm->k == 2 && prm->engine == MDFS_ENGINE_BITSET)
        return fail(MDFS_E_LIMIT, "k=2 has the MFMA engines only in this build");
    if (prm->n_disc < 1) return fail(MDFS_E_ARG, "n_disc=%d < 1", prm->n_disc);
    if (prm->disc_offset < 0) return fail(MDFS_E_ARG, "disc_offset < 0");
    if (!(prm->range >= 0.0 && prm->range <= 1.0)) return fail(MDFS_E_ARG, "range=%g outside [0,1]", prm->range);
    if (!(prm->pseudocount >= 0.0) || !isfinite(prm->pseudocount))
        return fail(MDFS_E_ARG, "pseudocount=%g must be finite and >= 0", prm->pseudocount);
    if (prm->engine < 0 || prm->engine > 4) return fail(MDFS_E_ARG, "engine=%d", prm->engine);
    if (prm->workgroups != 0 && (prm->workgroups < 8 || prm->workgroups > 4096))
        return fail(MDFS_E_ARG, "workgroups=%d: 0 (whole GPU) or 8..4096", prm->workgroups);
    {
        const int sb = prm->tile & 0xff, nw = (prm->tile >> 8) & 0xf;
        if ((prm->tile & ~0xfff) || !(sb == 0 || sb == 2 || sb == 4 || sb == 8 || sb == 16) ||
            !(nw == 0 || nw == 4 || nw == 8))
            return fail(MDFS_E_ARG, "tile=0x%x: super-tile 2, 4, 8 or 16 (bits 0-7), waves 4 or 8 (bits 8-11)",
                        prm->tile);
    }
    return MDFS_OK;
}

static Layout layout_of(const mdfs_params *prm, size_t pair_budget = PAIR_BUDGET_DEFAULT)
{
    return make_layout(prm->n_obj, prm->n_var, prm->k, prm->divisions, prm->n_disc, pair_budget);
}

extern "C" size_t mdfs_workspace_size(const mdfs_params *prm)
{
    if (check_params(prm, false) != MDFS_OK) return 0;
    g_err[0] = 0;
    return layout_of(prm).total;
}

// Bound E on |IG_f32 - IG| of the float32 screen for a table of V voxels: rounding of the
// lookup tables (|L|, |Q (A + B)|), one rounding per voxel term, V-1 accumulations, the
// float32 F of the parent and the final subtraction; doubled for margin.  Sums are bounded by
// sum_v n_v = N, sum of pseudocounts V*beta and F <= N ln 2.
static double screen_err_bound(int64_t N, double b0, double b1, int V)
{
    const double u = ldexp(1.0, -24);
    const double beta = b0 + b1;
    const double lnN = fmax(1.0, log((double)N + beta + 3.0));
    const double S_L = (double)N * lnN;
    const double S_AB = ((double)N + V * beta) * lnN + V * 0.75;
    const double S_t = (double)N * log(2.0);
    return 2.0 * u * (S_L + 3.0 * S_AB + (V + 2) * S_t);
}

// Read and validate the decision, then fill in everything the launches need.
static int setup(const mdfs_params *prm, const uint8_t *y, void *ws, size_t ws_bytes, void *stream,
                 Problem &P, int64_t n1_given = -1, size_t pair_budget = PAIR_BUDGET_DEFAULT)
{
    P = Problem{};
    P.L = layout_of(prm, pair_budget);
    if (ws_bytes < P.L.total)
        return fail(MDFS_E_NOMEM, "workspace %zu bytes < required %zu", ws_bytes, P.L.total);
    P.ws = static_cast<char *>(ws);
    P.stream = static_cast<hipStream_t>(stream);
    // test hook: a smaller candidate capacity exercises the overflow -> collect-pass path
    if (const char *cap = getenv("MDFS_TEST_CAP")) {
        long long c = atoll(cap);
        if (c > 0 && c < P.L.cap) P.L.cap = c;
    }
    P.disc_offset = prm->disc_offset;
    P.workgroups = prm->workgroups;
    P.supertile = prm->tile & 0xff;
    P.sweep_waves = (prm->tile >> 8) & 0xf;
    P.cancel = const_cast<const uint32_t *>(prm->cancel);
    P.range = prm->range;
    P.seed = prm->seed;
    const int64_t N = prm->n_obj;
    int64_t n1 = n1_given;
    if (y && n1 < 0) {
        std::vector<uint8_t> hy((size_t)N);
        hipError_t e = hipMemcpyAsync(hy.data(), y, (size_t)N, hipMemcpyDeviceToHost, P.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(P.stream);
        if (e != hipSuccess) return hip_fail(e, "reading y");
        n1 = 0;
        for (int64_t n = 0; n < N; ++n) {
            if (hy[n] > 1) return fail(MDFS_E_Y, "y[%lld]=%d is not 0 or 1", (long long)n, (int)hy[n]);
            n1 += hy[n];
        }
    }
    if (y) {
        const int64_t n0 = N - n1;
        if (n0 == 0 || n1 == 0) return fail(MDFS_E_Y, "decision has a single class");
        if (n0 > MAX_CLASS_OBJ || n1 > MAX_CLASS_OBJ)
            return fail(MDFS_E_LIMIT, "class sizes %lld/%lld exceed %d", (long long)n0, (long long)n1, MAX_CLASS_OBJ);
        P.N0 = (int)n0;
        P.N1 = (int)n1;
        const double m = (double)(n0 < n1 ? n0 : n1);
        P.beta0 = prm->pseudocount * (double)n0 / m;
        P.beta1 = prm->pseudocount * (double)n1 / m;
        // one-hot encoding of the pair contraction: E2M1 nibbles while float32 accumulation of
        // n1 * 4096 + n0 is exact, int8 bytes otherwise (or when asked for)
        const bool f4_fits = n0 <= MAX_CLASS_OBJ_F4 && n1 <= MAX_CLASS_OBJ_F4;
        if (prm->engine == MDFS_ENGINE_MFMA_FP4 && !f4_fits)
            return fail(MDFS_E_LIMIT, "fp4 engine: class sizes %lld/%lld exceed %d", (long long)n0, (long long)n1,
                        MAX_CLASS_OBJ_F4);
        P.fp4 = f4_fits && prm->engine != MDFS_ENGINE_MFMA;
        P.kobj = P.fp4 ? KOBJ_F4 : KOBJ_I8;
        P.K0pad = (P.N0 + P.kobj - 1) / P.kobj * P.kobj;
        P.KB0 = P.K0pad / P.kobj;
        P.KB = P.KB0 + (P.N1 + P.kobj - 1) / P.kobj;
        P.Kpad = P.KB * P.kobj;
        // the pair sweep keeps its entropy tables in LDS next to the operand stages
        const size_t lds = prm->k == 1 ? 0 : sweep2_lds_bytes(P, false) > sweep2_lds_bytes(P, true) ? sweep2_lds_bytes(P, false)
                                                                                  : sweep2_lds_bytes(P, true);
        if (lds > LDS_MAX)
            return fail(MDFS_E_LIMIT, "n_obj=%lld: the int8 sweep's LDS tables need %zu bytes > %zu",
                        (long long)N, lds, LDS_MAX);
        const int C = prm->divisions + 1;
        P.err_bound = screen_err_bound(N, P.beta0, P.beta1, C * C);
        // k = 3: the triple's own F (C^3 voxels) plus the float32 F of the parent pair
        if (prm->k == 3) P.err_bound += screen_err_bound(N, P.beta0, P.beta1, C * C * C);
        // k = 4, 5: the tuple's F (C^k voxels) and a parent's float32 F (C^(k-1) voxels)
        if (prm->k >= 4) {
            const int V = prm->k == 4 ? C * C * C * C : C * C * C * C * C;
            P.err_bound = screen_err_bound(N, P.beta0, P.beta1, V) + screen_err_bound(N, P.beta0, P.beta1, V / C);
        }
        // k >= 4 engine: bitsets for k = 4 with two or three classes and for k = 5 with two,
        // unless the histogram engine is asked for; the histogram engine otherwise
        P.hist = prm->k >= 4 && (C > (prm->k == 4 ? 3 : 2) || prm->engine == MDFS_ENGINE_HIST);
        P.sweep45 = prm->k >= 4 && !P.hist && C == 2;
        if (P.sweep45 && sweep45_lds_bytes(P) > LDS_MAX)
            return fail(MDFS_E_LIMIT, "k=%d bitset sweep: LDS tables and prefix words need %zu bytes > %zu", prm->k,
                        sweep45_lds_bytes(P), LDS_MAX);
        if (P.hist && sweep_hist_lds_bytes(P) > LDS_MAX)
            return fail(MDFS_E_LIMIT, "histogram engine: LDS tables and histograms need %zu bytes > %zu",
                        sweep_hist_lds_bytes(P), LDS_MAX);
        // k = 3 engine: matrix cores for two or three classes in the fp4 encoding (auto or asked for)
        P.k3_mfma = prm->k == 3 && (prm->divisions == 1 || prm->divisions == 2) && P.fp4 &&
                    (prm->engine == MDFS_ENGINE_AUTO || prm->engine == MDFS_ENGINE_MFMA_FP4);
        if (prm->k == 3 && prm->engine == MDFS_ENGINE_MFMA_FP4 && !P.k3_mfma)
            return fail(MDFS_E_LIMIT, "k=3 matrix-core engine needs d = 2 or 3 and classes < 4096 objects");
        if (P.k3_mfma && sweep3m_lds_bytes(P) > LDS_MAX)
            return fail(MDFS_E_LIMIT, "k=3 matrix-core sweep: LDS tables too large");
        if (P.k3_mfma) sweep3m_tile_counts(P.L.p, P.L.W, P.n_ablk3, P.n_tiles3);
    }
    return MDFS_OK;
}

#define LAUNCH(call)                                      \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

static int read_status(const Problem &P, Status &st)
{
    hipError_t e = hipMemcpyAsync(&st, P.ws + P.L.status, sizeof(Status), hipMemcpyDeviceToHost, P.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P.stream);
    if (e != hipSuccess) return hip_fail(e, "reading status");
    if (st.cancelled) return fail(MDFS_E_CANCELLED, "cancelled through the cancel word; outputs undefined");
    if (st.nan_flag) return fail(MDFS_E_NAN, "data holds a NaN");
    if (st.code_flag) return fail(MDFS_E_ARG, "codes hold a value above divisions");
    return MDFS_OK;
}

// The encoding step: discretise the data, or take the caller's codes.
static hipError_t launch_encode(const Problem &P, const float *data)
{
    return P.codes_in ? launch_encode_codes(P) : launch_discretize(P, data, nullptr, true);
}

// Pair sweep (k = 2) or, per discretisation, pair data then triple sweep (k = 3).  counts !=
// nullptr: the count export of discretisation disc_sel (k = 2: every pair; k = 3: the triples
// (i_sel, j, l)), completed from the marginals and pair tables of that discretisation.
static int sweep_pass(const Problem &P, int32_t *counts, int disc_sel, bool collect, int i_sel = -1)
{
    if (P.L.k == 2) {
        LAUNCH(launch_reset_queue(P));
        LAUNCH(launch_sweep2(P, counts, disc_sel, collect));
        if (counts) LAUNCH(launch_complete_pairs(P, counts, disc_sel));
    } else if (P.L.k >= 4) {
        for (int r = 0; r < P.L.R; ++r) {
            if (P.hist) LAUNCH(launch_sweep_hist(P, r, collect));
            else if (P.sweep45) LAUNCH(launch_sweep45(P, r, collect));
            else LAUNCH(launch_sweep4(P, r, collect));
        }
    } else {
        // per chunk of up to RC discretisations: one launch of the pair sweep for all their pair
        // data, one of the triple sweep over all their tiles
        for (int r0 = 0; r0 < P.L.R; r0 += P.L.RC) {
            const int nr = P.L.R - r0 < P.L.RC ? P.L.R - r0 : P.L.RC;
            int32_t *cr = (counts && disc_sel >= r0 && disc_sel < r0 + nr) ? counts : nullptr;
            LAUNCH(launch_reset_queue(P));
            LAUNCH(launch_pairs(P, r0, nr, collect));
            if (P.k3_mfma) LAUNCH(launch_sweep3m(P, r0, nr, collect, cr, i_sel, disc_sel));
            else LAUNCH(launch_sweep3(P, r0, nr, collect, cr, i_sel, disc_sel));
            // before the next chunk's pair data replace this one's
            if (cr) LAUNCH(launch_complete_triples(P, cr, disc_sel, r0, i_sel));
        }
    }
    return MDFS_OK;
}

static int run_sweep(Problem &P, const float *data, const uint8_t *y, int32_t *counts, int disc_sel,
                     PhaseTimer *tm = nullptr, int i_sel = -1)
{
    if (tm) tm->mark(0);
    LAUNCH(launch_init(P));
    if (P.k3_mfma) LAUNCH(launch_tiles3(P));
    LAUNCH(launch_class_perm(P, y));
    LAUNCH(launch_tables(P));
    if (tm) tm->mark(1);
    LAUNCH(launch_encode(P, data));
    if (tm) tm->mark(2);
    int rc = sweep_pass(P, counts, disc_sel, false, i_sel);
    if (rc) return rc;
    // If the opportunistic candidate appends overflowed, sweep again with the final float32
    // maxima as fixed thresholds: that pass appends exactly the (tuple, discretisation) pairs
    // within the re-score window.
    Status st;
    rc = read_status(P, st);
    if (rc) return rc;
    if (st.overflow) {
        LAUNCH(launch_collect_decide(P, false));
        LAUNCH(launch_reset_candidates(P, true));
        rc = sweep_pass(P, nullptr, -1, true);
        if (rc) return rc;
    }
    if (tm) tm->mark(3);
    return MDFS_OK;
}

extern "C" int mdfs_discretize(const mdfs_params *prm, const float *data, uint8_t *codes, void *ws,
                               size_t ws_bytes, void *stream)
{
    int rc = check_params(prm, false);
    if (rc) return rc;
    if (!data || !codes || !ws) return fail(MDFS_E_ARG, "null pointer");
    Problem P;
    if ((rc = setup(prm, nullptr, ws, ws_bytes, stream, P))) return rc;
    LAUNCH(launch_init(P));
    LAUNCH(launch_discretize(P, data, codes, false));
    Status st;
    if ((rc = read_status(P, st))) return rc;
    g_err[0] = 0;
    return MDFS_OK;
}

extern "C" int mdfs_add_contrast(const float *data, int64_t n_obj, int64_t n_var, int64_t n_contrast,
                                 uint64_t seed, float *out, int32_t *src, void *stream)
{
    if (!data || !out) return fail(MDFS_E_ARG, "data and out must be non-null");
    if (n_obj < 1 || n_obj > (int64_t(1) << 30) || n_var < 1 || n_var > INT32_MAX || n_contrast < 0 ||
        n_contrast > (int64_t(1) << 24))
        return fail(MDFS_E_ARG, "need 1 <= n_obj <= 2^30, 1 <= n_var < 2^31, 0 <= n_contrast <= 2^24");
    const char *d0 = reinterpret_cast<const char *>(data), *d1 = d0 + sizeof(float) * n_obj * n_var;
    const char *o0 = reinterpret_cast<const char *>(out), *o1 = o0 + sizeof(float) * n_obj * (n_var + n_contrast);
    if (o0 < d1 && d0 < o1) return fail(MDFS_E_ARG, "out overlaps data");
    if (src)
        for (int64_t c = 0; c < n_contrast; ++c) src[c] = (int32_t)contrast_source(seed, c, n_var);
    hipError_t e = launch_contrast(data, n_obj, n_var, n_contrast, seed, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "contrast variables");
    g_err[0] = 0;
    return MDFS_OK;
}

// k = 1: F of the decision alone (one voxel holding every object), binary64.
static double root_F(const Problem &P)
{
    const double n0 = P.N0, n1 = P.N1, n = n0 + n1, s = n + P.beta0 + P.beta1;
    auto xlx = [](double x) { return x > 0.0 ? x * log(x) : 0.0; };
    return n * log(s) - (n / s) * (xlx(n0 + P.beta0) + xlx(n1 + P.beta1));
}

static int max_ig_impl(const mdfs_params *prm, const float *data, const uint8_t *codes, const uint8_t *y,
                       float *ig_max, int32_t *argmax, int32_t *argmax_disc, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_params(prm);
    if (rc) return rc;
    if (!(data || codes) || !y || !ig_max || !ws) return fail(MDFS_E_ARG, "null pointer");
    Problem P;
    if ((rc = setup(prm, y, ws, ws_bytes, stream, P))) return rc;
    P.codes_in = codes;
    if (prm->k == 1) {
        // no tuples: discretise, per-variable F in binary64, maximum over discretisations
        PhaseTimer tm((prm->flags & MDFS_FLAG_TIMING) != 0, P.stream);
        tm.mark(0);
        LAUNCH(launch_init(P));
        LAUNCH(launch_class_perm(P, y));
        tm.mark(1);
        LAUNCH(launch_encode(P, data));
        tm.mark(2);
        tm.mark(3);
        LAUNCH(launch_ig1(P, root_F(P), ig_max, argmax_disc));
        tm.mark(4);
        Status st;
        if ((rc = read_status(P, st))) return rc;
        tm.publish();
        g_err[0] = 0;
        return MDFS_OK;
    }
    PhaseTimer tm((prm->flags & MDFS_FLAG_TIMING) != 0, P.stream);
    if ((rc = run_sweep(P, data, y, nullptr, -1, &tm))) return rc;
    LAUNCH(launch_finalize(P, ig_max, argmax, argmax_disc));
    tm.mark(4);
    Status st;
    if ((rc = read_status(P, st))) return rc;
    tm.publish();
    if (st.overflow) return fail(MDFS_E_OVERFLOW, "candidate buffer overflow (%u appends)", st.n_cand);
    g_err[0] = 0;
    return MDFS_OK;
}

extern "C" int mdfs_max_ig(const mdfs_params *prm, const float *data, const uint8_t *y, float *ig_max,
                           int32_t *argmax, int32_t *argmax_disc, void *ws, size_t ws_bytes, void *stream)
{
    return max_ig_impl(prm, data, nullptr, y, ig_max, argmax, argmax_disc, ws, ws_bytes, stream);
}

extern "C" int mdfs_max_ig_codes(const mdfs_params *prm, const uint8_t *codes, const uint8_t *y, float *ig_max,
                                 int32_t *argmax, int32_t *argmax_disc, void *ws, size_t ws_bytes, void *stream)
{
    return max_ig_impl(prm, nullptr, codes, y, ig_max, argmax, argmax_disc, ws, ws_bytes, stream);
}

static int max_ig_async_impl(const mdfs_params *prm, const float *data, const uint8_t *y, int64_t n1, float *ig_max,
                             int32_t *argmax, int32_t *argmax_disc, void *ws, size_t ws_bytes, void *stream,
                             size_t pair_budget = PAIR_BUDGET_DEFAULT)
{
    int rc = check_params(prm);
    if (rc) return rc;
    if (!data || !y || !ig_max || !ws) return fail(MDFS_E_ARG, "null pointer");
    if (prm->flags & MDFS_FLAG_TIMING) return fail(MDFS_E_ARG, "timing reads events back: not in the asynchronous call");
    if (n1 < 1 || n1 >= prm->n_obj) return fail(MDFS_E_Y, "n1=%lld: both classes must be non-empty", (long long)n1);
    Problem P;
    if ((rc = setup(prm, y, ws, ws_bytes, stream, P, n1, pair_budget))) return rc;
    LAUNCH(launch_init(P));
    if (P.k3_mfma) LAUNCH(launch_tiles3(P));
    LAUNCH(launch_class_perm(P, y, n1));
    if (prm->k == 1) {
        LAUNCH(launch_encode(P, data));
        LAUNCH(launch_ig1(P, root_F(P), ig_max, argmax_disc));
    } else {
        LAUNCH(launch_tables(P));
        LAUNCH(launch_encode(P, data));
        if ((rc = sweep_pass(P, nullptr, -1, false))) return rc;
        // the collect pass is always enqueued; its kernels exit at once unless an append overflowed
        LAUNCH(launch_collect_decide(P, false));
        LAUNCH(launch_reset_candidates(P, true));
        if ((rc = sweep_pass(P, nullptr, -1, true))) return rc;
        LAUNCH(launch_finalize(P, ig_max, argmax, argmax_disc));
    }
    g_err[0] = 0;
    return MDFS_OK;
}

extern "C" int mdfs_max_ig_async(const mdfs_params *prm, const float *data, const uint8_t *y, int64_t n1,
                                 float *ig_max, int32_t *argmax, int32_t *argmax_disc, void *ws, size_t ws_bytes,
                                 void *stream)
{
    return max_ig_async_impl(prm, data, y, n1, ig_max, argmax, argmax_disc, ws, ws_bytes, stream);
}

// ---- the entry point that allocates nothing
// Its workspace is a file-scope device array of fixed size; every GPU that loads the library holds
// its own copy until the process ends.  In host code `scratch` names a host-side stand-in, not a
// device address: its device address is taken once per device with hipGetSymbolAddress (with that
// device current) and only that address is passed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

// Device address of this device's scratch array (nullptr and an error message on failure).
static void *scratch_on(int dev)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            fail(MDFS_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// The device status word of the last call on `st`, as mdfs_check_status reports it.
__global__ void k_status_code(const Status *st, int32_t *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    out[0] = st->y_flag ? MDFS_E_Y : st->cancelled ? MDFS_E_CANCELLED : st->nan_flag ? MDFS_E_NAN
           : st->code_flag ? MDFS_E_ARG : st->overflow ? MDFS_E_OVERFLOW : MDFS_OK;
}

extern "C" int mdfs_max_ig_noalloc(const mdfs_params *prm, const float *data, const uint8_t *y, int64_t n1,
                                   float *ig_max, int32_t *argmax, int32_t *argmax_disc, int32_t *status_out,
                                   void *stream)
{
    int rc = check_params(prm);
    if (rc) return rc;
    // k = 3: fewer discretisations' pair data at once (more launches, the same results) where the
    // default would not fit the array
    size_t pair_budget = PAIR_BUDGET_DEFAULT;
    while (layout_of(prm, pair_budget).total > NOALLOC_SCRATCH_BYTES && layout_of(prm, pair_budget).RC > 1)
        pair_budget /= 2;
    const size_t need = layout_of(prm, pair_budget).total;
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(MDFS_E_NOMEM, "this problem needs %zu bytes of workspace; the allocation-free call holds %zu per GPU",
                    need, NOALLOC_SCRATCH_BYTES);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(MDFS_E_LIMIT, "device %d >= %d", dev, NOALLOC_MAX_DEVICES);
    void *ws = scratch_on(dev);
    if (!ws) return MDFS_E_HIP;
    if ((rc = max_ig_async_impl(prm, data, y, n1, ig_max, argmax, argmax_disc, ws, NOALLOC_SCRATCH_BYTES, stream,
                                pair_budget)))
        return rc;
    if (status_out) {
        const Layout L = layout_of(prm, pair_budget);
        hipLaunchKernelGGL(k_status_code, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                           reinterpret_cast<const Status *>(static_cast<char *>(ws) + L.status), status_out);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "status kernel");
    }
    g_err[0] = 0;
    return MDFS_OK;
}

extern "C" size_t mdfs_batch_workspace_size(void) { return 256; }

// Side streams of the batched call: the per-problem kernels around the fused sweep (the encoding
// before it; the collect pass, re-score and outputs after it) of different problems run on up to
// four streams (the caller's and three side streams), so that their small launches overlap
// instead of queueing one after another on the caller's stream.  One pool per host thread and
// device, so that calls from several threads share no stream or event; created on the first call
// that is not under stream capture (a call under capture with no pool yet runs on the caller's
// stream alone); default priority; destroyed when the thread ends.
constexpr int N_SIDE = 3;
struct SidePool {
    bool ok = false;
    hipStream_t s[N_SIDE] = {};
    hipEvent_t fork = nullptr, join[N_SIDE] = {};
    ~SidePool()
    {
        if (!ok) return;
        for (int i = 0; i < N_SIDE; ++i) {
            (void)hipEventDestroy(join[i]);
            (void)hipStreamDestroy(s[i]);
        }
        (void)hipEventDestroy(fork);
    }
};
constexpr int SIDE_MAX_DEVICES = 64;
static thread_local SidePool g_side[SIDE_MAX_DEVICES];

static SidePool *side_pool(hipStream_t stream)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SIDE_MAX_DEVICES) return nullptr;
    SidePool &sp = g_side[dev];
    if (sp.ok) return &sp;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    bool good = hipEventCreateWithFlags(&sp.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < N_SIDE && good; ++i)
        good = hipStreamCreateWithFlags(&sp.s[i], hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&sp.join[i], hipEventDisableTiming) == hipSuccess;
    if (!good) return nullptr;   // a partial pool is kept unused (not marked ok)
    sp.ok = true;
    return &sp;
}

// The side streams wait for the work enqueued so far on `stream` / `stream` waits for theirs.
static hipError_t side_fork(const SidePool *sp, hipStream_t stream)
{
    if (!sp) return hipSuccess;
    hipError_t e = hipEventRecord(sp->fork, stream);
    for (int i = 0; i < N_SIDE && e == hipSuccess; ++i) e = hipStreamWaitEvent(sp->s[i], sp->fork, 0);
    return e;
}
static hipError_t side_join(const SidePool *sp, hipStream_t stream)
{
    if (!sp) return hipSuccess;
    hipError_t e = hipSuccess;
    for (int i = 0; i < N_SIDE && e == hipSuccess; ++i) {
        e = hipEventRecord(sp->join[i], sp->s[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(stream, sp->join[i], 0);
    }
    return e;
}

// A batch of k >= 3 problems: every problem is validated first (so that an argument error
// leaves nothing enqueued), then each runs the asynchronous call's launches on stream i mod 4,
// forked from and joined back into the caller's stream: small problems that do not fill the
// GPU run concurrently.
static int batch_streams(int n, const mdfs_params *prm, const float *const *data, const uint8_t *const *y,
                         const int64_t *n1, float *const *ig_max, int32_t *const *argmax,
                         int32_t *const *argmax_disc, void *const *ws, const size_t *ws_bytes, void *stream)
{
    for (int i = 0; i < n; ++i) {
        int rc = check_params(&prm[i]);
        if (rc) return rc;
        if (prm[i].k != prm[0].k) return fail(MDFS_E_K, "problem %d: one k per batch", i);
    }
    for (int i = 0; i < n; ++i) {
        if (prm[i].flags & MDFS_FLAG_TIMING) return fail(MDFS_E_ARG, "timing is not available in a batch");
        if (!data[i] || !y[i] || !ig_max[i] || !ws[i]) return fail(MDFS_E_ARG, "problem %d: null pointer", i);
        if (n1[i] < 1 || n1[i] >= prm[i].n_obj)
            return fail(MDFS_E_Y, "problem %d: n1=%lld: both classes must be non-empty", i, (long long)n1[i]);
        if (ws_bytes[i] < layout_of(&prm[i]).total)
            return fail(MDFS_E_NOMEM, "problem %d: workspace %zu bytes < required %zu", i, ws_bytes[i],
                        layout_of(&prm[i]).total);
    }
    const hipStream_t main_stream = static_cast<hipStream_t>(stream);
    const SidePool *sp = n > 1 ? side_pool(main_stream) : nullptr;
    LAUNCH(side_fork(sp, main_stream));
    for (int i = 0; i < n; ++i) {
        const hipStream_t st = (sp && i % (N_SIDE + 1) != 0) ? sp->s[i % (N_SIDE + 1) - 1] : main_stream;
        const int rc = max_ig_async_impl(&prm[i], data[i], y[i], n1[i], ig_max[i], argmax ? argmax[i] : nullptr,
                                         argmax_disc ? argmax_disc[i] : nullptr, ws[i], ws_bytes[i], st);
        if (rc) return rc;
    }
    LAUNCH(side_join(sp, main_stream));
    g_err[0] = 0;
    return MDFS_OK;
}

extern "C" int mdfs_max_ig_batch(int n, const mdfs_params *prm, const float *const *data, const uint8_t *const *y,
                                 const int64_t *n1, float *const *ig_max, int32_t *const *argmax,
                                 int32_t *const *argmax_disc, void *const *ws, const size_t *ws_bytes, void *batch_ws,
                                 size_t batch_ws_bytes, void *stream)
{
    if (n < 1 || n > MAX_BATCH) return fail(MDFS_E_ARG, "n=%d: a batch holds 1..%d problems", n, MAX_BATCH);
    if (!prm || !data || !y || !n1 || !ig_max || !ws || !ws_bytes || !batch_ws)
        return fail(MDFS_E_ARG, "null pointer");
    if (batch_ws_bytes < sizeof(Status)) return fail(MDFS_E_NOMEM, "batch workspace %zu bytes < %zu", batch_ws_bytes,
                                                     sizeof(Status));
    if (prm[0].k != 2) return batch_streams(n, prm, data, y, n1, ig_max, argmax, argmax_disc, ws, ws_bytes, stream);
    std::vector<Problem> Ps((size_t)n);
    std::vector<const Problem *> pp((size_t)n);
    for (int i = 0; i < n; ++i) {
        int rc = check_params(&prm[i]);
        if (rc) return rc;
        if (prm[i].k != 2) return fail(MDFS_E_K, "problem %d: k=%d in a batch of k=2 problems", i, prm[i].k);
        if (prm[i].divisions != prm[0].divisions) return fail(MDFS_E_LIMIT, "problem %d: one divisions per batch", i);
        if ((prm[i].tile & 0xff) != (prm[0].tile & 0xff))
            return fail(MDFS_E_LIMIT, "problem %d: one super-tile side per batch (the shared queue's unit)", i);
        if (prm[i].flags & MDFS_FLAG_TIMING) return fail(MDFS_E_ARG, "timing is not available in a batch");
        if (!data[i] || !y[i] || !ig_max[i] || !ws[i]) return fail(MDFS_E_ARG, "problem %d: null pointer", i);
        if (n1[i] < 1 || n1[i] >= prm[i].n_obj)
            return fail(MDFS_E_Y, "problem %d: n1=%lld: both classes must be non-empty", i, (long long)n1[i]);
        if ((rc = setup(&prm[i], y[i], ws[i], ws_bytes[i], stream, Ps[(size_t)i], n1[i]))) return rc;
        pp[(size_t)i] = &Ps[(size_t)i];
        if (Ps[(size_t)i].fp4 != Ps[0].fp4)
            return fail(MDFS_E_LIMIT, "problem %d: one encoding per batch (fp4 needs classes < 4096 objects)", i);
    }
    // problem i's own kernels run on stream i mod 4 (0: the caller's)
    const hipStream_t main_stream = static_cast<hipStream_t>(stream);
    const SidePool *sp = n > 1 ? side_pool(main_stream) : nullptr;
    auto on_stream = [&](int i) {
        Problem P = Ps[(size_t)i];
        if (sp && i % (N_SIDE + 1) != 0) P.stream = sp->s[i % (N_SIDE + 1) - 1];
        return P;
    };
    // per problem: status, class order (checked against n1 on the device), tables, encoding
    LAUNCH(side_fork(sp, main_stream));
    for (int i = 0; i < n; ++i) {
        const Problem P = on_stream(i);
        LAUNCH(launch_init(P));
        LAUNCH(launch_class_perm(P, y[i], n1[i]));
        LAUNCH(launch_tables(P));
        LAUNCH(launch_encode(P, data[i]));
    }
    LAUNCH(side_join(sp, main_stream));
    // the maximum pass of every problem in one persistent launch
    Problem Q = Ps[0];
    Q.ws = static_cast<char *>(batch_ws);
    Q.L.status = 0;
    LAUNCH(launch_reset_queue(Q));
    LAUNCH(launch_sweep2_batch(pp.data(), n, static_cast<Status *>(batch_ws)));
    // per problem: the gated collect pass, then re-score and outputs
    LAUNCH(side_fork(sp, main_stream));
    for (int i = 0; i < n; ++i) {
        const Problem P = on_stream(i);
        LAUNCH(launch_collect_decide(P, false));
        LAUNCH(launch_reset_candidates(P, true));
        int rc = sweep_pass(P, nullptr, -1, true);
        if (rc) return rc;
        LAUNCH(launch_finalize(P, ig_max[i], argmax ? argmax[i] : nullptr, argmax_disc ? argmax_disc[i] : nullptr));
    }
    LAUNCH(side_join(sp, main_stream));
    g_err[0] = 0;
    return MDFS_OK;
}

extern "C" int mdfs_check_status(const mdfs_params *prm, const void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_params(prm, false);
    if (rc) return rc;
    if (!ws) return fail(MDFS_E_ARG, "null pointer");
    const Layout L = layout_of(prm);
    if (ws_bytes < L.total) return fail(MDFS_E_NOMEM, "workspace %zu bytes < required %zu", ws_bytes, L.total);
    Status st;
    hipError_t e = hipMemcpyAsync(&st, static_cast<const char *>(ws) + L.status, sizeof(Status), hipMemcpyDeviceToHost,
                                  static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "reading status");
    if (st.y_flag) return fail(MDFS_E_Y, "y disagrees with n1 or holds a value other than 0 and 1");
    if (st.cancelled) return fail(MDFS_E_CANCELLED, "cancelled through the cancel word; outputs undefined");
    if (st.nan_flag) return fail(MDFS_E_NAN, "data holds a NaN");
    if (st.code_flag) return fail(MDFS_E_ARG, "codes hold a value above divisions");
    if (st.overflow) return fail(MDFS_E_OVERFLOW, "candidate buffer overflow (%u appends)", st.n_cand);
    g_err[0] = 0;
    return MDFS_OK;
}

extern "C" int mdfs_pair_counts(const mdfs_params *prm, const float *data, const uint8_t *y, int32_t disc,
                                int32_t *counts, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_params(prm);
    if (rc) return rc;
    if (prm->k == 1) return fail(MDFS_E_K, "k=1 has no tuples (mdfs_max_ig covers it)");
    if (prm->k != 2) return fail(MDFS_E_K, "pair counts need k=2");
    if (!data || !y || !counts || !ws) return fail(MDFS_E_ARG, "null pointer");
    if (disc < 0 || disc >= prm->n_disc) return fail(MDFS_E_ARG, "disc=%d outside [0,%d)", disc, prm->n_disc);
    Problem P;
    if ((rc = setup(prm, y, ws, ws_bytes, stream, P))) return rc;
    if ((rc = run_sweep(P, data, y, counts, disc))) return rc;
    Status st;
    if ((rc = read_status(P, st))) return rc;
    g_err[0] = 0;
    return MDFS_OK;
}

extern "C" int mdfs_triple_counts(const mdfs_params *prm, const float *data, const uint8_t *y, int32_t disc,
                                  int32_t i_sel, int32_t *counts, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_params(prm);
    if (rc) return rc;
    if (prm->k != 3) return fail(MDFS_E_K, "triple counts need k=3");
    if (!data || !y || !counts || !ws) return fail(MDFS_E_ARG, "null pointer");
    if (disc < 0 || disc >= prm->n_disc) return fail(MDFS_E_ARG, "disc=%d outside [0,%d)", disc, prm->n_disc);
    if (i_sel < 0 || i_sel + 2 >= prm->n_var)
        return fail(MDFS_E_ARG, "i_sel=%d: needs two larger variables below n_var=%lld", i_sel, (long long)prm->n_var);
    Problem P;
    if ((rc = setup(prm, y, ws, ws_bytes, stream, P))) return rc;
    if ((rc = run_sweep(P, data, y, counts, disc, nullptr, i_sel))) return rc;
    Status st;
    if ((rc = read_status(P, st))) return rc;
    g_err[0] = 0;
    return MDFS_OK;
}

extern "C" int mdfs_interesting_tuples(const mdfs_params *prm, const float *data, const uint8_t *y, double ig_thr,
                                       int32_t *var, int32_t *partners, int32_t *disc, double *ig, int64_t max_out,
                                       int64_t *n_found, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_params(prm);
    if (rc) return rc;
    if (prm->k == 1) return fail(MDFS_E_K, "k=1 has no tuples (mdfs_max_ig covers it)");
    if (prm->k >= 4) return fail(MDFS_E_K, "k=%d interesting tuples are not built (mdfs_max_ig covers k=4, 5)", prm->k);
    if (!data || !y || !ws || !n_found) return fail(MDFS_E_ARG, "null pointer");
    if (max_out < 0 || (max_out > 0 && (!var || !partners || !disc || !ig)))
        return fail(MDFS_E_ARG, "max_out=%lld with a null output array", (long long)max_out);
    if (!(ig_thr == ig_thr)) return fail(MDFS_E_ARG, "ig_thr is NaN");
    *n_found = 0;
    Problem P;
    if ((rc = setup(prm, y, ws, ws_bytes, stream, P))) return rc;
    LAUNCH(launch_init(P));
    if (P.k3_mfma) LAUNCH(launch_tiles3(P));
    LAUNCH(launch_class_perm(P, y));
    LAUNCH(launch_tables(P));
    LAUNCH(launch_encode(P, data));
    // one collect pass with every variable's threshold at ig_thr (the largest float32 not above
    // it): it appends every tuple whose float32 IG lies within the screen window of ig_thr,
    // a superset of those whose binary64 IG reaches it
    float t = (float)ig_thr;
    if ((double)t > ig_thr) t = nextafterf(t, -INFINITY);
    LAUNCH(launch_fill_g(P, f32_key(t)));
    LAUNCH(launch_collect_decide(P, true));
    if ((rc = sweep_pass(P, nullptr, -1, true))) return rc;
    Status st;
    if ((rc = read_status(P, st))) return rc;
    if (st.overflow) {
        *n_found = st.n_cand;
        return fail(MDFS_E_OVERFLOW, "more than %lld candidates near ig_thr; raise the threshold",
                    (long long)P.L.cap);
    }
    LAUNCH(launch_emit(P, ig_thr, var, partners, disc, ig, max_out));
    if ((rc = read_status(P, st))) return rc;
    *n_found = st.n_emit;
    g_err[0] = 0;
    return MDFS_OK;
}

extern "C" int mdfs_screen_max(const mdfs_params *prm, const float *data, const uint8_t *y, float *ig32,
                               double *err_bound, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_params(prm);
    if (rc) return rc;
    if (prm->k == 1) return fail(MDFS_E_K, "k=1 has no tuples (mdfs_max_ig covers it)");
    if (!data || !y || !ig32 || !ws) return fail(MDFS_E_ARG, "null pointer");
    Problem P;
    if ((rc = setup(prm, y, ws, ws_bytes, stream, P))) return rc;
    if ((rc = run_sweep(P, data, y, nullptr, -1))) return rc;
    LAUNCH(launch_screen_out(P, ig32));
    Status st;
    if ((rc = read_status(P, st))) return rc;
    if (err_bound) *err_bound = P.err_bound;
    g_err[0] = 0;
    return MDFS_OK;
}
