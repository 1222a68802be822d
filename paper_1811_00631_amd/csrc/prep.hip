// prep.hip -- everything before the tuple sweep: workspace layout, status/key initialisation,
// class-sorted object order, entropy lookup tables and the discretise+encode kernel.
//
// Discretisation follows the paper's randomised rank-based scheme (section "Algorithm and
// implementation", the paragraph on range and shares): per variable and discretisation,
// `divisions+1` shares drawn from U(1-range, 1+range) fix `divisions` cut positions in the
// sorted variable, and the values at those positions are the class thresholds.  Share and cut
// arithmetic is binary64 with explicitly rounded operations (no contraction), so every
// discretisation is reproducible bit for bit.
#include "mdfs_internal.h"

#include <algorithm>

#include <math.h>

namespace mdfs {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(int64_t N, int64_t p, int k, int divisions, int R, size_t pair_budget)
{
    Layout L{};
    L.N = N;
    L.p = p;
    L.p_pad = (p + VAR_PAD - 1) / VAR_PAD * VAR_PAD;
    L.k = k;
    L.C = divisions + 1;
    L.W = divisions;
    L.R = R;
    L.Kpad_max = (N + KOBJ_F4 - 1) / KOBJ_F4 * KOBJ_F4 + 2 * KOBJ_F4;
    L.rows_pad = L.p_pad * L.W;
    L.cap = (p * 256 > (1 << 20)) ? p * 256 : (1 << 20);
    L.words_max = (N + 31) / 32 + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.status = take(sizeof(Status));
    L.pos = take(sizeof(int32_t) * N);
    L.perm = take(sizeof(int32_t) * (size_t)L.Kpad_max);
    L.tabEA = take(sizeof(float) * (N + 1));
    L.tabEB = take(sizeof(float) * (N + 1));
    L.tabLQ = take(sizeof(float) * 2 * (N + 1));
    L.marg = take(sizeof(uint32_t) * (size_t)R * L.p_pad * L.C);
    L.F1 = take(sizeof(float) * (size_t)R * L.p_pad);
    // >= one byte per position; k = 1 needs no tuple encoding, only binary64 F of each variable
    L.onehot = take((k == 1 || k >= 4) ? 0 : (size_t)R * L.Kpad_max * L.rows_pad);
    L.F1d = take(k == 1 ? sizeof(double) * (size_t)R * L.p_pad : 0);
    L.G32 = take(sizeof(uint32_t) * L.p_pad);
    L.max64 = take(sizeof(uint64_t) * L.p_pad);
    L.keyw = take(sizeof(uint64_t) * L.p_pad);
    L.ovf = take(sizeof(uint32_t) * L.p_pad);
    L.cand = take(sizeof(Cand) * L.cap);
    L.ig64 = take(sizeof(double) * L.cap);
    if (k >= 4) {
        // bitsets (the bitset sweeps of k = 4 and of k = 5 with two classes) and class-sorted
        // codes [R][p][N] (the histogram sweep and the binary64 re-score of k >= 4)
        L.bits = take(uses_bits(L) ? sizeof(uint32_t) * (size_t)R * 2 * L.words_max * L.p_pad * L.W : 0);
        L.ccodes = take((size_t)R * p * N);
        L.ptab = L.F2 = L.a3pref = L.a3blk = o;
    } else if (k == 3) {
        L.bits = take(sizeof(uint32_t) * (size_t)R * 2 * L.words_max * L.p_pad * L.W);
        // the pair data of up to RC discretisations (at most pair_budget bytes, at least one): one
        // launch of the pair sweep and one of the triple sweep per chunk of discretisations
        const size_t per_r = (size_t)L.p_pad * L.p_pad * (sizeof(uint32_t) * L.W * L.W + sizeof(float));
        L.RC = (int)std::min<size_t>((size_t)R, std::max<size_t>(1, pair_budget / per_r));
        L.ptab = take(sizeof(uint32_t) * (size_t)L.RC * L.p_pad * L.p_pad * L.W * L.W);
        L.F2 = take(sizeof(float) * (size_t)L.RC * L.p_pad * L.p_pad);
        const int64_t n_ablk_max = L.p_pad * ((L.p_pad + 31) / 32);
        L.a3pref = take(sizeof(int64_t) * (size_t)(n_ablk_max + 1));
        L.a3blk = take(sizeof(int32_t) * (size_t)n_ablk_max);
    } else {
        L.bits = L.ptab = L.F2 = L.a3pref = L.a3blk = o;
    }
    if (k < 4) L.ccodes = o;
    L.total = o;
    return L;
}

// ------------------------------------------------------------------ init
__global__ void k_init(Status *st, uint32_t *G32, uint64_t *max64, uint64_t *keyw, uint32_t *ovf,
                       uint32_t *marg, float *F1, int64_t p_pad, int64_t n_marg)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (i < (int64_t)(sizeof(Status) / 4)) reinterpret_cast<uint32_t *>(st)[i] = 0;
    for (int64_t v = i; v < p_pad; v += stride) {
        G32[v] = 0x007fffffu; // key of -inf
        max64[v] = 0ull;
        keyw[v] = ~0ull;
        ovf[v] = 0u;
    }
    for (int64_t j = i; j < n_marg; j += stride) marg[j] = 0u;
    (void)F1;
}

// Before a collect pass: empty the candidate buffer and the overflow marks, keep the maxima.
__global__ void k_reset_candidates(Status *st, uint32_t *ovf, int64_t p_pad, int gated)
{
    if (gated && st->collect_go == 0) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i == 0) { st->n_cand = 0; st->overflow = 0; }
    for (int64_t v = i; v < p_pad; v += (int64_t)gridDim.x * blockDim.x) ovf[v] = 0u;
}

__global__ void k_reset_queue(Status *st)
{
    if (threadIdx.x < 16) st->next_tile[threadIdx.x] = 0u;
}

__global__ void k_fill_g(uint32_t *G32, int64_t p_pad, uint32_t key)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < p_pad; v += (int64_t)gridDim.x * blockDim.x)
        G32[v] = key;
}

hipError_t launch_fill_g(const Problem &P, uint32_t key)
{
    hipLaunchKernelGGL(k_fill_g, dim3(64), dim3(256), 0, P.stream, P.at<uint32_t>(P.L.G32), P.L.p_pad, key);
    return hipGetLastError();
}

hipError_t launch_reset_queue(const Problem &P)
{
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, P.stream, P.at<Status>(P.L.status));
    return hipGetLastError();
}

hipError_t launch_reset_candidates(const Problem &P, bool gated)
{
    hipLaunchKernelGGL(k_reset_candidates, dim3(64), dim3(256), 0, P.stream, P.at<Status>(P.L.status),
                       P.at<uint32_t>(P.L.ovf), P.L.p_pad, gated ? 1 : 0);
    return hipGetLastError();
}

__global__ void k_collect_decide(Status *st, int force)
{
    if (threadIdx.x == 0) st->collect_go = (force || st->overflow) ? 1u : 0u;
}

hipError_t launch_collect_decide(const Problem &P, bool force)
{
    hipLaunchKernelGGL(k_collect_decide, dim3(1), dim3(64), 0, P.stream, P.at<Status>(P.L.status), force ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_init(const Problem &P)
{
    const Layout &L = P.L;
    int64_t n_marg = (int64_t)L.R * L.p_pad * L.C;
    int grid = (int)((L.p_pad + 255) / 256);
    if (grid < 64) grid = 64;
    hipLaunchKernelGGL(k_init, dim3(grid), dim3(256), 0, P.stream, P.at<Status>(L.status),
                       P.at<uint32_t>(L.G32), P.at<uint64_t>(L.max64), P.at<uint64_t>(L.keyw),
                       P.at<uint32_t>(L.ovf), P.at<uint32_t>(L.marg), P.at<float>(L.F1), L.p_pad, n_marg);
    return hipGetLastError();
}

// ------------------------------------------------------------------ class-sorted order
// One workgroup: pos[n] = position of object n in the class-sorted order (class 0 first, each
// class in original order, class 1 starting at K0pad); perm[position] = object or -1 (padding).
__global__ __launch_bounds__(1024) void k_class_perm(const uint8_t *__restrict__ y, int N, int K0pad,
                                                     int Kpad, int32_t *pos, int32_t *perm, int64_t n1_check,
                                                     Status *st)
{
    __shared__ int s1[1024];
    const int t = threadIdx.x, T = blockDim.x;
    for (int i = t; i < Kpad; i += T) perm[i] = -1;
    const int chunk = (N + T - 1) / T;
    const int lo = t * chunk, hi = min(N, lo + chunk);
    int ones = 0, bad = 0;
    for (int n = lo; n < hi; ++n) {
        ones += y[n] != 0;
        bad |= y[n] > 1;
    }
    s1[t] = ones;
    __syncthreads();
    // exclusive scan (Hillis-Steele on a copy is enough for 1024 entries)
    for (int off = 1; off < T; off <<= 1) {
        int v = (t >= off) ? s1[t - off] : 0;
        __syncthreads();
        s1[t] += v;
        __syncthreads();
    }
    int ones_before = s1[t] - ones;
    int zeros_before = (lo < N ? lo : N) - ones_before;
    const int total_ones = s1[T - 1];
    const int any_bad = __syncthreads_or(bad);
    if (n1_check >= 0 && (any_bad || total_ones != n1_check)) {
        // the class sizes the launch was sized for are wrong: flag it and write no positions
        // (perm stays all padding, so the sweeps count nothing and touch nothing out of range)
        if (t == 0) st->y_flag = 1u;
        return;
    }
    __syncthreads();   // every perm[i] = -1 above is visible before the positions are written
    for (int n = lo; n < hi; ++n) {
        int p;
        if (y[n]) p = K0pad + ones_before++;
        else p = zeros_before++;
        pos[n] = p;
        perm[p] = n;
    }
}

hipError_t launch_class_perm(const Problem &P, const uint8_t *y, int64_t n1_check)
{
    hipLaunchKernelGGL(k_class_perm, dim3(1), dim3(1024), 0, P.stream, y, (int)P.L.N, P.K0pad,
                       P.Kpad, P.at<int32_t>(P.L.pos), P.at<int32_t>(P.L.perm), n1_check, P.at<Status>(P.L.status));
    return hipGetLastError();
}

// ------------------------------------------------------------------ entropy tables
// For one voxel with n0 objects of class 0, n1 of class 1 and n = n0 + n1, the pseudocounted
// class probabilities are p^d = (n^d + beta^d) / (n + beta), beta = beta0 + beta1, and
//     n h(p) = n ln(n + beta) - n/(n + beta) * [ E(n0 + beta0) + E(n1 + beta1) ],  E(x) = x ln x.
// EA[n0] = E(n0 + beta0), EB[n1] = E(n1 + beta1), LQ[n] = (n ln(n + beta), n / (n + beta)).
// Evaluated in binary64, stored as float32 (the float32 screen of the sweep).
__device__ inline double xlogx(double x) { return x > 0.0 ? x * log(x) : 0.0; }

__global__ void k_tables(int N, int N0, int N1, double b0, double b1, float *EA, float *EB, float2 *LQ)
{
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n > N) return;
    EA[n] = n <= N0 ? (float)xlogx(n + b0) : 0.0f;
    EB[n] = n <= N1 ? (float)xlogx(n + b1) : 0.0f;
    double s = n + b0 + b1;
    LQ[n] = n > 0 ? make_float2((float)(n * log(s)), (float)(n / s)) : make_float2(0.f, 0.f);
}

hipError_t launch_tables(const Problem &P)
{
    int N = (int)P.L.N;
    hipLaunchKernelGGL(k_tables, dim3((N + 256) / 256), dim3(256), 0, P.stream, N, P.N0, P.N1, P.beta0,
                       P.beta1, P.at<float>(P.L.tabEA), P.at<float>(P.L.tabEB), P.at<float2>(P.L.tabLQ));
    return hipGetLastError();
}

// ------------------------------------------------------------------ discretise + encode
// SplitMix64 (Steele, Lea & Flood 2014): state advances by the golden gamma, output is the
// variant-13 style finaliser.  The draw for (seed, disc, var, j) absorbs each key component
// with one step whose state is the previous output plus (component + 1) * gamma.
__device__ inline uint64_t sm64_fin(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__device__ inline uint64_t share_bits(uint64_t seed, uint64_t disc, uint64_t var, uint64_t j)
{
    const uint64_t g = 0x9e3779b97f4a7c15ull;
    uint64_t h = sm64_fin(seed + g);
    h = sm64_fin(h + (disc + 1) * g);
    h = sm64_fin(h + (var + 1) * g);
    return sm64_fin(h + (j + 1) * g);
}

// Cut positions of one (discretisation, variable): c shares, cumulative sums, t_j =
// floor(N cum_j / S) kept in [1, N-1], strictly increasing and leaving room for later classes.
template <int C>
__device__ void cut_positions(int N, double range, uint64_t seed, uint64_t disc, uint64_t var, int *t)
{
    double s[C];
    const double lo = __dsub_rn(1.0, range), width = __dmul_rn(2.0, range);
    for (int j = 0; j < C; ++j) {
        double u = __dmul_rn((double)(share_bits(seed, disc, var, (uint64_t)j) >> 11), 0x1.0p-53);
        s[j] = __dadd_rn(lo, __dmul_rn(width, u));
    }
    double S = 0.0;
    for (int j = 0; j < C; ++j) S = __dadd_rn(S, s[j]);
    double cum = 0.0;
    int prev = 0;
    for (int j = 1; j < C; ++j) {
        cum = __dadd_rn(cum, s[j - 1]);
        double qv = __ddiv_rn(__dmul_rn((double)N, cum), S);
        int tj = (int)floor(qv);
        tj = max(tj, 1);
        tj = min(tj, N - 1);
        if (j > 1) tj = max(tj, prev + 1);
        tj = min(tj, N - (C - j));
        t[j - 1] = tj;
        prev = tj;
    }
}

template <int C>
__device__ inline int code_of(float x, const float *thr)
{
    int c = 0;
#pragma unroll
    for (int j = 0; j < C - 1; ++j) c += (x >= thr[j]) ? 1 : 0;
    return c;
}

constexpr int DISC_THREADS = 256;   // 4 waves: more variables in flight per CU (512: 2.1 ms, 256: 1.5 ms at the headline)
constexpr int DISC_RCHUNK = 256;   // discretisations whose thresholds are staged at once

// Value of rank k (0-based) in the union of two ascending arrays A[na], B[nb] (k < na + nb):
// merge-path selection.  The number i of A elements among the k+1 smallest (A first on ties)
// is the count of i with A[i] <= B[k-i], a predicate that holds for a prefix of the feasible
// range [max(0, k+1-nb), min(k+1, na)); the answer is the larger of the last element taken
// from each side.  Equal to sort(A u B)[k].
__device__ inline float kth_of_two(const float *A, int na, const float *B, int nb, int k)
{
    int lo = max(0, k + 1 - nb), hi = min(k + 1, na);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A[mid] <= B[k - mid]) lo = mid + 1;
        else hi = mid;
    }
    if (lo == 0) return B[k];
    if (k - lo < 0) return A[lo - 1];
    return fmaxf(A[lo - 1], B[k - lo]);
}

// Number of elements of the ascending array A[n] that are < v.
__device__ inline int count_below(const float *A, int n, float v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One workgroup per variable.  LDS: xcs[Kpad] (the variable in class-sorted order, for the
// encodings), srt[N] (class 0's values then class 1's, each sorted ascending; one segment of N
// values when the class order is not given), thresholds of a chunk of discretisations.
// Threshold q_j is the value of rank t_j of the whole variable, selected from the two sorted
// classes; the per-class counts at or above each threshold come from binary searches, so the
// marginals cost O(c log N) per discretisation.  Outputs (each optional): codes in original
// object order, one-hot rows in class-sorted order, per-class marginal counts packed
// (n1 << 16 | n0), and F1 = N H(y|x).
template <int C>
__global__ __launch_bounds__(DISC_THREADS) void k_discretize(
    const float *__restrict__ data, int N, int p, int R, int disc_offset, double range,
    uint64_t seed, const int32_t *__restrict__ perm, int K0pad, int N0, int N1, int KB, int Kpad, int fp4,
    int64_t rows_pad, uint8_t *__restrict__ codes, int8_t *__restrict__ onehot,
    uint32_t *__restrict__ marg, float *__restrict__ F1, double *__restrict__ F1d, int64_t p_pad, double b0,
    double b1, Status *st,
    uint32_t *__restrict__ bits, int64_t words_max, uint8_t *__restrict__ ccodes)
{
    constexpr int W = C - 1;
    extern __shared__ float lds[];
    float *xcs = lds;                       // [Kpad]
    float *srt = xcs + Kpad;                // [N]
    float *thr = srt + N;                   // [DISC_RCHUNK][C-1]
    __shared__ int hist[DISC_RCHUNK * 2 * C];
    __shared__ double fterm[DISC_RCHUNK * C];
    const int v = blockIdx.x;
    const int t = threadIdx.x;
    if (v >= p) {
        // padding variable (encode launches cover p_pad): zero one-hot rows, so the sweeps
        // count 0 for it
        if (!onehot) return;
        const int nrow = KB * W * (KBLK / 4);
        for (int rr = 0; rr < R; ++rr)
            for (int idx = t; idx < nrow; idx += DISC_THREADS) {
                const int kb = idx / (W * (KBLK / 4)), a = (idx / (KBLK / 4)) % W, q4 = idx % (KBLK / 4);
                *reinterpret_cast<uint32_t *>(onehot + onehot_off(rr, (int64_t)v * W + a, kb, q4 * 4, KB, rows_pad)) = 0u;
            }
        return;
    }
    const float *x = data + (int64_t)v * N;
    // segments of srt: [0, n0) and [n0, n0 + n1)
    const int n0 = perm ? N0 : N, n1 = perm ? N1 : 0;

    bool bad = false;
    if (perm) {
        for (int i = t; i < Kpad; i += DISC_THREADS) {
            const int n = perm[i];
            const float val = n >= 0 ? x[n] : 0.0f;
            bad |= (val != val);
            xcs[i] = val;
            if (i < N0) srt[i] = val;
            else if (i >= K0pad && i < K0pad + N1) srt[N0 + i - K0pad] = val;
        }
    } else {
        for (int i = t; i < N; i += DISC_THREADS) {
            const float val = x[i];
            bad |= (val != val);
            srt[i] = val;
        }
    }
    if (bad) atomicOr(&st->nan_flag, 1u);
    __syncthreads();

    // Both segments sorted ascending by one bitonic network each (the form whose first step at
    // every merge size compares mirrored positions, so every compare-exchange is ascending).
    // A segment of n values runs the network of the next power of two with virtual +inf
    // padding; a pair whose upper index is >= n never exchanges, so it is skipped.
    {
        int m0 = 1, m1 = 1;
        while (m0 < n0) m0 <<= 1;
        while (m1 < n1) m1 <<= 1;
        if (n1 == 0) m1 = 0;
        const int mx = max(m0, m1);
        for (int kk = 2; kk <= mx; kk <<= 1) {
            const int h0 = kk <= m0 ? m0 >> 1 : 0, h1 = kk <= m1 ? m1 >> 1 : 0;
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int q = t; q < h0 + h1; q += DISC_THREADS) {
                    const bool sg = q >= h0;
                    const int qq = sg ? q - h0 : q, n = sg ? n1 : n0;
                    float *a = srt + (sg ? n0 : 0);
                    const int i = ((qq & ~(j - 1)) << 1) | (qq & (j - 1));
                    const int partner = (j == (kk >> 1)) ? (i ^ (kk - 1)) : (i + j);
                    if (partner < n) {
                        const float lo_v = a[i], hi_v = a[partner];
                        if (lo_v > hi_v) {
                            a[i] = hi_v;
                            a[partner] = lo_v;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }

    for (int rb = 0; rb < R; rb += DISC_RCHUNK) {
        const int nr = min(DISC_RCHUNK, R - rb);
        // thresholds, and per class the count of values >= each threshold (hist[.., j + 1])
        for (int i = t; i < nr * (C - 1); i += DISC_THREADS) {
            const int rr = i / (C - 1), j = i % (C - 1);
            int tc[C - 1];
            cut_positions<C>(N, range, seed, (uint64_t)(disc_offset + rb + rr), (uint64_t)v, tc);
            const float q = kth_of_two(srt, n0, srt + n0, n1, tc[j]);
            thr[rr * (C - 1) + j] = q;
            hist[(rr * 2 + 0) * C + j + 1] = n0 - count_below(srt, n0, q);
            hist[(rr * 2 + 1) * C + j + 1] = n1 - count_below(srt + n0, n1, q);
        }
        __syncthreads();
        for (int rr = 0; rr < nr; ++rr) {
            const int r = rb + rr;
            const float *th = thr + rr * (C - 1);
            if (codes) {
                uint8_t *out = codes + ((int64_t)r * p + v) * N;
                for (int n = t; n < N; n += DISC_THREADS) out[n] = (uint8_t)code_of<C>(x[n], th);
            }
        }
        if (onehot) {
            // a thread per group of `per` consecutive class-sorted positions (one dword of a
            // (K block, bin) row chunk: one byte (int8 1) or one nibble (E2M1 2.0) each): the
            // codes are taken once per position and scattered into the W rows' dwords
            const int per = fp4 ? 8 : 4;
            const int ngrp = KB * (KBLK / 4);
            for (int g = t; g < ngrp; g += DISC_THREADS) {
                const int kb = g / (KBLK / 4), q4 = g % (KBLK / 4);
                float xv[8];
                bool ok[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int ps = g * per + e;
                    ok[e] = e < per && ((ps < N0) || (ps >= K0pad && ps < K0pad + N1));
                    xv[e] = ok[e] ? xcs[ps] : 0.0f;
                }
                for (int rr = 0; rr < nr; ++rr) {
                    const float *th = thr + rr * (C - 1);
                    uint32_t word[W];
#pragma unroll
                    for (int a = 0; a < W; ++a) word[a] = 0;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int c = ok[e] ? code_of<C>(xv[e], th) : W;
                        const uint32_t bit = fp4 ? (F4_TWO << (4 * e)) : (1u << (8 * e));
#pragma unroll
                        for (int a = 0; a < W; ++a) word[a] |= (c == a) ? bit : 0u;
                    }
#pragma unroll
                    for (int a = 0; a < W; ++a) {
                        const int64_t off = onehot_off(rb + rr, (int64_t)v * W + a, kb, q4 * 4, KB, rows_pad);
                        *reinterpret_cast<uint32_t *>(onehot + off) = word[a];
                    }
                }
            }
        }
        if (bits) {
            for (int rr = 0; rr < nr; ++rr) {
                const int r = rb + rr;
                const float *th = thr + rr * (C - 1);
                // bitset word w of class y: class-sorted positions y_off + 32w .. +31, bin a
                const int w0 = (N0 + 31) / 32, w1 = (N1 + 31) / 32;
                for (int idx = t; idx < (w0 + w1) * W; idx += DISC_THREADS) {
                    const int a = idx % W, wy = idx / W;
                    const int y = wy < w0 ? 0 : 1, w = y ? wy - w0 : wy;
                    const int base_ps = (y ? K0pad : 0) + 32 * w, ny = y ? N1 : N0;
                    uint32_t word = 0;
                    for (int e = 0; e < 32; ++e) {
                        const bool valid = 32 * w + e < ny;
                        const bool hit = valid && code_of<C>(xcs[base_ps + e], th) == a;
                        word |= (hit ? 1u : 0u) << e;
                    }
                    bits[((((int64_t)r * 2 + y) * words_max + w) * p_pad + v) * W + a] = word;
                }
            }
        }
        if (ccodes) {
            // class-sorted codes without padding: class 0's objects, then class 1's
            for (int rr = 0; rr < nr; ++rr) {
                const float *th = thr + rr * (C - 1);
                uint8_t *out = ccodes + ((int64_t)(rb + rr) * p + v) * N;
                for (int ps = t; ps < N0 + N1; ps += DISC_THREADS)
                    out[ps] = (uint8_t)code_of<C>(xcs[ps < N0 ? ps : K0pad + ps - N0], th);
            }
        }
        if (marg || F1) {
            // bin a of class d holds G_d(a) - G_d(a+1) values, G_d(a) = count >= threshold a
            // (G_d(0) = n_d, G_d(C) = 0); packed marginals and the F terms of every (r, bin)
            for (int i = t; i < nr * C; i += DISC_THREADS) {
                const int rr = i / C, a = i % C, r = rb + rr;
                const int *g0 = hist + (rr * 2 + 0) * C, *g1 = hist + (rr * 2 + 1) * C;
                const int h0 = (a == 0 ? n0 : g0[a]) - (a + 1 < C ? g0[a + 1] : 0);
                const int h1 = (a == 0 ? n1 : g1[a]) - (a + 1 < C ? g1[a + 1] : 0);
                if (marg) marg[((int64_t)r * p_pad + v) * C + a] = ((uint32_t)h1 << 16) | (uint32_t)h0;
                const double d0 = h0, d1 = h1, n = d0 + d1;
                double term = 0.0;
                if (n > 0) {
                    const double sden = n + b0 + b1;
                    term = n * log(sden) - (n / sden) * (xlogx(d0 + b0) + xlogx(d1 + b1));
                }
                fterm[i] = term;
            }
            __syncthreads();
            if (F1)
                for (int rr = t; rr < nr; rr += DISC_THREADS) {
                    double Fv = 0.0;
                    for (int a = 0; a < C; ++a) Fv += fterm[rr * C + a];
                    F1[(int64_t)(rb + rr) * p_pad + v] = (float)Fv;
                    if (F1d) F1d[(int64_t)(rb + rr) * p_pad + v] = Fv;
                }
        }
        __syncthreads();
    }
}

template <int C>
static hipError_t disc_launch(const Problem &P, const float *data, uint8_t *codes, bool encode)
{
    const Layout &L = P.L;
    const int N = (int)L.N;
    const int Kpad = P.Kpad;
    size_t lds = sizeof(float) * ((size_t)Kpad + N + DISC_RCHUNK * (C - 1));
    auto kern = k_discretize<C>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int64_t nblk = encode ? L.p_pad : L.p;   // encode: also zero the padding variables' rows
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(DISC_THREADS), lds, P.stream, data, N, (int)L.p,
                       L.R, P.disc_offset, P.range, P.seed, encode ? P.at<int32_t>(L.perm) : nullptr, P.K0pad, P.N0, P.N1, P.KB,
                       P.Kpad, P.fp4 ? 1 : 0, L.rows_pad, codes,
                       (encode && (L.k == 2 || L.k == 3)) ? P.at<int8_t>(L.onehot) : nullptr,
                       encode ? P.at<uint32_t>(L.marg) : nullptr, encode ? P.at<float>(L.F1) : nullptr,
                       (encode && L.k == 1) ? P.at<double>(L.F1d) : nullptr, L.p_pad, P.beta0, P.beta1, P.at<Status>(L.status),
                       (encode && uses_bits(L)) ? P.at<uint32_t>(L.bits) : nullptr, L.words_max,
                       (encode && L.k >= 4) ? P.at<uint8_t>(L.ccodes) : nullptr);
    return hipGetLastError();
}

// Encoding from caller-supplied codes [R][p][N] (values 0 .. C-1): one workgroup per variable,
// per discretisation the codes gathered into class-sorted order in LDS, then the same outputs as
// the encoding half of k_discretize (one-hot rows, bitsets, packed per-class marginals, F1).  A
// code >= C raises the status flag (the call then fails); it matches no bin.
template <int C>
__global__ __launch_bounds__(DISC_THREADS) void k_encode_codes(
    const uint8_t *__restrict__ codes, int N, int p, int R, const int32_t *__restrict__ perm, int K0pad, int N0,
    int N1, int KB, int Kpad, int fp4, int64_t rows_pad, int8_t *__restrict__ onehot, uint32_t *__restrict__ marg,
    float *__restrict__ F1, double *__restrict__ F1d, int64_t p_pad, double b0, double b1, Status *st,
    uint32_t *__restrict__ bits, int64_t words_max, uint8_t *__restrict__ ccodes)
{
    constexpr int W = C - 1;
    extern __shared__ uint8_t cls[];        // [Kpad] codes in class-sorted order; C at padding
    __shared__ int hist[2 * C];
    __shared__ double fterm[C];
    const int v = blockIdx.x;
    const int t = threadIdx.x;
    if (v >= p) {
        if (!onehot) return;
        const int nrow = KB * W * (KBLK / 4);
        for (int rr = 0; rr < R; ++rr)
            for (int idx = t; idx < nrow; idx += DISC_THREADS) {
                const int kb = idx / (W * (KBLK / 4)), a = (idx / (KBLK / 4)) % W, q4 = idx % (KBLK / 4);
                *reinterpret_cast<uint32_t *>(onehot + onehot_off(rr, (int64_t)v * W + a, kb, q4 * 4, KB, rows_pad)) = 0u;
            }
        return;
    }
    for (int r = 0; r < R; ++r) {
        const uint8_t *cv = codes + ((int64_t)r * p + v) * N;
        bool bad = false;
        for (int i = t; i < Kpad; i += DISC_THREADS) {
            const int n = perm[i];
            const uint8_t c = n >= 0 ? cv[n] : (uint8_t)C;
            bad |= n >= 0 && c >= C;
            cls[i] = c;
        }
        if (t < 2 * C) hist[t] = 0;
        if (bad) atomicOr(&st->code_flag, 1u);
        __syncthreads();
        if (onehot) {
            const int per = fp4 ? 8 : 4;
            for (int g = t; g < KB * (KBLK / 4); g += DISC_THREADS) {
                const int kb = g / (KBLK / 4), q4 = g % (KBLK / 4);
                uint32_t word[W];
#pragma unroll
                for (int a = 0; a < W; ++a) word[a] = 0;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    if (e >= per) break;
                    const int c = cls[g * per + e];
                    const uint32_t bit = fp4 ? (F4_TWO << (4 * e)) : (1u << (8 * e));
#pragma unroll
                    for (int a = 0; a < W; ++a) word[a] |= (c == a) ? bit : 0u;
                }
#pragma unroll
                for (int a = 0; a < W; ++a)
                    *reinterpret_cast<uint32_t *>(onehot + onehot_off(r, (int64_t)v * W + a, kb, q4 * 4, KB, rows_pad)) =
                        word[a];
            }
        }
        if (bits) {
            const int w0 = (N0 + 31) / 32, w1 = (N1 + 31) / 32;
            for (int idx = t; idx < (w0 + w1) * W; idx += DISC_THREADS) {
                const int a = idx % W, wy = idx / W;
                const int y = wy < w0 ? 0 : 1, w = y ? wy - w0 : wy;
                const int base_ps = (y ? K0pad : 0) + 32 * w, ny = y ? N1 : N0;
                uint32_t word = 0;
                for (int e = 0; e < 32; ++e) {
                    const bool hit = 32 * w + e < ny && cls[base_ps + e] == a;
                    word |= (hit ? 1u : 0u) << e;
                }
                bits[((((int64_t)r * 2 + y) * words_max + w) * p_pad + v) * W + a] = word;
            }
        }
        if (ccodes) {
            uint8_t *out = ccodes + ((int64_t)r * p + v) * N;
            // a code above divisions fails the call (code_flag); it is clamped so that no kernel
            // indexes past its C^k cells meanwhile
            for (int ps = t; ps < N0 + N1; ps += DISC_THREADS) {
                const uint8_t c = cls[ps < N0 ? ps : K0pad + ps - N0];
                out[ps] = c < C ? c : (uint8_t)(C - 1);
            }
        }
        if (marg || F1) {
            int loc[2][C];
#pragma unroll
            for (int a = 0; a < C; ++a) loc[0][a] = loc[1][a] = 0;
            for (int i = t; i < Kpad; i += DISC_THREADS) {
                const int c = cls[i], y = i >= K0pad ? 1 : 0;
#pragma unroll
                for (int a = 0; a < C; ++a) {
                    loc[0][a] += (c == a && y == 0) ? 1 : 0;
                    loc[1][a] += (c == a && y == 1) ? 1 : 0;
                }
            }
#pragma unroll
            for (int a = 0; a < C; ++a) {
                if (loc[0][a]) atomicAdd(&hist[a], loc[0][a]);
                if (loc[1][a]) atomicAdd(&hist[C + a], loc[1][a]);
            }
            __syncthreads();
            if (t < C) {
                const int h0 = hist[t], h1 = hist[C + t];
                if (marg) marg[((int64_t)r * p_pad + v) * C + t] = ((uint32_t)h1 << 16) | (uint32_t)h0;
                const double d0 = h0, d1 = h1, n = d0 + d1;
                double term = 0.0;
                if (n > 0) {
                    const double sden = n + b0 + b1;
                    term = n * log(sden) - (n / sden) * (xlogx(d0 + b0) + xlogx(d1 + b1));
                }
                fterm[t] = term;
            }
            __syncthreads();
            if (t == 0 && F1) {
                double Fv = 0.0;
                for (int a = 0; a < C; ++a) Fv += fterm[a];
                F1[(int64_t)r * p_pad + v] = (float)Fv;
                if (F1d) F1d[(int64_t)r * p_pad + v] = Fv;
            }
        }
        __syncthreads();   // cls and hist are rewritten for the next discretisation
    }
}

template <int C>
static hipError_t encode_codes_launch(const Problem &P)
{
    const Layout &L = P.L;
    auto kern = k_encode_codes<C>;
    hipLaunchKernelGGL(kern, dim3((unsigned)L.p_pad), dim3(DISC_THREADS), (size_t)P.Kpad, P.stream, P.codes_in,
                       (int)L.N, (int)L.p, L.R, P.at<int32_t>(L.perm), P.K0pad, P.N0, P.N1, P.KB, P.Kpad,
                       P.fp4 ? 1 : 0, L.rows_pad, (L.k == 2 || L.k == 3) ? P.at<int8_t>(L.onehot) : nullptr,
                       P.at<uint32_t>(L.marg), P.at<float>(L.F1), L.k == 1 ? P.at<double>(L.F1d) : nullptr, L.p_pad,
                       P.beta0, P.beta1, P.at<Status>(L.status), uses_bits(L) ? P.at<uint32_t>(L.bits) : nullptr,
                       L.words_max, L.k >= 4 ? P.at<uint8_t>(L.ccodes) : nullptr);
    return hipGetLastError();
}

hipError_t launch_encode_codes(const Problem &P)
{
    switch (P.L.C) {
    case 2: return encode_codes_launch<2>(P);
    case 3: return encode_codes_launch<3>(P);
    case 5: return encode_codes_launch<5>(P);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_discretize(const Problem &P, const float *data, uint8_t *codes, bool encode)
{
    switch (P.L.C) {
    case 2: return disc_launch<2>(P, data, codes, encode);
    case 3: return disc_launch<3>(P, data, codes, encode);
    case 5: return disc_launch<5>(P, data, codes, encode);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mdfs
