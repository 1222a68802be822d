// finalize.hip -- binary64 re-score of the sweep's candidates and the argmax tie rule.
//
// The sweep keeps, for each variable, its float32 maximum G and appends every (tuple,
// discretisation) whose float32 IG may lie within 2E + tau of the final maximum (E = proven
// float32 error bound, tau = the tie tolerance).  Here each surviving candidate's table is
// recounted exactly from the class-sorted one-hot encoding and its IG evaluated in binary64
// (equation IGmax with the pseudocounted entropies of section "Algorithm and implementation"),
// the maximum is taken over those values, and among candidates within tau of it the smallest
// discretisation index, then the lexicographically smallest partner tuple, wins.
#include "mdfs_internal.h"

namespace mdfs {

__device__ inline double xlogx64(double x) { return x > 0.0 ? x * log(x) : 0.0; }

// n h(p) for one voxel in binary64 (n = n0 + n1 objects, pseudocounts b0, b1).
__device__ inline double voxel64(double n0, double n1, double b0, double b1)
{
    const double n = n0 + n1;
    if (n == 0.0) return 0.0;
    const double s = n + b0 + b1;
    return n * log(s) - (n / s) * (xlogx64(n0 + b0) + xlogx64(n1 + b1));
}

__device__ inline float window32(float w_abs, float g)
{
    float ag = fabsf(g);
    return w_abs + 2e-9f * (ag > 1.f ? ag : 1.f) + 1e-30f;
}

__device__ inline int wave_sum(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Code of variable v at position e of K block kb, read back from its one-hot rows (the last
// bin has no row: none of the W rows set).  int8: byte e; fp4: nibble e of the row chunk.
template <int W>
__device__ inline int code_from_onehot(const int8_t *onehot, int r, int kb, int KB, int64_t rows_pad, int64_t v,
                                       int e, bool fp4)
{
    const int byte = fp4 ? (e >> 1) : e, sh = fp4 ? 4 * (e & 1) : 0;
    int c = W;
#pragma unroll
    for (int a = W - 1; a >= 0; --a)
        if ((onehot[onehot_off(r, v * W + a, kb, byte, KB, rows_pad)] >> sh) & 0xf) c = a;
    return c;
}

struct RescoreArgs {
    const Cand *cand;
    const Status *st;
    int64_t cap;
    const uint32_t *G32;
    float w_abs;
    const int8_t *onehot;
    int64_t rows_pad;
    int KB, K0pad, Kpad, N0, N1, kobj;
    bool fp4;
    double b0, b1;
    double *ig64;
    uint64_t *max64;
    int k;
};

// One wave per candidate (grid-stride).  k = 2: table of (v, m); k = 3: table of (v, m1, m2).
// (k >= 4: k_rescore_hist, which recounts from the class-sorted codes into an LDS histogram.)
template <int C, int K>
__global__ __launch_bounds__(256) void k_rescore(RescoreArgs a)
{
    constexpr int W = C - 1;
    static_assert(K == 2 || K == 3, "k >= 4 is re-scored by k_rescore_hist");
    constexpr int NC = (K == 2) ? C * C : C * C * C;
    const int lane = threadIdx.x & 63;
    const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nc = min((int64_t)a.st->n_cand, a.cap);
    for (int64_t ci = wid; ci < nc; ci += nw) {
        const Cand x = a.cand[ci];
        const float g = key_f32(a.G32[x.v]);
        if (!(x.ig32 >= g - window32(a.w_abs, g))) {
            if (lane == 0) a.ig64[ci] = -INFINITY;
            continue;
        }
        int64_t m1, m2 = 0;
        if (K == 2) m1 = x.partner;
        else { m1 = x.partner >> 16; m2 = x.partner & 0xffff; }
        int cnt[2][NC];
#pragma unroll
        for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int c = 0; c < NC; ++c) cnt[d][c] = 0;
        for (int ps = lane; ps < a.Kpad; ps += 64) {
            const int kb = ps / a.kobj, e = ps % a.kobj;
            const bool c0 = ps < a.K0pad;
            const bool valid = c0 ? (ps < a.N0) : (ps - a.K0pad < a.N1);
            int cell = code_from_onehot<W>(a.onehot, x.r, kb, a.KB, a.rows_pad, x.v, e, a.fp4) * C +
                       code_from_onehot<W>(a.onehot, x.r, kb, a.KB, a.rows_pad, m1, e, a.fp4);
            if (K >= 3) cell = cell * C + code_from_onehot<W>(a.onehot, x.r, kb, a.KB, a.rows_pad, m2, e, a.fp4);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                cnt[0][c] += (valid && c0 && cell == c) ? 1 : 0;
                cnt[1][c] += (valid && !c0 && cell == c) ? 1 : 0;
            }
        }
#pragma unroll
        for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int c = 0; c < NC; ++c) cnt[d][c] = wave_sum(cnt[d][c]);
        if (lane == 0) {
            // F of the full table (v first axis) and of the parent = table marginalised over v
            double Ft = 0.0, Fp = 0.0;
            constexpr int PC = NC / C;
            for (int c = 0; c < NC; ++c) Ft += voxel64(cnt[0][c], cnt[1][c], a.b0, a.b1);
            for (int pc = 0; pc < PC; ++pc) {
                int s0 = 0, s1 = 0;
                for (int cv = 0; cv < C; ++cv) { s0 += cnt[0][cv * PC + pc]; s1 += cnt[1][cv * PC + pc]; }
                Fp += voxel64(s0, s1, a.b0, a.b1);
            }
            const double ig = Fp - Ft;
            a.ig64[ci] = ig;
            atomicMax((unsigned long long *)&a.max64[x.v], (unsigned long long)f64_key(ig));
        }
    }
}

__global__ void k_select(const Cand *cand, const Status *st, int64_t cap, const double *ig64,
                         const uint64_t *max64, uint64_t *keyw)
{
    const int64_t nc = min((int64_t)st->n_cand, cap);
    for (int64_t ci = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; ci < nc;
         ci += (int64_t)gridDim.x * blockDim.x) {
        const double ig = ig64[ci];
        if (!(ig > -INFINITY)) continue;
        const Cand x = cand[ci];
        const double mx = key_f64(max64[x.v]);
        if (ig >= mx - tie_tau(mx))
            atomicMin((unsigned long long *)&keyw[x.v], ((unsigned long long)(uint32_t)x.r << 32) | x.partner);
    }
}

__global__ void k_output(int64_t p, int k, int disc_offset, const uint64_t *max64, const uint64_t *keyw,
                         const uint32_t *ovf, float *ig_max, int32_t *argmax, int32_t *argmax_disc)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= p) return;
    const bool bad = ovf[v] != 0 || keyw[v] == ~0ull;
    const uint64_t key = keyw[v];
    ig_max[v] = bad ? NAN : (float)key_f64(max64[v]);
    if (argmax_disc) argmax_disc[v] = bad ? -1 : disc_offset + (int32_t)(key >> 32);
    if (argmax) {
        const uint32_t pt = (uint32_t)key;
        if (k == 2) argmax[v] = bad ? -1 : (int32_t)pt;
        else if (k >= 4) {
            // the lexicographic rank of the partner tuple among the (k-1)-subsets of p variables
            int part[4] = {-1, -1, -1, -1};
            if (!bad) lex_unrank(pt, k - 1, p, part);
            for (int q = 0; q < k - 1; ++q) argmax[(int64_t)(k - 1) * v + q] = bad ? -1 : part[q];
        } else {
            argmax[2 * v] = bad ? -1 : (int32_t)(pt >> 16);
            argmax[2 * v + 1] = bad ? -1 : (int32_t)(pt & 0xffff);
        }
    }
}

template <int C, int K>
static void rescore_launch(const Problem &P, const RescoreArgs &a)
{
    hipLaunchKernelGGL((k_rescore<C, K>), dim3(1024), dim3(256), 0, P.stream, a);
}

static RescoreArgs rescore_args(const Problem &P)
{
    const Layout &L = P.L;
    RescoreArgs a{};
    a.cand = P.at<Cand>(L.cand);
    a.st = P.at<Status>(L.status);
    a.cap = L.cap;
    a.G32 = P.at<uint32_t>(L.G32);
    a.w_abs = (float)(2.0 * P.err_bound);
    a.onehot = P.at<int8_t>(L.onehot);
    a.rows_pad = L.rows_pad;
    a.KB = P.KB;
    a.K0pad = P.K0pad;
    a.Kpad = P.Kpad;
    a.kobj = P.kobj;
    a.fp4 = P.fp4;
    a.N0 = P.N0;
    a.N1 = P.N1;
    a.b0 = P.beta0;
    a.b1 = P.beta1;
    a.ig64 = P.at<double>(L.ig64);
    a.max64 = P.at<uint64_t>(L.max64);
    a.k = L.k;
    return a;
}

static hipError_t rescore_all(const Problem &P, const RescoreArgs &a)
{
    const Layout &L = P.L;
    if (L.k == 2) {
        switch (L.C) {
        case 2: rescore_launch<2, 2>(P, a); break;
        case 3: rescore_launch<3, 2>(P, a); break;
        case 5: rescore_launch<5, 2>(P, a); break;
        default: return hipErrorInvalidValue;
        }
    } else if (L.k >= 4) {
        return launch_rescore_hist(P);   // from the class-sorted codes, any class count
    } else {
        switch (L.C) {
        case 2: rescore_launch<2, 3>(P, a); break;
        case 3: rescore_launch<3, 3>(P, a); break;
        case 5: rescore_launch<5, 3>(P, a); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const Problem &P, float *ig_max, int32_t *argmax, int32_t *argmax_disc)
{
    const Layout &L = P.L;
    const RescoreArgs a = rescore_args(P);
    hipError_t e = rescore_all(P, a);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_select, dim3(256), dim3(256), 0, P.stream, a.cand, a.st, a.cap, a.ig64, a.max64,
                       P.at<uint64_t>(L.keyw));
    hipLaunchKernelGGL(k_output, dim3((unsigned)((L.p + 255) / 256)), dim3(256), 0, P.stream, L.p, L.k,
                       P.disc_offset, a.max64, P.at<uint64_t>(L.keyw), P.at<uint32_t>(L.ovf), ig_max, argmax,
                       argmax_disc);
    return hipGetLastError();
}

// ComputeInterestingTuples output: every re-scored candidate with IG >= thr, compacted (the
// order is that of the atomic counter, i.e. unspecified).
__global__ void k_emit(const Cand *cand, Status *st, int64_t cap, const double *ig64, double thr, int k,
                       int disc_offset, int32_t *var, int32_t *partners, int32_t *disc, double *ig, int64_t max_out)
{
    const int64_t nc = min((int64_t)st->n_cand, cap);
    for (int64_t ci = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; ci < nc;
         ci += (int64_t)gridDim.x * blockDim.x) {
        const double g = ig64[ci];
        if (!(g >= thr)) continue;
        const Cand x = cand[ci];
        const uint32_t at = atomicAdd(&st->n_emit, 1u);
        if ((int64_t)at >= max_out) continue;
        var[at] = x.v;
        if (k == 2) partners[at] = (int32_t)x.partner;
        else {
            partners[2 * (int64_t)at] = (int32_t)(x.partner >> 16);
            partners[2 * (int64_t)at + 1] = (int32_t)(x.partner & 0xffff);
        }
        disc[at] = disc_offset + x.r;
        ig[at] = g;
    }
}

hipError_t launch_emit(const Problem &P, double thr, int32_t *var, int32_t *partners, int32_t *disc, double *ig,
                       int64_t max_out)
{
    const RescoreArgs a = rescore_args(P);
    hipError_t e = rescore_all(P, a);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_emit, dim3(256), dim3(256), 0, P.stream, a.cand, P.at<Status>(P.L.status), a.cap, a.ig64,
                       thr, P.L.k, P.disc_offset, var, partners, disc, ig, max_out);
    return hipGetLastError();
}

// k = 1 (the one-dimensional analysis): IG(x_i) = F(y) - F(x_i) in binary64 for every
// discretisation; the maximum, and the smallest discretisation within tau of it.
__global__ void k_ig1(int64_t p, int R, int64_t p_pad, const double *F1d, double F0, int disc_offset,
                      float *ig_max, int32_t *argmax_disc)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= p) return;
    double M = -INFINITY;
    for (int r = 0; r < R; ++r) M = fmax(M, F0 - F1d[(int64_t)r * p_pad + v]);
    int best = 0;
    for (int r = 0; r < R; ++r)
        if (F0 - F1d[(int64_t)r * p_pad + v] >= M - tie_tau(M)) { best = r; break; }
    ig_max[v] = (float)M;
    if (argmax_disc) argmax_disc[v] = disc_offset + best;
}

hipError_t launch_ig1(const Problem &P, double F0, float *ig_max, int32_t *argmax_disc)
{
    hipLaunchKernelGGL(k_ig1, dim3((unsigned)((P.L.p + 255) / 256)), dim3(256), 0, P.stream, P.L.p, P.L.R, P.L.p_pad,
                       P.at<double>(P.L.F1d), F0, P.disc_offset, ig_max, argmax_disc);
    return hipGetLastError();
}

__global__ void k_screen_out(int64_t p, const uint32_t *G32, float *ig32)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v < p) ig32[v] = key_f32(G32[v]);
}

hipError_t launch_screen_out(const Problem &P, float *ig32)
{
    hipLaunchKernelGGL(k_screen_out, dim3((unsigned)((P.L.p + 255) / 256)), dim3(256), 0, P.stream, P.L.p,
                       P.at<uint32_t>(P.L.G32), ig32);
    return hipGetLastError();
}

}  // namespace mdfs
