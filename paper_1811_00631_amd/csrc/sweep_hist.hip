// sweep_hist.hip -- the k = 4 and k = 5 tuple sweep for any class count (per-tuple histograms).
//
// The counters N^d of section "Algorithm and implementation" for one K-tuple T (K = 4 or 5) and
// one discretisation are a histogram of the C^K voxels per class.  One wave takes one tuple at a
// time (tuples in colexicographic rank order, drawn from an atomic counter); its 64 lanes stride
// over the class-sorted objects, form each object's voxel index from the K variables' codes
// (one coalesced byte load per variable and 64 objects) and add 1 to the wave's LDS histogram of
// that class (class 0 occupies the first N0 positions).  Every cell is counted directly, so the
// class count only sets the histogram size (C^K = 32 .. 3125 cells), and each parent table
// T \ {t_m} is the histogram summed over axis m: the entropy of a parent needs no stored data
// of lower order.  This is the engine for the cases the bitset sweeps do not cover (k = 5 with
// three or five classes, k = 4 with five); the others can be asked for too.
//
// Epilogue: F = sum_v n_v h(p_v) in float32 from the lookup tables (the screen of the other
// sweeps, error bound E for C^K and C^(K-1) voxels), IG(t_m | T \ {t_m}) = F(T \ {t_m}) - F(T) for
// every member (equation IGmax), maxima and candidate appends under the same rules.  Candidates
// carry the lexicographic rank of their partner tuple; the binary64 re-score recounts each one's
// table from the class-sorted codes the same way.
#include "mdfs_internal.h"

namespace mdfs {

namespace {

__host__ __device__ constexpr int ipow(int c, int k) { return k == 0 ? 1 : c * ipow(c, k - 1); }
// words of one wave's histogram: both classes' C^K cells
__host__ __device__ constexpr int hist_words(int C, int K) { return 2 * ipow(C, K); }

struct HistArgs {
    const uint8_t *ccodes;   // [R][p][N] class-sorted codes
    const float *EA, *EB;
    const float2 *LQ;
    int N0, N1, N;
    int p;
    int r;
    int64_t n_tuples;        // C(p, K)
    uint32_t *G32;
    Cand *cand;
    int64_t cap;
    Status *st;
    uint32_t *ovf;
    float w_abs;
    int collect;
    const uint32_t *cancel;
    int tab_off, hist_off;   // LDS byte offsets of the tables and of the per-wave histograms
};

__device__ inline float winh(float w_abs, float g)
{
    const float ag = fabsf(g);
    return w_abs + 2e-9f * (ag > 1.f ? ag : 1.f) + 1e-30f;
}

__device__ inline float wave_sumf(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// K-tuple of colexicographic rank u: t[K-1] the largest x with C(x, K) <= u, and so on.
template <int K>
__device__ inline void tuple_of(uint64_t u, int (&t)[K])
{
#pragma unroll
    for (int m = K; m >= 1; --m) {
        // estimate from x^m / m! ~ u, then correct
        double f = 1.0;
        for (int i = 2; i <= m; ++i) f *= i;
        int64_t x = (int64_t)pow((double)u * f, 1.0 / m) + m;
        while (x >= m && binom_u64(x, m) > u) --x;
        while (binom_u64(x + 1, m) <= u) ++x;
        t[m - 1] = (int)x;
        u -= binom_u64(x, m);
    }
}

// one voxel's n h(p) from the LDS tables (int32 counts per class)
__device__ inline float vox(int n0, int n1, const float *EA, const float *EB, const float2 *LQ)
{
    const float2 lq = LQ[n0 + n1];
    return lq.x - lq.y * (EA[n0] + EB[n1]);
}

__device__ inline void puth(const HistArgs &a, uint32_t at, int v, uint32_t partner, float ig)
{
    if (at < a.cap) a.cand[at] = Cand{v, a.r, partner, ig};
    else { atomicOr(&a.ovf[v], 1u); atomicOr(&a.st->overflow, 1u); }
}

template <int C, int K, int NW>
__global__ __launch_bounds__(NW * 64) void k_sweep_hist(HistArgs a)
{
    constexpr int NCELL = ipow(C, K), NSUB = ipow(C, K - 1);
    if (a.collect && a.st->collect_go == 0) return;   // collect pass not needed (uniform)
    extern __shared__ __attribute__((aligned(16))) char smem[];
    float *EA = reinterpret_cast<float *>(smem + a.tab_off);
    float *EB = EA + (a.N0 + 1);
    float2 *LQ = reinterpret_cast<float2 *>(EB + (a.N1 + 1) + ((a.N0 + a.N1) & 1));
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int x = t; x <= a.N0; x += NW * 64) EA[x] = a.EA[x];
    for (int x = t; x <= a.N1; x += NW * 64) EB[x] = a.EB[x];
    for (int x = t; x <= a.N; x += NW * 64) LQ[x] = a.LQ[x];
    __syncthreads();
    uint32_t *h0 = reinterpret_cast<uint32_t *>(smem + a.hist_off) + wave * hist_words(C, K);
    uint32_t *h1 = h0 + NCELL;
    const uint8_t *cr = a.ccodes + (int64_t)a.r * a.p * a.N;

    uint32_t taken = 0;   // tuples taken by this wave (cancel polling)
    for (;;) {
        uint64_t u = 0;
        // a 64-bit counter over next_tile[0..1]: C(512, 5) and C(2048, 4) exceed 2^32
        if (lane == 0)
            u = cancel_poll(a.cancel, taken, a.st)
                    ? ~0ull
                    : (uint64_t)atomicAdd(reinterpret_cast<unsigned long long *>(&a.st->next_tile[0]), 1ull);
        ++taken;
        u = ((uint64_t)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
            (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
        if (u >= (uint64_t)a.n_tuples) break;
        int tv[K];
        tuple_of<K>(u, tv);
#pragma unroll
        for (int m = 0; m < K; ++m) tv[m] = __builtin_amdgcn_readfirstlane(tv[m]);

        // ---- histogram: zero, then one add per object (LDS operations of a wave complete in order)
        for (int c = lane; c < NCELL; c += 64) { h0[c] = 0u; h1[c] = 0u; }
        const uint8_t *row[K];
#pragma unroll
        for (int m = 0; m < K; ++m) row[m] = cr + (int64_t)tv[m] * a.N;
        for (int ps = lane; ps < a.N; ps += 64) {
            int cell = 0;
#pragma unroll
            for (int m = 0; m < K; ++m) cell = cell * C + row[m][ps];
            atomicAdd(ps < a.N0 ? &h0[cell] : &h1[cell], 1u);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): every add has landed
        __builtin_amdgcn_wave_barrier();

        // ---- F of the tuple and of its K parents (the histogram summed over one axis)
        float Ft = 0.f;
        for (int c = lane; c < NCELL; c += 64) Ft += vox((int)h0[c], (int)h1[c], EA, EB, LQ);
        Ft = wave_sumf(Ft);
        float ig[K];
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int stride = ipow(C, K - 1 - m);   // axis m's digit weight in the cell index
            float Fp = 0.f;
            for (int sidx = lane; sidx < NSUB; sidx += 64) {
                // sub-cell index without axis m: high part (axes < m) and low part (axes > m)
                const int hi = sidx / stride, lo = sidx % stride;
                const int base = hi * stride * C + lo;
                int s0 = 0, s1 = 0;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    s0 += (int)h0[base + c * stride];
                    s1 += (int)h1[base + c * stride];
                }
                Fp += vox(s0, s1, EA, EB, LQ);
            }
            ig[m] = wave_sumf(Fp) - Ft;
        }

        // ---- maxima and candidates (uniform values: lane 0 publishes)
        if (lane == 0) {
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const int v = tv[m];
                const float g = key_f32(a.G32[v]);
                const float top = a.collect ? g : fmaxf(g, ig[m]);
                if (ig[m] >= top - winh(a.w_abs, top)) {
                    int part[K - 1], q = 0;
#pragma unroll
                    for (int o = 0; o < K; ++o)
                        if (o != m) part[q++] = tv[o];
                    const uint32_t at = atomicAdd(&a.st->n_cand, 1u);
                    puth(a, at, v, lex_rank(part, K - 1, a.p), ig[m]);
                }
                if (!a.collect && ig[m] > g) atomicMax(&a.G32[v], f32_key(ig[m]));
            }
        }
    }
}

// ---- binary64 re-score of k >= 4 candidates: one wave per candidate recounts the table of
// (v, partners) into an LDS histogram (v the leading axis) and evaluates F of the table and of
// its parent (the table summed over v's axis) with binary64 logarithms.
__device__ inline double xlogx64h(double x) { return x > 0.0 ? x * log(x) : 0.0; }
__device__ inline double voxel64h(double n0, double n1, double b0, double b1)
{
    const double n = n0 + n1;
    if (n == 0.0) return 0.0;
    const double s = n + b0 + b1;
    return n * log(s) - (n / s) * (xlogx64h(n0 + b0) + xlogx64h(n1 + b1));
}

__device__ inline double wave_sumd(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

struct RescoreHArgs {
    const Cand *cand;
    const Status *st;
    int64_t cap;
    const uint32_t *G32;
    float w_abs;
    const uint8_t *ccodes;
    int N0, N, p;
    double b0, b1;
    double *ig64;
    uint64_t *max64;
};

template <int C, int K, int NW>
__global__ __launch_bounds__(NW * 64) void k_rescore_hist(RescoreHArgs a)
{
    constexpr int NCELL = ipow(C, K), PC = ipow(C, K - 1);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t *h0 = reinterpret_cast<uint32_t *>(smem) + wave * hist_words(C, K);
    uint32_t *h1 = h0 + NCELL;
    const int64_t wid = (int64_t)blockIdx.x * NW + wave, nw = (int64_t)gridDim.x * NW;
    const int64_t nc = min((int64_t)a.st->n_cand, a.cap);
    for (int64_t ci = wid; ci < nc; ci += nw) {
        const Cand x = a.cand[ci];
        const float g = key_f32(a.G32[x.v]);
        if (!(x.ig32 >= g - winh(a.w_abs, g))) {
            if (lane == 0) a.ig64[ci] = -INFINITY;
            continue;
        }
        int part[K - 1];
        lex_unrank(x.partner, K - 1, a.p, part);
        const uint8_t *cr = a.ccodes + (int64_t)x.r * a.p * a.N;
        const uint8_t *row[K];
        row[0] = cr + (int64_t)x.v * a.N;
#pragma unroll
        for (int m = 1; m < K; ++m) row[m] = cr + (int64_t)part[m - 1] * a.N;
        for (int c = lane; c < NCELL; c += 64) { h0[c] = 0u; h1[c] = 0u; }
        for (int ps = lane; ps < a.N; ps += 64) {
            int cell = 0;
#pragma unroll
            for (int m = 0; m < K; ++m) cell = cell * C + row[m][ps];
            atomicAdd(ps < a.N0 ? &h0[cell] : &h1[cell], 1u);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        double Ft = 0.0, Fp = 0.0;
        for (int c = lane; c < NCELL; c += 64) Ft += voxel64h(h0[c], h1[c], a.b0, a.b1);
        for (int pc = lane; pc < PC; pc += 64) {
            int s0 = 0, s1 = 0;
#pragma unroll
            for (int cv = 0; cv < C; ++cv) { s0 += (int)h0[cv * PC + pc]; s1 += (int)h1[cv * PC + pc]; }
            Fp += voxel64h(s0, s1, a.b0, a.b1);
        }
        Ft = wave_sumd(Ft);
        Fp = wave_sumd(Fp);
        __builtin_amdgcn_wave_barrier();   // the histogram is rewritten for the next candidate
        if (lane == 0) {
            const double igv = Fp - Ft;
            a.ig64[ci] = igv;
            atomicMax((unsigned long long *)&a.max64[x.v], (unsigned long long)f64_key(igv));
        }
    }
}

// waves per workgroup: 4, or 2 where one wave's histogram exceeds 16 KB (five classes and five
// variables: 25 KB)
template <int C, int K> constexpr int hist_waves() { return hist_words(C, K) * 4 > 16384 ? 2 : 4; }

size_t tables_bytes(const Problem &P)
{
    const size_t b = sizeof(float) * (size_t)(P.N0 + 1 + P.N1 + 1 + 1) + sizeof(float2) * (P.L.N + 1);
    return (b + 15) & ~size_t(15);
}

template <int C, int K>
hipError_t hist_launch(const Problem &P, int r, bool collect)
{
    constexpr int NW = hist_waves<C, K>();
    const Layout &L = P.L;
    HistArgs a{};
    a.ccodes = P.at<uint8_t>(L.ccodes);
    a.EA = P.at<float>(L.tabEA);
    a.EB = P.at<float>(L.tabEB);
    a.LQ = P.at<float2>(L.tabLQ);
    a.N0 = P.N0;
    a.N1 = P.N1;
    a.N = (int)L.N;
    a.p = (int)L.p;
    a.r = r;
    a.n_tuples = (int64_t)binom_u64(L.p, K);
    a.G32 = P.at<uint32_t>(L.G32);
    a.cand = P.at<Cand>(L.cand);
    a.cap = L.cap;
    a.st = P.at<Status>(L.status);
    a.ovf = P.at<uint32_t>(L.ovf);
    a.w_abs = (float)(2.0 * P.err_bound);
    a.collect = collect ? 1 : 0;
    a.cancel = P.cancel;
    a.hist_off = 0;
    a.tab_off = NW * hist_words(C, K) * 4;
    const size_t lds = (size_t)a.tab_off + tables_bytes(P);
    auto kern = k_sweep_hist<C, K, NW>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int grid = P.workgroups > 0 ? P.workgroups : 2048;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), lds, P.stream, a);
    return hipGetLastError();
}

template <int C, int K>
hipError_t rescore_hist_launch(const Problem &P)
{
    constexpr int NW = hist_waves<C, K>();
    const Layout &L = P.L;
    RescoreHArgs a{};
    a.cand = P.at<Cand>(L.cand);
    a.st = P.at<Status>(L.status);
    a.cap = L.cap;
    a.G32 = P.at<uint32_t>(L.G32);
    a.w_abs = (float)(2.0 * P.err_bound);
    a.ccodes = P.at<uint8_t>(L.ccodes);
    a.N0 = P.N0;
    a.N = (int)L.N;
    a.p = (int)L.p;
    a.b0 = P.beta0;
    a.b1 = P.beta1;
    a.ig64 = P.at<double>(L.ig64);
    a.max64 = P.at<uint64_t>(L.max64);
    const size_t lds = (size_t)NW * hist_words(C, K) * 4;
    auto kern = k_rescore_hist<C, K, NW>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(1024), dim3(NW * 64), lds, P.stream, a);
    return hipGetLastError();
}

}  // namespace

size_t sweep_hist_lds_bytes(const Problem &P)
{
    const int C = P.L.C, K = P.L.k;
    if (K < 4 || K > 5 || (C != 2 && C != 3 && C != 5)) return 0;
    const int words = 2 * (K == 4 ? C * C * C * C : C * C * C * C * C);
    const int nw = words * 4 > 16384 ? 2 : 4;
    return (size_t)nw * words * 4 + tables_bytes(P);
}

hipError_t launch_sweep_hist(const Problem &P, int r, bool collect)
{
    hipError_t e = launch_reset_queue(P);
    if (e != hipSuccess) return e;
    const int key = P.L.k * 10 + P.L.C;
    switch (key) {
    case 42: return hist_launch<2, 4>(P, r, collect);
    case 43: return hist_launch<3, 4>(P, r, collect);
    case 45: return hist_launch<5, 4>(P, r, collect);
    case 52: return hist_launch<2, 5>(P, r, collect);
    case 53: return hist_launch<3, 5>(P, r, collect);
    case 55: return hist_launch<5, 5>(P, r, collect);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rescore_hist(const Problem &P)
{
    const int key = P.L.k * 10 + P.L.C;
    switch (key) {
    case 42: return rescore_hist_launch<2, 4>(P);
    case 43: return rescore_hist_launch<3, 4>(P);
    case 45: return rescore_hist_launch<5, 4>(P);
    case 52: return rescore_hist_launch<2, 5>(P);
    case 53: return rescore_hist_launch<3, 5>(P);
    case 55: return rescore_hist_launch<5, 5>(P);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mdfs
