// sweep45.hip -- the k = 4 and k = 5 tuple sweeps for two classes (divisions = 1) on per-class
// bitsets.
//
// Every k-tuple is split into a prefix, its k - 2 smallest variables, and a pair m < n above the
// prefix.  One wave takes a prefix from the work counter and its lanes take the pairs above it,
// 64 at a time.  A prefix whose largest member is l has C(p - 1 - l, 2) pairs, so the lanes
// stay busy.
//
// Counting (the counters N^d of section "Algorithm and implementation", for the 4D and 5D
// analyses the paper times): b_v is the stored bitset of variable v's first bin.  For a set S of
// the tuple's members, g(S) = the number of a class's objects with every member of S in the
// first bin = popcount(AND of b_v over v in S), g(empty) = the class size.  The subsets of the
// prefix are the same for the whole wave and are counted once per prefix.  The other subsets
// hold m, n or both and take one AND and one V_BCNT_U32_B32 per 32-object word each, which is
// 3 * 2^(k-2) per word.  The 2^k cell counts then follow exactly by inclusion-exclusion, a
// Moebius transform over the subset lattice.  Both classes share one packed counter
// (class 1 << 16 | class 0); the transform is linear and every final cell fits in 16 bits, so
// the packed arithmetic is exact modulo 2^32.
//
// Epilogue: F_k = sum over the 2^k voxels of n_v h(p_v), and the F of the k parent
// (k-1)-tuples, each the table summed over one axis.  Both are float32 sums from the lookup
// tables.  IG of a member = F(parent without it) - F_k (equation IGmax).  Maxima and candidate
// appends follow the rules of the other sweeps.  A candidate's partner is the lexicographic
// rank of the other k - 1 members.
#include "mdfs_internal.h"

namespace mdfs {

namespace {

struct Sweep45Args {
    const uint32_t *bits;    // [R][2][words_max][p_pad] (W = 1: the first bin)
    const float *EA, *EB;
    const float2 *LQ;
    int N0, N1, N;
    int p;
    int64_t p_pad, words_max;
    int w0, w1;              // bitset words of class 0 / class 1
    int r;
    int64_t n_prefix;        // C(p, k - 2)
    uint32_t *G32;
    Cand *cand;
    int64_t cap;
    Status *st;
    uint32_t *ovf;
    float w_abs;
    int collect;
    const uint32_t *cancel;  // caller's cancel word (nullable)
    int tw_off;              // LDS byte offset of the waves' prefix words
};

constexpr int S45_THREADS = 256;

// A value passed through an empty volatile asm: volatile asm statements keep their program
// order, so work that depends on the result cannot start before the asms ahead of it.
template <class T>
__device__ __forceinline__ T ordered(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

__device__ inline float window45(float w_abs, float g)
{
    const float ag = fabsf(g);
    return w_abs + 2e-9f * (ag > 1.f ? ag : 1.f) + 1e-30f;
}

__device__ inline float wave_max45(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
    return x;
}

__device__ inline uint32_t wave_sum45(uint32_t x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += (uint32_t)__shfl_xor((int)x, o);
    return x;
}

// The t-subset of colexicographic rank u (u = sum over s of C(c[s-1], s), c ascending).
template <int T>
__device__ inline void colex_unrank(uint64_t u, int p, int *c)
{
#pragma unroll
    for (int s = T; s >= 1; --s) {
        // the largest x < p with C(x, s) <= u
        int lo = s - 1, hi = p - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (binom_u64(mid, s) <= u) lo = mid;
            else hi = mid - 1;
        }
        c[s - 1] = lo;
        u -= binom_u64(lo, s);
    }
}

// candidate record at a reserved slot, or the overflow marks when the buffer is full
__device__ inline void put45(const Sweep45Args &a, uint32_t at, int v, uint32_t partner, float ig)
{
    if (at < a.cap) a.cand[at] = Cand{v, a.r, partner, ig};
    else { atomicOr(&a.ovf[v], 1u); atomicOr(&a.st->overflow, 1u); }
}

template <int K>
__global__ __launch_bounds__(S45_THREADS) void k_sweep45(Sweep45Args a)
{
    constexpr int NP = K - 2;             // prefix members
    constexpr int NS = 1 << NP;           // subsets of the prefix
    constexpr int NC = 1 << K;            // cells
    if (a.collect && a.st->collect_go == 0) return;   // collect pass not needed (uniform)
    extern __shared__ __attribute__((aligned(16))) char smem[];
    float *EA = reinterpret_cast<float *>(smem);
    float *EB = EA + (a.N0 + 1);
    float2 *LQ = reinterpret_cast<float2 *>(EB + (a.N1 + 1) + ((a.N0 + a.N1) & 1));
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // this wave's prefix words: for every bitset word (class 1's, then class 0's) the AND over
    // each subset of the prefix, NS words (the empty subset's slot unused)
    uint4 *tws = reinterpret_cast<uint4 *>(smem + a.tw_off) + (size_t)wave * (a.w0 + a.w1) * (NS / 4);
    for (int x = t; x <= a.N0; x += S45_THREADS) EA[x] = a.EA[x];
    for (int x = t; x <= a.N1; x += S45_THREADS) EB[x] = a.EB[x];
    for (int x = t; x <= a.N; x += S45_THREADS) LQ[x] = a.LQ[x];
    __syncthreads();
    // byte offsets of EB and of the (L, Q) pairs from the start of the array (EA, LDS address 0)
    const uint32_t offB = 4u * (uint32_t)(a.N0 + 1);
    const uint32_t offL = (uint32_t)(reinterpret_cast<char *>(LQ) - reinterpret_cast<char *>(EA));

    const int64_t plane = a.p_pad;       // u32 per bitset word plane
    const uint32_t *bits1 = a.bits + ((int64_t)a.r * 2 + 1) * a.words_max * plane;
    const uint32_t *bits0 = a.bits + ((int64_t)a.r * 2 + 0) * a.words_max * plane;
    const uint32_t n_all = ((uint32_t)a.N1 << 16) | (uint32_t)a.N0;

    uint32_t taken = 0;   // prefixes taken by this wave (cancel polling)
    for (;;) {
        uint32_t u = 0;
        if (lane == 0) u = cancel_poll(a.cancel, taken, a.st) ? 0xffffffffu : atomicAdd(&a.st->next_tile[0], 1u);
        ++taken;
        u = __builtin_amdgcn_readfirstlane(u);
        if ((int64_t)u >= a.n_prefix) break;
        int pre[NP];
        colex_unrank<NP>(u, a.p, pre);
#pragma unroll
        for (int s = 0; s < NP; ++s) pre[s] = __builtin_amdgcn_readfirstlane(pre[s]);
        const int last = pre[NP - 1];
        const int64_t M = a.p - 1 - last;             // variables above the prefix
        const int64_t npairs = M * (M - 1) / 2;
        if (npairs == 0) continue;

        // ---- g(S) of the prefix subsets: lanes over words, then a wave sum
        uint32_t gpre[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) gpre[s] = 0;
#pragma unroll
        for (int cls = 1; cls >= 0; --cls) {
            const uint32_t *bw = cls ? bits1 : bits0;
            const int nw = cls ? a.w1 : a.w0;
            uint32_t part[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) part[s] = 0;
            for (int w = lane; w < nw; w += 64) {
                const uint32_t *row = bw + (int64_t)w * plane;
                uint32_t tw[NS];
                tw[0] = 0xffffffffu;
#pragma unroll
                for (int b = 0; b < NP; ++b) {
                    const uint32_t x = row[pre[b]];
#pragma unroll
                    for (int s = 0; s < (1 << b); ++s) tw[s | (1 << b)] = tw[s] & x;
                }
#pragma unroll
                for (int s = 1; s < NS; ++s) part[s] += __builtin_popcount(tw[s]);
                uint4 *dst = tws + (size_t)((cls ? 0 : a.w1) + w) * (NS / 4);
#pragma unroll
                for (int h = 0; h < NS / 4; ++h) dst[h] = make_uint4(tw[4 * h], tw[4 * h + 1], tw[4 * h + 2], tw[4 * h + 3]);
            }
#pragma unroll
            for (int s = 1; s < NS; ++s) gpre[s] += wave_sum45(part[s]) << (cls ? 16 : 0);
        }
        gpre[0] = n_all;
        // the words written by the wave's lanes are read by all of them below
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        float G[NP], run[NP];
#pragma unroll
        for (int s = 0; s < NP; ++s) {
            G[s] = key_f32(a.G32[pre[s]]);
            run[s] = -INFINITY;
        }

        for (int64_t q0 = 0; q0 < npairs; q0 += 64) {
            // the lane's pair (m, n), last < m < n, in colexicographic order above the prefix
            const int64_t q = q0 + lane;
            const bool act = q < npairs;
            const int64_t qc = act ? q : 0;
            int64_t nn = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)qc)) * 0.5);
            while (nn * (nn - 1) / 2 > qc) --nn;
            while ((nn + 1) * nn / 2 <= qc) ++nn;
            const int m = last + 1 + (int)(qc - nn * (nn - 1) / 2), n = last + 1 + (int)nn;

            uint32_t am_[NS], an_[NS], amn[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) am_[s] = an_[s] = amn[s] = 0;
#pragma unroll
            for (int cls = 1; cls >= 0; --cls) {
                const uint32_t *bw = cls ? bits1 : bits0;
                const int nw = cls ? a.w1 : a.w0;
                const uint4 *twc = tws + (size_t)(cls ? 0 : a.w1) * (NS / 4);
#pragma unroll 2
                for (int w = 0; w < nw; ++w) {
                    const uint32_t *row = bw + (int64_t)w * plane;
                    uint32_t tw[NS];
#pragma unroll
                    for (int h = 0; h < NS / 4; ++h) {   // the same LDS address in every lane
                        const uint4 v = twc[(size_t)w * (NS / 4) + h];
                        tw[4 * h] = v.x;
                        tw[4 * h + 1] = v.y;
                        tw[4 * h + 2] = v.z;
                        tw[4 * h + 3] = v.w;
                    }
                    const uint32_t bm = row[m], bn = row[n], bmn = bm & bn;
                    am_[0] += __builtin_popcount(bm);
                    an_[0] += __builtin_popcount(bn);
                    amn[0] += __builtin_popcount(bmn);
#pragma unroll
                    for (int s = 1; s < NS; ++s) {
                        am_[s] += __builtin_popcount(tw[s] & bm);
                        an_[s] += __builtin_popcount(tw[s] & bn);
                        amn[s] += __builtin_popcount(tw[s] & bmn);
                    }
                }
                if (cls == 1) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        am_[s] <<= 16;
                        an_[s] <<= 16;
                        amn[s] <<= 16;
                    }
                }
            }

            // g over all 2^K subsets (bits 0 .. K-3 the prefix, K-2 m, K-1 n), then the cells
            uint32_t g[NC];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                g[s] = gpre[s];
                g[s | (1 << NP)] = am_[s];
                g[s | (2 << NP)] = an_[s];
                g[s | (3 << NP)] = amn[s];
            }
            // Moebius transform: g[S] becomes the count of objects whose first-bin members are
            // exactly S (the others in the second bin)
#pragma unroll
            for (int b = 0; b < K; ++b)
#pragma unroll
                for (int s = 0; s < NC; ++s)
                    if (!(s & (1 << b))) g[s] -= g[s | (1 << b)];

            // Table reads go in groups of 8 cells: each group's counts pass through an ordered
            // empty asm after the previous group's sum, so that one group's reads, not all 112,
            // are in flight at once (registers).
            float FK = 0.f;
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                FK += vox_lds(ordered(g[s] << 2), offB, offL);
                if ((s & 7) == 7) FK = ordered(FK);
            }
            float ig[K];
#pragma unroll
            for (int b = 0; b < K; ++b) {
                float Fp = 0.f;   // parent without member b: the table summed over axis b
#pragma unroll
                for (int h = 0; h < NC / 2; ++h) {
                    const int lo = h & ((1 << b) - 1), s = ((h >> b) << (b + 1)) | lo;   // bit b clear
                    Fp += vox_lds(ordered((g[s] + g[s | (1 << b)]) << 2), offB, offL);
                    if ((h & 7) == 7) Fp = ordered(Fp);
                }
                ig[b] = act ? Fp - FK : -INFINITY;
            }

            // ---- members m and n: one value per lane
            const float Gm = key_f32(a.G32[m]), Gn = key_f32(a.G32[n]);
            const bool fm = act && ig[NP] >= Gm - window45(a.w_abs, Gm);
            const bool fn = act && ig[NP + 1] >= Gn - window45(a.w_abs, Gn);
            if (fm && !a.collect && ig[NP] > Gm) atomicMax(&a.G32[m], f32_key(ig[NP]));
            if (fn && !a.collect && ig[NP + 1] > Gn) atomicMax(&a.G32[n], f32_key(ig[NP + 1]));
            // ---- prefix members: chunk maxima over the lanes
            bool fp[NP];
            uint32_t mine = (uint32_t)fm + (uint32_t)fn;
#pragma unroll
            for (int s = 0; s < NP; ++s) {
                const float mx = wave_max45(ig[s]);
                const float top = a.collect ? G[s] : fmaxf(mx, G[s]);
                fp[s] = act && ig[s] >= top - window45(a.w_abs, top);
                mine += (uint32_t)fp[s];
                run[s] = fmaxf(run[s], mx);
                if (!a.collect) G[s] = fmaxf(G[s], mx);
            }
            uint32_t at = reserve_slots(&a.st->n_cand, mine, lane);
            int c[K - 1];
            if (fm) {   // partner: the prefix and n
#pragma unroll
                for (int s = 0; s < NP; ++s) c[s] = pre[s];
                c[NP] = n;
                put45(a, at++, m, lex_rank(c, K - 1, a.p), ig[NP]);
            }
            if (fn) {   // partner: the prefix and m
#pragma unroll
                for (int s = 0; s < NP; ++s) c[s] = pre[s];
                c[NP] = m;
                put45(a, at++, n, lex_rank(c, K - 1, a.p), ig[NP + 1]);
            }
#pragma unroll
            for (int s = 0; s < NP; ++s) {
                if (!fp[s]) continue;
                int e = 0;   // partner: the prefix without member s, then m and n
#pragma unroll
                for (int o = 0; o < NP; ++o)
                    if (o != s) c[e++] = pre[o];
                c[NP - 1] = m;
                c[NP] = n;
                put45(a, at++, pre[s], lex_rank(c, K - 1, a.p), ig[s]);
            }
        }
        if (!a.collect && lane == 0) {
#pragma unroll
            for (int s = 0; s < NP; ++s)
                if (run[s] > -INFINITY) atomicMax(&a.G32[pre[s]], f32_key(run[s]));
        }
    }
}

size_t sweep45_tables_bytes(const Problem &P)
{
    const size_t b = sizeof(float) * (size_t)(P.N0 + 1 + P.N1 + 1 + 1) + sizeof(float2) * (P.L.N + 1);
    return (b + 15) / 16 * 16;
}

template <int K>
hipError_t sweep45_launch(const Problem &P, int r, bool collect)
{
    const Layout &L = P.L;
    Sweep45Args a{};
    a.bits = P.at<uint32_t>(L.bits);
    a.EA = P.at<float>(L.tabEA);
    a.EB = P.at<float>(L.tabEB);
    a.LQ = P.at<float2>(L.tabLQ);
    a.N0 = P.N0;
    a.N1 = P.N1;
    a.N = (int)L.N;
    a.p = (int)L.p;
    a.p_pad = L.p_pad;
    a.words_max = L.words_max;
    a.w0 = (P.N0 + 31) / 32;
    a.w1 = (P.N1 + 31) / 32;
    a.r = r;
    a.n_prefix = (int64_t)binom_u64(L.p, K - 2);
    a.G32 = P.at<uint32_t>(L.G32);
    a.cand = P.at<Cand>(L.cand);
    a.cap = L.cap;
    a.st = P.at<Status>(L.status);
    a.ovf = P.at<uint32_t>(L.ovf);
    a.w_abs = (float)(2.0 * P.err_bound);
    a.collect = collect ? 1 : 0;
    a.cancel = P.cancel;
    const size_t lds = sweep45_lds_bytes(P);
    a.tw_off = (int)sweep45_tables_bytes(P);
    auto kern = k_sweep45<K>;
    // the epilogue addresses EA by its offset in the dynamic LDS array: no static LDS before it
    static const hipError_t lds_ok = lds_array_at_zero({(const void *)kern});
    if (lds_ok != hipSuccess) return lds_ok;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(P.workgroups > 0 ? 2 * P.workgroups : 1024), dim3(S45_THREADS), lds, P.stream, a);
    return hipGetLastError();
}

}  // namespace

size_t sweep45_lds_bytes(const Problem &P)
{
    const size_t ns = P.L.k == 5 ? 8 : 4;
    const size_t words = (size_t)(P.N0 + 31) / 32 + (size_t)(P.N1 + 31) / 32;
    return sweep45_tables_bytes(P) + (S45_THREADS / 64) * words * ns * sizeof(uint32_t);
}

hipError_t launch_sweep45(const Problem &P, int r, bool collect)
{
    if (P.L.W != 1) return hipErrorInvalidValue;
    hipError_t e = launch_reset_queue(P);
    if (e != hipSuccess) return e;
    switch (P.L.k) {
    case 4: return sweep45_launch<4>(P, r, collect);
    case 5: return sweep45_launch<5>(P, r, collect);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mdfs
