// sweep4.hip -- the k = 4 tuple sweep with per-class bitsets (AND + popcount), C <= 3 classes.
//
// For one discretisation every quadruple i < j < l < m gets its full per-class voxel table
// (the counters N^d of section "Algorithm and implementation", for the 4D analysis the paper
// times).  One wave takes a triple (i, j, l), its lanes take 64 fourth variables m > l at a time.
// All C^4 cells are counted directly: per 32-object word the C^3 triple words
// B_i[a] & B_j[b] & B_l[c] are wave-uniform, the lane's B_m[e] words are coalesced loads, and
// V_BCNT_U32_B32 accumulates popcount(B_i[a] & B_j[b] & B_l[c] & B_m[e]).  The last bin's
// bitset, not stored, is the complement of the others within the class's valid objects.  Both
// classes share one counter (class 1 first, shifted by 16, then class 0).
//
// Epilogue: F4 = sum_v n_v h(p_v) over the C^4 voxels and the F of the four sub-triples, each
// the table summed over one axis, in float32 from the lookup tables; IG(i | j, l, m) =
// F(j, l, m) - F4 and likewise for j, l and m (equation IGmax with k = 4).  Maxima and candidate
// appends follow the rules of the other sweeps; partners are packed 10 bits each (p <= 1024).
#include "mdfs_internal.h"

namespace mdfs {

namespace {

struct Sweep4Args {
    const uint32_t *bits;    // [R][2][words_max][p_pad][W]
    const float *EA, *EB;
    const float2 *LQ;
    int N0, N1, N;
    int p;
    int64_t p_pad, words_max;
    int w0, w1;              // bitset words of class 0 / class 1
    int r;
    int64_t n_triples;       // C(p, 3)
    uint32_t *G32;
    Cand *cand;
    int64_t cap;
    Status *st;
    uint32_t *ovf;
    float w_abs;
    int collect;
    const uint32_t *cancel;  // caller's cancel word (nullable)
};

constexpr int S4_THREADS = 256;

// A value passed through an empty volatile asm: volatile asm statements keep their program
// order, so work that depends on the result cannot start before the asms ahead of it.
template <class T>
__device__ __forceinline__ T ordered4(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

__device__ inline float window4(float w_abs, float g)
{
    const float ag = fabsf(g);
    return w_abs + 2e-9f * (ag > 1.f ? ag : 1.f) + 1e-30f;
}

__device__ inline float wave_max4(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
    return x;
}

// partner triple a < b < c as its lexicographic rank among the 3-subsets of the p variables
__device__ inline uint32_t pack3(int a, int b, int c, int p)
{
    const int t[3] = {a, b, c};
    return lex_rank(t, 3, p);
}

// candidate record at a reserved slot, or the overflow marks when the buffer is full
__device__ inline void put4(const Sweep4Args &a, uint32_t at, int v, uint32_t partner, float ig)
{
    if (at < a.cap) a.cand[at] = Cand{v, a.r, partner, ig};
    else { atomicOr(&a.ovf[v], 1u); atomicOr(&a.st->overflow, 1u); }
}

// Triple of rank u in the order of its largest member: u = C(l,3) + C(j,2) + i, i < j < l.
__device__ inline void triple_of(int64_t u, int &i, int &j, int &l)
{
    auto c3 = [](int64_t x) { return x * (x - 1) * (x - 2) / 6; };
    auto c2 = [](int64_t x) { return x * (x - 1) / 2; };
    int64_t L = (int64_t)cbrt(6.0 * (double)u) + 2;
    while (L > 2 && c3(L) > u) --L;
    while (c3(L + 1) <= u) ++L;
    u -= c3(L);
    int64_t J = (int64_t)((sqrt(8.0 * (double)u + 1.0) + 1.0) * 0.5);
    while (J > 1 && c2(J) > u) --J;
    while (c2(J + 1) <= u) ++J;
    i = (int)(u - c2(J));
    j = (int)J;
    l = (int)L;
}

template <int W>
__global__ __launch_bounds__(S4_THREADS) void k_sweep4(Sweep4Args a)
{
    constexpr int C = W + 1;
    if (a.collect && a.st->collect_go == 0) return;   // collect pass not needed (uniform)
    extern __shared__ __attribute__((aligned(16))) char smem[];
    float *EA = reinterpret_cast<float *>(smem);
    float *EB = EA + (a.N0 + 1);
    float2 *LQ = reinterpret_cast<float2 *>(EB + (a.N1 + 1) + ((a.N0 + a.N1) & 1));
    const int t = threadIdx.x, lane = t & 63;
    for (int x = t; x <= a.N0; x += S4_THREADS) EA[x] = a.EA[x];
    for (int x = t; x <= a.N1; x += S4_THREADS) EB[x] = a.EB[x];
    for (int x = t; x <= a.N; x += S4_THREADS) LQ[x] = a.LQ[x];
    __syncthreads();
    // byte offsets of EB and of the (L, Q) pairs from the start of the array (EA, LDS address 0)
    const uint32_t offB = 4u * (uint32_t)(a.N0 + 1);
    const uint32_t offL = (uint32_t)(reinterpret_cast<char *>(LQ) - reinterpret_cast<char *>(EA));

    const int64_t plane = a.p_pad * W;   // u32 per bitset word plane
    const uint32_t *bits1 = a.bits + ((int64_t)a.r * 2 + 1) * a.words_max * plane;
    const uint32_t *bits0 = a.bits + ((int64_t)a.r * 2 + 0) * a.words_max * plane;

    uint32_t taken = 0;   // triples taken by this wave (cancel polling)
    for (;;) {
        uint32_t u = 0;
        if (lane == 0) u = cancel_poll(a.cancel, taken, a.st) ? 0xffffffffu : atomicAdd(&a.st->next_tile[0], 1u);
        ++taken;
        u = __builtin_amdgcn_readfirstlane(u);
        if ((int64_t)u >= a.n_triples) break;
        int i, j, l;
        triple_of((int64_t)u, i, j, l);
        i = __builtin_amdgcn_readfirstlane(i);
        j = __builtin_amdgcn_readfirstlane(j);
        l = __builtin_amdgcn_readfirstlane(l);
        if (l + 1 >= a.p) continue;   // no fourth variable

        float Gi = key_f32(a.G32[i]), Gj = key_f32(a.G32[j]), Gl = key_f32(a.G32[l]);
        float runi = -INFINITY, runj = -INFINITY, runl = -INFINITY;

        for (int m0 = l + 1; m0 < a.p; m0 += 64) {
            const int m = m0 + lane;
            const bool act = m < a.p;
            const int mc = act ? m : (a.p - 1);   // in-bounds stand-in for idle lanes

            uint32_t cnt[C][C][C][C];
#pragma unroll
            for (int x = 0; x < C; ++x)
#pragma unroll
                for (int y = 0; y < C; ++y)
#pragma unroll
                    for (int z = 0; z < C; ++z)
#pragma unroll
                        for (int e = 0; e < C; ++e) cnt[x][y][z][e] = 0;
#pragma unroll
            for (int cls = 1; cls >= 0; --cls) {
                const uint32_t *bw = cls ? bits1 : bits0;
                const int nw = cls ? a.w1 : a.w0, ny = cls ? a.N1 : a.N0;
                for (int w = 0; w < nw; ++w) {
                    const uint32_t *row = bw + (int64_t)w * plane;
                    const int rem = ny - 32 * w;
                    const uint32_t valid = rem >= 32 ? 0xffffffffu : ((1u << rem) - 1u);
                    uint32_t bi[C], bj[C], bl[C], bm[C];
                    uint32_t oi = 0, oj = 0, ol = 0, om = 0;
#pragma unroll
                    for (int x = 0; x < W; ++x) {
                        bi[x] = __builtin_amdgcn_readfirstlane(row[(int64_t)i * W + x]);
                        bj[x] = __builtin_amdgcn_readfirstlane(row[(int64_t)j * W + x]);
                        bl[x] = __builtin_amdgcn_readfirstlane(row[(int64_t)l * W + x]);
                        bm[x] = row[(int64_t)mc * W + x];
                        oi |= bi[x];
                        oj |= bj[x];
                        ol |= bl[x];
                        om |= bm[x];
                    }
                    bi[W] = ~oi & valid;
                    bj[W] = ~oj & valid;
                    bl[W] = ~ol & valid;
                    bm[W] = ~om & valid;
#pragma unroll
                    for (int x = 0; x < C; ++x)
#pragma unroll
                        for (int y = 0; y < C; ++y) {
                            const uint32_t pij = bi[x] & bj[y];
#pragma unroll
                            for (int z = 0; z < C; ++z) {
                                const uint32_t tijl = pij & bl[z];
#pragma unroll
                                for (int e = 0; e < C; ++e)
                                    cnt[x][y][z][e] += __builtin_popcount(tijl & bm[e]);   // v_bcnt_u32_b32
                            }
                        }
                }
                if (cls == 1) {
#pragma unroll
                    for (int x = 0; x < C; ++x)
#pragma unroll
                        for (int y = 0; y < C; ++y)
#pragma unroll
                            for (int z = 0; z < C; ++z)
#pragma unroll
                                for (int e = 0; e < C; ++e) cnt[x][y][z][e] <<= 16;
                }
            }

            // F of the quadruple and of its four sub-triples (the table summed over one axis).
            // Table reads go in groups (at three classes the quadruple's 81 voxels, then the
            // sub-triples' voxels 36 at a time): each group's counts pass through an ordered asm
            // after the previous group's sum has, so a group's reads wait for the one before and
            // the registers they hold stay fewer (210 VGPRs, two waves per SIMD, where all reads
            // at once took 367 and one).
            float F4 = 0.f, Fjlm = 0.f, Film = 0.f, Fijm = 0.f, Fijl = 0.f;
#pragma unroll
            for (int x = 0; x < C; ++x)
#pragma unroll
                for (int y = 0; y < C; ++y)
#pragma unroll
                    for (int z = 0; z < C; ++z)
#pragma unroll
                        for (int e = 0; e < C; ++e) {
                            F4 += vox_lds(ordered4(cnt[x][y][z][e] << 2), offB, offL);
                            if ((((x * C + y) * C + z) * C + e) % 81 == 80) F4 = ordered4(F4);
                        }
#pragma unroll
            for (int s1 = 0; s1 < C; ++s1)
#pragma unroll
                for (int s2 = 0; s2 < C; ++s2)
#pragma unroll
                    for (int s3 = 0; s3 < C; ++s3) {
                        uint32_t sa = 0, sb = 0, sc = 0, se = 0;
#pragma unroll
                        for (int o = 0; o < C; ++o) {
                            sa += cnt[o][s1][s2][s3];   // over i: (j, l, m)
                            sb += cnt[s1][o][s2][s3];   // over j: (i, l, m)
                            sc += cnt[s1][s2][o][s3];   // over l: (i, j, m)
                            se += cnt[s1][s2][s3][o];   // over m: (i, j, l)
                        }
                        Fjlm += vox_lds(ordered4(sa << 2), offB, offL);
                        Film += vox_lds(ordered4(sb << 2), offB, offL);
                        Fijm += vox_lds(ordered4(sc << 2), offB, offL);
                        Fijl += vox_lds(ordered4(se << 2), offB, offL);
                        if (((s1 * C + s2) * C + s3) % 9 == 8) {
                            Fjlm = ordered4(Fjlm);
                            Film = ordered4(Film);
                            Fijm = ordered4(Fijm);
                            Fijl = ordered4(Fijl);
                        }
                    }
            const float igi = act ? Fjlm - F4 : -INFINITY;
            const float igj = act ? Film - F4 : -INFINITY;
            const float igl = act ? Fijm - F4 : -INFINITY;
            const float igm = act ? Fijl - F4 : -INFINITY;

            // ---- member m: one value per lane
            const float Gm = key_f32(a.G32[mc]);
            const bool am = act && igm >= Gm - window4(a.w_abs, Gm);
            if (am && !a.collect && igm > Gm) atomicMax(&a.G32[m], f32_key(igm));
            // ---- members i, j, l: chunk maxima over the lanes
            const float mi = wave_max4(igi), mj = wave_max4(igj), ml = wave_max4(igl);
            const float topi = a.collect ? Gi : fmaxf(mi, Gi), topj = a.collect ? Gj : fmaxf(mj, Gj),
                        topl = a.collect ? Gl : fmaxf(ml, Gl);
            const bool ai = act && igi >= topi - window4(a.w_abs, topi);
            const bool aj = act && igj >= topj - window4(a.w_abs, topj);
            const bool al = act && igl >= topl - window4(a.w_abs, topl);
            // one slot reservation per chunk for the wave's records
            uint32_t at = reserve_slots(&a.st->n_cand, (uint32_t)am + (uint32_t)ai + (uint32_t)aj + (uint32_t)al, lane);
            if (am) put4(a, at++, m, pack3(i, j, l, a.p), igm);
            if (ai) put4(a, at++, i, pack3(j, l, m, a.p), igi);
            if (aj) put4(a, at++, j, pack3(i, l, m, a.p), igj);
            if (al) put4(a, at++, l, pack3(i, j, m, a.p), igl);
            runi = fmaxf(runi, mi);
            runj = fmaxf(runj, mj);
            runl = fmaxf(runl, ml);
            if (!a.collect) {
                Gi = fmaxf(Gi, mi);
                Gj = fmaxf(Gj, mj);
                Gl = fmaxf(Gl, ml);
            }
        }
        if (!a.collect && lane == 0) {
            if (runi > -INFINITY) atomicMax(&a.G32[i], f32_key(runi));
            if (runj > -INFINITY) atomicMax(&a.G32[j], f32_key(runj));
            if (runl > -INFINITY) atomicMax(&a.G32[l], f32_key(runl));
        }
    }
}

template <int W>
hipError_t sweep4_launch(const Problem &P, int r, bool collect)
{
    const Layout &L = P.L;
    Sweep4Args a{};
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
    a.n_triples = L.p * (L.p - 1) * (L.p - 2) / 6;
    a.G32 = P.at<uint32_t>(L.G32);
    a.cand = P.at<Cand>(L.cand);
    a.cap = L.cap;
    a.st = P.at<Status>(L.status);
    a.ovf = P.at<uint32_t>(L.ovf);
    a.w_abs = (float)(2.0 * P.err_bound);
    a.collect = collect ? 1 : 0;
    a.cancel = P.cancel;
    const size_t lds = sizeof(float) * (size_t)(P.N0 + 1 + P.N1 + 1 + 1) + sizeof(float2) * (L.N + 1) + 16;
    auto kern = k_sweep4<W>;
    // the epilogue addresses EA by its offset in the dynamic LDS array: no static LDS before it
    static const hipError_t lds_ok = lds_array_at_zero({(const void *)kern});
    if (lds_ok != hipSuccess) return lds_ok;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(P.workgroups > 0 ? 2 * P.workgroups : 1024), dim3(S4_THREADS), lds, P.stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep4(const Problem &P, int r, bool collect)
{
    hipError_t e = launch_reset_queue(P);
    if (e != hipSuccess) return e;
    switch (P.L.W) {
    case 1: return sweep4_launch<1>(P, r, collect);
    case 2: return sweep4_launch<2>(P, r, collect);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mdfs
