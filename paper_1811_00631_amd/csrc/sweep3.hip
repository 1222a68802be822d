// sweep3.hip -- the k = 3 tuple sweep with per-class bitsets (AND + popcount).
//
// For one discretisation, every triple i < j < l gets its per-class voxel table (the counters
// N^d of section "Algorithm and implementation").  Each variable is stored as W = C-1 bin
// bitsets per class over class-sorted objects ([class][word][variable][bin] u32).  One wave
// takes a pair (i, j); its lanes take 64 third variables l > j at a time.  The pair words
// B_i[a] & B_j[b] are wave-uniform: lane u holds word u of each run of 64 (one coalesced load
// per run) and the word loop takes them with V_READLANE; the lane's B_l[e] words are
// coalesced vector loads, and V_BCNT_U32_B32 accumulates popcount(B_i[a] & B_j[b] & B_l[e])
// for the W^3 bin triples a, b, e < W.  Both classes share one counter: class 1 first, shift by
// 16, then class 0, as in the pair sweep.  The remaining C^3 - W^3 voxels follow exactly from
// the three pair tables (emitted by the pair sweep for this discretisation) and the marginals.
//
// Epilogue: F3 = sum_v n_v h(p_v) in float32 from the lookup tables; the parents are the pair
// F values of the same float32 screen, IG(i|j,l) = F(j,l) - F3 and likewise for j and l
// (equation IGmax with k = 3).  Maxima and candidate appends follow the pair sweep's rules.
#include "mdfs_internal.h"

namespace mdfs {

struct Sweep3Args {
    const uint32_t *bits;    // [R][2][words_max][p_pad][W]
    const uint32_t *ptab;    // [nr][p_pad][p_pad][W*W] packed counts of pairs i < j
    const float *F2;         // [nr][p_pad][p_pad] float32 F of pairs i < j
    int64_t ptab_stride, f2_stride;   // elements per discretisation of ptab and F2
    const uint32_t *marg;    // [R][p_pad][C] packed per-class marginals
    const float *EA, *EB;
    const float2 *LQ;
    int N0, N1, N;
    int p;
    int64_t p_pad, words_max;
    int w0, w1;              // bitset words of class 0 / class 1
    int r0, nr;              // discretisations r0 .. r0 + nr - 1 in this launch
    int64_t n_pairs;         // C(p, 2)
    uint32_t *G32;
    Cand *cand;
    int64_t cap;
    Status *st;
    uint32_t *ovf;
    float w_abs;
    int collect;
    int32_t *counts_out;     // count export: [p][p][2][C][C][C], triples (i_sel, j, l) of disc_sel
    int i_sel, disc_sel;
    const uint32_t *cancel;  // caller's cancel word (nullable)
};

// threads per workgroup: 8 waves at two classes (59 VGPRs: 8 waves per SIMD at 4 workgroups per
// CU), else 4
__host__ __device__ constexpr int s3_threads(int W) { return W == 1 ? 512 : 256; }

// A value passed through an empty volatile asm: volatile asm statements keep their program
// order, so work that depends on the result cannot start before the asms ahead of it.
template <class T>
__device__ __forceinline__ T ordered3(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

__device__ inline float window3(float w_abs, float g)
{
    float ag = fabsf(g);
    return w_abs + 2e-9f * (ag > 1.f ? ag : 1.f) + 1e-30f;
}

__device__ inline float wave_max(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
    return x;
}

// Full C x C packed table of a pair from its W x W packed counts and the two marginals.
template <int W>
__device__ inline void full_pair(const uint32_t *pw, const uint32_t *Mx, const uint32_t *My, uint32_t (&n)[W + 1][W + 1])
{
    constexpr int C = W + 1;
#pragma unroll
    for (int x = 0; x < W; ++x)
#pragma unroll
        for (int y = 0; y < W; ++y) n[x][y] = pw[x * W + y];
#pragma unroll
    for (int x = 0; x < W; ++x) {
        uint32_t s = Mx[x];
#pragma unroll
        for (int y = 0; y < W; ++y) s -= n[x][y];
        n[x][W] = s;
    }
#pragma unroll
    for (int y = 0; y < C; ++y) {
        uint32_t s = My[y];
#pragma unroll
        for (int x = 0; x < W; ++x) s -= n[x][y];
        n[W][y] = s;
    }
}

// candidate record at a reserved slot, or the overflow marks when the buffer is full
__device__ inline void put3(const Sweep3Args &a, int r, uint32_t at, int v, uint32_t partner, float ig)
{
    if (at < a.cap) a.cand[at] = Cand{v, r, partner, ig};
    else { atomicOr(&a.ovf[v], 1u); atomicOr(&a.st->overflow, 1u); }
}

template <int W, bool EXPORT = false>
__global__ __launch_bounds__(s3_threads(W), W == 1 ? 8 : 1) void k_sweep3(Sweep3Args a)
{
    constexpr int C = W + 1;
    if (a.collect && a.st->collect_go == 0) return;   // collect pass not needed (uniform)
    extern __shared__ __attribute__((aligned(16))) char smem[];
    float *EA = reinterpret_cast<float *>(smem);
    float *EB = EA + (a.N0 + 1);
    float2 *LQ = reinterpret_cast<float2 *>(EB + (a.N1 + 1) + ((a.N0 + a.N1) & 1));
    const int t = threadIdx.x, lane = t & 63;
    for (int i = t; i <= a.N0; i += s3_threads(W)) EA[i] = a.EA[i];
    for (int i = t; i <= a.N1; i += s3_threads(W)) EB[i] = a.EB[i];
    for (int i = t; i <= a.N; i += s3_threads(W)) LQ[i] = a.LQ[i];
    __syncthreads();
    // byte offsets of EB and of the (L, Q) pairs from the start of the array (EA)
    const uint32_t offB = 4u * (uint32_t)(a.N0 + 1);
    const uint32_t offL = (uint32_t)(reinterpret_cast<char *>(LQ) - reinterpret_cast<char *>(EA));

    const int64_t plane = a.p_pad * W;                 // u32 per bitset word plane

    uint32_t taken = 0;   // pairs taken by this wave (cancel polling)
    for (;;) {
        // one pair per wave, taken in order of increasing j (largest amount of work first)
        uint32_t u = 0;
        if (lane == 0) u = cancel_poll(a.cancel, taken, a.st) ? 0xffffffffu : atomicAdd(&a.st->next_tile[0], 1u);
        ++taken;
        u = __builtin_amdgcn_readfirstlane(u);
        if ((int64_t)u >= a.n_pairs * a.nr) break;
        // pair u of discretisation r = r0 + rr of the launch
        const int rr = (int)(u / (uint32_t)a.n_pairs);
        u -= (uint32_t)rr * (uint32_t)a.n_pairs;
        const int r = a.r0 + rr;
        const uint32_t *margr = a.marg + (int64_t)r * a.p_pad * C;
        const uint32_t *bits1 = a.bits + ((int64_t)r * 2 + 1) * a.words_max * plane;
        const uint32_t *bits0 = a.bits + ((int64_t)r * 2 + 0) * a.words_max * plane;
        const uint32_t *ptab = a.ptab + (int64_t)rr * a.ptab_stride;
        const float *F2 = a.F2 + (int64_t)rr * a.f2_stride;
        int64_t jj = (int64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
        while ((jj + 1) * (jj + 2) / 2 <= (int64_t)u) ++jj;
        while (jj * (jj + 1) / 2 > (int64_t)u) --jj;
        const int i = __builtin_amdgcn_readfirstlane((int)((int64_t)u - jj * (jj + 1) / 2));
        const int j = __builtin_amdgcn_readfirstlane((int)jj + 1);
        if (j + 1 >= a.p) continue;   // no third variable

        uint32_t Mi[C], Mj[C];
#pragma unroll
        for (int c = 0; c < C; ++c) { Mi[c] = margr[(int64_t)i * C + c]; Mj[c] = margr[(int64_t)j * C + c]; }
        uint32_t Nij[C][C];
        full_pair<W>(ptab + ((int64_t)i * a.p_pad + j) * (W * W), Mi, Mj, Nij);
        const float F2ij = F2[(int64_t)i * a.p_pad + j];
        float Gi = key_f32(a.G32[i]), Gj = key_f32(a.G32[j]);
        float runi = -INFINITY, runj = -INFINITY;

        for (int l0 = j + 1; l0 < a.p; l0 += 64) {
            const int l = l0 + lane;
            const bool act = l < a.p;
            const int lc = act ? l : (a.p - 1);   // in-bounds stand-in for idle lanes
            // the lane's pair data and marginals, loaded before the count loop so that their
            // latency overlaps it
            uint32_t Ml[C], pil[W * W], pjl[W * W];
#pragma unroll
            for (int c = 0; c < C; ++c) Ml[c] = margr[(int64_t)lc * C + c];
#pragma unroll
            for (int k = 0; k < W * W; ++k) {
                pil[k] = ptab[((int64_t)i * a.p_pad + lc) * (W * W) + k];
                pjl[k] = ptab[((int64_t)j * a.p_pad + lc) * (W * W) + k];
            }
            const float Fjl = F2[(int64_t)j * a.p_pad + lc], Fil = F2[(int64_t)i * a.p_pad + lc];
            const float Gl = key_f32(a.G32[lc]);

            // ---- counts of the W^3 leading bin triples (class 1, shift, class 0)
            uint32_t cnt[W][W][W];
#pragma unroll
            for (int x = 0; x < W; ++x)
#pragma unroll
                for (int y = 0; y < W; ++y)
#pragma unroll
                    for (int z = 0; z < W; ++z) cnt[x][y][z] = 0;
#pragma unroll
            for (int cls = 1; cls >= 0; --cls) {
                const uint32_t *bw = cls ? bits1 : bits0;
                const int nw = cls ? a.w1 : a.w0;
                for (int wb = 0; wb < nw; wb += 64) {
                    // lane u holds word wb + u of the pair's words B_i[x] & B_j[y] (one coalesced
                    // load per 64 words); the word loop reads them with readlane
                    uint32_t pw[W][W];
                    {
                        const int wu = wb + lane;
                        const uint32_t *row = bw + (int64_t)(wu < nw ? wu : nw - 1) * plane;
                        uint32_t bi[W], bj[W];
#pragma unroll
                        for (int x = 0; x < W; ++x) {
                            bi[x] = row[(int64_t)i * W + x];
                            bj[x] = row[(int64_t)j * W + x];
                        }
#pragma unroll
                        for (int x = 0; x < W; ++x)
#pragma unroll
                            for (int y = 0; y < W; ++y) pw[x][y] = bi[x] & bj[y];
                    }
                    const int wn = nw - wb < 64 ? nw - wb : 64;
                    for (int u = 0; u < wn; ++u) {
                        const uint32_t *row = bw + (int64_t)(wb + u) * plane;
                        uint32_t bl[W];
#pragma unroll
                        for (int z = 0; z < W; ++z) bl[z] = row[(int64_t)lc * W + z];
#pragma unroll
                        for (int x = 0; x < W; ++x)
#pragma unroll
                            for (int y = 0; y < W; ++y) {
                                const uint32_t pij = __builtin_amdgcn_readlane(pw[x][y], u);
#pragma unroll
                                for (int z = 0; z < W; ++z)
                                    cnt[x][y][z] += __builtin_popcount(pij & bl[z]);   // v_bcnt_u32_b32
                            }
                    }
                }
                if (cls == 1) {
#pragma unroll
                    for (int x = 0; x < W; ++x)
#pragma unroll
                        for (int y = 0; y < W; ++y)
#pragma unroll
                            for (int z = 0; z < W; ++z) cnt[x][y][z] <<= 16;
                }
            }

            // count export (EXPORT: this kernel plus the store): the W^3 directly counted cells of
            // the triples (i_sel, j, l); launch_complete_triples fills in the others
            if (EXPORT && i == a.i_sel && r == a.disc_sel && act) {
                int32_t *o = a.counts_out + ((int64_t)j * a.p + l) * 2 * C * C * C;
#pragma unroll
                for (int x = 0; x < W; ++x)
#pragma unroll
                    for (int y = 0; y < W; ++y)
#pragma unroll
                        for (int z = 0; z < W; ++z) {
                            o[(x * C + y) * C + z] = (int32_t)(cnt[x][y][z] & 0xffffu);
                            o[C * C * C + (x * C + y) * C + z] = (int32_t)(cnt[x][y][z] >> 16);
                        }
            }

            // ---- F of the full C^3 table, one slab x at a time (x = bin of i): a slab x < W from
            // its leading counts and the (i, j), (i, l) tables; the last slab from the (j, l)
            // table minus the running sums S of the slabs before it.  Slab by slab, each slab's
            // counts passing through an ordered asm after the previous slab's sum, so that only
            // one slab's table reads are in flight and the full table is never held at once
            // (the voxels are summed in the same order as over the full table).
            uint32_t Nil[C][C], Njl[C][C];
            full_pair<W>(pil, Mi, Ml, Nil);
            full_pair<W>(pjl, Mj, Ml, Njl);
            uint32_t S[C][C];
#pragma unroll
            for (int y = 0; y < C; ++y)
#pragma unroll
                for (int z = 0; z < C; ++z) S[y][z] = 0u;
            float F3 = 0.f;
#pragma unroll
            for (int x = 0; x < C; ++x) {
                uint32_t sl[C][C];
                if (x < W) {
#pragma unroll
                    for (int y = 0; y < W; ++y) {
                        uint32_t s_ = Nij[x][y];
#pragma unroll
                        for (int z = 0; z < W; ++z) {
                            sl[y][z] = cnt[x][y][z];
                            s_ -= sl[y][z];
                        }
                        sl[y][W] = s_;
                    }
#pragma unroll
                    for (int z = 0; z < W; ++z) {
                        uint32_t s_ = Nil[x][z];
#pragma unroll
                        for (int y = 0; y < W; ++y) s_ -= sl[y][z];
                        sl[W][z] = s_;
                    }
                    uint32_t s_ = Nil[x][W];
#pragma unroll
                    for (int y = 0; y < W; ++y) s_ -= sl[y][W];
                    sl[W][W] = s_;
#pragma unroll
                    for (int y = 0; y < C; ++y)
#pragma unroll
                        for (int z = 0; z < C; ++z) S[y][z] += sl[y][z];
                } else {
#pragma unroll
                    for (int y = 0; y < C; ++y)
#pragma unroll
                        for (int z = 0; z < C; ++z) sl[y][z] = Njl[y][z] - S[y][z];
                }
#pragma unroll
                for (int y = 0; y < C; ++y)
#pragma unroll
                    for (int z = 0; z < C; ++z) F3 += vox_lds(ordered3(sl[y][z] << 2), offB, offL);
                F3 = ordered3(F3);
            }

            const float igi = act ? Fjl - F3 : -INFINITY;    // gain of x_i given (x_j, x_l)
            const float igj = act ? Fil - F3 : -INFINITY;    // gain of x_j given (x_i, x_l)
            const float igl = act ? F2ij - F3 : -INFINITY;   // gain of x_l given (x_i, x_j)

            // ---- member l: one value per lane
            const bool al = act && igl >= Gl - window3(a.w_abs, Gl);
            if (al && !a.collect && igl > Gl) atomicMax(&a.G32[l], f32_key(igl));
            // ---- members i and j: chunk maxima over the lanes
            const float mi = wave_max(igi), mj = wave_max(igj);
            const float topi = a.collect ? Gi : fmaxf(mi, Gi), topj = a.collect ? Gj : fmaxf(mj, Gj);
            const bool ai = act && igi >= topi - window3(a.w_abs, topi);
            const bool aj = act && igj >= topj - window3(a.w_abs, topj);
            // one slot reservation per chunk for the wave's records
            uint32_t at = reserve_slots(&a.st->n_cand, (uint32_t)al + (uint32_t)ai + (uint32_t)aj, lane);
            if (al) put3(a, r, at++, l, ((uint32_t)i << 16) | (uint32_t)j, igl);
            if (ai) put3(a, r, at++, i, ((uint32_t)j << 16) | (uint32_t)l, igi);
            if (aj) put3(a, r, at++, j, ((uint32_t)i << 16) | (uint32_t)l, igj);
            runi = fmaxf(runi, mi);
            runj = fmaxf(runj, mj);
            if (!a.collect) { Gi = fmaxf(Gi, mi); Gj = fmaxf(Gj, mj); }
        }
        if (!a.collect && lane == 0) {
            if (runi > -INFINITY) atomicMax(&a.G32[i], f32_key(runi));
            if (runj > -INFINITY) atomicMax(&a.G32[j], f32_key(runj));
        }
    }
}

template <int W>
static hipError_t sweep3_launch(const Problem &P, int r0, int nr, bool collect, int32_t *counts_out, int i_sel,
                                int disc_sel)
{
    const Layout &L = P.L;
    Sweep3Args a{};
    a.bits = P.at<uint32_t>(L.bits);
    a.ptab = P.at<uint32_t>(L.ptab);
    a.F2 = P.at<float>(L.F2);
    a.marg = P.at<uint32_t>(L.marg);
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
    a.r0 = r0;
    a.nr = nr;
    a.ptab_stride = L.p_pad * L.p_pad * W * W;
    a.f2_stride = L.p_pad * L.p_pad;
    a.n_pairs = L.p * (L.p - 1) / 2;
    a.G32 = P.at<uint32_t>(L.G32);
    a.cand = P.at<Cand>(L.cand);
    a.cap = L.cap;
    a.st = P.at<Status>(L.status);
    a.ovf = P.at<uint32_t>(L.ovf);
    a.w_abs = (float)(2.0 * P.err_bound);
    a.collect = collect ? 1 : 0;
    a.counts_out = counts_out;
    a.i_sel = i_sel;
    a.disc_sel = disc_sel;
    a.cancel = P.cancel;
    size_t lds = sizeof(float) * (size_t)(P.N0 + 1 + P.N1 + 1 + 1) + sizeof(float2) * (L.N + 1) + 16;
    auto kern = counts_out ? k_sweep3<W, true> : k_sweep3<W>;
    // the epilogue addresses EA by its offset in the dynamic LDS array: no static LDS before it
    static const hipError_t lds_ok = lds_array_at_zero({(const void *)k_sweep3<W, true>, (const void *)k_sweep3<W>});
    if (lds_ok != hipSuccess) return lds_ok;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // resident waves per SIMD: 8 at W = 1 (4 workgroups of 8 waves per CU), 5-6 at W = 2 (6 of
    // 4, registers permitting), 4 otherwise
    const int grid = P.workgroups > 0 ? 2 * P.workgroups : (W == 2 ? 1536 : 1024);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(s3_threads(W)), lds, P.stream, a);
    return hipGetLastError();
}

hipError_t launch_sweep3(const Problem &P, int r0, int nr, bool collect, int32_t *counts_out, int i_sel, int disc_sel)
{
    hipError_t e = launch_reset_queue(P);
    if (e != hipSuccess) return e;
    switch (P.L.W) {
    case 1: return sweep3_launch<1>(P, r0, nr, collect, counts_out, i_sel, disc_sel);
    case 2: return sweep3_launch<2>(P, r0, nr, collect, counts_out, i_sel, disc_sel);
    case 4: return sweep3_launch<4>(P, r0, nr, collect, counts_out, i_sel, disc_sel);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- count export, completion
// The triple sweep stored the W^3 directly counted cells of the triples (i_sel, j, l) of the
// selected discretisation into counts [p][p][2][C][C][C] (axes: bins of x_i, x_j, x_l).  Every
// other cell follows exactly from the three pair tables of the same discretisation (their W x W
// counts in the workspace, completed from the marginals) by subtracting the cells already known
// along one axis, the same relations the sweeps use.  One thread per (j, l), i_sel < j < l.
// The pair counts are n1 << 16 | n0 shifted left by pshift (2 when the matrix-core triple sweep
// is their reader).
template <int C>
__global__ __launch_bounds__(256) void k_complete_triples(int32_t *counts, const uint32_t *ptab, const uint32_t *marg,
                                                          int r, int i_sel, int64_t p, int64_t p_pad, int pshift)
{
    constexpr int W = C - 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * p) return;
    const int64_t j = t / p, l = t % p, i = i_sel;
    if (!(i < j && j < l)) return;
    const uint32_t *M = marg + (int64_t)r * p_pad * C;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        auto part = [d](uint32_t x) { return (int32_t)(d ? x >> 16 : x & 0xffffu); };
        // full C x C table of the pair (a, b), a < b
        auto pair = [&](int64_t a_, int64_t b_, int32_t (&n)[C][C]) {
            const uint32_t *pw = ptab + (a_ * p_pad + b_) * (W * W);
            for (int x = 0; x < W; ++x)
                for (int y = 0; y < W; ++y) n[x][y] = part(pw[x * W + y] >> pshift);
            for (int x = 0; x < W; ++x) {
                int32_t s = part(M[a_ * C + x]);
                for (int y = 0; y < W; ++y) s -= n[x][y];
                n[x][W] = s;
            }
            for (int y = 0; y < C; ++y) {
                int32_t s = part(M[b_ * C + y]);
                for (int x = 0; x < W; ++x) s -= n[x][y];
                n[W][y] = s;
            }
        };
        int32_t Nij[C][C], Nil[C][C], Njl[C][C];
        pair(i, j, Nij);
        pair(i, l, Nil);
        pair(j, l, Njl);
        int32_t *o = counts + (t * 2 + d) * C * C * C;
        auto T = [&](int x, int y, int z) -> int32_t & { return o[(x * C + y) * C + z]; };
        for (int x = 0; x < W; ++x)
            for (int y = 0; y < W; ++y) {
                int32_t s = Nij[x][y];
                for (int z = 0; z < W; ++z) s -= T(x, y, z);
                T(x, y, W) = s;
            }
        for (int x = 0; x < W; ++x)
            for (int z = 0; z < W; ++z) {
                int32_t s = Nil[x][z];
                for (int y = 0; y < W; ++y) s -= T(x, y, z);
                T(x, W, z) = s;
            }
        for (int y = 0; y < W; ++y)
            for (int z = 0; z < W; ++z) {
                int32_t s = Njl[y][z];
                for (int x = 0; x < W; ++x) s -= T(x, y, z);
                T(W, y, z) = s;
            }
        for (int x = 0; x < W; ++x) {
            int32_t s = Nil[x][W];
            for (int y = 0; y < W; ++y) s -= T(x, y, W);
            T(x, W, W) = s;
        }
        for (int y = 0; y < W; ++y) {
            int32_t s = Njl[y][W];
            for (int x = 0; x < W; ++x) s -= T(x, y, W);
            T(W, y, W) = s;
        }
        for (int z = 0; z < W; ++z) {
            int32_t s = Njl[W][z];
            for (int x = 0; x < W; ++x) s -= T(x, W, z);
            T(W, W, z) = s;
        }
        int32_t s = Njl[W][W];
        for (int x = 0; x < W; ++x) s -= T(x, W, W);
        T(W, W, W) = s;
    }
}

hipError_t launch_complete_triples(const Problem &P, int32_t *counts, int r, int r0, int i_sel)
{
    const int64_t n = P.L.p * P.L.p;
    const dim3 grid((unsigned)((n + 255) / 256));
    const uint32_t *ptab = P.at<uint32_t>(P.L.ptab) + (int64_t)(r - r0) * P.L.p_pad * P.L.p_pad * P.L.W * P.L.W;
    const uint32_t *marg = P.at<uint32_t>(P.L.marg);
    const int pshift = P.k3_mfma ? 2 : 0;   // the pair sweep's stored form for that engine
    switch (P.L.C) {
    case 2: hipLaunchKernelGGL(k_complete_triples<2>, grid, dim3(256), 0, P.stream, counts, ptab, marg, r, i_sel, P.L.p, P.L.p_pad,
                               pshift); break;
    case 3: hipLaunchKernelGGL(k_complete_triples<3>, grid, dim3(256), 0, P.stream, counts, ptab, marg, r, i_sel, P.L.p, P.L.p_pad,
                               pshift); break;
    case 5: hipLaunchKernelGGL(k_complete_triples<5>, grid, dim3(256), 0, P.stream, counts, ptab, marg, r, i_sel, P.L.p, P.L.p_pad,
                               pshift); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mdfs
