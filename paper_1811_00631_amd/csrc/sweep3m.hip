// sweep3m.hip -- the k = 3 tuple sweep on the matrix cores (one-hot pair x one-hot variable).
//
// For one discretisation, the per-class table of every triple i < j < l (the counters N^d of
// section "Algorithm and implementation") is, on its first W = C-1 bins of every variable, the
// contraction over objects of the pair one-hot column (x_i = a and x_j = b) with the one-hot
// column (x_l = e).  In the E2M1 (fp4) one-hot encoding of the pair sweep (2.0 or 0 per
// object) the pair column is the bitwise AND of the two variables' columns, so the same
// V_MFMA_F32_16X16X128_F8F6F4 contraction gives n1 * 2^14 + 4 n0 per (a, b, e) exactly.
//
// Tile: one i; A rows (j, a, b) for 32 consecutive j (128 rows), B rows (l, e) for 64
// consecutive l (128 rows).  The j rows and the two rows of i are staged in LDS (fetched
// straight into LDS one K block ahead into a 2-stage ring) and ANDed when the A fragments
// are read.  The remaining C^3 - W^3 voxels follow exactly from the three pair tables (from
// the pair sweep of the same discretisation) and the marginals.  Epilogue: F3 = sum_v n_v h(p_v)
// in float32 from the LDS tables; IG(i|j,l) = F(j,l) - F3 and likewise for j and l (equation
// IGmax with k = 3), maxima and candidate appends as in the bitset engine.  `k_sweep3m` is the
// three-class kernel (W = 2), `k_sweep3m1` the two-class one (W = 1, below); five classes use
// the bitset engine.
#include "mdfs_internal.h"

#include <vector>

namespace mdfs {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int M3_THREADS = 256;
constexpr int M3_JV = 32;                        // j variables per A tile (4 rows each)
constexpr int M3_LV = 64;                        // l variables per B tile (2 rows each)
constexpr int M3_JROWS = 2 * M3_JV;              // one-hot rows of the j block
constexpr int M3_STAGE = (M3_JROWS + TILE_ROWS) * KBLK + 2 * KBLK + 128;   // j rows | l rows | i rows | pad
constexpr int M3_NSTAGE = 2;   // operand stages, fetched one K block ahead (3 stages: 2.4% slower)

struct Sweep3mArgs {
    const int8_t *onehot;
    const uint32_t *ptab;    // [nr][p_pad][p_pad][W*W] packed ((4 n1) << 16 | 4 n0: byte offsets
                             // of the tables, as the pair sweep stores them for this engine)
                             // W x W counts of pairs
    const float *F2;         // [nr][p_pad][p_pad] float32 F of pairs
    int64_t ptab_stride, f2_stride;   // elements per discretisation of ptab and F2
    const uint32_t *marg;    // [R][p_pad][3]
    const float *EA, *EB;
    const float2 *LQ;
    const int64_t *apref;    // [n_ablk + 1] first tile of each A block (i, jb)
    const int32_t *ablk;     // [n_ablk] i * 256 + jb
    int64_t n_ablk, n_tiles;
    int N0, N1, N;
    int p;
    int64_t p_pad, rows_pad;
    int KB, KB0, r0, nr, nLB;   // discretisations r0 .. r0 + nr - 1 in this launch
    uint32_t *G32;
    Cand *cand;
    int64_t cap;
    Status *st;
    uint32_t *ovf;
    float w_abs;
    int collect;
    int snext_off;
    int stage_off;           // two-class kernel: LDS byte offset of the operand stages
    int32_t *counts_out;     // count export: [p][p][2][C][C][C], triples (i_sel, j, l) of disc_sel
    int i_sel, disc_sel;
    const uint32_t *cancel;  // caller's cancel word (nullable)
};

__device__ inline int lds_sw(int row, int j) { return row * KBLK + ((j ^ ((row >> 1) & 3)) << 4); }

__device__ inline float win3(float w_abs, float g)
{
    const float ag = fabsf(g);
    return w_abs + 2e-9f * (ag > 1.f ? ag : 1.f) + 1e-30f;
}

__device__ inline uint32_t swap1(uint32_t x) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false); }
__device__ inline float swap1f(float x) { return __builtin_bit_cast(float, swap1(__builtin_bit_cast(uint32_t, x))); }

// Loads at 32-bit byte offsets from a wave-uniform base: a buffer resource over `bytes` bytes
// (word 3: the 32-bit data format that raw loads take); a read past the end returns 0.  The
// pair tables of one discretisation stay below 2^31 bytes (p_pad <= 8192).
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ inline uint32_t ld32(__amdgpu_buffer_rsrc_t rs, uint32_t off) { return __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0); }
__device__ inline float ldf(__amdgpu_buffer_rsrc_t rs, uint32_t off) { return __builtin_bit_cast(float, ld32(rs, off)); }
__device__ inline v4i ld128(__amdgpu_buffer_rsrc_t rs, uint32_t off)
{
    return __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
}

// A value that every lane holds, made visibly uniform (scalar registers and loads downstream).
__device__ inline int64_t uniform64(int64_t x)
{
    const uint64_t u = (uint64_t)x;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Sum of n h(p) over NV packed counts (4 n1) << 16 | 4 n0 with the fixed LDS table layout of
// capacity T (EA at 0, EB at 4T, (L, Q) pairs at 8T); a packed 0 contributes exactly 0.
template <int T, int NV>
__device__ inline float vox_sum(const uint32_t (&P)[NV])
{
    typedef float vf2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) const float lds_f32;
    typedef __attribute__((address_space(3))) const vf2 lds_f32x2;
    float ea[NV], eb[NV];
    vf2 lq[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const uint32_t a0 = P[v] & 0xffffu, a1 = P[v] >> 16;
        // The triple sweeps declare no static LDS (group segment size 0; the launch checks it),
        // so the tables at the start of the dynamic array sit at LDS address 0 and these byte
        // offsets are their addresses: no base add per read.
        ea[v] = *reinterpret_cast<const lds_f32 *>((uintptr_t)a0);
        eb[v] = *reinterpret_cast<const lds_f32 *>((uintptr_t)(4 * T + a1));
        lq[v] = *reinterpret_cast<const lds_f32x2 *>((uintptr_t)(8 * T + 2 * (a0 + a1)));
    }
    // summed in voxel order, starting from the first term
    float F = lq[0].x - lq[0].y * (ea[0] + eb[0]);
#pragma unroll
    for (int v = 1; v < NV; ++v) F += lq[v].x - lq[v].y * (ea[v] + eb[v]);
    return F;
}

// Full 3 x 3 packed table of a pair from its 2 x 2 direct counts and the two marginals.
__device__ inline void full3(const uint32_t (&d)[4], const uint32_t (&Mx)[3], const uint32_t (&My)[3], uint32_t (&n)[3][3])
{
    n[0][0] = d[0]; n[0][1] = d[1]; n[1][0] = d[2]; n[1][1] = d[3];
    n[0][2] = Mx[0] - d[0] - d[1];
    n[1][2] = Mx[1] - d[2] - d[3];
    n[2][0] = My[0] - d[0] - d[2];
    n[2][1] = My[1] - d[1] - d[3];
    n[2][2] = My[2] - n[0][2] - n[1][2];
}

// candidate record at a reserved slot, or the overflow marks when the buffer is full
__device__ inline void put(const Sweep3mArgs &a, int r, uint32_t at, int v, uint32_t partner, float ig)
{
    if (at < a.cap) a.cand[at] = Cand{v, r, partner, ig};
    else { atomicOr(&a.ovf[v], 1u); atomicOr(&a.st->overflow, 1u); }
}

template <int T, bool EXPORT = false>
__global__ __launch_bounds__(M3_THREADS, 2) void k_sweep3m(Sweep3mArgs a)
{
    constexpr int C = 3;
    if (a.collect && a.st->collect_go == 0) return;   // collect pass not needed (uniform)
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char *stage = smem + 24 * T;
    int64_t *s_next = reinterpret_cast<int64_t *>(smem + a.snext_off);

    const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    const int q = lane >> 4, c16 = lane & 15, e = c16 & 1;

    {
        float *tf = reinterpret_cast<float *>(smem);
        for (int i = t; i <= a.N0; i += M3_THREADS) tf[i] = a.EA[i];
        for (int i = t; i <= a.N1; i += M3_THREADS) tf[T + i] = a.EB[i];
        float2 *lq = reinterpret_cast<float2 *>(smem + 8 * T);
        for (int i = t; i <= a.N; i += M3_THREADS) lq[i] = a.LQ[i];
    }
    auto repack = [](uint32_t x) -> uint32_t { return x << 2; };   // n1 << 16 | n0 -> fp4 packing
    const int64_t nrb = a.rows_pad / TILE_ROWS;
    constexpr int kstride = TILE_ROWS * KBLK;
    const int n1blk = a.KB - a.KB0;

    uint32_t taken = 0;   // tiles taken by this workgroup (cancel polling)
    for (;;) {
        __syncthreads();
        if (t == 0) *s_next = cancel_poll(a.cancel, taken++, a.st) ? a.n_tiles * a.nr : atomicAdd(&a.st->next_tile[0], 1u);
        __syncthreads();
        const int64_t u_all = uniform64(*s_next);
        if (u_all >= a.n_tiles * a.nr) break;
        // tile u of the list, under discretisation r = r0 + rr of the launch
        const int rr = (int)(u_all / a.n_tiles);
        const int64_t u = u_all - (int64_t)rr * a.n_tiles;
        const int r = a.r0 + rr;
        const uint32_t *margr = a.marg + (int64_t)r * a.p_pad * C;
        const uint32_t *ptab = a.ptab + (int64_t)rr * a.ptab_stride;
        const float *F2 = a.F2 + (int64_t)rr * a.f2_stride;
        // A block: last k with apref[k] <= u
        int64_t lo = 0, hi = a.n_ablk - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (a.apref[mid] <= u) lo = mid; else hi = mid - 1;
        }
        const int ab = a.ablk[lo];
        const int i = ab >> 8, jb = ab & 255;
        const int lb = jb / 2 + (int)(u - a.apref[lo]);

        // The tile's per-l data (and, below, i's): loaded before the K loop, so their latency
        // overlaps it (the maxima read here are lower bounds of the final ones, as any are).
        int jv[4], lv[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) jv[m] = jb * M3_JV + 16 * wr + 4 * m + q;
#pragma unroll
        for (int n = 0; n < 4; ++n) lv[n] = lb * M3_LV + 32 * wc + 8 * n + (c16 >> 1);
        // indices past p are clamped for the loads; such triples are invalid and masked
        auto clampv = [&](int v) { return v < a.p ? v : a.p - 1; };
        // pair data of (u, v): 2 x 2 counts at byte offset 16 (u p_pad + v), F at 4 (u p_pad + v);
        // u < v for every valid triple (an invalid one may read the unwritten lower triangle,
        // and its counts are masked); bases re-read as uniform (a resource sits in scalar registers)
        const uint32_t pp = (uint32_t)a.p_pad;
        const __amdgpu_buffer_rsrc_t rsP = rsrc(reinterpret_cast<const void *>(uniform64((int64_t)ptab)), 16u * pp * pp);
        const __amdgpu_buffer_rsrc_t rsF = rsrc(reinterpret_cast<const void *>(uniform64((int64_t)F2)), 4u * pp * pp);
        auto pair4 = [&](uint32_t uv, uint32_t (&d)[4]) {
            const v4i pw = ld128(rsP, 16u * uv);
#pragma unroll
            for (int x = 0; x < 4; ++x) d[x] = (uint32_t)pw[x];
        };
        uint32_t Mi[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) Mi[c] = repack(margr[(int64_t)i * C + c]);
        // per-l data for the whole tile; per-j data (one m block at a time) loaded in the loops
        uint32_t Ml[4][3], Pil[4][4], lc[4];
        float Fil[4], gL[4], gJ[4];
        struct JData {
            uint32_t M[3], P[4], jrow;
            float F;
        };
        auto load_j = [&](int m, JData &d) {
            const int j = clampv(jv[m]);
#pragma unroll
            for (int c = 0; c < 3; ++c) d.M[c] = repack(margr[(int64_t)j * C + c]);
            d.jrow = (uint32_t)j * pp;
            pair4((uint32_t)i * pp + (uint32_t)j, d.P);
            d.F = ldf(rsF, 4u * ((uint32_t)i * pp + (uint32_t)j));
        };
#pragma unroll
        for (int m = 0; m < 4; ++m) gJ[m] = key_f32(a.G32[clampv(jv[m])]);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const int l = clampv(lv[n]);
            lc[n] = (uint32_t)l;
#pragma unroll
            for (int c = 0; c < 3; ++c) Ml[n][c] = repack(margr[(int64_t)l * C + c]);
            pair4((uint32_t)i * pp + lc[n], Pil[n]);
            Fil[n] = ldf(rsF, 4u * ((uint32_t)i * pp + lc[n]));
            const float g = key_f32(a.G32[l]);
            gL[n] = g;
        }
        const float Gi = key_f32(a.G32[i]);
        // ---------------------------------------------------------------- K loop
        // ---------------------------------------------------------------- K loop
        // operand sources in the panel-major one-hot encoding
        const int8_t *panJ = a.onehot + ((int64_t)r * nrb + jb / 2) * a.KB * kstride + (jb & 1) * M3_JROWS * KBLK;
        const int8_t *panL = a.onehot + ((int64_t)r * nrb + lb) * a.KB * kstride;
        const int8_t *panI = a.onehot + ((int64_t)r * nrb + (2 * i) / TILE_ROWS) * a.KB * kstride +
                             ((2 * i) % TILE_ROWS) * KBLK;
        auto kblock = [&](int s_) { return s_ < n1blk ? a.KB0 + s_ : s_ - n1blk; };
        auto stage_at = [&](int s_) { return stage + (s_ % M3_NSTAGE) * M3_STAGE; };
        // 13 fetches of 1 KB per K block: 4 for the 64 j rows, 8 for the 128 l rows (stage
        // rows 64..191), 1 for the two rows of i (lanes 0..7).  Wave w takes fetches w, w+4,
        // w+8, w+12 (wave 0 four, the others three).
        auto issue = [&](int s_) {
            const int64_t kb_off = (int64_t)kblock(s_) * kstride;
            char *st_ = stage_at(s_);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int f = wave + 4 * k;
                if (f > 12) break;
                if (f < 12) {
                    // j rows (f < 4) or l rows: 16 stage rows, swizzle applied on the global side
                    const int srow = 16 * f + (lane >> 2);
                    const int j = (lane & 3) ^ ((srow >> 1) & 3);
                    const int8_t *src = f < 4 ? panJ + kb_off + srow * KBLK + j * 16
                                              : panL + kb_off + (srow - M3_JROWS) * KBLK + j * 16;
                    __builtin_amdgcn_global_load_lds((const void *)src,
                                                     (__attribute__((address_space(3))) void *)(st_ + f * 1024), 16, 0, 0);
                } else if (lane < 8) {
                    // the two rows of i, unswizzled (rows 0 and 1 have swizzle 0)
                    const int8_t *src = panI + kb_off + (lane >> 2) * KBLK + (lane & 3) * 16;
                    __builtin_amdgcn_global_load_lds((const void *)src,
                                                     (__attribute__((address_space(3))) void *)(st_ + 12 * 1024), 16, 0, 0);
                }
            }
        };
        v4f acc[4][4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = v4f{0.f, 0.f, 0.f, 0.f};
        // A fragment of block m: lane reads A-tile row rho = 64 wr + 16 m + c16, i.e. j-local
        // 16 wr + 4 m + c16 / 4 with bins a = (c16 >> 1) & 1 (of i) and b = c16 & 1 (of j)
        const int ia = (c16 >> 1) & 1;
        int offJ[4], offL[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) offJ[m] = lds_sw(2 * (16 * wr + 4 * m + (c16 >> 2)) + (c16 & 1), q);
#pragma unroll
        for (int n = 0; n < 4; ++n) offL[n] = M3_JROWS * KBLK + lds_sw(wc * 64 + 16 * n + c16, q);
        const int offI = (M3_JROWS + TILE_ROWS) * KBLK + lds_sw(ia, q);

        // Two stages: step s waits for its own fetches of block s (the only ones outstanding),
        // passes a barrier (block s is complete, and every wave has finished reading block s-1,
        // whose stage the fetch of block s+1 then takes) and fetches block s+1 before reading
        // the fragments of block s.
        issue(0);
        for (int s = 0; s < a.KB; ++s) {
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
            __builtin_amdgcn_s_barrier();
            if (s + 1 < a.KB) issue(s + 1);
            const char *st_ = stage_at(s);
            const v4i fi = *reinterpret_cast<const v4i *>(st_ + offI);
            v4i fa[4], fb[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) fa[m] = *reinterpret_cast<const v4i *>(st_ + offJ[m]) & fi;
#pragma unroll
            for (int n = 0; n < 4; ++n) fb[n] = *reinterpret_cast<const v4i *>(st_ + offL[n]);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const v8i a8{fa[m][0], fa[m][1], fa[m][2], fa[m][3], 0, 0, 0, 0};
                    const v8i b8{fb[n][0], fb[n][1], fb[n][2], fb[n][3], 0, 0, 0, 0};
                    acc[m][n] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, acc[m][n], 4, 4, 0, 0, 0, 0);
                }
            if (s == n1blk - 1) {
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < 4; ++n) acc[m][n] = acc[m][n] * 4096.0f;
            }
        }

        // ---------------------------------------------------------------- epilogue
        // lane (q, c16) of block (m, n): D[a][b] = T[a][b][e] of the triple (i, j_m, l_n),
        // (a, b) = register index, packed (4 n1) << 16 | 4 n0
        v4i cnt[4][4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n)
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const uint32_t uu = (uint32_t)acc[m][n][x];
                    cnt[m][n][x] = (int)(__umul24(uu >> 14, 245760u) + uu);
                }
        // count export (EXPORT: this kernel plus the store): T[a][b][e] of the triples (i_sel, j, l)
        if (EXPORT && i == a.i_sel && r == a.disc_sel) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const int j = jb * M3_JV + 16 * wr + 4 * m + q, l = lb * M3_LV + 32 * wc + 8 * n + (c16 >> 1);
                    if (!(i < j && j < l && l < a.p)) continue;
                    int32_t *o = a.counts_out + ((int64_t)j * a.p + l) * 2 * 27;
#pragma unroll
                    for (int x = 0; x < 4; ++x) {
                        const uint32_t v = (uint32_t)cnt[m][n][x] >> 2;
                        o[((x >> 1) * 3 + (x & 1)) * 3 + e] = (int32_t)(v & 0xffffu);
                        o[27 + ((x >> 1) * 3 + (x & 1)) * 3 + e] = (int32_t)(v >> 16);
                    }
                }
        }

        // F3 of triple (i, j_m, l_n) on the lane pair (e = 0, 1) from the 2 x 2 direct counts dj
        // of (j_m, l_n)
        auto triple = [&](int m, int n, const JData &jd, const uint32_t (&dj)[4]) -> float {
            const bool valid = (i < jv[m]) & (jv[m] < lv[n]) & (lv[n] < a.p);
            uint32_t Nij[3][3], Nil[3][3], Njl[3][3];
            full3(jd.P, Mi, jd.M, Nij);
            full3(Pil[n], Mi, Ml[n], Nil);
            full3(dj, jd.M, Ml[n], Njl);
            const v4i &ac = cnt[m][n];
            uint32_t D[2][2], Dp[2][2];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                D[x >> 1][x & 1] = (uint32_t)ac[x];
                Dp[x >> 1][x & 1] = swap1((uint32_t)ac[x]);     // partner lane: T[a][b][1-e]
            }
            const uint32_t Nil_ae0 = e ? Nil[0][1] : Nil[0][0], Nil_ae1 = e ? Nil[1][1] : Nil[1][0];
            const uint32_t Njl_be0 = e ? Njl[0][1] : Njl[0][0], Njl_be1 = e ? Njl[1][1] : Njl[1][0];
            const uint32_t Njl_2e = e ? Njl[2][1] : Njl[2][0];
            uint32_t V[14];
            // slab z = e
            V[0] = D[0][0]; V[1] = D[0][1]; V[2] = D[1][0]; V[3] = D[1][1];
            V[4] = Nil_ae0 - D[0][0] - D[0][1];          // T[0][2][e]
            V[5] = Nil_ae1 - D[1][0] - D[1][1];          // T[1][2][e]
            V[6] = Njl_be0 - D[0][0] - D[1][0];          // T[2][0][e]
            V[7] = Njl_be1 - D[0][1] - D[1][1];          // T[2][1][e]
            V[8] = Njl_2e - V[4] - V[5];                 // T[2][2][e]
            // slab z = 2: T[a][b][2] from the (i, j) table
            uint32_t Z[2][2];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) Z[x][y] = Nij[x][y] - D[x][y] - Dp[x][y];
            const uint32_t Z02 = Nil[0][2] - Z[0][0] - Z[0][1];   // T[0][2][2]
            const uint32_t Z12 = Nil[1][2] - Z[1][0] - Z[1][1];   // T[1][2][2]
            const uint32_t Z20 = Njl[0][2] - Z[0][0] - Z[1][0];   // T[2][0][2]
            const uint32_t Z21 = Njl[1][2] - Z[0][1] - Z[1][1];   // T[2][1][2]
            const uint32_t Z22 = Njl[2][2] - Z02 - Z12;           // T[2][2][2]
            V[9] = e ? Z02 : Z[0][0];
            V[10] = e ? Z12 : Z[0][1];
            V[11] = e ? Z20 : Z[1][0];
            V[12] = e ? Z21 : Z[1][1];
            V[13] = e ? 0u : Z22;
            // an invalid triple may combine unrelated tables: its counts are not counts
#pragma unroll
            for (int k = 0; k < 14; ++k) V[k] = valid ? V[k] : 0u;
            // two batches of 7 (the table reads of a batch are issued together; 14 at once
            // would not leave room for the tile's counts)
            uint32_t V0[7], V1[7];
#pragma unroll
            for (int k = 0; k < 7; ++k) { V0[k] = V[k]; V1[k] = V[7 + k]; }
            const float f = vox_sum<T, 7>(V0) + vox_sum<T, 7>(V1);
            return f + swap1f(f);
        };

        // One pass, row by row (block row m: the j_m of the lane's q): the row's (j, l) pair data
        // are loaded first, all loads in flight together; the row's triples are evaluated and
        // their F kept, the maxima of the row's members reduced over the wave, and the row's
        // appends decided against thresholds that are the larger of the maximum read before the
        // tile and the wave's maximum so far (both below the final maximum, so every triple
        // within the window of the final maximum is appended); a row whose wave maxima all stay
        // below their thresholds appends nothing and skips the selection; one slot reservation
        // per row; the j_m maximum goes out with its row.
        float mi = -INFINITY, ml[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) ml[n] = -INFINITY;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            JData jd;
            load_j(m, jd);
            uint32_t Pjl[4][4];
            float F3r[4], Fjlr[4], mjm = -INFINITY;
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                pair4(jd.jrow + lc[n], Pjl[n]);
                Fjlr[n] = ldf(rsF, 4u * (jd.jrow + lc[n]));
            }
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                F3r[n] = 0.f;
                const bool valid = (i < jv[m]) & (jv[m] < lv[n]) & (lv[n] < a.p);
                // wave-uniform skip of a block without any valid triple (near the diagonal of
                // the (j, l) blocks and past p): its maxima would stay -inf
                if (!__any(valid)) continue;
                F3r[n] = triple(m, n, jd, Pjl[n]);
                mi = fmaxf(mi, valid ? Fjlr[n] - F3r[n] : -INFINITY);     // gain of x_i given (x_j, x_l)
                mjm = fmaxf(mjm, valid ? Fil[n] - F3r[n] : -INFINITY);    // gain of x_j given (x_i, x_l)
                ml[n] = fmaxf(ml[n], valid ? jd.F - F3r[n] : -INFINITY);  // gain of x_l given (x_i, x_j)
            }
            // wave maxima so far: i over all lanes; j_m over the lanes of one q; l_n over the
            // lanes of one c16 / 2 (the two lanes of a pair hold the same values)
            float wi = mi, wj = mjm, wl[4];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) wi = fmaxf(wi, __shfl_xor(wi, o));
            wj = fmaxf(wj, __shfl_xor(wj, 2));
            wj = fmaxf(wj, __shfl_xor(wj, 4));
            wj = fmaxf(wj, __shfl_xor(wj, 8));
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                float x = ml[n];
                x = fmaxf(x, __shfl_xor(x, 16));
                wl[n] = fmaxf(x, __shfl_xor(x, 32));
            }
            const float tI = a.collect ? Gi : fmaxf(Gi, wi), thI = tI - win3(a.w_abs, tI);
            const float tJ = a.collect ? gJ[m] : fmaxf(gJ[m], wj), thJ = tJ - win3(a.w_abs, tJ);
            float thL[4];
            bool hot = wi >= thI || wj >= thJ;
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const float tL = a.collect ? gL[n] : fmaxf(gL[n], wl[n]);
                thL[n] = tL - win3(a.w_abs, tL);
                hot |= wl[n] >= thL[n];
            }
            if (__any(hot)) {
                uint32_t sel = 0;   // bit 3 n + member
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const bool valid = (e == 0) & (i < jv[m]) & (jv[m] < lv[n]) & (lv[n] < a.p);   // one lane per triple
                    if (valid && Fjlr[n] - F3r[n] >= thI) sel |= 1u << (3 * n);
                    if (valid && Fil[n] - F3r[n] >= thJ) sel |= 2u << (3 * n);
                    if (valid && jd.F - F3r[n] >= thL[n]) sel |= 4u << (3 * n);
                }
                uint32_t at = reserve_slots(&a.st->n_cand, __popc(sel), lane);
                if (sel) {
                    const int j = jv[m];
#pragma unroll
                    for (int n = 0; n < 4; ++n) {
                        const int l = lv[n];
                        if (sel & (1u << (3 * n))) put(a, r, at++, i, ((uint32_t)j << 16) | (uint32_t)l, Fjlr[n] - F3r[n]);
                        if (sel & (2u << (3 * n))) put(a, r, at++, j, ((uint32_t)i << 16) | (uint32_t)l, Fil[n] - F3r[n]);
                        if (sel & (4u << (3 * n))) put(a, r, at++, l, ((uint32_t)i << 16) | (uint32_t)j, jd.F - F3r[n]);
                    }
                }
            }
            if (!a.collect && c16 == 0 && jv[m] < a.p && wj > gJ[m]) atomicMax(&a.G32[jv[m]], f32_key(wj));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mi = fmaxf(mi, __shfl_xor(mi, o));
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            float x = ml[n];
            x = fmaxf(x, __shfl_xor(x, 16));
            ml[n] = fmaxf(x, __shfl_xor(x, 32));
        }
        if (a.collect) continue;
        // only where the tile raised the maximum read before (maxima only grow)
        if (lane == 0 && mi > Gi) atomicMax(&a.G32[i], f32_key(mi));
#pragma unroll
        for (int n = 0; n < 4; ++n)
            if (q == 0 && e == 0 && ml[n] > gL[n]) atomicMax(&a.G32[lv[n]], f32_key(ml[n]));
    }
}

// ---------------------------------------------------------------------------------------------
// Two classes (W = 1): one one-hot row per variable.  Tile: one i; A rows = the 128 j of block jb
// (each ANDed with the row of i when its fragment is read), B rows = the 128 l of block lb.  The
// lane (q, c16) of 16 x 16 block (m, n) holds T[0][0][0] of the four triples (i, j, l) with
// j = 128 jb + 64 wr + 16 m + 4 q + x (register x) and l = 128 lb + 64 wc + 16 n + c16.  The other
// seven cells follow from the three pair counts N(0,0) and the bin-0 marginals, each by a
// subtraction whose two class halves stay >= 0 (no borrow between the packed halves):
//   T001 = Nij - T000          T010 = Nil - T000          T100 = Njl - T000
//   T011 = (Mi - Nij) - T010   T101 = (Mj - Nij) - T100   T110 = (Ml - Nil) - T100
//   T111 = ((N - Mi) - (Mj - Nij)) - T110
// (a, b, e = bins of i, j, l; Mx = bin-0 count of x; N = class sizes).
constexpr int M1_V = 128;                                   // j and l variables per tile side
constexpr int M1_STAGE = 2 * TILE_ROWS * KBLK + KBLK + 64;  // j rows | l rows | i row | pad
constexpr int M1_NSTAGE = 2;   // operand stages: fetched one K block ahead (two workgroups per CU)

// NWV waves per workgroup: 4 (a 2 x 2 wave grid, 4 x 4 blocks of 16 x 16 triples per wave) or 8
// (2 x 4, 4 x 2 blocks per wave).  The launch uses 4: with 8 the epilogue needs 211 VGPRs (one
// workgroup per CU, 8.4 ms against 7.4 on the Madelon-shaped d = 2 call) or spills at 128.
template <int T, bool EXPORT = false, int NWV = 4>
__global__ __launch_bounds__(NWV * 64, 2) void k_sweep3m1(Sweep3mArgs a)
{
    constexpr int C = 2;
    constexpr int NT = NWV * 64;
    constexpr int NN = 16 / NWV;          // 16 x 16 column (l) blocks per wave; row (j) blocks: 4
    constexpr int LSPAN = 16 * NN;        // l variables per wave
    if (a.collect && a.st->collect_go == 0) return;   // collect pass not needed (uniform)
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char *stage = smem + a.stage_off;   // after the (L, Q) pairs of n = 0 .. N
    int64_t *s_next = reinterpret_cast<int64_t *>(smem + a.snext_off);

    const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wr = wave / (NWV / 2), wc = wave % (NWV / 2);
    const int q = lane >> 4, c16 = lane & 15;

    {
        float *tf = reinterpret_cast<float *>(smem);
        for (int i = t; i <= a.N0; i += NT) tf[i] = a.EA[i];
        for (int i = t; i <= a.N1; i += NT) tf[T + i] = a.EB[i];
        float2 *lq = reinterpret_cast<float2 *>(smem + 8 * T);
        for (int i = t; i <= a.N; i += NT) lq[i] = a.LQ[i];
    }
    auto repack = [](uint32_t x) -> uint32_t { return x << 2; };   // n1 << 16 | n0 -> fp4 packing
    const uint32_t Ntot = ((uint32_t)a.N1 << 18) | ((uint32_t)a.N0 << 2);
    const int64_t nrb = a.rows_pad / TILE_ROWS;
    constexpr int kstride = TILE_ROWS * KBLK;
    const int n1blk = a.KB - a.KB0;

    uint32_t taken = 0;   // tiles taken by this workgroup (cancel polling)
    for (;;) {
        __syncthreads();
        if (t == 0) *s_next = cancel_poll(a.cancel, taken++, a.st) ? a.n_tiles * a.nr : atomicAdd(&a.st->next_tile[0], 1u);
        __syncthreads();
        const int64_t u_all = uniform64(*s_next);
        if (u_all >= a.n_tiles * a.nr) break;
        // tile u of the list, under discretisation r = r0 + rr of the launch
        const int rr = (int)(u_all / a.n_tiles);
        const int64_t u = u_all - (int64_t)rr * a.n_tiles;
        const int r = a.r0 + rr;
        const uint32_t *margr = a.marg + (int64_t)r * a.p_pad * C;
        const uint32_t *ptab = a.ptab + (int64_t)rr * a.ptab_stride;
        const float *F2 = a.F2 + (int64_t)rr * a.f2_stride;
        int64_t lo = 0, hi = a.n_ablk - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (a.apref[mid] <= u) lo = mid; else hi = mid - 1;
        }
        const int ab = a.ablk[lo];
        const int i = ab >> 8, jb = ab & 255;
        const int lb = jb + (int)(u - a.apref[lo]);

        // ---------------------------------------------------------------- K loop
        const int8_t *panJ = a.onehot + ((int64_t)r * nrb + jb) * a.KB * kstride;
        const int8_t *panL = a.onehot + ((int64_t)r * nrb + lb) * a.KB * kstride;
        const int8_t *panI = a.onehot + ((int64_t)r * nrb + i / TILE_ROWS) * a.KB * kstride + (i % TILE_ROWS) * KBLK;
        auto kblock = [&](int s_) { return s_ < n1blk ? a.KB0 + s_ : s_ - n1blk; };
        auto stage_at = [&](int s_) { return stage + (s_ % M1_NSTAGE) * M1_STAGE; };
        // 17 fetches per K block: 8 of 1 KB for the j rows, 8 for the l rows (stage rows
        // 128..255), one of 64 bytes for the row of i (lanes 0..3).  Wave w takes fetches w,
        // w + NWV, ..., and wave 0 also the row of i.
        auto issue = [&](int s_) {
            const int64_t kb_off = (int64_t)kblock(s_) * kstride;
            char *st_ = stage_at(s_);
#pragma unroll
            for (int k = 0; k < 16 / NWV; ++k) {
                const int f = wave + NWV * k;
                const int srow = 16 * f + (lane >> 2);
                const int j = (lane & 3) ^ ((srow >> 1) & 3);
                const int8_t *src = f < 8 ? panJ + kb_off + srow * KBLK + j * 16
                                          : panL + kb_off + (srow - TILE_ROWS) * KBLK + j * 16;
                __builtin_amdgcn_global_load_lds((const void *)src,
                                                 (__attribute__((address_space(3))) void *)(st_ + f * 1024), 16, 0, 0);
            }
            if (wave == 0 && lane < 4) {
                const int8_t *src = panI + kb_off + lane * 16;
                __builtin_amdgcn_global_load_lds((const void *)src,
                                                 (__attribute__((address_space(3))) void *)(st_ + 16 * 1024), 16, 0, 0);
            }
        };
        v4f acc[4][NN];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < NN; ++n) acc[m][n] = v4f{0.f, 0.f, 0.f, 0.f};
        int offJ[4], offL[NN];
#pragma unroll
        for (int m = 0; m < 4; ++m) offJ[m] = lds_sw(64 * wr + 16 * m + c16, q);
#pragma unroll
        for (int n = 0; n < NN; ++n) offL[n] = TILE_ROWS * KBLK + lds_sw(LSPAN * wc + 16 * n + c16, q);
        const int offI = 2 * TILE_ROWS * KBLK + 16 * q;

        // Two stages: step s waits for its own fetches of block s (the only ones outstanding),
        // passes a barrier (block s is complete, and every wave has finished reading block s-1,
        // whose stage the fetch of block s+1 then takes) and fetches block s+1 before reading
        // the fragments of block s.
        issue(0);
        for (int s = 0; s < a.KB; ++s) {
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
            __builtin_amdgcn_s_barrier();
            if (s + 1 < a.KB) issue(s + 1);
            const char *st_ = stage_at(s);
            const v4i fi = *reinterpret_cast<const v4i *>(st_ + offI);
            v4i fa[4], fb[NN];
#pragma unroll
            for (int m = 0; m < 4; ++m) fa[m] = *reinterpret_cast<const v4i *>(st_ + offJ[m]) & fi;
#pragma unroll
            for (int n = 0; n < NN; ++n) fb[n] = *reinterpret_cast<const v4i *>(st_ + offL[n]);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < NN; ++n) {
                    const v8i a8{fa[m][0], fa[m][1], fa[m][2], fa[m][3], 0, 0, 0, 0};
                    const v8i b8{fb[n][0], fb[n][1], fb[n][2], fb[n][3], 0, 0, 0, 0};
                    acc[m][n] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, acc[m][n], 4, 4, 0, 0, 0, 0);
                }
            if (s == n1blk - 1) {
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < NN; ++n) acc[m][n] = acc[m][n] * 4096.0f;
            }
        }

        // ---------------------------------------------------------------- epilogue
        v4i cnt[4][NN];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < NN; ++n)
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const uint32_t uu = (uint32_t)acc[m][n][x];
                    cnt[m][n][x] = (int)(__umul24(uu >> 14, 245760u) + uu);
                }
        auto jvar = [&](int m, int x) { return jb * M1_V + 64 * wr + 16 * m + 4 * q + x; };
        // count export (EXPORT: this kernel plus the store): T[0][0][0] of the triples (i_sel, j, l)
        if (EXPORT && i == a.i_sel && r == a.disc_sel) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < NN; ++n)
#pragma unroll
                    for (int x = 0; x < 4; ++x) {
                        const int j = jvar(m, x), l = lb * M1_V + LSPAN * wc + 16 * n + c16;
                        if (!(i < j && j < l && l < a.p)) continue;
                        int32_t *o = a.counts_out + ((int64_t)j * a.p + l) * 2 * 8;
                        const uint32_t v = (uint32_t)cnt[m][n][x] >> 2;
                        o[0] = (int32_t)(v & 0xffffu);
                        o[8] = (int32_t)(v >> 16);
                    }
        }
        int lv[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) lv[n] = lb * M1_V + LSPAN * wc + 16 * n + c16;
        // pair data of (u, v) at byte offset 4 (u p_pad + v), every u, v < p_pad filled in (the
        // pair sweep's u < v < p and k_square_pairs' rest): every slot's counts are counts
        const uint32_t pp4 = 4u * (uint32_t)a.p_pad;
        const uint32_t pbytes = pp4 * (uint32_t)a.p_pad;
        // (bases re-read as uniform: a resource must sit in scalar registers)
        const __amdgpu_buffer_rsrc_t rsP = rsrc(reinterpret_cast<const void *>(uniform64((int64_t)ptab)), pbytes);
        const __amdgpu_buffer_rsrc_t rsF = rsrc(reinterpret_cast<const void *>(uniform64((int64_t)F2)), pbytes);
        const uint32_t io = (uint32_t)i * pp4;
        uint32_t lo4[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) lo4[n] = 4u * (uint32_t)lv[n];
        const uint32_t Mi = repack(margr[(uint32_t)i * C]);
        const uint32_t Ni1 = Ntot - Mi;                     // class sizes of x_i = 1
        uint32_t Ml[NN], Nil[NN];
        float Fil[NN], gL_read[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            const int l = lv[n];
            Ml[n] = repack(margr[(uint32_t)l * C]);
            Nil[n] = ld32(rsP, io + lo4[n]);
            Fil[n] = ldf(rsF, io + lo4[n]);
            gL_read[n] = key_f32(a.G32[l]);
        }
        const float Gi = key_f32(a.G32[i]);
        struct JData {
            uint32_t Nij[4], Mj[4], jo[4];   // N(0,0) of (i, j); bin-0 count of j; row offset of j
            float F[4], g[4];
        };
        auto load_j = [&](int m, JData &d) {
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const int j = jvar(m, x);
                d.jo[x] = (uint32_t)j * pp4;
                d.Mj[x] = repack(margr[(uint32_t)j * C]);
                d.Nij[x] = ld32(rsP, io + 4u * (uint32_t)j);
                d.F[x] = ldf(rsF, io + 4u * (uint32_t)j);
                d.g[x] = key_f32(a.G32[j]);
            }
        };
        // F3 of triple (i, j(m, x), l_n) from its direct count D and the pair count Njl of (j, l_n)
        auto triple = [&](int n, int x, const JData &jd, uint32_t D, uint32_t Njl) -> float {
            uint32_t V[8];
            V[0] = D;                                   // T000
            V[1] = jd.Nij[x] - D;                       // T001
            V[2] = Nil[n] - D;                          // T010
            V[3] = Njl - D;                             // T100
            const uint32_t Bj = jd.Mj[x] - jd.Nij[x];   // x_i = 1, x_j = 0
            V[4] = (Mi - jd.Nij[x]) - V[2];             // T011
            V[5] = Bj - V[3];                           // T101
            V[6] = (Ml[n] - Nil[n]) - V[3];             // T110
            V[7] = (Ni1 - Bj) - V[6];                   // T111
            return vox_sum<T, 8>(V);
        };

        // One pass, row by row (block row m: the j(m, x) of the lane's q): the row's (j, l) pair
        // data are loaded first, all loads in flight together; the F of the row's triples are
        // kept, the maxima of the row's members reduced over the wave, and the row's appends
        // decided against thresholds that are the larger of the maximum read before the tile and
        // the wave's maximum so far (both below the final maximum, so every triple within the
        // window of the final maximum is appended); a row whose wave maxima all stay below their
        // thresholds appends nothing and skips the selection; one slot reservation per row.
        float mi = -INFINITY, ml[NN];
#pragma unroll
        for (int n = 0; n < NN; ++n) ml[n] = -INFINITY;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            // the row's direct counts first (the row index is not a constant: the tile may live
            // in scratch memory), then the pair data, so that one wait covers every load
            v4i crow[NN];
#pragma unroll
            for (int n = 0; n < NN; ++n) crow[n] = cnt[m][n];
            JData jd;
            load_j(m, jd);
            uint32_t Njl[NN][4];
            float F3r[NN][4], Fjlr[NN][4], mjx[4];
#pragma unroll
            for (int n = 0; n < NN; ++n)
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const uint32_t o = jd.jo[x] + lo4[n];
                    Njl[n][x] = ld32(rsP, o);
                    Fjlr[n][x] = ldf(rsF, o);
                }
#pragma unroll
            for (int x = 0; x < 4; ++x) mjx[x] = -INFINITY;
#pragma unroll
            for (int n = 0; n < NN; ++n) {
#pragma unroll
                for (int x = 0; x < 4; ++x) F3r[n][x] = 0.f;
                // wave-uniform skip of a block without any valid triple
                if (!__any(i < jvar(m, 3) && jvar(m, 0) < lv[n] && lv[n] < a.p)) continue;
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int jraw = jvar(m, x);
                    const bool valid = (i < jraw) & (jraw < lv[n]) & (lv[n] < a.p);
                    const float F3 = triple(n, x, jd, (uint32_t)crow[n][x], Njl[n][x]);
                    F3r[n][x] = F3;
                    mi = fmaxf(mi, valid ? Fjlr[n][x] - F3 : -INFINITY);   // gain of x_i given (x_j, x_l)
                    mjx[x] = fmaxf(mjx[x], valid ? Fil[n] - F3 : -INFINITY);  // gain of x_j given (x_i, x_l)
                    ml[n] = fmaxf(ml[n], valid ? jd.F[x] - F3 : -INFINITY);  // gain of x_l given (x_i, x_j)
                }
            }
            // wave maxima so far: i over all lanes, j(m, x) over the 16 lanes of one q, l_n over
            // the lanes of one c16
            float wi = mi, wj[4], wl[NN];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) wi = fmaxf(wi, __shfl_xor(wi, o));
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                float y = mjx[x];
                y = fmaxf(y, __shfl_xor(y, 1));
                y = fmaxf(y, __shfl_xor(y, 2));
                y = fmaxf(y, __shfl_xor(y, 4));
                wj[x] = fmaxf(y, __shfl_xor(y, 8));
            }
#pragma unroll
            for (int n = 0; n < NN; ++n) {
                float y = ml[n];
                y = fmaxf(y, __shfl_xor(y, 16));
                wl[n] = fmaxf(y, __shfl_xor(y, 32));
            }
            const float tI = a.collect ? Gi : fmaxf(Gi, wi);
            const float thI = tI - win3(a.w_abs, tI);
            float thJ[4], thL[NN];
            bool hot = wi >= thI;
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const float tJ = a.collect ? jd.g[x] : fmaxf(jd.g[x], wj[x]);
                thJ[x] = tJ - win3(a.w_abs, tJ);
                hot |= wj[x] >= thJ[x];
            }
#pragma unroll
            for (int n = 0; n < NN; ++n) {
                const float tL = a.collect ? gL_read[n] : fmaxf(gL_read[n], wl[n]);
                thL[n] = tL - win3(a.w_abs, tL);
                hot |= wl[n] >= thL[n];
            }
            if (__any(hot)) {
                uint64_t sel = 0;   // bit 3 (4 n + x) + member
#pragma unroll
                for (int n = 0; n < NN; ++n)
#pragma unroll
                    for (int x = 0; x < 4; ++x) {
                        const int jraw = jvar(m, x);
                        const bool valid = (i < jraw) & (jraw < lv[n]) & (lv[n] < a.p);
                        const int b = 3 * (4 * n + x);
                        if (valid && Fjlr[n][x] - F3r[n][x] >= thI) sel |= 1ull << b;
                        if (valid && Fil[n] - F3r[n][x] >= thJ[x]) sel |= 2ull << b;
                        if (valid && jd.F[x] - F3r[n][x] >= thL[n]) sel |= 4ull << b;
                    }
                uint32_t at = reserve_slots(&a.st->n_cand, (uint32_t)__popcll(sel), lane);
                if (sel) {
#pragma unroll
                    for (int n = 0; n < NN; ++n)
#pragma unroll
                        for (int x = 0; x < 4; ++x) {
                            const int j = jvar(m, x), l = lv[n], b = 3 * (4 * n + x);
                            const float F3 = F3r[n][x];
                            if (sel & (1ull << b)) put(a, r, at++, i, ((uint32_t)j << 16) | (uint32_t)l, Fjlr[n][x] - F3);
                            if (sel & (2ull << b)) put(a, r, at++, j, ((uint32_t)i << 16) | (uint32_t)l, Fil[n] - F3);
                            if (sel & (4ull << b)) put(a, r, at++, l, ((uint32_t)i << 16) | (uint32_t)j, jd.F[x] - F3);
                        }
                }
            }
            // j(m, x) appears in this row only: its maximum goes out now
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const int j = jvar(m, x);
                if (!a.collect && c16 == 0 && j < a.p && wj[x] > jd.g[x]) atomicMax(&a.G32[j], f32_key(wj[x]));
            }
        }
        // i is the tile's; l_n is shared by the lanes of one c16
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mi = fmaxf(mi, __shfl_xor(mi, o));
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            float y = ml[n];
            y = fmaxf(y, __shfl_xor(y, 16));
            ml[n] = fmaxf(y, __shfl_xor(y, 32));
        }
        if (a.collect) continue;
        // only where the tile raised the maximum read before (maxima only grow)
        if (lane == 0 && mi > Gi) atomicMax(&a.G32[i], f32_key(mi));
#pragma unroll
        for (int n = 0; n < NN; ++n)
            if (q == 0 && ml[n] > gL_read[n]) atomicMax(&a.G32[lv[n]], f32_key(ml[n]));
    }
}

// LDS of the triple sweeps: tables EA [0, 4T), EB [4T, 8T), (L, Q) pairs from 8T; three classes:
// stages from 24T (compile-time offsets), two classes: stages after the N + 1 pairs in use
size_t m1_stage_off(int T, int N) { return ((size_t)8 * T + 8 * ((size_t)N + 1) + 127) & ~(size_t)127; }
size_t sweep3m_lds_of(int T, int W, int N)
{
    return W == 1 ? m1_stage_off(T, N) + M1_NSTAGE * M1_STAGE + 16 : (size_t)24 * T + M3_NSTAGE * M3_STAGE + 16;
}

int m3_capacity(const Problem &P)
{
    const int need = (P.N0 > P.N1 ? P.N0 : P.N1) + 1;
    for (int T = 1024; T <= 4096; T *= 2)
        if (need <= T) return T;
    return 0;
}

template <int T, int W>
hipError_t m3_launch(const Problem &P, int r0, int nr, bool collect, int32_t *counts_out, int i_sel, int disc_sel)
{
    const Layout &L = P.L;
    Sweep3mArgs a{};
    a.onehot = P.at<int8_t>(L.onehot);
    a.ptab = P.at<uint32_t>(L.ptab);
    a.F2 = P.at<float>(L.F2);
    a.marg = P.at<uint32_t>(L.marg);
    a.EA = P.at<float>(L.tabEA);
    a.EB = P.at<float>(L.tabEB);
    a.LQ = P.at<float2>(L.tabLQ);
    a.apref = P.at<int64_t>(L.a3pref);
    a.ablk = P.at<int32_t>(L.a3blk);
    a.n_ablk = P.n_ablk3;
    a.n_tiles = P.n_tiles3;
    a.N0 = P.N0;
    a.N1 = P.N1;
    a.N = (int)L.N;
    a.p = (int)L.p;
    a.p_pad = L.p_pad;
    a.rows_pad = L.rows_pad;
    a.KB = P.KB;
    a.KB0 = P.KB0;
    a.r0 = r0;
    a.nr = nr;
    a.ptab_stride = L.p_pad * L.p_pad * W * W;
    a.f2_stride = L.p_pad * L.p_pad;
    a.nLB = (int)((L.p + (W == 1 ? M1_V : M3_LV) - 1) / (W == 1 ? M1_V : M3_LV));
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
    const size_t lds = sweep3m_lds_of(T, W, (int)L.N);
    a.stage_off = (int)m1_stage_off(T, (int)L.N);
    a.snext_off = (int)(lds - 16);
    constexpr int nwv = 4;
    auto kern = W == 1 ? (counts_out ? k_sweep3m1<T, true, nwv> : k_sweep3m1<T, false, nwv>)
                       : (counts_out ? k_sweep3m<T, true> : k_sweep3m<T>);
    // the epilogue's table reads take LDS addresses equal to their offsets in the dynamic array:
    // no static LDS may come before it
    static const hipError_t lds_ok =
        lds_array_at_zero({(const void *)k_sweep3m1<T, true, nwv>, (const void *)k_sweep3m1<T, false, nwv>,
                           (const void *)k_sweep3m<T, true>, (const void *)k_sweep3m<T>});
    if (lds_ok != hipSuccess) return lds_ok;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(P.workgroups > 0 ? P.workgroups : 512), dim3(nwv * 64), lds, P.stream, a);
    return hipGetLastError();
}

}  // namespace

size_t sweep3m_lds_bytes(const Problem &P) { return sweep3m_lds_of(m3_capacity(P), P.L.W, (int)P.L.N); }

// Tile list of the triple sweep with JV j variables and LV l variables per tile (W = 2: 32 and
// 64; W = 1: 128 and 128): A blocks (i, jb) with jb >= (i + 1) / JV (some j > i) and
// jb * JV < p - 1, in order of i then jb, each with l blocks lb = jb * JV / LV .. nLB - 1.
// apref[k] = first tile of A block k, ablk[k] = i * 256 + jb, apref[n_ablk] = number of tiles.
static void m3_geometry(int W, int64_t p, int64_t &JV, int64_t &LV, int64_t &nJB, int64_t &nLB)
{
    JV = W == 1 ? M1_V : M3_JV;
    LV = W == 1 ? M1_V : M3_LV;
    nJB = (p + JV - 1) / JV;
    nLB = (p + LV - 1) / LV;
}

// A blocks and tiles of the list, on the host (the launch needs both before the list exists).
void sweep3m_tile_counts(int64_t p, int W, int64_t &n_ablk, int64_t &n_tiles)
{
    int64_t JV, LV, nJB, nLB;
    m3_geometry(W, p, JV, LV, nJB, nLB);
    n_ablk = n_tiles = 0;
    for (int64_t i = 0; i + 2 < p; ++i)
        for (int64_t jb = (i + 1) / JV; jb < nJB && jb * JV < p - 1; ++jb) {
            ++n_ablk;
            n_tiles += nLB - jb * JV / LV;
        }
}

// The list itself, built on the device by one workgroup (so that an asynchronous or captured
// call needs no host-to-device copy): each thread counts the A blocks and tiles of a contiguous
// range of i, a block-wide exclusive scan gives every range its first entry and first tile,
// then each thread writes its entries.
__global__ __launch_bounds__(1024) void k_tiles3(int64_t p, int64_t JV, int64_t LV, int64_t nJB, int64_t nLB,
                                                 int64_t *apref, int32_t *ablk)
{
    __shared__ int64_t sA[1024], sT[1024];
    const int t = threadIdx.x;
    const int64_t ni = p >= 3 ? p - 2 : 0;            // i = 0 .. p - 3
    const int64_t per = (ni + 1023) / 1024;
    const int64_t i0 = t * per < ni ? t * per : ni, i1 = i0 + per < ni ? i0 + per : ni;
    int64_t ca = 0, ct = 0;
    for (int64_t i = i0; i < i1; ++i)
        for (int64_t jb = (i + 1) / JV; jb < nJB && jb * JV < p - 1; ++jb) {
            ++ca;
            ct += nLB - jb * JV / LV;
        }
    sA[t] = ca;
    sT[t] = ct;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t xa = t >= d ? sA[t - d] : 0, xt = t >= d ? sT[t - d] : 0;
        __syncthreads();
        sA[t] += xa;
        sT[t] += xt;
        __syncthreads();
    }
    int64_t ka = sA[t] - ca, kt = sT[t] - ct;
    for (int64_t i = i0; i < i1; ++i)
        for (int64_t jb = (i + 1) / JV; jb < nJB && jb * JV < p - 1; ++jb) {
            apref[ka] = kt;
            ablk[ka] = (int32_t)(i * 256 + jb);
            ++ka;
            kt += nLB - jb * JV / LV;
        }
    if (t == 1023) apref[sA[1023]] = sT[1023];
}

hipError_t launch_tiles3(const Problem &P)
{
    int64_t JV, LV, nJB, nLB;
    m3_geometry(P.L.W, P.L.p, JV, LV, nJB, nLB);
    hipLaunchKernelGGL(k_tiles3, dim3(1), dim3(1024), 0, P.stream, P.L.p, JV, LV, nJB, nLB,
                       P.at<int64_t>(P.L.a3pref), P.at<int32_t>(P.L.a3blk));
    return hipGetLastError();
}

// The triple tiles read the pair tables of every (u, v) they touch, u >= v and padding variables
// (v >= p) included, while the pair sweep writes u < v < p only.  This fills in the rest so that
// whatever three variables a tile slot names, its derived counts are counts of real variables
// (non-negative and at most the class sizes), and the epilogue need not mask them: below the
// diagonal the transpose, on it the variable against itself (4 M_u(a) where a = b, else 0: the
// counts are stored as byte offsets, (4 n1) << 16 | 4 n0, for this engine), and for
// a padding variable, whose one-hot rows are zero (every object in the last bin), zeros, with the
// class sizes in the last bin of its marginals.  One launch per chunk of discretisations, for the
// two-class kernel (8.5% faster without its masks); the three-class one keeps its masks (1.7%
// faster than this pass plus unmasked slots).
template <int W>
__global__ __launch_bounds__(256) void k_square_pairs(uint32_t *ptab, uint32_t *marg, int64_t p, int64_t p_pad, int r0,
                                                      int nr, uint32_t ntot)
{
    constexpr int C = W + 1;
    const int64_t n = (int64_t)nr * p_pad * p_pad, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += stride) {
        const int64_t rr = idx / (p_pad * p_pad), uv = idx - rr * p_pad * p_pad;
        const int64_t u = uv / p_pad, v = uv - u * p_pad;
        if (u < v && v < p) continue;   // written by the pair sweep
        uint32_t *dst = ptab + idx * (W * W);
        if (u >= p || v >= p) {
#pragma unroll
            for (int k = 0; k < W * W; ++k) dst[k] = 0u;
        } else if (u == v) {
            const uint32_t *m = marg + ((int64_t)(r0 + rr) * p_pad + u) * C;
#pragma unroll
            for (int x = 0; x < W; ++x)
#pragma unroll
                for (int y = 0; y < W; ++y) dst[x * W + y] = x == y ? m[x] << 2 : 0u;
        } else {
            const uint32_t *src = ptab + ((rr * p_pad + v) * p_pad + u) * (W * W);
#pragma unroll
            for (int x = 0; x < W; ++x)
#pragma unroll
                for (int y = 0; y < W; ++y) dst[x * W + y] = src[y * W + x];
        }
    }
    const int64_t npad = (int64_t)nr * (p_pad - p);
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < npad; idx += stride) {
        const int64_t rr = idx / (p_pad - p), v = p + (idx - rr * (p_pad - p));
        marg[((int64_t)(r0 + rr) * p_pad + v) * C + W] = ntot;
    }
}

hipError_t launch_sweep3m(const Problem &P, int r0, int nr, bool collect, int32_t *counts_out, int i_sel, int disc_sel)
{
    hipError_t e = launch_reset_queue(P);
    if (e != hipSuccess) return e;
    if (P.L.W == 1) {
        const uint32_t ntot = ((uint32_t)P.N1 << 16) | (uint32_t)P.N0;
        hipLaunchKernelGGL(k_square_pairs<1>, dim3(1024), dim3(256), 0, P.stream, P.at<uint32_t>(P.L.ptab),
                           P.at<uint32_t>(P.L.marg), P.L.p, P.L.p_pad, r0, nr, ntot);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const bool w1 = P.L.W == 1;
    switch (m3_capacity(P)) {
    case 1024: return w1 ? m3_launch<1024, 1>(P, r0, nr, collect, counts_out, i_sel, disc_sel)
                         : m3_launch<1024, 2>(P, r0, nr, collect, counts_out, i_sel, disc_sel);
    case 2048: return w1 ? m3_launch<2048, 1>(P, r0, nr, collect, counts_out, i_sel, disc_sel)
                         : m3_launch<2048, 2>(P, r0, nr, collect, counts_out, i_sel, disc_sel);
    case 4096: return w1 ? m3_launch<4096, 1>(P, r0, nr, collect, counts_out, i_sel, disc_sel)
                         : m3_launch<4096, 2>(P, r0, nr, collect, counts_out, i_sel, disc_sel);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mdfs
