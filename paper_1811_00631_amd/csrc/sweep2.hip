// sweep2.hip -- the k = 2 tuple sweep on the gfx950 matrix cores.
//
// Counting (the voxel counters N^d of section "Algorithm and implementation", named there the
// most time-consuming part): with objects sorted by class and each variable one-hot encoded on
// its first W = C-1 bins, the per-class pair tables are the Gram products X_d^T X_d.  A tile of
// 128 x 128 one-hot rows is accumulated on the matrix cores in one of two encodings:
//   fp4:  E2M1 nibbles (1.0 = 0b0010), V_MFMA_F32_16X16X128_F8F6F4, float32 accumulators.
//         Class-1 objects are accumulated first, the accumulator is scaled by 4096, then
//         class-0 objects are added: n1 * 4096 + n0 < 2^24 is an exact float32 integer while
//         each class has < 4096 objects.  Half the operand bytes and twice the rate of int8.
//   int8: bytes, V_MFMA_I32_16X16X64_I8, int32 accumulators shifted left by 16 between the
//         classes: (n1 << 16) | n0 for classes < 32768 objects.
// Either way the epilogue works on packed integers n1 << SH | n0 (SH = 12 or 16).  The dropped
// last bin of each variable is rebuilt exactly from the per-class marginals (packed
// subtraction never borrows because every reconstructed count is >= 0).
//
// Epilogue (the pseudocounted entropy of the class-probability equation and IG of equation
// IGmax): per pair F2 = sum_v n_v h(p_v) from float32 lookup tables indexed by integer counts,
// IG(i|j) = F1(j) - F2 and IG(j|i) = F1(i) - F2.  This float32 value is a screen with a proven
// bound E on its error: each variable's float32 maximum is kept with an atomic max on an
// order-preserving key, and every (pair, discretisation) that may be within 2E + tau of the
// final maximum is appended to a candidate buffer; the finalize pass re-scores candidates in
// binary64 from exact recounts.
#include "mdfs_internal.h"

namespace mdfs {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
template <bool F4> struct AccOf { typedef v4i type; };
template <> struct AccOf<true> { typedef v4f type; };

constexpr int SW_THREADS = 256;          // 4 waves, 2 x 2 wave grid, 64 x 64 outputs per wave
constexpr int SB = 8;                    // a super-tile is SB x SB tiles
constexpr int XCDS = 8;                  // workgroup b runs on XCD b % 8
constexpr int WG_PER_XCD = SB * SB;      // resident workgroups per XCD (2 per CU)
constexpr int STAGE_BYTES = 2 * TILE_ROWS * KBLK;   // A and B tiles of one K block
constexpr int NSTAGE = 3;                           // LDS ring of K blocks

struct Sweep2Args {
    const int8_t *onehot;
    const uint32_t *marg;
    const float *F1;
    const float *EA, *EB;
    const float2 *LQ;
    int N0, N1, N;
    int p;
    int64_t p_pad, rows_pad;
    int R, KB, KB0;
    int nbv;                 // variable blocks of TV = TILE_ROWS / W variables
    int nsb;                 // super-blocks of SB variable blocks
    int64_t super_per_r, n_super;
    uint32_t *G32;
    Cand *cand;
    int64_t cap;
    Status *st;
    uint32_t *ovf;
    float w_abs;
    int32_t *counts_out;     // debug: full tables of discretisation disc_sel
    int disc_sel;
    int collect;             // second pass: G32 holds the final maxima; append only
    int r_base;              // first discretisation of this launch
    uint32_t *ptab;          // pair mode: packed (W x W) counts [p_pad][p_pad][W*W]
    float *F2out;            // pair mode: float32 F of each pair table [p_pad][p_pad]
};

// What one launch of the pair sweep produces.
enum SweepMode { SWEEP_MAX = 0, SWEEP_DEBUG_COUNTS = 1, SWEEP_PAIRS = 2 };

// Swizzled LDS address of 16-byte chunk j (0..3) of tile row `row` (64 bytes per row).
__device__ inline int lds_addr(int row, int j) { return row * KBLK + ((j ^ ((row >> 1) & 3)) << 4); }

template <int SH>
__device__ inline float vox_term(uint32_t P, const float *EA, const float *EB, const float2 *LQ)
{
    const uint32_t n0 = P & ((1u << SH) - 1u), n1 = P >> SH;
    const float2 lq = LQ[n0 + n1];
    return lq.x - lq.y * (EA[n0] + EB[n1]);
}

__device__ inline float rescore_window(float w_abs, float g)
{
    float ag = fabsf(g);
    return w_abs + 2e-9f * (ag > 1.f ? ag : 1.f) + 1e-30f;
}

// Triangular tile index -> (bi, bj), bi <= bj.
__device__ inline void tri_index(int64_t tt, int &bi, int &bj)
{
    int64_t j = (int64_t)((sqrt(8.0 * (double)tt + 1.0) - 1.0) * 0.5);
    while ((j + 1) * (j + 2) / 2 <= tt) ++j;
    while (j * (j + 1) / 2 > tt) --j;
    bj = (int)j;
    bi = (int)(tt - j * (j + 1) / 2);
}

template <int W, int MODE, bool F4>
__global__ __launch_bounds__(SW_THREADS, 2) void k_sweep2(Sweep2Args a)
{
    constexpr int C = W + 1;
    constexpr int SH = F4 ? 12 : 16;     // packing n1 << SH | n0 of the counts
    constexpr uint32_t MASK = (1u << SH) - 1u;
    typedef typename AccOf<F4>::type Acc;
    constexpr int TV = TILE_ROWS / W;    // variables per tile side
    constexpr int NP = (W == 1) ? 4 : 1; // pairs held per lane per 16x16 block
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char *stage = smem;                  // [NSTAGE buffers][A 8 KB | B 8 KB]
    float *EA = reinterpret_cast<float *>(smem + NSTAGE * STAGE_BYTES);
    float *EB = EA + (a.N0 + 1);
    float2 *LQ = reinterpret_cast<float2 *>(EB + (a.N1 + 1) + ((a.N0 + a.N1) & 1));

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int q = lane >> 4, c16 = lane & 15;

    for (int i = t; i <= a.N0; i += SW_THREADS) EA[i] = a.EA[i];
    for (int i = t; i <= a.N1; i += SW_THREADS) EB[i] = a.EB[i];
    for (int i = t; i <= a.N; i += SW_THREADS) LQ[i] = a.LQ[i];

    // Persistent, XCD-aware schedule.  The super-tiles sup = x, x+8, x+16 ... belong to XCD x;
    // the workgroups resident on that XCD take its tiles (super-tile by super-tile, slot by
    // slot) from one atomic counter, so at any time they work on the same SB x SB block of
    // tiles and share its SB row panels and SB column panels in the XCD's L2.
    const int xcd = (int)(__builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & 7);  // HW_REG_XCC_ID
    const int64_t n_mine = ((a.n_super - xcd + XCDS - 1) / XCDS) * (SB * SB);
    __shared__ int64_t s_next;
    for (;;) {
    __syncthreads();   // everyone has read the previous s_next
    if (t == 0) s_next = atomicAdd(&a.st->next_tile[xcd], 1u);
    __syncthreads();
    const int64_t item = s_next;
    if (item >= n_mine) break;
    const int64_t sup = xcd + XCDS * (item / (SB * SB));
    const int slot = (int)(item % (SB * SB));
    const int r = a.r_base + (int)(sup / a.super_per_r);
    int SI, SJ;
    tri_index(sup % a.super_per_r, SI, SJ);
    const int bi = SI * SB + slot / SB, bj = SJ * SB + slot % SB;
    if (bi > bj || bj >= a.nbv) continue;   // workgroup-uniform

    // ---------------------------------------------------------------- K loop
    // operand panels: TILE_ROWS one-hot rows x all K blocks, contiguous (panel-major layout)
    const int64_t nrb = a.rows_pad / TILE_ROWS;
    const int8_t *panA = a.onehot + ((int64_t)r * nrb + bi) * a.KB * TILE_ROWS * KBLK;
    const int8_t *panB = a.onehot + ((int64_t)r * nrb + bj) * a.KB * TILE_ROWS * KBLK;
    const int n1blk = a.KB - a.KB0;      // class-1 K blocks, accumulated first
    // this thread's two 16-byte chunks of the A tile and two of the B tile
    const int ra0 = t >> 2, ja0 = t & 3, ra1 = (t + SW_THREADS) >> 2, ja1 = (t + SW_THREADS) & 3;
    const int offA0 = ra0 * KBLK + ja0 * 16, offA1 = ra1 * KBLK + ja1 * 16;
    const int sA0 = lds_addr(ra0, ja0), sA1 = lds_addr(ra1, ja1);
    constexpr int kstride = TILE_ROWS * KBLK;

    Acc acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = Acc{0, 0, 0, 0};

    // K blocks in processing order: class 1 first, then class 0
    auto kblock = [&](int s_) { return s_ < n1blk ? a.KB0 + s_ : s_ - n1blk; };
    auto stage_at = [&](int s_) { return stage + (s_ % NSTAGE) * STAGE_BYTES; };
    // Software pipeline over a ring of NSTAGE LDS stages.  Iteration s: global loads of block
    // s+3 go out, the fragments of block s are read from LDS and multiplied, and block s+2
    // (loaded one iteration earlier) is written to LDS; one barrier per iteration.
    v4i g0, g1, g2, g3, h0, h1, h2, h3;
    auto gl = [&](int s_, v4i &x0, v4i &x1, v4i &x2, v4i &x3) {
        const int64_t kb_off = (int64_t)kblock(s_) * kstride;
        x0 = *reinterpret_cast<const v4i *>(panA + kb_off + offA0);
        x1 = *reinterpret_cast<const v4i *>(panA + kb_off + offA1);
        x2 = *reinterpret_cast<const v4i *>(panB + kb_off + offA0);
        x3 = *reinterpret_cast<const v4i *>(panB + kb_off + offA1);
    };
    auto st4 = [&](int s_, const v4i &x0, const v4i &x1, const v4i &x2, const v4i &x3) {
        char *A = stage_at(s_), *B = A + TILE_ROWS * KBLK;
        *reinterpret_cast<v4i *>(A + sA0) = x0;
        *reinterpret_cast<v4i *>(A + sA1) = x1;
        *reinterpret_cast<v4i *>(B + sA0) = x2;
        *reinterpret_cast<v4i *>(B + sA1) = x3;
    };
    const int fa_off0 = lds_addr(wr * 64 + c16, q), fb_off0 = lds_addr(wc * 64 + c16, q);
    v4i fa[4], fb[4];
    auto frags = [&](int s_, v4i (&xa)[4], v4i (&xb)[4]) {
        const char *A = stage_at(s_), *B = A + TILE_ROWS * KBLK;
#pragma unroll
        for (int m = 0; m < 4; ++m) xa[m] = *reinterpret_cast<const v4i *>(A + fa_off0 + m * 16 * KBLK);
#pragma unroll
        for (int n = 0; n < 4; ++n) xb[n] = *reinterpret_cast<const v4i *>(B + fb_off0 + n * 16 * KBLK);
    };
    gl(0, g0, g1, g2, g3);
    st4(0, g0, g1, g2, g3);
    if (a.KB > 1) { gl(1, g0, g1, g2, g3); st4(1, g0, g1, g2, g3); }
    if (a.KB > 2) gl(2, g0, g1, g2, g3);
    __syncthreads();
    // One pipeline step; the register sets (x = block s+2, y <- block s+3) swap roles between
    // consecutive steps, so no copy forces an early wait on the loads in flight.
    auto kstep = [&](int s_, v4i &x0, v4i &x1, v4i &x2, v4i &x3, v4i &y0, v4i &y1, v4i &y2, v4i &y3) {
        if (s_ + 3 < a.KB) gl(s_ + 3, y0, y1, y2, y3);
        frags(s_, fa, fb);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n)
            {
                if constexpr (F4) {
                    // A/B: 16 rows x 128 objects, lane l holds row l % 16, 32 nibbles of
                    // objects 32 (l / 16) ..; cbsz = blgp = 4 selects E2M1 for both operands
                    const v8i a8{fa[m][0], fa[m][1], fa[m][2], fa[m][3], 0, 0, 0, 0};
                    const v8i b8{fb[n][0], fb[n][1], fb[n][2], fb[n][3], 0, 0, 0, 0};
                    acc[m][n] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, acc[m][n], 4, 4, 0, 0, 0, 0);
                } else {
                    acc[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[m], fb[n], acc[m][n], 0, 0, 0);
                }
            }
        if (s_ == n1blk - 1) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    if constexpr (F4) acc[m][n] = acc[m][n] * 4096.0f;
                    else acc[m][n] = acc[m][n] << 16;
                }
        }
        if (s_ + 2 < a.KB) st4(s_ + 2, x0, x1, x2, x3);
        __syncthreads();
    };
    int s = 0;
    for (; s + 1 < a.KB; s += 2) {
        kstep(s, g0, g1, g2, g3, h0, h1, h2, h3);
        kstep(s + 1, h0, h1, h2, h3, g0, g1, g2, g3);
    }
    if (s < a.KB) kstep(s, g0, g1, g2, g3, h0, h1, h2, h3);

    // ---------------------------------------------------------------- epilogue
    // packed integer counts n1 << SH | n0 (float32 accumulators hold exact integers < 2^24)
    v4i cnt[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            if constexpr (F4) {
#pragma unroll
                for (int e = 0; e < 4; ++e) cnt[m][n][e] = (int)(uint32_t)acc[m][n][e];
            } else {
                cnt[m][n] = acc[m][n];
            }
        }
    // Lane geometry of the 16x16 output block (m, n): lane holds rows 4q..4q+3 of column c16.
    // Row/column index = variable * W + bin within the block.
    const int64_t I0 = (int64_t)bi * TV, J0 = (int64_t)bj * TV;
    const int odd = lane & 1;
    auto row_var = [&](int m, int s) -> int64_t {
        if (W == 1) return I0 + wr * 64 + m * 16 + 4 * q + s;
        return I0 + wr * 32 + m * 8 + 2 * q + odd;
    };
    auto col_var = [&](int n) -> int64_t {
        if (W == 1) return J0 + wc * 64 + n * 16 + c16;
        return J0 + wc * 32 + n * 8 + (c16 >> 1);
    };
    const uint32_t *margr = a.marg + (int64_t)r * a.p_pad * C;
    const float *F1r = a.F1 + (int64_t)r * a.p_pad;

    // marginals are stored n1 << 16 | n0; repack to the accumulators' SH
    auto repack = [](uint32_t x) -> uint32_t { return SH == 16 ? x : ((x >> 16) << SH) | (x & 0xffffu); };
    uint32_t Mr[4][NP][C], Mc[4][C];
    float Fr[4][NP], Fc[4];
    float thrR[4][NP], thrC[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int s = 0; s < NP; ++s) {
            int64_t v = row_var(m, s);
#pragma unroll
            for (int c = 0; c < C; ++c) Mr[m][s][c] = repack(margr[v * C + c]);
            Fr[m][s] = F1r[v];
            float gk = key_f32(a.G32[v]);
            thrR[m][s] = gk - rescore_window(a.w_abs, gk);
        }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        int64_t v = col_var(n);
#pragma unroll
        for (int c = 0; c < C; ++c) Mc[n][c] = repack(margr[v * C + c]);
        Fc[n] = F1r[v];
        float gk = key_f32(a.G32[v]);
        thrC[n] = gk - rescore_window(a.w_abs, gk);
    }

    // Full per-class table of the lane's pair(s) in block (m, n): packed counts tab[a][b].
    auto pair_table = [&](int m, int n, int s, uint32_t (&tab)[C][C]) {
        const v4i &ac = cnt[m][n];
        if constexpr (W == 1) {
            uint32_t n00 = (uint32_t)ac[s];
            tab[0][0] = n00;
            tab[0][1] = Mr[m][s][0] - n00;
            tab[1][0] = Mc[n][0] - n00;
            tab[1][1] = Mc[n][1] - tab[0][1];
        } else {
            const uint32_t a0 = ac[0], a1 = ac[1], a2 = ac[2], a3 = ac[3];
            const uint32_t s0 = odd ? a0 : a2, s1 = odd ? a1 : a3;
            const uint32_t x0 = (uint32_t)__builtin_amdgcn_mov_dpp((int)s0, 0xB1, 0xF, 0xF, false);
            const uint32_t x1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)s1, 0xB1, 0xF, 0xF, false);
            const uint32_t n00 = odd ? x0 : a0, n10 = odd ? x1 : a1;
            const uint32_t n01 = odd ? a2 : x0, n11 = odd ? a3 : x1;
            tab[0][0] = n00; tab[0][1] = n01; tab[1][0] = n10; tab[1][1] = n11;
            tab[0][2] = Mr[m][s][0] - n00 - n01;
            tab[1][2] = Mr[m][s][1] - n10 - n11;
            tab[2][0] = Mc[n][0] - n00 - n10;
            tab[2][1] = Mc[n][1] - n01 - n11;
            tab[2][2] = Mc[n][2] - tab[0][2] - tab[1][2];
        }
    };
    auto pair_F2 = [&](const uint32_t (&tab)[C][C]) {
        float F = 0.f;
#pragma unroll
        for (int x = 0; x < C; ++x)
#pragma unroll
            for (int y = 0; y < C; ++y) F += vox_term<SH>(tab[x][y], EA, EB, LQ);
        return F;
    };

    float rmax[4][NP], cmax[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int s = 0; s < NP; ++s) rmax[m][s] = -INFINITY;
#pragma unroll
    for (int n = 0; n < 4; ++n) cmax[n] = -INFINITY;
    bool hot = false;

    const bool emit = MODE == SWEEP_DEBUG_COUNTS && r == a.disc_sel;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int s = 0; s < NP; ++s) {
                uint32_t tab[C][C];
                pair_table(m, n, s, tab);
                const int64_t rv = row_var(m, s), cv = col_var(n);
                const bool valid = rv < cv && cv < a.p;
                const float F2 = pair_F2(tab);
                if constexpr (MODE == SWEEP_PAIRS) {
                    // parent data of the k = 3 sweep: the W x W packed counts and F of the pair
                    if (valid) {
                        uint32_t *o = a.ptab + (rv * a.p_pad + cv) * (W * W);
#pragma unroll
                        for (int x = 0; x < W; ++x)
#pragma unroll
                            for (int y = 0; y < W; ++y)
                                o[x * W + y] = ((tab[x][y] >> SH) << 16) | (tab[x][y] & MASK);
                        a.F2out[rv * a.p_pad + cv] = F2;
                    }
                    continue;
                }
                const float igR = valid ? Fc[n] - F2 : -INFINITY;   // gain of rv given cv
                const float igC = valid ? Fr[m][s] - F2 : -INFINITY; // gain of cv given rv
                rmax[m][s] = fmaxf(rmax[m][s], igR);
                cmax[n] = fmaxf(cmax[n], igC);
                hot |= (igR >= thrR[m][s]) | (igC >= thrC[n]);

                if (emit && valid) {
                    int32_t *o = a.counts_out + ((int64_t)rv * a.p + cv) * 2 * C * C;
#pragma unroll
                    for (int x = 0; x < C; ++x)
#pragma unroll
                        for (int y = 0; y < C; ++y) {
                            o[x * C + y] = (int32_t)(tab[x][y] & MASK);
                            o[C * C + x * C + y] = (int32_t)(tab[x][y] >> SH);
                        }
                }
            }

    if constexpr (MODE == SWEEP_PAIRS) continue;
    // wave-level maxima per variable: lanes sharing a row variable differ in the bits that
    // select the column; lanes sharing a column variable differ in the row-selecting bits
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int s = 0; s < NP; ++s) {
            float x = rmax[m][s];
            if (W == 1) { x = fmaxf(x, __shfl_xor(x, 1)); }
            x = fmaxf(x, __shfl_xor(x, 2));
            x = fmaxf(x, __shfl_xor(x, 4));
            x = fmaxf(x, __shfl_xor(x, 8));
            rmax[m][s] = x;
        }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        float x = cmax[n];
        if (W == 2) x = fmaxf(x, __shfl_xor(x, 1));
        x = fmaxf(x, __shfl_xor(x, 16));
        x = fmaxf(x, __shfl_xor(x, 32));
        cmax[n] = x;
    }
    // appends (second pass over the same accumulators), only if some value reached the
    // pre-tile threshold
    if (__any(hot)) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int s = 0; s < NP; ++s) {
                float g = key_f32(a.G32[row_var(m, s)]);
                float top = a.collect ? g : fmaxf(g, rmax[m][s]);
                thrR[m][s] = top - rescore_window(a.w_abs, top);
            }
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            float g = key_f32(a.G32[col_var(n)]);
            float top = a.collect ? g : fmaxf(g, cmax[n]);
            thrC[n] = top - rescore_window(a.w_abs, top);
        }
        // recompute from the accumulators (appends are rare); the empty asm stops the compiler
        // from keeping the first pass's values alive instead
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) asm volatile("" : "+v"(cnt[m][n]) : : "memory");
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n)
#pragma unroll
                for (int s = 0; s < NP; ++s) {
                    const int64_t rv = row_var(m, s), cv = col_var(n);
                    const bool valid = rv < cv && cv < a.p;
                    uint32_t tab[C][C];
                    pair_table(m, n, s, tab);
                    const float F2 = pair_F2(tab);
                    const float igR = Fc[n] - F2, igC = Fr[m][s] - F2;
                    if (valid && igR >= thrR[m][s]) {
                        uint32_t at = atomicAdd(&a.st->n_cand, 1u);
                        if (at < a.cap) a.cand[at] = Cand{(int32_t)rv, r, (uint32_t)cv, igR};
                        else { atomicOr(&a.ovf[rv], 1u); atomicOr(&a.st->overflow, 1u); }
                    }
                    if (valid && igC >= thrC[n]) {
                        uint32_t at = atomicAdd(&a.st->n_cand, 1u);
                        if (at < a.cap) a.cand[at] = Cand{(int32_t)cv, r, (uint32_t)rv, igC};
                        else { atomicOr(&a.ovf[cv], 1u); atomicOr(&a.st->overflow, 1u); }
                    }
                }
    }

    // publish the maxima: one lane per variable (the collect pass leaves the final maxima alone)
    if (a.collect) continue;
    const bool row_leader = (W == 1) ? (c16 == 0) : ((c16 >> 1) == 0);
    const bool col_leader = (W == 1) ? (q == 0) : (q == 0 && odd == 0);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int s = 0; s < NP; ++s)
            if (row_leader && rmax[m][s] > -INFINITY) atomicMax(&a.G32[row_var(m, s)], f32_key(rmax[m][s]));
#pragma unroll
    for (int n = 0; n < 4; ++n)
        if (col_leader && cmax[n] > -INFINITY) atomicMax(&a.G32[col_var(n)], f32_key(cmax[n]));
    }   // work items
}

template <int W, bool F4>
static hipError_t sweep_launch(const Problem &P, int32_t *counts_out, int disc_sel, bool collect, int pair_r)
{
    const Layout &L = P.L;
    Sweep2Args a{};
    a.onehot = P.at<int8_t>(L.onehot);
    a.marg = P.at<uint32_t>(L.marg);
    a.F1 = P.at<float>(L.F1);
    a.EA = P.at<float>(L.tabEA);
    a.EB = P.at<float>(L.tabEB);
    a.LQ = P.at<float2>(L.tabLQ);
    a.N0 = P.N0;
    a.N1 = P.N1;
    a.N = (int)L.N;
    a.p = (int)L.p;
    a.p_pad = L.p_pad;
    a.rows_pad = L.rows_pad;
    a.R = L.R;
    a.KB = P.KB;
    a.KB0 = P.KB0;
    constexpr int TV = TILE_ROWS / W;
    a.nbv = (int)((L.p + TV - 1) / TV);
    a.nsb = (a.nbv + SB - 1) / SB;
    a.super_per_r = (int64_t)a.nsb * (a.nsb + 1) / 2;
    a.n_super = a.super_per_r * (pair_r >= 0 ? 1 : L.R);
    a.r_base = pair_r >= 0 ? pair_r : 0;
    a.ptab = pair_r >= 0 ? P.at<uint32_t>(L.ptab) : nullptr;
    a.F2out = pair_r >= 0 ? P.at<float>(L.F2) : nullptr;
    a.G32 = P.at<uint32_t>(L.G32);
    a.cand = P.at<Cand>(L.cand);
    a.cap = L.cap;
    a.st = P.at<Status>(L.status);
    a.ovf = P.at<uint32_t>(L.ovf);
    a.w_abs = (float)(2.0 * P.err_bound);
    a.counts_out = counts_out;
    a.disc_sel = disc_sel;
    a.collect = collect ? 1 : 0;
    size_t lds = NSTAGE * STAGE_BYTES + sizeof(float) * (size_t)(P.N0 + 1 + P.N1 + 1 + 1) + sizeof(float2) * (L.N + 1) + 16;
    auto kern = pair_r >= 0 ? k_sweep2<W, SWEEP_PAIRS, F4>
                            : (counts_out ? k_sweep2<W, SWEEP_DEBUG_COUNTS, F4> : k_sweep2<W, SWEEP_MAX, F4>);
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int grid = XCDS * WG_PER_XCD;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(SW_THREADS), lds, P.stream, a);
    return hipGetLastError();
}

template <bool F4>
static hipError_t sweep_dispatch(const Problem &P, int32_t *counts_out, int disc_sel, bool collect, int pair_r)
{
    switch (P.L.W) {
    case 1: return sweep_launch<1, F4>(P, counts_out, disc_sel, collect, pair_r);
    case 2: return sweep_launch<2, F4>(P, counts_out, disc_sel, collect, pair_r);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep2(const Problem &P, int32_t *counts_out, int disc_sel, bool collect)
{
    return P.fp4 ? sweep_dispatch<true>(P, counts_out, disc_sel, collect, -1)
                 : sweep_dispatch<false>(P, counts_out, disc_sel, collect, -1);
}

hipError_t launch_pairs(const Problem &P, int r)
{
    return P.fp4 ? sweep_dispatch<true>(P, nullptr, -1, false, r) : sweep_dispatch<false>(P, nullptr, -1, false, r);
}

}  // namespace mdfs
