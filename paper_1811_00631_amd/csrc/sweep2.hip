// sweep2.hip -- the k = 2 tuple sweep on the gfx950 matrix cores.
//
// Counting (the voxel counters N^d of section "Algorithm and implementation", named there the
// most time-consuming part): with objects sorted by class and each variable one-hot encoded on
// its first W = C-1 bins, the per-class pair tables are the Gram products X_d^T X_d.  A tile of
// 128 x 128 one-hot rows is accumulated with V_MFMA_I32_16X16X64_I8 (int8 in, int32 out, exact
// since counts <= N).  Both classes share one accumulator: class-1 objects are accumulated
// first, the accumulator is shifted left by 16, then class-0 objects are added, so each int32
// holds (n1 << 16) | n0 (each class < 32768 objects).  The dropped last bin of each variable
// is rebuilt exactly from the per-class marginals (packed 16-bit subtraction never borrows
// because every reconstructed count is >= 0).
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

constexpr int SW_THREADS = 256;          // 4 waves, 2 x 2 wave grid, 64 x 64 outputs per wave
constexpr int STAGE_BYTES = 2 * TILE_ROWS * KBLK;   // A and B tiles of one K block

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
    int64_t tiles_per_r, n_tiles, per_xcd;
    uint32_t *G32;
    Cand *cand;
    int64_t cap;
    Status *st;
    uint32_t *ovf;
    float w_abs;
    int32_t *counts_out;     // debug: full tables of discretisation disc_sel
    int disc_sel;
};

// Swizzled LDS address of 16-byte chunk j (0..3) of tile row `row` (64 bytes per row).
__device__ inline int lds_addr(int row, int j) { return row * KBLK + ((j ^ ((row >> 1) & 3)) << 4); }

__device__ inline float vox_term(uint32_t P, const float *EA, const float *EB, const float2 *LQ)
{
    const uint32_t n0 = P & 0xffffu, n1 = P >> 16;
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

template <int W, bool EMIT>
__global__ __launch_bounds__(SW_THREADS, 2) void k_sweep2(Sweep2Args a)
{
    constexpr int C = W + 1;
    constexpr int TV = TILE_ROWS / W;    // variables per tile side
    constexpr int NP = (W == 1) ? 4 : 1; // pairs held per lane per 16x16 block
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char *stage = smem;                  // [2 buffers][A 8 KB | B 8 KB]
    float *EA = reinterpret_cast<float *>(smem + 2 * STAGE_BYTES);
    float *EB = EA + (a.N0 + 1);
    float2 *LQ = reinterpret_cast<float2 *>(EB + (a.N1 + 1) + ((a.N0 + a.N1) & 1));

    // XCD-aware tile order: blocks b, b+8, b+16 ... run on one XCD; give each XCD a contiguous
    // range of the tile enumeration so neighbouring tiles share operand panels in its L2.
    const int64_t b = blockIdx.x;
    const int64_t tile = (b & 7) * a.per_xcd + (b >> 3);
    if (tile >= a.n_tiles) return;
    const int r = (int)(tile / a.tiles_per_r);
    int bi, bj;
    tri_index(tile % a.tiles_per_r, bi, bj);

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int q = lane >> 4, c16 = lane & 15;

    for (int i = t; i <= a.N0; i += SW_THREADS) EA[i] = a.EA[i];
    for (int i = t; i <= a.N1; i += SW_THREADS) EB[i] = a.EB[i];
    for (int i = t; i <= a.N; i += SW_THREADS) LQ[i] = a.LQ[i];

    // ---------------------------------------------------------------- K loop
    const int64_t rowA0 = (int64_t)bi * TILE_ROWS, rowB0 = (int64_t)bj * TILE_ROWS;
    const int8_t *base = a.onehot + (int64_t)r * a.KB * a.rows_pad * KBLK;
    const int n1blk = a.KB - a.KB0;      // class-1 K blocks, accumulated first
    auto kb_of = [&](int s) { return s < n1blk ? a.KB0 + s : s - n1blk; };
    // this thread's two chunks of A and two of B
    const int id0 = t, id1 = t + SW_THREADS;
    const int ra0 = id0 >> 2, ja0 = id0 & 3, ra1 = id1 >> 2, ja1 = id1 & 3;
    uint4 g[4];
    auto gload = [&](int kb) {
        const int8_t *blk = base + (int64_t)kb * a.rows_pad * KBLK;
        g[0] = *reinterpret_cast<const uint4 *>(blk + (rowA0 + ra0) * KBLK + ja0 * 16);
        g[1] = *reinterpret_cast<const uint4 *>(blk + (rowA0 + ra1) * KBLK + ja1 * 16);
        g[2] = *reinterpret_cast<const uint4 *>(blk + (rowB0 + ra0) * KBLK + ja0 * 16);
        g[3] = *reinterpret_cast<const uint4 *>(blk + (rowB0 + ra1) * KBLK + ja1 * 16);
    };
    auto sstore = [&](int buf) {
        char *A = stage + buf * STAGE_BYTES, *B = A + TILE_ROWS * KBLK;
        *reinterpret_cast<uint4 *>(A + lds_addr(ra0, ja0)) = g[0];
        *reinterpret_cast<uint4 *>(A + lds_addr(ra1, ja1)) = g[1];
        *reinterpret_cast<uint4 *>(B + lds_addr(ra0, ja0)) = g[2];
        *reinterpret_cast<uint4 *>(B + lds_addr(ra1, ja1)) = g[3];
    };

    v4i acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = v4i{0, 0, 0, 0};

    gload(kb_of(0));
    sstore(0);
    __syncthreads();
    for (int s = 0; s < a.KB; ++s) {
        if (s + 1 < a.KB) gload(kb_of(s + 1));
        const char *A = stage + (s & 1) * STAGE_BYTES, *B = A + TILE_ROWS * KBLK;
        v4i fa[4], fb[4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
            fa[m] = *reinterpret_cast<const v4i *>(A + lds_addr(wr * 64 + m * 16 + c16, q));
#pragma unroll
        for (int n = 0; n < 4; ++n)
            fb[n] = *reinterpret_cast<const v4i *>(B + lds_addr(wc * 64 + n * 16 + c16, q));
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n)
                acc[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[m], fb[n], acc[m][n], 0, 0, 0);
        if (s == n1blk - 1) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) acc[m][n] = acc[m][n] << 16;
        }
        if (s + 1 < a.KB) sstore((s + 1) & 1);
        __syncthreads();
    }

    // ---------------------------------------------------------------- epilogue
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

    uint32_t Mr[4][NP][C], Mc[4][C];
    float Fr[4][NP], Fc[4];
    float thrR[4][NP], thrC[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int s = 0; s < NP; ++s) {
            int64_t v = row_var(m, s);
#pragma unroll
            for (int c = 0; c < C; ++c) Mr[m][s][c] = margr[v * C + c];
            Fr[m][s] = F1r[v];
            float gk = key_f32(a.G32[v]);
            thrR[m][s] = gk - rescore_window(a.w_abs, gk);
        }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        int64_t v = col_var(n);
#pragma unroll
        for (int c = 0; c < C; ++c) Mc[n][c] = margr[v * C + c];
        Fc[n] = F1r[v];
        float gk = key_f32(a.G32[v]);
        thrC[n] = gk - rescore_window(a.w_abs, gk);
    }

    // Full per-class table of the lane's pair(s) in block (m, n): packed counts tab[a][b].
    auto pair_table = [&](int m, int n, int s, uint32_t (&tab)[C][C]) {
        const v4i &ac = acc[m][n];
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
            for (int y = 0; y < C; ++y) F += vox_term(tab[x][y], EA, EB, LQ);
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
    // W = 2 keeps the lane's 32 IG values for the append pass; W = 1 (64 pairs per lane)
    // recomputes them instead.
    constexpr int KEEP = (W == 2) ? 16 : 1;
    float keepR[KEEP], keepC[KEEP];

    const bool emit = EMIT && r == a.disc_sel;
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
                const float igR = valid ? Fc[n] - F2 : -INFINITY;   // gain of rv given cv
                const float igC = valid ? Fr[m][s] - F2 : -INFINITY; // gain of cv given rv
                if constexpr (W == 2) { keepR[m * 4 + n] = igR; keepC[m * 4 + n] = igC; }
                rmax[m][s] = fmaxf(rmax[m][s], igR);
                cmax[n] = fmaxf(cmax[n], igC);
                hot |= (igR >= thrR[m][s]) | (igC >= thrC[n]);
                if (emit && valid) {
                    int32_t *o = a.counts_out + ((int64_t)rv * a.p + cv) * 2 * C * C;
#pragma unroll
                    for (int x = 0; x < C; ++x)
#pragma unroll
                        for (int y = 0; y < C; ++y) {
                            o[x * C + y] = (int32_t)(tab[x][y] & 0xffffu);
                            o[C * C + x * C + y] = (int32_t)(tab[x][y] >> 16);
                        }
                }
            }

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
                float top = fmaxf(g, rmax[m][s]);
                thrR[m][s] = top - rescore_window(a.w_abs, top);
            }
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            float g = key_f32(a.G32[col_var(n)]);
            float top = fmaxf(g, cmax[n]);
            thrC[n] = top - rescore_window(a.w_abs, top);
        }
        if constexpr (W != 2) {
            // recompute from the accumulators; the empty asm stops the compiler from keeping
            // the first pass's values alive instead
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) asm volatile("" : "+v"(acc[m][n]) : : "memory");
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n)
#pragma unroll
                for (int s = 0; s < NP; ++s) {
                    const int64_t rv = row_var(m, s), cv = col_var(n);
                    const bool valid = rv < cv && cv < a.p;
                    float igR, igC;
                    if constexpr (W == 2) {
                        igR = keepR[m * 4 + n];
                        igC = keepC[m * 4 + n];
                    } else {
                        uint32_t tab[C][C];
                        pair_table(m, n, s, tab);
                        const float F2 = pair_F2(tab);
                        igR = Fc[n] - F2;
                        igC = Fr[m][s] - F2;
                    }
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

    // publish the maxima: one lane per variable
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
}

template <int W>
static hipError_t sweep_launch(const Problem &P, int32_t *counts_out, int disc_sel)
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
    a.tiles_per_r = (int64_t)a.nbv * (a.nbv + 1) / 2;
    a.n_tiles = a.tiles_per_r * L.R;
    a.per_xcd = (a.n_tiles + 7) / 8;
    a.G32 = P.at<uint32_t>(L.G32);
    a.cand = P.at<Cand>(L.cand);
    a.cap = L.cap;
    a.st = P.at<Status>(L.status);
    a.ovf = P.at<uint32_t>(L.ovf);
    a.w_abs = (float)(2.0 * P.err_bound);
    a.counts_out = counts_out;
    a.disc_sel = disc_sel;
    size_t lds = 2 * STAGE_BYTES + sizeof(float) * (size_t)(P.N0 + 1 + P.N1 + 1 + 1) + sizeof(float2) * (L.N + 1) + 16;
    auto kern = counts_out ? k_sweep2<W, true> : k_sweep2<W, false>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int64_t grid = a.per_xcd * 8;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(SW_THREADS), lds, P.stream, a);
    return hipGetLastError();
}

hipError_t launch_sweep2(const Problem &P, int32_t *counts_out, int disc_sel)
{
    switch (P.L.W) {
    case 1: return sweep_launch<1>(P, counts_out, disc_sel);
    case 2: return sweep_launch<2>(P, counts_out, disc_sel);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mdfs
