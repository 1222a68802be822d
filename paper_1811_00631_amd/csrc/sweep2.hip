// sweep2.hip -- the k = 2 tuple sweep on the gfx950 matrix cores.
//
// Counting (the voxel counters N^d of section "Algorithm and implementation", named there the
// most time-consuming part): with objects sorted by class and each variable one-hot encoded on
// its first W = C-1 bins, the per-class pair tables are the Gram products X_d^T X_d.  A tile of
// 128 x 128 one-hot rows is accumulated on the matrix cores in one of two encodings:
//   fp4:  E2M1 nibbles holding 2.0 (0b0100), V_MFMA_F32_16X16X128_F8F6F4, float32
//         accumulators; every product is 4.  Class-1 objects are accumulated first, the
//         accumulator is scaled by 4096, then class-0 objects are added: n1 * 2^14 + 4 n0 <
//         2^26, a multiple of 4, is an exact float32 value while each class has < 4096
//         objects.  Half the operand bytes and twice the rate of int8.  The epilogue converts
//         it to the packed integer (4 n1) << 16 | 4 n0, whose halves are byte offsets into
//         the float tables.
//   int8: bytes holding 1, V_MFMA_I32_16X16X64_I8, int32 accumulators shifted left by 16
//         between the classes: n1 << 16 | n0 for classes < 32768 objects.
// The dropped last bin of each variable is rebuilt exactly from the per-class marginals
// (packed subtraction never borrows because every reconstructed count is >= 0).
//
// Epilogue (the pseudocounted entropy of the class-probability equation and IG of equation
// IGmax): per pair F2 = sum_v n_v h(p_v) from float32 lookup tables indexed by integer counts,
// IG(i|j) = F1(j) - F2 and IG(j|i) = F1(i) - F2.  This float32 value is a screen with a proven
// bound E on its error: each variable's float32 maximum is kept with an atomic max on an
// order-preserving key, and every (pair, discretisation) that may be within 2E + tau of the
// final maximum is appended to a candidate buffer; the finalize pass re-scores candidates in
// binary64 from exact recounts.
#include "mdfs_internal.h"

#include <algorithm>

namespace mdfs {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
template <bool F4> struct AccOf { typedef v4i type; };
template <> struct AccOf<true> { typedef v4f type; };

// Template argument ENC of the sweep: 0 = int8 encoding (entropy tables placed at run time
// after the operand stages); T = 1024, 2048, 4096 = fp4 encoding with LDS entropy tables of
// capacity T per class at fixed addresses, so each lookup is one ds_read with an immediate
// offset:  EA [0, 4T)  EB [4T, 8T)  (L, Q) pairs [8T, 24T - 8)  (bytes; the pairs hold the
// 2T - 1 entries n = 0 .. 2T - 2), operand stages from 24T.  EA and EB stay separate: a
// gather at an 8-byte stride would use half of the LDS banks.
__host__ __device__ constexpr int stage_base(int ENC) { return ENC ? 24 * ENC : 0; }

// Waves per workgroup: 8 for three classes (2 x 4 wave grid, 64 x 32 outputs per wave; at most
// 128 VGPRs, so 4 waves per SIMD), else 4 (2 x 2 grid, 64 x 64 outputs per wave, 2 per SIMD; the
// two- and five-class epilogues hold more per lane).  The tile and its LDS are the same.
// Three classes may also run 4 waves (2 x 2 grid, 64 x 64 outputs per wave), a tuning choice.
__host__ __device__ constexpr int sw_waves(int W) { return W == 2 ? 8 : 4; }
constexpr int SB_DEFAULT = 8;            // a super-tile is sb x sb tiles (sb 2 .. 16, a tuning choice)
constexpr int XCDS = 8;                  // workgroup b runs on XCD b % 8
constexpr int WG_PER_XCD = 64;           // resident workgroups per XCD (2 per CU: LDS)
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
    int sb;                  // super-tile side in tiles
    int nsb;                 // super-blocks of sb variable blocks
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
    int gated;               // run only if Status::collect_go is set (the collect pass)
    int r_base;              // first discretisation of this launch
    int snext_off;           // LDS byte offset of the work-item broadcast slot
    uint32_t *ptab;          // pair mode: packed (W x W) counts [r - r_base][p_pad][p_pad][W*W]
    int pair_x4;             // pair mode: store (4 n1) << 16 | 4 n0 (the matrix-core triple
                             // sweeps' form) instead of n1 << 16 | n0
    float *F2out;            // pair mode: float32 F of each pair table [r - r_base][p_pad][p_pad]
    const uint32_t *cancel;  // caller's cancel word (nullable)
};

// What one launch of the pair sweep produces.
enum SweepMode { SWEEP_MAX = 0, SWEEP_PAIRS = 2 };

// Several problems in one persistent launch (maximum pass): their super-tiles are concatenated
// (pref = prefix of each problem's super-tile count) and drawn from one set of queues.  Passed
// by value in the kernel arguments, so a batch needs no host-to-device copy.
struct Sweep2Batch {
    Sweep2Args p[MAX_BATCH];
    int64_t pref[MAX_BATCH + 1];
    int nb;
    Status *queue;           // work counters of the batch
};

// Swizzled LDS address of 16-byte chunk j (0..3) of tile row `row` (64 bytes per row).
__device__ inline int lds_addr(int row, int j) { return row * KBLK + ((j ^ ((row >> 1) & 3)) << 4); }

typedef float vf2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) const float lds_f32;
typedef __attribute__((address_space(3))) const vf2 lds_f32x2;

// One voxel's n h(p) from the float32 tables, int8 packing n1 << 16 | n0.
__device__ inline float vox_term(uint32_t P, const float *EA, const float *EB, const float2 *LQ)
{
    const uint32_t n0 = P & 0xffffu, n1 = P >> 16;
    const float2 lq = LQ[n0 + n1];
    return lq.x - lq.y * (EA[n0] + EB[n1]);
}



// Sum of n h(p) over NV voxels (packed counts).  ENC != 0: fp4 packing (4 n1) << 16 | 4 n0,
// whose halves are the byte offsets of EA[n0], EB[n1] and twice their sum that of the (L, Q)
// pair of n in the fixed LDS layout; all table reads first, then the arithmetic, so the
// reads overlap.
// A packed count of 0 contributes exactly 0 (L[0] = Q[0] = 0).
template <int ENC, int NV>
__device__ inline float sum_vox(const uint32_t (&P)[NV], const char *smem, const float *EA, const float *EB,
                                const float2 *LQ)
{
    if constexpr (ENC != 0) {
        constexpr int T = ENC;
        float ea[NV], eb[NV];
        vf2 lq[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const uint32_t a0 = P[v] & 0xffffu, a1 = P[v] >> 16;
            // The sweep kernels declare no static LDS (group segment size 0), so the dynamic
            // array starts at LDS address 0 and these byte offsets are LDS addresses: each read
            // takes its offset register as is, the table base going into the instruction's
            // immediate offset (through `smem` every address would carry the base as one more
            // add: 4 instead of 3 VALU instructions per voxel).
            ea[v] = *reinterpret_cast<const lds_f32 *>((uintptr_t)a0);
            eb[v] = *reinterpret_cast<const lds_f32 *>((uintptr_t)(4 * T + a1));
            lq[v] = *reinterpret_cast<const lds_f32x2 *>((uintptr_t)(8 * T + 2 * (a0 + a1)));
        }
        // summed in voxel order, starting from the first term
        float F = lq[0].x - lq[0].y * (ea[0] + eb[0]);
#pragma unroll
        for (int v = 1; v < NV; ++v) F += lq[v].x - lq[v].y * (ea[v] + eb[v]);
        return F;
    } else {
        float F = vox_term(P[0], EA, EB, LQ);
#pragma unroll
        for (int v = 1; v < NV; ++v) F += vox_term(P[v], EA, EB, LQ);
        return F;
    }
}

__device__ inline uint32_t dpp_xor1(uint32_t x) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false); }
__device__ inline uint32_t dpp_xor2(uint32_t x) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false); }
__device__ inline float dpp_xor1f(float x) { return __builtin_bit_cast(float, dpp_xor1(__builtin_bit_cast(uint32_t, x))); }
__device__ inline float dpp_xor2f(float x) { return __builtin_bit_cast(float, dpp_xor2(__builtin_bit_cast(uint32_t, x))); }

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

template <int W, int MODE, int ENC, bool BATCH, bool EXPORT = false, int NWV = sw_waves(W)>
__device__ __forceinline__ void sweep2_run(Sweep2Args a, const Sweep2Batch *bt)
{
    constexpr bool F4 = ENC != 0;
    constexpr int T = ENC;
    constexpr int C = W + 1;
    typedef typename AccOf<F4>::type Acc;
    constexpr int TV = TILE_ROWS / W;    // variables per tile side
    constexpr int NP = (W == 1) ? 4 : 1; // pairs held per lane per 16x16 block
    constexpr int NWAVE = NWV, NT = NWAVE * 64;
    constexpr int NN = 16 / NWAVE;       // 16 x 16 column blocks per wave (row blocks: 4)
    constexpr int LPW = 16 / NWAVE;      // 1 KB operand fetches per wave and K block
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char *stage = smem + stage_base(ENC);   // [NSTAGE buffers][A 8 KB | B 8 KB]
    // int8: tables after the stages, at run-time offsets (per problem)
    float *EA = nullptr, *EB = nullptr;
    float2 *LQ = nullptr;
    int64_t *s_next_p = reinterpret_cast<int64_t *>(smem + a.snext_off);

    if (a.gated && a.st->collect_go == 0) return;   // workgroup-uniform
    const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wr = wave / (NWAVE / 2), wc = wave % (NWAVE / 2);
    const int q = lane >> 4, c16 = lane & 15;

    // the problem's entropy tables into LDS
    auto load_tables = [&]() {
        EA = reinterpret_cast<float *>(smem + NSTAGE * STAGE_BYTES);
        EB = EA + (a.N0 + 1);
        LQ = reinterpret_cast<float2 *>(EB + (a.N1 + 1) + ((a.N0 + a.N1) & 1));
        if constexpr (F4) {
            float *tf = reinterpret_cast<float *>(smem);
            for (int i = t; i <= a.N0; i += NT) tf[i] = a.EA[i];
            for (int i = t; i <= a.N1; i += NT) tf[T + i] = a.EB[i];
            float2 *lq = reinterpret_cast<float2 *>(smem + 8 * T);
            for (int i = t; i <= a.N; i += NT) lq[i] = a.LQ[i];
        } else {
            for (int i = t; i <= a.N0; i += NT) EA[i] = a.EA[i];
            for (int i = t; i <= a.N1; i += NT) EB[i] = a.EB[i];
            for (int i = t; i <= a.N; i += NT) LQ[i] = a.LQ[i];
        }
    };
    int cur = 0;   // batch: the problem whose arguments and tables are loaded
    load_tables();

    // Persistent, XCD-aware schedule.  The super-tiles sup = x, x+8, x+16 ... form queue x; the
    // workgroups resident on XCD x take its tiles (super-tile by super-tile, slot by slot) from
    // one atomic counter, so at any time they work on the same SB x SB block of tiles and share
    // its SB row panels and SB column panels in the XCD's L2.  A workgroup whose queue is
    // drained moves on to the next queues, so every tile is taken whatever the grid size and
    // wherever its workgroups run.
    const int xcd = (int)(__builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & 7);  // HW_REG_XCC_ID
    int my_q = xcd, q_seen = 0;   // thread 0's position in the queue walk
    uint32_t taken = 0;           // work items taken by this workgroup (cancel polling)
    for (;;) {
    __syncthreads();   // everyone has read the previous s_next
    if (t == 0) {
        int64_t it = -1;
        const int64_t n_super = BATCH ? bt->pref[bt->nb] : a.n_super;
        Status *qst = BATCH ? bt->queue : a.st;
        if (cancel_poll(a.cancel, taken++, a.st)) {
            if constexpr (BATCH)
                for (int b_ = 0; b_ < bt->nb; ++b_) atomicOr(&bt->p[b_].st->cancelled, 1u);
            q_seen = XCDS;   // take no more work
        }
        while (q_seen < XCDS) {
            const int64_t nq = ((n_super - my_q + XCDS - 1) / XCDS) * (a.sb * a.sb);
            it = (int64_t)atomicAdd(&qst->next_tile[my_q], 1u);
            if (it < nq) break;
            it = -1;
            my_q = (my_q + 1) & (XCDS - 1);
            ++q_seen;
        }
        s_next_p[0] = it;
        s_next_p[1] = my_q;
    }
    __syncthreads();
    const int64_t item = s_next_p[0];
    if (item < 0) break;
    int64_t sup = s_next_p[1] + XCDS * (item / (a.sb * a.sb));
    if constexpr (BATCH) {
        // the problem owning this super-tile; arguments and tables follow it (workgroup-uniform;
        // every wave finished the previous tile before the barriers of the fetch)
        int lo = 0, hi = bt->nb - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (bt->pref[mid] <= sup) lo = mid;
            else hi = mid - 1;
        }
        if (lo != cur) {
            cur = lo;
            a = bt->p[lo];
            load_tables();
            __syncthreads();
        }
        sup -= bt->pref[lo];
    }
    const int slot = (int)(item % (a.sb * a.sb));
    const int r = a.r_base + (int)(sup / a.super_per_r);
    int SI, SJ;
    tri_index(sup % a.super_per_r, SI, SJ);
    const int bi = SI * a.sb + slot / a.sb, bj = SJ * a.sb + slot % a.sb;
    if (bi > bj || bj >= a.nbv) continue;   // workgroup-uniform

    // ---------------------------------------------------------------- K loop
    // operand panels: TILE_ROWS one-hot rows x all K blocks, contiguous (panel-major layout)
    const int64_t nrb = a.rows_pad / TILE_ROWS;
    const int8_t *panA = a.onehot + ((int64_t)r * nrb + bi) * a.KB * TILE_ROWS * KBLK;
    const int8_t *panB = a.onehot + ((int64_t)r * nrb + bj) * a.KB * TILE_ROWS * KBLK;
    const int n1blk = a.KB - a.KB0;      // class-1 K blocks, accumulated first
    constexpr int kstride = TILE_ROWS * KBLK;

    Acc acc[4][NN];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NN; ++n) acc[m][n] = Acc{0, 0, 0, 0};

    // K blocks in processing order: class 1 first, then class 0
    auto kblock = [&](int s_) { return s_ < n1blk ? a.KB0 + s_ : s_ - n1blk; };
    auto stage_at = [&](int s_) { return stage + (s_ % NSTAGE) * STAGE_BYTES; };
    // Operands go from global memory straight into LDS (global_load_lds_dwordx4): one
    // instruction fills 1 KB = 16 rows, lane i's 16 bytes landing at offset 16 i.  A stage is
    // 16 such blocks (A rows 0..127, then B rows 0..127); wave w fills blocks LPW w ..
    // LPW w + LPW - 1, so the first half of the waves fetch the A panel and the second half the
    // B panel.  The swizzle of the stage layout is applied on the global side: lane i fetches
    // the chunk that belongs at its slot.
    const int8_t *pan = wave < NWAVE / 2 ? panA : panB;
    int goff[LPW];
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
        const int row = 16 * ((wave * LPW + i) & 7) + (lane >> 2);
        const int j = (lane & 3) ^ ((row >> 1) & 3);
        goff[i] = row * KBLK + j * 16;
    }
    auto issue = [&](int s_) {
        const int8_t *src = pan + (int64_t)kblock(s_) * kstride;
        char *dst = stage_at(s_) + wave * LPW * 1024;
#pragma unroll
        for (int i = 0; i < LPW; ++i)
            __builtin_amdgcn_global_load_lds((const void *)(src + goff[i]),
                                             (__attribute__((address_space(3))) void *)(dst + i * 1024), 16, 0, 0);
    };
    const int fa_off0 = lds_addr(wr * 64 + c16, q), fb_off0 = lds_addr(wc * 16 * NN + c16, q);
    auto frags = [&](int s_, v4i (&xa)[4], v4i (&xb)[NN]) {
        const char *A = stage_at(s_), *B = A + TILE_ROWS * KBLK;
#pragma unroll
        for (int m = 0; m < 4; ++m) xa[m] = *reinterpret_cast<const v4i *>(A + fa_off0 + m * 16 * KBLK);
#pragma unroll
        for (int n = 0; n < NN; ++n) xb[n] = *reinterpret_cast<const v4i *>(B + fb_off0 + n * 16 * KBLK);
    };
    // Software pipeline over a ring of NSTAGE = 3 LDS stages; blocks are fetched two steps ahead
    // and their fragments read one step ahead.  Step s: the wave waits until its fragment reads
    // of block s (issued during step s-1) and its fetches of block s+1 have completed (loads
    // complete in issue order, so the LPW fetches of block s+2 may still be outstanding), passes
    // a barrier (block s+1 is complete in LDS, and every wave holds the fragments of block s, so
    // its stage is free), issues the fragment reads of block s+1 and the fetch of block s+3 into
    // the stage of block s, then the MFMAs of block s: the reads for the next step are in flight
    // while this step's products go out.
    auto mma = [&](int s_, const v4i (&xa)[4], const v4i (&xb)[NN]) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < NN; ++n) {
                if constexpr (F4) {
                    // A/B: 16 rows x 128 objects, lane l holds row l % 16 and 32 nibbles of
                    // one quarter of the objects; cbsz = blgp = 4 selects E2M1 for both operands
                    const v8i a8{xa[m][0], xa[m][1], xa[m][2], xa[m][3], 0, 0, 0, 0};
                    const v8i b8{xb[n][0], xb[n][1], xb[n][2], xb[n][3], 0, 0, 0, 0};
                    acc[m][n] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, acc[m][n], 4, 4, 0, 0, 0, 0);
                } else {
                    acc[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xa[m], xb[n], acc[m][n], 0, 0, 0);
                }
            }
        if (s_ == n1blk - 1) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < NN; ++n) {
                    if constexpr (F4) acc[m][n] = acc[m][n] * 4096.0f;
                    else acc[m][n] = acc[m][n] << 16;
                }
        }
    };
    // the plain barrier: a fenced one would also drain the fetches still in flight
    // The LDS wait comes first and on every path, so that the compiler sees this step's
    // fragments complete wherever the MFMAs are reached and adds no wait of its own there (one
    // after the next step's fragment reads would serialise them with the MFMAs).
    auto step = [&](int s_, const v4i (&ca)[4], const v4i (&cb)[NN], v4i (&na)[4], v4i (&nb)[NN]) {
        __builtin_amdgcn_s_waitcnt(0xC07F);                                   // lgkmcnt(0)
        if (s_ + 1 < a.KB) {
            if (s_ + 2 < a.KB) __builtin_amdgcn_s_waitcnt(0x0F70 | LPW);   // vmcnt(LPW)
            else __builtin_amdgcn_s_waitcnt(0x0F70);                       // vmcnt(0)
            __builtin_amdgcn_s_barrier();
            frags(s_ + 1, na, nb);
            if (s_ + 3 < a.KB) issue(s_ + 3);
        }
        mma(s_, ca, cb);
    };
    v4i fa0[4], fb0[NN], fa1[4], fb1[NN];
    issue(0);
    if (a.KB > 1) issue(1);
    if (a.KB > 1) __builtin_amdgcn_s_waitcnt(0x0F70 | LPW);
    else __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_s_barrier();
    frags(0, fa0, fb0);
    if (a.KB > 2) issue(2);
    int s = 0;
    for (; s + 1 < a.KB; s += 2) {
        step(s, fa0, fb0, fa1, fb1);
        step(s + 1, fa1, fb1, fa0, fb0);
    }
    if (s < a.KB) step(s, fa0, fb0, fa1, fb1);

    // ---------------------------------------------------------------- epilogue
    // W >= 2: the first pass keeps each pair's float32 F for the append pass in the stage that
    // follows the last block's, 4 NN pairs x 64 lanes = 16 KB per workgroup.  That stage held block
    // KB - 3 (or nothing): every wave read its fragments and every fetch landed before the last
    // barrier of the K loop, and the next tile's first fetch follows the barriers at the top of
    // the tile loop.
    float *f2buf = reinterpret_cast<float *>(stage_at(a.KB));
    auto put_cand = [&](uint32_t at, int64_t v, int64_t partner, float ig) {
        if (at < a.cap) a.cand[at] = Cand{(int32_t)v, r, (uint32_t)partner, ig};
        else { atomicOr(&a.ovf[v], 1u); atomicOr(&a.st->overflow, 1u); }
    };
    // packed integer counts: int8 n1 << 16 | n0; fp4 (4 n1) << 16 | 4 n0 from the exact
    // float32 value u = n1 * 2^14 + 4 n0 as u + (u >> 14) * (2^18 - 2^14)
    v4i cnt[4][NN];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NN; ++n) {
            if constexpr (F4) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t u = (uint32_t)acc[m][n][e];
                    cnt[m][n][e] = (int)(__umul24(u >> 14, 245760u) + u);
                }
            } else {
                cnt[m][n] = acc[m][n];
            }
        }
    // Count export (EXPORT: the maximum pass with the same table capacity, encoding and LDS layout,
    // plus this store): for the selected discretisation every lane stores the W x W directly
    // counted cells it holds into their places in the caller's [p][p][2][C][C] tables;
    // launch_complete_pairs then fills in the cells of each variable's dropped last bin.
    if (EXPORT && r == a.disc_sel) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < NN; ++n)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    // lane (q, c16) holds rows 4q .. 4q + 3 of column c16 of block (m, n)
                    const int row = wr * 64 + m * 16 + 4 * q + e, col = wc * 16 * NN + n * 16 + c16;
                    const int64_t rv = (int64_t)bi * TV + row / W, cv = (int64_t)bj * TV + col / W;
                    if (rv < cv && cv < a.p) {
                        const uint32_t v = F4 ? (uint32_t)cnt[m][n][e] >> 2 : (uint32_t)cnt[m][n][e];
                        int32_t *o = a.counts_out + (rv * a.p + cv) * 2 * C * C + (row % W) * C + col % W;
                        o[0] = (int32_t)(v & 0xffffu);
                        o[C * C] = (int32_t)(v >> 16);
                    }
                }
    }

    if constexpr (W == 4) {
        static_assert(NN == 4, "the five-class epilogue assumes 4 x 4 blocks per wave");
        // Five classes: block (m, n) holds 4 x 4 pairs.  The lane holds the four row bins of row
        // variable q and column bin b = c16 % 4 of column variable c16 / 4, so a pair's 4 x 4
        // direct counts lie on one lane quad.  Each lane evaluates its column's voxels (4 direct
        // and the rebuilt last-row voxel (4, b)), the rebuilt last-column voxel (b, 4) from the
        // quad's row sums, lane b = 0 also the corner (4, 4); F of the pair is the quad sum,
        // identical on the four lanes.
        const int b = c16 & 3;
        const int64_t I0 = (int64_t)bi * TV, J0 = (int64_t)bj * TV;
        auto rv_of = [&](int m) -> int64_t { return I0 + wr * 16 + m * 4 + q; };
        auto cv_of = [&](int n) -> int64_t { return J0 + wc * 16 + n * 4 + (c16 >> 2); };
        const uint32_t *margr = a.marg + (int64_t)r * a.p_pad * C;
        const float *F1r = a.F1 + (int64_t)r * a.p_pad;
        auto repack = [](uint32_t x) -> uint32_t { return F4 ? x << 2 : x; };
        uint32_t Mrb[4], Mrs[4], Mcb[4], Mc4[4];
        float Fr[4], Fc[4], thrR[4], thrC[4], gR[4], gC[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int64_t v = rv_of(m);
            uint32_t sum4 = 0;
#pragma unroll
            for (int x = 0; x < 4; ++x) sum4 += repack(margr[v * C + x]);
            Mrs[m] = sum4;
            Mrb[m] = repack(margr[v * C + b]);
            Fr[m] = F1r[v];
            const float gk = key_f32(a.G32[v]);
            gR[m] = gk;
            thrR[m] = gk - rescore_window(a.w_abs, gk);
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const int64_t v = cv_of(n);
            Mcb[n] = repack(margr[v * C + b]);
            Mc4[n] = repack(margr[v * C + 4]);
            Fc[n] = F1r[v];
            const float gk = key_f32(a.G32[v]);
            gC[n] = gk;
            thrC[n] = gk - rescore_window(a.w_abs, gk);
        }
        // the lane's voxels of pair (m, n) and the quad sum F; vx[0..3] direct (x, b),
        // vx[4] = (4, b), vx[5] = (b, 4), vx[6] = corner on lane b = 0 (else 0)
        auto quad_pair = [&](int m, int n, uint32_t (&vx)[7]) -> float {
            const v4i &ac = cnt[m][n];
            uint32_t S[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                vx[x] = (uint32_t)ac[x];
                const uint32_t t_ = vx[x] + dpp_xor1(vx[x]);
                S[x] = t_ + dpp_xor2(t_);
            }
            vx[4] = Mcb[n] - (vx[0] + vx[1] + vx[2] + vx[3]);
            const uint32_t Sb = b == 0 ? S[0] : (b == 1 ? S[1] : (b == 2 ? S[2] : S[3]));
            vx[5] = Mrb[m] - Sb;
            vx[6] = b == 0 ? Mc4[n] - (Mrs[m] - (S[0] + S[1] + S[2] + S[3])) : 0u;
            float f = sum_vox<ENC, 7>(vx, smem, EA, EB, LQ);
            f += dpp_xor1f(f);
            return f + dpp_xor2f(f);
        };
        auto dec = [](uint32_t P_) -> uint32_t { return F4 ? P_ >> 2 : P_; };   // -> n1 << 16 | n0
        float rmax[4], cmax[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) rmax[m] = cmax[m] = -INFINITY;
        bool hot = false;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                uint32_t vx[7];
                const float F2 = quad_pair(m, n, vx);
                if constexpr (MODE != SWEEP_PAIRS) f2buf[(wave * 4 * NN + m * NN + n) * 64 + lane] = F2;
                const int64_t rv = rv_of(m), cv = cv_of(n);
                const bool valid = rv < cv && cv < a.p;
                if constexpr (MODE == SWEEP_PAIRS) {
                    if (valid) {
                        const int64_t pc = (int64_t)(r - a.r_base) * a.p_pad * a.p_pad + rv * a.p_pad + cv;
                        uint32_t *o = a.ptab + pc * (W * W);
#pragma unroll
                        for (int x = 0; x < 4; ++x) o[x * W + b] = a.pair_x4 ? dec(vx[x]) << 2 : dec(vx[x]);
                        if (b == 0) a.F2out[pc] = F2;
                    }
                    continue;
                }
                const float igR = valid ? Fc[n] - F2 : -INFINITY;
                const float igC = valid ? Fr[m] - F2 : -INFINITY;
                rmax[m] = fmaxf(rmax[m], igR);
                cmax[n] = fmaxf(cmax[n], igC);
                hot |= (igR >= thrR[m]) | (igC >= thrC[n]);
            }
        if constexpr (MODE == SWEEP_PAIRS) continue;
        // wave maxima: a pair's value is replicated on its quad; row variables differ in q,
        // column variables in c16 / 4
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            float x = rmax[m];
            x = fmaxf(x, __shfl_xor(x, 4));
            rmax[m] = fmaxf(x, __shfl_xor(x, 8));
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            float x = cmax[n];
            x = fmaxf(x, __shfl_xor(x, 16));
            cmax[n] = fmaxf(x, __shfl_xor(x, 32));
        }
        if (__any(hot)) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const float g = key_f32(a.G32[rv_of(m)]);
                const float top = a.collect ? g : fmaxf(g, rmax[m]);
                thrR[m] = top - rescore_window(a.w_abs, top);
            }
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const float g = key_f32(a.G32[cv_of(n)]);
                const float top = a.collect ? g : fmaxf(g, cmax[n]);
                thrC[n] = top - rescore_window(a.w_abs, top);
            }
            // which pairs append (bit m * 4 + n), then one slot reservation for the wave
            uint32_t selR = 0, selC = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const float F2 = f2buf[(wave * 4 * NN + m * NN + n) * 64 + lane];   // the first pass's
                    const int64_t rv = rv_of(m), cv = cv_of(n);
                    const bool valid = b == 0 && rv < cv && cv < a.p;   // one lane per pair
                    const float igR = Fc[n] - F2, igC = Fr[m] - F2;
                    if (valid && igR >= thrR[m]) selR |= 1u << (m * 4 + n);
                    if (valid && igC >= thrC[n]) selC |= 1u << (m * 4 + n);
                }
            uint32_t at = reserve_slots(&a.st->n_cand, __popc(selR) + __popc(selC), lane);
            if (selR | selC) {
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < 4; ++n) {
                        const uint32_t bit = 1u << (m * 4 + n);
                        if ((selR | selC) & bit) {
                            const float F2 = f2buf[(wave * 4 * NN + m * NN + n) * 64 + lane];
                            if (selR & bit) put_cand(at++, rv_of(m), cv_of(n), Fc[n] - F2);
                            if (selC & bit) put_cand(at++, cv_of(n), rv_of(m), Fr[m] - F2);
                        }
                    }
            }
        }
        if (a.collect) continue;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (c16 == 0 && rmax[m] > gR[m]) atomicMax(&a.G32[rv_of(m)], f32_key(rmax[m]));
#pragma unroll
        for (int n = 0; n < 4; ++n)
            if (q == 0 && b == 0 && cmax[n] > gC[n]) atomicMax(&a.G32[cv_of(n)], f32_key(cmax[n]));
        continue;
    } else {
    // Lane geometry of the 16x16 output block (m, n): lane holds rows 4q..4q+3 of column c16.
    // Row/column index = variable * W + bin within the block.
    const int64_t I0 = (int64_t)bi * TV, J0 = (int64_t)bj * TV;
    const int odd = lane & 1;
    auto row_var = [&](int m, int s) -> int64_t {
        if (W == 1) return I0 + wr * 64 + m * 16 + 4 * q + s;
        return I0 + wr * 32 + m * 8 + 2 * q + odd;
    };
    auto col_var = [&](int n) -> int64_t {
        if (W == 1) return J0 + wc * 16 * NN + n * 16 + c16;
        return J0 + wc * 8 * NN + n * 8 + (c16 >> 1);
    };
    const uint32_t *margr = a.marg + (int64_t)r * a.p_pad * C;
    const float *F1r = a.F1 + (int64_t)r * a.p_pad;

    // marginals are stored n1 << 16 | n0; the fp4 packing is 4 times that
    auto repack = [](uint32_t x) -> uint32_t { return F4 ? x << 2 : x; };
    uint32_t Mr[4][NP][C], Mc[NN][C];
    float Fr[4][NP], Fc[NN];
    float thrR[4][NP], thrC[NN], gR[4][NP], gC[NN];   // thresholds; maxima as read (a lower bound)
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int s = 0; s < NP; ++s) {
            int64_t v = row_var(m, s);
#pragma unroll
            for (int c = 0; c < C; ++c) Mr[m][s][c] = repack(margr[v * C + c]);
            Fr[m][s] = F1r[v];
            float gk = key_f32(a.G32[v]);
            gR[m][s] = gk;
            thrR[m][s] = gk - rescore_window(a.w_abs, gk);
        }
#pragma unroll
    for (int n = 0; n < NN; ++n) {
        int64_t v = col_var(n);
#pragma unroll
        for (int c = 0; c < C; ++c) Mc[n][c] = repack(margr[v * C + c]);
        Fc[n] = F1r[v];
        float gk = key_f32(a.G32[v]);
        gC[n] = gk;
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
        uint32_t P[C * C];
#pragma unroll
        for (int v = 0; v < C * C; ++v) P[v] = tab[v / C][v % C];
        return sum_vox<ENC, C * C>(P, smem, EA, EB, LQ);
    };

    float rmax[4][NP], cmax[NN];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int s = 0; s < NP; ++s) rmax[m][s] = -INFINITY;
#pragma unroll
    for (int n = 0; n < NN; ++n) cmax[n] = -INFINITY;
    bool hot = false;

#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NN; ++n)
#pragma unroll
            for (int s = 0; s < NP; ++s) {
                uint32_t tab[C][C];
                pair_table(m, n, s, tab);
                const int64_t rv = row_var(m, s), cv = col_var(n);
                const bool valid = rv < cv && cv < a.p;
                const float F2 = pair_F2(tab);
                if constexpr (MODE != SWEEP_PAIRS && W == 2) f2buf[(wave * 4 * NN + m * NN + n) * 64 + lane] = F2;
                if constexpr (MODE == SWEEP_PAIRS) {
                    // parent data of the k = 3 sweep: the W x W packed counts and F of the pair
                    if (valid) {
                        const int64_t pc = (int64_t)(r - a.r_base) * a.p_pad * a.p_pad + rv * a.p_pad + cv;
                        uint32_t *o = a.ptab + pc * (W * W);
#pragma unroll
                        for (int x = 0; x < W; ++x)
#pragma unroll
                            for (int y = 0; y < W; ++y) {
                                const uint32_t v = F4 ? tab[x][y] >> 2 : tab[x][y];   // n1 << 16 | n0
                                o[x * W + y] = a.pair_x4 ? v << 2 : v;
                            }
                        a.F2out[pc] = F2;
                    }
                    continue;
                }
                const float igR = valid ? Fc[n] - F2 : -INFINITY;   // gain of rv given cv
                const float igC = valid ? Fr[m][s] - F2 : -INFINITY; // gain of cv given rv
                rmax[m][s] = fmaxf(rmax[m][s], igR);
                cmax[n] = fmaxf(cmax[n], igC);
                hot |= (igR >= thrR[m][s]) | (igC >= thrC[n]);
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
    for (int n = 0; n < NN; ++n) {
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
        for (int n = 0; n < NN; ++n) {
            float g = key_f32(a.G32[col_var(n)]);
            float top = a.collect ? g : fmaxf(g, cmax[n]);
            thrC[n] = top - rescore_window(a.w_abs, top);
        }
        // W = 2: F of each pair from the first pass (LDS); W = 1 (64 values per lane, more than
        // the stage holds): recomputed from the accumulators in four rounds of 16 (the empty asm
        // stops the compiler from keeping the first pass's values alive instead), each round's F
        // parked in the same LDS buffer.  Per round: which pairs append (bit m * NN + n), one slot
        // reservation for the wave, then the records.
        if constexpr (W == 1) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < NN; ++n) asm volatile("" : "+v"(cnt[m][n]) : : "memory");
        }
#pragma unroll
        for (int s = 0; s < NP; ++s) {
            uint32_t selR = 0, selC = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < NN; ++n) {
                    float *slot = &f2buf[(wave * 4 * NN + m * NN + n) * 64 + lane];
                    if constexpr (W == 1) {
                        uint32_t tab[C][C];
                        pair_table(m, n, s, tab);
                        *slot = pair_F2(tab);
                    }
                    const float F2 = *slot;
                    const int64_t rv = row_var(m, s), cv = col_var(n);
                    const bool valid = rv < cv && cv < a.p;
                    const float igR = Fc[n] - F2, igC = Fr[m][s] - F2;
                    if (valid && igR >= thrR[m][s]) selR |= 1u << (m * NN + n);
                    if (valid && igC >= thrC[n]) selC |= 1u << (m * NN + n);
                }
            uint32_t at = reserve_slots(&a.st->n_cand, __popc(selR) + __popc(selC), lane);
            if (selR | selC) {
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < NN; ++n) {
                        const uint32_t bit = 1u << (m * NN + n);
                        if ((selR | selC) & bit) {
                            const float F2 = f2buf[(wave * 4 * NN + m * NN + n) * 64 + lane];
                            if (selR & bit) put_cand(at++, row_var(m, s), col_var(n), Fc[n] - F2);
                            if (selC & bit) put_cand(at++, col_var(n), row_var(m, s), Fr[m][s] - F2);
                        }
                    }
            }
        }
    }

    // publish the maxima: one lane per variable, only where the tile raised the maximum read
    // before (maxima only grow); the collect pass leaves the final maxima alone
    if (a.collect) continue;
    const bool row_leader = (W == 1) ? (c16 == 0) : ((c16 >> 1) == 0);
    const bool col_leader = (W == 1) ? (q == 0) : (q == 0 && odd == 0);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int s = 0; s < NP; ++s)
            if (row_leader && rmax[m][s] > gR[m][s]) atomicMax(&a.G32[row_var(m, s)], f32_key(rmax[m][s]));
#pragma unroll
    for (int n = 0; n < NN; ++n)
        if (col_leader && cmax[n] > gC[n]) atomicMax(&a.G32[col_var(n)], f32_key(cmax[n]));
    }   // W <= 2
    }   // work items
}

template <int W, int MODE, int ENC, bool EXPORT = false, int NWV = sw_waves(W)>
__global__ __launch_bounds__(NWV * 64, 2) __attribute__((amdgpu_waves_per_eu(NWV / 2, NWV / 2))) void k_sweep2(Sweep2Args a)
{
    sweep2_run<W, MODE, ENC, false, EXPORT, NWV>(a, nullptr);
}

// Waves per workgroup of the fused batch sweep: 4 for every class count.  With three classes the
// batch path needs a few more registers than 128, so 8-wave workgroups would fit one per CU; 4-wave
// ones (64 x 64 outputs per wave) fit two, as the LDS allows.
__host__ __device__ constexpr int batch_waves(int) { return 4; }

template <int W, int ENC>
__global__ __launch_bounds__(batch_waves(W) * 64, 2) __attribute__((amdgpu_waves_per_eu(batch_waves(W) / 2, batch_waves(W) / 2))) void k_sweep2_batch(Sweep2Batch bt)
{
    sweep2_run<W, SWEEP_MAX, ENC, true, false, batch_waves(W)>(bt.p[0], &bt);
}

// Table capacity of the fp4 layout for these class sizes (0 = does not fit any).
static int fp4_capacity(const Problem &P)
{
    const int need = (P.N0 > P.N1 ? P.N0 : P.N1) + 1;
    for (int T = 1024; T <= 4096; T *= 2)
        if (need <= T) return T;
    return 0;
}

size_t sweep2_lds_bytes(const Problem &P, bool max_mode)
{
    if (P.fp4) {
        const int T = max_mode ? fp4_capacity(P) : 4096;
        return (size_t)stage_base(T) + NSTAGE * STAGE_BYTES + 16;
    }
    size_t tab = sizeof(float) * (size_t)(P.N0 + 1 + P.N1 + 1 + 1) + sizeof(float2) * (P.L.N + 1);
    return NSTAGE * STAGE_BYTES + ((tab + 15) & ~size_t(15)) + 16;
}

int sweep2_fp4_capacity(const Problem &P) { return fp4_capacity(P); }

// Arguments of one problem's pair sweep.
template <int W>
static Sweep2Args sweep_args(const Problem &P, int32_t *counts_out, int disc_sel, bool collect, int pair_r, bool gated,
                             int pair_nr = 1)
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
    a.sb = P.supertile > 0 ? P.supertile : SB_DEFAULT;
    a.nsb = (a.nbv + a.sb - 1) / a.sb;
    a.super_per_r = (int64_t)a.nsb * (a.nsb + 1) / 2;
    a.n_super = a.super_per_r * (pair_r >= 0 ? pair_nr : L.R);
    a.r_base = pair_r >= 0 ? pair_r : 0;
    a.ptab = pair_r >= 0 ? P.at<uint32_t>(L.ptab) : nullptr;
    a.pair_x4 = pair_r >= 0 && P.k3_mfma ? 1 : 0;
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
    a.gated = gated ? 1 : 0;
    a.cancel = P.cancel;
    return a;
}

template <int W, int ENC>
static hipError_t sweep_launch(const Problem &P, int32_t *counts_out, int disc_sel, bool collect, int pair_r,
                               bool gated, int pair_nr)
{
    Sweep2Args a = sweep_args<W>(P, counts_out, disc_sel, collect, pair_r, gated, pair_nr);
    const size_t lds = sweep2_lds_bytes(P, pair_r < 0);
    a.snext_off = (int)(lds - 16);
    // three classes, maximum pass: 4-wave workgroups when asked for (a tuning choice)
    const bool four = W == 2 && pair_r < 0 && !counts_out && P.sweep_waves == 4;
    auto kern = pair_r >= 0 ? k_sweep2<W, SWEEP_PAIRS, ENC>
                            : (counts_out ? k_sweep2<W, SWEEP_MAX, ENC, true>
                                          : (four ? k_sweep2<W, SWEEP_MAX, ENC, false, 4> : k_sweep2<W, SWEEP_MAX, ENC>));
    if constexpr (ENC != 0) {
        // the fp4 epilogue reads its tables at LDS addresses equal to their array offsets
        static const hipError_t lds_ok =
            lds_array_at_zero({(const void *)k_sweep2<W, SWEEP_PAIRS, ENC>, (const void *)k_sweep2<W, SWEEP_MAX, ENC, true>,
                               (const void *)k_sweep2<W, SWEEP_MAX, ENC, false, 4>, (const void *)k_sweep2<W, SWEEP_MAX, ENC>});
        if (lds_ok != hipSuccess) return lds_ok;
    }
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // no more workgroups than tile slots (each loads its tables before it takes a tile), at least
    // one per XCD; the queue walk hands every tile to some workgroup whatever the grid
    const int64_t slots = a.n_super * (a.sb * a.sb);
    const int grid = P.workgroups > 0 ? P.workgroups
                                      : (int)std::min<int64_t>(XCDS * WG_PER_XCD, std::max<int64_t>(XCDS, slots));
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3((four ? 4 : sw_waves(W)) * 64), lds, P.stream, a);
    return hipGetLastError();
}

template <int W>
static hipError_t sweep_dispatch(const Problem &P, int32_t *counts_out, int disc_sel, bool collect, int pair_r,
                                 bool gated, int pair_nr)
{
    if (!P.fp4) return sweep_launch<W, 0>(P, counts_out, disc_sel, collect, pair_r, gated, pair_nr);
    // the maximum sweep (and with it the count export) is instantiated per table capacity
    // (occupancy); the pair data of the triple sweeps use the largest
    if (pair_r >= 0) return sweep_launch<W, 4096>(P, counts_out, disc_sel, collect, pair_r, gated, pair_nr);
    switch (fp4_capacity(P)) {
    case 1024: return sweep_launch<W, 1024>(P, counts_out, disc_sel, collect, pair_r, gated, pair_nr);
    case 2048: return sweep_launch<W, 2048>(P, counts_out, disc_sel, collect, pair_r, gated, pair_nr);
    case 4096: return sweep_launch<W, 4096>(P, counts_out, disc_sel, collect, pair_r, gated, pair_nr);
    default: return hipErrorInvalidValue;
    }
}

static hipError_t sweep_any(const Problem &P, int32_t *counts_out, int disc_sel, bool collect, int pair_r, bool gated,
                            int pair_nr = 1)
{
    switch (P.L.W) {
    case 1: return sweep_dispatch<1>(P, counts_out, disc_sel, collect, pair_r, gated, pair_nr);
    case 2: return sweep_dispatch<2>(P, counts_out, disc_sel, collect, pair_r, gated, pair_nr);
    case 4: return sweep_dispatch<4>(P, counts_out, disc_sel, collect, pair_r, gated, pair_nr);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep2(const Problem &P, int32_t *counts_out, int disc_sel, bool collect)
{
    return sweep_any(P, counts_out, disc_sel, collect, -1, collect);
}

hipError_t launch_pairs(const Problem &P, int r0, int nr, bool gated)
{
    return sweep_any(P, nullptr, -1, false, r0, gated, nr);
}

// ---------------------------------------------------------------- count export, completion
// The maximum pass stored the W x W directly counted cells of every pair i < j of the selected
// discretisation into counts [p][p][2][C][C]; the cells of the dropped last bin of either variable
// follow exactly from the per-class marginals: n[a][W] = M_i[a] - sum_b<W n[a][b] and
// n[W][b] = M_j[b] - sum_a<W n[a][b].  One thread per (i, j).
template <int C>
__global__ __launch_bounds__(256) void k_complete_pairs(int32_t *counts, const uint32_t *marg, int r, int64_t p,
                                                        int64_t p_pad)
{
    constexpr int W = C - 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * p) return;
    const int64_t i = t / p, j = t % p;
    if (i >= j) return;
    const uint32_t *Mi = marg + ((int64_t)r * p_pad + i) * C, *Mj = marg + ((int64_t)r * p_pad + j) * C;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        int32_t *o = counts + (t * 2 + d) * C * C;
        auto part = [d](uint32_t x) { return (int32_t)(d ? x >> 16 : x & 0xffffu); };
#pragma unroll
        for (int x = 0; x < W; ++x) {
            int32_t s = part(Mi[x]);
#pragma unroll
            for (int y = 0; y < W; ++y) s -= o[x * C + y];
            o[x * C + W] = s;
        }
#pragma unroll
        for (int y = 0; y < C; ++y) {
            int32_t s = part(Mj[y]);
#pragma unroll
            for (int x = 0; x < W; ++x) s -= o[x * C + y];
            o[W * C + y] = s;
        }
    }
}

hipError_t launch_complete_pairs(const Problem &P, int32_t *counts, int r)
{
    const int64_t n = P.L.p * P.L.p;
    const dim3 grid((unsigned)((n + 255) / 256));
    const uint32_t *marg = P.at<uint32_t>(P.L.marg);
    switch (P.L.C) {
    case 2: hipLaunchKernelGGL(k_complete_pairs<2>, grid, dim3(256), 0, P.stream, counts, marg, r, P.L.p, P.L.p_pad); break;
    case 3: hipLaunchKernelGGL(k_complete_pairs<3>, grid, dim3(256), 0, P.stream, counts, marg, r, P.L.p, P.L.p_pad); break;
    case 5: hipLaunchKernelGGL(k_complete_pairs<5>, grid, dim3(256), 0, P.stream, counts, marg, r, P.L.p, P.L.p_pad); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- several problems, one launch
template <int W, int ENC>
static hipError_t batch_launch(const Problem *const *Ps, int n, Status *queue, size_t lds)
{
    Sweep2Batch b{};
    b.nb = n;
    b.queue = queue;
    b.pref[0] = 0;
    for (int i = 0; i < n; ++i) {
        b.p[i] = sweep_args<W>(*Ps[i], nullptr, -1, false, -1, false);
        b.p[i].snext_off = (int)(lds - 16);   // one LDS size for the whole launch
        b.pref[i + 1] = b.pref[i] + b.p[i].n_super;
    }
    auto kern = k_sweep2_batch<W, ENC>;
    if constexpr (ENC != 0) {
        static const hipError_t lds_ok = lds_array_at_zero({(const void *)kern});
        if (lds_ok != hipSuccess) return lds_ok;
    }
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int grid = Ps[0]->workgroups > 0 ? Ps[0]->workgroups : XCDS * WG_PER_XCD;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(batch_waves(W) * 64), lds, Ps[0]->stream, b);
    return hipGetLastError();
}

template <int W>
static hipError_t batch_dispatch(const Problem *const *Ps, int n, Status *queue)
{
    // one encoding and table capacity for all: the largest any problem needs
    size_t lds = 0;
    int T = 0;
    for (int i = 0; i < n; ++i) {
        lds = std::max(lds, sweep2_lds_bytes(*Ps[i], true));
        T = std::max(T, fp4_capacity(*Ps[i]));
    }
    if (!Ps[0]->fp4) return batch_launch<W, 0>(Ps, n, queue, lds);
    lds = (size_t)stage_base(T) + NSTAGE * STAGE_BYTES + 16;
    switch (T) {
    case 1024: return batch_launch<W, 1024>(Ps, n, queue, lds);
    case 2048: return batch_launch<W, 2048>(Ps, n, queue, lds);
    case 4096: return batch_launch<W, 4096>(Ps, n, queue, lds);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep2_batch(const Problem *const *Ps, int n, Status *queue)
{
    if (n < 1 || n > MAX_BATCH) return hipErrorInvalidValue;
    for (int i = 1; i < n; ++i)
        if (Ps[i]->L.W != Ps[0]->L.W || Ps[i]->fp4 != Ps[0]->fp4) return hipErrorInvalidValue;
    switch (Ps[0]->L.W) {
    case 1: return batch_dispatch<1>(Ps, n, queue);
    case 2: return batch_dispatch<2>(Ps, n, queue);
    case 4: return batch_dispatch<4>(Ps, n, queue);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mdfs
