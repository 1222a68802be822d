// mdfs_internal.h -- declarations shared by the HIP sources of libmdfs (gfx950 only).
//
// Device memory layout of one problem inside the caller's workspace, the candidate record of
// the max reduction, order-preserving integer keys for floating-point atomics, and the
// launchers each .hip file exports to the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <initializer_list>
#include <vector>

namespace mdfs {

// One-hot bytes per row and K block.  The int8 encoding holds 64 objects per K block (one byte
// each), the E2M1 (fp4) encoding 128 (one nibble each).  Objects are permuted class-0-first and
// each class is padded to a whole K block of the encoding in use.
constexpr int KBLK = 64;
constexpr int KOBJ_I8 = 64;
constexpr int KOBJ_F4 = 128;
// E2M1 bit pattern of 2.0 (sign 0, biased exponent 10, mantissa 0): the fp4 one-hot value,
// so that each product is 4 and counts arrive as byte offsets of float tables.
constexpr uint32_t F4_TWO = 0x4u;
// The fp4 engine accumulates n1 * 2^14 + 4 n0 in float32: exact while both classes are < 4096.
constexpr int MAX_CLASS_OBJ_F4 = 4095;
// Output rows of one sweep tile (one-hot rows = variables x (classes-1) bins).
constexpr int TILE_ROWS = 128;
// Variables are padded to a multiple of this (covers every tile width).
constexpr int VAR_PAD = 128;
constexpr int MAX_NOBJ = 16384;
constexpr int MAX_CLASS_OBJ = 32767;
// k = 3: the matrix-core tile list holds j blocks of 32 variables below 256 (p <= 8192)
constexpr int MAX_K3_VARS = 8192;
// k >= 4 candidates carry the lexicographic rank of their partner tuple in 32 bits:
// C(2048, 3) and C(512, 4) are below 2^32
constexpr int MAX_K4_VARS = 2048;
constexpr int MAX_K5_VARS = 512;
constexpr int MAX_BATCH = 12;          // problems fused in one persistent pair-sweep launch

// Status words at the start of the workspace.
struct Status {
    uint32_t nan_flag;    // data held a NaN
    uint32_t n_cand;      // candidate records appended (may exceed capacity)
    uint32_t overflow;    // some append did not fit
    uint32_t n_emit;      // records written by the interesting-tuples emit pass
    uint32_t code_flag;   // caller-supplied codes held a value above divisions
    uint32_t collect_go;  // the gated collect pass runs (set on the device before it)
    uint32_t y_flag;      // y disagreed with the class-1 count given to an asynchronous call
    uint32_t cancelled;   // a sweep kernel saw the caller's cancel word set and stopped early
    uint32_t pad0[8];
    uint32_t next_tile[16];   // per-XCD work counters of the persistent sweep (reset per pass)
    uint32_t pad[32];
};

// One candidate of the max reduction: variable v reached ig32 with partner(s) under disc r.
// For k = 2 `partner` is the other variable; for k = 3 it packs (m1 | m2 << 16), m1 < m2.
struct Cand {
    int32_t v;
    int32_t r;
    uint32_t partner;
    float ig32;
};

// Byte offsets of every array inside the workspace (all 256-byte aligned).
struct Layout {
    // problem sizes
    int64_t N, p, p_pad;
    int k, C, W;          // classes C = divisions+1, one-hot width W = C-1
    int R;
    int RC;               // k = 3: discretisations whose pair data are held at once (one launch pair)
    int64_t Kpad_max;     // class-sorted positions reserved: worst-case padding of either encoding
    int64_t rows_pad;     // p_pad * W
    int64_t cap;          // candidate capacity
    int64_t words_max;    // bitset words (32 objects) per class, worst case (k=3)
    // offsets
    size_t status, pos, perm, tabEA, tabEB, tabLQ, marg, F1, onehot, G32, max64, keyw, ovf,
        cand, ig64, bits, ptab, F2, a3pref, a3blk, F1d, ccodes, total;
};

// k = 3 holds the pair data of as many discretisations as fit in pair_budget bytes (at least one)
constexpr size_t PAIR_BUDGET_DEFAULT = size_t(64) << 20;
Layout make_layout(int64_t N, int64_t p, int k, int divisions, int R, size_t pair_budget = PAIR_BUDGET_DEFAULT);
// per-class bitsets are built for k = 3, k = 4 and, with two classes, k = 5
inline bool uses_bits(const Layout &L) { return L.k == 3 || L.k == 4 || (L.k == 5 && L.C == 2); }

// Byte offset of (discretisation r, one-hot row, K block kb, byte) in the panel-major one-hot
// encoding [r][row / TILE_ROWS][kb][row % TILE_ROWS][KBLK]: the rows of one sweep panel are
// contiguous over all K blocks, so a tile streams one contiguous run per operand.  Position e of
// a K block sits in byte e (int8) or in byte e / 2, low nibble for even e (fp4).
__host__ __device__ inline int64_t onehot_off(int r, int64_t row, int kb, int byte, int KB, int64_t rows_pad)
{
    const int64_t nrb = rows_pad / TILE_ROWS;
    return ((((int64_t)r * nrb + row / TILE_ROWS) * KB + kb) * TILE_ROWS + row % TILE_ROWS) * KBLK + byte;
}

// Order-preserving maps from floats to unsigned integers (larger float -> larger key).
__host__ __device__ inline uint32_t f32_key(float f)
{
    uint32_t b = __builtin_bit_cast(uint32_t, f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ inline float key_f32(uint32_t k)
{
    uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __builtin_bit_cast(float, b);
}
__host__ __device__ inline uint64_t f64_key(double f)
{
    uint64_t b = __builtin_bit_cast(uint64_t, f);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ inline double key_f64(uint64_t k)
{
    uint64_t b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
    return __builtin_bit_cast(double, b);
}

// Partner tuples of k >= 4 candidates: the lexicographic rank of the ascending tuple among the
// m-subsets of {0 .. n-1} (so that comparing ranks compares tuples as the tie rule does).  The
// subsets whose first element is below x, given the earlier elements end before a, number
// C(n - a, m) - C(n - x, m) (hockey-stick identity).
__host__ __device__ inline uint64_t binom_u64(int64_t n, int k)
{
    if (k < 0 || n < k) return 0;
    uint64_t r = 1;
    for (int i = 0; i < k; ++i) r = r * (uint64_t)(n - i) / (uint64_t)(i + 1);   // C(n, i + 1), exact
    return r;
}
__host__ __device__ inline uint32_t lex_rank(const int *c, int m, int64_t n)
{
    uint64_t r = 0;
    int64_t a = 0;
    for (int i = 0; i < m; ++i) {
        r += binom_u64(n - a, m - i) - binom_u64(n - c[i], m - i);
        a = c[i] + 1;
    }
    return (uint32_t)r;
}
__host__ __device__ inline void lex_unrank(uint64_t r, int m, int64_t n, int *c)
{
    int64_t a = 0;
    for (int i = 0; i < m; ++i) {
        const uint64_t top = binom_u64(n - a, m - i);
        int64_t x = a;
        while (top - binom_u64(n - x - 1, m - i) <= r) ++x;   // subsets with first element <= x
        r -= top - binom_u64(n - x, m - i);
        c[i] = (int)x;
        a = x + 1;
    }
}

// Tie tolerance of the argmax: candidates within tau of the maximum are tied.
__host__ __device__ inline double tie_tau(double m) { return 1e-9 * (fabs(m) > 1.0 ? fabs(m) : 1.0); }

// n h(p) of one voxel from the entropy tables of the bitset sweeps, which lay EA, EB and the
// (L, Q) pairs out in that order at the start of their dynamic LDS array.  P4 = (4 n1) << 16 |
// 4 n0 (the packed count shifted left by 2) holds the counts' byte offsets in its halves; each
// class has fewer than 16384 objects, as the entropy tables of every sweep must fit in LDS.  The
// array sits at LDS address 0 when the kernel declares no static LDS (checked at launch by
// lds_array_at_zero), so 4 n0 is the address of EA[n0]; EB and the pairs follow at byte offsets
// offB and offL: five VALU instructions per voxel with the shift, where indexing the tables by
// n0, n1 and n takes seven.
__device__ inline float vox_lds(uint32_t P4, uint32_t offB, uint32_t offL)
{
    typedef float vf2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) const float lds_f32;
    typedef __attribute__((address_space(3))) const vf2 lds_f32x2;
    const uint32_t a0 = P4 & 0xffffu, a1 = P4 >> 16;
    const float ea = *reinterpret_cast<const lds_f32 *>((uintptr_t)a0);
    const float eb = *reinterpret_cast<const lds_f32 *>((uintptr_t)(offB + a1));
    const vf2 lq = *reinterpret_cast<const lds_f32x2 *>((uintptr_t)(offL + 2 * (a0 + a1)));
    return lq.x - lq.y * (ea + eb);
}

// hipSuccess when none of the kernels declares static LDS, so that each one's dynamic LDS array
// starts at LDS address 0 (what vox_lds and the fp4 sweeps' table reads rely on).
inline hipError_t lds_array_at_zero(std::initializer_list<const void *> kernels)
{
    for (const void *k : kernels) {
        hipFuncAttributes fa{};
        const hipError_t e = hipFuncGetAttributes(&fa, k);
        if (e != hipSuccess) return e;
        if (fa.sharedSizeBytes != 0) return hipErrorInvalidDeviceFunction;
    }
    return hipSuccess;
}

// First of the `mine` consecutive candidate slots of this lane: an exclusive prefix sum of the
// lanes' counts and one device-scope atomic per wave for the wave's total (every lane of the
// wave must take part).  The sweeps append through it so that a wave waits on one returning
// atomic on the shared counter per round of appends, not one per record.
__device__ __forceinline__ uint32_t reserve_slots(uint32_t *counter, uint32_t mine, int lane)
{
    if (!__any(mine != 0)) return 0;
    uint32_t incl = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, d);
        if (lane >= d) incl += y;
    }
    const uint32_t total = (uint32_t)__shfl((int)incl, 63);
    uint32_t base = 0;
    if (total != 0) {
        if (lane == 0) base = atomicAdd(counter, total);
        base = (uint32_t)__shfl((int)base, 0);
    }
    return base + incl - mine;
}

// The caller's cancel word (host-mapped, nullable), read with a system-scope load so that a
// host write made while the kernel runs is seen.  Persistent sweeps poll it every 16 work items
// (`taken` counts the items a workgroup or wave has taken) and, when it is set, record it in
// Status::cancelled and stop taking work.
__device__ inline bool cancel_poll(const uint32_t *cancel, uint32_t taken, Status *st)
{
    if (cancel == nullptr || (taken & 15u) != 0) return false;
    if (__hip_atomic_load(const_cast<uint32_t *>(cancel), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == 0)
        return false;
    atomicOr(&st->cancelled, 1u);
    return true;
}

// Everything a launch sequence needs about one problem (sizes, pseudocounts, buffers).
struct Problem {
    Layout L;
    int N0, N1;                   // class sizes
    bool fp4;                     // one-hot in E2M1 nibbles (else int8 bytes)
    int kobj;                     // objects per K block: KOBJ_F4 or KOBJ_I8
    int K0pad, Kpad, KB0, KB;     // class-0 padded size, all positions, K blocks (class 0, all)
    double beta0, beta1;
    int disc_offset;
    double range;
    uint64_t seed;
    double err_bound;             // float32 screen error bound E (per IG)
    bool k3_mfma;                 // k = 3 on the matrix cores (else bitsets)
    bool hist;                    // k >= 4 on the per-tuple histogram engine (else bitsets)
    bool sweep45;                 // k >= 4 on bitsets with two classes (prefix waves, pair lanes)
    int workgroups;               // persistent sweep grid (0 = the whole GPU)
    int supertile;                // pair sweep: super-tile side in tiles (0 = default)
    int sweep_waves;              // pair sweep, three classes: waves per workgroup (0 = default)
    int64_t n_ablk3, n_tiles3;    // tile list of the k = 3 matrix-core sweep
    const uint8_t *codes_in = nullptr;   // caller-supplied codes [R][p][N] replace the discretisation
    const uint32_t *cancel = nullptr;    // caller's host-mapped cancel word (nullable)
    char *ws;
    hipStream_t stream;
    template <class T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

// ---- launchers (each returns hipSuccess or the launch error)
hipError_t launch_init(const Problem &P);
// n1_check >= 0: y is also checked on the device against that class-1 count (y_flag on mismatch,
// then nothing is written)
hipError_t launch_class_perm(const Problem &P, const uint8_t *y, int64_t n1_check = -1);
hipError_t launch_tables(const Problem &P);
hipError_t launch_discretize(const Problem &P, const float *data, uint8_t *codes, bool encode);
// the encoding, marginals and F1 from caller-supplied codes (P.codes_in) instead of discretising
hipError_t launch_encode_codes(const Problem &P);
hipError_t launch_sweep2(const Problem &P, int32_t *counts_out, int disc_sel, bool collect = false);
// the count export: cells of the dropped last bins of every pair from the marginals of disc r
hipError_t launch_complete_pairs(const Problem &P, int32_t *counts, int r);
// LDS bytes per workgroup of the pair sweep (max_mode: the maximum sweep, else debug/pair modes)
size_t sweep2_lds_bytes(const Problem &P, bool max_mode);
constexpr size_t LDS_MAX = 160 * 1024;
// gated: only when the collect pass will run (Status::collect_go)
hipError_t launch_reset_candidates(const Problem &P, bool gated = false);
// Status::collect_go = force ? 1 : (a candidate append overflowed)
hipError_t launch_collect_decide(const Problem &P, bool force);
// pair data (W x W counts and float32 F of every pair) of discretisations r0 .. r0 + nr - 1
hipError_t launch_pairs(const Problem &P, int r0, int nr, bool gated = false);
// The maximum pass of several k = 2 problems in one persistent launch (same d and encoding);
// `queue` holds the batch's work counters (a Status in device memory).
hipError_t launch_sweep2_batch(const Problem *const *Ps, int n, Status *queue);
// Table capacity of the fp4 pair sweep for a problem's class sizes (0 = does not fit).
int sweep2_fp4_capacity(const Problem &P);
// k = 3 sweeps of discretisation r; counts_out != nullptr: also the count export of the triples
// (i_sel, j, l), directly counted cells only (launch_complete_triples fills in the others)
hipError_t launch_sweep3(const Problem &P, int r0, int nr, bool collect, int32_t *counts_out = nullptr,
                         int i_sel = -1, int disc_sel = -1);
// cells of the dropped last bins of the exported triples, from the pair data of discretisation
// r (held in the chunk that starts at r0)
hipError_t launch_complete_triples(const Problem &P, int32_t *counts, int r, int r0, int i_sel);
// k = 4 bitset sweep of discretisation r, three classes (sweep4.hip)
hipError_t launch_sweep4(const Problem &P, int r, bool collect);
// k = 4 or 5 bitset sweep of discretisation r, two classes (sweep45.hip)
hipError_t launch_sweep45(const Problem &P, int r, bool collect);
// LDS bytes per workgroup of that sweep (tables and the waves' prefix words)
size_t sweep45_lds_bytes(const Problem &P);
// k = 4 or 5 per-tuple histogram sweep of discretisation r, any class count (sweep_hist.hip)
hipError_t launch_sweep_hist(const Problem &P, int r, bool collect);
// binary64 re-score of k >= 4 candidates from the class-sorted codes (sweep_hist.hip)
hipError_t launch_rescore_hist(const Problem &P);
// LDS bytes per workgroup of the histogram sweep (0 = not built for these sizes)
size_t sweep_hist_lds_bytes(const Problem &P);
hipError_t launch_sweep3m(const Problem &P, int r0, int nr, bool collect, int32_t *counts_out = nullptr,
                          int i_sel = -1, int disc_sel = -1);
size_t sweep3m_lds_bytes(const Problem &P);
// tile list of the k = 3 matrix-core sweep: its size on the host, the list itself on the device
void sweep3m_tile_counts(int64_t p, int W, int64_t &n_ablk, int64_t &n_tiles);
hipError_t launch_tiles3(const Problem &P);
hipError_t launch_reset_queue(const Problem &P);
hipError_t launch_finalize(const Problem &P, float *ig_max, int32_t *argmax, int32_t *argmax_disc);
// every variable's threshold key set to `key` (the interesting-tuples collect pass)
hipError_t launch_fill_g(const Problem &P, uint32_t key);
// binary64 re-score of the candidates, then every record with IG >= thr written out
hipError_t launch_emit(const Problem &P, double thr, int32_t *var, int32_t *partners, int32_t *disc, double *ig,
                       int64_t max_out);
hipError_t launch_screen_out(const Problem &P, float *ig32);
// k = 1: IG(i) = F(root) - F(x_i) per discretisation, max and tie rule over discretisations
hipError_t launch_ig1(const Problem &P, double F0, float *ig_max, int32_t *argmax_disc);
// contrast variables (contrast.hip): the source variable of contrast variable c, and the launch
// that writes the originals then the permuted copies into out [n_var + n_contrast][n_obj]
int64_t contrast_source(uint64_t seed, int64_t c, int64_t n_var);
hipError_t launch_contrast(const float *data, int64_t n_obj, int64_t n_var, int64_t n_contrast, uint64_t seed,
                           float *out, hipStream_t stream);

}  // namespace mdfs
