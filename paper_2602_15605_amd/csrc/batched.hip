// Batched form: many windows (masks) of uneven lmax in one contraction launch.
//
// For a set of masks the l3 reduction is a contraction
//
//     Xi_X^m(l1, l2) = sum_{l3} A_X(l1, l2, l3) W'_X^m(l3),
//
// where the "3j^2 tile" A_X does not depend on the mask:
//     A_TT = (l1 l2 l3; 0 0 0)^2,  A_TE = A_TT N',  A_EE = A_TT N'^2
// (Sec. 2 eqs. K_TT, K_EE; App. A; the (-2 2 0) factor N' s as in the strip
// kernels, with s applied per row at the end).  Along a diagonal d the pairs
// (l1, l1 + d) form the M dimension, k (l3 = d + 2k) the K dimension and the
// masks the N dimension, so the contraction runs on the matrix cores:
//
//   * masks are sorted by lmax and split into column groups of 16;
//   * one wavefront owns a diagonal d and TM*16 consecutive l1 of a group; it
//     generates its A elements on the VALU (g/h windows and the per-k factors
//     staged in LDS, as in the strip kernels) in the A-operand layout of the
//     MFMA and contracts them against the W' tile (k x 16 masks) loaded from
//     an L2-resident table ahead of its use (two steps in float32, one in
//     BF16x3, whose A generation per step is eight times longer);
//   * float32 form: v_mfma_f32_16x16x4f32 (lane l holds row l % 16, k offset
//     l / 16 of A and k offset l / 16, mask l % 16 of B);
//     BF16x3 form: v_mfma_f32_16x16x32_bf16 (lane l holds row l % 16,
//     k offsets 8 (l / 16) .. + 7); every float32 operand is split into
//     bfloat16 hi + lo and the product is hi*hi + hi*lo + lo*hi, three MFMAs
//     accumulating in float32 (the dropped lo*lo and the two split residues
//     bound the product's relative error by 3 * 2^-16, bfloat16 keeping 8
//     significant bits);
//   * every `flush` steps the float32 matrix-core accumulators are added into
//     Kahan (sum, compensation) pairs (float32 form) or plain float32 sums
//     (BF16x3, whose operand splits bound the error);
//   * each mask's Xi goes to its own packed triangle [3][tri(lmax_m)], the
//     store layout of the single-mask path; the MFMA output tile (lane l holds
//     rows 4 (l/16) + i, mask l % 16) writes 16 consecutive l1 of a mask in
//     one 128-byte run.
// A fill pass then writes each mask's K (the single-mask fill, one job per
// mask, all masks in one launch).
#include <algorithm>
#include <type_traits>

#include "couple_internal.hpp"

namespace couple {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

constexpr int kGroup = kMaskGroup;  // masks per MFMA column block
constexpr int kBThreads = 64;
constexpr int kChunkF32 = 128;      // k staged per chunk: 32 float32 steps (16 x 16 x 4 form)
constexpr int kChunkBF16 = 256;     // 8 BF16x3 steps

// Zero rows after the last l3 of the 16-mask float32 W' table, so the prefetch of
// the two steps past a wavefront's last one stays in bounds without a test.
constexpr int kF32TailRows = 32;

struct BatchArgs {
    int n_groups;
    // per group
    int L[kMaxGroups];              // largest lmax in the group
    int n_items[kMaxGroups];        // work items of the group
    int bmax[kMaxGroups];
    long long wt_off[kMaxGroups];   // offset of the group's W' table (elements)
    int wt_len[kMaxGroups];         // float32: rows 2L+1+tail; BF16x3: j slots per (x, piece, parity, mask)
    // per mask of a group (lmax -1: empty column)
    int lmax[kMaxGroups][kGroup];
    long long xi_off[kMaxGroups][kGroup];   // offset of the mask's Xi store [3][tri(lmax)] (doubles)
    // shared
    const double* g;                // float64 g(p)
    const float* gf;                // float32 g(p)
    const float* hf;                // float32 1/((2p+1) g(p))
    const double* cl;
    const void* wtab;               // W' tables of every group
    double* xi;                     // Xi workspace base
    int g_len, h_len;
    int flush;                      // MFMA steps per accumulator flush
};

// Waves per SIMD the register allocation is held to (the largest that does
// not spill; the attribute also lets the accumulators share the unified
// register file instead of a separate AGPR allocation).
template <int TM>
constexpr int kF32Waves = TM <= 2 ? 4 : 2;
template <int TM>
constexpr int kBF16Waves = TM == 1 ? 3 : (TM == 2 ? 2 : 1);

template <int TM, int KC>
struct BWin {
    static constexpr int kRows = 16 * TM;
    static constexpr int kLen = kRows + KC + 3;
};

// Kahan step: (s, c) += v.
__device__ inline void kahan_add(float& s, float& c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Work item -> (group, level b, diagonal d); items of a group are numbered
// with the longest rows (largest b) first.
template <int TM>
__device__ inline void decode_item(const BatchArgs& a, int item, int* grp_out, int* b_out, int* d_out) {
    constexpr int kRows = 16 * TM;
    int grp = 0;
    while (grp < a.n_groups - 1 && item >= a.n_items[grp]) {
        item -= a.n_items[grp];
        ++grp;
    }
    const int L = a.L[grp];
    int b = a.bmax[grp];
    for (; b > 0; --b) {
        const int nb = L - kRows * b + 1;
        if (nb > 0) {
            if (item < nb) break;
            item -= nb;
        }
    }
    *grp_out = grp;
    *b_out = b;
    *d_out = item;
}

// Stage the chunk of k = kch .. kch + KC - 1: the g / h windows of the
// wavefront's rows, S(k) = g(k) g(d+k) (0 outside 0 <= k <= kmax) and
// D(k) = c(d + 2k) - c(d + 2 ke), ke = max(kch, 0) the chunk's expansion
// point (chunk_expansion), an integer exact in float32 while below 2^24 (l3 up
// to about 8000) and rounded once above.  Fully unrolled, so every global load
// is in flight before the first LDS write.
template <int TM, int KC>
__device__ inline void stage_chunk(const BatchArgs& a, float* s_g, float* s_h, float* s_s, float* s_dc, int A0,
                                   int d, int kch, int kmax, int lane) {
    using W = BWin<TM, KC>;
    constexpr int NW = (W::kLen + kBThreads - 1) / kBThreads;
    constexpr int NK = KC / kBThreads;
    const int g_base = A0 - kch - KC - 3;
    const int h_base = A0 + d + kch;
    float gv[NW], hv[NW];
    double ga[NK], gb[NK];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int slot = lane + kBThreads * i;
        const int eg = g_base + slot, eh = h_base + slot;
        gv[i] = (slot < W::kLen && eg >= 0 && eg < a.g_len) ? a.gf[eg] : 0.0f;
        hv[i] = (slot < W::kLen && eh >= 0 && eh < a.h_len) ? a.hf[eh] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < NK; ++i) {
        const int k = kch + lane + kBThreads * i;
        const bool ok = k >= 0 && k <= kmax;
        ga[i] = ok ? a.g[k] : 0.0;
        gb[i] = ok ? a.g[d + k] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int slot = lane + kBThreads * i;
        if (slot < W::kLen) {
            s_g[slot] = gv[i];
            s_h[slot] = hv[i];
        }
    }
    const int l3c = d + 2 * max(kch, 0);
#pragma unroll
    for (int i = 0; i < NK; ++i) {
        const int s = lane + kBThreads * i;
        const int k = kch + s;
        const int l3 = d + 2 * k;
        s_s[s] = (float)(ga[i] * gb[i]);
        s_dc[s] = (k >= 0 && k <= kmax) ? (float)(l3 * (l3 + 1) - l3c * (l3c + 1)) : 0.0f;
    }
}

// Xi store of the wavefront's rows: lane (r, q) holds rows 4q + i of each row
// tile for mask r of the group.  The (-2 2 0) row factor s = c_l1 c_l2 / 2
// (App. B.3) is applied here in float64.
template <int TM>
__device__ inline void store_xi(const BatchArgs& a, int grp, int d, int A0, int lane, const float (&ks)[TM][3][4],
                                const float (&kc)[TM][3][4]) {
    const int r = lane & 15, q = lane >> 4;
    const int lm = a.lmax[grp][r];
    if (lm < d) return;
    double* xi = a.xi + a.xi_off[grp][r];
    const long long tri = tri_size(lm);
    const long long off = diag_offset(lm, d);
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int l1 = A0 + 16 * t + 4 * q + i;
            if (l1 <= lm - d) {
                const double sp = 0.5 * a.cl[l1] * a.cl[l1 + d];
                const long long idx = off + l1;
                xi[idx] = (double)ks[t][0][i] - (double)kc[t][0][i];
                xi[tri + idx] = sp * ((double)ks[t][1][i] - (double)kc[t][1][i]);
                xi[2 * tri + idx] = (sp * sp) * ((double)ks[t][2][i] - (double)kc[t][2][i]);
            }
        }
}

// Row constants: gam = a + b - 1 and beta = 2ab + 1, both exact, with
// N' = t^2 - beta and t = c - gam.
template <int TM>
__device__ inline void row_constants(int A0, int d, int r, int (&gam)[TM], long long (&beta)[TM]) {
#pragma unroll
    for (int t = 0; t < TM; ++t) {
        const long long l1 = A0 + 16 * t + r, l2 = l1 + d;
        const long long aa = l1 * (l1 + 1), bb = l2 * (l2 + 1);
        gam[t] = (int)(aa + bb - 1);
        beta[t] = 2 * aa * bb + 1;
    }
}

// N' expanded about a chunk's first valid l3 (c_s = l3c (l3c + 1), l3c for
// k = max(kch, 0): a point outside the row's range would inflate Q): with
// T = c_s - gam and D = c - c_s, N' = Q + D (2T + D), Q = T^2 - beta exact in
// int64.  Per step N' = fma(D, rf + D, qf) with qf = fl(Q), rf = fl(2T): the
// cancellation of t^2 against beta happens exactly, once per chunk.
template <int TM>
__device__ inline void chunk_expansion(int l3c, const int (&gam)[TM], const long long (&beta)[TM], float (&qf)[TM],
                                       float (&rf)[TM]) {
    const long long c = (long long)l3c * (l3c + 1);
#pragma unroll
    for (int t = 0; t < TM; ++t) {
        const long long T = c - gam[t];
        qf[t] = (float)(double)(T * T - beta[t]);
        rf[t] = 2.0f * (float)T;
    }
}

// Add the matrix-core accumulators into the running sums: Kahan pairs
// (COMP), or a plain float32 sum.
template <int TM, bool COMP>
__device__ inline void flush_acc(f4v (&acc)[TM][3], float (&ks)[TM][3][4], float (&kc)[TM][3][4]) {
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int x = 0; x < 3; ++x) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (COMP)
                    kahan_add(ks[t][x][i], kc[t][x][i], acc[t][x][i]);
                else
                    ks[t][x][i] += acc[t][x][i];
            }
            acc[t][x] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
        }
}

// ---------------------------------------------------------------------------
// float32 matrix-core form: steps of 4 k, lane k offset q = lane / 16.
// W' table per group: [3][wt_len][16] float32, row l3, zero beyond 2 lmax_m
// and in the tail rows.
template <int TM>
__global__ void __launch_bounds__(kBThreads) __attribute__((amdgpu_waves_per_eu(kF32Waves<TM>, 8)))
batched_mfma_f32_kernel(BatchArgs a) {
    constexpr int KC = kChunkF32;
    using W = BWin<TM, KC>;
    __shared__ float s_g[W::kLen];
    __shared__ float s_h[W::kLen];
    __shared__ float s_s[KC];
    __shared__ float s_dc[KC];

    int grp, b, d;
    decode_item<TM>(a, blockIdx.x, &grp, &b, &d);
    const int L = a.L[grp];
    const int A0 = W::kRows * b;
    const int n_valid = L - d + 1;
    const int kmax = min(A0 + W::kRows, n_valid) - 1;

    const int lane = threadIdx.x;
    const int r = lane & 15, q = lane >> 4;
    // B operand: W'_X(l3)[mask r], l3 = d + 2k, k = 4 step + q; a step advances 8 rows
    const float* pb = static_cast<const float*>(a.wtab) + a.wt_off[grp] + (long long)(d + 2 * q) * kGroup + r;
    const long long xs = (long long)a.wt_len[grp] * kGroup;
    constexpr int kStepRows = 8 * kGroup;

    int gam[TM];
    long long beta[TM];
    row_constants<TM>(A0, d, r, gam, beta);
    f4v acc[TM][3];
    float ks[TM][3][4], kc[TM][3][4];
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            acc[t][x] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < 4; ++i) ks[t][x][i] = kc[t][x][i] = 0.0f;
        }

    // two B buffers: even steps use bA, odd steps bB; each is refilled for the
    // step two ahead right after its use
    float bA[3], bB[3];
    bA[0] = pb[0];
    bA[1] = pb[xs];
    bA[2] = pb[2 * xs];
    bB[0] = pb[kStepRows];
    bB[1] = pb[kStepRows + xs];
    bB[2] = pb[kStepRows + 2 * xs];
    pb += 2 * kStepRows;

    int since_flush = 0;
    for (int kch = 0; kch <= kmax; kch += KC) {
        const int kc_n = min(KC, kmax - kch + 1);
        __syncthreads();
        stage_chunk<TM, KC>(a, s_g, s_h, s_s, s_dc, A0, d, kch, kmax, lane);
        float qf[TM], rf[TM];
        chunk_expansion<TM>(d + 2 * max(kch, 0), gam, beta, qf, rf);
        __syncthreads();
        const int g_base = A0 - kch - KC - 3;

        auto step = [&](int s0, float (&bv)[3]) {
            const int s = s0 + q;
            const float S = s_s[s];
            const float D = s_dc[s];
            float x2[TM], y[TM], z[TM];
#pragma unroll
            for (int t = 0; t < TM; ++t) {
                const int l1 = A0 + 16 * t + r;
                const float gv = s_g[l1 - (kch + s) - g_base];
                const float hv = s_h[l1 - A0 + s];
                x2[t] = S * (gv * hv);
                const float N = __builtin_fmaf(D, rf[t] + D, qf[t]);
                y[t] = x2[t] * N;
                z[t] = y[t] * N;
            }
#pragma unroll
            for (int t = 0; t < TM; ++t) {
                acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x2[t], bv[0], acc[t][0], 0, 0, 0);
                acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(y[t], bv[1], acc[t][1], 0, 0, 0);
                acc[t][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(z[t], bv[2], acc[t][2], 0, 0, 0);
            }
            bv[0] = pb[0];
            bv[1] = pb[xs];
            bv[2] = pb[2 * xs];
            pb += kStepRows;
            if (++since_flush >= a.flush) {
                since_flush = 0;
                flush_acc<TM, true>(acc, ks, kc);
            }
        };
        // KC is a multiple of 8, so every chunk starts on an even step.  Steps
        // run in unconditional pairs, so the compiler sees both W' buffers in
        // flight at the loop head: a step past kmax has S(k) = 0 (staged zero)
        // and adds nothing, and its W' loads stay inside the zero tail rows.
        for (int s0 = 0; s0 < kc_n; s0 += 8) {
            step(s0, bA);
            step(s0 + 4, bB);
        }
    }
    flush_acc<TM, true>(acc, ks, kc);
    store_xi<TM>(a, grp, d, A0, lane, ks, kc);
}

// ---------------------------------------------------------------------------
// float32 matrix-core form on 4 x 4 x 1 blocks (v_mfma_f32_4x4x1f32, sixteen
// independent blocks per instruction), for masks of uneven lmax.
//
// The masks are sorted by lmax (descending) and taken four at a time: an
// instruction multiplies, for one l3, the A values of 64 pairs (one per lane,
// block b = lane / 4 holding the pairs of lanes 4b .. 4b + 3) by the W' of four
// masks (B: lane 4b + j holds mask j of the tile), and block b's 4 x 4
// accumulator holds (pair of lane 4b + i, mask j) in register i of lane
// 4b + j.  A work item is (diagonal d, R * 64 consecutive l1, end-aligned as in
// the strip kernels); it runs one pass over k per tile of four masks, for the
// tiles whose largest lmax reaches the block (the masks are a sorted prefix),
// each pass only up to that tile's largest lmax.  So the contraction carries at
// most three idle mask columns, instead of up to fifteen in a 16-mask tile.
// Per pass and step a lane generates its R pairs' A values on the VALU as the
// strip kernels do (g / h register windows, N' = Q + D (2T + D) expanded about
// each split) and issues 3 R MFMAs; the W' of its mask comes from the
// L2-resident table as one aligned float4 per four steps, a group ahead.
constexpr int kChunk4 = 256;                 // k staged per chunk
constexpr int kRebase4 = 128;                // steps per exact split of N'
constexpr int kMaxMasks = kMaxGroups * kGroup;

struct Batch4Args {
    int n_masks;                             // sorted by lmax, descending
    int n_masks4;                            // rounded up to a multiple of 4
    int L0;                                  // largest lmax
    int lmax[kMaxMasks];
    long long xi_off[kMaxMasks];             // Xi store [3][tri(lmax)] of each mask (doubles)
    const double* g;                         // float64 g(p)
    const float* gf;                         // float32 g(p)
    const float* hf;                         // float32 1/((2p+1) g(p))
    const double* cl;
    const float* wtab;                       // [3][n_masks4][2][jn] float32, W'_x,m(p + 2j)
    int jn;                                  // j slots per (x, m, p), a multiple of 4
    double* xi;
    int g_len, h_len;
    int flush;                               // 16-step groups per accumulator flush
};

template <int R, int KC>
struct Win4 {
    static constexpr int kB = kBThreads * R;
    static constexpr int kLen = kB + KC - 1;
    static constexpr int kPhys = kLen + kLen / R + 1;   // one padding word per R entries
    __device__ static inline int phys(int slot) { return slot + slot / R; }
};

// Work item -> (d, A) over the triangle of the largest lmax L: blocks of B
// rows aligned to each diagonal's last row, numbered longest first (the
// closed form of the strip kernels).  False: the item has no block.
template <int B>
__device__ inline bool decode_tri(int L, int item, int* d_out, int* A_out) {
    int m = (int)((sqrtf(8.0f * (float)item / (float)B + 1.0f) - 1.0f) * 0.5f);
    while (B * (m + 1) * (m + 2) / 2 <= item) ++m;
    while (m > 0 && B * m * (m + 1) / 2 > item) --m;
    const int rem = item - B * m * (m + 1) / 2;
    const int j = rem / B;
    const int d = B * (m - j) + (rem - B * j);
    const int n_valid = L - d + 1;
    if (d > L || n_valid <= B * j) return false;
    *d_out = d;
    *A_out = n_valid - B * (j + 1);
    return true;
}

// Xi of one tile: lane 4b + j holds mask 4t + j; accumulator r, register i is
// the pair l1 = A + R (4b + i) + r.  s = c_l1 c_l2 / 2 (App. B.3) in float64.
template <int R>
__device__ inline void store_xi4(const Batch4Args& a, int t, int d, int A, int lane, const float (&ks)[R][3][4],
                                 const float (&kc)[R][3][4]) {
    const int m = 4 * t + (lane & 3), b = lane >> 2;
    if (m >= a.n_masks) return;
    const int lm = a.lmax[m];
    if (lm < d) return;
    double* xi = a.xi + a.xi_off[m];
    const long long tri = tri_size(lm);
    const long long off = diag_offset(lm, d);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int l1 = A + R * (4 * b + i) + r;
            if (l1 >= 0 && l1 <= lm - d) {
                const double sp = 0.5 * a.cl[l1] * a.cl[l1 + d];
                const long long idx = off + l1;
                xi[idx] = (double)ks[r][0][i] - (double)kc[r][0][i];
                xi[tri + idx] = sp * ((double)ks[r][1][i] - (double)kc[r][1][i]);
                xi[2 * tri + idx] = (sp * sp) * ((double)ks[r][2][i] - (double)kc[r][2][i]);
            }
        }
}

// acc += a * (B operand of lane group g, broadcast to all four groups): the
// MFMA's B lane-group pattern 4 + g (an immediate; g is a constant once the
// step loop is unrolled).
__device__ inline f4v mfma4_bgroup(float av, float bv, f4v c, int g) {
    switch (g) {
    case 0: return __builtin_amdgcn_mfma_f32_4x4x1f32(av, bv, c, 0, 0, 4);
    case 1: return __builtin_amdgcn_mfma_f32_4x4x1f32(av, bv, c, 0, 0, 5);
    case 2: return __builtin_amdgcn_mfma_f32_4x4x1f32(av, bv, c, 0, 0, 6);
    default: return __builtin_amdgcn_mfma_f32_4x4x1f32(av, bv, c, 0, 0, 7);
    }
}

// Waves per SIMD the register allocation is held to (no spills; the
// accumulators share the unified register file).
template <int R>
constexpr int kF32x4Waves = 2;

// LDS of one work item of the 4 x 4 form.
template <int R>
struct Lds4 {
    using W = Win4<R, kChunk4>;
    float g[W::kPhys];
    float h[W::kPhys];
    float2 sd[kChunk4];                      // S(k) = g(k) g(d+k), D(k) = c(l3) - c(expansion point)
};

// One pass of a work item over k for NT consecutive tiles t0 .. t0 + NT - 1 of
// four masks: the A values of the lane's R rows are generated once per step and
// contracted against the W' of all NT tiles (3 R NT MFMAs per step).
template <int R, int NT>
__device__ inline void pass4(const Batch4Args& a, Lds4<R>& L, int d, int A, int t0, int kmax, int k_org,
                             int lane) {
    constexpr int KC = kChunk4;
    constexpr int RB = kRebase4;
    using W = Win4<R, KC>;
    constexpr int B = W::kB;
    constexpr int NW = (W::kLen + kBThreads - 1) / kBThreads;   // window entries staged per lane
    constexpr int NK = KC / kBThreads;                           // steps staged per lane
    const int l1_0 = A + R * lane;
    const int p = d & 1, jd = (d - p) >> 1;
    const long long xs4 = (long long)a.n_masks4 * 2 * a.jn / 4;   // float4 stride between spectra
    const long long ts4 = 2LL * a.jn;                             // float4 stride between tiles (4 masks)
    // W' of mask 4t + (lane & 3): lane group g = lane / 16 loads steps 4g .. 4g + 3 of
    // every 16-step group; step 4g + c of the group is component c, broadcast from
    // lane group g to the whole wave by the MFMA's B lane-group pattern 4 + g
    const f4v* pb = reinterpret_cast<const f4v*>(
        a.wtab + ((long long)(4 * t0 + (lane & 3)) * 2 + p) * a.jn + (jd + k_org) + 4 * (lane >> 4));
    f4v acc[NT][R][3];
    float ks[NT][R][3][4], kc[NT][R][3][4];
    float gw[R], hw[R], qf[R], rf[R];
    int tq[R];
    long long q64[R];
    // N' is expanded about each split's first step; the first split's steps
    // k_org .. -1 only pad the W' alignment (S = 0), so its expansion point is
    // k = 0, the first real step (about k_org, Q would exceed N' by up to
    // ~60x for l1 = 2 rows and its rounding would show in N')
    int c_cur = d * (d + 1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                acc[u][r][x] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int i = 0; i < 4; ++i) ks[u][r][x][i] = kc[u][r][x][i] = 0.0f;
            }
        const long long l1 = l1_0 + r, l2 = l1 + d;
        const long long aa = l1 * (l1 + 1), bb = l2 * (l2 + 1);
        const long long tt = (long long)c_cur - (aa + bb - 1);
        tq[r] = (int)tt;
        q64[r] = tt * tt - (2 * aa * bb + 1);
        qf[r] = rf[r] = 0.0f;
    }
    // two W' buffers per tile: even groups use bA, odd groups bB; each is refilled
    // for the group two ahead right after its use, so a load has a group to land
    f4v bA[NT][3], bB[NT][3];
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            bA[u][x] = pb[u * ts4 + x * xs4];
            bB[u][x] = pb[u * ts4 + x * xs4 + 4];
        }
    pb += 8;
    int since_flush = 0;

    // one 16-step group: A values on the VALU, 3 R NT MFMAs per step
    auto group = [&](const float* pg, const float* ph, int sb, const f4v (&bc)[NT][3]) {
#pragma unroll
        for (int wg = 0; wg < 16 / R; ++wg, pg -= R + 1, ph += R + 1) {
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int st = wg * R + u;                 // step within the 16-step group
#pragma unroll
                for (int j = R - 1; j > 0; --j) gw[j] = gw[j - 1];
                gw[0] = pg[-u];
#pragma unroll
                for (int j = 0; j < R - 1; ++j) hw[j] = hw[j + 1];
                hw[R - 1] = ph[u + (u >= 1 ? 1 : 0)];
                const float2 sd = L.sd[sb + st];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float x2 = sd.x * (gw[r] * hw[r]);
                    const float N = __builtin_fmaf(sd.y, rf[r] + sd.y, qf[r]);
                    const float y = x2 * N;
                    const float z = y * N;
#pragma unroll
                    for (int v = 0; v < NT; ++v) {
                        acc[v][r][0] = mfma4_bgroup(x2, bc[v][0][st & 3], acc[v][r][0], st >> 2);
                        acc[v][r][1] = mfma4_bgroup(y, bc[v][1][st & 3], acc[v][r][1], st >> 2);
                        acc[v][r][2] = mfma4_bgroup(z, bc[v][2][st & 3], acc[v][r][2], st >> 2);
                    }
                }
            }
        }
        if (++since_flush >= a.flush) {
            since_flush = 0;
#pragma unroll
            for (int v = 0; v < NT; ++v) flush_acc<R, true>(acc[v], ks[v], kc[v]);
        }
    };

    // Chunk staging: every global load of a chunk is issued before its first LDS store.
    // (Issuing the next chunk's loads before a chunk's steps, into registers, was
    // measured no faster and spills at two rows per lane.)
    //   windows: g(e), e = A - k0 - KC + 1 + slot, slots KC - kc_r .. kLen - 1;
    //            h(e), e = A + d + k0 + slot, slots 0 .. B + kc_r - 2;
    //   per step: S(k) = g(k) g(d+k) (0 past kmax) and D(k).
    float gv[NW], hv[NW];
    double ga[NK], gb[NK];
    auto load_chunk = [&](int k0) {
        const int kc_r = (min(KC, kmax - k0 + 1) + 31) / 32 * 32;
        const int g_base = A - k0 - KC + 1, h_base = A + d + k0, g_off = KC - kc_r;
        const int n_win = B + kc_r - 1;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int i = lane + q * kBThreads;
            const int eg = g_base + g_off + i, eh = h_base + i;
            gv[q] = (i < n_win && eg >= 0 && eg < a.g_len) ? a.gf[eg] : 0.0f;
            hv[q] = (i < n_win && eh >= 0 && eh < a.h_len) ? a.hf[eh] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < NK; ++q) {
            const int k = k0 + lane + q * kBThreads;
            const bool ok = k >= 0 && k <= kmax;
            ga[q] = ok ? a.g[k] : 0.0;
            gb[q] = ok ? a.g[d + k] : 0.0;
        }
    };
    auto store_chunk = [&](int k0) {
        const int kc_r = (min(KC, kmax - k0 + 1) + 31) / 32 * 32;
        const int g_off = KC - kc_r, n_win = B + kc_r - 1;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int i = lane + q * kBThreads;
            if (i < n_win) {
                L.g[W::phys(g_off + i)] = gv[q];
                L.h[W::phys(i)] = hv[q];
            }
        }
#pragma unroll
        for (int q = 0; q < NK; ++q) {
            const int s = lane + q * kBThreads;
            const int k = k0 + s;
            const int l3 = d + 2 * k;
            const int l3c = d + 2 * max(k0 + s / RB * RB, 0);   // this step's expansion point
            if (s < kc_r) L.sd[s] = float2{(float)(ga[q] * gb[q]), (float)(l3 * (l3 + 1) - l3c * (l3c + 1))};
        }
    };
    for (int k0 = k_org; k0 <= kmax; k0 += KC) {
        const int kc_n = min(KC, kmax - k0 + 1);
        const int kc_r = (kc_n + 31) / 32 * 32;   // whole pairs of 16-step groups; S = 0 past kmax
        __syncthreads();
        load_chunk(k0);
        store_chunk(k0);
        __syncthreads();
        if (k0 == k_org) {
#pragma unroll
            for (int j = 0; j < R - 1; ++j) gw[j] = L.g[W::phys(R * lane + j + KC)];
            gw[R - 1] = 0.0f;
            hw[0] = 0.0f;
#pragma unroll
            for (int j = 1; j < R; ++j) hw[j] = L.h[W::phys(R * lane + j - 1)];
        }
        const float* pg = L.g + (R + 1) * (lane + KC / R - 1) + (R - 1);
        const float* ph = L.h + (R + 1) * lane + (R - 1);
        for (int sb = 0; sb < kc_r; sb += 32, pg -= 32 / R * (R + 1), ph += 32 / R * (R + 1)) {
            if (sb % RB == 0) {
                // (T, Q) moved to this split's expansion point c_s exactly: Q(c + D) = Q + D T + D (T + D)
                const int l3c = d + 2 * max(k0 + sb, 0);
                const int cc = l3c * (l3c + 1);
                const int Ds = cc - c_cur;
                c_cur = cc;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    q64[r] += (long long)Ds * tq[r];
                    tq[r] += Ds;
                    q64[r] += (long long)Ds * tq[r];
                    qf[r] = (float)(double)q64[r];
                    rf[r] = 2.0f * (float)tq[r];
                }
            }
            // the refills are pinned between the groups (the scheduler would sink
            // them to their next use and expose the load latency)
            group(pg, ph, sb, bA);
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int x = 0; x < 3; ++x) bA[u][x] = pb[u * ts4 + x * xs4];
            __builtin_amdgcn_sched_barrier(0);
            group(pg - 16 / R * (R + 1), ph + 16 / R * (R + 1), sb + 16, bB);
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int x = 0; x < 3; ++x) bB[u][x] = pb[u * ts4 + x * xs4 + 4];
            __builtin_amdgcn_sched_barrier(0);
            pb += 8;
        }
    }
#pragma unroll
    for (int v = 0; v < NT; ++v) {
        flush_acc<R, true>(acc[v], ks[v], kc[v]);
        store_xi4<R>(a, t0 + v, d, A, lane, ks[v], kc[v]);
    }
}

template <int R, int NT>
__global__ void __launch_bounds__(kBThreads) __attribute__((amdgpu_waves_per_eu(kF32x4Waves<R>, 8)))
batched_mfma4_f32_kernel(Batch4Args a) {
    static_assert(16 % R == 0, "window groups of R steps tile the 16-step W' groups");
    static_assert(kChunk4 % kRebase4 == 0 && kRebase4 % 32 == 0, "chunks hold whole splits and pairs of W' groups");
    constexpr int B = kBThreads * R;
    __shared__ Lds4<R> L;
    int d, A;
    if (!decode_tri<B>(a.L0, blockIdx.x, &d, &A)) return;
    const int lane = threadIdx.x;
    const int row_min = max(A, 0);
    // masks whose lmax reaches a row of the block: a prefix of the sorted list
    int n_act = 0;
    while (n_act < a.n_masks && a.lmax[n_act] >= row_min + d) ++n_act;
    // k origin shifted so that j = (l3 - p)/2 of the first step is a multiple of 4
    const int jd = (d - (d & 1)) >> 1;
    const int k_org = -(jd & 3);
    const int n_tiles = (n_act + 3) / 4;
    int t = 0;
    // tiles in pairs while two remain (one A generation feeds both), then singly;
    // a pass runs to its first tile's largest lmax
    if (NT == 2)
        for (; t + 2 <= n_tiles; t += 2) pass4<R, 2>(a, L, d, A, t, min(A + B - 1, a.lmax[4 * t] - d), k_org, lane);
    for (; t < n_tiles; ++t) pass4<R, 1>(a, L, d, A, t, min(A + B - 1, a.lmax[4 * t] - d), k_org, lane);
}

// ---------------------------------------------------------------------------
// BF16x3 matrix-core form: steps of 32 k, lane k offsets 8q .. 8q + 7.
//
// The k origin is shifted so that j = (l3 - p) / 2 (p = d mod 2) of every
// lane's first k is a multiple of 8: the W' table per group is
// [3][2 pieces (hi, lo)][2 parities][16 masks][wt_len j slots] bfloat16, and
// a lane's 8 values of one (spectrum, piece) are one aligned 16-byte load.
// k < 0 and k > kmax contribute 0 through S(k) = 0.

// v -> (hi, lo) bfloat16 with hi = RN(v), lo = RN(v - hi): 8 values, packed
// two at a time by v_cvt_pk_bf16_f32; float(hi) is read back from the packed
// bits (a byte permute moves the low half up, a mask keeps the high half).
__device__ inline void split_bf16(const float (&v)[8], bf8v& hi, bf8v& lo) {
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        const bf2v h = {(__bf16)v[e], (__bf16)v[e + 1]};
        const unsigned hb = __builtin_bit_cast(unsigned, h);
        // bytes [hb.1, hb.0, 0, 0]: selector 1 / 0 pick bytes of the second operand, 0x0c gives 0
        const float f0 = __builtin_bit_cast(float, __builtin_amdgcn_perm(0u, hb, 0x01000c0cu));
        const float f1 = __builtin_bit_cast(float, hb & 0xffff0000u);
        const bf2v l = {(__bf16)(v[e] - f0), (__bf16)(v[e + 1] - f1)};
        hi[e] = h[0];
        hi[e + 1] = h[1];
        lo[e] = l[0];
        lo[e + 1] = l[1];
    }
}

struct BTile {
    bf8v v[3][2];    // [spectrum][hi, lo]
};

template <int TM>
__global__ void __launch_bounds__(kBThreads) __attribute__((amdgpu_waves_per_eu(kBF16Waves<TM>, 8)))
batched_mfma_bf16x3_kernel(BatchArgs a) {
    constexpr int KC = kChunkBF16;  // a multiple of two steps of 32 k
    using W = BWin<TM, KC>;
    __shared__ float s_g[W::kLen];
    __shared__ float s_h[W::kLen];
    __shared__ __attribute__((aligned(16))) float s_s[KC];
    __shared__ __attribute__((aligned(16))) float s_dc[KC];

    int grp, b, d;
    decode_item<TM>(a, blockIdx.x, &grp, &b, &d);
    const int L = a.L[grp];
    const int A0 = W::kRows * b;
    const int n_valid = L - d + 1;
    const int kmax = min(A0 + W::kRows, n_valid) - 1;

    const int lane = threadIdx.x;
    const int r = lane & 15, q = lane >> 4;
    const int p = d & 1, jd = (d - p) >> 1;
    const int k_org = -(jd & 7);                 // first k: j = jd + k_org is a multiple of 8
    const int jn = a.wt_len[grp];                // a multiple of 8
    const __bf16* base = static_cast<const __bf16*>(a.wtab) + a.wt_off[grp] +
                         (long long)(p * kGroup + r) * jn + (jd + k_org) + 8 * q;
    const u4v* pb = reinterpret_cast<const u4v*>(base);
    const long long xpv = 2LL * kGroup * jn / 8;  // stride between (spectrum, piece) blocks, 16-byte units

    auto load_b = [&](BTile& bt) {
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int h = 0; h < 2; ++h) bt.v[x][h] = __builtin_bit_cast(bf8v, pb[(2 * x + h) * xpv]);
        pb += 4;                                  // 32 j
    };

    int gam[TM];
    long long beta[TM];
    row_constants<TM>(A0, d, r, gam, beta);
    f4v acc[TM][3];
    float ks[TM][3][4], kc[TM][3][4];
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            acc[t][x] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < 4; ++i) ks[t][x][i] = kc[t][x][i] = 0.0f;
        }

    // one W' buffer, refilled for the next step right after the step's MFMAs
    // have read it (the next step's A generation covers the load)
    BTile bt;
    load_b(bt);

    int since_flush = 0;
    for (int kch = k_org; kch <= kmax; kch += KC) {
        __syncthreads();
        stage_chunk<TM, KC>(a, s_g, s_h, s_s, s_dc, A0, d, kch, kmax, lane);
        float qf[TM], rf[TM];
        chunk_expansion<TM>(d + 2 * max(kch, 0), gam, beta, qf, rf);
        __syncthreads();
        const int g_base = A0 - kch - KC - 3;

        auto step = [&](int s0, BTile& bt) {
            const int sb = s0 + 8 * q;               // this lane's first k offset in the chunk
            float S[8], D[8];
            {
                const f4v s0v = *reinterpret_cast<const f4v*>(&s_s[sb]);
                const f4v s1v = *reinterpret_cast<const f4v*>(&s_s[sb + 4]);
                const f4v d0v = *reinterpret_cast<const f4v*>(&s_dc[sb]);
                const f4v d1v = *reinterpret_cast<const f4v*>(&s_dc[sb + 4]);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    S[e] = s0v[e];
                    S[e + 4] = s1v[e];
                    D[e] = d0v[e];
                    D[e + 4] = d1v[e];
                }
            }
#pragma unroll
            for (int t = 0; t < TM; ++t) {
                const int l1 = A0 + 16 * t + r;
                const float* pg = &s_g[l1 - (kch + sb) - g_base];
                const float* ph = &s_h[l1 - A0 + sb];
                // one spectrum at a time: x2, then y = x2 N', then z = y N', each
                // split and contracted (hi*hi, hi*lo, lo*hi) before the next
                float v[8], N[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    v[e] = S[e] * (pg[-e] * ph[e]);
                    N[e] = __builtin_fmaf(D[e], rf[t] + D[e], qf[t]);
                }
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    if (x > 0) {
#pragma unroll
                        for (int e = 0; e < 8; ++e) v[e] *= N[e];
                    }
                    bf8v ah, al;
                    split_bf16(v, ah, al);
                    acc[t][x] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bt.v[x][0], acc[t][x], 0, 0, 0);
                    acc[t][x] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bt.v[x][1], acc[t][x], 0, 0, 0);
                    acc[t][x] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bt.v[x][0], acc[t][x], 0, 0, 0);
                }
            }
            load_b(bt);
            if (++since_flush >= a.flush) {
                since_flush = 0;
                flush_acc<TM, false>(acc, ks, kc);
            }
        };
        // KC is a multiple of 64, so every chunk starts on an even step
        for (int s0 = 0; s0 < KC && kch + s0 <= kmax; s0 += 64) {
            step(s0, bt);
            if (kch + s0 + 32 <= kmax) step(s0 + 32, bt);
        }
    }
    flush_acc<TM, false>(acc, ks, kc);
    store_xi<TM>(a, grp, d, A0, lane, ks, kc);
}

// ---------------------------------------------------------------------------
// W' tables of every group, (2l+1) W_l / 4 pi rounded once from float64.
// W' table layouts (one per matrix-core form)
enum : int { kTabF32x16 = 0, kTabBF16 = 1, kTabF32x4 = 2 };

struct WPrepArgs {
    int n_groups;
    int layout;                     // kTabF32x16, kTabBF16 (per group) or kTabF32x4 (all masks, in [0])
    int wt_len[kMaxGroups];         // x16: rows per group; BF16x3: j slots per group; x4: j slots (in [0])
    long long wt_off[kMaxGroups];
    long long n_elem[kMaxGroups];   // entries (x16, x4) or BF16x3 (spectrum, parity, mask, j) slots
    int n_masks[kMaxGroups];
    int lmax[kMaxGroups][kGroup];
    const double* w[kMaxGroups][3][kGroup];
    void* wtab;
};

constexpr double kInv4PiB = 0.079577471545947667884441881686257181;

__device__ inline double wprime(const WPrepArgs& a, int grp, int x, int m, int l) {
    if (m >= a.n_masks[grp] || l > 2 * a.lmax[grp][m] || !a.w[grp][x][m]) return 0.0;
    return a.w[grp][x][m][l] * ((2.0 * l + 1.0) * kInv4PiB);
}

__global__ void batched_wprep_kernel(WPrepArgs a) {
    const int grp = blockIdx.y;
    if (grp >= a.n_groups) return;
    if (a.layout == kTabF32x4 && grp > 0) return;   // that table covers every mask at once
    const int len = a.wt_len[grp];
    const int n4 = (a.n_groups * kGroup);    // mask slots of the x4 table (sorted order)
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < a.n_elem[grp];
         e += (long long)gridDim.x * blockDim.x) {
        if (a.layout == kTabF32x16) {
            // per group [x][l3][m]
            const int x = (int)(e / ((long long)len * kGroup));
            const int rem = (int)(e % ((long long)len * kGroup));
            const int l = rem / kGroup, m = rem % kGroup;
            static_cast<float*>(a.wtab)[a.wt_off[grp] + e] = (float)wprime(a, grp, x, m, l);
        } else if (a.layout == kTabF32x4) {
            // [x][mask][p][j], l3 = p + 2 j; mask mi = 16 group + index in the group
            const int j = (int)(e % len);
            const long long rest = e / len;
            const int pp = (int)(rest % 2);
            const int mi = (int)((rest / 2) % n4);
            const int x = (int)(rest / (2LL * n4));
            static_cast<float*>(a.wtab)[e] = (float)wprime(a, mi / kGroup, x, mi % kGroup, pp + 2 * j);
        } else {
            // slot e = ((x * 2 + p) * 16 + m) * len + j, l3 = p + 2 j; pieces hi / lo
            // go to blocks 2x and 2x + 1 of [6][2][16][len]
            const int j = (int)(e % len);
            const long long rest = e / len;
            const int m = (int)(rest % kGroup);
            const int p = (int)((rest / kGroup) % 2);
            const int x = (int)(rest / (2 * kGroup));
            const float v = (float)wprime(a, grp, x, m, p + 2 * j);
            const __bf16 hi = (__bf16)v;
            const __bf16 lo = (__bf16)(v - (float)hi);
            __bf16* t = static_cast<__bf16*>(a.wtab) + a.wt_off[grp];
            const long long inner = ((long long)p * kGroup + m) * len + j;
            const long long blk = 2LL * kGroup * len;
            t[(2LL * x) * blk + inner] = hi;
            t[(2LL * x + 1) * blk + inner] = lo;
        }
    }
}

// Table geometry.  float32, 16-mask form: per group of largest lmax L, rows l3 of 16 masks.
inline int f32_rows(int L) { return 2 * L + 1 + kF32TailRows; }
inline size_t f32_table_elems(int L) { return 3ULL * (size_t)f32_rows(L) * kGroup; }
// float32, 4-mask form: a pass runs n groups of 16 steps from j = jd + k_org,
// n <= (kmax - k_org + 32) / 16 (pairs of groups), and loads the two groups after
// its last, so it reads j < jd + k_org + 16 (n + 2) <= jd + kmax + 64 <= L0 + 64
// (jd + kmax <= d/2 + L0 - d); j slots L0 + 64 rounded up to 4, for every mask
// slot of the groups.
inline int f32x4_slots(int L0) { return ((L0 + 64 + 3) / 4) * 4; }
inline size_t f32x4_table_elems(int L0, int n_groups) {
    return 3ULL * (size_t)(n_groups * kGroup) * 2 * (size_t)f32x4_slots(L0);
}
// Tile settings (row_tiles) of the two float32 forms: 1, 2, 4 = 16-row tiles of the
// 16-mask form; 64, 128 = rows per wavefront of the 4-mask form.
inline bool f32x4_tiles(int tm) { return tm == 64 || tm == 128; }
// A wavefront's last executed step starts at j <= jd + kmax <= L ((l3 - p) / 2 for
// l3 <= 2L) and it has loaded the step after it: j <= L + 63.  A multiple of 8.
inline int bf16_slots(int L) { return ((L + 64 + 7) / 8) * 8; }
inline size_t bf16_table_elems(int L) { return 3ULL * 2 * 2 * kGroup * (size_t)bf16_slots(L); }

}  // namespace

size_t batched_workspace_bytes(const BatchPlan& p) {
    size_t xi = 0, bf = 0, f32_16 = 0;
    for (int gi = 0; gi < p.n_groups; ++gi) {
        for (int m = 0; m < p.n_masks[gi]; ++m) xi += 3ULL * (size_t)tri_size(p.lmax[gi][m]);
        bf += bf16_table_elems(p.L[gi]);
        f32_16 += f32_table_elems(p.L[gi]);
    }
    const size_t f32 = std::max(f32_16, p.n_groups > 0 ? f32x4_table_elems(p.L[0], p.n_groups) : 0);
    // Xi (float64), then one 256-byte aligned W' table region large enough for either form
    const size_t tab = std::max(f32 * sizeof(float), bf * sizeof(__bf16));
    return xi * sizeof(double) + tab + 256;
}

hipError_t launch_batched(couple_ctx* ctx, const BatchPlan& p, int precision, const int* spec_src, int n_out,
                          int xi_only, hipStream_t s) {
    const bool bf16 = precision == COUPLE_MFMA_BF16X3;
    const bool x4 = !bf16 && f32x4_tiles(p.tm);
    const int layout = bf16 ? kTabBF16 : (x4 ? kTabF32x4 : kTabF32x16);
    double* xi = reinterpret_cast<double*>(ctx->bws);
    long long xi_off[kMaxGroups][kGroup];
    size_t xi_doubles = 0;
    for (int gi = 0; gi < kMaxGroups; ++gi)
        for (int m = 0; m < kGroup; ++m) {
            xi_off[gi][m] = (long long)xi_doubles;
            if (gi < p.n_groups && m < p.n_masks[gi]) xi_doubles += 3ULL * (size_t)tri_size(p.lmax[gi][m]);
        }
    void* wtab = reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(xi + xi_doubles) + 255) &
                                         ~static_cast<uintptr_t>(255));
    long long wt_off[kMaxGroups];
    int wt_len[kMaxGroups];
    long long off = 0;
    for (int gi = 0; gi < p.n_groups; ++gi) {
        wt_off[gi] = off;
        wt_len[gi] = bf16 ? bf16_slots(p.L[gi]) : (x4 ? f32x4_slots(p.L[0]) : f32_rows(p.L[gi]));
        off += (long long)(bf16 ? bf16_table_elems(p.L[gi]) : f32_table_elems(p.L[gi]));
    }

    // W' tables
    {
        WPrepArgs w;
        w.n_groups = p.n_groups;
        w.layout = layout;
        w.wtab = wtab;
        for (int gi = 0; gi < p.n_groups; ++gi) {
            w.wt_len[gi] = wt_len[gi];
            w.wt_off[gi] = wt_off[gi];
            w.n_elem[gi] = bf16 ? 3LL * 2 * kGroup * wt_len[gi]
                                : (x4 ? (long long)f32x4_table_elems(p.L[0], p.n_groups)
                                      : (long long)f32_table_elems(p.L[gi]));
            w.n_masks[gi] = p.n_masks[gi];
            for (int m = 0; m < kGroup; ++m) {
                w.lmax[gi][m] = m < p.n_masks[gi] ? p.lmax[gi][m] : -1;
                for (int x = 0; x < 3; ++x) w.w[gi][x][m] = m < p.n_masks[gi] ? p.w[gi][x][m] : nullptr;
            }
        }
        prof_begin(ctx, s);
        hipLaunchKernelGGL(batched_wprep_kernel, dim3(256, p.n_groups), dim3(256), 0, s, w);
        prof_end(ctx, s, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // contraction, float32 4-mask form: one launch over the triangle of the largest lmax
    if (x4) {
        Batch4Args a;
        a.n_masks = 0;
        for (int gi = 0; gi < p.n_groups; ++gi)
            for (int m = 0; m < p.n_masks[gi]; ++m) {
                a.lmax[a.n_masks] = p.lmax[gi][m];
                a.xi_off[a.n_masks] = xi_off[gi][m];
                ++a.n_masks;
            }
        for (int m = a.n_masks; m < kMaxMasks; ++m) {
            a.lmax[m] = -1;
            a.xi_off[m] = 0;
        }
        a.n_masks4 = p.n_groups * kGroup;
        a.L0 = p.L[0];
        a.g = ctx->g_pad + kTablePad;
        a.gf = ctx->gf_pad + kTablePad;
        a.hf = ctx->hf_pad + kTablePad;
        a.cl = ctx->cl;
        a.wtab = static_cast<const float*>(wtab);
        a.jn = f32x4_slots(a.L0);
        a.xi = xi;
        a.g_len = ctx->lmax_max + 1;
        a.h_len = 2 * ctx->lmax_max + 1;
        a.flush = p.flush > 0 ? p.flush : 1;
        // row_tiles 64: one row per lane, tiles of masks in pairs; 128: two rows per
        // lane, one tile per pass.  Work items over the triangle of L0.
        const int R = p.tm == 64 ? 1 : 2;
        const long long B = (long long)kBThreads * R;
        const long long M = a.L0 / B;
        const long long total = B * (M + 1) * (M + 2) / 2;
        prof_begin(ctx, s);
        if (R == 1)
            hipLaunchKernelGGL((batched_mfma4_f32_kernel<1, 2>), dim3((unsigned)total), dim3(kBThreads), 0, s, a);
        else
            hipLaunchKernelGGL((batched_mfma4_f32_kernel<2, 1>), dim3((unsigned)total), dim3(kBThreads), 0, s, a);
        prof_end(ctx, s, 1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // contraction, 16-mask forms (float32, BF16x3): groups of 16 masks
    auto contract = [&](auto tm_tag) -> hipError_t {
        constexpr int TM = decltype(tm_tag)::value;
        BatchArgs a;
        a.n_groups = p.n_groups;
        long long total = 0;
        for (int gi = 0; gi < p.n_groups; ++gi) {
            const int L = p.L[gi];
            const int B = 16 * TM;
            a.L[gi] = L;
            a.bmax[gi] = L / B;
            long long n = 0;
            for (int bb = a.bmax[gi]; bb >= 0; --bb) {
                const int nb = L - B * bb + 1;
                if (nb > 0) n += nb;
            }
            a.n_items[gi] = (int)n;
            total += n;
            a.wt_off[gi] = wt_off[gi];
            a.wt_len[gi] = wt_len[gi];
            for (int m = 0; m < kGroup; ++m) {
                a.lmax[gi][m] = m < p.n_masks[gi] ? p.lmax[gi][m] : -1;
                a.xi_off[gi][m] = xi_off[gi][m];
            }
        }
        a.g = ctx->g_pad + kTablePad;
        a.gf = ctx->gf_pad + kTablePad;
        a.hf = ctx->hf_pad + kTablePad;
        a.cl = ctx->cl;
        a.wtab = wtab;
        a.xi = xi;
        a.g_len = ctx->lmax_max + 1;
        a.h_len = 2 * ctx->lmax_max + 1;
        a.flush = p.flush > 0 ? p.flush : 1;
        prof_begin(ctx, s);
        if (bf16)
            hipLaunchKernelGGL(batched_mfma_bf16x3_kernel<TM>, dim3((unsigned)total), dim3(kBThreads), 0, s, a);
        else
            hipLaunchKernelGGL(batched_mfma_f32_kernel<TM>, dim3((unsigned)total), dim3(kBThreads), 0, s, a);
        prof_end(ctx, s, 1);
        return hipGetLastError();
    };
    if (!x4) {
        hipError_t e;
        if (p.tm == 1)
            e = contract(std::integral_constant<int, 1>());
        else if (p.tm == 4)
            e = contract(std::integral_constant<int, 4>());
        else
            e = contract(std::integral_constant<int, 2>());
        if (e != hipSuccess) return e;
    }
    // fill: one job per mask
    {
        FillJob jobs[kMaxFillJobs];
        int n_jobs = 0;
        for (int gi = 0; gi < p.n_groups; ++gi)
            for (int m = 0; m < p.n_masks[gi]; ++m) {
                FillJob& j = jobs[n_jobs++];
                j.xi = xi + xi_off[gi][m];
                j.xi_stride = tri_size(p.lmax[gi][m]);
                j.out = p.out[gi][m];
                j.lmax = p.lmax[gi][m];
                j.dmax = p.lmax[gi][m];
                j.block0 = 0;
            }
        prof_begin(ctx, s);
        hipError_t e = launch_fill_jobs(jobs, n_jobs, spec_src, n_out, xi_only, s);
        prof_end(ctx, s, 2);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace couple
