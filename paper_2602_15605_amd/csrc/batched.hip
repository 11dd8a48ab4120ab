// Batched form: many windows (masks) of uneven lmax in one launch.
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
//   * one wavefront owns a diagonal d and TM*16 consecutive l1 of a group; per
//     step of 4 k it generates its A elements on the VALU (one per lane and
//     row tile, the v_mfma_f32_16x16x4f32 operand layout: lane l holds row
//     l % 16, k offset l / 16) and issues 3*TM MFMAs against the W' tile
//     (k x 16 masks, lane l holds k offset l / 16, mask l % 16), loaded from
//     the L2-resident W' table two steps ahead of its use;
//   * every kFlush MFMA steps the float32 matrix-core accumulators are added
//     into Kahan (sum, compensation) pairs, which bounds the float32
//     accumulation error to a few ulp per block;
//   * Xi goes to a mask-interleaved packed triangle, Xi[d, l1][16], which the
//     output tile of the MFMA (lane l holds rows 4 (l/16) + i, mask l % 16)
//     writes in 128-byte rows.
// A fill pass then writes each mask's K (mask-major; columns beyond a mask's
// own lmax are not written).
#include <type_traits>

#include "couple_internal.hpp"

namespace couple {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kGroup = kMaskGroup;  // masks per MFMA column block
constexpr int kBChunk = 64;         // k steps staged per chunk (multiple of 4)
constexpr int kBThreads = 64;

struct BatchArgs {
    int n_groups;
    // per group
    int L[kMaxGroups];              // largest lmax in the group
    int n_items[kMaxGroups];        // work items of the group
    int bmax[kMaxGroups];
    long long xi_off[kMaxGroups];   // offset of the group's Xi (doubles)
    long long wt_off[kMaxGroups];   // offset of the group's W' table (floats)
    // shared
    const double* g;                // float64 g(p)
    const float* gf;                // float32 g(p)
    const float* hf;                // float32 1/((2p+1) g(p))
    const double* cl;
    const float* wtab;              // W' tables, [3][2L+1][16] per group
    double* xi;                     // Xi workspace base
    int g_len, h_len;
    int flush;                      // MFMA steps per Kahan flush
};

template <int TM>
struct BWin {
    static constexpr int kRows = 16 * TM;
    static constexpr int kLen = kRows + kBChunk + 3;
};

// Kahan step: (s, c) += v.
__device__ inline void kahan_add(float& s, float& c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

template <int TM>
__global__ void __launch_bounds__(kBThreads)
batched_mfma_f32_kernel(BatchArgs a) {
    using W = BWin<TM>;
    constexpr int KC = kBChunk;
    __shared__ float s_g[W::kLen];
    __shared__ float s_h[W::kLen];
    __shared__ float s_s[KC + 4];       // S(k) = g(k) g(d+k), float32
    __shared__ float s_dc[KC + 4];      // D(k) = c(k) - c(chunk start), exact in float32

    // ---- work item: group, then level b (descending), diagonal d ----
    int item = blockIdx.x;
    int grp = 0;
    while (grp < a.n_groups - 1 && item >= a.n_items[grp]) {
        item -= a.n_items[grp];
        ++grp;
    }
    const int L = a.L[grp];
    int b = a.bmax[grp];
    for (; b > 0; --b) {
        const int nb = L - W::kRows * b + 1;
        if (nb > 0) {
            if (item < nb) break;
            item -= nb;
        }
    }
    const int d = item;
    const int A0 = W::kRows * b;
    const int n_valid = L - d + 1;
    const int kmax = min(A0 + W::kRows, n_valid) - 1;

    const int lane = threadIdx.x;
    const int r = lane & 15, q = lane >> 4;
    const int wl = 2 * L + 1;
    // B operand: W'_X(l3)[mask r] with l3 = d + 2k, k = 4 step + q
    const float* wt = a.wtab + a.wt_off[grp] + r;
    const long long xs = (long long)wl * kGroup;    // stride between spectra

    int gam[TM];
    float beta[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
        const long long l1 = A0 + 16 * t + r, l2 = l1 + d;
        const long long aa = l1 * (l1 + 1), bb = l2 * (l2 + 1);
        gam[t] = (int)(aa + bb - 1);
        beta[t] = (float)(2.0 * (double)aa * (double)bb + 1.0);
    }
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

    const int n_steps = (kmax + 4) / 4;          // steps of 4 k
    // B prefetch two steps ahead (0 beyond the row or the window)
    auto load_b = [&](int step, float* bv) {
        const int l3 = d + 2 * (4 * step + q);
        const bool ok = step < n_steps && l3 < wl;
        const float* p = wt + (long long)l3 * kGroup;
        bv[0] = ok ? p[0] : 0.0f;
        bv[1] = ok ? p[xs] : 0.0f;
        bv[2] = ok ? p[2 * xs] : 0.0f;
    };
    float b0[3], b1[3];
    load_b(0, b0);
    load_b(1, b1);

    int since_flush = 0;
    for (int k0 = 0; k0 <= kmax; k0 += KC) {
        const int kc_n = min(KC, kmax - k0 + 1);
        __syncthreads();
        const int g_base = A0 - k0 - KC - 3;
        const int h_base = A0 + d + k0;
        for (int slot = lane; slot < W::kLen; slot += kBThreads) {
            const int eg = g_base + slot, eh = h_base + slot;
            s_g[slot] = (eg >= 0 && eg < a.g_len) ? a.gf[eg] : 0.0f;
            s_h[slot] = (eh >= 0 && eh < a.h_len) ? a.hf[eh] : 0.0f;
        }
        const int l3c = d + 2 * k0;
        for (int s = lane; s < KC + 4; s += kBThreads) {
            float sv = 0.0f, dv = 0.0f;
            if (s < kc_n) {
                const int k = k0 + s;
                sv = (float)(a.g[k] * a.g[d + k]);
                const int l3 = d + 2 * k;
                dv = (float)(l3 * (l3 + 1) - l3c * (l3c + 1));
            }
            s_s[s] = sv;
            s_dc[s] = dv;
        }
        // t = T + D(k), T = c(d + 2 k0) - (a + b - 1) = T_hi + T_lo exactly
        float thi[TM], tlo[TM];
#pragma unroll
        for (int t = 0; t < TM; ++t) {
            const int T = l3c * (l3c + 1) - gam[t];
            thi[t] = (float)T;
            tlo[t] = (float)(T - (int)thi[t]);
        }
        __syncthreads();

        for (int s0 = 0; s0 < kc_n; s0 += 4) {
            const int s = s0 + q;                 // this lane's k offset in the chunk
            const float S = s_s[s];
            const float D = s_dc[s];
            const float btt = b0[0], btp = b0[1], bpp = b0[2];
            b0[0] = b1[0];
            b0[1] = b1[1];
            b0[2] = b1[2];
            load_b((k0 + s0) / 4 + 2, b1);
#pragma unroll
            for (int t = 0; t < TM; ++t) {
                const int l1 = A0 + 16 * t + r;
                const float gv = s_g[l1 - (k0 + s) - g_base];
                const float hv = s_h[l1 - A0 + s];
                const float x2 = S * (gv * hv);
                const float tt = thi[t] + (D + tlo[t]);
                const float N = __builtin_fmaf(tt, tt, -beta[t]);
                const float y = x2 * N;
                const float z = y * N;
                acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x2, btt, acc[t][0], 0, 0, 0);
                acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(y, btp, acc[t][1], 0, 0, 0);
                acc[t][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(z, bpp, acc[t][2], 0, 0, 0);
            }
            if (++since_flush >= a.flush) {
                since_flush = 0;
#pragma unroll
                for (int t = 0; t < TM; ++t)
#pragma unroll
                    for (int x = 0; x < 3; ++x) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) kahan_add(ks[t][x][i], kc[t][x][i], acc[t][x][i]);
                        acc[t][x] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
                    }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int i = 0; i < 4; ++i) kahan_add(ks[t][x][i], kc[t][x][i], acc[t][x][i]);

    // ---- store: lane holds rows 4q + i of each row tile, mask column r ----
    const long long tri = (long long)(L + 1) * (L + 2) / 2;
    double* xi = a.xi + a.xi_off[grp];
    const long long off = diag_offset(L, d);
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int l1 = A0 + 16 * t + 4 * q + i;
            if (l1 < n_valid) {
                const double sp = 0.5 * a.cl[l1] * a.cl[l1 + d];
                const long long idx = (off + l1) * kGroup + r;
                xi[idx] = (double)ks[t][0][i] - (double)kc[t][0][i];
                xi[tri * kGroup + idx] = sp * ((double)ks[t][1][i] - (double)kc[t][1][i]);
                xi[2 * tri * kGroup + idx] = (sp * sp) * ((double)ks[t][2][i] - (double)kc[t][2][i]);
            }
        }
}

// W' tables of every group: [3][2L+1][16] float32, (2l+1) W_l / 4 pi rounded once.
struct WPrepArgs {
    int n_groups;
    int L[kMaxGroups];
    long long wt_off[kMaxGroups];
    int n_masks[kMaxGroups];
    int lmax[kMaxGroups][kGroup];
    const double* w[kMaxGroups][3][kGroup];
    float* wtab;
};

constexpr double kInv4PiB = 0.079577471545947667884441881686257181;

__global__ void batched_wprep_kernel(WPrepArgs a) {
    const int grp = blockIdx.y;
    if (grp >= a.n_groups) return;
    const int wl = 2 * a.L[grp] + 1;
    float* wt = a.wtab + a.wt_off[grp];
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < 3LL * wl * kGroup;
         e += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(e / ((long long)wl * kGroup));
        const int rem = (int)(e % ((long long)wl * kGroup));
        const int l = rem / kGroup, m = rem % kGroup;
        float v = 0.0f;
        if (m < a.n_masks[grp] && l <= 2 * a.lmax[grp][m] && a.w[grp][x][m])
            v = (float)(a.w[grp][x][m][l] * ((2.0 * l + 1.0) * kInv4PiB));
        wt[e] = v;
    }
}

// K of every mask from the mask-interleaved Xi: one work-group per (group
// tile pair, mask); the tile is read diagonal by diagonal and written row by
// row and mirrored, as in fill_kernel.
struct BFillArgs {
    int n_groups;
    int L[kMaxGroups];
    long long xi_off[kMaxGroups];
    int n_masks[kMaxGroups];
    int lmax[kMaxGroups][kGroup];
    double* out[kMaxGroups][kGroup];
    int n_tiles[kMaxGroups];
    long long pair_base[kMaxGroups];    // first block index of the group
    const double* xi;
    int n_out;
    int src[4];
};

constexpr int kT = 64;

__global__ void __launch_bounds__(256) batched_fill_kernel(BFillArgs a) {
    __shared__ double tile[kT][kT + 1];
    long long blk = blockIdx.x;
    int grp = 0;
    while (grp < a.n_groups - 1 && blk >= a.pair_base[grp + 1]) ++grp;
    blk -= a.pair_base[grp];
    const int m = (int)(blk % kGroup);
    const int pair = (int)(blk / kGroup);
    if (m >= a.n_masks[grp]) return;
    const int lmax = a.lmax[grp][m];
    int I = 0, rem = pair;
    const int nt = a.n_tiles[grp];
    while (rem >= nt - I) {
        rem -= nt - I;
        ++I;
    }
    const int J = I + rem;
    const int r0 = kT * I, c0 = kT * J;
    if (r0 > lmax || c0 > lmax) return;
    const int L = a.L[grp];
    const long long tri = (long long)(L + 1) * (L + 2) / 2;
    const double* xi = a.xi + a.xi_off[grp];
    const int t = threadIdx.x;
    const long long ld = lmax + 1;
    int last_src = -1;
    for (int o = 0; o < a.n_out; ++o) {
        const int src = a.src[o];
        if (src != last_src) {
            __syncthreads();
            for (int idx = t; idx < (2 * kT - 1) * kT; idx += 256) {
                const int rr = idx % kT, dl = idx / kT;
                const int cc = rr + dl - (kT - 1);
                if (cc < 0 || cc >= kT) continue;
                const int l1 = r0 + rr, l2 = c0 + cc;
                if (l1 > lmax || l2 > lmax || l2 < l1) continue;
                tile[rr][cc] = xi[((long long)src * tri + diag_offset(L, l2 - l1) + l1) * kGroup + m];
            }
            __syncthreads();
            last_src = src;
        }
        double* out = a.out[grp][m] + (long long)o * ld * ld;
        if (I == J) {
            for (int idx = t; idx < kT * kT; idx += 256) {
                const int rr = idx / kT, cc = idx % kT;
                const int l1 = r0 + rr, l2 = c0 + cc;
                if (l1 > lmax || l2 > lmax) continue;
                out[l1 * ld + l2] = (2.0 * l2 + 1.0) * ((cc >= rr) ? tile[rr][cc] : tile[cc][rr]);
            }
        } else {
            for (int idx = t; idx < kT * kT; idx += 256) {
                const int rr = idx / kT, cc = idx % kT;
                const int l1 = r0 + rr, l2 = c0 + cc;
                if (l1 <= lmax && l2 <= lmax) out[l1 * ld + l2] = (2.0 * l2 + 1.0) * tile[rr][cc];
            }
            for (int idx = t; idx < kT * kT; idx += 256) {
                const int cc = idx / kT, rr = idx % kT;
                const int l1 = r0 + rr, l2 = c0 + cc;
                if (l1 <= lmax && l2 <= lmax) out[l2 * ld + l1] = (2.0 * l1 + 1.0) * tile[rr][cc];
            }
        }
    }
}

}  // namespace

size_t batched_workspace_bytes(const BatchPlan& p) {
    size_t doubles = 0, floats = 0;
    for (int gi = 0; gi < p.n_groups; ++gi) {
        const long long L = p.L[gi];
        doubles += 3ULL * (size_t)((L + 1) * (L + 2) / 2) * kGroup;
        floats += 3ULL * (size_t)(2 * L + 1) * kGroup;
    }
    return doubles * sizeof(double) + floats * sizeof(float) + 256;
}

hipError_t launch_batched(couple_ctx* ctx, const BatchPlan& p, int precision, const int* spec_src, int n_out,
                          hipStream_t s) {
    (void)precision;
    double* xi = reinterpret_cast<double*>(ctx->bws);
    size_t xi_doubles = 0;
    long long xi_off[kMaxGroups], wt_off[kMaxGroups];
    size_t wt_floats = 0;
    for (int gi = 0; gi < p.n_groups; ++gi) {
        const long long L = p.L[gi];
        xi_off[gi] = (long long)xi_doubles;
        xi_doubles += 3ULL * (size_t)((L + 1) * (L + 2) / 2) * kGroup;
    }
    for (int gi = 0; gi < p.n_groups; ++gi) {
        wt_off[gi] = (long long)wt_floats;
        wt_floats += 3ULL * (size_t)(2 * p.L[gi] + 1) * kGroup;
    }
    float* wtab = reinterpret_cast<float*>(xi + xi_doubles);

    // W' tables
    {
        WPrepArgs w;
        w.n_groups = p.n_groups;
        w.wtab = wtab;
        for (int gi = 0; gi < p.n_groups; ++gi) {
            w.L[gi] = p.L[gi];
            w.wt_off[gi] = wt_off[gi];
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
    // contraction
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
            a.xi_off[gi] = xi_off[gi];
            a.wt_off[gi] = wt_off[gi];
        }
        a.g = ctx->g_pad + kTablePad;
        a.gf = ctx->gf_pad + kTablePad;
        a.hf = ctx->hf_pad + kTablePad;
        a.cl = ctx->cl;
        a.wtab = wtab;
        a.xi = xi;
        a.g_len = ctx->lmax_max + 1;
        a.h_len = 2 * ctx->lmax_max + 1;
        a.flush = p.flush > 0 ? p.flush : 8;
        prof_begin(ctx, s);
        hipLaunchKernelGGL(batched_mfma_f32_kernel<TM>, dim3((unsigned)total), dim3(kBThreads), 0, s, a);
        prof_end(ctx, s, 1);
        return hipGetLastError();
    };
    {
        hipError_t e;
        if (p.tm == 1)
            e = contract(std::integral_constant<int, 1>());
        else if (p.tm == 4)
            e = contract(std::integral_constant<int, 4>());
        else
            e = contract(std::integral_constant<int, 2>());
        if (e != hipSuccess) return e;
    }
    // fill
    {
        BFillArgs f;
        f.n_groups = p.n_groups;
        f.xi = xi;
        f.n_out = n_out;
        for (int i = 0; i < 4; ++i) f.src[i] = i < n_out ? spec_src[i] : 0;
        long long base = 0;
        for (int gi = 0; gi < p.n_groups; ++gi) {
            f.L[gi] = p.L[gi];
            f.xi_off[gi] = xi_off[gi];
            f.n_masks[gi] = p.n_masks[gi];
            f.n_tiles[gi] = (p.L[gi] + kT) / kT;
            f.pair_base[gi] = base;
            base += (long long)f.n_tiles[gi] * (f.n_tiles[gi] + 1) / 2 * kGroup;
            for (int m = 0; m < kGroup; ++m) {
                f.lmax[gi][m] = m < p.n_masks[gi] ? p.lmax[gi][m] : -1;
                f.out[gi][m] = m < p.n_masks[gi] ? p.out[gi][m] : nullptr;
            }
        }
        for (int gi = p.n_groups; gi < kMaxGroups; ++gi) f.pair_base[gi] = base;
        prof_begin(ctx, s);
        hipLaunchKernelGGL(batched_fill_kernel, dim3((unsigned)base), dim3(256), 0, s, f);
        prof_end(ctx, s, 2);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace couple
