// The l3 reduction of the coupling kernels (Sec. 2 eqs. K_TT, K_EE; App. A)
// on the packed upper triangle Xi(l1, l1 + d), d >= 0.
//
// Per term, with l2 = l1 + d and l3 = d + 2k (k = 0 .. l1: even L only, so
// the parity projectors of App. A are structural), the halved triangle
// combinations of eq. trianglecombos are p1 = d + k, p2 = k, p3 = l1 - k and
// p = l1 + d + k.  From eq. 000_sq_main,
//
//     (l1 l2 l3; 0 0 0)^2 = g(p1) g(p2) g(p3) / ((2p+1) g(p))
//                         = [g(k) g(d+k)] * [g(l1-k) * h(l1+d+k)],
//
// with h(p) = 1/((2p+1) g(p)).  The first factor depends on (d, k) only and
// is folded, together with the scaled window W'_l3 = (2 l3 + 1) W_l3/(4 pi),
// into per-step constants U_X(k) shared by a whole wavefront; the second is
// a product of two table values that slide by one entry per step.
//
// The (-2 2 0) symbol.  The two-term closed form of App. B.3
// (eq. 022_linear_closedform), applied with (j1, j2, j3) = (l3, l1, l2) --
// the m = 0 column first, as the cyclic permutation of eq. permutation
// requires -- expresses (l1 l2 l3; -2 2 0) through (l1 l2 l3; 0 0 0) and
// (l1 l2+2 l3; 0 0 0).  The ratio of those two (0 0 0) symbols follows from
// eq. 000_sq_main and eq. g_rec (the same step as App. B.5), and with it the
// closed form collapses to a single multiple of the (0 0 0) symbol:
//
//     (l1 l2 l3; -2 2 0) = (l1 l2 l3; 0 0 0) * N' / (2 lambda eta),
//     N' = u (u - 2) - 2 a b,   u = a + b - c,
//     a = l1(l1+1), b = l2(l2+1), c = l3(l3+1),
//     lambda eta = sqrt(a (a-2) b (b-2)) = 1/(c_l1 c_l2).
//
// N' is an integer; here it is evaluated as N' = c (c - 2(a+b-1)) + a(a-2) + b(b-2)
// with one fused multiply-add, rounded once while a(a-2) + b(b-2) < 2^53
// (lmax <= 8000); beyond, that sum is not exact and N' cancels against it when
// l1 << l2, so N' = t^2 - (2ab+1), t = c - (a+b-1), with 2ab+1 split exactly
// into two doubles (see strip_fp64_kernel).  The
// "(2,-2,0) recurrence" is thus an integer update of c along the strip.  The
// three kernels then are
//
//     Xi_TT = sum_k U_TT(k) P,   Xi_TE = s sum_k U_TP(k) P N',
//     Xi_EE = s^2 sum_k U_PP(k) P N'^2,     P = g(l1-k) h(l1+d+k),  s = c_l1 c_l2 / 2,
//
// and s = 0 for l1 < 2 or l2 < 2, where the (-2 2 0) symbol vanishes.
//
// Odd L (the EB kernel of App. A, S^EB = (-2 2 0)^2 on odd L).  With
// (j1, j2, j3) = (l3, l1, l2) and J = L odd, the (0 0 0) term of
// eq. 022_rearranged vanishes, and both (0 -1 1) symbols reduce to the one
// (0 0 0) symbol of even total Y' = (l1, l2+1, l3; 0 0 0): the unshifted one
// by eq. joneodd, the shifted one (even total) by eq. joneevensimp with
// j3 -> j3 + 1.  Collecting the factors,
//
//     (l1 l2 l3; -2 2 0)^2 = Y'^2 s^2 (sig(sig+1) - c)(c - d(d+1))(c + mu)^2,
//     sig = l1 + l2 + 1,  tau = sig + 1,  mu = 2 (l1+2)(l2+2) - tau(tau+1),
//
// every factor an integer.  Y'^2 is the (0 0 0)^2 of the pair (l1, l2+1),
// i.e. the TT term of diagonal d+1 with l3 = d + 1 + 2k, so the odd-L pass is
// the same strip walk on diagonal d+1 with U_EB(k) = W'_PP(l3) g(k) g(d+1+k)
// (c - d(d+1)) and the row factor (sig(sig+1) - c)(c + mu)^2; its last step
// (l3 = l1 + l2 + 1) has sig(sig+1) - c = 0.
//
// Mapping.  One wavefront per work item (d, block of 64 R consecutive l1);
// lane i owns l1 = A + R i + j, j < R, and walks k.  g(l1 - k) and
// h(l1 + d + k) are kept in registers as windows of R values that slide by
// one per step (one LDS read each per step for R terms); U_X(k) and c(k) are
// read by the whole wave from one LDS address.  Terms with k > l1 read the
// zero guard of the g window and vanish, so lanes of a wave share one trip
// count.  Table windows are staged in LDS in chunks of 256 steps
// with one padding word per R entries (a lane stride of R+1 doubles is free
// of bank conflicts).  Work items are numbered longest first.
#include "couple_internal.hpp"

namespace couple {
namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;  // 1/(4 pi)

__global__ void scale_windows_kernel(const double* __restrict__ wtt, const double* __restrict__ wtp,
                                     const double* __restrict__ wpp, int n, int stride,
                                     double* __restrict__ wp, float* __restrict__ wpf) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const double f = (2.0 * l + 1.0) * kInv4Pi;
    const double a = wtt ? wtt[l] * f : 0.0;
    const double b = wtp ? wtp[l] * f : 0.0;
    const double c = wpp ? wpp[l] * f : 0.0;
    wp[l] = a;
    wp[stride + l] = b;
    wp[2 * stride + l] = c;
    wpf[l] = (float)a;
    wpf[stride + l] = (float)b;
    wpf[2 * stride + l] = (float)c;
}

// The windows of up to kBandMasks masks (NULL: spectrum not needed), one set
// per blockIdx.y, into the context's window sets (the float32 copies are not
// written: the multi-mask strip does not read them).
struct MaskWindows {
    const double* w[kBandMasks][3];
    int n[kBandMasks];   // entries of mask m's windows to read; W' = 0 from there on
};

__global__ void scale_windows_masks_kernel(MaskWindows mw, int n, int stride, double* __restrict__ wp) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const int m = blockIdx.y;
    const double f = (2.0 * l + 1.0) * kInv4Pi;
    double* out = wp + 3LL * stride * m;
    const bool in = l < mw.n[m];
#pragma unroll
    for (int x = 0; x < 3; ++x) out[(long long)x * stride + l] = (in && mw.w[m][x]) ? mw.w[m][x][l] * f : 0.0;
}

// Exponent of the suffix maximum of |W'_x| over each parity: one work-group per
// (spectrum x, parity p) and window set (blockIdx.y), threads over contiguous runs of l3 = p + 2 i.  Each
// run's maximum, a suffix maximum across the runs (Hillis-Steele in LDS), then
// each run walked backwards.  The float32 strip kernels scale an item's
// staged U by 2^-e at its first l3 (the largest |W'| it can meet then lies in
// [1/2, 1)) and its sums back by 2^e in float64, both exact: a window whose
// tail falls below float32's normal range (about 1e-38) then still leaves
// the terms that dominate every element inside it.
constexpr int kExpThreads = 1024;
__global__ void __launch_bounds__(kExpThreads) window_exponents_kernel(const double* __restrict__ wp, int n,
                                                                      int stride, int* __restrict__ wexp) {
    __shared__ double s_max[kExpThreads];
    const int x = blockIdx.x >> 1, p = blockIdx.x & 1;
    const int cnt = n > p ? (n - p + 1) / 2 : 0;
    const int per = (cnt + kExpThreads - 1) / kExpThreads;
    const int t = threadIdx.x;
    const int i0 = min(cnt, t * per), i1 = min(cnt, i0 + per);
    const long long set = 3LL * stride * blockIdx.y;     // window set (mask) of this work-group
    const double* w = wp + set + (long long)x * stride + p;
    int* e = wexp + set + (long long)x * stride + p;
    double m = 0.0;
    for (int i = i0; i < i1; ++i) m = fmax(m, fabs(w[2 * i]));
    s_max[t] = m;
    __syncthreads();
    for (int off = 1; off < kExpThreads; off <<= 1) {
        const double v = t + off < kExpThreads ? s_max[t + off] : 0.0;
        __syncthreads();
        s_max[t] = fmax(s_max[t], v);
        __syncthreads();
    }
    double run = t + 1 < kExpThreads ? s_max[t + 1] : 0.0;
    for (int i = i1 - 1; i >= i0; --i) {
        run = fmax(run, fabs(w[2 * i]));
        int ex = 0;
        if (run > 0.0) (void)frexp(run, &ex);
        e[2 * i] = min(1000, max(-1000, ex));
    }
}

struct StripArgs {
    const double* g;     // g(p), index 0 = p 0, valid 0 .. lmax_max
    const double* h;     // 1/((2p+1) g(p)), valid 0 .. 2 lmax_max
    const double* wp;    // scaled windows, 3 x wp_stride
    const int* wexp;     // float32 kernels: exponents of the suffix maxima of |W'| (window_exponents_kernel)
    const double* cl;    // c_l
    double* xi;          // 3 packed triangles of xi_stride
    long long xi_stride;
    int wp_stride;
    int g_len, h_len;    // valid lengths of g and h
    int lmax;
    int dmax;            // largest diagonal computed
    int band;            // dmax < lmax: items on a (block, diagonal) grid
    int l3_lo, l3_hi;
    // strip_fp32c_masks_kernel: mask m's windows at wp + m wp_mask_stride (exponents
    // likewise in wexp); its Xi triangles at xi + m_xi[m], m_stride[m] apart,
    // for rows l1 <= m_lmax[m] - d (lmax is the largest m_lmax)
    int n_masks;
    int wp_mask_stride;
    int m_lmax[kBandMasks];
    long long m_xi[kBandMasks];
    long long m_stride[kBandMasks];
};

// Work item -> (d, A): the block of rows A .. A + B - 1 of diagonal d, aligned
// to the diagonal's last row l1 = lmax - d, so that the one partial block of a
// diagonal holds its shortest rows (lanes with l1 < 0 are idle).  Block j of
// diagonal d starts at A = lmax - d + 1 - B (j + 1) and runs lmax + 1 - d - B j
// steps.  Returns false for an item that has no block.
//   Whole triangle: level m = j + floor(d / B) holds (m + 1) B items with
//   B m (m + 1) / 2 before it; trips fall with m, so longest run first.
//   Band (dmax < lmax): phases of kBandPhase diagonals in order of d, each
//   phase block by block; the band bounds every trip.
template <int B>
__device__ inline bool strip_item(const StripArgs& a, int item, int* d_out, int* A_out) {
    int d, j;
    if (a.band) {
        // phase p holds diagonals p kBandPhase .. + w - 1 of all J blocks, block-major
        const int J = (a.lmax + B) / B;
        const int p = item / (J * kBandPhase);
        const int w = min(kBandPhase, a.dmax + 1 - p * kBandPhase);
        const int r = item - p * J * kBandPhase;
        j = r / w;
        d = p * kBandPhase + r - j * w;
    } else {
        int m = (int)((sqrtf(8.0f * (float)item / (float)B + 1.0f) - 1.0f) * 0.5f);
        while (B * (m + 1) * (m + 2) / 2 <= item) ++m;
        while (m > 0 && B * m * (m + 1) / 2 > item) --m;
        const int rem = item - B * m * (m + 1) / 2;
        j = rem / B;
        d = B * (m - j) + (rem - B * j);
    }
    const int n_valid = a.lmax - d + 1;
    if (d > a.dmax || n_valid <= B * j) return false;
    *d_out = d;
    *A_out = n_valid - B * (j + 1);
    return true;
}

template <int R, int KC>
struct Win {
    static constexpr int kB = kWave * R;                // l1 per item
    static constexpr int kLen = kB + KC - 1;            // window length
    static constexpr int kPhys = kLen + kLen / R + 1;   // with padding
    __device__ static inline int phys(int slot) { return slot + slot / R; }
};

// Kernel modes: TT only; TT + TE + EE (even L); EB (odd L); TT + EE (even L,
// no TE: the TE window is not staged and its sum is not formed); EE only
// (even L, neither TT nor TE).
enum : int { kModeTT = 0, kModePol = 1, kModeEB = 2, kModePolEE = 3, kModeEE = 4 };

// WIDE (lmax > kNarrowLmax): a(a-2) + b(b-2) exceeds 2^53 and N' cancels
// against it when l1 << l2, so N' is taken as t^2 - (2ab + 1) with t exact and
// 2ab + 1 = beta_hi + beta_lo split exactly: one more operation per term.
// (kNarrowLmax: strip_params.hpp)

template <int R, int MODE, bool WIDE>
__global__ void __launch_bounds__(kWave)
strip_fp64_kernel(StripArgs a) {
    constexpr bool POL = MODE == kModePol || MODE == kModePolEE || MODE == kModeEE;
    constexpr bool TE = MODE == kModePol;
    constexpr bool TTS = MODE != kModeEE;               // the first sum (TT, or EB's)
    constexpr bool EB = MODE == kModeEB;
    constexpr int KC = kStripChunkF64;
    using W = Win<R, KC>;
    constexpr int B = W::kB;
    __shared__ double s_g[W::kPhys];
    __shared__ double s_h[W::kPhys];
    __shared__ double4 s_u[KC];

    int d, A;                                            // l2 = l1 + d; rows A .. A + B - 1
    if (!strip_item<B>(a, blockIdx.x, &d, &A)) return;
    const int de = EB ? d + 1 : d;                       // l3 = de + 2k
    const int n_valid = a.lmax - d + 1;                  // l1 = 0 .. n_valid - 1
    const int blk_max = A + B - 1;                       // largest l1 in this block
    const int k_lo = max(0, (a.l3_lo - de + 1) >> 1);    // ceil((l3_lo - de)/2)
    const int k_hi = min(blk_max, (a.l3_hi - de) >> 1);  // floor((l3_hi - de)/2)

    const int lane = threadIdx.x;
    const int l1_0 = A + R * lane;

    // even L: N' = c (c - gam2) + kap, every piece exact while lmax <= kNarrowLmax;
    //   WIDE: N' = t^2 - kap - blo, t = c - gam2, gam2 = a + b - 1, kap + blo = 2ab + 1.
    // EB: gam2 = sig(sig+1), kap = mu.
    double tt[R], te[R], ee[R], gam2[R], kap[R], blo[R], gw[R], hw[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        tt[j] = te[j] = ee[j] = 0.0;
        blo[j] = 0.0;
        const long long l1 = l1_0 + j, l2 = l1 + d;
        if (EB) {
            const long long sg = l1 + l2 + 1, tau = sg + 1;
            gam2[j] = (double)(sg * (sg + 1));
            kap[j] = (double)(2 * (l1 + 2) * (l2 + 2) - tau * (tau + 1));
        } else if (WIDE) {
            const long long aa = l1 * (l1 + 1), bb = l2 * (l2 + 1);
            const long long beta = 2 * aa * bb + 1;
            gam2[j] = (double)(aa + bb - 1);
            kap[j] = (double)beta;
            blo[j] = (double)(beta - (long long)kap[j]);
        } else {
            const long long aa = l1 * (l1 + 1), bb = l2 * (l2 + 1);
            gam2[j] = (double)(2 * (aa + bb - 1));
            kap[j] = (double)(aa * (aa - 2) + bb * (bb - 2));
        }
    }

    const double* wtt = a.wp;
    const double* wtp = a.wp + a.wp_stride;
    const double* wpp = a.wp + 2 * a.wp_stride;

    for (int k0 = k_lo; k0 <= k_hi; k0 += KC) {
        const int kc = min(KC, k_hi - k0 + 1);
        // steps are taken in groups of R; the staged U of steps kc .. kc_r - 1 is 0
        const int kc_r = (kc + R - 1) / R * R;
        __syncthreads();
        // stage g(e), e = A - k0 - KC + 1 + slot; h(e), e = A + d + k0 + slot.  The steps
        // k0 .. k0 + kc_r - 1 read g slots KC - kc_r .. kLen - 1 and h slots 0 .. B + kc_r - 2.
        const int g_base = A - k0 - KC + 1;
        const int h_base = A + de + k0;
        const int g_off = KC - kc_r, n_win = B + kc_r - 1;
        // the chunk's global loads in two batches (windows, then per-step factors)
        constexpr int NS = (W::kLen + kWave - 1) / kWave;
        constexpr int NU = KC / kWave;
        double gv[NS], hv[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int i = lane + q * kWave;
            const int eg = g_base + g_off + i, eh = h_base + i;
            gv[q] = (i < n_win && eg >= 0 && eg < a.g_len) ? a.g[eg] : 0.0;
            hv[q] = (i < n_win && eh >= 0 && eh < a.h_len) ? a.h[eh] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int i = lane + q * kWave;
            if (i < n_win) {
                s_g[W::phys(g_off + i)] = gv[q];
                s_h[W::phys(i)] = hv[q];
            }
        }
        double ga[NU], gb[NU], w0[NU], w1[NU], w2[NU];
#pragma unroll
        for (int e = 0; e < NU; ++e) {
            const int s = lane + e * kWave;
            ga[e] = gb[e] = w0[e] = w1[e] = w2[e] = 0.0;
            if (s < kc) {
                const int k = k0 + s, l3 = de + 2 * k;
                ga[e] = a.g[k];
                gb[e] = a.g[de + k];
                if (EB || POL) w2[e] = wpp[l3];
                if (!EB && TTS) w0[e] = wtt[l3];
                if (TE) w1[e] = wtp[l3];
            }
        }
#pragma unroll
        for (int e = 0; e < NU; ++e) {
            const int s = lane + e * kWave;
            double4 u = {0.0, 0.0, 0.0, 0.0};
            if (s < kc) {
                const int k = k0 + s;
                const int l3 = de + 2 * k;
                const double gg = ga[e] * gb[e];
                const long long c = (long long)l3 * (l3 + 1);
                if (EB) {
                    u.x = w2[e] * gg * (double)(c - (long long)d * (d + 1));
                    u.w = (double)c;
                } else {
                    if (TTS) u.x = w0[e] * gg;
                    if (POL) {
                        if (TE) u.y = w1[e] * gg;
                        u.z = w2[e] * gg;
                        u.w = (double)c;
                    }
                }
            }
            if (s < kc_r) s_u[s] = u;
        }
        __syncthreads();

        if (k0 == k_lo) {
            // windows as they stand one step before k_lo: every step below
            // first slides them by one and then reads the new entry
#pragma unroll
            for (int j = 0; j < R - 1; ++j) gw[j] = s_g[W::phys(R * lane + j + KC)];
            gw[R - 1] = 0.0;
            hw[0] = 0.0;
#pragma unroll
            for (int j = 1; j < R; ++j) hw[j] = s_h[W::phys(R * lane + j - 1)];
        }
        // phys(R lane + KC - 1 - s) and phys(R lane + R - 1 + s) for s = s0 + u:
        // per group of R steps the g pointer moves down and the h pointer up by R + 1
        const double* pg = s_g + (R + 1) * (lane + KC / R - 1) + (R - 1);
        const double* ph = s_h + (R + 1) * lane + (R - 1);
        for (int s0 = 0; s0 < kc_r; s0 += R, pg -= R + 1, ph += R + 1) {
            const double4* pu = s_u + s0;
#pragma unroll
            for (int u = 0; u < R; ++u) {
#pragma unroll
                for (int j = R - 1; j > 0; --j) gw[j] = gw[j - 1];
                gw[0] = pg[-u];
#pragma unroll
                for (int j = 0; j < R - 1; ++j) hw[j] = hw[j + 1];
                hw[R - 1] = ph[u + (u >= 1 ? 1 : 0)];
                const double4 uu = pu[u];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const double P = gw[j] * hw[j];
                    if (EB) {
                        // (sig(sig+1) - c) (c + mu)^2, each factor an exact integer
                        const double f1 = gam2[j] - uu.w;
                        const double f3 = uu.w + kap[j];
                        tt[j] = __builtin_fma(uu.x, P * ((f1 * f3) * f3), tt[j]);
                        continue;
                    }
                    if (TTS) tt[j] = __builtin_fma(uu.x, P, tt[j]);
                    if (POL) {
                        double N;
                        if (WIDE) {
                            const double t = uu.w - gam2[j];
                            N = __builtin_fma(t, t, -kap[j]) - blo[j];
                        } else {
                            const double dc = uu.w - gam2[j];
                            N = __builtin_fma(uu.w, dc, kap[j]);
                        }
                        const double y = P * N;
                        if (TE) te[j] = __builtin_fma(uu.y, y, te[j]);
                        const double z = y * N;
                        ee[j] = __builtin_fma(uu.z, z, ee[j]);
                    }
                }
            }
        }
    }

    // ---- store Xi on the packed triangle ----
    const long long off = diag_offset(a.lmax, d);
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int l1 = l1_0 + j;
        if (l1 >= 0 && l1 < n_valid) {
            if (EB) {
                const double s = 0.5 * a.cl[l1] * a.cl[l1 + d];
                a.xi[3 * a.xi_stride + off + l1] = (s * s) * tt[j];
                continue;
            }
            if (TTS) a.xi[off + l1] = tt[j];
            if (POL) {
                const double s = 0.5 * a.cl[l1] * a.cl[l1 + d];
                if (TE) a.xi[a.xi_stride + off + l1] = s * te[j];
                a.xi[2 * a.xi_stride + off + l1] = (s * s) * ee[j];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP32-compensated variant.  Same mapping and staging as strip_fp64_kernel;
// the terms are float32:
//   P = g(l1-k) h(l1+d+k) from float32 tables (each rounded once from the
//       double-double build),
//   U_X(k) formed in float64 from the float64 tables and windows and rounded
//       once to float32,
//   N' = t^2 - (2ab + 1) with t = c - (a + b - 1) is an integer polynomial in
//       c, and both t^2 and 2ab + 1 exceed 2^24 for l >~ 2900 while N' may be
//       much smaller, so it is expanded about the start of each split of
//       kStripRebase steps: with the exact integers T = c_s - (a + b - 1) and
//       Q = T^2 - (2ab + 1) = N'(c_s) at the split's c_s, and the staged
//       per-step integer D(k) = c(k) - c_s (|D| < 2^24, exact in float32),
//           N' = Q + D (2T + D) = fma(D, 2T + D, Q),
//       one add and one fused multiply-add per row and term.  Per lane and
//       row, T (int32) and Q (int64) are carried from split to split exactly
//       (Q += D_s T; T += D_s; Q += D_s T, D_s = c(next split) - c_s) and
//       rounded once to float32 there.  The error of N' is a few roundings of
//       max(|Q|, |N'|), the size of N' itself over the split, instead of
//       the size of t^2.
//   EB: f1 = sig(sig+1) - c and f3 = c + mu are linear in c; per split the
//       lane's first row splits T = sig(sig+1) - c_s and T3 = c_s + mu into
//       float32 T_hi + T_lo exactly, so f1 = T_hi + (T_lo - D) and
//       f3 = T3_hi + (D + T3_lo) round once; row j adds its exact integer
//       offset (below 2^19) to those.
// Accumulation, three levels per spectrum and lane-owned l1: kCompBlock
// consecutive terms are summed with float32 FMA into a block sum; block sums
// are added plainly into a mid sum; every kCompPeriod steps (and at the end of
// a chunk) the mid sum enters a Kahan (sum, compensation) pair in float32.
// The pair is combined and rescaled by s = c_l1 c_l2 / 2 in float64.  The
// mid level holds at most kCompPeriod / kCompBlock block sums, so its rounding
// stays at the size of the per-term rounding while the Kahan step runs once
// per 64 terms instead of once per 16.
constexpr int kCompBlock = 4 * kStripR;
constexpr int kCompPeriod = 64;

template <int R, int MODE>
__global__ void __launch_bounds__(kWave, MODE == kModePolEE ? 5 : 1)
strip_fp32c_kernel(StripArgs a, const float* __restrict__ gf, const float* __restrict__ hf) {
    constexpr bool POL = MODE == kModePol || MODE == kModePolEE || MODE == kModeEE;
    constexpr bool TE = MODE == kModePol;
    constexpr bool TTS = MODE != kModeEE;               // the first sum (TT, or EB's)
    constexpr bool EB = MODE == kModeEB;
    constexpr int KC = kStripChunkF32;
    using W = Win<R, KC>;
    constexpr int B = W::kB;
    constexpr int G = kCompBlock;
    constexpr int RB = kStripRebase;
    constexpr int CP = kCompPeriod;
    static_assert(KC % RB == 0 && RB % G == 0 && G % R == 0 && CP % G == 0,
                  "chunk must hold whole splits and blocks");
    __shared__ float s_g[W::kPhys];
    __shared__ float s_h[W::kPhys];
    __shared__ float4 s_u[KC];

    int d, A;                                            // l2 = l1 + d; rows A .. A + B - 1
    if (!strip_item<B>(a, blockIdx.x, &d, &A)) return;
    const int de = EB ? d + 1 : d;                       // l3 = de + 2k
    const int n_valid = a.lmax - d + 1;
    const int blk_max = A + B - 1;
    const int k_lo = max(0, (a.l3_lo - de + 1) >> 1);
    const int k_hi = min(blk_max, (a.l3_hi - de) >> 1);

    const int lane = threadIdx.x;
    const int l1_0 = A + R * lane;

    // Kahan pairs (sum, compensation) and mid sums per spectrum and lane-owned l1
    float kt[R], kte[R], kee[R], ct[R], cte[R], cee[R];
    float mt[R], mte[R], mee[R];
    float gw[R], hw[R];
    // EB: gam = sig(sig+1), mu, and the exact offsets of rows j from the lane's first row
    int gam[R], mu[R];
    float dg[R], dm[R];
    // even L, polarized: T = c_s - (a + b - 1) and Q = T^2 - (2ab + 1) at the current
    // split start c_s, exact, and their float32 forms qf = fl(Q), rf = fl(2T)
    int tq[R];
    long long q64[R];
    float qf[R], rf[R];
    int c_cur = 0;
    {
        const int l3s = de + 2 * k_lo;
        c_cur = l3s * (l3s + 1);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        kt[j] = kte[j] = kee[j] = ct[j] = cte[j] = cee[j] = 0.0f;
        mt[j] = mte[j] = mee[j] = 0.0f;
        qf[j] = rf[j] = 0.0f;
        const long long l1 = l1_0 + j, l2 = l1 + d;
        if (EB) {
            const long long sg = l1 + l2 + 1, tau = sg + 1;
            gam[j] = (int)(sg * (sg + 1));
            mu[j] = (int)(2 * (l1 + 2) * (l2 + 2) - tau * (tau + 1));
            tq[j] = 0;
            q64[j] = 0;
        } else {
            const long long aa = l1 * (l1 + 1), bb = l2 * (l2 + 1);
            gam[j] = mu[j] = 0;
            const long long t = (long long)c_cur - (aa + bb - 1);
            tq[j] = (int)t;
            q64[j] = t * t - (2 * aa * bb + 1);
        }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        dg[j] = (float)(gam[j] - gam[0]);
        dm[j] = (float)(mu[j] - mu[0]);
    }

    const double* wtt = a.wp;
    const double* wtp = a.wp + a.wp_stride;
    const double* wpp = a.wp + 2 * a.wp_stride;
    // per-item power-of-two scales of U (exact): from the largest |W'| at or above
    // the item's first l3, so the dominant terms sit near 1 in float32
    const int l3f = min(de + 2 * k_lo, a.l3_hi);      // an item with no step in the band stores zeros
    const int ex_tt = a.wexp[l3f], ex_tp = a.wexp[a.wp_stride + l3f], ex_pp = a.wexp[2 * a.wp_stride + l3f];

    for (int k0 = k_lo; k0 <= k_hi; k0 += KC) {
        const int kc = min(KC, k_hi - k0 + 1);
        // steps run in blocks of G; the staged U of steps kc .. kc_r - 1 is 0
        const int kc_r = (kc + G - 1) / G * G;
        __syncthreads();
        const int g_base = A - k0 - KC + 1;
        const int h_base = A + de + k0;
        // the steps k0 .. k0 + kc_r - 1 read g slots KC - kc_r .. kLen - 1 and
        // h slots 0 .. B + kc_r - 2: only those are staged
        const int g_off = KC - kc_r;
        for (int i = lane; i < B + kc_r - 1; i += kWave) {
            const int eg = g_base + g_off + i, eh = h_base + i;
            s_g[W::phys(g_off + i)] = (eg >= 0 && eg < a.g_len) ? gf[eg] : 0.0f;
            s_h[W::phys(i)] = (eh >= 0 && eh < a.h_len) ? hf[eh] : 0.0f;
        }
        for (int s = lane; s < kc_r; s += kWave) {
            float4 u = {0.0f, 0.0f, 0.0f, 0.0f};
            if (s < kc) {
                const int k = k0 + s;
                const int l3 = de + 2 * k;
                const int l3c = de + 2 * (k0 + s / RB * RB);     // l3 at this step's split
                const double gg = a.g[k] * a.g[de + k];
                if (EB) {
                    const long long c = (long long)l3 * (l3 + 1);
                    u.x = (float)(ldexp(wpp[l3] * gg, -ex_pp) * (double)(c - (long long)d * (d + 1)));
                    u.w = (float)(l3 * (l3 + 1) - l3c * (l3c + 1));
                } else {
                    if (TTS) u.x = (float)ldexp(wtt[l3] * gg, -ex_tt);
                    if (POL) {
                        if (TE) u.y = (float)ldexp(wtp[l3] * gg, -ex_tp);
                        u.z = (float)ldexp(wpp[l3] * gg, -ex_pp);
                        u.w = (float)(l3 * (l3 + 1) - l3c * (l3c + 1));
                    }
                }
            }
            s_u[s] = u;
        }
        __syncthreads();

        if (k0 == k_lo) {
#pragma unroll
            for (int j = 0; j < R - 1; ++j) gw[j] = s_g[W::phys(R * lane + j + KC)];
            gw[R - 1] = 0.0f;
            hw[0] = 0.0f;
#pragma unroll
            for (int j = 1; j < R; ++j) hw[j] = s_h[W::phys(R * lane + j - 1)];
        }
        float thi = 0.0f, tlo = 0.0f, t3hi = 0.0f, t3lo = 0.0f;   // EB: first row's split
        const float* pg = s_g + (R + 1) * (lane + KC / R - 1) + (R - 1);
        const float* ph = s_h + (R + 1) * lane + (R - 1);
        for (int sb = 0; sb < kc_r; sb += G) {
            if (sb % RB == 0) {
                const int l3c = de + 2 * (k0 + sb);
                const int cc = l3c * (l3c + 1);
                if (EB) {
                    // f1 = sig(sig+1) - c = T - D(k), T = sig(sig+1) - c_s, and
                    // f3 = c + mu = T3 + D(k), T3 = c_s + mu, each split exactly into hi + lo
                    const int T = gam[0] - cc;
                    thi = (float)T;
                    tlo = (float)(T - (int)thi);
                    const int T3 = cc + mu[0];
                    t3hi = (float)T3;
                    t3lo = (float)(T3 - (int)t3hi);
                } else if (POL) {
                    // move (T, Q) from the previous split start to c_s = cc, exactly:
                    // Q(c + D) = Q(c) + D (2T + D) = Q + D T + D (T + D)
                    const int Ds = cc - c_cur;
                    c_cur = cc;
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        q64[j] += (long long)Ds * tq[j];
                        tq[j] += Ds;
                        q64[j] += (long long)Ds * tq[j];
                        qf[j] = (float)(double)q64[j];
                        rf[j] = 2.0f * (float)tq[j];
                    }
                }
            }
            float bt[R], bte[R], bee[R];
#pragma unroll
            for (int j = 0; j < R; ++j) bt[j] = bte[j] = bee[j] = 0.0f;
#pragma unroll
            for (int q = 0; q < G / R; ++q, pg -= R + 1, ph += R + 1) {
                const int s0 = sb + q * R;
                const float4* pu = s_u + s0;
#pragma unroll
                for (int u = 0; u < R; ++u) {
#pragma unroll
                    for (int j = R - 1; j > 0; --j) gw[j] = gw[j - 1];
                    gw[0] = pg[-u];
#pragma unroll
                    for (int j = 0; j < R - 1; ++j) hw[j] = hw[j + 1];
                    hw[R - 1] = ph[u + (u >= 1 ? 1 : 0)];
                    const float4 uu = pu[u];
                    // EB: first row exact split; rows j > 0 add their exact integer offsets
                    const float f10 = thi + (tlo - uu.w), f30 = t3hi + (uu.w + t3lo);
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const float P = gw[j] * hw[j];
                        if (EB) {
                            const float f1 = j == 0 ? f10 : f10 + dg[j];
                            const float f3 = j == 0 ? f30 : f30 + dm[j];
                            bt[j] = __builtin_fmaf(uu.x, P * ((f1 * f3) * f3), bt[j]);
                            continue;
                        }
                        if (TTS) bt[j] = __builtin_fmaf(uu.x, P, bt[j]);
                        if (POL) {
                            // N' = Q + D (2T + D)
                            const float N = __builtin_fmaf(uu.w, rf[j] + uu.w, qf[j]);
                            const float y = P * N;
                            if (TE) bte[j] = __builtin_fmaf(uu.y, y, bte[j]);
                            const float z = y * N;
                            bee[j] = __builtin_fmaf(uu.z, z, bee[j]);
                        }
                    }
                }
            }
            // block sums into the mid sums
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (TTS) mt[j] += bt[j];
                if (TE) mte[j] += bte[j];
                if (POL) mee[j] += bee[j];
            }
            if ((sb + G) % CP != 0 && sb + G < kc_r) continue;
            // Kahan step: mid sums into the pairs
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (TTS) {
                    const float yv = mt[j] - ct[j];
                    const float tv = kt[j] + yv;
                    ct[j] = (tv - kt[j]) - yv;
                    kt[j] = tv;
                    mt[j] = 0.0f;
                }
                if (TE) {
                    const float yv = mte[j] - cte[j];
                    const float tv = kte[j] + yv;
                    cte[j] = (tv - kte[j]) - yv;
                    kte[j] = tv;
                    mte[j] = 0.0f;
                }
                if (POL) {
                    const float yw = mee[j] - cee[j];
                    const float tw = kee[j] + yw;
                    cee[j] = (tw - kee[j]) - yw;
                    kee[j] = tw;
                    mee[j] = 0.0f;
                }
            }
        }
    }

    const long long off = diag_offset(a.lmax, d);
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int l1 = l1_0 + j;
        if (l1 >= 0 && l1 < n_valid) {
            if (EB) {
                const double s = 0.5 * a.cl[l1] * a.cl[l1 + d];
                a.xi[3 * a.xi_stride + off + l1] = ldexp((s * s) * ((double)kt[j] - (double)ct[j]), ex_pp);
                continue;
            }
            if (TTS) a.xi[off + l1] = ldexp((double)kt[j] - (double)ct[j], ex_tt);
            if (POL) {
                const double s = 0.5 * a.cl[l1] * a.cl[l1 + d];
                if (TE) a.xi[a.xi_stride + off + l1] = ldexp(s * ((double)kte[j] - (double)cte[j]), ex_tp);
                a.xi[2 * a.xi_stride + off + l1] = ldexp((s * s) * ((double)kee[j] - (double)cee[j]), ex_pp);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP32-compensated strip over up to four masks of one call.  The masks share
// the band and the spectra, so P = g(l1-k) h(l1+d+k), N' and the products P N'
// and P N'^2 of a term are the same for all of them: only U_X(k) =
// W'_X(l3) g(k) g(d+k) differs.  One wave computes an item for all M masks,
// the shared factors once per term and then one FMA per mask and spectrum, so
// the g/h windows and the N' expansion are staged and formed once for the
// group.  The grid is that of the largest lmax among the masks; a mask stores
// only its own rows (l1 <= its lmax - d), and its windows are 0 above its
// 2 lmax.  Each mask's U is formed and scaled as in strip_fp32c_kernel (its
// own suffix-maximum exponents), rounded once to float32 and staged in packed
// float4 slots.  Accumulation per mask, spectrum and row: G-term FMA blocks;
// with CP > G, CP/G block sums are added plainly into a mid sum; every CP steps
// (and at a chunk's end) a Kahan step in float32; the pair is combined,
// rescaled and unscaled in float64.  The odd-L mode (EB) shares P and the
// exact f1 f3^2 factor of strip_fp32c_kernel's EB mode the same way.
template <int MODE, int M, int G, int CP>
__global__ void __launch_bounds__(kWave)
strip_fp32c_masks_kernel(StripArgs a, const float* __restrict__ gf, const float* __restrict__ hf) {
    constexpr int R = kStripR;
    constexpr bool POL = MODE == kModePol || MODE == kModePolEE || MODE == kModeEE;
    constexpr bool TE = MODE == kModePol;
    constexpr bool TTS = MODE != kModeEE;               // the first sum (TT, or EB's)
    constexpr bool EB = MODE == kModeEB;
    constexpr bool MID = CP > G;
    constexpr int KC = kStripChunkF32;
    using W = Win<R, KC>;
    constexpr int B = W::kB;
    constexpr int RB = kStripRebase;
    static_assert(M >= 1 && M <= 4, "one float4 lane per mask");
    static_assert(KC % RB == 0 && RB % G == 0 && G % R == 0 && CP % G == 0 && KC % CP == 0,
                  "chunk must hold whole splits, blocks and Kahan periods");
    __shared__ float s_g[W::kPhys];
    __shared__ float s_h[W::kPhys];
    // a step's U packed into NV float4: slots x[m] = m, y[m] = NX + m, z[m] = NX + NY + m,
    // then D (N' expansion, or EB's c - c_s) in slot NU when that fits the last float4, else in s_uw
    constexpr bool DW = POL || EB;
    constexpr int NX = TTS ? M : 0, NY = TE ? M : 0, NZ = POL ? M : 0;
    constexpr int NU = NX + NY + NZ;
    constexpr bool WPACK = DW && NU % 4 != 0;
    constexpr int NV = (NU + (WPACK ? 1 : 0) + 3) / 4;
    __shared__ float4 s_u4[KC][NV];
    __shared__ float s_uw[(DW && !WPACK) ? KC : 1];

    int d, A;                                            // l2 = l1 + d; rows A .. A + B - 1
    if (!strip_item<B>(a, blockIdx.x, &d, &A)) return;
    const int de = EB ? d + 1 : d;                       // l3 = de + 2k
    const int blk_max = A + B - 1;
    const int k_lo = max(0, (a.l3_lo - de + 1) >> 1);
    const int k_hi = min(blk_max, (a.l3_hi - de) >> 1);
    const int lane = threadIdx.x;
    const int l1_0 = A + R * lane;

    float kt[R][M], kte[R][M], kee[R][M], ct[R][M], cte[R][M], cee[R][M];
    float mt[R][M], mte[R][M], mee[R][M];
    float gw[R], hw[R], qf[R], rf[R];
    // T = c_s - (a + b - 1) and Q = T^2 - (2ab + 1) at the current split start
    // c_s, exact, carried from split to split (strip_fp32c_kernel)
    int tq[R];
    long long q64[R];
    // EB: gam = sig(sig+1), mu, and the exact offsets of rows j from the lane's first row
    int gam[R], mu[R];
    float dg[R], dm[R];
    int c_cur;
    {
        const int l3s = de + 2 * k_lo;
        c_cur = l3s * (l3s + 1);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        qf[j] = rf[j] = 0.0f;
        const long long l1 = l1_0 + j, l2 = l1 + d;
        if (EB) {
            const long long sg = l1 + l2 + 1, tau = sg + 1;
            gam[j] = (int)(sg * (sg + 1));
            mu[j] = (int)(2 * (l1 + 2) * (l2 + 2) - tau * (tau + 1));
            tq[j] = 0;
            q64[j] = 0;
        } else {
            const long long aa = l1 * (l1 + 1), bb = l2 * (l2 + 1);
            const long long t = (long long)c_cur - (aa + bb - 1);
            gam[j] = mu[j] = 0;
            tq[j] = (int)t;
            q64[j] = t * t - (2 * aa * bb + 1);
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            kt[j][m] = kte[j][m] = kee[j][m] = ct[j][m] = cte[j][m] = cee[j][m] = 0.0f;
            mt[j][m] = mte[j][m] = mee[j][m] = 0.0f;
        }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        dg[j] = (float)(gam[j] - gam[0]);
        dm[j] = (float)(mu[j] - mu[0]);
    }
    // per-mask power-of-two scales at the item's first l3 (strip_fp32c_kernel)
    const int l3f = min(de + 2 * k_lo, a.l3_hi);
    int ex_tt[M], ex_tp[M], ex_pp[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int* we = a.wexp + (long long)m * a.wp_mask_stride;
        const bool on = m < a.n_masks;
        ex_tt[m] = on ? we[l3f] : 0;
        ex_tp[m] = on ? we[a.wp_stride + l3f] : 0;
        ex_pp[m] = on ? we[2 * a.wp_stride + l3f] : 0;
    }

    for (int k0 = k_lo; k0 <= k_hi; k0 += KC) {
        const int kc = min(KC, k_hi - k0 + 1);
        const int kc_r = (kc + G - 1) / G * G;           // staged U of steps kc .. kc_r - 1 is 0
        __syncthreads();
        const int g_base = A - k0 - KC + 1;
        const int h_base = A + de + k0;
        const int g_off = KC - kc_r;
        for (int i = lane; i < B + kc_r - 1; i += kWave) {
            const int eg = g_base + g_off + i, eh = h_base + i;
            s_g[W::phys(g_off + i)] = (eg >= 0 && eg < a.g_len) ? gf[eg] : 0.0f;
            s_h[W::phys(i)] = (eh >= 0 && eh < a.h_len) ? hf[eh] : 0.0f;
        }
        for (int st = lane; st < kc_r; st += kWave) {
            float uf[4 * NV];
#pragma unroll
            for (int i = 0; i < 4 * NV; ++i) uf[i] = 0.0f;
            float uw = 0.0f;
            if (st < kc) {
                const int k = k0 + st;
                const int l3 = de + 2 * k;
                const int l3c = de + 2 * (k0 + st / RB * RB);   // l3 at this step's split
                const double gg = a.g[k] * a.g[de + k];
                const long long c = (long long)l3 * (l3 + 1);
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    if (m >= a.n_masks) continue;
                    const double* w = a.wp + (long long)m * a.wp_mask_stride;
                    if (EB)
                        uf[m] = (float)(ldexp(w[2 * a.wp_stride + l3] * gg, -ex_pp[m]) *
                                        (double)(c - (long long)d * (d + 1)));
                    else if (TTS)
                        uf[m] = (float)ldexp(w[l3] * gg, -ex_tt[m]);
                    if (TE) uf[NX + m] = (float)ldexp(w[a.wp_stride + l3] * gg, -ex_tp[m]);
                    if (POL) uf[NX + NY + m] = (float)ldexp(w[2 * a.wp_stride + l3] * gg, -ex_pp[m]);
                }
                if (DW) uw = (float)(l3 * (l3 + 1) - l3c * (l3c + 1));
            }
            if (WPACK) uf[NU] = uw;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                s_u4[st][v] = make_float4(uf[4 * v], uf[4 * v + 1], uf[4 * v + 2], uf[4 * v + 3]);
            if (DW && !WPACK) s_uw[st] = uw;
        }
        __syncthreads();

        if (k0 == k_lo) {
#pragma unroll
            for (int j = 0; j < R - 1; ++j) gw[j] = s_g[W::phys(R * lane + j + KC)];
            gw[R - 1] = 0.0f;
            hw[0] = 0.0f;
#pragma unroll
            for (int j = 1; j < R; ++j) hw[j] = s_h[W::phys(R * lane + j - 1)];
        }
        const float* pg = s_g + (R + 1) * (lane + KC / R - 1) + (R - 1);
        const float* ph = s_h + (R + 1) * lane + (R - 1);
        float thi = 0.0f, tlo = 0.0f, t3hi = 0.0f, t3lo = 0.0f;   // EB: first row's split
        for (int sb = 0; sb < kc_r; sb += G) {
            if (EB && sb % RB == 0) {
                // f1 = sig(sig+1) - c = T - D(k), T = sig(sig+1) - c_s, and
                // f3 = c + mu = T3 + D(k), T3 = c_s + mu, each split exactly into hi + lo
                const int l3c = de + 2 * (k0 + sb);
                const int cc = l3c * (l3c + 1);
                const int T = gam[0] - cc;
                thi = (float)T;
                tlo = (float)(T - (int)thi);
                const int T3 = cc + mu[0];
                t3hi = (float)T3;
                t3lo = (float)(T3 - (int)t3hi);
            }
            if (POL && sb % RB == 0) {
                // move (T, Q) to this split's c_s: Q(c + D) = Q + D T + D (T + D)
                const int l3c = d + 2 * (k0 + sb);
                const int cc = l3c * (l3c + 1);
                const int Ds = cc - c_cur;
                c_cur = cc;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    q64[j] += (long long)Ds * tq[j];
                    tq[j] += Ds;
                    q64[j] += (long long)Ds * tq[j];
                    qf[j] = (float)(double)q64[j];
                    rf[j] = 2.0f * (float)tq[j];
                }
            }
            float bt[R][M], bte[R][M], bee[R][M];
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int m = 0; m < M; ++m) bt[j][m] = bte[j][m] = bee[j][m] = 0.0f;
#pragma unroll
            for (int q = 0; q < G / R; ++q, pg -= R + 1, ph += R + 1) {
                const int s0 = sb + q * R;
#pragma unroll
                for (int u = 0; u < R; ++u) {
#pragma unroll
                    for (int j = R - 1; j > 0; --j) gw[j] = gw[j - 1];
                    gw[0] = pg[-u];
#pragma unroll
                    for (int j = 0; j < R - 1; ++j) hw[j] = hw[j + 1];
                    hw[R - 1] = ph[u + (u >= 1 ? 1 : 0)];
                    float uf[4 * NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const float4 q4 = s_u4[s0 + u][v];
                        uf[4 * v] = q4.x;
                        uf[4 * v + 1] = q4.y;
                        uf[4 * v + 2] = q4.z;
                        uf[4 * v + 3] = q4.w;
                    }
                    const float w = !DW ? 0.0f : WPACK ? uf[WPACK ? NU : 0] : s_uw[s0 + u];
                    const float* xs = uf;
                    const float* ys = uf + NX;
                    const float* zs = uf + NX + NY;
                    // EB: first row exact split; rows j > 0 add their exact integer offsets
                    const float f10 = thi + (tlo - w), f30 = t3hi + (w + t3lo);
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const float P = gw[j] * hw[j];
                        if (EB) {
                            const float f1 = j == 0 ? f10 : f10 + dg[j];
                            const float f3 = j == 0 ? f30 : f30 + dm[j];
                            const float e = P * ((f1 * f3) * f3);
#pragma unroll
                            for (int m = 0; m < M; ++m) bt[j][m] = __builtin_fmaf(xs[m], e, bt[j][m]);
                            continue;
                        }
                        if (TTS)
#pragma unroll
                            for (int m = 0; m < M; ++m) bt[j][m] = __builtin_fmaf(xs[m], P, bt[j][m]);
                        if (POL) {
                            const float N = __builtin_fmaf(w, rf[j] + w, qf[j]);   // N' = Q + D (2T + D)
                            const float y = P * N;
                            if (TE)
#pragma unroll
                                for (int m = 0; m < M; ++m) bte[j][m] = __builtin_fmaf(ys[m], y, bte[j][m]);
                            const float z = y * N;
#pragma unroll
                            for (int m = 0; m < M; ++m) bee[j][m] = __builtin_fmaf(zs[m], z, bee[j][m]);
                        }
                    }
                }
            }
            if (MID) {
#pragma unroll
                for (int j = 0; j < R; ++j)
#pragma unroll
                    for (int m = 0; m < M; ++m) {
                        if (TTS) mt[j][m] += bt[j][m];
                        if (TE) mte[j][m] += bte[j][m];
                        if (POL) mee[j][m] += bee[j][m];
                    }
                if ((sb + G) % CP != 0 && sb + G < kc_r) continue;
            }
            // Kahan step of the mid sums (or the block sums) into the pairs
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    if (TTS) {
                        const float v = MID ? mt[j][m] : bt[j][m];
                        const float yv = v - ct[j][m];
                        const float tv = kt[j][m] + yv;
                        ct[j][m] = (tv - kt[j][m]) - yv;
                        kt[j][m] = tv;
                        mt[j][m] = 0.0f;
                    }
                    if (TE) {
                        const float v = MID ? mte[j][m] : bte[j][m];
                        const float yv = v - cte[j][m];
                        const float tv = kte[j][m] + yv;
                        cte[j][m] = (tv - kte[j][m]) - yv;
                        kte[j][m] = tv;
                        mte[j][m] = 0.0f;
                    }
                    if (POL) {
                        const float v = MID ? mee[j][m] : bee[j][m];
                        const float yv = v - cee[j][m];
                        const float tv = kee[j][m] + yv;
                        cee[j][m] = (tv - kee[j][m]) - yv;
                        kee[j][m] = tv;
                        mee[j][m] = 0.0f;
                    }
                }
        }
    }

#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (m >= a.n_masks || d > a.m_lmax[m]) continue;
        double* xm = a.xi + a.m_xi[m] + diag_offset(a.m_lmax[m], d);
        const long long st = a.m_stride[m];
        const int rows = a.m_lmax[m] - d + 1;            // this mask's rows of diagonal d
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int l1 = l1_0 + j;
            if (l1 < 0 || l1 >= rows) continue;
            const double sc = (POL || EB) ? 0.5 * a.cl[l1] * a.cl[l1 + d] : 0.0;
            if (EB) {
                xm[3 * st + l1] = ldexp((sc * sc) * ((double)kt[j][m] - (double)ct[j][m]), ex_pp[m]);
                continue;
            }
            if (TTS) xm[l1] = ldexp((double)kt[j][m] - (double)ct[j][m], ex_tt[m]);
            if (TE) xm[st + l1] = ldexp(sc * ((double)kte[j][m] - (double)cte[j][m]), ex_tp[m]);
            if (POL) xm[2 * st + l1] = ldexp((sc * sc) * ((double)kee[j][m] - (double)cee[j][m]), ex_pp[m]);
        }
    }
}

// ---------------------------------------------------------------------------
// Float64 strip over up to four masks of one call (strip_fp32c_masks_kernel's
// layout and sharing: P, N', P N' and P N'^2 once per term, one FMA per mask
// and spectrum).  Each mask's U and sums are those of strip_fp64_kernel: a
// plain FMA chain per row in step order, so the chunk length (kStripChunkF64Masks
// steps, short enough for the masks' float64 U to leave LDS for two waves per
// SIMD) does not change a result bit.  The odd-L mode (EB) forms
// strip_fp64_kernel's exact f1 f3^2 factor once per term for all masks.

template <int MODE, int M, bool WIDE>
__global__ void __launch_bounds__(kWave)
strip_fp64_masks_kernel(StripArgs a) {
    constexpr int R = kStripR;
    constexpr bool POL = MODE == kModePol || MODE == kModePolEE || MODE == kModeEE;
    constexpr bool TE = MODE == kModePol;
    constexpr bool TTS = MODE != kModeEE;               // the first sum (TT, or EB's)
    constexpr bool EB = MODE == kModeEB;
    constexpr int KC = kStripChunkF64Masks;
    using W = Win<R, KC>;
    constexpr int B = W::kB;
    static_assert(M >= 1 && M <= kBandMasks, "masks per launch");
    static_assert(KC % R == 0 && KC % kWave == 0, "chunk of whole step groups and lanes");
    // a step's U in NV double2: slots x[m] = m, y[m] = NX + m, z[m] = NX + NY + m, then c
    constexpr int NX = TTS ? M : 0, NY = TE ? M : 0, NZ = POL ? M : 0;
    constexpr int NU = NX + NY + NZ + ((POL || EB) ? 1 : 0);
    constexpr int NV = (NU + 1) / 2;
    __shared__ double s_g[W::kPhys];
    __shared__ double s_h[W::kPhys];
    __shared__ double2 s_u2[KC][NV];

    int d, A;                                            // l2 = l1 + d; rows A .. A + B - 1
    if (!strip_item<B>(a, blockIdx.x, &d, &A)) return;
    const int de = EB ? d + 1 : d;                       // l3 = de + 2k
    const int blk_max = A + B - 1;
    const int k_lo = max(0, (a.l3_lo - de + 1) >> 1);
    const int k_hi = min(blk_max, (a.l3_hi - de) >> 1);
    const int lane = threadIdx.x;
    const int l1_0 = A + R * lane;

    // N' per row as in strip_fp64_kernel (narrow: c (c - gam2) + kap; WIDE: t^2 - kap - blo);
    // EB: gam2 = sig(sig+1), kap = mu
    double tt[R][M], te[R][M], ee[R][M], gam2[R], kap[R], blo[R], gw[R], hw[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
#pragma unroll
        for (int m = 0; m < M; ++m) tt[j][m] = te[j][m] = ee[j][m] = 0.0;
        blo[j] = 0.0;
        const long long l1 = l1_0 + j, l2 = l1 + d;
        const long long aa = l1 * (l1 + 1), bb = l2 * (l2 + 1);
        if (EB) {
            const long long sg = l1 + l2 + 1, tau = sg + 1;
            gam2[j] = (double)(sg * (sg + 1));
            kap[j] = (double)(2 * (l1 + 2) * (l2 + 2) - tau * (tau + 1));
        } else if (WIDE) {
            const long long beta = 2 * aa * bb + 1;
            gam2[j] = (double)(aa + bb - 1);
            kap[j] = (double)beta;
            blo[j] = (double)(beta - (long long)kap[j]);
        } else {
            gam2[j] = (double)(2 * (aa + bb - 1));
            kap[j] = (double)(aa * (aa - 2) + bb * (bb - 2));
        }
    }

    for (int k0 = k_lo; k0 <= k_hi; k0 += KC) {
        const int kc = min(KC, k_hi - k0 + 1);
        const int kc_r = (kc + R - 1) / R * R;           // staged U of steps kc .. kc_r - 1 is 0
        __syncthreads();
        const int g_base = A - k0 - KC + 1;
        const int h_base = A + de + k0;
        const int g_off = KC - kc_r, n_win = B + kc_r - 1;
        for (int i = lane; i < n_win; i += kWave) {
            const int eg = g_base + g_off + i, eh = h_base + i;
            s_g[W::phys(g_off + i)] = (eg >= 0 && eg < a.g_len) ? a.g[eg] : 0.0;
            s_h[W::phys(i)] = (eh >= 0 && eh < a.h_len) ? a.h[eh] : 0.0;
        }
        for (int st = lane; st < kc_r; st += kWave) {
            double uf[2 * NV];
#pragma unroll
            for (int i = 0; i < 2 * NV; ++i) uf[i] = 0.0;
            if (st < kc) {
                const int k = k0 + st;
                const int l3 = de + 2 * k;
                const double gg = a.g[k] * a.g[de + k];
                const long long c = (long long)l3 * (l3 + 1);
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    if (m >= a.n_masks) continue;
                    const double* w = a.wp + (long long)m * a.wp_mask_stride;
                    if (EB)
                        uf[m] = w[2 * a.wp_stride + l3] * gg * (double)(c - (long long)d * (d + 1));
                    else if (TTS)
                        uf[m] = w[l3] * gg;
                    if (TE) uf[NX + m] = w[a.wp_stride + l3] * gg;
                    if (POL) uf[NX + NY + m] = w[2 * a.wp_stride + l3] * gg;
                }
                if (POL || EB) uf[NU - 1] = (double)c;
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) s_u2[st][v] = make_double2(uf[2 * v], uf[2 * v + 1]);
        }
        __syncthreads();

        if (k0 == k_lo) {
#pragma unroll
            for (int j = 0; j < R - 1; ++j) gw[j] = s_g[W::phys(R * lane + j + KC)];
            gw[R - 1] = 0.0;
            hw[0] = 0.0;
#pragma unroll
            for (int j = 1; j < R; ++j) hw[j] = s_h[W::phys(R * lane + j - 1)];
        }
        const double* pg = s_g + (R + 1) * (lane + KC / R - 1) + (R - 1);
        const double* ph = s_h + (R + 1) * lane + (R - 1);
        for (int s0 = 0; s0 < kc_r; s0 += R, pg -= R + 1, ph += R + 1) {
#pragma unroll
            for (int u = 0; u < R; ++u) {
#pragma unroll
                for (int j = R - 1; j > 0; --j) gw[j] = gw[j - 1];
                gw[0] = pg[-u];
#pragma unroll
                for (int j = 0; j < R - 1; ++j) hw[j] = hw[j + 1];
                hw[R - 1] = ph[u + (u >= 1 ? 1 : 0)];
                double uf[2 * NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double2 q2 = s_u2[s0 + u][v];
                    uf[2 * v] = q2.x;
                    uf[2 * v + 1] = q2.y;
                }
                const double c = (POL || EB) ? uf[(POL || EB) ? NU - 1 : 0] : 0.0;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const double P = gw[j] * hw[j];
                    if (EB) {
                        // (sig(sig+1) - c) (c + mu)^2, each factor an exact integer
                        const double f1 = gam2[j] - c;
                        const double f3 = c + kap[j];
                        const double e = P * ((f1 * f3) * f3);
#pragma unroll
                        for (int m = 0; m < M; ++m) tt[j][m] = __builtin_fma(uf[m], e, tt[j][m]);
                        continue;
                    }
                    if (TTS)
#pragma unroll
                        for (int m = 0; m < M; ++m) tt[j][m] = __builtin_fma(uf[m], P, tt[j][m]);
                    if (POL) {
                        double N;
                        if (WIDE) {
                            const double t = c - gam2[j];
                            N = __builtin_fma(t, t, -kap[j]) - blo[j];
                        } else {
                            const double dc = c - gam2[j];
                            N = __builtin_fma(c, dc, kap[j]);
                        }
                        const double y = P * N;
                        if (TE)
#pragma unroll
                            for (int m = 0; m < M; ++m) te[j][m] = __builtin_fma(uf[NX + m], y, te[j][m]);
                        const double z = y * N;
#pragma unroll
                        for (int m = 0; m < M; ++m) ee[j][m] = __builtin_fma(uf[NX + NY + m], z, ee[j][m]);
                    }
                }
            }
        }
    }

#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (m >= a.n_masks || d > a.m_lmax[m]) continue;
        double* xm = a.xi + a.m_xi[m] + diag_offset(a.m_lmax[m], d);
        const long long st = a.m_stride[m];
        const int rows = a.m_lmax[m] - d + 1;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int l1 = l1_0 + j;
            if (l1 < 0 || l1 >= rows) continue;
            const double sc = (POL || EB) ? 0.5 * a.cl[l1] * a.cl[l1 + d] : 0.0;
            if (EB) {
                xm[3 * st + l1] = (sc * sc) * tt[j][m];
                continue;
            }
            if (TTS) xm[l1] = tt[j][m];
            if (TE) xm[st + l1] = sc * te[j][m];
            if (POL) xm[2 * st + l1] = (sc * sc) * ee[j][m];
        }
    }
}

}  // namespace

hipError_t launch_scale_windows(const couple_ctx* ctx, const double* wtt, const double* wtp,
                                const double* wpp, int n, hipStream_t s) {
    const int stride = 2 * ctx->lmax_max + 1;
    hipLaunchKernelGGL(scale_windows_kernel, dim3((n + 255) / 256), dim3(256), 0, s, wtt, wtp, wpp, n,
                       stride, ctx->wp, ctx->wpf);
    return hipGetLastError();
}

hipError_t launch_window_exponents(const couple_ctx* ctx, int n, hipStream_t s, int n_masks) {
    const int stride = 2 * ctx->lmax_max + 1;
    hipLaunchKernelGGL(window_exponents_kernel, dim3(6, n_masks), dim3(kExpThreads), 0, s, ctx->wp, n, stride,
                       ctx->wexp);
    return hipGetLastError();
}

hipError_t launch_scale_windows_masks(const couple_ctx* ctx, const double* const* wtt, const double* const* wtp,
                                      const double* const* wpp, int n_masks, int n, const int* n_m, hipStream_t s) {
    if (n_masks < 1 || n_masks > kBandMasks) return hipErrorInvalidValue;
    MaskWindows w;
    for (int m = 0; m < kBandMasks; ++m) {
        const bool on = m < n_masks;
        w.w[m][0] = on && wtt ? wtt[m] : nullptr;
        w.w[m][1] = on && wtp ? wtp[m] : nullptr;
        w.w[m][2] = on && wpp ? wpp[m] : nullptr;
        w.n[m] = on ? std::min(n, n_m ? n_m[m] : n) : 0;
    }
    hipLaunchKernelGGL(scale_windows_masks_kernel, dim3((n + 255) / 256, n_masks), dim3(256), 0, s, w, n,
                       2 * ctx->lmax_max + 1, ctx->wp);
    return hipGetLastError();
}

// Items of the strip grid (see strip_item).
static long long count_items(int lmax, int dmax, int B, bool band) {
    if (band) {
        const long long J = (lmax + B) / B;
        return J * (dmax + 1);
    }
    const long long M = lmax / B;
    return (long long)B * (M + 1) * (M + 2) / 2;
}

namespace {

// The polarised and EB modes for one row count R per lane.
template <int R>
hipError_t launch_strip_modes(const couple_ctx* ctx, const StripArgs& a, int lmax, int mode, int precision,
                              long long n_items, hipStream_t s) {
    const dim3 grid((unsigned)n_items), block(kWave);
    if (precision == COUPLE_FP32C) {
        const float* gf = ctx->gf_pad + kTablePad;
        const float* hf = ctx->hf_pad + kTablePad;
        if (mode == kStripEB)
            hipLaunchKernelGGL((strip_fp32c_kernel<R, kModeEB>), grid, block, 0, s, a, gf, hf);
        else if (mode == kStripPol)
            hipLaunchKernelGGL((strip_fp32c_kernel<R, kModePol>), grid, block, 0, s, a, gf, hf);
        else if (mode == kStripPolEE)
            hipLaunchKernelGGL((strip_fp32c_kernel<R, kModePolEE>), grid, block, 0, s, a, gf, hf);
        else if (mode == kStripEE)
            hipLaunchKernelGGL((strip_fp32c_kernel<R, kModeEE>), grid, block, 0, s, a, gf, hf);
        else
            return hipErrorInvalidValue;
    } else {
        if (mode == kStripEB)
            hipLaunchKernelGGL((strip_fp64_kernel<R, kModeEB, false>), grid, block, 0, s, a);
        else if (mode == kStripPol && lmax > kNarrowLmax)
            hipLaunchKernelGGL((strip_fp64_kernel<R, kModePol, true>), grid, block, 0, s, a);
        else if (mode == kStripPol)
            hipLaunchKernelGGL((strip_fp64_kernel<R, kModePol, false>), grid, block, 0, s, a);
        else if (mode == kStripPolEE && lmax > kNarrowLmax)
            hipLaunchKernelGGL((strip_fp64_kernel<R, kModePolEE, true>), grid, block, 0, s, a);
        else if (mode == kStripPolEE)
            hipLaunchKernelGGL((strip_fp64_kernel<R, kModePolEE, false>), grid, block, 0, s, a);
        else if (mode == kStripEE && lmax > kNarrowLmax)
            hipLaunchKernelGGL((strip_fp64_kernel<R, kModeEE, true>), grid, block, 0, s, a);
        else if (mode == kStripEE)
            hipLaunchKernelGGL((strip_fp64_kernel<R, kModeEE, false>), grid, block, 0, s, a);
        else
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_strip(const couple_ctx* ctx, int lmax, int mode, int precision, int l3_lo, int l3_hi,
                        hipStream_t s) {
    constexpr int R = kStripR;
    StripArgs a;
    a.g = ctx->g_pad + kTablePad;
    a.h = ctx->h_pad + kTablePad;
    a.wp = ctx->wp;
    a.wexp = ctx->wexp;
    a.cl = ctx->cl;
    a.xi = ctx->xi;
    a.xi_stride = tri_size(lmax);
    a.wp_stride = 2 * ctx->lmax_max + 1;
    a.g_len = ctx->lmax_max + 1;
    a.h_len = 2 * ctx->lmax_max + 1;
    a.lmax = lmax;
    a.dmax = std::min(lmax, l3_hi);
    a.l3_lo = l3_lo;
    a.l3_hi = l3_hi;
    a.band = a.dmax < lmax ? 1 : 0;
    if (mode == kStripTT) {
        constexpr int RT = kStripRTT;
        const long long n_tt = count_items(lmax, a.dmax, kWave * RT, a.band != 0);
        if (n_tt <= 0) return hipSuccess;
        if (n_tt > 0x7fffffffLL) return hipErrorInvalidValue;
        const dim3 grid((unsigned)n_tt), block(kWave);
        if (precision == COUPLE_FP32C)
            hipLaunchKernelGGL((strip_fp32c_kernel<RT, kModeTT>), grid, block, 0, s, a, ctx->gf_pad + kTablePad,
                               ctx->hf_pad + kTablePad);
        else
            hipLaunchKernelGGL((strip_fp64_kernel<RT, kModeTT, false>), grid, block, 0, s, a);
        return hipGetLastError();
    }
    // 256-row blocks (R = 4) unless they would leave the chip short of work
    // items: then 128-row blocks (R = 2)
    const long long n4 = count_items(lmax, a.dmax, kWave * R, a.band != 0);
    if (n4 <= 0) return hipSuccess;
    if (n4 < (precision == COUPLE_FP32C ? kStripSmallItemsF32 : kStripSmallItemsF64)) {
        const long long n2 = count_items(lmax, a.dmax, kWave * kStripRSmall, a.band != 0);
        if (n2 > 0x7fffffffLL) return hipErrorInvalidValue;
        return launch_strip_modes<kStripRSmall>(ctx, a, lmax, mode, precision, n2, s);
    }
    if (n4 > 0x7fffffffLL) return hipErrorInvalidValue;
    return launch_strip_modes<R>(ctx, a, lmax, mode, precision, n4, s);
}

int strip_masks_per_launch(int mode, int precision) {
    if (precision == COUPLE_FP64) return mode == kStripPolEE ? kMasksPolEEF64 : mode == kStripPol ? kMasksPolF64 : kBandMasks;
    return mode == kStripPolEE ? kMasksPolEE : mode == kStripPol ? kMasksPol : kBandMasks;
}

bool strip_masks_bitwise(int mode, int precision, int lmax, int l3_hi) {
    // FP32C's EB rows round f1 and f3 from the lane's first row: a lane must hold the
    // same rows as in launch_strip, which drops to kStripRSmall rows per lane on
    // small item counts
    if (mode != kStripEB || precision != COUPLE_FP32C) return true;
    const int dmax = std::min(lmax, l3_hi);
    return count_items(lmax, dmax, kWave * kStripR, dmax < lmax) >= kStripSmallItemsF32;
}

hipError_t launch_strip_masks(const couple_ctx* ctx, int mode, int precision, int n_masks, const int* lmax_m,
                              double* xi, const long long* xi_off, int l3_lo, int l3_hi, hipStream_t s) {
    if (n_masks < 1 || n_masks > strip_masks_per_launch(mode, precision)) return hipErrorInvalidValue;
    int lmax = 0;
    for (int m = 0; m < n_masks; ++m) lmax = std::max(lmax, lmax_m[m]);
    StripArgs a;
    a.g = ctx->g_pad + kTablePad;
    a.h = ctx->h_pad + kTablePad;
    a.wp = ctx->wp;
    a.wexp = ctx->wexp;
    a.cl = ctx->cl;
    a.xi = xi;
    a.xi_stride = 0;
    a.wp_stride = 2 * ctx->lmax_max + 1;
    a.g_len = ctx->lmax_max + 1;
    a.h_len = 2 * ctx->lmax_max + 1;
    a.lmax = lmax;
    a.dmax = std::min(lmax, l3_hi);
    a.l3_lo = l3_lo;
    a.l3_hi = l3_hi;
    a.band = a.dmax < lmax ? 1 : 0;
    a.n_masks = n_masks;
    a.wp_mask_stride = 3 * a.wp_stride;
    for (int m = 0; m < kBandMasks; ++m) {
        const bool on = m < n_masks;
        a.m_lmax[m] = on ? lmax_m[m] : -1;
        a.m_xi[m] = on ? xi_off[m] : 0;
        // a mask's Xi triangles hold its diagonals 0 .. min(its lmax, l3_hi)
        a.m_stride[m] = on ? diag_offset(lmax_m[m], std::min(lmax_m[m], l3_hi) + 1) : 0;
    }
    const long long n_items = count_items(lmax, a.dmax, kWave * kStripR, a.band != 0);
    if (n_items <= 0) return hipSuccess;
    if (n_items > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)n_items), block(kWave);
    const float* gf = ctx->gf_pad + kTablePad;
    const float* hf = ctx->hf_pad + kTablePad;
    if (precision == COUPLE_FP64) {
        const bool wide = lmax > kNarrowLmax;
        if (mode == kStripPolEE && wide)
            hipLaunchKernelGGL((strip_fp64_masks_kernel<kModePolEE, kMasksPolEEF64, true>), grid, block, 0, s, a);
        else if (mode == kStripPolEE)
            hipLaunchKernelGGL((strip_fp64_masks_kernel<kModePolEE, kMasksPolEEF64, false>), grid, block, 0, s, a);
        else if (mode == kStripPol && wide)
            hipLaunchKernelGGL((strip_fp64_masks_kernel<kModePol, kMasksPolF64, true>), grid, block, 0, s, a);
        else if (mode == kStripPol)
            hipLaunchKernelGGL((strip_fp64_masks_kernel<kModePol, kMasksPolF64, false>), grid, block, 0, s, a);
        else if (mode == kStripTT)
            hipLaunchKernelGGL((strip_fp64_masks_kernel<kModeTT, kBandMasks, false>), grid, block, 0, s, a);
        else if (mode == kStripEE && wide)
            hipLaunchKernelGGL((strip_fp64_masks_kernel<kModeEE, kBandMasks, true>), grid, block, 0, s, a);
        else if (mode == kStripEE)
            hipLaunchKernelGGL((strip_fp64_masks_kernel<kModeEE, kBandMasks, false>), grid, block, 0, s, a);
        else if (mode == kStripEB)
            hipLaunchKernelGGL((strip_fp64_masks_kernel<kModeEB, kBandMasks, false>), grid, block, 0, s, a);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    constexpr int G = kCompBlock, CP = kCompPeriod;
    if (mode == kStripPolEE)
        hipLaunchKernelGGL((strip_fp32c_masks_kernel<kModePolEE, kMasksPolEE, G, CP>), grid, block, 0, s, a, gf, hf);
    else if (mode == kStripPol)
        hipLaunchKernelGGL((strip_fp32c_masks_kernel<kModePol, kMasksPol, G, CP>), grid, block, 0, s, a, gf, hf);
    else if (mode == kStripTT)
        hipLaunchKernelGGL((strip_fp32c_masks_kernel<kModeTT, kBandMasks, G, CP>), grid, block, 0, s, a, gf, hf);
    else if (mode == kStripEE)
        hipLaunchKernelGGL((strip_fp32c_masks_kernel<kModeEE, kBandMasks, G, CP>), grid, block, 0, s, a, gf, hf);
    else if (mode == kStripEB)
        hipLaunchKernelGGL((strip_fp32c_masks_kernel<kModeEB, kBandMasks, G, CP>), grid, block, 0, s, a, gf, hf);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace couple

