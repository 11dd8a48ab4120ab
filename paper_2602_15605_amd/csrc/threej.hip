// Rows of Wigner 3j symbols (l1 l2 l3; -m m 0), m = 0, 1, 2, over every
// l3 = |l1 - l2| .. l1 + l2, from the g(p) tables in closed form.
//
// (0 0 0): eq. 000_sq_main, X^2 = g(P-l1) g(P-l2) g(P-l3) / ((2P+1) g(P)),
//   P = L/2, sign (-1)^P, zero for odd L (L = l1 + l2 + l3).
// (-1 1 0) = (l3 l1 l2; 0 -1 1) (cyclic), the J_(-1,1) family of App. B:
//   odd L  (eq. joneodd with (j1, j2, j3) = (l3, l1, l2)):
//     -1/2 [(L+2)(L-2 l3+1)(L-2 l1+1)(L-2 l2) / (a b)]^{1/2} (l1, l2+1, l3; 0 0 0);
//   even L: eq. joneeven's two (0 0 0) terms of opposite sign collapse, by the
//     (0 0 0) ratio of eq. g_rec, to the single product
//     -(l1 l2 l3; 0 0 0) (a + b - c) / (2 sqrt(a b)),
//   with a = l1(l1+1), b = l2(l2+1), c = l3(l3+1); zero for l1 or l2 < 1.
// (-2 2 0): App. B.3 (eq. 022_linear_closedform) for even L,
//     X N' c_l1 c_l2 / 2,  N' = c (c - 2(a+b-1)) + a(a-2) + b(b-2);
//   odd L (eq. 022_rearranged with eqs. joneodd, joneevensimp at j3 + 1):
//     -Y' (c + mu) (c_l1 c_l2 / 2) [(sig(sig+1) - c)(c - d(d+1))]^{1/2},
//     Y' = (l1, l2+1, l3; 0 0 0), sig = l1 + l2 + 1, tau = sig + 1,
//     mu = 2 (l1+2)(l2+2) - tau(tau+1), d = l2 - l1;
//   zero for l1 or l2 < 2.
// Every integer factor is exact in int64; the only roundings are the table
// values, the products and one square root, so there is no cancellation.
//
// The second kernel below extends this to (l1 l2 l3; m1 m2 m3) with small
// magnetic numbers, (1 1 -2) and (2 2 -4) among them.
//
// One 256-thread work-group per (l1, l2) pair, threads over l3.  The pairs
// are read from device memory, so the kernel itself checks them: a pair
// outside [0, lmax_max] gives a row of NaN and reads no table.
#include "couple_internal.hpp"

namespace couple {
namespace {

constexpr int kThreejThreads = 256;
constexpr int kThreejBatch = 4;

struct ThreejArgs {
    const double* g;             // g(p), p = 0 .. lmax_max
    const double* h;             // 1/((2p+1) g(p)), p = 0 .. 2 lmax_max
    const double* cl;            // c_l, l = 0 .. lmax_max
    const int* l1;
    const int* l2;
    double* out;                 // [n_pairs][stride]
    long long stride;
    int lmax_max;
    int m;
};

// (j1 j2 j3; 0 0 0) with the triangle rule; every index stays inside the
// tables when j1, j2 <= lmax_max + 1 and j3 <= j1 + j2 - 1 or j1, j2 <= lmax_max.
__device__ inline double x000(const ThreejArgs& a, long long j1, long long j2, long long j3) {
    const long long L = j1 + j2 + j3;
    if (L & 1) return 0.0;
    if (j3 < (j1 > j2 ? j1 - j2 : j2 - j1) || j3 > j1 + j2) return 0.0;
    const long long P = L / 2;
    const double v = sqrt(a.g[P - j1] * a.g[P - j2] * a.g[P - j3] * a.h[P]);
    return (P & 1) ? -v : v;
}

// m = 1, 2, with rowf from row_factor.  Both parities share one (0 0 0)
// evaluation: (l1 l2 l3) for even L and (l1, l2+1, l3) for odd L, whose total
// is then even.  Neighbouring l3 alternate in parity, so the two factors are
// both formed and one is selected per lane, which keeps the wave on a single
// path.  The factor of the parity not taken can be the root of a negative
// number; it is discarded.
__device__ inline double symbol(const ThreejArgs& a, long long l1, long long l2, long long l3, double rowf) {
    const long long L = l1 + l2 + l3;
    const long long odd = L & 1;
    const double x = x000(a, l1, l2 + odd, l3);
    const long long A = l1 * (l1 + 1), B = l2 * (l2 + 1), C = l3 * (l3 + 1);
    if (a.m == 1) {
        if (l1 < 1 || l2 < 1) return 0.0;
        const double num = (double)((L + 2) * (L - 2 * l3 + 1)) * (double)((L - 2 * l1 + 1) * (L - 2 * l2));
        const double f = odd ? sqrt(num) : (double)(A + B - C);
        return f * rowf * x;
    }
    if (l1 < 2 || l2 < 2) return 0.0;
    const long long np = C * (C - 2 * (A + B - 1)) + A * (A - 2) + B * (B - 2);
    const long long sg = l1 + l2 + 1, tau = sg + 1, d = l2 - l1;
    const long long mu = 2 * (l1 + 2) * (l2 + 2) - tau * (tau + 1);
    const long long f1 = sg * (sg + 1) - C, f2 = C - d * (d + 1);
    const double f = odd ? -(double)(C + mu) * sqrt((double)f1 * (double)f2) : (double)np;
    return x * f * rowf;
}

// The factor shared by a whole row: m = 1: -1 / (2 sqrt(a b)); m = 2: c_l1 c_l2 / 2.
__device__ inline double row_factor(const ThreejArgs& a, long long l1, long long l2) {
    if (a.m == 1) return (l1 < 1 || l2 < 1) ? 0.0 : -0.5 / sqrt((double)(l1 * (l1 + 1)) * (double)(l2 * (l2 + 1)));
    if (a.m == 2) return (l1 < 2 || l2 < 2) ? 0.0 : 0.5 * a.cl[l1] * a.cl[l2];
    return 1.0;
}

// Each thread computes kThreejBatch symbols of its row before it stores any,
// so their table reads are in flight together.  For m = 0 the symbols of odd
// L vanish; a row starts at L = 2 max(l1, l2), so its even entries are the
// even-L ones, and each thread takes a pair of entries: it evaluates the even
// one and writes a zero beside it.
__global__ void __launch_bounds__(kThreejThreads) threej_rows_kernel(ThreejArgs a) {
    const long long p = blockIdx.x;
    const int l1 = a.l1[p], l2 = a.l2[p];
    double* row = a.out + p * a.stride;
    if (l1 < 0 || l2 < 0 || l1 > a.lmax_max || l2 > a.lmax_max) {
        for (long long i = threadIdx.x; i < a.stride; i += kThreejThreads) row[i] = __builtin_nan("");
        return;
    }
    const long long jmin = l1 > l2 ? l1 - l2 : l2 - l1;
    const long long n = (long long)l1 + l2 - jmin + 1;
    if (a.m == 0) {
        for (long long q0 = threadIdx.x; 2 * q0 < a.stride; q0 += (long long)kThreejThreads * kThreejBatch) {
            double v[kThreejBatch];
#pragma unroll
            for (int q = 0; q < kThreejBatch; ++q) {
                const long long i = 2 * (q0 + (long long)q * kThreejThreads);
                v[q] = i < n ? x000(a, l1, l2, jmin + i) : 0.0;
            }
#pragma unroll
            for (int q = 0; q < kThreejBatch; ++q) {
                const long long i = 2 * (q0 + (long long)q * kThreejThreads);
                if (i < a.stride) row[i] = v[q];
                if (i + 1 < a.stride) row[i + 1] = 0.0;
            }
        }
        return;
    }
    const double rowf = row_factor(a, l1, l2);
    for (long long i0 = threadIdx.x; i0 < a.stride; i0 += (long long)kThreejThreads * kThreejBatch) {
        double v[kThreejBatch];
#pragma unroll
        for (int q = 0; q < kThreejBatch; ++q) {
            const long long i = i0 + (long long)q * kThreejThreads;
            v[q] = i < n ? symbol(a, l1, l2, jmin + i, rowf) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kThreejBatch; ++q) {
            const long long i = i0 + (long long)q * kThreejThreads;
            if (i < a.stride) row[i] = v[q];
        }
    }
}

// ---------------------------------------------------------------------------
// Rows of (l1 l2 l3; m1 m2 m3), m3 = -m1 - m2, for small magnetic numbers: the
// (1 1 -2) and (2 2 -4) families of the Conclusion and their relatives.
//
// Every triple with zero sum has two entries of one sign (or zero) and one of
// the other.  A cyclic permutation of the columns (no sign) puts the odd one
// last and, when the first two are <= 0, the m-flip (a factor (-1)^L) makes
// them >= 0.  The host does this once per call (same for every element); what
// is left is F_ab(x, y, z) = (x y z; a b -a-b) with 0 <= a, b <= 2, where
// (x, y, z) is the rotated (l1, l2, l3).
//
// On the lines a = 0 and b = 0 F_ab is an App. B symbol: (0 -1 1) and
// (0 -2 2) up to a permutation and an m-flip.  The lowering relation of E57
// Sec. 3.7,
//   sqrt((x+a)(x-a+1)) F_{a-1,b} + sqrt((y+b)(y-b+1)) F_{a,b-1}
//     + sqrt((z+a+b)(z-a-b+1)) F_ab = 0,
// fills the quadrant from them.  Taken numerically that relation cancels where
// z << x ~ y (its two large terms nearly cancel; about 2e-6 relative for
// (2 2 -4) near l = 6000), so the chain is collapsed symbolically to one
// closed form per family and parity:
//   even L:  F_ab = X N_ab(A, B, C) / (2 D_ab),   X = (x y z; 0 0 0),
//   odd L:   F_ab = W N_ab(A, B, C) / (2 D_ab),
//            W = (-1)^P [8 p1 p2 p3 (L+2) g(p1) g(p2) g(p3) h(P)]^{1/2},
//            P = (L+1)/2, p_i = P - l_i; W equals
//            (x, y, z+1; 0 0 0) [(L+2)(L+1-2x)(L+1-2y)(L-2z)]^{1/2}, the odd-L
//            form of App. B, written symmetrically;
//   D_ab^2 = prod_{k<a} (A - k(k+1)) prod_{k<b} (B - k(k+1)) prod_{k<a+b} (C - k(k+1)),
//   A = x(x+1), B = y(y+1), C = z(z+1),
// with the integer polynomials N_ab of family_numerator.  N_ab is evaluated
// exactly in 128-bit integers (below 2^118 for l <= 16384; A, B, C and s, t
// are even, so the halvings are exact), so the roundings are its conversion,
// the table product, D_ab and two square roots: no cancellation anywhere.
// Even and odd L alternate along a row; both numerators are formed and one is
// kept per lane, as in symbol() above.

struct FamilyArgs {
    const double* g;
    const double* h;
    const int* l1;
    const int* l2;
    double* out;                 // [n_pairs][stride]
    long long stride;
    int lmax_max;
    int rot;                     // (x, y, z) = (l1, l2, l3) rotated left by rot
    int flip;                    // 1: times (-1)^L
};

// Sign and magnitude, then the two 64-bit words of |v|: the high word
// rounds only above 2^53 (|v| >= 2^117), the low word's rounding (at most
// 2^11) is far below the last place of a result >= 2^64 and exact below it,
// and the sum rounds once.  (Converting a negative v by words would leave
// its low word near 2^64, where that rounding is not negligible.)
__device__ inline double i128_to_double(__int128 v) {
    const bool neg = v < 0;
    const unsigned __int128 m = neg ? (unsigned __int128)(-v) : (unsigned __int128)v;
    const double r = (double)(unsigned long long)(m >> 64) * 18446744073709551616.0 + (double)(unsigned long long)m;
    return neg ? -r : r;
}

// N_ab(A, B, C) for L even (odd = 0) and odd (odd = 1); s = A - B, t = A + B.
template <int AB>
__device__ inline __int128 family_numerator(int odd, __int128 A, __int128 B, __int128 C) {
    const __int128 s = A - B, t = A + B;
    switch (AB) {
    case 0:  // (0 0 0)
        return odd ? 0 : 2;
    case 1:  // (0 1 -1)
        return odd ? (__int128)1 : s - C;
    case 2:  // (0 2 -2)
        return odd ? s - C + 2 : C * C - C * (t + s + 2) + s * s + 2 * s;
    case 3:  // (1 0 -1)
        return odd ? (__int128)-1 : -(s + C);
    case 4:  // (1 1 -2)
        return odd ? -s : C * t - s * s;
    case 5:  // (1 2 -3)
        return odd ? C * A - s * s - 3 * s - t
                   : -C * C * A + C * ((s * s + 3 * s * t) / 2 + s + 3 * t) - s * s * s - 3 * s * s - s * t;
    case 6:  // (2 0 -2)
        return odd ? s + C - 2 : C * C - C * (t - s + 2) + s * s - 2 * s;
    case 7:  // (2 1 -3)
        return odd ? -C * B + s * s - 3 * s + t
                   : -C * C * B + C * ((s * s - 3 * s * t) / 2 - s + 3 * t) + s * s * s - 3 * s * s + s * t;
    default:  // (2 2 -4)
        return odd ? s * (C * (2 - t) + s * s + 4 * t - 12)
                   : C * C * ((s * s + t * t) / 2 - 2 * t) + C * (-2 * s * s * t + s * s - 3 * t * t + 12 * t) +
                         s * s * (s * s + 4 * t - 12);
    }
}

template <int AB>
__device__ inline double family_symbol(const FamilyArgs& f, long long l1, long long l2, long long l3) {
    constexpr int a = AB / 3, b = AB % 3;
    const long long x = f.rot == 0 ? l1 : (f.rot == 1 ? l2 : l3);
    const long long y = f.rot == 0 ? l2 : (f.rot == 1 ? l3 : l1);
    const long long z = f.rot == 0 ? l3 : (f.rot == 1 ? l1 : l2);
    if (x < a || y < b || z < a + b) return 0.0;
    const long long L = l1 + l2 + l3;
    const int odd = (int)(L & 1);
    const long long P = (L + 1) / 2;
    const long long p1 = P - l1, p2 = P - l2, p3 = P - l3;
    const long long A = x * (x + 1), B = y * (y + 1), C = z * (z + 1);
    double base = f.g[p1] * f.g[p2] * f.g[p3] * f.h[P];
    if (odd) base *= (double)(8 * p1 * p2 * p3) * (double)(L + 2);
    double d2 = 1.0;
#pragma unroll
    for (int k = 0; k < a; ++k) d2 *= (double)(A - k * (k + 1));
#pragma unroll
    for (int k = 0; k < b; ++k) d2 *= (double)(B - k * (k + 1));
#pragma unroll
    for (int k = 0; k < a + b; ++k) d2 *= (double)(C - k * (k + 1));
    const double n = i128_to_double(family_numerator<AB>(odd, A, B, C));
    double v = sqrt(base) * n / (2.0 * sqrt(d2));
    if (P & 1) v = -v;
    if (f.flip && odd) v = -v;
    return v;
}

template <int AB>
__global__ void __launch_bounds__(kThreejThreads) threej_family_kernel(FamilyArgs f) {
    const long long p = blockIdx.x;
    const int l1 = f.l1[p], l2 = f.l2[p];
    double* row = f.out + p * f.stride;
    if (l1 < 0 || l2 < 0 || l1 > f.lmax_max || l2 > f.lmax_max) {
        for (long long i = threadIdx.x; i < f.stride; i += kThreejThreads) row[i] = __builtin_nan("");
        return;
    }
    const long long jmin = l1 > l2 ? l1 - l2 : l2 - l1;
    const long long n = (long long)l1 + l2 - jmin + 1;
    for (long long i0 = threadIdx.x; i0 < f.stride; i0 += (long long)kThreejThreads * kThreejBatch) {
        double v[kThreejBatch];
#pragma unroll
        for (int q = 0; q < kThreejBatch; ++q) {
            const long long i = i0 + (long long)q * kThreejThreads;
            v[q] = i < n ? family_symbol<AB>(f, l1, l2, jmin + i) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kThreejBatch; ++q) {
            const long long i = i0 + (long long)q * kThreejThreads;
            if (i < f.stride) row[i] = v[q];
        }
    }
}

}  // namespace

hipError_t launch_threej_family(const couple_ctx* ctx, int rot, int flip, int a, int b, int n_pairs, const int* l1,
                                const int* l2, double* out, long long stride, hipStream_t s) {
    FamilyArgs f;
    f.g = ctx->g_pad + kTablePad;
    f.h = ctx->h_pad + kTablePad;
    f.l1 = l1;
    f.l2 = l2;
    f.out = out;
    f.stride = stride;
    f.lmax_max = ctx->lmax_max;
    f.rot = rot;
    f.flip = flip;
    const dim3 grid((unsigned)n_pairs), block(kThreejThreads);
    switch (3 * a + b) {
    case 0: hipLaunchKernelGGL(threej_family_kernel<0>, grid, block, 0, s, f); break;
    case 1: hipLaunchKernelGGL(threej_family_kernel<1>, grid, block, 0, s, f); break;
    case 2: hipLaunchKernelGGL(threej_family_kernel<2>, grid, block, 0, s, f); break;
    case 3: hipLaunchKernelGGL(threej_family_kernel<3>, grid, block, 0, s, f); break;
    case 4: hipLaunchKernelGGL(threej_family_kernel<4>, grid, block, 0, s, f); break;
    case 5: hipLaunchKernelGGL(threej_family_kernel<5>, grid, block, 0, s, f); break;
    case 6: hipLaunchKernelGGL(threej_family_kernel<6>, grid, block, 0, s, f); break;
    case 7: hipLaunchKernelGGL(threej_family_kernel<7>, grid, block, 0, s, f); break;
    case 8: hipLaunchKernelGGL(threej_family_kernel<8>, grid, block, 0, s, f); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_threej_rows(const couple_ctx* ctx, int m, int n_pairs, const int* l1, const int* l2, double* out,
                              long long stride, hipStream_t s) {
    ThreejArgs a;
    a.g = ctx->g_pad + kTablePad;
    a.h = ctx->h_pad + kTablePad;
    a.cl = ctx->cl;
    a.l1 = l1;
    a.l2 = l2;
    a.out = out;
    a.stride = stride;
    a.lmax_max = ctx->lmax_max;
    a.m = m;
    hipLaunchKernelGGL(threej_rows_kernel, dim3((unsigned)n_pairs), dim3(kThreejThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace couple
