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

}  // namespace

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
