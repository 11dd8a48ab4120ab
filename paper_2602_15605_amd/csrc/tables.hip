// Look-up tables of Sec. 3.1: g(p) = (2p)!/(2^{2p} (p!)^2) from the
// recurrence g(p) = (p - 1/2)/p * g(p-1), g(0) = 1 (eq. g_rec), the
// reciprocal 1/((2p+1) g(p)) (eq. 000_sq_main with J + 1 = 2p + 1), and
// c_l = [(l-1) l (l+1)(l+2)]^{-1/2} (the 1/(lambda eta) factor of App. B.3).
//
// The paper accumulates ln g(p) and exponentiates; here the running product
// itself is carried in double-double (about 106 bits) so that the float64
// tables come out rounded once from a value accurate far below their
// half-ulp.  One work-group computes the whole prefix product: each thread
// multiplies out a contiguous segment of ratios, the segment products are
// combined by an exclusive scan in LDS, and each thread then walks its
// segment again.
#include "couple_internal.hpp"

namespace couple {
namespace {

struct dd {
    double hi, lo;
};

// The error-free transforms below rely on every product and sum being
// rounded separately: no contraction into fused multiply-adds except the
// explicit __builtin_fma calls.
#pragma clang fp contract(off)

__device__ inline dd dd_fast_two_sum(double a, double b) {
    const double s = a + b;
    const double e = b - (s - a);
    return {s, e};
}

__device__ inline dd dd_mul(dd a, dd b) {
    const double p = a.hi * b.hi;
    const double e = __builtin_fma(a.hi, b.hi, -p);
    const double lo = e + (a.hi * b.lo + a.lo * b.hi);
    return dd_fast_two_sum(p, lo);
}

// (2p - 1)/(2p) as a double-double (p >= 1).
__device__ inline dd dd_ratio(int p) {
    const double num = 2.0 * p - 1.0, den = 2.0 * p;
    const double q = num / den;
    const double r = __builtin_fma(-q, den, num);  // exact residual
    return dd_fast_two_sum(q, r / den);
}

// y * x for a double-double y and a double x.
__device__ inline dd dd_scale(dd y, double x) {
    const double p = y.hi * x;
    const double e = __builtin_fma(y.hi, x, -p) + y.lo * x;
    return dd_fast_two_sum(p, e);
}

// 1/y for a double-double y > 0 (one Newton step on the float64 reciprocal).
__device__ inline dd dd_recip(dd y) {
    const double r = 1.0 / y.hi;
    const double p = y.hi * r;
    const double pe = __builtin_fma(y.hi, r, -p);
    const double e = ((1.0 - p) - pe) - y.lo * r;  // 1 - y r
    return dd_fast_two_sum(r, r * e);
}

#pragma clang fp contract(on)

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads)
build_tables_kernel(int lmax_max, double* __restrict__ g_pad, double* __restrict__ h_pad,
                    float* __restrict__ gf_pad, float* __restrict__ hf_pad,
                    double* __restrict__ cl) {
    __shared__ double s_hi[kThreads];
    __shared__ double s_lo[kThreads];
    const int t = threadIdx.x;
    const int n = 2 * lmax_max + 1;              // p = 0 .. 2 lmax_max
    const int seg = (n + kThreads - 1) / kThreads;
    const int p0 = t * seg, p1 = min(n, p0 + seg);

    // product of the ratios of this segment (ratio(p) takes g(p-1) to g(p))
    dd acc = {1.0, 0.0};
    for (int p = max(p0, 1); p < p1; ++p) acc = dd_mul(acc, dd_ratio(p));
    s_hi[t] = acc.hi;
    s_lo[t] = acc.lo;
    __syncthreads();
    // inclusive Hillis-Steele scan of the segment products
    for (int off = 1; off < kThreads; off <<= 1) {
        dd mine = {s_hi[t], s_lo[t]};
        if (t >= off) mine = dd_mul(dd{s_hi[t - off], s_lo[t - off]}, mine);
        __syncthreads();
        s_hi[t] = mine.hi;
        s_lo[t] = mine.lo;
        __syncthreads();
    }
    dd g = (t == 0) ? dd{1.0, 0.0} : dd{s_hi[t - 1], s_lo[t - 1]};  // g(p0 - 1) or g(0)
    double* g_tab = g_pad + kTablePad;
    double* h_tab = h_pad + kTablePad;
    float* gf_tab = gf_pad + kTablePad;
    float* hf_tab = hf_pad + kTablePad;
    for (int p = p0; p < p1; ++p) {
        if (p >= 1) g = dd_mul(g, dd_ratio(p));
        // here g = g(p)
        if (p <= lmax_max) {
            g_tab[p] = g.hi;
            gf_tab[p] = (float)g.hi;
        }
        const dd h = dd_recip(dd_scale(g, 2.0 * p + 1.0));
        h_tab[p] = h.hi;
        hf_tab[p] = (float)h.hi;
    }
    // zero guard bands
    for (int i = t; i < kTablePad; i += kThreads) {
        g_pad[i] = 0.0;
        gf_pad[i] = 0.0f;
        h_pad[i] = 0.0;
        hf_pad[i] = 0.0f;
        g_pad[kTablePad + lmax_max + 1 + i] = 0.0;
        gf_pad[kTablePad + lmax_max + 1 + i] = 0.0f;
        h_pad[kTablePad + n + i] = 0.0;
        hf_pad[kTablePad + n + i] = 0.0f;
    }
    // c_l: the product (l-1) l (l+1)(l+2) < 2^56 is rounded once
    for (int l = t; l <= lmax_max; l += kThreads) {
        if (l < 2) {
            cl[l] = 0.0;
        } else {
            const double x = (double)((long long)(l - 1) * l) * (double)((long long)(l + 1) * (l + 2));
            cl[l] = 1.0 / sqrt(x);
        }
    }
}

}  // namespace

hipError_t launch_build_tables(couple_ctx* ctx, hipStream_t s) {
    hipLaunchKernelGGL(build_tables_kernel, dim3(1), dim3(kThreads), 0, s, ctx->lmax_max, ctx->g_pad,
                       ctx->h_pad, ctx->gf_pad, ctx->hf_pad, ctx->cl);
    return hipGetLastError();
}

}  // namespace couple
