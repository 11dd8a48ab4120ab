// Binned MASTER solve (Sec. 2, eq. pseudo_cl).
//
// The expectation of the pseudo-spectra is linear in the true spectra:
//   <C~^TT> = K^TT C^TT,
//   <C~^EE> = K^EE C^EE + K^EB C^BB,   <C~^BB> = K^EB C^EE + K^BB C^BB
// (the B-mode line by the structure App. A states: Xi_BB has the form of
// Xi_EE and Xi_BE = Xi_EB).  With the binning of couple_band (row-bin
// average, column-bin sum, C_l constant inside a bin) the binned system is
// K_{b b'} C_{b'} = C~_b, C~_b = (1/n_b) sum_{l in b} C~_l.
//
// bin_spectra_kernel: one thread per (spectrum, bin), the bin's sum in l order.
// master_solve_kernel: one work-group assembles [K | C~] (TT, or the 2 x 2
// block system for E/B) in the caller's workspace, eliminates with partial
// pivoting (largest |pivot|, the first row on ties), keeping the pivot row and
// the multipliers in LDS, and back-substitutes every right-hand side.  The
// trailing update is row by row per wavefront, 64 consecutive columns per
// instruction.  A zero pivot (a singular system) gives NaN in every output.
#include "couple_internal.hpp"

namespace couple {
namespace {

constexpr int kSolveThreads = 1024;
constexpr int kSolveWaves = kSolveThreads / kWave;

struct BinSpecArgs {
    const double* cl;            // [n_spec][cl_stride]
    long long cl_stride;
    double* out;                 // [n_spec][n_bins]
    const int* edges_dev;        // n_bins + 1 edges on the device (n_bins > kInlineBins)
    int inline_edges;
    int edges_in[kInlineBins + 1];
    int n_spec, n_bins;
};

__global__ void __launch_bounds__(256) bin_spectra_kernel(BinSpecArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n_spec * a.n_bins) return;
    const int s = t / a.n_bins, b = t - s * a.n_bins;
    const int* E = a.inline_edges ? a.edges_in : a.edges_dev;
    const int lo = E[b], hi = E[b + 1];
    const double* c = a.cl + (long long)s * a.cl_stride;
    double acc = 0.0;
    for (int l = lo; l < hi; ++l) acc += c[l];
    a.out[(long long)s * a.n_bins + b] = acc / (double)(hi - lo);
}

struct SolveArgs {
    const double* K;             // TT: [n][n]; E/B: [3][n][n] in the order EE, BB, EB
    const double* rhs;           // [n_rhs][m]
    double* work;                // [m][m + n_rhs]
    double* x;                   // [n_rhs][m]
    int n, m, n_rhs, pol;
};

__global__ void __launch_bounds__(kSolveThreads) master_solve_kernel(SolveArgs a) {
    __shared__ double s_row[kSolveMaxCols];      // pivot row
    __shared__ double s_mul[kSolveMaxCols];      // multipliers of the column
    __shared__ double s_red[kSolveThreads];
    __shared__ int s_idx[kSolveThreads];
    const int t = threadIdx.x;
    const int lane = t % kWave, wave = t / kWave;
    const int n = a.n, m = a.m, nr = a.n_rhs;
    const long long ld = (long long)m + nr;
    double* A = a.work;

    // assemble [K | C~]
    for (int r = wave; r < m; r += kSolveWaves) {
        for (int c = lane; c < (int)ld; c += kWave) {
            double v;
            if (c >= m) {
                v = a.rhs[(long long)(c - m) * m + r];
            } else if (!a.pol) {
                v = a.K[(long long)r * n + c];
            } else {
                const int br = r / n, bc = c / n;
                const int blk = br != bc ? 2 : br;    // [EE EB; EB BB]
                v = a.K[((long long)blk * n + (r - br * n)) * n + (c - bc * n)];
            }
            A[r * ld + c] = v;
        }
    }
    __syncthreads();

    bool singular = false;
    for (int k = 0; k < m; ++k) {
        // pivot search over rows k .. m-1 of column k
        double best = -1.0;
        int bi = m;
        for (int i = k + t; i < m; i += kSolveThreads) {
            const double v = fabs(A[i * ld + k]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        s_red[t] = best;
        s_idx[t] = bi;
        __syncthreads();
        for (int w = kSolveThreads / 2; w > 0; w >>= 1) {
            if (t < w) {
                const double o = s_red[t + w];
                const int oi = s_idx[t + w];
                if (o > s_red[t] || (o == s_red[t] && oi < s_idx[t])) {
                    s_red[t] = o;
                    s_idx[t] = oi;
                }
            }
            __syncthreads();
        }
        const int p = s_idx[0];
        if (!(s_red[0] > 0.0)) {             // zero (or NaN) pivot column: the system is singular
            singular = true;
            break;
        }
        // swap rows k and p from column k on; the pivot row goes to LDS
        for (int c = k + t; c < (int)ld; c += kSolveThreads) {
            const double vk = A[k * ld + c], vp = A[p * ld + c];
            s_row[c] = vp;
            if (p != k) {
                A[k * ld + c] = vp;
                A[p * ld + c] = vk;
            }
        }
        __syncthreads();
        for (int i = k + 1 + t; i < m; i += kSolveThreads) s_mul[i] = A[i * ld + k] / s_row[k];
        __syncthreads();
        // trailing update: rows k+1 .. m-1, columns k+1 .. ld-1
        for (int i = k + 1 + wave; i < m; i += kSolveWaves) {
            const double f = s_mul[i];
            double* Ai = A + i * ld;
            for (int c = k + 1 + lane; c < (int)ld; c += kWave) Ai[c] = __builtin_fma(-f, s_row[c], Ai[c]);
        }
        __syncthreads();
    }

    if (singular) {
        for (long long e = t; e < (long long)nr * m; e += kSolveThreads) a.x[e] = __builtin_nan("");
        return;
    }
    // back substitution, every right-hand side at once (columns m .. ld-1 of A)
    for (int i = m - 1; i >= 0; --i) {
        const double u = A[i * ld + i];
        for (int r = t; r < nr; r += kSolveThreads) A[i * ld + m + r] /= u;
        __syncthreads();
        for (int q = wave; q < i; q += kSolveWaves) {
            const double f = A[q * ld + i];
            for (int r = lane; r < nr; r += kWave) A[q * ld + m + r] = __builtin_fma(-f, A[i * ld + m + r], A[q * ld + m + r]);
        }
        __syncthreads();
    }
    for (long long e = t; e < (long long)nr * m; e += kSolveThreads) {
        const int r = (int)(e / m), i = (int)(e - (long long)r * m);
        a.x[e] = A[i * ld + m + r];
    }
}

}  // namespace

hipError_t launch_bin_spectra(const couple_ctx* ctx, int n_spec, const double* cl, int cl_stride,
                              const int* bin_edges_host, int n_bins, double* out, hipStream_t s) {
    BinSpecArgs a;
    a.cl = cl;
    a.cl_stride = cl_stride;
    a.out = out;
    a.edges_dev = ctx->edges_dev;
    a.inline_edges = n_bins <= kInlineBins ? 1 : 0;
    for (int i = 0; i <= kInlineBins; ++i) a.edges_in[i] = (a.inline_edges && i <= n_bins) ? bin_edges_host[i] : 0;
    a.n_spec = n_spec;
    a.n_bins = n_bins;
    const int total = n_spec * n_bins;
    hipLaunchKernelGGL(bin_spectra_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_master_solve(int pol, int n, const double* K, int n_rhs, const double* rhs, double* work,
                               double* x, hipStream_t s) {
    SolveArgs a;
    a.K = K;
    a.rhs = rhs;
    a.work = work;
    a.x = x;
    a.n = n;
    a.m = pol ? 2 * n : n;
    a.n_rhs = n_rhs;
    a.pol = pol;
    if (a.m + n_rhs > kSolveMaxCols) return hipErrorInvalidValue;
    hipLaunchKernelGGL(master_solve_kernel, dim3(1), dim3(kSolveThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace couple
