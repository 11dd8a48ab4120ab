// From the packed upper triangle Xi(l1, l1 + d) to the output matrices.
//
// Xi is symmetric in (l1, l2); K is not: K_{l1 l2} = (2 l2 + 1) Xi(l1, l2)
// (Sec. 2 eqs. K_TT, K_EE; App. A).  The paper fills the lower triangle from
// the upper one (Sec. 4.1); here that is done on Xi, and each 64 x 64 tile
// of K is written with its own column factor.
//
// fill: one work-group per upper tile pair (I <= J) of one job (a Xi store
// and its output matrices; the batched form fills every mask in one launch).  The tile of Xi is read
// diagonal by diagonal (consecutive l1 are consecutive in memory), kept in
// LDS, and written twice: K[l1][l2] row by row and the mirrored tile
// K[l2][l1] = (2 l1 + 1) Xi(l1, l2), also row by row, so both halves are
// coalesced.  K is written once and never read back here, so the stores
// are non-temporal.  K^BB is written from the same LDS values as K^EE.  Xi_EB is
// symmetric as well (the (-2 2 0)^2 of odd L is even under l1 <-> l2).
//
// bin: K_{b b'} = (1/n_b) sum_{l1 in b} sum_{l2 in b'} K_{l1 l2}; one
// work-group per unordered bin pair reads its Xi elements once and writes
// both K_{b b'} and K_{b' b}, reduced in a fixed order.
#include "couple_internal.hpp"

namespace couple {
namespace {

constexpr int kT = 64;           // tile edge
constexpr int kFillThreads = 512;  // 8 waves per tile: more stores in flight per LDS tile

struct FillArgs {
    FillJob job[kMaxFillJobs];
    int n_jobs;
    int n_out;
    int xi_only;                 // write Xi (column factor 1) instead of K
    int src[kMaxOut];            // Xi index of each output
};

__device__ inline void pair_from_index(int t, int n, int* I, int* J) {
    // t enumerates (I, J), I <= J, row by row: row I holds n - I pairs
    int i = 0;
    int rem = t;
    while (rem >= n - i) {
        rem -= n - i;
        ++i;
    }
    *I = i;
    *J = i + rem;
}

__global__ void __launch_bounds__(kFillThreads)
fill_kernel(FillArgs a) {
    __shared__ double tile[kT][kT + 1];
    // job of this block: blocks [block0, block0 + n_tiles (n_tiles + 1) / 2) of each job
    int jb = 0;
    while (jb + 1 < a.n_jobs && (int)blockIdx.x >= a.job[jb + 1].block0) ++jb;
    const FillJob& job = a.job[jb];
    const int lmax = job.lmax;
    int I, J;
    pair_from_index((int)blockIdx.x - job.block0, (lmax + kT) / kT, &I, &J);
    const int r0 = kT * I, c0 = kT * J;
    const int t = threadIdx.x;
    const long long ld = lmax + 1;
    const long long xi_stride = job.xi_stride;
    int last_src = -1;

    for (int o = 0; o < a.n_out; ++o) {
        const int src = a.src[o];
        if (src != last_src) {
            __syncthreads();
            const double* xi = job.xi + (long long)src * xi_stride;
            // diagonals d = dj + dl - 63, dl = 0 .. 126; element (r, c = r + dl - 63)
            for (int idx = t; idx < (2 * kT - 1) * kT; idx += kFillThreads) {
                const int r = idx % kT;
                const int dl = idx / kT;
                const int c = r + dl - (kT - 1);
                if (c < 0 || c >= kT) continue;
                const int l1 = r0 + r, l2 = c0 + c;
                if (l1 > lmax || l2 > lmax || l2 < l1) continue;
                const int d = l2 - l1;
                tile[r][c] = (d <= job.dmax) ? xi[diag_offset(lmax, d) + l1] : 0.0;
            }
            __syncthreads();
            last_src = src;
        }
        double* out = job.out + (long long)o * ld * ld;
        // column factor fs l + 1: 2 l + 1 for K, 1 for Xi
        const double fs = a.xi_only ? 0.0 : 2.0;
        if (I == J) {
            for (int idx = t; idx < kT * kT; idx += kFillThreads) {
                const int r = idx / kT, c = idx % kT;
                const int l1 = r0 + r, l2 = c0 + c;
                if (l1 > lmax || l2 > lmax) continue;
                const double x = (c >= r) ? tile[r][c] : tile[c][r];
                __builtin_nontemporal_store((fs * l2 + 1.0) * x, &out[l1 * ld + l2]);
            }
        } else {
            for (int idx = t; idx < kT * kT; idx += kFillThreads) {
                const int r = idx / kT, c = idx % kT;
                const int l1 = r0 + r, l2 = c0 + c;
                if (l1 <= lmax && l2 <= lmax) __builtin_nontemporal_store((fs * l2 + 1.0) * tile[r][c], &out[l1 * ld + l2]);
            }
            for (int idx = t; idx < kT * kT; idx += kFillThreads) {
                const int c = idx / kT, r = idx % kT;
                const int l1 = r0 + r, l2 = c0 + c;
                if (l1 <= lmax && l2 <= lmax) __builtin_nontemporal_store((fs * l1 + 1.0) * tile[r][c], &out[l2 * ld + l1]);
            }
        }
    }
}

constexpr int kBinThreads = 256;
constexpr int kBinWaves = kBinThreads / kWave;
constexpr int kBinUnroll = 4;    // diagonals per wave with their loads in flight together

struct BinArgs {
    const double* xi;
    long long xi_stride;
    long long xi_mask_stride;    // between the Xi stores of consecutive masks (blockIdx.z)
    double* out;
    long long out_mask_stride;   // between the outputs of consecutive masks
    const int* edges;            // device copy of n_bins + 1 edges (when n_bins > kInlineBins)
    int inline_edges;            // edges are in edges_in
    int edges_in[kInlineBins + 1];
    int n_bins;
    int lmax;
    int dmax;
    int n_out;
    int xi_only;                 // bin Xi instead of K
    int n_src;                   // distinct Xi stores among the outputs
    int src[kMaxOut];            // Xi index of each distinct store
    int slot[kMaxOut];           // which distinct store output i reads
};

// One work-group per row bin bb and two adjacent column bins bc0 = bb +
// 2 blockIdx.x and bc1 = bc0 + 1 (when it exists) on a 2D grid (x: the offset
// pair, up to the widest reach of the band in bins; y: bb), so n_bins up to
// lmax_max + 1 stays within the 32-bit work-item count of each grid dimension.
// Pairs the band does not reach are zeroed before the launch.  Xi(l1, l2) =
// Xi(l2, l1), so every element is read once, from the upper triangle
// (d = l2 - l1 >= 0, lanes over consecutive l1 of one diagonal: contiguous in
// the packed store; with two column bins a diagonal's run covers the whole
// row bin), and feeds both outputs of its pair (bb, bc), bc = bc0 or bc1:
//   out[bb][bc] = (1/n_bb) sum (fs l2 + 1) Xi(l1, l2),
//   out[bc][bb] = (1/n_bc) sum (fs l1 + 1) Xi(l1, l2);
// in a diagonal pair both sums land in out[bb][bb], the d = 0 elements once.
// Outputs that share a Xi store (K^EE and K^BB) share its sums.  Each lane
// sums its own elements in a fixed order, then the waves and the work-group
// reduce in a fixed order, so the result does not depend on timing.  NS = the
// number of distinct stores, so that only their sums take registers.
template <int NS>
__global__ void __launch_bounds__(kBinThreads)
bin_kernel(BinArgs a) {
    __shared__ double red[kBinWaves][4 * NS];
    // mask blockIdx.z of the launch (locals: the argument block stays read-only)
    const double* __restrict__ xis = a.xi + a.xi_mask_stride * blockIdx.z;
    double* __restrict__ outs = a.out + a.out_mask_stride * blockIdx.z;
    const int bb = blockIdx.y, bc0 = blockIdx.y + 2 * blockIdx.x;
    if (bc0 >= a.n_bins) return;
    const bool two = bc0 + 1 < a.n_bins;
    const int* E = a.inline_edges ? a.edges_in : a.edges;
    const int r_lo = E[bb], r_hi = E[bb + 1];
    const int c_lo = E[bc0], c_mid = E[bc0 + 1], c_hi = two ? E[bc0 + 2] : c_mid;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const double fs = a.xi_only ? 0.0 : 2.0;  // column factor fs l2 + 1
    // d = l2 - l1 over both pairs (the bins are ordered and disjoint: d >= 1 off the diagonal)
    const int d_lo = max(c_lo - (r_hi - 1), 0);
    const int d_hi = min(c_hi - 1 - r_lo, a.dmax);
    // sums [0]: pair (bb, bc0), [1]: pair (bb, bc1); a: row-bin orientation, b: mirrored
    double sa[2][NS], sb[2][NS];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int s = 0; s < NS; ++s) sa[q][s] = sb[q][s] = 0.0;
    for (int l1c = r_lo; l1c < r_hi; l1c += kWave) {
        // the diagonals that meet rows l1c .. l1c + 63 of this row bin inside the column bins
        const int row_end = min(l1c + kWave, r_hi);
        const int dk_lo = max(d_lo, c_lo - (row_end - 1)), dk_hi = min(d_hi, c_hi - 1 - l1c);
        const int l1 = l1c + lane;
        for (int d0 = dk_lo + wave; d0 <= dk_hi; d0 += kBinWaves * kBinUnroll) {
            double x[kBinUnroll][NS], wa[kBinUnroll], wb[kBinUnroll];
            bool hi_bin[kBinUnroll];
#pragma unroll
            for (int u = 0; u < kBinUnroll; ++u) {
                const int d = d0 + u * kBinWaves, l2 = l1 + d;
                const bool ok = d <= dk_hi && l1 < row_end && l2 >= c_lo && l2 < c_hi;
                hi_bin[u] = l2 >= c_mid;
                wa[u] = ok ? fs * l2 + 1.0 : 0.0;
                wb[u] = (ok && d > 0) ? fs * l1 + 1.0 : 0.0;
                const long long off = ok ? diag_offset(a.lmax, d) + l1 : 0;
#pragma unroll
                for (int s = 0; s < NS; ++s) x[u][s] = ok ? xis[(long long)a.src[s] * a.xi_stride + off] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kBinUnroll; ++u) {
                const double wa0 = hi_bin[u] ? 0.0 : wa[u], wa1 = hi_bin[u] ? wa[u] : 0.0;
                const double wb0 = hi_bin[u] ? 0.0 : wb[u], wb1 = hi_bin[u] ? wb[u] : 0.0;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    sa[0][s] = __builtin_fma(wa0, x[u][s], sa[0][s]);
                    sb[0][s] = __builtin_fma(wb0, x[u][s], sb[0][s]);
                    sa[1][s] = __builtin_fma(wa1, x[u][s], sa[1][s]);
                    sb[1][s] = __builtin_fma(wb1, x[u][s], sb[1][s]);
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) {
                sa[q][s] += __shfl_down(sa[q][s], off, kWave);
                sb[q][s] += __shfl_down(sb[q][s], off, kWave);
            }
        }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                red[wave][4 * s + 2 * q] = sa[q][s];
                red[wave][4 * s + 2 * q + 1] = sb[q][s];
            }
    }
    __syncthreads();
    const int o = threadIdx.x % kMaxOut, q = threadIdx.x / kMaxOut;   // output o of pair (bb, bc0 + q)
    if (o < a.n_out && q < (two ? 2 : 1)) {
        const int s = a.slot[o];
        const int bc = bc0 + q;
        double A = 0.0, B = 0.0;
        for (int w = 0; w < kBinWaves; ++w) {
            A += red[w][4 * s + 2 * q];
            B += red[w][4 * s + 2 * q + 1];
        }
        double* out = outs + (long long)o * a.n_bins * a.n_bins;
        const int n_bc = E[bc + 1] - E[bc];
        if (bb == bc) {
            out[(long long)bb * a.n_bins + bb] = (A + B) / (double)(r_hi - r_lo);
        } else {
            out[(long long)bb * a.n_bins + bc] = A / (double)(r_hi - r_lo);
            out[(long long)bc * a.n_bins + bb] = B / (double)n_bc;
        }
    }
}

__global__ void zero_kernel(double* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = 0.0;
}

}  // namespace

hipError_t launch_zero(double* out, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, out, n);
    return hipGetLastError();
}

hipError_t launch_fill_jobs(const FillJob* jobs, int n_jobs, const int* spec_src, int n_out, int xi,
                            hipStream_t s) {
    if (n_jobs < 1 || n_jobs > kMaxFillJobs) return hipErrorInvalidValue;
    FillArgs a;
    long long blocks = 0;
    for (int j = 0; j < n_jobs; ++j) {
        a.job[j] = jobs[j];
        a.job[j].block0 = (int)blocks;
        const long long nt = (jobs[j].lmax + kT) / kT;
        blocks += nt * (nt + 1) / 2;
    }
    a.n_jobs = n_jobs;
    a.n_out = n_out;
    a.xi_only = xi;
    for (int i = 0; i < kMaxOut; ++i) a.src[i] = i < n_out ? spec_src[i] : 0;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(kFillThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill(const couple_ctx* ctx, int lmax, int dmax, const int* spec_src, int n_out,
                       double* out, int xi, hipStream_t s, const double* xi_src, long long xi_stride) {
    FillJob j;
    j.xi = xi_src ? xi_src : ctx->xi;
    j.xi_stride = xi_src ? xi_stride : tri_size(lmax);
    j.out = out;
    j.lmax = lmax;
    j.dmax = dmax;
    j.block0 = 0;
    return launch_fill_jobs(&j, 1, spec_src, n_out, xi, s);
}

hipError_t launch_bin(const couple_ctx* ctx, int lmax, int dmax, const int* spec_src, int n_out,
                      const int* bin_edges_host, const int* bin_edges_dev, int n_bins, double* out, int xi,
                      hipStream_t s, const double* xi_src, long long xi_stride, int n_masks,
                      long long xi_mask_stride) {
    if (n_masks < 1 || n_masks > 65535) return hipErrorInvalidValue;
    BinArgs a;
    a.xi = xi_src ? xi_src : ctx->xi;
    a.xi_stride = xi_src ? xi_stride : tri_size(lmax);
    a.xi_mask_stride = xi_mask_stride;
    a.out = out;
    a.out_mask_stride = (long long)n_out * n_bins * n_bins;
    a.edges = bin_edges_dev;
    a.inline_edges = n_bins <= kInlineBins ? 1 : 0;
    for (int i = 0; i <= kInlineBins; ++i) a.edges_in[i] = (a.inline_edges && i <= n_bins) ? bin_edges_host[i] : 0;
    a.n_bins = n_bins;
    a.lmax = lmax;
    a.dmax = dmax;
    a.n_out = n_out;
    a.xi_only = xi;
    // distinct Xi stores, in order of first use
    a.n_src = 0;
    for (int i = 0; i < kMaxOut; ++i) a.src[i] = a.slot[i] = 0;
    for (int i = 0; i < n_out; ++i) {
        int k = 0;
        while (k < a.n_src && a.src[k] != spec_src[i]) ++k;
        if (k == a.n_src) a.src[a.n_src++] = spec_src[i];
        a.slot[i] = k;
    }
    // reach: the largest bc - bb of a pair with an element inside the band
    // (E[bc] - (E[bb + 1] - 1) <= dmax); the bound is monotone in bb
    const int* E = bin_edges_host;
    int reach = 0;
    for (int bb = 0, bc = 0; bb < n_bins; ++bb) {
        if (bc < bb) bc = bb;
        while (bc + 1 < n_bins && E[bc + 1] - (E[bb + 1] - 1) <= dmax) ++bc;
        reach = std::max(reach, bc - bb);
    }
    if (reach + 1 < n_bins) {
        const hipError_t e = launch_zero(out, (size_t)n_masks * n_out * n_bins * n_bins, s);
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)((reach + 2) / 2), (unsigned)n_bins, (unsigned)n_masks), block(kBinThreads);
    switch (a.n_src) {
    case 1: hipLaunchKernelGGL(bin_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(bin_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(bin_kernel<3>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(bin_kernel<4>, grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace couple
