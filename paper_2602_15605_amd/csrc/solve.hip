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
// block system for E/B) in the caller's workspace and runs a blocked LU with
// partial pivoting (largest |pivot|, the first row on ties):
//   * a panel of NB columns (8, or 4 when the rows would not fit) is
//     factorised in LDS: by one wave, with no work-group barrier per column,
//     when it has at most kWavePanelRows rows, else by every wave; the
//     pivot's arg-max over a wave runs on DPP lane moves;
//   * right of the panel, each column applies the panel's row exchanges and
//     the unit-lower forward substitution U12 = L11^-1 A12;
//   * the trailing block gets A22 -= L21 U12: lanes over 64 consecutive
//     columns (U12 in registers), the waves split over (column chunk, row
//     group) tasks, and each lane loads 8 rows before it stores any, so A is
//     read once per panel with several loads in flight.
// Then the right-hand sides (columns m .. of the augmented matrix) are back-
// substituted in blocks of kBackBlock rows from the bottom, a chunk of them
// held in LDS: one wave per right-hand side solves the diagonal block (lanes
// over its rows), then every thread updates rows above from U read straight
// from memory.  A zero pivot (a singular system) gives NaN in every output.
#include <mutex>

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

// One step of the arg-max: the pair of the lane that DPP control Ctrl names
// (a row shift or a row broadcast; rows outside RowMask and lanes with no
// source keep their own pair) replaces this lane's pair if it is larger.
template <int Ctrl, int RowMask>
__device__ inline void argmax_dpp_step(double& v, int& idx) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffff), hi = (int)(b >> 32);
    const int olo = __builtin_amdgcn_update_dpp(lo, lo, Ctrl, RowMask, 0xf, false);
    const int ohi = __builtin_amdgcn_update_dpp(hi, hi, Ctrl, RowMask, 0xf, false);
    const int oi = __builtin_amdgcn_update_dpp(idx, idx, Ctrl, RowMask, 0xf, false);
    const double ov = __longlong_as_double(((long long)ohi << 32) | (unsigned int)olo);
    if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
    }
}

// The value of lane i (the same i in every lane) in every lane, from registers.
__device__ inline double lane_value(double v, int i) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), i);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), i);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Largest (|v|, first row on ties) over the 64 lanes of a wave (all active),
// returned in every lane.  Shifts by 1, 2, 4, 8 within each row of 16 lanes
// leave each row's result in its lane 15; broadcasting lane 15 into the next
// row and lane 31 into rows 2 and 3 leaves the wave's result in lane 63.
__device__ inline void wave_argmax(double& v, int& idx) {
    argmax_dpp_step<0x111, 0xf>(v, idx);    // row_shr:1
    argmax_dpp_step<0x112, 0xf>(v, idx);    // row_shr:2
    argmax_dpp_step<0x114, 0xf>(v, idx);    // row_shr:4
    argmax_dpp_step<0x118, 0xf>(v, idx);    // row_shr:8
    argmax_dpp_step<0x142, 0xa>(v, idx);    // row_bcast:15 into rows 1 and 3
    argmax_dpp_step<0x143, 0xc>(v, idx);    // row_bcast:31 into rows 2 and 3
    v = lane_value(v, kWave - 1);
    idx = __builtin_amdgcn_readlane(idx, kWave - 1);
}

// Panel of NB columns in LDS: rows k0 .. m-1 (at most kPanelDoubles / NB).
constexpr int kPanelDoubles = 16384;
constexpr int kRowBatch = 8;      // rows of the trailing update loaded before any is stored
constexpr int kWavePanelRows = 512;  // panels up to this many rows are factorised by one wave
constexpr int kBackBlock = 64;    // rows per diagonal block of the back substitution

template <int NB>
__global__ void __launch_bounds__(kSolveThreads) master_solve_kernel(SolveArgs a) {
    __shared__ double s_panel[kPanelDoubles];    // [row - k0][NB]
    __shared__ int s_perm[NB];                   // row exchanges of the panel (panel rows)
    __shared__ int s_sing;                       // the panel met a zero pivot
    __shared__ double s_cv[kSolveWaves];         // per-wave pivot candidates (tall panels)
    __shared__ int s_ci[kSolveWaves];
    __shared__ double s_pv;                      // chosen pivot magnitude and panel row
    __shared__ int s_pi;
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
    for (int k0 = 0; k0 < m; k0 += NB) {
        const int nb = min(NB, m - k0);
        const int mr = m - k0;
        // panel: rows k0 .. m-1, columns k0 .. k0+nb-1
        for (int e = t; e < mr * NB; e += kSolveThreads) {
            const int r = e / NB, j = e - r * NB;
            s_panel[e] = j < nb ? A[(k0 + r) * ld + k0 + j] : 0.0;
        }
        __syncthreads();
        if (mr <= kWavePanelRows) {
            // short panel: one wave, no work-group barrier per column
            if (wave == 0) {
                bool sing = false;
                for (int j = 0; j < nb; ++j) {
                    double best = -1.0;
                    int bi = mr;
                    for (int r = j + lane; r < mr; r += kWave) {
                        const double v = fabs(s_panel[r * NB + j]);
                        if (v > best) {
                            best = v;
                            bi = r;
                        }
                    }
                    wave_argmax(best, bi);
                    if (!(best > 0.0)) {         // zero (or NaN) pivot column: the system is singular
                        sing = true;
                        break;
                    }
                    bi = min(max(bi, j), mr - 1);    // a candidate row of this column
                    if (lane < NB && bi != j) {
                        const double x = s_panel[j * NB + lane];
                        s_panel[j * NB + lane] = s_panel[bi * NB + lane];
                        s_panel[bi * NB + lane] = x;
                    }
                    if (lane == 0) s_perm[j] = bi;
                    // the exchanged rows are read by other lanes of this wave
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    // multipliers of column j and the rank-1 update of the panel's later columns
                    const double piv = s_panel[j * NB + j];
                    for (int r = j + 1 + lane; r < mr; r += kWave) {
                        const double l = s_panel[r * NB + j] / piv;
                        s_panel[r * NB + j] = l;
#pragma unroll
                        for (int cc = 0; cc < NB; ++cc)
                            if (cc > j && cc < nb) s_panel[r * NB + cc] = __builtin_fma(-l, s_panel[j * NB + cc], s_panel[r * NB + cc]);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
                if (lane == 0) s_sing = sing ? 1 : 0;
            }
            __syncthreads();
            singular = s_sing != 0;
        } else {
            // tall panel: every wave scans rows; four work-group barriers per column
            for (int j = 0; j < nb; ++j) {
                double best = -1.0;
                int bi = mr;
                for (int r = j + t; r < mr; r += kSolveThreads) {
                    const double v = fabs(s_panel[r * NB + j]);
                    if (v > best) {
                        best = v;
                        bi = r;
                    }
                }
                wave_argmax(best, bi);
                if (lane == 0) {
                    s_cv[wave] = best;
                    s_ci[wave] = bi;
                }
                __syncthreads();
                if (wave == 0) {
                    double v = lane < kSolveWaves ? s_cv[lane] : -1.0;
                    int idx = lane < kSolveWaves ? s_ci[lane] : mr;
                    wave_argmax(v, idx);
                    if (lane == 0) {
                        s_pv = v;
                        s_pi = idx;
                    }
                }
                __syncthreads();
                if (!(s_pv > 0.0)) {             // zero (or NaN) pivot column: the system is singular
                    singular = true;
                    break;
                }
                const int p = min(max(s_pi, j), mr - 1);    // a candidate row of this column
                if (t < NB && p != j) {
                    const double x = s_panel[j * NB + t];
                    s_panel[j * NB + t] = s_panel[p * NB + t];
                    s_panel[p * NB + t] = x;
                }
                if (t == 0) s_perm[j] = p;
                __syncthreads();
                // multipliers of column j and the rank-1 update of the panel's later columns
                const double piv = s_panel[j * NB + j];
                for (int r = j + 1 + t; r < mr; r += kSolveThreads) {
                    const double l = s_panel[r * NB + j] / piv;
                    s_panel[r * NB + j] = l;
#pragma unroll
                    for (int cc = 0; cc < NB; ++cc)
                        if (cc > j && cc < nb) s_panel[r * NB + cc] = __builtin_fma(-l, s_panel[j * NB + cc], s_panel[r * NB + cc]);
                }
                __syncthreads();
            }
        }
        if (singular) break;
        // U11 back to A; right of the panel: the row exchanges, then U12 = L11^-1 A12
        for (int e = t; e < nb * nb; e += kSolveThreads) {
            const int r = e / nb, j = e - r * nb;
            A[(k0 + r) * ld + k0 + j] = s_panel[r * NB + j];
        }
        const int c0 = k0 + nb;
        for (int c = c0 + t; c < (int)ld; c += kSolveThreads) {
            for (int j = 0; j < nb; ++j) {
                const int p = s_perm[j];
                if (p != j) {
                    const double x = A[(k0 + j) * ld + c];
                    A[(k0 + j) * ld + c] = A[(k0 + p) * ld + c];
                    A[(k0 + p) * ld + c] = x;
                }
            }
            double u[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if (j < nb) {
                    double v = A[(k0 + j) * ld + c];
#pragma unroll
                    for (int i = 0; i < NB; ++i)
                        if (i < j) v = __builtin_fma(-s_panel[j * NB + i], u[i], v);
                    u[j] = v;
                    A[(k0 + j) * ld + c] = v;
                }
            }
        }
        __syncthreads();
        // trailing update A22 -= L21 U12: lanes over 64 consecutive columns; the
        // waves take (column chunk, row group) tasks
        const int nchunk = ((int)ld - c0 + kWave - 1) / kWave;
        const int groups = max(1, kSolveWaves / nchunk);
        for (int task = wave; task < nchunk * groups; task += kSolveWaves) {
            const int chunk = task % nchunk, grp = task / nchunk;
            const int c = c0 + chunk * kWave + lane;
            const bool live = c < (int)ld;
            double u[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) u[j] = (live && j < nb) ? A[(k0 + j) * ld + c] : 0.0;
            for (int i0 = c0 + grp * kRowBatch; i0 < m; i0 += groups * kRowBatch) {
                double v[kRowBatch];
#pragma unroll
                for (int q = 0; q < kRowBatch; ++q) v[q] = (live && i0 + q < m) ? A[(i0 + q) * ld + c] : 0.0;
#pragma unroll
                for (int q = 0; q < kRowBatch; ++q) {
                    if (i0 + q < m) {
                        const double* L = s_panel + (i0 + q - k0) * NB;
#pragma unroll
                        for (int j = 0; j < NB; ++j) v[q] = __builtin_fma(-L[j], u[j], v[q]);
                    }
                }
#pragma unroll
                for (int q = 0; q < kRowBatch; ++q)
                    if (live && i0 + q < m) A[(i0 + q) * ld + c] = v[q];
            }
        }
        __syncthreads();
    }

    if (singular) {
        for (long long e = t; e < (long long)nr * m; e += kSolveThreads) a.x[e] = __builtin_nan("");
        return;
    }
    // back substitution in blocks of kBackBlock rows from the bottom; a chunk
    // of rc right-hand sides is held in LDS (the panel buffer, free now)
    double* Ub = s_panel;                                    // [kBackBlock][kBackBlock + 1]
    double* Xs = s_panel + kBackBlock * (kBackBlock + 1);    // [m][rc]
    const int rc_max = (kPanelDoubles - kBackBlock * (kBackBlock + 1)) / m;
    for (int r0 = 0; r0 < nr; r0 += rc_max) {
        const int rc = min(rc_max, nr - r0);
        __syncthreads();
        for (int e = t; e < m * rc; e += kSolveThreads) {
            const int q = e / rc, c = e - q * rc;
            Xs[e] = A[q * ld + m + r0 + c];
        }
        for (int ie = m; ie > 0; ie -= kBackBlock) {
            const int ib = max(0, ie - kBackBlock), bs = ie - ib;
            for (int e = t; e < bs * bs; e += kSolveThreads) {
                const int r = e / bs, c = e - r * bs;
                Ub[r * (kBackBlock + 1) + c] = A[(ib + r) * ld + ib + c];
            }
            __syncthreads();
            // diagonal block: one wave per right-hand side, lanes over its rows
            for (int c = wave; c < rc; c += kSolveWaves) {
                double xv = lane < bs ? Xs[(ib + lane) * rc + c] : 0.0;
                for (int i = bs - 1; i >= 0; --i) {
                    const double xi = lane_value(xv, i) / Ub[i * (kBackBlock + 1) + i];
                    if (lane == i) xv = xi;
                    else if (lane < i) xv = __builtin_fma(-Ub[lane * (kBackBlock + 1) + i], xi, xv);
                }
                if (lane < bs) Xs[(ib + lane) * rc + c] = xv;
            }
            __syncthreads();
            // rows above the block: X[q] -= U[q][ib .. ie) X[ib .. ie)
            for (int e = t; e < ib * rc; e += kSolveThreads) {
                const int q = e / rc, c = e - q * rc;
                const double* Uq = A + (long long)q * ld + ib;
                double acc = 0.0;
#pragma unroll 8
                for (int j = 0; j < bs; ++j) acc = __builtin_fma(Uq[j], Xs[(ib + j) * rc + c], acc);
                Xs[e] -= acc;
            }
            __syncthreads();
        }
        for (long long e = t; e < (long long)rc * m; e += kSolveThreads) {
            const int c = (int)(e / m), i = (int)(e - (long long)c * m);
            a.x[(long long)(r0 + c) * m + i] = Xs[i * rc + c];
        }
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

// Workspace of couple_master_solve_noalloc: the [m][m + n_rhs] system lives in
// this file-scope device array instead of a caller or library allocation.
// Every GPU the library runs on holds its own copy until the process ends.
// Host code never passes the array's name to a kernel: it uses the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kNoallocSolveDoubles];

static std::mutex g_scratch_mutex;
static double* g_scratch_ptr[kMaxDevices] = {};

hipError_t noalloc_scratch(int device, double** ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        // called with `device` current: the symbol resolves to that GPU's copy
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
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
    // the widest panel whose m rows fit in LDS (16 columns would spill registers)
    if (a.m * 8 <= kPanelDoubles)
        hipLaunchKernelGGL(master_solve_kernel<8>, dim3(1), dim3(kSolveThreads), 0, s, a);
    else
        hipLaunchKernelGGL(master_solve_kernel<4>, dim3(1), dim3(kSolveThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace couple
