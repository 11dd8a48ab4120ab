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
//
// The solve is Gaussian elimination with partial pivoting (largest |pivot|,
// the first row on ties) on the augmented matrix [K | C~] (TT, or the 2 x 2
// block system for E/B) in the caller's workspace, then back substitution.
// Panels are factorised in LDS by one work-group:
//   * a panel of NB columns (8, or 4, 2 or 1 when its rows would not fit) by
//     one wave, with no work-group barrier per column, when it has at most
//     kWavePanelRows rows, else by every wave; the pivot's arg-max over a wave
//     runs on DPP lane moves;
//   * right of the panel, each column applies the panel's row exchanges and
//     the unit-lower forward substitution U12 = L11^-1 A12;
//   * the trailing block gets A22 -= L21 U12: lanes over 64 consecutive
//     columns (U12 in registers), the waves split over (column chunk, row
//     group) tasks, and each lane loads 8 rows before it stores any.
// Small systems (m < kMultiMin) run all of it in one work-group
// (master_solve_kernel).  Larger ones split the matrix into outer panels of
// kOuterNB columns and spread the O(m^3) part over the chip:
//   solve_assemble_kernel     [K | C~] into the workspace, one work-group per row;
//   solve_panel_kernel        one work-group factorises the outer panel (rows
//                             k0 .. m-1) in inner panels of NB columns as above,
//                             keeping the row exchanges of the panel's earlier
//                             columns (the L21 the update reads) in step;
//   solve_swap_trsm_kernel    right of the outer panel, 64 columns per
//                             work-group: the panel's row exchanges, composed
//                             into one permutation of the touched rows and
//                             applied through LDS, then U12 = L11^-1 A12;
//   solve_update_kernel       A22 -= L21 U12 in 64 x 64 tiles (4 x 4 per
//                             thread, the depth-64 operands staged in LDS);
//   solve_back_kernel         back substitution (one work-group).
// The panel's pivots travel from the panel kernel to the swap kernel in the
// first kOuterNB entries of x, and x[kOuterNB] is a singular flag that every
// later kernel reads first; back substitution overwrites all of x last.
// Back substitution: the right-hand sides (columns m .. of the augmented
// matrix) in blocks of kBackBlock rows from the bottom, a chunk of them held in
// LDS: one wave per right-hand side solves the diagonal block (lanes over its
// rows), then every thread updates rows above from U read straight from memory.
// A zero pivot (a singular system) gives NaN in every output.
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

// The work-group's LDS for factorising one panel.
template <int NB>
struct PanelLds {
    double panel[kPanelDoubles];     // [row - k0][NB]
    int perm[NB];                    // row exchanges of the panel (panel rows)
    int sing;                        // the panel met a zero pivot
    double cv[kSolveWaves];          // per-wave pivot candidates (tall panels)
    int ci[kSolveWaves];
    double pv;                       // chosen pivot magnitude and panel row
    int pi;
    int trow[2 * NB];                // rows the exchanges touch (panel-relative): the panel's top first
    int tsrc[2 * NB];                // the row whose old values land in trow[i]
    int tn;
};

// Compose the panel's exchanges (row j <-> perm[j], in order) into one
// permutation of the rows they touch: after all of them, row trow[i] holds
// what row tsrc[i] held before.  One thread; at most 2 NB rows.
template <int NB>
__device__ inline void compose_exchanges(PanelLds<NB>& L, int nb) {
    int n = nb;
    for (int j = 0; j < nb; ++j) L.trow[j] = L.tsrc[j] = j;
    for (int j = 0; j < nb; ++j) {
        const int p = L.perm[j];
        if (p == j) continue;
        int ip = -1;
        for (int i = 0; i < n; ++i)
            if (L.trow[i] == p) ip = i;
        if (ip < 0) {
            ip = n++;
            L.trow[ip] = L.tsrc[ip] = p;
        }
        const int tmp = L.tsrc[j];
        L.tsrc[j] = L.tsrc[ip];
        L.tsrc[ip] = tmp;
    }
    L.tn = n;
}

// Rows k0 .. k0+mr-1, columns k0 .. k0+nb-1 of A into L.panel (columns nb ..
// NB-1 zero).  Each thread issues kLoadBatch loads before it stores any.
constexpr int kLoadBatch = 8;
template <int NB>
__device__ inline void load_panel(PanelLds<NB>& L, const double* A, long long ld, int k0, int mr, int nb) {
    const int total = mr * NB;
    for (int e0 = threadIdx.x; e0 < total; e0 += kSolveThreads * kLoadBatch) {
        double v[kLoadBatch];
#pragma unroll
        for (int q = 0; q < kLoadBatch; ++q) {
            const int e = e0 + q * kSolveThreads;
            const int r = e / NB, j = e - r * NB;
            v[q] = (e < total && j < nb) ? A[(k0 + r) * ld + k0 + j] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kLoadBatch; ++q) {
            const int e = e0 + q * kSolveThreads;
            if (e < total) L.panel[e] = v[q];
        }
    }
}

// Entry (r, c) of the augmented matrix [K | C~]: TT, or [EE EB; EB BB] for E/B.
__device__ inline double assembled(const SolveArgs& a, int r, int c) {
    if (c >= a.m) return a.rhs[(long long)(c - a.m) * a.m + r];
    if (!a.pol) return a.K[(long long)r * a.n + c];
    const int n = a.n, br = r / n, bc = c / n;
    const int blk = br != bc ? 2 : br;
    return a.K[((long long)blk * n + (r - br * n)) * n + (c - bc * n)];
}

// Factorise the mr x nb panel in L.panel with partial pivoting: multipliers
// below the diagonal, U11 on and above it, the exchanges in L.perm.  Called by
// every thread of the work-group; returns true (in every thread) on a zero or
// NaN pivot column.
template <int NB>
__device__ bool factor_panel(PanelLds<NB>& L, int mr, int nb) {
    const int t = threadIdx.x;
    const int lane = t % kWave, wave = t / kWave;
    double* s_panel = L.panel;
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
                if (lane == 0) L.perm[j] = bi;
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
            if (lane == 0) L.sing = sing ? 1 : 0;
        }
        __syncthreads();
        return L.sing != 0;
    }
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
            L.cv[wave] = best;
            L.ci[wave] = bi;
        }
        __syncthreads();
        if (wave == 0) {
            double v = lane < kSolveWaves ? L.cv[lane] : -1.0;
            int idx = lane < kSolveWaves ? L.ci[lane] : mr;
            wave_argmax(v, idx);
            if (lane == 0) {
                L.pv = v;
                L.pi = idx;
            }
        }
        __syncthreads();
        if (!(L.pv > 0.0)) return true;      // zero (or NaN) pivot column: the system is singular
        const int p = min(max(L.pi, j), mr - 1);    // a candidate row of this column
        if (t < NB && p != j) {
            const double x = s_panel[j * NB + t];
            s_panel[j * NB + t] = s_panel[p * NB + t];
            s_panel[p * NB + t] = x;
        }
        if (t == 0) L.perm[j] = p;
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
    return false;
}

// Column c right of the panel at k0 (nb columns, factorised in s_panel):
// the panel's row exchanges, then U12 = L11^-1 A12 in place.
template <int NB>
__device__ inline void exchange_and_solve_column(double* A, long long ld, int k0, int nb, const PanelLds<NB>& L,
                                                 long long c, bool solve) {
    for (int j = 0; j < nb; ++j) {
        const int p = L.perm[j];
        if (p != j) {
            const double x = A[(k0 + j) * ld + c];
            A[(k0 + j) * ld + c] = A[(k0 + p) * ld + c];
            A[(k0 + p) * ld + c] = x;
        }
    }
    if (!solve) return;
    double u[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j < nb) {
            double v = A[(k0 + j) * ld + c];
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (i < j) v = __builtin_fma(-L.panel[j * NB + i], u[i], v);
            u[j] = v;
            A[(k0 + j) * ld + c] = v;
        }
    }
}

// As exchange_and_solve_column with the exchanges composed (compose_exchanges):
// every touched row is loaded before any is stored, so the loads overlap.
template <int NB>
__device__ inline void permute_and_solve_column(double* A, long long ld, int k0, int nb, const PanelLds<NB>& L,
                                                long long c, bool solve) {
    const int n = L.tn;
    double v[2 * NB];
#pragma unroll
    for (int i = 0; i < 2 * NB; ++i)
        if (i < n) v[i] = A[(k0 + L.tsrc[i]) * ld + c];
    if (solve) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j < nb) {
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    if (i < j) v[j] = __builtin_fma(-L.panel[j * NB + i], v[i], v[j]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 2 * NB; ++i)
        if (i < n && (i < nb || L.trow[i] != L.tsrc[i])) A[(k0 + L.trow[i]) * ld + c] = v[i];
}

// A[r][c] -= L21[r] U12[c] for rows k0+nb .. m-1 and columns c0 .. ce-1
// (c0 = k0 + nb), L21 in s_panel.  Lanes go over lpr consecutive columns,
// lpr the narrowest power of two (8 .. 64) that covers them, so a wave works
// on 64 / lpr row sets at once; the waves take (column chunk, row group)
// tasks, and each lane loads RB rows before it stores any.
template <int NB, int RB>
__device__ inline void panel_trailing_update(double* A, long long ld, int m, int k0, int nb, int ce,
                                             const PanelLds<NB>& L) {
    const int t = threadIdx.x;
    const int lane = t % kWave, wave = t / kWave;
    const int c0 = k0 + nb, w = ce - c0;
    int lpr = kWave;
    while (lpr > 8 && lpr / 2 >= w) lpr /= 2;
    const int sets = kWave / lpr, sub = lane / lpr, cl = lane % lpr;
    const int nchunk = (w + lpr - 1) / lpr;
    const int groups = max(1, kSolveWaves / nchunk);
    for (int task = wave; task < nchunk * groups; task += kSolveWaves) {
        const int chunk = task % nchunk, grp = task / nchunk;
        const int c = c0 + chunk * lpr + cl;
        const bool live = c < ce;
        double u[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) u[j] = (live && j < nb) ? A[(k0 + j) * ld + c] : 0.0;
        for (int i0 = c0 + (grp * sets + sub) * RB; i0 < m; i0 += groups * sets * RB) {
            double v[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) v[q] = (live && i0 + q < m) ? A[(i0 + q) * ld + c] : 0.0;
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                if (i0 + q < m) {
                    const double* Lr = L.panel + (i0 + q - k0) * NB;
#pragma unroll
                    for (int j = 0; j < NB; ++j) v[q] = __builtin_fma(-Lr[j], u[j], v[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < RB; ++q)
                if (live && i0 + q < m) A[(i0 + q) * ld + c] = v[q];
        }
    }
}

// Back substitution with U in A[0 .. m)[0 .. m) and the right-hand sides in
// columns m .. m+nr; buf: LDS of buf_doubles >= kBackBlock (kBackBlock + 1) + m.
__device__ void back_substitute(const double* A, long long ld, int m, int nr, double* x, double* buf,
                                int buf_doubles) {
    const int t = threadIdx.x;
    const int lane = t % kWave, wave = t / kWave;
    double* Ub = buf;                                    // [kBackBlock][kBackBlock + 1]
    double* Xs = buf + kBackBlock * (kBackBlock + 1);    // [m][rc]
    const int rc_max = (buf_doubles - kBackBlock * (kBackBlock + 1)) / m;
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
            x[(long long)(r0 + c) * m + i] = Xs[i * rc + c];
        }
    }
}

template <int NB>
__global__ void __launch_bounds__(kSolveThreads) master_solve_kernel(SolveArgs a) {
    __shared__ PanelLds<NB> L;
    const int t = threadIdx.x;
    const int lane = t % kWave, wave = t / kWave;
    const int m = a.m, nr = a.n_rhs;
    const long long ld = (long long)m + nr;
    double* A = a.work;

    // assemble [K | C~]
    for (int r = wave; r < m; r += kSolveWaves)
        for (int c = lane; c < (int)ld; c += kWave) A[r * ld + c] = assembled(a, r, c);
    __syncthreads();

    bool singular = false;
    for (int k0 = 0; k0 < m; k0 += NB) {
        const int nb = min(NB, m - k0);
        const int mr = m - k0;
        // panel: rows k0 .. m-1, columns k0 .. k0+nb-1
        load_panel<NB>(L, A, ld, k0, mr, nb);
        __syncthreads();
        singular = factor_panel<NB>(L, mr, nb);
        if (singular) break;
        // U11 back to A; right of the panel: the row exchanges, then U12 = L11^-1 A12
        for (int e = t; e < nb * nb; e += kSolveThreads) {
            const int r = e / nb, j = e - r * nb;
            A[(k0 + r) * ld + k0 + j] = L.panel[r * NB + j];
        }
        for (int c = k0 + nb + t; c < (int)ld; c += kSolveThreads) exchange_and_solve_column<NB>(A, ld, k0, nb, L, c, true);
        __syncthreads();
        panel_trailing_update<NB, kRowBatch>(A, ld, m, k0, nb, (int)ld, L);
        __syncthreads();
    }

    if (singular) {
        for (long long e = t; e < (long long)nr * m; e += kSolveThreads) a.x[e] = __builtin_nan("");
        return;
    }
    // back substitution; the panel buffer is free now
    back_substitute(A, ld, m, nr, a.x, L.panel, kPanelDoubles);
}

// ---------------------------------------------------------------------------
// Multi-work-group path (m >= kMultiMin).
constexpr int kOuterNB = 32;               // columns per outer panel
constexpr int kSingularSlot = kOuterNB;    // x[kSingularSlot]: an outer panel met a zero pivot
constexpr int kSwapCols = 64;              // columns per work-group of the swap + TRSM kernel
constexpr int kSwapThreads = 256;
constexpr int kUpdTile = 64;               // the update kernel's tile: kUpdTile x kUpdTile entries
constexpr int kUpdThreads = 256;           // 16 x 16 threads, 4 x 4 entries each
constexpr int kBackDoubles = 20000;        // back-substitution LDS (m <= 15840 with one right-hand side)
static_assert(kOuterNB <= kWave, "the swap kernel's mapping keeps two touched rows per lane of one wave");
constexpr int kPanelRowBatch = 16;         // rows loaded before any is stored in the panel kernel's update
                                           // (half that for 8-column panels, which would spill)
constexpr int kMultiMin = 400;             // systems of at least this many unknowns take this path
static_assert(kMultiMin > kSingularSlot, "x must hold the pivots and the flag");
static_assert(kSolveMaxCols - 1 <= kPanelDoubles, "every panel's rows must fit an LDS panel of one column");
static_assert(kBackBlock * (kBackBlock + 1) + kSolveMaxCols <= kBackDoubles,
              "back substitution holds at least one right-hand side of every system in LDS");

struct OuterArgs {
    double* A;                   // the augmented matrix [m][ld]
    double* x;                   // pivots of the outer panel in x[0 .. nbo), the flag in x[kSingularSlot]
    long long ld;
    int m, k0, nbo;
};

__global__ void __launch_bounds__(256) solve_assemble_kernel(SolveArgs a) {
    const int r = blockIdx.x;
    const long long ld = (long long)a.m + a.n_rhs;
    for (int c = threadIdx.x; c < (int)ld; c += 256) a.work[r * ld + c] = assembled(a, r, c);
}

// One work-group factorises the outer panel: columns k0 .. k0+nbo-1, rows
// k0 .. m-1, in inner panels of NB columns.  Every inner panel is written back
// whole (its multipliers are the L21 of the update kernel), its row exchanges
// go to the outer panel's other columns (left ones too, so L21 stays in row
// order) and its U12 and trailing update stay inside the outer panel.
template <int NB>
__global__ void __launch_bounds__(kSolveThreads) solve_panel_kernel(OuterArgs a) {
    __shared__ PanelLds<NB> L;
    const int t = threadIdx.x;
    const int m = a.m, k0 = a.k0, ce = a.k0 + a.nbo;
    const long long ld = a.ld;
    double* A = a.A;
    if (k0 == 0) {
        if (t == 0) a.x[kSingularSlot] = 0.0;
    } else if (a.x[kSingularSlot] != 0.0) {
        return;                                   // an earlier panel was singular
    }
    for (int kk = k0; kk < ce; kk += NB) {
        const int nb = min(NB, ce - kk), mr = m - kk;
        load_panel<NB>(L, A, ld, kk, mr, nb);
        __syncthreads();
        if (factor_panel<NB>(L, mr, nb)) {
            if (t == 0) a.x[kSingularSlot] = 1.0;
            return;
        }
        for (int e = t; e < mr * nb; e += kSolveThreads) {
            const int r = e / nb, j = e - r * nb;
            A[(kk + r) * ld + kk + j] = L.panel[r * NB + j];
        }
        if (t < nb) a.x[kk - k0 + t] = (double)(kk + L.perm[t]);
        if (t == 0) compose_exchanges<NB>(L, nb);
        __syncthreads();
        // the other columns of the outer panel: left ones get the exchanges,
        // right ones the exchanges and U12
        const int nleft = kk - k0, nother = nleft + (ce - kk - nb);
        for (int q = t; q < nother; q += kSolveThreads) {
            const int c = q < nleft ? k0 + q : kk + nb + (q - nleft);
            permute_and_solve_column<NB>(A, ld, kk, nb, L, c, q >= nleft);
        }
        __syncthreads();
        if (kk + nb < ce) panel_trailing_update<NB, (NB >= 8 ? kPanelRowBatch / 2 : kPanelRowBatch)>(A, ld, m, kk, nb, ce, L);
        __syncthreads();
    }
}

// Right of the outer panel, kSwapCols columns per work-group: the nbo row
// exchanges of the panel composed into one permutation of the rows they touch
// (the top block k0 .. k0+nbo-1 and at most nbo rows below it), applied by
// reading every source row before writing any, then U12 = L11^-1 A12 for the
// top block (one thread per column).
__global__ void __launch_bounds__(kSwapThreads) solve_swap_trsm_kernel(OuterArgs a) {
    __shared__ double s_l[kOuterNB][kOuterNB + 1];
    __shared__ double s_tile[2 * kOuterNB][kSwapCols];
    __shared__ int s_row[2 * kWave];             // touched rows: the top block first (two per lane)
    __shared__ int s_src[2 * kWave];             // the row whose old values land in s_row[i]
    __shared__ int s_n;
    if (a.x[kSingularSlot] != 0.0) return;
    const int t = threadIdx.x;
    const int lane = t % kSwapCols, grp = t / kSwapCols;
    constexpr int kGroups = kSwapThreads / kSwapCols;
    const int k0 = a.k0, nbo = a.nbo;
    const long long ld = a.ld;
    const double* Ac = a.A;
    const long long c = (long long)(k0 + nbo) + (long long)blockIdx.x * kSwapCols + lane;
    const bool live = c < ld;
    // L11: every thread issues its 16 loads before it stores any
    {
        constexpr int kPer = kOuterNB * kOuterNB / kSwapThreads;
        double v[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = t + q * kSwapThreads, r = e / kOuterNB, j = e - r * kOuterNB;
            v[q] = (r < nbo && j < nbo) ? Ac[(k0 + r) * ld + k0 + j] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = t + q * kSwapThreads, r = e / kOuterNB, j = e - r * kOuterNB;
            s_l[r][j] = v[q];
        }
    }
    if (t < kWave) {
        // one wave: lane i keeps touched rows i and i + 64 in registers; a
        // ballot finds where the pivot row sits
        const int l = t;
        int row0 = l < nbo ? k0 + l : -1, src0 = row0;
        int row1 = -1, src1 = -1;
        int n = nbo;
        const int piv = l < nbo ? (int)a.x[l] : 0;       // all pivots in one load
        for (int j = 0; j < nbo; ++j) {
            const int p = __shfl(piv, j);
            if (p == k0 + j) continue;
            const unsigned long long h0 = __ballot(row0 == p), h1 = __ballot(row1 == p);
            int ip;
            if (h0) {
                ip = __ffsll((long long)h0) - 1;
            } else if (h1) {
                ip = kWave + __ffsll((long long)h1) - 1;
            } else {
                ip = n++;
                if (l == ip - kWave) row1 = src1 = p;     // p > k0 + nbo - 1 here, so ip >= nbo
                if (ip < kWave && l == ip) row0 = src0 = p;
            }
            // swap the sources of positions j (< nbo <= 64) and ip
            const int sj = __shfl(src0, j);
            const int sip = ip < kWave ? __shfl(src0, ip) : __shfl(src1, ip - kWave);
            if (l == j) src0 = sip;
            if (ip < kWave) {
                if (l == ip) src0 = sj;
            } else if (l == ip - kWave) {
                src1 = sj;
            }
        }
        s_row[l] = row0;
        s_src[l] = src0;
        s_row[kWave + l] = row1;
        s_src[kWave + l] = src1;
        if (l == 0) s_n = n;
    }
    __syncthreads();
    const int n = s_n;
    {
        constexpr int kPer = 2 * kOuterNB / kGroups;     // touched rows per thread, loaded before any store
        double v[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int i = grp + q * kGroups;
            v[q] = (i < n && live) ? Ac[(long long)s_src[i] * ld + c] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int i = grp + q * kGroups;
            if (i < n) s_tile[i][lane] = v[q];
        }
    }
    __syncthreads();
    if (!live) return;
    double* A = a.A;
    for (int i = nbo + grp; i < n; i += kGroups) A[(long long)s_row[i] * ld + c] = s_tile[i][lane];
    if (grp == 0) {
        for (int j = 0; j < nbo; ++j) {
            double v = s_tile[j][lane];
            for (int i = 0; i < j; ++i) v = __builtin_fma(-s_l[j][i], s_tile[i][lane], v);
            s_tile[j][lane] = v;
            A[(k0 + j) * ld + c] = v;
        }
    }
}

// A22 -= L21 U12 over rows and columns k0+nbo .. (m and ld), depth nbo:
// kUpdTile x kUpdTile entries per work-group, 4 x 4 per thread.
__global__ void __launch_bounds__(kUpdThreads) solve_update_kernel(OuterArgs a) {
    __shared__ double s_lt[kOuterNB][kUpdTile + 1];    // L21 transposed: [k][row]
    __shared__ double s_u[kOuterNB][kUpdTile];         // U12: [k][column]
    if (a.x[kSingularSlot] != 0.0) return;
    const int t = threadIdx.x;
    const int tr = t / 16, tc = t % 16;
    const int k0 = a.k0, nbo = a.nbo, m = a.m;
    const long long ld = a.ld;
    const long long c0 = (long long)k0 + nbo;
    const long long rb = c0 + (long long)blockIdx.y * kUpdTile, cb = c0 + (long long)blockIdx.x * kUpdTile;
    double* A = a.A;
    for (int e = t; e < kUpdTile * kOuterNB; e += kUpdThreads) {
        const int r = e / kOuterNB, k = e - r * kOuterNB;
        s_lt[k][r] = (k < nbo && rb + r < m) ? A[(rb + r) * ld + k0 + k] : 0.0;
    }
    for (int e = t; e < kOuterNB * kUpdTile; e += kUpdThreads) {
        const int k = e / kUpdTile, cc = e - k * kUpdTile;
        s_u[k][cc] = (k < nbo && cb + cc < ld) ? A[(k0 + k) * ld + cb + cc] : 0.0;
    }
    __syncthreads();
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k = 0; k < nbo; ++k) {
        double l[4], u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            l[q] = s_lt[k][tr * 4 + q];
            u[q] = s_u[k][tc * 4 + q];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fma(l[i], u[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const long long r = rb + tr * 4 + i;
        if (r >= m) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long c = cb + tc * 4 + j;
            if (c < ld) A[r * ld + c] -= acc[i][j];
        }
    }
}

__global__ void __launch_bounds__(kSolveThreads) solve_back_kernel(SolveArgs a) {
    __shared__ double buf[kBackDoubles];
    const int t = threadIdx.x;
    const int m = a.m, nr = a.n_rhs;
    const bool singular = a.x[kSingularSlot] != 0.0;
    __syncthreads();                              // every thread has read the flag before x is written
    if (singular) {
        for (long long e = t; e < (long long)nr * m; e += kSolveThreads) a.x[e] = __builtin_nan("");
        return;
    }
    back_substitute(a.work, (long long)m + nr, m, nr, a.x, buf, kBackDoubles);
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
    if (a.m < kMultiMin) {
        // the widest panel whose m rows fit in LDS (16 columns would spill registers; m < 400 here)
        if (a.m * 8 <= kPanelDoubles)
            hipLaunchKernelGGL(master_solve_kernel<8>, dim3(1), dim3(kSolveThreads), 0, s, a);
        else
            hipLaunchKernelGGL(master_solve_kernel<4>, dim3(1), dim3(kSolveThreads), 0, s, a);
        return hipGetLastError();
    }
    const int m = a.m;
    const long long ld = (long long)m + n_rhs;
    hipLaunchKernelGGL(solve_assemble_kernel, dim3((unsigned)m), dim3(256), 0, s, a);
    for (int k0 = 0; k0 < m; k0 += kOuterNB) {
        OuterArgs o;
        o.A = work;
        o.x = x;
        o.ld = ld;
        o.m = m;
        o.k0 = k0;
        o.nbo = min(kOuterNB, m - k0);
        // the widest inner panel whose rows fit in LDS
        if ((m - k0) * 8 <= kPanelDoubles)
            hipLaunchKernelGGL(solve_panel_kernel<8>, dim3(1), dim3(kSolveThreads), 0, s, o);
        else if ((m - k0) * 4 <= kPanelDoubles)
            hipLaunchKernelGGL(solve_panel_kernel<4>, dim3(1), dim3(kSolveThreads), 0, s, o);
        else if ((m - k0) * 2 <= kPanelDoubles)
            hipLaunchKernelGGL(solve_panel_kernel<2>, dim3(1), dim3(kSolveThreads), 0, s, o);
        else
            hipLaunchKernelGGL(solve_panel_kernel<1>, dim3(1), dim3(kSolveThreads), 0, s, o);
        const long long c0 = (long long)k0 + o.nbo;    // < ld: there is at least one right-hand side
        const unsigned col_groups = (unsigned)((ld - c0 + kSwapCols - 1) / kSwapCols);
        hipLaunchKernelGGL(solve_swap_trsm_kernel, dim3(col_groups), dim3(kSwapThreads), 0, s, o);
        if (c0 < m)
            hipLaunchKernelGGL(solve_update_kernel,
                               dim3((unsigned)((ld - c0 + kUpdTile - 1) / kUpdTile),
                                    (unsigned)((m - c0 + kUpdTile - 1) / kUpdTile)),
                               dim3(kUpdThreads), 0, s, o);
    }
    hipLaunchKernelGGL(solve_back_kernel, dim3(1), dim3(kSolveThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace couple
