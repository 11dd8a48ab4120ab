// Internal declarations shared by the libcouple translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "couple.h"
#include "strip_params.hpp"

namespace couple {

// Batched form: masks sorted by lmax and split into column groups of 16.
constexpr int kMaxGroups = 4;          // up to 64 masks per call
constexpr int kMaskGroup = 16;
struct BatchPlan {
    int n_groups = 0;
    int n_masks[kMaxGroups] = {0, 0, 0, 0};
    int L[kMaxGroups] = {0, 0, 0, 0};              // largest lmax of the group
    int lmax[kMaxGroups][kMaskGroup];
    const double* w[kMaxGroups][3][kMaskGroup];    // W_TT, W_TP, W_PP (NULL: unused)
    double* out[kMaxGroups][kMaskGroup];
    int flush = 8;                                  // MFMA steps (4-mask form: 16-step groups) per flush
    int tm = 2;                                     // 16-row tiles (1, 2, 4); float32 4-mask form: 64, 128 rows
};

}  // namespace couple

struct couple_ctx {
    int device = 0;
    int lmax_max = 0;
    // look-up tables (device); g and h carry kTablePad zeros on both sides
    double* g_pad = nullptr;     // g(p),            p = -pad .. lmax_max + pad
    double* h_pad = nullptr;     // 1/((2p+1)g(p)),  p = -pad .. 2 lmax_max + pad
    float* gf_pad = nullptr;
    float* hf_pad = nullptr;
    double* cl = nullptr;        // c_l, l = 0 .. lmax_max
    // workspace
    double* xi = nullptr;        // 4 packed upper triangles (TT, TE, EE, EB)
    double* wp = nullptr;        // scaled windows (2l+1) W_l / (4 pi), 3 x (2 lmax_max + 1)
    float* wpf = nullptr;        // float32 copies
    int* wexp = nullptr;         // FP32C scale exponents: suffix maxima of |W'| per parity, 3 x (2 lmax_max + 1)
    int* edges_dev = nullptr;    // bin edges (device), lmax_max + 2
    int* edges_host = nullptr;   // pinned staging for the bin edges
    double* solve_scratch = nullptr;  // this device's copy of the no-alloc solve workspace
    size_t dev_bytes = 0;        // device bytes of the tables and workspace above
    void* bws = nullptr;         // batched workspace (couple_reserve_batched)
    size_t bws_bytes = 0;
    // tile shape of the batched matrix-core kernels, [0] float32, [1] BF16x3
    int batched_flush[2] = {8, 4};   // MFMA steps per flush (float32 4-mask form: 16-step groups)
    int batched_tm[2] = {2, 2};      // 16-row tiles per wavefront (float32 4-mask form: 64 or 128 rows)
    std::string err;
    // measurement hook: event pairs recorded around each kernel
    bool profiling = false;
    struct Mark {
        hipEvent_t start, stop;
        int stage;
    };
    std::vector<Mark> marks;
    hipEvent_t pending_start = nullptr;
    double prof_ms[COUPLE_N_STAGES] = {0, 0, 0};
    int prof_count[COUPLE_N_STAGES] = {0, 0, 0};
};

namespace couple {

// LUT build (tables.hip)
hipError_t launch_build_tables(couple_ctx* ctx, hipStream_t s);

// strip kernels (strip.hip): Xi on the packed upper triangle.
//   mode kStripTT: Xi_TT; kStripPol: Xi_TT, Xi_TE, Xi_EE (even L); kStripPolEE:
//   Xi_TT, Xi_EE (even L, for calls that ask for no TE); kStripEE: Xi_EE alone;
//   kStripEB: Xi_EB (odd L, fourth triangle).  l3 restricted to [l3_lo, l3_hi].
hipError_t launch_scale_windows(const couple_ctx* ctx, const double* wtt, const double* wtp,
                                const double* wpp, int n, hipStream_t s);
// The windows of n_masks <= kBandMasks masks into the context's window sets
// 0 .. n_masks - 1 (float64 only), for launch_strip_masks; wtt/wtp/wpp NULL
// where the spectrum is not needed.
// n_m[m] (NULL: all n): entries of mask m's windows to read, W' = 0 from there to n.
hipError_t launch_scale_windows_masks(const couple_ctx* ctx, const double* const* wtt, const double* const* wtp,
                                      const double* const* wpp, int n_masks, int n, const int* n_m, hipStream_t s);
// wexp[x][l3] = e with max |W'_x(l3')| over l3' = l3, l3 + 2, .. < n in [2^(e-1), 2^e)
// (0 where that maximum is 0), for the float32 strip kernels' per-item scaling
// for window sets 0 .. n_masks - 1
hipError_t launch_window_exponents(const couple_ctx* ctx, int n, hipStream_t s, int n_masks = 1);
hipError_t launch_strip(const couple_ctx* ctx, int lmax, int mode, int precision, int l3_lo,
                        int l3_hi, hipStream_t s);
// Masks one launch_strip_masks call takes in a mode.
int strip_masks_per_launch(int mode, int precision);
// Whether launch_strip_masks gives a mask of this lmax and l3_hi the bits launch_strip
// gives it (false only for FP32C's EB when launch_strip would use short lanes).
bool strip_masks_bitwise(int mode, int precision, int lmax, int l3_hi);
// FP32C or FP64 over masks 0 .. n_masks - 1 (n_masks <= strip_masks_per_launch) of the window sets,
// l3 in [l3_lo, l3_hi]: mask m (lmax_m[m]) gets its Xi triangles (TT, TE, EE slots for even L,
// the EB slot 3 for odd L) of diagonals 0 .. min(lmax_m[m], l3_hi) at xi + xi_off[m], each slot
// min(lmax_m[m], l3_hi) + 1 diagonals long.
hipError_t launch_strip_masks(const couple_ctx* ctx, int mode, int precision, int n_masks, const int* lmax_m,
                              double* xi, const long long* xi_off, int l3_lo, int l3_hi, hipStream_t s);

// fill / bin kernels (fill.hip); Xi exists for diagonals d <= dmax and is 0 beyond.
//   spec_src[i] = which Xi (0 TT, 1 TE, 2 EE, 3 EB) output i comes from, n_out <= kMaxOut outputs.
constexpr int kMaxOut = 5;
//   xi != 0: write Xi itself (no (2 l2 + 1) column factor).
//   xi_src / xi_stride: the Xi store to read (default: the context's, stride tri(lmax)).
hipError_t launch_fill(const couple_ctx* ctx, int lmax, int dmax, const int* spec_src, int n_out,
                       double* out, int xi, hipStream_t s, const double* xi_src = nullptr,
                       long long xi_stride = 0);
// Up to kInlineBins bins the edges travel in the kernel arguments (no upload,
// nothing to synchronise); longer lists are read from bin_edges_dev.
constexpr int kInlineBins = 512;
//   n_masks: masks binned by the one launch, their Xi stores xi_mask_stride apart
//   and their outputs n_out n_bins^2 apart.
hipError_t launch_bin(const couple_ctx* ctx, int lmax, int dmax, const int* spec_src, int n_out,
                      const int* bin_edges_host, const int* bin_edges_dev, int n_bins, double* out, int xi,
                      hipStream_t s, const double* xi_src = nullptr, long long xi_stride = 0, int n_masks = 1,
                      long long xi_mask_stride = 0);
// One fill job: Xi store [3][tri(lmax)] (Xi for diagonals d <= dmax, 0 beyond)
// and its n_out output matrices [n_out][lmax+1][lmax+1].  block0 is set by
// launch_fill_jobs.
constexpr int kMaxFillJobs = kMaxGroups * kMaskGroup;
struct FillJob {
    const double* xi;
    long long xi_stride;   // between the Xi triangles of the store
    double* out;
    int lmax;
    int dmax;
    int block0;
};
hipError_t launch_fill_jobs(const FillJob* jobs, int n_jobs, const int* spec_src, int n_out, int xi,
                            hipStream_t s);
// out[0 .. n) = 0 with a kernel (safe inside captured graphs)
hipError_t launch_zero(double* out, size_t n, hipStream_t s);

// rows of 3j symbols (l1 l2 l3; -m m 0) from the tables (threej.hip)
hipError_t launch_threej_rows(const couple_ctx* ctx, int m, int n_pairs, const int* l1, const int* l2, double* out,
                              long long stride, hipStream_t s);
// rows of (l1 l2 l3; m1 m2 m3) in the canonical form (x y z; a b -a-b),
// 0 <= a, b <= 2, (x, y, z) = (l1, l2, l3) rotated left by rot, times (-1)^L if flip
hipError_t launch_threej_family(const couple_ctx* ctx, int rot, int flip, int a, int b, int n_pairs, const int* l1,
                                const int* l2, double* out, long long stride, hipStream_t s);

// binned MASTER solve (solve.hip)
constexpr int kSolveMaxCols = 15840;   // unknowns + right-hand sides of one solve
hipError_t launch_bin_spectra(const couple_ctx* ctx, int n_spec, const double* cl, int cl_stride,
                              const int* bin_edges_host, int n_bins, double* out, hipStream_t s);
hipError_t launch_master_solve(int pol, int n, const double* K, int n_rhs, const double* rhs, double* work,
                               double* x, hipStream_t s);
// couple_master_solve_noalloc: the device address of this GPU's copy of the
// file-scope workspace array (resolved once per device, with that device current).
constexpr long long kNoallocSolveDoubles = COUPLE_NOALLOC_SOLVE_DOUBLES;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, double** ptr);

// measurement hook: event marks around a kernel of stage `stage` (no-op unless profiling)
void prof_begin(couple_ctx* ctx, hipStream_t s);
void prof_end(couple_ctx* ctx, hipStream_t s, int stage);

// batched form (batched.hip)
size_t batched_workspace_bytes(const BatchPlan& p);
hipError_t launch_batched(couple_ctx* ctx, const BatchPlan& p, int precision, const int* spec_src, int n_out,
                          int xi, hipStream_t s);

}  // namespace couple
