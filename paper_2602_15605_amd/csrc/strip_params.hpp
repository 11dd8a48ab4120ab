// Parameters of the strip kernels and the packed-triangle indexing they share
// with the fill, bin and batched kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace couple {

// Lanes of a wavefront on CDNA4.
constexpr int kWave = 64;

// Number of consecutive l1 values a lane of the strip kernel owns.  The
// G/H windows slide by one per l3 step, so each step loads one new G and
// one new H value per lane for R terms.
constexpr int kStripR = 4;
// The TT-only sum costs two operations per term, so there the two window
// reads per step dominate; eight rows per lane halve them per term.
constexpr int kStripRTT = 8;
// Launches that would have fewer work items of 64 R rows than these take
// kStripRSmall rows per lane, four times as many items with a quarter of the
// staircase each: float32 below 8192 items (full triangle: lmax <= 1918),
// float64 below 4096 (lmax <= 1321), where the measured crossovers lie; above them the
// longer rows per lane win.
constexpr int kStripRSmall = 2;
constexpr long long kStripSmallItemsF32 = 8192;
constexpr long long kStripSmallItemsF64 = 4096;

// Band-limited grids run in phases of this many consecutive diagonals, the
// phases in order of d and each phase block by block.  A diagonal's trip,
// (l3_hi - d)/2 steps for all but its lowest-l1 block, falls with d, so the
// phases run longest first; inside a phase, waves dispatched together share
// their block's g and h windows.  Measured on the 10^4 / l3 <= 1000 band
// (FP32C, FP64 strip per mask): 0.406 / 0.708 ms with all diagonals of a block
// in turn, 0.394 / 0.707 diagonal by diagonal, 0.383 / 0.680 with 256-diagonal
// phases and 0.377 / 0.677 with 64.
constexpr int kBandPhase = 64;

// l3 steps staged in LDS per chunk by the float64 and float32 strip kernels.
constexpr int kStripChunkF64 = 256;
constexpr int kStripChunkF32 = 256;
// Masks per launch of the multi-mask float32 kernel: at most 4 (one float4
// lane each).  Its sums take 16 VGPRs per mask and spectrum (four rows, block,
// mid and Kahan pair).  TT + EE with four masks needs 230 VGPRs (two waves per
// SIMD, as the 14 KB of LDS would allow at most 2.75): on the 8-mask 10^4 band
// it ran 1.75 ms against 2.18 ms with two masks per launch (156 VGPRs, three
// waves).  TT + TE + EE takes three (228 VGPRs; four would need 256, one
// wave): the 32-mask batched call's strip ran 12.5 ms against 13.4 ms with two.
constexpr int kBandMasks = 4;
constexpr int kMasksPolEE = 4;
constexpr int kMasksPol = 3;
// The float64 multi-mask kernel (one float64 sum per mask, spectrum and row;
// 248 VGPRs for TT + EE with four masks, two waves per SIMD).  On the 8-mask
// 10^4 band (strip per call): 2.45 ms with four masks per launch and 128-step
// chunks, 2.49 ms with 64-step chunks, 3.07 / 3.39 ms with three / two masks,
// against 5.37 ms for one launch per mask.
constexpr int kMasksPolEEF64 = 4;
constexpr int kMasksPolF64 = 2;
constexpr int kStripChunkF64Masks = 128;

// float32 strip kernel: steps per exact split of t = c - (a + b - 1).  Within
// one split the staged D(k) = c(l3) - c(l3 at the split) is below
// 254 (2 l3 + 255) < 2^24 for l3 <= 2 x 16384, hence exact in float32.
constexpr int kStripRebase = 128;

// Above this lmax the float64 kernels form N' in the WIDE way (two more
// exact pieces per row), since a(a-2) + b(b-2) no longer fits 2^53.
constexpr int kNarrowLmax = 8000;

// Zero guard band around the device copies of g(p) and 1/((2p+1)g(p)).
constexpr int kTablePad = 64;

// Offset of diagonal d of the packed upper-triangle store for lmax:
// diagonal d holds Xi(l1, l1 + d) for l1 = 0 .. lmax - d.
__host__ __device__ inline long long diag_offset(int lmax, int d) {
    return (long long)d * (lmax + 1) - (long long)d * (d - 1) / 2;
}
__host__ __device__ inline long long tri_size(int lmax) {
    return (long long)(lmax + 1) * (lmax + 2) / 2;
}

// Strip kernel modes: Xi_TT; Xi_TT, Xi_TE, Xi_EE (even L); Xi_EB (odd L).
enum { kStripTT = 0, kStripPol = 1, kStripEB = 2, kStripPolEE = 3, kStripEE = 4 };

}  // namespace couple
