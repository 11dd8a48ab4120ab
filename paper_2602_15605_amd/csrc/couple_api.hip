// Host side of the C ABI declared in include/couple.h: argument checks,
// context ownership and the launch sequence
//   scale windows -> strip (l3 reduction on the upper triangle) -> fill or bin.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "couple_internal.hpp"

namespace {

std::string g_init_error;  // text of the last failed couple_init (no context to hold it)

int fail(couple_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_init_error = buf;
    return code;
}

// Optional cap on the device bytes one context may hold (tables, workspace and
// batched workspace), from COUPLE_MAX_DEVICE_BYTES; 0 = no cap.  Checked on the
// host before any allocation, so a request beyond it fails with ENOMEM.
size_t device_byte_cap() {
    const char* v = std::getenv("COUPLE_MAX_DEVICE_BYTES");
    if (!v || !*v) return 0;
    char* end = nullptr;
    const unsigned long long n = std::strtoull(v, &end, 10);
    return (end && *end == '\0') ? (size_t)n : 0;
}

int hip_fail(couple_ctx* ctx, hipError_t e, const char* what) {
    return fail(ctx, COUPLE_EDEVICE, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// Fold recorded event pairs into the per-stage totals.
hipError_t drain_marks(couple_ctx* c) {
    hipError_t first = hipSuccess;
    for (auto& m : c->marks) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(m.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.start, m.stop);
        if (e == hipSuccess) {
            c->prof_ms[m.stage] += ms;
            c->prof_count[m.stage] += 1;
        } else if (first == hipSuccess) {
            first = e;
        }
        (void)hipEventDestroy(m.start);
        (void)hipEventDestroy(m.stop);
    }
    c->marks.clear();
    return first;
}

// Event pair around one launch when the measurement hook is on.
struct Timed {
    couple_ctx* c;
    hipStream_t s;
    int stage;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(couple_ctx* c_, hipStream_t s_, int stage_) : c(c_), s(s_), stage(stage_) {
        if (!c->profiling) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess ||
            hipEventRecord(a, s) != hipSuccess) {
            a = b = nullptr;
        }
    }
    ~Timed() {
        if (!a) return;
        if (hipEventRecord(b, s) == hipSuccess) {
            c->marks.push_back({a, b, stage});
        } else {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    }
};

void release(couple_ctx* c) {
    if (!c) return;
    (void)drain_marks(c);
    if (c->pending_start) (void)hipEventDestroy(c->pending_start);
    (void)hipFree(c->bws);
    (void)hipFree(c->g_pad);
    (void)hipFree(c->h_pad);
    (void)hipFree(c->gf_pad);
    (void)hipFree(c->hf_pad);
    (void)hipFree(c->cl);
    (void)hipFree(c->xi);
    (void)hipFree(c->wp);
    (void)hipFree(c->wpf);
    (void)hipFree(c->wexp);
    (void)hipFree(c->edges_dev);
    if (c->edges_host) (void)hipHostFree(c->edges_host);
    delete c;
}

// Order of outputs (TT, TE, EE, BB) -> Xi source (TT 0, TE 1, EE/BB 2).
int output_sources(unsigned spectra, int* src) {
    int n = 0;
    if (spectra & COUPLE_TT) src[n++] = 0;
    if (spectra & COUPLE_TE) src[n++] = 1;
    if (spectra & COUPLE_EE) src[n++] = 2;
    if (spectra & COUPLE_BB) src[n++] = 2;
    if (spectra & COUPLE_EB) src[n++] = 3;
    return n;
}

// Checks shared by couple_matrix and couple_band.
int check_common(couple_ctx* ctx, const double* W_TT, const double* W_TP, const double* W_PP, int lmax,
                 unsigned spectra, int precision, const double* out) {
    if (lmax < 0 || lmax > ctx->lmax_max)
        return fail(ctx, COUPLE_EINVAL, "lmax=%d outside [0, lmax_max=%d]", lmax, ctx->lmax_max);
    const unsigned spec = spectra & ~(unsigned)COUPLE_XI;
    if (spec == 0 || (spec & ~0x1Fu))
        return fail(ctx, COUPLE_EINVAL,
                    "spectra mask 0x%x: must be a non-empty OR of TT|TE|EE|BB|EB, optionally with COUPLE_XI",
                    spectra);
    if (precision != COUPLE_FP64 && precision != COUPLE_FP32C)
        return fail(ctx, COUPLE_EINVAL,
                    "precision %d: COUPLE_FP64 or COUPLE_FP32C here (the matrix-core forms are batched only)",
                    precision);
    if ((spectra & COUPLE_TT) && !W_TT) return fail(ctx, COUPLE_EINVAL, "TT requested but W_TT is NULL");
    if ((spectra & COUPLE_TE) && !W_TP) return fail(ctx, COUPLE_EINVAL, "TE requested but W_TP is NULL");
    if ((spectra & (COUPLE_EE | COUPLE_BB | COUPLE_EB)) && !W_PP)
        return fail(ctx, COUPLE_EINVAL, "EE/BB/EB requested but W_PP is NULL");
    if (!out) return fail(ctx, COUPLE_EINVAL, "out is NULL");
    if (reinterpret_cast<uintptr_t>(out) % alignof(double))
        return fail(ctx, COUPLE_EINVAL, "out is not 8-byte aligned");
    return COUPLE_OK;
}

// Xi slots a call's strip launches fill per mask: TT, TE, EE, then EB's (odd L).
int xi_slots(unsigned spectra) { return (spectra & COUPLE_EB) ? 4 : 3; }

// Whether a call needs the even-L strip (any of TT, TE, EE, BB).
bool needs_even(unsigned spectra) { return (spectra & (COUPLE_TT | COUPLE_TE | COUPLE_EE | COUPLE_BB)) != 0; }

// The even-L strip mode a call's spectra need.
int strip_mode(unsigned spectra) {
    const bool pol = (spectra & (COUPLE_TE | COUPLE_EE | COUPLE_BB)) != 0;
    return !pol                    ? couple::kStripTT
           : (spectra & COUPLE_TE) ? couple::kStripPol
           : (spectra & COUPLE_TT) ? couple::kStripPolEE
                                   : couple::kStripEE;
}

int run_reduction(couple_ctx* ctx, const double* W_TT, const double* W_TP, const double* W_PP, int lmax,
                  unsigned spectra, int precision, int l3_lo, int l3_hi, hipStream_t s) {
    const bool pol = (spectra & (COUPLE_TE | COUPLE_EE | COUPLE_BB)) != 0;
    const bool even = pol || (spectra & COUPLE_TT);
    // windows are needed for l3 <= min(l3_hi, 2 lmax)
    const int n = std::min(l3_hi, 2 * lmax) + 1;
    hipError_t e;
    {
        Timed t(ctx, s, 0);
        e = couple::launch_scale_windows(ctx, (spectra & COUPLE_TT) ? W_TT : nullptr,
                                         (spectra & COUPLE_TE) ? W_TP : nullptr,
                                         (spectra & (COUPLE_EE | COUPLE_BB | COUPLE_EB)) ? W_PP : nullptr, n, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "scale_windows launch");
    if (precision == COUPLE_FP32C) {
        Timed t(ctx, s, 0);
        e = couple::launch_window_exponents(ctx, n, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "window_exponents launch");
    if (even) {
        Timed t(ctx, s, 1);
        e = couple::launch_strip(ctx, lmax, strip_mode(spectra), precision, l3_lo, std::min(l3_hi, 2 * lmax), s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "strip launch");
    if (spectra & COUPLE_EB) {
        Timed t(ctx, s, 1);
        e = couple::launch_strip(ctx, lmax, couple::kStripEB, precision, l3_lo, std::min(l3_hi, 2 * lmax), s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "odd-L strip launch");
    return COUPLE_OK;
}

}  // namespace

namespace couple {

void prof_begin(couple_ctx* c, hipStream_t s) {
    if (!c->profiling) return;
    if (c->pending_start) (void)hipEventDestroy(c->pending_start);
    c->pending_start = nullptr;
    hipEvent_t a = nullptr;
    if (hipEventCreate(&a) == hipSuccess && hipEventRecord(a, s) == hipSuccess) c->pending_start = a;
    else if (a) (void)hipEventDestroy(a);
}

void prof_end(couple_ctx* c, hipStream_t s, int stage) {
    if (!c->profiling || !c->pending_start) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, s) == hipSuccess) {
        c->marks.push_back({c->pending_start, b, stage});
    } else {
        (void)hipEventDestroy(c->pending_start);
        if (b) (void)hipEventDestroy(b);
    }
    c->pending_start = nullptr;
}

}  // namespace couple

extern "C" {

int couple_init(int lmax_max, couple_ctx** out_ctx) {
    if (!out_ctx) return fail(nullptr, COUPLE_EINVAL, "ctx pointer is NULL");
    *out_ctx = nullptr;
    if (lmax_max < 0 || lmax_max > COUPLE_LMAX_LIMIT)
        return fail(nullptr, COUPLE_EINVAL, "lmax_max=%d outside [0, %d]", lmax_max, COUPLE_LMAX_LIMIT);
    couple_ctx* c = new (std::nothrow) couple_ctx();
    if (!c) return fail(nullptr, COUPLE_ENOMEM, "host allocation of the context failed");
    c->lmax_max = lmax_max;
    const size_t pad = couple::kTablePad;
    const size_t ng = lmax_max + 1 + 2 * pad, nh = 2 * (size_t)lmax_max + 1 + 2 * pad;
    const size_t nw = 3 * (2 * (size_t)lmax_max + 1);
    struct {
        void** p;
        size_t bytes;
    } allocs[] = {
        {(void**)&c->g_pad, ng * sizeof(double)},   {(void**)&c->h_pad, nh * sizeof(double)},
        {(void**)&c->gf_pad, ng * sizeof(float)},   {(void**)&c->hf_pad, nh * sizeof(float)},
        {(void**)&c->cl, (lmax_max + 1) * sizeof(double)},
        {(void**)&c->xi, 4 * (size_t)couple::tri_size(lmax_max) * sizeof(double)},
        {(void**)&c->wp, couple::kBandMasks * nw * sizeof(double)},      {(void**)&c->wpf, nw * sizeof(float)},
        {(void**)&c->wexp, couple::kBandMasks * nw * sizeof(int)},
        {(void**)&c->edges_dev, (lmax_max + 2) * sizeof(int)},
    };
    size_t total = 0;
    for (auto& a : allocs) total += a.bytes;
    const size_t cap = device_byte_cap();
    if (cap && total > cap) {
        release(c);
        return fail(nullptr, COUPLE_ENOMEM, "lmax_max=%d needs %zu device bytes, above COUPLE_MAX_DEVICE_BYTES=%zu",
                    lmax_max, total, cap);
    }
    c->dev_bytes = total;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        release(c);
        return fail(nullptr, COUPLE_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    for (auto& a : allocs) {
        e = hipMalloc(a.p, a.bytes);
        if (e != hipSuccess) {
            release(c);
            return fail(nullptr, COUPLE_ENOMEM, "hipMalloc of %zu bytes: %s", a.bytes, hipGetErrorString(e));
        }
    }
    e = hipHostMalloc((void**)&c->edges_host, (lmax_max + 2) * sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) {
        release(c);
        return fail(nullptr, COUPLE_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    e = couple::launch_build_tables(c, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        release(c);
        return fail(nullptr, COUPLE_EDEVICE, "table build: %s", hipGetErrorString(e));
    }
    // this device's copy of the couple_master_solve_noalloc workspace (device current)
    e = couple::noalloc_scratch(c->device, &c->solve_scratch);
    if (e != hipSuccess) {
        release(c);
        return fail(nullptr, COUPLE_EDEVICE, "hipGetSymbolAddress of the solve workspace: %s",
                    hipGetErrorString(e));
    }
    *out_ctx = c;
    return COUPLE_OK;
}

void couple_free(couple_ctx* ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    release(ctx);
}

const char* couple_last_error(const couple_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

int couple_lmax_max(const couple_ctx* ctx) { return ctx ? ctx->lmax_max : -1; }

int couple_matrix(couple_ctx* ctx, const double* W_TT, const double* W_TP, const double* W_PP, int w_len,
                  int lmax, unsigned spectra, int precision, double* out, void* stream) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    int rc = check_common(ctx, W_TT, W_TP, W_PP, lmax, spectra, precision, out);
    if (rc) return rc;
    if (w_len < 2 * lmax + 1)
        return fail(ctx, COUPLE_EINVAL, "w_len=%d < 2*lmax+1=%d (W_L is needed up to L = 2 lmax)", w_len,
                    2 * lmax + 1);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = run_reduction(ctx, W_TT, W_TP, W_PP, lmax, spectra, precision, 0, 2 * lmax, s);
    if (rc) return rc;
    int src[couple::kMaxOut];
    const int n_out = output_sources(spectra, src);
    hipError_t e;
    {
        Timed t(ctx, s, 2);
        e = couple::launch_fill(ctx, lmax, lmax, src, n_out, out, (spectra & COUPLE_XI) ? 1 : 0, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "fill launch");
    return COUPLE_OK;
}

}  // extern "C"

namespace {

// Checks of couple_band / couple_band_batched beyond check_common.
int check_band(couple_ctx* ctx, int l3_lo, int l3_hi, int w_len, int lmax, const int* bin_edges, int n_bins) {
    if (l3_lo < 0 || l3_hi < l3_lo) return fail(ctx, COUPLE_EINVAL, "bad l3 band [%d, %d]", l3_lo, l3_hi);
    const int hi = std::min(l3_hi, 2 * lmax);
    if (w_len < hi + 1) return fail(ctx, COUPLE_EINVAL, "w_len=%d < %d", w_len, hi + 1);
    if (bin_edges) {
        if (n_bins < 1 || n_bins > lmax + 1)
            return fail(ctx, COUPLE_EINVAL, "n_bins=%d outside [1, lmax+1]", n_bins);
        if (bin_edges[0] < 0 || bin_edges[n_bins] > lmax + 1)
            return fail(ctx, COUPLE_EINVAL, "bin edges must lie in [0, lmax+1]");
        for (int b = 0; b < n_bins; ++b)
            if (bin_edges[b + 1] <= bin_edges[b])
                return fail(ctx, COUPLE_EINVAL, "bin edges must be strictly increasing (at %d)", b);
    }
    return COUPLE_OK;
}

int upload_edges(couple_ctx* ctx, const int* bin_edges, int n_bins, hipStream_t s) {
    // stage through pinned memory; wait for any earlier upload still reading it
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "stream sync before edge upload");
    std::memcpy(ctx->edges_host, bin_edges, (n_bins + 1) * sizeof(int));
    e = hipMemcpyAsync(ctx->edges_dev, ctx->edges_host, (n_bins + 1) * sizeof(int), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "edge upload");
    return COUPLE_OK;
}

// One mask of a band-limited call, edges (if any) already on the device.
int band_one(couple_ctx* ctx, int l3_lo, int l3_hi, const double* W_TT, const double* W_TP, const double* W_PP,
             int lmax, unsigned spectra, int precision, const int* bin_edges, int n_bins, double* out,
             hipStream_t s) {
    const bool binned = bin_edges != nullptr;
    int src[couple::kMaxOut];
    const int n_out = output_sources(spectra, src);
    const int hi = std::min(l3_hi, 2 * lmax);
    const int dmax = std::min(lmax, hi);
    hipError_t e;
    if (l3_lo > hi) {
        // empty band: every element is 0
        const size_t n = binned ? (size_t)n_out * n_bins * n_bins : (size_t)n_out * (lmax + 1) * (lmax + 1);
        e = couple::launch_zero(out, n, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "zero fill launch");
        return COUPLE_OK;
    }
    int rc = run_reduction(ctx, W_TT, W_TP, W_PP, lmax, spectra, precision, l3_lo, hi, s);
    if (rc) return rc;
    {
        Timed t(ctx, s, 2);
        const int xi = (spectra & COUPLE_XI) ? 1 : 0;
        e = binned ? couple::launch_bin(ctx, lmax, dmax, src, n_out, bin_edges, ctx->edges_dev, n_bins, out, xi, s)
                   : couple::launch_fill(ctx, lmax, dmax, src, n_out, out, xi, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, binned ? "bin launch" : "fill launch");
    return COUPLE_OK;
}

// Masks per launch of the multi-mask strips for a batched band call, or 1
// where they do not apply: they need FP32C or FP64, a non-empty band, room in
// the Xi workspace for the group's triangles of diagonals 0 .. dmax (three per
// mask, TT, TE and EE slots, four with EB), and for EB in FP32C the lanes of
// the one-mask strip (strip_masks_bitwise).
int masks_per_launch(const couple_ctx* ctx, int n_masks, int l3_lo, int l3_hi, int lmax, unsigned spectra,
                     int precision) {
    if ((precision != COUPLE_FP32C && precision != COUPLE_FP64) || n_masks < 2) return 1;
    const int hi = std::min(l3_hi, 2 * lmax);
    if (l3_lo > hi) return 1;
    if ((spectra & COUPLE_EB) && !couple::strip_masks_bitwise(couple::kStripEB, precision, lmax, hi)) return 1;
    const long long band = couple::diag_offset(lmax, std::min(lmax, hi) + 1);
    const long long room = 4 * couple::tri_size(ctx->lmax_max) / (xi_slots(spectra) * band);
    int per = couple::kBandMasks;
    if (needs_even(spectra)) per = std::min(per, couple::strip_masks_per_launch(strip_mode(spectra), precision));
    if (spectra & COUPLE_EB) per = std::min(per, couple::strip_masks_per_launch(couple::kStripEB, precision));
    return (int)std::min<long long>({(long long)per, room, (long long)n_masks});
}

// n_masks (<= kBandMasks) masks of a batched band call in one strip launch
// (and one odd-L launch for EB): their windows are scaled into the context's
// window sets 0 .. n_masks - 1, the strips write each mask's Xi triangles
// (stride: diagonals 0 .. dmax) one after the other, and one bin (or fill)
// launch serves every mask of the group.
int band_masks(couple_ctx* ctx, int n_masks, int l3_lo, int l3_hi, const double* const* W_TT,
               const double* const* W_TP, const double* const* W_PP, int lmax, unsigned spectra, int precision,
               const int* bin_edges, int n_bins, double* out, size_t per_mask, hipStream_t s) {
    const int hi = std::min(l3_hi, 2 * lmax);
    const int dmax = std::min(lmax, hi);
    const int n = hi + 1;
    const long long stride = couple::diag_offset(lmax, dmax + 1);
    const long long mask_stride = xi_slots(spectra) * stride;
    hipError_t e;
    {
        Timed t(ctx, s, 0);
        e = couple::launch_scale_windows_masks(ctx, (spectra & COUPLE_TT) ? W_TT : nullptr,
                                               (spectra & COUPLE_TE) ? W_TP : nullptr,
                                               (spectra & (COUPLE_EE | COUPLE_BB | COUPLE_EB)) ? W_PP : nullptr,
                                               n_masks, n, nullptr, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "scale_windows launch");
    if (precision == COUPLE_FP32C) {
        Timed t(ctx, s, 0);
        e = couple::launch_window_exponents(ctx, n, s, n_masks);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "window_exponents launch");
    {
        Timed t(ctx, s, 1);
        int lm[couple::kBandMasks];
        long long off[couple::kBandMasks];
        for (int m = 0; m < n_masks; ++m) {
            lm[m] = lmax;
            off[m] = mask_stride * m;
        }
        if (needs_even(spectra))
            e = couple::launch_strip_masks(ctx, strip_mode(spectra), precision, n_masks, lm, ctx->xi, off, l3_lo,
                                           hi, s);
        if (e == hipSuccess && (spectra & COUPLE_EB))
            e = couple::launch_strip_masks(ctx, couple::kStripEB, precision, n_masks, lm, ctx->xi, off, l3_lo, hi,
                                           s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "multi-mask strip launch");
    int src[couple::kMaxOut];
    const int n_out = output_sources(spectra, src);
    const int xi = (spectra & COUPLE_XI) ? 1 : 0;
    if (bin_edges) {
        // one zero and one bin launch for the group's masks (outputs per_mask apart)
        Timed t(ctx, s, 2);
        e = couple::launch_bin(ctx, lmax, dmax, src, n_out, bin_edges, ctx->edges_dev, n_bins, out, xi, s, ctx->xi,
                               stride, n_masks, mask_stride);
    } else {
        // one fill launch for the group's masks
        couple::FillJob jobs[couple::kBandMasks];
        for (int m = 0; m < n_masks; ++m) {
            jobs[m].xi = ctx->xi + mask_stride * m;
            jobs[m].xi_stride = stride;
            jobs[m].out = out + m * per_mask;
            jobs[m].lmax = lmax;
            jobs[m].dmax = dmax;
            jobs[m].block0 = 0;
        }
        Timed t(ctx, s, 2);
        e = couple::launch_fill_jobs(jobs, n_masks, src, n_out, xi, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, bin_edges ? "bin launch" : "fill launch");
    return COUPLE_OK;
}

}  // namespace

extern "C" {

int couple_band(couple_ctx* ctx, int l3_lo, int l3_hi, const double* W_TT, const double* W_TP,
                const double* W_PP, int w_len, int lmax, unsigned spectra, int precision, const int* bin_edges,
                int n_bins, double* out, void* stream) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    int rc = check_common(ctx, W_TT, W_TP, W_PP, lmax, spectra, precision, out);
    if (rc) return rc;
    rc = check_band(ctx, l3_lo, l3_hi, w_len, lmax, bin_edges, n_bins);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (bin_edges && n_bins > couple::kInlineBins) {
        rc = upload_edges(ctx, bin_edges, n_bins, s);
        if (rc) return rc;
    }
    return band_one(ctx, l3_lo, l3_hi, W_TT, W_TP, W_PP, lmax, spectra, precision, bin_edges, n_bins, out, s);
}

int couple_band_batched(couple_ctx* ctx, int n_masks, int l3_lo, int l3_hi, const double* const* W_TT,
                        const double* const* W_TP, const double* const* W_PP, int w_len, int lmax,
                        unsigned spectra, int precision, const int* bin_edges, int n_bins, double* out,
                        void* stream) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    if (n_masks < 1) return fail(ctx, COUPLE_EINVAL, "n_masks=%d < 1", n_masks);
    const bool need_tt = spectra & COUPLE_TT, need_tp = spectra & COUPLE_TE,
               need_pp = spectra & (COUPLE_EE | COUPLE_BB | COUPLE_EB);
    if ((need_tt && !W_TT) || (need_tp && !W_TP) || (need_pp && !W_PP))
        return fail(ctx, COUPLE_EINVAL, "a requested spectrum's window array is NULL");
    for (int m = 0; m < n_masks; ++m) {
        int rc = check_common(ctx, need_tt ? W_TT[m] : nullptr, need_tp ? W_TP[m] : nullptr,
                              need_pp ? W_PP[m] : nullptr, lmax, spectra, precision, out);
        if (rc) {
            ctx->err = "mask " + std::to_string(m) + ": " + ctx->err;
            return rc;
        }
    }
    int rc = check_band(ctx, l3_lo, l3_hi, w_len, lmax, bin_edges, n_bins);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (bin_edges && n_bins > couple::kInlineBins) {
        rc = upload_edges(ctx, bin_edges, n_bins, s);
        if (rc) return rc;
    }
    int src[couple::kMaxOut];
    const int n_out = output_sources(spectra, src);
    const size_t per_mask = bin_edges ? (size_t)n_out * n_bins * n_bins : (size_t)n_out * (lmax + 1) * (lmax + 1);
    const int group = masks_per_launch(ctx, n_masks, l3_lo, l3_hi, lmax, spectra, precision);
    if (group > 1) {
        for (int m0 = 0; m0 < n_masks; m0 += group) {
            const int g = std::min(group, n_masks - m0);
            rc = band_masks(ctx, g, l3_lo, l3_hi, need_tt ? W_TT + m0 : nullptr, need_tp ? W_TP + m0 : nullptr,
                            need_pp ? W_PP + m0 : nullptr, lmax, spectra, precision, bin_edges, n_bins,
                            out + m0 * per_mask, per_mask, s);
            if (rc) return rc;
        }
        return COUPLE_OK;
    }
    for (int m = 0; m < n_masks; ++m) {
        rc = band_one(ctx, l3_lo, l3_hi, need_tt ? W_TT[m] : nullptr, need_tp ? W_TP[m] : nullptr,
                      need_pp ? W_PP[m] : nullptr, lmax, spectra, precision, bin_edges, n_bins,
                      out + m * per_mask, s);
        if (rc) return rc;
    }
    return COUPLE_OK;
}

}  // extern "C"

namespace {

// Batched FP32C or FP64 full matrices through the multi-mask strips: masks
// sorted[0 .. n_masks - 1] (indices into lmax_i, W_*, out), in order of lmax,
// descending; groups of strip_masks_per_launch consecutive masks, one strip
// launch each (two with EB: even and odd L) over the grid of the group's
// largest lmax (a smaller mask's terms outside its triangle are formed and not
// stored; its windows are 0 beyond its 2 lmax).  Their Xi stores lie side by side in the
// batched workspace when it is reserved for all of them, else in the
// context's Xi workspace; one fill launch follows for the masks it holds.
int matrix_masks(couple_ctx* ctx, int n_masks, const int* sorted, const int* lmax_i, const double* const* W_TT,
                 const double* const* W_TP, const double* const* W_PP, unsigned spectra, int precision,
                 double* const* out, hipStream_t s) {
    const int mode = strip_mode(spectra);
    const bool even = needs_even(spectra), eb = (spectra & COUPLE_EB) != 0;
    const int slots = xi_slots(spectra);
    int per = couple::kBandMasks;
    if (even) per = std::min(per, couple::strip_masks_per_launch(mode, precision));
    if (eb) per = std::min(per, couple::strip_masks_per_launch(couple::kStripEB, precision));
    long long total = 0;
    for (int i = 0; i < n_masks; ++i) total += slots * couple::tri_size(lmax_i[sorted[i]]);
    double* buf = ctx->xi;
    long long cap = 4 * couple::tri_size(ctx->lmax_max);
    if (ctx->bws && (long long)(ctx->bws_bytes / sizeof(double)) >= total && total > cap) {
        buf = static_cast<double*>(ctx->bws);
        cap = (long long)(ctx->bws_bytes / sizeof(double));
    }
    int src[couple::kMaxOut];
    const int n_out = output_sources(spectra, src);
    const int xi_only = (spectra & COUPLE_XI) ? 1 : 0;
    hipError_t e = hipSuccess;
    int i = 0;
    while (i < n_masks) {
        couple::FillJob jobs[couple::kMaxFillJobs];
        int n_jobs = 0;
        long long used = 0;
        while (i < n_masks && n_jobs < couple::kMaxFillJobs) {
            int g = std::min({per, n_masks - i, couple::kMaxFillJobs - n_jobs});
            auto need = [&](int k) {
                long long b = 0;
                for (int q = 0; q < k; ++q) b += slots * couple::tri_size(lmax_i[sorted[i + q]]);
                return b;
            };
            while (g > 0 && used + need(g) > cap) --g;
            // float64 forms N' by the group's largest lmax: keep a group on one side of kNarrowLmax
            while (g > 1 && (lmax_i[sorted[i + g - 1]] > couple::kNarrowLmax) !=
                                (lmax_i[sorted[i]] > couple::kNarrowLmax))
                --g;
            // FP32C's EB rows round from the lane's first row, and the group's grid puts a
            // mask's rows in lanes as the one-mask grid does only when their lmax agree mod
            // the rows per lane
            if (eb && precision == COUPLE_FP32C)
                for (int q = 1; q < g; ++q)
                    if ((lmax_i[sorted[i]] - lmax_i[sorted[i + q]]) % couple::kStripR != 0) {
                        g = q;
                        break;
                    }
            if (g == 0) break;
            int lm[couple::kBandMasks], nm[couple::kBandMasks];
            long long off[couple::kBandMasks];
            const double *wt[couple::kBandMasks], *wtp[couple::kBandMasks], *wpp[couple::kBandMasks];
            long long o = used;
            for (int k = 0; k < g; ++k) {
                const int m = sorted[i + k];
                lm[k] = lmax_i[m];
                nm[k] = 2 * lm[k] + 1;
                off[k] = o;
                o += slots * couple::tri_size(lm[k]);
                wt[k] = (spectra & COUPLE_TT) ? W_TT[m] : nullptr;
                wtp[k] = (spectra & COUPLE_TE) ? W_TP[m] : nullptr;
                wpp[k] = (spectra & (COUPLE_EE | COUPLE_BB | COUPLE_EB)) ? W_PP[m] : nullptr;
                couple::FillJob& j = jobs[n_jobs++];
                j.xi = buf + off[k];
                j.xi_stride = couple::tri_size(lm[k]);
                j.out = out[m];
                j.lmax = lm[k];
                j.dmax = lm[k];
                j.block0 = 0;
            }
            const int L = *std::max_element(lm, lm + g);
            {
                Timed t(ctx, s, 0);
                e = couple::launch_scale_windows_masks(ctx, wt, wtp, wpp, g, 2 * L + 1, nm, s);
            }
            if (e != hipSuccess) return hip_fail(ctx, e, "scale_windows launch");
            if (precision == COUPLE_FP32C) {
                Timed t(ctx, s, 0);
                e = couple::launch_window_exponents(ctx, 2 * L + 1, s, g);
            }
            if (e != hipSuccess) return hip_fail(ctx, e, "window_exponents launch");
            {
                Timed t(ctx, s, 1);
                if (even) e = couple::launch_strip_masks(ctx, mode, precision, g, lm, buf, off, 0, 2 * L, s);
                if (e == hipSuccess && eb)
                    e = couple::launch_strip_masks(ctx, couple::kStripEB, precision, g, lm, buf, off, 0, 2 * L, s);
            }
            if (e != hipSuccess) return hip_fail(ctx, e, "multi-mask strip launch");
            used = o;
            i += g;
        }
        if (n_jobs == 0) return fail(ctx, COUPLE_EDEVICE, "no room for one mask's Xi");
        {
            Timed t(ctx, s, 2);
            e = couple::launch_fill_jobs(jobs, n_jobs, src, n_out, xi_only, s);
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "fill launch");
    }
    return COUPLE_OK;
}

// Sort masks by lmax (descending, stable) into column groups of 16.
int make_plan(couple_ctx* ctx, int n_masks, const int* lmax_i, couple::BatchPlan* p, int* order) {
    if (n_masks < 1 || n_masks > couple::kMaxGroups * couple::kMaskGroup)
        return fail(ctx, COUPLE_EINVAL, "n_masks=%d outside [1, %d]", n_masks,
                    couple::kMaxGroups * couple::kMaskGroup);
    if (!lmax_i) return fail(ctx, COUPLE_EINVAL, "lmax_i is NULL");
    for (int m = 0; m < n_masks; ++m) {
        if (lmax_i[m] < 0 || lmax_i[m] > ctx->lmax_max)
            return fail(ctx, COUPLE_EINVAL, "mask %d: lmax=%d outside [0, lmax_max=%d]", m, lmax_i[m],
                        ctx->lmax_max);
        order[m] = m;
    }
    for (int i = 1; i < n_masks; ++i) {
        const int v = order[i];
        int j = i;
        while (j > 0 && lmax_i[order[j - 1]] < lmax_i[v]) {
            order[j] = order[j - 1];
            --j;
        }
        order[j] = v;
    }
    p->n_groups = (n_masks + couple::kMaskGroup - 1) / couple::kMaskGroup;
    for (int gi = 0; gi < p->n_groups; ++gi) {
        p->n_masks[gi] = std::min(couple::kMaskGroup, n_masks - gi * couple::kMaskGroup);
        p->L[gi] = lmax_i[order[gi * couple::kMaskGroup]];
        for (int m = 0; m < couple::kMaskGroup; ++m) {
            p->lmax[gi][m] = m < p->n_masks[gi] ? lmax_i[order[gi * couple::kMaskGroup + m]] : -1;
            p->out[gi][m] = nullptr;
            for (int x = 0; x < 3; ++x) p->w[gi][x][m] = nullptr;
        }
    }
    return COUPLE_OK;
}

}  // namespace

extern "C" {

int couple_reserve_batched(couple_ctx* ctx, int n_masks, const int* lmax_i) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    couple::BatchPlan p;
    int order[couple::kMaxGroups * couple::kMaskGroup];
    int rc = make_plan(ctx, n_masks, lmax_i, &p, order);
    if (rc) return rc;
    const size_t need = couple::batched_workspace_bytes(p);
    if (need <= ctx->bws_bytes) return COUPLE_OK;
    const size_t cap = device_byte_cap();
    if (cap && ctx->dev_bytes + need > cap)
        return fail(ctx, COUPLE_ENOMEM,
                    "the batched workspace needs %zu device bytes; with the context's %zu that is above "
                    "COUPLE_MAX_DEVICE_BYTES=%zu",
                    need, ctx->dev_bytes, cap);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "sync before workspace change");
    (void)hipFree(ctx->bws);
    ctx->bws = nullptr;
    ctx->bws_bytes = 0;
    e = hipMalloc(&ctx->bws, need);
    if (e != hipSuccess) {
        ctx->bws = nullptr;
        return fail(ctx, COUPLE_ENOMEM, "hipMalloc of %zu bytes for the batched workspace: %s", need,
                    hipGetErrorString(e));
    }
    ctx->bws_bytes = need;
    return COUPLE_OK;
}

int couple_matrix_batched(couple_ctx* ctx, int n_masks, const int* lmax_i, const double* const* W_TT,
                          const double* const* W_TP, const double* const* W_PP, const int* w_len_i,
                          unsigned spectra, int precision, double* const* out, void* stream) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    couple::BatchPlan p;
    int order[couple::kMaxGroups * couple::kMaskGroup];
    int rc = make_plan(ctx, n_masks, lmax_i, &p, order);
    if (rc) return rc;
    if (!w_len_i || !out) return fail(ctx, COUPLE_EINVAL, "w_len_i or out is NULL");
    const bool need_tt = spectra & COUPLE_TT, need_tp = spectra & COUPLE_TE,
               need_pp = spectra & (COUPLE_EE | COUPLE_BB | COUPLE_EB);
    if ((need_tt && !W_TT) || (need_tp && !W_TP) || (need_pp && !W_PP))
        return fail(ctx, COUPLE_EINVAL, "a requested spectrum's window array is NULL");
    const bool mfma = precision == COUPLE_MFMA_FP32 || precision == COUPLE_MFMA_BF16X3;
    if (mfma && (spectra & COUPLE_EB))
        return fail(ctx, COUPLE_ENOTSUP, "EB is not in the matrix-core batched form (use COUPLE_FP64 or COUPLE_FP32C)");
    for (int m = 0; m < n_masks; ++m) {
        rc = check_common(ctx, need_tt ? W_TT[m] : nullptr, need_tp ? W_TP[m] : nullptr,
                          need_pp ? W_PP[m] : nullptr, lmax_i[m], spectra, mfma ? COUPLE_FP64 : precision,
                          out[m]);
        if (rc == COUPLE_OK && w_len_i[m] < 2 * lmax_i[m] + 1)
            rc = fail(ctx, COUPLE_EINVAL, "w_len=%d < 2*lmax+1=%d", w_len_i[m], 2 * lmax_i[m] + 1);
        if (rc) {
            ctx->err = "mask " + std::to_string(m) + ": " + ctx->err;
            return rc;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int sorted[couple::kMaxGroups * couple::kMaskGroup];
    int n_sorted = 0;
    for (int gi = 0; gi < p.n_groups; ++gi)
        for (int m = 0; m < p.n_masks[gi]; ++m) sorted[n_sorted++] = order[gi * couple::kMaskGroup + m];
    // masks (sorted by lmax, descending) through the multi-mask strips: all of them, but with
    // EB only those whose one-mask strip gets the same bits (strip_masks_bitwise holds from
    // some lmax up); the rest run couple_matrix one by one
    int n_multi = 0;
    if ((precision == COUPLE_FP32C || precision == COUPLE_FP64) && n_masks >= 2) {
        n_multi = n_masks;
        if (spectra & COUPLE_EB)
            while (n_multi > 0 && !couple::strip_masks_bitwise(couple::kStripEB, precision, lmax_i[sorted[n_multi - 1]],
                                                               2 * lmax_i[sorted[n_multi - 1]]))
                --n_multi;
        if (n_multi < 2) n_multi = 0;
    }
    if (n_multi > 0) {
        rc = matrix_masks(ctx, n_multi, sorted, lmax_i, W_TT, W_TP, W_PP, spectra, precision, out, s);
        if (rc) return rc;
    }
    if (!mfma) {
        // float64 / float32-compensated: one couple_matrix per remaining mask, back to back on s
        for (int i = n_multi; i < n_masks; ++i) {
            const int m = sorted[i];
            rc = couple_matrix(ctx, need_tt ? W_TT[m] : nullptr, need_tp ? W_TP[m] : nullptr,
                               need_pp ? W_PP[m] : nullptr, w_len_i[m], lmax_i[m], spectra, precision, out[m],
                               stream);
            if (rc) {
                ctx->err = "mask " + std::to_string(m) + ": " + ctx->err;
                return rc;
            }
        }
        return COUPLE_OK;
    }
    const size_t need = couple::batched_workspace_bytes(p);
    if (need > ctx->bws_bytes)
        return fail(ctx, COUPLE_EINVAL, "batched workspace too small (%zu < %zu bytes): call couple_reserve_batched",
                    ctx->bws_bytes, need);
    for (int gi = 0; gi < p.n_groups; ++gi)
        for (int m = 0; m < p.n_masks[gi]; ++m) {
            const int src = order[gi * couple::kMaskGroup + m];
            p.w[gi][0][m] = need_tt ? W_TT[src] : nullptr;
            p.w[gi][1][m] = need_tp ? W_TP[src] : nullptr;
            p.w[gi][2][m] = need_pp ? W_PP[src] : nullptr;
            p.out[gi][m] = out[src];
        }
    const int ti = precision == COUPLE_MFMA_BF16X3 ? 1 : 0;
    p.flush = ctx->batched_flush[ti];
    p.tm = ctx->batched_tm[ti];
    int src4[couple::kMaxOut];
    const int n_out = output_sources(spectra, src4);
    hipError_t e = couple::launch_batched(ctx, p, precision, src4, n_out, (spectra & COUPLE_XI) ? 1 : 0, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "batched launch");
    return COUPLE_OK;
}

namespace {
int tile_index(couple_ctx* ctx, int precision, int* ti) {
    if (precision == COUPLE_MFMA_FP32) {
        *ti = 0;
        return COUPLE_OK;
    }
    if (precision == COUPLE_MFMA_BF16X3) {
        *ti = 1;
        return COUPLE_OK;
    }
    return fail(ctx, COUPLE_EINVAL, "precision=%d has no batched tile shape (COUPLE_MFMA_FP32 or COUPLE_MFMA_BF16X3)",
                precision);
}
}  // namespace

int couple_set_batched_tiles(couple_ctx* ctx, int precision, int row_tiles, int flush) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    int ti;
    int rc = tile_index(ctx, precision, &ti);
    if (rc) return rc;
    if (ti == 0 && (row_tiles == 64 || row_tiles == 128)) {
        // the 4-mask form: flush in groups of 16 l3 steps
        if (flush < 1 || flush > 4) return fail(ctx, COUPLE_EINVAL, "flush=%d outside [1, 4] (16-step groups)", flush);
    } else {
        if (row_tiles != 1 && row_tiles != 2 && row_tiles != 4)
            return fail(ctx, COUPLE_EINVAL, "row_tiles=%d: must be 1, 2 or 4%s", row_tiles,
                        ti == 0 ? " (16-mask form) or 64, 128 (4-mask form)" : "");
        if (flush < 1 || flush > 16) return fail(ctx, COUPLE_EINVAL, "flush=%d outside [1, 16]", flush);
    }
    ctx->batched_tm[ti] = row_tiles;
    ctx->batched_flush[ti] = flush;
    return COUPLE_OK;
}

int couple_get_batched_tiles(couple_ctx* ctx, int precision, int* row_tiles, int* flush) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    int ti;
    int rc = tile_index(ctx, precision, &ti);
    if (rc) return rc;
    if (row_tiles) *row_tiles = ctx->batched_tm[ti];
    if (flush) *flush = ctx->batched_flush[ti];
    return COUPLE_OK;
}

int couple_autotune_batched(couple_ctx* ctx, int precision, int n_masks, const int* lmax_i,
                            const double* const* W_TT, const double* const* W_TP, const double* const* W_PP,
                            const int* w_len_i, unsigned spectra, double* const* out, void* stream,
                            int* best_row_tiles, int* best_flush, float* best_ms) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    int ti;
    int rc = tile_index(ctx, precision, &ti);
    if (rc) return rc;
    // (row_tiles, flush) candidates.  float32: the 16-mask form (flush every 16 or 32 l3)
    // and the 4-mask form (flush every 32 l3); BF16x3: flush every 64 or 128 l3.
    static const int kCand[2][8][2] = {{{1, 4}, {1, 8}, {2, 4}, {2, 8}, {4, 4}, {4, 8}, {64, 2}, {128, 2}},
                                       {{1, 2}, {1, 4}, {2, 2}, {2, 4}, {4, 2}, {4, 4}, {0, 0}, {0, 0}}};
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(ctx, COUPLE_EDEVICE, "event creation failed");
    }
    const int tm0 = ctx->batched_tm[ti], fl0 = ctx->batched_flush[ti];
    float best = 3.4e38f;
    int btm = tm0, bfl = fl0;
    for (const auto& cand : kCand[ti]) {
        const int tm = cand[0], fl = cand[1];
        if (tm == 0) continue;
        ctx->batched_tm[ti] = tm;
        ctx->batched_flush[ti] = fl;
        rc = couple_matrix_batched(ctx, n_masks, lmax_i, W_TT, W_TP, W_PP, w_len_i, spectra, precision, out,
                                   stream);  // warm-up (and argument check)
        if (rc) break;
        (void)hipEventRecord(e0, s);
        rc = couple_matrix_batched(ctx, n_masks, lmax_i, W_TT, W_TP, W_PP, w_len_i, spectra, precision, out,
                                   stream);
        (void)hipEventRecord(e1, s);
        if (rc) break;
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = hip_fail(ctx, e, "autotune timing");
            break;
        }
        if (ms < best) {
            best = ms;
            btm = tm;
            bfl = fl;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        ctx->batched_tm[ti] = tm0;
        ctx->batched_flush[ti] = fl0;
        return rc;
    }
    ctx->batched_tm[ti] = btm;
    ctx->batched_flush[ti] = bfl;
    if (best_row_tiles) *best_row_tiles = btm;
    if (best_flush) *best_flush = bfl;
    if (best_ms) *best_ms = best;
    return COUPLE_OK;
}

int couple_tables(const couple_ctx* ctx, double* g, double* h, double* cl, float* gf, float* hf) {
    if (!ctx) return COUPLE_EINVAL;
    couple_ctx* c = const_cast<couple_ctx*>(ctx);
    const size_t pad = couple::kTablePad;
    const size_t ng = ctx->lmax_max + 1, nh = 2 * (size_t)ctx->lmax_max + 1;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && g) e = hipMemcpy(g, ctx->g_pad + pad, ng * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && h) e = hipMemcpy(h, ctx->h_pad + pad, nh * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && cl) e = hipMemcpy(cl, ctx->cl, ng * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && gf) e = hipMemcpy(gf, ctx->gf_pad + pad, ng * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess && hf) e = hipMemcpy(hf, ctx->hf_pad + pad, nh * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "table copy");
    return COUPLE_OK;
}

int couple_profile(couple_ctx* ctx, int enable) {
    if (!ctx) return COUPLE_EINVAL;
    hipError_t e = drain_marks(ctx);
    for (int i = 0; i < COUPLE_N_STAGES; ++i) {
        ctx->prof_ms[i] = 0.0;
        ctx->prof_count[i] = 0;
    }
    ctx->profiling = enable != 0;
    if (e != hipSuccess) return hip_fail(ctx, e, "profile reset");
    return COUPLE_OK;
}

int couple_profile_read(couple_ctx* ctx, double* ms, int* counts) {
    if (!ctx) return COUPLE_EINVAL;
    hipError_t e = drain_marks(ctx);
    for (int i = 0; i < COUPLE_N_STAGES; ++i) {
        if (ms) ms[i] = ctx->prof_ms[i];
        if (counts) counts[i] = ctx->prof_count[i];
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "profile read");
    return COUPLE_OK;
}

}  // extern "C"

extern "C" {

int couple_bin_spectra(couple_ctx* ctx, int n_spec, const double* cl, int cl_len, const int* bin_edges, int n_bins,
                       double* out, void* stream) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    if (n_spec < 1) return fail(ctx, COUPLE_EINVAL, "n_spec=%d < 1", n_spec);
    if (!cl || !out) return fail(ctx, COUPLE_EINVAL, "cl or out is NULL");
    if (reinterpret_cast<uintptr_t>(cl) % alignof(double) || reinterpret_cast<uintptr_t>(out) % alignof(double))
        return fail(ctx, COUPLE_EINVAL, "cl or out is not 8-byte aligned");
    if (!bin_edges) return fail(ctx, COUPLE_EINVAL, "bin_edges is NULL");
    if (n_bins < 1 || n_bins > ctx->lmax_max + 1)
        return fail(ctx, COUPLE_EINVAL, "n_bins=%d outside [1, lmax_max+1=%d]", n_bins, ctx->lmax_max + 1);
    if (bin_edges[0] < 0 || bin_edges[n_bins] > cl_len)
        return fail(ctx, COUPLE_EINVAL, "bin edges must lie in [0, cl_len=%d]", cl_len);
    for (int b = 0; b < n_bins; ++b)
        if (bin_edges[b + 1] <= bin_edges[b])
            return fail(ctx, COUPLE_EINVAL, "bin edges must be strictly increasing (at %d)", b);
    if ((long long)n_spec * n_bins > 0x7fffffffLL) return fail(ctx, COUPLE_EINVAL, "n_spec * n_bins too large");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n_bins > couple::kInlineBins) {
        int rc = upload_edges(ctx, bin_edges, n_bins, s);
        if (rc) return rc;
    }
    hipError_t e = couple::launch_bin_spectra(ctx, n_spec, cl, cl_len, bin_edges, n_bins, out, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "bin_spectra launch");
    return COUPLE_OK;
}

int couple_master_solve(couple_ctx* ctx, int pol, int n, const double* K, int n_rhs, const double* rhs, double* work,
                        double* x, void* stream) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    if (pol != 0 && pol != 1) return fail(ctx, COUPLE_EINVAL, "pol=%d: 0 (TT) or 1 (E/B block)", pol);
    if (n < 1 || n_rhs < 1) return fail(ctx, COUPLE_EINVAL, "n=%d and n_rhs=%d must be >= 1", n, n_rhs);
    const long long m = pol ? 2LL * n : n;
    if (m + n_rhs > couple::kSolveMaxCols)
        return fail(ctx, COUPLE_EINVAL, "%lld unknowns + %d right-hand sides exceed %d", m, n_rhs,
                    couple::kSolveMaxCols);
    const double* ptrs[] = {K, rhs, work, x};
    for (const double* p : ptrs) {
        if (!p) return fail(ctx, COUPLE_EINVAL, "K, rhs, work and x must be non-NULL");
        if (reinterpret_cast<uintptr_t>(p) % alignof(double))
            return fail(ctx, COUPLE_EINVAL, "K, rhs, work and x must be 8-byte aligned");
    }
    hipError_t e = couple::launch_master_solve(pol, n, K, n_rhs, rhs, work, x, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "master_solve launch");
    return COUPLE_OK;
}

int couple_master_solve_noalloc(couple_ctx* ctx, int pol, int n, const double* K, int n_rhs, const double* rhs,
                                double* x, void* stream) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    if (pol != 0 && pol != 1) return fail(ctx, COUPLE_EINVAL, "pol=%d: 0 (TT) or 1 (E/B block)", pol);
    if (n < 1 || n_rhs < 1) return fail(ctx, COUPLE_EINVAL, "n=%d and n_rhs=%d must be >= 1", n, n_rhs);
    const long long m = pol ? 2LL * n : n;
    if (m + n_rhs > couple::kSolveMaxCols)
        return fail(ctx, COUPLE_EINVAL, "%lld unknowns + %d right-hand sides exceed %d", m, n_rhs,
                    couple::kSolveMaxCols);
    if (m * (m + n_rhs) > couple::kNoallocSolveDoubles)
        return fail(ctx, COUPLE_EINVAL,
                    "the system needs %lld x %lld float64, more than the %lld of the static workspace "
                    "(use couple_master_solve with a workspace)",
                    m, m + n_rhs, couple::kNoallocSolveDoubles);
    const double* ptrs[] = {K, rhs, x};
    for (const double* p : ptrs) {
        if (!p) return fail(ctx, COUPLE_EINVAL, "K, rhs and x must be non-NULL");
        if (reinterpret_cast<uintptr_t>(p) % alignof(double))
            return fail(ctx, COUPLE_EINVAL, "K, rhs and x must be 8-byte aligned");
    }
    if (!ctx->solve_scratch) return fail(ctx, COUPLE_EDEVICE, "the static solve workspace has no address");
    hipError_t e = couple::launch_master_solve(pol, n, K, n_rhs, rhs, ctx->solve_scratch, x,
                                               static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "master_solve launch");
    return COUPLE_OK;
}

}  // extern "C"

extern "C" {

int couple_threej_rows(couple_ctx* ctx, int m, int n_pairs, const int* l1, const int* l2, double* out,
                       long long stride, void* stream) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    if (m < 0 || m > 2) return fail(ctx, COUPLE_EINVAL, "m=%d: 0, 1 or 2 ((l1 l2 l3; -m m 0))", m);
    if (n_pairs < 1) return fail(ctx, COUPLE_EINVAL, "n_pairs=%d < 1", n_pairs);
    if (stride < 1) return fail(ctx, COUPLE_EINVAL, "stride=%lld < 1", stride);
    if (!l1 || !l2 || !out) return fail(ctx, COUPLE_EINVAL, "l1, l2 and out must be non-NULL");
    if (reinterpret_cast<uintptr_t>(l1) % alignof(int) || reinterpret_cast<uintptr_t>(l2) % alignof(int) ||
        reinterpret_cast<uintptr_t>(out) % alignof(double))
        return fail(ctx, COUPLE_EINVAL, "l1, l2 (4 bytes) or out (8 bytes) misaligned");
    hipError_t e = couple::launch_threej_rows(ctx, m, n_pairs, l1, l2, out, stride, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "threej_rows launch");
    return COUPLE_OK;
}

int couple_threej_rows_m(couple_ctx* ctx, int m1, int m2, int n_pairs, const int* l1, const int* l2, double* out,
                         long long stride, void* stream) {
    if (!ctx) return COUPLE_EINVAL;
    ctx->err.clear();
    // canonical form: rotate the columns until the first two magnetic numbers
    // share a sign, flip them to >= 0 if needed; both must then be <= 2
    const long long ms[3] = {m1, m2, -(long long)m1 - m2};
    int rot = -1, flip = 0, fa = 0, fb = 0;
    for (int r = 0; r < 3 && rot < 0; ++r) {
        const long long p = ms[r], q = ms[(r + 1) % 3];
        if (p >= 0 && q >= 0 && p <= 2 && q <= 2) {
            rot = r, flip = 0, fa = (int)p, fb = (int)q;
        } else if (p <= 0 && q <= 0 && p >= -2 && q >= -2) {
            rot = r, flip = 1, fa = (int)-p, fb = (int)-q;
        }
    }
    if (rot < 0)
        return fail(ctx, COUPLE_EINVAL,
                    "(m1, m2, m3) = (%d, %d, %lld): the two entries of equal sign must be at most 2 in magnitude", m1,
                    m2, ms[2]);
    if (n_pairs < 1) return fail(ctx, COUPLE_EINVAL, "n_pairs=%d < 1", n_pairs);
    if (stride < 1) return fail(ctx, COUPLE_EINVAL, "stride=%lld < 1", stride);
    if (!l1 || !l2 || !out) return fail(ctx, COUPLE_EINVAL, "l1, l2 and out must be non-NULL");
    if (reinterpret_cast<uintptr_t>(l1) % alignof(int) || reinterpret_cast<uintptr_t>(l2) % alignof(int) ||
        reinterpret_cast<uintptr_t>(out) % alignof(double))
        return fail(ctx, COUPLE_EINVAL, "l1, l2 (4 bytes) or out (8 bytes) misaligned");
    hipError_t e = couple::launch_threej_family(ctx, rot, flip, fa, fb, n_pairs, l1, l2, out, stride,
                                                static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "threej_rows_m launch");
    return COUPLE_OK;
}

}  // extern "C"
