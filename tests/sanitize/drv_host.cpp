// Host argument paths of libcouple (every entry point with bad arguments, the
// device byte cap, couple_init without a device) under AddressSanitizer and
// UndefinedBehaviorSanitizer: no GPU is needed or used.
#include <cstdio>
#include <cstdlib>
#include "couple.h"
int main() {
    int bad = 0;
    couple_ctx* h = nullptr;
    auto expect = [&](int got, int want, const char* what) {
        if (got != want) { std::printf("%s: got %d want %d\n", what, got, want); bad = 1; }
    };
    expect(couple_init(-1, &h), COUPLE_EINVAL, "init lmax<0");
    expect(couple_init(COUPLE_LMAX_LIMIT + 1, &h), COUPLE_EINVAL, "init lmax>limit");
    expect(couple_init(10, nullptr), COUPLE_EINVAL, "init NULL");
    setenv("COUPLE_MAX_DEVICE_BYTES", "4096", 1);
    expect(couple_init(500, &h), COUPLE_ENOMEM, "init above cap");
    setenv("COUPLE_MAX_DEVICE_BYTES", "12x", 1);      // not a number: no cap
    unsetenv("COUPLE_MAX_DEVICE_BYTES");
    int rc = couple_init(8, &h);                      // no GPU here: EDEVICE
    if (rc == COUPLE_OK) couple_free(h); else expect(rc, COUPLE_EDEVICE, "init without device");
    std::printf("last error: %s\n", couple_last_error(nullptr));
    expect(couple_matrix(nullptr, nullptr, nullptr, nullptr, 0, 0, 1, 0, nullptr, nullptr), COUPLE_EINVAL, "matrix");
    expect(couple_band(nullptr, 0, 1, nullptr, nullptr, nullptr, 0, 0, 1, 0, nullptr, 0, nullptr, nullptr),
           COUPLE_EINVAL, "band");
    expect(couple_band_batched(nullptr, 1, 0, 1, nullptr, nullptr, nullptr, 0, 0, 1, 0, nullptr, 0, nullptr, nullptr),
           COUPLE_EINVAL, "band_batched");
    int lm[2] = {10, 20};
    expect(couple_reserve_batched(nullptr, 2, lm), COUPLE_EINVAL, "reserve");
    expect(couple_matrix_batched(nullptr, 2, lm, nullptr, nullptr, nullptr, nullptr, 15, COUPLE_MFMA_FP32, nullptr,
                                 nullptr), COUPLE_EINVAL, "matrix_batched");
    expect(couple_set_batched_tiles(nullptr, COUPLE_MFMA_FP32, 2, 8), COUPLE_EINVAL, "set_tiles");
    int rt = 0, fl = 0;
    expect(couple_get_batched_tiles(nullptr, COUPLE_MFMA_FP32, &rt, &fl), COUPLE_EINVAL, "get_tiles");
    expect(couple_autotune_batched(nullptr, COUPLE_MFMA_FP32, 2, lm, nullptr, nullptr, nullptr, nullptr, 15, nullptr,
                                   nullptr, nullptr, nullptr, nullptr), COUPLE_EINVAL, "autotune");
    expect(couple_profile(nullptr, 1), COUPLE_EINVAL, "profile");
    expect(couple_profile_read(nullptr, nullptr, nullptr), COUPLE_EINVAL, "profile_read");
    expect(couple_bin_spectra(nullptr, 1, nullptr, 0, nullptr, 1, nullptr, nullptr), COUPLE_EINVAL, "bin_spectra");
    expect(couple_master_solve(nullptr, 0, 1, nullptr, 1, nullptr, nullptr, nullptr, nullptr), COUPLE_EINVAL, "solve");
    expect(couple_master_solve_noalloc(nullptr, 0, 1, nullptr, 1, nullptr, nullptr, nullptr), COUPLE_EINVAL,
           "solve_noalloc");
    expect(couple_threej_rows(nullptr, 0, 1, nullptr, nullptr, nullptr, 1, nullptr), COUPLE_EINVAL, "threej");
    expect(couple_tables(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr), COUPLE_EINVAL, "tables");
    expect(couple_lmax_max(nullptr), -1, "lmax_max");
    couple_free(nullptr);
    std::printf("host driver %s\n", bad ? "FAILED" : "ok");
    return bad;
}
