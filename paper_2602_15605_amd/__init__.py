"""MASTER mode-coupling matrices K^TT, K^TE, K^EE, K^BB on AMD MI355X (gfx950).

The computation lives in ``libcouple.so`` (HIP kernels behind the C ABI of
``include/couple.h``); ``couple`` is its Python binding and ``synth`` makes
seeded synthetic window spectra.
"""
from .couple import (BB, EE, TE, TT, CoupleError, Context, couple_band, couple_band_batched, couple_free,  # noqa: F401
                     couple_init, couple_last_error, couple_matrix, couple_matrix_batched, couple_profile,
                     couple_profile_read, couple_reserve_batched, couple_autotune_batched,
                     couple_set_batched_tiles, couple_get_batched_tiles,
                     couple_tables, load_library)
