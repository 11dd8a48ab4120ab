"""The C ABI on the CPU: the library loads, exports every entry point that
include/couple.h declares, rejects bad arguments that need no device, and
neither links nor names the oracle.  No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "couple.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(couple_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2602_15605_amd import couple
    if not os.path.exists(couple.LIB_PATH):
        from paper_2602_15605_amd import build
        build.build()
    return couple.load_library()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("couple_init", "couple_matrix", "couple_band", "couple_free", "couple_last_error",
              "couple_tables", "couple_lmax_max"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2602_15605_amd import couple
    out = subprocess.run(["nm", "-D", "--defined-only", couple.LIB_PATH], check=True,
                         capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for name in _declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_library_does_not_touch_the_oracle():
    from paper_2602_15605_amd import couple
    syms = subprocess.run(["nm", "-D", couple.LIB_PATH], check=True, capture_output=True, text=True).stdout
    assert "oracle" not in syms
    deps = subprocess.run(["readelf", "-d", couple.LIB_PATH], check=True, capture_output=True, text=True).stdout
    assert "oracle" not in deps
    for fn in os.listdir(os.path.join(ROOT, "paper_2602_15605_amd")):
        if fn.endswith(".py"):
            src = open(os.path.join(ROOT, "paper_2602_15605_amd", fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn


def test_host_side_argument_errors(lib):
    h = ctypes.c_void_p()
    assert lib.couple_init(-1, ctypes.byref(h)) == -1
    assert "lmax_max" in lib.couple_last_error(None).decode()
    assert lib.couple_init(16385, ctypes.byref(h)) == -1
    assert lib.couple_init(10, None) == -1
    assert lib.couple_matrix(None, None, None, None, 0, 0, 1, 0, None, None) == -1
    assert lib.couple_band(None, 0, 1, None, None, None, 0, 0, 1, 0, None, 0, None, None) == -1
    assert lib.couple_tables(None, None, None, None, None, None) == -1
    assert lib.couple_lmax_max(None) == -1
    assert lib.couple_bin_spectra(None, 1, None, 0, None, 1, None, None) == -1
    assert lib.couple_master_solve(None, 0, 1, None, 1, None, None, None, None) == -1
    assert lib.couple_master_solve_noalloc(None, 0, 1, None, 1, None, None, None) == -1
    lib.couple_free(None)


def test_binding_fails_loudly_without_the_library(tmp_path):
    from paper_2602_15605_amd import couple
    saved = couple._lib
    try:
        couple._lib = None
        with pytest.raises(couple.CoupleError):
            couple.load_library(str(tmp_path / "missing.so"))
    finally:
        couple._lib = saved


def test_enum_values_match_the_binding():
    """Spectrum bits, the output-form flag and precisions are the same numbers
    in the header and in the Python binding."""
    from paper_2602_15605_amd import couple
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    vals = {k: int(v) for k, v in re.findall(r"\b(COUPLE_[A-Z0-9_]+)\s*=\s*(-?\d+)", text)}
    for name, bit in couple.SPECTRUM_BITS.items():
        assert vals["COUPLE_" + name] == bit
    assert vals["COUPLE_XI"] == couple.XI
    assert couple.XI & 0x1F == 0
    assert vals["COUPLE_FP64"] == couple.PRECISIONS["fp64"]
    assert vals["COUPLE_FP32C"] == couple.PRECISIONS["fp32c"]
    assert vals["COUPLE_MFMA_FP32"] == couple.PRECISIONS["mfma_fp32"]
    assert vals["COUPLE_MFMA_BF16X3"] == couple.PRECISIONS["mfma_bf16x3"]
    m = re.search(r"#define\s+COUPLE_NOALLOC_SOLVE_DOUBLES\s+\(1LL << (\d+)\)", open(HEADER).read())
    assert m and (1 << int(m.group(1))) == couple.NOALLOC_SOLVE_DOUBLES


def test_device_byte_cap_gives_enomem(lib, monkeypatch):
    """COUPLE_MAX_DEVICE_BYTES is checked on the host before any device call,
    so a context above it is refused with ENOMEM (also on a machine without a
    GPU)."""
    from paper_2602_15605_amd import couple
    monkeypatch.setenv("COUPLE_MAX_DEVICE_BYTES", "1000000")
    h = ctypes.c_void_p()
    assert lib.couple_init(2000, ctypes.byref(h)) == couple.COUPLE_ENOMEM
    assert not h.value
    msg = lib.couple_last_error(None).decode()
    assert "COUPLE_MAX_DEVICE_BYTES" in msg and "lmax_max=2000" in msg


def test_no_device_gives_edevice(lib, monkeypatch):
    """Without a usable GPU, couple_init fails with EDEVICE and a message (the
    device error path); on a GPU machine the context is simply released."""
    from paper_2602_15605_amd import couple
    monkeypatch.delenv("COUPLE_MAX_DEVICE_BYTES", raising=False)
    h = ctypes.c_void_p()
    rc = lib.couple_init(8, ctypes.byref(h))
    if rc == couple.COUPLE_OK:
        lib.couple_free(h)
        pytest.skip("a GPU is visible here")
    assert rc == couple.COUPLE_EDEVICE
    assert not h.value
    assert lib.couple_last_error(None).decode()
