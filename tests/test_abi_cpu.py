"""Host-side checks of the C-ABI library that need no GPU: every symbol the
header declares is exported, and argument validation that runs before any
device call returns the documented status codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "liftfft.h")


def _lib():
    from paper_0811_2535_amd import binding
    try:
        return binding.lib()
    except binding.LibraryNotBuilt:
        pytest.skip("libliftfft.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fft_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fft_plan_create", "fft_execute", "fft_plan_destroy", "fft_strerror"):
        assert required in names


def test_every_declared_symbol_is_exported():
    L = _lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_lists_match_header():
    from paper_0811_2535_amd import binding
    assert sorted(binding.EXPORTED) == declared_functions()


def test_abi_version():
    import re
    with open(HEADER) as f:
        declared = int(re.search(r"#define LIFTFFT_ABI_VERSION (\d+)", f.read()).group(1))
    assert _lib().fft_abi_version() == declared


def test_strerror_covers_codes():
    L = _lib()
    for code in range(-10, 1):
        s = L.fft_strerror(code)
        assert s and s != b"unknown status code", code
    assert L.fft_strerror(-1234) == b"unknown status code"


@pytest.mark.parametrize("n,batch,dtype,want", [
    (0, 1, 0, -1), (1, 1, 0, -1), (3, 1, 0, -1), (1000, 1, 0, -1), (-8, 1, 0, -1),
    (1024, 0, 0, -1), (1024, -5, 1, -1), (1024, 1, 2, -2), (1024, 1, -1, -2),
    (1 << 31, 1, 0, -8), (1 << 30, 1, 1, -8), (1 << 32, 1, 1, -8), (1 << 20, 1 << 60, 0, -1),
])
def test_create_validation(n, batch, dtype, want):
    L = _lib()
    h = ctypes.c_void_p(123)
    assert L.fft_plan_create(n, batch, dtype, ctypes.byref(h)) == want
    assert h.value is None  # *plan_out cleared on failure


def test_create_rejects_bad_options():
    from paper_0811_2535_amd.binding import PlanOpts
    L = _lib()
    h = ctypes.c_void_p()
    cases = [(PlanOpts(0, 3, 0), -9), (PlanOpts(0, 4, 0), -8), (PlanOpts(10, 0, 0), -9),
             (PlanOpts(-1, 0, 0), -9), (PlanOpts(0, 0, 3), -9), (PlanOpts(0, 32, 0), -9)]
    for opts, want in cases:
        assert L.fft_plan_create_ex(1024, 1, 0, ctypes.byref(opts), ctypes.byref(h)) == want
    bad = PlanOpts(0, 0, 0, 0, 0)
    bad.scratch_width = 3
    assert L.fft_plan_create_ex(1024, 1, 0, ctypes.byref(PlanOpts(0, 0, 0, 3, 0)),
                                ctypes.byref(h)) == -9
    # contradictory flags: split and full exchange; persistent and one tile
    assert L.fft_plan_create_ex(1024, 1, 0, ctypes.byref(PlanOpts(0, 0, 0, 0, 6)),
                                ctypes.byref(h)) == -9
    assert L.fft_plan_create_ex(1024, 1, 0, ctypes.byref(PlanOpts(0, 0, 0, 0, 24)),
                                ctypes.byref(h)) == -9
    assert L.fft_plan_create_ex(1024, 1, 0, ctypes.byref(PlanOpts(0, 0, 0, 0, 64)),
                                ctypes.byref(h)) == -9
    for vpt in (-16, 8, 64):
        assert L.fft_plan_create_ex(1024, 1, 0, ctypes.byref(PlanOpts(0, 0, 0, 0, 0, vpt)),
                                    ctypes.byref(h)) == -9
        assert L.fft_plan_create_ex(1024, 1, 0, ctypes.byref(PlanOpts(0, 0, 0, 0, 0, 0, vpt)),
                                    ctypes.byref(h)) == -9
    assert L.fft_plan_create_ex(1024, 1, 0, ctypes.byref(PlanOpts(0, 0, 0, 0, 0, 0, 0, -4)),
                                ctypes.byref(h)) == -9
    assert L.fft_plan_create_ex(1024, 1, 0, ctypes.byref(bad), ctypes.byref(h)) == -9
    assert L.fft_plan_create(1024, 1, 0, None) == -4


def test_null_plan_paths():
    L = _lib()
    assert L.fft_execute(None, None, None, -1, None) == -4
    assert L.fft_plan_destroy(None) == 0
    assert L.fft_plan_get_info(None, None) == -4
    assert L.fft_plan_set_timing(None, 1) == -4


def test_create_many_validation():
    """Argument checks of fft_plan_create_many (all host-side, before any
    device work)."""
    L = _lib()

    def arr(*v):
        return (ctypes.c_int64 * len(v))(*v)

    h = ctypes.c_void_p(123)
    assert L.fft_plan_create_many(None, 1, 0, 0, ctypes.byref(h)) == -4
    assert L.fft_plan_create_many(arr(8), 1, 0, 0, None) == -4
    assert L.fft_plan_create_many(arr(8), 0, 0, 0, ctypes.byref(h)) == -1
    assert h.value is None
    assert L.fft_plan_create_many(arr(8), 1, 7, 0, ctypes.byref(h)) == -2
    for bad in ((8, 12), (8, 1), (8, 0), (8, -16)):
        assert L.fft_plan_create_many(arr(*bad), 2, 0, 0, ctypes.byref(h)) == -1, bad
    assert L.fft_plan_create_many(arr(8, 1 << 25), 2, 0, 0, ctypes.byref(h)) == -8
    assert L.fft_plan_create_many(arr(8, 1 << 25), 2, 1, 0, ctypes.byref(h)) == -8
    assert L.fft_plan_create_many(arr(8, 1 << 29), 2, 0, 0, ctypes.byref(h)) == -8
    # the packed buffer must stay below 2^32 bytes (32-bit buffer descriptors)
    big = arr(*([1 << 24] * 32))
    assert L.fft_plan_create_many(big, 32, 0, 0, ctypes.byref(h)) == -8
    # flags: 0 or FFT_OPT_GRAPH; every other bit is refused before any device work
    for flags in (1, 2, 4, 16, 32, 128, 256, 512, 2048, 4096, 1 << 31, 0xFFFFFFFF, 64 | 1, 8 | 1024):
        assert L.fft_plan_create_many(arr(8, 16), 2, 0, flags, ctypes.byref(h)) == -9, flags
        assert h.value is None


def test_create_many_signature_matches_header():
    """The header declares fft_plan_create_many with a uint32_t flags word
    (the boundary's own signature), and the binding passes it as one."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    decl = re.search(r"int\s+fft_plan_create_many\(([^)]*)\)", text).group(1)
    params = [" ".join(p.split()) for p in decl.split(",")]
    assert params == ["const int64_t *lengths", "int64_t count", "int dtype", "uint32_t flags",
                      "fft_plan **plan_out"]
    execute = re.search(r"int\s+fft_execute\(([^)]*)\)", text).group(1)
    assert " ".join(execute.split(",")[0].split()) == "const fft_plan *plan"
    L = _lib()
    assert L.fft_plan_create_many.argtypes[3] is ctypes.c_uint32


def test_create_tuned_validation():
    from paper_0811_2535_amd.binding import TuneResult
    L = _lib()
    h = ctypes.c_void_p(123)
    res = TuneResult()
    assert L.fft_plan_create_tuned(1024, 1, 0, 0, None, ctypes.byref(res)) == -4
    assert L.fft_plan_create_tuned(1024, 1, 0, -1, ctypes.byref(h), ctypes.byref(res)) == -9
    assert h.value is None


def test_level_options_validation():
    """Two- and three-level flags: contradictory or two-level-only options
    with the three-level lift are refused before any device work."""
    from paper_0811_2535_amd.binding import FFT_OPT_THREE_LEVEL, FFT_OPT_TWO_LEVEL, PlanOpts
    L = _lib()
    h = ctypes.c_void_p(123)
    both = PlanOpts(0, 0, 0, 0, FFT_OPT_TWO_LEVEL | FFT_OPT_THREE_LEVEL)
    assert L.fft_plan_create_ex(1 << 24, 1, 0, ctypes.byref(both), ctypes.byref(h)) == -9
    assert h.value is None
    for opts in (PlanOpts(8, 0, 0, 0, FFT_OPT_THREE_LEVEL), PlanOpts(0, 0, 0, 4, FFT_OPT_THREE_LEVEL),
                 PlanOpts(0, 0, 0, 0, FFT_OPT_THREE_LEVEL, 0, 16), PlanOpts(0, 0, 0, 0, FFT_OPT_THREE_LEVEL, 0, 0, 4)):
        assert L.fft_plan_create_ex(1 << 24, 1, 0, ctypes.byref(opts), ctypes.byref(h)) == -9
    assert L.fft_plan_create_ex(1 << 24, 1, 0, ctypes.byref(PlanOpts(0, 0, 0, 0, 512)), ctypes.byref(h)) == -9


def test_info_struct_matches_header():
    """The binding's fft_plan_info mirrors the header's field list."""
    from paper_0811_2535_amd.binding import PlanInfo
    text = open(HEADER).read()
    body = text[text.index("typedef struct fft_plan_info {"):text.index("} fft_plan_info;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in re.findall(r"(?:int32_t|int64_t)\s+([^;]+);", body):
        names += [v.strip() for v in decl.split(",")]
    assert [f for f, _ in PlanInfo._fields_] == names



def test_create_paper_validation():
    """fft_plan_create_paper refuses invalid processor counts and breakpoints
    (Section 4.8: psize >= m, log2 m + 1 <= bp <= log2 psize + 1) before any
    device work."""
    L = _lib()
    h = ctypes.c_void_p(123)
    t = 12
    for lm, bp, want in ((-1, 1, -9), (7, 8, -9), (3, 3, -9), (3, 11, -9), (0, 0, -9), (0, 14, -9)):
        assert L.fft_plan_create_paper(1 << t, 1, 0, lm, bp, ctypes.byref(h)) == want, (lm, bp)
        assert h.value is None
    assert L.fft_plan_create_paper(1000, 1, 0, 1, 2, ctypes.byref(h)) == -1
    assert L.fft_plan_create_paper(1 << 12, 0, 0, 1, 2, ctypes.byref(h)) == -1
    assert L.fft_plan_create_paper(1 << 12, 1, 5, 1, 2, ctypes.byref(h)) == -2
    assert L.fft_plan_create_paper(1 << 21, 1, 0, 4, 6, ctypes.byref(h)) == -8
    assert L.fft_plan_create_paper(1 << 12, 1, 0, 1, 2, None) == -4


def test_opts_struct_matches_header():
    """The binding's fft_plan_opts mirrors the header's field list."""
    from paper_0811_2535_amd.binding import PlanOpts
    text = open(HEADER).read()
    body = text[text.index("typedef struct fft_plan_opts {"):text.index("} fft_plan_opts;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in re.findall(r"int32_t\s+([^;]+);", body):
        names += [v.strip() for v in decl.split(",")]
    assert [f for f, _ in PlanOpts._fields_] == names


def test_tile_order_validation():
    """tile_order without FFT_OPT_TILE_ORDER, bytes above 0x7f other than
    0x80, a fourth byte, and a spread with FFT_OPT_NO_XCD_REMAP are refused
    with FFT_E_ARG before any device work."""
    from paper_0811_2535_amd.binding import FFT_OPT_NO_XCD_REMAP, FFT_OPT_TILE_ORDER, PlanOpts
    L = _lib()
    h = ctypes.c_void_p(123)

    def create(flags, order, n=1 << 16):
        o = PlanOpts(0, 0, 0, 0, flags)
        o.tile_order = order
        return L.fft_plan_create_ex(n, 1, 0, ctypes.byref(o), ctypes.byref(h))

    assert create(0, 0x12) == -9
    for bad in (0x81, 0xff, 0x8100, 0x810000, 0x01000000):
        assert create(FFT_OPT_TILE_ORDER, bad) == -9, hex(bad)
    assert create(FFT_OPT_TILE_ORDER | FFT_OPT_NO_XCD_REMAP, 0x02) == -9
    assert create(FFT_OPT_TILE_ORDER | FFT_OPT_NO_XCD_REMAP, 0x0300) == -9
    assert h.value is None


def test_row_lane_option_validation():
    """FFT_OPT_ROW_LANES without FFT_OPT_TWO_LEVEL, or with another kernel
    variant, a slab width or another tile width, is refused with FFT_E_ARG
    before any device work."""
    from paper_0811_2535_amd.binding import (FFT_OPT_LDS_PREFETCH, FFT_OPT_PERSISTENT, FFT_OPT_ROW_LANES,
                                             FFT_OPT_SPLIT_EXCHANGE, FFT_OPT_TWO_LEVEL, PlanOpts)
    L = _lib()
    h = ctypes.c_void_p(123)
    TWO = FFT_OPT_TWO_LEVEL
    for opts in (PlanOpts(12, 0, 0, 0, FFT_OPT_ROW_LANES),
                 PlanOpts(12, 0, 0, 0, TWO | FFT_OPT_ROW_LANES | FFT_OPT_SPLIT_EXCHANGE),
                 PlanOpts(12, 0, 0, 0, TWO | FFT_OPT_ROW_LANES | FFT_OPT_PERSISTENT),
                 PlanOpts(12, 0, 0, 0, TWO | FFT_OPT_ROW_LANES | FFT_OPT_LDS_PREFETCH),
                 PlanOpts(12, 0, 4, 0, TWO | FFT_OPT_ROW_LANES),
                 PlanOpts(12, 0, 0, 0, TWO | FFT_OPT_ROW_LANES, 0, 0, 4)):
        assert L.fft_plan_create_ex(1 << 24, 1, 0, ctypes.byref(opts), ctypes.byref(h)) == -9
    assert h.value is None
