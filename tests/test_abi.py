"""The C-ABI library loads and exports every symbol include/dmpt.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "dmpt.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmpt_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    for s in ("dmpt_init", "dmpt_response", "dmpt_destroy", "dmpt_layer_products"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2203_09621_amd import _native
    lib = ctypes.CDLL(_native.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(_native.EXPORTS) == declared_symbols()


def test_status_strings_and_defaults_without_gpu():
    from paper_2203_09621_amd import _native
    assert _native.LIB.dmpt_status_str(-4).decode() == "DMPT_ENOCONV"
    o = _native.default_options()
    assert o.precision == _native.PRECISION["split_fp16"] and o.max_layers == 100
    # the last field, written by the library: the structure layouts agree
    assert o.graph == 1 and o.tile_threshold == -1


def test_struct_sizes_match_c_layout():
    from paper_2203_09621_amd import _native
    assert ctypes.sizeof(_native.DmptOptions) == 32
    assert ctypes.sizeof(_native.DmptProblemStats) == 8 * 4 + 8 * 4
    # 4+4+32+4+4+256 = 304, then 4 + 8 + 1 + 8 + 1 + 1 doubles, then 2 int32
    assert ctypes.sizeof(_native.DmptStats) == 304 + 8 * 23 + 8
