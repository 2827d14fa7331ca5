"""The C ABI without a GPU: libnnef.so loads, exports every function that
include/nnef.h declares, and nnef_plan rejects malformed input with the
documented status before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nnef.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nnef_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2602_02759_amd import nnef
    if not os.path.exists(nnef.LIB_PATH):
        pytest.skip("libnnef.so is not built (run __graft_entry__.build())")
    return nnef.lib()


def test_header_declares_the_core_entry_points():
    names = declared_functions()
    for n in ("nnef_plan", "nnef_step", "nnef_loss", "nnef_loss_device", "nnef_plan_destroy",
              "nnef_last_error", "nnef_default_options"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_the_header():
    from paper_2602_02759_amd import nnef
    declared = set(declared_functions())
    assert set(nnef.EXPORTS) <= declared
    assert declared <= set(nnef.EXPORTS), sorted(declared - set(nnef.EXPORTS))


STATUS = {"OK": 0, "E_PARSE": 1, "E_SHAPE": 2, "E_LOSS_UNSUPPORTED": 3, "E_ARG": 4}


@pytest.mark.parametrize("model,sizes,ranks,ab,status", [
    ("ir,jr,kr", [4, 5, 6], [3], (1, 0), "E_PARSE"),          # no '->'
    ("ir,jr,kr->ijk", [4, 5, 6], [3], (1, 0), "OK"),
    ("ii,jr->ij", [4, 5], [3], (1, 0), "E_PARSE"),            # letter repeated in an operand
    ("ir,jr->ijj", [4, 5, 5], [3], (1, 0), "E_PARSE"),        # output letter repeated
    ("ir,jr->ijk", [4, 5, 6], [3], (1, 0), "E_PARSE"),        # output letter in no operand
    ("i1,jr->ij", [4, 5], [3], (1, 0), "E_PARSE"),            # not a letter
    ("ir,jr->ij", [4], [3], (1, 0), "E_SHAPE"),               # size count
    ("ir,jr->ij", [4, 0], [3], (1, 0), "E_SHAPE"),            # non-positive size
    ("ir,jr->ij", [4, 5], [0], (1, 0), "E_SHAPE"),            # non-positive rank
    ("ir,jr->ij", [4, 5], [3, 2], (1, 0), "E_SHAPE"),         # rank count
    ("ir,jr,kr->ijk", [1024, 1024, 1024], [3], (1, 0), "E_SHAPE"),  # 2^30 entries
    ("ir,jr->ij", [4, 5], [3], (0, 0.5), "E_LOSS_UNSUPPORTED"),      # alpha = 0, beta != 1
    ("ir,jr->ij", [4, 5], [3], (float("nan"), 1), "E_LOSS_UNSUPPORTED"),
])
def test_plan_validation(lib, model, sizes, ranks, ab, status):
    from paper_2602_02759_amd import nnef
    try:
        h = nnef.nnef_plan(model, sizes, ranks, ab[0], ab[1])
    except nnef.NnefError as e:
        if status == "OK":
            # a valid plan fails only at the device step when there is no GPU
            assert e.status not in (STATUS["E_PARSE"], STATUS["E_SHAPE"], STATUS["E_LOSS_UNSUPPORTED"])
        else:
            assert e.status == STATUS[status], (e.status, str(e))
            assert lib.nnef_last_error()  # a message is set
        return
    nnef.nnef_plan_destroy(h)
    assert status == "OK"


def test_null_arguments(lib):
    from paper_2602_02759_amd import nnef
    h = ctypes.c_void_p()
    st = lib.nnef_plan(None, None, 0, None, 0, 1.0, 0.0, None, ctypes.byref(h))
    assert st == STATUS["E_ARG"]
    assert lib.nnef_step(None, None, None, None, 1, None, None) == STATUS["E_ARG"]
    lib.nnef_plan_destroy(None)  # accepted, no effect
    # the binding's precision names follow the header's nnef_prec enum
    text = open(HEADER).read()
    body = re.search(r"typedef enum \{([^}]*)\} nnef_prec;", text).group(1)
    enum = {k.strip(): int(v) for k, v in re.findall(r"NNEF_(\w+)\s*=\s*(\d+)", body)}
    assert {k.lower(): v for k, v in enum.items()} == nnef.PREC
