"""The C-ABI library loads and exports every entry point include/pes.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "pes.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pes_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for required in ("pes_create", "pes_destroy", "pes_set_data", "pes_loglike", "pes_response"):
        assert required in syms


def test_library_exports_every_declared_symbol():
    so = os.path.join(ROOT, "paper_2602_12011_amd", "libpes.so")
    assert os.path.exists(so), "libpes.so not built (run __graft_entry__.build())"
    lib = ctypes.CDLL(so)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_strerror_without_gpu():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2602_12011_amd", "libpes.so"))
    lib.pes_strerror.restype = ctypes.c_char_p
    assert lib.pes_strerror(0) == b"ok"
    assert lib.pes_strerror(-1) == b"invalid argument"
    # a null config is rejected before any device work
    assert lib.pes_create(None, None) == -1


def test_argument_checks_without_gpu():
    """Entry points reject a null context or an unknown mode before any device
    work (PES_EINVAL = -1)."""
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2602_12011_amd", "libpes.so"))
    v = ctypes.c_void_p
    lib.pes_set_schedule.argtypes = [v, ctypes.c_int]
    lib.pes_set_grad_method.argtypes = [v, ctypes.c_int]
    lib.pes_set_tuning.argtypes = [v, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.pes_noise.argtypes = [v, ctypes.c_uint64, v, v]
    lib.pes_probe.argtypes = [v, v, ctypes.c_int64, ctypes.c_int, v, v]
    lib.pes_loglike.argtypes = [v, v, ctypes.c_int64, v, v]
    lib.pes_fisher.argtypes = [v, v, ctypes.c_int64, v, v]
    assert lib.pes_set_schedule(None, 0) == -1
    assert lib.pes_set_grad_method(None, 0) == -1
    assert lib.pes_set_tuning(None, 1, 16, 0) == -1
    assert lib.pes_noise(None, 1, None, None) == -1
    assert lib.pes_probe(None, None, 1, 0, None, None) == -1
    assert lib.pes_loglike(None, None, 1, None, None) == -1
    assert lib.pes_fisher(None, None, 1, None, None) == -1
