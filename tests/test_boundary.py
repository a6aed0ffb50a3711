"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol include/mrrr.h declares, and rejects bad arguments before launching."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1401_4950_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1401_4950_amd import _build
        _build.build()
    return _lib.load()


def test_exports_match_header(lib):
    from paper_1401_4950_amd import _lib
    hdr = open(os.path.join(ROOT, "include", "mrrr.h")).read()
    declared = set(re.findall(r"\b(mrrr_[a-z_]+)\s*\(", hdr))
    assert declared == set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_defaults_and_status_strings(lib):
    from paper_1401_4950_amd import _lib
    o = _lib.default_options()
    assert o.jobz == 1 and o.sign_convention == 1
    assert o.gaptol == 1e-3 and o.rtol_class == 1e-5
    assert o.perturb_xi == 8.0 and o.max_rqi == 10 and o.max_shift_tries == 16
    assert o.lanes_per_eig == 64 and o.bundle == 64 and not o.tune
    assert o.check_tol == 20.0   # the last field: the ctypes mirror has the header's layout
    for code in range(0, 8):
        assert lib.mrrr_status_string(code)
    assert b"invalid" in lib.mrrr_status_string(-3)


def test_argument_validation_without_gpu(lib):
    from paper_1401_4950_amd import _lib
    o = _lib.default_options()
    m = ctypes.c_int64(-1)
    # null handle is argument 1
    assert lib.mrrr_dstemr(None, 10, None, None, 0, 0.0, 0.0, 0, 0, ctypes.byref(o), ctypes.byref(m),
                           None, None, 10, None) == -1
    assert lib.mrrr_dstemr_batched(None, 1, None, None, None, None, None, None, None, None) == -1
    assert lib.mrrr_dstemr_backward(None, 3, None, None, 3, None, None, 3, 1e-8, None, None, None) == -1
    assert lib.mrrr_dstemr_backward_batched(None, 1, None, None, None, None, None, None, 1e-8, None, None,
                                            None) == -1
    assert lib.mrrr_create(None, 0) == -1
    assert lib.mrrr_destroy(None) == -1
    assert lib.mrrr_set_stream(None, None) == -1


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    h = ctypes.c_void_p()
    code = lib.mrrr_create(ctypes.byref(h), 0)
    assert code != 0


def test_package_has_no_cpu_path():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_1401_4950_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
