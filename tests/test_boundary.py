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


def test_batched_layout_validation():
    """The binding sizes and checks the batched layout on the host, before
    anything reaches the C ABI: Z entries follow the z offsets, bad offsets
    and overlapping Z blocks are refused."""
    from paper_1401_4950_amd import batched_layout
    noff, zoff, rows, ztot = batched_layout([0, 3, 5, 5, 9])
    assert noff == [0, 3, 5, 5, 9] and zoff is None and rows == 9 and ztot == 9 + 4 + 0 + 16
    # a spread layout needs max(z_b + n_b^2) entries, not sum n_b^2
    _, zoff, _, ztot = batched_layout([0, 3, 5], z_offsets=[100, 0])
    assert zoff == [100, 0] and ztot == 109
    _, _, _, ztot = batched_layout([0, 2, 2, 4], z_offsets=[0, 3, 4])   # empty matrix: any offset
    assert ztot == 8
    for bad in ([1, 3], [0, 3, 2], []):
        with pytest.raises(ValueError):
            batched_layout(bad)
    with pytest.raises(ValueError):
        batched_layout([0, 3, 5], z_offsets=[-1, 10])
    with pytest.raises(ValueError):
        batched_layout([0, 3, 5], z_offsets=[0, 8])          # 3x3 block ends at 9
    with pytest.raises(ValueError):
        batched_layout([0, 3, 5], z_offsets=[0])             # one offset per matrix


def test_negative_z_offsets_refused_by_the_c_abi(lib):
    """The library itself refuses negative Z offsets (argument 6) before any
    device work, so a caller of the C ABI cannot make it write below Z."""
    from paper_1401_4950_amd import _lib
    noff = (ctypes.c_int64 * 3)(0, 3, 5)
    zoff = (ctypes.c_int64 * 2)(0, -9)
    o = _lib.default_options()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    h = ctypes.c_void_p(0x1000)
    assert lib.mrrr_dstemr_batched(h, 2, noff, fake, fake, zoff, ctypes.byref(o), fake, fake, None) == -6
    assert lib.mrrr_dstemr_backward_batched(h, 2, noff, fake, fake, zoff, None, None, 1e-8, fake, fake,
                                            None) == -6


def _header_fields(struct_name):
    hdr = open(os.path.join(ROOT, "include", "mrrr.h")).read()
    head = hdr[: re.search(r"\}\s*" + struct_name + r";", hdr).start()]
    body = head[head.rindex("typedef struct {") + len("typedef struct {"):]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    return re.findall(r"\b(?:int32_t|int64_t|uint64_t|double|void\s*\*|const int32_t\s*\*)\s*\**\s*(\w+)\s*;",
                      body)


@pytest.mark.parametrize("struct,mirror", [("mrrr_stats_t", "Stats"), ("mrrr_options_t", "Options")])
def test_ctypes_mirrors_follow_the_header(struct, mirror):
    """The binding's ctypes structures list the header's fields in order."""
    from paper_1401_4950_amd import _lib
    assert _header_fields(struct) == [f for f, _ in getattr(_lib, mirror)._fields_]
