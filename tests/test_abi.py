"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2107_05681_amd as meld
    if not os.path.exists(meld.LIB_PATH):
        from paper_2107_05681_amd import build
        build.build()
    return meld, meld.load_library()


def _declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(meld_\w+)\s*\(", text))
    return names


def test_exports_every_declared_function():
    meld, lib = _lib()
    declared = _declared_functions()
    assert declared, "no declarations found"
    assert declared == set(meld.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_version():
    _, lib = _lib()
    assert lib.meld_version() >= 100


def test_null_context_is_rejected_without_gpu_work():
    meld, lib = _lib()
    assert lib.meld_sort_u32(None, None, None, 10, 1, None) == meld.EINVAL
    assert b"ctx is NULL" in lib.meld_last_error()
    s = meld.side(1, 0, 1, 1)
    assert lib.meld_divergent_region_f32(None, None, None, 10, None, 16, 0, 0, s, s, 1,
                                         None) == meld.EINVAL
    assert lib.meld_segmented_sort_u32(None, None, None, 3, 1, None) == meld.EINVAL
    assert lib.meld_sort_u32_steps(None, None, None, 8, 3, 1, None) == meld.EINVAL
    assert lib.meld_create(0, None) == meld.EINVAL
    lib.meld_destroy(None)


def test_python_binding_rejects_non_cuda_tensors():
    torch = pytest.importorskip("torch")
    meld, _ = _lib()
    with pytest.raises(TypeError):
        meld.sort(torch.zeros(4, dtype=torch.int32))
    with pytest.raises(TypeError):
        meld.divergent_region(torch.zeros(4), torch.ones(4), 0, 0, meld.side(1, 0, 1, 1),
                              meld.side(1, 0, 1, 1))
    with pytest.raises(ValueError):
        meld._variant("fastest")
