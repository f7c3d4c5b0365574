"""The C ABI library loads on a machine without a GPU, exports every function declared in
include/*.h, and its argument checks (which run before any HIP call) behave as documented."""
import ctypes
import pathlib
import re

import pytest

ROOT = pathlib.Path(__file__).resolve().parent.parent


def declared_functions():
    names = []
    for h in sorted((ROOT / "include").glob("*.h")):
        text = re.sub(r"/\*.*?\*/", "", h.read_text(), flags=re.S)
        names += re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def B():
    import paper_2002_05265_amd.binding as B

    if not B.LIB_PATH.exists():
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    B.lib()
    return B


def test_every_declared_symbol_is_exported(B):
    names = declared_functions()
    assert "lbm_init" in names and "lbm_step" in names and "lbm_moments" in names
    L = ctypes.CDLL(str(B.LIB_PATH))
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(B.EXPORTS) <= set(names)


def test_population_bytes(B):
    # two copies x 9 planes, each plane rounded up to 256 bytes plus a 1 KiB skew
    assert B.lbm_population_bytes(64, 64, B.LBM_F64) == 2 * 9 * (64 * 64 * 8 + 1024)
    assert B.lbm_population_bytes(10, 3, B.LBM_F32_SHIFTED) == 2 * 9 * (64 * 4 + 1024)
    assert B.lbm_population_bytes(10, 3, B.LBM_F16_SHIFTED) == 2 * 9 * (128 * 2 + 1024)
    assert B.lbm_population_bytes(4096, 4096, B.LBM_F32_SHIFTED) == 2 * 9 * (4096 * 4096 * 4 + 1024)
    assert B.lbm_population_bytes(1, 64, B.LBM_F64) == 0
    assert B.lbm_population_bytes(64, 64, 7) == 0
    assert B.lbm_population_bytes(40000, 40000, B.LBM_F64) == 0


@pytest.mark.parametrize("args,code", [
    ((1, 8, 0, 4, 1.0), -1),     # nx < 2
    ((8, 8, 5, 4, 1.0), -1),     # unknown precision
    ((8, 8, 0, 5, 1.0), -1),     # eq_order not in {2,3,4}
    ((8, 8, 1, 4, 0.0), -1),     # shifted storage needs rho0 > 0
])
def test_init_argument_errors(B, args, code):
    with pytest.raises(B.LbmError) as e:
        B.lbm_init(*args, 0, 0, 0, 0, 0, 0)
    assert e.value.code == code
    assert B.lbm_last_error() != ""


def test_null_context_errors(B):
    with pytest.raises(B.LbmError) as e:
        B.lbm_step(0, B.LBM_BGK, [1.0] * 5, 1)
    assert e.value.code == -4
    with pytest.raises(B.LbmError):
        B.lbm_status(0)
    with pytest.raises(B.LbmError) as e:
        B.lbm_moments_noalloc(0, None, None, None, None)
    assert e.value.code == -4
    for call in (lambda: B.lbm_set_adjoint_depth(0, 2), lambda: B.lbm_get_adjoint_depth(0),
                 lambda: B.lbm_step3_raw_many(0, B.LBM_BGK, [1.0] * 5, [1], [2], 0)):
        with pytest.raises(B.LbmError) as e:
            call()
        assert e.value.code == -4
    B.lbm_destroy(0)  # NULL is accepted
