"""CPU-side checks of the native library: it builds, loads, and exports every
symbol include/vccl.h declares.  No compute call is made (no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vccl.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vccl[A-Z]\w*)\s*\(", text)))


def test_header_declares_the_paper_api():
    names = _declared()
    for must in ("vcclCommInitAll", "vcclCommDestroy", "vcclCommAbort", "vcclAllReduce", "vcclBroadcast",
                 "vcclReduce", "vcclAllGather", "vcclReduceScatter", "vcclGroupStart", "vcclGroupEnd"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2507_04786_amd as vccl
    lib = ctypes.CDLL(vccl.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(vccl.EXPORTED) == _declared()


def test_error_strings_and_version():
    import paper_2507_04786_amd as vccl
    assert vccl.vcclGetVersion() == 1
    for code in range(8):
        assert vccl.vcclGetErrorString(code)
    assert "invalid argument" in vccl.vcclGetErrorString(vccl.vcclInvalidArgument)


def test_group_end_without_start_is_invalid_usage():
    import paper_2507_04786_amd as vccl
    try:
        vccl.vcclGroupEnd()
    except vccl.VcclError as e:
        assert e.code == vccl.vcclInvalidUsage
    else:
        raise AssertionError("expected vcclInvalidUsage")
    vccl.vcclGroupStart()
    vccl.vcclGroupEnd()  # an empty group is fine


def test_init_rejects_bad_rank_counts():
    import paper_2507_04786_amd as vccl
    for n in (0, 1, 17):
        try:
            vccl.vcclCommInitAll(n)
        except vccl.VcclError as e:
            assert e.code in (vccl.vcclInvalidArgument, vccl.vcclUnhandledHipError)
        else:
            raise AssertionError("expected an error")


def test_c_client_builds_against_the_header(tmp_path):
    """include/vccl.h is plain C: a C11 program using the collectives, groups
    and error strings compiles without warnings and links against the
    library (it runs in the GPU tests)."""
    import pytest
    from tests import c_client_build as cb
    why = cb.available()
    if why:
        pytest.skip(why)
    out = tmp_path / "c_client"
    cb.build(str(out))
    assert out.exists() and os.access(str(out), os.X_OK)


def test_init_rejects_bad_ring_orders():
    """Ring orders are checked before the device is touched: every row must
    be a permutation of the ranks, and there are 1..VCCL_MAX_RINGS rows."""
    import ctypes as C
    import paper_2507_04786_amd as vccl
    lib = vccl.lib()
    arr = (C.c_void_p * 4)()
    for rows in ([[0, 1, 1, 3]], [[0, 1, 2, 4]], [[0, 1, 2, -1]], [[0, 1, 2, 3]] * 5):
        flat = [r for row in rows for r in row]
        res = lib.vcclCommInitAllRings(arr, 4, None, len(rows), (C.c_int * len(flat))(*flat))
        assert res == vccl.vcclInvalidArgument, rows
    flat = (C.c_int * 4)(0, 1, 2, 3)
    assert lib.vcclCommInitAllRings(arr, 4, None, 0, flat) == vccl.vcclInvalidArgument
    try:
        vccl.vcclCommInitAll(4, rings=[[0, 1, 2]])
    except ValueError:
        pass
    else:
        raise AssertionError("expected a ValueError for a short ring")
