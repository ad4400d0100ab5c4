"""C-ABI checks that need no GPU: the library loads, exports every function
include/dfhip.h declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dfhip.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:df_status|const char \*|int64_t)\s*(df_\w+)\s*\(", text, flags=re.M))


def test_library_exports_every_declared_symbol():
    from paper_1611_03226_amd import dfhip as D
    names = _declared()
    assert len(names) >= 18
    lib = C.CDLL(D.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert names == set(D.EXPORTED)          # the binding covers exactly the header


def test_version_and_error_string():
    from paper_1611_03226_amd import dfhip as D
    assert D.df_version().startswith("dfhip")
    assert isinstance(D.df_last_error(None), str)


def _have_gpu():
    import torch
    return torch.cuda.is_available()


@pytest.mark.skipif(_have_gpu(), reason="checks the no-device error path")
def test_graph_create_without_device_reports_edevice():
    from paper_1611_03226_amd import dfhip as D
    with pytest.raises(D.DFError) as e:
        D.df_graph_create(0)
    assert e.value.code == D.DF_EDEVICE


def test_null_graph_is_rejected():
    from paper_1611_03226_amd import dfhip as D
    lib = D._lib
    n = C.c_int64()
    assert lib.df_fire(None, 0, 1, 0, C.byref(n)) == D.DF_EINVAL
    assert lib.df_push(None, 0, None, 1, 0) == D.DF_EINVAL
    assert lib.df_sync(None) == D.DF_EINVAL
    assert lib.df_graph_create(None, 0, None) == D.DF_EINVAL


@pytest.mark.parametrize("args,ok", [
    ((1, 100, 7, 4, 4, 0), False),      # len not a multiple of r
    ((1, 64, 8, 17, 4, 0), False),      # too many branches
    ((1, 64, 8, 4, 33, 0), False),      # too many taps
    ((1, 64, 4, 4, 8, 0), False),       # r < M - 1
    ((1, 64, 8, 4, 4, 2), False),       # bad history mode
    ((0, 64, 8, 4, 4, 0), True),        # empty: nothing to do
])
def test_stateless_argument_validation(args, ok):
    from paper_1611_03226_amd import dfhip as D
    st = D._lib.df_dpd_forward(None, None, None, None, None, *args)
    assert (st == D.DF_OK) if ok else (st == D.DF_EINVAL)


def test_stateless_null_pointers_and_work_size():
    from paper_1611_03226_amd import dfhip as D
    lib = D._lib
    assert lib.df_dpd_forward(None, None, None, None, None, 2, 64, 8, 4, 4, 0) == D.DF_EINVAL
    assert lib.df_mp_input_adjoint(None, None, None, None, None, 2, 64, 4, 4) == D.DF_EINVAL
    assert lib.df_mp_input_adjoint(None, None, None, None, None, 2, 64, 0, 4) == D.DF_EINVAL
    # work: one fp32 complex partial per (workgroup, branch, tap); a workgroup
    # takes 4096 outputs of a firing
    wb = D.df_dpd_coeff_adjoint_work_bytes(64, 65536, 65536, 10, 16)
    assert wb == 64 * 16 * 10 * 16 * 8
    wb2 = D.df_dpd_coeff_adjoint_work_bytes(2, 4096, 256, 4, 8)
    assert wb2 == 2 * 16 * 1 * 4 * 8 * 8
    assert lib.df_dpd_coeff_adjoint(None, None, None, None, None, 2, 4096, 256, 4, 8, 0, None, 0) == D.DF_EINVAL


def test_stream_copy_validation():
    from paper_1611_03226_amd import dfhip as D
    lib = D._lib
    assert lib.df_stream_copy(None, None, None, 0) == D.DF_OK          # nothing to copy
    assert lib.df_stream_copy(None, None, None, 24) == D.DF_EINVAL     # not a multiple of 16
    assert lib.df_stream_copy(None, None, None, -16) == D.DF_EINVAL
    assert lib.df_stream_copy(None, None, None, 32) == D.DF_EINVAL     # null pointers


def test_paper_channel_bytes_matches_eq1():
    """The library's Eq. (1) helper (host arithmetic) against the oracle's,
    and the motion network's total against Table 1 (3.46 MB)."""
    from oracle import fifo_layout as fl
    from paper_1611_03226_amd import dfhip as D
    for s, r, d in [(1, 1, False), (8, 4096, False), (76800, 4, True), (4, 32768, True), (3, 7, True)]:
        assert D.df_paper_channel_bytes(s, r, d) == fl.capacity_bytes(s, r, d)
    total = sum(D.df_paper_channel_bytes(s, r, d) for s, r, d in fl.paper_motion_channels(320, 240, 4))
    assert round(total / 1e6, 2) == 3.46
    assert D.df_paper_channel_bytes(0, 4, False) == -1 and D.df_paper_channel_bytes(8, 0, True) == -1


# ---------------------------------------------------------------- binding checks
# The binding checks every buffer against the channel's token type before it
# hands a pointer to the library (no device needed for these).

def test_host_source_dtype_and_size_checks():
    from paper_1611_03226_amd import dfhip as D
    # int64 control tokens that fit are converted, not reinterpreted
    a, n = D.host_tokens(np.array([1, 2, 3], np.int64), D.DF_I32, 1)
    assert a.dtype == np.int32 and list(a) == [1, 2, 3] and n == 3
    a, n = D.host_tokens([4, 5], D.DF_I32, 1)
    assert a.dtype == np.int32 and n == 2
    with pytest.raises(ValueError):
        D.host_tokens(np.array([1 << 40], np.int64), D.DF_I32, 1)      # does not fit int32
    with pytest.raises(ValueError):
        D.host_tokens(np.zeros(8, np.float32), D.DF_C64, 1)             # float pairs are not complex64
    with pytest.raises(ValueError):
        D.host_tokens(np.zeros(4, np.complex64), D.DF_C64, 1, 5)        # fewer tokens than claimed
    with pytest.raises(ValueError):
        D.host_tokens(np.zeros(10, np.uint8), D.DF_U8, 4)               # not whole 4-byte tokens
    a, n = D.host_tokens(np.zeros((3, 2, 2), np.uint8), D.DF_U8, 4)    # frames: tokens = frames
    assert n == 3
    a, n = D.host_tokens(np.zeros(4, np.complex128), D.DF_C64, 1)
    assert a.dtype == np.complex64 and n == 4


def test_host_destination_checks():
    from paper_1611_03226_amd import dfhip as D
    assert D.host_dest(np.zeros((5, 4, 4), np.uint8), D.DF_U8, 16) == 5
    assert D.host_dest(np.zeros(80, np.uint8), D.DF_U8, 16) == 5       # flat buffer: whole frames only
    with pytest.raises(ValueError):
        D.host_dest(np.zeros(80, np.uint8), D.DF_U8, 16, 6)            # no room for 6 frames
    with pytest.raises(ValueError):
        D.host_dest(np.zeros(8, np.float32), D.DF_C64, 1)
    with pytest.raises(ValueError):
        D.host_dest(np.zeros(8, np.complex64)[::2], D.DF_C64, 1)       # not contiguous
    ro = np.zeros(4, np.complex64)
    ro.setflags(write=False)
    with pytest.raises(ValueError):
        D.host_dest(ro, D.DF_C64, 1)


def test_tensor_buffer_checks():
    import torch
    from paper_1611_03226_amd import dfhip as D
    assert D.device_tokens(torch.zeros(6, dtype=torch.complex64), D.DF_C64, 1) == 6
    assert D.device_tokens(torch.zeros(6, dtype=torch.complex64), D.DF_C64, 1, 4) == 4
    with pytest.raises(ValueError):
        D.device_tokens(torch.zeros(12, dtype=torch.float32), D.DF_C64, 1)
    with pytest.raises(ValueError):
        D.device_tokens(torch.zeros(6, dtype=torch.complex64), D.DF_C64, 1, 7)
    x = torch.zeros(2, 64, dtype=torch.complex64)
    h = torch.zeros(3, 4, dtype=torch.complex64)
    D.check_dpd_tensors(x, torch.zeros(2, 8, dtype=torch.int32), h, x.clone(), 8)
    for bad in (dict(ctrl=torch.zeros(2, 8, dtype=torch.int64)),          # ctrl dtype
                dict(ctrl=torch.zeros(2, 7, dtype=torch.int32)),          # ctrl shape
                dict(y=torch.zeros(2, 32, dtype=torch.complex64)),        # y shape
                dict(h=torch.zeros(3, 4, dtype=torch.float32)),           # h dtype
                dict(r=7)):                                               # L % r
        kw = dict(x=x, ctrl=torch.zeros(2, 8, dtype=torch.int32), h=h, y=x.clone(), r=8)
        kw.update(bad)
        with pytest.raises(ValueError):
            D.check_dpd_tensors(**kw)


def test_status_codes_match_header():
    from paper_1611_03226_amd import dfhip as D
    text = open(HEADER).read()
    for name, code in (("DF_ECONTROL", D.DF_ECONTROL), ("DF_EINDEX", D.DF_EINDEX)):
        assert re.search(rf"{name}\s*=\s*{code}\b", text), name
