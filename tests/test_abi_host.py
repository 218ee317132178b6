"""Host-only checks of the C ABI (no GPU): the library loads, exports every
symbol include/rsvd.h declares, and validates problems before any launch."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsvd.h")


@pytest.fixture(scope="module")
def lib():
    from paper_0909_4061_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:rsvd_status|size_t|const char\*)\s+(rsvd_\w+)\s*\(", text, re.M)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ("rsvd_range_finder", "rsvd_power_iter", "rsvd_project", "rsvd_svd"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_0909_4061_amd import _lib
    names = declared_functions()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(lib, n), f"{n} not exported"
    assert sorted(_lib.EXPORTS) == names


def _prob(**kw):
    from paper_0909_4061_amd import problem
    import torch
    base = dict(m=2000, n=1000, k=20, p=10, q=0, dtype=torch.float64)
    base.update(kw)
    m, n, k, p, q = (base.pop(x) for x in ("m", "n", "k", "p", "q"))
    return problem(m, n, k, p, q, **base)


@pytest.mark.parametrize("kw,expect", [
    ({}, 0),
    ({"k": 0}, 1),
    ({"p": -1}, 1),
    ({"q": -1}, 1),
    ({"k": 995, "p": 10}, 1),            # l > min(m, n)
    ({"m": 0}, 1),
    ({"lda": 999}, 1),                    # lda < n
    ({"k": 120, "p": 9}, 4),              # l = 129 > RSVD_MAX_L
    ({"prec": "bf16x3"}, 4),              # BF16 arithmetic needs FP32 data
    ({"k": 128, "p": 0}, 0),
    ({"k": 1, "p": 0}, 0),
    # SRFT: q = 0, n a power of two in [8, 16384] (FP32) / [8, 8192] (FP64)
    ({"n": 1024, "sketch": "srft"}, 0),
    ({"n": 1024, "sketch": "srft", "q": 1}, 4),
    ({"n": 1000, "sketch": "srft"}, 4),
    ({"n": 8192, "sketch": "srft"}, 0),
    ({"m": 20000, "n": 16384, "sketch": "srft"}, 4),
    ({"m": 20000, "n": 16384, "sketch": "srft", "dtype": "f32"}, 0),
    ({"m": 40000, "n": 32768, "sketch": "srft", "dtype": "f32"}, 4),
    ({"m": 8, "n": 8, "k": 4, "p": 4, "sketch": "srft"}, 0),
    ({"m": 8, "n": 4, "k": 2, "p": 2, "sketch": "srft"}, 4),
    # Givens-chain sketch: the SRFT's constraints
    ({"n": 1024, "sketch": "gsrft"}, 0),
    ({"n": 1024, "sketch": "gsrft", "q": 1}, 4),
    ({"n": 1000, "sketch": "gsrft"}, 4),
    ({"n": 8192, "sketch": "gsrft"}, 0),
    ({"m": 20000, "n": 16384, "sketch": "gsrft"}, 4),
    ({"m": 20000, "n": 16384, "sketch": "gsrft", "dtype": "f32"}, 0),
    ({"m": 8, "n": 8, "k": 4, "p": 4, "sketch": "gsrft"}, 0),
])
def test_validate(lib, kw, expect):
    import torch
    kw = dict(kw)
    if kw.get("dtype") == "f32":
        kw["dtype"] = torch.float32
    pr = _prob(**kw)
    assert lib.rsvd_validate(ctypes.byref(pr)) == expect
    ws = lib.rsvd_workspace_bytes(ctypes.byref(pr))
    assert (ws > 0) == (expect == 0)


def test_bad_enum_is_invalid(lib):
    pr = _prob()
    pr.dtype = 7
    assert lib.rsvd_validate(ctypes.byref(pr)) == 1
    assert lib.rsvd_validate(None) == 1


def test_workspace_grows_with_m(lib):
    small = lib.rsvd_workspace_bytes(ctypes.byref(_prob(m=2000)))
    big = lib.rsvd_workspace_bytes(ctypes.byref(_prob(m=20000)))
    assert big > small > 0


def test_status_strings(lib):
    for s in range(8):
        assert lib.rsvd_status_string(s)
    assert b"unknown" in lib.rsvd_status_string(99)


def test_null_arguments_fail_before_launch(lib):
    pr = _prob()
    # no handle: rejected on the host, nothing touches a device
    assert lib.rsvd_range_finder(None, ctypes.byref(pr), None, None, None, 0, None) == 1
    assert lib.rsvd_power_iter(None, ctypes.byref(pr), None, None, None, 0, None) == 1
    assert lib.rsvd_project(None, ctypes.byref(pr), None, None, None, None, 0, None) == 1
    assert lib.rsvd_svd(None, ctypes.byref(pr), None, None, None, None, None, None, 0, None) == 1
    assert lib.rsvd_sketch(None, ctypes.byref(pr), None, None, None, 0, None) == 1
    assert lib.rsvd_draw_srft(None, ctypes.byref(pr), None, None, None) == 1
    assert lib.rsvd_device_status(None, None, None) == 1
    assert lib.rsvd_profile_enable(None, 4) == 1
    assert lib.rsvd_profile_select(None, 0) == 1
    assert lib.rsvd_profile_read(None, None, None) == 1
    assert lib.rsvd_create(None, 0) == 1
    # symmetric Stage B: no handle, and a non-square problem, are refused on the host
    sq = _prob(m=500, n=500)
    assert lib.rsvd_eigh(None, ctypes.byref(sq), None, None, None, None, None, 0, None) == 1
    assert lib.rsvd_nystrom(None, ctypes.byref(sq), None, None, None, None, None, 0, None) == 1
    rect = _prob(m=600, n=500)
    assert lib.rsvd_eigh(None, ctypes.byref(rect), None, None, None, None, None, 0, None) == 1
    assert lib.rsvd_nystrom(None, ctypes.byref(rect), None, None, None, None, None, 0, None) == 1
    assert lib.rsvd_eigh_onepass(None, ctypes.byref(sq), None, None, None, None, 0, None) == 1
    assert lib.rsvd_eigh_onepass(None, ctypes.byref(rect), None, None, None, None, 0, None) == 1
    assert lib.rsvd_svd_onepass(None, ctypes.byref(rect), None, None, None, None, None, 0, None) == 1


def test_batched_workspace_and_validation(lib):
    import torch
    from paper_0909_4061_amd import RsvdProblem, problem
    ok = [problem(300, 200, 10, 8, 1, dtype=torch.float32), problem(64, 64, 4, 8, 1, dtype=torch.float32)]
    arr = (RsvdProblem * 2)(*ok)
    assert lib.rsvd_batched_workspace_bytes(2, arr) > 0
    assert lib.rsvd_batched_workspace_bytes(0, arr) == 0
    mixed = (RsvdProblem * 2)(ok[0], problem(64, 64, 4, 8, 1, dtype=torch.float64))
    assert lib.rsvd_batched_workspace_bytes(2, mixed) == 0           # dtypes differ
    other_q = (RsvdProblem * 2)(ok[0], problem(64, 64, 4, 8, 2, dtype=torch.float32))
    assert lib.rsvd_batched_workspace_bytes(2, other_q) == 0         # q differs
    srft = (RsvdProblem * 1)(problem(64, 64, 4, 8, 0, dtype=torch.float32, sketch="srft"))
    assert lib.rsvd_batched_workspace_bytes(1, srft) == 0            # Gaussian sketch only
    bad = (RsvdProblem * 1)(problem(64, 64, 60, 8, 1, dtype=torch.float32))
    assert lib.rsvd_batched_workspace_bytes(1, bad) == 0             # l > min(m, n)
    # no handle: rejected on the host before any launch
    assert lib.rsvd_batched(None, 2, arr, None, None, None, None, None, 0, None) == 1


def test_adjoint_workspace_and_validation(lib):
    import torch
    from paper_0909_4061_amd import RsvdProblem, problem
    f32 = problem(300, 200, 10, 8, 1, dtype=torch.float32, prec="bf16x3")
    one = lib.rsvd_backward_workspace_bytes(ctypes.byref(f32))
    fwd = lib.rsvd_workspace_bytes(ctypes.byref(f32))
    assert one > fwd > 0                                              # bases, factors and adjoint temporaries
    srft = problem(64, 64, 4, 8, 0, dtype=torch.float32, sketch="srft")
    assert lib.rsvd_backward_workspace_bytes(ctypes.byref(srft)) == 0  # fixed Gaussian test matrix only
    # a larger q keeps more bases
    assert lib.rsvd_backward_workspace_bytes(ctypes.byref(problem(300, 200, 10, 8, 3, dtype=torch.float32))) > \
        lib.rsvd_backward_workspace_bytes(ctypes.byref(problem(300, 200, 10, 8, 1, dtype=torch.float32)))
    ok = (RsvdProblem * 2)(f32, problem(96, 80, 16, 8, 1, dtype=torch.float32, prec="bf16x3"))
    both = lib.rsvd_backward_batched_workspace_bytes(2, ok)
    assert both > 0
    assert lib.rsvd_backward_batched_workspace_bytes(0, ok) == 0
    mixed_prec = (RsvdProblem * 2)(f32, problem(96, 80, 16, 8, 1, dtype=torch.float32))
    assert lib.rsvd_backward_batched_workspace_bytes(2, mixed_prec) == 0
    assert lib.rsvd_backward_batched_workspace_bytes(1, (RsvdProblem * 1)(srft)) == 0
    # no handle: rejected on the host, nothing touches a device
    pr = ctypes.byref(f32)
    assert lib.rsvd_backward(None, pr, None, None, None, None, None, None, 0, None) == 1
    assert lib.rsvd_forward_kept(None, pr, None, None, None, None, None, 0, None) == 1
    assert lib.rsvd_backward_kept(None, pr, None, None, None, None, None, None, 0, None) == 1
    assert lib.rsvd_backward_batched(None, 2, ok, None, None, None, None, None, None, 0, None) == 1
    assert lib.rsvd_batched_kept(None, 2, ok, None, None, None, None, None, 0, None) == 1
    assert lib.rsvd_backward_batched_kept(None, 2, ok, None, None, None, None, None, None, 0, None) == 1


@pytest.mark.parametrize("sketch", ["srft", 1])
def test_srft_under_autograd_is_refused(lib, sketch):
    # The adjoint holds an explicit Gaussian Omega fixed; an SRFT call that requires grad must
    # raise before any device work instead of returning Gaussian-sketch factors.
    import torch
    import paper_0909_4061_amd as rs
    A = torch.zeros(64, 32, dtype=torch.float32, requires_grad=True)
    with pytest.raises(rs.RsvdError) as e:
        rs.rsvd(A, 4, 2, 0, sketch=sketch)
    assert e.value.status == rs._lib.RSVD_E_UNSUPPORTED
    # the same call without grad is not refused by this check (it then needs a device tensor)
    with torch.no_grad(), pytest.raises(ValueError):
        rs.rsvd(A, 4, 2, 0, sketch=sketch)


def test_full_static_size_limit_before_handle(lib):
    # rsvd_full_static checks the problem and its workspace size on the host before it looks at
    # the handle or any pointer: an oversized problem is refused with RSVD_E_WORKSPACE.
    from paper_0909_4061_amd import _lib
    big = _prob(m=4096, n=2048, k=64, p=16, q=1, dtype=__import__("torch").float32)
    assert lib.rsvd_full_workspace_bytes(ctypes.byref(big)) > _lib.RSVD_STATIC_SCRATCH_BYTES
    assert lib.rsvd_full_static(None, ctypes.byref(big), None, None, None, None, None) == _lib.RSVD_E_WORKSPACE
    small = _prob()
    assert lib.rsvd_full_workspace_bytes(ctypes.byref(small)) <= _lib.RSVD_STATIC_SCRATCH_BYTES
    assert lib.rsvd_full_static(None, ctypes.byref(small), None, None, None, None, None) == _lib.RSVD_E_INVAL
    bad = _prob(k=0)
    assert lib.rsvd_full_static(None, ctypes.byref(bad), None, None, None, None, None) == _lib.RSVD_E_INVAL


def test_range_finder_tol_validation(lib):
    from paper_0909_4061_amd import _lib
    ok = _prob(m=700, n=400, k=16, p=112)          # b0 = 16, lmax = 128 = 16 * 2^3
    assert lib.rsvd_range_finder_tol_workspace_bytes(ctypes.byref(ok), 10) > 0
    assert lib.rsvd_range_finder_tol_workspace_bytes(ctypes.byref(ok), 17) == 0   # r > b0
    assert lib.rsvd_range_finder_tol_workspace_bytes(ctypes.byref(ok), 0) == 0
    odd = _prob(m=700, n=400, k=16, p=32)          # lmax = 48 = 16 * 3: not a doubling schedule
    assert lib.rsvd_range_finder_tol_workspace_bytes(ctypes.byref(odd), 10) == 0
    powered = _prob(m=700, n=400, k=16, p=112, q=1)
    assert lib.rsvd_range_finder_tol_workspace_bytes(ctypes.byref(powered), 10) == 0
    l_out, est = ctypes.c_int32(0), ctypes.c_double(0.0)
    assert lib.rsvd_range_finder_tol(None, ctypes.byref(ok), 1e-3, 10, None, None, ctypes.byref(l_out),
                                     ctypes.byref(est), None, 0, None) == _lib.RSVD_E_INVAL
    assert lib.rsvd_range_finder_tol(None, ctypes.byref(odd), 1e-3, 10, None, None, ctypes.byref(l_out),
                                     ctypes.byref(est), None, 0, None) == _lib.RSVD_E_INVAL
    assert lib.rsvd_range_finder_tol(None, ctypes.byref(powered), 1e-3, 10, None, None, ctypes.byref(l_out),
                                     ctypes.byref(est), None, 0, None) == _lib.RSVD_E_UNSUPPORTED
