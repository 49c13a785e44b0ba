"""C-ABI checks that need no GPU: the library loads, exports every function
include/polymat.h declares, and rejects bad arguments on the host before it
touches the device (every call below fails validation or, for a zero
gauge-fixing step, returns before any work, so nothing is ever enqueued and
no pointer is dereferenced)."""
import ctypes
import os
import re

import pytest

import paper_2001_02835_amd as pm
from paper_2001_02835_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polymat.h")

# fake, 256-byte aligned "device" addresses; only ever passed to calls that
# must fail validation
FAKE_A, FAKE_B, FAKE_C, FAKE_WS = 0x10000000, 0x20000000, 0x30000000, 0x40000000


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)
    keep = [n for n in names if n.startswith(("polymat_", "nspt_"))]
    return sorted(set(keep))


def test_library_loads_and_exports_every_declared_function():
    lib = pm.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(nat.SIGNATURES), "binding and header disagree"
    assert lib.polymat_abi_version() == 1


def test_strerror_texts():
    for s in range(6):
        assert isinstance(nat.strerror(s), str) and nat.strerror(s)
    assert nat.strerror(99) == "unknown status"


def test_check_mode_switches_and_nonfinite_status_has_text():
    lib = pm.lib()
    assert nat.PM_ERR_NONFINITE == 5
    assert "finite" in nat.strerror(nat.PM_ERR_NONFINITE)
    assert lib.polymat_check_enable(1) == nat.PM_OK
    # validation still happens first: an invalid call returns before any check
    assert lib.polymat_mul(None, FAKE_B, FAKE_C, 9, 7, 0, 0.0, FAKE_WS, 1 << 30, None) == nat.PM_ERR_INVALID
    assert lib.polymat_check_enable(0) == nat.PM_OK


def test_noalloc_rejects_sizes_before_any_device_call():
    lib = pm.lib()
    f = lib.polymat_mul_noalloc
    assert f(FAKE_A, FAKE_B, FAKE_C, 0, 7, 0, 0.0, None) == nat.PM_ERR_INVALID         # n < 1
    assert f(FAKE_A, FAKE_B, FAKE_C, 9, -1, 0, 0.0, None) == nat.PM_ERR_INVALID        # ntrunc < 0
    assert f(FAKE_A, FAKE_B, FAKE_C, 9, 7, 3, 0.0, None) == nat.PM_ERR_INVALID         # bad precision
    assert f(FAKE_A, FAKE_B, FAKE_C, 9, 64, 0, 0.0, None) == nat.PM_ERR_UNSUPPORTED    # ntrunc too large
    # workspace beyond the built-in array: N = 300, ntrunc = 63, FP64
    assert lib.polymat_workspace_size(300, 63, 0, 1) > nat.NOALLOC_SCRATCH_BYTES
    assert f(FAKE_A, FAKE_B, FAKE_C, 300, 63, 0, 0.0, None) == nat.PM_ERR_UNSUPPORTED
    # the largest benchmarked single products fit
    for prec, nt in ((0, 31), (1, 63), (2, 63)):
        assert 0 < lib.polymat_workspace_size(225, nt, prec, 1) <= nat.NOALLOC_SCRATCH_BYTES


def test_transform_length():
    lib = pm.lib()
    assert [lib.polymat_transform_length(t) for t in (0, 1, 3, 7, 15, 31, 63, 5, 12)] == \
        [4, 4, 8, 16, 32, 64, 128, 16, 32]
    assert lib.polymat_transform_length(-1) == 0
    assert lib.polymat_transform_length(64) == 0


def test_workspace_size_queries():
    lib = pm.lib()
    w1 = lib.polymat_workspace_size(225, 31, nat.PM_PREC_FP64, 1)
    assert w1 >= 3 * 64 * 225 * 225 * 16
    assert lib.polymat_workspace_size(225, 31, nat.PM_PREC_FP64, 4) == 4 * w1
    assert lib.polymat_workspace_size(225, 31, nat.PM_PREC_FP32, 1) < w1
    assert lib.polymat_workspace_size(225, 31, nat.PM_PREC_BF16X3, 1) < w1
    for bad in [(0, 7, 0, 1), (9, -1, 0, 1), (9, 64, 0, 1), (9, 7, 3, 1), (9, 7, 0, 0), (5000, 7, 0, 1)]:
        assert lib.polymat_workspace_size(*bad) == 0
    assert lib.polymat_transform_workspace_size() >= 8 * 129


def _mul(A=FAKE_A, B=FAKE_B, C=FAKE_C, n=9, nt=7, prec=0, scale=0.0, ws=FAKE_WS, wsb=0, stream=None):
    return pm.lib().polymat_mul(A, B, C, n, nt, prec, scale, ws, wsb, stream)


def test_polymat_mul_rejects_bad_arguments():
    need = pm.lib().polymat_workspace_size(9, 7, 0, 1)
    E = nat.PM_ERR_INVALID
    assert _mul(A=None, wsb=need) == E
    assert _mul(B=None, wsb=need) == E
    assert _mul(C=None, wsb=need) == E
    assert _mul(A=FAKE_A + 8, wsb=need) == E             # misaligned
    assert _mul(n=0, wsb=need) == E
    assert _mul(n=-3, wsb=need) == E
    assert _mul(nt=-1, wsb=need) == E
    assert _mul(nt=64, wsb=need) == nat.PM_ERR_UNSUPPORTED
    assert _mul(prec=7, wsb=need) == E
    assert _mul(scale=-1.0, wsb=need) == E
    assert _mul(scale=float("nan"), wsb=need) == E
    assert _mul(scale=float("inf"), wsb=need) == E
    assert _mul(ws=None, wsb=need) == E
    assert _mul(ws=FAKE_WS + 64, wsb=need) == E          # workspace must be 256-B aligned
    assert _mul(wsb=need - 1) == nat.PM_ERR_WORKSPACE
    assert _mul(ws=FAKE_A, wsb=need) == E                # workspace overlaps A
    assert _mul(ws=FAKE_C - 256, wsb=need) == E          # workspace overlaps C


def test_batched_rejects_bad_arguments():
    lib = pm.lib()
    arr = (nat.PmProblem * 2)()
    for i in range(2):
        arr[i].A, arr[i].B, arr[i].C = FAKE_A, FAKE_B, FAKE_C + i * 0x1000000
        arr[i].n, arr[i].ntrunc, arr[i].op_a, arr[i].op_b, arr[i].scale = 9, 7, 0, 0, 0.0
    need = lib.polymat_batched_workspace_size(arr, 2, 0)
    assert need == 2 * lib.polymat_workspace_size(9, 7, 0, 1)
    assert lib.polymat_mul_batched(arr, 0, 0, FAKE_WS, need, None) == nat.PM_ERR_INVALID
    assert lib.polymat_mul_batched(None, 1, 0, FAKE_WS, need, None) == nat.PM_ERR_INVALID
    assert lib.polymat_mul_batched(arr, 2, 0, FAKE_WS, need - 1, None) == nat.PM_ERR_WORKSPACE
    arr[1].op_a = 2
    assert lib.polymat_batched_workspace_size(arr, 2, 0) == 0
    assert lib.polymat_mul_batched(arr, 2, 0, FAKE_WS, need, None) == nat.PM_ERR_INVALID
    arr[1].op_a = 1
    arr[1].C = FAKE_C + 128                                # two outputs overlap
    assert lib.polymat_mul_batched(arr, 2, 0, FAKE_WS, need, None) == nat.PM_ERR_INVALID


def test_transform_entry_points_reject_bad_arguments():
    lib = pm.lib()
    w = lib.polymat_transform_workspace_size()
    E = nat.PM_ERR_INVALID
    assert lib.polymat_forward_transform(FAKE_A, FAKE_B, 9, 7, 0.0, FAKE_WS, w, None) == E  # scale must be > 0
    assert lib.polymat_forward_transform(None, FAKE_B, 9, 7, 1.0, FAKE_WS, w, None) == E
    assert lib.polymat_forward_transform(FAKE_A, FAKE_B, 9, 7, 1.0, FAKE_WS, w - 1, None) == nat.PM_ERR_WORKSPACE
    assert lib.polymat_forward_transform(FAKE_A, FAKE_A + 256, 9, 7, 1.0, FAKE_WS, w, None) == E  # overlap
    assert lib.polymat_inverse_transform(FAKE_A, FAKE_B, 9, 99, 1.0, FAKE_WS, w, None) == nat.PM_ERR_UNSUPPORTED
    assert lib.polymat_inverse_transform(FAKE_A, FAKE_B, 0, 7, 1.0, FAKE_WS, w, None) == E


def test_nspt_rejects_bad_arguments():
    lib = pm.lib()
    good = nat.NsptParams(9, 3, 1, 7, 0.01)
    for bad in [nat.NsptParams(10, 3, 1, 7, 0.01),     # n != L*L
                nat.NsptParams(9, 3, 1, 7, -0.01),     # eps <= 0
                nat.NsptParams(9, 3, 1, 64, 0.01),     # ntrunc too large
                nat.NsptParams(16, 4, 1, 7, 0.01)]:    # even L
        assert lib.nspt_workspace_size(1, ctypes.byref(bad), 0) == 0
        assert lib.nspt_langevin_step(FAKE_A, FAKE_B, 1, ctypes.byref(bad), 0, FAKE_WS, 1 << 40, None) != nat.PM_OK
    need = lib.nspt_workspace_size(2, ctypes.byref(good), 0)
    assert need > 0
    assert lib.nspt_workspace_size(0, ctypes.byref(good), 0) == 0
    assert lib.nspt_langevin_step(FAKE_A, FAKE_B, 2, ctypes.byref(good), 0, FAKE_WS, need - 1, None) == \
        nat.PM_ERR_WORKSPACE
    assert lib.nspt_langevin_step(None, FAKE_B, 2, ctypes.byref(good), 0, FAKE_WS, need, None) == nat.PM_ERR_INVALID


def test_md_trajectory_rejects_bad_arguments():
    lib = pm.lib()
    good = nat.NsptParams(9, 3, 1, 7, 0.1)
    need = lib.nspt_workspace_size(1, ctypes.byref(good), 0)
    P = FAKE_A + (1 << 32)
    eta = FAKE_B + (1 << 33)
    call = lambda U, Pp, e, R, prm, ns, ws, nb: lib.nspt_md_trajectory(U, Pp, e, R, ctypes.byref(prm), ns, 0, ws,
                                                                       nb, None)
    assert call(FAKE_A, P, eta, 1, good, 0, FAKE_WS, need) == nat.PM_ERR_INVALID          # nsteps < 1
    assert call(FAKE_A, P, eta, 1, good, 100001, FAKE_WS, need) == nat.PM_ERR_INVALID     # nsteps too large
    assert call(None, P, eta, 1, good, 4, FAKE_WS, need) == nat.PM_ERR_INVALID            # no U
    assert call(FAKE_A, None, eta, 1, good, 4, FAKE_WS, need) == nat.PM_ERR_INVALID       # no P
    assert call(FAKE_A, FAKE_A, eta, 1, good, 4, FAKE_WS, need) == nat.PM_ERR_INVALID     # U and P overlap
    assert call(FAKE_A, P, eta, 1, good, 4, FAKE_WS, need - 1) == nat.PM_ERR_WORKSPACE
    assert call(FAKE_A, P, eta, 1, nat.NsptParams(9, 3, 1, 7, 0.0), 4, FAKE_WS, need) == nat.PM_ERR_INVALID


def test_naive_rejects_bad_arguments():
    lib = pm.lib()
    f = lib.polymat_mul_naive
    assert f(None, FAKE_B, FAKE_C, 9, 3, 0, 0, None) == nat.PM_ERR_INVALID
    assert f(FAKE_A, FAKE_B, FAKE_C, 0, 3, 0, 0, None) == nat.PM_ERR_INVALID          # n < 1
    assert f(FAKE_A, FAKE_B, FAKE_C, 9, -1, 0, 0, None) == nat.PM_ERR_INVALID         # ntrunc < 0
    assert f(FAKE_A, FAKE_B, FAKE_C, 9, 64, 0, 0, None) == nat.PM_ERR_UNSUPPORTED     # ntrunc too large
    assert f(FAKE_A, FAKE_B, FAKE_C, 9, 3, 2, 0, None) == nat.PM_ERR_INVALID          # bad op
    assert f(FAKE_A, FAKE_B, FAKE_A, 9, 3, 0, 0, None) == nat.PM_ERR_INVALID          # C aliases A
    assert f(FAKE_A + 8, FAKE_B, FAKE_C, 9, 3, 0, 0, None) == nat.PM_ERR_INVALID      # misaligned


def test_action_rejects_bad_arguments():
    lib = pm.lib()
    good = nat.NsptParams(9, 3, 1, 7, 0.01)
    need = lib.nspt_workspace_size(1, ctypes.byref(good), 0)
    S = FAKE_C
    assert lib.nspt_action(None, 1, ctypes.byref(good), 0, S, FAKE_WS, need, None) == nat.PM_ERR_INVALID
    assert lib.nspt_action(FAKE_A, 1, ctypes.byref(good), 0, None, FAKE_WS, need, None) == nat.PM_ERR_INVALID
    assert lib.nspt_action(FAKE_A, 1, ctypes.byref(good), 0, S, FAKE_WS, need - 1, None) == nat.PM_ERR_WORKSPACE
    assert lib.nspt_action(FAKE_A, 1, ctypes.byref(good), 0, FAKE_A, FAKE_WS, need, None) == nat.PM_ERR_INVALID
    assert lib.nspt_action(FAKE_A, 0, ctypes.byref(good), 0, S, FAKE_WS, need, None) == nat.PM_ERR_INVALID


def test_wilson_loop_rejects_bad_arguments():
    lib = pm.lib()
    good = nat.NsptParams(9, 3, 1, 7, 0.01)
    need = lib.nspt_workspace_size(1, ctypes.byref(good), 0)
    f = lambda a, b, W=FAKE_C, nb=need: lib.nspt_wilson_loop(FAKE_A, 1, ctypes.byref(good), a, b, 0, W, FAKE_WS, nb,
                                                            None)
    assert f(0, 1) == nat.PM_ERR_INVALID
    assert f(1, 5) == nat.PM_ERR_INVALID
    assert f(2, 2, W=None) == nat.PM_ERR_INVALID
    assert f(2, 2, nb=need - 1) == nat.PM_ERR_WORKSPACE


def test_gauge_fix_rejects_bad_arguments():
    lib = pm.lib()
    good = nat.NsptParams(9, 3, 1, 7, 0.01)
    need = lib.nspt_workspace_size(1, ctypes.byref(good), 0)
    f = lambda U=FAKE_A, alpha=0.1, prm=good, ws=FAKE_WS, nb=need: lib.nspt_gauge_fix(U, 1, ctypes.byref(prm), alpha,
                                                                                      0, ws, nb, None)
    assert f(alpha=-0.1) == nat.PM_ERR_INVALID
    assert f(alpha=float("nan")) == nat.PM_ERR_INVALID
    assert f(alpha=float("inf")) == nat.PM_ERR_INVALID
    assert f(U=None) == nat.PM_ERR_INVALID
    assert f(U=FAKE_A + 8) == nat.PM_ERR_INVALID                                   # misaligned
    assert f(U=FAKE_WS) == nat.PM_ERR_INVALID                                      # U overlaps the workspace
    assert f(nb=need - 1) == nat.PM_ERR_WORKSPACE
    assert f(prm=nat.NsptParams(10, 3, 1, 7, 0.01)) == nat.PM_ERR_INVALID          # n != L^2
    assert f(alpha=0.0) == nat.PM_OK                                               # Omega = 1: nothing to do


def test_limits_of_counts_and_sizes():
    lib = pm.lib()
    good = nat.NsptParams(9, 3, 1, 7, 0.01)
    assert lib.nspt_workspace_size(1024, ctypes.byref(good), 0) > 0
    assert lib.nspt_workspace_size(1025, ctypes.byref(good), 0) == 0            # more than 1024 replicas
    assert lib.polymat_workspace_size(4096, 0, nat.PM_PREC_FP64, 1) > 0            # largest matrix
    assert lib.polymat_workspace_size(4097, 0, nat.PM_PREC_FP64, 1) == 0
    assert lib.polymat_workspace_size(9, 7, nat.PM_PREC_FP64, 4097) == 0           # batch above the limit
    arr = (nat.PmProblem * 1)()
    arr[0].A, arr[0].B, arr[0].C = FAKE_A, FAKE_B, FAKE_C
    arr[0].n, arr[0].ntrunc = 9, 7
    assert lib.polymat_batched_workspace_size(arr, 4097, 0) == 0
    assert lib.polymat_mul_batched(arr, 4097, 0, FAKE_WS, 1 << 40, None) == nat.PM_ERR_INVALID


def test_noise_and_steps_reject_bad_arguments():
    lib = pm.lib()
    E = nat.PM_ERR_INVALID
    assert lib.nspt_noise(None, 1, 9, 1, 0, None) == E
    assert lib.nspt_noise(FAKE_A, 0, 9, 1, 0, None) == E
    assert lib.nspt_noise(FAKE_A, 1025, 9, 1, 0, None) == E
    assert lib.nspt_noise(FAKE_A, 1, 0, 1, 0, None) == E
    assert lib.nspt_noise(FAKE_A, 1, 4097, 1, 0, None) == E
    assert lib.nspt_noise(FAKE_A + 8, 1, 9, 1, 0, None) == E                        # misaligned
    good = nat.NsptParams(9, 3, 1, 7, 0.01)
    need = lib.nspt_workspace_size(1, ctypes.byref(good), 0)
    f = lambda U=FAKE_A, prm=good, ns=2, nb=need: lib.nspt_langevin_steps(U, 1, ctypes.byref(prm), 5, 0, ns, 0,
                                                                          FAKE_WS, nb, None)
    assert f(ns=0) == E
    assert f(ns=100001) == E
    assert f(U=None) == E
    assert f(U=FAKE_WS) == E                                                        # U overlaps the workspace
    assert f(nb=need - 1) == nat.PM_ERR_WORKSPACE
    assert f(prm=nat.NsptParams(9, 3, 1, 7, 0.0)) == E


@pytest.mark.parametrize("lang,std", [("c", "-std=c99"), ("c++", "-std=c++11")])
def test_header_is_plain_c_and_cxx(lang, std):
    """include/polymat.h needs no HIP or torch headers: it compiles as C99
    and as C++11 with warnings as errors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc" if lang == "c" else "g++")
    if cc is None:
        pytest.skip("no host compiler")
    r = subprocess.run([cc, std, "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only", "-x", lang, HEADER],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
