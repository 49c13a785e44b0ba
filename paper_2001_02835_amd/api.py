"""Python binding of the polymat C ABI over torch device tensors.

The functions here only marshal arguments: they check dtypes and devices,
allocate caller-side output and workspace tensors, and pass raw device
pointers and the current HIP stream to libpolymat.so.  Every step of the
computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from typing import Iterable, Optional, Sequence

import torch

from . import _native as nat

PRECISIONS = {"fp64": nat.PM_PREC_FP64, "fp32": nat.PM_PREC_FP32, "bf16x3": nat.PM_PREC_BF16X3}


def _prec(p) -> int:
    if isinstance(p, str):
        if p not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        return PRECISIONS[p]
    return int(p)


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _series_check(x: torch.Tensor, name: str) -> None:
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex128 or not x.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA (HIP) tensor")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def workspace(nbytes: int, device) -> torch.Tensor:
    """A device byte buffer of at least nbytes (256-byte aligned by the caching allocator)."""
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if t.data_ptr() % 256:
        raise RuntimeError("workspace allocation is not 256-byte aligned")
    return t


def transform_length(ntrunc: int) -> int:
    return int(nat.lib().polymat_transform_length(int(ntrunc)))


def workspace_size(n: int, ntrunc: int, precision="fp64", count: int = 1) -> int:
    return int(nat.lib().polymat_workspace_size(int(n), int(ntrunc), _prec(precision), int(count)))


def polymat_mul(A: torch.Tensor, B: torch.Tensor, C: Optional[torch.Tensor] = None,
                precision="fp64", scale: float = 0.0, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """C = A * B (truncated star product) for complex128 [ntrunc+1, n, n] device tensors."""
    _series_check(A, "A")
    _series_check(B, "B")
    if A.shape != B.shape or A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("A and B must both have shape [ntrunc+1, n, n]")
    if C is None:
        C = torch.empty_like(A)
    _series_check(C, "C")
    nt, n = A.shape[0] - 1, A.shape[1]
    p = _prec(precision)
    need = nat.lib().polymat_workspace_size(n, nt, p, 1)
    if need == 0:
        raise ValueError("invalid size or precision")
    if ws is None:
        ws = workspace(need, A.device)
    st = nat.lib().polymat_mul(A.data_ptr(), B.data_ptr(), C.data_ptr(), n, nt, p, float(scale),
                               ws.data_ptr(), ws.numel(), _stream_ptr(A.device))
    nat.check(st, "polymat_mul")
    return C


def polymat_mul_noalloc(A: torch.Tensor, B: torch.Tensor, C: Optional[torch.Tensor] = None,
                        precision="fp64", scale: float = 0.0) -> torch.Tensor:
    """C = A * B on the library's built-in device scratch array (no workspace
    argument; products up to PM_NOALLOC_SCRATCH_BYTES of workspace)."""
    _series_check(A, "A")
    _series_check(B, "B")
    if A.shape != B.shape or A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("A and B must both have shape [ntrunc+1, n, n]")
    if C is None:
        C = torch.empty_like(A)
    _series_check(C, "C")
    nt, n = A.shape[0] - 1, A.shape[1]
    st = nat.lib().polymat_mul_noalloc(A.data_ptr(), B.data_ptr(), C.data_ptr(), n, nt, _prec(precision),
                                       float(scale), _stream_ptr(A.device))
    nat.check(st, "polymat_mul_noalloc")
    return C


def _problems(items) -> ctypes.Array:
    arr = (nat.PmProblem * len(items))()
    for i, it in enumerate(items):
        A, B, C = it["A"], it["B"], it["C"]
        for t, nm in ((A, "A"), (B, "B"), (C, "C")):
            _series_check(t, nm)
        arr[i].A = A.data_ptr()
        arr[i].B = B.data_ptr()
        arr[i].C = C.data_ptr()
        arr[i].n = A.shape[1]
        arr[i].ntrunc = A.shape[0] - 1
        arr[i].op_a = int(it.get("op_a", 0))
        arr[i].op_b = int(it.get("op_b", 0))
        arr[i].scale = float(it.get("scale", 0.0))
        if B.shape != A.shape or C.shape != A.shape:
            raise ValueError("every problem needs A, B, C of one shape")
    return arr


def batched_workspace_size(items: Sequence[dict], precision="fp64") -> int:
    arr = _problems(items)
    return int(nat.lib().polymat_batched_workspace_size(arr, len(items), _prec(precision)))


def polymat_mul_naive(A: torch.Tensor, B: torch.Tensor, C: Optional[torch.Tensor] = None,
                      op_a: int = 0, op_b: int = 0) -> torch.Tensor:
    """C = op_a(A) * op_b(B) by the direct convolution of eq. (5) (FP64); C must
    not overlap A or B.  Series [ntrunc+1, n, n] complex128."""
    _series_check(A, "A")
    _series_check(B, "B")
    if A.shape != B.shape or A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("A and B must be [ntrunc+1, n, n] of one shape")
    if C is None:
        C = torch.empty_like(A)
    _series_check(C, "C")
    nt1, n = A.shape[0], A.shape[1]
    st = nat.lib().polymat_mul_naive(A.data_ptr(), B.data_ptr(), C.data_ptr(), n, nt1 - 1, int(op_a), int(op_b),
                                     _stream_ptr(A.device))
    nat.check(st, "polymat_mul_naive")
    return C


def polymat_mul_batched(items: Sequence[dict], precision="fp64", ws: Optional[torch.Tensor] = None):
    """Each item: dict(A=, B=, C=, op_a=0|1, op_b=0|1, scale=0.0); C = op_a(A) * op_b(B)."""
    if not items:
        return
    arr = _problems(items)
    p = _prec(precision)
    need = nat.lib().polymat_batched_workspace_size(arr, len(items), p)
    if need == 0:
        raise ValueError("invalid batch")
    dev = items[0]["A"].device
    if ws is None:
        ws = workspace(need, dev)
    st = nat.lib().polymat_mul_batched(arr, len(items), p, ws.data_ptr(), ws.numel(), _stream_ptr(dev))
    nat.check(st, "polymat_mul_batched")


def forward_transform(A: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
    """At^(p) = sum_k scale^k A^(k) w^{kp}: complex128 [L, n, n]."""
    _series_check(A, "A")
    nt, n = A.shape[0] - 1, A.shape[1]
    L = transform_length(nt)
    At = torch.empty((L, n, n), dtype=torch.complex128, device=A.device)
    ws = workspace(nat.lib().polymat_transform_workspace_size(), A.device)
    st = nat.lib().polymat_forward_transform(A.data_ptr(), At.data_ptr(), n, nt, float(scale),
                                             ws.data_ptr(), ws.numel(), _stream_ptr(A.device))
    nat.check(st, "polymat_forward_transform")
    return At


def inverse_transform(Ct: torch.Tensor, ntrunc: int, scale: float = 1.0) -> torch.Tensor:
    """C^(k) = scale^-k (1/L) sum_p Ct^(p) w^{-kp}, k <= ntrunc."""
    _series_check(Ct, "Ct")
    n = Ct.shape[1]
    C = torch.empty((ntrunc + 1, n, n), dtype=torch.complex128, device=Ct.device)
    ws = workspace(nat.lib().polymat_transform_workspace_size(), Ct.device)
    st = nat.lib().polymat_inverse_transform(Ct.data_ptr(), C.data_ptr(), n, int(ntrunc), float(scale),
                                             ws.data_ptr(), ws.numel(), _stream_ptr(Ct.device))
    nat.check(st, "polymat_inverse_transform")
    return C


def nspt_params(L: int, k: int, ntrunc: int, eps: float) -> nat.NsptParams:
    return nat.NsptParams(L * L, L, k, ntrunc, float(eps))


def nspt_workspace_size(replicas: int, params: nat.NsptParams, precision="fp64") -> int:
    return int(nat.lib().nspt_workspace_size(int(replicas), ctypes.byref(params), _prec(precision)))


def nspt_langevin_step(U: torch.Tensor, eta: torch.Tensor, params: nat.NsptParams, precision="fp64",
                       ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One Euler-Langevin step of U [R, 4, ntrunc+1, n, n] in place, noise eta [R, 4, n, n]."""
    _series_check(U, "U")
    _series_check(eta, "eta")
    R = U.shape[0]
    p = _prec(precision)
    need = nat.lib().nspt_workspace_size(R, ctypes.byref(params), p)
    if need == 0:
        raise ValueError("invalid NSPT parameters")
    if ws is None:
        ws = workspace(need, U.device)
    st = nat.lib().nspt_langevin_step(U.data_ptr(), eta.data_ptr(), R, ctypes.byref(params), p,
                                      ws.data_ptr(), ws.numel(), _stream_ptr(U.device))
    nat.check(st, "nspt_langevin_step")
    return U


def nspt_md_trajectory(U: torch.Tensor, P: torch.Tensor, params: nat.NsptParams, nsteps: int,
                       eta: Optional[torch.Tensor] = None, precision="fp64",
                       ws: Optional[torch.Tensor] = None):
    """One leapfrog trajectory (step params.eps) of U and the momentum series P,
    both [R, 4, ntrunc+1, n, n], in place; eta [R, 4, n, n] refreshes P first."""
    _series_check(U, "U")
    _series_check(P, "P")
    if eta is not None:
        _series_check(eta, "eta")
    R = U.shape[0]
    p = _prec(precision)
    need = nat.lib().nspt_workspace_size(R, ctypes.byref(params), p)
    if need == 0:
        raise ValueError("invalid NSPT parameters")
    if ws is None:
        ws = workspace(need, U.device)
    st = nat.lib().nspt_md_trajectory(U.data_ptr(), P.data_ptr(), None if eta is None else eta.data_ptr(), R,
                                      ctypes.byref(params), int(nsteps), p, ws.data_ptr(), ws.numel(),
                                      _stream_ptr(U.device))
    nat.check(st, "nspt_md_trajectory")
    return U, P


def nspt_noise(replicas: int, n: int, seed: int, step: int, device="cuda:0") -> torch.Tensor:
    """Counter-based Langevin noise complex128 [replicas, 4, n, n] of one step."""
    eta = torch.empty((replicas, 4, n, n), dtype=torch.complex128, device=device)
    st = nat.lib().nspt_noise(eta.data_ptr(), int(replicas), int(n), int(seed), int(step), _stream_ptr(eta.device))
    nat.check(st, "nspt_noise")
    return eta


def nspt_langevin_steps(U: torch.Tensor, params: nat.NsptParams, seed: int, step0: int, nsteps: int,
                        precision="fp64", ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """nsteps Langevin steps of U [R, 4, ntrunc+1, n, n] in place, noise drawn on the device."""
    _series_check(U, "U")
    R = U.shape[0]
    p = _prec(precision)
    need = nat.lib().nspt_workspace_size(R, ctypes.byref(params), p)
    if need == 0:
        raise ValueError("invalid NSPT parameters")
    if ws is None:
        ws = workspace(need, U.device)
    st = nat.lib().nspt_langevin_steps(U.data_ptr(), R, ctypes.byref(params), int(seed), int(step0), int(nsteps), p,
                                       ws.data_ptr(), ws.numel(), _stream_ptr(U.device))
    nat.check(st, "nspt_langevin_steps")
    return U


def nspt_gauge_fix(U: torch.Tensor, params: nat.NsptParams, alpha: float, precision="fp64",
                   ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One stochastic gauge-fixing step of step size alpha on U [R, 4, ntrunc+1, n, n], in place."""
    _series_check(U, "U")
    R = U.shape[0]
    p = _prec(precision)
    need = nat.lib().nspt_workspace_size(R, ctypes.byref(params), p)
    if need == 0:
        raise ValueError("invalid NSPT parameters")
    if ws is None:
        ws = workspace(need, U.device)
    st = nat.lib().nspt_gauge_fix(U.data_ptr(), R, ctypes.byref(params), float(alpha), p, ws.data_ptr(),
                                  ws.numel(), _stream_ptr(U.device))
    nat.check(st, "nspt_gauge_fix")
    return U


def nspt_action(U: torch.Tensor, params: nat.NsptParams, precision="fp64",
                ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Action series S^(k) (float64 [R, ntrunc+1]) of link series U [R, 4, ntrunc+1, n, n]."""
    _series_check(U, "U")
    R, nord = U.shape[0], U.shape[2]
    p = _prec(precision)
    need = nat.lib().nspt_workspace_size(R, ctypes.byref(params), p)
    if need == 0:
        raise ValueError("invalid NSPT parameters")
    if ws is None:
        ws = workspace(need, U.device)
    S = torch.empty((R, nord), dtype=torch.float64, device=U.device)
    st = nat.lib().nspt_action(U.data_ptr(), R, ctypes.byref(params), p, S.data_ptr(), ws.data_ptr(), ws.numel(),
                               _stream_ptr(U.device))
    nat.check(st, "nspt_action")
    return S


def nspt_wilson_loop(U: torch.Tensor, params: nat.NsptParams, a: int, b: int, precision="fp64",
                     ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """a x b Wilson-loop series W^(k) (float64 [R, ntrunc+1]) of link series U [R, 4, ntrunc+1, n, n]."""
    _series_check(U, "U")
    R, nord = U.shape[0], U.shape[2]
    p = _prec(precision)
    need = nat.lib().nspt_workspace_size(R, ctypes.byref(params), p)
    if need == 0:
        raise ValueError("invalid NSPT parameters")
    if ws is None:
        ws = workspace(need, U.device)
    W = torch.empty((R, nord), dtype=torch.float64, device=U.device)
    st = nat.lib().nspt_wilson_loop(U.data_ptr(), R, ctypes.byref(params), int(a), int(b), p, W.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream_ptr(U.device))
    nat.check(st, "nspt_wilson_loop")
    return W


def check_enable(on: bool = True) -> None:
    """Turn the finiteness check of polymat_mul / polymat_mul_batched on or off:
    while on, those calls synchronise the stream and raise PolymatError with
    status PM_ERR_NONFINITE when an operand or a result coefficient is not finite."""
    nat.check(nat.lib().polymat_check_enable(1 if on else 0), "polymat_check_enable")


def timing_enable(on: bool = True) -> None:
    """Bracket every library launch with HIP events (for measurement only)."""
    nat.check(nat.lib().polymat_timing_enable(1 if on else 0), "polymat_timing_enable")


def timing_read() -> dict:
    """{phase: (milliseconds, launches)} since the last read; waits for the events."""
    n = len(nat.PHASES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int * n)()
    nat.check(nat.lib().polymat_timing_read(ms, cnt), "polymat_timing_read")
    return {nat.PHASES[i]: (ms[i], cnt[i]) for i in range(n)}
