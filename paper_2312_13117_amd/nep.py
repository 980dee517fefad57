"""ctypes binding of libnep.so (include/nep.h).  Argument marshalling only.

Device memory and streams come from PyTorch (torch.cuda tensors, current stream);
every step of the method runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnep.so")

NEP_OK, NEP_WARN_SINGULAR_NODE, NEP_WARN_REFINE_FALLBACK, NEP_WARN_SATURATED = 0, 1, 2, 3
NEP_FP64, NEP_FP32_REFINE = 0, 1


class nep_problem(C.Structure):
    _fields_ = [("n", C.c_int), ("nterms", C.c_int), ("A_dev", C.POINTER(C.c_void_p)),
                ("phi_kind", C.POINTER(C.c_int)), ("phi_param", C.POINTER(C.c_double))]


class nep_elementwise_delay(C.Structure):
    _fields_ = [("n", C.c_int), ("A0_dev", C.c_void_p), ("A1_dev", C.c_void_p), ("tau_dev", C.c_void_p)]


class nep_region(C.Structure):
    _fields_ = [("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("nx", C.c_int), ("ny", C.c_int)]


class nep_options(C.Structure):
    _fields_ = [("N", C.c_int), ("s", C.c_int), ("L", C.c_int), ("tol_ind", C.c_double),
                ("tol_svd", C.c_double), ("tol_ver", C.c_double), ("precision", C.c_int),
                ("max_refine", C.c_int), ("batch", C.c_int), ("streams", C.c_int),
                ("pivot", C.c_int), ("graph", C.c_int)]


class nep_stats(C.Structure):
    _fields_ = [("node_solves", C.c_int64), ("lu_count", C.c_int64), ("lu_flops", C.c_double),
                ("refine_sweeps", C.c_int64), ("refine_fallbacks", C.c_int64),
                ("singular_nodes", C.c_int64), ("ms_total", C.c_double), ("ms_assemble", C.c_double),
                ("ms_lu", C.c_double), ("ms_solve", C.c_double), ("ms_refine", C.c_double),
                ("ms_sums", C.c_double), ("ms_gemm", C.c_double), ("gemm_launches", C.c_int64),
                ("gemm_flops", C.c_double), ("ms_gemm_busy", C.c_double)]


_lib = None


def lib():
    """Load libnep.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_13117_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, ip, dp, u8p = C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_uint8)
    L.nep_plan.argtypes = [C.POINTER(nep_problem), C.c_int, C.POINTER(nep_region), C.POINTER(nep_options),
                           vp, C.POINTER(vp)]
    L.nep_indicator.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), dp, u8p, dp]
    L.nep_beyn.argtypes = [vp, ip, C.c_int, C.POINTER(vp), vp, ip, dp, u8p, vp]
    L.nep_verify.argtypes = [vp, ip, vp, C.c_int, dp, u8p]
    L.nep_refine.argtypes = [vp, ip, vp, C.c_int, C.c_int, dp, u8p, vp, C.c_int]
    L.nep_copy_sums.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, vp]
    L.nep_set_assembler.argtypes = [vp, C.c_int, vp, vp]
    L.nep_assemble_elementwise_delay.argtypes = [vp, C.c_int, vp, C.c_int, vp, C.c_longlong, vp]
    L.nep_assemble_circle_double_layer.argtypes = [vp, C.c_int, vp, C.c_int, vp, C.c_longlong, vp]
    L.nep_dedup.argtypes = [vp, dp, C.c_int, C.c_double, u8p]
    L.nep_merge.argtypes = [vp, C.c_int, C.c_double, vp, C.POINTER(C.c_int), ip]
    L.nep_own.argtypes = [dp, vp, C.c_int, C.c_double, u8p]
    L.nep_total_disks.argtypes = [vp]
    L.nep_disk_offset.argtypes = [vp, C.c_int]
    L.nep_get_stats.argtypes = [vp, C.POINTER(nep_stats)]
    L.nep_destroy.argtypes = [vp]
    L.nep_destroy.restype = None
    L.nep_status_str.argtypes = [C.c_int]
    L.nep_status_str.restype = C.c_char_p
    L.nep_last_error.argtypes = [vp]
    L.nep_last_error.restype = C.c_char_p
    fp = C.c_void_p
    L.nep_mlp_param_count.argtypes = []
    L.nep_mlp_workspace_floats.argtypes = [C.c_int]
    L.nep_mlp_workspace_floats.restype = C.c_size_t
    L.nep_mlp_forward.argtypes = [fp, fp, fp, C.c_int, fp, fp, vp]
    L.nep_mlp_forward_noalloc.argtypes = [fp, fp, fp, C.c_int, fp, vp]
    L.nep_mfma_peak.argtypes = [C.c_int, C.c_int, dp]
    L.nep_mlp_grad.argtypes = [fp, fp, fp, fp, C.c_int, fp, C.POINTER(C.c_float), fp, vp]
    L.nep_mlp_adam.argtypes = [fp, fp, fp, fp, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.nep_mlp_features.argtypes = [fp, C.c_int, C.c_int, fp, C.c_int, fp, fp, fp, vp]
    for f in ("nep_plan", "nep_indicator", "nep_beyn", "nep_verify", "nep_refine", "nep_set_assembler",
              "nep_assemble_elementwise_delay", "nep_assemble_circle_double_layer", "nep_copy_sums", "nep_dedup", "nep_merge", "nep_own",
              "nep_total_disks", "nep_disk_offset", "nep_get_stats", "nep_mlp_param_count", "nep_mlp_forward",
              "nep_mlp_forward_noalloc", "nep_mfma_peak",
              "nep_mlp_grad", "nep_mlp_adam", "nep_mlp_features"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


class NepError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _check(status: int, plan_handle=None) -> int:
    if status < 0:
        L = lib()
        msg = L.nep_last_error(plan_handle).decode() or L.nep_status_str(status).decode()
        raise NepError(status, msg)
    return status


def _ptr(a):
    return C.cast(a.ctypes.data, C.c_void_p) if isinstance(a, np.ndarray) else C.c_void_p(a)


def _dev_complex(x, torch):
    """Host complex array -> contiguous complex128 tensor on cuda:0 (or None); a cuda
    complex128 tensor is used as it is."""
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        t = x.to(device="cuda", dtype=torch.complex128)
    else:
        t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")
    return t.contiguous()


def _is_assembled(pr) -> bool:
    """An elementwise delay problem (no split form): assembled by the library's
    nep_assemble_elementwise_delay."""
    return hasattr(pr, "tau") and hasattr(pr, "A0")


def _is_circle(pr) -> bool:
    """The unit disk's double-layer problem: assembled by nep_assemble_circle_double_layer."""
    return type(pr).__name__ == "CircleDoubleLayer"


def _dev_real(x, torch):
    if isinstance(x, torch.Tensor):
        return x.to(device="cuda", dtype=torch.float64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda").contiguous()


def upload_problem(pr):
    """A copy of a gen.Problem (or gen.ElementwiseDelay) whose matrices are device
    tensors (uploaded once and shared by every plan entry that refers to it)."""
    import copy
    import torch
    q = copy.copy(pr)
    if _is_circle(pr):
        return q
    if _is_assembled(pr):
        q.A0, q.A1, q.tau = _dev_complex(pr.A0, torch), _dev_complex(pr.A1, torch), _dev_real(pr.tau, torch)
    else:
        q.coeffs = [_dev_complex(A, torch) for A in pr.coeffs]
    return q


@dataclass
class Plan:
    handle: C.c_void_p
    nprob: int
    n: List[int]
    N: int
    s: int
    L: int
    total_disks: int
    keep_alive: list = field(default_factory=list)


def nep_plan(problems, regions, opts, stream=None) -> Plan:
    """problems: gen.Problem list (coefficients uploaded here to device tensors);
    regions: gen.Region list; opts: gen.Options (with optional .batch)."""
    import torch
    L = lib()
    keep = []
    cp = (nep_problem * len(problems))()
    assembled = []
    split_terms = {}
    for i, pr in enumerate(problems):
        if _is_circle(pr):
            assembled.append((i, None))
            cp[i] = nep_problem(pr.n, 0, None, None, None)
            continue
        if _is_assembled(pr):
            t0, t1, tt = _dev_complex(pr.A0, torch), _dev_complex(pr.A1, torch), _dev_real(pr.tau, torch)
            ctx = nep_elementwise_delay(pr.n, t0.data_ptr(), t1.data_ptr(), tt.data_ptr())
            keep += [t0, t1, tt, ctx]
            assembled.append((i, ctx))
            cp[i] = nep_problem(pr.n, 0, None, None, None)
            continue
        if id(pr) in split_terms:            # the same problem object again (one entry per cell)
            cp[i] = split_terms[id(pr)]
            continue
        devs = []
        for A in pr.coeffs:
            t = _dev_complex(A, torch)
            keep.append(t)
            devs.append(t.data_ptr() if t is not None else None)
        arr = (C.c_void_p * len(devs))(*devs)
        kinds = (C.c_int * len(devs))(*pr.phi_kind)
        pars = (C.c_double * len(devs))(*pr.phi_param)
        keep += [arr, kinds, pars, pr]
        cp[i] = nep_problem(pr.n, len(devs), arr, kinds, pars)
        split_terms[id(pr)] = cp[i]
    cr = (nep_region * len(regions))()
    for i, r in enumerate(regions):
        cr[i] = nep_region(r.x0, r.x1, r.y0, r.y1, r.nx, r.ny)
    batch, streams = int(getattr(opts, "batch", 0) or 0), int(getattr(opts, "streams", 0) or 0)
    if batch == 0 and streams == 0 and not os.environ.get("NEP_NO_TUNING"):
        # launch configuration from the autotuner's table (never changes a result bit)
        from . import autotune
        e = autotune.lookup(max(p.n for p in problems), opts.precision)
        if e is not None:
            batch, streams = int(e["batch"]), int(e["streams"])
    co = nep_options(opts.N, opts.s, opts.L, opts.tol_ind, opts.tol_svd, opts.tol_ver, opts.precision,
                     opts.max_refine, batch, streams,
                     int(getattr(opts, "pivot", 0) or 0), int(getattr(opts, "graph", 0) or 0))
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    h = C.c_void_p()
    _check(L.nep_plan(cp, len(problems), cr, C.byref(co), C.c_void_p(stream), C.byref(h)), None)
    for i, ctx in assembled:
        if ctx is None:
            st = L.nep_set_assembler(h, i, C.cast(L.nep_assemble_circle_double_layer, C.c_void_p), None)
        else:
            st = L.nep_set_assembler(h, i, C.cast(L.nep_assemble_elementwise_delay, C.c_void_p), C.byref(ctx))
        if st < 0:
            msg = L.nep_last_error(h).decode()
            L.nep_destroy(h)
            raise NepError(st, msg)
    nd = L.nep_total_disks(h)
    return Plan(h, len(problems), [p.n for p in problems], opts.N, opts.s, opts.L, nd, keep)


def _dev_list(xs, torch):
    """_dev_complex over a per-entry list; an object given for many entries (the same
    probe block for every cell) is converted once."""
    done = {}
    out = []
    for x in xs:
        if id(x) not in done:
            done[id(x)] = _dev_complex(x, torch)
        out.append(done[id(x)])
    return out


def _ptr_array(tensors):
    return (C.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])


def nep_indicator(plan: Plan, F, V=None, want_profiles: bool = False):
    """F, V: per-problem device complex128 tensors (n x s, n x L), or host arrays.
    Returns (ind [nd x s], flags [nd] bool, profiles [nd x N x s] or None, status)."""
    import torch
    L = lib()
    Ft = _dev_list(F, torch)
    Vt = _dev_list(V, torch) if V is not None else None
    plan.keep_alive.append(Ft)            # the plan may re-sweep with F in nep_beyn
    nd = plan.total_disks
    ind = np.zeros(nd * plan.s)
    flags = np.zeros(nd, np.uint8)
    prof = np.zeros(nd * plan.N * plan.s) if want_profiles else None
    st = L.nep_indicator(plan.handle, _ptr_array(Ft), _ptr_array(Vt) if Vt is not None else None,
                         ind.ctypes.data_as(C.POINTER(C.c_double)), flags.ctypes.data_as(C.POINTER(C.c_uint8)),
                         prof.ctypes.data_as(C.POINTER(C.c_double)) if prof is not None else None)
    _check(st, plan.handle)
    return (ind.reshape(nd, plan.s), flags.astype(bool),
            prof.reshape(nd, plan.N, plan.s) if prof is not None else None, st)


def nep_beyn(plan: Plan, disk_ids: Sequence[int], V=None, want_vectors: bool = False):
    """Returns (eig [k x L] complex, p [k], sv [k x L], keep [k x L] bool, vectors or None, status)."""
    import torch
    L = lib()
    ids = np.ascontiguousarray(np.asarray(disk_ids, dtype=np.int32))
    k = len(ids)
    eig = np.zeros(k * plan.L, np.complex128)
    p = np.zeros(k, np.int32)
    sv = np.zeros(k * plan.L)
    keep = np.zeros(k * plan.L, np.uint8)
    vt = None
    if want_vectors and k > 0:
        vt = torch.zeros((k, max(plan.n), plan.L), dtype=torch.complex128, device="cuda")
    Vt = _dev_list(V, torch) if V is not None else None
    st = L.nep_beyn(plan.handle, ids.ctypes.data_as(C.POINTER(C.c_int32)), k,
                    _ptr_array(Vt) if Vt is not None else None, _ptr(eig),
                    p.ctypes.data_as(C.POINTER(C.c_int32)), sv.ctypes.data_as(C.POINTER(C.c_double)),
                    keep.ctypes.data_as(C.POINTER(C.c_uint8)), C.c_void_p(vt.data_ptr()) if vt is not None else None)
    _check(st, plan.handle)
    return (eig.reshape(k, plan.L), p, sv.reshape(k, plan.L), keep.reshape(k, plan.L).astype(bool), vt, st)


def nep_verify(plan: Plan, prob_ids: Sequence[int], lam: Sequence[complex]):
    L = lib()
    m = len(lam)
    pid = np.ascontiguousarray(np.asarray(prob_ids, dtype=np.int32))
    la = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128))
    sig = np.zeros(m)
    acc = np.zeros(m, np.uint8)
    st = L.nep_verify(plan.handle, pid.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(la), m,
                      sig.ctypes.data_as(C.POINTER(C.c_double)), acc.ctypes.data_as(C.POINTER(C.c_uint8)))
    _check(st, plan.handle)
    return sig, acc.astype(bool)


def nep_refine(plan: Plan, prob_ids: Sequence[int], lam: Sequence[complex], iters: int = 2,
               want_vectors: bool = False):
    """(refined lambda, sigma_min at it, accepted, vectors [m x max n] or None) -- see
    nep_refine in nep.h."""
    L = lib()
    m = len(lam)
    pid = np.ascontiguousarray(np.asarray(prob_ids, dtype=np.int32))
    la = np.array(lam, dtype=np.complex128, copy=True, order="C")
    sig = np.zeros(m)
    acc = np.zeros(m, np.uint8)
    ldv = max(plan.n) if want_vectors else 0
    vec = np.zeros((m, ldv), np.complex128) if want_vectors else None
    st = L.nep_refine(plan.handle, pid.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(la), m, int(iters),
                      sig.ctypes.data_as(C.POINTER(C.c_double)), acc.ctypes.data_as(C.POINTER(C.c_uint8)),
                      _ptr(vec) if vec is not None else None, ldv)
    _check(st, plan.handle)
    return la, sig, acc.astype(bool), vec


def _copy_sums_uniform(plan: Plan, first: int, count: int, n: int):
    L = lib()
    PfN = np.zeros((count, n, plan.s), np.complex128)
    PfN2 = np.zeros((count, n, plan.s), np.complex128)
    C0 = np.zeros((count, n, plan.L), np.complex128) if plan.L else None
    C1 = np.zeros((count, n, plan.L), np.complex128) if plan.L else None
    _check(L.nep_copy_sums(plan.handle, first, count, _ptr(PfN), _ptr(PfN2),
                           _ptr(C0) if C0 is not None else None, _ptr(C1) if C1 is not None else None),
           plan.handle)
    return PfN, PfN2, C0, C1


def nep_copy_sums(plan: Plan, first: int, count: int):
    """Sums of disks [first, first + count): arrays [count, n, cols] when the disks share
    n (always for a single-problem plan), else per-disk lists of [n, cols] arrays."""
    L = lib()
    if plan.nprob == 1:
        return _copy_sums_uniform(plan, first, count, plan.n[0])
    offs = [L.nep_disk_offset(plan.handle, p) for p in range(plan.nprob)] + [plan.total_disks]
    parts = []
    for p in range(plan.nprob):
        a, b = max(first, offs[p]), min(first + count, offs[p + 1])
        if a < b:
            parts.append(_copy_sums_uniform(plan, a, b - a, plan.n[p]))
    out = []
    for k in range(4):
        if parts and parts[0][k] is None:
            out.append(None)
        else:
            out.append([x for part in parts for x in part[k]])
    return tuple(out)


def nep_dedup(lam, sigma, rel: float = 1e-8):
    L = lib()
    la = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128))
    sg = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64))
    keep = np.zeros(len(la), np.uint8)
    _check(L.nep_dedup(_ptr(la), sg.ctypes.data_as(C.POINTER(C.c_double)), len(la), rel,
                       keep.ctypes.data_as(C.POINTER(C.c_uint8))))
    return keep.astype(bool)


def nep_merge(centres, tol_eps: float):
    """(merged values, group index of every centre): pmCIMa's merge of flagged centres."""
    L = lib()
    z = np.ascontiguousarray(np.asarray(centres, dtype=np.complex128))
    out = np.zeros(len(z), np.complex128)
    grp = np.zeros(len(z), np.int32)
    cnt = C.c_int(0)
    _check(L.nep_merge(_ptr(z), len(z), tol_eps, _ptr(out), C.byref(cnt),
                       grp.ctypes.data_as(C.POINTER(C.c_int32))))
    return out[:cnt.value].copy(), grp


def nep_own(cells, lam, band: float = 1e-6):
    """Mask of the candidates kept by the cell that produced them (cells: m x 4 rows
    (x0, x1, y0, y1) of each candidate's producing cell)."""
    L = lib()
    c = np.ascontiguousarray(np.asarray(cells, dtype=np.float64).reshape(-1, 4))
    la = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128))
    keep = np.zeros(len(la), np.uint8)
    _check(L.nep_own(c.ctypes.data_as(C.POINTER(C.c_double)), _ptr(la), len(la), band,
                     keep.ctypes.data_as(C.POINTER(C.c_uint8))))
    return keep.astype(bool)


def nep_get_stats(plan: Plan) -> dict:
    L = lib()
    s = nep_stats()
    _check(L.nep_get_stats(plan.handle, C.byref(s)), plan.handle)
    return {f: getattr(s, f) for f, _ in nep_stats._fields_}


def nep_destroy(plan: Plan) -> None:
    if plan.handle:
        lib().nep_destroy(plan.handle)
        plan.handle = C.c_void_p()


@dataclass
class Result:
    ind: np.ndarray
    flags: np.ndarray
    flagged: np.ndarray
    eig: np.ndarray
    p: np.ndarray
    sv: np.ndarray
    keep: np.ndarray
    cand_disk: np.ndarray
    cand: np.ndarray
    sigma: np.ndarray
    accepted: np.ndarray
    eigs: np.ndarray
    status: dict


def pmcimb(plan: Plan, F, V, disk_problem=None) -> Result:
    """The three steps in order: indicators (and moments) -> Beyn on flagged disks ->
    sigma_min verification of the kept candidates -> merge of duplicates."""
    ind, flags, _, st1 = nep_indicator(plan, F, V)
    flagged = np.nonzero(flags)[0]
    eig, p, sv, keep, _, st2 = nep_beyn(plan, flagged) if len(flagged) else (
        np.zeros((0, plan.L), np.complex128), np.zeros(0, np.int32), np.zeros((0, plan.L)),
        np.zeros((0, plan.L), bool), None, 0)
    cd, cl = [], []
    for i, d in enumerate(flagged):
        for k in range(int(p[i])):
            if keep[i, k]:
                cd.append(d)
                cl.append(eig[i, k])
    cd = np.asarray(cd, dtype=np.int64)
    cl = np.asarray(cl, dtype=np.complex128)
    if disk_problem is None:
        disk_problem = np.zeros(plan.total_disks, np.int32)
    sig, acc = nep_verify(plan, disk_problem[cd] if len(cd) else [], cl) if len(cl) else (np.zeros(0), np.zeros(0, bool))
    al, asg = cl[acc], sig[acc]
    kd = nep_dedup(al, asg) if len(al) else np.zeros(0, bool)
    eigs = al[kd]
    order = np.lexsort((eigs.imag, eigs.real))
    return Result(ind, flags, flagged, eig, p, sv, keep, cd, cl, sig, acc, eigs[order],
                  {"indicator": st1, "beyn": st2})


# ---------------------------------------------------------------- screener network
def _fptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def nep_mlp_param_count() -> int:
    return lib().nep_mlp_param_count()


def nep_mlp_workspace_floats(B: int) -> int:
    return lib().nep_mlp_workspace_floats(B)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def nep_mlp_forward(params, X, idx, B, probs, work):
    _check(lib().nep_mlp_forward(_fptr(params), _fptr(X), _fptr(idx), B, _fptr(probs), _fptr(work), _stream()))


def nep_mlp_forward_noalloc(params, X, idx, B, probs):
    _check(lib().nep_mlp_forward_noalloc(_fptr(params), _fptr(X), _fptr(idx), B, _fptr(probs), _stream()))


NEP_MLP_NOALLOC_MAX_B = 4096


def nep_mfma_peak(precision: int = NEP_FP64, iters: int = 8192) -> float:
    """Measured matrix-core rate (TFLOP/s) of the MFMA shape the LU update uses."""
    t = C.c_double(0.0)
    _check(lib().nep_mfma_peak(precision, iters, C.byref(t)))
    return t.value


def nep_mlp_grad(params, X, Y, idx, B, grad, work, want_loss=False):
    loss = C.c_float(0.0)
    _check(lib().nep_mlp_grad(_fptr(params), _fptr(X), _fptr(Y), _fptr(idx), B, _fptr(grad),
                              C.byref(loss) if want_loss else None, _fptr(work), _stream()))
    return loss.value if want_loss else None


def nep_mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().nep_mlp_adam(_fptr(params), _fptr(grad), _fptr(m), _fptr(v), step, lr, beta1, beta2, eps,
                              _stream()))


def nep_mlp_features(profiles, rows, ncol, stat_rows, mean, sd, X):
    _check(lib().nep_mlp_features(_fptr(profiles), rows, ncol, _fptr(stat_rows),
                                  0 if stat_rows is None else int(stat_rows.numel()), _fptr(mean), _fptr(sd),
                                  _fptr(X), _stream()))
