"""ctypes binding of librmips: argument marshalling only.

Every step of the computation runs in the library's HIP kernels; PyTorch
provides device memory (inputs, outputs, workspace) and the current stream.
The binding refuses to run without the compiled library.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librmips.so")

RMIPS_OK, RMIPS_EINVAL, RMIPS_EWORKSPACE, RMIPS_ENONFINITE, RMIPS_EUNSUPPORTED, \
    RMIPS_EDEVICE = range(6)
PREC = {"fp32": 0, "bf16": 1, "fp8": 2, "fp8_e4m3": 2, "fp6": 3, "fp6_e2m3": 3, "fp4": 4,
        "fp4_e2m1": 4}
K_MAX, N_MAX, D_MAX = 32, 1024, 256

EXPORTS = [
    "rmips_create", "rmips_destroy", "rmips_last_error", "rmips_set_stream", "rmips_sync",
    "rmips_set_profiling", "rmips_profile_entry",
    "rmips_set_candidate_cap", "rmips_set_batch", "rmips_set_bound_output", "rmips_set_dprime",
    "rmips_set_prepass",
    "rmips_thresholds_workspace_size", "rmips_scores_workspace_size",
    "rmips_topn_workspace_size", "rmips_soft_workspace_size",
    "rmips_thresholds", "rmips_scores", "rmips_topn", "rmips_soft_fwd",
    "rmips_soft_bwd", "rmips_soft_bwd_noalloc", "rmips_soft_fwd_grad", "rmips_soft_scale",
    "rmips_index_size", "rmips_index_workspace_size", "rmips_index_build",
    "rmips_index_topn", "rmips_index_thresholds", "rmips_index_bounds",
    "rmips_budget_index_size", "rmips_budget_workspace_size", "rmips_budget_build",
    "rmips_budget_topn", "rmips_budget_state",
]
BUDGET_KINDS = {"exp": 0, "uniform": 1, "linear": 2, "quadratic": 3}


class RmipsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"librmips status {status}: {msg}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("visited_items", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("cand_pairs", ctypes.c_int64), ("cand_listed", ctypes.c_int64),
                ("overflow_users", ctypes.c_int64),
                ("refine_users", ctypes.c_int64),
                ("recheck_pairs", ctypes.c_int64), ("screened_pairs", ctypes.c_int64),
                ("bound_pairs", ctypes.c_int64), ("thresh_pairs", ctypes.c_int64),
                ("count_pairs", ctypes.c_int64), ("count_launches", ctypes.c_int64),
                ("refine_pairs", ctypes.c_int64),
                ("ms_thresh", ctypes.c_float), ("ms_bound", ctypes.c_float),
                ("ms_count", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("ms_screen", ctypes.c_float), ("ms_count_kernels", ctypes.c_float),
                ("ms_bound_kernel", ctypes.c_float), ("rebound_items", ctypes.c_int64),
                ("rebound_pairs", ctypes.c_int64), ("prepass_dprime", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Budget(ctypes.Structure):
    _fields_ = [("b1", ctypes.c_int64), ("B2", ctypes.c_int64), ("kind", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("gamma", ctypes.c_double)]


class BudgetInfo(ctypes.Structure):
    _fields_ = [("u_prime", ctypes.c_int64), ("u_dprime", ctypes.c_int64),
                ("cert3", ctypes.c_int64), ("cert4", ctypes.c_int64),
                ("scanned4", ctypes.c_int64), ("beta", ctypes.c_double),
                ("ms_total", ctypes.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BudgetQStats(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int64), ("rescanned_users", ctypes.c_int64),
                ("rescan_calls", ctypes.c_int64), ("visited_items", ctypes.c_int64),
                ("processed_items", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("ms_init", ctypes.c_float), ("ms_total", ctypes.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_lock = threading.Lock()


def load():
    """Load librmips.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"librmips is not built ({LIB_PATH} missing); "
                           "run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, f32, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                             ctypes.c_float, ctypes.c_size_t)
    st = ctypes.c_int
    lib.rmips_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
    lib.rmips_create.restype = st
    lib.rmips_destroy.argtypes = [vp]
    lib.rmips_destroy.restype = None
    lib.rmips_last_error.argtypes = [vp]
    lib.rmips_last_error.restype = ctypes.c_char_p
    lib.rmips_set_stream.argtypes = [vp, vp]
    lib.rmips_set_stream.restype = st
    lib.rmips_sync.argtypes = [vp]
    lib.rmips_sync.restype = st
    lib.rmips_set_profiling.argtypes = [vp, i32]
    lib.rmips_set_profiling.restype = st
    lib.rmips_profile_entry.argtypes = [vp, i32, ctypes.c_char_p, i32,
                                        ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
    lib.rmips_profile_entry.restype = st
    lib.rmips_set_candidate_cap.argtypes = [vp, i32]
    lib.rmips_set_candidate_cap.restype = st
    lib.rmips_set_batch.argtypes = [vp, i32, i32]
    lib.rmips_set_batch.restype = st
    lib.rmips_set_bound_output.argtypes = [vp, vp]
    lib.rmips_set_bound_output.restype = st
    lib.rmips_set_dprime.argtypes = [vp, i32]
    lib.rmips_set_dprime.restype = st
    lib.rmips_set_prepass.argtypes = [vp, i32]
    lib.rmips_set_prepass.restype = st
    lib.rmips_thresholds_workspace_size.argtypes = [i64, i64, i32, i32, ctypes.c_int]
    lib.rmips_thresholds_workspace_size.restype = sz
    lib.rmips_scores_workspace_size.argtypes = [i64, i64, i32, ctypes.c_int]
    lib.rmips_scores_workspace_size.restype = sz
    lib.rmips_topn_workspace_size.argtypes = [i64, i64, i32, i32, i32, ctypes.c_int]
    lib.rmips_topn_workspace_size.restype = sz
    lib.rmips_soft_workspace_size.argtypes = [i64, i64, i32]
    lib.rmips_soft_workspace_size.restype = sz
    lib.rmips_thresholds.argtypes = [vp, vp, i64, vp, i64, i32, i32, ctypes.c_int, vp, sz,
                                     vp, vp, vp]
    lib.rmips_thresholds.restype = st
    lib.rmips_scores.argtypes = [vp, vp, i64, vp, vp, vp, vp, i64, i32, ctypes.c_int, vp, sz,
                                 vp]
    lib.rmips_scores.restype = st
    lib.rmips_topn.argtypes = [vp, vp, i64, vp, i64, i32, i32, i32, ctypes.c_int, vp, sz,
                               vp, vp, ctypes.POINTER(Stats)]
    lib.rmips_topn.restype = st
    lib.rmips_soft_fwd.argtypes = [vp, vp, i64, vp, vp, i64, i32, f32, vp, sz, vp]
    lib.rmips_soft_fwd.restype = st
    lib.rmips_soft_bwd.argtypes = [vp, vp, i64, vp, vp, i64, i32, f32, vp, vp, sz, vp]
    lib.rmips_soft_bwd.restype = st
    lib.rmips_soft_bwd_noalloc.argtypes = [vp, vp, i64, vp, vp, i64, i32, f32, vp, vp]
    lib.rmips_soft_bwd_noalloc.restype = st
    lib.rmips_soft_fwd_grad.argtypes = [vp, vp, i64, vp, vp, i64, i32, f32, vp, sz, vp, vp]
    lib.rmips_soft_fwd_grad.restype = st
    lib.rmips_soft_scale.argtypes = [vp, vp, i64, i32, vp, vp]
    lib.rmips_soft_scale.restype = st
    lib.rmips_index_size.argtypes = [i64, i64, i32, i32, ctypes.c_int]
    lib.rmips_index_size.restype = sz
    lib.rmips_index_workspace_size.argtypes = [i64, i64, i32, i32, ctypes.c_int]
    lib.rmips_index_workspace_size.restype = sz
    lib.rmips_index_build.argtypes = [vp, vp, i64, vp, i64, i32, i32, ctypes.c_int, vp, sz,
                                      vp, sz]
    lib.rmips_index_build.restype = st
    lib.rmips_index_topn.argtypes = [vp, vp, i64, vp, i64, i32, i32, ctypes.c_int, vp, sz,
                                     i32, i32, vp, sz, vp, vp, ctypes.POINTER(Stats)]
    lib.rmips_index_topn.restype = st
    lib.rmips_index_thresholds.argtypes = [vp, i64, i64, i32, i32, ctypes.c_int, vp, sz, i32,
                                           vp, vp]
    lib.rmips_index_thresholds.restype = st
    lib.rmips_index_bounds.argtypes = [vp, i64, i64, i32, i32, ctypes.c_int, vp, sz, i32, vp]
    lib.rmips_index_bounds.restype = st
    lib.rmips_budget_index_size.argtypes = [i64, i64, i32, i32]
    lib.rmips_budget_index_size.restype = sz
    lib.rmips_budget_workspace_size.argtypes = [i64, i64, i32, i32, ctypes.c_int]
    lib.rmips_budget_workspace_size.restype = sz
    lib.rmips_budget_build.argtypes = [vp, vp, i64, vp, i64, i32, i32, ctypes.c_int,
                                       ctypes.POINTER(Budget), vp, sz, vp, sz,
                                       ctypes.POINTER(BudgetInfo)]
    lib.rmips_budget_build.restype = st
    lib.rmips_budget_topn.argtypes = [vp, vp, i64, vp, i64, i32, i32, ctypes.c_int, vp, sz,
                                      i32, i32, vp, sz, vp, vp, ctypes.POINTER(BudgetQStats)]
    lib.rmips_budget_topn.restype = st
    lib.rmips_budget_state.argtypes = [vp, i64, i64, i32, i32, vp, sz, vp, vp, vp, vp, vp, vp,
                                       vp, vp, vp]
    lib.rmips_budget_state.restype = st
    _lib = lib
    return lib


_ctx = {}


def _context(device: torch.device):
    """Per-device context, pointed at torch's current stream."""
    lib = load()
    idx = device.index if device.index is not None else torch.cuda.current_device()
    with _lock:
        c = _ctx.get(idx)
        if c is None:
            h = ctypes.c_void_p()
            s = lib.rmips_create(ctypes.byref(h), idx, None)
            if s != RMIPS_OK:
                raise RmipsError(s, f"rmips_create failed on device {idx}")
            c = h
            _ctx[idx] = c
    stream = torch.cuda.current_stream(idx).cuda_stream
    lib.rmips_set_stream(c, ctypes.c_void_p(stream))
    return c


def _check(ctx, status):
    if status != RMIPS_OK:
        msg = load().rmips_last_error(ctx)
        raise RmipsError(status, msg.decode() if msg else "")


def _dev_f32(x, name):
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32
            and x.is_contiguous() and x.dim() == 2):
        raise ValueError(f"{name} must be a contiguous 2-D float32 CUDA tensor")
    return x


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _workspace(nbytes, device):
    if nbytes == 0:
        raise RmipsError(RMIPS_EINVAL, "invalid sizes")
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def sync(device=None):
    """rmips_sync: wait for the stream and raise if an input check of an
    earlier thresholds / scores call failed."""
    dev = device or torch.device("cuda", torch.cuda.current_device())
    ctx = _context(dev)
    _check(ctx, load().rmips_sync(ctx))


def set_profiling(on, device=None):
    """rmips_set_profiling on the device's context (on=True clears the totals)."""
    dev = device or torch.device("cuda", torch.cuda.current_device())
    ctx = _context(dev)
    _check(ctx, load().rmips_set_profiling(ctx, 1 if on else 0))


def profile(device=None):
    """Per-kernel totals since profiling was switched on: a list of
    (name, launches, total ms) in the order the kernels first ran."""
    dev = device or torch.device("cuda", torch.cuda.current_device())
    lib = load()
    ctx = _context(dev)
    out = []
    buf = ctypes.create_string_buffer(128)
    nl, ms = ctypes.c_int64(), ctypes.c_double()
    i = 0
    while lib.rmips_profile_entry(ctx, i, buf, 128, ctypes.byref(nl), ctypes.byref(ms)) == RMIPS_OK:
        out.append((buf.value.decode(), int(nl.value), float(ms.value)))
        i += 1
    return out


def thresholds(U, P, k, prec="fp32", with_topk=False, cand_cap=None, check=True):
    """tau (float64), tau_id (int32) [, topk ids (int32, n x k)] on U's device.
    check=True waits for the call (rmips_sync) and raises on bad input;
    check=False returns at once (the check is reported by sync())."""
    U, P = _dev_f32(U, "U"), _dev_f32(P, "P")
    n, d = U.shape
    m = P.shape[0]
    if P.shape[1] != d:
        raise ValueError("U and P must have the same number of columns")
    lib = load()
    ctx = _context(U.device)
    lib.rmips_set_candidate_cap(ctx, int(cand_cap or 0))
    p = PREC[prec]
    ws = _workspace(lib.rmips_thresholds_workspace_size(n, m, d, k, p), U.device)
    tau = torch.empty(n, dtype=torch.float64, device=U.device)
    tid = torch.empty(n, dtype=torch.int32, device=U.device)
    topk = torch.empty((n, k), dtype=torch.int32, device=U.device) if with_topk else None
    status = lib.rmips_thresholds(ctx, _ptr(U), n, _ptr(P), m, d, k, p, _ptr(ws),
                                  ws.numel(), _ptr(tau), _ptr(tid), _ptr(topk))
    lib.rmips_set_candidate_cap(ctx, 0)
    _check(ctx, status)
    if check:
        _check(ctx, lib.rmips_sync(ctx))
    return (tau, tid, topk) if with_topk else (tau, tid)


def scores(U, tau, tau_id, Q, q_ids=None, prec="fp32", check=True):
    """|T_k(q)| for each row of Q (int32 on U's device); check as in
    thresholds()."""
    U, Q = _dev_f32(U, "U"), _dev_f32(Q, "Q")
    n, d = U.shape
    nq = Q.shape[0]
    if tau.dtype != torch.float64 or tau_id.dtype != torch.int32:
        raise ValueError("tau must be float64 and tau_id int32")
    if q_ids is not None and (q_ids.dtype != torch.int32 or q_ids.numel() != nq):
        raise ValueError("q_ids must be int32 with one entry per query")
    lib = load()
    ctx = _context(U.device)
    p = PREC[prec]
    ws = _workspace(lib.rmips_scores_workspace_size(n, nq, d, p), U.device)
    out = torch.empty(nq, dtype=torch.int32, device=U.device)
    _check(ctx, lib.rmips_scores(ctx, _ptr(U), n, _ptr(tau.contiguous()),
                                 _ptr(tau_id.contiguous()), _ptr(Q),
                                 _ptr(q_ids.contiguous()) if q_ids is not None else None,
                                 nq, d, p, _ptr(ws), ws.numel(), _ptr(out)))
    if check:
        _check(ctx, lib.rmips_sync(ctx))
    return out


def topn_workspace(n, m, d, k, N, prec="fp32", device=None):
    lib = load()
    return _workspace(lib.rmips_topn_workspace_size(n, m, d, k, N, PREC[prec]),
                      device or torch.device("cuda"))


def topn(U, P, k, N, prec="fp32", ws=None, cand_cap=None, batch=None, bound_out=None,
         dprime=None, prepass=None):
    """Top-N item ids and scores (host int32 numpy arrays) and a stats dict.
    bound_out: optional int32 device tensor of m entries that receives the
    Eq. (3)/(6) bound count of every item (caller order).  dprime: the split
    dimension d' of that bound (None or 0: d' = d; 1..62: a rotation onto
    the users' top-d' eigenvectors).  prepass: d' of the rotated pre-pass
    before the d' = d bound (None: automatic, 0: none, 1..62)."""
    import numpy as np
    U, P = _dev_f32(U, "U"), _dev_f32(P, "P")
    n, d = U.shape
    m = P.shape[0]
    lib = load()
    ctx = _context(U.device)
    p = PREC[prec]
    need = lib.rmips_topn_workspace_size(n, m, d, k, N, p)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, U.device)
    ids = np.empty(N, np.int32)
    sc = np.empty(N, np.int32)
    st = Stats()
    # the knobs are set only when asked for, and reset after the call (d'
    # first: an invalid value then leaves nothing set)
    if bound_out is not None and (bound_out.dtype != torch.int32 or bound_out.numel() != m
                                  or not bound_out.is_cuda or not bound_out.is_contiguous()):
        raise ValueError("bound_out must be a contiguous int32 device tensor of m entries")
    if dprime:
        _check(ctx, lib.rmips_set_dprime(ctx, int(dprime)))
    if prepass is not None:
        s = lib.rmips_set_prepass(ctx, int(prepass))
        if s != 0:
            if dprime:
                lib.rmips_set_dprime(ctx, 0)
            _check(ctx, s)
    if bound_out is not None:
        lib.rmips_set_bound_output(ctx, _ptr(bound_out))
    if cand_cap:
        lib.rmips_set_candidate_cap(ctx, int(cand_cap))
    if batch:
        lib.rmips_set_batch(ctx, int(batch[0]), int(batch[1]))
    status = lib.rmips_topn(ctx, _ptr(U), n, _ptr(P), m, d, k, N, p, _ptr(ws), ws.numel(),
                            ids.ctypes.data_as(ctypes.c_void_p),
                            sc.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st))
    if cand_cap:
        lib.rmips_set_candidate_cap(ctx, 0)
    if batch:
        lib.rmips_set_batch(ctx, 0, 0)
    if dprime:
        lib.rmips_set_dprime(ctx, 0)
    if prepass is not None:
        lib.rmips_set_prepass(ctx, -1)
    if bound_out is not None:
        lib.rmips_set_bound_output(ctx, None)
    _check(ctx, status)
    return ids, sc, st.as_dict()


def _soft_args(U, tau, Q, T):
    U, Q = _dev_f32(U, "U"), _dev_f32(Q, "Q")
    if tau.dtype != torch.float32 or tau.dim() != 1 or tau.numel() != U.shape[0]:
        raise ValueError("tau must be a float32 vector with one entry per user")
    if U.shape[1] != Q.shape[1]:
        raise ValueError("U and Q must have the same number of columns")
    return U, tau.contiguous(), Q, float(T)


def soft_fwd(U, tau, Q, T):
    """S[i] = sum_u sigmoid((u . q_i - tau_u) / T), float32 on U's device."""
    U, tau, Q, T = _soft_args(U, tau, Q, T)
    n, d = U.shape
    nq = Q.shape[0]
    lib = load()
    ctx = _context(U.device)
    ws = _workspace(lib.rmips_soft_workspace_size(n, nq, d), U.device)
    S = torch.empty(nq, dtype=torch.float32, device=U.device)
    _check(ctx, lib.rmips_soft_fwd(ctx, _ptr(U), n, _ptr(tau), _ptr(Q), nq, d, T, _ptr(ws),
                                   ws.numel(), _ptr(S)))
    return S


def soft_bwd(U, tau, Q, T, dS):
    """dQ[i] = dS[i] * sum_u sigmoid'(z_ui) / T * u, float32 on U's device."""
    U, tau, Q, T = _soft_args(U, tau, Q, T)
    n, d = U.shape
    nq = Q.shape[0]
    dS = dS.to(torch.float32).contiguous()
    lib = load()
    ctx = _context(U.device)
    ws = _workspace(lib.rmips_soft_workspace_size(n, nq, d), U.device)
    dQ = torch.empty((nq, d), dtype=torch.float32, device=U.device)
    _check(ctx, lib.rmips_soft_bwd(ctx, _ptr(U), n, _ptr(tau), _ptr(Q), nq, d, T, _ptr(dS),
                                   _ptr(ws), ws.numel(), _ptr(dQ)))
    return dQ


class Index:
    """A k_max index (rmips_index_build) over device tensors U and P: each
    user's kmax largest values and the bound of every item for every
    k <= kmax, held in a device buffer; topn() answers any (k, N)."""

    def __init__(self, U, P, kmax, prec="fp32", dprime=None):
        U, P = _dev_f32(U, "U"), _dev_f32(P, "P")
        if P.shape[1] != U.shape[1]:
            raise ValueError("U and P must have the same number of columns")
        self.U, self.P = U, P
        self.n, self.d = U.shape
        self.m = P.shape[0]
        self.kmax, self.prec, self.p = int(kmax), prec, PREC[prec]
        lib = load()
        ctx = _context(U.device)
        self.buf = _workspace(lib.rmips_index_size(self.n, self.m, self.d, self.kmax, self.p),
                              U.device)
        self.ws = _workspace(lib.rmips_index_workspace_size(self.n, self.m, self.d, self.kmax,
                                                            self.p), U.device)
        if dprime:
            _check(ctx, lib.rmips_set_dprime(ctx, int(dprime)))
        try:
            _check(ctx, lib.rmips_index_build(ctx, _ptr(U), self.n, _ptr(P), self.m, self.d,
                                              self.kmax, self.p, _ptr(self.buf),
                                              self.buf.numel(), _ptr(self.ws), self.ws.numel()))
        finally:
            if dprime:
                lib.rmips_set_dprime(ctx, 0)

    def _args(self):
        return (self.n, self.m, self.d, self.kmax, self.p, _ptr(self.buf), self.buf.numel())

    def topn(self, k, N):
        """Top-N ids and scores (host int32 numpy arrays) for this k, and stats."""
        import numpy as np
        lib = load()
        ctx = _context(self.U.device)
        ids = np.empty(N, np.int32)
        sc = np.empty(N, np.int32)
        st = Stats()
        _check(ctx, lib.rmips_index_topn(ctx, _ptr(self.U), self.n, _ptr(self.P), self.m,
                                         self.d, self.kmax, self.p, _ptr(self.buf),
                                         self.buf.numel(), int(k), int(N), _ptr(self.ws),
                                         self.ws.numel(), ids.ctypes.data_as(ctypes.c_void_p),
                                         sc.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st)))
        return ids, sc, st.as_dict()

    def thresholds(self, k):
        """(tau, tau_id) of S_k on the device."""
        lib = load()
        ctx = _context(self.U.device)
        tau = torch.empty(self.n, dtype=torch.float64, device=self.U.device)
        tid = torch.empty(self.n, dtype=torch.int32, device=self.U.device)
        _check(ctx, lib.rmips_index_thresholds(ctx, *self._args(), int(k), _ptr(tau), _ptr(tid)))
        return tau, tid

    def bounds(self, k):
        """uscore_k of every item (caller order, int32 on the device)."""
        lib = load()
        ctx = _context(self.U.device)
        out = torch.empty(self.m, dtype=torch.int32, device=self.U.device)
        _check(ctx, lib.rmips_index_bounds(ctx, *self._args(), int(k), _ptr(out)))
        return out


class BudgetIndex:
    """The budgeted index (rmips_budget_build: Alg. 1 under an inner-product
    budget, Sec. 4.2) over device tensors U and P; topn() runs Alg. 2 with
    Inc-RMIPS (Sec. 4.3) for any k <= kmax.  b1 = B1/n positions per user in
    step (3), B2 the dynamic budget, kind one of "exp" (Eq. 4, beta from
    Eq. 5), "uniform", "linear", "quadratic"."""

    def __init__(self, U, P, kmax, b1, B2, kind="exp", alpha=1.0, gamma=0.0, prec="fp32"):
        U, P = _dev_f32(U, "U"), _dev_f32(P, "P")
        if P.shape[1] != U.shape[1]:
            raise ValueError("U and P must have the same number of columns")
        self.U, self.P = U, P
        self.n, self.d = U.shape
        self.m = P.shape[0]
        self.kmax, self.prec, self.p = int(kmax), prec, PREC[prec]
        lib = load()
        ctx = _context(U.device)
        self.buf = _workspace(lib.rmips_budget_index_size(self.n, self.m, self.d, self.kmax),
                              U.device)
        self.ws = _workspace(lib.rmips_budget_workspace_size(self.n, self.m, self.d, self.kmax,
                                                             self.p), U.device)
        bud = Budget(int(b1), int(B2), BUDGET_KINDS[kind], float(alpha), float(gamma))
        info = BudgetInfo()
        _check(ctx, lib.rmips_budget_build(ctx, _ptr(U), self.n, _ptr(P), self.m, self.d,
                                           self.kmax, self.p, ctypes.byref(bud), _ptr(self.buf),
                                           self.buf.numel(), _ptr(self.ws), self.ws.numel(),
                                           ctypes.byref(info)))
        self.info = info.as_dict()

    def topn(self, k, N):
        """Top-N ids and scores (host int32 numpy arrays) for this k, and stats."""
        import numpy as np
        lib = load()
        ctx = _context(self.U.device)
        ids = np.empty(N, np.int32)
        sc = np.empty(N, np.int32)
        st = BudgetQStats()
        _check(ctx, lib.rmips_budget_topn(ctx, _ptr(self.U), self.n, _ptr(self.P), self.m,
                                          self.d, self.kmax, self.p, _ptr(self.buf),
                                          self.buf.numel(), int(k), int(N), _ptr(self.ws),
                                          self.ws.numel(), ids.ctypes.data_as(ctypes.c_void_p),
                                          sc.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st)))
        return ids, sc, st.as_dict()

    def state(self):
        """The index's per-user and per-item state as device tensors: order,
        pos, lam, Av, Aj, key, rank, b2, uscore (kmax x m)."""
        lib = load()
        ctx = _context(self.U.device)
        dev = self.U.device
        n, m, kx = self.n, self.m, self.kmax
        out = {
            "order": torch.empty(m, dtype=torch.int32, device=dev),
            "pos": torch.empty(n, dtype=torch.int32, device=dev),
            "lam": torch.empty(n, dtype=torch.float64, device=dev),
            "Av": torch.empty((n, kx), dtype=torch.float64, device=dev),
            "Aj": torch.empty((n, kx), dtype=torch.int32, device=dev),
            "key": torch.empty(n, dtype=torch.int32, device=dev),
            "rank": torch.empty(n, dtype=torch.int32, device=dev),
            "b2": torch.empty(n, dtype=torch.int64, device=dev),
            "uscore": torch.empty((kx, m), dtype=torch.int32, device=dev),
        }
        _check(ctx, lib.rmips_budget_state(ctx, n, m, self.d, kx, _ptr(self.buf),
                                           self.buf.numel(), *[_ptr(out[k]) for k in (
                                               "order", "pos", "lam", "Av", "Aj", "key", "rank",
                                               "b2", "uscore")]))
        return out


def soft_fwd_grad(U, tau, Q, T):
    """(S, G): the relaxed score and its unscaled gradient sum_u sigmoid'/T u,
    float32 on U's device, in one pass."""
    U, tau, Q, T = _soft_args(U, tau, Q, T)
    n, d = U.shape
    nq = Q.shape[0]
    lib = load()
    ctx = _context(U.device)
    ws = _workspace(lib.rmips_soft_workspace_size(n, nq, d), U.device)
    S = torch.empty(nq, dtype=torch.float32, device=U.device)
    G = torch.empty((nq, d), dtype=torch.float32, device=U.device)
    _check(ctx, lib.rmips_soft_fwd_grad(ctx, _ptr(U), n, _ptr(tau), _ptr(Q), nq, d, T,
                                        _ptr(ws), ws.numel(), _ptr(S), _ptr(G)))
    return S, G


def soft_scale(G, dS):
    """dQ = dS[:, None] * G in the library's kernel (float32, device)."""
    G = G.contiguous()
    nq, d = G.shape
    dS = dS.to(torch.float32).contiguous()
    lib = load()
    ctx = _context(G.device)
    dQ = torch.empty_like(G)
    _check(ctx, lib.rmips_soft_scale(ctx, _ptr(G), nq, d, _ptr(dS), _ptr(dQ)))
    return dQ


def soft_bwd_noalloc(U, tau, Q, T, dS, out=None):
    """rmips_soft_bwd_noalloc: the gradient with the library's static scratch
    (no workspace); `out` (nq x d float32, device) may be given."""
    U, tau, Q, T = _soft_args(U, tau, Q, T)
    n, d = U.shape
    nq = Q.shape[0]
    dS = dS.to(torch.float32).contiguous()
    lib = load()
    ctx = _context(U.device)
    dQ = out if out is not None else torch.empty((nq, d), dtype=torch.float32,
                                                 device=U.device)
    _check(ctx, lib.rmips_soft_bwd_noalloc(ctx, _ptr(U), n, _ptr(tau), _ptr(Q), nq, d, T,
                                           _ptr(dS), _ptr(dQ)))
    return dQ


class SoftScore(torch.autograd.Function):
    """Relaxed score S(Q): the forward pass forms S and its unscaled gradient
    in one pass over the users (rmips_soft_fwd_grad), the backward pass scales
    the gradient by the upstream dS (rmips_soft_scale).  The gradient flows to
    Q only (users and thresholds are data)."""

    @staticmethod
    def forward(ctx, Q, U, tau, T):
        S, G = soft_fwd_grad(U, tau, Q.contiguous(), T)
        ctx.save_for_backward(G)
        return S

    @staticmethod
    def backward(ctx, dS):
        (G,) = ctx.saved_tensors
        return soft_scale(G, dS), None, None, None
