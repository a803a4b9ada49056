"""Python binding of libsk (Sinkhorn preprocessing for optimal assignment on MI355X).

Argument marshalling only: every step of the path runs in libsk's HIP kernels
or its host C++ solver. PyTorch supplies device memory (tensors as buffers) and
the HIP stream; nothing else. The binding fails loudly when libsk.so is
missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsk.so")

SK_OK, SK_EINVAL, SK_ENOMEM, SK_ENOCONV, SK_EINFEASIBLE, SK_EAGAIN, SK_EDEVICE, SK_ENOSUPPORT = range(8)
STATUS_NAMES = ["SK_OK", "SK_EINVAL", "SK_ENOMEM", "SK_ENOCONV", "SK_EINFEASIBLE", "SK_EAGAIN",
                "SK_EDEVICE", "SK_ENOSUPPORT"]
STORAGE = {"i16": 0, "bf16": 1, "f32": 2}
MAX_LADDER = 32
SENTINEL = -32768

EXPORTS = ["sk_potentials_bytes", "sk_arena_bytes", "sk_create", "sk_destroy", "sk_last_error",
           "sk_scale", "sk_prune", "sk_solve_reduced", "sk_submit", "sk_poll", "sk_completed", "sk_scale_batch",
           "sk_batch_arena_bytes", "sk_profile_enable", "sk_profile_read", "sk_set_tile_table",
           "sk_solve", "sk_solve_arena_bytes", "sk_scale_static", "sk_real_arena_bytes",
           "sk_scale_real", "sk_solve_real", "sk_solve_reduced_real"]
TILE_TABLE = os.path.join(HERE, "tile_table_gfx950.json")


class SkError(RuntimeError):
    def __init__(self, status, message=""):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")


class Params(ctypes.Structure):
    _fields_ = [("p_ladder", ctypes.c_int32 * MAX_LADDER), ("n_p", ctypes.c_int32),
                ("tol", ctypes.c_double), ("max_iters_per_stage", ctypes.c_int64),
                ("check_every", ctypes.c_int32), ("threshold", ctypes.c_double),
                ("storage", ctypes.c_int32), ("opt_ratio", ctypes.c_double),
                ("warm_start", ctypes.c_int32), ("fused", ctypes.c_int32),
                ("deform_a", ctypes.c_double), ("method", ctypes.c_int32),
                ("prescale", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("residual_fp32", ctypes.c_double), ("residual_fp64", ctypes.c_double),
                ("col_residual_fp64", ctypes.c_double),
                ("residual_exact_fp64", ctypes.c_double),
                ("col_residual_exact_fp64", ctypes.c_double), ("ub", ctypes.c_double),
                ("iters_total", ctypes.c_int64), ("iters_stage", ctypes.c_int64 * MAX_LADDER),
                ("p_final", ctypes.c_int32), ("stages_capped", ctypes.c_int32),
                ("nnz_kept", ctypes.c_int64), ("absorbs", ctypes.c_int32),
                ("seconds", ctypes.c_double), ("log_gamma", ctypes.c_double),
                ("threshold_used", ctypes.c_double), ("stages_evaluated", ctypes.c_int32),
                ("optimal_proved", ctypes.c_int32), ("p_scale", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "iters_stage"}
        d["iters_stage"] = list(self.iters_stage)
        return d


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("w", ctypes.c_void_p)]


CSRReal = CSR  # same layout; w points to float32


_lib = None
loaded_tile_table = []  # (n_max, seg_rows) entries the binding passed to sk_set_tile_table


def lib():
    """Loads libsk.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__; __graft_entry__.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.sk_potentials_bytes.argtypes = [i32]
        L.sk_potentials_bytes.restype = sz
        L.sk_arena_bytes.argtypes = [i32, i32]
        L.sk_arena_bytes.restype = sz
        L.sk_batch_arena_bytes.argtypes = [i32, ctypes.POINTER(i32), i32]
        L.sk_batch_arena_bytes.restype = sz
        L.sk_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, vp, sz]
        L.sk_create.restype = ctypes.c_int
        L.sk_destroy.argtypes = [vp]
        L.sk_destroy.restype = ctypes.c_int
        L.sk_last_error.argtypes = [vp]
        L.sk_last_error.restype = ctypes.c_char_p
        L.sk_scale.argtypes = [vp, vp, i32, ctypes.POINTER(Params), vp, ctypes.POINTER(Report)]
        L.sk_scale.restype = ctypes.c_int
        L.sk_scale_static.argtypes = [vp, vp, i32, ctypes.POINTER(Params), vp,
                                      ctypes.POINTER(Report)]
        L.sk_scale_static.restype = ctypes.c_int
        L.sk_real_arena_bytes.argtypes = [i32, i64]
        L.sk_real_arena_bytes.restype = sz
        L.sk_scale_real.argtypes = [vp, vp, i32, ctypes.POINTER(Params), vp, ctypes.POINTER(Report)]
        L.sk_scale_real.restype = ctypes.c_int
        L.sk_solve_real.argtypes = [vp, vp, i32, ctypes.POINTER(Params), vp, ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(Report)]
        L.sk_solve_real.restype = ctypes.c_int
        L.sk_solve_reduced_real.argtypes = [ctypes.POINTER(CSRReal), ctypes.POINTER(i32),
                                            ctypes.POINTER(ctypes.c_double)]
        L.sk_solve_reduced_real.restype = ctypes.c_int
        L.sk_scale_batch.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(i32),
                                     ctypes.POINTER(Params), ctypes.POINTER(vp),
                                     ctypes.POINTER(Report)]
        L.sk_scale_batch.restype = ctypes.c_int
        L.sk_prune.argtypes = [vp, vp, i32, vp, ctypes.POINTER(Params), ctypes.POINTER(CSR)]
        L.sk_prune.restype = ctypes.c_int
        L.sk_completed.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), i32]
        L.sk_completed.restype = i32
        L.sk_solve_reduced.argtypes = [ctypes.POINTER(CSR), ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.sk_solve_reduced.restype = ctypes.c_int
        L.sk_solve.argtypes = [vp, vp, i32, ctypes.POINTER(Params), vp, ctypes.POINTER(i32),
                               ctypes.POINTER(i64), ctypes.POINTER(Report)]
        L.sk_solve.restype = ctypes.c_int
        L.sk_solve_arena_bytes.argtypes = [i32, i32, i64]
        L.sk_solve_arena_bytes.restype = sz
        L.sk_submit.argtypes = [vp, vp, i32, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_uint64)]
        L.sk_submit.restype = ctypes.c_int
        L.sk_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(i64),
                              ctypes.POINTER(Report)]
        L.sk_poll.restype = ctypes.c_int
        L.sk_profile_enable.argtypes = [vp, ctypes.c_int]
        L.sk_profile_enable.restype = ctypes.c_int
        L.sk_profile_read.argtypes = [vp, ctypes.POINTER(KernelStat), i32]
        L.sk_profile_read.restype = i32
        L.sk_set_tile_table.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32), i32]
        L.sk_set_tile_table.restype = ctypes.c_int
        _lib = L
        if os.path.exists(TILE_TABLE) and not os.environ.get("SK_NO_TILE_TABLE"):
            load_tile_table(TILE_TABLE)
    return _lib


def set_tile_table(entries):
    """entries: list of (n_max, seg_rows), n_max ascending; [] = built-in rule."""
    global loaded_tile_table
    nm = (ctypes.c_int32 * max(len(entries), 1))(*[int(a) for a, _ in entries])
    sr = (ctypes.c_int32 * max(len(entries), 1))(*[int(b) for _, b in entries])
    st = lib().sk_set_tile_table(nm, sr, len(entries))
    if st != SK_OK:
        raise SkError(st, "sk_set_tile_table")
    loaded_tile_table = [(int(a), int(b)) for a, b in entries]


def load_tile_table(path):
    import json
    with open(path) as f:
        tab = json.load(f)
    set_tile_table([(e["n_max"], e["seg_rows"]) for e in tab["entries"]])


def make_params(ladder, tol=1e-5, max_iters=20000, check_every=32, threshold=1e-4,
                storage="i16", opt_ratio=0.0, warm_start=False, fused=False,
                deform_a=0.0, method="sinkhorn", prescale=False) -> Params:
    p = Params()
    ladder = [int(x) for x in ladder]
    if not 1 <= len(ladder) <= MAX_LADDER:
        raise ValueError("ladder length must be in [1, 32]")
    for k, v in enumerate(ladder):
        p.p_ladder[k] = v
    p.n_p = len(ladder)
    p.tol = float(tol)
    p.max_iters_per_stage = int(max_iters)
    p.check_every = int(check_every)
    p.threshold = float(threshold)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.opt_ratio = float(opt_ratio)
    p.warm_start = 1 if warm_start else 0
    p.fused = 1 if fused else 0
    p.deform_a = float(deform_a)
    p.method = {"sinkhorn": 0, "newton": 1}[method] if isinstance(method, str) else int(method)
    p.prescale = 1 if prescale else 0
    return p


def paper_params(n, ladder=None, opt_ratio=2.0, max_iters=100000, check_every=32) -> Params:
    """Algorithm alg:alg1's defaults (Section 4.2): p0 = 100 raised by 50 per
    round on the prescaled matrix (Section 4.1.1), eps = t = 1/n; the
    experiments' required ratio is about 2. The ladder holds the 32 rounds
    p = 100, 150, ..., 1650 unless given."""
    lad = ladder if ladder is not None else [100 + 50 * k for k in range(MAX_LADDER)]
    return make_params(lad, tol=1.0 / n, max_iters=max_iters, check_every=check_every,
                       threshold=1.0 / n, opt_ratio=opt_ratio, prescale=True)


def potentials_bytes(n):
    return int(lib().sk_potentials_bytes(int(n)))


def split_potentials(pot, n):
    """(log u, log v) as float64 numpy arrays from a potentials buffer (host copy)."""
    raw = pot.detach().cpu().numpy() if hasattr(pot, "detach") else np.asarray(pot)
    raw = raw.view(np.uint8)
    F = raw[0:4 * n].view(np.int32).astype(np.float64)
    phi = raw[4 * n:8 * n].view(np.float32).astype(np.float64)
    G = raw[8 * n:12 * n].view(np.int32).astype(np.float64)
    gam = raw[12 * n:16 * n].view(np.float32).astype(np.float64)
    return F + phi, G + gam


def pack_potentials(log_u, log_v):
    """Inverse of split_potentials: bytes of (F, phi, G, gam) as a uint8 numpy array."""
    log_u = np.asarray(log_u, dtype=np.float64)
    log_v = np.asarray(log_v, dtype=np.float64)
    F = np.rint(log_u)
    G = np.rint(log_v)
    parts = [F.astype(np.int32), (log_u - F).astype(np.float32), G.astype(np.int32),
             (log_v - G).astype(np.float32)]
    return np.concatenate([a.view(np.uint8) for a in parts])


def solve_reduced(row_ptr, col, w, n):
    """Exact max-weight perfect matching of a host CSR instance.
    Returns (perm, weight); raises SkError(SK_EINFEASIBLE) without a matching."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.int16)
    csr = CSR(int(n), int(row_ptr[-1]) if len(row_ptr) else 0, row_ptr.ctypes.data,
              col.ctypes.data if col.size else None, w.ctypes.data if w.size else None)
    perm = np.empty(int(n), dtype=np.int32)
    weight = ctypes.c_int64(0)
    st = lib().sk_solve_reduced(ctypes.byref(csr),
                                perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                ctypes.byref(weight))
    if st != SK_OK:
        raise SkError(st, "sk_solve_reduced")
    return perm, weight.value


def solve_reduced_real(row_ptr, col, w, n):
    """Exact max-weight perfect matching of a host CSR instance with real
    (float32) weights. Returns (perm, weight); raises SkError(SK_EINFEASIBLE)
    without a matching."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    csr = CSRReal(int(n), int(row_ptr[-1]) if len(row_ptr) else 0, row_ptr.ctypes.data,
                  col.ctypes.data if col.size else None, w.ctypes.data if w.size else None)
    perm = np.empty(int(n), dtype=np.int32)
    weight = ctypes.c_double(0.0)
    st = lib().sk_solve_reduced_real(ctypes.byref(csr),
                                     perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     ctypes.byref(weight))
    if st != SK_OK:
        raise SkError(st, "sk_solve_reduced_real")
    return perm, weight.value


@dataclass
class Result:
    status: int
    report: dict
    potentials: object  # torch uint8 tensor on the device


class Context:
    """A libsk context with a device arena allocated through torch."""

    def __init__(self, device=0, arena_bytes=64 << 20, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ptr = None
        self.arena = None
        self._alloc(int(arena_bytes))

    def _alloc(self, nbytes):
        torch = self.torch
        if self._ptr is not None:
            self.torch.cuda.synchronize(self.device)
            lib().sk_destroy(self._ptr)
            self._ptr = None
        self.arena = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=self.device)
        ptr = ctypes.c_void_p()
        st = lib().sk_create(ctypes.byref(ptr), self.device.index or 0,
                             ctypes.c_void_p(self.stream.cuda_stream),
                             ctypes.c_void_p(self.arena.data_ptr()), self.arena.numel())
        if st != SK_OK:
            raise SkError(st, "sk_create")
        self._ptr = ptr
        if getattr(self, "_profiling", False):
            # a larger arena means a new library context: timing stays on
            # (launches timed before the regrow are not carried over)
            self._check(lib().sk_profile_enable(self._ptr, 1), "sk_profile_enable")

    def ensure_arena(self, nbytes):
        if self.arena is None or self.arena.numel() < nbytes:
            self._alloc(int(nbytes))

    def close(self):
        if self._ptr is not None:
            lib().sk_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return lib().sk_last_error(self._ptr).decode()

    def _check(self, st, what, ok=(SK_OK,)):
        if st not in ok:
            raise SkError(st, f"{what}: {self.last_error()}")
        return st

    def profile(self, enable=True):
        """Turns HIP-event timing of every launch on/off (and resets it)."""
        self._check(lib().sk_profile_enable(self._ptr, 1 if enable else 0), "sk_profile_enable")
        self._profiling = bool(enable)

    def profile_read(self):
        """{kernel name: (launches, total milliseconds)} since the last enable."""
        buf = (KernelStat * 32)()
        k = lib().sk_profile_read(self._ptr, buf, 32)
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
                for i in range(min(k, 32))}

    def new_potentials(self, n):
        return self.torch.zeros(potentials_bytes(n), dtype=self.torch.uint8, device=self.device)

    def scale(self, W, params, potentials=None):
        """W: int16 CUDA tensor (n, n), contiguous. Returns Result; status
        SK_OK or SK_ENOCONV (a capped stage), other statuses raise."""
        assert W.dtype == self.torch.int16 and W.is_cuda and W.is_contiguous()
        n = W.shape[0]
        self.ensure_arena(lib().sk_arena_bytes(n, params.storage))
        pot = potentials if potentials is not None else self.new_potentials(n)
        rep = Report()
        st = lib().sk_scale(self._ptr, ctypes.c_void_p(W.data_ptr()), n, ctypes.byref(params),
                            ctypes.c_void_p(pot.data_ptr()), ctypes.byref(rep))
        self._check(st, "sk_scale", ok=(SK_OK, SK_ENOCONV))
        return Result(st, rep.as_dict(), pot)

    def scale_static(self, W, params, potentials=None):
        """As scale(), through sk_scale_static: the library's static device
        scratch instead of the context's arena (no device allocation)."""
        assert W.dtype == self.torch.int16 and W.is_cuda and W.is_contiguous()
        n = W.shape[0]
        pot = potentials if potentials is not None else self.new_potentials(n)
        rep = Report()
        st = lib().sk_scale_static(self._ptr, ctypes.c_void_p(W.data_ptr()), n,
                                   ctypes.byref(params), ctypes.c_void_p(pot.data_ptr()),
                                   ctypes.byref(rep))
        self._check(st, "sk_scale_static", ok=(SK_OK, SK_ENOCONV))
        return Result(st, rep.as_dict(), pot)

    def scale_real(self, W, params, potentials=None):
        """Real-valued log-weights: W float32 CUDA tensor (n, n), -inf for a
        zero entry. Returns Result; status SK_OK or SK_ENOCONV."""
        assert W.dtype == self.torch.float32 and W.is_cuda and W.is_contiguous()
        n = int(W.shape[0])
        self.ensure_arena(lib().sk_real_arena_bytes(n, 0))
        pot = potentials if potentials is not None else self.new_potentials(n)
        rep = Report()
        st = lib().sk_scale_real(self._ptr, ctypes.c_void_p(W.data_ptr()), n, ctypes.byref(params),
                                 ctypes.c_void_p(pot.data_ptr()), ctypes.byref(rep))
        self._check(st, "sk_scale_real", ok=(SK_OK, SK_ENOCONV))
        return Result(st, rep.as_dict(), pot)

    def solve_real(self, W, params, potentials=None, max_kept=None):
        """Algorithm alg:alg1 on real-valued log-weights through sk_solve_real
        (see paper_params for the paper's defaults). Returns a dict as
        solve(); weight is a float."""
        assert W.dtype == self.torch.float32 and W.is_cuda and W.is_contiguous()
        n = int(W.shape[0])
        kept = int(max_kept) if max_kept is not None else n * n
        pot = potentials if potentials is not None else self.new_potentials(n)
        perm = np.empty(n, dtype=np.int32)
        self.ensure_arena(lib().sk_real_arena_bytes(n, kept))
        weight = ctypes.c_double(0.0)
        rep = Report()
        st = lib().sk_solve_real(self._ptr, ctypes.c_void_p(W.data_ptr()), n, ctypes.byref(params),
                                 ctypes.c_void_p(pot.data_ptr()),
                                 perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 ctypes.byref(weight), ctypes.byref(rep))
        self._check(st, "sk_solve_real", ok=(SK_OK, SK_ENOCONV, SK_EINFEASIBLE))
        r = rep.as_dict()
        out = dict(status=st, report=r, nnz=int(r["nnz_kept"]), potentials=pot)
        if st == SK_EINFEASIBLE:
            out.update(perm=None, weight=None, log_gamma=None)
        else:
            out.update(perm=perm, weight=float(weight.value), log_gamma=r["log_gamma"])
        return out

    def scale_batch(self, Ws, params, potentials=None):
        """Ws: list of int16 CUDA tensors. Returns list of Result (shared status)."""
        count = len(Ws)
        ns = (ctypes.c_int32 * count)(*[int(w.shape[0]) for w in Ws])
        self.ensure_arena(lib().sk_batch_arena_bytes(count, ns, params.storage))
        pots = potentials if potentials is not None else [self.new_potentials(int(w.shape[0])) for w in Ws]
        wp = (ctypes.c_void_p * count)(*[w.data_ptr() for w in Ws])
        pp = (ctypes.c_void_p * count)(*[p.data_ptr() for p in pots])
        reps = (Report * count)()
        st = lib().sk_scale_batch(self._ptr, count, wp, ns, ctypes.byref(params), pp, reps)
        self._check(st, "sk_scale_batch", ok=(SK_OK, SK_ENOCONV))
        return [Result(st, reps[k].as_dict(), pots[k]) for k in range(count)]

    def submit(self, W, params):
        """Queues a served request (W: int16 numpy array, host). Returns a ticket;
        raises SkError(SK_EAGAIN) when the queue is full."""
        W = np.ascontiguousarray(W, dtype=np.int16)
        t = ctypes.c_uint64(0)
        st = lib().sk_submit(self._ptr, W.ctypes.data, int(W.shape[0]), ctypes.byref(params),
                             ctypes.byref(t))
        self._check(st, "sk_submit")
        return t.value

    def completed(self, max_tickets=1024):
        """Tickets of finished requests not collected yet (sk_completed)."""
        buf = (ctypes.c_uint64 * max_tickets)()
        k = lib().sk_completed(self._ptr, buf, max_tickets)
        if k < 0:
            raise SkError(SK_EINVAL, "sk_completed")
        return [int(buf[i]) for i in range(k)]

    def poll(self, ticket, n):
        """None while the request runs, else (status, perm, weight, report)."""
        perm = np.empty(int(n), dtype=np.int32)
        weight = ctypes.c_int64(0)
        rep = Report()
        st = lib().sk_poll(self._ptr, ctypes.c_uint64(ticket),
                           perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           ctypes.byref(weight), ctypes.byref(rep))
        if st == SK_EAGAIN:
            return None
        if st == SK_EINVAL:
            raise SkError(st, f"sk_poll: {self.last_error()}")
        return st, perm, weight.value, rep.as_dict()

    def prune(self, W, potentials, params, capacity=None):
        """Reduced matrix as device tensors (row_ptr int64, col int32, w int16)."""
        torch = self.torch
        n = W.shape[0]
        self.ensure_arena(lib().sk_arena_bytes(n, 0))
        cap = int(capacity) if capacity is not None else max(4 * n, 1)
        for _ in range(2):
            row_ptr = torch.empty(n + 1, dtype=torch.int64, device=self.device)
            col = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
            w = torch.empty(max(cap, 1), dtype=torch.int16, device=self.device)
            csr = CSR(n, cap, row_ptr.data_ptr(), col.data_ptr(), w.data_ptr())
            st = lib().sk_prune(self._ptr, ctypes.c_void_p(W.data_ptr()), n,
                                ctypes.c_void_p(potentials.data_ptr()), ctypes.byref(params),
                                ctypes.byref(csr))
            if st == SK_ENOMEM and csr.nnz > cap:
                cap = int(csr.nnz)
                continue
            self._check(st, "sk_prune")
            nnz = int(csr.nnz)
            return row_ptr, col[:nnz], w[:nnz]
        raise SkError(SK_ENOMEM, "sk_prune capacity")

    def solve(self, W, params, potentials=None, max_kept=None):
        """The whole path for one instance through sk_solve: continuation in p,
        certificate, reduced matrix, exact solve of it and log gamma; with
        params.opt_ratio >= 1 the adaptive loop of Algorithm alg:alg1. Returns
        a dict (status SK_OK or SK_ENOCONV; perm/weight None when no reduced
        matrix had a perfect matching)."""
        assert W.dtype == self.torch.int16 and W.is_cuda and W.is_contiguous()
        n = int(W.shape[0])
        kept = int(max_kept) if max_kept is not None else min(n * n, 64 * n + 4096)
        pot = potentials if potentials is not None else self.new_potentials(n)
        perm = np.empty(n, dtype=np.int32)
        for attempt in range(2):
            self.ensure_arena(lib().sk_solve_arena_bytes(n, params.storage, kept))
            weight = ctypes.c_int64(0)
            rep = Report()
            st = lib().sk_solve(self._ptr, ctypes.c_void_p(W.data_ptr()), n, ctypes.byref(params),
                                ctypes.c_void_p(pot.data_ptr()),
                                perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                ctypes.byref(weight), ctypes.byref(rep))
            if st == SK_ENOMEM and attempt == 0 and kept < n * n:
                kept = n * n  # the reduced matrix kept more entries than budgeted
                continue
            break
        self._check(st, "sk_solve", ok=(SK_OK, SK_ENOCONV, SK_EINFEASIBLE))
        r = rep.as_dict()
        out = dict(status=st, report=r, nnz=int(r["nnz_kept"]), potentials=pot)
        if st == SK_EINFEASIBLE:
            out.update(perm=None, weight=None, log_gamma=None)
        else:
            out.update(perm=perm, weight=int(weight.value), log_gamma=r["log_gamma"])
        return out
