"""Python binding of libsmp (include/smp.h): the same entry points, taking torch
tensors for device memory and torch streams for ordering. Argument marshalling
only: every step of the method runs in the HIP kernels behind the C-ABI.
"""

import ctypes
import math

import torch

from . import _lib
from ._lib import SmpJobResult, SmpOmega, SmpParams, SmpServerStats
from ._lib import SMP_B_IS_A, SMP_OMEGA_REUSE, SMP_OMEGA_SPLIT, SMP_PREC_BF16, SMP_PREC_FP32, SMP_PREC_FP8  # noqa: F401
from ._lib import SMP_ERR_BUSY, SMP_ERR_NUMERIC, SMP_MAT_A, SMP_MAT_B  # noqa: F401


class SmpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_status_name(status)} ({status}): {msg}")
        self.status = status


def _status_name(s):
    lib = _lib.load()
    return lib.smp_status_str(s).decode()


def _ptr(t, dtype=None, name="tensor", dense=True):
    """Device address of a tensor; dense buffers must be contiguous (A and B
    only need unit column stride and pass dense=False)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if dense and not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not dense and t.dim() == 2 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return ctypes.c_void_p(t.data_ptr())


def default_m(n1, n2, r):
    """4 n r ln n with n = max(n1, n2)."""
    n = max(n1, n2)
    return 4.0 * n * r * math.log(n)


def make_params(d, n1, n2, k, r, T=10, m=None, seed=161006656, prec=_lib.SMP_PREC_FP32,
                omega_mode=_lib.SMP_OMEGA_REUSE, b_is_a=False, init_iters=0, sampler="binomial", sketch="gaussian"):
    """smp_params; sampler "binomial" (one coin per entry) or "multinomial"
    (row-wise draws, SMP_SAMPLE_MULTINOMIAL); sketch "gaussian" or "srht"
    (SMP_SKETCH_SRHT, FP32)."""
    if sampler not in ("binomial", "multinomial"):
        raise ValueError(f"unknown sampler {sampler!r}")
    if sketch not in ("gaussian", "srht"):
        raise ValueError(f"unknown sketch {sketch!r}")
    p = SmpParams()
    p.d, p.n1, p.n2 = int(d), int(n1), int(n2)
    p.k, p.r, p.T = int(k), int(r), int(T)
    p.prec, p.omega_mode = int(prec), int(omega_mode)
    p.flags = ((_lib.SMP_B_IS_A if b_is_a else 0) | (_lib.SMP_SAMPLE_MULTINOMIAL if sampler == "multinomial" else 0)
               | (_lib.SMP_SKETCH_SRHT if sketch == "srht" else 0))
    p.m = float(default_m(n1, n2, r) if m is None else m)
    p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    p.init_iters = int(init_iters)
    p.reserved = 0
    return p


def smp_tune_lookup(p):
    """(cap, splits) stored for this parameter set's sketch shape ((0, 0): none)."""
    lib = _lib.load()
    cap, spl = ctypes.c_int32(), ctypes.c_int32()
    s = lib.smp_tune_lookup(ctypes.byref(p), ctypes.byref(cap), ctypes.byref(spl))
    if s != _lib.SMP_OK:
        raise SmpError(s, lib.smp_last_error(None).decode())
    return cap.value, spl.value


def smp_tune_save(path):
    lib = _lib.load()
    s = lib.smp_tune_save(str(path).encode())
    if s != _lib.SMP_OK:
        raise SmpError(s, lib.smp_last_error(None).decode())


def smp_tune_load(path):
    lib = _lib.load()
    s = lib.smp_tune_load(str(path).encode())
    if s != _lib.SMP_OK:
        raise SmpError(s, lib.smp_last_error(None).decode())


def smp_tune_clear():
    _lib.load().smp_tune_clear()


def smp_check_params(p):
    lib = _lib.load()
    s = lib.smp_check_params(ctypes.byref(p))
    if s != _lib.SMP_OK:
        raise SmpError(s, lib.smp_last_error(None).decode())


def smp_workspace_size(p):
    lib = _lib.load()
    out = ctypes.c_size_t(0)
    s = lib.smp_workspace_size(ctypes.byref(p), ctypes.byref(out))
    if s != _lib.SMP_OK:
        raise SmpError(s, lib.smp_last_error(None).decode())
    return out.value


class Omega:
    """Caller-owned device arrays of the sampled set (the smp_omega struct)."""

    def __init__(self, n1, n2, cap, device, split=False):
        self.n1, self.n2, self.cap = n1, n2, cap
        kw = dict(device=device)
        self.row_ptr = torch.zeros(n1 + 1, dtype=torch.int64, **kw)
        self.col_ptr = torch.zeros(n2 + 1, dtype=torch.int64, **kw)
        c = max(cap, 1)
        self.col_idx = torch.zeros(c, dtype=torch.int32, **kw)
        self.row_idx = torch.zeros(c, dtype=torch.int32, **kw)
        self.w_csr = torch.zeros(c, dtype=torch.float64, **kw)
        self.w_csc = torch.zeros(c, dtype=torch.float64, **kw)
        self.mt_csr = torch.zeros(c, dtype=torch.float64, **kw)
        self.mt_csc = torch.zeros(c, dtype=torch.float64, **kw)
        self.sub_csr = torch.zeros(c, dtype=torch.uint8, **kw) if split else None
        self.sub_csc = torch.zeros(c, dtype=torch.uint8, **kw) if split else None
        self.nnz = 0

    def struct(self):
        o = SmpOmega()
        o.n1, o.n2, o.cap, o.nnz = self.n1, self.n2, self.cap, self.nnz
        for name in ("row_ptr", "col_idx", "w_csr", "mt_csr", "sub_csr",
                     "col_ptr", "row_idx", "w_csc", "mt_csc", "sub_csc"):
            t = getattr(self, name)
            setattr(o, name, t.data_ptr() if t is not None else None)
        return o


class Context:
    """An smp_ctx bound to a device and a torch stream (the current stream by default)."""

    def __init__(self, device=0, stream=None):
        self.lib = _lib.load()
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.device = dev
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        self.stream = st
        h = ctypes.c_void_p()
        s = self.lib.smp_create(ctypes.byref(h), dev.index or 0, ctypes.c_void_p(st.cuda_stream))
        if s != _lib.SMP_OK:
            raise SmpError(s, self.lib.smp_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.smp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s):
        if s != _lib.SMP_OK:
            raise SmpError(s, self.lib.smp_last_error(self.h).decode())

    # ---- entry points (same names as the C-ABI)
    def smp_pi_fill(self, p, l0, nrows, out):
        self._check(self.lib.smp_pi_fill(self.h, ctypes.byref(p), int(l0), int(nrows),
                                         _ptr(out, torch.float32, "out")))

    def smp_sketch(self, p, A, B, At, Bt, na2, nb2):
        lda = A.stride(0)
        ldb = B.stride(0) if B is not None else 0
        if A.stride(1) != 1 or (B is not None and B.stride(1) != 1):
            raise ValueError("A and B must have unit column stride")
        self._check(self.lib.smp_sketch(self.h, ctypes.byref(p), _ptr(A, torch.float32, "A", dense=False), lda,
                                        _ptr(B, torch.float32, "B", dense=False), ldb, _ptr(At, torch.float32, "At"),
                                        _ptr(Bt, torch.float32, "Bt"), _ptr(na2, torch.float32, "na2"),
                                        _ptr(nb2, torch.float32, "nb2")))

    def smp_sketch_begin(self, p):
        st = ctypes.c_void_p()
        self._check(self.lib.smp_sketch_begin(self.h, ctypes.byref(p), ctypes.byref(st)))
        return st

    def smp_sketch_push(self, st, A_rows, B_rows, row0):
        nrows = A_rows.shape[0]
        ldb = B_rows.stride(0) if B_rows is not None else 0
        self._check(self.lib.smp_sketch_push(self.h, st, _ptr(A_rows, torch.float32, "A_rows", dense=False), A_rows.stride(0),
                                             _ptr(B_rows, torch.float32, "B_rows", dense=False), ldb, int(row0), int(nrows)))

    def smp_sketch_end(self, st, At, Bt, na2, nb2):
        self._check(self.lib.smp_sketch_end(self.h, st, _ptr(At, torch.float32, "At"), _ptr(Bt, torch.float32, "Bt"),
                                            _ptr(na2, torch.float32, "na2"), _ptr(nb2, torch.float32, "nb2")))

    def smp_sketch_free(self, st):
        self.lib.smp_sketch_free(st)

    def smp_sketch_push_coo(self, st, which, rows, cols, vals):
        """Entries (rows[e], cols[e], vals[e]) of A (which = SMP_MAT_A) or B, in any order."""
        nnz = rows.numel()
        if cols.numel() != nnz or vals.numel() != nnz:
            raise ValueError("rows, cols and vals differ in length")
        self._check(self.lib.smp_sketch_push_coo(self.h, st, int(which), _ptr(rows, torch.int64, "rows"),
                                                 _ptr(cols, torch.int32, "cols"), _ptr(vals, torch.float32, "vals"),
                                                 nnz))

    def smp_sketch_push_csr(self, st, which, row0, row_ptr, cols, vals):
        """CSR rows row0 .. row0 + len(row_ptr) - 2 of A (which = SMP_MAT_A) or B."""
        nnz = cols.numel()
        if vals.numel() != nnz:
            raise ValueError("cols and vals differ in length")
        self._check(self.lib.smp_sketch_push_csr(self.h, st, int(which), int(row0), row_ptr.numel() - 1,
                                                 _ptr(row_ptr, torch.int64, "row_ptr"), _ptr(cols, torch.int32, "cols"),
                                                 _ptr(vals, torch.float32, "vals"), nnz))

    def smp_tune_sketch(self, p, A, B):
        """Time the sketch pass's launch shapes on A and B (B None: SMP_B_IS_A)
        and keep the fastest for this shape; returns (cap, splits, ms)."""
        if A.stride(1) != 1 or (B is not None and B.stride(1) != 1):
            raise ValueError("A and B must have unit column stride")
        cap, spl, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self._check(self.lib.smp_tune_sketch(self.h, ctypes.byref(p), _ptr(A, torch.float32, "A", dense=False),
                                             A.stride(0), _ptr(B, torch.float32, "B", dense=False),
                                             B.stride(0) if B is not None else 0, ctypes.byref(cap),
                                             ctypes.byref(spl), ctypes.byref(ms)))
        return cap.value, spl.value, ms.value

    def smp_solve_sketched(self, p, At, Bt, na2, nb2, U, V, sigma=None):
        self._check(self.lib.smp_solve_sketched(self.h, ctypes.byref(p), _ptr(At, torch.float32, "At"),
                                                _ptr(Bt, torch.float32, "Bt"), _ptr(na2, torch.float32, "na2"),
                                                _ptr(nb2, torch.float32, "nb2"), _ptr(U, torch.float64, "U"),
                                                _ptr(V, torch.float64, "V"), _ptr(sigma, torch.float64, "sigma")))

    def smp_sample(self, p, na2, nb2, om):
        o = om.struct()
        s = self.lib.smp_sample(self.h, ctypes.byref(p), _ptr(na2, torch.float32, "na2"),
                                _ptr(nb2, torch.float32, "nb2"), ctypes.byref(o))
        om.nnz = o.nnz
        self._check(s)
        return om.nnz

    def smp_estimate(self, p, At, Bt, na2, nb2, om):
        o = om.struct()
        self._check(self.lib.smp_estimate(self.h, ctypes.byref(p), _ptr(At, torch.float32, "At"),
                                          _ptr(Bt, torch.float32, "Bt"), _ptr(na2, torch.float32, "na2"),
                                          _ptr(nb2, torch.float32, "nb2"), ctypes.byref(o)))

    def smp_estimate_noalloc(self, p, At, Bt, na2, nb2, om):
        o = om.struct()
        self._check(self.lib.smp_estimate_noalloc(self.h, ctypes.byref(p), _ptr(At, torch.float32, "At"),
                                                  _ptr(Bt, torch.float32, "Bt"), _ptr(na2, torch.float32, "na2"),
                                                  _ptr(nb2, torch.float32, "nb2"), ctypes.byref(o)))

    def smp_waltmin(self, p, om, na2, U, V, sigma=None):
        o = om.struct()
        self._check(self.lib.smp_waltmin(self.h, ctypes.byref(p), ctypes.byref(o), _ptr(na2, torch.float32, "na2"),
                                         _ptr(U, torch.float64, "U"), _ptr(V, torch.float64, "V"),
                                         _ptr(sigma, torch.float64, "sigma")))

    def smp_sketch_group(self, params, As, Bs, Ats, Bts, na2s, nb2s):
        """smp_sketch for every BF16 job of the lists in grouped launches (B
        None, or SMP_B_IS_A in the job's flags: B = A; Bt and nb2 may then be
        None)."""
        n = len(params)
        if not (len(As) == len(Bs) == len(Ats) == len(Bts) == len(na2s) == len(nb2s) == n):
            raise ValueError("job lists differ in length")
        for X in list(As) + [b for b in Bs if b is not None]:
            if X.stride(1) != 1:
                raise ValueError("A and B must have unit column stride")
        P = (SmpParams * max(1, n))(*params)
        ptrs = lambda ts, nm, dense=True: (ctypes.c_void_p * max(1, n))(
            *[_ptr(t, torch.float32, nm, dense=dense) for t in ts])
        lds = lambda ts: (ctypes.c_int64 * max(1, n))(*[t.stride(0) if t is not None else 0 for t in ts])
        self._check(self.lib.smp_sketch_group(self.h, n, P, ptrs(As, "A", False), lds(As), ptrs(Bs, "B", False),
                                              lds(Bs), ptrs(Ats, "At"), ptrs(Bts, "Bt"), ptrs(na2s, "na2"),
                                              ptrs(nb2s, "nb2")))

    def smp_waltmin_group(self, params, omegas, na2s, Us, Vs, sigmas=None, graph=True):
        """smp_waltmin for every job of the lists at once (grouped launches,
        one HIP graph per group of equal launch sequences with graph=True)."""
        n = len(params)
        if not (len(omegas) == len(na2s) == len(Us) == len(Vs) == n) or (sigmas is not None and len(sigmas) != n):
            raise ValueError("job lists differ in length")
        P = (SmpParams * max(1, n))(*params)
        O = (SmpOmega * max(1, n))(*[o.struct() for o in omegas])
        ptrs = lambda ts, dt, nm: (ctypes.c_void_p * max(1, n))(*[_ptr(t, dt, nm) for t in ts])
        na = ptrs(na2s, torch.float32, "na2")
        U = ptrs(Us, torch.float64, "U")
        V = ptrs(Vs, torch.float64, "V")
        S = ptrs(sigmas, torch.float64, "sigma") if sigmas is not None else None
        self._check(self.lib.smp_waltmin_group(self.h, n, P, O, na, U, V, S, int(bool(graph))))

    def smp_set_timing(self, enable=True):
        """True or 1: every stage; 2: the sketch stage only; False or 0: off."""
        self._check(self.lib.smp_set_timing(self.h, int(enable)))

    def smp_stage_times(self):
        """ms of the last call's stages: sketch kernel, sketch reduction,
        sampling, estimate, WAltMin."""
        arr = (ctypes.c_float * 5)()
        self._check(self.lib.smp_stage_times(self.h, arr, 5))
        return dict(zip(("sketch", "sketch_finish", "sample", "estimate", "waltmin"), list(arr)))

    def smp_solve(self, p, A, B, U, V, sigma=None):
        if A.stride(1) != 1 or (B is not None and B.stride(1) != 1):
            raise ValueError("A and B must have unit column stride")
        Bp = B if B is not None else A
        self._check(self.lib.smp_solve(self.h, ctypes.byref(p), _ptr(A, torch.float32, "A", dense=False), A.stride(0),
                                       _ptr(Bp, torch.float32, "B", dense=False), Bp.stride(0), _ptr(U, torch.float64, "U"),
                                       _ptr(V, torch.float64, "V"), _ptr(sigma, torch.float64, "sigma")))

    # ---- comparison methods (Section 4)
    def smp_svd_sketch(self, p, At, Bt, U, V, sigma=None):
        self._check(self.lib.smp_svd_sketch(self.h, ctypes.byref(p), _ptr(At, torch.float32, "At"),
                                            _ptr(Bt, torch.float32, "Bt"), _ptr(U, torch.float64, "U"),
                                            _ptr(V, torch.float64, "V"), _ptr(sigma, torch.float64, "sigma")))

    def _ab(self, A, B):
        if A.stride(1) != 1 or (B is not None and B.stride(1) != 1):
            raise ValueError("A and B must have unit column stride")
        Bp = B if B is not None else A
        return (_ptr(A, torch.float32, "A", dense=False), A.stride(0), _ptr(Bp, torch.float32, "B", dense=False),
                Bp.stride(0))

    def smp_solve_svd_sketch(self, p, A, B, U, V, sigma=None):
        self._check(self.lib.smp_solve_svd_sketch(self.h, ctypes.byref(p), *self._ab(A, B), _ptr(U, torch.float64, "U"),
                                                  _ptr(V, torch.float64, "V"), _ptr(sigma, torch.float64, "sigma")))

    def smp_column_norms(self, p, A, B, na2, nb2):
        self._check(self.lib.smp_column_norms(self.h, ctypes.byref(p), *self._ab(A, B),
                                              _ptr(na2, torch.float32, "na2"), _ptr(nb2, torch.float32, "nb2")))

    def smp_exact_entries(self, p, A, B, om):
        o = om.struct()
        self._check(self.lib.smp_exact_entries(self.h, ctypes.byref(p), *self._ab(A, B), ctypes.byref(o)))

    def smp_lela(self, p, A, B, U, V, sigma=None):
        self._check(self.lib.smp_lela(self.h, ctypes.byref(p), *self._ab(A, B), _ptr(U, torch.float64, "U"),
                                      _ptr(V, torch.float64, "V"), _ptr(sigma, torch.float64, "sigma")))


def _job_dict(r):
    return {"status": int(r.status), "worker": int(r.worker), "queue_ms": float(r.queue_ms),
            "run_ms": float(r.run_ms)}


class Server:
    """smp_server: independent jobs (one smp_solve each) run by `workers`
    threads, each with its own context and HIP stream, admitted in order
    within `hbm_budget` bytes of library workspace (0: no budget). The
    tensors of a job are kept referenced until the job is waited for."""

    def __init__(self, device=0, workers=4, hbm_budget=0):
        self.lib = _lib.load()
        dev = torch.device(device if not isinstance(device, int) else f"cuda:{device}")
        self.device = dev
        h = ctypes.c_void_p()
        st = self.lib.smp_server_create(dev.index or 0, int(workers), int(hbm_budget), ctypes.byref(h))
        if st != 0:
            raise SmpError(st, "smp_server_create failed")
        self.h = h
        self._held = {}

    def submit(self, p, A, B, U, V, sigma=None):
        """Queue one job; returns its id. The inputs must be complete on the
        device: the current torch stream is synchronised first, because the
        workers' streams do not wait on it."""
        if A.stride(1) != 1 or (B is not None and B.stride(1) != 1):
            raise ValueError("A and B must have unit column stride")
        Bp = B if B is not None else A
        torch.cuda.current_stream(self.device).synchronize()
        jid = ctypes.c_uint64()
        st = self.lib.smp_server_submit(self.h, ctypes.byref(p), _ptr(A, torch.float32, "A", dense=False), A.stride(0),
                                        _ptr(Bp, torch.float32, "B", dense=False), Bp.stride(0),
                                        _ptr(U, torch.float64, "U"), _ptr(V, torch.float64, "V"),
                                        _ptr(sigma, torch.float64, "sigma"), ctypes.byref(jid))
        if st != 0:
            raise SmpError(st, "smp_server_submit rejected the job")
        self._held[jid.value] = (p, A, B, U, V, sigma)
        return jid.value

    def try_submit(self, p, A, B, U, V, sigma=None):
        """Queue the job only if it can start at once (smp_server_try_submit);
        returns its id, or None when the server answers SMP_ERR_BUSY."""
        if A.stride(1) != 1 or (B is not None and B.stride(1) != 1):
            raise ValueError("A and B must have unit column stride")
        Bp = B if B is not None else A
        torch.cuda.current_stream(self.device).synchronize()
        jid = ctypes.c_uint64()
        st = self.lib.smp_server_try_submit(self.h, ctypes.byref(p), _ptr(A, torch.float32, "A", dense=False),
                                            A.stride(0), _ptr(Bp, torch.float32, "B", dense=False), Bp.stride(0),
                                            _ptr(U, torch.float64, "U"), _ptr(V, torch.float64, "V"),
                                            _ptr(sigma, torch.float64, "sigma"), ctypes.byref(jid))
        if st == _lib.SMP_ERR_BUSY:
            return None
        if st != 0:
            raise SmpError(st, "smp_server_try_submit rejected the job")
        self._held[jid.value] = (p, A, B, U, V, sigma)
        return jid.value

    def wait(self, job_id):
        """Block until the job is done; returns {status, worker, queue_ms,
        run_ms} (and `error` when the job failed)."""
        r = SmpJobResult()
        st = self.lib.smp_server_wait(self.h, ctypes.c_uint64(job_id), ctypes.byref(r))
        if st != 0:
            raise SmpError(st, f"unknown job {job_id}")
        self._held.pop(job_id, None)
        out = _job_dict(r)
        if r.status != 0:
            out["error"] = self.lib.smp_server_last_error(self.h).decode()
        return out

    def stats(self):
        s = SmpServerStats()
        st = self.lib.smp_server_get_stats(self.h, ctypes.byref(s))
        if st != 0:
            raise SmpError(st, "smp_server_get_stats failed")
        return {f: int(getattr(s, f)) for f, _ in SmpServerStats._fields_}

    def close(self):
        if self.h:
            self.lib.smp_server_destroy(self.h)
            self.h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(jobs, device=0, workers=4, hbm_budget=0):
    """smp_solve_batch over a list of jobs, each a dict with keys p, A, B
    (None for A = B), U, V, sigma (optional). Returns the per-job results and
    the batch status."""
    lib = _lib.load()
    n = len(jobs)
    P = (SmpParams * n)(*[j["p"] for j in jobs])
    vp = ctypes.c_void_p
    A = (vp * n)(*[_ptr(j["A"], torch.float32, "A", dense=False) for j in jobs])
    lda = (ctypes.c_int64 * n)(*[j["A"].stride(0) for j in jobs])
    Bs = [j["B"] if j["B"] is not None else j["A"] for j in jobs]
    B = (vp * n)(*[_ptr(b, torch.float32, "B", dense=False) for b in Bs])
    ldb = (ctypes.c_int64 * n)(*[b.stride(0) for b in Bs])
    U = (vp * n)(*[_ptr(j["U"], torch.float64, "U") for j in jobs])
    V = (vp * n)(*[_ptr(j["V"], torch.float64, "V") for j in jobs])
    S = (vp * n)(*[_ptr(j.get("sigma"), torch.float64, "sigma") for j in jobs])
    res = (SmpJobResult * n)()
    torch.cuda.current_stream().synchronize()
    st = lib.smp_solve_batch(int(device), n, P, A, lda, B, ldb, U, V, S, int(workers), int(hbm_budget), res)
    return st, [_job_dict(r) for r in res]


def _batch_arrays(jobs):
    n = len(jobs)
    P = (SmpParams * n)(*[j["p"] for j in jobs])
    vp = ctypes.c_void_p
    A = (vp * n)(*[_ptr(j["A"], torch.float32, "A", dense=False) for j in jobs])
    lda = (ctypes.c_int64 * n)(*[j["A"].stride(0) for j in jobs])
    Bs = [j["B"] if j["B"] is not None else j["A"] for j in jobs]
    B = (vp * n)(*[_ptr(b, torch.float32, "B", dense=False) for b in Bs])
    ldb = (ctypes.c_int64 * n)(*[b.stride(0) for b in Bs])
    U = (vp * n)(*[_ptr(j["U"], torch.float64, "U") for j in jobs])
    V = (vp * n)(*[_ptr(j["V"], torch.float64, "V") for j in jobs])
    S = (vp * n)(*[_ptr(j.get("sigma"), torch.float64, "sigma") for j in jobs])
    return n, P, A, lda, B, ldb, U, V, S


def solve_batch_group(jobs, device=0, workers=4, graph=True):
    """smp_solve_batch_group over a list of jobs (keys as solve_batch): steps
    2-4 on `workers` threads, then WAltMin for all jobs grouped. Returns the
    per-job results and the batch status."""
    lib = _lib.load()
    n, P, A, lda, B, ldb, U, V, S = _batch_arrays(jobs)
    res = (SmpJobResult * n)()
    torch.cuda.current_stream().synchronize()
    st = lib.smp_solve_batch_group(int(device), n, P, A, lda, B, ldb, U, V, S, int(workers), int(bool(graph)), res)
    return st, [_job_dict(r) for r in res]


def solve(A, B, k, r, T=10, m=None, seed=161006656, prec=_lib.SMP_PREC_FP32, omega_mode=_lib.SMP_OMEGA_REUSE,
          ctx=None, init_iters=0):
    """Alg. 1 on device tensors A (d x n1), B (d x n2, or None for A = B).
    Returns (U, sigma, V): U diag(sigma) V^T approximates A^T B."""
    d, n1 = A.shape
    n2 = n1 if B is None else B.shape[1]
    p = make_params(d, n1, n2, k, r, T, m, seed, prec, omega_mode, b_is_a=B is None, init_iters=init_iters)
    ctx = ctx or Context(A.device)
    U = torch.empty(n1, r, dtype=torch.float64, device=A.device)
    V = torch.empty(n2, r, dtype=torch.float64, device=A.device)
    s = torch.empty(r, dtype=torch.float64, device=A.device)
    ctx.smp_solve(p, A, B, U, V, s)
    return U, s, V
