"""ctypes binding of libshci_pt2.so (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; PyTorch
supplies device memory and the current stream.  There is no CPU fallback:
importing this module without the built library raises at first use.

Determinants are passed as int64 tensors of shape [N, 4] holding the uint64
words (alpha_lo, alpha_hi, beta_lo, beta_hi) bit for bit.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshci_pt2.so")

SHCI_FP64 = 0
SHCI_FP32C = 1
_PREC = {"fp64": SHCI_FP64, "fp32c": SHCI_FP32C, SHCI_FP64: SHCI_FP64, SHCI_FP32C: SHCI_FP32C}
OPS = {"det": 0, "grad": 1, "grad_keep": 2, "sample": 3, "sample_grad": 4, "draws": 5}
GRAD_MODES = {"auto": 0, "keep": 1, "recompute": 2}

STATUS = {0: "SHCI_OK", -1: "SHCI_ERR_ARG", -2: "SHCI_ERR_NORB", -3: "SHCI_ERR_DET",
          -4: "SHCI_ERR_DUP", -5: "SHCI_ERR_NONFINITE", -6: "SHCI_ERR_WORKSPACE",
          -7: "SHCI_ERR_SINGULAR", -8: "SHCI_ERR_HIP"}


class ShciError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Stats(C.Structure):
    _fields_ = [("n_terms", C.c_int64), ("n_terms_gen", C.c_int64), ("n_unique", C.c_int64),
                ("n_intruder", C.c_int64), ("min_abs_denom", C.c_double),
                ("n_buckets", C.c_int32), ("n_retries", C.c_int32),
                ("ms_gen", C.c_double), ("ms_sort", C.c_double), ("ms_reduce", C.c_double),
                ("ms_total", C.c_double), ("ms_k_count", C.c_double), ("ms_k_write", C.c_double),
                ("ms_k_reduce", C.c_double), ("n_records", C.c_int64), ("key_words", C.c_int32),
                ("value_bytes", C.c_int32), ("n_chunks", C.c_int32), ("n_part_launches", C.c_int32),
                ("ms_k_part", C.c_double), ("n_part_records", C.c_int64), ("n_terms_all", C.c_int64),
                ("n_hashes", C.c_int64), ("n_singletons", C.c_int64), ("ms_k_split", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Export(C.Structure):
    _fields_ = [("u_keys", C.c_void_p), ("u_A", C.c_void_p), ("u_D", C.c_void_p),
                ("u_cnt", C.c_void_p), ("u_cap", C.c_int64), ("u_n", C.c_int64),
                ("t_keys", C.c_void_p), ("t_i", C.c_void_p), ("t_val", C.c_void_p),
                ("t_cap", C.c_int64), ("t_n", C.c_int64)]


class Batch(C.Structure):
    _fields_ = [("sum", C.c_double), ("sumsq", C.c_double), ("n_unique", C.c_int64), ("n_terms", C.c_int64)]


class ThreeStep(C.Structure):
    _fields_ = [("e2", C.c_double), ("err", C.c_double), ("e2_dtm", C.c_double), ("e2_psto", C.c_double),
                ("err_psto", C.c_double), ("psto_batches_used", C.c_int32), ("e2_sto", C.c_double),
                ("err_sto", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                               "paper_1809_04600_amd/build.sh")
        L = C.CDLL(LIB_PATH)
        p, i, i64, d = C.c_void_p, C.c_int, C.c_int64, C.c_double
        L.shci_pt2_last_error.restype = C.c_char_p
        L.shci_pt2_version.restype = C.c_char_p
        L.shci_pt2_ctx_create.argtypes = [i, i, i, p, p, p, C.POINTER(p)]
        L.shci_pt2_ctx_create.restype = i
        L.shci_pt2_ctx_destroy.argtypes = [p]
        L.shci_pt2_ctx_destroy.restype = None
        L.shci_pt2_ctx_set_workspace_limit.argtypes = [p, C.c_size_t]
        L.shci_pt2_ctx_set_workspace_limit.restype = i
        L.shci_pt2_ctx_set_record_limit.argtypes = [p, C.c_int64]
        L.shci_pt2_ctx_set_record_limit.restype = i
        L.shci_pt2_ctx_set_grouping.argtypes = [p, i]
        L.shci_pt2_ctx_set_grouping.restype = i
        L.shci_pt2_ctx_set_lanes.argtypes = [p, i]
        L.shci_pt2_ctx_set_lanes.restype = i
        L.shci_pt2_ctx_set_split_bucket.argtypes = [p, C.c_int64]
        L.shci_pt2_ctx_set_split_bucket.restype = i
        u64, sz, i32 = C.c_uint64, C.c_size_t, C.c_int32
        L.shci_pt2_workspace_size.argtypes = [p, i, i64, i64, i32, i32, i, C.POINTER(sz)]
        L.shci_pt2_workspace_size.restype = i
        L.shci_pt2_det.argtypes = [p, p, p, i64, d, d, i, p, sz, p, C.POINTER(d), C.POINTER(Stats),
                                   C.POINTER(Export)]
        L.shci_pt2_det.restype = i
        L.shci_pt2_det_static.argtypes = [p, p, p, i64, d, d, i, p, C.POINTER(d), C.POINTER(Stats)]
        L.shci_pt2_det_static.restype = i
        L.shci_pt2_sample.argtypes = [p, p, p, i64, d, d, d, i32, i32, p, u64, i, p, sz, p, p,
                                      C.POINTER(d), C.POINTER(d), C.POINTER(Stats)]
        L.shci_pt2_sample.restype = i
        L.shci_pt2_draws.argtypes = [p, p, i64, u64, i32, i32, p, sz, p, p]
        L.shci_pt2_draws.restype = i
        L.shci_pt2_alias_table.argtypes = [p, p, i64, p, sz, p, p, p]
        L.shci_pt2_alias_table.restype = i
        L.shci_pt2_sample_grad.argtypes = [p, p, p, i64, d, d, d, i32, i32, p, u64, i, p, sz, p, p,
                                           C.POINTER(d), C.POINTER(d), p, C.POINTER(d), C.POINTER(Stats)]
        L.shci_pt2_sample_grad.restype = i
        L.shci_pt2_sample_batched.argtypes = [p, p, p, i64, d, d, d, i32, i32, p, i32, p, u64,
                                              i, p, sz, p, p, C.POINTER(d), C.POINTER(d), C.POINTER(Stats)]
        L.shci_pt2_sample_batched.restype = i
        L.shci_pt2_det_batches.argtypes = [p, p, p, i64, d, d, d, i32, p, i32, i, p, sz, p, p,
                                           C.POINTER(Stats)]
        L.shci_pt2_det_batches.restype = i
        L.shci_pt2_three_step.argtypes = [p, p, p, i64, d, d, d, d, d, i32, i32, i32,
                                          i32, p, p, u64, i, p, sz, p, p, C.POINTER(ThreeStep)]
        L.shci_pt2_three_step.restype = i
        L.shci_pt2_select.argtypes = [p, p, p, i64, d, d, i, d, i, p, p, p, i64, C.POINTER(i64),
                                      C.POINTER(Stats)]
        L.shci_pt2_select.restype = i
        L.shci_pt2_grad.argtypes = [p, p, p, i64, d, d, i, i, p, sz, p, C.POINTER(d), p, C.POINTER(d),
                                    C.POINTER(Stats)]
        L.shci_pt2_grad.restype = i
        L.shci_pt2_hc.argtypes = [p, p, p, i64, p, p, p, C.POINTER(d), C.POINTER(Stats)]
        L.shci_pt2_hc.restype = i
        _lib = L
    return _lib


def _check(code: int):
    if code != 0:
        raise ShciError(code, lib().shci_pt2_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, shape=None, name="tensor"):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {shape}")
    return C.c_void_p(t.data_ptr())


@dataclass
class DetResult:
    e2: float
    stats: dict
    unique: dict | None = None
    terms: dict | None = None


class Context:
    """Integral set on the device plus the library's tables (shci_pt2_ctx)."""

    def __init__(self, h1: torch.Tensor, eri: torch.Tensor, n_alpha: int, n_beta: int):
        n = h1.shape[0]
        self.n, self.na, self.nb = n, n_alpha, n_beta
        h1 = h1.contiguous()
        eri = eri.contiguous()
        ptr = C.c_void_p()
        _check(lib().shci_pt2_ctx_create(n, n_alpha, n_beta, _dev(h1, torch.float64, (n, n), "h1"),
                                         _dev(eri, torch.float64, (n, n, n, n), "eri"), _stream(),
                                         C.byref(ptr)))
        self._ptr = ptr

    _ws = None

    def set_workspace(self, ws):
        """Device workspace passed to every PT2 call: a uint8 device tensor,
        a size in bytes (allocated through torch), or None (the library's own
        grow-only buffers)."""
        if ws is None or isinstance(ws, torch.Tensor):
            self._ws = ws
        else:
            self._ws = torch.empty(int(ws), dtype=torch.uint8, device="cuda")

    def workspace_size(self, op, n_det, n_records=0, n_samples=0, n_draws=0, precision="fp64") -> int:
        out = C.c_size_t()
        _check(lib().shci_pt2_workspace_size(self._ptr, OPS[op], int(n_det), int(n_records), int(n_samples),
                                             int(n_draws), _PREC[precision], C.byref(out)))
        return out.value

    def _wsarg(self, ws):
        w = self._ws if ws is None else ws
        if w is False or w is None:
            return C.c_void_p(None), 0
        if not (w.is_cuda and w.dtype == torch.uint8 and w.is_contiguous()):
            raise ValueError("workspace must be a contiguous uint8 device tensor")
        return C.c_void_p(w.data_ptr()), w.numel()

    def close(self):
        if getattr(self, "_ptr", None):
            lib().shci_pt2_ctx_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_workspace_limit(self, nbytes: int):
        _check(lib().shci_pt2_ctx_set_workspace_limit(self._ptr, nbytes))

    def set_record_limit(self, max_records: int):
        """Records per generation pass (0 = automatic); above it the
        deterministic paths use hash batches and sampling uses chunks."""
        _check(lib().shci_pt2_ctx_set_record_limit(self._ptr, int(max_records)))

    def set_grouping(self, mode: str):
        """"split" (singleton split where the call needs no per-a output),
        "records" (every screened term becomes a record) or "auto" (split for
        sampling passes and deterministic passes of 1e8 terms or more)."""
        m = {"auto": 0, "records": 1, "split": 2}
        if mode not in m:
            raise ValueError(f"grouping must be one of {sorted(m)}")
        _check(lib().shci_pt2_ctx_set_grouping(self._ptr, m[mode]))

    def set_lanes(self, lanes: int):
        """Sample chunks in flight at once with a caller workspace (1 or 2)."""
        _check(lib().shci_pt2_ctx_set_lanes(self._ptr, int(lanes)))

    def set_split_bucket(self, hashes: int):
        """Hashes per bucket of the singleton split's repeat finder."""
        _check(lib().shci_pt2_ctx_set_split_bucket(self._ptr, int(hashes)))

    def _inputs(self, dets, c):
        nd = c.shape[0]
        return _dev(dets, torch.int64, (nd, 4), "dets"), _dev(c, torch.float64, (nd,), "c"), nd

    def det(self, dets, c, e0, eps2, precision="fp64", unique_cap=0, terms_cap=0, ws=None) -> DetResult:
        """Deterministic screened PT2.  ws: workspace tensor for this call
        (False: none, None: the context's set_workspace)."""
        pd, pc, nd = self._inputs(dets, c)
        pw, nw = self._wsarg(ws)
        e2 = C.c_double()
        st = Stats()
        ex = None
        bufs = {}
        if unique_cap or terms_cap:
            ex = Export()
            dev = c.device
            if unique_cap:
                bufs["u_keys"] = torch.zeros((unique_cap, 4), dtype=torch.int64, device=dev)
                bufs["u_A"] = torch.zeros(unique_cap, dtype=torch.float64, device=dev)
                bufs["u_D"] = torch.zeros(unique_cap, dtype=torch.float64, device=dev)
                bufs["u_cnt"] = torch.zeros(unique_cap, dtype=torch.int32, device=dev)
                ex.u_keys = bufs["u_keys"].data_ptr()
                ex.u_A = bufs["u_A"].data_ptr()
                ex.u_D = bufs["u_D"].data_ptr()
                ex.u_cnt = bufs["u_cnt"].data_ptr()
                ex.u_cap = unique_cap
            if terms_cap:
                bufs["t_keys"] = torch.zeros((terms_cap, 4), dtype=torch.int64, device=dev)
                bufs["t_i"] = torch.zeros(terms_cap, dtype=torch.int32, device=dev)
                bufs["t_val"] = torch.zeros(terms_cap, dtype=torch.float64, device=dev)
                ex.t_keys = bufs["t_keys"].data_ptr()
                ex.t_i = bufs["t_i"].data_ptr()
                ex.t_val = bufs["t_val"].data_ptr()
                ex.t_cap = terms_cap
        _check(lib().shci_pt2_det(self._ptr, pd, pc, nd, float(e0), float(eps2), _PREC[precision],
                                  pw, nw, _stream(), C.byref(e2), C.byref(st),
                                  C.byref(ex) if ex is not None else None))
        r = DetResult(e2.value, st.as_dict())
        if ex is not None and unique_cap:
            m = min(ex.u_n, unique_cap)
            r.unique = {"n": ex.u_n, "keys": bufs["u_keys"][:m], "A": bufs["u_A"][:m],
                        "D": bufs["u_D"][:m], "cnt": bufs["u_cnt"][:m]}
        if ex is not None and terms_cap:
            m = min(ex.t_n, terms_cap)
            r.terms = {"n": ex.t_n, "keys": bufs["t_keys"][:m], "i": bufs["t_i"][:m],
                       "val": bufs["t_val"][:m]}
        return r

    def det_static(self, dets, c, e0, eps2, precision="fp64"):
        """shci_pt2_det on the library's fixed device workspace (no allocation)."""
        pd, pc, nd = self._inputs(dets, c)
        e2 = C.c_double()
        st = Stats()
        _check(lib().shci_pt2_det_static(self._ptr, pd, pc, nd, float(e0), float(eps2), _PREC[precision],
                                         _stream(), C.byref(e2), C.byref(st)))
        return DetResult(e2.value, st.as_dict())

    def grad(self, dets, c, e0, eps2, precision="fp64", mode="auto", ws=None):
        """E2, dE2/dc (device tensor), dE2/dE0, stats.  mode: "auto", "keep"
        or "recompute" (the adjoint's source of the connections)."""
        pd, pc, nd = self._inputs(dets, c)
        pw, nw = self._wsarg(ws)
        g = torch.empty(nd, dtype=torch.float64, device=c.device)
        e2 = C.c_double()
        de0 = C.c_double()
        st = Stats()
        _check(lib().shci_pt2_grad(self._ptr, pd, pc, nd, float(e0), float(eps2), _PREC[precision],
                                   GRAD_MODES[mode], pw, nw, _stream(), C.byref(e2),
                                   C.c_void_p(g.data_ptr()), C.byref(de0), C.byref(st)))
        return e2.value, g, de0.value, st.as_dict()

    def _draws_arg(self, draws, n_samples, n_draws):
        if draws is None:
            if not n_samples or not n_draws:
                raise ValueError("the seed path needs n_samples and n_draws")
            return C.c_void_p(None), int(n_samples), int(n_draws)
        ns, ndraw = draws.shape
        return _dev(draws, torch.int32, (ns, ndraw), "draws"), ns, ndraw

    def sample(self, dets, c, e0, eps2, eps2_d, draws, precision="fp64", *, seed=0, n_samples=None,
               n_draws=None, ws=None):
        """Per-sample S_s(eps2) - S_s(eps2_d).  draws: int32 [ns, nd] device
        tensor, or None with n_samples, n_draws and seed (draws made on the
        device by the alias method)."""
        pd, pc, nd = self._inputs(dets, c)
        pdr, ns, ndraw = self._draws_arg(draws, n_samples, n_draws)
        pw, nw = self._wsarg(ws)
        out = torch.empty(ns, dtype=torch.float64, device=c.device)
        mean = C.c_double()
        sem = C.c_double()
        st = Stats()
        _check(lib().shci_pt2_sample(self._ptr, pd, pc, nd, float(e0), float(eps2), float(eps2_d),
                                     ns, ndraw, pdr, int(seed) & (2**64 - 1), _PREC[precision], pw, nw,
                                     _stream(), C.c_void_p(out.data_ptr()), C.byref(mean), C.byref(sem),
                                     C.byref(st)))
        return out, mean.value, sem.value, st.as_dict()

    def draws(self, c, n_samples, n_draws, seed, ws=None):
        """Draws of the seed path: int32 device tensor [n_samples, n_draws]."""
        nd = c.shape[0]
        pc = _dev(c, torch.float64, (nd,), "c")
        pw, nw = self._wsarg(ws)
        out = torch.empty((n_samples, n_draws), dtype=torch.int32, device=c.device)
        _check(lib().shci_pt2_draws(self._ptr, pc, nd, int(seed) & (2**64 - 1), int(n_samples), int(n_draws),
                                    pw, nw, _stream(), C.c_void_p(out.data_ptr())))
        return out

    def alias_table(self, c, ws=None):
        """(thresholds as int64 tensor with the uint64 bits, aliases int32) of the seed path."""
        nd = c.shape[0]
        pc = _dev(c, torch.float64, (nd,), "c")
        pw, nw = self._wsarg(ws)
        thr = torch.empty(nd, dtype=torch.int64, device=c.device)
        al = torch.empty(nd, dtype=torch.int32, device=c.device)
        _check(lib().shci_pt2_alias_table(self._ptr, pc, nd, pw, nw, _stream(), C.c_void_p(thr.data_ptr()),
                                          C.c_void_p(al.data_ptr())))
        return thr, al

    def sample_batched(self, dets, c, e0, eps2, eps2_d, draws, n_batches, sample_batch, precision="fp64", *,
                       seed=0, n_samples=None, n_draws=None, ws=None):
        """Stochastic estimates keeping one hash batch of P per sample (times
        n_batches); sample_batch None: batches from the seed."""
        pd, pc, nd = self._inputs(dets, c)
        pdr, ns, ndraw = self._draws_arg(draws, n_samples, n_draws)
        psb = C.c_void_p(None) if sample_batch is None else _dev(sample_batch, torch.int32, (ns,), "sample_batch")
        pw, nw = self._wsarg(ws)
        out = torch.empty(ns, dtype=torch.float64, device=c.device)
        mean = C.c_double()
        sem = C.c_double()
        st = Stats()
        _check(lib().shci_pt2_sample_batched(self._ptr, pd, pc, nd, float(e0), float(eps2), float(eps2_d),
                                             ns, ndraw, pdr, int(n_batches), psb, int(seed) & (2**64 - 1),
                                             _PREC[precision], pw, nw, _stream(), C.c_void_p(out.data_ptr()),
                                             C.byref(mean), C.byref(sem), C.byref(st)))
        return out, mean.value, sem.value, st.as_dict()

    def det_batches(self, dets, c, e0, eps2, eps2_hi, n_batches, batches, precision="fp64", ws=None):
        """Per-batch (sum, sum of squares, count of a, kept terms) of
        e_a = (A_a(eps2)^2 - A_a(eps2_hi)^2) / D_a for the listed hash batches."""
        pd, pc, nd = self._inputs(dets, c)
        pw, nw = self._wsarg(ws)
        bl = (C.c_int32 * len(batches))(*[int(b) for b in batches])
        out = (Batch * len(batches))()
        st = Stats()
        _check(lib().shci_pt2_det_batches(self._ptr, pd, pc, nd, float(e0), float(eps2), float(eps2_hi),
                                          int(n_batches), bl, len(batches), _PREC[precision], pw, nw, _stream(),
                                          out, C.byref(st)))
        return [(o.sum, o.sumsq, o.n_unique, o.n_terms) for o in out], st.as_dict()

    def select(self, dets, c, e0, eps_gen, mode="hci", threshold=0.0, cap=1 << 20, precision="fp64"):
        """New determinants from one pass: mode "hci" (every a reached with
        |H_ai c_i| > eps_gen; value A_a) or "cipsi" (|A_a^2/D_a| > threshold
        after preselection at eps_gen; value A_a^2/D_a).  Returns (keys
        int64 [m, 4], values [m])."""
        pd, pc, nd = self._inputs(dets, c)
        dev = c.device
        keys = torch.zeros((cap, 4), dtype=torch.int64, device=dev)
        vals = torch.zeros(cap, dtype=torch.float64, device=dev)
        n_out = C.c_int64()
        st = Stats()
        m = {"hci": 0, "cipsi": 1}[mode]
        _check(lib().shci_pt2_select(self._ptr, pd, pc, nd, float(e0), float(eps_gen), m, float(threshold),
                                     _PREC[precision], _stream(), C.c_void_p(keys.data_ptr()),
                                     C.c_void_p(vals.data_ptr()), cap, C.byref(n_out), C.byref(st)))
        k = n_out.value
        return keys[:k], vals[:k]

    def hc(self, dets, c):
        """y = H c on the variational space and <c|H|c>/<c|c>: returns
        (y tensor, connections per row tensor (int32 view of uint32), e_var,
        stats)."""
        pd, pc, nd = self._inputs(dets, c)
        y = torch.empty(nd, dtype=torch.float64, device=c.device)
        conn = torch.empty(nd, dtype=torch.int32, device=c.device)
        ev = C.c_double()
        st = Stats()
        _check(lib().shci_pt2_hc(self._ptr, pd, pc, nd, _stream(), C.c_void_p(y.data_ptr()),
                                 C.c_void_p(conn.data_ptr()), C.byref(ev), C.byref(st)))
        return y, conn, ev.value, st.as_dict()

    def three_step(self, dets, c, e0, eps2_dtm, eps2_psto, eps2, target_error, nb_psto, nb_sto, draws,
                   sample_batch, precision="fp64", *, seed=0, n_samples=None, n_draws=None, ws=None):
        """The 3-step correction; returns (result dict, per-sample tensor).
        draws / sample_batch None: made from the seed on the device."""
        pd, pc, nd = self._inputs(dets, c)
        pdr, ns, ndraw = self._draws_arg(draws, n_samples, n_draws)
        psb = C.c_void_p(None) if sample_batch is None else _dev(sample_batch, torch.int32, (ns,), "sample_batch")
        pw, nw = self._wsarg(ws)
        out = torch.empty(ns, dtype=torch.float64, device=c.device)
        res = ThreeStep()
        _check(lib().shci_pt2_three_step(self._ptr, pd, pc, nd, float(e0), float(eps2_dtm), float(eps2_psto),
                                         float(eps2), float(target_error), int(nb_psto), int(nb_sto), ns, ndraw,
                                         pdr, psb, int(seed) & (2**64 - 1), _PREC[precision], pw, nw, _stream(),
                                         C.c_void_p(out.data_ptr()), C.byref(res)))
        return res.as_dict(), out

    def sample_grad(self, dets, c, e0, eps2, eps2_d, draws, precision="fp64", *, seed=0, n_samples=None,
                    n_draws=None, ws=None):
        """Per-sample estimates and the adjoint of their mean: returns
        (per_sample, mean, sem, dE/dc tensor, dE/dE0, stats)."""
        pd, pc, nd = self._inputs(dets, c)
        pdr, ns, ndraw = self._draws_arg(draws, n_samples, n_draws)
        pw, nw = self._wsarg(ws)
        out = torch.empty(ns, dtype=torch.float64, device=c.device)
        g = torch.empty(nd, dtype=torch.float64, device=c.device)
        mean = C.c_double()
        sem = C.c_double()
        de0 = C.c_double()
        st = Stats()
        _check(lib().shci_pt2_sample_grad(self._ptr, pd, pc, nd, float(e0), float(eps2), float(eps2_d),
                                          ns, ndraw, pdr, int(seed) & (2**64 - 1), _PREC[precision], pw, nw,
                                          _stream(),
                                          C.c_void_p(out.data_ptr()), C.byref(mean), C.byref(sem),
                                          C.c_void_p(g.data_ptr()), C.byref(de0), C.byref(st)))
        return out, mean.value, sem.value, g, de0.value, st.as_dict()


def dets_tensor(dets_u64, device="cuda"):
    """numpy uint64 [N,4] -> int64 device tensor with the same bits."""
    import numpy as np
    a = np.ascontiguousarray(dets_u64, dtype=np.uint64).view(np.int64)
    return torch.from_numpy(a).to(device)


def dets_numpy(t: torch.Tensor):
    """int64 tensor -> numpy uint64 with the same bits."""
    return t.detach().cpu().numpy().view("uint64")
