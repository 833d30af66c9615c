"""ctypes binding of librr.so (C ABI in include/rr.h).  Argument marshalling only."""

import ctypes as C
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))

MODE_QUANTILE, MODE_THRESHOLD, MODE_CHI2_QUANTILE = 0, 1, 2
PREC_SPLIT_BF16, PREC_FP32, PREC_FIXED_I8, PREC_GRAM_BF16 = 0, 1, 2, 3
X_FP64, X_FP32 = 0, 1
METRIC_MAHALANOBIS, METRIC_DIAGONAL, METRIC_MAX_SMD = 0, 1, 2
STATUS = {0: "RR_OK", 1: "RR_E_ARG", 2: "RR_E_SINGULAR", 3: "RR_E_CAPACITY", 4: "RR_E_RANGE",
          5: "RR_E_OBS", 6: "RR_E_DEVICE", 7: "RR_E_UNSUPPORTED"}

# (name, restype, argtypes) of every exported symbol
_P, _I, _I64, _U64, _D = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double
SIGNATURES = [
    ("rr_prepare", _I, [_P, _I, _I64, _I64, _I64, _I64, _D, _P, C.POINTER(_P)]),
    ("rr_prepare_metric", _I, [_P, _I, _I64, _I64, _I64, _I64, _D, _I, _P, C.POINTER(_P)]),
    ("rr_free", None, [_P]),
    ("rr_last_error", C.c_char_p, []),
    ("rr_problem_n", _I64, [_P]),
    ("rr_problem_d", _I64, [_P]),
    ("rr_problem_n1", _I64, [_P]),
    ("rr_problem_lambda", _D, [_P]),
    ("rr_draw_balance", _I, [_P, _U64, _U64, _U64, _I, _D, _I, _P, _P, _P, _U64, C.POINTER(_U64), _P]),
    ("rr_draw_balance_async", _I, [_P, _U64, _U64, _U64, _I, _D, _I, _P, _P, _P, _U64, _P, _P, _P]),
    ("rr_draw_exact", _I, [_P, _I, _D, _I, _P, _P, _P, _U64, C.POINTER(_U64), _P]),
    ("rr_regenerate", _I, [_P, _U64, _I, _P, _U64, _P, _P]),
    ("rr_balance_keys", _I, [_P, _U64, _I, _P, _U64, _I, _P, _P, _P, _P]),
    ("rr_balance_keys_noalloc", _I, [_P, _U64, _I, _P, _U64, _I, _P, _P, _P, _P]),
    ("rr_rand_test", _I, [_P, _U64, _I, _P, _U64, _U64, _P, _P, _I64, _P, C.POINTER(_D), _P]),
    ("rr_rand_test_interval", _I, [_P, _U64, _I, _P, _U64, _U64, _P, _P, _I64, _D, _P, C.POINTER(_D), _P,
                                   C.POINTER(_I), _P]),
    ("rr_draw_balance_batched", _I, [_P, _I64, _P, _U64, _U64, _I, _D, _I, _P, _P, _U64, _P, _P]),
    ("rr_last_timing", _I, [C.POINTER(_D), C.POINTER(_D), C.POINTER(_D), C.POINTER(_I64), C.POINTER(_U64)]),
    ("rr_tune_report", _I, [C.c_char_p, _U64, C.POINTER(_U64)]),
    ("rr_diagnose", _I, [_I64, _I64, _I64, _D, _D, _D, _P]),
    ("rr_q_star", _I, [_I64, _I64, _I64, _D, _D, _D, _D, _D, _D, C.POINTER(_D)]),
    ("rr_realized_rmse", _I, [_I64, _I64, _I64, _D, _D, _D, C.POINTER(_D), C.POINTER(_D)]),
]


class _Design(C.Structure):
    _fields_ = [(name, C.c_double) for name in ("c_q", "a_q", "v_a", "expected_M", "rmse_reduction",
                                                "mse_complete", "mse_accept")]

_lib = None


class RRError(RuntimeError):
    def __init__(self, status, msg, count=None):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = STATUS.get(status, status)
        self.count = count


def lib_path():
    return os.environ.get("RR_LIB", os.path.join(HERE, "librr.so"))


def load():
    """Load librr.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        path = lib_path()
        if not os.path.exists(path):
            raise RuntimeError(f"librr.so not built ({path}); run paper_2501_07642_amd.build")
        lib = C.CDLL(path)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(status, count=None):
    if status != 0:
        raise RRError(status, load().rr_last_error().decode(), count)


def _torch():
    import torch
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def quantile_count(q, N):
    """k = ceil(q N (1 - 1e-12)) clamped to [1, N] (the library's count for q-quantile acceptance)."""
    return int(min(max(math.ceil(q * N * (1.0 - 1e-12)), 1), N))


class Problem:
    """Owns an rr_problem handle (rr_prepare / rr_free)."""

    def __init__(self, handle, device):
        self._h = handle
        self.device = device

    @property
    def handle(self):
        return self._h

    @property
    def n(self):
        return load().rr_problem_n(self._h)

    @property
    def d(self):
        return load().rr_problem_d(self._h)

    @property
    def n1(self):
        return load().rr_problem_n1(self._h)

    @property
    def lam(self):
        return load().rr_problem_lambda(self._h)

    def free(self):
        if self._h:
            load().rr_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def rr_prepare(X, n1, ridge_rel=0.0, metric=None):
    """Prepare a problem; metric None / METRIC_MAHALANOBIS whitens, METRIC_DIAGONAL standardises."""
    torch = _torch()
    if not X.is_cuda:
        raise ValueError("X must be a device tensor")
    X = X.contiguous()
    dt = {torch.float64: X_FP64, torch.float32: X_FP32}[X.dtype]
    n, d = X.shape
    h = C.c_void_p()
    if metric is None:
        _check(load().rr_prepare(_ptr(X), dt, n, d, d, n1, float(ridge_rel), _stream(), C.byref(h)))
    else:
        _check(load().rr_prepare_metric(_ptr(X), dt, n, d, d, n1, float(ridge_rel), int(metric), _stream(),
                                        C.byref(h)))
    return Problem(h, X.device)


def _draw_outputs(capacity, device):
    torch = _torch()
    keys = torch.empty(capacity, dtype=torch.int64, device=device)
    M = torch.empty(capacity, dtype=torch.float64, device=device)
    flags = torch.empty(capacity, dtype=torch.uint8, device=device)
    return keys, M, flags


def rr_draw_balance(P, seed, key_begin, num_draws, mode=MODE_QUANTILE, q_or_a=0.01,
                    precision=PREC_SPLIT_BF16, capacity=None):
    """Returns (keys int64 [K], M float64 [K], flags uint8 [K]) on the device (keys as uint64 bits)."""
    if capacity is None:
        capacity = quantile_count(q_or_a, num_draws) if mode == MODE_QUANTILE else num_draws
    keys, M, flags = _draw_outputs(max(capacity, 1), P.device)
    cnt = C.c_uint64()
    st = load().rr_draw_balance(P.handle, seed, key_begin, num_draws, mode, float(q_or_a), precision,
                                _ptr(keys), _ptr(M), _ptr(flags), capacity, C.byref(cnt), _stream())
    _check(st, cnt.value)
    k = cnt.value
    return keys[:k], M[:k], flags[:k]


def rr_draw_balance_async(P, seed, key_begin, num_draws, mode=MODE_QUANTILE, q_or_a=0.01,
                          precision=PREC_SPLIT_BF16, capacity=None, out=None):
    """Enqueues the pool on torch's current stream and returns (keys, M, flags, count, status) device
    tensors without waiting; count (int64 [1]) and status (int32 [1]) are written on the device.
    `out` may pass (keys, M, flags) tensors to fill instead of fresh ones."""
    torch = _torch()
    if capacity is None:
        capacity = quantile_count(q_or_a, num_draws) if mode == MODE_QUANTILE else num_draws
    keys, M, flags = out if out is not None else _draw_outputs(max(capacity, 1), P.device)
    count = torch.zeros(1, dtype=torch.int64, device=P.device)
    status = torch.full((1,), -1, dtype=torch.int32, device=P.device)
    _check(load().rr_draw_balance_async(P.handle, seed, key_begin, num_draws, mode, float(q_or_a), precision,
                                        _ptr(keys), _ptr(M), _ptr(flags), capacity, _ptr(count), _ptr(status),
                                        _stream()))
    return keys, M, flags, count, status


def rr_draw_exact(P, mode=MODE_QUANTILE, q_or_a=0.01, precision=PREC_SPLIT_BF16, capacity=None):
    if capacity is None:
        # the library rejects C(n, n1) >= 2^40 itself (RR_E_RANGE); cap the buffer request
        total = min(math.comb(P.n, P.n1), 1 << 31)
        capacity = quantile_count(q_or_a, total) if mode == MODE_QUANTILE else total
    keys, M, flags = _draw_outputs(max(capacity, 1), P.device)
    cnt = C.c_uint64()
    st = load().rr_draw_exact(P.handle, mode, float(q_or_a), precision, _ptr(keys), _ptr(M), _ptr(flags),
                              capacity, C.byref(cnt), _stream())
    _check(st, cnt.value)
    k = cnt.value
    return keys[:k], M[:k], flags[:k]


def rr_regenerate(P, seed, keys, exact=False):
    torch = _torch()
    keys = keys.contiguous()
    nw = (P.n + 31) // 32
    out = torch.empty((keys.numel(), nw), dtype=torch.int32, device=keys.device)
    _check(load().rr_regenerate(P.handle, seed, int(exact), _ptr(keys), keys.numel(), _ptr(out), _stream()))
    return out


def rr_balance_keys(P, seed, keys, precision=PREC_SPLIT_BF16, exact=False, want_m32=True, want_m64=True):
    torch = _torch()
    keys = keys.contiguous()
    K = keys.numel()
    m32 = torch.empty(K, dtype=torch.float32, device=keys.device) if want_m32 else None
    err = torch.empty(K, dtype=torch.float32, device=keys.device) if want_m32 else None
    m64 = torch.empty(K, dtype=torch.float64, device=keys.device) if want_m64 else None
    _check(load().rr_balance_keys(P.handle, seed, int(exact), _ptr(keys), K, precision, _ptr(m32), _ptr(err),
                                  _ptr(m64), _stream()))
    return m32, err, m64


def rr_balance_keys_noalloc(P, seed, keys, m32, err, m64, precision=PREC_SPLIT_BF16, exact=False):
    """The allocation-free variant: the caller passes the output tensors (or None); the call only
    enqueues work on torch's current stream."""
    keys = keys.contiguous()
    _check(load().rr_balance_keys_noalloc(P.handle, seed, int(exact), _ptr(keys), keys.numel(), precision,
                                          _ptr(m32), _ptr(err), _ptr(m64), _stream()))
    return m32, err, m64


def rr_rand_test(P, seed, keys, obs_index, Y, tau0, exact=False):
    """Returns (counts uint64-as-int64 tensor [G], tau_hat float)."""
    torch = _torch()
    keys = keys.contiguous()
    Y = Y.contiguous()
    tau = [float(t) for t in tau0]
    G = len(tau)
    taus = (C.c_double * max(G, 1))(*tau)
    counts = torch.empty(max(G, 1), dtype=torch.int64, device=keys.device)
    th = C.c_double()
    _check(load().rr_rand_test(P.handle, seed, int(exact), _ptr(keys), keys.numel(), obs_index, _ptr(Y),
                               C.cast(taus, C.c_void_p), G, _ptr(counts), C.byref(th), _stream()))
    return counts[:G], th.value


def rr_rand_test_interval(P, seed, keys, obs_index, Y, tau0, alpha=0.05, exact=False):
    """Returns (counts, tau_hat, (lo, hi), contiguous): the test plus its inversion over the grid."""
    torch = _torch()
    keys = keys.contiguous()
    Y = Y.contiguous()
    tau = [float(t) for t in tau0]
    G = len(tau)
    taus = (C.c_double * max(G, 1))(*tau)
    counts = torch.empty(max(G, 1), dtype=torch.int64, device=keys.device)
    th = C.c_double()
    ci = (C.c_double * 2)()
    contig = C.c_int()
    _check(load().rr_rand_test_interval(P.handle, seed, int(exact), _ptr(keys), keys.numel(), obs_index, _ptr(Y),
                                        C.cast(taus, C.c_void_p), G, float(alpha), _ptr(counts), C.byref(th),
                                        C.cast(ci, C.c_void_p), C.byref(contig), _stream()))
    return counts[:G], th.value, (ci[0], ci[1]), bool(contig.value)


def rr_draw_balance_batched(problems, seeds, key_begin, num_draws, mode=MODE_QUANTILE, q_or_a=0.01,
                            precision=PREC_SPLIT_BF16, capacity=None):
    """Returns a list of (keys, M) per problem."""
    torch = _torch()
    npb = len(problems)
    if npb == 0:
        return []
    if capacity is None:
        capacity = quantile_count(q_or_a, num_draws) if mode == MODE_QUANTILE else num_draws
    dev = problems[0].device
    keys = [torch.empty(max(capacity, 1), dtype=torch.int64, device=dev) for _ in range(npb)]
    Ms = [torch.empty(max(capacity, 1), dtype=torch.float64, device=dev) for _ in range(npb)]
    H = (C.c_void_p * npb)(*[p.handle for p in problems])
    S = (C.c_uint64 * npb)(*[int(s) for s in seeds])
    KP = (C.c_void_p * npb)(*[k.data_ptr() for k in keys])
    MP = (C.c_void_p * npb)(*[m.data_ptr() for m in Ms])
    cnt = (C.c_uint64 * npb)()
    _check(load().rr_draw_balance_batched(C.cast(H, C.c_void_p), npb, C.cast(S, C.c_void_p), key_begin,
                                          num_draws, mode, float(q_or_a), precision, C.cast(KP, C.c_void_p),
                                          C.cast(MP, C.c_void_p), capacity, C.cast(cnt, C.c_void_p), _stream()))
    return [(keys[i][:cnt[i]], Ms[i][:cnt[i]]) for i in range(npb)]


def rr_last_timing():
    t, ck, gk, nl, band = C.c_double(), C.c_double(), C.c_double(), C.c_int64(), C.c_uint64()
    _check(load().rr_last_timing(C.byref(t), C.byref(ck), C.byref(gk), C.byref(nl), C.byref(band)))
    return dict(total_ms=t.value, contract_ms=ck.value, gen_ms=gk.value, launches=nl.value, band=band.value)


def rr_tune_report():
    """The autotuner's choices of this process (dict parsed from the library's JSON report)."""
    import json
    need = C.c_uint64()
    load().rr_tune_report(None, 0, C.byref(need))
    buf = C.create_string_buffer(max(int(need.value), 1))
    _check(load().rr_tune_report(buf, len(buf), C.byref(need)))
    return json.loads(buf.value.decode())


def rr_diagnose(n1, n0, d, q, sigma=1.0, r2=0.0):
    """Design closed forms at acceptance probability q (host computation in the library)."""
    out = _Design()
    _check(load().rr_diagnose(n1, n0, d, float(q), float(sigma), float(r2), C.cast(C.byref(out), C.c_void_p)))
    return {name: getattr(out, name) for name, _ in _Design._fields_}


def rr_realized_rmse(n1, n0, d, M, sigma=1.0, r2=0.0):
    """(typical-orientation RMSE, Cauchy-Schwarz bound) of an assignment with balance M (chi^2 scale)."""
    t, b = C.c_double(), C.c_double()
    _check(load().rr_realized_rmse(n1, n0, d, float(M), float(sigma), float(r2), C.byref(t), C.byref(b)))
    return t.value, b.value


def rr_q_star(n1, n0, d, sigma, r2, tau, alpha=0.05, power=0.8, q_lo=1e-300):
    """Largest q meeting the power-derived RMSE target, or None when no q >= q_lo does."""
    q = C.c_double()
    st = load().rr_q_star(n1, n0, d, float(sigma), float(r2), float(tau), float(alpha), float(power),
                          float(q_lo), C.byref(q))
    if STATUS.get(st) == "RR_E_RANGE":
        return None
    _check(st)
    return q.value
