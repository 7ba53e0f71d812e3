"""ctypes binding of libpmc (include/pmc.h): argument marshalling only.

Every computation happens in the HIP library; this module converts Python
values to the C structs, passes device pointers of torch tensors through,
and raises PmcError on a negative status.  Importing it fails loudly if the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(or python paper_2108_03076_amd/build.py)")

# torch (the source of device buffers and streams) ships its own HIP runtime;
# load it first so that the library binds to that same runtime instead of
# initialising a second one in the process (which then finds no device).
try:
    import torch  # noqa: F401
except ImportError:
    pass

lib = C.CDLL(LIB_PATH)

STATUS = {0: "OK", -1: "E_ARG", -2: "E_PARSE", -3: "E_TYPE", -4: "E_TENV", -5: "E_HORIZON",
          -6: "E_NOT_PD", -7: "E_UNSUPPORTED", -8: "E_HIP", -9: "E_OOM"}
RNG = {"philox": 0, "sobol": 1}
PREC = {"f32": 0, "f64": 1}
MODE = {"auto": 0, "two_phase": 1, "fused": 2}
ENGINE = {"auto": 0, "interpreter": 1, "compiled": 2}


class PmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Gbm(C.Structure):
    _fields_ = [("n_assets", C.c_int), ("spot", C.POINTER(C.c_double)), ("vol", C.POINTER(C.c_double)),
                ("corr", C.POINTER(C.c_double)), ("rate", C.c_double), ("years_per_day", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("n_paths", C.c_uint64), ("rng", C.c_int), ("seed", C.c_uint64), ("instance", C.c_uint32),
                ("precision", C.c_int), ("t_now", C.c_int32), ("party_from", C.c_char_p),
                ("party_to", C.c_char_p), ("mode", C.c_int), ("payoffs_dev", C.c_void_p), ("block", C.c_int),
                ("engine", C.c_int), ("history", C.POINTER(C.c_double)), ("history_len", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("price", C.c_double), ("std_err", C.c_double), ("sum", C.c_double), ("sum_sq", C.c_double),
                ("n_paths", C.c_uint64), ("path_dates", C.c_uint64), ("n_slots", C.c_int),
                ("mode_used", C.c_int), ("ms", C.c_double), ("gen_ms", C.c_double), ("eval_ms", C.c_double),
                ("engine_used", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Batch(C.Structure):
    _fields_ = [("n_inst", C.c_int), ("tenv", C.POINTER(C.c_int32)), ("params", C.POINTER(C.c_double)),
                ("per_instance_model", C.c_int), ("spot", C.POINTER(C.c_double)),
                ("vol", C.POINTER(C.c_double)), ("corr", C.POINTER(C.c_double)),
                ("instance_ids", C.POINTER(C.c_uint32))]


class PayoffInfo(C.Structure):
    _fields_ = [("n_instr", C.c_int), ("n_regs", C.c_int), ("loop_depth", C.c_int),
                ("n_time_exprs", C.c_int), ("n_parties", C.c_int), ("n_assets", C.c_int),
                ("n_params", C.c_int), ("n_tvars", C.c_int)]


class RiskOpts(C.Structure):
    _fields_ = [("rel_spot_bump", C.c_double), ("abs_vol_bump", C.c_double)]


class Greeks(C.Structure):
    _fields_ = [("price", C.c_double), ("std_err", C.c_double), ("delta", C.c_double * 4),
                ("gamma", C.c_double * 4), ("vega", C.c_double * 4), ("ms", C.c_double)]


class TrainOpts(C.Structure):
    _fields_ = [("batch", C.c_int), ("lr_max", C.c_double), ("lr_min", C.c_double),
                ("total_steps", C.c_int64), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("eager", C.c_int)]


_vp, _i, _u64, _i64 = C.c_void_p, C.c_int, C.c_uint64, C.c_int64
_sig = {
    "pmc_version": (C.c_char_p, []),
    "pmc_ctx_create": (_i, [_i, _vp, C.POINTER(_vp)]),
    "pmc_ctx_destroy": (None, [_vp]),
    "pmc_last_error": (C.c_char_p, [_vp]),
    "pmc_payoff_load": (_i, [_vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_char_p), _i, C.POINTER(C.c_char_p), _i,
                             C.POINTER(C.c_char_p), _i, C.POINTER(_vp)]),
    "pmc_payoff_free": (None, [_vp]),
    "pmc_contract_compile": (_i, [C.c_char_p, C.c_size_t, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "pmc_contract_load": (_i, [_vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_char_p), _i, C.POINTER(C.c_char_p), _i,
                               C.POINTER(C.c_char_p), _i, C.POINTER(_vp)]),
    "pmc_payoff_source": (_i, [_vp, C.POINTER(C.c_int32), C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "pmc_payoff_cut": (_i, [_vp, _vp, C.POINTER(_vp)]),
    "pmc_payoff_get_info": (_i, [_vp, C.POINTER(PayoffInfo)]),
    "pmc_payoff_grid": (_i, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _i, C.POINTER(_i), C.POINTER(_i)]),
    "pmc_payoff_streams": (_i, [_vp, C.POINTER(C.c_int32), C.c_int32, C.POINTER(_i)]),
    "pmc_price": (_i, [_vp, _vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(Gbm), C.POINTER(Opts),
                       C.POINTER(Result)]),
    "pmc_price_noalloc": (_i, [_vp, _vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(Gbm),
                               C.POINTER(Opts), C.POINTER(Result)]),
    "pmc_price_batch": (_i, [_vp, _vp, C.POINTER(Batch), C.POINTER(Gbm), C.POINTER(Opts), C.POINTER(Result)]),
    "pmc_risk_batch": (_i, [_vp, _vp, C.POINTER(Batch), C.POINTER(Gbm), C.POINTER(Opts), C.POINTER(RiskOpts),
                            C.POINTER(Greeks)]),
    "pmc_autotune_batch": (_i, [_vp, _vp, C.POINTER(Batch), C.POINTER(Gbm), C.POINTER(Opts), C.c_char_p,
                                C.POINTER(_i), C.POINTER(_i), C.POINTER(_i)]),
    "pmc_gen_paths": (_i, [_vp, _vp, C.POINTER(C.c_int32), C.POINTER(Gbm), C.POINTER(Opts), _vp, _vp, _vp]),
    "pmc_eval_paths": (_i, [_vp, _vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(Gbm),
                            C.POINTER(Opts), _vp, C.POINTER(Result)]),
    "pmc_probe_valu": (_i, [_vp, _i, C.POINTER(C.c_double)]),
    "pmc_cholesky": (_i, [_vp, C.POINTER(C.c_double), _i, _i, C.POINTER(C.c_double)]),
    "pmc_mlp_create": (_i, [_vp, _i, _i, _u64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                            C.POINTER(_vp)]),
    "pmc_mlp_free": (None, [_vp]),
    "pmc_mlp_num_params": (_i64, [_vp]),
    "pmc_mlp_save": (_i, [_vp, C.c_char_p]),
    "pmc_mlp_load": (_i, [_vp, C.c_char_p, C.POINTER(_vp)]),
    "pmc_mlp_get_params": (_i, [_vp, C.POINTER(C.c_float)]),
    "pmc_mlp_set_params": (_i, [_vp, C.POINTER(C.c_float)]),
    "pmc_mlp_train_epoch": (_i, [_vp, _vp, _vp, _i64, C.POINTER(TrainOpts), C.POINTER(C.c_double)]),
    "pmc_mlp_infer": (_i, [_vp, _vp, _vp, _i64]),
    "pmc_mlp_price": (_i, [_vp, C.POINTER(C.c_double), _i64, _vp, C.POINTER(Batch), C.POINTER(Gbm),
                           C.POINTER(Opts), C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "pmc_mlp_loss_grad": (_i, [_vp, _vp, _vp, _i64, C.POINTER(C.c_double), C.POINTER(C.c_float)]),
}
EXPORTED = []
for _name, (_res, _args) in _sig.items():
    if hasattr(lib, _name):
        _f = getattr(lib, _name)
        _f.restype, _f.argtypes = _res, _args
        EXPORTED.append(_name)


def _strs(xs):
    arr = (C.c_char_p * max(1, len(xs)))()
    for i, x in enumerate(xs):
        arr[i] = x.encode()
    return arr


def _dbl(xs):
    a = np.ascontiguousarray(np.asarray(xs, dtype=np.float64).reshape(-1))
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i32(xs):
    a = np.ascontiguousarray(np.asarray(xs, dtype=np.int32).reshape(-1))
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A pmc_ctx on one device and stream (torch's current stream by default)."""

    def __init__(self, device=0, stream=None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        st = lib.pmc_ctx_create(int(device), C.c_void_p(stream), C.byref(h))
        if st != 0:
            msg = lib.pmc_last_error(None)
            raise PmcError(st, "pmc_ctx_create failed: " + (msg.decode() if msg else ""))
        self.h = h
        self._keep = []

    def close(self):
        if self.h:
            lib.pmc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st):
        if st != 0:
            raise PmcError(st, lib.pmc_last_error(self.h).decode())

    def load(self, il, assets, params=(), tvars=()):
        return Payoff(self, il, assets, params, tvars)

    def probe_valu(self, kind):
        """Sustained vector-ALU lane operations per second for one instruction
        class (pmc_probe_valu): 0 FP32 FMA, 1 int32 xor+add, 2 v_mad_u64_u32
        + add, 3 FP32 exp2 + multiply, 4 FP32 FMA and int32 xor interleaved."""
        out = C.c_double()
        self.check(lib.pmc_probe_valu(self.h, int(kind), C.byref(out)))
        return out.value

    def cholesky(self, mats):
        m = np.ascontiguousarray(np.asarray(mats, dtype=np.float64))
        n, k = (1, m.shape[0]) if m.ndim == 2 else (m.shape[0], m.shape[1])
        out = np.zeros_like(m)
        self.check(lib.pmc_cholesky(self.h, m.ctypes.data_as(C.POINTER(C.c_double)), n, k,
                                    out.ctypes.data_as(C.POINTER(C.c_double))))
        return out


class _NoContext:
    """Stand-in for calls that need no device (loading, grid queries)."""
    h = None

    @staticmethod
    def check(st):
        if st != 0:
            raise PmcError(st, lib.pmc_last_error(None).decode())


class Payoff:
    def __init__(self, ctx, il: str, assets, params=(), tvars=()):
        self.h = None
        self.ctx = ctx if ctx is not None else _NoContext()
        self.assets, self.params, self.tvars = list(assets), list(params), list(tvars)
        h = C.c_void_p()
        b = il.encode()
        a, p, t = _strs(self.assets), _strs(self.params), _strs(self.tvars)
        self.ctx.check(lib.pmc_payoff_load(self.ctx.h, b, len(b), a, len(self.assets), p, len(self.params), t,
                                           len(self.tvars), C.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if self.h:
                lib.pmc_payoff_free(self.h)
                self.h = None
        except Exception:
            pass

    def info(self):
        o = PayoffInfo()
        self.ctx.check(lib.pmc_payoff_get_info(self.h, C.byref(o)))
        return {k: getattr(o, k) for k, _ in o._fields_}

    def cut(self):
        """The time-parameterised payoff (cutPayoff, Sec. 4.1)."""
        h = C.c_void_p()
        self.ctx.check(lib.pmc_payoff_cut(self.ctx.h, self.h, C.byref(h)))
        new = Payoff.__new__(Payoff)
        new.h, new.ctx = h, self.ctx
        new.assets, new.params, new.tvars = self.assets, self.params, self.tvars
        return new

    def source(self, tenv=None):
        """Device source of the compiled engine for this payoff: generic, or
        generated for one template environment (pmc_payoff_source)."""
        tp = None
        if tenv is not None:
            t, tp = _i32(tenv if len(tenv) else [0])
        n = C.c_size_t()
        self.ctx.check(lib.pmc_payoff_source(self.h, tp, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value + 1)
        self.ctx.check(lib.pmc_payoff_source(self.h, tp, buf, n.value + 1, C.byref(n)))
        return buf.value.decode()

    def streams(self, tenv=(), sim_from=0):
        """pmc_payoff_streams: whether the expression reads its dates in
        non-decreasing order for this environment (paths can be streamed)."""
        t, tp = _i32(tenv if len(tenv) else [0])
        out = C.c_int()
        self.ctx.check(lib.pmc_payoff_streams(self.h, tp, int(sim_from), C.byref(out)))
        return bool(out.value)

    def grid(self, tenv=()):
        t, tp = _i32(tenv if len(tenv) else [0])
        n, hz = C.c_int(), C.c_int()
        self.ctx.check(lib.pmc_payoff_grid(self.h, tp, None, 0, C.byref(n), C.byref(hz)))
        days = np.zeros(max(1, n.value), dtype=np.int32)
        self.ctx.check(lib.pmc_payoff_grid(self.h, tp, days.ctypes.data_as(C.POINTER(C.c_int32)),
                                           days.size, C.byref(n), C.byref(hz)))
        return days[:n.value].tolist(), hz.value


def compile_contract(cl_text):
    """Payoff-language text of a contract-language contract
    (pmc_contract_compile)."""
    b = cl_text.encode()
    n = C.c_size_t()
    _NoContext.check(lib.pmc_contract_compile(b, len(b), None, 0, C.byref(n)))
    buf = C.create_string_buffer(n.value + 1)
    _NoContext.check(lib.pmc_contract_compile(b, len(b), buf, n.value + 1, C.byref(n)))
    return buf.value.decode()


def load_contract(cl_text, assets, params=(), tvars=(), ctx=None):
    """A payoff loaded from contract-language text (pmc_contract_load)."""
    c = ctx if ctx is not None else _NoContext()
    new = Payoff.__new__(Payoff)
    new.h = None
    new.ctx = c
    new.assets, new.params, new.tvars = list(assets), list(params), list(tvars)
    h = C.c_void_p()
    b = cl_text.encode()
    a, p, t = _strs(new.assets), _strs(new.params), _strs(new.tvars)
    c.check(lib.pmc_contract_load(c.h, b, len(b), a, len(new.assets), p, len(new.params), t, len(new.tvars),
                                  C.byref(h)))
    new.h = h
    return new


def load_payoff(il, assets, params=(), tvars=(), ctx=None):
    """Load a payoff expression; ctx may be None (no device needed)."""
    return Payoff(ctx, il, assets, params, tvars)


def make_model(spot, vol, corr=None, rate=0.03, years_per_day=1.0):
    """Gbm struct plus the arrays it points to (keep the tuple alive)."""
    s, sp = _dbl(spot)
    v, vp = _dbl(vol)
    keep = [s, v]
    cp = None
    if corr is not None:
        c, cp = _dbl(corr)
        keep.append(c)
    g = Gbm(int(s.size), sp, vp, cp, float(rate), float(years_per_day))
    return g, keep


def make_opts(n_paths, rng="philox", seed=42, instance=0, precision="f32", t_now=0, parties=("X", "Y"),
              mode="auto", payoffs=None, block=0, engine="auto", history=None):
    """Opts struct; history (optional) is [n_assets][n] prices on days
    t_now - n + 1 .. t_now (kept alive by the struct)."""
    hp, hl, keep = None, 0, None
    if history is not None:
        keep = np.ascontiguousarray(np.asarray(history, dtype=np.float64))
        hl = int(keep.shape[-1]) if keep.ndim else 1
        hp = keep.ctypes.data_as(C.POINTER(C.c_double))
    o = Opts(int(n_paths), RNG[rng], int(seed), int(instance), PREC[precision], int(t_now),
             parties[0].encode(), parties[1].encode(), MODE[mode], _ptr(payoffs), int(block), ENGINE[engine],
             hp, hl)
    o._history = keep
    return o


def price(payoff: Payoff, tenv=(), params=(), *, spot, vol, corr=None, rate=0.03, years_per_day=1.0, **opts):
    g, keep = make_model(spot, vol, corr, rate, years_per_day)
    o = make_opts(**opts)
    t, tp = _i32(tenv if len(tenv) else [0])
    p, pp = _dbl(params if len(params) else [0.0])
    r = Result()
    payoff.ctx.check(lib.pmc_price(payoff.ctx.h, payoff.h, tp, pp, C.byref(g), C.byref(o), C.byref(r)))
    return r.as_dict()


def price_noalloc(payoff: Payoff, tenv=(), params=(), *, spot, vol, corr=None, rate=0.03, years_per_day=1.0,
                  **opts):
    """pmc_price_noalloc: pmc_price by the interpreter, fused, with no device
    allocation (the library's static per-device scratch)."""
    g, keep = make_model(spot, vol, corr, rate, years_per_day)
    o = make_opts(**opts)
    t, tp = _i32(tenv if len(tenv) else [0])
    p, pp = _dbl(params if len(params) else [0.0])
    r = Result()
    payoff.ctx.check(lib.pmc_price_noalloc(payoff.ctx.h, payoff.h, tp, pp, C.byref(g), C.byref(o), C.byref(r)))
    return r.as_dict()


class Pricer:
    """A prepared pmc_price call: the arguments are marshalled once and each
    call runs one complete pricing through the C ABI (for timing loops)."""

    def __init__(self, payoff: Payoff, tenv=(), params=(), *, spot, vol, corr=None, rate=0.03,
                 years_per_day=1.0, **opts):
        self.payoff = payoff
        self.g, self._keep = make_model(spot, vol, corr, rate, years_per_day)
        self.o = make_opts(**opts)
        self.t, tp = _i32(tenv if len(tenv) else [0])
        self.p, pp = _dbl(params if len(params) else [0.0])
        self.r = Result()
        self._args = (payoff.ctx.h, payoff.h, tp, pp, C.byref(self.g), C.byref(self.o), C.byref(self.r))

    def __call__(self):
        st = lib.pmc_price(*self._args)
        if st != 0:
            self.payoff.ctx.check(st)
        return self.r


class Surrogate:
    """The learned surrogate (pmc_mlp_*): an MLP n_in -> width x 3 -> 1 trained
    and evaluated by the library's BF16 matrix-core kernels."""

    def __init__(self, ctx: Context, lo, hi, y_scale=100.0, width=256, seed=0):
        lo_a, lo_p = _dbl(lo)
        hi_a, hi_p = _dbl(hi)
        self.ctx, self.n_in = ctx, int(lo_a.size)
        h = C.c_void_p()
        ctx.check(lib.pmc_mlp_create(ctx.h, self.n_in, int(width), int(seed), lo_p, hi_p, float(y_scale),
                                     C.byref(h)))
        self.h = h
        self.n_params = int(lib.pmc_mlp_num_params(h))

    def save(self, path):
        """Writes the network to a file (pmc_mlp_save)."""
        self.ctx.check(lib.pmc_mlp_save(self.h, str(path).encode()))

    @classmethod
    def load(cls, ctx: Context, path):
        """A network read back from a pmc_mlp_save file (pmc_mlp_load)."""
        h = C.c_void_p()
        ctx.check(lib.pmc_mlp_load(ctx.h, str(path).encode(), C.byref(h)))
        self = cls.__new__(cls)
        self.ctx, self.h = ctx, h
        self.n_params = int(lib.pmc_mlp_num_params(h))
        return self

    def __del__(self):
        try:
            if self.h:
                lib.pmc_mlp_free(self.h)
                self.h = None
        except Exception:
            pass

    def get_params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        self.ctx.check(lib.pmc_mlp_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_params(self, p):
        a = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        self.ctx.check(lib.pmc_mlp_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float))))

    def train_epoch(self, x, y, batch=4096, lr_max=1e-3, lr_min=1e-5, total_steps=1, beta1=0.9, beta2=0.999,
                    eps=1e-8, eager=False):
        o = TrainOpts(int(batch), float(lr_max), float(lr_min), int(total_steps), float(beta1), float(beta2),
                      float(eps), int(bool(eager)))
        loss = C.c_double()
        self.ctx.check(lib.pmc_mlp_train_epoch(self.h, _ptr(x), _ptr(y), int(y.numel()), C.byref(o),
                                               C.byref(loss)))
        return loss.value

    def infer(self, x, y):
        self.ctx.check(lib.pmc_mlp_infer(self.h, _ptr(x), _ptr(y), int(y.numel())))

    def price(self, x, payoff, tenv, params, *, spot, vol, corr=None, rate=0.03, years_per_day=1.0,
              per_instance_model=False, instance_ids=None, **opts):
        """pmc_mlp_price: the network's price for points inside its input box,
        Monte Carlo (instance i of the batch tenv/params/model) outside it.
        Returns (price [n], Monte Carlo standard error [n] (0 for network
        prices), route [n]: 0 network, 1 Monte Carlo)."""
        xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        n = int(xa.shape[0])
        b, nb, keep = _batch(payoff, tenv, params, spot, vol, corr, per_instance_model, instance_ids)
        A = len(payoff.assets)
        if per_instance_model:
            g, keep2 = make_model([100.0] * A, [0.0] * A, None, rate, years_per_day)
        else:
            g, keep2 = make_model(spot, vol, corr, rate, years_per_day)
        o = make_opts(**opts)
        pr = np.zeros(n)
        se = np.zeros(n)
        route = np.zeros(n, dtype=np.int32)
        self.ctx.check(lib.pmc_mlp_price(self.h, xa.ctypes.data_as(C.POINTER(C.c_double)), n, payoff.h, C.byref(b),
                                         C.byref(g), C.byref(o), pr.ctypes.data_as(C.POINTER(C.c_double)),
                                         se.ctypes.data_as(C.POINTER(C.c_double)),
                                         route.ctypes.data_as(C.POINTER(C.c_int))))
        return pr, se, route

    def loss_grad(self, x, y):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_double()
        self.ctx.check(lib.pmc_mlp_loss_grad(self.h, _ptr(x), _ptr(y), int(y.numel()), C.byref(loss),
                                             g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, g


def eval_paths(payoff: Payoff, paths, tenv=(), params=(), *, spot, vol, corr=None, rate=0.03,
               years_per_day=1.0, **opts):
    g, keep = make_model(spot, vol, corr, rate, years_per_day)
    o = make_opts(**opts)
    t, tp = _i32(tenv if len(tenv) else [0])
    p, pp = _dbl(params if len(params) else [0.0])
    r = Result()
    payoff.ctx.check(lib.pmc_eval_paths(payoff.ctx.h, payoff.h, tp, pp, C.byref(g), C.byref(o), _ptr(paths),
                                        C.byref(r)))
    return r.as_dict()


def gen_paths(payoff: Payoff, paths, words=None, normals=None, tenv=(), *, spot, vol, corr=None, rate=0.03,
              years_per_day=1.0, **opts):
    g, keep = make_model(spot, vol, corr, rate, years_per_day)
    o = make_opts(**opts)
    t, tp = _i32(tenv if len(tenv) else [0])
    payoff.ctx.check(lib.pmc_gen_paths(payoff.ctx.h, payoff.h, tp, C.byref(g), C.byref(o), _ptr(paths),
                                       _ptr(words), _ptr(normals)))


def _batch(payoff, tenv, params, spot, vol, corr, per_instance_model, instance_ids):
    n = int(np.asarray(tenv).reshape(len(tenv), -1).shape[0]) if len(payoff.tvars) else int(len(params))
    keep = []
    t, tp = _i32(tenv) if len(payoff.tvars) else (None, None)
    p, pp = _dbl(params) if len(payoff.params) else (None, None)
    keep += [t, p]
    sp = vp = cp = ip = None
    if per_instance_model:
        s, sp = _dbl(spot)
        v, vp = _dbl(vol)
        keep += [s, v]
        if corr is not None:
            c, cp = _dbl(corr)
            keep.append(c)
    if instance_ids is not None:
        ids = np.ascontiguousarray(np.asarray(instance_ids, dtype=np.uint32))
        ip = ids.ctypes.data_as(C.POINTER(C.c_uint32))
        keep.append(ids)
    b = Batch(n, tp, pp, 1 if per_instance_model else 0, sp, vp, cp, ip)
    return b, n, keep


def price_batch(payoff: Payoff, tenv, params, *, spot, vol, corr=None, rate=0.03, years_per_day=1.0,
                per_instance_model=False, instance_ids=None, **opts):
    """tenv [n_inst][n_tvars], params [n_inst][n_params]; shared model unless
    per_instance_model (then spot/vol [n_inst][A], corr [n_inst][A][A])."""
    b, n, keep = _batch(payoff, tenv, params, spot, vol, corr, per_instance_model, instance_ids)
    A = len(payoff.assets)
    if per_instance_model:
        g, keep2 = make_model([100.0] * A, [0.0] * A, None, rate, years_per_day)
    else:
        g, keep2 = make_model(spot, vol, corr, rate, years_per_day)
    o = make_opts(**opts)
    out = (Result * n)()
    payoff.ctx.check(lib.pmc_price_batch(payoff.ctx.h, payoff.h, C.byref(b), C.byref(g), C.byref(o), out))
    return [r.as_dict() for r in out]


class BatchPricer:
    """A prepared pmc_price_batch call: the arguments are marshalled once
    and each call runs one complete batched pricing through the C ABI,
    leaving the raw results in `out` (for timing loops; `results()` turns
    them into the dicts price_batch returns)."""

    def __init__(self, payoff: Payoff, tenv, params, *, spot, vol, corr=None, rate=0.03, years_per_day=1.0,
                 per_instance_model=False, instance_ids=None, **opts):
        self.payoff = payoff
        self.b, self.n, self._keep = _batch(payoff, tenv, params, spot, vol, corr, per_instance_model, instance_ids)
        A = len(payoff.assets)
        if per_instance_model:
            self.g, self._keep2 = make_model([100.0] * A, [0.0] * A, None, rate, years_per_day)
        else:
            self.g, self._keep2 = make_model(spot, vol, corr, rate, years_per_day)
        self.o = make_opts(**opts)
        self.out = (Result * self.n)()
        self._args = (payoff.ctx.h, payoff.h, C.byref(self.b), C.byref(self.g), C.byref(self.o), self.out)

    def __call__(self):
        st = lib.pmc_price_batch(*self._args)
        if st != 0:
            self.payoff.ctx.check(st)
        return self.out

    def results(self):
        return [r.as_dict() for r in self.out]


def risk_batch(payoff: Payoff, tenv, params, *, spot, vol, corr=None, rate=0.03, years_per_day=1.0,
               per_instance_model=False, instance_ids=None, rel_spot_bump=0.01, abs_vol_bump=0.01, **opts):
    """Bump-and-revalue Greeks of every instance on common random numbers
    (pmc_risk_batch): a list of dicts with price, std_err, delta[A],
    gamma[A], vega[A] and ms."""
    b, n, keep = _batch(payoff, tenv, params, spot, vol, corr, per_instance_model, instance_ids)
    A = len(payoff.assets)
    if per_instance_model:
        g, keep2 = make_model([100.0] * A, [0.0] * A, None, rate, years_per_day)
    else:
        g, keep2 = make_model(spot, vol, corr, rate, years_per_day)
    o = make_opts(**opts)
    r = RiskOpts(float(rel_spot_bump), float(abs_vol_bump))
    out = (Greeks * n)()
    payoff.ctx.check(lib.pmc_risk_batch(payoff.ctx.h, payoff.h, C.byref(b), C.byref(g), C.byref(o), C.byref(r),
                                        out))
    return [{"price": x.price, "std_err": x.std_err, "delta": list(x.delta)[:A], "gamma": list(x.gamma)[:A],
             "vega": list(x.vega)[:A], "ms": x.ms} for x in out]


def autotune_batch(payoff: Payoff, tenv, params, *, spot, vol, corr=None, rate=0.03, years_per_day=1.0,
                   per_instance_model=False, instance_ids=None, cache_path=None, **opts):
    b, n, keep = _batch(payoff, tenv, params, spot, vol, corr, per_instance_model, instance_ids)
    A = len(payoff.assets)
    if per_instance_model:
        g, keep2 = make_model([100.0] * A, [0.0] * A, None, rate, years_per_day)
    else:
        g, keep2 = make_model(spot, vol, corr, rate, years_per_day)
    o = make_opts(**opts)
    bl, pp, ln = C.c_int(), C.c_int(), C.c_int()
    payoff.ctx.check(lib.pmc_autotune_batch(payoff.ctx.h, payoff.h, C.byref(b), C.byref(g), C.byref(o),
                                            cache_path.encode() if cache_path else None, C.byref(bl),
                                            C.byref(pp), C.byref(ln)))
    return bl.value, pp.value, ln.value
