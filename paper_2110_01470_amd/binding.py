"""ctypes binding of the C ABI in include/sso.h (libsso.so).

Argument marshalling only: every step of the optimiser runs in the HIP
kernels of libsso.so.  PyTorch supplies the device workspace (a uint8 tensor)
and the HIP stream, nothing else.  There is no CPU fallback: if libsso.so is
missing or no GPU is present, constructing a Swarm raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH

OK, E_INVAL, E_NOMEM, E_HIP, E_UNSUPPORTED, E_STATE = 0, -1, -2, -3, -4, -5
OBJ = {"sphere": 0, "ripple": 1, "dense": 2, "f1": 11, "f2": 12, "f3": 13, "f4": 14, "f5": 15,
       "f6": 16, "f7": 17, "f8": 18, "f9": 19}
ORDER_GPS, ORDER_EQ21 = 0, 1
ENGINE = {"auto": 0, "stream": 1, "resident": 2}
STORAGE = {"auto": 0, "f32": 1, "u24": 2}
CONTRACTION = {"auto": 0, "f32": 1, "bf16x3": 2, "f16x2": 3}


class SSOError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sso error {code}: {msg}")
        self.code = code
        self.msg = msg


class Config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("d", ctypes.c_uint32),
        ("lo", ctypes.c_float),
        ("hi", ctypes.c_float),
        ("cg", ctypes.c_double),
        ("cp", ctypes.c_double),
        ("cw", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("swarm_id", ctypes.c_uint32),
        ("kind", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("engine", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("lanes", ctypes.c_uint32),
        ("trace_cap", ctypes.c_uint32),
        ("s", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
        ("a", ctypes.c_void_p),
        ("polish_every", ctypes.c_uint32),
        ("polish_steps", ctypes.c_uint32),
        ("polish_lr", ctypes.c_float),
        ("contraction", ctypes.c_int32),
    ]


_lib = None


def load():
    """Load libsso.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    cfgp = ctypes.POINTER(Config)
    sig = {
        "sso_workspace_bytes": (ctypes.c_size_t, [cfgp]),
        "sso_init": (ctypes.c_int, [cfgp, P, ctypes.c_size_t, P, ctypes.POINTER(P)]),
        "sso_step": (ctypes.c_int, [P]),
        "sso_run": (ctypes.c_int, [P, u32]),
        "sso_get_best": (ctypes.c_int, [P, P, P, P, P]),
        "sso_get_state": (ctypes.c_int, [P, P, P, P, P]),
        "sso_set_state": (ctypes.c_int, [P, P, P, P, u64]),
        "sso_get_trace": (ctypes.c_int, [P, u64, u32, P, P, P]),
        "sso_debug_rng": (ctypes.c_int, [P, u64, P]),
        "sso_eval": (ctypes.c_int, [P, P, u32, P, P, P]),
        "sso_polish": (ctypes.c_int, [P, u32, ctypes.c_float, P]),
        "sso_destroy": (None, [P]),
        "sso_run_static": (ctypes.c_int, [cfgp, u32, P, P, P, P]),
        "sso_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "sso_last_error": (ctypes.c_char_p, [P]),
        "sso_get_mapping": (ctypes.c_int, [P, P, P, P, P]),
        "sso_batch_workspace_bytes": (ctypes.c_size_t, [cfgp, u32]),
        "sso_batch_init": (ctypes.c_int, [cfgp, u32, P, ctypes.c_size_t, P, ctypes.POINTER(P)]),
        "sso_batch_run": (ctypes.c_int, [P, u32]),
        "sso_batch_tune": (ctypes.c_int, [P, u32, P, P, P]),
        "sso_batch_set_mapping": (ctypes.c_int, [P, u32, u32]),
        "sso_batch_mapping": (ctypes.c_int, [P, P, P, P, P]),
        "sso_batch_get_results": (ctypes.c_int, [P, P, P, P, P]),
        "sso_batch_get_best": (ctypes.c_int, [P, u32, P, P, P]),
        "sso_batch_get_state": (ctypes.c_int, [P, u32, P, P, P, P]),
        "sso_batch_set_state": (ctypes.c_int, [P, u32, P, P, P, u64]),
        "sso_batch_get_trace": (ctypes.c_int, [P, u32, u64, u32, P, P, P]),
        "sso_batch_destroy": (None, [P]),
        "sso_batch_last_error": (ctypes.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def make_config(n, d, kind, lo, hi, cg, cp, cw, seed, s, w=None, a=None, swarm_id=0,
                order=ORDER_GPS, engine="auto", lanes=0, trace_cap=0, storage="auto",
                polish_every=0, polish_steps=0, polish_lr=0.0, contraction="auto"):
    """Returns (Config, keepalive) with host arrays pinned in `keepalive`."""
    s, w, a = _f32(s), _f32(w), _f32(a)
    cfg = Config(n=n, d=d, lo=lo, hi=hi, cg=cg, cp=cp, cw=cw, seed=seed, swarm_id=swarm_id,
                 kind=OBJ[kind] if isinstance(kind, str) else kind, order=order,
                 engine=ENGINE[engine] if isinstance(engine, str) else engine,
                 storage=STORAGE[storage] if isinstance(storage, str) else storage, lanes=lanes,
                 trace_cap=trace_cap, s=s.ctypes.data if s is not None else None,
                 w=w.ctypes.data if w is not None else None,
                 a=a.ctypes.data if a is not None else None, polish_every=polish_every,
                 polish_steps=polish_steps, polish_lr=polish_lr,
                 contraction=CONTRACTION[contraction] if isinstance(contraction, str) else contraction)
    return cfg, (s, w, a)


def workspace_bytes(cfg):
    lib = load()
    nbytes = lib.sso_workspace_bytes(ctypes.byref(cfg))
    if nbytes == 0:
        raise SSOError(E_INVAL, lib.sso_last_error(None).decode())
    return nbytes


STATIC_SCRATCH_BYTES = 64 * 1024 * 1024


def run_static(n, d, kind, lo, hi, cg, cp, cw, seed, s, w=None, generations=0, device="cuda",
               stream=None, **cfg_kw):
    """sso_run_static: initialise and run `generations` generations in the
    library's static device array (no workspace, no context), gBest written to
    device tensors.  Returns (g [d], fG, gidx) after synchronising the stream.
    Raises SSOError with the library's code (SSO_E_NOMEM when the swarm's state
    exceeds STATIC_SCRATCH_BYTES)."""
    import torch

    lib = load()
    cfg, keep = make_config(n, d, kind, lo, hi, cg, cp, cw, seed, s, w, **cfg_kw)
    dev = torch.device(device)
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    g = torch.empty(d, dtype=torch.float32, device=dev)
    f = torch.empty(1, dtype=torch.float32, device=dev)
    idx = torch.empty(1, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        rc = lib.sso_run_static(ctypes.byref(cfg), generations, ctypes.c_void_p(stream.cuda_stream),
                                g.data_ptr(), f.data_ptr(), idx.data_ptr())
    if rc != OK:
        raise SSOError(rc, lib.sso_last_error(None).decode())
    stream.synchronize()
    del keep
    return (g.cpu().numpy(), float(f.cpu()[0]), int(idx.cpu().numpy().view(np.uint32)[0]))


class Swarm:
    """One swarm on one GPU.  Mirrors sso_init / sso_step / sso_run /
    sso_get_best and the state, trace and RNG hooks."""

    def __init__(self, n, d, kind, lo, hi, cg, cp, cw, seed, s, w=None, a=None, swarm_id=0,
                 order=ORDER_GPS, engine="auto", lanes=0, trace_cap=0, storage="auto",
                 polish_every=0, polish_steps=0, polish_lr=0.0, contraction="auto",
                 device="cuda", stream=None):
        import torch

        self._lib = load()
        self.n, self.d = n, d
        self._cfg, self._keep = make_config(n, d, kind, lo, hi, cg, cp, cw, seed, s, w, a,
                                            swarm_id, order, engine, lanes, trace_cap, storage,
                                            polish_every, polish_steps, polish_lr, contraction)
        nbytes = workspace_bytes(self._cfg)
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # The kernels use the workspace on self.stream: once the tensor is
        # dropped, torch's allocator must not hand the memory out again before
        # the work queued there has finished.
        self.workspace.record_stream(self.stream)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self._lib.sso_init(ctypes.byref(self._cfg), self.workspace.data_ptr(), nbytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if rc != OK:
            raise SSOError(rc, self._lib.sso_last_error(None).decode())
        self._ctx = ctx

    def _check(self, rc):
        if rc != OK:
            raise SSOError(rc, self._lib.sso_last_error(self._ctx).decode())

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.sso_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self):
        self._check(self._lib.sso_step(self._ctx))
        return self

    def run(self, generations):
        self._check(self._lib.sso_run(self._ctx, generations))
        return self

    def mapping(self):
        """(engine, row storage, lanes per particle, dense contraction) the
        config resolved to, as names ("stream"/"resident", "f32"/"u24",
        lanes, "f32"/"bf16x3"/"f16x2")."""
        eng = ctypes.c_int()
        sto = ctypes.c_int()
        lanes = ctypes.c_uint32()
        con = ctypes.c_int()
        self._check(self._lib.sso_get_mapping(self._ctx, ctypes.byref(eng), ctypes.byref(sto),
                                              ctypes.byref(lanes), ctypes.byref(con)))
        names = {v: k for k, v in ENGINE.items()}
        stores = {v: k for k, v in STORAGE.items()}
        cons = {v: k for k, v in CONTRACTION.items()}
        return names[eng.value], stores[sto.value], int(lanes.value), cons[con.value]

    def best(self):
        """(g [d], fG, gidx, generations done)."""
        g = np.zeros(self.d, np.float32)
        f = ctypes.c_float()
        idx = ctypes.c_uint32()
        gen = ctypes.c_uint64()
        self._check(self._lib.sso_get_best(self._ctx, _ptr(g), ctypes.byref(f), ctypes.byref(idx),
                                           ctypes.byref(gen)))
        return g, float(f.value), int(idx.value), int(gen.value)

    def state(self):
        """(x [n,d], p [n,d], fp [n], t)."""
        x = np.zeros((self.n, self.d), np.float32)
        p = np.zeros((self.n, self.d), np.float32)
        fp = np.zeros(self.n, np.float32)
        t = ctypes.c_uint64()
        self._check(self._lib.sso_get_state(self._ctx, _ptr(x), _ptr(p), _ptr(fp),
                                            ctypes.byref(t)))
        return x, p, fp, int(t.value)

    def set_state(self, x, p, fp, t):
        x = _f32(x).reshape(self.n, self.d)
        p = _f32(p).reshape(self.n, self.d)
        fp = _f32(fp).reshape(self.n)
        self._check(self._lib.sso_set_state(self._ctx, _ptr(x), _ptr(p), _ptr(fp), t))
        return self

    def trace(self, first, count):
        """(fG [count], gidx [count], improved [count]) for generations first.."""
        fg = np.zeros(count, np.float32)
        gi = np.zeros(count, np.uint32)
        im = np.zeros(count, np.uint32)
        self._check(self._lib.sso_get_trace(self._ctx, first, count, _ptr(fg), _ptr(gi), _ptr(im)))
        return fg, gi, im

    def polish(self, steps, lr=0.0):
        """Gradient polish of every pBest (DENSE); returns the step size used."""
        used = ctypes.c_float()
        self._check(self._lib.sso_polish(self._ctx, steps, lr, ctypes.byref(used)))
        return float(used.value)

    def eval(self, x, gout=None, f=True, grad=False):
        """f and/or gout * grad f at the rows of x (an (m, d) float32 device
        tensor), computed by the library's kernels on this swarm's stream.
        Returns (f or None, grad or None) as device tensors."""
        import torch

        if x.dtype != torch.float32 or x.dim() != 2 or x.shape[1] != self.d or not x.is_cuda:
            raise ValueError("x must be an (m, d) float32 GPU tensor")
        x = x.contiguous()
        m = x.shape[0]
        fo = torch.empty(m, dtype=torch.float32, device=x.device) if f else None
        go = torch.empty_like(x) if grad else None
        if gout is not None:
            gout = gout.to(dtype=torch.float32).contiguous()
            if gout.shape != (m,):
                raise ValueError("gout must have shape (m,)")
        cur = torch.cuda.current_stream(x.device)
        self.stream.wait_stream(cur)
        self._check(self._lib.sso_eval(
            self._ctx, ctypes.c_void_p(x.data_ptr()), m,
            ctypes.c_void_p(gout.data_ptr()) if gout is not None else None,
            ctypes.c_void_p(fo.data_ptr()) if fo is not None else None,
            ctypes.c_void_p(go.data_ptr()) if go is not None else None))
        cur.wait_stream(self.stream)
        for tns in (x, gout, fo, go):
            if tns is not None:
                tns.record_stream(self.stream)
        return fo, go

    def rng_words_into(self, t, out, count=1):
        """Enqueue the device's Philox words of generations t .. t + count - 1
        into `out` (each overwriting the last), an int32 device tensor of
        n * d elements, on the swarm's stream, ordered after the work already
        queued on the current stream (no host wait).  count > 1 keeps the
        launches back to back, for timing the word kernel."""
        import torch

        if out.numel() != self.n * self.d or out.dtype.itemsize != 4 or not out.is_contiguous():
            raise ValueError("out must be a contiguous 4-byte tensor of n * d elements")
        cur = torch.cuda.current_stream(out.device)
        self.stream.wait_stream(cur)
        ptr = ctypes.c_void_p(out.data_ptr())
        for k in range(count):
            self._check(self._lib.sso_debug_rng(self._ctx, t + k, ptr))
        cur.wait_stream(self.stream)
        out.record_stream(self.stream)

    def debug_rng(self, t):
        """The device's Philox words of generation t, as an [n, d] uint32 array."""
        import torch

        out = torch.empty(self.n * self.d, dtype=torch.int32, device=self.device)
        self._check(self._lib.sso_debug_rng(self._ctx, t, ctypes.c_void_p(out.data_ptr())))
        self.stream.synchronize()
        return out.cpu().numpy().view(np.uint32).reshape(self.n, self.d)


# Candidate mapping rules of sso_batch_tune (target chunks per lane) and
# workgroup sizes (waves); it times every pair.
TUNE_CANDIDATES = (1, 2, 4, 8, 16)
TUNE_WAVES = (4, 8)


class Batch:
    """Many independent swarms advanced together (sso_batch_*).

    `swarms` is a list of dicts with the keyword arguments of make_config
    (n, d, kind, lo, hi, cg, cp, cw, seed, s, w, swarm_id, order, lanes,
    trace_cap, storage)."""

    def __init__(self, swarms, device="cuda", stream=None):
        import torch

        self._lib = load()
        self.count = len(swarms)
        self.sizes = [(int(sw["n"]), int(sw["d"])) for sw in swarms]
        arr = (Config * self.count)()
        self._keep = []
        for k, sw in enumerate(swarms):
            kw = dict(sw)
            cfg, keep = make_config(kw.pop("n"), kw.pop("d"), kw.pop("kind"), kw.pop("lo"),
                                    kw.pop("hi"), kw.pop("cg"), kw.pop("cp"), kw.pop("cw"),
                                    kw.pop("seed"), kw.pop("s"), kw.pop("w", None), None, **kw)
            arr[k] = cfg
            self._keep.append(keep)
        self._cfgs = arr
        nbytes = self._lib.sso_batch_workspace_bytes(arr, self.count)
        if nbytes == 0:
            raise SSOError(E_INVAL, self._lib.sso_batch_last_error(None).decode())
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace.record_stream(self.stream)  # as for Swarm
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self._lib.sso_batch_init(arr, self.count, self.workspace.data_ptr(), nbytes,
                                          ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(ctx))
        if rc != OK:
            raise SSOError(rc, self._lib.sso_batch_last_error(None).decode())
        self._ctx = ctx

    def _check(self, rc):
        if rc != OK:
            raise SSOError(rc, self._lib.sso_batch_last_error(self._ctx).decode())

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.sso_batch_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, generations):
        self._check(self._lib.sso_batch_run(self._ctx, generations))
        return self

    def step(self):
        return self.run(1)

    def tune(self, generations):
        """(chosen rule, chosen waves per workgroup, {(rule, waves): milliseconds})."""
        cpl = ctypes.c_uint32()
        waves = ctypes.c_uint32()
        ms = np.zeros(len(TUNE_CANDIDATES) * len(TUNE_WAVES), np.float32)
        self._check(self._lib.sso_batch_tune(self._ctx, generations, ctypes.byref(cpl),
                                             ctypes.byref(waves), _ptr(ms)))
        keys = [(r, w) for r in TUNE_CANDIDATES for w in TUNE_WAVES]
        return int(cpl.value), int(waves.value), dict(zip(keys, ms.tolist()))

    def set_mapping(self, rule, waves):
        """Use mapping rule `rule` and workgroups of `waves` waves; back to
        generation 0."""
        self._check(self._lib.sso_batch_set_mapping(self._ctx, rule, waves))

    def mapping(self):
        """(rule, waves per workgroup, lanes per particle of every swarm,
        workgroups per launch)."""
        cpl = ctypes.c_uint32()
        waves = ctypes.c_uint32()
        tiles = ctypes.c_uint32()
        lanes = np.zeros(self.count, np.uint32)
        self._check(self._lib.sso_batch_mapping(self._ctx, ctypes.byref(cpl), ctypes.byref(waves),
                                                _ptr(lanes), ctypes.byref(tiles)))
        return int(cpl.value), int(waves.value), lanes, int(tiles.value)

    def results(self):
        """(fG [count], gidx [count], improved [count], generations done)."""
        f = np.zeros(self.count, np.float32)
        gi = np.zeros(self.count, np.uint32)
        im = np.zeros(self.count, np.uint32)
        gen = ctypes.c_uint64()
        self._check(self._lib.sso_batch_get_results(self._ctx, _ptr(f), _ptr(gi), _ptr(im),
                                                    ctypes.byref(gen)))
        return f, gi, im, int(gen.value)

    def view(self, k):
        """Swarm k with the one-swarm read/write interface (no stepping)."""
        return _BatchSwarm(self, k)


class _BatchSwarm:
    def __init__(self, batch, k):
        self.batch, self.k = batch, k
        # An index out of range reaches the library, which rejects it.
        self.n, self.d = batch.sizes[k] if 0 <= k < batch.count else (1, 1)

    def _check(self, rc):
        self.batch._check(rc)

    def best(self):
        lib, ctx = self.batch._lib, self.batch._ctx
        g = np.zeros(self.d, np.float32)
        f = ctypes.c_float()
        idx = ctypes.c_uint32()
        self._check(lib.sso_batch_get_best(ctx, self.k, _ptr(g), ctypes.byref(f), ctypes.byref(idx)))
        _, _, _, gen = self.state(with_rows=False)
        return g, float(f.value), int(idx.value), gen

    def state(self, with_rows=True):
        lib, ctx = self.batch._lib, self.batch._ctx
        x = np.zeros((self.n, self.d), np.float32) if with_rows else None
        p = np.zeros((self.n, self.d), np.float32) if with_rows else None
        fp = np.zeros(self.n, np.float32)
        t = ctypes.c_uint64()
        self._check(lib.sso_batch_get_state(ctx, self.k, _ptr(x), _ptr(p), _ptr(fp),
                                            ctypes.byref(t)))
        return x, p, fp, int(t.value)

    def set_state(self, x, p, fp, t):
        lib, ctx = self.batch._lib, self.batch._ctx
        x = _f32(x).reshape(self.n, self.d)
        p = _f32(p).reshape(self.n, self.d)
        fp = _f32(fp).reshape(self.n)
        self._check(lib.sso_batch_set_state(ctx, self.k, _ptr(x), _ptr(p), _ptr(fp), t))
        return self

    def trace(self, first, count):
        lib, ctx = self.batch._lib, self.batch._ctx
        fg = np.zeros(count, np.float32)
        gi = np.zeros(count, np.uint32)
        im = np.zeros(count, np.uint32)
        self._check(lib.sso_batch_get_trace(ctx, self.k, first, count, _ptr(fg), _ptr(gi),
                                            _ptr(im)))
        return fg, gi, im


def dense_objective(x, swarm):
    """f(x) = ||A (x_i - s)||^2 for the rows of x, differentiable in x: the
    forward and the backward pass (2 A^T A (x - s) times the incoming
    gradient) run in the library's MFMA kernels (sso_eval)."""
    return _DenseObjective.apply(x, swarm)


def _make_dense_objective():
    import torch

    class DenseObjective(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, swarm):
            f, _ = swarm.eval(x, f=True, grad=False)
            ctx.save_for_backward(x)
            ctx.swarm = swarm
            return f

        @staticmethod
        def backward(ctx, gout):
            (x,) = ctx.saved_tensors
            _, gx = ctx.swarm.eval(x, gout=gout, f=False, grad=True)
            return gx, None

    return DenseObjective


class _LazyFunction:
    def __init__(self):
        self._fn = None

    def apply(self, *args):
        if self._fn is None:
            self._fn = _make_dense_objective()
        return self._fn.apply(*args)


_DenseObjective = _LazyFunction()
