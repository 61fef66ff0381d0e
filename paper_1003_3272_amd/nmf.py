"""ctypes binding of the C ABI in include/nmf.h (argument marshalling only).

Every step of the factorization runs in the HIP library libnmf.so; this
module only converts torch CUDA tensors to device pointers and status codes to
exceptions.  There is no CPU fallback: if the library is missing, load()
raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmf.so")

NMF_OK = 0
NMF_ENOTCONVERGED = 1
NMF_EINVAL = -1
NMF_ENOMEM = -2
NMF_EDEVICE = -3
NMF_ENONFINITE = -4
NMF_EUNSUPPORTED = -5

FP32, BF16 = 0, 1
REL_CHANGE, GAP_NORMALIZED = 0, 1
MAX_RANK = 256
STAGES = ("gemm_vht", "update_w", "gram_w", "gemm_wtv", "update_h", "gram_h", "objective")

_PRECISION = {"fp32": FP32, "bf16": BF16}
_TOL = {"rel_change": REL_CHANGE, "gap": GAP_NORMALIZED, "gap_normalized": GAP_NORMALIZED}


class NmfOptions(ctypes.Structure):
    _fields_ = [
        ("precision", c_int32),
        ("tol_kind", c_int32),
        ("tol", c_double),
        ("check_every", c_int32),
        ("validate", c_int32),
        ("seed", c_uint64),
        ("use_graph", c_int32),
        ("reserved", c_int32),
    ]


class NmfError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} (status {status})")


_lib = None


def load(path: str = LIB_PATH):
    """Load libnmf.so and declare the C signatures.  Raises OSError when the
    library has not been built (run paper_1003_3272_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"HIP library not built: {path} is missing "
                      "(python paper_1003_3272_amd/build.py)")
    lib = ctypes.CDLL(path)
    P = c_void_p
    lib.nmf_default_options.argtypes = [POINTER(NmfOptions)]
    lib.nmf_default_options.restype = None
    lib.nmf_init.argtypes = [POINTER(P), P, c_int64, c_int64, c_int64, c_int32, P, P,
                             POINTER(NmfOptions), P]
    lib.nmf_init.restype = c_int32
    lib.nmf_step.argtypes = [P, c_int32]
    lib.nmf_step.restype = c_int32
    lib.nmf_update_w.argtypes = [P]
    lib.nmf_update_w.restype = c_int32
    lib.nmf_update_h.argtypes = [P]
    lib.nmf_update_h.restype = c_int32
    lib.nmf_objective.argtypes = [P, POINTER(c_double)]
    lib.nmf_objective.restype = c_int32
    lib.nmf_solve.argtypes = [P, c_int32, POINTER(c_int32), POINTER(c_double),
                              POINTER(c_double), c_int32]
    lib.nmf_solve.restype = c_int32
    lib.nmf_profile_start.argtypes = [P, c_int32]
    lib.nmf_profile_start.restype = c_int32
    lib.nmf_profile_stop.argtypes = [P, POINTER(c_double), POINTER(c_int32)]
    lib.nmf_profile_stop.restype = c_int32
    lib.nmf_mlp_create.argtypes = [POINTER(P), c_int32, c_int32, c_int32, c_int64, P, P, P, P, P]
    lib.nmf_mlp_create.restype = c_int32
    lib.nmf_mlp_predict.argtypes = [P, P, c_int64, c_int64, P]
    lib.nmf_mlp_predict.restype = c_int32
    lib.nmf_mlp_train_step.argtypes = [P, P, c_int64, c_int64, P, ctypes.c_float,
                                       POINTER(c_double)]
    lib.nmf_mlp_train_step.restype = c_int32
    lib.nmf_mlp_grads.argtypes = [P, P, c_int64, c_int64, P, P, P, P, P, POINTER(c_double)]
    lib.nmf_mlp_grads.restype = c_int32
    lib.nmf_mlp_get_params.argtypes = [P, P, P, P, P]
    lib.nmf_mlp_get_params.restype = c_int32
    lib.nmf_mlp_destroy.argtypes = [P]
    lib.nmf_mlp_destroy.restype = None
    lib.nmf_destroy.argtypes = [P]
    lib.nmf_destroy.restype = None
    lib.nmf_strerror.argtypes = [c_int32]
    lib.nmf_strerror.restype = ctypes.c_char_p
    lib.nmf_version.argtypes = []
    lib.nmf_version.restype = c_int32
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().nmf_strerror(int(status)).decode()


def options(precision="fp32", tol_kind="rel_change", tol=1e-9, check_every=1,
            validate=False, seed=0, use_graph=True) -> NmfOptions:
    o = NmfOptions()
    load().nmf_default_options(byref(o))
    o.precision = _PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.tol_kind = _TOL[tol_kind] if isinstance(tol_kind, str) else int(tol_kind)
    o.tol = float(tol)
    o.check_every = int(check_every)
    o.validate = 1 if validate else 0
    o.seed = int(seed)
    o.use_graph = 1 if use_graph else 0
    return o


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


class Nmf:
    """One factorization context over torch CUDA tensors.

    V: (p, n) float32 CUDA tensor with unit column stride (any row stride).
    W: (p, r) and H: (r, n) contiguous float32 CUDA tensors, updated in place.
    """

    def __init__(self, V, W, H, precision="fp32", tol_kind="rel_change", tol=1e-9,
                 check_every=1, validate=False, seed=0, use_graph=True, stream=None):
        import torch
        lib = load()
        for name, t in (("V", V), ("W", W), ("H", H)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
                raise TypeError(f"{name} must be a float32 CUDA tensor")
        if V.dim() != 2 or V.stride(1) != 1:
            raise ValueError("V must be 2-D with unit column stride")
        if not (W.is_contiguous() and H.is_contiguous()):
            raise ValueError("W and H must be contiguous")
        p, n = V.shape
        r = W.shape[1]
        if W.shape != (p, r) or H.shape != (r, n):
            raise ValueError("shape mismatch: need V (p, n), W (p, r), H (r, n)")
        self._keep = (V, W, H)
        self.V, self.W, self.H = V, W, H
        self.p, self.n, self.r = p, n, r
        self.opts = options(precision, tol_kind, tol, check_every, validate, seed, use_graph)
        self.stream = stream
        self._ctx = c_void_p()
        st = lib.nmf_init(byref(self._ctx), c_void_p(V.data_ptr()), p, n, V.stride(0), r,
                          c_void_p(W.data_ptr()), c_void_p(H.data_ptr()), byref(self.opts),
                          _stream_handle(stream))
        if st != NMF_OK:
            self._ctx = c_void_p()
            raise NmfError(st, "nmf_init")

    def _check(self, st, what):
        if st not in (NMF_OK, NMF_ENOTCONVERGED):
            raise NmfError(st, what)
        return st

    def step(self, iters: int = 1):
        self._check(load().nmf_step(self._ctx, int(iters)), "nmf_step")

    def update_w(self):
        self._check(load().nmf_update_w(self._ctx), "nmf_update_w")

    def update_h(self):
        self._check(load().nmf_update_h(self._ctx), "nmf_update_h")

    def objective(self) -> float:
        f = c_double()
        self._check(load().nmf_objective(self._ctx, byref(f)), "nmf_objective")
        return f.value

    def solve(self, max_iters: int, trace_len: int = 0):
        """Returns (converged, iters_done, f, trace list)."""
        it = c_int32()
        f = c_double()
        buf = (c_double * max(trace_len, 1))()
        st = load().nmf_solve(self._ctx, int(max_iters), byref(it), byref(f),
                              buf if trace_len > 0 else None, int(trace_len))
        self._check(st, "nmf_solve")
        ntr = 0
        if trace_len > 0:
            ce = self.opts.check_every
            ntr = min(trace_len, 1 + (it.value + ce - 1) // ce)
        return st == NMF_OK, it.value, f.value, [buf[i] for i in range(ntr)]

    def profile_start(self, max_records: int):
        self._check(load().nmf_profile_start(self._ctx, int(max_records)), "nmf_profile_start")

    def profile_stop(self):
        """Returns {stage: (total_ms, launches)} from the HIP-event profiler."""
        ms = (c_double * len(STAGES))()
        cnt = (c_int32 * len(STAGES))()
        self._check(load().nmf_profile_stop(self._ctx, ms, cnt), "nmf_profile_stop")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}

    def close(self):
        if self._ctx:
            load().nmf_destroy(self._ctx)
            self._ctx = c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t):
    return c_void_p(t.data_ptr())


class Mlp:
    """Warm-start network h0 = softplus(M2 relu(M1 v + b1) + b2) on the GPU.

    params: [M1 (hidden x p), b1, M2 (r x hidden), b2] float32 tensors (any
    device; copied to the GPU).  V arguments are (p, n) float32 CUDA tensors
    with unit column stride; H arguments are (r, n) contiguous.
    """

    def __init__(self, params, max_batch, stream=None):
        import torch
        lib = load()
        M1, b1, M2, b2 = (torch.as_tensor(x, dtype=torch.float32).cuda().contiguous()
                          for x in params)
        self.hidden, self.p = M1.shape
        self.r = M2.shape[0]
        self.stream = stream
        self._m = c_void_p()
        st = lib.nmf_mlp_create(byref(self._m), self.p, self.hidden, self.r, int(max_batch),
                                _ptr(M1), _ptr(b1), _ptr(M2), _ptr(b2), _stream_handle(stream))
        if st != NMF_OK:
            self._m = c_void_p()
            raise NmfError(st, "nmf_mlp_create")

    @staticmethod
    def _check(st, what):
        if st != NMF_OK:
            raise NmfError(st, what)

    def predict(self, V, H0=None):
        import torch
        n = V.shape[1]
        if H0 is None:
            H0 = torch.empty((self.r, n), dtype=torch.float32, device=V.device)
        self._check(load().nmf_mlp_predict(self._m, _ptr(V), n, V.stride(0), _ptr(H0)),
                    "nmf_mlp_predict")
        return H0

    def train_step(self, V, H, lr, want_loss=True):
        loss = c_double()
        self._check(load().nmf_mlp_train_step(self._m, _ptr(V), V.shape[1], V.stride(0), _ptr(H),
                                              float(lr), byref(loss) if want_loss else None),
                    "nmf_mlp_train_step")
        return loss.value if want_loss else None

    def grads(self, V, H):
        import torch
        dev = V.device
        g = [torch.empty((self.hidden, self.p), device=dev), torch.empty(self.hidden, device=dev),
             torch.empty((self.r, self.hidden), device=dev), torch.empty(self.r, device=dev)]
        loss = c_double()
        self._check(load().nmf_mlp_grads(self._m, _ptr(V), V.shape[1], V.stride(0), _ptr(H),
                                         *[_ptr(x) for x in g], byref(loss)), "nmf_mlp_grads")
        return g, loss.value

    def params(self):
        import torch
        out = [torch.empty((self.hidden, self.p), device="cuda"),
               torch.empty(self.hidden, device="cuda"),
               torch.empty((self.r, self.hidden), device="cuda"), torch.empty(self.r, device="cuda")]
        self._check(load().nmf_mlp_get_params(self._m, *[_ptr(x) for x in out]),
                    "nmf_mlp_get_params")
        return out

    def close(self):
        if self._m:
            load().nmf_mlp_destroy(self._m)
            self._m = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
