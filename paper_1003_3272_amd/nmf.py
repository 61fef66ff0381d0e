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
EUCLIDEAN, POISSON = 0, 1
MAX_RANK = 256
STAGES = ("gemm_vht", "update_w", "gram_w", "gemm_wtv", "update_h", "gram_h", "objective")

_PRECISION = {"fp32": FP32, "bf16": BF16}
_TOL = {"rel_change": REL_CHANGE, "gap": GAP_NORMALIZED, "gap_normalized": GAP_NORMALIZED}
_LOSS = {"euclidean": EUCLIDEAN, "poisson": POISSON, "kl": POISSON}


class NmfOptions(ctypes.Structure):
    _fields_ = [
        ("precision", c_int32),
        ("tol_kind", c_int32),
        ("tol", c_double),
        ("check_every", c_int32),
        ("validate", c_int32),
        ("seed", c_uint64),
        ("use_graph", c_int32),
        ("loss", c_int32),
    ]


class NmfProblem(ctypes.Structure):
    """One problem of the batched tier (device pointers, row-major)."""
    _fields_ = [("V", c_void_p), ("W", c_void_p), ("H", c_void_p), ("p", c_int64),
                ("n", c_int64), ("ldv", c_int64), ("r", c_int32), ("reserved", c_int32)]


BATCH_TABLE_LEN = 9


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
    lib.nmf_prepare_graphs.argtypes = [P]
    lib.nmf_prepare_graphs.restype = c_int32
    lib.nmf_update_w.argtypes = [P]
    lib.nmf_update_w.restype = c_int32
    lib.nmf_update_h.argtypes = [P]
    lib.nmf_update_h.restype = c_int32
    lib.nmf_objective.argtypes = [P, POINTER(c_double)]
    lib.nmf_objective.restype = c_int32
    lib.nmf_solve.argtypes = [P, c_int32, POINTER(c_int32), POINTER(c_double),
                              POINTER(c_double), c_int32]
    lib.nmf_solve.restype = c_int32
    lib.nmf_solve_qn.argtypes = [P, c_int32, c_int32, POINTER(c_int32), POINTER(c_int32),
                                 POINTER(c_double), POINTER(c_double), c_int32]
    lib.nmf_solve_qn.restype = c_int32
    lib.nmf_refit_w.argtypes = [P, ctypes.c_float]
    lib.nmf_refit_w.restype = c_int32
    lib.nmf_data_norm2.argtypes = [P, POINTER(c_double)]
    lib.nmf_data_norm2.restype = c_int32
    lib.nmf_profile_start.argtypes = [P, c_int32]
    lib.nmf_profile_start.restype = c_int32
    lib.nmf_profile_stop.argtypes = [P, POINTER(c_double), POINTER(c_int32)]
    lib.nmf_profile_stop.restype = c_int32
    lib.nmf_normalize_gauge.argtypes = [P, c_int64, c_int32, P, c_int64, P]
    lib.nmf_normalize_gauge.restype = c_int32
    lib.nmf_normalize_gauge_noalloc.argtypes = [P, c_int64, c_int32, P, c_int64, P]
    lib.nmf_normalize_gauge_noalloc.restype = c_int32
    lib.nmf_mlp_create.argtypes = [POINTER(P), c_int32, c_int32, c_int32, c_int64, P, P, P, P, P]
    lib.nmf_mlp_create.restype = c_int32
    lib.nmf_mlp_predict.argtypes = [P, P, c_int64, c_int64, P]
    lib.nmf_mlp_predict.restype = c_int32
    lib.nmf_mlp_train_step.argtypes = [P, P, c_int64, c_int64, P, c_int64, ctypes.c_float,
                                       POINTER(c_double)]
    lib.nmf_mlp_train_step.restype = c_int32
    lib.nmf_mlp_grads.argtypes = [P, P, c_int64, c_int64, P, c_int64, P, P, P, P,
                                  POINTER(c_double)]
    lib.nmf_mlp_grads.restype = c_int32
    lib.nmf_mlp_get_params.argtypes = [P, P, P, P, P]
    lib.nmf_mlp_get_params.restype = c_int32
    lib.nmf_ws_set_dictionary.argtypes = [P, P]
    lib.nmf_ws_set_dictionary.restype = c_int32
    lib.nmf_ws_predict.argtypes = [P, P, c_int64, c_int64, c_int64, P, P]
    lib.nmf_ws_predict.restype = c_int32
    lib.nmf_ws_train.argtypes = [P, POINTER(P), POINTER(P), c_int32, c_int64, c_int64, c_int64,
                                 c_int32, c_int32, ctypes.c_float, ctypes.c_float, c_uint64,
                                 POINTER(c_double)]
    lib.nmf_ws_train.restype = c_int32
    lib.nmf_mlp_destroy.argtypes = [P]
    lib.nmf_mlp_destroy.restype = None
    lib.nmf_destroy.argtypes = [P]
    lib.nmf_destroy.restype = None
    lib.nmf_batch_create.argtypes = [POINTER(P), POINTER(NmfProblem), c_int32, P]
    lib.nmf_batch_create.restype = c_int32
    for name in ("nmf_batch_load", "nmf_batch_check"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = c_int32
    lib.nmf_batch_step.argtypes = [P, c_int32]
    lib.nmf_batch_step.restype = c_int32
    lib.nmf_batch_objective.argtypes = [P, POINTER(c_double)]
    lib.nmf_batch_objective.restype = c_int32
    lib.nmf_batch_get_table.argtypes = [P, POINTER(c_int32)]
    lib.nmf_batch_get_table.restype = c_int32
    lib.nmf_batch_set_table.argtypes = [P, POINTER(c_int32)]
    lib.nmf_batch_set_table.restype = c_int32
    lib.nmf_batch_tune.argtypes = [P, c_int32, POINTER(c_double)]
    lib.nmf_batch_tune.restype = c_int32
    lib.nmf_batch_destroy.argtypes = [P]
    lib.nmf_batch_destroy.restype = None
    lib.nmf_batch_solve.argtypes = [POINTER(NmfProblem), c_int32, c_int32, POINTER(NmfOptions),
                                     POINTER(c_int32), POINTER(c_double), P]
    lib.nmf_batch_solve.restype = c_int32
    lib.nmf_pet_create.argtypes = [POINTER(P), P, c_int64, c_int64, P, c_int32, c_int32, c_double,
                                   P, c_int32, P]
    lib.nmf_pet_create.restype = c_int32
    lib.nmf_pet_layout.argtypes = [P, POINTER(c_int32)]
    lib.nmf_pet_layout.restype = c_int32
    lib.nmf_pet_step.argtypes = [P, c_int32]
    lib.nmf_pet_step.restype = c_int32
    lib.nmf_pet_objective.argtypes = [P, POINTER(c_double)]
    lib.nmf_pet_objective.restype = c_int32
    lib.nmf_pet_solve.argtypes = [P, c_int32, c_double, c_int32, POINTER(c_int32),
                                  POINTER(c_double)]
    lib.nmf_pet_solve.restype = c_int32
    lib.nmf_pet_solve_qn.argtypes = [P, c_int32, c_int32, c_double, c_int32, POINTER(c_int32),
                                     POINTER(c_int32), POINTER(c_double), POINTER(c_double),
                                     c_int32]
    lib.nmf_pet_solve_qn.restype = c_int32
    lib.nmf_pet_destroy.argtypes = [P]
    lib.nmf_pet_destroy.restype = None
    lib.nmf_ceiling.argtypes = [c_int32, P, c_int64, c_int32, POINTER(c_double), P]
    lib.nmf_ceiling.restype = c_int32
    lib.nmf_strerror.argtypes = [c_int32]
    lib.nmf_strerror.restype = ctypes.c_char_p
    lib.nmf_version.argtypes = []
    lib.nmf_version.restype = c_int32
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().nmf_strerror(int(status)).decode()


def options(precision="fp32", tol_kind="rel_change", tol=1e-9, check_every=1,
            validate=False, seed=0, use_graph=True, loss="euclidean") -> NmfOptions:
    o = NmfOptions()
    load().nmf_default_options(byref(o))
    o.precision = _PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.tol_kind = _TOL[tol_kind] if isinstance(tol_kind, str) else int(tol_kind)
    o.tol = float(tol)
    o.check_every = int(check_every)
    o.validate = 1 if validate else 0
    o.seed = int(seed)
    o.use_graph = 1 if use_graph else 0
    o.loss = _LOSS[loss] if isinstance(loss, str) else int(loss)
    return o


def normalize_gauge(W, H, stream=None):
    """In place: unit-norm columns of W (p x r), rows of H (r x n) rescaled."""
    st = load().nmf_normalize_gauge(c_void_p(W.data_ptr()), W.shape[0], W.shape[1],
                                    c_void_p(H.data_ptr()), H.shape[1], _stream_handle(stream))
    if st != NMF_OK:
        raise NmfError(st, "nmf_normalize_gauge")


def normalize_gauge_noalloc(W, H, stream=None):
    """normalize_gauge through the entry point that allocates no device
    memory (its scratch is a static device array shared by every call on the
    GPU: do not overlap calls on one GPU)."""
    st = load().nmf_normalize_gauge_noalloc(c_void_p(W.data_ptr()), W.shape[0], W.shape[1],
                                            c_void_p(H.data_ptr()), H.shape[1],
                                            _stream_handle(stream))
    if st != NMF_OK:
        raise NmfError(st, "nmf_normalize_gauge_noalloc")


CEILING_KINDS = {"hbm_read": 0, "mfma_f32": 1, "mfma_bf16": 2, "mfma_f64": 3, "fma_f64": 4,
                 "mfma_f32_32": 5, "mfma_bf16_32": 6}


def ceiling(kind, buf, reps=10, stream=None):
    """Measured rate of the current device for one kind of CEILING_KINDS
    (bytes/s for hbm_read, flop/s otherwise); buf is a CUDA tensor of at
    least 64 MiB whose contents are overwritten."""
    rate = c_double(0.0)
    st = load().nmf_ceiling(CEILING_KINDS[kind] if isinstance(kind, str) else int(kind),
                            c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                            int(reps), byref(rate), _stream_handle(stream))
    if st != NMF_OK:
        raise NmfError(st, "nmf_ceiling")
    return rate.value


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


class Nmf:
    """One factorization context over torch CUDA tensors (loss "euclidean":
    the multiplicative update of ||V - W H||^2; "poisson": the square-root
    update of the Poisson log-likelihood, whose objective() returns L).

    V: (p, n) float32 CUDA tensor with unit column stride (any row stride).
    W: (p, r) and H: (r, n) contiguous float32 CUDA tensors, updated in place.
    """

    def __init__(self, V, W, H, precision="fp32", tol_kind="rel_change", tol=1e-9,
                 check_every=1, validate=False, seed=0, use_graph=True, stream=None,
                 loss="euclidean"):
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
        self.opts = options(precision, tol_kind, tol, check_every, validate, seed, use_graph,
                            loss)
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

    def prepare_graphs(self):
        """Capture the iteration graphs now (no device work; W, H unchanged)."""
        self._check(load().nmf_prepare_graphs(self._ctx), "nmf_prepare_graphs")

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

    def solve_qn(self, max_iters: int, q: int = 4, trace_len: int = 0):
        """QN(q)-accelerated solve (nmf_solve_qn).  Returns (converged,
        map evaluations, accepted QN steps, f, trace list)."""
        it, acc, f = c_int32(), c_int32(), c_double()
        buf = (c_double * max(trace_len, 1))()
        st = load().nmf_solve_qn(self._ctx, int(q), int(max_iters), byref(it), byref(acc),
                                 byref(f), buf if trace_len > 0 else None, int(trace_len))
        self._check(st, "nmf_solve_qn")
        ntr = min(trace_len, 1 + it.value // 2) if trace_len > 0 else 0
        return st == NMF_OK, it.value, acc.value, f.value, [buf[i] for i in range(ntr)]

    def refit_w(self, floor_rel: float = 1e-3):
        """W <- max(V H^T (H H^T + delta I)^-1, floor_rel * max W): the
        least-squares dictionary for the current H (asynchronous)."""
        self._check(load().nmf_refit_w(self._ctx, float(floor_rel)), "nmf_refit_w")

    def data_norm2(self) -> float:
        """||V||_F^2 (float64), as used by the gap stopping rule."""
        v = c_double()
        self._check(load().nmf_data_norm2(self._ctx, byref(v)), "nmf_data_norm2")
        return v.value

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


def _check_rows(V, H):
    """Training batches: float32 device matrices with unit column stride and
    the same number of columns."""
    import torch
    for x, name in ((V, "V"), (H, "H")):
        if x.dtype != torch.float32 or not x.is_cuda or x.dim() != 2 or x.stride(1) != 1:
            raise ValueError(f"{name} must be a 2-D float32 device tensor with unit column stride")
    if V.shape[1] != H.shape[1]:
        raise ValueError("V and H must have the same number of columns")


class Mlp:
    """Warm-start network h0 = softplus(M2 relu(M1 v + b1) + b2) on the GPU.

    params: [M1 (hidden x p), b1, M2 (r x hidden), b2] float32 tensors (any
    device; copied to the GPU).  V and training-target H arguments are (p, n)
    and (r, n) float32 CUDA tensors with unit column stride (column slices of
    wider matrices are accepted); predict's output H0 is contiguous.
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
        _check_rows(V, H)
        self._check(load().nmf_mlp_train_step(self._m, _ptr(V), V.shape[1], V.stride(0), _ptr(H),
                                              H.stride(0), float(lr),
                                              byref(loss) if want_loss else None),
                    "nmf_mlp_train_step")
        return loss.value if want_loss else None

    def grads(self, V, H):
        import torch
        dev = V.device
        g = [torch.empty((self.hidden, self.p), device=dev), torch.empty(self.hidden, device=dev),
             torch.empty((self.r, self.hidden), device=dev), torch.empty(self.r, device=dev)]
        loss = c_double()
        _check_rows(V, H)
        self._check(load().nmf_mlp_grads(self._m, _ptr(V), V.shape[1], V.stride(0), _ptr(H),
                                         H.stride(0), *[_ptr(x) for x in g], byref(loss)),
                    "nmf_mlp_grads")
        return g, loss.value

    def set_dictionary(self, Wbar):
        """Store the mean dictionary W-bar (p x r float32 CUDA tensor) that
        ws_predict hands out as W0."""
        import torch
        if Wbar.dtype != torch.float32 or not Wbar.is_cuda or tuple(Wbar.shape) != (self.p, self.r):
            raise ValueError(f"W-bar must be a ({self.p}, {self.r}) float32 CUDA tensor")
        self._wbar = Wbar.contiguous()
        self._check(load().nmf_ws_set_dictionary(self._m, _ptr(self._wbar)),
                    "nmf_ws_set_dictionary")

    def ws_predict(self, V, W0=None, H0=None):
        """Warm start for V (p, n): returns (W0 = W-bar, H0 = network(V))."""
        import torch
        p, n = V.shape
        if W0 is None:
            W0 = torch.empty((self.p, self.r), dtype=torch.float32, device=V.device)
        if H0 is None:
            H0 = torch.empty((self.r, n), dtype=torch.float32, device=V.device)
        self._check(load().nmf_ws_predict(self._m, _ptr(V), p, n, V.stride(0), _ptr(W0),
                                          _ptr(H0)), "nmf_ws_predict")
        return W0, H0

    def train_loop(self, Vs, Hs, epochs, lr, batch, decay=1.0, seed=0):
        """The library's training loop (nmf_ws_train) over the pairs
        (Vs[i], Hs[i]); returns the mean minibatch loss of every epoch."""
        if len(Vs) != len(Hs) or not Vs:
            raise ValueError("need as many target matrices as input matrices")
        n, ldv, ldh = Vs[0].shape[1], Vs[0].stride(0), Hs[0].stride(0)
        for V, H in zip(Vs, Hs):
            _check_rows(V, H)
            if V.shape != (self.p, n) or H.shape != (self.r, n) or V.stride(0) != ldv \
                    or H.stride(0) != ldh:
                raise ValueError("all matrices need the same shapes and row strides")
        vp = (c_void_p * len(Vs))(*[V.data_ptr() for V in Vs])
        hp = (c_void_p * len(Hs))(*[H.data_ptr() for H in Hs])
        losses = (c_double * int(epochs))()
        self._check(load().nmf_ws_train(self._m, vp, hp, len(Vs), n, ldv, ldh, int(epochs),
                                        int(batch), float(lr), float(decay), int(seed), losses),
                    "nmf_ws_train")
        return list(losses)

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


def _problem_list(problems):
    """NmfProblem array from (V, W, H) float32 device tensors: V (p, n) with
    unit column stride, W (p, r) and H (r, n) contiguous."""
    import torch
    arr = (NmfProblem * len(problems))()
    for i, (V, W, H) in enumerate(problems):
        for x, name in ((V, "V"), (W, "W"), (H, "H")):
            if x.dtype != torch.float32 or not x.is_cuda or x.dim() != 2:
                raise ValueError(f"problem {i}: {name} must be a 2-D float32 device tensor")
        if V.stride(1) != 1 or not W.is_contiguous() or not H.is_contiguous():
            raise ValueError(f"problem {i}: V needs unit column stride, W and H contiguous")
        p, n = V.shape
        r = W.shape[1]
        if W.shape[0] != p or H.shape != (r, n):
            raise ValueError(f"problem {i}: shapes V {tuple(V.shape)}, W {tuple(W.shape)}, "
                             f"H {tuple(H.shape)} do not match")
        arr[i] = NmfProblem(V.data_ptr(), W.data_ptr(), H.data_ptr(), p, n, V.stride(0), r, 0)
    return arr


def batch_solve(problems, max_iters, tol_kind="rel_change", tol=1e-9, check_every=1,
                validate=False, seed=0, stream=None):
    """nmf_batch_solve: solve every (V, W, H) of the list (W, H updated in
    place) until every problem meets the stopping rule or max_iters.
    Returns (converged, iters_done, objectives)."""
    import numpy as np
    arr = _problem_list(problems)
    opts = options("fp32", tol_kind, tol, check_every, validate, seed, True)
    it = c_int32()
    out = (c_double * len(problems))()
    st = load().nmf_batch_solve(arr, len(problems), int(max_iters), byref(opts), byref(it), out,
                                _stream_handle(stream))
    if st not in (NMF_OK, NMF_ENOTCONVERGED):
        raise NmfError(st, "nmf_batch_solve")
    return st == NMF_OK, it.value, np.array(out[:], dtype=np.float64)


class Batch:
    """Batched tier: many independent problems (V_b, W_b, H_b) advanced by one
    persistent kernel launch per step call.  W_b and H_b are read at
    creation (and by load()) and overwritten in place after every step."""

    def __init__(self, problems, stream=None):
        self._refs = [tuple(t) for t in problems]
        self.count = len(self._refs)
        arr = _problem_list(self._refs)
        self._b = c_void_p()
        st = load().nmf_batch_create(byref(self._b), arr, self.count, _stream_handle(stream))
        if st != NMF_OK:
            self._b = c_void_p()
            raise NmfError(st, "nmf_batch_create")

    @staticmethod
    def _check(st, what):
        if st != NMF_OK:
            raise NmfError(st, what)

    def step(self, iters=1):
        self._check(load().nmf_batch_step(self._b, int(iters)), "nmf_batch_step")

    def load(self):
        self._check(load().nmf_batch_load(self._b), "nmf_batch_load")

    def check(self):
        self._check(load().nmf_batch_check(self._b), "nmf_batch_check")

    def objective(self):
        import numpy as np
        out = (c_double * self.count)()
        self._check(load().nmf_batch_objective(self._b, out), "nmf_batch_objective")
        return np.array(out[:], dtype=np.float64)

    @property
    def table(self):
        t = (c_int32 * BATCH_TABLE_LEN)()
        self._check(load().nmf_batch_get_table(self._b, t), "nmf_batch_get_table")
        return list(t)

    @table.setter
    def table(self, values):
        t = (c_int32 * BATCH_TABLE_LEN)(*[int(v) for v in values])
        self._check(load().nmf_batch_set_table(self._b, t), "nmf_batch_set_table")

    def save_table(self, path):
        """Write the installed tile table to a JSON file (to install it again
        with load_table instead of re-tuning)."""
        import json
        with open(path, "w") as fh:
            json.dump({"nmf_batch_table": self.table}, fh)

    def load_table(self, path):
        """Install a tile table written by save_table."""
        import json
        with open(path) as fh:
            self.table = json.load(fh)["nmf_batch_table"]

    def tune(self, trial_iters=5):
        """Autotune the tile table on this batch; returns ms per iteration of
        the table it installs."""
        ms = c_double()
        self._check(load().nmf_batch_tune(self._b, int(trial_iters), byref(ms)), "nmf_batch_tune")
        return ms.value

    def close(self):
        if self._b:
            load().nmf_batch_destroy(self._b)
            self._b = c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pet:
    """Penalized PET reconstruction (Algorithm 2) on the GPU: E (d, p) and
    y (d,) float32 CUDA tensors, lam (p,) float32 CUDA tensor updated in
    place, p = rows * cols pixels in row-major order."""

    LAYOUTS = {"auto": 0, "dense": 1, "sparse": 2}

    def __init__(self, E, y, lam, rows, cols, mu, layout="auto", stream=None):
        import torch
        for name, t in (("E", E), ("y", y), ("lam", lam)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 \
                    or not t.is_contiguous():
                raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
        d, p = E.shape
        if y.shape != (d,) or lam.shape != (p,):
            raise ValueError("shapes: E (d, p), y (d,), lam (p,)")
        self._keep = (E, y, lam)
        self._m = c_void_p()
        st = load().nmf_pet_create(byref(self._m), _ptr(E), d, p, _ptr(y), int(rows), int(cols),
                                   float(mu), _ptr(lam), self.LAYOUTS[layout],
                                   _stream_handle(stream))
        if st != NMF_OK:
            self._m = c_void_p()
            raise NmfError(st, "nmf_pet_create")

    def _check(self, st, what):
        if st not in (NMF_OK, NMF_ENOTCONVERGED):
            raise NmfError(st, what)
        return st

    @property
    def layout(self):
        v = c_int32()
        self._check(load().nmf_pet_layout(self._m, byref(v)), "nmf_pet_layout")
        return {1: "dense", 2: "sparse"}[v.value]

    def step(self, iters=1):
        self._check(load().nmf_pet_step(self._m, int(iters)), "nmf_pet_step")

    def objective(self):
        f = c_double()
        self._check(load().nmf_pet_objective(self._m, byref(f)), "nmf_pet_objective")
        return f.value

    def solve(self, max_iters, tol=1e-9, check_every=1):
        """Returns (converged, iterations, f)."""
        it, f = c_int32(), c_double()
        st = self._check(load().nmf_pet_solve(self._m, int(max_iters), float(tol),
                                              int(check_every), byref(it), byref(f)),
                         "nmf_pet_solve")
        return st == NMF_OK, it.value, f.value

    def solve_qn(self, max_evals, q=10, tol=1e-9, check_every=2, trace_len=0):
        """QN(q)-accelerated solve; returns (converged, evaluations,
        accepted, f, trace)."""
        ev, acc, f = c_int32(), c_int32(), c_double()
        tr = (c_double * max(trace_len, 1))()
        st = self._check(load().nmf_pet_solve_qn(self._m, int(q), int(max_evals), float(tol),
                                                 int(check_every), byref(ev), byref(acc),
                                                 byref(f), tr if trace_len > 0 else None,
                                                 int(trace_len)), "nmf_pet_solve_qn")
        n = min(trace_len, 1 + ev.value // 2)
        return st == NMF_OK, ev.value, acc.value, f.value, list(tr[:n])

    def close(self):
        if self._m:
            load().nmf_pet_destroy(self._m)
            self._m = c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
