"""MI355X (gfx950) solver for the ENDGame Helmholtz pressure-correction system  A x = b.

Thin ctypes binding over ``libendgame.so`` (the C ABI declared in ``include/endgame.h``).  It
only marshals arguments: every step of the solve runs in the library's HIP kernels.  PyTorch
supplies device memory and the stream (``torch.cuda.current_stream()``).  There is no CPU
fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libendgame.so")

# enum eg_mode
FP64, FP32_IR, FP32_IR_BF16, FP32_IR_FP16, LEARNED_FP64, LEARNED_FP32_IR, FP32_MP = range(7)
MODE_NAMES = {FP64: "fp64", FP32_IR: "fp32_ir", FP32_IR_BF16: "fp32_ir_bf16", FP32_IR_FP16: "fp32_ir_fp16",
              LEARNED_FP64: "learned_fp64", LEARNED_FP32_IR: "learned_fp32_ir", FP32_MP: "fp32_mp"}
# enum eg_prec
PREC_FP64, PREC_FP32, PREC_BF16, PREC_FP16 = range(4)
# enum eg_status
CONVERGED, MAXIT, BREAKDOWN, STALLED = 0, 1, 2, 3
EINVAL, ENOMEM, EHIP, ENONFINITE, ENOPC = -1, -2, -3, -4, -5

EXPORTED = ["eg_create_operator", "eg_solve", "eg_get_info", "eg_residual_history", "eg_set_stream", "eg_set_option",
            "eg_apply", "eg_apply_precond", "eg_residual", "eg_dot", "eg_get_shape", "eg_destroy_operator",
            "eg_last_error", "eg_kernel_stats", "eg_reset_kernel_stats", "eg_net_create", "eg_net_destroy",
            "eg_net_set_weights", "eg_net_get_weights", "eg_attach_learned_pc", "eg_net_apply", "eg_net_loss_grad",
            "eg_harvest", "eg_harvest_krylov", "eg_net_train", "eg_net_eval", "eg_net_set_loss",
            "eg_train_learned_pc", "eg_save_learned_pc", "eg_load_learned_pc", "eg_get_learned_pc",
            "eg_dot_noalloc"]
PC_IMAGE_BYTES = 16 + 4 * 15233
N_NET_PARAMS = 15233
# enum eg_kernel
K_THOMAS_P, K_SPMV_V, K_THOMAS_S, K_SPMV_T, K_UPDATE, K_RESIDUAL, K_SOR_P, K_SOR_S = range(8)


class EndgameError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"endgame error {code}: {msg}")
        self.code = code


class _Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("outer_steps", ctypes.c_int), ("restarts", ctypes.c_int),
                ("fallbacks", ctypes.c_int), ("true_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


@dataclass
class SolveInfo:
    status: int
    iterations: int
    outer_steps: int
    restarts: int
    fallbacks: int
    true_rel_residual: float
    seconds: float


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load ``libendgame.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1811_03852_amd.build`")
    lib = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    sig = {
        "eg_create_operator": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "eg_solve": ([vp, vp, vp, ctypes.c_double, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "eg_get_info": ([vp, ctypes.POINTER(_Info)], ctypes.c_int),
        "eg_residual_history": ([vp, dp, ctypes.c_int], ctypes.c_int),
        "eg_set_stream": ([vp, vp], ctypes.c_int),
        "eg_set_option": ([vp, ctypes.c_char_p, ctypes.c_double], ctypes.c_int),
        "eg_apply": ([vp, vp, vp, ctypes.c_int], ctypes.c_int),
        "eg_apply_precond": ([vp, vp, vp, ctypes.c_int], ctypes.c_int),
        "eg_residual": ([vp, vp, vp, vp, dp], ctypes.c_int),
        "eg_dot": ([vp, vp, vp, ctypes.c_long, ctypes.c_int, dp], ctypes.c_int),
        "eg_get_shape": ([vp, ip, ip, ip], ctypes.c_int),
        "eg_destroy_operator": ([vp], None),
        "eg_last_error": ([], ctypes.c_char_p),
        "eg_kernel_stats": ([vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_long), dp], ctypes.c_int),
        "eg_reset_kernel_stats": ([vp], ctypes.c_int),
        "eg_net_create": ([ctypes.c_ulonglong, ctypes.POINTER(vp)], ctypes.c_int),
        "eg_net_destroy": ([vp], None),
        "eg_net_set_weights": ([vp, vp, ctypes.c_long], ctypes.c_int),
        "eg_net_get_weights": ([vp, vp, ctypes.c_long], ctypes.c_int),
        "eg_attach_learned_pc": ([vp, vp], ctypes.c_int),
        "eg_net_apply": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "eg_net_loss_grad": ([vp, vp, vp, vp, dp, vp], ctypes.c_int),
        "eg_harvest": ([vp, vp, ctypes.c_int, vp, vp], ctypes.c_int),
        "eg_harvest_krylov": ([vp, vp, ctypes.c_int, vp, vp], ctypes.c_int),
        "eg_net_train": ([vp, vp, ctypes.c_int, vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_double, ctypes.c_ulonglong, dp], ctypes.c_int),
        "eg_net_eval": ([vp, vp, ctypes.c_int, vp, vp, vp, ctypes.c_int, dp], ctypes.c_int),
        "eg_net_set_loss": ([vp, ctypes.c_int], ctypes.c_int),
        "eg_train_learned_pc": ([vp, ctypes.c_char_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint], ctypes.c_int),
        "eg_save_learned_pc": ([vp, vp, ctypes.c_long], ctypes.c_int),
        "eg_load_learned_pc": ([vp, vp, ctypes.c_long], ctypes.c_int),
        "eg_get_learned_pc": ([vp, ctypes.POINTER(vp)], ctypes.c_int),
        "eg_dot_noalloc": ([vp, vp, ctypes.c_long, ctypes.c_int, vp, dp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise EndgameError(rc, _lib.eg_last_error().decode())
    return rc


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA/HIP torch.Tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _args(*specs):
    """Device pointers of tensor arguments after checking what the C ABI assumes of each: a
    contiguous tensor of ``numel`` elements of ``dtype`` on ``device``.  ``specs`` are tuples
    (tensor, name, dtype, numel, device); None tensors pass through as None.  The shapes and
    types of all arguments are checked before their placement.  Raises before any library call."""
    import torch
    for t, name, dtype, numel, _ in specs:
        if t is None:
            continue
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name}: expected a torch.Tensor")
        if t.dtype != dtype:
            raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
        if t.numel() != numel:
            raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: tensor must be contiguous")
    out = []
    for t, name, _, _, device in specs:
        if t is None:
            out.append(None)
            continue
        if not t.is_cuda:
            raise TypeError(f"{name}: expected a CUDA/HIP tensor")
        if device is not None and t.device != device:
            raise ValueError(f"{name}: on {t.device}, the operator lives on {device}")
        out.append(t.data_ptr())
    return out


def _arg(t, name: str, dtype, numel: int, device=None) -> int:
    return _args((t, name, dtype, numel, device))[0]


def _vec_dtype(prec: int):
    import torch
    return torch.float64 if prec == PREC_FP64 else torch.float32


def dot_noalloc(a, b) -> float:
    """<a, b> with FP64 products and sums, allocating nothing (eg_dot_noalloc): a and b are
    float64 or float32 device tensors of equal length and dtype; ordered on torch's current
    stream of their device."""
    import torch
    lib = load_library()
    if not isinstance(a, torch.Tensor) or a.dtype not in (torch.float64, torch.float32):
        raise ValueError("a: expected a float64 or float32 tensor")
    pa, pb = _args((a, "a", a.dtype, a.numel(), None), (b, "b", a.dtype, a.numel(), a.device))
    prec = PREC_FP64 if a.dtype == torch.float64 else PREC_FP32
    s = torch.cuda.current_stream(a.device).cuda_stream
    out = ctypes.c_double()
    with torch.cuda.device(a.device):
        _check(lib.eg_dot_noalloc(pa, pb, a.numel(), prec, ctypes.c_void_p(s), ctypes.byref(out)))
    return out.value


class Operator:
    """A 7-point Helmholtz operator resident on the GPU.

    ``coeffs``: CUDA float64 tensor of shape (7, nlev, nlat, nlon), planes W, E, S, N, D, U, C
    (couplings as magnitudes; the matrix entries are their negatives; C is the diagonal).
    """

    def __init__(self, coeffs):
        import torch
        lib = load_library()
        if coeffs.dtype != torch.float64 or coeffs.dim() != 4 or coeffs.shape[0] != 7:
            raise ValueError("coeffs must be float64 of shape (7, nlev, nlat, nlon)")
        _, nlev, nlat, nlon = (int(s) for s in coeffs.shape)
        self.nlon, self.nlat, self.nlev = nlon, nlat, nlev
        self.n = nlon * nlat * nlev
        self.device = coeffs.device
        h = ctypes.c_void_p()
        self._sync_stream_ptr = None
        _check(lib.eg_create_operator(_ptr(coeffs), nlon, nlat, nlev, ctypes.byref(h)))
        self._h = h
        self._bind_stream()

    def _bind_stream(self):
        import torch
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._sync_stream_ptr:
            _check(_lib.eg_set_stream(self._h, ctypes.c_void_p(s)))
            self._sync_stream_ptr = s

    def close(self):
        if getattr(self, "_h", None):
            _lib.eg_destroy_operator(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_option(self, key: str, value: float):
        _check(_lib.eg_set_option(self._h, key.encode(), float(value)))

    def solve(self, b, x, tol: float = 1e-8, maxit: int = 20000, mode: int = FP64) -> SolveInfo:
        """Solve in place: ``x`` holds the initial guess and receives the solution."""
        import torch
        pb, px = _args((b, "b", torch.float64, self.n, self.device), (x, "x", torch.float64, self.n, self.device))
        self._bind_stream()
        status = _check(_lib.eg_solve(self._h, pb, px, float(tol), int(maxit), int(mode)))
        info = _Info()
        _check(_lib.eg_get_info(self._h, ctypes.byref(info)))
        return SolveInfo(status, info.iterations, info.outer_steps, info.restarts, info.fallbacks,
                         info.true_rel_residual, info.seconds)

    def history(self):
        import numpy as np
        cnt = _check(_lib.eg_residual_history(self._h, None, 0))
        buf = np.zeros(max(cnt, 1))
        _lib.eg_residual_history(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cnt)
        return buf[:cnt]

    def _prec_arg(self, prec: int):
        if prec not in (PREC_FP64, PREC_FP32, PREC_BF16, PREC_FP16):
            raise ValueError(f"unknown precision {prec}")
        return _vec_dtype(prec)

    def apply(self, x, y=None, prec: int = PREC_FP64):
        import torch
        dt = self._prec_arg(prec)
        _args((x, "x", dt, self.n, None), (y, "y", dt, self.n, None))
        px = _arg(x, "x", dt, self.n, self.device)
        if y is None:
            y = torch.empty_like(x)
        py = _arg(y, "y", dt, self.n, self.device)
        if py == px:
            raise ValueError("x and y must not overlap")
        self._bind_stream()
        _check(_lib.eg_apply(self._h, px, py, int(prec)))
        return y

    def precond(self, q, z=None, prec: int = PREC_FP64):
        import torch
        dt = self._prec_arg(prec)
        _args((q, "q", dt, self.n, None), (z, "z", dt, self.n, None))
        pq = _arg(q, "q", dt, self.n, self.device)
        if z is None:
            z = torch.empty_like(q)
        pz = _arg(z, "z", dt, self.n, self.device)
        if pz == pq:
            raise ValueError("q and z must not overlap")
        self._bind_stream()
        _check(_lib.eg_apply_precond(self._h, pq, pz, int(prec)))
        return z

    def residual(self, b, x, r=None) -> float:
        import torch
        pb, px, pr = _args((b, "b", torch.float64, self.n, self.device), (x, "x", torch.float64, self.n, self.device),
                           (r, "r", torch.float64, self.n, self.device))
        self._bind_stream()
        rel = ctypes.c_double()
        _check(_lib.eg_residual(self._h, pb, px, pr, ctypes.byref(rel)))
        return rel.value

    def kernel_stats(self, kernel: int, prec: int) -> tuple[int, float]:
        """(timed launches, total device ms) of one kernel class; needs set_option("profile", 1)."""
        cnt = ctypes.c_long()
        ms = ctypes.c_double()
        _check(_lib.eg_kernel_stats(self._h, int(kernel), int(prec), ctypes.byref(cnt), ctypes.byref(ms)))
        return cnt.value, ms.value

    def reset_kernel_stats(self):
        _check(_lib.eg_reset_kernel_stats(self._h))

    def attach(self, net: "Net | None"):
        """Use ``net`` in the LEARNED modes (None detaches)."""
        _check(_lib.eg_attach_learned_pc(self._h, None if net is None else net._h))
        self._net = net

    def train_learned_pc(self, harvest_cfg: str = "", epochs: int = 20, lr: float = 1e-3, seed: int = 0):
        """Harvest (residual, error) pairs from this operator's own solves and train its own
        network on them; it becomes the learned preconditioner (see eg_train_learned_pc)."""
        if epochs < 0 or not lr > 0:
            raise ValueError("need epochs >= 0 and lr > 0")
        self._bind_stream()
        _check(_lib.eg_train_learned_pc(self._h, harvest_cfg.encode(), int(epochs), float(lr), int(seed) & 0xFFFFFFFF))

    def save_learned_pc(self) -> bytes:
        """The learned preconditioner's weights as a byte image (header + FP32 weights)."""
        size = _check(_lib.eg_save_learned_pc(self._h, None, 0))
        buf = ctypes.create_string_buffer(size)
        _check(_lib.eg_save_learned_pc(self._h, ctypes.cast(buf, ctypes.c_void_p), size))
        return buf.raw

    def load_learned_pc(self, image: bytes):
        """Load an image from save_learned_pc into this operator's own network."""
        if not isinstance(image, (bytes, bytearray)):
            raise TypeError("image must be bytes")
        buf = ctypes.create_string_buffer(bytes(image), len(image))
        _check(_lib.eg_load_learned_pc(self._h, ctypes.cast(buf, ctypes.c_void_p), len(image)))

    def learned_pc(self) -> "Net":
        """The network the learned modes use (borrowed from the operator: do not close it)."""
        h = ctypes.c_void_p()
        _check(_lib.eg_get_learned_pc(self._h, ctypes.byref(h)))
        return Net._borrowed(h, self)

    def harvest(self, b, nsnap: int):
        """(r, e) float tensors of shape (count, n) from the solver's own FP64 iterates."""
        import torch
        if nsnap < 1:
            raise ValueError("nsnap must be >= 1")
        pb = _arg(b, "b", torch.float64, self.n, self.device)
        self._bind_stream()
        r = torch.empty((nsnap, self.n), dtype=torch.float32, device=b.device)
        e = torch.empty_like(r)
        cnt = _check(_lib.eg_harvest(self._h, pb, int(nsnap), _ptr(r), _ptr(e)))
        return r[:cnt].contiguous(), e[:cnt].contiguous()

    def harvest_krylov(self, b, nvec: int, errors: bool = True):
        """(r, e) float tensors of shape (count, n): the FGMRES basis vectors of b and A^{-1} of
        each (e is None when ``errors`` is False)."""
        import torch
        if not 1 <= nvec <= 64:
            raise ValueError("nvec must be in 1..64")
        pb = _arg(b, "b", torch.float64, self.n, self.device)
        self._bind_stream()
        r = torch.empty((nvec, self.n), dtype=torch.float32, device=b.device)
        e = torch.empty_like(r) if errors else None
        cnt = _check(_lib.eg_harvest_krylov(self._h, pb, int(nvec), _ptr(r), _ptr(e) if errors else None))
        return r[:cnt].contiguous(), (e[:cnt].contiguous() if errors else None)

    def dot(self, a, b) -> float:
        """<a, b> with FP64 products and sums; a and b: float64 or float32 tensors of equal
        length and dtype (any length) on the operator's device."""
        import torch
        if not isinstance(a, torch.Tensor) or a.dtype not in (torch.float64, torch.float32):
            raise ValueError("a: expected a float64 or float32 tensor")
        pa, pb = _args((a, "a", a.dtype, a.numel(), self.device), (b, "b", a.dtype, a.numel(), self.device))
        prec = PREC_FP64 if a.dtype == torch.float64 else PREC_FP32
        self._bind_stream()
        out = ctypes.c_double()
        _check(_lib.eg_dot(self._h, pa, pb, a.numel(), prec, ctypes.byref(out)))
        return out.value


class Net:
    """The learned preconditioner's network (weights on the GPU)."""

    def __init__(self, seed: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.eg_net_create(int(seed), ctypes.byref(h)))
        self._h = h

    @classmethod
    def _borrowed(cls, handle, owner):
        """A view of a network the library owns (an operator's own network): never destroyed
        from Python; keeps its operator alive."""
        net = cls.__new__(cls)
        net._h = handle
        net._owner = owner
        return net

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self._h = None
            return
        if getattr(self, "_h", None):
            _lib.eg_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    LOSS_ERROR, LOSS_RESIDUAL = 0, 1

    def set_loss(self, kind: int):
        _check(_lib.eg_net_set_loss(self._h, int(kind)))

    def get_weights(self):
        import numpy as np
        w = np.zeros(N_NET_PARAMS, dtype=np.float32)
        _check(_lib.eg_net_get_weights(self._h, w.ctypes.data_as(ctypes.c_void_p), w.size))
        return w

    def set_weights(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(_lib.eg_net_set_weights(self._h, w.ctypes.data_as(ctypes.c_void_p), w.size))

    def apply(self, op: Operator, q, delta=None):
        """M(q) in FP32 (q: float tensor of n); returns z (and fills ``delta`` if given)."""
        import torch
        pq, pd = _args((q, "q", torch.float32, op.n, op.device), (delta, "delta", torch.float32, op.n, op.device))
        op._bind_stream()
        z = torch.empty_like(q)
        _check(_lib.eg_net_apply(op._h, self._h, pq, _ptr(z), pd))
        return z

    def loss_grad(self, op: Operator, r, e):
        import numpy as np
        import torch
        pr, pe = _args((r, "r", torch.float32, op.n, op.device), (e, "e", torch.float32, op.n, op.device))
        op._bind_stream()
        loss = ctypes.c_double()
        g = np.zeros(N_NET_PARAMS, dtype=np.float32)
        _check(_lib.eg_net_loss_grad(op._h, self._h, pr, pe, ctypes.byref(loss), g.ctypes.data_as(ctypes.c_void_p)))
        return loss.value, g

    @staticmethod
    def _pairs(ops, r, e, pair_op):
        """Checked marshalling of a training set: r and e float32 of shape (len(pair_op), n) on
        the operators' device, every operator of the same grid, every pair_op index valid."""
        import numpy as np
        import torch
        if not ops:
            raise ValueError("need at least one operator")
        n, device = ops[0].n, ops[0].device
        for o in ops:
            if (o.nlon, o.nlat, o.nlev) != (ops[0].nlon, ops[0].nlat, ops[0].nlev) or o.device != device:
                raise ValueError("all training operators must have the same grid and device")
        po = np.ascontiguousarray(pair_op, dtype=np.int32).ravel()
        if po.size < 1 or po.min() < 0 or po.max() >= len(ops):
            raise ValueError("pair_op must hold operator indices in [0, len(ops))")
        for name, t in (("r", r), ("e", e)):
            if not isinstance(t, torch.Tensor) or tuple(t.shape) != (po.size, n):
                raise ValueError(f"{name}: expected shape ({po.size}, {n}), got "
                                 f"{tuple(t.shape) if isinstance(t, torch.Tensor) else type(t)}")
        pr, pe = _args((r, "r", torch.float32, po.size * n, device), (e, "e", torch.float32, po.size * n, device))
        arr = (ctypes.c_void_p * len(ops))(*[o._h.value for o in ops])
        return arr, po, pr, pe

    def train(self, ops, r, e, pair_op, epochs: int, batch: int = 16, lr: float = 1e-3, seed: int = 0):
        """Adam training; returns the per-epoch mean training loss (numpy array)."""
        import numpy as np
        arr, po, pr, pe = self._pairs(ops, r, e, pair_op)
        if epochs < 0 or batch < 1 or not lr > 0:
            raise ValueError("need epochs >= 0, batch >= 1, lr > 0")
        ops[0]._bind_stream()
        hist = np.zeros(max(epochs, 1))
        _check(_lib.eg_net_train(self._h, arr, len(ops), pr, pe, po.ctypes.data_as(ctypes.c_void_p),
                                 po.size, int(epochs), int(batch), float(lr), int(seed),
                                 hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return hist[:epochs]

    def eval(self, ops, r, e, pair_op) -> float:
        arr, po, pr, pe = self._pairs(ops, r, e, pair_op)
        ops[0]._bind_stream()
        out = ctypes.c_double()
        _check(_lib.eg_net_eval(self._h, arr, len(ops), pr, pe, po.ctypes.data_as(ctypes.c_void_p),
                                po.size, ctypes.byref(out)))
        return out.value
