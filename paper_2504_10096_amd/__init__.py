"""Python binding of the MI355X structured BSE eigensolver (``include/bse.h``).

Argument marshalling only: every step of the solve runs in the HIP library
``libbse.so`` built in-tree for gfx950.  PyTorch provides device memory and
the stream.  There is no CPU fallback: without the built library, or without
a GPU, the calls raise.

    s = Solver("ph", n, storage="c128")      # or "hilo" for the mixed path
    s.set_packed("A", ap)                   # LAPACK-'U' packed, device complex
    s.set_packed("B", bp)
    omega, X, Y, stats = s.solve(k=32, tol=1e-10)
    dA, dB = s.backward(g)                  # gradient of sum g_c omega_c

``BSEEigs`` wraps solve/backward as a ``torch.autograd.Function`` over the
packed triangles.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbse.so")

OK, ERR_INVALID_ARG, ERR_OOM, ERR_DEVICE, ERR_NOT_PD, ERR_NOT_CONVERGED, ERR_NONFINITE, ERR_BAD_STATE = range(8)
TDA, PSEUDO_HERMITIAN = 0, 1
STORE_C128, STORE_HILO = 0, 1
C64, C128 = 0, 1
PREC_FP64, PREC_MIXED, PREC_HI_FP64 = 0, 1, 2
BLOCK_A, BLOCK_B = 0, 1
OP_A, OP_K1, OP_K2, OP_H = 0, 1, 2, 3
COMP_PACKED, COMP_LOWRANK, COMP_DIAG, COMP_STORED = 0, 1, 2, 3

EXPORTS = ["bse_create", "bse_create_ex", "bse_set_packed", "bse_apply", "bse_apply_noalloc", "bse_solve", "bse_backward", "bse_strength",
           "bse_direct", "bse_haydock", "bse_haydock_spectrum", "bse_destroy", "bse_status_string",
           "bse_last_error"]


class SolveOpts(ctypes.Structure):
    _fields_ = [("ncv", ctypes.c_int32), ("keep", ctypes.c_int32), ("max_restarts", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("switch_tol", ctypes.c_double), ("start_seed", ctypes.c_uint64),
                ("fp32_arith", ctypes.c_int32), ("block", ctypes.c_int32),
                ("refine_start", ctypes.c_int32), ("variant", ctypes.c_int32), ("warm_k", ctypes.c_int32),
                ("reserved_", ctypes.c_int32), ("warm_x", ctypes.c_void_p), ("warm_y", ctypes.c_void_p)]


VARIANT_FOLDED, VARIANT_COUPLED, VARIANT_DUAL, VARIANT_H_BLOCK = 0, 1, 2, 3


class Stats(ctypes.Structure):
    _fields_ = [("n_converged", ctypes.c_int32), ("restarts", ctypes.c_int32), ("steps_fp32", ctypes.c_int64),
                ("steps_fp64", ctypes.c_int64), ("passes", ctypes.c_int64), ("ms_total", ctypes.c_double),
                ("ms_fp32_phase", ctypes.c_double), ("ms_fp64_phase", ctypes.c_double),
                ("ms_final", ctypes.c_double), ("max_rel_residual", ctypes.c_double),
                ("bytes_per_pass_fp32", ctypes.c_double), ("bytes_per_pass_fp64", ctypes.c_double),
                ("samples_fp32", ctypes.c_int64), ("samples_fp64", ctypes.c_int64),
                ("ms_block_fp32", ctypes.c_double), ("ms_block_fp64", ctypes.c_double),
                ("samples_fused", ctypes.c_int64), ("ms_block_fused", ctypes.c_double),
                ("fused_vectors", ctypes.c_int64), ("block", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("ms_gemm", ctypes.c_double), ("gemm_flops", ctypes.c_double),
                ("ms_dense_form", ctypes.c_double), ("ms_dense_factor", ctypes.c_double),
                ("ms_dense_eig", ctypes.c_double), ("ms_matvec", ctypes.c_double), ("ms_orth", ctypes.c_double),
                ("ms_small", ctypes.c_double), ("ms_restart", ctypes.c_double), ("ms_residual", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


def torch_allocator(device):
    """bse_allocator backed by PyTorch's caching allocator on `device` (the library's device
    memory then shows in torch.cuda.memory_allocated and is reused by torch after close)."""
    dev = torch.device(device).index if not isinstance(device, int) else device

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev, stream=int(stream or 0))
        except Exception:  # out of memory: the library reports BSE_ERR_OUT_OF_MEMORY
            return None

    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    return Allocator(_ALLOC_FN(_alloc), _FREE_FN(_free), None)


class Component(ctypes.Structure):
    _fields_ = [("target", ctypes.c_int32), ("form", ctypes.c_int32), ("data", ctypes.c_void_p),
                ("rank", ctypes.c_int64), ("scale", ctypes.c_double)]


class BSEError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class NotPositiveDefinite(BSEError):
    pass


class NotConverged(BSEError):
    pass


_lib = None


def load_library():
    """Load libbse.so; raises if it was not built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "bse_create": ([ctypes.POINTER(vp), i32, i64, i32, vp], i32),
        "bse_create_ex": ([ctypes.POINTER(vp), i32, i64, i32, vp, ctypes.POINTER(Allocator)], i32),
        "bse_set_packed": ([vp, i32, i64, i64, vp, i32], i32),
        "bse_apply": ([vp, i32, i32, i64, vp, vp], i32),
        "bse_apply_noalloc": ([vp, i32, i32, i64, vp, vp], i32),
        "bse_solve": ([vp, i32, dbl, ctypes.POINTER(SolveOpts), vp, vp, vp, ctypes.POINTER(Stats)], i32),
        "bse_backward": ([vp, vp, vp, vp], i32),
        "bse_strength": ([vp, vp, i32, ctypes.POINTER(Component), ctypes.POINTER(dbl)], i32),
        "bse_direct": ([vp, i32, vp, vp, vp, ctypes.POINTER(Stats)], i32),
        "bse_haydock": ([vp, i32, vp, i32, dbl, i32, vp, i32, dbl, vp, vp, ctypes.POINTER(dbl), vp,
                         ctypes.POINTER(i32), ctypes.POINTER(Stats)], i32),
        "bse_haydock_spectrum": ([i32, i32, vp, vp, dbl, vp, i32, dbl, vp, vp], i32),
        "bse_destroy": ([vp], i32),
        "bse_status_string": ([i32], ctypes.c_char_p),
        "bse_last_error": ([vp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _stream_ptr(device):
    return torch.cuda.current_stream(device).cuda_stream


def _dev_ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One handle of the C ABI: a resonant block (and a coupling block for 'ph')."""

    def __init__(self, kind, n, storage="c128", device=None, allocator=None):
        """allocator: None (the library's hipMalloc) or "torch" (PyTorch's caching allocator,
        through bse_create_ex)."""
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the BSE solver needs a HIP device")
        self.kind = {"tda": TDA, "ph": PSEUDO_HERMITIAN}[kind]
        self.n = int(n)
        self.storage = {"c128": STORE_C128, "hilo": STORE_HILO}[storage]
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._h = ctypes.c_void_p()
        self._alloc = None
        if allocator not in (None, "torch"):
            raise ValueError("allocator must be None or 'torch'")
        with torch.cuda.device(self.device):
            stream = ctypes.c_void_p(_stream_ptr(self.device))
            if allocator == "torch":
                self._alloc = torch_allocator(self.device.index)  # kept alive until close
                self._check(lib.bse_create_ex(ctypes.byref(self._h), self.kind, self.n, self.storage, stream,
                                              ctypes.byref(self._alloc)), "bse_create_ex", created=False)
            else:
                self._check(lib.bse_create(ctypes.byref(self._h), self.kind, self.n, self.storage, stream),
                            "bse_create", created=False)
        self.last_stats = None

    # -- helpers ---------------------------------------------------------------
    def _check(self, st, what, created=True):
        if st == OK:
            return
        lib = load_library()
        detail = lib.bse_last_error(self._h).decode() if created and self._h else ""
        msg = f"{what}: {lib.bse_status_string(st).decode()}" + (f" ({detail})" if detail else "")
        cls = {ERR_NOT_PD: NotPositiveDefinite, ERR_NOT_CONVERGED: NotConverged}.get(st, BSEError)
        raise cls(st, msg)

    def close(self):
        if self._h:
            load_library().bse_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- C ABI calls -----------------------------------------------------------
    def set_packed(self, which, packed, j0=0, j1=None):
        """Columns j0..j1-1 of the upper triangle in LAPACK-'U' packed order (device c128 or c64)."""
        j1 = self.n if j1 is None else int(j1)
        if packed.dtype not in (torch.complex128, torch.complex64):
            raise ValueError("packed data must be complex128 or complex64")
        expect = j1 * (j1 + 1) // 2 - j0 * (j0 + 1) // 2
        if packed.numel() < expect:
            raise ValueError(f"packed chunk has {packed.numel()} entries, needs {expect}")
        dt = C128 if packed.dtype == torch.complex128 else C64
        blk = {"A": BLOCK_A, "B": BLOCK_B}[which]
        with torch.cuda.device(self.device):
            self._check(load_library().bse_set_packed(self._h, blk, int(j0), j1, _dev_ptr(packed), dt),
                        "bse_set_packed")

    def set_packed_raw(self, which, ptr, j0, j1, c64=False):
        blk = {"A": BLOCK_A, "B": BLOCK_B}[which]
        self._check(load_library().bse_set_packed(self._h, blk, int(j0), int(j1), ctypes.c_void_p(ptr),
                                                  C64 if c64 else C128), "bse_set_packed")

    def apply(self, op, x, precision="fp64", out=None, noalloc=False):
        """y = op(x); x: (nvec, N) complex128 (nvec, 2N for 'H'), rows are vectors.  precision:
        "fp64" (FP64 operator), "fp32" (complex FP32 on hi), "hi64" (FP64 arithmetic on hi).
        out: optional preallocated result (same shape as x).  noalloc: call bse_apply_noalloc
        (the library allocates nothing; partial sums in its fixed per-device array)."""
        opc = {"A": OP_A, "K1": OP_K1, "K2": OP_K2, "H": OP_H}[op]
        length = 2 * self.n if opc == OP_H else self.n
        x = x.reshape(-1, length)
        _dev_ptr(x, torch.complex128, "x")
        if out is None:
            y = torch.empty_like(x)
        else:
            y = out.reshape(-1, length)
            if y.shape != x.shape or y.data_ptr() != out.data_ptr():
                raise ValueError("out must be a contiguous tensor shaped like x")
            _dev_ptr(y, torch.complex128, "out")
        prec = {"fp64": PREC_FP64, "fp32": PREC_MIXED, "hi64": PREC_HI_FP64}[precision]
        fn = load_library().bse_apply_noalloc if noalloc else load_library().bse_apply
        with torch.cuda.device(self.device):
            self._check(fn(self._h, opc, prec, x.shape[0], _dev_ptr(x), _dev_ptr(y)),
                        "bse_apply_noalloc" if noalloc else "bse_apply")
        return y

    def solve(self, k, tol, precision="fp64", ncv=0, keep=0, max_restarts=0, switch_tol=0.0, seed=1,
              raise_not_converged=True, fp32_arith=False, block=0, refine_start=0, variant=0, warm=None):
        """Lowest k pairs.  Returns (omega[k] f64, X[k, N] c128, Y[k, N] c128 or None, stats dict);
        row c of X/Y is pair c (column c of the column-major N x k ABI layout).  With
        precision="mixed", fp32_arith selects complex FP32 arithmetic for the bulk passes
        (default: FP64 arithmetic on the FP32-stored triangles).  block: vectors per read of the
        triangles in the Lanczos iteration (0: automatic).  variant (PH): 0 the K1-metric
        iteration on K2 K1, 1 the Lanczos process on H in the M inner product, 2 the dual
        K2-metric iteration on K1 K2, 3 block Lanczos on H in the M inner product over C^2N
        (`block` full-H vectors per read; default 4 from N = 16384 on, else 2).  warm: (X, Y) of a
        previous solve of a nearby matrix (rows = pairs, Y None for TDA) to start from."""
        k = int(k)
        dev = self.device
        omega = torch.empty(k, dtype=torch.float64, device=dev)
        X = torch.empty((k, self.n), dtype=torch.complex128, device=dev)
        Y = torch.empty((k, self.n), dtype=torch.complex128, device=dev) if self.kind == PSEUDO_HERMITIAN else None
        opts = SolveOpts(int(ncv), int(keep), int(max_restarts), PREC_MIXED if precision == "mixed" else PREC_FP64,
                         float(switch_tol), int(seed), 1 if fp32_arith else 0, int(block), int(refine_start),
                         int(variant))
        if warm is not None:
            wx, wy = warm
            wx = wx.to(device=dev, dtype=torch.complex128).reshape(-1, self.n).contiguous()
            opts.warm_k = wx.shape[0]
            opts.warm_x = wx.data_ptr()
            if wy is not None:
                wy = wy.to(device=dev, dtype=torch.complex128).reshape(-1, self.n).contiguous()
                if wy.shape != wx.shape:
                    raise ValueError("warm X and Y must have the same shape")
                opts.warm_y = wy.data_ptr()
        stats = Stats()
        with torch.cuda.device(dev):
            st = load_library().bse_solve(self._h, k, float(tol), ctypes.byref(opts), _dev_ptr(omega),
                                          _dev_ptr(X), _dev_ptr(Y), ctypes.byref(stats))
        self.last_stats = stats.as_dict()
        self.solved_k = None
        if st == ERR_NOT_CONVERGED and not raise_not_converged:
            return omega, X, Y, self.last_stats
        self._check(st, "bse_solve")
        self.solved_k = k
        return omega, X, Y, self.last_stats

    def _weights(self, g):
        """Eigenvalue weights on the device, one per pair of the last successful solve."""
        g = g.to(device=self.device, dtype=torch.float64).contiguous()
        if getattr(self, "solved_k", None) is not None and g.numel() != self.solved_k:
            raise ValueError(f"g has {g.numel()} weights; the last solve returned {self.solved_k} pairs")
        return g

    def backward(self, g, want_a=True, want_b=True):
        """Packed gradients (dL/dA, dL/dB) of L = sum_c g_c omega_c (LAPACK-'U', off-diagonal x2)."""
        g = self._weights(g)
        m = self.n * (self.n + 1) // 2
        da = torch.empty(m, dtype=torch.complex128, device=self.device) if want_a else None
        db = (torch.empty(m, dtype=torch.complex128, device=self.device)
              if (want_b and self.kind == PSEUDO_HERMITIAN) else None)
        with torch.cuda.device(self.device):
            self._check(load_library().bse_backward(self._h, _dev_ptr(g), _dev_ptr(da), _dev_ptr(db)),
                        "bse_backward")
        return da, db


    def direct(self, k):
        """Lowest k pairs by the dense direct solve (PH: the structure-preserving Cholesky /
        skew-symmetric route).  Returns (omega[k], X[k, N], Y[k, N] or None, stats dict)."""
        k = int(k)
        dev = self.device
        omega = torch.empty(k, dtype=torch.float64, device=dev)
        X = torch.empty((k, self.n), dtype=torch.complex128, device=dev)
        Y = torch.empty((k, self.n), dtype=torch.complex128, device=dev) if self.kind == PSEUDO_HERMITIAN else None
        stats = Stats()
        with torch.cuda.device(dev):
            st = load_library().bse_direct(self._h, k, _dev_ptr(omega), _dev_ptr(X), _dev_ptr(Y),
                                           ctypes.byref(stats))
        self._check(st, "bse_direct")
        self.last_stats = stats.as_dict()
        return omega, X, Y, self.last_stats

    def haydock(self, d, n_iter, tol=0.0, freq=None, eta=0.1, precision="fp64"):
        """Lanczos-Haydock recursion from dipole vectors d: (N,) or (nd, N) complex, nd >= 1
        advancing together (up to four per read of the triangles).  Returns (alpha, beta f64
        device tensors, norm2, chi c128 device tensor or None, stats dict) with shapes
        (nd, n), (nd, n), (nd,), (nd, nw) -- or (n,), (n,), float, (nw,) for a 1-D d -- where n
        is the number of steps done.  chi(z) at z = freq + i eta is the response
        d^H (z - A)^{-1} d (TDA) or q^H Omega (z - H)^{-1} q, q = [d; conj(d)] (PH).
        precision: "fp64", "hi64" (FP64 arithmetic on the complex64 hi triangles) or "fp32"."""
        dev = self.device
        single = d.dim() == 1
        d = d.to(device=dev, dtype=torch.complex128).reshape(-1, self.n).contiguous()  # row q = dipole q
        nd = d.shape[0]
        alpha = torch.zeros((nd, int(n_iter)), dtype=torch.float64, device=dev)
        beta = torch.zeros((nd, int(n_iter)), dtype=torch.float64, device=dev)
        chi = None
        nw = 0
        if freq is not None:
            freq = freq.to(device=dev, dtype=torch.float64).contiguous()
            nw = freq.numel()
            chi = torch.empty((nd, nw), dtype=torch.complex128, device=dev)
        prec = {"fp64": PREC_FP64, "hi64": PREC_HI_FP64, "fp32": PREC_MIXED}[precision]
        norm2 = (ctypes.c_double * nd)()
        done = ctypes.c_int32(0)
        stats = Stats()
        with torch.cuda.device(dev):
            st = load_library().bse_haydock(self._h, nd, _dev_ptr(d), int(n_iter), float(tol), prec,
                                            _dev_ptr(freq), nw, float(eta), _dev_ptr(alpha), _dev_ptr(beta),
                                            norm2, _dev_ptr(chi), ctypes.byref(done), ctypes.byref(stats))
        self._check(st, "bse_haydock")
        n = done.value
        alpha, beta = alpha[:, :n], beta[:, :n]
        nn = [norm2[q] for q in range(nd)]
        if single:
            return alpha[0], beta[0], nn[0], None if chi is None else chi[0], stats.as_dict()
        return alpha, beta, nn, chi, stats.as_dict()

    def strength(self, g, comps):
        """Scalars Re<G, C_q> of L = sum_c g_c omega_c for components given as
        (target 'A'|'B', form 'packed'|'lowrank'|'diag'|'stored', data tensor or None, scale).
        packed: LAPACK-'U' complex128; lowrank: N x r complex128 factor F (C = s F F^H for A,
        s F F^T for B); diag: N float64 (A only); stored: the stored block itself."""
        g = self._weights(g)
        forms = {"packed": COMP_PACKED, "lowrank": COMP_LOWRANK, "diag": COMP_DIAG, "stored": COMP_STORED}
        arr = (Component * len(comps))()
        keep = []
        for q, (target, form, data, scale) in enumerate(comps):
            rank = 0
            ptr = None
            if data is not None:
                if form == "lowrank":
                    data = data.to(self.device, torch.complex128).t().contiguous()  # column-major N x r
                    rank = data.shape[0]
                elif form == "diag":
                    data = data.to(self.device, torch.float64).contiguous()
                else:
                    data = data.to(self.device, torch.complex128).contiguous()
                keep.append(data)
                ptr = data.data_ptr()
            arr[q] = Component({"A": BLOCK_A, "B": BLOCK_B}[target], forms[form], ptr, rank, float(scale))
        out = (ctypes.c_double * len(comps))()
        with torch.cuda.device(self.device):
            self._check(load_library().bse_strength(self._h, _dev_ptr(g), len(comps), arr, out), "bse_strength")
        return [float(v) for v in out]


def from_packed(ap, bp=None, storage="c128"):
    """A Solver filled from device packed triangles (B given => pseudo-Hermitian)."""
    n = int(round(((8 * ap.numel() + 1) ** 0.5 - 1) / 2))
    s = Solver("ph" if bp is not None else "tda", n, storage=storage, device=ap.device.index)
    s.set_packed("A", ap.contiguous())
    if bp is not None:
        s.set_packed("B", bp.contiguous())
    return s


class BSEEigs(torch.autograd.Function):
    """omega = lowest-k eigenvalues (TDA) or positive pairs (PH) of the packed blocks.

    forward(ap, bp, k, tol, storage, precision) -> (omega, X, Y);  bp may be None (TDA).
    backward returns packed gradients for ap and bp from the eigenvalue
    gradient; gradients with respect to X and Y are not supported.
    """

    @staticmethod
    def forward(ctx, ap, bp, k, tol, storage="c128", precision="fp64"):
        s = from_packed(ap.detach(), None if bp is None else bp.detach(), storage=storage)
        omega, X, Y, _ = s.solve(k, tol, precision=precision)
        ctx.solver = s
        ctx.has_b = bp is not None
        if Y is None:
            Y = torch.zeros(0, dtype=torch.complex128, device=ap.device)
        ctx.mark_non_differentiable(X, Y)
        return omega, X, Y

    @staticmethod
    def backward(ctx, g_omega, g_x, g_y):
        if g_x is not None and torch.count_nonzero(g_x) > 0:
            raise NotImplementedError("gradients with respect to the eigenvectors are not supported")
        if g_y is not None and g_y.numel() and torch.count_nonzero(g_y) > 0:
            raise NotImplementedError("gradients with respect to the eigenvectors are not supported")
        da, db = ctx.solver.backward(g_omega)
        return da, (db if ctx.has_b else None), None, None, None, None


def haydock_spectrum(kind, alpha, beta, norm2, freq, eta):
    """chi(freq + i eta) from Haydock coefficients (device tensors) on their device."""
    kind_i = PSEUDO_HERMITIAN if kind == "ph" else TDA
    alpha = alpha.to(torch.float64).contiguous()
    beta = beta.to(device=alpha.device, dtype=torch.float64).contiguous()
    freq = freq.to(device=alpha.device, dtype=torch.float64).contiguous()
    chi = torch.empty(freq.numel(), dtype=torch.complex128, device=alpha.device)
    with torch.cuda.device(alpha.device):
        st = load_library().bse_haydock_spectrum(kind_i, alpha.numel(), _dev_ptr(alpha), _dev_ptr(beta),
                                                 float(norm2), _dev_ptr(freq), freq.numel(), float(eta),
                                                 _dev_ptr(chi), ctypes.c_void_p(_stream_ptr(alpha.device)))
    if st != OK:
        raise BSEError(st, "bse_haydock_spectrum failed")
    return chi
