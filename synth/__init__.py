"""Seeded synthetic BSE-shaped inputs shared by the oracle, the tests and the bench.

The module generates inputs only; it holds none of the eigensolver's arithmetic.
Matrices follow ``entry.h``:

    A = diag(eps) + s*I + alpha*Kx - beta*W,   B = alpha*B0

with eps sorted U[1, 8] eV, Kx = X X^H / N (X: N x 32, E|x|^2 = 0.25),
W_ij = 0.3 exp(-|i-j|/64) exp(i phi_ij) (Hermitian random phases) and
B0 = c Y Y^T (Y: N x 32, E|y|^2 = 1) scaled to a prescribed 2-norm.
Host (``pack_host``) and device (``DeviceGen``) produce bit-identical entries.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
RANK = 32
NPHASE = 65536

# Workload constants of the synthetic matrices.
EPS_LO, EPS_HI = 1.0, 8.0
X_VAR, Y_VAR = 0.25, 1.0
W_AMP, W_DECAY = 0.3, 64.0
LAMBDA_MIN_TARGET = 1.0  # lambda_min(A) of the pseudo-Hermitian workloads after the shift (eV)
B_NORM_FRAC = 0.25       # ||B||_2 = 0.25 * lambda_min(A)

STREAM_EPS, STREAM_X, STREAM_Y, STREAM_W, STREAM_LOSS, STREAM_VEC = 1, 2, 3, 4, 5, 6


class SynParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("seed", ctypes.c_uint64), ("with_b", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("shift", ctypes.c_double), ("kx_scale", ctypes.c_double),
                ("b0_scale", ctypes.c_double)]


_host = None
_dev = None
_dp = ctypes.POINTER(ctypes.c_double)


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _lib_host():
    global _host
    if _host is None:
        path = os.path.join(HERE, "libsynth.so")
        if not os.path.exists(path):
            raise RuntimeError("synth/libsynth.so is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        lib.syn_make_tables.restype = ctypes.c_int
        lib.syn_make_tables.argtypes = [ctypes.c_int64, ctypes.c_uint64] + [ctypes.c_double] * 6 + [_dp] * 7
        lib.syn_pack_host.restype = ctypes.c_int
        lib.syn_pack_host.argtypes = [ctypes.POINTER(SynParams)] + [_dp] * 7 + [ctypes.c_int32, ctypes.c_int64,
                                                                                  ctypes.c_int64, _dp]
        lib.syn_entry_host.restype = None
        lib.syn_entry_host.argtypes = [ctypes.POINTER(SynParams)] + [_dp] * 7 + [ctypes.c_int32, ctypes.c_int64,
                                                                                   ctypes.c_int64, _dp]
        lib.syn_direct_band.restype = ctypes.c_int
        lib.syn_direct_band.argtypes = [ctypes.POINTER(SynParams), _dp, _dp, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, _dp]
        lib.syn_sym_factor_norm.restype = ctypes.c_double
        lib.syn_sym_factor_norm.argtypes = [ctypes.c_int64, _dp, _dp]
        lib.syn_uniform.restype = ctypes.c_int
        lib.syn_uniform.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, _dp]
        lib.syn_philox_block.restype = None
        lib.syn_philox_block.argtypes = [ctypes.c_uint32] * 6 + [ctypes.POINTER(ctypes.c_uint32)]
        _host = lib
    return _host


def philox_block(ctr, key):
    out = (ctypes.c_uint32 * 4)()
    _lib_host().syn_philox_block(*[int(c) for c in ctr], *[int(k) for k in key], out)
    return [int(v) for v in out]


def uniform(seed, stream, count):
    out = np.empty(count, dtype=np.float64)
    _lib_host().syn_uniform(seed, stream, count, _ptr(out))
    return out


class Tables:
    """Small tables from which every matrix entry is evaluated."""

    def __init__(self, n, seed):
        self.n, self.seed = int(n), int(seed)
        f = RANK * self.n
        self.eps = np.empty(self.n)
        self.xr, self.xi, self.yr, self.yi = (np.empty(f) for _ in range(4))
        self.amp = np.empty(self.n)
        self.cs = np.empty(2 * NPHASE)
        rc = _lib_host().syn_make_tables(self.n, self.seed, EPS_LO, EPS_HI, X_VAR, Y_VAR, W_AMP, W_DECAY,
                                         _ptr(self.eps), _ptr(self.xr), _ptr(self.xi), _ptr(self.yr),
                                         _ptr(self.yi), _ptr(self.amp), _ptr(self.cs))
        if rc:
            raise ValueError("syn_make_tables failed")

    def ptrs(self):
        return [_ptr(a) for a in (self.eps, self.xr, self.xi, self.yr, self.yi, self.amp, self.cs)]

    def x_factor(self):
        return (self.xr + 1j * self.xi).reshape(self.n, RANK)

    def y_factor(self):
        return (self.yr + 1j * self.yi).reshape(self.n, RANK)

    def direct_row_radius(self):
        """max_i sum_j |W_ij|: a Gershgorin bound on ||W||_2."""
        n = self.n
        c = np.concatenate([[0.0], np.cumsum(self.amp)])
        i = np.arange(n)
        # row i: sum_{d=0}^{n-1-i} amp[d] + sum_{d=1}^{i} amp[d]
        rows = c[n - i] + (c[i + 1] - c[1])
        return float(rows.max())

    def sym_factor_norm(self):
        return float(_lib_host().syn_sym_factor_norm(self.n, _ptr(self.yr), _ptr(self.yi)))


SHIFTS_FILE = os.path.join(HERE, "shifts.json")
_shifts = None


def recorded_lambda_min_raw(n, seed):
    """lambda_min of the raw block A_raw (no shift, alpha = beta = 1) as recorded in shifts.json
    (computed once by the FP64 oracle, see oracle/make_shifts.py), or None."""
    global _shifts
    if _shifts is None:
        import json
        _shifts = json.load(open(SHIFTS_FILE)) if os.path.exists(SHIFTS_FILE) else {}
    rec = _shifts.get(f"{int(n)}:{int(seed)}")
    return None if rec is None else float(rec["lambda_min_raw"])


def recipe_shift(lambda_min_raw):
    """s = 1 - lambda_min(A_raw), rounded up to 1e-6 eV (0 if A_raw is already above 1 eV)."""
    return max(0.0, math.ceil((LAMBDA_MIN_TARGET - float(lambda_min_raw)) * 1e6) / 1e6)


class Matrix:
    """A seeded synthetic matrix pair: parameters + tables.

    Pseudo-Hermitian recipes (``recipe``):
      "baseline"  s = 1 - lambda_min(A_raw) rounded up to 1e-6 eV, so lambda_min(A) = 1 eV, and
                  ||B||_2 = 0.25 lambda_min(A).  lambda_min(A_raw) is passed in
                  (``lambda_min_raw``) or looked up in shifts.json; this module computes no
                  eigenvalues.
      "certified" s from a Gershgorin bound of the direct term (lambda_min(A) >= 1 eV without an
                  eigen-solve, in practice lambda_min(A) ~ 35 eV and weak coupling,
                  ||B||_2 = 0.25 eV); kept as a named extra workload.
    TDA matrices are literal (no shift, no B).
    """

    def __init__(self, n, seed, ph, alpha=1.0, beta=1.0, shift=None, b_norm=None, tables=None,
                 recipe="baseline", lambda_min_raw=None):
        self.tables = tables if tables is not None else Tables(n, seed)
        self.n, self.seed, self.ph = int(n), int(seed), bool(ph)
        self.alpha, self.beta = float(alpha), float(beta)
        t = self.tables
        self.r_w = t.direct_row_radius()
        self.recipe = recipe if ph else "literal"
        self.lambda_min_raw = None
        if shift is None and ph:
            if recipe == "baseline":
                lm = lambda_min_raw if lambda_min_raw is not None else recorded_lambda_min_raw(n, seed)
                if lm is None:
                    raise ValueError(f"no recorded lambda_min(A_raw) for n={n}, seed={seed}: pass "
                                     "lambda_min_raw= (from the oracle), or run oracle/make_shifts.py "
                                     f"{n}:{seed}, or use recipe='certified'")
                self.lambda_min_raw = float(lm)
                shift = recipe_shift(lm)
            elif recipe == "certified":
                # lambda_min(A) >= eps_min + s - beta*r_W  (Kx is PSD)
                shift = max(0.0, LAMBDA_MIN_TARGET - (float(t.eps[0]) - self.beta * self.r_w))
            else:
                raise ValueError(f"unknown recipe {recipe!r}")
        self.shift = float(shift) if shift is not None else 0.0
        if self.lambda_min_raw is not None:
            # lambda_min(A) at alpha = beta = 1 (the shift is fixed under changes of alpha, beta)
            self.lambda_min_a = self.lambda_min_raw + self.shift
        else:
            self.lambda_min_a = float(t.eps[0]) + self.shift - self.beta * self.r_w
        if b_norm is None:
            b_norm = B_NORM_FRAC * self.lambda_min_a if ph else 0.0
        self.b_norm = float(b_norm)
        sig = t.sym_factor_norm() if ph else 1.0
        self.b0_scale = self.b_norm / sig if ph else 0.0
        self.kx_scale = 1.0 / self.n

    def params(self, alpha=None, beta=None):
        p = SynParams()
        p.n, p.seed, p.with_b = self.n, self.seed, int(self.ph)
        p.alpha = self.alpha if alpha is None else float(alpha)
        p.beta = self.beta if beta is None else float(beta)
        p.shift, p.kx_scale, p.b0_scale = self.shift, self.kx_scale, self.b0_scale
        return p

    def pack_host(self, which, j0=0, j1=None, alpha=None, beta=None):
        """LAPACK-'U' packed columns j0..j1-1 of A (which=0) or B (which=1), complex128."""
        j1 = self.n if j1 is None else int(j1)
        cnt = j1 * (j1 + 1) // 2 - j0 * (j0 + 1) // 2
        out = np.empty(cnt, dtype=np.complex128)
        p = self.params(alpha, beta)
        rc = _lib_host().syn_pack_host(ctypes.byref(p), *self.tables.ptrs(), int(which), int(j0), j1,
                                       out.ctypes.data_as(_dp))
        if rc:
            raise ValueError("syn_pack_host failed")
        return out

    def entry(self, which, i, j):
        out = np.empty(2)
        p = self.params()
        _lib_host().syn_entry_host(ctypes.byref(p), *self.tables.ptrs(), int(which), int(i), int(j), _ptr(out))
        return complex(out[0], out[1])

    def direct_band(self, i0, i1, band):
        """Upper band of W (without beta): rows i0..i1-1, columns i..i+band-1."""
        out = np.empty((i1 - i0) * band, dtype=np.complex128)
        p = self.params()
        _lib_host().syn_direct_band(ctypes.byref(p), _ptr(self.tables.amp), _ptr(self.tables.cs), int(i0),
                                    int(i1), int(band), out.ctypes.data_as(_dp))
        return out.reshape(i1 - i0, band)


class DeviceGen:
    """Device generator: same entries as ``Matrix.pack_host``, written to device memory."""

    def __init__(self, mat, alpha=None, beta=None):
        global _dev
        if _dev is None:
            path = os.path.join(HERE, "libsynth_dev.so")
            if not os.path.exists(path):
                raise RuntimeError("synth/libsynth_dev.so is not built; run __graft_entry__.build()")
            lib = ctypes.CDLL(path)
            lib.synd_create.restype = ctypes.c_int
            lib.synd_create.argtypes = [ctypes.POINTER(SynParams)] + [_dp] * 7 + [ctypes.POINTER(ctypes.c_void_p)]
            lib.synd_pack.restype = ctypes.c_int
            lib.synd_pack.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p]
            lib.synd_destroy.restype = ctypes.c_int
            lib.synd_destroy.argtypes = [ctypes.c_void_p]
            _dev = lib
        self.mat = mat
        self._p = mat.params(alpha, beta)
        self._h = ctypes.c_void_p()
        rc = _dev.synd_create(ctypes.byref(self._p), *mat.tables.ptrs(), ctypes.byref(self._h))
        if rc:
            raise RuntimeError(f"synd_create failed ({rc})")

    def pack(self, which, j0, j1, out_ptr, stream_ptr):
        rc = _dev.synd_pack(self._h, int(which), int(j0), int(j1), ctypes.c_void_p(out_ptr),
                            ctypes.c_void_p(stream_ptr))
        if rc:
            raise RuntimeError(f"synd_pack failed ({rc})")

    def close(self):
        if self._h:
            _dev.synd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Workloads: (kind, N, k, tol, seed).  PH workloads use the "baseline" recipe (lambda_min(A) = 1 eV,
# ||B||_2 = 0.25 lambda_min(A)); TDA workloads are literal (no shift, no B).
WORKLOADS = {
    0: dict(name="tda_n1024_k16", ph=False, n=1024, k=16, tol=1e-10, seed=10096),
    1: dict(name="ph_n4096_k32", ph=True, n=4096, k=32, tol=1e-10, seed=10097),
    2: dict(name="tda_n32768_k64", ph=False, n=32768, k=64, tol=1e-8, seed=10098),
    3: dict(name="ph_grad_n16384_k32", ph=True, n=16384, k=32, tol=1e-10, seed=10099),
    4: dict(name="ph_n100000_k100", ph=True, n=100000, k=100, tol=1e-8, seed=10100),
}


def workload_matrix(idx, n=None):
    w = WORKLOADS[idx]
    return Matrix(w["n"] if n is None else n, w["seed"], w["ph"])


def loss_weights(seed, k):
    return uniform(seed, STREAM_LOSS, k)


def test_vectors(seed, n, nvec):
    """Seeded complex test vectors (standard normal real/imag via numpy on a Philox-derived seed)."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    return rng.standard_normal((n, nvec)) + 1j * rng.standard_normal((n, nvec))


def dipole(seed, n):
    """Seeded synthetic dipole vector for optical spectra: N i.i.d. circular complex normal
    entries CN(0, 1) (real and imaginary parts N(0, 1/2)), Philox-keyed like test_vectors."""
    rng = np.random.Generator(np.random.Philox(key=seed + 0x5D1))
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * np.sqrt(0.5)


def packed_index(i, j):
    """Offset of (i, j), i <= j, in LAPACK-'U' packed storage."""
    return i + j * (j + 1) // 2

