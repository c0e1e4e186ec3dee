"""The solver's driver (bse_solver.cpp) on the CPU: the same source compiled with
g++ against a host backend of the kernel launchers (tests/native/host_backend.cpp,
plain loops), so that restarts, the FP64 refinement, both pseudo-Hermitian
variants, the Haydock recurrence and every error path run in the CPU suite.
Results are checked against the oracle.  Failure injection is forced from the
host (indefinite M, a NaN entry, a one-restart budget, invalid arguments); no
GPU is involved.  This backend is test infrastructure, not a fallback: the
package never loads it."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import oracle.haydock as hy
import synth
from conftest import pack_upper, ph_matrix, random_herm, random_sym, synth_matrix

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2504_10096_amd", "csrc")

OK, INVALID, OOM, DEVICE, NOT_PD, NOT_CONV, NONFINITE, BAD_STATE = range(8)
vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double


# the ABI structs of include/bse.h, as the binding declares them (kept in one place so that a field
# added to the header cannot leave a shorter struct here for the library to write past)
from paper_2504_10096_amd import Allocator, SolveOpts as Opts, Stats  # noqa: E402
from paper_2504_10096_amd import _ALLOC_FN, _FREE_FN  # noqa: E402


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("hostdrv") / "libbse_hostdrv.so")
    cmd = ["g++", "-O2", "-std=c++17", "-pthread", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-fcx-limited-range", "-w", os.path.join(HERE, "native", "host_backend.cpp"),
           os.path.join(CSRC, "bse_solver.cpp"), os.path.join(CSRC, "bse_smalleig.cpp"), "-o", so,
           "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib", "-Wl,-Bsymbolic"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("host compiler or ROCm libraries unavailable: " + r.stderr[-300:])
    L = ctypes.CDLL(so)
    L.bse_create.argtypes = [ctypes.POINTER(vp), i32, i64, i32, vp]
    L.bse_create_ex.argtypes = [ctypes.POINTER(vp), i32, i64, i32, vp, ctypes.POINTER(Allocator)]
    L.bse_set_packed.argtypes = [vp, i32, i64, i64, vp, i32]
    L.bse_solve.argtypes = [vp, i32, dbl, ctypes.POINTER(Opts), vp, vp, vp, ctypes.POINTER(Stats)]
    L.bse_haydock.argtypes = [vp, i32, vp, i32, dbl, i32, vp, i32, dbl, vp, vp, ctypes.POINTER(dbl), vp,
                              ctypes.POINTER(i32), ctypes.POINTER(Stats)]
    L.bse_backward.argtypes = [vp, vp, vp, vp]
    L.bse_destroy.argtypes = [vp]
    L.bse_last_error.argtypes = [vp]
    L.bse_last_error.restype = ctypes.c_char_p
    return L


class Handle:
    def __init__(self, L, kind, ap, bp=None, storage=0):
        self.L, self.kind = L, kind
        self.n = int(round(((8 * len(ap) + 1) ** 0.5 - 1) / 2))
        self.h = vp()
        assert L.bse_create(ctypes.byref(self.h), kind, self.n, storage, None) == OK
        self.keep = [np.ascontiguousarray(ap, dtype=np.complex128)]
        assert L.bse_set_packed(self.h, 0, 0, self.n, self.keep[0].ctypes.data, 1) == OK
        if bp is not None:
            self.keep.append(np.ascontiguousarray(bp, dtype=np.complex128))
            assert L.bse_set_packed(self.h, 1, 0, self.n, self.keep[1].ctypes.data, 1) == OK

    def solve(self, k, tol, **kw):
        om = np.zeros(k)
        X = np.zeros((k, self.n), complex)
        Y = np.zeros((k, self.n), complex) if self.kind else None
        o = Opts(kw.get("ncv", 0), kw.get("keep", 0), kw.get("max_restarts", 0), kw.get("precision", 0), 0.0, 1,
                 kw.get("fp32_arith", 0), kw.get("block", 0), 0, kw.get("variant", 0))
        warm = kw.get("warm")
        if warm is not None:  # previous (X, Y) as returned: n x k, column c = pair c
            wx = np.ascontiguousarray(warm[0].T, dtype=np.complex128)
            wy = None if warm[1] is None else np.ascontiguousarray(warm[1].T, dtype=np.complex128)
            self.keep_warm = (wx, wy)
            o.warm_k, o.warm_x = wx.shape[0], wx.ctypes.data
            o.warm_y = None if wy is None else wy.ctypes.data
        st = Stats()
        rc = self.L.bse_solve(self.h, k, tol, ctypes.byref(o), om.ctypes.data, X.ctypes.data,
                              None if Y is None else Y.ctypes.data, ctypes.byref(st))
        return rc, om, X.T, None if Y is None else Y.T, st

    def haydock(self, D, n_iter):
        D = np.ascontiguousarray(np.atleast_2d(D), dtype=np.complex128)
        nd = D.shape[0]
        al, be = np.zeros((nd, n_iter)), np.zeros((nd, n_iter))
        nn, done, st = (dbl * nd)(), i32(0), Stats()
        rc = self.L.bse_haydock(self.h, nd, D.ctypes.data, n_iter, 0.0, 0, None, 0, 0.1, al.ctypes.data,
                                be.ctypes.data, nn, None, ctypes.byref(done), ctypes.byref(st))
        return rc, al[:, :done.value], be[:, :done.value], list(nn), st

    def error(self):
        return self.L.bse_last_error(self.h).decode()

    def close(self):
        self.L.bse_destroy(self.h)


def ph_case(n=120, seed=5):
    m = ph_matrix(n, seed)
    return m.pack_host(0), m.pack_host(1)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("storage,precision,fp32,tol", [(0, 0, 0, 1e-10), (1, 1, 0, 1e-8), (1, 1, 1, 1e-8)])
def test_ph_solve_matches_oracle(lib, variant, storage, precision, fp32, tol):
    ap, bp = ph_case()
    h = Handle(lib, 1, ap, bp, storage)
    rc, om, X, Y, st = h.solve(5, tol, variant=variant, precision=precision, fp32_arith=fp32, ncv=32)
    if variant == 3 and fp32:  # the fused full-H passes have no complex FP32 form
        assert rc == INVALID
        h.close()
        return
    assert rc == OK, h.error()
    ref, _, _ = oracle.ph(ap, bp, 5, vectors=False)
    assert np.max(np.abs(om - ref) / ref) < tol
    assert oracle.residual_ph(ap, bp, om, X, Y).max() <= tol * 1.01
    nrm = np.sum(np.abs(X) ** 2, axis=0) - np.sum(np.abs(Y) ** 2, axis=0)
    assert np.max(np.abs(nrm - 1)) < 1e-9
    assert st.restarts >= 1 and st.passes > 0
    h.close()


@pytest.mark.parametrize("block", [1, 2])
def test_tda_solve_matches_oracle(lib, block):
    m = synth.Matrix(150, 6, ph=False)
    ap = m.pack_host(0)
    h = Handle(lib, 0, ap)
    rc, lam, X, _, st = h.solve(6, 1e-10, block=block, ncv=32)
    assert rc == OK, h.error()
    ref, _ = oracle.tda(ap, 6, vectors=False)
    assert np.max(np.abs(lam - ref) / np.abs(ref)) < 1e-10
    assert oracle.residual_tda(ap, lam, X).max() <= 1e-10 * 1.01
    assert st.block == block
    h.close()


@pytest.mark.parametrize("block", [1, 2, 3, 4])
def test_ph_block_full_h_matches_oracle(lib, block):
    """Variant 3 (block Lanczos on H in the M inner product) with 1..4 full-H vectors per read:
    the oracle's pairs, residuals within tol, normalized vectors, one read per block step."""
    ap, bp = ph_case(200, 9)
    k = 10
    h = Handle(lib, 1, ap, bp, 1)
    rc, om, X, Y, st = h.solve(k, 1e-8, variant=3, block=block, precision=1)
    assert rc == OK, h.error()
    assert st.block == block
    ref, _, _ = oracle.ph(ap, bp, k, vectors=False)
    assert np.max(np.abs(om - ref) / ref) < 1e-8
    assert oracle.residual_ph(ap, bp, om, X, Y).max() <= 1e-8 * 1.01
    nrm = np.sum(np.abs(X) ** 2, axis=0) - np.sum(np.abs(Y) ** 2, axis=0)
    assert np.max(np.abs(nrm - 1)) < 1e-9
    assert st.steps_fp32 > 0 and st.steps_fp32 % block == 0
    h.close()


@pytest.mark.parametrize("kind", ["tda", "ph", "ph3"])
def test_warm_start_from_nearby_matrix(lib, kind):
    """A solve started from the eigenvectors of a nearby matrix (alpha + 1e-6, as in a finite
    difference) finds the same pairs as a cold solve of that matrix, in fewer passes (ph3: the
    block full-H iteration, variant 3)."""
    variant = 3 if kind == "ph3" else 0
    kind = "ph" if kind == "ph3" else kind
    n, k, tol = 160, 8, 1e-12
    base = synth_matrix(n, 12, kind == "ph")
    near = synth.Matrix(n, 12, ph=kind == "ph", alpha=1.0 + 1e-6, tables=base.tables, shift=base.shift,
                        b_norm=base.b_norm if kind == "ph" else None)
    blocks = lambda m: (m.pack_host(0), m.pack_host(1) if kind == "ph" else None)
    h0 = Handle(lib, int(kind == "ph"), *blocks(base))
    rc, om0, X0, Y0, _ = h0.solve(k, tol, ncv=32, variant=variant)
    assert rc == OK, h0.error()
    h0.close()
    ap, bp = blocks(near)
    h1 = Handle(lib, int(kind == "ph"), ap, bp)
    rc, om_c, _, _, st_c = h1.solve(k, tol, ncv=32, variant=variant)
    assert rc == OK, h1.error()
    rc, om_w, Xw, Yw, st_w = h1.solve(k, tol, ncv=32, warm=(X0, Y0), variant=variant)
    assert rc == OK, h1.error()
    assert np.max(np.abs(om_w - om_c) / np.abs(om_c)) < 1e-11
    rel = oracle.residual_ph(ap, bp, om_w, Xw, Yw) if kind == "ph" else oracle.residual_tda(ap, om_w, Xw)
    assert rel.max() <= tol * 1.01
    print(f"{kind}: passes cold {st_c.passes}, warm {st_w.passes}")
    assert st_w.passes < st_c.passes, (st_w.passes, st_c.passes)
    # invalid warm arguments are rejected before any work
    o = Opts()
    o.warm_k = 3
    assert lib.bse_solve(h1.h, k, tol, ctypes.byref(o), om_w.ctypes.data, Xw.ctypes.data,
                         None if Yw is None else Yw.ctypes.data, None) == INVALID
    h1.close()


def test_backward_through_host_driver(lib):
    ap, bp = ph_case(80, 7)
    h = Handle(lib, 1, ap, bp)
    rc, om, X, Y, _ = h.solve(4, 1e-12)
    assert rc == OK
    g = synth.loss_weights(3, 4)
    m = len(ap)
    ga, gb = np.zeros(m, complex), np.zeros(m, complex)
    assert lib.bse_backward(h.h, g.ctypes.data, ga.ctypes.data, gb.ctypes.data) == OK
    ra, rb = oracle.grad_ph(X, Y, g)
    assert np.max(np.abs(ga - ra)) < 1e-12 * np.max(np.abs(ra))
    assert np.max(np.abs(gb - rb)) < 1e-12 * np.max(np.abs(rb))
    h.close()


def test_not_positive_definite_is_reported(lib):
    n = 60
    A = np.diag(np.arange(1.0, n + 1)).astype(complex)
    B = np.zeros((n, n), dtype=complex)
    B[0, 0] = 1.6  # ||B|| > lambda_min(A): M indefinite
    for variant in (0, 1, 2, 3):
        h = Handle(lib, 1, pack_upper(A), pack_upper(B))
        rc, *_ = h.solve(4, 1e-10, variant=variant)
        assert rc == NOT_PD, (variant, rc, h.error())
        d = np.zeros(n, complex)
        d[0] = 1j  # <d, K1 d> = 1 - 1.6 < 0
        rc, *_ = h.haydock(d, 4)
        assert rc == NOT_PD
        h.close()


def test_not_converged_returns_best(lib):
    m = synth.Matrix(200, 9, ph=False)
    ap = m.pack_host(0)
    h = Handle(lib, 0, ap)
    rc, lam, X, _, st = h.solve(8, 1e-13, max_restarts=1, ncv=24)
    assert rc == NOT_CONV
    assert st.restarts == 1 and st.n_converged < 8
    assert np.all(np.isfinite(lam)) and np.all(np.isfinite(X))
    # the partial results are Ritz pairs of a subspace: each value is its vector's
    # Rayleigh quotient and, by interlacing, not below the matching eigenvalue
    ref, _ = oracle.tda(ap, 8, vectors=False)
    AX = oracle.apply_dense("A", ap, X.T).T
    rq = np.real(np.sum(np.conj(X) * AX, axis=0)) / np.sum(np.abs(X) ** 2, axis=0)
    assert np.max(np.abs(rq - lam)) < 1e-10 * np.max(np.abs(lam))
    assert np.all(lam >= ref - 1e-10)
    h.close()


@pytest.mark.parametrize("variant", [0, 2, 3])
def test_ph_not_converged_returns_pairs_of_h(lib, variant):
    """An unreachable tol (1e-17): after the restart budget the best approximations come back as (X, Y) of H
    itself (the dual iteration's vectors are mapped back from diag(I, -I) H diag(I, -I)),
    normalized, and the lowest pairs, converged by then, have small residuals with respect to H
    (a Y of the wrong sign would leave a residual of the size of Y)."""
    ap, bp = ph_case(150, 4)
    h = Handle(lib, 1, ap, bp)
    # variant 3 keeps both signs of omega: a basis twice as large for the same progress
    rc, om, X, Y, st = h.solve(6, 1e-17, max_restarts=20, ncv=48 if variant == 3 else 24, variant=variant)
    assert rc == NOT_CONV
    nrm = np.sum(np.abs(X) ** 2, axis=0) - np.sum(np.abs(Y) ** 2, axis=0)
    assert np.max(np.abs(nrm - 1)) < 1e-9
    rel = oracle.residual_ph(ap, bp, om, X, Y)
    assert rel[0] < 1e-6, rel
    assert np.min(np.linalg.norm(Y, axis=0)) > 1e-3  # the check above sees the sign of Y
    ref, _, _ = oracle.ph(ap, bp, 6, vectors=False)
    # the folded iterations approach omega^2 from above (extreme eigenvalues of K2 K1); on H the
    # wanted omega are interior, and a Ritz value may sit below by O(residual^2 / gap)
    assert np.all(om >= ref * (1 - (1e-6 if variant == 3 else 1e-12)))
    h.close()


def test_nonfinite_input_is_reported(lib):
    n = 40
    A = random_herm(np.random.default_rng(2), n)
    A[3, 7] = np.nan
    A[7, 3] = np.nan
    h = Handle(lib, 0, pack_upper(A))
    rc, *_ = h.solve(3, 1e-10)
    assert rc == NONFINITE, h.error()
    h.close()


def test_invalid_arguments(lib):
    ap = pack_upper(random_herm(np.random.default_rng(1), 30))
    h = Handle(lib, 0, ap)
    for k, tol in [(0, 1e-8), (31, 1e-8), (3, 0.0), (3, -1.0)]:
        rc, *_ = h.solve(k, tol)
        assert rc == INVALID, (k, tol)
    rc, *_ = h.solve(3, 1e-8, variant=4)
    assert rc == INVALID
    rc, *_ = h.solve(3, 1e-8, precision=1)  # mixed needs hi + lo storage
    assert rc == INVALID
    g = np.ones(3)
    assert lib.bse_backward(h.h, g.ctypes.data, None, None) == BAD_STATE  # before a solve
    om, X, Y = np.zeros(3), np.zeros((3, 30), complex), np.zeros((3, 30), complex)
    assert lib.bse_solve(h.h, 3, 1e-8, None, om.ctypes.data, X.ctypes.data, Y.ctypes.data, None) == INVALID
    assert lib.bse_solve(h.h, 3, 1e-8, None, None, X.ctypes.data, None, None) == INVALID
    rc, *_ = h.haydock(np.zeros(30, complex), 4)  # zero dipole
    assert rc == INVALID
    h.close()


@pytest.mark.parametrize("kind", [0, 1])
def test_haydock_several_dipoles(lib, kind):
    rng = np.random.default_rng(kind)
    n = 90
    A, B = random_herm(rng, n, lam_min=1.0), random_sym(rng, n, 0.5)
    ap, bp = pack_upper(A), pack_upper(B)
    h = Handle(lib, kind, ap, bp if kind else None)
    D = np.stack([synth.dipole(30 + q, n) for q in range(5)])  # a group of four and one more
    rc, al, be, nn, st = h.haydock(D, 12)
    assert rc == OK, h.error()
    assert st.passes == (12 * 2 if kind == 0 else (1 + 2 * 12) * 2)
    for q in range(5):
        if kind == 0:
            ra, rb, rn = hy.lanczos_tda(hy.dense_ops(ap), D[q], 12)
        else:
            k1, k2 = hy.dense_ops(ap, bp)
            ra, rb, rn = hy.lanczos_ph(k1, k2, D[q], 12)
        assert np.max(np.abs(al[q] - ra)) <= 1e-11 * np.max(np.abs(ra))
        assert np.max(np.abs(be[q] - rb)) <= 1e-11 * np.max(np.abs(rb))
        assert abs(nn[q] - rn) <= 1e-12 * rn
    h.close()


class CountingAllocator:
    """bse_allocator over libc malloc/free that tracks live blocks; fail_at = n makes the n-th
    request (1-based) return NULL."""

    def __init__(self, fail_at=0):
        self.libc = ctypes.CDLL(None)
        self.libc.malloc.restype, self.libc.malloc.argtypes = vp, [ctypes.c_size_t]
        self.libc.free.argtypes = [vp]
        self.live, self.calls, self.fail_at = {}, 0, fail_at
        self.struct = Allocator(_ALLOC_FN(self._alloc), _FREE_FN(self._free), None)

    def _alloc(self, nbytes, stream, ctx):
        self.calls += 1
        if self.calls == self.fail_at:
            return None
        p = self.libc.malloc(nbytes)
        self.libc.memset(ctypes.c_void_p(p), 0, ctypes.c_size_t(nbytes))
        self.live[p] = nbytes
        return p

    def _free(self, ptr, stream, ctx):
        assert ptr in self.live, "free of a pointer the allocator did not return"
        del self.live[ptr]
        self.libc.free(ctypes.c_void_p(ptr))


def test_allocator_hook_takes_every_buffer(lib):
    """bse_create_ex: the triangles and every workspace of solve / backward / Haydock come from
    the caller's allocator, results equal those of bse_create's handle, and destroy returns every
    block.  A NULL from the allocator at any request of create is OUT_OF_MEMORY with nothing
    leaked."""
    ap, bp = ph_case(90, 11)
    n, k = 90, 4
    ref = Handle(lib, 1, ap, bp)
    rc, om0, X0, Y0, _ = ref.solve(k, 1e-12)
    assert rc == OK
    al = CountingAllocator()
    h = vp()
    assert lib.bse_create_ex(ctypes.byref(h), 1, n, 0, None, ctypes.byref(al.struct)) == OK
    assert sum(al.live.values()) >= 2 * 16 * n * (n + 1) // 2
    other = Handle.__new__(Handle)
    other.L, other.kind, other.n, other.h = lib, 1, n, h
    other.keep = [np.ascontiguousarray(ap), np.ascontiguousarray(bp)]
    assert lib.bse_set_packed(h, 0, 0, n, other.keep[0].ctypes.data, 1) == OK
    assert lib.bse_set_packed(h, 1, 0, n, other.keep[1].ctypes.data, 1) == OK
    calls = al.calls
    rc, om1, X1, Y1, _ = other.solve(k, 1e-12)
    assert rc == OK and al.calls > calls  # the solve's workspaces went through the hook
    assert np.array_equal(om0, om1) and np.array_equal(X0, X1) and np.array_equal(Y0, Y1)
    g = synth.loss_weights(3, k)
    ga, gb = np.zeros(len(ap), complex), np.zeros(len(ap), complex)
    assert lib.bse_backward(h, g.ctypes.data, ga.ctypes.data, gb.ctypes.data) == OK
    d = np.random.default_rng(2).standard_normal(n) + 0j
    assert other.haydock(d, 6)[0] == OK
    # a NULL from the allocator inside a solve is OUT_OF_MEMORY; the handle stays usable
    al.fail_at = al.calls + 1
    rc, *_ = other.solve(k, 1e-12)
    assert rc == OOM, rc
    rc, om2, *_ = other.solve(k, 1e-12)
    assert rc == OK and np.array_equal(om0, om2)
    other.close()
    assert not al.live
    ref.close()
    # allocator failure at each request of create: OUT_OF_MEMORY and nothing left allocated
    n_create = CountingAllocator()
    assert lib.bse_create_ex(ctypes.byref(h), 1, n, 1, None, ctypes.byref(n_create.struct)) == OK
    lib.bse_destroy(h)
    for fail_at in range(1, n_create.calls + 1):
        bad = CountingAllocator(fail_at)
        h = vp()
        assert lib.bse_create_ex(ctypes.byref(h), 1, n, 1, None, ctypes.byref(bad.struct)) == OOM
        assert not bad.live, fail_at
    # an allocator without both functions is rejected
    half = Allocator(al.struct.alloc, _FREE_FN(), None)
    assert lib.bse_create_ex(ctypes.byref(h), 1, n, 0, None, ctypes.byref(half)) == INVALID
