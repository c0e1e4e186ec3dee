"""bse_apply_noalloc (the entry point that allocates nothing) against bse_apply, through the C ABI.

Two calls in a row on different handles, the second with a smaller input, each compared with
bse_apply on the same inputs (same kernels, so the results agree to the last bit; the bar checked
is the pass parity bar, 1e-13 relative), the first also against the dense FP64 definition; and a
call whose partial sums exceed the fixed array fails with INVALID_ARG before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2504_10096_amd as bse
from conftest import pack_upper, random_herm, random_sym

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _solver(kind, n, storage, seed):
    rng = np.random.default_rng(seed)
    A = random_herm(rng, n)
    ap = pack_upper(A)
    s = bse.Solver(kind, n, storage=storage)
    s.set_packed("A", torch.as_tensor(ap).to(DEV))
    bp = None
    if kind == "ph":
        bp = pack_upper(random_sym(rng, n, 0.4))
        s.set_packed("B", torch.as_tensor(bp).to(DEV))
    return s, ap, bp, rng


def _call(s, fn, op, prec, x):
    y = torch.full_like(x, complex(np.nan, np.nan))  # every output entry must be written
    lib = bse.load_library()
    with torch.cuda.device(s.device):
        st = getattr(lib, fn)(s._h, op, prec, x.shape[0], ctypes.c_void_p(x.data_ptr()),
                              ctypes.c_void_p(y.data_ptr()))
    torch.cuda.synchronize()
    assert st == bse.OK, (fn, lib.bse_last_error(s._h))
    return y.cpu().numpy()


CASES = [(bse.OP_A, bse.PREC_FP64, 3), (bse.OP_K1, bse.PREC_FP64, 1), (bse.OP_K2, bse.PREC_FP64, 4),
         (bse.OP_H, bse.PREC_FP64, 2), (bse.OP_H, bse.PREC_MIXED, 1), (bse.OP_K1, bse.PREC_HI_FP64, 2),
         (bse.OP_A, bse.PREC_MIXED, 1)]


def test_noalloc_matches_apply_two_calls():
    names = {bse.OP_A: "A", bse.OP_K1: "K1", bse.OP_K2: "K2", bse.OP_H: "H"}
    # first call: N = 1500 (several blocks, ragged tail), hi + lo storage; second: N = 700, fewer vectors
    for n, nvec_cap, seed in [(1500, 4, 11), (700, 1, 12)]:
        s, ap, bp, rng = _solver("ph", n, "hilo", seed)
        for op, prec, nvec in CASES:
            nvec = min(nvec, nvec_cap)
            length = 2 * n if op == bse.OP_H else n
            print(f"noalloc n={n} op={names[op]} prec={prec} nvec={nvec}", flush=True)
            xh = rng.standard_normal((nvec, length)) + 1j * rng.standard_normal((nvec, length))
            x = torch.as_tensor(xh).to(DEV)
            ref = _call(s, "bse_apply", op, prec, x)
            got = _call(s, "bse_apply_noalloc", op, prec, x)
            assert np.all(np.isfinite(got))
            assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
            if prec == bse.PREC_FP64 and n == 1500:
                dense = oracle.apply_dense(names[op], ap, xh, bp)
                assert np.max(np.abs(got - dense)) <= 1e-13 * np.max(np.abs(dense))
        s.close()


def test_noalloc_rejects_oversized_call():
    # PH N = 12000 (block edge 256, 1128 blocks): four fused full-H products need
    # 2 * 4 * 1128 * 256 * 2 complex partials, more than the 64 MiB array; one fits
    n = 12000
    s = bse.Solver("ph", n, storage="c128")
    lib = bse.load_library()
    x = torch.zeros((4, 2 * n), dtype=torch.complex128, device=DEV)
    y = torch.empty_like(x)
    with torch.cuda.device(s.device):
        st = lib.bse_apply_noalloc(s._h, bse.OP_H, bse.PREC_FP64, 4, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(y.data_ptr()))
    assert st == bse.ERR_INVALID_ARG
    assert b"workspace too small" in lib.bse_last_error(s._h)
    y1 = s.apply("H", x[:1], noalloc=True)  # zero triangles, zero vector: a valid call that fits
    torch.cuda.synchronize()
    assert torch.count_nonzero(y1).item() == 0
    s.close()
