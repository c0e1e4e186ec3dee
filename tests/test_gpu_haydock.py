"""GPU parity of the Lanczos-Haydock path (bse_haydock, bse_haydock_spectrum)
against the oracle: recurrence coefficients element by element against the
oracle's FP64 recurrence, the device continued fraction against the oracle's
fraction of the same coefficients, converged spectra against the dense
resolvent definitions, reduced-precision passes against the oracle on the
complex64-rounded matrix, and the edge and error cases."""
import numpy as np
import pytest
import torch

import oracle.haydock as hy
import paper_2504_10096_amd as bse
import synth
from conftest import hi_operator, pack_upper, ph_matrix, random_herm, random_sym, synth_matrix

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ETA = 0.1


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def make_solver(kind, ap, bp=None, storage="c128"):
    n = int(round(((8 * len(ap) + 1) ** 0.5 - 1) / 2))
    s = bse.Solver(kind, n, storage=storage)
    s.set_packed("A", dev(ap))
    if bp is not None:
        s.set_packed("B", dev(bp))
    return s


def oracle_recurrence(kind, ap, bp, d, n_iter):
    ops = hy.dense_ops(ap, bp if kind == "ph" else None)
    if kind == "tda":
        return hy.lanczos_tda(ops, d, n_iter)
    return hy.lanczos_ph(ops[0], ops[1], d, n_iter)


def exact_chi(kind, ap, bp, d, z):
    return hy.chi_tda_exact(ap, d, z) if kind == "tda" else hy.chi_ph_exact(ap, bp, d, z)


def case(kind, n):
    m = synth_matrix(n, 400 + n, kind == "ph")
    ap = m.pack_host(0)
    bp = m.pack_host(1) if kind == "ph" else None
    return ap, bp, synth.dipole(n, n), window(m)


def window(m):
    """Frequencies covering the spectrum of a seeded matrix: from below its certified lower
    bound to above eps_max + shift + the direct term's row radius."""
    return m.lambda_min_a - 1.0, m.shift + 9.0 + m.beta * m.r_w


@pytest.mark.parametrize("kind", ["tda", "ph"])
@pytest.mark.parametrize("n", [300, 1000])
def test_coefficients_match_oracle(kind, n):
    print(f"haydock coefficients {kind} n={n}", flush=True)
    ap, bp, d, (lo, hi) = case(kind, n)
    s = make_solver(kind, ap, bp)
    freq = np.linspace(lo, hi, 64)
    al, be, nn, chi, st = s.haydock(dev(d), 30, freq=dev(freq), eta=ETA)
    ra, rb, rn = oracle_recurrence(kind, ap, bp, d, 30)
    al, be = host(al), host(be)
    assert len(al) == 30
    # before orthogonality is lost the two recurrences agree to rounding
    assert np.max(np.abs(al[:20] - ra[:20])) <= 1e-11 * np.max(np.abs(ra))
    assert np.max(np.abs(be[:20] - rb[:20])) <= 1e-11 * np.max(np.abs(rb))
    assert abs(nn - rn) <= 1e-12 * rn
    # the device fraction of these coefficients equals the oracle's fraction of them
    ref = hy.continued_fraction(al, be, nn, freq + 1j * ETA, kind)
    assert np.max(np.abs(host(chi) - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert st["passes"] == (30 if kind == "tda" else 61)  # PH: one K1 pass for the start vector
    s.close()


@pytest.mark.parametrize("kind", ["tda", "ph"])
@pytest.mark.parametrize("n", [300, 1000])
def test_converged_spectrum_matches_definition(kind, n):
    print(f"haydock spectrum {kind} n={n}", flush=True)
    ap, bp, d, (lo, hi) = case(kind, n)
    s = make_solver(kind, ap, bp)
    freq = np.linspace(max(lo, 0.05), hi, 16)
    al, be, nn, chi, st = s.haydock(dev(d), 3 * n, tol=1e-11, freq=dev(freq), eta=ETA)
    assert len(al) < 3 * n and len(al) % 20 == 0  # stopped at a check
    ex = exact_chi(kind, ap, bp, d, freq + 1j * ETA)
    assert np.max(np.abs(host(chi) - ex)) <= 1e-8 * np.max(np.abs(ex))
    # absorption is positive at positive frequency
    assert np.all(-host(chi).imag > 0)
    print("steps", len(al), "passes", st["passes"], flush=True)
    s.close()


@pytest.mark.parametrize("kind", ["tda", "ph"])
def test_reduced_precision_passes(kind):
    n = 700
    ap, bp, d, _ = case(kind, n)
    ap32, bp32 = hi_operator(ap, bp)  # hi = fl32(a) (round to nearest), FP64 diagonal of A
    s = make_solver(kind, ap, bp, storage="hilo")
    # FP64 operator from hi + lo: the FP64 recurrence
    al, be, nn, _, _ = s.haydock(dev(d), 20, precision="fp64")
    ra, rb, rn = oracle_recurrence(kind, ap, bp, d, 20)
    assert np.max(np.abs(host(al) - ra)) <= 1e-11 * np.max(np.abs(ra))
    # FP64 arithmetic on hi: the recurrence of the complex64-rounded matrix (FP64 diagonal of A)
    al, be, nn, _, _ = s.haydock(dev(d), 20, precision="hi64")
    ra, rb, rn = oracle_recurrence(kind, ap32, bp32, d, 20)
    assert np.max(np.abs(host(al) - ra)) <= 1e-11 * np.max(np.abs(ra))
    assert np.max(np.abs(host(be) - rb)) <= 1e-11 * np.max(np.abs(rb))
    # complex FP32 products: the same within single-precision rounding
    al, be, nn, _, _ = s.haydock(dev(d), 10, precision="fp32")
    assert np.max(np.abs(host(al) - ra[:10])) <= 1e-5 * np.max(np.abs(ra))
    assert np.max(np.abs(host(be) - rb[:10])) <= 1e-5 * np.max(np.abs(rb))
    s.close()


@pytest.mark.parametrize("n", [1, 2, 17])
def test_tiny_sizes_fraction_is_exact(n):
    rng = np.random.default_rng(70 + n)
    A, B = random_herm(rng, n, lam_min=1.0), random_sym(rng, n, 0.5)
    ap, bp = pack_upper(A), pack_upper(B)
    d = synth.dipole(70 + n, n)
    freq = np.linspace(0.3, 9.0, 12)
    z = freq + 1j * ETA
    for kind in ("tda", "ph"):
        s = make_solver(kind, ap, bp if kind == "ph" else None)
        _, _, _, chi, _ = s.haydock(dev(d), 4 * n + 4, freq=dev(freq), eta=ETA)
        ex = exact_chi(kind, ap, bp, d, z)
        assert np.max(np.abs(host(chi) - ex)) <= 1e-9 * np.max(np.abs(ex)), kind
        s.close()


def test_b_zero_and_standalone_spectrum():
    n = 400
    m = ph_matrix(n, 91)
    ap = m.pack_host(0)
    bp = np.zeros_like(ap)
    d = synth.dipole(91, n)
    lo, hi = window(m)
    freq = np.linspace(lo, hi, 24)
    z = freq + 1j * ETA
    s = make_solver("ph", ap, bp)
    al, be, nn, chi, _ = s.haydock(dev(d), 3 * n, tol=1e-11, freq=dev(freq), eta=ETA)
    tda = hy.chi_tda_exact(ap, d, z)
    tda_m = hy.chi_tda_exact(ap, d, -np.conj(z))
    assert np.max(np.abs(host(chi) - (tda + np.conj(tda_m)))) <= 1e-8 * np.max(np.abs(tda))
    chi2 = bse.haydock_spectrum("ph", al, be, nn, dev(freq), ETA)
    assert torch.equal(chi2, chi)
    s.close()


def test_deterministic_bitwise():
    ap, bp, d, _ = case("ph", 600)
    s = make_solver("ph", ap, bp)
    a = s.haydock(dev(d), 40)
    b = s.haydock(dev(d), 40)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2]
    s.close()


def test_errors():
    n = 60
    A = np.diag(np.arange(1.0, n + 1)).astype(complex)
    B = np.zeros((n, n), dtype=complex)
    B[0, 0] = 1.6
    s = make_solver("ph", pack_upper(A), pack_upper(B))
    d = np.zeros(n, complex)
    d[0] = 1j  # <d, K1 d> = 1 - 1.6 < 0
    with pytest.raises(bse.NotPositiveDefinite):
        s.haydock(dev(d), 4)
    with pytest.raises(bse.BSEError) as e:
        s.haydock(dev(np.zeros(n, complex)), 4)
    assert e.value.status == bse.ERR_INVALID_ARG
    d = synth.dipole(1, n)
    for kw in [dict(n_iter=0), dict(n_iter=4, tol=-1.0), dict(n_iter=4, tol=1e-6),
               dict(n_iter=4, precision="hi64")]:
        with pytest.raises(bse.BSEError) as e:
            s.haydock(dev(d), **kw)
        assert e.value.status == bse.ERR_INVALID_ARG, kw
    with pytest.raises(bse.BSEError) as e:
        s.haydock(dev(d), 4, freq=dev(np.linspace(1, 2, 3)), eta=0.0)
    assert e.value.status == bse.ERR_INVALID_ARG
    s.close()


@pytest.mark.parametrize("kind", ["tda", "ph"])
@pytest.mark.parametrize("nd", [3, 5])
def test_several_dipoles_match_single_runs(kind, nd):
    """nd dipoles advancing together (groups of up to four per read of the triangles) give
    the single-dipole recurrences and spectra; the reads are shared."""
    n = 700
    ap, bp, _, (lo, hi) = case(kind, n)
    D = np.stack([synth.dipole(500 + q, n) for q in range(nd)])
    freq = np.linspace(max(lo, 0.05), hi, 32)
    s = make_solver(kind, ap, bp, storage="hilo")
    for prec in ("fp64", "hi64"):
        al, be, nn, chi, st = s.haydock(dev(D), 40, freq=dev(freq), eta=ETA, precision=prec)
        groups = (nd + 3) // 4
        assert st["passes"] == (40 * groups if kind == "tda" else (1 + 2 * 40) * groups)
        for q in range(nd):
            a1, b1, n1, c1, _ = s.haydock(dev(D[q]), 40, freq=dev(freq), eta=ETA, precision=prec)
            assert np.max(np.abs(host(al[q]) - host(a1))) <= 1e-11 * np.max(np.abs(host(a1))), (prec, q)
            assert np.max(np.abs(host(be[q]) - host(b1))) <= 1e-11 * np.max(np.abs(host(b1))), (prec, q)
            assert abs(nn[q] - n1) <= 1e-13 * n1
            assert np.max(np.abs(host(chi[q]) - host(c1))) <= 1e-10 * np.max(np.abs(host(c1))), (prec, q)
    # and against the oracle's recurrence
    al, be, nn, _, _ = s.haydock(dev(D), 20)
    for q in range(nd):
        ra, rb, rn = oracle_recurrence(kind, ap, bp, D[q], 20)
        assert np.max(np.abs(host(al[q]) - ra)) <= 1e-11 * np.max(np.abs(ra))
    s.close()
