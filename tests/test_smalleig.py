"""Host eigensolvers of the library (projected problems of the restart and
of the FP64 refinement) against LAPACK through numpy, built from the same
source with g++ (no GPU)."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("smalleig") / "smalleig")
    cmd = ["g++", "-O2", "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(HERE, "native", "smalleig_driver.cpp"),
           os.path.join(ROOT, "paper_2504_10096_amd", "csrc", "bse_smalleig.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("host compiler unavailable: " + r.stderr[-300:])
    return exe


def run(exe, kind, a):
    m = a.shape[0]
    if kind == "s":
        body = " ".join(f"{v:.17g}" for v in a.T.ravel())
    else:
        body = " ".join(f"{v.real:.17g} {v.imag:.17g}" for v in a.T.ravel())
    out = subprocess.run([exe], input=f"{kind} {m}\n{body}\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    assert out[0] == "1"
    w = np.array([float(x) for x in out[1:1 + m]])
    if kind == "s":
        z = np.array([float(x) for x in out[1 + m:1 + m + m * m]]).reshape(m, m).T
    else:
        pairs = [x.split() for x in out[1 + m:1 + m + m * m]]
        z = np.array([float(p[0]) + 1j * float(p[1]) for p in pairs]).reshape(m, m).T
    return w, z


@pytest.mark.parametrize("m", [1, 2, 3, 17, 64])
def test_sym_eig(driver, m):
    rng = np.random.default_rng(m)
    a = rng.standard_normal((m, m))
    a = a + a.T
    w, z = run(driver, "s", a)
    ref = np.linalg.eigvalsh(a)
    scale = max(1.0, np.abs(ref).max())
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - ref).max() <= 1e-13 * scale
    assert np.abs(z.T @ z - np.eye(m)).max() <= 1e-13
    assert np.abs(a @ z - z * w).max() <= 1e-12 * scale


@pytest.mark.parametrize("m", [1, 2, 5, 31, 80])
def test_herm_eig(driver, m):
    rng = np.random.default_rng(100 + m)
    a = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    a = a + a.conj().T
    w, z = run(driver, "h", a)
    ref = np.linalg.eigvalsh(a)
    scale = max(1.0, np.abs(ref).max())
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - ref).max() <= 1e-13 * scale
    assert np.abs(z.conj().T @ z - np.eye(m)).max() <= 1e-13
    assert np.abs(a @ z - z * w).max() <= 1e-12 * scale


def test_herm_eig_degenerate_and_real(driver):
    # repeated eigenvalues (a complex rotation of diag(1, 1, 2, 2, 3)) and a real input
    rng = np.random.default_rng(7)
    q, _ = np.linalg.qr(rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5)))
    a = q @ np.diag([1.0, 1.0, 2.0, 2.0, 3.0]) @ q.conj().T
    w, z = run(driver, "h", a)
    assert np.abs(w - [1, 1, 2, 2, 3]).max() <= 1e-13
    assert np.abs(z.conj().T @ z - np.eye(5)).max() <= 1e-13
    b = rng.standard_normal((6, 6))
    b = b + b.T
    w, z = run(driver, "h", b.astype(complex))
    assert np.abs(w - np.linalg.eigvalsh(b)).max() <= 1e-13 * np.abs(w).max()


def test_thread_pool_after_fork(tmp_path):
    """A child made by fork() after the pool has started gets a pool of its own (no wait for
    the parent's worker threads) and the same result."""
    exe = str(tmp_path / "smalleig_fork")
    cmd = ["g++", "-O2", "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "paper_2504_10096_amd", "csrc"),
           os.path.join(HERE, "native", "smalleig_fork.cpp"),
           os.path.join(ROOT, "paper_2504_10096_amd", "csrc", "bse_smalleig.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("host compiler unavailable: " + r.stderr[-300:])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, env={**os.environ, "OMP_NUM_THREADS": "4"})
    assert out.returncode == 0, out.stdout + out.stderr
    vals = dict(line.split() for line in out.stdout.strip().splitlines())
    assert vals["parent"] == vals["child"]


@pytest.mark.parametrize("m", [1, 3, 40, 130])
def test_cholesky_and_triangular_solves(driver, m):
    """zchol / zlsolve / zlhsolve against numpy: L lower with a positive diagonal, L L^H = G,
    L X1 = C, L^H X2 = C; an indefinite G is reported (status 0)."""
    rng = np.random.default_rng(300 + m)
    x = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    g = x @ x.conj().T + m * np.eye(m)
    c = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    body = " ".join(f"{v.real:.17g} {v.imag:.17g}" for v in np.concatenate([g.T.ravel(), c.T.ravel()]))
    out = subprocess.run([driver], input=f"c {m}\n{body}\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    assert out[0] == "1"
    vals = np.array([complex(float(a), float(b)) for a, b in (ln.split() for ln in out[1:1 + 2 * m * m])])
    x1 = vals[:m * m].reshape(m, m).T
    x2 = vals[m * m:].reshape(m, m).T
    lref = np.linalg.cholesky(g)
    scale = np.abs(c).max()
    assert np.abs(lref @ x1 - c).max() <= 1e-11 * scale * m
    assert np.abs(lref.conj().T @ x2 - c).max() <= 1e-11 * scale * m
    # not positive definite: status 0
    gbad = g - (np.abs(np.linalg.eigvalsh(g)).max() + 1.0) * np.eye(m)
    body = " ".join(f"{v.real:.17g} {v.imag:.17g}" for v in np.concatenate([gbad.T.ravel(), c.T.ravel()]))
    out = subprocess.run([driver], input=f"c {m}\n{body}\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    assert out[0] == "0"


@pytest.mark.parametrize("m,k,clustered", [(2, 1, False), (10, 3, False), (400, 12, False), (600, 20, True)])
def test_tridiag0_lowest_positive(driver, m, k, clustered):
    """Zero-diagonal symmetric tridiagonal (the real form of -i T for the skew tridiagonal T of the
    direct solve): the k smallest positive eigenvalues and orthonormal vectors against numpy."""
    rng = np.random.default_rng(m + k)
    f = rng.uniform(0.05, 3.0, m - 1)
    if clustered:
        # two equal halves joined by a tiny coupling: every eigenvalue comes as a nearly equal pair
        h = m // 2
        f[h:] = f[:h - 1]
        f[h - 1] = 1e-10
    body = " ".join(f"{v:.17g}" for v in f)
    out = subprocess.run([driver], input=f"t {m} {k}\n{body}\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    assert out[0] == "1"
    w = np.array([float(x) for x in out[1:1 + k]])
    z = np.array([float(x) for x in out[1 + k:1 + k + m * k]]).reshape(k, m).T
    S = np.diag(f, 1) + np.diag(f, -1)
    ev = np.linalg.eigvalsh(S)
    ref = np.sort(ev[ev > 0])[:k]
    scale = np.abs(ev).max()
    assert np.abs(w - ref).max() <= 1e-13 * scale
    assert np.abs(z.T @ z - np.eye(k)).max() <= 1e-10
    assert np.abs(S @ z - z * w).max() <= 1e-11 * scale
