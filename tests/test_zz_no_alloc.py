"""sbd_sigma_noalloc (the sigma entry point whose workspace is the library's
static device scratch) against sbd_sigma, through the C ABI: the same kernels
and launch configuration, so the outputs must agree bit for bit, which is
inside the parity bar of sigma (FP64 within 1e-12 of the oracle, checked here
too).  Two products in a row, the second on a smaller basis, so the second
reads a scratch that still holds the first one's contents."""
import ctypes

import numpy as np
import pytest

import oracle
import workload as wl

torch = pytest.importorskip("torch")
sbd = pytest.importorskip("paper_2601_16637_amd")
from paper_2601_16637_amd import _native  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SCRATCH_BYTES = 256 << 20  # SBD_NOALLOC_SCRATCH_BYTES of include/sbd.h


def system(nstr):
    W = wl.make_config("sel16", nstr=nstr)
    bas = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta)
    exc = sbd.Excitations(bas)
    ham = sbd.Hamiltonian(bas, exc, W.h, W.eri, W.e_core)
    return W, ham


def call_abi(fn, ham, x, y, nvec, prec, shift, layout):
    """One call of sbd_sigma or sbd_sigma_noalloc through ctypes; returns the status."""
    return getattr(_native.load(), fn)(ham.basis._h, ham.exc._h, ham._h, int(nvec), int(prec),
                                        float(shift), ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(y.data_ptr()), int(layout),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


CASES = [  # (precision, vectors, layout, shift)
    (0, 1, 0, 0.0),
    (1, 1, 0, -200.0),
    (0, 4, 1, 0.0),
    (1, 8, 1, -150.0),
    (0, 2, 0, 0.0),
]


def run_cases(W, ham, seed):
    N = W.ndet
    rng = np.random.default_rng(seed)
    out = []
    for prec, nvec, layout, shift in CASES:
        dt = torch.float64 if prec == 0 else torch.float32
        x = torch.tensor(rng.standard_normal(N * nvec), device=DEV, dtype=dt)
        y_ref = torch.full_like(x, float("nan"))
        y_new = torch.full_like(x, float("nan"))
        assert call_abi("sbd_sigma", ham, x, y_ref, nvec, prec, shift, layout) == 0, sbd.last_error()
        assert call_abi("sbd_sigma_noalloc", ham, x, y_new, nvec, prec, shift, layout) == 0, sbd.last_error()
        torch.cuda.synchronize()
        assert torch.equal(y_ref, y_new), (prec, nvec, layout)
        out.append((prec, nvec, layout, shift, x.cpu().numpy().astype(np.float64),
                    y_new.cpu().numpy().astype(np.float64)))
    return out


def test_noalloc_equals_sigma_two_calls_second_smaller():
    big_W, big = system(1000)      # 1e6 determinants: up to 64 MB of scratch (FP64, 4 vectors)
    small_W, small = system(300)   # 9e4 determinants
    run_cases(big_W, big, 1)
    res = run_cases(small_W, small, 2)
    # the second (smaller) product against the oracle's FP64 sigma
    S = oracle.OracleSystem.from_workload(small_W)
    N = small_W.ndet
    for prec, nvec, layout, shift, x, y in res:
        if prec != 0:
            continue
        X = x.reshape(N, nvec).T if layout == 1 else x.reshape(nvec, N)
        Y = y.reshape(N, nvec).T if layout == 1 else y.reshape(nvec, N)
        for v in range(nvec):
            yo = S.sigma(X[v]) - shift * X[v]
            assert np.linalg.norm(Y[v] - yo) <= 1e-12 * np.linalg.norm(yo)


def test_noalloc_repeated_calls_on_one_stream():
    """Several products in a row on one stream, alternating bases, each
    checked against sbd_sigma."""
    (W1, h1), (W2, h2) = system(400), system(250)
    for i in range(3):
        run_cases(W1, h1, 10 + i)
        run_cases(W2, h2, 20 + i)


def test_noalloc_rejects_workspace_above_limit():
    W, ham = system(None)  # 4e6 determinants
    N = W.ndet
    nvec = 8
    assert 2 * N * nvec * 8 > SCRATCH_BYTES
    x = torch.zeros(N * nvec, device=DEV, dtype=torch.float64)
    y = torch.zeros_like(x)
    rc = call_abi("sbd_sigma_noalloc", ham, x, y, nvec, 0, 0.0, 1)
    assert rc == -5  # SBD_ERR_NOMEM
    assert "static scratch" in sbd.last_error()
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(y)) == 0   # rejected before any device work
    # one vector of the same basis fits (2 * 4e6 * 8 bytes = 64 MB)
    xs = torch.randn(N, device=DEV, dtype=torch.float64)
    ya, yb = torch.empty_like(xs), torch.empty_like(xs)
    assert call_abi("sbd_sigma_noalloc", ham, xs, ya, 1, 0, 0.0, 0) == 0
    assert call_abi("sbd_sigma", ham, xs, yb, 1, 0, 0.0, 0) == 0
    torch.cuda.synchronize()
    assert torch.equal(ya, yb)


def test_noalloc_assembled_needs_no_scratch():
    """A handle holding the assembled H takes the CSR product, which uses no
    workspace; the result is still that of sbd_sigma."""
    W, ham = system(300)
    ham.assemble(3)
    N = W.ndet
    x = torch.randn(N * 8, device=DEV, dtype=torch.float64)
    ya, yb = torch.empty_like(x), torch.empty_like(x)
    assert call_abi("sbd_sigma_noalloc", ham, x, ya, 8, 0, 0.0, 1) == 0
    assert call_abi("sbd_sigma", ham, x, yb, 8, 0, 0.0, 1) == 0
    torch.cuda.synchronize()
    assert torch.equal(ya, yb)
