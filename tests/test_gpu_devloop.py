"""Device-driven Davidson iterations (opts.device_iterations): every decision of
an iteration taken on the device, iterations queued in batches between host
checks and replayed from one captured HIP graph.  Energies against the oracle
(1e-8 Ha plain, 1e-6 Ha mixed), eigenpairs certified by the oracle's sigma,
restarts exercised, and graph replays bitwise equal to eager launches of the
same device-driven iteration."""
import numpy as np
import pytest

import oracle
import workload as wl

torch = pytest.importorskip("torch")
sbd = pytest.importorskip("paper_2601_16637_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def system(name="sel16", nstr=200):
    W = wl.make_config(name, nstr=nstr)
    bas = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta)
    exc = sbd.Excitations(bas)
    ham = sbd.Hamiltonian(bas, exc, W.h, W.eri, W.e_core)
    return W, ham


@pytest.mark.parametrize("nroots,prec,max_space", [(1, 0, 20), (1, 1, 20), (1, 0, 5), (2, 0, 12), (2, 1, 12),
                                                    (4, 1, 16), (3, 0, 9)])
def test_device_iterations_energies_vs_oracle(nroots, prec, max_space):
    W, ham = system()
    S = oracle.OracleSystem.from_workload(W)
    ref = oracle.davidson(S.sigma, S.diag(), nroots, tol=1e-9, max_space=30)
    vec = torch.empty(nroots * W.ndet, device=DEV, dtype=torch.float64)
    tol = 1e-8 if prec == 0 else 1e-7
    e, rep, st = sbd.davidson(ham, nroots, vectors=vec, tol_residual=tol, sigma_prec=prec, max_space=max_space,
                              device_iterations=4, use_graph=1)
    assert st == 0 and rep["device_iterations"] > 0
    assert np.abs(e[:nroots] - np.array(ref.energies[:nroots])).max() <= (1e-8 if prec == 0 else 1e-6)
    V = vec.cpu().numpy().reshape(nroots, W.ndet)
    for r in range(nroots):  # every returned pair is an eigenpair of the oracle's H
        res = S.sigma(V[r]) - e[r] * V[r]
        assert np.linalg.norm(res) <= 2 * tol, (r, np.linalg.norm(res))
    if max_space <= 2 * nroots + 3:
        assert rep["restarts"] > 0


@pytest.mark.parametrize("nroots,prec", [(1, 0), (1, 1), (2, 1)])
def test_device_iterations_graph_equals_eager(nroots, prec):
    """The same device-driven iteration launched eagerly and replayed from the
    captured graph: bitwise equal energies, eigenvectors and iteration counts."""
    W, ham = system(nstr=300)
    out = []
    for g in (0, 1):
        vec = torch.empty(nroots * W.ndet, device=DEV, dtype=torch.float64)
        e, rep, st = sbd.davidson(ham, nroots, vectors=vec, tol_residual=1e-7, sigma_prec=prec, max_space=14,
                                  device_iterations=3, use_graph=g)
        assert st == 0
        out.append((e, rep, vec.cpu().numpy()))
    (e0, r0, v0), (e1, r1, v1) = out
    assert np.array_equal(e0, e1)
    assert r0["iterations"] == r1["iterations"] and r0["device_iterations"] == r1["device_iterations"]
    assert np.array_equal(v0, v1)


def test_device_iterations_fci8_dense_and_full_bitstring():
    """fci8 against dense eigh; the full-bitstring operator through the same
    device-driven iteration."""
    W, ham = system("fci8", None)
    S = oracle.OracleSystem.from_workload(W)
    ev = np.linalg.eigvalsh(S.dense_h())
    e, rep, st = sbd.davidson(ham, 2, tol_residual=1e-8, device_iterations=5, use_graph=1)
    assert st == 0 and np.abs(e[:2] - ev[:2]).max() <= 1e-8
    F = wl.make_full_config("full16", ndet=3000, nstr=100)
    fb = sbd.FullBasis(F.norb, F.n_alpha, F.n_beta, F.dets)
    fh = sbd.FullHamiltonian(fb, F.h, F.eri, F.e_core)
    FS = oracle.FullOracleSystem(F.norb, F.dets, F.h, F.eri, F.e_core)
    evf = np.linalg.eigvalsh(FS.dense_h())
    ef, repf, stf = sbd.full_davidson(fh, 1, tol_residual=1e-8, device_iterations=4, use_graph=1)
    assert stf == 0 and repf["device_iterations"] > 0 and abs(ef[0] - evf[0]) <= 1e-8


def test_device_iterations_fall_back_when_unsupported():
    """Several roots without block sigma, and bases above 2^21 determinants,
    keep the host-driven iteration."""
    W, ham = system()
    e, rep, st = sbd.davidson(ham, 2, tol_residual=1e-7, device_iterations=4, block_sigma=0)
    assert st == 0 and rep["device_iterations"] == 0
    W, ham = system(nstr=1500)
    assert W.ndet > 1 << 21
    e, rep, st = sbd.davidson(ham, 1, tol_residual=1e-6, device_iterations=4)
    assert st == 0 and rep["device_iterations"] == 0


@pytest.mark.parametrize("nroots,prec", [(1, 0), (2, 0), (1, 1)])
def test_device_iterations_count_like_host_driven(nroots, prec):
    """A device-driven solve takes the host-driven solve's path: the same
    energies (to the tolerance) in about the same number of iterations (the
    warm-started Ritz step rounds differently), each counted once across the
    hand-overs between device batches and host iterations."""
    W, ham = system(nstr=250)
    res = {}
    for dev in (0, 8):
        e, rep, st = sbd.davidson(ham, nroots, tol_residual=1e-8, sigma_prec=prec, max_space=16,
                                  device_iterations=dev, use_graph=1)
        assert st == 0
        res[dev] = (e[:nroots], rep)
    (eh, rh), (ed, rd) = res[0], res[8]
    assert rd["device_iterations"] > 0 and rh["device_iterations"] == 0
    assert np.abs(eh - ed).max() <= 1e-9
    assert abs(rd["iterations"] - rh["iterations"]) <= 2, (rh["iterations"], rd["iterations"])
    assert rd["device_iterations"] <= rd["iterations"]
