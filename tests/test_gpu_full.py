"""GPU parity of the full-bitstring path (Sec. II-F, Sec. III-F): determinant
lists that are not Cartesian products, through the C ABI, against the CPU
oracle's full-bitstring system.

Bars: sorted determinants and connection lists (ket index, electrons moved)
bit-exact; diagonal and FP64 sigma within 1e-12 relative; FP32 sigma within
its componentwise rounding bound; energies within 1e-8 Ha (FP64) and 1e-6 Ha
(mixed precision) of dense diagonalisation or the oracle's Davidson.
"""
import numpy as np
import pytest

import oracle
import workload as wl

torch = pytest.importorskip("torch")
sbd = pytest.importorskip("paper_2601_16637_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def random_dets(norb, na, nb, count, seed):
    """count distinct determinants drawn uniformly from all alpha x beta pairs."""
    A, B = wl.all_strings(norb, na), wl.all_strings(norb, nb)
    rng = np.random.default_rng(seed)
    pick = rng.choice(A.size * B.size, min(count, A.size * B.size), replace=False)
    return np.stack([A[pick // B.size], B[pick % B.size]], axis=1).astype(np.uint64)


def lists():
    """(name, norb, n_alpha, n_beta, dets, h, eri, e_core)"""
    out = []
    for name, nd, ns in (("full16", 20000, 400), ("full16", 3000, 100), ("full26", 20000, 1500)):
        W = wl.make_full_config(name, ndet=nd, nstr=ns)
        out.append((f"{name}-{nd}", W.norb, W.n_alpha, W.n_beta, W.dets, W.h, W.eri, W.e_core))
    for norb, na, nb, cnt, seed in ((8, 4, 4, 2000, 1), (7, 2, 4, 500, 2), (6, 0, 3, 20, 3), (10, 5, 3, 4000, 4)):
        h, eri, ec = wl.make_integrals(norb, 300 + seed)
        out.append((f"random{norb}-{na}-{nb}", norb, na, nb, random_dets(norb, na, nb, cnt, seed), h, eri, ec))
    return out


LISTS = lists()
IDS = [c[0] for c in LISTS]


def gpu_full(norb, na, nb, dets, h, eri, ec):
    B = sbd.FullBasis(norb, na, nb, dets)
    H = sbd.FullHamiltonian(B, h, eri, ec)
    return B, H


def run_sigma(H, x, prec=0, shift=0.0, nvec=1, layout=0):
    dt = torch.float64 if prec == 0 else torch.float32
    xd = torch.tensor(np.ascontiguousarray(x), device=DEV, dtype=dt)
    yd = torch.empty_like(xd)
    sbd.full_sigma(H, xd, yd, nvec=nvec, prec=prec, shift=shift, layout=layout)
    torch.cuda.synchronize()
    return yd.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("case", LISTS, ids=IDS)
def test_full_basis_and_connections_bitexact(case):
    name, norb, na, nb, dets, h, eri, ec = case
    rng = np.random.default_rng(5)
    shuffled = dets[rng.permutation(dets.shape[0])]
    with_dups = np.concatenate([shuffled, shuffled[: max(1, dets.shape[0] // 7)]])
    B = sbd.FullBasis(norb, na, nb, with_dups)
    S = oracle.FullOracleSystem(norb, dets, h, eri, ec)
    d, rp, J, deg = B.export()
    assert B.N == S.N
    assert np.array_equal(d, S.dets)
    assert np.array_equal(rp, S.row_ptr)
    assert np.array_equal(J, S.J)
    assert np.array_equal(deg, S.deg)
    assert B.nalpha == np.unique(S.dets[:, 0]).size


@pytest.mark.parametrize("ndet", [16384, 16385, 20480, 24577])
def test_full_scan_chunk_boundaries(ndet):
    """Lists whose lengths sit at the chunk boundaries of the multi-workgroup
    scan (4096 entries per workgroup, one workgroup up to 16384): the unique
    compaction (with duplicates given), the alpha groups and the connection
    row pointers stay bit-exact against the oracle."""
    W = wl.make_full_config("full16", ndet=ndet, nstr=400)
    rng = np.random.default_rng(ndet)
    given = np.concatenate([W.dets, W.dets[rng.integers(0, ndet, 4099)]])[rng.permutation(ndet + 4099)]
    B = sbd.FullBasis(W.norb, W.n_alpha, W.n_beta, given)
    S = oracle.FullOracleSystem(W.norb, W.dets, W.h, W.eri, W.e_core)
    d, rp, J, deg = B.export()
    assert B.N == S.N == ndet
    assert np.array_equal(d, S.dets) and np.array_equal(rp, S.row_ptr)
    assert np.array_equal(J, S.J) and np.array_equal(deg, S.deg)
    assert B.nalpha == np.unique(S.dets[:, 0]).size


@pytest.mark.parametrize("case", LISTS, ids=IDS)
def test_full_diag_and_sigma_fp64(case):
    name, norb, na, nb, dets, h, eri, ec = case
    B, H = gpu_full(norb, na, nb, dets, h, eri, ec)
    S = oracle.FullOracleSystem(norb, dets, h, eri, ec)
    dg = torch.empty(S.N, device=DEV, dtype=torch.float64)
    H.diag_into(dg)
    torch.cuda.synchronize()
    do = S.diag()
    assert np.abs(dg.cpu().numpy() - do).max() <= 1e-12 * np.abs(do).max()
    X = wl.random_vector(S.N, 11, nvec=3)
    for shift in (0.0, -123.5):
        Y = run_sigma(H, X, nvec=3, shift=shift)
        Yo = S.sigma(X) - shift * X
        for v in range(3):
            assert np.linalg.norm(Y[v] - Yo[v]) <= 1e-12 * np.linalg.norm(Yo[v])
    # interleaved layout [det][v] for 1, 2, 4, 8 vectors gives the same columns
    for nv in (1, 2, 4, 8):
        Xn = wl.random_vector(S.N, 20 + nv, nvec=nv)
        Yi = run_sigma(H, Xn.T.copy(), nvec=nv, layout=1).reshape(S.N, nv).T
        Yo = S.sigma(Xn).reshape(nv, S.N)
        for v in range(nv):
            assert np.linalg.norm(Yi[v] - Yo[v]) <= 1e-12 * np.linalg.norm(Yo[v])


@pytest.mark.parametrize("case", [c for c in LISTS if c[4].shape[0] <= 4000], ids=[c[0] for c in LISTS
                                                                                     if c[4].shape[0] <= 4000])
def test_full_sigma_fp32_rounding_bound(case):
    """FP32 sigma (elements rounded once, FP32 gathers and sums) on H - shift:
    |s32 - s64|_I <= 2 (z_I + 2) u32 (|H - shift| |x32|)_I with z_I the row's
    stored terms, against the oracle's dense H."""
    name, norb, na, nb, dets, h, eri, ec = case
    B, H = gpu_full(norb, na, nb, dets, h, eri, ec)
    S = oracle.FullOracleSystem(norb, dets, h, eri, ec)
    shift = float(S.diag().min())
    x = np.random.default_rng(3).standard_normal(S.N).astype(np.float32)
    y32 = run_sigma(H, x, prec=1, shift=shift)
    Hs = S.dense_h() - shift * np.eye(S.N)
    xd = x.astype(np.float64)
    z = np.diff(S.row_ptr) + 1
    bound = 2 * (z + 2) * 2.0 ** -24 * (np.abs(Hs) @ np.abs(xd))
    assert np.all(np.abs(y32 - Hs @ xd) <= bound)


def test_full_sigma_hermitian_and_deterministic():
    W = wl.make_full_config("full16", ndet=20000, nstr=400)
    B, H = gpu_full(W.norb, W.n_alpha, W.n_beta, W.dets, W.h, W.eri, W.e_core)
    x, y = wl.random_vector(B.N, 1)[0], wl.random_vector(B.N, 2)[0]
    Hx, Hy = run_sigma(H, x), run_sigma(H, y)
    assert abs(x @ Hy - Hx @ y) <= 1e-13 * abs(x @ Hy)
    assert np.array_equal(run_sigma(H, x), Hx)


def test_full_on_cartesian_product_equals_half_path():
    """The full-bitstring path on the complete alpha x beta product of two
    string sets reproduces the alpha x beta path: the same connections (every
    connected pair of the half path's count) and sigma."""
    W = wl.make_config("sel16", nstr=60)
    dets = np.array([(a, b) for a in W.alpha for b in W.beta], dtype=np.uint64)
    B, H = gpu_full(W.norb, W.n_alpha, W.n_beta, dets, W.h, W.eri, W.e_core)
    hb = sbd.Basis(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta)
    hx = sbd.Excitations(hb)
    hh = sbd.Hamiltonian(hb, hx, W.h, W.eri, W.e_core)
    assert B.N == hb.N
    assert B.N + B.nconn == oracle.OracleSystem.from_workload(W).nnz()
    x = wl.random_vector(B.N, 4)[0]
    xd = torch.tensor(x, device=DEV)
    yd = torch.empty_like(xd)
    sbd.sigma(hh, xd, yd)
    torch.cuda.synchronize()
    yh = yd.cpu().numpy()
    yf = run_sigma(H, x)
    assert np.linalg.norm(yf - yh) <= 1e-12 * np.linalg.norm(yh)


def test_full_edge_lists():
    """One determinant, two unconnected ones, empty alpha shell, norb = 64."""
    h, eri, ec = wl.make_integrals(6, 401)
    for dets in ([(0b000111, 0b000111)], [(0b000111, 0b000111), (0b111000, 0b111000)]):
        d = np.array(dets, dtype=np.uint64)
        B, H = gpu_full(6, 3, 3, d, h, eri, ec)
        S = oracle.FullOracleSystem(6, d, h, eri, ec)
        assert B.nconn == 0
        x = np.arange(1.0, B.N + 1)
        assert np.abs(run_sigma(H, x) - S.sigma(x)).max() <= 1e-12 * np.abs(S.sigma(x)).max()
    # norb = 64 with the top orbitals occupied (bit 63 of both words)
    norb = 64
    rng = np.random.default_rng(9)
    hi = [(1 << 63) | (1 << 62), (1 << 63) | (1 << 1), (1 << 62) | (1 << 1), 0b11, (1 << 63) | 1]
    dets = np.array([(a, b) for a in hi for b in hi[:3]], dtype=np.uint64)
    h64 = np.diag(np.sort(rng.uniform(-5, 1, norb)))
    L = rng.normal(0, 0.05, (3, norb, norb))
    L = (L + L.transpose(0, 2, 1)) / 2
    eri64 = np.einsum("kpq,krs->pqrs", L, L)
    B, H = gpu_full(norb, 2, 2, dets, h64, eri64, 1.0)
    S = oracle.FullOracleSystem(norb, dets, h64, eri64, 1.0)
    d, rp, J, deg = B.export()
    assert np.array_equal(d, S.dets) and np.array_equal(J, S.J) and np.array_equal(deg, S.deg)
    x = wl.random_vector(B.N, 5)[0]
    assert np.linalg.norm(run_sigma(H, x) - S.sigma(x)) <= 1e-12 * np.linalg.norm(S.sigma(x))


def test_full_rejects_bad_input():
    h, eri, ec = wl.make_integrals(6, 402)
    with pytest.raises(sbd.SBDError) as ei:
        sbd.FullBasis(6, 3, 3, np.array([(0b000111, 0b001111)], dtype=np.uint64))
    assert ei.value.status == -3
    with pytest.raises(sbd.SBDError) as ei:
        sbd.FullBasis(6, 3, 3, np.array([(0b1000000011, 0b000111)], dtype=np.uint64))
    assert ei.value.status == -3
    B, H = gpu_full(6, 3, 3, random_dets(6, 3, 3, 50, 1), h, eri, ec)
    x = torch.zeros(B.N, device=DEV, dtype=torch.float64)
    with pytest.raises(sbd.SBDError):
        sbd.full_sigma(H, x, x)
    with pytest.raises(sbd.SBDError):
        sbd.full_sigma(H, x, torch.empty_like(x), nvec=3, layout=1)


@pytest.mark.parametrize("case", [c for c in LISTS if c[4].shape[0] <= 4000], ids=[c[0] for c in LISTS
                                                                                     if c[4].shape[0] <= 4000])
def test_full_davidson_vs_dense(case):
    name, norb, na, nb, dets, h, eri, ec = case
    B, H = gpu_full(norb, na, nb, dets, h, eri, ec)
    S = oracle.FullOracleSystem(norb, dets, h, eri, ec)
    ev = np.linalg.eigvalsh(S.dense_h())
    k = min(2, S.N)
    e, rep, st = sbd.full_davidson(H, k, tol_residual=1e-8, max_space=24)
    assert st == 0
    assert np.abs(e[:k] - ev[:k]).max() <= 1e-8
    if S.N >= 10:
        e32, rep32, st32 = sbd.full_davidson(H, k, tol_residual=1e-7, sigma_prec=1, max_space=24)
        assert st32 == 0 and np.abs(e32[:k] - ev[:k]).max() <= 1e-6


def test_full_davidson_vs_oracle_and_vectors():
    """full16 with 20,000 determinants: plain and mixed energies and the
    eigenvector against the oracle's Davidson on the oracle's sigma; a block
    solve of 3 roots with interleaved sigma and graph replay."""
    W = wl.make_full_config("full16", ndet=20000, nstr=400)
    B, H = gpu_full(W.norb, W.n_alpha, W.n_beta, W.dets, W.h, W.eri, W.e_core)
    S = oracle.FullOracleSystem(W.norb, W.dets, W.h, W.eri, W.e_core)
    ref = oracle.davidson(S.sigma, S.diag(), 3, tol=1e-9, max_space=30)
    v = torch.empty(B.N, device=DEV, dtype=torch.float64)
    e, rep, st = sbd.full_davidson(H, 1, vectors=v, tol_residual=1e-8)
    assert st == 0 and abs(e[0] - ref.energies[0]) <= 1e-8
    u = v.cpu().numpy()
    r = S.sigma(u) - e[0] * u
    assert np.linalg.norm(r) <= 1e-7
    e32, _, st32 = sbd.full_davidson(H, 1, tol_residual=1e-7, sigma_prec=1)
    assert st32 == 0 and abs(e32[0] - ref.energies[0]) <= 1e-6
    eb, repb, stb = sbd.full_davidson(H, 3, tol_residual=1e-7, sigma_prec=1, use_graph=1, block_sigma=1,
                                      max_space=24)
    assert stb == 0 and np.abs(eb[:3] - np.array(ref.energies[:3])).max() <= 1e-6


@pytest.mark.parametrize("name", ["full16", "full26"])
def test_full_size_sampled_rows(name):
    """Full-size lists (1e6 and 4e6 determinants): connection counts and FP64
    sigma on sampled rows against the oracle, which finds each sampled row's
    neighbours by comparing it with every determinant of the list."""
    W = wl.make_full_config(name)
    B, H = gpu_full(W.norb, W.n_alpha, W.n_beta, W.dets, W.h, W.eri, W.e_core)
    S = oracle.FullOracleSystem(W.norb, W.dets, W.h, W.eri, W.e_core, connections=False)
    d, rp, J, deg = B.export()
    assert np.array_equal(d, S.dets)
    rng = np.random.default_rng(17)
    idx = np.unique(np.concatenate([rng.integers(0, B.N, 200), [0, B.N - 1]]))
    # connections of some sampled rows by a vectorised comparison with every determinant
    for i in idx[:: max(1, idx.size // 10)]:
        xa = S.dets[:, 0] ^ S.dets[i, 0]
        xb = S.dets[:, 1] ^ S.dets[i, 1]
        tot = np.zeros(B.N, dtype=np.int64)
        for wv in (xa, xb):
            b = wv.view(np.uint8).reshape(-1, 8)
            tot += np.unpackbits(b, axis=1).sum(axis=1, dtype=np.int64)
        nb = np.flatnonzero((tot == 2) | (tot == 4))
        assert np.array_equal(J[rp[i]:rp[i + 1]], nb)
        assert np.array_equal(deg[rp[i]:rp[i + 1]], tot[nb] // 2)
    x = wl.random_vector(B.N, 6)[0]
    y = run_sigma(H, x)
    yo = S.sigma_rows(x, idx)
    assert np.abs(y[idx] - yo).max() <= 1e-12 * np.abs(yo).max()


@pytest.mark.parametrize("seed", range(9200, 9224))
def test_full_random_shapes(seed):
    """Random small determinant lists (norb 2-12, any electron counts, from one
    determinant up to a few thousand, duplicates given): bit-exact sorted lists
    and connections, FP64 sigma elementwise within 1e-12 of the oracle's
    (relative to the row's magnitude sum) and the lowest energy against the
    oracle's dense H."""
    rng = np.random.default_rng(seed)
    norb = int(rng.integers(2, 13))
    na, nb = int(rng.integers(0, norb + 1)), int(rng.integers(0, norb + 1))
    total = len(wl.all_strings(norb, na)) * len(wl.all_strings(norb, nb))
    count = int(rng.integers(1, min(total, 3000) + 1))
    dets = random_dets(norb, na, nb, count, seed)
    h, eri, ec = wl.make_integrals(norb, seed + 1)
    given = np.concatenate([dets, dets[: max(1, count // 5)]])[rng.permutation(count + max(1, count // 5))]
    B, H = gpu_full(norb, na, nb, given, h, eri, ec)
    S = oracle.FullOracleSystem(norb, dets, h, eri, ec)
    d, rp, J, deg = B.export()
    assert np.array_equal(d, S.dets) and np.array_equal(rp, S.row_ptr)
    assert np.array_equal(J, S.J) and np.array_equal(deg, S.deg)
    Hd = S.dense_h()
    x = wl.random_vector(S.N, seed + 2)[0]
    y = run_sigma(H, x)
    mag = np.abs(Hd) @ np.abs(x)
    assert np.all(np.abs(y - Hd @ x) <= 1e-12 * mag)
    e, rep, st = sbd.full_davidson(H, 1, tol_residual=1e-8)
    assert st == 0
    assert abs(e[0] - np.linalg.eigvalsh(Hd)[0]) <= 1e-8


@pytest.mark.parametrize("case", [c for c in LISTS if c[4].shape[0] <= 20000], ids=[c[0] for c in LISTS
                                                                                      if c[4].shape[0] <= 20000])
def test_full_assembled_bitwise_matrix_free(case):
    """The explicit realization (every connection's element kept, Sec. II-A)
    gives bitwise the matrix-free product in both precisions, one vector and
    2, 4, 8 interleaved vectors, and the same Davidson energies; releasing it
    returns to the matrix-free product."""
    name, norb, na, nb, dets, h, eri, ec = case
    B, H = gpu_full(norb, na, nb, dets, h, eri, ec)
    N = B.N
    X = wl.random_vector(N, 31, nvec=8)
    shift = -151.25
    free = {}
    for prec in (0, 1):
        free[(prec, 1)] = run_sigma(H, X[0], prec=prec, shift=shift)
        for nv in (2, 4, 8):
            free[(prec, nv)] = run_sigma(H, X[:nv].T.copy(), prec=prec, shift=shift, nvec=nv, layout=1)
    e_free, _, _ = sbd.full_davidson(H, 2, tol_residual=1e-8, max_space=16)
    H.assemble(3)
    assert H.assembled() == 3
    for prec in (0, 1):
        assert np.array_equal(run_sigma(H, X[0], prec=prec, shift=shift), free[(prec, 1)])
        for nv in (2, 4, 8):
            y = run_sigma(H, X[:nv].T.copy(), prec=prec, shift=shift, nvec=nv, layout=1)
            assert np.array_equal(y, free[(prec, nv)]), (prec, nv)
    e_asm, _, st = sbd.full_davidson(H, 2, tol_residual=1e-8, max_space=16)
    assert st == 0 and np.array_equal(e_asm[:2], e_free[:2])
    H.release_assembled()
    assert H.assembled() == 0
    assert np.array_equal(run_sigma(H, X[0], shift=shift), free[(0, 1)])


def test_full_assemble_limits_and_errors():
    """A byte limit below the elements' size fails with SBD_ERR_NOMEM and
    leaves the Hamiltonian matrix-free; FP32 alone leaves FP64 matrix-free;
    a Hamiltonian of another list is refused."""
    W = wl.make_full_config("full16", ndet=3000, nstr=100)
    B, H = gpu_full(W.norb, W.n_alpha, W.n_beta, W.dets, W.h, W.eri, W.e_core)
    nconn = B.export()[1][-1]
    with pytest.raises(sbd.SBDError) as ei:
        H.assemble(1, max_bytes=8 * nconn - 1)
    assert ei.value.status == -5 and H.assembled() == 0
    H.assemble(1, max_bytes=8 * nconn)
    assert H.assembled() == 1
    H.assemble(2)
    assert H.assembled() == 2
    x = wl.random_vector(B.N, 3)[0]
    S = oracle.FullOracleSystem(W.norb, W.dets, W.h, W.eri, W.e_core)
    assert np.linalg.norm(run_sigma(H, x) - S.sigma(x)) <= 1e-12 * np.linalg.norm(S.sigma(x))
    with pytest.raises(sbd.SBDError):
        H.assemble(4)
    W2 = wl.make_full_config("full16", ndet=500, nstr=100)
    B2, _ = gpu_full(W2.norb, W2.n_alpha, W2.n_beta, W2.dets, W2.h, W2.eri, W2.e_core)
    with pytest.raises(sbd.SBDError) as ei:
        check_other = sbd.load().sbd_full_assemble(H._h, B2._h, 1, 0, None)
        sbd._native.check(check_other)
    assert ei.value.status == -8
