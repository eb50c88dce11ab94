"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what it pins.  The paper prints no energies and no worked
example, so the pins are the operator definition of Eq. 3 applied term by
term (tier 0), closed forms, invariants, textbook values and library
eigensolvers.
"""
import json
import math
import os
from itertools import combinations

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import workload as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _system(norb, na_el, nb_el, seed, nsub_a=None, nsub_b=None, sub_seed=7):
    h, eri, ec = wl.make_integrals(norb, seed)
    A = wl.all_strings(norb, na_el)
    B = wl.all_strings(norb, nb_el)
    rng = np.random.default_rng(sub_seed)
    if nsub_a is not None and nsub_a < A.size:
        A = np.sort(rng.choice(A, nsub_a, replace=False))
    if nsub_b is not None and nsub_b < B.size:
        B = np.sort(rng.choice(B, nsub_b, replace=False))
    return oracle.OracleSystem(norb, A, B, h, eri, ec)


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("norb,na,nb,sa,sb", [
    (4, 2, 2, None, None), (5, 3, 2, None, None), (5, 2, 1, None, None),
    (4, 0, 2, None, None), (3, 3, 1, None, None), (6, 3, 2, 12, 9), (6, 2, 2, 10, 11),
])
def test_p1_tier0_operator_equals_slater_condon(norb, na, nb, sa, sb):
    """Pin: generic Slater-Condon H (tier 1) equals Eq. 3 applied term by term."""
    S = _system(norb, na, nb, seed=norb * 10 + na, nsub_a=sa, nsub_b=sb)
    H1 = S.dense_h()
    H0 = oracle.tier0_dense_h(norb, S.alpha, S.beta, S.h, S.eri, S.e_core)
    scale = max(1.0, np.abs(H0).max())
    assert np.abs(H1 - H0).max() <= 1e-13 * scale
    assert np.abs(H1 - H1.T).max() == 0.0 or np.abs(H1 - H1.T).max() <= 1e-14 * scale


def test_p1_sigma_equals_dense_on_subsets():
    """Pin: sigma over the table neighbourhood equals brute-force dense H x."""
    S = _system(6, 3, 3, seed=5, nsub_a=14, nsub_b=17)
    Hd = S.dense_h()
    X = wl.random_vector(S.N, 3, nvec=3)
    Y = S.sigma(X)
    assert np.abs(Y - X @ Hd.T).max() <= 1e-13 * np.abs(Hd).max()
    idx = np.array([0, 5, S.N - 1, S.N // 2])
    assert np.allclose(S.sigma_at(X[1], idx), (Hd @ X[1])[idx], rtol=0, atol=1e-12)


# ---------------------------------------------------------------- P2
def test_p2_no_two_electron_spectrum_closed_form():
    """Pin: with (pq|rs) = 0, full-CI eigenvalues are sums of eig(h)."""
    norb, na, nb = 5, 2, 2
    h, _, ec = wl.make_integrals(norb, 3)
    eri = np.zeros((norb,) * 4)
    S = oracle.OracleSystem(norb, wl.all_strings(norb, na), wl.all_strings(norb, nb), h, eri, ec)
    ev = np.linalg.eigvalsh(S.dense_h())
    eps = np.linalg.eigvalsh(h)
    sums_a = [sum(eps[list(c)]) for c in combinations(range(norb), na)]
    sums_b = [sum(eps[list(c)]) for c in combinations(range(norb), nb)]
    closed = np.sort([ec + x + y for x in sums_a for y in sums_b])
    assert np.allclose(np.sort(ev), closed, rtol=0, atol=1e-11)


# ---------------------------------------------------------------- P3
def _p3_integrals(norb, g, seed=11):
    rng = np.random.default_rng(seed)
    h = np.diag(np.sort(rng.uniform(-3, 1, norb)))
    eri = np.zeros((norb,) * 4)
    eri[0, 0, 1, 1] = eri[1, 1, 0, 0] = g
    return h, eri


def test_p3_convention_pin_diagonal_hamiltonian():
    """Pin of the chemists' reading: only (00|11) nonzero gives g n0 n1, a diagonal H."""
    norb, g = 4, 0.37
    h, eri = _p3_integrals(norb, g)
    A, B = wl.all_strings(norb, 2), wl.all_strings(norb, 1)
    S = oracle.OracleSystem(norb, A, B, h, eri, 1.5)
    Hd = S.dense_h()
    off = Hd - np.diag(np.diag(Hd))
    assert np.abs(off).max() == 0.0
    for ia, a in enumerate(S.alpha):
        for ib, b in enumerate(S.beta):
            n = [((int(a) >> p) & 1) + ((int(b) >> p) & 1) for p in range(norb)]
            e = 1.5 + sum(h[p, p] * n[p] for p in range(norb)) + g * n[0] * n[1]
            assert abs(Hd[ia * S.nb + ib, ia * S.nb + ib] - e) < 1e-13


def test_p3_physicists_order_would_fail():
    """Power of the P3 pin: the operator order printed in Eq. 3 taken literally with
    chemists' integrals (a+_p a+_q a_s a_r) gives a non-diagonal H, so the pin
    discriminates between the two readings.  The mistake is planted in a copy
    of tier 0 on the CPU."""
    norb, g = 4, 0.37
    h, eri = _p3_integrals(norb, g)
    # relabel: literal order a+_p a+_q a_s a_r with (pq|rs) equals the chemists'
    # operator with integral array E[p,r,q,s] = eri[p,q,r,s]
    eri_lit = eri.transpose(0, 2, 1, 3).copy()
    A, B = wl.all_strings(norb, 2), wl.all_strings(norb, 1)
    H0 = oracle.tier0_dense_h(norb, A, B, h, eri_lit, 1.5)
    off = H0 - np.diag(np.diag(H0))
    assert np.abs(off).max() > 0.1


# ---------------------------------------------------------------- P4
def test_p4_aufbau_diagonal_is_closed_shell_hf():
    """Pin: Aufbau x Aufbau diagonal = E_core + 2 sum h_ii + sum_ij [2(ii|jj) - (ij|ji)]."""
    norb, m = 7, 3
    h, eri, ec = wl.make_integrals(norb, 21)
    A = wl.all_strings(norb, m)
    S = oracle.OracleSystem(norb, A, A, h, eri, ec)
    occ = range(m)
    e = ec + 2 * sum(h[i, i] for i in occ) + sum(
        2 * eri[i, i, j, j] - eri[i, j, j, i] for i in occ for j in occ)
    aufbau = (1 << m) - 1
    ia = int(np.searchsorted(S.alpha, np.uint64(aufbau)))
    assert abs(S.diag()[ia * S.nb + ia] - e) < 1e-12 * max(1, abs(e))


# ---------------------------------------------------------------- P5
def test_p5_constant_shift_any_basis():
    """Pin: h = mu I, (pq|rs) = lam d_pq d_rs gives (E_core + mu Ne + lam Ne(Ne-1)/2) I."""
    norb, na, nb = 10, 4, 3
    mu, lam = -0.8, 0.45
    h = mu * np.eye(norb)
    eri = np.zeros((norb,) * 4)
    for p in range(norb):
        for r in range(norb):
            eri[p, p, r, r] = lam
    A = wl.sample_strings(norb, na, 60, 1)
    B = wl.sample_strings(norb, nb, 50, 2)
    S = oracle.OracleSystem(norb, A, B, h, eri, 2.0)
    ne = na + nb
    c = 2.0 + mu * ne + lam * ne * (ne - 1) / 2
    x = wl.random_vector(S.N, 4)[0]
    assert np.abs(S.sigma(x) - c * x).max() < 1e-13


def test_p5_shift_moves_every_eigenvalue():
    norb, na, nb = 5, 2, 2
    h, eri, ec = wl.make_integrals(norb, 8)
    mu, lam = 0.3, 0.2
    eri2 = eri.copy()
    for p in range(norb):
        for r in range(norb):
            eri2[p, p, r, r] += lam
    S1 = oracle.OracleSystem(norb, wl.all_strings(norb, na), wl.all_strings(norb, nb), h, eri, ec)
    S2 = oracle.OracleSystem(norb, wl.all_strings(norb, na), wl.all_strings(norb, nb),
                             h + mu * np.eye(norb), eri2, ec)
    ne = na + nb
    d = mu * ne + lam * ne * (ne - 1) / 2
    assert np.allclose(np.linalg.eigvalsh(S2.dense_h()), np.linalg.eigvalsh(S1.dense_h()) + d,
                       rtol=0, atol=1e-11)


# ---------------------------------------------------------------- P6
def test_p6_trace_closed_form_full_ci():
    """Pin: sum of the diagonal over full CI equals its combinatorial closed form
    and the sum of the eigenvalues."""
    n, na, nb = 6, 3, 2
    h, eri, ec = wl.make_integrals(n, 31)
    S = oracle.OracleSystem(n, wl.all_strings(n, na), wl.all_strings(n, nb), h, eri, ec)
    C = math.comb
    Na, Nb = C(n, na), C(n, nb)
    trh = np.trace(h)
    Kp = sum(eri[p, p, q, q] - eri[p, q, q, p] for p in range(n) for q in range(p + 1, n))
    J = sum(eri[p, p, q, q] for p in range(n) for q in range(n))
    closed = (Na * Nb * ec + Nb * C(n - 1, na - 1) * trh + Na * C(n - 1, nb - 1) * trh
              + Nb * C(n - 2, na - 2) * Kp + Na * C(n - 2, nb - 2) * Kp
              + C(n - 1, na - 1) * C(n - 1, nb - 1) * J)
    tr = S.diag().sum()
    assert abs(tr - closed) < 1e-10 * abs(closed)
    assert abs(np.linalg.eigvalsh(S.dense_h()).sum() - closed) < 1e-9 * abs(closed)


# ---------------------------------------------------------------- P7
def test_p7_hermiticity_sampled_basis():
    """Invariant: <x, H y> = <H x, y> on a sampled basis."""
    W = wl.make_config("sel16", nstr=150)
    S = oracle.OracleSystem.from_workload(W)
    x, y = wl.random_vector(S.N, 11, nvec=2)
    a = x @ S.sigma(y)
    b = S.sigma(x) @ y
    assert abs(a - b) <= 1e-13 * np.linalg.norm(S.sigma(x))


# ---------------------------------------------------------------- P8
def test_p8_alpha_beta_swap():
    """Invariant: swapping the alpha and beta string sets (n_alpha = n_beta)
    transposes sigma and leaves the spectrum unchanged."""
    W = wl.make_config("sel16", nstr=40)
    B = wl.sample_strings(16, 8, 55, 99)
    S1 = oracle.OracleSystem(16, W.alpha, B, W.h, W.eri, W.e_core)
    S2 = oracle.OracleSystem(16, B, W.alpha, W.h, W.eri, W.e_core)
    Cm = wl.random_vector(S1.N, 5)[0].reshape(S1.na, S1.nb)
    y1 = S1.sigma(Cm.reshape(-1)).reshape(S1.na, S1.nb)
    y2 = S2.sigma(Cm.T.reshape(-1)).reshape(S2.na, S2.nb)
    assert np.abs(y1.T - y2).max() < 1e-12 * np.abs(y1).max()


# ---------------------------------------------------------------- P9
def test_p9_variational_and_monotone_ritz():
    """Invariants: E(subset) >= E(full); E0 <= min H_ii; Ritz values never rise."""
    W = wl.make_config("fci8")
    S = oracle.OracleSystem.from_workload(W)
    e_full = np.linalg.eigvalsh(S.dense_h())[0]
    sub = oracle.OracleSystem(8, W.alpha[::2], W.beta[1::2], W.h, W.eri, W.e_core)
    e_sub = np.linalg.eigvalsh(sub.dense_h())[0]
    assert e_sub >= e_full - 1e-12
    assert e_full <= S.diag().min()
    r = oracle.davidson(S.sigma, S.diag(), 1, tol=1e-9, max_space=8)
    th = [hh["theta"][0] for hh in r.history]
    assert all(b <= a + 1e-12 for a, b in zip(th, th[1:]))


# ---------------------------------------------------------------- P10
def _apply_string(s, ops):
    """Apply ('a', p) / ('c', p) right to left on a one-spin string; returns (sign, s)."""
    sign = 1
    for kind, p in ops:
        occ = (s >> p) & 1
        if (kind == "a" and not occ) or (kind == "c" and occ):
            return 0, s
        if bin(s & ((1 << p) - 1)).count("1") % 2:
            sign = -sign
        s = s ^ (1 << p)
    return sign, s


@pytest.mark.parametrize("norb,n", [(8, 4), (7, 2), (6, 5), (5, 0), (9, 3)])
def test_p10_table_lengths_and_signs_full_space(norb, n):
    """Pin: full-space row lengths n(norb-n) and C(n,2)C(norb-n,2); every entry's
    sign equals the phase of the operator string applied in Python."""
    A = wl.all_strings(norb, n)
    t1 = oracle.exc_table(A, norb, 1)
    t2 = oracle.exc_table(A, norb, 2)
    assert np.all(np.diff(t1.row_ptr) == n * (norb - n))
    assert np.all(np.diff(t2.row_ptr) == math.comb(n, 2) * math.comb(norb - n, 2))
    for I in range(A.size):
        for e in range(t1.row_ptr[I], t1.row_ptr[I + 1]):
            i, a = (int(v) for v in t1.orbs[e])
            sg, res = _apply_string(int(A[t1.J[e]]), [("a", i), ("c", a)])
            assert res == int(A[I]) and sg == t1.sign[e]
        Js = t2.J[t2.row_ptr[I]:t2.row_ptr[I + 1]]
        assert np.all(np.diff(Js) > 0)
        for e in range(t2.row_ptr[I], t2.row_ptr[I + 1]):
            i, j, a, b = (int(v) for v in t2.orbs[e])
            assert i < j and a < b
            sg, res = _apply_string(int(A[t2.J[e]]), [("a", i), ("a", j), ("c", b), ("c", a)])
            assert res == int(A[I]) and sg == t2.sign[e]


def test_sort_unique_matches_numpy():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 1 << 62, 500, dtype=np.uint64)
    x = np.concatenate([x, x[:100], np.array([0, (1 << 64) - 1], dtype=np.uint64)])
    assert np.array_equal(oracle.sort_unique(x), np.unique(x))


# ---------------------------------------------------------------- P11
def test_p11_davidson_vs_dense_several_roots():
    """Library pin: Davidson energies equal numpy.linalg.eigh of the dense H."""
    W = wl.make_config("fci8")
    S = oracle.OracleSystem.from_workload(W)
    ev = np.linalg.eigvalsh(S.dense_h())[:4]
    r = oracle.davidson(S.sigma, S.diag(), 4, tol=1e-8, max_space=24)
    assert r.converged
    assert np.abs(r.energies - ev).max() < 1e-9


def test_p11_davidson_vs_arpack():
    """Library pin: Davidson on a sampled basis equals ARPACK Lanczos (eigsh)."""
    W = wl.make_config("sel16", nstr=120)
    S = oracle.OracleSystem.from_workload(W)
    op = spla.LinearOperator((S.N, S.N), matvec=lambda v: S.sigma(np.asarray(v).reshape(-1)),
                             dtype=np.float64)
    ev = np.sort(spla.eigsh(op, k=2, which="SA", tol=1e-12)[0])
    r = oracle.davidson(S.sigma, S.diag(), 2, tol=1e-7, max_space=20)
    assert r.converged
    assert np.abs(r.energies - ev).max() < 1e-8


# ---------------------------------------------------------------- golden
def test_golden_h2_sto3g():
    g = json.load(open(os.path.join(GOLD, "h2_sto3g.json")))
    n = g["norb"]
    h = np.array(g["h"])
    eri = np.zeros((n,) * 4)
    for p, q, r, s, v in g["eri_nonzero"]:
        p, q, r, s = int(p), int(q), int(r), int(s)
        for a, b, c, d in [(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                           (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)]:
            eri[a, b, c, d] = v
    S = oracle.OracleSystem(n, wl.all_strings(n, 1), wl.all_strings(n, 1), h, eri, g["e_nuc"])
    ev = np.linalg.eigvalsh(S.dense_h())
    assert abs(ev[0] - g["e_fci"]) < g["tol"]
    aufbau_diag = S.diag()[0]
    assert abs(aufbau_diag - g["e_hf"]) < g["tol"]


def test_golden_hubbard_dimer():
    g = json.load(open(os.path.join(GOLD, "hubbard_dimer.json")))
    for t, U in g["cases"]:
        h = np.array([[0.0, -t], [-t, 0.0]])
        eri = np.zeros((2,) * 4)
        eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
        S = oracle.OracleSystem(2, wl.all_strings(2, 1), wl.all_strings(2, 1), h, eri, 0.0)
        e0 = np.linalg.eigvalsh(S.dense_h())[0]
        assert abs(e0 - (U - math.sqrt(U * U + 16 * t * t)) / 2) < 1e-12
        r = oracle.davidson(S.sigma, S.diag(), 1, tol=1e-10)
        assert abs(r.energies[0] - e0) < 1e-10


def test_damped_inverse_eq7():
    d = np.array([-2.0, -1e-12, 0.0, 1e-12, 3.0])
    out = oracle.damped_inverse(d, 0.0, 1e-8)
    assert np.allclose(out, [-0.5, -1e8, 1e8, 1e8, 1 / 3.0])


# ------------------------------------------------------------------ basis transfer (warm starts)
def _map_brute(af, bf, at, bt, x):
    """Determinant by determinant: look the (alpha, beta) pair up in the old basis."""
    pos = {(int(a), int(b)): i * len(bf) + j for i, a in enumerate(af) for j, b in enumerate(bf)}
    return np.array([x[pos[(int(a), int(b))]] if (int(a), int(b)) in pos else 0.0 for a in at for b in bt])


def test_map_vector_brute_force_tiny():
    """Mapping between overlapping, nested and disjoint string sets equals the
    determinant-by-determinant lookup."""
    full = wl.all_strings(7, 3)
    rng = np.random.default_rng(5)
    for t in range(6):
        af = np.sort(rng.choice(full, 9, replace=False))
        bf = np.sort(rng.choice(full, 7, replace=False))
        at = np.sort(rng.choice(full, 11, replace=False)) if t % 2 else np.sort(np.union1d(af, full[:4]))
        bt = np.sort(rng.choice(full, 5, replace=False))
        x = rng.standard_normal(af.size * bf.size)
        assert np.array_equal(oracle.map_vector(af, bf, at, bt, x), _map_brute(af, bf, at, bt, x))
    # several vectors at once, and an empty overlap
    X = rng.standard_normal((3, af.size * bf.size))
    Y = oracle.map_vector(af, bf, at, bt, X)
    for v in range(3):
        assert np.array_equal(Y[v], _map_brute(af, bf, at, bt, X[v]))
    lo, hi = full[:10], full[10:20]
    assert not oracle.map_vector(lo, lo, hi, hi, np.ones(100)).any()


def test_map_vector_embedding_keeps_rayleigh_quotient():
    """Carried into a larger basis, an eigenvector of the smaller one keeps its
    norm and its energy (the larger H restricted to the old determinants is the
    old H), and carried back it is unchanged: the transfer respects the
    alpha-major determinant order the sigma uses."""
    norb, n = 8, 3
    h, eri, ec = wl.make_integrals(norb, 91)
    big_a = wl.sample_strings(norb, n, 40, 92)
    big_b = wl.sample_strings(norb, n, 36, 93)
    rng = np.random.default_rng(94)
    sa = np.sort(rng.choice(big_a, 25, replace=False))
    sb = np.sort(rng.choice(big_b, 20, replace=False))
    small = oracle.OracleSystem(norb, sa, sb, h, eri, ec)
    e, vecs = oracle.dense_lowest(small.dense_h(), 1)
    x = vecs[0]
    big = oracle.OracleSystem(norb, big_a, big_b, h, eri, ec)
    y = oracle.map_vector(sa, sb, big_a, big_b, x)
    assert abs(np.linalg.norm(y) - 1.0) < 1e-12
    assert abs(y @ big.sigma(y) - e[0]) < 1e-10 * abs(e[0])
    assert np.array_equal(oracle.map_vector(big_a, big_b, sa, sb, y), x)


# ---------------------------------------------------------------- connected-pair count
def _count_connected_brute(S):
    """Pairs (I, J) of determinants differing by at most two electrons, counted
    over every pair of the basis (no tables): the stored terms of H including
    the diagonal."""
    A = S.alpha.astype(np.uint64)
    B = S.beta.astype(np.uint64)

    def popc(v):
        v = v.copy()
        c = np.zeros(v.shape, dtype=np.int64)
        while np.any(v):
            c += (v & np.uint64(1)).astype(np.int64)
            v >>= np.uint64(1)
        return c

    da = popc(A[:, None] ^ A[None, :]) // 2   # electrons moved within alpha
    db = popc(B[:, None] ^ B[None, :]) // 2
    # a determinant pair (ia,ib)-(ja,jb) is connected iff da + db <= 2
    hist_a = np.bincount(da.ravel(), minlength=3)[:3]
    hist_b = np.bincount(db.ravel(), minlength=3)[:3]
    return int(sum(hist_a[i] * hist_b[j] for i in range(3) for j in range(3) if i + j <= 2))


@pytest.mark.parametrize("norb,na,nb,sa,sb", [
    (6, 3, 3, None, None), (7, 3, 2, None, None), (6, 0, 2, None, None), (5, 5, 2, None, None),
    (8, 4, 4, 30, 25), (10, 3, 5, 40, 60), (6, 6, 0, None, None), (9, 1, 4, None, 50),
])
def test_nnz_equals_brute_force_pair_count(norb, na, nb, sa, sb):
    """OracleSystem.nnz (N + nb (P1a + P2a) + na (P1b + P2b) + P1a P1b from the
    tables) equals a count over all determinant pairs of those differing by at
    most two electrons, with unequal electron counts, empty and full shells."""
    S = _system(norb, na, nb, 5, sa, sb)
    assert S.nnz() == _count_connected_brute(S)


def test_nnz_equals_dense_structure_and_row_terms():
    """On a small basis the count equals the number of structurally connected
    entries of the dense H (pairs within two electrons, whatever their value),
    and row_terms gives the per-row counts."""
    S = _system(6, 3, 2, 9, 14, 12)
    A, B = S.alpha, S.beta
    z = np.zeros(S.N, dtype=np.int64)
    for I in range(S.N):
        ia, ib = divmod(I, S.nb)
        for J in range(S.N):
            ja, jb = divmod(J, S.nb)
            d = (bin(int(A[ia]) ^ int(A[ja])).count("1") + bin(int(B[ib]) ^ int(B[jb])).count("1")) // 2
            z[I] += d <= 2
    assert z.sum() == S.nnz()
    assert np.array_equal(S.row_terms(np.arange(S.N)), z)


# ---------------------------------------------------------------- componentwise bound
@pytest.mark.parametrize("norb,na,nb,sa,sb,shift", [
    (6, 3, 3, None, None, 0.0), (7, 3, 2, 20, None, -3.5), (6, 2, 2, 10, 11, 12.0),
])
def test_sigma_abs_equals_dense_magnitudes(norb, na, nb, sa, sb, shift):
    """(|H - shift I| |x|)_I from the table walk equals the same product formed
    with the brute-force dense H (all pairs, no tables), at every row."""
    S = _system(norb, na, nb, 17, sa, sb)
    x = np.random.default_rng(3).standard_normal(S.N)
    Hd = S.dense_h()
    ref = np.abs(Hd - shift * np.eye(S.N)) @ np.abs(x)
    got = S.sigma_abs_at(x, np.arange(S.N), shift)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_sigma_abs_bounds_rounding_of_float32_product():
    """The bound holds for a plain FP32 evaluation of (H - shift) x32 (numpy,
    rows summed in FP32): |y32 - y64|_I <= 2 (z_I + 2) u32 (|H - shift||x32|)_I."""
    S = _system(7, 3, 3, 21)
    shift = float(S.diag().min())
    x = np.random.default_rng(4).standard_normal(S.N).astype(np.float32).astype(np.float64)
    Hs = S.dense_h() - shift * np.eye(S.N)
    y64 = Hs @ x
    y32 = (Hs.astype(np.float32) @ x.astype(np.float32)).astype(np.float64)
    bound = 2 * (S.row_terms(np.arange(S.N)) + 2) * 2.0 ** -24 * S.sigma_abs_at(x, np.arange(S.N), shift)
    assert np.all(np.abs(y32 - y64) <= bound)


# ---------------------------------------------------------------- full-bitstring bases
def _random_dets(norb, na, nb, count, seed):
    A, B = wl.all_strings(norb, na), wl.all_strings(norb, nb)
    pairs = np.array([(a, b) for a in A for b in B], dtype=np.uint64)
    rng = np.random.default_rng(seed)
    pick = rng.choice(pairs.shape[0], min(count, pairs.shape[0]), replace=False)
    return pairs[pick]


@pytest.mark.parametrize("norb,na,nb,count,seed", [
    (4, 2, 2, 20, 1), (5, 3, 2, 40, 2), (5, 1, 2, 25, 3), (6, 3, 3, 60, 4), (4, 0, 3, 4, 5), (6, 2, 4, 90, 6),
])
def test_full_tier0_operator_equals_slater_condon(norb, na, nb, count, seed):
    """Full-bitstring oracle on determinant lists that are not Cartesian
    products: dense H from the generic Slater-Condon rules equals the operator
    terms of Eq. 3 applied to each determinant (tier 0), elementwise."""
    h, eri, ec = wl.make_integrals(norb, 60 + seed)
    S = oracle.FullOracleSystem(norb, _random_dets(norb, na, nb, count, seed), h, eri, ec)
    H0 = oracle.tier0_dense_h_dets(norb, [tuple(map(int, d)) for d in S.dets], h, eri, ec)
    assert np.abs(S.dense_h() - H0).max() <= 1e-13 * max(1.0, np.abs(H0).max())


@pytest.mark.parametrize("norb,na,nb,count,seed", [(6, 3, 3, 200, 7), (7, 2, 3, 300, 8), (8, 4, 4, 400, 9)])
def test_full_connections_and_sigma_brute_force(norb, na, nb, count, seed):
    """Connection lists equal a pairwise comparison written out in Python
    (rows sorted by J, degree = electrons moved), and the table-driven sigma
    equals the dense H (all pairs, no lists) applied to a vector."""
    h, eri, ec = wl.make_integrals(norb, 70 + seed)
    S = oracle.FullOracleSystem(norb, _random_dets(norb, na, nb, count, seed), h, eri, ec)
    D = [(int(a), int(b)) for a, b in S.dets]
    for i in range(S.N):
        row = [(j, (bin(D[i][0] ^ D[j][0]).count("1") + bin(D[i][1] ^ D[j][1]).count("1")) // 2)
               for j in range(S.N) if j != i]
        row = [(j, k) for j, k in row if k in (1, 2)]
        lo, hi = S.row_ptr[i], S.row_ptr[i + 1]
        assert [j for j, _ in row] == S.J[lo:hi].tolist()
        assert [k for _, k in row] == S.deg[lo:hi].tolist()
    x = np.random.default_rng(seed).standard_normal((2, S.N))
    assert np.abs(S.sigma(x) - x @ S.dense_h().T).max() <= 1e-12 * np.abs(S.dense_h()).max()
    assert np.array_equal(S.diag(), np.diag(S.dense_h()))


def test_full_on_cartesian_product_equals_half_bitstring():
    """On the Cartesian product of alpha and beta string sets, sorted by alpha
    then beta, the full-bitstring oracle reproduces the alpha x beta oracle:
    the same determinant order (ia * nb + ib), diagonal and sigma."""
    W = wl.make_config("sel16", nstr=40)
    half = oracle.OracleSystem.from_workload(W)
    dets = np.array([(a, b) for a in W.alpha for b in W.beta], dtype=np.uint64)
    full = oracle.FullOracleSystem(W.norb, dets[::-1], W.h, W.eri, W.e_core)
    assert np.array_equal(full.dets, dets)
    assert full.nnz() == half.nnz()
    x = wl.random_vector(full.N, 3)[0]
    assert np.abs(full.sigma(x) - half.sigma(x)).max() <= 1e-12 * np.abs(half.sigma(x)).max()
    assert np.abs(full.diag() - half.diag()).max() <= 1e-12 * np.abs(half.diag()).max()


def test_full_variational_subsets():
    """Lowest eigenvalue over a determinant list never lies below full CI, and
    never rises when determinants are added."""
    norb, n = 6, 3
    h, eri, ec = wl.make_integrals(norb, 91)
    allp = _random_dets(norb, n, n, 10 ** 6, 1)
    e_fci = np.linalg.eigvalsh(oracle.FullOracleSystem(norb, allp, h, eri, ec).dense_h())[0]
    small = oracle.FullOracleSystem(norb, allp[:150], h, eri, ec)
    big = oracle.FullOracleSystem(norb, allp[:300], h, eri, ec)
    e_s = np.linalg.eigvalsh(small.dense_h())[0]
    e_b = np.linalg.eigvalsh(big.dense_h())[0]
    assert e_fci <= e_b + 1e-10 and e_b <= e_s + 1e-10


@pytest.mark.parametrize("norb,na,nb,count,seed", [(6, 3, 3, 200, 11), (7, 3, 2, 300, 12)])
def test_full_sigma_rows_equals_dense(norb, na, nb, count, seed):
    """The row-sampled sigma of a determinant list (neighbours found per row by
    comparing with every determinant, no lists) equals the dense H applied to
    the vector at those rows; it needs no connection lists."""
    h, eri, ec = wl.make_integrals(norb, 80 + seed)
    dets = _random_dets(norb, na, nb, count, seed)
    S = oracle.FullOracleSystem(norb, dets, h, eri, ec)
    S2 = oracle.FullOracleSystem(norb, dets, h, eri, ec, connections=False)
    x = np.random.default_rng(seed).standard_normal(S.N)
    idx = np.array([0, S.N - 1, S.N // 2, 7, 7, 3])
    ref = S.dense_h()[idx] @ x
    got = S2.sigma_rows(x, idx)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(S.dense_h()).max() * np.abs(x).sum()
