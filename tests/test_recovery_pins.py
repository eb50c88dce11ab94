"""Pins of the oracle's sample post-processing (configuration recovery of an
SQD iteration) against facts that do not come from the oracle itself: the
published SplitMix64 output, the closed forms of the flip weight, occupations
of a single determinant and a brute-force sum over determinants, recovery
cases whose outcome is forced, and the draw frequencies the weights imply."""
import math

import numpy as np
import pytest

import workload as wl
from oracle import recovery as rec


def test_splitmix64_published_value_and_uniform_range():
    # the generator's first output from state 0 (the reference implementation's test value)
    assert rec.splitmix64(0) == 0xE220A8397B1DCDAF
    us = [rec.uniform(12345, c) for c in range(2000)]
    assert min(us) >= 0.0 and max(us) < 1.0
    assert abs(np.mean(us) - 0.5) < 0.03


def test_flip_weight_closed_forms():
    for h in (0.25, 0.5, 7 / 26):
        assert rec.flip_weight(0.0, h) == 0.0
        assert math.isclose(rec.flip_weight(h, h), rec.DELTA)
        assert math.isclose(rec.flip_weight(h + 1e-12, h), rec.DELTA, rel_tol=1e-9)
        assert math.isclose(rec.flip_weight(1.0, h), 1.0)
        ys = np.linspace(0, 1, 101)
        ws = [rec.flip_weight(y, h) for y in ys]
        assert all(b >= a for a, b in zip(ws, ws[1:]))
    assert rec.flip_weight(0.0, 0.0) == 0.0 and rec.flip_weight(1.0, 0.0) == 1.0


def test_occupations_single_determinant_and_brute_force():
    norb, na, nb = 6, 3, 2
    A, B = wl.all_strings(norb, na), wl.all_strings(norb, nb)
    x = np.zeros(A.size * B.size)
    x[4 * B.size + 7] = -2.0
    oa, ob = rec.occupations(norb, A, B, x)
    assert np.array_equal(oa, [(int(A[4]) >> p) & 1 for p in range(norb)])
    assert np.array_equal(ob, [(int(B[7]) >> p) & 1 for p in range(norb)])
    x = wl.random_vector(A.size * B.size, 3)[0]
    oa, ob = rec.occupations(norb, A, B, x)
    ra, rb = np.zeros(norb), np.zeros(norb)
    for ia, a in enumerate(A):
        for ib, b in enumerate(B):
            w = x[ia * B.size + ib] ** 2
            for p in range(norb):
                ra[p] += w * ((int(a) >> p) & 1)
                rb[p] += w * ((int(b) >> p) & 1)
    n2 = float(x @ x)
    assert np.allclose(oa, ra / n2, rtol=1e-13, atol=1e-15) and np.allclose(ob, rb / n2, rtol=1e-13, atol=1e-15)
    assert math.isclose(oa.sum(), na, rel_tol=1e-13) and math.isclose(ob.sum(), nb, rel_tol=1e-13)


def test_occupations_of_a_list_equal_product_occupations():
    """Over a complete product listed determinant by determinant (in the
    product's order) the list form gives the product form's occupations."""
    norb, na, nb = 6, 2, 3
    A, B = wl.all_strings(norb, na), wl.all_strings(norb, nb)
    dets = np.array([(a, b) for a in A for b in B], dtype=np.uint64)
    x = wl.random_vector(dets.shape[0], 4)[0]
    pa, pb = rec.occupations(norb, A, B, x)
    la, lb = rec.occupations_dets(norb, dets, x)
    assert np.allclose(pa, la, rtol=1e-14, atol=1e-15) and np.allclose(pb, lb, rtol=1e-14, atol=1e-15)
    u = np.zeros(dets.shape[0])
    u[5] = 3.0
    la, lb = rec.occupations_dets(norb, dets, u)
    assert np.array_equal(la, [(int(dets[5, 0]) >> p) & 1 for p in range(norb)])
    assert np.array_equal(lb, [(int(dets[5, 1]) >> p) & 1 for p in range(norb)])


@pytest.mark.parametrize("extra_a,extra_b", [(1, 0), (-1, 0), (2, -1), (0, 2), (-2, 1)])
def test_recovery_forced_by_exact_occupations(extra_a, extra_b):
    """Occupations exactly 0/1 on a determinant D: a sample that differs from D
    only by extra (or missing) electrons has zero weight on every other bit,
    so recovery returns D whatever the uniforms."""
    norb, na, nb = 10, 4, 3
    Da, Db = 0b0000101101, 0b0011000100
    occ_a = np.array([(Da >> p) & 1 for p in range(norb)], dtype=float)
    occ_b = np.array([(Db >> p) & 1 for p in range(norb)], dtype=float)

    def perturb(word, k, seed):
        rng = np.random.default_rng(seed)
        if k > 0:
            free = [p for p in range(norb) if not (word >> p) & 1]
            for p in rng.choice(free, k, replace=False):
                word |= 1 << int(p)
        elif k < 0:
            occ = [p for p in range(norb) if (word >> p) & 1]
            for p in rng.choice(occ, -k, replace=False):
                word &= ~(1 << int(p))
        return word

    for seed in range(20):
        s = np.array([[perturb(Da, extra_a, seed), perturb(Db, extra_b, seed + 100)]], dtype=np.uint64)
        out, nc = rec.recover(s, norb, na, nb, occ_a, occ_b, seed=seed)
        assert nc == int(extra_a != 0 or extra_b != 0)
        assert out.tolist() == [[Da, Db]]


def test_recovery_invariants_on_noisy_samples():
    norb, na, nb = 12, 5, 4
    S = wl.sample_configurations(norb, na, nb, 3000, 11)
    N = wl.add_readout_noise(S, norb, 0.03, 12)
    rng = np.random.default_rng(13)
    occ_a, occ_b = rng.random(norb), rng.random(norb)
    pc = lambda v: bin(int(v)).count("1")
    wrong = [i for i, (a, b) in enumerate(N) if pc(a) != na or pc(b) != nb]
    assert len(wrong) > 300
    out, nc = rec.recover(N, norb, na, nb, occ_a, occ_b, seed=99)
    assert nc == len(wrong) and out.shape == N.shape
    for (a0, b0), (a1, b1) in zip(N, out):
        a0, b0, a1, b1 = int(a0), int(b0), int(a1), int(b1)
        assert pc(a1) == na and pc(b1) == nb and a1 < (1 << norb) and b1 < (1 << norb)
        for w0, w1, n in ((a0, a1, na), (b0, b1, nb)):
            if pc(w0) > n:
                assert w1 & ~w0 == 0      # only removals
            elif pc(w0) < n:
                assert w0 & ~w1 == 0      # only additions
            else:
                assert w0 == w1
    kept, nc0 = rec.recover(N, norb, na, nb)  # no occupations: wrong samples dropped, order kept
    assert nc0 == 0
    assert kept.tolist() == [list(map(int, r)) for i, r in enumerate(N) if i not in set(wrong)]


def test_recovery_draw_frequencies_follow_weights():
    """One surplus electron: the removed bit is drawn with probability
    weight / total over the occupied bits (checked to 4 standard errors over
    20,000 independent counters)."""
    norb, na = 8, 3
    word = 0b10110001  # 4 electrons, one too many
    occ = np.array([0.9, 0.2, 0.5, 0.4, 0.95, 0.1, 0.3, 0.6])
    cand = [p for p in range(norb) if (word >> p) & 1]
    h = na / norb
    w = np.array([rec.flip_weight(abs(1.0 - occ[p]), h) for p in cand])
    prob = w / w.sum()
    M = 20000
    S = np.tile(np.array([[word, 0b111]], dtype=np.uint64), (M, 1))
    out, _ = rec.recover(S, norb, na, 3, occ, np.ones(norb), seed=2024)
    removed = [int(word) & ~int(a) for a in out[:, 0]]
    freq = np.array([sum(1 for r in removed if r == (1 << p)) for p in cand]) / M
    assert np.all(np.abs(freq - prob) <= 4 * np.sqrt(prob * (1 - prob) / M) + 1e-12)
