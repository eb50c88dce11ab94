"""CPU oracle of the sample post-processing of an SQD iteration (test
infrastructure: only the tests use it; it imports nothing from the product).

Sec. I describes the classical side of SQD as taking the device's sampled
configurations, filtering them, and diagonalising over the subspace they span,
iteration after iteration.  Samples of a noisy device can carry the wrong
number of electrons in a spin sector.  These functions correct them from the
previous iteration's solution, one bit at a time (the configuration-recovery
step of the SQD workflow the paper builds on, restated here in our own reading):

* ``occupations``: the average occupation of every spin-orbital over a
  normalised vector in the alpha x beta product basis,
  n_sp = sum_I |c_I|^2 occ_sp(I);
* ``flip_weight``: the weight of a bit whose sampled value x_p lies at
  distance y = |x_p - n_sp| from that average: a ramp of slope delta / h up to
  the spin's filling h = n_s / norb, then a steeper ramp from delta to 1;
* ``recover``: a sample with too many electrons in a spin loses occupied bits,
  one with too few gains empty bits, chosen one after another without
  replacement with probability proportional to their weights (inverse CDF over
  the remaining candidates in increasing orbital order); samples with the
  right counts pass unchanged; without occupations (the first iteration),
  samples with wrong counts are dropped;
* ``splitmix64`` / ``uniform``: the counter-based generator of the uniforms,
  SplitMix64 (Steele, Lea and Flood, 2014), top 53 bits scaled by 2^-53.

All decisions are taken in FP64 in the order written here, which the library
follows as well, so the recovered samples are compared bit for bit.
"""
from __future__ import annotations

import numpy as np

DELTA = 0.01
MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (the state advanced once by the golden
    gamma, then the two xor-shift-multiply rounds and a final xor-shift)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def uniform(seed: int, counter: int) -> float:
    """Uniform in [0, 1) for (seed, counter): 53 top bits of
    splitmix64(seed + counter) times 2^-53."""
    return float(splitmix64((seed + counter) & MASK64) >> 11) * (1.0 / 9007199254740992.0)


def draw_counter(sample: int, spin: int, j: int) -> int:
    """Counter of the j-th draw for a sample's spin sector (64 per sector)."""
    return (sample * 2 + spin) * 64 + j


def occupations(norb: int, alpha, beta, vec) -> tuple[np.ndarray, np.ndarray]:
    """(n_alpha[p], n_beta[p]) of a vector over the product basis, index
    ia * len(beta) + ib, normalised by its squared norm."""
    alpha = np.asarray(alpha, dtype=np.uint64)
    beta = np.asarray(beta, dtype=np.uint64)
    w = np.asarray(vec, dtype=np.float64).reshape(alpha.size, beta.size) ** 2
    total = w.sum()
    out = []
    for strings, ws in ((alpha, w.sum(axis=1)), (beta, w.sum(axis=0))):
        occ = np.zeros(norb)
        for p in range(norb):
            bit = ((strings >> np.uint64(p)) & np.uint64(1)).astype(bool)
            occ[p] = ws[bit].sum() / total
        out.append(occ)
    return out[0], out[1]


def occupations_dets(norb: int, dets, vec) -> tuple[np.ndarray, np.ndarray]:
    """The same over a determinant list (rows: alpha word, beta word), one
    vector entry per determinant."""
    dets = np.asarray(dets, dtype=np.uint64).reshape(-1, 2)
    w = np.asarray(vec, dtype=np.float64) ** 2
    total = w.sum()
    out = []
    for col in (0, 1):
        occ = np.zeros(norb)
        for p in range(norb):
            bit = ((dets[:, col] >> np.uint64(p)) & np.uint64(1)).astype(bool)
            occ[p] = w[bit].sum() / total
        out.append(occ)
    return out[0], out[1]


def flip_weight(y: float, h: float, delta: float = DELTA) -> float:
    """Weight of a bit at distance y from its average occupation, filling h."""
    if y <= h:
        return delta * y / h if h > 0.0 else 0.0
    return delta + (1.0 - delta) * (y - h) / (1.0 - h)


def _recover_word(word: int, n: int, norb: int, occ: np.ndarray, seed: int, sample: int, spin: int) -> int:
    w = bin(word).count("1")
    if w == n:
        return word
    h = n / norb
    remove = w > n
    cand = [p for p in range(norb) if ((word >> p) & 1) == (1 if remove else 0)]
    x = 1.0 if remove else 0.0
    wts = [flip_weight(abs(x - float(occ[p])), h) for p in cand]
    for j in range(abs(w - n)):
        u = uniform(seed, draw_counter(sample, spin, j))
        total = 0.0
        for v in wts:
            total += v
        if total > 0.0:
            target = u * total
            cum = 0.0
            pick = -1
            for i, v in enumerate(wts):
                cum += v
                if target < cum:
                    pick = i
                    break
            if pick < 0:  # rounding: the last candidate of nonzero weight
                pick = max(i for i, v in enumerate(wts) if v > 0.0)
        else:
            pick = int(u * len(cand))
        word ^= 1 << cand[pick]
        del cand[pick]
        del wts[pick]
    return word


def recover(samples, norb: int, n_alpha: int, n_beta: int, occ_alpha=None, occ_beta=None,
            seed: int = 0) -> tuple[np.ndarray, int]:
    """Samples (rows: alpha word, beta word) after recovery, in order; and the
    number of samples corrected.  Without occupations, samples with a wrong
    electron count are dropped instead."""
    samples = np.asarray(samples, dtype=np.uint64).reshape(-1, 2)
    out = []
    corrected = 0
    for i, (a, b) in enumerate(samples):
        a, b = int(a), int(b)
        ok = bin(a).count("1") == n_alpha and bin(b).count("1") == n_beta
        if ok:
            out.append((a, b))
            continue
        if occ_alpha is None:
            continue
        out.append((_recover_word(a, n_alpha, norb, np.asarray(occ_alpha), seed, i, 0),
                    _recover_word(b, n_beta, norb, np.asarray(occ_beta), seed, i, 1)))
        corrected += 1
    return np.array(out, dtype=np.uint64).reshape(-1, 2), corrected
