"""Seeded synthetic inputs for selected-basis diagonalisation.

This module only draws inputs: one- and two-electron integrals, a core energy
and alpha/beta occupation bitstring sets.  It holds none of the method's
arithmetic (no matrix elements, no excitation tables, no sigma) and is shared
by the CPU oracle, the tests and the benchmark so both sides of every parity
check read the very same arrays.

Conventions
-----------
* Orbital p is bit p of a ``uint64`` half-bitstring (bit 0 = lowest orbital).
* Integrals: ``h[p, q]`` symmetric; ``eri[p, q, r, s]`` is the chemists'
  integral (pq|rs), built as sum_k L^k_pq L^k_rs with symmetric L^k, so it has
  the full 8-fold permutational symmetry and is positive semidefinite as a
  (pq),(rs) matrix.
* The string sets stand in for the quantum-sampled configurations of the
  paper's experiment (Sec. IV, Fe4S4 with 6,000 sampled 36-bit
  configurations), which are not available: strings are drawn without
  replacement with probability proportional to exp(-0.7 * excitation level
  relative to the Aufbau string), the Aufbau string always included.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

E_CORE_DEFAULT = 10.0
LEVEL_DECAY = 0.7
_ENUMERATE_LIMIT = 2_000_000


def make_integrals(norb: int, seed: int):
    """Return (h, eri, e_core) for ``norb`` spatial orbitals.

    Draw order with ``numpy.random.default_rng(seed)``:
    1. orbital energies uniform in [-20, 2], sorted ascending, on the diagonal
       of h;
    2. off-diagonal h_pq (p < q, row-major) ~ N(0, 0.1) * exp(-|p-q|/4);
    3. for k = 0 .. 2*norb-1, the upper triangle (with diagonal, row-major) of
       a symmetric L^k ~ N(0, 0.3/sqrt(k+1)).
    """
    if norb < 1:
        raise ValueError("norb must be >= 1")
    rng = np.random.default_rng(seed)
    eps = np.sort(rng.uniform(-20.0, 2.0, norb))
    h = np.diag(eps).astype(np.float64)
    iu, ju = np.triu_indices(norb, 1)
    off = rng.normal(0.0, 0.1, size=iu.size) * np.exp(-np.abs(iu - ju) / 4.0)
    h[iu, ju] = off
    h[ju, iu] = off
    it, jt = np.triu_indices(norb, 0)
    nl = 2 * norb
    L = np.zeros((nl, norb, norb))
    for k in range(nl):
        v = rng.normal(0.0, 0.3 / math.sqrt(k + 1), size=it.size)
        L[k, it, jt] = v
        L[k, jt, it] = v
    Lm = L.reshape(nl, norb * norb)
    eri = (Lm.T @ Lm).reshape(norb, norb, norb, norb)
    # exact symmetrisation guards against last-bit asymmetry of the product
    eri = 0.5 * (eri + eri.transpose(2, 3, 0, 1))
    return h, np.ascontiguousarray(eri), E_CORE_DEFAULT


def all_strings(norb: int, n: int) -> np.ndarray:
    """Every occupation string with ``n`` of ``norb`` bits set, ascending.

    Built by the recurrence S(m, k) = S(m-1, k) + (S(m-1, k-1) with bit m-1 set),
    keeping only the k that can still reach n; for n > norb/2 the strings are the
    complements of the (norb - n)-subsets."""
    if 2 * n > norb:
        full = np.uint64((1 << norb) - 1)
        out = all_strings(norb, norb - n) ^ full
        out.sort()
        return out
    level = {0: np.zeros(1, dtype=np.uint64)}
    for m in range(1, norb + 1):
        bit = np.uint64(1) << np.uint64(m - 1)
        lo, hi = max(0, n - (norb - m)), min(m, n)
        nxt = {}
        for k in range(lo, hi + 1):
            parts = [level[k]] if k in level else []
            if k - 1 in level:
                parts.append(level[k - 1] | bit)
            nxt[k] = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint64)
        level = nxt
    out = level[n].copy()
    out.sort()
    return out


_POPCOUNT8 = np.array([bin(i).count("1") for i in range(256)], dtype=np.int64)


def _level(strings: np.ndarray, n: int) -> np.ndarray:
    aufbau = np.uint64((1 << n) - 1)
    x = strings & ~aufbau
    # popcount of uint64 via byte table
    b = x.view(np.uint8).reshape(-1, 8)
    return _POPCOUNT8[b].sum(axis=1)


def sample_strings(norb: int, n: int, count: int, seed: int,
                   decay: float = LEVEL_DECAY) -> np.ndarray:
    """Sorted unique occupation strings drawn without replacement.

    P(string) is proportional to exp(-decay * level), level = number of
    electrons outside the Aufbau orbitals.  When all C(norb, n) strings can be
    enumerated this uses weighted sampling keys u**(1/w) (Efraimidis and
    Spirakis); otherwise a level is drawn with probability proportional to
    C(n,k) C(norb-n,k) exp(-decay k), then k holes and k particles uniformly,
    rejecting duplicates.  Both realise successive sampling proportional to
    the weight.  The Aufbau string is always included.
    """
    if not (0 <= n <= norb <= 64):
        raise ValueError("need 0 <= n <= norb <= 64")
    total = math.comb(norb, n)
    count = min(int(count), total)
    if count <= 0:
        return np.zeros(0, dtype=np.uint64)
    rng = np.random.default_rng(seed)
    aufbau = (1 << n) - 1
    if count == total:
        return all_strings(norb, n)
    if total <= _ENUMERATE_LIMIT:
        pool = all_strings(norb, n)
        w = np.exp(-decay * _level(pool, n).astype(np.float64))
        u = rng.uniform(size=pool.size)
        key = np.log(u) / w          # log of u**(1/w); larger is better
        key[pool == np.uint64(aufbau)] = np.inf
        pick = np.argpartition(-key, count - 1)[:count]
        out = np.sort(pool[pick])
        return out
    kmax = min(n, norb - n)
    ks = np.arange(kmax + 1)
    wk = np.array([math.comb(n, k) * math.comb(norb - n, k) * math.exp(-decay * k) for k in ks])
    pk = wk / wk.sum()
    # candidates in batches, in draw order: level k, then k holes among the
    # occupied and k particles among the empty orbitals (random orders, first k);
    # the first occurrence of each string is kept until `count` are chosen
    chosen, seen = [aufbau], {aufbau}
    one = np.uint64(1)
    while len(chosen) < count:
        M = max(1024, 2 * (count - len(chosen)))
        ks = rng.choice(kmax + 1, size=M, p=pk)
        holes = np.argsort(rng.random((M, n)), axis=1)[:, :kmax].astype(np.uint64)
        parts = (np.argsort(rng.random((M, norb - n)), axis=1)[:, :kmax] + n).astype(np.uint64)
        cand = np.full(M, np.uint64(aufbau), dtype=np.uint64)
        for j in range(kmax):
            sel = ks > j
            cand[sel] = (cand[sel] & ~(one << holes[sel, j])) | (one << parts[sel, j])
        for v in cand.tolist():
            if v not in seen:
                seen.add(v)
                chosen.append(v)
                if len(chosen) == count:
                    break
    return np.array(sorted(chosen), dtype=np.uint64)


@dataclass
class Workload:
    name: str
    norb: int
    n_alpha: int
    n_beta: int
    alpha: np.ndarray
    beta: np.ndarray
    h: np.ndarray
    eri: np.ndarray
    e_core: float
    nroots: int = 1
    tol: float = 1e-6
    meta: dict = field(default_factory=dict)

    @property
    def ndet(self) -> int:
        return int(self.alpha.size) * int(self.beta.size)


# The five synthetic configurations: (name, norb, n, strings per spin,
# roots, seeds (integrals, alpha, beta), residual tolerance).
CONFIGS = {
    "fci8": dict(norb=8, n=4, nstr=None, nroots=1, seeds=(101, 0, 0), tol=1e-8),
    "sel16": dict(norb=16, n=8, nstr=2000, nroots=1, seeds=(102, 2001, 2002), tol=1e-6),
    "sel26": dict(norb=26, n=7, nstr=10000, nroots=1, seeds=(103, 3001, 3002), tol=1e-6),
    "block20": dict(norb=20, n=8, nstr=5000, nroots=4, seeds=(104, 4001, 4002), tol=1e-6),
}


def make_config(name: str, nstr: int | None = None) -> Workload:
    """Build one of the named synthetic workloads (optionally with fewer strings)."""
    c = CONFIGS[name]
    norb, n = c["norb"], c["n"]
    si, sa, sb = c["seeds"]
    h, eri, ecore = make_integrals(norb, si)
    k = nstr if nstr is not None else c["nstr"]
    if k is None:
        a = all_strings(norb, n)
        b = all_strings(norb, n)
    else:
        a = sample_strings(norb, n, k, sa)
        b = sample_strings(norb, n, k, sb)
    return Workload(name, norb, n, n, a, b, h, eri, ecore, c["nroots"], c["tol"],
                    meta=dict(seeds=c["seeds"], nstr=k))


def sample_product_subset(alpha: np.ndarray, beta: np.ndarray, n_alpha: int, n_beta: int, count: int,
                          seed: int, decay: float = LEVEL_DECAY) -> np.ndarray:
    """Unique determinants (rows: alpha string, beta string), sorted by alpha
    then beta string, drawn from the product of two string pools without
    replacement: a stand-in for a list of sampled configurations that is not a
    Cartesian product (most pairs of the pools are absent).

    P(alpha, beta) is proportional to exp(-decay * (level_alpha + level_beta))
    (level = electrons outside the Aufbau orbitals): candidates draw their
    alpha and beta strings independently with weights exp(-decay * level), and
    the first occurrence of each pair is kept until `count` pairs are found.
    The pair of the pools' first strings (their Aufbau strings when present)
    is always included.
    """
    alpha = np.ascontiguousarray(alpha, dtype=np.uint64)
    beta = np.ascontiguousarray(beta, dtype=np.uint64)
    na, nb = alpha.size, beta.size
    count = min(int(count), na * nb)
    if count <= 0:
        return np.zeros((0, 2), dtype=np.uint64)
    rng = np.random.default_rng(seed)
    wa = np.exp(-decay * _level(alpha, n_alpha).astype(np.float64))
    wb = np.exp(-decay * _level(beta, n_beta).astype(np.float64))
    ca, cb = np.cumsum(wa / wa.sum()), np.cumsum(wb / wb.sum())
    ia0 = int(np.argmin(_level(alpha, n_alpha)))
    ib0 = int(np.argmin(_level(beta, n_beta)))
    keys = np.array([ia0 * nb + ib0], dtype=np.int64)
    while True:
        _, first = np.unique(keys, return_index=True)
        if first.size >= count:
            break
        M = max(1 << 16, 2 * (count - first.size))
        ia = np.minimum(np.searchsorted(ca, rng.random(M), side="right"), na - 1)
        ib = np.minimum(np.searchsorted(cb, rng.random(M), side="right"), nb - 1)
        keys = np.concatenate([keys[np.sort(first)], ia.astype(np.int64) * nb + ib])
    keep = np.sort(keys[np.sort(first)[:count]])
    out = np.empty((count, 2), dtype=np.uint64)
    out[:, 0] = alpha[keep // nb]
    out[:, 1] = beta[keep % nb]
    order = np.lexsort((out[:, 1], out[:, 0]))
    return out[order]


def sample_configurations(norb: int, n_alpha: int, n_beta: int, count: int, seed: int,
                          decay: float = LEVEL_DECAY) -> np.ndarray:
    """Sampled configurations with repeats, in drawing order (rows: alpha
    string, beta string): a stand-in for the measurement record of a quantum
    device that an SQD run diagonalises in growing prefixes.  Each spin's
    string draws its excitation level k with probability proportional to
    C(n,k) C(norb-n,k) exp(-decay k), then k holes among the n lowest orbitals
    and k particles among the others, uniformly."""
    rng = np.random.default_rng(seed)
    out = np.empty((count, 2), dtype=np.uint64)
    one = np.uint64(1)
    for col, n in ((0, n_alpha), (1, n_beta)):
        kmax = min(n, norb - n)
        wk = np.array([math.comb(n, k) * math.comb(norb - n, k) * math.exp(-decay * k) for k in range(kmax + 1)])
        kk = rng.choice(kmax + 1, size=count, p=wk / wk.sum())
        holes = np.argsort(rng.random((count, max(n, 1))), axis=1)[:, :kmax].astype(np.uint64)
        parts = (np.argsort(rng.random((count, max(norb - n, 1))), axis=1)[:, :kmax] + n).astype(np.uint64)
        s = np.full(count, np.uint64((1 << n) - 1), dtype=np.uint64)
        for j in range(kmax):
            sel = kk > j
            s[sel] = (s[sel] & ~(one << holes[sel, j])) | (one << parts[sel, j])
        out[:, col] = s
    return out


def add_readout_noise(samples: np.ndarray, norb: int, p_flip: float, seed: int) -> np.ndarray:
    """Sampled configurations with every bit below norb of both words flipped
    independently with probability p_flip: a stand-in for a noisy device's
    records, whose strings can carry the wrong number of electrons."""
    rng = np.random.default_rng(seed)
    out = np.array(samples, dtype=np.uint64, copy=True).reshape(-1, 2)
    flips = rng.random((out.shape[0], 2, norb)) < p_flip
    weights = (np.uint64(1) << np.arange(norb, dtype=np.uint64))
    mask = (flips * weights).sum(axis=2, dtype=np.uint64)
    return out ^ mask


@dataclass
class FullWorkload:
    """A full-bitstring workload: an explicit determinant list."""
    name: str
    norb: int
    n_alpha: int
    n_beta: int
    dets: np.ndarray  # (N, 2) uint64: alpha string, beta string
    h: np.ndarray
    eri: np.ndarray
    e_core: float
    nroots: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def ndet(self) -> int:
        return int(self.dets.shape[0])


# Full-bitstring workloads: determinant lists drawn from the product of a
# product workload's alpha and beta string sets (same integrals), with the
# seed of the draw.
FULL_CONFIGS = {
    "full16": dict(pool="sel16", ndet=1_000_000, nroots=1, seed=5101),
    "full26": dict(pool="sel26", ndet=4_000_000, nroots=1, seed=5102),
}


def make_full_config(name: str, ndet: int | None = None, nstr: int | None = None) -> FullWorkload:
    """A named full-bitstring workload, optionally with fewer determinants or
    smaller string pools."""
    c = FULL_CONFIGS[name]
    P = make_config(c["pool"], nstr=nstr)
    n = ndet if ndet is not None else c["ndet"]
    d = sample_product_subset(P.alpha, P.beta, P.n_alpha, P.n_beta, n, c["seed"])
    return FullWorkload(name, P.norb, P.n_alpha, P.n_beta, d, P.h, P.eri, P.e_core, c["nroots"],
                        meta=dict(seeds=(P.meta["seeds"][0], P.meta["seeds"][1], P.meta["seeds"][2], c["seed"]),
                                  ndet=n, pool=c["pool"], nstr=P.alpha.size))


def serving_stream(nreq: int = 256, seed: int = 5000, rate: float = 20.0,
                   norb_range=(12, 32), ndet_range=(1e4, 2e7)):
    """Request descriptors of the serving workload (no arrays, cheap).

    Poisson arrivals at ``rate`` per second; norb uniform in the range,
    n = floor(norb/2) - 1 electrons per spin, a log-uniform target
    determinant count, sqrt of it strings per spin (capped at C(norb, n)),
    1 or 2 roots.  Request r draws its integrals with seed+r and its alpha and
    beta strings with seed+r+100000 and seed+r+200000.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(nreq):
        t += rng.exponential(1.0 / rate)
        norb = int(rng.integers(norb_range[0], norb_range[1] + 1))
        n = norb // 2 - 1
        ndet = math.exp(rng.uniform(math.log(ndet_range[0]), math.log(ndet_range[1])))
        nstr = min(int(round(math.sqrt(ndet))), math.comb(norb, n))
        nroots = int(rng.integers(1, 3))
        out.append(dict(index=r, arrival=t, norb=norb, n=n, nstr=nstr, nroots=nroots,
                        seeds=(seed + r, seed + r + 100000, seed + r + 200000)))
    return out


def make_request(desc: dict) -> Workload:
    """Materialise the arrays of one serving request."""
    norb, n = desc["norb"], desc["n"]
    si, sa, sb = desc["seeds"]
    h, eri, ecore = make_integrals(norb, si)
    a = sample_strings(norb, n, desc["nstr"], sa)
    b = sample_strings(norb, n, desc["nstr"], sb)
    return Workload(f"req{desc['index']}", norb, n, n, a, b, h, eri, ecore,
                    desc["nroots"], 1e-6, meta=dict(desc))


def random_vector(ndet: int, seed: int, nvec: int = 1) -> np.ndarray:
    """Unit-norm random FP64 vectors, shape (nvec, ndet)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nvec, ndet))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x
