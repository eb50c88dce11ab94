"""CPU FP64 oracle for selected-basis diagonalisation (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the product path never imports it, and it imports nothing from the
product.  It shares only the seeded input generators (``workload``) with the
HIP path.

Three tiers, each written from the paper (Sec. II):

* tier 0 (``tier0_dense_h``): the second-quantised Hamiltonian of Eq. 3
  applied operator by operator to full spin-orbital strings (numpy, tiny
  cases).  No Slater-Condon case analysis.
* tier 1 (``OracleSystem``; C in ``sbd_oracle.c``): brute-force excitation
  tables, the diagonal, generic spin-orbital Slater-Condon matrix elements
  (Eq. 4) and the matrix-free sigma y = H x.
* tier 2 (``davidson``): the Davidson iteration of Sec. II-C with the
  damped diagonal preconditioner of Eqs. 6-7, modified Gram-Schmidt with a
  second pass, and restart; dense ``numpy.linalg.eigh`` for small spaces.

``map_vector`` carries a vector from one determinant basis to another (the
warm start of a later SQD iteration's solve, Sec. I and the free choice of the
Davidson start vector, Sec. II-C).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

from .build import build as build_oracle, LIB_PATH

_lib = None


def lib():
    """Load the oracle's C library, compiling it with gcc if it is not built."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORC_LIB_PATH") or LIB_PATH  # e.g. the sanitized build
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build_oracle()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int
        d = ctypes.c_double
        L.orc_sort_unique.argtypes = [P, i64]
        L.orc_sort_unique.restype = i64
        L.orc_exc_table.argtypes = [P, i64, i32, i32, P, P, P, P]
        L.orc_exc_table.restype = i32
        tab = [P] * 8
        L.orc_sigma.argtypes = [i32, P, P, d, P, i64, P, i64] + tab + [i32, P, P]
        L.orc_sigma.restype = i32
        L.orc_sigma_at.argtypes = [i32, P, P, d, P, i64, P, i64] + tab + [P, P, i64, P]
        L.orc_sigma_at.restype = i32
        L.orc_sigma_abs_at.argtypes = [i32, P, P, d, P, i64, P, i64] + tab + [P, d, P, i64, P]
        L.orc_sigma_abs_at.restype = i32
        L.orc_diag.argtypes = [i32, P, P, d, P, i64, P, i64, P]
        L.orc_diag.restype = i32
        L.orc_dense_h.argtypes = [i32, P, P, d, P, i64, P, i64, P]
        L.orc_dense_h.restype = i32
        L.orc_hij.argtypes = [i32, P, P, d, ctypes.c_uint64, ctypes.c_uint64,
                              ctypes.c_uint64, ctypes.c_uint64]
        L.orc_hij.restype = d
        L.orc_full_sort_unique.argtypes = [P, i64]
        L.orc_full_sort_unique.restype = i64
        L.orc_full_connections.argtypes = [P, i64, P, P, P]
        L.orc_full_connections.restype = i32
        L.orc_full_sigma.argtypes = [i32, P, P, d, P, i64, P, P, i32, P, P]
        L.orc_full_sigma.restype = i32
        L.orc_full_sigma_rows.argtypes = [i32, P, P, d, P, i64, P, i64, P, P]
        L.orc_full_sigma_rows.restype = i32
        L.orc_full_diag.argtypes = [i32, P, P, d, P, i64, P]
        L.orc_full_diag.restype = i32
        L.orc_full_dense_h.argtypes = [i32, P, P, d, P, i64, P]
        L.orc_full_dense_h.restype = i32
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------------------
# Tier 1: strings, tables, diagonal, sigma (C)
# ---------------------------------------------------------------------------

def sort_unique(strings) -> np.ndarray:
    """Ascending unsigned order, duplicates removed."""
    s = np.array(strings, dtype=np.uint64).copy()
    k = lib().orc_sort_unique(_p(s), s.size)
    return s[:k].copy()


@dataclass
class ExcTable:
    """CSR excitation table of one spin and one kind (1 = single, 2 = double)."""
    row_ptr: np.ndarray   # int64 [n+1]
    J: np.ndarray         # int32 [nnz] ket string index, ascending within a row
    orbs: np.ndarray      # uint8 [nnz, 2*kind]: (i, a) or (i, j, a, b)
    sign: np.ndarray      # int8 [nnz]


def exc_table(strings: np.ndarray, norb: int, kind: int) -> ExcTable:
    """Brute-force pairwise table (every string pair compared by popcount)."""
    s = np.ascontiguousarray(strings, dtype=np.uint64)
    n = s.size
    rp = np.zeros(n + 1, dtype=np.int64)
    rc = lib().orc_exc_table(_p(s), n, norb, kind, _p(rp), None, None, None)
    if rc != 0:
        raise ValueError("bad table kind")
    nnz = int(rp[-1])
    J = np.zeros(max(nnz, 1), dtype=np.int32)
    orbs = np.zeros((max(nnz, 1), 2 * kind), dtype=np.uint8)
    sign = np.zeros(max(nnz, 1), dtype=np.int8)
    lib().orc_exc_table(_p(s), n, norb, kind, _p(rp), _p(J), _p(orbs), _p(sign))
    return ExcTable(rp, J[:nnz], orbs[:nnz], sign[:nnz])


class OracleSystem:
    """A selected basis (alpha x beta strings) with its Hamiltonian."""

    def __init__(self, norb, alpha, beta, h, eri, e_core):
        self.norb = int(norb)
        self.alpha = sort_unique(alpha)
        self.beta = sort_unique(beta)
        self.h = np.ascontiguousarray(h, dtype=np.float64)
        self.eri = np.ascontiguousarray(eri, dtype=np.float64)
        self.e_core = float(e_core)
        self.na, self.nb = self.alpha.size, self.beta.size
        self.N = self.na * self.nb
        self.a1 = exc_table(self.alpha, self.norb, 1)
        self.a2 = exc_table(self.alpha, self.norb, 2)
        self.b1 = exc_table(self.beta, self.norb, 1)
        self.b2 = exc_table(self.beta, self.norb, 2)
        self._diag = None

    @classmethod
    def from_workload(cls, w):
        return cls(w.norb, w.alpha, w.beta, w.h, w.eri, w.e_core)

    def _common(self):
        return (self.norb, _p(self.h), _p(self.eri), self.e_core,
                _p(self.alpha), self.na, _p(self.beta), self.nb,
                _p(self.a1.row_ptr), _p(self.a1.J), _p(self.a2.row_ptr), _p(self.a2.J),
                _p(self.b1.row_ptr), _p(self.b1.J), _p(self.b2.row_ptr), _p(self.b2.J))

    def sigma(self, x: np.ndarray) -> np.ndarray:
        """y = H x; x of shape (N,) or (nvec, N)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        single = x.ndim == 1
        X = x.reshape(1, -1) if single else x
        if X.shape[1] != self.N:
            raise ValueError("vector length != number of determinants")
        Y = np.empty_like(X)
        for v0 in range(0, X.shape[0], 64):
            xs = np.ascontiguousarray(X[v0:v0 + 64])
            ys = np.empty_like(xs)
            lib().orc_sigma(*self._common(), xs.shape[0], _p(xs), _p(ys))
            Y[v0:v0 + 64] = ys
        return Y[0] if single else Y

    def sigma_at(self, x: np.ndarray, idx) -> np.ndarray:
        """(H x)_I for the determinant indices in idx (one vector)."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        y = np.empty(idx.size, dtype=np.float64)
        lib().orc_sigma_at(*self._common(), _p(x), _p(idx), idx.size, _p(y))
        return y

    def sigma_abs_at(self, x: np.ndarray, idx, shift: float = 0.0) -> np.ndarray:
        """(|H - shift I| |x|)_I for the determinant indices in idx (one vector):
        the magnitude sum that bounds the rounding error of (H - shift) x."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        y = np.empty(idx.size, dtype=np.float64)
        lib().orc_sigma_abs_at(*self._common(), _p(x), float(shift), _p(idx), idx.size, _p(y))
        return y

    def row_terms(self, idx) -> np.ndarray:
        """z_I, the number of stored terms of row I of H (the determinant itself
        and its Slater-Condon neighbours in the basis), for I in idx."""
        idx = np.asarray(idx, dtype=np.int64)
        ia, ib = idx // self.nb, idx % self.nb
        la = lambda t, i: t.row_ptr[i + 1] - t.row_ptr[i]
        s1a, s2a, s1b, s2b = la(self.a1, ia), la(self.a2, ia), la(self.b1, ib), la(self.b2, ib)
        return 1 + s1a + s2a + s1b + s2b + s1a * s1b

    def diag(self) -> np.ndarray:
        if self._diag is None:
            d = np.empty(self.N, dtype=np.float64)
            lib().orc_diag(self.norb, _p(self.h), _p(self.eri), self.e_core,
                           _p(self.alpha), self.na, _p(self.beta), self.nb, _p(d))
            self._diag = d
        return self._diag

    def dense_h(self) -> np.ndarray:
        """H over all determinant pairs, brute force (no tables).  Small N only."""
        if self.N > 20000:
            raise ValueError("dense H only for small bases")
        out = np.empty((self.N, self.N), dtype=np.float64)
        lib().orc_dense_h(self.norb, _p(self.h), _p(self.eri), self.e_core,
                          _p(self.alpha), self.na, _p(self.beta), self.nb, _p(out))
        return out

    def hij(self, ia, ib, ja, jb) -> float:
        return float(lib().orc_hij(self.norb, _p(self.h), _p(self.eri), self.e_core,
                                   int(self.alpha[ia]), int(self.beta[ib]),
                                   int(self.alpha[ja]), int(self.beta[jb])))

    def nnz(self) -> int:
        """Connected (bra, ket) pairs including the diagonal:
        N + nb (P1a + P2a) + na (P1b + P2b) + P1a P1b, P = table entries."""
        p1a = int(self.a1.row_ptr[-1]); p2a = int(self.a2.row_ptr[-1])
        p1b = int(self.b1.row_ptr[-1]); p2b = int(self.b2.row_ptr[-1])
        return self.N + self.nb * (p1a + p2a) + self.na * (p1b + p2b) + p1a * p1b


# ---------------------------------------------------------------------------
# Full-bitstring bases (Sec. II-F, Sec. III-F): arbitrary determinant lists
# ---------------------------------------------------------------------------

def full_sort_unique(dets) -> np.ndarray:
    """Determinants as rows (alpha string, beta string), sorted by alpha then
    beta ascending, duplicates removed."""
    d = np.ascontiguousarray(np.asarray(dets, dtype=np.uint64).reshape(-1, 2)).copy()
    k = lib().orc_full_sort_unique(_p(d), d.shape[0])
    return d[:k].copy()


class FullOracleSystem:
    """A selected basis given as a list of determinants (one packed
    spin-orbital string each: alpha word, beta word) with its Hamiltonian.
    Connections come from comparing every pair of determinants; matrix
    elements from the same generic Slater-Condon rules as OracleSystem."""

    def __init__(self, norb, dets, h, eri, e_core, connections=True):
        """connections=False skips the all-pairs connection lists (then only
        diag, dense_h and sigma_rows are available)."""
        self.norb = int(norb)
        self.dets = full_sort_unique(dets)
        self.N = self.dets.shape[0]
        self.h = np.ascontiguousarray(h, dtype=np.float64)
        self.eri = np.ascontiguousarray(eri, dtype=np.float64)
        self.e_core = float(e_core)
        self.row_ptr = self.J = self.deg = None
        if not connections:
            return
        rp = np.zeros(self.N + 1, dtype=np.int64)
        lib().orc_full_connections(_p(self.dets), self.N, _p(rp), None, None)
        nnz = int(rp[-1])
        J = np.zeros(max(nnz, 1), dtype=np.int32)
        deg = np.zeros(max(nnz, 1), dtype=np.int8)
        lib().orc_full_connections(_p(self.dets), self.N, _p(rp), _p(J), _p(deg))
        self.row_ptr, self.J, self.deg = rp, J[:nnz], deg[:nnz]

    def _ham(self):
        return (self.norb, _p(self.h), _p(self.eri), self.e_core, _p(self.dets), self.N)

    def sigma(self, x: np.ndarray) -> np.ndarray:
        """y = H x; x of shape (N,) or (nvec, N)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        X = x.reshape(-1, self.N)
        Y = np.empty_like(X)
        lib().orc_full_sigma(*self._ham(), _p(self.row_ptr), _p(self.J), X.shape[0], _p(X), _p(Y))
        return Y.reshape(x.shape)

    def diag(self) -> np.ndarray:
        out = np.empty(self.N)
        lib().orc_full_diag(*self._ham(), _p(out))
        return out

    def sigma_rows(self, x: np.ndarray, idx) -> np.ndarray:
        """(H x)_I at the rows idx only, each row's neighbours found by
        comparing it with every determinant (no connection lists)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.empty(idx.size)
        lib().orc_full_sigma_rows(*self._ham(), _p(idx), idx.size, _p(x), _p(out))
        return out

    def dense_h(self) -> np.ndarray:
        """H over all determinant pairs, brute force (no connection lists)."""
        if self.N > 20000:
            raise ValueError("dense H only for small bases")
        out = np.empty((self.N, self.N))
        lib().orc_full_dense_h(*self._ham(), _p(out))
        return out

    def nnz(self) -> int:
        """Stored terms of H: the diagonal plus every connection."""
        return self.N + int(self.row_ptr[-1])


# ---------------------------------------------------------------------------
# Tier 0: operator definition of Eq. 3 on full spin-orbital strings (numpy)
# ---------------------------------------------------------------------------

def _popcount(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.int64)
    c = np.zeros_like(x)
    while np.any(x):
        c += x & 1
        x = x >> 1
    return c


def _annihilate(st, ph, P):
    occ = (st >> P) & 1
    sgn = 1 - 2 * (_popcount(st & ((1 << P) - 1)) & 1)
    return st & ~np.int64(1 << P), ph * occ * sgn


def _create(st, ph, P):
    emp = 1 - ((st >> P) & 1)
    sgn = 1 - 2 * (_popcount(st & ((1 << P) - 1)) & 1)
    return st | np.int64(1 << P), ph * emp * sgn


def tier0_dense_h(norb, alpha, beta, h, eri, e_core) -> np.ndarray:
    """H_ij = <Phi_i|H|Phi_j> by applying every operator term of Eq. 3.

    A determinant (alpha string a, beta string b) is the spin-orbital string
    a | (b << norb): alpha creators first, then beta, each ascending.  The
    Hamiltonian is sum_{pq,s} h_pq a+_ps a_qs
    + 1/2 sum_{pqrs,s,t} (pq|rs) a+_ps a+_rt a_st a_qs + e_core,
    applied right to left to every ket at once; components landing outside
    the selected set are dropped (projection onto the subspace).
    Intended for norb <= 6.
    """
    alpha = sort_unique(alpha)
    beta = sort_unique(beta)
    dets = [(int(a), int(b)) for a in alpha for b in beta]
    return tier0_dense_h_dets(norb, dets, h, eri, e_core)


def tier0_dense_h_dets(norb, dets, h, eri, e_core) -> np.ndarray:
    """tier0_dense_h over an explicit list of determinants (alpha string,
    beta string), in the given order: row/column i is determinant dets[i]."""
    N = len(dets)
    full = np.array([int(a) | (int(b) << norb) for a, b in dets], dtype=np.int64)
    order = np.argsort(full)
    sorted_full = full[order]
    H = np.zeros((N, N))
    H[np.arange(N), np.arange(N)] += e_core

    def scatter(st, ph, coef):
        nz = ph != 0
        if not np.any(nz):
            return
        cols = np.nonzero(nz)[0]
        pos = np.searchsorted(sorted_full, st[nz])
        pos = np.minimum(pos, N - 1)
        hit = sorted_full[pos] == st[nz]
        rows = order[pos[hit]]
        np.add.at(H, (rows, cols[hit]), coef * ph[nz][hit])

    ones = np.ones(N, dtype=np.int64)
    for s in (0, 1):
        for p in range(norb):
            for q in range(norb):
                if h[p, q] == 0.0:
                    continue
                st, ph = _annihilate(full, ones, q + s * norb)
                st, ph = _create(st, ph, p + s * norb)
                scatter(st, ph, h[p, q])
    for s in (0, 1):
        for t in (0, 1):
            for p in range(norb):
                for q in range(norb):
                    for r in range(norb):
                        for u in range(norb):
                            g = eri[p, q, r, u]
                            if g == 0.0:
                                continue
                            st, ph = _annihilate(full, ones, q + s * norb)
                            st, ph = _annihilate(st, ph, u + t * norb)
                            st, ph = _create(st, ph, r + t * norb)
                            st, ph = _create(st, ph, p + s * norb)
                            scatter(st, ph, 0.5 * g)
    return H


# ---------------------------------------------------------------------------
# Tier 2: Davidson (Sec. II-C) and dense reference
# ---------------------------------------------------------------------------

@dataclass
class DavidsonResult:
    energies: np.ndarray
    vectors: np.ndarray            # (nroots, N)
    residuals: np.ndarray
    iterations: int
    converged: bool
    history: list = field(default_factory=list)   # per iteration: thetas, |r|, |dtheta|, ortho loss


def damped_inverse(diag: np.ndarray, theta: float, delta: float) -> np.ndarray:
    """1 / (sign(d) max(|d|, delta)) with d = H_ii - theta and sign(0) = +1 (Eq. 7)."""
    d = diag - theta
    sgn = np.where(d >= 0.0, 1.0, -1.0)
    return 1.0 / (sgn * np.maximum(np.abs(d), delta))


def davidson(apply_h, diag: np.ndarray, nroots: int = 1, tol: float = 1e-6,
             max_space: int = 20, max_iter: int = 200, delta: float = 1e-8,
             guess: np.ndarray | None = None, restart_keep: int | None = None) -> DavidsonResult:
    """Lowest ``nroots`` eigenpairs of H by the Davidson method (Sec. II-C).

    apply_h(X) returns H X for X of shape (k, N).  Steps per iteration, in the
    paper's order: w_j = H v_j for new basis vectors; T = V^T W; smallest
    Ritz pairs (theta, y) of T; u = V y and r = H u - theta u = W y - theta u;
    stop when every ||r||_2 <= tol; t = damped (D - theta I)^-1 r (Eqs. 6-7);
    orthogonalise t against the subspace by modified Gram-Schmidt with one
    re-orthogonalisation pass and append it; restart by collapsing onto the
    current lowest Ritz vectors when the subspace is full.
    """
    N = diag.size
    nroots = int(nroots)
    if not (1 <= nroots <= N):
        raise ValueError("need 1 <= nroots <= N")
    max_space = max(max_space, 2 * nroots + 1)
    keep = restart_keep if restart_keep is not None else min(2 * nroots, max_space - nroots)
    if guess is None:
        # unit vectors on the lowest diagonal entries (ties -> lowest index)
        idx = np.argsort(diag, kind="stable")[:nroots]
        V = np.zeros((nroots, N))
        V[np.arange(nroots), idx] = 1.0
    else:
        V = np.array(guess, dtype=np.float64).reshape(-1, N)
        V = _orthonormal_rows(V)
    W = apply_h(V)
    hist = []
    theta_prev = None
    conv = np.zeros(nroots, dtype=bool)
    it = 0
    while True:
        it += 1
        T = V @ W.T
        T = 0.5 * (T + T.T)
        evals, evecs = np.linalg.eigh(T)
        theta = evals[:nroots]
        Y = evecs[:, :nroots]
        U = Y.T @ V
        R = Y.T @ W - theta[:, None] * U
        rn = np.linalg.norm(R, axis=1)
        ortho = float(np.linalg.norm(V @ V.T - np.eye(V.shape[0])))
        dth = np.abs(theta - theta_prev) if theta_prev is not None else np.full(nroots, np.inf)
        hist.append(dict(theta=theta.copy(), rnorm=rn.copy(), dtheta=dth, ortho=ortho, m=V.shape[0]))
        theta_prev = theta.copy()
        conv = rn <= tol
        if np.all(conv) or it >= max_iter:
            return DavidsonResult(theta.copy(), U, rn, it, bool(np.all(conv)), hist)
        new = []
        for k in range(nroots):
            if conv[k]:
                continue
            t = R[k] * damped_inverse(diag, theta[k], delta)
            new.append(t)
        if V.shape[0] + len(new) > max_space:
            # restart: collapse onto the lowest Ritz vectors (no new sigma needed)
            Yk = evecs[:, :keep]
            V = Yk.T @ V
            W = Yk.T @ W
            V, W = _reorth_pair(V, W)
        added = []
        for t in new:
            t = t.copy()
            n0 = np.linalg.norm(t)
            for _ in range(2):                      # MGS + one re-orthogonalisation
                for v in V:
                    t -= (v @ t) * v
                for v in added:
                    t -= (v @ t) * v
            n1 = np.linalg.norm(t)
            if n1 <= 1e-12 * max(n0, 1e-300):
                continue
            added.append(t / n1)
        if not added:
            return DavidsonResult(theta.copy(), U, rn, it, bool(np.all(conv)), hist)
        A = np.array(added)
        V = np.vstack([V, A])
        W = np.vstack([W, apply_h(A)])


def _orthonormal_rows(V):
    out = []
    for v in V:
        v = v.copy()
        for _ in range(2):
            for u in out:
                v -= (u @ v) * u
        nv = np.linalg.norm(v)
        if nv > 1e-12:
            out.append(v / nv)
    return np.array(out)


def _reorth_pair(V, W):
    # V rows are orthonormal up to rounding after a collapse; keep W consistent
    G = V @ V.T
    L = np.linalg.cholesky(G)
    Li = np.linalg.inv(L)
    return Li @ V, Li @ W


def map_vector(alpha_from, beta_from, alpha_to, beta_to, x: np.ndarray) -> np.ndarray:
    """Coefficients of x (over the determinants alpha_from x beta_from,
    alpha-major) on the determinants alpha_to x beta_to: the coefficient of the
    same determinant where it exists in the old basis, else 0.  All string
    arrays sorted ascending and unique.  x may hold several vectors as rows."""
    af, bf = np.asarray(alpha_from, np.uint64), np.asarray(beta_from, np.uint64)
    at, bt = np.asarray(alpha_to, np.uint64), np.asarray(beta_to, np.uint64)
    X = np.atleast_2d(np.asarray(x, np.float64)).reshape(-1, af.size, bf.size)
    ia = np.searchsorted(af, at)
    ib = np.searchsorted(bf, bt)
    a_ok = (ia < af.size) & (af[np.minimum(ia, max(af.size - 1, 0))] == at) if af.size else np.zeros(at.size, bool)
    b_ok = (ib < bf.size) & (bf[np.minimum(ib, max(bf.size - 1, 0))] == bt) if bf.size else np.zeros(bt.size, bool)
    Y = np.zeros((X.shape[0], at.size, bt.size))
    ra, rb = np.nonzero(a_ok)[0], np.nonzero(b_ok)[0]
    Y[:, ra[:, None], rb[None, :]] = X[:, ia[ra][:, None], ib[rb][None, :]]
    return Y.reshape(X.shape[0], -1) if np.ndim(x) > 1 else Y.reshape(-1)


def dense_lowest(Hd: np.ndarray, nroots: int = 1):
    w, v = np.linalg.eigh(Hd)
    return w[:nroots], v[:, :nroots].T
