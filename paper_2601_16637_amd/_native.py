"""ctypes binding of libsbd.so: argument marshalling only.

Every computation runs in the HIP library.  There is no CPU fallback: if the
library is missing, loading raises ``RuntimeError``.  Device buffers are
passed as torch tensors (their ``data_ptr()``) or raw integer addresses;
streams as ``torch.cuda.Stream``, a raw ``hipStream_t`` integer, or None for
torch's current stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SBD_LIB_PATH selects another build of the same sources (the sanitized host build)
LIB_PATH = os.environ.get("SBD_LIB_PATH") or os.path.join(HERE, "libsbd.so")

SBD_OK = 0
SBD_NOT_CONVERGED = 1
FP64, FP32 = 0, 1
STATUS_NAMES = {0: "SBD_OK", 1: "SBD_NOT_CONVERGED", -1: "SBD_ERR_ARG", -2: "SBD_ERR_NORB",
                -3: "SBD_ERR_STRING", -4: "SBD_ERR_INTEGRALS", -5: "SBD_ERR_NOMEM",
                -6: "SBD_ERR_HIP", -7: "SBD_ERR_NUMERIC", -8: "SBD_ERR_STATE"}

# Every symbol include/sbd.h declares.
EXPORTED = ["sbd_last_error", "sbd_version", "sbd_source_hash", "sbd_release_cached_memory",
            "sbd_memory_stats", "sbd_build_basis", "sbd_basis_sizes",
            "sbd_basis_strings", "sbd_free_basis", "sbd_build_excitations", "sbd_exc_count",
            "sbd_exc_export", "sbd_free_exc", "sbd_set_hamiltonian", "sbd_ham_diag",
            "sbd_free_ham", "sbd_sigma", "sbd_sigma_noalloc", "sbd_sigma_timed", "sbd_autotune", "sbd_get_tune", "sbd_set_tune", "sbd_gram", "sbd_map_vectors",
            "sbd_ham_assemble", "sbd_ham_release_assembled", "sbd_ham_assembled",
            "sbd_davidson_default_opts", "sbd_davidson", "sbd_serve_estimate", "sbd_serve_create",
            "sbd_serve_submit", "sbd_serve_wait", "sbd_serve_destroy",
            "sbd_full_build_basis", "sbd_full_basis_sizes", "sbd_full_basis_export", "sbd_free_full_basis",
            "sbd_full_set_hamiltonian", "sbd_full_ham_diag", "sbd_free_full_ham", "sbd_full_sigma",
            "sbd_full_davidson", "sbd_full_map_vectors", "sbd_full_assemble", "sbd_full_release_assembled",
            "sbd_full_assembled",
            "sbd_sqd_default_opts", "sbd_sqd_run", "sbd_occupations", "sbd_full_occupations",
            "sbd_recover_configurations"]


class SBDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class DavidsonOpts(ctypes.Structure):
    _fields_ = [("tol_residual", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("max_space", ctypes.c_int), ("precond_delta", ctypes.c_double),
                ("sigma_prec", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("use_autotune", ctypes.c_int), ("guess", ctypes.c_void_p),
                ("n_guess", ctypes.c_int), ("verbose", ctypes.c_int),
                ("block_sigma", ctypes.c_int), ("device_iterations", ctypes.c_int)]


class DavidsonReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("sigma_calls", ctypes.c_int),
                ("sigma_calls_fp64", ctypes.c_int), ("converged", ctypes.c_int),
                ("restarts", ctypes.c_int), ("refinements", ctypes.c_int),
                ("reorthogonalisations", ctypes.c_int),
                ("fp32_error_scale", ctypes.c_double), ("residual", ctypes.c_double * 64),
                ("ortho_loss", ctypes.c_double), ("t_sigma_ms", ctypes.c_double),
                ("t_update_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("t_workspace_ms", ctypes.c_double), ("t_autotune_ms", ctypes.c_double),
                ("n_history", ctypes.c_int), ("theta_history", ctypes.c_double * 512),
                ("time_history_ms", ctypes.c_double * 512), ("device_iterations", ctypes.c_int),
                ("t_device_ms", ctypes.c_double)]

    def as_dict(self, nroots: int) -> dict:
        n = self.n_history
        return dict(iterations=self.iterations, sigma_calls=self.sigma_calls,
                    sigma_calls_fp64=self.sigma_calls_fp64, converged=bool(self.converged),
                    restarts=self.restarts, refinements=self.refinements,
                    reorthogonalisations=self.reorthogonalisations,
                    fp32_error_scale=self.fp32_error_scale,
                    residual=list(self.residual[:nroots]),
                    ortho_loss=self.ortho_loss, t_sigma_ms=self.t_sigma_ms,
                    t_update_ms=self.t_update_ms, t_total_ms=self.t_total_ms,
                    t_workspace_ms=self.t_workspace_ms, t_autotune_ms=self.t_autotune_ms,
                    theta_history=list(self.theta_history[:n]),
                    time_history_ms=list(self.time_history_ms[:n]),
                    device_iterations=self.device_iterations, t_device_ms=self.t_device_ms)


class SqdOpts(ctypes.Structure):
    _fields_ = [("davidson", DavidsonOpts), ("warm_start", ctypes.c_int), ("spin_union", ctypes.c_int),
                ("full_bitstring", ctypes.c_int), ("recovery", ctypes.c_int), ("recovery_seed", ctypes.c_uint64)]


class SqdStep(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("warm", ctypes.c_int), ("samples", ctypes.c_int64),
                ("n_alpha_str", ctypes.c_int64), ("n_beta_str", ctypes.c_int64), ("ndet", ctypes.c_int64),
                ("iterations", ctypes.c_int), ("sigma_calls", ctypes.c_int), ("residual", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("corrected", ctypes.c_int64), ("dropped", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [("norb", ctypes.c_int), ("n_alpha", ctypes.c_int), ("n_beta", ctypes.c_int),
                ("alpha_strings", ctypes.c_void_p), ("n_alpha_in", ctypes.c_int64),
                ("beta_strings", ctypes.c_void_p), ("n_beta_in", ctypes.c_int64),
                ("h1", ctypes.c_void_p), ("eri", ctypes.c_void_p), ("e_core", ctypes.c_double),
                ("nroots", ctypes.c_int), ("opts", DavidsonOpts)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("message", ctypes.c_char * 256),
                ("energies", ctypes.c_double * 8), ("report", DavidsonReport),
                ("ndet", ctypes.c_int64), ("queue_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("admit_at_ms", ctypes.c_double), ("done_at_ms", ctypes.c_double),
                ("region_bytes", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t)]


_lib = None


def load():
    """Load libsbd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build() or python -m paper_2601_16637_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    L.sbd_source_hash.restype = ctypes.c_char_p
    L.sbd_source_hash.argtypes = []
    from .build import source_hash
    built, here = L.sbd_source_hash().decode(), source_hash()
    if built != here:
        raise RuntimeError(f"{LIB_PATH} was built from other sources (hash {built}, sources "
                           f"{here}): rebuild it (python -m paper_2601_16637_amd.build)")
    P, i32, i64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    L.sbd_last_error.restype = ctypes.c_char_p
    L.sbd_last_error.argtypes = []
    L.sbd_version.restype = i32
    L.sbd_release_cached_memory.argtypes = []
    L.sbd_memory_stats.argtypes = [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    L.sbd_build_basis.argtypes = [i32, i32, i32, P, i64, P, i64, P, PP]
    L.sbd_basis_sizes.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.sbd_basis_strings.argtypes = [P, P, P]
    L.sbd_free_basis.argtypes = [P]
    L.sbd_free_basis.restype = None
    L.sbd_build_excitations.argtypes = [P, P, PP]
    L.sbd_exc_count.argtypes = [P, i32, i32, ctypes.POINTER(i64)]
    L.sbd_exc_export.argtypes = [P, i32, i32, P, P, P, P]
    L.sbd_free_exc.argtypes = [P]
    L.sbd_free_exc.restype = None
    L.sbd_set_hamiltonian.argtypes = [P, P, P, P, d, P, PP]
    L.sbd_ham_diag.argtypes = [P, P, P]
    L.sbd_free_ham.argtypes = [P]
    L.sbd_free_ham.restype = None
    L.sbd_sigma.argtypes = [P, P, P, i32, i32, d, P, P, i32, P]
    L.sbd_sigma_noalloc.argtypes = [P, P, P, i32, i32, d, P, P, i32, P]
    L.sbd_sigma_timed.argtypes = [P, P, P, i32, i32, d, P, P, i32, P, P]
    L.sbd_autotune.argtypes = [P, P, P, i32, i32, i32, P, ctypes.POINTER(d)]
    L.sbd_get_tune.argtypes = [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                               ctypes.POINTER(i32)]
    L.sbd_set_tune.argtypes = [P, i32, i32, i32, i32, i32]
    L.sbd_gram.argtypes = [P, i32, P, i32, i64, P, P]
    L.sbd_map_vectors.argtypes = [P, P, i32, P, P, P]
    L.sbd_ham_assemble.argtypes = [P, P, i32, ctypes.c_size_t, P, ctypes.POINTER(i64)]
    L.sbd_ham_release_assembled.argtypes = [P]
    L.sbd_ham_assembled.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.sbd_davidson_default_opts.argtypes = [ctypes.POINTER(DavidsonOpts)]
    L.sbd_davidson_default_opts.restype = None
    L.sbd_davidson.argtypes = [P, P, P, i32, ctypes.POINTER(DavidsonOpts), P, P,
                               ctypes.POINTER(DavidsonReport), P]
    L.sbd_full_build_basis.argtypes = [i32, i32, i32, P, i64, P, PP]
    L.sbd_full_basis_sizes.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.sbd_full_basis_export.argtypes = [P, P, P, P, P]
    L.sbd_free_full_basis.argtypes = [P]
    L.sbd_full_set_hamiltonian.argtypes = [P, P, P, d, P, PP]
    L.sbd_full_ham_diag.argtypes = [P, P, P]
    L.sbd_free_full_ham.argtypes = [P]
    L.sbd_full_sigma.argtypes = [P, P, i32, i32, d, P, P, i32, P]
    L.sbd_full_davidson.argtypes = [P, P, i32, ctypes.POINTER(DavidsonOpts), P, P,
                                    ctypes.POINTER(DavidsonReport), P]
    L.sbd_full_map_vectors.argtypes = [P, P, i32, P, P, P]
    L.sbd_full_assemble.argtypes = [P, P, i32, ctypes.c_size_t, P]
    L.sbd_full_release_assembled.argtypes = [P]
    L.sbd_full_assembled.argtypes = [P, ctypes.POINTER(i32)]
    L.sbd_sqd_default_opts.argtypes = [ctypes.POINTER(SqdOpts)]
    L.sbd_sqd_default_opts.restype = None
    L.sbd_sqd_run.argtypes = [i32, i32, i32, P, P, d, P, i64, P, i32, i32, ctypes.POINTER(SqdOpts), P,
                              ctypes.POINTER(SqdStep), P]
    L.sbd_serve_estimate.argtypes = [ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_size_t)]
    L.sbd_serve_create.argtypes = [ctypes.c_size_t, i32, PP]
    L.sbd_serve_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.sbd_serve_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result)]
    L.sbd_serve_destroy.argtypes = [P]
    L.sbd_serve_destroy.restype = None
    for name in EXPORTED:
        if name not in ("sbd_last_error", "sbd_version", "sbd_source_hash", "sbd_free_basis",
                        "sbd_free_exc",
                        "sbd_free_ham", "sbd_davidson_default_opts", "sbd_serve_destroy"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def last_error() -> str:
    return load().sbd_last_error().decode()


def check(status: int) -> int:
    if status < 0:
        raise SBDError(status, last_error())
    return status


def release_cached_memory() -> None:
    """Return the library's cached device blocks to the driver."""
    check(load().sbd_release_cached_memory())


def memory_stats() -> dict:
    """Bytes of the current device held by the library's block cache."""
    c, u = ctypes.c_size_t(), ctypes.c_size_t()
    check(load().sbd_memory_stats(ctypes.byref(c), ctypes.byref(u)))
    return dict(cached_bytes=c.value, in_use_bytes=u.value)


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return ctypes.c_void_p(x)
    return ctypes.c_void_p(x.data_ptr())


def _host(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Basis:
    """Selected alpha x beta basis (sbd_build_basis)."""

    def __init__(self, norb, n_alpha, n_beta, alpha, beta, stream=None):
        L = load()
        a = np.ascontiguousarray(alpha, dtype=np.uint64)
        b = np.ascontiguousarray(beta, dtype=np.uint64)
        h = ctypes.c_void_p()
        check(L.sbd_build_basis(int(norb), int(n_alpha), int(n_beta), _host(a), a.size,
                                _host(b), b.size, _stream(stream), ctypes.byref(h)))
        self._h = h
        self.norb, self.n_alpha, self.n_beta = int(norb), int(n_alpha), int(n_beta)
        na, nb = ctypes.c_int64(), ctypes.c_int64()
        check(L.sbd_basis_sizes(h, ctypes.byref(na), ctypes.byref(nb)))
        self.na, self.nb = na.value, nb.value
        self.N = self.na * self.nb

    def strings(self):
        a = np.zeros(self.na, dtype=np.uint64)
        b = np.zeros(self.nb, dtype=np.uint64)
        check(load().sbd_basis_strings(self._h, _host(a), _host(b)))
        return a, b

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.sbd_free_basis(self._h)
            self._h = None


class Excitations:
    """Same-spin single/double excitation tables (sbd_build_excitations)."""

    def __init__(self, basis: Basis, stream=None):
        self.basis = basis
        h = ctypes.c_void_p()
        check(load().sbd_build_excitations(basis._h, _stream(stream), ctypes.byref(h)))
        self._h = h

    def count(self, spin: int, kind: int) -> int:
        n = ctypes.c_int64()
        check(load().sbd_exc_count(self._h, spin, kind, ctypes.byref(n)))
        return n.value

    def export(self, spin: int, kind: int):
        nstr = self.basis.na if spin == 0 else self.basis.nb
        nnz = self.count(spin, kind)
        rp = np.zeros(nstr + 1, dtype=np.int64)
        J = np.zeros(max(nnz, 1), dtype=np.int32)
        orbs = np.zeros((max(nnz, 1), 2 * kind), dtype=np.uint8)
        sign = np.zeros(max(nnz, 1), dtype=np.int8)
        check(load().sbd_exc_export(self._h, spin, kind, _host(rp), _host(J), _host(orbs),
                                    _host(sign)))
        return rp, J[:nnz], orbs[:nnz], sign[:nnz]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.sbd_free_exc(self._h)
            self._h = None


class Hamiltonian:
    """Integrals, cached diagonal and per-entry coefficients (sbd_set_hamiltonian)."""

    def __init__(self, basis: Basis, exc: Excitations, h1, eri, e_core, stream=None):
        self.basis, self.exc = basis, exc
        h1 = np.ascontiguousarray(h1, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        n = basis.norb
        if h1.size != n * n or eri.size != n ** 4:
            raise ValueError("integral arrays have the wrong size for norb")
        h = ctypes.c_void_p()
        check(load().sbd_set_hamiltonian(basis._h, exc._h, _host(h1), _host(eri),
                                         float(e_core), _stream(stream), ctypes.byref(h)))
        self._h = h

    def autotune(self, prec: int = FP64, nvec: int = 1, layout: int = 0, stream=None) -> float:
        """Pick the fastest sigma launch configuration for this shape (sbd_autotune)."""
        ms = ctypes.c_double()
        check(load().sbd_autotune(self.basis._h, self.exc._h, self._h, int(prec), int(nvec),
                                  int(layout), _stream(stream), ctypes.byref(ms)))
        return ms.value

    def assemble(self, precisions: int = 3, max_bytes: int = 0, stream=None) -> int:
        """Explicit CSR realization of H (sbd_ham_assemble); returns the stored
        entries.  precisions: 1 FP64, 2 FP32, 3 both."""
        nnz = ctypes.c_int64()
        check(load().sbd_ham_assemble(self._h, self.exc._h, int(precisions), int(max_bytes), _stream(stream),
                                      ctypes.byref(nnz)))
        return nnz.value

    def release_assembled(self):
        check(load().sbd_ham_release_assembled(self._h))

    def assembled(self):
        """(stored entries, precision bits) of the assembled matrix (sbd_ham_assembled)."""
        nnz, pr = ctypes.c_int64(), ctypes.c_int()
        check(load().sbd_ham_assembled(self._h, ctypes.byref(nnz), ctypes.byref(pr)))
        return nnz.value, pr.value

    def get_tune(self, prec: int = FP64):
        rw, lds, wide, split = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(load().sbd_get_tune(self._h, int(prec), ctypes.byref(rw), ctypes.byref(lds),
                                  ctypes.byref(wide), ctypes.byref(split)))
        return dict(stream_rw=rw.value, ab_lds_bytes=lds.value, stream_wide=wide.value,
                    stream_split=split.value)

    def set_tune(self, prec: int = FP64, stream_rw: int = 1, ab_lds_bytes: int = 147456,
                 stream_wide: int = 1, stream_split: int = 1):
        check(load().sbd_set_tune(self._h, int(prec), int(stream_rw), int(ab_lds_bytes),
                                  int(stream_wide), int(stream_split)))

    def diag_into(self, out, stream=None):
        check(load().sbd_ham_diag(self._h, _dptr(out), _stream(stream)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.sbd_free_ham(self._h)
            self._h = None


def sigma(ham: Hamiltonian, c, out, nvec: int = 1, prec: int = FP64, shift: float = 0.0,
          layout: int = 0, stream=None):
    """out = (H - shift) c on device buffers (sbd_sigma)."""
    check(load().sbd_sigma(ham.basis._h, ham.exc._h, ham._h, int(nvec), int(prec), float(shift),
                           _dptr(c), _dptr(out), int(layout), _stream(stream)))
    return out


def sigma_noalloc(ham: Hamiltonian, c, out, nvec: int = 1, prec: int = FP64, shift: float = 0.0,
                  layout: int = 0, stream=None):
    """out = (H - shift) c with the workspace in the library's static device
    scratch instead of a handle-owned buffer (sbd_sigma_noalloc)."""
    check(load().sbd_sigma_noalloc(ham.basis._h, ham.exc._h, ham._h, int(nvec), int(prec), float(shift),
                                   _dptr(c), _dptr(out), int(layout), _stream(stream)))
    return out


SIGMA_STAGES = ("transpose", "alpha_stream", "beta_stream", "alpha_beta", "transpose_add")


def sigma_timed(ham: Hamiltonian, c, out, nvec: int = 1, prec: int = FP64, shift: float = 0.0,
                layout: int = 0, stream=None) -> dict:
    """sigma with HIP-event timing of its five launches (sbd_sigma_timed); returns ms per stage."""
    ms = np.zeros(5, dtype=np.float64)
    check(load().sbd_sigma_timed(ham.basis._h, ham.exc._h, ham._h, int(nvec), int(prec),
                                 float(shift), _dptr(c), _dptr(out), int(layout),
                                 _stream(stream), _host(ms)))
    return dict(zip(SIGMA_STAGES, ms.tolist()))


def map_vectors(basis_from: "Basis", basis_to: "Basis", x_from, x_to, nvec: int = 1, stream=None):
    """Carry nvec FP64 device vectors from one basis into another (sbd_map_vectors):
    determinants absent from basis_from get 0."""
    check(load().sbd_map_vectors(basis_from._h, basis_to._h, int(nvec), _dptr(x_from), _dptr(x_to),
                                 _stream(stream)))


def occupations(basis: "Basis", vec, stream=None) -> tuple:
    """Spin-orbital occupations of an FP64 device vector over a product basis
    (sbd_occupations): (alpha occupations, beta occupations), norb each."""
    occ = np.zeros(2 * basis.norb, dtype=np.float64)
    check(load().sbd_occupations(basis._h, _dptr(vec), _host(occ), _stream(stream)))
    return occ[:basis.norb].copy(), occ[basis.norb:].copy()


def full_occupations(basis: "FullBasis", vec, stream=None) -> tuple:
    """Spin-orbital occupations of an FP64 device vector over a determinant
    list (sbd_full_occupations): (alpha occupations, beta occupations)."""
    occ = np.zeros(2 * basis.norb, dtype=np.float64)
    check(load().sbd_full_occupations(basis._h, _dptr(vec), _host(occ), _stream(stream)))
    return occ[:basis.norb].copy(), occ[basis.norb:].copy()


def recover_configurations(norb, n_alpha, n_beta, samples, occ_alpha=None, occ_beta=None, seed: int = 0):
    """Samples (rows: alpha string, beta string) filtered and corrected
    (sbd_recover_configurations); returns (samples out, number corrected)."""
    smp = np.ascontiguousarray(np.asarray(samples, dtype=np.uint64).reshape(-1, 2))
    out = np.zeros_like(smp)
    occ = None
    if occ_alpha is not None:
        occ = np.ascontiguousarray(np.concatenate([np.asarray(occ_alpha, dtype=np.float64),
                                                   np.asarray(occ_beta, dtype=np.float64)]))
    n_out, n_corr = ctypes.c_int64(), ctypes.c_int64()
    check(load().sbd_recover_configurations(int(norb), int(n_alpha), int(n_beta), _host(smp), smp.shape[0],
                                            _host(occ) if occ is not None else None, ctypes.c_uint64(int(seed)),
                                            _host(out), ctypes.byref(n_out), ctypes.byref(n_corr)))
    return out[:n_out.value].copy(), n_corr.value


def gram(A, ma: int, X, k: int, N: int, stream=None) -> np.ndarray:
    """A^T X for device row blocks (sbd_gram): returns an (ma, k) host array."""
    out = np.zeros((ma, k), dtype=np.float64)
    check(load().sbd_gram(_dptr(A), int(ma), _dptr(X), int(k), int(N), _host(out),
                          _stream(stream)))
    return out


def default_opts() -> DavidsonOpts:
    o = DavidsonOpts()
    load().sbd_davidson_default_opts(ctypes.byref(o))
    return o


def davidson(ham: Hamiltonian, nroots: int = 1, vectors=None, stream=None, **kw):
    """Lowest eigenpairs (sbd_davidson).  Keyword options are DavidsonOpts fields;
    ``guess`` may be a device tensor of shape (n_guess, N).  Returns
    (energies ndarray, report dict, status)."""
    o = default_opts()
    for k, v in kw.items():
        if k == "guess":
            o.guess = _dptr(v).value if v is not None else None
            continue
        if not hasattr(o, k):
            raise TypeError(f"unknown Davidson option {k}")
        setattr(o, k, v)
    e = np.zeros(nroots, dtype=np.float64)
    rep = DavidsonReport()
    st = check(load().sbd_davidson(ham.basis._h, ham.exc._h, ham._h, int(nroots),
                                   ctypes.byref(o), _host(e), _dptr(vectors), ctypes.byref(rep),
                                   _stream(stream)))
    return e, rep.as_dict(nroots), st


class FullBasis:
    """Full-bitstring basis: an arbitrary determinant list (sbd_full_build_basis).
    ``dets`` has one row per determinant: alpha string, beta string."""

    def __init__(self, norb, n_alpha, n_beta, dets, stream=None):
        L = load()
        d = np.ascontiguousarray(np.asarray(dets, dtype=np.uint64).reshape(-1, 2))
        h = ctypes.c_void_p()
        check(L.sbd_full_build_basis(int(norb), int(n_alpha), int(n_beta), _host(d), d.shape[0],
                                     _stream(stream), ctypes.byref(h)))
        self._h = h
        self.norb, self.n_alpha, self.n_beta = int(norb), int(n_alpha), int(n_beta)
        n, c, g = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(L.sbd_full_basis_sizes(h, ctypes.byref(n), ctypes.byref(c), ctypes.byref(g)))
        self.N, self.nconn, self.nalpha = n.value, c.value, g.value

    def export(self):
        """(sorted determinants (N, 2), row_ptr, J, electrons moved) on the host."""
        d = np.zeros((self.N, 2), dtype=np.uint64)
        rp = np.zeros(self.N + 1, dtype=np.int64)
        J = np.zeros(max(self.nconn, 1), dtype=np.int32)
        deg = np.zeros(max(self.nconn, 1), dtype=np.int8)
        check(load().sbd_full_basis_export(self._h, _host(d), _host(rp), _host(J), _host(deg)))
        return d, rp, J[:self.nconn], deg[:self.nconn]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.sbd_free_full_basis(self._h)
            self._h = None


class FullHamiltonian:
    """Integrals and cached diagonal over a determinant list (sbd_full_set_hamiltonian)."""

    def __init__(self, basis: FullBasis, h1, eri, e_core, stream=None):
        self.basis = basis
        h1 = np.ascontiguousarray(h1, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        n = basis.norb
        if h1.size != n * n or eri.size != n ** 4:
            raise ValueError("integral arrays have the wrong size for norb")
        h = ctypes.c_void_p()
        check(load().sbd_full_set_hamiltonian(basis._h, _host(h1), _host(eri), float(e_core),
                                              _stream(stream), ctypes.byref(h)))
        self._h = h

    def diag_into(self, out, stream=None):
        check(load().sbd_full_ham_diag(self._h, _dptr(out), _stream(stream)))

    def assemble(self, precisions: int = 3, max_bytes: int = 0, stream=None):
        """Keep every connection's element (sbd_full_assemble); precisions: 1 FP64, 2 FP32, 3 both."""
        check(load().sbd_full_assemble(self._h, self.basis._h, int(precisions), int(max_bytes),
                                       _stream(stream)))

    def release_assembled(self):
        check(load().sbd_full_release_assembled(self._h))

    def assembled(self) -> int:
        """Assembled precision bits (sbd_full_assembled): 1 FP64, 2 FP32, 0 none."""
        pr = ctypes.c_int()
        check(load().sbd_full_assembled(self._h, ctypes.byref(pr)))
        return pr.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.sbd_free_full_ham(self._h)
            self._h = None


def full_sigma(ham: FullHamiltonian, c, out, nvec: int = 1, prec: int = FP64, shift: float = 0.0,
               layout: int = 0, stream=None):
    """out = (H - shift) c over a determinant list (sbd_full_sigma)."""
    check(load().sbd_full_sigma(ham.basis._h, ham._h, int(nvec), int(prec), float(shift), _dptr(c),
                                _dptr(out), int(layout), _stream(stream)))
    return out


def full_davidson(ham: FullHamiltonian, nroots: int = 1, vectors=None, stream=None, **kw):
    """Lowest eigenpairs over a determinant list (sbd_full_davidson); options and
    return value as davidson()."""
    o = default_opts()
    for k, v in kw.items():
        if k == "guess":
            o.guess = _dptr(v).value if v is not None else None
            continue
        if not hasattr(o, k):
            raise TypeError(f"unknown Davidson option {k}")
        setattr(o, k, v)
    e = np.zeros(nroots, dtype=np.float64)
    rep = DavidsonReport()
    st = check(load().sbd_full_davidson(ham.basis._h, ham._h, int(nroots), ctypes.byref(o), _host(e),
                                        _dptr(vectors), ctypes.byref(rep), _stream(stream)))
    return e, rep.as_dict(nroots), st


def full_map_vectors(basis_from: "FullBasis", basis_to: "FullBasis", x_from, x_to, nvec: int = 1, stream=None):
    """Carry nvec FP64 device vectors from one determinant list to another
    (sbd_full_map_vectors): determinants absent from basis_from get 0."""
    check(load().sbd_full_map_vectors(basis_from._h, basis_to._h, int(nvec), _dptr(x_from), _dptr(x_to),
                                      _stream(stream)))
    return x_to


def sqd_run(norb, n_alpha, n_beta, h1, eri, e_core, samples, step_samples, nroots: int = 1,
            warm_start: bool = True, spin_union: bool = False, full_bitstring: bool = False,
            recovery: bool = False, recovery_seed: int = 0, stream=None, **kw):
    """Successive solves on a growing set of sampled configurations
    (sbd_sqd_run): step s uses the first step_samples[s] rows of ``samples``
    (alpha string, beta string), filtered and corrected first with
    ``recovery``.  Keyword options are DavidsonOpts fields.
    Returns (energies (nsteps, nroots), list of step reports)."""
    smp = np.ascontiguousarray(np.asarray(samples, dtype=np.uint64).reshape(-1, 2))
    steps_in = np.ascontiguousarray(step_samples, dtype=np.int64)
    h = np.ascontiguousarray(h1, dtype=np.float64)
    g = np.ascontiguousarray(eri, dtype=np.float64)
    if h.size != norb * norb or g.size != norb ** 4:
        raise ValueError("integral arrays have the wrong size for norb")
    o = SqdOpts()
    load().sbd_sqd_default_opts(ctypes.byref(o))
    o.warm_start, o.spin_union = int(bool(warm_start)), int(bool(spin_union))
    o.full_bitstring = int(bool(full_bitstring))
    o.recovery, o.recovery_seed = int(bool(recovery)), int(recovery_seed)
    for k, v in kw.items():
        if not hasattr(o.davidson, k) or k == "guess":
            raise TypeError(f"unknown or unsupported option {k}")
        setattr(o.davidson, k, v)
    ns = steps_in.size
    e = np.zeros((ns, nroots), dtype=np.float64)
    reps = (SqdStep * ns)()
    check(load().sbd_sqd_run(int(norb), int(n_alpha), int(n_beta), _host(h), _host(g), float(e_core), _host(smp),
                             smp.shape[0], _host(steps_in), ns, int(nroots), ctypes.byref(o), _host(e), reps,
                             _stream(stream)))
    return e, [r.as_dict() for r in reps]


def _opts(**kw) -> DavidsonOpts:
    o = default_opts()
    for k, v in kw.items():
        if not hasattr(o, k) or k == "guess":
            raise TypeError(f"unknown or unsupported option {k}")
        setattr(o, k, v)
    return o


def _request(norb, n_alpha, n_beta, alpha, beta, h1, eri, e_core, nroots, **opts):
    a = np.ascontiguousarray(alpha, dtype=np.uint64)
    b = np.ascontiguousarray(beta, dtype=np.uint64)
    h = np.ascontiguousarray(h1, dtype=np.float64)
    g = np.ascontiguousarray(eri, dtype=np.float64)
    if h.size != norb * norb or g.size != norb ** 4:
        raise ValueError("integral arrays have the wrong size for norb")
    q = Request(int(norb), int(n_alpha), int(n_beta), _host(a), a.size, _host(b), b.size,
                _host(h), _host(g), float(e_core), int(nroots), _opts(**opts))
    return q, (a, b, h, g)  # the arrays must outlive the call that reads them


def serve_estimate(norb, n_alpha, n_beta, alpha, beta, h1, eri, e_core, nroots, **opts) -> int:
    """Device bytes a request reserves in a server's slab (sbd_serve_estimate)."""
    q, keep = _request(norb, n_alpha, n_beta, alpha, beta, h1, eri, e_core, nroots, **opts)
    n = ctypes.c_size_t()
    check(load().sbd_serve_estimate(ctypes.byref(q), ctypes.byref(n)))
    return n.value


class Server:
    """Continuous-batching solve server (sbd_serve_*): one HBM slab, several
    worker streams; requests are admitted in arrival order as workers and
    slab space free up."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 4):
        h = ctypes.c_void_p()
        check(load().sbd_serve_create(int(hbm_budget_bytes), int(max_inflight), ctypes.byref(h)))
        self._h = h

    def submit(self, norb, n_alpha, n_beta, alpha, beta, h1, eri, e_core, nroots=1, **opts) -> int:
        q, keep = _request(norb, n_alpha, n_beta, alpha, beta, h1, eri, e_core, nroots, **opts)
        t = ctypes.c_uint64()
        check(load().sbd_serve_submit(self._h, ctypes.byref(q), ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int) -> dict:
        r = Result()
        check(load().sbd_serve_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(r)))
        return dict(status=r.status, message=r.message.decode(errors="replace"),
                    energies=np.array(r.energies[:8]), report=r.report.as_dict(8), ndet=r.ndet,
                    queue_ms=r.queue_ms, run_ms=r.run_ms, latency_ms=r.latency_ms,
                    admit_at_ms=r.admit_at_ms, done_at_ms=r.done_at_ms,
                    region_bytes=r.region_bytes, peak_bytes=r.peak_bytes)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.sbd_serve_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
