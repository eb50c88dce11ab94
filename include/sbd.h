/*
 * sbd.h - C ABI of the MI355X (gfx950) selected-basis diagonalisation library.
 *
 * The library computes, on one AMD GPU, the lowest eigenpairs of the
 * electronic Hamiltonian restricted to a selected determinant basis (paper
 * Sec. II, Eqs. 1-2).  The basis is the Cartesian product of a set of alpha
 * and a set of beta occupation bitstrings ("half-bitstrings", Sec. II-B);
 * determinant (ia, ib) has index ia * n_beta_str + ib where ia/ib index the
 * SORTED string lists (Sec. III-B, task loop).  The Hamiltonian is given by
 * one-electron integrals h_pq, two-electron integrals (pq|rs) and a core
 * energy (Eq. 3).
 *
 * Conventions used by every entry point
 *   - Bit p of a uint64 string is spatial orbital p (bit 0 = orbital 0), so
 *     1 <= norb <= 64.  A string for spin s must have exactly n_s bits set,
 *     all below norb.
 *   - (pq|rs) is the chemists' two-electron integral stored at
 *     ((p*norb + q)*norb + r)*norb + s; it must have the 8-fold symmetry
 *     (pq|rs) = (qp|rs) = (pq|sr) = (rs|pq).  The two-body operator is
 *     1/2 sum (pq|rs) a+_p a+_r a_s a_q with spin conserved within (pq) and
 *     within (rs).  h is norb x norb row-major and symmetric.
 *   - A determinant is (alpha creators, ascending)(beta creators, ascending)
 *     acting on the vacuum; this fixes the signs of the vector components.
 *   - All functions return an int status: 0 (SBD_OK), a positive warning or a
 *     negative error.  On error nothing is written to outputs and a message
 *     is available from sbd_last_error() on the calling thread.  Argument
 *     validation happens on the host before any device work.
 *   - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is enqueued on it; calls that return host data synchronise
 *     it before returning.
 *   - Handles are created by the library, are immutable after creation, may
 *     be used from several streams at once, and are released with the
 *     matching sbd_free_* call.  Host input arrays are borrowed only for the
 *     duration of the call (the library copies them).  Device vectors passed
 *     to sbd_sigma / sbd_davidson are owned by the caller, contiguous, and
 *     8-byte aligned (16-byte recommended).
 */
#ifndef SBD_H
#define SBD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SBD_OK = 0,
    SBD_NOT_CONVERGED = 1,   /* warning: outputs valid, residual above tolerance after max_iter */
    SBD_ERR_ARG = -1,        /* null pointer, negative size, nroots > N, bad option value        */
    SBD_ERR_NORB = -2,       /* norb < 1 or norb > 64                                            */
    SBD_ERR_STRING = -3,     /* popcount != n_spin, or a bit at or above norb is set             */
    SBD_ERR_INTEGRALS = -4,  /* h not symmetric or (pq|rs) not 8-fold symmetric (1e-10 relative) */
    SBD_ERR_NOMEM = -5,      /* device allocation failed or exceeds the allowed budget           */
    SBD_ERR_HIP = -6,        /* HIP runtime error; the message carries hipGetErrorString          */
    SBD_ERR_NUMERIC = -7,    /* NaN or Inf met during the computation                            */
    SBD_ERR_STATE = -8       /* handles that do not belong together                              */
} sbd_status;

typedef enum { SBD_FP64 = 0, SBD_FP32 = 1 } sbd_precision;

/* Message of the last failing call on this thread (never NULL). */
const char* sbd_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int sbd_version(void);
/* Hash of the sources the library was built from (16 hex digits); bindings
 * compare it with their own sources to refuse a stale build. */
const char* sbd_source_hash(void);

/*
 * Device memory of the library.  Every device buffer the library owns
 * (handles, sigma workspaces, Davidson subspaces) comes from a per-device
 * cache: a released buffer is kept, after the device has synchronised, and
 * handed out again to a later request of about the same size, so successive
 * solves of one workload do not map and unmap tens of gigabytes each time.
 * Buffers carved from a serving slab are not part of it.
 * sbd_release_cached_memory returns every cached (unused) block of every
 * device to the driver; it synchronises the devices that have cached blocks.
 * sbd_memory_stats reports, for the current device, the bytes held in the
 * cache unused and the bytes handed out to live buffers.
 * Errors: sbd_memory_stats returns SBD_ERR_ARG for a NULL pointer.
 */
int sbd_release_cached_memory(void);
int sbd_memory_stats(size_t* cached_bytes, size_t* in_use_bytes);

typedef struct sbd_basis sbd_basis;
typedef struct sbd_exc sbd_exc;
typedef struct sbd_ham sbd_ham;

/*
 * Selected basis (Sec. II-B half-bitstrings; Sec. III-B bra/ket index layout).
 *   alpha_strings / beta_strings: host arrays of n_*_in strings in any order,
 *   duplicates allowed.  The library validates them (popcount, bits below
 *   norb), sorts each list ascending as unsigned integers and removes
 *   duplicates on the device.  n_*_in >= 1.
 * Errors: SBD_ERR_NORB, SBD_ERR_STRING, SBD_ERR_ARG, SBD_ERR_NOMEM, SBD_ERR_HIP.
 */
int sbd_build_basis(int norb, int n_alpha, int n_beta,
                    const uint64_t* alpha_strings, int64_t n_alpha_in,
                    const uint64_t* beta_strings, int64_t n_beta_in,
                    void* stream, sbd_basis** out);
/* Numbers of unique sorted strings per spin (synchronises the build stream). */
int sbd_basis_sizes(const sbd_basis* b, int64_t* n_alpha_str, int64_t* n_beta_str);
/* Host copies of the sorted unique strings (arrays sized by sbd_basis_sizes). */
int sbd_basis_strings(const sbd_basis* b, uint64_t* alpha_out, uint64_t* beta_out);
void sbd_free_basis(sbd_basis* b);

/*
 * Same-spin excitation tables (Slater-Condon neighbourhoods, Eq. 4; the
 * singles/doubles lists of the task loop in Sec. III-B).  For spin s and
 * bra string I, the single table lists every ket J of the same spin with
 * popcount(I ^ J) == 2, the double table every J with popcount(I ^ J) == 4,
 * as CSR rows sorted by ascending ket index J.  A single records (i, a):
 * i in J\I is annihilated and a in I\J created; a double records (i, j, a, b)
 * with i < j in J\I and a < b in I\J.  sign is the phase of a+_a a_i |J>
 * (single) or a+_a a+_b a_j a_i |J> (double), operators applied right to
 * left.  Built on the device by a wavefront ballot/popcount scan, an
 * exclusive scan of the row counts and a compaction.
 */
int sbd_build_excitations(const sbd_basis* b, void* stream, sbd_exc** out);
/* Number of entries of a table.  spin: 0 alpha, 1 beta; kind: 1 single, 2 double. */
int sbd_exc_count(const sbd_exc* e, int spin, int kind, int64_t* nnz);
/*
 * Host copy of a table: row_ptr[n_str+1] (int64), J[nnz] (int32),
 * orbs[nnz*2*kind] (uint8: (i,a) or (i,j,a,b)), sign[nnz] (int8, +1/-1).
 * Any output pointer may be NULL to skip it.
 */
int sbd_exc_export(const sbd_exc* e, int spin, int kind,
                   int64_t* row_ptr, int32_t* J, uint8_t* orbs, int8_t* sign);
void sbd_free_exc(sbd_exc* e);

/*
 * Hamiltonian on a basis (Eq. 3).  Uploads h and (pq|rs), builds the
 * diagonal H_ii (cached, Sec. II-E) and per-table-entry matrix-element
 * coefficients in FP64 and FP32.  h1: norb*norb host array; eri: norb^4
 * host array; e_core is added to every diagonal element.
 * Errors: SBD_ERR_INTEGRALS (asymmetric input), SBD_ERR_STATE (exc not built
 * from b), SBD_ERR_ARG, SBD_ERR_NOMEM, SBD_ERR_HIP.
 */
int sbd_set_hamiltonian(const sbd_basis* b, const sbd_exc* e,
                        const double* h1, const double* eri, double e_core,
                        void* stream, sbd_ham** out);
/* Copy the FP64 diagonal H_ii (N values) into a caller-owned device buffer. */
int sbd_ham_diag(const sbd_ham* h, double* diag_dev, void* stream);
void sbd_free_ham(sbd_ham* h);

/*
 * Matrix-free sigma = (H - shift I) c (Eq. 4, apply_H of Sec. II-B; the
 * three task types of Sec. III-B: alpha-beta, beta-beta, alpha-alpha).
 *   nvec vectors of N = n_alpha_str * n_beta_str determinants.
 *   prec SBD_FP64: c, sigma are double; SBD_FP32: float, with FP32 gathers
 *   and FP32 accumulation (the diagonal term is formed as (float)(H_ii - shift)).
 *   layout 0: vector v at offset v*N ([v][ia][ib]); layout 1: interleaved,
 *   element (det, v) at det*nvec + v ([ia][ib][v]).
 *   c and sigma are caller-owned device pointers that must not overlap.
 * Each sigma element is produced by one thread in a fixed order: results are
 * bitwise reproducible run to run.
 * A workspace of 2 * N * (layout ? nvec : 1) elements per stream is kept by
 * the Hamiltonian handle (allocated on first use, freed with the handle).
 * Errors: SBD_ERR_ARG (nvec < 1, layout 1 with nvec not in {1, 2, 4, 8},
 * null pointers, c == sigma, bad precision), SBD_ERR_STATE, SBD_ERR_NOMEM,
 * SBD_ERR_HIP.
 */
int sbd_sigma(const sbd_basis* b, const sbd_exc* e, const sbd_ham* h,
              int nvec, int prec, double shift,
              const void* c, void* sigma, int layout, void* stream);

/*
 * sbd_sigma without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, semantics, layouts and results as
 * sbd_sigma (the same kernels and launch configuration, so the output is
 * bitwise that of sbd_sigma); only the workspace differs: a static device
 * array of SBD_NOALLOC_SCRATCH_BYTES that each GPU holds from the first call
 * on it until the process ends.  The call makes no hipMalloc/hipFree and
 * allocates nothing else on the device.
 *   The workspace need is 2 * N * (layout ? nvec : 1) * (8 for FP64, 4 for
 *   FP32) bytes; a larger need fails with SBD_ERR_NOMEM before any device
 *   work.  A handle assembled in prec (sbd_ham_assemble) needs no workspace.
 *   All calls on one device share its array: calls that overlap on one GPU
 *   (other streams or threads) race and must be serialised by the caller;
 *   calls ordered on one stream are safe.  The array keeps the last call's
 *   contents; nothing has to be cleared between calls.
 * Errors: those of sbd_sigma; SBD_ERR_NOMEM (workspace above the maximum).
 */
#define SBD_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int sbd_sigma_noalloc(const sbd_basis* b, const sbd_exc* e, const sbd_ham* h,
                      int nvec, int prec, double shift,
                      const void* c, void* sigma, int layout, void* stream);

/*
 * Autotuner of the sigma launch configuration (the schedule of the sigma
 * kernels: rows per wavefront of the same-spin stream kernel, LDS budget of
 * the alpha-beta kernel).  Times a fixed candidate set on scratch vectors of
 * this shape (prec, nvec, layout as in sbd_sigma) and stores the fastest in
 * the Hamiltonian handle for that precision; results are cached per shape for the process, so a
 * second call on the same shape costs nothing.  best_ms (nullable) receives
 * the winner's time per sigma, or -1 when taken from the cache (or when the
 * precision is assembled, see sbd_ham_assemble: then nothing is tuned).  Must not run
 * concurrently with other calls on the same handle.  Sigma results do not
 * depend on the choice beyond floating-point summation order.
 * Errors: SBD_ERR_ARG, SBD_ERR_STATE, SBD_ERR_NOMEM, SBD_ERR_HIP.
 */
int sbd_autotune(const sbd_basis* b, const sbd_exc* e, sbd_ham* h, int prec, int nvec,
                 int layout, void* stream, double* best_ms);
/* Read or set the sigma launch configuration of a handle for one precision
 * (stream_rw in {1, 2}: output rows per wavefront of the stream kernel;
 * ab_lds_bytes in [4096, 1 MiB], capped at the device's LDS per workgroup;
 * stream_wide in {0, 1}: 16-byte instead of 8-byte lane loads in the row
 * streams where the vector width and row alignment allow; stream_split in
 * {1, 2, 4}: ket entries a stream wavefront loads per step, each by 64/split
 * lanes, which narrows the column tile by that factor (needs stream_rw = 1)).
 * A new handle starts at stream_rw 1, ab_lds_bytes 147456, stream_wide 1,
 * stream_split 1 (the autotuner's usual pick).
 * Any output pointer of sbd_get_tune may be NULL.  Errors: SBD_ERR_ARG. */
int sbd_get_tune(const sbd_ham* h, int prec, int* stream_rw, int* ab_lds_bytes, int* stream_wide,
                 int* stream_split);
int sbd_set_tune(sbd_ham* h, int prec, int stream_rw, int ab_lds_bytes, int stream_wide,
                 int stream_split);

/*
 * sbd_sigma with HIP events recorded on `stream` around its five launches;
 * synchronises the stream and writes the elapsed milliseconds of each stage
 * of the first vector to stage_ms[5]: transpose of c, alpha-side row stream
 * (with the diagonal), beta-side row stream, alpha-beta term, transpose-add.
 * Same results and errors as sbd_sigma (plus SBD_ERR_ARG for stage_ms NULL).
 */
int sbd_sigma_timed(const sbd_basis* b, const sbd_exc* e, const sbd_ham* h,
                    int nvec, int prec, double shift, const void* c, void* sigma, int layout,
                    void* stream, double* stage_ms);

/*
 * Explicit realization of H (Sec. II-A): assemble every connected pair of the
 * basis into a CSR matrix owned by the handle (32-bit columns, FP64 values,
 * and FP32 values when requested), built from the same tables and
 * coefficients as the matrix-free sigma.  Row I = (ia, ib) stores the
 * diagonal, the alpha singles and doubles of ia, the beta singles and doubles
 * of ib, then the alpha-single x beta-single pairs; each nonzero H_IJ once.
 * precisions: 1 = FP64, 2 = FP32, 3 = both.  max_bytes (0 = no limit) bounds
 * the device bytes of the matrix; the entry count is known (and written to
 * nnz_out, nullable) before anything large is allocated.  While a precision
 * is assembled, sbd_sigma, sbd_sigma_timed (the product is reported as the
 * alpha-stream stage, the other stages as 0) and sbd_davidson on this handle
 * apply H through the CSR product y = (H - shift) x for that precision, with
 * the same layouts; sbd_ham_release_assembled returns to the matrix-free
 * sigma.  Synchronises the stream.  Not to be called while other calls use
 * the handle.  Errors: SBD_ERR_ARG (null, precisions outside 1..3, 2^31 or
 * more determinants), SBD_ERR_STATE (tables of another basis), SBD_ERR_NOMEM
 * (allocation failed, or larger than max_bytes: the handle is unchanged),
 * SBD_ERR_HIP.
 */
int sbd_ham_assemble(sbd_ham* h, const sbd_exc* e, int precisions, size_t max_bytes, void* stream,
                     int64_t* nnz_out);
int sbd_ham_release_assembled(sbd_ham* h);
/* Stored entries of the assembled matrix (0 if none) and the assembled
 * precisions (bit 0 FP64, bit 1 FP32); either pointer may be NULL. */
int sbd_ham_assembled(const sbd_ham* h, int64_t* nnz, int* precisions);

/*
 * Transfer of vectors between two bases of the same orbital and electron
 * counts, for warm starts of successive solves: an SQD iteration refines the
 * configuration set (Sec. I), and the Davidson start vector is free to choose
 * (Sec. II-C), so the previous eigenvector, carried into the new basis, starts
 * the next solve.  x_to[v][ia][ib] = x_from[v][ja][jb] where alpha string ia
 * of `to` is string ja of `from` and beta string ib of `to` is string jb of
 * `from`; 0 for determinants of `to` absent from `from`.  x_from: nvec device
 * vectors of (from alphas x from betas) doubles, alpha-major, back to back;
 * x_to: nvec device vectors of (to alphas x to betas) doubles, caller-owned,
 * must not overlap x_from.  Values are copied, not rescaled (the copy of a
 * unit vector has norm <= 1).  Synchronises the stream.
 * Errors: SBD_ERR_ARG (null pointer, nvec < 1), SBD_ERR_STATE (different
 * orbital or electron counts), SBD_ERR_NOMEM, SBD_ERR_HIP.
 */
int sbd_map_vectors(const sbd_basis* from, const sbd_basis* to, int nvec, const double* x_from,
                    double* x_to, void* stream);

/*
 * Tall-skinny projection out = A^T X (the Gram-Schmidt / Rayleigh-Ritz
 * projections of the Davidson update, Sec. II-C), one HBM sweep per row group
 * on the FP64 vector units.  A: ma device vectors of N doubles at A + j*N (1 <= ma <= 48);
 * X: k device vectors at X + q*N (1 <= k <= 8).  out: host array of ma*k
 * doubles, out[j*k + q] = A_j . X_q, summed in a fixed order (deterministic).
 * Synchronises the stream.  Errors: SBD_ERR_ARG, SBD_ERR_NOMEM, SBD_ERR_HIP.
 */
int sbd_gram(const double* A, int ma, const double* X, int k, int64_t N, double* out,
             void* stream);

/* Options of sbd_davidson; sbd_davidson_default_opts fills the defaults. */
typedef struct {
    double tol_residual;   /* ||H u - theta u||_2 per root (unit u); default 1e-6                 */
    int max_iter;          /* iterations (subspace expansions); default 200                        */
    int max_space;         /* subspace size before restart; default 20 (>= 2*nroots+1)             */
    double precond_delta;  /* delta of the damped denominators (Eq. 7); default 1e-8 Ha            */
    int sigma_prec;        /* SBD_FP64 (plain) or SBD_FP32 (FP32 sigma + FP64 refinement)          */
    int use_graph;         /* 1: replay each sigma launch sequence (staging, the five sigma
                              launches, restore) from a HIP graph captured on its second use; one
                              graph per (vector count, width, precision) serves every basis row
                              through a device-resident row index.  The solve then runs on a
                              private stream ordered after `stream`                               */
    int use_autotune;      /* 1: run sbd_autotune for the sigma shapes this solve uses             */
    const double* guess;   /* optional device pointer, n_guess x N initial vectors (NULL = none)   */
    int n_guess;
    int verbose;           /* 1: print one line per iteration to stderr                            */
    int block_sigma;       /* 1 (default): the new vectors of an iteration share one interleaved
                              sigma (several roots); 0: one sigma launch sequence per vector      */
    int device_iterations; /* 0 (default): the host takes each iteration's decisions.  n > 0:
                              iterations run device-driven (Ritz pairs by a one-workgroup Jacobi,
                              convergence, restart and acceptance of corrections decided on the
                              device, two Gram-Schmidt passes per correction) in batches of n
                              between host checks; with use_graph each iteration is one replay of
                              a captured HIP graph that serves every subspace size.  When the
                              device stops (convergence, an FP64 refresh of a mixed-precision
                              solve, stagnation) one host iteration handles it.  Needs
                              N <= 2^21 determinants (larger bases stream gigabytes per
                              iteration, where the host's decisions cost nothing), nroots <= 8,
                              max_space >= 2 nroots + 1 and, for several roots, block_sigma;
                              otherwise the host decides every iteration                      */
} sbd_davidson_opts;

typedef struct {
    int iterations;        /* expansions performed                                                  */
    int sigma_calls;       /* sigma applications (vectors)                                          */
    int sigma_calls_fp64;  /* of which in FP64                                                      */
    int converged;         /* 1 if every root met tol_residual                                      */
    int restarts;          /* thick restarts (subspace full)                                        */
    int refinements;       /* SBD_FP32: FP64 refreshes of the Ritz basis                            */
    int reorthogonalisations; /* second Gram-Schmidt passes taken (|t'| < |t|/sqrt(2))              */
    double fp32_error_scale; /* SBD_FP32: calibrated ||sigma32(v) - sigma64(v)|| per unit vector    */
    double residual[64];   /* final ||r||_2 per root                                                */
    double ortho_loss;     /* ||V^T V - I||_F at exit                                               */
    double t_sigma_ms, t_update_ms, t_total_ms;
    double t_workspace_ms; /* acquiring the device workspace (block cache or driver)                */
    double t_autotune_ms;  /* opts.use_autotune: timing the sigma candidates (0 when cached)        */
    int n_history;         /* entries filled in theta_history                                       */
    double theta_history[512]; /* lowest Ritz value per iteration (first 512 iterations)            */
    double time_history_ms[512]; /* wall time since the call started, per iteration                 */
    int device_iterations; /* iterations run device-driven (opts.device_iterations)                 */
    double t_device_ms;    /* wall time of the device-driven batches (their sigma included)         */
} sbd_davidson_report;

void sbd_davidson_default_opts(sbd_davidson_opts* o);

/*
 * Lowest nroots eigenpairs by the Davidson method (Sec. II-C): sigma of new
 * basis vectors, projected matrix T = V^T W, smallest Ritz pairs, residual
 * r = W y - theta V y, damped diagonal preconditioner (Eqs. 6-7),
 * classical Gram-Schmidt against the subspace with a second pass when the
 * first removes more than 1 - 1/sqrt(2) of the norm, restart onto
 * the lowest Ritz vectors at max_space, block variant for several roots.
 * Initial vectors: opts->guess (if any), then unit vectors on the nroots
 * lowest diagonal elements (lowest index on ties), orthonormalised; vectors
 * that depend on earlier ones are dropped.  The unit vectors are added after a
 * guess too, so that a guess lying in a block of H that does not couple to
 * the lowest state (sparse determinant lists) cannot hide it.
 *   energies: host array of nroots (including e_core), ascending.
 *   vectors : optional caller-owned device array nroots x N (FP64, unit norm).
 *   report  : optional host struct.
 * Returns SBD_OK, SBD_NOT_CONVERGED (outputs valid), or an error
 * (SBD_ERR_ARG, SBD_ERR_STATE, SBD_ERR_NOMEM, SBD_ERR_NUMERIC, SBD_ERR_HIP).
 * Workspace (2*max_space + 2*nroots vectors of N doubles, plus FP32 copies
 * in SBD_FP32 mode) is taken from the library's device block cache for the
 * call and returned to it before returning (see sbd_release_cached_memory).
 */
int sbd_davidson(const sbd_basis* b, const sbd_exc* e, const sbd_ham* h, int nroots,
                 const sbd_davidson_opts* opts, double* energies, double* vectors,
                 sbd_davidson_report* report, void* stream);

/* ------------------------------------------------------------------ SQD loop
 * Successive solves of a sample-based quantum diagonalisation run (Sec. I: the
 * classical diagonalisation is repeated as the configuration set is refined).
 * Step s takes the first step_samples[s] sampled configurations (samples:
 * host array of 2 * nsamples words, alpha string then beta string of each
 * sampled determinant, in the order they were drawn, duplicates allowed),
 * forms the selected basis as the Cartesian product of their distinct alpha
 * and beta strings (Sec. II-B; with spin_union, when n_alpha == n_beta, both
 * spins use every sampled string), builds tables and Hamiltonian, and solves
 * for the lowest nroots eigenpairs with sbd_davidson.  With warm_start each
 * step after the first starts from the previous step's eigenvectors carried
 * into the new basis (sbd_map_vectors; Sec. II-C admits any start vector).
 * energies: host, nsteps x nroots (roots beyond a step's N are 0).  steps
 * (nullable): host array of nsteps reports.  step_samples must be
 * non-decreasing, so the bases are nested and the lowest energy cannot rise
 * from one step to the next (variational principle).  With recovery, the
 * samples of a step are first filtered (Sec. I: the sampled configurations are
 * filtered before the subspace is formed) by sbd_recover_configurations: at
 * the first step samples with a wrong electron count are dropped, at later
 * steps they are corrected from the occupations (sbd_occupations) of the
 * previous step's lowest root; the bases are then no longer nested.
 * Errors: SBD_ERR_ARG, SBD_ERR_INTEGRALS, those of the calls it makes.
 */
typedef struct {
    sbd_davidson_opts davidson;  /* per-step solve options (guess must be unset) */
    int warm_start;              /* default 1 */
    int spin_union;              /* default 0 */
    int full_bitstring;          /* default 0.  1: the basis of a step is the set of distinct
                                    sampled determinants (full-bitstring path, Sec. II-F:
                                    sbd_full_build_basis, sbd_full_davidson, transfer by
                                    sbd_full_map_vectors); the step report's n_alpha_str is
                                    then the number of distinct alpha strings and
                                    n_beta_str 0.  Not with spin_union. */
    int recovery;                /* default 0.  1: filter and correct the samples of every
                                    step (see above); product or full-bitstring bases */
    uint64_t recovery_seed;      /* default 0: seed of the recovery's uniforms */
} sbd_sqd_opts;
typedef struct {
    int status;                  /* sbd_davidson status of the step (0 or SBD_NOT_CONVERGED) */
    int warm;                    /* 1 if started from the previous step's vectors */
    int64_t samples;             /* configurations taken in */
    int64_t n_alpha_str, n_beta_str, ndet;
    int iterations, sigma_calls;
    double residual;             /* largest final residual norm */
    double setup_ms, solve_ms;   /* basis, tables, Hamiltonian (+ transfer); Davidson */
    int64_t corrected, dropped;  /* with recovery: samples corrected, samples dropped */
} sbd_sqd_step;
void sbd_sqd_default_opts(sbd_sqd_opts* o);

/*
 * Average occupation of every spin-orbital in a vector over a product basis
 * (the input of the sample recovery below): occ[p] = sum_I |c_I|^2 [alpha
 * orbital p occupied in I] / sum_I |c_I|^2, occ[norb + p] the same for beta.
 * vec: device, N = n_alpha_str * n_beta_str doubles (index ia * nb + ib);
 * occ: host, 2 * norb doubles.  Fixed reduction order (reproducible).
 * Synchronises the stream.  Errors: SBD_ERR_ARG, SBD_ERR_NOMEM, SBD_ERR_HIP.
 */
int sbd_occupations(const sbd_basis* b, const double* vec, double* occ, void* stream);

/*
 * Filtering of sampled configurations before an SQD solve (Sec. I).  samples:
 * host, 2 * nsamples words (alpha string, beta string).  Samples with the
 * right electron counts are copied to out unchanged.  Without occupations
 * (occ null) the others are dropped; with occ (2 * norb values, as
 * sbd_occupations writes them) each wrong spin string is corrected: with w
 * electrons instead of n, |w - n| orbitals are drawn one after another
 * without replacement among the occupied (w > n) or empty (w < n) ones, with
 * probability proportional to the weight of y = |x_p - occ_p| (x_p the
 * sampled bit): delta * y / h for y <= h, delta + (1 - delta)(y - h) / (1 - h)
 * above, h = n / norb, delta = 0.01; and flipped.  Uniform j of sample i, spin
 * s (0 alpha, 1 beta) is the top 53 bits of SplitMix64(seed + (2 i + s) 64 +
 * j) times 2^-53; the orbital is the first, in increasing order, whose
 * cumulative weight exceeds u times the total.  out: host, room for 2 *
 * nsamples words, filled in sample order; *n_out samples written,
 * *n_corrected (nullable) of them corrected.  Host only, no device work.
 * Errors: SBD_ERR_ARG, SBD_ERR_NORB, SBD_ERR_STRING (a bit at or above norb).
 */
int sbd_recover_configurations(int norb, int n_alpha, int n_beta, const uint64_t* samples, int64_t nsamples,
                               const double* occ, uint64_t seed, uint64_t* out, int64_t* n_out,
                               int64_t* n_corrected);
int sbd_sqd_run(int norb, int n_alpha, int n_beta, const double* h1, const double* eri, double e_core,
                const uint64_t* samples, int64_t nsamples, const int64_t* step_samples, int nsteps,
                int nroots, const sbd_sqd_opts* opts, double* energies, sbd_sqd_step* steps, void* stream);

/* ------------------------------------------------------------------ full bitstrings
 * Full-bitstring representation (Sec. II-F "Support for Half- and
 * Full-Bitstring Paths", Sec. III-F "Extension to Full-Bitstring
 * Representations"): the selected basis is an arbitrary list of determinants,
 * not a Cartesian product of alpha and beta strings.  A determinant is one
 * packed spin-orbital string held in two uint64 words, {alpha string, beta
 * string} (alpha orbital p = bit p of word 0, beta orbital p = bit p of word
 * 1); phases follow the same convention as the alpha x beta path (alpha
 * creators, ascending, before beta creators, ascending).  Excitations are
 * generated from the bitstrings by popcounts, bit scans and parities, and
 * matrix elements are formed from them on the fly in every sigma (Eq. 3, the
 * Slater-Condon rules of Eq. 4), with the diagonal cached (Sec. II-E).
 */
typedef struct sbd_fbasis sbd_fbasis;  /* determinant list and its connections */
typedef struct sbd_fham sbd_fham;      /* integrals and diagonal over an sbd_fbasis */

/*
 * Build a determinant list: dets is a host array of 2 * ndet words (alpha,
 * beta per determinant), any order, duplicates allowed; each alpha word must
 * have n_alpha set bits and each beta word n_beta, all below norb.  The list
 * is sorted by (alpha word, beta word) ascending and deduplicated on the
 * device; determinant I of every later call is row I of that order.  The
 * connections of each determinant (the others that differ from it by one or
 * two electrons, Eq. 4) are built too: CSR rows sorted by ket index.
 * Errors: SBD_ERR_NORB, SBD_ERR_ARG (ndet < 1, ndet > 2^30, bad counts),
 * SBD_ERR_STRING, SBD_ERR_NOMEM, SBD_ERR_HIP.
 */
int sbd_full_build_basis(int norb, int n_alpha, int n_beta, const uint64_t* dets, int64_t ndet,
                         void* stream, sbd_fbasis** out);
/* Unique determinants, stored connections (each ordered pair once) and
 * distinct alpha strings of a list; each pointer nullable. */
int sbd_full_basis_sizes(const sbd_fbasis* b, int64_t* ndet, int64_t* nconn, int64_t* nalpha);
/* Host copies (each nullable): the sorted determinants (2 * ndet words), the
 * connection row pointers (ndet + 1), kets (nconn) and electrons moved (1 or
 * 2 per connection). */
int sbd_full_basis_export(const sbd_fbasis* b, uint64_t* dets, int64_t* row_ptr, int32_t* J, int8_t* deg);
void sbd_free_full_basis(sbd_fbasis* b);

/*
 * Hamiltonian over a determinant list (Eq. 3): h1 norb*norb and eri norb^4
 * host arrays as in sbd_set_hamiltonian, e_core added to every diagonal
 * element.  Uploads the integrals, derives the single-excitation spectator
 * tables (ai|kk), (ak|ki), the antisymmetrised same-spin double elements
 * (ai|bj) - (aj|bi) over orbital pairs a < b, i < j (8 (norb(norb-1)/2)^2
 * bytes), and caches the FP64 diagonal H_II (Sec. II-E).
 * Errors: SBD_ERR_INTEGRALS, SBD_ERR_ARG, SBD_ERR_NOMEM, SBD_ERR_HIP.
 */
int sbd_full_set_hamiltonian(const sbd_fbasis* b, const double* h1, const double* eri, double e_core,
                             void* stream, sbd_fham** out);
/* Copy the FP64 diagonal H_II (ndet values) into a caller-owned device buffer. */
int sbd_full_ham_diag(const sbd_fham* h, double* diag_dev, void* stream);
void sbd_free_full_ham(sbd_fham* h);

/*
 * sigma = (H - shift I) c over a determinant list (apply_H of Sec. II-B over
 * the full-bitstring path).  nvec, prec, layout and ownership as in
 * sbd_sigma, N = ndet.  Every connection's element is formed in FP64 from the
 * two bitstrings; in SBD_FP32 it is rounded once to FP32 and the gathers and
 * accumulation are FP32.  A fixed group of lanes per row (8 to 64, from the
 * list's mean row length) sums in a fixed order: results are bitwise
 * reproducible.  No workspace.
 * Errors: SBD_ERR_ARG, SBD_ERR_STATE (h built on another list), SBD_ERR_HIP.
 */
int sbd_full_sigma(const sbd_fbasis* b, const sbd_fham* h, int nvec, int prec, double shift,
                   const void* c, void* sigma, int layout, void* stream);
/*
 * Lowest nroots eigenpairs over a determinant list (Eq. 2): the Davidson
 * iteration of sbd_davidson (same options, report and outputs, vectors
 * nroots x ndet) with sbd_full_sigma as its sigma.  use_autotune has no
 * effect (the full-bitstring sigma has one launch configuration).
 */
int sbd_full_davidson(const sbd_fbasis* b, const sbd_fham* h, int nroots, const sbd_davidson_opts* opts,
                      double* energies, double* vectors, sbd_davidson_report* report, void* stream);

/*
 * Carry nvec FP64 vectors from one determinant list to another (the
 * full-bitstring counterpart of sbd_map_vectors, for successive solves of an
 * SQD run, Sec. I): x_to[v][i] = x_from[v][j] where determinant j of `from`
 * equals determinant i of `to`, else 0.  Vectors row-major, nvec x ndet of
 * each list, device pointers; the lists must have the same orbital and
 * electron counts.  Asynchronous on stream.  Errors: SBD_ERR_ARG, SBD_ERR_HIP.
 */
int sbd_full_map_vectors(const sbd_fbasis* from, const sbd_fbasis* to, int nvec, const double* x_from,
                         double* x_to, void* stream);
/* Spin-orbital occupations of a vector over a determinant list, as
 * sbd_occupations (vec: device, ndet doubles in the list's order; occ: host,
 * 2 * norb).  Synchronises the stream.  Errors: SBD_ERR_ARG, SBD_ERR_NOMEM,
 * SBD_ERR_HIP. */
int sbd_full_occupations(const sbd_fbasis* b, const double* vec, double* occ, void* stream);

/*
 * Explicit realization over a determinant list (Sec. II-A for the list of
 * Sec. II-F): the element of every stored connection of b, formed once by the
 * evaluation sbd_full_sigma uses and kept with h in the connection order
 * (FP64 and, when requested, its FP32 rounding: 8 and 4 bytes per connection;
 * the diagonal stays the cached FP64 H_II).  precisions: 1 = FP64, 2 = FP32,
 * 3 = both.  max_bytes (0 = no limit) bounds the bytes of the elements; a
 * larger need fails with SBD_ERR_NOMEM before any allocation.  While a
 * precision is assembled, sbd_full_sigma and sbd_full_davidson in that
 * precision read the stored elements instead of evaluating them, summing in
 * the same order, so the product is bitwise the matrix-free one.
 * sbd_full_release_assembled returns to the matrix-free product.  Synchronises
 * the stream; a failure leaves h unchanged.  Not to be called while other
 * calls use h.  Errors: SBD_ERR_ARG (null, precisions outside 1..3),
 * SBD_ERR_STATE (h built on another list), SBD_ERR_NOMEM, SBD_ERR_HIP.
 */
int sbd_full_assemble(sbd_fham* h, const sbd_fbasis* b, int precisions, size_t max_bytes, void* stream);
int sbd_full_release_assembled(sbd_fham* h);
/* The assembled precisions of h (bit 0 FP64, bit 1 FP32; 0 = matrix-free). */
int sbd_full_assembled(const sbd_fham* h, int* precisions);

/* ------------------------------------------------------------------ serving
 * Continuous batching of whole solves (one SQD iteration each: the classical
 * diagonalisation that follows every sampling round, Sec. I and Sec. II).
 * A server owns one device slab of hbm_budget_bytes and max_inflight worker
 * threads, each with its own HIP stream (default priority).  A submitted
 * request is copied, queued in arrival order, and admitted when a worker is
 * free and a contiguous region of its estimated size (sbd_serve_estimate) is
 * free in the slab (a later request that fits may pass a head that does not,
 * at most 64 times per head); every device buffer of the request (basis, tables,
 * Hamiltonian, Davidson vectors) is carved from that region, so requests run
 * concurrently on the device with their vectors resident, and no device
 * allocation or free happens on the serving path.  The region returns to the
 * slab after the request's stream has synchronised.  A request's results do
 * not depend on what else runs (every kernel is deterministic and uses only
 * its own region), except through opts.use_autotune, which times launches.
 */
typedef struct sbd_server sbd_server;

typedef struct {
    int norb, n_alpha, n_beta;
    const uint64_t* alpha_strings; /* host, n_alpha_in strings, any order, duplicates allowed */
    int64_t n_alpha_in;
    const uint64_t* beta_strings;  /* host */
    int64_t n_beta_in;
    const double* h1;              /* host, norb*norb */
    const double* eri;             /* host, norb^4, chemists' (pq|rs) */
    double e_core;
    int nroots;                    /* 1..8 */
    sbd_davidson_opts opts;        /* opts.guess must be NULL */
} sbd_request;

typedef struct {
    int status;                    /* status of the solve (or of the first step that failed) */
    char message[256];             /* sbd_last_error() of the worker when status < 0 */
    double energies[8];
    sbd_davidson_report report;
    int64_t ndet;                  /* N of the request's basis */
    double queue_ms;               /* submit -> admission */
    double run_ms;                 /* admission -> result */
    double latency_ms;             /* submit -> result */
    double admit_at_ms, done_at_ms;  /* admission and completion, ms since the server was created */
    size_t region_bytes;           /* reserved for the request */
    size_t peak_bytes;             /* actually carved from the region */
} sbd_result;

/* Upper bound on the device bytes one request needs (its region size).
 * Errors: SBD_ERR_ARG. */
int sbd_serve_estimate(const sbd_request* req, size_t* bytes);
/* Allocates the slab (hbm_budget_bytes) and starts max_inflight (1..64)
 * workers on the current device.  Errors: SBD_ERR_ARG, SBD_ERR_NOMEM, SBD_ERR_HIP. */
int sbd_serve_create(size_t hbm_budget_bytes, int max_inflight, sbd_server** out);
/* Copies the request's host arrays and queues it; *ticket identifies it.
 * Errors: SBD_ERR_ARG (bad request), SBD_ERR_NOMEM (its estimate exceeds the
 * budget, so it could never be admitted), SBD_ERR_STATE (server stopping). */
int sbd_serve_submit(sbd_server* s, const sbd_request* req, uint64_t* ticket);
/* Blocks until the request has finished and moves its result to *out (each
 * ticket can be waited once).  Returns SBD_OK or SBD_ERR_ARG (unknown ticket). */
int sbd_serve_wait(sbd_server* s, uint64_t ticket, sbd_result* out);
/* Finishes the running requests, fails the queued ones (a thread waiting on one
 * receives status SBD_ERR_STATE), joins the workers, waits until every thread
 * inside sbd_serve_wait on this server has returned, and frees the slab.
 * Results not yet waited for are discarded.  No call on the server may start
 * after sbd_serve_destroy has been entered. */
void sbd_serve_destroy(sbd_server* s);

#ifdef __cplusplus
}
#endif
#endif /* SBD_H */
