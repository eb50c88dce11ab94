// Internal declarations shared by the host core (abi.cpp, davidson.cpp) and
// the HIP kernels (*.hip).  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sbd.h"

namespace sbd {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
// h symmetric and (pq|rs) 8-fold symmetric to 1e-10 relative, all finite
int validate_integrals(int n, const double* h, const double* eri);

#define SBD_HIP(call)                                           \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return ::sbd::hip_fail(e_, #call); \
    } while (0)

// Region of a serving slab that one request allocates from (serve.cpp).  While
// a thread has a region installed, every DevBuf it allocates is carved from the
// region by a bump pointer and released with it when the request has finished
// (after its stream synchronised), so the serving path never calls hipMalloc
// or hipFree, and hipFree's device-wide synchronisation never stalls other
// requests' work.
struct Region {
    char* base = nullptr;
    size_t size = 0;
    size_t used = 0;  // bump pointer
    size_t peak = 0;
};
Region* current_region();

// Caching device allocator (pool.cpp): blocks released by DevBuf are kept per
// device, after a device synchronisation, and reused for requests of about the
// same size; sbd_release_cached_memory() hands them back to the driver.
hipError_t pool_alloc(size_t n, void** out);
void pool_free(void* p);
void pool_stats(size_t* cached, size_t* in_use);
void pool_release_cached();

// Device buffer owned by a handle.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool regional = false;  // carved from a serving region: nothing to free here
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), regional(o.regional) {
        o.p = nullptr;
        o.bytes = 0;
        o.regional = false;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            regional = o.regional;
            o.p = nullptr;
            o.bytes = 0;
            o.regional = false;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    hipError_t alloc(size_t n) {
        release();
        bytes = n;
        if (n == 0) return hipSuccess;
        if (Region* r = current_region()) {
            const size_t off = (r->used + 255) & ~size_t(255);
            if (off + n > r->size) {
                bytes = 0;
                return hipErrorOutOfMemory;
            }
            p = r->base + off;
            r->used = off + n;
            if (r->used > r->peak) r->peak = r->used;
            regional = true;
            return hipSuccess;
        }
        return pool_alloc(n, &p);
    }
    void release() {
        if (p && !regional) pool_free(p);
        p = nullptr;
        bytes = 0;
        regional = false;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------- handles
struct SpinStrings {
    int64_t n = 0;              // unique sorted strings
    DevBuf d;                   // uint64[n]
    std::vector<uint64_t> host; // sorted copy
};

}  // namespace sbd

struct sbd_basis {
    int norb = 0, n_el[2] = {0, 0};
    sbd::SpinStrings s[2];  // 0 alpha, 1 beta
    uint64_t id = 0;        // unique per basis, ties tables/hamiltonians to it
};

namespace sbd {
// One CSR table: row_ptr[n+1], ket index J, packed orbitals, sign.
struct Table {
    int kind = 1;
    int64_t nnz = 0;
    DevBuf row_ptr;  // int64[n+1]
    DevBuf J;        // int32[nnz]
    DevBuf orb;      // uint32[nnz]: i | j<<8 | a<<16 | b<<24 (double); i | a<<8 (single)
    DevBuf sign;     // int8[nnz]
    DevBuf pack;     // singles only: uint64 J | i << 32 | a << 40 | (sign < 0) << 48
    DevBuf sell;     // singles only: pack entries in sliced-ELL order (64-position slices)
    DevBuf sell_off; // int64[nslice+1]: first entry of each slice (slot-major, 64 per slot)
    DevBuf sell_pos; // int32[n]: string held by each sliced-ELL position (see sell_positions)
    int64_t sell_entries = 0;
    // singles only, when the spin has at most 2^18 strings: the sliced-ELL entries
    // in 32 bits, J | (a*norb + i) << 18 | (sign < 0) << 31; padding J = 0,
    // pair index norb*norb (it reads a zero of the staged integral slice)
    DevBuf sell32;
};
}  // namespace sbd

struct sbd_exc {
    uint64_t basis_id = 0;
    int64_t n[2] = {0, 0};
    sbd::Table t[2][2];  // [spin][kind-1]
    uint64_t id = 0;
};

namespace sbd {
// Hamiltonian data per spin: coefficients per table entry and the spectator
// table G[pair(a,i)][string] = sum_{k in string} (ai|kk).
// Launch parameters of the sigma kernels (picked per shape by the autotuner).
struct SigmaTune {
    int ab_threads = 1024;       // threads per alpha-beta workgroup
    // defaults: the configuration the autotuner picks at most measured shapes
    int ab_lds_bytes = 147456;   // LDS budget for the staged row of the alpha-beta kernel
    int stream_rows = 4;         // wavefronts per stream workgroup
    int stream_rw = 1;           // output rows per stream wavefront (1 or 2)
    int stream_wide = 1;         // 1: 16-byte lane loads in the row streams where possible
    int stream_split = 1;        // ket entries per load step of a stream wavefront (1, 2, 4)
    int ab_compact = 1;          // 1: alpha-beta walk over the 32-bit beta entries where built
};

struct SpinCoef {
    DevBuf c1_64, c1_32;  // single base coefficient s*(h_ai + sum_{k in J} ((ai|kk)-(ak|ki)))
    DevBuf ps1;           // int32 per single: pair(a,i) << 1 | (sign < 0)
    DevBuf c2_64, c2_32;  // double coefficient s*((ai|bj) - (aj|bi))
    DevBuf G64, G32;      // spectator table of THIS spin's strings: [npair][n]
    DevBuf dspin;         // double[n]: same-spin diagonal part of each string
};
}  // namespace sbd

struct sbd_ham {
    uint64_t basis_id = 0, exc_id = 0;
    sbd::SigmaTune tune[2];         // sigma launch configuration per precision
    int norb = 0;
    int64_t na = 0, nb = 0;
    double e_core = 0.0;
    double diag_min = 0.0;
    sbd::DevBuf h64, eri64, eri32;  // integrals on device
    sbd::SpinCoef sc[2];
    sbd::DevBuf diag;               // double[N]
    // explicit realization (sbd_ham_assemble): H in CSR, FP64 values and optionally FP32
    sbd::DevBuf csr_rp, csr_col, csr_v64, csr_v32;
    int64_t csr_nnz = 0;
    bool csr_has[2] = {false, false};  // per precision (0 FP64, 1 FP32)
    std::mutex ws_mu;               // per-stream sigma workspaces of sbd_sigma
    std::map<hipStream_t, std::unique_ptr<sbd::DevBuf>> ws;
};

namespace sbd {

inline int pair_index(int a, int i) {  // symmetric pair (a,i) -> triangular index
    int hi = a > i ? a : i, lo = a > i ? i : a;
    return hi * (hi + 1) / 2 + lo;
}
inline int npairs(int norb) { return norb * (norb + 1) / 2; }

// ---------------------------------------------------------------- kernels
// All launchers enqueue on `st` and return hipGetLastError() of the launch.

// Basis: sort ascending and dedupe `n` strings in d_in (device, capacity >= pow2(n)).
// Writes unique strings to d_out, count to d_count (device int64).
hipError_t launch_sort_unique(uint64_t* d_work, int64_t n, uint64_t* d_out, int64_t* d_count,
                              int64_t* d_tmp_i64, hipStream_t st);

// Excitation tables.
hipError_t launch_exc_count(const uint64_t* d_s, int64_t n, int64_t* d_cnt1, int64_t* d_cnt2,
                            hipStream_t st);
// d_out[0] = 0, d_out[i + 1] = d_in[0] + ... + d_in[i] (n + 1 words, not in place).
// d_tmp: scan_tmp_words(n) words of device scratch for the multi-workgroup
// form, or null (one workgroup; slow for long inputs).
int64_t scan_tmp_words(int64_t n);
hipError_t launch_exclusive_scan(const int64_t* d_in, int64_t n, int64_t* d_out /*n+1*/, int64_t* d_tmp,
                                 hipStream_t st);
hipError_t launch_exc_fill(const uint64_t* d_s, int64_t n, const int64_t* rp1, const int64_t* rp2,
                           int32_t* J1, uint32_t* orb1, int8_t* sg1, int32_t* J2, uint32_t* orb2,
                           int8_t* sg2, hipStream_t st);
// 32-bit sliced-ELL entries (Table::sell32) from the 64-bit ones
constexpr int kSellJBits = 18;
hipError_t launch_sell_compact(const uint64_t* sell, int64_t n_entries, int norb, uint32_t* out, hipStream_t st);
hipError_t launch_pack_singles(int64_t nnz, const int32_t* J, const uint32_t* orb, const int8_t* sg,
                               uint64_t* pack, hipStream_t st);
// sliced-ELL: slots[slice] = 64 * longest row of the slice; then fill from the scan
// Sliced-ELL copy of a singles table over positions p < n, position p holding
// string pos[p]: slot count per 64-position slice, then the padded fill.
hipError_t launch_sell_len(const int64_t* rp, const int32_t* pos, int64_t n, int64_t* slots,
                           hipStream_t st);
hipError_t launch_sell_fill(const int64_t* rp, const uint64_t* pack, const int32_t* pos, int64_t n,
                            const int64_t* off, uint64_t* sell, hipStream_t st);
// Threads per workgroup of the alpha-beta kernel for nb beta strings; a thread
// handles the positions lane + q * threads, one per window of `threads` positions.
inline int ab_block_threads(int64_t nb) { return nb > 512 ? 1024 : (nb > 256 ? 512 : 256); }

// Hamiltonian pieces.
hipError_t launch_string_diag(const uint64_t* d_s, int64_t n, int norb, const double* h,
                              const double* eri, double* out, hipStream_t st);
hipError_t launch_spectator(const uint64_t* d_s, int64_t n, int norb, const double* eri,
                            double* G64, float* G32, hipStream_t st);
hipError_t launch_single_coef(const uint64_t* d_s, int64_t nnz, const int32_t* J,
                              const uint32_t* orb, const int8_t* sg, int norb, const double* h,
                              const double* eri, double* c64, float* c32, int32_t* ps,
                              hipStream_t st);
hipError_t launch_double_coef(int64_t nnz, const uint32_t* orb, const int8_t* sg, int norb,
                              const double* eri, double* c64, float* c32, hipStream_t st);
hipError_t launch_full_diag(const uint64_t* d_a, int64_t na, const double* da,
                            const double* db, const double* Gb /*[npair][nb]*/, int64_t nb,
                            int norb, double e_core, double* diag, hipStream_t st);
hipError_t launch_d2f(const double* in, float* out, int64_t n, hipStream_t st);

// Sigma.  Tables and coefficients of both spins, one precision.
template <class T>
struct SigmaArgs {
    int64_t na, nb;
    int norb;
    // alpha tables
    const int64_t* a1p; const int32_t* a1J; const T* a1c; const int32_t* a1ps;
    const uint64_t* a1pack;
    const int64_t* a2p; const int32_t* a2J; const T* a2c;
    // beta tables
    const int64_t* b1p; const int32_t* b1J; const T* b1c; const int32_t* b1ps;
    const uint64_t* b1pack;
    const uint64_t* b1sell; const int64_t* b1sell_off; const int32_t* b1sell_pos;
    const uint32_t* b1sell32;  // null when the compact table is absent
    const int64_t* b2p; const int32_t* b2J; const T* b2c;
    const T* Ga;   // [npair][na]  sum_{k in alpha(ia)} (pair|kk)
    const T* Gb;   // [npair][nb]
    const T* eri;  // norb^4
    const double* diag;
    double shift;
};

// Inputs of the explicit assembly (k_csr.hip): the FP64 tables and coefficients.
struct CsrTables {
    int64_t na, nb;
    int norb;
    const int64_t *a1p, *a2p, *b1p, *b2p;
    const int32_t *a1J, *a2J, *b1J, *b2J;
    const double *a1c, *a2c, *b1c, *b2c;
    const int32_t *a1ps, *b1ps;
    const uint64_t *a1pack, *b1pack;
    const double *Ga, *Gb;
    const double* eri;
    const double* diag;
};
// cnt[I] = stored entries of row I (diagonal included)
hipError_t launch_csr_count(const CsrTables& t, int64_t* cnt, hipStream_t st);
// columns and values of every row at rp[I] (v32 nullable)
hipError_t launch_csr_fill(const CsrTables& t, const int64_t* rp, int32_t* col, double* v64, float* v32,
                           hipStream_t st);
// y = (H - shift) x over the CSR; nv interleaved vectors per determinant (1, 2, 4, 8)
template <class T>
hipError_t launch_spmv(const int64_t* rp, const int32_t* col, const T* val, int64_t N, int nv, double shift,
                       const T* x, T* y, hipStream_t st);

// Workspace bytes needed by launch_sigma for nvec vectors of type T.
size_t sigma_workspace_bytes(int64_t N, int nvec, int layout, size_t elem);
// Argument checks of the sigma entry points (abi.cpp; host only, no device work).
int sigma_validate(const sbd_basis* b, const sbd_exc* x, const sbd_ham* H, int nvec, int prec,
                   double shift, const void* c, const void* sigma, int layout);
// sigma through the assembled CSR when H holds it for prec, else the five-launch
// matrix-free product with ws as its workspace (sigma_workspace_bytes); ev nullable.
int sigma_internal(const sbd_exc* x, const sbd_ham* H, int nvec, int prec, double shift,
                   const void* c, void* y, int layout, void* ws, hipStream_t st, hipEvent_t* ev = nullptr);

// ev (nullable): six events recorded on st around the five launches of the
// first vector (transpose, alpha stream, beta stream, alpha-beta, transpose-add).
template <class T>
hipError_t launch_sigma(const SigmaArgs<T>& A, int nvec, const T* c, T* y, int layout, void* ws,
                        const SigmaTune& tune, hipStream_t st, hipEvent_t* ev = nullptr);

// Full-bitstring determinant lists (k_full.hip).  A determinant is two words
// {alpha string, beta string}; lists are sorted by (alpha, beta) ascending.
// Sort and dedupe n determinants in `work` (device, capacity pow2(n)); unique
// ones to `out`, their count to d_count (device int64); scratch: 2 n + 1 +
// scan_tmp_words(n) device words.
hipError_t launch_full_sort_unique(void* work, int64_t n, void* out, int64_t* d_count, int64_t* scratch,
                                   hipStream_t st);
// flag[i] = 1 where determinant i starts a group of equal alpha strings
hipError_t launch_full_group_flags(const void* dets, int64_t n, int64_t* flag, hipStream_t st);
// from gpos (gpos[i+1] = group starts in [0, i]): group alpha strings ua, group
// offsets goff[ng + 1], group of each determinant grp
hipError_t launch_full_group_fill(const void* dets, int64_t n, const int64_t* gpos, uint64_t* ua, int64_t* goff,
                                  int32_t* grp, hipStream_t st);
// groups whose alpha strings differ by at most two electrons (self included):
// counts when rp is null, else neighbour group gj and alpha degree gd per row
hipError_t launch_full_group_nbr(const uint64_t* ua, int64_t ng, int64_t* cnt, const int64_t* rp, int32_t* gj,
                                 int8_t* gd, hipStream_t st);
// bw[i] = beta word of determinant i (n words)
hipError_t launch_full_beta(const void* dets, int64_t n, uint64_t* bw, hipStream_t st);
// connections (one or two electrons moved) of every determinant, from the beta
// words bw and the alpha groups: counts when rp is null, else ket J and
// electrons moved deg, rows sorted by J
hipError_t launch_full_conn(const uint64_t* bw, int64_t n, const int32_t* grp, const int64_t* goff,
                            const int64_t* gn_rp, const int32_t* gn_j, const int8_t* gn_d, int64_t* cnt,
                            const int64_t* rp, int32_t* J, int8_t* deg, hipStream_t st);
// integral tables: jt/kt norb^3 ((ai|kk), (ak|ki)), jd/kd norb^2 ((pp|qq), (pq|qp)),
// and dd npair^2 (npair = norb(norb-1)/2): dd[P(a,b) npair + P(i,j)] = (ai|bj) - (aj|bi)
// for a < b, i < j, P(p,q) = q(q-1)/2 + p
hipError_t launch_full_tables(const double* eri, int n, double* jt, double* kt, double* jd, double* kd,
                              double* dd, hipStream_t st);
hipError_t launch_full_diag(const void* dets, int64_t nd, int n, const double* h, const double* jd,
                            const double* kd, double e_core, double* out, hipStream_t st);
struct FullSigmaArgs {
    int64_t n = 0;
    int norb = 0;
    const void* dets = nullptr;
    const int64_t* rp = nullptr;
    const int32_t* J = nullptr;
    int64_t nconn = 0;
    const double *h = nullptr, *eri = nullptr, *jt = nullptr, *kt = nullptr, *dd = nullptr, *diag = nullptr;
    double shift = 0.0;
    const double* v64 = nullptr;  // assembled elements per connection (FP64 / FP32), or null
    const float* v32 = nullptr;
};
// y = (H - shift) x over a determinant list (layout and nvec as sbd_sigma),
// from the assembled elements of the vectors' precision where given
template <class T>
hipError_t launch_full_sigma(const FullSigmaArgs& S, int nvec, const T* x, T* y, int layout, hipStream_t st);
// out[e] = the element of connection e (in the connection order), rounded once to T
template <class T>
hipError_t launch_full_values(const FullSigmaArgs& S, T* out, hipStream_t st);
// occ[spin * norb + p]: occupation of spin-orbital p in the vector c over the
// list; scratch: full_occupation_scratch_words(n, norb) doubles
int64_t full_occupation_scratch_words(int64_t n, int norb);
hipError_t launch_full_occupations(const void* dets, const double* c, int64_t n, int norb, double* scratch,
                                   double* occ, hipStream_t st);
// xt[v][i] = xf[v][j] for the determinant j of the sorted list `from` equal to
// determinant i of `to`, else 0 (nvec vectors of nf and nt doubles)
hipError_t launch_full_map(const void* from, int64_t nf, const void* to, int64_t nt, int nvec, const double* xf,
                           double* xt, hipStream_t st);

// Device-resident state of device-driven Davidson iterations (k_devloop.hip).
constexpr int kDlMaxSpace = 48;   // subspace rows
constexpr int kDlMaxRoots = 8;
constexpr int kDlMaxKeep = 16;    // vectors kept by a thick restart
constexpr int kDlBlocks = 256;    // grid of the sweeps (partial sums per block)
constexpr int kDlHistory = 512;
// Largest basis the device-driven iterations take: their sweeps run on at most
// kDlBlocks workgroups (few waves per CU), which pays where an iteration is
// bound by launches and host round trips, not where it streams gigabytes.
constexpr int64_t kDlMaxN = (int64_t)1 << 21;
enum { kDlRunning = 0, kDlConverged = 1, kDlRefresh = 2, kDlMaxIter = 3, kDlStagnation = 4, kDlNumeric = 5 };
struct DlState {
    int m, k, ms, keep;          // subspace size, roots, maximum size, restart size
    int it, max_iter;            // iterations so far (all of the solve), limit
    int stop;                    // kDl* reason; nonzero makes the rest of a queued batch a no-op
    int restart, m_old, m_cur, since_cert, restarts;
    int active[kDlMaxRoots], row[kDlMaxRoots];
    int hist_n;
    int zm;                      // size of the previous Ritz step's decomposition kept for a warm start (0: none)
    unsigned cnt[8];             // completion counters of the fused reductions (zero between launches)
    double tol, delta, rho;
    double theta[kDlMaxRoots], rnorm[kDlMaxRoots], tnorm[kDlMaxRoots], ebnd[kDlMaxRoots];
    double scale[kDlMaxRoots];
    double evals[kDlMaxSpace];
    double h[kDlMaxSpace];
    double T[kDlMaxSpace * kDlMaxSpace];
    double Y[kDlMaxSpace * kDlMaxRoots];
    double Yc[kDlMaxSpace * kDlMaxKeep];
    double ebound[kDlMaxSpace + 8];
    double red[kDlMaxSpace * kDlMaxRoots];
    double hist_theta[kDlHistory];
    unsigned long long hist_clock[kDlHistory];  // device wall clock at each iteration's decision
};
// One device-driven iteration: Ritz pairs, residuals, decisions, restart,
// Gram-Schmidt of the corrections, the row index of the coming sigma
// (rows [m_old, m_old + k); row ms when stopped); then, after that sigma,
// the new entries of T.  part: kDlBlocks x (kDlMaxSpace x kDlMaxRoots) doubles;
// zbuf: kDlMaxSpace x (kDlMaxSpace + 1) doubles, the previous Ritz step's
// eigenvectors and eigenvalues (valid while S->zm > 0).  ms is the subspace
// limit of the solve (the kernels are specialised for k and ms).
hipError_t dl_iteration_pre(DlState* S, double* V, double* W, const double* diag, double* tmp, double* scr,
                            int64_t N, int k, int ms, double* part, int* rowsel, double* zbuf, hipStream_t st);
// *out = the device wall clock (s_memrealtime)
hipError_t launch_clock_read(unsigned long long* out, hipStream_t st);
hipError_t dl_iteration_post(DlState* S, const double* V, const double* W, int64_t N, int k, double* part,
                             hipStream_t st);

// The operator a Davidson solve works on: N determinants, the FP64 diagonal
// (start vectors, preconditioner), and y = (H - shift) c for nvec vectors in
// either layout (as sbd_sigma), with a workspace of ws_bytes(nvec, layout,
// element size) bytes.  The alpha x beta product basis and the
// full-bitstring determinant list each provide one.
struct SigmaOp {
    int64_t N = 0;
    const double* diag = nullptr;
    std::function<int(int nvec, int prec, double shift, const void* c, void* y, int layout, void* ws,
                      hipStream_t st)>
        apply;
    std::function<size_t(int nvec, int layout, size_t elem)> ws_bytes;
};
// Davidson options with defaults filled in and checked (nroots k, N determinants).
int davidson_options(int k, int64_t N, const sbd_davidson_opts* in, sbd_davidson_opts* o);
// The Davidson iteration of sbd_davidson on any operator (options already
// validated; t_start: when the caller's call began, for the report's times).
int davidson_run(const SigmaOp& op, int k, const sbd_davidson_opts& o, double* energies, double* vectors,
                 sbd_davidson_report* report, void* stream, std::chrono::steady_clock::time_point t_start,
                 double t_autotune);

// Dense vector kernels for Davidson (FP64 unless noted).  Vectors are rows
// of length N stored contiguously: A + j*N.
// out[r][i] = sum_j A[j][i] Y[j*ldy + r], r < k (Y on device, m x k column block)
hipError_t launch_combination(const double* A, int m, const double* d_Y, int ldy, int k,
                              double* out, int64_t N, hipStream_t st);
hipError_t launch_scale(double* x, int64_t N, double s, hipStream_t st);
// lexicographic successor minimum: smallest (v,i) > (vprev, iprev); writes value/index
hipError_t launch_argmin_after(const double* v, int64_t N, double vprev, int64_t iprev,
                               double* d_val, int64_t* d_idx, double* d_part_v,
                               int64_t* d_part_i, hipStream_t st);
hipError_t launch_set_unit(double* x, int64_t N, int64_t idx, hipStream_t st);
// Block sigma staging: out[i*nv + v] = src row v (v < cnt), zero for cnt <= v < nv;
// dst row v = y[., v] (+ shift * x row v when x is given).  With d_row (device
// int), src, x and dst are offset by that many rows, read when the kernel runs.
template <class T>
hipError_t launch_interleave(const double* src, const int* d_row, int cnt, int nv, int64_t N, T* out,
                             hipStream_t st);
template <class T>
hipError_t launch_deinterleave(const T* y, int cnt, int nv, int64_t N, const double* x, double shift,
                               double* dst, const int* d_row, hipStream_t st);
// *d_p = v (a one-thread kernel: usable where memset and memcpy nodes are not wanted)
hipError_t launch_set_int(int* d_p, int v, hipStream_t st);
// *d_val = max_i v[i]; d_part holds kRedBlocks partials
hipError_t launch_max(const double* v, int64_t N, double* d_val, double* d_part, hipStream_t st);

hipError_t launch_fill_pattern(void* p, int64_t n, int prec, hipStream_t st);
// map[i] = position of to[i] in the sorted from[0..nfrom), or -1
hipError_t launch_string_map(const uint64_t* to, int64_t nto, const uint64_t* from, int64_t nfrom,
                             int64_t* map, hipStream_t st);
// y[v][ia][ib] = x[v][amap[ia]][bmap[ib]] (0 where either map is -1); y has nvec x na x nb,
// x has nvec vectors of n_from = (old alpha count) x nb_from
hipError_t launch_map_vectors(const int64_t* amap, const int64_t* bmap, int64_t na, int64_t nb, int64_t nb_from,
                              int64_t n_from, int nvec, const double* x, double* y, hipStream_t st);
hipError_t launch_f64_to_f32(const double* x, float* y, int64_t n, hipStream_t st);
// occ[spin * norb + p]: occupation of spin-orbital p in the vector c over the
// product of the sorted strings sa (na) and sb (nb), c[ia * nb + ib];
// scratch: occupation_scratch_words(na, nb) doubles
int64_t occupation_scratch_words(int64_t na, int64_t nb);
hipError_t launch_occupations(const double* c, const uint64_t* sa, int64_t na, const uint64_t* sb, int64_t nb,
                              int norb, double* scratch, double* occ, hipStream_t st);
hipError_t launch_f32_to_f64_axpy(const float* y32, const double* x, double shift, double* y,
                                  int64_t n, hipStream_t st);

// Tall-skinny passes of the Davidson update (k_project.hip).  Each reduces its
// rows into out (device) in a fixed order; part holds kPassRows x kRedBlocks
// partials.  m, mp, mw <= 48 and k <= 8.
// pass_resid rows: [0,k) |r_q|^2, [k,2k) |t_q|^2, then (proj) [2k + j*k + q) V_j . t_q
hipError_t pass_resid(const double* V, const double* W, int m, int k, const double* Y,
                      const double* theta, const double* diag, double delta, double* T, int64_t N,
                      bool proj, double* part, double* out, hipStream_t st);
// the residual pass that also projects each t_q on W: rows as pass_resid with
// proj, then [2k + m*k + j*k + q) W_j . t_q; available when pass_resid_w_fits(m, k)
bool pass_resid_w_fits(int m, int k);
hipError_t pass_resid_w(const double* V, const double* W, int m, int k, const double* Y,
                        const double* theta, const double* diag, double delta, double* T, int64_t N,
                        double* part, double* out, hipStream_t st);
// T_q <- T_q - sum_j V_j H[j*k + q] for q < k (in place), rows [q1*k + q2) = T_q1 . T_q2;
// available when pass_subb_fits(m, k)
bool pass_subb_fits(int m, int k);
hipError_t pass_subb(const double* V, int m, const double* H, double* T, int k, int64_t N, double* part,
                     double* out, hipStream_t st);
// dst <- (t - V h) * s, and dst32 <- (float)dst when dst32 is not null; no sums
// (dst must not alias V)
hipError_t pass_subs(const double* V, int m, const double* h, const double* t, double s, double* dst,
                     float* dst32, int64_t N, hipStream_t st);
// y <- (double)y32 + shift * x;  out[0] = x . y.  With row (device int) not
// null, x and y are the bases of V and W and the row *row of each is used.
hipError_t pass_restore(const float* y32, const double* x, double shift, double* y, int64_t N,
                        const int* row, double* part, double* out, hipStream_t st);
// t <- t - V h;  rows [0] |t|^2, [1 + j) V_j . t
hipError_t pass_sub1(const double* V, int m, const double* h, double* t, int64_t N, double* part,
                     double* out, hipStream_t st);
// dst <- t - V h;  rows [0] |dst|^2, [1 + j) V_j . dst (j < m), [1 + m + j) W_j . dst (j < mw);
// available when pass_sub1w_fits(m, mw) (dst may alias t)
bool pass_sub1w_fits(int m, int mw);
hipError_t pass_sub1w(const double* V, int m, const double* h, const double* t, double* dst,
                      const double* W, int mw, int64_t N, double* part, double* out, hipStream_t st);
// dst <- t - V h;  rows [0] |dst|^2, [1 + j) W_j . dst  (j < mw)
hipError_t pass_sub2(const double* V, int m, const double* h, const double* t, double* dst,
                     const double* W, int mw, int64_t N, double* part, double* out, hipStream_t st);
// rows [j*k + q) = P_j . X_q   (mp <= 48, k <= 8; split into row groups as needed)
hipError_t pass_project(const double* P, int mp, const double* X, int k, int64_t N, double* part,
                        double* out, hipStream_t st);

// Reduction scratch sizing.
constexpr int kRedBlocks = 1024;
constexpr int kPassRows = 512;

}  // namespace sbd
