// C ABI of the full-bitstring path (Sec. II-F, Sec. III-F): a selected basis
// given as an arbitrary list of determinants, each one packed spin-orbital
// string, instead of a Cartesian product of alpha and beta strings.  Host-side
// validation, handle construction and launches; the kernels are in k_full.hip.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace sbd;

struct sbd_fbasis {
    uint64_t id = 0;
    int norb = 0, n_el[2] = {0, 0};
    int64_t n = 0;                // unique determinants
    DevBuf dets;                  // n x {alpha word, beta word}, sorted
    std::vector<uint64_t> host;   // the same, 2n words
    int64_t ngroups = 0;          // distinct alpha strings
    DevBuf ua, goff, grp;         // group alpha strings, offsets [ng+1], group of each determinant
    int64_t gnnz = 0;
    DevBuf gn_rp, gn_j, gn_d;     // neighbour groups (alpha within two electrons)
    int64_t nconn = 0;
    DevBuf rp, J, deg;            // connections: CSR [n+1], ket, electrons moved
};

struct sbd_fham {
    uint64_t basis_id = 0;
    int norb = 0;
    int64_t n = 0;
    double e_core = 0.0;
    DevBuf h64, eri64, jt, kt, jd, kd, dd, diag;
    DevBuf v64, v32;   // assembled elements per connection (explicit realization)
    int asm_prec = 0;  // bit 0: FP64 assembled, bit 1: FP32
};

namespace {

std::atomic<uint64_t> g_next_fid{1};

int validate_dets(int norb, int na, int nb, const uint64_t* d, int64_t n) {
    if (!d || n < 1) return fail(SBD_ERR_ARG, "need at least one determinant");
    const uint64_t high = norb >= 64 ? 0ull : ~((1ull << norb) - 1ull);
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t a = d[2 * i], b = d[2 * i + 1];
        if ((a & high) || (b & high))
            return fail(SBD_ERR_STRING, "determinant " + std::to_string(i) + " has a bit at or above norb");
        if (__builtin_popcountll(a) != na || __builtin_popcountll(b) != nb)
            return fail(SBD_ERR_STRING, "determinant " + std::to_string(i) + " has the wrong electron count");
    }
    return SBD_OK;
}

FullSigmaArgs sigma_args(const sbd_fbasis* B, const sbd_fham* H) {
    FullSigmaArgs A;
    A.n = B->n;
    A.nconn = B->nconn;
    A.norb = B->norb;
    A.dets = B->dets.p;
    A.rp = B->rp.as<int64_t>();
    A.J = B->J.as<int32_t>();
    A.h = H->h64.as<double>();
    A.eri = H->eri64.as<double>();
    A.jt = H->jt.as<double>();
    A.kt = H->kt.as<double>();
    A.dd = H->dd.as<double>();
    A.diag = H->diag.as<double>();
    return A;
}

int full_sigma_launch(const sbd_fbasis* B, const sbd_fham* H, int nvec, int prec, double shift, const void* c,
                      void* y, int layout, hipStream_t st) {
    FullSigmaArgs A = sigma_args(B, H);
    A.shift = shift;
    if (H->asm_prec & 1) A.v64 = H->v64.as<double>();
    if (H->asm_prec & 2) A.v32 = H->v32.as<float>();
    hipError_t e = prec == SBD_FP64
                       ? launch_full_sigma<double>(A, nvec, (const double*)c, (double*)y, layout, st)
                       : launch_full_sigma<float>(A, nvec, (const float*)c, (float*)y, layout, st);
    if (e != hipSuccess) return hip_fail(e, "sbd_full_sigma launch");
    return SBD_OK;
}

}  // namespace

extern "C" {

int sbd_full_build_basis(int norb, int n_alpha, int n_beta, const uint64_t* dets, int64_t ndet, void* stream,
                         sbd_fbasis** out) {
    if (!out) return fail(SBD_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (norb < 1 || norb > 64) return fail(SBD_ERR_NORB, "norb must be in [1, 64]");
    if (n_alpha < 0 || n_alpha > norb || n_beta < 0 || n_beta > norb)
        return fail(SBD_ERR_ARG, "electron counts must be in [0, norb]");
    int rc = validate_dets(norb, n_alpha, n_beta, dets, ndet);
    if (rc) return rc;
    if (ndet > ((int64_t)1 << 30)) return fail(SBD_ERR_ARG, "too many determinants (limit 2^30)");
    hipStream_t st = (hipStream_t)stream;
    std::unique_ptr<sbd_fbasis> B(new sbd_fbasis());
    B->norb = norb;
    B->n_el[0] = n_alpha;
    B->n_el[1] = n_beta;
    int64_t P = 1;
    while (P < ndet) P <<= 1;
    DevBuf work, cnt, scan, tmp, uniq;
    hipError_t e = work.alloc(16 * (size_t)P);
    if (e == hipSuccess) e = cnt.alloc(sizeof(int64_t));
    if (e == hipSuccess) e = B->dets.alloc(16 * (size_t)ndet);
    // scan scratch, sized for the longest scan below (the determinants given)
    if (e == hipSuccess) e = tmp.alloc(sizeof(int64_t) * (size_t)scan_tmp_words(ndet));
    if (e == hipSuccess) e = uniq.alloc(sizeof(int64_t) * (size_t)(2 * ndet + 1 + scan_tmp_words(ndet)));
    if (e == hipSuccess) e = hipMemcpyAsync(work.p, dets, 16 * (size_t)ndet, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_full_sort_unique(work.p, ndet, B->dets.p, cnt.as<int64_t>(), uniq.as<int64_t>(), st);
    int64_t n = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&n, cnt.p, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "sbd_full_build_basis (sort)");
    B->n = n;
    work.release();
    uniq.release();
    // groups of equal alpha strings
    DevBuf flag;
    e = flag.alloc(sizeof(int64_t) * n);
    if (e == hipSuccess) e = scan.alloc(sizeof(int64_t) * (n + 1));
    if (e == hipSuccess) e = launch_full_group_flags(B->dets.p, n, flag.as<int64_t>(), st);
    if (e == hipSuccess) e = launch_exclusive_scan(flag.as<int64_t>(), n, scan.as<int64_t>(), tmp.as<int64_t>(), st);
    int64_t ng = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&ng, scan.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "sbd_full_build_basis (groups)");
    B->ngroups = ng;
    e = B->ua.alloc(sizeof(uint64_t) * ng);
    if (e == hipSuccess) e = B->goff.alloc(sizeof(int64_t) * (ng + 1));
    if (e == hipSuccess) e = B->grp.alloc(sizeof(int32_t) * n);
    if (e == hipSuccess)
        e = launch_full_group_fill(B->dets.p, n, scan.as<int64_t>(), B->ua.as<uint64_t>(), B->goff.as<int64_t>(),
                                   B->grp.as<int32_t>(), st);
    // neighbour groups
    DevBuf gcnt;
    if (e == hipSuccess) e = gcnt.alloc(sizeof(int64_t) * ng);
    if (e == hipSuccess) e = B->gn_rp.alloc(sizeof(int64_t) * (ng + 1));
    if (e == hipSuccess)
        e = launch_full_group_nbr(B->ua.as<uint64_t>(), ng, gcnt.as<int64_t>(), nullptr, nullptr, nullptr, st);
    if (e == hipSuccess) e = launch_exclusive_scan(gcnt.as<int64_t>(), ng, B->gn_rp.as<int64_t>(), tmp.as<int64_t>(), st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&B->gnnz, B->gn_rp.as<int64_t>() + ng, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "sbd_full_build_basis (alpha neighbours)");
    e = B->gn_j.alloc(sizeof(int32_t) * std::max<int64_t>(B->gnnz, 1));
    if (e == hipSuccess) e = B->gn_d.alloc(std::max<int64_t>(B->gnnz, 1));
    if (e == hipSuccess)
        e = launch_full_group_nbr(B->ua.as<uint64_t>(), ng, nullptr, B->gn_rp.as<int64_t>(), B->gn_j.as<int32_t>(),
                                  B->gn_d.as<int8_t>(), st);
    // connections of every determinant
    DevBuf bw;
    if (e == hipSuccess) e = bw.alloc(sizeof(uint64_t) * n);
    if (e == hipSuccess) e = launch_full_beta(B->dets.p, n, bw.as<uint64_t>(), st);
    if (e == hipSuccess) e = B->rp.alloc(sizeof(int64_t) * (n + 1));
    if (e == hipSuccess)
        e = launch_full_conn(bw.as<uint64_t>(), n, B->grp.as<int32_t>(), B->goff.as<int64_t>(), B->gn_rp.as<int64_t>(),
                             B->gn_j.as<int32_t>(), B->gn_d.as<int8_t>(), flag.as<int64_t>(), nullptr, nullptr,
                             nullptr, st);
    if (e == hipSuccess) e = launch_exclusive_scan(flag.as<int64_t>(), n, B->rp.as<int64_t>(), tmp.as<int64_t>(), st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&B->nconn, B->rp.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "sbd_full_build_basis (connection counts)");
    e = B->J.alloc(sizeof(int32_t) * std::max<int64_t>(B->nconn, 1));
    if (e == hipSuccess) e = B->deg.alloc(std::max<int64_t>(B->nconn, 1));
    if (e == hipSuccess)
        e = launch_full_conn(bw.as<uint64_t>(), n, B->grp.as<int32_t>(), B->goff.as<int64_t>(), B->gn_rp.as<int64_t>(),
                             B->gn_j.as<int32_t>(), B->gn_d.as<int8_t>(), nullptr, B->rp.as<int64_t>(),
                             B->J.as<int32_t>(), B->deg.as<int8_t>(), st);
    B->host.resize(2 * (size_t)n);
    if (e == hipSuccess) e = hipMemcpyAsync(B->host.data(), B->dets.p, 16 * (size_t)n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "sbd_full_build_basis (connections)");
    B->id = g_next_fid++;
    *out = B.release();
    return SBD_OK;
}

int sbd_full_basis_sizes(const sbd_fbasis* B, int64_t* ndet, int64_t* nconn, int64_t* nalpha) {
    if (!B) return fail(SBD_ERR_ARG, "null basis");
    if (ndet) *ndet = B->n;
    if (nconn) *nconn = B->nconn;
    if (nalpha) *nalpha = B->ngroups;
    return SBD_OK;
}

int sbd_full_basis_export(const sbd_fbasis* B, uint64_t* dets, int64_t* row_ptr, int32_t* J, int8_t* deg) {
    if (!B) return fail(SBD_ERR_ARG, "null basis");
    if (dets) std::memcpy(dets, B->host.data(), 16 * (size_t)B->n);
    if (row_ptr) SBD_HIP(hipMemcpy(row_ptr, B->rp.p, sizeof(int64_t) * (B->n + 1), hipMemcpyDeviceToHost));
    if (J && B->nconn) SBD_HIP(hipMemcpy(J, B->J.p, sizeof(int32_t) * B->nconn, hipMemcpyDeviceToHost));
    if (deg && B->nconn) SBD_HIP(hipMemcpy(deg, B->deg.p, (size_t)B->nconn, hipMemcpyDeviceToHost));
    return SBD_OK;
}

void sbd_free_full_basis(sbd_fbasis* B) { delete B; }

int sbd_full_set_hamiltonian(const sbd_fbasis* B, const double* h1, const double* eri, double e_core,
                             void* stream, sbd_fham** out) {
    if (!B || !h1 || !eri || !out) return fail(SBD_ERR_ARG, "null argument");
    *out = nullptr;
    if (!std::isfinite(e_core)) return fail(SBD_ERR_INTEGRALS, "e_core is not finite");
    const int n = B->norb;
    int rc = validate_integrals(n, h1, eri);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    std::unique_ptr<sbd_fham> H(new sbd_fham());
    H->basis_id = B->id;
    H->norb = n;
    H->n = B->n;
    H->e_core = e_core;
    const size_t n2 = (size_t)n * n, n3 = n2 * n, n4 = n3 * n, npair = (size_t)n * (n - 1) / 2;
    hipError_t e = H->h64.alloc(sizeof(double) * n2);
    if (e == hipSuccess) e = H->eri64.alloc(sizeof(double) * n4);
    if (e == hipSuccess) e = H->jt.alloc(sizeof(double) * n3);
    if (e == hipSuccess) e = H->kt.alloc(sizeof(double) * n3);
    if (e == hipSuccess) e = H->jd.alloc(sizeof(double) * n2);
    if (e == hipSuccess) e = H->kd.alloc(sizeof(double) * n2);
    if (e == hipSuccess) e = H->dd.alloc(sizeof(double) * npair * npair);
    if (e == hipSuccess) e = H->diag.alloc(sizeof(double) * B->n);
    if (e == hipSuccess) e = hipMemcpyAsync(H->h64.p, h1, sizeof(double) * n2, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(H->eri64.p, eri, sizeof(double) * n4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_full_tables(H->eri64.as<double>(), n, H->jt.as<double>(), H->kt.as<double>(), H->jd.as<double>(),
                               H->kd.as<double>(), H->dd.as<double>(), st);
    if (e == hipSuccess)
        e = launch_full_diag(B->dets.p, B->n, n, H->h64.as<double>(), H->jd.as<double>(), H->kd.as<double>(),
                             e_core, H->diag.as<double>(), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "sbd_full_set_hamiltonian");
    *out = H.release();
    return SBD_OK;
}

int sbd_full_ham_diag(const sbd_fham* H, double* diag_dev, void* stream) {
    if (!H || !diag_dev) return fail(SBD_ERR_ARG, "null argument");
    SBD_HIP(hipMemcpyAsync(diag_dev, H->diag.p, sizeof(double) * H->n, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return SBD_OK;
}

void sbd_free_full_ham(sbd_fham* H) { delete H; }

int sbd_full_sigma(const sbd_fbasis* B, const sbd_fham* H, int nvec, int prec, double shift, const void* c,
                   void* sigma, int layout, void* stream) {
    if (!B || !H || !c || !sigma) return fail(SBD_ERR_ARG, "null argument");
    if (H->basis_id != B->id) return fail(SBD_ERR_STATE, "Hamiltonian belongs to another basis");
    if (nvec < 1) return fail(SBD_ERR_ARG, "nvec must be >= 1");
    if (layout != 0 && layout != 1) return fail(SBD_ERR_ARG, "layout must be 0 or 1");
    if (layout == 1 && nvec != 1 && nvec != 2 && nvec != 4 && nvec != 8)
        return fail(SBD_ERR_ARG, "interleaved layout supports nvec in {1, 2, 4, 8}");
    if (prec != SBD_FP64 && prec != SBD_FP32) return fail(SBD_ERR_ARG, "bad precision");
    if (!std::isfinite(shift)) return fail(SBD_ERR_ARG, "shift is not finite");
    if (c == sigma) return fail(SBD_ERR_ARG, "c and sigma must not alias");
    return full_sigma_launch(B, H, nvec, prec, shift, c, sigma, layout, (hipStream_t)stream);
}

int sbd_full_map_vectors(const sbd_fbasis* from, const sbd_fbasis* to, int nvec, const double* x_from,
                         double* x_to, void* stream) {
    if (!from || !to || !x_from || !x_to) return fail(SBD_ERR_ARG, "null argument");
    if (nvec < 1) return fail(SBD_ERR_ARG, "nvec must be >= 1");
    if (from->norb != to->norb || from->n_el[0] != to->n_el[0] || from->n_el[1] != to->n_el[1])
        return fail(SBD_ERR_ARG, "the lists have different orbital or electron counts");
    const hipError_t e = launch_full_map(from->dets.p, from->n, to->dets.p, to->n, nvec, x_from, x_to,
                                         (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sbd_full_map_vectors launch");
    return SBD_OK;
}

int sbd_full_occupations(const sbd_fbasis* B, const double* vec, double* occ, void* stream) {
    if (!B || !vec || !occ) return fail(SBD_ERR_ARG, "null argument");
    hipStream_t st = (hipStream_t)stream;
    DevBuf scratch, od;
    SBD_HIP(scratch.alloc(sizeof(double) * (size_t)full_occupation_scratch_words(B->n, B->norb)));
    SBD_HIP(od.alloc(sizeof(double) * 2 * (size_t)B->norb));
    SBD_HIP(launch_full_occupations(B->dets.p, vec, B->n, B->norb, scratch.as<double>(), od.as<double>(), st));
    SBD_HIP(hipMemcpyAsync(occ, od.p, sizeof(double) * 2 * (size_t)B->norb, hipMemcpyDeviceToHost, st));
    SBD_HIP(hipStreamSynchronize(st));
    return SBD_OK;
}

int sbd_full_assemble(sbd_fham* H, const sbd_fbasis* B, int precisions, size_t max_bytes, void* stream) {
    if (!B || !H) return fail(SBD_ERR_ARG, "null argument");
    if (H->basis_id != B->id) return fail(SBD_ERR_STATE, "Hamiltonian belongs to another basis");
    if (precisions < 1 || precisions > 3) return fail(SBD_ERR_ARG, "precisions must be 1, 2 or 3");
    const size_t nc = (size_t)B->nconn;
    const size_t bytes = nc * (((precisions & 1) ? 8 : 0) + ((precisions & 2) ? 4 : 0));
    if (max_bytes && bytes > max_bytes)
        return fail(SBD_ERR_NOMEM, "sbd_full_assemble: the elements need " + std::to_string(bytes) +
                                       " bytes, more than max_bytes = " + std::to_string(max_bytes));
    hipStream_t st = (hipStream_t)stream;
    const FullSigmaArgs A = sigma_args(B, H);
    // built aside, so that a failure leaves the handle as it was
    DevBuf v64, v32;
    hipError_t e = hipSuccess;
    if ((precisions & 1) && nc) e = v64.alloc(sizeof(double) * nc);
    if (e == hipSuccess && (precisions & 2) && nc) e = v32.alloc(sizeof(float) * nc);
    if (e != hipSuccess) return hip_fail(e, "sbd_full_assemble allocation");
    if ((precisions & 1) && nc) e = launch_full_values<double>(A, v64.as<double>(), st);
    if (e == hipSuccess && (precisions & 2) && nc) e = launch_full_values<float>(A, v32.as<float>(), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "sbd_full_assemble");
    H->v64 = std::move(v64);
    H->v32 = std::move(v32);
    H->asm_prec = precisions;
    return SBD_OK;
}

int sbd_full_release_assembled(sbd_fham* H) {
    if (!H) return fail(SBD_ERR_ARG, "null argument");
    H->v64 = DevBuf();
    H->v32 = DevBuf();
    H->asm_prec = 0;
    return SBD_OK;
}

int sbd_full_assembled(const sbd_fham* H, int* precisions) {
    if (!H) return fail(SBD_ERR_ARG, "null argument");
    if (precisions) *precisions = H->asm_prec;
    return SBD_OK;
}

int sbd_full_davidson(const sbd_fbasis* B, const sbd_fham* H, int nroots, const sbd_davidson_opts* opts_in,
                      double* energies, double* vectors, sbd_davidson_report* report, void* stream) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!B || !H || !energies) return fail(SBD_ERR_ARG, "null argument");
    if (H->basis_id != B->id) return fail(SBD_ERR_STATE, "Hamiltonian belongs to another basis");
    sbd_davidson_opts o;
    int rc = davidson_options(nroots, B->n, opts_in, &o);
    if (rc) return rc;
    SigmaOp op;
    op.N = B->n;
    op.diag = H->diag.as<double>();
    op.apply = [B, H](int nvec, int prec, double shift, const void* c, void* y, int layout, void*, hipStream_t s2) {
        return full_sigma_launch(B, H, nvec, prec, shift, c, y, layout, s2);
    };
    op.ws_bytes = [](int, int, size_t) { return (size_t)0; };  // no workspace
    return davidson_run(op, nroots, o, energies, vectors, report, stream, t_start, 0.0);
}

}  // extern "C"
