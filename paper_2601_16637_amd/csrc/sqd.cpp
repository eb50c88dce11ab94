// Successive solves of an SQD run (Sec. I): the configuration set grows as
// more sampled configurations are taken in, and each step diagonalises H over
// the Cartesian product of the sampled alpha and beta strings (Sec. II-B),
// optionally starting Davidson from the previous step's eigenvectors carried
// into the new basis (Sec. II-C allows any start vector).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <vector>

#include "internal.h"

using namespace sbd;

namespace {

struct StepHandles {
    sbd_basis* b = nullptr;
    sbd_exc* x = nullptr;
    sbd_ham* h = nullptr;
    sbd_fbasis* fb = nullptr;  // full-bitstring steps
    sbd_fham* fh = nullptr;
    ~StepHandles() {
        if (h) sbd_free_ham(h);
        if (x) sbd_free_exc(x);
        if (b) sbd_free_basis(b);
        if (fh) sbd_free_full_ham(fh);
        if (fb) sbd_free_full_basis(fb);
    }
};

}  // namespace

extern "C" void sbd_sqd_default_opts(sbd_sqd_opts* o) {
    if (!o) return;
    sbd_davidson_default_opts(&o->davidson);
    o->warm_start = 1;
    o->spin_union = 0;
    o->full_bitstring = 0;
}

extern "C" int sbd_sqd_run(int norb, int n_alpha, int n_beta, const double* h1, const double* eri, double e_core,
                           const uint64_t* samples, int64_t nsamples, const int64_t* step_samples, int nsteps,
                           int nroots, const sbd_sqd_opts* opts_in, double* energies, sbd_sqd_step* steps,
                           void* stream) {
    if (!h1 || !eri || !samples || !step_samples || !energies) return fail(SBD_ERR_ARG, "null argument");
    if (nsteps < 1 || nsamples < 1) return fail(SBD_ERR_ARG, "need at least one step and one sample");
    if (nroots < 1 || nroots > 8) return fail(SBD_ERR_ARG, "nroots must be in [1, 8]");
    for (int s = 0; s < nsteps; ++s)
        if (step_samples[s] < 1 || step_samples[s] > nsamples || (s > 0 && step_samples[s] < step_samples[s - 1]))
            return fail(SBD_ERR_ARG, "step_samples must be non-decreasing prefix lengths in [1, nsamples]");
    sbd_sqd_opts o;
    sbd_sqd_default_opts(&o);
    if (opts_in) o = *opts_in;
    if (o.spin_union && n_alpha != n_beta) return fail(SBD_ERR_ARG, "spin_union needs n_alpha == n_beta");
    if (o.spin_union && o.full_bitstring) return fail(SBD_ERR_ARG, "spin_union applies to product bases only");
    if (o.davidson.n_guess != 0 || o.davidson.guess) return fail(SBD_ERR_ARG, "guess is set by the SQD loop");
    int rc = validate_integrals(norb, h1, eri);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;

    std::unique_ptr<StepHandles> prev;
    DevBuf prev_vec;
    int prev_k = 0;
    for (int s = 0; s < nsteps; ++s) {
        const auto t0 = std::chrono::steady_clock::now();
        // the configuration set of this step: the first step_samples[s] samples
        const int64_t m = step_samples[s];
        std::unique_ptr<StepHandles> cur(new StepHandles());
        int64_t na = 0, nb = 0, N = 0;
        if (o.full_bitstring) {  // the basis is the set of distinct sampled determinants
            rc = sbd_full_build_basis(norb, n_alpha, n_beta, samples, m, stream, &cur->fb);
            if (!rc) rc = sbd_full_set_hamiltonian(cur->fb, h1, eri, e_core, stream, &cur->fh);
            if (rc) return rc;
            int64_t nconn = 0;
            sbd_full_basis_sizes(cur->fb, &N, &nconn, &na);
        } else {
            std::vector<uint64_t> A((size_t)m), B((size_t)m);
            for (int64_t i = 0; i < m; ++i) {
                A[(size_t)i] = samples[2 * i];
                B[(size_t)i] = samples[2 * i + 1];
            }
            if (o.spin_union) {  // both spins take every sampled string
                A.insert(A.end(), B.begin(), B.end());
                B = A;
            }
            rc = sbd_build_basis(norb, n_alpha, n_beta, A.data(), (int64_t)A.size(), B.data(), (int64_t)B.size(),
                                 stream, &cur->b);
            if (!rc) rc = sbd_build_excitations(cur->b, stream, &cur->x);
            if (!rc) rc = sbd_set_hamiltonian(cur->b, cur->x, h1, eri, e_core, stream, &cur->h);
            if (rc) return rc;
            sbd_basis_sizes(cur->b, &na, &nb);
            N = na * nb;
        }
        const int k = (int)std::min<int64_t>(nroots, N);
        DevBuf guess, vec;
        sbd_davidson_opts dopt = o.davidson;
        hipError_t e = vec.alloc(sizeof(double) * (size_t)k * N);
        if (e != hipSuccess) return hip_fail(e, "sbd_sqd_run vectors");
        int warm = 0;
        if (o.warm_start && prev) {
            e = guess.alloc(sizeof(double) * (size_t)k * N);
            if (e != hipSuccess) return hip_fail(e, "sbd_sqd_run guess");
            const int kg = std::min(k, prev_k);
            rc = o.full_bitstring
                     ? sbd_full_map_vectors(prev->fb, cur->fb, kg, prev_vec.as<double>(), guess.as<double>(), stream)
                     : sbd_map_vectors(prev->b, cur->b, kg, prev_vec.as<double>(), guess.as<double>(), stream);
            if (rc) return rc;
            dopt.guess = guess.as<double>();
            dopt.n_guess = kg;
            warm = 1;
        }
        const auto t1 = std::chrono::steady_clock::now();
        double ev[8] = {0};
        sbd_davidson_report rep;
        std::memset(&rep, 0, sizeof(rep));
        const int st_dav = o.full_bitstring
                               ? sbd_full_davidson(cur->fb, cur->fh, k, &dopt, ev, vec.as<double>(), &rep, stream)
                               : sbd_davidson(cur->b, cur->x, cur->h, k, &dopt, ev, vec.as<double>(), &rep, stream);
        if (st_dav < 0) return st_dav;
        SBD_HIP(hipStreamSynchronize(st));
        const auto t2 = std::chrono::steady_clock::now();
        for (int r = 0; r < nroots; ++r) energies[(size_t)s * nroots + r] = r < k ? ev[r] : 0.0;
        if (steps) {
            sbd_sqd_step& out = steps[s];
            std::memset(&out, 0, sizeof(out));
            out.status = st_dav;
            out.samples = m;
            out.n_alpha_str = na;
            out.n_beta_str = nb;
            out.ndet = N;
            out.warm = warm;
            out.iterations = rep.iterations;
            out.sigma_calls = rep.sigma_calls;
            out.residual = *std::max_element(rep.residual, rep.residual + k);
            out.setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
            out.solve_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
        }
        prev = std::move(cur);
        prev_vec = std::move(vec);
        prev_k = k;
    }
    return SBD_OK;
}
