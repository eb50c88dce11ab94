// Successive solves of an SQD run (Sec. I): the configuration set grows as
// more sampled configurations are taken in, and each step diagonalises H over
// the Cartesian product of the sampled alpha and beta strings (Sec. II-B),
// optionally starting Davidson from the previous step's eigenvectors carried
// into the new basis (Sec. II-C allows any start vector).  Optionally the
// samples are filtered first (Sec. I): those with a wrong electron count are
// corrected from the previous step's orbital occupations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
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

// ------------------------------------------------------------------ recovery
// Samples with a wrong electron count in a spin are corrected bit by bit from
// the average spin-orbital occupations of the previous solution: surplus
// electrons leave occupied orbitals, missing ones enter empty orbitals, each
// orbital drawn (without replacement) with probability proportional to the
// weight of its distance from the average occupation.  Uniforms come from
// SplitMix64 (Steele, Lea and Flood, 2014) on seed + counter, so a run is
// reproducible and the sequence of decisions is fixed: FP64, candidates in
// increasing orbital order.

uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t seed, uint64_t counter) {
    return (double)(splitmix64(seed + counter) >> 11) * (1.0 / 9007199254740992.0);
}

// weight of a bit at distance y from its average occupation, for a spin whose
// filling is h = electrons / norb: slope delta / h up to h, then from delta to 1
double flip_weight(double y, double h) {
    const double delta = 0.01;
    if (y <= h) return h > 0.0 ? delta * y / h : 0.0;
    return delta + (1.0 - delta) * (y - h) / (1.0 - h);
}

uint64_t recover_word(uint64_t word, int n, int norb, const double* occ, uint64_t seed, int64_t sample, int spin) {
    const int w = __builtin_popcountll(word);
    if (w == n) return word;
    const double h = (double)n / (double)norb;
    const bool remove = w > n;
    const double x = remove ? 1.0 : 0.0;
    int cand[64];
    double wt[64];
    int nc = 0;
    for (int p = 0; p < norb; ++p)
        if ((int)((word >> p) & 1ull) == (remove ? 1 : 0)) {
            cand[nc] = p;
            wt[nc] = flip_weight(std::fabs(x - occ[p]), h);
            ++nc;
        }
    const int k = remove ? w - n : n - w;
    for (int j = 0; j < k; ++j) {
        const double u = uniform01(seed, ((uint64_t)sample * 2 + (uint64_t)spin) * 64 + (uint64_t)j);
        double total = 0.0;
        for (int i = 0; i < nc; ++i) total += wt[i];
        int pick = -1;
        if (total > 0.0) {
            const double target = u * total;
            double cum = 0.0;
            for (int i = 0; i < nc && pick < 0; ++i) {
                cum += wt[i];
                if (target < cum) pick = i;
            }
            for (int i = nc - 1; pick < 0 && i >= 0; --i)  // rounding: last candidate of nonzero weight
                if (wt[i] > 0.0) pick = i;
        } else {
            pick = (int)(u * nc);
        }
        word ^= 1ull << cand[pick];
        for (int i = pick; i + 1 < nc; ++i) {
            cand[i] = cand[i + 1];
            wt[i] = wt[i + 1];
        }
        --nc;
    }
    return word;
}

}  // namespace

extern "C" int sbd_recover_configurations(int norb, int n_alpha, int n_beta, const uint64_t* samples,
                                          int64_t nsamples, const double* occ, uint64_t seed, uint64_t* out,
                                          int64_t* n_out, int64_t* n_corrected) {
    if (!out || !n_out || (nsamples > 0 && !samples)) return fail(SBD_ERR_ARG, "null argument");
    if (norb < 1 || norb > 64) return fail(SBD_ERR_NORB, "norb must be in [1, 64]");
    if (n_alpha < 0 || n_alpha > norb || n_beta < 0 || n_beta > norb)
        return fail(SBD_ERR_ARG, "electron counts must be in [0, norb]");
    if (nsamples < 0) return fail(SBD_ERR_ARG, "nsamples must be >= 0");
    if (occ)
        for (int p = 0; p < 2 * norb; ++p)
            if (!std::isfinite(occ[p])) return fail(SBD_ERR_ARG, "occupations must be finite");
    const uint64_t high = norb >= 64 ? 0ull : ~((1ull << norb) - 1ull);
    for (int64_t i = 0; i < nsamples; ++i)
        if ((samples[2 * i] & high) || (samples[2 * i + 1] & high))
            return fail(SBD_ERR_STRING, "sample " + std::to_string(i) + " has a bit at or above norb");
    int64_t m = 0, corrected = 0;
    for (int64_t i = 0; i < nsamples; ++i) {
        const uint64_t a = samples[2 * i], b = samples[2 * i + 1];
        if (__builtin_popcountll(a) == n_alpha && __builtin_popcountll(b) == n_beta) {
            out[2 * m] = a;
            out[2 * m + 1] = b;
            ++m;
        } else if (occ) {
            out[2 * m] = recover_word(a, n_alpha, norb, occ, seed, i, 0);
            out[2 * m + 1] = recover_word(b, n_beta, norb, occ + norb, seed, i, 1);
            ++m;
            ++corrected;
        }
    }
    *n_out = m;
    if (n_corrected) *n_corrected = corrected;
    return SBD_OK;
}

extern "C" int sbd_occupations(const sbd_basis* b, const double* vec, double* occ, void* stream) {
    if (!b || !vec || !occ) return fail(SBD_ERR_ARG, "null argument");
    const int64_t na = b->s[0].n, nb = b->s[1].n;
    const int norb = b->norb;
    hipStream_t st = (hipStream_t)stream;
    DevBuf scratch, od;
    SBD_HIP(scratch.alloc(sizeof(double) * (size_t)occupation_scratch_words(na, nb)));
    SBD_HIP(od.alloc(sizeof(double) * 2 * (size_t)norb));
    SBD_HIP(launch_occupations(vec, b->s[0].d.as<uint64_t>(), na, b->s[1].d.as<uint64_t>(), nb, norb,
                               scratch.as<double>(), od.as<double>(), st));
    SBD_HIP(hipMemcpyAsync(occ, od.p, sizeof(double) * 2 * (size_t)norb, hipMemcpyDeviceToHost, st));
    SBD_HIP(hipStreamSynchronize(st));
    return SBD_OK;
}

extern "C" void sbd_sqd_default_opts(sbd_sqd_opts* o) {
    if (!o) return;
    sbd_davidson_default_opts(&o->davidson);
    o->warm_start = 1;
    o->spin_union = 0;
    o->full_bitstring = 0;
    o->recovery = 0;
    o->recovery_seed = 0;
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
    std::vector<uint64_t> rec;  // recovered samples of the step
    std::vector<double> occ;    // occupations of the previous step's lowest root
    for (int s = 0; s < nsteps; ++s) {
        const auto t0 = std::chrono::steady_clock::now();
        // the configuration set of this step: the first step_samples[s] samples
        int64_t m = step_samples[s];
        const uint64_t* smp = samples;
        int64_t corrected = 0, dropped = 0;
        if (o.recovery) {  // wrong electron counts: dropped at the first step, corrected after it
            if (prev) {
                occ.assign(2 * (size_t)norb, 0.0);
                rc = o.full_bitstring ? sbd_full_occupations(prev->fb, prev_vec.as<double>(), occ.data(), stream)
                                      : sbd_occupations(prev->b, prev_vec.as<double>(), occ.data(), stream);
                if (rc) return rc;
            }
            rec.resize(2 * (size_t)m);
            int64_t kept = 0;
            rc = sbd_recover_configurations(norb, n_alpha, n_beta, samples, m, prev ? occ.data() : nullptr,
                                            o.recovery_seed, rec.data(), &kept, &corrected);
            if (rc) return rc;
            if (kept == 0) return fail(SBD_ERR_ARG, "no sample with the right electron counts");
            dropped = m - kept;
            m = kept;
            smp = rec.data();
        }
        std::unique_ptr<StepHandles> cur(new StepHandles());
        int64_t na = 0, nb = 0, N = 0;
        if (o.full_bitstring) {  // the basis is the set of distinct sampled determinants
            rc = sbd_full_build_basis(norb, n_alpha, n_beta, smp, m, stream, &cur->fb);
            if (!rc) rc = sbd_full_set_hamiltonian(cur->fb, h1, eri, e_core, stream, &cur->fh);
            if (rc) return rc;
            int64_t nconn = 0;
            sbd_full_basis_sizes(cur->fb, &N, &nconn, &na);
        } else {
            std::vector<uint64_t> A((size_t)m), B((size_t)m);
            for (int64_t i = 0; i < m; ++i) {
                A[(size_t)i] = smp[2 * i];
                B[(size_t)i] = smp[2 * i + 1];
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
            out.samples = step_samples[s];
            out.corrected = corrected;
            out.dropped = dropped;
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
