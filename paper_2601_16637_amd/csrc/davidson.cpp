// Davidson eigensolver driver (Sec. II-C) with device-resident FP64 vectors.
//
// Per iteration, in the paper's order: sigma of the new basis vectors,
// projected matrix T = V^T W (updated column by column), smallest Ritz pairs
// of T, residual r = W y - theta V y fused with the damped diagonal
// preconditioner (Eqs. 6-7), convergence test on ||r||_2, orthogonalisation
// of each correction against the subspace (two classical Gram-Schmidt
// passes: "twice is enough"), expansion, and a restart onto the lowest Ritz
// vectors when the subspace is full.  Several roots are solved together as a
// block.
//
// SBD_FP32 mode (mixed precision): sigma of new basis vectors is computed in
// FP32 on (H - shift I), shift = lowest diagonal element, and restored in
// FP64; everything else stays FP64.  Residual-correction refinement: when the
// inner residuals (which carry the FP32 sigma error) fall below the target,
// one FP64 sigma of the Ritz vectors certifies the true residuals; if they
// are not yet below tol the subspace restarts from the Ritz vectors with their
// exact FP64 sigma and the inner iteration continues.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>

#include "internal.h"

namespace sbd {

int sigma_internal(const sbd_exc* x, const sbd_ham* H, int nvec, int prec, double shift,
                   const void* c, void* y, int layout, void* ws, hipStream_t st);

// Cyclic Jacobi eigensolver for a symmetric m x m matrix (row-major).  On exit
// w holds eigenvalues ascending and Z (row-major, column k = eigenvector k).
static void jacobi_eigh(int m, std::vector<double> A, std::vector<double>& w,
                        std::vector<double>& Z) {
    Z.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Z[i * m + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double a = A[i * m + j] * A[i * m + j];
                tot += a;
                if (i != j) off += a;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                double apq = A[p * m + q];
                if (apq == 0.0) continue;
                double app = A[p * m + p], aqq = A[q * m + q];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < m; ++k) {
                    double akp = A[k * m + p], akq = A[k * m + q];
                    A[k * m + p] = c * akp - s * akq;
                    A[k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {
                    double apk = A[p * m + k], aqk = A[q * m + k];
                    A[p * m + k] = c * apk - s * aqk;
                    A[q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    double zkp = Z[k * m + p], zkq = Z[k * m + q];
                    Z[k * m + p] = c * zkp - s * zkq;
                    Z[k * m + q] = s * zkp + c * zkq;
                }
            }
    }
    std::vector<int> ord(m);
    for (int i = 0; i < m; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return A[a * m + a] < A[b * m + b]; });
    w.resize(m);
    std::vector<double> Zs((size_t)m * m);
    for (int k = 0; k < m; ++k) {
        w[k] = A[ord[k] * m + ord[k]];
        for (int i = 0; i < m; ++i) Zs[i * m + k] = Z[i * m + ord[k]];
    }
    // fix sign: largest-magnitude component positive (deterministic output)
    for (int k = 0; k < m; ++k) {
        int imax = 0;
        for (int i = 1; i < m; ++i)
            if (std::fabs(Zs[i * m + k]) > std::fabs(Zs[imax * m + k])) imax = i;
        if (Zs[imax * m + k] < 0)
            for (int i = 0; i < m; ++i) Zs[i * m + k] = -Zs[i * m + k];
    }
    Z.swap(Zs);
}

namespace {

struct Work {
    DevBuf V, W, tmp, scr, part, small, d_idx, d32a, d32b, sws;
};

using clk = std::chrono::steady_clock;
inline double ms_since(clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

}  // namespace

// FP32 sigma of FP64 vectors: y = H x via (H - shift) in FP32 plus shift*x in FP64.
hipError_t launch_f64_to_f32(const double* x, float* y, int64_t n, hipStream_t st);
hipError_t launch_f32_to_f64_axpy(const float* y32, const double* x, double shift, double* y,
                                  int64_t n, hipStream_t st);

}  // namespace sbd

using namespace sbd;

extern "C" void sbd_davidson_default_opts(sbd_davidson_opts* o) {
    if (!o) return;
    o->tol_residual = 1e-6;
    o->max_iter = 200;
    o->max_space = 20;
    o->precond_delta = 1e-8;
    o->sigma_prec = SBD_FP64;
    o->use_graph = 0;
    o->use_autotune = 0;
    o->guess = nullptr;
    o->n_guess = 0;
    o->verbose = 0;
}

extern "C" int sbd_davidson(const sbd_basis* b, const sbd_exc* x, const sbd_ham* H, int nroots,
                            const sbd_davidson_opts* opts_in, double* energies, double* vectors,
                            sbd_davidson_report* report, void* stream) {
    auto t_start = clk::now();
    if (!b || !x || !H || !energies) return fail(SBD_ERR_ARG, "null argument");
    if (x->basis_id != b->id || H->basis_id != b->id || H->exc_id != x->id)
        return fail(SBD_ERR_STATE, "handles do not belong together");
    sbd_davidson_opts o;
    sbd_davidson_default_opts(&o);
    if (opts_in) o = *opts_in;
    const int64_t N = H->na * H->nb;
    const int k = nroots;
    if (k < 1 || k > 8 || k > N) return fail(SBD_ERR_ARG, "nroots must be in [1, min(8, N)]");
    if (!(o.tol_residual > 0) || o.max_iter < 1 || !(o.precond_delta > 0))
        return fail(SBD_ERR_ARG, "bad Davidson options");
    if (o.sigma_prec != SBD_FP64 && o.sigma_prec != SBD_FP32) return fail(SBD_ERR_ARG, "bad sigma_prec");
    if (o.n_guess < 0 || (o.n_guess > 0 && !o.guess)) return fail(SBD_ERR_ARG, "bad guess");
    int ms = std::max(o.max_space, 2 * k + 1);
    ms = std::min<int64_t>(ms, std::max<int64_t>(N, 1));
    ms = std::min(ms, 64);
    const int keep = std::max(k, std::min(2 * k, ms - k));
    const bool mixed = (o.sigma_prec == SBD_FP32);
    hipStream_t st = (hipStream_t)stream;
    if (o.use_autotune) {
        // launch configuration only: sigma values do not depend on it beyond rounding order
        int rc = sbd_autotune(b, x, const_cast<sbd_ham*>(H), SBD_FP64, 1, 0, stream, nullptr);
        if (!rc && mixed) rc = sbd_autotune(b, x, const_cast<sbd_ham*>(H), SBD_FP32, 1, 0, stream, nullptr);
        if (rc) return rc;
    }

    Work w;
    hipError_t e = w.V.alloc(sizeof(double) * (size_t)ms * N);
    if (e == hipSuccess) e = w.W.alloc(sizeof(double) * (size_t)ms * N);
    if (e == hipSuccess) e = w.tmp.alloc(sizeof(double) * (size_t)std::max(k, keep) * N);
    if (e == hipSuccess) e = w.scr.alloc(sizeof(double) * (size_t)keep * N);
    if (e == hipSuccess) e = w.sws.alloc(sigma_workspace_bytes(N, 1, 0, sizeof(double)));
    if (e == hipSuccess) e = w.part.alloc(sizeof(double) * 16 * kRedBlocks);
    if (e == hipSuccess) e = w.small.alloc(sizeof(double) * 64 * 16);
    if (e == hipSuccess) e = w.d_idx.alloc(sizeof(int64_t) * (kRedBlocks + 1));
    if (mixed && e == hipSuccess) e = w.d32a.alloc(sizeof(float) * (size_t)ms * N);
    if (mixed && e == hipSuccess) e = w.d32b.alloc(sizeof(float) * (size_t)ms * N);
    if (e != hipSuccess) return hip_fail(e, "sbd_davidson workspace");

    double* V = w.V.as<double>();
    double* W = w.W.as<double>();
    double* tmp = w.tmp.as<double>();
    double* part = w.part.as<double>();
    double* sm = w.small.as<double>();  // [0..64): dot results, [64..): y upload, [128..]: misc
    const double* diag = H->diag.as<double>();

    double t_sigma = 0.0, t_update = 0.0;
    int sigma_calls = 0, sigma64 = 0, restarts = 0;
    double shift = 0.0;

    // ---- lowest diagonal entries (also the FP32 shift)
    std::vector<int64_t> low_idx;
    {
        double vprev = -INFINITY;
        int64_t iprev = -1;
        int need = (o.n_guess >= k) ? 1 : k;
        for (int r = 0; r < need; ++r) {
            e = launch_argmin_after(diag, N, vprev, iprev, sm + 128, w.d_idx.as<int64_t>(), part,
                                    w.d_idx.as<int64_t>() + 1, st);
            if (e != hipSuccess) return hip_fail(e, "argmin");
            double hv;
            int64_t hi;
            SBD_HIP(hipMemcpyAsync(&hv, sm + 128, sizeof(double), hipMemcpyDeviceToHost, st));
            SBD_HIP(hipMemcpyAsync(&hi, w.d_idx.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            SBD_HIP(hipStreamSynchronize(st));
            low_idx.push_back(hi);
            vprev = hv;
            iprev = hi;
            if (r == 0) shift = hv;
        }
    }

    // sigma of vectors V[j0 .. j0+cnt) into W[j0 ..)
    auto apply_sigma = [&](int j0, int cnt, bool fp64) -> int {
        auto t0 = clk::now();
        int rc;
        if (!mixed || fp64) {
            rc = sigma_internal(x, H, cnt, SBD_FP64, 0.0, V + (size_t)j0 * N, W + (size_t)j0 * N, 0,
                                w.sws.p, st);
            sigma64 += cnt;
        } else {
            float* x32 = w.d32a.as<float>();
            float* y32 = w.d32b.as<float>();
            hipError_t ee = launch_f64_to_f32(V + (size_t)j0 * N, x32, (int64_t)cnt * N, st);
            if (ee != hipSuccess) return hip_fail(ee, "to f32");
            rc = sigma_internal(x, H, cnt, SBD_FP32, shift, x32, y32, 0, w.sws.p, st);
            if (rc) return rc;
            ee = launch_f32_to_f64_axpy(y32, V + (size_t)j0 * N, shift, W + (size_t)j0 * N,
                                        (int64_t)cnt * N, st);
            if (ee != hipSuccess) return hip_fail(ee, "from f32");
        }
        sigma_calls += cnt;
        hipError_t ee = hipStreamSynchronize(st);
        if (ee != hipSuccess) return hip_fail(ee, "sigma");
        t_sigma += ms_since(t0);
        return rc;
    };
    // h[0..m) = V[0..m)^T vec, host copy
    auto project = [&](const double* A, int m, const double* vec, std::vector<double>& out) -> int {
        out.assign(m, 0.0);
        if (m == 0) return SBD_OK;
        hipError_t ee = launch_multidot(A, m, vec, N, sm, part, st);
        if (ee != hipSuccess) return hip_fail(ee, "multidot");
        SBD_HIP(hipMemcpyAsync(out.data(), sm, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        SBD_HIP(hipStreamSynchronize(st));
        return SBD_OK;
    };
    // orthogonalise vec against V[0..m) twice; returns norm after / before
    auto orthogonalise = [&](double* vec, int m, double& nbefore, double& nafter) -> int {
        std::vector<double> h;
        int rc = project(vec, 1, vec, h);
        if (rc) return rc;
        nbefore = std::sqrt(std::max(h[0], 0.0));
        for (int pass = 0; pass < 2 && m > 0; ++pass) {
            rc = project(V, m, vec, h);
            if (rc) return rc;
            SBD_HIP(hipMemcpyAsync(sm + 64, h.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
            hipError_t ee = launch_sub_combination(V, m, sm + 64, vec, N, st);
            if (ee != hipSuccess) return hip_fail(ee, "sub_combination");
        }
        rc = project(vec, 1, vec, h);
        if (rc) return rc;
        nafter = std::sqrt(std::max(h[0], 0.0));
        return SBD_OK;
    };

    // ---- initial subspace
    int m = 0;
    if (o.n_guess > 0) {
        int ng = std::min(o.n_guess, ms - k);
        for (int g = 0; g < ng; ++g) {
            SBD_HIP(hipMemcpyAsync(V + (size_t)m * N, o.guess + (size_t)g * N, sizeof(double) * N,
                                   hipMemcpyDeviceToDevice, st));
            double nb0, nb1;
            int rc = orthogonalise(V + (size_t)m * N, m, nb0, nb1);
            if (rc) return rc;
            if (nb1 <= 1e-12 * std::max(nb0, 1e-300)) continue;
            SBD_HIP(launch_scale(V + (size_t)m * N, N, 1.0 / nb1, st));
            ++m;
        }
    }
    for (size_t r = 0; m < k && r < low_idx.size(); ++r) {
        SBD_HIP(launch_set_unit(V + (size_t)m * N, N, low_idx[r], st));
        double nb0, nb1;
        int rc = orthogonalise(V + (size_t)m * N, m, nb0, nb1);
        if (rc) return rc;
        if (nb1 <= 1e-12 * std::max(nb0, 1e-300)) continue;
        SBD_HIP(launch_scale(V + (size_t)m * N, N, 1.0 / nb1, st));
        ++m;
    }
    if (m < k) return fail(SBD_ERR_ARG, "could not form nroots independent start vectors");
    {
        // the start vectors get an exact FP64 sigma, so the first residuals are certified
        int rc = apply_sigma(0, m, true);
        if (rc) return rc;
    }
    std::vector<double> T((size_t)ms * ms, 0.0);
    for (int j = 0; j < m; ++j) {
        std::vector<double> col;
        int rc = project(V, m, W + (size_t)j * N, col);
        if (rc) return rc;
        for (int i = 0; i < m; ++i) T[i * ms + j] = col[i];
    }

    std::vector<double> theta(k, 0.0), rnorm(k, INFINITY);
    std::vector<double> evals, Z;
    int it = 0;
    bool converged = false;
    double last_true_r = INFINITY;
    int hist_n = 0;
    std::vector<double> hist_theta, hist_time;
    int status = SBD_OK;
    bool certified = true;  // residuals computed from an all-FP64 W
    double best_inner = INFINITY;
    int since_cert = 0;
    while (true) {
        ++it;
        auto tu0 = clk::now();
        // small eigenproblem on the symmetrised T
        std::vector<double> Tm((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Tm[i * m + j] = 0.5 * (T[i * ms + j] + T[j * ms + i]);
        jacobi_eigh(m, Tm, evals, Z);
        for (int r = 0; r < k; ++r) theta[r] = evals[r];
        // residuals + preconditioned corrections into tmp[r]
        for (int r = 0; r < k; ++r) {
            std::vector<double> y(m);
            for (int i = 0; i < m; ++i) y[i] = Z[i * m + r];
            SBD_HIP(hipMemcpyAsync(sm + 64, y.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
            hipError_t ee = launch_residual_precond(V, W, m, sm + 64, theta[r], diag, o.precond_delta,
                                                    tmp + (size_t)r * N, N, sm + 128, part, st);
            if (ee != hipSuccess) return hip_fail(ee, "residual");
            double rr[2];
            SBD_HIP(hipMemcpyAsync(rr, sm + 128, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
            SBD_HIP(hipStreamSynchronize(st));
            rnorm[r] = std::sqrt(std::max(rr[0], 0.0));
            if (!std::isfinite(rr[0]) || !std::isfinite(rr[1]) || !std::isfinite(theta[r]))
                return fail(SBD_ERR_NUMERIC, "non-finite residual in Davidson");
        }
        if (hist_n < 512) {
            hist_theta.push_back(theta[0]);
            hist_time.push_back(ms_since(t_start));
            ++hist_n;
        }
        if (o.verbose)
            std::fprintf(stderr, "[sbd] it %d m %d theta0 %.12f |r|max %.3e\n", it, m, theta[0],
                         *std::max_element(rnorm.begin(), rnorm.end()));
        bool inner_conv = true;
        for (int r = 0; r < k; ++r) inner_conv = inner_conv && (rnorm[r] <= o.tol_residual);
        if (inner_conv && certified) {
            converged = true;
            t_update += ms_since(tu0);
            break;
        }
        if (it >= o.max_iter) {
            t_update += ms_since(tu0);
            break;
        }
        t_update += ms_since(tu0);

        double rmax = *std::max_element(rnorm.begin(), rnorm.end());
        bool refine = false;
        if (certified) {
            last_true_r = rmax;
            best_inner = INFINITY;
            since_cert = 0;
        } else {
            // inner residuals carry the FP32 sigma error: refine when they reach the
            // target, drop well below the last certified value, stop improving, or
            // when the subspace is full
            ++since_cert;
            bool stagnant = since_cert >= 3 && rmax > 0.7 * best_inner;
            refine = inner_conv || rmax <= 0.1 * last_true_r || stagnant || (m + k > ms);
            best_inner = std::min(best_inner, rmax);
        }
        if (mixed && refine) {
            // Refinement step: collapse onto the Ritz vectors and recompute their
            // sigma in FP64; the residuals of the next pass are then exact.
            auto tr0 = clk::now();
            const int kk = std::min(keep, m);
            std::vector<double> Y((size_t)m * kk);
            for (int i = 0; i < m; ++i)
                for (int c = 0; c < kk; ++c) Y[i * kk + c] = Z[i * m + c];
            double* dY = sm + 256;
            SBD_HIP(hipMemcpyAsync(dY, Y.data(), sizeof(double) * m * kk, hipMemcpyHostToDevice, st));
            SBD_HIP(launch_combination(V, m, dY, kk, kk, tmp, N, st));
            SBD_HIP(hipMemcpyAsync(V, tmp, sizeof(double) * kk * N, hipMemcpyDeviceToDevice, st));
            m = kk;
            t_update += ms_since(tr0);
            int rc = apply_sigma(0, m, true);
            if (rc) return rc;
            for (int j = 0; j < m; ++j) {
                std::vector<double> col;
                rc = project(V, m, W + (size_t)j * N, col);
                if (rc) return rc;
                for (int i = 0; i < m; ++i) T[i * ms + j] = col[i];
            }
            ++restarts;
            certified = true;
            continue;
        }

        auto tu1 = clk::now();
        int nnew = 0;
        for (int r = 0; r < k; ++r)
            if (rnorm[r] > o.tol_residual) ++nnew;
        if (m + nnew > ms) {
            // thick restart: V <- V Y_keep, W <- W Y_keep, T <- diag(theta)
            const int kk = std::min(keep, m);
            std::vector<double> Y((size_t)m * kk);
            for (int i = 0; i < m; ++i)
                for (int c = 0; c < kk; ++c) Y[i * kk + c] = Z[i * m + c];
            double* dY = sm + 256;
            SBD_HIP(hipMemcpyAsync(dY, Y.data(), sizeof(double) * m * kk, hipMemcpyHostToDevice, st));
            // the corrections in tmp survive; the collapse goes through scr
            SBD_HIP(launch_combination(V, m, dY, kk, kk, w.scr.as<double>(), N, st));
            SBD_HIP(hipMemcpyAsync(V, w.scr.p, sizeof(double) * kk * N, hipMemcpyDeviceToDevice, st));
            SBD_HIP(launch_combination(W, m, dY, kk, kk, w.scr.as<double>(), N, st));
            SBD_HIP(hipMemcpyAsync(W, w.scr.p, sizeof(double) * kk * N, hipMemcpyDeviceToDevice, st));
            std::fill(T.begin(), T.end(), 0.0);
            for (int c = 0; c < kk; ++c) T[c * ms + c] = evals[c];
            m = kk;
            ++restarts;
        }
        int m_old = m;
        for (int r = 0; r < k; ++r) {
            if (rnorm[r] <= o.tol_residual) continue;
            double* t = tmp + (size_t)r * N;
            double n0, n1;
            int rc = orthogonalise(t, m, n0, n1);
            if (rc) return rc;
            if (!(n1 > 1e-12 * std::max(n0, 1e-300))) continue;
            SBD_HIP(hipMemcpyAsync(V + (size_t)m * N, t, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
            SBD_HIP(launch_scale(V + (size_t)m * N, N, 1.0 / n1, st));
            ++m;
        }
        t_update += ms_since(tu1);
        if (m == m_old) {
            status = SBD_NOT_CONVERGED;  // stagnation: no new direction
            break;
        }
        int rc = apply_sigma(m_old, m - m_old, false);
        if (rc) return rc;
        if (mixed) certified = false;
        auto tu2 = clk::now();
        for (int j = m_old; j < m; ++j) {
            std::vector<double> col;
            rc = project(V, m, W + (size_t)j * N, col);
            if (rc) return rc;
            for (int i = 0; i < m; ++i) {
                T[i * ms + j] = col[i];
                T[j * ms + i] = col[i];
            }
        }
        t_update += ms_since(tu2);
    }

    // ---- outputs
    for (int r = 0; r < k; ++r) energies[r] = theta[r];
    if (vectors) {
        std::vector<double> Y((size_t)m * k);
        for (int i = 0; i < m; ++i)
            for (int c = 0; c < k; ++c) Y[i * k + c] = Z[i * m + c];
        double* dY = sm + 256;
        SBD_HIP(hipMemcpyAsync(dY, Y.data(), sizeof(double) * m * k, hipMemcpyHostToDevice, st));
        SBD_HIP(launch_combination(V, m, dY, k, k, vectors, N, st));
    }
    double ortho = 0.0;
    for (int j = 0; j < m; ++j) {
        std::vector<double> col;
        int rc = project(V, m, V + (size_t)j * N, col);
        if (rc) return rc;
        for (int i = 0; i < m; ++i) {
            double d = col[i] - (i == j ? 1.0 : 0.0);
            ortho += d * d;
        }
    }
    SBD_HIP(hipStreamSynchronize(st));
    if (report) {
        report->iterations = it;
        report->sigma_calls = sigma_calls;
        report->sigma_calls_fp64 = sigma64;
        report->converged = converged ? 1 : 0;
        report->restarts = restarts;
        for (int r = 0; r < 64; ++r) report->residual[r] = r < k ? rnorm[r] : 0.0;
        report->ortho_loss = std::sqrt(ortho);
        report->t_sigma_ms = t_sigma;
        report->t_update_ms = t_update;
        report->t_total_ms = ms_since(t_start);
        report->n_history = hist_n;
        for (int i = 0; i < hist_n; ++i) {
            report->theta_history[i] = hist_theta[i];
            report->time_history_ms[i] = hist_time[i];
        }
    }
    if (status != SBD_OK) return status;
    return converged ? SBD_OK : SBD_NOT_CONVERGED;
}
