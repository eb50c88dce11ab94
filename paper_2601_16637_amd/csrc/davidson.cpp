// Davidson eigensolver driver (Sec. II-C) with device-resident FP64 vectors.
//
// Per iteration, in the paper's order: sigma of the new basis vectors,
// projected matrix T = V^T W, smallest Ritz pairs of T, residual
// r = W y - theta V y fused with the damped diagonal preconditioner (Eqs. 6-7),
// convergence test on ||r||_2, orthogonalisation of each correction against
// the subspace (two classical Gram-Schmidt passes, "twice is enough"),
// expansion, and a restart onto the lowest Ritz vectors when the subspace is
// full.  Several roots are solved together as a block.
//
// The vector work is fused sweeps over the subspace, each with its projections
// fused in (k_project.hip):
//   1. residual + preconditioner together with the first projection V^T t,
//   2. v <- t - V h1 together with |v|, V^T v and W^T v (the new column of T:
//      T_{j,new} = w_j . v_new = v_j . H v_new),
//   3. only if the first pass cancelled much of t (|v| < |t|/sqrt(2)): a second
//      classical pass v <- v - V (V^T v) with |v| and W^T v.
// Only the reduced scalars travel to the host.
//
// SBD_FP32 mode (mixed precision): sigma of new basis vectors is computed in
// FP32 on (H - shift I), shift = lowest diagonal element, and restored in
// FP64; everything else stays FP64.  Residual-correction refinement: the start
// vectors get an FP64 sigma, so the first residuals are exact.  Every basis
// vector carries a bound e_j on the error of its sigma (0 for FP64, rho for
// FP32, with rho = ||sigma32(v) - sigma64(v)|| per unit vector), and a
// combination z carries sqrt(sum_j (z_j e_j)^2).  A Ritz vector made mostly of
// exact directions plus small FP32 corrections thus has a small error even
// though each FP32 sigma is only good to ~1e-7 relative.  The subspace is
// refreshed (collapsed onto the Ritz vectors, their sigma recomputed in FP64)
// only when the inner residuals reach the target, when a root's error bound
// exceeds a fifth of its residual (or, as a fallback, after 2*max_space
// iterations without an exact residual).  Each
// refresh measures the true error of the collapsed sigma and rescales rho to
// it.  Convergence is only declared on exact (all-FP64) residuals.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <cstring>
#include <memory>
#include <tuple>
#include <vector>

#include "internal.h"

namespace sbd {

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

using clk = std::chrono::steady_clock;
inline double ms_since(clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// Offsets (in doubles) inside the small device scratch buffer.
constexpr int kRed = 0;       // reduced rows of the residual pass (<= 2*8 + 48*8)
constexpr int kH1 = 512;      // first projection (<= 48)
constexpr int kH2 = 576;      // |t'|^2, then the second projection (<= 1 + 48)
constexpr int kP2 = 640;      // |v_new|^2, then W^T v_new (<= 1 + 48)
constexpr int kY = 704;       // Ritz coefficients, m x k (<= 48 x 8)
constexpr int kTheta = 1088;  // Ritz values (<= 8)
constexpr int kYc = 1152;     // collapse coefficients, m x keep (<= 48 x 16)
constexpr int kProj = 2048;   // projection results (<= 48 x 8)
constexpr int kMisc = 3072;   // argmin value
constexpr int kOne = 3080;    // the constant 1.0 (Gram-Schmidt coefficient of a difference)
constexpr int kDiff = 3096;   // |sigma32 - sigma64|^2 rows of a refresh (2 per vector, <= 16 vectors)
constexpr int kW1 = 3200;     // fused first Gram-Schmidt pass: |t'|^2, V^T t', W^T t' (<= 1 + 48 + 48)
constexpr int kDot = 3400;    // v . w of a vector restored from an FP32 sigma
// A second classical pass runs only when the first removed more than this
// fraction of the norm: ||t'|| < ||t|| / sqrt(2) (Daniel-Gragg-Kaufman-Stewart)
constexpr double kReorth = 0.70710678118654752;
constexpr int kSmall = 4096;
constexpr int kPartRows = kPassRows;

struct OwnedStream {
    hipStream_t s = nullptr;
    ~OwnedStream() {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    }
};

struct Solver {
    const SigmaOp* op;
    hipStream_t st;
    int64_t N;
    int ms, k, keep;
    bool mixed;
    double shift = 0.0;
    DevBuf V, W, tmp, scr, part, small, idx, x32, y32, sws, x64, y64;
    double* sm = nullptr;
    double t_sigma = 0.0;
    int sigma_calls = 0, sigma64 = 0;
    int reorth = 0;          // second Gram-Schmidt passes taken
    int nvmax = 1;           // widest interleaved block sigma the staging buffers hold
    bool use_graph = false;  // replay each sigma launch sequence from a captured HIP graph
    // captured sigma sequences, keyed by (count, width, FP64); a key is captured
    // on its second use (the first runs eagerly) and serves every basis row
    std::map<std::tuple<int, int, bool>, hipGraphExec_t> graphs;
    std::map<std::tuple<int, int, bool>, int> seen;
    DevBuf rowsel;           // device int: basis row of the sigma being replayed
    // device-driven iterations: state, partial sums, captured iteration graph
    bool dev = false;
    DevBuf dls, dlpart, dlz;
    hipGraphExec_t dl_graph = nullptr;
    int dev_iters = 0;       // iterations run device-driven
    double t_device = 0.0;
    int staged_row = -1;     // basis row whose FP32 copy already sits in x32 (eager path)
    int dot_row = -1;        // basis row whose v . w the last restore left at sm + kDot
    double dot_value = 0.0;  // that v . w, read back by apply_sigma

    ~Solver() {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
        if (dl_graph) (void)hipGraphExecDestroy(dl_graph);
    }

    double* Vr(int j) { return V.as<double>() + (size_t)j * N; }
    double* Wr(int j) { return W.as<double>() + (size_t)j * N; }

    int alloc() {
        // device-driven iterations: spare rows past ms take the sigma of a stopped iteration
        const size_t rows = (size_t)ms + (dev ? kDlMaxRoots : 0);
        hipError_t e = V.alloc(sizeof(double) * rows * N);
        if (e == hipSuccess) e = W.alloc(sizeof(double) * rows * N);
        if (e == hipSuccess) e = tmp.alloc(sizeof(double) * (size_t)std::max(k, keep) * N);
        // (device-driven iterations collapse V and W together through scratch)
        if (e == hipSuccess) e = scr.alloc(sizeof(double) * (size_t)keep * N * (dev ? 2 : 1));
        if (e == hipSuccess) e = part.alloc(sizeof(double) * kPartRows * kRedBlocks);
        if (e == hipSuccess) e = small.alloc(sizeof(double) * kSmall);
        if (e == hipSuccess) e = idx.alloc(sizeof(int64_t) * (kRedBlocks + 1));
        if (e == hipSuccess) e = sws.alloc(op->ws_bytes(nvmax, nvmax > 1 ? 1 : 0, sizeof(double)));
        // FP64 staging: block sigma, graph replays, device-driven iterations
        const bool stage64 = nvmax > 1 || use_graph || dev;
        if (stage64 && e == hipSuccess) e = x64.alloc(sizeof(double) * (size_t)nvmax * N);
        if (stage64 && e == hipSuccess) e = y64.alloc(sizeof(double) * (size_t)nvmax * N);
        if ((use_graph || dev) && e == hipSuccess) e = rowsel.alloc(sizeof(int));
        if (dev && e == hipSuccess) e = dls.alloc(sizeof(DlState));
        if (dev && e == hipSuccess) e = dlpart.alloc(sizeof(double) * (size_t)kDlBlocks * kDlMaxSpace * kDlMaxRoots);
        if (dev && e == hipSuccess) e = dlz.alloc(sizeof(double) * (size_t)kDlMaxSpace * (kDlMaxSpace + 1));
        if (mixed && e == hipSuccess) e = x32.alloc(sizeof(float) * (size_t)std::max(ms, nvmax) * N);
        if (mixed && e == hipSuccess) e = y32.alloc(sizeof(float) * (size_t)std::max(ms, nvmax) * N);
        if (e != hipSuccess) return hip_fail(e, "sbd_davidson workspace");
        sm = small.as<double>();
        return SBD_OK;
    }

    // Width of the interleaved sigma for cnt vectors: 1 (one launch sequence per
    // vector) or the next power of two >= cnt (one gather walk for all of them).
    int block_width(int cnt) const {
        if (cnt < 2 || nvmax < 2) return 1;
        const int nv = cnt <= 2 ? 2 : (cnt <= 4 ? 4 : 8);
        return nv <= nvmax ? nv : 1;
    }

    // Device work of W[j .. j+c) = H V[j .. j+c): conversions, sigma, restore.
    int sigma_launches(int j, int c, int nv, bool p64) {
        int rc = SBD_OK;
        hipError_t e = hipSuccess;
        if (nv == 1) {
            if (p64) return op->apply(c, SBD_FP64, 0.0, Vr(j), Wr(j), 0, sws.p, st);
            // the Gram-Schmidt sweep may have written the FP32 copy already
            if (!(c == 1 && staged_row == j)) e = launch_f64_to_f32(Vr(j), x32.as<float>(), (int64_t)c * N, st);
            staged_row = -1;
            if (e == hipSuccess) rc = op->apply(c, SBD_FP32, shift, x32.p, y32.p, 0, sws.p, st);
            if (e == hipSuccess && !rc) {
                if (c == 1) {  // restore with the diagonal entry v . w of T
                    e = pass_restore(y32.as<float>(), Vr(j), shift, Wr(j), N, nullptr, part.as<double>(),
                                     sm + kDot, st);
                    dot_row = j;
                } else {
                    e = launch_f32_to_f64_axpy(y32.as<float>(), Vr(j), shift, Wr(j), (int64_t)c * N, st);
                }
            }
        } else if (p64) {
            e = launch_interleave<double>(Vr(j), nullptr, c, nv, N, x64.as<double>(), st);
            if (e == hipSuccess) rc = op->apply(nv, SBD_FP64, 0.0, x64.p, y64.p, 1, sws.p, st);
            if (e == hipSuccess && !rc)
                e = launch_deinterleave<double>(y64.as<double>(), c, nv, N, nullptr, 0.0, Wr(j), nullptr, st);
        } else {
            e = launch_interleave<float>(Vr(j), nullptr, c, nv, N, x32.as<float>(), st);
            if (e == hipSuccess) rc = op->apply(nv, SBD_FP32, shift, x32.p, y32.p, 1, sws.p, st);
            if (e == hipSuccess && !rc)
                e = launch_deinterleave<float>(y32.as<float>(), c, nv, N, Vr(j), shift, Wr(j), nullptr, st);
        }
        if (e != hipSuccess) return hip_fail(e, "sigma staging");
        return rc;
    }

    // Device-indexed form of the same work for graph replays: the basis row is
    // read from rowsel on the device, so one captured sequence serves every row.
    // Vectors always pass through the staging buffers (interleaved form, width 1
    // included), which makes the launch sequence independent of the row.
    int sigma_launches_indexed(int c, int nv, bool p64) {
        const int* dj = rowsel.as<int>();
        int rc = SBD_OK;
        hipError_t e = hipSuccess;
        const int layout = nv > 1 ? 1 : 0;
        if (p64) {
            e = launch_interleave<double>(V.as<double>(), dj, c, nv, N, x64.as<double>(), st);
            if (e == hipSuccess) rc = op->apply(nv, SBD_FP64, 0.0, x64.p, y64.p, layout, sws.p, st);
            if (e == hipSuccess && !rc)
                e = launch_deinterleave<double>(y64.as<double>(), c, nv, N, nullptr, 0.0, W.as<double>(), dj, st);
        } else {
            e = launch_interleave<float>(V.as<double>(), dj, c, nv, N, x32.as<float>(), st);
            if (e == hipSuccess) rc = op->apply(nv, SBD_FP32, shift, x32.p, y32.p, layout, sws.p, st);
            if (e == hipSuccess && !rc) {
                if (c == 1 && nv == 1)  // the same restore, with v . w, as the eager path
                    e = pass_restore(y32.as<float>(), V.as<double>(), shift, W.as<double>(), N, dj,
                                     part.as<double>(), sm + kDot, st);
                else
                    e = launch_deinterleave<float>(y32.as<float>(), c, nv, N, V.as<double>(), shift,
                                                   W.as<double>(), dj, st);
            }
        }
        if (e != hipSuccess) return hip_fail(e, "sigma staging");
        return rc;
    }

    // The same work, replayed from a captured graph when use_graph is set.  The
    // graph of a (count, width, precision) is captured on its second use and
    // serves every basis row: the row index is set on the device before a replay.
    int sigma_group(int j, int c, int nv, bool p64) {
        if (!use_graph) return sigma_launches(j, c, nv, p64);
        SBD_HIP(launch_set_int(rowsel.as<int>(), j, st));
        if (!p64 && c == 1 && nv == 1) dot_row = j;  // the sequence's restore leaves v . w
        const auto key = std::make_tuple(c, nv, p64);
        auto it = graphs.find(key);
        if (it == graphs.end()) {
            if (seen[key]++ == 0) return sigma_launches_indexed(c, nv, p64);  // first use: eager
            SBD_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            const int rc = sigma_launches_indexed(c, nv, p64);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(st, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "sigma capture");
            hipGraphExec_t ex = nullptr;
            const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e2 != hipSuccess) return hip_fail(e2, "sigma graph instantiate");
            it = graphs.emplace(key, ex).first;
        }
        SBD_HIP(hipGraphLaunch(it->second, st));
        return SBD_OK;
    }

    // W[j0 .. j0+cnt) = H V[j0 .. j0+cnt)
    int apply_sigma(int j0, int cnt, bool fp64) {
        auto t0 = clk::now();
        dot_row = -1;
        const bool p64 = !mixed || fp64;
        for (int d = 0; d < cnt;) {
            int c = std::min(cnt - d, 8);
            const int nv = block_width(c);
            if (nv == 1) c = 1;
            const int rc = sigma_group(j0 + d, c, nv, p64);
            if (rc) return rc;
            d += c;
        }
        staged_row = -1;  // a pre-staged copy serves only the sigma that follows it
        if (p64) sigma64 += cnt;
        sigma_calls += cnt;
        // a single vector's restore left v . w on the device: bring it back with
        // the same synchronisation
        hipError_t e = hipSuccess;
        if (cnt == 1 && dot_row == j0) e = hipMemcpyAsync(&dot_value, sm + kDot, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "sigma");
        t_sigma += ms_since(t0);
        return SBD_OK;
    }

    // One device-driven iteration (no host decision): the pre-sigma kernels, the
    // sigma of rows [m_old, m_old + k) through the staging buffers, the T update.
    int dl_launch(int nv) {
        DlState* d = dls.as<DlState>();
        SBD_HIP(dl_iteration_pre(d, V.as<double>(), W.as<double>(), op->diag, tmp.as<double>(), scr.as<double>(),
                                 N, k, ms, dlpart.as<double>(), rowsel.as<int>(), dlz.as<double>(), st));
        const int rc = sigma_launches_indexed(k, nv, !mixed);
        if (rc) return rc;
        SBD_HIP(dl_iteration_post(d, V.as<double>(), W.as<double>(), N, k, dlpart.as<double>(), st));
        return SBD_OK;
    }

    // Device-driven iterations from the host's state (m, T, error bounds) until
    // the device stops; the host reads the state back every `batch` iterations.
    // The iteration is replayed from a graph captured on first use when graphs
    // are on (one graph for every subspace size: all sizes live on the device).
    int device_batches(int batch, int max_iter, double tol, double delta, double rho, int& m,
                       std::vector<double>& T, std::vector<double>& ebound, int& since_cert, int& it,
                       int& restarts, std::vector<double>& hist_theta, std::vector<double>& hist_time,
                       int& hist_n, clk::time_point t_start) {
        const auto t0 = clk::now();
        std::unique_ptr<DlState> h(new DlState());
        std::memset(h.get(), 0, sizeof(DlState));
        h->m = m; h->k = k; h->ms = ms; h->keep = keep;
        h->it = it; h->max_iter = max_iter; h->since_cert = since_cert;
        h->tol = tol; h->delta = delta; h->rho = mixed ? rho : 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) h->T[i * ms + j] = T[i * ms + j];
        for (int j = 0; j < ms + 8 && j < kDlMaxSpace + 8; ++j) h->ebound[j] = ebound[j];
        DlState* d = dls.as<DlState>();
        SBD_HIP(hipMemcpyAsync(d, h.get(), sizeof(DlState), hipMemcpyHostToDevice, st));
        SBD_HIP(hipStreamSynchronize(st));
        static const double clock_khz = [] {
            int dev = 0, r = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&r, hipDeviceAttributeWallClockRate, dev) != hipSuccess || r <= 0)
                return 100000.0;
            return (double)r;
        }();
        const double host0 = ms_since(t_start);
        SBD_HIP(launch_clock_read(&d->hist_clock[kDlHistory - 1], st));
        const int nv = k == 1 ? 1 : block_width(k);
        const int it0 = it;
        // Batch length: the replays queued after the device stops still launch
        // (as no-ops), so each batch is sized to end near the predicted stop:
        // from each root's residual decrease per iteration over the last batch,
        // the iterations until every root meets tol (or, in mixed precision,
        // until the first root's sigma error bound reaches a fifth of its
        // residual, which asks for an FP64 refresh); at most `batch`.
        int nb = std::min(batch, 4);
        std::vector<double> r_prev(k, -1.0);
        int it_prev = it;
        while (true) {
            for (int b = 0; b < nb; ++b) {
                if (use_graph) {
                    if (!dl_graph) {
                        SBD_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                        const int rc = dl_launch(nv);
                        hipGraph_t g = nullptr;
                        const hipError_t e = hipStreamEndCapture(st, &g);
                        if (rc) {
                            if (g) (void)hipGraphDestroy(g);
                            return rc;
                        }
                        if (e != hipSuccess) return hip_fail(e, "device iteration capture");
                        const hipError_t e2 = hipGraphInstantiate(&dl_graph, g, nullptr, nullptr, 0);
                        (void)hipGraphDestroy(g);
                        if (e2 != hipSuccess) return hip_fail(e2, "device iteration graph instantiate");
                    }
                    SBD_HIP(hipGraphLaunch(dl_graph, st));
                } else {
                    const int rc = dl_launch(nv);
                    if (rc) return rc;
                }
            }
            SBD_HIP(hipMemcpyAsync(h.get(), d, sizeof(DlState), hipMemcpyDeviceToHost, st));
            SBD_HIP(hipStreamSynchronize(st));
            if (h->stop) break;
            double n_conv = 0.0, n_err = INFINITY;
            bool known = h->it > it_prev;
            for (int q = 0; q < k && known; ++q) {
                const double r = h->rnorm[q];
                if (r <= tol) continue;
                if (!(r_prev[q] > r)) {
                    known = false;
                    break;
                }
                const double lrate = std::log(r / r_prev[q]) / (double)(h->it - it_prev);
                n_conv = std::max(n_conv, std::log(tol / r) / lrate);
                if (mixed && h->ebnd[q] > 0.0) n_err = std::min(n_err, std::log(5.0 * h->ebnd[q] / r) / lrate);
            }
            for (int q = 0; q < k; ++q) r_prev[q] = h->rnorm[q];
            it_prev = h->it;
            if (known) {
                const double n = std::max(1.0, std::ceil(std::min(n_conv, n_err)));
                nb = (int)std::min<double>(n, (double)batch);
            } else {
                nb = batch;
            }
            nb = std::max(1, std::min(nb, max_iter - h->it));
        }
        // the host's view of the state
        m = h->m;
        for (int i = 0; i < ms; ++i)
            for (int j = 0; j < ms; ++j) T[i * ms + j] = (i < m && j < m) ? h->T[i * ms + j] : 0.0;
        for (int j = 0; j < ms + 8 && j < kDlMaxSpace + 8; ++j) ebound[j] = h->ebound[j];
        since_cert = h->since_cert;
        restarts += h->restarts;
        const int done = h->it - it0;
        it = h->it;
        dev_iters += done;
        sigma_calls += done * k;
        if (!mixed) sigma64 += done * k;
        const unsigned long long c0 = h->hist_clock[kDlHistory - 1];
        for (int i = 0; i < h->hist_n && hist_n < 512; ++i) {
            hist_theta.push_back(h->hist_theta[i]);
            hist_time.push_back(host0 + (double)(h->hist_clock[i] - c0) / clock_khz);
            ++hist_n;
        }
        t_device += ms_since(t0);
        return SBD_OK;
    }

    // out[j*k + q] = P_j . X_q for j < mp, q < k (host copy); k <= 8, mp <= 48
    int project(const double* P, int mp, const double* X, int k, std::vector<double>& out) {
        out.assign((size_t)mp * k, 0.0);
        if (mp == 0 || k == 0) return SBD_OK;
        SBD_HIP(pass_project(P, mp, X, k, N, part.as<double>(), sm + kProj, st));
        SBD_HIP(hipMemcpyAsync(out.data(), sm + kProj, sizeof(double) * mp * k, hipMemcpyDeviceToHost, st));
        SBD_HIP(hipStreamSynchronize(st));
        return SBD_OK;
    }

    // Orthogonalise t against V[0..m) into V[m] by classical Gram-Schmidt: a
    // first pass, and a second one when the first cancelled much of t (norm
    // below n0/sqrt(2), n0 = |t| before).  The first projection V^T t must be on
    // the device at sm+kH1.  mw rows of W have a sigma.  On return u holds
    // W[0..mw)^T v_new / |v_new| and accept tells whether the vector survived
    // (|v_new| > 1e-12 |t|).
    int orthonormalise(double* t, int m, int mw, double n0, std::vector<double>& u, bool& accept) {
        if (m >= ms) return fail(SBD_ERR_STATE, "internal: no free subspace row for a new vector");
        double* p = part.as<double>();
        u.assign(mw, 0.0);
        const double* h2 = sm + kH2 + 1;
        const double* src = t;
        if (pass_sub1w_fits(m, mw)) {
            // first pass straight into V[m], with V^T t' and W^T t' in one sweep
            SBD_HIP(pass_sub1w(V.as<double>(), m, sm + kH1, t, Vr(m), W.as<double>(), mw, N, p,
                               sm + kW1, st));
            std::vector<double> r(1 + m + mw);
            SBD_HIP(hipMemcpyAsync(r.data(), sm + kW1, sizeof(double) * r.size(), hipMemcpyDeviceToHost, st));
            SBD_HIP(hipStreamSynchronize(st));
            const double n1 = std::sqrt(std::max(r[0], 0.0));
            if (std::isfinite(n1) && n1 >= kReorth * n0 && n1 > 0.0) {
                accept = true;
                SBD_HIP(launch_scale(Vr(m), N, 1.0 / n1, st));
                for (int j = 0; j < mw; ++j) u[j] = r[1 + m + j] / n1;
                return SBD_OK;
            }
            h2 = sm + kW1 + 1;  // second pass from t' in V[m] (in place)
            src = Vr(m);
        } else {
            SBD_HIP(pass_sub1(V.as<double>(), m, sm + kH1, t, N, p, sm + kH2, st));
        }
        ++reorth;
        SBD_HIP(pass_sub2(V.as<double>(), m, h2, src, Vr(m), W.as<double>(), mw, N, p, sm + kP2, st));
        std::vector<double> r(mw + 1);
        SBD_HIP(hipMemcpyAsync(r.data(), sm + kP2, sizeof(double) * (mw + 1), hipMemcpyDeviceToHost, st));
        SBD_HIP(hipStreamSynchronize(st));
        const double n1 = std::sqrt(std::max(r[0], 0.0));
        accept = n1 > 1e-12 * std::max(n0, 1e-300) && std::isfinite(n1);
        if (!accept) return SBD_OK;
        SBD_HIP(launch_scale(Vr(m), N, 1.0 / n1, st));
        for (int j = 0; j < mw; ++j) u[j] = r[1 + j] / n1;
        return SBD_OK;
    }

    // first projection of t against V[0..m) into sm+kH1 (no host copy)
    int first_projection(const double* t, int m) {
        if (m == 0) return SBD_OK;
        SBD_HIP(pass_project(V.as<double>(), m, t, 1, N, part.as<double>(), sm + kH1, st));
        return SBD_OK;
    }

    // V[0..kk) <- V Yc, W[0..kk) <- W Yc (Yc: the first kk columns of Z)
    int collapse(const std::vector<double>& Z, int m, int kk, bool with_w) {
        std::vector<double> Y((size_t)m * kk);
        for (int i = 0; i < m; ++i)
            for (int c = 0; c < kk; ++c) Y[i * kk + c] = Z[i * m + c];
        SBD_HIP(hipMemcpyAsync(sm + kYc, Y.data(), sizeof(double) * m * kk, hipMemcpyHostToDevice, st));
        SBD_HIP(launch_combination(V.as<double>(), m, sm + kYc, kk, kk, scr.as<double>(), N, st));
        SBD_HIP(hipMemcpyAsync(V.p, scr.p, sizeof(double) * kk * N, hipMemcpyDeviceToDevice, st));
        if (with_w) {
            SBD_HIP(launch_combination(W.as<double>(), m, sm + kYc, kk, kk, scr.as<double>(), N, st));
            SBD_HIP(hipMemcpyAsync(W.p, scr.p, sizeof(double) * kk * N, hipMemcpyDeviceToDevice, st));
        }
        return SBD_OK;
    }

    // T[0..m) x [0..m) from scratch (after an FP64 refinement)
    int rebuild_T(int m, std::vector<double>& T) {
        for (int j0 = 0; j0 < m; j0 += 8) {
            const int kc = std::min(8, m - j0);
            std::vector<double> g;
            int rc = project(V.as<double>(), m, Wr(j0), kc, g);
            if (rc) return rc;
            for (int i = 0; i < m; ++i)
                for (int q = 0; q < kc; ++q) T[i * ms + j0 + q] = g[i * kc + q];
        }
        return SBD_OK;
    }
};

}  // namespace

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
    o->block_sigma = 1;
    o->device_iterations = 0;
}

extern "C" int sbd_davidson(const sbd_basis* b, const sbd_exc* x, const sbd_ham* H, int nroots,
                            const sbd_davidson_opts* opts_in, double* energies, double* vectors,
                            sbd_davidson_report* report, void* stream) {
    auto t_start = clk::now();
    if (!b || !x || !H || !energies) return fail(SBD_ERR_ARG, "null argument");
    if (x->basis_id != b->id || H->basis_id != b->id || H->exc_id != x->id)
        return fail(SBD_ERR_STATE, "handles do not belong together");
    sbd_davidson_opts o;
    const int64_t N = H->na * H->nb;
    const int k = nroots;
    int rc0 = davidson_options(k, N, opts_in, &o);
    if (rc0) return rc0;
    double t_autotune = 0.0;
    if (o.use_autotune) {
        const auto ta = clk::now();
        // launch configuration only: sigma values do not depend on it beyond rounding
        // order.  Tuned for the sigma shape the solve issues most: k interleaved
        // vectors for a block solve, single vectors otherwise.
        const int nvt = (k < 2 || !o.block_sigma) ? 1 : (k <= 2 ? 2 : (k <= 4 ? 4 : 8));
        const int lay = nvt > 1 ? 1 : 0;
        int rc = sbd_autotune(b, x, const_cast<sbd_ham*>(H), SBD_FP64, nvt, lay, stream, nullptr);
        if (!rc && o.sigma_prec == SBD_FP32)
            rc = sbd_autotune(b, x, const_cast<sbd_ham*>(H), SBD_FP32, nvt, lay, stream, nullptr);
        if (rc) return rc;
        t_autotune = ms_since(ta);
    }

    SigmaOp op;
    op.N = N;
    op.diag = H->diag.as<double>();
    op.apply = [x, H](int nvec, int prec, double shift, const void* c, void* y, int layout, void* ws,
                      hipStream_t s2) { return sigma_internal(x, H, nvec, prec, shift, c, y, layout, ws, s2); };
    op.ws_bytes = [N](int nvec, int layout, size_t elem) { return sigma_workspace_bytes(N, nvec, layout, elem); };
    return davidson_run(op, k, o, energies, vectors, report, stream, t_start, t_autotune);
}

namespace sbd {

int davidson_options(int k, int64_t N, const sbd_davidson_opts* in, sbd_davidson_opts* o) {
    sbd_davidson_default_opts(o);
    if (in) *o = *in;
    if (k < 1 || k > 8 || k > N) return fail(SBD_ERR_ARG, "nroots must be in [1, min(8, N)]");
    if (!(o->tol_residual > 0) || o->max_iter < 1 || !(o->precond_delta > 0))
        return fail(SBD_ERR_ARG, "bad Davidson options");
    if (o->sigma_prec != SBD_FP64 && o->sigma_prec != SBD_FP32) return fail(SBD_ERR_ARG, "bad sigma_prec");
    if (o->n_guess < 0 || (o->n_guess > 0 && !o->guess)) return fail(SBD_ERR_ARG, "bad guess");
    return SBD_OK;
}

int davidson_run(const SigmaOp& op, int k, const sbd_davidson_opts& o, double* energies, double* vectors,
                 sbd_davidson_report* report, void* stream, std::chrono::steady_clock::time_point t_start,
                 double t_autotune) {
    const int64_t N = op.N;
    int ms = std::max(o.max_space, 2 * k + 1);
    ms = (int)std::min<int64_t>(ms, std::max<int64_t>(N, 1));
    ms = std::min(ms, 48);
    hipStream_t st = (hipStream_t)stream;
    double t_workspace = 0.0;
    // graph capture needs a stream of its own (the legacy default stream cannot
    // be captured): the solve then runs on a private stream ordered after `stream`
    OwnedStream own;
    if (o.use_graph) {
        SBD_HIP(hipStreamSynchronize(st));
        SBD_HIP(hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking));
        st = own.s;
    }

    Solver S;
    S.op = &op;
    S.st = st;
    S.N = N;
    S.ms = ms;
    S.k = k;
    S.keep = std::max(k, std::min(2 * k, ms - k));
    S.mixed = (o.sigma_prec == SBD_FP32);
    // block solves gather all new vectors of an iteration in one interleaved sigma
    S.nvmax = (k < 2 || !o.block_sigma) ? 1 : (k <= 2 ? 2 : (k <= 4 ? 4 : 8));
    S.use_graph = o.use_graph != 0;
    S.dev = o.device_iterations > 0 && N <= kDlMaxN && k <= kDlMaxRoots && ms >= 2 * k + 1 &&
            ms <= kDlMaxSpace && S.keep <= kDlMaxKeep && (k == 1 || S.nvmax >= k);
    const auto tw = clk::now();
    int rc = S.alloc();
    if (rc) return rc;
    t_workspace = ms_since(tw);
    double* sm = S.sm;
    double* part = S.part.as<double>();
    double* tmp = S.tmp.as<double>();
    const double* diag = op.diag;
    double t_update = 0.0;
    int restarts = 0;

    // ---- lowest diagonal entries (start vectors, and the FP32 shift)
    std::vector<int64_t> low_idx;
    {
        double vprev = -INFINITY;
        int64_t iprev = -1;
        for (int r = 0; r < k; ++r) {
            hipError_t e = launch_argmin_after(diag, N, vprev, iprev, sm + kMisc, S.idx.as<int64_t>(),
                                               part, S.idx.as<int64_t>() + 1, st);
            if (e != hipSuccess) return hip_fail(e, "argmin");
            double hv;
            int64_t hi;
            SBD_HIP(hipMemcpyAsync(&hv, sm + kMisc, sizeof(double), hipMemcpyDeviceToHost, st));
            SBD_HIP(hipMemcpyAsync(&hi, S.idx.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            SBD_HIP(hipStreamSynchronize(st));
            low_idx.push_back(hi);
            vprev = hv;
            iprev = hi;
            if (r == 0) S.shift = hv;
        }
    }

    // FP32 sigma error per unit vector: start from 2^-24 max|H_ii - shift|, the
    // rounding of the dominant diagonal term; refreshes calibrate it
    double rho = 0.0;
    if (S.mixed) {
        SBD_HIP(launch_max(diag, N, sm + kMisc, part, st));
        double dmax = 0.0;
        const double one = 1.0;
        SBD_HIP(hipMemcpyAsync(&dmax, sm + kMisc, sizeof(double), hipMemcpyDeviceToHost, st));
        SBD_HIP(hipMemcpyAsync(sm + kOne, &one, sizeof(double), hipMemcpyHostToDevice, st));
        SBD_HIP(hipStreamSynchronize(st));
        rho = std::ldexp(std::max(dmax - S.shift, 1.0), -24);
    }
    std::vector<double> ebound(ms + 8, 0.0);  // error bound of each basis vector's sigma
    int refinements = 0;

    // ---- initial subspace: guesses, then the unit vectors of the k lowest
    // diagonal entries, orthonormalised.  The unit vectors are added after a
    // guess too: where H falls apart into blocks that do not couple (sparse
    // determinant lists), an iteration started in one block never leaves it,
    // and a carried guess can sit in a block that no longer holds the lowest
    // state.
    int m = 0;
    auto add_start = [&](const double* src, int64_t unit) -> int {
        double* t = tmp;
        if (src) {
            SBD_HIP(hipMemcpyAsync(t, src, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
        } else {
            SBD_HIP(launch_set_unit(t, N, unit, st));
        }
        std::vector<double> nn;
        int rc2 = S.project(t, 1, t, 1, nn);
        if (rc2) return rc2;
        rc2 = S.first_projection(t, m);
        if (rc2) return rc2;
        std::vector<double> u;
        bool ok = false;
        rc2 = S.orthonormalise(t, m, 0, std::sqrt(std::max(nn[0], 0.0)), u, ok);
        if (rc2) return rc2;
        if (ok) ++m;
        return SBD_OK;
    };
    for (int g = 0; g < o.n_guess && m < ms - k; ++g) {
        rc = add_start(o.guess + (size_t)g * N, 0);
        if (rc) return rc;
    }
    for (size_t r = 0; r < low_idx.size() && (m < k || m < ms - k); ++r) {
        rc = add_start(nullptr, low_idx[r]);
        if (rc) return rc;
    }
    if (m < k) return fail(SBD_ERR_ARG, "could not form nroots independent start vectors");
    // the start vectors' sigma in the solve's precision: in mixed precision they
    // carry the FP32 error bound like every later vector (a start vector that is
    // already an eigenvector is then certified by the first refresh)
    rc = S.apply_sigma(0, m, false);
    if (rc) return rc;
    for (int j = 0; j < m; ++j) ebound[j] = S.mixed ? rho : 0.0;
    std::vector<double> T((size_t)ms * ms, 0.0);
    rc = S.rebuild_T(m, T);
    if (rc) return rc;

    std::vector<double> theta(k, 0.0), rnorm(k, INFINITY), tnorm(k, 0.0);
    std::vector<double> evals, Z;
    int it = 0;
    bool converged = false;
    int since_cert = 0;
    bool certified = !S.mixed;  // residuals computed from an all-FP64 W
    std::vector<double> ebnd(k, 0.0);
    int hist_n = 0;
    std::vector<double> hist_theta, hist_time;
    int status = SBD_OK;
    while (true) {
        if (S.dev) {
            // device-driven iterations until the device stops; the host iteration
            // below then handles the stop (convergence, FP64 refresh, stagnation)
            int hn = hist_n;
            rc = S.device_batches(o.device_iterations, o.max_iter, o.tol_residual, o.precond_delta, rho, m, T,
                                  ebound, since_cert, it, restarts, hist_theta, hist_time, hn, t_start);
            if (rc) return rc;
            hist_n = hn;
            // the host iteration below repeats the Ritz step and residual of the
            // device's last iteration (counted there) to act on its stop
            --it;
        }
        ++it;
        auto tu0 = clk::now();
        std::vector<double> Tm((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Tm[i * m + j] = 0.5 * (T[i * ms + j] + T[j * ms + i]);
        jacobi_eigh(m, Tm, evals, Z);
        for (int r = 0; r < k; ++r) theta[r] = evals[r];
        // error bound of each Ritz vector's sigma; exact when it is zero
        certified = true;
        for (int r = 0; r < k; ++r) {
            double s2 = 0.0;
            for (int j = 0; j < m; ++j) s2 += (Z[j * m + r] * ebound[j]) * (Z[j * m + r] * ebound[j]);
            ebnd[r] = std::sqrt(s2);
            certified = certified && ebnd[r] == 0.0;
        }
        // fused residual / preconditioner for all roots with the first projections
        // V^T t_q, and W^T t_q when they fit the same sweep
        const bool with_w = pass_resid_w_fits(m, k);
        std::vector<double> red(2 * k + (size_t)(with_w ? 2 : 1) * m * k);
        {
            std::vector<double> Y((size_t)m * k);
            for (int j = 0; j < m; ++j)
                for (int q = 0; q < k; ++q) Y[j * k + q] = Z[j * m + q];
            SBD_HIP(hipMemcpyAsync(sm + kY, Y.data(), sizeof(double) * m * k, hipMemcpyHostToDevice, st));
            SBD_HIP(hipMemcpyAsync(sm + kTheta, theta.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
            if (with_w)
                SBD_HIP(pass_resid_w(S.V.as<double>(), S.W.as<double>(), m, k, sm + kY, sm + kTheta, diag,
                                     o.precond_delta, tmp, N, part, sm + kRed, st));
            else
                SBD_HIP(pass_resid(S.V.as<double>(), S.W.as<double>(), m, k, sm + kY, sm + kTheta, diag,
                                   o.precond_delta, tmp, N, true, part, sm + kRed, st));
            SBD_HIP(hipMemcpyAsync(red.data(), sm + kRed, sizeof(double) * red.size(), hipMemcpyDeviceToHost, st));
            SBD_HIP(hipStreamSynchronize(st));
            for (int q = 0; q < k; ++q) {
                if (!std::isfinite(red[q]) || !std::isfinite(red[k + q]) || !std::isfinite(theta[q]))
                    return fail(SBD_ERR_NUMERIC, "non-finite residual in Davidson");
                rnorm[q] = std::sqrt(std::max(red[q], 0.0));
                tnorm[q] = std::sqrt(std::max(red[k + q], 0.0));
            }
        }
        if (hist_n < 512) {
            hist_theta.push_back(theta[0]);
            hist_time.push_back(ms_since(t_start));
            ++hist_n;
        }
        if (o.verbose)
            std::fprintf(stderr, "[sbd] it %d m %d theta0 %.12f |r|max %.3e%s\n", it, m, theta[0],
                         *std::max_element(rnorm.begin(), rnorm.end()), certified ? " (exact)" : "");
        bool inner_conv = true;
        for (int r = 0; r < k; ++r) inner_conv = inner_conv && (rnorm[r] <= o.tol_residual);
        t_update += ms_since(tu0);
        if (inner_conv && certified) {
            converged = true;
            break;
        }
        if (it >= o.max_iter) break;

        bool refine = false;
        if (certified) {
            since_cert = 0;
        } else {
            ++since_cert;
            // No refresh merely because the residual progresses slowly: a refresh
            // collapses the subspace, and collapsing during a plateau keeps the
            // solver from ever finding a lower state the subspace is building towards.
            // The long-run fallback covers a mis-calibrated error scale.
            const bool overdue = since_cert >= 2 * ms;
            bool err_dominated = false;
            for (int r = 0; r < k; ++r)
                err_dominated = err_dominated || (rnorm[r] > o.tol_residual && ebnd[r] > 0.2 * rnorm[r]);
            refine = inner_conv || err_dominated || overdue;
        }
        if (S.mixed && refine) {
            // collapse onto the k Ritz vectors of the roots and recompute their
            // sigma in FP64; the collapsed mixed sigma (kept in tmp) calibrates rho.
            // Only the roots are kept: further kept vectors would carry FP32 error
            // bounds as large as those that forced the refresh and force the next.
            auto tr0 = clk::now();
            const int kk = std::min(k, m);
            std::vector<double> pred(kk, 0.0);
            for (int c = 0; c < kk; ++c) {
                double s2 = 0.0;
                for (int j = 0; j < m; ++j) s2 += (Z[j * m + c] * ebound[j]) * (Z[j * m + c] * ebound[j]);
                pred[c] = std::sqrt(s2);
            }
            rc = S.collapse(Z, m, kk, false);  // also leaves the coefficients at sm + kYc
            if (rc) return rc;
            SBD_HIP(launch_combination(S.W.as<double>(), m, sm + kYc, kk, kk, tmp, N, st));
            m = kk;
            t_update += ms_since(tr0);
            rc = S.apply_sigma(0, m, true);
            if (rc) return rc;
            auto tr1 = clk::now();
            std::vector<double> dif(2 * kk);
            for (int c = 0; c < kk; ++c)
                SBD_HIP(pass_sub1(S.Wr(c), 1, sm + kOne, tmp + (size_t)c * N, N, part, sm + kDiff + 2 * c, st));
            SBD_HIP(hipMemcpyAsync(dif.data(), sm + kDiff, sizeof(double) * 2 * kk, hipMemcpyDeviceToHost, st));
            SBD_HIP(hipStreamSynchronize(st));
            double amax = 0.0, pmax = 0.0;
            for (int c = 0; c < kk; ++c) {
                amax = std::max(amax, std::sqrt(std::max(dif[2 * c], 0.0)));
                pmax = std::max(pmax, pred[c]);
            }
            if (pmax > 0.0 && std::isfinite(amax))
                rho *= std::min(1e3, std::max(1e-3, amax / pmax));
            for (int c = 0; c < ms + 8; ++c) ebound[c] = 0.0;
            std::fill(T.begin(), T.end(), 0.0);
            rc = S.rebuild_T(m, T);
            if (rc) return rc;
            t_update += ms_since(tr1);
            ++refinements;
            if (o.verbose)
                std::fprintf(stderr, "[sbd] refresh: sigma32 error %.3e (bound %.3e), rho %.3e\n", amax,
                             pmax, rho);
            continue;
        }

        auto tu1 = clk::now();
        int nnew = 0;
        for (int r = 0; r < k; ++r)
            if (rnorm[r] > o.tol_residual) ++nnew;
        bool h1_valid = true;  // the residual pass projected every t_q on V[0..m)
        if (m + nnew > ms) {
            // thick restart: V <- V Y_keep, W <- W Y_keep, T <- diag(theta)
            const int kk = std::min(S.keep, m);
            std::vector<double> en(kk, 0.0);
            for (int c = 0; c < kk; ++c) {
                double s2 = 0.0;
                for (int j = 0; j < m; ++j) s2 += (Z[j * m + c] * ebound[j]) * (Z[j * m + c] * ebound[j]);
                en[c] = std::sqrt(s2);
            }
            for (int c = 0; c < ms + 8; ++c) ebound[c] = c < kk ? en[c] : 0.0;
            rc = S.collapse(Z, m, kk, true);
            if (rc) return rc;
            std::fill(T.begin(), T.end(), 0.0);
            for (int c = 0; c < kk; ++c) T[c * ms + c] = evals[c];
            m = kk;
            ++restarts;
            h1_valid = false;
        }
        const int m_old = m;
        // Block Gram-Schmidt (the block variant of Sec. II-C) when every root adds a
        // correction: one sweep subtracts V H from all k corrections and sums their
        // Gram matrix G (a second sweep when a column kept less than 1/sqrt(2) of
        // its norm), G = R^T R by Cholesky, the new basis vectors are T' R^-1 (one
        // combination), and T's new columns come from one projection of T' on W.
        // A nearly dependent block (a Cholesky pivot below 1 % of its column's
        // norm) falls back to the one-root-at-a-time path below.
        bool block_done = false;
        if (k >= 2 && nnew == k && m >= 1 && m + k <= ms && pass_subb_fits(m, k)) {
            std::vector<double> Hm((size_t)m * k);
            if (h1_valid) {
                for (int j = 0; j < m; ++j)
                    for (int q = 0; q < k; ++q) Hm[j * k + q] = red[2 * k + j * k + q];
            } else {
                rc = S.project(S.V.as<double>(), m, tmp, k, Hm);
                if (rc) return rc;
            }
            std::vector<double> G((size_t)k * k);
            for (int pass = 0; pass < 2; ++pass) {
                SBD_HIP(hipMemcpyAsync(sm + kY, Hm.data(), sizeof(double) * m * k, hipMemcpyHostToDevice, st));
                SBD_HIP(pass_subb(S.V.as<double>(), m, sm + kY, tmp, k, N, part, sm + kProj, st));
                SBD_HIP(hipMemcpyAsync(G.data(), sm + kProj, sizeof(double) * k * k, hipMemcpyDeviceToHost, st));
                SBD_HIP(hipStreamSynchronize(st));
                if (pass == 1) break;
                bool again = false;  // a column kept less than 1/sqrt(2) of its norm
                for (int q = 0; q < k; ++q)
                    if (!(G[q * k + q] >= kReorth * kReorth * tnorm[q] * tnorm[q])) again = true;
                if (!again) break;
                ++S.reorth;  // second sweep with H = V^T T'
                rc = S.project(S.V.as<double>(), m, tmp, k, Hm);
                if (rc) return rc;
            }
            // Cholesky G = R^T R (R upper), with relative pivots of at least 1e-4; a
            // column left with less than 1e-12 of its norm before the sweeps is noise
            // (the one-root path drops such a vector)
            std::vector<double> R((size_t)k * k, 0.0);
            bool ok = true;
            for (int i = 0; i < k && ok; ++i) {
                double d = G[i * k + i];
                for (int p = 0; p < i; ++p) d -= R[p * k + i] * R[p * k + i];
                if (!std::isfinite(d) || !(d > 1e-4 * G[i * k + i]) ||
                    !(G[i * k + i] > 1e-24 * tnorm[i] * tnorm[i])) {
                    ok = false;
                    break;
                }
                R[i * k + i] = std::sqrt(d);
                for (int j = i + 1; j < k; ++j) {
                    double e = G[i * k + j];
                    for (int p = 0; p < i; ++p) e -= R[p * k + i] * R[p * k + j];
                    R[i * k + j] = e / R[i * k + i];
                }
            }
            if (ok) {
                // Rinv = R^-1 (upper triangular), by back substitution column by column
                std::vector<double> Ri((size_t)k * k, 0.0);
                for (int c = 0; c < k; ++c) {
                    Ri[c * k + c] = 1.0 / R[c * k + c];
                    for (int i = c - 1; i >= 0; --i) {
                        double e = 0.0;
                        for (int p = i + 1; p <= c; ++p) e += R[i * k + p] * Ri[p * k + c];
                        Ri[i * k + c] = -e / R[i * k + i];
                    }
                }
                SBD_HIP(hipMemcpyAsync(sm + kYc, Ri.data(), sizeof(double) * k * k, hipMemcpyHostToDevice, st));
                SBD_HIP(launch_combination(tmp, k, sm + kYc, k, k, S.Vr(m), N, st));
                std::vector<double> P;
                rc = S.project(S.W.as<double>(), m, tmp, k, P);  // W^T T'
                if (rc) return rc;
                for (int j = 0; j < m; ++j)
                    for (int q = 0; q < k; ++q) {
                        double u = 0.0;
                        for (int p = 0; p <= q; ++p) u += P[j * k + p] * Ri[p * k + q];
                        T[j * ms + m + q] = T[(m + q) * ms + j] = u;
                    }
                m += k;
                block_done = true;
            } else {
                h1_valid = false;  // the corrections in tmp are now T': project them afresh
            }
        }
        for (int r = 0; r < k && !block_done; ++r) {
            if (rnorm[r] <= o.tol_residual) continue;
            // no room left: a basis of N < 2 nroots determinants restarts onto
            // more vectors than leave space for one correction per root
            if (m >= ms) break;
            double* t = tmp + (size_t)r * N;
            if (h1_valid && m == m_old) {
                // projection of root r from the residual pass: rows [2k + j*k + r)
                std::vector<double> h1(m);
                double hh = 0.0;
                for (int j = 0; j < m; ++j) {
                    h1[j] = red[2 * k + j * k + r];
                    hh += h1[j] * h1[j];
                }
                SBD_HIP(hipMemcpyAsync(sm + kH1, h1.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
                // One Gram-Schmidt pass suffices when it keeps at least 1/sqrt(2) of
                // the norm.  With V orthonormal, |t - V h|^2 = |t|^2 - |h|^2 is known
                // before the pass, and W^T (t - V h) = W^T t - (V^T W)^T h follows from
                // the residual sweep's sums and T, so the new vector takes a single
                // subtract-and-scale sweep over V and t.
                const double n0 = tnorm[r], n1sq = n0 * n0 - hh;
                if (with_w && n0 > 0.0 && std::isfinite(n1sq) && n1sq >= kReorth * kReorth * n0 * n0) {
                    const double inv = 1.0 / std::sqrt(n1sq);
                    // the FP32 copy for the coming sigma, when that sigma takes this row alone
                    const bool stage = S.mixed && !S.use_graph && S.block_width(nnew) == 1;
                    SBD_HIP(pass_subs(S.V.as<double>(), m, sm + kH1, t, inv, S.Vr(m),
                                      stage ? S.x32.as<float>() : nullptr, N, st));
                    S.staged_row = stage ? m : -1;
                    for (int j = 0; j < m; ++j) {
                        double th = red[2 * k + (size_t)m * k + j * k + r];
                        for (int i = 0; i < m; ++i) th -= h1[i] * T[i * ms + j];
                        T[j * ms + m] = T[m * ms + j] = th * inv;
                    }
                    ++m;
                    continue;
                }
            } else {
                rc = S.first_projection(t, m);
                if (rc) return rc;
            }
            std::vector<double> u;
            bool ok = false;
            rc = S.orthonormalise(t, m, m_old, tnorm[r], u, ok);
            if (rc) return rc;
            if (!ok) continue;
            for (int j = 0; j < m_old; ++j) {
                T[j * ms + m] = u[j];
                T[m * ms + j] = u[j];
            }
            ++m;
        }
        SBD_HIP(hipStreamSynchronize(st));  // the update's passes end here, not inside the sigma timer
        t_update += ms_since(tu1);
        if (m == m_old) {
            status = SBD_NOT_CONVERGED;  // stagnation: no new direction
            break;
        }
        rc = S.apply_sigma(m_old, m - m_old, false);
        if (rc) return rc;
        for (int j = m_old; j < m; ++j) ebound[j] = S.mixed ? rho : 0.0;
        auto tu2 = clk::now();
        // T entries among the new vectors: V_new^T W_new (one pass, or the
        // restore's v . w for a single vector)
        {
            const int nn = m - m_old;
            std::vector<double> g;
            if (nn == 1 && S.dot_row == m_old) {
                g.assign(1, S.dot_value);
            } else {
                rc = S.project(S.Vr(m_old), nn, S.Wr(m_old), nn, g);
            }
            if (rc) return rc;
            for (int i = 0; i < nn; ++i)
                for (int j = 0; j < nn; ++j) T[(m_old + i) * ms + m_old + j] = g[i * nn + j];
        }
        t_update += ms_since(tu2);
    }

    // ---- outputs
    for (int r = 0; r < k; ++r) energies[r] = theta[r];
    if (vectors) {
        std::vector<double> Y((size_t)m * k);
        for (int i = 0; i < m; ++i)
            for (int c = 0; c < k; ++c) Y[i * k + c] = Z[i * m + c];
        SBD_HIP(hipMemcpyAsync(sm + kYc, Y.data(), sizeof(double) * m * k, hipMemcpyHostToDevice, st));
        SBD_HIP(launch_combination(S.V.as<double>(), m, sm + kYc, k, k, vectors, N, st));
    }
    double ortho = 0.0;
    for (int j0 = 0; j0 < m; j0 += 8) {
        const int kc = std::min(8, m - j0);
        std::vector<double> g;
        rc = S.project(S.V.as<double>(), m, S.Vr(j0), kc, g);
        if (rc) return rc;
        for (int i = 0; i < m; ++i)
            for (int q = 0; q < kc; ++q) {
                const double dd = g[i * kc + q] - (i == j0 + q ? 1.0 : 0.0);
                ortho += dd * dd;
            }
    }
    SBD_HIP(hipStreamSynchronize(st));
    if (report) {
        report->iterations = it;
        report->sigma_calls = S.sigma_calls;
        report->sigma_calls_fp64 = S.sigma64;
        report->converged = converged ? 1 : 0;
        report->restarts = restarts;
        report->refinements = refinements;
        report->reorthogonalisations = S.reorth;
        report->fp32_error_scale = S.mixed ? rho : 0.0;
        for (int r = 0; r < 64; ++r) report->residual[r] = r < k ? rnorm[r] : 0.0;
        report->ortho_loss = std::sqrt(ortho);
        report->t_sigma_ms = S.t_sigma;
        report->t_update_ms = t_update;
        report->t_total_ms = ms_since(t_start);
        report->t_workspace_ms = t_workspace;
        report->t_autotune_ms = t_autotune;
        report->n_history = hist_n;
        report->device_iterations = S.dev_iters;
        report->t_device_ms = S.t_device;
        for (int i = 0; i < hist_n; ++i) {
            report->theta_history[i] = hist_theta[i];
            report->time_history_ms[i] = hist_time[i];
        }
    }
    if (status != SBD_OK) return status;
    return converged ? SBD_OK : SBD_NOT_CONVERGED;
}

}  // namespace sbd
