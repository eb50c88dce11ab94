// Device-driven Davidson iterations (Sec. II-C, the iteration of Eq. 5 with
// the damped preconditioner of Eq. 7): every decision of an iteration --
// the Ritz pairs of the projected matrix T, convergence, restart, acceptance of
// each correction -- is taken on the device from the device-resident state
// DlState, so one iteration is a fixed sequence of launches that a HIP graph
// captures once and replays for every subspace size.  Kernels of a finished or
// stopped solve return at once (the flag is read from device memory), so the
// host may queue many iterations and look at the state only every few.
//
// The small eigensolve is a parallel (round-robin ordered) Jacobi iteration
// in one workgroup; the tall-skinny sweeps are grid-stride loops with per-block
// partial sums reduced in a fixed order, so results are bitwise repeatable.
#include "internal.h"

namespace sbd {
namespace {

constexpr int kTB = 256;

__device__ __forceinline__ double wsum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// sum of one value per thread over the block (kTB threads), in every thread
__device__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = wsum(v);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    const double s = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return s;
}

// Block sums of n values per thread (n <= NMAX), one barrier: wavefront
// butterflies, then the four wavefronts' sums added in a fixed order by the
// first n threads, which write part[r * nblk + blockIdx.x]
template <int NMAX>
__device__ void block_sums_to(const double* v, int n, double (*red)[NMAX], double* part, int nblk) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < NMAX; ++r) {
        if (r < n) {
            const double x = wsum(v[r]);
            if (lane == 0) red[wv][r] = x;
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x)
        part[(size_t)r * nblk + blockIdx.x] = ((red[0][r] + red[1][r]) + red[2][r]) + red[3][r];
}

__device__ __forceinline__ double damped(double d, double delta) {
    const double a = fabs(d);
    return (d >= 0.0 ? 1.0 : -1.0) / (a > delta ? a : delta);
}

// True in the block of the grid that finishes last (after every block wrote its
// partial sums); that block then reduces them.  The counter is reset for the
// next launch.  Every block of the grid must call it.
__device__ bool last_block(unsigned* cnt) {
    __shared__ bool is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned total = gridDim.x * gridDim.y;
        const unsigned prev = atomicAdd(cnt, 1u);
        is_last = prev == total - 1;
        if (is_last) *cnt = 0u;
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last;
}

// out[r] = sum_b part[r * nblk + b] for r < rows, in a fixed order: one
// wavefront per row, its lanes striding over the blocks, then a butterfly
__device__ void reduce_rows(const double* part, int nblk, int rows, double* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int r = wv; r < rows; r += nw) {
        double s = 0.0;
        for (int b = lane; b < nblk; b += 64) s += part[(size_t)r * nblk + b];
        s = wsum(s);
        if (lane == 0) out[r] = s;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ Ritz pairs
// Eigenpairs of sym(T[0:m, 0:m]) by parallel Jacobi rotations (round-robin
// pairing: m/2 disjoint rotations per step, m-1 steps per sweep) in one
// wavefront; then the k lowest into theta / Y (m x k, ld k), the keep lowest
// into Yc (m x keep, ld keep), all eigenvalues ascending into evals; each
// eigenvector's largest component made positive.  Also the Ritz vectors'
// sigma error bounds ebnd.
__global__ void __launch_bounds__(64) k_dl_ritz(DlState* S) {
    if (S->stop) return;
    __shared__ double A[kDlMaxSpace][kDlMaxSpace + 1];
    __shared__ double Z[kDlMaxSpace][kDlMaxSpace + 1];
    __shared__ double cs[kDlMaxSpace / 2][2];
    __shared__ int pr[kDlMaxSpace / 2][2];
    __shared__ int order[kDlMaxSpace];
    const int m = S->m, tid = threadIdx.x;
    const int ms = S->ms;
    for (int e = tid; e < m * m; e += 64) {
        const int i = e / m, j = e % m;
        A[i][j] = 0.5 * (S->T[i * ms + j] + S->T[j * ms + i]);
        Z[i][j] = i == j ? 1.0 : 0.0;
    }
    // round-robin on mm = m rounded up to even (index mm-1 is a dummy when m is odd)
    const int mm = (m + 1) & ~1;
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        double o = 0.0, d = 0.0;
        for (int e = tid; e < m * m; e += 64) {
            const int i = e / m, j = e % m;
            (i == j ? d : o) += A[i][j] * A[i][j];
        }
        o = wsum(o);
        d = wsum(d);
        if (o == 0.0 || o <= 1e-30 * (d + o)) break;  // uniform: every lane holds the sums
        for (int step = 0; step < mm - 1; ++step) {
            // pairs of this step: position 0 fixed, the others rotate
            if (tid < mm / 2) {
                auto at = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + step) % (mm - 1); };
                int p = at(tid), q = at(mm - 1 - tid);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                pr[tid][0] = p;
                pr[tid][1] = q;
                double c = 1.0, s = 0.0;
                if (q < m && A[p][q] != 0.0) {
                    const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                cs[tid][0] = c;
                cs[tid][1] = s;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int e = tid; e < (mm / 2) * m; e += 64) {
                const int r = e / m, col = e % m;
                const int p = pr[r][0], q = pr[r][1];
                if (q < m) {
                    const double c = cs[r][0], s = cs[r][1];
                    const double ap = A[p][col], aq = A[q][col];
                    A[p][col] = c * ap - s * aq;
                    A[q][col] = s * ap + c * aq;
                }
            }
            __syncthreads();
            // columns: A <- A J, Z <- Z J
            for (int e = tid; e < (mm / 2) * m; e += 64) {
                const int r = e / m, row = e % m;
                const int p = pr[r][0], q = pr[r][1];
                if (q < m) {
                    const double c = cs[r][0], s = cs[r][1];
                    const double ap = A[row][p], aq = A[row][q];
                    A[row][p] = c * ap - s * aq;
                    A[row][q] = s * ap + c * aq;
                    const double zp = Z[row][p], zq = Z[row][q];
                    Z[row][p] = c * zp - s * zq;
                    Z[row][q] = s * zp + c * zq;
                }
            }
            __syncthreads();
        }
    }
    if (tid == 0) {  // ascending order (stable on ties)
        for (int i = 0; i < m; ++i) order[i] = i;
        for (int i = 1; i < m; ++i) {
            const int o = order[i];
            int j = i - 1;
            while (j >= 0 && A[order[j]][order[j]] > A[o][o]) {
                order[j + 1] = order[j];
                --j;
            }
            order[j + 1] = o;
        }
    }
    __syncthreads();
    const int k = S->k, keep = S->keep;
    for (int c = tid; c < m; c += 64) {
        const int o = order[c];
        int imax = 0;
        for (int i = 1; i < m; ++i)
            if (fabs(Z[i][o]) > fabs(Z[imax][o])) imax = i;
        const double sg = Z[imax][o] < 0.0 ? -1.0 : 1.0;
        S->evals[c] = A[o][o];
        for (int i = 0; i < m; ++i) {
            const double z = sg * Z[i][o];
            if (c < k) S->Y[i * k + c] = z;
            if (c < keep) S->Yc[i * keep + c] = z;
        }
        if (c < k) {
            S->theta[c] = A[o][o];
            double s2 = 0.0;
            for (int i = 0; i < m; ++i) {
                const double t = Z[i][o] * S->ebound[i];
                s2 += t * t;
            }
            S->ebnd[c] = sqrt(s2);
        }
    }
}

// Convergence, the mixed-precision refresh triggers, restart (one thread, from
// the reduced |r_q|^2 and |t_q|^2 in red[0, 2k)).
__device__ void dl_decide(DlState* S) {
    const int k = S->k;
    bool all = true, certified = true, err_dom = false;
    int nact = 0;
    for (int q = 0; q < k; ++q) {
        const double r2 = S->red[q], t2 = S->red[k + q];
        if (!isfinite(r2) || !isfinite(t2) || !isfinite(S->theta[q])) {
            S->stop = kDlNumeric;
            return;
        }
        S->rnorm[q] = sqrt(r2 > 0.0 ? r2 : 0.0);
        S->tnorm[q] = sqrt(t2 > 0.0 ? t2 : 0.0);
        const bool act = S->rnorm[q] > S->tol;
        S->active[q] = act;
        nact += act;
        all = all && !act;
        certified = certified && S->ebnd[q] == 0.0;
        err_dom = err_dom || (act && S->ebnd[q] > 0.2 * S->rnorm[q]);
    }
    if (S->hist_n < kDlHistory - 1) {  // the last slot holds the batch's start clock
        S->hist_theta[S->hist_n] = S->theta[0];
        S->hist_clock[S->hist_n] = __builtin_amdgcn_s_memrealtime();
        S->hist_n += 1;
    }
    S->it += 1;
    if (all && certified) {
        S->stop = kDlConverged;
        return;
    }
    if (!certified) {  // mixed precision: the host refreshes in FP64
        S->since_cert += 1;
        if (all || err_dom || S->since_cert >= 2 * S->ms) {
            S->stop = kDlRefresh;
            return;
        }
    } else {
        S->since_cert = 0;
    }
    if (S->it >= S->max_iter) {
        S->stop = kDlMaxIter;
        return;
    }
    // restart when the unconverged roots' corrections no longer fit (the sigma of
    // rows [m, m + k) may reach the spare rows past ms, which exist for this)
    S->restart = S->m + nact > S->ms;
}

// ------------------------------------------------------------------ residuals
// t_q = (W y_q - theta_q V y_q) / damped(diag - theta_q), q < k; the last block
// reduces |r_q|^2, |t_q|^2 and takes the iteration's decisions
__global__ void __launch_bounds__(kTB) k_dl_resid(DlState* S, const double* __restrict__ V,
                                                  const double* __restrict__ W, const double* __restrict__ diag,
                                                  int64_t N, double* __restrict__ t, double* __restrict__ part) {
    if (S->stop) return;
    __shared__ double red2[4][2 * kDlMaxRoots];
    const int m = S->m, k = S->k;
    double r2[kDlMaxRoots], t2[kDlMaxRoots];
#pragma unroll
    for (int q = 0; q < kDlMaxRoots; ++q) r2[q] = t2[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) {
        double vy[kDlMaxRoots], wy[kDlMaxRoots];
#pragma unroll
        for (int q = 0; q < kDlMaxRoots; ++q) vy[q] = wy[q] = 0.0;
        for (int j = 0; j < m; ++j) {
            const double v = V[(size_t)j * N + i], w = W[(size_t)j * N + i];
#pragma unroll
            for (int q = 0; q < kDlMaxRoots; ++q)
                if (q < k) {
                    const double y = S->Y[j * k + q];
                    vy[q] += v * y;
                    wy[q] += w * y;
                }
        }
        const double d = diag[i];
#pragma unroll
        for (int q = 0; q < kDlMaxRoots; ++q)
            if (q < k) {
                const double r = wy[q] - S->theta[q] * vy[q];
                const double tv = r * damped(d - S->theta[q], S->delta);
                t[(size_t)q * N + i] = tv;
                r2[q] += r * r;
                t2[q] += tv * tv;
            }
    }
    double v2[2 * kDlMaxRoots];
#pragma unroll
    for (int q = 0; q < kDlMaxRoots; ++q) {
        v2[q] = r2[q];
        v2[kDlMaxRoots + q] = t2[q];
    }
    // rows [0, k) |r|^2 and [k, 2k) |t|^2: pack t2 right after the k r2 values
#pragma unroll
    for (int q = 0; q < kDlMaxRoots; ++q)
        if (q < k) v2[k + q] = t2[q];
    block_sums_to<2 * kDlMaxRoots>(v2, 2 * k, red2, part, gridDim.x);
    if (!last_block(&S->cnt[0])) return;
    reduce_rows(part, gridDim.x, 2 * k, S->red);
    if (threadIdx.x == 0) dl_decide(S);
}

// Thick restart: rows c < keep of V Yc, then of W Yc, into scratch.
__global__ void __launch_bounds__(kTB) k_dl_collapse(const DlState* __restrict__ S, const double* __restrict__ V,
                                                     const double* __restrict__ W, int64_t N,
                                                     double* __restrict__ out) {
    if (S->stop || !S->restart) return;
    const int m = S->m, keep = S->keep;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) {
        double av[kDlMaxKeep], aw[kDlMaxKeep];
#pragma unroll
        for (int c = 0; c < kDlMaxKeep; ++c) av[c] = aw[c] = 0.0;
        for (int j = 0; j < m; ++j) {
            const double v = V[(size_t)j * N + i], w = W[(size_t)j * N + i];
#pragma unroll
            for (int c = 0; c < kDlMaxKeep; ++c)
                if (c < keep) {
                    const double y = S->Yc[j * keep + c];
                    av[c] += v * y;
                    aw[c] += w * y;
                }
        }
#pragma unroll
        for (int c = 0; c < kDlMaxKeep; ++c)
            if (c < keep) {
                out[(size_t)c * N + i] = av[c];
                out[(size_t)(keep + c) * N + i] = aw[c];
            }
    }
}

// After a restart: the collapsed rows back into V and W, then (last block)
// T = diag(lowest keep eigenvalues), the carried error bounds, m = keep.  With
// or without a restart, the iteration's Gram-Schmidt starts from m.
__global__ void __launch_bounds__(kTB) k_dl_restart_end(DlState* S, const double* __restrict__ src, int64_t N,
                                                        double* __restrict__ V, double* __restrict__ W) {
    if (S->stop) return;
    if (!S->restart) {
        if (blockIdx.x == 0 && threadIdx.x == 0) S->m_cur = S->m_old = S->m;
        return;
    }
    const int keep = S->keep;
    const int64_t n = (int64_t)keep * N;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
        V[i] = src[i];
        W[i] = src[n + i];
    }
    if (!last_block(&S->cnt[1])) return;
    if (threadIdx.x != 0) return;
    const int m = S->m, ms = S->ms;
    double eb[kDlMaxKeep];
    for (int c = 0; c < keep; ++c) {
        double s2 = 0.0;
        for (int j = 0; j < m; ++j) {
            const double t = S->Yc[j * keep + c] * S->ebound[j];
            s2 += t * t;
        }
        eb[c] = sqrt(s2);
    }
    for (int i = 0; i < ms * ms; ++i) S->T[i] = 0.0;
    for (int c = 0; c < kDlMaxSpace + 8; ++c) S->ebound[c] = c < keep ? eb[c] : 0.0;
    for (int c = 0; c < keep; ++c) S->T[c * ms + c] = S->evals[c];
    S->m = keep;
    S->m_cur = S->m_old = keep;
    S->restarts += 1;
    S->restart = 0;
}

// ------------------------------------------------------------------ Gram-Schmidt
// projections h_j = V_j . t for j < m_cur (last block: into h); only for an active root
__global__ void __launch_bounds__(kTB) k_dl_proj(DlState* S, int q, const double* __restrict__ V,
                                                 const double* __restrict__ t, int64_t N, double* __restrict__ part) {
    if (S->stop || !S->active[q]) return;
    __shared__ double redm[4][kDlMaxSpace];
    const int m = S->m_cur;
    double acc[kDlMaxSpace];
#pragma unroll
    for (int j = 0; j < kDlMaxSpace; ++j) acc[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) {
        const double x = t[i];
#pragma unroll
        for (int j = 0; j < kDlMaxSpace; ++j)
            if (j < m) acc[j] += V[(size_t)j * N + i] * x;
    }
    block_sums_to<kDlMaxSpace>(acc, m, redm, part, gridDim.x);
    if (!last_block(&S->cnt[2])) return;
    reduce_rows(part, gridDim.x, m, S->h);
}

// t <- t - sum_j h_j V_j (j < m_cur); last block: |t|^2, and after the second
// pass the acceptance of the correction (kept more than 1e-12 of its norm):
// it becomes row m_cur of V
__global__ void __launch_bounds__(kTB) k_dl_sub(DlState* S, int q, int second, const double* __restrict__ V,
                                                double* __restrict__ t, int64_t N, double* __restrict__ part) {
    if (S->stop) return;
    if (!S->active[q]) {
        if (second && blockIdx.x == 0 && threadIdx.x == 0) S->row[q] = -1;
        return;
    }
    __shared__ double red[4];
    const int m = S->m_cur;
    double n2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) {
        double x = t[i];
        for (int j = 0; j < m; ++j) x -= S->h[j] * V[(size_t)j * N + i];
        t[i] = x;
        n2 += x * x;
    }
    const double s = block_sum(n2, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (!last_block(&S->cnt[3]) || !second) return;
    double* tot_p = &S->red[kDlMaxSpace * kDlMaxRoots - 1];
    reduce_rows(part, gridDim.x, 1, tot_p);
    if (threadIdx.x != 0) return;
    const double tot = *tot_p;
    S->row[q] = -1;
    const double n1 = sqrt(tot > 0.0 ? tot : 0.0);
    const double n0 = S->tnorm[q];
    if (!(n1 > 1e-12 * (n0 > 1e-300 ? n0 : 1e-300)) || !isfinite(n1)) return;
    S->scale[q] = 1.0 / n1;
    S->row[q] = S->m_cur;
    S->m_cur += 1;
}

// root q's accepted correction into its row of V; block 0 also sets the row
// index of the coming sigma (rows [m_old, m_old + k); a stopped solve's sigma
// goes to the spare rows past ms)
__global__ void __launch_bounds__(kTB) k_dl_store(const DlState* __restrict__ S, int q,
                                                  const double* __restrict__ t, int64_t N, double* __restrict__ V,
                                                  int* rowsel) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *rowsel = S->stop ? S->ms : S->m_old;
    if (S->stop || S->row[q] < 0) return;
    const double s = S->scale[q];
    double* dst = V + (size_t)S->row[q] * N;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) dst[i] = t[i] * s;
}

// new entries of T for the new rows c < m_cur - m_old: W_i . V_{m_old + c} for
// the old rows i < m_old (in mixed precision their W may be exact FP64, which
// keeps the couplings to the refreshed Ritz vectors free of the new vectors'
// FP32 sigma error) and V_i . W_{m_old + c} among the new rows; a block of the
// grid's y dimension takes 8 rows i.  Last block: the entries into T, the new
// rows' sigma error bounds, m = m_cur; no accepted correction stops the solve
// (stagnation).
__global__ void __launch_bounds__(kTB) k_dl_tproj(DlState* S, const double* __restrict__ V,
                                                  const double* __restrict__ W, int64_t N,
                                                  double* __restrict__ part) {
    if (S->stop) return;
    __shared__ double redt[4][8 * kDlMaxRoots];
    const int m = S->m_cur, mo = S->m_old, na = S->m_cur - S->m_old;
    const int i0 = blockIdx.y * 8;
    if (i0 < m && na > 0) {
        double acc[8][kDlMaxRoots];
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int c = 0; c < kDlMaxRoots; ++c) acc[a][c] = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) {
            double vn[kDlMaxRoots], wn[kDlMaxRoots];
#pragma unroll
            for (int c = 0; c < kDlMaxRoots; ++c) {
                vn[c] = c < na ? V[(size_t)(mo + c) * N + i] : 0.0;
                wn[c] = c < na ? W[(size_t)(mo + c) * N + i] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < 8; ++a)
                if (i0 + a < m) {
                    const bool old = i0 + a < mo;
                    const double x = old ? W[(size_t)(i0 + a) * N + i] : V[(size_t)(i0 + a) * N + i];
#pragma unroll
                    for (int c = 0; c < kDlMaxRoots; ++c) acc[a][c] += x * (old ? vn[c] : wn[c]);
                }
        }
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int c = 0; c < kDlMaxRoots; ++c)
                if (c < na) {
                    const double x = wsum(acc[a][c]);
                    if (lane == 0) redt[wv][a * kDlMaxRoots + c] = x;
                }
        __syncthreads();
        for (int e = threadIdx.x; e < 8 * kDlMaxRoots; e += blockDim.x) {
            const int a = e / kDlMaxRoots, c = e % kDlMaxRoots;
            if (c < na && i0 + a < m)
                part[(size_t)((i0 + a) * kDlMaxRoots + c) * gridDim.x + blockIdx.x] =
                    ((redt[0][e] + redt[1][e]) + redt[2][e]) + redt[3][e];
        }
    }
    if (!last_block(&S->cnt[4])) return;
    {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
        for (int r = wv; r < m * kDlMaxRoots; r += nw) {
            if (r % kDlMaxRoots >= na) continue;  // uniform per wavefront
            double s = 0.0;
            for (int b = lane; b < (int)gridDim.x; b += 64) s += part[(size_t)r * gridDim.x + b];
            s = wsum(s);
            if (lane == 0) S->red[r] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int ms = S->ms;
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < na; ++c) {
            const double v = S->red[i * kDlMaxRoots + c];
            S->T[i * ms + mo + c] = v;
            S->T[(mo + c) * ms + i] = v;
        }
    for (int j = mo; j < m; ++j) S->ebound[j] = S->rho;
    if (m == mo) S->stop = kDlStagnation;
    S->m = m;
}

__global__ void k_clock(unsigned long long* out) { *out = __builtin_amdgcn_s_memrealtime(); }

inline unsigned grid_for(int64_t N) {
    const int64_t b = (N + kTB - 1) / kTB;
    return (unsigned)(b < kDlBlocks ? (b < 1 ? 1 : b) : kDlBlocks);
}

}  // namespace

hipError_t launch_clock_read(unsigned long long* out, hipStream_t st) {
    hipLaunchKernelGGL(k_clock, dim3(1), dim3(1), 0, st, out);
    return hipGetLastError();
}

// One device-driven iteration up to (not including) the sigma of the new vectors.
hipError_t dl_iteration_pre(DlState* S, double* V, double* W, const double* diag, double* tmp, double* scr,
                            int64_t N, int k, double* part, int* rowsel, hipStream_t st) {
    const unsigned g = grid_for(N);
    hipLaunchKernelGGL(k_dl_ritz, dim3(1), dim3(64), 0, st, S);
    hipLaunchKernelGGL(k_dl_resid, dim3(g), dim3(kTB), 0, st, S, V, W, diag, N, tmp, part);
    // thick restart onto the keep lowest Ritz vectors (V and W through scratch)
    hipLaunchKernelGGL(k_dl_collapse, dim3(g), dim3(kTB), 0, st, S, V, W, N, scr);
    hipLaunchKernelGGL(k_dl_restart_end, dim3(g), dim3(kTB), 0, st, S, scr, N, V, W);
    // two classical Gram-Schmidt passes per root, acceptance, the new row of V
    for (int q = 0; q < k; ++q) {
        double* t = tmp + (size_t)q * N;
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(k_dl_proj, dim3(g), dim3(kTB), 0, st, S, q, V, t, N, part);
            hipLaunchKernelGGL(k_dl_sub, dim3(g), dim3(kTB), 0, st, S, q, pass, V, t, N, part);
        }
        hipLaunchKernelGGL(k_dl_store, dim3(g), dim3(kTB), 0, st, S, q, t, N, V, rowsel);
    }
    return hipGetLastError();
}

// The rest of the iteration, after the sigma of rows [m_old, m_old + k).
hipError_t dl_iteration_post(DlState* S, const double* V, const double* W, int64_t N, double* part,
                             hipStream_t st) {
    const unsigned g = grid_for(N);
    hipLaunchKernelGGL(k_dl_tproj, dim3(g, kDlMaxSpace / 8), dim3(kTB), 0, st, S, V, W, N, part);
    return hipGetLastError();
}

}  // namespace sbd
