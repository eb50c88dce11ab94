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

// out[r] = sum_b part[r * nblk + b] for r < rows (nblk <= kDlBlocks), in a
// fixed order: one wavefront per row, its lanes striding over the blocks,
// then a butterfly.  A wavefront loads four rows' partial sums before adding
// any, so their latencies overlap.
__device__ void reduce_rows(const double* part, int nblk, int rows, double* out) {
    constexpr int kB = kDlBlocks / 64, kU = 4;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int r0 = wv; r0 < rows; r0 += nw * kU) {
        double x[kU][kB];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int r = r0 + u * nw;
#pragma unroll
            for (int c = 0; c < kB; ++c) {
                const int b = lane + 64 * c;
                x[u][c] = (r < rows && b < nblk) ? part[(size_t)r * nblk + b] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int r = r0 + u * nw;
            if (r < rows) {  // uniform per wavefront
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < kB; ++c) s += x[u][c];
                s = wsum(s);
                if (lane == 0) out[r] = s;
            }
        }
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
//
// Warm start: zbuf keeps the eigenvectors Zs (ld kDlMaxSpace) and eigenvalues
// zd of the previous call's matrix, whose zm x zm block T still leads the
// current one.  In the basis diag(Zs, I) that block is diag(zd) to within the
// previous call's convergence threshold, so the rotations start from an
// arrowhead matrix, diag(zd) bordered by the new rows Zs^T T[0:zm, zm:m], and
// accumulate onto diag(Zs, I); a few sweeps then suffice instead of a full
// solve.  zm = 0 (set by the host's upload and by a restart) starts cold.
// Round-robin pairing of mm (even) indices, pair r of a step: position 0
// stays, the others rotate by one per step (step < mm - 1, r < mm / 2).
__device__ __forceinline__ void rr_pair(int r, int step, int mm, int& p, int& q) {
    const int n1 = mm - 1;
    int a = 0;
    if (r > 0) {
        a = r - 1 + step;
        if (a >= n1) a -= n1;
        a += 1;
    }
    int b = mm - 2 - r + step;
    if (b >= n1) b -= n1;
    b += 1;
    p = a < b ? a : b;
    q = a < b ? b : a;
}

__global__ void __launch_bounds__(64) k_dl_ritz(DlState* S, double* __restrict__ zbuf) {
    if (S->stop) return;
    __shared__ double A[kDlMaxSpace][kDlMaxSpace + 1];
    __shared__ double Z[kDlMaxSpace][kDlMaxSpace + 1];
    __shared__ double arrow[kDlMaxSpace][kDlMaxRoots];
    __shared__ double2 cs[kDlMaxSpace / 2];
    __shared__ int pr[kDlMaxSpace / 2][2];
    __shared__ int order[kDlMaxSpace];
    double* Zs = zbuf;
    double* zd = zbuf + kDlMaxSpace * kDlMaxSpace;
    const int m = S->m, tid = threadIdx.x;
    const int ms = S->ms;
    const int zm0 = S->zm;
    const int zm = (zm0 > 0 && zm0 <= m && m - zm0 <= kDlMaxRoots) ? zm0 : 0;
    // lane = column j: the symmetrised T, and the starting rotation diag(Zs, I)
    if (tid < m) {
        const int j = tid;
        for (int i = 0; i < m; ++i) {
            A[i][j] = 0.5 * (S->T[i * ms + j] + S->T[j * ms + i]);
            Z[i][j] = (i < zm && j < zm) ? Zs[i * kDlMaxSpace + j] : (i == j ? 1.0 : 0.0);
        }
    }
    __syncthreads();
    if (zm > 0) {
        // lane p < zm: arrow[p][r - zm] = sum_l Zs[l][p] A[l][r] for the new rows r
        if (tid < zm) {
            for (int r = zm; r < m; ++r) {
                double s = 0.0;
                for (int l = 0; l < zm; ++l) s += Z[l][tid] * A[l][r];
                arrow[tid][r - zm] = s;
            }
        }
        __syncthreads();
        if (tid < m) {
            const int j = tid;
            for (int i = 0; i < m; ++i) {
                if (i < zm && j < zm) A[i][j] = i == j ? zd[i] : 0.0;
                else if (i < zm) A[i][j] = arrow[i][j - zm];
                else if (j < zm) A[i][j] = arrow[j][i - zm];
            }
        }
        __syncthreads();
    }
    // round-robin on mm = m rounded up to even (index mm-1 is a dummy when m is odd)
    const int mm = (m + 1) & ~1;
    // this lane's work items (pair r, index) of a rotation phase, items
    // e = tid + 64 it over the (mm / 2) x m of them, fixed for the whole call
    constexpr int kItems = (kDlMaxSpace / 2) * kDlMaxSpace / 64;
    int wr[kItems], wc[kItems];
    const int nitems = (mm / 2) * m;
    const int nit = (nitems + 63) / 64;
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int e = tid + 64 * it;
        wr[it] = e < nitems ? e / m : kDlMaxSpace / 2;  // past the items: a pair index no step has
        wc[it] = e < nitems ? e % m : 0;
    }
    bool conv = false;
    for (int sweep = 0; sweep < 40; ++sweep) {
        double o = 0.0, d = 0.0;
        if (tid < m)
            for (int i = 0; i < m; ++i) {
                const double a = A[i][tid];
                if (i == tid) d += a * a;
                else o += a * a;
            }
        o = wsum(o);
        d = wsum(d);
        if (o == 0.0 || o <= 1e-30 * (d + o)) {  // uniform: every lane holds the sums
            conv = true;
            break;
        }
        for (int step = 0; step < mm - 1; ++step) {
            const int np = mm / 2;
            if (tid < np) {
                int p, q;
                rr_pair(tid, step, mm, p, q);
                pr[tid][0] = p;
                pr[tid][1] = q;
                double c = 1.0, s = 0.0;
                if (q < m && A[p][q] != 0.0) {
                    const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                cs[tid] = make_double2(c, s);
            }
            __syncthreads();
            // rows: A <- J^T A; lane work items (pair, column) from the table
#pragma unroll
            for (int it = 0; it < kItems; ++it) {
                if (it >= nit) break;  // uniform
                const int r = wr[it], col = wc[it];
                const int p = r < np ? pr[r][0] : 0, q = r < np ? pr[r][1] : m;
                if (q < m) {
                    const double2 R = cs[r];
                    const double ap = A[p][col], aq = A[q][col];
                    A[p][col] = R.x * ap - R.y * aq;
                    A[q][col] = R.y * ap + R.x * aq;
                }
            }
            __syncthreads();
            // columns: A <- A J, Z <- Z J (the same items, col read as a row)
#pragma unroll
            for (int it = 0; it < kItems; ++it) {
                if (it >= nit) break;  // uniform
                const int r = wr[it], row = wc[it];
                const int p = r < np ? pr[r][0] : 0, q = r < np ? pr[r][1] : m;
                if (q < m) {
                    const double2 R = cs[r];
                    const double ap = A[row][p], aq = A[row][q];
                    A[row][p] = R.x * ap - R.y * aq;
                    A[row][q] = R.y * ap + R.x * aq;
                    const double zp = Z[row][p], zq = Z[row][q];
                    Z[row][p] = R.x * zp - R.y * zq;
                    Z[row][q] = R.y * zp + R.x * zq;
                }
            }
            __syncthreads();
        }
    }
    // ascending order, stable on ties: lane c's rank among the diagonal
    if (tid < m) {
        const double ev = A[tid][tid];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double e = A[j][j];
            rank += (e < ev || (e == ev && j < tid)) ? 1 : 0;
        }
        order[rank] = tid;
        // the decomposition for the next call's warm start
        for (int i = 0; i < m; ++i) Zs[i * kDlMaxSpace + tid] = Z[i][tid];
        zd[tid] = ev;
    }
    if (tid == 0) S->zm = conv ? m : 0;
    __syncthreads();
    const int k = S->k, keep = S->keep;
    if (tid < m) {
        const int c = tid;
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
// the reduced |r_q|^2 in red[q] and |t_q|^2 in red[kr + q]).
__device__ void dl_decide(DlState* S, int kr) {
    const int k = S->k;
    bool all = true, certified = true, err_dom = false;
    int nact = 0;
    for (int q = 0; q < k; ++q) {
        const double r2 = S->red[q], t2 = S->red[kr + q];
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
// The sweeps below read rows of V and W kCh at a time: a chunk's rows past m
// re-read row m - 1 (cached) and their terms are dropped, so every load of a
// chunk is issued before the first is used instead of one row at a time.
constexpr int kCh = 8;

__device__ __forceinline__ double row_at(const double* __restrict__ X, int j, int m, int64_t N, int64_t i) {
    return X[(size_t)(j < m ? j : m - 1) * N + i];
}

// t_q = (W y_q - theta_q V y_q) / damped(diag - theta_q), q < k <= KR; the last
// block reduces |r_q|^2, |t_q|^2 and takes the iteration's decisions
template <int KR>
__global__ void __launch_bounds__(kTB) k_dl_resid(DlState* S, const double* __restrict__ V,
                                                  const double* __restrict__ W, const double* __restrict__ diag,
                                                  int64_t N, double* __restrict__ t, double* __restrict__ part) {
    if (S->stop) return;
    __shared__ double red2[4][2 * KR];
    const int m = S->m, k = S->k;
    double r2[KR], t2[KR];
#pragma unroll
    for (int q = 0; q < KR; ++q) r2[q] = t2[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) {
        double vy[KR], wy[KR];
#pragma unroll
        for (int q = 0; q < KR; ++q) vy[q] = wy[q] = 0.0;
        for (int j0 = 0; j0 < m; j0 += kCh) {
            double v[kCh], w[kCh];
#pragma unroll
            for (int u = 0; u < kCh; ++u) {
                v[u] = row_at(V, j0 + u, m, N, i);
                w[u] = row_at(W, j0 + u, m, N, i);
            }
#pragma unroll
            for (int u = 0; u < kCh; ++u)
                if (j0 + u < m) {
#pragma unroll
                    for (int q = 0; q < KR; ++q)
                        if (q < k) {
                            const double y = S->Y[(j0 + u) * k + q];
                            vy[q] += v[u] * y;
                            wy[q] += w[u] * y;
                        }
                }
        }
        const double d = diag[i];
#pragma unroll
        for (int q = 0; q < KR; ++q)
            if (q < k) {
                const double r = wy[q] - S->theta[q] * vy[q];
                const double tv = r * damped(d - S->theta[q], S->delta);
                t[(size_t)q * N + i] = tv;
                r2[q] += r * r;
                t2[q] += tv * tv;
            }
    }
    // rows [0, KR): |r|^2, rows [KR, 2 KR): |t|^2
    double v2[2 * KR];
#pragma unroll
    for (int q = 0; q < KR; ++q) {
        v2[q] = r2[q];
        v2[KR + q] = t2[q];
    }
    block_sums_to<2 * KR>(v2, 2 * KR, red2, part, gridDim.x);
    if (!last_block(&S->cnt[0])) return;
    reduce_rows(part, gridDim.x, 2 * KR, S->red);
    if (threadIdx.x == 0) dl_decide(S, KR);
}

// One root (k = 1): the residual sweep above, which also takes the first
// Gram-Schmidt projections h_j = V_j . t (j < m) of the correction, so that
// pass needs no sweep of its own.  After a thick restart the new basis is
// V Yc, and its projections are Yc^T h (carried by k_dl_restart_end).
template <int NCH>
__global__ void __launch_bounds__(kTB) k_dl_resid1p(DlState* S, const double* __restrict__ V,
                                                    const double* __restrict__ W, const double* __restrict__ diag,
                                                    int64_t N, double* __restrict__ t, double* __restrict__ part) {
    if (S->stop) return;
    constexpr int R = NCH * kCh;
    __shared__ double redp[4][2 + R];
    const int m = S->m;
    const double theta = S->theta[0], delta = S->delta;
    double acc[2 + R];
#pragma unroll
    for (int j = 0; j < 2 + R; ++j) acc[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) {
        double vy = 0.0, wy = 0.0;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (c * kCh < m) {
                double v[kCh], w[kCh];
#pragma unroll
                for (int u = 0; u < kCh; ++u) {
                    v[u] = row_at(V, c * kCh + u, m, N, i);
                    w[u] = row_at(W, c * kCh + u, m, N, i);
                }
#pragma unroll
                for (int u = 0; u < kCh; ++u)
                    if (c * kCh + u < m) {
                        const double y = S->Y[c * kCh + u];
                        vy += v[u] * y;
                        wy += w[u] * y;
                    }
            }
        const double r = wy - theta * vy;
        const double tv = r * damped(diag[i] - theta, delta);
        t[i] = tv;
        acc[0] += r * r;
        acc[1] += tv * tv;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (c * kCh < m) {
                double v[kCh];
#pragma unroll
                for (int u = 0; u < kCh; ++u) v[u] = row_at(V, c * kCh + u, m, N, i);
#pragma unroll
                for (int u = 0; u < kCh; ++u) acc[2 + c * kCh + u] += v[u] * tv;  // rows >= m unused
            }
    }
    block_sums_to<2 + R>(acc, 2 + m, redp, part, gridDim.x);
    if (!last_block(&S->cnt[0])) return;
    reduce_rows(part, gridDim.x, 2, S->red);
    reduce_rows(part + 2 * (size_t)gridDim.x, gridDim.x, m, S->h);
    if (threadIdx.x == 0) dl_decide(S, 1);
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
        for (int j0 = 0; j0 < m; j0 += kCh) {
            double v[kCh], w[kCh];
#pragma unroll
            for (int u = 0; u < kCh; ++u) {
                v[u] = row_at(V, j0 + u, m, N, i);
                w[u] = row_at(W, j0 + u, m, N, i);
            }
#pragma unroll
            for (int u = 0; u < kCh; ++u)
                if (j0 + u < m) {
#pragma unroll
                    for (int c = 0; c < kDlMaxKeep; ++c)
                        if (c < keep) {
                            const double y = S->Yc[(j0 + u) * keep + c];
                            av[c] += v[u] * y;
                            aw[c] += w[u] * y;
                        }
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
                                                        double* __restrict__ V, double* __restrict__ W, int carry_h) {
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
    if (carry_h) {  // the first projections of the correction in the new basis: Yc^T h
        double hn[kDlMaxKeep];
        for (int c = 0; c < keep; ++c) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += S->Yc[j * keep + c] * S->h[j];
            hn[c] = s;
        }
        for (int c = 0; c < keep; ++c) S->h[c] = hn[c];
    }
    for (int i = 0; i < ms * ms; ++i) S->T[i] = 0.0;
    for (int c = 0; c < kDlMaxSpace + 8; ++c) S->ebound[c] = c < keep ? eb[c] : 0.0;
    for (int c = 0; c < keep; ++c) S->T[c * ms + c] = S->evals[c];
    S->m = keep;
    S->m_cur = S->m_old = keep;
    S->restarts += 1;
    S->restart = 0;
    S->zm = 0;  // T is now diagonal: the next Ritz step starts cold
}

// ------------------------------------------------------------------ Gram-Schmidt
// projections h_j = V_j . t for j < m_cur <= NCH * kCh (last block: into h);
// only for an active root
template <int NCH>
__global__ void __launch_bounds__(kTB) k_dl_proj(DlState* S, int q, const double* __restrict__ V,
                                                 const double* __restrict__ t, int64_t N, double* __restrict__ part) {
    if (S->stop || !S->active[q]) return;
    constexpr int R = NCH * kCh;
    __shared__ double redm[4][R];
    const int m = S->m_cur;
    double acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) {
        const double x = t[i];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (c * kCh < m) {
                double v[kCh];
#pragma unroll
                for (int u = 0; u < kCh; ++u) v[u] = row_at(V, c * kCh + u, m, N, i);
#pragma unroll
                for (int u = 0; u < kCh; ++u) acc[c * kCh + u] += v[u] * x;  // rows >= m unused
            }
    }
    block_sums_to<R>(acc, m, redm, part, gridDim.x);
    if (!last_block(&S->cnt[2])) return;
    reduce_rows(part, gridDim.x, m, S->h);
}

// t <- t - sum_j h_j V_j (j < m_cur, in order); last block: |t|^2, and after
// the second pass the acceptance of the correction (kept more than 1e-12 of
// its norm): it becomes row m_cur of V
template <int NCH>
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
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (c * kCh < m) {
                double v[kCh];
#pragma unroll
                for (int u = 0; u < kCh; ++u) v[u] = row_at(V, c * kCh + u, m, N, i);
#pragma unroll
                for (int u = 0; u < kCh; ++u)
                    if (c * kCh + u < m) x -= S->h[c * kCh + u] * v[u];
            }
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

// The first pass's subtraction t <- t - sum_j h_j V_j (j < m_cur, in order)
// fused with the second pass's projections h_j = V_j . t of the result (last
// block: into h)
template <int NCH>
__global__ void __launch_bounds__(kTB) k_dl_subproj(DlState* S, int q, const double* __restrict__ V,
                                                    double* __restrict__ t, int64_t N, double* __restrict__ part) {
    if (S->stop || !S->active[q]) return;
    constexpr int R = NCH * kCh;
    __shared__ double redm[4][R];
    const int m = S->m_cur;
    double acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) {
        double x = t[i];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (c * kCh < m) {
                double v[kCh];
#pragma unroll
                for (int u = 0; u < kCh; ++u) v[u] = row_at(V, c * kCh + u, m, N, i);
#pragma unroll
                for (int u = 0; u < kCh; ++u)
                    if (c * kCh + u < m) x -= S->h[c * kCh + u] * v[u];
            }
        t[i] = x;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (c * kCh < m) {
                double v[kCh];
#pragma unroll
                for (int u = 0; u < kCh; ++u) v[u] = row_at(V, c * kCh + u, m, N, i);
#pragma unroll
                for (int u = 0; u < kCh; ++u) acc[c * kCh + u] += v[u] * x;  // rows >= m unused
            }
    }
    block_sums_to<R>(acc, m, redm, part, gridDim.x);
    if (!last_block(&S->cnt[2])) return;
    reduce_rows(part, gridDim.x, m, S->h);
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

// new entries of T for the new rows c < m_cur - m_old <= KR: W_i . V_{m_old + c}
// for the old rows i < m_old (in mixed precision their W may be exact FP64,
// which keeps the couplings to the refreshed Ritz vectors free of the new
// vectors' FP32 sigma error) and V_i . W_{m_old + c} among the new rows; the
// rows i are taken kCh at a time, each chunk summed over the block before the
// next.  Last block: the entries into T, the new rows' sigma error bounds,
// m = m_cur; no accepted correction stops the solve (stagnation).
template <int KR>
__global__ void __launch_bounds__(kTB) k_dl_tproj(DlState* S, const double* __restrict__ V,
                                                  const double* __restrict__ W, int64_t N,
                                                  double* __restrict__ part) {
    if (S->stop) return;
    __shared__ double redt[4][kCh * KR];
    const int m = S->m_cur, mo = S->m_old, na = S->m_cur - S->m_old;
    const int nblk = gridDim.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (na > 0) {
        for (int a0 = 0; a0 < m; a0 += kCh) {
            double acc[kCh][KR];
#pragma unroll
            for (int a = 0; a < kCh; ++a)
#pragma unroll
                for (int c = 0; c < KR; ++c) acc[a][c] = 0.0;
            for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kTB) {
                double vn[KR], wn[KR], x[kCh];
#pragma unroll
                for (int c = 0; c < KR; ++c) {
                    const size_t r = (size_t)(mo + (c < na ? c : na - 1)) * N + i;
                    vn[c] = V[r];
                    wn[c] = W[r];
                }
#pragma unroll
                for (int a = 0; a < kCh; ++a) {
                    const int j = a0 + a < m ? a0 + a : m - 1;
                    x[a] = (j < mo ? W : V)[(size_t)j * N + i];
                }
#pragma unroll
                for (int a = 0; a < kCh; ++a) {
                    const bool old = a0 + a < mo;
#pragma unroll
                    for (int c = 0; c < KR; ++c) acc[a][c] += x[a] * (old ? vn[c] : wn[c]);
                }
            }
#pragma unroll
            for (int a = 0; a < kCh; ++a)
#pragma unroll
                for (int c = 0; c < KR; ++c)
                    if (c < na && a0 + a < m) {  // uniform
                        const double x = wsum(acc[a][c]);
                        if (lane == 0) redt[wv][a * KR + c] = x;
                    }
            __syncthreads();
            for (int e = threadIdx.x; e < kCh * KR; e += blockDim.x) {
                const int a = e / KR, c = e % KR;
                if (c < na && a0 + a < m)
                    part[(size_t)((a0 + a) * KR + c) * nblk + blockIdx.x] =
                        ((redt[0][e] + redt[1][e]) + redt[2][e]) + redt[3][e];
            }
            __syncthreads();
        }
    }
    if (!last_block(&S->cnt[4])) return;
    // rows a * KR + c; those with c >= na hold no partial sums and are not used
    reduce_rows(part, nblk, m * KR, S->red);
    if (threadIdx.x != 0) return;
    const int ms = S->ms;
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < na; ++c) {
            const double v = S->red[i * KR + c];
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

namespace {

template <int KR>
void launch_pre(DlState* S, double* V, double* W, const double* diag, double* tmp, double* scr, int64_t N, int k,
                int nch, double* part, int* rowsel, double* zbuf, hipStream_t st) {
    const unsigned g = grid_for(N);
    const bool one = KR == 1;  // one root: the residual sweep also takes the first projections
    hipLaunchKernelGGL(k_dl_ritz, dim3(1), dim3(64), 0, st, S, zbuf);
    if (one) {
        switch (nch) {
#define SBD_DL_R1(C)                                                                                    \
    case C:                                                                                             \
        hipLaunchKernelGGL(k_dl_resid1p<C>, dim3(g), dim3(kTB), 0, st, S, V, W, diag, N, tmp, part);    \
        break;
            SBD_DL_R1(1)
            SBD_DL_R1(2)
            SBD_DL_R1(3)
            SBD_DL_R1(4)
            SBD_DL_R1(5)
            default:
            SBD_DL_R1(6)
#undef SBD_DL_R1
        }
    } else {
        hipLaunchKernelGGL(k_dl_resid<KR>, dim3(g), dim3(kTB), 0, st, S, V, W, diag, N, tmp, part);
    }
    // thick restart onto the keep lowest Ritz vectors (V and W through scratch)
    hipLaunchKernelGGL(k_dl_collapse, dim3(g), dim3(kTB), 0, st, S, V, W, N, scr);
    hipLaunchKernelGGL(k_dl_restart_end, dim3(g), dim3(kTB), 0, st, S, scr, N, V, W, one ? 1 : 0);
    // two classical Gram-Schmidt passes per root (the first subtraction fused
    // with the second projection), acceptance, the new row of V
    for (int q = 0; q < k; ++q) {
        double* t = tmp + (size_t)q * N;
        switch (nch) {
#define SBD_DL_GS(C)                                                                                    \
    case C:                                                                                             \
        if (!one) hipLaunchKernelGGL(k_dl_proj<C>, dim3(g), dim3(kTB), 0, st, S, q, V, t, N, part);     \
        hipLaunchKernelGGL(k_dl_subproj<C>, dim3(g), dim3(kTB), 0, st, S, q, V, t, N, part);            \
        hipLaunchKernelGGL(k_dl_sub<C>, dim3(g), dim3(kTB), 0, st, S, q, 1, V, t, N, part);             \
        break;
            SBD_DL_GS(1)
            SBD_DL_GS(2)
            SBD_DL_GS(3)
            SBD_DL_GS(4)
            SBD_DL_GS(5)
            default:
            SBD_DL_GS(6)
#undef SBD_DL_GS
        }
        hipLaunchKernelGGL(k_dl_store, dim3(g), dim3(kTB), 0, st, S, q, t, N, V, rowsel);
    }
}

}  // namespace

// One device-driven iteration up to (not including) the sigma of the new vectors.
hipError_t dl_iteration_pre(DlState* S, double* V, double* W, const double* diag, double* tmp, double* scr,
                            int64_t N, int k, int ms, double* part, int* rowsel, double* zbuf, hipStream_t st) {
    if (k < 1 || k > kDlMaxRoots || ms < 1 || ms > kDlMaxSpace) return hipErrorInvalidValue;
    const int nch = (ms + kCh - 1) / kCh;
    if (k == 1) launch_pre<1>(S, V, W, diag, tmp, scr, N, k, nch, part, rowsel, zbuf, st);
    else if (k == 2) launch_pre<2>(S, V, W, diag, tmp, scr, N, k, nch, part, rowsel, zbuf, st);
    else if (k <= 4) launch_pre<4>(S, V, W, diag, tmp, scr, N, k, nch, part, rowsel, zbuf, st);
    else launch_pre<8>(S, V, W, diag, tmp, scr, N, k, nch, part, rowsel, zbuf, st);
    return hipGetLastError();
}

// The rest of the iteration, after the sigma of rows [m_old, m_old + k).
hipError_t dl_iteration_post(DlState* S, const double* V, const double* W, int64_t N, int k, double* part,
                             hipStream_t st) {
    const unsigned g = grid_for(N);
    if (k == 1) hipLaunchKernelGGL(k_dl_tproj<1>, dim3(g), dim3(kTB), 0, st, S, V, W, N, part);
    else if (k == 2) hipLaunchKernelGGL(k_dl_tproj<2>, dim3(g), dim3(kTB), 0, st, S, V, W, N, part);
    else if (k <= 4) hipLaunchKernelGGL(k_dl_tproj<4>, dim3(g), dim3(kTB), 0, st, S, V, W, N, part);
    else hipLaunchKernelGGL(k_dl_tproj<8>, dim3(g), dim3(kTB), 0, st, S, V, W, N, part);
    return hipGetLastError();
}

}  // namespace sbd
