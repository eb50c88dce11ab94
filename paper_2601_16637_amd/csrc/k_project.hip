// Tall-skinny passes of the Davidson update (Sec. II-C).
//
// Every pass is one sweep over the N determinants; each thread owns EPT
// determinants per grid-stride step and keeps, in registers, the values of all
// subspace rows it needs for them (at most MB rows, loaded back to back so a
// wavefront has MB-deep memory-level parallelism).  From those registers it
// computes the elementwise result (residual + damped preconditioner, or the
// Gram-Schmidt subtraction t - V h, or just the vectors to project), writes
// it, and accumulates the projections G[j][q] = P_j . out_q in registers.  HBM
// sees every byte once; nothing is re-read and the sweep has no barrier.
//
// The projections are a tall-skinny product with at most eight columns: well
// under one FP64 flop per byte of HBM traffic, so the pass is bound by HBM and
// runs on the vector ALUs (on gfx950 the FP64 matrix-core peak is no higher
// than the FP64 vector peak).
//
// Each block reduces its accumulators (wavefront shuffles, then the four
// wavefronts in LDS in a fixed order) and writes part[row][block]; rows are
// reduced across blocks in a fixed order afterwards, so results are bitwise
// repeatable.  Row layout:
//   [0, NR)              norms (mode dependent, see below)
//   [NR + j*k + q)       G[j][q] = P_j . out_q   for j < mp, q < k
// When a projection does not fit the register budget of a pass, the pass runs
// without it and a separate projection pass fills the same rows.  RESIDW is
// RESID that also projects every correction on W (rows [2k + m*k + j*k + q)),
// so that a Gram-Schmidt step that needs one pass can take the new column of
// V^T W from these sums; SUBS is the subtraction (t - V h) * s with no sums;
// SUBB subtracts V H from k vectors at once and sums their k x k Gram matrix
// (rows [q1*k + q2)), the first step of a block Gram-Schmidt.
#include <algorithm>

#include "internal.h"

namespace sbd {
namespace {

constexpr int kTB = 256;       // threads per block
constexpr int kMaxOut = 8;     // output vectors per pass

enum Mode { RESID = 0, SUB1 = 1, SUB2 = 2, PROJ = 3, SUBW = 4, RESIDW = 5, SUBS = 6, SUBB = 7 };

struct PassArgs {
    int64_t N;
    int m;            // rows of V combined elementwise (RESID, SUB1, SUB2)
    int k;            // output vectors
    int mp;           // rows of the projected matrix P (0: no projection)
    int mw;           // SUBW: rows of W projected besides the m rows of V
    const double* V;  // subspace basis, row j at V + j*N
    const double* W;  // sigma of the basis
    const double* P;  // projected matrix (V or W or A)
    const double* X;  // PROJ: k input vectors; SUB1/SUB2: t
    double* out;      // RESID: k corrections; SUB1: t (in place); SUB2, SUBW: destination
    const double* coef;   // RESID: Y (m x k, row-major); SUB: h (m)
    const double* theta;  // RESID: k Ritz values
    const double* diag;
    double delta;
    double scale;     // SUBS: factor applied to t - V h
    float* out32;     // SUBS: optional FP32 copy of the result
    double* part;
};

__device__ __forceinline__ double damped_inv(double d, double delta) {
    const double a = fabs(d);
    const double den = a > delta ? a : delta;
    return (d >= 0.0 ? 1.0 : -1.0) / den;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

constexpr int ept_for(int mb) { return mb <= 8 ? 2 : 1; }

// MODE: pass kind; MB: bound on rows held per determinant (m and mp <= MB);
// KO: bound on outputs (k <= KO); PRJ: whether the pass accumulates projections.
template <int MODE, int MB, int KO, bool PRJ>
__global__ void __launch_bounds__(kTB) k_pass(PassArgs A) {
    constexpr int EPT = ept_for(MB);
    constexpr bool RES = MODE == RESID || MODE == RESIDW;
    constexpr int NAJ = MODE == SUBB ? KO : (PRJ ? ((MODE == SUBW || MODE == RESIDW) ? 2 * MB : MB) : 1);
    constexpr int NAQ = (RES || MODE == PROJ || MODE == SUBB) ? KO : 1;  // accumulator columns
    __shared__ double red[4][MODE == SUBW ? 1 + 2 * MB
                             : MODE == SUBS ? 1
                             : MODE == RESIDW ? 2 * kMaxOut + 2 * MB * KO
                             : MODE == SUBB ? KO * KO
                                              : 2 * kMaxOut + MB * KO];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = A.m, k = A.k, mp = A.mp;
    const int64_t N = A.N;
    const double* __restrict__ cf = A.coef;
    // multi-root residual passes read their m x k coefficients from LDS (broadcast
    // reads), which keeps them out of the scalar registers, and load every row
    // without a branch (rows past m load row m-1, a cache hit; their terms are
    // dropped by selects, never multiplied in): with k > 1 the scalar registers
    // cannot hold the coefficients and branch-guarded loads serialise.  With one
    // root the guarded form measures faster.
    constexpr bool STAGED = (RES || MODE == SUBB) && KO > 1;
    __shared__ double ys[STAGED ? MB * KO : 1];
    if constexpr (STAGED) {
        for (int i = threadIdx.x; i < m * k; i += kTB) ys[i] = cf[i];
        __syncthreads();
    }

    double acc[NAJ][NAQ];
#pragma unroll
    for (int j = 0; j < NAJ; ++j)
#pragma unroll
        for (int q = 0; q < NAQ; ++q) acc[j][q] = 0.0;
    double nrm[2 * KO];
#pragma unroll
    for (int q = 0; q < 2 * KO; ++q) nrm[q] = 0.0;
    double th[KO];
#pragma unroll
    for (int q = 0; q < KO; ++q) th[q] = (RES && q < k) ? A.theta[q] : 0.0;

    const int64_t step = (int64_t)gridDim.x * kTB * EPT;
    for (int64_t base = (int64_t)blockIdx.x * kTB * EPT + tid; base < N; base += step) {
        int64_t ix[EPT];
        bool in[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            ix[u] = base + (int64_t)u * kTB;
            in[u] = ix[u] < N;
        }
        if constexpr (RES) {
            double v[MB][EPT], w[MB][EPT], d[EPT];
#pragma unroll
            for (int j = 0; j < MB; ++j) {
                if constexpr (STAGED) {
                    const size_t jr = (size_t)(j < m ? j : m - 1);
#pragma unroll
                    for (int u = 0; u < EPT; ++u) {
                        v[j][u] = in[u] ? A.V[jr * N + ix[u]] : 0.0;
                        w[j][u] = in[u] ? A.W[jr * N + ix[u]] : 0.0;
                    }
                } else if (j < m) {
#pragma unroll
                    for (int u = 0; u < EPT; ++u) {
                        v[j][u] = in[u] ? A.V[(size_t)j * N + ix[u]] : 0.0;
                        w[j][u] = in[u] ? A.W[(size_t)j * N + ix[u]] : 0.0;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < EPT; ++u) d[u] = in[u] ? A.diag[ix[u]] : 0.0;
#pragma unroll
            for (int q = 0; q < KO; ++q) {
                if (q < k) {
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    double vy = 0.0, wy = 0.0;
#pragma unroll
                    for (int j = 0; j < MB; ++j) {
                        if constexpr (STAGED) {
                            const double c = ys[(j < m ? j : 0) * k + q];
                            vy += j < m ? v[j][u] * c : 0.0;
                            wy += j < m ? w[j][u] * c : 0.0;
                        } else if (j < m) {
                            vy += v[j][u] * cf[j * k + q];
                            wy += w[j][u] * cf[j * k + q];
                        }
                    }
                    const double r = wy - th[q] * vy;
                    const double t = in[u] ? r * damped_inv(d[u] - th[q], A.delta) : 0.0;
                    if (in[u]) A.out[(size_t)q * N + ix[u]] = t;
                    nrm[q] += r * r;
                    nrm[KO + q] += t * t;
                    if constexpr (PRJ) {
#pragma unroll
                        for (int j = 0; j < MB; ++j)
                            if (j < mp) acc[j][q] += v[j][u] * t;
                    }
                    if constexpr (MODE == RESIDW) {
#pragma unroll
                        for (int j = 0; j < MB; ++j)
                            if (j < mp) acc[MB + j][q] += w[j][u] * t;
                    }
                }
                }
            }
        } else if constexpr (MODE == SUBB) {
            // t'_q = t_q - sum_j V_j H[j][q] for q < k (in place allowed), Gram t'^T t';
            // rows loaded without branches as in the staged residual pass
            double v[MB][EPT], x[KO][EPT];
#pragma unroll
            for (int q = 0; q < KO; ++q) {
                const size_t qr = (size_t)(q < k ? q : k - 1);
#pragma unroll
                for (int u = 0; u < EPT; ++u) x[q][u] = in[u] ? A.X[qr * N + ix[u]] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < MB; ++j) {
                const size_t jr = (size_t)(j < m ? j : m - 1);
#pragma unroll
                for (int u = 0; u < EPT; ++u) v[j][u] = in[u] ? A.V[jr * N + ix[u]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                double o[KO];
#pragma unroll
                for (int q = 0; q < KO; ++q) {
                    o[q] = 0.0;
                    if (q < k) {
                        double sv = 0.0;
#pragma unroll
                        for (int j = 0; j < MB; ++j) {
                            const double c = STAGED ? ys[(j < m ? j : 0) * k + q] : cf[(j < m ? j : 0) * k + q];
                            sv += j < m ? v[j][u] * c : 0.0;
                        }
                        o[q] = in[u] ? x[q][u] - sv : 0.0;
                        if (in[u]) A.out[(size_t)q * N + ix[u]] = o[q];
                    }
                }
#pragma unroll
                for (int q1 = 0; q1 < KO; ++q1)
#pragma unroll
                    for (int q2 = 0; q2 < KO; ++q2)
                        if (q1 < k && q2 < k) acc[q1][q2] += o[q1] * o[q2];
            }
        } else if constexpr (MODE == SUBS) {
            double v[MB][EPT], x[EPT];
#pragma unroll
            for (int u = 0; u < EPT; ++u) x[u] = in[u] ? A.X[ix[u]] : 0.0;
#pragma unroll
            for (int j = 0; j < MB; ++j)
                if (j < m) {
#pragma unroll
                    for (int u = 0; u < EPT; ++u) v[j][u] = in[u] ? A.V[(size_t)j * N + ix[u]] : 0.0;
                }
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                double sv = 0.0;
#pragma unroll
                for (int j = 0; j < MB; ++j)
                    if (j < m) sv += v[j][u] * cf[j];
                if (in[u]) {
                    const double o = (x[u] - sv) * A.scale;
                    A.out[ix[u]] = o;
                    if (A.out32) A.out32[ix[u]] = (float)o;
                }
            }
        } else if constexpr (MODE == SUB1 || MODE == SUB2) {
            double v[MB][EPT], x[EPT];
            double w[PRJ && MODE == SUB2 ? MB : 1][EPT];
#pragma unroll
            for (int u = 0; u < EPT; ++u) x[u] = in[u] ? A.X[ix[u]] : 0.0;
#pragma unroll
            for (int j = 0; j < MB; ++j)
                if (j < m) {
#pragma unroll
                    for (int u = 0; u < EPT; ++u) v[j][u] = in[u] ? A.V[(size_t)j * N + ix[u]] : 0.0;
                }
            if constexpr (PRJ && MODE == SUB2) {
#pragma unroll
                for (int j = 0; j < MB; ++j)
                    if (j < mp) {
#pragma unroll
                        for (int u = 0; u < EPT; ++u) w[j][u] = in[u] ? A.W[(size_t)j * N + ix[u]] : 0.0;
                    }
            }
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                double sv = 0.0;
#pragma unroll
                for (int j = 0; j < MB; ++j)
                    if (j < m) sv += v[j][u] * cf[j];
                const double t = in[u] ? x[u] - sv : 0.0;
                if (in[u]) A.out[ix[u]] = t;
                nrm[0] += t * t;
                if constexpr (PRJ) {
#pragma unroll
                    for (int j = 0; j < MB; ++j)
                        if (j < mp) acc[j][0] += (MODE == SUB1 ? v[j][u] : w[MODE == SUB2 ? j : 0][u]) * t;
                }
            }
        } else if constexpr (MODE == SUBW) {
            // t' = t - V h with both projections V^T t' (a possible second pass) and
            // W^T t' (the new column of T when one pass suffices)
            double v[MB][EPT], w[MB][EPT], x[EPT];
            const int mw = A.mw;
#pragma unroll
            for (int u = 0; u < EPT; ++u) x[u] = in[u] ? A.X[ix[u]] : 0.0;
#pragma unroll
            for (int j = 0; j < MB; ++j)
                if (j < m) {
#pragma unroll
                    for (int u = 0; u < EPT; ++u) v[j][u] = in[u] ? A.V[(size_t)j * N + ix[u]] : 0.0;
                }
#pragma unroll
            for (int j = 0; j < MB; ++j)
                if (j < mw) {
#pragma unroll
                    for (int u = 0; u < EPT; ++u) w[j][u] = in[u] ? A.W[(size_t)j * N + ix[u]] : 0.0;
                }
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                double sv = 0.0;
#pragma unroll
                for (int j = 0; j < MB; ++j)
                    if (j < m) sv += v[j][u] * cf[j];
                const double t = in[u] ? x[u] - sv : 0.0;
                if (in[u]) A.out[ix[u]] = t;
                nrm[0] += t * t;
#pragma unroll
                for (int j = 0; j < MB; ++j) {
                    if (j < m) acc[j][0] += v[j][u] * t;
                    if (j < mw) acc[MB + j][0] += w[j][u] * t;
                }
            }
        } else {  // PROJ
            // with several vectors, rows loaded without branches (past the end: the
            // last row again, a cache hit; those sums are never stored)
            double p[MB][EPT], x[KO][EPT];
#pragma unroll
            for (int q = 0; q < KO; ++q) {
                if constexpr (KO > 1) {
                    const size_t qr = (size_t)(q < k ? q : k - 1);
#pragma unroll
                    for (int u = 0; u < EPT; ++u) x[q][u] = in[u] ? A.X[qr * N + ix[u]] : 0.0;
                } else if (q < k) {
#pragma unroll
                    for (int u = 0; u < EPT; ++u) x[q][u] = in[u] ? A.X[(size_t)q * N + ix[u]] : 0.0;
                }
            }
#pragma unroll
            for (int j = 0; j < MB; ++j) {
                if constexpr (KO > 1) {
                    const size_t jr = (size_t)(j < mp ? j : mp - 1);
#pragma unroll
                    for (int u = 0; u < EPT; ++u) p[j][u] = in[u] ? A.P[jr * N + ix[u]] : 0.0;
                } else if (j < mp) {
#pragma unroll
                    for (int u = 0; u < EPT; ++u) p[j][u] = in[u] ? A.P[(size_t)j * N + ix[u]] : 0.0;
                }
            }
#pragma unroll
            for (int j = 0; j < MB; ++j)
                if (j < mp) {
#pragma unroll
                    for (int q = 0; q < KO; ++q)
                        if (q < k) {
#pragma unroll
                            for (int u = 0; u < EPT; ++u) acc[j][q] += p[j][u] * x[q][u];
                        }
                }
        }
    }

    // ---- block reduction: wavefront shuffles, then the four wavefronts in order
    if constexpr (MODE == SUBS) return;  // no sums
    const int NR = RES ? 2 * k : ((MODE == PROJ || MODE == SUBB) ? 0 : 1);
    const int kq = (RES || MODE == PROJ || MODE == SUBB) ? k : 1;
#pragma unroll
    for (int q = 0; q < 2 * KO; ++q) {
        const double x = wave_sum(nrm[q]);
        if (lane == 0) {
            // RESID: [0,k) |r_q|^2, [k,2k) |t_q|^2;  SUB: [0] |t|^2
            if (RES && q < KO && q < k) red[wv][q] = x;
            if (RES && q >= KO && q - KO < k) red[wv][k + q - KO] = x;
            if ((MODE == SUB1 || MODE == SUB2 || MODE == SUBW) && q == 0) red[wv][0] = x;
        }
    }
    if constexpr (MODE == SUBB) {
#pragma unroll
        for (int q1 = 0; q1 < KO; ++q1)
#pragma unroll
            for (int q2 = 0; q2 < KO; ++q2) {
                const double x = wave_sum(acc[q1][q2]);
                if (lane == 0 && q1 < k && q2 < k) red[wv][q1 * k + q2] = x;
            }
    } else if constexpr (MODE == SUBW) {
        // rows [1 + j) V_j . t' (j < m), then [1 + m + j) W_j . t' (j < mw)
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            const double xv = wave_sum(acc[j][0]);
            const double xw = wave_sum(acc[MB + j][0]);
            if (lane == 0 && j < m) red[wv][1 + j] = xv;
            if (lane == 0 && j < A.mw) red[wv][1 + m + j] = xw;
        }
    } else if constexpr (PRJ) {
#pragma unroll
        for (int j = 0; j < NAJ; ++j)
#pragma unroll
            for (int q = 0; q < NAQ; ++q) {
                const double x = wave_sum(acc[j][q]);
                // RESIDW: W rows follow the mp*k V rows
                const int jj = j < MB ? j : j - MB, off = j < MB ? 0 : mp * kq;
                if (lane == 0 && jj < mp && q < kq) red[wv][NR + off + jj * kq + q] = x;
            }
    }
    __syncthreads();
    const int rows = (MODE == SUBW)   ? 1 + m + A.mw
                     : (MODE == SUBB) ? k * k
                                      : NR + (PRJ ? (MODE == RESIDW ? 2 : 1) * mp * kq : 0);
    for (int r = tid; r < rows; r += kTB)
        A.part[(size_t)r * gridDim.x + blockIdx.x] = ((red[0][r] + red[1][r]) + red[2][r]) + red[3][r];
}

// out[r] = sum_b part[r][b], fixed order, one block per row
__global__ void k_reduce(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    __shared__ double sh[kTB];
    const int r = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kTB) s += part[(size_t)r * nblk + b];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = kTB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = sh[0];
}

// y = (double)y32 + shift * x with the block partials of x . y in part[block]
// (the FP32 sigma of a basis vector restored to FP64, and its diagonal entry
// of V^T W, in one sweep)
// (row: optional device index; x and y then point at row *row of V and W)
__global__ void __launch_bounds__(kTB) k_restore(const float* __restrict__ y32, const double* __restrict__ xb,
                                                 double shift, double* __restrict__ yb, int64_t N,
                                                 const int* __restrict__ row, double* __restrict__ part) {
    __shared__ double red[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t off = row ? (int64_t)row[0] * N : 0;
    const double* __restrict__ x = xb + off;
    double* __restrict__ y = yb + off;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + tid; i < N; i += (int64_t)gridDim.x * kTB) {
        const double xv = x[i];
        const double w = (double)y32[i] + shift * xv;
        y[i] = w;
        acc += xv * w;
    }
    acc = wave_sum(acc);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (tid == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Register budget (FP64 values held per thread, two VGPRs each): the row
// values of the pass plus its accumulators.  Beyond it a projection is split off.
constexpr int kRegBudget = 96;

int mb_for(int rows) {
    const int steps[] = {4, 8, 16, 24, 32, 48};
    for (int s : steps)
        if (rows <= s) return s;
    return -1;
}
int ko_for(int k) { return k <= 1 ? 1 : (k <= 2 ? 2 : (k <= 4 ? 4 : (k <= 8 ? 8 : -1))); }

// FP64 values held per thread by an instantiation: row values plus accumulators
constexpr int held(int mode, int mb, int ko, bool prj) {
    return ept_for(mb) *
           ((mode == RESID)  ? 2 * mb + (prj ? mb * ko : 0)
            : (mode == RESIDW) ? 2 * mb + 2 * mb * ko
            : (mode == SUBS)   ? mb + 1
            : (mode == SUBB)   ? mb + ko + ko * ko
            : (mode == SUB1) ? mb + (prj ? mb : 0)
            : (mode == SUB2) ? mb + (prj ? 2 * mb : 0)
            : (mode == SUBW) ? 4 * mb
                             : mb + ko + mb * ko);
}
// Instantiations that exist: the PRJ forms within the budget; the non-PRJ
// Gram-Schmidt forms (also used with no subspace yet, m = 0); the non-PRJ
// residual forms where the PRJ form of the same size does not fit.
constexpr bool exists(int mode, int mb, int ko, bool prj) {
    return mode == SUBW                                 ? ko == 1 && prj && held(mode, mb, 1, true) <= kRegBudget
           : mode == RESIDW                          ? prj && held(mode, mb, ko, true) <= kRegBudget
           : mode == SUBS                            ? ko == 1 && !prj
           : mode == SUBB                            ? prj && held(mode, mb, ko, true) <= kRegBudget
           : (mode == SUB1 || mode == SUB2) && ko != 1 ? false
           : prj                                    ? held(mode, mb, ko, true) <= kRegBudget
           : mode == PROJ                           ? false
           : mode == RESID                          ? held(mode, mb, ko, true) > kRegBudget
                                                    : true;
}

template <int MODE, int MB, int KO, bool PRJ>
hipError_t launch_k(const PassArgs& A, unsigned* nb_out, hipStream_t st) {
    if constexpr (!exists(MODE, MB, KO, PRJ)) {
        return hipErrorInvalidValue;
    } else {
    // one resident wave of blocks per CU slot: fill the chip once, then grid-stride
    // (thread-safe one-time query per instantiation; single-device library state)
    static const int slots = [] {
        int dev = 0, cus = 0, nbk = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nbk, k_pass<MODE, MB, KO, PRJ>, kTB, 0) !=
                hipSuccess)
            return 256;
        return std::max(1, nbk) * std::max(1, cus);
    }();
    const int64_t per_block = (int64_t)kTB * ept_for(MB);
    int64_t nb = (A.N + per_block - 1) / per_block;
    const int64_t cap = std::min<int64_t>(slots, kRedBlocks);
    if (nb > cap) nb = cap;
    if (nb < 1) nb = 1;
    *nb_out = (unsigned)nb;
    hipLaunchKernelGGL((k_pass<MODE, MB, KO, PRJ>), dim3((unsigned)nb), dim3(kTB), 0, st, A);
    return hipGetLastError();
    }
}

template <int MODE, int KO, bool PRJ>
hipError_t by_mb(int mb, const PassArgs& A, unsigned* nb, hipStream_t st) {
    switch (mb) {
        case 4: return launch_k<MODE, 4, KO, PRJ>(A, nb, st);
        case 8: return launch_k<MODE, 8, KO, PRJ>(A, nb, st);
        case 16: return launch_k<MODE, 16, KO, PRJ>(A, nb, st);
        case 24: return launch_k<MODE, 24, KO, PRJ>(A, nb, st);
        case 32: return launch_k<MODE, 32, KO, PRJ>(A, nb, st);
        case 48: return launch_k<MODE, 48, KO, PRJ>(A, nb, st);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE, bool PRJ>
hipError_t by_ko(int ko, int mb, const PassArgs& A, unsigned* nb, hipStream_t st) {
    switch (ko) {
        case 1: return by_mb<MODE, 1, PRJ>(mb, A, nb, st);
        case 2: return by_mb<MODE, 2, PRJ>(mb, A, nb, st);
        case 4: return by_mb<MODE, 4, PRJ>(mb, A, nb, st);
        case 8: return by_mb<MODE, 8, PRJ>(mb, A, nb, st);
        default: return hipErrorInvalidValue;
    }
}

bool fits(int mode, int rows, int k, bool prj) {
    const int mb = mb_for(rows), ko = ko_for(k);
    return mb > 0 && ko > 0 &&
           held(mode, mb, (mode == SUB1 || mode == SUB2 || mode == SUBW || mode == SUBS) ? 1 : ko, prj) <=
               kRegBudget;
}

// One pass; `rows` results reduced into out.  The caller checked fits().
hipError_t run_pass(int mode, const PassArgs& A, int rows, double* out, hipStream_t st) {
    const bool prj = A.mp > 0;
    const int need = std::max({mode == PROJ ? 0 : A.m, A.mp, mode == SUBW ? A.mw : 0});
    const int mb = mb_for(need < 1 ? 1 : need);
    const int ko = (mode == RESID || mode == RESIDW || mode == PROJ || mode == SUBB) ? ko_for(A.k) : 1;
    if (mb < 0 || ko < 0 || rows > kPassRows) return hipErrorInvalidValue;
    if (mode == SUBW && !fits(SUBW, need, 1, true)) return hipErrorInvalidValue;
    unsigned nb = 0;
    hipError_t e = hipErrorInvalidValue;
    if (mode == RESID) e = prj ? by_ko<RESID, true>(ko, mb, A, &nb, st) : by_ko<RESID, false>(ko, mb, A, &nb, st);
    else if (mode == RESIDW) e = by_ko<RESIDW, true>(ko, mb, A, &nb, st);
    else if (mode == SUBS) e = by_mb<SUBS, 1, false>(mb, A, &nb, st);
    else if (mode == SUBB) e = by_ko<SUBB, true>(ko, mb, A, &nb, st);
    else if (mode == SUB1) e = prj ? by_mb<SUB1, 1, true>(mb, A, &nb, st) : by_mb<SUB1, 1, false>(mb, A, &nb, st);
    else if (mode == SUB2) e = prj ? by_mb<SUB2, 1, true>(mb, A, &nb, st) : by_mb<SUB2, 1, false>(mb, A, &nb, st);
    else if (mode == SUBW) e = by_mb<SUBW, 1, true>(mb, A, &nb, st);
    else e = by_ko<PROJ, true>(ko, mb, A, &nb, st);
    if (e != hipSuccess) return e;
    if (rows > 0) hipLaunchKernelGGL(k_reduce, dim3(rows), dim3(kTB), 0, st, A.part, (int)nb, out);
    return hipGetLastError();
}

}  // namespace
}  // namespace sbd

namespace sbd {

hipError_t pass_project(const double* P, int mp, const double* X, int k, int64_t N, double* part,
                        double* out, hipStream_t st) {
    if (mp < 1 || mp > 48 || k < 1 || k > kMaxOut) return hipErrorInvalidValue;
    // row groups small enough for the register budget; each group is one sweep over X
    int step = mp;
    while (step > 1 && !fits(PROJ, step, k, true)) step = (step + 1) / 2;
    if (!fits(PROJ, step, k, true)) return hipErrorInvalidValue;
    for (int j0 = 0; j0 < mp; j0 += step) {
        PassArgs A{};
        const int g = std::min(step, mp - j0);
        A.N = N; A.m = 0; A.k = k; A.mp = g;
        A.P = P + (size_t)j0 * N; A.X = X; A.part = part;
        hipError_t e = run_pass(PROJ, A, g * k, out + (size_t)j0 * k, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t pass_resid(const double* V, const double* W, int m, int k, const double* Y,
                      const double* theta, const double* diag, double delta, double* T, int64_t N,
                      bool proj, double* part, double* out, hipStream_t st) {
    if (m < 1 || m > 48 || k < 1 || k > kMaxOut) return hipErrorInvalidValue;
    // the fused form whenever it fits (without proj its projection rows are not reduced)
    const bool fused = fits(RESID, m, k, true);
    PassArgs A{};
    A.N = N; A.m = m; A.k = k; A.mp = fused ? m : 0;
    A.V = V; A.W = W; A.P = V; A.out = T; A.coef = Y; A.theta = theta; A.diag = diag;
    A.delta = delta; A.part = part;
    hipError_t e = run_pass(RESID, A, 2 * k + (proj ? A.mp * k : 0), out, st);
    if (e == hipSuccess && proj && !fused) e = pass_project(V, m, T, k, N, part, out + 2 * k, st);
    return e;
}

hipError_t pass_restore(const float* y32, const double* x, double shift, double* y, int64_t N,
                        const int* row, double* part, double* out, hipStream_t st) {
    static const int slots = [] {
        int dev = 0, cus = 0, nbk = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nbk, k_restore, kTB, 0) != hipSuccess)
            return 256;
        return std::max(1, nbk) * std::max(1, cus);
    }();
    int64_t nb = (N + kTB - 1) / kTB;
    nb = std::min<int64_t>(nb, std::min<int64_t>(slots, kRedBlocks));
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_restore, dim3((unsigned)nb), dim3(kTB), 0, st, y32, x, shift, y, N, row, part);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kTB), 0, st, part, (int)nb, out);
    return hipGetLastError();
}

bool pass_resid_w_fits(int m, int k) { return m >= 1 && k >= 1 && k <= kMaxOut && fits(RESIDW, m, k, true); }

hipError_t pass_resid_w(const double* V, const double* W, int m, int k, const double* Y,
                        const double* theta, const double* diag, double delta, double* T, int64_t N,
                        double* part, double* out, hipStream_t st) {
    if (!pass_resid_w_fits(m, k)) return hipErrorInvalidValue;
    PassArgs A{};
    A.N = N; A.m = m; A.k = k; A.mp = m;
    A.V = V; A.W = W; A.P = V; A.out = T; A.coef = Y; A.theta = theta; A.diag = diag;
    A.delta = delta; A.part = part;
    return run_pass(RESIDW, A, 2 * k + 2 * m * k, out, st);
}

bool pass_subb_fits(int m, int k) { return m >= 1 && k >= 1 && k <= kMaxOut && fits(SUBB, m, k, true); }

hipError_t pass_subb(const double* V, int m, const double* H, double* T, int k, int64_t N, double* part,
                     double* out, hipStream_t st) {
    if (!pass_subb_fits(m, k)) return hipErrorInvalidValue;
    PassArgs A{};
    A.N = N; A.m = m; A.k = k; A.mp = m;
    A.V = V; A.X = T; A.out = T; A.coef = H; A.part = part;
    return run_pass(SUBB, A, k * k, out, st);
}

hipError_t pass_subs(const double* V, int m, const double* h, const double* t, double s, double* dst,
                     float* dst32, int64_t N, hipStream_t st) {
    if (m < 1 || m > 48 || !fits(SUBS, m, 1, false)) return hipErrorInvalidValue;
    PassArgs A{};
    A.N = N; A.m = m; A.k = 1; A.mp = 0;
    A.V = V; A.X = t; A.out = dst; A.out32 = dst32; A.coef = h; A.scale = s;
    return run_pass(SUBS, A, 0, nullptr, st);
}

hipError_t pass_sub1(const double* V, int m, const double* h, double* t, int64_t N, double* part,
                     double* out, hipStream_t st) {
    if (m < 0 || m > 48) return hipErrorInvalidValue;
    const bool fused = m > 0 && fits(SUB1, m, 1, true);
    PassArgs A{};
    A.N = N; A.m = m; A.k = 1; A.mp = fused ? m : 0;
    A.V = V; A.P = V; A.X = t; A.out = t; A.coef = h; A.part = part;
    hipError_t e = run_pass(SUB1, A, 1 + A.mp, out, st);
    if (e == hipSuccess && m > 0 && !fused) e = pass_project(V, m, t, 1, N, part, out + 1, st);
    return e;
}

bool pass_sub1w_fits(int m, int mw) {
    return m >= 1 && mw >= 0 && fits(SUBW, std::max(m, mw), 1, true);
}

hipError_t pass_sub1w(const double* V, int m, const double* h, const double* t, double* dst,
                      const double* W, int mw, int64_t N, double* part, double* out, hipStream_t st) {
    if (!pass_sub1w_fits(m, mw)) return hipErrorInvalidValue;
    PassArgs A{};
    A.N = N; A.m = m; A.k = 1; A.mp = m; A.mw = mw;
    A.V = V; A.W = W; A.X = t; A.out = dst; A.coef = h; A.part = part;
    return run_pass(SUBW, A, 1 + m + mw, out, st);
}

hipError_t pass_sub2(const double* V, int m, const double* h, const double* t, double* dst,
                     const double* W, int mw, int64_t N, double* part, double* out, hipStream_t st) {
    if (m < 0 || m > 48 || mw < 0 || mw > 48) return hipErrorInvalidValue;
    const bool fused = mw > 0 && fits(SUB2, std::max(m, mw), 1, true);
    PassArgs A{};
    A.N = N; A.m = m; A.k = 1; A.mp = fused ? mw : 0;
    A.V = V; A.W = W; A.P = W; A.X = t; A.out = dst; A.coef = h; A.part = part;
    hipError_t e = run_pass(SUB2, A, 1 + A.mp, out, st);
    if (e == hipSuccess && mw > 0 && !fused) e = pass_project(W, mw, dst, 1, N, part, out + 1, st);
    return e;
}

}  // namespace sbd
