// Tall-skinny passes of the Davidson update (Sec. II-C).
//
// Every pass walks the N determinants in tiles of 256 (one element per
// thread).  An elementwise phase computes up to eight output vectors for the
// tile (residual + damped preconditioner, or a Gram-Schmidt subtraction
// t - V h, or just loads the vectors to project) and stages them in LDS.  A
// contraction phase then accumulates G += P[:, tile]^T out[tile, :]: wavefront
// w owns the rows j = w, w+4, ... of P and re-reads them with one coalesced
// 512-byte load per 64 determinants (the rows were just streamed by the
// elementwise phase, so these loads hit L2), multiplying with the outputs in
// LDS.  Each (row, output) accumulator lives in exactly one wavefront, so the
// register budget is (rows per wave) x (outputs) and HBM sees every byte once.
//
// Each block writes its partial sums to part[row][block]; rows are reduced in a
// fixed order afterwards (deterministic).  Row layout:
//   [0, NR)              norms (mode dependent, see below)
//   [NR + j*k + q)       G[j][q] = P_j . out_q   for j < mp, q < k
#include "internal.h"

namespace sbd {
namespace {

constexpr int kTB = 256;       // threads per block = determinants per tile
constexpr int kMaxOut = 8;     // output vectors per pass

enum Mode { RESID = 0, SUB1 = 1, SUB2 = 2, PROJ = 3 };

struct PassArgs {
    int64_t N;
    int mode;
    int m;            // rows of V used by the elementwise phase
    int k;            // output vectors
    int mp;           // rows of the projected matrix P
    const double* V;  // subspace basis, row j at V + j*N
    const double* W;  // sigma of the basis
    const double* P;  // projected matrix (V or W or A)
    const double* X;  // PROJ: k input vectors; SUB1/SUB2: t
    double* out;      // RESID: k corrections; SUB1: t (in place); SUB2: destination
    const double* coef;   // RESID: Y (m x k, row-major); SUB: h (m)
    const double* theta;  // RESID: k Ritz values
    const double* diag;
    double delta;
    double* part;
};

__device__ __forceinline__ double damped_inv(double d, double delta) {
    const double a = fabs(d);
    const double den = a > delta ? a : delta;
    return (d >= 0.0 ? 1.0 : -1.0) / den;
}

// JW = rows of P per wavefront (mp <= 4*JW), KO = outputs (k <= KO).
template <int JW, int KO>
__global__ void __launch_bounds__(kTB) k_pass(PassArgs A) {
    __shared__ double ot[KO][kTB];          // outputs of the tile, [q][e]
    __shared__ double cs[64 * kMaxOut];     // Y or h
    __shared__ double th[kMaxOut];
    __shared__ double nsum[4][2 * kMaxOut];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = A.m, k = A.k, mp = A.mp;
    const int ncoef = (A.mode == RESID) ? m * k : ((A.mode == PROJ) ? 0 : m);
    for (int i = tid; i < ncoef; i += kTB) cs[i] = A.coef[i];
    if (A.mode == RESID && tid < k) th[tid] = A.theta[tid];
    __syncthreads();

    double acc[JW][KO];
#pragma unroll
    for (int jj = 0; jj < JW; ++jj)
#pragma unroll
        for (int q = 0; q < KO; ++q) acc[jj][q] = 0.0;
    double nrm[2 * KO];
#pragma unroll
    for (int q = 0; q < 2 * KO; ++q) nrm[q] = 0.0;

    const int64_t N = A.N;
    for (int64_t c0 = (int64_t)blockIdx.x * kTB; c0 < N; c0 += (int64_t)gridDim.x * kTB) {
        const int64_t i = c0 + tid;
        const bool in = i < N;
        // ---- elementwise phase: one determinant per thread
        if (A.mode == RESID) {
            double vy[KO], wy[KO];
#pragma unroll
            for (int q = 0; q < KO; ++q) vy[q] = wy[q] = 0.0;
            if (in) {
#pragma unroll 4
                for (int j = 0; j < m; ++j) {
                    const double vj = A.V[(size_t)j * N + i];
                    const double wj = A.W[(size_t)j * N + i];
#pragma unroll
                    for (int q = 0; q < KO; ++q)
                        if (q < k) {
                            vy[q] += vj * cs[j * k + q];
                            wy[q] += wj * cs[j * k + q];
                        }
                }
            }
            const double d = in ? A.diag[i] : 0.0;
#pragma unroll
            for (int q = 0; q < KO; ++q) {
                if (q < k) {
                    const double r = wy[q] - th[q] * vy[q];
                    const double tq = in ? r * damped_inv(d - th[q], A.delta) : 0.0;
                    if (in) A.out[(size_t)q * N + i] = tq;
                    nrm[q] += in ? r * r : 0.0;
                    nrm[KO + q] += tq * tq;
                    ot[q][tid] = tq;
                }
            }
        } else if (A.mode == SUB1 || A.mode == SUB2) {
            double s = 0.0;
            if (in) {
#pragma unroll 4
                for (int j = 0; j < m; ++j) s += A.V[(size_t)j * N + i] * cs[j];
            }
            const double tv = in ? A.X[i] - s : 0.0;
            if (in) A.out[i] = tv;
            nrm[0] += tv * tv;
            ot[0][tid] = tv;
        } else {  // PROJ
#pragma unroll
            for (int q = 0; q < KO; ++q)
                if (q < k) ot[q][tid] = in ? A.X[(size_t)q * N + i] : 0.0;
        }
        __syncthreads();
        // ---- contraction phase: wave wv owns rows j = wv + 4*jj of P
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
            const int j = wv + 4 * jj;
            if (j >= mp) break;  // uniform within the wave
            const double* pr = A.P + (size_t)j * N + c0;
#pragma unroll
            for (int g = 0; g < kTB / 64; ++g) {
                const int e = 64 * g + lane;
                const double a = (c0 + e < N) ? pr[e] : 0.0;
#pragma unroll
                for (int q = 0; q < KO; ++q)
                    if (q < k) acc[jj][q] += a * ot[q][e];
            }
        }
        __syncthreads();
    }
    // ---- reductions: norms over the block, projections within their wave
#pragma unroll
    for (int q = 0; q < 2 * KO; ++q) {
        double x = nrm[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) nsum[wv][q] = x;
    }
    __syncthreads();
    const int NR = (A.mode == RESID) ? 2 * k : ((A.mode == PROJ) ? 0 : 1);
    const int nblk = gridDim.x;
    if (tid < NR) {
        // RESID rows: [0,k) |r_q|^2 = nrm[q], [k,2k) |t_q|^2 = nrm[KO+q];  SUB rows: [0] = nrm[0]
        const int src = (A.mode == RESID && tid >= k) ? (KO + tid - k) : tid;
        double sum = 0.0;
        for (int w = 0; w < 4; ++w) sum += nsum[w][src];
        A.part[(size_t)tid * nblk + blockIdx.x] = sum;
    }
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) {
        const int j = wv + 4 * jj;
#pragma unroll
        for (int q = 0; q < KO; ++q) {
            double x = acc[jj][q];
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
            if (lane == 0 && j < mp && q < k) A.part[(size_t)(NR + j * k + q) * nblk + blockIdx.x] = x;
        }
    }
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

unsigned pass_blocks(int64_t N) {
    int64_t b = (N + kTB - 1) / kTB;
    if (b < 1) b = 1;
    if (b > kRedBlocks) b = kRedBlocks;
    return (unsigned)b;
}

template <int JW, int KO>
void launch_k(const PassArgs& A, unsigned nb, hipStream_t st) {
    hipLaunchKernelGGL((k_pass<JW, KO>), dim3(nb), dim3(kTB), 0, st, A);
}

// Register budget of the contraction: JW * KO <= 32 accumulators per lane.
hipError_t run_pass(const PassArgs& A, int rows, double* out, hipStream_t st) {
    const unsigned nb = pass_blocks(A.N);
    if (A.k < 1 || A.k > kMaxOut || A.mp > 48 || A.m > 64 || rows > 512) return hipErrorInvalidValue;
    const int jw = A.mp <= 16 ? 4 : (A.mp <= 32 ? 8 : 12);
    const int ko = A.k <= 1 ? 1 : (A.k <= 2 ? 2 : (A.k <= 4 ? 4 : 8));
    if (jw * ko > 32) return hipErrorInvalidValue;
    switch (jw * 100 + ko) {
        case 401: launch_k<4, 1>(A, nb, st); break;
        case 402: launch_k<4, 2>(A, nb, st); break;
        case 404: launch_k<4, 4>(A, nb, st); break;
        case 408: launch_k<4, 8>(A, nb, st); break;
        case 801: launch_k<8, 1>(A, nb, st); break;
        case 802: launch_k<8, 2>(A, nb, st); break;
        case 804: launch_k<8, 4>(A, nb, st); break;
        case 1201: launch_k<12, 1>(A, nb, st); break;
        case 1202: launch_k<12, 2>(A, nb, st); break;
        default: return hipErrorInvalidValue;
    }
    if (rows > 0) hipLaunchKernelGGL(k_reduce, dim3(rows), dim3(kTB), 0, st, A.part, (int)nb, out);
    return hipGetLastError();
}

}  // namespace
}  // namespace sbd

namespace sbd {

hipError_t pass_resid(const double* V, const double* W, int m, int k, const double* Y,
                      const double* theta, const double* diag, double delta, double* T, int64_t N,
                      bool proj, double* part, double* out, hipStream_t st) {
    PassArgs A{};
    A.N = N; A.mode = RESID; A.m = m; A.k = k; A.mp = proj ? m : 0;
    if (proj && !pass_fits(m, k)) return hipErrorInvalidValue;
    A.V = V; A.W = W; A.P = V; A.out = T; A.coef = Y; A.theta = theta; A.diag = diag;
    A.delta = delta; A.part = part;
    return run_pass(A, 2 * k + A.mp * k, out, st);
}

hipError_t pass_sub1(const double* V, int m, const double* h, double* t, int64_t N, double* part,
                     double* out, hipStream_t st) {
    PassArgs A{};
    A.N = N; A.mode = SUB1; A.m = m; A.k = 1; A.mp = m;
    A.V = V; A.P = V; A.X = t; A.out = t; A.coef = h; A.part = part;
    return run_pass(A, 1 + m, out, st);
}

hipError_t pass_sub2(const double* V, int m, const double* h, const double* t, double* dst,
                     const double* W, int mw, int64_t N, double* part, double* out, hipStream_t st) {
    PassArgs A{};
    A.N = N; A.mode = SUB2; A.m = m; A.k = 1; A.mp = mw;
    A.V = V; A.W = W; A.P = W; A.X = t; A.out = dst; A.coef = h; A.part = part;
    return run_pass(A, 1 + mw, out, st);
}

hipError_t pass_project(const double* P, int mp, const double* X, int k, int64_t N, double* part,
                        double* out, hipStream_t st) {
    // row groups small enough for the register budget; each group is one pass over X
    int step = mp;
    while (!pass_fits(step, k)) step = (step + 1) / 2;
    for (int j0 = 0; j0 < mp; j0 += step) {
        PassArgs A{};
        const int g = mp - j0 < step ? mp - j0 : step;
        A.N = N; A.mode = PROJ; A.m = 0; A.k = k; A.mp = g;
        A.P = P + (size_t)j0 * N; A.X = X; A.part = part;
        hipError_t e = run_pass(A, g * k, out + (size_t)j0 * k, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

bool pass_fits(int mp, int k) {
    const int jw = mp <= 16 ? 4 : (mp <= 32 ? 8 : 12);
    const int ko = k <= 1 ? 1 : (k <= 2 ? 2 : (k <= 4 ? 4 : 8));
    return mp <= 48 && k <= 8 && jw * ko <= 32;
}

}  // namespace sbd
