// Dense FP64 vector kernels of the Davidson update (Sec. II-C): projections
// V^T x, linear combinations V Y, the fused residual + damped diagonal
// preconditioner (Eqs. 6-7), and reductions.  All reductions are two-stage
// with a fixed block count and a fixed combination order, so results do not
// depend on scheduling.  These kernels are bound by HBM bandwidth: each pass
// streams the subspace vectors once.
#include "internal.h"

namespace sbd {
namespace {

constexpr int kVB = 256;      // threads per block
constexpr int kDotRows = 8;   // rows of V handled per projection pass

inline unsigned red_blocks(int64_t N) {
    int64_t b = (N + kVB * 4 - 1) / (kVB * 4);
    if (b < 1) b = 1;
    if (b > kRedBlocks) b = kRedBlocks;
    return (unsigned)b;
}

template <int R>
__device__ void block_reduce_store(double (&v)[R], double* part, int stride_blocks) {
    __shared__ double sh[R][kVB / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double x = v[r];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) sh[r][w] = x;
    }
    __syncthreads();
    if (threadIdx.x < R) {
        double s = 0.0;
        for (int k = 0; k < kVB / 64; ++k) s += sh[threadIdx.x][k];
        part[(size_t)threadIdx.x * stride_blocks + blockIdx.x] = s;
    }
}

// part[r][block] = sum over this block's share of A[j0+r][i] * x[i]
__global__ void __launch_bounds__(kVB) k_multidot_part(const double* __restrict__ A, int j0,
                                                       int rows, const double* __restrict__ x,
                                                       int64_t N, double* part) {
    double acc[kDotRows];
#pragma unroll
    for (int r = 0; r < kDotRows; ++r) acc[r] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB) {
        double xi = x[i];
#pragma unroll
        for (int r = 0; r < kDotRows; ++r)
            if (r < rows) acc[r] += A[(size_t)(j0 + r) * N + i] * xi;
    }
    block_reduce_store<kDotRows>(acc, part, gridDim.x);
}

// out[j0+r] = sum_b part[r][b] (fixed order), r < rows
__global__ void k_reduce_parts(const double* part, int nblk, int rows, double* out, int j0) {
    int r = blockIdx.x;
    if (r >= rows) return;
    __shared__ double sh[kVB];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kVB) s += part[(size_t)r * nblk + b];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = kVB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j0 + r] = sh[0];
}

__global__ void __launch_bounds__(kVB) k_sub_comb(const double* __restrict__ A, int m,
                                                  const double* __restrict__ h, double* x,
                                                  int64_t N) {
    __shared__ double hs[64];
    if (threadIdx.x < m) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += A[(size_t)j * N + i] * hs[j];
        x[i] -= s;
    }
}

__global__ void __launch_bounds__(kVB) k_comb(const double* __restrict__ A, int m,
                                              const double* __restrict__ Y, int ldy, int k,
                                              double* out, int64_t N) {
    __shared__ double ys[64 * 8];
    for (int t = threadIdx.x; t < m * k; t += kVB) {
        int j = t / k, r = t % k;
        ys[j * 8 + r] = Y[j * ldy + r];
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB) {
        double s[8];
        for (int r = 0; r < 8; ++r) s[r] = 0.0;
        for (int j = 0; j < m; ++j) {
            double a = A[(size_t)j * N + i];
            for (int r = 0; r < k; ++r) s[r] += a * ys[j * 8 + r];
        }
        for (int r = 0; r < k; ++r) out[(size_t)r * N + i] = s[r];
    }
}

__device__ __forceinline__ double damped_inv(double d, double delta) {
    double a = fabs(d);
    double den = a > delta ? a : delta;
    return (d >= 0.0 ? 1.0 : -1.0) / den;
}

// t = (W y - theta V y) / damp(diag - theta); part[0][b] = sum r^2, part[1][b] = sum t^2
__global__ void __launch_bounds__(kVB) k_resid_precond(const double* __restrict__ V,
                                                       const double* __restrict__ W, int m,
                                                       const double* __restrict__ y, double theta,
                                                       const double* __restrict__ diag,
                                                       double delta, double* t, int64_t N,
                                                       double* part) {
    __shared__ double ys[64];
    if (threadIdx.x < m) ys[threadIdx.x] = y[threadIdx.x];
    __syncthreads();
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB) {
        double wy = 0.0, vy = 0.0;
        for (int j = 0; j < m; ++j) {
            wy += W[(size_t)j * N + i] * ys[j];
            vy += V[(size_t)j * N + i] * ys[j];
        }
        double r = wy - theta * vy;
        double ti = r * damped_inv(diag[i] - theta, delta);
        t[i] = ti;
        acc[0] += r * r;
        acc[1] += ti * ti;
    }
    block_reduce_store<2>(acc, part, gridDim.x);
}

__global__ void k_scale(double* x, int64_t N, double s) {
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB)
        x[i] *= s;
}

__global__ void k_copy(const double* x, double* y, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB)
        y[i] = x[i];
}

__device__ __forceinline__ bool lex_less(double v1, int64_t i1, double v2, int64_t i2) {
    return v1 < v2 || (v1 == v2 && i1 < i2);
}

// smallest (v[i], i) lexicographically greater than (vprev, iprev)
__global__ void __launch_bounds__(kVB) k_argmin_after(const double* __restrict__ v, int64_t N,
                                                      double vprev, int64_t iprev, double* pv,
                                                      int64_t* pi) {
    double bv = INFINITY;
    int64_t bi = -1;
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB) {
        double x = v[i];
        if (lex_less(vprev, iprev, x, i) && (bi < 0 || lex_less(x, i, bv, bi))) {
            bv = x;
            bi = i;
        }
    }
    __shared__ double sv[kVB];
    __shared__ int64_t si[kVB];
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = kVB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            double v2 = sv[threadIdx.x + off];
            int64_t i2 = si[threadIdx.x + off];
            if (i2 >= 0 && (si[threadIdx.x] < 0 || lex_less(v2, i2, sv[threadIdx.x], si[threadIdx.x]))) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pv[blockIdx.x] = sv[0];
        pi[blockIdx.x] = si[0];
    }
}

__global__ void k_argmin_final(const double* pv, const int64_t* pi, int nblk, double* ov,
                               int64_t* oi) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double bv = INFINITY;
    int64_t bi = -1;
    for (int b = 0; b < nblk; ++b)
        if (pi[b] >= 0 && (bi < 0 || lex_less(pv[b], pi[b], bv, bi))) {
            bv = pv[b];
            bi = pi[b];
        }
    *ov = bv;
    *oi = bi;
}

__global__ void k_set_unit(double* x, int64_t N, int64_t idx) {
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB)
        x[i] = (i == idx) ? 1.0 : 0.0;
}

__global__ void k_f64_to_f32(const double* x, float* y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVB)
        y[i] = (float)x[i];
}

// y = (double)y32 + shift * x
__global__ void k_f32_to_f64_axpy(const float* y32, const double* x, double shift, double* y,
                                  int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVB)
        y[i] = (double)y32[i] + shift * x[i];
}

// Deterministic bounded test pattern: x_i = sin(0.37 i) (FP64 or FP32).
__global__ void k_fill_pattern(void* p, int64_t n, int prec) {
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVB) {
        const double v = sin(0.37 * (double)(i % 1000003));
        if (prec == 0)
            static_cast<double*>(p)[i] = v;
        else
            static_cast<float*>(p)[i] = (float)v;
    }
}

}  // namespace

hipError_t launch_fill_pattern(void* p, int64_t n, int prec, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_pattern, dim3(red_blocks(n)), dim3(kVB), 0, st, p, n, prec);
    return hipGetLastError();
}

hipError_t launch_multidot(const double* A, int m, const double* x, int64_t N, double* d_out,
                           double* d_part, hipStream_t st) {
    unsigned nb = red_blocks(N);
    for (int j0 = 0; j0 < m; j0 += kDotRows) {
        int rows = (m - j0) < kDotRows ? (m - j0) : kDotRows;
        hipLaunchKernelGGL(k_multidot_part, dim3(nb), dim3(kVB), 0, st, A, j0, rows, x, N, d_part);
        hipLaunchKernelGGL(k_reduce_parts, dim3(rows), dim3(kVB), 0, st, d_part, (int)nb, rows,
                           d_out, j0);
    }
    return hipGetLastError();
}

hipError_t launch_sub_combination(const double* A, int m, const double* d_h, double* x, int64_t N,
                                  hipStream_t st) {
    if (m <= 0) return hipSuccess;
    if (m > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sub_comb, dim3(red_blocks(N)), dim3(kVB), 0, st, A, m, d_h, x, N);
    return hipGetLastError();
}

hipError_t launch_combination(const double* A, int m, const double* d_Y, int ldy, int k,
                              double* out, int64_t N, hipStream_t st) {
    if (m > 64 || k > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_comb, dim3(red_blocks(N)), dim3(kVB), 0, st, A, m, d_Y, ldy, k, out, N);
    return hipGetLastError();
}

hipError_t launch_residual_precond(const double* V, const double* W, int m, const double* d_y,
                                   double theta, const double* diag, double delta, double* t,
                                   int64_t N, double* d_out, double* d_part, hipStream_t st) {
    if (m > 64) return hipErrorInvalidValue;
    unsigned nb = red_blocks(N);
    hipLaunchKernelGGL(k_resid_precond, dim3(nb), dim3(kVB), 0, st, V, W, m, d_y, theta, diag,
                       delta, t, N, d_part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(2), dim3(kVB), 0, st, d_part, (int)nb, 2, d_out, 0);
    return hipGetLastError();
}

hipError_t launch_scale(double* x, int64_t N, double s, hipStream_t st) {
    hipLaunchKernelGGL(k_scale, dim3(red_blocks(N)), dim3(kVB), 0, st, x, N, s);
    return hipGetLastError();
}

hipError_t launch_copy(const double* x, double* y, int64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_copy, dim3(red_blocks(N)), dim3(kVB), 0, st, x, y, N);
    return hipGetLastError();
}

hipError_t launch_argmin_after(const double* v, int64_t N, double vprev, int64_t iprev,
                               double* d_val, int64_t* d_idx, double* d_part_v,
                               int64_t* d_part_i, hipStream_t st) {
    unsigned nb = red_blocks(N);
    hipLaunchKernelGGL(k_argmin_after, dim3(nb), dim3(kVB), 0, st, v, N, vprev, iprev, d_part_v,
                       d_part_i);
    hipLaunchKernelGGL(k_argmin_final, dim3(1), dim3(64), 0, st, d_part_v, d_part_i, (int)nb,
                       d_val, d_idx);
    return hipGetLastError();
}

hipError_t launch_set_unit(double* x, int64_t N, int64_t idx, hipStream_t st) {
    hipLaunchKernelGGL(k_set_unit, dim3(red_blocks(N)), dim3(kVB), 0, st, x, N, idx);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double* x, float* y, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(red_blocks(n)), dim3(kVB), 0, st, x, y, n);
    return hipGetLastError();
}

hipError_t launch_f32_to_f64_axpy(const float* y32, const double* x, double shift, double* y,
                                  int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_f32_to_f64_axpy, dim3(red_blocks(n)), dim3(kVB), 0, st, y32, x, shift, y, n);
    return hipGetLastError();
}

}  // namespace sbd
