// Dense FP64 vector kernels of the Davidson driver (Sec. II-C): linear
// combinations V Y (collapse and restart), scaling, precision conversions for
// the FP32 sigma, start-vector selection, the transfer of vectors between two
// bases (warm starts of successive solves) and small reductions.  Reductions are
// two-stage with a fixed block count and a fixed combination order, so results
// do not depend on scheduling.  These kernels are bound by HBM bandwidth.
#include <algorithm>

#include "internal.h"

namespace sbd {
namespace {

constexpr int kVB = 256;      // threads per block

inline unsigned red_blocks(int64_t N) {
    int64_t b = (N + kVB * 4 - 1) / (kVB * 4);
    if (b < 1) b = 1;
    if (b > kRedBlocks) b = kRedBlocks;
    return (unsigned)b;
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

__global__ void k_scale(double* x, int64_t N, double s) {
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB)
        x[i] *= s;
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

// out[i*nv + v] = src[v*N + i] for v < cnt (as T), 0 for cnt <= v < nv: the
// interleaved layout of a block sigma, k values of one determinant contiguous.
// With d_row, src is offset by (*d_row) rows read on the device (graph replays).
template <class T>
__global__ void __launch_bounds__(kVB) k_interleave(const double* __restrict__ src,
                                                    const int* __restrict__ d_row, int cnt, int nv,
                                                    int64_t N, T* __restrict__ out) {
    if (d_row) src += (size_t)(*d_row) * N;
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB)
        for (int v = 0; v < nv; ++v) out[i * nv + v] = v < cnt ? (T)src[(size_t)v * N + i] : (T)0;
}

// dst[v*N + i] = y[i*nv + v] (+ shift * x[v*N + i] when x is given), v < cnt;
// with d_row, x and dst are offset by (*d_row) rows read on the device
template <class T>
__global__ void __launch_bounds__(kVB) k_deinterleave(const T* __restrict__ y, int cnt, int nv,
                                                      int64_t N, const double* __restrict__ x,
                                                      double shift, double* __restrict__ dst,
                                                      const int* __restrict__ d_row) {
    if (d_row) {
        const size_t off = (size_t)(*d_row) * N;
        if (x) x += off;
        dst += off;
    }
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB)
        for (int v = 0; v < cnt; ++v) {
            const double a = (double)y[i * nv + v];
            dst[(size_t)v * N + i] = x ? a + shift * x[(size_t)v * N + i] : a;
        }
}

// block maxima of v, then the maximum of the block values
__global__ void __launch_bounds__(kVB) k_max(const double* __restrict__ v, int64_t N, double* pv) {
    double b = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kVB)
        b = fmax(b, v[i]);
    __shared__ double sv[kVB];
    sv[threadIdx.x] = b;
    __syncthreads();
    for (int off = kVB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sv[threadIdx.x] = fmax(sv[threadIdx.x], sv[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) pv[blockIdx.x] = sv[0];
}

__global__ void k_max_final(const double* pv, int nblk, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double b = -INFINITY;
    for (int i = 0; i < nblk; ++i) b = fmax(b, pv[i]);
    *out = b;
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

// map[i] = index of to[i] in the sorted array from[0..nfrom), or -1
__global__ void k_string_map(const uint64_t* __restrict__ to, int64_t nto, const uint64_t* __restrict__ from,
                             int64_t nfrom, int64_t* __restrict__ map) {
    for (int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x; i < nto; i += (int64_t)gridDim.x * kVB) {
        const uint64_t s = to[i];
        int64_t lo = 0, hi = nfrom;  // first position with from[pos] >= s
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (from[mid] < s) lo = mid + 1; else hi = mid;
        }
        map[i] = (lo < nfrom && from[lo] == s) ? lo : -1;
    }
}

// y[v][ia][ib] = x[v][amap[ia]][bmap[ib]] when both strings exist in the old
// basis, else 0.  Grid: x over beta columns, y over (vector, alpha row).
__global__ void k_map_vectors(const int64_t* __restrict__ amap, const int64_t* __restrict__ bmap, int64_t na,
                              int64_t nb, int64_t nb_from, int64_t n_from, int nvec,
                              const double* __restrict__ x, double* __restrict__ y) {
    const int64_t nrows = (int64_t)nvec * na;
    for (int64_t row = blockIdx.y; row < nrows; row += gridDim.y) {
        const int64_t v = row / na, ia = row - v * na;
        const int64_t ja = amap[ia];
        const double* xr = x + v * n_from + (ja >= 0 ? ja : 0) * nb_from;
        double* yr = y + (v * na + ia) * nb;
        for (int64_t ib = (int64_t)blockIdx.x * kVB + threadIdx.x; ib < nb; ib += (int64_t)gridDim.x * kVB) {
            const int64_t jb = bmap[ib];
            yr[ib] = (ja >= 0 && jb >= 0) ? xr[jb] : 0.0;
        }
    }
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

hipError_t launch_combination(const double* A, int m, const double* d_Y, int ldy, int k,
                              double* out, int64_t N, hipStream_t st) {
    if (m > 64 || k > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_comb, dim3(red_blocks(N)), dim3(kVB), 0, st, A, m, d_Y, ldy, k, out, N);
    return hipGetLastError();
}

hipError_t launch_scale(double* x, int64_t N, double s, hipStream_t st) {
    hipLaunchKernelGGL(k_scale, dim3(red_blocks(N)), dim3(kVB), 0, st, x, N, s);
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

template <class T>
hipError_t launch_interleave(const double* src, const int* d_row, int cnt, int nv, int64_t N, T* out,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_interleave<T>, dim3(red_blocks(N)), dim3(kVB), 0, st, src, d_row, cnt, nv,
                       N, out);
    return hipGetLastError();
}
template hipError_t launch_interleave<double>(const double*, const int*, int, int, int64_t, double*,
                                              hipStream_t);
template hipError_t launch_interleave<float>(const double*, const int*, int, int, int64_t, float*,
                                             hipStream_t);

template <class T>
hipError_t launch_deinterleave(const T* y, int cnt, int nv, int64_t N, const double* x, double shift,
                               double* dst, const int* d_row, hipStream_t st) {
    hipLaunchKernelGGL(k_deinterleave<T>, dim3(red_blocks(N)), dim3(kVB), 0, st, y, cnt, nv, N, x,
                       shift, dst, d_row);
    return hipGetLastError();
}
template hipError_t launch_deinterleave<double>(const double*, int, int, int64_t, const double*, double,
                                                double*, const int*, hipStream_t);
template hipError_t launch_deinterleave<float>(const float*, int, int, int64_t, const double*, double,
                                               double*, const int*, hipStream_t);

__global__ void k_set_int(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_set_int(int* d_p, int v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, d_p, v);
    return hipGetLastError();
}

hipError_t launch_max(const double* v, int64_t N, double* d_val, double* d_part, hipStream_t st) {
    unsigned nb = red_blocks(N);
    hipLaunchKernelGGL(k_max, dim3(nb), dim3(kVB), 0, st, v, N, d_part);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(64), 0, st, d_part, (int)nb, d_val);
    return hipGetLastError();
}

hipError_t launch_set_unit(double* x, int64_t N, int64_t idx, hipStream_t st) {
    hipLaunchKernelGGL(k_set_unit, dim3(red_blocks(N)), dim3(kVB), 0, st, x, N, idx);
    return hipGetLastError();
}

hipError_t launch_string_map(const uint64_t* to, int64_t nto, const uint64_t* from, int64_t nfrom,
                             int64_t* map, hipStream_t st) {
    if (nto == 0) return hipSuccess;
    hipLaunchKernelGGL(k_string_map, dim3(red_blocks(nto)), dim3(kVB), 0, st, to, nto, from, nfrom, map);
    return hipGetLastError();
}

hipError_t launch_map_vectors(const int64_t* amap, const int64_t* bmap, int64_t na, int64_t nb, int64_t nb_from,
                              int64_t n_from, int nvec, const double* x, double* y, hipStream_t st) {
    if (na == 0 || nb == 0 || nvec == 0) return hipSuccess;
    const int64_t gx = std::min<int64_t>((nb + kVB - 1) / kVB, 64);
    const int64_t gy = std::min<int64_t>((int64_t)nvec * na, 65535);
    hipLaunchKernelGGL(k_map_vectors, dim3((unsigned)gx, (unsigned)gy), dim3(kVB), 0, st, amap, bmap, na, nb,
                       nb_from, n_from, nvec, x, y);
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

// ------------------------------------------------------------------ occupations
// Spin-orbital occupations of a vector over the alpha x beta product basis
// (the input of the sample recovery of an SQD iteration): the squared entries
// summed per row (alpha string) and per column (beta string), then for every
// orbital the share of that weight on the strings that hold it.  Fixed
// reduction orders, so the result does not depend on scheduling.
namespace {

constexpr int kOccRows = 128;  // rows per partial column sum (at least)

__device__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = kVB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// wa[ia] = sum_ib c[ia, ib]^2: one workgroup per row
__global__ void __launch_bounds__(kVB) k_row_sq(const double* __restrict__ c, int64_t nb, double* __restrict__ wa) {
    __shared__ double sh[kVB];
    const double* r = c + (int64_t)blockIdx.x * nb;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < nb; j += kVB) s += r[j] * r[j];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) wa[blockIdx.x] = s;
}

// part[q * nb + ib] = sum of c[ia, ib]^2 over the rows of chunk q
__global__ void __launch_bounds__(kVB) k_col_sq_part(const double* __restrict__ c, int64_t na, int64_t nb,
                                                     int64_t rows, double* __restrict__ part) {
    const int64_t ib = (int64_t)blockIdx.x * kVB + threadIdx.x;
    if (ib >= nb) return;
    const int64_t r0 = (int64_t)blockIdx.y * rows, r1 = r0 + rows < na ? r0 + rows : na;
    double s = 0.0;
    for (int64_t ia = r0; ia < r1; ++ia) {
        const double v = c[ia * nb + ib];
        s += v * v;
    }
    part[(int64_t)blockIdx.y * nb + ib] = s;
}

__global__ void __launch_bounds__(kVB) k_col_sq_sum(const double* __restrict__ part, int64_t nq, int64_t nb,
                                                    double* __restrict__ wb) {
    const int64_t ib = (int64_t)blockIdx.x * kVB + threadIdx.x;
    if (ib >= nb) return;
    double s = 0.0;
    for (int64_t q = 0; q < nq; ++q) s += part[q * nb + ib];
    wb[ib] = s;
}

// occ[spin * norb + p] = (sum of w over the strings holding p) / (sum of w):
// one workgroup per (orbital, spin)
__global__ void __launch_bounds__(kVB) k_orb_occ(const uint64_t* __restrict__ sa, const double* __restrict__ wa,
                                                 int64_t na, const uint64_t* __restrict__ sb,
                                                 const double* __restrict__ wb, int64_t nb, int norb,
                                                 double* __restrict__ occ) {
    __shared__ double sh[kVB];
    const int p = blockIdx.x, spin = blockIdx.y;
    const uint64_t* s = spin ? sb : sa;
    const double* w = spin ? wb : wa;
    const int64_t n = spin ? nb : na;
    double tot = 0.0, hold = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kVB) {
        tot += w[i];
        if ((s[i] >> p) & 1ull) hold += w[i];
    }
    tot = block_sum(tot, sh);
    hold = block_sum(hold, sh);
    if (threadIdx.x == 0) occ[spin * norb + p] = tot > 0.0 ? hold / tot : 0.0;
}

}  // namespace

int64_t occupation_scratch_words(int64_t na, int64_t nb) {
    int64_t rows = kOccRows;
    if ((na + rows - 1) / rows > 65535) rows = (na + 65534) / 65535;
    const int64_t nq = (na + rows - 1) / rows;
    return na + nb + nq * nb;
}

hipError_t launch_occupations(const double* c, const uint64_t* sa, int64_t na, const uint64_t* sb, int64_t nb,
                              int norb, double* scratch, double* occ, hipStream_t st) {
    int64_t rows = kOccRows;
    if ((na + rows - 1) / rows > 65535) rows = (na + 65534) / 65535;
    const int64_t nq = (na + rows - 1) / rows;
    double *wa = scratch, *wb = scratch + na, *part = scratch + na + nb;
    const unsigned cb = (unsigned)((nb + kVB - 1) / kVB);
    hipLaunchKernelGGL(k_row_sq, dim3((unsigned)na), dim3(kVB), 0, st, c, nb, wa);
    hipLaunchKernelGGL(k_col_sq_part, dim3(cb, (unsigned)nq), dim3(kVB), 0, st, c, na, nb, rows, part);
    hipLaunchKernelGGL(k_col_sq_sum, dim3(cb), dim3(kVB), 0, st, part, nq, nb, wb);
    hipLaunchKernelGGL(k_orb_occ, dim3((unsigned)norb, 2), dim3(kVB), 0, st, sa, wa, na, sb, wb, nb, norb, occ);
    return hipGetLastError();
}

}  // namespace sbd
