// Explicitly assembled Hamiltonian (the explicit realization of Sec. II-A):
// the connected pairs of every determinant row stored in CSR, built from the
// same excitation tables and coefficients as the matrix-free sigma (Eq. 4),
// and the sparse product y = (H - shift) x over it.
//
// Row I = (ia, ib) holds, in this order: the diagonal H_II; the alpha singles
// and doubles of ia (ket (ja, ib), in table order); the beta singles and
// doubles of ib (ket (ia, jb)); the products of the alpha singles of ia and
// the beta singles of ib (ket (ja, jb), alpha-single major).  A single's
// coefficient adds the spectator term of the other spin's string, and an
// alpha-beta pair's is sa sb (a_a i_a | b_b i_b).  The three groups reach
// disjoint kets, so every nonzero H_IJ appears once.
//
// Assembly: one thread per row counts its entries, a scan gives row_ptr, and
// one wavefront per row writes the row with lane-parallel, coalesced stores.
// The product: one wavefront per row, lanes striding over the row's entries,
// partial sums reduced across the wavefront in a fixed order (deterministic).
// It streams 12 or 8 bytes per stored entry from HBM (FP64 or FP32 value plus
// a 32-bit column) and gathers x through the caches.
#include "internal.h"

namespace sbd {
namespace {

constexpr int kCB = 256;  // threads per block

__global__ void k_csr_count(CsrTables S, int64_t* __restrict__ cnt) {
    const int64_t N = S.na * S.nb;
    for (int64_t I = (int64_t)blockIdx.x * kCB + threadIdx.x; I < N; I += (int64_t)gridDim.x * kCB) {
        const int64_t ia = I / S.nb, ib = I - ia * S.nb;
        const int64_t sa = S.a1p[ia + 1] - S.a1p[ia], da = S.a2p[ia + 1] - S.a2p[ia];
        const int64_t sb = S.b1p[ib + 1] - S.b1p[ib], db = S.b2p[ib + 1] - S.b2p[ib];
        cnt[I] = 1 + sa + da + sb + db + sa * sb;
    }
}

// one wavefront per row; F32: also write the FP32 values
template <bool F32>
__global__ void __launch_bounds__(kCB) k_csr_fill(CsrTables S, const int64_t* __restrict__ rp,
                                                  int32_t* __restrict__ col, double* __restrict__ v64,
                                                  float* __restrict__ v32) {
    const int lane = threadIdx.x & 63;
    const int64_t nb = S.nb, N = S.na * nb;
    const int64_t wpg = (int64_t)gridDim.x * (kCB / 64);
    const int n = S.norb;
    for (int64_t I = (int64_t)blockIdx.x * (kCB / 64) + (threadIdx.x >> 6); I < N; I += wpg) {
        const int64_t ia = I / nb, ib = I - ia * nb;
        int64_t o = rp[I];
        auto put = [&](int64_t at, int64_t c, double v) {
            col[at] = (int32_t)c;
            v64[at] = v;
            if (F32) v32[at] = (float)v;
        };
        if (lane == 0) put(o, I, S.diag[I]);
        o += 1;
        // alpha singles and doubles: ket (ja, ib)
        const int64_t a10 = S.a1p[ia], a11 = S.a1p[ia + 1];
        for (int64_t e = a10 + lane; e < a11; e += 64) {
            const int ps = S.a1ps[e];
            const double g = S.Gb[(int64_t)(ps >> 1) * nb + ib];
            put(o + (e - a10), (int64_t)S.a1J[e] * nb + ib, S.a1c[e] + ((ps & 1) ? -g : g));
        }
        o += a11 - a10;
        const int64_t a20 = S.a2p[ia], a21 = S.a2p[ia + 1];
        for (int64_t e = a20 + lane; e < a21; e += 64) put(o + (e - a20), (int64_t)S.a2J[e] * nb + ib, S.a2c[e]);
        o += a21 - a20;
        // beta singles and doubles: ket (ia, jb)
        const int64_t b10 = S.b1p[ib], b11 = S.b1p[ib + 1];
        for (int64_t e = b10 + lane; e < b11; e += 64) {
            const int ps = S.b1ps[e];
            const double g = S.Ga[(int64_t)(ps >> 1) * S.na + ia];
            put(o + (e - b10), ia * nb + S.b1J[e], S.b1c[e] + ((ps & 1) ? -g : g));
        }
        o += b11 - b10;
        const int64_t b20 = S.b2p[ib], b21 = S.b2p[ib + 1];
        for (int64_t e = b20 + lane; e < b21; e += 64) put(o + (e - b20), ia * nb + S.b2J[e], S.b2c[e]);
        o += b21 - b20;
        // alpha single x beta single: ket (ja, jb)
        const int64_t ns = b11 - b10, np = (a11 - a10) * ns;
        for (int64_t p = lane; p < np; p += 64) {
            const int64_t ea = a10 + p / ns, eb = b10 + p % ns;
            const uint64_t pa = S.a1pack[ea], pb = S.b1pack[eb];
            const int ai = (int)((pa >> 32) & 255), aa = (int)((pa >> 40) & 255);
            const int bi = (int)((pb >> 32) & 255), bb = (int)((pb >> 40) & 255);
            const double g = S.eri[(((int64_t)aa * n + ai) * n + bb) * n + bi];
            const bool neg = (((pa >> 48) ^ (pb >> 48)) & 1) != 0;
            put(o + p, (int64_t)(pa & 0xffffffffull) * nb + (int64_t)(pb & 0xffffffffull), neg ? -g : g);
        }
    }
}

// y[I][v] = sum_e val[e] x[col[e]][v] - shift x[I][v]; one wavefront per row
template <class T, int NV>
__global__ void __launch_bounds__(kCB) k_spmv(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                              const T* __restrict__ val, int64_t N, T shift,
                                              const T* __restrict__ x, T* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int64_t wpg = (int64_t)gridDim.x * (kCB / 64);
    for (int64_t I = (int64_t)blockIdx.x * (kCB / 64) + (threadIdx.x >> 6); I < N; I += wpg) {
        T acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = T(0);
        const int64_t e1 = rp[I + 1];
        for (int64_t e = rp[I] + lane; e < e1; e += 64) {
            const T a = val[e];
            const T* xr = x + (int64_t)col[e] * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += a * xr[v];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc[v] += __shfl_xor(acc[v], off, 64);
        }
        if (lane < NV) {
            T s = acc[0];
#pragma unroll
            for (int v = 1; v < NV; ++v) s = lane == v ? acc[v] : s;
            y[I * NV + lane] = s - shift * x[I * NV + lane];
        }
    }
}

unsigned row_blocks(int64_t rows) {
    const int64_t b = (rows + (kCB / 64) - 1) / (kCB / 64);
    return (unsigned)(b < 65536 * 4 ? b : 65536 * 4);
}

template <class T, int NV>
hipError_t spmv_nv(const int64_t* rp, const int32_t* col, const T* val, int64_t N, double shift, const T* x,
                   T* y, hipStream_t st) {
    hipLaunchKernelGGL((k_spmv<T, NV>), dim3(row_blocks(N)), dim3(kCB), 0, st, rp, col, val, N, (T)shift, x,
                       y);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_csr_count(const CsrTables& t, int64_t* cnt, hipStream_t st) {
    const CsrTables& S = t;
    const int64_t N = t.na * t.nb;
    if (N == 0) return hipSuccess;
    const int64_t b = (N + kCB - 1) / kCB;
    hipLaunchKernelGGL(k_csr_count, dim3((unsigned)(b < 65536 ? b : 65536)), dim3(kCB), 0, st, S, cnt);
    return hipGetLastError();
}

hipError_t launch_csr_fill(const CsrTables& t, const int64_t* rp, int32_t* col, double* v64, float* v32,
                           hipStream_t st) {
    const CsrTables& S = t;
    const int64_t N = t.na * t.nb;
    if (N == 0) return hipSuccess;
    if (v32)
        hipLaunchKernelGGL(k_csr_fill<true>, dim3(row_blocks(N)), dim3(kCB), 0, st, S, rp, col, v64, v32);
    else
        hipLaunchKernelGGL(k_csr_fill<false>, dim3(row_blocks(N)), dim3(kCB), 0, st, S, rp, col, v64, v32);
    return hipGetLastError();
}

template <class T>
hipError_t launch_spmv(const int64_t* rp, const int32_t* col, const T* val, int64_t N, int nv, double shift,
                       const T* x, T* y, hipStream_t st) {
    if (N == 0) return hipSuccess;
    switch (nv) {
        case 1: return spmv_nv<T, 1>(rp, col, val, N, shift, x, y, st);
        case 2: return spmv_nv<T, 2>(rp, col, val, N, shift, x, y, st);
        case 4: return spmv_nv<T, 4>(rp, col, val, N, shift, x, y, st);
        case 8: return spmv_nv<T, 8>(rp, col, val, N, shift, x, y, st);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_spmv<double>(const int64_t*, const int32_t*, const double*, int64_t, int, double,
                                        const double*, double*, hipStream_t);
template hipError_t launch_spmv<float>(const int64_t*, const int32_t*, const float*, int64_t, int, double,
                                       const float*, float*, hipStream_t);

}  // namespace sbd
