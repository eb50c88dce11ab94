// Matrix-free sigma = (H - shift) c over the alpha x beta determinant basis
// (Eq. 4; the three task types of Sec. III-B).
//
// Owner computes: the thread that owns output element (ia, ib) accumulates
// every contribution to it in registers, in a fixed order, and stores it
// once.  No atomics, so results are bitwise reproducible (the paper resolves
// write races with atomicAdd instead).
//
//   diag     : (H_ii - shift) c[ia, ib]
//   task 2   : alpha singles/doubles  sum_{Ja} coef * c[Ja, ib]   (row stream,
//              consecutive ib are consecutive addresses -> coalesced)
//   task 1   : beta singles/doubles   sum_{Jb} coef * c[ia, Jb]   (gather in row ia)
//   task 0   : alpha single x beta single  sa sb (ai|bj) c[Ja, Jb]
//
// Single coefficients add the spectator term of the other spin read from
// G[pair][string]; the rest of each coefficient is per table entry.
#include "internal.h"

namespace sbd {
namespace {

constexpr int kSigBlock = 256;

template <class T, int NV>
__global__ void __launch_bounds__(kSigBlock) k_sigma_rows(SigmaArgs<T> A, const T* __restrict__ c,
                                                          T* __restrict__ y) {
    const int64_t nb = A.nb, na = A.na;
    const int n = A.norb;
    int64_t ib = (int64_t)blockIdx.x * kSigBlock + threadIdx.x;
    if (ib >= nb) return;
    for (int64_t ia = blockIdx.y; ia < na; ia += gridDim.y) {
        const int64_t det = ia * nb + ib;
        T acc[NV];
        const T dg = (T)(A.diag[det] - A.shift);
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = dg * c[det * NV + v];

        // task 2: alpha singles (coefficient depends on beta string ib)
        for (int64_t e = A.a1p[ia]; e < A.a1p[ia + 1]; ++e) {
            const int64_t ja = A.a1J[e];
            const int ps = A.a1ps[e];
            const T g = A.Gb[(int64_t)(ps >> 1) * nb + ib];
            const T coef = A.a1c[e] + ((ps & 1) ? -g : g);
            const T* src = c + (ja * nb + ib) * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += coef * src[v];
        }
        // task 2: alpha doubles
        for (int64_t e = A.a2p[ia]; e < A.a2p[ia + 1]; ++e) {
            const int64_t ja = A.a2J[e];
            const T coef = A.a2c[e];
            const T* src = c + (ja * nb + ib) * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += coef * src[v];
        }
        // task 1: beta singles (coefficient depends on alpha string ia)
        for (int64_t e = A.b1p[ib]; e < A.b1p[ib + 1]; ++e) {
            const int64_t jb = A.b1J[e];
            const int ps = A.b1ps[e];
            const T g = A.Ga[(int64_t)(ps >> 1) * na + ia];
            const T coef = A.b1c[e] + ((ps & 1) ? -g : g);
            const T* src = c + (ia * nb + jb) * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += coef * src[v];
        }
        // task 1: beta doubles
        for (int64_t e = A.b2p[ib]; e < A.b2p[ib + 1]; ++e) {
            const int64_t jb = A.b2J[e];
            const T coef = A.b2c[e];
            const T* src = c + (ia * nb + jb) * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += coef * src[v];
        }
        // task 0: alpha single x beta single
        for (int64_t ea = A.a1p[ia]; ea < A.a1p[ia + 1]; ++ea) {
            const int64_t ja = A.a1J[ea];
            const uint32_t oa = A.a1o[ea];
            const int ai = oa & 255, aa = (oa >> 8) & 255;
            const T* slice = A.eri + ((size_t)aa * n + ai) * n * n;  // (a_a i_a | . .)
            const int sa = A.a1s[ea];
            for (int64_t eb = A.b1p[ib]; eb < A.b1p[ib + 1]; ++eb) {
                const int64_t jb = A.b1J[eb];
                const uint32_t ob = A.b1o[eb];
                const int bi = ob & 255, ba = (ob >> 8) & 255;
                const T g = slice[ba * n + bi];
                const T coef = (sa * A.b1s[eb] < 0) ? -g : g;
                const T* src = c + (ja * nb + jb) * NV;
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] += coef * src[v];
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) y[det * NV + v] = acc[v];
    }
}

template <class T, int NV>
hipError_t launch_rows(const SigmaArgs<T>& A, const T* c, T* y, hipStream_t st) {
    unsigned gx = (unsigned)((A.nb + kSigBlock - 1) / kSigBlock);
    unsigned gy = (unsigned)(A.na < 65535 ? A.na : 65535);
    hipLaunchKernelGGL((k_sigma_rows<T, NV>), dim3(gx, gy), dim3(kSigBlock), 0, st, A, c, y);
    return hipGetLastError();
}

}  // namespace

template <class T>
hipError_t launch_sigma(const SigmaArgs<T>& A, int nvec, const T* c, T* y, int layout,
                        hipStream_t st) {
    if (A.na == 0 || A.nb == 0) return hipSuccess;
    if (layout == 0) {
        const int64_t N = A.na * A.nb;
        for (int v = 0; v < nvec; ++v) {
            hipError_t e = launch_rows<T, 1>(A, c + v * N, y + v * N, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    switch (nvec) {
        case 1: return launch_rows<T, 1>(A, c, y, st);
        case 2: return launch_rows<T, 2>(A, c, y, st);
        case 3: return launch_rows<T, 3>(A, c, y, st);
        case 4: return launch_rows<T, 4>(A, c, y, st);
        case 5: return launch_rows<T, 5>(A, c, y, st);
        case 6: return launch_rows<T, 6>(A, c, y, st);
        case 7: return launch_rows<T, 7>(A, c, y, st);
        case 8: return launch_rows<T, 8>(A, c, y, st);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_sigma<double>(const SigmaArgs<double>&, int, const double*, double*,
                                         int, hipStream_t);
template hipError_t launch_sigma<float>(const SigmaArgs<float>&, int, const float*, float*, int,
                                        hipStream_t);

}  // namespace sbd
