// Hamiltonian set-up kernels: the cached diagonal (Sec. II-E) and the
// matrix-element coefficients of every excitation-table entry (Eq. 4 with the
// Slater-Condon forms of the half-bitstring split).
//
// For a determinant |Ia, Ib> the diagonal is
//   E_core + d_a(Ia) + d_b(Ib) + sum_{p in Ia} sum_{q in Ib} (pp|qq),
//   d_s(I) = sum_{p in I} h_pp + sum_{p<q in I} [(pp|qq) - (pq|qp)].
// A same-spin single i -> a between bra I and ket J (sign s) has
//   s * [h_ai + sum_{k in J} ((ai|kk) - (ak|ki)) + sum_{k in other spin} (ai|kk)];
// the last term depends on the other spin's string and is read at sigma time
// from the spectator table G[pair(a,i)][string] = sum_{k in string} (ai|kk).
// A same-spin double (i,j) -> (a,b) has s * [(ai|bj) - (aj|bi)].
#include "internal.h"

namespace sbd {
namespace {

__device__ __forceinline__ double eri_at(const double* eri, int n, int p, int q, int r, int s) {
    return eri[(((size_t)p * n + q) * n + r) * n + s];
}

__device__ __forceinline__ int tri(int a, int i) {
    int hi = a > i ? a : i, lo = a > i ? i : a;
    return hi * (hi + 1) / 2 + lo;
}

__global__ void k_string_diag(const uint64_t* __restrict__ s, int64_t n, int norb,
                              const double* __restrict__ h, const double* __restrict__ eri,
                              double* out) {
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= n) return;
    uint64_t x = s[I];
    double e = 0.0;
    for (uint64_t m = x; m; m &= m - 1) {
        int p = __builtin_ctzll(m);
        e += h[p * norb + p];
        for (uint64_t r = m & (m - 1); r; r &= r - 1) {
            int q = __builtin_ctzll(r);
            e += eri_at(eri, norb, p, p, q, q) - eri_at(eri, norb, p, q, q, p);
        }
    }
    out[I] = e;
}

// G[pair][I] for every unordered orbital pair (a >= i) and string I.
__global__ void k_spectator(const uint64_t* __restrict__ s, int64_t n, int norb,
                            const double* __restrict__ eri, double* G64, float* G32) {
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int pr = blockIdx.y;
    if (I >= n) return;
    // decode triangular pair index
    int hi = 0;
    while ((hi + 1) * (hi + 2) / 2 <= pr) ++hi;
    int lo = pr - hi * (hi + 1) / 2;
    uint64_t x = s[I];
    double g = 0.0;
    for (uint64_t m = x; m; m &= m - 1) {
        int k = __builtin_ctzll(m);
        g += eri_at(eri, norb, hi, lo, k, k);
    }
    G64[(size_t)pr * n + I] = g;
    G32[(size_t)pr * n + I] = (float)g;
}

__global__ void k_single_coef(const uint64_t* __restrict__ s, int64_t nnz,
                              const int32_t* __restrict__ J, const uint32_t* __restrict__ orb,
                              const int8_t* __restrict__ sg, int norb, const double* __restrict__ h,
                              const double* __restrict__ eri, double* c64, float* c32,
                              int32_t* ps) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    uint64_t ket = s[J[e]];
    int i = orb[e] & 255, a = (orb[e] >> 8) & 255;
    double v = h[a * norb + i];
    for (uint64_t m = ket; m; m &= m - 1) {
        int k = __builtin_ctzll(m);
        v += eri_at(eri, norb, a, i, k, k) - eri_at(eri, norb, a, k, k, i);
    }
    double c = sg[e] * v;
    c64[e] = c;
    c32[e] = (float)c;
    ps[e] = (tri(a, i) << 1) | (sg[e] < 0 ? 1 : 0);
}

__global__ void k_double_coef(int64_t nnz, const uint32_t* __restrict__ orb,
                              const int8_t* __restrict__ sg, int norb,
                              const double* __restrict__ eri, double* c64, float* c32) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    uint32_t o = orb[e];
    int i = o & 255, j = (o >> 8) & 255, a = (o >> 16) & 255, b = (o >> 24) & 255;
    double c = sg[e] * (eri_at(eri, norb, a, i, b, j) - eri_at(eri, norb, a, j, b, i));
    c64[e] = c;
    c32[e] = (float)c;
}

// diag[ia*nb + ib]: one row per blockIdx.y, columns across threads.
__global__ void k_full_diag(const uint64_t* __restrict__ sa, int64_t na, const double* __restrict__ da,
                            const double* __restrict__ db, const double* __restrict__ Gb,
                            int64_t nb, double e_core, double* diag) {
    int64_t ib = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ib >= nb) return;
    for (int64_t ia = blockIdx.y; ia < na; ia += gridDim.y) {
        double e = e_core + da[ia] + db[ib];
        for (uint64_t m = sa[ia]; m; m &= m - 1) {
            int p = __builtin_ctzll(m);
            e += Gb[(size_t)(p * (p + 1) / 2 + p) * nb + ib];
        }
        diag[ia * nb + ib] = e;
    }
}

__global__ void k_d2f(const double* in, float* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_string_diag(const uint64_t* d_s, int64_t n, int norb, const double* h,
                              const double* eri, double* out, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_string_diag, dim3(nblk(n, 256)), dim3(256), 0, st, d_s, n, norb, h,
                           eri, out);
    return hipGetLastError();
}

hipError_t launch_spectator(const uint64_t* d_s, int64_t n, int norb, const double* eri,
                            double* G64, float* G32, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_spectator, dim3(nblk(n, 256), npairs(norb)), dim3(256), 0, st, d_s, n,
                           norb, eri, G64, G32);
    return hipGetLastError();
}

hipError_t launch_single_coef(const uint64_t* d_s, int64_t nnz, const int32_t* J,
                              const uint32_t* orb, const int8_t* sg, int norb, const double* h,
                              const double* eri, double* c64, float* c32, int32_t* ps,
                              hipStream_t st) {
    if (nnz > 0)
        hipLaunchKernelGGL(k_single_coef, dim3(nblk(nnz, 256)), dim3(256), 0, st, d_s, nnz, J, orb,
                           sg, norb, h, eri, c64, c32, ps);
    return hipGetLastError();
}

hipError_t launch_double_coef(int64_t nnz, const uint32_t* orb, const int8_t* sg, int norb,
                              const double* eri, double* c64, float* c32, hipStream_t st) {
    if (nnz > 0)
        hipLaunchKernelGGL(k_double_coef, dim3(nblk(nnz, 256)), dim3(256), 0, st, nnz, orb, sg,
                           norb, eri, c64, c32);
    return hipGetLastError();
}

hipError_t launch_full_diag(const uint64_t* d_a, int64_t na, const double* da, const double* db,
                            const double* Gb, int64_t nb, int /*norb*/, double e_core,
                            double* diag, hipStream_t st) {
    if (na > 0 && nb > 0)
        hipLaunchKernelGGL(k_full_diag, dim3(nblk(nb, 256), (unsigned)(na < 65535 ? na : 65535)),
                           dim3(256), 0, st, d_a, na, da, db, Gb, nb, e_core, diag);
    return hipGetLastError();
}

hipError_t launch_d2f(const double* in, float* out, int64_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_d2f, dim3(nblk(n, 256)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

}  // namespace sbd
