// String sort/dedupe and same-spin excitation tables on gfx950.
//
// Sorting: bitonic network over a power-of-two padded array; stages whose
// partner distance fits a 1024-element tile run in LDS, larger distances as
// global compare-exchange passes.  Deduplication and CSR row pointers use a
// single-workgroup chunked scan (these steps run once per solve on at most a
// few million items).
//
// Excitation tables (Slater-Condon neighbourhoods, Eq. 4): one wavefront per
// bra string I scans all strings J of the spin, staged through LDS in chunks;
// popcount(I ^ J) == 2 marks a single and == 4 a double.  A wave ballot plus a
// masked popcount gives each hit its slot, so every row comes out sorted by J
// without a per-row sort.
#include "internal.h"

namespace sbd {

namespace {

constexpr int kTile = 1024;

__global__ void k_pad_max(uint64_t* a, int64_t n, int64_t P) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + n;
    if (i < P) a[i] = ~0ull;
}

__global__ void k_bitonic_global(uint64_t* a, int64_t P, int64_t k, int64_t j) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    int64_t l = i ^ j;
    if (l <= i) return;
    bool up = (i & k) == 0;
    uint64_t x = a[i], y = a[l];
    if ((x > y) == up) {
        a[i] = y;
        a[l] = x;
    }
}

// All stages j = jstart, jstart/2, ..., 1 of merge size k inside tiles of T elements.
__global__ void __launch_bounds__(kTile) k_bitonic_local(uint64_t* a, int64_t k, int64_t jstart,
                                                          int T) {
    __shared__ uint64_t s[kTile];
    int t = threadIdx.x;
    int64_t base = (int64_t)blockIdx.x * T;
    s[t] = a[base + t];
    for (int64_t j = jstart; j > 0; j >>= 1) {
        __syncthreads();
        int l = t ^ (int)j;
        if (l > t) {
            bool up = ((base + t) & k) == 0;
            uint64_t x = s[t], y = s[l];
            if ((x > y) == up) {
                s[t] = y;
                s[l] = x;
            }
        }
    }
    __syncthreads();
    a[base + t] = s[t];
}

// Block-wide exclusive scan of one int64 per thread (blockDim == 1024).
__device__ int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        int64_t add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t incl = sh[t];
    *total = sh[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

// Unique compaction of a sorted array (first n entries are the real data).
__global__ void __launch_bounds__(1024) k_unique_single(const uint64_t* a, int64_t n,
                                                        uint64_t* out, int64_t* count) {
    __shared__ int64_t sh[1024];
    int64_t carry = 0;
    for (int64_t base = 0; base < n; base += blockDim.x) {
        int64_t i = base + threadIdx.x;
        int64_t f = (i < n && (i == 0 || a[i] != a[i - 1])) ? 1 : 0;
        int64_t tot;
        int64_t pos = block_exclusive_scan(f, sh, &tot);
        if (f) out[carry + pos] = a[i];
        carry += tot;
    }
    if (threadIdx.x == 0) *count = carry;
}

// out[0] = 0, out[i+1] = sum_{k<=i} in[k]; four items per thread per chunk.
__global__ void __launch_bounds__(1024) k_scan_single(const int64_t* in, int64_t n, int64_t* out) {
    __shared__ int64_t sh[1024];
    int64_t carry = 0;
    const int per = 4;
    if (threadIdx.x == 0) out[0] = 0;
    for (int64_t base = 0; base < n; base += (int64_t)blockDim.x * per) {
        int64_t i0 = base + (int64_t)threadIdx.x * per;
        int64_t v[per];
        int64_t s = 0;
        for (int q = 0; q < per; ++q) {
            v[q] = (i0 + q < n) ? in[i0 + q] : 0;
            s += v[q];
        }
        int64_t tot;
        int64_t pre = block_exclusive_scan(s, sh, &tot);
        int64_t run = carry + pre;
        for (int q = 0; q < per; ++q) {
            run += v[q];
            if (i0 + q < n) out[i0 + q + 1] = run;
        }
        carry += tot;
    }
}

// Multi-workgroup form of the same scan for long inputs: chunk sums, a scan of
// the chunk sums, then each chunk scanned again from its offset.
constexpr int kScanPer = 4;
constexpr int64_t kScanChunk = 1024 * kScanPer;  // elements per workgroup

__global__ void __launch_bounds__(1024) k_scan_part(const int64_t* in, int64_t n, int64_t* part) {
    __shared__ int64_t sh[1024];
    const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    int64_t s = 0;
    for (int q = 0; q < kScanPer; ++q) s += (i0 + q < n) ? in[i0 + q] : 0;
    int64_t tot;
    block_exclusive_scan(s, sh, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// out[i + 1] = off[chunk] + inclusive sum of in over the chunk up to i
__global__ void __launch_bounds__(1024) k_scan_apply(const int64_t* in, int64_t n, const int64_t* off,
                                                     int64_t* out) {
    __shared__ int64_t sh[1024];
    const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    int64_t v[kScanPer];
    int64_t s = 0;
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = (i0 + q < n) ? in[i0 + q] : 0;
        s += v[q];
    }
    int64_t tot;
    int64_t run = off[blockIdx.x] + block_exclusive_scan(s, sh, &tot);
    for (int q = 0; q < kScanPer; ++q) {
        run += v[q];
        if (i0 + q < n) out[i0 + q + 1] = run;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
}

constexpr int kExcWaves = 8;        // bra strings per workgroup
constexpr int kExcChunk = 2048;     // ket strings staged in LDS per pass

__device__ __forceinline__ int wave_sum(int v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ void __launch_bounds__(kExcWaves * 64) k_exc_count(const uint64_t* __restrict__ s,
                                                              int64_t n, int64_t* cnt1,
                                                              int64_t* cnt2) {
    __shared__ uint64_t chunk[kExcChunk];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t I = (int64_t)blockIdx.x * kExcWaves + w;
    uint64_t bra = (I < n) ? s[I] : 0ull;
    int c1 = 0, c2 = 0;
    for (int64_t base = 0; base < n; base += kExcChunk) {
        int len = (int)((n - base) < kExcChunk ? (n - base) : kExcChunk);
        __syncthreads();
        for (int t = threadIdx.x; t < len; t += blockDim.x) chunk[t] = s[base + t];
        __syncthreads();
        if (I < n)
            for (int t = lane; t < len; t += 64) {
                int pc = __popcll(bra ^ chunk[t]);
                c1 += (pc == 2);
                c2 += (pc == 4);
            }
    }
    c1 = wave_sum(c1);
    c2 = wave_sum(c2);
    if (I < n && lane == 0) {
        cnt1[I] = c1;
        cnt2[I] = c2;
    }
}

__device__ __forceinline__ uint64_t below(int p) { return (1ull << p) - 1ull; }

__global__ void __launch_bounds__(kExcWaves * 64) k_exc_fill(
    const uint64_t* __restrict__ s, int64_t n, const int64_t* __restrict__ rp1,
    const int64_t* __restrict__ rp2, int32_t* J1, uint32_t* orb1, int8_t* sg1, int32_t* J2,
    uint32_t* orb2, int8_t* sg2) {
    __shared__ uint64_t chunk[kExcChunk];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t I = (int64_t)blockIdx.x * kExcWaves + w;
    uint64_t bra = (I < n) ? s[I] : 0ull;
    int64_t o1 = (I < n) ? rp1[I] : 0, o2 = (I < n) ? rp2[I] : 0;
    const uint64_t lanemask_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t base = 0; base < n; base += kExcChunk) {
        int len = (int)((n - base) < kExcChunk ? (n - base) : kExcChunk);
        __syncthreads();
        for (int t = threadIdx.x; t < len; t += blockDim.x) chunk[t] = s[base + t];
        __syncthreads();
        if (I >= n) continue;
        for (int t0 = 0; t0 < len; t0 += 64) {
            int t = t0 + lane;
            uint64_t ket = (t < len) ? chunk[t] : bra;
            int pc = __popcll(bra ^ ket);
            bool is1 = (t < len) && pc == 2;
            bool is2 = (t < len) && pc == 4;
            uint64_t m1 = __ballot(is1), m2 = __ballot(is2);
            if (is1) {
                int64_t e = o1 + __popcll(m1 & lanemask_lt);
                int i = __builtin_ctzll(ket & ~bra);  // annihilated from the ket
                int a = __builtin_ctzll(bra & ~ket);  // created
                uint64_t k1 = ket ^ (1ull << i);
                int par = __popcll(ket & below(i)) + __popcll(k1 & below(a));
                J1[e] = (int32_t)(base + t);
                orb1[e] = (uint32_t)i | ((uint32_t)a << 8);
                sg1[e] = (par & 1) ? -1 : 1;
            }
            if (is2) {
                int64_t e = o2 + __popcll(m2 & lanemask_lt);
                uint64_t x = ket & ~bra, y = bra & ~ket;
                int i = __builtin_ctzll(x);
                int j = __builtin_ctzll(x & (x - 1));
                int a = __builtin_ctzll(y);
                int b = __builtin_ctzll(y & (y - 1));
                // a+_a a+_b a_j a_i |ket>, right to left
                uint64_t k1 = ket ^ (1ull << i);
                uint64_t k2 = k1 ^ (1ull << j);
                uint64_t k3 = k2 | (1ull << b);
                int par = __popcll(ket & below(i)) + __popcll(k1 & below(j)) +
                          __popcll(k2 & below(b)) + __popcll(k3 & below(a));
                J2[e] = (int32_t)(base + t);
                orb2[e] = (uint32_t)i | ((uint32_t)j << 8) | ((uint32_t)a << 16) |
                          ((uint32_t)b << 24);
                sg2[e] = (par & 1) ? -1 : 1;
            }
            o1 += __popcll(m1);
            o2 += __popcll(m2);
        }
    }
}

__global__ void k_pack_singles(int64_t nnz, const int32_t* __restrict__ J,
                               const uint32_t* __restrict__ orb, const int8_t* __restrict__ sg,
                               uint64_t* pack) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    uint32_t o = orb[e];
    pack[e] = (uint64_t)(uint32_t)J[e] | ((uint64_t)(o & 255) << 32) |
              ((uint64_t)((o >> 8) & 255) << 40) | ((uint64_t)(sg[e] < 0 ? 1 : 0) << 48);
}

// Sliced-ELL copy of a singles table: slices of 64 consecutive strings, each
// padded to its longest row and stored slot-major (entry s of the slice's 64
// rows is contiguous), so one wavefront reading entry s of 64 consecutive
// columns issues one coalesced load.  Padding entries are ~0.
__global__ void k_sell_len(const int64_t* __restrict__ rp, const int32_t* __restrict__ pos,
                           int64_t n, int64_t nslice, int64_t* slots) {
    const int64_t sl = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (sl >= nslice) return;
    const int64_t p = sl * 64 + lane;
    const int64_t i = (p < n) ? pos[p] : 0;
    int len = (p < n) ? (int)(rp[i + 1] - rp[i]) : 0;
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(len, off, 64);
        len = o > len ? o : len;
    }
    if (lane == 0) slots[sl] = (int64_t)len * 64;
}

__global__ void k_sell_fill(const int64_t* __restrict__ rp, const uint64_t* __restrict__ pack,
                            const int32_t* __restrict__ pos, int64_t n, int64_t nslice,
                            const int64_t* __restrict__ off, uint64_t* sell) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nslice * 64) return;
    const int64_t sl = g >> 6;
    const int lane = (int)(g & 63);
    const int64_t len = (off[sl + 1] - off[sl]) / 64;
    const int64_t i = (g < n) ? pos[g] : 0;
    const int64_t r0 = (g < n) ? rp[i] : 0, rl = (g < n) ? rp[i + 1] - rp[i] : 0;
    for (int64_t s = 0; s < len; ++s)
        sell[off[sl] + s * 64 + lane] = (s < rl) ? pack[r0 + s] : ~0ull;
}

// 32-bit form of the sliced-ELL singles: J | (a*norb + i) << 18 | neg << 31;
// padding entries take J = 0 and the pair index norb*norb.
__global__ void k_sell_compact(const uint64_t* __restrict__ sell, int64_t ne, int norb, uint32_t* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const uint64_t e = sell[i];
    if (e == ~0ull) {
        out[i] = (uint32_t)(norb * norb) << kSellJBits;
        return;
    }
    const uint32_t J = (uint32_t)(e & 0xffffffffull);
    const uint32_t g = (uint32_t)((e >> 40) & 255) * (uint32_t)norb + (uint32_t)((e >> 32) & 255);
    out[i] = J | (g << kSellJBits) | ((uint32_t)((e >> 48) & 1) << 31);
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_sell_compact(const uint64_t* sell, int64_t ne, int norb, uint32_t* out, hipStream_t st) {
    if (ne > 0)
        hipLaunchKernelGGL(k_sell_compact, dim3(blocks_for(ne, 256)), dim3(256), 0, st, sell, ne, norb, out);
    return hipGetLastError();
}

hipError_t launch_sort_unique(uint64_t* d_work, int64_t n, uint64_t* d_out, int64_t* d_count,
                              int64_t* /*d_tmp*/, hipStream_t st) {
    int64_t P = 1;
    while (P < n) P <<= 1;
    if (P > n) {
        hipLaunchKernelGGL(k_pad_max, dim3(blocks_for(P - n, 256)), dim3(256), 0, st, d_work, n, P);
    }
    int T = (int)(P < kTile ? P : kTile);
    unsigned tiles = (unsigned)(P / T);
    for (int64_t k = 2; k <= P; k <<= 1) {
        int64_t j = k >> 1;
        for (; j >= T; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_global, dim3(blocks_for(P, 256)), dim3(256), 0, st,
                               d_work, P, k, j);
        hipLaunchKernelGGL(k_bitonic_local, dim3(tiles), dim3(T), 0, st, d_work, k, j, T);
    }
    hipLaunchKernelGGL(k_unique_single, dim3(1), dim3(1024), 0, st, d_work, n, d_out, d_count);
    return hipGetLastError();
}

hipError_t launch_exc_count(const uint64_t* d_s, int64_t n, int64_t* c1, int64_t* c2,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_exc_count, dim3(blocks_for(n, kExcWaves)), dim3(kExcWaves * 64), 0, st,
                       d_s, n, c1, c2);
    return hipGetLastError();
}

int64_t scan_tmp_words(int64_t n) {
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    return 2 * nb + 1;
}

hipError_t launch_exclusive_scan(const int64_t* d_in, int64_t n, int64_t* d_out, int64_t* d_tmp,
                                 hipStream_t st) {
    if (!d_tmp || n <= 4 * kScanChunk) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, d_in, n, d_out);
        return hipGetLastError();
    }
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    int64_t *part = d_tmp, *off = d_tmp + nb;  // nb chunk sums, nb + 1 offsets
    hipLaunchKernelGGL(k_scan_part, dim3((unsigned)nb), dim3(1024), 0, st, d_in, n, part);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, part, nb, off);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(1024), 0, st, d_in, n, off, d_out);
    return hipGetLastError();
}

hipError_t launch_exc_fill(const uint64_t* d_s, int64_t n, const int64_t* rp1, const int64_t* rp2,
                           int32_t* J1, uint32_t* orb1, int8_t* sg1, int32_t* J2, uint32_t* orb2,
                           int8_t* sg2, hipStream_t st) {
    hipLaunchKernelGGL(k_exc_fill, dim3(blocks_for(n, kExcWaves)), dim3(kExcWaves * 64), 0, st,
                       d_s, n, rp1, rp2, J1, orb1, sg1, J2, orb2, sg2);
    return hipGetLastError();
}

hipError_t launch_sell_len(const int64_t* rp, const int32_t* pos, int64_t n, int64_t* slots,
                           hipStream_t st) {
    const int64_t nslice = (n + 63) / 64;
    if (nslice > 0)
        hipLaunchKernelGGL(k_sell_len, dim3(blocks_for(nslice, 4)), dim3(256), 0, st, rp, pos, n,
                           nslice, slots);
    return hipGetLastError();
}

hipError_t launch_sell_fill(const int64_t* rp, const uint64_t* pack, const int32_t* pos, int64_t n,
                            const int64_t* off, uint64_t* sell, hipStream_t st) {
    const int64_t nslice = (n + 63) / 64;
    if (nslice > 0)
        hipLaunchKernelGGL(k_sell_fill, dim3(blocks_for(nslice * 64, 256)), dim3(256), 0, st, rp,
                           pack, pos, n, nslice, off, sell);
    return hipGetLastError();
}

hipError_t launch_pack_singles(int64_t nnz, const int32_t* J, const uint32_t* orb, const int8_t* sg,
                               uint64_t* pack, hipStream_t st) {
    if (nnz > 0)
        hipLaunchKernelGGL(k_pack_singles, dim3(blocks_for(nnz, 256)), dim3(256), 0, st, nnz, J, orb,
                           sg, pack);
    return hipGetLastError();
}

}  // namespace sbd
