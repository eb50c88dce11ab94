// Matrix-free sigma = (H - shift) c over the alpha x beta determinant basis
// (Eq. 4; the three task types of Sec. III-B).
//
// Vectors are stored alpha-major, c[ia][ib] (index ia*nb + ib), optionally
// with nv vectors interleaved per determinant ([ia][ib][v]).  One sigma is
// five launches on one stream:
//
//   1. transpose   cT[ib][ia] = c[ia][ib]                         (LDS tiles)
//   2. stream      y[ia][:]  = (H_diag - shift) c[ia][:]
//                            + sum_{Ja in S1/S2 alpha(ia)} coef * c[Ja][:]   (task 2)
//   3. stream      yT[ib][:] = sum_{Jb in S1/S2 beta(ib)} coef * cT[Jb][:]   (task 1)
//   4. alpha-beta  y[ia][ib] += sum_{Ja in S1a(ia)} sum_{Jb in S1b(ib)}
//                              sa sb (a_a i_a | b_b j_b) c[Ja][Jb]         (task 0)
//   5. transpose   y[ia][ib] += yT[ib][ia]                          (LDS tiles)
//
// The same-spin work (tasks 1 and 2, about 65-95 % of all connected pairs)
// thus becomes a row stream: one wavefront owns one output row and one
// 64-column tile, walks the row's excitation list with wave-uniform (scalar)
// loads of the ket index and coefficient, and reads the ket row segment with
// one coalesced load per entry.  Tiles are assigned so that the workgroups
// resident on one XCD share a column tile, keeping in[:, tile] in that XCD's
// L2.  The alpha-beta term stages the ket row c[Ja][:] and the integral slice
// (a_a i_a | . .) in LDS and gathers from there.
//
// Every output element is written by one owner in a fixed order: no atomics,
// results are bitwise reproducible.
#include "internal.h"

namespace sbd {
namespace {

// ------------------------------------------------------------------ transpose
template <class T, int NV, bool ADD>
__global__ void __launch_bounds__(256) k_transpose(const T* __restrict__ in, T* __restrict__ out,
                                                   int64_t nrow, int64_t ncol, int64_t nby) {
    constexpr int TD = 32;
    __shared__ T tile[TD][TD * NV + 1];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int64_t c0 = (int64_t)blockIdx.x * TD;
    for (int64_t by = blockIdx.y; by < nby; by += gridDim.y) {
        const int64_t r0 = by * TD;
        __syncthreads();
        for (int j = ty; j < TD; j += 8) {
            const int64_t r = r0 + j, c = c0 + tx;
            if (r < nrow && c < ncol) {
#pragma unroll
                for (int v = 0; v < NV; ++v) tile[j][tx * NV + v] = in[(r * ncol + c) * NV + v];
            }
        }
        __syncthreads();
        for (int j = ty; j < TD; j += 8) {
            const int64_t c = c0 + j, r = r0 + tx;
            if (c < ncol && r < nrow) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const T val = tile[tx][j * NV + v];
                    T* dst = out + (c * nrow + r) * NV + v;
                    if (ADD)
                        *dst += val;
                    else
                        *dst = val;
                }
            }
        }
    }
}

// Single-vector transpose with 16-byte accesses on both sides: a TD x TD tile
// (64 x 64 floats) is read as rows of 16 vectors of E = 16/sizeof(T)
// elements, staged in LDS, and written as rows of the transpose.  Needs ncol
// and nrow to be multiples of E (16-byte aligned rows).
template <class T, bool ADD>
__global__ void __launch_bounds__(256) k_transpose_v(const T* __restrict__ in, T* __restrict__ out,
                                                     int64_t nrow, int64_t ncol, int64_t nby) {
    constexpr int E = 16 / (int)sizeof(T);
    constexpr int TD = 16 * E;
    constexpr int RPT = TD / 16;  // tile rows per thread per phase
    __shared__ T tile[TD][TD + 1];
    const int tv = threadIdx.x & 15, tr = threadIdx.x >> 4;  // vector column, row group
    const int64_t c0 = (int64_t)blockIdx.x * TD;
    for (int64_t by = blockIdx.y; by < nby; by += gridDim.y) {
        const int64_t r0 = by * TD;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int j = tr + 16 * k;
            const int64_t r = r0 + j, c = c0 + tv * E;
            if (r < nrow && c < ncol) {
                const float4 q = *reinterpret_cast<const float4*>(in + r * ncol + c);
                T v[E];
                __builtin_memcpy(v, &q, 16);
#pragma unroll
                for (int e = 0; e < E; ++e) tile[j][tv * E + e] = v[e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int j = tr + 16 * k;             // output row within the tile (input column)
            const int64_t c = c0 + j, r = r0 + tv * E;
            if (c < ncol && r < nrow) {
                T v[E];
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = tile[tv * E + e][j];
                float4* dst = reinterpret_cast<float4*>(out + c * nrow + r);
                if (ADD) {
                    const float4 o = *dst;
                    T w[E];
                    __builtin_memcpy(w, &o, 16);
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] += w[e];
                }
                float4 q;
                __builtin_memcpy(&q, v, 16);
                *dst = q;
            }
        }
    }
}

// ------------------------------------------------------------------ row stream
template <class T>
struct StreamArgs {
    int64_t nrow, ncol;
    int64_t ntiles, row_blocks;
    int rows_per_wg;
    const int64_t* p1; const int32_t* J1; const T* c1; const int32_t* ps1;
    const int64_t* p2; const int32_t* J2; const T* c2;
    const T* G;           // [npair][ncol]: spectator of the column spin
    const double* diag;   // [nrow][ncol] or null
    double shift;
};

// Broadcast lane k's value of v to the whole wavefront (k wave-uniform).
__device__ __forceinline__ int bcast(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ float bcast(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double bcast(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Load W = VEC*NV consecutive values (vectorised when aligned by construction).
template <class T, int W>
struct Vec {
    T x[W];
};
template <class T, int W>
__device__ __forceinline__ Vec<T, W> vload(const T* p) {
    Vec<T, W> v;
    if constexpr (W * sizeof(T) == 16) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        __builtin_memcpy(&v, &q, 16);
    } else if constexpr (W * sizeof(T) == 8) {
        const float2 q = *reinterpret_cast<const float2*>(p);
        __builtin_memcpy(&v, &q, 8);
    } else {
#pragma unroll
        for (int i = 0; i < W; ++i) v.x[i] = p[i];
    }
    return v;
}

// One wavefront = RW output rows (RW = 1 or 2) and VEC*64/RW consecutive
// columns: with RW = 2 each half-wave owns one row, which halves the column
// tile (and so the per-XCD working set in[:, tile]) at the same bytes per load
// instruction.  Each row's entry list is fetched with one vector load per 64/RW
// entries and broadcast lane by lane (v_readlane), so ket-row loads never wait
// on scalar memory; 8 (narrow elements) or 4 ket rows are in flight per step.
template <class T, int NV, int VEC, int RW>
__global__ void __launch_bounds__(256) k_stream(StreamArgs<T> A, const T* __restrict__ in,
                                                T* __restrict__ out) {
    constexpr int W = NV * VEC;
    constexpr int HL = 64 / RW;  // lanes per row
    constexpr int UNR = W * (int)sizeof(T) <= 16 ? 8 : 4;  // ket rows in flight per step
    const int lane = threadIdx.x & 63;
    const int half = RW == 2 ? (lane >> 5) : 0;
    const int hl = lane & (HL - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // workgroups are dispatched round-robin over the 8 XCDs: give each XCD its
    // own sequence of column tiles so its resident waves share one tile
    const int64_t g = blockIdx.x;
    const int xcd = (int)(g & 7);
    const int64_t l = g >> 3;
    const int64_t tl = l / A.row_blocks;
    const int64_t rb = l - tl * A.row_blocks;
    const int64_t tile = tl * 8 + xcd;
    const int64_t rwave = (rb * A.rows_per_wg + wv) * RW;  // first row of this wave
    if (tile >= A.ntiles || rwave >= A.nrow || wv >= A.rows_per_wg) return;
    const int64_t r = rwave + half;
    const bool rok = r < A.nrow;
    const int64_t rr = rok ? r : rwave;
    const int64_t ncol = A.ncol;
    const int64_t col = (tile * HL + hl) * VEC;   // first of VEC columns (ncol % VEC == 0)
    const bool act = rok && col < ncol;
    const int64_t cc = col < ncol ? col : 0;

    T acc[W];
    if (A.diag) {
        const Vec<T, W> x = vload<T, W>(in + (rr * ncol + cc) * NV);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            const T dg = (T)(A.diag[rr * ncol + cc + q] - A.shift);
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[q * NV + v] = dg * x.x[q * NV + v];
        }
    } else {
#pragma unroll
        for (int i = 0; i < W; ++i) acc[i] = T(0);
    }
    // entry ranges of the wave's rows (uniform per half)
    const int64_t r0 = rwave, r1 = (RW == 2 && rwave + 1 < A.nrow) ? rwave + 1 : rwave;
    // singles: coefficient = base + sign * G[pair][col]
    {
        const int64_t a0 = A.p1[r0], a1 = A.p1[r0 + 1];
        const int64_t b0 = A.p1[r1], b1 = (RW == 2 && r1 != r0) ? A.p1[r1 + 1] : b0;
        const int64_t my0 = half ? b0 : a0, my1 = half ? b1 : a1;
        const int64_t n0 = a1 - a0, n1 = b1 - b0;
        const int64_t nmax = n0 > n1 ? n0 : n1;
        for (int64_t base = 0; base < nmax; base += HL) {
            const int64_t mine = my1 - my0 - base;
            const int cnt = (int)(mine < HL ? (mine < 0 ? 0 : mine) : HL);
            const int mj = hl < cnt ? A.J1[my0 + base + hl] : 0;
            const int mp = hl < cnt ? A.ps1[my0 + base + hl] : 0;
            const T mc = hl < cnt ? A.c1[my0 + base + hl] : T(0);
            const int64_t lim = (nmax - base) < HL ? (nmax - base) : HL;
            for (int k = 0; k < lim; ++k) {
                int j = bcast(mj, k), ps = bcast(mp, k);
                T cb = bcast(mc, k);
                if (RW == 2) {
                    const int j2 = bcast(mj, k + 32), p2 = bcast(mp, k + 32);
                    const T c2 = bcast(mc, k + 32);
                    j = half ? j2 : j;
                    ps = half ? p2 : ps;
                    cb = half ? c2 : cb;
                }
                if (k < cnt) {
                    const Vec<T, VEC> gv = vload<T, VEC>(A.G + (int64_t)(ps >> 1) * ncol + cc);
                    const Vec<T, W> x = vload<T, W>(in + ((int64_t)j * ncol + cc) * NV);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) {
                        const T coef = cb + ((ps & 1) ? -gv.x[q] : gv.x[q]);
#pragma unroll
                        for (int v = 0; v < NV; ++v) acc[q * NV + v] += coef * x.x[q * NV + v];
                    }
                }
            }
        }
    }
    // doubles: coefficient per entry; UNR ket rows in flight
    {
        const int64_t a0 = A.p2[r0], a1 = A.p2[r0 + 1];
        const int64_t b0 = A.p2[r1], b1 = (RW == 2 && r1 != r0) ? A.p2[r1 + 1] : b0;
        const int64_t my0 = half ? b0 : a0, my1 = half ? b1 : a1;
        const int64_t n0 = a1 - a0, n1 = b1 - b0;
        const int64_t nmax = n0 > n1 ? n0 : n1;
        for (int64_t base = 0; base < nmax; base += HL) {
            const int64_t mine = my1 - my0 - base;
            const int cnt = (int)(mine < HL ? (mine < 0 ? 0 : mine) : HL);
            const int mj = hl < cnt ? A.J2[my0 + base + hl] : 0;
            const T mc = hl < cnt ? A.c2[my0 + base + hl] : T(0);
            const int lim = (int)((nmax - base) < HL ? (nmax - base) : HL);
            for (int k = 0; k < lim; k += UNR) {
                int j[UNR];
                T f[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int kk = (k + u) < HL ? (k + u) : (HL - 1);
                    int jv = bcast(mj, kk);
                    T fv = bcast(mc, kk);
                    if (RW == 2) {
                        const int j2 = bcast(mj, kk + 32);
                        const T f2 = bcast(mc, kk + 32);
                        jv = half ? j2 : jv;
                        fv = half ? f2 : fv;
                    }
                    const bool ok = (k + u) < cnt;
                    j[u] = ok ? jv : (int)rr;   // padded entries read a valid row with weight 0
                    f[u] = ok ? fv : T(0);
                }
                Vec<T, W> x[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) x[u] = vload<T, W>(in + ((int64_t)j[u] * ncol + cc) * NV);
#pragma unroll
                for (int u = 0; u < UNR; ++u)
#pragma unroll
                    for (int i = 0; i < W; ++i) acc[i] += f[u] * x[u].x[i];
            }
        }
    }
    if (act) {
        T* dst = out + (r * ncol + col) * NV;
#pragma unroll
        for (int i = 0; i < W; ++i) dst[i] = acc[i];
    }
}

// Ket-split form: one wavefront = one output row and (64/G)*VEC consecutive
// columns; its lanes form G groups that take G different ket entries of the row
// per load step (group g takes entries g, g+G, ...; each lane gets its entry by
// a lane shuffle).  A load instruction still moves 64 lanes' worth of bytes, but
// the column tile, and so the per-XCD working set in[:, tile], is G times
// narrower than the one-row form's.  The G partial sums of a column are added
// across the groups at the end of the row in a fixed order.
template <class T, int NV, int VEC, int G>
__global__ void __launch_bounds__(256) k_stream_ks(StreamArgs<T> A, const T* __restrict__ in,
                                                   T* __restrict__ out) {
    constexpr int W = NV * VEC;
    constexpr int GL = 64 / G;  // lanes per group
    constexpr int UNR = W * (int)sizeof(T) <= 16 ? 8 : 4;  // load steps in flight
    const int lane = threadIdx.x & 63;
    const int grp = lane / GL, gl = lane % GL;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t g = blockIdx.x;
    const int xcd = (int)(g & 7);
    const int64_t l = g >> 3;
    const int64_t tl = l / A.row_blocks;
    const int64_t rb = l - tl * A.row_blocks;
    const int64_t tile = tl * 8 + xcd;
    const int64_t r = rb * A.rows_per_wg + wv;
    if (tile >= A.ntiles || r >= A.nrow || wv >= A.rows_per_wg) return;  // wave-uniform
    const int64_t ncol = A.ncol;
    const int64_t col = (tile * GL + gl) * VEC;  // first of VEC columns (ncol % VEC == 0)
    const bool act = col < ncol;
    const int64_t cc = act ? col : 0;

    T acc[W];
#pragma unroll
    for (int i = 0; i < W; ++i) acc[i] = T(0);
    if (A.diag && grp == 0) {
        const Vec<T, W> x = vload<T, W>(in + (r * ncol + cc) * NV);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            const T dg = (T)(A.diag[r * ncol + cc + q] - A.shift);
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[q * NV + v] = dg * x.x[q * NV + v];
        }
    }
    // singles: coefficient = base + sign * G[pair][col]
    {
        const int64_t a0 = A.p1[r], a1 = A.p1[r + 1];
        for (int64_t base = a0; base < a1; base += 64) {
            const int cnt = (int)((a1 - base) < 64 ? (a1 - base) : 64);
            const int mj = lane < cnt ? A.J1[base + lane] : 0;
            const int mp = lane < cnt ? A.ps1[base + lane] : 0;
            const T mc = lane < cnt ? A.c1[base + lane] : T(0);
            for (int s = 0; s < cnt; s += G) {
                const int k = s + grp;
                const int j = __shfl(mj, k & 63, 64), ps = __shfl(mp, k & 63, 64);
                const T cb = __shfl(mc, k & 63, 64);
                if (k < cnt) {
                    const Vec<T, VEC> gv = vload<T, VEC>(A.G + (int64_t)(ps >> 1) * ncol + cc);
                    const Vec<T, W> x = vload<T, W>(in + ((int64_t)j * ncol + cc) * NV);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) {
                        const T coef = cb + ((ps & 1) ? -gv.x[q] : gv.x[q]);
#pragma unroll
                        for (int v = 0; v < NV; ++v) acc[q * NV + v] += coef * x.x[q * NV + v];
                    }
                }
            }
        }
    }
    // doubles: UNR steps of G entries in flight
    {
        const int64_t a0 = A.p2[r], a1 = A.p2[r + 1];
        for (int64_t base = a0; base < a1; base += 64) {
            const int cnt = (int)((a1 - base) < 64 ? (a1 - base) : 64);
            const int mj = lane < cnt ? A.J2[base + lane] : 0;
            const T mc = lane < cnt ? A.c2[base + lane] : T(0);
            for (int s = 0; s < cnt; s += G * UNR) {
                int j[UNR];
                T f[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int k = s + u * G + grp;
                    const int jv = __shfl(mj, k & 63, 64);
                    const T fv = __shfl(mc, k & 63, 64);
                    const bool ok = k < cnt;
                    j[u] = ok ? jv : (int)r;  // padded entries read a valid row with weight 0
                    f[u] = ok ? fv : T(0);
                }
                Vec<T, W> x[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u)
                    if (s + u * G < cnt)  // wave-uniform: skip steps past the row's end
                        x[u] = vload<T, W>(in + ((int64_t)j[u] * ncol + cc) * NV);
#pragma unroll
                for (int u = 0; u < UNR; ++u)
                    if (s + u * G < cnt)
#pragma unroll
                        for (int i = 0; i < W; ++i) acc[i] += f[u] * x[u].x[i];
            }
        }
    }
    // sum over the groups: (g0 + g1) + (g2 + g3), the same in every lane
#pragma unroll
    for (int i = 0; i < W; ++i) {
        if constexpr (G >= 2) acc[i] += __shfl_xor(acc[i], GL, 64);
        if constexpr (G >= 4) acc[i] += __shfl_xor(acc[i], 2 * GL, 64);
    }
    if (act && grp == 0) {
        T* dst = out + (r * ncol + col) * NV;
#pragma unroll
        for (int i = 0; i < W; ++i) dst[i] = acc[i];
    }
}

// ------------------------------------------------------------------ alpha-beta
template <class T>
struct AbArgs {
    int64_t na, nb;
    int norb;
    int64_t win;        // ket-row window staged in LDS (determinants)
    int krows;          // alpha singles (ket rows) staged together
    const int64_t* a1p; const uint64_t* a1pack;
    const uint64_t* b1sell; const int64_t* b1sell_off;  // beta singles, sliced-ELL
    const int32_t* b1pos;                               // beta string of each ELL position
    const T* eri;
};

// Copy n elements global -> LDS with 16-byte loads for the aligned body
// (scalar head and tail, so nothing outside [src, src+n) is read).
template <class T>
__device__ __forceinline__ void stage_row(T* __restrict__ dst, const T* __restrict__ src, int64_t n) {
    constexpr int E = 16 / sizeof(T);
    const int bd = blockDim.x, tid = threadIdx.x;
    int64_t head = (int64_t)(((16 - ((uintptr_t)src & 15)) & 15) / sizeof(T));
    if (head > n) head = n;
    for (int64_t k = tid; k < head; k += bd) dst[k] = src[k];
    const int64_t nv = (n - head) / E;
    const float4* s4 = reinterpret_cast<const float4*>(src + head);
    T* d = dst + head;
#pragma unroll 4
    for (int64_t k = tid; k < nv; k += bd) {
        const float4 q = s4[k];
        T tmp[E];
        __builtin_memcpy(tmp, &q, 16);
#pragma unroll
        for (int i = 0; i < E; ++i) d[k * E + i] = tmp[i];
    }
    for (int64_t k = head + nv * E + tid; k < n; k += bd) dst[k] = src[k];
}

// One workgroup = one bra row ia and a block of Q*blockDim columns.  The
// alpha singles (Ja, i_a -> a_a) of ia are taken K at a time: their ket rows
// c[Ja][:] (or a window of them) and integral slices (a_a i_a | . .) are staged
// in LDS, then each thread walks the beta singles of its Q positions.  The beta
// singles are read from the sliced-ELL table, so entry s of a wavefront's 64
// positions is one coalesced load; each entry is loaded once per group of K
// rows, and the Q positions' entries are fetched step by step (independent
// loads).  Position p holds beta string b1pos[p]: the table's positions are
// arranged so the workgroup's wavefronts carry similar work (sell_positions).
template <class T, int NV, int Q>
__global__ void __launch_bounds__(1024) k_ab(AbArgs<T> A, const T* __restrict__ c,
                                             T* __restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = A.norb;
    const int sl_stride = (n * n + 3) & ~3;
    const int K = A.krows;
    T* slices = reinterpret_cast<T*>(smem);
    T* rows = slices + (size_t)K * sl_stride;
    const int64_t row_stride = A.win * NV;
    const int64_t ia = blockIdx.x;
    const int64_t nb = A.nb;
    const int64_t col0 = (int64_t)blockIdx.y * blockDim.x * Q + threadIdx.x;
    const int64_t t0 = A.a1p[ia], t1 = A.a1p[ia + 1];
    if (t0 == t1) return;  // no alpha single: nothing to add (uniform exit)

    // beta singles of the wave's 64-column slices: one slice per q, read slot-major
    const int lane = threadIdx.x & 63;
    const int64_t wcol0 = (int64_t)blockIdx.y * blockDim.x * Q + (threadIdx.x & ~63);
    T acc[Q][NV];
    int64_t soff[Q];
    int slen[Q];
    int maxlen = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t ibw = wcol0 + (int64_t)q * blockDim.x;
        const int64_t sl = ibw >> 6;
        soff[q] = (ibw < nb) ? A.b1sell_off[sl] : 0;
        slen[q] = (ibw < nb) ? (int)((A.b1sell_off[sl + 1] - soff[q]) >> 6) : 0;
        maxlen = slen[q] > maxlen ? slen[q] : maxlen;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[q][v] = T(0);
    }
    for (int64_t tg = t0; tg < t1; tg += K) {
        const int kk = (int)((t1 - tg) < K ? (t1 - tg) : K);
        int sa_bits = 0;
        for (int tt = 0; tt < kk; ++tt) sa_bits |= (int)((A.a1pack[tg + tt] >> 48) & 1) << tt;
        for (int64_t w0 = 0; w0 < nb; w0 += A.win) {
            const int64_t wl = (nb - w0) < A.win ? (nb - w0) : A.win;
            __syncthreads();
            for (int tt = 0; tt < kk; ++tt) {
                const uint64_t pa = A.a1pack[tg + tt];
                const int64_t ja = (int64_t)(pa & 0xffffffffull);
                if (w0 == 0) {
                    const int ai = (int)((pa >> 32) & 255), aa = (int)((pa >> 40) & 255);
                    const T* sl = A.eri + ((size_t)aa * n + ai) * n * n;  // (a_a i_a | . .)
                    for (int k = threadIdx.x; k < n * n; k += blockDim.x)
                        slices[tt * sl_stride + k] = sl[k];
                }
                stage_row<T>(rows + tt * row_stride, c + (ja * nb + w0) * NV, wl * NV);
            }
            __syncthreads();
            for (int s = 0; s < maxlen; ++s) {
                uint64_t pb[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q)
                    pb[q] = (s < slen[q]) ? A.b1sell[soff[q] + (int64_t)s * 64 + lane] : ~0ull;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    if (pb[q] == ~0ull) continue;
                    const int64_t jb = (int64_t)(pb[q] & 0xffffffffull) - w0;
                    if (jb < 0 || jb >= wl) continue;
                    const int gidx = (int)((pb[q] >> 40) & 255) * n + (int)((pb[q] >> 32) & 255);
                    const int sb = (int)((pb[q] >> 48) & 1);
                    for (int tt = 0; tt < kk; ++tt) {
                        const T gv = slices[tt * sl_stride + gidx];
                        const T coef = (((sa_bits >> tt) & 1) ^ sb) ? -gv : gv;
                        const T* x = rows + tt * row_stride + jb * NV;
#pragma unroll
                        for (int v = 0; v < NV; ++v) acc[q][v] += coef * x[v];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t p = col0 + (int64_t)q * blockDim.x;  // sliced-ELL position
        if (p < nb) {
            const int64_t ib = A.b1pos[p];
            T* dst = y + (ia * nb + ib) * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) dst[v] += acc[q][v];
        }
    }
}

// Alpha-beta term over the 32-bit sliced-ELL beta singles (Table::sell32).  The
// same work as k_ab with a lean walk: the alpha single's sign is folded into
// its staged integral slice, the beta single's sign is the entry's top bit, and
// padding entries read a zero placed after the slice, so the walk has no
// per-lane branches; a wavefront's 64 positions form one slice, so its slot
// loop is uniform (scalar loop bound and offsets).  WIN: ket rows staged in
// column windows (entries outside the window read the zero).
template <class T>
struct Ab2Args {
    int64_t na, nb;
    int norb;
    int64_t win;    // ket columns staged per row (nb: whole rows)
    int krows;      // alpha singles staged together
    const int64_t* a1p;
    const uint64_t* a1pack;
    const uint32_t* sell;
    const int64_t* sell_off;
    const int32_t* pos;
    const T* eri;
};

template <class T, int NV, int Q, int KT, bool WIN>
__global__ void __launch_bounds__(1024) k_ab2(Ab2Args<T> A, const T* __restrict__ c, T* __restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = A.norb, n2 = n * n;
    const int S = (n2 + 1 + 3) & ~3;  // slice stride: the pair's integrals, then a zero
    T* slices = reinterpret_cast<T*>(smem);
    T* rows = slices + (size_t)KT * S;
    const int64_t rstride = A.win * NV;
    const int64_t ia = blockIdx.x;
    const int64_t nb = A.nb;
    const int64_t t0 = A.a1p[ia], t1 = A.a1p[ia + 1];
    if (t0 == t1) return;  // no alpha single: nothing to add (uniform exit)
    const int lane = threadIdx.x & 63;
    const int64_t wcol0 = (int64_t)blockIdx.y * blockDim.x * Q +
                          __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63u));
    int64_t soff[Q];
    int slen[Q];
    T acc[Q][NV];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t ibw = wcol0 + (int64_t)q * blockDim.x;
        const int64_t sl = ibw >> 6;
        soff[q] = ibw < nb ? A.sell_off[sl] : 0;
        slen[q] = ibw < nb ? (int)((A.sell_off[sl + 1] - A.sell_off[sl]) >> 6) : 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[q][v] = T(0);
    }
    const uint32_t jmask = (1u << kSellJBits) - 1u;
    const uint32_t pad = (uint32_t)n2 << kSellJBits;  // reads the zero after the slice
    constexpr int UA = 4;  // entries whose loads, then LDS reads, are issued together
    for (int64_t tg = t0; tg < t1; tg += KT) {
        const int kk = (int)((t1 - tg) < KT ? (t1 - tg) : KT);
        // rows of unused slots alias row 0: their slices are all zero
        int rb[KT];
#pragma unroll
        for (int tt = 0; tt < KT; ++tt) rb[tt] = (tt < kk ? tt : 0) * (int)rstride;
        for (int64_t w0 = 0; w0 < nb; w0 += A.win) {
            const int64_t wl = (nb - w0) < A.win ? (nb - w0) : A.win;
            __syncthreads();
            for (int tt = 0; tt < KT; ++tt) {
                if (w0 == 0) {  // (a_a i_a | . .) times the alpha single's sign; zeros for unused slots
                    if (tt < kk) {
                        const uint64_t pa = A.a1pack[tg + tt];
                        const int ai = (int)((pa >> 32) & 255), aa = (int)((pa >> 40) & 255);
                        const bool neg = (pa >> 48) & 1;
                        const T* sl = A.eri + ((size_t)aa * n + ai) * n2;
                        for (int k = threadIdx.x; k < n2; k += blockDim.x) {
                            const T v = sl[k];
                            slices[tt * S + k] = neg ? -v : v;
                        }
                    } else {
                        for (int k = threadIdx.x; k < n2; k += blockDim.x) slices[tt * S + k] = T(0);
                    }
                    if (threadIdx.x == 0) slices[tt * S + n2] = T(0);
                }
                if (tt < kk) {
                    const int64_t ja = (int64_t)(A.a1pack[tg + tt] & 0xffffffffull);
                    stage_row<T>(rows + tt * rstride, c + (ja * nb + w0) * NV, wl * NV);
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const uint32_t* ep = A.sell + soff[q] + lane;
                const int L = slen[q];
                // UA slots' entries are loaded before any is used (slots past the
                // slice's end read as padding), then all their LDS reads are issued
                for (int s = 0; s < L; s += UA) {
                    uint32_t e[UA];
#pragma unroll
                    for (int u = 0; u < UA; ++u) e[u] = (s + u < L) ? ep[(int64_t)(s + u) * 64] : pad;
                    T gv[UA][KT], xv[UA][KT][NV];
                    bool ng[UA];
#pragma unroll
                    for (int u = 0; u < UA; ++u) {
                        int jb = (int)(e[u] & jmask);
                        int g = (int)((e[u] >> kSellJBits) & 0x1fffu);
                        ng[u] = (e[u] >> 31) != 0;
                        if (WIN) {
                            const bool in = (unsigned)(jb - w0) < (unsigned)wl;
                            jb = in ? (int)(jb - w0) : 0;
                            g = in ? g : n2;
                        }
#pragma unroll
                        for (int tt = 0; tt < KT; ++tt) {
                            gv[u][tt] = slices[tt * S + g];
#pragma unroll
                            for (int v = 0; v < NV; ++v) xv[u][tt][v] = rows[rb[tt] + jb * NV + v];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < UA; ++u)
#pragma unroll
                        for (int tt = 0; tt < KT; ++tt) {
                            const T gs = ng[u] ? -gv[u][tt] : gv[u][tt];
#pragma unroll
                            for (int v = 0; v < NV; ++v) acc[q][v] += gs * xv[u][tt][v];
                        }
                }
            }
        }
    }
    const int64_t col0 = (int64_t)blockIdx.y * blockDim.x * Q + threadIdx.x;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t p = col0 + (int64_t)q * blockDim.x;  // sliced-ELL position
        if (p < nb) {
            const int64_t ib = A.pos[p];
            T* dst = y + (ia * nb + ib) * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) dst[v] += acc[q][v];
        }
    }
}

// ------------------------------------------------------------------ launchers
// 16-byte aligned (vectors are only guaranteed 8-byte alignment)
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

template <class T, int NV, bool ADD>
hipError_t transpose(const T* in, T* out, int64_t nrow, int64_t ncol, hipStream_t st) {
    constexpr int E = 16 / (int)sizeof(T);
    // FP32 only: for FP64 the 32 x 32 tile's 8-byte accesses are already 256-byte rows and measure faster
    if (sizeof(T) == 4 && NV == 1 && ncol % E == 0 && nrow % E == 0 && aligned16(in) && aligned16(out)) {
        constexpr int TD = 16 * E;
        const int64_t nbx = (ncol + TD - 1) / TD, nby = (nrow + TD - 1) / TD;
        const unsigned gy = (unsigned)(nby < 65535 ? nby : 65535);
        hipLaunchKernelGGL((k_transpose_v<T, ADD>), dim3((unsigned)nbx, gy), dim3(256), 0, st, in, out,
                           nrow, ncol, nby);
        return hipGetLastError();
    }
    const int64_t nbx = (ncol + 31) / 32, nby = (nrow + 31) / 32;
    const unsigned gy = (unsigned)(nby < 65535 ? nby : 65535);
    hipLaunchKernelGGL((k_transpose<T, NV, ADD>), dim3((unsigned)nbx, gy), dim3(256), 0, st, in,
                       out, nrow, ncol, nby);
    return hipGetLastError();
}

template <class T, int NV, int VEC, int G>
hipError_t stream_ks(StreamArgs<T> S, const T* in, T* out, int rows_per_wg, hipStream_t st) {
    S.rows_per_wg = rows_per_wg;
    S.ntiles = (S.ncol + (64 / G) * VEC - 1) / ((64 / G) * VEC);
    S.row_blocks = (S.nrow + rows_per_wg - 1) / rows_per_wg;
    const int64_t tiles8 = (S.ntiles + 7) / 8 * 8;
    const int64_t nblk = tiles8 * S.row_blocks;
    if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_stream_ks<T, NV, VEC, G>), dim3((unsigned)nblk), dim3(64 * rows_per_wg), 0,
                       st, S, in, out);
    return hipGetLastError();
}

template <class T, int NV, int VEC, int RW>
hipError_t stream_vec(StreamArgs<T> S, const T* in, T* out, int rows_per_wg, hipStream_t st) {
    S.rows_per_wg = rows_per_wg;
    S.ntiles = (S.ncol + (64 / RW) * VEC - 1) / ((64 / RW) * VEC);
    const int64_t rows_per_block = (int64_t)rows_per_wg * RW;
    S.row_blocks = (S.nrow + rows_per_block - 1) / rows_per_block;
    const int64_t tiles8 = (S.ntiles + 7) / 8 * 8;
    const int64_t nblk = tiles8 * S.row_blocks;
    if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_stream<T, NV, VEC, RW>), dim3((unsigned)nblk), dim3(64 * rows_per_wg), 0,
                       st, S, in, out);
    return hipGetLastError();
}

template <class T, int NV, int VEC>
hipError_t stream_rw(StreamArgs<T> S, const T* in, T* out, const SigmaTune& tune, hipStream_t st) {
    if (tune.stream_split == 4) return stream_ks<T, NV, VEC, 4>(S, in, out, tune.stream_rows, st);
    if (tune.stream_split == 2) return stream_ks<T, NV, VEC, 2>(S, in, out, tune.stream_rows, st);
    if (tune.stream_rw == 2) return stream_vec<T, NV, VEC, 2>(S, in, out, tune.stream_rows, st);
    return stream_vec<T, NV, VEC, 1>(S, in, out, tune.stream_rows, st);
}

// Columns per lane: B gives 8-byte lane loads (FP32 single vectors take two
// columns); the wide form doubles that to 16-byte loads where the vector width
// allows.  Both need every row to start on a multiple of VEC columns.
template <class T, int NV>
hipError_t stream(StreamArgs<T> S, const T* in, T* out, const SigmaTune& tune, hipStream_t st) {
    constexpr int B = NV * (int)sizeof(T) >= 8 ? 1 : 8 / (NV * (int)sizeof(T));
    constexpr bool CAN_WIDE = NV * (int)sizeof(T) * B * 2 <= 16;
    if constexpr (CAN_WIDE) {
        if (tune.stream_wide && S.ncol % (2 * B) == 0 && aligned16(in) && aligned16(out))
            return stream_rw<T, NV, 2 * B>(S, in, out, tune, st);
    }
    if constexpr (B > 1) {
        if (S.ncol % B != 0) return stream_rw<T, NV, 1>(S, in, out, tune, st);
    }
    return stream_rw<T, NV, B>(S, in, out, tune, st);
}

int max_lds_per_block() {
    static const int v = [] {
        int dev = 0, x = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            x = 65536;
        return x;
    }();
    return v;
}

template <class T, int NV, int Q>
hipError_t ab_launch(const AbArgs<T>& A, const T* c, T* y, int threads, size_t lds, int64_t passes,
                     hipStream_t st) {
    auto kern = k_ab<T, NV, Q>;
    // raise the dynamic LDS limit to the hardware maximum once per instantiation (thread-safe,
    // and never inside a stream capture after the first eager launch)
    static const hipError_t attr = max_lds_per_block() > 65536
                                       ? hipFuncSetAttribute((const void*)kern,
                                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                                             max_lds_per_block())
                                       : hipSuccess;
    if (lds > 65536 && attr != hipSuccess) return attr;
    hipLaunchKernelGGL(kern, dim3((unsigned)A.na, (unsigned)passes), dim3(threads), lds, st, A, c,
                       y);
    return hipGetLastError();
}

template <class T, int NV, int Q, int KT>
hipError_t ab2_launch_k(const Ab2Args<T>& A, const T* c, T* y, int threads, size_t lds, int64_t passes,
                        hipStream_t st) {
    const bool win = A.win < A.nb;
    auto kern = win ? k_ab2<T, NV, Q, KT, true> : k_ab2<T, NV, Q, KT, false>;
    static const hipError_t attr_w = max_lds_per_block() > 65536
                                         ? hipFuncSetAttribute((const void*)k_ab2<T, NV, Q, KT, true>,
                                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                                               max_lds_per_block())
                                         : hipSuccess;
    static const hipError_t attr_f = max_lds_per_block() > 65536
                                         ? hipFuncSetAttribute((const void*)k_ab2<T, NV, Q, KT, false>,
                                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                                               max_lds_per_block())
                                         : hipSuccess;
    const hipError_t attr = win ? attr_w : attr_f;
    if (lds > 65536 && attr != hipSuccess) return attr;
    hipLaunchKernelGGL(kern, dim3((unsigned)A.na, (unsigned)passes), dim3(threads), lds, st, A, c, y);
    return hipGetLastError();
}

// KT: staged rows per group as a compile-time count (1, 2 or 4; A.krows is set to it)
template <class T, int NV, int Q>
hipError_t ab2_launch(Ab2Args<T> A, const T* c, T* y, int threads, size_t slice_bytes, size_t row_bytes,
                      int64_t passes, hipStream_t st) {
    const int KT = A.krows >= 4 ? 4 : (A.krows >= 2 ? 2 : 1);
    A.krows = KT;
    const size_t lds = (size_t)KT * (slice_bytes + row_bytes);
    if (KT == 4) return ab2_launch_k<T, NV, Q, 4>(A, c, y, threads, lds, passes, st);
    if (KT == 2) return ab2_launch_k<T, NV, Q, 2>(A, c, y, threads, lds, passes, st);
    return ab2_launch_k<T, NV, Q, 1>(A, c, y, threads, lds, passes, st);
}

// Largest columns-per-thread of the alpha-beta kernel that keeps the
// accumulators and entry bounds within 64 VGPRs (1024-thread workgroups allow 128).
template <class T, int NV>
constexpr int ab_qmax() {
    constexpr int per_q = NV * (int)sizeof(T) / 4 + 2;
    constexpr int q = 40 / per_q;
    return q >= 12 ? 12 : (q >= 10 ? 10 : (q >= 8 ? 8 : (q >= 6 ? 6 : (q >= 4 ? 4 : (q >= 2 ? 2 : 1)))));
}

template <class T, int NV>
hipError_t alpha_beta(AbArgs<T> A, const T* c, T* y, const SigmaTune& tune, const uint32_t* sell32,
                      hipStream_t st) {
    if (A.na > 0x7fffffffLL) return hipErrorInvalidValue;
    const int threads = ab_block_threads(A.nb);
    constexpr int QM = ab_qmax<T, NV>();
    // column passes (each restages the ket rows), columns spread evenly over them
    const int64_t passes = (A.nb + (int64_t)threads * QM - 1) / ((int64_t)threads * QM);
    const int64_t per = (A.nb + passes * threads - 1) / (passes * threads);  // columns per thread
    constexpr int steps[7] = {1, 2, 4, 6, 8, 10, 12};
    int Q = 1;
    for (int s : steps)
        if (s <= QM) {
            Q = s;
            if (s >= per) break;
        }
    // the compact walk stages one more slice element (a zero read by padding entries)
    const size_t slice_bytes = (size_t)((A.norb * A.norb + (sell32 ? 1 : 0) + 3) & ~3) * sizeof(T);
    size_t budget = (size_t)tune.ab_lds_bytes;
    const size_t hw = (size_t)max_lds_per_block();
    if (budget > hw) budget = hw;
    const size_t row_bytes = (size_t)A.nb * NV * sizeof(T);
    int64_t K = (int64_t)(budget / (slice_bytes + row_bytes));
    if (K > 8) K = 8;
    if (K >= 1) {
        A.krows = (int)K;  // whole ket rows, K at a time
        A.win = A.nb;
    } else {
        A.krows = 1;       // one ket row, staged in windows
        if (budget < slice_bytes + 64 * NV * sizeof(T)) budget = slice_bytes + 64 * NV * sizeof(T);
        int64_t win = (int64_t)((budget - slice_bytes) / (NV * sizeof(T)));
        A.win = win > A.nb ? A.nb : win;
    }
    const size_t lds = (size_t)A.krows * (slice_bytes + (size_t)A.win * NV * sizeof(T));
    if (sell32) {
        Ab2Args<T> B{};
        B.na = A.na; B.nb = A.nb; B.norb = A.norb; B.win = A.win; B.krows = A.krows;
        B.a1p = A.a1p; B.a1pack = A.a1pack; B.sell = sell32; B.sell_off = A.b1sell_off; B.pos = A.b1pos;
        B.eri = A.eri;
        const size_t rb = (size_t)A.win * NV * sizeof(T);
        switch (Q) {
            case 1: return ab2_launch<T, NV, 1>(B, c, y, threads, slice_bytes, rb, passes, st);
            case 2: return ab2_launch<T, NV, (QM < 2 ? QM : 2)>(B, c, y, threads, slice_bytes, rb, passes, st);
            case 4: return ab2_launch<T, NV, (QM < 4 ? QM : 4)>(B, c, y, threads, slice_bytes, rb, passes, st);
            case 6: return ab2_launch<T, NV, (QM < 6 ? QM : 6)>(B, c, y, threads, slice_bytes, rb, passes, st);
            case 8: return ab2_launch<T, NV, (QM < 8 ? QM : 8)>(B, c, y, threads, slice_bytes, rb, passes, st);
            case 10: return ab2_launch<T, NV, (QM < 10 ? QM : 10)>(B, c, y, threads, slice_bytes, rb, passes, st);
            default: return ab2_launch<T, NV, QM>(B, c, y, threads, slice_bytes, rb, passes, st);
        }
    }
    switch (Q) {
        case 1: return ab_launch<T, NV, 1>(A, c, y, threads, lds, passes, st);
        case 2: return ab_launch<T, NV, (QM < 2 ? QM : 2)>(A, c, y, threads, lds, passes, st);
        case 4: return ab_launch<T, NV, (QM < 4 ? QM : 4)>(A, c, y, threads, lds, passes, st);
        case 6: return ab_launch<T, NV, (QM < 6 ? QM : 6)>(A, c, y, threads, lds, passes, st);
        case 8: return ab_launch<T, NV, (QM < 8 ? QM : 8)>(A, c, y, threads, lds, passes, st);
        case 10: return ab_launch<T, NV, (QM < 10 ? QM : 10)>(A, c, y, threads, lds, passes, st);
        default: return ab_launch<T, NV, QM>(A, c, y, threads, lds, passes, st);
    }
}

// Optional per-stage timing: events[0..5] recorded around the five launches.
template <class T, int NV>
hipError_t sigma_nv(const SigmaArgs<T>& A, const T* c, T* y, T* cT, T* yT, const SigmaTune& tune,
                    hipStream_t st, hipEvent_t* ev) {
    const int64_t na = A.na, nb = A.nb;
    auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], st) : hipSuccess; };
    hipError_t e = mark(0);
    if (e == hipSuccess) e = transpose<T, NV, false>(c, cT, na, nb, st);
    if (e == hipSuccess) e = mark(1);
    if (e != hipSuccess) return e;
    StreamArgs<T> Sa{};
    Sa.nrow = na; Sa.ncol = nb;
    Sa.p1 = A.a1p; Sa.J1 = A.a1J; Sa.c1 = A.a1c; Sa.ps1 = A.a1ps;
    Sa.p2 = A.a2p; Sa.J2 = A.a2J; Sa.c2 = A.a2c;
    Sa.G = A.Gb; Sa.diag = A.diag; Sa.shift = A.shift;
    e = stream<T, NV>(Sa, c, y, tune, st);
    if (e == hipSuccess) e = mark(2);
    if (e != hipSuccess) return e;
    StreamArgs<T> Sb{};
    Sb.nrow = nb; Sb.ncol = na;
    Sb.p1 = A.b1p; Sb.J1 = A.b1J; Sb.c1 = A.b1c; Sb.ps1 = A.b1ps;
    Sb.p2 = A.b2p; Sb.J2 = A.b2J; Sb.c2 = A.b2c;
    Sb.G = A.Ga; Sb.diag = nullptr; Sb.shift = 0.0;
    e = stream<T, NV>(Sb, cT, yT, tune, st);
    if (e == hipSuccess) e = mark(3);
    if (e != hipSuccess) return e;
    AbArgs<T> B{};
    B.na = na; B.nb = nb; B.norb = A.norb;
    B.a1p = A.a1p; B.a1pack = A.a1pack; B.b1sell = A.b1sell; B.b1sell_off = A.b1sell_off;
    B.b1pos = A.b1sell_pos;
    B.eri = A.eri;
    e = alpha_beta<T, NV>(B, c, y, tune, tune.ab_compact ? A.b1sell32 : nullptr, st);
    if (e == hipSuccess) e = mark(4);
    if (e != hipSuccess) return e;
    e = transpose<T, NV, true>(yT, y, nb, na, st);
    if (e == hipSuccess) e = mark(5);
    return e;
}

}  // namespace

size_t sigma_workspace_bytes(int64_t N, int nvec, int layout, size_t elem) {
    const int nv = layout == 0 ? 1 : nvec;
    return 2 * (size_t)N * nv * elem;
}

template <class T>
hipError_t launch_sigma(const SigmaArgs<T>& A, int nvec, const T* c, T* y, int layout, void* ws,
                        const SigmaTune& tune, hipStream_t st, hipEvent_t* ev) {
    if (A.na == 0 || A.nb == 0) return hipSuccess;
    const int64_t N = A.na * A.nb;
    const int nv = layout == 0 ? 1 : nvec;
    T* cT = static_cast<T*>(ws);
    T* yT = cT + (size_t)N * nv;
    if (layout == 0) {
        for (int v = 0; v < nvec; ++v) {
            hipError_t e = sigma_nv<T, 1>(A, c + v * N, y + v * N, cT, yT, tune, st, v == 0 ? ev : nullptr);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    switch (nvec) {
        case 1: return sigma_nv<T, 1>(A, c, y, cT, yT, tune, st, ev);
        case 2: return sigma_nv<T, 2>(A, c, y, cT, yT, tune, st, ev);
        case 4: return sigma_nv<T, 4>(A, c, y, cT, yT, tune, st, ev);
        case 8: return sigma_nv<T, 8>(A, c, y, cT, yT, tune, st, ev);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_sigma<double>(const SigmaArgs<double>&, int, const double*, double*,
                                         int, void*, const SigmaTune&, hipStream_t, hipEvent_t*);
template hipError_t launch_sigma<float>(const SigmaArgs<float>&, int, const float*, float*, int,
                                        void*, const SigmaTune&, hipStream_t, hipEvent_t*);

}  // namespace sbd
