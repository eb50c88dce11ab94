// Full-bitstring determinant lists (Sec. II-F, Sec. III-F) on gfx950.
//
// A determinant is one packed spin-orbital string over 2 x 64 bits: alpha
// orbital p is bit p of word 0, beta orbital p bit p of word 1.  Phases count
// the occupied spin-orbitals below the one acted on, so alpha creators come
// before beta creators (the same convention as the alpha x beta path).  The
// list is any set of determinants, not a Cartesian product; it is kept sorted
// by (alpha word, beta word) ascending, so determinants sharing an alpha string
// form a contiguous group sorted by beta string.
//
// Connections (the Slater-Condon neighbourhood of Eq. 4: the determinants that
// differ by one or two electrons) are found group-wise: the alpha strings of
// the groups are compared all-pairs (popcount of the XOR <= 4, itself
// included), and a determinant then visits only the groups whose alpha string is
// that close, testing popcount(alpha XOR) + popcount(beta XOR) in {2, 4}: a
// group two alpha electrons away by a binary search for the same beta string,
// the others by a scan.  Rows come out sorted by ket index because groups and
// their members are visited in ascending order and hits are placed in order.
//
// sigma is matrix-free: each connection's matrix element is formed from the two
// bitstrings alone (bit scans for the moved orbitals, popcounts of masked words
// for the phase, integrals by index), as the excitation generator of the
// full-bitstring representation prescribes, and accumulated per bra row by a
// fixed group of lanes in a fixed order (bitwise reproducible, no atomics).
// Same-spin doubles read one antisymmetrised integral from a pair table.
#include "internal.h"

namespace sbd {

namespace {

constexpr int kTile = 1024;

struct Det {
    uint64_t a, b;  // alpha word, beta word
};

__device__ __forceinline__ bool det_gt(const Det& x, const Det& y) {
    return x.a > y.a || (x.a == y.a && x.b > y.b);
}
__device__ __forceinline__ bool det_ne(const Det& x, const Det& y) { return x.a != y.a || x.b != y.b; }
__device__ __forceinline__ uint64_t below(int p) { return (1ull << p) - 1ull; }

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// ------------------------------------------------------------------ sort
__global__ void k_det_pad(Det* a, int64_t n, int64_t P) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + n;
    if (i < P) a[i] = Det{~0ull, ~0ull};
}

__global__ void k_det_bitonic_global(Det* a, int64_t P, int64_t k, int64_t j) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const int64_t l = i ^ j;
    if (l <= i) return;
    const bool up = (i & k) == 0;
    const Det x = a[i], y = a[l];
    if (det_gt(x, y) == up) {
        a[i] = y;
        a[l] = x;
    }
}

// stages j = jstart, ..., 1 of merge size k inside tiles of T elements
__global__ void __launch_bounds__(kTile) k_det_bitonic_local(Det* a, int64_t k, int64_t jstart, int T) {
    __shared__ Det s[kTile];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * T;
    s[t] = a[base + t];
    for (int64_t j = jstart; j > 0; j >>= 1) {
        __syncthreads();
        const int l = t ^ (int)j;
        if (l > t) {
            const bool up = ((base + t) & k) == 0;
            const Det x = s[t], y = s[l];
            if (det_gt(x, y) == up) {
                s[t] = y;
                s[l] = x;
            }
        }
    }
    __syncthreads();
    a[base + t] = s[t];
}

// unique compaction of the sorted list (first n entries real): flags of the
// first entry of each run of equal determinants, then a scatter to the scanned
// positions; the count is pos[n]
__global__ void k_det_flags(const Det* a, int64_t n, int64_t* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = (i == 0 || det_ne(a[i], a[i - 1])) ? 1 : 0;
}

__global__ void k_det_scatter(const Det* a, int64_t n, const int64_t* pos, Det* out, int64_t* count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && pos[i + 1] != pos[i]) out[pos[i]] = a[i];
    if (i == 0) *count = pos[n];
}

// ------------------------------------------------------------------ alpha groups
__global__ void k_group_flags(const Det* d, int64_t n, int64_t* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = (i == 0 || d[i].a != d[i - 1].a) ? 1 : 0;
}

// gpos[i + 1] = number of group starts in [0, i]
__global__ void k_group_fill(const Det* d, int64_t n, const int64_t* gpos, uint64_t* ua, int64_t* goff,
                             int32_t* grp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t g = gpos[i + 1] - 1;
    grp[i] = (int32_t)g;
    if (i == 0 || d[i].a != d[i - 1].a) {
        ua[g] = d[i].a;
        goff[g] = i;
    }
    if (i == n - 1) goff[g + 1] = n;
}

constexpr int kWaves = 8;      // rows per workgroup
constexpr int kChunk = 2048;   // strings staged in LDS per pass

__device__ __forceinline__ int wave_sum(int v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Alpha strings of the groups within two electrons of each group's (itself
// included): count pass (FILL = false) and fill pass with the alpha degree
// (electrons moved, 0..2) of each neighbour group.
template <bool FILL>
__global__ void __launch_bounds__(kWaves * 64) k_group_nbr(const uint64_t* __restrict__ ua, int64_t ng,
                                                           int64_t* cnt, const int64_t* __restrict__ rp,
                                                           int32_t* gj, int8_t* gd) {
    __shared__ uint64_t chunk[kChunk];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * kWaves + w;
    const uint64_t u = (g < ng) ? ua[g] : 0ull;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t o = (FILL && g < ng) ? rp[g] : 0;
    int c = 0;
    for (int64_t base = 0; base < ng; base += kChunk) {
        const int len = (int)((ng - base) < kChunk ? (ng - base) : kChunk);
        __syncthreads();
        for (int t = threadIdx.x; t < len; t += blockDim.x) chunk[t] = ua[base + t];
        __syncthreads();
        if (g >= ng) continue;
        for (int t0 = 0; t0 < len; t0 += 64) {
            const int t = t0 + lane;
            const uint64_t v = (t < len) ? chunk[t] : u;
            const int pc = __popcll(u ^ v);
            const bool hit = (t < len) && pc <= 4;
            if (FILL) {
                const uint64_t m = __ballot(hit);
                if (hit) {
                    const int64_t e = o + __popcll(m & lt);
                    gj[e] = (int32_t)(base + t);
                    gd[e] = (int8_t)(pc >> 1);
                }
                o += __popcll(m);
            } else {
                c += hit;
            }
        }
    }
    if (!FILL) {
        c = wave_sum(c);
        if (g < ng && lane == 0) cnt[g] = c;
    }
}

// beta words of the sorted list, contiguous (the connection passes read only these)
__global__ void k_det_beta(const Det* __restrict__ d, int64_t n, uint64_t* __restrict__ bw) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bw[i] = d[i].b;
}

// Connections of each determinant: count pass and fill pass (ket index and
// electrons moved, 1 or 2), rows sorted by ket.  The neighbour groups are taken
// 64 at a time, in ascending order.  A group whose alpha string is two electrons
// away can hold only one connection, the determinant with the same beta string:
// each lane finds it for one such group by binary search (the group is sorted
// by beta string).  The other groups (alpha string equal or one electron away)
// are scanned by the whole wavefront, one group after another, so hits are
// placed in ascending ket order by a wave ballot.
template <bool FILL>
__global__ void __launch_bounds__(kWaves * 64) k_conn(const uint64_t* __restrict__ bw, int64_t n,
                                                      const int32_t* __restrict__ grp,
                                                      const int64_t* __restrict__ goff,
                                                      const int64_t* __restrict__ gn_rp,
                                                      const int32_t* __restrict__ gn_j,
                                                      const int8_t* __restrict__ gn_d, int64_t* cnt,
                                                      const int64_t* __restrict__ rp, int32_t* J, int8_t* deg) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t I = (int64_t)blockIdx.x * kWaves + w;
    if (I >= n) return;  // wave-uniform
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t ib = bw[I];
    const int g = grp[I];
    int64_t o = FILL ? rp[I] : 0;
    int c = 0;
    const int64_t e0 = gn_rp[g], e1 = gn_rp[g + 1];
    for (int64_t eb = e0; eb < e1; eb += 64) {
        const int64_t e = eb + lane;
        const bool dbl = e < e1 && gn_d[e] == 2;
        int hitK = -1;
        if (dbl) {
            const int h = gn_j[e];
            const int64_t end = goff[h + 1];
            int64_t lo = goff[h], hi = end;  // first member with beta string >= ib
            while (lo < hi) {
                const int64_t mid = lo + ((hi - lo) >> 1);
                if (bw[mid] < ib) lo = mid + 1;
                else hi = mid;
            }
            if (lo < end && bw[lo] == ib) hitK = (int)lo;
        }
        if (!FILL) c += hitK >= 0;
        const uint64_t dmask = __ballot(dbl), hmask = __ballot(hitK >= 0);
        const int m = (int)((e1 - eb) < 64 ? (e1 - eb) : 64);
        for (int t = 0; t < m; ++t) {  // wave-uniform
            if ((dmask >> t) & 1) {
                if (FILL && ((hmask >> t) & 1)) {
                    const int K = __shfl(hitK, t, 64);
                    if (lane == 0) {
                        J[o] = (int32_t)K;
                        deg[o] = 2;
                    }
                    ++o;
                }
                continue;
            }
            const int h = gn_j[eb + t];
            const int pa = 2 * (int)gn_d[eb + t];
            const int64_t k0 = goff[h], k1 = goff[h + 1];
            for (int64_t t0 = k0; t0 < k1; t0 += 64) {
                const int64_t K = t0 + lane;
                const bool ok = K < k1;
                const int tot = pa + (ok ? __popcll(ib ^ bw[K]) : 0);
                const bool hit = ok && (tot == 2 || tot == 4);
                if (FILL) {
                    const uint64_t hm = __ballot(hit);
                    if (hit) {
                        const int64_t q = o + __popcll(hm & lt);
                        J[q] = (int32_t)K;
                        deg[q] = (int8_t)(tot >> 1);
                    }
                    o += __popcll(hm);
                } else {
                    c += hit;
                }
            }
        }
    }
    if (!FILL) {
        c = wave_sum(c);
        if (lane == 0) cnt[I] = c;
    }
}

// ------------------------------------------------------------------ Hamiltonian
// Index of the orbital pair p < q among the n(n-1)/2 pairs.
__device__ __forceinline__ int pair_index(int p, int q) { return q * (q - 1) / 2 + p; }

// Tables of the single-excitation spectator terms: jt[(a n + i) n + k] = (ai|kk),
// kt[(a n + i) n + k] = (ak|ki); jd[p n + q] = (pp|qq), kd[p n + q] = (pq|qp);
// and the antisymmetrised same-spin double elements
// dd[P(a,b) npair + P(i,j)] = (ai|bj) - (aj|bi) for a < b, i < j.
__global__ void k_full_tables(const double* __restrict__ eri, int n, double* jt, double* kt, double* jd,
                              double* kd, double* dd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n3 = (int64_t)n * n * n;
    const int64_t np = (int64_t)n * (n - 1) / 2;
    if (t < np * np) {
        // invert the pair index: q is the largest with q(q-1)/2 <= P
        const int P = (int)(t / np), Q = (int)(t % np);
        int b = 1, j = 1;
        while ((b + 1) * b / 2 <= P) ++b;
        while ((j + 1) * j / 2 <= Q) ++j;
        const int a = P - b * (b - 1) / 2, i = Q - j * (j - 1) / 2;
        const int64_t nn = n;
        dd[t] = eri[((a * nn + i) * nn + b) * nn + j] - eri[((a * nn + j) * nn + b) * nn + i];
    }
    if (t < n3) {
        const int k = (int)(t % n), i = (int)((t / n) % n), a = (int)(t / ((int64_t)n * n));
        const int64_t nn = n;
        jt[t] = eri[((a * nn + i) * nn + k) * nn + k];
        kt[t] = eri[((a * nn + k) * nn + k) * nn + i];
    }
    if (t < (int64_t)n * n) {
        const int q = (int)(t % n), p = (int)(t / n);
        const int64_t nn = n;
        jd[t] = eri[((p * nn + p) * nn + q) * nn + q];
        kd[t] = eri[((p * nn + q) * nn + q) * nn + p];
    }
}

// H_II = E_core + sum_{p in I} h_pp + sum over occupied pairs of the same spin
// [(pp|qq) - (pq|qp)] + sum over an alpha and a beta orbital (pp|qq).
__global__ void k_full_diag(const Det* __restrict__ d, int64_t nd, int n, const double* __restrict__ h,
                            const double* __restrict__ jd, const double* __restrict__ kd, double e_core,
                            double* out) {
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nd) return;
    const uint64_t w[2] = {d[I].a, d[I].b};
    double v = e_core;
    for (int s = 0; s < 2; ++s)
        for (uint64_t m = w[s]; m; m &= m - 1) {
            const int p = __builtin_ctzll(m);
            v += h[p * n + p];
            for (uint64_t r = m & (m - 1); r; r &= r - 1) {  // q > p of the same spin
                const int q = __builtin_ctzll(r);
                v += jd[p * n + q] - kd[p * n + q];
            }
        }
    for (uint64_t m = w[0]; m; m &= m - 1) {
        const int p = __builtin_ctzll(m);
        for (uint64_t r = w[1]; r; r &= r - 1) v += jd[p * n + __builtin_ctzll(r)];
    }
    out[I] = v;
}

struct FullArgs {
    int64_t n;
    int norb;
    const Det* d;
    const int64_t* rp;
    const int32_t* J;
    const double* h;    // norb x norb
    const double* eri;  // norb^4
    const double* jt;   // norb^3: (ai|kk)
    const double* kt;   // norb^3: (ak|ki)
    const double* dd;   // npair^2: (ai|bj) - (aj|bi), a < b, i < j
    int npair;          // norb (norb - 1) / 2
    const double* diag;
    double shift;
    const void* vals;   // assembled elements per connection (T), or null
};

// Phase of a+_a a_i |w> (i in w, a not): the occupied orbitals strictly between.
__device__ __forceinline__ int single_parity(uint64_t w, int i, int a) {
    return __popcll(w & below(i)) + __popcll((w ^ (1ull << i)) & below(a));
}

// <bra|H|ket> for bra != ket connected (one or two electrons moved), FP64.
__device__ double full_element(const Det& bra, const Det& ket, const FullArgs& A) {
    const int n = A.norb;
    const int64_t nn = n;
    const uint64_t da = bra.a ^ ket.a, db = bra.b ^ ket.b;
    const int pa = __popcll(da), pb = __popcll(db);
    if (pa + pb == 2) {  // single i -> a in one spin; spectators of both spins
        const bool al = pa == 2;
        const uint64_t wk = al ? ket.a : ket.b, wb = al ? bra.a : bra.b, other = al ? ket.b : ket.a;
        const int i = __builtin_ctzll(wk & ~wb), a = __builtin_ctzll(wb & ~wk);
        const double* jr = A.jt + (a * nn + i) * nn;
        const double* kr = A.kt + (a * nn + i) * nn;
        double v = A.h[a * n + i];
        for (uint64_t m = wk; m; m &= m - 1) {
            const int k = __builtin_ctzll(m);
            v += jr[k] - kr[k];
        }
        for (uint64_t m = other; m; m &= m - 1) v += jr[__builtin_ctzll(m)];
        return (single_parity(wk, i, a) & 1) ? -v : v;
    }
    if (pa == 4 || pb == 4) {  // double within one spin: a+_a a+_b a_j a_i, i < j, a < b
        const uint64_t wk = pa == 4 ? ket.a : ket.b, wb = pa == 4 ? bra.a : bra.b;
        const uint64_t x = wk & ~wb, y = wb & ~wk;
        const int i = __builtin_ctzll(x), j = __builtin_ctzll(x & (x - 1));
        const int a = __builtin_ctzll(y), b = __builtin_ctzll(y & (y - 1));
        const uint64_t k1 = wk ^ (1ull << i), k2 = k1 ^ (1ull << j), k3 = k2 | (1ull << b);
        const int par = __popcll(wk & below(i)) + __popcll(k1 & below(j)) + __popcll(k2 & below(b)) +
                        __popcll(k3 & below(a));
        const double v = A.dd[(int64_t)pair_index(a, b) * A.npair + pair_index(i, j)];
        return (par & 1) ? -v : v;
    }
    // one alpha and one beta electron: alpha i -> a, beta j -> b, element (ai|bj)
    const int i = __builtin_ctzll(ket.a & ~bra.a), a = __builtin_ctzll(bra.a & ~ket.a);
    const int j = __builtin_ctzll(ket.b & ~bra.b), b = __builtin_ctzll(bra.b & ~ket.b);
    const int par = single_parity(ket.a, i, a) + single_parity(ket.b, j, b);
    const double v = A.eri[((a * nn + i) * nn + b) * nn + j];
    return (par & 1) ? -v : v;
}

// y[I] = (H_II - shift) x[I] + sum_J H_IJ x[J]: G lanes per bra row (64 / G
// rows per wavefront), the lanes over the row's connections, NV interleaved
// vectors per determinant.  Each element is formed once in FP64 and, for FP32
// vectors, rounded once (ASM: read from the assembled values, which hold
// exactly those numbers); partial sums are combined by a fixed butterfly
// within the row's lanes.
template <class T, int NV, bool ASM, int G>
__global__ void __launch_bounds__(256) k_full_sigma(FullArgs A, const T* __restrict__ x, T* __restrict__ y) {
    const int lane = threadIdx.x & 63, sub = lane & (G - 1);
    const int64_t I = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 / G) + lane / G;
    // a whole row group leaves together, so the butterfly below (lane offsets
    // below G) only reads lanes of the same row
    if (I >= A.n) return;
    const Det bra = A.d[I];
    T acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = T(0);
    const int64_t e1 = A.rp[I + 1];
    for (int64_t e = A.rp[I] + sub; e < e1; e += G) {
        const int64_t J = A.J[e];
        const T hv = ASM ? static_cast<const T*>(A.vals)[e] : (T)full_element(bra, A.d[J], A);
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += hv * x[J * NV + v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
        for (int off = G / 2; off > 0; off >>= 1) acc[v] += __shfl_xor(acc[v], off, 64);
    if (sub == 0) {
        const T dg = (T)(A.diag[I] - A.shift);
#pragma unroll
        for (int v = 0; v < NV; ++v) y[I * NV + v] = dg * x[I * NV + v] + acc[v];
    }
}

// The element of every stored connection, in the connection order: one
// wavefront per bra row, its lanes over the row's connections (the matrix-free
// product's evaluation, kept instead of summed).
template <class T>
__global__ void __launch_bounds__(256) k_full_values(FullArgs A, T* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t I = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (I >= A.n) return;  // wave-uniform
    const Det bra = A.d[I];
    const int64_t e1 = A.rp[I + 1];
    for (int64_t e = A.rp[I] + lane; e < e1; e += 64) out[e] = (T)full_element(bra, A.d[A.J[e]], A);
}

// x_to[v][i] = x_from[v][j] where from[j] == to[i] (binary search in the sorted
// from-list), else 0: one thread per determinant of the new list.
__global__ void k_full_map(const Det* __restrict__ from, int64_t nf, const Det* __restrict__ to, int64_t nt,
                           int nvec, const double* __restrict__ xf, double* __restrict__ xt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    const Det d = to[i];
    int64_t lo = 0, hi = nf;  // first index with from[j] >= d
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (det_gt(d, from[mid])) lo = mid + 1;
        else hi = mid;
    }
    const bool hit = lo < nf && !det_ne(from[lo], d);
    for (int v = 0; v < nvec; ++v) xt[(size_t)v * nt + i] = hit ? xf[(size_t)v * nf + lo] : 0.0;
}

// Spin-orbital occupations of a vector over the list (input of the sample
// recovery of an SQD iteration): part[j * nq + q] = sum over the determinants
// of chunk q of c_I^2 [orbital j of spin j / norb occupied] (j < 2 norb), or
// of c_I^2 (j = 2 norb); then per j the chunk sums in order.
constexpr int kOccChunk = 8192;

__device__ double occ_block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    return sh[0];
}

__global__ void __launch_bounds__(256) k_full_occ_part(const Det* __restrict__ d, const double* __restrict__ c,
                                                       int64_t n, int norb, int64_t nq, double* __restrict__ part) {
    __shared__ double sh[256];
    const int64_t q = blockIdx.x;
    const int j = blockIdx.y;
    const int64_t i0 = q * kOccChunk, i1 = i0 + kOccChunk < n ? i0 + kOccChunk : n;
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const double w = c[i] * c[i];
        if (j == 2 * norb) {
            s += w;
        } else {
            const uint64_t word = j < norb ? d[i].a : d[i].b;
            if ((word >> (j % norb)) & 1ull) s += w;
        }
    }
    s = occ_block_sum(s, sh);
    if (threadIdx.x == 0) part[(int64_t)j * nq + q] = s;
}

__global__ void __launch_bounds__(256) k_full_occ_sum(const double* __restrict__ part, int64_t nq, int norb,
                                                      double* __restrict__ occ) {
    __shared__ double sh[256];
    const int j = blockIdx.x;
    double s = 0.0, t = 0.0;
    for (int64_t q = threadIdx.x; q < nq; q += 256) {
        s += part[(int64_t)j * nq + q];
        t += part[(int64_t)2 * norb * nq + q];
    }
    s = occ_block_sum(s, sh);
    __syncthreads();
    t = occ_block_sum(t, sh);
    if (threadIdx.x == 0) occ[j] = t > 0.0 ? s / t : 0.0;
}

}  // namespace

// ------------------------------------------------------------------ launchers
int64_t full_occupation_scratch_words(int64_t n, int norb) {
    const int64_t nq = (n + kOccChunk - 1) / kOccChunk;
    return (2 * (int64_t)norb + 1) * nq;
}

hipError_t launch_full_occupations(const void* dets, const double* c, int64_t n, int norb, double* scratch,
                                   double* occ, hipStream_t st) {
    const int64_t nq = (n + kOccChunk - 1) / kOccChunk;
    hipLaunchKernelGGL(k_full_occ_part, dim3((unsigned)nq, (unsigned)(2 * norb + 1)), dim3(256), 0, st,
                       static_cast<const Det*>(dets), c, n, norb, nq, scratch);
    hipLaunchKernelGGL(k_full_occ_sum, dim3((unsigned)(2 * norb)), dim3(256), 0, st, scratch, nq, norb, occ);
    return hipGetLastError();
}
hipError_t launch_full_map(const void* from, int64_t nf, const void* to, int64_t nt, int nvec, const double* xf,
                           double* xt, hipStream_t st) {
    if (nt > 0)
        hipLaunchKernelGGL(k_full_map, dim3(blocks_for(nt, 256)), dim3(256), 0, st, static_cast<const Det*>(from),
                           nf, static_cast<const Det*>(to), nt, nvec, xf, xt);
    return hipGetLastError();
}
hipError_t launch_full_sort_unique(void* work, int64_t n, void* out, int64_t* d_count, int64_t* scratch,
                                   hipStream_t st) {
    Det* a = static_cast<Det*>(work);
    int64_t P = 1;
    while (P < n) P <<= 1;
    if (P > n) hipLaunchKernelGGL(k_det_pad, dim3(blocks_for(P - n, 256)), dim3(256), 0, st, a, n, P);
    const int T = (int)(P < kTile ? P : kTile);
    const unsigned tiles = (unsigned)(P / T);
    for (int64_t k = 2; k <= P; k <<= 1) {
        int64_t j = k >> 1;
        for (; j >= T; j >>= 1)
            hipLaunchKernelGGL(k_det_bitonic_global, dim3(blocks_for(P, 256)), dim3(256), 0, st, a, P, k, j);
        hipLaunchKernelGGL(k_det_bitonic_local, dim3(tiles), dim3(T), 0, st, a, k, j, T);
    }
    int64_t *flag = scratch, *pos = scratch + n, *tmp = scratch + 2 * n + 1;
    hipLaunchKernelGGL(k_det_flags, dim3(blocks_for(n, 256)), dim3(256), 0, st, a, n, flag);
    hipError_t e = launch_exclusive_scan(flag, n, pos, tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_det_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, st, a, n, pos,
                       static_cast<Det*>(out), d_count);
    return hipGetLastError();
}

hipError_t launch_full_group_flags(const void* dets, int64_t n, int64_t* flag, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_group_flags, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                           static_cast<const Det*>(dets), n, flag);
    return hipGetLastError();
}

hipError_t launch_full_group_fill(const void* dets, int64_t n, const int64_t* gpos, uint64_t* ua, int64_t* goff,
                                  int32_t* grp, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_group_fill, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                           static_cast<const Det*>(dets), n, gpos, ua, goff, grp);
    return hipGetLastError();
}

hipError_t launch_full_group_nbr(const uint64_t* ua, int64_t ng, int64_t* cnt, const int64_t* rp, int32_t* gj,
                                 int8_t* gd, hipStream_t st) {
    if (ng <= 0) return hipGetLastError();
    if (rp)
        hipLaunchKernelGGL(k_group_nbr<true>, dim3(blocks_for(ng, kWaves)), dim3(kWaves * 64), 0, st, ua, ng,
                           cnt, rp, gj, gd);
    else
        hipLaunchKernelGGL(k_group_nbr<false>, dim3(blocks_for(ng, kWaves)), dim3(kWaves * 64), 0, st, ua, ng,
                           cnt, rp, gj, gd);
    return hipGetLastError();
}

hipError_t launch_full_beta(const void* dets, int64_t n, uint64_t* bw, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_det_beta, dim3(blocks_for(n, 256)), dim3(256), 0, st, static_cast<const Det*>(dets), n,
                           bw);
    return hipGetLastError();
}

hipError_t launch_full_conn(const uint64_t* bw, int64_t n, const int32_t* grp, const int64_t* goff,
                            const int64_t* gn_rp, const int32_t* gn_j, const int8_t* gn_d, int64_t* cnt,
                            const int64_t* rp, int32_t* J, int8_t* deg, hipStream_t st) {
    if (n <= 0) return hipGetLastError();
    if (rp)
        hipLaunchKernelGGL(k_conn<true>, dim3(blocks_for(n, kWaves)), dim3(kWaves * 64), 0, st, bw, n, grp, goff,
                           gn_rp, gn_j, gn_d, cnt, rp, J, deg);
    else
        hipLaunchKernelGGL(k_conn<false>, dim3(blocks_for(n, kWaves)), dim3(kWaves * 64), 0, st, bw, n, grp, goff,
                           gn_rp, gn_j, gn_d, cnt, rp, J, deg);
    return hipGetLastError();
}

hipError_t launch_full_tables(const double* eri, int n, double* jt, double* kt, double* jd, double* kd,
                              double* dd, hipStream_t st) {
    const int64_t n3 = (int64_t)n * n * n, np = (int64_t)n * (n - 1) / 2;
    const int64_t m = n3 > np * np ? n3 : np * np;
    hipLaunchKernelGGL(k_full_tables, dim3(blocks_for(m, 256)), dim3(256), 0, st, eri, n, jt, kt, jd, kd, dd);
    return hipGetLastError();
}

hipError_t launch_full_diag(const void* dets, int64_t nd, int n, const double* h, const double* jd,
                            const double* kd, double e_core, double* out, hipStream_t st) {
    if (nd > 0)
        hipLaunchKernelGGL(k_full_diag, dim3(blocks_for(nd, 256)), dim3(256), 0, st,
                           static_cast<const Det*>(dets), nd, n, h, jd, kd, e_core, out);
    return hipGetLastError();
}

namespace {

FullArgs full_args(const FullSigmaArgs& S) {
    FullArgs A{};
    A.n = S.n;
    A.norb = S.norb;
    A.d = static_cast<const Det*>(S.dets);
    A.rp = S.rp;
    A.J = S.J;
    A.h = S.h;
    A.eri = S.eri;
    A.jt = S.jt;
    A.kt = S.kt;
    A.dd = S.dd;
    A.npair = S.norb * (S.norb - 1) / 2;
    A.diag = S.diag;
    A.shift = S.shift;
    return A;
}

template <class T, bool ASM, int G>
hipError_t full_sigma_layouts(const FullArgs& A, int nvec, const T* x, T* y, int layout, hipStream_t st) {
    const dim3 grid(blocks_for(A.n, 4 * (64 / G))), block(256);
    if (layout == 0) {
        for (int v = 0; v < nvec; ++v)
            hipLaunchKernelGGL((k_full_sigma<T, 1, ASM, G>), grid, block, 0, st, A, x + (size_t)v * A.n,
                               y + (size_t)v * A.n);
        return hipGetLastError();
    }
    switch (nvec) {
        case 1: hipLaunchKernelGGL((k_full_sigma<T, 1, ASM, G>), grid, block, 0, st, A, x, y); break;
        case 2: hipLaunchKernelGGL((k_full_sigma<T, 2, ASM, G>), grid, block, 0, st, A, x, y); break;
        case 4: hipLaunchKernelGGL((k_full_sigma<T, 4, ASM, G>), grid, block, 0, st, A, x, y); break;
        case 8: hipLaunchKernelGGL((k_full_sigma<T, 8, ASM, G>), grid, block, 0, st, A, x, y); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Lanes per bra row, from the list's mean row length m: about m / 2, a power of
// two from 8 to 64.  Fewer lanes per row put several short rows in one
// wavefront (more connections in flight per wave); at m = 28 sixteen lanes
// beat 64 by a quarter, at m = 275 64 lanes are best.
int full_lanes(int64_t n, int64_t nconn) {
    const double m = n > 0 ? (double)nconn / (double)n : 0.0;
    return m >= 96 ? 64 : m >= 48 ? 32 : m >= 12 ? 16 : 8;
}

template <class T, bool ASM>
hipError_t full_sigma_lanes(const FullArgs& A, int64_t nconn, int nvec, const T* x, T* y, int layout,
                            hipStream_t st) {
    switch (full_lanes(A.n, nconn)) {
        case 64: return full_sigma_layouts<T, ASM, 64>(A, nvec, x, y, layout, st);
        case 32: return full_sigma_layouts<T, ASM, 32>(A, nvec, x, y, layout, st);
        case 16: return full_sigma_layouts<T, ASM, 16>(A, nvec, x, y, layout, st);
        default: return full_sigma_layouts<T, ASM, 8>(A, nvec, x, y, layout, st);
    }
}

}  // namespace

template <class T>
hipError_t launch_full_values(const FullSigmaArgs& S, T* out, hipStream_t st) {
    if (S.n <= 0) return hipGetLastError();
    const FullArgs A = full_args(S);
    hipLaunchKernelGGL((k_full_values<T>), dim3(blocks_for(S.n, 4)), dim3(256), 0, st, A, out);
    return hipGetLastError();
}

template hipError_t launch_full_values<double>(const FullSigmaArgs&, double*, hipStream_t);
template hipError_t launch_full_values<float>(const FullSigmaArgs&, float*, hipStream_t);

template <class T>
hipError_t launch_full_sigma(const FullSigmaArgs& S, int nvec, const T* x, T* y, int layout, hipStream_t st) {
    if (S.n <= 0) return hipGetLastError();
    FullArgs A = full_args(S);
    const void* vals = sizeof(T) == 8 ? (const void*)S.v64 : (const void*)S.v32;
    if (vals) {
        A.vals = vals;
        return full_sigma_lanes<T, true>(A, S.nconn, nvec, x, y, layout, st);
    }
    return full_sigma_lanes<T, false>(A, S.nconn, nvec, x, y, layout, st);
}

template hipError_t launch_full_sigma<double>(const FullSigmaArgs&, int, const double*, double*, int, hipStream_t);
template hipError_t launch_full_sigma<float>(const FullSigmaArgs&, int, const float*, float*, int, hipStream_t);

}  // namespace sbd
