// C ABI entry points: argument validation on the host, handle construction,
// and kernel launches.  See include/sbd.h for the contract of each call.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>

#include "internal.h"

namespace sbd {

static thread_local std::string g_err = "";
static std::atomic<uint64_t> g_next_id{1};

void set_error(const std::string& msg) { g_err = msg; }

int fail(int status, const std::string& msg) {
    g_err = msg;
    return status;
}

int hip_fail(hipError_t e, const char* what) {
    std::string m = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
    g_err = m;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SBD_ERR_NOMEM;
    return SBD_ERR_HIP;
}

static int validate_strings(int norb, int nel, const uint64_t* s, int64_t n, const char* which) {
    if (!s || n < 1) return fail(SBD_ERR_ARG, std::string(which) + ": need at least one string");
    const uint64_t high = norb >= 64 ? 0ull : ~((1ull << norb) - 1ull);
    for (int64_t i = 0; i < n; ++i) {
        if (s[i] & high)
            return fail(SBD_ERR_STRING, std::string(which) + " string " + std::to_string(i) +
                                            " has a bit at or above norb");
        if (__builtin_popcountll(s[i]) != nel)
            return fail(SBD_ERR_STRING, std::string(which) + " string " + std::to_string(i) +
                                            " has popcount != " + std::to_string(nel));
    }
    return SBD_OK;
}

int validate_integrals(int n, const double* h, const double* eri) {
    double hmax = 0.0, gmax = 0.0;
    for (int i = 0; i < n * n; ++i) {
        if (!std::isfinite(h[i])) return fail(SBD_ERR_INTEGRALS, "h has a non-finite entry");
        hmax = std::max(hmax, std::fabs(h[i]));
    }
    const size_t n4 = (size_t)n * n * n * n;
    for (size_t i = 0; i < n4; ++i) {
        if (!std::isfinite(eri[i])) return fail(SBD_ERR_INTEGRALS, "eri has a non-finite entry");
        gmax = std::max(gmax, std::fabs(eri[i]));
    }
    const double th = 1e-10 * std::max(hmax, 1e-300), tg = 1e-10 * std::max(gmax, 1e-300);
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            if (std::fabs(h[p * n + q] - h[q * n + p]) > th)
                return fail(SBD_ERR_INTEGRALS, "h is not symmetric");
    auto G = [&](int p, int q, int r, int s) { return eri[(((size_t)p * n + q) * n + r) * n + s]; };
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s) {
                    double v = G(p, q, r, s);
                    if (std::fabs(v - G(q, p, r, s)) > tg || std::fabs(v - G(p, q, s, r)) > tg ||
                        std::fabs(v - G(r, s, p, q)) > tg)
                        return fail(SBD_ERR_INTEGRALS, "eri is not 8-fold symmetric");
                }
    return SBD_OK;
}

}  // namespace sbd

using namespace sbd;

extern "C" {

const char* sbd_last_error(void) { return g_err.c_str(); }

int sbd_version(void) { return 100; }
#ifndef SBD_SOURCE_HASH
#define SBD_SOURCE_HASH "unknown"
#endif
const char* sbd_source_hash(void) { return SBD_SOURCE_HASH; }

// ------------------------------------------------------------------ basis
int sbd_build_basis(int norb, int n_alpha, int n_beta, const uint64_t* alpha_strings,
                    int64_t n_alpha_in, const uint64_t* beta_strings, int64_t n_beta_in,
                    void* stream, sbd_basis** out) {
    if (!out) return fail(SBD_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (norb < 1 || norb > 64) return fail(SBD_ERR_NORB, "norb must be in [1, 64]");
    if (n_alpha < 0 || n_alpha > norb || n_beta < 0 || n_beta > norb)
        return fail(SBD_ERR_ARG, "electron counts must be in [0, norb]");
    int rc = validate_strings(norb, n_alpha, alpha_strings, n_alpha_in, "alpha");
    if (rc) return rc;
    rc = validate_strings(norb, n_beta, beta_strings, n_beta_in, "beta");
    if (rc) return rc;
    if (n_alpha_in > (int64_t)1 << 30 || n_beta_in > (int64_t)1 << 30)
        return fail(SBD_ERR_ARG, "too many strings (limit 2^30 per spin)");

    hipStream_t st = (hipStream_t)stream;
    sbd_basis* b = new sbd_basis();
    b->norb = norb;
    b->n_el[0] = n_alpha;
    b->n_el[1] = n_beta;
    const uint64_t* src[2] = {alpha_strings, beta_strings};
    int64_t nin[2] = {n_alpha_in, n_beta_in};
    for (int s = 0; s < 2; ++s) {
        int64_t P = 1;
        while (P < nin[s]) P <<= 1;
        DevBuf work, cnt;
        hipError_t e = work.alloc(sizeof(uint64_t) * P);
        if (e == hipSuccess) e = cnt.alloc(sizeof(int64_t));
        if (e == hipSuccess) e = b->s[s].d.alloc(sizeof(uint64_t) * nin[s]);
        if (e == hipSuccess)
            e = hipMemcpyAsync(work.p, src[s], sizeof(uint64_t) * nin[s], hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = launch_sort_unique(work.as<uint64_t>(), nin[s], b->s[s].d.as<uint64_t>(),
                                   cnt.as<int64_t>(), nullptr, st);
        int64_t count = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&count, cnt.p, sizeof(int64_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) {
            b->s[s].n = count;
            b->s[s].host.resize(count);
            e = hipMemcpyAsync(b->s[s].host.data(), b->s[s].d.p, sizeof(uint64_t) * count,
                               hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
        }
        if (e != hipSuccess) {
            delete b;
            return hip_fail(e, "sbd_build_basis");
        }
    }
    b->id = g_next_id++;
    *out = b;
    return SBD_OK;
}

int sbd_basis_sizes(const sbd_basis* b, int64_t* na, int64_t* nb) {
    if (!b || !na || !nb) return fail(SBD_ERR_ARG, "null argument");
    *na = b->s[0].n;
    *nb = b->s[1].n;
    return SBD_OK;
}

int sbd_basis_strings(const sbd_basis* b, uint64_t* a, uint64_t* bb) {
    if (!b) return fail(SBD_ERR_ARG, "null basis");
    if (a) std::memcpy(a, b->s[0].host.data(), sizeof(uint64_t) * b->s[0].n);
    if (bb) std::memcpy(bb, b->s[1].host.data(), sizeof(uint64_t) * b->s[1].n);
    return SBD_OK;
}

void sbd_free_basis(sbd_basis* b) { delete b; }

// ------------------------------------------------------------------ tables
// Position -> string map of the sliced-ELL singles table.  The alpha-beta
// kernel's thread t handles positions t + q*W (W = its workgroup size, one per
// window of W positions), a wavefront 64 consecutive positions per window, and a
// workgroup lasts as long as its slowest wavefront.  Inside each window the
// strings are sorted by descending row length (64-position slices of similar
// lengths: little padding), and the window's slices are rotated by q*(S/2 - 1)
// (S = slices per window, co-prime with it), so each wavefront meets long and
// short slices in turn and the wavefronts of a workgroup carry similar work.
static std::vector<int32_t> sell_positions(const std::vector<int64_t>& rp, int W) {
    const int64_t n = (int64_t)rp.size() - 1;
    std::vector<int32_t> pos((size_t)std::max<int64_t>(n, 1));
    std::vector<int32_t> win;
    for (int64_t w0 = 0, q = 0; w0 < n; w0 += W, ++q) {
        const int64_t w1 = std::min<int64_t>(n, w0 + W);
        win.resize((size_t)(w1 - w0));
        std::iota(win.begin(), win.end(), (int32_t)w0);
        std::stable_sort(win.begin(), win.end(), [&](int32_t a, int32_t b) {
            return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
        });
        // whole slices rotate; a last window's partial slice keeps its place at the end
        const int64_t S = (w1 - w0) / 64;
        const int64_t r = S > 1 ? (q * (W / 128 - 1)) % S : 0;
        for (int64_t j = 0; j < w1 - w0; ++j) {
            const int64_t sl = j / 64, dst = (r && sl < S) ? ((sl + r) % S) * 64 + j % 64 : j;
            pos[(size_t)(w0 + dst)] = win[(size_t)j];
        }
    }
    return pos;
}

int sbd_build_excitations(const sbd_basis* b, void* stream, sbd_exc** out) {
    if (!b || !out) return fail(SBD_ERR_ARG, "null argument");
    *out = nullptr;
    hipStream_t st = (hipStream_t)stream;
    sbd_exc* x = new sbd_exc();
    x->basis_id = b->id;
    for (int s = 0; s < 2; ++s) {
        const int64_t n = b->s[s].n;
        x->n[s] = n;
        DevBuf c1, c2;
        Table& t1 = x->t[s][0];
        Table& t2 = x->t[s][1];
        t1.kind = 1;
        t2.kind = 2;
        hipError_t e = c1.alloc(sizeof(int64_t) * n);
        if (e == hipSuccess) e = c2.alloc(sizeof(int64_t) * n);
        if (e == hipSuccess) e = t1.row_ptr.alloc(sizeof(int64_t) * (n + 1));
        if (e == hipSuccess) e = t2.row_ptr.alloc(sizeof(int64_t) * (n + 1));
        if (e == hipSuccess)
            e = launch_exc_count(b->s[s].d.as<uint64_t>(), n, c1.as<int64_t>(), c2.as<int64_t>(), st);
        if (e == hipSuccess) e = launch_exclusive_scan(c1.as<int64_t>(), n, t1.row_ptr.as<int64_t>(), nullptr, st);
        if (e == hipSuccess) e = launch_exclusive_scan(c2.as<int64_t>(), n, t2.row_ptr.as<int64_t>(), nullptr, st);
        int64_t tot[2] = {0, 0};
        if (e == hipSuccess)
            e = hipMemcpyAsync(&tot[0], t1.row_ptr.as<int64_t>() + n, sizeof(int64_t),
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&tot[1], t2.row_ptr.as<int64_t>() + n, sizeof(int64_t),
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) {
            t1.nnz = tot[0];
            t2.nnz = tot[1];
            for (Table* t : {&t1, &t2}) {
                size_t m = (size_t)std::max<int64_t>(t->nnz, 1);
                if (e == hipSuccess) e = t->J.alloc(sizeof(int32_t) * m);
                if (e == hipSuccess) e = t->orb.alloc(sizeof(uint32_t) * m);
                if (e == hipSuccess) e = t->sign.alloc(sizeof(int8_t) * m);
            }
        }
        if (e == hipSuccess)
            e = launch_exc_fill(b->s[s].d.as<uint64_t>(), n, t1.row_ptr.as<int64_t>(),
                                t2.row_ptr.as<int64_t>(), t1.J.as<int32_t>(), t1.orb.as<uint32_t>(),
                                t1.sign.as<int8_t>(), t2.J.as<int32_t>(), t2.orb.as<uint32_t>(),
                                t2.sign.as<int8_t>(), st);
        if (e == hipSuccess) e = t1.pack.alloc(sizeof(uint64_t) * (size_t)std::max<int64_t>(t1.nnz, 1));
        if (e == hipSuccess)
            e = launch_pack_singles(t1.nnz, t1.J.as<int32_t>(), t1.orb.as<uint32_t>(),
                                    t1.sign.as<int8_t>(), t1.pack.as<uint64_t>(), st);
        // sliced-ELL copy of the singles (used when this spin is gathered per lane),
        // over positions that balance the work of the alpha-beta kernel's wavefronts
        const int64_t nslice = (n + 63) / 64;
        std::vector<int64_t> rp_h((size_t)n + 1);
        std::vector<int32_t> pos;
        if (e == hipSuccess)
            e = hipMemcpyAsync(rp_h.data(), t1.row_ptr.p, sizeof(int64_t) * (size_t)(n + 1),
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) {
            pos = sell_positions(rp_h, ab_block_threads(n));
            e = t1.sell_pos.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
        }
        if (e == hipSuccess && n > 0)
            e = hipMemcpyAsync(t1.sell_pos.p, pos.data(), sizeof(int32_t) * (size_t)n,
                               hipMemcpyHostToDevice, st);
        DevBuf slots;
        if (e == hipSuccess) e = slots.alloc(sizeof(int64_t) * (size_t)std::max<int64_t>(nslice, 1));
        if (e == hipSuccess) e = t1.sell_off.alloc(sizeof(int64_t) * (size_t)(nslice + 1));
        if (e == hipSuccess)
            e = launch_sell_len(t1.row_ptr.as<int64_t>(), t1.sell_pos.as<int32_t>(), n,
                                slots.as<int64_t>(), st);
        if (e == hipSuccess)
            e = launch_exclusive_scan(slots.as<int64_t>(), nslice, t1.sell_off.as<int64_t>(), nullptr, st);
        int64_t sell_total = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&sell_total, t1.sell_off.as<int64_t>() + nslice, sizeof(int64_t),
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) {
            t1.sell_entries = sell_total;
            e = t1.sell.alloc(sizeof(uint64_t) * (size_t)std::max<int64_t>(sell_total, 1));
        }
        if (e == hipSuccess)
            e = launch_sell_fill(t1.row_ptr.as<int64_t>(), t1.pack.as<uint64_t>(),
                                 t1.sell_pos.as<int32_t>(), n, t1.sell_off.as<int64_t>(),
                                 t1.sell.as<uint64_t>(), st);
        // 32-bit entries for the alpha-beta kernel (ket index in 18 bits)
        if (e == hipSuccess && n <= ((int64_t)1 << kSellJBits)) {
            e = t1.sell32.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(sell_total, 1));
            if (e == hipSuccess)
                e = launch_sell_compact(t1.sell.as<uint64_t>(), sell_total, b->norb, t1.sell32.as<uint32_t>(), st);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            delete x;
            return hip_fail(e, "sbd_build_excitations");
        }
    }
    x->id = g_next_id++;
    *out = x;
    return SBD_OK;
}

int sbd_exc_count(const sbd_exc* x, int spin, int kind, int64_t* nnz) {
    if (!x || !nnz || spin < 0 || spin > 1 || kind < 1 || kind > 2)
        return fail(SBD_ERR_ARG, "bad argument");
    *nnz = x->t[spin][kind - 1].nnz;
    return SBD_OK;
}

int sbd_exc_export(const sbd_exc* x, int spin, int kind, int64_t* row_ptr, int32_t* J,
                   uint8_t* orbs, int8_t* sign) {
    if (!x || spin < 0 || spin > 1 || kind < 1 || kind > 2) return fail(SBD_ERR_ARG, "bad argument");
    const Table& t = x->t[spin][kind - 1];
    const int64_t n = x->n[spin];
    if (row_ptr) SBD_HIP(hipMemcpy(row_ptr, t.row_ptr.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    if (t.nnz == 0) return SBD_OK;
    if (J) SBD_HIP(hipMemcpy(J, t.J.p, sizeof(int32_t) * t.nnz, hipMemcpyDeviceToHost));
    if (sign) SBD_HIP(hipMemcpy(sign, t.sign.p, sizeof(int8_t) * t.nnz, hipMemcpyDeviceToHost));
    if (orbs) {
        std::vector<uint32_t> o(t.nnz);
        SBD_HIP(hipMemcpy(o.data(), t.orb.p, sizeof(uint32_t) * t.nnz, hipMemcpyDeviceToHost));
        const int w = 2 * kind;
        for (int64_t e = 0; e < t.nnz; ++e)
            for (int q = 0; q < w; ++q) orbs[e * w + q] = (uint8_t)((o[e] >> (8 * q)) & 255);
    }
    return SBD_OK;
}

void sbd_free_exc(sbd_exc* x) { delete x; }

// ------------------------------------------------------------------ hamiltonian
int sbd_set_hamiltonian(const sbd_basis* b, const sbd_exc* x, const double* h1, const double* eri,
                        double e_core, void* stream, sbd_ham** out) {
    if (!b || !x || !h1 || !eri || !out) return fail(SBD_ERR_ARG, "null argument");
    *out = nullptr;
    if (x->basis_id != b->id) return fail(SBD_ERR_STATE, "excitation tables belong to another basis");
    if (!std::isfinite(e_core)) return fail(SBD_ERR_INTEGRALS, "e_core is not finite");
    const int n = b->norb;
    int rc = validate_integrals(n, h1, eri);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    sbd_ham* H = new sbd_ham();
    H->basis_id = b->id;
    H->exc_id = x->id;
    H->norb = n;
    H->na = b->s[0].n;
    H->nb = b->s[1].n;
    H->e_core = e_core;
    const size_t n4 = (size_t)n * n * n * n;
    hipError_t e = H->h64.alloc(sizeof(double) * n * n);
    if (e == hipSuccess) e = H->eri64.alloc(sizeof(double) * n4);
    if (e == hipSuccess) e = H->eri32.alloc(sizeof(float) * n4);
    if (e == hipSuccess) e = hipMemcpyAsync(H->h64.p, h1, sizeof(double) * n * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(H->eri64.p, eri, sizeof(double) * n4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_d2f(H->eri64.as<double>(), H->eri32.as<float>(), (int64_t)n4, st);
    const int np = npairs(n);
    for (int s = 0; s < 2 && e == hipSuccess; ++s) {
        SpinCoef& C = H->sc[s];
        const int64_t ns = b->s[s].n;
        const Table& t1 = x->t[s][0];
        const Table& t2 = x->t[s][1];
        const size_t m1 = (size_t)std::max<int64_t>(t1.nnz, 1), m2 = (size_t)std::max<int64_t>(t2.nnz, 1);
        if (e == hipSuccess) e = C.c1_64.alloc(sizeof(double) * m1);
        if (e == hipSuccess) e = C.c1_32.alloc(sizeof(float) * m1);
        if (e == hipSuccess) e = C.ps1.alloc(sizeof(int32_t) * m1);
        if (e == hipSuccess) e = C.c2_64.alloc(sizeof(double) * m2);
        if (e == hipSuccess) e = C.c2_32.alloc(sizeof(float) * m2);
        if (e == hipSuccess) e = C.G64.alloc(sizeof(double) * (size_t)np * ns);
        if (e == hipSuccess) e = C.G32.alloc(sizeof(float) * (size_t)np * ns);
        if (e == hipSuccess) e = C.dspin.alloc(sizeof(double) * ns);
        const uint64_t* ds = b->s[s].d.as<uint64_t>();
        if (e == hipSuccess) e = launch_string_diag(ds, ns, n, H->h64.as<double>(), H->eri64.as<double>(), C.dspin.as<double>(), st);
        if (e == hipSuccess) e = launch_spectator(ds, ns, n, H->eri64.as<double>(), C.G64.as<double>(), C.G32.as<float>(), st);
        if (e == hipSuccess)
            e = launch_single_coef(ds, t1.nnz, t1.J.as<int32_t>(), t1.orb.as<uint32_t>(), t1.sign.as<int8_t>(), n,
                                   H->h64.as<double>(), H->eri64.as<double>(), C.c1_64.as<double>(),
                                   C.c1_32.as<float>(), C.ps1.as<int32_t>(), st);
        if (e == hipSuccess)
            e = launch_double_coef(t2.nnz, t2.orb.as<uint32_t>(), t2.sign.as<int8_t>(), n, H->eri64.as<double>(),
                                   C.c2_64.as<double>(), C.c2_32.as<float>(), st);
    }
    const int64_t N = H->na * H->nb;
    if (e == hipSuccess) e = H->diag.alloc(sizeof(double) * N);
    if (e == hipSuccess)
        e = launch_full_diag(b->s[0].d.as<uint64_t>(), H->na, H->sc[0].dspin.as<double>(),
                             H->sc[1].dspin.as<double>(), H->sc[1].G64.as<double>(), H->nb, n, e_core,
                             H->diag.as<double>(), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete H;
        return hip_fail(e, "sbd_set_hamiltonian");
    }
    *out = H;
    return SBD_OK;
}

int sbd_ham_diag(const sbd_ham* H, double* diag_dev, void* stream) {
    if (!H || !diag_dev) return fail(SBD_ERR_ARG, "null argument");
    SBD_HIP(hipMemcpyAsync(diag_dev, H->diag.p, sizeof(double) * H->na * H->nb,
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SBD_OK;
}

void sbd_free_ham(sbd_ham* H) { delete H; }

}  // extern "C"

namespace sbd {
template <class T>
static SigmaArgs<T> make_args(const sbd_exc* x, const sbd_ham* H, double shift);

template <>
SigmaArgs<double> make_args<double>(const sbd_exc* x, const sbd_ham* H, double shift) {
    SigmaArgs<double> A{};
    A.na = H->na; A.nb = H->nb; A.norb = H->norb;
    const Table *a1 = &x->t[0][0], *a2 = &x->t[0][1], *b1 = &x->t[1][0], *b2 = &x->t[1][1];
    A.a1p = a1->row_ptr.as<int64_t>(); A.a1J = a1->J.as<int32_t>(); A.a1pack = a1->pack.as<uint64_t>();
    A.a1c = H->sc[0].c1_64.as<double>(); A.a1ps = H->sc[0].ps1.as<int32_t>();
    A.a2p = a2->row_ptr.as<int64_t>(); A.a2J = a2->J.as<int32_t>(); A.a2c = H->sc[0].c2_64.as<double>();
    A.b1p = b1->row_ptr.as<int64_t>(); A.b1J = b1->J.as<int32_t>(); A.b1pack = b1->pack.as<uint64_t>();
    A.b1sell = b1->sell.as<uint64_t>(); A.b1sell_off = b1->sell_off.as<int64_t>();
    A.b1sell_pos = b1->sell_pos.as<int32_t>();
    A.b1sell32 = b1->sell32.as<uint32_t>();
    A.b1c = H->sc[1].c1_64.as<double>(); A.b1ps = H->sc[1].ps1.as<int32_t>();
    A.b2p = b2->row_ptr.as<int64_t>(); A.b2J = b2->J.as<int32_t>(); A.b2c = H->sc[1].c2_64.as<double>();
    A.Ga = H->sc[0].G64.as<double>(); A.Gb = H->sc[1].G64.as<double>();
    A.eri = H->eri64.as<double>(); A.diag = H->diag.as<double>(); A.shift = shift;
    return A;
}

template <>
SigmaArgs<float> make_args<float>(const sbd_exc* x, const sbd_ham* H, double shift) {
    SigmaArgs<float> A{};
    A.na = H->na; A.nb = H->nb; A.norb = H->norb;
    const Table *a1 = &x->t[0][0], *a2 = &x->t[0][1], *b1 = &x->t[1][0], *b2 = &x->t[1][1];
    A.a1p = a1->row_ptr.as<int64_t>(); A.a1J = a1->J.as<int32_t>(); A.a1pack = a1->pack.as<uint64_t>();
    A.a1c = H->sc[0].c1_32.as<float>(); A.a1ps = H->sc[0].ps1.as<int32_t>();
    A.a2p = a2->row_ptr.as<int64_t>(); A.a2J = a2->J.as<int32_t>(); A.a2c = H->sc[0].c2_32.as<float>();
    A.b1p = b1->row_ptr.as<int64_t>(); A.b1J = b1->J.as<int32_t>(); A.b1pack = b1->pack.as<uint64_t>();
    A.b1sell = b1->sell.as<uint64_t>(); A.b1sell_off = b1->sell_off.as<int64_t>();
    A.b1sell_pos = b1->sell_pos.as<int32_t>();
    A.b1sell32 = b1->sell32.as<uint32_t>();
    A.b1c = H->sc[1].c1_32.as<float>(); A.b1ps = H->sc[1].ps1.as<int32_t>();
    A.b2p = b2->row_ptr.as<int64_t>(); A.b2J = b2->J.as<int32_t>(); A.b2c = H->sc[1].c2_32.as<float>();
    A.Ga = H->sc[0].G32.as<float>(); A.Gb = H->sc[1].G32.as<float>();
    A.eri = H->eri32.as<float>(); A.diag = H->diag.as<double>(); A.shift = shift;
    return A;
}

// y = (H - shift) c through the assembled CSR (nvec vectors, either layout);
// ev (nullable): the six stage events, all but the first two after the product
static int spmv_internal(const sbd_ham* H, int nvec, int prec, double shift, const void* c, void* y,
                         int layout, hipStream_t st, hipEvent_t* ev) {
    const int64_t N = H->na * H->nb;
    const int64_t* rp = H->csr_rp.as<int64_t>();
    const int32_t* col = H->csr_col.as<int32_t>();
    hipError_t e = ev ? hipEventRecord(ev[0], st) : hipSuccess;
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], st);
    const int nv = layout == 1 ? nvec : 1;
    const int reps = layout == 1 ? 1 : nvec;
    for (int v = 0; v < reps && e == hipSuccess; ++v) {
        if (prec == SBD_FP64)
            e = launch_spmv<double>(rp, col, H->csr_v64.as<double>(), N, nv, shift,
                                    (const double*)c + (size_t)v * N, (double*)y + (size_t)v * N, st);
        else
            e = launch_spmv<float>(rp, col, H->csr_v32.as<float>(), N, nv, shift,
                                   (const float*)c + (size_t)v * N, (float*)y + (size_t)v * N, st);
    }
    for (int i = 2; i < 6 && e == hipSuccess && ev; ++i) e = hipEventRecord(ev[i], st);
    if (e != hipSuccess) return hip_fail(e, "sbd_sigma (assembled) launch");
    return SBD_OK;
}

int sigma_internal(const sbd_exc* x, const sbd_ham* H, int nvec, int prec, double shift,
                   const void* c, void* y, int layout, void* ws, hipStream_t st, hipEvent_t* ev) {
    if (H->csr_has[prec == SBD_FP64 ? 0 : 1]) return spmv_internal(H, nvec, prec, shift, c, y, layout, st, ev);
    hipError_t e;
    const SigmaTune tune = H->tune[prec == SBD_FP64 ? 0 : 1];
    if (prec == SBD_FP64)
        e = launch_sigma<double>(make_args<double>(x, H, shift), nvec, (const double*)c, (double*)y,
                                 layout, ws, tune, st, ev);
    else
        e = launch_sigma<float>(make_args<float>(x, H, shift), nvec, (const float*)c, (float*)y,
                                layout, ws, tune, st, ev);
    if (e != hipSuccess) return hip_fail(e, "sbd_sigma launch");
    return SBD_OK;
}

// Per-stream sigma workspace owned by the Hamiltonian handle (grown on demand).
void* ham_workspace(const sbd_ham* Hc, hipStream_t st, size_t bytes, int* rc) {
    sbd_ham* H = const_cast<sbd_ham*>(Hc);
    std::lock_guard<std::mutex> g(H->ws_mu);
    auto& buf = H->ws[st];
    if (!buf) buf.reset(new DevBuf());
    if (buf->bytes < bytes) {
        hipError_t e = buf->alloc(bytes);
        if (e != hipSuccess) {
            *rc = hip_fail(e, "sigma workspace");
            return nullptr;
        }
    }
    *rc = SBD_OK;
    return buf->p;
}
}  // namespace sbd

namespace sbd {
// Argument checks shared by the sigma entry points (no device work).
int sigma_validate(const sbd_basis* b, const sbd_exc* x, const sbd_ham* H, int nvec, int prec,
                   double shift, const void* c, const void* sigma, int layout) {
    if (!b || !x || !H || !c || !sigma) return fail(SBD_ERR_ARG, "null argument");
    if (x->basis_id != b->id || H->basis_id != b->id || H->exc_id != x->id)
        return fail(SBD_ERR_STATE, "handles do not belong together");
    if (nvec < 1) return fail(SBD_ERR_ARG, "nvec must be >= 1");
    if (layout != 0 && layout != 1) return fail(SBD_ERR_ARG, "layout must be 0 or 1");
    if (layout == 1 && nvec > 8) return fail(SBD_ERR_ARG, "interleaved layout supports nvec <= 8");
    if (prec != SBD_FP64 && prec != SBD_FP32) return fail(SBD_ERR_ARG, "bad precision");
    if (!std::isfinite(shift)) return fail(SBD_ERR_ARG, "shift is not finite");
    if (c == sigma) return fail(SBD_ERR_ARG, "c and sigma must not alias");
    if (layout == 1 && nvec != 1 && nvec != 2 && nvec != 4 && nvec != 8)
        return fail(SBD_ERR_ARG, "interleaved layout supports nvec in {1, 2, 4, 8}");
    return SBD_OK;
}
}  // namespace sbd

static int sigma_entry(const sbd_basis* b, const sbd_exc* x, const sbd_ham* H, int nvec, int prec,
                       double shift, const void* c, void* sigma, int layout, void* stream,
                       hipEvent_t* ev) {
    int rc = sigma_validate(b, x, H, nvec, prec, shift, c, sigma, layout);
    if (rc) return rc;
    const int64_t N = H->na * H->nb;
    void* ws = ham_workspace(H, (hipStream_t)stream,
                             sigma_workspace_bytes(N, nvec, layout, prec == SBD_FP64 ? 8 : 4), &rc);
    if (!ws && N > 0) return rc;
    return sigma_internal(x, H, nvec, prec, shift, c, sigma, layout, ws, (hipStream_t)stream, ev);
}

extern "C" int sbd_sigma(const sbd_basis* b, const sbd_exc* x, const sbd_ham* H, int nvec, int prec,
                         double shift, const void* c, void* sigma, int layout, void* stream) {
    return sigma_entry(b, x, H, nvec, prec, shift, c, sigma, layout, stream, nullptr);
}

extern "C" int sbd_sigma_timed(const sbd_basis* b, const sbd_exc* x, const sbd_ham* H, int nvec,
                               int prec, double shift, const void* c, void* sigma, int layout,
                               void* stream, double* stage_ms) {
    if (!stage_ms) return fail(SBD_ERR_ARG, "stage_ms is NULL");
    hipEvent_t ev[6];
    for (int i = 0; i < 6; ++i) SBD_HIP(hipEventCreate(&ev[i]));
    int rc = sigma_entry(b, x, H, nvec, prec, shift, c, sigma, layout, stream, ev);
    hipError_t e = rc ? hipSuccess : hipEventSynchronize(ev[5]);
    for (int i = 0; i < 5 && !rc && e == hipSuccess; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        stage_ms[i] = ms;
    }
    for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "sbd_sigma_timed");
    return SBD_OK;
}

extern "C" int sbd_ham_assemble(sbd_ham* H, const sbd_exc* x, int precisions, size_t max_bytes, void* stream,
                                int64_t* nnz_out) {
    if (!H || !x) return fail(SBD_ERR_ARG, "null argument");
    if (H->exc_id != x->id) return fail(SBD_ERR_STATE, "tables do not belong to this Hamiltonian");
    if (precisions < 1 || precisions > 3) return fail(SBD_ERR_ARG, "precisions must be 1 (FP64), 2 (FP32) or 3");
    const int64_t N = H->na * H->nb;
    if (N >= ((int64_t)1 << 31)) return fail(SBD_ERR_ARG, "assembly needs fewer than 2^31 determinants");
    hipStream_t st = (hipStream_t)stream;
    CsrTables t{};
    t.na = H->na; t.nb = H->nb; t.norb = H->norb;
    const Table *a1 = &x->t[0][0], *a2 = &x->t[0][1], *b1 = &x->t[1][0], *b2 = &x->t[1][1];
    t.a1p = a1->row_ptr.as<int64_t>(); t.a2p = a2->row_ptr.as<int64_t>();
    t.b1p = b1->row_ptr.as<int64_t>(); t.b2p = b2->row_ptr.as<int64_t>();
    t.a1J = a1->J.as<int32_t>(); t.a2J = a2->J.as<int32_t>(); t.b1J = b1->J.as<int32_t>(); t.b2J = b2->J.as<int32_t>();
    t.a1c = H->sc[0].c1_64.as<double>(); t.a2c = H->sc[0].c2_64.as<double>();
    t.b1c = H->sc[1].c1_64.as<double>(); t.b2c = H->sc[1].c2_64.as<double>();
    t.a1ps = H->sc[0].ps1.as<int32_t>(); t.b1ps = H->sc[1].ps1.as<int32_t>();
    t.a1pack = a1->pack.as<uint64_t>(); t.b1pack = b1->pack.as<uint64_t>();
    t.Ga = H->sc[0].G64.as<double>(); t.Gb = H->sc[1].G64.as<double>();
    t.eri = H->eri64.as<double>(); t.diag = H->diag.as<double>();
    // row lengths, their scan, then the size check before the large allocations
    DevBuf cnt, rp, tmp;
    SBD_HIP(cnt.alloc(sizeof(int64_t) * (size_t)std::max<int64_t>(N, 1)));
    SBD_HIP(rp.alloc(sizeof(int64_t) * (size_t)(N + 1)));
    SBD_HIP(tmp.alloc(sizeof(int64_t) * (size_t)scan_tmp_words(N)));
    SBD_HIP(launch_csr_count(t, cnt.as<int64_t>(), st));
    SBD_HIP(launch_exclusive_scan(cnt.as<int64_t>(), N, rp.as<int64_t>(), tmp.as<int64_t>(), st));
    int64_t nnz = 0;
    SBD_HIP(hipMemcpyAsync(&nnz, rp.as<int64_t>() + N, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SBD_HIP(hipStreamSynchronize(st));
    const bool f32 = (precisions & 2) != 0;
    const size_t need = (size_t)nnz * (sizeof(int32_t) + sizeof(double) + (f32 ? sizeof(float) : 0)) +
                        sizeof(int64_t) * (size_t)(N + 1);
    if (nnz_out) *nnz_out = nnz;
    if (max_bytes && need > max_bytes) return fail(SBD_ERR_NOMEM, "assembled Hamiltonian exceeds max_bytes");
    DevBuf col, v64, v32;
    SBD_HIP(col.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
    SBD_HIP(v64.alloc(sizeof(double) * (size_t)std::max<int64_t>(nnz, 1)));
    if (f32) SBD_HIP(v32.alloc(sizeof(float) * (size_t)std::max<int64_t>(nnz, 1)));
    SBD_HIP(launch_csr_fill(t, rp.as<int64_t>(), col.as<int32_t>(), v64.as<double>(), f32 ? v32.as<float>() : nullptr,
                            st));
    SBD_HIP(hipStreamSynchronize(st));
    H->csr_rp = std::move(rp);
    H->csr_col = std::move(col);
    H->csr_v64 = std::move(v64);
    H->csr_v32 = std::move(v32);
    H->csr_nnz = nnz;
    H->csr_has[0] = (precisions & 1) != 0;
    H->csr_has[1] = f32;
    return SBD_OK;
}

extern "C" int sbd_ham_release_assembled(sbd_ham* H) {
    if (!H) return fail(SBD_ERR_ARG, "null argument");
    H->csr_has[0] = H->csr_has[1] = false;
    H->csr_nnz = 0;
    H->csr_rp = DevBuf();
    H->csr_col = DevBuf();
    H->csr_v64 = DevBuf();
    H->csr_v32 = DevBuf();
    return SBD_OK;
}

extern "C" int sbd_ham_assembled(const sbd_ham* H, int64_t* nnz, int* precisions) {
    if (!H) return fail(SBD_ERR_ARG, "null argument");
    if (nnz) *nnz = H->csr_nnz;
    if (precisions) *precisions = (H->csr_has[0] ? 1 : 0) | (H->csr_has[1] ? 2 : 0);
    return SBD_OK;
}

extern "C" int sbd_map_vectors(const sbd_basis* from, const sbd_basis* to, int nvec, const double* x_from,
                               double* x_to, void* stream) {
    if (!from || !to || !x_from || !x_to) return fail(SBD_ERR_ARG, "null argument");
    if (nvec < 1) return fail(SBD_ERR_ARG, "nvec must be >= 1");
    if (from->norb != to->norb || from->n_el[0] != to->n_el[0] || from->n_el[1] != to->n_el[1])
        return fail(SBD_ERR_STATE, "bases differ in orbital or electron counts");
    hipStream_t st = (hipStream_t)stream;
    const int64_t na = to->s[0].n, nb = to->s[1].n, naf = from->s[0].n, nbf = from->s[1].n;
    DevBuf amap, bmap;
    SBD_HIP(amap.alloc(sizeof(int64_t) * (size_t)std::max<int64_t>(na, 1)));
    SBD_HIP(bmap.alloc(sizeof(int64_t) * (size_t)std::max<int64_t>(nb, 1)));
    SBD_HIP(launch_string_map(to->s[0].d.as<uint64_t>(), na, from->s[0].d.as<uint64_t>(), naf,
                              amap.as<int64_t>(), st));
    SBD_HIP(launch_string_map(to->s[1].d.as<uint64_t>(), nb, from->s[1].d.as<uint64_t>(), nbf,
                              bmap.as<int64_t>(), st));
    SBD_HIP(launch_map_vectors(amap.as<int64_t>(), bmap.as<int64_t>(), na, nb, nbf, naf * nbf, nvec, x_from,
                               x_to, st));
    SBD_HIP(hipStreamSynchronize(st));
    return SBD_OK;
}

extern "C" int sbd_gram(const double* A, int ma, const double* X, int k, int64_t N, double* out,
                        void* stream) {
    if (!A || !X || !out || N < 1) return fail(SBD_ERR_ARG, "null argument or N < 1");
    if (ma < 1 || ma > 48 || k < 1 || k > 8) return fail(SBD_ERR_ARG, "need 1 <= ma <= 48, 1 <= k <= 8");
    hipStream_t st = (hipStream_t)stream;
    DevBuf part, res;
    SBD_HIP(part.alloc(sizeof(double) * (size_t)ma * k * kRedBlocks));
    SBD_HIP(res.alloc(sizeof(double) * (size_t)ma * k));
    SBD_HIP(pass_project(A, ma, X, k, N, part.as<double>(), res.as<double>(), st));
    SBD_HIP(hipMemcpyAsync(out, res.p, sizeof(double) * (size_t)ma * k, hipMemcpyDeviceToHost, st));
    SBD_HIP(hipStreamSynchronize(st));
    return SBD_OK;
}
