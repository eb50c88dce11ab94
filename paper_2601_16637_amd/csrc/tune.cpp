// Autotuner of the sigma launch configuration.
//
// For one problem shape (alpha/beta string counts, orbitals, precision,
// vectors per launch) it times a small set of candidate configurations of the
// sigma kernels on scratch vectors with HIP events and keeps the fastest.
// Results are cached process-wide per shape and stored in the Hamiltonian
// handle, which every later sigma on that handle uses.  The candidates differ
// only in scheduling (rows per wavefront, LDS budget of the alpha-beta
// kernel); all produce the same sigma up to summation order.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace sbd {

int sigma_internal(const sbd_exc* x, const sbd_ham* H, int nvec, int prec, double shift,
                   const void* c, void* y, int layout, void* ws, hipStream_t st,
                   hipEvent_t* ev = nullptr);
hipError_t launch_fill_pattern(void* p, int64_t n, int prec, hipStream_t st);

namespace {
using Key = std::tuple<int64_t, int64_t, int, int, int, int>;
std::mutex g_mu;
std::map<Key, SigmaTune> g_cache;
}  // namespace

std::vector<SigmaTune> tune_candidates() {
    std::vector<SigmaTune> out;
    for (int wide : {0, 1})
        for (int rw : {1, 2})
            for (int lds : {49152, 98304, 147456}) {
                SigmaTune t;
                t.stream_rw = rw;
                t.ab_lds_bytes = lds;
                t.stream_wide = wide;
                out.push_back(t);
            }
    return out;
}

}  // namespace sbd

using namespace sbd;

extern "C" int sbd_autotune(const sbd_basis* b, const sbd_exc* x, sbd_ham* H, int prec, int nvec,
                            int layout, void* stream, double* best_ms) {
    if (!b || !x || !H) return fail(SBD_ERR_ARG, "null argument");
    if (x->basis_id != b->id || H->basis_id != b->id || H->exc_id != x->id)
        return fail(SBD_ERR_STATE, "handles do not belong together");
    if (prec != SBD_FP64 && prec != SBD_FP32) return fail(SBD_ERR_ARG, "bad precision");
    if (nvec < 1 || (layout == 1 && nvec != 1 && nvec != 2 && nvec != 4 && nvec != 8) ||
        (layout != 0 && layout != 1))
        return fail(SBD_ERR_ARG, "bad nvec/layout");
    const Key key{H->na, H->nb, H->norb, prec, nvec, layout};
    {
        std::lock_guard<std::mutex> g(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            H->tune[prec] = it->second;
            if (best_ms) *best_ms = -1.0;
            return SBD_OK;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = H->na * H->nb;
    const size_t elem = prec == SBD_FP64 ? 8 : 4;
    DevBuf cbuf, ybuf, ws;
    SBD_HIP(cbuf.alloc(elem * (size_t)N * nvec));
    SBD_HIP(ybuf.alloc(elem * (size_t)N * nvec));
    SBD_HIP(ws.alloc(sigma_workspace_bytes(N, nvec, layout, elem)));
    SBD_HIP(launch_fill_pattern(cbuf.p, N * nvec, prec, st));
    hipEvent_t e0, e1;
    SBD_HIP(hipEventCreate(&e0));
    SBD_HIP(hipEventCreate(&e1));
    const SigmaTune saved = H->tune[prec];
    SigmaTune best = saved;
    float best_t = 1e30f;
    int rc = SBD_OK;
    for (const SigmaTune& cand : tune_candidates()) {
        H->tune[prec] = cand;
        rc = sigma_internal(x, H, nvec, prec, 0.0, cbuf.p, ybuf.p, layout, ws.p, st);  // warm-up
        if (rc) break;
        hipError_t e = hipEventRecord(e0, st);
        for (int r = 0; r < 3 && e == hipSuccess && !rc; ++r)
            rc = sigma_internal(x, H, nvec, prec, 0.0, cbuf.p, ybuf.p, layout, ws.p, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune timing");
            break;
        }
        if (rc) break;
        if (ms < best_t) {
            best_t = ms;
            best = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        H->tune[prec] = saved;
        return rc;
    }
    H->tune[prec] = best;
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_cache[key] = best;
    }
    if (best_ms) *best_ms = best_t / 3.0;
    return SBD_OK;
}

extern "C" int sbd_get_tune(const sbd_ham* H, int prec, int* stream_rw, int* ab_lds_bytes,
                            int* stream_wide) {
    if (!H || (prec != SBD_FP64 && prec != SBD_FP32)) return fail(SBD_ERR_ARG, "bad argument");
    if (stream_rw) *stream_rw = H->tune[prec].stream_rw;
    if (ab_lds_bytes) *ab_lds_bytes = H->tune[prec].ab_lds_bytes;
    if (stream_wide) *stream_wide = H->tune[prec].stream_wide;
    return SBD_OK;
}

extern "C" int sbd_set_tune(sbd_ham* H, int prec, int stream_rw, int ab_lds_bytes, int stream_wide) {
    if (!H || (prec != SBD_FP64 && prec != SBD_FP32)) return fail(SBD_ERR_ARG, "bad argument");
    if (stream_rw != 1 && stream_rw != 2) return fail(SBD_ERR_ARG, "stream_rw must be 1 or 2");
    if (ab_lds_bytes < 4096 || ab_lds_bytes > (1 << 20)) return fail(SBD_ERR_ARG, "bad LDS budget");
    if (stream_wide != 0 && stream_wide != 1) return fail(SBD_ERR_ARG, "stream_wide must be 0 or 1");
    H->tune[prec].stream_rw = stream_rw;
    H->tune[prec].ab_lds_bytes = ab_lds_bytes;
    H->tune[prec].stream_wide = stream_wide;
    return SBD_OK;
}
