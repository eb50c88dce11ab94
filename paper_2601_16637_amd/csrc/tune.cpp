// Autotuner of the sigma launch configuration.
//
// For one problem shape (alpha/beta string counts, orbitals, precision,
// vectors per launch) it times a small set of candidate configurations of the
// sigma kernels on scratch vectors with HIP events and keeps the fastest.
// Results are cached process-wide per shape and stored in the Hamiltonian
// handle, which every later sigma on that handle uses.  The candidates differ
// only in scheduling (the row-stream shape, tuned on the stream stages; then
// the LDS budget of the alpha-beta kernel, tuned on its stage); all produce
// the same sigma up to summation order.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace sbd {

hipError_t launch_fill_pattern(void* p, int64_t n, int prec, hipStream_t st);

namespace {
using Key = std::tuple<int64_t, int64_t, int, int, int, int>;
std::mutex g_mu;
std::map<Key, SigmaTune> g_cache;
}  // namespace

// Row-stream shapes: lane loads of 8 or 16 bytes, each with one row per
// wavefront, two rows per wavefront, or one row with 2 or 4 ket entries per
// load step.  The alpha-beta LDS budget is tuned separately.
std::vector<SigmaTune> stream_candidates() {
    std::vector<SigmaTune> out;
    for (int wide : {0, 1})
        for (int shape : {0, 1, 2, 3}) {
            SigmaTune t;
            t.stream_wide = wide;
            t.stream_rw = shape == 1 ? 2 : 1;
            t.stream_split = shape == 2 ? 2 : (shape == 3 ? 4 : 1);
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
    if (H->csr_has[prec == SBD_FP64 ? 0 : 1]) {  // assembled: the CSR product has nothing to tune
        if (best_ms) *best_ms = -1.0;
        return SBD_OK;
    }
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
    const SigmaTune saved = H->tune[prec];
    SigmaTune best = saved;
    // mean time of the stages [s0, s1) over three sigmas after a warm-up (ev:
    // the six stage boundaries of the first vector); s0 < 0: the whole call
    hipEvent_t ev[6];
    int nev = 0;
    for (; nev < 6; ++nev)
        if (hipEventCreate(&ev[nev]) != hipSuccess) break;
    auto timed = [&](int s0, int s1, float* ms) -> int {
        if (nev < 6) return hip_fail(hipErrorOutOfMemory, "autotune events");
        int r = sigma_internal(x, H, nvec, prec, 0.0, cbuf.p, ybuf.p, layout, ws.p, st);
        if (s0 < 0) {
            hipError_t e = r ? hipSuccess : hipEventRecord(ev[0], st);
            for (int rep = 0; rep < 3 && !r && e == hipSuccess; ++rep)
                r = sigma_internal(x, H, nvec, prec, 0.0, cbuf.p, ybuf.p, layout, ws.p, st);
            if (!r && e == hipSuccess) e = hipEventRecord(ev[1], st);
            if (!r && e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float t = 0.f;
            if (!r && e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
            if (!r && e != hipSuccess) r = hip_fail(e, "autotune timing");
            *ms = t / 3.f;
            return r;
        }
        float tot = 0.f;
        for (int rep = 0; rep < 3 && !r; ++rep) {
            r = sigma_internal(x, H, nvec, prec, 0.0, cbuf.p, ybuf.p, layout, ws.p, st, ev);
            hipError_t e = r ? hipSuccess : hipEventSynchronize(ev[5]);
            float t = 0.f;
            if (!r && e == hipSuccess) e = hipEventElapsedTime(&t, ev[s0], ev[s1]);
            if (!r && e != hipSuccess) r = hip_fail(e, "autotune timing");
            tot += t;
        }
        *ms = tot / 3.f;
        return r;
    };
    int rc = SBD_OK;
    // 1. the row-stream shape: alpha and beta streams (stages 1 and 2)
    float best_stream = 1e30f;
    for (const SigmaTune& cand : stream_candidates()) {
        SigmaTune t = saved;
        t.stream_wide = cand.stream_wide;
        t.stream_rw = cand.stream_rw;
        t.stream_split = cand.stream_split;
        H->tune[prec] = t;
        float ms = 0.f;
        rc = timed(1, 3, &ms);
        if (rc) break;
        if (ms < best_stream) {
            best_stream = ms;
            best = t;
        }
    }
    // 2. the alpha-beta LDS budget (stage 3), then the whole sigma of the winner
    float best_t = 1e30f;
    if (!rc) {
        float best_ab = 1e30f;
        SigmaTune pick = best;
        for (int lds : {49152, 98304, 147456}) {
            SigmaTune t = best;
            t.ab_lds_bytes = lds;
            H->tune[prec] = t;
            float ms = 0.f;
            rc = timed(3, 4, &ms);
            if (rc) break;
            if (ms < best_ab) {
                best_ab = ms;
                pick = t;
            }
        }
        best = pick;
        H->tune[prec] = best;
        if (!rc) rc = timed(-1, 0, &best_t);
    }
    for (int i = 0; i < nev; ++i) (void)hipEventDestroy(ev[i]);
    if (rc) {
        H->tune[prec] = saved;
        return rc;
    }
    H->tune[prec] = best;
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_cache[key] = best;
    }
    if (best_ms) *best_ms = best_t;
    return SBD_OK;
}

extern "C" int sbd_get_tune(const sbd_ham* H, int prec, int* stream_rw, int* ab_lds_bytes,
                            int* stream_wide, int* stream_split) {
    if (!H || (prec != SBD_FP64 && prec != SBD_FP32)) return fail(SBD_ERR_ARG, "bad argument");
    if (stream_rw) *stream_rw = H->tune[prec].stream_rw;
    if (ab_lds_bytes) *ab_lds_bytes = H->tune[prec].ab_lds_bytes;
    if (stream_wide) *stream_wide = H->tune[prec].stream_wide;
    if (stream_split) *stream_split = H->tune[prec].stream_split;
    return SBD_OK;
}

extern "C" int sbd_set_tune(sbd_ham* H, int prec, int stream_rw, int ab_lds_bytes, int stream_wide,
                            int stream_split) {
    if (!H || (prec != SBD_FP64 && prec != SBD_FP32)) return fail(SBD_ERR_ARG, "bad argument");
    if (stream_rw != 1 && stream_rw != 2) return fail(SBD_ERR_ARG, "stream_rw must be 1 or 2");
    if (ab_lds_bytes < 4096 || ab_lds_bytes > (1 << 20)) return fail(SBD_ERR_ARG, "bad LDS budget");
    if (stream_wide != 0 && stream_wide != 1) return fail(SBD_ERR_ARG, "stream_wide must be 0 or 1");
    if (stream_split != 1 && stream_split != 2 && stream_split != 4)
        return fail(SBD_ERR_ARG, "stream_split must be 1, 2 or 4");
    if (stream_split > 1 && stream_rw != 1) return fail(SBD_ERR_ARG, "stream_split > 1 needs stream_rw = 1");
    H->tune[prec].stream_rw = stream_rw;
    H->tune[prec].ab_lds_bytes = ab_lds_bytes;
    H->tune[prec].stream_wide = stream_wide;
    H->tune[prec].stream_split = stream_split;
    return SBD_OK;
}
