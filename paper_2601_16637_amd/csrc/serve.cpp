// Serving loop: continuous batching of whole selected-basis solves.
//
// One request is one SQD iteration's classical step: basis, excitation
// tables, Hamiltonian and Davidson (Sec. II).  The server owns one device slab
// (the HBM budget) and a pool of worker threads, each driving its own HIP
// stream.  Requests queue in arrival order; the head is admitted as soon as a
// worker is idle and a contiguous region of its estimated size is free in the
// slab.  When the head does not fit the free slab space, a later request that
// fits may pass it, but the head is passed at most kMaxBypass times, so a
// large request cannot be starved by a stream of small ones.  The worker installs the region as the thread's allocation arena, so
// every device buffer of the request is carved from it (no hipMalloc/hipFree
// on the serving path: hipFree would synchronise the whole device and stall
// the other requests), runs the solve on its stream, synchronises that stream,
// and returns the region.  Several requests thus overlap on the device with
// their vectors resident, and each one's result is independent of the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>

#include "internal.h"

namespace sbd {
namespace {
thread_local Region* tl_region = nullptr;
}
Region* current_region() { return tl_region; }
}  // namespace sbd

using namespace sbd;

namespace {

using clk = std::chrono::steady_clock;
constexpr size_t kRegionAlign = size_t(2) << 20;  // 2 MiB: keeps the slab's free list short
constexpr int kMaxBypass = 64;  // later requests that may be admitted past a head that does not fit

double ms_between(clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

struct Job {
    uint64_t ticket = 0;
    sbd_request req{};
    std::vector<uint64_t> A, B;
    std::vector<double> h, eri;
    size_t est = 0;
    int bypassed = 0;  // later requests admitted while this one waited at the head
    clk::time_point t_submit;
};

}  // namespace

struct sbd_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job*> queue;
    std::map<uint64_t, sbd_result> done;
    std::map<uint64_t, bool> known;  // submitted and not yet waited for
    char* slab = nullptr;
    size_t budget = 0;
    std::map<size_t, size_t> freel;  // free slab blocks: offset -> length
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    bool stop = false;
    int waiters = 0;  // threads inside sbd_serve_wait
    uint64_t next = 1;
    int device = 0;
    clk::time_point t0 = clk::now();
};

namespace {

// first fit; caller holds the lock
bool slab_take(sbd_server* s, size_t n, size_t* off) {
    for (auto it = s->freel.begin(); it != s->freel.end(); ++it) {
        if (it->second < n) continue;
        *off = it->first;
        const size_t rest = it->second - n, o2 = it->first + n;
        s->freel.erase(it);
        if (rest) s->freel[o2] = rest;
        return true;
    }
    return false;
}

void slab_give(sbd_server* s, size_t off, size_t n) {
    auto it = s->freel.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != s->freel.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        s->freel.erase(nx);
    }
    if (it != s->freel.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            s->freel.erase(it);
        }
    }
}

void run_job(const Job& j, hipStream_t st, sbd_result& r) {
    const sbd_request& q = j.req;
    sbd_basis* b = nullptr;
    sbd_exc* x = nullptr;
    sbd_ham* H = nullptr;
    int rc = sbd_build_basis(q.norb, q.n_alpha, q.n_beta, j.A.data(), (int64_t)j.A.size(),
                             j.B.data(), (int64_t)j.B.size(), st, &b);
    if (rc == SBD_OK) rc = sbd_build_excitations(b, st, &x);
    if (rc == SBD_OK) rc = sbd_set_hamiltonian(b, x, j.h.data(), j.eri.data(), q.e_core, st, &H);
    if (rc == SBD_OK) {
        int64_t na = 0, nb = 0;
        rc = sbd_basis_sizes(b, &na, &nb);
        r.ndet = na * nb;
    }
    if (rc == SBD_OK) rc = sbd_davidson(b, x, H, q.nroots, &q.opts, r.energies, nullptr, &r.report, st);
    r.status = rc;
    if (rc < 0) std::strncpy(r.message, sbd_last_error(), sizeof(r.message) - 1);
    sbd_free_ham(H);
    sbd_free_exc(x);
    sbd_free_basis(b);
}

// Next job to admit, with its slab offset; caller holds the lock.  The head
// if it fits; otherwise the first later job that fits, while the head has
// been passed fewer than kMaxBypass times.
bool admit(sbd_server* s, Job** out, size_t* off) {
    if (s->queue.empty()) return false;
    Job* head = s->queue.front();
    if (slab_take(s, head->est, off)) {
        s->queue.pop_front();
        *out = head;
        return true;
    }
    if (head->bypassed >= kMaxBypass) return false;
    for (auto it = std::next(s->queue.begin()); it != s->queue.end(); ++it) {
        if ((*it)->est > head->est || !slab_take(s, (*it)->est, off)) continue;
        *out = *it;
        s->queue.erase(it);
        ++head->bypassed;
        return true;
    }
    return false;
}

void worker(sbd_server* s, int w) {
    (void)hipSetDevice(s->device);
    hipStream_t st = s->streams[w];
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        size_t off = 0;
        Job* j = nullptr;
        s->cv_work.wait(lk, [&] {
            if (s->stop) return true;
            return admit(s, &j, &off);
        });
        if (s->stop) break;
        lk.unlock();

        sbd_result r;
        std::memset(&r, 0, sizeof(r));
        const auto t_admit = clk::now();
        Region reg;
        reg.base = s->slab + off;
        reg.size = j->est;
        tl_region = &reg;
        run_job(*j, st, r);
        const hipError_t e = hipStreamSynchronize(st);  // the region's buffers are idle after this
        tl_region = nullptr;
        if (e != hipSuccess && r.status >= 0) {
            r.status = SBD_ERR_HIP;
            std::strncpy(r.message, hipGetErrorString(e), sizeof(r.message) - 1);
        }
        const auto t_end = clk::now();
        r.queue_ms = ms_between(j->t_submit, t_admit);
        r.run_ms = ms_between(t_admit, t_end);
        r.latency_ms = ms_between(j->t_submit, t_end);
        r.admit_at_ms = ms_between(s->t0, t_admit);
        r.done_at_ms = ms_between(s->t0, t_end);
        r.region_bytes = j->est;
        r.peak_bytes = reg.peak;

        lk.lock();
        slab_give(s, off, j->est);
        s->done[j->ticket] = r;
        delete j;
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

}  // namespace

extern "C" int sbd_serve_estimate(const sbd_request* q, size_t* bytes) {
    if (!q || !bytes) return fail(SBD_ERR_ARG, "null argument");
    if (q->norb < 1 || q->norb > 64 || q->n_alpha_in < 1 || q->n_beta_in < 1 || q->nroots < 1 ||
        q->nroots > 8 || q->n_alpha < 0 || q->n_beta < 0 || q->n_alpha > q->norb || q->n_beta > q->norb)
        return fail(SBD_ERR_ARG, "bad request sizes");
    const double nin[2] = {(double)q->n_alpha_in, (double)q->n_beta_in};
    const int nel[2] = {q->n_alpha, q->n_beta};
    const double N = nin[0] * nin[1];
    const int norb = q->norb, k = q->nroots;
    const sbd_davidson_opts& o = q->opts;
    // Davidson workspace (csrc/davidson.cpp)
    double ms = std::min(std::max(o.max_space, 2 * k + 1), 48);
    ms = std::min(ms, N);
    const double keep = std::max<double>(k, std::min<double>(2 * k, ms - k));
    const bool mixed = o.sigma_prec == SBD_FP32;
    const double nvmax = (k < 2 || !o.block_sigma) ? 1 : (k <= 2 ? 2 : (k <= 4 ? 4 : 8));  // block width
    // device-driven iterations (when the solve can take them): spare rows of V and W, a
    // second collapse scratch, FP64 staging, the device state and its partial sums
    const bool dev = o.device_iterations > 0 && k <= kDlMaxRoots && N <= (double)kDlMaxN;
    const bool stage64 = nvmax > 1 || o.use_graph || dev;
    double total = 2 * (ms + (dev ? kDlMaxRoots : 0)) * N * 8 + std::max<double>(k, keep) * N * 8 +
                   keep * N * 8 * (dev ? 2 : 1) + 2 * N * nvmax * 8 + (stage64 ? 2 * nvmax * N * 8 : 0.0) +
                   (mixed ? 2 * std::max(ms, nvmax) * N * 4 : 0.0) + 8.0 * kPassRows * kRedBlocks +
                   (dev ? sizeof(DlState) + 8.0 * kDlBlocks * kDlMaxSpace * kDlMaxRoots +
                              8.0 * kDlMaxSpace * (kDlMaxSpace + 1)
                        : 0.0) +
                   65536.0;
    // Hamiltonian: integrals, diagonal, spectator tables and per-string diagonal parts
    const double np = norb * (norb + 1) / 2.0;
    total += 8.0 * norb * norb + 12.0 * std::pow((double)norb, 4) + 8 * N;
    for (int s = 0; s < 2; ++s) {
        const double ns = nin[s];
        const int n = nel[s];
        const double s1 = std::min(n * (double)(norb - n), ns - 1);
        const double s2 = std::min(binom(n, 2) * binom(norb - n, 2), ns - 1);
        total += np * ns * 12 + ns * 8;
        // tables: J, orbitals, sign, packed, sliced-ELL (64- and 32-bit) singles, coefficients,
        // row pointers, build temporaries; the basis sort's power-of-two scratch
        total += ns * (s1 * (4 + 4 + 1 + 8 + 16 + 8 + 12 + 4) + s2 * (4 + 4 + 1 + 12)) + 6 * (ns + 1) * 8;
        double p2 = 1;
        while (p2 < ns) p2 *= 2;
        total += p2 * 8 + ns * 8 + 64;
    }
    if (o.use_autotune) total += 4 * N * 8 + (mixed ? 4 * N * 4 : 0.0);
    total = total * 1.1 + (64 << 20);
    size_t b = (size_t)total;
    b = (b + kRegionAlign - 1) / kRegionAlign * kRegionAlign;
    *bytes = b;
    return SBD_OK;
}

extern "C" int sbd_serve_create(size_t budget, int max_inflight, sbd_server** out) {
    if (!out || budget < kRegionAlign || max_inflight < 1 || max_inflight > 64)
        return fail(SBD_ERR_ARG, "bad server arguments");
    *out = nullptr;
    auto* s = new sbd_server();
    s->budget = budget / kRegionAlign * kRegionAlign;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipMalloc((void**)&s->slab, s->budget);
    if (e != hipSuccess) {
        delete s;
        return e == hipErrorOutOfMemory ? fail(SBD_ERR_NOMEM, "serving slab") : hip_fail(e, "serving slab");
    }
    s->freel[0] = s->budget;
    for (int w = 0; w < max_inflight; ++w) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) break;
        s->streams.push_back(st);
    }
    if (e != hipSuccess) {
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        (void)hipFree(s->slab);
        delete s;
        return hip_fail(e, "serving streams");
    }
    for (int w = 0; w < max_inflight; ++w) s->workers.emplace_back(worker, s, w);
    *out = s;
    return SBD_OK;
}

extern "C" int sbd_serve_submit(sbd_server* s, const sbd_request* q, uint64_t* ticket) {
    if (!s || !q || !ticket || !q->alpha_strings || !q->beta_strings || !q->h1 || !q->eri)
        return fail(SBD_ERR_ARG, "null argument");
    if (q->opts.guess || q->opts.n_guess) return fail(SBD_ERR_ARG, "serving requests take no guess");
    size_t est = 0;
    int rc = sbd_serve_estimate(q, &est);
    if (rc) return rc;
    if (est > s->budget) return fail(SBD_ERR_NOMEM, "request larger than the serving budget");
    auto* j = new Job();
    j->req = *q;
    j->A.assign(q->alpha_strings, q->alpha_strings + q->n_alpha_in);
    j->B.assign(q->beta_strings, q->beta_strings + q->n_beta_in);
    const size_t n2 = (size_t)q->norb * q->norb;
    j->h.assign(q->h1, q->h1 + n2);
    j->eri.assign(q->eri, q->eri + n2 * n2);
    j->req.alpha_strings = j->req.beta_strings = nullptr;
    j->req.h1 = j->req.eri = nullptr;
    j->est = est;
    j->t_submit = clk::now();
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) {
            delete j;
            return fail(SBD_ERR_STATE, "server is stopping");
        }
        j->ticket = s->next++;
        *ticket = j->ticket;
        s->known[j->ticket] = true;
        s->queue.push_back(j);
    }
    s->cv_work.notify_all();
    return SBD_OK;
}

extern "C" int sbd_serve_wait(sbd_server* s, uint64_t ticket, sbd_result* out) {
    if (!s || !out) return fail(SBD_ERR_ARG, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return fail(SBD_ERR_ARG, "unknown ticket");
    ++s->waiters;
    s->cv_done.wait(lk, [&] { return s->done.count(ticket) > 0; });
    *out = s->done[ticket];
    s->done.erase(ticket);
    s->known.erase(ticket);
    --s->waiters;
    s->cv_done.notify_all();  // sbd_serve_destroy may be waiting for the last waiter to leave
    return SBD_OK;
}

extern "C" void sbd_serve_destroy(sbd_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        // queued requests fail: their waiters (if any) get SBD_ERR_STATE
        for (Job* j : s->queue) {
            sbd_result r;
            std::memset(&r, 0, sizeof(r));
            r.status = SBD_ERR_STATE;
            std::strncpy(r.message, "server destroyed before the request was admitted",
                         sizeof(r.message) - 1);
            r.queue_ms = r.latency_ms = ms_between(j->t_submit, clk::now());
            s->done[j->ticket] = r;
            delete j;
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    for (auto& t : s->workers) t.join();  // running requests finish and post their results
    {
        // threads blocked in sbd_serve_wait hold the server: let them take their results first
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->waiters == 0; });
    }
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    (void)hipFree(s->slab);
    delete s;
}
