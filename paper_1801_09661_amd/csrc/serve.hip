// Request loop of the C ABI (oem_server_*): worker threads, one stream and
// one reusable handle each, admission of queued requests by device bytes in
// arrival order, completions with timestamps.  Every request runs the same
// entry points as a direct caller would (oem_gram, oem_fit_path, oem_cv);
// the workers only move data and keep several requests in flight.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>

#include "oem_internal.h"

using namespace oem;

namespace {

struct Pending {
    oem_request r;
    int64_t bytes;
    double t_arrival;
};

} // namespace

struct oem_server_s {
    int device = 0;
    int32_t prec = OEM_FP64;
    oem_path_opts opts{};
    int64_t budget = 0;
    int nslots = 1;
    int64_t in_use = 0;
    int running = 0;
    bool stop = false;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> pending;
    std::deque<oem_completion> done;
    std::vector<std::thread> workers;
};

namespace {

double now_s()
{
    using clk = std::chrono::steady_clock;
    static const clk::time_point t0 = clk::now();
    return std::chrono::duration<double>(clk::now() - t0).count();
}

bool is_device_ptr(const void *p)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();   // plain host memory the runtime does not know
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Device bytes a request holds while in flight: staged X and y, per-fold and
// derived Grams, path outputs and the Lanczos workspace.
int64_t request_bytes(const oem_request &r, int L)
{
    const int64_t p = r.p, K = r.nfolds, nq = K == 1 ? 1 : K + 1;
    int64_t b = r.n * r.p * 4 + r.n * 8;
    b += (K + 2 * nq) * p * p * 8;
    b += nq * (int64_t)L * (p + 4) * 8;
    if (p > 128) b += nq * (int64_t)(std::min<int64_t>(p, 1024) + 1) * p * 8;
    return b;
}

struct Worker {
    oem_gram_s *h = nullptr;
    hipStream_t st = nullptr;
    DevBuf xbuf, ybuf, outb;
    std::vector<int32_t> it_host;
};

int run_request(oem_server_s *S, Worker &W, const oem_request &r)
{
    hipStream_t st = W.st;
    const int L = S->opts.nlambda, K = r.nfolds, nq = K == 1 ? 1 : K + 1;
    const float *Xd = r.X;
    const double *yd = r.y;
    int64_t ldx = r.ldx;
    if (!is_device_ptr(r.X)) {
        // host rows: only the p used columns cross the bus (a 2-D copy when
        // the rows are strided), into a dense device block
        const size_t row = (size_t)r.p * sizeof(float);
        int rc = W.xbuf.ensure((size_t)r.n * row);
        if (rc) return rc;
        if (r.ldx == r.p)
            OEM_HIP_CHECK(hipMemcpyAsync(W.xbuf.ptr, r.X, (size_t)r.n * row, hipMemcpyHostToDevice, st));
        else
            OEM_HIP_CHECK(hipMemcpy2DAsync(W.xbuf.ptr, row, r.X, (size_t)r.ldx * sizeof(float), row, (size_t)r.n,
                                           hipMemcpyHostToDevice, st));
        Xd = W.xbuf.as<float>();
        ldx = r.p;
    }
    if (!is_device_ptr(r.y)) {
        int rc = W.ybuf.ensure((size_t)r.n * sizeof(double));
        if (rc) return rc;
        OEM_HIP_CHECK(hipMemcpyAsync(W.ybuf.ptr, r.y, (size_t)r.n * sizeof(double), hipMemcpyHostToDevice, st));
        yd = W.ybuf.as<double>();
    }
    int rc = handle_reconfigure(W.h, r.p, K, S->prec, OEM_X_F32, r.fold_seed, st);
    if (rc) return rc;
    rc = oem_gram(W.h, Xd, r.n, ldx, yd, 0, nullptr, st);
    if (rc) return rc;
    // device outputs: beta (K + 1) x L x p, lambda L, cvm, cvsd L, iters (K + 1) x L, small ints
    const size_t nb = (size_t)nq * L * r.p, nl = (size_t)L;
    rc = W.outb.ensure((nb + 3 * nl) * sizeof(double) + ((size_t)nq * L + 8) * sizeof(int32_t) + 64);
    if (rc) return rc;
    double *beta = W.outb.as<double>();
    double *lam = beta + nb;
    double *cvm = lam + nl;
    double *cvsd = cvm + nl;
    int32_t *iters = reinterpret_cast<int32_t *>(cvsd + nl);
    int32_t *small = iters + (size_t)nq * L;
    oem_path_opts o = S->opts;
    o.groups = r.groups;
    o.sync = 0;
    if (K == 1) {
        rc = oem_fit_path(W.h, -1, &r.pen, 1, &o, beta, lam, iters, nullptr, nullptr, nullptr, st);
    } else {
        rc = oem_cv(W.h, &r.pen, 1, &o, beta, beta + (size_t)L * r.p, lam, cvm, cvsd, small, small + 1,
                    small + 2, iters, st);
    }
    if (rc < 0) return rc;
    OEM_HIP_CHECK(hipMemcpyAsync(r.beta, beta, (size_t)L * r.p * sizeof(double), hipMemcpyDeviceToHost, st));
    if (r.lambda) OEM_HIP_CHECK(hipMemcpyAsync(r.lambda, lam, nl * sizeof(double), hipMemcpyDeviceToHost, st));
    if (K > 1 && r.cvm) OEM_HIP_CHECK(hipMemcpyAsync(r.cvm, cvm, nl * sizeof(double), hipMemcpyDeviceToHost, st));
    if (K > 1 && r.i_min) OEM_HIP_CHECK(hipMemcpyAsync(r.i_min, small, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    W.it_host.resize((size_t)nq * L);
    OEM_HIP_CHECK(hipMemcpyAsync(W.it_host.data(), iters, W.it_host.size() * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, st));
    OEM_HIP_CHECK(hipStreamSynchronize(st));
    for (int32_t v : W.it_host)
        if (v < 0) return OEM_NOT_CONVERGED;
    return OEM_OK;
}

void worker_main(oem_server_s *S, int slot)
{
    (void)hipSetDevice(S->device);
    oem::lanczos_single_workgroup = true;   // several workers run on the GPU at once
    // buffers that a request outgrows are freed only between requests, once
    // they add up to a quarter of this worker's share of the byte budget:
    // each hipFree waits for every worker's kernels
    oem::DeferredFrees held;
    oem::deferred_frees = &held;
    const size_t share = (size_t)(S->budget / S->nslots);
    const size_t held_cap = share / 4;
    Worker W;
    W.h = new oem_gram_s();
    W.h->device = S->device;
    const bool ok = hipStreamCreateWithFlags(&W.st, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
        Pending job;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] {
                if (S->pending.empty()) return S->stop;
                const Pending &h = S->pending.front();
                return S->in_use == 0 || S->in_use + h.bytes <= S->budget;
            });
            if (S->pending.empty()) break;   // stop requested and nothing queued
            job = S->pending.front();
            S->pending.pop_front();
            S->in_use += job.bytes;
            ++S->running;
        }
        if (held.bytes > held_cap) oem::flush_deferred_frees(held);
        const double t_admit = now_s();
        const int status = ok ? run_request(S, W, job.r) : OEM_E_HIP;
        const double t_done = now_s();
        // an idle worker's staging of X, y and the outputs stays within its
        // share of the budget
        if (W.xbuf.bytes + W.ybuf.bytes + W.outb.bytes > share)
            for (DevBuf *b : {&W.xbuf, &W.ybuf, &W.outb}) b->release();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->in_use -= job.bytes;
            --S->running;
            S->done.push_back(oem_completion{job.r.id, status, slot, job.t_arrival, t_admit, t_done, job.bytes});
        }
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
    if (W.st) (void)hipStreamSynchronize(W.st);
    oem::deferred_frees = nullptr;
    oem::flush_deferred_frees(held);
    for (DevBuf *b : {&W.xbuf, &W.ybuf, &W.outb}) b->release();
    oem_gram_free(W.h);
    if (W.st) (void)hipStreamDestroy(W.st);
}

} // namespace

extern "C" {

double oem_server_now(void) { return now_s(); }

int oem_server_create(int32_t nslots, int64_t device_bytes, int32_t precision,
                      const oem_path_opts *opts, oem_server *out)
{
    if (!out) return fail(OEM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (nslots < 1 || nslots > 16) return fail(OEM_E_INVAL, "nslots must be in [1, 16]");
    if (device_bytes < 1) return fail(OEM_E_INVAL, "device_bytes must be >= 1");
    if (precision != OEM_FP64 && precision != OEM_SPLIT_BF16 && precision != OEM_BF16)
        return fail(OEM_E_INVAL, "unknown precision");
    if (!opts || opts->nlambda < 1 || opts->maxit < 1 || !(opts->tol >= 0.0) ||
        !(opts->lambda_min_ratio > 0.0 && opts->lambda_min_ratio <= 1.0))
        return fail(OEM_E_INVAL, "bad path options");
    if (opts->intercept || opts->beta0) return fail(OEM_E_INVAL, "server options take no intercept");
    if (opts->lambda || opts->groups || opts->w || opts->cg)
        return fail(OEM_E_INVAL, "server options take no lambda, groups or weights");
    oem_server_s *S = new oem_server_s();
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return fail(OEM_E_HIP, "hipGetDevice failed");
    }
    (void)now_s();
    S->prec = precision;
    S->opts = *opts;
    S->budget = device_bytes;
    S->nslots = nslots;
    for (int i = 0; i < nslots; ++i) S->workers.emplace_back(worker_main, S, i);
    *out = S;
    return OEM_OK;
}

int oem_server_submit(oem_server S, const oem_request *req)
{
    if (!S || !req) return fail(OEM_E_INVAL, "server or request is NULL");
    const oem_request &r = *req;
    if (r.p < 1 || r.p > 4096 || r.n < 1 || r.n > INT32_MAX || r.ldx < r.p || !r.X || !r.y || !r.beta)
        return fail(OEM_E_INVAL, "request: bad p, n, ldx or pointer");
    if (r.nfolds < 1 || r.nfolds > 64) return fail(OEM_E_INVAL, "request: nfolds must be in [1, 64]");
    if (group_penalty(r.pen.kind) && !r.groups) return fail(OEM_E_INVAL, "request: group penalty without groups");
    Pending job{r, request_bytes(r, S->opts.nlambda), r.t_arrival >= 0.0 ? r.t_arrival : now_s()};
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return fail(OEM_E_STATE, "server is stopping");
        S->pending.push_back(job);
    }
    S->cv_work.notify_all();
    return OEM_OK;
}

int oem_server_poll(oem_server S, oem_completion *out, int32_t max, int32_t *count, int32_t wait)
{
    if (!S || !out || !count || max < 1) return fail(OEM_E_INVAL, "bad poll arguments");
    std::unique_lock<std::mutex> lk(S->mu);
    if (wait)
        S->cv_done.wait(lk, [&] { return !S->done.empty() || (S->pending.empty() && S->running == 0); });
    int32_t k = 0;
    while (k < max && !S->done.empty()) {
        out[k++] = S->done.front();
        S->done.pop_front();
    }
    *count = k;
    return OEM_OK;
}

int oem_server_drain(oem_server S)
{
    if (!S) return fail(OEM_E_INVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->pending.empty() && S->running == 0; });
    return OEM_OK;
}

void oem_server_free(oem_server S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (std::thread &t : S->workers) t.join();
    delete S;
}

} // extern "C"
