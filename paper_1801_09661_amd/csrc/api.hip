// C ABI of liboem (declared in include/oem.h): argument checks, device
// buffer management and the order of kernel launches.  No arithmetic of the
// method happens here; every step runs in the kernels of gram.hip,
// derive.hip and path.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

#include "gram_common.h"
#include "oem_internal.h"

namespace oem {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

int DevBuf::ensure(size_t need)
{
    if (need <= bytes && ptr) return OEM_OK;
    release();
    if (need == 0) need = 8;
    bool ok = hipMalloc(&ptr, need) == hipSuccess;
    if (!ok && deferred_frees && !deferred_frees->ptrs.empty()) {
        // the held-back frees may be what is missing
        (void)hipGetLastError();
        flush_deferred_frees(*deferred_frees);
        ok = hipMalloc(&ptr, need) == hipSuccess;
    }
    if (!ok) {
        ptr = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        return fail(OEM_E_NOMEM, "device allocation of " + std::to_string(need) + " bytes failed");
    }
    bytes = need;
    return OEM_OK;
}

thread_local DeferredFrees *deferred_frees = nullptr;

void DevBuf::release()
{
    if (ptr) {
        if (deferred_frees) {
            deferred_frees->ptrs.push_back(ptr);
            deferred_frees->bytes += bytes;
        } else {
            (void)hipFree(ptr);
        }
    }
    ptr = nullptr;
    bytes = 0;
}

void flush_deferred_frees(DeferredFrees &d)
{
    for (void *q : d.ptrs) (void)hipFree(q);
    d.ptrs.clear();
    d.bytes = 0;
}

static inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

static int num_problems(const oem_gram_s *h) { return h->K == 1 ? 1 : h->K + 1; }

// Group structure of one fit: CSR member lists (ascending variable index
// within each group), weights; all in one device buffer.
struct GroupPlan {
    int ngroups = 0;
    std::vector<int32_t> gstart, gidx;
    std::vector<double> w, cg;
    const int32_t *d_gstart = nullptr, *d_gidx = nullptr;
    const double *d_w = nullptr, *d_cg = nullptr;
};

static int build_groups(oem_gram_s *h, const oem_path_opts *o, bool need_groups, GroupPlan &gp,
                        hipStream_t s)
{
    const int p = h->p;
    if (o->groups) {
        int ng = 0;
        for (int j = 0; j < p; ++j) {
            if (o->groups[j] < 0) return fail(OEM_E_INVAL, "negative group id");
            ng = std::max(ng, o->groups[j] + 1);
        }
        gp.ngroups = ng;
        std::vector<int32_t> cnt(ng + 1, 0);
        for (int j = 0; j < p; ++j) cnt[o->groups[j] + 1]++;
        for (int g = 0; g < ng; ++g)
            if (cnt[g + 1] == 0) return fail(OEM_E_INVAL, "group ids must use every id in [0, ngroups)");
        gp.gstart.assign(ng + 1, 0);
        for (int g = 0; g < ng; ++g) gp.gstart[g + 1] = gp.gstart[g] + cnt[g + 1];
        gp.gidx.assign(p, 0);
        std::vector<int32_t> fill(ng, 0);
        for (int j = 0; j < p; ++j) {
            const int g = o->groups[j];
            gp.gidx[gp.gstart[g] + fill[g]++] = j;
        }
        gp.cg.resize(ng);
        for (int g = 0; g < ng; ++g) {
            const double c = o->cg ? o->cg[g] : std::sqrt((double)(gp.gstart[g + 1] - gp.gstart[g]));
            if (!(c > 0.0)) return fail(OEM_E_INVAL, "group weights must be > 0");
            gp.cg[g] = c;
        }
    } else if (need_groups) {
        return fail(OEM_E_INVAL, "a group penalty needs opts->groups");
    }
    if (o->w) {
        gp.w.assign(o->w, o->w + p);
        for (double v : gp.w)
            if (!(v >= 0.0)) return fail(OEM_E_INVAL, "variable weights must be >= 0");
    }
    const size_t bytes = (gp.gstart.size() + gp.gidx.size()) * sizeof(int32_t) + 16 +
                         (gp.w.size() + gp.cg.size()) * sizeof(double);
    int rc = h->groupbuf.ensure(bytes);
    if (rc) return rc;
    std::vector<char> host(bytes, 0);
    size_t off = 0;
    auto put = [&](const void *src, size_t nb) {
        size_t at = off;
        if (nb) std::memcpy(host.data() + at, src, nb);
        off += nb;
        off = (off + 7) & ~size_t(7);
        return at;
    };
    const size_t o_gs = put(gp.gstart.data(), gp.gstart.size() * sizeof(int32_t));
    const size_t o_gi = put(gp.gidx.data(), gp.gidx.size() * sizeof(int32_t));
    const size_t o_w = put(gp.w.data(), gp.w.size() * sizeof(double));
    const size_t o_cg = put(gp.cg.data(), gp.cg.size() * sizeof(double));
    rc = stage_upload(h, kUpGroups, h->groupbuf.ptr, host.data(), bytes, s);
    if (rc) return rc;
    char *base = static_cast<char *>(h->groupbuf.ptr);
    if (!gp.gstart.empty()) {
        gp.d_gstart = reinterpret_cast<const int32_t *>(base + o_gs);
        gp.d_gidx = reinterpret_cast<const int32_t *>(base + o_gi);
        gp.d_cg = reinterpret_cast<const double *>(base + o_cg);
    }
    if (!gp.w.empty()) gp.d_w = reinterpret_cast<const double *>(base + o_w);
    return OEM_OK;
}

// Combine, standardise and compute d for every problem, once per change of
// the accumulated statistics; copies d and the row counts to the host.
static int ensure_derived(oem_gram_s *h, int standardize, int intercept, hipStream_t s)
{
    if (h->derived_valid && h->derived_std == standardize && h->derived_icpt == intercept) return OEM_OK;
    if (h->rows_seen <= 0) return fail(OEM_E_STATE, "no rows accumulated");
    if (intercept && !h->colsums_known)
        return fail(OEM_E_STATE, "an intercept needs the column sums, which imported statistics lack");
    int rc = launch_combine(h, standardize, intercept, s);
    if (rc) return rc;
    rc = launch_lanczos(h, s);
    if (rc) return rc;
    const int nq = num_problems(h);
    h->d_host.assign(nq, 0.0);
    h->n_host.assign(nq, 0);
    h->lz_host.assign(nq, 0);
    OEM_HIP_CHECK(hipMemcpyAsync(h->d_host.data(), h->dq.ptr, nq * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
    OEM_HIP_CHECK(hipMemcpyAsync(h->n_host.data(), h->ntrain.ptr, nq * sizeof(int64_t),
                                 hipMemcpyDeviceToHost, s));
    OEM_HIP_CHECK(hipMemcpyAsync(h->lz_host.data(), h->lzsteps.ptr, nq * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, s));
    OEM_HIP_CHECK(hipStreamSynchronize(s));
    // d must be a finite positive upper bound of lambda_1 for the iteration
    // to be defined (Section 2.1).  A negative step count with a finite d is
    // the documented fallback (Lanczos did not settle: d is a Gershgorin
    // bound, still >= lambda_1).
    for (int q = 0; q < nq; ++q) {
        if (h->lz_host[q] == kLanczosTimedOut)
            return fail(OEM_E_HIP, "eigenvalue bound of problem " + std::to_string(q) +
                                       ": the multi-workgroup Lanczos timed out waiting for its workgroups");
        if (h->n_host[q] > 0 && !(std::isfinite(h->d_host[q]) && h->d_host[q] > 0.0))
            return fail(OEM_E_INVAL, "eigenvalue bound d of problem " + std::to_string(q) +
                                         " is not a finite positive number (non-finite or all-zero statistics)");
    }
    h->derived_valid = true;
    h->derived_std = standardize;
    h->derived_icpt = intercept;
    return OEM_OK;
}

static int check_opts(const oem_path_opts *o)
{
    if (!o) return fail(OEM_E_INVAL, "opts is NULL");
    if (o->nlambda < 1) return fail(OEM_E_INVAL, "nlambda must be >= 1");
    if (o->maxit < 1) return fail(OEM_E_INVAL, "maxit must be >= 1");
    if (!(o->tol >= 0.0)) return fail(OEM_E_INVAL, "tol must be >= 0");
    if (o->intercept != 0 && o->intercept != 1) return fail(OEM_E_INVAL, "intercept must be 0 or 1");
    if (!o->lambda && !(o->lambda_min_ratio > 0.0 && o->lambda_min_ratio <= 1.0))
        return fail(OEM_E_INVAL, "lambda_min_ratio must be in (0, 1]");
    return OEM_OK;
}

static int check_penalty(const oem_penalty &pn, double d)
{
    switch (pn.kind) {
    case OEM_LASSO:
    case OEM_GRP_LASSO:
        break;
    case OEM_ENET:
        if (!(pn.alpha > 0.0 && pn.alpha <= 1.0)) return fail(OEM_E_INVAL, "elastic net alpha must be in (0, 1]");
        break;
    case OEM_MCP:
    case OEM_GRP_MCP:
        if (!(pn.gamma > 1.0)) return fail(OEM_E_INVAL, "MCP needs gamma > 1");
        if (!(pn.gamma * d > 1.0)) return fail(OEM_E_INVAL, "MCP needs gamma * d > 1");
        break;
    case OEM_SCAD:
    case OEM_GRP_SCAD:
        if (!(pn.gamma > 2.0)) return fail(OEM_E_INVAL, "SCAD needs gamma > 2");
        if (!((pn.gamma - 1.0) * d > 1.0)) return fail(OEM_E_INVAL, "SCAD needs (gamma - 1) d > 1");
        break;
    case OEM_SGL:
        if (!(pn.tau >= 0.0 && pn.tau <= 1.0)) return fail(OEM_E_INVAL, "sparse group lasso tau must be in [0, 1]");
        return OEM_OK;
    default:
        return fail(OEM_E_INVAL, "unknown penalty kind");
    }
    if (pn.tau != 0.0) return fail(OEM_E_INVAL, "penalty tau applies to the sparse group lasso only and must be 0");
    return OEM_OK;
}

// lambda sequences (npen x L) into h->lam: explicit, or grids from the
// full-data problem's standardised X^T y.
static int prepare_lambda(oem_gram_s *h, const oem_penalty *pen, int npen,
                          const oem_path_opts *o, const GroupPlan &gp, hipStream_t s)
{
    const int L = o->nlambda;
    const size_t nl = (size_t)npen * L;
    int rc = h->lam.ensure(nl * sizeof(double) + npen * sizeof(oem_penalty) + 64);
    if (rc) return rc;
    double *dl = h->lam.as<double>();
    if (o->lambda) {
        for (size_t i = 0; i < nl; ++i)
            if (!(o->lambda[i] >= 0.0)) return fail(OEM_E_INVAL, "lambda values must be >= 0");
        return stage_upload(h, kUpLambda, dl, o->lambda, nl * sizeof(double), s);
    }
    oem_penalty *dpen = reinterpret_cast<oem_penalty *>(dl + nl);
    rc = stage_upload(h, kUpLambda, dpen, pen, npen * sizeof(oem_penalty), s);
    if (rc) return rc;
    return launch_lambda_grid(h->cs.as<double>(), h->p, gp.d_gstart, gp.d_gidx, gp.ngroups, gp.d_w,
                              gp.d_cg, dpen, npen, L, o->lambda_min_ratio, dl, s);
}

static PathDesc make_desc(oem_gram_s *h, int q, const oem_penalty &pn, const oem_path_opts *o,
                          const GroupPlan &gp, const double *lam, double *beta, int32_t *iters,
                          double *kkt, double *obj)
{
    const size_t pp = (size_t)h->p * h->p;
    PathDesc d{};
    d.G = h->Gs.as<double>() + q * pp;
    d.c = h->cs.as<double>() + (size_t)q * h->p;
    d.s = h->sc.as<double>() + (size_t)q * h->p;
    d.yyn = h->yyn.as<double>() + q;
    d.d = h->dq.as<double>() + q;
    d.lambda = lam;
    d.beta = beta;
    d.beta_std = nullptr;
    d.lstart = nullptr;
    d.bws = nullptr;
    d.iters = iters;
    d.kkt = kkt;
    d.obj = obj;
    d.gstart = gp.d_gstart;
    d.gidx = gp.d_gidx;
    d.w = gp.d_w;
    d.cg = gp.d_cg;
    d.p = h->p;
    d.L = o->nlambda;
    d.kind = pn.kind;
    d.ngroups = gp.ngroups;
    d.alpha = pn.alpha;
    d.gamma = pn.gamma;
    d.tau = pn.tau;
    d.tol = o->tol;
    d.maxit = o->maxit;
    d.xbar = h->xbar.as<double>() + (size_t)q * h->p;
    d.ybar = h->ybar.as<double>() + q;
    d.beta0 = nullptr;
    return d;
}

int stage_upload(oem_gram_s *h, int slot, void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return OEM_OK;
    UploadStage &u = h->up;
    if (u.pending[slot]) {
        // the previous copy out of this slot has run before its bytes change
        OEM_HIP_CHECK(hipEventSynchronize(u.done[slot]));
        u.pending[slot] = false;
    }
    if (!u.done[slot]) OEM_HIP_CHECK(hipEventCreateWithFlags(&u.done[slot], hipEventDisableTiming));
    std::vector<char> &b = u.bytes[slot];
    b.assign(static_cast<const char *>(src), static_cast<const char *>(src) + bytes);
    OEM_HIP_CHECK(hipMemcpyAsync(dst, b.data(), bytes, hipMemcpyHostToDevice, s));
    OEM_HIP_CHECK(hipEventRecord(u.done[slot], s));
    u.pending[slot] = true;
    return OEM_OK;
}

void free_upload_stage(oem_gram_s *h)
{
    for (int k = 0; k < kUpSlots; ++k)
        if (h->up.done[k]) {
            (void)hipEventDestroy(h->up.done[k]);
            h->up.done[k] = nullptr;
            h->up.pending[k] = false;
        }
}

static int upload_descs(oem_gram_s *h, const std::vector<PathDesc> &descs, hipStream_t s)
{
    int rc = h->paths.ensure(descs.size() * sizeof(PathDesc));
    if (rc) return rc;
    return stage_upload(h, kUpDescs, h->paths.ptr, descs.data(), descs.size() * sizeof(PathDesc), s);
}

static int finish_sync(const int32_t *d_iters, size_t count, hipStream_t s)
{
    std::vector<int32_t> it(count);
    OEM_HIP_CHECK(hipMemcpyAsync(it.data(), d_iters, count * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    OEM_HIP_CHECK(hipStreamSynchronize(s));
    for (int32_t v : it)
        if (v < 0) {
            set_error("some lambda reached maxit before the convergence test held");
            return OEM_NOT_CONVERGED;
        }
    return OEM_OK;
}

// Give a handle new dimensions (buffers only grow) and clear its sums.
int handle_reconfigure(oem_gram_s *h, int32_t p, int32_t K, int32_t prec, int32_t xdt, uint64_t seed,
                       hipStream_t s)
{
    h->p = p;
    h->K = K;
    h->prec = prec;
    h->xdt = xdt;
    h->seed = seed;
    const size_t pp = (size_t)p * p, nq = (K == 1) ? 1 : (size_t)K + 1;
    int rc = OEM_OK;
    rc = rc ? rc : h->Gk.ensure((size_t)K * pp * sizeof(double));
    rc = rc ? rc : h->bk.ensure((size_t)K * p * sizeof(double));
    rc = rc ? rc : h->yyk.ensure((size_t)K * sizeof(double));
    rc = rc ? rc : h->nk.ensure((size_t)K * sizeof(int64_t));
    rc = rc ? rc : h->csk.ensure((size_t)K * p * sizeof(double));
    rc = rc ? rc : h->ysk.ensure((size_t)K * sizeof(double));
    rc = rc ? rc : h->xbar.ensure(nq * p * sizeof(double));
    rc = rc ? rc : h->ybar.ensure(nq * sizeof(double));
    rc = rc ? rc : h->Gs.ensure(nq * pp * sizeof(double));
    rc = rc ? rc : h->cs.ensure(nq * p * sizeof(double));
    rc = rc ? rc : h->sc.ensure(nq * p * sizeof(double));
    rc = rc ? rc : h->yyn.ensure(nq * sizeof(double));
    rc = rc ? rc : h->dq.ensure(nq * sizeof(double));
    rc = rc ? rc : h->ntrain.ensure(nq * sizeof(int64_t));
    rc = rc ? rc : h->lzsteps.ensure(nq * sizeof(int32_t));
    if (rc) return rc;
    return oem_gram_reset(h, s);
}

// ------------------------------------------------------------------ static workspace
// Workspace of oem_gram_noalloc (row lists and partial sums of one pass):
// a file-scope device array, so that entry point allocates nothing.  Each
// device holds its own copy until the process ends.  In host code the
// array's name is not a device address: its address on a device comes from
// hipGetSymbolAddress, called once per device with that device current and
// kept below; only that address is passed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, char *> g_scratch_addr;

// Address of `scratch` on device `dev`, which must be the current device.
static int noalloc_scratch(int dev, char **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(OEM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = g_scratch_addr.emplace(dev, static_cast<char *>(ptr)).first;
    }
    *out = it->second;
    return OEM_OK;
}

} // namespace oem

struct oem_batch_s {
    std::vector<oem_problem> probs;
    std::vector<oem_gram_s *> hs;
    int32_t prec = OEM_FP64, xdt = OEM_X_F32, npen = 0;
    std::vector<oem_penalty> pens;
    oem_path_opts opts{};
    oem::DevBuf descs, order, jobs, iters_own, pathws;
    std::vector<oem::LzLaunch> lz;
    oem::PathPlan plan;
    std::vector<int32_t *> iters_of;   // per problem: where its iteration counts go
    std::vector<size_t> iters_len;     // and how many there are
    std::vector<oem::GroupPlan> groups;   // per problem (device copies in its handle)
    std::vector<char> explicit_lam;    // per problem: lambda_in given (no grid)
    std::vector<double *> beta_folds;  // per CV problem: fold coefficients
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace oem;

extern "C" {

const char *oem_last_error(void) { return g_last_error.c_str(); }

const char *oem_version(void) { return "oem-mi355x 0.1 (gfx950)"; }

int oem_gram_create(int32_t p, int32_t nfolds, int32_t precision, int32_t x_dtype,
                    uint64_t fold_seed, oem_handle *out)
{
    if (!out) return fail(OEM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (p < 1 || p > 4096) return fail(OEM_E_INVAL, "p must be in [1, 4096]");
    if (nfolds < 1 || nfolds > 64) return fail(OEM_E_INVAL, "nfolds must be in [1, 64]");
    if (precision != OEM_FP64 && precision != OEM_SPLIT_BF16 && precision != OEM_BF16)
        return fail(OEM_E_INVAL, "unknown precision");
    if (x_dtype != OEM_X_F32 && x_dtype != OEM_X_F64) return fail(OEM_E_INVAL, "unknown x_dtype");
    oem_gram_s *h = new oem_gram_s();
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(OEM_E_HIP, "hipGetDevice failed");
    }
    // the static workspace's address on this device, once per device
    char *scratch_addr = nullptr;
    int rc = noalloc_scratch(h->device, &scratch_addr);
    if (rc == OEM_OK) rc = handle_reconfigure(h, p, nfolds, precision, x_dtype, fold_seed, nullptr);
    if (rc == OEM_OK) rc = (hipStreamSynchronize(nullptr) == hipSuccess) ? OEM_OK : OEM_E_HIP;
    if (rc) {
        oem_gram_free(h);
        return rc == OEM_E_HIP ? fail(OEM_E_HIP, "initialisation failed") : rc;
    }
    *out = h;
    return OEM_OK;
}

void oem_gram_free(oem_handle h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_host_stage(h);
    free_upload_stage(h);
    for (DevBuf *b : {&h->Gk, &h->bk, &h->yyk, &h->nk, &h->csk, &h->ysk, &h->xbar, &h->ybar, &h->Gs, &h->cs, &h->sc, &h->yyn,
                      &h->dq, &h->ntrain, &h->lzsteps, &h->partial, &h->partial_n, &h->rowlist, &h->lanczos,
                      &h->paths, &h->order, &h->lam, &h->betaw, &h->groupbuf, &h->cvw, &h->flag, &h->pathws, &h->lzjobs})
        b->release();
    delete h;
}

int oem_gram_reset(oem_handle h, void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    hipStream_t s = as_stream(stream);
    const size_t pp = (size_t)h->p * h->p, K = h->K;
    int rc = launch_fill_f64(h->Gk.as<double>(), K * pp, 0.0, s);
    rc = rc ? rc : launch_fill_f64(h->bk.as<double>(), K * h->p, 0.0, s);
    rc = rc ? rc : launch_fill_f64(h->yyk.as<double>(), K, 0.0, s);
    rc = rc ? rc : launch_fill_i64(h->nk.as<int64_t>(), K, 0, s);
    rc = rc ? rc : launch_fill_f64(h->csk.as<double>(), K * h->p, 0.0, s);
    rc = rc ? rc : launch_fill_f64(h->ysk.as<double>(), K, 0.0, s);
    h->derived_valid = false;
    h->colsums_known = true;
    h->rows_seen = 0;
    return rc;
}

int oem_gram(oem_handle h, const void *X, int64_t n, int64_t ldx, const double *y,
             int64_t row_offset, const uint8_t *foldid, void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    if (n < 0 || n > INT32_MAX) return fail(OEM_E_INVAL, "n must be in [0, 2^31 - 1]");
    if (n == 0) return OEM_OK;
    if (!X || !y) return fail(OEM_E_INVAL, "X and y must not be NULL");
    if (ldx < h->p) return fail(OEM_E_INVAL, "ldx must be >= p");
    if (row_offset < 0) return fail(OEM_E_INVAL, "row_offset must be >= 0");
    int rc = launch_gram(h, X, n, ldx, y, row_offset, foldid, as_stream(stream));
    if (rc) return rc;
    h->rows_seen += n;
    h->derived_valid = false;
    return OEM_OK;
}

int oem_logistic_path(const void *X, int32_t x_dtype, int64_t n, int64_t ldx, int32_t p, const double *y,
                      const oem_penalty *pen, int32_t npen, const oem_path_opts *opts,
                      const oem_logistic_opts *lo, double *beta, double *lambda, int32_t *newton_iters,
                      double *kkt, double *obj, void *stream)
{
    if (!X || !y || !beta) return fail(OEM_E_INVAL, "X, y and beta must not be NULL");
    if (p < 1 || p > 2048) return fail(OEM_E_INVAL, "logistic paths take p in [1, 2048]");
    if (n < 1 || n > INT32_MAX) return fail(OEM_E_INVAL, "n must be in [1, 2^31 - 1]");
    if (ldx < p) return fail(OEM_E_INVAL, "ldx must be >= p");
    if (x_dtype != OEM_X_F32 && x_dtype != OEM_X_F64) return fail(OEM_E_INVAL, "unknown x_dtype");
    if (!pen || npen < 1) return fail(OEM_E_INVAL, "need at least one penalty");
    int rc = check_opts(opts);
    if (rc) return rc;
    if (!lo || !(lo->newton_tol > 0.0) || lo->newton_maxit < 1)
        return fail(OEM_E_INVAL, "logistic options: newton_tol > 0 and newton_maxit >= 1");
    if (!opts->standardize || opts->intercept)
        return fail(OEM_E_INVAL, "logistic paths standardise and fit no intercept");
    bool need_groups = false;
    for (int i = 0; i < npen; ++i) {
        rc = check_penalty(pen[i], INFINITY);   // gamma d conditions are checked at every step
        if (rc) return rc;
        need_groups |= group_penalty(pen[i].kind);
    }
    hipStream_t s = as_stream(stream);
    oem_handle h = nullptr;
    rc = oem_gram_create(p, 1, OEM_FP64, x_dtype, 0, &h);
    if (rc) return rc;
    GroupPlan gp;
    rc = build_groups(h, opts, need_groups, gp, s);
    if (rc == OEM_OK)
        rc = logistic_path(h, X, n, ldx, y, pen, npen, opts, lo, gp.d_gstart, gp.d_gidx, gp.ngroups, gp.d_w,
                           gp.d_cg, beta, lambda, newton_iters, kkt, obj, s);
    const std::string err = rc ? std::string(oem_last_error()) : std::string();
    oem_gram_free(h);
    if (rc) set_error(err);
    return rc;
}

int oem_gram_csr(oem_handle h, const int64_t *rowptr, const int32_t *colidx, const void *values,
                 int64_t nnz, int64_t n, const double *y, int64_t row_offset, const uint8_t *foldid,
                 void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    if (n < 0 || n > INT32_MAX) return fail(OEM_E_INVAL, "n must be in [0, 2^31 - 1]");
    if (nnz < 0) return fail(OEM_E_INVAL, "nnz must be >= 0");
    if (n == 0) return OEM_OK;
    if (!rowptr || !y || (nnz > 0 && (!colidx || !values)))
        return fail(OEM_E_INVAL, "rowptr, y (and colidx, values when nnz > 0) must not be NULL");
    if (row_offset < 0) return fail(OEM_E_INVAL, "row_offset must be >= 0");
    if (h->prec != OEM_FP64) return fail(OEM_E_INVAL, "sparse rows take the FP64 Gram form");
    int rc = launch_gram_csr(h, rowptr, colidx, values, nnz, n, y, row_offset, foldid, as_stream(stream));
    if (rc) return rc;
    h->rows_seen += n;
    h->derived_valid = false;
    return OEM_OK;
}

int oem_gram_host(oem_handle h, const void *X, int64_t n, int64_t ldx, const double *y,
                  int64_t row_offset, const uint8_t *foldid, int64_t chunk_rows, void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    if (n < 0) return fail(OEM_E_INVAL, "n must be >= 0");
    if (n == 0) return OEM_OK;
    if (!X || !y) return fail(OEM_E_INVAL, "X and y must not be NULL");
    if (ldx < h->p) return fail(OEM_E_INVAL, "ldx must be >= p");
    if (row_offset < 0) return fail(OEM_E_INVAL, "row_offset must be >= 0");
    if (chunk_rows < 1 || chunk_rows > INT32_MAX) return fail(OEM_E_INVAL, "chunk_rows must be in [1, 2^31 - 1]");
    if (h->prec != OEM_FP64 && h->xdt != OEM_X_F32) return fail(OEM_E_INVAL, "the BF16 Gram forms take FP32 X");
    return gram_from_host(h, X, n, ldx, y, row_offset, foldid, chunk_rows, as_stream(stream));
}

int oem_gram_noalloc(oem_handle h, const void *X, int64_t n, int64_t ldx, const double *y,
                     int64_t row_offset, const uint8_t *foldid, void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    if (n < 0 || n > INT32_MAX) return fail(OEM_E_INVAL, "n must be in [0, 2^31 - 1]");
    if (n == 0) return OEM_OK;
    if (!X || !y) return fail(OEM_E_INVAL, "X and y must not be NULL");
    if (ldx < h->p) return fail(OEM_E_INVAL, "ldx must be >= p");
    if (row_offset < 0) return fail(OEM_E_INVAL, "row_offset must be >= 0");
    int dev = 0;
    OEM_HIP_CHECK(hipGetDevice(&dev));
    if (dev != h->device) return fail(OEM_E_INVAL, "the handle belongs to another device");
    const size_t need = gram_work_bytes(h, n);
    if (need > kNoAllocScratchBytes)
        return fail(OEM_E_INVAL, "a pass over " + std::to_string(n) + " rows needs " + std::to_string(need) +
                                     " bytes of workspace, more than the " +
                                     std::to_string(kNoAllocScratchBytes) +
                                     "-byte static workspace; pass the rows in smaller blocks");
    char *base = nullptr;
    int rc = noalloc_scratch(dev, &base);
    if (rc) return rc;
    GramWork ws;
    ws.base = base;
    ws.bytes = kNoAllocScratchBytes;
    rc = launch_gram(h, X, n, ldx, y, row_offset, foldid, as_stream(stream), &ws);
    if (rc) return rc;
    h->rows_seen += n;
    h->derived_valid = false;
    return OEM_OK;
}

int oem_gram_import(oem_handle h, int32_t fold, const double *XtX, const double *Xty, double yty,
                    int64_t n, int32_t scaled, void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    if (fold < 0 || fold >= h->K) return fail(OEM_E_INVAL, "fold out of range");
    if (!XtX || !Xty || n <= 0) return fail(OEM_E_INVAL, "XtX, Xty must be set and n > 0");
    hipStream_t s = as_stream(stream);
    const size_t pp = (size_t)h->p * h->p;
    double *G = h->Gk.as<double>() + fold * pp;
    double *b = h->bk.as<double>() + (size_t)fold * h->p;
    OEM_HIP_CHECK(hipMemcpyAsync(G, XtX, pp * sizeof(double), hipMemcpyDeviceToDevice, s));
    OEM_HIP_CHECK(hipMemcpyAsync(b, Xty, h->p * sizeof(double), hipMemcpyDeviceToDevice, s));
    const double yv = scaled ? yty * (double)n : yty;
    int rc = launch_fill_f64(h->yyk.as<double>() + fold, 1, yv, s);
    rc = rc ? rc : launch_fill_i64(h->nk.as<int64_t>() + fold, 1, n, s);
    if (rc) return rc;
    if (scaled) {
        rc = launch_scale_f64(G, pp, (double)n, s);
        rc = rc ? rc : launch_scale_f64(b, h->p, (double)n, s);
        if (rc) return rc;
    }
    h->rows_seen += n;
    h->derived_valid = false;
    h->colsums_known = false;   // no column sums come with imported statistics
    return OEM_OK;
}

int oem_debug_lanczos_steps(void *handle, int32_t *steps, int32_t nq)
{
    oem_gram_s *h = static_cast<oem_gram_s *>(handle);
    if (!h || !steps || nq < 0) return fail(OEM_E_INVAL, "bad arguments");
    if (!h->derived_valid) return fail(OEM_E_STATE, "nothing derived yet");
    const int n = std::min<int>(nq, (int)h->lz_host.size());
    for (int i = 0; i < n; ++i) steps[i] = h->lz_host[i];
    return (int)h->lz_host.size();
}

int oem_gram_export_colsums(oem_handle h, double *colsum, double *ysum, void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    if (!h->colsums_known) return fail(OEM_E_STATE, "imported statistics carry no column sums");
    hipStream_t s = as_stream(stream);
    const size_t K = h->K;
    if (colsum)
        OEM_HIP_CHECK(hipMemcpyAsync(colsum, h->csk.ptr, K * h->p * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (ysum) OEM_HIP_CHECK(hipMemcpyAsync(ysum, h->ysk.ptr, K * sizeof(double), hipMemcpyDeviceToDevice, s));
    return OEM_OK;
}

int oem_gram_export(oem_handle h, double *G, double *b, double *yy, int64_t *nk, void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    hipStream_t s = as_stream(stream);
    const size_t pp = (size_t)h->p * h->p, K = h->K;
    if (G) OEM_HIP_CHECK(hipMemcpyAsync(G, h->Gk.ptr, K * pp * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (b) OEM_HIP_CHECK(hipMemcpyAsync(b, h->bk.ptr, K * h->p * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (yy) OEM_HIP_CHECK(hipMemcpyAsync(yy, h->yyk.ptr, K * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (nk) OEM_HIP_CHECK(hipMemcpyAsync(nk, h->nk.ptr, K * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    return OEM_OK;
}

int oem_fit_path(oem_handle h, int32_t fold, const oem_penalty *pen, int32_t npen,
                 const oem_path_opts *opts, double *beta, double *lambda, int32_t *iters,
                 double *kkt, double *obj, double *d_out, void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    if (!pen || npen < 1) return fail(OEM_E_INVAL, "need at least one penalty");
    if (!beta) return fail(OEM_E_INVAL, "beta must not be NULL");
    int rc = check_opts(opts);
    if (rc) return rc;
    if (fold < -1 || fold >= h->K || (h->K == 1 && fold != -1))
        return fail(OEM_E_INVAL, "fold out of range");
    hipStream_t s = as_stream(stream);
    rc = ensure_derived(h, opts->standardize ? 1 : 0, opts->intercept, s);
    if (rc) return rc;
    const int q = (fold < 0) ? 0 : 1 + fold;
    if (h->n_host[q] <= 0) return fail(OEM_E_INVAL, "the selected rows are empty");
    if (h->n_host[0] <= 0) return fail(OEM_E_INVAL, "no rows in the full data");
    bool need_groups = false;
    for (int i = 0; i < npen; ++i) {
        rc = check_penalty(pen[i], h->d_host[q]);
        if (rc) return rc;
        need_groups |= group_penalty(pen[i].kind);
    }
    GroupPlan gp;
    rc = build_groups(h, opts, need_groups, gp, s);
    if (rc) return rc;
    rc = prepare_lambda(h, pen, npen, opts, gp, s);
    if (rc) return rc;
    const int L = opts->nlambda;
    const size_t nl = (size_t)npen * L;
    rc = h->flag.ensure(nl * sizeof(int32_t));
    if (rc) return rc;
    int32_t *it = iters ? iters : h->flag.as<int32_t>();
    std::vector<PathDesc> descs;
    for (int i = 0; i < npen; ++i)
        descs.push_back(make_desc(h, q, pen[i], opts, gp, h->lam.as<double>() + (size_t)i * L,
                                  beta + (size_t)i * L * h->p, it + (size_t)i * L,
                                  kkt ? kkt + (size_t)i * L : nullptr,
                                  obj ? obj + (size_t)i * L : nullptr));
    if (opts->intercept && opts->beta0)
        for (int i = 0; i < npen; ++i) descs[i].beta0 = opts->beta0 + (size_t)i * L;
    rc = attach_path_handover(descs, h->pathws);
    if (rc) return rc;
    rc = upload_descs(h, descs, s);
    if (rc) return rc;
    rc = launch_paths(h->paths.as<PathDesc>(), descs, h->order, s, h);
    if (rc) return rc;
    if (opts->intercept && opts->beta0) {
        rc = launch_intercepts(h->paths.as<PathDesc>(), (int)descs.size(), s);
        if (rc) return rc;
    }
    if (lambda)
        OEM_HIP_CHECK(hipMemcpyAsync(lambda, h->lam.ptr, nl * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (d_out)
        OEM_HIP_CHECK(hipMemcpyAsync(d_out, h->dq.as<double>() + q, sizeof(double), hipMemcpyDeviceToDevice, s));
    if (opts->sync) return finish_sync(it, nl, s);
    return OEM_OK;
}

int oem_cv(oem_handle h, const oem_penalty *pen, int32_t npen, const oem_path_opts *opts,
           double *beta_full, double *beta_folds, double *lambda, double *cvm, double *cvsd,
           int32_t *i_min, int32_t *i_1se, int32_t *best, int32_t *iters, void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    if (h->K < 2) return fail(OEM_E_INVAL, "cross validation needs nfolds >= 2");
    if (!pen || npen < 1) return fail(OEM_E_INVAL, "need at least one penalty");
    if (!beta_full || !cvm) return fail(OEM_E_INVAL, "beta_full and cvm must not be NULL");
    int rc = check_opts(opts);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    rc = ensure_derived(h, opts->standardize ? 1 : 0, opts->intercept, s);
    if (rc) return rc;
    const int K = h->K, p = h->p, L = opts->nlambda;
    for (int q = 0; q <= K; ++q)
        if (h->n_host[q] <= 0) return fail(OEM_E_INVAL, "a fold leaves no training rows");
    // held-out rows of fold k: all rows less its training rows (Section 3 CV
    // error divides by their count)
    for (int k = 0; k < K; ++k)
        if (h->n_host[0] - h->n_host[1 + k] <= 0)
            return fail(OEM_E_INVAL, "fold " + std::to_string(k) + " has no held-out rows");
    bool need_groups = false;
    for (int i = 0; i < npen; ++i) {
        for (int q = 0; q <= K; ++q) {
            rc = check_penalty(pen[i], h->d_host[q]);
            if (rc) return rc;
        }
        need_groups |= group_penalty(pen[i].kind);
    }
    GroupPlan gp;
    rc = build_groups(h, opts, need_groups, gp, s);
    if (rc) return rc;
    rc = prepare_lambda(h, pen, npen, opts, gp, s);
    if (rc) return rc;
    const size_t nl = (size_t)npen * L;
    const size_t fold_beta = (size_t)K * nl * p;
    double *bf = beta_folds;
    if (!bf) {
        rc = h->betaw.ensure(fold_beta * sizeof(double));
        if (rc) return rc;
        bf = h->betaw.as<double>();
    }
    rc = h->flag.ensure((size_t)(K + 1) * nl * sizeof(int32_t));
    if (rc) return rc;
    int32_t *it = iters ? iters : h->flag.as<int32_t>();
    // scratch: per-fold MSE (npen x K x L), cvm/cvsd if not requested, the
    // intercepts of the full data (npen x L) and of the folds (K x npen x L)
    rc = h->cvw.ensure((nl * K + 2 * nl + nl + nl * K) * sizeof(double) + 64);
    if (rc) return rc;
    double *mse = h->cvw.as<double>();
    double *cvsd_w = cvsd ? cvsd : mse + nl * K;
    double *b0_full = (opts->intercept && opts->beta0) ? opts->beta0 : mse + nl * K + 2 * nl;
    double *b0_folds = mse + nl * K + 3 * nl;
    std::vector<PathDesc> descs;
    for (int q = 0; q <= K; ++q)
        for (int i = 0; i < npen; ++i) {
            double *b = (q == 0) ? beta_full + (size_t)i * L * p
                                 : bf + ((size_t)(q - 1) * npen + i) * L * p;
            descs.push_back(make_desc(h, q, pen[i], opts, gp, h->lam.as<double>() + (size_t)i * L, b,
                                      it + ((size_t)q * npen + i) * L, nullptr, nullptr));
            if (opts->intercept)
                descs.back().beta0 = (q == 0) ? b0_full + (size_t)i * L
                                              : b0_folds + ((size_t)(q - 1) * npen + i) * L;
        }
    rc = attach_path_handover(descs, h->pathws);
    if (rc) return rc;
    rc = upload_descs(h, descs, s);
    if (rc) return rc;
    rc = launch_paths(h->paths.as<PathDesc>(), descs, h->order, s, h);
    if (rc) return rc;
    if (opts->intercept) {
        rc = launch_intercepts(h->paths.as<PathDesc>(), (int)descs.size(), s);
        if (rc) return rc;
    }
    rc = launch_cv(h->Gk.as<double>(), h->bk.as<double>(), h->yyk.as<double>(), h->nk.as<int64_t>(),
                   h->csk.as<double>(), h->ysk.as<double>(), opts->intercept ? b0_folds : nullptr,
                   K, p, npen, L, bf, mse, cvm, cvsd_w, i_min, i_1se, best, s);
    if (rc) return rc;
    if (lambda)
        OEM_HIP_CHECK(hipMemcpyAsync(lambda, h->lam.ptr, nl * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (opts->sync) return finish_sync(it, (size_t)(K + 1) * nl, s);
    return OEM_OK;
}

int oem_gram_autotune(oem_handle h, const void *X, int64_t n, int64_t ldx, const double *y,
                      void *stream)
{
    if (!h) return fail(OEM_E_INVAL, "handle is NULL");
    if (n < 1 || n > INT32_MAX) return fail(OEM_E_INVAL, "n must be in [1, 2^31 - 1]");
    if (!X || !y) return fail(OEM_E_INVAL, "X and y must not be NULL");
    if (ldx < h->p) return fail(OEM_E_INVAL, "ldx must be >= p");
    hipStream_t s = as_stream(stream);
    const int cand[] = {256, 512, 1024, 2048, 4096, 8192};
    hipEvent_t e0, e1;
    OEM_HIP_CHECK(hipEventCreate(&e0));
    OEM_HIP_CHECK(hipEventCreate(&e1));
    int best = kGramDefaultTarget;
    float best_ms = INFINITY;
    int rc = OEM_OK;
    for (int c : cand) {
        gram_set_target(h->prec, h->K, h->p, n, c);
        rc = launch_gram(h, X, n, ldx, y, 0, nullptr, s);   // sizes the buffers
        if (rc) break;
        if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(OEM_E_HIP, "hipEventRecord failed"); break; }
        for (int r = 0; r < 2 && !rc; ++r) rc = launch_gram(h, X, n, ldx, y, 0, nullptr, s);
        if (rc) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(OEM_E_HIP, "timing the Gram pass failed");
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    gram_set_target(h->prec, h->K, h->p, n, best);
    if (rc) return rc;
    rc = oem_gram_reset(h, stream);
    if (rc) return rc;
    OEM_HIP_CHECK(hipStreamSynchronize(s));
    return OEM_OK;
}

void oem_batch_free(oem_batch b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (oem_gram_s *h : b->hs) oem_gram_free(h);
    for (DevBuf *d : {&b->descs, &b->order, &b->jobs, &b->iters_own, &b->pathws}) d->release();
    delete b;
}

int oem_batch_run(oem_batch b, void *stream)
{
    if (!b) return fail(OEM_E_INVAL, "batch is NULL");
    hipStream_t s = as_stream(stream);
    const int L = b->opts.nlambda, npen = b->npen;
    const size_t nl = (size_t)npen * L;
    for (size_t i = 0; i < b->hs.size(); ++i) {
        oem_gram_s *h = b->hs[i];
        const oem_problem &pr = b->probs[i];
        int rc = oem_gram_reset(h, stream);
        rc = rc ? rc : launch_gram(h, pr.X, pr.n, pr.ldx, pr.y, 0, nullptr, s);
        rc = rc ? rc : launch_combine(h, 1, 0, s);
        if (rc) return rc;
    }
    int rc = launch_lanczos_jobs(b->jobs.as<LzJob>(), b->lz, s);
    if (rc) return rc;
    for (size_t i = 0; i < b->hs.size(); ++i) {
        if (b->explicit_lam[i]) continue;
        oem_gram_s *h = b->hs[i];
        const GroupPlan &gp = b->groups[i];
        double *dl = h->lam.as<double>();
        rc = launch_lambda_grid(h->cs.as<double>(), h->p, gp.d_gstart, gp.d_gidx, gp.ngroups, gp.d_w,
                                gp.d_cg, reinterpret_cast<const oem_penalty *>(dl + nl), npen, L,
                                b->opts.lambda_min_ratio, dl, s);
        if (rc) return rc;
    }
    rc = launch_paths_planned(b->descs.as<PathDesc>(), b->order.as<int>(), b->plan, s);
    if (rc) return rc;
    // held-out error and selection of the cross-validation problems
    for (size_t i = 0; i < b->hs.size(); ++i) {
        oem_gram_s *h = b->hs[i];
        const oem_problem &pr = b->probs[i];
        if (h->K < 2) continue;
        const int K = h->K;
        double *mse = h->cvw.as<double>();
        double *cvsd = pr.cvsd ? pr.cvsd : mse + nl * K;
        rc = launch_cv(h->Gk.as<double>(), h->bk.as<double>(), h->yyk.as<double>(), h->nk.as<int64_t>(),
                       h->csk.as<double>(), h->ysk.as<double>(), nullptr, K, h->p, npen, L, b->beta_folds[i],
                       mse, pr.cvm, cvsd, pr.i_min, pr.i_1se, pr.best, s);
        if (rc) return rc;
    }
    for (size_t i = 0; i < b->hs.size(); ++i)
        if (b->probs[i].lambda)
            OEM_HIP_CHECK(hipMemcpyAsync(b->probs[i].lambda, b->hs[i]->lam.ptr, nl * sizeof(double),
                                         hipMemcpyDeviceToDevice, s));
    return OEM_OK;
}

int oem_batch_run_graph(oem_batch b, void *stream)
{
    if (!b) return fail(OEM_E_INVAL, "batch is NULL");
    hipStream_t s = as_stream(stream);
    if (!s) return fail(OEM_E_INVAL, "graph capture needs a stream other than the null stream");
    if (!b->exec) {
        OEM_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
        const int rc = oem_batch_run(b, stream);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(s, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (ec != hipSuccess) return fail(OEM_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(ec));
        b->graph = g;
        OEM_HIP_CHECK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    OEM_HIP_CHECK(hipGraphLaunch(b->exec, s));
    return OEM_OK;
}

int oem_batch_status(oem_batch b, void *stream)
{
    if (!b) return fail(OEM_E_INVAL, "batch is NULL");
    hipStream_t s = as_stream(stream);
    OEM_HIP_CHECK(hipStreamSynchronize(s));
    for (size_t i = 0; i < b->iters_of.size(); ++i) {
        std::vector<int32_t> it(b->iters_len[i]);
        OEM_HIP_CHECK(hipMemcpy(it.data(), b->iters_of[i], it.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int32_t v : it)
            if (v < 0) {
                set_error("some lambda of some problem reached maxit before the convergence test held");
                return OEM_NOT_CONVERGED;
            }
    }
    return OEM_OK;
}

int oem_batch_create(const oem_problem *probs, int32_t nprob, int32_t precision, int32_t x_dtype,
                     const oem_penalty *pen, int32_t npen, const oem_path_opts *opts, oem_batch *out)
{
    if (!out) return fail(OEM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!probs || nprob < 1) return fail(OEM_E_INVAL, "need at least one problem");
    if (!pen || npen < 1) return fail(OEM_E_INVAL, "need at least one penalty");
    int rc = check_opts(opts);
    if (rc) return rc;
    if (!opts->standardize) return fail(OEM_E_INVAL, "batched fits need standardize = 1");
    if (opts->groups || opts->lambda || opts->w || opts->cg)
        return fail(OEM_E_INVAL, "batched fits take groups and lambda per problem (opts->groups, lambda, w, cg "
                                 "must be NULL)");
    if (opts->intercept) return fail(OEM_E_INVAL, "batched fits take no intercept");
    bool need_groups = false;
    for (int i = 0; i < npen; ++i) {
        rc = check_penalty(pen[i], 1.0);   // standardised: d >= 1
        if (rc) return rc;
        need_groups |= group_penalty(pen[i].kind);
    }
    const int L = opts->nlambda;
    const size_t nl = (size_t)npen * L;
    for (int i = 0; i < nprob; ++i) {
        const oem_problem &q = probs[i];
        const std::string who = "problem " + std::to_string(i) + ": ";
        if (q.p < 1 || q.p > 4096 || q.n < 1 || q.n > INT32_MAX || q.ldx < q.p || !q.X || !q.y || !q.beta)
            return fail(OEM_E_INVAL, who + "bad p, n, ldx or pointer");
        if (q.nfolds < 0 || q.nfolds > 64) return fail(OEM_E_INVAL, who + "nfolds must be in [0, 64]");
        if (q.nfolds >= 2 && !q.cvm) return fail(OEM_E_INVAL, who + "cross validation needs cvm");
        if (need_groups && !q.groups) return fail(OEM_E_INVAL, who + "a group penalty needs groups");
        if (q.lambda_in)
            for (size_t e = 0; e < nl; ++e)
                if (!(q.lambda_in[e] >= 0.0)) return fail(OEM_E_INVAL, who + "lambda values must be >= 0");
    }
    oem_batch_s *b = new oem_batch_s();
    b->probs.assign(probs, probs + nprob);
    b->prec = precision;
    b->xdt = x_dtype;
    b->npen = npen;
    b->pens.assign(pen, pen + npen);
    b->opts = *opts;
    b->opts.sync = 0;
    hipStream_t s = nullptr;
    auto bail = [&](int code) {
        oem_batch_free(b);
        return code;
    };
    auto nq_of = [](const oem_problem &q) { return q.nfolds >= 2 ? q.nfolds + 1 : 1; };
    // handles, tuning, buffers sized by one pass each
    size_t own_iters = 0;
    for (int i = 0; i < nprob; ++i)
        if (!probs[i].iters) own_iters += nq_of(probs[i]) * nl;
    rc = b->iters_own.ensure(std::max<size_t>(own_iters, 1) * sizeof(int32_t));
    if (rc) return bail(rc);
    size_t own_off = 0;
    std::vector<LzJob> jobs;
    std::vector<PathDesc> descs;
    b->groups.resize(nprob);
    for (int i = 0; i < nprob; ++i) {
        const oem_problem &q = b->probs[i];
        const int K = q.nfolds >= 2 ? q.nfolds : 1, nq = nq_of(q);
        oem_gram_s *h = nullptr;
        rc = oem_gram_create(q.p, K, precision, x_dtype, q.fold_seed, &h);
        if (rc) return bail(rc);
        b->hs.push_back(h);
        if ((double)q.n * q.p >= 4194304.0) {
            rc = oem_gram_autotune(h, q.X, q.n, q.ldx, q.y, nullptr);
            if (rc) return bail(rc);
        }
        rc = launch_gram(h, q.X, q.n, q.ldx, q.y, 0, nullptr, s);
        if (rc) return bail(rc);
        // groups of this problem (device copies in the handle)
        oem_path_opts po = b->opts;
        po.groups = q.groups;
        GroupPlan &gp = b->groups[i];
        rc = build_groups(h, &po, need_groups, gp, s);
        if (rc) return bail(rc);
        // lambda: the problem's own values, or the grid of every run
        rc = h->lam.ensure(nl * sizeof(double) + npen * sizeof(oem_penalty) + 64);
        if (rc) return bail(rc);
        if (q.lambda_in) {
            if (hipMemcpy(h->lam.ptr, q.lambda_in, nl * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
                return bail(fail(OEM_E_HIP, "copying the lambda values failed"));
        }
        b->explicit_lam.push_back(q.lambda_in ? 1 : 0);
        if (hipMemcpy(h->lam.as<double>() + nl, pen, npen * sizeof(oem_penalty), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(OEM_E_HIP, "copying the penalties failed"));
        // d of the full data and of every fold's training rows
        const size_t ws = lanczos_workspace_doubles(q.p);
        if (ws) {
            rc = h->lanczos.ensure((size_t)nq * ws * sizeof(double) + 64);
            if (rc) return bail(rc);
        }
        const size_t pp = (size_t)q.p * q.p;
        for (int g = 0; g < nq; ++g)
            jobs.push_back(LzJob{h->Gs.as<double>() + g * pp, ws ? h->lanczos.as<double>() + g * ws : nullptr,
                                 h->dq.as<double>() + g, h->lzsteps.as<int32_t>() + g, q.p, lanczos_mmax(q.p)});
        int32_t *it = q.iters ? q.iters : b->iters_own.as<int32_t>() + own_off;
        if (!q.iters) own_off += nq * nl;
        b->iters_of.push_back(it);
        b->iters_len.push_back(nq * nl);
        double *bf = nullptr;
        if (K >= 2) {
            // fold coefficients (the caller's or the handle's), held-out error scratch
            bf = q.beta_folds;
            if (!bf) {
                rc = h->betaw.ensure((size_t)K * nl * q.p * sizeof(double));
                if (rc) return bail(rc);
                bf = h->betaw.as<double>();
            }
            rc = h->cvw.ensure((nl * K + 2 * nl) * sizeof(double) + 64);
            if (rc) return bail(rc);
        }
        b->beta_folds.push_back(bf);
        for (int g = 0; g < nq; ++g)
            for (int k = 0; k < npen; ++k) {
                double *beta = g == 0 ? q.beta + (size_t)k * L * q.p : bf + ((size_t)(g - 1) * npen + k) * L * q.p;
                descs.push_back(make_desc(h, g, pen[k], &po, gp, h->lam.as<double>() + (size_t)k * L, beta,
                                          it + ((size_t)g * npen + k) * L,
                                          (g == 0 && q.kkt) ? q.kkt + (size_t)k * L : nullptr,
                                          (g == 0 && q.obj) ? q.obj + (size_t)k * L : nullptr));
            }
    }
    lanczos_job_plan(jobs, b->lz);
    rc = attach_path_handover(descs, b->pathws);
    if (rc) return bail(rc);
    plan_paths(descs, b->plan);
    rc = b->jobs.ensure(jobs.size() * sizeof(LzJob));
    rc = rc ? rc : b->descs.ensure(descs.size() * sizeof(PathDesc));
    rc = rc ? rc : b->order.ensure(b->plan.order.size() * sizeof(int));
    if (rc) return bail(rc);
    if (hipMemcpy(b->jobs.ptr, jobs.data(), jobs.size() * sizeof(LzJob), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->descs.ptr, descs.data(), descs.size() * sizeof(PathDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->order.ptr, b->plan.order.data(), b->plan.order.size() * sizeof(int),
                  hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(OEM_E_HIP, "uploading the batch tables failed"));
    // one full run: every buffer reaches its size, so later runs allocate nothing
    rc = oem_batch_run(b, nullptr);
    if (rc) return bail(rc);
    if (hipDeviceSynchronize() != hipSuccess) return bail(fail(OEM_E_HIP, "the first batch run failed"));
    // every fold of a CV problem needs training rows and held-out rows
    for (int i = 0; i < nprob; ++i) {
        oem_gram_s *h = b->hs[i];
        if (h->K < 2) continue;
        std::vector<int64_t> nt(h->K + 1);
        if (hipMemcpy(nt.data(), h->ntrain.ptr, nt.size() * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
            return bail(fail(OEM_E_HIP, "reading the fold row counts failed"));
        for (int k = 0; k < h->K; ++k)
            if (nt[1 + k] <= 0 || nt[0] - nt[1 + k] <= 0)
                return bail(fail(OEM_E_INVAL, "problem " + std::to_string(i) + ": fold " + std::to_string(k) +
                                                  " has no training or no held-out rows"));
    }
    *out = b;
    return OEM_OK;
}

} // extern "C"
