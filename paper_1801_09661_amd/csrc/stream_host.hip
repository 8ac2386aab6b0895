// Out-of-core Gram pass (Section 5.7: a design matrix that does not fit in
// memory, read from disk through memory mapping).  The rows of a host-resident
// X (ordinary memory, a memory-mapped file, or pinned memory) stream through
// two pinned staging slots and two device slots of `chunk_rows` rows each:
// packing chunk c + 1 on the CPU, the DMA of chunk c + 1 and the Gram kernels
// of chunk c overlap.  Each chunk is one accumulating Gram pass with its
// global row offset, so fold membership follows the global row index and the
// sums equal those of oem_gram called on the same row blocks.
#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "oem_internal.h"

namespace oem {

struct HostStage {
    int64_t chunk_rows = 0;
    int p = 0, esize = 0;
    size_t x_bytes = 0, y_off = 0, f_off = 0, slot_bytes = 0;
    void *pin[2] = {nullptr, nullptr};   // pinned: packed rows (p columns), y, fold ids
    DevBuf dev[2];
    hipStream_t copy = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr};    // the slot's DMA has finished
    hipEvent_t consumed[2] = {nullptr, nullptr};  // the slot's Gram pass has finished
    bool used[2] = {false, false};
};

void free_host_stage(oem_gram_s *h)
{
    HostStage *st = h->stage;
    if (!st) return;
    for (int i = 0; i < 2; ++i) {
        if (st->copied[i]) (void)hipEventDestroy(st->copied[i]);
        if (st->consumed[i]) (void)hipEventDestroy(st->consumed[i]);
        if (st->pin[i]) (void)hipHostFree(st->pin[i]);
        st->dev[i].release();
    }
    if (st->copy) (void)hipStreamDestroy(st->copy);
    delete st;
    h->stage = nullptr;
}

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Staging for chunks of `rows` rows of this handle's shape (kept and reused
// while the chunk size and shape stay the same).
static int ensure_stage(oem_gram_s *h, int64_t rows)
{
    const int esize = h->xdt == OEM_X_F64 ? 8 : 4;
    HostStage *st = h->stage;
    if (st && st->chunk_rows == rows && st->p == h->p && st->esize == esize) return OEM_OK;
    free_host_stage(h);
    st = new HostStage();
    h->stage = st;
    st->chunk_rows = rows;
    st->p = h->p;
    st->esize = esize;
    st->x_bytes = (size_t)rows * h->p * esize;
    st->y_off = align256(st->x_bytes);
    st->f_off = align256(st->y_off + (size_t)rows * sizeof(double));
    st->slot_bytes = align256(st->f_off + (size_t)rows);
    for (int i = 0; i < 2; ++i) {
        if (hipHostMalloc(&st->pin[i], st->slot_bytes, hipHostMallocDefault) != hipSuccess) {
            st->pin[i] = nullptr;
            free_host_stage(h);
            return fail(OEM_E_NOMEM, "pinned staging of " + std::to_string(st->slot_bytes) + " bytes failed");
        }
        int rc = st->dev[i].ensure(st->slot_bytes);
        if (rc) {
            free_host_stage(h);
            return rc;
        }
        if (hipEventCreateWithFlags(&st->copied[i], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&st->consumed[i], hipEventDisableTiming) != hipSuccess) {
            free_host_stage(h);
            return fail(OEM_E_HIP, "hipEventCreate failed");
        }
    }
    if (hipStreamCreateWithFlags(&st->copy, hipStreamNonBlocking) != hipSuccess) {
        st->copy = nullptr;
        free_host_stage(h);
        return fail(OEM_E_HIP, "hipStreamCreate failed");
    }
    return OEM_OK;
}

// Is ptr host memory the GPU can read directly (pinned or registered)?
static bool host_pinned(const void *ptr)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();   // ordinary pageable memory
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

static bool device_memory(const void *ptr)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

// Pack rows [r0, r0 + rows) of X (row stride ldx) into dst (stride p) with a
// few host threads.
static void pack_rows(char *dst, const char *X, int64_t r0, int64_t rows, int64_t ldx, int p, int esize)
{
    const size_t row_bytes = (size_t)p * esize, src_stride = (size_t)ldx * esize;
    const int64_t per_thread_min = 2048;
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(8, rows / per_thread_min));
    auto work = [&](int64_t a, int64_t b) {
        if ((int64_t)p == ldx) {
            std::memcpy(dst + (size_t)a * row_bytes, X + (size_t)(r0 + a) * src_stride, (size_t)(b - a) * row_bytes);
        } else {
            for (int64_t r = a; r < b; ++r)
                std::memcpy(dst + (size_t)r * row_bytes, X + (size_t)(r0 + r) * src_stride, row_bytes);
        }
    };
    if (nt == 1) {
        work(0, rows);
        return;
    }
    std::vector<std::thread> th;
    const int64_t step = (rows + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        const int64_t a = t * step, b = std::min(rows, a + step);
        if (a < b) th.emplace_back(work, a, b);
    }
    for (auto &t : th) t.join();
}

int gram_from_host(oem_gram_s *h, const void *X, int64_t n, int64_t ldx, const double *y,
                   int64_t row_offset, const uint8_t *foldid, int64_t chunk_rows, hipStream_t s)
{
    if (device_memory(X) || device_memory(y) || (foldid && device_memory(foldid)))
        return fail(OEM_E_INVAL, "X, y and foldid must be host memory (device rows go to oem_gram)");
    const int64_t rows = std::min<int64_t>(chunk_rows, n);
    int rc = ensure_stage(h, rows);
    if (rc) return rc;
    HostStage *st = h->stage;
    const bool x_pinned = host_pinned(X);
    const char *Xc = static_cast<const char *>(X);
    const int64_t nchunks = (n + rows - 1) / rows;
    for (int64_t c = 0; c < nchunks; ++c) {
        const int slot = (int)(c & 1);
        const int64_t r0 = c * rows, m = std::min(rows, n - r0);
        char *pin = static_cast<char *>(st->pin[slot]);
        char *dev = st->dev[slot].as<char>();
        // the pinned slot is free once its previous DMA finished; the device
        // slot once the Gram pass that read it finished
        if (st->used[slot]) {
            OEM_HIP_CHECK(hipEventSynchronize(st->copied[slot]));
            OEM_HIP_CHECK(hipStreamWaitEvent(st->copy, st->consumed[slot], 0));
        }
        if (!x_pinned) pack_rows(pin, Xc, r0, m, ldx, h->p, st->esize);
        std::memcpy(pin + st->y_off, y + r0, (size_t)m * sizeof(double));
        if (foldid) std::memcpy(pin + st->f_off, foldid + r0, (size_t)m);
        const size_t row_bytes = (size_t)h->p * st->esize;
        if (x_pinned)
            OEM_HIP_CHECK(hipMemcpy2DAsync(dev, row_bytes, Xc + (size_t)r0 * ldx * st->esize,
                                           (size_t)ldx * st->esize, row_bytes, (size_t)m,
                                           hipMemcpyHostToDevice, st->copy));
        else
            OEM_HIP_CHECK(hipMemcpyAsync(dev, pin, (size_t)m * row_bytes, hipMemcpyHostToDevice, st->copy));
        OEM_HIP_CHECK(hipMemcpyAsync(dev + st->y_off, pin + st->y_off, (size_t)m * sizeof(double),
                                     hipMemcpyHostToDevice, st->copy));
        if (foldid)
            OEM_HIP_CHECK(hipMemcpyAsync(dev + st->f_off, pin + st->f_off, (size_t)m, hipMemcpyHostToDevice,
                                         st->copy));
        OEM_HIP_CHECK(hipEventRecord(st->copied[slot], st->copy));
        OEM_HIP_CHECK(hipStreamWaitEvent(s, st->copied[slot], 0));
        rc = launch_gram(h, dev, m, h->p, reinterpret_cast<const double *>(dev + st->y_off), row_offset + r0,
                         foldid ? reinterpret_cast<const uint8_t *>(dev + st->f_off) : nullptr, s);
        if (rc) return rc;
        OEM_HIP_CHECK(hipEventRecord(st->consumed[slot], s));
        st->used[slot] = true;
        h->rows_seen += m;
        h->derived_valid = false;
    }
    // the caller's host arrays are not read after return
    for (int i = 0; i < 2; ++i)
        if (st->used[i]) OEM_HIP_CHECK(hipEventSynchronize(st->copied[i]));
    return OEM_OK;
}

} // namespace oem
