// scratch.cpp -- library-owned scratch memory for the routes that need a
// workspace (operand packing of direct-to-LDS GEMMs, the channels-last conv
// transposes, the e4m3 amax partials).
//
// One buffer per device, grown on demand and kept until mlk_release().  A use
// holds the library's scratch lock from begin() to end(): begin() makes the
// caller's stream wait (on the device) for the event recorded by the previous
// use, on whatever stream that ran, and end() records the event again after
// the work that reads the buffer has been enqueued.  Calls on any streams are
// therefore ordered on the buffer without a host synchronisation, and without
// the per-call stream-ordered allocate / free pair (whose free costs ~20 us of
// host time per call).  Requests above kScratchCacheMax are not cached: they
// take a stream-ordered allocation of their own, freed after the use.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "internal.hpp"

namespace mlk {

namespace {

constexpr size_t kScratchCacheMax = (size_t)512 << 20;
constexpr size_t kScratchGranule = (size_t)2 << 20;

struct DeviceScratch {
    void* ptr = nullptr;
    size_t size = 0;
    hipEvent_t done = nullptr;  // recorded after the last use's work
    bool used = false;
};

std::mutex g_scratch_mu;
std::map<int, DeviceScratch> g_scratch;

}  // namespace

// a use abandoned on an error path still releases the buffer in stream order
ScratchUse::~ScratchUse() { (void)end(); }

mlk_status ScratchUse::begin(size_t bytes, hipStream_t st, const char* what) {
    stream_ = st;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return fail(MLK_ERR_CONFIG, "%s needs library scratch memory, which is not used under stream capture; "
                    "choose a configuration without it", what);
    lock_ = std::unique_lock<std::mutex>(g_scratch_mu);
    if (bytes > kScratchCacheMax) {
        e = hipMallocAsync(&own_, bytes, st);
        if (e != hipSuccess) {
            own_ = nullptr;
            lock_.unlock();
            return hip_fail(e, "scratch allocation");
        }
        ptr_ = own_;
        return MLK_OK;
    }
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) {
        lock_.unlock();
        return hip_fail(e, "hipGetDevice");
    }
    DeviceScratch& d = g_scratch[dev];
    if (!d.done && (e = hipEventCreateWithFlags(&d.done, hipEventDisableTiming)) != hipSuccess) {
        d.done = nullptr;
        lock_.unlock();
        return hip_fail(e, "scratch event");
    }
    if (d.used && (e = hipStreamWaitEvent(st, d.done, 0)) != hipSuccess) {
        lock_.unlock();
        return hip_fail(e, "scratch wait");
    }
    if (d.size < bytes) {
        // the wait above orders this free after every earlier use
        const size_t want = std::min(kScratchCacheMax, std::max(bytes, 2 * d.size));
        if (d.ptr) (void)hipFreeAsync(d.ptr, st);
        d.ptr = nullptr;
        d.size = 0;
        const size_t nb = (want + kScratchGranule - 1) / kScratchGranule * kScratchGranule;
        if ((e = hipMallocAsync(&d.ptr, nb, st)) != hipSuccess) {
            d.ptr = nullptr;
            lock_.unlock();
            return hip_fail(e, "scratch allocation");
        }
        d.size = nb;
    }
    ptr_ = d.ptr;
    dev_ = dev;
    return MLK_OK;
}

mlk_status ScratchUse::end() {
    if (!lock_.owns_lock()) return MLK_OK;
    hipError_t e = hipSuccess;
    if (own_) {
        e = hipFreeAsync(own_, stream_);
        own_ = nullptr;
    } else {
        DeviceScratch& d = g_scratch[dev_];
        e = hipEventRecord(d.done, stream_);
        d.used = true;
    }
    lock_.unlock();
    return e == hipSuccess ? MLK_OK : hip_fail(e, "scratch release");
}

void release_scratch() {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (auto& kv : g_scratch) {
        if (hipSetDevice(kv.first) != hipSuccess) continue;
        (void)hipDeviceSynchronize();
        if (kv.second.ptr) (void)hipFreeAsync(kv.second.ptr, nullptr);
        (void)hipDeviceSynchronize();
        if (kv.second.done) (void)hipEventDestroy(kv.second.done);
    }
    g_scratch.clear();
    if (have_cur) (void)hipSetDevice(cur);
}

}  // namespace mlk
