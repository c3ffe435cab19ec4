// Device memory of geometries (tables, SIRT weights), recycled: a destroyed
// geometry's blocks go to a per-device list of idle blocks instead of
// hipFree, which waits for the whole device.  A later geometry takes an idle
// block that fits, after the events of the work queued with the block's
// previous owner have completed, so destroying a geometry never waits and
// reusing memory never races with work still queued against it.
#include <algorithm>
#include <memory>
#include <mutex>
#include <vector>

#include "fanproj_internal.h"

namespace fanproj {
namespace {

// Idle bytes a device may keep; beyond this the largest idle blocks are
// freed (after their events).
constexpr size_t kPoolIdleCap = size_t(1) << 30;

struct EventSet {
    std::vector<MarkPtr> marks;
    void wait() const {
        for (const MarkPtr &m : marks)
            if (m && hipEventSynchronize(m->ev) != hipSuccess) (void)hipGetLastError();
    }
};

struct IdleBlock {
    int device;
    void *ptr;
    size_t bytes;
    std::shared_ptr<EventSet> after;   // work of the previous owner
};

std::mutex g_pool_mu;
std::vector<IdleBlock> g_idle;

}  // namespace

hipError_t pool_alloc(int dev, size_t bytes, void **out, size_t *capacity) {
    IdleBlock got{-1, nullptr, 0, nullptr};
    {
        std::lock_guard<std::mutex> lock(g_pool_mu);
        size_t best = (size_t)-1;
        int at = -1;
        for (size_t k = 0; k < g_idle.size(); ++k) {
            const IdleBlock &b = g_idle[k];
            // fits, and wastes at most half of the block (or 4 MiB)
            if (b.device == dev && b.bytes >= bytes &&
                b.bytes <= std::max(2 * bytes, bytes + (size_t(4) << 20)) && b.bytes < best) {
                best = b.bytes;
                at = (int)k;
            }
        }
        if (at >= 0) {
            got = g_idle[at];
            g_idle.erase(g_idle.begin() + at);
        }
    }
    if (got.ptr) {
        if (got.after) got.after->wait();
        *out = got.ptr;
        *capacity = got.bytes;
        return hipSuccess;
    }
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        *capacity = 0;
        return e;
    }
    *out = p;
    *capacity = bytes;
    return hipSuccess;
}

void pool_release(int dev, const std::vector<std::pair<void *, size_t>> &blocks,
                  const std::vector<MarkPtr> &after) {
    auto set = std::make_shared<EventSet>();
    set->marks = after;
    std::vector<IdleBlock> spill;
    {
        std::lock_guard<std::mutex> lock(g_pool_mu);
        for (const auto &b : blocks)
            if (b.first) g_idle.push_back(IdleBlock{dev, b.first, b.second, set});
        size_t idle = 0;
        for (const IdleBlock &b : g_idle)
            if (b.device == dev) idle += b.bytes;
        while (idle > kPoolIdleCap) {
            int at = -1;
            for (size_t k = 0; k < g_idle.size(); ++k)
                if (g_idle[k].device == dev && (at < 0 || g_idle[k].bytes > g_idle[at].bytes))
                    at = (int)k;
            if (at < 0) break;
            idle -= g_idle[at].bytes;
            spill.push_back(g_idle[at]);
            g_idle.erase(g_idle.begin() + at);
        }
    }
    for (const IdleBlock &b : spill) {
        if (b.after) b.after->wait();
        (void)hipFree(b.ptr);
    }
}

}  // namespace fanproj
