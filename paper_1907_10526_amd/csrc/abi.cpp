// The C ABI of libfanproj: argument checks, device selection, batching into
// kernel launches, the lazily built SIRT weights, and error text.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fanproj_internal.h"

namespace fanproj {
namespace {

thread_local std::string g_last_error;

// A pointer is accepted when HIP knows it as device (or managed) memory of
// the geometry's device.
fp_status check_device_ptr(const void *p, int dev, const char *what) {
    if (!p) {
        set_error(std::string(what) + " is NULL");
        return FP_ERR_INVALID_ARG;
    }
    hipPointerAttribute_t attr{};
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error(std::string(what) + " is not device memory");
        return FP_ERR_INVALID_ARG;
    }
    const bool device_mem = attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
    if (!device_mem) {
        set_error(std::string(what) + " is not device memory");
        return FP_ERR_INVALID_ARG;
    }
    if (attr.type == hipMemoryTypeDevice && attr.device != dev) {
        set_error(std::string(what) + " lives on device " + std::to_string(attr.device) +
                  ", the geometry on device " + std::to_string(dev));
        return FP_ERR_INVALID_ARG;
    }
    return FP_OK;
}

int chunk_for(int remaining, int max_nb) {
    int nb = 1;
    while (nb * 2 <= remaining && nb * 2 <= max_nb) nb *= 2;
    return nb;
}

int back_max_chunk(const DevGeom &g) { return std::max(back_max_batch<float>(g), 1); }

// Images per launch of the quarter-turn forms (the back kernel holds four
// view quarters per image).
int quarter_max_chunk(const fp_geometry *g) {
    return std::max(1, std::min(kQuarterMaxChunk, back_max_batch<float>(g->dev_quarter) / 4));
}

// Free events of the marks, per device (never destroyed: marks held by
// static objects are released during exit).
struct MarkEvents {
    std::mutex mu;
    std::vector<std::vector<hipEvent_t>> free;   // [device]
};
MarkEvents &mark_events() {
    static MarkEvents *m = new MarkEvents;
    return *m;
}

// Device scratch of the launches (the forward's padded image copies, the
// back projection's view-group partials, the grouped SIRT buffers).  Each
// device keeps a set of buffers for the life of the process.  A call takes a
// buffer that no other host thread is enqueuing with, makes its stream wait
// for the mark of the buffer's last use and, after its launches, hands the
// buffer its own mark (the one mark the call records, finish_call).  Reuse
// across calls, streams and threads is so ordered on the device with no host
// synchronisation and no allocation in steady state.  A buffer grows (after its last use has
// finished) when a call needs more than it holds.
struct ScratchSlot {
    void *ptr = nullptr;
    size_t bytes = 0;
    MarkPtr last;   // mark of the last use (null: none pending)
    bool busy = false;
};
std::mutex g_scratch_mu;
std::vector<std::vector<std::unique_ptr<ScratchSlot>>> g_scratch;   // [device][slot]

ScratchSlot *take_slot(int dev, size_t bytes) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1);
    ScratchSlot *fit = nullptr, *any = nullptr;
    for (auto &p : g_scratch[dev]) {
        if (p->busy) continue;
        if (p->bytes >= bytes && (!fit || p->bytes < fit->bytes)) fit = p.get();
        if (!any || p->bytes > any->bytes) any = p.get();
    }
    ScratchSlot *s = fit ? fit : any;
    if (!s) {
        g_scratch[dev].push_back(std::make_unique<ScratchSlot>());
        s = g_scratch[dev].back().get();
    }
    s->busy = true;
    return s;
}

class Scratch {
  public:
    Scratch(int dev, size_t bytes, hipStream_t s) : dev_(dev), stream_(s) {
        slot_ = take_slot(dev, bytes);
        if (slot_->bytes < bytes) {
            // grow: wait for the buffer's last use, then replace it
            if (slot_->last) err_ = hipEventSynchronize(slot_->last->ev);
            slot_->last.reset();
            if (err_ == hipSuccess && slot_->ptr) err_ = hipFree(slot_->ptr);
            if (err_ == hipSuccess) {
                slot_->ptr = nullptr;
                slot_->bytes = 0;
                err_ = hipMalloc(&slot_->ptr, bytes);
                if (err_ == hipSuccess) slot_->bytes = bytes;
                else slot_->ptr = nullptr;
            }
        }
        if (err_ == hipSuccess && slot_->last) err_ = hipStreamWaitEvent(s, slot_->last->ev, 0);
    }
    // The call's mark, recorded after its launches (see finish_call).
    void set_mark(const MarkPtr &m) { mark_ = m; marked_ = true; }
    ~Scratch() {
        if (err_ == hipSuccess) {
            // (a call that ends early records its own mark here)
            if (!marked_) mark_ = record_mark(dev_, stream_);
            if (!mark_) {
                // no mark: the buffer is free once this stream's work is done
                if (hipStreamSynchronize(stream_) != hipSuccess) (void)hipGetLastError();
            }
            slot_->last = mark_;
        }
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        slot_->busy = false;
    }
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    float *get() const { return err_ == hipSuccess ? static_cast<float *>(slot_->ptr) : nullptr; }
    void *raw() const { return err_ == hipSuccess ? slot_->ptr : nullptr; }
    hipError_t status() const { return err_; }

  private:
    ScratchSlot *slot_ = nullptr;
    int dev_;
    hipStream_t stream_;
    hipError_t err_ = hipSuccess;
    MarkPtr mark_;
    bool marked_ = false;
};

// The end of a call that launched work for `g` on `s`: one mark, kept by the
// call's scratch buffer (if any) and by the geometry.
void finish_call(const fp_geometry *g, hipStream_t s, Scratch *scratch) {
    const MarkPtr m = record_mark(g->device, s);
    if (scratch) scratch->set_mark(m);
    note_use(g, s, m);
}

fp_status scratch_error(const char *fn, hipError_t e) {
    (void)hipGetLastError();
    set_error(std::string(fn) + ": scratch allocation failed: " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? FP_ERR_OUT_OF_MEMORY : FP_ERR_DEVICE;
}

fp_status check_call(const fp_geometry *g, int32_t batch, const char *fn) {
    if (!g) {
        set_error(std::string(fn) + ": geometry is NULL");
        return FP_ERR_INVALID_ARG;
    }
    if (batch < 1) {
        set_error(std::string(fn) + ": batch must be >= 1");
        return FP_ERR_INVALID_ARG;
    }
    return FP_OK;
}

fp_status ensure_weights(fp_geometry *g, hipStream_t stream) {
    std::lock_guard<std::mutex> lock(g->weights_mu);
    if (g->weights_ready) return FP_OK;
    const size_t nr = (size_t)g->nv * g->nd, np = (size_t)g->nx * g->ny;
    hipError_t e = hipSuccess;
    if (!g->row_w)
        e = pool_alloc(g->device, nr * sizeof(float), reinterpret_cast<void **>(&g->row_w),
                       &g->row_cap);
    if (e == hipSuccess && !g->col_w)
        e = pool_alloc(g->device, np * sizeof(float), reinterpret_cast<void **>(&g->col_w),
                       &g->col_cap);
    if (e != hipSuccess) {
        set_error(std::string("fp_sirt_step: allocating the SIRT weights failed: ") +
                  hipGetErrorString(e));
        return FP_ERR_OUT_OF_MEMORY;
    }
    e = launch_forward<float>(g->dev, FwdMode::kOnes, 1, nullptr, nullptr, g->row_w, nullptr,
                              nullptr, nullptr, stream);
    if (e != hipSuccess) return device_error("fp_sirt_step: row sums", e);
    e = launch_back<float>(g->dev, BackMode::kOnes, 1, nullptr, g->col_w, nullptr, nullptr, 0.0f,
                           stream);
    if (e != hipSuccess) return device_error("fp_sirt_step: column sums", e);
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_error("fp_sirt_step: building the weights", e);
    g->weight_bytes = (nr + np) * sizeof(float);
    g->weights_ready = true;
    return FP_OK;
}

}  // namespace

Mark::~Mark() {
    if (!ev) return;
    MarkEvents &me = mark_events();
    std::lock_guard<std::mutex> lock(me.mu);
    if ((int)me.free.size() <= dev) me.free.resize(dev + 1);
    me.free[dev].push_back(ev);
}

MarkPtr record_mark(int dev, hipStream_t s) {
    hipEvent_t ev = nullptr;
    {
        MarkEvents &me = mark_events();
        std::lock_guard<std::mutex> lock(me.mu);
        if ((int)me.free.size() > dev && !me.free[dev].empty()) {
            ev = me.free[dev].back();
            me.free[dev].pop_back();
        }
    }
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming | hipEventDisableSystemFence) !=
                   hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    auto m = std::make_shared<Mark>();
    m->ev = ev;
    m->dev = dev;
    if (hipEventRecord(ev, s) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;   // (the event goes back to the free list)
    }
    return m;
}

void note_use(const fp_geometry *gc, hipStream_t s, const MarkPtr &m) {
    fp_geometry *g = const_cast<fp_geometry *>(gc);
    std::lock_guard<std::mutex> lock(g->use_mu);
    if (!m) {
        g->untracked = true;
        return;
    }
    for (auto &u : g->uses)
        if (u.first == s) {
            u.second = m;
            return;
        }
    g->uses.emplace_back(s, m);
}

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

fp_status device_error(const char *what, hipError_t e) {
    (void)hipGetLastError();
    set_error(std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
    return FP_ERR_DEVICE;
}

}  // namespace fanproj

using namespace fanproj;

extern "C" const char *fp_last_error(void) { return g_last_error.c_str(); }

namespace fanproj {
namespace {

template <typename Real>
fp_status forward_impl(const fp_geometry *gc, const Real *image, Real *sino, int32_t batch,
                       void *stream, const char *fn) {
    clear_error();
    fp_status st = check_call(gc, batch, fn);
    if (st != FP_OK) return st;
    fp_geometry *g = const_cast<fp_geometry *>(gc);
    DeviceGuard guard(g->device);
    if (guard.status() != hipSuccess) return device_error(fn, guard.status());
    if ((st = check_device_ptr(image, g->device, "image")) != FP_OK) return st;
    if ((st = check_device_ptr(sino, g->device, "sino")) != FP_OK) return st;
    if constexpr (sizeof(Real) == sizeof(double)) {
        if ((st = ensure_f64_tables(g)) != FP_OK) return st;
    }
    const size_t np = (size_t)g->nx * g->ny, nr = (size_t)g->nv * g->nd;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if constexpr (sizeof(Real) == sizeof(float)) {
        if (g->quarter) {
            const int max_nb = chunk_for(batch, quarter_max_chunk(g));
            Scratch work(g->device, forward_quarter_work_bytes(g->dev_quarter, max_nb), s);
            if (work.status() != hipSuccess) return scratch_error(fn, work.status());
            for (int b0 = 0; b0 < batch;) {
                const int nb = chunk_for(batch - b0, max_nb);
                hipError_t e = launch_forward_quarter(g->dev_quarter, FwdMode::kPlain, nb,
                                                      image + b0 * np, work.get(), sino + b0 * nr,
                                                      nullptr, nullptr, s);
                if (e != hipSuccess) return device_error(fn, e);
                b0 += nb;
            }
            finish_call(g, s, &work);
            return FP_OK;
        }
    }
    const int max_nb = chunk_for(batch, kMaxBatchChunk);
    Scratch work(g->device, forward_work_bytes<Real>(g->dev, max_nb), s);
    if (work.status() != hipSuccess) return scratch_error(fn, work.status());
    for (int b0 = 0; b0 < batch;) {
        const int nb = chunk_for(batch - b0, kMaxBatchChunk);
        hipError_t e = launch_forward<Real>(g->dev, FwdMode::kPlain, nb, image + b0 * np,
                                            reinterpret_cast<Real *>(work.get()), sino + b0 * nr,
                                            nullptr, nullptr, nullptr, s);
        if (e != hipSuccess) return device_error(fn, e);
        b0 += nb;
    }
    finish_call(g, s, &work);
    return FP_OK;
}

template <typename Real>
fp_status back_impl(const fp_geometry *gc, const Real *sino, Real *image, int32_t batch,
                    void *stream, const char *fn) {
    clear_error();
    fp_status st = check_call(gc, batch, fn);
    if (st != FP_OK) return st;
    fp_geometry *g = const_cast<fp_geometry *>(gc);
    DeviceGuard guard(g->device);
    if (guard.status() != hipSuccess) return device_error(fn, guard.status());
    if ((st = check_device_ptr(sino, g->device, "sino")) != FP_OK) return st;
    if ((st = check_device_ptr(image, g->device, "image")) != FP_OK) return st;
    if constexpr (sizeof(Real) == sizeof(double)) {
        if ((st = ensure_f64_tables(g)) != FP_OK) return st;
    }
    const int max_nb = back_max_batch<Real>(g->dev);
    if (max_nb < 1) {
        set_error(std::string(fn) + ": the geometry's cell ranges do not fit the on-chip staging "
                                    "in this precision");
        return FP_ERR_UNSUPPORTED;
    }
    const size_t np = (size_t)g->nx * g->ny, nr = (size_t)g->nv * g->nd;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if constexpr (sizeof(Real) == sizeof(float)) {
        // one image: the octant form; a batch: the quarter-turn form, two
        // images per launch (measured faster than the octant form image by
        // image)
        if (g->octant && batch == 1) {
            Scratch partial(g->device, back_octant_work_bytes(g->dev_octant), s);
            if (partial.status() != hipSuccess) return scratch_error(fn, partial.status());
            hipError_t e = launch_back_octant(g->dev_octant, BackMode::kPlain, sino, image,
                                              partial.get(), nullptr, 0.0f, s);
            if (e != hipSuccess) return device_error(fn, e);
            finish_call(g, s, &partial);
            return FP_OK;
        }
        if (g->quarter) {
            const int qnb = chunk_for(batch, quarter_max_chunk(g));
            Scratch partial(g->device, back_quarter_work_bytes(g->dev_quarter, qnb), s);
            if (partial.status() != hipSuccess) return scratch_error(fn, partial.status());
            for (int b0 = 0; b0 < batch;) {
                const int nb = chunk_for(batch - b0, qnb);
                hipError_t e = launch_back_quarter(g->dev_quarter, BackMode::kPlain, nb,
                                                   sino + b0 * nr, image + b0 * np, partial.get(),
                                                   nullptr, 0.0f, s);
                if (e != hipSuccess) return device_error(fn, e);
                b0 += nb;
            }
            finish_call(g, s, &partial);
            return FP_OK;
        }
    }
    const size_t pbytes = back_work_bytes<Real>(g->dev, chunk_for(batch, max_nb));
    Scratch partial(g->device, std::max<size_t>(pbytes, 256), s);
    if (partial.status() != hipSuccess) return scratch_error(fn, partial.status());
    for (int b0 = 0; b0 < batch;) {
        const int nb = chunk_for(batch - b0, max_nb);
        hipError_t e = launch_back<Real>(g->dev, BackMode::kPlain, nb, sino + b0 * nr,
                                         image + b0 * np,
                                         pbytes ? reinterpret_cast<Real *>(partial.get()) : nullptr,
                                         nullptr, Real(0), s);
        if (e != hipSuccess) return device_error(fn, e);
        b0 += nb;
    }
    finish_call(g, s, &partial);
    return FP_OK;
}

}  // namespace
}  // namespace fanproj

extern "C" fp_status fp_forward(const fp_geometry *g, const float *image, float *sino,
                                int32_t batch, void *stream) {
    return forward_impl<float>(g, image, sino, batch, stream, "fp_forward");
}

extern "C" fp_status fp_back(const fp_geometry *g, const float *sino, float *image, int32_t batch,
                             void *stream) {
    return back_impl<float>(g, sino, image, batch, stream, "fp_back");
}

extern "C" fp_status fp_forward_f64(const fp_geometry *g, const double *image, double *sino,
                                    int32_t batch, void *stream) {
    return forward_impl<double>(g, image, sino, batch, stream, "fp_forward_f64");
}

extern "C" fp_status fp_back_f64(const fp_geometry *g, const double *sino, double *image,
                                 int32_t batch, void *stream) {
    return back_impl<double>(g, sino, image, batch, stream, "fp_back_f64");
}

namespace fanproj {
namespace {

fp_status reference_impl(const fp_geometry *g, bool forward, const double *in, double *out,
                         int32_t batch, int32_t quad, void *stream, const char *fn) {
    clear_error();
    fp_status st = check_call(g, batch, fn);
    if (st != FP_OK) return st;
    if (quad < 0 || quad > 24) {
        set_error(std::string(fn) + ": quad_points must be 0 (default 16) or 1 .. 24");
        return FP_ERR_INVALID_ARG;
    }
    DeviceGuard guard(g->device);
    if (guard.status() != hipSuccess) return device_error(fn, guard.status());
    if ((st = check_device_ptr(in, g->device, forward ? "image" : "sino")) != FP_OK) return st;
    if ((st = check_device_ptr(out, g->device, forward ? "sino" : "image")) != FP_OK) return st;
    const hipError_t e = launch_reference(g, forward, in, out, batch, quad ? quad : 16,
                                          static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(fn, e);
    finish_call(g, static_cast<hipStream_t>(stream), nullptr);
    return FP_OK;
}

}  // namespace
}  // namespace fanproj

extern "C" fp_status fp_forward_reference(const fp_geometry *g, const double *image, double *sino,
                                          int32_t batch, int32_t quad_points, void *stream) {
    return reference_impl(g, true, image, sino, batch, quad_points, stream, "fp_forward_reference");
}

extern "C" fp_status fp_back_reference(const fp_geometry *g, const double *sino, double *image,
                                       int32_t batch, int32_t quad_points, void *stream) {
    return reference_impl(g, false, sino, image, batch, quad_points, stream, "fp_back_reference");
}

namespace fanproj {

fp_status sirt_check(const fp_geometry *g, const float *image, const float *sino_meas,
                     float relaxation, const float *work, int32_t batch, const char *fn) {
    fp_status st = check_call(g, batch, fn);
    if (st != FP_OK) return st;
    if (!std::isfinite(relaxation)) {
        set_error(std::string(fn) + ": relaxation must be finite");
        return FP_ERR_INVALID_ARG;
    }
    if ((st = check_device_ptr(image, g->device, (std::string(fn) + ": image").c_str())) != FP_OK)
        return st;
    if ((st = check_device_ptr(sino_meas, g->device, (std::string(fn) + ": sino_meas").c_str())) !=
        FP_OK)
        return st;
    return check_device_ptr(work, g->device, (std::string(fn) + ": work").c_str());
}

Form sirt_form(const fp_geometry *g, int32_t batch) {
    if (g->octant && batch == 1) return Form::kOctant;
    return g->quarter ? Form::kQuarter : Form::kPlain;
}

int sirt_max_chunk(const fp_geometry *g, Form form) {
    if (form == Form::kOctant) return 1;
    if (form == Form::kQuarter) return quarter_max_chunk(g);
    return std::min(kMaxBatchChunk, back_max_chunk(g->dev));
}

size_t sirt_scratch_bytes(const fp_geometry *g, int nb, Form form, size_t *partial_offset) {
    const size_t copies = form == Form::kPlain ? forward_work_bytes<float>(g->dev, nb)
                                               : forward_quarter_work_bytes(g->dev_quarter, nb);
    const size_t aligned = (copies + 255) / 256 * 256;
    if (partial_offset) *partial_offset = aligned;
    return aligned + (form == Form::kOctant    ? back_octant_work_bytes(g->dev_octant)
                      : form == Form::kQuarter ? back_quarter_work_bytes(g->dev_quarter, nb)
                                               : back_work_bytes<float>(g->dev, nb));
}

fp_status sirt_step_launch(const fp_geometry *g, float *image, const float *sino_meas,
                           float relaxation, float *work, int32_t batch, int max_nb, Form form,
                           void *scratch, hipStream_t s, const char *fn) {
    const size_t np = (size_t)g->nx * g->ny, nr = (size_t)g->nv * g->nd;
    size_t poff = 0;
    (void)sirt_scratch_bytes(g, max_nb, form, &poff);
    float *copies = static_cast<float *>(scratch);
    float *partial = reinterpret_cast<float *>(static_cast<char *>(scratch) + poff);
    if (form == Form::kOctant) {   // quarter-turn forward, octant back
        for (int b = 0; b < batch; ++b) {
            hipError_t e = launch_forward_quarter(g->dev_quarter, FwdMode::kSirtResidual, 1,
                                                  image + b * np, copies, work + b * nr,
                                                  sino_meas + b * nr, g->row_w, s);
            if (e != hipSuccess) return device_error((std::string(fn) + ": forward launch").c_str(), e);
            e = launch_back_octant(g->dev_octant, BackMode::kSirtUpdate, work + b * nr,
                                   image + b * np, partial, g->col_w, relaxation, s);
            if (e != hipSuccess) return device_error((std::string(fn) + ": back launch").c_str(), e);
        }
        return FP_OK;
    }
    if (form == Form::kQuarter) {
        for (int b0 = 0; b0 < batch;) {
            const int nb = chunk_for(batch - b0, max_nb);
            hipError_t e = launch_forward_quarter(g->dev_quarter, FwdMode::kSirtResidual, nb,
                                                  image + b0 * np, copies, work + b0 * nr,
                                                  sino_meas + b0 * nr, g->row_w, s);
            if (e != hipSuccess) return device_error((std::string(fn) + ": forward launch").c_str(), e);
            e = launch_back_quarter(g->dev_quarter, BackMode::kSirtUpdate, nb, work + b0 * nr,
                                    image + b0 * np, partial, g->col_w, relaxation, s);
            if (e != hipSuccess) return device_error((std::string(fn) + ": back launch").c_str(), e);
            b0 += nb;
        }
        return FP_OK;
    }
    const bool use_partial = back_work_bytes<float>(g->dev, 1) > 0;
    for (int b0 = 0; b0 < batch;) {
        const int nb = chunk_for(batch - b0, max_nb);
        hipError_t e = launch_forward<float>(g->dev, FwdMode::kSirtResidual, nb, image + b0 * np,
                                             copies, work + b0 * nr, nullptr, sino_meas + b0 * nr,
                                             g->row_w, s);
        if (e != hipSuccess) return device_error((std::string(fn) + ": forward launch").c_str(), e);
        e = launch_back<float>(g->dev, BackMode::kSirtUpdate, nb, work + b0 * nr, image + b0 * np,
                               use_partial ? partial : nullptr, g->col_w, relaxation, s);
        if (e != hipSuccess) return device_error((std::string(fn) + ": back launch").c_str(), e);
        b0 += nb;
    }
    return FP_OK;
}

}  // namespace fanproj

extern "C" fp_status fp_sirt_step(const fp_geometry *g_const, float *image, const float *sino_meas,
                                  float relaxation, float *work, int32_t batch, void *stream) {
    clear_error();
    fp_status st = check_call(g_const, batch, "fp_sirt_step");
    if (st != FP_OK) return st;
    // The weights are the only state a geometry acquires after creation.
    fp_geometry *g = const_cast<fp_geometry *>(g_const);
    DeviceGuard guard(g->device);
    if (guard.status() != hipSuccess)
        return device_error("fp_sirt_step: hipSetDevice", guard.status());
    if ((st = sirt_check(g, image, sino_meas, relaxation, work, batch, "fp_sirt_step")) != FP_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = ensure_weights(g, s)) != FP_OK) return st;
    const Form form = sirt_form(g, batch);
    const int max_nb = chunk_for(batch, sirt_max_chunk(g, form));
    Scratch scratch(g->device,
                    std::max<size_t>(sirt_scratch_bytes(g, max_nb, form, nullptr), 256), s);
    if (scratch.status() != hipSuccess) return scratch_error("fp_sirt_step", scratch.status());
    st = sirt_step_launch(g, image, sino_meas, relaxation, work, batch, max_nb, form,
                          scratch.raw(), s, "fp_sirt_step");
    if (st == FP_OK) finish_call(g, s, &scratch);
    return st;
}

extern "C" fp_status fp_count_nonzero(const fp_geometry *g, int64_t *count, void *stream) {
    clear_error();
    fp_status st = check_call(g, 1, "fp_count_nonzero");
    if (st != FP_OK) return st;
    if (!count) {
        set_error("fp_count_nonzero: count is NULL");
        return FP_ERR_INVALID_ARG;
    }
    DeviceGuard guard(g->device);
    if (guard.status() != hipSuccess)
        return device_error("fp_count_nonzero: hipSetDevice", guard.status());
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = count_work_bytes(g->dev);
    Scratch work(g->device, bytes, s);
    if (work.status() != hipSuccess) return scratch_error("fp_count_nonzero", work.status());
    unsigned long long total = 0;
    hipError_t e = launch_count(g->dev, work.raw(), s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&total, static_cast<char *>(work.raw()) + bytes - sizeof(total),
                           sizeof(total), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error("fp_count_nonzero", e);
    *count = (int64_t)total;
    return FP_OK;
}

extern "C" size_t fp_sirt_scratch_bytes(const fp_geometry *g, int32_t batch) {
    if (!g || batch < 1) return 0;
    const Form form = sirt_form(g, batch);
    const int max_nb = chunk_for(batch, sirt_max_chunk(g, form));
    return sirt_scratch_bytes(g, max_nb, form, nullptr);
}

extern "C" fp_status fp_sirt_prepare(const fp_geometry *gc, void *stream) {
    clear_error();
    fp_status st = check_call(gc, 1, "fp_sirt_prepare");
    if (st != FP_OK) return st;
    fp_geometry *g = const_cast<fp_geometry *>(gc);
    DeviceGuard guard(g->device);
    if (guard.status() != hipSuccess) return device_error("fp_sirt_prepare", guard.status());
    return ensure_weights(g, static_cast<hipStream_t>(stream));
}

namespace {
// Scratch of one job of a grouped step, in the job's form.
const DevGeom &multi_geom(const fp_geometry *g) { return g->quarter ? g->dev_quarter : g->dev; }
size_t multi_job_bytes(const fp_geometry *g) {
    return (multi_copies_bytes(multi_geom(g)) + 255) / 256 * 256 +
           (multi_partial_bytes(multi_geom(g), g->quarter) + 255) / 256 * 256;
}
}  // namespace

extern "C" fp_status fp_sirt_step_multi(const fp_sirt_job *jobs, int32_t n_jobs, void *stream) {
    clear_error();
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) {
        set_error("fp_sirt_step_multi: jobs is NULL or n_jobs < 0");
        return FP_ERR_INVALID_ARG;
    }
    if (n_jobs == 0) return FP_OK;
    if (!jobs[0].geometry) {
        set_error("fp_sirt_step_multi: job 0 has no geometry");
        return FP_ERR_INVALID_ARG;
    }
    const int dev = jobs[0].geometry->device;
    DeviceGuard guard(dev);
    if (guard.status() != hipSuccess) return device_error("fp_sirt_step_multi", guard.status());
    hipStream_t s = static_cast<hipStream_t>(stream);
    fp_status st;
    size_t scratch_bytes = 0;
    for (int k = 0; k < n_jobs; ++k) {
        const fp_sirt_job &J = jobs[k];
        const std::string tag = "fp_sirt_step_multi: job " + std::to_string(k);
        if (!J.geometry) {
            set_error(tag + " has no geometry");
            return FP_ERR_INVALID_ARG;
        }
        if (J.geometry->device != dev) {
            set_error(tag + " lives on another device");
            return FP_ERR_INVALID_ARG;
        }
        if (!std::isfinite(J.relaxation)) {
            set_error(tag + ": relaxation must be finite");
            return FP_ERR_INVALID_ARG;
        }
        if ((st = check_device_ptr(J.image, dev, (tag + " image").c_str())) != FP_OK) return st;
        if ((st = check_device_ptr(J.sino_meas, dev, (tag + " sino_meas").c_str())) != FP_OK) return st;
        if ((st = check_device_ptr(J.work, dev, (tag + " work").c_str())) != FP_OK) return st;
        if ((st = ensure_weights(const_cast<fp_geometry *>(J.geometry), s)) != FP_OK) return st;
        scratch_bytes += multi_job_bytes(J.geometry);
    }
    Scratch scratch(dev, scratch_bytes, s);
    if (scratch.status() != hipSuccess) return scratch_error("fp_sirt_step_multi", scratch.status());
    char *base = static_cast<char *>(scratch.raw());
    size_t off = 0;
    // grouped launches of up to kMaxJobsPerLaunch jobs of one form and beam
    // shape: the quarter-turn jobs first, then the plain ones (each job's
    // order within its group kept)
    for (int form = 1; form >= 0; --form) {
        for (int beam : {FP_FAN_FLAT, FP_FAN_ARC, FP_PARALLEL}) {
            std::vector<int> idx;
            for (int k = 0; k < n_jobs; ++k)
                if ((int)jobs[k].geometry->quarter == form && jobs[k].geometry->beam == beam)
                    idx.push_back(k);
            for (size_t k0 = 0; k0 < idx.size(); k0 += kMaxJobsPerLaunch) {
                MultiArgs args{};
                args.n = (int)std::min<size_t>(kMaxJobsPerLaunch, idx.size() - k0);
                args.quarter = form;
                args.beam = beam;
                unsigned fwd = 0, items = 0;
                for (int k = 0; k < args.n; ++k) {
                    const fp_sirt_job &J = jobs[idx[k0 + k]];
                    const fp_geometry *g = J.geometry;
                    MultiJob &M = args.job[k];
                    M.g = multi_geom(g);
                    M.copies = reinterpret_cast<float *>(base + off);
                    M.partial = reinterpret_cast<float *>(
                        base + off + (multi_copies_bytes(M.g) + 255) / 256 * 256);
                    off += multi_job_bytes(g);
                    M.image = J.image;
                    M.image_out = J.image;
                    M.y_meas = J.sino_meas;
                    M.work = J.work;
                    M.row_w = g->row_w;
                    M.col_w = g->col_w;
                    M.relaxation = J.relaxation;
                    M.fwd_begin = fwd;
                    const int rays = fwd_rays_per_block(form ? 4 : 1);
                    fwd += (unsigned)M.g.nv * (unsigned)((M.g.nd + rays - 1) / rays);
                    M.back_begin = items;
                    items += (unsigned)(M.g.tiles_x * M.g.tiles_y * M.g.back_groups);
                    args.cap = std::max(args.cap, M.g.back_cap);
                }
                args.fwd_blocks = fwd;
                args.back_items = items;
                hipError_t e = launch_sirt_multi(args, s);
                if (e != hipSuccess) return device_error("fp_sirt_step_multi: launch", e);
            }
        }
    }
    {
        const MarkPtr m = record_mark(dev, s);
        scratch.set_mark(m);
        for (int k = 0; k < n_jobs; ++k) note_use(jobs[k].geometry, s, m);
    }
    return FP_OK;
}
