// fp_sirt_step_noalloc: the SIRT step of fp_sirt_step with its launch
// scratch (the forward's padded image copies and the back projection's
// partial sums) in a fixed device array instead of the library's growable
// buffers, so a call allocates nothing.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "fanproj_internal.h"

namespace fanproj {
namespace {

// The fixed scratch.  Every device the library runs on holds one copy (at
// its own address) from the module's load until the process ends.  Host
// code never passes the array's name to a kernel: it passes the device
// address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[FP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (current), looked up once.
fp_status scratch_address(int dev, void **out, const char *fn) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error(std::string(fn) + ": device index " + std::to_string(dev) + " out of range");
        return FP_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return device_error((std::string(fn) + ": hipGetSymbolAddress").c_str(),
                                e != hipSuccess ? e : hipErrorInvalidSymbol);
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return FP_OK;
}

// The largest batch chunk (a power of two) whose scratch fits the array.
int fitting_chunk(const fp_geometry *g, Form form) {
    int nb = sirt_max_chunk(g, form);
    while (nb > 1 && sirt_scratch_bytes(g, nb, form, nullptr) > FP_NOALLOC_SCRATCH_BYTES)
        nb /= 2;
    return nb;
}

}  // namespace
}  // namespace fanproj

using namespace fanproj;

extern "C" fp_status fp_sirt_step_noalloc(const fp_geometry *g, float *image,
                                          const float *sino_meas, float relaxation, float *work,
                                          int32_t batch, void *stream) {
    const char *fn = "fp_sirt_step_noalloc";
    clear_error();
    if (!g) {
        set_error(std::string(fn) + ": geometry is NULL");
        return FP_ERR_INVALID_ARG;
    }
    DeviceGuard guard(g->device);
    if (guard.status() != hipSuccess) return device_error(fn, guard.status());
    fp_status st = sirt_check(g, image, sino_meas, relaxation, work, batch, fn);
    if (st != FP_OK) return st;
    {
        std::lock_guard<std::mutex> lock(const_cast<fp_geometry *>(g)->weights_mu);
        if (!g->weights_ready) {
            set_error(std::string(fn) + ": the SIRT weights are not built; call fp_sirt_prepare "
                                        "(or fp_sirt_step) on this geometry first");
            return FP_ERR_INVALID_ARG;
        }
    }
    // the form fp_sirt_step takes where one image's scratch fits, else the
    // next simpler one (octant, quarter-turn, plain)
    Form form = sirt_form(g, batch);
    int max_nb = fitting_chunk(g, form);
    while (form != Form::kPlain &&
           sirt_scratch_bytes(g, max_nb, form, nullptr) > FP_NOALLOC_SCRATCH_BYTES) {
        form = form == Form::kOctant ? Form::kQuarter : Form::kPlain;
        max_nb = fitting_chunk(g, form);
    }
    const size_t need = sirt_scratch_bytes(g, max_nb, form, nullptr);
    if (need > FP_NOALLOC_SCRATCH_BYTES) {
        set_error(std::string(fn) + ": one image needs " + std::to_string(need) +
                  " bytes of scratch, more than the fixed " +
                  std::to_string((size_t)FP_NOALLOC_SCRATCH_BYTES) + " bytes");
        return FP_ERR_UNSUPPORTED;
    }
    void *p = nullptr;
    if ((st = scratch_address(g->device, &p, fn)) != FP_OK) return st;
    return sirt_step_launch(g, image, sino_meas, relaxation, work, batch, max_nb, form, p,
                            static_cast<hipStream_t>(stream), fn);
}
