// rms_run_noalloc: rms_run on a device scratch array of the library's own,
// for callers that cannot allocate device memory.
//
// Every buffer of a run (tables, walker order, persistent-walk state and
// control words, per-walker records, reduction partials, results) is laid out
// in `scratch`, a file-scope device array of RMS_NOALLOC_MAX_BYTES that each
// GPU the library runs on holds until the process ends.  Host code never uses
// the array's name as an address (on the host it is only a stand-in for the
// symbol): at a device's first call the entry point asks the runtime for the
// array's address on that device and keeps it, with two timing events, per
// device.  The run's kernels are the ones rms_run launches, and every buffer
// that must start at zero is cleared by a kernel of the run itself, so a call
// does not depend on what the previous call left in the array.
#include <hip/hip_runtime.h>

#include <chrono>
#include <mutex>
#include <string>

#include "rms_host.h"

namespace {

static __device__ __align__(256) unsigned char scratch[RMS_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;

struct DeviceScratch {
    void* ptr = nullptr;  // address of `scratch` on the device
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool ready = false;
};

std::mutex g_m;
DeviceScratch g_dev[kMaxDevices];

// The device's scratch address and events, set up at its first call (the
// device is current).
int device_scratch(int dev, DeviceScratch** out) {
    if (dev < 0 || dev >= kMaxDevices) return rms::fail(RMS_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_m);
    DeviceScratch& d = g_dev[dev];
    if (!d.ready) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return rms::hip_fail("scratch address", e);
        if (!d.ev0 && (e = hipEventCreate(&d.ev0)) != hipSuccess)
            return rms::hip_fail("scratch events", e);
        if (!d.ev1 && (e = hipEventCreate(&d.ev1)) != hipSuccess)
            return rms::hip_fail("scratch events", e);
        d.ptr = p;
        d.ready = true;
    }
    *out = &d;
    return RMS_OK;
}

}  // namespace

extern "C" int rms_run_noalloc(const rms_substrate* sub, const rms_params* params, uint64_t seed,
                               int64_t n_walkers, int64_t n_steps, double dt_ms, int n_shapes,
                               const double* waveform, int n_dirs, const double* dirs, int n_b,
                               const double* bvals, int precision, void* hip_stream,
                               rms_result* out) {
    const auto t0 = std::chrono::steady_clock::now();
    rms::clear_error();
    if (!out) return rms::fail(RMS_E_INVALID_ARG, "result is required");
    rms::RunSetup r;
    int rc = rms::prepare_run(sub, params, seed, n_walkers, n_steps, dt_ms, n_shapes, waveform,
                              n_dirs, dirs, n_b, bvals, precision, r);
    if (rc) return rc;

    int prev_dev = 0;
    hipError_t e = hipGetDevice(&prev_dev);
    if (e != hipSuccess) return rms::hip_fail("hipGetDevice", e);
    struct DeviceGuard {
        int prev;
        ~DeviceGuard() { (void)hipSetDevice(prev); }
    } guard{prev_dev};
    if ((e = hipSetDevice(sub->device)) != hipSuccess) return rms::hip_fail("hipSetDevice", e);

    // sizes are checked after the device is current: the persistent walk's
    // state buffer depends on the device's compute-unit count
    const size_t need = rms::DeviceRun::layout_bytes(*sub, r, false);
    if (need > static_cast<size_t>(RMS_NOALLOC_MAX_BYTES))
        return rms::fail(RMS_E_INVALID_ARG,
                         "rms_run_noalloc: the run needs " + std::to_string(need) +
                             " bytes of device scratch, more than RMS_NOALLOC_MAX_BYTES (" +
                             std::to_string(static_cast<size_t>(RMS_NOALLOC_MAX_BYTES)) +
                             "); use fewer walkers or rms_run");
    DeviceScratch* d = nullptr;
    rc = device_scratch(sub->device, &d);
    if (rc) return rc;

    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    rms::DeviceRun dr;  // binds the scratch; owns no memory
    rc = dr.bind(*sub, r, false, stream, d->ptr);
    if (rc) return rc;
    return rms::execute_run(r, dr, stream, d->ev0, d->ev1, t0, out);
}
