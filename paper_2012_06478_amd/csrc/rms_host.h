// Host-side internals shared by rms_run (rms_api.cpp) and the server
// (rms_server.cpp): the substrate object, per-run preparation and the device
// buffers of one run.  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "rms.h"
#include "rms_internal.h"

struct rms_substrate {
    int device = 0;
    int label_bytes = 1;      // bytes per label of the caller's volume
    int dev_label_bytes = 1;  // bytes per entry of the padded device volume
    int64_t dims[3] = {0, 0, 0};
    double voxel_um = 0.0;
    int n_labels = 0;
    std::vector<double> D, kappa, T2;
    std::vector<uint8_t> dead;
    void* d_labels = nullptr;  // padded volume with halo flags (rms_internal.h)
    uint32_t* d_allowed = nullptr;
    uint32_t n_allowed = 0;
    std::vector<int64_t> label_count;  // voxels per label
};

namespace rms {

// (2 cos, 2 sin) of the angles 2 pi j / kTrigSize, each rounded once from
// long double (the factor 2 is exact), then kLeadCoefficients: the table of
// the double-precision direction draw (kTrigSize + 1 entries).
inline void fill_trig_table(double2* cs) {
    const long double two_pi = 6.283185307179586476925286766559005768394L;
    for (int j = 0; j < kTrigSize; ++j) {
        const long double t = two_pi * static_cast<long double>(j) / kTrigSize;
        cs[j].x = 2.0 * static_cast<double>(cosl(t));
        cs[j].y = 2.0 * static_cast<double>(sinl(t));
    }
    cs[kTrigSize] = kLeadCoefficients;
}

// Stream-ordered device allocation from the library's own pool on the
// current device (freed with hipFreeAsync).
hipError_t run_malloc(void** p, size_t bytes, hipStream_t s);

// Records a failure for rms_last_error() on the calling thread; returns code.
int fail(int code, const std::string& msg);
int hip_fail(const char* what, hipError_t e);
void clear_error();
const char* last_error();

// Everything a run needs that the host computes: validated sizes, per-label
// tables (section 2.1.3, 2.1.4) and per-shape waveform scaling (section 2.3).
struct RunSetup {
    const rms_substrate* sub = nullptr;
    uint64_t seed = 0;
    int64_t n_walkers = 0, n_steps = 0;
    double dt = 0.0;
    int precision = RMS_FP64;
    int n_shapes = 0, n_dirs = 0, n_b = 0, n_sig = 0;
    int n_acc = 0, width = 0, n_blocks = 0, n_res = 0;
    std::vector<double> sigma, inv_t2;
    std::vector<float> sigma_f, inv_t2_f;
    std::vector<uint64_t> thr;     // permeation thresholds floor(P 2^32) in [0, 2^32]
    std::vector<uint32_t> thr_mt;  // saturation thresholds (end of section 2.1.3), or empty
    std::vector<uint64_t> accept;  // start acceptance per label (spin concentrations), or empty
    double max_sigma = 0.0, max_p = 0.0;
    std::vector<double> gdt;
    std::vector<double2> trig;  // [kTrigSize + 1] angle table (fill_trig_table)
    std::vector<double> b_disc, kg, unit;
    std::vector<int> sig_shape;
};

// Validates the arguments of rms_run and fills `out`.  Returns RMS_OK or an
// RMS_E_* code (with the message recorded).
int prepare_run(const rms_substrate* sub, const rms_params* params, uint64_t seed,
                int64_t n_walkers, int64_t n_steps, double dt_ms, int n_shapes,
                const double* waveform, int n_dirs, const double* dirs, int n_b,
                const double* bvals, int precision, RunSetup& out);

// Device bytes a run holds while it is in flight (resumable: with the walker
// states a packed launch keeps between slices).
size_t device_bytes(const RunSetup& r, bool resumable);

// The device buffers of one run, uploaded on stream s and released
// stream-ordered on s.
struct DeviceRun {
    hipStream_t s = nullptr;
    std::vector<void*> ptrs;
    WalkPlan wp{};
    ReducePlan rp{};
    // allocates the run's block from the library's pool, then bind()s it
    int create(const rms_substrate& sub, const RunSetup& r, bool resumable, hipStream_t s);
    // device bytes of the run's block (every buffer, 256-byte aligned)
    static size_t layout_bytes(const rms_substrate& sub, const RunSetup& r, bool resumable);
    // lays the run's buffers out in `base` (at least layout_bytes(), owned by
    // the caller: release() does not free it) and uploads the tables on s
    int bind(const rms_substrate& sub, const RunSetup& r, bool resumable, hipStream_t s,
             void* base);
    void release();
    ~DeviceRun() { release(); }
};

// The device work of rms_run on buffers already laid out by dr (start
// attempts, walker order, walk, reductions), the copies of the results and
// the wait for them on `stream`; ev0 and ev1 bracket the walk launch.
// Fills `out` (wall_s from t0).
int execute_run(const RunSetup& r, DeviceRun& dr, hipStream_t stream, hipEvent_t ev0,
                hipEvent_t ev1, std::chrono::steady_clock::time_point t0, rms_result* out);

// Walker slots of servers created afterwards (RMS_OPT_SERVER_WALKERS; 0:
// automatic).
void set_server_walkers(int64_t walkers);

// Copies the reduced results (device layout of ReducePlan::result) into the
// caller's rms_result.
void fill_result(const RunSetup& r, const double* res, rms_result* out);

}  // namespace rms
