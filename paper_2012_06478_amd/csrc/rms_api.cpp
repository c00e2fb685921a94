// Host side of the C ABI declared in include/rms.h: argument validation,
// per-run tables, device buffers and kernel launches.  Every numerical step
// of the walk and of the reductions runs in the kernels; this file computes
// only the per-label and per-shape constants the kernels read.
#include "rms.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rms_internal.h"

struct rms_substrate {
    int device = 0;
    int label_bytes = 1;
    int64_t dims[3] = {0, 0, 0};
    double voxel_um = 0.0;
    int n_labels = 0;
    std::vector<double> D, kappa, T2;
    std::vector<uint8_t> dead;
    void* d_labels = nullptr;
    uint32_t* d_allowed = nullptr;
    uint32_t n_allowed = 0;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(const char* what, hipError_t e) {
    return fail(RMS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define RMS_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(#call, e_); \
    } while (0)

// Device buffers of one run, released on every exit path.
struct RunBuffers {
    hipStream_t s = nullptr;
    std::vector<void*> ptrs;
    ~RunBuffers() {
        if (!ptrs.empty()) {
            hipStreamSynchronize(s);
            for (void* p : ptrs) hipFreeAsync(p, s);
            hipStreamSynchronize(s);
        }
    }
    template <typename T>
    hipError_t alloc(T** p, size_t count) {
        void* q = nullptr;
        hipError_t e = hipMallocAsync(&q, std::max<size_t>(count, 1) * sizeof(T), s);
        if (e == hipSuccess) ptrs.push_back(q);
        *p = static_cast<T*>(q);
        return e;
    }
};

// Tissue tables of one run (section 2.1.3 and 2.1.4).
struct Tables {
    std::vector<double> sigma, inv_t2;
    std::vector<float> sigma_f, inv_t2_f;
    std::vector<uint32_t> thr;
    double max_sigma = 0.0, max_p = 0.0;
};

// Step length ds = sqrt(2 d D dt), d = 3, in voxel units (Eq. step-size).
// Permeation probability: solve Appendix C.1 for the input permeability that
// yields the genuine kappa, kappa0 = kappa / (1 + kappa (ds1/D1 + ds2/D2) C/2),
// and use P = kappa0 ds1 C / D1 (Eq. perm-prob) with C = C_3 = 2/3; this is
// Eq. (perm-prob-general).  A membrane word w (uniform on 0..2^32-1)
// permeates iff w < floor(P 2^32).
int build_tables(const rms_substrate& sub, const double* D, const double* kappa,
                 const double* T2, double dt, Tables& t) {
    const int L = sub.n_labels;
    const double C3 = 2.0 / 3.0;
    t.sigma.assign(L, 0.0);
    t.inv_t2.assign(L, 0.0);
    std::vector<double> ds(L, 0.0);
    for (int l = 0; l < L; ++l) {
        if (sub.dead[l]) continue;
        if (!(D[l] > 0.0) || !std::isfinite(D[l]))
            return fail(RMS_E_INVALID_ARG, "D[" + std::to_string(l) + "] must be > 0");
        ds[l] = std::sqrt(6.0 * D[l] * dt);
        t.sigma[l] = ds[l] / sub.voxel_um;
        t.max_sigma = std::max(t.max_sigma, t.sigma[l]);
        if (T2) {
            if (!(T2[l] > 0.0))
                return fail(RMS_E_INVALID_ARG, "T2[" + std::to_string(l) + "] must be > 0");
            t.inv_t2[l] = std::isinf(T2[l]) ? 0.0 : 1.0 / T2[l];
        }
    }
    if (!(t.max_sigma < 1.0))
        return fail(RMS_E_STEP_TOO_LARGE,
                    "step length " + std::to_string(t.max_sigma) +
                        " voxels: a step must be shorter than the voxel (at most three face "
                        "interactions per step)");
    t.thr.assign(static_cast<size_t>(L) * L, 0u);
    for (int a = 0; a < L; ++a) {
        for (int b = 0; b < L; ++b) {
            uint32_t th = 0;
            if (a == b) {
                th = 0xFFFFFFFFu;  // never consulted: equal labels pass
            } else if (!sub.dead[a] && !sub.dead[b] && kappa) {
                const double k = kappa[static_cast<size_t>(a) * L + b];
                if (!(k >= 0.0) || !std::isfinite(k))
                    return fail(RMS_E_INVALID_ARG, "kappa must be finite and >= 0");
                if (k != kappa[static_cast<size_t>(b) * L + a])
                    return fail(RMS_E_INVALID_ARG, "kappa must be symmetric");
                if (k > 0.0) {
                    const double k0 = k / (1.0 + 0.5 * k * C3 * (ds[a] / D[a] + ds[b] / D[b]));
                    const double P = std::min(1.0, k0 * ds[a] * C3 / D[a]);
                    t.max_p = std::max(t.max_p, P);
                    if (P > 0.5)
                        return fail(RMS_E_PROB_TOO_LARGE,
                                    "permeation probability " + std::to_string(P) +
                                        " > 0.5: lower dt or kappa");
                    th = static_cast<uint32_t>(std::floor(std::ldexp(P, 32)));
                }
            }
            t.thr[static_cast<size_t>(a) * L + b] = th;
        }
    }
    t.sigma_f.assign(t.sigma.begin(), t.sigma.end());
    t.inv_t2_f.assign(t.inv_t2.begin(), t.inv_t2.end());
    return RMS_OK;
}

}  // namespace

extern "C" {

int rms_abi_version(void) { return RMS_ABI_VERSION; }

const char* rms_last_error(void) { return g_err.c_str(); }

int rms_create_substrate(const void* labels, int label_bytes, const int64_t dims[3],
                         double voxel_um, int n_labels, const double* D, const double* kappa,
                         const double* T2, const uint8_t* dead, rms_substrate** out) {
    g_err.clear();
    if (!out) return fail(RMS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!labels || !dims || !D) return fail(RMS_E_INVALID_ARG, "labels, dims and D are required");
    if (label_bytes != 1 && label_bytes != 2)
        return fail(RMS_E_INVALID_ARG, "label_bytes must be 1 or 2");
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1)
        return fail(RMS_E_INVALID_ARG, "dims must be >= 1");
    const int64_t nvox = dims[0] * dims[1] * dims[2];
    if (dims[0] > (1 << 30) || dims[1] > (1 << 30) || dims[2] > (1 << 30) ||
        nvox >= (int64_t(1) << 31))
        return fail(RMS_E_INVALID_ARG, "volume must hold fewer than 2^31 voxels");
    if (!(voxel_um > 0.0) || !std::isfinite(voxel_um))
        return fail(RMS_E_INVALID_ARG, "voxel_um must be > 0");
    if (n_labels < 1 || n_labels > RMS_MAX_LABELS)
        return fail(RMS_E_INVALID_ARG, "n_labels must be in 1..RMS_MAX_LABELS");
    if (label_bytes == 1 && n_labels > 256)
        return fail(RMS_E_INVALID_ARG, "uint8 labels allow at most 256 labels");

    auto* sub = new (std::nothrow) rms_substrate;
    if (!sub) return fail(RMS_E_OOM, "host allocation failed");
    sub->label_bytes = label_bytes;
    for (int a = 0; a < 3; ++a) sub->dims[a] = dims[a];
    sub->voxel_um = voxel_um;
    sub->n_labels = n_labels;
    sub->D.assign(D, D + n_labels);
    if (kappa) sub->kappa.assign(kappa, kappa + static_cast<size_t>(n_labels) * n_labels);
    if (T2) sub->T2.assign(T2, T2 + n_labels);
    sub->dead.assign(n_labels, 0);
    if (dead)
        for (int l = 0; l < n_labels; ++l) sub->dead[l] = dead[l] ? 1 : 0;

    // every label in range; list the voxels a walker may start in
    std::vector<uint32_t> allowed;
    bool any_dead = false;
    for (int l = 0; l < n_labels; ++l) any_dead |= sub->dead[l] != 0;
    for (int64_t i = 0; i < nvox; ++i) {
        const int l = label_bytes == 1 ? static_cast<const uint8_t*>(labels)[i]
                                       : static_cast<const uint16_t*>(labels)[i];
        if (l >= n_labels) {
            delete sub;
            return fail(RMS_E_LABEL_RANGE, "voxel " + std::to_string(i) + " has label " +
                                               std::to_string(l) + " >= n_labels");
        }
        if (any_dead && !sub->dead[l]) allowed.push_back(static_cast<uint32_t>(i));
    }
    if (any_dead && allowed.empty()) {
        delete sub;
        return fail(RMS_E_INVALID_ARG, "every voxel is dead");
    }
    sub->n_allowed = any_dead ? static_cast<uint32_t>(allowed.size()) : static_cast<uint32_t>(nvox);

    hipError_t e = hipGetDevice(&sub->device);
    if (e == hipSuccess) e = hipMalloc(&sub->d_labels, static_cast<size_t>(nvox) * label_bytes);
    if (e == hipSuccess)
        e = hipMemcpy(sub->d_labels, labels, static_cast<size_t>(nvox) * label_bytes,
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && any_dead) {
        e = hipMalloc(reinterpret_cast<void**>(&sub->d_allowed), allowed.size() * sizeof(uint32_t));
        if (e == hipSuccess)
            e = hipMemcpy(sub->d_allowed, allowed.data(), allowed.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        const int rc = hip_fail(e == hipErrorOutOfMemory ? "device allocation" : "substrate upload", e);
        rms_destroy_substrate(sub);
        return e == hipErrorOutOfMemory ? fail(RMS_E_OOM, g_err) : rc;
    }
    *out = sub;
    return RMS_OK;
}

void rms_destroy_substrate(rms_substrate* sub) {
    if (!sub) return;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(sub->device);
    if (sub->d_labels) hipFree(sub->d_labels);
    if (sub->d_allowed) hipFree(sub->d_allowed);
    hipSetDevice(prev);
    delete sub;
}

int rms_run(const rms_substrate* sub, const rms_params* params, uint64_t seed, int64_t n_walkers,
            int64_t n_steps, double dt_ms, int n_shapes, const double* waveform, int n_dirs,
            const double* dirs, int n_b, const double* bvals, int precision, void* hip_stream,
            rms_result* out) {
    const auto t0 = std::chrono::steady_clock::now();
    g_err.clear();
    if (!sub || !out) return fail(RMS_E_INVALID_ARG, "substrate and result are required");
    if (n_walkers < 1) return fail(RMS_E_INVALID_ARG, "n_walkers must be >= 1");
    if (n_walkers > (int64_t(1) << 40)) return fail(RMS_E_INVALID_ARG, "n_walkers too large");
    if (n_steps < 0 || n_steps > 0xFFFFFFFELL)
        return fail(RMS_E_INVALID_ARG, "n_steps must be in [0, 2^32 - 2]");
    if (!(dt_ms > 0.0) || !std::isfinite(dt_ms)) return fail(RMS_E_INVALID_ARG, "dt must be > 0");
    if (n_shapes < 0 || n_shapes > RMS_MAX_SHAPES)
        return fail(RMS_E_INVALID_ARG, "n_shapes must be in 0..RMS_MAX_SHAPES");
    if (n_dirs < 0 || n_b < 0) return fail(RMS_E_INVALID_ARG, "n_dirs and n_b must be >= 0");
    if ((n_shapes > 0 && n_steps > 0 && !waveform) || (n_dirs > 0 && !dirs) || (n_b > 0 && !bvals))
        return fail(RMS_E_INVALID_ARG, "missing waveform, dirs or bvals");
    const int64_t n_sig64 = int64_t(n_shapes) * n_b * n_dirs;
    if (n_sig64 > RMS_MAX_SIGNALS)
        return fail(RMS_E_INVALID_ARG, "n_shapes * n_b * n_dirs exceeds RMS_MAX_SIGNALS");
    const int n_sig = static_cast<int>(n_sig64);
    if (precision != RMS_FP64 && precision != RMS_MIXED)
        return fail(RMS_E_INVALID_ARG, "precision must be RMS_FP64 or RMS_MIXED");

    const double* D = sub->D.data();
    const double* kappa = sub->kappa.empty() ? nullptr : sub->kappa.data();
    const double* T2 = sub->T2.empty() ? nullptr : sub->T2.data();
    if (params) {
        if (params->n_labels != sub->n_labels || !params->D)
            return fail(RMS_E_INVALID_ARG, "params must give D for every label of the substrate");
        D = params->D;
        kappa = params->kappa;
        T2 = params->T2;
    }
    Tables tab;
    int rc = build_tables(*sub, D, kappa, T2, dt_ms, tab);
    if (rc) return rc;

    // waveform scale: phi = sum_k Q_k g.dx_k with Q_k = dt sum_{i>=k} G_i, so the
    // discrete b of a unit shape is dt sum_k Q_k^2 (section 2.3, Eq. signal)
    std::vector<double> b_disc(n_shapes, 0.0), kscale(static_cast<size_t>(n_shapes) * n_b, 0.0);
    std::vector<double> gdt(static_cast<size_t>(n_shapes) * n_steps);
    for (int s = 0; s < n_shapes; ++s) {
        const double* G = waveform + static_cast<size_t>(s) * n_steps;
        double sum = 0.0, sabs = 0.0;
        for (int64_t i = 0; i < n_steps; ++i) {
            if (!std::isfinite(G[i])) return fail(RMS_E_INVALID_ARG, "waveform must be finite");
            sum += G[i];
            sabs += std::fabs(G[i]);
            gdt[static_cast<size_t>(s) * n_steps + i] = dt_ms * G[i];
        }
        if (std::fabs(sum) > 1e-9 * sabs)
            return fail(RMS_E_UNBALANCED_WAVEFORM,
                        "shape " + std::to_string(s) + " is not balanced (sum of samples " +
                            std::to_string(sum) + ")");
        double Q = 0.0, acc = 0.0;
        for (int64_t k = n_steps - 1; k >= 0; --k) {
            Q += dt_ms * G[k];
            acc += Q * Q;
        }
        b_disc[s] = dt_ms * acc;
        for (int j = 0; j < n_b; ++j) {
            if (!(bvals[j] >= 0.0) || !std::isfinite(bvals[j]))
                return fail(RMS_E_INVALID_ARG, "b values must be finite and >= 0");
            if (bvals[j] > 0.0 && !(b_disc[s] > 0.0))
                return fail(RMS_E_INVALID_ARG, "b > 0 needs a nonzero waveform shape");
            kscale[static_cast<size_t>(s) * n_b + j] =
                bvals[j] > 0.0 ? std::sqrt(bvals[j] / b_disc[s]) : 0.0;
        }
    }
    std::vector<double> unit(static_cast<size_t>(n_dirs) * 3);
    for (int d = 0; d < n_dirs; ++d) {
        const double* g = dirs + 3 * d;
        const double nrm = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        if (!(nrm > 0.0) || !std::isfinite(nrm))
            return fail(RMS_E_INVALID_ARG, "gradient directions must be nonzero");
        for (int a = 0; a < 3; ++a) unit[3 * d + a] = g[a] / nrm;
    }
    std::vector<double> kg(static_cast<size_t>(std::max(n_sig, 1)) * 3);
    std::vector<int> sig_shape(std::max(n_sig, 1));
    for (int s = 0; s < n_shapes; ++s)
        for (int j = 0; j < n_b; ++j)
            for (int d = 0; d < n_dirs; ++d) {
                const int q = (s * n_b + j) * n_dirs + d;
                for (int a = 0; a < 3; ++a)
                    kg[3 * q + a] = kscale[static_cast<size_t>(s) * n_b + j] * unit[3 * d + a];
                sig_shape[q] = s;
            }

    int prev_dev = 0;
    RMS_HIP(hipGetDevice(&prev_dev));
    struct DeviceGuard {
        int prev;
        ~DeviceGuard() { hipSetDevice(prev); }
    } guard{prev_dev};
    RMS_HIP(hipSetDevice(sub->device));

    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    RunBuffers buf;
    buf.s = stream;
    const int L = sub->n_labels;
    const int width = RMS_DUMP_WIDTH(n_shapes);
    const int n_acc = rms::kAccFixed + 2 * n_sig;
    const int n_blocks = static_cast<int>((n_walkers + rms::kBlock - 1) / rms::kBlock);
    const int n_res = n_acc + 2 * n_dirs;

    double *d_sigma, *d_it2, *d_gdt, *d_wstate, *d_kg, *d_partial, *d_sums, *d_res, *d_dirs;
    float *d_sigma_f, *d_it2_f, *d_gdt_f;
    uint32_t* d_thr;
    int* d_sig_shape;
    auto oom = [&](hipError_t e, const char* what) {
        return e == hipErrorOutOfMemory ? fail(RMS_E_OOM, std::string("device allocation: ") + what)
                                        : hip_fail(what, e);
    };
    hipError_t e = hipSuccess;
#define RMS_ALLOC(ptr, n)                                 \
    if ((e = buf.alloc(&ptr, (n))) != hipSuccess) return oom(e, #ptr)
    RMS_ALLOC(d_sigma, L);
    RMS_ALLOC(d_it2, L);
    RMS_ALLOC(d_sigma_f, L);
    RMS_ALLOC(d_it2_f, L);
    RMS_ALLOC(d_thr, static_cast<size_t>(L) * L);
    RMS_ALLOC(d_gdt, gdt.size());
    RMS_ALLOC(d_gdt_f, gdt.size());
    RMS_ALLOC(d_wstate, static_cast<size_t>(n_walkers) * width);
    RMS_ALLOC(d_kg, kg.size());
    RMS_ALLOC(d_sig_shape, sig_shape.size());
    RMS_ALLOC(d_partial, static_cast<size_t>(n_acc) * n_blocks);
    RMS_ALLOC(d_sums, n_acc);
    RMS_ALLOC(d_res, n_res);
    RMS_ALLOC(d_dirs, unit.size());
#undef RMS_ALLOC
    std::vector<float> gdt_f(gdt.begin(), gdt.end());
    RMS_HIP(hipMemcpyAsync(d_sigma, tab.sigma.data(), L * sizeof(double), hipMemcpyHostToDevice, stream));
    RMS_HIP(hipMemcpyAsync(d_it2, tab.inv_t2.data(), L * sizeof(double), hipMemcpyHostToDevice, stream));
    RMS_HIP(hipMemcpyAsync(d_sigma_f, tab.sigma_f.data(), L * sizeof(float), hipMemcpyHostToDevice, stream));
    RMS_HIP(hipMemcpyAsync(d_it2_f, tab.inv_t2_f.data(), L * sizeof(float), hipMemcpyHostToDevice, stream));
    RMS_HIP(hipMemcpyAsync(d_thr, tab.thr.data(), tab.thr.size() * sizeof(uint32_t), hipMemcpyHostToDevice, stream));
    if (!gdt.empty()) {
        RMS_HIP(hipMemcpyAsync(d_gdt, gdt.data(), gdt.size() * sizeof(double), hipMemcpyHostToDevice, stream));
        RMS_HIP(hipMemcpyAsync(d_gdt_f, gdt_f.data(), gdt_f.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    }
    RMS_HIP(hipMemcpyAsync(d_kg, kg.data(), kg.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    RMS_HIP(hipMemcpyAsync(d_sig_shape, sig_shape.data(), sig_shape.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    if (!unit.empty())
        RMS_HIP(hipMemcpyAsync(d_dirs, unit.data(), unit.size() * sizeof(double), hipMemcpyHostToDevice, stream));

    rms::WalkPlan wp{};
    wp.labels = sub->d_labels;
    wp.label_bytes = sub->label_bytes;
    wp.nx = static_cast<int>(sub->dims[0]);
    wp.ny = static_cast<int>(sub->dims[1]);
    wp.nz = static_cast<int>(sub->dims[2]);
    wp.allowed = sub->d_allowed;
    wp.n_allowed = sub->n_allowed;
    wp.n_labels = L;
    wp.sigma = d_sigma;
    wp.inv_t2 = d_it2;
    wp.thr = d_thr;
    wp.sigma_f = d_sigma_f;
    wp.inv_t2_f = d_it2_f;
    wp.seed = seed;
    wp.n_walkers = n_walkers;
    wp.n_steps = n_steps;
    wp.dt = dt_ms;
    wp.voxel_um = sub->voxel_um;
    wp.n_shapes = n_shapes;
    wp.gdt = d_gdt;
    wp.gdt_f = d_gdt_f;
    wp.wstate = d_wstate;
    wp.state = nullptr;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    RMS_HIP(hipEventCreate(&ev0));
    struct EventGuard {
        hipEvent_t a, b;
        ~EventGuard() {
            if (a) hipEventDestroy(a);
            if (b) hipEventDestroy(b);
        }
    } eguard{ev0, nullptr};
    RMS_HIP(hipEventCreate(&ev1));
    eguard.b = ev1;
    RMS_HIP(hipEventRecord(ev0, stream));
    e = rms::launch_walk(wp, precision, stream);
    if (e != hipSuccess) return hip_fail("walk kernel launch", e);
    RMS_HIP(hipEventRecord(ev1, stream));

    rms::ReducePlan rp{};
    rp.wstate = d_wstate;
    rp.n_walkers = n_walkers;
    rp.width = width;
    rp.n_shapes = n_shapes;
    rp.n_sig = n_sig;
    rp.kg = d_kg;
    rp.sig_shape = d_sig_shape;
    rp.n_acc = n_acc;
    rp.n_blocks = n_blocks;
    rp.partial = d_partial;
    rp.sums = d_sums;
    rp.n_dirs = n_dirs;
    rp.dirs = d_dirs;
    rp.t_ms = static_cast<double>(n_steps) * dt_ms;
    rp.result = d_res;
    e = rms::launch_reduce(rp, stream);
    if (e != hipSuccess) return hip_fail("reduction kernel launch", e);

    std::vector<double> res(n_res);
    RMS_HIP(hipMemcpyAsync(res.data(), d_res, n_res * sizeof(double), hipMemcpyDeviceToHost, stream));
    if (out->walker_dump)
        RMS_HIP(hipMemcpyAsync(out->walker_dump, d_wstate,
                               static_cast<size_t>(n_walkers) * width * sizeof(double),
                               hipMemcpyDeviceToHost, stream));
    RMS_HIP(hipStreamSynchronize(stream));
    float ms = 0.0f;
    RMS_HIP(hipEventElapsedTime(&ms, ev0, ev1));

    out->sum_alpha = res[0];
    for (int k = 0; k < 6; ++k) out->m2[k] = res[1 + k];
    for (int k = 0; k < 15; ++k) out->m4[k] = res[7 + k];
    out->n_face_events = static_cast<int64_t>(res[22]);
    out->n_membrane_hits = static_cast<int64_t>(res[23]);
    out->n_permeations = static_cast<int64_t>(res[24]);
    if (out->signal) std::memcpy(out->signal, res.data() + rms::kAccFixed, sizeof(double) * 2 * n_sig);
    if (out->D_dir) std::memcpy(out->D_dir, res.data() + n_acc, sizeof(double) * n_dirs);
    if (out->K_dir) std::memcpy(out->K_dir, res.data() + n_acc + n_dirs, sizeof(double) * n_dirs);
    if (out->b_disc) std::memcpy(out->b_disc, b_disc.data(), sizeof(double) * n_shapes);
    out->max_perm_prob = tab.max_p;
    out->max_step_over_voxel = tab.max_sigma;
    out->kernel_ms = ms;
    out->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return RMS_OK;
}

}  // extern "C"
