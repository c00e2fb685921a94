// Host side of the C ABI declared in include/rms.h: argument validation,
// per-run tables, device buffers and kernel launches of rms_run.  Every
// numerical step of the walk and of the reductions runs in the kernels; this
// file computes only the per-label and per-shape constants the kernels read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <mutex>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "rms_host.h"

namespace rms {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(const char* what, hipError_t e) {
    return fail(e == hipErrorOutOfMemory ? RMS_E_OOM : RMS_E_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

const char* last_error() { return g_err.c_str(); }

#define RMS_HIP(call)                                       \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return rms::hip_fail(#call, e_); \
    } while (0)

namespace {

// Step length ds = sqrt(2 d D dt), d = 3, in voxel units (Eq. step-size).
// Permeation probability: solve Appendix C.1 for the input permeability that
// yields the genuine kappa, kappa0 = kappa / (1 + kappa (ds1/D1 + ds2/D2) C/2),
// and use P = kappa0 ds1 C / D1 (Eq. perm-prob) with C = C_3 = 2/3; this is
// Eq. (perm-prob-general).  A membrane word w (uniform on 0..2^32-1)
// permeates iff w < floor(P 2^32).
//
// With spin concentrations c (App. C, general case) a membrane between labels
// a < b (side 1 = a) uses Eq. (gen-perm-prob): P_a->b = kappa0 ds_a C / D_a r^lam,
// P_b->a = kappa0 ds_b C / D_b r^(lam-1), r = c_b / c_a, with
// kappa0 = kappa / (1 + kappa A), A = (ds_a/D_a r^lam + ds_b/D_b r^(lam-1)) C/2
// (Eq. gen-kappa-correction); lam < 0 takes 1 / (1 + c_b sqrt(D_b) / (c_a
// sqrt(D_a))).  Baxter's rule (Eq. alt-perm-prob1-2): from the side of larger
// c sqrt(D) the probability is the ratio of the two, from the other 1.  The
// thresholds are 64-bit, so a probability of 1 is the threshold 2^32 that
// every 32-bit word lies below.
struct PermModel {
    const double* conc;  // or null: all equal
    double lambda;
    int model;           // RMS_PERM_KAPPA or RMS_PERM_BAXTER
};

int build_tables(const rms_substrate& sub, const double* D, const double* kappa,
                 const double* T2, double dt, const PermModel& pm, RunSetup& t) {
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
    constexpr uint64_t kAlways = uint64_t(1) << 32;
    t.thr.assign(static_cast<size_t>(L) * L, 0u);
    for (int a = 0; a < L; ++a) {
        for (int b = 0; b < L; ++b) {
            uint64_t th = 0;
            if (a == b) {
                th = kAlways;  // never consulted: equal labels pass
            } else if (!sub.dead[a] && !sub.dead[b] && kappa) {
                const double k = kappa[static_cast<size_t>(a) * L + b];
                if (!(k >= 0.0) || !std::isfinite(k))
                    return fail(RMS_E_INVALID_ARG, "kappa must be finite and >= 0");
                if (k != kappa[static_cast<size_t>(b) * L + a])
                    return fail(RMS_E_INVALID_ARG, "kappa must be symmetric");
                if (k > 0.0) {
                    double P;
                    if (pm.model == RMS_PERM_BAXTER) {
                        const double ha = (pm.conc ? pm.conc[a] : 1.0) * std::sqrt(D[a]);
                        const double hb = (pm.conc ? pm.conc[b] : 1.0) * std::sqrt(D[b]);
                        P = ha >= hb ? hb / ha : 1.0;
                    } else if (pm.conc) {
                        const int s1 = std::min(a, b), s2 = std::max(a, b);
                        const double c1 = pm.conc[s1], c2 = pm.conc[s2];
                        const double lam =
                            pm.lambda < 0.0
                                ? 1.0 / (1.0 + c2 * std::sqrt(D[s2]) / (c1 * std::sqrt(D[s1])))
                                : pm.lambda;
                        const double f12 = std::pow(c2 / c1, lam);
                        const double f21 = std::pow(c2 / c1, lam - 1.0);
                        const double A = 0.5 * C3 * (ds[s1] / D[s1] * f12 + ds[s2] / D[s2] * f21);
                        const double k0 = k / (1.0 + k * A);
                        P = std::min(1.0, a == s1 ? k0 * ds[s1] * C3 / D[s1] * f12
                                                  : k0 * ds[s2] * C3 / D[s2] * f21);
                    } else {
                        const double k0 = k / (1.0 + 0.5 * k * C3 * (ds[a] / D[a] + ds[b] / D[b]));
                        P = std::min(1.0, k0 * ds[a] * C3 / D[a]);
                    }
                    t.max_p = std::max(t.max_p, P);
                    if (pm.model != RMS_PERM_BAXTER && P > RMS_MAX_PERM_PROB)
                        return fail(RMS_E_PROB_TOO_LARGE,
                                    "permeation probability " + std::to_string(P) +
                                        " > RMS_MAX_PERM_PROB (0.1): lower dt or kappa");
                    th = P >= 1.0 ? kAlways
                                  : static_cast<uint64_t>(std::floor(std::ldexp(P, 32)));
                }
            }
            t.thr[static_cast<size_t>(a) * L + b] = th;
        }
    }
    t.sigma_f.assign(t.sigma.begin(), t.sigma.end());
    t.inv_t2_f.assign(t.inv_t2.begin(), t.inv_t2.end());
    return RMS_OK;
}

// Saturation thresholds at absorbing membranes (magnetization transfer, end
// of section 2.1.3): a walker in label a meeting label b is saturated with
// P_MT = rho[a][b] ds_a C_3 / D_a (C_3 of Eq. perm-prob); threshold
// floor(P_MT 2^32).  No table (the plain kernels) when no face absorbs.
int build_mt_table(const rms_substrate& sub, const double* D, const double* rho, double dt,
                   RunSetup& t) {
    const int L = sub.n_labels;
    const double C3 = 2.0 / 3.0;
    t.thr_mt.assign(static_cast<size_t>(L) * L, 0u);
    bool any = false;
    for (int a = 0; a < L; ++a) {
        for (int b = 0; b < L; ++b) {
            const double r = rho[static_cast<size_t>(a) * L + b];
            if (!(r >= 0.0) || !std::isfinite(r))
                return fail(RMS_E_INVALID_ARG, "rho must be finite and >= 0");
            if (a == b || sub.dead[a] || r == 0.0) continue;
            const double P = std::min(1.0, r * std::sqrt(6.0 * D[a] * dt) * C3 / D[a]);
            if (P > RMS_MAX_PERM_PROB)
                return fail(RMS_E_PROB_TOO_LARGE,
                            "saturation probability " + std::to_string(P) +
                                " > RMS_MAX_PERM_PROB (0.1): lower dt or rho");
            const uint32_t th = static_cast<uint32_t>(std::floor(std::ldexp(P, 32)));
            t.thr_mt[static_cast<size_t>(a) * L + b] = th;
            any |= th != 0u;
        }
    }
    if (!any) t.thr_mt.clear();
    return RMS_OK;
}

// Multiplier and shift for exact division of n < 2^31 by d >= 1:
// n / d == (n m) >> sh with sh = 31 + ceil(log2 d), m = ceil(2^sh / d) < 2^32.
void div_magic(uint32_t d, uint32_t* m, uint32_t* sh) {
    uint32_t s = 0;
    while ((uint64_t(1) << s) < d) ++s;
    *sh = 31 + s;
    *m = static_cast<uint32_t>(((uint64_t(1) << *sh) + d - 1) / d);
}

template <typename T>
hipError_t upload(T* dst, const std::vector<T>& src, hipStream_t s) {
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

}  // namespace

int prepare_run(const rms_substrate* sub, const rms_params* params, uint64_t seed,
                int64_t n_walkers, int64_t n_steps, double dt_ms, int n_shapes,
                const double* waveform, int n_dirs, const double* dirs, int n_b,
                const double* bvals, int precision, RunSetup& r) {
    if (!sub) return fail(RMS_E_INVALID_ARG, "substrate is required");
    if (n_walkers < 1) return fail(RMS_E_INVALID_ARG, "n_walkers must be >= 1");
    // walker indices are 32-bit (the high counter word of every stream is 0;
    // 2^32 - 1 marks an empty thread slot); the records alone of that many
    // walkers would need more than the device's memory
    if (n_walkers > 0xFFFFFFFELL)
        return fail(RMS_E_INVALID_ARG, "n_walkers must be in [1, 2^32 - 2]");
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
    if (precision != RMS_FP64 && precision != RMS_MIXED)
        return fail(RMS_E_INVALID_ARG, "precision must be RMS_FP64 or RMS_MIXED");

    r.sub = sub;
    r.seed = seed;
    r.n_walkers = n_walkers;
    r.n_steps = n_steps;
    r.dt = dt_ms;
    r.precision = precision;
    r.n_shapes = n_shapes;
    r.n_dirs = n_dirs;
    r.n_b = n_b;
    r.n_sig = static_cast<int>(n_sig64);
    r.width = RMS_DUMP_WIDTH(n_shapes);
    r.n_acc = kAccFixed + 2 * r.n_sig;
    // blocks of the contribution kernel: each thread folds up to four walkers
    r.n_blocks = static_cast<int>((n_walkers + 4 * kBlock - 1) / (4 * kBlock));
    r.n_res = r.n_acc + 2 * n_dirs;

    const double* D = sub->D.data();
    const double* kappa = sub->kappa.empty() ? nullptr : sub->kappa.data();
    const double* T2 = sub->T2.empty() ? nullptr : sub->T2.data();
    PermModel pm{nullptr, 0.0, RMS_PERM_KAPPA};
    if (params) {
        if (params->n_labels != sub->n_labels || !params->D)
            return fail(RMS_E_INVALID_ARG, "params must give D for every label of the substrate");
        D = params->D;
        kappa = params->kappa;
        T2 = params->T2;
        pm = PermModel{params->conc, params->lambda, params->perm_model};
        if (pm.model != RMS_PERM_KAPPA && pm.model != RMS_PERM_BAXTER)
            return fail(RMS_E_INVALID_ARG, "perm_model must be RMS_PERM_KAPPA or RMS_PERM_BAXTER");
        if (pm.conc && pm.model == RMS_PERM_KAPPA && !(pm.lambda <= 1.0))
            return fail(RMS_E_INVALID_ARG, "lambda must be <= 1 (negative: the closed form)");
    }
    if (pm.conc) {
        // start density proportional to the concentration (App. C, general case)
        const int L = sub->n_labels;
        double cmax = 0.0, csum = 0.0;
        for (int l = 0; l < L; ++l) {
            if (sub->dead[l]) continue;
            if (!(pm.conc[l] > 0.0) || !std::isfinite(pm.conc[l]))
                return fail(RMS_E_INVALID_ARG, "conc must be finite and > 0 for labels not dead");
            cmax = std::max(cmax, pm.conc[l]);
            csum += pm.conc[l] * static_cast<double>(sub->label_count[l]);
        }
        if (csum < 1e-3 * cmax * static_cast<double>(sub->n_allowed))
            return fail(RMS_E_INVALID_ARG, "conc: mean start acceptance below 1e-3");
        r.accept.assign(L, 0u);
        for (int l = 0; l < L; ++l)
            if (!sub->dead[l])
                r.accept[l] = static_cast<uint64_t>(std::floor(std::ldexp(pm.conc[l] / cmax, 32)));
    }
    int rc = build_tables(*sub, D, kappa, T2, dt_ms, pm, r);
    if (rc) return rc;
    if (params && params->rho) {
        rc = build_mt_table(*sub, D, params->rho, dt_ms, r);
        if (rc) return rc;
    }

    // waveform scale: phi = sum_k Q_k g.dx_k with Q_k = dt sum_{i>=k} G_i, so the
    // discrete b of a unit shape is dt sum_k Q_k^2 (section 2.3, Eq. signal)
    r.b_disc.assign(n_shapes, 0.0);
    std::vector<double> kscale(static_cast<size_t>(n_shapes) * n_b, 0.0);
    r.trig.resize(kTrigSize + 1);
    fill_trig_table(r.trig.data());
    r.gdt.assign(static_cast<size_t>(n_shapes) * n_steps, 0.0);
    for (int s = 0; s < n_shapes; ++s) {
        const double* G = waveform + static_cast<size_t>(s) * n_steps;
        double sum = 0.0, sabs = 0.0;
        for (int64_t i = 0; i < n_steps; ++i) {
            if (!std::isfinite(G[i])) return fail(RMS_E_INVALID_ARG, "waveform must be finite");
            sum += G[i];
            sabs += std::fabs(G[i]);
            r.gdt[static_cast<size_t>(s) * n_steps + i] = dt_ms * G[i];
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
        r.b_disc[s] = dt_ms * acc;
        for (int j = 0; j < n_b; ++j) {
            if (!(bvals[j] >= 0.0) || !std::isfinite(bvals[j]))
                return fail(RMS_E_INVALID_ARG, "b values must be finite and >= 0");
            if (bvals[j] > 0.0 && !(r.b_disc[s] > 0.0))
                return fail(RMS_E_INVALID_ARG, "b > 0 needs a nonzero waveform shape");
            kscale[static_cast<size_t>(s) * n_b + j] =
                bvals[j] > 0.0 ? std::sqrt(bvals[j] / r.b_disc[s]) : 0.0;
        }
    }
    r.unit.assign(static_cast<size_t>(n_dirs) * 3, 0.0);
    for (int d = 0; d < n_dirs; ++d) {
        const double* g = dirs + 3 * d;
        const double nrm = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        if (!(nrm > 0.0) || !std::isfinite(nrm))
            return fail(RMS_E_INVALID_ARG, "gradient directions must be nonzero");
        for (int a = 0; a < 3; ++a) r.unit[3 * d + a] = g[a] / nrm;
    }
    r.kg.assign(static_cast<size_t>(std::max(r.n_sig, 1)) * 3, 0.0);
    r.sig_shape.assign(std::max(r.n_sig, 1), 0);
    for (int s = 0; s < n_shapes; ++s)
        for (int j = 0; j < n_b; ++j)
            for (int d = 0; d < n_dirs; ++d) {
                const int q = (s * n_b + j) * n_dirs + d;
                for (int a = 0; a < 3; ++a)
                    r.kg[3 * q + a] = kscale[static_cast<size_t>(s) * n_b + j] * r.unit[3 * d + a];
                r.sig_shape[q] = s;
            }
    return RMS_OK;
}

size_t device_bytes(const RunSetup& r, bool resumable) {
    const size_t L = static_cast<size_t>(r.sub->n_labels);
    size_t b = L * (2 * sizeof(double) + 2 * sizeof(float)) + L * L * sizeof(uint64_t);
    b += r.thr_mt.size() * sizeof(uint32_t) + r.accept.size() * sizeof(uint64_t);
    if (!r.accept.empty()) b += static_cast<size_t>(r.n_walkers) * sizeof(uint32_t);
    b += r.gdt.size() * sizeof(double) + 2 * kTrigSize * sizeof(double);
    b += static_cast<size_t>(r.n_walkers) * r.width * sizeof(double);
    b += r.kg.size() * sizeof(double) + r.sig_shape.size() * sizeof(int);
    b += static_cast<size_t>(r.n_acc) * r.n_blocks * sizeof(double);
    b += (static_cast<size_t>(r.n_acc) + r.n_res + r.unit.size()) * sizeof(double);
    if (resumable)
        b += static_cast<size_t>(r.n_walkers) *
             walker_state_bytes(r.precision, r.sub->label_bytes, r.n_shapes);
    b += order_bytes(r.n_walkers);
    if (!resumable && seg_state_bytes(r.precision, r.n_shapes, r.n_walkers) > 0)
        b += seg_state_bytes(r.precision, r.n_shapes, r.n_walkers) + seg_ctl_bytes(r.n_walkers);
    return b + 64 * 1024;  // allocation granularity slack
}

// Device memory of the runs comes from a stream-ordered pool of the
// library's own, one per device (created at the first run there, kept until
// the process ends), not from the device's default pool that other code in
// the process may use.  Freed run memory stays in it, up to kPoolKeepBytes,
// instead of going back to the driver at each synchronization, so
// back-to-back runs do not map their memory again (0.2-0.4 ms a run).
constexpr uint64_t kPoolKeepBytes = uint64_t(4) << 30;
constexpr int kMaxDevices = 64;

hipError_t run_pool(hipMemPool_t* out) {
    static std::mutex m;
    static hipMemPool_t pools[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(m);
    if (!pools[dev]) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        e = hipMemPoolCreate(&pool, &props);
        if (e != hipSuccess) return e;
        uint64_t keep = kPoolKeepBytes;
        e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        if (e != hipSuccess) {
            (void)hipMemPoolDestroy(pool);
            return e;
        }
        pools[dev] = pool;
    }
    *out = pools[dev];
    return hipSuccess;
}

hipError_t run_malloc(void** p, size_t bytes, hipStream_t s) {
    hipMemPool_t pool = nullptr;
    const hipError_t e = run_pool(&pool);
    if (e != hipSuccess) return e;
    return hipMallocFromPoolAsync(p, bytes, pool, s);
}

// Offsets of every buffer of one run inside its single device block,
// 256-byte aligned pieces.
struct RunLayout {
    size_t sigma, it2, sigma_f, it2_f, thr, thr_mt, accept, start_try, gdt, trig, wstate, kg,
        sig_shape, partial, sums, res, dirs, state, order, seg_state, seg_ctl;
    size_t state_b, order_b, seg_b;
    size_t total;
};

RunLayout run_layout(const rms_substrate& sub, const RunSetup& r, bool resumable) {
    const size_t L = static_cast<size_t>(sub.n_labels);
    RunLayout o{};
    size_t total = 0;
    const auto take = [&total](size_t bytes) {
        const size_t off = total;
        total += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return off;
    };
    o.sigma = take(L * sizeof(double));
    o.it2 = take(L * sizeof(double));
    o.sigma_f = take(L * sizeof(float));
    o.it2_f = take(L * sizeof(float));
    o.thr = take(L * L * sizeof(uint64_t));
    o.thr_mt = take(r.thr_mt.size() * sizeof(uint32_t));
    o.accept = take(r.accept.size() * sizeof(uint64_t));
    o.start_try = take(r.accept.empty() ? 0 : static_cast<size_t>(r.n_walkers) * sizeof(uint32_t));
    o.gdt = take(r.gdt.size() * sizeof(double));
    o.trig = take((kTrigSize + 1) * sizeof(double2));
    o.wstate = take(static_cast<size_t>(r.n_walkers) * r.width * sizeof(double));
    o.kg = take(r.kg.size() * sizeof(double));
    o.sig_shape = take(r.sig_shape.size() * sizeof(int));
    o.partial = take(static_cast<size_t>(r.n_acc) * r.n_blocks * sizeof(double));
    o.sums = take(static_cast<size_t>(r.n_acc) * sizeof(double));
    o.res = take(static_cast<size_t>(r.n_res) * sizeof(double));
    o.dirs = take(r.unit.size() * sizeof(double));
    o.state_b = resumable ? static_cast<size_t>(r.n_walkers) *
                                walker_state_bytes(r.precision, sub.label_bytes, r.n_shapes)
                          : 0;
    o.state = take(o.state_b);
    o.order_b = order_bytes(r.n_walkers);
    o.order = take(o.order_b);
    o.seg_b = resumable ? 0 : seg_state_bytes(r.precision, r.n_shapes, r.n_walkers);
    o.seg_state = take(o.seg_b);
    o.seg_ctl = take(o.seg_b > 0 ? seg_ctl_bytes(r.n_walkers) : 0);
    o.total = total;
    return o;
}

int DeviceRun::create(const rms_substrate& sub, const RunSetup& r, bool resumable,
                      hipStream_t stream) {
    s = stream;
    // One device allocation for the whole run, carved into 256-byte aligned
    // pieces (an allocation and a free per buffer cost about 90 us each).
    void* base = nullptr;
    RMS_HIP(run_malloc(&base, run_layout(sub, r, resumable).total, s));
    ptrs.push_back(base);
    return bind(sub, r, resumable, stream, base);
}

size_t DeviceRun::layout_bytes(const rms_substrate& sub, const RunSetup& r, bool resumable) {
    return run_layout(sub, r, resumable).total;
}

int DeviceRun::bind(const rms_substrate& sub, const RunSetup& r, bool resumable,
                    hipStream_t stream, void* base) {
    s = stream;
    const RunLayout o = run_layout(sub, r, resumable);
    uint8_t* const b = static_cast<uint8_t*>(base);
    double* d_sigma = reinterpret_cast<double*>(b + o.sigma);
    double* d_it2 = reinterpret_cast<double*>(b + o.it2);
    float* d_sigma_f = reinterpret_cast<float*>(b + o.sigma_f);
    float* d_it2_f = reinterpret_cast<float*>(b + o.it2_f);
    uint64_t* d_thr = reinterpret_cast<uint64_t*>(b + o.thr);
    uint32_t* d_thr_mt = r.thr_mt.empty() ? nullptr : reinterpret_cast<uint32_t*>(b + o.thr_mt);
    uint64_t* d_accept = r.accept.empty() ? nullptr : reinterpret_cast<uint64_t*>(b + o.accept);
    uint32_t* d_start_try =
        r.accept.empty() ? nullptr : reinterpret_cast<uint32_t*>(b + o.start_try);
    double* d_gdt = reinterpret_cast<double*>(b + o.gdt);
    double2* d_trig = reinterpret_cast<double2*>(b + o.trig);
    double* d_wstate = reinterpret_cast<double*>(b + o.wstate);
    double* d_kg = reinterpret_cast<double*>(b + o.kg);
    int* d_sig_shape = reinterpret_cast<int*>(b + o.sig_shape);
    double* d_partial = reinterpret_cast<double*>(b + o.partial);
    double* d_sums = reinterpret_cast<double*>(b + o.sums);
    double* d_res = reinterpret_cast<double*>(b + o.res);
    double* d_dirs = reinterpret_cast<double*>(b + o.dirs);
    void* d_state = o.state_b ? static_cast<void*>(b + o.state) : nullptr;
    uint32_t* d_order = o.order_b ? reinterpret_cast<uint32_t*>(b + o.order) : nullptr;
    uint8_t* d_seg_state = o.seg_b ? b + o.seg_state : nullptr;
    uint32_t* d_seg_ctl = o.seg_b ? reinterpret_cast<uint32_t*>(b + o.seg_ctl) : nullptr;
    RMS_HIP(upload(d_sigma, r.sigma, s));
    RMS_HIP(upload(d_it2, r.inv_t2, s));
    RMS_HIP(upload(d_sigma_f, r.sigma_f, s));
    RMS_HIP(upload(d_it2_f, r.inv_t2_f, s));
    RMS_HIP(upload(d_thr, r.thr, s));
    if (d_thr_mt) RMS_HIP(upload(d_thr_mt, r.thr_mt, s));
    if (d_accept) RMS_HIP(upload(d_accept, r.accept, s));
    RMS_HIP(upload(d_gdt, r.gdt, s));
    RMS_HIP(upload(d_trig, r.trig, s));
    RMS_HIP(upload(d_kg, r.kg, s));
    RMS_HIP(upload(d_sig_shape, r.sig_shape, s));
    RMS_HIP(upload(d_dirs, r.unit, s));

    wp = WalkPlan{};
    wp.labels = sub.d_labels;
    wp.label_bytes = sub.dev_label_bytes;
    wp.nx = static_cast<int>(sub.dims[0]);
    wp.ny = static_cast<int>(sub.dims[1]);
    wp.nz = static_cast<int>(sub.dims[2]);
    wp.px = wp.nx + 2;
    wp.pxy = wp.px * (wp.ny + 2);
    div_magic(static_cast<uint32_t>(sub.dims[0]), &wp.div_nx_m, &wp.div_nx_sh);
    div_magic(static_cast<uint32_t>(sub.dims[0] * sub.dims[1]), &wp.div_nxy_m, &wp.div_nxy_sh);
    div_magic(static_cast<uint32_t>(wp.px), &wp.div_px_m, &wp.div_px_sh);
    div_magic(static_cast<uint32_t>(wp.pxy), &wp.div_pxy_m, &wp.div_pxy_sh);
    wp.allowed = sub.d_allowed;
    wp.accept = d_accept;
    wp.start_try = d_start_try;
    wp.n_allowed = sub.n_allowed;
    wp.n_labels = sub.n_labels;
    wp.sigma = d_sigma;
    wp.inv_t2 = d_it2;
    wp.thr = d_thr;
    wp.thr_mt = d_thr_mt;
    wp.sigma_f = d_sigma_f;
    wp.inv_t2_f = d_it2_f;
    wp.seed = r.seed;
    wp.n_walkers = r.n_walkers;
    wp.n_steps = r.n_steps;
    wp.dt = r.dt;
    wp.voxel_um = sub.voxel_um;
    wp.n_shapes = r.n_shapes;
    wp.gdt = d_gdt;
    wp.trig = d_trig;
    wp.wstate = d_wstate;
    wp.state = d_state;
    wp.order = d_order;
    wp.n_slots = d_order ? order_slots(r.n_walkers) : r.n_walkers;
    wp.seg_state = d_order ? d_seg_state : nullptr;
    wp.seg_ctl = d_order ? d_seg_ctl : nullptr;

    rp = ReducePlan{};
    rp.wstate = d_wstate;
    rp.n_walkers = r.n_walkers;
    rp.width = r.width;
    rp.n_shapes = r.n_shapes;
    rp.n_sig = r.n_sig;
    rp.kg = d_kg;
    rp.sig_shape = d_sig_shape;
    rp.n_acc = r.n_acc;
    rp.n_blocks = r.n_blocks;
    rp.partial = d_partial;
    rp.sums = d_sums;
    rp.n_dirs = r.n_dirs;
    rp.dirs = d_dirs;
    rp.t_ms = static_cast<double>(r.n_steps) * r.dt;
    rp.result = d_res;
    return RMS_OK;
}

void DeviceRun::release() {
    if (ptrs.empty()) return;
    (void)hipStreamSynchronize(s);
    for (void* p : ptrs) (void)hipFreeAsync(p, s);
    (void)hipStreamSynchronize(s);
    ptrs.clear();
}

int execute_run(const RunSetup& r, DeviceRun& dr, hipStream_t stream, hipEvent_t ev0,
                hipEvent_t ev1, std::chrono::steady_clock::time_point t0, rms_result* out) {
    RMS_HIP(launch_start_try(dr.wp, stream));
    RMS_HIP(launch_order(dr.wp, stream));
    RMS_HIP(hipEventRecord(ev0, stream));
    int kind = RMS_WALK_ONE_LAUNCH;
    RMS_HIP(launch_walk(dr.wp, r.precision, stream, &kind));
    RMS_HIP(hipEventRecord(ev1, stream));
    RMS_HIP(launch_reduce(dr.rp, stream));

    std::vector<double> res(r.n_res);
    RMS_HIP(hipMemcpyAsync(res.data(), dr.rp.result, r.n_res * sizeof(double),
                           hipMemcpyDeviceToHost, stream));
    uint32_t seg_fail = 0u;
    if (dr.wp.seg_ctl)
        RMS_HIP(hipMemcpyAsync(&seg_fail, dr.wp.seg_ctl + kSegErrorWord, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, stream));
    if (out->walker_dump)
        RMS_HIP(hipMemcpyAsync(out->walker_dump, dr.wp.wstate,
                               static_cast<size_t>(r.n_walkers) * r.width * sizeof(double),
                               hipMemcpyDeviceToHost, stream));
    RMS_HIP(hipStreamSynchronize(stream));
    if (seg_fail != 0u)
        return fail(RMS_E_WAIT_GAVE_UP,
                    "walk: a wave of the persistent walk gave up waiting for the previous "
                    "segment of its walkers; every wave stopped, no result");
    float ms = 0.0f;
    RMS_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    fill_result(r, res.data(), out);
    out->kernel_ms = ms;
    out->queue_s = 0.0;
    out->walk_kernel = kind;
    out->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return RMS_OK;
}

void fill_result(const RunSetup& r, const double* res, rms_result* out) {
    out->sum_alpha = res[0];
    for (int k = 0; k < 6; ++k) out->m2[k] = res[1 + k];
    for (int k = 0; k < 15; ++k) out->m4[k] = res[7 + k];
    out->n_face_events = static_cast<int64_t>(res[22]);
    out->n_membrane_hits = static_cast<int64_t>(res[23]);
    out->n_permeations = static_cast<int64_t>(res[24]);
    if (out->signal) std::memcpy(out->signal, res + kAccFixed, sizeof(double) * 2 * r.n_sig);
    if (out->D_dir) std::memcpy(out->D_dir, res + r.n_acc, sizeof(double) * r.n_dirs);
    if (out->K_dir) std::memcpy(out->K_dir, res + r.n_acc + r.n_dirs, sizeof(double) * r.n_dirs);
    if (out->b_disc) std::memcpy(out->b_disc, r.b_disc.data(), sizeof(double) * r.n_shapes);
    out->max_perm_prob = r.max_p;
    out->max_step_over_voxel = r.max_sigma;
}

namespace {

// Host threads for the passes over a label volume (the 400x400x1000 volume
// took about 0.5 s on one core): up to 16, one for small volumes.
int volume_threads(int64_t nvox) {
    if (nvox < (int64_t(1) << 22)) return 1;
    const unsigned hc = std::thread::hardware_concurrency();
    return hc == 0 ? 1 : static_cast<int>(std::min(hc, 16u));
}

// f(begin, end, t) over nt contiguous ranges of [0, n) on nt threads; ranges
// whose thread could not be started run on the calling thread.
template <class F>
void parallel_ranges(int64_t n, int nt, const F& f) {
    std::vector<std::thread> th;
    int started = 1;
    try {
        th.reserve(static_cast<size_t>(nt));
        for (int t = 1; t < nt; ++t) {
            th.emplace_back(f, n * t / nt, n * (t + 1) / nt, t);
            ++started;
        }
    } catch (...) {
    }
    f(int64_t(0), n / nt, 0);
    for (int t = started; t < nt; ++t) f(n * t / nt, n * (t + 1) / nt, t);
    for (auto& x : th) x.join();
}

// Voxels per label over [b, e); the index of the first voxel whose label is
// out of range (or -1), and, with dead labels, the voxels a walker may start in.
template <typename T>
void scan_labels(const T* lab, int64_t b, int64_t e, int n_labels, const uint8_t* dead,
                 int64_t* count, int64_t* first_bad, std::vector<uint32_t>* allowed) {
    for (int64_t i = b; i < e; ++i) {
        const uint32_t l = lab[i];
        if (l >= static_cast<uint32_t>(n_labels)) {
            *first_bad = i;
            return;
        }
        ++count[l];
        if (dead && !dead[l]) allowed->push_back(static_cast<uint32_t>(i));
    }
}

// Padded planes [zb, ze) of the device volume: each entry the label of the
// voxel it stands for (periodic wrap in the halo) with the halo flags of the
// axes along which it lies outside the volume in the bits from `shift` up.
template <typename Src, typename Dst>
void pad_planes(const Src* lab, Dst* pad, int64_t nx, int64_t ny, int64_t nz, int shift,
                int64_t zb, int64_t ze) {
    const int64_t px = nx + 2, py = ny + 2, pz = nz + 2;
    for (int64_t zp = zb; zp < ze; ++zp) {
        const int64_t z = (zp + nz - 1) % nz;
        const uint32_t fz = zp == 0 || zp == pz - 1 ? 4u : 0u;
        for (int64_t yp = 0; yp < py; ++yp) {
            const int64_t y = (yp + ny - 1) % ny;
            const uint32_t f = fz | (yp == 0 || yp == py - 1 ? 2u : 0u);
            const Src* src = lab + (z * ny + y) * nx;
            Dst* dst = pad + (zp * py + yp) * px;
            const uint32_t fi = f << shift, fh = (f | 1u) << shift;
            for (int64_t x = 0; x < nx; ++x) dst[x + 1] = static_cast<Dst>(src[x] | fi);
            dst[0] = static_cast<Dst>(src[nx - 1] | fh);
            dst[nx + 1] = static_cast<Dst>(src[0] | fh);
        }
    }
}

template <typename Dst>
void pad_volume(const void* labels, int label_bytes, Dst* pad, const int64_t dims[3], int shift,
                int nt) {
    parallel_ranges(dims[2] + 2, nt, [&](int64_t zb, int64_t ze, int) {
        if (label_bytes == 1)
            pad_planes(static_cast<const uint8_t*>(labels), pad, dims[0], dims[1], dims[2], shift,
                       zb, ze);
        else
            pad_planes(static_cast<const uint16_t*>(labels), pad, dims[0], dims[1], dims[2],
                       shift, zb, ze);
    });
}

}  // namespace

}  // namespace rms

extern "C" {

int rms_abi_version(void) { return RMS_ABI_VERSION; }

const char* rms_last_error(void) { return rms::last_error(); }

int rms_create_substrate(const void* labels, int label_bytes, const int64_t dims[3],
                         double voxel_um, int n_labels, const double* D, const double* kappa,
                         const double* T2, const uint8_t* dead, rms_substrate** out) {
    using rms::fail;
    rms::clear_error();
    if (!out) return fail(RMS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!labels || !dims || !D) return fail(RMS_E_INVALID_ARG, "labels, dims and D are required");
    if (label_bytes != 1 && label_bytes != 2)
        return fail(RMS_E_INVALID_ARG, "label_bytes must be 1 or 2");
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1)
        return fail(RMS_E_INVALID_ARG, "dims must be >= 1");
    if (dims[0] > (1 << 30) || dims[1] > (1 << 30) || dims[2] > (1 << 30) ||
        (dims[0] + 2) * (dims[1] + 2) * (dims[2] + 2) >= (int64_t(1) << 31))
        return fail(RMS_E_INVALID_ARG,
                    "volume with its one-voxel halo must hold fewer than 2^31 voxels");
    const int64_t nvox = dims[0] * dims[1] * dims[2];
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

    // every label in range; list the voxels a walker may start in (per
    // thread over contiguous ranges, joined in voxel order)
    std::vector<uint32_t> allowed;
    bool any_dead = false;
    for (int l = 0; l < n_labels; ++l) any_dead |= sub->dead[l] != 0;
    sub->label_count.assign(n_labels, 0);
    const int nt = rms::volume_threads(nvox);
    std::vector<std::vector<int64_t>> counts;
    std::vector<std::vector<uint32_t>> allowed_t;
    std::vector<int64_t> first_bad;
    std::vector<uint8_t> oom;
    try {
        counts.assign(nt, std::vector<int64_t>(n_labels, 0));
        allowed_t.resize(nt);
        first_bad.assign(nt, -1);
        oom.assign(nt, 0);
        rms::parallel_ranges(nvox, nt, [&](int64_t b, int64_t e, int t) {
            const uint8_t* dl = any_dead ? sub->dead.data() : nullptr;
            try {  // nothing may leave a thread's function
                if (label_bytes == 1)
                    rms::scan_labels(static_cast<const uint8_t*>(labels), b, e, n_labels, dl,
                                     counts[t].data(), &first_bad[t], &allowed_t[t]);
                else
                    rms::scan_labels(static_cast<const uint16_t*>(labels), b, e, n_labels, dl,
                                     counts[t].data(), &first_bad[t], &allowed_t[t]);
            } catch (...) {
                oom[t] = 1;
            }
        });
        if (std::find(oom.begin(), oom.end(), uint8_t(1)) != oom.end()) throw std::bad_alloc();
        for (int t = 0; t < nt; ++t) {
            if (first_bad[t] >= 0) {  // the ranges are in voxel order: the first one found
                const int64_t i = first_bad[t];
                const int l = label_bytes == 1 ? static_cast<const uint8_t*>(labels)[i]
                                               : static_cast<const uint16_t*>(labels)[i];
                delete sub;
                return fail(RMS_E_LABEL_RANGE, "voxel " + std::to_string(i) + " has label " +
                                                   std::to_string(l) + " >= n_labels");
            }
            for (int l = 0; l < n_labels; ++l) sub->label_count[l] += counts[t][l];
            allowed.insert(allowed.end(), allowed_t[t].begin(), allowed_t[t].end());
            std::vector<uint32_t>().swap(allowed_t[t]);
        }
    } catch (const std::bad_alloc&) {
        delete sub;
        return fail(RMS_E_OOM, "host allocation failed");
    }
    if (any_dead && allowed.empty()) {
        delete sub;
        return fail(RMS_E_INVALID_ARG, "every voxel is dead");
    }
    sub->n_allowed = any_dead ? static_cast<uint32_t>(allowed.size()) : static_cast<uint32_t>(nvox);

    // padded device volume with the periodic halo and its flags
    sub->dev_label_bytes = label_bytes == 1 && n_labels <= rms::kMaxLabelsU8 ? 1 : 2;
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    const int64_t px = nx + 2, py = ny + 2, pz = nz + 2;
    const int shift = rms::halo_shift(sub->dev_label_bytes);
    const size_t n_pad = static_cast<size_t>(px * py * pz);
    std::unique_ptr<uint16_t[]> pad16;  // every entry is written below
    std::unique_ptr<uint8_t[]> pad8;
    if (sub->dev_label_bytes == 1) pad8.reset(new (std::nothrow) uint8_t[n_pad]);
    else pad16.reset(new (std::nothrow) uint16_t[n_pad]);
    if (!pad8 && !pad16) {
        delete sub;
        return fail(RMS_E_OOM, "host allocation failed");
    }
    if (sub->dev_label_bytes == 1) rms::pad_volume(labels, label_bytes, pad8.get(), dims, shift, nt);
    else rms::pad_volume(labels, label_bytes, pad16.get(), dims, shift, nt);
    const size_t pad_bytes = n_pad * sub->dev_label_bytes;
    const void* pad_src = sub->dev_label_bytes == 1 ? static_cast<const void*>(pad8.get())
                                                    : static_cast<const void*>(pad16.get());

    hipError_t e = hipGetDevice(&sub->device);
    if (e == hipSuccess) e = hipMalloc(&sub->d_labels, pad_bytes);
    if (e == hipSuccess) e = hipMemcpy(sub->d_labels, pad_src, pad_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && any_dead) {
        e = hipMalloc(reinterpret_cast<void**>(&sub->d_allowed), allowed.size() * sizeof(uint32_t));
        if (e == hipSuccess)
            e = hipMemcpy(sub->d_allowed, allowed.data(), allowed.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        const int rc = rms::hip_fail("substrate upload", e);
        rms_destroy_substrate(sub);
        return rc;
    }
    *out = sub;
    return RMS_OK;
}

void rms_destroy_substrate(rms_substrate* sub) {
    if (!sub) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(sub->device);
    if (sub->d_labels) (void)hipFree(sub->d_labels);
    if (sub->d_allowed) (void)hipFree(sub->d_allowed);
    (void)hipSetDevice(prev);
    delete sub;
}

int rms_run(const rms_substrate* sub, const rms_params* params, uint64_t seed, int64_t n_walkers,
            int64_t n_steps, double dt_ms, int n_shapes, const double* waveform, int n_dirs,
            const double* dirs, int n_b, const double* bvals, int precision, void* hip_stream,
            rms_result* out) {
    const auto t0 = std::chrono::steady_clock::now();
    rms::clear_error();
    if (!out) return rms::fail(RMS_E_INVALID_ARG, "result is required");
    rms::RunSetup r;
    int rc = rms::prepare_run(sub, params, seed, n_walkers, n_steps, dt_ms, n_shapes, waveform,
                              n_dirs, dirs, n_b, bvals, precision, r);
    if (rc) return rc;

    int prev_dev = 0;
    RMS_HIP(hipGetDevice(&prev_dev));
    struct DeviceGuard {
        int prev;
        ~DeviceGuard() { (void)hipSetDevice(prev); }
    } guard{prev_dev};
    RMS_HIP(hipSetDevice(sub->device));

    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    rms::DeviceRun dr;
    rc = dr.create(*sub, r, false, stream);
    if (rc) return rc;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    struct EventGuard {
        hipEvent_t* a;
        hipEvent_t* b;
        ~EventGuard() {
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
        }
    } eguard{&ev0, &ev1};
    RMS_HIP(hipEventCreate(&ev0));
    RMS_HIP(hipEventCreate(&ev1));
    return rms::execute_run(r, dr, stream, ev0, ev1, t0, out);
}

int rms_set_option(int option, int64_t value) {
    rms::clear_error();
    switch (option) {
        case RMS_OPT_WALK_KERNEL:
            if (value != RMS_WALK_AUTO && value != RMS_WALK_ONE_LAUNCH &&
                value != RMS_WALK_PERSISTENT)
                return rms::fail(RMS_E_INVALID_ARG, "RMS_OPT_WALK_KERNEL: RMS_WALK_AUTO, "
                                                    "RMS_WALK_ONE_LAUNCH or RMS_WALK_PERSISTENT");
            rms::set_walk_choice(static_cast<int>(value));
            return RMS_OK;
        case RMS_OPT_SERVER_WALKERS:
            if (value < 0)
                return rms::fail(RMS_E_INVALID_ARG, "RMS_OPT_SERVER_WALKERS: >= 0 (0: automatic)");
            rms::set_server_walkers(value);
            return RMS_OK;
        case RMS_OPT_SEG_POLL_LIMIT:
            if (value < 0 || value > int64_t(0xFFFFFFFEu))
                return rms::fail(RMS_E_INVALID_ARG, "RMS_OPT_SEG_POLL_LIMIT: 0 .. 2^32 - 2 polls");
            rms::set_seg_poll_limit(static_cast<uint32_t>(value));
            return RMS_OK;
        default:
            return rms::fail(RMS_E_INVALID_ARG, "unknown option " + std::to_string(option));
    }
}

int rms_spherical_mean(int n_b, int n_dirs, const double* signal, double* out) {
    rms::clear_error();
    if (n_b < 1 || n_dirs < 1 || !signal || !out)
        return rms::fail(RMS_E_INVALID_ARG, "spherical mean: n_b, n_dirs >= 1 and arrays required");
    for (int j = 0; j < n_b; ++j) {
        double re = 0.0, im = 0.0;
        for (int d = 0; d < n_dirs; ++d) {
            re += signal[(static_cast<size_t>(j) * n_dirs + d) * 2];
            im += signal[(static_cast<size_t>(j) * n_dirs + d) * 2 + 1];
        }
        out[2 * j] = re / n_dirs;
        out[2 * j + 1] = im / n_dirs;
    }
    return RMS_OK;
}

// Per direction: y_j = ln Re S(b_j) = a1 b_j + a2 b_j^2 over 0 < b_j <= b_max,
// least squares through the origin (the normal equations of the two-column
// design [b, b^2]); D = -a1 and K = 6 a2 / a1^2.
int rms_cumulant_fit(int n_b, const double* bvals, int n_dirs, const double* signal,
                     double b_max, double* D_out, double* K_out) {
    rms::clear_error();
    if (n_b < 1 || n_dirs < 1 || !bvals || !signal || !D_out || !K_out)
        return rms::fail(RMS_E_INVALID_ARG, "cumulant fit: sizes and arrays required");
    int used = 0;
    for (int j = 0; j < n_b; ++j) used += bvals[j] > 0.0 && bvals[j] <= b_max;
    if (used < 2)
        return rms::fail(RMS_E_INVALID_ARG, "cumulant fit: needs two b values in (0, b_max]");
    for (int d = 0; d < n_dirs; ++d) {
        double s11 = 0.0, s12 = 0.0, s22 = 0.0, t1 = 0.0, t2 = 0.0;
        for (int j = 0; j < n_b; ++j) {
            const double b = bvals[j];
            if (!(b > 0.0 && b <= b_max)) continue;
            const double S = signal[(static_cast<size_t>(j) * n_dirs + d) * 2];
            if (!(S > 0.0)) return rms::fail(RMS_E_INVALID_ARG, "cumulant fit: signal <= 0");
            const double y = std::log(S);
            s11 += b * b;
            s12 += b * b * b;
            s22 += b * b * b * b;
            t1 += b * y;
            t2 += b * b * y;
        }
        const double det = s11 * s22 - s12 * s12;
        const double a1 = (t1 * s22 - t2 * s12) / det;
        const double a2 = (s11 * t2 - s12 * t1) / det;
        D_out[d] = -a1;
        K_out[d] = 6.0 * a2 / (a1 * a1);
    }
    return RMS_OK;
}

int rms_run_record(const rms_substrate* sub, const rms_params* params, uint64_t seed,
                   int64_t n_walkers, int64_t n_steps, double dt_ms, int n_shapes,
                   const double* waveform, int n_dirs, const double* dirs, int n_b,
                   const double* bvals, int precision, void* hip_stream, const rms_record* rec,
                   rms_result* out) {
    using rms::fail;
    const auto t0 = std::chrono::steady_clock::now();
    rms::clear_error();
    if (!out) return fail(RMS_E_INVALID_ARG, "result is required");
    if (!rec) return fail(RMS_E_INVALID_ARG, "record list is required");
    if (rec->n_rec < 1 || rec->n_rec > RMS_MAX_RECORDS)
        return fail(RMS_E_INVALID_ARG, "n_rec must be in 1..RMS_MAX_RECORDS");
    if (!rec->steps || !rec->sum_alpha || !rec->m2 || !rec->m4)
        return fail(RMS_E_INVALID_ARG, "record steps, sum_alpha, m2 and m4 are required");
    rms::RunSetup r;
    int rc = rms::prepare_run(sub, params, seed, n_walkers, n_steps, dt_ms, n_shapes, waveform,
                              n_dirs, dirs, n_b, bvals, precision, r);
    if (rc) return rc;
    const int n_rec = rec->n_rec;
    for (int k = 0; k < n_rec; ++k)
        if (rec->steps[k] < 1 || rec->steps[k] > n_steps ||
            (k > 0 && rec->steps[k] <= rec->steps[k - 1]))
            return fail(RMS_E_INVALID_ARG, "record steps must ascend strictly within 1..n_steps");

    int prev_dev = 0;
    RMS_HIP(hipGetDevice(&prev_dev));
    struct DeviceGuard {
        int prev;
        ~DeviceGuard() { (void)hipSetDevice(prev); }
    } guard{prev_dev};
    RMS_HIP(hipSetDevice(sub->device));

    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    rms::DeviceRun dr;
    rc = dr.create(*sub, r, true, stream);
    if (rc) return rc;

    // Two walk plans that differ only in the buffer the walker records go to,
    // the items of the two halves of the thread slots for each plan (one item
    // per block; their step range is set on the device before each interval),
    // and the reduced values of each record (the layout of ReducePlan::result
    // without signals).  The halves walk on two streams and the records of
    // consecutive intervals alternate between the two buffers, so one half's
    // next interval fills the partly idle last round of waves of the other
    // half's, and a record is reduced while the walk goes on.  The result is
    // the same: each walker's steps and each reduction are unchanged.
    const int64_t n_items64 = (dr.wp.n_slots + rms::kBlock - 1) / rms::kBlock;
    if (n_items64 > INT32_MAX) return fail(RMS_E_INVALID_ARG, "too many walkers");
    const int n_items = static_cast<int>(n_items64);
    // half A is a multiple of 8 blocks, so every block keeps the XCD (block
    // index mod 8) its walkers were ordered for
    const int h_a = n_items >= 16 ? n_items / 2 / 8 * 8 : n_items;
    const int h_b = n_items - h_a;
    const int rec_stride = rms::kAccFixed + 2 * n_dirs;
    const size_t items_b = (static_cast<size_t>(n_items) * sizeof(rms::PackedItem) + 255) / 256 * 256;
    const size_t wst_b = (static_cast<size_t>(n_walkers) * r.width * sizeof(double) + 255) / 256 * 256;
    const size_t o_items = (2 * sizeof(rms::WalkPlan) + 255) / 256 * 256;  // plans[2], an array
    const size_t o_rec = o_items + 2 * items_b;
    const size_t o_wst = o_rec + (static_cast<size_t>(n_rec) * rec_stride * sizeof(double) + 255) /
                                     256 * 256;
    const size_t extra = o_wst + wst_b;
    void* xb = nullptr;
    RMS_HIP(rms::run_malloc(&xb, extra, stream));
    dr.ptrs.push_back(xb);
    uint8_t* xbase = static_cast<uint8_t*>(xb);
    auto* d_plan = reinterpret_cast<rms::WalkPlan*>(xbase);
    auto* d_rec = reinterpret_cast<double*>(xbase + o_rec);
    double* wst[2] = {dr.wp.wstate, reinterpret_cast<double*>(xbase + o_wst)};
    rms::PackedItem* d_items[2] = {reinterpret_cast<rms::PackedItem*>(xbase + o_items),
                                   reinterpret_cast<rms::PackedItem*>(xbase + o_items + items_b)};
    rms::WalkPlan plans[2] = {dr.wp, dr.wp};
    plans[1].wstate = wst[1];
    RMS_HIP(hipMemcpyAsync(d_plan, plans, sizeof(plans), hipMemcpyHostToDevice, stream));
    // host staging must outlive the asynchronous copies: keep both item lists
    std::vector<rms::PackedItem> items(2 * static_cast<size_t>(n_items));
    for (int q = 0; q < 2; ++q) {
        for (int i = 0; i < n_items; ++i)
            items[static_cast<size_t>(q) * n_items + i] =
                rms::PackedItem{static_cast<int64_t>(i) * rms::kBlock, q, 0u, 0u, 0u};
        RMS_HIP(hipMemcpyAsync(d_items[q], items.data() + static_cast<size_t>(q) * n_items,
                               static_cast<size_t>(n_items) * sizeof(rms::PackedItem),
                               hipMemcpyHostToDevice, stream));
    }

    // events and the second stream; on every exit the first stream waits for
    // the second before the run's memory is released
    std::vector<hipEvent_t> events;
    hipStream_t sb = nullptr;
    struct StreamGuard {
        hipStream_t a;
        hipStream_t* b;
        std::vector<hipEvent_t>* ev;
        ~StreamGuard() {
            if (*b) {
                hipEvent_t e = nullptr;
                if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) {
                    (void)hipEventRecord(e, *b);
                    (void)hipStreamWaitEvent(a, e, 0);
                    (void)hipEventDestroy(e);
                }
                (void)hipStreamDestroy(*b);
            }
            for (hipEvent_t e : *ev) (void)hipEventDestroy(e);
        }
    } sguard{stream, &sb, &events};
    const auto new_event = [&](bool timing, hipEvent_t* e) -> hipError_t {
        *e = nullptr;
        const hipError_t err = timing ? hipEventCreate(e)
                                      : hipEventCreateWithFlags(e, hipEventDisableTiming);
        if (err == hipSuccess) events.push_back(*e);
        return err;
    };
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_setup = nullptr;
    RMS_HIP(new_event(true, &ev0));
    RMS_HIP(new_event(true, &ev1));
    RMS_HIP(new_event(false, &ev_setup));
    if (h_b > 0) RMS_HIP(hipStreamCreateWithFlags(&sb, hipStreamNonBlocking));
    RMS_HIP(rms::launch_start_try(dr.wp, stream));
    RMS_HIP(rms::launch_order(dr.wp, stream));
    RMS_HIP(hipEventRecord(ev0, stream));
    if (sb) {
        RMS_HIP(hipEventRecord(ev_setup, stream));
        RMS_HIP(hipStreamWaitEvent(sb, ev_setup, 0));
    }
    std::vector<hipEvent_t> ev_b(static_cast<size_t>(n_rec) + 1, nullptr);
    std::vector<hipEvent_t> ev_r(static_cast<size_t>(n_rec), nullptr);
    const bool mt = !r.thr_mt.empty();
    int last_q = 0;
    int64_t b = 0;
    for (int k = 0; k <= n_rec; ++k) {
        const int64_t e = k < n_rec ? rec->steps[k] : n_steps;
        const int q = k % 2;  // record buffer of this interval
        if (e > b) {  // one launch per half and interval; an intermediate end writes the records
            const uint32_t flags = e < n_steps ? rms::kItemRecord : 0u;
            RMS_HIP(rms::launch_item_range(d_items[q], h_a, static_cast<uint32_t>(b),
                                           static_cast<uint32_t>(e), flags, stream));
            RMS_HIP(rms::launch_walk_packed(d_items[q], h_a, d_plan, precision,
                                            sub->dev_label_bytes, r.n_shapes, mt, stream));
            if (sb) {
                // buffer q was last read by the reduction of record k - 2
                if (k >= 2 && ev_r[k - 2]) RMS_HIP(hipStreamWaitEvent(sb, ev_r[k - 2], 0));
                RMS_HIP(rms::launch_item_range(d_items[q] + h_a, h_b, static_cast<uint32_t>(b),
                                               static_cast<uint32_t>(e), flags, sb));
                RMS_HIP(rms::launch_walk_packed(d_items[q] + h_a, h_b, d_plan, precision,
                                                sub->dev_label_bytes, r.n_shapes, mt, sb));
                RMS_HIP(new_event(false, &ev_b[k]));
                RMS_HIP(hipEventRecord(ev_b[k], sb));
            }
            last_q = q;
            b = e;
        }
        if (k < n_rec) {
            if (sb && ev_b[k]) RMS_HIP(hipStreamWaitEvent(stream, ev_b[k], 0));
            rms::ReducePlan rr = dr.rp;
            rr.wstate = wst[q];
            rr.n_shapes = 0;
            rr.n_sig = 0;
            rr.n_acc = rms::kAccFixed;
            rr.t_ms = static_cast<double>(rec->steps[k]) * r.dt;
            rr.result = d_rec + static_cast<size_t>(k) * rec_stride;
            RMS_HIP(rms::launch_reduce(rr, stream));
            if (sb) {
                RMS_HIP(new_event(false, &ev_r[k]));
                RMS_HIP(hipEventRecord(ev_r[k], stream));
            }
        }
    }
    if (sb) {  // the second stream's last interval
        hipEvent_t ev_end = nullptr;
        RMS_HIP(new_event(false, &ev_end));
        RMS_HIP(hipEventRecord(ev_end, sb));
        RMS_HIP(hipStreamWaitEvent(stream, ev_end, 0));
    }
    RMS_HIP(hipEventRecord(ev1, stream));
    rms::ReducePlan rfin = dr.rp;
    rfin.wstate = wst[last_q];
    RMS_HIP(rms::launch_reduce(rfin, stream));

    std::vector<double> res(r.n_res), recv(static_cast<size_t>(n_rec) * rec_stride);
    RMS_HIP(hipMemcpyAsync(res.data(), dr.rp.result, r.n_res * sizeof(double),
                           hipMemcpyDeviceToHost, stream));
    RMS_HIP(hipMemcpyAsync(recv.data(), d_rec, recv.size() * sizeof(double),
                           hipMemcpyDeviceToHost, stream));
    if (out->walker_dump)
        RMS_HIP(hipMemcpyAsync(out->walker_dump, wst[last_q],
                               static_cast<size_t>(n_walkers) * r.width * sizeof(double),
                               hipMemcpyDeviceToHost, stream));
    RMS_HIP(hipStreamSynchronize(stream));
    float ms = 0.0f;
    RMS_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    rms::fill_result(r, res.data(), out);
    for (int k = 0; k < n_rec; ++k) {
        const double* v = recv.data() + static_cast<size_t>(k) * rec_stride;
        rec->sum_alpha[k] = v[0];
        for (int q = 0; q < 6; ++q) rec->m2[6 * k + q] = v[1 + q];
        for (int q = 0; q < 15; ++q) rec->m4[15 * k + q] = v[7 + q];
        for (int d = 0; d < n_dirs; ++d) {
            if (rec->D_dir) rec->D_dir[static_cast<size_t>(k) * n_dirs + d] = v[rms::kAccFixed + d];
            if (rec->K_dir)
                rec->K_dir[static_cast<size_t>(k) * n_dirs + d] = v[rms::kAccFixed + n_dirs + d];
        }
    }
    out->walk_kernel = RMS_WALK_PACKED;
    out->kernel_ms = ms;
    out->queue_s = 0.0;
    out->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return RMS_OK;
}

}  // extern "C"
