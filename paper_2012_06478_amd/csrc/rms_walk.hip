// Walk kernel, double-precision form, for gfx950.
//
// One lane carries one walker through all of its steps with the whole state
// in registers: integer voxel index, offset inside the voxel (voxel units),
// current label with its step length and 1/T2, unwrapped displacement, the
// phase vector of every gradient shape and R = sum t_c / T2_c.  The only
// memory traffic inside the step loop is the neighbour-label gather at each
// face the step reaches, the (wave-uniform, scalar) waveform sample and, at
// membranes only, the permeation threshold.
//
// Method (Lee, Fieremans & Novikov, arXiv 2012.06478):
//   - a step has fixed length ds = sqrt(6 D dt) and a uniform random direction
//     (section 2.2, items 2-3; section 2.1.3, Eq. step-size);
//   - with ds below the voxel size a step meets at most one face per axis, so
//     at most three (section 2.1.1 and the corner-reflector figure); a face
//     between equal labels is transparent, one between different labels is a
//     membrane: permeate with the probability of Eq. (perm-prob-general), else
//     reflect specularly (section 2.1.3, section 2.2 items 3-4);
//   - the phase accumulates g . x along the path and the T2 weight the time
//     spent per compartment (section 2.3, Eq. signal; section 2.1.4).
//
// Face walk.  Reflection flips one component of the direction and passing
// changes only the voxel index, so the path length at which the step reaches
// each axis' face is fixed at the start of the step: e_a = gap_a / |v_a|.  The
// kernel sorts the three e_a once and visits them in order while they lie
// inside the path budget; only a permeation into a label with another step
// length changes that budget (the remaining share of the step's duration is
// kept).  The end point on each axis then follows in closed form.  This
// replaces the per-event re-evaluation of all three distances.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the seed with
// counter (index, substream, walker_lo, walker_hi): substream 0 block j gives
// the directions of steps 2j+1 and 2j+2, substream 1 block i-1 the membrane
// words of step i, substream 2 blocks 0-1 the start.
#include "rms_internal.h"

namespace rms {
namespace {

__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// (w + 1/2) 2^-32, exact in double
__device__ __forceinline__ double unit_open(uint32_t w) {
    return fma(static_cast<double>(w), 0x1p-32, 0x1p-33);
}

template <typename T>
__device__ __forceinline__ T pick3(int a, T x, T y, T z) {
    return a == 0 ? x : (a == 1 ? y : z);
}

__device__ __forceinline__ int wrap_step(int c, int d, int n) {
    c += d;
    c = c < 0 ? c + n : c;
    return c >= n ? c - n : c;
}

template <typename LabelT, int NS>
struct WalkerF64 {
    int ix, iy, iz, l;
    double o[3];
    double sig, it2;
    double d[3];
    double R;
    double ph[NS > 0 ? NS : 1][3];
    uint32_t nface, nhit, nperm;

    // One step (index i0 = i - 1) with direction words wa, wb.
    __device__ __forceinline__ void step(const WalkPlan& p, const LabelT* __restrict__ lab,
                                         uint32_t i0, uint32_t wa, uint32_t wb, uint32_t wlo,
                                         uint32_t whi, uint32_t k0, uint32_t k1) {
        const double u1 = unit_open(wa);
        const double u2 = unit_open(wb);
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);
        const double rho = 2.0 * sqrt(u1 * (1.0 - u1));
        const double v[3] = {rho * cs, rho * sn, 1.0 - 2.0 * u1};

        // path length to the face each axis moves toward
        double e[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double av = fabs(v[a]);
            const double gap = fmax(v[a] > 0.0 ? 1.0 - o[a] : o[a], 0.0);
            e[a] = av > 0.0 ? gap / av : INFINITY;
        }
        // stable sort of (e, axis): ties keep x < y < z
        double s0 = e[0], s1 = e[1], s2 = e[2];
        int a0 = 0, a1 = 1, a2 = 2;
        if (s1 < s0) { const double t = s0; s0 = s1; s1 = t; const int q = a0; a0 = a1; a1 = q; }
        if (s2 < s1) { const double t = s1; s1 = s2; s2 = t; const int q = a1; a1 = a2; a2 = q; }
        if (s1 < s0) { const double t = s0; s0 = s1; s1 = t; const int q = a0; a0 = a1; a1 = q; }

        double P = 0.0, tau = 1.0, pend = sig;
        uint32_t passed = 0, refl = 0;
        int mw_used = 0;
        uint4 mw = make_uint4(0, 0, 0, 0);
        bool go = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double ek = k == 0 ? s0 : (k == 1 ? s1 : s2);
            const int a = k == 0 ? a0 : (k == 1 ? a1 : a2);
            go = go && (ek < pend);
            if (go) {
                ++nface;
                const int sgn = pick3(a, v[0], v[1], v[2]) > 0.0 ? 1 : -1;
                const int cx = a == 0 ? wrap_step(ix, sgn, p.nx) : ix;
                const int cy = a == 1 ? wrap_step(iy, sgn, p.ny) : iy;
                const int cz = a == 2 ? wrap_step(iz, sgn, p.nz) : iz;
                const int nl = lab[cx + p.nx * (cy + p.ny * cz)];
                bool cross = true;
                if (nl != l) {
                    ++nhit;
                    if (mw_used == 0) mw = philox4x32_10(i0, 1u, wlo, whi, k0, k1);
                    const uint32_t word = mw_used == 0 ? mw.x : (mw_used == 1 ? mw.y : mw.z);
                    ++mw_used;
                    cross = word < p.thr[l * p.n_labels + nl];
                    if (cross) {
                        ++nperm;
                        const double dtau = fmin((ek - P) / sig, tau);
                        R = fma(p.dt * dtau, it2, R);
                        tau -= dtau;
                        P = ek;
                        l = nl;
                        sig = p.sigma[nl];
                        it2 = p.inv_t2[nl];
                        pend = fma(tau, sig, P);
                    }
                }
                if (cross) {
                    passed |= 1u << a;
                    ix = cx;
                    iy = cy;
                    iz = cz;
                } else {
                    refl |= 1u << a;
                }
            }
        }
        const double lend = fma(tau, sig, P);
        R = fma(p.dt * tau, it2, R);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool pos = v[a] > 0.0;
            const double rest = (lend - e[a]) * v[a];  // signed travel after the face
            double on;
            if (refl & (1u << a)) on = (pos ? 1.0 : 0.0) - rest;
            else if (passed & (1u << a)) on = (pos ? 0.0 : 1.0) + rest;
            else on = fma(lend, v[a], o[a]);
            on = fmin(fmax(on, 0.0), 1.0);
            const double shift = (passed & (1u << a)) ? (pos ? 1.0 : -1.0) : 0.0;
            d[a] += (on - o[a]) + shift;
            o[a] = on;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double g = p.gdt[static_cast<int64_t>(s) * p.n_steps + i0];
            if (g != 0.0) {
                ph[s][0] = fma(g, d[0], ph[s][0]);
                ph[s][1] = fma(g, d[1], ph[s][1]);
                ph[s][2] = fma(g, d[2], ph[s][2]);
            }
        }
    }
};

template <typename LabelT, int NS>
__global__ __launch_bounds__(kBlock) void walk_fp64_kernel(WalkPlan p) {
    const int64_t w = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (w >= p.n_walkers) return;
    const LabelT* __restrict__ lab = static_cast<const LabelT*>(p.labels);
    const uint32_t wlo = static_cast<uint32_t>(w), whi = static_cast<uint32_t>(w >> 32);
    const uint32_t k0 = static_cast<uint32_t>(p.seed), k1 = static_cast<uint32_t>(p.seed >> 32);

    // start: uniform over allowed voxels, uniform inside the voxel (section 2.2, item 1)
    const uint4 b0 = philox4x32_10(0u, 2u, wlo, whi, k0, k1);
    const uint4 b1 = philox4x32_10(1u, 2u, wlo, whi, k0, k1);
    const uint64_t r64 = (static_cast<uint64_t>(b0.y) << 32) | b0.x;
    const uint32_t rank = static_cast<uint32_t>(__umul64hi(r64, static_cast<uint64_t>(p.n_allowed)));
    const uint32_t lin = p.allowed ? p.allowed[rank] : rank;
    const uint32_t nxy = static_cast<uint32_t>(p.nx) * static_cast<uint32_t>(p.ny);

    WalkerF64<LabelT, NS> W;
    W.iz = static_cast<int>(lin / nxy);
    const uint32_t rem = lin - static_cast<uint32_t>(W.iz) * nxy;
    W.iy = static_cast<int>(rem / static_cast<uint32_t>(p.nx));
    W.ix = static_cast<int>(rem - static_cast<uint32_t>(W.iy) * static_cast<uint32_t>(p.nx));
    W.o[0] = unit_open(b0.z);
    W.o[1] = unit_open(b0.w);
    W.o[2] = unit_open(b1.x);
    W.l = lab[lin];
    const int l0 = W.l;
    W.sig = p.sigma[W.l];
    W.it2 = p.inv_t2[W.l];
    W.d[0] = W.d[1] = W.d[2] = 0.0;
    W.R = 0.0;
#pragma unroll
    for (int s = 0; s < (NS > 0 ? NS : 1); ++s) W.ph[s][0] = W.ph[s][1] = W.ph[s][2] = 0.0;
    W.nface = W.nhit = W.nperm = 0;

    const uint32_t n = static_cast<uint32_t>(p.n_steps);
    for (uint32_t j = 0; 2 * j < n; ++j) {
        const uint4 wd = philox4x32_10(j, 0u, wlo, whi, k0, k1);
        W.step(p, lab, 2 * j, wd.x, wd.y, wlo, whi, k0, k1);
        if (2 * j + 1 < n) W.step(p, lab, 2 * j + 1, wd.z, wd.w, wlo, whi, k0, k1);
    }

    double* out = p.wstate + w * (kDumpFixed + 3 * NS);
    out[0] = W.d[0] * p.voxel_um;
    out[1] = W.d[1] * p.voxel_um;
    out[2] = W.d[2] * p.voxel_um;
    out[3] = W.R;
    out[4] = W.l;
    out[5] = W.ix;
    out[6] = W.iy;
    out[7] = W.iz;
    out[8] = W.o[0];
    out[9] = W.o[1];
    out[10] = W.o[2];
    out[11] = l0;
    out[12] = W.nface;
    out[13] = W.nhit;
    out[14] = W.nperm;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        out[15 + 3 * s] = W.ph[s][0] * p.voxel_um;
        out[16 + 3 * s] = W.ph[s][1] * p.voxel_um;
        out[17 + 3 * s] = W.ph[s][2] * p.voxel_um;
    }
}

template <typename LabelT>
hipError_t dispatch_ns(const WalkPlan& p, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((p.n_walkers + kBlock - 1) / kBlock));
    switch (p.n_shapes) {
        case 0: walk_fp64_kernel<LabelT, 0><<<grid, kBlock, 0, s>>>(p); break;
        case 1: walk_fp64_kernel<LabelT, 1><<<grid, kBlock, 0, s>>>(p); break;
        case 2: walk_fp64_kernel<LabelT, 2><<<grid, kBlock, 0, s>>>(p); break;
        case 3: walk_fp64_kernel<LabelT, 3><<<grid, kBlock, 0, s>>>(p); break;
        case 4: walk_fp64_kernel<LabelT, 4><<<grid, kBlock, 0, s>>>(p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_walk_fp64(const WalkPlan& p, hipStream_t s) {
    if (p.n_walkers <= 0) return hipSuccess;
    return p.label_bytes == 1 ? dispatch_ns<uint8_t>(p, s) : dispatch_ns<uint16_t>(p, s);
}

}  // namespace rms
