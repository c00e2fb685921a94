// Signal and moment reductions for gfx950 (section 2.3 of arXiv 2012.06478:
// S = <alpha exp(-i phi)> / <alpha>, alpha-weighted displacement moments,
// D and K per gradient direction).
//
// Three kernels, all in double precision and in a fixed order, so a result
// depends only on the walker count and never on scheduling:
//   contrib   one lane per walker computes its accumulated values (alpha,
//             alpha dx_i dx_j, alpha dx_i dx_j dx_k dx_l, the event counters and
//             alpha (cos phi, -sin phi) for every signal); each wave sums them
//             with cross-lane shuffles, the block adds its four waves in order
//             and writes one partial per value;
//   final     one block per value adds the block partials (fixed strided
//             split, fixed tree);
//   finalize  divides by sum(alpha) and contracts M2, M4 with each direction.
#include "rms_internal.h"

namespace rms {
namespace {

constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(kBlock) void contrib_kernel(ReducePlan p) {
    extern __shared__ double lds[];  // [n_acc][kWaves]
    const int64_t w = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const bool valid = w < p.n_walkers;
    const double* st = p.wstate + (valid ? w : 0) * p.width;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double alpha = valid ? exp(-st[3]) : 0.0;
    const double X[3] = {valid ? st[0] : 0.0, valid ? st[1] : 0.0, valid ? st[2] : 0.0};

    auto put = [&](int k, double v) {
        v = wave_sum(v);
        if (lane == 0) lds[k * kWaves + wave] = v;
    };
    put(0, alpha);
    int k = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) put(k++, alpha * X[a] * X[b]);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b)
#pragma unroll
            for (int c = b; c < 3; ++c)
#pragma unroll
                for (int d = c; d < 3; ++d) put(k++, alpha * X[a] * X[b] * X[c] * X[d]);
    put(22, valid ? st[12] : 0.0);
    put(23, valid ? st[13] : 0.0);
    put(24, valid ? st[14] : 0.0);

    const int per_shape = p.n_shapes > 0 ? p.n_sig / p.n_shapes : 0;
    for (int s = 0; s < p.n_shapes; ++s) {
        const double f0 = valid ? st[kDumpFixed + 3 * s] : 0.0;
        const double f1 = valid ? st[kDumpFixed + 3 * s + 1] : 0.0;
        const double f2 = valid ? st[kDumpFixed + 3 * s + 2] : 0.0;
        for (int q = s * per_shape; q < (s + 1) * per_shape; ++q) {
            const double phi = fma(p.kg[3 * q], f0, fma(p.kg[3 * q + 1], f1, p.kg[3 * q + 2] * f2));
            double sn, cs;
            sincos(phi, &sn, &cs);
            put(kAccFixed + 2 * q, alpha * cs);
            put(kAccFixed + 2 * q + 1, -alpha * sn);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < p.n_acc; j += kBlock) {
        double acc = lds[j * kWaves];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) acc += lds[j * kWaves + q];
        p.partial[static_cast<int64_t>(j) * p.n_blocks + blockIdx.x] = acc;
    }
}

__global__ __launch_bounds__(kBlock) void final_kernel(ReducePlan p) {
    __shared__ double s[kBlock];
    const int k = blockIdx.x;
    const double* row = p.partial + static_cast<int64_t>(k) * p.n_blocks;
    double acc = 0.0;
    for (int b = threadIdx.x; b < p.n_blocks; b += kBlock) acc += row[b];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) p.sums[k] = s[0];
}

// multiplicity of the M4 entry with index tuple (a <= b <= c <= d)
__device__ __forceinline__ double m4_mult(int a, int b, int c, int d) {
    int n[3] = {0, 0, 0};
    n[a]++;
    n[b]++;
    n[c]++;
    n[d]++;
    const int f[5] = {1, 1, 2, 6, 24};
    return 24.0 / (f[n[0]] * f[n[1]] * f[n[2]]);
}

__global__ __launch_bounds__(kBlock) void finalize_kernel(ReducePlan p) {
    const double sa = p.sums[0];
    const int t = threadIdx.x;
    if (t == 0) p.result[0] = sa;
    if (t >= 1 && t < 22) p.result[t] = p.sums[t] / sa;
    if (t >= 22 && t < 25) p.result[t] = p.sums[t];
    for (int j = kAccFixed + t; j < kAccFixed + 2 * p.n_sig; j += kBlock)
        p.result[j] = p.sums[j] / sa;
    const int base = kAccFixed + 2 * p.n_sig;
    for (int dd = t; dd < p.n_dirs; dd += kBlock) {
        const double g[3] = {p.dirs[3 * dd], p.dirs[3 * dd + 1], p.dirs[3 * dd + 2]};
        double w2 = 0.0, w4 = 0.0;
        int k = 1;
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b) w2 += (a == b ? 1.0 : 2.0) * (p.sums[k++] / sa) * g[a] * g[b];
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b)
                for (int c = b; c < 3; ++c)
                    for (int d = c; d < 3; ++d)
                        w4 += m4_mult(a, b, c, d) * (p.sums[k++] / sa) * g[a] * g[b] * g[c] * g[d];
        p.result[base + dd] = p.t_ms > 0.0 ? w2 / (2.0 * p.t_ms) : 0.0;
        p.result[base + p.n_dirs + dd] = w2 > 0.0 ? w4 / (w2 * w2) - 3.0 : 0.0;
    }
}

}  // namespace

hipError_t launch_reduce(const ReducePlan& p, hipStream_t s) {
    const size_t lds = static_cast<size_t>(p.n_acc) * kWaves * sizeof(double);
    contrib_kernel<<<p.n_blocks, kBlock, lds, s>>>(p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    final_kernel<<<p.n_acc, kBlock, 0, s>>>(p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    finalize_kernel<<<1, kBlock, 0, s>>>(p);
    return hipGetLastError();
}

}  // namespace rms
