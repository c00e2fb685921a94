// Signal and moment reductions for gfx950 (section 2.3 of arXiv 2012.06478:
// S = <alpha exp(-i phi)> / <alpha>, alpha-weighted displacement moments,
// D and K per gradient direction).
//
// Three kernels, all in double precision and in a fixed order, so a result
// depends only on the walker count and never on scheduling:
//   contrib   each lane computes the accumulated values of up to four walkers (alpha,
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

// Each thread folds up to kFold walkers (block b covers walkers b W .. b W +
// W - 1, W = fold x kBlock, fold = ceil(n_walkers / (n_blocks kBlock)) <=
// kFold; walker j kBlock + t of the block goes to thread t), adding their
// values in a fixed order before the wave sums, so the cross-lane work is
// shared by several walkers.
constexpr int kFold = 4;

__global__ __launch_bounds__(kBlock) void contrib_kernel(ReducePlan p) {
    extern __shared__ double lds[];  // [n_acc][kWaves]
    const int64_t span = static_cast<int64_t>(p.n_blocks) * kBlock;
    const int fold = static_cast<int>((p.n_walkers + span - 1) / span);  // <= kFold (host)
    const int64_t w0 = static_cast<int64_t>(blockIdx.x) * fold * kBlock + threadIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    bool valid[kFold];
    const double* st[kFold];
    double alpha[kFold], X[kFold][3];
#pragma unroll
    for (int j = 0; j < kFold; ++j) {
        const int64_t w = w0 + static_cast<int64_t>(j) * kBlock;
        valid[j] = j < fold && w < p.n_walkers;
        st[j] = p.wstate + (valid[j] ? w : 0) * p.width;
        alpha[j] = valid[j] ? exp(-st[j][3]) : 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) X[j][a] = valid[j] ? st[j][a] : 0.0;
    }

    auto put = [&](int k, double v) {
        v = wave_sum(v);
        if (lane == 0) lds[k * kWaves + wave] = v;
    };
    {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < kFold; ++j) v += alpha[j];
        put(0, v);
    }
    int k = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) {
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < kFold; ++j) v += alpha[j] * X[j][a] * X[j][b];
            put(k++, v);
        }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b)
#pragma unroll
            for (int c = b; c < 3; ++c)
#pragma unroll
                for (int d = c; d < 3; ++d) {
                    double v = 0.0;
#pragma unroll
                    for (int j = 0; j < kFold; ++j)
                        v += alpha[j] * X[j][a] * X[j][b] * X[j][c] * X[j][d];
                    put(k++, v);
                }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < kFold; ++j) v += valid[j] ? st[j][12 + c] : 0.0;
        put(22 + c, v);
    }

    const int per_shape = p.n_shapes > 0 ? p.n_sig / p.n_shapes : 0;
    for (int s = 0; s < p.n_shapes; ++s) {
        double f[kFold][3];
#pragma unroll
        for (int j = 0; j < kFold; ++j)
#pragma unroll
            for (int a = 0; a < 3; ++a) f[j][a] = valid[j] ? st[j][kDumpFixed + 3 * s + a] : 0.0;
        for (int q = s * per_shape; q < (s + 1) * per_shape; ++q) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int j = 0; j < kFold; ++j) {
                const double phi =
                    fma(p.kg[3 * q], f[j][0], fma(p.kg[3 * q + 1], f[j][1], p.kg[3 * q + 2] * f[j][2]));
                double sn, cs;
                sincos(phi, &sn, &cs);
                re += alpha[j] * cs;
                im -= alpha[j] * sn;
            }
            put(kAccFixed + 2 * q, re);
            put(kAccFixed + 2 * q + 1, im);
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
