// Walk kernels for gfx950 (the walkers themselves are in rms_device.h).
//
// walk_kernel         one run: lane = walker, all steps in registers, then the
//                     per-walker record.  The only memory traffic inside the
//                     step loop is the neighbour-label gather at each face a
//                     step reaches, the wave-uniform waveform sample (scalar
//                     load) and, at membranes only, the permeation threshold.
// walk_packed_kernel  several runs in one launch (the server): block = (run,
//                     256 walkers, range of steps) from a work list; the walker
//                     resumes from its stored state and stores it again, so a
//                     run can be advanced in slices between which other runs
//                     join.  The arithmetic of a step is the same code as in
//                     walk_kernel, so a walker's result does not depend on how
//                     its steps were sliced.
#include "rms.h"
#include "rms_device.h"

namespace rms {
namespace {

using dev::Ids;

// Five waves per SIMD: the double-precision walker then fits 96 registers
// (a few bytes of spill outside the step) and runs about 7% faster than at
// four; the mixed walker needs fewer registers and is not affected.
#define RMS_WALK_OCCUPANCY __attribute__((amdgpu_waves_per_eu(5, 8)))

template <class Walker, typename LabelT>
__global__ __launch_bounds__(kBlock) RMS_WALK_OCCUPANCY void walk_kernel(WalkPlan p) {
    const int64_t w = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (w >= p.n_walkers) return;
    const LabelT* __restrict__ lab = static_cast<const LabelT*>(p.labels);
    const Ids id{static_cast<uint32_t>(w), static_cast<uint32_t>(w >> 32),
                 static_cast<uint32_t>(p.seed), static_cast<uint32_t>(p.seed >> 32)};
    Walker W;
    W.init(p, lab, id);
    dev::walk_range(p, lab, W, 0u, static_cast<uint32_t>(p.n_steps), id);
    W.finish(p, p.wstate + w * (kDumpFixed + 3 * p.n_shapes));
}

template <class Walker, typename LabelT>
__global__ __launch_bounds__(kBlock) RMS_WALK_OCCUPANCY void walk_packed_kernel(const PackedItem* __restrict__ items,
                                                             const WalkPlan* __restrict__ plans) {
    const PackedItem it = items[blockIdx.x];
    const WalkPlan p = plans[it.plan];
    const int64_t w = it.first_walker + threadIdx.x;
    if (w >= p.n_walkers) return;
    const LabelT* __restrict__ lab = static_cast<const LabelT*>(p.labels);
    const Ids id{static_cast<uint32_t>(w), static_cast<uint32_t>(w >> 32),
                 static_cast<uint32_t>(p.seed), static_cast<uint32_t>(p.seed >> 32)};
    Walker* st = static_cast<Walker*>(p.state) + w;
    Walker W;
    if (it.step_begin == 0) W.init(p, lab, id);
    else W = *st;
    dev::walk_range(p, lab, W, it.step_begin, it.step_end, id);
    if (it.step_end == static_cast<uint32_t>(p.n_steps))
        W.finish(p, p.wstate + w * (kDumpFixed + 3 * p.n_shapes));
    else
        *st = W;
}

template <template <typename, int> class Walker, typename LabelT>
hipError_t run_ns(const WalkPlan& p, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((p.n_walkers + kBlock - 1) / kBlock));
    switch (p.n_shapes) {
        case 0: walk_kernel<Walker<LabelT, 0>, LabelT><<<grid, kBlock, 0, s>>>(p); break;
        case 1: walk_kernel<Walker<LabelT, 1>, LabelT><<<grid, kBlock, 0, s>>>(p); break;
        case 2: walk_kernel<Walker<LabelT, 2>, LabelT><<<grid, kBlock, 0, s>>>(p); break;
        case 3: walk_kernel<Walker<LabelT, 3>, LabelT><<<grid, kBlock, 0, s>>>(p); break;
        case 4: walk_kernel<Walker<LabelT, 4>, LabelT><<<grid, kBlock, 0, s>>>(p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <template <typename, int> class Walker, typename LabelT>
hipError_t packed_ns(const PackedItem* items, int n_items, const WalkPlan* plans, int ns,
                     hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(n_items));
    switch (ns) {
        case 0: walk_packed_kernel<Walker<LabelT, 0>, LabelT><<<grid, kBlock, 0, s>>>(items, plans); break;
        case 1: walk_packed_kernel<Walker<LabelT, 1>, LabelT><<<grid, kBlock, 0, s>>>(items, plans); break;
        case 2: walk_packed_kernel<Walker<LabelT, 2>, LabelT><<<grid, kBlock, 0, s>>>(items, plans); break;
        case 3: walk_packed_kernel<Walker<LabelT, 3>, LabelT><<<grid, kBlock, 0, s>>>(items, plans); break;
        case 4: walk_packed_kernel<Walker<LabelT, 4>, LabelT><<<grid, kBlock, 0, s>>>(items, plans); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <template <typename, int> class Walker>
size_t state_bytes_ns(int ns) {
    switch (ns) {
        case 0: return sizeof(Walker<uint16_t, 0>);
        case 1: return sizeof(Walker<uint16_t, 1>);
        case 2: return sizeof(Walker<uint16_t, 2>);
        case 3: return sizeof(Walker<uint16_t, 3>);
        case 4: return sizeof(Walker<uint16_t, 4>);
        default: return 0;
    }
}

}  // namespace

hipError_t launch_walk(const WalkPlan& p, int precision, hipStream_t s) {
    if (p.n_walkers <= 0) return hipSuccess;
    const bool u8 = p.label_bytes == 1;
    if (precision == RMS_FP64)
        return u8 ? run_ns<dev::WalkerF64, uint8_t>(p, s) : run_ns<dev::WalkerF64, uint16_t>(p, s);
    return u8 ? run_ns<dev::WalkerMixed, uint8_t>(p, s) : run_ns<dev::WalkerMixed, uint16_t>(p, s);
}

hipError_t launch_walk_packed(const PackedItem* items, int n_items, const WalkPlan* plans,
                              int precision, int label_bytes, int n_shapes, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    const bool u8 = label_bytes == 1;
    if (precision == RMS_FP64)
        return u8 ? packed_ns<dev::WalkerF64, uint8_t>(items, n_items, plans, n_shapes, s)
                  : packed_ns<dev::WalkerF64, uint16_t>(items, n_items, plans, n_shapes, s);
    return u8 ? packed_ns<dev::WalkerMixed, uint8_t>(items, n_items, plans, n_shapes, s)
              : packed_ns<dev::WalkerMixed, uint16_t>(items, n_items, plans, n_shapes, s);
}

size_t walker_state_bytes(int precision, int /*label_bytes*/, int n_shapes) {
    return precision == RMS_FP64 ? state_bytes_ns<dev::WalkerF64>(n_shapes)
                                 : state_bytes_ns<dev::WalkerMixed>(n_shapes);
}

}  // namespace rms
