// Walk kernels for gfx950 (the walkers themselves are in rms_device.h).
//
// walk_kernel         one run: lane = walker, all steps in registers, then the
//                     per-walker record.  The only memory traffic inside the
//                     step loop is the neighbour-label gather at each face a
//                     step reaches, the wave-uniform waveform sample and, at
//                     membranes only, the permeation threshold (the angle
//                     table and the series coefficients of the direction
//                     draw come from LDS).
// walk_packed_kernel  several runs in one launch (the server): block = (run,
//                     256 walkers, range of steps) from a work list; the walker
//                     resumes from its stored state and stores it again, so a
//                     run can be advanced in slices between which other runs
//                     join.  The arithmetic of a step is the same code as in
//                     walk_kernel, so a walker's result does not depend on how
//                     its steps were sliced.
#include <atomic>

#include "rms.h"
#include "rms_device.h"

namespace rms {
namespace {

using dev::Ids;

// Waves per SIMD each walker asks for: five for the double-precision walker,
// which then fits 96 registers (without spilling up to two waveform shapes)
// and runs about 7% faster than at four; six for the mixed walker, which keeps
// it within 80 registers (left free, it grows past 85 with two waveform
// shapes and drops to five waves, 16% slower).  The absorbing-membrane forms
// carry four more words per step and ask for one wave fewer: squeezed to the
// plain forms' counts they reload a spilled value every step (FP64 77.2
// against 71.5 ms, mixed 62.4 against 59.0 ms on the 200^3 packing).
#define RMS_WALK_OCCUPANCY __attribute__((amdgpu_waves_per_eu(Walker::kWaves, 8)))

// The angle table of the double-precision direction draw, copied to LDS by
// the whole block before any thread leaves (one 16-byte entry per thread, so
// a step reads its entry with one LDS load; thread 0 also copies the
// coefficient entry behind the angles).
static_assert(kBlock == kTrigSize, "one table entry per thread");
template <class Walker>
__device__ __forceinline__ void load_trig(const WalkPlan& p, double2* trig) {
    if constexpr (Walker::kTrig) {
        trig[threadIdx.x] = p.trig[threadIdx.x];
        if (threadIdx.x == 0) trig[kTrigSize] = p.trig[kTrigSize];
        __syncthreads();
    }
}

template <class Walker, typename LabelT>
__global__ __launch_bounds__(kBlock) RMS_WALK_OCCUPANCY void walk_kernel(WalkPlan p) {
    __shared__ double2 trig[Walker::kTrig ? kTrigSize + 1 : 1];
    load_trig<Walker>(p, trig);
    const int64_t slot = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    int64_t w = slot;
    if (p.order) {
        if (slot >= p.n_slots) return;
        const uint32_t o = p.order[slot];
        if (o == kNoWalker) return;
        w = o;
    } else if (w >= p.n_walkers) {
        return;
    }
    const LabelT* __restrict__ lab = static_cast<const LabelT*>(p.labels);
    const Ids id = dev::walker_ids<Walker>(w, p.seed);
    Walker W;
    W.init(p, lab, id);
    dev::walk_range(p, lab, W, 0u, static_cast<uint32_t>(p.n_steps), id, trig);
    W.finish(p, p.wstate + w * (kDumpFixed + 3 * p.n_shapes));
}

template <class Walker, typename LabelT>
__global__ __launch_bounds__(kBlock) RMS_WALK_OCCUPANCY void walk_packed_kernel(const PackedItem* __restrict__ items,
                                                             const WalkPlan* __restrict__ plans) {
    const PackedItem it = items[blockIdx.x];
    const WalkPlan p = plans[it.plan];
    __shared__ double2 trig[Walker::kTrig ? kTrigSize + 1 : 1];
    load_trig<Walker>(p, trig);
    const int64_t slot = it.first_slot + threadIdx.x;
    int64_t w = slot;
    if (p.order) {
        if (slot >= p.n_slots) return;
        const uint32_t o = p.order[slot];
        if (o == kNoWalker) return;
        w = o;
    } else if (w >= p.n_walkers) {
        return;
    }
    const LabelT* __restrict__ lab = static_cast<const LabelT*>(p.labels);
    const Ids id = dev::walker_ids<Walker>(w, p.seed);
    Walker* st = static_cast<Walker*>(p.state) + w;
    Walker W;
    if (it.step_begin == 0) W.init(p, lab, id);
    else W = *st;
    dev::walk_range<true>(p, lab, W, it.step_begin, it.step_end, id, trig);
    double* rec = p.wstate + w * (kDumpFixed + 3 * p.n_shapes);
    if (it.step_end == static_cast<uint32_t>(p.n_steps)) {
        W.finish(p, rec);
    } else {
        *st = W;
        if (it.flags & kItemRecord) W.finish(p, rec);
    }
}

// Accepted start attempt per walker (spin concentrations): the rejection loop
// runs here, once, so the walk kernels only read the attempt index.
__global__ __launch_bounds__(kBlock) void start_try_kernel(WalkPlan p) {
    const int64_t w = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (w >= p.n_walkers) return;
    const Ids id{static_cast<uint32_t>(w), 0u, static_cast<uint32_t>(p.seed),
                 static_cast<uint32_t>(p.seed >> 32)};
    p.start_try[w] = dev::start_try_of(p, id);
}

// Step range and flags of every item of a packed launch (a run recorded at
// several steps walks one interval per launch over the same items).
__global__ __launch_bounds__(kBlock) void item_range_kernel(PackedItem* items, int n,
                                                            uint32_t b, uint32_t e,
                                                            uint32_t flags) {
    const int i = static_cast<int>(blockIdx.x) * kBlock + static_cast<int>(threadIdx.x);
    if (i < n) {
        items[i].step_begin = b;
        items[i].step_end = e;
        items[i].flags = flags;
    }
}

// ---------------------------------------------------------------------------
// Walker order.  The walk gathers labels at random places of the volume; a
// 16 MB volume misses the 4 MB L2 of each XCD.  Blocks are dealt to the eight
// XCDs round-robin (block b on XCD b mod 8), so the walkers are sorted by the
// Morton code of their start cell (2^cb cells per axis, cb from 1 to 6 so
// that a cell holds about four walkers), the sorted list is cut
// into eight equal runs, and run c fills blocks c, c + 8, c + 16, ...: each
// XCD then walks one compact part of the volume and the lanes of a wave start
// close together.  A walker's result depends only on its index, so the order
// changes no result.  Counting sort: cell histogram, two-level scan, scatter
// with atomic slot counters (the order of walkers inside one cell is
// arbitrary).

constexpr int kXcds = 8;
constexpr int kMaxCellBits = 6;

int cell_bits(int64_t n) {  // about four walkers per cell
    int cb = 1;
    while (cb < kMaxCellBits && (int64_t(4) << (3 * cb)) < n) ++cb;
    return cb;
}

int64_t order_chunk(int64_t n) {  // walkers per XCD run, whole blocks
    const int64_t per = (n + kXcds - 1) / kXcds;
    return (per + kBlock - 1) / kBlock * kBlock;
}

bool order_used(int64_t n) { return n >= 1 && n < static_cast<int64_t>(kNoWalker); }

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // bit i -> bit 3i
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < kMaxCellBits; ++i) r |= ((v >> i) & 1u) << (3 * i);
    return r;
}

__global__ __launch_bounds__(kBlock) void order_init_kernel(uint32_t* order, int64_t n_slots,
                                                            uint32_t* count, uint32_t n_cells) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n_slots) order[i] = kNoWalker;
    if (i < n_cells) count[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void order_keys_kernel(WalkPlan p, uint32_t* count,
                                                            uint32_t* keys, int cb) {
    const int64_t w = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (w >= p.n_walkers) return;
    const Ids id{static_cast<uint32_t>(w), 0u, static_cast<uint32_t>(p.seed),
                 static_cast<uint32_t>(p.seed >> 32)};
    const dev::Start st = dev::draw_start(p, id);
    const dev::Coords k = dev::coords_of(static_cast<uint32_t>(st.lin), static_cast<uint32_t>(p.nx),
                                         static_cast<uint32_t>(p.nx) * static_cast<uint32_t>(p.ny),
                                         p.div_nx_m, p.div_nx_sh, p.div_nxy_m, p.div_nxy_sh);
    const int n[3] = {p.nx, p.ny, p.nz};
    uint32_t key = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint32_t c = static_cast<uint32_t>((static_cast<uint64_t>(k.c[a]) << cb) / n[a]);
        key |= spread3(c) << a;
    }
    keys[w] = key;
    atomicAdd(&count[key], 1u);
}

// Exclusive prefix sum of the n_cells cell counts in two levels: each block
// of kScanChunk threads scans one chunk of counts in LDS (in place, within
// the chunk) and writes the chunk's total; one block then scans the totals,
// which the scatter adds to the position inside the chunk.
constexpr uint32_t kScanChunk = 1024;
constexpr uint32_t kMaxChunks = (1u << (3 * kMaxCellBits)) / kScanChunk;

template <uint32_t N>
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t* part, uint32_t v) {
    part[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t off = 1; off < N; off <<= 1) {  // Hillis-Steele
        const uint32_t u = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += u;
        __syncthreads();
    }
    return part[threadIdx.x];
}

__global__ __launch_bounds__(kScanChunk) void order_scan_chunks_kernel(uint32_t* count,
                                                                       uint32_t n_cells,
                                                                       uint32_t* totals) {
    __shared__ uint32_t part[kScanChunk];
    const uint32_t i = blockIdx.x * kScanChunk + threadIdx.x;
    const uint32_t v = i < n_cells ? count[i] : 0u;
    const uint32_t inc = block_inclusive_scan<kScanChunk>(part, v);
    if (i < n_cells) count[i] = inc - v;
    if (threadIdx.x == kScanChunk - 1) totals[blockIdx.x] = inc;
}

__global__ __launch_bounds__(kMaxChunks) void order_scan_totals_kernel(uint32_t* totals,
                                                                       uint32_t n_chunks) {
    __shared__ uint32_t part[kMaxChunks];
    const uint32_t v = threadIdx.x < n_chunks ? totals[threadIdx.x] : 0u;
    const uint32_t inc = block_inclusive_scan<kMaxChunks>(part, v);
    if (threadIdx.x < n_chunks) totals[threadIdx.x] = inc - v;
}

__global__ __launch_bounds__(kBlock) void order_scatter_kernel(const uint32_t* keys, uint32_t* next,
                                                               const uint32_t* totals,
                                                               uint32_t* order, int64_t n,
                                                               int64_t chunk) {
    const int64_t w = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (w >= n) return;
    const uint32_t key = keys[w];
    const int64_t pos = static_cast<int64_t>(atomicAdd(&next[key], 1u)) +
                        totals[key / kScanChunk];  // place in the sorted list
    const int64_t c = pos / chunk, j = pos - c * chunk;
    order[((j / kBlock) * kXcds + c) * kBlock + j % kBlock] = static_cast<uint32_t>(w);
}

// ---------------------------------------------------------------------------
// Persistent segmented walk (ordered runs).  A launch whose waves all walk
// every step ends with a partly filled last round of resident waves and a
// ramp-down while they finish; at 1e6 walkers that is 5-8% of the launch.
// Here the grid holds only as many blocks as can be resident, and each wave
// takes work items (64 slots, segment of about n_steps/16 steps, 2048 to 4096) from the
// queue of its XCD (block b serves queue b mod 8, the XCD the walker order
// gave those slots) in segment-major order, so all walkers advance together
// and the last partial round is one short segment.  A walker state lives in
// registers during a segment and in `seg_state` between segments.  Before
// segment s of a slot wave a wave waits until segment s - 1 of it is done;
// that item was handed out about one segment-round earlier, so the wait
// almost never polls.  Only a running wave can hold an item, so every chain
// of waits ends at a wave that is walking: no deadlock, whatever the number
// of resident waves.  The wait is bounded all the same: past the poll limit
// polls the wave raises the failure flag, every wave then stops taking items,
// and the host reports the run as failed.  The loop has no block barrier:
// items, waits and completion counters are per wave, and the lane that
// fetches broadcasts the item with readfirstlane.

constexpr uint32_t kSegPollLimit = 1u << 20;  // default: polls of 1-2 us, about a second

// Launch options (rms_set_option): which walk kernel runs and the poll limit
// of the persistent walk's waits.  Process-wide; read at each launch.
std::atomic<int> g_walk_choice{RMS_WALK_AUTO};
std::atomic<uint32_t> g_seg_poll_limit{kSegPollLimit};
// At least 2048 steps a segment: fewer segment boundaries (each moves the
// walker states through HBM) against a shorter last segment; at 1e6 walkers x
// 1e4 steps five segments beat ten by 1.6% (FP64 63.0 against 64.1 ms, mixed
// 52.7 against 53.4 ms) and two lose 3%.
constexpr int64_t kSegMinSteps = 2048;
// At most 4096 steps a segment (about 10 ms at full occupancy), so that a
// wave never waits anywhere near the poll limit, however long the walk.
constexpr int64_t kSegMaxSteps = 4096;
constexpr int64_t kSegTarget = 16;            // segments per walk, at most, up to kSegMaxSteps
constexpr uint32_t kWave = 64;
constexpr uint32_t kWavesPerBlock = kBlock / kWave;

static_assert(kSegQueues == kXcds, "one queue per XCD");

uint32_t seg_steps_of(int64_t n_steps) {
    int64_t s = (n_steps + kSegTarget - 1) / kSegTarget;
    s = (s + 3) / 4 * 4;  // segments start on a block of both Philox streams
    s = s > kSegMaxSteps ? kSegMaxSteps : s;
    return static_cast<uint32_t>(s < kSegMinSteps ? kSegMinSteps : s);
}

__global__ __launch_bounds__(kBlock) void seg_init_kernel(uint32_t* ctl, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) ctl[i] = 0u;
}

template <class Walker, typename LabelT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Walker::kWaves, 8))) void walk_seg_kernel(
    WalkPlan p, uint32_t n_seg, uint32_t seg_steps, uint32_t waves_per_queue,
    uint32_t poll_limit) {
    __shared__ double2 trig[Walker::kTrig ? kTrigSize + 1 : 1];
    load_trig<Walker>(p, trig);  // the only block barrier, before the loop
    const LabelT* __restrict__ lab = static_cast<const LabelT*>(p.labels);
    Walker* st = static_cast<Walker*>(p.seg_state);
    uint32_t* head = p.seg_ctl;
    uint32_t* fail_flag = p.seg_ctl + kSegErrorWord;
    uint32_t* done = p.seg_ctl + kSegCtlFixed;  // per slot wave
    const uint32_t queue = blockIdx.x % kSegQueues;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t n_items = waves_per_queue * n_seg;
    const uint32_t n_steps = static_cast<uint32_t>(p.n_steps);
    for (;;) {
        uint32_t got = 0;
        if (lane == 0) got = atomicAdd(&head[queue], 1u);
        uint32_t it = __builtin_amdgcn_readfirstlane(got);  // the wave's item
        if (it < n_items &&
            __hip_atomic_load(fail_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            it = n_items;
        if (it >= n_items) break;
        const uint32_t seg = it / waves_per_queue;
        const uint32_t k = it % waves_per_queue;  // k-th slot wave of this queue
        const uint32_t sw = ((k / kWavesPerBlock) * kSegQueues + queue) * kWavesPerBlock +
                            k % kWavesPerBlock;
        if (seg > 0) {
            uint32_t polls = 0;
            while (__hip_atomic_load(&done[sw], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < seg) {
                if (++polls > poll_limit) break;
                __builtin_amdgcn_s_sleep(8);
            }
            if (polls > poll_limit) {
                if (lane == 0) atomicOr(fail_flag, 1u);
                break;
            }
        }
        const uint32_t b = seg * seg_steps;
        const uint32_t e = n_steps - b < seg_steps ? n_steps : b + seg_steps;
        const int64_t slot = static_cast<int64_t>(sw) * kWave + lane;
        const uint32_t w = p.order[slot];
        if (w != kNoWalker) {
            const Ids id = dev::walker_ids<Walker>(w, p.seed);
            Walker W;
            if (seg == 0) W.init(p, lab, id);
            else W = st[slot];
            dev::walk_range(p, lab, W, b, e, id, trig);
            if (e == n_steps)
                W.finish(p, p.wstate + static_cast<int64_t>(w) * (kDumpFixed + 3 * p.n_shapes));
            else
                st[slot] = W;
        }
        if (lane == 0)  // after this wave's stores (release at agent scope)
            __hip_atomic_store(&done[sw], seg + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Resident blocks of the persistent walk: occupancy times compute units,
// whole multiples of the queue count.
template <class Walker, typename LabelT>
int seg_grid() {
    static const int g = [] {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, walk_seg_kernel<Walker, LabelT>,
                                                         kBlock, 0) != hipSuccess)
            return kSegQueues;
        const int n = per_cu * cus;
        return n - n % kSegQueues > kSegQueues ? n - n % kSegQueues : kSegQueues;
    }();
    return g;
}

// The persistent walk pays only where a one-launch walk loses much of its
// time to the partly filled last round of waves: between 1.5 and 4.5 rounds
// of resident waves (measured at 200^3, kernel ms one launch / persistent:
// FP64 0.7e6 walkers 48.1 / 45.7, 1e6 66.6 / 64.7, 2e6 120.3 / 123.7, 1e7
// 555.7 / 595.6; mixed 0.7e6 40.8 / 38.3, 1e6 56.6 / 53.7, 3e6 144.7 /
// 151.0).  Just above one round every item of the first segments is handed
// out at once and many waves poll for segments of their slots still running
// (0.4e6 walkers: FP64 33.7 / 48.2, mixed 31.0 / 82.6), and below one round
// all of them do.  Other walks, and walks so long that the item count (slot
// waves x segments) would pass 2^30, take the one-launch kernel.
template <template <typename, int> class Walker, typename LabelT, int NS>
hipError_t run_seg(const WalkPlan& p, hipStream_t s, int* kind) {
    const int grid_blocks = seg_grid<Walker<LabelT, NS>, LabelT>();
    const uint32_t seg_steps = seg_steps_of(p.n_steps);
    const int64_t n_seg64 = p.n_steps == 0 ? 1 : (p.n_steps + seg_steps - 1) / seg_steps;
    const int64_t wpq64 = p.n_slots / kWave / kSegQueues;
    const int64_t slot_waves = p.n_slots / kWave;
    const int64_t resident = static_cast<int64_t>(grid_blocks) * kWavesPerBlock;
    const int choice = g_walk_choice.load(std::memory_order_relaxed);
    const bool in_window = 2 * slot_waves > 3 * resident && 2 * slot_waves <= 9 * resident;
    const bool persistent = (choice == RMS_WALK_AUTO ? in_window : choice == RMS_WALK_PERSISTENT) &&
                            wpq64 * n_seg64 <= (int64_t(1) << 30);
    *kind = persistent ? RMS_WALK_PERSISTENT : RMS_WALK_ONE_LAUNCH;
    // queue heads, failure word and completion counters start at zero; the
    // host reads the failure word after either kernel
    const int64_t n_ctl = kSegCtlFixed + p.n_slots / kWave;
    seg_init_kernel<<<dim3(static_cast<unsigned>((n_ctl + kBlock - 1) / kBlock)), kBlock, 0, s>>>(
        p.seg_ctl, n_ctl);
    if (!persistent) {
        walk_kernel<Walker<LabelT, NS>, LabelT>
            <<<dim3(static_cast<unsigned>((p.n_slots + kBlock - 1) / kBlock)), kBlock, 0, s>>>(p);
        return hipGetLastError();
    }
    const uint32_t n_seg = static_cast<uint32_t>(n_seg64);
    const uint32_t wpq = static_cast<uint32_t>(wpq64);
    walk_seg_kernel<Walker<LabelT, NS>, LabelT>
        <<<dim3(static_cast<unsigned>(grid_blocks)), kBlock, 0, s>>>(
            p, n_seg, seg_steps, wpq, g_seg_poll_limit.load(std::memory_order_relaxed));
    return hipGetLastError();
}

template <template <typename, int> class Walker, typename LabelT>
hipError_t run_seg_ns(const WalkPlan& p, hipStream_t s, int* kind) {
    switch (p.n_shapes) {
        case 0: return run_seg<Walker, LabelT, 0>(p, s, kind);
        case 1: return run_seg<Walker, LabelT, 1>(p, s, kind);
        case 2: return run_seg<Walker, LabelT, 2>(p, s, kind);
        case 3: return run_seg<Walker, LabelT, 3>(p, s, kind);
        case 4: return run_seg<Walker, LabelT, 4>(p, s, kind);
        default: return hipErrorInvalidValue;
    }
}

template <template <typename, int> class Walker, typename LabelT>
hipError_t run_ns(const WalkPlan& p, hipStream_t s) {
    const int64_t slots = p.order ? p.n_slots : p.n_walkers;
    const dim3 grid(static_cast<unsigned>((slots + kBlock - 1) / kBlock));
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

size_t order_bytes(int64_t n) {
    if (!order_used(n)) return 0;
    return static_cast<size_t>(kXcds * order_chunk(n) + (int64_t(1) << (3 * cell_bits(n))) + n +
                               kMaxChunks) *
           sizeof(uint32_t);
}

int64_t order_slots(int64_t n) { return order_used(n) ? kXcds * order_chunk(n) : n; }

// Ordered runs that may take the persistent walk get its state buffer: up to
// 4.5 rounds of the largest resident wave count of the walkers (six per
// SIMD); run_seg makes the exact choice from the kernel's occupancy.
size_t seg_state_bytes(int precision, int n_shapes, int64_t n) {
    if (!order_used(n)) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int64_t max_walkers = int64_t(9) * cus * 4 * 6 * kWave / 2;
    if (n > max_walkers) return 0;
    return static_cast<size_t>(order_slots(n)) * walker_state_bytes(precision, 2, n_shapes);
}

size_t seg_ctl_bytes(int64_t n) {
    if (!order_used(n)) return 0;
    return static_cast<size_t>(kSegCtlFixed + order_slots(n) / kWave) * sizeof(uint32_t);
}

// Scratch behind p.order: order[n_slots], count[n_cells], keys[n_walkers],
// totals[kMaxChunks].
hipError_t launch_order(const WalkPlan& p, hipStream_t s) {
    if (!p.order) return hipSuccess;
    const int64_t n = p.n_walkers;
    const int cb = cell_bits(n);
    const uint32_t n_cells = 1u << (3 * cb);
    uint32_t* count = p.order + p.n_slots;
    uint32_t* keys = count + n_cells;
    uint32_t* totals = keys + n;
    const uint32_t n_chunks = (n_cells + kScanChunk - 1) / kScanChunk;
    const int64_t init = p.n_slots > n_cells ? p.n_slots : n_cells;
    order_init_kernel<<<dim3(static_cast<unsigned>((init + kBlock - 1) / kBlock)), kBlock, 0, s>>>(
        p.order, p.n_slots, count, n_cells);
    const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock));
    order_keys_kernel<<<grid, kBlock, 0, s>>>(p, count, keys, cb);
    order_scan_chunks_kernel<<<n_chunks, kScanChunk, 0, s>>>(count, n_cells, totals);
    order_scan_totals_kernel<<<1, kMaxChunks, 0, s>>>(totals, n_chunks);
    order_scatter_kernel<<<grid, kBlock, 0, s>>>(keys, count, totals, p.order, n, order_chunk(n));
    return hipGetLastError();
}

void set_walk_choice(int choice) { g_walk_choice.store(choice, std::memory_order_relaxed); }

void set_seg_poll_limit(uint32_t polls) {
    g_seg_poll_limit.store(polls, std::memory_order_relaxed);
}

hipError_t launch_walk(const WalkPlan& p, int precision, hipStream_t s, int* kind) {
    *kind = RMS_WALK_ONE_LAUNCH;
    if (p.n_walkers <= 0) return hipSuccess;
    const bool u8 = p.label_bytes == 1;
    const bool seg = p.order && p.seg_state && p.seg_ctl;
    if (p.thr_mt) {  // absorbing membranes
        if (seg) {
            if (precision == RMS_FP64)
                return u8 ? run_seg_ns<dev::WalkerF64MT, uint8_t>(p, s, kind)
                          : run_seg_ns<dev::WalkerF64MT, uint16_t>(p, s, kind);
            return u8 ? run_seg_ns<dev::WalkerMixedMT, uint8_t>(p, s, kind)
                      : run_seg_ns<dev::WalkerMixedMT, uint16_t>(p, s, kind);
        }
        if (precision == RMS_FP64)
            return u8 ? run_ns<dev::WalkerF64MT, uint8_t>(p, s)
                      : run_ns<dev::WalkerF64MT, uint16_t>(p, s);
        return u8 ? run_ns<dev::WalkerMixedMT, uint8_t>(p, s)
                  : run_ns<dev::WalkerMixedMT, uint16_t>(p, s);
    }
    if (seg) {
        if (precision == RMS_FP64)
            return u8 ? run_seg_ns<dev::WalkerF64, uint8_t>(p, s, kind)
                      : run_seg_ns<dev::WalkerF64, uint16_t>(p, s, kind);
        return u8 ? run_seg_ns<dev::WalkerMixed, uint8_t>(p, s, kind)
                  : run_seg_ns<dev::WalkerMixed, uint16_t>(p, s, kind);
    }
    if (precision == RMS_FP64)
        return u8 ? run_ns<dev::WalkerF64, uint8_t>(p, s) : run_ns<dev::WalkerF64, uint16_t>(p, s);
    return u8 ? run_ns<dev::WalkerMixed, uint8_t>(p, s) : run_ns<dev::WalkerMixed, uint16_t>(p, s);
}

hipError_t launch_start_try(const WalkPlan& p, hipStream_t s) {
    if (!p.accept || !p.start_try || p.n_walkers <= 0) return hipSuccess;
    start_try_kernel<<<dim3(static_cast<unsigned>((p.n_walkers + kBlock - 1) / kBlock)), kBlock, 0,
                       s>>>(p);
    return hipGetLastError();
}

hipError_t launch_item_range(PackedItem* items, int n_items, uint32_t step_begin,
                             uint32_t step_end, uint32_t flags, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    item_range_kernel<<<dim3(static_cast<unsigned>((n_items + kBlock - 1) / kBlock)), kBlock, 0,
                        s>>>(items, n_items, step_begin, step_end, flags);
    return hipGetLastError();
}

hipError_t launch_walk_packed(const PackedItem* items, int n_items, const WalkPlan* plans,
                              int precision, int label_bytes, int n_shapes, bool mt,
                              hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    const bool u8 = label_bytes == 1;
    if (mt) {
        if (precision == RMS_FP64)
            return u8 ? packed_ns<dev::WalkerF64MT, uint8_t>(items, n_items, plans, n_shapes, s)
                      : packed_ns<dev::WalkerF64MT, uint16_t>(items, n_items, plans, n_shapes, s);
        return u8 ? packed_ns<dev::WalkerMixedMT, uint8_t>(items, n_items, plans, n_shapes, s)
                  : packed_ns<dev::WalkerMixedMT, uint16_t>(items, n_items, plans, n_shapes, s);
    }
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
