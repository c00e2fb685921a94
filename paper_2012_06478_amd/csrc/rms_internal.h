// Internal interface between the host side of the library (rms_api.cpp) and
// the gfx950 kernels (rms_walk.hip, rms_reduce.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rms {

constexpr int kBlock = 256;  // threads per block of every kernel here
constexpr int kDumpFixed = 15;

// Device label volume: the nx*ny*nz labels inside a one-voxel periodic halo,
// (nx+2)*(ny+2)*(nz+2) entries, x fastest, so the voxel across any face of an
// interior voxel is one stride away.  A halo entry holds the label of the
// periodic image, with bit a of its flag field set when it lies beyond the
// volume along axis a; interior entries have no flags.  uint8 entries (at most
// kMaxLabelsU8 labels) keep the flags in bits 5-7, uint16 entries in 13-15.
constexpr int kMaxLabelsU8 = 32;
constexpr int halo_shift(int label_bytes) { return label_bytes == 1 ? 5 : 13; }

// Everything the walk kernel reads.  All pointers are device pointers.
struct WalkPlan {
    const void* labels;  // padded device label volume (above), uint8 or uint16
    int label_bytes;     // bytes per entry of `labels`
    int nx, ny, nz;
    int px, pxy;         // strides of y and z in the padded volume: nx+2, (nx+2)(ny+2)
    uint32_t div_nx_m, div_nx_sh;    // n / nx == (n div_nx_m) >> div_nx_sh for n < 2^31
    uint32_t div_nxy_m, div_nxy_sh;  // n / (nx ny), likewise
    uint32_t div_px_m, div_px_sh;    // n / px, likewise
    uint32_t div_pxy_m, div_pxy_sh;  // n / pxy, likewise
    const uint32_t* allowed;  // ascending linear indices of non-dead voxels, or null (all)
    uint32_t n_allowed;
    const uint64_t* accept;   // [n_labels] start acceptance thresholds floor(c / max c 2^32)
                              // with spin concentrations, or null: uniform start
    uint32_t* start_try;      // [n_walkers] accepted start attempt of each walker (filled by
                              // launch_start_try before the walk), or null: attempt 0
    int n_labels;
    const double* sigma;    // [n_labels] step length per label, voxel units
    const double* inv_t2;   // [n_labels] 1/T2 (0 for none)
    const uint64_t* thr;    // [n_labels^2] permeation thresholds floor(P 2^32) in [0, 2^32]:
                            // a 32-bit word < thr permeates (2^32: always)
    const uint32_t* thr_mt; // [n_labels^2] saturation thresholds at absorbing membranes, or
                            // null: no membrane absorbs
    const float* sigma_f;   // fp32 copies for the mixed form
    const float* inv_t2_f;
    uint64_t seed;
    int64_t n_walkers;
    int64_t n_steps;
    double dt;
    double voxel_um;
    int n_shapes;
    const double* gdt;   // [n_shapes][n_steps] dt * G_s[i]
    const double2* trig; // [kTrigSize + 1] 2 cos, 2 sin of 2 pi j / kTrigSize, then the
                         // series' leading coefficients (fill_trig_table)
    double* wstate;      // [n_walkers][kDumpFixed + 3 n_shapes] per-walker results
    void* state;         // [n_walkers] resumable walker states (packed launches), or null
    uint32_t* order;     // [n_slots] walker of each thread slot (kNoWalker: none), or
                         // null: slot i runs walker i; followed by the ordering scratch
    int64_t n_slots;
    void* seg_state;     // [n_slots] walker states between segments of the persistent
                         // walk (slot order), or null: one thread per walker, whole walk
    uint32_t* seg_ctl;   // [kSegCtlFixed + n_slots / 64] queue heads, wait-failure
                         // flag, segments finished per wave of 64 slots
};

constexpr uint32_t kNoWalker = 0xFFFFFFFFu;

// Angles of the direction table: (2 cos, 2 sin) of 2 pi j / kTrigSize,
// followed by one entry holding the leading coefficients (-1/7!, -1/6!) of
// the sine and cosine series of the remainder angle.
constexpr int kTrigSize = 256;
constexpr double2 kLeadCoefficients = {-1.0 / 5040.0, -1.0 / 720.0};

// Control words of the persistent walk: eight queue heads, then the flag a
// block sets when a wait for an earlier segment gives up.
constexpr int kSegQueues = 8;
constexpr int kSegErrorWord = kSegQueues;
constexpr int kSegCtlFixed = kSegQueues + 1;

// One block of a packed launch: thread slots [first_slot, first_slot + kBlock)
// of plan `plan` (walker = slot, or plan.order[slot]), steps [step_begin,
// step_end) from any step_begin.  flags: kItemRecord also writes each
// walker's record (plan.wstate) when the range stops before the last step.
struct PackedItem {
    int64_t first_slot;
    int plan;
    uint32_t step_begin, step_end;
    uint32_t flags;
};
constexpr uint32_t kItemRecord = 1u;

// Everything the reduction kernels read.
struct ReducePlan {
    const double* wstate;
    int64_t n_walkers;
    int width;   // doubles per walker record
    int n_shapes;
    int n_sig;   // n_shapes * n_b * n_dirs
    const double* kg;      // [n_sig][3] k_{s,b} * unit direction, um^-1 ms^-1
    const int* sig_shape;  // [n_sig] shape of each signal
    int n_acc;             // 25 + 2 n_sig accumulated values per walker
    int n_blocks;          // blocks of the contribution kernel
    double* partial;       // [n_acc][n_blocks]
    double* sums;          // [n_acc]
    int n_dirs;
    const double* dirs;    // [n_dirs][3] unit directions
    double t_ms;           // n_steps * dt
    double* result;        // [25 + 2 n_sig + 2 n_dirs]
};

constexpr int kAccFixed = 25;  // alpha, 6 M2, 15 M4, 3 counters

// Whole walk of every walker of one run (precision RMS_FP64 or RMS_MIXED);
// *kind receives the walk kernel launched (RMS_WALK_ONE_LAUNCH or
// RMS_WALK_PERSISTENT).
hipError_t launch_walk(const WalkPlan& p, int precision, hipStream_t s, int* kind);
// Options of the walk launch (rms_set_option): kernel choice (RMS_WALK_AUTO,
// RMS_WALK_ONE_LAUNCH, RMS_WALK_PERSISTENT) and the persistent walk's poll
// limit.
void set_walk_choice(int choice);
void set_seg_poll_limit(uint32_t polls);
// A packed launch over several runs that share precision, label width, shape
// count and whether membranes absorb (mt: every plan has thr_mt): each block advances its walkers by a range of steps, starting
// from the stored state (or the start when step_begin == 0) and storing the
// state again (or the final record when step_end == n_steps; with kItemRecord
// the record as well).
hipError_t launch_walk_packed(const PackedItem* items, int n_items, const WalkPlan* plans,
                              int precision, int label_bytes, int n_shapes, bool mt,
                              hipStream_t s);
// Sets the step range and flags of items[0, n_items) on the device.
hipError_t launch_item_range(PackedItem* items, int n_items, uint32_t step_begin,
                             uint32_t step_end, uint32_t flags, hipStream_t s);
// Walker order for one run (rms_walk.hip): slots in blocks that run on one
// XCD take walkers whose start voxels are close.  order_bytes() is the device
// memory it needs (0 when the run keeps slot i = walker i), order_slots() the
// thread slots of the walk launch; launch_order() fills p.order.
size_t order_bytes(int64_t n_walkers);
// Device memory of the persistent walk of an ordered run (state + control).
size_t seg_state_bytes(int precision, int n_shapes, int64_t n_walkers);
size_t seg_ctl_bytes(int64_t n_walkers);
int64_t order_slots(int64_t n_walkers);
hipError_t launch_order(const WalkPlan& p, hipStream_t s);
// Accepted start attempt of every walker when the start is weighted by spin
// concentration (p.accept and p.start_try set); a no-op otherwise.
hipError_t launch_start_try(const WalkPlan& p, hipStream_t s);
// Bytes of one resumable walker state.
size_t walker_state_bytes(int precision, int label_bytes, int n_shapes);
hipError_t launch_reduce(const ReducePlan& p, hipStream_t s);

}  // namespace rms
