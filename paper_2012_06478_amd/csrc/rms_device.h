// Device-side walkers for gfx950: the per-walker state and one step of the
// Monte Carlo walk of Lee, Fieremans & Novikov (arXiv 2012.06478), in two
// precision forms.  Included by the kernel translation unit only.
//
// Method:
//   - a step has fixed length ds = sqrt(6 D dt) and a uniform random direction
//     (section 2.2, items 2-3; section 2.1.3, Eq. step-size);
//   - with ds below the voxel size a step meets at most one face per axis, so
//     at most three (section 2.1.1 and the corner-reflector figure); a face
//     between equal labels is transparent, one between different labels is a
//     membrane: permeate with the probability of Eq. (perm-prob-general), else
//     reflect specularly (section 2.1.3, section 2.2 items 3-4);
//   - the phase accumulates g . (x - x0) after every step and the T2 weight the
//     time spent in each compartment (section 2.3, Eq. signal; section 2.1.4
//     Eq. wt-relax).
//
// Face walk.  Reflection flips one component of the direction and passing
// changes only the voxel index, so the path length at which a step reaches
// each axis' face is fixed at the start of the step: e_a = gap_a / |v_a|.  A
// step decides which faces lie inside its path budget (gap_a < budget |v_a|)
// and in which order they come (e_a < e_b iff gap_a |v_b| < gap_b |v_a|) with
// multiplications only, then visits them in that order; only a permeation
// into a label with another step length moves the budget (the remaining share
// of the step's duration is kept), and only then is an e_a divided out.  The
// end point on each axis follows in closed form.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit
// seed with counter (index, substream, walker_lo, walker_hi): substream 0
// block j gives the directions of steps 2j+1 (words 0, 1) and 2j+2 (words 2,
// 3); the first membrane word of step i is word (i-1) mod 4 of substream 1
// block (i-1)/4 (computed for the whole wave once per four steps, since some
// lane of a wave meets a membrane in most steps); the rare second and third
// membrane words of a step are words 0 and 1 of substream 3 block i-1;
// substream 2 blocks 0 and 1 give the start.  A walker's trajectory therefore
// depends only on (seed, walker index, step index), and a walk can stop after
// any step and resume from its stored state with identical results.
//
// Mixed form: the position is an exact int32 voxel index plus an fp32 offset,
// so a coordinate keeps the same absolute precision anywhere in the volume
// (the point of taking voxel membership from the integer part, section
// 2.1.1).  Directions take u1, u2 from the top 24 bits of the same words and
// use the hardware sine and cosine (argument in revolutions, so 2 pi u needs
// no range reduction); face tests, end points and budgets are fp32; the
// displacement is a double holding the whole voxels crossed minus the start
// offset (exact) plus the fp32 offset; the phase and R accumulate in fp64 (a
// double FMA issues at the fp32 rate on gfx950, so this costs less than a
// compensated fp32 sum).
// Permeation uses the same 32-bit thresholds and words as the fp64 form.
#pragma once

#include "rms_internal.h"

namespace rms {
namespace dev {

// a ^ b ^ c in one instruction (gfx950 three-input bit operation, truth
// table 0x96 over the operand patterns 0xF0, 0xCC, 0xAA)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// The counter words of Philox4x32-10 as the walkers use them: (index,
// substream, walker, high word) with key (k0, k1) = the seed.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = xor3(static_cast<uint32_t>(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3(static_cast<uint32_t>(p0 >> 32), c3, k1);
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// The same generator for counters whose index and substream are the same
// across the wave and whose high word is 0: the first round's n2 and p0 and
// the second round's p1 and c3 are then wave-uniform, and the xors of those
// two rounds pair the uniform terms first, so that the compiler keeps them
// in scalar registers and each vector result costs one instruction (a vector
// instruction reads at most one scalar register).
__device__ __forceinline__ uint4 philox4x32_10_uniform(uint32_t c0, uint32_t c1, uint32_t c2,
                                                       uint32_t k0, uint32_t k1) {
    uint32_t c3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t h0 = static_cast<uint32_t>(p0 >> 32), h1 = static_cast<uint32_t>(p1 >> 32);
        uint32_t n0, n2;
        if (r == 0) {
            n0 = h1 ^ (c1 ^ k0);
            n2 = (h0 ^ c3) ^ k1;
        } else if (r == 1) {
            n0 = c1 ^ (h1 ^ k0);
            n2 = h0 ^ (c3 ^ k1);
        } else {
            n0 = xor3(h1, c1, k0);
            n2 = xor3(h0, c3, k1);
        }
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// (w + 1/2) 2^-32, exact in double (both steps are exact)
__device__ __forceinline__ double unit_open(uint32_t w) {
    return (static_cast<double>(w) + 0.5) * 0x1p-32;
}

// fma(a, b, k) with the constant k taken from a scalar register pair: written
// as the three-operand instruction so the compiler does not keep the
// polynomial coefficients in vector registers and copy one before every
// accumulate.
struct FmaSgpr {
    __device__ __forceinline__ double operator()(double a, double b, double k) const {
        double d;
        asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(k));
        return d;
    }
};

// 2 cos(2 pi u) and 2 sin(2 pi u) for u = (w + 1/2) 2^-32, within a few ulp
// (the factor 2 of the direction's transverse length comes from the table,
// exactly).  The top eight bits of w pick the angle A = 2 pi j / 256, whose
// (2 cos A, 2 sin A) `tab` holds as one 16-byte entry; the rest is
// a = 2 pi (w mod 2^24 + 1/2) 2^-32 in (0, 2 pi / 256), whose sine and cosine
// are the Taylor series through a^7 and a^6 (the next terms are below 1e-17
// there), evaluated by Horner's rule in a^2; the angle-sum formulas combine
// the two.  `lead` holds the series' leading coefficients (-1/7!, -1/6!),
// kLeadCoefficients: the walker reads them from LDS at each step rather than
// keeping them in registers.  `fk` is the fused multiply-add used for the
// Horner steps (its third operand is a coefficient).
template <class Fma>
__host__ __device__ __forceinline__ void sincos_2pi_word(uint32_t w, const double2* tab,
                                                         double2 lead, double* s_out,
                                                         double* c_out, Fma fk) {
    const double2 e = tab[w >> 24];
    const double cA = e.x, sA = e.y;
    const double a = (static_cast<double>(w & 0xFFFFFFu) + 0.5) * (6.283185307179586 * 0x1p-32);
    const double z = a * a;
    double ps = fk(z, lead.x, 1.0 / 120.0);  // sin a = a (1 - z/3! + z^2/5! - z^3/7!)
    ps = fk(z, ps, -1.0 / 6.0);
    const double sa = fma(a * z, ps, a);
    double pc = fk(z, lead.y, 1.0 / 24.0);   // cos a = 1 - z/2! + z^2/4! - z^3/6!
    pc = fma(z, pc, -0.5);
    const double ca = fma(z, pc, 1.0);
    *c_out = fma(cA, ca, -(sA * sa));
    *s_out = fma(sA, ca, cA * sa);
}

// sqrt(y) for finite normal y > 0: the hardware reciprocal square root
// estimate, one coupled Newton step on (sqrt y, 1/(2 sqrt y)) and a final
// residual correction (Goldschmidt's iteration).
__device__ __forceinline__ double sqrt_pos(double y) {
    const double r = __builtin_amdgcn_rsq(y);
    double g = y * r;
    double h = 0.5 * r;
    const double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    const double d = fma(-g, g, y);
    return fma(d, h, g);
}

// Walker identity and Philox key.
struct Ids {
    uint32_t wlo, whi, k0, k1;
};

// Identity of walker w (below 2^32 - 1: the host refuses larger runs, so the
// high counter word is 0) under the given seed.  Walkers with
// kUniformCounters take the high word as the constant 0 and walk with the
// streams specialised for it (philox4x32_10_uniform); the double-precision
// walker takes it as w >> 32, which the compiler cannot prove 0 where the
// walker index is 64 bits wide: specialised, it ran 2% slower on the 200^3
// packing (and, before its series coefficients moved to LDS, spilled).
template <class Walker>
__device__ __forceinline__ Ids walker_ids(int64_t w, uint64_t seed) {
    const uint32_t hi = Walker::kUniformCounters ? 0u : static_cast<uint32_t>(w >> 32);
    return Ids{static_cast<uint32_t>(w), hi, static_cast<uint32_t>(seed),
               static_cast<uint32_t>(seed >> 32)};
}

// Block of substream 3 for step index i0: the second and third membrane words
// of the step.  Few steps hit a membrane twice, so the block is computed only
// on that branch; the empty asm on the counter keeps the compiler from
// evaluating the ten rounds speculatively on every step.
__device__ __forceinline__ uint4 rare_block(uint32_t i0, const Ids& id) {
    uint32_t c = i0;
    asm volatile("" : "+v"(c));
    return philox4x32_10(c, 3u, id.wlo, id.whi, id.k0, id.k1);
}

// n / d for n < 2^31 as (n m) >> sh with m = ceil(2^sh / d), sh = 31 +
// ceil(log2 d): exact, because the error n (m - 2^sh/d) / 2^sh stays below
// 2^-ceil(log2 d) <= 1/d.  m and sh come from the host.
__device__ __forceinline__ uint32_t div_magic(uint32_t n, uint32_t m, uint32_t sh) {
    return static_cast<uint32_t>((static_cast<uint64_t>(n) * m) >> sh);
}

// Order in which a step reaches the faces of its three axes, by multiplying
// only: axis a reaches its face after path length e_a = g_a / m_a (g_a >= 0 the
// gap to the face, m_a = |v_a| > 0), and e_a <= e_b exactly when
// g_a m_b <= g_b m_a.  For each pair i < j the sign of fma(g_i, m_j, -g_j m_i)
// decides whether i comes first (ties go to the lower axis, as when the nearest
// face is taken with x < y < z on ties: a walker left exactly on two faces by a
// corner reflection has two zero gaps); the three bits (0 before 1, 0 before 2,
// 1 before 2) index the permutation, stored as 2-bit fields of two constants.
// Patterns no order gives (reachable only by rounding at near-ties) map to
// (0, 1, 2).
template <typename Real>
__host__ __device__ __forceinline__ void event_order(const Real g[3], const Real m[3], int ax[3]) {
    const auto first = [&](int i, int j) -> uint32_t {
        return fma(g[i], m[j], -(g[j] * m[i])) <= Real(0) ? 1u : 0u;
    };
    const uint32_t sh = 2u * (first(0, 1) | (first(0, 2) << 1) | (first(1, 2) << 2));
    constexpr uint32_t kFirst = 0x110Au;   // first axis for patterns 0..7: 2 2 0 0 1 0 1 0
    constexpr uint32_t kSecond = 0x4691u;  // second axis:                  1 0 1 2 2 1 0 1
    ax[0] = static_cast<int>((kFirst >> sh) & 3u);
    ax[1] = static_cast<int>((kSecond >> sh) & 3u);
    ax[2] = 3 - ax[0] - ax[1];
}

// m ? x : y for a word m of all ones or all zeros, as one three-input bit
// operation per 32-bit half (truth table 0xE4 over the operand patterns 0xF0,
// 0xCC, 0xAA).  gfx950 issues these two at a time from different waves,
// where a select on a lane mask (a VOP3 instruction) issues alone; the end
// point's selects use them with masks taken from the reflect and pass bits.
__device__ __forceinline__ double select_bits(uint32_t m, double x, double y) {
    const uint64_t xb = __double_as_longlong(x), yb = __double_as_longlong(y);
    const uint32_t lo = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(xb),
                                                    static_cast<uint32_t>(yb), m, 0xE4);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(xb >> 32),
                                                    static_cast<uint32_t>(yb >> 32), m, 0xE4);
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

__device__ __forceinline__ float select_bits(uint32_t m, float x, float y) {
    return __uint_as_float(__builtin_amdgcn_bitop3_b32(__float_as_uint(x), __float_as_uint(y), m, 0xE4));
}

// all ones if bit a of w is set, else zero
__device__ __forceinline__ uint32_t bit_mask(uint32_t w, int a) {
    return static_cast<uint32_t>(static_cast<int32_t>(w << (31 - a)) >> 31);
}

// v[a] for a runtime axis index a in {0, 1, 2}, as two selects (the three
// reads are unconditional so the compiler does not branch on a)
template <typename T>
__device__ __forceinline__ T pick(const T (&v)[3], int a) {
    const T v0 = v[0], v1 = v[1], v2 = v[2];
    const T r = a == 1 ? v1 : v2;
    return a == 0 ? v0 : r;
}

struct Coords {
    int c[3];
};

// Coordinates of linear index lin (< 2^31) in a volume of row length n1 and
// plane size n12, with the division magic numbers of n1 and n12.
__device__ __forceinline__ Coords coords_of(uint32_t lin, uint32_t n1, uint32_t n12,
                                            uint32_t m1, uint32_t sh1, uint32_t m12,
                                            uint32_t sh12) {
    const uint32_t z = div_magic(lin, m12, sh12);
    const uint32_t r = lin - z * n12;
    const uint32_t y = div_magic(r, m1, sh1);
    Coords k;
    k.c[0] = static_cast<int>(r - y * n1);
    k.c[1] = static_cast<int>(y);
    k.c[2] = static_cast<int>(z);
    return k;
}

// Index in the padded device volume of voxel `lin` of the nx*ny*nz volume.
__device__ __forceinline__ int padded_index(const WalkPlan& p, int lin) {
    const Coords k = coords_of(static_cast<uint32_t>(lin), static_cast<uint32_t>(p.nx),
                               static_cast<uint32_t>(p.nx) * static_cast<uint32_t>(p.ny),
                               p.div_nx_m, p.div_nx_sh, p.div_nxy_m, p.div_nxy_sh);
    return (k.c[0] + 1) + p.px * (k.c[1] + 1) + p.pxy * (k.c[2] + 1);
}

// Voxel coordinates of an interior index of the padded volume.
__device__ __forceinline__ Coords volume_coords(const WalkPlan& p, int plin) {
    Coords k = coords_of(static_cast<uint32_t>(plin), static_cast<uint32_t>(p.px),
                         static_cast<uint32_t>(p.pxy), p.div_px_m, p.div_px_sh, p.div_pxy_m,
                         p.div_pxy_sh);
    k.c[0] -= 1;
    k.c[1] -= 1;
    k.c[2] -= 1;
    return k;
}

// Halo flag field and label of a padded-volume entry.
template <typename LabelT>
struct LabelBits {
    static constexpr int kShift = halo_shift(static_cast<int>(sizeof(LabelT)));
    static constexpr uint32_t kMask = (1u << kShift) - 1u;
};

// A step starts in an interior voxel and crosses at most one face per axis, so
// every voxel it visits lies within one voxel of the volume along each axis:
// inside the padded volume.  If it ends in the halo (flag bit a set on the
// entry it ended in: it passed the face at the volume's end along axis a),
// it moves back by one period along each flagged axis, in the direction
// opposite to its pass.
// (Offsets here are in bytes of the padded volume, `bytes` per entry.)
__device__ __forceinline__ uint32_t wrap_halo(const WalkPlan& p, uint32_t off, uint32_t flags,
                                              uint32_t posm, int bytes) {
    const int per[3] = {p.nx * bytes, p.ny * p.px * bytes, p.nz * p.pxy * bytes};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if ((flags >> a) & 1u) off -= static_cast<uint32_t>(((posm >> a) & 1u) ? per[a] : -per[a]);
    return off;
}

// Permeation threshold from label l into label nl (both below 4096, so the
// byte offset 8 (l L + nl) fits 32 bits and l L is a 24-bit multiply): a
// 64-bit floor(P 2^32), so that P = 1 (2^32) permeates on every word.
__device__ __forceinline__ uint64_t threshold(const WalkPlan& p, int l, int nl) {
    const uint32_t off = (__umul24(static_cast<uint32_t>(l), static_cast<uint32_t>(p.n_labels)) +
                          static_cast<uint32_t>(nl)) * 8u;
    return *reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(p.thr) + off);
}

// Saturation threshold for a walker in label l meeting label nl at an
// absorbing membrane (0: the face does not absorb); layout as threshold().
__device__ __forceinline__ uint32_t threshold_mt(const WalkPlan& p, int l, int nl) {
    const uint32_t off = (__umul24(static_cast<uint32_t>(l), static_cast<uint32_t>(p.n_labels)) +
                          static_cast<uint32_t>(nl)) * 4u;
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(p.thr_mt) + off);
}

// Entry at byte offset `off` of the padded label volume.  Offsets stay below
// 2^32 (fewer than 2^31 entries of at most two bytes), so the load takes a
// 32-bit offset from the volume's base and needs no 64-bit address arithmetic.
template <typename LabelT>
__device__ __forceinline__ uint32_t entry(const LabelT* __restrict__ lab, uint32_t off) {
    return *reinterpret_cast<const LabelT*>(reinterpret_cast<const char*>(lab) + off);
}

// Start (section 2.2, item 1): uniform over the voxels that are not dead, then
// uniform inside the voxel.  With spin concentrations (App. C, general case)
// the start density is proportional to the voxel's concentration: attempt j
// draws from substream 2 blocks 2j and 2j + 1 and is kept when word 1 of the
// second is below the label's acceptance threshold floor(c / max c 2^32); at
// most kMaxStartTries attempts (the host refuses mean acceptance below 1e-3).
struct Start {
    int lin;
    uint32_t wox, woy, woz;  // offset words
};

constexpr uint32_t kMaxStartTries = 65536u;

// Attempt j of the start draw; *accept_word is word 1 of its second block.
__device__ __forceinline__ Start start_attempt(const WalkPlan& p, const Ids& id, uint32_t j,
                                               uint32_t* accept_word) {
    const uint4 b0 = philox4x32_10(2u * j, 2u, id.wlo, id.whi, id.k0, id.k1);
    const uint4 b1 = philox4x32_10(2u * j + 1u, 2u, id.wlo, id.whi, id.k0, id.k1);
    const uint64_t r64 = (static_cast<uint64_t>(b0.y) << 32) | b0.x;
    const uint32_t rank =
        static_cast<uint32_t>(__umul64hi(r64, static_cast<uint64_t>(p.n_allowed)));
    Start s;
    s.lin = static_cast<int>(p.allowed ? p.allowed[rank] : rank);
    s.wox = b0.z;
    s.woy = b0.w;
    s.woz = b1.x;
    *accept_word = b1.y;
    return s;
}

// The accepted attempt of a walker's start with spin concentrations (run by a
// kernel of its own before the walk, which stores it in p.start_try).
__device__ __forceinline__ uint32_t start_try_of(const WalkPlan& p, const Ids& id) {
    for (uint32_t j = 0;; ++j) {
        uint32_t w;
        const Start s = start_attempt(p, id, j, &w);
        if (j + 1 == kMaxStartTries) return j;
        const int e = padded_index(p, s.lin);  // an interior entry: the label, no flags
        const uint32_t lv = p.label_bytes == 1 ? static_cast<const uint8_t*>(p.labels)[e]
                                               : static_cast<const uint16_t*>(p.labels)[e];
        if (static_cast<uint64_t>(w) < p.accept[lv]) return j;
    }
}

// The start of walker w (id): the first attempt, or the accepted one found
// before the walk when the start is weighted by spin concentration.
__device__ __forceinline__ Start draw_start(const WalkPlan& p, const Ids& id) {
    uint32_t j = 0u;
    if (p.start_try)
        j = p.start_try[(static_cast<uint64_t>(id.whi) << 32) | id.wlo];
    uint32_t w;
    return start_attempt(p, id, j, &w);
}

// ---------------------------------------------------------------------------
// Double-precision form.
// ---------------------------------------------------------------------------
// MT: membranes may absorb (magnetization transfer, end of section 2.1.3):
// at a membrane hit a walker is saturated with the pair's probability, by a
// word of its own (the first membrane of step i: word (i-1) mod 4 of
// substream 4 block (i-1)/4, computed for the wave with the first membrane
// block; the second and third: words 2 and 3 of the substream-3 block), and
// keeps walking with weight 0 (Eq. wt-mt), held as R = infinity.  Without MT
// that code is not compiled.
template <typename LabelT, int NS, bool MT>
struct WalkerF64T {
    static constexpr int kShapes = NS > 0 ? NS : 1;
    static constexpr bool kTrig = true;  // direction from the LDS angle table
    // waves per SIMD the walk kernels ask for: five (96 registers); the
    // absorbing form holds four more words per step and is given four
    static constexpr int kWaves = MT ? 4 : 5;
    static constexpr bool kMT = MT;
    // streams specialised for a zero high counter word (walker_ids)
    static constexpr bool kUniformCounters = false;
    uint32_t lb;     // byte offset of the voxel's entry in the padded volume
    int l, l0;       // label, label at the start
    uint32_t nface, nhit, nperm;
    double o[3];
    double sig, dti2;  // step length (voxel units) and dt / T2 of the current label
    double d[3];  // displacement, voxel units
    double R;
    double ph[kShapes][3];  // phase vector, voxel units x ms

    __device__ __forceinline__ void init(const WalkPlan& p, const LabelT* __restrict__ lab,
                                         const Ids& id) {
        const Start s = draw_start(p, id);
        lb = static_cast<uint32_t>(padded_index(p, s.lin)) * sizeof(LabelT);
        o[0] = unit_open(s.wox);
        o[1] = unit_open(s.woy);
        o[2] = unit_open(s.woz);
        l = l0 = entry(lab, lb);  // interior: no flags
        sig = p.sigma[l];
        dti2 = p.dt * p.inv_t2[l];
        d[0] = d[1] = d[2] = 0.0;
        R = 0.0;
#pragma unroll
        for (int q = 0; q < kShapes; ++q) ph[q][0] = ph[q][1] = ph[q][2] = 0.0;
        nface = nhit = nperm = 0;
    }

    // One step (index i0 = i - 1) with direction words wa, wb and first
    // membrane word m1.
    __device__ __forceinline__ void step(const WalkPlan& p, const LabelT* __restrict__ lab,
                                         uint32_t i0, uint32_t wa, uint32_t wb, uint32_t m1,
                                         [[maybe_unused]] uint32_t t1,
                                         const Ids& id, const double2* trig) {
        const double u1 = unit_open(wa);
        double sn2, cs2;  // 2 sin and 2 cos of 2 pi u2, u2 = unit_open(wb)
        // the series' leading coefficients from the LDS entry behind the angle
        // table, read at every step (volatile): held in registers across
        // steps they would take four of the walker's 96
        using LdsDouble = const volatile __attribute__((address_space(3))) double;
        LdsDouble* lv = (LdsDouble*)(trig + kTrigSize);
        double2 lead;
        lead.x = lv[0];
        lead.y = lv[1];
        sincos_2pi_word(wb, trig, lead, &sn2, &cs2, FmaSgpr());
        // transverse length 2 sqrt(u1 (1 - u1)); the 2 is in cs2 and sn2
        const double sq = sqrt_pos(u1 * (1.0 - u1));
        const double v[3] = {sq * cs2, sq * sn2, 1.0 - 2.0 * u1};

        // per axis: the gap |F - o| to the face the step moves toward (F = 1
        // moving up, else 0; o stays in [0, 1]) and |v|; a face lies inside
        // the budget sig when gap < sig |v|
        double g[3], m[3];
        uint32_t posm = 0, evm = 0;
        int sst[3];  // byte step in the padded volume across the face each axis moves toward
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool pos = v[a] > 0.0;
            const int st = (a == 0 ? 1 : (a == 1 ? p.px : p.pxy)) * static_cast<int>(sizeof(LabelT));
            sst[a] = pos ? st : -st;
            posm |= pos ? (1u << a) : 0u;
            m[a] = fabs(v[a]);
            g[a] = fabs((pos ? 1.0 : 0.0) - o[a]);
            evm |= g[a] < sig * m[a] ? (1u << a) : 0u;
        }
        int nev = __builtin_popcount(evm);
        int ax[3];
        event_order(g, m, ax);
        // each lane's byte steps in LDS, one row per axis, so that an event's
        // step is read by its axis index instead of picked by two selects
        __shared__ int32_t sst_lds[3][kBlock];
        const uint32_t tid = threadIdx.x;
        sst_lds[0][tid] = sst[0];
        sst_lds[1][tid] = sst[1];
        sst_lds[2][tid] = sst[2];
        // Offsets and entries of the voxels the events reach if every face
        // passes (the common case), loaded together so the step waits for
        // memory once rather than once per event.
        const int nev0 = nev;
        uint32_t cpath[3], rsp[3];  // rsp[k] is set, and read, only for k < nev0
        {
            uint32_t c = lb;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                c += static_cast<uint32_t>(sst_lds[ax[k]][tid]);
                cpath[k] = c;
                if (k < nev0) rsp[k] = entry(lab, c);
            }
        }
        bool spec = true;  // every face so far passed: cpath and rsp hold the voxels reached

        // gap to axis a's face, and the path length to it (divided out only
        // after a permeation)
        const auto face_gap = [&](int a) {
            const double va = pick(v, a), oa = pick(o, a);
            return va > 0.0 ? 1.0 - oa : oa;
        };
        const auto face_len = [&](int a) { return face_gap(a) / fabs(pick(v, a)); };
        double P = 0.0, tau = 1.0;
        uint32_t done = 0, refl = 0;  // axes whose face the step reached; those it reflected at
        uint32_t rawc = 0;  // entry of the voxel last passed into (its halo flags)
        int mw_used = 0;
        uint4 mw;  // words of substream 3, computed before the second membrane hit reads them
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k < nev) {
                const int a = ax[k];
                done |= 1u << a;
                uint32_t nbk, raw;
                if (spec && k < nev0) {
                    nbk = cpath[k];
                    raw = rsp[k];
                } else {  // after a reflection, or a face a permeation brought in
                    nbk = lb + static_cast<uint32_t>(sst_lds[a][tid]);
                    raw = entry(lab, nbk);
                }
                const int nl = static_cast<int>(raw & LabelBits<LabelT>::kMask);
                bool cross = true;
                if (nl != l) {
                    ++nhit;
                    [[maybe_unused]] uint64_t tp = 0u;
                    [[maybe_unused]] uint32_t tm = 0u;
                    if constexpr (MT) {  // both thresholds in one memory round trip
                        tp = threshold(p, l, nl);
                        tm = threshold_mt(p, l, nl);
                    }
                    if (mw_used == 1) mw = rare_block(i0, id);
                    if constexpr (MT) {
                        const uint32_t u = mw_used == 0 ? t1 : (mw_used == 1 ? mw.z : mw.w);
                        if (u < tm) R = INFINITY;  // saturated: weight 0 from here on
                    }
                    const uint32_t word = mw_used == 0 ? m1 : (mw_used == 1 ? mw.x : mw.y);
                    ++mw_used;
                    if constexpr (MT) cross = word < tp;
                    else cross = word < threshold(p, l, nl);
                    if (cross) {
                        ++nperm;
                        const double ek = fmax(face_len(a), P);
                        const double dtau = fmin((ek - P) / sig, tau);
                        R = fma(dtau, dti2, R);
                        tau -= dtau;
                        P = ek;
                        l = nl;
                        sig = p.sigma[nl];
                        dti2 = p.dt * p.inv_t2[nl];
                        // the later faces, in order, that lie inside the new budget:
                        // face_len < pend compared as gap < pend |v| (no division)
                        const double pend = fma(tau, sig, P);
                        nev = k + 1;
#pragma unroll
                        for (int j = k + 1; j < 3; ++j)
                            if (nev == j && face_gap(ax[j]) < pend * fabs(pick(v, ax[j])))
                                nev = j + 1;
                    }
                }
                if (cross) {
                    lb = nbk;
                    rawc = raw;
                } else {
                    refl |= 1u << a;
                    spec = false;
                }
            }
        }
        const uint32_t passed = done & ~refl;
        nface += __builtin_popcount(done);
        const uint32_t halo = rawc >> LabelBits<LabelT>::kShift;
        if (__builtin_expect(halo != 0u, 0))
            lb = wrap_halo(p, lb, halo, posm, static_cast<int>(sizeof(LabelT)));
        const double lend = fma(tau, sig, P);
        R = fma(tau, dti2, R);
        // End point per axis from the free end point o + lend v: mirrored about
        // the face after a reflection; after a pass the same point, one voxel
        // further along the axis.  The displacement is that point minus o.
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool pos = (posm >> a) & 1u;
            const double fr = fma(lend, v[a], o[a]);
            const double t = select_bits(bit_mask(refl, a), (pos ? 2.0 : 0.0) - fr, fr);
            d[a] += t - o[a];
            // +-1 after a pass, else 0: only the high word is not zero (the and
            // as a three-input operation, truth table 0xC0, for the same reason)
            const uint32_t one_hi = pos ? 0x3FF00000u : 0xBFF00000u;
            const uint32_t shift_hi = __builtin_amdgcn_bitop3_b32(bit_mask(passed, a), one_hi, 0u, 0xC0);
            const double shift =
                __longlong_as_double(static_cast<long long>(static_cast<uint64_t>(shift_hi) << 32));
            o[a] = fmin(fmax(t - shift, 0.0), 1.0);
        }
        // phase: a zero gradient sample adds exactly nothing, so no test for it
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const double g = p.gdt[static_cast<int64_t>(q) * p.n_steps + i0];
            ph[q][0] = fma(g, d[0], ph[q][0]);
            ph[q][1] = fma(g, d[1], ph[q][1]);
            ph[q][2] = fma(g, d[2], ph[q][2]);
        }
    }

    // Per-walker record (layout of RMS_DUMP_WIDTH in rms.h).
    __device__ __forceinline__ void finish(const WalkPlan& p, double* out) const {
        const Coords k = volume_coords(p, static_cast<int>(lb / sizeof(LabelT)));
        out[0] = d[0] * p.voxel_um;
        out[1] = d[1] * p.voxel_um;
        out[2] = d[2] * p.voxel_um;
        out[3] = R;
        out[4] = l;
        out[5] = k.c[0];
        out[6] = k.c[1];
        out[7] = k.c[2];
        out[8] = o[0];
        out[9] = o[1];
        out[10] = o[2];
        out[11] = l0;
        out[12] = nface;
        out[13] = nhit;
        out[14] = nperm;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            out[15 + 3 * q] = ph[q][0] * p.voxel_um;
            out[16 + 3 * q] = ph[q][1] * p.voxel_um;
            out[17 + 3 * q] = ph[q][2] * p.voxel_um;
        }
    }
};

template <typename LabelT, int NS>
using WalkerF64 = WalkerF64T<LabelT, NS, false>;
template <typename LabelT, int NS>
using WalkerF64MT = WalkerF64T<LabelT, NS, true>;

// ---------------------------------------------------------------------------
// Mixed-precision form.
// ---------------------------------------------------------------------------
// (w + 1/2) 2^-32 rounded to the nearest float
__device__ __forceinline__ float unit_open_f(uint32_t w) {
    return static_cast<float>(unit_open(w));
}

template <typename LabelT, int NS, bool MT>
struct WalkerMixedT {
    static constexpr int kShapes = NS > 0 ? NS : 1;
    static constexpr bool kTrig = false;  // hardware sine and cosine
    // waves per SIMD the walk kernels ask for: six (80 registers, a small
    // spill); the absorbing form holds four more words per step and is given five
    static constexpr int kWaves = MT ? 5 : 6;
    static constexpr bool kMT = MT;
    // streams specialised for a zero high counter word (walker_ids)
    static constexpr bool kUniformCounters = true;
    uint32_t lb;  // byte offset of the voxel's entry in the padded volume
    int l, l0;
    uint32_t nface, nhit, nperm;
    float o[3];      // offset in the voxel, [0, 1]
    double base[3];  // n - o0, n the signed count of voxels crossed and o0 the
                     // start offset (exact in double): the displacement is base + o
    float sig, dti2;  // step length (voxel units) and dt / T2 of the current label
    double R;             // sum of t_c / T2_c
    double ph[kShapes][3];  // phase vector, voxel units x ms

    __device__ __forceinline__ void init(const WalkPlan& p, const LabelT* __restrict__ lab,
                                         const Ids& id) {
        const Start s = draw_start(p, id);
        lb = static_cast<uint32_t>(padded_index(p, s.lin)) * sizeof(LabelT);
        o[0] = unit_open_f(s.wox);
        o[1] = unit_open_f(s.woy);
        o[2] = unit_open_f(s.woz);
#pragma unroll
        for (int a = 0; a < 3; ++a) base[a] = -static_cast<double>(o[a]);
        l = l0 = entry(lab, lb);  // interior: no flags
        sig = p.sigma_f[l];
        dti2 = static_cast<float>(p.dt) * p.inv_t2_f[l];
        R = 0.0;
#pragma unroll
        for (int q = 0; q < kShapes; ++q)
#pragma unroll
            for (int a = 0; a < 3; ++a) ph[q][a] = 0.0;
        nface = nhit = nperm = 0;
    }

    __device__ __forceinline__ void step(const WalkPlan& p, const LabelT* __restrict__ lab,
                                         uint32_t i0, uint32_t wa, uint32_t wb, uint32_t m1,
                                         [[maybe_unused]] uint32_t t1,
                                         const Ids& id, const double2* trig) {
        // uniform deviates from the top 24 bits of each word: (k + 1/2) 2^-24
        const float u1 = fmaf(static_cast<float>(wa >> 8), 0x1p-24f, 0x1p-25f);
        const float u2 = fmaf(static_cast<float>(wb >> 8), 0x1p-24f, 0x1p-25f);
        const float cs = __builtin_amdgcn_cosf(u2);  // cos(2 pi u2)
        const float sn = __builtin_amdgcn_sinf(u2);  // sin(2 pi u2)
        // hardware square root (about 1 ulp): u1 (1 - u1) >= 2^-26, far from
        // the denormal range the library sqrtf guards against
        const float rho = 2.0f * __builtin_amdgcn_sqrtf(u1 * (1.0f - u1));
        const float v[3] = {rho * cs, rho * sn, fmaf(-2.0f, u1, 1.0f)};

        float g[3], m[3];
        uint32_t posm = 0, evm = 0;
        int sst[3];  // byte step in the padded volume across the face each axis moves toward
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool pos = v[a] > 0.0f;
            const int st = (a == 0 ? 1 : (a == 1 ? p.px : p.pxy)) * static_cast<int>(sizeof(LabelT));
            sst[a] = pos ? st : -st;
            posm |= pos ? (1u << a) : 0u;
            m[a] = fabsf(v[a]);
            g[a] = pos ? 1.0f - o[a] : o[a];  // o stays in [0, 1]
            evm |= g[a] < sig * m[a] ? (1u << a) : 0u;
        }
        int nev = __builtin_popcount(evm);
        int ax[3];
        event_order(g, m, ax);
        // Offsets and entries of the voxels the events reach if every face
        // passes (the common case), loaded together so the step waits for
        // memory once rather than once per event.
        const int nev0 = nev;
        uint32_t cpath[3], rsp[3];  // rsp[k] is set, and read, only for k < nev0
        {
            uint32_t c = lb;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                c += static_cast<uint32_t>(pick(sst, ax[k]));
                cpath[k] = c;
                if (k < nev0) rsp[k] = entry(lab, c);
            }
        }
        bool spec = true;  // every face so far passed: cpath and rsp hold the voxels reached

        // gap to axis a's face, and the path length to it (divided out only
        // after a permeation)
        const auto face_gap = [&](int a) {
            const float va = pick(v, a), oa = pick(o, a);
            return va > 0.0f ? 1.0f - oa : oa;
        };
        const auto face_len = [&](int a) { return face_gap(a) / fabsf(pick(v, a)); };
        float P = 0.0f, tau = 1.0f;
        uint32_t done = 0, refl = 0;  // axes whose face the step reached; those it reflected at
        uint32_t rawc = 0;  // entry of the voxel last passed into (its halo flags)
        int mw_used = 0;
        uint4 mw;  // words of substream 3, computed before the second membrane hit reads them
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k < nev) {
                const int a = ax[k];
                done |= 1u << a;
                uint32_t nbk, raw;
                if (spec && k < nev0) {
                    nbk = cpath[k];
                    raw = rsp[k];
                } else {  // after a reflection, or a face a permeation brought in
                    nbk = lb + static_cast<uint32_t>(pick(sst, a));
                    raw = entry(lab, nbk);
                }
                const int nl = static_cast<int>(raw & LabelBits<LabelT>::kMask);
                bool cross = true;
                if (nl != l) {
                    ++nhit;
                    [[maybe_unused]] uint64_t tp = 0u;
                    [[maybe_unused]] uint32_t tm = 0u;
                    if constexpr (MT) {  // both thresholds in one memory round trip
                        tp = threshold(p, l, nl);
                        tm = threshold_mt(p, l, nl);
                    }
                    if (mw_used == 1) mw = rare_block(i0, id);
                    if constexpr (MT) {
                        const uint32_t u = mw_used == 0 ? t1 : (mw_used == 1 ? mw.z : mw.w);
                        if (u < tm) R = INFINITY;  // saturated: weight 0 from here on
                    }
                    const uint32_t word = mw_used == 0 ? m1 : (mw_used == 1 ? mw.x : mw.y);
                    ++mw_used;
                    if constexpr (MT) cross = word < tp;
                    else cross = word < threshold(p, l, nl);
                    if (cross) {
                        ++nperm;
                        const float ek = fmaxf(face_len(a), P);
                        const float dtau = fminf((ek - P) / sig, tau);
                        R += static_cast<double>(dtau * dti2);
                        tau -= dtau;
                        P = ek;
                        l = nl;
                        sig = p.sigma_f[nl];
                        dti2 = static_cast<float>(p.dt) * p.inv_t2_f[nl];
                        // the later faces, in order, that lie inside the new budget:
                        // face_len < pend compared as gap < pend |v| (no division)
                        const float pend = fmaf(tau, sig, P);
                        nev = k + 1;
#pragma unroll
                        for (int j = k + 1; j < 3; ++j)
                            if (nev == j && face_gap(ax[j]) < pend * fabsf(pick(v, ax[j])))
                                nev = j + 1;
                    }
                }
                if (cross) {
                    lb = nbk;
                    rawc = raw;
                } else {
                    refl |= 1u << a;
                    spec = false;
                }
            }
        }
        const uint32_t passed = done & ~refl;
        nface += __builtin_popcount(done);
        const uint32_t halo = rawc >> LabelBits<LabelT>::kShift;
        if (__builtin_expect(halo != 0u, 0))
            lb = wrap_halo(p, lb, halo, posm, static_cast<int>(sizeof(LabelT)));
        const float lend = fmaf(tau, sig, P);
        R += static_cast<double>(tau * dti2);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool pos = (posm >> a) & 1u;
            const float fr = fmaf(lend, v[a], o[a]);
            const float t = select_bits(bit_mask(refl, a), (pos ? 2.0f : 0.0f) - fr, fr);
            // +-1 after a pass, else 0 (the and as a three-input operation,
            // truth table 0xC0, as in select_bits)
            const uint32_t one = pos ? 0x3F800000u : 0xBF800000u;
            const float shift =
                __uint_as_float(__builtin_amdgcn_bitop3_b32(bit_mask(passed, a), one, 0u, 0xC0));
            o[a] = fminf(fmaxf(t - shift, 0.0f), 1.0f);
            base[a] += static_cast<double>(shift);  // exact: whole voxels
        }
        // displacement base + o = n + o - o0 (one rounding at most, far below
        // the fp32 offset's own resolution); a zero gradient sample adds
        // exactly nothing, so no test for it
        double dsp[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) dsp[a] = base[a] + static_cast<double>(o[a]);
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const double g = p.gdt[static_cast<int64_t>(q) * p.n_steps + i0];
#pragma unroll
            for (int a = 0; a < 3; ++a) ph[q][a] = fma(g, dsp[a], ph[q][a]);
        }
    }

    __device__ __forceinline__ void finish(const WalkPlan& p, double* out) const {
        const Coords k = volume_coords(p, static_cast<int>(lb / sizeof(LabelT)));
#pragma unroll
        for (int a = 0; a < 3; ++a) out[a] = (base[a] + static_cast<double>(o[a])) * p.voxel_um;
        out[3] = R;
        out[4] = l;
        out[5] = k.c[0];
        out[6] = k.c[1];
        out[7] = k.c[2];
        out[8] = o[0];
        out[9] = o[1];
        out[10] = o[2];
        out[11] = l0;
        out[12] = nface;
        out[13] = nhit;
        out[14] = nperm;
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                out[15 + 3 * q + a] =
                    ph[q][a] * p.voxel_um;
    }
};

template <typename LabelT, int NS>
using WalkerMixed = WalkerMixedT<LabelT, NS, false>;
template <typename LabelT, int NS>
using WalkerMixedMT = WalkerMixedT<LabelT, NS, true>;

// Steps [b, e) of one walker, two steps (one direction block) per iteration,
// each taking its direction words from fixed fields of the block (a range
// that starts or ends inside a pair skips the step outside it under a
// wave-uniform test); the first-membrane block (four steps) is computed by
// the iterations that open one and by the first.  A scheduling barrier
// between the steps keeps them from being interleaved, which would raise
// register use.  kAnyStart false: b is a multiple of 4 (step 0, a segment of
// the persistent walk or a server slice); true: any b (a walk resumed after a
// record step).
template <bool kAnyStart = false, class Walker, typename LabelT>
__device__ __forceinline__ void walk_range(const WalkPlan& p, const LabelT* __restrict__ lab,
                                           Walker& W, uint32_t b, uint32_t e, const Ids& id,
                                           const double2* trig) {
    const auto block = [&](uint32_t index, uint32_t substream) {
        if constexpr (Walker::kUniformCounters)
            return philox4x32_10_uniform(index, substream, id.wlo, id.k0, id.k1);
        else
            return philox4x32_10(index, substream, id.wlo, id.whi, id.k0, id.k1);
    };
    uint4 wm = make_uint4(0, 0, 0, 0);
    [[maybe_unused]] uint4 wt = make_uint4(0, 0, 0, 0);  // saturation words (MT only)
    const uint32_t first = b & ~1u;
    for (uint32_t q0 = first; q0 < e; q0 += 2) {
        if ((q0 & 3u) == 0 || q0 == first) {
            wm = block(q0 >> 2, 1u);
            if constexpr (Walker::kMT) wt = block(q0 >> 2, 4u);
        }
        const bool hi = (q0 & 2u) != 0;  // the membrane block's third and fourth steps
        const uint4 wd = block(q0 >> 1, 0u);
        if (!kAnyStart || q0 >= b)
            W.step(p, lab, q0, wd.x, wd.y, hi ? wm.z : wm.x, hi ? wt.z : wt.x, id, trig);
        __builtin_amdgcn_sched_barrier(0);
        if (q0 + 1 < e)
            W.step(p, lab, q0 + 1, wd.z, wd.w, hi ? wm.w : wm.y, hi ? wt.w : wt.y, id, trig);
        __builtin_amdgcn_sched_barrier(0);
    }
}

}  // namespace dev
}  // namespace rms
