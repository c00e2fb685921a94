/*
 * rms_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of the Monte Carlo
 * random walk of the Realistic Microstructure Simulator (Lee, Fieremans &
 * Novikov, "RMS: Monte Carlo simulations of diffusion in three-dimensional
 * cell segmentations of microscopy images", arXiv 2012.06478).  It exists to
 * check the GPU library against: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.  The product library never links,
 * loads or calls anything in this directory, and this file includes nothing
 * from the product library.
 *
 * Every function names the passage of the paper it follows.  Where the paper
 * is silent the reading taken is stated in place:
 *   - the counter-based generator is Philox4x32-10 (Salmon, Moraes, Dror &
 *     Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), keyed by the
 *     64-bit seed, with counter words (index, substream, walker_lo, walker_hi):
 *       substream 0: step directions; block j feeds steps 2j+1 (words 0,1) and
 *                    2j+2 (words 2,3);
 *       substream 1: the first membrane decision of step i uses word (i-1) mod 4
 *                    of block (i-1)/4;
 *       substream 3: the second and third membrane decisions of step i (rare:
 *                    two or three membranes met in one step) use words 0 and 1
 *                    of block i-1;
 *       substream 2: the walker's start, blocks 0 and 1;
 *       saturation at absorbing membranes: the first membrane met in step i
 *                    uses word (i-1) mod 4 of substream 4 block (i-1)/4, the
 *                    second and third words 2 and 3 of substream 3 block i-1;
 *   - a word w maps to the uniform deviate (w + 1/2) 2^-32, exact in FP64;
 *   - the volume is periodic; displacements are unwrapped;
 *   - after a permeation into a compartment of different diffusivity the
 *     remaining fraction of the step's duration is kept, so the remaining
 *     length scales with that compartment's step length;
 *   - the phase is the right Riemann sum dt * sum_i g_i . (x_i - x_0) over the
 *     post-step positions, with the waveform scaled so that its discrete b
 *     value equals the requested one;
 *   - kurtosis uses moments weighted by alpha and divided by sum(alpha);
 *   - moments recorded at an earlier step t (D(t) and K(t), section 2.3) weight
 *     each walker by alpha(t) = exp(-R(t)), the T2 integral up to that step;
 *   - unequal spin concentrations c (App. C, general case): walkers start
 *     with density proportional to c (a uniform voxel draw accepted with
 *     probability c / max c, attempt j using substream 2 blocks 2j and 2j+1,
 *     word 1 of the second deciding, at most 65536 attempts); a membrane's
 *     "side 1" is its label of lower index when the exponent lambda is fixed,
 *     and a negative lambda takes the value that minimises the correction;
 *     Baxter's alternative permeation, when chosen, applies to the membranes
 *     with kappa > 0 (kappa's value is then unused);
 *   - an absorbing membrane (magnetization transfer, end of section 2.1.3)
 *     saturates a walker that meets it with probability P_MT, decided at the
 *     face with a word of its own, independent of the permeation word; the
 *     saturated walker keeps walking with weight 0 (Eq. wt-mt), held as
 *     R = infinity so that alpha = exp(-R) = 0.
 *
 * All arithmetic is IEEE double; build with -ffp-contract=off.
 */
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RMSO_OK 0
#define RMSO_E_INVALID_ARG (-1)
#define RMSO_E_LABEL_RANGE (-2)
#define RMSO_E_STEP_TOO_LARGE (-3)
#define RMSO_E_BAD_B (-4)
#define RMSO_E_OOM (-6)
#define RMSO_E_CORNER (-9) /* more than three face events in one step */

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11, section 3.3 and its reference table).  */
/* ------------------------------------------------------------------------- */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void rmso_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

static void philox_block(uint64_t seed, uint32_t index, uint32_t substream, uint64_t walker,
                         uint32_t out[4]) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint32_t ctr[4] = {index, substream, (uint32_t)walker, (uint32_t)(walker >> 32)};
    rmso_philox4x32_10(ctr, key, out);
}

double rmso_uniform(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* Step direction (section 2.2, item 2: constant length, random direction in
 * 3d).  Archimedes' mapping: the z component is uniform on (-1, 1) and the
 * azimuth uniform on (0, 2 pi), which is uniform on the unit sphere. */
void rmso_direction(uint32_t wa, uint32_t wb, double v[3]) {
    const double u1 = rmso_uniform(wa);
    const double u2 = rmso_uniform(wb);
    const double vz = 1.0 - 2.0 * u1;
    const double rho = 2.0 * sqrt(u1 * (1.0 - u1));
    const double phi = 2.0 * M_PI * u2;
    v[0] = rho * cos(phi);
    v[1] = rho * sin(phi);
    v[2] = vz;
}

/* ------------------------------------------------------------------------- */
/* Per-run tables (section 2.1.3).                                            */
/* ------------------------------------------------------------------------- */

/* Step size of Eq. (step-size), d = 3: ds = sqrt(2 d D0 dt). */
double rmso_step_size(double D, double dt) { return sqrt(2.0 * 3.0 * D * dt); }

/* Permeation probability from compartment 1 to 2, Eq. (perm-prob-general)
 * with C_3 = 2/3 (Eq. perm-prob), which already contains the correction of
 * the input permeability of Appendix C.1, Eqs. (kappa-correction) and
 * (kappa-factor-prob).  Clamped to 1 (the paper requires P << 1). */
double rmso_perm_prob(double kappa, double D1, double D2, double dt) {
    if (kappa <= 0.0) return 0.0;
    const double C3 = 2.0 / 3.0;
    const double ds1 = rmso_step_size(D1, dt);
    const double ds2 = rmso_step_size(D2, dt);
    const double num = kappa * ds1 / D1 * C3;
    const double den = 1.0 + 0.5 * kappa * (ds1 / D1 + ds2 / D2) * C3;
    const double P = num / den;
    return P > 1.0 ? 1.0 : P;
}

/* Permeation probabilities across one membrane between side 1 and side 2
 * with spin concentrations c1, c2 (App. C, general case and the alternative
 * approach).  model 0: Eq. (gen-perm-prob), P_1->2 = kappa0 ds1/D1 C_d
 * (c2/c1)^lambda and P_2->1 = kappa0 ds2/D2 C_d (c2/c1)^(lambda-1), with the
 * input permeability corrected by Eq. (gen-kappa-correction),
 * kappa = kappa0 / (1 - alpha_lambda), alpha_lambda the mean of the two
 * probabilities (Eq. gen-kappa-factor-prob); lambda < 0 takes the minimiser
 * of alpha_lambda, 1 / (1 + c2 sqrt(D2) / (c1 sqrt(D1))).  model 1:
 * Eq. (alt-perm-prob1-2), probability c_low sqrt(D_low) / (c_high sqrt(D_high))
 * from the side of larger c sqrt(D) and 1 from the other.  Both clamped to 1. */
void rmso_conc_perm_probs(double kappa, double D1, double D2, double c1, double c2,
                          double lambda, int model, double dt, double* P12, double* P21) {
    const double C3 = 2.0 / 3.0;
    *P12 = *P21 = 0.0;
    if (kappa <= 0.0) return;
    if (model == 1) {
        const double h1 = c1 * sqrt(D1), h2 = c2 * sqrt(D2);
        if (h1 >= h2) {
            *P12 = h2 / h1;
            *P21 = 1.0;
        } else {
            *P12 = 1.0;
            *P21 = h1 / h2;
        }
        return;
    }
    const double lam = lambda < 0.0 ? 1.0 / (1.0 + c2 * sqrt(D2) / (c1 * sqrt(D1))) : lambda;
    const double ds1 = rmso_step_size(D1, dt), ds2 = rmso_step_size(D2, dt);
    const double r = c2 / c1;
    const double A = 0.5 * (ds1 / D1 * pow(r, lam) + ds2 / D2 * pow(r, lam - 1.0)) * C3;
    const double k0 = kappa / (1.0 + kappa * A);
    const double p12 = k0 * ds1 / D1 * C3 * pow(r, lam);
    const double p21 = k0 * ds2 / D2 * C3 * pow(r, lam - 1.0);
    *P12 = p12 > 1.0 ? 1.0 : p12;
    *P21 = p21 > 1.0 ? 1.0 : p21;
}

/* Threshold of a probability: a word w < floor(P 2^32) passes. */
static uint64_t threshold_of(double P) {
    double t = floor(P * 4294967296.0);
    if (t > 4294967296.0) t = 4294967296.0;
    return (uint64_t)t;
}

/* Permeation thresholds with spin concentrations (rmso_conc_perm_probs for
 * each pair a < b of labels that are not dead, side 1 = a).  A probability of
 * 1 (Baxter's rule from the low-flux side) is the threshold 2^32, which every
 * 32-bit permeation word lies below. */
int rmso_conc_tables(int n_labels, const double* D, const double* kappa, const uint8_t* dead,
                     const double* conc, double lambda, int model, double dt, uint64_t* thresh) {
    if (model != 0 && model != 1) return RMSO_E_INVALID_ARG;
    if (model == 0 && lambda > 1.0) return RMSO_E_INVALID_ARG;
    for (int a = 0; a < n_labels; ++a)
        if (!(dead && dead[a]) && conc && (!(conc[a] > 0.0) || isinf(conc[a])))
            return RMSO_E_INVALID_ARG;
    for (int a = 0; a < n_labels; ++a)
        for (int b = a + 1; b < n_labels; ++b) {
            if (dead && (dead[a] || dead[b])) continue;
            const double k = kappa ? kappa[a * n_labels + b] : 0.0;
            double P12, P21;
            rmso_conc_perm_probs(k, D[a], D[b], conc ? conc[a] : 1.0, conc ? conc[b] : 1.0,
                                 lambda, model, dt, &P12, &P21);
            thresh[a * n_labels + b] = threshold_of(P12);
            thresh[b * n_labels + a] = threshold_of(P21);
        }
    return RMSO_OK;
}

/* Saturation probability at an absorbing membrane (end of section 2.1.3):
 * P_MT = rho ds C_3 / D0 with rho the surface relaxivity, ds and D0 of the
 * walker's compartment and C_3 = 2/3 as in Eq. (perm-prob).  Clamped to 1. */
double rmso_mt_prob(double rho, double D, double dt) {
    if (rho <= 0.0) return 0.0;
    const double C3 = 2.0 / 3.0;
    const double P = rho * rmso_step_size(D, dt) / D * C3;
    return P > 1.0 ? 1.0 : P;
}

/* Saturation thresholds for a walker in label a meeting a face to label b,
 * rho[a * n_labels + b] (a saturation word w < T saturates; T = floor(P 2^32);
 * 0 on equal labels, which are no membrane). */
int rmso_mt_tables(int n_labels, const double* D, const double* rho, const uint8_t* dead,
                   double dt, uint64_t* thresh_mt) {
    if (n_labels <= 0 || !rho || !(dt > 0.0)) return RMSO_E_INVALID_ARG;
    for (int a = 0; a < n_labels; ++a)
        for (int b = 0; b < n_labels; ++b) {
            const double r = rho[a * n_labels + b];
            if (!(r >= 0.0) || isinf(r)) return RMSO_E_INVALID_ARG;
            double P = 0.0;
            if (a != b && !(dead && dead[a])) P = rmso_mt_prob(r, D[a], dt);
            double t = floor(P * 4294967296.0);
            if (t > 4294967296.0) t = 4294967296.0;
            thresh_mt[a * n_labels + b] = (uint64_t)t;
        }
    return RMSO_OK;
}

/* Tables for one run: step length per label in voxel units, the 33-bit
 * permeation thresholds (a membrane word w < T permeates; T = floor(P 2^32)),
 * and 1/T2 per label (T2 = inf gives 0), section 2.1.4 Eq. (wt-relax).
 * A face between equal labels is transparent (section 2.2, item 3); a dead
 * label is never entered (section 2.2, item 1). */
int rmso_tables(int n_labels, const double* D, const double* kappa, const double* T2,
                const uint8_t* dead, double dt, double voxel_um, double* sigma,
                uint64_t* thresh, double* inv_T2) {
    if (n_labels <= 0 || !(dt > 0.0) || !(voxel_um > 0.0)) return RMSO_E_INVALID_ARG;
    double smax = 0.0;
    for (int l = 0; l < n_labels; ++l) {
        const int is_dead = dead && dead[l];
        if (!is_dead && !(D[l] > 0.0)) return RMSO_E_INVALID_ARG;
        sigma[l] = is_dead ? 0.0 : rmso_step_size(D[l], dt) / voxel_um;
        if (sigma[l] > smax) smax = sigma[l];
        if (T2) {
            if (!(T2[l] > 0.0)) return RMSO_E_INVALID_ARG;
            inv_T2[l] = isinf(T2[l]) ? 0.0 : 1.0 / T2[l];
        } else {
            inv_T2[l] = 0.0;
        }
    }
    /* At most three face interactions per step only if ds < voxel size
     * (section 2.1.1). */
    if (!(smax < 1.0)) return RMSO_E_STEP_TOO_LARGE;
    for (int a = 0; a < n_labels; ++a) {
        for (int b = 0; b < n_labels; ++b) {
            double P;
            if (a == b) P = 1.0;
            else if ((dead && (dead[a] || dead[b]))) P = 0.0;
            else P = rmso_perm_prob(kappa ? kappa[a * n_labels + b] : 0.0, D[a], D[b], dt);
            double t = floor(P * 4294967296.0);
            if (t > 4294967296.0) t = 4294967296.0;
            thresh[a * n_labels + b] = (uint64_t)t;
        }
    }
    return RMSO_OK;
}

/* Scale of each waveform shape so that its discrete b value equals the
 * requested b (section 2.3, Eq. signal).  With Q_k = dt sum_{i>=k} G_i the
 * phase is sum_k Q_k g . dx_k, so b_s = dt sum_k Q_k^2 for a unit shape. */
int rmso_bscale(int n_shapes, int64_t n_steps, double dt, const double* waveform, int n_b,
                const double* bvals, double* b_disc, double* kscale) {
    for (int s = 0; s < n_shapes; ++s) {
        const double* G = waveform + (size_t)s * (size_t)n_steps;
        double Q = 0.0, acc = 0.0;
        for (int64_t k = n_steps - 1; k >= 0; --k) {
            Q += dt * G[k];
            acc += Q * Q;
        }
        b_disc[s] = dt * acc;
        for (int j = 0; j < n_b; ++j) {
            if (bvals[j] < 0.0) return RMSO_E_BAD_B;
            if (bvals[j] == 0.0) kscale[s * n_b + j] = 0.0;
            else if (b_disc[s] > 0.0) kscale[s * n_b + j] = sqrt(bvals[j] / b_disc[s]);
            else return RMSO_E_BAD_B;
        }
    }
    return RMSO_OK;
}

/* ------------------------------------------------------------------------- */
/* The walk.                                                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    const void* labels;
    int label_bytes;
    int64_t dims[3];
    int n_labels;
    double voxel_um;
    double dt;
    const double* sigma;
    const uint64_t* thresh;
    const double* inv_T2;
    const uint64_t* thresh_mt; /* saturation thresholds, or NULL: no absorbing membranes */
} rmso_geom;

typedef struct {
    int64_t vox[3];
    double off[3]; /* in [0, 1], voxel units */
    int label;
    double dx[3];  /* unwrapped displacement, micrometres */
    double R;      /* sum_c t_c / T2_c */
    int64_t n_face, n_hit, n_perm;
} rmso_walker;

static int label_at(const rmso_geom* g, const int64_t v[3]) {
    const int64_t idx = v[0] + g->dims[0] * (v[1] + g->dims[1] * v[2]);
    if (g->label_bytes == 1) return ((const uint8_t*)g->labels)[idx];
    return ((const uint16_t*)g->labels)[idx];
}

static double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

/* One step of one walker (section 2.2, items 2-4; section 2.1.1 and the
 * corner-reflector figure; section 2.1.2-2.1.3).  v is the unit direction,
 * mw are the step's membrane words (the caller supplies them lazily through
 * get_mw: index k < 3 is the permeation word of the k-th membrane met, 16 + k
 * its saturation word).  The walker travels along v; each time the remaining path reaches
 * a voxel face it either passes (same label on the other side), permeates
 * with probability P (different label), or is reflected specularly
 * (component normal to the face flips).  Returns the number of face events or
 * RMSO_E_CORNER if a fourth one would be needed. */
typedef uint32_t (*mw_source)(void* ctx, int index);

static int walk_step(const rmso_geom* g, rmso_walker* w, const double v_in[3], mw_source get_mw,
                     void* mw_ctx) {
    double v[3] = {v_in[0], v_in[1], v_in[2]};
    double tau = 1.0; /* fraction of the step duration still to travel */
    int events = 0, mw_used = 0;
    for (;;) {
        const double sig = g->sigma[w->label];
        const double lam = tau * sig; /* remaining path length, voxel units */
        int axis = -1;
        double dmin = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (v[a] == 0.0) continue;
            double gap = v[a] > 0.0 ? 1.0 - w->off[a] : w->off[a];
            if (gap < 0.0) gap = 0.0;
            const double d = gap / fabs(v[a]);
            if (d < lam && (axis < 0 || d < dmin)) {
                axis = a;
                dmin = d;
            }
        }
        if (axis < 0) {
            for (int a = 0; a < 3; ++a) {
                w->off[a] = clamp01(w->off[a] + lam * v[a]);
                w->dx[a] += lam * v[a] * g->voxel_um;
            }
            w->R += tau * g->dt * g->inv_T2[w->label];
            return events;
        }
        if (events == 3) return RMSO_E_CORNER;
        ++events;
        /* move to the face */
        for (int a = 0; a < 3; ++a) {
            w->dx[a] += dmin * v[a] * g->voxel_um;
            if (a == axis) w->off[a] = v[a] > 0.0 ? 1.0 : 0.0;
            else w->off[a] = clamp01(w->off[a] + dmin * v[a]);
        }
        double dtau = dmin / sig;
        if (dtau > tau) dtau = tau;
        w->R += dtau * g->dt * g->inv_T2[w->label];
        tau -= dtau;
        ++w->n_face;
        int64_t nb[3] = {w->vox[0], w->vox[1], w->vox[2]};
        nb[axis] += v[axis] > 0.0 ? 1 : -1;
        if (nb[axis] < 0) nb[axis] += g->dims[axis];
        if (nb[axis] >= g->dims[axis]) nb[axis] -= g->dims[axis];
        const int nl = label_at(g, nb);
        int cross;
        if (nl == w->label) {
            cross = 1;
        } else {
            ++w->n_hit;
            if (g->thresh_mt) {
                const uint64_t tm = g->thresh_mt[w->label * g->n_labels + nl];
                if (tm > 0 && (uint64_t)get_mw(mw_ctx, 16 + mw_used) < tm) w->R = INFINITY;
            }
            const uint32_t m = get_mw(mw_ctx, mw_used++);
            cross = (uint64_t)m < g->thresh[w->label * g->n_labels + nl];
            if (cross) ++w->n_perm;
        }
        if (cross) {
            w->vox[0] = nb[0];
            w->vox[1] = nb[1];
            w->vox[2] = nb[2];
            w->off[axis] = v[axis] > 0.0 ? 0.0 : 1.0;
            w->label = nl;
        } else {
            v[axis] = -v[axis];
        }
    }
}

/* Membrane words of step i (index = i - 1): the first from substream 1, the
 * second and third from substream 3. */
typedef struct {
    uint64_t seed, walker;
    uint32_t index;
} philox_mw_ctx;

static uint32_t philox_mw(void* p, int k) {
    const philox_mw_ctx* c = (const philox_mw_ctx*)p;
    uint32_t w[4];
    if (k == 16) {
        philox_block(c->seed, c->index / 4u, 4u, c->walker, w);
        return w[c->index % 4u];
    }
    if (k > 16) {
        philox_block(c->seed, c->index, 3u, c->walker, w);
        return w[k - 15];
    }
    if (k == 0) {
        philox_block(c->seed, c->index / 4u, 1u, c->walker, w);
        return w[c->index % 4u];
    }
    philox_block(c->seed, c->index, 3u, c->walker, w);
    return w[k - 1];
}

/* Words handed in by a unit test. */
typedef struct {
    const uint32_t* words;
} fixed_mw_ctx;

static uint32_t fixed_mw(void* p, int k) { return ((fixed_mw_ctx*)p)->words[k]; }

/* A single step from a hand-placed state, for unit tests of the face walk. */
int rmso_single_step(const void* labels, int label_bytes, const int64_t dims[3], int n_labels,
                     double voxel_um, double dt, const double* sigma, const uint64_t* thresh,
                     const double* inv_T2, int64_t vox[3], double off[3], int* label,
                     const double v[3], const uint32_t mwords[3], double dx[3], double* R,
                     int64_t counts[3]) {
    rmso_geom g = {labels, label_bytes, {dims[0], dims[1], dims[2]}, n_labels, voxel_um, dt,
                   sigma, thresh, inv_T2};
    rmso_walker w;
    memset(&w, 0, sizeof w);
    for (int a = 0; a < 3; ++a) {
        w.vox[a] = vox[a];
        w.off[a] = off[a];
    }
    w.label = *label;
    fixed_mw_ctx mc = {mwords};
    const int r = walk_step(&g, &w, v, fixed_mw, &mc);
    for (int a = 0; a < 3; ++a) {
        vox[a] = w.vox[a];
        off[a] = w.off[a];
        dx[a] = w.dx[a];
    }
    *label = w.label;
    *R = w.R;
    counts[0] = w.n_face;
    counts[1] = w.n_hit;
    counts[2] = w.n_perm;
    return r;
}

/* ------------------------------------------------------------------------- */
/* Whole run.                                                                 */
/* ------------------------------------------------------------------------- */
typedef struct {
    rmso_geom g;
    uint64_t seed;
    int64_t n_walkers;
    const int64_t* walker_ids;
    int64_t n_steps;
    int n_shapes;
    const double* waveform;
    const int64_t* allowed; /* NULL: every voxel allowed */
    int64_t n_allowed;
    const uint64_t* accept; /* start acceptance threshold per label, or NULL: uniform start */
    /* per-walker results */
    double* w_dx;   /* [n][3] */
    double* w_phi;  /* [n][3*n_shapes] */
    double* w_R;    /* [n] */
    int64_t* w_cnt; /* [n][3] */
    int32_t* w_lab; /* [n][2] start, end label */
    int64_t* w_vox; /* [n][3] final voxel */
    double* w_off;  /* [n][3] final offset */
    int n_rec;               /* record steps (ascending, 1..n_steps) */
    const int64_t* rec_steps;
    double* w_rec;           /* [n][n_rec][4] displacement (um) and R after each record step */
    atomic_llong next;
    atomic_int err;
} run_ctx;

static void walk_one(run_ctx* c, int64_t slot) {
    const uint64_t wid = (uint64_t)(c->walker_ids ? c->walker_ids[slot] : slot);
    rmso_walker w;
    memset(&w, 0, sizeof w);
    /* Start (section 2.2, item 1): uniform over the voxels that are not dead,
     * then uniform inside the voxel. */
    uint32_t b0[4], b1[4];
    int64_t lin = 0;
    for (uint32_t j = 0;; ++j) {
        philox_block(c->seed, 2u * j, 2u, wid, b0);
        philox_block(c->seed, 2u * j + 1u, 2u, wid, b1);
        const uint64_t r64 = ((uint64_t)b0[1] << 32) | b0[0];
        const int64_t rank =
            (int64_t)(((unsigned __int128)r64 * (unsigned __int128)c->n_allowed) >> 64);
        lin = c->allowed ? c->allowed[rank] : rank;
        if (!c->accept || j + 1 == 65536u) break;
        const int64_t vv[3] = {lin % c->g.dims[0], (lin / c->g.dims[0]) % c->g.dims[1],
                               lin / (c->g.dims[0] * c->g.dims[1])};
        if ((uint64_t)b1[1] < c->accept[label_at(&c->g, vv)]) break;
    }
    w.vox[0] = lin % c->g.dims[0];
    w.vox[1] = (lin / c->g.dims[0]) % c->g.dims[1];
    w.vox[2] = lin / (c->g.dims[0] * c->g.dims[1]);
    w.off[0] = rmso_uniform(b0[2]);
    w.off[1] = rmso_uniform(b0[3]);
    w.off[2] = rmso_uniform(b1[0]);
    w.label = label_at(&c->g, w.vox);
    const int start_label = w.label;

    double phi[3 * 8];
    memset(phi, 0, sizeof phi);
    uint32_t dirw[4];
    int rec = 0; /* next record */
    for (int64_t i = 1; i <= c->n_steps; ++i) {
        const int64_t j = (i - 1) / 2;
        if (((i - 1) & 1) == 0) philox_block(c->seed, (uint32_t)j, 0u, wid, dirw);
        const int h = (int)((i - 1) & 1);
        double v[3];
        rmso_direction(dirw[2 * h], dirw[2 * h + 1], v);
        philox_mw_ctx mc = {c->seed, wid, (uint32_t)(i - 1)};
        const int r = walk_step(&c->g, &w, v, philox_mw, &mc);
        if (r < 0) {
            atomic_store(&c->err, r);
            return;
        }
        /* phase (section 2.3, Eq. signal): right Riemann sum of g . (x - x0) */
        for (int s = 0; s < c->n_shapes; ++s) {
            const double G = c->waveform[(size_t)s * (size_t)c->n_steps + (size_t)(i - 1)];
            for (int a = 0; a < 3; ++a) phi[3 * s + a] += c->g.dt * G * w.dx[a];
        }
        if (rec < c->n_rec && c->rec_steps[rec] == i) {
            double* o = c->w_rec + ((size_t)slot * (size_t)c->n_rec + (size_t)rec) * 4;
            for (int a = 0; a < 3; ++a) o[a] = w.dx[a];
            o[3] = w.R;
            ++rec;
        }
    }
    for (int a = 0; a < 3; ++a) {
        c->w_dx[3 * slot + a] = w.dx[a];
        c->w_vox[3 * slot + a] = w.vox[a];
        c->w_off[3 * slot + a] = w.off[a];
    }
    for (int s = 0; s < 3 * c->n_shapes; ++s) c->w_phi[(size_t)slot * 3 * c->n_shapes + s] = phi[s];
    c->w_R[slot] = w.R;
    c->w_cnt[3 * slot + 0] = w.n_face;
    c->w_cnt[3 * slot + 1] = w.n_hit;
    c->w_cnt[3 * slot + 2] = w.n_perm;
    c->w_lab[2 * slot + 0] = start_label;
    c->w_lab[2 * slot + 1] = w.label;
}

static void* worker(void* p) {
    run_ctx* c = (run_ctx*)p;
    for (;;) {
        const long long b = atomic_fetch_add(&c->next, 16);
        if (b >= c->n_walkers || atomic_load(&c->err)) break;
        const long long e = b + 16 < c->n_walkers ? b + 16 : c->n_walkers;
        for (long long s = b; s < e; ++s) walk_one(c, s);
    }
    return NULL;
}

/* Signal and moments (section 2.3): S = <alpha e^{-i phi}> / <alpha>,
 * D = <alpha (dx.g)^2> / (2 t <alpha>), K = <alpha (dx.g)^4> <alpha> /
 * <alpha (dx.g)^2>^2 - 3, with alpha = exp(-R) (section 2.1.4).
 *
 * walker_dump (optional) receives per walker, in order:
 *   dx[3] (um), R, end label, end voxel[3], end offset[3], start label,
 *   face events, membrane hits, permeations, phase[3*n_shapes]
 * (15 + 3 n_shapes doubles). */
int rmso_run(const void* labels, int label_bytes, const int64_t dims[3], double voxel_um,
             int n_labels, const double* D, const double* kappa, const double* T2,
             const uint8_t* dead, uint64_t seed, int64_t n_walkers, const int64_t* walker_ids,
             int64_t n_steps, double dt, int n_shapes, const double* waveform, int n_dirs,
             const double* dirs, int n_b, const double* bvals, int n_threads, double* signal,
             double* m2, double* m4, double* D_dir, double* K_dir, double* sum_alpha,
             double* b_disc, int64_t counters[3], double* walker_dump, int n_rec,
             const int64_t* rec_steps, double* rec_out, const double* rho, const double* conc,
             double lambda, int perm_model) {
    if (!labels || (label_bytes != 1 && label_bytes != 2) || !dims || n_walkers < 0 ||
        n_steps < 0 || n_steps > 0xFFFFFFFFLL || n_shapes < 0 || n_shapes > 8 || n_dirs < 0 ||
        n_b < 0 || (n_shapes > 0 && !waveform) || (n_dirs > 0 && !dirs) || n_rec < 0 ||
        (n_rec > 0 && (!rec_steps || !rec_out)))
        return RMSO_E_INVALID_ARG;
    for (int r = 0; r < n_rec; ++r)
        if (rec_steps[r] < 1 || rec_steps[r] > n_steps || (r > 0 && rec_steps[r] <= rec_steps[r - 1]))
            return RMSO_E_INVALID_ARG;
    const int64_t nvox = dims[0] * dims[1] * dims[2];
    if (dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0) return RMSO_E_INVALID_ARG;
    for (int64_t i = 0; i < nvox; ++i) {
        const int l = label_bytes == 1 ? ((const uint8_t*)labels)[i] : ((const uint16_t*)labels)[i];
        if (l >= n_labels) return RMSO_E_LABEL_RANGE;
    }
    double* sigma = malloc(sizeof(double) * n_labels);
    double* inv_T2 = malloc(sizeof(double) * n_labels);
    uint64_t* thresh = malloc(sizeof(uint64_t) * (size_t)n_labels * n_labels);
    double* kscale = malloc(sizeof(double) * (size_t)(n_shapes * n_b + 1));
    double* bd = malloc(sizeof(double) * (size_t)(n_shapes + 1));
    int rc = (sigma && inv_T2 && thresh && kscale && bd) ? RMSO_OK : RMSO_E_OOM;
    if (rc == RMSO_OK)
        rc = rmso_tables(n_labels, D, kappa, T2, dead, dt, voxel_um, sigma, thresh, inv_T2);
    if (rc == RMSO_OK && (conc || perm_model != 0))
        rc = rmso_conc_tables(n_labels, D, kappa, dead, conc, lambda, perm_model, dt, thresh);
    uint64_t* thresh_mt = NULL;
    if (rc == RMSO_OK && rho) {
        thresh_mt = malloc(sizeof(uint64_t) * (size_t)n_labels * n_labels);
        rc = thresh_mt ? rmso_mt_tables(n_labels, D, rho, dead, dt, thresh_mt) : RMSO_E_OOM;
    }
    if (rc == RMSO_OK) rc = rmso_bscale(n_shapes, n_steps, dt, waveform, n_b, bvals, bd, kscale);

    int64_t* allowed = NULL;
    int64_t n_allowed = nvox;
    if (rc == RMSO_OK && dead) {
        int any = 0;
        for (int l = 0; l < n_labels; ++l) any |= dead[l] != 0;
        if (any) {
            allowed = malloc(sizeof(int64_t) * (size_t)nvox);
            if (!allowed) rc = RMSO_E_OOM;
            n_allowed = 0;
            for (int64_t i = 0; rc == RMSO_OK && i < nvox; ++i) {
                const int l =
                    label_bytes == 1 ? ((const uint8_t*)labels)[i] : ((const uint16_t*)labels)[i];
                if (!dead[l]) allowed[n_allowed++] = i;
            }
            if (rc == RMSO_OK && n_allowed == 0) rc = RMSO_E_INVALID_ARG;
        }
    }
    /* start density proportional to the spin concentration: a uniform draw
     * over the allowed voxels is accepted with probability c / max c; the
     * mean acceptance must be at least 1e-3 */
    uint64_t* accept = NULL;
    if (rc == RMSO_OK && conc) {
        double cmax = 0.0, csum = 0.0;
        for (int l = 0; l < n_labels; ++l)
            if (!(dead && dead[l]) && conc[l] > cmax) cmax = conc[l];
        for (int64_t i = 0; i < nvox; ++i) {
            const int l = label_bytes == 1 ? ((const uint8_t*)labels)[i] : ((const uint16_t*)labels)[i];
            if (!(dead && dead[l])) csum += conc[l];
        }
        accept = malloc(sizeof(uint64_t) * (size_t)n_labels);
        if (!accept) rc = RMSO_E_OOM;
        else if (!(cmax > 0.0) || csum < 1e-3 * cmax * (double)n_allowed) rc = RMSO_E_INVALID_ARG;
        for (int l = 0; rc == RMSO_OK && l < n_labels; ++l)
            accept[l] = (dead && dead[l]) ? 0 : threshold_of(conc[l] / cmax);
    }
    run_ctx* c = calloc(1, sizeof(run_ctx));
    if (!c) rc = RMSO_E_OOM;
    const size_t n = (size_t)n_walkers;
    if (rc == RMSO_OK) {
        c->g = (rmso_geom){labels, label_bytes, {dims[0], dims[1], dims[2]}, n_labels, voxel_um,
                           dt, sigma, thresh, inv_T2, thresh_mt};
        c->seed = seed;
        c->n_walkers = n_walkers;
        c->walker_ids = walker_ids;
        c->n_steps = n_steps;
        c->n_shapes = n_shapes;
        c->waveform = waveform;
        c->allowed = allowed;
        c->n_allowed = n_allowed;
        c->accept = accept;
        c->w_dx = malloc(sizeof(double) * 3 * n + 8);
        c->w_phi = malloc(sizeof(double) * 3 * (size_t)n_shapes * n + 8);
        c->w_R = malloc(sizeof(double) * n + 8);
        c->w_cnt = malloc(sizeof(int64_t) * 3 * n + 8);
        c->w_lab = malloc(sizeof(int32_t) * 2 * n + 8);
        c->w_vox = malloc(sizeof(int64_t) * 3 * n + 8);
        c->w_off = malloc(sizeof(double) * 3 * n + 8);
        c->n_rec = n_rec;
        c->rec_steps = rec_steps;
        c->w_rec = malloc(sizeof(double) * 4 * (size_t)n_rec * n + 8);
        if (!c->w_dx || !c->w_phi || !c->w_R || !c->w_cnt || !c->w_lab || !c->w_vox || !c->w_off ||
            !c->w_rec)
            rc = RMSO_E_OOM;
    }
    if (rc == RMSO_OK) {
        atomic_init(&c->next, 0);
        atomic_init(&c->err, 0);
        if (n_threads < 1) n_threads = 1;
        pthread_t* th = malloc(sizeof(pthread_t) * (size_t)n_threads);
        int started = 0;
        for (int t = 0; th && t < n_threads; ++t)
            if (pthread_create(&th[t], NULL, worker, c) == 0) ++started;
        if (started == 0) worker(c);
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
        free(th);
        rc = atomic_load(&c->err);
    }
    if (rc == RMSO_OK) {
        /* Sums over walkers in ascending walker order. */
        const int n_sig = n_shapes * n_b * n_dirs;
        double* re = calloc((size_t)n_sig + 1, sizeof(double));
        double* im = calloc((size_t)n_sig + 1, sizeof(double));
        double* p2 = calloc((size_t)n_dirs + 1, sizeof(double));
        double* p4 = calloc((size_t)n_dirs + 1, sizeof(double));
        double* gh = malloc(sizeof(double) * 3 * ((size_t)n_dirs + 1));
        double sa = 0.0, s2[6] = {0}, s4[15] = {0};
        int64_t cnt[3] = {0, 0, 0};
        if (!re || !im || !p2 || !p4 || !gh) rc = RMSO_E_OOM;
        for (int d = 0; rc == RMSO_OK && d < n_dirs; ++d) {
            const double nrm = sqrt(dirs[3 * d] * dirs[3 * d] + dirs[3 * d + 1] * dirs[3 * d + 1] +
                                    dirs[3 * d + 2] * dirs[3 * d + 2]);
            if (!(nrm > 0.0)) rc = RMSO_E_INVALID_ARG;
            for (int a = 0; a < 3; ++a) gh[3 * d + a] = dirs[3 * d + a] / nrm;
        }
        for (size_t k = 0; rc == RMSO_OK && k < n; ++k) {
            const double alpha = exp(-c->w_R[k]);
            const double* x = c->w_dx + 3 * k;
            sa += alpha;
            for (int s = 0; s < n_shapes; ++s) {
                const double* ph = c->w_phi + (size_t)k * 3 * n_shapes + 3 * s;
                for (int j = 0; j < n_b; ++j) {
                    for (int d = 0; d < n_dirs; ++d) {
                        const double proj =
                            gh[3 * d] * ph[0] + gh[3 * d + 1] * ph[1] + gh[3 * d + 2] * ph[2];
                        const double p = kscale[s * n_b + j] * proj;
                        const int q = (s * n_b + j) * n_dirs + d;
                        re[q] += alpha * cos(p);
                        im[q] += -alpha * sin(p);
                    }
                }
            }
            int q = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = a; b < 3; ++b) s2[q++] += alpha * x[a] * x[b];
            q = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = a; b < 3; ++b)
                    for (int e = b; e < 3; ++e)
                        for (int f = e; f < 3; ++f) s4[q++] += alpha * x[a] * x[b] * x[e] * x[f];
            for (int d = 0; d < n_dirs; ++d) {
                const double pr = gh[3 * d] * x[0] + gh[3 * d + 1] * x[1] + gh[3 * d + 2] * x[2];
                p2[d] += alpha * pr * pr;
                p4[d] += alpha * pr * pr * pr * pr;
            }
            for (int t = 0; t < 3; ++t) cnt[t] += c->w_cnt[3 * k + t];
        }
        if (rc == RMSO_OK) {
            const double t = (double)n_steps * dt;
            for (int q = 0; q < n_sig; ++q) {
                if (signal) {
                    signal[2 * q] = re[q] / sa;
                    signal[2 * q + 1] = im[q] / sa;
                }
            }
            for (int q = 0; q < 6; ++q)
                if (m2) m2[q] = s2[q] / sa;
            for (int q = 0; q < 15; ++q)
                if (m4) m4[q] = s4[q] / sa;
            for (int d = 0; d < n_dirs; ++d) {
                const double w2 = p2[d] / sa, w4 = p4[d] / sa;
                if (D_dir) D_dir[d] = t > 0.0 ? w2 / (2.0 * t) : 0.0;
                if (K_dir) K_dir[d] = w2 > 0.0 ? w4 / (w2 * w2) - 3.0 : 0.0;
            }
            if (sum_alpha) *sum_alpha = sa;
            if (b_disc)
                for (int s = 0; s < n_shapes; ++s) b_disc[s] = bd[s];
            if (counters)
                for (int q = 0; q < 3; ++q) counters[q] = cnt[q];
            /* recorded moments, the same sums at each record step t: rec_out
             * per record holds sum alpha(t), M2[6], M4[15], D[n_dirs], K[n_dirs] */
            for (int r = 0; r < n_rec; ++r) {
                double* o = rec_out + (size_t)r * (22 + 2 * (size_t)n_dirs);
                double ra = 0.0, r2[6] = {0}, r4[15] = {0};
                for (int d = 0; d < n_dirs; ++d) p2[d] = p4[d] = 0.0;
                for (size_t k = 0; k < n; ++k) {
                    const double* x = c->w_rec + (k * (size_t)n_rec + (size_t)r) * 4;
                    const double alpha = exp(-x[3]);
                    ra += alpha;
                    int q = 0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = a; b < 3; ++b) r2[q++] += alpha * x[a] * x[b];
                    q = 0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = a; b < 3; ++b)
                            for (int e = b; e < 3; ++e)
                                for (int f = e; f < 3; ++f)
                                    r4[q++] += alpha * x[a] * x[b] * x[e] * x[f];
                    for (int d = 0; d < n_dirs; ++d) {
                        const double pr =
                            gh[3 * d] * x[0] + gh[3 * d + 1] * x[1] + gh[3 * d + 2] * x[2];
                        p2[d] += alpha * pr * pr;
                        p4[d] += alpha * pr * pr * pr * pr;
                    }
                }
                const double tr = (double)rec_steps[r] * dt;
                o[0] = ra;
                for (int q = 0; q < 6; ++q) o[1 + q] = r2[q] / ra;
                for (int q = 0; q < 15; ++q) o[7 + q] = r4[q] / ra;
                for (int d = 0; d < n_dirs; ++d) {
                    const double w2 = p2[d] / ra, w4 = p4[d] / ra;
                    o[22 + d] = w2 / (2.0 * tr);
                    o[22 + n_dirs + d] = w2 > 0.0 ? w4 / (w2 * w2) - 3.0 : 0.0;
                }
            }
            if (walker_dump) {
                const size_t K = 15 + 3 * (size_t)n_shapes;
                for (size_t k = 0; k < n; ++k) {
                    double* o = walker_dump + k * K;
                    for (int a = 0; a < 3; ++a) o[a] = c->w_dx[3 * k + a];
                    o[3] = c->w_R[k];
                    o[4] = c->w_lab[2 * k + 1];
                    for (int a = 0; a < 3; ++a) o[5 + a] = (double)c->w_vox[3 * k + a];
                    for (int a = 0; a < 3; ++a) o[8 + a] = c->w_off[3 * k + a];
                    o[11] = c->w_lab[2 * k + 0];
                    for (int a = 0; a < 3; ++a) o[12 + a] = (double)c->w_cnt[3 * k + a];
                    for (int s = 0; s < 3 * n_shapes; ++s)
                        o[15 + s] = c->w_phi[k * 3 * (size_t)n_shapes + s];
                }
            }
        }
        free(re);
        free(im);
        free(p2);
        free(p4);
        free(gh);
    }
    if (c) {
        free(c->w_dx);
        free(c->w_phi);
        free(c->w_R);
        free(c->w_cnt);
        free(c->w_lab);
        free(c->w_vox);
        free(c->w_off);
        free(c->w_rec);
        free(c);
    }
    free(allowed);
    free(accept);
    free(sigma);
    free(inv_T2);
    free(thresh);
    free(thresh_mt);
    free(kscale);
    free(bd);
    return rc;
}
