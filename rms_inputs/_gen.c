/*
 * _gen.c -- seeded generators of synthetic label volumes (inputs only; no
 * part of the walk).  Volumes are [nz][ny][nx] with x fastest, periodic.
 * The random stream is splitmix64 (Steele, Lea & Flood, OOPSLA 2014), so a
 * seed gives the same volume on every machine.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t s;
} rng_t;

static uint64_t next64(rng_t* r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double unif(rng_t* r) { return (double)(next64(r) >> 11) * 0x1p-53; }
static double normal(rng_t* r) {
    double u = unif(r), v = unif(r);
    if (u < 1e-300) u = 1e-300;
    return sqrt(-2.0 * log(u)) * cos(2.0 * M_PI * v);
}
static int64_t randint(rng_t* r, int64_t n) { return (int64_t)(unif(r) * (double)n); }
static int64_t wrap(int64_t i, int64_t n) {
    i %= n;
    return i < 0 ? i + n : i;
}

static void rotation(rng_t* r, double R[9]) {
    double q[4], n = 0.0;
    for (int i = 0; i < 4; ++i) {
        q[i] = normal(r);
        n += q[i] * q[i];
    }
    n = sqrt(n);
    const double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w); R[2] = 2 * (x * z + y * w);
    R[3] = 2 * (x * y + z * w); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
    R[6] = 2 * (x * z - y * w); R[7] = 2 * (y * z + x * w); R[8] = 1 - 2 * (x * x + y * y);
}

static const int NB[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                             {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

/* Random sequential addition of randomly oriented ellipsoids in an n^3
 * volume (labels 1..n_cells, background 0).  Cell c draws semi-axes uniform
 * in [lo, hi] um and a uniform rotation, then tries up to max_tries uniform
 * centres (voxel centres); a placement is accepted when none of its voxels is
 * taken or face-adjacent to an earlier cell.  After max_tries failures the
 * semi-axes shrink by `shrink`.  semi_out receives the final semi-axes.
 * Returns 0, or -1 when a cell cannot be placed at all. */
int gen_ellipsoids(int64_t n, double voxel_um, int n_cells, double lo, double hi,
                   uint64_t seed, int max_tries, double shrink, uint16_t* lab,
                   double* semi_out) {
    rng_t rng = {seed};
    const int64_t nv = n * n * n;
    uint8_t* blocked = calloc((size_t)nv, 1);
    if (!blocked) return -2;
    memset(lab, 0, sizeof(uint16_t) * (size_t)nv);
    int rc = 0;
    for (int c = 1; c <= n_cells && rc == 0; ++c) {
        double ax[3], R[9];
        for (int a = 0; a < 3; ++a) ax[a] = (lo + (hi - lo) * unif(&rng)) / voxel_um;
        rotation(&rng, R);
        for (;;) {
            const double amax = fmax(ax[0], fmax(ax[1], ax[2]));
            const int h = (int)ceil(amax) + 1;
            const int64_t side = 2 * h + 1;
            int32_t* off = malloc(sizeof(int32_t) * 3 * (size_t)(side * side * side));
            int64_t m = 0;
            for (int dz = -h; dz <= h; ++dz)
                for (int dy = -h; dy <= h; ++dy)
                    for (int dx = -h; dx <= h; ++dx) {
                        /* body frame coordinates: R^T p with p = (dx, dy, dz) */
                        const double bx = R[0] * dx + R[3] * dy + R[6] * dz;
                        const double by = R[1] * dx + R[4] * dy + R[7] * dz;
                        const double bz = R[2] * dx + R[5] * dy + R[8] * dz;
                        const double q = (bx / ax[0]) * (bx / ax[0]) +
                                         (by / ax[1]) * (by / ax[1]) +
                                         (bz / ax[2]) * (bz / ax[2]);
                        if (q <= 1.0) {
                            off[3 * m] = dx;
                            off[3 * m + 1] = dy;
                            off[3 * m + 2] = dz;
                            ++m;
                        }
                    }
            /* shuffle, so an overlapping candidate is usually rejected early */
            for (int64_t i = m - 1; i > 0; --i) {
                const int64_t j = randint(&rng, i + 1);
                for (int t = 0; t < 3; ++t) {
                    const int32_t s = off[3 * i + t];
                    off[3 * i + t] = off[3 * j + t];
                    off[3 * j + t] = s;
                }
            }
            int placed = 0;
            for (int t = 0; t < max_tries && !placed; ++t) {
                const int64_t cx = randint(&rng, n), cy = randint(&rng, n), cz = randint(&rng, n);
                int ok = 1;
                for (int64_t i = 0; i < m && ok; ++i) {
                    const int64_t x = wrap(cx + off[3 * i], n), y = wrap(cy + off[3 * i + 1], n),
                                  z = wrap(cz + off[3 * i + 2], n);
                    if (blocked[x + n * (y + n * z)]) ok = 0;
                }
                if (!ok) continue;
                for (int64_t i = 0; i < m; ++i) {
                    const int64_t x = wrap(cx + off[3 * i], n), y = wrap(cy + off[3 * i + 1], n),
                                  z = wrap(cz + off[3 * i + 2], n);
                    lab[x + n * (y + n * z)] = (uint16_t)c;
                    for (int k = 0; k < 7; ++k) {
                        const int64_t xx = wrap(x + NB[k][0], n), yy = wrap(y + NB[k][1], n),
                                      zz = wrap(z + NB[k][2], n);
                        blocked[xx + n * (yy + n * zz)] = 1;
                    }
                }
                placed = 1;
            }
            free(off);
            if (placed) {
                for (int a = 0; a < 3; ++a) semi_out[3 * (c - 1) + a] = ax[a] * voxel_um;
                break;
            }
            for (int a = 0; a < 3; ++a) ax[a] *= shrink;
            if (fmax(ax[0], fmax(ax[1], ax[2])) < 1.0) {
                rc = -1;
                break;
            }
        }
    }
    free(blocked);
    return rc;
}

/* A bundle of beaded, undulating tubes along z (labels 1..n_axons in label 0)
 * in an nx x ny x nz volume.  Tube a: base radius exp(N(mu, sigma)) um;
 * Gaussian beads (relative height bead_amp, width bead_w um) at Poisson-spaced
 * z with mean spacing bead_sp um; one undulation harmonic per transverse axis
 * with wavelength uniform in [lam_lo, lam_hi] um and amplitude slope x
 * wavelength; an axis tilted from z by an angle uniform in [0, max_tilt]
 * (radians) with uniform azimuth.  A slice of the tube is the disk of radius
 * r(z)/cos(tilt) about the centre line.  Voxels are claimed first-come and a
 * tube never takes a voxel face-adjacent to an earlier tube.  r0_out receives
 * the base radii.  Returns 0. */
int gen_axons(int64_t nx, int64_t ny, int64_t nz, double voxel_um, int n_axons, uint64_t seed,
              double mu, double sigma, double bead_sp, double bead_w, double bead_amp,
              double lam_lo, double lam_hi, double slope, double max_tilt, uint16_t* lab,
              double* r0_out) {
    rng_t rng = {seed};
    const int64_t nv = nx * ny * nz;
    uint8_t* blocked = calloc((size_t)nv, 1);
    if (!blocked) return -2;
    memset(lab, 0, sizeof(uint16_t) * (size_t)nv);
    const double Lz = (double)nz * voxel_um;
    double* rz = malloc(sizeof(double) * (size_t)nz);
    double* xz = malloc(sizeof(double) * (size_t)nz);
    double* yz = malloc(sizeof(double) * (size_t)nz);
    for (int a = 1; a <= n_axons; ++a) {
        const double r0 = exp(mu + sigma * normal(&rng));
        const double cx = unif(&rng) * (double)nx * voxel_um;
        const double cy = unif(&rng) * (double)ny * voxel_um;
        const double tilt = unif(&rng) * max_tilt;
        const double az = unif(&rng) * 2.0 * M_PI;
        const double lx = lam_lo + (lam_hi - lam_lo) * unif(&rng);
        const double ly = lam_lo + (lam_hi - lam_lo) * unif(&rng);
        const double px = unif(&rng) * 2.0 * M_PI, py = unif(&rng) * 2.0 * M_PI;
        r0_out[a - 1] = r0;
        for (int64_t k = 0; k < nz; ++k) rz[k] = 0.0;
        /* Poisson-spaced beads: exponential gaps */
        for (double z = -log(1.0 - unif(&rng)) * bead_sp; z < Lz;
             z += -log(1.0 - unif(&rng)) * bead_sp) {
            for (int64_t k = 0; k < nz; ++k) {
                double d = fabs(((double)k + 0.5) * voxel_um - z);
                if (Lz - d < d) d = Lz - d;
                rz[k] += exp(-0.5 * (d / bead_w) * (d / bead_w));
            }
        }
        double rmax = 0.0;
        for (int64_t k = 0; k < nz; ++k) {
            const double zc = ((double)k + 0.5) * voxel_um, dz = zc - 0.5 * Lz;
            const double bump = rz[k] < 1.0 ? rz[k] : 1.0;
            rz[k] = r0 * (1.0 + bead_amp * bump) / cos(tilt);
            if (rz[k] > rmax) rmax = rz[k];
            xz[k] = cx + tan(tilt) * cos(az) * dz + slope * lx * cos(2.0 * M_PI * zc / lx + px);
            yz[k] = cy + tan(tilt) * sin(az) * dz + slope * ly * cos(2.0 * M_PI * zc / ly + py);
        }
        const int h = (int)ceil(rmax / voxel_um) + 1;
        for (int64_t k = 0; k < nz; ++k) {
            const int64_t ix0 = (int64_t)floor(xz[k] / voxel_um);
            const int64_t iy0 = (int64_t)floor(yz[k] / voxel_um);
            for (int dy = -h; dy <= h; ++dy)
                for (int dx = -h; dx <= h; ++dx) {
                    const double gx = ((double)(ix0 + dx) + 0.5) * voxel_um - xz[k];
                    const double gy = ((double)(iy0 + dy) + 0.5) * voxel_um - yz[k];
                    if (gx * gx + gy * gy > rz[k] * rz[k]) continue;
                    const int64_t x = wrap(ix0 + dx, nx), y = wrap(iy0 + dy, ny);
                    const int64_t idx = x + nx * (y + ny * k);
                    if (blocked[idx] || lab[idx]) continue;
                    lab[idx] = (uint16_t)a;
                }
        }
        /* block the face neighbours of this tube's voxels for later tubes */
        for (int64_t k = 0; k < nz; ++k) {
            const int64_t ix0 = (int64_t)floor(xz[k] / voxel_um);
            const int64_t iy0 = (int64_t)floor(yz[k] / voxel_um);
            for (int dy = -h; dy <= h; ++dy)
                for (int dx = -h; dx <= h; ++dx) {
                    const int64_t x = wrap(ix0 + dx, nx), y = wrap(iy0 + dy, ny);
                    if (lab[x + nx * (y + ny * k)] != (uint16_t)a) continue;
                    for (int q = 0; q < 7; ++q) {
                        const int64_t xx = wrap(x + NB[q][0], nx), yy = wrap(y + NB[q][1], ny),
                                      zz = wrap(k + NB[q][2], nz);
                        blocked[xx + nx * (yy + ny * zz)] = 1;
                    }
                }
        }
    }
    free(rz);
    free(xz);
    free(yz);
    free(blocked);
    return 0;
}
