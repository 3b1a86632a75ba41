/* Synthetic-input generator: continuous phantoms made of ellipsoids, their exact
 * line integrals (non-TOF and TOF), attenuation chords, voxelisation and Poisson
 * sampling with a counter-based generator.
 *
 * This is data generation only: the phantom is continuous and its projections
 * are closed-form integrals, not the discrete projector of the reconstruction.
 *
 * Shape record (9 doubles): cx cy cz ax ay az rot_z_rad value pad.
 * An ellipsoid with semi-axes (ax, ay, az) is rotated by rot_z about z and
 * centred at c; its value is an additive increment (nested shapes compose).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define SHAPE_STRIDE 9

/* Entry/exit parameters (lambda along p1 + lambda*u) of a line with an ellipsoid;
 * returns 0 when the line misses it. */
static int ellipsoid_hit(const double *sh, const double p1[3], const double u[3],
                         double *l0, double *l1) {
    double cr = cos(sh[6]), sr = sin(sh[6]);
    double d[3] = {p1[0] - sh[0], p1[1] - sh[1], p1[2] - sh[2]};
    /* rotate into the ellipsoid frame (inverse rotation) */
    double q[3] = {cr * d[0] + sr * d[1], -sr * d[0] + cr * d[1], d[2]};
    double w[3] = {cr * u[0] + sr * u[1], -sr * u[0] + cr * u[1], u[2]};
    double A = 0, B = 0, C = -1.0;
    for (int a = 0; a < 3; ++a) {
        double inv = 1.0 / (sh[3 + a] * sh[3 + a]);
        A += w[a] * w[a] * inv;
        B += 2.0 * q[a] * w[a] * inv;
        C += q[a] * q[a] * inv;
    }
    double disc = B * B - 4 * A * C;
    if (A <= 0 || disc <= 0) return 0;
    double sq = sqrt(disc);
    *l0 = (-B - sq) / (2 * A);
    *l1 = (-B + sq) / (2 * A);
    return 1;
}

static double G(double z) { return z * erf(z) + exp(-z * z) / sqrt(M_PI); }

/* F(u) = integral from 0 to u of erf(clamp(v / s, -c, c)) dv (even in u);
 * c <= 0 means no clamp. */
static double F(double u, double s, double c) {
    double v = fabs(u);
    if (c <= 0 || v <= c * s) return s * (G(v / s) - 1.0 / sqrt(M_PI));
    return s * (G(c) - 1.0 / sqrt(M_PI)) + erf(c) * (v - c * s);
}

/* Integral over t in [A, B] of the TOF weight of bin centre tb and half-width
 * h: the Gaussian kernel truncated to +-nsig sigma, integrated over the bin. */
static double tof_seg(double A, double B, double tb, double h, double sigma, double nsig) {
    if (B <= A) return 0.0;
    double s = sqrt(2.0) * sigma, c = nsig > 0 ? nsig / sqrt(2.0) : 0.0;
    return 0.5 * (F(tb + h - A, s, c) - F(tb + h - B, s, c) - F(tb - h - A, s, c) + F(tb - h - B, s, c));
}

/* Line integrals of the phantom for lines x planes (x TOF bins).
 * p1xy/p2xy: [n_lines][2] transaxial endpoints; z1/z2: [n_planes] axial ends.
 * out: [n_lines][n_planes][n_tof] float. */
void gen_project(long n_lines, const double *p1xy, const double *p2xy, long n_planes,
                 const double *z1, const double *z2, int n_shapes, const double *shapes,
                 int n_tof, double tof_bin, double sigma, double nsig, float *out) {
#pragma omp parallel for schedule(dynamic, 16)
    for (long L = 0; L < n_lines; ++L) {
        double tb[64];
        for (int b = 0; b < n_tof; ++b) tb[b] = (b - (n_tof - 1) / 2.0) * tof_bin;
        for (long p = 0; p < n_planes; ++p) {
            double P1[3] = {p1xy[2 * L], p1xy[2 * L + 1], z1[p]};
            double U[3] = {p2xy[2 * L] - P1[0], p2xy[2 * L + 1] - P1[1], z2[p] - z1[p]};
            double len = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
            float *o = out + (L * n_planes + p) * n_tof;
            double acc[64];
            for (int b = 0; b < n_tof; ++b) acc[b] = 0.0;
            for (int s = 0; s < n_shapes; ++s) {
                const double *sh = shapes + SHAPE_STRIDE * s;
                double l0, l1;
                if (!ellipsoid_hit(sh, P1, U, &l0, &l1)) continue;
                if (l0 < 0) l0 = 0;
                if (l1 > 1) l1 = 1;
                if (l1 <= l0) continue;
                double t0 = (l0 - 0.5) * len, t1 = (l1 - 0.5) * len;
                if (n_tof == 1) {
                    acc[0] += sh[7] * (t1 - t0);
                } else {
                    for (int b = 0; b < n_tof; ++b) {
                        double A = t0, B = t1;
                        if (nsig > 0) {  /* the weight vanishes beyond h + nsig sigma */
                            double lo = tb[b] - 0.5 * tof_bin - nsig * sigma, hi = tb[b] + 0.5 * tof_bin + nsig * sigma;
                            if (A < lo) A = lo;
                            if (B > hi) B = hi;
                        }
                        acc[b] += sh[7] * tof_seg(A, B, tb[b], 0.5 * tof_bin, sigma, nsig);
                    }
                }
            }
            for (int b = 0; b < n_tof; ++b) o[b] = (float)acc[b];
        }
    }
}

/* Chord length (mm) of each line x plane through one ellipsoid. out: [n_lines][n_planes]. */
void gen_chord(long n_lines, const double *p1xy, const double *p2xy, long n_planes,
               const double *z1, const double *z2, const double *shape, double *out) {
#pragma omp parallel for schedule(static)
    for (long L = 0; L < n_lines; ++L) {
        for (long p = 0; p < n_planes; ++p) {
            double P1[3] = {p1xy[2 * L], p1xy[2 * L + 1], z1[p]};
            double U[3] = {p2xy[2 * L] - P1[0], p2xy[2 * L + 1] - P1[1], z2[p] - z1[p]};
            double len = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
            double l0, l1, c = 0.0;
            if (ellipsoid_hit(shape, P1, U, &l0, &l1)) {
                if (l0 < 0) l0 = 0;
                if (l1 > 1) l1 = 1;
                if (l1 > l0) c = (l1 - l0) * len;
            }
            out[L * n_planes + p] = c;
        }
    }
}

/* Supersampled voxelisation: value = mean over ss_xy^2 * ss_z sub-points of the
 * sum of the increments of the shapes containing the sub-point. */
void gen_voxelize(int nx, int ny, int nz, double vx, double vy, double vz, int ss_xy, int ss_z,
                  int n_shapes, const double *shapes, double *out) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                double cx = (ix - (nx - 1) / 2.0) * vx, cy = (iy - (ny - 1) / 2.0) * vy,
                       cz = (iz - (nz - 1) / 2.0) * vz;
                double acc = 0.0;
                for (int sz = 0; sz < ss_z; ++sz)
                    for (int sy = 0; sy < ss_xy; ++sy)
                        for (int sx = 0; sx < ss_xy; ++sx) {
                            double px = cx + ((sx + 0.5) / ss_xy - 0.5) * vx;
                            double py = cy + ((sy + 0.5) / ss_xy - 0.5) * vy;
                            double pz = ss_z > 1 ? cz + ((sz + 0.5) / ss_z - 0.5) * vz : cz;
                            for (int s = 0; s < n_shapes; ++s) {
                                const double *sh = shapes + SHAPE_STRIDE * s;
                                double cr = cos(sh[6]), sr = sin(sh[6]);
                                double dx = px - sh[0], dy = py - sh[1], dz = pz - sh[2];
                                double qx = cr * dx + sr * dy, qy = -sr * dx + cr * dy;
                                double r = qx * qx / (sh[3] * sh[3]) + qy * qy / (sh[4] * sh[4]) +
                                           dz * dz / (sh[5] * sh[5]);
                                if (r <= 1.0) acc += sh[7];
                            }
                        }
                out[((long)iz * ny + iy) * nx + ix] = acc / (ss_xy * ss_xy * ss_z);
            }
}

/* ---- counter-based uniform generator (SplitMix64 finaliser, Steele et al. 2014) ---- */
static inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline double unif(uint64_t key, uint64_t *ctr) {
    uint64_t r = mix64(key + 0x632BE59BD9B4E019ULL * (++*ctr));
    return ((r >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* One Poisson variate: inversion for small means, PTRS transformed rejection
 * (Hoermann 1993) for larger ones. */
static uint32_t poisson_draw(double lam, uint64_t key) {
    uint64_t ctr = 0;
    if (!(lam > 0)) return 0;
    if (lam < 10.0) {
        double u = unif(key, &ctr), p = exp(-lam), F = p;
        uint32_t k = 0;
        while (u > F && k < 1000) {
            ++k;
            p *= lam / k;
            F += p;
        }
        return k;
    }
    double slam = sqrt(lam), loglam = log(lam);
    double b = 0.931 + 2.53 * slam, a = -0.059 + 0.02483 * b;
    double invalpha = 1.1239 + 1.1328 / (b - 3.4), vr = 0.9277 - 3.6224 / (b - 2);
    for (;;) {
        double U = unif(key, &ctr) - 0.5, V = unif(key, &ctr);
        double us = 0.5 - fabs(U);
        double k = floor((2 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= vr) return (uint32_t)k;
        if (k < 0 || (us < 0.013 && V > us)) continue;
        if (log(V) + log(invalpha) - log(a / (us * us) + b) <= -lam + k * loglam - lgamma(k + 1))
            return (uint32_t)k;
    }
}

/* Poisson samples of mean[j] (float) for j in [0, n); element j depends only on
 * (seed, offset + j), so a large array can be drawn in chunks.  dtype 0: uint8, 1: uint16, 2: float32.  Returns the largest draw
 * (so a caller can detect that a narrow type saturated). */
uint32_t gen_poisson(long n, long offset, const float *mean, uint64_t seed, int dtype, void *out) {
    uint32_t gmax = 0;
    uint64_t skey = mix64(seed ^ 0xA5A5A5A5DEADBEEFULL);
#pragma omp parallel for schedule(static) reduction(max : gmax)
    for (long j = 0; j < n; ++j) {
        uint32_t k = poisson_draw((double)mean[j], mix64(skey ^ (uint64_t)(j + offset)));
        if (k > gmax) gmax = k;
        if (dtype == 0) ((uint8_t *)out)[j] = (uint8_t)(k > 255 ? 255 : k);
        else if (dtype == 1) ((uint16_t *)out)[j] = (uint16_t)(k > 65535 ? 65535 : k);
        else ((float *)out)[j] = (float)k;
    }
    return gmax;
}
