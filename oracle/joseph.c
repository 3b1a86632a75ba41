/* ORACLE — test infrastructure only.  Plain FP64 CPU reference of the Joseph
 * line-integral projector and its exact adjoint.  It shares no code with the GPU
 * library and is never part of the product path.
 *
 * The paper takes the system model A as given (data fidelity D(Ax + r, y),
 * Section 1, eq. (1); its simulations use an external projector, Section 3.1).
 * The projector follows Joseph's ray-driven scheme (Joseph 1982), written from
 * its definition:
 *
 *   For a line p1 -> p2 with direction u = p2 - p1, pick the principal axis m
 *   maximising |u_m| / v_m (ties within a relative 1e-9 go to the lowest axis).
 *   At every voxel-centre plane i along m whose crossing parameter
 *   lambda = (o_m + i v_m - p1_m) / u_m lies in [0, 1], evaluate the image by
 *   (bi)linear interpolation in the two remaining axes, treating voxels outside
 *   the grid as zero.  The line integral is l * sum(samples) with the step
 *   length l = v_m |u| / |u_m|.
 *
 *   TOF: a sample at signed distance t = (lambda - 1/2)|u| from the LOR centre
 *   contributes to TOF bin b (centre t_b, width w) with the Gaussian kernel
 *   (standard deviation sigma) truncated to |t' - t| <= nsig sigma and
 *   integrated over the bin:
 *     1/2 [E(t_b + w/2 - t) - E(t_b - w/2 - t)],  E(u) = erf(clamp(u / (sqrt2 sigma), -c, c)),
 *   c = nsig / sqrt2 (no clamp when nsig <= 0).  The weight is continuous in t
 *   and the weights of a sample whose truncation window lies inside the bins
 *   sum to erf(nsig / sqrt2).
 *
 * The adjoint scatters exactly the same (voxel, weight) pairs.
 *
 * Image: [nz][ny][nx], voxel (ix, iy, iz) centred at o + (ix vx, iy vy, iz vz),
 * o = -((n - 1)/2) v per axis.  Sinogram values: [nlor][ntof].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* erf of u / (sqrt2 sigma), with the argument clamped to +-nsig/sqrt2. */
static double clamped_erf(double u, double sigma, double nsig) {
    double z = u / (sqrt(2.0) * sigma);
    if (nsig > 0) {
        double c = nsig / sqrt(2.0);
        if (z > c) z = c;
        if (z < -c) z = -c;
    }
    return erf(z);
}

static int principal_axis(const double u[3], const double v[3]) {
    int m = 0;
    double best = fabs(u[0]) / v[0];
    for (int a = 1; a < 3; ++a) {
        double r = fabs(u[a]) / v[a];
        if (r > best * (1.0 + 1e-9)) {
            best = r;
            m = a;
        }
    }
    return m;
}

/* Visit every (voxel index, weight, tof weights) of one LOR.
 * mode 0: forward, acc[b] += w * img[idx] * tofw[b]
 * mode 1: adjoint, img[idx] += w * sum_b tofw[b] * vals[b] */
static void joseph_lor(int mode, const double *p1, const double *p2, const int n[3],
                       const double v[3], int ntof, double tof_bin, double sigma, double nsig,
                       double *img, double *vals) {
    double o[3], u[3];
    for (int a = 0; a < 3; ++a) {
        o[a] = -0.5 * (n[a] - 1) * v[a];
        u[a] = p2[a] - p1[a];
    }
    double len = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    int m = principal_axis(u, v);
    int A = (m + 1) % 3, B = (m + 2) % 3;
    double ell = v[m] * len / fabs(u[m]);
    double acc[64];
    for (int b = 0; b < ntof; ++b) acc[b] = 0.0;
    long stride[3] = {1, n[0], (long)n[0] * n[1]};
    for (int i = 0; i < n[m]; ++i) {
        double lam = (o[m] + i * v[m] - p1[m]) / u[m];
        if (lam < 0.0 || lam > 1.0) continue;
        double xa = (p1[A] + lam * u[A] - o[A]) / v[A];
        double xb = (p1[B] + lam * u[B] - o[B]) / v[B];
        double ja = floor(xa), jb = floor(xb);
        double fa = xa - ja, fb = xb - jb;
        double tw[64];
        double twsum = 0.0;
        if (ntof == 1) {
            tw[0] = 1.0;
        } else {
            double t = (lam - 0.5) * len;
            for (int b = 0; b < ntof; ++b) {
                double tb = (b - 0.5 * (ntof - 1)) * tof_bin;
                tw[b] = 0.5 * (clamped_erf(tb + 0.5 * tof_bin - t, sigma, nsig) -
                               clamped_erf(tb - 0.5 * tof_bin - t, sigma, nsig));
            }
        }
        if (mode == 1)
            for (int b = 0; b < ntof; ++b) twsum += tw[b] * vals[b];
        for (int ea = 0; ea < 2; ++ea) {
            long ia = (long)ja + ea;
            if (ia < 0 || ia >= n[A]) continue;
            double wa = ea ? fa : 1.0 - fa;
            for (int eb = 0; eb < 2; ++eb) {
                long ib = (long)jb + eb;
                if (ib < 0 || ib >= n[B]) continue;
                double w = wa * (eb ? fb : 1.0 - fb);
                long idx = i * stride[m] + ia * stride[A] + ib * stride[B];
                if (mode == 0) {
                    for (int b = 0; b < ntof; ++b) acc[b] += w * img[idx] * tw[b];
                } else {
                    img[idx] += ell * w * twsum;
                }
            }
        }
    }
    if (mode == 0)
        for (int b = 0; b < ntof; ++b) vals[b] = ell * acc[b];
}

/* adjoint == 0: sino[l][b] = (P img)[l][b]
 * adjoint == 1: img = P^T sino (img is overwritten) */
void orc_joseph(int adjoint, long nlor, const double *p1, const double *p2, int nx, int ny,
                int nz, double vx, double vy, double vz, int ntof, double tof_bin, double sigma,
                double nsig, double *img, double *sino, int nthreads) {
    int n[3] = {nx, ny, nz};
    double v[3] = {vx, vy, vz};
    long nvox = (long)nx * ny * nz;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    if (!adjoint) {
#pragma omp parallel for schedule(dynamic, 64)
        for (long l = 0; l < nlor; ++l)
            joseph_lor(0, p1 + 3 * l, p2 + 3 * l, n, v, ntof, tof_bin, sigma, nsig, img,
                       sino + l * ntof);
        return;
    }
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *part = (double *)calloc((size_t)nt * nvox, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = part + (size_t)tid * nvox;
#pragma omp for schedule(static)
        for (long l = 0; l < nlor; ++l)
            joseph_lor(1, p1 + 3 * l, p2 + 3 * l, n, v, ntof, tof_bin, sigma, nsig, mine,
                       sino + l * ntof);
    }
    for (long k = 0; k < nvox; ++k) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += part[(size_t)t * nvox + k];
        img[k] = s;
    }
    free(part);
}
