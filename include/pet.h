/* pet.h — C ABI of the MI355X (gfx950) library for RDP-regularised PET
 * reconstruction with prior-aware preconditioned SVRG.
 *
 * Problem (Section 1, eq. (1) with the prior of eq. (prior)):
 *     minimise  D(A x + r, y) + beta S(x) + i_{>=0}(x),
 * D the Poisson (KL) data fidelity (Section 1.2), S the relative difference
 * prior (eq. (rdp)), A = diag(mult) P with P the Joseph line-integral
 * projector (TOF-resolved when the scanner has TOF bins) and r > 0 the additive
 * background.  The data are split into n subsets of interleaved views
 * (Section 2.4): subset i holds views v = i, i + n, i + 2n, ...
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Image:     float [nz][ny][nx] (x fastest), voxel (ix, iy, iz) centred at
 *            ((ix - (nx-1)/2) vx, (iy - (ny-1)/2) vy, (iz - (nz-1)/2) vz) mm.
 * Sinogram:  flat index ((view * n_rad + radial) * n_planes + plane) * n_tof + tof
 *            (view-major, TOF innermost).  Every sinogram argument is a FULL
 *            sinogram (all views); a call on subset i reads/writes only the views
 *            of subset i and leaves the others untouched.  subset = -1 means all
 *            views.
 * mult:      float per LOR, index (view * n_rad + radial) * n_planes + plane,
 *            shared by all TOF bins of the LOR.
 * Pointers:  device pointers unless stated otherwise; all are caller-owned and
 *            never freed by the library.  Only pet_geom_create allocates (its
 *            geometry tables and a scratch arena owned by the handle).
 * Streams:   `stream` is a hipStream_t (NULL = default stream).  Calls enqueue
 *            work on it and return without synchronising, except
 *            pet_geom_create / pet_geom_destroy (synchronous) and the host-side
 *            reads of pet_osem_epoch / pet_svrg_epoch noted below.
 * Threads:   a pet_geom handle owns scratch memory: calls on one handle must
 *            not overlap in time (same or different streams).  Separate handles
 *            are independent.
 * Errors:    argument errors return PET_E_ARG before anything is enqueued;
 *            a HIP launch failure returns PET_E_HIP.  pet_last_error() returns a
 *            thread-local message for the last non-OK status.  Domain
 *            preconditions (x >= 0, r > 0, y >= 0) are the caller's: values
 *            outside them give unspecified results (the paper's d(s, t) and R(x)
 *            are infinite there) unless the handle's PET_CHECK flag is set
 *            (pet_geom_set_flags), which turns them into PET_E_DOMAIN and a
 *            non-finite objective into PET_E_NUMERIC.
 */
#ifndef PET_H
#define PET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PET_OK = 0,
    PET_E_ARG = 1,
    PET_E_DOMAIN = 2,
    PET_E_OOM = 3,
    PET_E_HIP = 4,
    PET_E_NUMERIC = 5,
    PET_E_STATE = 6
} pet_status;

enum { PET_SCANNER_PARALLEL2D = 0, PET_SCANNER_CYLINDER = 1 };
enum { PET_BACK_AUTO = 0, PET_BACK_SCATTER = 1, PET_BACK_GATHER = 2 };
enum { PET_Y_F32 = 0, PET_Y_U16 = 1, PET_Y_U8 = 2 };

/* Scanner + image description.
 * PET_SCANNER_CYLINDER: n_crystals per ring (= 2 n_views), ring radius, rings
 *   at z_r = (r - (n_rings-1)/2) ring_pitch; LOR (view v, radial k, plane p)
 *   joins s n - h t (ring r1) to s n + h t (ring r2) with phi = pi v / n_views,
 *   n = (cos phi, sin phi), t = (-sin phi, cos phi),
 *   s = R sin(pi (k - (n_rad-1)/2) / n_crystals), h = sqrt(R^2 - s^2);
 *   planes (r1, r2) with |r2 - r1| <= max_ring_diff ordered by segment
 *   d = r2 - r1 = 0, -1, +1, -2, +2, ... and r1 ascending.
 * PET_SCANNER_PARALLEL2D: nz = 1, one plane, s = (k - (n_rad-1)/2) rad_spacing,
 *   endpoints s n -/+ half_length t.
 * TOF (n_tof > 1): bin b centred at t_b = (b - (n_tof-1)/2) tof_bin along the
 *   LOR (signed distance from the LOR centre towards the second endpoint);
 *   weight of a point at t: the Gaussian kernel (sigma tof_sigma) truncated to
 *   |t' - t| <= tof_nsigma sigma, integrated over the bin [t_b -/+ tof_bin/2].
 *   At most 32 bins, and at most 8 of them may overlap one point's window
 *   (PET_E_ARG otherwise); a TOF segment holds at most 64 planes.
 */
typedef struct {
    int kind;
    int nx, ny, nz;
    double vx, vy, vz;
    int n_views, n_rad;
    double radius_mm;
    int n_crystals, n_rings;
    double ring_pitch_mm;
    int max_ring_diff;
    double rad_spacing_mm, half_length_mm;
    int n_tof;
    double tof_bin_mm, tof_sigma_mm, tof_nsigma;
    int n_subsets;
    /* Image-space resolution model (Section 3.1): A = P G with G an isotropic
     * Gaussian of this FWHM in mm (0: none).  G is separable, with sampled
     * weights exp(-d^2 / (2 sigma_a^2)) over |d| <= floor(4 sigma_a + 1/2)
     * voxels of axis a, normalised to sum 1, and zero outside the grid (so G
     * is symmetric and A^T = G P^T); 2D grids (nz = 1) blur in x and y only.
     * At most 16 voxels of radius. */
    double psf_fwhm_mm;
} pet_geom_desc;

typedef struct pet_geom_s *pet_geom;

/* Build the geometry tables (FP64 on the host, FP32 on the device) and the
 * scratch arena on the current HIP device.  Synchronous.  PET_E_ARG for an
 * inconsistent description or one the projector does not support (a principal
 * axis along z, LOR endpoints inside the padded image box, a sheet larger than
 * the LDS); PET_E_OOM if device allocation fails. */
pet_status pet_geom_create(const pet_geom_desc *desc, pet_geom *out);
pet_status pet_geom_destroy(pet_geom g);

/* Sizes: number of sinogram bins (incl. TOF) and LORs of `subset` (-1: all),
 * and voxels.  Any output pointer may be NULL. */
pet_status pet_geom_info(pet_geom g, int subset, int64_t *n_bins, int64_t *n_lors, int64_t *n_vox);

/* Forward model of one subset (eq. (1)): out = mult * (P_subset x) + add.
 * mult, add nullable (1 and 0).  Writes only the bins of the subset's views. */
pet_status pet_fwd(pet_geom g, int subset, const float *x, const float *mult, const float *add,
                   float *out, void *stream);

/* Adjoint (Section 2.3: A^T enters the gradient of eq. (template) and A^T 1
 * the preconditioner of eq. (preconditioner)): x_out (+)= P_subset^T (mult * sino).
 * sino NULL means all ones (so pet_back(g, -1, NULL, mult, sens, 0, ...) gives
 * the sensitivity A^T 1).  accumulate = 0 overwrites x_out.  algo:
 *   PET_BACK_SCATTER  line-driven scatter: each sample of each LOR adds its two
 *                     axial interpolation shares to an LDS sheet of its line
 *                     with FP64 LDS atomics;
 *   PET_BACK_GATHER   cell-driven gather: each sheet cell sums, without
 *                     atomics, the shares of the samples that land on it,
 *                     found from each segment's affine axial map (TOF weights
 *                     from the tabulated bin-integrated Gaussian);
 *   PET_BACK_AUTO     the scatter, measured faster on every workload here.
 * Both spread the sheets over the transaxial neighbours with global float
 * atomics, so the sum order is not deterministic; both give the same
 * (sample, weight) pairs.  PET_E_ARG for PET_BACK_GATHER when the per-plane
 * tables of the line exceed the LDS. */
pet_status pet_back(pet_geom g, int subset, const float *sino, const float *mult, float *x_out,
                    int accumulate, int algo, void *stream);

/* Gradient of the subset data term D_i (Section 2, eq. (template)):
 * grad_out = P_i^T [mult (1 - y / (mult P_i x + add))], fused per LOR (no
 * sinogram-sized intermediate).  y has type y_dtype.  kl_out (device double,
 * nullable) receives sum over the subset's bins of d(ybar, y) (FP64). */
pet_status pet_subset_grad(pet_geom g, int subset, const float *x, const void *y, int y_dtype,
                           const float *add, const float *mult, float *grad_out, double *kl_out,
                           void *stream);

/* Allocation-free pet_subset_grad, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and errors as pet_subset_grad;
 * the call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  Its work buffers (the two transposed image sheets and the two
 * gradient sheets of the geometry, one FP64 partial per line of the subset
 * and, with a resolution model, two image-sized buffers) are carved from one
 * static device array of PET_NOALLOC_SCRATCH_BYTES, 256-byte aligned.  Every
 * device holds its own copy from the library's load until the process ends
 * (the address is looked up once per device, at pet_geom_create or at the
 * first call).  PET_E_ARG when the geometry needs more than that (C1/C2-sized
 * 128x128x71 geometries need about 21 MB).  All calls on one device share the
 * array and it keeps the last call's contents: each call clears what must
 * start at zero, and calls that overlap in time on one device (different
 * streams, threads or handles) race on it and must be serialised. */
#define PET_NOALLOC_SCRATCH_BYTES ((size_t)24 << 20)
pet_status pet_subset_grad_noalloc(pet_geom g, int subset, const float *x, const void *y, int y_dtype,
                                   const float *add, const float *mult, float *grad_out, double *kl_out,
                                   void *stream);

/* Zero-count-aware data term -------------------------------------------------
 * The KL data fidelity has d(s, 0) = s (Section 1.2): a bin without counts
 * adds mult P x + add to the objective and mult P^T 1 to the gradient at every
 * x.  With sens_i = P_i^T mult (pet_back with sino = NULL on subset i),
 *     grad D_i(x) = sens_i - P_i^T [mult y / ybar(x)],
 *     D_i(x)      = <sens_i, x> + sum_i add - sum_i y + sum_{i, y > 0} y log(y / ybar(x)),
 * where only bins with y > 0 enter the terms that depend on ybar.  A pet_counts
 * object holds those bins of one data set (y, add, mult) on one geometry,
 * compacted per transaxial line, TOF bin major within a line (16 bytes per
 * bin: index within its transaxial line, y, add, mult), with per-line offsets
 * and, per subset, its lines with counts ordered by decreasing count.  The
 * kernels that use it take one workgroup per such line and one to sixteen
 * lanes per compacted bin, walking only the samples inside the bin's TOF
 * window.  The TOF weight of a sample at signed
 * distance t from the LOR centre in bin b is the geometry's truncated,
 * bin-integrated Gaussian, a function of d = t - t_b alone; it is tabulated
 * from FP64 at 4097 nodes over its support |d| <= bin/2 + nsig sigma and
 * interpolated linearly (C2's 40 mm bins and 60 mm FWHM: nodes 0.047 mm
 * apart, interpolation error below 1e-6 of the largest weight).  Results equal
 * those of the dense kernels up to rounding and that interpolation. */
typedef struct pet_counts_s *pet_counts;

/* Compact the bins with y > 0 of (y, add, mult) for geometry g (full
 * sinograms; add, mult nullable: 0 and 1).  Synchronous; allocates the list
 * and its index on the current device (the inputs may be freed afterwards),
 * and, for geometries without a resolution model, n_subsets pairs of
 * gradient-sheet buffers for one-launch snapshot passes (about 10 MB per
 * subset on a 128x128x71 grid).
 * PET_E_ARG if the geometry's sheets and TOF table exceed the LDS; PET_E_OOM if
 * device allocation fails. */
pet_status pet_counts_create(pet_geom g, const void *y, int y_dtype, const float *add, const float *mult,
                             pet_counts *out);
pet_status pet_counts_destroy(pet_counts c);

/* Bins with counts of `subset` (-1: all) and the FP64 sums of y and of add over
 * all of its bins.  Any output pointer may be NULL. */
pet_status pet_counts_info(pet_counts c, int subset, int64_t *n_items, double *sum_y, double *sum_add);

/* Subset gradient from the compacted bins: grad_out = sens_subset -
 * P_i^T [mult y / ybar] with ybar = mult P_i x + add, or, with sens_subset NULL,
 * the part that depends on x, -P_i^T [mult y / ybar], alone.  kl_out (device
 * double, nullable; needs sens_subset) receives D_i(x) in FP64 as above.
 * PET_E_ARG if c was made for another geometry. */
pet_status pet_subset_grad_counts(pet_geom g, pet_counts c, int subset, const float *x, const float *sens_subset,
                                  float *grad_out, double *kl_out, void *stream);

/* pet_objective from the compacted bins: D(A x + r, y) + beta S(x) in FP64
 * (device double), with sens = P^T mult over all subsets. */
pet_status pet_objective_counts(pet_geom g, pet_counts c, const float *x, const float *sens, const float *kappa,
                                const float w[27], float beta, float gamma, float eps, double *out, void *stream);

/* pet_osem_epoch from the compacted bins (Section 3.1 initialisation): for
 * each subset i in order[] (host array of n_subsets entries),
 * x <- x * P_i^T(mult y / ybar) / P_i^T mult, where only bins with y > 0 enter
 * the numerator (the others add 0 to it).  mult is the LOR array the counts
 * were made with (nullable: 1); it enters P_i^T mult, which on a TOF geometry
 * is computed with the bins' weights summed per sample.  Voxels with
 * P_i^T mult = 0 keep x.  xmax_out (device float, nullable) receives max(x)
 * after the epoch; sens_out (device, n_vox floats, nullable) the sensitivity
 * P^T mult over all subsets, summed in FP32 from the epoch's subset
 * sensitivities in order[] (equal to pet_back's up to rounding), so that a
 * reconstruction needs no separate sensitivity pass.  PET_E_ARG if c was made
 * for another geometry. */
pet_status pet_osem_epoch_counts(pet_geom g, pet_counts c, float *x, const float *mult, const int32_t *order,
                                 float *xmax_out, float *sens_out, void *stream);

/* Relative difference prior (eq. (rdp)) and its derivatives (Appendix A),
 * scaled by beta: grad_out = beta dS/dx, hessdiag_out = beta d2S/dx2 (nullable),
 * value_out = beta S (device double, nullable).  w[27]: weight of neighbour
 * offset (dz, dy, dx) at index (dz+1)*9 + (dy+1)*3 + (dx+1) (centre ignored);
 * neighbours outside the grid are omitted.  kappa nullable (1). */
pet_status pet_rdp_grad_hessdiag(pet_geom g, const float *x, const float *kappa, const float w[27],
                                 float beta, float gamma, float eps, float *grad_out,
                                 float *hessdiag_out, double *value_out, void *stream);

/* Prior-aware preconditioner (eq. (preconditioner)):
 * D = (x + delta) / (sens + alpha hessdiag (x + delta)), D = 0 where the
 * denominator is 0.  hessdiag is the diagonal of the Hessian of beta S. */
pet_status pet_precond(pet_geom g, const float *x, const float *sens, const float *hessdiag,
                       float alpha, float delta, float *D_out, void *stream);

/* One OSEM epoch (Section 3.1 initialisation): for each subset i in order[]
 * (host array of n_subsets entries): x <- x * P_i^T(mult y / ybar) / P_i^T mult
 * (voxels with P_i^T mult = 0 keep x).  xmax_out (device float, nullable)
 * receives max(x) after the epoch. */
pet_status pet_osem_epoch(pet_geom g, float *x, const void *y, int y_dtype, const float *add,
                          const float *mult, const int32_t *order, float *xmax_out, void *stream);

/* Objective D(A x + r, y) + beta S(x) in FP64 (device double). */
pet_status pet_objective(pet_geom g, const float *x, const void *y, int y_dtype, const float *add,
                         const float *mult, const float *kappa, const float w[27], float beta,
                         float gamma, float eps, double *out, void *stream);

/* Caller-owned state of preconditioned SVRG (Algorithm 1).  Device buffers
 * sized from pet_geom_info: ghat_i [n_subsets][n_vox] float, ghat [n_vox]
 * double, x_snap [n_vox] float, D [n_vox] float, sens [n_vox] float (A^T 1
 * over all subsets, e.g. from pet_back).  ghat_i stores the data-term part of
 * the subset gradients at the snapshot; the prior enters each step through its
 * exact current gradient, which equals Algorithm 1's estimator (the prior's
 * 1/n shares cancel). */
typedef struct {
    float *ghat_i;
    double *ghat;
    float *x_snap;
    float *D;
    const float *sens;
    const void *y;
    int y_dtype;
    const float *add;
    const float *mult;
    const float *kappa;
    float w[27];
    float beta, gamma, eps, alpha, delta;
    int omega;
    int64_t k;
    /* ALG2/ALG3 extensions (pet_svrg_epoch_ex), all nullable device buffers:
     * bb [4] double: short Barzilai-Borwein state {p.q, q.D q, tau_bb, updates},
     *   reset at k = 0 with tau_bb = +inf; every step of an epoch then uses
     *   min(tau[j], tau_bb);
     * g_prev [n_vox] float: full gradient at the last snapshot (needed with bb);
     * gnorm [n_subsets] double: ||grad J_i(xhat)|| at the last snapshot
     *   (importance sampling, Section 2.4). */
    double *bb;
    float *g_prev;
    double *gnorm;
    /* Zero-count-aware path (nullable): a pet_counts made from this state's y,
     * add and mult on the same geometry.  When set, pet_svrg_epoch(_ex) walks
     * only the bins with counts: the sensitivity terms P_i^T mult cancel in
     * n (grad D_i(x) - ghat_i), so ghat_i holds -P_i^T[mult y / ybar(xhat)] and
     * ghat = sens + sum_i ghat_i, the same full gradient as the dense path;
     * objective_out is computed from the compacted bins.  The iterates equal
     * the dense path's up to rounding.  Not with gnorm (PET_E_ARG).  SAGA and
     * SGD take it too (see pet_saga_epoch); the reverse mode and batches use
     * the dense kernels (PET_E_ARG if set).  Without a kappa image or a
     * resolution model, a snapshot pass runs as one launch over the lines of
     * all subsets, each subset into gradient sheets of its own (held by the
     * counts handle, see pet_counts_create); epochs that share one counts
     * handle must not overlap in time (as for a geometry handle). */
    pet_counts counts;
    /* Objective at the snapshots (nullable device double): every snapshot
     * iteration writes Phi(xhat) = D(A xhat + r, y) + beta S(xhat) in FP64,
     * summed from the snapshot's own subset passes (their per-line KL
     * partials; with counts, plus <sens, xhat> and the data sums) and one RDP
     * value pass, so it costs no extra projection (eq. (1), Section 1.2). */
    double *snap_objective;
} pet_svrg_state;

/* One epoch = n_subsets iterations of Algorithm 1 with the nonnegativity
 * proximal step of eq. (sgm).  Iteration j (global k = state->k + j):
 *   if update_pc[j]: D <- pet_precond at x;
 *   if k mod (omega n) == 0: snapshot (all ghat_i, ghat = sum ghat_i in FP64,
 *     x_snap = x) and g = ghat + beta grad S(x);
 *   else i = subset_seq[j], g = n (grad D_i(x) - ghat_i) + ghat + beta grad S(x);
 *   x <- max(0, x - tau[j] D g).
 * subset_seq, tau, update_pc are HOST arrays of n_subsets entries.  state->k
 * advances by n_subsets; a fresh state starts at k = 0 (a snapshot iteration)
 * and D must hold a preconditioner before the first iteration that does not
 * update it.  PET_E_STATE for k < 0.  x is updated in place.  objective_out (device double,
 * nullable) receives the objective at the final x (one extra forward pass). */
pet_status pet_svrg_epoch(pet_geom g, pet_svrg_state *state, float *x, const int32_t *subset_seq,
                          const float *tau, const uint8_t *update_pc, double *objective_out,
                          void *stream);

/* pet_svrg_epoch with the ALG2/ALG3 options (Section 2.2, Section 2.4, Section 4
 * and its table of hyperparameters).  opt (host, nullable = pet_svrg_epoch):
 *   bb_update [n] flags: at these iterations (snapshots only; PET_E_ARG
 *     otherwise) recompute tau_bb = p.q / q.D q from the last two snapshots,
 *     p the difference of the snapshot images and q of their full gradients
 *     (the short BB step in the metric of the diagonal preconditioner D; the
 *     paper's p.q / q.q for D = I); kept when either dot is not positive.  The
 *     new bound already applies to that iteration's step.  Needs state->bb.
 *   weight [n] floats (> 0): estimator weight w of the sampled subset,
 *     g = w (grad D_i(x) - ghat_i) + ghat + beta grad S(x); w = n is uniform
 *     sampling, w = 1 / p_i importance sampling with replacement.
 * With state->gnorm set, every snapshot also writes ||grad J_i(xhat)||. */
typedef struct {
    const uint8_t *bb_update;
    const float *weight;
} pet_svrg_options;
pet_status pet_svrg_epoch_ex(pet_geom g, pet_svrg_state *state, float *x, const int32_t *subset_seq,
                             const float *tau, const uint8_t *update_pc, const pet_svrg_options *opt,
                             double *objective_out, void *stream);

/* The other stochastic estimators of Section 2.1, on the same iteration,
 * state, schedules and clipped step as pet_svrg_epoch (J_i = D_i + (beta/n) S,
 * eq. (template)):
 *   SAGA, eq. (saga): g = n (grad J_i(x) - T_i) + sum_q T_q, then
 *     T_i <- grad J_i(x).  The table T lives in state->ghat_i (n_subsets images,
 *     FP32) and its sum in state->ghat (FP64).  When state->k == 0 the table is
 *     filled at the current x before the first iteration (all subsets; that
 *     iteration then steps along sum_q T_q, the full gradient).
 *   SGD: g = n grad J_i(x) = n grad D_i(x) + beta grad S(x); ghat_i / ghat are
 *     not used (may be null) on the dense path.
 * With state->counts (the zero-count-aware data term, as for pet_svrg_epoch)
 * the line kernels walk only the bins with counts, which give
 * h_i(x) = -P_i^T[mult y / ybar] with grad D_i = P_i^T mult + h_i:
 *   SAGA's table then holds h_i + (beta/n) grad S (the P_i^T mult cancel in
 *     grad J_i - T_i) and state->ghat holds its sum plus state->sens;
 *   SGD needs state->ghat_i: at state->k == 0 it receives the subset
 *     sensitivities P_i^T mult (one dense back projection per subset), which
 *     later epochs of the same state reuse.
 * Iterates agree with the dense path up to rounding.
 * x_snap and omega are not used.  A state serves one estimator: the SVRG
 * snapshot table (data gradients only) is not a SAGA table.  Same argument
 * rules and errors as pet_svrg_epoch. */
pet_status pet_saga_epoch(pet_geom g, pet_svrg_state *state, float *x, const int32_t *subset_seq,
                          const float *tau, const uint8_t *update_pc, double *objective_out,
                          void *stream);
pet_status pet_sgd_epoch(pet_geom g, pet_svrg_state *state, float *x, const int32_t *subset_seq,
                         const float *tau, const uint8_t *update_pc, double *objective_out,
                         void *stream);

/* Reverse mode (unrolled reconstruction) -----------------------------------
 * Derivatives for differentiating through pet_svrg_epoch (Algorithm 1 with the
 * clipped step of eq. (sgm)); the second derivatives of the data term follow
 * from eq. (template) with d(s, t) of Section 2, those of the prior from
 * Appendix A.
 *
 * Data-term Hessian-vector product of one subset (-1: all):
 * hv_out (+)= P^T [mult^2 y / ybar^2 (mult P v)] with ybar = mult P x + add
 * (bins with y = 0 contribute 0).  ybar_work: caller-owned device scratch of
 * n_bins floats; the subset's bins receive ybar.  accumulate = 0 overwrites. */
pet_status pet_subset_hvp(pet_geom g, int subset, const float *x, const float *v, const void *y,
                          int y_dtype, const float *add, const float *mult, float *ybar_work,
                          float *hv_out, int accumulate, void *stream);

/* Prior Hessian-vector product: hv_out (+)= beta H_S(x) v with
 * H_ii = 2 sum_j w k_i k_j (2 x_j + eps)^2 / psi^3 and
 * H_ij = -2 w k_i k_j (2 x_i + eps)(2 x_j + eps) / psi^3 (neighbours j),
 * psi = x_i + x_j + gamma |x_i - x_j| + eps.  gdot_out (device double,
 * nullable) ACCUMULATES sum_i dS/dx_i v_i (unscaled by beta). */
pet_status pet_rdp_hvp(pet_geom g, const float *x, const float *kappa, const float w[27], float beta,
                       float gamma, float eps, const float *v, float *hv_out, int accumulate,
                       double *gdot_out, void *stream);

/* Vector-Jacobian product of the prior-aware preconditioner
 * D(x, beta) = (x + delta) / (sens + alpha beta h_S(x) (x + delta)) (h_S the
 * unscaled prior Hessian diagonal; D = 0 where the denominator is 0):
 * xbar += (dD/dx)^T Dbar (a 27-point stencil, since h_S couples neighbours),
 * betabar (device double) += <dD/dbeta, Dbar>. */
pet_status pet_precond_vjp(pet_geom g, const float *x, const float *sens, const float *kappa,
                           const float w[27], float beta, float gamma, float eps, float alpha,
                           float delta, const float *Dbar, float *xbar, double *betabar, void *stream);

/* Buffers of pet_svrg_epoch_vjp, all caller-owned device memory.
 *   x_start     the iterate at the epoch's first iteration (forward checkpoint)
 *   x_snap_src  the iterate of the snapshot iteration whose table the epoch
 *               uses, when the epoch does not start with a snapshot (else NULL)
 *   D_start     the preconditioner in effect before the epoch, when its first
 *               iteration does not update it (else NULL)
 *   xbar        in: dL/dx after the epoch; out: dL/dx_start
 *   Dbar, gbar_i [n_subsets][n_vox], gbar: adjoints of the preconditioner and
 *               of the snapshot table and sum in effect; carried from one
 *               epoch's call to the previous epoch's (start them at 0)
 *   betabar     device double, accumulates dL/dbeta
 *   xs [(n_subsets + 1) n_vox], est [n_subsets n_vox], ybar_work [n_bins],
 *   v [2 n_vox]: workspace. */
typedef struct {
    const float *x_start;
    const float *x_snap_src;
    const float *D_start;
    float *xbar;
    float *Dbar;
    float *gbar_i;
    float *gbar;
    double *betabar;
    float *xs;
    float *est;
    float *ybar_work;
    float *v;
} pet_svrg_vjp_bufs;

/* Reverse of one pet_svrg_epoch for a scalar loss L: with state->k at the
 * epoch's first iteration and the same subset_seq / tau / update_pc (host
 * arrays), recomputes the epoch from the checkpoint (keeping its iterates and
 * estimators), then sweeps the iterations backwards:
 *   u = xbar [x_next > 0];  Dbar += -tau u est;  v = -tau D u;  xbar = u
 *     + beta H_S(x) v + (n H_i(x) v, gbar_i -= n v, gbar += v)        regular
 *     + beta H_S(x) v + sum_q H_q(x) (gbar_q + gbar + v), gbar* = 0   snapshot
 *     + (dD/dx)^T Dbar, Dbar = 0                                    D update
 *   betabar += <grad S(x), v> (+ <dD/dbeta, Dbar> at a D update).
 * Preconditioner updates and snapshots must fall on the epoch's first
 * iteration (PET_E_ARG otherwise).  The state's ghat_i, ghat and D are
 * overwritten (recompute scratch); state->k is not advanced. */
pet_status pet_svrg_epoch_vjp(pet_geom g, const pet_svrg_state *state, pet_svrg_vjp_bufs *bufs,
                              const int32_t *subset_seq, const float *tau, const uint8_t *update_pc,
                              void *stream);

/* Batches of reconstructions ------------------------------------------------
 * Many independent reconstructions (members), each with its own geometry,
 * sizes, TOF setting, data, beta and number of subsets, advanced together by
 * preconditioned SVRG (Algorithm 1 with the clipped step of eq. (sgm)).
 * A round is one epoch of every member: step j of the round performs
 * iteration j of each member with j < n_subsets, as the same five launches
 * for the whole batch; the subset gradients of a step are one persistent
 * launch that takes (member, transaxial line) work items from a counter.  A
 * member's results equal those of pet_svrg_epoch on the same schedule up to
 * the summation order of the floating-point atomics. */
typedef struct pet_batch_s *pet_batch;

/* members: geometries (distinct handles, one device), SVRG states (as for
 * pet_svrg_epoch; their buffers and the images x[r] must stay alive, and the
 * geometries' scratch belongs to the batch while it runs) and images (device,
 * in/out).  Allocates gradient-sheet slots for every subset of every member,
 * the device schedule and a stream of its own.  At most 64 members.  A
 * member with a resolution model (psf_fwhm_mm > 0) passes its image through G
 * before the sheets and its gathered gradients through G after them, as
 * pet_svrg_epoch does; the extra passes are launched only when some member
 * has one. */
pet_status pet_batch_create(const pet_geom *geoms, pet_svrg_state *const *states, float *const *x,
                            int n_members, pet_batch *out);
pet_status pet_batch_destroy(pet_batch b);

/* n_rounds rounds.  subset_seq / tau / update_pc: HOST arrays holding, member
 * after member (creation order), n_rounds * n_subsets(member) entries each,
 * as for that member's consecutive pet_svrg_epoch calls.  Every member's
 * state->k must be a multiple of its n_subsets (PET_E_STATE) and advances by
 * n_subsets per round.  use_graph != 0: the launches of a round are captured
 * in a HIP graph on first use and replayed; the round's schedule is copied to
 * the device before each replay.  Ordered after prior work on `stream`; later
 * work on `stream` waits for the rounds. */
pet_status pet_batch_epochs(pet_batch b, int n_rounds, const int32_t *subset_seq, const float *tau,
                            const uint8_t *update_pc, int use_graph, void *stream);

/* One round: pet_batch_epochs with n_rounds = 1 (member r's schedule is its
 * n_subsets entries, members in creation order). */
pet_status pet_batch_epoch(pet_batch b, const int32_t *subset_seq, const float *tau, const uint8_t *update_pc,
                           int use_graph, void *stream);

/* Launch-shape autotuner: times the batched subset-gradient step (subset 0 of
 * every member) for workgroup sizes of 16, 12 and 8 waves, one or two
 * workgroups per compute unit and two work-item orders (longest lines
 * first / creation order), and keeps the fastest.  Touches only scratch
 * sheets.  config_out (host int[3], nullable): workgroups, waves, order;
 * best_ms_out (host, nullable): its time. */
pet_status pet_batch_autotune(pet_batch b, int *config_out, double *best_ms_out, void *stream);

/* Sets the launch shape of the batched subset-gradient step by hand
 * (workgroups, waves per workgroup 1..16, order 0 = longest lines first,
 * 1 = creation order); PET_E_ARG if the sheets do not fit. */
pet_status pet_batch_set_launch(pet_batch b, int workgroups, int waves, int order);

/* Debug checks -------------------------------------------------------------
 * pet_geom_set_flags(g, PET_CHECK) makes the entry points of this handle check
 * the domain of the problem on the device before their work and wait for the
 * result (the calls become synchronous), returning PET_E_DOMAIN with a message
 * naming the argument and the number of offending elements when
 *   an image x (or sens, kappa, a preconditioner's Hessian diagonal) has a
 *     negative or non-finite voxel: the prior R(x) is +inf for x < 0
 *     (eq. (prior)), the problem's domain is x >= 0;
 *   the counts y have a negative or non-finite bin: d(s, t) = +inf for t < 0
 *     (Section 1.2);
 *   the background add is negative, non-finite, or 0 in a bin with y > 0
 *     (add NULL with any y > 0 counts as such): with x >= 0 and mult >= 0,
 *     add > 0 is what keeps s = mult P x + add > 0 where t > 0, and
 *     d(s, t) = +inf for s <= 0 with t > 0 (Section 1.2);
 *   mult has a negative or non-finite entry; a sinogram passed to pet_back,
 *     or pet_fwd's add, has a non-finite entry.
 * Whole arrays are checked (all views).  Entry points that produce the FP64
 * objective (pet_objective, and the epoch functions given objective_out) then
 * wait for it and return PET_E_NUMERIC if it is not finite.  Checked:
 * pet_fwd, pet_back, pet_subset_grad(_noalloc), pet_rdp_grad_hessdiag,
 * pet_precond, pet_osem_epoch, pet_objective, pet_svrg_epoch(_ex),
 * pet_saga_epoch, pet_sgd_epoch, pet_subset_hvp.  Without the flag (the
 * default) nothing is checked and values outside the domain give unspecified
 * results.
 *
 * PET_SMALL_CHUNKS caps the chunks of the zero-count-aware kernels at 16 bins
 * of a line (normally what the LDS holds, thousands), so that tests can run
 * their chunked path on small problems; results agree up to rounding.
 * PET_SIGNED_SHEETS makes the zero-count-aware kernels accumulate their
 * fixed-point gradient sheets in the signed form that they otherwise take
 * only for chunks with a negative mean (outside the domain), so that tests
 * can run it on well-conditioned data; results agree up to rounding.
 * flags: a combination of PET_CHECK, PET_SMALL_CHUNKS and PET_SIGNED_SHEETS
 * (PET_E_ARG for other bits). */
enum { PET_CHECK = 1, PET_SMALL_CHUNKS = 2, PET_SIGNED_SHEETS = 4 };
pet_status pet_geom_set_flags(pet_geom g, unsigned flags);

/* Instrumentation --------------------------------------------------------
 * Work of the line kernels on `subset` (-1: all), exactly as they traverse it:
 * out[0] = Joseph samples, out[1] = sample-TOF-bin pairs with nonzero weight
 * support (= samples without TOF).  out: device doubles[2]. */
pet_status pet_work_counts(pet_geom g, int subset, double *out, void *stream);

/* Time every line-kernel launch of a handle with a HIP event pair recorded on
 * the launch stream (enable != 0), and read the accumulated time and count of
 * one kernel (PET_KERNEL_*) since the last read; reading synchronises on the
 * recorded events and resets that kernel's record. */
enum { PET_KERNEL_FWD = 0, PET_KERNEL_BACK = 1, PET_KERNEL_GRAD = 2, PET_KERNEL_EM = 3, PET_KERNEL_OBJ = 4,
       PET_KERNEL_HVP = 6, PET_KERNEL_COUNTS = 7 /* zero-count-aware line kernel, every mode */,
       PET_KERNEL_GATHER = 8 /* gather adjoint of pet_back */ };
pet_status pet_profile_enable(pet_geom g, int enable);
pet_status pet_profile_read(pet_geom g, int kernel, double *total_ms, int64_t *launches);

const char *pet_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
