// Internal declarations of the gfx950 PET library: device geometry tables,
// kernel argument blocks and launch helpers shared by the host entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/pet.h"

namespace pet {

// Padding (voxels) of the transposed "sheet" images on each side of the
// transaxial interpolation axis and of z.  Samples may sit up to 1.5 voxels
// outside the grid (conservative sample ranges); padded zeros make them exact.
constexpr int PADA = 2;
constexpr int PADZ = 2;
constexpr int NT_MAX = 32;     // TOF bins supported
constexpr int NT_BLK = 16;     // TOF bins a lane holds in registers at once
constexpr int NINT_MAX = 2 * NT_MAX - 1;  // intervals between the 2 n_tof window edges
constexpr int NT_BLOCK = 1024;  // non-TOF line kernel: most threads per workgroup (16 waves)
constexpr int IMG_BLOCK = 256;  // image-space kernels: threads per workgroup
constexpr int TOF_MAX_WAVES = 16;  // TOF line kernel: at most 16 segment waves
constexpr int WS_MAX = 8;       // TOF bins overlapping one point
// per-wave TOF interval cut indices: n_int + 1 of them, padded to 4
__host__ __device__ inline int tof_cuts_pad(int n_int) { return (n_int + 1 + 3) & ~3; }

// One transaxial line (view, radial): sample i along the principal axis m sits
// at lambda(i) = lam0 + i dlam on the LOR; its coordinate along the other
// transaxial axis, in voxel units, is xa0 + i dxa.  Samples outside
// [i_lo, i_hi] cannot touch the grid (i_lo > i_hi: line misses the image).
struct LineP {
    float lam0, dlam, xa0, dxa;
    float vm_um;  // v_m / |u_m|: step length = vm_um * |u|
    float lt2;    // squared transaxial length of u
    int16_t i_lo, i_hi;
    int32_t axis; // principal axis: 0 = x, 1 = y
};
static_assert(sizeof(LineP) == 32, "LineP layout");

// One plane (ring pair): z index coordinate of a sample is zb + lambda zs.
struct PlaneP {
    float zb, zs, dz2;
    int32_t seg;
};

// One segment (ring difference): planes p0 .. p0 + np - 1, all with the same
// squared axial extent dz2 (so the same |u| on a given line).
struct SegP {
    int32_t p0, np;
    float dz2;
    int32_t pad;
};

// TOF interval table.  The t axis (signed distance from the LOR centre) is cut
// at every support edge t_b -/+ (bin/2 + nsig sigma) of a bin's weight; inside
// interval s the bins with nonzero weight are bf[s] .. bf[s] + na[s] - 1.
struct TofTable {
    int n_tof;
    int n_int;
    float edge[NINT_MAX + 1];
    int bf[NINT_MAX];
    int na[NINT_MAX];
    float tb[NT_MAX];
    float half_bin;         // tof_bin / 2
    float inv_sqrt2_sigma;  // 1 / (sqrt2 sigma)
    float erf_clamp;        // nsig / sqrt2: truncation of the Gaussian kernel
};

enum Mode { M_FWD = 0, M_BACK = 1, M_GRAD = 2, M_EM = 3, M_OBJ = 4, M_COUNT = 5, M_HVP = 6, M_NMODES = 7 };

struct ProjArgs {
    const LineP *lines;
    const PlaneP *planes;
    const int *views;
    const SegP *segs;
    int n_rad, n_planes, nx, ny, nz, rz;
    int n_seg, rows_max, ws, tstride;  // TOF: segments, sheet rows (max), bins per point, table row stride
    // transposed padded images: T[0] principal x: [nx][ny+4][nz+4]; T[1] principal y: [ny][nx+4][nz+4]
    const float *T0, *T1;
    float *G0, *G1;
    const void *y;
    int y_dtype;
    const float *add, *mult, *sino;
    const float *ybar;  // M_HVP: mean data mult P x + add at the linearisation point
    float *out;
    double *partial;  // one double per block (KL sum), or null
    TofTable tof;
    // line kernels: workgroup b takes line order[b], the launch's lines
    // longest first (the hardware dispatches workgroups in index order)
    const int *order;
    // non-TOF line kernel, M_BACK on a TOF geometry: each sample weighted by
    // the sum of its TOF bins' weights (the backprojection of mult alone)
    int tof_fold;
};

// ---- zero-count-aware data term (counts.hip) --------------------------------
// One bin with y > 0 of a transaxial line, with what the counts kernel needs
// of its LOR (computed once, at compaction): the sample rows that reach the
// grid and the bin's TOF window, the TOF table position and the padded axial
// position as affine functions of the row, mult times the step length, the
// count and the background.
struct CountRec {
    int16_t is, ie;  // sample rows [is, ie] (empty: is > ie)
    float pA, pB;    // TOF table position of row i: pA i + pB (0 without TOF)
    float zA, zB;    // padded axial position of row i: zA i + zB
    float me;        // mult * ell, ell the LOR's step length (mm)
    float y, add;
};
static_assert(sizeof(CountRec) == 32, "CountRec layout");
constexpr int NW_TAB = 4096;    // intervals of the tabulated TOF weight W(d)
constexpr int CNT_BLOCK = 512;   // threads per workgroup of the counts line kernel
constexpr int CNT_QCAP = 2048;   // bins per chunk of the counts line kernel (four rounds of one bin per thread)
constexpr int CU_LDS_BYTES = 160 * 1024;  // LDS of one gfx950 CU

// One line with counts as a workgroup of the counts kernel sees it: the
// line's geometry and the range of its bins in the item array.
struct CountLine {
    LineP L;
    int64_t i0;    // first item
    int32_t n;     // items
    int32_t slot;  // subset of the line's view: its gradient sheets in a launch over all subsets
};
static_assert(sizeof(CountLine) == 48, "CountLine layout");

struct CountArgs {
    const CountRec *items;
    const CountLine *desc;    // the launch's lines (workgroup b takes desc[b])
    const float2 *wtab;       // TOF: (W_k, W_{k+1} - W_k) at the table's NW_TAB nodes
    int sheet_floats, tab_floats;  // LDS layout: sheet region, TOF table (floats)
    int nw, n_tof;
    float wD;                 // support of W: |d| <= wD
    float inv_dx, pos0, pos_max;  // table position of d: d * inv_dx + pos0, clamped to [0, pos_max]
    int q_cap;                // bins per chunk of a line (at most CNT_QCAP with M_GRAD)
    int force_signed;         // signed fixed-point sheets for every chunk (tests)
    int64_t slot_floats;      // 0, or the stride of per-subset gradient sheets (G0, G1 + slot * stride)
};

// ---- batches of reconstructions -------------------------------------------
constexpr int PSF_RMAX = 16;  // resolution model: kernel radius limit (voxels)
// One axis of the separable resolution kernel: weights w[0..r] of offsets 0..r
// (symmetric), and the axis (0 = x, 1 = y, 2 = z).
struct PsfAxis {
    int r, axis;
    float w[PSF_RMAX + 1];
};

constexpr int BATCH_MAX = 64;
enum BStepFlags { B_ACTIVE = 1, B_SNAP = 2, B_UPDATE = 4 };

// What one member does at one step of a round (device schedule).
struct BStep {
    int subset;
    float tau;
    int flags;
    int pad;
};

// One member of a batch as the batched kernels see it.
struct BMember {
    ProjArgs pa;               // geometry tables, image sheets, data; G0/G1 = slot 0
    const int *views;          // [n_sub + 1][views_stride] view lists (last row: all views)
    const int *sub_nviews;     // views per subset
    int views_stride, n_sub, n_views, is_tof, tof_waves, nx, ny, nz;
    int64_t n_vox, g_slot;     // voxels; floats per gradient-sheet slot (G1 = G0 + t0 within a slot)
    int64_t t0_elems;
    // SVRG state (Algorithm 1)
    float *x, *xtmp, *g, *ghat_i, *D;
    double *ghat;
    const float *sens, *kappa;
    float w[27];
    float beta, gamma, eps, alpha, delta, n_subf;
    const BStep *steps;        // [max_steps] of the current round
    // resolution model (psf_passes = 0: none): axis passes, and two image-sized
    // work buffers for G x
    int psf_passes;
    PsfAxis psf[3];
    float *psf_a, *psf_b;
};

}  // namespace pet


struct pet_geom_s {
    pet_geom_desc d;
    // resolution model: passes (x, y[, z]) and two image-sized work buffers
    int psf_passes = 0;
    pet::PsfAxis psf[3]{};
    float *psf_a = nullptr, *psf_b = nullptr;
    int device;
    int n_planes;
    int64_t n_vox;
    int max_views;                      // views per subset (max)
    std::vector<std::vector<int>> subset_views;
    std::vector<int> seg_of_plane;
    // device tables
    pet::LineP *lines = nullptr;
    pet::PlaneP *planes = nullptr;
    pet::SegP *segs = nullptr;
    pet::SegP *gsegs = nullptr;         // plain segments in plane order (gather adjoint)
    int n_gseg = 0;
    int n_seg = 0, rows_max = 0, tof_ws = 0, tof_tstride = 0, tof_waves = 0;
    int nt_threads = pet::NT_BLOCK;     // non-TOF line kernel: threads per workgroup
    int *views_dev = nullptr;           // [n_subsets + 1][max(max_views, n_views)]; last row: all views
    int views_stride = 0;
    // line launches: per subset (then all views) the subset's lines, longest
    // first, at line_order + order_off[row]
    int *line_order = nullptr;
    std::vector<int64_t> order_off;
    pet::TofTable tof{};
    // TOF weight of a point at signed distance d from a bin centre,
    // W(d) = 1/2 [E(bin/2 - d) - E(-bin/2 - d)] (E the clamped erf), at NW_TAB + 1
    // nodes over its support |d| <= wD, as (W_k, W_{k+1} - W_k) pairs
    float2 *wtab = nullptr;   // TOF weight table: (W_k, W_{k+1} - W_k) at NW_TAB nodes (gather adjoint)
    float *wtabf = nullptr;   // and W at the NW_TAB + 1 nodes (counts kernels)
    float wD = 0.f;
    size_t lds_bytes = 0;
    size_t max_lds = 0;                 // the device's LDS limit per workgroup
    // scratch arena
    float *T0 = nullptr, *T1 = nullptr, *G0 = nullptr, *G1 = nullptr;
    size_t t0_elems = 0, t1_elems = 0;
    float *g = nullptr, *xtmp = nullptr, *grad = nullptr, *hess = nullptr, *num = nullptr, *sensi = nullptr;
    double *partial = nullptr;
    size_t n_partial = 0;
    double *dscratch = nullptr;         // a few device doubles
    float *fscratch = nullptr;          // a few device floats
    // debug flags (PET_CHECK) and the device counters of the domain checks
    unsigned flags = 0;
    unsigned *check_counts = nullptr;
    // optional HIP-event timing of the line kernels, per mode
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events[pet::M_NMODES + 2];  // then: counts, gather kernels
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pool;
};

// Compacted bins with counts y > 0 of one data set on one geometry
// (pet_counts_create).
struct pet_counts_s {
    pet_geom_s *g = nullptr;
    int n_subsets = 0;
    int64_t n_items = 0;
    pet::CountRec *items = nullptr;   // per line, TOF bin major
    int64_t *line_off = nullptr;      // [n_lines + 1]
    int *lines = nullptr;             // per subset (then all views): lines with counts, most first
    pet::CountLine *desc = nullptr;   // the same lines with their geometry and item ranges
    std::vector<int64_t> lines_off;        // [n_subsets + 2] offsets into lines
    std::vector<int64_t> items_per_subset; // [n_subsets + 1]
    std::vector<double> sum_y, sum_add;    // [n_subsets + 1] over every bin of the subset (then all)
    // snapshot passes in one launch: n_subsets pairs of gradient sheets
    // (G0 then G1 of each, slot_floats apart), allocated at creation where the
    // fused step serves the geometry (else null), interiors zero between
    // snapshots
    float *slots = nullptr;
    int64_t slot_floats = 0;
};

namespace pet {

constexpr int PROF_COUNTS = M_NMODES;      // profiling slot of the counts line kernel
constexpr int PROF_GATHER = M_NMODES + 1;  // and of the gather adjoint

// error state (api.cpp)
pet_status fail(pet_status s, const std::string &msg);
pet_status hip_check(hipError_t e, const char *what);

// projector launches (proj.hip)
hipError_t launch_line_kernel(pet_geom_s *g, int mode, int subset, const ProjArgs &a, hipStream_t s);
// persistent batched subset-gradient line kernel over the work items of one step
hipError_t launch_line_batched(const BMember *mem, const int *order, int n_mem, int step, int *counter, int blocks,
                               int waves, size_t lds, hipStream_t s);
// raise the batched kernel's dynamic-LDS limit (outside any stream capture)
hipError_t prime_line_batched(size_t lds);
// line-kernel argument block of a geometry (all views), and of one subset (-1: all views)
ProjArgs geom_proj_args(pet_geom_s *g);
ProjArgs subset_proj_args(pet_geom_s *g, int subset);
// device address of the allocation-free entry point's static scratch array on
// `device` (looked up once per device; noalloc.cpp)
pet_status noalloc_scratch(int device, void **out);
// workgroups of a line launch of `subset` (-1: all views), one per line, each
// writing one FP64 partial
int n_line_blocks(const pet_geom_s *g, int subset);

// zero-count-aware line kernels (counts.hip): mode M_GRAD (gradient sheets
// receive -P^T[mult y / ybar], block partials of sum y log(y / ybar)) or M_OBJ
// (partials only), over the lines with counts of `subset` (-1: all)
// slot_floats > 0 (subset -1 only): each line's shares go to the sheets of
// its view's subset, a.G0 / a.G1 + slot * slot_floats
hipError_t launch_line_counts(pet_geom_s *g, const pet_counts_s *c, int mode, int subset, const ProjArgs &a,
                              hipStream_t s, int64_t slot_floats = 0);
int counts_blocks(const pet_counts_s *c, int subset);
size_t counts_lds_bytes(const pet_geom_s *g, int mode);

// cell-driven (gather) adjoint into the gradient sheets (gather.hip)
hipError_t launch_line_gather(pet_geom_s *g, int subset, const ProjArgs &a, hipStream_t s);
size_t gather_lds_bytes(const pet_geom_s *g);

// image kernels (image.hip)
// Work buffers of the sheet conversions: transposed image sheets T0 / T1,
// gradient sheets G0 / G1 (t0_elems / t1_elems floats each) and, with a
// resolution model, two image-sized buffers.  A handle's own are geom_bufs(g).
struct SheetBufs {
    float *T0, *T1, *G0, *G1, *psf_a, *psf_b;
};
SheetBufs geom_bufs(const pet_geom_s *g);
hipError_t launch_to_sheets_b(const pet_geom_s *g, const SheetBufs &w, const float *x, hipStream_t s);
hipError_t launch_zero_sheets_b(const pet_geom_s *g, const SheetBufs &w, hipStream_t s);
hipError_t launch_from_sheets_b(const pet_geom_s *g, const SheetBufs &w, float *out, int accumulate, hipStream_t s);
hipError_t launch_clear_image_sheets(const pet_geom_s *g, const SheetBufs &w, hipStream_t s);
hipError_t launch_psf_b(const pet_geom_s *g, const SheetBufs &w, const float *in, float *out, int accumulate,
                        hipStream_t s);
hipError_t launch_to_sheets(const pet_geom_s *g, const float *x, hipStream_t s);
hipError_t launch_zero_sheets(const pet_geom_s *g, hipStream_t s);
hipError_t launch_from_sheets(const pet_geom_s *g, float *out, int accumulate, hipStream_t s);
hipError_t launch_rdp(const pet_geom_s *g, const float *x, const float *kappa, const float *w27,
                      float beta, float gamma, float eps, float *grad, float *hess, double *partial,
                      hipStream_t s);
hipError_t launch_precond(const pet_geom_s *g, const float *x, const float *sens, const float *hess,
                          float alpha, float delta, float *D, hipStream_t s);
hipError_t launch_reduce_sum(const double *partial, int n, double *out, int accumulate, hipStream_t s);
hipError_t launch_osem_update(const pet_geom_s *g, float *x, const float *num, const float *sens, hipStream_t s,
                              float sgn = 1.f);
hipError_t launch_max(const pet_geom_s *g, const float *x, float *out, hipStream_t s);
// domain checks (debug mode, PET_CHECK): count violations of a condition
enum DomainKind {
    CHK_NONNEG = 0,  // finite and >= 0 (images, mult, sensitivities)
    CHK_FINITE = 1,  // finite
    CHK_COUNTS = 2,  // counts y: finite and >= 0
    CHK_ADD = 3,     // background: finite, >= 0, and > 0 where y > 0
    CHK_NO_ADD = 4,  // no background given: every y must be 0
};
constexpr int CHECK_SLOTS = 8;  // counters of one call's checks
hipError_t launch_domain_count(const float *p, int kind, int64_t n, const void *y, int ydt, unsigned *count,
                               hipStream_t s);
hipError_t launch_fill_u32(unsigned *p, int n, unsigned val, hipStream_t s);
// PET_CHECK set on the handle, and the checks of an entry point's image and
// data with the counters at `counts` (api.cpp)
bool checking(const pet_geom_s *g);
pet_status check_data(pet_geom_s *g, unsigned *counts, hipStream_t s, const char *fn, const float *x, const void *y,
                      int ydt, const float *add, const float *mult);
hipError_t launch_svrg_step(const pet_geom_s *g, const float *x, const float *kappa, const float *w27, float beta,
                            float gamma, float eps, int update_pc, const float *sens, float alpha, float delta,
                            float *D, int snapshot, const float *gi, const float *ghat_i, const double *ghat,
                            float n_sub, float tau, float *x_out, float *est_out, hipStream_t s);
bool step_tile_ok(const pet_geom_s *g);
hipError_t launch_svrg_step_tile(const pet_geom_s *g, const float *x, const float *w27, float beta, float gamma,
                                 float eps, int update_pc, const float *sens, float alpha, float delta, float *D,
                                 int snapshot, const float *ghat_i, const double *ghat, float w, float tau,
                                 const double *tau_bb, int bb_store, float *g_prev, float *x_out, hipStream_t s);
hipError_t launch_svrg_step_ex(const pet_geom_s *g, const float *x, const float *kappa, const float *w27, float beta,
                               float gamma, float eps, int update_pc, const float *sens, float alpha, float delta,
                               float *D, int snapshot, const float *gi, const float *ghat_i, const double *ghat,
                               float w, float tau, const double *tau_bb, int bb_mode, const float *x_snap,
                               float *g_prev, float *grad_out, float *x_out, hipStream_t s);
hipError_t launch_bb_finish(const pet_geom_s *g, double *bb, hipStream_t s);
hipError_t launch_bb_init(double *bb, hipStream_t s);
hipError_t launch_step_stored(const pet_geom_s *g, const float *x, const float *D, const float *est, float tau,
                              const double *tau_bb, float *x_out, hipStream_t s);
hipError_t launch_subset_norms(const pet_geom_s *g, const float *ghat_i, const float *bgrad, double *out,
                               hipStream_t s);
enum SgmEstimator { SGM_SAGA = 1, SGM_SGD = 2 };
hipError_t launch_saga_table_prior(const pet_geom_s *g, float *table, double *table_sum, const float *bgrad,
                                  hipStream_t s, const float *base = nullptr);
hipError_t launch_sgm_step(const pet_geom_s *g, int estimator, const float *x, const float *kappa, const float *w27,
                           float beta, float gamma, float eps, int update_pc, const float *sens, float alpha,
                           float delta, float *D, int first, const float *gi, float *table_i, double *table_sum,
                           float n_sub, float tau, float *x_out, hipStream_t s);
// ghat_i <- the gradient sheets' image; ghat (+)= it in FP64 (first: ghat = base + it, base nullable)
// clear (only without a resolution model): zero the gradient sheets' cells
// after reading them
// (G0, G1: other gradient sheets than the handle's, nullable)
hipError_t launch_snapshot_accum(const pet_geom_s *g, float *ghat_i, double *ghat, float *gcopy, int first,
                                 hipStream_t s, const float *base = nullptr, int clear = 0, float *G0 = nullptr,
                                 float *G1 = nullptr);
// the same for the n_sub pairs of sheets (G0, G1 + q stride) of a one-launch
// snapshot pass, in one launch: ghat_i[q] for every q, ghat = base + their sum
// in FP64 (subset order), every pair's cells cleared after reading
hipError_t launch_snapshot_accum_slots(const pet_geom_s *g, float *G0, float *G1, int64_t stride, int n_sub,
                                       float *ghat_i, double *ghat, const float *base, hipStream_t s);
// FP64 dot product into *out (accumulate: add), through `partial`
int dot_blocks(int64_t n);
hipError_t launch_dot(const float *a, const float *b, int64_t n, double *partial, double *out, int accumulate,
                      hipStream_t s);
hipError_t launch_add_scalar(double *out, double val, hipStream_t s);
// resolution model G (no-op pass-through when the geometry has none)
hipError_t launch_psf(const pet_geom_s *g, const float *in, float *out, int accumulate, hipStream_t s);
int rdp_blocks(const pet_geom_s *g);
hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t s);
hipError_t launch_fill(float *dst, int64_t n, float val, hipStream_t s);
// batched image-space kernels (batch.hip): one launch each for all active members of a step
// psf_max: the most resolution-model passes of any member (0: no member has one)
hipError_t launch_b_prep(const BMember *mem, int n_mem, int step, int *counter, int psf_max, hipStream_t s);
hipError_t launch_b_gather(const BMember *mem, int n_mem, int step, int psf_max, hipStream_t s);
hipError_t launch_b_step(const BMember *mem, int n_mem, int step, hipStream_t s);
hipError_t launch_b_commit(const BMember *mem, int n_mem, int step, hipStream_t s);
// reverse-mode kernels (adjoint.hip)
int adj_blocks(const pet_geom_s *g);
hipError_t launch_rdp_hvp(const pet_geom_s *g, const float *x, const float *kappa, const float *w27, float beta,
                          float gamma, float eps, const float *v, float *out, int accumulate, double *partial,
                          hipStream_t s);
hipError_t launch_precond_vjp(const pet_geom_s *g, const float *x, const float *kappa, const float *w27, float beta,
                              float gamma, float eps, const float *sens, float alpha, float delta,
                              const float *Dbar, float *xbar, float *e_tmp, double *partial, hipStream_t s);
hipError_t launch_step_vjp(const pet_geom_s *g, const float *x_next, const float *D, const float *est, float tau,
                           float *xbar, float *Dbar, float *v, hipStream_t s);
hipError_t launch_lincomb(float *out, float ca, const float *a, float cb, const float *b, int64_t n, hipStream_t s);

}  // namespace pet
