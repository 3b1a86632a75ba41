// C entry points of the gfx950 PET library (declared in include/pet.h).
// Argument checking happens here, before anything is enqueued; the work itself
// is a sequence of kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <initializer_list>
#include <string>
#include <utility>

#include "pet_internal.h"

namespace pet {

thread_local std::string g_last_error;

pet_status fail(pet_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

pet_status hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return PET_OK;
    return fail(PET_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

bool valid_subset(pet_geom g, int subset) { return subset >= -1 && subset < g->d.n_subsets; }
bool valid_dtype(int dt) { return dt == PET_Y_F32 || dt == PET_Y_U16 || dt == PET_Y_U8; }

const int *views_of(pet_geom g, int subset) {
    int row = subset < 0 ? g->d.n_subsets : subset;
    return g->views_dev + (size_t)row * g->views_stride;
}

ProjArgs base_args(pet_geom g, int subset) {
    ProjArgs a{};
    a.lines = g->lines;
    a.planes = g->planes;
    a.views = views_of(g, subset);
    a.segs = g->segs;
    a.n_seg = g->n_seg;
    a.rows_max = g->rows_max;
    a.ws = g->tof_ws;
    a.tstride = g->tof_tstride;
    a.n_rad = g->d.n_rad;
    a.n_planes = g->n_planes;
    a.nx = g->d.nx;
    a.ny = g->d.ny;
    a.nz = g->d.nz;
    a.rz = g->d.nz + 2 * PADZ;
    a.T0 = g->T0;
    a.T1 = g->T1;
    a.G0 = g->G0;
    a.G1 = g->G1;
    a.tof = g->tof;
    a.order = g->line_order + g->order_off[subset < 0 ? g->d.n_subsets : subset];
    return a;
}

// ---- debug checks (PET_CHECK) ---------------------------------------------
// One condition on one argument: p (float array of n elements; null for the
// conditions on y alone) and the message that names it.
struct Dom {
    const float *p;
    int kind;
    int64_t n;
    const char *what;
};

// Counts the violations of every condition on the device (one counter each),
// waits for them and returns PET_E_DOMAIN naming the first violated one.
// Conditions on a null array are skipped (except those on y alone).
pet_status check_domain(unsigned *counts, hipStream_t s, const char *fn, const void *y, int ydt,
                        std::initializer_list<Dom> list) {
    hipError_t e = launch_fill_u32(counts, CHECK_SLOTS, 0u, s);
    int k = 0;
    for (const Dom &d : list) {
        const bool y_only = d.kind == CHK_COUNTS || d.kind == CHK_NO_ADD;
        if (e == hipSuccess && k < CHECK_SLOTS && (d.p || (y_only && y)))
            e = launch_domain_count(d.p, d.kind, d.n, y, ydt, counts + k, s);
        ++k;
    }
    unsigned h[CHECK_SLOTS] = {};
    if (e == hipSuccess) e = hipMemcpyAsync(h, counts, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_check(e, fn);
    k = 0;
    for (const Dom &d : list) {
        if (k < CHECK_SLOTS && h[k]) return fail(PET_E_DOMAIN, std::string(fn) + ": " + std::to_string(h[k]) + " " + d.what);
        ++k;
    }
    return PET_OK;
}

constexpr const char *MSG_X = "image voxels are negative or not finite (the prior R(x) is +inf for x < 0, eq. (prior))";
constexpr const char *MSG_Y = "count bins are negative or not finite (d(s, t) = +inf for t < 0, Section 1.2)";
constexpr const char *MSG_ADD = "background bins are negative, not finite, or 0 where y > 0 (r > 0 keeps d(s, t) "
                                "finite where t > 0, Section 1.2)";
constexpr const char *MSG_NO_ADD = "bins have counts y > 0 but no background was given (r > 0 keeps d(s, t) finite "
                                   "where t > 0, Section 1.2)";
constexpr const char *MSG_MULT = "multiplicative factors are negative or not finite";

}  // namespace

// Checks of an entry point's image x and data (y, add, mult), with the
// counters at `counts` (CHECK_SLOTS of them).
pet_status check_data(pet_geom g, unsigned *counts, hipStream_t s, const char *fn, const float *x, const void *y,
                      int ydt, const float *add, const float *mult) {
    int64_t nb = 0, nl = 0;
    pet_geom_info(g, -1, &nb, &nl, nullptr);
    return check_domain(counts, s, fn, y, ydt,
                        {{x, CHK_NONNEG, g->n_vox, MSG_X},
                         {nullptr, CHK_COUNTS, nb, MSG_Y},
                         {add, add ? CHK_ADD : CHK_NO_ADD, nb, add ? MSG_ADD : MSG_NO_ADD},
                         {mult, CHK_NONNEG, nl, MSG_MULT}});
}

namespace {

// PET_CHECK: waits for a device FP64 objective and returns PET_E_NUMERIC if it
// is not finite.
pet_status check_numeric(hipStream_t s, const double *val, const char *fn) {
    double h = 0.0;
    hipError_t e = hipMemcpyAsync(&h, val, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_check(e, fn);
    if (!std::isfinite(h)) return fail(PET_E_NUMERIC, std::string(fn) + ": the FP64 objective is not finite");
    return PET_OK;
}

}  // namespace

bool checking(const pet_geom_s *g) { return (g->flags & PET_CHECK) != 0; }

namespace {

// Data-term gradient of one subset into the gradient sheets (G0, G1); the
// image sheets must already hold x.  Optionally FP64 KL sum into kl_out.
hipError_t subset_grad_sheets(pet_geom g, int subset, const void *y, int dt, const float *add, const float *mult,
                              double *kl_out, int kl_accumulate, hipStream_t s, bool zeroed = false) {
    hipError_t e = zeroed ? hipSuccess : launch_zero_sheets(g, s);
    if (e != hipSuccess) return e;
    ProjArgs a = base_args(g, subset);
    a.y = y;
    a.y_dtype = dt;
    a.add = add;
    a.mult = mult;
    a.partial = kl_out ? g->partial : nullptr;
    e = launch_line_kernel(g, M_GRAD, subset, a, s);
    if (e != hipSuccess || !kl_out) return e;
    return launch_reduce_sum(g->partial, n_line_blocks(g, subset), kl_out, kl_accumulate, s);
}

hipError_t objective_impl(pet_geom g, const float *x, const void *y, int dt, const float *add, const float *mult,
                          const float *kappa, const float *w27, float beta, float gamma, float eps, double *out,
                          hipStream_t s) {
    hipError_t e = launch_to_sheets(g, x, s);
    if (e != hipSuccess) return e;
    ProjArgs a = base_args(g, -1);
    a.y = y;
    a.y_dtype = dt;
    a.add = add;
    a.mult = mult;
    a.partial = g->partial;
    e = launch_line_kernel(g, M_OBJ, -1, a, s);
    if (e == hipSuccess) e = launch_reduce_sum(g->partial, n_line_blocks(g, -1), out, 0, s);
    if (e == hipSuccess) e = launch_rdp(g, x, kappa, w27, beta, gamma, eps, nullptr, nullptr, g->partial, s);
    if (e == hipSuccess) e = launch_reduce_sum(g->partial, rdp_blocks(g), out, 1, s);
    return e;
}

// H_subset(x) v = P^T [mult^2 y / ybar^2 (mult P v)] with ybar = mult P x + add
// written to ybar_work (the subset's bins) on the way.
hipError_t hvp_impl(pet_geom g, int subset, const float *x, const float *v, const void *y, int dt, const float *add,
                    const float *mult, float *ybar_work, float *out, int accumulate, hipStream_t s) {
    hipError_t e = launch_to_sheets(g, x, s);
    ProjArgs a = base_args(g, subset);
    a.add = add;
    a.mult = mult;
    a.out = ybar_work;
    if (e == hipSuccess) e = launch_line_kernel(g, M_FWD, subset, a, s);
    if (e == hipSuccess) e = launch_to_sheets(g, v, s);
    if (e == hipSuccess) e = launch_zero_sheets(g, s);
    ProjArgs b = base_args(g, subset);
    b.y = y;
    b.y_dtype = dt;
    b.mult = mult;
    b.ybar = ybar_work;
    if (e == hipSuccess) e = launch_line_kernel(g, M_HVP, subset, b, s);
    if (e == hipSuccess) e = launch_from_sheets(g, out, accumulate, s);
    return e;
}

// Zero-count-aware part of one subset's gradient, -P_i^T[mult y / ybar], into
// the gradient sheets (the image sheets must hold x); optionally the FP64 sum
// of y log(y / ybar) over the subset's bins with counts into *ylogy_out.
hipError_t counts_grad_sheets(pet_geom g, const pet_counts_s *c, int subset, double *ylogy_out, hipStream_t s,
                              int accumulate = 0, bool zeroed = false) {
    hipError_t e = zeroed ? hipSuccess : launch_zero_sheets(g, s);
    ProjArgs a = base_args(g, subset);
    a.partial = ylogy_out ? g->partial : nullptr;
    if (e == hipSuccess) e = launch_line_counts(g, c, M_GRAD, subset, a, s);
    if (e == hipSuccess && ylogy_out)
        e = launch_reduce_sum(g->partial, counts_blocks(c, subset), ylogy_out, accumulate, s);
    return e;
}

// D(x) from the compacted bins, <sens, x> + sum add - sum y + sum y log(y / ybar)
// (all subsets), plus beta S(x), into *out.
hipError_t objective_counts_impl(pet_geom g, const pet_counts_s *c, const float *x, const float *sens,
                                 const float *kappa, const float *w27, float beta, float gamma, float eps,
                                 double *out, hipStream_t s) {
    hipError_t e = launch_to_sheets(g, x, s);
    ProjArgs a = base_args(g, -1);
    a.partial = g->partial;
    if (e == hipSuccess) e = launch_line_counts(g, c, M_OBJ, -1, a, s);
    if (e == hipSuccess) e = launch_reduce_sum(g->partial, counts_blocks(c, -1), out, 0, s);
    if (e == hipSuccess) e = launch_dot(sens, x, g->n_vox, g->partial, out, 1, s);
    if (e == hipSuccess) e = launch_add_scalar(out, c->sum_add[c->n_subsets] - c->sum_y[c->n_subsets], s);
    if (e == hipSuccess) e = launch_rdp(g, x, kappa, w27, beta, gamma, eps, nullptr, nullptr, g->partial, s);
    if (e == hipSuccess) e = launch_reduce_sum(g->partial, rdp_blocks(g), out, 1, s);
    return e;
}

}  // namespace

ProjArgs geom_proj_args(pet_geom_s *g) { return base_args(g, -1); }
ProjArgs subset_proj_args(pet_geom_s *g, int subset) { return base_args(g, subset); }

}  // namespace pet

using namespace pet;

extern "C" const char *pet_last_error(void) { return g_last_error.c_str(); }

extern "C" pet_status pet_fwd(pet_geom g, int subset, const float *x, const float *mult, const float *add, float *out,
                              void *stream) {
    if (!g || !x || !out) return fail(PET_E_ARG, "pet_fwd: null argument");
    if (!valid_subset(g, subset)) return fail(PET_E_ARG, "pet_fwd: subset out of range");
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        int64_t nb = 0, nl = 0;
        pet_geom_info(g, -1, &nb, &nl, nullptr);
        const pet_status st = check_domain(g->check_counts, s, "pet_fwd", nullptr, 0,
                                           {{x, CHK_NONNEG, g->n_vox, MSG_X},
                                            {add, CHK_FINITE, nb, "background bins are not finite"},
                                            {mult, CHK_NONNEG, nl, MSG_MULT}});
        if (st != PET_OK) return st;
    }
    hipError_t e = launch_to_sheets(g, x, s);
    if (e != hipSuccess) return hip_check(e, "pet_fwd");
    ProjArgs a = base_args(g, subset);
    a.add = add;
    a.mult = mult;
    a.out = out;
    return hip_check(launch_line_kernel(g, M_FWD, subset, a, s), "pet_fwd");
}

extern "C" pet_status pet_back(pet_geom g, int subset, const float *sino, const float *mult, float *x_out,
                               int accumulate, int algo, void *stream) {
    if (!g || !x_out) return fail(PET_E_ARG, "pet_back: null argument");
    if (!valid_subset(g, subset)) return fail(PET_E_ARG, "pet_back: subset out of range");
    if (algo != PET_BACK_AUTO && algo != PET_BACK_SCATTER && algo != PET_BACK_GATHER)
        return fail(PET_E_ARG, "pet_back: unknown algo");
    if (algo == PET_BACK_GATHER && gather_lds_bytes(g) > g->max_lds)
        return fail(PET_E_ARG, "pet_back: the gather's plane tables exceed the LDS for this geometry");
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        int64_t nb = 0, nl = 0;
        pet_geom_info(g, -1, &nb, &nl, nullptr);
        const pet_status st = check_domain(g->check_counts, s, "pet_back", nullptr, 0,
                                           {{sino, CHK_FINITE, nb, "sinogram bins are not finite"},
                                            {mult, CHK_NONNEG, nl, MSG_MULT}});
        if (st != PET_OK) return st;
    }
    hipError_t e = launch_zero_sheets(g, s);
    if (e != hipSuccess) return hip_check(e, "pet_back");
    ProjArgs a = base_args(g, subset);
    a.sino = sino;
    a.mult = mult;
    // PET_BACK_AUTO takes the scatter, the faster of the two on every measured geometry
    e = algo == PET_BACK_GATHER ? launch_line_gather(g, subset, a, s) : launch_line_kernel(g, M_BACK, subset, a, s);
    if (e == hipSuccess) e = launch_from_sheets(g, x_out, accumulate, s);
    return hip_check(e, "pet_back");
}

extern "C" pet_status pet_subset_grad(pet_geom g, int subset, const float *x, const void *y, int y_dtype,
                                      const float *add, const float *mult, float *grad_out, double *kl_out,
                                      void *stream) {
    if (!g || !x || !y || !grad_out) return fail(PET_E_ARG, "pet_subset_grad: null argument");
    if (!valid_subset(g, subset)) return fail(PET_E_ARG, "pet_subset_grad: subset out of range");
    if (!valid_dtype(y_dtype)) return fail(PET_E_ARG, "pet_subset_grad: bad y dtype");
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        const pet_status st = check_data(g, g->check_counts, s, "pet_subset_grad", x, y, y_dtype, add, mult);
        if (st != PET_OK) return st;
    }
    hipError_t e = launch_to_sheets(g, x, s);
    if (e == hipSuccess) e = subset_grad_sheets(g, subset, y, y_dtype, add, mult, kl_out, 0, s);
    if (e == hipSuccess) e = launch_from_sheets(g, grad_out, 0, s);
    return hip_check(e, "pet_subset_grad");
}

extern "C" pet_status pet_rdp_grad_hessdiag(pet_geom g, const float *x, const float *kappa, const float w[27],
                                            float beta, float gamma, float eps, float *grad_out, float *hessdiag_out,
                                            double *value_out, void *stream) {
    if (!g || !x || !w) return fail(PET_E_ARG, "pet_rdp_grad_hessdiag: null argument");
    if (!grad_out && !hessdiag_out && !value_out) return PET_OK;
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        const pet_status st = check_domain(g->check_counts, s, "pet_rdp_grad_hessdiag", nullptr, 0,
                                           {{x, CHK_NONNEG, g->n_vox, MSG_X},
                                            {kappa, CHK_NONNEG, g->n_vox, "kappa voxels are negative or not finite"}});
        if (st != PET_OK) return st;
    }
    hipError_t e = launch_rdp(g, x, kappa, w, beta, gamma, eps, grad_out, hessdiag_out, value_out ? g->partial : nullptr, s);
    if (e == hipSuccess && value_out) e = launch_reduce_sum(g->partial, rdp_blocks(g), value_out, 0, s);
    return hip_check(e, "pet_rdp_grad_hessdiag");
}

extern "C" pet_status pet_precond(pet_geom g, const float *x, const float *sens, const float *hessdiag, float alpha,
                                  float delta, float *D_out, void *stream) {
    if (!g || !x || !sens || !hessdiag || !D_out) return fail(PET_E_ARG, "pet_precond: null argument");
    if (checking(g)) {
        const pet_status st =
            check_domain(g->check_counts, (hipStream_t)stream, "pet_precond", nullptr, 0,
                         {{x, CHK_NONNEG, g->n_vox, MSG_X},
                          {sens, CHK_NONNEG, g->n_vox, "sensitivity voxels are negative or not finite"},
                          {hessdiag, CHK_NONNEG, g->n_vox, "Hessian-diagonal voxels are negative or not finite"}});
        if (st != PET_OK) return st;
    }
    return hip_check(launch_precond(g, x, sens, hessdiag, alpha, delta, D_out, (hipStream_t)stream), "pet_precond");
}

extern "C" pet_status pet_osem_epoch(pet_geom g, float *x, const void *y, int y_dtype, const float *add,
                                     const float *mult, const int32_t *order, float *xmax_out, void *stream) {
    if (!g || !x || !y || !order) return fail(PET_E_ARG, "pet_osem_epoch: null argument");
    if (!valid_dtype(y_dtype)) return fail(PET_E_ARG, "pet_osem_epoch: bad y dtype");
    for (int j = 0; j < g->d.n_subsets; ++j)
        if (order[j] < 0 || order[j] >= g->d.n_subsets) return fail(PET_E_ARG, "pet_osem_epoch: order entry out of range");
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        const pet_status st = check_data(g, g->check_counts, s, "pet_osem_epoch", x, y, y_dtype, add, mult);
        if (st != PET_OK) return st;
    }
    hipError_t e = hipSuccess;
    for (int j = 0; j < g->d.n_subsets && e == hipSuccess; ++j) {
        int i = order[j];
        // P_i^T mult
        e = launch_zero_sheets(g, s);
        ProjArgs a = base_args(g, i);
        a.mult = mult;
        if (e == hipSuccess) e = launch_line_kernel(g, M_BACK, i, a, s);
        if (e == hipSuccess) e = launch_from_sheets(g, g->sensi, 0, s);
        // P_i^T (mult y / ybar)
        if (e == hipSuccess) e = launch_to_sheets(g, x, s);
        if (e == hipSuccess) e = launch_zero_sheets(g, s);
        ProjArgs b = base_args(g, i);
        b.y = y;
        b.y_dtype = y_dtype;
        b.add = add;
        b.mult = mult;
        if (e == hipSuccess) e = launch_line_kernel(g, M_EM, i, b, s);
        if (e == hipSuccess) e = launch_from_sheets(g, g->num, 0, s);
        if (e == hipSuccess) e = launch_osem_update(g, x, g->num, g->sensi, s);
    }
    if (e == hipSuccess && xmax_out) e = launch_max(g, x, xmax_out, s);
    return hip_check(e, "pet_osem_epoch");
}

extern "C" pet_status pet_objective(pet_geom g, const float *x, const void *y, int y_dtype, const float *add,
                                    const float *mult, const float *kappa, const float w[27], float beta, float gamma,
                                    float eps, double *out, void *stream) {
    if (!g || !x || !y || !w || !out) return fail(PET_E_ARG, "pet_objective: null argument");
    if (!valid_dtype(y_dtype)) return fail(PET_E_ARG, "pet_objective: bad y dtype");
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        pet_status st = check_data(g, g->check_counts, s, "pet_objective", x, y, y_dtype, add, mult);
        if (st == PET_OK && kappa)
            st = check_domain(g->check_counts, s, "pet_objective", nullptr, 0,
                              {{kappa, CHK_NONNEG, g->n_vox, "kappa voxels are negative or not finite"}});
        if (st != PET_OK) return st;
    }
    const pet_status st =
        hip_check(objective_impl(g, x, y, y_dtype, add, mult, kappa, w, beta, gamma, eps, out, s), "pet_objective");
    if (st != PET_OK || !checking(g)) return st;
    return check_numeric(s, out, "pet_objective");
}

// PET_CHECK for the epoch functions: the image, the data of the state, its
// sensitivity and kappa.
static pet_status check_epoch_domain(pet_geom g, const pet_svrg_state *st, const float *x, hipStream_t s,
                                     const char *name) {
    pet_status cs = check_data(g, g->check_counts, s, name, x, st->y, st->y_dtype, st->add, st->mult);
    if (cs == PET_OK)
        cs = check_domain(g->check_counts, s, name, nullptr, 0,
                          {{st->sens, CHK_NONNEG, g->n_vox, "sensitivity voxels are negative or not finite"},
                           {st->kappa, CHK_NONNEG, g->n_vox, "kappa voxels are negative or not finite"}});
    return cs;
}

static pet_status svrg_epoch_impl(pet_geom g, pet_svrg_state *st, float *x, const int32_t *subset_seq,
                                  const float *tau, const uint8_t *update_pc, const pet_svrg_options *opt,
                                  double *objective_out, void *stream, const char *name) {
    const std::string nm(name);
    if (!g || !st || !x || !subset_seq || !tau || !update_pc) return fail(PET_E_ARG, nm + ": null argument");
    if (!st->ghat_i || !st->ghat || !st->x_snap || !st->D || !st->sens || !st->y)
        return fail(PET_E_ARG, nm + ": incomplete state");
    if (st->bb && !st->g_prev) return fail(PET_E_ARG, nm + ": g_prev is needed with bb");
    if (st->counts && st->counts->g != g) return fail(PET_E_ARG, nm + ": counts were made for another geometry");
    if (st->counts && st->gnorm) return fail(PET_E_ARG, nm + ": gnorm is not available with counts");
    if (!valid_dtype(st->y_dtype)) return fail(PET_E_ARG, nm + ": bad y dtype");
    if (st->omega < 1) return fail(PET_E_ARG, nm + ": omega must be >= 1");
    if (st->k < 0) return fail(PET_E_STATE, nm + ": negative iteration counter");
    const int n = g->d.n_subsets;
    const int64_t om = (int64_t)st->omega * n;
    for (int j = 0; j < n; ++j) {
        if (subset_seq[j] < 0 || subset_seq[j] >= n) return fail(PET_E_ARG, nm + ": subset_seq entry out of range");
        if (opt && opt->weight && !(opt->weight[j] > 0.f && std::isfinite(opt->weight[j])))
            return fail(PET_E_ARG, nm + ": weights must be positive and finite");
        if (opt && opt->bb_update && opt->bb_update[j] && (st->k + j) % om != 0)
            return fail(PET_E_ARG, nm + ": bb_update only at snapshot iterations");
        if (opt && opt->bb_update && opt->bb_update[j] && !st->bb)
            return fail(PET_E_ARG, nm + ": bb_update needs state->bb");
    }
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        const pet_status cs = check_epoch_domain(g, st, x, s, name);
        if (cs != PET_OK) return cs;
    }
    hipError_t e = hipSuccess;
    const int64_t nv = g->n_vox;
    const double *tau_bb = st->bb ? st->bb + 2 : nullptr;
    // the iterate alternates between x and the handle's xtmp (the step reads
    // neighbours, so it cannot update in place); one copy at the end if needed
    float *cur = x, *nxt = g->xtmp;
    // Fused steps (k_step_tile) leave the image sheets of the new iterate and
    // cleared gradient sheets behind, so that the next iteration converts
    // nothing: `sheets` = the image sheets hold cur, `zeroed` = the gradient
    // sheets' interiors are zero.
    const bool fuse = step_tile_ok(g) && !st->kappa && !st->gnorm;
    bool sheets = false, zeroed = false;
    for (int j = 0; j < n && e == hipSuccess; ++j) {
        const int64_t k = st->k + j;
        const bool snap = (k % om) == 0;
        const int i = subset_seq[j];
        const float w = (opt && opt->weight) ? opt->weight[j] : (float)n;
        if (st->bb && k == 0) e = launch_bb_init(st->bb, s);
        if (e == hipSuccess && !sheets) e = launch_to_sheets(g, cur, s);
        sheets = false;
        if (snap) {
            // with snap_objective, the snapshot's own passes also sum the data
            // term at xhat (no extra projection)
            double *so = st->snap_objective;
            // zero-count-aware with fused steps: the n subset gradients in one
            // launch over all lines (most counts first, so that no launch ends
            // on a tail of long lines), each subset into its own pair of
            // gradient sheets
            const bool one_launch = st->counts && st->counts->slots && fuse;
            if (one_launch) {
                pet_counts_s *c = st->counts;
                ProjArgs a = base_args(g, -1);
                a.G0 = c->slots;
                a.G1 = c->slots + g->t0_elems;
                a.partial = so ? g->partial : nullptr;
                if (e == hipSuccess) e = launch_line_counts(g, c, M_GRAD, -1, a, s, c->slot_floats);
                if (e == hipSuccess && so) e = launch_reduce_sum(g->partial, counts_blocks(c, -1), so, 0, s);
                if (e == hipSuccess)
                    e = launch_snapshot_accum_slots(g, c->slots, c->slots + g->t0_elems, c->slot_floats, n,
                                                    st->ghat_i, st->ghat, st->sens, s);
            }
            for (int q = 0; q < n && e == hipSuccess && !one_launch; ++q) {
                e = st->counts ? counts_grad_sheets(g, st->counts, q, so, s, q > 0, zeroed)
                               : subset_grad_sheets(g, q, st->y, st->y_dtype, st->add, st->mult, so, q > 0, s,
                                                    zeroed);
                // zero-count-aware tables hold the x-dependent parts; ghat starts from sens
                // (with fused steps the accumulation also clears the gradient sheets)
                if (e == hipSuccess)
                    e = launch_snapshot_accum(g, st->ghat_i + (size_t)q * nv, st->ghat, nullptr, q == 0, s,
                                              st->counts ? st->sens : nullptr, fuse);
                zeroed = fuse;
            }
            if (e == hipSuccess && so && st->counts) {
                // D = <sens, x> + sum r - sum y + sum y log(y / ybar)
                e = launch_dot(st->sens, cur, nv, g->partial, so, 1, s);
                const pet_counts_s *c = st->counts;
                if (e == hipSuccess) e = launch_add_scalar(so, c->sum_add[c->n_subsets] - c->sum_y[c->n_subsets], s);
            }
            if (e == hipSuccess && so)
                e = launch_rdp(g, cur, st->kappa, st->w, st->beta, st->gamma, st->eps, nullptr, nullptr, g->partial, s);
            if (e == hipSuccess && so) e = launch_reduce_sum(g->partial, rdp_blocks(g), so, 1, s);
            // BB bookkeeping: 0 none, 1 keep the full gradient, 2 also recompute the step bound
            const int bb_mode = !st->bb ? 0 : (opt && opt->bb_update && opt->bb_update[j] && k > 0) ? 2 : 1;
            float *grad_out = st->gnorm ? g->num : nullptr;
            if (e == hipSuccess && fuse && bb_mode < 2) {
                e = launch_svrg_step_tile(g, cur, st->w, st->beta, st->gamma, st->eps, update_pc[j], st->sens,
                                          st->alpha, st->delta, st->D, 1, st->ghat_i + (size_t)i * nv, st->ghat, w,
                                          tau[j], tau_bb, bb_mode == 1, st->g_prev, nxt, s);
                sheets = true;
            } else if (e == hipSuccess) {
                e = launch_svrg_step_ex(g, cur, st->kappa, st->w, st->beta, st->gamma, st->eps, update_pc[j], st->sens,
                                        st->alpha, st->delta, st->D, 1, g->g, st->ghat_i + (size_t)i * nv, st->ghat, w,
                                        tau[j], tau_bb, bb_mode, st->x_snap, st->g_prev, grad_out, nxt, s);
            }
            if (e == hipSuccess && bb_mode == 2) {
                e = launch_bb_finish(g, st->bb, s);
                if (e == hipSuccess) e = launch_step_stored(g, cur, st->D, st->g_prev, tau[j], tau_bb, nxt, s);
            }
            if (e == hipSuccess && st->gnorm) e = launch_subset_norms(g, st->ghat_i, g->num, st->gnorm, s);
            if (e == hipSuccess) e = launch_copy(st->x_snap, cur, nv, s);
        } else {
            e = st->counts ? counts_grad_sheets(g, st->counts, i, nullptr, s, 0, zeroed)
                           : subset_grad_sheets(g, i, st->y, st->y_dtype, st->add, st->mult, nullptr, 0, s, zeroed);
            if (fuse) {
                if (e == hipSuccess)
                    e = launch_svrg_step_tile(g, cur, st->w, st->beta, st->gamma, st->eps, update_pc[j], st->sens,
                                              st->alpha, st->delta, st->D, 0, st->ghat_i + (size_t)i * nv, st->ghat,
                                              w, tau[j], tau_bb, 0, nullptr, nxt, s);
                sheets = zeroed = true;
            } else {
                if (e == hipSuccess) e = launch_from_sheets(g, g->g, 0, s);
                if (e == hipSuccess)
                    e = launch_svrg_step_ex(g, cur, st->kappa, st->w, st->beta, st->gamma, st->eps, update_pc[j],
                                            st->sens, st->alpha, st->delta, st->D, 0, g->g,
                                            st->ghat_i + (size_t)i * nv, st->ghat, w, tau[j], tau_bb, 0, nullptr,
                                            nullptr, nullptr, nxt, s);
            }
        }
        std::swap(cur, nxt);
    }
    if (e == hipSuccess && cur != x) e = launch_copy(x, cur, nv, s);
    if (e != hipSuccess) return hip_check(e, name);
    st->k += n;
    if (objective_out)
        e = st->counts ? objective_counts_impl(g, st->counts, x, st->sens, st->kappa, st->w, st->beta, st->gamma,
                                               st->eps, objective_out, s)
                       : objective_impl(g, x, st->y, st->y_dtype, st->add, st->mult, st->kappa, st->w, st->beta,
                                        st->gamma, st->eps, objective_out, s);
    const pet_status rs = hip_check(e, name);
    if (rs != PET_OK || !objective_out || !checking(g)) return rs;
    return check_numeric(s, objective_out, name);
}

extern "C" pet_status pet_svrg_epoch(pet_geom g, pet_svrg_state *st, float *x, const int32_t *subset_seq,
                                     const float *tau, const uint8_t *update_pc, double *objective_out, void *stream) {
    return svrg_epoch_impl(g, st, x, subset_seq, tau, update_pc, nullptr, objective_out, stream, "pet_svrg_epoch");
}

extern "C" pet_status pet_svrg_epoch_ex(pet_geom g, pet_svrg_state *st, float *x, const int32_t *subset_seq,
                                        const float *tau, const uint8_t *update_pc, const pet_svrg_options *opt,
                                        double *objective_out, void *stream) {
    return svrg_epoch_impl(g, st, x, subset_seq, tau, update_pc, opt, objective_out, stream, "pet_svrg_epoch_ex");
}

// SAGA (eq. (saga)) and SGD epochs: the same iteration as pet_svrg_epoch with
// another estimator (Section 2.1).  SAGA fills its table of grad J_i at the
// current x when the state is fresh (k = 0).
static pet_status sgm_epoch(pet_geom g, pet_svrg_state *st, int estimator, float *x, const int32_t *subset_seq,
                            const float *tau, const uint8_t *update_pc, double *objective_out, void *stream,
                            const char *name) {
    const std::string nm(name);
    if (!g || !st || !x || !subset_seq || !tau || !update_pc) return fail(PET_E_ARG, nm + ": null argument");
    const pet_counts_s *cnt = st->counts;
    if (!st->D || !st->sens || !st->y || (estimator == SGM_SAGA && (!st->ghat_i || !st->ghat)) ||
        (cnt && !st->ghat_i))
        return fail(PET_E_ARG, nm + ": incomplete state");
    if (!valid_dtype(st->y_dtype)) return fail(PET_E_ARG, nm + ": bad y dtype");
    if (st->k < 0) return fail(PET_E_STATE, nm + ": negative iteration counter");
    if (cnt && cnt->g != g) return fail(PET_E_ARG, nm + ": counts were made for another geometry");
    const int n = g->d.n_subsets;
    for (int j = 0; j < n; ++j)
        if (subset_seq[j] < 0 || subset_seq[j] >= n) return fail(PET_E_ARG, nm + ": subset_seq entry out of range");
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        const pet_status cs = check_epoch_domain(g, st, x, s, name);
        if (cs != PET_OK) return cs;
    }
    hipError_t e = hipSuccess;
    const int64_t nv = g->n_vox;
    // Zero-count-aware path: the line kernels give h_i(x) = -P_i^T[mult y / ybar]
    // only, and grad D_i = sens_i + h_i.  SAGA's table then holds h_i + (beta /
    // n) grad S (the sens_i cancel in n(grad J_i - T_i)) and its sum starts
    // from sens = sum_i sens_i; SGD keeps the n subset sensitivities sens_i in
    // state->ghat_i (back projections of mult, filled at k = 0) and adds them
    // to h_i in the step.
    if (cnt && estimator == SGM_SGD && st->k == 0) {
        for (int q = 0; q < n && e == hipSuccess; ++q) {
            e = launch_zero_sheets(g, s);
            ProjArgs a = base_args(g, q);
            a.mult = st->mult;
            if (e == hipSuccess) e = launch_line_kernel(g, M_BACK, q, a, s);
            if (e == hipSuccess) e = launch_from_sheets(g, st->ghat_i + (size_t)q * nv, 0, s);
        }
    }
    for (int j = 0; j < n && e == hipSuccess; ++j) {
        const int64_t k = st->k + j;
        const int i = subset_seq[j];
        const bool first = estimator == SGM_SAGA && k == 0;
        e = launch_to_sheets(g, x, s);
        if (first) {
            // table of data gradients at x, then the prior shares and the sum
            for (int q = 0; q < n && e == hipSuccess; ++q) {
                e = cnt ? counts_grad_sheets(g, cnt, q, nullptr, s)
                        : subset_grad_sheets(g, q, st->y, st->y_dtype, st->add, st->mult, nullptr, 0, s);
                if (e == hipSuccess) e = launch_snapshot_accum(g, st->ghat_i + (size_t)q * nv, st->ghat, nullptr, q == 0, s);
            }
            if (e == hipSuccess)
                e = launch_rdp(g, x, st->kappa, st->w, st->beta, st->gamma, st->eps, g->num, nullptr, nullptr, s);
            if (e == hipSuccess) e = launch_saga_table_prior(g, st->ghat_i, st->ghat, g->num, s, cnt ? st->sens : nullptr);
        } else {
            e = cnt ? counts_grad_sheets(g, cnt, i, nullptr, s)
                    : subset_grad_sheets(g, i, st->y, st->y_dtype, st->add, st->mult, nullptr, 0, s);
            if (e == hipSuccess) e = launch_from_sheets(g, g->g, 0, s);
        }
        float *table_i = estimator == SGM_SAGA || cnt ? st->ghat_i + (size_t)i * nv : nullptr;
        if (e == hipSuccess)
            e = launch_sgm_step(g, estimator, x, st->kappa, st->w, st->beta, st->gamma, st->eps, update_pc[j],
                                st->sens, st->alpha, st->delta, st->D, first, g->g, table_i, st->ghat, (float)n,
                                tau[j], g->xtmp, s);
        if (e == hipSuccess) e = launch_copy(x, g->xtmp, nv, s);
    }
    if (e != hipSuccess) return hip_check(e, name);
    st->k += n;
    if (objective_out)
        e = cnt ? objective_counts_impl(g, cnt, x, st->sens, st->kappa, st->w, st->beta, st->gamma, st->eps,
                                        objective_out, s)
                : objective_impl(g, x, st->y, st->y_dtype, st->add, st->mult, st->kappa, st->w, st->beta, st->gamma,
                                 st->eps, objective_out, s);
    const pet_status rs = hip_check(e, name);
    if (rs != PET_OK || !objective_out || !checking(g)) return rs;
    return check_numeric(s, objective_out, name);
}

extern "C" pet_status pet_saga_epoch(pet_geom g, pet_svrg_state *st, float *x, const int32_t *subset_seq,
                                     const float *tau, const uint8_t *update_pc, double *objective_out, void *stream) {
    return sgm_epoch(g, st, SGM_SAGA, x, subset_seq, tau, update_pc, objective_out, stream, "pet_saga_epoch");
}

extern "C" pet_status pet_sgd_epoch(pet_geom g, pet_svrg_state *st, float *x, const int32_t *subset_seq,
                                    const float *tau, const uint8_t *update_pc, double *objective_out, void *stream) {
    return sgm_epoch(g, st, SGM_SGD, x, subset_seq, tau, update_pc, objective_out, stream, "pet_sgd_epoch");
}

extern "C" pet_status pet_work_counts(pet_geom g, int subset, double *out, void *stream) {
    if (!g || !out) return fail(PET_E_ARG, "pet_work_counts: null argument");
    if (!valid_subset(g, subset)) return fail(PET_E_ARG, "pet_work_counts: subset out of range");
    hipStream_t s = (hipStream_t)stream;
    ProjArgs a = base_args(g, subset);
    a.partial = g->partial;
    const int nb = n_line_blocks(g, subset);
    hipError_t e = launch_line_kernel(g, M_COUNT, subset, a, s);
    if (e == hipSuccess) e = launch_reduce_sum(g->partial, nb, out, 0, s);
    if (e == hipSuccess) e = launch_reduce_sum(g->partial + nb, nb, out + 1, 0, s);
    return hip_check(e, "pet_work_counts");
}

extern "C" pet_status pet_profile_enable(pet_geom g, int enable) {
    if (!g) return fail(PET_E_ARG, "pet_profile_enable: null handle");
    g->profiling = enable != 0;
    return PET_OK;
}

extern "C" pet_status pet_geom_set_flags(pet_geom g, unsigned flags) {
    if (!g) return fail(PET_E_ARG, "pet_geom_set_flags: null handle");
    if (flags & ~(unsigned)(PET_CHECK | PET_SMALL_CHUNKS | PET_SIGNED_SHEETS))
        return fail(PET_E_ARG, "pet_geom_set_flags: unknown flag");
    g->flags = flags;
    return PET_OK;
}

extern "C" pet_status pet_profile_read(pet_geom g, int kernel, double *total_ms, int64_t *launches) {
    if (!g || !total_ms || !launches) return fail(PET_E_ARG, "pet_profile_read: null argument");
    if (kernel < 0 || kernel > PROF_GATHER || kernel == M_COUNT) return fail(PET_E_ARG, "pet_profile_read: unknown kernel");
    double ms = 0.0;
    auto &v = g->prof_events[kernel];
    for (auto &ev : v) {
        hipError_t e = hipEventSynchronize(ev.second);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, ev.first, ev.second);
        if (e != hipSuccess) return hip_check(e, "pet_profile_read");
        ms += t;
        g->prof_pool.push_back(ev);
    }
    *total_ms = ms;
    *launches = (int64_t)v.size();
    v.clear();
    return PET_OK;
}

extern "C" pet_status pet_subset_hvp(pet_geom g, int subset, const float *x, const float *v, const void *y,
                                     int y_dtype, const float *add, const float *mult, float *ybar_work,
                                     float *hv_out, int accumulate, void *stream) {
    if (!g || !x || !v || !y || !ybar_work || !hv_out) return fail(PET_E_ARG, "pet_subset_hvp: null argument");
    if (!valid_subset(g, subset)) return fail(PET_E_ARG, "pet_subset_hvp: subset out of range");
    if (!valid_dtype(y_dtype)) return fail(PET_E_ARG, "pet_subset_hvp: bad y dtype");
    if (checking(g)) {
        pet_status cs = check_data(g, g->check_counts, (hipStream_t)stream, "pet_subset_hvp", x, y, y_dtype, add, mult);
        if (cs == PET_OK)
            cs = check_domain(g->check_counts, (hipStream_t)stream, "pet_subset_hvp", nullptr, 0,
                              {{v, CHK_FINITE, g->n_vox, "direction voxels are not finite"}});
        if (cs != PET_OK) return cs;
    }
    return hip_check(hvp_impl(g, subset, x, v, y, y_dtype, add, mult, ybar_work, hv_out, accumulate,
                              (hipStream_t)stream),
                     "pet_subset_hvp");
}

extern "C" pet_status pet_rdp_hvp(pet_geom g, const float *x, const float *kappa, const float w[27], float beta,
                                  float gamma, float eps, const float *v, float *hv_out, int accumulate,
                                  double *gdot_out, void *stream) {
    if (!g || !x || !w || !v || !hv_out) return fail(PET_E_ARG, "pet_rdp_hvp: null argument");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_rdp_hvp(g, x, kappa, w, beta, gamma, eps, v, hv_out, accumulate,
                                  gdot_out ? g->partial : nullptr, s);
    if (e == hipSuccess && gdot_out) e = launch_reduce_sum(g->partial, adj_blocks(g), gdot_out, 1, s);
    return hip_check(e, "pet_rdp_hvp");
}

extern "C" pet_status pet_precond_vjp(pet_geom g, const float *x, const float *sens, const float *kappa,
                                      const float w[27], float beta, float gamma, float eps, float alpha, float delta,
                                      const float *Dbar, float *xbar, double *betabar, void *stream) {
    if (!g || !x || !sens || !w || !Dbar || !xbar || !betabar) return fail(PET_E_ARG, "pet_precond_vjp: null argument");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_precond_vjp(g, x, kappa, w, beta, gamma, eps, sens, alpha, delta, Dbar, xbar, g->hess,
                                      g->partial, s);
    if (e == hipSuccess) e = launch_reduce_sum(g->partial, adj_blocks(g), betabar, 1, s);
    return hip_check(e, "pet_precond_vjp");
}

extern "C" pet_status pet_svrg_epoch_vjp(pet_geom g, const pet_svrg_state *st, pet_svrg_vjp_bufs *b,
                                         const int32_t *subset_seq, const float *tau, const uint8_t *update_pc,
                                         void *stream) {
    if (!g || !st || !b || !subset_seq || !tau || !update_pc) return fail(PET_E_ARG, "pet_svrg_epoch_vjp: null argument");
    if (!st->ghat_i || !st->ghat || !st->D || !st->sens || !st->y)
        return fail(PET_E_ARG, "pet_svrg_epoch_vjp: incomplete state");
    if (!b->x_start || !b->xbar || !b->Dbar || !b->gbar_i || !b->gbar || !b->betabar || !b->xs || !b->est ||
        !b->ybar_work || !b->v)
        return fail(PET_E_ARG, "pet_svrg_epoch_vjp: incomplete buffers");
    if (!valid_dtype(st->y_dtype)) return fail(PET_E_ARG, "pet_svrg_epoch_vjp: bad y dtype");
    if (st->counts) return fail(PET_E_ARG, "pet_svrg_epoch_vjp: runs the dense kernels (state->counts must be NULL)");
    if (st->omega < 1 || st->k < 0) return fail(PET_E_ARG, "pet_svrg_epoch_vjp: bad omega or iteration counter");
    const int n = g->d.n_subsets;
    const int64_t nv = g->n_vox;
    const int64_t om = (int64_t)st->omega * n;
    for (int j = 0; j < n; ++j) {
        if (subset_seq[j] < 0 || subset_seq[j] >= n) return fail(PET_E_ARG, "pet_svrg_epoch_vjp: subset_seq entry out of range");
        if (j > 0 && update_pc[j]) return fail(PET_E_ARG, "pet_svrg_epoch_vjp: preconditioner updates only at the epoch's first iteration");
        if (j > 0 && (st->k + j) % om == 0) return fail(PET_E_ARG, "pet_svrg_epoch_vjp: snapshots only at the epoch's first iteration");
    }
    const bool snap0 = st->k % om == 0;
    if (!snap0 && !b->x_snap_src) return fail(PET_E_ARG, "pet_svrg_epoch_vjp: x_snap_src needed (epoch without snapshot)");
    if (!update_pc[0] && !b->D_start) return fail(PET_E_ARG, "pet_svrg_epoch_vjp: D_start needed (no update at the epoch start)");
    hipStream_t s = (hipStream_t)stream;
    float *v = b->v, *tmp = b->v + nv;
    auto xs = [&](int j) { return b->xs + (size_t)j * nv; };
    hipError_t e = hipSuccess;

    // ---- recompute the epoch, keeping every iterate and estimator ----
    if (!snap0) {
        e = launch_to_sheets(g, b->x_snap_src, s);
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            e = subset_grad_sheets(g, i, st->y, st->y_dtype, st->add, st->mult, nullptr, 0, s);
            if (e == hipSuccess) e = launch_snapshot_accum(g, st->ghat_i + (size_t)i * nv, st->ghat, nullptr, i == 0, s);
        }
    }
    if (e == hipSuccess && !update_pc[0]) e = launch_copy(st->D, b->D_start, nv, s);
    if (e == hipSuccess) e = launch_copy(xs(0), b->x_start, nv, s);
    for (int j = 0; j < n && e == hipSuccess; ++j) {
        const bool snap = (st->k + j) % om == 0;
        const int i = subset_seq[j];
        e = launch_to_sheets(g, xs(j), s);
        if (snap) {
            for (int q = 0; q < n && e == hipSuccess; ++q) {
                e = subset_grad_sheets(g, q, st->y, st->y_dtype, st->add, st->mult, nullptr, 0, s);
                if (e == hipSuccess) e = launch_snapshot_accum(g, st->ghat_i + (size_t)q * nv, st->ghat, nullptr, q == 0, s);
            }
        } else {
            e = subset_grad_sheets(g, i, st->y, st->y_dtype, st->add, st->mult, nullptr, 0, s);
            if (e == hipSuccess) e = launch_from_sheets(g, g->g, 0, s);
        }
        if (e == hipSuccess)
            e = launch_svrg_step(g, xs(j), st->kappa, st->w, st->beta, st->gamma, st->eps, update_pc[j], st->sens,
                                 st->alpha, st->delta, st->D, snap, g->g, st->ghat_i + (size_t)i * nv, st->ghat,
                                 (float)n, tau[j], xs(j + 1), b->est + (size_t)j * nv, s);
    }

    // ---- reverse sweep ----
    for (int j = n - 1; j >= 0 && e == hipSuccess; --j) {
        const bool snap = (st->k + j) % om == 0;
        const int i = subset_seq[j];
        // clip and step: xbar <- u, Dbar += -tau u est, v = -tau D u
        e = launch_step_vjp(g, xs(j + 1), st->D, b->est + (size_t)j * nv, tau[j], b->xbar, b->Dbar, v, s);
        // prior: xbar += beta H_S v, dL/dbeta += <grad S, v>
        if (e == hipSuccess)
            e = launch_rdp_hvp(g, xs(j), st->kappa, st->w, st->beta, st->gamma, st->eps, v, b->xbar, 1, g->partial, s);
        if (e == hipSuccess) e = launch_reduce_sum(g->partial, adj_blocks(g), b->betabar, 1, s);
        if (e != hipSuccess) break;
        if (!snap) {
            // est = n (g_i(x) - ghat_i) + ghat + ...: xbar += n H_i v, gbar_i -= n v, gbar += v
            float *gbi = b->gbar_i + (size_t)i * nv;
            e = launch_lincomb(tmp, (float)n, v, 0.f, nullptr, nv, s);
            if (e == hipSuccess)
                e = hvp_impl(g, i, xs(j), tmp, st->y, st->y_dtype, st->add, st->mult, b->ybar_work, b->xbar, 1, s);
            if (e == hipSuccess) e = launch_lincomb(gbi, 1.f, gbi, -(float)n, v, nv, s);
            if (e == hipSuccess) e = launch_lincomb(b->gbar, 1.f, b->gbar, 1.f, v, nv, s);
        } else {
            // est = ghat + ...: the snapshot table and sum were produced here from x_j
            e = launch_lincomb(b->gbar, 1.f, b->gbar, 1.f, v, nv, s);
            for (int q = 0; q < n && e == hipSuccess; ++q) {
                float *gbq = b->gbar_i + (size_t)q * nv;
                e = launch_lincomb(tmp, 1.f, gbq, 1.f, b->gbar, nv, s);
                if (e == hipSuccess)
                    e = hvp_impl(g, q, xs(j), tmp, st->y, st->y_dtype, st->add, st->mult, b->ybar_work, b->xbar, 1, s);
                if (e == hipSuccess) e = launch_fill(gbq, nv, 0.f, s);
            }
            if (e == hipSuccess) e = launch_fill(b->gbar, nv, 0.f, s);
        }
        if (e == hipSuccess && update_pc[j]) {
            e = launch_precond_vjp(g, xs(j), st->kappa, st->w, st->beta, st->gamma, st->eps, st->sens, st->alpha,
                                   st->delta, b->Dbar, b->xbar, tmp, g->partial, s);
            if (e == hipSuccess) e = launch_reduce_sum(g->partial, adj_blocks(g), b->betabar, 1, s);
            if (e == hipSuccess) e = launch_fill(b->Dbar, nv, 0.f, s);
        }
    }
    return hip_check(e, "pet_svrg_epoch_vjp");
}

extern "C" pet_status pet_subset_grad_counts(pet_geom g, pet_counts c, int subset, const float *x,
                                             const float *sens_subset, float *grad_out, double *kl_out, void *stream) {
    if (!g || !c || !x || !grad_out) return fail(PET_E_ARG, "pet_subset_grad_counts: null argument");
    if (c->g != g) return fail(PET_E_ARG, "pet_subset_grad_counts: counts were made for another geometry");
    if (!valid_subset(g, subset)) return fail(PET_E_ARG, "pet_subset_grad_counts: subset out of range");
    if (kl_out && !sens_subset) return fail(PET_E_ARG, "pet_subset_grad_counts: kl_out needs sens_subset");
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        pet_status cs = check_domain(g->check_counts, s, "pet_subset_grad_counts", nullptr, 0,
                                     {{x, CHK_NONNEG, g->n_vox, MSG_X},
                                      {sens_subset, CHK_NONNEG, g->n_vox,
                                       "sensitivity voxels are negative or not finite"}});
        if (cs != PET_OK) return cs;
    }
    const int row = subset < 0 ? c->n_subsets : subset;
    hipError_t e = launch_to_sheets(g, x, s);
    if (e == hipSuccess) e = counts_grad_sheets(g, c, subset, kl_out, s);
    if (e == hipSuccess) e = launch_from_sheets(g, grad_out, 0, s);
    if (e == hipSuccess && sens_subset) e = launch_lincomb(grad_out, 1.f, grad_out, 1.f, sens_subset, g->n_vox, s);
    if (e == hipSuccess && kl_out) e = launch_dot(sens_subset, x, g->n_vox, g->partial, kl_out, 1, s);
    if (e == hipSuccess && kl_out) e = launch_add_scalar(kl_out, c->sum_add[row] - c->sum_y[row], s);
    return hip_check(e, "pet_subset_grad_counts");
}

extern "C" pet_status pet_osem_epoch_counts(pet_geom g, pet_counts c, float *x, const float *mult,
                                            const int32_t *order, float *xmax_out, float *sens_out, void *stream) {
    if (!g || !c || !x || !order) return fail(PET_E_ARG, "pet_osem_epoch_counts: null argument");
    if (c->g != g) return fail(PET_E_ARG, "pet_osem_epoch_counts: counts were made for another geometry");
    for (int j = 0; j < g->d.n_subsets; ++j)
        if (order[j] < 0 || order[j] >= g->d.n_subsets)
            return fail(PET_E_ARG, "pet_osem_epoch_counts: order entry out of range");
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        int64_t nl = 0;
        pet_geom_info(g, -1, nullptr, &nl, nullptr);
        const pet_status cs = check_domain(g->check_counts, s, "pet_osem_epoch_counts", nullptr, 0,
                                           {{x, CHK_NONNEG, g->n_vox, MSG_X}, {mult, CHK_NONNEG, nl, MSG_MULT}});
        if (cs != PET_OK) return cs;
    }
    hipError_t e = hipSuccess;
    for (int j = 0; j < g->d.n_subsets && e == hipSuccess; ++j) {
        const int i = order[j];
        // P_i^T mult
        e = launch_zero_sheets(g, s);
        ProjArgs a = base_args(g, i);
        a.mult = mult;
        if (e == hipSuccess) e = launch_line_kernel(g, M_BACK, i, a, s);
        if (e == hipSuccess) e = launch_from_sheets(g, g->sensi, 0, s);
        if (e == hipSuccess && sens_out)
            e = j == 0 ? launch_copy(sens_out, g->sensi, g->n_vox, s)
                       : launch_lincomb(sens_out, 1.f, sens_out, 1.f, g->sensi, g->n_vox, s);
        // -P_i^T (mult y / ybar) from the bins with counts; the update negates
        if (e == hipSuccess) e = launch_to_sheets(g, x, s);
        if (e == hipSuccess) e = counts_grad_sheets(g, c, i, nullptr, s);
        if (e == hipSuccess) e = launch_from_sheets(g, g->num, 0, s);
        if (e == hipSuccess) e = launch_osem_update(g, x, g->num, g->sensi, s, -1.f);
    }
    if (e == hipSuccess && xmax_out) e = launch_max(g, x, xmax_out, s);
    return hip_check(e, "pet_osem_epoch_counts");
}

extern "C" pet_status pet_objective_counts(pet_geom g, pet_counts c, const float *x, const float *sens,
                                           const float *kappa, const float w[27], float beta, float gamma, float eps,
                                           double *out, void *stream) {
    if (!g || !c || !x || !sens || !w || !out) return fail(PET_E_ARG, "pet_objective_counts: null argument");
    if (c->g != g) return fail(PET_E_ARG, "pet_objective_counts: counts were made for another geometry");
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        const pet_status cs = check_domain(g->check_counts, s, "pet_objective_counts", nullptr, 0,
                                           {{x, CHK_NONNEG, g->n_vox, MSG_X},
                                            {sens, CHK_NONNEG, g->n_vox, "sensitivity voxels are negative or not finite"},
                                            {kappa, CHK_NONNEG, g->n_vox, "kappa voxels are negative or not finite"}});
        if (cs != PET_OK) return cs;
    }
    const pet_status st = hip_check(objective_counts_impl(g, c, x, sens, kappa, w, beta, gamma, eps, out, s),
                                    "pet_objective_counts");
    if (st != PET_OK || !checking(g)) return st;
    return check_numeric(s, out, "pet_objective_counts");
}
