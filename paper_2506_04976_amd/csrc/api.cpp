// C entry points of the gfx950 PET library (declared in include/pet.h).
// Argument checking happens here, before anything is enqueued; the work itself
// is a sequence of kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

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
    return a;
}

// Data-term gradient of one subset into the gradient sheets (G0, G1); the
// image sheets must already hold x.  Optionally FP64 KL sum into kl_out.
hipError_t subset_grad_sheets(pet_geom g, int subset, const void *y, int dt, const float *add, const float *mult,
                              double *kl_out, int kl_accumulate, hipStream_t s) {
    hipError_t e = launch_zero_sheets(g, s);
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

}  // namespace
}  // namespace pet

using namespace pet;

extern "C" const char *pet_last_error(void) { return g_last_error.c_str(); }

extern "C" pet_status pet_fwd(pet_geom g, int subset, const float *x, const float *mult, const float *add, float *out,
                              void *stream) {
    if (!g || !x || !out) return fail(PET_E_ARG, "pet_fwd: null argument");
    if (!valid_subset(g, subset)) return fail(PET_E_ARG, "pet_fwd: subset out of range");
    hipStream_t s = (hipStream_t)stream;
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
    if (algo != PET_BACK_AUTO && algo != PET_BACK_SCATTER) return fail(PET_E_ARG, "pet_back: unknown algo");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_zero_sheets(g, s);
    if (e != hipSuccess) return hip_check(e, "pet_back");
    ProjArgs a = base_args(g, subset);
    a.sino = sino;
    a.mult = mult;
    e = launch_line_kernel(g, M_BACK, subset, a, s);
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
    hipError_t e = launch_rdp(g, x, kappa, w, beta, gamma, eps, grad_out, hessdiag_out, value_out ? g->partial : nullptr, s);
    if (e == hipSuccess && value_out) e = launch_reduce_sum(g->partial, rdp_blocks(g), value_out, 0, s);
    return hip_check(e, "pet_rdp_grad_hessdiag");
}

extern "C" pet_status pet_precond(pet_geom g, const float *x, const float *sens, const float *hessdiag, float alpha,
                                  float delta, float *D_out, void *stream) {
    if (!g || !x || !sens || !hessdiag || !D_out) return fail(PET_E_ARG, "pet_precond: null argument");
    return hip_check(launch_precond(g, x, sens, hessdiag, alpha, delta, D_out, (hipStream_t)stream), "pet_precond");
}

extern "C" pet_status pet_osem_epoch(pet_geom g, float *x, const void *y, int y_dtype, const float *add,
                                     const float *mult, const int32_t *order, float *xmax_out, void *stream) {
    if (!g || !x || !y || !order) return fail(PET_E_ARG, "pet_osem_epoch: null argument");
    if (!valid_dtype(y_dtype)) return fail(PET_E_ARG, "pet_osem_epoch: bad y dtype");
    for (int j = 0; j < g->d.n_subsets; ++j)
        if (order[j] < 0 || order[j] >= g->d.n_subsets) return fail(PET_E_ARG, "pet_osem_epoch: order entry out of range");
    hipStream_t s = (hipStream_t)stream;
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
    return hip_check(objective_impl(g, x, y, y_dtype, add, mult, kappa, w, beta, gamma, eps, out, (hipStream_t)stream),
                     "pet_objective");
}

extern "C" pet_status pet_svrg_epoch(pet_geom g, pet_svrg_state *st, float *x, const int32_t *subset_seq,
                                     const float *tau, const uint8_t *update_pc, double *objective_out, void *stream) {
    if (!g || !st || !x || !subset_seq || !tau || !update_pc) return fail(PET_E_ARG, "pet_svrg_epoch: null argument");
    if (!st->ghat_i || !st->ghat || !st->x_snap || !st->D || !st->sens || !st->y)
        return fail(PET_E_ARG, "pet_svrg_epoch: incomplete state");
    if (!valid_dtype(st->y_dtype)) return fail(PET_E_ARG, "pet_svrg_epoch: bad y dtype");
    if (st->omega < 1) return fail(PET_E_ARG, "pet_svrg_epoch: omega must be >= 1");
    if (st->k < 0) return fail(PET_E_STATE, "pet_svrg_epoch: negative iteration counter");
    const int n = g->d.n_subsets;
    for (int j = 0; j < n; ++j)
        if (subset_seq[j] < 0 || subset_seq[j] >= n) return fail(PET_E_ARG, "pet_svrg_epoch: subset_seq entry out of range");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    const int64_t nv = g->n_vox;
    for (int j = 0; j < n && e == hipSuccess; ++j) {
        const int64_t k = st->k + j;
        const bool snap = (k % ((int64_t)st->omega * n)) == 0;
        e = launch_to_sheets(g, x, s);
        if (snap) {
            for (int i = 0; i < n && e == hipSuccess; ++i) {
                e = subset_grad_sheets(g, i, st->y, st->y_dtype, st->add, st->mult, nullptr, 0, s);
                if (e == hipSuccess) e = launch_snapshot_accum(g, st->ghat_i + (size_t)i * nv, st->ghat, nullptr, i == 0, s);
            }
            if (e == hipSuccess) e = launch_copy(st->x_snap, x, nv, s);
        } else {
            const int i = subset_seq[j];
            e = subset_grad_sheets(g, i, st->y, st->y_dtype, st->add, st->mult, nullptr, 0, s);
            if (e == hipSuccess) e = launch_from_sheets(g, g->g, 0, s);
        }
        if (e == hipSuccess) {
            const int i = subset_seq[j];
            e = launch_svrg_step(g, x, st->kappa, st->w, st->beta, st->gamma, st->eps, update_pc[j], st->sens,
                                 st->alpha, st->delta, st->D, snap, g->g, st->ghat_i + (size_t)i * nv, st->ghat,
                                 (float)n, tau[j], g->xtmp, s);
        }
        if (e == hipSuccess) e = launch_copy(x, g->xtmp, nv, s);
    }
    if (e != hipSuccess) return hip_check(e, "pet_svrg_epoch");
    st->k += n;
    if (objective_out)
        e = objective_impl(g, x, st->y, st->y_dtype, st->add, st->mult, st->kappa, st->w, st->beta, st->gamma,
                           st->eps, objective_out, s);
    return hip_check(e, "pet_svrg_epoch");
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

extern "C" pet_status pet_profile_read(pet_geom g, int kernel, double *total_ms, int64_t *launches) {
    if (!g || !total_ms || !launches) return fail(PET_E_ARG, "pet_profile_read: null argument");
    if (kernel < 0 || kernel >= M_COUNT) return fail(PET_E_ARG, "pet_profile_read: unknown kernel");
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
