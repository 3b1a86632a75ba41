// Batches of independent reconstructions (C entry points pet_batch_*): every
// member runs preconditioned SVRG (Algorithm 1) on its own geometry, data and
// state; a round advances every member by one epoch of its own n_subsets
// iterations, step j of the round touching the members with j < n_subsets.
// Each step is five launches for the whole batch (prep, the persistent line
// kernel, gather, step, commit); a round can be captured once in a HIP graph
// and replayed, with the round's schedule copied to the device before each
// replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "pet_internal.h"

using namespace pet;

struct pet_batch_s {
    int n = 0;
    int device = 0;
    std::vector<pet_geom> geoms;
    std::vector<pet_svrg_state *> states;
    std::vector<float *> slots;
    std::vector<int *> sub_nviews;
    std::vector<size_t> lds_base, lds_per_wave;  // per member: sheets + one wave's table
    std::vector<int> tof_waves;
    std::vector<double> line_cost;
    BMember *d_mem = nullptr;
    BStep *d_steps = nullptr, *h_steps = nullptr;
    int max_steps = 0;
    int *d_order = nullptr, *d_counter = nullptr;
    int blocks = 0, waves = TOF_MAX_WAVES, order_kind = 0;
    int psf_max = 0;  // most resolution-model passes of any member
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_copy = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
    bool copy_pending = false;
};

namespace {

size_t batch_lds(const pet_batch_s *b, int waves) {
    size_t m = 0;
    for (int r = 0; r < b->n; ++r) m = std::max(m, b->lds_base[r] + (size_t)std::min(b->tof_waves[r], waves) * b->lds_per_wave[r]);
    return m;
}

hipError_t upload_order(pet_batch_s *b) {
    std::vector<int> ord(b->n);
    std::iota(ord.begin(), ord.end(), 0);
    if (b->order_kind == 0)  // longest lines first
        std::stable_sort(ord.begin(), ord.end(), [&](int p, int q) { return b->line_cost[p] > b->line_cost[q]; });
    return hipMemcpy(b->d_order, ord.data(), sizeof(int) * b->n, hipMemcpyHostToDevice);
}

void drop_graph(pet_batch_s *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

hipError_t enqueue_step(pet_batch_s *b, int j, hipStream_t s) {
    hipError_t e = launch_b_prep(b->d_mem, b->n, j, b->d_counter, b->psf_max, s);
    if (e == hipSuccess)
        e = launch_line_batched(b->d_mem, b->d_order, b->n, j, b->d_counter, b->blocks, b->waves,
                                batch_lds(b, b->waves), s);
    if (e == hipSuccess) e = launch_b_gather(b->d_mem, b->n, j, b->psf_max, s);
    if (e == hipSuccess) e = launch_b_step(b->d_mem, b->n, j, s);
    if (e == hipSuccess) e = launch_b_commit(b->d_mem, b->n, j, s);
    return e;
}

hipError_t enqueue_round(pet_batch_s *b, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int j = 0; j < b->max_steps && e == hipSuccess; ++j) e = enqueue_step(b, j, s);
    return e;
}

// Copy the host schedule to the device on the batch stream (after the
// previous copy has left the pinned buffer).
hipError_t push_steps(pet_batch_s *b) {
    hipError_t e = hipMemcpyAsync(b->d_steps, b->h_steps, sizeof(BStep) * (size_t)b->n * b->max_steps,
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->ev_copy, b->stream);
    b->copy_pending = e == hipSuccess;
    return e;
}

hipError_t wait_copy(pet_batch_s *b) {
    if (!b->copy_pending) return hipSuccess;
    b->copy_pending = false;
    return hipEventSynchronize(b->ev_copy);
}

void destroy(pet_batch_s *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (float *p : b->slots)
        if (p) (void)hipFree(p);
    for (int *p : b->sub_nviews)
        if (p) (void)hipFree(p);
    if (b->d_mem) (void)hipFree(b->d_mem);
    if (b->d_steps) (void)hipFree(b->d_steps);
    if (b->h_steps) (void)hipHostFree(b->h_steps);
    if (b->d_order) (void)hipFree(b->d_order);
    if (b->d_counter) (void)hipFree(b->d_counter);
    for (hipEvent_t ev : {b->ev_in, b->ev_out, b->ev_copy, b->ev_t0, b->ev_t1})
        if (ev) (void)hipEventDestroy(ev);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // namespace

extern "C" pet_status pet_batch_create(const pet_geom *geoms, pet_svrg_state *const *states, float *const *x,
                                       int n_members, pet_batch *out) {
    if (!geoms || !states || !x || !out) return fail(PET_E_ARG, "pet_batch_create: null argument");
    if (n_members < 1 || n_members > BATCH_MAX)
        return fail(PET_E_ARG, "pet_batch_create: between 1 and " + std::to_string(BATCH_MAX) + " members");
    for (int r = 0; r < n_members; ++r) {
        if (!geoms[r] || !states[r] || !x[r]) return fail(PET_E_ARG, "pet_batch_create: null member");
        const pet_svrg_state *st = states[r];
        if (!st->ghat_i || !st->ghat || !st->D || !st->sens || !st->y)
            return fail(PET_E_ARG, "pet_batch_create: incomplete state of member " + std::to_string(r));
        if (st->counts)
            return fail(PET_E_ARG, "pet_batch_create: batches run the dense kernels (member " + std::to_string(r) +
                                       " has counts)");
        if (st->y_dtype != PET_Y_F32 && st->y_dtype != PET_Y_U16 && st->y_dtype != PET_Y_U8)
            return fail(PET_E_ARG, "pet_batch_create: bad y dtype");
        if (st->omega < 1) return fail(PET_E_ARG, "pet_batch_create: omega must be >= 1");
        for (int q = 0; q < r; ++q)
            if (geoms[q] == geoms[r]) return fail(PET_E_ARG, "pet_batch_create: members need distinct geometries");
        if (geoms[r]->device != geoms[0]->device) return fail(PET_E_ARG, "pet_batch_create: members on one device");
    }
    pet_batch_s *b = new (std::nothrow) pet_batch_s();
    if (!b) return fail(PET_E_OOM, "pet_batch_create: host allocation");
    b->n = n_members;
    b->device = geoms[0]->device;
    hipError_t e = hipSetDevice(b->device);
    std::vector<BMember> hm(n_members);
    for (int r = 0; r < n_members && e == hipSuccess; ++r) {
        pet_geom g = geoms[r];
        const pet_svrg_state *st = states[r];
        b->geoms.push_back(g);
        b->states.push_back(states[r]);
        b->max_steps = std::max(b->max_steps, g->d.n_subsets);
        BMember &m = hm[r];
        std::memset(&m, 0, sizeof(m));
        m.pa = geom_proj_args(g);
        m.pa.y = st->y;
        m.pa.y_dtype = st->y_dtype;
        m.pa.add = st->add;
        m.pa.mult = st->mult;
        m.pa.partial = nullptr;
        const int64_t slot = (int64_t)(g->t0_elems + g->t1_elems);
        float *sl = nullptr;
        e = hipMalloc(&sl, sizeof(float) * (size_t)slot * g->d.n_subsets);
        if (e == hipSuccess) e = hipMemset(sl, 0, sizeof(float) * (size_t)slot * g->d.n_subsets);
        b->slots.push_back(sl);
        m.pa.G0 = sl;
        m.pa.G1 = sl + g->t0_elems;
        std::vector<int> cnt(g->d.n_subsets);
        for (int i = 0; i < g->d.n_subsets; ++i) cnt[i] = (int)g->subset_views[i].size();
        int *dc = nullptr;
        if (e == hipSuccess) e = hipMalloc(&dc, sizeof(int) * cnt.size());
        if (e == hipSuccess) e = hipMemcpy(dc, cnt.data(), sizeof(int) * cnt.size(), hipMemcpyHostToDevice);
        b->sub_nviews.push_back(dc);
        m.views = g->views_dev;
        m.sub_nviews = dc;
        m.views_stride = g->views_stride;
        m.n_sub = g->d.n_subsets;
        m.n_views = g->d.n_views;
        m.is_tof = g->d.n_tof > 1;
        m.tof_waves = m.is_tof ? g->tof_waves : 1;
        m.nx = g->d.nx;
        m.ny = g->d.ny;
        m.nz = g->d.nz;
        m.n_vox = g->n_vox;
        m.g_slot = slot;
        m.t0_elems = (int64_t)g->t0_elems;
        m.x = x[r];
        m.xtmp = g->xtmp;
        m.g = g->g;
        m.ghat_i = st->ghat_i;
        m.D = st->D;
        m.ghat = st->ghat;
        m.sens = st->sens;
        m.kappa = st->kappa;
        for (int i = 0; i < 27; ++i) m.w[i] = st->w[i];
        m.beta = st->beta;
        m.gamma = st->gamma;
        m.eps = st->eps;
        m.alpha = st->alpha;
        m.delta = st->delta;
        m.n_subf = (float)g->d.n_subsets;
        // resolution model: G x in the geometry's work images, G over gathered
        // images with two work images in each gradient-sheet slot
        m.psf_passes = g->psf_passes;
        for (int p = 0; p < 3; ++p) m.psf[p] = g->psf[p];
        m.psf_a = g->psf_a;
        m.psf_b = g->psf_b;
        b->psf_max = std::max(b->psf_max, g->psf_passes);
        if (g->psf_passes && slot < 2 * (int64_t)g->n_vox) e = hipErrorInvalidValue;
        // LDS of the line bodies: sheets, plus one TOF table per wave
        const int rz = g->d.nz + 2 * PADZ;
        const size_t sheet = ((size_t)g->rows_max * rz + 3) & ~(size_t)3;
        b->lds_base.push_back(3 * sheet * sizeof(float));
        size_t pw = 0;
        if (m.is_tof) {
            const int e1 = g->tof_ws > 4 ? g->tof_ws - 4 : 0;
            pw = (((size_t)g->rows_max * (4 + e1) + tof_cuts_pad(g->tof.n_int) + 3) & ~(size_t)3) * sizeof(float);
        }
        b->lds_per_wave.push_back(pw);
        b->tof_waves.push_back(m.tof_waves);
        b->line_cost.push_back((double)g->n_planes * g->rows_max * (m.is_tof ? 4.0 : 1.0));
    }
    if (e == hipSuccess) e = hipMalloc(&b->d_steps, sizeof(BStep) * (size_t)n_members * b->max_steps);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_steps, sizeof(BStep) * (size_t)n_members * b->max_steps);
    for (int r = 0; r < n_members && e == hipSuccess; ++r) hm[r].steps = b->d_steps + (size_t)r * b->max_steps;
    if (e == hipSuccess) e = hipMalloc(&b->d_mem, sizeof(BMember) * n_members);
    if (e == hipSuccess) e = hipMemcpy(b->d_mem, hm.data(), sizeof(BMember) * n_members, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&b->d_order, sizeof(int) * n_members);
    if (e == hipSuccess) e = hipMalloc(&b->d_counter, sizeof(int));
    if (e == hipSuccess) e = hipMemset(b->d_counter, 0, sizeof(int));
    if (e == hipSuccess) e = upload_order(b);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    b->blocks = std::max(cus, 1);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    for (hipEvent_t *ev : {&b->ev_in, &b->ev_out, &b->ev_copy, &b->ev_t0, &b->ev_t1})
        if (e == hipSuccess) e = hipEventCreate(ev);
    int max_lds = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device);
    if (e == hipSuccess && batch_lds(b, b->waves) > (size_t)max_lds) {
        destroy(b);
        return fail(PET_E_ARG, "pet_batch_create: a member's line sheets exceed the LDS");
    }
    if (e == hipSuccess) e = prime_line_batched(batch_lds(b, b->waves));
    if (e != hipSuccess) {
        destroy(b);
        return hip_check(e, "pet_batch_create");
    }
    *out = b;
    return PET_OK;
}

extern "C" pet_status pet_batch_destroy(pet_batch b) {
    destroy(b);
    return PET_OK;
}

extern "C" pet_status pet_batch_epochs(pet_batch b, int n_rounds, const int32_t *subset_seq, const float *tau,
                                       const uint8_t *update_pc, int use_graph, void *stream) {
    if (!b || !subset_seq || !tau || !update_pc) return fail(PET_E_ARG, "pet_batch_epochs: null argument");
    if (n_rounds < 0) return fail(PET_E_ARG, "pet_batch_epochs: negative round count");
    // host schedule layout: member r's block of n_rounds * n_r entries, members in order
    std::vector<size_t> off(b->n + 1, 0);
    for (int r = 0; r < b->n; ++r) {
        const int nr = b->geoms[r]->d.n_subsets;
        off[r + 1] = off[r] + (size_t)n_rounds * nr;
        if (b->states[r]->k < 0 || b->states[r]->k % nr != 0)
            return fail(PET_E_STATE, "pet_batch_epochs: member iteration counters must sit at epoch starts");
        for (size_t i = off[r]; i < off[r + 1]; ++i)
            if (subset_seq[i] < 0 || subset_seq[i] >= nr)
                return fail(PET_E_ARG, "pet_batch_epochs: subset_seq entry out of range");
    }
    hipStream_t cs = (hipStream_t)stream;
    hipError_t e = hipSetDevice(b->device);
    for (int round = 0; round < n_rounds && e == hipSuccess; ++round) {
        e = wait_copy(b);
        for (int r = 0; r < b->n && e == hipSuccess; ++r) {
            const pet_svrg_state *st = b->states[r];
            const int nr = b->geoms[r]->d.n_subsets;
            const int64_t period = (int64_t)st->omega * nr;
            for (int j = 0; j < b->max_steps; ++j) {
                BStep &s = b->h_steps[(size_t)r * b->max_steps + j];
                if (j >= nr) {
                    s = BStep{0, 0.f, 0, 0};
                    continue;
                }
                const size_t i = off[r] + (size_t)round * nr + j;
                const int64_t k = st->k + j;
                s.subset = subset_seq[i];
                s.tau = tau[i];
                s.flags = B_ACTIVE | (k % period == 0 ? B_SNAP : 0) | (update_pc[i] ? B_UPDATE : 0);
                s.pad = 0;
            }
        }
        if (e == hipSuccess) e = hipEventRecord(b->ev_in, cs);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
        if (e == hipSuccess) e = push_steps(b);
        if (e == hipSuccess) {
            if (use_graph) {
                if (!b->exec) {
                    e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
                    if (e == hipSuccess) {
                        hipError_t ec = enqueue_round(b, b->stream);
                        e = hipStreamEndCapture(b->stream, &b->graph);
                        if (e == hipSuccess) e = ec;
                    }
                    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
                    if (e != hipSuccess) drop_graph(b);
                }
                if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
            } else {
                e = enqueue_round(b, b->stream);
            }
        }
        if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, b->ev_out, 0);
        for (int r = 0; r < b->n && e == hipSuccess; ++r) b->states[r]->k += b->geoms[r]->d.n_subsets;
    }
    return hip_check(e, "pet_batch_epochs");
}

extern "C" pet_status pet_batch_epoch(pet_batch b, const int32_t *subset_seq, const float *tau,
                                      const uint8_t *update_pc, int use_graph, void *stream) {
    return pet_batch_epochs(b, 1, subset_seq, tau, update_pc, use_graph, stream);
}

extern "C" pet_status pet_batch_autotune(pet_batch b, int *config_out, double *best_ms_out, void *stream) {
    if (!b) return fail(PET_E_ARG, "pet_batch_autotune: null batch");
    hipStream_t cs = (hipStream_t)stream;
    hipError_t e = hipSetDevice(b->device);
    if (e == hipSuccess) e = wait_copy(b);
    // a regular step of subset 0 for every member (touches only scratch sheets)
    for (int r = 0; r < b->n; ++r)
        for (int j = 0; j < b->max_steps; ++j)
            b->h_steps[(size_t)r * b->max_steps + j] = BStep{0, 0.f, j == 0 ? B_ACTIVE : 0, 0};
    if (e == hipSuccess) e = hipEventRecord(b->ev_in, cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
    if (e == hipSuccess) e = push_steps(b);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    int max_lds = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device);
    const int saved[3] = {b->blocks, b->waves, b->order_kind};
    int best[3] = {b->blocks, b->waves, b->order_kind};
    float best_ms = 1e30f;
    for (int waves : {16, 12, 8})
        for (int mult : {1, 2})
            for (int ok : {0, 1}) {
                if (e != hipSuccess) break;
                if (batch_lds(b, waves) > (size_t)max_lds) continue;
                b->waves = waves;
                b->blocks = std::max(cus, 1) * mult;
                b->order_kind = ok;
                e = upload_order(b);
                float ms = 0.f;
                for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
                    e = launch_b_prep(b->d_mem, b->n, 0, b->d_counter, b->psf_max, b->stream);
                    if (e == hipSuccess) e = hipEventRecord(b->ev_t0, b->stream);
                    if (e == hipSuccess)
                        e = launch_line_batched(b->d_mem, b->d_order, b->n, 0, b->d_counter, b->blocks, b->waves,
                                                batch_lds(b, b->waves), b->stream);
                    if (e == hipSuccess) e = hipEventRecord(b->ev_t1, b->stream);
                    if (e == hipSuccess) e = hipEventSynchronize(b->ev_t1);
                    float t = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&t, b->ev_t0, b->ev_t1);
                    if (rep > 0) ms += t;  // first repetition warms up
                }
                if (e == hipSuccess && ms / 2.f < best_ms) {
                    best_ms = ms / 2.f;
                    best[0] = b->blocks;
                    best[1] = b->waves;
                    best[2] = b->order_kind;
                }
            }
    if (e != hipSuccess) {
        b->blocks = saved[0];
        b->waves = saved[1];
        b->order_kind = saved[2];
        (void)upload_order(b);
        return hip_check(e, "pet_batch_autotune");
    }
    b->blocks = best[0];
    b->waves = best[1];
    b->order_kind = best[2];
    e = upload_order(b);
    drop_graph(b);  // launch shapes are baked into a captured round
    if (config_out) {
        config_out[0] = b->blocks;
        config_out[1] = b->waves;
        config_out[2] = b->order_kind;
    }
    if (best_ms_out) *best_ms_out = best_ms;
    if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, b->ev_out, 0);
    return hip_check(e, "pet_batch_autotune");
}

extern "C" pet_status pet_batch_set_launch(pet_batch b, int workgroups, int waves, int order) {
    if (!b) return fail(PET_E_ARG, "pet_batch_set_launch: null batch");
    if (workgroups < 1 || waves < 1 || waves > TOF_MAX_WAVES || (order != 0 && order != 1))
        return fail(PET_E_ARG, "pet_batch_set_launch: workgroups >= 1, 1 <= waves <= 16, order 0 or 1");
    int max_lds = 0;
    hipError_t e = hipSetDevice(b->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device);
    if (e == hipSuccess && batch_lds(b, waves) > (size_t)max_lds)
        return fail(PET_E_ARG, "pet_batch_set_launch: too many waves for the LDS");
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_check(e, "pet_batch_set_launch");
    b->blocks = workgroups;
    b->waves = waves;
    b->order_kind = order;
    drop_graph(b);
    return hip_check(upload_order(b), "pet_batch_set_launch");
}
