// Image-space kernels of a batch of reconstructions: one launch per kernel and
// step for all members that are active at the step.  Each launch walks the
// concatenation of the active members' index ranges with a grid-stride loop;
// every workgroup first forms the prefix sums of the ranges (at most BATCH_MAX
// members) in LDS.
//
// Per step of Algorithm 1 (Appendix B) with the clipped step of eq. (sgm):
//   prep    image sheets from x (from G x with a resolution model), zero the
//           gradient-sheet slots in use, zero the line kernel's work counter
//   (line)  subset gradients (proj.hip, k_line_batched)
//   gather  slot 0 -> g (regular step) or every slot s -> ghat_s and
//           ghat = sum_s ghat_s in FP64 (snapshot step); with a resolution
//           model the gathered images pass through G (G^T = G) before the
//           FP64 sum, with the slots' memory as work space
//   step    RDP gradient (+ Hessian diagonal and eq. (preconditioner) at an
//           update), estimator and clipped step into xtmp
//   commit  x <- xtmp
#include "pet_internal.h"

namespace pet {
namespace {

constexpr int B_BLOCK = 256;
constexpr int B_GRID = 2048;

enum Range { R_VOX, R_SLOTS, R_PSF_X, R_PSF_G, R_PSF_SUM };

// Prefix sums over members of the index range each kernel covers at `step`.
// The resolution-model ranges cover the members with more than `pass` passes:
// their image (R_PSF_X), their gathered images (R_PSF_G: n_sub at a snapshot,
// else one) or, at a snapshot, the FP64 sum (R_PSF_SUM).
__device__ __forceinline__ int64_t member_ranges(const BMember *mem, int n_mem, int step, Range what,
                                                 int64_t *cum, int pass = 0) {
    if (threadIdx.x == 0) {
        int64_t c = 0;
        for (int q = 0; q < n_mem; ++q) {
            cum[q] = c;
            const BStep st = mem[q].steps[step];
            if (st.flags & B_ACTIVE) {
                const bool snap = (st.flags & B_SNAP) != 0;
                const bool psf = mem[q].psf_passes > pass;
                if (what == R_VOX)
                    c += mem[q].n_vox;
                else if (what == R_SLOTS)
                    c += mem[q].g_slot * (snap ? mem[q].n_sub : 1);
                else if (what == R_PSF_X)
                    c += psf ? mem[q].n_vox : 0;
                else if (what == R_PSF_G)
                    c += psf ? mem[q].n_vox * (snap ? mem[q].n_sub : 1) : 0;
                else
                    c += psf && snap ? mem[q].n_vox : 0;
            }
        }
        cum[n_mem] = c;
    }
    __syncthreads();
    return cum[n_mem];
}

__device__ __forceinline__ int member_of(const int64_t *cum, int n_mem, int64_t i) {
    int q = 0;
    while (q + 1 < n_mem && cum[q + 1] <= i) ++q;
    return q;
}

__device__ __forceinline__ float sheet_at(const BMember &m, int64_t slot_off, int ix, int iy, int iz) {
    const int rz = m.nz + 2 * PADZ;
    const float *G0 = m.pa.G0 + slot_off, *G1 = m.pa.G1 + slot_off;
    return G1[((size_t)iy * (m.nx + 2 * PADA) + ix + PADA) * rz + iz + PADZ] +
           G0[((size_t)ix * (m.ny + 2 * PADA) + iy + PADA) * rz + iz + PADZ];
}

// One axis pass of the resolution model (Section 3.1) at voxel v of an
// nx * ny * nz image: sum_{|d| <= r} w[|d|] in[v + d e_axis], zero outside the
// grid (the same sum, in the same order, as the single-geometry pass).
__device__ __forceinline__ float psf_axis_at(const float *in, int64_t v, int nx, int ny, int nz, const PsfAxis &k) {
    const int64_t stride = k.axis == 0 ? 1 : (k.axis == 1 ? nx : (int64_t)nx * ny);
    const int len = k.axis == 0 ? nx : (k.axis == 1 ? ny : nz);
    const int c = (int)((v / stride) % len);
    const int lo = -min(c, k.r), hi = min(len - 1 - c, k.r);
    float acc = 0.f;
    for (int d = lo; d <= hi; ++d) acc = fmaf(k.w[d < 0 ? -d : d], in[v + d * stride], acc);
    return acc;
}

// The image the sheets are built from: x, or G x after the last pass of
// k_b_psf_x (psf_a after three passes, psf_b after two).
__device__ __forceinline__ const float *sheet_source(const BMember &m) {
    if (!m.psf_passes) return m.x;
    return m.psf_passes % 2 == 1 ? m.psf_a : m.psf_b;
}

// Pass `pass` of G x: x -> psf_a -> psf_b [-> psf_a].
__global__ void __launch_bounds__(B_BLOCK) k_b_psf_x(const BMember *__restrict__ mem, int n_mem, int step, int pass) {
    __shared__ int64_t cum[BATCH_MAX + 1];
    const int64_t total = member_ranges(mem, n_mem, step, R_PSF_X, cum, pass);
    for (int64_t i = blockIdx.x * (int64_t)B_BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * B_BLOCK) {
        const int q = member_of(cum, n_mem, i);
        const BMember &m = mem[q];
        const int64_t v = i - cum[q];
        const float *src = pass == 0 ? m.x : (pass % 2 == 1 ? m.psf_a : m.psf_b);
        float *dst = pass % 2 == 0 ? m.psf_a : m.psf_b;
        dst[v] = psf_axis_at(src, v, m.nx, m.ny, m.nz, m.psf[pass]);
    }
}

// Pass `pass` of G over the gathered images I (g, or ghat_s for every slot s
// at a snapshot), in place through two work images A_s, B_s held in slot s's
// memory (free once gathered; a slot holds at least two images):
// I -> A_s -> I (two passes) or I -> A_s -> B_s -> I (three).
__global__ void __launch_bounds__(B_BLOCK) k_b_psf_g(const BMember *__restrict__ mem, int n_mem, int step, int pass) {
    __shared__ int64_t cum[BATCH_MAX + 1];
    const int64_t total = member_ranges(mem, n_mem, step, R_PSF_G, cum, pass);
    for (int64_t i = blockIdx.x * (int64_t)B_BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * B_BLOCK) {
        const int q = member_of(cum, n_mem, i);
        const BMember &m = mem[q];
        const int64_t l = i - cum[q];
        const int64_t sl = l / m.n_vox, v = l - sl * m.n_vox;
        float *img = (m.steps[step].flags & B_SNAP) ? m.ghat_i + (size_t)sl * m.n_vox : m.g;
        float *A = m.pa.G0 + (size_t)sl * m.g_slot, *B = A + m.n_vox;
        const bool last = pass == m.psf_passes - 1;
        const float *src = pass == 0 ? img : (pass % 2 == 1 ? A : B);
        float *dst = last ? img : (pass % 2 == 0 ? A : B);
        dst[v] = psf_axis_at(src, v, m.nx, m.ny, m.nz, m.psf[pass]);
    }
}

// Snapshot with a resolution model: ghat = sum_s ghat_s in FP64, after G.
__global__ void __launch_bounds__(B_BLOCK) k_b_psf_sum(const BMember *__restrict__ mem, int n_mem, int step) {
    __shared__ int64_t cum[BATCH_MAX + 1];
    const int64_t total = member_ranges(mem, n_mem, step, R_PSF_SUM, cum);
    for (int64_t i = blockIdx.x * (int64_t)B_BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * B_BLOCK) {
        const int q = member_of(cum, n_mem, i);
        const BMember &m = mem[q];
        const int64_t v = i - cum[q];
        double sum = 0.0;
        for (int s = 0; s < m.n_sub; ++s) sum += (double)m.ghat_i[(size_t)s * m.n_vox + v];
        m.ghat[v] = sum;
    }
}

__global__ void __launch_bounds__(B_BLOCK) k_b_to_sheets(const BMember *__restrict__ mem, int n_mem, int step) {
    __shared__ int64_t cum[BATCH_MAX + 1];
    const int64_t total = member_ranges(mem, n_mem, step, R_VOX, cum);
    for (int64_t i = blockIdx.x * (int64_t)B_BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * B_BLOCK) {
        const int q = member_of(cum, n_mem, i);
        const BMember &m = mem[q];
        const int64_t v = i - cum[q];
        const int ix = v % m.nx, iy = (v / m.nx) % m.ny, iz = v / ((int64_t)m.nx * m.ny);
        const int rz = m.nz + 2 * PADZ;
        const float val = sheet_source(m)[v];
        float *T0 = const_cast<float *>(m.pa.T0), *T1 = const_cast<float *>(m.pa.T1);
        T0[((size_t)ix * (m.ny + 2 * PADA) + iy + PADA) * rz + iz + PADZ] = val;
        T1[((size_t)iy * (m.nx + 2 * PADA) + ix + PADA) * rz + iz + PADZ] = val;
    }
}

__global__ void __launch_bounds__(B_BLOCK) k_b_zero_slots(const BMember *__restrict__ mem, int n_mem, int step,
                                                          int *__restrict__ counter) {
    __shared__ int64_t cum[BATCH_MAX + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
    const int64_t total = member_ranges(mem, n_mem, step, R_SLOTS, cum);
    for (int64_t i = blockIdx.x * (int64_t)B_BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * B_BLOCK) {
        const int q = member_of(cum, n_mem, i);
        mem[q].pa.G0[i - cum[q]] = 0.f;
    }
}

__global__ void __launch_bounds__(B_BLOCK) k_b_gather(const BMember *__restrict__ mem, int n_mem, int step) {
    __shared__ int64_t cum[BATCH_MAX + 1];
    const int64_t total = member_ranges(mem, n_mem, step, R_VOX, cum);
    for (int64_t i = blockIdx.x * (int64_t)B_BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * B_BLOCK) {
        const int q = member_of(cum, n_mem, i);
        const BMember &m = mem[q];
        const int64_t v = i - cum[q];
        const int ix = v % m.nx, iy = (v / m.nx) % m.ny, iz = v / ((int64_t)m.nx * m.ny);
        if (m.steps[step].flags & B_SNAP) {
            double sum = 0.0;
            for (int s = 0; s < m.n_sub; ++s) {
                const float gs = sheet_at(m, (int64_t)s * m.g_slot, ix, iy, iz);
                m.ghat_i[(size_t)s * m.n_vox + v] = gs;
                sum += (double)gs;
            }
            if (!m.psf_passes) m.ghat[v] = sum;
        } else {
            m.g[v] = sheet_at(m, 0, ix, iy, iz);
        }
    }
}

// RDP stencil (eq. (rdp), Appendix A) of member m at voxel v with the fused
// preconditioner update and clipped SVRG step.
__device__ __forceinline__ void member_step(const BMember &m, const BStep &st, int64_t v) {
    const int ix = v % m.nx, iy = (v / m.nx) % m.ny, iz = v / ((int64_t)m.nx * m.ny);
    const float xi = m.x[v];
    const float ki = m.kappa ? m.kappa[v] : 1.f;
    float g = 0.f, h = 0.f;
    const bool upd = (st.flags & B_UPDATE) != 0;
    for (int dz = -1; dz <= 1; ++dz) {
        const int jz = iz + dz;
        if (jz < 0 || jz >= m.nz) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int jy = iy + dy;
            if (jy < 0 || jy >= m.ny) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                const int jx = ix + dx;
                if (jx < 0 || jx >= m.nx) continue;
                const int64_t u = ((int64_t)jz * m.ny + jy) * m.nx + jx;
                const float xj = m.x[u];
                const float wk = m.w[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] * ki * (m.kappa ? m.kappa[u] : 1.f);
                const float d = xi - xj;
                const float ad = fabsf(d);
                const float phi = xi + xj + m.gamma * ad + m.eps;
                const float rphi = 1.f / phi;
                g = fmaf(wk * d * (2.f * phi - (d + m.gamma * ad)), rphi * rphi, g);
                if (upd) {
                    const float c = 2.f * xj + m.eps;
                    h = fmaf(2.f * wk * c * c, rphi * rphi * rphi, h);
                }
            }
        }
    }
    const float bg = m.beta * g;
    float Dv;
    if (upd) {
        const float xd = xi + m.delta;
        const float den = m.sens[v] + m.alpha * (m.beta * h) * xd;
        Dv = den != 0.f ? xd / den : 0.f;
        m.D[v] = Dv;
    } else {
        Dv = m.D[v];
    }
    float est;
    if (st.flags & B_SNAP)
        est = (float)m.ghat[v] + bg;
    else
        est = fmaf(m.n_subf, m.g[v] - m.ghat_i[(size_t)st.subset * m.n_vox + v], (float)m.ghat[v]) + bg;
    m.xtmp[v] = fmaxf(0.f, fmaf(-st.tau * Dv, est, xi));
}

__global__ void __launch_bounds__(B_BLOCK) k_b_step(const BMember *__restrict__ mem, int n_mem, int step) {
    __shared__ int64_t cum[BATCH_MAX + 1];
    const int64_t total = member_ranges(mem, n_mem, step, R_VOX, cum);
    for (int64_t i = blockIdx.x * (int64_t)B_BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * B_BLOCK) {
        const int q = member_of(cum, n_mem, i);
        member_step(mem[q], mem[q].steps[step], i - cum[q]);
    }
}

__global__ void __launch_bounds__(B_BLOCK) k_b_commit(const BMember *__restrict__ mem, int n_mem, int step) {
    __shared__ int64_t cum[BATCH_MAX + 1];
    const int64_t total = member_ranges(mem, n_mem, step, R_VOX, cum);
    for (int64_t i = blockIdx.x * (int64_t)B_BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * B_BLOCK) {
        const int q = member_of(cum, n_mem, i);
        const int64_t v = i - cum[q];
        mem[q].x[v] = mem[q].xtmp[v];
    }
}

}  // namespace

hipError_t launch_b_prep(const BMember *mem, int n_mem, int step, int *counter, int psf_max, hipStream_t s) {
    for (int p = 0; p < psf_max; ++p)
        hipLaunchKernelGGL(k_b_psf_x, dim3(B_GRID), dim3(B_BLOCK), 0, s, mem, n_mem, step, p);
    hipLaunchKernelGGL(k_b_to_sheets, dim3(B_GRID), dim3(B_BLOCK), 0, s, mem, n_mem, step);
    hipLaunchKernelGGL(k_b_zero_slots, dim3(B_GRID), dim3(B_BLOCK), 0, s, mem, n_mem, step, counter);
    return hipGetLastError();
}

hipError_t launch_b_gather(const BMember *mem, int n_mem, int step, int psf_max, hipStream_t s) {
    hipLaunchKernelGGL(k_b_gather, dim3(B_GRID), dim3(B_BLOCK), 0, s, mem, n_mem, step);
    for (int p = 0; p < psf_max; ++p)
        hipLaunchKernelGGL(k_b_psf_g, dim3(B_GRID), dim3(B_BLOCK), 0, s, mem, n_mem, step, p);
    if (psf_max) hipLaunchKernelGGL(k_b_psf_sum, dim3(B_GRID), dim3(B_BLOCK), 0, s, mem, n_mem, step);
    return hipGetLastError();
}

hipError_t launch_b_step(const BMember *mem, int n_mem, int step, hipStream_t s) {
    hipLaunchKernelGGL(k_b_step, dim3(B_GRID), dim3(B_BLOCK), 0, s, mem, n_mem, step);
    return hipGetLastError();
}

hipError_t launch_b_commit(const BMember *mem, int n_mem, int step, hipStream_t s) {
    hipLaunchKernelGGL(k_b_commit, dim3(B_GRID), dim3(B_BLOCK), 0, s, mem, n_mem, step);
    return hipGetLastError();
}

}  // namespace pet
