// Reverse-mode kernels for the unrolled preconditioned SVRG: the Hessian-vector
// product of the relative difference prior, the vector-Jacobian product of the
// prior-aware preconditioner, and the elementwise reverse of the clipped step.
//
// Notation (eq. (rdp), Appendix A): for voxel i and neighbour j with weight w
// and kappa_i kappa_j, d = x_i - x_j, psi = x_i + x_j + gamma |d| + eps,
// c_j = 2 x_j + eps.  Then
//   dS/dx_i        = sum_j w kk d (2 psi - d - gamma |d|) / psi^2
//   d2S/dx_i^2     = h_i = 2 sum_j w kk c_j^2 / psi^3
//   d2S/dx_i dx_j  = -2 w kk c_i c_j / psi^3            (j a neighbour of i)
// so (H v)_i = sum_j 2 w kk c_j / psi^3 (c_j v_i - c_i v_j).
#include "pet_internal.h"

namespace pet {
namespace {

constexpr int ADJ_BLOCK = 256;

struct W27a {
    float w[27];
};

struct StencilArgs {
    const float *x, *kappa;
    W27a w;
    float beta, gamma, eps;
    int nx, ny, nz;
};

__device__ __forceinline__ float sgnf(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

// out (+)= beta H_S(x) v; partial[block] = sum over the block of dS/dx_i v_i
// (unscaled by beta), FP64.
__global__ void __launch_bounds__(ADJ_BLOCK) k_rdp_hvp(StencilArgs a, const float *__restrict__ v,
                                                       float *__restrict__ out, int accumulate,
                                                       double *__restrict__ partial) {
    const int64_t n = (int64_t)a.nx * a.ny * a.nz;
    const int64_t i = blockIdx.x * (int64_t)ADJ_BLOCK + threadIdx.x;
    double dot = 0.0;
    if (i < n) {
        const int ix = i % a.nx, iy = (i / a.nx) % a.ny, iz = i / ((int64_t)a.nx * a.ny);
        const float xi = a.x[i], vi = v[i];
        const float ki = a.kappa ? a.kappa[i] : 1.f;
        const float ci = 2.f * xi + a.eps;
        float hv = 0.f, g = 0.f;
        for (int dz = -1; dz <= 1; ++dz) {
            const int jz = iz + dz;
            if (jz < 0 || jz >= a.nz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int jy = iy + dy;
                if (jy < 0 || jy >= a.ny) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0 && dz == 0) continue;
                    const int jx = ix + dx;
                    if (jx < 0 || jx >= a.nx) continue;
                    const int64_t j = ((int64_t)jz * a.ny + jy) * a.nx + jx;
                    const float xj = a.x[j];
                    const float wk = a.w.w[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] * ki * (a.kappa ? a.kappa[j] : 1.f);
                    const float d = xi - xj, ad = fabsf(d);
                    const float psi = xi + xj + a.gamma * ad + a.eps;
                    const float r = 1.f / psi;
                    const float cj = 2.f * xj + a.eps;
                    hv = fmaf(2.f * wk * cj * r * r * r, cj * vi - ci * v[j], hv);
                    if (partial) g = fmaf(wk * d * (2.f * psi - (d + a.gamma * ad)), r * r, g);
                }
            }
        }
        const float o = a.beta * hv;
        out[i] = accumulate ? out[i] + o : o;
        dot = (double)g * (double)vi;
    }
    if (partial) {
        __shared__ double red[ADJ_BLOCK / 64];
        for (int off = 32; off > 0; off >>= 1) dot += __shfl_down(dot, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dot;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < ADJ_BLOCK / 64; ++w) s += red[w];
            partial[blockIdx.x] = s;
        }
    }
}

// Preconditioner D_j = N_j / M_j with N_j = x_j + delta and
// M_j = sens_j + alpha beta h_j(x) N_j (D_j = 0 where M_j = 0).  Pass 1, per
// voxel j: xbar_j += Dbar_j (1 / M_j - alpha beta h_j N_j / M_j^2),
// e_j = Dbar_j alpha beta N_j^2 / M_j^2, and the per-block FP64 partial of
// dL/dbeta = sum_j Dbar_j (-alpha h_j N_j^2 / M_j^2).
__global__ void __launch_bounds__(ADJ_BLOCK) k_precond_vjp1(StencilArgs a, const float *__restrict__ sens,
                                                            float alpha, float delta, const float *__restrict__ Dbar,
                                                            float *__restrict__ xbar, float *__restrict__ e_out,
                                                            double *__restrict__ partial) {
    const int64_t n = (int64_t)a.nx * a.ny * a.nz;
    const int64_t i = blockIdx.x * (int64_t)ADJ_BLOCK + threadIdx.x;
    double bb = 0.0;
    if (i < n) {
        const int ix = i % a.nx, iy = (i / a.nx) % a.ny, iz = i / ((int64_t)a.nx * a.ny);
        const float xi = a.x[i];
        const float ki = a.kappa ? a.kappa[i] : 1.f;
        float h = 0.f;
        for (int dz = -1; dz <= 1; ++dz) {
            const int jz = iz + dz;
            if (jz < 0 || jz >= a.nz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int jy = iy + dy;
                if (jy < 0 || jy >= a.ny) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0 && dz == 0) continue;
                    const int jx = ix + dx;
                    if (jx < 0 || jx >= a.nx) continue;
                    const int64_t j = ((int64_t)jz * a.ny + jy) * a.nx + jx;
                    const float xj = a.x[j];
                    const float wk = a.w.w[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] * ki * (a.kappa ? a.kappa[j] : 1.f);
                    const float psi = xi + xj + a.gamma * fabsf(xi - xj) + a.eps;
                    const float r = 1.f / psi;
                    const float cj = 2.f * xj + a.eps;
                    h = fmaf(2.f * wk * cj * cj, r * r * r, h);
                }
            }
        }
        const float N = xi + delta;
        const float ab = alpha * a.beta;
        const float M = sens[i] + ab * h * N;
        const float db = Dbar[i];
        float e = 0.f;
        if (M != 0.f) {
            const float rM = 1.f / M;
            xbar[i] += db * (rM - ab * h * N * rM * rM);
            e = db * ab * N * N * rM * rM;
            bb = -(double)db * (double)alpha * (double)h * (double)N * (double)N * (double)rM * (double)rM;
        }
        e_out[i] = e;
    }
    __shared__ double red[ADJ_BLOCK / 64];
    for (int off = 32; off > 0; off >>= 1) bb += __shfl_down(bb, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = bb;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < ADJ_BLOCK / 64; ++w) s += red[w];
        partial[blockIdx.x] = s;
    }
}

// Pass 2: xbar_m -= sum_j e_j dh_j/dx_m, i.e. over neighbours k of m
//   2 w kk [ -3 e_m c_k^2 (1 + gamma s) / psi^4 + e_k (4 c_m / psi^3 - 3 c_m^2 (1 + gamma s) / psi^4) ]
// with s = sign(x_m - x_k) (sign(0) = 0).
__global__ void __launch_bounds__(ADJ_BLOCK) k_precond_vjp2(StencilArgs a, const float *__restrict__ e,
                                                            float *__restrict__ xbar) {
    const int64_t n = (int64_t)a.nx * a.ny * a.nz;
    const int64_t m = blockIdx.x * (int64_t)ADJ_BLOCK + threadIdx.x;
    if (m >= n) return;
    const int ix = m % a.nx, iy = (m / a.nx) % a.ny, iz = m / ((int64_t)a.nx * a.ny);
    const float xm = a.x[m], em = e[m];
    const float km = a.kappa ? a.kappa[m] : 1.f;
    const float cm = 2.f * xm + a.eps;
    float acc = 0.f;
    for (int dz = -1; dz <= 1; ++dz) {
        const int jz = iz + dz;
        if (jz < 0 || jz >= a.nz) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int jy = iy + dy;
            if (jy < 0 || jy >= a.ny) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                const int jx = ix + dx;
                if (jx < 0 || jx >= a.nx) continue;
                const int64_t k = ((int64_t)jz * a.ny + jy) * a.nx + jx;
                const float xk = a.x[k];
                const float wk = a.w.w[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] * km * (a.kappa ? a.kappa[k] : 1.f);
                const float dlt = xm - xk;
                const float psi = xm + xk + a.gamma * fabsf(dlt) + a.eps;
                const float r = 1.f / psi;
                const float r3 = r * r * r, r4 = r3 * r;
                const float q = 1.f + a.gamma * sgnf(dlt);
                const float ck = 2.f * xk + a.eps;
                acc = fmaf(2.f * wk, -3.f * em * ck * ck * q * r4 + e[k] * (4.f * cm * r3 - 3.f * cm * cm * q * r4), acc);
            }
        }
    }
    xbar[m] -= acc;
}

// Reverse of x_next = max(0, x - tau D est):
//   u = xbar_next [x_next > 0]   (a tie at 0 passes nothing)
//   Dbar += -tau u est;  v = -tau D u;  xbar = u
__global__ void k_step_vjp(const float *__restrict__ x_next, const float *__restrict__ D,
                           const float *__restrict__ est, float tau, float *__restrict__ xbar,
                           float *__restrict__ Dbar, float *__restrict__ v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float u = x_next[i] > 0.f ? xbar[i] : 0.f;
        Dbar[i] = fmaf(-tau * u, est[i], Dbar[i]);
        v[i] = -tau * D[i] * u;
        xbar[i] = u;
    }
}

// out = ca a + cb b (b nullable -> out = ca a)
__global__ void k_lincomb(float *__restrict__ out, float ca, const float *__restrict__ a, float cb,
                          const float *__restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = b ? fmaf(ca, a[i], cb * b[i]) : ca * a[i];
}

inline dim3 adj_grid(int64_t n) {
    int64_t b = (n + ADJ_BLOCK - 1) / ADJ_BLOCK;
    return dim3((unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 65536));
}

StencilArgs stencil_args(const pet_geom_s *g, const float *x, const float *kappa, const float *w27, float beta,
                         float gamma, float eps) {
    StencilArgs a{};
    a.x = x;
    a.kappa = kappa;
    for (int i = 0; i < 27; ++i) a.w.w[i] = w27[i];
    a.beta = beta;
    a.gamma = gamma;
    a.eps = eps;
    a.nx = g->d.nx;
    a.ny = g->d.ny;
    a.nz = g->d.nz;
    return a;
}

}  // namespace

int adj_blocks(const pet_geom_s *g) { return (int)((g->n_vox + ADJ_BLOCK - 1) / ADJ_BLOCK); }

hipError_t launch_rdp_hvp(const pet_geom_s *g, const float *x, const float *kappa, const float *w27, float beta,
                          float gamma, float eps, const float *v, float *out, int accumulate, double *partial,
                          hipStream_t s) {
    const StencilArgs a = stencil_args(g, x, kappa, w27, beta, gamma, eps);
    hipLaunchKernelGGL(k_rdp_hvp, dim3(adj_blocks(g)), dim3(ADJ_BLOCK), 0, s, a, v, out, accumulate, partial);
    return hipGetLastError();
}

hipError_t launch_precond_vjp(const pet_geom_s *g, const float *x, const float *kappa, const float *w27, float beta,
                              float gamma, float eps, const float *sens, float alpha, float delta,
                              const float *Dbar, float *xbar, float *e_tmp, double *partial, hipStream_t s) {
    const StencilArgs a = stencil_args(g, x, kappa, w27, beta, gamma, eps);
    hipLaunchKernelGGL(k_precond_vjp1, dim3(adj_blocks(g)), dim3(ADJ_BLOCK), 0, s, a, sens, alpha, delta, Dbar, xbar,
                       e_tmp, partial);
    hipLaunchKernelGGL(k_precond_vjp2, dim3(adj_blocks(g)), dim3(ADJ_BLOCK), 0, s, a, e_tmp, xbar);
    return hipGetLastError();
}

hipError_t launch_step_vjp(const pet_geom_s *g, const float *x_next, const float *D, const float *est, float tau,
                           float *xbar, float *Dbar, float *v, hipStream_t s) {
    hipLaunchKernelGGL(k_step_vjp, adj_grid(g->n_vox), dim3(ADJ_BLOCK), 0, s, x_next, D, est, tau, xbar, Dbar, v,
                       g->n_vox);
    return hipGetLastError();
}

hipError_t launch_lincomb(float *out, float ca, const float *a, float cb, const float *b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb, adj_grid(n), dim3(ADJ_BLOCK), 0, s, out, ca, a, cb, b, n);
    return hipGetLastError();
}

}  // namespace pet
