// Image-space kernels for gfx950: transposed sheet images for the line
// kernels, the relative-difference-prior stencil fused with the prior-aware
// preconditioner and the preconditioned SVRG step, snapshot accumulation in
// FP64, the OSEM multiplicative update and deterministic FP64 reductions.
#include "pet_internal.h"

#include <cfloat>

namespace pet {
namespace {

// x [iz][iy][ix] -> T0 [ix][iy + PADA][iz + PADZ] and T1 [iy][ix + PADA][iz + PADZ]
// (interiors only; the zero borders are set once at creation).
// Through LDS tiles: workgroup (32 consecutive x, one y) reads the
// image rows x[z][y][x0 .. x0 + 31] for every z (coalesced along x) and writes,
// per x, the z-contiguous rows of both sheets (coalesced along z).
constexpr int TT = 32;
constexpr int TILE_UNROLL = 8;
__global__ void __launch_bounds__(256) k_to_sheets_t(const float *__restrict__ x, float *__restrict__ T0,
                                                     float *__restrict__ T1, int nx, int ny, int nz, int rz) {
    extern __shared__ float tile[];  // [nz][TT + 1]
    const int x0 = blockIdx.x * TT, iy = blockIdx.y;
    const int w = min(TT, nx - x0);
    // (TILE_UNROLL loads per thread in flight before their LDS writes)
    for (int e0 = threadIdx.x; e0 < nz * TT; e0 += TILE_UNROLL * blockDim.x) {
        float val[TILE_UNROLL];
#pragma unroll
        for (int u = 0; u < TILE_UNROLL; ++u) {
            const int e = e0 + u * blockDim.x;
            const int z = e / TT, xx = e - z * TT;
            val[u] = e < nz * TT && xx < w ? x[((size_t)z * ny + iy) * nx + x0 + xx] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < TILE_UNROLL; ++u) {
            const int e = e0 + u * blockDim.x;
            const int z = e / TT, xx = e - z * TT;
            if (e < nz * TT) tile[z * (TT + 1) + xx] = val[u];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < w * nz; e += blockDim.x) {
        const int xx = e / nz, z = e - xx * nz;
        const float val = tile[z * (TT + 1) + xx];
        const int ix = x0 + xx;
        T0[((size_t)ix * (ny + 2 * PADA) + iy + PADA) * rz + z + PADZ] = val;
        T1[((size_t)iy * (nx + 2 * PADA) + ix + PADA) * rz + z + PADZ] = val;
    }
}

// Sum of the two gradient sheets at the voxels of one workgroup's tile
// (32 consecutive x, one y, every z) into LDS, read z-contiguous.
__device__ __forceinline__ void sheets_to_tile(const float *__restrict__ G0, const float *__restrict__ G1,
                                               float *tile, int x0, int w, int iy, int nx, int ny, int nz, int rz) {
    for (int e0 = threadIdx.x; e0 < w * nz; e0 += TILE_UNROLL * blockDim.x) {
        float a[TILE_UNROLL], b[TILE_UNROLL];
#pragma unroll
        for (int u = 0; u < TILE_UNROLL; ++u) {
            const int e = e0 + u * blockDim.x;
            const int xx = e / nz, z = e - xx * nz;
            const int ix = x0 + xx;
            a[u] = b[u] = 0.f;
            if (e < w * nz) {
                a[u] = G1[((size_t)iy * (nx + 2 * PADA) + ix + PADA) * rz + z + PADZ];
                b[u] = G0[((size_t)ix * (ny + 2 * PADA) + iy + PADA) * rz + z + PADZ];
            }
        }
#pragma unroll
        for (int u = 0; u < TILE_UNROLL; ++u) {
            const int e = e0 + u * blockDim.x;
            const int xx = e / nz, z = e - xx * nz;
            if (e < w * nz) tile[z * (TT + 1) + xx] = a[u] + b[u];
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_from_sheets_t(const float *__restrict__ G0, const float *__restrict__ G1,
                                                       float *__restrict__ out, int nx, int ny, int nz, int rz,
                                                       int accumulate) {
    extern __shared__ float tile[];
    const int x0 = blockIdx.x * TT, iy = blockIdx.y;
    const int w = min(TT, nx - x0);
    sheets_to_tile(G0, G1, tile, x0, w, iy, nx, ny, nz, rz);
    for (int e = threadIdx.x; e < nz * TT; e += blockDim.x) {
        const int z = e / TT, xx = e - z * TT;
        if (xx >= w) continue;
        const size_t v = ((size_t)z * ny + iy) * nx + x0 + xx;
        const float sv = tile[z * (TT + 1) + xx];
        out[v] = accumulate ? out[v] + sv : sv;
    }
}

// Both gradient sheets to zero in one launch: 16-byte stores when both are
// 16-byte aligned and hold a multiple of 4 floats.
__global__ void k_zero2_v4(float4 *__restrict__ a, int64_t na4, float4 *__restrict__ b, int64_t nb4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < na4 + nb4; i += stride) {
        if (i < na4)
            a[i] = z;
        else
            b[i - na4] = z;
    }
}

__global__ void k_zero2(float *__restrict__ a, int64_t na, float *__restrict__ b, int64_t nb) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < na + nb; i += stride) {
        if (i < na)
            a[i] = 0.f;
        else
            b[i - na] = 0.f;
    }
}

__global__ void k_fill(float *__restrict__ p, int64_t n, float val) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = val;
}

struct W27 {
    float w[27];
};

enum RdpFlags {
    R_GRAD_OUT = 1,   // write beta * grad S
    R_HESS_OUT = 2,   // write beta * diag Hess S
    R_VALUE = 4,      // per-block FP64 partial sums of beta * S
    R_PRECOND = 8,    // write D = (x + delta) / (sens + alpha beta H (x + delta))
    R_UPDATE = 16,    // SVRG step with clip into x_out
    R_SNAPSHOT = 32,  // estimator is ghat + beta grad S (snapshot iteration)
    R_EST_OUT = 64,   // also write the estimator (for the reverse pass)
    R_SAGA = 128,     // SAGA estimator and table update (eq. (saga))
    R_SGD = 256,      // SGD estimator n grad J_i
    R_BB_STORE = 512, // keep the snapshot's full gradient in g_prev
    R_BB_DOT = 1024,  // short-BB dots against the previous snapshot; no step
};

struct RdpArgs {
    const float *x, *kappa;
    W27 w;
    float beta, gamma, eps;
    int nx, ny, nz;
    float *grad, *hess;
    double *partial;
    // preconditioner
    const float *sens;
    float alpha, delta;
    float *D;
    // update
    const float *gi, *ghat_i;
    const double *ghat;
    float n_sub, tau;
    float *x_out, *est_out;
    // SAGA: table entry of the sampled subset and the table's FP64 sum
    float *table_i;
    double *table_sum;
    // short Barzilai-Borwein step: previous snapshot image and full gradient,
    // and the current step bound (device, nullable)
    const float *x_snap;
    float *g_prev;
    const double *tau_bb;
};

// RDP sums of one voxel over its 26 neighbours (eq. (rdp); derivatives as in
// Appendix A): with d = x_i - x_j, phi = x_i + x_j + gamma |d| + eps and
// c = 2 x_j + eps (= s - d + eps, s = x_i + x_j),
//   dS/dx_i   += w k_i k_j d (phi + c) / phi^2     (2 phi - d - gamma |d| = phi + c)
//   d2S/dx_i^2 += 2 w k_i k_j c^2 / phi^3
//   S         += 1/2 w k_i k_j d^2 / phi          (each ordered pair once, halved).
// Branch-free: neighbour coordinates are clamped to the grid and a neighbour
// outside it gets 1 / phi = 0, so it adds nothing.  1 / phi is the hardware
// reciprocal, within 1 ulp.
template <int F, bool KAPPA>
__device__ __forceinline__ void rdp_sums(const RdpArgs &a, int v, int ix, int iy, int iz, float xi, float &g, float &h,
                                         float &sv) {
    const int nxy = a.nx * a.ny;
    const float ki = KAPPA ? a.kappa[v] : 1.f;
    const float xe = xi + a.eps;
    int jz[3], jy[3], jx[3];
    bool oz[3], oy[3], ox[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int z = iz + k - 1, y = iy + k - 1, x = ix + k - 1;
        oz[k] = z >= 0 && z < a.nz;
        oy[k] = y >= 0 && y < a.ny;
        ox[k] = x >= 0 && x < a.nx;
        jz[k] = min(max(z, 0), a.nz - 1) * nxy;
        jy[k] = min(max(y, 0), a.ny - 1) * a.nx;
        jx[k] = min(max(x, 0), a.nx - 1);
    }
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int rowb = jz[dz] + jy[dy];
            const bool ozy = oz[dz] && oy[dy];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                if (dz == 1 && dy == 1 && dx == 1) continue;
                const int u = rowb + jx[dx];
                const float xj = a.x[u];
                float wk = a.w.w[dz * 9 + dy * 3 + dx];
                if (KAPPA) wk *= ki * a.kappa[u];
                const float d = xi - xj;
                const float phi = fmaf(a.gamma, fabsf(d), xe + xj);
                const float r = ozy && ox[dx] ? __builtin_amdgcn_rcpf(phi) : 0.f;
                const float c = fmaf(2.f, xj, a.eps);
                const float r2 = r * r;
                g = fmaf(wk * d * (phi + c), r2, g);
                if (F & (R_HESS_OUT | R_PRECOND)) h = fmaf(2.f * wk * c * c, r2 * r, h);
                if (F & R_VALUE) sv = fmaf(wk * d * d, r, sv);
            }
        }
    }
}

// What the flags ask for at one voxel once its RDP sums are known (gradient,
// Hessian diagonal, value, preconditioner, the fused estimator and step).
// gi: the sampled subset's data gradient at the voxel (regular iterations).
// Returns the new iterate (xi when no step is taken).
template <int F>
__device__ __forceinline__ float rdp_finish(const RdpArgs &a, int v, float xi, float g, float h, float sv, float gi,
                                            double &val, double &pq, double &qdq) {
    const float bg = a.beta * g;
    const float bh = a.beta * h;
    if (F & R_GRAD_OUT) a.grad[v] = bg;
    if (F & R_HESS_OUT) a.hess[v] = bh;
    if (F & R_VALUE) val = 0.5 * (double)a.beta * (double)sv;
    float Dv = 0.f;
    if (F & R_PRECOND) {
        const float xd = xi + a.delta;
        const float den = a.sens[v] + a.alpha * bh * xd;
        Dv = den != 0.f ? xd / den : 0.f;
        a.D[v] = Dv;
    } else if (F & R_UPDATE) {
        Dv = a.D[v];
    }
    float xn = xi;
    if (F & R_UPDATE) {
        float est;
        if (F & R_SAGA) {
            // J_i = D_i + (beta / n) S, eq. (template); the table holds
            // grad J_i at the iterate where subset i was last sampled
            if (F & R_SNAPSHOT) {
                est = (float)a.table_sum[v];  // first iteration: table just filled at x
            } else {
                const float ji = gi + bg / a.n_sub;
                const float ti = a.table_i[v];
                est = fmaf(a.n_sub, ji - ti, (float)a.table_sum[v]);
                a.table_sum[v] += (double)ji - (double)ti;
                a.table_i[v] = ji;
            }
        } else if (F & R_SGD) {
            // (table_i: the part of the subset's data gradient that the
            // sheets do not hold, its sensitivity on the zero-count-aware path)
            est = fmaf(a.n_sub, a.table_i ? gi + a.table_i[v] : gi, bg);
        } else if (F & R_SNAPSHOT) {
            est = (float)a.ghat[v] + bg;
        } else {
            est = fmaf(a.n_sub, gi - a.ghat_i[v], (float)a.ghat[v]) + bg;
        }
        if (F & R_EST_OUT) a.est_out[v] = est;
        if (F & R_BB_DOT) {
            // p = x - x_snap_prev, q = est - g_prev (both full gradients)
            const double p = (double)xi - (double)a.x_snap[v];
            const double q = (double)est - (double)a.g_prev[v];
            pq = p * q;
            qdq = q * q * (double)Dv;
        }
        if (F & (R_BB_STORE | R_BB_DOT)) a.g_prev[v] = est;
        if (!(F & R_BB_DOT)) {
            const float tau = a.tau_bb ? fminf(a.tau, (float)*a.tau_bb) : a.tau;
            xn = fmaxf(0.f, fmaf(-tau * Dv, est, xi));
            a.x_out[v] = xn;
        }
    }
    return xn;
}

// Whether the estimator of these flags reads the sampled subset's gradient.
template <int F>
constexpr bool reads_gi() {
    return (F & R_UPDATE) && !(F & R_SNAPSHOT);
}

// One thread per voxel: the RDP sums, then what the flags ask for (gradient,
// Hessian diagonal, value, preconditioner, the fused estimator and step).
// (32-bit voxel indices: images hold fewer than 2^31 voxels)
template <int F>
__global__ void __launch_bounds__(IMG_BLOCK) k_rdp(RdpArgs a) {
    const int nxy = a.nx * a.ny;
    const int n = nxy * a.nz;
    const int v = blockIdx.x * IMG_BLOCK + threadIdx.x;
    double val = 0.0, pq = 0.0, qdq = 0.0;
    if (v < n) {
        const int iz = v / nxy;
        const int rem = v - iz * nxy;
        const int iy = rem / a.nx;
        const int ix = rem - iy * a.nx;
        const float xi = a.x[v];
        float g = 0.f, h = 0.f, sv = 0.f;
        if (a.kappa)
            rdp_sums<F, true>(a, v, ix, iy, iz, xi, g, h, sv);
        else
            rdp_sums<F, false>(a, v, ix, iy, iz, xi, g, h, sv);
        (void)rdp_finish<F>(a, v, xi, g, h, sv, reads_gi<F>() ? a.gi[v] : 0.f, val, pq, qdq);
    }
    if (F & R_BB_DOT) {
        __shared__ double red2[2][IMG_BLOCK / 64];
        for (int off = 32; off > 0; off >>= 1) {
            pq += __shfl_down(pq, off, 64);
            qdq += __shfl_down(qdq, off, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            red2[0][threadIdx.x >> 6] = pq;
            red2[1][threadIdx.x >> 6] = qdq;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int w = 0; w < IMG_BLOCK / 64; ++w) {
                s0 += red2[0][w];
                s1 += red2[1][w];
            }
            a.partial[blockIdx.x] = s0;
            a.partial[gridDim.x + blockIdx.x] = s1;
        }
    }
    if (F & R_VALUE) {
        __shared__ double red[IMG_BLOCK / 64];
        for (int off = 32; off > 0; off >>= 1) val += __shfl_down(val, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = val;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < IMG_BLOCK / 64; ++w) s += red[w];
            a.partial[blockIdx.x] = s;
        }
    }
}

// ---- the step of an iteration fused with the sheet conversions -------------
// Workgroup: the voxels of one tile (TT consecutive x, one y, every z), as in
// the sheet transposes.  It
//  * sums the subset's data gradient from the two gradient sheets into LDS
//    (reads z-contiguous) and clears the cells it read, so that the next
//    subset's line kernels start from zero sheets;
//  * stages the iterate with a one-voxel halo (three y rows, TT + 2 x, nz + 2 z)
//    in LDS for the 26-neighbour RDP sums;
//  * takes the step of rdp_finish for every voxel of the tile;
//  * writes the new iterate as an image and, through LDS, as the two
//    transposed image sheets that the next subset's line kernels read.
// Without a kappa image and a resolution model; no block reductions.
constexpr int STEP_BLOCK = 512;

__host__ __device__ constexpr int halo_elems(int nz) { return 3 * (nz + 2) * (TT + 2); }

template <int F>
__global__ void __launch_bounds__(STEP_BLOCK) k_step_tile(RdpArgs a, float *__restrict__ G0, float *__restrict__ G1,
                                                         float *__restrict__ T0, float *__restrict__ T1, int rz) {
    extern __shared__ float lds[];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    float *halo = lds;                          // [3][nz + 2][TT + 2]
    float *tile = lds + halo_elems(nz);         // [nz][TT + 1]: gradient in, new iterate out
    const int x0 = blockIdx.x * TT, iy = blockIdx.y;
    const int w = min(TT, nx - x0);
    const int hz = nz + 2, hx = TT + 2;
    // halo of the iterate (outside the grid: 0, masked out by the sums):
    // thread t takes column t mod hx of every (blockDim / hx)-th row of each
    // y slice, TILE_UNROLL loads in flight before their LDS writes
    {
        const int RS = (int)blockDim.x / hx;
        const int c = (int)threadIdx.x % hx, r0 = (int)threadIdx.x / hx;
        const int x = x0 + c - 1;
        const bool xin = x >= 0 && x < nx;
        if (r0 < RS)
            for (int dy = 0; dy < 3; ++dy) {
                const int y = iy + dy - 1;
                const bool yin = xin && y >= 0 && y < ny;
                for (int zz0 = r0; zz0 < hz; zz0 += TILE_UNROLL * RS) {
                    float val[TILE_UNROLL];
#pragma unroll
                    for (int u = 0; u < TILE_UNROLL; ++u) {
                        const int z = zz0 + u * RS - 1;
                        val[u] = yin && z >= 0 && z < nz ? a.x[(z * ny + y) * nx + x] : 0.f;
                    }
#pragma unroll
                    for (int u = 0; u < TILE_UNROLL; ++u) {
                        const int zz = zz0 + u * RS;
                        if (zz < hz) halo[(dy * hz + zz) * hx + c] = val[u];
                    }
                }
            }
    }
    // the sheets' cells of the tile: thread t takes axial cell t mod nz of
    // every (blockDim / nz)-th column (z-contiguous reads and writes)
    const int CS = (int)blockDim.x / nz;
    const int zq = (int)threadIdx.x % nz, xq = (int)threadIdx.x / nz;
    const bool col_on = xq < CS;
    const int g1row = (iy * (nx + 2 * PADA) + PADA) * rz + zq + PADZ;  // G1/T1 cell (iy, x0 + xx)
    const int g0col = (iy + PADA) * rz + zq + PADZ;                    // G0/T0 cell (x0 + xx, iy)
    const int g0stride = (ny + 2 * PADA) * rz;
    if (reads_gi<F>() && col_on) {
        // the subset's gradient, then zero cells for the next subset
        for (int xx0 = xq; xx0 < w; xx0 += TILE_UNROLL * CS) {
            float ga[TILE_UNROLL], gb[TILE_UNROLL];
#pragma unroll
            for (int u = 0; u < TILE_UNROLL; ++u) {
                const int xx = xx0 + u * CS, ix = x0 + xx;
                ga[u] = gb[u] = 0.f;
                if (xx < w) {
                    ga[u] = G1[g1row + ix * rz];
                    gb[u] = G0[g0col + ix * g0stride];
                }
            }
#pragma unroll
            for (int u = 0; u < TILE_UNROLL; ++u) {
                const int xx = xx0 + u * CS, ix = x0 + xx;
                if (xx >= w) continue;
                tile[zq * (TT + 1) + xx] = ga[u] + gb[u];
                G1[g1row + ix * rz] = 0.f;
                G0[g0col + ix * g0stride] = 0.f;
            }
        }
    }
    __syncthreads();
    const int nxy = nx * ny;
    for (int e = threadIdx.x; e < nz * TT; e += blockDim.x) {
        const int z = e / TT, xx = e - z * TT;
        if (xx >= w) continue;
        const int ix = x0 + xx;
        const int v = (z * ny + iy) * nx + ix;
        // RDP sums over the 26 neighbours from the halo (rdp_sums with LDS reads)
        const float *hc = halo + (1 * hz + z + 1) * hx + xx + 1;
        const float xi = *hc;
        const float xe = xi + a.eps;
        float g = 0.f, h = 0.f, sv = 0.f;
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
            const bool oz = z + dz - 1 >= 0 && z + dz - 1 < nz;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const bool ozy = oz && iy + dy - 1 >= 0 && iy + dy - 1 < ny;
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    if (dz == 1 && dy == 1 && dx == 1) continue;
                    const bool in = ozy && ix + dx - 1 >= 0 && ix + dx - 1 < nx;
                    const float xj = halo[(dy * hz + z + dz) * hx + xx + dx];
                    const float wk = a.w.w[dz * 9 + dy * 3 + dx];
                    const float d = xi - xj;
                    const float phi = fmaf(a.gamma, fabsf(d), xe + xj);
                    const float r = in ? __builtin_amdgcn_rcpf(phi) : 0.f;
                    const float c = fmaf(2.f, xj, a.eps);
                    const float r2 = r * r;
                    g = fmaf(wk * d * (phi + c), r2, g);
                    if (F & (R_HESS_OUT | R_PRECOND)) h = fmaf(2.f * wk * c * c, r2 * r, h);
                }
            }
        }
        (void)nxy;
        double val = 0.0, pq = 0.0, qdq = 0.0;
        const float gi = reads_gi<F>() ? tile[z * (TT + 1) + xx] : 0.f;
        tile[z * (TT + 1) + xx] = rdp_finish<F>(a, v, xi, g, h, sv, gi, val, pq, qdq);
    }
    __syncthreads();
    if (col_on)
        for (int xx = xq; xx < w; xx += CS) {
            const float val = tile[zq * (TT + 1) + xx];
            const int ix = x0 + xx;
            T0[g0col + ix * g0stride] = val;
            T1[g1row + ix * rz] = val;
        }
}

__global__ void k_precond(const float *__restrict__ x, const float *__restrict__ sens, const float *__restrict__ hess,
                          float alpha, float delta, float *__restrict__ D, int64_t n) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const float xd = x[v] + delta;
        const float den = sens[v] + alpha * hess[v] * xd;
        D[v] = den != 0.f ? xd / den : 0.f;
    }
}

// ghat_i = g (data gradient of subset i at the snapshot); ghat (+)= g in FP64.
// (clear: the gradient sheets' cells read here are set to zero afterwards, so
// that the next subset's line kernels need no separate clearing)
__global__ void __launch_bounds__(256) k_snapshot_accum(float *__restrict__ G0, float *__restrict__ G1,
                                                        float *__restrict__ ghat_i, double *__restrict__ ghat,
                                                        float *__restrict__ gcopy, int nx, int ny, int nz, int rz,
                                                        int first, const float *__restrict__ base, int clear) {
    extern __shared__ float tile[];
    const int x0 = blockIdx.x * TT, iy = blockIdx.y;
    const int w = min(TT, nx - x0);
    sheets_to_tile(G0, G1, tile, x0, w, iy, nx, ny, nz, rz);
    if (clear)
        for (int e = threadIdx.x; e < w * nz; e += blockDim.x) {
            const int xx = e / nz, z = e - xx * nz;
            const int ix = x0 + xx;
            G1[((size_t)iy * (nx + 2 * PADA) + ix + PADA) * rz + z + PADZ] = 0.f;
            G0[((size_t)ix * (ny + 2 * PADA) + iy + PADA) * rz + z + PADZ] = 0.f;
        }
    for (int e = threadIdx.x; e < nz * TT; e += blockDim.x) {
        const int z = e / TT, xx = e - z * TT;
        if (xx >= w) continue;
        const size_t v = ((size_t)z * ny + iy) * nx + x0 + xx;
        const float s = tile[z * (TT + 1) + xx];
        ghat_i[v] = s;
        if (gcopy) gcopy[v] = s;
        ghat[v] = (first ? (base ? (double)base[v] : 0.0) : ghat[v]) + (double)s;
    }
}

// The snapshot table from a one-launch snapshot pass: for each subset q in
// turn, its gradient from the q-th pair of sheets (G0, G1 + q stride) into
// ghat_i[q], those cells zeroed after reading; ghat = base + the n gradients
// in FP64, added in subset order (as one k_snapshot_accum per subset does)
// and held in registers over the subsets.  A thread keeps the same voxels of
// the tile for every subset: at most SNAP_VPT of them (nz TT <= SNAP_VPT 256).
constexpr int SNAP_VPT = 16;

__global__ void __launch_bounds__(256) k_snapshot_accum_slots(float *__restrict__ G0, float *__restrict__ G1,
                                                              int64_t stride, int n_sub, float *__restrict__ ghat_i,
                                                              int64_t nv, double *__restrict__ ghat, int nx, int ny,
                                                              int nz, int rz, const float *__restrict__ base) {
    extern __shared__ float tile[];
    const int x0 = blockIdx.x * TT, iy = blockIdx.y;
    const int w = min(TT, nx - x0);
    double acc[SNAP_VPT];
#pragma unroll
    for (int u = 0; u < SNAP_VPT; ++u) {
        const int e = threadIdx.x + u * blockDim.x;
        const int z = e / TT, xx = e - z * TT;
        acc[u] = base && e < nz * TT && xx < w ? (double)base[((size_t)z * ny + iy) * nx + x0 + xx] : 0.0;
    }
    for (int q = 0; q < n_sub; ++q) {
        float *g0 = G0 + (size_t)q * stride, *g1 = G1 + (size_t)q * stride;
        sheets_to_tile(g0, g1, tile, x0, w, iy, nx, ny, nz, rz);
        for (int e = threadIdx.x; e < w * nz; e += blockDim.x) {
            const int xx = e / nz, z = e - xx * nz;
            const int ix = x0 + xx;
            g1[((size_t)iy * (nx + 2 * PADA) + ix + PADA) * rz + z + PADZ] = 0.f;
            g0[((size_t)ix * (ny + 2 * PADA) + iy + PADA) * rz + z + PADZ] = 0.f;
        }
        float *gq = ghat_i + (size_t)q * nv;
#pragma unroll
        for (int u = 0; u < SNAP_VPT; ++u) {
            const int e = threadIdx.x + u * blockDim.x;
            const int z = e / TT, xx = e - z * TT;
            if (e < nz * TT && xx < w) {
                const float s = tile[z * (TT + 1) + xx];
                gq[((size_t)z * ny + iy) * nx + x0 + xx] = s;
                acc[u] += (double)s;
            }
        }
        __syncthreads();  // (before the next subset's tile)
    }
#pragma unroll
    for (int u = 0; u < SNAP_VPT; ++u) {
        const int e = threadIdx.x + u * blockDim.x;
        const int z = e / TT, xx = e - z * TT;
        if (e < nz * TT && xx < w) ghat[((size_t)z * ny + iy) * nx + x0 + xx] = acc[u];
    }
}

// SAGA table at the first iteration: the data gradients of every subset are
// in table (n x nvox); add each subset's prior share (beta / n) grad S(x) and
// form the table's sum in FP64 from the stored entries.
__global__ void k_saga_table_prior(float *__restrict__ table, double *__restrict__ table_sum,
                                   const float *__restrict__ bgrad, int n_sub, int64_t nv,
                                   const float *__restrict__ base) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const float share = bgrad[v] / (float)n_sub;
        double sum = base ? (double)base[v] : 0.0;
        for (int i = 0; i < n_sub; ++i) {
            const float t = table[(size_t)i * nv + v] + share;
            table[(size_t)i * nv + v] = t;
            sum += (double)t;
        }
        table_sum[v] = sum;
    }
}

// One axis of the resolution model: out (+)= sum_{|d| <= r} w[|d|] in[v + d e_axis]
// with zero outside the grid (Section 3.1: image-space Gaussian).
__global__ void __launch_bounds__(IMG_BLOCK) k_psf_axis(const float *__restrict__ in, float *__restrict__ out, int nx,
                                                       int ny, int nz, PsfAxis k, int accumulate) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t stride = k.axis == 0 ? 1 : (k.axis == 1 ? nx : (int64_t)nx * ny);
    const int len = k.axis == 0 ? nx : (k.axis == 1 ? ny : nz);
    for (int64_t v = blockIdx.x * (int64_t)IMG_BLOCK + threadIdx.x; v < n; v += (int64_t)gridDim.x * IMG_BLOCK) {
        const int c = (int)((v / stride) % len);
        const int lo = -min(c, k.r), hi = min(len - 1 - c, k.r);
        float acc = 0.f;
        for (int d = lo; d <= hi; ++d) acc = fmaf(k.w[d < 0 ? -d : d], in[v + d * stride], acc);
        out[v] = accumulate ? out[v] + acc : acc;
    }
}

// x -> FP64 running sum of subset gradients (snapshot with a resolution model)
__global__ void k_accum_image(const float *__restrict__ img, double *__restrict__ ghat, float *__restrict__ gcopy,
                              int64_t n, int first, const float *__restrict__ base) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const float s = img[v];
        if (gcopy) gcopy[v] = s;
        ghat[v] = (first ? (base ? (double)base[v] : 0.0) : ghat[v]) + (double)s;
    }
}

// Short Barzilai-Borwein step from the block partials of p.q and q.D q:
// bb = {p.q, q.D q, tau_bb, number of updates}; tau_bb is kept when either
// dot is not positive.
__global__ void __launch_bounds__(1024) k_bb_finish(const double *__restrict__ partial, int nb, double *__restrict__ bb) {
    __shared__ double red[2][1024 / 64];
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < nb; i += 1024) {
        s0 += partial[i];
        s1 += partial[nb + i];
    }
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_down(s0, off, 64);
        s1 += __shfl_down(s1, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s0;
        red[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double pq = 0.0, qdq = 0.0;
        for (int w = 0; w < 1024 / 64; ++w) {
            pq += red[0][w];
            qdq += red[1][w];
        }
        bb[0] = pq;
        bb[1] = qdq;
        if (pq > 0.0 && qdq > 0.0) bb[2] = pq / qdq;
        bb[3] += 1.0;
    }
}

__global__ void k_bb_init(double *bb) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        bb[0] = 0.0;
        bb[1] = 0.0;
        bb[2] = __builtin_inf();
        bb[3] = 0.0;
    }
}

// Step along a stored estimator: x_out = max(0, x - min(tau, tau_bb) D est).
__global__ void k_step_stored(const float *__restrict__ x, const float *__restrict__ D, const float *__restrict__ est,
                              float tau, const double *__restrict__ tau_bb, float *__restrict__ x_out, int64_t n) {
    const float t = tau_bb ? fminf(tau, (float)*tau_bb) : tau;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        x_out[v] = fmaxf(0.f, fmaf(-t * D[v], est[v], x[v]));
}

// ||grad J_i(xhat)|| for every subset: the data-only snapshot gradient plus
// the subset's prior share, one workgroup per subset (FP64 sum of squares).
__global__ void __launch_bounds__(1024) k_subset_norms(const float *__restrict__ ghat_i, const float *__restrict__ bgrad,
                                                       int n_sub, int64_t nv, double *__restrict__ out) {
    __shared__ double red[1024 / 64];
    const int i = blockIdx.x;
    double s = 0.0;
    for (int64_t v = threadIdx.x; v < nv; v += 1024) {
        const double t = (double)ghat_i[(size_t)i * nv + v] + (double)bgrad[v] / (double)n_sub;
        s += t * t;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 1024 / 64; ++w) t += red[w];
        out[i] = sqrt(t);
    }
}

// x <- x * (sgn num) / sens where sens > 0 (sgn = -1: num holds the negated
// ratio backprojection of the zero-count-aware kernels)
__global__ void k_osem_update(float *__restrict__ x, const float *__restrict__ num, const float *__restrict__ sens,
                              int64_t n, float sgn) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        float s = sens[v];
        if (s > 0.f) x[v] = x[v] * (sgn * num[v]) / s;
    }
}

// Single-block deterministic reductions.
// Domain checks (debug mode): count the elements of p that violate the
// condition `kind` into *count.  y (nullable, dtype ydt) is the counts array
// that the CHK_ADD / CHK_NO_ADD conditions refer to, element by element.
__device__ __forceinline__ float y_at(const void *y, int dt, int64_t i) {
    if (dt == PET_Y_U8) return (float)((const uint8_t *)y)[i];
    if (dt == PET_Y_U16) return (float)((const uint16_t *)y)[i];
    return ((const float *)y)[i];
}

__global__ void k_domain_count(const float *__restrict__ p, int kind, int64_t n, const void *__restrict__ y, int ydt,
                               unsigned *__restrict__ count) {
    unsigned bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        bool ok = true;
        if (kind == CHK_NONNEG) {
            const float v = p[i];
            ok = v >= 0.f && v <= FLT_MAX;
        } else if (kind == CHK_FINITE) {
            const float v = p[i];
            ok = v >= -FLT_MAX && v <= FLT_MAX;
        } else if (kind == CHK_COUNTS) {
            const float v = y_at(y, ydt, i);
            ok = v >= 0.f && v <= FLT_MAX;
        } else if (kind == CHK_ADD) {
            const float v = p[i];
            ok = v >= 0.f && v <= FLT_MAX && (v > 0.f || !(y_at(y, ydt, i) > 0.f));
        } else if (kind == CHK_NO_ADD) {
            ok = !(y_at(y, ydt, i) > 0.f);
        }
        bad += ok ? 0u : 1u;
    }
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_down(bad, off, 64);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(count, bad);
}

__global__ void k_fill_u32(unsigned *__restrict__ p, int n, unsigned val) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = val;
}

__global__ void k_reduce_sum(const double *__restrict__ p, int n, double *__restrict__ out, int accumulate) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += p[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = accumulate ? *out + red[0] : red[0];
}

__global__ void k_max(const float *__restrict__ x, int64_t n, float *__restrict__ out) {
    __shared__ float red[1024];
    float m = -INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, x[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_copy(float *__restrict__ d, const float *__restrict__ s, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) d[i] = s[i];
}

// transposes through LDS tiles: workgroups (x tile, y), LDS nz x (TT + 1) floats
inline dim3 tile_grid(const pet_geom_s *g) { return dim3((unsigned)((g->d.nx + TT - 1) / TT), (unsigned)g->d.ny); }
inline size_t tile_lds(const pet_geom_s *g) { return sizeof(float) * (size_t)g->d.nz * (TT + 1); }

inline dim3 grid_for(int64_t n) {
    int64_t b = (n + IMG_BLOCK - 1) / IMG_BLOCK;
    return dim3((unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 65536));
}

template <int F>
hipError_t rdp_launch(const RdpArgs &a, int64_t n, hipStream_t s) {
    dim3 grid((unsigned)((n + IMG_BLOCK - 1) / IMG_BLOCK));
    hipLaunchKernelGGL((k_rdp<F>), grid, dim3(IMG_BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace

// G in -> out through the work buffers psf_a / psf_b: pass p reads `in` (p = 0)
// or the previous pass's buffer and writes buffer p % 2, the last pass writes
// `out` (accumulating if asked).  `in` may be psf_b; `out` must not be the
// buffer the last pass reads (psf_b for three passes, psf_a for two).
hipError_t launch_psf_b(const pet_geom_s *g, const SheetBufs &w, const float *in, float *out, int accumulate,
                        hipStream_t s) {
    if (!g->psf_passes) return hipErrorInvalidValue;
    float *buf[2] = {w.psf_a, w.psf_b};
    for (int p = 0; p < g->psf_passes; ++p) {
        const float *src = p == 0 ? in : buf[(p - 1) % 2];
        const bool last = p == g->psf_passes - 1;
        float *dst = last ? out : buf[p % 2];
        hipLaunchKernelGGL(k_psf_axis, grid_for(g->n_vox), dim3(IMG_BLOCK), 0, s, src, dst, g->d.nx, g->d.ny,
                           g->d.nz, g->psf[p], last ? accumulate : 0);
    }
    return hipGetLastError();
}

hipError_t launch_psf(const pet_geom_s *g, const float *in, float *out, int accumulate, hipStream_t s) {
    return launch_psf_b(g, geom_bufs(g), in, out, accumulate, s);
}

SheetBufs geom_bufs(const pet_geom_s *g) { return SheetBufs{g->T0, g->T1, g->G0, g->G1, g->psf_a, g->psf_b}; }

// The line kernels read x (or G x with a resolution model) through the sheets.
hipError_t launch_to_sheets_b(const pet_geom_s *g, const SheetBufs &w, const float *x, hipStream_t s) {
    const float *src = x;
    if (g->psf_passes) {
        float *gx = g->psf_passes == 3 ? w.psf_a : w.psf_b;
        const hipError_t e = launch_psf_b(g, w, x, gx, 0, s);
        if (e != hipSuccess) return e;
        src = gx;
    }
    hipLaunchKernelGGL(k_to_sheets_t, tile_grid(g), dim3(256), tile_lds(g), s, src, w.T0, w.T1, g->d.nx, g->d.ny,
                       g->d.nz, g->d.nz + 2 * PADZ);
    return hipGetLastError();
}

hipError_t launch_to_sheets(const pet_geom_s *g, const float *x, hipStream_t s) {
    return launch_to_sheets_b(g, geom_bufs(g), x, s);
}

// Whole image sheets to zero, padding included (k_to_sheets rewrites only the
// interior; the borders of the handle's own sheets are cleared once at creation).
hipError_t launch_clear_image_sheets(const pet_geom_s *g, const SheetBufs &w, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, grid_for((int64_t)g->t0_elems), dim3(IMG_BLOCK), 0, s, w.T0, (int64_t)g->t0_elems, 0.f);
    hipLaunchKernelGGL(k_fill, grid_for((int64_t)g->t1_elems), dim3(IMG_BLOCK), 0, s, w.T1, (int64_t)g->t1_elems, 0.f);
    return hipGetLastError();
}

hipError_t launch_zero_sheets_b(const pet_geom_s *g, const SheetBufs &w, hipStream_t s) {
    const int64_t n0 = (int64_t)g->t0_elems, n1 = (int64_t)g->t1_elems;
    if ((reinterpret_cast<uintptr_t>(w.G0) | reinterpret_cast<uintptr_t>(w.G1)) % 16 == 0 && n0 % 4 == 0 &&
        n1 % 4 == 0)
        hipLaunchKernelGGL(k_zero2_v4, grid_for((n0 + n1) / 4), dim3(IMG_BLOCK), 0, s,
                           reinterpret_cast<float4 *>(w.G0), n0 / 4, reinterpret_cast<float4 *>(w.G1), n1 / 4);
    else
        hipLaunchKernelGGL(k_zero2, grid_for(n0 + n1), dim3(IMG_BLOCK), 0, s, w.G0, n0, w.G1, n1);
    return hipGetLastError();
}

hipError_t launch_zero_sheets(const pet_geom_s *g, hipStream_t s) { return launch_zero_sheets_b(g, geom_bufs(g), s); }

// Gradient sheets -> image (then G^T = G with a resolution model).
hipError_t launch_from_sheets_b(const pet_geom_s *g, const SheetBufs &w, float *out, int accumulate, hipStream_t s) {
    if (g->psf_passes) {
        hipLaunchKernelGGL(k_from_sheets_t, tile_grid(g), dim3(256), tile_lds(g), s, w.G0, w.G1, w.psf_b, g->d.nx,
                           g->d.ny, g->d.nz, g->d.nz + 2 * PADZ, 0);
        const hipError_t e = hipGetLastError();
        return e != hipSuccess ? e : launch_psf_b(g, w, w.psf_b, out, accumulate, s);
    }
    hipLaunchKernelGGL(k_from_sheets_t, tile_grid(g), dim3(256), tile_lds(g), s, w.G0, w.G1, out, g->d.nx, g->d.ny,
                       g->d.nz, g->d.nz + 2 * PADZ, accumulate);
    return hipGetLastError();
}

hipError_t launch_from_sheets(const pet_geom_s *g, float *out, int accumulate, hipStream_t s) {
    return launch_from_sheets_b(g, geom_bufs(g), out, accumulate, s);
}

hipError_t launch_rdp(const pet_geom_s *g, const float *x, const float *kappa, const float *w27, float beta,
                      float gamma, float eps, float *grad, float *hess, double *partial, hipStream_t s) {
    RdpArgs a{};
    a.x = x;
    a.kappa = kappa;
    for (int i = 0; i < 27; ++i) a.w.w[i] = w27[i];
    a.beta = beta;
    a.gamma = gamma;
    a.eps = eps;
    a.nx = g->d.nx;
    a.ny = g->d.ny;
    a.nz = g->d.nz;
    a.grad = grad;
    a.hess = hess;
    a.partial = partial;
    int f = (grad ? 1 : 0) | (hess ? 2 : 0) | (partial ? 4 : 0);
    switch (f) {
        case 1: return rdp_launch<R_GRAD_OUT>(a, g->n_vox, s);
        case 2: return rdp_launch<R_HESS_OUT>(a, g->n_vox, s);
        case 3: return rdp_launch<R_GRAD_OUT | R_HESS_OUT>(a, g->n_vox, s);
        case 4: return rdp_launch<R_VALUE>(a, g->n_vox, s);
        case 5: return rdp_launch<R_GRAD_OUT | R_VALUE>(a, g->n_vox, s);
        case 6: return rdp_launch<R_HESS_OUT | R_VALUE>(a, g->n_vox, s);
        case 7: return rdp_launch<R_GRAD_OUT | R_HESS_OUT | R_VALUE>(a, g->n_vox, s);
        default: return hipSuccess;
    }
}

int rdp_blocks(const pet_geom_s *g) { return (int)((g->n_vox + IMG_BLOCK - 1) / IMG_BLOCK); }

hipError_t launch_precond(const pet_geom_s *g, const float *x, const float *sens, const float *hess, float alpha,
                          float delta, float *D, hipStream_t s) {
    hipLaunchKernelGGL(k_precond, grid_for(g->n_vox), dim3(IMG_BLOCK), 0, s, x, sens, hess, alpha, delta, D, g->n_vox);
    return hipGetLastError();
}

hipError_t launch_svrg_step(const pet_geom_s *g, const float *x, const float *kappa, const float *w27, float beta,
                            float gamma, float eps, int update_pc, const float *sens, float alpha, float delta,
                            float *D, int snapshot, const float *gi, const float *ghat_i, const double *ghat,
                            float n_sub, float tau, float *x_out, float *est_out, hipStream_t s) {
    RdpArgs a{};
    a.x = x;
    a.kappa = kappa;
    for (int i = 0; i < 27; ++i) a.w.w[i] = w27[i];
    a.beta = beta;
    a.gamma = gamma;
    a.eps = eps;
    a.nx = g->d.nx;
    a.ny = g->d.ny;
    a.nz = g->d.nz;
    a.sens = sens;
    a.alpha = alpha;
    a.delta = delta;
    a.D = D;
    a.gi = gi;
    a.ghat_i = ghat_i;
    a.ghat = ghat;
    a.n_sub = n_sub;
    a.tau = tau;
    a.x_out = x_out;
    a.est_out = est_out;
    const int f = (update_pc ? 4 : 0) | (snapshot ? 2 : 0) | (est_out ? 1 : 0);
    switch (f) {
        case 0: return rdp_launch<R_UPDATE>(a, g->n_vox, s);
        case 1: return rdp_launch<R_UPDATE | R_EST_OUT>(a, g->n_vox, s);
        case 2: return rdp_launch<R_UPDATE | R_SNAPSHOT>(a, g->n_vox, s);
        case 3: return rdp_launch<R_UPDATE | R_SNAPSHOT | R_EST_OUT>(a, g->n_vox, s);
        case 4: return rdp_launch<R_PRECOND | R_UPDATE>(a, g->n_vox, s);
        case 5: return rdp_launch<R_PRECOND | R_UPDATE | R_EST_OUT>(a, g->n_vox, s);
        case 6: return rdp_launch<R_PRECOND | R_UPDATE | R_SNAPSHOT>(a, g->n_vox, s);
        default: return rdp_launch<R_PRECOND | R_UPDATE | R_SNAPSHOT | R_EST_OUT>(a, g->n_vox, s);
    }
}

template <int F>
hipError_t step_tile_launch(const pet_geom_s *g, const RdpArgs &a, hipStream_t s) {
    const int nz = g->d.nz;
    const size_t lds = sizeof(float) * ((size_t)halo_elems(nz) + (size_t)nz * (TT + 1));
    hipLaunchKernelGGL((k_step_tile<F>), tile_grid(g), dim3(STEP_BLOCK), lds, s, a, g->G0, g->G1, g->T0, g->T1,
                       nz + 2 * PADZ);
    return hipGetLastError();
}

// Whether the fused step (k_step_tile) serves a handle: no resolution model
// (the sheets then hold G x) and a tile that fits the default LDS.
bool step_tile_ok(const pet_geom_s *g) {
    const size_t lds = sizeof(float) * ((size_t)halo_elems(g->d.nz) + (size_t)g->d.nz * (TT + 1));
    return g->psf_passes == 0 && lds <= 64 * 1024;
}

// SVRG step of one iteration fused with the sheet conversions (k_step_tile):
// regular iterations read the sampled subset's data gradient from the
// handle's gradient sheets and clear them; every iteration writes x_out and
// the handle's image sheets of x_out.  bb_store: keep the snapshot's full
// gradient in g_prev.  No kappa image; the caller checks step_tile_ok.
hipError_t launch_svrg_step_tile(const pet_geom_s *g, const float *x, const float *w27, float beta, float gamma,
                                 float eps, int update_pc, const float *sens, float alpha, float delta, float *D,
                                 int snapshot, const float *ghat_i, const double *ghat, float w, float tau,
                                 const double *tau_bb, int bb_store, float *g_prev, float *x_out, hipStream_t s) {
    RdpArgs a{};
    a.x = x;
    for (int i = 0; i < 27; ++i) a.w.w[i] = w27[i];
    a.beta = beta;
    a.gamma = gamma;
    a.eps = eps;
    a.nx = g->d.nx;
    a.ny = g->d.ny;
    a.nz = g->d.nz;
    a.sens = sens;
    a.alpha = alpha;
    a.delta = delta;
    a.D = D;
    a.ghat_i = ghat_i;
    a.ghat = ghat;
    a.n_sub = w;
    a.tau = tau;
    a.tau_bb = tau_bb;
    a.x_out = x_out;
    a.g_prev = g_prev;
    const int code = (update_pc ? 1 : 0) | (snapshot ? 2 : 0) | (snapshot && bb_store ? 4 : 0);
    switch (code) {
        case 0: return step_tile_launch<R_UPDATE>(g, a, s);
        case 1: return step_tile_launch<R_UPDATE | R_PRECOND>(g, a, s);
        case 2: return step_tile_launch<R_UPDATE | R_SNAPSHOT>(g, a, s);
        case 3: return step_tile_launch<R_UPDATE | R_SNAPSHOT | R_PRECOND>(g, a, s);
        case 6: return step_tile_launch<R_UPDATE | R_SNAPSHOT | R_BB_STORE>(g, a, s);
        default: return step_tile_launch<R_UPDATE | R_SNAPSHOT | R_PRECOND | R_BB_STORE>(g, a, s);
    }
}

// SVRG iteration with the ALG2/ALG3 extensions: estimator weight `w` of the
// sampled subset (n for uniform sampling), the step bound tau_bb (device,
// nullable) and, at a snapshot, the BB bookkeeping (bb_mode 1: keep the full
// gradient in g_prev; 2: also the dots into g->partial, no step) and the
// prior gradient into grad_out (nullable; for the subset-gradient norms).
hipError_t launch_svrg_step_ex(const pet_geom_s *g, const float *x, const float *kappa, const float *w27, float beta,
                               float gamma, float eps, int update_pc, const float *sens, float alpha, float delta,
                               float *D, int snapshot, const float *gi, const float *ghat_i, const double *ghat,
                               float w, float tau, const double *tau_bb, int bb_mode, const float *x_snap,
                               float *g_prev, float *grad_out, float *x_out, hipStream_t s) {
    RdpArgs a{};
    a.x = x;
    a.kappa = kappa;
    for (int i = 0; i < 27; ++i) a.w.w[i] = w27[i];
    a.beta = beta;
    a.gamma = gamma;
    a.eps = eps;
    a.nx = g->d.nx;
    a.ny = g->d.ny;
    a.nz = g->d.nz;
    a.sens = sens;
    a.alpha = alpha;
    a.delta = delta;
    a.D = D;
    a.gi = gi;
    a.ghat_i = ghat_i;
    a.ghat = ghat;
    a.n_sub = w;
    a.tau = tau;
    a.tau_bb = tau_bb;
    a.x_out = x_out;
    a.x_snap = x_snap;
    a.g_prev = g_prev;
    a.grad = grad_out;
    a.partial = g->partial;
    const int64_t n = g->n_vox;
    if (!snapshot) {
        return update_pc ? rdp_launch<R_PRECOND | R_UPDATE>(a, n, s) : rdp_launch<R_UPDATE>(a, n, s);
    }
    constexpr int B = R_UPDATE | R_SNAPSHOT;
    const int code = (update_pc ? 1 : 0) | (grad_out ? 2 : 0) | (bb_mode << 2);
    switch (code) {
        case 0: return rdp_launch<B>(a, n, s);
        case 1: return rdp_launch<B | R_PRECOND>(a, n, s);
        case 2: return rdp_launch<B | R_GRAD_OUT>(a, n, s);
        case 3: return rdp_launch<B | R_PRECOND | R_GRAD_OUT>(a, n, s);
        case 4: return rdp_launch<B | R_BB_STORE>(a, n, s);
        case 5: return rdp_launch<B | R_BB_STORE | R_PRECOND>(a, n, s);
        case 6: return rdp_launch<B | R_BB_STORE | R_GRAD_OUT>(a, n, s);
        case 7: return rdp_launch<B | R_BB_STORE | R_PRECOND | R_GRAD_OUT>(a, n, s);
        case 8: return rdp_launch<B | R_BB_DOT>(a, n, s);
        case 9: return rdp_launch<B | R_BB_DOT | R_PRECOND>(a, n, s);
        case 10: return rdp_launch<B | R_BB_DOT | R_GRAD_OUT>(a, n, s);
        case 11: return rdp_launch<B | R_BB_DOT | R_PRECOND | R_GRAD_OUT>(a, n, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bb_finish(const pet_geom_s *g, double *bb, hipStream_t s) {
    hipLaunchKernelGGL(k_bb_finish, dim3(1), dim3(1024), 0, s, g->partial, rdp_blocks(g), bb);
    return hipGetLastError();
}

hipError_t launch_bb_init(double *bb, hipStream_t s) {
    hipLaunchKernelGGL(k_bb_init, dim3(1), dim3(64), 0, s, bb);
    return hipGetLastError();
}

hipError_t launch_step_stored(const pet_geom_s *g, const float *x, const float *D, const float *est, float tau,
                              const double *tau_bb, float *x_out, hipStream_t s) {
    hipLaunchKernelGGL(k_step_stored, grid_for(g->n_vox), dim3(IMG_BLOCK), 0, s, x, D, est, tau, tau_bb, x_out,
                       g->n_vox);
    return hipGetLastError();
}

hipError_t launch_subset_norms(const pet_geom_s *g, const float *ghat_i, const float *bgrad, double *out,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_subset_norms, dim3(g->d.n_subsets), dim3(1024), 0, s, ghat_i, bgrad, g->d.n_subsets,
                       g->n_vox, out);
    return hipGetLastError();
}

hipError_t launch_saga_table_prior(const pet_geom_s *g, float *table, double *table_sum, const float *bgrad,
                                  hipStream_t s, const float *base) {
    hipLaunchKernelGGL(k_saga_table_prior, grid_for(g->n_vox), dim3(IMG_BLOCK), 0, s, table, table_sum, bgrad,
                       g->d.n_subsets, g->n_vox, base);
    return hipGetLastError();
}

hipError_t launch_sgm_step(const pet_geom_s *g, int estimator, const float *x, const float *kappa, const float *w27,
                           float beta, float gamma, float eps, int update_pc, const float *sens, float alpha,
                           float delta, float *D, int first, const float *gi, float *table_i, double *table_sum,
                           float n_sub, float tau, float *x_out, hipStream_t s) {
    RdpArgs a{};
    a.x = x;
    a.kappa = kappa;
    for (int i = 0; i < 27; ++i) a.w.w[i] = w27[i];
    a.beta = beta;
    a.gamma = gamma;
    a.eps = eps;
    a.nx = g->d.nx;
    a.ny = g->d.ny;
    a.nz = g->d.nz;
    a.sens = sens;
    a.alpha = alpha;
    a.delta = delta;
    a.D = D;
    a.gi = gi;
    a.table_i = table_i;
    a.table_sum = table_sum;
    a.n_sub = n_sub;
    a.tau = tau;
    a.x_out = x_out;
    if (estimator == SGM_SGD)
        return update_pc ? rdp_launch<R_PRECOND | R_UPDATE | R_SGD>(a, g->n_vox, s)
                         : rdp_launch<R_UPDATE | R_SGD>(a, g->n_vox, s);
    switch ((update_pc ? 2 : 0) | (first ? 1 : 0)) {
        case 0: return rdp_launch<R_UPDATE | R_SAGA>(a, g->n_vox, s);
        case 1: return rdp_launch<R_UPDATE | R_SAGA | R_SNAPSHOT>(a, g->n_vox, s);
        case 2: return rdp_launch<R_PRECOND | R_UPDATE | R_SAGA>(a, g->n_vox, s);
        default: return rdp_launch<R_PRECOND | R_UPDATE | R_SAGA | R_SNAPSHOT>(a, g->n_vox, s);
    }
}

hipError_t launch_snapshot_accum(const pet_geom_s *g, float *ghat_i, double *ghat, float *gcopy, int first,
                                 hipStream_t s, const float *base, int clear, float *G0, float *G1) {
    if (G0 && g->psf_passes) return hipErrorInvalidValue;  // (the resolution model reads the handle's sheets)
    if (g->psf_passes) {
        hipError_t e = launch_from_sheets(g, ghat_i, 0, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_accum_image, grid_for(g->n_vox), dim3(IMG_BLOCK), 0, s, ghat_i, ghat, gcopy, g->n_vox,
                           first, base);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_snapshot_accum, tile_grid(g), dim3(256), tile_lds(g), s, G0 ? G0 : g->G0, G1 ? G1 : g->G1,
                       ghat_i, ghat, gcopy, g->d.nx, g->d.ny, g->d.nz, g->d.nz + 2 * PADZ, first, base, clear);
    return hipGetLastError();
}

hipError_t launch_snapshot_accum_slots(const pet_geom_s *g, float *G0, float *G1, int64_t stride, int n_sub,
                                       float *ghat_i, double *ghat, const float *base, hipStream_t s) {
    if (g->psf_passes) return hipErrorInvalidValue;  // (the resolution model reads the handle's sheets)
    if ((int64_t)g->d.nz * TT > (int64_t)SNAP_VPT * 256) {
        // taller tiles than a thread's registers hold: one launch per subset
        hipError_t e = hipSuccess;
        for (int q = 0; q < n_sub && e == hipSuccess; ++q)
            e = launch_snapshot_accum(g, ghat_i + (size_t)q * g->n_vox, ghat, nullptr, q == 0, s, base, 1,
                                      G0 + (size_t)q * stride, G1 + (size_t)q * stride);
        return e;
    }
    hipLaunchKernelGGL(k_snapshot_accum_slots, tile_grid(g), dim3(256), tile_lds(g), s, G0, G1, stride, n_sub, ghat_i,
                       g->n_vox, ghat, g->d.nx, g->d.ny, g->d.nz, g->d.nz + 2 * PADZ, base);
    return hipGetLastError();
}

hipError_t launch_reduce_sum(const double *partial, int n, double *out, int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(1024), 0, s, partial, n, out, accumulate);
    return hipGetLastError();
}

hipError_t launch_osem_update(const pet_geom_s *g, float *x, const float *num, const float *sens, hipStream_t s,
                              float sgn) {
    hipLaunchKernelGGL(k_osem_update, grid_for(g->n_vox), dim3(IMG_BLOCK), 0, s, x, num, sens, g->n_vox, sgn);
    return hipGetLastError();
}

// FP64 block partials of sum a[v] b[v] (IMG_BLOCK threads per block).
__global__ void k_dot_partial(const float *__restrict__ a, const float *__restrict__ b, int64_t n,
                              double *__restrict__ partial) {
    __shared__ double red[IMG_BLOCK / 64];
    double acc = 0.0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        acc += (double)a[v] * (double)b[v];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < IMG_BLOCK / 64; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

__global__ void k_add_scalar(double *__restrict__ out, double val) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out += val;
}

// *out (+)= sum a[v] b[v] in FP64 (block partials in `partial`, at least
// dot_blocks(n) doubles, then one reduction).
int dot_blocks(int64_t n) { return (int)grid_for(n).x; }

hipError_t launch_dot(const float *a, const float *b, int64_t n, double *partial, double *out, int accumulate,
                      hipStream_t s) {
    const dim3 grid = grid_for(n);
    hipLaunchKernelGGL(k_dot_partial, grid, dim3(IMG_BLOCK), 0, s, a, b, n, partial);
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_reduce_sum(partial, (int)grid.x, out, accumulate, s);
}

hipError_t launch_add_scalar(double *out, double val, hipStream_t s) {
    hipLaunchKernelGGL(k_add_scalar, dim3(1), dim3(64), 0, s, out, val);
    return hipGetLastError();
}

hipError_t launch_domain_count(const float *p, int kind, int64_t n, const void *y, int ydt, unsigned *count,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_domain_count, grid_for(n), dim3(IMG_BLOCK), 0, s, p, kind, n, y, ydt, count);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, int n, unsigned val, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, val);
    return hipGetLastError();
}

hipError_t launch_max(const pet_geom_s *g, const float *x, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_max, dim3(1), dim3(1024), 0, s, x, g->n_vox, out);
    return hipGetLastError();
}

hipError_t launch_fill(float *dst, int64_t n, float val, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, grid_for(n), dim3(IMG_BLOCK), 0, s, dst, n, val);
    return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, grid_for(n), dim3(IMG_BLOCK), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace pet
