// Device helpers shared by the line kernels (proj.hip, counts.hip): the
// z range of a LOR's samples, the per-line LDS sheets (transaxial
// interpolation of the image in, gradient sheet out) and block sums.
#pragma once

#include "pet_internal.h"

namespace pet {
namespace {

// Sample range [is, ie] of a LOR restricted to samples whose z coordinate can
// touch the grid (xi_z in [-1.5, nz + 0.5]).
template <bool FAST = false>
__device__ __forceinline__ void z_clip(const LineP &L, const PlaneP &P, int nz, int &is, int &ie) {
    is = L.i_lo;
    ie = L.i_hi;
    if (P.zs != 0.f) {
        // FAST: reciprocals instead of divisions, for callers that clamp the
        // axial position themselves (the range is then only a work bound)
        const float rzs = FAST ? __builtin_amdgcn_rcpf(P.zs) : 0.f, rdl = FAST ? __builtin_amdgcn_rcpf(L.dlam) : 0.f;
        float la = FAST ? (-1.5f - P.zb) * rzs : (-1.5f - P.zb) / P.zs;
        float lb = FAST ? ((float)nz + 0.5f - P.zb) * rzs : ((float)nz + 0.5f - P.zb) / P.zs;
        float ia = FAST ? (fminf(la, lb) - L.lam0) * rdl : (fminf(la, lb) - L.lam0) / L.dlam;
        float ib = FAST ? (fmaxf(la, lb) - L.lam0) * rdl : (fmaxf(la, lb) - L.lam0) / L.dlam;
        float lo = ceilf(fminf(ia, ib)), hi = floorf(fmaxf(ia, ib));
        if (lo > (float)is) is = lo > (float)ie ? ie + 1 : (int)lo;
        if (hi < (float)ie) ie = hi < (float)is ? is - 1 : (int)hi;
    } else if (P.zb < -1.5f || P.zb > (float)nz + 0.5f) {
        ie = is - 1;
    }
}

// Block prologue: image sheet X (transaxial interpolation of the transposed
// image) and / or zeroed gradient sheet Z.  Z accumulates in FP64: LDS FP64
// atomic adds run at full rate on gfx950, FP32 ones do not.
// The loads of SHEET_UNROLL elements per thread are issued before any of them
// is used, so that a workgroup waits for memory a few times per line rather
// than once per element it builds.
constexpr int SHEET_UNROLL = 4;

template <bool NEED_X, bool NEED_Z>
__device__ __forceinline__ void build_sheets(const ProjArgs &a, const LineP &L, int nrow, float *X, double *Z) {
    const int rz = a.rz;
    const int n = nrow * rz;
    if (NEED_X) {
        const float *T = L.axis ? a.T1 : a.T0;
        const size_t other_stride = (size_t)((L.axis ? a.nx : a.ny) + 2 * PADA) * rz;
        const int step = (int)blockDim.x;
        for (int e0 = threadIdx.x; e0 < n; e0 += SHEET_UNROLL * step) {
            float t0[SHEET_UNROLL], t1[SHEET_UNROLL], f[SHEET_UNROLL];
#pragma unroll
            for (int u = 0; u < SHEET_UNROLL; ++u) {
                const int e = e0 + u * step;
                t0[u] = t1[u] = f[u] = 0.f;
                if (e < n) {
                    const int r = e / rz;
                    const int zp = e - r * rz;
                    const int i = L.i_lo + r;
                    const float xa = fmaf((float)i, L.dxa, L.xa0);
                    const float jf = floorf(xa);
                    f[u] = xa - jf;
                    const size_t base = (size_t)i * other_stride + (size_t)((int)jf + PADA) * rz + zp;
                    t0[u] = T[base];
                    t1[u] = T[base + rz];
                }
            }
#pragma unroll
            for (int u = 0; u < SHEET_UNROLL; ++u) {
                const int e = e0 + u * step;
                if (e < n) X[e] = fmaf(f[u], t1[u] - t0[u], t0[u]);
            }
        }
    }
    if (NEED_Z)
        for (int e = threadIdx.x; e < n; e += blockDim.x) Z[e] = 0.0;
}

// Block epilogue: spread the gradient sheet over the two transaxial neighbours.
__device__ __forceinline__ void scatter_sheet(const ProjArgs &a, const LineP &L, int nrow, const double *Z,
                                              int64_t g_off = 0) {
    const int rz = a.rz;
    float *Gout = (L.axis ? a.G1 : a.G0) + g_off;
    const size_t other_stride = (size_t)((L.axis ? a.nx : a.ny) + 2 * PADA) * rz;
    for (int e = threadIdx.x; e < nrow * rz; e += blockDim.x) {
        float val = (float)Z[e];
        if (val == 0.f) continue;
        int r = e / rz;
        int zp = e - r * rz;
        int i = L.i_lo + r;
        float xa = fmaf((float)i, L.dxa, L.xa0);
        float jf = floorf(xa);
        float f = xa - jf;
        size_t base = (size_t)i * other_stride + (size_t)((int)jf + PADA) * rz + zp;
        float a1 = val * f;
        atomicAdd(&Gout[base], val - a1);
        atomicAdd(&Gout[base + rz], a1);
    }
}

// Block sums of two doubles into partial[blockIdx.x] (and, for the work counts,
// partial[gridDim.x + blockIdx.x]).
__device__ __forceinline__ void block_sums(double v0, double v1, double *partial, bool two) {
    __shared__ double red[2][TOF_MAX_WAVES];
    for (int off = 32; off > 0; off >>= 1) {
        v0 += __shfl_down(v0, off, 64);
        v1 += __shfl_down(v1, off, 64);
    }
    const int nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = v0;
        red[1][threadIdx.x >> 6] = v1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int w = 0; w < nw; ++w) {
            s0 += red[0][w];
            s1 += red[1][w];
        }
        partial[blockIdx.x] = s0;
        if (two) partial[gridDim.x + blockIdx.x] = s1;
    }
}

}  // namespace
}  // namespace pet
