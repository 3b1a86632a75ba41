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

// Sheet cells (row r, padded axial position zp) are dealt to the threads of
// a workgroup by column: thread t keeps zp = t mod rz and takes rows
// t / rz, t / rz + R, ... with R = blockDim / rz (the threads past R rz idle).
// No division per cell; needs rz <= blockDim (else one cell per thread and
// pass, with a division each).
struct SheetWalk {
    int r0, zp, R;
    bool on;
};

__device__ __forceinline__ SheetWalk sheet_walk(int rz) {
    SheetWalk w;
    w.R = (int)blockDim.x / rz;
    w.r0 = (int)threadIdx.x / rz;
    w.zp = (int)threadIdx.x - w.r0 * rz;
    w.on = w.r0 < w.R;
    return w;
}

// Row i of a line: the transposed image row it interpolates, at the
// transaxial position xa = i dxa + xa0 (cell jf, fraction f).  Offsets are
// 32-bit: a transposed image holds fewer than 2^31 floats (pet_geom_create).
struct SheetRow {
    int base;  // offset of (i, jf + PADA, 0) in the transposed image
    float f;
};

__device__ __forceinline__ SheetRow sheet_row(const LineP &L, int i, int other_stride, int rz) {
    SheetRow s;
    const float xa = fmaf((float)i, L.dxa, L.xa0);
    const float jf = floorf(xa);
    s.f = xa - jf;
    s.base = i * other_stride + ((int)jf + PADA) * rz;
    return s;
}

// Block prologue: image sheet X (transaxial interpolation of the transposed
// image) and / or zeroed gradient sheet Z.  Z accumulates in FP64: LDS FP64
// atomic adds run at full rate on gfx950, FP32 ones do not.
// The loads of SHEET_UNROLL rows per thread are issued before any of them is
// used, so that a workgroup waits for memory a few times per line rather than
// once per element it builds.
constexpr int SHEET_UNROLL = 8;

template <bool NEED_X, bool NEED_Z>
__device__ __forceinline__ void build_sheets(const ProjArgs &a, const LineP &L, int nrow, float *X, double *Z) {
    const int rz = a.rz;
    const int n = nrow * rz;
    if (NEED_X) {
        const float *T = L.axis ? a.T1 : a.T0;
        const int other_stride = ((L.axis ? a.nx : a.ny) + 2 * PADA) * rz;
        if (rz <= (int)blockDim.x) {
            const SheetWalk w = sheet_walk(rz);
            if (w.on) {
                for (int rb = w.r0; rb < nrow; rb += SHEET_UNROLL * w.R) {
                    float t0[SHEET_UNROLL], t1[SHEET_UNROLL], f[SHEET_UNROLL];
#pragma unroll
                    for (int u = 0; u < SHEET_UNROLL; ++u) {
                        const int r = rb + u * w.R;
                        t0[u] = t1[u] = f[u] = 0.f;
                        if (r < nrow) {
                            const SheetRow sr = sheet_row(L, L.i_lo + r, other_stride, rz);
                            f[u] = sr.f;
                            const float *src = T + sr.base + w.zp;
                            t0[u] = src[0];
                            t1[u] = src[rz];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < SHEET_UNROLL; ++u) {
                        const int r = rb + u * w.R;
                        if (r < nrow) X[r * rz + w.zp] = fmaf(f[u], t1[u] - t0[u], t0[u]);
                    }
                }
            }
        } else {
            for (int e = threadIdx.x; e < n; e += blockDim.x) {
                const int r = e / rz;
                const int zp = e - r * rz;
                const SheetRow sr = sheet_row(L, L.i_lo + r, other_stride, rz);
                const float *src = T + sr.base + zp;
                X[e] = fmaf(sr.f, src[rz] - src[0], src[0]);
            }
        }
    }
    if (NEED_Z)
        for (int e = threadIdx.x; e < n; e += blockDim.x) Z[e] = 0.0;
}

// One sheet cell's value spread over the two transaxial neighbours.
__device__ __forceinline__ void spread_cell(float *Gout, const SheetRow &sr, int zp, int rz, float val) {
    const float a1 = val * sr.f;
    atomicAdd(&Gout[sr.base + zp], val - a1);
    atomicAdd(&Gout[sr.base + zp + rz], a1);
}

// Block epilogue: spread the gradient sheet over the two transaxial neighbours.
__device__ __forceinline__ void scatter_sheet(const ProjArgs &a, const LineP &L, int nrow, const double *Z,
                                              int64_t g_off = 0) {
    const int rz = a.rz;
    float *Gout = (L.axis ? a.G1 : a.G0) + g_off;
    const int other_stride = ((L.axis ? a.nx : a.ny) + 2 * PADA) * rz;
    if (rz <= (int)blockDim.x) {
        const SheetWalk w = sheet_walk(rz);
        if (!w.on) return;
        for (int r = w.r0; r < nrow; r += w.R) {
            const float val = (float)Z[r * rz + w.zp];
            if (val == 0.f) continue;
            spread_cell(Gout, sheet_row(L, L.i_lo + r, other_stride, rz), w.zp, rz, val);
        }
    } else {
        for (int e = threadIdx.x; e < nrow * rz; e += blockDim.x) {
            const float val = (float)Z[e];
            if (val == 0.f) continue;
            const int r = e / rz;
            spread_cell(Gout, sheet_row(L, L.i_lo + r, other_stride, rz), e - r * rz, rz, val);
        }
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
