// Joseph projector kernels for gfx950 (forward, adjoint, fused subset gradient,
// EM ratio, KL objective, work counts), line-driven with LDS sheets.
//
// Separability used here: every LOR of a transaxial line (view, radial) has the
// same principal axis m, the same sample positions lambda(i) along m and the
// same transaxial interpolation coordinate; only z (and the step length via
// |u|) depends on the ring pair.  A workgroup therefore owns one line:
//   1. it interpolates the image once along the transaxial axis into an LDS
//      "sheet" X[i][z] (rows i along m, z padded), reading a z-contiguous
//      transposed copy of the image so the loads are coalesced;
//   2. threads take the planes (ring pairs) of the line and walk the samples
//      with one linear interpolation in z from LDS per sample;
//   3. the adjoint accumulates Z[i][z] in LDS with LDS atomics and finally
//      spreads the sheet back over the two transaxial neighbours with global
//      atomics into a z-contiguous transposed gradient image.
// TOF: all planes of one ring-difference segment share |u|, hence the signed
// distance t(i) of every sample and its TOF weights.  One wave takes one
// segment (one plane per lane), fills a table with the weights of the line's
// samples (increasing-t order) once, and the lanes read it by broadcast.
// The arithmetic is Joseph's: sample value = bilinear interpolation of the
// image in the two non-principal axes, line integral = step length * sum.
#include "line_sheets.h"

#include <climits>

namespace pet {
namespace {

__device__ __forceinline__ float load_y(const void *y, int dt, int64_t idx) {
    if (dt == PET_Y_U8) return (float)((const uint8_t *)y)[idx];
    if (dt == PET_Y_U16) return (float)((const uint16_t *)y)[idx];
    return ((const float *)y)[idx];
}

// The nt values src[base .. base + nt) of one LOR (one block of at most
// NT_BLK TOF bins), all loads issued before the first use (zero above nt).
template <typename T>
__device__ __forceinline__ void load_row(const T *src, int64_t base, int nt, float (&v)[NT_BLK]) {
#pragma unroll
    for (int b = 0; b < NT_BLK; ++b) v[b] = b < nt ? (float)src[base + b] : 0.f;
}
__device__ __forceinline__ void load_y_row(const void *y, int dt, int64_t base, int nt, float (&v)[NT_BLK]) {
    if (dt == PET_Y_U8)
        load_row((const uint8_t *)y, base, nt, v);
    else if (dt == PET_Y_U16)
        load_row((const uint16_t *)y, base, nt, v);
    else
        load_row((const float *)y, base, nt, v);
}

// Poisson deviance term d(ybar, y) of the KL data fidelity, FP64.
__device__ __forceinline__ double kl_term(float ybar, float yv) {
    double s = ybar, t = yv;
    if (t > 0.0) return s - t + t * log(t / s);
    return s;
}

// Number of samples of [is, ie] (in increasing-t order) with t < e.
__device__ __forceinline__ int cut_count(float e, float len, float lam0, float dlam, int is, int ie) {
    float lam_e = e / len + 0.5f;
    float r = (lam_e - lam0) / dlam;
    int nq = ie - is + 1;
    int c;
    if (dlam > 0.f) {
        float cr = ceilf(r);
        c = cr < (float)is ? 0 : (cr > (float)(ie + 1) ? nq : (int)cr - is);
    } else {
        float fr = floorf(r);
        c = fr >= (float)ie ? 0 : (fr < (float)(is - 1) ? nq : ie - (int)fr);
    }
    return c;
}

// ---------------------------------------------------------------------------
// Non-TOF: threads over planes (dense), one line per workgroup.
// One transaxial line (all its planes) of a non-TOF geometry, by the whole
// workgroup; returns this thread's FP64 partial (KL or sample count).
__device__ __forceinline__ float clamped_erf(float u, float inv_s, float c) {
    return erff(fminf(fmaxf(u * inv_s, -c), c));
}

// Sum over all TOF bins of the weights of a sample at signed distance t from
// the LOR centre.  The bins [t_b - w/2, t_b + w/2] tile [lo, hi] = [t_first -
// w/2, t_last + w/2] without gaps, so the sum of 1/2 [E(t_b + w/2 - t) -
// E(t_b - w/2 - t)] telescopes to 1/2 [E(hi - t) - E(lo - t)]; where both
// ends are clamped (t at least nsig sigma inside [lo, hi]) it is erf(c).
struct TofFold {
    float lo, hi, inv_s, c, inside;
};

__device__ __forceinline__ TofFold tof_fold_of(const TofTable &T) {
    const float h = T.half_bin;
    return {T.tb[0] - h, T.tb[T.n_tof - 1] + h, T.inv_sqrt2_sigma, T.erf_clamp, erff(T.erf_clamp)};
}

__device__ __forceinline__ float tof_fold_weight(const TofFold &f, float t) {
    const float e1 = (f.hi - t) * f.inv_s, e0 = (f.lo - t) * f.inv_s;
    if (e1 >= f.c && e0 <= -f.c) return f.inside;
    return 0.5f * (erff(fminf(fmaxf(e1, -f.c), f.c)) - erff(fminf(fmaxf(e0, -f.c), f.c)));
}

template <int MODE>
__device__ __forceinline__ double line_nt_body(const ProjArgs &a, int line, float *smem, int64_t g_off = 0) {
    constexpr bool NEED_X = MODE != M_BACK && MODE != M_COUNT;
    constexpr bool NEED_Z = MODE == M_BACK || MODE == M_GRAD || MODE == M_EM || MODE == M_HVP;
    const LineP L = a.lines[line];
    const int nrow = L.i_hi - L.i_lo + 1;
    const int rz = a.rz;
    const int sheet = (a.rows_max * rz + 3) & ~3;
    float *X = smem;
    double *Z = reinterpret_cast<double *>(smem + (NEED_X ? sheet : 0));
    if (nrow > 0 && MODE != M_COUNT) build_sheets<NEED_X, NEED_Z>(a, L, nrow, X, Z);
    __syncthreads();

    // planes in rounds of blockDim threads; the planes of a last, partial round
    // take c threads each (c a power of two: the threads of a plane are lanes of
    // one wave), which split its rows and add their forward sums by shuffles
    const int nb = blockDim.x;
    const int full = a.n_planes / nb * nb;
    const int rem = a.n_planes - full;
    int c = 1;
    while (rem > 0 && c < 64 && rem * (2 * c) <= nb) c *= 2;
    double kl = 0.0;
    for (int base = 0; base < a.n_planes; base += nb) {
        const bool tail = base >= full;
        const int cc = tail ? c : 1;
        const int p = base + (tail ? (int)threadIdx.x / c : (int)threadIdx.x);
        const int ch = tail ? (int)threadIdx.x % c : 0;
        const bool act = p < a.n_planes;
        const PlaneP P = a.planes[act ? p : 0];
        const int64_t lor = (int64_t)line * a.n_planes + p;
        const float len = sqrtf(L.lt2 + P.dz2);
        const float ell = L.vm_um * len;
        int is = 0, ie = -1;
        if (act && nrow > 0) z_clip(L, P, a.nz, is, ie);
        if constexpr (MODE == M_COUNT) {
            if (ch == 0 && ie >= is) kl += (double)(ie - is + 1);
            continue;
        }
        // padded axial cell of sample i: u = zA i + zB = z + PADZ, clamped to
        // [0, nz + 2] (the clamp only guards the LDS bounds; z-clipped samples
        // lie inside), where truncation is the floor
        const float zA = P.zs * L.dlam, zB = fmaf(L.lam0, P.zs, P.zb) + (float)PADZ;
        const float umax = (float)(a.nz + PADZ);
        float s = 0.f;
        if (NEED_X) {
            const float *xr = X + (is + ch - L.i_lo) * rz;
            for (int i = is + ch; i <= ie; i += cc, xr += cc * rz) {
                const float u = __builtin_amdgcn_fmed3f(fmaf((float)i, zA, zB), 0.f, umax);
                const int j = (int)u;
                const float x0 = xr[j], x1 = xr[j + 1];
                s += fmaf(__builtin_amdgcn_fractf(u), x1 - x0, x0);
            }
            for (int o = 1; o < cc; o <<= 1) s += __shfl_xor(s, o, 64);
        }
        if (!act) continue;
        const float m = a.mult ? a.mult[lor] : 1.f;
        float Q = 0.f;
        if constexpr (MODE == M_BACK) {
            Q = (a.sino ? a.sino[lor] : 1.f) * m * ell;
        } else if constexpr (MODE == M_HVP) {
            // data-term Hessian: mult^2 y / ybar^2 (P v), then back
            const float yv = load_y(a.y, a.y_dtype, lor);
            const float yb = a.ybar[lor];
            Q = yv != 0.f ? m * m * yv / (yb * yb) * (s * ell) * ell : 0.f;
        } else {
            float ybar = fmaf(m, s * ell, a.add ? a.add[lor] : 0.f);
            if constexpr (MODE == M_FWD) {
                if (ch == 0) a.out[lor] = ybar;
                continue;
            } else {
                float yv = load_y(a.y, a.y_dtype, lor);
                if (a.partial && ch == 0) kl += kl_term(ybar, yv);
                // a bin without counts has d(s, 0) = s: derivative 1 and EM ratio 0,
                // also where ybar = 0 (no 0 * inf)
                if constexpr (MODE == M_GRAD) Q = m * (yv != 0.f ? 1.f - yv / ybar : 1.f) * ell;
                if constexpr (MODE == M_EM) Q = yv != 0.f ? m * (yv / ybar) * ell : 0.f;
            }
        }
        if constexpr (NEED_Z) {
            double *zr = Z + (is + ch - L.i_lo) * rz;
            if (MODE == M_BACK && a.tof_fold) {
                // TOF: sample i at t = (lambda(i) - 1/2) |u| carries the sum of
                // its bins' weights (uniform branch)
                const TofFold F = tof_fold_of(a.tof);
                for (int i = is + ch; i <= ie; i += cc, zr += cc * rz) {
                    const float u = __builtin_amdgcn_fmed3f(fmaf((float)i, zA, zB), 0.f, umax);
                    const int j = (int)u;
                    const float t = (fmaf((float)i, L.dlam, L.lam0) - 0.5f) * len;
                    const float q = Q * tof_fold_weight(F, t);
                    const float a1 = q * __builtin_amdgcn_fractf(u);
                    atomicAdd(&zr[j], (double)(q - a1));
                    atomicAdd(&zr[j + 1], (double)a1);
                }
            } else {
                for (int i = is + ch; i <= ie; i += cc, zr += cc * rz) {
                    const float u = __builtin_amdgcn_fmed3f(fmaf((float)i, zA, zB), 0.f, umax);
                    const int j = (int)u;
                    const float a1 = Q * __builtin_amdgcn_fractf(u);
                    atomicAdd(&zr[j], (double)(Q - a1));
                    atomicAdd(&zr[j + 1], (double)a1);
                }
            }
        }
    }
    if (NEED_Z && nrow > 0) {
        __syncthreads();
        scatter_sheet(a, L, nrow, Z, g_off);
    }
    return kl;
}

template <int MODE>
__global__ void __launch_bounds__(NT_BLOCK) k_line_nt(ProjArgs a) {
    extern __shared__ float4 smem4[];
    // one line per workgroup, the launch's lines longest first
    const double kl = line_nt_body<MODE>(a, a.order[blockIdx.x], reinterpret_cast<float *>(smem4));
    if (MODE != M_FWD && MODE != M_BACK && a.partial) block_sums(kl, kl, a.partial, MODE == M_COUNT);
}

// ---------------------------------------------------------------------------
// TOF: one wave per segment, one plane per lane, shared per-segment table.
//
// Per wave the LDS holds, for the segment being processed:
//   cuts[s]  (s = 0 .. n_int)   first sample (t order) at or beyond edge s;
//   w4[q], w1[q]                the TOF weights of the bins active at sample q
//                               (first four in a float4, the rest after).
// Samples q are numbered in increasing t along the LOR; the sample index,
// lambda and the sheet row follow from q and are the same for all lanes.

// erf of u / (sqrt2 sigma) with the argument clamped to the truncation window.

// Per-wave TOF weight table of one LOR (one segment of the line): lane s
// computes the cut cuts[s] (rows before interval s in t order) and returns it;
// each row q of a non-empty interval gets the weights of its na bins.
__device__ __forceinline__ int fill_table(const ProjArgs &a, const LineP &L, float len, int *cuts, float *w4,
                                          float *w1) {
    const int lane = threadIdx.x & 63;
    const int nq = L.i_hi - L.i_lo + 1;
    const int e1 = a.ws > 4 ? a.ws - 4 : 0;
    int *sid = reinterpret_cast<int *>(w4);  // interval of row q, parked in w4[q].x
    int cut = 0;
    if (lane <= a.tof.n_int) {
        cut = cut_count(a.tof.edge[lane], len, L.lam0, L.dlam, L.i_lo, L.i_hi);
        cuts[lane] = cut;
    }
    for (int q = lane; q < nq; q += 64) sid[4 * q] = -1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // lane s marks the rows of interval s
    if (lane < a.tof.n_int && a.tof.na[lane] > 0) {
        const int hi = cuts[lane + 1];
        for (int q = cut; q < hi; ++q) sid[4 * q] = lane;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const float inv_s = a.tof.inv_sqrt2_sigma, c = a.tof.erf_clamp, h = a.tof.half_bin;
    for (int q = lane; q < nq; q += 64) {
        const int s = sid[4 * q];
        if (s < 0) continue;
        const int na = a.tof.na[s];
        const int i = L.dlam > 0.f ? L.i_lo + q : L.i_hi - q;
        const float lam = fmaf((float)i, L.dlam, L.lam0);
        const float t = (lam - 0.5f) * len;
        // weights of bins bf .. bf + na - 1 from shared bin edges
        const float t0 = a.tof.tb[a.tof.bf[s]] - h - t;
        float e_prev = clamped_erf(t0, inv_s, c);
        float w[WS_MAX];
        for (int j = 0; j < WS_MAX; ++j) w[j] = 0.f;
        for (int j = 0; j < na; ++j) {
            const float e_next = clamped_erf(t0 + (float)(j + 1) * (2.f * h), inv_s, c);
            w[j] = 0.5f * (e_next - e_prev);
            e_prev = e_next;
        }
        reinterpret_cast<float4 *>(w4)[q] = make_float4(w[0], w[1], w[2], w[3]);
        for (int j = 0; j < e1; ++j) w1[q * e1 + j] = w[4 + j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return cut;
}

// Weights of sample q (all lanes read the same row: broadcast reads).
template <int NA>
__device__ __forceinline__ void read_w(const float *w4, const float *w1, int e1, int q, float (&w)[NA]) {
    const float4 v = reinterpret_cast<const float4 *>(w4)[q];
    if (NA > 0) w[0] = v.x;
    if (NA > 1) w[1] = v.y;
    if (NA > 2) w[2] = v.z;
    if (NA > 3) w[3] = v.w;
#pragma unroll
    for (int j = 4; j < NA; ++j) w[j] = w1[q * e1 + (j - 4)];
}

// Sample loops of one TOF interval: n rows walked in t order from row pointer
// xr / zr (row of the first sample, z padding skipped), principal-plane index
// fi stepping by dfi and row stride drz, taking every wstep-th row (the line
// kernels walk every row: wstep = 1).  The weights of a row are the same for
// every lane that walks it (broadcast LDS reads when the whole wave does); the
// axial position of a sample in plane i is zA * i + zB (voxel units).
template <int NA>
__device__ __forceinline__ void read_wq(const float *wq, const float *w1q, float (&w)[NA]) {
    const float4 v = *reinterpret_cast<const float4 *>(wq);
    if (NA > 0) w[0] = v.x;
    if (NA > 1) w[1] = v.y;
    if (NA > 2) w[2] = v.z;
    if (NA > 3) w[3] = v.w;
#pragma unroll
    for (int j = 4; j < NA; ++j) w[j] = w1q[j - 4];
}

// Axial positions are taken in padded-row cells, u = z + PADZ: a sample at
// axial position z interpolates cells floor(u) and floor(u) + 1 of its sheet
// row (the row pointer is the row start).  u is clamped to [0, nz + 2], where
// the truncating conversion is the floor and v_fract the fraction.

// Forward: no lane predicate.  A sample outside the z-valid range
// [-1.5, nz + 0.5] (u outside [0.5, nz + 2.5]) interpolates between two cells
// of the zero padding and adds exactly zero, as does a lane without a plane
// (zA = 0, zB = 0).
template <int NA>
__device__ __forceinline__ void tof_fwd_run(float zA, float zB, float umax, const float *xr, int drz, float fi,
                                            float dfi, const float *wq, const float *w1q, int e1, int wstep, int n,
                                            float *win) {
#pragma unroll 2
    for (; n > 0; --n) {
        float w[NA];
        read_wq<NA>(wq, w1q, w);
        const float u = __builtin_amdgcn_fmed3f(fmaf(fi, zA, zB), 0.f, umax);
        const int j = (int)u;
        const float f = __builtin_amdgcn_fractf(u);
        const float x0 = xr[j], x1 = xr[j + 1];
        const float v = fmaf(f, x1 - x0, x0);
#pragma unroll
        for (int b = 0; b < NA; ++b) win[b] = fmaf(v, w[b], win[b]);
        xr += drz;
        fi += dfi;
        wq += 4 * wstep;
        w1q += e1 * wstep;
    }
}

// Adjoint: a lane adds its samples k = q - qlo in [0, span] only.
template <int NA>
__device__ __forceinline__ void tof_back_run(float zA, float zB, float umax, double *zr, int drz, float fi, float dfi,
                                             const float *wq, const float *w1q, int e1, int wstep, int n, int k,
                                             unsigned span, const float *win) {
#pragma unroll 2
    for (; n > 0; --n) {
        float w[NA];
        read_wq<NA>(wq, w1q, w);
        float Q = 0.f;
#pragma unroll
        for (int b = 0; b < NA; ++b) Q = fmaf(win[b], w[b], Q);
        if ((unsigned)k <= span) {
            // (the clamp only guards the LDS bounds; valid samples lie inside)
            const float u = __builtin_amdgcn_fmed3f(fmaf(fi, zA, zB), 0.f, umax);
            const int j = (int)u;
            const float a1 = Q * __builtin_amdgcn_fractf(u);
            atomicAdd(&zr[j], (double)(Q - a1));
            atomicAdd(&zr[j + 1], (double)a1);
        }
        zr += drz;
        fi += dfi;
        wq += 4 * wstep;
        w1q += e1 * wstep;
        k += wstep;
    }
}

// Bin window <-> the per-bin accumulators of one block of NT_BLK bins.  The
// window's first bin relative to the block, REL (from -(WS_MAX - 1) to
// NT_BLK - 1), is a template argument so that every register index is static:
// indexing a register array by a run-time value compiles to indexed register
// moves, which the compiler may execute speculatively for indices the source
// guards out and which then write registers past the array.
template <int REL>
__device__ __forceinline__ void add_window(float (&acc)[NT_BLK], const float (&win)[WS_MAX], int na) {
#pragma unroll
    for (int j = 0; j < WS_MAX; ++j)
        if (REL + j >= 0 && REL + j < NT_BLK && j < na) acc[REL + j] += win[j];
}

template <int REL>
__device__ __forceinline__ void get_window(const float (&acc)[NT_BLK], float (&win)[WS_MAX], int na) {
#pragma unroll
    for (int j = 0; j < WS_MAX; ++j) win[j] = (REL + j >= 0 && REL + j < NT_BLK && j < na) ? acc[REL + j] : 0.f;
}

static_assert(NT_BLK == 16 && WS_MAX == 8, "the window switch below covers first bins -7 .. 15 of a block");
#define PET_REL_SWITCH(FN, ...)                \
    switch (rel) {                             \
        case -7: FN<-7>(__VA_ARGS__); break;   \
        case -6: FN<-6>(__VA_ARGS__); break;   \
        case -5: FN<-5>(__VA_ARGS__); break;   \
        case -4: FN<-4>(__VA_ARGS__); break;   \
        case -3: FN<-3>(__VA_ARGS__); break;   \
        case -2: FN<-2>(__VA_ARGS__); break;   \
        case -1: FN<-1>(__VA_ARGS__); break;   \
        case 0: FN<0>(__VA_ARGS__); break;     \
        case 1: FN<1>(__VA_ARGS__); break;     \
        case 2: FN<2>(__VA_ARGS__); break;     \
        case 3: FN<3>(__VA_ARGS__); break;     \
        case 4: FN<4>(__VA_ARGS__); break;     \
        case 5: FN<5>(__VA_ARGS__); break;     \
        case 6: FN<6>(__VA_ARGS__); break;     \
        case 7: FN<7>(__VA_ARGS__); break;     \
        case 8: FN<8>(__VA_ARGS__); break;     \
        case 9: FN<9>(__VA_ARGS__); break;     \
        case 10: FN<10>(__VA_ARGS__); break;   \
        case 11: FN<11>(__VA_ARGS__); break;   \
        case 12: FN<12>(__VA_ARGS__); break;   \
        case 13: FN<13>(__VA_ARGS__); break;   \
        case 14: FN<14>(__VA_ARGS__); break;   \
        default: FN<15>(__VA_ARGS__); break;   \
    }

#define PET_NA_SWITCH(FN, ...)              \
    switch (na) {                           \
        case 1: FN<1>(__VA_ARGS__); break;  \
        case 2: FN<2>(__VA_ARGS__); break;  \
        case 3: FN<3>(__VA_ARGS__); break;  \
        case 4: FN<4>(__VA_ARGS__); break;  \
        case 5: FN<5>(__VA_ARGS__); break;  \
        case 6: FN<6>(__VA_ARGS__); break;  \
        case 7: FN<7>(__VA_ARGS__); break;  \
        default: FN<8>(__VA_ARGS__); break; \
    }

// Live intervals of a segment wave as a bit mask (bit s: interval s).  With the
// rows split over C chunks, chunk k takes the k-th set bit (-1 if there are
// fewer), and the wave then drops the lowest C.
__device__ __forceinline__ int kth_interval(uint64_t mk, int k) {
    for (int i = 0; i < k && mk; ++i) mk &= mk - 1;
    return mk ? (int)__builtin_ctzll(mk) : -1;
}
__device__ __forceinline__ uint64_t drop_intervals(uint64_t mk, int c) {
    for (int i = 0; i < c && mk; ++i) mk &= mk - 1;
    return mk;
}

// One transaxial line of a TOF geometry by the whole workgroup, segments
// spread over the first nwaves waves (the others only help with the sheets);
// adds this thread's FP64 partials (KL or samples, and sample-bin pairs) to
// kl and pairs.
template <int MODE>
__device__ __forceinline__ void line_tof_body(const ProjArgs &a, int line, float *smem, int nwaves, double &kl,
                                              double &pairs, int64_t g_off = 0) {
    constexpr bool NEED_X = MODE != M_BACK && MODE != M_COUNT;
    constexpr bool NEED_Z = MODE == M_BACK || MODE == M_GRAD || MODE == M_EM || MODE == M_HVP;
    const int lane = threadIdx.x & 63;
    // wave index and wave count are wave-uniform: the segment loop below runs
    // under scalar control flow
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    nwaves = __builtin_amdgcn_readfirstlane(nwaves);
    const LineP L = a.lines[line];
    const int nrow = L.i_hi - L.i_lo + 1;
    const int rz = a.rz;
    const int nt = a.tof.n_tof;
    // LDS: X sheet (float) | Z sheet (double) | per wave: w4 [rows][4], w1 [rows][e1], cuts
    const int sheet = (a.rows_max * rz + 3) & ~3;
    const int ws = a.ws;  // widest bin window of any interval
    const int e1 = ws > 4 ? ws - 4 : 0;
    const int per_wave = a.rows_max * (4 + e1) + tof_cuts_pad(a.tof.n_int);
    float *X = smem;
    double *Z = reinterpret_cast<double *>(smem + (NEED_X ? sheet : 0));
    float *wave_mem = smem + (NEED_X ? sheet : 0) + (NEED_Z ? 2 * sheet : 0) + wave * ((per_wave + 3) & ~3);
    float *w4 = wave_mem;
    float *w1 = wave_mem + 4 * a.rows_max;
    int *cuts = (int *)(w1 + a.rows_max * e1);
    if (nrow > 0 && MODE != M_COUNT) build_sheets<NEED_X, NEED_Z>(a, L, nrow, X, Z);
    __syncthreads();

    // lane s holds the bin count and first bin of interval s
    const int na_l = lane < a.tof.n_int ? a.tof.na[lane] : 0;
    const int bf_l = lane < a.tof.n_int ? a.tof.bf[lane] : 0;

    // segments -k and +k have the same oblique length and so the same weight
    // table: the segment list puts such pairs in consecutive rounds of a wave,
    // which then fills the table once
    float table_dz2 = -1.f;
    for (int sg = wave; wave < nwaves && sg < a.n_seg; sg += nwaves) {
        const SegP S = a.segs[sg];
        // lanes: plane pl of the segment and chunk ch; a segment of at most 32
        // planes splits its live intervals over C = 64 / np_pad chunks (np_pad
        // the planes rounded up to a power of two)
        int lg = 0;
        while ((1 << lg) < S.np) ++lg;
        lg = __builtin_amdgcn_readfirstlane(lg);
        const int np_pad = 1 << lg, C = 64 >> lg;
        const bool has = (lane & (np_pad - 1)) < S.np;
        const int p = S.p0 + (has ? (lane & (np_pad - 1)) : 0);
        const PlaneP P = a.planes[p];
        const int64_t lor = (int64_t)line * a.n_planes + p;
        const float len = sqrtf(L.lt2 + S.dz2);
        const float ell = L.vm_um * len;
        int is = 0, ie = -1;
        if (nrow > 0 && has) z_clip<true>(L, P, a.nz, is, ie);
        // this lane's samples in t order: q in [qlo, qhi]
        const int qlo = L.dlam > 0.f ? is - L.i_lo : L.i_hi - ie;
        const int qhi = L.dlam > 0.f ? ie - L.i_lo : L.i_hi - is;

        if constexpr (MODE == M_COUNT) {
            if (nrow > 0 && ie >= is && lane < np_pad) {
                kl += (double)(ie - is + 1);
                for (int s = 0; s < a.tof.n_int; ++s) {
                    const int na = a.tof.na[s];
                    if (na <= 0) continue;
                    const int c0 = max(cut_count(a.tof.edge[s], len, L.lam0, L.dlam, L.i_lo, L.i_hi), qlo);
                    const int c1 = min(cut_count(a.tof.edge[s + 1], len, L.lam0, L.dlam, L.i_lo, L.i_hi), qhi + 1);
                    if (c1 > c0) pairs += (double)na * (c1 - c0);
                }
            }
        } else {
            int cut = 0;
            if (S.dz2 != table_dz2) {
                cut = nrow > 0 ? fill_table(a, L, len, cuts, w4, w1) : 0;
                table_dz2 = S.dz2;
            } else if (nrow > 0 && lane <= a.tof.n_int) {
                cut = cuts[lane];  // kept in the table by the fill
            }
            // axial sample position of row i: xz = zA * i + zB
            // padded axial cell of row i: u = zA * i + zB (z + PADZ)
            const float zA = P.zs * L.dlam, zB = fmaf(L.lam0, P.zs, P.zb) + (float)PADZ;
            const float zAf = has ? zA : 0.f, zBf = has ? zB : 0.f, umax = (float)(a.nz + PADZ);
            const int drz = L.dlam > 0.f ? rz : -rz;
            const float dfi = L.dlam > 0.f ? 1.f : -1.f;
            // back-projection predicate: k = q - qlo_b in [0, span]; a lane with
            // no samples gets a base far below every row
            const unsigned span = qlo <= qhi ? (unsigned)(qhi - qlo) : 0u;
            const int qlo_b = qlo <= qhi ? qlo : -(1 << 30);
            const int cut_next = __shfl_down(cut, 1, 64);
            // intervals with bins whose rows meet some lane's sample range
            int qa = qlo <= qhi ? qlo : INT_MAX, qb = qlo <= qhi ? qhi : -1;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                qa = min(qa, __shfl_xor(qa, o, 64));
                qb = max(qb, __shfl_xor(qb, o, 64));
            }
            const bool meets = nrow > 0 && na_l > 0 && max(cut, qa) < min(cut_next, qb + 1);
            const float m = has ? (a.mult ? a.mult[lor] : 1.f) : 0.f;
            const int64_t base = lor * nt;

            // TOF bins in blocks of NT_BLK held in registers (one block unless
            // the geometry has more bins); an interval whose bins straddle two
            // blocks is walked once per block
            for (int b0 = 0; b0 < nt; b0 += NT_BLK) {
                const int nb = min(NT_BLK, nt - b0);
                const uint64_t live_mask = __ballot(meets && bf_l < b0 + NT_BLK && bf_l + na_l > b0);
                float acc[NT_BLK];
#pragma unroll
                for (int b = 0; b < NT_BLK; ++b) acc[b] = 0.f;

                // ---- forward projection ----
                if (NEED_X) {
                    if (C == 1) {
                        // every lane walks the same rows of one interval at a time: a scalar loop
                        for (uint64_t mk = live_mask; mk; mk &= mk - 1) {
                            const int s = __builtin_amdgcn_readfirstlane(__builtin_ctzll(mk));
                            const int na = __builtin_amdgcn_readlane(na_l, s);
                            const int c0 = __builtin_amdgcn_readlane(cut, s);
                            const int c1 = __builtin_amdgcn_readlane(cut_next, s);
                            const int rel = __builtin_amdgcn_readlane(bf_l, s) - b0;
                            float win[WS_MAX];
#pragma unroll
                            for (int j = 0; j < WS_MAX; ++j) win[j] = 0.f;
                            const int i0 = L.dlam > 0.f ? L.i_lo + c0 : L.i_hi - c0;
                            const float *xr0 = X + (i0 - L.i_lo) * rz;
                            PET_NA_SWITCH(tof_fwd_run, zAf, zBf, umax, xr0, drz, (float)i0, dfi, w4 + 4 * c0,
                                          w1 + c0 * e1, e1, 1, c1 - c0, win)
                            PET_REL_SWITCH(add_window, acc, win, na)
                        }
                    } else {
                        // chunk k = lane >> lg takes all rows of the k-th of the next C live
                        // intervals, with the geometry's widest window (the weights past an
                        // interval's own bins are zero)
                        for (uint64_t mk = live_mask; mk; mk = drop_intervals(mk, C)) {
                            const int s = kth_interval(mk, lane >> lg);
                            const int sc = s < 0 ? 0 : s;
                            // every lane shuffles (a lane-permute reads zero from a lane that
                            // is switched off), then selects
                            const int c0 = __shfl(cut, sc, 64), c1 = __shfl(cut_next, sc, 64);
                            const int nas = __shfl(na_l, sc, 64), bfs = __shfl(bf_l, sc, 64);
                            const int rel = s < 0 ? 0 : bfs - b0;
                            const int nl = s < 0 ? 0 : c1 - c0;
                            float win[WS_MAX];
#pragma unroll
                            for (int j = 0; j < WS_MAX; ++j) win[j] = 0.f;
                            const int i0 = L.dlam > 0.f ? L.i_lo + c0 : L.i_hi - c0;
                            const float *xr0 = X + (i0 - L.i_lo) * rz;
                            {
                                const int na = ws;
                                PET_NA_SWITCH(tof_fwd_run, zAf, zBf, umax, xr0, drz, (float)i0, dfi, w4 + 4 * c0,
                                              w1 + c0 * e1, e1, 1, nl, win)
                            }
                            {
                                const int na = s < 0 ? 0 : nas;
                                PET_REL_SWITCH(add_window, acc, win, na)
                            }
                        }
                    }
                    // the chunks of a plane hold partial sums over their intervals
                    for (int o = np_pad; o < 64; o <<= 1) {
#pragma unroll
                        for (int b = 0; b < NT_BLK; ++b) acc[b] += __shfl_xor(acc[b], o, 64);
                    }
                }

                // ---- ratio / output ----
                if (has) {
                    const int64_t bb = base + b0;
                    if constexpr (MODE == M_BACK) {
                        float sv[NT_BLK];
                        if (a.sino) load_row(a.sino, bb, nb, sv);
#pragma unroll
                        for (int b = 0; b < NT_BLK; ++b) acc[b] = (a.sino ? sv[b] : 1.f) * m * ell;
                    } else if constexpr (MODE == M_HVP) {
                        float yb[NT_BLK], yv[NT_BLK];
                        load_row(a.ybar, bb, nb, yb);
                        load_y_row(a.y, a.y_dtype, bb, nb, yv);
#pragma unroll
                        for (int b = 0; b < NT_BLK; ++b)
                            acc[b] = (b < nb && yv[b] != 0.f) ? m * m * yv[b] / (yb[b] * yb[b]) * (acc[b] * ell) * ell
                                                              : 0.f;
                    } else {
                        float ad[NT_BLK], yv[NT_BLK];
#pragma unroll
                        for (int b = 0; b < NT_BLK; ++b) ad[b] = 0.f;
                        if (a.add) load_row(a.add, bb, nb, ad);
                        if constexpr (MODE != M_FWD) load_y_row(a.y, a.y_dtype, bb, nb, yv);
#pragma unroll
                        for (int b = 0; b < NT_BLK; ++b) {
                            if (b >= nb) continue;
                            const float ybar = fmaf(m, acc[b] * ell, ad[b]);
                            if constexpr (MODE == M_FWD) {
                                if (lane < np_pad) a.out[bb + b] = ybar;
                            } else {
                                if (a.partial && lane < np_pad) kl += kl_term(ybar, yv[b]);
                                if constexpr (MODE == M_GRAD)
                                    acc[b] = m * (yv[b] != 0.f ? fmaf(-yv[b], __builtin_amdgcn_rcpf(ybar), 1.f) : 1.f) * ell;
                                if constexpr (MODE == M_EM)
                                    acc[b] = yv[b] != 0.f ? m * (yv[b] * __builtin_amdgcn_rcpf(ybar)) * ell : 0.f;
                            }
                        }
                    }
                }

                // ---- adjoint into the LDS gradient sheet ----
                if (NEED_Z) {
                    if (C == 1) {
                        for (uint64_t mk = live_mask; mk; mk &= mk - 1) {
                            const int s = __builtin_amdgcn_readfirstlane(__builtin_ctzll(mk));
                            const int na = __builtin_amdgcn_readlane(na_l, s);
                            const int c0 = __builtin_amdgcn_readlane(cut, s);
                            const int c1 = __builtin_amdgcn_readlane(cut_next, s);
                            const int rel = __builtin_amdgcn_readlane(bf_l, s) - b0;
                            float win[WS_MAX];
                            PET_REL_SWITCH(get_window, acc, win, na)
                            const int i0 = L.dlam > 0.f ? L.i_lo + c0 : L.i_hi - c0;
                            double *zr0 = Z + (i0 - L.i_lo) * rz;
                            PET_NA_SWITCH(tof_back_run, zA, zB, umax, zr0, drz, (float)i0, dfi, w4 + 4 * c0,
                                          w1 + c0 * e1, e1, 1, c1 - c0, c0 - qlo_b, span, win)
                        }
                    } else {
                        // the intervals split over the chunks as in the forward pass
                        for (uint64_t mk = live_mask; mk; mk = drop_intervals(mk, C)) {
                            const int s = kth_interval(mk, lane >> lg);
                            const int sc = s < 0 ? 0 : s;
                            // every lane shuffles (a lane-permute reads zero from a lane that
                            // is switched off), then selects
                            const int c0 = __shfl(cut, sc, 64), c1 = __shfl(cut_next, sc, 64);
                            const int nas = __shfl(na_l, sc, 64), bfs = __shfl(bf_l, sc, 64);
                            const int rel = s < 0 ? 0 : bfs - b0;
                            const int nl = s < 0 ? 0 : c1 - c0;
                            float win[WS_MAX];
                            {
                                const int na = s < 0 ? 0 : nas;
                                PET_REL_SWITCH(get_window, acc, win, na)
                            }
                            const int i0 = L.dlam > 0.f ? L.i_lo + c0 : L.i_hi - c0;
                            double *zr0 = Z + (i0 - L.i_lo) * rz;
                            {
                                const int na = ws;
                                PET_NA_SWITCH(tof_back_run, zA, zB, umax, zr0, drz, (float)i0, dfi, w4 + 4 * c0,
                                              w1 + c0 * e1, e1, 1, nl, c0 - qlo_b, span, win)
                            }
                        }
                    }
                }
            }
            // the next segment may overwrite this wave's table
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (NEED_Z && nrow > 0) {
        __syncthreads();
        scatter_sheet(a, L, nrow, Z, g_off);
    }
}

// One line per workgroup, in the order a.order (longest first).
template <int MODE>
__global__ void __launch_bounds__(64 * TOF_MAX_WAVES) k_line_tof(ProjArgs a) {
    extern __shared__ float4 smem4[];
    double kl = 0.0, pairs = 0.0;
    line_tof_body<MODE>(a, a.order[blockIdx.x], reinterpret_cast<float *>(smem4), blockDim.x >> 6, kl, pairs);
    if (MODE != M_FWD && MODE != M_BACK && a.partial) block_sums(kl, pairs, a.partial, MODE == M_COUNT);
}

// Persistent subset-gradient kernel over a batch: the work items of one step
// are the transaxial lines of every active member (all lines at a snapshot,
// each into the gradient-sheet slot of its view's subset; else the lines of
// the step's subset into slot 0), concatenated in `order`.  Workgroups take
// items from a global counter (zeroed by the step's prep kernel) until none
// is left.
__global__ void __launch_bounds__(64 * TOF_MAX_WAVES) k_line_batched(const BMember *__restrict__ mem,
                                                                     const int *__restrict__ order, int n_mem,
                                                                     int step, int *__restrict__ counter) {
    extern __shared__ float4 smem4[];
    float *smem = reinterpret_cast<float *>(smem4);
    __shared__ int s_cum[BATCH_MAX + 1];
    __shared__ int s_item;
    if (threadIdx.x == 0) {
        int c = 0;
        for (int q = 0; q < n_mem; ++q) {
            s_cum[q] = c;
            const BMember &m = mem[order[q]];
            const BStep st = m.steps[step];
            if (st.flags & B_ACTIVE) c += ((st.flags & B_SNAP) ? m.n_views : m.sub_nviews[st.subset]) * m.pa.n_rad;
        }
        s_cum[n_mem] = c;
    }
    __syncthreads();
    const int total = s_cum[n_mem];
    const int nw = blockDim.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= total) break;
        int q = 0;
        while (s_cum[q + 1] <= item) ++q;
        const BMember &m = mem[order[q]];
        const BStep st = m.steps[step];
        const int local = item - s_cum[q];
        const int n_rad = m.pa.n_rad;
        const int jv = local / n_rad;
        const int k = local - jv * n_rad;
        const bool snap = (st.flags & B_SNAP) != 0;
        const int view = snap ? jv : m.views[st.subset * m.views_stride + jv];
        const int64_t g_off = snap ? (int64_t)(jv % m.n_sub) * m.g_slot : 0;
        if (m.is_tof) {
            double kl = 0.0, pairs = 0.0;
            line_tof_body<M_GRAD>(m.pa, view * n_rad + k, smem, min(m.tof_waves, nw), kl, pairs, g_off);
        } else {
            line_nt_body<M_GRAD>(m.pa, view * n_rad + k, smem, g_off);
        }
        __syncthreads();
    }
}

template <int MODE>
hipError_t launch_mode(const pet_geom_s *g, dim3 grid, const ProjArgs &a, hipStream_t s) {
    const size_t lds = MODE == M_COUNT ? 0 : g->lds_bytes;
    if (g->d.n_tof > 1)
        hipLaunchKernelGGL((k_line_tof<MODE>), grid, dim3(64 * g->tof_waves), lds, s, a);
    else
        hipLaunchKernelGGL((k_line_nt<MODE>), grid, dim3(g->nt_threads), lds, s, a);
    return hipGetLastError();
}

// Raise the dynamic-LDS limit of the line kernels to what this geometry needs
// (checked against the device limit at creation).  Only needed above the
// default; a failure here is reported by the launch itself.
void set_lds_attr(size_t need) {
    static size_t granted = 64 * 1024;
    if (need <= granted) return;
    const void *fns[] = {(const void *)k_line_nt<M_FWD>,   (const void *)k_line_nt<M_BACK>,
                         (const void *)k_line_nt<M_GRAD>,  (const void *)k_line_nt<M_EM>,
                         (const void *)k_line_nt<M_OBJ>,   (const void *)k_line_nt<M_HVP>,
                         (const void *)k_line_tof<M_FWD>,  (const void *)k_line_tof<M_BACK>,
                         (const void *)k_line_tof<M_GRAD>, (const void *)k_line_tof<M_EM>,
                         (const void *)k_line_tof<M_OBJ>,  (const void *)k_line_tof<M_HVP>};
    hipError_t e = hipSuccess;
    for (const void *f : fns)
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
    if (e == hipSuccess) granted = need;
    (void)hipGetLastError();
}

// TOF backprojection of mult alone (the sensitivity P^T mult, no sinogram):
// with the bins' weights summed per sample, the non-TOF walk does it, one
// sample loop per LOR instead of one per TOF bin.  Its FP64 gradient sheet
// (rows_max x rz) is the only LDS it needs, less than the TOF kernels'.
hipError_t launch_back_fold(const pet_geom_s *g, dim3 grid, const ProjArgs &a0, hipStream_t s) {
    ProjArgs a = a0;
    a.tof_fold = 1;
    const size_t lds = sizeof(double) * (((size_t)g->rows_max * (g->d.nz + 2 * PADZ) + 3) & ~(size_t)3);
    hipLaunchKernelGGL((k_line_nt<M_BACK>), grid, dim3(g->nt_threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_line_kernel_impl(const pet_geom_s *g, int mode, dim3 grid, const ProjArgs &a, hipStream_t s) {
    set_lds_attr(g->lds_bytes);
    switch (mode) {
        case M_FWD: return launch_mode<M_FWD>(g, grid, a, s);
        case M_BACK:
            if (g->d.n_tof > 1 && !a.sino) return launch_back_fold(g, grid, a, s);
            return launch_mode<M_BACK>(g, grid, a, s);
        case M_GRAD: return launch_mode<M_GRAD>(g, grid, a, s);
        case M_EM: return launch_mode<M_EM>(g, grid, a, s);
        case M_OBJ: return launch_mode<M_OBJ>(g, grid, a, s);
        case M_COUNT: return launch_mode<M_COUNT>(g, grid, a, s);
        case M_HVP: return launch_mode<M_HVP>(g, grid, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t prime_line_batched(size_t lds) {
    static size_t granted = 64 * 1024;
    if (lds <= granted) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void *)k_line_batched, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) granted = lds;
    return e;
}

hipError_t launch_line_batched(const BMember *mem, const int *order, int n_mem, int step, int *counter, int blocks,
                               int waves, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(k_line_batched, dim3(blocks), dim3(64 * waves), lds, s, mem, order, n_mem, step, counter);
    return hipGetLastError();
}

int n_line_blocks(const pet_geom_s *g, int subset) {
    const int nv = subset < 0 ? g->d.n_views : (int)g->subset_views[subset].size();
    return nv * g->d.n_rad;
}

hipError_t launch_line_kernel(pet_geom_s *g, int mode, int subset, const ProjArgs &a, hipStream_t s) {
    dim3 grid(n_line_blocks(g, subset));
    if (grid.x == 0) return hipSuccess;
    if (!g->profiling) return launch_line_kernel_impl(g, mode, grid, a, s);
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!g->prof_pool.empty()) {
        ev = g->prof_pool.back();
        g->prof_pool.pop_back();
    } else {
        hipError_t e = hipEventCreate(&ev.first);
        if (e == hipSuccess) e = hipEventCreate(&ev.second);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(ev.first, s);
    if (e == hipSuccess) e = launch_line_kernel_impl(g, mode, grid, a, s);
    if (e == hipSuccess) e = hipEventRecord(ev.second, s);
    g->prof_events[mode].push_back(ev);
    return e;
}

}  // namespace pet
