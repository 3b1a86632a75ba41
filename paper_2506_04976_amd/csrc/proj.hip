// Joseph projector kernels for gfx950 (forward, adjoint, fused subset gradient,
// EM ratio, KL objective), line-driven with LDS sheets.
//
// Separability used here: every LOR of a transaxial line (view, radial) has the
// same principal axis m, the same sample positions lambda(i) along m and the
// same transaxial interpolation coordinate; only z (and the step length via
// |u|) depends on the ring pair.  A workgroup therefore owns one line:
//   1. it interpolates the image once along the transaxial axis into an LDS
//      "sheet" X[i][z] (rows i along m, z padded), reading a z-contiguous
//      transposed copy of the image so the loads are coalesced;
//   2. each thread takes planes (ring pairs) of the line and walks the samples
//      with one linear interpolation in z from LDS per sample (TOF: weighted
//      into the TOF bins through an interval table and a weight table in LDS);
//   3. the adjoint accumulates Z[i][z] in LDS with LDS atomics and finally
//      spreads the sheet back over the two transaxial neighbours with global
//      atomics into a z-contiguous transposed gradient image.
// The arithmetic is Joseph's: sample value = bilinear interpolation of the
// image in the two non-principal axes, line integral = step length * sum.
#include "pet_internal.h"

namespace pet {
namespace {

__device__ __forceinline__ float load_y(const void *y, int dt, int64_t idx) {
    if (dt == PET_Y_U8) return (float)((const uint8_t *)y)[idx];
    if (dt == PET_Y_U16) return (float)((const uint16_t *)y)[idx];
    return ((const float *)y)[idx];
}

// Poisson deviance term d(ybar, y) of the KL data fidelity, FP64.
__device__ __forceinline__ double kl_term(float ybar, float yv) {
    double s = ybar, t = yv;
    if (t > 0.0) return s - t + t * log(t / s);
    return s;
}

__device__ __forceinline__ float tof_w(const float *lut, float d, float inv_h) {
    float u = fminf(fabsf(d) * inv_h, (float)LUT_N);
    int j = min((int)u, LUT_N - 1);
    float f = u - (float)j;
    float l0 = lut[j], l1 = lut[j + 1];
    return fmaf(f, l1 - l0, l0);
}

// Number of samples (in increasing-t order) with t < e.
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

struct LorGeo {
    float lam0, dlam, zb, zs, len;
    int is, ie, ilo, rz;
};

// Forward TOF accumulation over the samples q in [c0, c1) of one interval with
// NA active bins starting at bin bf.
template <int NA>
__device__ __forceinline__ void tof_fwd_run(const LorGeo &G, const float *X, const float *lut, float inv_h,
                                            const float *tbj, int c0, int c1, float *win) {
    for (int q = c0; q < c1; ++q) {
        int i = G.dlam > 0.f ? G.is + q : G.ie - q;
        float lam = fmaf((float)i, G.dlam, G.lam0);
        float xz = fmaf(lam, G.zs, G.zb);
        float jf = floorf(xz);
        float f = xz - jf;
        int r = (i - G.ilo) * G.rz + (int)jf + PADZ;
        float x0 = X[r], x1 = X[r + 1];
        float v = fmaf(f, x1 - x0, x0);
        float t = (lam - 0.5f) * G.len;
#pragma unroll
        for (int j = 0; j < NA; ++j) win[j] = fmaf(v, tof_w(lut, t - tbj[j], inv_h), win[j]);
    }
}

template <int NA>
__device__ __forceinline__ void tof_back_run(const LorGeo &G, float *Z, const float *lut, float inv_h,
                                             const float *tbj, int c0, int c1, const float *win) {
    for (int q = c0; q < c1; ++q) {
        int i = G.dlam > 0.f ? G.is + q : G.ie - q;
        float lam = fmaf((float)i, G.dlam, G.lam0);
        float xz = fmaf(lam, G.zs, G.zb);
        float jf = floorf(xz);
        float f = xz - jf;
        int r = (i - G.ilo) * G.rz + (int)jf + PADZ;
        float t = (lam - 0.5f) * G.len;
        float Q = 0.f;
#pragma unroll
        for (int j = 0; j < NA; ++j) Q = fmaf(win[j], tof_w(lut, t - tbj[j], inv_h), Q);
        float a1 = Q * f;
        atomicAdd(&Z[r], Q - a1);
        atomicAdd(&Z[r + 1], a1);
    }
}

template <int W>
__device__ __forceinline__ void tof_dispatch_fwd(int na, const LorGeo &G, const float *X, const float *lut,
                                                 float inv_h, const float *tbj, int c0, int c1, float *win) {
    switch (na) {
        case 1: tof_fwd_run<1>(G, X, lut, inv_h, tbj, c0, c1, win); break;
        case 2: tof_fwd_run<2>(G, X, lut, inv_h, tbj, c0, c1, win); break;
        case 3: tof_fwd_run<3>(G, X, lut, inv_h, tbj, c0, c1, win); break;
        case 4: tof_fwd_run<4>(G, X, lut, inv_h, tbj, c0, c1, win); break;
        default:
            if constexpr (W > 4) {
                switch (na) {
                    case 5: tof_fwd_run<5>(G, X, lut, inv_h, tbj, c0, c1, win); break;
                    case 6: tof_fwd_run<6>(G, X, lut, inv_h, tbj, c0, c1, win); break;
                    case 7: tof_fwd_run<7>(G, X, lut, inv_h, tbj, c0, c1, win); break;
                    default: tof_fwd_run<8>(G, X, lut, inv_h, tbj, c0, c1, win); break;
                }
            }
    }
}

template <int W>
__device__ __forceinline__ void tof_dispatch_back(int na, const LorGeo &G, float *Z, const float *lut,
                                                  float inv_h, const float *tbj, int c0, int c1, const float *win) {
    switch (na) {
        case 1: tof_back_run<1>(G, Z, lut, inv_h, tbj, c0, c1, win); break;
        case 2: tof_back_run<2>(G, Z, lut, inv_h, tbj, c0, c1, win); break;
        case 3: tof_back_run<3>(G, Z, lut, inv_h, tbj, c0, c1, win); break;
        case 4: tof_back_run<4>(G, Z, lut, inv_h, tbj, c0, c1, win); break;
        default:
            if constexpr (W > 4) {
                switch (na) {
                    case 5: tof_back_run<5>(G, Z, lut, inv_h, tbj, c0, c1, win); break;
                    case 6: tof_back_run<6>(G, Z, lut, inv_h, tbj, c0, c1, win); break;
                    case 7: tof_back_run<7>(G, Z, lut, inv_h, tbj, c0, c1, win); break;
                    default: tof_back_run<8>(G, Z, lut, inv_h, tbj, c0, c1, win); break;
                }
            }
    }
}

// W = 0: non-TOF; W = 4 / 8: TOF with at most W bins overlapping any point.
template <int W, int MODE>
__global__ void __launch_bounds__(LINE_BLOCK) k_line(ProjArgs a) {
    extern __shared__ float smem[];
    constexpr bool NEED_X = MODE != M_BACK && MODE != M_COUNT;
    constexpr bool NEED_Z = MODE == M_BACK || MODE == M_GRAD || MODE == M_EM;
    constexpr int NTA = W == 0 ? 1 : NT_MAX;
    const int tid = threadIdx.x;
    const int jv = blockIdx.x / a.n_rad;
    const int k = blockIdx.x - jv * a.n_rad;
    const int line = a.views[jv] * a.n_rad + k;
    const LineP L = a.lines[line];
    const int nrow = L.i_hi - L.i_lo + 1;  // <= 0: line misses the image
    const int rz = a.rz;
    const int nt = W == 0 ? 1 : a.tof.n_tof;
    const int n_other = L.axis ? a.nx : a.ny;  // size of the transaxial interpolation axis
    const size_t other_stride = (size_t)(n_other + 2 * PADA) * rz;

    float *X = smem;
    float *Z = smem + (NEED_X ? max(nrow, 0) * rz : 0);
    float *lut = Z + (NEED_Z ? max(nrow, 0) * rz : 0);

    if (nrow > 0 && MODE != M_COUNT) {
        if (W > 0)
            for (int e = tid; e <= LUT_N; e += LINE_BLOCK) lut[e] = a.lut[e];
        const float *T = L.axis ? a.T1 : a.T0;
        for (int e = tid; e < nrow * rz; e += LINE_BLOCK) {
            int r = e / rz;
            int zp = e - r * rz;
            if (NEED_X) {
                int i = L.i_lo + r;
                float xa = fmaf((float)i, L.dxa, L.xa0);
                float jf = floorf(xa);
                float f = xa - jf;
                size_t base = (size_t)i * other_stride + (size_t)((int)jf + PADA) * rz + zp;
                float t0 = T[base], t1 = T[base + rz];
                X[e] = fmaf(f, t1 - t0, t0);
            }
            if (NEED_Z) Z[e] = 0.f;
        }
    }
    __syncthreads();

    double kl = 0.0, cnt_pairs = 0.0;
    for (int p = tid; p < a.n_planes; p += LINE_BLOCK) {
        const PlaneP P = a.planes[p];
        const int64_t lor = (int64_t)line * a.n_planes + p;
        LorGeo G;
        G.lam0 = L.lam0;
        G.dlam = L.dlam;
        G.zb = P.zb;
        G.zs = P.zs;
        G.len = sqrtf(L.lt2 + P.dz2);
        G.ilo = L.i_lo;
        G.rz = rz;
        G.is = L.i_lo;
        G.ie = L.i_hi;
        const float ell = L.vm_um * G.len;
        if (nrow > 0) {
            // restrict to samples whose z coordinate can touch the grid
            if (P.zs != 0.f) {
                float la = (-1.5f - P.zb) / P.zs, lb = ((float)a.nz + 0.5f - P.zb) / P.zs;
                float ia = (fminf(la, lb) - L.lam0) / L.dlam, ib = (fmaxf(la, lb) - L.lam0) / L.dlam;
                float lo = ceilf(fminf(ia, ib)), hi = floorf(fmaxf(ia, ib));
                if (lo > (float)G.is) G.is = lo > (float)G.ie ? G.ie + 1 : (int)lo;
                if (hi < (float)G.ie) G.ie = hi < (float)G.is ? G.is - 1 : (int)hi;
            } else if (P.zb < -1.5f || P.zb > (float)a.nz + 0.5f) {
                G.ie = G.is - 1;
            }
        } else {
            G.ie = G.is - 1;
        }

        float acc[NTA];
#pragma unroll
        for (int b = 0; b < NTA; ++b) acc[b] = 0.f;

        if constexpr (MODE == M_COUNT) {
            // the work of this LOR exactly as the other modes traverse it:
            // samples, and sample-bin pairs (TOF; equal to samples without TOF)
            if (G.ie >= G.is) {
                const double ns = (double)(G.ie - G.is + 1);
                double np = ns;
                if constexpr (W > 0) {
                    np = 0.0;
                    for (int s = 0; s < a.tof.n_int; ++s) {
                        const int na = a.tof.na[s];
                        if (na <= 0) continue;
                        const int c0 = cut_count(a.tof.edge[s], G.len, G.lam0, G.dlam, G.is, G.ie);
                        const int c1 = cut_count(a.tof.edge[s + 1], G.len, G.lam0, G.dlam, G.is, G.ie);
                        if (c1 > c0) np += (double)na * (c1 - c0);
                    }
                }
                kl += ns;
                cnt_pairs += np;
            }
            continue;
        }

        // ---- forward projection ----
        if (NEED_X && G.ie >= G.is) {
            if constexpr (W == 0) {
                float s = 0.f;
                for (int i = G.is; i <= G.ie; ++i) {
                    float lam = fmaf((float)i, G.dlam, G.lam0);
                    float xz = fmaf(lam, G.zs, G.zb);
                    float jf = floorf(xz);
                    float f = xz - jf;
                    int r = (i - G.ilo) * rz + (int)jf + PADZ;
                    float x0 = X[r], x1 = X[r + 1];
                    s += fmaf(f, x1 - x0, x0);
                }
                acc[0] = s;
            } else {
                for (int s = 0; s < a.tof.n_int; ++s) {
                    const int na = a.tof.na[s];
                    if (na <= 0) continue;
                    const int c0 = cut_count(a.tof.edge[s], G.len, G.lam0, G.dlam, G.is, G.ie);
                    const int c1 = cut_count(a.tof.edge[s + 1], G.len, G.lam0, G.dlam, G.is, G.ie);
                    const int bf = a.tof.bf[s];
                    float tbj[W], win[W];
#pragma unroll
                    for (int j = 0; j < W; ++j) {
                        tbj[j] = a.tof.tb[min(bf + j, NT_MAX - 1)];
                        win[j] = 0.f;
                    }
                    if (c1 > c0) tof_dispatch_fwd<W>(na, G, X, lut, a.tof.lut_inv_h, tbj, c0, c1, win);
#pragma unroll
                    for (int j = 0; j < W; ++j)
                        if (j < na) acc[bf + j] += win[j];
                }
            }
        }

        // ---- ratio / output ----
        const float m = a.mult ? a.mult[lor] : 1.f;
        for (int b = 0; b < nt; ++b) {
            const int64_t idx = lor * nt + b;
            if constexpr (MODE == M_BACK) {
                acc[b] = (a.sino ? a.sino[idx] : 1.f) * m * ell;
            } else {
                float ybar = fmaf(m, acc[b] * ell, a.add ? a.add[idx] : 0.f);
                if constexpr (MODE == M_FWD) {
                    a.out[idx] = ybar;
                } else {
                    float yv = load_y(a.y, a.y_dtype, idx);
                    if (a.partial) kl += kl_term(ybar, yv);
                    if constexpr (MODE == M_GRAD) acc[b] = m * (1.f - yv / ybar) * ell;
                    if constexpr (MODE == M_EM) acc[b] = m * (yv / ybar) * ell;
                }
            }
        }

        // ---- adjoint into the LDS gradient sheet ----
        if (NEED_Z && G.ie >= G.is) {
            if constexpr (W == 0) {
                const float Q = acc[0];
                for (int i = G.is; i <= G.ie; ++i) {
                    float lam = fmaf((float)i, G.dlam, G.lam0);
                    float xz = fmaf(lam, G.zs, G.zb);
                    float jf = floorf(xz);
                    float f = xz - jf;
                    int r = (i - G.ilo) * rz + (int)jf + PADZ;
                    float a1 = Q * f;
                    atomicAdd(&Z[r], Q - a1);
                    atomicAdd(&Z[r + 1], a1);
                }
            } else {
                for (int s = 0; s < a.tof.n_int; ++s) {
                    const int na = a.tof.na[s];
                    if (na <= 0) continue;
                    const int c0 = cut_count(a.tof.edge[s], G.len, G.lam0, G.dlam, G.is, G.ie);
                    const int c1 = cut_count(a.tof.edge[s + 1], G.len, G.lam0, G.dlam, G.is, G.ie);
                    const int bf = a.tof.bf[s];
                    float tbj[W], win[W];
#pragma unroll
                    for (int j = 0; j < W; ++j) {
                        tbj[j] = a.tof.tb[min(bf + j, NT_MAX - 1)];
                        win[j] = (j < na) ? acc[min(bf + j, NTA - 1)] : 0.f;
                    }
                    if (c1 > c0) tof_dispatch_back<W>(na, G, Z, lut, a.tof.lut_inv_h, tbj, c0, c1, win);
                }
            }
        }
    }

    // ---- spread the gradient sheet over the two transaxial neighbours ----
    if (NEED_Z && nrow > 0) {
        __syncthreads();
        float *Gout = L.axis ? a.G1 : a.G0;
        for (int e = tid; e < nrow * rz; e += LINE_BLOCK) {
            float val = Z[e];
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

    // ---- FP64 block sums: KL terms (or sample / pair counts) ----
    if (MODE != M_FWD && MODE != M_BACK && a.partial) {
        __shared__ double red[2][LINE_BLOCK / 64];
        for (int off = 32; off > 0; off >>= 1) {
            kl += __shfl_down(kl, off, 64);
            cnt_pairs += __shfl_down(cnt_pairs, off, 64);
        }
        if ((tid & 63) == 0) {
            red[0][tid >> 6] = kl;
            red[1][tid >> 6] = cnt_pairs;
        }
        __syncthreads();
        if (tid == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int w = 0; w < LINE_BLOCK / 64; ++w) {
                s0 += red[0][w];
                s1 += red[1][w];
            }
            a.partial[blockIdx.x] = s0;
            if (MODE == M_COUNT) a.partial[gridDim.x + blockIdx.x] = s1;
        }
    }
}

template <int W>
hipError_t launch_w(int mode, dim3 grid, size_t lds, const ProjArgs &a, hipStream_t s) {
    switch (mode) {
        case M_FWD: hipLaunchKernelGGL((k_line<W, M_FWD>), grid, dim3(LINE_BLOCK), lds, s, a); break;
        case M_BACK: hipLaunchKernelGGL((k_line<W, M_BACK>), grid, dim3(LINE_BLOCK), lds, s, a); break;
        case M_GRAD: hipLaunchKernelGGL((k_line<W, M_GRAD>), grid, dim3(LINE_BLOCK), lds, s, a); break;
        case M_EM: hipLaunchKernelGGL((k_line<W, M_EM>), grid, dim3(LINE_BLOCK), lds, s, a); break;
        case M_OBJ: hipLaunchKernelGGL((k_line<W, M_OBJ>), grid, dim3(LINE_BLOCK), lds, s, a); break;
        case M_COUNT: hipLaunchKernelGGL((k_line<W, M_COUNT>), grid, dim3(LINE_BLOCK), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Raise the dynamic-LDS limit of the line kernels to what this geometry needs
// (checked against the device limit at creation).  Only needed above the
// default; a failure here is reported by the launch itself.
template <int W>
void set_lds_attr(size_t need) {
    static size_t granted = 64 * 1024;
    if (need <= granted) return;
    hipError_t e = hipFuncSetAttribute((const void *)k_line<W, M_FWD>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void *)k_line<W, M_BACK>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void *)k_line<W, M_GRAD>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void *)k_line<W, M_EM>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void *)k_line<W, M_OBJ>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
    if (e == hipSuccess) granted = need;
    (void)hipGetLastError();
}

}  // namespace

int n_line_blocks(const pet_geom_s *g, int subset) {
    int nv = subset < 0 ? g->d.n_views : (int)g->subset_views[subset].size();
    return nv * g->d.n_rad;
}

static hipError_t launch_line_kernel_impl(const pet_geom_s *g, int mode, dim3 grid, const ProjArgs &a, hipStream_t s) {
    int wmax = 0;
    if (g->d.n_tof > 1) {
        wmax = 1;
        for (int i = 0; i < g->tof.n_int; ++i) wmax = std::max(wmax, g->tof.na[i]);
    }
    if (wmax == 0) {
        set_lds_attr<0>(g->lds_bytes);
        return launch_w<0>(mode, grid, g->lds_bytes, a, s);
    }
    if (wmax <= 4) {
        set_lds_attr<4>(g->lds_bytes);
        return launch_w<4>(mode, grid, g->lds_bytes, a, s);
    }
    set_lds_attr<8>(g->lds_bytes);
    return launch_w<8>(mode, grid, g->lds_bytes, a, s);
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
