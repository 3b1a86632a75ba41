// Zero-count-aware data term: the bins with counts y > 0, compacted once, and
// the line kernels that walk only them.
//
// The separable Kullback-Leibler data term of Section 1.2 has d(s, 0) = s, so
// a bin without counts contributes mult P x + add to the objective and mult P^T 1
// to the gradient, whatever x is.  The subset gradient therefore splits as
//     grad D_i(x) = P_i^T mult - P_i^T [mult y / ybar(x)],
// where only bins with y > 0 enter the second term, and the objective as
//     D(x) = <P^T mult, x> + sum add - sum y + sum_{y > 0} y log(y / ybar(x)).
// In the SVRG estimator of eq. (svrg) the first term cancels between
// grad D_i(x) and the stored grad D_i(xhat); the full gradient at the
// snapshot is the sensitivity P^T mult plus the sum of the second terms.  So
// the line kernels here compute h_i(x) = -P_i^T [mult y / ybar(x)] and
// sum_{y > 0} y log(y / ybar) from the compacted bins only.
//
// Work layout.  One workgroup per transaxial line with at least one count,
// as in the dense kernels: the image sheet X[i][z] (transaxial interpolation)
// and the FP64 gradient sheet Z[i][z] in LDS, one compacted bin per thread.
// A thread walks the samples of its LOR inside the TOF window of its bin,
// forward and back.  The TOF weight of a sample at signed distance t from
// the LOR centre in bin b depends only on d = t - t_b (the kernel is shift
// invariant): W(d) = 1/2 [E(w/2 - d) - E(-w/2 - d)], E the clamped erf.  It
// is tabulated once per geometry at NW_TAB + 1 nodes over its support
// |d| <= w/2 + nsig sigma (FP64 on the host) and interpolated linearly from
// LDS.
#include "line_sheets.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <new>
#include <vector>

namespace pet {
namespace {

__device__ __forceinline__ float count_y(const void *y, int dt, int64_t idx) {
    if (dt == PET_Y_U8) return (float)((const uint8_t *)y)[idx];
    if (dt == PET_Y_U16) return (float)((const uint16_t *)y)[idx];
    return ((const float *)y)[idx];
}

// Bins with y > 0 per transaxial line, and the FP64 sums of y and of add over
// all bins of the line (add null: 0).
__global__ void __launch_bounds__(256) k_counts_per_line(const void *__restrict__ y, int dt,
                                                         const float *__restrict__ add, int64_t bins_per_line,
                                                         int *__restrict__ cnt, double *__restrict__ ysum,
                                                         double *__restrict__ asum) {
    __shared__ int s_c[4];
    __shared__ double s_y[4], s_a[4];
    const int64_t base = (int64_t)blockIdx.x * bins_per_line;
    int c = 0;
    double sy = 0.0, sa = 0.0;
    for (int64_t k = threadIdx.x; k < bins_per_line; k += blockDim.x) {
        const float v = count_y(y, dt, base + k);
        c += v > 0.f ? 1 : 0;
        sy += (double)v;
        if (add) sa += (double)add[base + k];
    }
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_down(c, off, 64);
        sy += __shfl_down(sy, off, 64);
        sa += __shfl_down(sa, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_c[w] = c;
        s_y[w] = sy;
        s_a[w] = sa;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int ct = 0;
        double yt = 0.0, at = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            ct += s_c[i];
            yt += s_y[i];
            at += s_a[i];
        }
        cnt[blockIdx.x] = ct;
        ysum[blockIdx.x] = yt;
        asum[blockIdx.x] = at;
    }
}

// Compaction of one line's bins with y > 0, TOF bin major (then plane): the
// records that share a wave then have TOF windows at the same place along the
// line, so their sample loops run for about the same number of rows.
__global__ void __launch_bounds__(256) k_counts_fill(const void *__restrict__ y, int dt, const float *__restrict__ add,
                                                     const float *__restrict__ mult, int64_t bins_per_line, int n_tof,
                                                     int n_planes, const int64_t *__restrict__ line_off,
                                                     CountItem *__restrict__ items) {
    __shared__ int s_w[4];
    const int64_t base = (int64_t)blockIdx.x * bins_per_line;
    int64_t out = line_off[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t q0 = 0; q0 < bins_per_line; q0 += blockDim.x) {
        const int64_t q = q0 + threadIdx.x;  // (TOF bin, plane) rank
        const int64_t bq = q / n_planes;
        const int64_t k = (q - bq * n_planes) * n_tof + bq;  // sinogram index within the line
        const float v = q < bins_per_line ? count_y(y, dt, base + k) : 0.f;
        const bool has = v > 0.f;
        const uint64_t m = __ballot(has);
        if (lane == 0) s_w[w] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
        for (int i = 0; i < nw; ++i) {
            before += i < w ? s_w[i] : 0;
            total += s_w[i];
        }
        if (has) {
            const int rank = before + __popcll(m & ((1ull << lane) - 1ull));
            const int plane = (int)(k / n_tof);
            CountItem it;
            it.pt = (uint32_t)k;
            it.y = v;
            it.add = add ? add[base + k] : 0.f;
            it.mult = mult ? mult[(int64_t)blockIdx.x * n_planes + plane] : 1.f;
            items[out + rank] = it;
        }
        out += total;
        __syncthreads();
    }
}

// TOF weight W(d) from the LDS table, at table position pos = d / dx + NW/2:
// linear interpolation between nodes; the position is clamped to the table,
// whose end nodes are 0.
__device__ __forceinline__ float tof_weight_at(const float2 *tab, float pos, float pos_max) {
    pos = __builtin_amdgcn_fmed3f(pos, 0.f, pos_max);
    const float2 t = tab[(int)pos];
    return fmaf(__builtin_amdgcn_fractf(pos), t.y, t.x);
}

// Geometry of one compacted bin within its line: the sample rows [is, ie]
// (z range, then TOF window), the table position pos(i) = pA i + pB of row i,
// the padded axial position u(i) = zA i + zB and the length factor ell.
struct RecGeo {
    int is, ie;
    float pA, pB, zA, zB, ell;
};

template <bool TOF>
__device__ __forceinline__ RecGeo rec_geo(const ProjArgs &a, const CountArgs &c, const LineP &L, const CountItem &e,
                                          bool act) {
    RecGeo r;
    const int p = TOF ? (int)(e.pt / (uint32_t)c.n_tof) : (int)e.pt;
    const int b = TOF ? (int)(e.pt - (uint32_t)p * (uint32_t)c.n_tof) : 0;
    const PlaneP P = a.planes[p];
    const float len = sqrtf(L.lt2 + P.dz2);
    r.ell = L.vm_um * len;
    z_clip<true>(L, P, a.nz, r.is, r.ie);  // (u is clamped by the loops)
    if (!act) r.ie = r.is - 1;
    r.pA = r.pB = 0.f;
    if (TOF) {
        // d(i) = t(i) - t_b, t(i) = (lambda(i) - 1/2) |u| the signed distance
        // from the LOR centre; rows outside |d| <= D (one row of margin, where
        // the table gives 0) are skipped
        const float d0 = fmaf(L.lam0 - 0.5f, len, -a.tof.tb[b]);
        const float dd = L.dlam * len;
        const float rdd = __builtin_amdgcn_rcpf(dd);
        const float ia = (-c.wD - d0) * rdd, ib = (c.wD - d0) * rdd;
        // clamped to [is, ie] (an empty window gives is > ie) before the
        // conversion; the one-row margin covers the reciprocal's rounding
        const float lo = fminf(fmaxf(floorf(fminf(ia, ib)) - 1.f, (float)r.is), (float)(r.ie + 1));
        const float hi = fmaxf(fminf(ceilf(fmaxf(ia, ib)) + 1.f, (float)r.ie), (float)(r.is - 1));
        r.is = (int)lo;
        r.ie = (int)hi;
        r.pA = dd * c.inv_dx;
        r.pB = fmaf(d0, c.inv_dx, c.pos0);
    }
    r.zA = P.zs * L.dlam;
    r.zB = fmaf(L.lam0, P.zs, P.zb) + (float)PADZ;
    return r;
}

// Sum over the workgroup, the same value in every thread (wave sums by
// shuffles, then the wave partials in a fixed order).
__device__ __forceinline__ float block_sum_all(float v, float *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float t = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    return t;
}

// Packed fixed-point gradient sheet.  A sample with weight q at axial
// position u = j + f adds (1 - f) q to cell j and f q to cell j + 1.  Cell j
// holds two 32-bit integer accumulators in one 64-bit word, A[j] (sum of q)
// and B[j] (sum of f q), as A + 2^32 B, so that one 64-bit integer atomic
// add (far cheaper in LDS than two FP64 ones) records a sample; the cell's
// value is then A[j] - B[j] + B[j - 1].  q is scaled by 2^30 / sum_bins |Q|
// (Q the bin's factor mult y / ybar ell, TOF weights <= 1), so neither sum can
// leave 31 bits.  Integer sums do not depend on the order of the adds.
__device__ __forceinline__ void deposit_packed(unsigned long long *zr, int j, float qs, float f) {
    const int A = (int)__builtin_rintf(qs);
    const int B = (int)__builtin_rintf(qs * f);
    const unsigned long long v =
        (unsigned long long)(uint32_t)A | ((unsigned long long)(uint32_t)(B + (A >> 31)) << 32);
    atomicAdd(&zr[j], v);
}

// The two accumulators of a packed cell: the low word read as signed is A,
// and (w - A) is exactly 2^32 B.
__device__ __forceinline__ void unpack_cell(unsigned long long w, long long &A, long long &B) {
    const int lo = (int)(uint32_t)w;
    A = lo;
    B = ((long long)w - (long long)lo) >> 32;
}

// Spread the packed sheet over the two transaxial neighbours (the readout of
// the FP64 sheet in the dense kernels, after unpacking).  A line whose bound
// is not finite (a bin with ybar = 0) adds NaN to every cell it covers.
__device__ __forceinline__ void scatter_sheet_packed(const ProjArgs &a, const LineP &L, int nrow,
                                                     const unsigned long long *Zu, float inv_scale, bool finite) {
    const int rz = a.rz;
    float *Gout = L.axis ? a.G1 : a.G0;
    const size_t other_stride = (size_t)((L.axis ? a.nx : a.ny) + 2 * PADA) * rz;
    for (int e = threadIdx.x; e < nrow * rz; e += blockDim.x) {
        const int r = e / rz;
        const int zp = e - r * rz;
        long long A, B, Ap, Bp = 0;
        unpack_cell(Zu[e], A, B);
        if (zp > 0) unpack_cell(Zu[e - 1], Ap, Bp);
        const long long V = A - B + Bp;
        float val = (float)V * inv_scale;
        if (!finite) val = __builtin_nanf("");
        else if (V == 0) continue;
        const int i = L.i_lo + r;
        const float xa = fmaf((float)i, L.dxa, L.xa0);
        const float jf = floorf(xa);
        const float f = xa - jf;
        const size_t base = (size_t)i * other_stride + (size_t)((int)jf + PADA) * rz + zp;
        const float a1 = val * f;
        atomicAdd(&Gout[base], val - a1);
        atomicAdd(&Gout[base + rz], a1);
    }
}

// One workgroup per line with counts.  MODE M_GRAD: gradient sheets receive
// -P^T [mult y / ybar]; M_OBJ: no gradient.  Both write the workgroup's FP64
// sum of y log(y / ybar) when a.partial is set.
//
// The line's bins are taken in chunks of at most c.q_cap.  Phase one walks
// every bin of the chunk forward (ybar, the log term, Q = mult y / ybar ell,
// kept in LDS); with M_GRAD, phase two walks them again and adds -Q W(t - t_b)
// times the axial interpolation weights to the packed sheet, scaled by the
// chunk's sum of |Q|.  A chunk's sheet is read out before the next starts.
template <bool TOF, int MODE>
__global__ void __launch_bounds__(CNT_BLOCK) k_line_counts(ProjArgs a, CountArgs c) {
    extern __shared__ float4 smem4[];
    float *smem = reinterpret_cast<float *>(smem4);
    __shared__ float red[CNT_BLOCK / 64];
    constexpr bool NEED_Z = MODE == M_GRAD;
    const int line = c.lines[blockIdx.x];
    const LineP L = a.lines[line];
    const int nrow = L.i_hi - L.i_lo + 1;
    const int rz = a.rz;
    const int sheet = (a.rows_max * rz + 3) & ~3;
    float *X = smem;
    unsigned long long *Zu = reinterpret_cast<unsigned long long *>(smem + sheet);
    float2 *tab = reinterpret_cast<float2 *>(smem + (NEED_Z ? 3 : 1) * sheet);
    float *Qs = smem + (NEED_Z ? 3 : 1) * sheet + (TOF ? 2 * NW_TAB : 0);
    if (TOF) {
        // (all of a thread's table loads in flight at once; the kernel runs
        // with CNT_BLOCK threads)
        static_assert(NW_TAB % CNT_BLOCK == 0, "the table load assumes CNT_BLOCK divides NW_TAB");
        float2 w[NW_TAB / CNT_BLOCK];
#pragma unroll
        for (int u = 0; u < NW_TAB / CNT_BLOCK; ++u) w[u] = c.wtab[threadIdx.x + u * CNT_BLOCK];
#pragma unroll
        for (int u = 0; u < NW_TAB / CNT_BLOCK; ++u) tab[threadIdx.x + u * CNT_BLOCK] = w[u];
    }
    if (nrow > 0) build_sheets<true, NEED_Z>(a, L, nrow, X, reinterpret_cast<double *>(Zu));
    __syncthreads();

    double kl = 0.0;
    const int64_t i0 = c.line_off[line], i1 = c.line_off[line + 1];
    const float umax = (float)(a.nz + PADZ);
    // (a line that misses the image still has bins with counts: ybar = add there,
    // and its y log(y / add) enters the sum; its sample ranges are empty)
    for (int64_t c0 = i0; c0 < i1; c0 += c.q_cap) {
        const int64_t c1 = c0 + c.q_cap < i1 ? c0 + c.q_cap : i1;
        // C lanes per bin (a power of two, consecutive lanes of one wave) take
        // every C-th sample of its window; C grows while the chunk's bins
        // still fill the workgroup, so that lines with few bins keep every
        // wave busy
        const int n_c = (int)(c1 - c0);
        int C = 1;
        while (C < 16 && n_c * (2 * C) <= (int)blockDim.x) C *= 2;
        const int ch = threadIdx.x & (C - 1);
        const int nslot = blockDim.x / C;
        const float fC = (float)C;
        float qabs = 0.f;
        for (int64_t it0 = c0; it0 < c1; it0 += nslot) {
            // every lane runs every round: the forward sums are added across
            // the C lanes of a bin by shuffles
            const int64_t it = it0 + threadIdx.x / C;
            const bool act = it < c1;
            const CountItem e = act ? c.items[it] : CountItem{0u, 0.f, 1.f, 0.f};
            const RecGeo g = rec_geo<TOF>(a, c, L, e, act);
            // rows as floats (exact integers): no conversion per sample
            const float fis = (float)(g.is + ch), fie = (float)g.ie;
            float s = 0.f;
            const float *xr = X + (g.is + ch - L.i_lo) * rz;
            for (float fi = fis; fi <= fie; fi += fC, xr += C * rz) {
                const float u = __builtin_amdgcn_fmed3f(fmaf(fi, g.zA, g.zB), 0.f, umax);
                const int j = (int)u;
                const float x0 = xr[j], x1 = xr[j + 1];
                const float v = fmaf(__builtin_amdgcn_fractf(u), x1 - x0, x0);
                s = TOF ? fmaf(tof_weight_at(tab, fmaf(fi, g.pA, g.pB), c.pos_max), v, s) : s + v;
            }
            for (int o = 1; o < C; o <<= 1) s += __shfl_xor(s, o, 64);
            if (!act || ch != 0) continue;
            const float ybar = fmaf(e.mult, s * g.ell, e.add);
            // (the FP64 logarithm only when the sums are wanted)
            if (a.partial) kl += (double)e.y * log((double)e.y / (double)ybar);
            if (NEED_Z) {
                const float Q = e.mult * e.y * __builtin_amdgcn_rcpf(ybar) * g.ell;
                Qs[it - c0] = Q;
                qabs += fabsf(Q);
            }
        }
        if (!NEED_Z) continue;  // uniform
        // (the barrier inside also publishes Qs)
        const float bound = block_sum_all(qabs, red);
        const bool finite = bound < INFINITY;  // false for inf and NaN
        const float scale = finite && bound > 0.f ? 0x1p30f / bound : 0.f;
        if (scale > 0.f) {
            for (int64_t it0 = c0; it0 < c1; it0 += nslot) {
                const int64_t it = it0 + threadIdx.x / C;
                const bool act = it < c1;
                const CountItem e = act ? c.items[it] : CountItem{0u, 0.f, 1.f, 0.f};
                const RecGeo g = rec_geo<TOF>(a, c, L, e, act);
                const float qsc = act ? -Qs[act ? (int)(it - c0) : 0] * scale : 0.f;  // (index < q_cap)
                const float fis = (float)(g.is + ch), fie = (float)g.ie;
                unsigned long long *zr = Zu + (g.is + ch - L.i_lo) * rz;
                for (float fi = fis; fi <= fie; fi += fC, zr += C * rz) {
                    const float qw = TOF ? qsc * tof_weight_at(tab, fmaf(fi, g.pA, g.pB), c.pos_max) : qsc;
                    const float u = __builtin_amdgcn_fmed3f(fmaf(fi, g.zA, g.zB), 0.f, umax);
                    deposit_packed(zr, (int)u, qw, __builtin_amdgcn_fractf(u));
                }
            }
        }
        __syncthreads();
        if (nrow > 0 && (scale > 0.f || !finite))
            scatter_sheet_packed(a, L, nrow, Zu, finite ? 1.f / scale : 0.f, finite);
        if (c1 < i1) {
            // the next chunk starts from a zero sheet (after every readout)
            __syncthreads();
            for (int k = threadIdx.x; k < nrow * rz; k += blockDim.x) Zu[k] = 0ull;
            __syncthreads();
        }
    }
    if (a.partial) block_sums(kl, kl, a.partial, false);
}

template <bool TOF, int MODE>
void set_counts_lds(size_t need) {
    static size_t granted = 64 * 1024;
    if (need <= granted) return;
    if (hipFuncSetAttribute((const void *)k_line_counts<TOF, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)need) == hipSuccess)
        granted = need;
    (void)hipGetLastError();
}

template <bool TOF, int MODE>
hipError_t launch_counts_mode(const pet_geom_s *g, const pet_counts_s *cs, int nblk, int threads, size_t lds,
                              const ProjArgs &a, const CountArgs &c, hipStream_t s) {
    set_counts_lds<TOF, MODE>(lds);
    hipLaunchKernelGGL((k_line_counts<TOF, MODE>), dim3(nblk), dim3(threads), lds, s, a, c);
    return hipGetLastError();
}

}  // namespace

// LDS of the sheets and the TOF table (dynamic), and what the gradient mode
// keeps per bin of a chunk: its factor Q, 4 bytes.
static size_t counts_lds_base(const pet_geom_s *g, int mode) {
    const size_t sheet = ((size_t)g->rows_max * (g->d.nz + 2 * PADZ) + 3) & ~(size_t)3;
    const size_t tab = g->d.n_tof > 1 ? sizeof(float2) * NW_TAB : 0;
    return (mode == M_GRAD ? 3 : 1) * sheet * sizeof(float) + tab;
}

// Bins per chunk: what the LDS left after the sheets, the table and 1 KB of
// static shared memory holds, at most 8192 (0 if less than 256 fit).
static int counts_q_cap(const pet_geom_s *g) {
    const size_t base = counts_lds_base(g, M_GRAD) + 1024;
    if (base >= g->max_lds) return 0;
    const size_t fit = ((g->max_lds - base) / sizeof(float)) & ~(size_t)3;
    return fit < 256 ? 0 : (int)std::min<size_t>(fit, 8192);
}

size_t counts_lds_bytes(const pet_geom_s *g, int mode) {
    return counts_lds_base(g, mode) + (mode == M_GRAD ? sizeof(float) * (size_t)counts_q_cap(g) : 0);
}

int counts_blocks(const pet_counts_s *cs, int subset) {
    const int row = subset < 0 ? cs->n_subsets : subset;
    return (int)(cs->lines_off[row + 1] - cs->lines_off[row]);
}

hipError_t launch_line_counts(pet_geom_s *g, const pet_counts_s *cs, int mode, int subset, const ProjArgs &a,
                              hipStream_t s) {
    const int nblk = counts_blocks(cs, subset);
    if (nblk == 0) return hipSuccess;
    CountArgs c{};
    c.items = cs->items;
    c.line_off = cs->line_off;
    c.lines = cs->lines + cs->lines_off[subset < 0 ? cs->n_subsets : subset];
    c.wtab = g->wtab;
    c.nw = NW_TAB;
    c.n_tof = g->d.n_tof;
    c.wD = g->wD;
    c.inv_dx = (float)(NW_TAB / (2.0 * g->wD));
    c.pos0 = (float)(NW_TAB / 2);
    c.pos_max = (float)NW_TAB - 1e-3f;
    c.q_cap = mode != M_GRAD ? (1 << 30) : (g->flags & PET_SMALL_CHUNKS) ? std::min(16, counts_q_cap(g)) : counts_q_cap(g);
    const size_t lds = counts_lds_bytes(g, mode);
    const bool tof = g->d.n_tof > 1;
    const int threads = CNT_BLOCK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipSuccess;
    if (g->profiling) {
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (!g->prof_pool.empty()) {
            ev = g->prof_pool.back();
            g->prof_pool.pop_back();
        } else {
            e = hipEventCreate(&ev.first);
            if (e == hipSuccess) e = hipEventCreate(&ev.second);
            if (e != hipSuccess) return e;
        }
        e0 = ev.first;
        e1 = ev.second;
        g->prof_events[PROF_COUNTS].push_back(ev);
        e = hipEventRecord(e0, s);
    }
    if (e == hipSuccess) {
        if (mode == M_GRAD)
            e = tof ? launch_counts_mode<true, M_GRAD>(g, cs, nblk, threads, lds, a, c, s)
                    : launch_counts_mode<false, M_GRAD>(g, cs, nblk, threads, lds, a, c, s);
        else
            e = tof ? launch_counts_mode<true, M_OBJ>(g, cs, nblk, threads, lds, a, c, s)
                    : launch_counts_mode<false, M_OBJ>(g, cs, nblk, threads, lds, a, c, s);
    }
    if (e == hipSuccess && e1) e = hipEventRecord(e1, s);
    return e;
}

}  // namespace pet

using namespace pet;

extern "C" pet_status pet_counts_create(pet_geom g, const void *y, int y_dtype, const float *add, const float *mult,
                                        pet_counts *out) {
    if (!g || !y || !out) return fail(PET_E_ARG, "pet_counts_create: null argument");
    if (y_dtype != PET_Y_F32 && y_dtype != PET_Y_U16 && y_dtype != PET_Y_U8)
        return fail(PET_E_ARG, "pet_counts_create: bad y dtype");
    const int n_lines = g->d.n_views * g->d.n_rad;
    const int64_t bpl = (int64_t)g->n_planes * g->d.n_tof;
    if (bpl > (int64_t)UINT32_MAX) return fail(PET_E_ARG, "pet_counts_create: too many bins per line");
    if (counts_q_cap(g) == 0)
        return fail(PET_E_ARG, "pet_counts_create: the sheets and TOF table of this geometry exceed the LDS");
    pet_counts_s *c = new (std::nothrow) pet_counts_s();
    if (!c) return fail(PET_E_OOM, "pet_counts_create: host allocation failed");
    c->g = g;
    c->n_subsets = g->d.n_subsets;
    int *d_cnt = nullptr;
    double *d_ys = nullptr, *d_as = nullptr;
    hipError_t e = hipMalloc(&d_cnt, sizeof(int) * n_lines);
    if (e == hipSuccess) e = hipMalloc(&d_ys, sizeof(double) * n_lines);
    if (e == hipSuccess) e = hipMalloc(&d_as, sizeof(double) * n_lines);
    if (e == hipSuccess)
        hipLaunchKernelGGL(k_counts_per_line, dim3(n_lines), dim3(256), 0, 0, y, y_dtype, add, bpl, d_cnt, d_ys, d_as);
    if (e == hipSuccess) e = hipGetLastError();
    std::vector<int> cnt(n_lines);
    std::vector<double> ys(n_lines), as(n_lines);
    if (e == hipSuccess) e = hipMemcpy(cnt.data(), d_cnt, sizeof(int) * n_lines, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(ys.data(), d_ys, sizeof(double) * n_lines, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(as.data(), d_as, sizeof(double) * n_lines, hipMemcpyDeviceToHost);
    std::vector<int64_t> off(n_lines + 1, 0);
    for (int l = 0; l < n_lines; ++l) off[l + 1] = off[l] + cnt[l];
    c->n_items = off[n_lines];
    if (e == hipSuccess) e = hipMalloc(&c->line_off, sizeof(int64_t) * (n_lines + 1));
    if (e == hipSuccess) e = hipMalloc(&c->items, sizeof(CountItem) * std::max<int64_t>(c->n_items, 1));
    if (e == hipSuccess) e = hipMemcpy(c->line_off, off.data(), sizeof(int64_t) * (n_lines + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && c->n_items > 0)
        hipLaunchKernelGGL(k_counts_fill, dim3(n_lines), dim3(256), 0, 0, y, y_dtype, add, mult, bpl, g->d.n_tof,
                           g->n_planes, c->line_off, c->items);
    if (e == hipSuccess) e = hipGetLastError();
    // per subset (then all views): its lines with counts, most counts first,
    // and the sums of y and add over all its bins
    const int n = g->d.n_subsets;
    std::vector<int> lines;
    c->lines_off.assign(n + 2, 0);
    c->sum_y.assign(n + 1, 0.0);
    c->sum_add.assign(n + 1, 0.0);
    c->items_per_subset.assign(n + 1, 0);
    for (int row = 0; row <= n; ++row) {
        std::vector<int> mine;
        std::vector<int> views;
        if (row < n) {
            views = g->subset_views[row];
        } else {
            views.resize(g->d.n_views);
            std::iota(views.begin(), views.end(), 0);
        }
        for (int v : views)
            for (int k = 0; k < g->d.n_rad; ++k) {
                const int l = v * g->d.n_rad + k;
                c->sum_y[row] += ys[l];
                c->sum_add[row] += as[l];
                c->items_per_subset[row] += cnt[l];
                if (cnt[l] > 0) mine.push_back(l);
            }
        std::stable_sort(mine.begin(), mine.end(), [&](int a, int b) { return cnt[a] > cnt[b]; });
        lines.insert(lines.end(), mine.begin(), mine.end());
        c->lines_off[row + 1] = (int64_t)lines.size();
    }
    if (e == hipSuccess) e = hipMalloc(&c->lines, sizeof(int) * std::max<size_t>(lines.size(), 1));
    if (e == hipSuccess && !lines.empty())
        e = hipMemcpy(c->lines, lines.data(), sizeof(int) * lines.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (d_cnt) (void)hipFree(d_cnt);
    if (d_ys) (void)hipFree(d_ys);
    if (d_as) (void)hipFree(d_as);
    if (e != hipSuccess) {
        pet_counts_destroy(c);
        return e == hipErrorOutOfMemory ? fail(PET_E_OOM, "pet_counts_create: device allocation failed")
                                        : hip_check(e, "pet_counts_create");
    }
    *out = c;
    return PET_OK;
}

extern "C" pet_status pet_counts_destroy(pet_counts c) {
    if (!c) return PET_OK;
    (void)hipDeviceSynchronize();
    void *ptrs[] = {c->items, c->line_off, c->lines};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete c;
    return PET_OK;
}

extern "C" pet_status pet_counts_info(pet_counts c, int subset, int64_t *n_items, double *sum_y, double *sum_add) {
    if (!c) return fail(PET_E_ARG, "pet_counts_info: null handle");
    if (subset < -1 || subset >= c->n_subsets) return fail(PET_E_ARG, "pet_counts_info: subset out of range");
    const int row = subset < 0 ? c->n_subsets : subset;
    if (n_items) *n_items = c->items_per_subset[row];
    if (sum_y) *sum_y = c->sum_y[row];
    if (sum_add) *sum_add = c->sum_add[row];
    return PET_OK;
}
